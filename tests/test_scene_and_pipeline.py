"""Input-generator checks (closed forms of the flow model) and an end-to-end oracle
invariant (static scene -> no power Doppler after the clutter filter)."""
import numpy as np
import pytest

from fqscene import get_config, make_scene
from fqscene.configs import scaled
from oracle import clutter, pipeline


def test_poiseuille_mean_speed_is_half_vmax():
    """Uniform seeding of a circular lumen with v(r) = vmax (1 - r^2/R^2): mean v = vmax/2."""
    cfg = scaled(get_config('c1'), frames=3, n_blood=20000, n_tissue=10)
    sc = make_scene(cfg)
    v = sc.vessels[0]
    speed = v.vmax * (1 - sc.blood_radial ** 2)
    assert abs(speed.mean() / (v.vmax / 2) - 1) < 0.02
    # displacement between frames along the axis (no wrap for these short times)
    d = (sc.blood_pos[1] - sc.blood_pos[0]).astype(np.float64) @ v.axis
    dt = 1.0 / cfg.acq.prf
    ok = np.abs(d) < v.half_len
    np.testing.assert_allclose(d[ok], speed[ok] * dt, atol=3e-9)


def test_blood_stays_in_lumen_and_tissue_outside():
    cfg = scaled(get_config('c2'), frames=4, n_tissue=20000, n_blood=5000)
    sc = make_scene(cfg)
    from fqscene.scene import _inside_any, tissue_displacement
    disp = tissue_displacement(cfg.scene.motion, sc.times)
    for f in range(4):
        p = sc.blood_pos[f].astype(np.float64) - disp[f]
        assert _inside_any(p, sc.vessels).mean() > 0.999
        t = sc.tissue_pos[f].astype(np.float64) - disp[f]
        assert _inside_any(t, sc.vessels).mean() < 1e-3


def test_murray_tree():
    cfg = scaled(get_config('c5'), frames=2, n_tissue=100, n_blood=1000)
    sc = make_scene(cfg)
    assert len(sc.vessels) == 31
    r = np.array([v.radius for v in sc.vessels])
    assert r.min() >= 50e-6 - 1e-12 and r.max() <= 600e-6 + 1e-12
    vm = np.array([v.vmax for v in sc.vessels])
    assert vm.min() >= 2e-3 - 1e-12 and vm.max() <= 40e-3 + 1e-12
    # depth-first order: parent i has children i+1 and i+1+size(subtree); check r_p^3 = r1^3 + r2^3
    def sub(i, gen):
        return 1 if gen == 4 else 1 + 2 * sub(0, gen + 1)
    def check(i, gen):
        if gen == 4:
            return
        c1 = i + 1
        c2 = i + 1 + sub(0, gen + 1)
        rp, r1, r2 = r[i], r[c1], r[c2]
        if 50e-6 < min(r1, r2) and max(rp, r1, r2) < 600e-6:
            assert abs(rp ** 3 - (r1 ** 3 + r2 ** 3)) < 1e-9 * rp ** 3 + 1e-24
        check(c1, gen + 1)
        check(c2, gen + 1)
    check(0, 0)


def test_static_scene_has_no_power_doppler_after_filter(orc):
    """Alg.1 static tissue and no blood: every frame is identical, S is rank 1 and the
    clutter filter with K = 1 leaves nothing (relative to the raw energy)."""
    cfg = scaled(get_config('c1'), frames=4, n_blood=0, n_tissue=150)
    acq = cfg.acq.with_(nx=8, ny=8, nz=8, z0=8e-3)
    import dataclasses
    cfg = dataclasses.replace(cfg, acq=acq)
    sc = make_scene(cfg)
    out = pipeline.run(cfg, sc, cutoff=1)
    raw = clutter.power_doppler(out['iq'])
    assert out['pd'].max() < 1e-20 * raw.max()


def test_ssm_rank_minimises_blood_pd_error_on_small_scene(orc):
    """On the small workload (static tissue, one vessel) the tissue rank read from the
    spatial-similarity matrix is the rank whose power Doppler is closest to the
    blood-only ground truth (the knee of the singular-value curve is not)."""
    import dataclasses
    cfg = get_config('c1')
    sc = make_scene(cfg)
    out = pipeline.run(cfg, sc, cutoff=-2)
    blood = dataclasses.replace(sc, tissue_amp=np.zeros_like(sc.tissue_amp))
    ref = clutter.power_doppler(pipeline.run(cfg, blood, cutoff=0)['iq'])

    def err_db(K):
        pd = clutter.power_doppler(clutter.filter_iq(out['iq'], out['V'], K)) if K else clutter.power_doppler(out['iq'])
        return 10 * np.log10(np.sum((pd - ref) ** 2) / np.sum(ref ** 2))

    errs = [err_db(K) for K in range(7)]
    assert out['K'] == int(np.argmin(errs))
    assert errs[out['K']] < -6.0


def _rk4(vel, r0, t1, steps=2000):
    r = np.array(r0, dtype=np.float64)
    h = t1 / steps
    for _ in range(steps):
        k1 = vel(r)
        k2 = vel(r + 0.5 * h * k1)
        k3 = vel(r + 0.5 * h * k2)
        k4 = vel(r + h * k3)
        r = r + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return r


def test_rotation_motion_solves_the_trajectory_integral():
    """Section 2.2.2: a scatterer's position is the integral of the velocity field along
    its path.  For V(r) = (0, -w, 0) x (r - c) the closed form of the generator must match
    a fourth-order Runge-Kutta integration of that field (to 1e-12 m)."""
    from fqscene import motion_sweep_configs, rigid_motion
    spec = motion_sweep_configs()['rot0.4'].scene
    W = np.array([0.0, -spec.rot_omega, 0.0])
    c = np.asarray(spec.rot_centre)
    t = np.array([0.0, 0.05, 0.199])
    R, d, cc = rigid_motion(spec, t)
    rng = np.random.default_rng(3)
    for p0 in rng.uniform(-5e-3, 15e-3, size=(4, 3)):
        for i, ti in enumerate(t):
            want = _rk4(lambda r: np.cross(W, r - c), p0, ti) if ti > 0 else p0
            got = cc + R[i] @ (p0 - cc) + d[i]
            np.testing.assert_allclose(got, want, atol=1e-12)
    # the velocity at t = 0 is the field itself: (-w (z - z_c), 0, w x)
    p0 = np.array([1e-3, 2e-3, 10e-3])
    R2, _, _ = rigid_motion(spec, np.array([0.0, 1e-6]))
    v = (R2[1] - R2[0]) @ (p0 - c) / 1e-6
    np.testing.assert_allclose(v, [-spec.rot_omega * (p0[2] - c[2]), 0.0, spec.rot_omega * p0[0]], rtol=1e-5)


@pytest.mark.parametrize('case', ['vx8_vz4', 'rot0.4'])
def test_sweep_scenes_move_rigidly_with_their_vessels(case):
    """Tissue follows the rigid motion exactly; blood stays inside the moved lumina and
    tissue outside them."""
    from fqscene import motion_sweep_configs, rigid_motion
    from fqscene.configs import scaled as sc_scaled
    from fqscene.scene import _inside_any
    cfg = sc_scaled(motion_sweep_configs()[case], frames=5)
    sc = make_scene(cfg)
    R, d, c = rigid_motion(cfg.scene, sc.times)
    p0 = sc.tissue_pos[0].astype(np.float64)
    def back(p, f):                                          # inverse rigid motion (R orthogonal)
        return (p.astype(np.float64) - c - d[f]) @ R[f] + c

    for f in range(5):
        tis = back(sc.tissue_pos[f], f)
        np.testing.assert_allclose(tis, back(sc.tissue_pos[0], 0), atol=2e-9)
        assert _inside_any(back(sc.blood_pos[f], f), sc.vessels).mean() > 0.999
        assert _inside_any(tis, sc.vessels).mean() < 1e-3
    if case.startswith('v'):
        v = np.asarray(cfg.scene.velocity)
        np.testing.assert_allclose(sc.tissue_pos[4].astype(np.float64) - p0, np.broadcast_to(v * sc.times[4], p0.shape),
                                   atol=2e-9)
