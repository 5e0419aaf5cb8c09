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
