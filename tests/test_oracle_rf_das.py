"""Pins of the CPU oracle's RF synthesis, demodulation and beamforming.

Each check compares the oracle against something other than its own formula:
closed forms of the pulse, exact sample shifts, a library analytic signal,
the point-spread-function peak and the Doppler phase of a moving scatterer.
"""
import math

import numpy as np
import pytest
from scipy.signal import hilbert

from fqscene import get_config
from fqscene.scene import point_scene
from oracle import native, pipeline

C1 = get_config('c1').acq


def _elem(acq, e):
    return np.array([(e % acq.nx_el - 0.5 * (acq.nx_el - 1)) * acq.pitch,
                     (e // acq.nx_el - 0.5 * (acq.ny_el - 1)) * acq.pitch, 0.0])


def _vox(acq, v):
    ix, iy, iz = v % acq.nx, (v // acq.nx) % acq.ny, v // (acq.nx * acq.ny)
    return np.array([acq.x0 + ix * acq.dx, acq.y0 + iy * acq.dy, acq.z0 + iz * acq.dz])


def _one(acq, r, amp=1.0, frames=1):
    return point_scene(np.asarray(r, np.float64)[None, None, :].repeat(frames, 0), [amp])


# ---------------------------------------------------------------- RF synthesis
def test_rf_one_sample_shift_normal_incidence(orc):
    """Angle 0, element straight above the scatterer: moving the scatterer down by
    c/(2 fs) delays the echo by exactly one sample and scales it by rho/rho'."""
    acq = C1.with_(tilts_deg=((0.0, 0.0),), n_frames=1)
    pe = _elem(acq, 37)
    z = 8.3e-3
    dz = acq.c / (2 * acq.fs)
    sel = np.array([[0, 0, 37]], np.int32)
    r1 = np.array([pe[0], pe[1], z])
    r2 = np.array([pe[0], pe[1], z + dz])
    # positions are float32 inputs; use values exactly representable to keep the shift exact
    r1 = r1.astype(np.float32).astype(np.float64)
    r2 = np.array([r1[0], r1[1], np.float32(r1[2] + dz)], dtype=np.float64)
    dz_exact = r2[2] - r1[2]
    a = native.rf_traces(acq, r1[None, None].astype(np.float32), np.ones(1, np.float32), sel)[0]
    b = native.rf_traces(acq, r2[None, None].astype(np.float32), np.ones(1, np.float32), sel)[0]
    # exact relation for the float32-representable shift: time shift 2 dz/c samples
    shift = 2 * dz_exact / acq.c * acq.fs
    assert abs(shift - 1.0) < 1e-5
    n = np.arange(acq.n_samples)
    pk = int(np.argmax(np.abs(a)))
    assert abs(pk - 2 * r1[2] / acq.c * acq.fs) <= 1.0
    # b[n+1] vs a[n] * rho/rho' up to the tiny residual of the float32 shift
    ratio = r1[2] / r2[2]
    win = slice(pk - 12, pk + 12)
    np.testing.assert_allclose(b[1:][win], a[:-1][win] * ratio, atol=2e-5 * np.abs(a).max())
    assert n.size == acq.n_samples


def test_rf_pulse_energy_closed_form(orc):
    """sum_n rf[n]^2 / fs = (A r_ref/rho)^2 * sigma sqrt(pi)/2 * (1 + exp(-(2 pi fc sigma)^2))."""
    acq = C1.with_(n_frames=1)
    r = np.array([0.4e-3, -0.7e-3, 9.1e-3])
    amp = 1.7
    sel = np.array([[0, a, e] for a in range(3) for e in (0, 100, 255)], np.int32)
    rf = native.rf_traces(acq, r[None, None].astype(np.float32), np.array([amp], np.float32), sel)
    sig = native.pulse_sigma(acq.fc)
    rr = r.astype(np.float32).astype(np.float64)
    for (f, a, e), tr in zip(sel, rf):
        rho = np.linalg.norm(rr - _elem(acq, e))
        A = amp * 1e-3 / rho
        want = A * A * sig * math.sqrt(math.pi) / 2 * (1 + math.exp(-(2 * math.pi * acq.fc * sig) ** 2))
        got = np.sum(tr ** 2) / acq.fs
        assert abs(got / want - 1) < 1e-6


def test_rf_tilt_convention(orc):
    """+theta_x steers the wavefront towards +x: at equal depth, a scatterer at +x is
    insonified (2 x sin theta)/c later than its mirror at -x (same element distance)."""
    acq = C1.with_(n_frames=1)
    a_idx = 2                                       # +5 deg
    th = math.radians(acq.tilts_deg[a_idx][0])
    x = 1.2e-3
    z = 9e-3
    # elements mirrored in x so both receive paths have equal length
    e_plus = 8 + 16 * 7                              # x = +0.15 mm
    e_minus = 7 + 16 * 7                             # x = -0.15 mm
    p = native.rf_traces(acq, np.array([[[x, 0.0, z]]], np.float32), np.ones(1, np.float32),
                         np.array([[0, a_idx, e_plus]], np.int32))[0]
    m = native.rf_traces(acq, np.array([[[-x, 0.0, z]]], np.float32), np.ones(1, np.float32),
                         np.array([[0, a_idx, e_minus]], np.int32))[0]
    t = np.arange(acq.n_samples) / acq.fs
    tp = np.sum(t * p ** 2) / np.sum(p ** 2)
    tm = np.sum(t * m ** 2) / np.sum(m ** 2)
    want = 2 * np.float32(x) * math.sin(th) / acq.c
    assert abs((tp - tm) - want) < 1e-3 / acq.fs


def test_rf_superposition(orc):
    """RF_total = RF_phantom + RF_flow (Algorithm 1): the RF of a union of scatterer
    sets equals the sum of their RFs."""
    acq = C1.with_(n_frames=2)
    rng = np.random.default_rng(3)
    pa = rng.uniform([-2e-3, -2e-3, 6e-3], [2e-3, 2e-3, 12e-3], size=(2, 20, 3)).astype(np.float32)
    pb = rng.uniform([-2e-3, -2e-3, 6e-3], [2e-3, 2e-3, 12e-3], size=(2, 7, 3)).astype(np.float32)
    aa = rng.normal(size=20).astype(np.float32)
    ab = rng.normal(size=7).astype(np.float32)
    sel = np.array([[1, 0, 5], [0, 2, 200], [1, 1, 128]], np.int32)
    ra = native.rf_traces(acq, pa, aa, sel)
    rb = native.rf_traces(acq, pb, ab, sel)
    rab = native.rf_traces(acq, np.concatenate([pa, pb], 1), np.concatenate([aa, ab]), sel)
    np.testing.assert_allclose(rab, ra + rb, atol=1e-12)


# ---------------------------------------------------------------- rf2iq
def test_rf2iq_envelope_and_phase(orc):
    """Isolated pulse: |b| follows the Gaussian envelope (A r_ref/rho) exp(-t^2/2s^2)
    within 1e-3 of its peak, and arg b = -2 pi fc tau across the pulse."""
    acq = C1.with_(n_frames=1)
    r = np.array([0.3e-3, 0.2e-3, 9.37e-3], np.float32)
    e = 90
    rf = native.rf_traces(acq, r[None, None], np.ones(1, np.float32), np.array([[0, 1, e]], np.int32))
    b = native.rf2iq(rf.astype(np.float32), acq.fc, acq.fs)[0]
    rr = r.astype(np.float64)
    rho = np.linalg.norm(rr - _elem(acq, e))
    tau = rr[2] / acq.c + rho / acq.c                 # angle 1 is 0 deg: t0 = 0
    sig = native.pulse_sigma(acq.fc)
    t = np.arange(acq.n_samples) / acq.fs - tau
    env = 1e-3 / rho * np.exp(-t ** 2 / (2 * sig ** 2))
    peak = env.max()
    assert np.max(np.abs(np.abs(b) - env)) < 1e-3 * peak
    core = np.abs(t) < 1.5 * sig
    ph = np.angle(b[core] * np.exp(1j * 2 * np.pi * acq.fc * tau))
    assert np.max(np.abs(ph)) < 2e-3


def test_rf2iq_matches_fft_analytic_signal(orc):
    """For band-limited input, 2 LPF[rf e^{-i w t}] equals the FFT analytic signal
    (scipy.signal.hilbert) brought to baseband, up to the FIR's pass/stop error."""
    acq = C1.with_(n_frames=1)
    rng = np.random.default_rng(5)
    pos = rng.uniform([-2e-3, -2e-3, 6e-3], [2e-3, 2e-3, 12e-3], size=(1, 40, 3)).astype(np.float32)
    amp = rng.normal(size=40).astype(np.float32)
    rf = native.rf_traces(acq, pos, amp, np.array([[0, 0, 17]], np.int32))[0].astype(np.float32)
    b = native.rf2iq(rf[None], acq.fc, acq.fs)[0]
    n = np.arange(acq.n_samples)
    ref = hilbert(rf.astype(np.float64)) * np.exp(-2j * np.pi * acq.fc * n / acq.fs)
    inner = slice(40, acq.n_samples - 40)
    err = np.linalg.norm(b[inner] - ref[inner]) / np.linalg.norm(ref[inner])
    assert err < 2e-3


# ---------------------------------------------------------------- DAS
@pytest.mark.parametrize('v_ijk', [(10, 20, 30), (0, 0, 0), (31, 31, 63), (16, 3, 50)])
@pytest.mark.parametrize('interp', [0, 1])
def test_das_psf_peak_on_true_voxel(orc, v_ijk, interp):
    """A point scatterer at a voxel centre: the |IQ| maximum is that voxel, its value is
    A sum_e r_ref/rho_e (compounding averages over transmits), its phase is 0."""
    acq = C1.with_(n_frames=1)
    ix, iy, iz = v_ijk
    v = ix + acq.nx * (iy + acq.ny * iz)
    r = _vox(acq, v).astype(np.float32)
    sc = _one(acq, r, amp=1.0)
    rf = native.rf_full(acq, sc.tissue_pos, sc.tissue_amp).astype(np.float32)
    iq = pipeline.beamform(acq, rf, interp)[0]
    assert int(np.argmax(np.abs(iq))) == v
    rr = r.astype(np.float64)
    want = sum(1e-3 / np.linalg.norm(rr - _elem(acq, e)) for e in range(acq.n_elem))
    tol = 0.02 if interp == 0 else 0.005
    assert abs(abs(iq[v]) / want - 1) < tol
    assert abs(np.angle(iq[v])) < 1e-3


def test_das_doppler_phase(orc):
    """A scatterer moving along +z at v: lag-1 autocorrelation phase
    = -4 pi fc v T_prf / c * kappa, kappa = mean_{a,e} (u_az + z/rho_e)/2 (1 %),
    and within 3 % of the plain -4 pi fc v T_prf / c."""
    acq = C1.with_(n_frames=4)
    T = 1.0 / acq.prf
    vel = 10e-3
    r0 = np.array([0.0, 0.0, 10e-3])
    pos = np.stack([r0 + np.array([0, 0, vel * f * T]) for f in range(acq.n_frames)])[:, None, :]
    sc = point_scene(pos, [1.0])
    rf = native.rf_full(acq, sc.tissue_pos, sc.tissue_amp).astype(np.float32)
    # beamform a neighbourhood of the scatterer only
    iz0 = int(round((r0[2] - acq.z0) / acq.dz))
    # the 2 x 2 voxel columns straddling the scatterer's axis, +-1 voxel in depth
    vox = [ix + acq.nx * (iy + acq.ny * iz) for iz in range(iz0 - 1, iz0 + 2)
           for iy in range(15, 17) for ix in range(15, 17)]
    bb = native.rf2iq(rf, acq.fc, acq.fs)
    iq = native.das_from_bb(acq, bb, 0, vox)
    R1 = np.sum(np.conj(iq[:-1]) * iq[1:])
    plain = -4 * np.pi * acq.fc * vel * T / acq.c
    kap = []
    for (tx, ty) in acq.tilts_rad():
        uz = math.sqrt(1 - math.sin(tx) ** 2 - math.sin(ty) ** 2)
        for e in range(acq.n_elem):
            rho = np.linalg.norm(r0 - _elem(acq, e))
            kap.append(0.5 * (uz + r0[2] / rho))
    want = plain * np.mean(kap)
    got = np.angle(R1)
    assert got < 0
    assert abs(got / want - 1) < 0.01
    assert abs(got / plain - 1) < 0.03


def test_das_identical_transmits_average(orc):
    """Mean over transmits (Algorithm 3): three identical transmits give the same IQ as one."""
    a1 = C1.with_(tilts_deg=((0.0, 0.0),), n_frames=1)
    a3 = C1.with_(tilts_deg=((0.0, 0.0),) * 3, n_frames=1)
    rng = np.random.default_rng(9)
    rf1 = rng.standard_normal((1, 1, a1.n_elem, a1.n_samples)).astype(np.float32)
    rf3 = np.repeat(rf1, 3, axis=1)
    vox = rng.integers(0, a1.n_vox, 50)
    i1 = native.das_from_rf(a1, rf1, vox)
    i3 = native.das_from_rf(a3, rf3, vox)
    np.testing.assert_allclose(i3, i1, rtol=1e-12, atol=1e-12 * np.abs(i1).max())


def test_das_rf_path_equals_bb_path(orc):
    """On-demand demodulation (sampled voxels) equals full rf2iq followed by DAS."""
    acq = C1.with_(n_frames=2)
    rng = np.random.default_rng(11)
    rf = rng.standard_normal((2, acq.n_angles, acq.n_elem, acq.n_samples)).astype(np.float32)
    vox = rng.integers(0, acq.n_vox, 20)
    for interp in (0, 1):
        a = native.das_from_rf(acq, rf, vox, interp)
        b = native.das_from_bb(acq, native.rf2iq(rf, acq.fc, acq.fs), interp, vox)
        np.testing.assert_allclose(a, b, rtol=1e-10, atol=1e-12 * np.abs(b).max())
