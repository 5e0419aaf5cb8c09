"""Frequency-domain RF synthesis (Appendix D, Eq. 1-2; Algorithm 2) through the C ABI
against the FP64 oracle.

Tolerance: relative L2 1e-4 on RF.  Derivation: every 4-frequency chunk starts from
phases reduced in FP64, so the FP32 stepping carries at most three complex products
(~3e-7 relative); the transmit aperture sums add coherently, the echo sums over
scatterers incoherently (relative error ~1e-6), and the inverse transform steps at most
63 rotations between exact integer anchors (~4e-6)."""
import math

import numpy as np
import pytest

from helpers import dev, rel_l2
from oracle import pfield

pytestmark = pytest.mark.gpu

FC, FS, C, PITCH = 7.8e6, 31.25e6, 1540.0, 0.3e-3
TOL = 1e-4


def gpu_fd(nx, ny, tilts, pos, amp, T, elem_w=(0.0, 0.0), n_sub=(1, 1), atten=0.0, apod=None, static=False,
           block=None, prefill=None, floor=1e-7):
    import torch
    import paper_2509_05464_amd as fq
    probe = fq.make_probe(nx, ny, PITCH, PITCH, FC, FS, C)
    tx = fq.make_tx(tilts)
    pulse = fq.make_pulse(2.0, 5.0, 1e-3)
    fdp = fq.make_fd_params(elem_w, n_sub, atten, floor)
    F = pos.shape[0] if not static else 3
    S = amp.size
    wsb = fq.fd_workspace_size(probe, tx, pulse, fdp, T, block if block else max(S, 1))
    ws = torch.empty(wsb, dtype=torch.uint8, device='cuda')
    if prefill is None:
        rf = torch.empty((F, len(tilts), nx * ny, T), dtype=torch.float32, device='cuda')
    else:
        rf = dev(prefill.astype(np.float32))
    fq.fd_synth(probe, tx, pulse, fdp, dev(pos.astype(np.float32)), dev(amp.astype(np.float32)), rf, ws,
                pos_static=static, accumulate=prefill is not None,
                apod=None if apod is None else dev(apod.astype(np.float32)))
    return rf.cpu().numpy()


def oracle_fd(nx, ny, tilts, pos1, amp, T, **kw):
    return pfield.fd_rf(nx, ny, PITCH, FC, FS, C, tilts, pos1.astype(np.float32).astype(np.float64),
                        amp.astype(np.float32).astype(np.float64), T, **kw)


def scatterers(n, rng, F=1, z=(4e-3, 8e-3)):
    p = np.stack([rng.uniform(-1.5e-3, 1.5e-3, n), rng.uniform(-1.5e-3, 1.5e-3, n), rng.uniform(*z, n)], 1)
    pos = np.repeat(p[None], F, 0) + np.arange(F)[:, None, None] * np.array([0.0, 0.0, 20e-6])
    return pos, rng.normal(0, 1, n)


def test_point_elements(gpu):
    rng = np.random.default_rng(1)
    tilts = [(math.radians(-5), 0.0), (0.0, math.radians(4))]
    pos, amp = scatterers(30, rng)
    got = gpu_fd(4, 4, tilts, pos, amp, 512)[0]
    want = oracle_fd(4, 4, tilts, pos[0], amp, 512)
    err = rel_l2(got, want)
    print('fd point elements rel L2', err)
    assert err < TOL


def test_directivity_sub_elements_attenuation_apodization_moving(gpu):
    rng = np.random.default_rng(2)
    tilts = [(math.radians(3), 0.0), (math.radians(-6), math.radians(2)), (0.0, 0.0)]
    pos, amp = scatterers(25, rng, F=3)
    apod = rng.uniform(0.2, 1.0, 20)
    kw = dict(elem_w=(0.27e-3, 0.25e-3), n_sub=(2, 3), atten=0.5, apod=apod)
    got = gpu_fd(5, 4, tilts, pos, amp, 480, **kw)
    for f in range(3):
        want = oracle_fd(5, 4, tilts, pos[f], amp, 480, elem_w=kw['elem_w'], n_sub=kw['n_sub'], atten=0.5, apod=apod)
        err = rel_l2(got[f], want)
        print('fd frame', f, 'rel L2', err)
        assert err < TOL


def test_two_transmit_groups(gpu):
    """11 transmits: two launch groups of at most 9."""
    rng = np.random.default_rng(3)
    tilts = [(math.radians(a), math.radians(b)) for a in (-6, 0, 6) for b in (-6, 0, 6)] + [(0.05, 0.0), (0.0, -0.05)]
    pos, amp = scatterers(10, rng)
    got = gpu_fd(3, 3, tilts, pos, amp, 400, elem_w=(0.2e-3, 0.2e-3))[0]
    want = oracle_fd(3, 3, tilts, pos[0], amp, 400, elem_w=(0.2e-3, 0.2e-3))
    assert rel_l2(got, want) < TOL


def test_static_scatterers_accumulate_into_every_frame(gpu):
    rng = np.random.default_rng(4)
    tilts = [(0.0, 0.0), (math.radians(5), 0.0)]
    pos, amp = scatterers(12, rng)
    pre = rng.standard_normal((3, 2, 16, 400)) * 1e-3
    got = gpu_fd(4, 4, tilts, pos, amp, 400, static=True, prefill=pre)
    want = oracle_fd(4, 4, tilts, pos[0], amp, 400)
    for f in range(3):
        assert rel_l2(got[f] - pre[f].astype(np.float32), want) < TOL


def test_scatterer_blocks_are_invisible(gpu):
    """Algorithm 2's memory partition: a minimum workspace (blocks of 256 scatterers, here
    three blocks) gives the full-workspace result up to FP32 summation order."""
    rng = np.random.default_rng(5)
    tilts = [(0.0, 0.0)]
    pos, amp = scatterers(700, rng)
    full = gpu_fd(4, 4, tilts, pos, amp, 400)
    part = gpu_fd(4, 4, tilts, pos, amp, 400, block=256)
    assert rel_l2(part, full) < 1e-6


def test_scatterers_behind_the_array_are_ignored(gpu):
    rng = np.random.default_rng(6)
    tilts = [(0.0, 0.0)]
    pos, amp = scatterers(8, rng)
    behind = np.concatenate([pos, np.array([[[0.0, 0.0, -1e-3]]])], axis=1)
    a2 = np.concatenate([amp, [5.0]])
    np.testing.assert_allclose(gpu_fd(4, 4, tilts, behind, a2, 400), gpu_fd(4, 4, tilts, pos, amp, 400),
                               rtol=0, atol=1e-6 * np.abs(gpu_fd(4, 4, tilts, pos, amp, 400)).max())


def test_single_path_closed_form_on_the_gpu(gpu):
    """One transmitting element, one scatterer, point elements: every receive trace is the
    pulse delayed by the two-way path, scaled by r_ref^2 / (r_tx r_rx)."""
    cen = pfield.element_centres(4, 4, PITCH, PITCH)
    p = np.array([0.4e-3, -0.2e-3, 6e-3])
    apod = np.zeros(16)
    apod[5] = 1.0
    got = gpu_fd(4, 4, [(0.0, 0.0)], p[None, None, :], np.array([0.7]), 512, apod=apod, floor=1e-12)[0, 0]
    p32 = p.astype(np.float32).astype(np.float64)
    sig = pfield.pulse_sigma_s(FC)
    r0 = np.linalg.norm(p32 - cen[5])
    for m in (0, 5, 15):
        r1 = np.linalg.norm(p32 - cen[m])
        want = np.float32(0.7) * (1e-3 / r0) * (1e-3 / r1) * pfield.pulse(np.arange(512) / FS - (r0 + r1) / C, FC, sig)
        assert rel_l2(got[m], want) < TOL
