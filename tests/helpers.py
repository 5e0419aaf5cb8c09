"""Shared helpers of the GPU tests: parameter structs from an fqscene acquisition,
device upload, and the relative-L2 metric."""
from __future__ import annotations

import numpy as np


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def structs(acq):
    import paper_2509_05464_amd as fq
    probe = fq.make_probe(acq.nx_el, acq.ny_el, acq.pitch, acq.pitch, acq.fc, acq.fs, acq.c)
    tx = fq.make_tx(acq.tilts_rad())
    grid = fq.make_grid(acq.nx, acq.ny, acq.nz, acq.x0, acq.y0, acq.z0, acq.dx, acq.dy, acq.dz)
    pulse = fq.make_pulse(2.0, 5.0, 1e-3)
    return probe, tx, grid, pulse


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def gpu_rf(acq, scene):
    """RF of a scene on the GPU: static tissue once + blood (Algorithm 1 composition)."""
    import torch
    import paper_2509_05464_amd as fq
    probe, tx, grid, pulse = structs(acq)
    rf = torch.empty((acq.n_frames, acq.n_angles, acq.n_elem, acq.n_samples), dtype=torch.float32, device='cuda')
    fq.rf_synth(probe, tx, pulse, dev(scene.tissue_pos), dev(scene.tissue_amp), rf,
                pos_static=scene.tissue_pos.shape[0] == 1, accumulate=False)
    if scene.blood_amp.size:
        fq.rf_synth(probe, tx, pulse, dev(scene.blood_pos), dev(scene.blood_amp), rf,
                    pos_static=False, accumulate=True)
    return rf


def gpu_das(acq, rf, interp=0, ws_bytes=None):
    import torch
    import paper_2509_05464_amd as fq
    probe, tx, grid, _ = structs(acq)
    F = rf.shape[0]
    need = fq.das_workspace_size(probe, tx, F, acq.n_samples, minimum=False) if ws_bytes is None else ws_bytes
    ws = torch.empty(need, dtype=torch.uint8, device='cuda')
    iq = torch.empty((F, acq.n_vox), dtype=torch.complex64, device='cuda')
    fq.das_beamform(probe, tx, grid, rf, iq, ws, interp)
    return iq


def gpu_svd_pd(iq, cutoff, mode=0):
    """Gram -> eig -> rank -> projection + PD; returns dict of device tensors."""
    import torch
    import paper_2509_05464_amd as fq
    nt, nv = iq.shape
    gws = torch.empty(fq.gram_workspace_size(nv, nt, mode), dtype=torch.uint8, device='cuda')
    G = torch.empty((nt, nt), dtype=torch.complex128, device='cuda')
    fq.casorati_gram(iq, G, gws, mode)
    sws = torch.empty(fq.svd_workspace_size(nv, nt), dtype=torch.uint8, device='cuda')
    sigma = torch.empty(nt, dtype=torch.float64, device='cuda')
    k = torch.zeros(1, dtype=torch.int32, device='cuda')
    status = torch.zeros(1, dtype=torch.int32, device='cuda')
    pd = torch.empty(nv, dtype=torch.float32, device='cuda')
    iqf = torch.empty_like(iq)
    fq.svd_clutter_filter(iq, G, sws, sigma, k, cutoff, iq_filt=iqf, pd=pd, status=status)
    return dict(G=G, sigma=sigma, k=k, status=status, pd=pd, iq_filt=iqf)


def designed_modes_casorati(nv, nt, k_tissue, seed, n_blood=6):
    """Casorati matrix S = U0 diag(s) V^H (returned frame-major, complex64 [nt][nv]) with
    designed spatial magnitudes |U0|: k_tissue modes share one smooth footprint over the
    whole volume, n_blood modes share a localised vessel footprint, the rest are
    independent speckle; V (complex128 [nt][nt]) is a seeded random unitary matrix and
    s spans 60 dB.  S V = U0 diag(s), so the SSM of S and V is the correlation matrix of
    the designed magnitudes and its tissue rank is k_tissue."""
    rng = np.random.default_rng(seed)
    x = np.arange(nv) / nv
    tissue = 1.0 + 0.5 * np.sin(2 * np.pi * 7 * x)
    vessel = np.where((x > 0.25) & (x < 0.35), 1.0, 0.05)
    mag = np.abs(rng.standard_normal((nv, nt)))
    for k in range(k_tissue):
        mag[:, k] = np.abs(tissue * (1 + 0.1 * rng.standard_normal(nv)))
    for k in range(k_tissue, min(nt, k_tissue + n_blood)):
        mag[:, k] = np.abs(vessel * (1 + 0.1 * rng.standard_normal(nv)))
    U0 = mag * np.exp(2j * np.pi * rng.random((nv, nt)))
    q, r = np.linalg.qr(rng.standard_normal((nt, nt)) + 1j * rng.standard_normal((nt, nt)))
    V = q * (np.diag(r) / np.abs(np.diag(r)))
    s = np.geomspace(1e3, 1.0, nt)
    S = (U0 * s) @ V.conj().T
    return np.ascontiguousarray(S.T).astype(np.complex64), V
