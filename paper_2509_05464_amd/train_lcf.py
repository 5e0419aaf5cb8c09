"""Train the learned slow-time clutter filter on simulated (mix, blood-only) IQ pairs.

The pairs come from this library's own RF synthesis and beamforming on seeded scenes:
for each scene the blood-only RF is synthesised and beamformed (target), then the
tissue RF is added to the same RF buffer (linearity) and beamformed again (input).
Training runs the HIP forward/backward/Adam kernels; this file only orchestrates.

    python -m paper_2509_05464_amd.train_lcf --config c4_train --seeds 1000-1063 \
        --steps 3000 --batch 4096 --out lcf_weights.npz
"""
from __future__ import annotations

import argparse
import time
from typing import Sequence

import numpy as np
import torch

from . import _lib as fq
from .learned import LearnedFilter


def _structs(acq):
    probe = fq.make_probe(acq.nx_el, acq.ny_el, acq.pitch, acq.pitch, acq.fc, acq.fs, acq.c)
    tx = fq.make_tx(acq.tilts_rad())
    grid = fq.make_grid(acq.nx, acq.ny, acq.nz, acq.x0, acq.y0, acq.z0, acq.dx, acq.dy, acq.dz)
    return probe, tx, grid, fq.make_pulse()


def make_pair(cfg, scene, rf: torch.Tensor, ws: torch.Tensor, mix_out: torch.Tensor, blood_out: torch.Tensor):
    """Beamformed blood-only and tissue+blood IQ of one scene (both complex64 [F][Nv])."""
    acq = cfg.acq
    probe, tx, grid, pulse = _structs(acq)
    dev = rf.device
    fq.rf_synth(probe, tx, pulse, torch.from_numpy(scene.blood_pos).to(dev), torch.from_numpy(scene.blood_amp).to(dev),
                rf, pos_static=False, accumulate=False)
    fq.das_beamform(probe, tx, grid, rf, blood_out, ws, fq.INTERP_LINEAR)
    fq.rf_synth(probe, tx, pulse, torch.from_numpy(scene.tissue_pos).to(dev),
                torch.from_numpy(scene.tissue_amp).to(dev), rf, pos_static=scene.tissue_static, accumulate=True)
    fq.das_beamform(probe, tx, grid, rf, mix_out, ws, fq.INTERP_LINEAR)


def make_pairs(cfg, seeds: Sequence[int], device=None, aug_seeds: Sequence[int] = ()):
    """Pairs of the workload's scenes for `seeds`, then of its seeded steady-motion variants
    (augmented_motion_config) for `aug_seeds`; all share the acquisition geometry."""
    from fqscene import augmented_motion_config, make_scene
    device = device or torch.device('cuda')
    acq = cfg.acq
    F, NV = acq.n_frames, acq.n_vox
    probe, tx, _, _ = _structs(acq)
    rf = torch.empty((F, acq.n_angles, acq.n_elem, acq.n_samples), dtype=torch.float32, device=device)
    ws = torch.empty(fq.das_workspace_size(probe, tx, F, acq.n_samples), dtype=torch.uint8, device=device)
    n = len(seeds) + len(aug_seeds)
    mix = torch.empty((n, F, NV), dtype=torch.complex64, device=device)
    blood = torch.empty_like(mix)
    for i, sd in enumerate(seeds):
        make_pair(cfg, make_scene(cfg, seed=sd), rf, ws, mix[i], blood[i])
    for i, sd in enumerate(aug_seeds):
        acfg = augmented_motion_config(cfg.name, sd)
        make_pair(acfg, make_scene(acfg), rf, ws, mix[len(seeds) + i], blood[len(seeds) + i])
    del rf, ws
    return mix, blood


def train(filt: LearnedFilter, mix: torch.Tensor, blood: torch.Tensor, steps: int, batch: int, seed: int = 0,
          log_every: int = 100, verbose: bool = True, lr_final: float = None):
    """Adam steps on random voxel series of the training volumes (constant rate, or a cosine
    decay from the filter's rate to lr_final).  Returns the loss history."""
    import math
    from fqscene import batch_indices
    n_vol, F, NV = mix.shape
    x = torch.empty((F, batch), dtype=torch.complex64, device=mix.device)
    y = torch.empty_like(x)
    hist = []
    lr0 = filt.lr
    t0 = time.time()
    for s in range(steps):
        if lr_final is not None:
            filt.lr = lr_final + 0.5 * (lr0 - lr_final) * (1.0 + math.cos(math.pi * s / max(1, steps - 1)))
        idx = torch.from_numpy(batch_indices(n_vol * NV, batch, seed + s)).to(mix.device)
        fq.lcf_gather(mix, idx, x)
        fq.lcf_gather(blood, idx, y)
        loss = filt.train_step(x, y)
        if s % log_every == 0 or s == steps - 1:
            hist.append((s, float(loss.item())))
            if verbose:
                print(f'[train] step {s} loss {hist[-1][1]:.4e} ({time.time() - t0:.1f}s)', flush=True)
    return hist


def pd_error_db(pd: torch.Tensor, pd_true: torch.Tensor) -> float:
    """10 log10(sum (PD - PD_true)^2 / sum PD_true^2) over the whole grid."""
    d = pd.double() - pd_true.double()
    return float(10 * torch.log10((d * d).sum() / (pd_true.double() ** 2).sum()).item())


def evaluate(filt: LearnedFilter, mix: torch.Tensor, blood: torch.Tensor, cutoff: int = -1) -> dict:
    """PD errors (dB vs the blood-only PD) of the learned filter, the SVD filter and no filter."""
    F, NV = mix.shape
    dev = mix.device
    pd_true = torch.empty(NV, dtype=torch.float32, device=dev)
    fq.power_doppler(blood, pd_true)
    pd_raw = torch.empty_like(pd_true)
    fq.power_doppler(mix, pd_raw)
    pd_l = torch.empty_like(pd_true)
    filt.infer(mix, pd_l)
    G = torch.empty((F, F), dtype=torch.complex128, device=dev)
    gws = torch.empty(fq.gram_workspace_size(NV, F, 0), dtype=torch.uint8, device=dev)
    fq.casorati_gram(mix, G, gws, fq.GRAM_FP32)
    sws = torch.empty(fq.svd_workspace_size(NV, F), dtype=torch.uint8, device=dev)
    sig = torch.empty(F, dtype=torch.float64, device=dev)
    k = torch.zeros(1, dtype=torch.int32, device=dev)
    pd_s = torch.empty_like(pd_true)
    fq.svd_clutter_filter(mix, G, sws, sig, k, cutoff, pd=pd_s)
    return {'learned_db': pd_error_db(pd_l, pd_true), 'svd_db': pd_error_db(pd_s, pd_true),
            'raw_db': pd_error_db(pd_raw, pd_true), 'svd_k': int(k.item())}


def main():
    from fqscene import get_config, lcf_init_weights
    ap = argparse.ArgumentParser()
    ap.add_argument('--config', default='c4_train')
    ap.add_argument('--seeds', default='1000-1063')
    ap.add_argument('--aug-seeds', default=None, help='seed range of steady-motion variants added to the training set')
    ap.add_argument('--steps', type=int, default=3000)
    ap.add_argument('--batch', type=int, default=4096)
    ap.add_argument('--lr', type=float, default=1e-3)
    ap.add_argument('--lr-final', type=float, default=None, help='cosine decay of the rate to this value')
    ap.add_argument('--init-seed', type=int, default=0)
    ap.add_argument('--eval-seed', type=int, default=None)
    ap.add_argument('--eval-config', default=None, help='workload of the held-out volume (default: --config)')
    ap.add_argument('--out', default='lcf_weights.npz')
    args = ap.parse_args()
    lo, hi = (int(v) for v in args.seeds.split('-'))
    cfg = get_config(args.config)
    t0 = time.time()
    aug = []
    if args.aug_seeds:
        alo, ahi = (int(v) for v in args.aug_seeds.split('-'))
        aug = list(range(alo, ahi + 1))
    mix, blood = make_pairs(cfg, list(range(lo, hi + 1)), aug_seeds=aug)
    torch.cuda.synchronize()
    print(f'[train] {mix.shape[0]} pairs in {time.time() - t0:.1f}s', flush=True)
    filt = LearnedFilter(lcf_init_weights(args.init_seed), lr=args.lr)
    train(filt, mix, blood, args.steps, args.batch, lr_final=args.lr_final)
    filt.save(args.out)
    if args.eval_seed is not None:
        del mix, blood
        torch.cuda.empty_cache()
        ecfg = get_config(args.eval_config or args.config)
        m, b = make_pairs(ecfg, [args.eval_seed])
        print('[eval]', ecfg.name, args.eval_seed, evaluate(filt, m[0], b[0]), flush=True)


if __name__ == '__main__':
    main()
