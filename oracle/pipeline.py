"""End-to-end FP64 oracle chain for small workloads: scene -> RF -> IQ -> PD.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from . import clutter, native


def rf_scene(acq, scene, pulse=None) -> np.ndarray:
    """RF of the whole scene (tissue + blood, linear superposition), float64 [F][A][E][T]."""
    rf = native.rf_full(acq, scene.tissue_pos, scene.tissue_amp, pulse)
    if scene.blood_amp.size:
        rf += native.rf_full(acq, scene.blood_pos, scene.blood_amp, pulse)
    return rf


def beamform(acq, rf32: np.ndarray, interp: int = 0) -> np.ndarray:
    """float32 RF [F][A][E][T] -> IQ complex128 [F][N_v] (rf2iq, then DAS, all voxels)."""
    bb = native.rf2iq(rf32, acq.fc, acq.fs)
    return native.das_from_bb(acq, bb, interp)


def run(cfg, scene, interp: int = 0, cutoff=None):
    """Returns dict(rf32, iq, pd, lam, V, K).  The RF is rounded to float32 before
    demodulation, the precision in which the GPU path receives it."""
    acq = cfg.acq
    rf32 = rf_scene(acq, scene).astype(np.float32)
    iq = beamform(acq, rf32, interp)
    k = cfg.cutoff if cutoff is None else cutoff
    pd, lam, V, K = clutter.svd_filter_pd(iq, k)
    return dict(rf32=rf32, iq=iq, pd=pd, lam=lam, V=V, K=K)
