"""ctypes front-end of the plain-C FP64 oracle (fq_oracle.c).

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, 'fq_oracle.c')
LIB = os.path.join(HERE, 'liboracle.so')
MAX_ANGLES = 64


def build(force: bool = True) -> str:
    """Compile fq_oracle.c with gcc (FP64, no fast-math, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + '.tmp'
        subprocess.check_call(['gcc', '-O2', '-fopenmp', '-shared', '-fPIC', '-Wall',
                               '-fno-fast-math', '-o', tmp, SRC, '-lm'])
        os.replace(tmp, LIB)
    return LIB


class OrcAcq(ctypes.Structure):
    _fields_ = [('nx_el', ctypes.c_int32), ('ny_el', ctypes.c_int32),
                ('pitch_x', ctypes.c_double), ('pitch_y', ctypes.c_double),
                ('fc', ctypes.c_double), ('fs', ctypes.c_double), ('c', ctypes.c_double),
                ('n_angles', ctypes.c_int32),
                ('tilt', (ctypes.c_double * 2) * MAX_ANGLES)]


class OrcGrid(ctypes.Structure):
    _fields_ = [('nx', ctypes.c_int32), ('ny', ctypes.c_int32), ('nz', ctypes.c_int32),
                ('x0', ctypes.c_double), ('y0', ctypes.c_double), ('z0', ctypes.c_double),
                ('dx', ctypes.c_double), ('dy', ctypes.c_double), ('dz', ctypes.c_double)]


class OrcPulse(ctypes.Structure):
    _fields_ = [('n_cycles', ctypes.c_double), ('trunc_sigmas', ctypes.c_double),
                ('r_ref', ctypes.c_double)]


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        P = ctypes.POINTER
        L.orc_rf_traces.argtypes = [P(OrcAcq), P(OrcPulse), ctypes.c_int32, ctypes.c_int64,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                    ctypes.c_void_p, ctypes.c_void_p]
        L.orc_fir_taps.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
        L.orc_rf2iq.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                ctypes.c_void_p, ctypes.c_void_p]
        for nm in ('orc_das_bb', 'orc_das_rf'):
            getattr(L, nm).argtypes = [P(OrcAcq), P(OrcGrid), ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_void_p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_acq(acq) -> OrcAcq:
    """Oracle parameter block from an fqscene.Acq."""
    q = OrcAcq()
    q.nx_el, q.ny_el = acq.nx_el, acq.ny_el
    q.pitch_x = q.pitch_y = acq.pitch
    q.fc, q.fs, q.c = acq.fc, acq.fs, acq.c
    tl = acq.tilts_rad()
    assert len(tl) <= MAX_ANGLES
    q.n_angles = len(tl)
    for i, (a, b) in enumerate(tl):
        q.tilt[i][0] = a
        q.tilt[i][1] = b
    return q


def make_grid(acq) -> OrcGrid:
    return OrcGrid(acq.nx, acq.ny, acq.nz, acq.x0, acq.y0, acq.z0, acq.dx, acq.dy, acq.dz)


PULSE_DEFAULT = dict(n_cycles=2.0, trunc_sigmas=5.0, r_ref=1e-3)


def make_pulse(n_cycles=2.0, trunc_sigmas=5.0, r_ref=1e-3) -> OrcPulse:
    return OrcPulse(n_cycles, trunc_sigmas, r_ref)


def rf_traces(acq, pos: np.ndarray, amp: np.ndarray, sel: np.ndarray,
              pulse: Optional[dict] = None) -> np.ndarray:
    """RF of selected traces.  pos float32 [Fp][S][3] (Fp == 1: static), amp float32 [S],
    sel int32 [n][3] rows (f, a, e).  Returns float64 [n][T]."""
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    amp = np.ascontiguousarray(amp, dtype=np.float32)
    sel = np.ascontiguousarray(sel, dtype=np.int32).reshape(-1, 3)
    out = np.zeros((sel.shape[0], acq.n_samples))
    q, pl = make_acq(acq), make_pulse(**(pulse or PULSE_DEFAULT))
    lib().orc_rf_traces(ctypes.byref(q), ctypes.byref(pl), pos.shape[0], pos.shape[1],
                        _ptr(pos), _ptr(amp), acq.n_samples, sel.shape[0], _ptr(sel), _ptr(out))
    return out


def all_traces(n_frames: int, n_angles: int, n_elem: int) -> np.ndarray:
    f, a, e = np.meshgrid(np.arange(n_frames), np.arange(n_angles), np.arange(n_elem), indexing='ij')
    return np.stack([f.ravel(), a.ravel(), e.ravel()], axis=1).astype(np.int32)


def rf_full(acq, pos: np.ndarray, amp: np.ndarray, pulse: Optional[dict] = None) -> np.ndarray:
    """Full RF float64 [F][A][E][T].  Static positions (Fp == 1) are evaluated once
    and the same traces are used for every frame."""
    F, A, E, T = acq.n_frames, acq.n_angles, acq.n_elem, acq.n_samples
    Fp = pos.shape[0]
    sel = all_traces(1 if Fp == 1 else F, A, E)
    out = rf_traces(acq, pos, amp, sel, pulse).reshape(-1, A, E, T)
    if Fp == 1:
        out = np.broadcast_to(out, (F, A, E, T)).copy()
    return out


def fir_taps(fc: float, fs: float) -> np.ndarray:
    h = np.zeros(33)
    lib().orc_fir_taps(fc, fs, _ptr(h))
    return h


def rf2iq(rf: np.ndarray, fc: float, fs: float) -> np.ndarray:
    """rf float32 [..., T] -> complex128 [..., T]."""
    rf = np.ascontiguousarray(rf, dtype=np.float32)
    T = rf.shape[-1]
    n = rf.size // T
    out = np.zeros(rf.shape + (2,))
    lib().orc_rf2iq(n, T, fc, fs, _ptr(rf), _ptr(out))
    return out[..., 0] + 1j * out[..., 1]


def bb_frames_inner(bb: np.ndarray) -> np.ndarray:
    """complex [F][A][E][T] -> float64 [A][E][T][F][2] (the oracle DAS's memory layout)."""
    F, A, E, T = bb.shape
    bbl = np.empty((A, E, T, F, 2))
    t = np.transpose(bb, (1, 2, 3, 0))
    bbl[..., 0] = t.real
    bbl[..., 1] = t.imag
    return bbl


def das_from_bb(acq, bb: np.ndarray, interp: int = 0,
                voxels: Optional[Sequence[int]] = None) -> np.ndarray:
    """bb complex [F][A][E][T] -> IQ complex128 [F][n_vox_sel] (all voxels by default)."""
    F, A, E, T = bb.shape
    assert A == acq.n_angles and E == acq.n_elem and T == acq.n_samples
    return das_from_layout(acq, bb_frames_inner(bb), interp, voxels)


def das_from_layout(acq, bbl: np.ndarray, interp: int = 0,
                    voxels: Optional[Sequence[int]] = None) -> np.ndarray:
    """DAS from the frames-innermost baseband bbl float64 [A][E][T][F][2]."""
    A, E, T, F, _ = bbl.shape
    bbl = np.ascontiguousarray(bbl)
    sel = np.arange(acq.n_vox, dtype=np.int64) if voxels is None else np.asarray(voxels, np.int64)
    out = np.zeros((sel.size, F, 2))
    q, g = make_acq(acq), make_grid(acq)
    lib().orc_das_bb(ctypes.byref(q), ctypes.byref(g), F, T, _ptr(bbl), interp, sel.size,
                     _ptr(np.ascontiguousarray(sel)), _ptr(out))
    return np.ascontiguousarray((out[..., 0] + 1j * out[..., 1]).T)


def das_from_rf(acq, rf: np.ndarray, voxels: Sequence[int], interp: int = 0) -> np.ndarray:
    """rf float32 [F][A][E][T] -> IQ complex128 [F][n_sel] at the selected voxels,
    demodulating each needed baseband tap on demand."""
    rf = np.ascontiguousarray(rf, dtype=np.float32)
    F, A, E, T = rf.shape
    sel = np.ascontiguousarray(np.asarray(voxels, np.int64))
    out = np.zeros((sel.size, F, 2))
    q, g = make_acq(acq), make_grid(acq)
    lib().orc_das_rf(ctypes.byref(q), ctypes.byref(g), F, T, _ptr(rf), interp, sel.size,
                     _ptr(sel), _ptr(out))
    return np.ascontiguousarray((out[..., 0] + 1j * out[..., 1]).T)


def pulse_sigma(fc: float, n_cycles: float = 2.0) -> float:
    """Gaussian envelope standard deviation for an envelope FWHM of n_cycles/fc."""
    return n_cycles / (2.0 * math.sqrt(2.0 * math.log(2.0)) * fc)
