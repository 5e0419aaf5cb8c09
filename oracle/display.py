"""Display post-processing of the reconstructed volumes, FP64 (numpy).

Test infrastructure only.

Section 2.4.2: B-mode volumes are log-compressed and shown over a dynamic range; power
Doppler (uPDI) volumes likewise after the clutter filter.  The results section shows
them over 75 dB (B-mode) and 60 dB (uPDI), and as maximum-intensity projections (MIPs)
of the 3-D power Doppler onto the x-y, x-z and y-z planes.

Readings: the reference level is the maximum of the array being displayed (0 dB), values
below the dynamic range are shown at its floor, power values use 10 log10 and
amplitudes 20 log10 (for complex IQ the amplitude is |IQ|).  Volumes are stored with
x fastest: vol[iz][iy][ix].
"""
from __future__ import annotations

import numpy as np


def display_db(x: np.ndarray, kind: str, dr_db: float) -> np.ndarray:
    """max(-dr, 10 log10(P / max P)) for power values ('power'), or
    max(-dr, 20 log10(|x| / max |x|)) for amplitudes / complex IQ ('iq').
    An all-zero input is shown at the floor."""
    if kind == 'power':
        p = np.asarray(x, dtype=np.float64)
    elif kind == 'iq':
        p = np.abs(np.asarray(x, dtype=np.complex128)) ** 2      # 20 log10 |x| = 10 log10 |x|^2
    else:
        raise ValueError(kind)
    peak = p.max() if p.size else 0.0
    out = np.full(p.shape, -float(dr_db))
    if peak > 0:
        with np.errstate(divide='ignore'):
            db = 10.0 * np.log10(p / peak)
        out = np.maximum(out, db)
    return out


def mip(vol: np.ndarray, plane: str) -> np.ndarray:
    """Maximum-intensity projection of vol[iz][iy][ix] onto a plane:
    'xy' -> [ny][nx] (max over z), 'xz' -> [nz][nx] (max over y), 'yz' -> [nz][ny] (max over x)."""
    axis = {'xy': 0, 'xz': 1, 'yz': 2}[plane]
    return np.asarray(vol).max(axis=axis)
