"""Seeded random stage inputs (RF records, Casorati matrices).

These let a single stage be checked at full size without running the stages
before it.  They are plain random draws; nothing here models the physics.
"""
from __future__ import annotations

import numpy as np


def random_rf(n_frames: int, n_angles: int, n_elem: int, n_samples: int, seed: int,
              scale: float = 1.0) -> np.ndarray:
    """float32 [F][A][E][T] white Gaussian RF."""
    rng = np.random.default_rng(seed)
    out = rng.standard_normal((n_frames, n_angles, n_elem, n_samples), dtype=np.float32)
    if scale != 1.0:
        out *= np.float32(scale)
    return out


def random_casorati(n_vox: int, n_t: int, seed: int, rank: int = 3,
                    tissue_db: float = 50.0, noise_db: float = 100.0) -> np.ndarray:
    """complex64 [N_t][N_v]: a rank-`rank` slowly varying 'tissue' part with
    singular values spaced 6 dB apart, plus white complex 'blood' at
    -tissue_db relative power, plus a small noise floor at -noise_db."""
    rng = np.random.default_rng(seed)
    t = np.arange(n_t) / max(n_t, 1)
    out = np.zeros((n_t, n_vox), dtype=np.complex64)
    for k in range(rank):
        amp = 10.0 ** (-6.0 * k / 20.0)
        freq = 0.3 * (k + 1)
        slow = (np.exp(2j * np.pi * freq * t) * amp).astype(np.complex64)   # [N_t]
        sp = (rng.standard_normal(n_vox, dtype=np.float32)
              + 1j * rng.standard_normal(n_vox, dtype=np.float32)).astype(np.complex64)
        out += slow[:, None] * sp[None, :]
    b = np.float32(10.0 ** (-tissue_db / 20.0) / np.sqrt(2.0))
    out += b * (rng.standard_normal((n_t, n_vox), dtype=np.float32)
                + 1j * rng.standard_normal((n_t, n_vox), dtype=np.float32))
    nz = np.float32(10.0 ** (-noise_db / 20.0) / np.sqrt(2.0))
    out += nz * (rng.standard_normal((n_t, n_vox), dtype=np.float32)
                 + 1j * rng.standard_normal((n_t, n_vox), dtype=np.float32))
    return out


# Parameter vector layout of the learned slow-time filter (an interface both
# sides agree on): W1[32][2][9] b1[32] W2[32][32][9] b2[32] W3[32][32][9] b3[32] W4[2][32] b4[2].
LCF_SHAPES = (((32, 2, 9), 18), ((32,), 0), ((32, 32, 9), 288), ((32,), 0),
              ((32, 32, 9), 288), ((32,), 0), ((2, 32), 32), ((2,), 0))


def lcf_init_weights(seed: int) -> np.ndarray:
    """float32 [19170]: weights ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)), biases 0."""
    rng = np.random.default_rng(seed)
    parts = []
    for shp, fan_in in LCF_SHAPES:
        n = int(np.prod(shp))
        if fan_in:
            bound = 1.0 / np.sqrt(fan_in)
            parts.append(rng.uniform(-bound, bound, size=n))
        else:
            parts.append(np.zeros(n))
    return np.concatenate(parts).astype(np.float32)


def batch_indices(n_series_total: int, batch: int, seed: int) -> np.ndarray:
    """int64 [batch] voxel-series indices drawn uniformly with replacement."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, n_series_total, size=batch, dtype=np.int64)
