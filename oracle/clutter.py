"""SVD clutter filter and power Doppler, FP64 (numpy).

Test infrastructure only.

Post-processing (Section 2.4.2, and the singular-value analyses of Section 3):
the slow-time ensemble is arranged as a Casorati matrix S (voxels x frames),
its leading singular components (tissue) are removed, and the power-Doppler
value of a voxel is the mean over frames of the squared magnitude of what
remains.

The singular value decomposition of S is taken through its Gram matrix:
G = S^H S = V diag(lambda) V^H, sigma_k = sqrt(lambda_k) (lambda descending,
negative round-off clamped to zero).  The filter keeps the orthogonal
complement of the K leading right singular vectors:
    S_f = S - (S V_K) V_K^H,   PD[v] = (1/N_t) sum_f |S_f[v, f]|^2.
The IQ arrays here use the frame-major layout iq[f][v] = S[v, f].
"""
from __future__ import annotations

from typing import Tuple

import numpy as np

CHUNK = 1 << 18


def gram(iq: np.ndarray) -> np.ndarray:
    """G = S^H S, complex128 [N_t][N_t]; iq is [N_t][N_v]."""
    nt, nv = iq.shape
    G = np.zeros((nt, nt), dtype=np.complex128)
    for v0 in range(0, nv, CHUNK):
        X = iq[:, v0:v0 + CHUNK].astype(np.complex128)
        G += X.conj() @ X.T
    return G


def eig_desc(G: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Eigenvalues (descending, clamped at 0) and eigenvectors (columns) of Hermitian G."""
    lam, V = np.linalg.eigh(G)
    lam = lam[::-1].copy()
    V = V[:, ::-1].copy()
    lam[lam < 0] = 0.0
    return lam, V


KNEE_FLOOR = 1e-6


def knee_cutoff(lam: np.ndarray, floor: float = KNEE_FLOOR) -> int:
    """Clutter rank from the singular-value curve (the paper marks the cutoff by
    eye on the first singular values, Section 3.2).  Written as the chord rule:
    d_k = 10 log10(max(lambda_k, floor lambda_1)/lambda_1), chord l_k from
    (1, d_1) to (N, d_N); k* = argmax over k in [2, N/2] of (l_k - d_k), the
    first index on ties; K = clamp(k* - 1, 1, N/2 - 1)  (k is 1-based).
    The floor (-60 dB): the cutoff is read off the singular-value curve by eye
    (Section 3.2), and the power-Doppler results are shown over a 60 dB dynamic
    range (Sections 3.1 and 3.3).  lambda_k is the energy of mode k, so modes more
    than 60 dB below the leading one lie outside the range the method displays;
    the rule reads the curve down to that level and treats the rest as flat (the
    chord's far end is taken at no less than -60 dB)."""
    lam = np.asarray(lam, dtype=np.float64)
    N = lam.size
    if N < 4:
        return 1
    l1 = lam[0]
    if not l1 > 0:
        return 1
    d = 10.0 * np.log10(np.maximum(lam, floor * l1) / l1)
    k = np.arange(1, N + 1)
    chord = d[0] + (d[-1] - d[0]) * (k - 1) / (N - 1)
    gap = chord - d
    best_k, best = 2, -np.inf
    for kk in range(2, N // 2 + 1):
        if gap[kk - 1] > best:
            best, best_k = gap[kk - 1], kk
    return int(min(max(best_k - 1, 1), N // 2 - 1))


def filter_iq(iq: np.ndarray, V: np.ndarray, K: int) -> np.ndarray:
    """S_f = S - (S V_K) V_K^H in the frame-major layout: returns complex128 [N_t][N_v]."""
    nt, nv = iq.shape
    VK = V[:, :K]
    out = np.empty((nt, nv), dtype=np.complex128)
    for v0 in range(0, nv, CHUNK):
        S = iq[:, v0:v0 + CHUNK].astype(np.complex128).T          # [nv][nt]
        P = S @ VK                                                 # [nv][K]
        out[:, v0:v0 + CHUNK] = (S - P @ VK.conj().T).T
    return out


def power_doppler(iq: np.ndarray) -> np.ndarray:
    """PD[v] = mean_f |iq[f, v]|^2 (float64 [N_v])."""
    iq = np.asarray(iq)
    return np.mean(np.abs(iq.astype(np.complex128)) ** 2, axis=0)


def svd_filter_pd(iq: np.ndarray, cutoff: int):
    """Full clutter-filter chain.  cutoff >= 0: fixed K; -1: knee rule; -2: rule on the
    spatial-similarity matrix (ssm_rank).
    Returns (pd float64 [N_v], lam float64 [N_t], V complex128, K)."""
    G = gram(iq)
    lam, V = eig_desc(G)
    if cutoff == -2:
        K = ssm_rank(iq, V)
    else:
        K = knee_cutoff(lam) if cutoff < 0 else int(cutoff)
    pd = power_doppler(filter_iq(iq, V, K)) if K > 0 else power_doppler(iq)
    return pd, lam, V, K


def projector(V: np.ndarray, K: int) -> np.ndarray:
    """V_K V_K^H (phase-invariant representation of the tissue subspace)."""
    VK = V[:, :K]
    return VK @ VK.conj().T


# --------------------------------------------------------------------------- spatial similarity
# The singular-value analyses of Section 3 (the figures of singular-value curves beside
# the correlation-coefficient matrices of the absolute values of the left singular
# vectors) inspect the spatial modes U = S V Sigma^-1.  The correlation coefficient is
# invariant to the positive scale 1/sigma_k of a column, so the modes are taken as the
# columns of S V directly.

def spatial_modes_abs(iq: np.ndarray, V: np.ndarray, n_modes: int) -> np.ndarray:
    """|S V_k| for k < n_modes: float64 [N_v][n_modes]; iq is [N_t][N_v], V [N_t][N_t]."""
    S = np.asarray(iq, dtype=np.complex128).T                  # [N_v][N_t]
    return np.abs(S @ np.asarray(V, dtype=np.complex128)[:, :n_modes])


def spatial_similarity(iq: np.ndarray, V: np.ndarray, n_modes: int) -> np.ndarray:
    """Correlation-coefficient matrix [n_modes][n_modes] of the columns of |S V| over voxels."""
    return np.corrcoef(spatial_modes_abs(iq, V, n_modes), rowvar=False)


def ssm_cutoff(C: np.ndarray) -> int:
    """Tissue rank from the spatial-similarity matrix.  The paper marks the cutoff by eye
    where the leading block of mutually similar modes ends; written here as a membership
    rule: mode k (0-based, k >= 1) joins the tissue block while its |U| is more alike to
    the modes before it than to the modes after it,
        a_k = mean_{i<k} C_ik,   b_k = mean_{k<j<M} C_kj,
    K = the first k in [1, min(M-2, M/2)] with not (a_k > b_k) (a NaN stops the block);
    K = max(1, M/2) when every such k joins."""
    C = np.asarray(C, dtype=np.float64)
    M = C.shape[0]
    cap = max(1, M // 2)
    for k in range(1, min(M - 2, cap) + 1):
        a = C[k, :k].mean()
        b = C[k, k + 1:].mean()
        if not a > b:
            return k
    return cap


SSM_MAX_MODES = 64


def ssm_rank(iq: np.ndarray, V: np.ndarray) -> int:
    """Tissue rank of the clutter filter's SSM mode: the rule above on the leading
    min(N_t, 64) spatial modes."""
    return ssm_cutoff(spatial_similarity(iq, V, min(iq.shape[0], SSM_MAX_MODES)))
