"""Pins of the oracle's Gram / eigendecomposition / rank selection / filter / PD and
of the BF16 emulation: brute-force SVD, closed forms, invariants, constructed spectra."""
import numpy as np
import pytest
import torch

from fqscene import random_casorati
from oracle import bf16, clutter


def _rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize('nv,nt', [(6, 4), (9, 5), (40, 7), (3, 3)])
def test_eigenvalues_equal_squared_singular_values(nv, nt):
    """sigma_k^2 of the Casorati matrix by numpy's SVD of S itself (not via the Gram)."""
    rng = np.random.default_rng(nv * 10 + nt)
    S = _rand_c(rng, nv, nt)
    lam, V = clutter.eig_desc(clutter.gram(S.T.copy()))
    sv = np.linalg.svd(S, compute_uv=False)
    want = np.zeros(nt)
    want[:sv.size] = sv ** 2
    np.testing.assert_allclose(lam, want, rtol=1e-12, atol=1e-12 * want[0])
    # right singular vectors span the same subspaces (projectors, phase-free)
    _, _, Vh = np.linalg.svd(S)
    for K in range(1, min(nv, nt)):
        np.testing.assert_allclose(clutter.projector(V, K), Vh[:K].conj().T @ Vh[:K], atol=1e-10)


def test_gram_2x2_closed_form():
    """lambda = (a+d)/2 +- sqrt(((a-d)/2)^2 + |b|^2) for G = [[a, b], [conj b, d]]."""
    rng = np.random.default_rng(1)
    S = _rand_c(rng, 5, 2)
    G = clutter.gram(S.T.copy())
    a, d, b = G[0, 0].real, G[1, 1].real, G[0, 1]
    root = np.sqrt(((a - d) / 2) ** 2 + abs(b) ** 2)
    lam, _ = clutter.eig_desc(G)
    np.testing.assert_allclose(lam, [(a + d) / 2 + root, (a + d) / 2 - root], rtol=1e-13)
    # G[0, 1] = sum_v conj(S[v,0]) S[v,1]
    np.testing.assert_allclose(b, np.sum(np.conj(S[:, 0]) * S[:, 1]), rtol=1e-13)


def test_gram_trace_and_psd():
    rng = np.random.default_rng(2)
    iq = _rand_c(rng, 11, 300)
    G = clutter.gram(iq)
    np.testing.assert_allclose(np.trace(G).real, np.sum(np.abs(iq) ** 2), rtol=1e-12)
    np.testing.assert_allclose(G, G.conj().T, atol=1e-12)
    assert np.linalg.eigvalsh(G).min() > -1e-9


def test_cutoff_zero_and_full():
    """K = 0 leaves the raw IQ energy mean_f |IQ|^2; K = N_t removes everything."""
    rng = np.random.default_rng(3)
    iq = _rand_c(rng, 8, 500)
    pd0, _, _, _ = clutter.svd_filter_pd(iq, 0)
    np.testing.assert_allclose(pd0, np.mean(np.abs(iq) ** 2, axis=0), rtol=1e-13)
    pdN, _, _, _ = clutter.svd_filter_pd(iq, 8)
    assert np.max(pdN) < 1e-24 * np.max(pd0) + 1e-26


@pytest.mark.parametrize('K', [1, 2, 5])
def test_parseval_and_orthogonality(K):
    """N_t sum_v PD[v] = sum_{k > K} lambda_k, and S_f V_K = 0."""
    iq = random_casorati(2000, 16, seed=4, rank=3, tissue_db=40).astype(np.complex128)
    pd, lam, V, _ = clutter.svd_filter_pd(iq, K)
    np.testing.assert_allclose(16 * pd.sum(), lam[K:].sum(), rtol=1e-9)
    Sf = clutter.filter_iq(iq, V, K)
    assert np.abs(Sf.T @ V[:, :K]).max() < 1e-10 * np.abs(iq).max()


def test_rank_one_scene_filters_to_zero():
    """A static scene repeats the same volume every frame: S is rank 1 and K >= 1 removes it."""
    rng = np.random.default_rng(5)
    vol = _rand_c(rng, 1000)
    iq = np.repeat(vol[None, :], 10, axis=0)
    pd, lam, _, _ = clutter.svd_filter_pd(iq, 1)
    assert lam[1] < 1e-12 * lam[0]
    assert pd.max() < 1e-20 * np.mean(np.abs(vol) ** 2)


def test_knee_constructed_spectrum():
    """0 dB to -40 dB over k = 1..4, then linearly to -60 dB: the knee is k* = 4, K = 3."""
    N = 20
    d = np.concatenate([np.linspace(0, -40, 4), np.linspace(-40, -60, N - 3)[1:]])
    assert d.size == N
    assert clutter.knee_cutoff(10 ** (d / 10)) == 3


def test_knee_ties_and_bounds():
    # a straight line in dB has no point below the chord: all gaps are 0 -> first index k=2 -> K=1
    lam = 10 ** (np.linspace(0, -50, 30) / 10)
    assert clutter.knee_cutoff(lam) == 1
    # a single dominant component followed by a flat floor: knee at k* = 2 -> K = 1
    lam = np.array([1.0] + [1e-6] * 15)
    assert clutter.knee_cutoff(lam) == 1
    # a spectrum with a deep drop after 6 components: K = 6
    lam = np.concatenate([10 ** (-np.arange(6) * 3 / 10), 10 ** ((-60 - np.arange(34) * 0.1) / 10)])
    assert clutter.knee_cutoff(lam) == 6
    # the result is bounded by N/2 - 1
    lam = np.concatenate([10 ** (-np.arange(15) / 10), [1e-12] * 5])
    assert 1 <= clutter.knee_cutoff(lam) <= 9


# ------------------------------------------------------------------ BF16
def test_bf16_round_matches_torch():
    """RNE bit rounding equals torch's float32 -> bfloat16 conversion, ties included."""
    rng = np.random.default_rng(6)
    x = np.concatenate([rng.standard_normal(100000).astype(np.float32) * 10.0 ** rng.uniform(-20, 20, 100000),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 1.0 + 2 ** -9,
                                  3.0 + 2 ** -7, 0.0, -0.0, 1e-40, 3.4e38], np.float32)]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(bf16.bf16_round(x), want)


def test_split_bf16_reconstruction():
    rng = np.random.default_rng(7)
    x = (rng.standard_normal(10000) * 10.0 ** rng.uniform(-5, 5, 10000)).astype(np.float32)
    hi, lo = bf16.split(x)
    rel = np.abs((hi.astype(np.float64) + lo) - x) / np.abs(x)
    assert rel.max() <= 2.0 ** -16
    assert np.abs(hi.astype(np.float64) - x).max() > 0      # the split is not trivially exact


def test_split_bf16_gram_error_vs_fp64():
    """The clutter filter uses the Gram only through its leading (tissue) eigenvectors.
    Split-BF16 (3 products) keeps the tissue projector within 1e-6 of FP64 and the
    filtered PD within 1e-4; plain BF16 (negative control) perturbs the projector
    by more than 30 dB more and misses the 1e-3 PD tolerance."""
    iq = random_casorati(20000, 12, seed=8, rank=2, tissue_db=45)
    G = clutter.gram(iq)
    lam, V = clutter.eig_desc(G)
    P = clutter.projector(V, 2)
    pd = clutter.power_doppler(clutter.filter_iq(iq, V, 2))
    res = {}
    for p in (3, 1):
        _, Ve = clutter.eig_desc(bf16.gram_split_bf16(iq, p))
        pde = clutter.power_doppler(clutter.filter_iq(iq, Ve, 2))
        res[p] = (np.linalg.norm(clutter.projector(Ve, 2) - P),
                  np.linalg.norm(pde - pd) / np.linalg.norm(pd))
    assert res[3][0] < 1e-6 and res[3][1] < 1e-4
    assert 20 * np.log10(res[1][0] / res[3][0]) > 30
    assert res[1][1] > 1e-3


def test_split_bf16_drops_lo_lo_gram():
    """The dropped lo*lo' term is a Gram of the BF16 residuals: the 3-product result
    equals the 4-product (exact-split) Gram minus sum_v lo lo^H, to FP64 rounding."""
    rng = np.random.default_rng(12)
    iq = (rng.standard_normal((5, 300)) + 1j * rng.standard_normal((5, 300))).astype(np.complex64)
    A, B = np.ascontiguousarray(iq.real), np.ascontiguousarray(iq.imag)
    Ah, Al = bf16.split(A)
    Bh, Bl = bf16.split(B)
    full = (Ah + Al).astype(np.float64) + 1j * (Bh + Bl).astype(np.float64)
    lo = Al.astype(np.float64) + 1j * Bl.astype(np.float64)
    want = full.conj() @ full.T - lo.conj() @ lo.T
    np.testing.assert_allclose(bf16.gram_split_bf16(iq, 3), want, rtol=1e-12, atol=1e-12)


def test_knee_floor_hides_unresolved_tail():
    """Eigenvalues below -60 dB (not resolved by an FP32 Gram) do not move the knee: a
    tail at -90 dB, at -200 dB or clamped to zero gives the same K as a flat -60 dB tail."""
    head = 10 ** (np.array([0, -8, -15, -22, -30, -45]) / 10)
    K = [clutter.knee_cutoff(np.concatenate([head, np.full(30, t)])) for t in (1e-6, 1e-9, 1e-20, 0.0)]
    assert len(set(K)) == 1
    assert K[0] == 6          # the six components above the floor are clutter


# ---------------------------------------------------------------- spatial similarity (SSM)

def _unitary(n, rng):
    q, r = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    return q * (np.diag(r) / np.abs(np.diag(r)))


def test_ssm_recovers_designed_spatial_modes():
    """S = U0 diag(s) V^H with V unitary gives S V = U0 diag(s): the SSM must equal the
    correlation of the designed magnitudes |U0| (any slip in the projection, e.g. V*
    instead of V or V^H instead of V, breaks the equality)."""
    rng = np.random.default_rng(11)
    nv, nt, m = 3000, 16, 6
    mag = np.abs(rng.standard_normal((nv, nt))) + 0.1
    mag[:, 1] = 2.0 * mag[:, 0] + 0.5          # mode 1 an increasing affine copy of mode 0
    mag[:, 2] = -0.5 * mag[:, 0] + 3.0         # mode 2 a decreasing one
    U0 = mag * np.exp(2j * np.pi * rng.random((nv, nt)))
    V = _unitary(nt, rng)
    s = np.geomspace(100.0, 0.01, nt)
    S = (U0 * s) @ V.conj().T                  # [N_v][N_t]
    C = clutter.spatial_similarity(S.T, V, m)
    want = np.corrcoef(mag[:, :m], rowvar=False)
    np.testing.assert_allclose(C, want, atol=1e-10)
    assert abs(C[0, 1] - 1.0) < 1e-12 and abs(C[0, 2] + 1.0) < 1e-12
    np.testing.assert_allclose(C, C.T, atol=1e-14)
    np.testing.assert_allclose(np.diag(C), 1.0, atol=1e-14)
    assert np.all(np.abs(C) <= 1.0 + 1e-12)
    # the wrong conjugation gives a different matrix
    Cw = np.corrcoef(np.abs(S @ V.conj()[:, :m]), rowvar=False)
    assert np.max(np.abs(Cw - want)) > 0.1


def _block_ssm(M, sizes, levels, background=0.02):
    """Correlation-like matrix with diagonal blocks of the given sizes and levels."""
    C = np.full((M, M), background)
    o = 0
    for n, lv in zip(sizes, levels):
        C[o:o + n, o:o + n] = lv
        o += n
    np.fill_diagonal(C, 1.0)
    return C


@pytest.mark.parametrize('k_tissue', [1, 2, 3, 5])
def test_ssm_cutoff_ends_the_leading_block(k_tissue):
    """A leading block of k modes followed by a second (blood-like) block: the rule
    returns k, also for a single tissue mode; a block of 1 has no inside pairs."""
    C = _block_ssm(24, [k_tissue, 6], [0.9, 0.7])
    assert clutter.ssm_cutoff(C) == k_tissue


def test_ssm_cutoff_degenerate_cases():
    # no similarity anywhere: a_1 = b_1 = 0 is not a join, K = 1
    assert clutter.ssm_cutoff(np.eye(20)) == 1
    # a leading block longer than M/2: every candidate joins, K is capped at M/2
    assert clutter.ssm_cutoff(_block_ssm(20, [15], [0.9])) == 10
    # all modes equally alike: a_1 = b_1 is not a join
    assert clutter.ssm_cutoff(np.full((20, 20), 0.8) + 0.2 * np.eye(20)) == 1
    # tiny matrices
    assert clutter.ssm_cutoff(np.eye(2)) == 1 and clutter.ssm_cutoff(np.ones((3, 3))) == 1
    # a NaN correlation (a mode with no spatial variation) enters b_1 or a_1 and stops
    # the block at its first mode
    for j in (0, 2, 9):
        C = _block_ssm(16, [4], [0.9])
        C[j, :] = np.nan
        C[:, j] = np.nan
        assert clutter.ssm_cutoff(C) == 1


@pytest.mark.parametrize('k_tissue', [1, 3, 5])
def test_ssm_rank_recovers_designed_tissue_modes(k_tissue):
    """S = U0 diag(s) V^H with designed spatial magnitudes: k tissue modes share one
    smooth footprint over the whole volume, six blood modes share a localised vessel
    footprint, the rest are independent speckle.  The SSM rule recovers k from S and V."""
    rng = np.random.default_rng(100 + k_tissue)
    nv, nt = 4000, 24
    x = np.arange(nv) / nv
    tissue = 1.0 + 0.5 * np.sin(2 * np.pi * 7 * x)
    vessel = np.where((x > 0.25) & (x < 0.35), 1.0, 0.05)
    mag = np.abs(rng.standard_normal((nv, nt)))
    for k in range(k_tissue):
        mag[:, k] = tissue * (1 + 0.1 * rng.standard_normal(nv))
    for k in range(k_tissue, k_tissue + 6):
        mag[:, k] = vessel * (1 + 0.1 * rng.standard_normal(nv))
    mag = np.abs(mag)
    U0 = mag * np.exp(2j * np.pi * rng.random((nv, nt)))
    V = _unitary(nt, rng)
    s = np.geomspace(1e3, 1.0, nt)
    S = (U0 * s) @ V.conj().T
    assert clutter.ssm_rank(S.T, V) == k_tissue
    pd, lam, Vo, K = clutter.svd_filter_pd(S.T, -2)
    assert K == k_tissue
