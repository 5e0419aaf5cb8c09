"""Spatial-similarity matrix (SSM) of the spatial modes and the tissue rank read from it
(the singular-value analyses of Section 3), through the C ABI against the FP64 oracle.

Tolerance on the correlations: 1e-4 absolute.  Derivation: |U| is formed in FP32 from
N_t-term products, so an element of a mode 60 dB below the first carries a relative
error of about 1e-4 (FP32 rounding of terms 1e3 times larger); errors that are
independent across voxels move a correlation over N_v voxels by about 1e-4/sqrt(N_v),
and the FP64 moments add nothing visible.  The rank is an integer decided in FP64 on
both sides: it must match exactly (the inputs keep every a_k - b_k far from 0)."""
import numpy as np
import pytest

from fqscene import get_config, make_scene, random_casorati
from helpers import designed_modes_casorati, dev, gpu_das, gpu_rf, rel_l2
from oracle import clutter, pipeline

pytestmark = pytest.mark.gpu

TOL_C = 1e-4


def gpu_ssm(iq, vecs, m):
    import torch
    import paper_2509_05464_amd as fq
    nt, nv = iq.shape
    ws = torch.empty(fq.ssm_workspace_size(nv, nt), dtype=torch.uint8, device='cuda')
    C = torch.empty((m, m), dtype=torch.float64, device='cuda')
    k = torch.full((1,), -7, dtype=torch.int32, device='cuda')
    fq.spatial_similarity(iq, vecs, m, ws, C, k)
    return C.cpu().numpy(), int(k.item())


def min_margin(C):
    """Smallest |a_k - b_k| over the k that the rank rule evaluates before it stops."""
    M = C.shape[0]
    ks = range(1, min(M - 2, max(1, M // 2), clutter.ssm_cutoff(C)) + 1)
    return min([abs(C[k, :k].mean() - C[k, k + 1:].mean()) for k in ks] or [np.inf])


@pytest.mark.parametrize('nv,k_tissue', [(3000, 1), (3000, 3), (2999, 5), (128, 2), (77, 3)])
def test_ssm_designed_modes(gpu, nv, k_tissue):
    """Tiles of 128 voxels with a ragged tail (3000), an odd voxel count (unaligned rows),
    exactly one tile, and less than one tile."""
    print('ssm designed', nv, k_tissue, flush=True)
    nt = 24
    iq, V = designed_modes_casorati(nv, nt, k_tissue, seed=40 + k_tissue)
    C, k = gpu_ssm(dev(iq), dev(V), nt)
    Co = clutter.spatial_similarity(iq, V, nt)
    err = np.max(np.abs(C - Co))
    print('ssm max abs err', err, 'k', k)
    assert err < TOL_C
    assert k == clutter.ssm_cutoff(C)
    assert k == clutter.ssm_cutoff(Co)
    if nv >= 1000:
        assert k == k_tissue


@pytest.mark.parametrize('m', [2, 3, 7, 24])
def test_ssm_leading_modes_only(gpu, m):
    """M below N_t reads only the leading columns of V; M = 2 and 3 give K = 1 by rule."""
    iq, V = designed_modes_casorati(1500, 24, 3, seed=7)
    C, k = gpu_ssm(dev(iq), dev(V), m)
    Co = clutter.spatial_similarity(iq, V, m)
    assert C.shape == (m, m)
    assert np.max(np.abs(C - Co)) < TOL_C
    assert k == clutter.ssm_cutoff(Co)
    if m <= 3:
        assert k == 1


def test_ssm_is_deterministic(gpu):
    iq, V = designed_modes_casorati(5000, 32, 3, seed=8)
    a = gpu_ssm(dev(iq), dev(V), 32)
    b = gpu_ssm(dev(iq), dev(V), 32)
    np.testing.assert_array_equal(a[0], b[0])
    assert a[1] == b[1]


@pytest.mark.parametrize('nv', [1, 500])
def test_ssm_without_spatial_variation_is_nan(gpu, nv):
    """Zero IQ (every |U| constant) and a single voxel: no variance, NaN correlations
    (as the oracle's correlation of constant columns), and the rank rule stops at 1."""
    V = np.eye(8, dtype=np.complex128)
    iq = np.zeros((8, nv), np.complex64)
    if nv == 1:
        iq[:, 0] = np.arange(1, 9)
    C, k = gpu_ssm(dev(iq), dev(V), 8)
    with np.errstate(invalid='ignore', divide='ignore'):
        Co = clutter.spatial_similarity(iq, V, 8)
    assert np.all(np.isnan(C)) and np.all(np.isnan(Co))
    assert k == 1 and clutter.ssm_cutoff(Co) == 1


def test_ssm_cutoff_in_clutter_filter_small_scene(gpu):
    """The small workload end to end on the GPU with the SSM cutoff: the rank and the
    power Doppler match the oracle chain with the same rule."""
    import torch
    import paper_2509_05464_amd as fq
    cfg = get_config('c1')
    acq = cfg.acq
    sc = make_scene(cfg)
    want = pipeline.run(cfg, sc, cutoff=-2)
    rf = gpu_rf(acq, sc)
    iq = gpu_das(acq, rf, 0)
    nt, nv = iq.shape
    gws = torch.empty(fq.gram_workspace_size(nv, nt, 0), dtype=torch.uint8, device='cuda')
    G = torch.empty((nt, nt), dtype=torch.complex128, device='cuda')
    fq.casorati_gram(iq, G, gws, 0)
    sws = torch.empty(fq.svd_workspace_size(nv, nt), dtype=torch.uint8, device='cuda')
    sigma = torch.empty(nt, dtype=torch.float64, device='cuda')
    k = torch.zeros(1, dtype=torch.int32, device='cuda')
    status = torch.zeros(1, dtype=torch.int32, device='cuda')
    pd = torch.empty(nv, dtype=torch.float32, device='cuda')
    fq.svd_clutter_filter(iq, G, sws, sigma, k, fq.CUTOFF_SSM, pd=pd, status=status)
    print('c1 ssm K gpu', int(k.item()), 'oracle', want['K'])
    assert int(status.item()) == 0
    assert int(k.item()) == want['K']
    err = rel_l2(pd.cpu().numpy(), want['pd'])
    print('c1 ssm pd rel L2', err)
    assert err < 1e-3
    # the leading modes' SSM from the GPU's own eigenvectors: modes far above the FP32
    # Gram's resolution agree with the oracle's
    lam = torch.empty(nt, dtype=torch.float64, device='cuda')
    vecs = torch.empty((nt, nt), dtype=torch.complex128, device='cuda')
    fq.hermitian_eig(G, sws, lam, vecs, status)
    C, kk = gpu_ssm(iq, vecs, nt)
    Co = clutter.spatial_similarity(want['iq'], want['V'], nt)
    e5 = np.max(np.abs(C[:5, :5] - Co[:5, :5]))
    print('c1 ssm leading 5 modes max abs err', e5)
    assert e5 < 1e-3
    assert kk == want['K']


def test_ssm_full_size(gpu):
    """Full throughput size (128^3 voxels, 200 frames, 64 modes) in the launch
    configuration the benchmark times: a seeded Casorati matrix whose voxels share a
    smooth amplitude envelope, the oracle's eigenvectors on both sides."""
    print('c2 ssm', flush=True)
    acq = get_config('c2').acq
    iq = random_casorati(acq.n_vox, acq.n_frames, seed=5, rank=4, tissue_db=45)
    x = np.arange(acq.n_vox) / acq.n_vox
    iq *= (1.0 + 0.5 * np.sin(2 * np.pi * 5 * x)).astype(np.float32)[None, :]
    lam, V = clutter.eig_desc(clutter.gram(iq))
    C, k = gpu_ssm(dev(iq), dev(V), 64)
    step = 1 << 18
    mags = np.concatenate([clutter.spatial_modes_abs(iq[:, v0:v0 + step], V, 64)
                           for v0 in range(0, acq.n_vox, step)])
    Co = np.corrcoef(mags, rowvar=False)
    err = np.max(np.abs(C - Co))
    print('c2 ssm max abs err', err, 'k', k, 'oracle k', clutter.ssm_cutoff(Co), 'margin', min_margin(Co))
    assert err < TOL_C
    assert k == clutter.ssm_cutoff(C)
    if min_margin(Co) > 1e-3:
        assert k == clutter.ssm_cutoff(Co)
