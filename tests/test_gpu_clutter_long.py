"""Clutter filter at long ensembles (the large configuration's 400 frames and the ABI
limit of 512; the eigensolver also on both sides of the register-resident reduction's
limit of 208 frames and with partial last block rows), and the beamformer with more
transmits than one pass over its staged delay windows holds, against the FP64 oracle.

Ensembles: a seeded Casorati matrix with a rank-6 tissue part (amplitudes 6 dB apart), white
blood 45 dB below it and a noise floor.  The FP64 oracle's Gram is handed to the GPU
eigensolver and filter, so eigenvalues, projectors, the knee and the power Doppler are
compared on the same matrix; the GPU's own FP32 Gram is checked separately."""
import numpy as np
import pytest

from fqscene import get_config, random_casorati
from helpers import dev, gpu_das, rel_l2, structs
from oracle import clutter, native

pytestmark = pytest.mark.gpu

NV = 24000


def _casorati(nt, seed):
    return random_casorati(NV, nt, seed=seed, rank=6, tissue_db=45)


@pytest.mark.parametrize('nt', [17, 100, 193, 200, 208, 209, 400, 512])
def test_eig_long_ensemble(gpu, nt):
    import torch
    print('eig n_t', nt, flush=True)
    iq = _casorati(nt, 40 + nt)
    Go = clutter.gram(iq)
    lam_o, V_o = clutter.eig_desc(Go)
    ws = torch.empty(gpu.svd_workspace_size(NV, nt), dtype=torch.uint8, device='cuda')
    lam = torch.empty(nt, dtype=torch.float64, device='cuda')
    vecs = torch.empty((nt, nt), dtype=torch.complex128, device='cuda')
    st = torch.full((1,), -1, dtype=torch.int32, device='cuda')
    gpu.hermitian_eig(dev(Go), ws, lam, vecs, st)
    assert int(st.item()) == 0
    l = lam.cpu().numpy()
    np.testing.assert_allclose(l, lam_o, rtol=1e-9, atol=1e-12 * lam_o[0])
    V = vecs.cpu().numpy()
    # projectors onto the leading K modes (the tissue modes are >= 10 dB apart; the sixth
    # sits ~3 dB above the blood floor, too close for a 1e-9 projector)
    for K in (1, 2, 3, 5):
        assert np.abs(clutter.projector(V, K) - clutter.projector(V_o, K)).max() < 1e-9


@pytest.mark.parametrize('nt', [400, 512])
def test_knee_and_filter_long_ensemble(gpu, nt):
    import torch
    print('filter n_t', nt, flush=True)
    iq = _casorati(nt, 50 + nt)
    Go = clutter.gram(iq)
    lam_o, V_o = clutter.eig_desc(Go)
    K_o = clutter.knee_cutoff(lam_o)
    ws = torch.empty(gpu.svd_workspace_size(NV, nt), dtype=torch.uint8, device='cuda')
    sigma = torch.empty(nt, dtype=torch.float64, device='cuda')
    k = torch.zeros(1, dtype=torch.int32, device='cuda')
    st = torch.full((1,), -1, dtype=torch.int32, device='cuda')
    pd = torch.empty(NV, dtype=torch.float32, device='cuda')
    iqf = torch.empty((nt, NV), dtype=torch.complex64, device='cuda')
    x = dev(iq)
    gpu.svd_clutter_filter(x, dev(Go), ws, sigma, k, -1, iq_filt=iqf, pd=pd, status=st)
    assert int(st.item()) == 0
    assert int(k.item()) == K_o
    np.testing.assert_allclose(sigma.cpu().numpy() ** 2, lam_o, rtol=1e-9, atol=1e-12 * lam_o[0])
    pd_o = clutter.power_doppler(clutter.filter_iq(iq, V_o, K_o))
    ep = rel_l2(pd.cpu().numpy(), pd_o)
    ef = rel_l2(iqf.cpu().numpy(), clutter.filter_iq(iq, V_o, K_o))
    print('n_t', nt, 'K', K_o, 'pd rel L2', ep, 'iq_filt rel L2', ef)
    assert ep < 1e-3 and ef < 1e-3
    # the GPU's own FP32 Gram: within FP32 accumulation of the FP64 Gram
    G = torch.empty((nt, nt), dtype=torch.complex128, device='cuda')
    gws = torch.empty(gpu.gram_workspace_size(NV, nt, 0), dtype=torch.uint8, device='cuda')
    gpu.casorati_gram(x, G, gws, 0)
    assert rel_l2(G.cpu().numpy(), Go) < 1e-6


@pytest.mark.parametrize('nt', [400, 512])
@pytest.mark.parametrize('K', [0, 3, 17, 64])
def test_fixed_cutoff_long_ensemble(gpu, nt, K):
    import torch
    print('fixed cutoff n_t', nt, 'K', K, flush=True)
    iq = random_casorati(6000, nt, seed=K + nt, rank=6, tissue_db=45)
    Go = clutter.gram(iq)
    lam_o, V_o = clutter.eig_desc(Go)
    ws = torch.empty(gpu.svd_workspace_size(6000, nt), dtype=torch.uint8, device='cuda')
    sigma = torch.empty(nt, dtype=torch.float64, device='cuda')
    k = torch.zeros(1, dtype=torch.int32, device='cuda')
    st = torch.full((1,), -1, dtype=torch.int32, device='cuda')
    pd = torch.empty(6000, dtype=torch.float32, device='cuda')
    gpu.svd_clutter_filter(dev(iq), dev(Go), ws, sigma, k, K, pd=pd, status=st)
    assert int(st.item()) == 0 and int(k.item()) == K
    pd_o = clutter.power_doppler(clutter.filter_iq(iq, V_o, K)) if K else clutter.power_doppler(iq)
    ep = rel_l2(pd.cpu().numpy(), pd_o)
    print('pd rel L2', ep)
    assert ep < 1e-3


def _many_tilts(n):
    """n plane waves: x tilts spread over +-12 degrees, y tilts alternating 0 / +-4."""
    tx = np.linspace(-12.0, 12.0, n)
    ty = [(0.0, 4.0, -4.0)[i % 3] for i in range(n)]
    return tuple((float(a), float(b)) for a, b in zip(tx, ty))


@pytest.mark.parametrize('n_angles', [11, 16, 32])
@pytest.mark.parametrize('interp', [0, 1])
def test_das_many_transmits(gpu, n_angles, interp):
    """More transmits than one LDS pass of the beamformer stages (9 at a time): the
    partial sums of later passes accumulate into the first pass's result."""
    print('das angles', n_angles, 'interp', interp, flush=True)
    acq = get_config('c1').acq.with_(tilts_deg=_many_tilts(n_angles), nx=20, ny=12, nz=8, n_frames=3)
    rng = np.random.default_rng(n_angles)
    rf = rng.standard_normal((acq.n_frames, acq.n_angles, acq.n_elem, acq.n_samples), dtype=np.float32)
    iq = gpu_das(acq, dev(rf), interp).cpu().numpy()
    vox = np.arange(acq.n_vox, dtype=np.int64)
    want = native.das_from_rf(acq, rf, vox, interp)
    err = rel_l2(iq, want)
    print('das rel L2', err)
    assert err < 1e-4


@pytest.mark.parametrize('nt', [20, 200])
@pytest.mark.parametrize('K', [1, 4, 5, 8, 9, 16])
def test_pd_alone_matches_explicit_projection(gpu, nt, K):
    """Power Doppler without the filtered IQ takes the FP64 norm difference
    ||s||^2 - ||s V_K||^2 up to K = 16; with the filtered IQ requested it is summed from
    the explicit residual.  Both against the FP64 oracle and against each other."""
    import torch
    print('pd alone n_t', nt, 'K', K, flush=True)
    nv = 9001   # ragged against every launch shape
    iq = random_casorati(nv, nt, seed=K * 7 + nt, rank=6, tissue_db=45)
    Go = clutter.gram(iq)
    lam_o, V_o = clutter.eig_desc(Go)
    pd_o = clutter.power_doppler(clutter.filter_iq(iq, V_o, K))
    ws = torch.empty(gpu.svd_workspace_size(nv, nt), dtype=torch.uint8, device='cuda')
    outs = []
    for explicit in (False, True):
        sigma = torch.empty(nt, dtype=torch.float64, device='cuda')
        k = torch.zeros(1, dtype=torch.int32, device='cuda')
        st = torch.full((1,), -1, dtype=torch.int32, device='cuda')
        pd = torch.empty(nv, dtype=torch.float32, device='cuda')
        iqf = torch.empty((nt, nv), dtype=torch.complex64, device='cuda') if explicit else None
        gpu.svd_clutter_filter(dev(iq), dev(Go), ws, sigma, k, K, iq_filt=iqf, pd=pd, status=st)
        assert int(st.item()) == 0 and int(k.item()) == K
        outs.append(pd.cpu().numpy())
    e_alone, e_expl, e_pair = rel_l2(outs[0], pd_o), rel_l2(outs[1], pd_o), rel_l2(outs[0], outs[1])
    print(f'pd rel L2: alone {e_alone:.2e} explicit {e_expl:.2e} alone vs explicit {e_pair:.2e}')
    assert e_alone < 1e-3 and e_expl < 1e-3 and e_pair < 1e-3
    assert (outs[0] >= 0).all()


@pytest.mark.parametrize('nt', [33, 65, 97, 200, 225, 300, 512])
@pytest.mark.parametrize('mode', [0, 3])
def test_gram_tile_groups(gpu, nt, mode):
    """The Gram's 32x32 tiles are dealt to workgroups in groups of four that read at most four
    frame blocks (2, 3, 4, 7, 8, 10 and 16 blocks here): every tile of the Hermitian result,
    against the FP64 oracle, on a voxel count ragged against the 4096-voxel ranges."""
    import torch
    print('gram tile groups n_t', nt, 'mode', mode, flush=True)
    nv = 12289
    iq = random_casorati(nv, nt, seed=nt + mode, rank=6, tissue_db=45)
    G = torch.empty((nt, nt), dtype=torch.complex128, device='cuda')
    ws = torch.empty(gpu.gram_workspace_size(nv, nt, mode), dtype=torch.uint8, device='cuda')
    gpu.casorati_gram(dev(iq), G, ws, mode)
    Gg = G.cpu().numpy()
    Go = clutter.gram(iq)
    err = rel_l2(Gg, Go)
    print('gram rel L2', err)
    assert err < 1e-6
    np.testing.assert_array_equal(Gg, Gg.conj().T)
    # every tile carries data: no 32x32 block of the result is off by more than the tolerance
    for I in range(0, nt, 32):
        for J in range(I, nt, 32):
            blk, ref = Gg[I:I + 32, J:J + 32], Go[I:I + 32, J:J + 32]
            assert np.linalg.norm(blk - ref) <= 1e-5 * np.linalg.norm(Go) + 1e-6 * np.linalg.norm(ref)
