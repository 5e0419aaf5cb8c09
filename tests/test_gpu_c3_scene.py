"""The clutter filter on the throughput workload's own scene (32x32 array, 9 plane waves,
128^3 voxels, 200 frames, moving tissue and three vessels; the precision variant runs on
the same seed), against the FP64 oracle applied to the same beamformed IQ:

- the knee rule on the GPU spectrum (FP32, three- and four-product split-BF16 Grams)
  picks the oracle's rank (or, where the chord rule is within 1e-6 dB of a tie, one of
  the tied ranks);
- the precision variant's error against the FP64 oracle, stated per result: the leading
  eigenvalue, the tissue projector V_K V_K^H at the oracle's rank, and the power Doppler
  on sampled voxels."""
import numpy as np
import pytest

from fqscene import get_config, make_scene
from helpers import dev, gpu_das, gpu_rf, gpu_svd_pd, rel_l2
from oracle import clutter

pytestmark = pytest.mark.gpu

CFG = get_config('c3')
ACQ = CFG.acq
N_SAMPLE = 65536


@pytest.fixture(scope='module')
def scene_iq(gpu):
    import torch
    print('c3 scene: rf_synth + das (full size)', flush=True)
    sc = make_scene(CFG)
    rf = gpu_rf(ACQ, sc)
    iq = gpu_das(ACQ, rf, 0)
    del rf
    torch.cuda.empty_cache()
    iq_h = iq.cpu().numpy()
    print('c3 scene: FP64 oracle Gram', flush=True)
    Go = clutter.gram(iq_h)
    lam_o, V_o = clutter.eig_desc(Go)
    K_o = clutter.knee_cutoff(lam_o)
    rng = np.random.default_rng(33)
    vox = np.sort(rng.choice(ACQ.n_vox, N_SAMPLE, replace=False))
    pd_o = clutter.power_doppler(clutter.filter_iq(iq_h[:, vox], V_o, K_o))
    print('c3 scene: oracle knee K', K_o, flush=True)
    return dict(iq=iq, Go=Go, lam_o=lam_o, V_o=V_o, K_o=K_o, vox=vox, pd_o=pd_o)


def _chord_gaps(lam):
    """The knee rule's chord-minus-spectrum values (dB) for k = 1..N (1-based)."""
    N = lam.size
    d = 10.0 * np.log10(np.maximum(lam, clutter.KNEE_FLOOR * lam[0]) / lam[0])
    k = np.arange(1, N + 1)
    return d[0] + (d[-1] - d[0]) * (k - 1) / (N - 1) - d


@pytest.mark.parametrize('mode', [0, 1, 3])
def test_knee_on_scene_matches_oracle(scene_iq, mode):
    import torch
    print('c3 knee, gram mode', mode, flush=True)
    out = gpu_svd_pd(scene_iq['iq'], -1, mode=mode)
    K = int(out['k'].item())
    K_o = scene_iq['K_o']
    gaps = _chord_gaps(scene_iq['lam_o'])
    best = gaps[1:ACQ.n_frames // 2].max()
    print('mode', mode, 'K gpu', K, 'K oracle', K_o, 'oracle gap at K gpu', gaps[K], 'best', best)
    assert int(out['status'].item()) == 0
    assert K == K_o or (K + 1 <= ACQ.n_frames // 2 and best - gaps[K] < 1e-6)
    vox = torch.from_numpy(scene_iq['vox']).cuda()
    pd = out['pd'][vox].cpu().numpy()
    if K == K_o:
        ep = rel_l2(pd, scene_iq['pd_o'])
        print('mode', mode, 'pd rel L2 vs FP64 oracle', ep)
        assert ep < 1e-3


@pytest.mark.parametrize('mode,tol_pd', [(0, 1e-3), (3, 1e-3), (1, 1e-2)])
def test_precision_variant_error_per_result(scene_iq, mode, tol_pd):
    """Mode 0 = FP32 Gram (the plain path), 3 = four-product split-BF16, 1 = three-product
    split-BF16; all at the oracle's rank so the error is that of the Gram alone."""
    import torch
    print('c3 per-result error, gram mode', mode, flush=True)
    K_o = scene_iq['K_o']
    out = gpu_svd_pd(scene_iq['iq'], K_o, mode=mode)
    G = out['G'].cpu().numpy()
    Go = scene_iq['Go']
    e_gram = rel_l2(G, Go)
    lam = out['sigma'].cpu().numpy() ** 2
    lam_o = scene_iq['lam_o']
    e_lam1 = abs(lam[0] - lam_o[0]) / lam_o[0]
    lam_g, V_g = clutter.eig_desc(G)
    e_proj = float(np.abs(clutter.projector(V_g, K_o) - clutter.projector(scene_iq['V_o'], K_o)).max())
    vox = torch.from_numpy(scene_iq['vox']).cuda()
    e_pd = rel_l2(out['pd'][vox].cpu().numpy(), scene_iq['pd_o'])
    print(f'mode {mode}: K {K_o}  gram {e_gram:.3e}  lambda_1 {e_lam1:.3e}  projector {e_proj:.3e}  pd {e_pd:.3e}')
    assert int(out['status'].item()) == 0
    assert e_gram < 1e-4 and e_lam1 < 1e-4
    assert e_pd < tol_pd
