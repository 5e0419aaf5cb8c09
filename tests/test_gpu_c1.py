"""GPU parity on the small workload (16x16 array, 3 transmits, 32x32x64 voxels, 20 frames):
every stage through the C ABI against the FP64 oracle on the same seeded inputs.

Tolerances: IQ relative L2 <= 1e-4 and PD relative L2 <= 1e-3 for the FP32 path; RF
relative L2 <= 2e-5 (FP32 synthesis of a sum of pulses, derived: per-sample FP32 rounding
of the delay and the recurrences is < 1e-6 relative)."""
import numpy as np
import pytest

from fqscene import get_config, make_scene
from helpers import dev, gpu_das, gpu_rf, gpu_svd_pd, rel_l2, structs
from oracle import bf16 as obf16
from oracle import clutter, native, pipeline

pytestmark = pytest.mark.gpu

CFG = get_config('c1')
ACQ = CFG.acq


@pytest.fixture(scope='module')
def ref():
    sc = make_scene(CFG)
    rf64 = pipeline.rf_scene(ACQ, sc)
    rf32 = rf64.astype(np.float32)
    iq_lin = pipeline.beamform(ACQ, rf32, 0)
    return dict(scene=sc, rf64=rf64, rf32=rf32, iq_lin=iq_lin)


def test_rf_synth_c1(gpu, ref):
    print('rf_synth c1 full', flush=True)
    rf = gpu_rf(ACQ, ref['scene']).cpu().numpy()
    err = rel_l2(rf, ref['rf64'])
    print('rf rel L2', err)
    assert err < 2e-5


def test_rf_synth_static_reuse_equals_per_frame(gpu, ref):
    """Static tissue computed once and written to every frame equals per-frame synthesis."""
    import torch
    sc = ref['scene']
    probe, tx, grid, pulse = structs(ACQ)
    shape = (ACQ.n_frames, ACQ.n_angles, ACQ.n_elem, ACQ.n_samples)
    a = torch.empty(shape, dtype=torch.float32, device='cuda')
    b = torch.empty(shape, dtype=torch.float32, device='cuda')
    pos = sc.tissue_pos[:, :300]
    amp = sc.tissue_amp[:300]
    gpu.rf_synth(probe, tx, pulse, dev(pos), dev(amp), a, pos_static=True)
    gpu.rf_synth(probe, tx, pulse, dev(np.repeat(pos, ACQ.n_frames, 0)), dev(amp), b, pos_static=False)
    assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) < 1e-6


@pytest.mark.parametrize('interp', [0, 1])
def test_das_c1(gpu, ref, interp):
    print('das c1 interp', interp, flush=True)
    want = ref['iq_lin'] if interp == 0 else pipeline.beamform(ACQ, ref['rf32'], 1)
    iq = gpu_das(ACQ, dev(ref['rf32']), interp).cpu().numpy()
    err = rel_l2(iq, want)
    print('iq rel L2', err)
    assert err < 1e-4


def test_das_chunking_is_invisible(gpu, ref):
    """Algorithm 3 processes the volume in memory-bounded chunks: a one-block workspace
    gives bit-identical IQ to the full workspace."""
    import paper_2509_05464_amd as fq
    probe, tx, _, _ = structs(ACQ)
    rf = dev(ref['rf32'])
    full = gpu_das(ACQ, rf, 0).cpu().numpy()
    small = gpu_das(ACQ, rf, 0, ws_bytes=fq.das_workspace_size(probe, tx, ACQ.n_frames, ACQ.n_samples, True))
    np.testing.assert_array_equal(small.cpu().numpy(), full)


def test_gram_fp32_c1(gpu, ref):
    iq = ref['iq_lin'].astype(np.complex64)
    out = gpu_svd_pd(dev(iq), 2)
    G = out['G'].cpu().numpy()
    want = clutter.gram(iq)
    err = rel_l2(G, want)
    print('gram rel L2', err)
    assert err < 1e-6
    np.testing.assert_array_equal(G, G.conj().T)


@pytest.mark.parametrize('mode,tol', [(1, 1e-6), (2, 1e-6), (3, 1e-6)])
def test_gram_bf16_modes_match_emulation(gpu, ref, mode, tol):
    """Split-BF16 with 3 (mode 1) or 4 (mode 3) products and plain BF16 (mode 2) equal
    the bit-exact emulation up to FP32 accumulation order."""
    iq = ref['iq_lin'].astype(np.complex64)
    out = gpu_svd_pd(dev(iq), 2, mode=mode)
    G = out['G'].cpu().numpy()
    want = obf16.gram_split_bf16(iq, {1: 3, 2: 1, 3: 4}[mode])
    err = rel_l2(G, want)
    print('bf16 mode', mode, 'vs emulation', err, 'vs fp64', rel_l2(G, clutter.gram(iq)))
    assert err < tol


def test_eig_c1(gpu, ref):
    import torch
    iq = ref['iq_lin'].astype(np.complex64)
    G = clutter.gram(iq)
    ws = torch.empty(gpu.svd_workspace_size(iq.shape[1], iq.shape[0]), dtype=torch.uint8, device='cuda')
    lam = torch.empty(iq.shape[0], dtype=torch.float64, device='cuda')
    vecs = torch.empty((iq.shape[0], iq.shape[0]), dtype=torch.complex128, device='cuda')
    st = torch.full((1,), -1, dtype=torch.int32, device='cuda')
    gpu.hermitian_eig(dev(G), ws, lam, vecs, st)
    lam_o, V_o = clutter.eig_desc(G)
    assert int(st.item()) == 0
    l = lam.cpu().numpy()
    np.testing.assert_allclose(l, lam_o, rtol=1e-9, atol=1e-12 * lam_o[0])
    V = vecs.cpu().numpy()
    for K in (1, 2, 3):
        assert np.abs(clutter.projector(V, K) - clutter.projector(V_o, K)).max() < 1e-9


def test_filter_pd_c1_fixed_cutoff(gpu, ref):
    iq = ref['iq_lin'].astype(np.complex64)
    out = gpu_svd_pd(dev(iq), CFG.cutoff)
    pd_o, lam_o, V_o, K = clutter.svd_filter_pd(iq.astype(np.complex128), CFG.cutoff)
    assert int(out['k'].item()) == K == 2
    err = rel_l2(out['pd'].cpu().numpy(), pd_o)
    print('pd rel L2', err)
    assert err < 1e-3
    # eigenvalues of the FP32-accumulated Gram: |d lambda_k| <= ||dG|| (Weyl), and the
    # Gram's accumulation error is ~1e-7 of ||G||, so compare lambda with atol 1e-6 lambda_1
    lam = out['sigma'].cpu().numpy() ** 2
    np.testing.assert_allclose(lam, lam_o, rtol=0, atol=1e-6 * lam_o[0])
    iqf = out['iq_filt'].cpu().numpy()
    assert rel_l2(iqf, clutter.filter_iq(iq.astype(np.complex128), V_o, K)) < 1e-3


@pytest.mark.parametrize('mode', [0, 3])
def test_knee_matches_oracle(gpu, ref, mode):
    """The knee on the GPU spectrum (FP32 or four-product split-BF16 Gram) picks the
    oracle's K, and the filtered PD matches."""
    iq = ref['iq_lin'].astype(np.complex64)
    out = gpu_svd_pd(dev(iq), -1, mode=mode)
    pd_o, lam_o, V_o, K = clutter.svd_filter_pd(iq.astype(np.complex128), -1)
    assert int(out['k'].item()) == K
    assert rel_l2(out['pd'].cpu().numpy(), pd_o) < 1e-3


def test_power_doppler_raw(gpu, ref):
    import torch
    iq = ref['iq_lin'].astype(np.complex64)
    pd = torch.empty(iq.shape[1], dtype=torch.float32, device='cuda')
    gpu.power_doppler(dev(iq), pd)
    assert rel_l2(pd.cpu().numpy(), clutter.power_doppler(iq)) < 1e-6


def test_cutoff_zero_is_raw_energy(gpu, ref):
    iq = ref['iq_lin'].astype(np.complex64)
    out = gpu_svd_pd(dev(iq), 0)
    assert rel_l2(out['pd'].cpu().numpy(), clutter.power_doppler(iq)) < 1e-6


def test_end_to_end_c1(gpu, ref):
    """scene -> rf_synth -> das_beamform -> casorati_gram -> svd_clutter_filter on the GPU
    against the oracle chain on the same scene."""
    print('end-to-end c1', flush=True)
    rf = gpu_rf(ACQ, ref['scene'])
    iq = gpu_das(ACQ, rf, 0)
    out = gpu_svd_pd(iq, CFG.cutoff)
    e_iq = rel_l2(iq.cpu().numpy(), ref['iq_lin'])
    pd_o, _, _, K = clutter.svd_filter_pd(ref['iq_lin'], CFG.cutoff)
    e_pd = rel_l2(out['pd'].cpu().numpy(), pd_o)
    print('e2e iq', e_iq, 'pd', e_pd)
    assert e_iq < 1e-4
    assert e_pd < 1e-3


def test_whole_path_is_bitwise_reproducible(gpu, ref):
    """RF synthesis (claims and refills in lane order), DAS, the Gram (fixed-order
    reductions), the eigensolver and the projection use no atomics: two runs of the whole
    path give identical bits."""
    runs = []
    for _ in range(2):
        rf = gpu_rf(ACQ, ref['scene'])
        iq = gpu_das(ACQ, rf, 0)
        out = gpu_svd_pd(iq, -1)
        runs.append((rf.cpu().numpy(), iq.cpu().numpy(), out['G'].cpu().numpy(), out['pd'].cpu().numpy(),
                     int(out['k'].item())))
    for a, b in zip(runs[0], runs[1]):
        if isinstance(a, int):
            assert a == b
        else:
            np.testing.assert_array_equal(a, b)
