"""Parity at the throughput workload's full size (32x32 array, 9 plane waves, 128^3 voxels,
200 frames), in the launch configuration the benchmark times, on outputs the oracle can
compute one by one: sampled RF traces of the real scene, sampled voxels of the DAS of a
seeded random RF, the full Gram and sampled PD values of a seeded Casorati matrix, and
sampled series of the learned filter."""
import numpy as np
import pytest

from fqscene import get_config, make_scene, random_casorati, lcf_init_weights
from helpers import dev, gpu_das, gpu_rf, gpu_svd_pd, rel_l2
from oracle import bf16 as obf16
from oracle import clutter, lcf as olcf, native

pytestmark = pytest.mark.gpu

CFG = get_config('c2')
ACQ = CFG.acq


def test_rf_synth_full_size_sampled_traces(gpu):
    print('c2 rf_synth', flush=True)
    sc = make_scene(CFG)
    rf = gpu_rf(ACQ, sc)
    rng = np.random.default_rng(1)
    n = 24
    sel = np.stack([rng.integers(0, ACQ.n_frames, n), rng.integers(0, ACQ.n_angles, n),
                    rng.integers(0, ACQ.n_elem, n)], 1).astype(np.int32)
    got = np.stack([rf[f, a, e].cpu().numpy() for f, a, e in sel])
    del rf
    want = native.rf_traces(ACQ, sc.tissue_pos, sc.tissue_amp, sel) + native.rf_traces(ACQ, sc.blood_pos,
                                                                                          sc.blood_amp, sel)
    err = rel_l2(got, want)
    print('c2 rf rel L2', err)
    assert err < 2e-5


@pytest.mark.parametrize('interp', [0, 1])
def test_das_full_size_sampled_voxels(gpu, interp):
    print('c2 das interp', interp, flush=True)
    rng = np.random.default_rng(2)
    rf = rng.standard_normal((ACQ.n_frames, ACQ.n_angles, ACQ.n_elem, ACQ.n_samples), dtype=np.float32)
    iq = gpu_das(ACQ, dev(rf), interp)
    # voxels at the corners, the tile edges and random positions
    corners = [0, ACQ.nx - 1, ACQ.n_vox - 1, ACQ.nx * ACQ.ny * (ACQ.nz - 1), 15 + ACQ.nx * 16 + ACQ.nx * ACQ.ny * 3]
    vox = np.concatenate([corners, rng.integers(0, ACQ.n_vox, 27)]).astype(np.int64)
    got = iq[:, torch_index(vox)].cpu().numpy()
    del iq
    want = native.das_from_rf(ACQ, rf, vox, interp)
    err = rel_l2(got, want)
    print('c2 das rel L2', err)
    assert err < 1e-4


def torch_index(v):
    import torch
    return torch.from_numpy(np.asarray(v, np.int64)).cuda()


def test_svd_filter_full_size(gpu):
    print('c2 svd', flush=True)
    iq = random_casorati(ACQ.n_vox, ACQ.n_frames, seed=3, rank=4, tissue_db=45)
    out = gpu_svd_pd(dev(iq), 4)
    G = out['G'].cpu().numpy()
    Go = clutter.gram(iq)
    eg = rel_l2(G, Go)
    lam, V = clutter.eig_desc(Go)
    rng = np.random.default_rng(4)
    vox = rng.integers(0, ACQ.n_vox, 4096)
    sub = iq[:, vox].astype(np.complex128)
    pd_o = clutter.power_doppler(clutter.filter_iq(sub, V, 4))
    pd = out['pd'].cpu().numpy()[vox]
    ep = rel_l2(pd, pd_o)
    print('c2 gram rel L2', eg, 'pd rel L2', ep)
    assert eg < 1e-6
    assert ep < 1e-3
    assert int(out['k'].item()) == 4


def test_learned_forward_full_size_sampled_series(gpu):
    import torch
    print('c2 learned', flush=True)
    iq = random_casorati(ACQ.n_vox, ACQ.n_frames, seed=5, rank=3, tissue_db=40)
    w = lcf_init_weights(3)
    wb = obf16.bf16_bits(w).view(np.int16)
    pd = torch.empty(ACQ.n_vox, dtype=torch.float32, device='cuda')
    gpu.lcf_forward(dev(w), dev(wb), dev(iq), 1e-30, None, None, pd)
    rng = np.random.default_rng(6)
    vox = rng.integers(0, ACQ.n_vox, 256)
    y = olcf.blood_estimate(w.astype(np.float64), iq[:, vox].astype(np.complex128), bf16=True)
    err = rel_l2(pd.cpu().numpy()[vox], np.mean(np.abs(y) ** 2, axis=0))
    print('c2 learned pd rel L2', err)
    assert err < 4e-3


def test_split_bf16_precision_variant_full_size(gpu):
    """The precision variant at full size (2.1M voxels x 200 frames): the three-product
    split-BF16 Gram on the matrix cores against its bit-exact FP64 emulation (only the
    accumulation order differs), and the power Doppler of that path, at the FP32 path's
    rank, against the FP64 oracle on sampled voxels."""
    print('c3 split-BF16', flush=True)
    iq = random_casorati(ACQ.n_vox, ACQ.n_frames, seed=7, rank=4, tissue_db=45)
    out = gpu_svd_pd(dev(iq), 4, mode=1)
    G = out['G'].cpu().numpy()
    Ge = obf16.gram_split_bf16(iq, 3)
    eg = rel_l2(G, Ge)
    Go = clutter.gram(iq)
    e_exact = rel_l2(G, Go)
    lam, V = clutter.eig_desc(Go)
    rng = np.random.default_rng(8)
    vox = rng.integers(0, ACQ.n_vox, 4096)
    pd_o = clutter.power_doppler(clutter.filter_iq(iq[:, vox].astype(np.complex128), V, 4))
    ep = rel_l2(out['pd'].cpu().numpy()[vox], pd_o)
    print('c3 split gram vs emulation', eg, 'vs exact', e_exact, 'pd vs FP64 oracle', ep)
    assert eg < 1e-6
    assert e_exact < 1e-4
    assert ep < 1e-3
    assert int(out['k'].item()) == 4
