"""Parity at the large configuration's geometry (32x32 array, 9 plane waves, 160x160x256
voxels, 1536 RF samples, PRF 2 kHz, 200k moving tissue + 30k blood scatterers in a
31-segment Murray tree), on its first 8 frames so that the case runs in seconds: sampled
RF traces of the real scene, sampled voxels of its beamformed IQ, and the full Gram with
sampled power-Doppler values of the clutter filter, against the FP64 oracle one by one.
Tolerances as for the throughput workload."""
import numpy as np
import pytest

from fqscene import get_config, make_scene
from fqscene.configs import scaled
from helpers import dev, gpu_das, gpu_rf, gpu_svd_pd, rel_l2
from oracle import clutter, native

pytestmark = pytest.mark.gpu

CFG = scaled(get_config('c5'), frames=8)
ACQ = CFG.acq


@pytest.fixture(scope='module')
def scene():
    return make_scene(CFG)


@pytest.fixture(scope='module')
def rf_iq(gpu, scene):
    print('c5 rf_synth + das (8 frames)', flush=True)
    rf = gpu_rf(ACQ, scene)
    iq = gpu_das(ACQ, rf, 0)
    return rf, iq


def test_c5_scene_is_the_large_configuration(scene):
    assert ACQ.n_elem == 1024 and ACQ.n_angles == 9 and (ACQ.nx, ACQ.ny, ACQ.nz) == (160, 160, 256)
    assert ACQ.n_samples == 1536 and ACQ.prf == 2000.0
    assert scene.tissue_amp.size == 200000 and scene.blood_amp.size == 30000 and len(scene.vessels) == 31


def test_c5_rf_sampled_traces(rf_iq, scene):
    rf, _ = rf_iq
    rng = np.random.default_rng(51)
    n = 16
    sel = np.stack([rng.integers(0, ACQ.n_frames, n), rng.integers(0, ACQ.n_angles, n),
                    rng.integers(0, ACQ.n_elem, n)], 1).astype(np.int32)
    got = np.stack([rf[f, a, e].cpu().numpy() for f, a, e in sel])
    want = native.rf_traces(ACQ, scene.tissue_pos, scene.tissue_amp, sel) + \
        native.rf_traces(ACQ, scene.blood_pos, scene.blood_amp, sel)
    err = rel_l2(got, want)
    print('c5 rf rel L2', err)
    assert err < 2e-5


def test_c5_das_sampled_voxels(rf_iq):
    import torch
    rf, iq = rf_iq
    rng = np.random.default_rng(52)
    corners = [0, ACQ.nx - 1, ACQ.n_vox - 1, ACQ.nx * ACQ.ny * (ACQ.nz - 1), 17 + ACQ.nx * 33 + ACQ.nx * ACQ.ny * 101]
    vox = np.concatenate([corners, rng.integers(0, ACQ.n_vox, 27)]).astype(np.int64)
    got = iq[:, torch.from_numpy(vox).cuda()].cpu().numpy()
    want = native.das_from_rf(ACQ, rf.cpu().numpy(), vox, 0)
    err = rel_l2(got, want)
    print('c5 das rel L2', err)
    assert err < 1e-4


def test_c5_clutter_filter(rf_iq):
    """The GPU IQ of the large volume through the filter at a fixed rank: full Gram and
    sampled PD against the oracle on the same (downloaded) IQ."""
    _, iq = rf_iq
    out = gpu_svd_pd(iq, 2)
    iq_h = iq.cpu().numpy()
    Go = clutter.gram(iq_h)
    eg = rel_l2(out['G'].cpu().numpy(), Go)
    lam, V = clutter.eig_desc(Go)
    rng = np.random.default_rng(53)
    vox = rng.integers(0, ACQ.n_vox, 4096)
    pd_o = clutter.power_doppler(clutter.filter_iq(iq_h[:, vox].astype(np.complex128), V, 2))
    ep = rel_l2(out['pd'].cpu().numpy()[vox], pd_o)
    print('c5 gram rel L2', eg, 'pd rel L2', ep)
    assert eg < 1e-6 and ep < 1e-3
