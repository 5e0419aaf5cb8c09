"""End to end on the GPU, a property that holds for any correct path: after the clutter
filter removes the static tissue of the small workload, the power Doppler inside the
vessel lumen is far above the power Doppler outside it.  Run with the time-domain RF
synthesis of the hot path and with the frequency-domain model (point elements and with
directivity, sub-elements and attenuation), whose RF feeds the same beamformer."""
import numpy as np
import pytest

from fqscene import get_config, make_scene
from fqscene.scene import _inside_any
from helpers import dev, gpu_das, gpu_rf, gpu_svd_pd

pytestmark = pytest.mark.gpu

CFG = get_config('c1')
ACQ = CFG.acq


def voxel_centres():
    ix = np.arange(ACQ.n_vox) % ACQ.nx
    iy = (np.arange(ACQ.n_vox) // ACQ.nx) % ACQ.ny
    iz = np.arange(ACQ.n_vox) // (ACQ.nx * ACQ.ny)
    return np.stack([ACQ.x0 + ix * ACQ.dx, ACQ.y0 + iy * ACQ.dy, ACQ.z0 + iz * ACQ.dz], 1)


def fd_rf(sc, elem_w, n_sub, atten):
    import torch
    import paper_2509_05464_amd as fq
    probe = fq.make_probe(ACQ.nx_el, ACQ.ny_el, ACQ.pitch, ACQ.pitch, ACQ.fc, ACQ.fs, ACQ.c)
    tx = fq.make_tx(ACQ.tilts_rad())
    pulse = fq.make_pulse(2.0, 5.0, 1e-3)
    fdp = fq.make_fd_params(elem_w, n_sub, atten, 1e-7)
    n = max(sc.tissue_amp.size, sc.blood_amp.size)
    ws = torch.empty(fq.fd_workspace_size(probe, tx, pulse, fdp, ACQ.n_samples, n), dtype=torch.uint8, device='cuda')
    rf = torch.empty((ACQ.n_frames, ACQ.n_angles, ACQ.n_elem, ACQ.n_samples), dtype=torch.float32, device='cuda')
    fq.fd_synth(probe, tx, pulse, fdp, dev(sc.tissue_pos), dev(sc.tissue_amp), rf, ws, pos_static=True)
    fq.fd_synth(probe, tx, pulse, fdp, dev(sc.blood_pos), dev(sc.blood_amp), rf, ws, accumulate=True)
    return rf


@pytest.mark.parametrize('model', ['time_domain', 'fd_point', 'fd_directive'])
def test_vessel_stands_out_after_the_clutter_filter(gpu, model):
    sc = make_scene(CFG)
    if model == 'time_domain':
        rf = gpu_rf(ACQ, sc)
    elif model == 'fd_point':
        rf = fd_rf(sc, (0.0, 0.0), (1, 1), 0.0)
    else:
        rf = fd_rf(sc, (0.27e-3, 0.27e-3), (2, 2), 0.5)
    iq = gpu_das(ACQ, rf, 0)
    raw = gpu_svd_pd(iq, 0)['pd'].cpu().numpy()
    pd = gpu_svd_pd(iq, 1)['pd'].cpu().numpy()
    inside = _inside_any(voxel_centres(), sc.vessels)
    # voxels well away from the lumen (beyond one pulse length from its wall)
    v = sc.vessels[0]
    d = voxel_centres() - v.centre
    s = d @ v.axis
    r = np.sqrt(np.maximum(np.einsum('ij,ij->i', d, d) - s * s, 0.0))
    outside = r > v.radius + 1.0e-3
    c_raw = raw[inside].mean() / raw[outside].mean()
    c_pd = pd[inside].mean() / pd[outside].mean()
    print(model, 'lumen/background PD before', c_raw, 'after', c_pd, 'voxels in lumen', int(inside.sum()))
    assert inside.sum() > 100 and outside.sum() > 10000
    assert c_pd > 30.0 and c_pd > 10.0 * c_raw
