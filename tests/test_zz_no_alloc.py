"""The allocation-free Gram entry point (partial tiles in the library's static device
array) against casorati_gram with a caller workspace, through the C ABI: two calls in a
row on the same GPU, the second with a smaller input, each checked against the
workspace entry point on the same data.  Only the number of voxel ranges differs
between the two, so the results agree to FP64 summation order."""
import numpy as np
import pytest

from fqscene import random_casorati
from helpers import dev, rel_l2

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize('mode', [0, 1, 3])
def test_noalloc_gram_matches_workspace_gram(gpu, mode):
    import torch
    for nv, nt in ((200000, 400), (30011, 200)):
        print('noalloc gram mode', mode, 'n_vox', nv, 'n_t', nt, flush=True)
        iq = dev(random_casorati(nv, nt, seed=nt + mode, rank=4, tissue_db=45))
        ws = torch.empty(gpu.gram_workspace_size(nv, nt, mode), dtype=torch.uint8, device='cuda')
        G_ref = torch.empty((nt, nt), dtype=torch.complex128, device='cuda')
        gpu.casorati_gram(iq, G_ref, ws, mode)
        G = torch.full((nt, nt), float('nan'), dtype=torch.complex128, device='cuda')
        gpu.casorati_gram_noalloc(iq, G, mode)
        torch.cuda.synchronize()
        g, r = G.cpu().numpy(), G_ref.cpu().numpy()
        assert np.isfinite(g).all()
        err = rel_l2(g, r)
        print('noalloc vs workspace rel L2', err)
        assert err < 1e-12
