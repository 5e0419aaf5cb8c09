"""Edge cases through the C ABI: ragged voxel tiles and frame blocks, empty scenes,
odd and tiny ensemble lengths, full cutoff, invalid arguments on the device path."""
import numpy as np
import pytest

from fqscene import get_config, random_casorati
from fqscene.scene import point_scene
from helpers import dev, gpu_das, gpu_svd_pd, rel_l2, structs
from oracle import clutter, native

pytestmark = pytest.mark.gpu

C1 = get_config('c1').acq


@pytest.mark.parametrize('interp', [0, 1])
def test_das_ragged_grid_and_frames(gpu, interp):
    """19x23x13 voxels (no dimension a multiple of the 16x16x4 tile) and 11 frames
    (a partial 8-frame block), against the oracle on seeded random RF."""
    acq = C1.with_(nx=19, ny=23, nz=13, n_frames=11, z0=6e-3)
    rng = np.random.default_rng(21)
    rf = rng.standard_normal((acq.n_frames, acq.n_angles, acq.n_elem, acq.n_samples)).astype(np.float32)
    iq = gpu_das(acq, dev(rf), interp).cpu().numpy()
    want = native.das_from_bb(acq, native.rf2iq(rf, acq.fc, acq.fs), interp)
    assert rel_l2(iq, want) < 1e-4


def test_rf_synth_empty_scene(gpu):
    import torch
    acq = C1.with_(n_frames=3)
    probe, tx, grid, pulse = structs(acq)
    rf = torch.full((3, acq.n_angles, acq.n_elem, acq.n_samples), 7.0, dtype=torch.float32, device='cuda')
    empty = torch.zeros((1, 0, 3), dtype=torch.float32, device='cuda')
    gpu.rf_synth(probe, tx, pulse, empty, torch.zeros(0, dtype=torch.float32, device='cuda'), rf, accumulate=True)
    assert float(rf.min()) == 7.0 and float(rf.max()) == 7.0
    gpu.rf_synth(probe, tx, pulse, empty, torch.zeros(0, dtype=torch.float32, device='cuda'), rf, accumulate=False)
    assert float(rf.abs().max()) == 0.0


@pytest.mark.parametrize('T', [200, 201])
def test_rf_synth_scatterer_at_record_edges(gpu, T):
    """Pulses cut by the start and the end of the record (taps outside [0, T) dropped), for
    an even and an odd record length (the half-rate trace of the spreading form holds
    (T + 1) / 2 samples)."""
    acq = C1.with_(n_frames=1, tilts_deg=((0.0, 0.0),), n_samples=T)
    probe, tx, grid, pulse = structs(acq)
    z_early = 1.0 * 1540 / 31.25e6 * 5        # arrives ~10 samples after t = 0
    z_late = 1540 / 31.25e6 * 198 / 2          # arrives near the last sample
    z_past = 1540 / 31.25e6 * (T + 12) / 2     # arrives after the record: only its leading tail is in
    pos = np.array([[[0.0, 0.0, z_early], [0.3e-3, 0.1e-3, z_late], [0.0, 0.0, z_past]]], np.float32)
    amp = np.array([1.0, -0.5, 2.0], np.float32)
    import torch
    rf = torch.empty((1, 1, acq.n_elem, acq.n_samples), dtype=torch.float32, device='cuda')
    gpu.rf_synth(probe, tx, pulse, dev(pos), dev(amp), rf)
    sel = np.array([[0, 0, e] for e in range(acq.n_elem)], np.int32)
    want = native.rf_traces(acq, pos, amp, sel)
    assert rel_l2(rf.cpu().numpy().reshape(acq.n_elem, -1), want) < 2e-5


@pytest.mark.parametrize('nt', [1, 3, 7, 33, 64])
def test_gram_eig_small_and_odd_ensembles(gpu, nt):
    import torch
    iq = random_casorati(3000, nt, seed=nt, rank=min(2, nt)).astype(np.complex64)
    out = gpu_svd_pd(dev(iq), min(1, nt))
    G = out['G'].cpu().numpy()
    Go = clutter.gram(iq)
    assert rel_l2(G, Go) < 1e-6
    ws = torch.empty(gpu.svd_workspace_size(3000, nt), dtype=torch.uint8, device='cuda')
    lam = torch.empty(nt, dtype=torch.float64, device='cuda')
    vecs = torch.empty((nt, nt), dtype=torch.complex128, device='cuda')
    st = torch.full((1,), -1, dtype=torch.int32, device='cuda')
    gpu.hermitian_eig(dev(Go), ws, lam, vecs, st)
    lo, Vo = clutter.eig_desc(Go)
    assert int(st.item()) == 0
    np.testing.assert_allclose(lam.cpu().numpy(), lo, rtol=1e-9, atol=1e-12 * lo[0])
    V = vecs.cpu().numpy()
    np.testing.assert_allclose(V.conj().T @ V, np.eye(nt), atol=1e-10)
    np.testing.assert_allclose((V * lam.cpu().numpy()) @ V.conj().T, Go, atol=1e-9 * np.abs(Go).max())



@pytest.mark.parametrize('nv,nt', [(1, 5), (63, 40), (4097, 70), (9001, 33), (12289, 7)])
def test_gram_ragged_and_odd_voxel_counts(gpu, nv, nt):
    """Voxel counts that leave a partial 64-voxel stage, odd counts (rows not 16-byte
    aligned: the element-wise loads) and counts over several 4096-voxel ranges, in every
    Gram mode: FP32 against the FP64 Gram, the BF16 modes against their bit-exact
    emulation."""
    import torch
    from oracle import bf16 as obf16
    iq = random_casorati(nv, nt, seed=nv + nt, rank=min(3, nt)).astype(np.complex64)
    x = dev(iq)
    for mode, want in ((0, clutter.gram(iq)), (1, obf16.gram_split_bf16(iq, 3)),
                       (2, obf16.gram_split_bf16(iq, 1)), (3, obf16.gram_split_bf16(iq, 4))):
        ws = torch.empty(max(1, gpu.gram_workspace_size(nv, nt, mode)), dtype=torch.uint8, device='cuda')
        G = torch.empty((nt, nt), dtype=torch.complex128, device='cuda')
        gpu.casorati_gram(x, G, ws, mode)
        assert rel_l2(G.cpu().numpy(), want) < 1e-6, mode


@pytest.mark.parametrize('nt,bad', [(20, np.nan), (200, np.nan), (200, np.inf)])
def test_non_finite_gram_reports_numeric_status(gpu, nt, bad):
    """A Gram with a non-finite entry (the register-resident tridiagonalisation at 20 and 200
    frames) is reported through the status word, not returned as a power-Doppler volume."""
    import torch
    NV = 3000
    iq = random_casorati(NV, nt, seed=nt, rank=2).astype(np.complex64)
    G = clutter.gram(iq)
    G[3, 5] = G[5, 3] = bad
    ws = torch.empty(gpu.svd_workspace_size(NV, nt), dtype=torch.uint8, device='cuda')
    sigma = torch.empty(nt, dtype=torch.float64, device='cuda')
    k = torch.zeros(1, dtype=torch.int32, device='cuda')
    st = torch.full((1,), -1, dtype=torch.int32, device='cuda')
    pd = torch.empty(NV, dtype=torch.float32, device='cuda')
    gpu.svd_clutter_filter(dev(iq), dev(G), ws, sigma, k, -1, pd=pd, status=st)
    assert int(st.item()) == 4   # FQ_E_NUMERIC
    assert 1 <= int(k.item()) <= 64

def test_full_cutoff_removes_everything(gpu):
    iq = random_casorati(2000, 12, seed=5).astype(np.complex64)
    out = gpu_svd_pd(dev(iq), 12)
    raw = clutter.power_doppler(iq)
    assert float(out['pd'].abs().max()) < 1e-5 * raw.max()


def test_degenerate_repeated_frames(gpu):
    """All frames identical: rank-one Casorati, eigenvalues 0 after the first, PD ~ 0 for K = 1."""
    rng = np.random.default_rng(4)
    vol = (rng.standard_normal(5000) + 1j * rng.standard_normal(5000)).astype(np.complex64)
    iq = np.repeat(vol[None], 10, 0)
    out = gpu_svd_pd(dev(iq), 1)
    s = out['sigma'].cpu().numpy()
    assert s[1] < 1e-3 * s[0]        # round-off of the FP32-accumulated Gram only
    assert float(out['pd'].max()) < 1e-8 * np.mean(np.abs(vol) ** 2)


def test_invalid_workspace_is_reported(gpu):
    import torch
    acq = C1.with_(n_frames=2)
    probe, tx, grid, _ = structs(acq)
    rf = torch.zeros((2, acq.n_angles, acq.n_elem, acq.n_samples), dtype=torch.float32, device='cuda')
    iq = torch.empty((2, acq.n_vox), dtype=torch.complex64, device='cuda')
    ws = torch.empty(1024, dtype=torch.uint8, device='cuda')
    with pytest.raises(gpu.FqError) as e:
        gpu.das_beamform(probe, tx, grid, rf, iq, ws)
    assert e.value.status == 2


@pytest.mark.parametrize('n_cycles,trunc', [(2.0, 5.0), (2.0, 3.0), (1.0, 2.0), (1.0, 1.2), (0.5, 1.0),
                                            (0.5, 1.5), (4.0, 4.5), (4.0, 4.6), (3.0, 5.0), (5.0, 6.0)])
def test_rf_synth_pulse_lengths(gpu, n_cycles, trunc):
    """Both forms of the synthesis at fc / fs = 7.8 / 31.25 MHz.  Direct form (pulse cut
    below 5 sigma, or narrower than 3.3 samples): half-widths J = floor(trunc * sigma) of
    both parities from 0 to the largest supported (10, 3, 2, 0, 1, 30, 31 samples), the
    taps added in pairs of samples whose first pair start and edge-tap masks depend on J.
    Spreading form (kept to >= 5 sigma, sigma >= 3.3 samples): 10, 16 and 26 half-rate taps
    (2, 3 and 5 cycles; the last one longer than the direct form supports).  Scatterers
    cover the whole record and beyond both ends, over two moving frames."""
    import torch
    import paper_2509_05464_amd as fq
    acq = C1.with_(n_frames=2)
    probe, tx, grid, _ = structs(acq)
    pulse = fq.make_pulse(n_cycles, trunc, 1e-3)
    rng = np.random.default_rng(int(10 * n_cycles + 100 * trunc))
    S = 300
    z_end = acq.n_samples * acq.c / acq.fs / 2
    pos = np.stack([rng.uniform(-3e-3, 3e-3, (2, S)), rng.uniform(-3e-3, 3e-3, (2, S)),
                    rng.uniform(0.02e-3, 1.03 * z_end, (2, S))], axis=2).astype(np.float32)
    amp = rng.standard_normal(S).astype(np.float32)
    rf = torch.empty((2, acq.n_angles, acq.n_elem, acq.n_samples), dtype=torch.float32, device='cuda')
    gpu.rf_synth(probe, tx, pulse, dev(pos), dev(amp), rf, pos_static=False)
    sel = native.all_traces(2, acq.n_angles, acq.n_elem)
    want = native.rf_traces(acq, pos, amp, sel, dict(n_cycles=n_cycles, trunc_sigmas=trunc, r_ref=1e-3))
    err = rel_l2(rf.cpu().numpy().reshape(sel.shape[0], -1), want)
    print('pulse', n_cycles, trunc, 'rf rel L2', err)
    assert err < 2e-5


@pytest.mark.parametrize('nt,cutoff', [(200, -1), (64, 20), (33, 3)])
def test_filter_apply_after_eig_equals_one_call(gpu, nt, cutoff):
    """The filter's last stage run by svd_filter_apply on a second stream, after a
    svd_clutter_filter call that stops at the cutoff, gives what one svd_clutter_filter
    call gives, bit for bit (filtered IQ and PD; PD alone too)."""
    import torch
    nv = 40000
    print('filter apply n_t', nt, 'cutoff', cutoff, flush=True)
    iq = dev(random_casorati(nv, nt, seed=300 + nt, rank=3).astype(np.complex64))
    G = torch.empty((nt, nt), dtype=torch.complex128, device='cuda')
    gws = torch.empty(gpu.gram_workspace_size(nv, nt, 0), dtype=torch.uint8, device='cuda')
    gpu.casorati_gram(iq, G, gws, 0)

    def run(ws, **out):
        sigma = torch.empty(nt, dtype=torch.float64, device='cuda')
        k = torch.zeros(1, dtype=torch.int32, device='cuda')
        st = torch.full((1,), -1, dtype=torch.int32, device='cuda')
        gpu.svd_clutter_filter(iq, G, ws, sigma, k, cutoff, status=st, **out)
        return k, st

    ws1 = torch.empty(gpu.svd_workspace_size(nv, nt), dtype=torch.uint8, device='cuda')
    ws2 = torch.empty_like(ws1)
    iqf1, pd1, pd1b = torch.empty_like(iq), torch.empty(nv, device='cuda'), torch.empty(nv, device='cuda')
    k1, st1 = run(ws1, iq_filt=iqf1, pd=pd1)
    run(ws1, pd=pd1b)
    k2, st2 = run(ws2)
    done = torch.cuda.Event()
    done.record()
    side = torch.cuda.Stream()
    iqf2, pd2, pd2b = torch.empty_like(iq), torch.empty(nv, device='cuda'), torch.empty(nv, device='cuda')
    with torch.cuda.stream(side):
        side.wait_event(done)
        gpu.svd_filter_apply(iq, ws2, k2, iq_filt=iqf2, pd=pd2)
        gpu.svd_filter_apply(iq, ws2, k2, pd=pd2b)
    torch.cuda.synchronize()
    assert int(st1.item()) == 0 and int(st2.item()) == 0
    assert int(k1.item()) == int(k2.item())
    assert torch.equal(iqf1, iqf2) and torch.equal(pd1, pd2) and torch.equal(pd1b, pd2b)
