"""The C-ABI library loads and exports every entry point include/fqpd.h declares, and
the binding rejects host tensors before any device call (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, 'include', 'fqpd.h')
LIB = os.path.join(ROOT, 'paper_2509_05464_amd', 'libfqpd.so')


def declared():
    text = open(HEADER).read()
    text = re.sub(r'/\*.*?\*/', '', text, flags=re.S)
    names = re.findall(r'^\s*(?:const\s+)?(?:int|size_t|char\s*\*|const\s+char\s*\*)\s*\**\s*(\w+)\s*\(',
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope='module')
def lib():
    if not os.path.exists(LIB):
        pytest.fail('libfqpd.so is not built (run __graft_entry__.build())')
    return ctypes.CDLL(LIB)


def test_header_declares_the_path():
    names = declared()
    for want in ('rf_synth', 'das_beamform', 'casorati_gram', 'svd_clutter_filter', 'power_doppler',
                 'lcf_forward', 'lcf_backward', 'lcf_adam_step', 'fq_workspace_size', 'fq_last_error'):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    from paper_2509_05464_amd import _lib
    assert set(declared()) <= set(_lib._SIGS)


def test_workspace_queries_without_gpu(lib):
    """Size queries are pure host arithmetic."""
    import paper_2509_05464_amd as fq
    from fqscene import get_config
    acq = get_config('c2').acq
    probe = fq.make_probe(acq.nx_el, acq.ny_el, acq.pitch, acq.pitch, acq.fc, acq.fs, acq.c)
    tx = fq.make_tx(acq.tilts_rad())
    full = fq.das_workspace_size(probe, tx, acq.n_frames, acq.n_samples, False)
    blk = fq.das_workspace_size(probe, tx, acq.n_frames, acq.n_samples, True)
    assert full == blk * 25 and blk == acq.n_angles * acq.n_elem * acq.n_samples * 8 * 8
    assert fq.gram_workspace_size(acq.n_vox, acq.n_frames, 0) > 0
    assert fq.svd_workspace_size(acq.n_vox, acq.n_frames) > 0
    pulse = fq.make_pulse()
    fdp = fq.make_fd_params((0.27e-3, 0.27e-3), (2, 2), 0.5)
    small = fq.fd_workspace_size(probe, tx, pulse, fdp, acq.n_samples, 256)
    big = fq.fd_workspace_size(probe, tx, pulse, fdp, acq.n_samples, 70000)
    assert 0 < small < big
    assert fq.fd_workspace_size(probe, tx, pulse, fq.make_fd_params(n_sub=(0, 1)), acq.n_samples, 256) == 0
    # the SSM pass: 512 workgroup partials of a 64 x 64 Gram plus 64 column sums at most,
    # and the filter's workspace covers it
    ssm = fq.ssm_workspace_size(acq.n_vox, acq.n_frames)
    assert 512 * (64 * 64 + 64) * 8 <= ssm < 512 * (64 * 64 + 64) * 8 + (1 << 20)
    assert fq.ssm_workspace_size(100, 20) < ssm
    assert fq.svd_workspace_size(acq.n_vox, acq.n_frames) > ssm
    assert fq.lcf_act_size(4096, 200) > 4096 * 200 * 194 * 2


def test_one_workspace_query_matches_the_per_call_queries(lib):
    """fq_workspace_size dispatches to the per-call queries; unknown kinds, a NULL query or
    a missing struct give 0 (host arithmetic only)."""
    import ctypes
    import paper_2509_05464_amd as fq
    from fqscene import get_config
    for name in ('c1', 'c2', 'c5'):
        acq = get_config(name).acq
        probe = fq.make_probe(acq.nx_el, acq.ny_el, acq.pitch, acq.pitch, acq.fc, acq.fs, acq.c)
        tx = fq.make_tx(acq.tilts_rad())
        F, T, NV = acq.n_frames, acq.n_samples, acq.n_vox
        assert fq.fq_workspace_size(fq.WS_DAS, probe, tx, n_t=F, n_samples=T) == \
            fq.das_workspace_size(probe, tx, F, T, False) > 0
        assert fq.fq_workspace_size(fq.WS_DAS_MIN, probe, tx, n_t=F, n_samples=T) == \
            fq.das_workspace_size(probe, tx, F, T, True) > 0
        for mode in (fq.GRAM_FP32, fq.GRAM_SPLIT_BF16, fq.GRAM_SPLIT4_BF16, fq.GRAM_BF16):
            assert fq.fq_workspace_size(fq.WS_GRAM, n=NV, n_t=F, gram_mode=mode) == \
                fq.gram_workspace_size(NV, F, mode) > 0
        assert fq.fq_workspace_size(fq.WS_SVD, n=NV, n_t=F) == fq.svd_workspace_size(NV, F) > 0
        assert fq.fq_workspace_size(fq.WS_SSM, n=NV, n_t=F) == fq.ssm_workspace_size(NV, F) > 0
        assert fq.fq_workspace_size(fq.WS_DISPLAY, n=NV) == fq.display_workspace_size(NV) > 0
        assert fq.fq_workspace_size(fq.WS_FALLBACK, n=NV) == fq.fallback_workspace_size(NV) > 0
        assert fq.fq_workspace_size(fq.WS_LCF_ACT, n=4096, n_t=F) == fq.lcf_act_size(4096, F) > 0
        pulse = fq.make_pulse()
        fdp = fq.make_fd_params((0.27e-3, 0.27e-3), (2, 2), 0.5)
        assert fq.fq_workspace_size(fq.WS_FD, probe, tx, pulse, fdp, n=1000, n_samples=T) == \
            fq.fd_workspace_size(probe, tx, pulse, fdp, T, 1000) > 0
        # a query without the structs it reads
        assert fq.fq_workspace_size(fq.WS_DAS, n_t=F, n_samples=T) == 0
        assert fq.fq_workspace_size(fq.WS_FD, probe, tx, n=1000, n_samples=T) == 0
    assert fq.fq_workspace_size(99, n=10, n_t=4) == 0
    assert fq.fq_workspace_size(fq.WS_GRAM, n=0, n_t=4) == 0
    assert lib.fq_workspace_size(fq.WS_GRAM, None) == 0


def test_invalid_arguments_return_status(lib):
    """Argument checks run on the host before any launch: bad sizes give FQ_E_INVALID
    with a message (here with null pointers, so nothing touches a device)."""
    import paper_2509_05464_amd as fq
    L = fq.lib()
    st = L.power_doppler(None, 10, 4, None, None)
    assert st == 1 and b'null' in L.fq_last_error()
    st = L.casorati_gram(None, 10, 0, 0, None, 0, None, None)
    assert st == 1
    st = L.svd_clutter_filter(None, 10, 600, None, 2, None, 0, None, None, None, None, None, None)
    assert st == 1 and b'n_t' in L.fq_last_error()
    st = L.svd_clutter_filter(None, 10, 20, None, -3, None, 0, None, None, None, None, None, None)
    assert st == 1 and b'cutoff' in L.fq_last_error()
    st = L.svd_filter_apply(None, 10, 600, None, 0, None, None, None, None)
    assert st == 1 and b'n_t' in L.fq_last_error()
    st = L.spatial_similarity(None, 10, 20, None, 1, None, 0, None, None, None)
    assert st == 1 and b'n_modes' in L.fq_last_error()
    st = L.spatial_similarity(None, 10, 20, None, 21, None, 0, None, None, None)
    assert st == 1 and b'n_modes' in L.fq_last_error()
    st = L.spatial_similarity(None, 10, 100, None, 65, None, 0, None, None, None)
    assert st == 1 and b'n_modes' in L.fq_last_error()
    st = L.spatial_similarity(None, 10, 20, None, 4, None, 0, None, None, None)
    assert st == 1 and b'null' in L.fq_last_error()
    st = L.display_db(None, 10, 4, 60.0, None, 0, None, None, None)
    assert st == 1 and b'kind' in L.fq_last_error()
    st = L.display_db(None, 10, 0, -5.0, None, 0, None, None, None)
    assert st == 1 and b'dr_db' in L.fq_last_error()
    st = L.mip(None, 4, 4, 4, 3, None, None)
    assert st == 1 and b'plane' in L.fq_last_error()
    st = L.mip(None, 0, 4, 4, 0, None, None)
    assert st == 1 and b'size' in L.fq_last_error()
    st = L.image_quality(None, None, 10, 64, 1.0, None, None)
    assert st == 1 and b'window' in L.fq_last_error()
    st = L.image_quality(None, None, 64, 64, 0.0, None, None)
    assert st == 1 and b'data_range' in L.fq_last_error()
    import ctypes
    probe = fq.make_probe(4, 4, 3e-4, 3e-4, 7.8e6, 31.25e6, 1540.0)
    tx = fq.make_tx([(0.0, 0.0)])
    pulse = fq.make_pulse()
    # RF synthesis: pulses neither form takes (a 5-cycle pulse cut at 4.9 sigma: direct form,
    # half-width 41 samples > 31; an 8-cycle pulse kept to 5 sigma: 48 half-rate taps, more
    # than the spreading form's 32, so it falls back to the direct form, half-width 68) and a
    # record longer than 8192 samples; the device pointers are placeholders that are never
    # dereferenced on these paths
    fake = ctypes.c_void_p(1 << 20)
    for n_cyc, trunc in ((5.0, 4.9), (8.0, 5.0)):
        long_pulse = fq.make_pulse(n_cyc, trunc, 1e-3)
        st = L.rf_synth(ctypes.byref(probe), ctypes.byref(tx), ctypes.byref(long_pulse), 1, 1, fake, 1, fake, 256,
                        0, fake, None)
        assert st == 1 and b'pulse longer' in L.fq_last_error()
    st = L.rf_synth(ctypes.byref(probe), ctypes.byref(tx), ctypes.byref(pulse), 1, 1, fake, 1, fake, 9000, 0,
                    fake, None)
    assert st == 1 and b'n_samples' in L.fq_last_error()
    bad = fq.make_fd_params(spectral_floor=0.0)
    st = L.fd_synth(ctypes.byref(probe), ctypes.byref(tx), ctypes.byref(pulse), ctypes.byref(bad), 1, 1, None, 0,
                    None, None, 64, 0, None, 0, None, None)
    assert st == 1 and b'spectral_floor' in L.fq_last_error()
