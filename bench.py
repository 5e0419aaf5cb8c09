#!/usr/bin/env python3
"""Throughput of the ultrafast power-Doppler reconstruction path on one MI355X.

One step = one pass of the whole path over one slow-time ensemble of the large
workload (32x32 array, 9 plane waves, 160x160x256 voxels, 400 frames at 2 kHz,
200k moving tissue scatterers + 30k blood scatterers in a 31-segment vessel tree):
RF synthesis -> rf2iq -> delay-and-sum -> Casorati Gram (FP32) -> FP64
eigendecomposition + knee -> projection + power Doppler, then the same clutter filter
from a split-BF16 Gram, then the learned filter (inference, fallback judge, one
training step).  Inputs (scatterer scenes) are resident in HBM before the timed
region.

Prints one JSON line.  `value` is DAS voxel*element*angle products (each frame
counted) per second of whole-step time, in G/s.  Beside the headline: the throughput
workload (128^3 voxels, 200 frames) under "c2", the DAS timing of the paper's
2 cm-cube shape for 1/3/10/30 frames under "p7_das", the filters compared at matched
error against the blood-only ground truth, and the FP64 oracle's CPU rate and its
per-result check of the precision variants.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3  # published MI355X FP32 vector peak (256 CUs, 2.4 GHz)
PEAK_FP32_MFMA_TFLOPS = 157.3    # published dense FP32 matrix-core peak
DAS_FLOP_PER_UNIT = 16           # two complex multiply-adds per voxel*element*angle*frame (linear)
def rf_taps(acq, n_scat: int) -> float:
    """Pulse samples of the direct sum (the definition): per (scatterer, element, transmit,
    frame) the samples with |n - x| <= 5 sigma, 2 * 5 sigma on average."""
    sig = 2.0 / (2.0 * np.sqrt(2.0 * np.log(2.0)) * acq.fc) * acq.fs
    return float(n_scat) * acq.n_elem * acq.n_angles * acq.n_frames * 2.0 * 5.0 * sig


def rf_work(acq, n_scat: int, moving: bool = True) -> dict:
    """Arithmetic of the RF synthesis as the library performs it for the 2-cycle pulse kept
    to 5 sigma (the spreading form: sigma >= 3.3 samples): per (scatterer, element,
    transmit, frame) NT half-rate complex taps at 6 FLOP (two multiplies by the tap ratio,
    two FMAs with the Gaussian factor, two adds into the trace); per trace T outputs of the
    interpolation filter, P + 1 complex-by-real MACs (4 FLOP) and the carrier (4 FLOP)."""
    sig = 2.0 / (2.0 * np.sqrt(2.0 * np.log(2.0)) * acq.fc) * acq.fs
    s2 = sig * sig
    q = 4.0 * 2.614 / s2
    alpha = max(1.0 / 3.0, 0.5 * (1.0 - np.sqrt(1.0 - q))) if q < 1.0 else 0.5
    aphi, bpsi = alpha * s2, (1.0 - alpha) * s2
    nt = 2 * int(np.ceil(0.5 * np.sqrt(24.0 * aphi)))
    P = int(np.ceil(np.sqrt(2.0 * bpsi * 17.0)))
    traces = acq.n_elem * acq.n_angles * (acq.n_frames if moving else 1)
    records = float(n_scat) * acq.n_elem * acq.n_angles * acq.n_frames
    flop = records * nt * 6.0 + float(traces) * acq.n_samples * ((P + 1) * 4.0 + 4.0)
    return {'kernel': 'rf_spread_kernel', 'taps': nt, 'psi_half_width': P, 'flop': flop,
            'work': f'{nt} half-rate complex taps per scatterer*element*angle*frame at 6 FLOP + '
                    f'per trace {acq.n_samples} outputs of a {2 * P + 1}-tap interpolation filter '
                    f'(4 FLOP per tap) and the carrier (4 FLOP)'}


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def profile_values(name: str):
    """The 'key: value' block of a committed profile summary, or None when the summary is
    missing or the kernel sources changed since it was measured."""
    import hashlib
    path = os.path.join(ROOT, 'profiles', name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ':' in line and not line.startswith(('#', '|', ' ', '-')):
            k, v = line.split(':', 1)
            kv[k.strip()] = v.strip()
    try:
        h = hashlib.sha256()
        for src in kv['sources'].split():
            with open(os.path.join(ROOT, src), 'rb') as fh:
                h.update(fh.read())
        return kv if h.hexdigest() == kv['sources_sha256'] else None
    except (KeyError, OSError):
        return None


def measured_fma_tflops():
    """FP32 FMA rate the library's own probe reached with plain (non-packed) FMAs, from the
    committed probe summary (None when missing or the probe source changed)."""
    kv = profile_values('roof_probes.md')
    return float(kv['fp32_fma_tflops']) if kv and 'fp32_fma_tflops' in kv else None


def measured_traffic(name: str):
    """HBM bytes per launch of a kernel from its committed counter summary (FETCH_SIZE and
    WRITE_SIZE runs, each scaled by a copy kernel of known size), or None when the
    summary is missing or the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, 'profiles', name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ':' in line and not line.startswith(('#', '|', ' ', '-')):
            k, v = line.split(':', 1)
            kv[k.strip()] = v.strip()
    try:
        h = hashlib.sha256()
        for src in kv['sources'].split():
            with open(os.path.join(ROOT, src), 'rb') as fh:
                h.update(fh.read())
        if h.hexdigest() != kv['sources_sha256']:
            return None
        return float(kv['traffic_bytes_per_launch'])
    except (KeyError, OSError, ValueError):
        return None


def cpu_baseline(cfg, budget_s: float = 20.0) -> dict:
    """The FP64 oracle timed on a bounded sample of the same workload, extrapolated to
    the full step (RF synthesis, rf2iq, DAS and the clutter filter all scale linearly in
    their sampled dimension)."""
    from fqscene import make_scene, random_rf, random_casorati
    from oracle import clutter, native
    acq = cfg.acq
    threads = int(os.environ.get('OMP_NUM_THREADS', os.cpu_count() or 1))
    sc = make_scene(cfg)
    F, A, E, T = acq.n_frames, acq.n_angles, acq.n_elem, acq.n_samples
    # RF: a sample of traces of frame 0 (tissue + blood)
    n_tr = 4 * threads
    rng = np.random.default_rng(0)
    sel = np.stack([np.zeros(n_tr, np.int32), rng.integers(0, A, n_tr), rng.integers(0, E, n_tr)], 1).astype(np.int32)
    t0 = time.perf_counter()
    native.rf_traces(acq, sc.tissue_pos[:1], sc.tissue_amp, sel)
    native.rf_traces(acq, sc.blood_pos[:1], sc.blood_amp, sel)
    t_rf = (time.perf_counter() - t0) / n_tr * (F * A * E)
    # rf2iq + DAS: 8 frames of seeded RF, all traces demodulated, a sample of voxels
    fs_ = 8
    rf = random_rf(fs_, A, E, T, seed=3)
    t0 = time.perf_counter()
    bb = native.rf2iq(rf, acq.fc, acq.fs)
    t_demod = (time.perf_counter() - t0) * F / fs_
    del rf
    n_vox = 8 * threads
    vox = rng.integers(0, acq.n_vox, n_vox)
    a8 = acq.with_(n_frames=fs_)
    t0 = time.perf_counter()
    bbl = native.bb_frames_inner(bb)
    t_demod += (time.perf_counter() - t0) * F / fs_
    del bb
    t0 = time.perf_counter()
    native.das_from_layout(a8, bbl, 0, vox)
    t_das = (time.perf_counter() - t0) / n_vox * acq.n_vox * F / fs_
    bb = bbl
    del bb
    # clutter filter on a sub-volume of a seeded Casorati matrix
    nv_s = 1 << 15
    iq = random_casorati(nv_s, F, seed=4)
    t0 = time.perf_counter()
    clutter.svd_filter_pd(iq, -1)
    t_svd = (time.perf_counter() - t0) * acq.n_vox / nv_s
    total = t_rf + t_demod + t_das + t_svd
    cpu_model = 'unknown'
    try:
        for line in open('/proc/cpuinfo'):
            if line.startswith('model name'):
                cpu_model = line.split(':', 1)[1].strip()
                break
    except OSError:
        pass
    return {
        'value': acq.das_units() / total / 1e9,
        'unit': 'Gvoxel*element*angle/s',
        'cores': threads,
        'cpu_model': cpu_model,
        'kind': 'oracle',
        'sample': (f'FP64 oracle on {threads} threads, extrapolated linearly to the full step: RF synthesis of '
                   f'{n_tr} traces of frame 0 (of {F * A * E}), rf2iq of all traces of {fs_} frames of seeded RF '
                   f'(of {F}), DAS of {n_vox} voxels x {fs_} frames (of {acq.n_vox} x {F}), Gram/eig/knee/filter/PD '
                   f'on {nv_s} voxels (of {acq.n_vox})'),
        'stage_s_extrapolated': {'rf_synth': t_rf, 'rf2iq': t_demod, 'das': t_das, 'svd_filter_pd': t_svd},
        'step_s_extrapolated': total,
    }


def das_only(cfg, args, fq, torch, dev):
    acq = cfg.acq
    F, A, E, T, NV = acq.n_frames, acq.n_angles, acq.n_elem, acq.n_samples, acq.n_vox
    probe = fq.make_probe(acq.nx_el, acq.ny_el, acq.pitch, acq.pitch, acq.fc, acq.fs, acq.c)
    tx = fq.make_tx(acq.tilts_rad())
    grid = fq.make_grid(acq.nx, acq.ny, acq.nz, acq.x0, acq.y0, acq.z0, acq.dx, acq.dy, acq.dz)
    gen = torch.Generator(device=dev)
    gen.manual_seed(3)
    rf = torch.randn((F, A, E, T), device=dev, generator=gen)
    ws = torch.empty(fq.das_workspace_size(probe, tx, F, T), dtype=torch.uint8, device=dev)
    iq = torch.empty((F, NV), dtype=torch.complex64, device=dev)
    fq.das_demodulate(probe, tx, rf, ws)
    del rf
    src = torch.zeros(1 << 31, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)                      # calibration copy: 2 GiB read + 2 GiB written
    for _ in range(args.warmup):
        fq.das_delay_sum(probe, tx, grid, T, ws, iq)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        fq.das_delay_sum(probe, tx, grid, T, ws, iq)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    units = acq.das_units()
    print(json.dumps({'kernel': 'das_kernel', 'workload': cfg.name, 'ms_per_launch': ms,
                      'gunits_per_s': units / (ms / 1e3) / 1e9,
                      'tflops': DAS_FLOP_PER_UNIT * units / (ms / 1e3) / 1e12}))


_CU_SPLIT = {}


def cu_split_streams(torch, n_small):
    """Two streams at the default priority: one held to n_small CUs spread over the XCDs
    (CU indices 0, 33, 66, ...), the other to the remaining CUs, by the HIP runtime's
    CU-mask stream (the runtime torch itself loaded).  Falls back to two ordinary streams
    if that call is not available; returns (streams, masked, release).  The pair is made
    once per process and kept to its end (making a second pair after destroying the first
    has failed its first launch)."""
    if n_small not in _CU_SPLIT:
        _CU_SPLIT[n_small] = _make_cu_split(torch, n_small)
    streams, masked = _CU_SPLIT[n_small]
    return streams, masked, torch.cuda.synchronize


def _make_cu_split(torch, n_small):
    import ctypes
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    path = None
    with open('/proc/self/maps') as f:
        for line in f:
            if 'libamdhip64' in line:
                path = line.split()[-1]
                break
    try:
        hip = ctypes.CDLL(path)
        create = hip.hipExtStreamCreateWithCUMask
        create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]
        destroy = hip.hipStreamDestroy
        destroy.argtypes = [ctypes.c_void_p]
    except (OSError, AttributeError, TypeError):
        return (torch.cuda.Stream(), torch.cuda.Stream()), False
    small = {(33 * i) % ncu for i in range(n_small)}
    nw = (ncu + 31) // 32
    handles = []
    for members in (set(range(ncu)) - small, small):
        words = [0] * nw
        for c in members:
            words[c // 32] |= 1 << (c % 32)
        h = ctypes.c_void_p()
        if create(ctypes.byref(h), nw, (ctypes.c_uint32 * nw)(*words)) != 0:
            for x in handles:
                destroy(x)
            return (torch.cuda.Stream(), torch.cuda.Stream()), False
        handles.append(h)
    return tuple(torch.cuda.ExternalStream(h.value) for h in handles), True


def capture_graph(fn, torch):
    """fn (a clutter-filter path: kernel launches only, its size classes chosen on the device)
    captured once as a HIP graph, after one run on a side stream; replaying it drops the launch
    gaps between its dependent kernels."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


def filters_only(cfg, args, fq, torch, dev):
    """The three power-Doppler paths (FP32 SVD, four-product split-BF16 SVD, learned inference)
    on the workload's own ensemble (scene -> RF -> DAS, untimed), each run `steps` times after
    `warmup`, for profiler runs (kernel traces and counters of the Gram, eigensolver,
    projection and learned-filter kernels)."""
    from paper_2509_05464_amd.learned import LearnedFilter
    from fqscene import lcf_init_weights, make_scene
    acq = cfg.acq
    F, A, E, T, NV = acq.n_frames, acq.n_angles, acq.n_elem, acq.n_samples, acq.n_vox
    sc = make_scene(cfg)
    probe = fq.make_probe(acq.nx_el, acq.ny_el, acq.pitch, acq.pitch, acq.fc, acq.fs, acq.c)
    tx = fq.make_tx(acq.tilts_rad())
    grid = fq.make_grid(acq.nx, acq.ny, acq.nz, acq.x0, acq.y0, acq.z0, acq.dx, acq.dy, acq.dz)
    pulse = fq.make_pulse(2.0, 5.0, 1e-3)
    rf = torch.empty((F, A, E, T), dtype=torch.float32, device=dev)
    t_pos, t_amp = torch.from_numpy(sc.tissue_pos).to(dev), torch.from_numpy(sc.tissue_amp).to(dev)
    b_pos, b_amp = torch.from_numpy(sc.blood_pos).to(dev), torch.from_numpy(sc.blood_amp).to(dev)
    fq.rf_synth(probe, tx, pulse, t_pos, t_amp, rf, pos_static=sc.tissue_static, accumulate=False)
    fq.rf_synth(probe, tx, pulse, b_pos, b_amp, rf, pos_static=False, accumulate=True)
    das_ws = torch.empty(fq.das_workspace_size(probe, tx, F, T), dtype=torch.uint8, device=dev)
    iq = torch.empty((F, NV), dtype=torch.complex64, device=dev)
    fq.das_demodulate(probe, tx, rf, das_ws)
    fq.das_delay_sum(probe, tx, grid, T, das_ws, iq, fq.INTERP_LINEAR)
    del rf, das_ws
    torch.cuda.empty_cache()
    wpath = os.path.join(ROOT, 'paper_2509_05464_amd', 'weights', 'lcf_c4.npz')
    filt = LearnedFilter.load(wpath, dev) if os.path.exists(wpath) else LearnedFilter(lcf_init_weights(0), dev)
    gws = torch.empty(fq.gram_workspace_size(NV, F, 0), dtype=torch.uint8, device=dev)
    sws = torch.empty(fq.svd_workspace_size(NV, F), dtype=torch.uint8, device=dev)
    G = torch.empty((F, F), dtype=torch.complex128, device=dev)
    sig = torch.empty(F, dtype=torch.float64, device=dev)
    k = torch.zeros(1, dtype=torch.int32, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    pd = torch.empty(NV, dtype=torch.float32, device=dev)
    paths = {
        'svd_fp32': lambda: (fq.casorati_gram(iq, G, gws, fq.GRAM_FP32),
                             fq.svd_clutter_filter(iq, G, sws, sig, k, cfg.cutoff, pd=pd, status=st)),
        'svd_split4_bf16': lambda: (fq.casorati_gram(iq, G, gws, fq.GRAM_SPLIT4_BF16),
                                    fq.svd_clutter_filter(iq, G, sws, sig, k, cfg.cutoff, pd=pd, status=st)),
        'learned': lambda: filt.infer(iq, pd),
    }
    out = {'workload': cfg.name, 'ms_per_volume': {}}
    for name, fn in paths.items():
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out['ms_per_volume'][name] = e0.elapsed_time(e1) / max(1, args.steps)
    out['ms_per_volume_graph'] = {}
    for name in ('svd_fp32', 'svd_split4_bf16'):
        g = capture_graph(paths[name], torch)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        out['ms_per_volume_graph'][name] = e0.elapsed_time(e1) / max(1, args.steps)
    out['k_used'] = int(k.item())
    print(json.dumps(out))


def rf_only(cfg, args, fq, torch, dev):
    """RF synthesis of the workload's scene (tissue, then blood added), for profiler runs."""
    from fqscene import make_scene
    acq = cfg.acq
    sc = make_scene(cfg)
    probe = fq.make_probe(acq.nx_el, acq.ny_el, acq.pitch, acq.pitch, acq.fc, acq.fs, acq.c)
    tx = fq.make_tx(acq.tilts_rad())
    pulse = fq.make_pulse(2.0, 5.0, 1e-3)
    t_pos, t_amp = torch.from_numpy(sc.tissue_pos).to(dev), torch.from_numpy(sc.tissue_amp).to(dev)
    b_pos, b_amp = torch.from_numpy(sc.blood_pos).to(dev), torch.from_numpy(sc.blood_amp).to(dev)
    rf = torch.empty((acq.n_frames, acq.n_angles, acq.n_elem, acq.n_samples), dtype=torch.float32, device=dev)

    all_pos = None if sc.tissue_static else torch.cat([t_pos, b_pos], dim=1).contiguous()
    all_amp = None if sc.tissue_static else torch.cat([t_amp, b_amp]).contiguous()
    src = torch.zeros(1 << 31, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)                      # calibration copy: 2 GiB read + 2 GiB written
    del src, dst

    def run():
        if sc.tissue_static:
            fq.rf_synth(probe, tx, pulse, t_pos, t_amp, rf, pos_static=True, accumulate=False)
            fq.rf_synth(probe, tx, pulse, b_pos, b_amp, rf, pos_static=False, accumulate=True)
        else:
            fq.rf_synth(probe, tx, pulse, all_pos, all_amp, rf, pos_static=False, accumulate=False)

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    n_scat = sc.tissue_amp.size + sc.blood_amp.size
    n_rec = n_scat * acq.n_elem * acq.n_angles * acq.n_frames
    w = rf_work(acq, n_scat)
    print(json.dumps({'kernel': w['kernel'], 'workload': cfg.name, 'ms_per_step': ms,
                      'records_per_s': n_rec / (ms / 1e3),
                      'pulse_samples_per_s_equivalent': rf_taps(acq, n_scat) / (ms / 1e3),
                      'tflops': w['flop'] / (ms / 1e3) / 1e12}))


def fd_only(cfg, args, fq, torch, dev):
    """Frequency-domain RF synthesis of the workload's scene (element 0.27 mm, 2 x 2
    sub-elements, 0.5 dB/(cm MHz)), frame by frame: per frame the transmit field and the
    echo are contractions over scatterer x sub-element x frequency x transmit."""
    from fqscene import make_scene
    acq = cfg.acq
    sc = make_scene(cfg)
    frames = acq.n_frames if args.fd_frames is None else args.fd_frames
    probe = fq.make_probe(acq.nx_el, acq.ny_el, acq.pitch, acq.pitch, acq.fc, acq.fs, acq.c)
    tx = fq.make_tx(acq.tilts_rad())
    pulse = fq.make_pulse(2.0, 5.0, 1e-3)
    fdp = fq.make_fd_params((0.9 * acq.pitch, 0.9 * acq.pitch), (2, 2), 0.5, 1e-7)
    t_pos = torch.from_numpy(np.ascontiguousarray(sc.tissue_pos[:frames] if not sc.tissue_static
                                                  else sc.tissue_pos)).to(dev)
    b_pos = torch.from_numpy(np.ascontiguousarray(sc.blood_pos[:frames])).to(dev)
    t_amp = torch.from_numpy(sc.tissue_amp).to(dev)
    b_amp = torch.from_numpy(sc.blood_amp).to(dev)
    if not sc.tissue_static:
        t_pos = torch.cat([t_pos, b_pos], dim=1).contiguous()
        t_amp = torch.cat([t_amp, b_amp]).contiguous()
    n_all = t_amp.numel()
    ws = torch.empty(fq.fd_workspace_size(probe, tx, pulse, fdp, acq.n_samples, n_all), dtype=torch.uint8, device=dev)
    rf = torch.empty((frames, acq.n_angles, acq.n_elem, acq.n_samples), dtype=torch.float32, device=dev)

    def run():
        fq.fd_synth(probe, tx, pulse, fdp, t_pos, t_amp, rf, ws, pos_static=sc.tissue_static, accumulate=False)
        if sc.tissue_static:
            fq.fd_synth(probe, tx, pulse, fdp, b_pos, b_amp, rf, ws, pos_static=False, accumulate=True)

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    # frequency band of the model (as the library selects it)
    sig = 2.0 / (2.0 * np.sqrt(2.0 * np.log(2.0)) * acq.fc)
    N = acq.n_samples + 2 * int(np.ceil(6.0 * sig * acq.fs))
    f = np.arange(N // 2 + 1) * acq.fs / N
    a2 = 2 * np.pi ** 2 * sig ** 2
    S = np.exp(-a2 * (f - acq.fc) ** 2) + np.exp(-a2 * (f + acq.fc) ** 2)
    K = int((S >= 1e-7 * S.max()).sum())
    scat_frames = (sc.tissue_amp.size if sc.tissue_static else 0) + \
        (sc.blood_amp.size * frames if sc.tissue_static else n_all * frames)
    units = scat_frames * acq.n_elem * K * acq.n_angles          # scatterer x element x frequency x transmit
    flop = 16.0 * units                                            # two complex multiply-adds (field, echo)
    print(json.dumps({'kernel': 'fd_synth', 'workload': cfg.name, 'frames': frames, 'frequency_samples': K,
                      'sub_elements': 4, 'ms': ms, 'ms_per_frame': ms / frames,
                      'gunits_per_s': units / (ms / 1e3) / 1e9,
                      'contraction_tflops': flop / (ms / 1e3) / 1e12}))


def roof_only(fq, torch, dev):
    """On-chip ceilings measured by the library's probes: LDS read bandwidth and FP32 FMA rate."""
    res = {}
    for name, which, iters, per_thread in (('lds_read', fq.PROBE_LDS_READ, 4000, 128.0),
                                           ('fp32_fma', fq.PROBE_FP32_FMA, 400, 256.0)):
        out = torch.empty(256 * 2048, dtype=torch.float32, device=dev)
        fq.roof_probe(which, out, 10)
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fq.roof_probe(which, out, iters)
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b) / 1e3)
        t = float(np.median(ts))
        work = out.numel() * per_thread * iters          # bytes (LDS) or FLOP (FMA)
        res[name] = {'s': t, 'per_s': work / t, 'per_cu_clock': work / t / (256 * 2.4e9)}
    res['lds_read']['unit'] = 'bytes'
    res['fp32_fma']['unit'] = 'FLOP'
    print(json.dumps({'probe': 'roof', **res}))


def workload_run(cfg, steps, warmup, args, fq, torch, dev, filt, train, full=True, keep_sample=0) -> dict:
    """Warm-up and timed steps of the whole path on one workload, then (untimed) each filter
    path alone, the spatial-similarity cutoff, the display, and the errors against the
    blood-only ground truth with the filters compared at matched error."""
    from fqscene import make_scene
    acq = cfg.acq
    F, A, E, T, NV = acq.n_frames, acq.n_angles, acq.n_elem, acq.n_samples, acq.n_vox
    _log(f'[bench] scene {cfg.name}')
    sc = make_scene(cfg)
    probe = fq.make_probe(acq.nx_el, acq.ny_el, acq.pitch, acq.pitch, acq.fc, acq.fs, acq.c)
    tx = fq.make_tx(acq.tilts_rad())
    grid = fq.make_grid(acq.nx, acq.ny, acq.nz, acq.x0, acq.y0, acq.z0, acq.dx, acq.dy, acq.dz)
    pulse = fq.make_pulse(2.0, 5.0, 1e-3)

    t_pos = torch.from_numpy(sc.tissue_pos).to(dev)
    t_amp = torch.from_numpy(sc.tissue_amp).to(dev)
    b_pos = torch.from_numpy(sc.blood_pos).to(dev)
    b_amp = torch.from_numpy(sc.blood_amp).to(dev)
    t_static = sc.tissue_static
    # moving tissue and blood share the frame axis: one synthesis call over both
    all_pos = None if t_static else torch.cat([t_pos, b_pos], dim=1).contiguous()
    all_amp = None if t_static else torch.cat([t_amp, b_amp]).contiguous()

    rf = torch.empty((F, A, E, T), dtype=torch.float32, device=dev)
    das_ws = torch.empty(fq.das_workspace_size(probe, tx, F, T), dtype=torch.uint8, device=dev)
    iq = torch.empty((F, NV), dtype=torch.complex64, device=dev)
    gws = torch.empty(max(fq.gram_workspace_size(NV, F, m) for m in (0, 1, 3)), dtype=torch.uint8, device=dev)
    G = torch.empty((F, F), dtype=torch.complex128, device=dev)
    G2 = torch.empty((F, F), dtype=torch.complex128, device=dev)
    sws = torch.empty(fq.svd_workspace_size(NV, F), dtype=torch.uint8, device=dev)
    sws2 = torch.empty_like(sws)
    sigma = torch.empty(F, dtype=torch.float64, device=dev)
    sigma2 = torch.empty_like(sigma)
    k1 = torch.zeros(1, dtype=torch.int32, device=dev)
    k2 = torch.zeros(1, dtype=torch.int32, device=dev)
    st1 = torch.zeros(1, dtype=torch.int32, device=dev)
    st2 = torch.zeros(1, dtype=torch.int32, device=dev)
    pd_svd = torch.empty(NV, dtype=torch.float32, device=dev)
    pd_split = torch.empty(NV, dtype=torch.float32, device=dev)
    pd_lcf = torch.empty(NV, dtype=torch.float32, device=dev)
    pd_out = torch.empty(NV, dtype=torch.float32, device=dev)
    fb_ws = torch.empty(fq.fallback_workspace_size(NV), dtype=torch.uint8, device=dev)
    fb_flag = torch.zeros(1, dtype=torch.int32, device=dev)
    fb_d = torch.zeros(1, dtype=torch.float32, device=dev)

    stages = ['rf_synth', 'rf2iq', 'das', 'gram_fp32', 'svd_fp32', 'gram_split_bf16', 'svd_split_bf16',
              'lcf_infer', 'fallback', 'lcf_train_step']
    ev_b = {n: torch.cuda.Event(enable_timing=True) for n in stages}
    ev_e = {n: torch.cuda.Event(enable_timing=True) for n in stages}
    # after the beamformer, the FP32 SVD filter, the split-BF16 SVD filter and the learned
    # filter only read the IQ: three streams of default priority
    s_main = torch.cuda.current_stream()
    side = (s_main,) * 3 if args.serial else tuple(torch.cuda.Stream() for _ in range(3))
    gws2 = torch.empty_like(gws)
    iq_ready, svd_done, split_done, lcf_done = (torch.cuda.Event() for _ in range(4))

    def stage(name, record, fn):
        if record:
            ev_b[name].record()
        fn()
        if record:
            ev_e[name].record()

    def synth():
        if t_static:
            fq.rf_synth(probe, tx, pulse, t_pos, t_amp, rf, pos_static=True, accumulate=False)
            fq.rf_synth(probe, tx, pulse, b_pos, b_amp, rf, pos_static=False, accumulate=True)
        else:
            fq.rf_synth(probe, tx, pulse, all_pos, all_amp, rf, pos_static=False, accumulate=False)

    def step(record: bool):
        stage('rf_synth', record, synth)
        stage('rf2iq', record, lambda: fq.das_demodulate(probe, tx, rf, das_ws))
        stage('das', record, lambda: fq.das_delay_sum(probe, tx, grid, T, das_ws, iq, fq.INTERP_LINEAR))
        iq_ready.record()
        with torch.cuda.stream(side[0]):
            side[0].wait_event(iq_ready)
            stage('gram_fp32', record, lambda: fq.casorati_gram(iq, G, gws, fq.GRAM_FP32))
            stage('svd_fp32', record, lambda: fq.svd_clutter_filter(iq, G, sws, sigma, k1, cfg.cutoff, pd=pd_svd,
                                                                     status=st1))
            svd_done.record()
        with torch.cuda.stream(side[1]):
            side[1].wait_event(iq_ready)
            stage('gram_split_bf16', record, lambda: fq.casorati_gram(iq, G2, gws2, fq.GRAM_SPLIT4_BF16))
            stage('svd_split_bf16', record, lambda: fq.svd_clutter_filter(iq, G2, sws2, sigma2, k2, cfg.cutoff,
                                                                           pd=pd_split, status=st2))
            split_done.record()
        with torch.cuda.stream(side[2]):
            side[2].wait_event(iq_ready)
            stage('lcf_infer', record, lambda: filt.infer(iq, pd_lcf))
            side[2].wait_event(svd_done)
            stage('fallback', record, lambda: fq.lcf_fallback(pd_lcf, pd_svd, pd_out, fb_flag, fb_d, fb_ws, -10.0))
            stage('lcf_train_step', record, train)
            lcf_done.record()
        for e in (svd_done, split_done, lcf_done):
            s_main.wait_event(e)

    # the in-step training updates the network; the PD paths and errors below are taken on
    # the weights as loaded
    saved = [t.clone() for t in (filt.w, filt.wb, filt.m, filt.v)]
    saved_step = filt.step
    _log(f'[bench] {cfg.name}: warmup')
    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    _log(f'[bench] {cfg.name}: timed')
    acc = np.zeros(len(stages))
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
        torch.cuda.synchronize()   # per-step sync so every event pair is complete; counted in the step time
        acc += np.array([ev_b[n].elapsed_time(ev_e[n]) for n in stages])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for t, v in zip((filt.w, filt.wb, filt.m, filt.v), saved):
        t.copy_(v)
    filt.step = saved_step
    ms_step = wall / steps * 1e3
    stage_ms = {s: float(v / steps) for s, v in zip(stages, acc)}
    units = acq.das_units()
    stage_ms_das = stage_ms['das']
    t_das = stage_ms_das / 1e3
    achieved = DAS_FLOP_PER_UNIT * units / t_das / 1e12
    stage_ms_rf = stage_ms['rf_synth']
    rf_w = rf_work(acq, sc.tissue_amp.size + sc.blood_amp.size)
    rf_achieved = rf_w['flop'] / (stage_ms_rf / 1e3) / 1e12

    out = {
        'metric': 'DAS Gvoxel*element*angle/s (whole step: RF synthesis, DAS, SVD and learned clutter filters, PD)',
        'value': units / (ms_step / 1e3) / 1e9,
        'unit': 'Gvoxel*element*angle/s',
        'n_gpus': 1,
        'steps': steps,
        'warmup': warmup,
        'ms_per_step': ms_step,
        'higher_is_better': True,
        'scaling': 'weak',
        'vs_baseline': None,
        'dtype': 'f32',
        'data': 'synthetic',
        'config': {
            'workload': (f'{cfg.name}: {acq.nx_el}x{acq.ny_el} array ({E} elements), {A} plane waves, '
                         f'{acq.nx}x{acq.ny}x{acq.nz} voxels, {F} frames at {acq.prf:g} Hz, {T} RF samples, '
                         f'{cfg.scene.n_tissue} tissue + {cfg.scene.n_blood} blood scatterers, '
                         f'cutoff {"knee" if cfg.cutoff < 0 else cfg.cutoff}'),
            'das_units_per_step': units,
        },
        'roofline': None,   # the dominant kernel's entry of `rooflines`, set below
        'rooflines': {
            'das_kernel': {
                'bound': 'alu',
                'work': 'delay-and-sum, linear interpolation: 16 FLOP per voxel*element*angle*frame',
                'achieved': achieved,
                'peak': PEAK_FP32_VECTOR_TFLOPS,
                'unit': 'TFLOP/s',
                'frac': achieved / PEAK_FP32_VECTOR_TFLOPS,
                'measured_fma_peak': measured_fma_tflops(),
                'traffic': measured_traffic(f'das_kernel_{cfg.name}_hbm_traffic.md'),
                'traffic_unit': 'bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, copy-calibrated)',
                'stage_ms': stage_ms_das,
            },
            'rf_spread_kernel': {
                'bound': 'alu',
                'work': rf_w['work'],
                'achieved': rf_achieved,
                'peak': PEAK_FP32_VECTOR_TFLOPS,
                'unit': 'TFLOP/s',
                'frac': rf_achieved / PEAK_FP32_VECTOR_TFLOPS,
                'measured_fma_peak': measured_fma_tflops(),
                'traffic': measured_traffic(f'rf_spread_{cfg.name}_hbm_traffic.md'),
                'traffic_unit': 'bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, copy-calibrated)',
                'stage_ms': stage_ms_rf,
                'pulse_samples_per_s_equivalent': rf_taps(acq, sc.tissue_amp.size + sc.blood_amp.size) /
                                                  (stage_ms_rf / 1e3),
                'valu_issue_per_cu_clock': (lambda kv: float(kv['valu_issue_per_cu_clock']) if kv else None)(
                    profile_values(f'rf_spread_{cfg.name}_sq_counters.md')),
            },
        },
        'stage_ms': stage_ms,
        'filter_streams': 1 if args.serial else 3,
        'das_gunits_per_s': units / t_das / 1e9,
        'pd_volumes_per_s': None,   # each path timed alone, set below
        'pd_volumes_per_s_in_step': {
            'svd_fp32': 1e3 / (stage_ms['gram_fp32'] + stage_ms['svd_fp32']),
            'svd_split4_bf16': 1e3 / (stage_ms['gram_split_bf16'] + stage_ms['svd_split_bf16']),
            'learned': 1e3 / stage_ms['lcf_infer'],
        },
        'learned_fallback': {'flag': int(fb_flag.item()), 'discrepancy_db_vs_svd': float(fb_d.item())},
        'k_used': {'svd_fp32': int(k1.item()), 'svd_split4_bf16': int(k2.item())},
        'eig_status': {'svd_fp32': int(st1.item()), 'svd_split4_bf16': int(st2.item())},
    }
    dominant = 'rf_spread_kernel' if stage_ms_rf > stage_ms_das else 'das_kernel'
    out['roofline'] = dict(out['rooflines'][dominant], kernel=dominant)
    if keep_sample:
        # every stride-th voxel of the ensemble, for the oracle's precision check (host copy)
        stride = max(1, NV // keep_sample)
        out['_iq_sample'] = iq[:, ::stride][:, :keep_sample].contiguous().cpu()

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    def graph_ms(fn, reps=5):
        return timed(capture_graph(fn, torch).replay, reps)

    # PD volumes/s of each clutter-filter path on its own (one stream, nothing beside it):
    # ensemble IQ in HBM -> PD volume; in the step the three paths share the GPU
    _log(f'[bench] {cfg.name}: PD paths alone')

    def svd_path(mode, cutoff, Gx, wsx, sig, kx, pdx, stx):
        return lambda: (fq.casorati_gram(iq, Gx, gws, mode),
                        fq.svd_clutter_filter(iq, Gx, wsx, sig, kx, cutoff, pd=pdx, status=stx))

    alone_ms = {
        'svd_fp32': timed(svd_path(fq.GRAM_FP32, cfg.cutoff, G, sws, sigma, k1, pd_svd, st1)),
        'svd_split4_bf16': timed(svd_path(fq.GRAM_SPLIT4_BF16, cfg.cutoff, G2, sws2, sigma2, k2, pd_split, st2)),
        'learned': timed(lambda: filt.infer(iq, pd_lcf)),
    }
    out['pd_volumes_per_s'] = {k: 1e3 / v for k, v in alone_ms.items()}
    out['pd_volumes_per_s_graph'] = {
        'svd_fp32': 1e3 / graph_ms(svd_path(fq.GRAM_FP32, cfg.cutoff, G, sws, sigma, k1, pd_svd, st1)),
        'svd_split4_bf16': 1e3 / graph_ms(svd_path(fq.GRAM_SPLIT4_BF16, cfg.cutoff, G2, sws2, sigma2, k2, pd_split,
                                                   st2)),
    }

    # a stream of ensembles: the same SVD path on two streams, volumes alternating, so one
    # volume's single-workgroup eigensolver runs beside the next volume's Gram
    def two_in_flight(mode, reps=8):
        sets = [(G, gws, sws, sigma, k1, st1, pd_svd), (G2, gws2, sws2, sigma2, k2, st2, pd_split)]
        strs = (torch.cuda.Stream(), torch.cuda.Stream())

        def run(n):
            for v in range(n):
                Gx, gx, sx, sg, kx, stx, pdx = sets[v % 2]
                with torch.cuda.stream(strs[v % 2]):
                    fq.casorati_gram(iq, Gx, gx, mode)
                    fq.svd_clutter_filter(iq, Gx, sx, sg, kx, cfg.cutoff, pd=pdx, status=stx)

        run(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(reps)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    out['pd_volumes_per_s_two_in_flight'] = {'svd_fp32': 1e3 / two_in_flight(fq.GRAM_FP32),
                                              'svd_split4_bf16': 1e3 / two_in_flight(fq.GRAM_SPLIT4_BF16)}

    # a stream of ensembles, pipelined: the eigendecomposition and cutoff of volume v on a
    # stream held to 8 CUs (one per XCD) while the other 248 form volume v+1's Gram and then
    # volume v's projection and PD (svd_filter_apply); the eigensolver's single workgroup needs
    # a whole CU, which a full-GPU Gram otherwise keeps taken
    def pipelined(mode, streams, reps=8):
        sets = [(G, gws, sws, sigma, k1, st1, pd_svd), (G2, gws2, sws2, sigma2, k2, st2, pd_split)]
        M, E = streams

        def run(n):
            done = [None] * n
            for v in range(n + 1):
                if v < n:
                    Gx, gx, sx, sg, kx, stx, pdx = sets[v % 2]
                    g = torch.cuda.Event()
                    with torch.cuda.stream(M):
                        fq.casorati_gram(iq, Gx, gx, mode)
                        g.record(M)
                    with torch.cuda.stream(E):
                        E.wait_event(g)
                        fq.svd_clutter_filter(iq, Gx, sx, sg, kx, cfg.cutoff, status=stx)
                        done[v] = torch.cuda.Event()
                        done[v].record(E)
                if v >= 1:
                    Gx, gx, sx, sg, kx, stx, pdx = sets[(v - 1) % 2]
                    with torch.cuda.stream(M):
                        M.wait_event(done[v - 1])
                        fq.svd_filter_apply(iq, sx, kx, pd=pdx)

        run(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(reps)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    # (every kernel of the path has run on the default stream above before the masked streams
    # are made; a failure here is reported in the line instead of ending the run)
    pipe_streams, masked, release = cu_split_streams(torch, 8)
    try:
        out['pd_volumes_per_s_pipelined'] = {'svd_fp32': 1e3 / pipelined(fq.GRAM_FP32, pipe_streams),
                                             'svd_split4_bf16': 1e3 / pipelined(fq.GRAM_SPLIT4_BF16, pipe_streams),
                                             'eig_cus': 8 if masked else None, 'cu_mask': masked}
    except fq.FqError as e:
        torch.cuda.synchronize()
        out['pd_volumes_per_s_pipelined'] = {'error': str(e), 'cu_mask': masked}
    release()
    out['pd_volumes_per_s_note'] = ('each path timed alone on one stream (mean of 5 after a warm-up): Gram + '
                                    'eigendecomposition + cutoff + fused projection and PD, or learned inference '
                                    'with PD; pd_volumes_per_s_two_in_flight: a stream of ensembles, the SVD path '
                                    'on two streams with volumes alternating (8 volumes, wall clock), one '
                                    "volume's eigensolver beside the next one's Gram; pd_volumes_per_s_pipelined: "
                                    'the same stream of ensembles with the eigendecomposition on a stream held to 8 '
                                    'CUs and Gram + projection/PD (svd_filter_apply) on the other 248 (8 volumes, '
                                    'wall clock); pd_volumes_per_s_graph: the '
                                    'SVD path captured once as a HIP graph and replayed (mean of 5); '
                                    'pd_volumes_per_s_in_step: the same stages inside the step, beside the other '
                                    'two filters')
    fq.lcf_fallback(pd_lcf, pd_svd, pd_out, fb_flag, fb_d, fb_ws, -10.0)
    out['learned_fallback'] = {'flag': int(fb_flag.item()), 'discrepancy_db_vs_svd': float(fb_d.item())}

    if full:
        # spatial-similarity matrix of the leading modes and the clutter filter with the SSM
        # cutoff, on the step's IQ and FP32 Gram (outside the step: the workload's cutoff is
        # the knee)
        _log(f'[bench] {cfg.name}: spatial similarity')
        M = min(F, fq.FQ_SSM_MAX_MODES)
        lam_e = torch.empty(F, dtype=torch.float64, device=dev)
        vecs = torch.empty((F, F), dtype=torch.complex128, device=dev)
        st3 = torch.zeros(1, dtype=torch.int32, device=dev)
        fq.casorati_gram(iq, G, gws, fq.GRAM_FP32)
        fq.hermitian_eig(G, sws, lam_e, vecs, st3)
        ssm_ws = torch.empty(fq.ssm_workspace_size(NV, F), dtype=torch.uint8, device=dev)
        C_ssm = torch.empty((M, M), dtype=torch.float64, device=dev)
        k_ssm = torch.zeros(1, dtype=torch.int32, device=dev)
        k3 = torch.zeros(1, dtype=torch.int32, device=dev)
        pd_ssm = torch.empty(NV, dtype=torch.float32, device=dev)
        sigma3 = torch.empty_like(sigma)
        ssm_ms = timed(lambda: fq.spatial_similarity(iq, vecs, M, ssm_ws, C_ssm, k_ssm))
        svd_ssm_ms = timed(lambda: fq.svd_clutter_filter(iq, G, sws, sigma3, k3, fq.CUTOFF_SSM, pd=pd_ssm,
                                                         status=st3))
        # MFMA work of one SSM pass: U = S V over the 64-mode tile (8 FLOP per complex
        # multiply-add) and the 64 x 64 Gram of |U| (2 FLOP per multiply-add)
        ssm_flop = 8.0 * NV * F * fq.FQ_SSM_MAX_MODES + 2.0 * NV * fq.FQ_SSM_MAX_MODES ** 2
        out['ssm'] = {
            'n_modes': M,
            'k_tissue': int(k_ssm.item()),
            'k_used_by_filter': int(k3.item()),
            'ms': ssm_ms,
            'achieved': ssm_flop / (ssm_ms / 1e3) / 1e12,
            'peak': PEAK_FP32_MFMA_TFLOPS,
            'unit': 'TFLOP/s',
            'frac': ssm_flop / (ssm_ms / 1e3) / 1e12 / PEAK_FP32_MFMA_TFLOPS,
            'svd_filter_with_ssm_cutoff_ms': svd_ssm_ms,
            'eig_status': int(st3.item()),
        }
        del vecs, ssm_ws

        # display: the PD volume over 60 dB and its three maximum-intensity projections
        disp_ws = torch.empty(fq.display_workspace_size(NV), dtype=torch.uint8, device=dev)
        pd_db = torch.empty((acq.nz, acq.ny, acq.nx), dtype=torch.float32, device=dev)
        mips = [torch.empty(shp, dtype=torch.float32, device=dev)
                for shp in ((acq.ny, acq.nx), (acq.nz, acq.nx), (acq.nz, acq.ny))]

        def show():
            fq.display_db(pd_svd.view(acq.nz, acq.ny, acq.nx), 60.0, disp_ws, pd_db)
            for plane, m in zip((fq.MIP_XY, fq.MIP_XZ, fq.MIP_YZ), mips):
                fq.mip(pd_db, plane, m)

        disp_ms = timed(show, reps=20)
        # algorithmic bytes: PD read twice (reference, then dB) and dB written, then three reads
        # of the dB volume for the projections
        disp_bytes = 4.0 * NV * (2 + 1 + 3)
        out['display'] = {'ms': disp_ms, 'gb_per_s': disp_bytes / (disp_ms / 1e3) / 1e9,
                          'what': 'PD volume over 60 dB + MIPs onto x-y, x-z, y-z'}
        del disp_ws, pd_db, mips

    if not args.no_truth:
        # untimed: ground-truth blood PD (DAS of blood-only RF) and each path's error
        _log(f'[bench] {cfg.name}: ground-truth pass and matched-error comparison')
        fq.rf_synth(probe, tx, pulse, b_pos, b_amp, rf, pos_static=False, accumulate=False)
        iq_b = torch.empty_like(iq)
        fq.das_beamform(probe, tx, grid, rf, iq_b, das_ws, fq.INTERP_LINEAR)
        pd_true = torch.empty(NV, dtype=torch.float32, device=dev)
        fq.power_doppler(iq_b, pd_true)
        del iq_b
        ref = pd_true.double()

        def err_db(p):
            return float(10 * torch.log10(((p.double() - ref) ** 2).sum() / (ref ** 2).sum()).item())

        def rel(p):
            return float((torch.linalg.norm(p.double() - pd_svd.double()) / torch.linalg.norm(pd_svd.double())).item())

        # the knee paths as the step ran them
        fq.casorati_gram(iq, G, gws, fq.GRAM_FP32)
        fq.svd_clutter_filter(iq, G, sws, sigma, k1, cfg.cutoff, pd=pd_svd)
        fq.casorati_gram(iq, G2, gws, fq.GRAM_SPLIT4_BF16)
        fq.svd_clutter_filter(iq, G2, sws2, sigma2, k2, cfg.cutoff, pd=pd_split)
        filt.infer(iq, pd_lcf)
        fq.lcf_fallback(pd_lcf, pd_svd, pd_out, fb_flag, fb_d, fb_ws, -10.0)
        errs = {'svd_fp32': err_db(pd_svd), 'svd_split4_bf16': err_db(pd_split),
                'learned': err_db(pd_lcf), 'learned_with_fallback': err_db(pd_out)}
        if full:
            errs['svd_fp32_ssm_cutoff'] = err_db(pd_ssm)
        # three-product split-BF16 Gram at the FP32 path's K (its own spectrum tail is biased)
        G3 = torch.empty_like(G)
        fq.casorati_gram(iq, G3, gws, fq.GRAM_SPLIT_BF16)
        pd_split3 = torch.empty_like(pd_svd)
        k3b = torch.zeros_like(k1)
        fq.svd_clutter_filter(iq, G3, sws2, sigma2, k3b, int(k1.item()), pd=pd_split3)
        errs['svd_split3_bf16_at_fp32_k'] = err_db(pd_split3)
        out['pd_error_db_vs_blood_truth'] = errs
        out['pd_rel_l2_vs_fp32_svd'] = {'svd_split4_bf16': rel(pd_split), 'svd_split3_bf16_at_fp32_k': rel(pd_split3)}

        # matched error: the SVD filter's error for every fixed rank, the rank at which it
        # reaches the learned filter's error, and each path's throughput there
        pd_k = torch.empty_like(pd_svd)
        kk = torch.zeros_like(k1)
        kmax = min(48, F // 2 - 1)
        by_k = {}
        for K in range(1, kmax + 1):
            fq.svd_clutter_filter(iq, G, sws, sigma, kk, K, pd=pd_k)
            by_k[K] = err_db(pd_k)
        k_best = min(by_k, key=by_k.get)
        e_l = errs['learned']
        reach = [K for K in sorted(by_k) if by_k[K] <= e_l]
        k_match = reach[0] if reach else k_best
        ms_match = {
            'svd_fp32': timed(svd_path(fq.GRAM_FP32, k_match, G, sws, sigma, kk, pd_k, st1)),
            'svd_split4_bf16': timed(svd_path(fq.GRAM_SPLIT4_BF16, k_match, G2, sws2, sigma2, kk, pd_k, st2)),
            'learned': alone_ms['learned'],
        }
        out['matched_error'] = {
            'svd_fp32_error_db_by_k': {str(K): v for K, v in by_k.items()},
            'svd_best': {'k': k_best, 'error_db': by_k[k_best]},
            'learned_error_db': e_l,
            'svd_k_at_learned_error': k_match if reach else None,
            'error_db_at_match': {'svd_fp32': by_k[k_match], 'learned': e_l},
            'pd_volumes_per_s_at_match': {k: 1e3 / v for k, v in ms_match.items()},
            'note': ('E_dB = 10 log10(sum (PD - PD_true)^2 / sum PD_true^2) over the grid, PD_true the power Doppler '
                     'of the blood-only ensemble; the SVD filter at the smallest fixed rank whose error is at or '
                     'below the learned filter\'s (its best rank if none is), each path timed alone'),
        }
    return out


def p7_das_timing(fq, torch, dev) -> dict:
    """The paper's DAS timing shape (Section 2.4.1): 32x32 elements at 7.81 MHz, 5 tilted
    plane waves, a 2 cm cube at 0.2 mm (100^3 voxels), for 1, 3, 10 and 30 frames: rf2iq +
    delay-and-sum of the whole ensemble (seeded random RF resident in HBM)."""
    from fqscene import get_config
    acq = get_config('p7').acq
    probe = fq.make_probe(acq.nx_el, acq.ny_el, acq.pitch, acq.pitch, acq.fc, acq.fs, acq.c)
    tx = fq.make_tx(acq.tilts_rad())
    grid = fq.make_grid(acq.nx, acq.ny, acq.nz, acq.x0, acq.y0, acq.z0, acq.dx, acq.dy, acq.dz)
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    res = {}
    for F in (1, 3, 10, 30):
        rf = torch.randn((F, acq.n_angles, acq.n_elem, acq.n_samples), device=dev, generator=gen)
        ws = torch.empty(fq.das_workspace_size(probe, tx, F, acq.n_samples), dtype=torch.uint8, device=dev)
        iq = torch.empty((F, acq.n_vox), dtype=torch.complex64, device=dev)
        fq.das_beamform(probe, tx, grid, rf, iq, ws, fq.INTERP_LINEAR)
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fq.das_beamform(probe, tx, grid, rf, iq, ws, fq.INTERP_LINEAR)
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        ms = float(np.median(ts))
        units = acq.n_vox * acq.n_elem * acq.n_angles * F
        res[str(F)] = {'ms': ms, 'ms_per_frame': ms / F, 'gunits_per_s': units / (ms / 1e3) / 1e9}
    return {'what': ('rf2iq + delay-and-sum, 32x32 elements, 5 plane waves, 100^3 voxels at 0.2 mm, median of 5; '
                     'the shape of the paper\'s DAS timing experiment (Section 2.4.1)'), 'frames': res}


def precision_vs_oracle(sub, fq, torch, dev) -> dict:
    """Error of the precision variants against the FP64 oracle, stated per result, on a
    voxel sample of the workload's own IQ (complex64 [N_t][n_sub] on the device): the Gram,
    the leading eigenvalue, the tissue projector at the oracle's knee rank, and the power
    Doppler."""
    from oracle import clutter
    nt, n_sub = sub.shape
    x = sub.cpu().numpy()
    Go = clutter.gram(x)
    lam_o, V_o = clutter.eig_desc(Go)
    K = clutter.knee_cutoff(lam_o)
    pd_o = clutter.power_doppler(clutter.filter_iq(x, V_o, K))
    gws = torch.empty(max(fq.gram_workspace_size(n_sub, nt, m) for m in (0, 1, 3)), dtype=torch.uint8, device=dev)
    sws = torch.empty(fq.svd_workspace_size(n_sub, nt), dtype=torch.uint8, device=dev)
    res = {'voxels': n_sub, 'k': K}
    for name, mode in (('fp32', fq.GRAM_FP32), ('split3_bf16', fq.GRAM_SPLIT_BF16),
                       ('split4_bf16', fq.GRAM_SPLIT4_BF16), ('bf16_control', fq.GRAM_BF16)):
        G = torch.empty((nt, nt), dtype=torch.complex128, device=dev)
        fq.casorati_gram(sub, G, gws, mode)
        lam = torch.empty(nt, dtype=torch.float64, device=dev)
        vecs = torch.empty((nt, nt), dtype=torch.complex128, device=dev)
        st = torch.zeros(1, dtype=torch.int32, device=dev)
        fq.hermitian_eig(G, sws, lam, vecs, st)
        sig = torch.empty(nt, dtype=torch.float64, device=dev)
        k = torch.zeros(1, dtype=torch.int32, device=dev)
        pd = torch.empty(n_sub, dtype=torch.float32, device=dev)
        fq.svd_clutter_filter(sub, G, sws, sig, k, K, pd=pd)
        Gh, lh, Vh, pdh = G.cpu().numpy(), lam.cpu().numpy(), vecs.cpu().numpy(), pd.cpu().numpy()
        res[name] = {
            'gram_rel_l2': float(np.linalg.norm(Gh - Go) / np.linalg.norm(Go)),
            'lambda1_rel': float(abs(lh[0] - lam_o[0]) / lam_o[0]),
            'projector_max_abs': float(np.abs(clutter.projector(Vh, K) - clutter.projector(V_o, K)).max()),
            'pd_rel_l2': float(np.linalg.norm(pdh - pd_o) / np.linalg.norm(pd_o)),
        }
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=3)
    ap.add_argument('--warmup', type=int, default=1)
    ap.add_argument('--config', default='c5')
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--no-extras', action='store_true',
                    help='skip the throughput-workload figures and the P7 DAS timing')
    ap.add_argument('--serial', action='store_true', help='run the filters after the beamformer on one stream')
    ap.add_argument('--no-truth', action='store_true', help='skip the untimed ground-truth error pass')
    ap.add_argument('--fd-frames', type=int, default=None, help='frames of the frequency-domain run (--only fd)')
    ap.add_argument('--only', choices=['das', 'rf', 'fd', 'roof', 'filters'], default=None,
                    help='das: the delay-and-sum kernel alone on the workload geometry (seeded random RF), '
                         'plus a 2 GiB device copy that calibrates byte counters; rf: RF synthesis of the '
                         'workload scene alone; fd: frequency-domain RF synthesis of the workload scene; '
                         'roof: the LDS-bandwidth and FP32-FMA probes; filters: the three power-Doppler '
                         'paths on a seeded random ensemble of the workload shape; for profiler runs')
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({'error': 'the path runs on one GPU: --gpus must be 1 (sharding across GPUs is designed, '
                                   'not implemented)'}))
        sys.exit(2)

    import torch
    import paper_2509_05464_amd as fq
    from fqscene import get_config

    cfg = get_config(args.config)
    dev = torch.device('cuda:0')
    torch.cuda.set_device(dev)
    if args.only == 'das':
        return das_only(cfg, args, fq, torch, dev)
    if args.only == 'rf':
        return rf_only(cfg, args, fq, torch, dev)
    if args.only == 'fd':
        return fd_only(cfg, args, fq, torch, dev)
    if args.only == 'roof':
        return roof_only(fq, torch, dev)
    if args.only == 'filters':
        return filters_only(cfg, args, fq, torch, dev)

    # learned filter: trained weights when present, and a small training set (untimed)
    from paper_2509_05464_amd.learned import LearnedFilter
    from paper_2509_05464_amd.train_lcf import make_pairs
    from fqscene import batch_indices, lcf_init_weights
    wpath = os.path.join(ROOT, 'paper_2509_05464_amd', 'weights', 'lcf_c4.npz')
    filt = LearnedFilter.load(wpath, dev) if os.path.exists(wpath) else LearnedFilter(lcf_init_weights(0), dev)
    _log('[bench] learned-filter training pairs')
    tr_cfg = get_config('c4_train')
    tr_mix, tr_blood = make_pairs(tr_cfg, [1000, 1001], dev)
    BATCH = 4096
    xb = torch.empty((tr_cfg.acq.n_frames, BATCH), dtype=torch.complex64, device=dev)
    yb = torch.empty_like(xb)
    idx_host = [torch.from_numpy(batch_indices(2 * tr_cfg.acq.n_vox, BATCH, 77 + i)).to(dev) for i in range(8)]
    step_no = [0]

    def train():
        idx = idx_host[step_no[0] % len(idx_host)]
        step_no[0] += 1
        fq.lcf_gather(tr_mix, idx, xb)
        fq.lcf_gather(tr_blood, idx, yb)
        filt.train_step(xb, yb)

    out = workload_run(cfg, args.steps, args.warmup, args, fq, torch, dev, filt, train, full=True,
                       keep_sample=0 if args.no_cpu_baseline else 1 << 16)
    sample = out.pop('_iq_sample', None)
    out['learned_fallback']['weights'] = os.path.basename(wpath) if os.path.exists(wpath) else 'untrained (seed 0)'
    torch.cuda.empty_cache()

    if not args.no_extras and cfg.name != 'c2':
        # the throughput workload (128^3 voxels, 200 frames) beside the headline: its own
        # whole-step rate, per-stage times, filter paths and errors
        c2 = workload_run(get_config('c2'), 3, 1, args, fq, torch, dev, filt, train, full=False)
        out['c2'] = {k: c2[k] for k in ('value', 'ms_per_step', 'config', 'rooflines', 'stage_ms', 'das_gunits_per_s',
                                       'pd_volumes_per_s', 'pd_volumes_per_s_two_in_flight', 'pd_volumes_per_s_pipelined',
                                       'pd_volumes_per_s_graph', 'pd_volumes_per_s_in_step',
                                       'learned_fallback', 'k_used',
                                       'eig_status', 'pd_error_db_vs_blood_truth', 'pd_rel_l2_vs_fp32_svd',
                                       'matched_error') if k in c2}
        out['c2']['steps'], out['c2']['warmup'] = 3, 1
        torch.cuda.empty_cache()
    if not args.no_extras:
        _log('[bench] P7 DAS timing')
        out['p7_das'] = p7_das_timing(fq, torch, dev)
        torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        _log('[bench] cpu baseline (oracle)')
        out['cpu_baseline'] = cpu_baseline(cfg)
        _log('[bench] precision variants against the FP64 oracle')
        out['precision_vs_fp64_oracle'] = precision_vs_oracle(sample.to(dev), fq, torch, dev)
    print(json.dumps(out))


if __name__ == '__main__':
    main()
