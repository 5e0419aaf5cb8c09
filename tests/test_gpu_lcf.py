"""GPU parity of the learned slow-time clutter filter (forward, gradients, Adam,
batch gather, SVD-fallback judge) against the FP64 oracle.

Tolerances (relative L2): against the oracle's BF16-rounding mode the GPU differs only
by FP32 accumulation order and the BF16 rounding decisions it flips (one BF16 ulp,
2^-8, on a few activations): forward 2e-3, gradient 5e-3; against the pure FP64
network the BF16 representation itself costs up to ~3e-2."""
import numpy as np
import pytest

from fqscene import lcf_init_weights
from helpers import dev, rel_l2
from oracle import bf16 as obf16
from oracle import lcf as olcf

pytestmark = pytest.mark.gpu


def _weights(seed):
    rng = np.random.default_rng(seed)
    w = lcf_init_weights(seed)
    w = (w + 0.05 * rng.standard_normal(w.size)).astype(np.float32)   # non-zero biases too
    return w, obf16.bf16_bits(w)


def _series(seed, n, T):
    rng = np.random.default_rng(seed)
    tt = np.arange(T)
    slow = np.exp(2j * np.pi * 0.01 * tt)[None, :] * (3 + rng.standard_normal((n, 1)))
    blood = 0.1 * (rng.standard_normal((n, T)) + 1j * rng.standard_normal((n, T)))
    mix = (slow + blood).astype(np.complex64)
    return mix, blood.astype(np.complex64)


def _gpu_forward(gpu, w, wb, x_tn, act=None):
    import torch
    nt, n = x_tn.shape
    y = torch.empty((nt, n), dtype=torch.complex64, device='cuda')
    pd = torch.empty(n, dtype=torch.float32, device='cuda')
    gpu.lcf_forward(dev(w), dev(wb.view(np.int16)), dev(x_tn), 1e-30, act, y, pd)
    return y.cpu().numpy(), pd.cpu().numpy()


@pytest.mark.parametrize('T,n', [(24, 37), (200, 64), (65, 5), (40, 11), (32, 3), (100, 6), (257, 9), (512, 7), (12, 8200)])
def test_forward_matches_oracle(gpu, T, n):
    w, wb = _weights(1)
    mix, _ = _series(2, n, T)
    y, pd = _gpu_forward(gpu, w, wb, np.ascontiguousarray(mix.T))
    y16 = olcf.blood_estimate(w.astype(np.float64), mix.T, bf16=True)
    y64 = olcf.blood_estimate(w.astype(np.float64), mix.T, bf16=False)
    e16, e64 = rel_l2(y, y16), rel_l2(y, y64)
    print('forward vs bf16 oracle', e16, 'vs fp64', e64)
    assert e16 < 2e-3
    assert e64 < 3e-2
    pd_o = np.mean(np.abs(y16) ** 2, axis=0)
    assert rel_l2(pd, pd_o) < 4e-3


@pytest.mark.parametrize('T,n', [(24, 300), (200, 96)])
def test_gradient_matches_oracle(gpu, T, n):
    import torch
    w, wb = _weights(3)
    mix, blood = _series(4, n, T)
    x = dev(np.ascontiguousarray(mix.T))
    tgt = dev(np.ascontiguousarray(blood.T))
    act = torch.empty(gpu.lcf_act_size(n, T), dtype=torch.uint8, device='cuda')
    y = torch.empty((T, n), dtype=torch.complex64, device='cuda')
    wt, wbt = dev(w), dev(wb.view(np.int16))
    gpu.lcf_forward(wt, wbt, x, 1e-30, act.view(torch.int16), y, None)
    grad = torch.empty(gpu.LCF_N_PARAM, dtype=torch.float32, device='cuda')
    loss = torch.empty(1, dtype=torch.float32, device='cuda')
    gpu.lcf_backward(wt, wbt, x, tgt, act.view(torch.int16), grad, loss, 1e-30)
    g = grad.cpu().numpy()
    xo, s = olcf.normalise(mix.astype(np.complex128))
    yt = np.stack([blood.real, blood.imag], axis=1) / s[:, None, None]
    l16, g16 = olcf.loss_and_grad(w.astype(np.float64), xo, yt, bf16=True)
    l64, g64 = olcf.loss_and_grad(w.astype(np.float64), xo, yt, bf16=False)
    print('grad vs bf16 oracle', rel_l2(g, g16), 'vs fp64', rel_l2(g, g64), 'loss', loss.item(), l16)
    assert abs(loss.item() / l16 - 1) < 2e-3
    assert rel_l2(g, g16) < 5e-3
    assert rel_l2(g, g64) < 5e-2
    # every parameter block is exercised (none silently zero)
    for name, shp in olcf.SHAPES:
        sl = olcf.unpack(np.arange(olcf.N_PARAM))[name].ravel().astype(int)
        assert np.linalg.norm(g[sl]) > 0, name
        assert rel_l2(g[sl], g16[sl]) < 2e-2, name


def test_backward_is_deterministic(gpu):
    import torch
    w, wb = _weights(5)
    mix, blood = _series(6, 200, 40)
    x, tgt = dev(np.ascontiguousarray(mix.T)), dev(np.ascontiguousarray(blood.T))
    wt, wbt = dev(w), dev(wb.view(np.int16))
    outs = []
    for _ in range(2):
        act = torch.empty(gpu.lcf_act_size(200, 40), dtype=torch.uint8, device='cuda')
        gpu.lcf_forward(wt, wbt, x, 1e-30, act.view(torch.int16), None, None)
        grad = torch.empty(gpu.LCF_N_PARAM, dtype=torch.float32, device='cuda')
        loss = torch.empty(1, dtype=torch.float32, device='cuda')
        gpu.lcf_backward(wt, wbt, x, tgt, act.view(torch.int16), grad, loss, 1e-30)
        outs.append(grad.cpu().numpy())
    np.testing.assert_array_equal(outs[0], outs[1])


def test_adam_matches_oracle(gpu):
    import torch
    rng = np.random.default_rng(7)
    w0 = rng.standard_normal(1000).astype(np.float32)
    w, m, v = dev(w0.copy()), dev(np.zeros(1000, np.float32)), dev(np.zeros(1000, np.float32))
    wb = torch.empty(1000, dtype=torch.int16, device='cuda')
    wo, mo, vo = w0.astype(np.float64), np.zeros(1000), np.zeros(1000)
    for step in range(1, 6):
        g = rng.standard_normal(1000).astype(np.float32)
        gpu.lcf_adam_step(w, wb, m, v, dev(g), step, lr=1e-2)
        wo, mo, vo = olcf.adam(wo, mo, vo, g.astype(np.float64), step, lr=1e-2)
    wg = w.cpu().numpy()
    assert np.abs(wg - wo).max() < 1e-5
    np.testing.assert_array_equal(wb.cpu().numpy().view(np.uint16), obf16.bf16_bits(wg))


def test_gather(gpu):
    rng = np.random.default_rng(8)
    src = (rng.standard_normal((3, 7, 50)) + 1j * rng.standard_normal((3, 7, 50))).astype(np.complex64)
    idx = rng.integers(0, 150, 33).astype(np.int64)
    import torch
    dst = torch.empty((7, 33), dtype=torch.complex64, device='cuda')
    gpu.lcf_gather(dev(src), dev(idx), dst)
    want = src.transpose(1, 0, 2).reshape(7, 150)[:, idx]
    np.testing.assert_array_equal(dst.cpu().numpy(), want)


@pytest.mark.parametrize('case', ['close', 'far', 'nan'])
def test_fallback_judge(gpu, case):
    import torch
    rng = np.random.default_rng(9)
    ps = rng.random(1000).astype(np.float32) + 0.1
    pl = ps * (1 + 0.01 * rng.standard_normal(1000)).astype(np.float32)
    if case == 'far':
        pl = pl + 3.0 * ps
    if case == 'nan':
        pl[17] = np.nan
    out = torch.empty(1000, dtype=torch.float32, device='cuda')
    flag = torch.zeros(1, dtype=torch.int32, device='cuda')
    d = torch.zeros(1, dtype=torch.float32, device='cuda')
    ws = torch.empty(gpu.fallback_workspace_size(1000), dtype=torch.uint8, device='cuda')
    gpu.lcf_fallback(dev(pl), dev(ps), out, flag, d, ws, tau_db=-10.0)
    want_d = 10 * np.log10(np.sum((pl.astype(np.float64) - ps) ** 2) / np.sum(ps.astype(np.float64) ** 2))
    if case == 'close':
        assert flag.item() == 0
        np.testing.assert_array_equal(out.cpu().numpy(), pl)
        assert abs(d.item() - want_d) < 1e-3
    else:
        assert flag.item() == 1
        np.testing.assert_array_equal(out.cpu().numpy(), ps)
