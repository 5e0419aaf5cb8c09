"""Pins of the learned-filter oracle: torch autograd (an independent implementation of
conv1d / GELU and their gradients), central finite differences, the impulse
response of a single layer, and torch's Adam."""
import numpy as np
import torch
import torch.nn.functional as Fn

from fqscene import lcf_init_weights
from oracle import lcf


def _torch_forward(w, x):
    p = {k: torch.tensor(v, dtype=torch.float64) for k, v in lcf.unpack(w).items()}
    for v in p.values():
        v.requires_grad_(True)
    xt = torch.tensor(x, dtype=torch.float64)
    h = Fn.gelu(Fn.conv1d(xt, p['W1'], p['b1'], padding=4), approximate='tanh')
    h = Fn.gelu(Fn.conv1d(h, p['W2'], p['b2'], padding=4), approximate='tanh')
    h = Fn.gelu(Fn.conv1d(h, p['W3'], p['b3'], padding=4), approximate='tanh')
    y = Fn.conv1d(h, p['W4'][:, :, None], p['b4'])
    return y, p


def _data(seed, n=3, T=24):
    rng = np.random.default_rng(seed)
    w = lcf_init_weights(seed).astype(np.float64)
    w += 0.05 * rng.standard_normal(w.size)          # non-zero biases too
    x = rng.standard_normal((n, 2, T))
    tgt = 0.3 * rng.standard_normal((n, 2, T))
    return w, x, tgt


def test_param_count():
    assert lcf.N_PARAM == 19170


def test_forward_and_gradient_match_torch_autograd():
    w, x, tgt = _data(1)
    y, _ = lcf.forward(w, x)
    yt, p = _torch_forward(w, x)
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)
    loss, g = lcf.loss_and_grad(w, x, tgt)
    lt = torch.mean((yt - torch.tensor(tgt)) ** 2)
    lt.backward()
    gt = np.concatenate([p[name].grad.numpy().ravel() for name, _ in lcf.SHAPES])
    assert abs(loss - lt.item()) < 1e-14
    np.testing.assert_allclose(g, gt, rtol=1e-10, atol=1e-14)


def test_gradient_finite_differences():
    w, x, tgt = _data(2, n=2, T=16)
    _, g = lcf.loss_and_grad(w, x, tgt)
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.choice(lcf.N_PARAM, 60, replace=False), np.arange(19104, 19170, 7)])
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (lcf.loss_and_grad(wp, x, tgt)[0] - lcf.loss_and_grad(wm, x, tgt)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g).max(), 1e-12) + 1e-6 * abs(g[i])


def test_conv_same_padding_impulse_response():
    """A unit impulse at t0 through one conv9 layer returns the kernel taps reversed in time:
    out[o, t0 - (k - 4)] = W[o, i, k] + b[o]; everything else equals the bias."""
    rng = np.random.default_rng(4)
    W = rng.standard_normal((3, 2, 9))
    b = rng.standard_normal(3)
    T, t0 = 30, 13
    z = np.zeros((1, 2, T))
    z[0, 1, t0] = 1.0
    out = lcf.conv(z, W, b)[0]
    for k in range(9):
        np.testing.assert_allclose(out[:, t0 - (k - 4)], W[:, 1, k] + b, rtol=1e-14)
    mask = np.ones(T, bool)
    mask[t0 - 4:t0 + 5] = False
    np.testing.assert_allclose(out[:, mask], np.repeat(b[:, None], mask.sum(), 1), rtol=1e-14)


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    w0 = rng.standard_normal(50)
    wt = torch.tensor(w0.copy(), requires_grad=True)
    opt = torch.optim.Adam([wt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 8):
        g = rng.standard_normal(50)
        opt.zero_grad()
        wt.grad = torch.tensor(g)
        opt.step()
        w, m, v = lcf.adam(w, m, v, g, step)
    np.testing.assert_allclose(w, wt.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_bf16_mode_close_to_fp64():
    """The BF16-rounding mode stays within BF16 resolution of the FP64 network."""
    w, x, tgt = _data(6)
    y64, _ = lcf.forward(w, x)
    y16, _ = lcf.forward(w, x, bf16=True)
    rel = np.linalg.norm(y16 - y64) / np.linalg.norm(y64)
    assert 1e-5 < rel < 2e-2
    _, g64 = lcf.loss_and_grad(w, x, tgt)
    _, g16 = lcf.loss_and_grad(w, x, tgt, bf16=True)
    assert np.linalg.norm(g16 - g64) / np.linalg.norm(g64) < 3e-2


def test_normalise_and_blood_estimate_scale():
    """Scaling a series by c scales the estimate by c (the network sees unit-RMS input)."""
    rng = np.random.default_rng(7)
    w = lcf_init_weights(7).astype(np.float64)
    iq = rng.standard_normal((20, 5)) + 1j * rng.standard_normal((20, 5))
    a = lcf.blood_estimate(w, iq)
    b = lcf.blood_estimate(w, 1000.0 * iq)
    np.testing.assert_allclose(b, 1000.0 * a, rtol=1e-9)
    x, s = lcf.normalise(iq.T)
    np.testing.assert_allclose(np.mean(np.sum(x ** 2, axis=1), axis=1), 1.0, rtol=1e-12)


def test_bf16_input_as_two_terms():
    """The BF16 mode's network input is hi + lo (hi = bf16(x), lo = bf16(x - hi)): within
    2^-16 of the FP32 value (2^-8 per rounding), where one BF16 alone is only within 2^-8.
    On a unit-RMS series whose second component sits 60 dB below the first, the single
    BF16's rounding noise is larger than that component, the two terms' noise well under
    1% of it."""
    rng = np.random.default_rng(11)
    x = rng.standard_normal(20000) * 10.0 ** rng.uniform(-3, 3, 20000)
    xf = x.astype(np.float32).astype(np.float64)
    two = lcf._q2(x, True)
    one = lcf._q(x, True)
    assert np.all(np.abs(two - xf) <= 2.0 ** -16 * np.abs(xf))
    assert np.max(np.abs(one - xf) / np.abs(xf)) > 2.0 ** -10
    t = np.arange(200)
    big = np.sqrt(2.0) * np.cos(2 * np.pi * 0.013 * t)
    small = 1e-3 * np.sqrt(2.0) * np.cos(2 * np.pi * 0.21 * t + 0.3)
    s = big + small
    e_two = np.linalg.norm(lcf._q2(s, True) - s) / np.linalg.norm(small)
    e_one = np.linalg.norm(lcf._q(s, True) - s) / np.linalg.norm(small)
    assert e_two < 1e-2 and e_one > 0.5


def test_gelu_tanh_form_against_torch():
    """The activation and its derivative against torch's tanh-form GELU (value and
    autograd derivative), GELU(0) = 0 and GELU'(0) = 1/2, and the tanh form within
    4.8e-4 of the erf form."""
    from scipy.special import erf
    z = np.linspace(-8.0, 8.0, 4001)
    zt = torch.tensor(z, dtype=torch.float64, requires_grad=True)
    y = Fn.gelu(zt, approximate='tanh')
    y.sum().backward()
    np.testing.assert_allclose(lcf.gelu(z), y.detach().numpy(), rtol=0, atol=1e-14)
    np.testing.assert_allclose(lcf.gelu_grad(z), zt.grad.numpy(), rtol=0, atol=1e-13)
    assert lcf.gelu(np.array([0.0]))[0] == 0.0 and abs(lcf.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15
    assert np.abs(lcf.gelu(z) - 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))).max() < 4.8e-4
