"""Learned slow-time clutter filter: forward, backward and Adam in FP64 (numpy).

Test infrastructure only.

The network maps one voxel's slow-time series to an estimate of its blood
component.  Input x = [Re, Im](S[v, :]) / s_v with s_v = sqrt(mean_f |S[v,f]|^2 + eps)
(shape [N][2][T]).  Layers:
    h1 = GELU(conv9(x;  W1[32,2,9],  b1))
    h2 = GELU(conv9(h1; W2[32,32,9], b2))
    h3 = GELU(conv9(h2; W3[32,32,9], b3))
    y  = conv1(h3; W4[2,32], b4)
conv9(z)[o,t] = b[o] + sum_i sum_{k=0..8} W[o,i,k] z[i, t+k-4] with zeros outside
[0, T) ("same" padding); GELU in its tanh form (Hendrycks & Gimpel),
    GELU(z) = z/2 (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))),
which stays within 4.8e-4 of the erf form z/2 (1 + erf(z/sqrt 2)).
Blood estimate S_b[v,f] = s_v (y0 + i y1); loss = mean over (n, channel, t) of
(y - y_target)^2 with y_target = [Re, Im](S_blood[v,:]) / s_v.

Parameter vector layout (float32 [19170]):
    W1 [32][2][9] | b1 [32] | W2 [32][32][9] | b2 [32] | W3 [32][32][9] | b3 [32] | W4 [2][32] | b4 [2]

`bf16=True` rounds at the points the GPU kernels round (RNE): weights and each
stored activation h1..h3 and pre-activation z1..z3 are BF16; the network input
(FP32 after normalisation) is kept as two BF16 terms, hi = bf16(x) and
lo = bf16(x - hi), whose sum carries ~16 significant bits (one BF16 alone puts its
rounding noise ~59 dB below the series power, which tissue dominates, i.e. at the
level of the weakest blood); the output-layer gradient and every accumulation stay
wide.
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

from .bf16 import bf16_round

C_HID = 32
KW = 9
PAD = 4
SHAPES = [('W1', (C_HID, 2, KW)), ('b1', (C_HID,)), ('W2', (C_HID, C_HID, KW)), ('b2', (C_HID,)),
          ('W3', (C_HID, C_HID, KW)), ('b3', (C_HID,)), ('W4', (2, C_HID)), ('b4', (2,))]
N_PARAM = int(sum(np.prod(s) for _, s in SHAPES))


def unpack(w: np.ndarray) -> Dict[str, np.ndarray]:
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(w[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(p: Dict[str, np.ndarray]) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


GELU_C = np.sqrt(2.0 / np.pi)
GELU_A = 0.044715


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(GELU_C * (z + GELU_A * z ** 3)))


def gelu_grad(z):
    """d GELU / dz: (1 + tanh u)/2 + z (1 - tanh^2 u) u'/2, u = C (z + A z^3)."""
    th = np.tanh(GELU_C * (z + GELU_A * z ** 3))
    return 0.5 * (1.0 + th) + 0.5 * z * (1.0 - th * th) * GELU_C * (1.0 + 3.0 * GELU_A * z * z)


def conv(z: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """z [N][Ci][T], W [Co][Ci][K] (K odd, 'same' zero padding) -> [N][Co][T]."""
    N, Ci, T = z.shape
    K = W.shape[2]
    p = K // 2
    zp = np.zeros((N, Ci, T + 2 * p))
    zp[:, :, p:p + T] = z
    out = np.broadcast_to(b[None, :, None], (N, W.shape[0], T)).copy()
    for k in range(K):
        out += np.einsum('oi,nit->not', W[:, :, k], zp[:, :, k:k + T])
    return out


def conv_backward(z: np.ndarray, W: np.ndarray, dout: np.ndarray):
    """Gradients of conv(z, W, b) given dL/dout: returns (dz, dW, db)."""
    N, Ci, T = z.shape
    K = W.shape[2]
    p = K // 2
    zp = np.zeros((N, Ci, T + 2 * p))
    zp[:, :, p:p + T] = z
    dW = np.zeros_like(W)
    dzp = np.zeros_like(zp)
    for k in range(K):
        dW[:, :, k] = np.einsum('not,nit->oi', dout, zp[:, :, k:k + T])
        dzp[:, :, k:k + T] += np.einsum('oi,not->nit', W[:, :, k], dout)
    db = dout.sum(axis=(0, 2))
    return dzp[:, :, p:p + T], dW, db


def normalise(iq_series: np.ndarray, eps: float = 1e-30) -> Tuple[np.ndarray, np.ndarray]:
    """iq_series complex [N][T] -> (x [N][2][T], s [N])."""
    s = np.sqrt(np.mean(np.abs(iq_series) ** 2, axis=1) + eps)
    x = np.stack([iq_series.real, iq_series.imag], axis=1) / s[:, None, None]
    return x, s


def _q(a, on):
    return bf16_round(a.astype(np.float32)).astype(np.float64) if on else a


def _q2(a, on):
    """hi + lo: two BF16 terms of the FP32 value (the remainder x - hi is exact in FP32)."""
    if not on:
        return a
    x = a.astype(np.float32)
    hi = bf16_round(x)
    lo = bf16_round((x - hi).astype(np.float32))
    return hi.astype(np.float64) + lo.astype(np.float64)


def forward(w: np.ndarray, x: np.ndarray, bf16: bool = False):
    """x [N][2][T] -> (y [N][2][T], cache)."""
    p = unpack(w)
    if bf16:
        p = {k: (_q(v, True) if k.startswith('W') else v) for k, v in p.items()}
    h0 = _q2(x, bf16)
    z1 = conv(h0, p['W1'], p['b1'])
    h1 = _q(gelu(z1), bf16)
    z2 = conv(h1, p['W2'], p['b2'])
    h2 = _q(gelu(z2), bf16)
    z3 = conv(h2, p['W3'], p['b3'])
    h3 = _q(gelu(z3), bf16)
    y = np.einsum('oi,nit->not', p['W4'], h3) + p['b4'][None, :, None]
    cache = dict(p=p, h0=h0, z1=_q(z1, bf16), h1=h1, z2=_q(z2, bf16), h2=h2, z3=_q(z3, bf16), h3=h3)
    return y, cache


def loss_and_grad(w: np.ndarray, x: np.ndarray, target: np.ndarray, bf16: bool = False):
    """Mean-squared-error loss and its gradient w.r.t. the parameter vector."""
    y, c = forward(w, x, bf16)
    diff = y - target
    loss = float(np.mean(diff ** 2))
    dy = 2.0 * diff / diff.size
    p = c['p']
    dW4 = np.einsum('not,nit->oi', dy, c['h3'])
    db4 = dy.sum(axis=(0, 2))
    dh3 = np.einsum('oi,not->nit', p['W4'], dy)
    dz3 = _q(dh3 * gelu_grad(c['z3']), bf16)
    dh2, dW3, db3 = conv_backward(c['h2'], p['W3'], dz3)
    dz2 = _q(dh2 * gelu_grad(c['z2']), bf16)
    dh1, dW2, db2 = conv_backward(c['h1'], p['W2'], dz2)
    dz1 = _q(dh1 * gelu_grad(c['z1']), bf16)
    _, dW1, db1 = conv_backward(c['h0'], p['W1'], dz1)
    g = pack(dict(W1=dW1, b1=db1, W2=dW2, b2=db2, W3=dW3, b3=db3, W4=dW4, b4=db4))
    return loss, g


def blood_estimate(w: np.ndarray, iq: np.ndarray, bf16: bool = False, eps: float = 1e-30) -> np.ndarray:
    """iq complex [N_t][N_v] (frame-major) -> blood estimate complex [N_t][N_v]."""
    x, s = normalise(iq.T, eps)
    y, _ = forward(w, x, bf16)
    return ((y[:, 0, :] + 1j * y[:, 1, :]) * s[:, None]).T


def adam(w, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments); returns new (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
