"""The approximation behind RF synthesis's spreading form, checked in FP64 on the CPU (no
GPU, no library): a sum of Gaussian-envelope pulses cut at 5 sigma equals, within the
stated bound, the real part of a carrier times a half-rate complex trace (scatterers
spread with a narrow Gaussian phi of variance alpha s^2) filtered with a Gaussian psi of
variance (1 - alpha) s^2.  The split rule, tap count and filter half-width are the ones
the library's host code documents: alpha = max(1/3, smallest alpha with half-rate
aliasing 2 exp(-pi^2 alpha (1 - alpha) s^2 / 2) <= 5e-6), NT = 2 ceil(sqrt(24 alpha s^2)/2),
P = ceil(sqrt(34 (1 - alpha) s^2)).  Bound: the 5-sigma cut (3.7e-6 of a peak), the
aliasing (5e-6) and the cut ends of phi and psi; the test allows 8e-6 relative L2."""
import math

import numpy as np
import pytest

NU = 7.8e6 / 31.25e6   # carrier cycles per sample


def split_params(sig):
    s2 = sig * sig
    q = 4.0 * 2.614 / s2
    alpha = max(1.0 / 3.0, 0.5 * (1.0 - math.sqrt(1.0 - q)))
    a, b = alpha * s2, (1.0 - alpha) * s2
    nt = 2 * math.ceil(0.5 * math.sqrt(24.0 * a))
    P = math.ceil(math.sqrt(2.0 * b * 17.0))
    return a, b, nt, P


def direct(x, A, T, sig, trunc=5.0):
    u = np.arange(T)[None, :] - x[:, None]
    g = np.exp(-u ** 2 / (2 * sig * sig)) * np.cos(2 * np.pi * NU * u) * (np.abs(u) <= trunc * sig)
    return (A[:, None] * g).sum(0)


def spread(x, A, T, sig):
    a, b, nt, P = split_params(sig)
    j0 = 1 - nt // 2
    G = 64
    buf = np.zeros((T + 1) // 2 + 2 * G, complex)
    mb = np.floor(0.5 * x).astype(int)
    f = x - 2 * mb
    c = A * np.exp(-2j * np.pi * NU * x)
    for j in range(j0, j0 + nt):
        np.add.at(buf, G + mb + j, c * np.exp(-(2 * j - f) ** 2 / (2 * a)))
    norm = 2.0 / math.sqrt(2 * math.pi * a * b / (sig * sig))
    n = np.arange(T)
    m = np.arange(-G, buf.size - G)
    t = n[:, None] - 2 * m[None, :]
    psi = np.where(np.abs(t) <= P, norm * np.exp(-t ** 2 / (2 * b)), 0.0)
    return (np.exp(2j * np.pi * NU * n) * (psi @ buf)).real


@pytest.mark.parametrize('n_cycles', [1.94, 2.0, 3.0, 5.0])
def test_spreading_matches_truncated_pulse_sum(n_cycles):
    sig = n_cycles / (2 * math.sqrt(2 * math.log(2)) * 7.8e6) * 31.25e6   # samples
    assert sig >= 3.3
    T, S = 256, 300
    J = math.floor(5 * sig)
    rng = np.random.default_rng(int(100 * n_cycles))
    x = rng.uniform(-(J + 2) + 1e-9, T + J + 1 - 1e-9, S)   # the kernels' acceptance window
    A = rng.standard_normal(S)
    ref = direct(x, A, T, sig)
    got = spread(x, A, T, sig)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print('cycles', n_cycles, 'sigma', sig, 'taps', split_params(sig)[2], 'rel L2', err)
    assert err < 8e-6


def test_split_rule_for_the_workloads_pulse():
    """2-cycle pulse at fc / fs = 7.8 / 31.25 MHz: 10 taps, filter half-width 17 samples."""
    sig = 2.0 / (2 * math.sqrt(2 * math.log(2)) * 7.8e6) * 31.25e6
    a, b, nt, P = split_params(sig)
    assert nt == 10 and P == 17
    assert abs(a / (sig * sig) - 0.344) < 1e-3
