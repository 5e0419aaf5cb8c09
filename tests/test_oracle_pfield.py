"""Pins of the frequency-domain echo-model oracle (Appendix D, Eq. 1-2)."""
import math

import numpy as np
import pytest

from oracle import pfield

FC, FS, C = 7.8e6, 31.25e6, 1540.0
PITCH = 0.3e-3
T = 512


def one_path(src, rcv, pos, amp=0.7, **kw):
    """RF at element rcv when only element src transmits (no tilt)."""
    apod = np.zeros(16)
    apod[src] = 1.0
    rf = pfield.fd_rf(4, 4, PITCH, FC, FS, C, [(0.0, 0.0)], np.array([pos]), np.array([amp]), T, apod=apod, **kw)
    return rf[0, rcv]


def test_single_path_is_the_delayed_pulse():
    """One transmitting element, one receiver, one scatterer, point elements: the echo is
    the pulse delayed by the two-way path and scaled by r_ref^2 / (r_tx r_rx)."""
    cen = pfield.element_centres(4, 4, PITCH, PITCH)
    pos = np.array([0.4e-3, -0.2e-3, 6e-3])
    sig = pfield.pulse_sigma_s(FC)
    for src, rcv in ((5, 5), (0, 15), (3, 12)):
        r0 = np.linalg.norm(pos - cen[src])
        r1 = np.linalg.norm(pos - cen[rcv])
        want = 0.7 * (1e-3 / r0) * (1e-3 / r1) * pfield.pulse(np.arange(T) / FS - (r0 + r1) / C, FC, sig)
        got = one_path(src, rcv, pos, floor=1e-12)
        assert np.max(np.abs(got - want)) < 1e-6 * np.max(np.abs(want))


def test_attenuation_downshifts_the_gaussian():
    """A Gaussian spectrum times e^{-beta f} is a Gaussian centred at fc - beta/(4 pi^2 s^2)
    scaled by exp(-beta fc + beta^2 / (8 pi^2 s^2)) (beta = alpha' x path length)."""
    cen = pfield.element_centres(4, 4, PITCH, PITCH)
    pos = np.array([0.1e-3, 0.3e-3, 8e-3])
    sig = pfield.pulse_sigma_s(FC)
    atten = 0.7                                   # dB / (cm MHz)
    r0 = np.linalg.norm(pos - cen[6])
    r1 = np.linalg.norm(pos - cen[9])
    beta = atten * pfield.NEPER_PER_DB * 100.0 / 1e6 * (r0 + r1)
    fc2 = FC - beta / (4 * math.pi ** 2 * sig ** 2)
    gain = math.exp(-beta * FC + beta ** 2 / (8 * math.pi ** 2 * sig ** 2))
    u = np.arange(T) / FS - (r0 + r1) / C
    want = 0.7 * (1e-3 / r0) * (1e-3 / r1) * gain * np.exp(-u ** 2 / (2 * sig ** 2)) * np.cos(2 * math.pi * fc2 * u)
    got = one_path(6, 9, pos, atten=atten, floor=1e-12)
    assert gain < 0.97 and fc2 < FC - 1e4           # the effect is visible
    assert np.max(np.abs(got - want)) < 5e-6 * np.max(np.abs(want))


def test_reciprocity_with_directivity_and_sub_elements():
    pos = np.array([0.9e-3, -0.5e-3, 5e-3])
    kw = dict(elem_w=(0.25e-3, 0.25e-3), n_sub=(2, 3))
    a = one_path(1, 14, pos, **kw)
    b = one_path(14, 1, pos, **kw)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


def test_sub_elements_converge_to_the_element_directivity_in_the_far_field():
    """Product theorem under Eq. 2's coherent sum: in the far field the sum over v
    sub-elements with directivity sinc(k b/v u) equals v times one element with sinc(k b u)
    (the mean option equals the element itself); the residual is the Fresnel term
    ~ k w^2 / (8 r) and falls like 1/r."""
    cen = pfield.element_centres(1, 1, PITCH, PITCH)
    f = FC
    errs = []
    for r in (1.0, 4.0):
        pos = np.array([[0.3 * r, -0.2 * r, 0.9 * r]])
        h1 = pfield.element_response(f, pos, cen, 0.3e-3, 0.3e-3, 1, 1, C, 1e-3, 0.0)
        h5 = pfield.element_response(f, pos, cen, 0.3e-3, 0.3e-3, 5, 5, C, 1e-3, 0.0)
        m5 = pfield.element_response(f, pos, cen, 0.3e-3, 0.3e-3, 5, 5, C, 1e-3, 0.0, sub_mean=True)
        errs.append(abs(h5[0, 0] / 25.0 - h1[0, 0]) / abs(h1[0, 0]))
        assert abs(m5[0, 0] - h5[0, 0] / 25.0) <= 1e-15 * abs(h5[0, 0])
    k = 2 * math.pi * f / C
    assert errs[0] < k * (0.3e-3) ** 2 / (8 * 1.0) * 2
    assert 3.0 < errs[0] / errs[1] < 5.0
    # the directivity is really applied: off axis the element is weaker than a point
    pos = np.array([[5e-3, 0.0, 5e-3]])
    hp = pfield.element_response(f, pos, cen, 0.0, 0.0, 1, 1, C, 1e-3, 0.0)
    hd = pfield.element_response(f, pos, cen, 0.3e-3, 0.3e-3, 1, 1, C, 1e-3, 0.0)
    x = k * 0.15e-3 * math.sin(math.pi / 4)
    assert abs(abs(hd[0, 0]) / abs(hp[0, 0]) - abs(math.sin(x) / x)) < 1e-12


def test_echo_scales_with_the_square_of_the_sub_element_count():
    """Eq. 1 sums the transmit field over every sub-element and Eq. 2 sums the receive
    element's sub-elements, so for a scatterer far on axis (where every sub-element sees
    the same path and directivity 1) splitting each element into v sub-elements scales the
    echo by v^2 on both legs (here v = 6: 36); the ratio approaches 36 as the Fresnel term
    k (w/2)^2 / (2 r) vanishes, and the mean option gives a response independent of v."""
    w = (0.2e-3, 0.2e-3)
    ratios, ratios_mean = [], []
    for z in (0.05, 0.2):
        pos = np.array([[0.0, 0.0, z]])
        T = 2 * int(z / C * FS) + 64
        kw = dict(elem_w=w)
        one = pfield.fd_rf(1, 1, PITCH, FC, FS, C, [(0.0, 0.0)], pos, np.ones(1), T, n_sub=(1, 1), **kw)
        six = pfield.fd_rf(1, 1, PITCH, FC, FS, C, [(0.0, 0.0)], pos, np.ones(1), T, n_sub=(2, 3), **kw)
        six_m = pfield.fd_rf(1, 1, PITCH, FC, FS, C, [(0.0, 0.0)], pos, np.ones(1), T, n_sub=(2, 3), sub_mean=True,
                             **kw)
        # amplitude ratio from the energies (insensitive to the sub-sample arrival time)
        ratios.append(math.sqrt(np.sum(six ** 2) / np.sum(one ** 2)))
        ratios_mean.append(math.sqrt(np.sum(six_m ** 2) / np.sum(one ** 2)))
    assert abs(ratios[0] - 36.0) < 1e-3 * 36.0
    assert abs(ratios[1] - 36.0) < 0.25 * abs(ratios[0] - 36.0)
    assert all(abs(r - 1.0) < 1e-4 for r in ratios_mean)


def test_superposition_and_zero_amplitude():
    kw = dict(elem_w=(0.2e-3, 0.2e-3), n_sub=(2, 2))
    tilts = [(math.radians(-5), 0.0), (0.0, math.radians(5))]
    p = np.array([[0.2e-3, 0.1e-3, 5e-3], [-0.4e-3, 0.3e-3, 7e-3]])
    a = np.array([0.5, -1.2])
    both = pfield.fd_rf(4, 4, PITCH, FC, FS, C, tilts, p, a, T, **kw)
    one = pfield.fd_rf(4, 4, PITCH, FC, FS, C, tilts, p[:1], a[:1], T, **kw)
    two = pfield.fd_rf(4, 4, PITCH, FC, FS, C, tilts, p[1:], a[1:], T, **kw)
    assert np.max(np.abs(both - one - two)) < 1e-12 * np.max(np.abs(both))
    zero = pfield.fd_rf(4, 4, PITCH, FC, FS, C, tilts, p, np.zeros(2), T, **kw)
    assert np.all(zero == 0.0)


def test_spectrum_and_frequency_samples():
    sig = pfield.pulse_sigma_s(FC)
    # the transform of the pulse at the carrier is sigma sqrt(2 pi) / 2 (plus a negligible mirror term)
    assert abs(pfield.pulse_spectrum(np.array([FC]), FC, sig)[0] / (sig * math.sqrt(2 * math.pi) / 2) - 1) < 1e-12
    N, js, f, w = pfield.frequency_samples(T, FS, FC, 1e-7)
    assert N == T + 2 * math.ceil(6 * sig * FS)
    assert js.min() >= 0 and js.max() <= N // 2 and np.all(np.diff(js) == 1)
    assert FC - 1e5 < f[np.argmax(w)] < FC + 1e5
