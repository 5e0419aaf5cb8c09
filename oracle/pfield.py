"""Frequency-domain point-scatterer echo model (Appendix D, Eq. 1 and Eq. 2; Algorithm 2),
FP64 (numpy).

Test infrastructure only.

Per angular frequency w = 2 pi f (wavenumber k = w / c) every scatterer s is a monopole of
reflectivity R_s.  The pressure that transmit a produces at s is the sum over the
(sub-)elements n of W_n e^{i k r_ns} / r_ns D(theta_ns, k) e^{i w dtau_n}, and the echo at
receive element m is R_s times that field times e^{i k r_ms} / r_ms D(theta_ms, k); the
element's signal is the sum over its sub-elements (Eq. 2).  Full-band RF is the sum over
frequency samples weighted by the pulse spectrum, transformed back to time.

Readings (the appendix gives the form, not the constants):
- elements of a matrix array are rectangles of size w_x x w_y centred on the element
  positions, split into v_x x v_y sub-elements at the centres of a regular subdivision;
  a sub-element's directivity is sinc(k b_x u_x) sinc(k b_y u_y) with b its half-widths,
  u the direction cosines towards the scatterer and sinc(x) = sin(x) / x (w = 0: D = 1);
- an element's response is the coherent sum over its sub-elements (Eq. 2), and the
  transmit field sums over every sub-element of the aperture (Eq. 1): an element split
  into v sub-elements responds about v times as strongly as one of them in the far field.
  The mean over the sub-elements (a response independent of the subdivision, whose
  far-field limit is the element's own directivity) is kept as an option (sub_mean);
- no elevation lens (a matrix array); transmit apodization W (default 1); transmit
  delays of the plane-wave law dtau = (u_a . p_e - min_e u_a . p_e) / c;
- amplitude (r_ref / r) on both legs; optional attenuation alpha (dB / (cm MHz)), i.e.
  k -> k + i alpha' f with alpha' in nepers per metre per hertz;
- time convention e^{-i w t}: RF(t) = 2 Re sum_j q_j S(f_j) P(f_j) e^{-i 2 pi f_j t} df with
  f_j = j df, df = fs / N, q_0 = q_{N/2} = 1/2 and q_j = 1 otherwise, where S is the
  continuous Fourier transform of the 2-cycle Gaussian pulse of the time-domain model;
  N = T + 2 ceil(6 sigma) samples so no echo inside the record wraps around; frequency
  samples whose spectral weight is below floor x max are skipped.
"""
from __future__ import annotations

import math
from typing import Optional, Tuple

import numpy as np

NEPER_PER_DB = 1.0 / (20.0 * math.log10(math.e))


def pulse_sigma_s(fc: float, n_cycles: float = 2.0) -> float:
    """Gaussian envelope standard deviation (seconds) of an n-cycle pulse (FWHM = n / fc)."""
    return n_cycles / (2.0 * math.sqrt(2.0 * math.log(2.0)) * fc)


def pulse_spectrum(f: np.ndarray, fc: float, sigma: float) -> np.ndarray:
    """Continuous Fourier transform of g(t) = exp(-t^2 / (2 sigma^2)) cos(2 pi fc t)."""
    a = 2.0 * math.pi ** 2 * sigma ** 2
    return sigma * math.sqrt(2.0 * math.pi) / 2.0 * (np.exp(-a * (f - fc) ** 2) + np.exp(-a * (f + fc) ** 2))


def pulse(t: np.ndarray, fc: float, sigma: float) -> np.ndarray:
    return np.exp(-t ** 2 / (2.0 * sigma ** 2)) * np.cos(2.0 * math.pi * fc * t)


def element_centres(nx_el: int, ny_el: int, pitch_x: float, pitch_y: float) -> np.ndarray:
    ix = np.arange(nx_el * ny_el) % nx_el
    iy = np.arange(nx_el * ny_el) // nx_el
    return np.stack([(ix - 0.5 * (nx_el - 1)) * pitch_x, (iy - 0.5 * (ny_el - 1)) * pitch_y,
                     np.zeros(nx_el * ny_el)], axis=1)


def sub_offsets(w: float, v: int) -> np.ndarray:
    """Centres of v equal parts of [-w/2, w/2]."""
    return ((np.arange(v) + 0.5) / v - 0.5) * w


def transmit_delays(tilts_rad, centres: np.ndarray, c: float) -> np.ndarray:
    """dtau[a][e] of the plane-wave transmits."""
    out = []
    for tx, ty in tilts_rad:
        sx, sy = math.sin(tx), math.sin(ty)
        u = np.array([sx, sy, math.sqrt(1.0 - sx * sx - sy * sy)])
        d = centres @ u
        out.append((d - d.min()) / c)
    return np.array(out)


def fft_length(n_samples: int, fs: float, fc: float, n_cycles: float = 2.0) -> int:
    return n_samples + 2 * int(math.ceil(6.0 * pulse_sigma_s(fc, n_cycles) * fs))


def frequency_samples(n_samples: int, fs: float, fc: float, floor: float, n_cycles: float = 2.0):
    """(N, j indices kept, f_j, weights q_j S(f_j) df)."""
    N = fft_length(n_samples, fs, fc, n_cycles)
    j = np.arange(N // 2 + 1)
    f = j * fs / N
    S = pulse_spectrum(f, fc, pulse_sigma_s(fc, n_cycles))
    keep = S >= floor * S.max()
    q = np.ones(j.size)
    q[0] = 0.5
    if N % 2 == 0:
        q[-1] = 0.5
    return N, j[keep], f[keep], (q * S * fs / N)[keep]


def element_response(f: float, pos: np.ndarray, centres: np.ndarray, wx: float, wy: float, vx: int, vy: int,
                     c: float, r_ref: float, atten: float, sub_mean: bool = False) -> np.ndarray:
    """H[e][s]: sum (Eq. 2), or mean if sub_mean, over the sub-elements of element e of
    (r_ref/r) e^{i k r} D (complex128)."""
    k = 2.0 * math.pi * f / c
    alpha = atten * NEPER_PER_DB * 100.0 * f / 1e6          # nepers per metre
    H = np.zeros((centres.shape[0], pos.shape[0]), dtype=np.complex128)
    for ox in sub_offsets(wx, vx):
        for oy in sub_offsets(wy, vy):
            p = centres + np.array([ox, oy, 0.0])
            d = pos[None, :, :] - p[:, None, :]                 # [e][s][3]
            r = np.sqrt(np.sum(d * d, axis=2))
            D = np.ones_like(r)
            if wx > 0:
                D *= np.sinc(k * (wx / (2 * vx)) * d[:, :, 0] / r / math.pi)   # numpy sinc is sin(pi x)/(pi x)
            if wy > 0:
                D *= np.sinc(k * (wy / (2 * vy)) * d[:, :, 1] / r / math.pi)
            H += (r_ref / r) * np.exp((1j * k - alpha) * r) * D
    return H / (vx * vy) if sub_mean else H


def fd_rf(nx_el: int, ny_el: int, pitch: float, fc: float, fs: float, c: float, tilts_rad, pos: np.ndarray,
          amp: np.ndarray, n_samples: int, elem_w: Tuple[float, float] = (0.0, 0.0), n_sub: Tuple[int, int] = (1, 1),
          atten: float = 0.0, apod: Optional[np.ndarray] = None, r_ref: float = 1e-3, floor: float = 1e-7,
          n_cycles: float = 2.0, sub_mean: bool = False) -> np.ndarray:
    """RF [A][E][T] of one frame of scatterers pos [S][3], amp [S] (float64)."""
    centres = element_centres(nx_el, ny_el, pitch, pitch)
    E = centres.shape[0]
    W = np.ones(E) if apod is None else np.asarray(apod, dtype=np.float64)
    dtau = transmit_delays(tilts_rad, centres, c)               # [A][E]
    N, js, fk, wk = frequency_samples(n_samples, fs, fc, floor, n_cycles)
    t = np.arange(n_samples)
    A = dtau.shape[0]
    rf = np.zeros((A, E, n_samples))
    pos = np.asarray(pos, dtype=np.float64)
    amp = np.asarray(amp, dtype=np.float64)
    for j, f, w in zip(js, fk, wk):
        H = element_response(f, pos, centres, elem_w[0], elem_w[1], n_sub[0], n_sub[1], c, r_ref, atten, sub_mean)
        tx = (W[None, :] * np.exp(1j * 2.0 * math.pi * f * dtau)) @ H       # [A][S] field at each scatterer
        P = (tx * amp[None, :]) @ H.T                                        # [A][E] echo at each element
        rf += 2.0 * np.real(w * P[:, :, None] * np.exp(-2j * math.pi * j * t / N)[None, None, :])
    return rf
