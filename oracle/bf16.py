"""BF16 rounding and the split-BF16 Gram emulation (numpy).

Test infrastructure only.

bfloat16 keeps the sign, the 8-bit exponent and the top 7 stored mantissa bits
of an IEEE float32.  Round-to-nearest-even on the bit pattern: add
0x7FFF + (bit 16 of the pattern) and clear the low 16 bits (finite inputs).

Split-BF16: hi = bf16(x), lo = bf16(x - hi) (x - hi is exact in float32), so
x ~= hi + lo to about 16 significant bits.  A product x*y is approximated by
the three BF16 products hi_x hi_y + hi_x lo_y + lo_x hi_y (the lo*lo term, of
relative size 2^-16, is dropped).  Each BF16 product is exact in float32.
"""
from __future__ import annotations

import numpy as np


def bf16_round(x: np.ndarray) -> np.ndarray:
    """float32 -> nearest bfloat16 value (ties to even), returned as float32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).reshape(x.shape)


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """uint16 bit patterns of bf16_round(x)."""
    return (bf16_round(x).view(np.uint32) >> 16).astype(np.uint16)


def split(x: np.ndarray):
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_round(x)
    lo = bf16_round((x - hi).astype(np.float32))
    return hi, lo


def _real_parts(iq: np.ndarray):
    iq = np.asarray(iq, dtype=np.complex64)
    return np.ascontiguousarray(iq.real), np.ascontiguousarray(iq.imag)


def gram_split_bf16(iq: np.ndarray, products: int = 3, chunk: int = 1 << 18) -> np.ndarray:
    """Emulated Gram G = S^H S from BF16 parts, every product and sum in FP64.

    products = 3: split-BF16 (hi hi + hi lo + lo hi); products = 4: adds lo lo;
    products = 1: plain BF16 (hi hi only, the negative control).  iq is complex64 [N_t][N_v] (frame-major).
    Re G = A^T A + B^T B and Im G = A^T B - B^T A for S = A + iB."""
    nt, nv = iq.shape
    G = np.zeros((nt, nt), dtype=np.complex128)
    for v0 in range(0, nv, chunk):
        A, B = _real_parts(iq[:, v0:v0 + chunk])
        Ah, Al = (p.astype(np.float64) for p in split(A))
        Bh, Bl = (p.astype(np.float64) for p in split(B))

        def prod(Xh, Xl, Yh, Yl):
            r = Xh @ Yh.T
            if products >= 3:
                r = r + Xh @ Yl.T + Xl @ Yh.T
            if products == 4:
                r = r + Xl @ Yl.T
            return r

        re = prod(Ah, Al, Ah, Al) + prod(Bh, Bl, Bh, Bl)
        im = prod(Ah, Al, Bh, Bl) - prod(Bh, Bl, Ah, Al)
        G += re + 1j * im
    return G
