"""bf16 hi/lo splitting and the split-precision product, emulated in FP64.

ORACLE -- test infrastructure only (see the package header).

Split precision (an extension; the paper itself runs complex64 with FP32
arithmetic, Sec. V): every float32 value x becomes
    x_hi = bf16_rne(x),  x_lo = bf16_rne(x - x_hi)
and every real product a*b is replaced by a_hi b_hi + a_hi b_lo + a_lo b_hi.
A complex product uses four such real products (4M form):
    re = (ar br) - (ai bi),   im = (ar bi) + (ai br),
or three (3M form): T1 = ar br, T2 = ai bi, T3 = (ar + ai)(br + bi), with
the sums formed in float32 like the other float32 planes, re = T1 - T2,
im = T3 - T1 - T2.
Each bf16 x bf16 product is exact in float32 and in float64, so the
emulation below (three-term products summed in float64, then the step
result rounded to complex64 as the device stores it) differs from the device
only by the device's float32 accumulation error.

bf16 rounding is done on the float32 bit pattern: add 0x7FFF plus the lowest
kept bit, then clear the low 16 bits (round to nearest, ties to even).
"""
from __future__ import annotations

import numpy as np

from .contract import pairwise


def bf16_rne(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bf16 (returned as float32 with zero low bits)."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    nan = np.isnan(f)
    out = r.view(np.float32).copy()
    out[nan] = f[nan]
    return out


def split(x: np.ndarray):
    f = np.asarray(x, dtype=np.float32)
    hi = bf16_rne(f)
    lo = bf16_rne((f.astype(np.float64) - hi.astype(np.float64)).astype(np.float32))
    return hi.astype(np.float64), lo.astype(np.float64)


def _real3(x, la, y, lb, keep):
    xh, xl = split(x)
    yh, yl = split(y)
    z1, lz = pairwise(xh, la, yh, lb, keep)
    z2, _ = pairwise(xh, la, yl, lb, keep)
    z3, _ = pairwise(xl, la, yh, lb, keep)
    return z1 + z2 + z3, lz


def split_step(x, la, y, lb, keep):
    """Drop-in replacement for :func:`oracle.contract.pairwise` that emulates
    the split-bf16 (3 products per real product) step and stores the result
    in complex64 precision."""
    xr, xi = np.real(x), np.imag(x)
    yr, yi = np.real(y), np.imag(y)
    rr, lz = _real3(xr, la, yr, lb, keep)
    ii, _ = _real3(xi, la, yi, lb, keep)
    ri, _ = _real3(xr, la, yi, lb, keep)
    ir, _ = _real3(xi, la, yr, lb, keep)
    re = (rr - ii).astype(np.float32).astype(np.float64)
    im = (ri + ir).astype(np.float32).astype(np.float64)
    return re + 1j * im, lz


def split_step_3m(x, la, y, lb, keep):
    """The split-bf16 step in the 3M form: three split real products
    T1 = ar br, T2 = ai bi, T3 = (ar + ai)(br + bi), the sum planes rounded
    to float32 before they are split; re = T1 - T2 and im = T3 - T1 - T2
    in float64, the result stored in complex64 precision."""
    xr, xi = np.real(x).astype(np.float32), np.imag(x).astype(np.float32)
    yr, yi = np.real(y).astype(np.float32), np.imag(y).astype(np.float32)
    xs = xr + xi   # float32 sums
    ys = yr + yi
    t1, lz = _real3(xr, la, yr, lb, keep)
    t2, _ = _real3(xi, la, yi, lb, keep)
    t3, _ = _real3(xs, la, ys, lb, keep)
    re = (t1 - t2).astype(np.float32).astype(np.float64)
    im = (t3 - t1 - t2).astype(np.float32).astype(np.float64)
    return re + 1j * im, lz


def c64_step(x, la, y, lb, keep):
    """Exact product, result rounded to complex64 (the storage precision)."""
    z, lz = pairwise(x, la, y, lb, keep)
    return z.astype(np.complex64).astype(np.complex128), lz
