"""Block-scaled FP8 (e4m3) quantisation, for checking the FP8 path.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's symbols are exact XOR sums; the FP8 path is this
implementation's precision choice, so this module follows the OCP 8-bit floating point
definition of E4M3 (1 sign bit, 4 exponent bits with bias 7, 3 mantissa
bits, no infinities, the all-ones pattern is NaN): normal values
2^(e-7) (1 + m/8) for exponent field e in 1..15 (largest 448), subnormal
values m 2^-9.  Rounding is to nearest, ties to even, and values beyond
448 saturate to +-448.

Per 128 x 128 block of a matrix: s = the smallest power of two with
amax <= 448 s (1 if amax = 0; at least 2^-122, so that the FP8x2 residual's
s / 16 is still a normal power of two), codes of x / s.  The paper fixes no
low-precision format; a power-of-two block scale is what the matrix unit's
own E8M0 scale operands represent exactly.  Dividing by a power of two is
exact, so x / s (float32) and every code agree bit for bit with the device.
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def e4m3_value(v):
    """Round float values to the nearest e4m3 value (ties to even), saturating."""
    v = np.asarray(v, dtype=np.float64)
    a = np.minimum(np.abs(v), E4M3_MAX)
    out = np.zeros_like(a)
    nz = a > 0
    # exponent of the binade, at least the smallest normal exponent -6
    e = np.floor(np.log2(np.where(nz, a, 1.0)))
    e = np.maximum(e, -6.0)
    step = np.exp2(e - 3.0)              # 3 mantissa bits (subnormal step 2^-9 at e = -6)
    q = np.rint(a / step) * step         # np.rint: round half to even
    out[nz] = q[nz]
    out = np.minimum(out, E4M3_MAX)
    return np.copysign(out, v)


def e4m3_code(v):
    """Bit patterns (uint8) of the e4m3 values nearest to v."""
    q = e4m3_value(v)
    sign = np.signbit(q).astype(np.uint8) << 7
    a = np.abs(q)
    code = np.zeros(a.shape, dtype=np.uint8)
    normal = a >= 2.0 ** -6
    e = np.floor(np.log2(np.where(normal, a, 1.0)))
    mant = np.where(normal, a / np.exp2(e) * 8 - 8, a / 2.0 ** -9)
    efield = np.where(normal, e + 7, 0)
    code = (efield.astype(np.int64) << 3 | np.rint(mant).astype(np.int64)).astype(np.uint8)
    return code | sign


def e4m3_decode(code):
    code = np.asarray(code, dtype=np.uint8)
    s = np.where(code & 0x80, -1.0, 1.0)
    e = (code >> 3) & 0xF
    m = code & 0x7
    val = np.where(e == 0, m * 2.0 ** -9, (1 + m / 8.0) * np.exp2(e.astype(np.float64) - 7))
    return s * val


MIN_SCALE_EXP = -122


def block_scale(amax) -> np.float32:
    """The smallest power of two s with amax <= 448 s, at least 2^-122;
    1 for amax = 0.  Stepped up from a start known to be at or below it."""
    amax = float(amax)
    if amax == 0.0:
        return np.float32(1.0)
    e = max(MIN_SCALE_EXP, int(np.floor(np.log2(amax / E4M3_MAX))) - 2)
    while E4M3_MAX * 2.0 ** e < amax:
        e += 1
    return np.float32(2.0 ** e)


def quantize_block(x, residual: bool = False):
    """Scale and codes of one float32 block; with residual, also the codes of
    (x/s - q) * 16.  Returns (scale, codes[, residual codes])."""
    x = np.asarray(x, dtype=np.float32)
    amax = np.float32(np.max(np.abs(x))) if x.size else np.float32(0)
    s = block_scale(amax)
    v = (x / s).astype(np.float32)
    c = e4m3_code(np.clip(v, -E4M3_MAX, E4M3_MAX))
    if not residual:
        return s, c
    r = ((v - e4m3_decode(c).astype(np.float32)).astype(np.float32) * np.float32(16)).astype(np.float32)
    return s, c, e4m3_code(np.clip(r, -E4M3_MAX, E4M3_MAX))


def coded_block_fp32(A, Mb, members, M):
    """Coded block sum in float32, members added in ascending order (the
    device's order), rows past M zero."""
    K = A.shape[1]
    acc = np.zeros((Mb, K), dtype=np.float32)
    for s in sorted(members):
        lo, hi = s * Mb, min((s + 1) * Mb, M)
        if hi > lo:
            acc[: hi - lo] = (acc[: hi - lo] + A[lo:hi].astype(np.float32)).astype(np.float32)
    return acc
