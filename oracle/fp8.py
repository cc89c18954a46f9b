"""Low-precision measurement forms of the encoder, in exact arithmetic.

Test infrastructure (part of the FP64 CPU oracle): never imported by the
product path.

The paper's case for the coder is a low-complexity encoder (Sections 1 and 3:
the encoder only multiplies the residual by a random matrix).  Two reduced-
precision forms of that product are defined here:

* int8 form: the residual r (integer, |r| <= 255) is written as two int8
  digits r = 16 h + l with l = r mod 16 in [0, 15] and h = floor(r / 16) in
  [-16, 15]; y~ = 16 (Q h) + Q l.  This is an identity, so the int8 form
  produces exactly the integer measurement y~ = Q r of `cs.measure`.
* FP8 form: Q and r are each rounded to the OCP FP8 E4M3 ("e4m3fn") format,
  round to nearest, ties to even, and the products are summed exactly:
  y~8 = e4m3(Q) e4m3(r).  For integers of magnitude <= 448 every E4M3 value
  is itself an integer, so y~8 is an integer and, for n <= 2048, equal to its
  FP32 accumulation.  A per-block power-of-two scale of r would change
  nothing: |r| <= 255 is always in E4M3's normal range, whose relative
  spacing does not depend on the scale; the quantiser's per-block exponent is
  the block scale.

E4M3 (OCP 8-bit floating point specification): 1 sign bit, 4 exponent bits
with bias 7, 3 mantissa bits; normal values (1 + m/8) 2^(E-7) for E = 1..15
(E = 15 with m = 7 is NaN, so the largest finite value is 448), subnormal
values (m/8) 2^-6; no infinities.
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def e4m3_round(x) -> np.ndarray:
    """Nearest E4M3 value of each element (ties to even mantissa), as float64.
    Magnitudes above the largest finite value are rejected (they do not occur
    for residuals and measurement entries)."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    if np.any(a > E4M3_MAX):
        raise ValueError("value outside the finite E4M3 range")
    out = np.zeros_like(a)
    nz = a > 0
    # exponent of the binade, clamped to the smallest normal exponent -6:
    # below it the spacing is that of the subnormals, 2^-9
    e = np.floor(np.log2(np.where(nz, a, 1.0)))
    e = np.maximum(e, -6.0)
    step = np.exp2(e - 3.0)                     # 3 mantissa bits
    q = a / step                                # in [8, 16) for normals
    fl = np.floor(q)
    rem = q - fl
    up = (rem > 0.5) | ((rem == 0.5) & (np.mod(fl, 2.0) == 1.0))
    out = np.where(nz, (fl + up) * step, 0.0)
    return np.sign(x) * out


def split_int8(r: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """r = 16 h + l with l in [0, 15], h = floor(r / 16); both fit int8 for
    |r| <= 255."""
    r = np.asarray(r, dtype=np.int64)
    h = np.floor_divide(r, 16)
    l = r - 16 * h
    return h, l


def measure_int8(q: np.ndarray, r_cols: np.ndarray) -> np.ndarray:
    """int8 form: 16 (Q h) + Q l in exact integers (equals Q r)."""
    h, l = split_int8(r_cols)
    qi = q.astype(np.int64)
    return 16 * (qi @ h) + qi @ l


def measure_fp8(q: np.ndarray, r_cols: np.ndarray) -> np.ndarray:
    """FP8 form: e4m3(Q) e4m3(r), summed exactly (integers)."""
    q8 = e4m3_round(q.astype(np.float64))
    r8 = e4m3_round(r_cols.astype(np.float64))
    if not (np.all(q8 == np.round(q8)) and np.all(r8 == np.round(r8))):
        raise ValueError("E4M3 values of these integers are not integers")
    return q8.astype(np.int64) @ r8.astype(np.int64)
