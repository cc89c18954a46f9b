"""Key-frame codec stand-in: integer 8x8 DCT, uniform step, Exp-Golomb bits.

Test infrastructure (part of the FP64 CPU oracle): never imported by the
product path.

The paper codes the key frame with a traditional intra codec (H.264 intra,
Sections 3.1 and 4) and needs only its decoded frame, which every CS frame of
the GOP subtracts (Section 3.2, eqs. (2)-(4)), and its bit count, which enters
the total compression ratio (Table I).  The stand-in is integer-defined so
that the decoded key frame, and every residual and code after it, is exactly
reproducible:

* T = round(2^10 C8), with C8[k, i] = a_k cos(pi (2i+1) k / 16),
  a_0 = sqrt(1/8), a_k = sqrt(2/8): the orthonormal 8-point DCT-II, scaled;
* forward: X = P - 128 per 8x8 block, Z = T X T^T (exact integers), and
  level = sgn(Z) * ((|Z| + 2^23) >> 24), i.e. Z / (step * 2^20) rounded half
  away from zero for step 16;
* inverse: V = T^T (step * level) T, decoded pixel
  clip(((V + 2^19) >> 20) + 128, 0, 255), with >> the floor shift;
* bits per 8x8 block, coefficients in zigzag order (anti-diagonals k+l = s
  from s = 0, walking with the row index decreasing on even s and increasing
  on odd s): ue(nnz), then ue(run of zeros before it) + se(level) per
  nonzero coefficient; ue(v) costs 2 floor(log2(v+1)) + 1 bits and
  se(v) = ue(2|v| - [v > 0]).

The quantiser rounding shift is written for a power-of-two step; any step
2^q is accepted (16 in every workload).
"""
from __future__ import annotations

import numpy as np


def dct_matrix(size: int) -> np.ndarray:
    """Orthonormal DCT-II matrix C[k, i] (float64)."""
    k = np.arange(size)[:, None]
    i = np.arange(size)[None, :]
    c = np.cos(np.pi * (2 * i + 1) * k / (2 * size))
    a = np.full((size, 1), np.sqrt(2.0 / size))
    a[0, 0] = np.sqrt(1.0 / size)
    return a * c


def int_dct8() -> np.ndarray:
    """T = round(2^10 C8) as int64 (no entry lies near a rounding tie)."""
    return np.rint(1024.0 * dct_matrix(8)).astype(np.int64)


def zigzag8() -> list[tuple[int, int]]:
    """Zigzag scan of an 8x8 block as (row, col) pairs."""
    order = []
    for s in range(15):
        rows = range(min(s, 7), max(0, s - 7) - 1, -1)
        if s % 2 == 1:
            rows = reversed(list(rows))
        for r in rows:
            order.append((r, s - r))
    return order


def _log2_shift(step: int) -> int:
    q = int(step).bit_length() - 1
    if step <= 0 or (1 << q) != step:
        raise ValueError("key quantiser step must be a power of two")
    return q


def ue_bits(v: int) -> int:
    """Length of the unsigned Exp-Golomb code of v >= 0."""
    return 2 * (int(v) + 1).bit_length() - 1


def se_bits(v: int) -> int:
    """Length of the signed Exp-Golomb code of v."""
    v = int(v)
    return ue_bits(2 * abs(v) - (1 if v > 0 else 0))


def encode_levels(frame: np.ndarray, step: int = 16) -> np.ndarray:
    """Quantised integer-DCT levels of an H x W uint8 frame (H, W multiples
    of 8).  Returns int64 levels, laid out like the frame (8x8 block of
    levels at the block's position, row index = vertical frequency)."""
    h, w = frame.shape
    if h % 8 or w % 8:
        raise ValueError("frame dimensions must be multiples of 8")
    t = int_dct8()
    shift = 20 + _log2_shift(step)
    half = 1 << (shift - 1)
    lev = np.zeros((h, w), dtype=np.int64)
    for by in range(0, h, 8):
        for bx in range(0, w, 8):
            x = frame[by:by + 8, bx:bx + 8].astype(np.int64) - 128
            z = t @ x @ t.T
            lev[by:by + 8, bx:bx + 8] = np.sign(z) * ((np.abs(z) + half) >> shift)
    return lev


def decode_levels(levels: np.ndarray, step: int = 16) -> np.ndarray:
    """Decoded key frame (uint8) from levels."""
    h, w = levels.shape
    t = int_dct8()
    out = np.zeros((h, w), dtype=np.uint8)
    for by in range(0, h, 8):
        for bx in range(0, w, 8):
            c = levels[by:by + 8, bx:bx + 8].astype(np.int64) * int(step)
            v = t.T @ c @ t
            p = ((v + (1 << 19)) >> 20) + 128
            out[by:by + 8, bx:bx + 8] = np.clip(p, 0, 255)
    return out


def block_bits(block_levels: np.ndarray) -> int:
    """Exp-Golomb bit count of one 8x8 block of levels."""
    seq = [int(block_levels[r, c]) for (r, c) in zigzag8()]
    nz = [i for i, v in enumerate(seq) if v != 0]
    bits = ue_bits(len(nz))
    prev = -1
    for i in nz:
        bits += ue_bits(i - prev - 1) + se_bits(seq[i])
        prev = i
    return bits


def frame_bits(levels: np.ndarray) -> int:
    h, w = levels.shape
    return sum(block_bits(levels[by:by + 8, bx:bx + 8])
               for by in range(0, h, 8) for bx in range(0, w, 8))
