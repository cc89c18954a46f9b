"""Whole-frame measurement: eq. (1) read literally.

Test infrastructure (part of the FP64 CPU oracle): never imported by the
product path.

The paper measures each CS frame as one vector x of all N = W H pixels
(Section 3.2, eq. (1): y = A x with A of size M x N).  Here the residual of a
whole frame (frame - decoded key frame, eqs. (2)-(3)) is measured by the
stream's matrix Q of size M x (W H) from the same counter generator as the
block form (entry (i, j) from the Philox block at counter (i W H + j) div 4
with second word W H), in exact integers, and quantised with the same
block-floating-point rule, the whole frame being one block:
y~_t = Q r_t, codes and one exponent per CS frame, 8 M + 8 bits per frame.
Q is defined entry by entry, so it never has to exist as a whole.
"""
from __future__ import annotations

import numpy as np

from . import cs, keyframe, philox


def measure(frames: np.ndarray, key_dec: np.ndarray, m: int, phi_seed: int,
            stream_id: int) -> np.ndarray:
    """y~ (G-1 x M, int64) of the CS frames 1..G-1 against the decoded key."""
    g, h, w = frames.shape
    n = h * w
    r = (frames[1:].astype(np.int64) - key_dec.astype(np.int64)[None]).reshape(g - 1, n).T
    q = philox.measurement_matrix_q(m, n, phi_seed, stream_id)
    # exact: |entries| < 2^53 in float64
    return np.rint(q.astype(np.float64) @ r.astype(np.float64)).astype(np.int64).T


def measure_rows(frames: np.ndarray, key_dec: np.ndarray, rows, phi_seed: int,
                 stream_id: int) -> np.ndarray:
    """Selected measurements y~[t, rows] (G-1 x len(rows)), from those rows
    of Q alone."""
    g, h, w = frames.shape
    n = h * w
    r = (frames[1:].astype(np.int64) - key_dec.astype(np.int64)[None]).reshape(g - 1, n)
    q = philox.measurement_rows_q(rows, n, phi_seed, stream_id)
    return r @ q.T


def encode_gop(frames: np.ndarray, m: int, key_qstep: int, phi_seed: int, stream_id: int):
    """Key levels and bits, y~, codes (G-1 x M) and exponents (G-1) of one
    GOP with whole-frame measurement."""
    lev = keyframe.encode_levels(frames[0], key_qstep)
    key_dec = keyframe.decode_levels(lev, key_qstep)
    y = measure(frames, key_dec, m, phi_seed, stream_id)
    codes, exps = cs.quantise(y.T)          # one column (block) per CS frame
    g = frames.shape[0]
    return {"key_levels": lev, "key_decoded": key_dec, "bits_key": keyframe.frame_bits(lev),
            "bits_cs": (g - 1) * (8 * m + 8), "y_int": y, "codes": codes.T, "exps": exps}
