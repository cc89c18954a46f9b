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

Decoding (eq. (1) with TVAL3, Section 4): each CS frame's residual is
recovered as one H x W image by the total-variation solver of oracle/tv.py
with Phi = s_Phi Q of size M x (H W), L = s_Phi^2 lambda_max(Q Q^T) from the
same FP64 power iteration as the block form, lam = frac ||Phi^T y^||_inf per
frame, and added to the decoded key frame (eq. (4)).
"""
from __future__ import annotations

import numpy as np

from . import cs, keyframe, philox, tv


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


def decode_gop(enc: dict, frames_shape, m: int, key_qstep: int, phi_seed: int, stream_id: int,
               iters: int, lambda_frac: float = 0.01):
    """Decoded frames (G x H x W uint8), the CS frames before rounding
    (G-1 x H x W), and per frame the FP64 TV objective, the relative residual
    ||Phi x - y^|| / ||y^|| and lam."""
    g, h, w = frames_shape
    n = h * w
    key_dec = keyframe.decode_levels(enc["key_levels"], key_qstep)
    q = philox.measurement_matrix_q(m, n, phi_seed, stream_id)
    s_phi = philox.phi_scale(m)
    phi = s_phi * q.astype(np.float64)
    L, _, _ = cs.lipschitz(q, s_phi)
    y = cs.dequantise(enc["codes"].T, enc["exps"], s_phi)        # M x (G-1)
    lam = tv.lambdas(phi, y, lambda_frac)
    x = tv.recover(phi, y, lam, L, (h, w), iters)                 # n x (G-1)
    frames = np.zeros((g, h, w), dtype=np.uint8)
    frames[0] = key_dec
    cs_f = key_dec.astype(np.float64)[None] + x.T.reshape(g - 1, h, w)
    frames[1:] = cs.round_to_u8(cs_f)
    obj = tv.objective(phi, y, x, lam, (h, w))
    r = phi @ x - y
    yn = np.sqrt(np.sum(y * y, axis=0))
    rel = np.where(yn > 0, np.sqrt(np.sum(r * r, axis=0)) / np.where(yn > 0, yn, 1.0), 0.0)
    return {"frames": frames, "cs_float": cs_f, "objective": obj, "rel_residual": rel,
            "lam": lam, "L": L}
