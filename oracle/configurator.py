"""Parameter configurator: the application-aware configurable mechanism.

Test infrastructure (part of the FP64 CPU oracle): never imported by the
product path.

The paper lets the encoder choose the GOP size and the measurement matrix
size for what the application needs (Sections 2-3; Fig. 6 shows total CR
and PSNR against the CS frames' CR, Table I adds the tracking success rate).
The tracker is not part of this work, so the requirement is a PSNR floor.
For each candidate (G, M) the coder runs over a calibration clip:

* the clip of F frames is cut into consecutive GOPs of G frames; a final
  shorter GOP takes the remaining frames (Section 4 codes a key frame and
  four CS frames per GOP; a one-frame GOP is a key frame alone);
* total CR = 8 F H W / (key bits + CS bits) (Table I); key and CS CR over
  their own frames;
* PSNR of each decoded frame, 10 log10(255^2 H W / SSE) (99.99 dB when the
  frame is exact), averaged over all frames and over the CS frames;
* the choice is the candidate of largest total CR whose all-frame mean
  PSNR meets the floor; ties keep the earlier candidate (G-major order);
  -1 when none meets it.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import codec


@dataclass
class Point:
    gop: int
    m: int
    bits_key: int
    bits_cs: int
    cr_total: float
    cr_key: float
    cr_cs: float
    psnr_all: float
    psnr_cs: float
    meets_floor: bool


def frame_psnr(ref: np.ndarray, dec: np.ndarray) -> float:
    """PSNR of one uint8 frame from its exact integer sum of squared errors."""
    d = ref.astype(np.int64) - dec.astype(np.int64)
    sse = int(np.sum(d * d))
    return 99.99 if sse == 0 else 10.0 * np.log10(255.0 * 255.0 * ref.size / sse)


def evaluate(clip: np.ndarray, base: codec.Params, gop: int, m: int, floor_db: float) -> Point:
    """Encode and decode the clip with GOP size `gop` and M = `m`."""
    f_total, h, w = clip.shape
    bits_key = bits_cs = 0
    psnrs, cs_psnrs = [], []
    n_gops = 0
    for f0 in range(0, f_total, gop):
        g = min(gop, f_total - f0)
        p = codec.Params(**{**base.__dict__, "gop": g, "m": m, "height": h, "width": w})
        frames = clip[f0:f0 + g]
        gs = codec.encode_gop(frames, p)
        dec = codec.decode_gop(gs, p)
        bits_key += gs.bits_key
        bits_cs += gs.bits_cs
        n_gops += 1
        for t in range(g):
            ps = frame_psnr(frames[t], dec.frames[t])
            psnrs.append(ps)
            if t > 0:
                cs_psnrs.append(ps)
    raw_key = 8.0 * h * w * n_gops
    raw_cs = 8.0 * h * w * (f_total - n_gops)
    psnr_all = float(np.mean(psnrs))
    return Point(gop, m, bits_key, bits_cs, (raw_key + raw_cs) / (bits_key + bits_cs),
                 raw_key / bits_key, raw_cs / bits_cs if bits_cs else 0.0, psnr_all,
                 float(np.mean(cs_psnrs)) if cs_psnrs else 0.0, psnr_all >= floor_db)


def choose(points: list[Point]) -> int:
    """Index of the largest total CR among the points that meet the floor
    (first one on ties), or -1."""
    best = -1
    for i, p in enumerate(points):
        if p.meets_floor and (best < 0 or p.cr_total > points[best].cr_total):
            best = i
    return best


def configure(clip: np.ndarray, base: codec.Params, gops, ms, floor_db: float):
    """Sweep the candidates G-major and choose.  Returns (points, best)."""
    points = [evaluate(clip, base, g, m, floor_db) for g in gops for m in ms]
    return points, choose(points)
