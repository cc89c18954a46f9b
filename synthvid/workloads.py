"""Per-stream parameter recipes for the synthetic workloads.

Each workload family is named by what it is, with its sizes.  A stream is one
camera: frame size, GOP length G (key frame included), block size B, number
of measurements M per B x B block, FISTA iteration count, the seeds of its
video and of its measurement matrix.  Nothing here computes any part of the
coding method.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

from .video import VideoSpec, surveillance_video

# family ids used in seeds
FAMILY_QCIF_TINY = 1
FAMILY_CIF_SWEEP = 2
FAMILY_VGA_PRECISION = 3
FAMILY_MIXED = 4
FAMILY_SERVING = 5


def phi_key(family: int, stream: int) -> tuple[int, int]:
    """(phi_seed, stream_id) of a stream's measurement-matrix generator."""
    return (0x1311141900000000 | (family << 16) | stream) & (2**64 - 1), stream


def m_from_rho(rho: float, n: int) -> int:
    """Measurements per block for a target ratio M/n (round half up)."""
    return int(np.floor(rho * n + 0.5))


@dataclass(frozen=True)
class StreamSpec:
    height: int
    width: int
    gop: int
    block: int
    m: int
    iters: int
    phi_seed: int
    stream_id: int
    video_seed: int
    n_objects: int
    key_qstep: int = 16
    lambda_frac: float = 0.01

    @property
    def n(self) -> int:
        return self.block * self.block

    @property
    def rho(self) -> float:
        return self.m / self.n

    def video(self, n_frames: int | None = None) -> np.ndarray:
        nf = self.gop if n_frames is None else n_frames
        return surveillance_video(VideoSpec(self.height, self.width, nf,
                                            self.n_objects, self.video_seed))

    def with_(self, **kw) -> "StreamSpec":
        return replace(self, **kw)


def qcif_tiny(stream: int = 0) -> StreamSpec:
    """176x144, one GOP of 4 frames, B=16 (n=256), M=64, 200 iterations."""
    s, sid = phi_key(FAMILY_QCIF_TINY, stream)
    return StreamSpec(144, 176, 4, 16, 64, 200, s, sid,
                      1000 * FAMILY_QCIF_TINY + stream, 2)


def cif_sweep(gop: int = 4, rho: float = 0.25, stream: int = 0,
              iters: int = 300) -> StreamSpec:
    """352x288, B=16, GOP in {4,8,16}, M/n in {0.1,0.2,0.3,0.5}."""
    s, sid = phi_key(FAMILY_CIF_SWEEP, stream)
    k = 3 + (stream % 3)
    return StreamSpec(288, 352, gop, 16, m_from_rho(rho, 256), iters, s, sid,
                      1000 * FAMILY_CIF_SWEEP + stream, k)


def vga_precision(rho: float = 0.25, stream: int = 0, gop: int = 16,
                  iters: int = 300) -> StreamSpec:
    """640x480, GOP 16, B=32 (n=1024), M/n in {0.1, 0.25}."""
    s, sid = phi_key(FAMILY_VGA_PRECISION, stream)
    k = 3 + (stream % 3)
    return StreamSpec(480, 640, gop, 32, m_from_rho(rho, 1024), iters, s, sid,
                      1000 * FAMILY_VGA_PRECISION + stream, k)


def mixed_streams(n_streams: int = 64, iters: int = 300) -> list[StreamSpec]:
    """Mixed batch: sizes 176x144 / 352x288 / 640x480, GOP {4,8,16,32},
    M/n {0.05,0.1,0.2,0.4}, B {16,32}, each stream its own seed."""
    sizes = [(144, 176), (288, 352), (480, 640)]
    gops = [4, 8, 16, 32]
    rhos = [0.05, 0.1, 0.2, 0.4]
    blocks = [16, 32]
    out = []
    for st in range(n_streams):
        h, w = sizes[st % 3]
        b = blocks[(st // 16) % 2]
        s, sid = phi_key(FAMILY_MIXED, st)
        out.append(StreamSpec(h, w, gops[st % 4], b,
                              m_from_rho(rhos[(st // 4) % 4], b * b), iters,
                              s, sid, 1000 * FAMILY_MIXED + st,
                              3 + (st % 3)))
    return out


def serving_cameras(n_cameras: int = 256, iters: int = 300,
                    seed: int = 5) -> list[tuple[StreamSpec, float]]:
    """Serving mix: 640x480 / 1280x720 alternating, 1-8 objects, GOP from
    {8,16,32} and M/n from {0.1,0.25} cycled, B=16; each camera gets a
    Poisson GOP rate uniform on [2, 20] GOP/s.  Returns (spec, rate)."""
    rng = np.random.default_rng(seed)
    sizes = [(480, 640), (720, 1280)]
    gops = [8, 16, 32]
    rhos = [0.1, 0.25]
    out = []
    for c in range(n_cameras):
        h, w = sizes[c % 2]
        s, sid = phi_key(FAMILY_SERVING, c)
        k = int(rng.integers(1, 9))
        rate = float(rng.uniform(2.0, 20.0))
        out.append((StreamSpec(h, w, gops[c % 3], 16,
                               m_from_rho(rhos[(c // 3) % 2], 256), iters,
                               s, sid, 1000 * FAMILY_SERVING + c, k), rate))
    return out
