"""Synthetic surveillance video generator (numpy PCG64, fully seeded).

Recipe (each frame is uint8 luma, H rows x W columns):

* background: white N(0,1) field, Gaussian blur sigma=8 px (periodic edges),
  normalised to mean 110 and standard deviation 30; plus fine texture: a white
  N(0,1) field blurred with sigma=0.7 px, scaled to standard deviation 6;
* k objects, each a rectangle or an ellipse (probability 1/2), width and height
  each uniform on {10..30} px, constant intensity uniform on [30, 225] and
  redrawn while within 40 grey levels of the mean background under it, moving
  at a constant speed uniform on [1, 3] px/frame in a uniform direction and
  bouncing off the frame borders;
* per-pixel, per-frame sensor noise N(0, 2^2), then round half to even and clip
  to [0, 255].
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.ndimage import gaussian_filter


@dataclass(frozen=True)
class VideoSpec:
    height: int
    width: int
    n_frames: int
    n_objects: int
    seed: int
    noise_sigma: float = 2.0


def _background(rng: np.random.Generator, h: int, w: int) -> np.ndarray:
    smooth = gaussian_filter(rng.standard_normal((h, w)), 8.0, mode="wrap")
    smooth = (smooth - smooth.mean()) / smooth.std() * 30.0 + 110.0
    tex = gaussian_filter(rng.standard_normal((h, w)), 0.7, mode="wrap")
    tex = tex / tex.std() * 6.0
    return smooth + tex


class _Object:
    def __init__(self, rng: np.random.Generator, bg: np.ndarray):
        h, w = bg.shape
        self.ellipse = bool(rng.integers(0, 2))
        self.ow = int(rng.integers(10, 31))
        self.oh = int(rng.integers(10, 31))
        self.cx = float(rng.uniform(self.ow / 2, w - self.ow / 2))
        self.cy = float(rng.uniform(self.oh / 2, h - self.oh / 2))
        speed = float(rng.uniform(1.0, 3.0))
        ang = float(rng.uniform(0.0, 2.0 * np.pi))
        self.vx = speed * np.cos(ang)
        self.vy = speed * np.sin(ang)
        y0, y1, x0, x1 = self._box(h, w)
        local = float(bg[y0:y1, x0:x1].mean())
        inten = float(rng.uniform(30.0, 225.0))
        for _ in range(64):
            if abs(inten - local) >= 40.0:
                break
            inten = float(rng.uniform(30.0, 225.0))
        self.intensity = inten

    def _box(self, h: int, w: int):
        y0 = max(int(np.floor(self.cy - self.oh / 2)), 0)
        y1 = min(int(np.ceil(self.cy + self.oh / 2)) + 1, h)
        x0 = max(int(np.floor(self.cx - self.ow / 2)), 0)
        x1 = min(int(np.ceil(self.cx + self.ow / 2)) + 1, w)
        return y0, y1, x0, x1

    def draw(self, img: np.ndarray) -> None:
        h, w = img.shape
        y0, y1, x0, x1 = self._box(h, w)
        if y1 <= y0 or x1 <= x0:
            return
        yy, xx = np.mgrid[y0:y1, x0:x1]
        dy = (yy + 0.5 - self.cy) / (self.oh / 2)
        dx = (xx + 0.5 - self.cx) / (self.ow / 2)
        if self.ellipse:
            mask = dx * dx + dy * dy <= 1.0
        else:
            mask = (np.abs(dx) <= 1.0) & (np.abs(dy) <= 1.0)
        img[y0:y1, x0:x1][mask] = self.intensity

    def step(self, h: int, w: int) -> None:
        self.cx += self.vx
        self.cy += self.vy
        if self.cx - self.ow / 2 < 0 or self.cx + self.ow / 2 > w:
            self.vx = -self.vx
            self.cx = min(max(self.cx, self.ow / 2), w - self.ow / 2)
        if self.cy - self.oh / 2 < 0 or self.cy + self.oh / 2 > h:
            self.vy = -self.vy
            self.cy = min(max(self.cy, self.oh / 2), h - self.oh / 2)


def surveillance_video(spec: VideoSpec) -> np.ndarray:
    """Return a uint8 array of shape (n_frames, height, width)."""
    rng = np.random.default_rng(spec.seed)
    h, w = spec.height, spec.width
    bg = _background(rng, h, w)
    objs = [_Object(rng, bg) for _ in range(spec.n_objects)]
    out = np.empty((spec.n_frames, h, w), dtype=np.uint8)
    for t in range(spec.n_frames):
        img = bg.copy()
        for o in objs:
            o.draw(img)
        img += rng.normal(0.0, spec.noise_sigma, size=img.shape)
        out[t] = np.clip(np.rint(img), 0, 255).astype(np.uint8)
        for o in objs:
            o.step(h, w)
    return out
