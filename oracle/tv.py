"""Total-variation recovery of a block residual, in the style of TVAL3.

Test infrastructure (part of the FP64 CPU oracle): never imported by the
product path.

The paper reconstructs its CS frames with TVAL3 (Section 4, reference [14]:
Li, Yin, Jiang and Zhang, an augmented Lagrangian method for total-variation
minimisation).  TVAL3 splits w_i = D_i x (D_i x the two forward differences at
pixel i), minimises the augmented Lagrangian alternately over w (a closed-
form 2-D shrinkage) and x (a gradient step), and updates the multipliers.
This module solves the penalised problem of eq. (1) with a TV regulariser,
per B x B block in the pixel domain (x = the residual block, A = Phi):

    min_x  lam TV(x) + 1/2 ||Phi x - y^||^2,   TV(x) = sum_i ||D_i x||_2

(isotropic TV; the penalised form because quantised measurements make
Phi x = y^ unattainable, as for the LASSO reading), by the linearised
alternating-direction iteration: x_0 = 0, nu_0 = 0, and for k = 1..T

    w    = shrink(D x + nu / beta, lam / beta)        (per pixel, 2-vectors)
    x   <- x - alpha (Phi^T (Phi x - y^) + D^T (nu + beta (D x - w)))
    nu  <- nu + beta (D x - w)                        (with the new x)

with shrink(v, t) = max(||v|| - t, 0) v / ||v||, alpha = 1 / (L + 8 beta),
L = ||Phi||^2 (the step constant of the LASSO path: ||Phi Psi|| = ||Phi||)
and ||D||^2 <= 8.  One gradient step replaces TVAL3's inner loop with its
Barzilai-Borwein step and non-monotone line search, so that every iterate is
fixed by the data alone.  Parameters: lam_b = frac ||Phi^T y^_b||_inf per
block and beta_b = 0.03 lam_b (1 where lam_b = 0).

D: horizontal and vertical forward differences inside the block with a zero
difference across the last column and the last row (Neumann boundary).  The
same functions take a whole H x W frame as one column when b = (H, W) (the
whole-frame reading of eq. (1), oracle/whole.py).
"""
from __future__ import annotations

import numpy as np

BETA_RATIO = 0.03


def _hw(b) -> tuple[int, int]:
    """Image shape of a column: b (a B x B block) or (height, width)."""
    return (b, b) if isinstance(b, (int, np.integer)) else (int(b[0]), int(b[1]))


def grad(x: np.ndarray, b) -> tuple[np.ndarray, np.ndarray]:
    """D x for image columns x (n x N; each a B x B block, or an H x W frame
    when b = (H, W)): horizontal and vertical differences."""
    hh, ww = _hw(b)
    X = x.reshape(hh, ww, -1)
    dh = np.zeros_like(X)
    dv = np.zeros_like(X)
    dh[:, :-1] = X[:, 1:] - X[:, :-1]
    dv[:-1, :] = X[1:, :] - X[:-1, :]
    return dh.reshape(hh * ww, -1), dv.reshape(hh * ww, -1)


def grad_adj(ph: np.ndarray, pv: np.ndarray, b) -> np.ndarray:
    """D^T (ph, pv): the adjoint of `grad`."""
    hh, ww = _hw(b)
    Ph = ph.reshape(hh, ww, -1)
    Pv = pv.reshape(hh, ww, -1)
    out = np.zeros_like(Ph)
    out[:, :-1] -= Ph[:, :-1]
    out[:, 1:] += Ph[:, :-1]
    out[:-1, :] -= Pv[:-1, :]
    out[1:, :] += Pv[:-1, :]
    return out.reshape(hh * ww, -1)


def tv_norm(x: np.ndarray, b) -> np.ndarray:
    """Isotropic TV of each block column."""
    dh, dv = grad(x, b)
    return np.sum(np.sqrt(dh * dh + dv * dv), axis=0)


def objective(phi: np.ndarray, y: np.ndarray, x: np.ndarray, lam: np.ndarray, b) -> np.ndarray:
    r = phi @ x - y
    return 0.5 * np.sum(r * r, axis=0) + lam * tv_norm(x, b)


def betas(lam: np.ndarray) -> np.ndarray:
    return np.where(lam > 0, BETA_RATIO * lam, 1.0)


def recover(phi: np.ndarray, y: np.ndarray, lam: np.ndarray, L: float, b, iters: int,
            return_dual: bool = False):
    """The iteration of the module docstring; x (n x N) and optionally the
    multipliers (nu_h, nu_v)."""
    n, nb = phi.shape[1], y.shape[1]
    beta = betas(lam)
    alpha = 1.0 / (L + 8.0 * beta)
    x = np.zeros((n, nb))
    nh = np.zeros((n, nb))
    nv = np.zeros((n, nb))
    for _ in range(iters):
        dh, dv = grad(x, b)
        vh = dh + nh / beta
        vv = dv + nv / beta
        mag = np.sqrt(vh * vh + vv * vv)
        sc = np.where(mag > 0, np.maximum(mag - lam / beta, 0.0) / np.where(mag > 0, mag, 1.0), 0.0)
        wh = sc * vh
        wv = sc * vv
        g = phi.T @ (phi @ x - y) + grad_adj(nh + beta * (dh - wh), nv + beta * (dv - wv), b)
        x = x - alpha * g
        dh, dv = grad(x, b)
        nh = nh + beta * (dh - wh)
        nv = nv + beta * (dv - wv)
    return (x, nh, nv) if return_dual else x


def lambdas(phi: np.ndarray, y: np.ndarray, frac: float) -> np.ndarray:
    """lam_b = frac ||Phi^T y^_b||_inf."""
    return frac * np.max(np.abs(phi.T @ y), axis=0)
