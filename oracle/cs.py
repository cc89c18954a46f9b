"""Compressive-sensing steps of the multiple-residual coder, in FP64.

Test infrastructure (part of the FP64 CPU oracle): never imported by the
product path.  Blocks are matrix columns: a residual of N_b blocks of n = B^2
pixels is an n x N_b matrix.

Readings of the paper (which measures and recovers whole frames with a
Gaussian matrix and TVAL3, Sections 3.2 and 4, and leaves the regulariser of
eq. (1) open):

* block-based sensing: each B x B block of a CS-frame residual is a signal
  x in R^n, n = B^2, vectorised row-major; blocks are numbered row-major over
  the frame; the residual is zero-padded up to whole blocks;
* measurement in integers: y~ = Q r with Q from the counter generator and r
  the integer residual; the real measurements are y = s_Phi y~;
* 8-bit block-floating-point quantiser, per block: m = max|y~|, the smallest
  e >= 0 with (m + h(e)) >> e <= 127 where h(0) = 0, h(e) = 2^(e-1), codes
  c = sgn(y~) ((|y~| + h(e)) >> e); the decoder uses y^ = s_Phi c 2^e;
* eq. (1) relaxed to the LASSO  min_s 1/2 ||A s - y^||^2 + lam ||s||_1  with
  A = Phi Psi, Psi the orthonormal 2-D DCT-II synthesis (x = Psi s  <=>
  X = C^T S C) and lam = frac * ||A^T y^||_inf per block;
* FISTA (Beck and Teboulle 2009) with constant step 1/L, L = 1.001 s_Phi^2
  lambda_max(Q Q^T) from a power iteration; MFISTA (its monotone variant,
  Beck and Teboulle, IEEE TIP 2009) and ISTA for checks;
* synthesis x^ = Psi s^ added to the decoded key frame (eq. (4)).
"""
from __future__ import annotations

import numpy as np

from .keyframe import dct_matrix


# ---------------------------------------------------------------- blocking

def blocks_shape(h: int, w: int, b: int) -> tuple[int, int]:
    """(blocks down, blocks across) after zero padding to whole blocks."""
    return (h + b - 1) // b, (w + b - 1) // b


def gather_blocks(res: np.ndarray, b: int) -> np.ndarray:
    """H x W residual -> n x N_b matrix (zero padding at the right/bottom)."""
    h, w = res.shape
    nby, nbx = blocks_shape(h, w, b)
    pad = np.zeros((nby * b, nbx * b), dtype=np.int64)
    pad[:h, :w] = res
    cols = np.empty((b * b, nby * nbx), dtype=np.int64)
    for by in range(nby):
        for bx in range(nbx):
            cols[:, by * nbx + bx] = pad[by * b:(by + 1) * b, bx * b:(bx + 1) * b].reshape(-1)
    return cols


def scatter_blocks(cols: np.ndarray, h: int, w: int, b: int) -> np.ndarray:
    """n x N_b block columns -> H x W frame (padding dropped)."""
    nby, nbx = blocks_shape(h, w, b)
    pad = np.zeros((nby * b, nbx * b), dtype=cols.dtype)
    for by in range(nby):
        for bx in range(nbx):
            pad[by * b:(by + 1) * b, bx * b:(bx + 1) * b] = cols[:, by * nbx + bx].reshape(b, b)
    return pad[:h, :w]


# ---------------------------------------------------------- measurement

def measure(q: np.ndarray, r_cols: np.ndarray) -> np.ndarray:
    """Exact integer measurements y~ = Q r (M x N_b, int64)."""
    return q.astype(np.int64) @ r_cols.astype(np.int64)


def quantise(y_int: np.ndarray):
    """Block-floating-point 8-bit codes.  Returns (codes int8 M x N_b,
    exps uint8 N_b)."""
    m_rows, nb = y_int.shape
    codes = np.zeros((m_rows, nb), dtype=np.int8)
    exps = np.zeros(nb, dtype=np.uint8)
    for j in range(nb):
        col = y_int[:, j]
        mx = int(np.max(np.abs(col))) if m_rows else 0
        e = 0
        while ((mx + (1 << (e - 1) if e else 0)) >> e) > 127:
            e += 1
        h = (1 << (e - 1)) if e else 0
        codes[:, j] = np.sign(col) * ((np.abs(col) + h) >> e)
        exps[j] = e
    return codes, exps


def dequantise(codes: np.ndarray, exps: np.ndarray, s_phi: float) -> np.ndarray:
    """y^ = s_Phi c 2^e (FP64, M x N_b)."""
    return s_phi * codes.astype(np.float64) * np.exp2(exps.astype(np.float64))[None, :]


# ---------------------------------------------------------------- basis

def synthesis_basis(b: int) -> np.ndarray:
    """Psi (n x n) with x = Psi s  <=>  X = C^T S C (row-major vec)."""
    c = dct_matrix(b)
    return np.kron(c.T, c.T)


def operator(q: np.ndarray, s_phi: float, b: int) -> np.ndarray:
    """A = Phi Psi = s_Phi Q Psi (FP64, M x n)."""
    return (s_phi * q.astype(np.float64)) @ synthesis_basis(b)


def lipschitz(q: np.ndarray, s_phi: float, tol: float = 1e-12,
              max_iter: int = 10000, safety: float = 1.001):
    """Step constant from an FP64 power iteration on the integer Gram Q Q^T.

    v0 = 1/sqrt(M) (all ones); each step forms w = G v, the Rayleigh quotient
    rq = v.w, stops once |rq - rq_prev| <= tol * rq, else v = w / ||w||.
    Returns (L_used = safety * s_Phi^2 * rq, rq, iterations)."""
    g = q.astype(np.float64) @ q.astype(np.float64).T
    m = g.shape[0]
    v = np.full(m, 1.0 / np.sqrt(m))
    rq_prev = 0.0
    rq = 0.0
    it = 0
    for it in range(1, max_iter + 1):
        w = g @ v
        rq = float(v @ w)
        if it > 1 and abs(rq - rq_prev) <= tol * rq:
            break
        rq_prev = rq
        nw = float(np.linalg.norm(w))
        if nw == 0.0:
            break
        v = w / nw
    return safety * s_phi * s_phi * rq, rq, it


def lambdas(a: np.ndarray, y_hat: np.ndarray, frac: float = 0.01,
            pixel_domain: bool = False, phi: np.ndarray | None = None) -> np.ndarray:
    """lam_b = frac * ||A^T y^_b||_inf (or ||Phi^T y^_b||_inf if asked)."""
    op = phi if pixel_domain else a
    return frac * np.max(np.abs(op.T @ y_hat), axis=0)


# ------------------------------------------------------------- recovery

def soft(u: np.ndarray, tau) -> np.ndarray:
    """Soft threshold: sgn(u) max(|u| - tau, 0)."""
    return np.sign(u) * np.maximum(np.abs(u) - tau, 0.0)


def objective(a: np.ndarray, y_hat: np.ndarray, s: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """Per-block F(s) = 1/2 ||A s - y^||^2 + lam ||s||_1."""
    r = a @ s - y_hat
    return 0.5 * np.sum(r * r, axis=0) + lam * np.sum(np.abs(s), axis=0)


def fista(a, y_hat, lam, L, iters, history=False):
    """Constant-step FISTA from s_0 = 0: for k = 1..T,
    s_k = soft(v_k - A^T(A v_k - y^)/L, lam/L),
    t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2,
    v_{k+1} = s_k + ((t_k - 1)/t_{k+1}) (s_k - s_{k-1});  v_1 = s_0, t_1 = 1."""
    n = a.shape[1]
    s_prev = np.zeros((n, y_hat.shape[1]))
    v = s_prev.copy()
    t = 1.0
    hist = []
    tau = lam / L
    for _ in range(iters):
        g = a.T @ (a @ v - y_hat)
        s = soft(v - g / L, tau)
        t_next = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        v = s + ((t - 1.0) / t_next) * (s - s_prev)
        s_prev, t = s, t_next
        if history:
            hist.append(objective(a, y_hat, s, lam))
    return (s_prev, hist) if history else s_prev


def ista(a, y_hat, lam, L, iters, history=False):
    """Proximal gradient without momentum: s_k = soft(s_{k-1} - grad/L)."""
    s = np.zeros((a.shape[1], y_hat.shape[1]))
    hist = []
    for _ in range(iters):
        s = soft(s - a.T @ (a @ s - y_hat) / L, lam / L)
        if history:
            hist.append(objective(a, y_hat, s, lam))
    return (s, hist) if history else s


def mfista(a, y_hat, lam, L, iters, history=False, iterates=False):
    """Monotone FISTA: z_k = prox step from v_k; s_k = z_k if F(z_k) <= F(s_{k-1})
    else s_{k-1} (per block); v_{k+1} = s_k + (t_k/t_{k+1})(z_k - s_k)
    + ((t_k - 1)/t_{k+1})(s_k - s_{k-1}).  With iterates=True the list of
    (v_k, z_k, s_k), k = 1..T, is returned as well (for the pins)."""
    n, nb = a.shape[1], y_hat.shape[1]
    s_prev = np.zeros((n, nb))
    v = s_prev.copy()
    t = 1.0
    f_prev = objective(a, y_hat, s_prev, lam)
    hist = []
    its = []
    for _ in range(iters):
        v_k = v
        z = soft(v - a.T @ (a @ v - y_hat) / L, lam / L)
        fz = objective(a, y_hat, z, lam)
        take = fz <= f_prev
        s = np.where(take[None, :], z, s_prev)
        f_s = np.where(take, fz, f_prev)
        t_next = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        v = s + (t / t_next) * (z - s) + ((t - 1.0) / t_next) * (s - s_prev)
        s_prev, f_prev, t = s, f_s, t_next
        if history:
            hist.append(f_s.copy())
        if iterates:
            its.append((v_k, z, s))
    out = (s_prev,)
    if history:
        out += (hist,)
    if iterates:
        out += (its,)
    return out if len(out) > 1 else s_prev


# ------------------------------------------------------------ synthesis

def synthesise(s_cols: np.ndarray, b: int) -> np.ndarray:
    """Pixel-domain residual blocks x^ = Psi s^ via X = C^T S C per block."""
    c = dct_matrix(b)
    out = np.empty_like(s_cols, dtype=np.float64)
    for j in range(s_cols.shape[1]):
        out[:, j] = (c.T @ s_cols[:, j].reshape(b, b) @ c).reshape(-1)
    return out


def round_to_u8(f: np.ndarray) -> np.ndarray:
    """clip(round-half-even(f), 0, 255) as uint8."""
    return np.clip(np.rint(f), 0, 255).astype(np.uint8)
