"""GOP-level encoder and decoder of the multiple-residual CS video coder.

Test infrastructure (part of the FP64 CPU oracle): never imported by the
product path.

Encoder (Section 3.1, Fig. 3): frame 0 of the GOP is the key frame, coded by
the intra stand-in; every other frame t subtracts the *decoded* key frame
(closed loop, Section 3.2 eqs. (2)-(3)): R_t = F_t - F^_key, and its blocks
are measured and quantised.  Decoder (Section 3.2, Fig. 4): the key frame is
decoded first, then each CS frame's residual is recovered and added back to
the decoded key frame (eq. (4)).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import cs, fp8, keyframe, philox, tv


@dataclass(frozen=True)
class Params:
    height: int
    width: int
    gop: int
    block: int
    m: int
    phi_seed: int
    stream_id: int
    iters: int = 300
    key_qstep: int = 16
    lambda_frac: float = 0.01
    solver: str = "fista"           # fista | ista | mfista | direct | tv
    pixel_domain_lambda: bool = False
    no_quant: bool = False          # test hook: y^ = s_Phi y~ exactly
    measure_form: str = "exact"     # exact | int8 | fp8 (encoder product, see fp8.py)

    @property
    def n(self) -> int:
        return self.block * self.block

    @staticmethod
    def from_spec(spec, **kw) -> "Params":
        base = dict(height=spec.height, width=spec.width, gop=spec.gop,
                    block=spec.block, m=spec.m, phi_seed=spec.phi_seed,
                    stream_id=spec.stream_id, iters=spec.iters,
                    key_qstep=spec.key_qstep, lambda_frac=spec.lambda_frac)
        base.update(kw)
        return Params(**base)


@dataclass
class GopStream:
    key_levels: np.ndarray          # int64 H x W
    codes: np.ndarray               # int8 (G-1) x N_b x M
    exps: np.ndarray                # uint8 (G-1) x N_b
    bits_key: int
    bits_cs: int
    key_decoded: np.ndarray = field(repr=False, default=None)   # uint8 H x W
    y_int: np.ndarray = field(repr=False, default=None)         # int64 (G-1) x N_b x M


def encode_gop(frames: np.ndarray, p: Params) -> GopStream:
    g, h, w = frames.shape
    if g != p.gop or (h, w) != (p.height, p.width):
        raise ValueError("frames do not match the parameters")
    lev = keyframe.encode_levels(frames[0], p.key_qstep)
    key_dec = keyframe.decode_levels(lev, p.key_qstep)
    bits_key = keyframe.frame_bits(lev)
    q = philox.measurement_matrix_q(p.m, p.n, p.phi_seed, p.stream_id)
    nby, nbx = cs.blocks_shape(h, w, p.block)
    nb = nby * nbx
    codes = np.zeros((g - 1, nb, p.m), dtype=np.int8)
    exps = np.zeros((g - 1, nb), dtype=np.uint8)
    y_all = np.zeros((g - 1, nb, p.m), dtype=np.int64)
    for t in range(1, g):
        res = frames[t].astype(np.int64) - key_dec.astype(np.int64)
        r_cols = cs.gather_blocks(res, p.block)
        if p.measure_form == "exact":
            y_int = cs.measure(q, r_cols)
        elif p.measure_form == "int8":
            y_int = fp8.measure_int8(q, r_cols)
        elif p.measure_form == "fp8":
            y_int = fp8.measure_fp8(q, r_cols)
        else:
            raise ValueError(f"unknown measurement form {p.measure_form!r}")
        c, e = cs.quantise(y_int)
        codes[t - 1] = c.T
        exps[t - 1] = e
        y_all[t - 1] = y_int.T
    bits_cs = (g - 1) * nb * (8 * p.m + 8)
    return GopStream(lev, codes, exps, bits_key, bits_cs, key_dec, y_all)


@dataclass
class Decoded:
    frames: np.ndarray              # uint8 G x H x W (frame 0 = decoded key)
    cs_float: np.ndarray            # float64 (G-1) x H x W
    objective: np.ndarray           # float64 (G-1) x N_b
    rel_residual: np.ndarray        # float64 (G-1) x N_b
    lam: np.ndarray                 # float64 (G-1) x N_b
    L: float
    s: np.ndarray                   # float64 (G-1) x N_b x n


def decode_gop(gs: GopStream, p: Params) -> Decoded:
    h, w, g, b = p.height, p.width, p.gop, p.block
    key_dec = keyframe.decode_levels(gs.key_levels, p.key_qstep)
    q = philox.measurement_matrix_q(p.m, p.n, p.phi_seed, p.stream_id)
    s_phi = philox.phi_scale(p.m)
    a = cs.operator(q, s_phi, b)
    L, _, _ = cs.lipschitz(q, s_phi)
    nb = gs.codes.shape[1]
    frames = np.zeros((g, h, w), dtype=np.uint8)
    frames[0] = key_dec
    cs_f = np.zeros((g - 1, h, w))
    obj = np.zeros((g - 1, nb))
    relr = np.zeros((g - 1, nb))
    lam_all = np.zeros((g - 1, nb))
    s_all = np.zeros((g - 1, nb, p.n))
    for t in range(1, g):
        if p.no_quant:
            y_hat = s_phi * gs.y_int[t - 1].T.astype(np.float64)
        else:
            y_hat = cs.dequantise(gs.codes[t - 1].T, gs.exps[t - 1], s_phi)
        if p.solver == "tv":
            # total-variation recovery in the pixel domain (oracle/tv.py);
            # s holds the pixel-domain residual x, the objective is TV's
            phi = s_phi * q.astype(np.float64)
            lam = tv.lambdas(phi, y_hat, p.lambda_frac)
            xr = tv.recover(phi, y_hat, lam, L, b, p.iters)
            f = key_dec.astype(np.float64) + cs.scatter_blocks(xr, h, w, b)
            cs_f[t - 1] = f
            frames[t] = cs.round_to_u8(f)
            obj[t - 1] = tv.objective(phi, y_hat, xr, lam, b)
            rn = np.linalg.norm(phi @ xr - y_hat, axis=0)
            yn = np.linalg.norm(y_hat, axis=0)
            relr[t - 1] = np.where(yn > 0, rn / np.where(yn > 0, yn, 1.0), 0.0)
            lam_all[t - 1] = lam
            s_all[t - 1] = xr.T
            continue
        if p.solver == "direct":
            # least squares on a square operator (M = n, lam = 0)
            s = np.linalg.solve(a, y_hat)
            lam = np.zeros(nb)
        else:
            lam = cs.lambdas(a, y_hat, p.lambda_frac, p.pixel_domain_lambda,
                             s_phi * q.astype(np.float64))
            solver = {"fista": cs.fista, "ista": cs.ista, "mfista": cs.mfista}[p.solver]
            s = solver(a, y_hat, lam, L, p.iters)
        x = cs.synthesise(s, b)
        f = key_dec.astype(np.float64) + cs.scatter_blocks(x, h, w, b)
        cs_f[t - 1] = f
        frames[t] = cs.round_to_u8(f)
        obj[t - 1] = cs.objective(a, y_hat, s, lam)
        rn = np.linalg.norm(a @ s - y_hat, axis=0)
        yn = np.linalg.norm(y_hat, axis=0)
        relr[t - 1] = np.where(yn > 0, rn / np.where(yn > 0, yn, 1.0), 0.0)
        lam_all[t - 1] = lam
        s_all[t - 1] = s.T
    return Decoded(frames, cs_f, obj, relr, lam_all, L, s_all)


# ---------------------------------------------------------------- metrics

def psnr(ref: np.ndarray, test: np.ndarray) -> float:
    """8-bit PSNR in dB; identical frames give 99.99."""
    d = ref.astype(np.float64) - test.astype(np.float64)
    mse = float(np.mean(d * d))
    return 99.99 if mse == 0 else 10.0 * np.log10(255.0 ** 2 / mse)


def total_cr_from_ratios(gop: int, cr_key: float, cr_cs: float) -> float:
    """Total compression ratio of a GOP of one key frame and G-1 CS frames
    whose frames compress by cr_key and cr_cs: raw bits over coded bits."""
    return gop / (1.0 / cr_key + (gop - 1) / cr_cs)


def cr_from_bits(p: Params, bits_key: int, bits_cs: int) -> dict:
    raw = 8 * p.height * p.width
    return {"total": p.gop * raw / (bits_key + bits_cs),
            "key": raw / bits_key,
            "cs": (p.gop - 1) * raw / bits_cs if bits_cs else float("inf")}
