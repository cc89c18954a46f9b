"""Pins of the oracle's GOP encoder/decoder: Table I's compression ratios,
the closed-loop invariant of eqs. (2)-(4), and end-to-end sanity on the
tiny QCIF workload."""
import os

import numpy as np
import pytest

import synthvid as sv
from oracle import codec, keyframe

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_total_cr.txt")


def _table1():
    rows = []
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            cr, g, k, c = line.split()
            rows.append((float(cr), int(g), float(k), float(c)))
    return rows


def test_table1_total_cr_reproduced():
    rows = _table1()
    assert len(rows) == 9
    for (cr, g, k, c) in rows:
        assert round(codec.total_cr_from_ratios(g, k, c), 2) == cr


def test_cr_from_bits_obeys_the_same_identity():
    spec = sv.qcif_tiny()
    p = codec.Params.from_spec(spec)
    gs = codec.encode_gop(spec.video(), p)
    cr = codec.cr_from_bits(p, gs.bits_key, gs.bits_cs)
    assert cr["total"] == pytest.approx(codec.total_cr_from_ratios(p.gop, cr["key"], cr["cs"]), rel=1e-12)
    nb = 9 * 11
    assert gs.bits_cs == (p.gop - 1) * nb * (8 * p.m + 8)
    assert gs.bits_key == keyframe.frame_bits(gs.key_levels)


@pytest.mark.parametrize("step", [16, 32, 64])
def test_closed_loop_cancels_key_frame_error(step):
    """Eq. (4): with exact measurements of a square operator and a direct
    solve, the decoded CS frame equals the source frame whatever the key
    coding error; the open-loop residual (vs the source key) would leave
    exactly the key error F^_key - F_key."""
    spec = sv.qcif_tiny().with_(height=32, width=48, block=4, m=16, gop=3)
    frames = spec.video()
    p = codec.Params.from_spec(spec, key_qstep=step, no_quant=True, solver="direct")
    gs = codec.encode_gop(frames, p)
    dec = codec.decode_gop(gs, p)
    key_err = gs.key_decoded.astype(np.float64) - frames[0]
    assert np.abs(key_err).max() > 0
    for t in (1, 2):
        assert np.max(np.abs(dec.cs_float[t - 1] - frames[t])) < 1e-9
        assert np.array_equal(dec.frames[t], frames[t])
        # open-loop control: recover F_t - F_key and add the decoded key
        open_loop = gs.key_decoded.astype(np.float64) + (frames[t].astype(np.float64) - frames[0])
        assert np.allclose(open_loop - frames[t], key_err)


def test_all_cs_frames_use_the_same_decoded_key():
    spec = sv.qcif_tiny().with_(gop=4)
    frames = spec.video()
    p = codec.Params.from_spec(spec, no_quant=True, iters=1)
    gs = codec.encode_gop(frames, p)
    from oracle import cs, philox
    q = philox.measurement_matrix_q(p.m, p.n, p.phi_seed, p.stream_id)
    for t in range(1, 4):
        res = frames[t].astype(np.int64) - gs.key_decoded
        assert np.array_equal(gs.y_int[t - 1], cs.measure(q, cs.gather_blocks(res, p.block)).T)


def test_tiny_end_to_end_quality():
    spec = sv.qcif_tiny()
    frames = spec.video()
    p = codec.Params.from_spec(spec)
    gs = codec.encode_gop(frames, p)
    dec = codec.decode_gop(gs, p)
    assert np.array_equal(dec.frames[0], gs.key_decoded)
    for t in range(1, p.gop):
        rec = codec.psnr(frames[t], dec.frames[t])
        key_only = codec.psnr(frames[t], gs.key_decoded)
        assert rec > key_only
        assert rec > 25.0
    assert np.all(dec.objective > 0) and np.all(dec.rel_residual < 1.0)


def test_lambda_scales_with_its_fraction():
    """lambda_b = frac * ||A^T y^_b||_inf is linear in frac: decoding the
    same stream with three times the fraction gives exactly three times every
    lambda, and a different recovery (a larger threshold), for the l1 and the
    TV solver alike."""
    spec = sv.qcif_tiny().with_(gop=2, iters=60)
    frames = spec.video()
    for solver in ("fista", "tv"):
        p1 = codec.Params.from_spec(spec, lambda_frac=0.01, solver=solver)
        p3 = codec.Params.from_spec(spec, lambda_frac=0.03, solver=solver)
        gs = codec.encode_gop(frames, p1)
        d1, d3 = codec.decode_gop(gs, p1), codec.decode_gop(gs, p3)
        assert np.all(d1.lam > 0)
        assert np.allclose(d3.lam, 3.0 * d1.lam, rtol=1e-12, atol=0)
        assert not np.array_equal(d1.cs_float, d3.cs_float)
