"""Pins of the oracle's whole-frame measurement (eq. (1) literal): the row
sampler against the full generator, linearity and the integer bound, and the
reduction to the block form when a frame is a single block."""
import numpy as np

import synthvid as sv
from oracle import codec, cs, keyframe, philox, whole


def test_rows_equal_full_matrix():
    q = philox.measurement_matrix_q(37, 104, 9, 4)
    rows = [0, 5, 36, 17]
    assert np.array_equal(philox.measurement_rows_q(rows, 104, 9, 4), q[rows])


def test_single_block_frame_equals_block_form():
    # a 16 x 16 frame is one block of B = 16: the whole-frame and block
    # measurements coincide (same counter layout, n = 256)
    rng = np.random.default_rng(1)
    frames = rng.integers(0, 256, size=(3, 16, 16), dtype=np.uint8)
    lev = keyframe.encode_levels(frames[0], 16)
    key = keyframe.decode_levels(lev, 16)
    y = whole.measure(frames, key, 40, 11, 2)
    q = philox.measurement_matrix_q(40, 256, 11, 2)
    for t in (1, 2):
        r = cs.gather_blocks(frames[t].astype(np.int64) - key.astype(np.int64), 16)
        assert np.array_equal(y[t - 1], cs.measure(q, r)[:, 0])


def test_linearity_bound_and_sampled_rows():
    spec = sv.qcif_tiny().with_(gop=3)
    frames = spec.video()
    lev = keyframe.encode_levels(frames[0], 16)
    key = keyframe.decode_levels(lev, 16)
    m = 300
    y = whole.measure(frames, key, m, 5, 1)
    n = 176 * 144
    r = frames[1:].astype(np.int64) - key.astype(np.int64)[None]
    assert np.all(np.abs(y) <= 32 * np.abs(r).reshape(2, -1).sum(axis=1)[:, None])
    rows = [0, 7, 299, 150]
    assert np.array_equal(whole.measure_rows(frames, key, rows, 5, 1), y[:, rows])
    # linearity in the residual: doubling the CS frames' residual doubles y~
    q = philox.measurement_matrix_q(m, n, 5, 1)
    assert np.array_equal(q @ (2 * r.reshape(2, -1).T), 2 * y.T)


def test_encode_gop_bits():
    spec = sv.qcif_tiny().with_(gop=4)
    frames = spec.video()
    e = whole.encode_gop(frames, 500, 16, 3, 0)
    assert e["codes"].shape == (3, 500) and e["exps"].shape == (3,)
    assert e["bits_cs"] == 3 * (8 * 500 + 8)
    ref = codec.encode_gop(frames, codec.Params.from_spec(spec))
    assert e["bits_key"] == ref.bits_key
    # the quantiser: largest code magnitude is 127 when y~ != 0
    assert np.abs(e["codes"].astype(np.int64)).max() <= 127


def test_rectangular_grad_adjoint_and_norm():
    from oracle import tv
    rng = np.random.default_rng(4)
    for hw in [(6, 10), (16, 8)]:
        n = hw[0] * hw[1]
        x = rng.standard_normal((n, 2))
        ph, pv = rng.standard_normal((n, 2)), rng.standard_normal((n, 2))
        dh, dv = tv.grad(x, hw)
        assert abs(np.sum(dh * ph + dv * pv) - np.sum(x * tv.grad_adj(ph, pv, hw))) < 1e-10
        # D^T D: sum of two 1-D Neumann Laplacians (rows of length W, columns
        # of length H): largest eigenvalue 2 + 2 cos(pi/H) + 2 + 2 cos(pi/W)
        dtd = np.stack([tv.grad_adj(*tv.grad(e[:, None], hw), hw)[:, 0] for e in np.eye(n)], 1)
        want = 4 + 2 * np.cos(np.pi / hw[0]) + 2 * np.cos(np.pi / hw[1])
        assert abs(np.max(np.linalg.eigvalsh(dtd)) - want) < 1e-9


def test_whole_frame_decode_recovers_the_scene():
    """The literal pipeline of the paper (whole-frame measurement, TV
    recovery, eq. (4)) on a small clip: the CS frames come back well above
    the key frame alone, and more measurements do better."""
    frames = sv.surveillance_video(sv.VideoSpec(48, 64, 3, 2, 77))
    out = {}
    for m in (300, 900):
        e = whole.encode_gop(frames, m, 16, 7, 1)
        d = whole.decode_gop(e, frames.shape, m, 16, 7, 1, iters=200)
        out[m] = np.mean([codec.psnr(frames[t], d["frames"][t]) for t in (1, 2)])
        key_only = np.mean([codec.psnr(frames[t], d["frames"][0]) for t in (1, 2)])
        assert out[m] > key_only
    assert out[900] > out[300]


def test_single_block_frame_decodes_as_block_tv():
    """A 16 x 16 frame is one B = 16 block: whole-frame decoding (eq. (1)
    with the TV solver on the frame as one image) must give exactly the
    block-form TV decode of the same GOP, pixel for pixel, with the same
    lambda, step constant, objective and relative residual."""
    rng = np.random.default_rng(8)
    base = rng.integers(60, 190, size=(16, 16))
    frames = np.stack([base, base + rng.integers(-20, 21, size=(16, 16)),
                       base + rng.integers(-30, 31, size=(16, 16))]).clip(0, 255).astype(np.uint8)
    m, seed, sid = 64, 0x5eed, 3
    e = whole.encode_gop(frames, m, 16, seed, sid)
    d = whole.decode_gop(e, frames.shape, m, 16, seed, sid, iters=120)
    p = codec.Params(16, 16, 3, 16, m, seed, sid, iters=120, solver="tv")
    gs = codec.encode_gop(frames, p)
    assert np.array_equal(gs.codes[:, 0, :], e["codes"]) and np.array_equal(gs.exps[:, 0], e["exps"])
    ref = codec.decode_gop(gs, p)
    assert np.array_equal(d["frames"], ref.frames)
    assert np.allclose(d["cs_float"], ref.cs_float, rtol=0, atol=1e-12)
    assert np.allclose(d["lam"], ref.lam[:, 0], rtol=1e-14, atol=0)
    assert d["L"] == ref.L
    assert np.allclose(d["objective"], ref.objective[:, 0], rtol=1e-12, atol=0)
    assert np.allclose(d["rel_residual"], ref.rel_residual[:, 0], rtol=1e-12, atol=0)
