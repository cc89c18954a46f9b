"""Pins of the oracle's block gather, integer measurement (y = A x of
Section 3.2, per block) and 8-bit block-floating-point quantiser."""
import numpy as np
import pytest

from oracle import cs, philox


def test_gather_scatter_round_trip_and_padding():
    rng = np.random.default_rng(0)
    for (h, w, b) in [(144, 176, 16), (144, 176, 32), (48, 40, 16), (720, 1280, 16)]:
        r = rng.integers(-255, 256, size=(h, w))
        cols = cs.gather_blocks(r, b)
        nby, nbx = cs.blocks_shape(h, w, b)
        assert cols.shape == (b * b, nby * nbx)
        assert np.array_equal(cs.scatter_blocks(cols, h, w, b), r)
        # every pixel appears exactly once; padding contributes zeros only
        assert cols.sum() == r.sum() and np.abs(cols).sum() == np.abs(r).sum()
    # padded block of the 176x144 frame at B=32: last block column has 16 live columns
    r = np.ones((144, 176), dtype=np.int64)
    cols = cs.gather_blocks(r, 32)
    last = cols[:, 5].reshape(32, 32)
    assert last[:, :16].all() and not last[:, 16:].any()


def test_measurement_linearity_exact():
    q = philox.measurement_matrix_q(64, 256, 3, 1)
    rng = np.random.default_rng(1)
    r1 = rng.integers(-255, 256, size=(256, 9))
    r2 = rng.integers(-255, 256, size=(256, 9))
    for (a, b) in [(1, 1), (3, -2), (-1, 0)]:
        lhs = cs.measure(q, a * r1 + b * r2)
        rhs = a * cs.measure(q, r1) + b * cs.measure(q, r2)
        assert np.array_equal(lhs, rhs)


@pytest.mark.parametrize("n", [256, 1024, 2048])
def test_measurement_exact_in_float32_accumulation(n):
    # |Q| <= 32, |r| <= 255: every partial sum stays below 2^24 for n <= 2048
    q = philox.measurement_matrix_q(16, n, 5, 0)
    r = np.full((n, 2), 255, dtype=np.int64)
    r[:, 1] = -255
    q_ext = np.where(q >= 0, 32, -32)            # worst-case magnitudes
    for qq in (q, q_ext):
        exact = cs.measure(qq, r)
        f32 = np.zeros(exact.shape, dtype=np.float32)
        for k in range(n):                       # sequential fp32 accumulation
            f32 += (qq[:, k:k + 1].astype(np.float32) * r[k:k + 1, :].astype(np.float32))
        assert np.array_equal(f32.astype(np.int64), exact)
    assert n * 32 * 255 < 2**24


@pytest.mark.parametrize("vals,e,codes", [
    ([127, -5, 0], 0, [127, -5, 0]),
    ([128, 1, -1], 1, [64, 1, -1]),           # (1+1)>>1 = 1: half rounds away
    ([254, 3, -3], 1, [127, 2, -2]),
    ([255, 2, -2], 2, [64, 1, -1]),           # (255+2)>>2 = 64
    ([-1000, 500, 7], 3, [-125, 63, 1]),      # (1000+4)>>3=125, (500+4)>>3=63
    ([0, 0, 0], 0, [0, 0, 0]),
])
def test_quantiser_hand_cases(vals, e, codes):
    c, ex = cs.quantise(np.array(vals, dtype=np.int64)[:, None])
    assert ex[0] == e
    assert list(c[:, 0]) == codes


def test_quantiser_bound_and_minimal_exponent():
    rng = np.random.default_rng(2)
    y = rng.integers(-(2**23), 2**23, size=(64, 200))
    y[:, :20] //= 1000                        # some quiet blocks
    c, e = cs.quantise(y)
    s_phi = philox.phi_scale(64)
    yh = cs.dequantise(c, e, s_phi)
    for j in range(y.shape[1]):
        ej = int(e[j])
        assert np.all(np.abs(c[:, j].astype(int)) <= 127)
        bound = s_phi * (2.0 ** (ej - 1) if ej else 0.0)
        assert np.all(np.abs(yh[:, j] - s_phi * y[:, j]) <= bound + 1e-12)
        if ej > 0:                            # one step less would overflow 8 bits
            mx = int(np.abs(y[:, j]).max())
            h = (1 << (ej - 2)) if ej > 1 else 0
            assert ((mx + h) >> (ej - 1)) > 127
