"""Pins of the oracle's counter generator and measurement matrix.

The Philox4x64-10 round function (Salmon et al., SC'11) is checked against
numpy's own, independently written Philox bit generator; the measurement
matrix against the moments of Binomial(64, 1/2) - 32 (Sections 1 and 4 only
ask for a random Gaussian matrix)."""
import numpy as np
import pytest

from oracle import philox

MASK = (1 << 64) - 1


def _numpy_philox(ctr, key):
    """numpy's Philox returns the block of counter+1 first."""
    c = [int(x) for x in ctr]
    # step the 256-bit counter back by one (borrow across words)
    for i in range(4):
        if c[i] == 0:
            c[i] = MASK          # borrow into the next word (wraps at 2^256)
        else:
            c[i] -= 1
            break
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(c, dtype=np.uint64))
    return tuple(int(x) for x in bg.random_raw(4))


@pytest.mark.parametrize("ctr,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 256, 0, 0), (0x1311141900030000, 0)),
    ((12345, 1024, 0, 0), (0x1311141900040005, 5)),
    ((0, 1, 0, 0), (MASK, MASK)),                 # borrow across words
    ((MASK, 7, 3, 9), (0xDEADBEEF, 0xC0FFEE)),
    ((2**40 + 3, 2**63, 2**62, 1), (1, 2)),
])
def test_round_function_matches_numpy(ctr, key):
    assert philox.philox4x64_10_scalar(ctr, key) == _numpy_philox(ctr, key)


def test_vector_matches_scalar():
    rng = np.random.default_rng(7)
    ctr = rng.integers(0, 2**63, size=(64, 4), dtype=np.uint64)
    k0, k1 = 0x1311141900010003, 3
    vec = philox.philox4x64_10(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3], k0, k1)
    for i in range(64):
        s = philox.philox4x64_10_scalar(tuple(int(x) for x in ctr[i]), (k0, k1))
        assert tuple(int(v[i]) for v in vec) == s


def test_q_entries_follow_counter_layout():
    m, n, seed, sid = 5, 256, 0x1311141900010000, 0
    q = philox.measurement_matrix_q(m, n, seed, sid)
    for (i, j) in [(0, 0), (0, 3), (1, 17), (4, 255), (3, 128)]:
        idx = i * n + j
        words = philox.philox4x64_10_scalar((idx // 4, n, 0, 0), (seed, sid))
        assert q[i, j] == bin(words[idx % 4]).count("1") - 32


def test_q_moments_binomial():
    q = philox.measurement_matrix_q(1024, 1024, 0x1311141900020001, 1).ravel().astype(np.float64)
    assert q.min() >= -32 and q.max() <= 32
    mean, var = q.mean(), q.var()
    kurt = np.mean((q - mean) ** 4) / var ** 2 - 3.0
    assert abs(mean) < 0.03                     # sd of mean: 4/1024
    assert abs(var - 16.0) < 0.15               # ~7 standard errors
    assert abs(kurt - (-1.0 / 32.0)) < 0.03     # excess kurtosis of Bin(64,1/2)


def test_phi_variance_is_one_over_m():
    m = 64
    q = philox.measurement_matrix_q(m, 256, 11, 2).astype(np.float64)
    phi = philox.phi_scale(m) * q
    assert abs(phi.var() * m - 1.0) < 0.05


def test_rows_nested_and_streams_independent():
    a = philox.measurement_matrix_q(26, 256, 99, 4)
    b = philox.measurement_matrix_q(128, 256, 99, 4)
    assert np.array_equal(a, b[:26])
    c = philox.measurement_matrix_q(26, 256, 99, 5)
    d = philox.measurement_matrix_q(26, 1024, 99, 4)
    assert not np.array_equal(a, c)
    assert not np.array_equal(a, d[:, :256])
