"""Pins of the oracle's reduced-precision measurement forms: the E4M3
rounding against its published definition (hand cases) and against torch's
independent float8_e4m3fn conversion, the int8 digit split, and both forms
against brute-force sums on tiny inputs."""
import numpy as np
import pytest
import torch

from oracle import codec, cs, fp8, philox


def test_e4m3_hand_cases():
    # spacing 1 below 16, 2 in [16, 32), 4 in [32, 64), ..., 32 in [256, 448]
    cases = {0: 0, 1: 1, 7: 7, 8: 8, 15: 15, 16: 16, 17: 16, 18: 18, 19: 20, 33: 32, 34: 32,
             35: 36, 100: 96, 104: 104, 108: 112, 255: 256, 240: 240, 248: 256, 440: 448,
             448: 448, -17: -16, -255: -256}
    for x, want in cases.items():
        assert fp8.e4m3_round(x) == want, x
    # binade and subnormal edges: smallest normal 2^-6, subnormal step 2^-9
    assert fp8.e4m3_round(2.0 ** -6) == 2.0 ** -6
    assert fp8.e4m3_round(2.0 ** -9) == 2.0 ** -9
    assert fp8.e4m3_round(0.75 * 2.0 ** -9) == 2.0 ** -9     # nearest subnormal
    assert fp8.e4m3_round(2.0 ** -10) == 0.0                 # tie 0 / 2^-9: even (0)
    assert fp8.e4m3_round(1.5 * 2.0 ** -9) == 2.0 ** -8      # tie 1 / 2 subnormal steps: even (2)
    assert fp8.e4m3_round(1.0625) == 1.0                     # tie 1 + 1/16: even mantissa 0
    assert fp8.e4m3_round(1.1875) == 1.25                    # tie 1 + 3/16: even mantissa 2
    with pytest.raises(ValueError):
        fp8.e4m3_round(449.0)


def test_e4m3_matches_torch_float8():
    rng = np.random.default_rng(3)
    xs = np.concatenate([np.arange(-448, 449, dtype=np.float64),
                         rng.uniform(-448, 448, 20000), rng.uniform(-1, 1, 20000),
                         rng.uniform(-2 ** -5, 2 ** -5, 5000)])
    ref = torch.from_numpy(xs).to(torch.float32).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    # xs are float64; torch converts through float32, which is exact for the
    # integers and only perturbs random floats far from E4M3 ties
    assert np.array_equal(fp8.e4m3_round(xs.astype(np.float32).astype(np.float64)), ref)


def test_e4m3_of_integers_are_integers_and_within_relative_half_ulp():
    x = np.arange(-448, 449)
    r = fp8.e4m3_round(x)
    assert np.all(r == np.round(r))
    nz = x != 0
    assert np.all(np.abs(r[nz] - x[nz]) <= np.abs(x[nz]) / 16.0)   # half of 2^-3 relative


def test_int8_split_digits():
    r = np.arange(-255, 256)
    h, l = fp8.split_int8(r)
    assert np.array_equal(16 * h + l, r)
    assert l.min() == 0 and l.max() == 15 and h.min() == -16 and h.max() == 15


def test_measurement_forms_brute_force():
    rng = np.random.default_rng(5)
    q = philox.measurement_matrix_q(8, 16, 11, 2)
    r = rng.integers(-255, 256, size=(16, 5))
    y_exact = cs.measure(q, r)
    assert np.array_equal(fp8.measure_int8(q, r), y_exact)
    y8 = fp8.measure_fp8(q, r)
    for i in range(8):
        for j in range(5):
            s = 0
            for k in range(16):
                s += int(fp8.e4m3_round(q[i, k])) * int(fp8.e4m3_round(r[k, j]))
            assert y8[i, j] == s
    # the FP8 form's error is bounded by the rounding of both operands
    bound = np.abs(q.astype(np.float64)) @ np.abs(r.astype(np.float64)) * (1 / 16 + 1 / 16 + 1 / 256)
    assert np.all(np.abs(y8 - y_exact) <= bound)


def test_fp8_form_fits_fp32_accumulation_at_full_size():
    # the largest partial sum for n = 1024: 1024 x 256 x 32 < 2^24
    assert 1024 * 256 * 32 < 2 ** 24
    q = philox.measurement_matrix_q(16, 1024, 1, 1)
    r = np.full((1024, 1), 255)
    y8 = fp8.measure_fp8(q, r)
    acc = np.zeros(16, dtype=np.float32)
    q8 = fp8.e4m3_round(q).astype(np.float32)
    r8 = np.float32(fp8.e4m3_round(255))
    for k in range(1024):
        acc = acc + q8[:, k] * r8
    assert np.array_equal(acc.astype(np.int64), y8[:, 0])


def test_encode_gop_measure_forms():
    import synthvid as sv
    spec = sv.qcif_tiny()
    frames = spec.video()
    ex = codec.encode_gop(frames, codec.Params.from_spec(spec))
    i8 = codec.encode_gop(frames, codec.Params.from_spec(spec, measure_form="int8"))
    f8 = codec.encode_gop(frames, codec.Params.from_spec(spec, measure_form="fp8"))
    assert np.array_equal(i8.codes, ex.codes) and np.array_equal(i8.exps, ex.exps)
    assert np.array_equal(f8.key_levels, ex.key_levels)
    # FP8 measurements differ, but by a few percent of the measurement scale
    d = np.abs(f8.y_int - ex.y_int)
    assert d.max() > 0
    assert d.max() <= 0.15 * np.abs(ex.y_int).max()
