"""Pins of the oracle's key-frame codec stand-in (the paper uses an H.264
intra codec for key frames, Sections 3.1 and 4; the stand-in is an integer
8x8 DCT with a uniform step and an Exp-Golomb bit count)."""
import numpy as np
import pytest
from scipy.fft import dctn, idctn

import synthvid as sv
from oracle import keyframe as kf


def test_integer_dct_close_to_orthonormal_dct():
    t = kf.int_dct8()
    exact = 1024.0 * kf.dct_matrix(8)
    assert np.all(np.abs(t - exact) <= 0.5)
    # no entry within 0.04 of a rounding tie: both sides round identically
    frac = np.abs(exact - np.floor(exact) - 0.5)
    assert frac.min() > 0.04
    dev = np.abs(t @ t.T / 2.0**20 - np.eye(8)).max()
    assert dev < 6e-4


def test_dct_matrix_matches_scipy():
    x = np.random.default_rng(0).standard_normal((8, 8))
    c = kf.dct_matrix(8)
    assert np.allclose(c @ x @ c.T, dctn(x, norm="ortho"), atol=1e-13)


def test_forward_transform_within_rounding_bound():
    rng = np.random.default_rng(1)
    t = kf.int_dct8()
    for _ in range(20):
        x = rng.integers(-128, 128, size=(8, 8)).astype(np.int64)
        z = (t @ x @ t.T) / 2.0**20
        ref = dctn(x.astype(np.float64), norm="ortho")
        assert np.all(np.abs(z - ref) <= 5e-4 * np.abs(x).sum())


def test_zigzag_is_jpeg_scan():
    zz = kf.zigzag8()
    assert len(set(zz)) == 64
    assert zz[:10] == [(0, 0), (0, 1), (1, 0), (2, 0), (1, 1), (0, 2),
                       (0, 3), (1, 2), (2, 1), (3, 0)]
    assert zz[-1] == (7, 7)
    for (a, b) in zip(zz, zz[1:]):
        assert abs(a[0] - b[0]) <= 1 and abs(a[1] - b[1]) <= 1 or \
            (a[0] + a[1] + 1 == b[0] + b[1])


@pytest.mark.parametrize("v,bits", [(0, 1), (1, 3), (2, 3), (3, 5), (6, 5), (7, 7), (14, 7), (15, 9)])
def test_ue_lengths(v, bits):
    assert kf.ue_bits(v) == bits


@pytest.mark.parametrize("v,bits", [(1, 3), (-1, 3), (2, 5), (-2, 5), (3, 5), (-3, 5), (4, 7), (-4, 7)])
def test_se_lengths(v, bits):
    assert kf.se_bits(v) == bits


def test_block_bits_hand_cases():
    z = np.zeros((8, 8), dtype=np.int64)
    assert kf.block_bits(z) == 1                     # ue(0)
    b = z.copy(); b[0, 0] = 1
    assert kf.block_bits(b) == 3 + 1 + 3             # ue(1)+ue(0)+se(1)
    b = z.copy(); b[1, 0] = -1                       # zigzag position 2
    assert kf.block_bits(b) == 3 + 3 + 3             # ue(1)+ue(2)+se(-1)
    b = z.copy(); b[0, 0] = 2; b[0, 1] = -3          # positions 0 and 1
    assert kf.block_bits(b) == 3 + (1 + 5) + (1 + 5)   # ue(2), se(2), se(-3)


def test_levels_are_rounded_quotients():
    rng = np.random.default_rng(2)
    frame = rng.integers(0, 256, size=(16, 24)).astype(np.uint8)
    lev = kf.encode_levels(frame, 16)
    t = kf.int_dct8()
    for by in (0, 8):
        for bx in (0, 8, 16):
            x = frame[by:by + 8, bx:bx + 8].astype(np.int64) - 128
            z = (t @ x @ t.T).astype(np.float64) / (16 * 2.0**20)
            expect = np.sign(z) * np.floor(np.abs(z) + 0.5)
            assert np.array_equal(lev[by:by + 8, bx:bx + 8], expect.astype(np.int64))


def test_flat_block_round_trip():
    for val in (0, 1, 77, 128, 200, 255):
        frame = np.full((8, 8), val, dtype=np.uint8)
        dec = kf.decode_levels(kf.encode_levels(frame, 16), 16)
        # DC only: error below half a quantiser step in the pixel domain
        assert np.all(np.abs(dec.astype(int) - val) <= 1)


def test_key_psnr_close_to_float_dct_codec():
    frame = sv.qcif_tiny().video(1)[0]
    dec = kf.decode_levels(kf.encode_levels(frame, 16), 16)
    ref = np.zeros(frame.shape)
    for by in range(0, frame.shape[0], 8):
        for bx in range(0, frame.shape[1], 8):
            x = frame[by:by + 8, bx:bx + 8].astype(np.float64) - 128
            c = dctn(x, norm="ortho") / 16
            c = np.sign(c) * np.floor(np.abs(c) + 0.5) * 16
            ref[by:by + 8, bx:bx + 8] = idctn(c, norm="ortho") + 128
    ref = np.clip(np.rint(ref), 0, 255)

    def psnr(a, b):
        return 10 * np.log10(255.0**2 / np.mean((a.astype(float) - b) ** 2))
    assert abs(psnr(frame, dec) - psnr(frame, ref)) < 0.2


def test_frame_dims_must_be_multiples_of_8():
    with pytest.raises(ValueError):
        kf.encode_levels(np.zeros((12, 16), dtype=np.uint8))
