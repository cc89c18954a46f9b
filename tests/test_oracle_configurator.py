"""Pins of the oracle's parameter configurator (Sections 2-3, Fig. 6,
Table I): the PSNR closed forms, the bit and CR accounting against the
Table I identity, the choice rule, and a small sweep with a partial GOP."""
import numpy as np

import synthvid as sv
from oracle import codec, configurator as cfg


def test_frame_psnr_closed_forms():
    a = np.full((16, 24), 100, dtype=np.uint8)
    assert cfg.frame_psnr(a, a) == 99.99
    b = a + 1                                     # SSE = H W: 20 log10(255)
    assert abs(cfg.frame_psnr(a, b) - 20 * np.log10(255.0)) < 1e-12
    c = a.copy()
    c[0, 0] = 0                                   # one pixel off by 100
    want = 10 * np.log10(255.0 ** 2 * a.size / 100.0 ** 2)
    assert abs(cfg.frame_psnr(a, c) - want) < 1e-12


def test_choose_rule():
    P = cfg.Point
    pts = [P(3, 25, 0, 0, 30.0, 0, 0, 31.0, 0, True),
           P(3, 12, 0, 0, 45.0, 0, 0, 29.0, 0, False),
           P(5, 25, 0, 0, 40.0, 0, 0, 30.5, 0, True),
           P(5, 12, 0, 0, 40.0, 0, 0, 30.2, 0, True)]   # tie with index 2: first kept
    assert cfg.choose(pts) == 2
    assert cfg.choose([p for p in pts if not p.meets_floor]) == -1
    assert cfg.choose([]) == -1


def test_sweep_accounting_matches_table_identity():
    spec = sv.qcif_tiny().with_(block=32, iters=60)
    clip = spec.video(9)                          # G = 3: three whole GOPs
    base = codec.Params.from_spec(spec)
    pts, best = cfg.configure(clip, base, [3], [25, 51], floor_db=0.0)
    nb = 6 * 5                                    # 176 x 144 at B = 32 (padded)
    for p, m in zip(pts, [25, 51]):
        assert p.m == m and p.gop == 3
        assert p.bits_cs == 3 * 2 * nb * (8 * m + 8)
        assert abs(p.cr_cs - 8.0 * 176 * 144 * 6 / p.bits_cs) < 1e-12
        # Table I identity: total = G / (1/CR_key + (G-1)/CR_cs)
        ident = codec.total_cr_from_ratios(3, p.cr_key, p.cr_cs)
        assert abs(p.cr_total - ident) < 1e-9 * ident
        assert p.meets_floor and 10 < p.psnr_cs < p.psnr_all < 99
    # fewer measurements: higher CR, lower quality; the floor of 0 keeps both
    assert pts[0].cr_total > pts[1].cr_total and pts[0].psnr_cs < pts[1].psnr_cs
    assert best == 0


def test_partial_gop_and_key_only_tail():
    spec = sv.qcif_tiny().with_(iters=40)
    clip = spec.video(7)                          # G = 3: GOPs of 3, 3 and 1 frames
    base = codec.Params.from_spec(spec)
    p = cfg.evaluate(clip, base, 3, 64, floor_db=0.0)
    nb = 11 * 9
    assert p.bits_cs == (2 + 2) * nb * (8 * 64 + 8)
    keys = [codec.encode_gop(clip[i:i + 1], codec.Params.from_spec(spec, gop=1)).bits_key
            for i in (0, 3, 6)]
    assert p.bits_key == sum(keys)
    assert abs(p.cr_key - 8.0 * 176 * 144 * 3 / p.bits_key) < 1e-12
    # the key-only GOP contributes its (intra-coded) frame to the PSNR mean only
    assert p.psnr_all > p.psnr_cs
