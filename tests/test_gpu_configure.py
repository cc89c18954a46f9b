"""The parameter configurator on the GPU against the oracle's sweep: bit
counts and compression ratios exact, PSNRs within the path's parity bar
(FP32 0.01 dB, BF16 0.1 dB), and the same choice unless a candidate's PSNR
lies within that bar of the floor.  Per-frame SSE is exact."""
import numpy as np
import pytest

import synthvid as sv
from oracle import codec, configurator as cfg
from tests.gpu_util import announce, ctx, dev, host  # noqa: F401

pytestmark = pytest.mark.gpu


def test_frame_sse_exact(ctx):
    announce("frame_sse")
    rng = np.random.default_rng(4)
    a = rng.integers(0, 256, size=(5, 144, 176), dtype=np.uint8)
    b = a.copy()
    b[1] = 0
    b[3, :7, :9] = 255
    got = host(ctx.frame_sse(dev(a), dev(b))).astype(np.int64)
    want = ((a.astype(np.int64) - b.astype(np.int64)) ** 2).reshape(5, -1).sum(axis=1)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("precision,tol", [("fp32", 0.01), ("bf16", 0.1)])
def test_configure_matches_oracle(ctx, precision, tol):
    import paper_1311_1419_amd as P
    announce(f"configure {precision}")
    spec = sv.qcif_tiny().with_(block=32, iters=100)
    clip = spec.video(8)                          # G = 3: GOPs of 3, 3, 2; G = 4: 4, 4
    gops, ms = [3, 4], [25, 51, 102]
    ref_pts, _ = cfg.configure(clip, codec.Params.from_spec(spec), gops, ms, floor_db=0.0)
    floor = float(np.median([p.psnr_all for p in ref_pts]))
    ref_pts, ref_best = cfg.configure(clip, codec.Params.from_spec(spec), gops, ms, floor)
    prec = P.CSV_FP32 if precision == "fp32" else P.CSV_BF16
    res = ctx.configure(dev(clip), P.Params.from_spec(spec, precision=prec), gops, ms, floor)
    pts = res["points"]
    assert len(pts) == len(ref_pts)
    for p, r in zip(pts, ref_pts):
        assert (p["gop"], p["m"]) == (r.gop, r.m)
        assert p["bits_key"] == r.bits_key and p["bits_cs"] == r.bits_cs
        assert p["cr_total"] == pytest.approx(r.cr_total, rel=1e-12)
        assert p["cr_key"] == pytest.approx(r.cr_key, rel=1e-12)
        assert p["cr_cs"] == pytest.approx(r.cr_cs, rel=1e-12)
        assert abs(p["psnr_all"] - r.psnr_all) <= tol
        assert abs(p["psnr_cs"] - r.psnr_cs) <= tol
        assert bool(p["meets_floor"]) == (p["psnr_all"] >= floor)
    # the GPU's choice is valid on its own measurements ...
    ok = [i for i, p in enumerate(pts) if p["meets_floor"]]
    if ok:
        top = max(pts[i]["cr_total"] for i in ok)
        assert res["best"] in ok and pts[res["best"]]["cr_total"] == top
    else:
        assert res["best"] == -1
    # ... and equals the oracle's unless some PSNR sits within the bar of the floor
    if all(abs(r.psnr_all - floor) > tol for r in ref_pts):
        assert res["best"] == ref_best


def test_configure_rejects_bad_candidates(ctx):
    import paper_1311_1419_amd as P
    spec = sv.qcif_tiny()
    clip = dev(spec.video(4))
    with pytest.raises(P.CsvError):
        ctx.configure(clip, P.Params.from_spec(spec), [0], [64], 20.0)
    with pytest.raises(P.CsvError):
        ctx.configure(clip, P.Params.from_spec(spec), [3], [300], 20.0)   # M > n
