"""Every compiled variant of the fused kernel meets the BF16 parity bar
against the FP64 oracle, and the autotuner times the variants, records a
choice, and writes a table that loads back."""
import json
import os

import numpy as np
import pytest

import synthvid as sv
from oracle import codec
from tests.gpu_util import announce, ctx, dev, host, psnr  # noqa: F401

pytestmark = pytest.mark.gpu

SPECS = [(sv.qcif_tiny(), "b16-m64"), (sv.cif_sweep(4, 0.1), "b16-m26"),
         (sv.cif_sweep(4, 0.3), "b16-m77"), (sv.cif_sweep(4, 0.5), "b16-m128"),
         (sv.vga_precision(0.25, gop=3), "b32-m256"),
         (sv.qcif_tiny().with_(block=32, m=102, gop=3, iters=300), "b32-m102"),
         (sv.qcif_tiny().with_(block=32, m=51, gop=2, iters=300), "b32-m51"),
         (sv.qcif_tiny().with_(block=32, m=205, gop=2, iters=300), "b32-m205"),
         (sv.vga_precision(0.4, gop=2), "b32-m410"),
         (sv.qcif_tiny().with_(block=32, m=25, gop=3, iters=300), "b32-m25"),
         (sv.qcif_tiny().with_(block=32, m=25, gop=2, iters=77), "b32-m25-t77")]


@pytest.mark.parametrize("spec", [s for s, _ in SPECS], ids=[i for _, i in SPECS])
def test_every_variant_meets_parity(ctx, spec):
    import paper_1311_1419_amd as P
    frames = spec.video()
    op = codec.Params.from_spec(spec)
    ref = codec.decode_gop(codec.encode_gop(frames, op), op)
    p = P.Params.from_spec(spec, precision=P.CSV_BF16)
    gs = ctx.encode_gop(dev(frames), p)
    name0, idx0, count = P.kernel_choice(spec.block, spec.m)
    try:
        for v in range(count):
            P.set_kernel_choice(spec.block, spec.m, v)
            announce(f"variant {P.kernel_choice(spec.block, spec.m)[0]} for B={spec.block} M={spec.m}")
            out, fl, _ = ctx.decode_gop(gs, p, want_float=True)
            out, fl = host(out), host(fl)
            for t in range(1, spec.gop):
                assert np.max(np.abs(fl[t - 1] - ref.cs_float[t - 1])) <= 4.0
                assert abs(psnr(frames[t], out[t]) - psnr(frames[t], ref.frames[t])) <= 0.1
    finally:
        P.set_kernel_choice(spec.block, spec.m, idx0)


def test_autotune_records_and_reloads(ctx, tmp_path):
    import paper_1311_1419_amd as P
    announce("autotune b16 m64")
    path = str(tmp_path / "tune.json")
    res = ctx.autotune(16, 64, iters=50, n_blocks=4096, json_path=path)
    assert len(res["times_ms"]) == P.kernel_choice(16, 64)[2]
    assert all(t > 0 for t in res["times_ms"])
    assert res["best"] == int(np.argmin(res["times_ms"]))
    table = json.load(open(path))
    assert table["arch"] == "gfx950"
    entry = [c for c in table["classes"] if c["n"] == 256 and c["Mp"] == 64][0]
    assert entry["variant"] == res["choice"] and len(entry["ms"]) == len(res["times_ms"])
    P.set_kernel_choice(16, 64, (res["best"] + 1) % len(res["times_ms"]))
    P.load_kernel_choices(path)
    assert P.kernel_choice(16, 64)[0] == res["choice"]
    P.set_kernel_choice(16, 64, 0)
    assert os.path.getsize(path) > 0
