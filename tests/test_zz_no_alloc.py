"""csv_measure_frame_noalloc (the allocation-free measurement entry point)
against csv_measure_frame on the GPU: two calls in a row, the second with a
smaller frame, equal bit for bit (measurements, codes, exponents), and no
device memory allocated by either call."""
import numpy as np
import pytest

import synthvid as sv
from tests.gpu_util import announce, ctx, dev, host  # noqa: F401

pytestmark = pytest.mark.gpu


def _case(ctx, spec, flags):
    import torch
    import paper_1311_1419_amd as P
    p = P.Params.from_spec(spec, precision=P.CSV_BF16, flags=flags)
    frames = dev(spec.video(2))
    lev, _ = ctx.key_encode(frames[0], spec.key_qstep)
    key = ctx.key_decode(lev, spec.key_qstep)
    q = ctx.phi_matrix(p)
    y_ref, c_ref, e_ref = ctx.measure_frame(p, frames[1], key)
    m, nb = p.resolve()
    y = torch.full((nb, m), -7, dtype=torch.int32, device="cuda")
    codes = torch.full((nb, m), 99, dtype=c_ref.dtype, device="cuda")
    exps = torch.full((nb,), 255, dtype=torch.uint8, device="cuda")
    return p, q, frames, key, (y_ref, c_ref, e_ref), (y, codes, exps)


def test_noalloc_measure_equals_measure_frame(ctx):
    import torch
    import paper_1311_1419_amd as P
    cases = [(sv.vga_precision(0.25, gop=2), 0),                        # 300 x 256 measurements
             (sv.qcif_tiny().with_(gop=2), P.CSV_FLAG_MEASURE_INT8),    # smaller: 99 x 64
             (sv.cif_sweep(2, 0.2), P.CSV_FLAG_MEASURE_FP8),
             (sv.qcif_tiny().with_(gop=2, m=40), P.CSV_FLAG_NO_QUANT)]
    prepared = []
    for spec, flags in cases:
        announce(f"noalloc measure prepare {spec.width}x{spec.height} B={spec.block} "
                 f"M={spec.m} flags={flags}")
        prepared.append(_case(ctx, spec, flags))
    torch.cuda.synchronize()
    # the device array is set up by the library's context creation (the
    # fixture's), so the calls below find it in place
    free0 = torch.cuda.mem_get_info()[0]
    for p, q, frames, key, ref, out in prepared:
        announce(f"noalloc measure {p.width}x{p.height} B={p.block} M={p.m} flags={p.flags}")
        P.measure_frame_noalloc(p, q, frames[1], key, *out)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    for p, q, frames, key, ref, out in prepared:
        for a, b in zip(ref, out):
            assert np.array_equal(host(a), host(b)), (p.width, p.flags)


def test_noalloc_limits_are_checked_before_gpu_work(ctx):
    import torch
    import paper_1311_1419_amd as P
    announce("noalloc measure limits")
    spec = sv.vga_precision(0.25, gop=2)
    p = P.Params.from_spec(spec, precision=P.CSV_BF16).with_(width=3840, height=2160, m=1024)
    dummy = torch.zeros(16, dtype=torch.int8, device="cuda")
    u8 = torch.zeros(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.CsvError) as ei:
        P.measure_frame_noalloc(p, dummy, u8, u8, None, dummy, u8)
    assert ei.value.code == -1 and "limit" in str(ei.value)
