"""Parity of the fused BF16 recovery (BF16 MFMA products, FP32 accumulation
and iterates) against the FP64 oracle.

Tolerances: per CS frame PSNR within 0.1 dB of the oracle's; recovered float
frames within 4 grey levels; FP64 objective within 1e-2 relative.  BF16 keeps
8 significant bits in the operator and in the two product operands, and the
objective at the recovered point is 1-2 orders of magnitude more sensitive
than the pixels.  Batched decoding must reproduce each GOP decoded alone bit
for bit (the tile shape of a block does not depend on the batch)."""
import numpy as np
import pytest

import synthvid as sv
from oracle import codec, cs, philox
from tests.gpu_util import announce, ctx, dev, host, psnr  # noqa: F401

pytestmark = pytest.mark.gpu

PSNR_TOL = 0.1
MAXABS_TOL = 4.0


def _bf16(spec, **kw):
    import paper_1311_1419_amd as P
    return P.Params.from_spec(spec, precision=P.CSV_BF16, **kw)


CASES = [
    (sv.qcif_tiny(), "qcif-b16-m64"),
    (sv.cif_sweep(4, 0.1), "cif-b16-m26"),
    (sv.cif_sweep(4, 0.3), "cif-b16-m77"),
    (sv.cif_sweep(4, 0.5), "cif-b16-m128"),
    (sv.vga_precision(0.1, gop=3), "vga-b32-m102"),
    (sv.vga_precision(0.25, gop=3), "vga-b32-m256"),
    (sv.qcif_tiny().with_(block=32, m=205, gop=3, iters=300), "qcif-b32-m205-padded"),
    (sv.qcif_tiny().with_(block=32, m=410, gop=2, iters=300), "qcif-b32-m410-padded"),
    (sv.qcif_tiny().with_(block=32, m=51, gop=3, iters=300), "qcif-b32-m51-padded"),
    (sv.cif_sweep(4, 0.25).with_(block=32, m=12, iters=300), "cif-b32-m12"),
    (sv.cif_sweep(8, 0.2), "cif-g8-b16-m51"),
    (sv.cif_sweep(16, 0.2), "cif-g16-b16-m51"),
    # odd and minimal iteration counts: the class defaults keep s and v in two
    # arrays that trade roles every iteration, so s_T sits in either
    (sv.qcif_tiny().with_(iters=77), "qcif-b16-m64-t77"),
    (sv.cif_sweep(4, 0.1).with_(iters=1), "cif-b16-m26-t1"),
    (sv.cif_sweep(4, 0.3).with_(iters=3), "cif-b16-m77-t3"),
    (sv.cif_sweep(4, 0.5).with_(iters=2), "cif-b16-m128-t2"),
    (sv.cif_sweep(4, 0.5).with_(iters=5), "cif-b16-m128-t5"),
    (sv.vga_precision(0.25, gop=2).with_(iters=7), "vga-b32-m256-t7"),
    (sv.qcif_tiny().with_(block=32, m=102, gop=2, iters=9), "qcif-b32-m102-t9"),
]


@pytest.mark.parametrize("spec", [c[0] for c in CASES], ids=[c[1] for c in CASES])
def test_decode_bf16_matches_oracle(ctx, spec):
    announce(f"decode bf16 {spec.width}x{spec.height} G={spec.gop} B={spec.block} M={spec.m}")
    frames = spec.video()
    op = codec.Params.from_spec(spec)
    ref = codec.decode_gop(codec.encode_gop(frames, op), op)
    p = _bf16(spec)
    gs = ctx.encode_gop(dev(frames), p)
    out, fl, obj = ctx.decode_gop(gs, p, want_float=True, want_obj=True)
    out, fl, obj = host(out), host(fl), host(obj)
    assert np.array_equal(out[0], ref.frames[0])
    for t in range(1, spec.gop):
        err = np.max(np.abs(fl[t - 1].astype(np.float64) - ref.cs_float[t - 1]))
        assert err <= MAXABS_TOL, f"frame {t}: max abs {err}"
        dp = abs(psnr(frames[t], out[t]) - psnr(frames[t], ref.frames[t]))
        assert dp <= PSNR_TOL, f"frame {t}: PSNR differs by {dp}"
    rel = np.abs(obj[..., 0] - ref.objective) / np.maximum(ref.objective, 1e-300)
    assert np.max(rel) <= 1e-2


def test_bf16_batch_equals_alone(ctx):
    """Each GOP decoded inside a mixed batch (several streams, sizes, M,
    block sizes and tile classes) equals the GOP decoded alone."""
    announce("bf16 batch vs alone")
    specs = [sv.qcif_tiny(), sv.cif_sweep(4, 0.1, stream=1), sv.vga_precision(0.25, gop=2, stream=2),
             sv.qcif_tiny().with_(block=32, m=102, stream_id=9, phi_seed=99),
             sv.cif_sweep(4, 0.1, stream=3)]
    items = []
    for spec in specs:
        p = _bf16(spec)
        items.append((ctx.encode_gop(dev(spec.video()), p), p))
    alone = [tuple(host(x) for x in ctx.decode_gop(gs, p, want_float=True)[:2]) for gs, p in items]
    mixed = ctx.decode_batch(items, want_float=True)
    for (fa, fla), (fm, flm, _) in zip(alone, mixed):
        assert np.array_equal(fa, host(fm))
        assert np.array_equal(fla, host(flm))


def test_bf16_deterministic_and_zero_residual(ctx):
    announce("bf16 determinism + zero residual")
    spec = sv.cif_sweep(4, 0.25)
    p = _bf16(spec)
    gs = ctx.encode_gop(dev(spec.video()), p)
    a = host(ctx.decode_gop(gs, p, want_float=True)[1])
    b = host(ctx.decode_gop(gs, p, want_float=True)[1])
    assert np.array_equal(a, b)
    frames = spec.video(1)
    key = host(ctx.key_decode(ctx.key_encode(dev(frames[0]))[0]))
    z = np.stack([frames[0], key, key, key])
    gz = ctx.encode_gop(dev(z), p)
    out, fl, obj = ctx.decode_gop(gz, p, want_float=True, want_obj=True)
    assert np.all(host(fl) == key[None].astype(np.float32))
    assert np.all(host(obj) == 0)


def test_bf16_full_size_sampled_blocks(ctx):
    """640x480, GOP 16, B=32, M=256 (4500 blocks, the benchmark's shape):
    the oracle recovers a sample of blocks one by one, including the last
    (ragged) tile, and the GPU's pixels for those blocks must agree."""
    announce("bf16 full-size vga g16 m256 sampled")
    spec = sv.vga_precision(0.25)
    frames = spec.video()
    p = _bf16(spec)
    gs = ctx.encode_gop(dev(frames), p)
    out, fl, _ = ctx.decode_gop(gs, p, want_float=True)
    fl = host(fl)
    key = host(out)[0].astype(np.float64)
    codes, exps = host(gs.codes), host(gs.exps)
    q = philox.measurement_matrix_q(spec.m, spec.n, spec.phi_seed, spec.stream_id)
    s_phi = philox.phi_scale(spec.m)
    a = cs.operator(q, s_phi, spec.block)
    L, _, _ = cs.lipschitz(q, s_phi)
    nb = codes.shape[1]
    rng = np.random.default_rng(0)
    picks = [(t, int(b)) for t in (0, 7, 14) for b in rng.choice(nb, 5, replace=False)]
    picks += [(14, nb - 1), (14, nb - 2)]
    nbx = spec.width // spec.block
    for t, b in picks:
        y = cs.dequantise(codes[t, b][:, None], exps[t, b:b + 1], s_phi)
        lam = cs.lambdas(a, y)
        s_hat = cs.fista(a, y, lam, L, spec.iters)
        x = cs.synthesise(s_hat, spec.block)[:, 0].reshape(spec.block, spec.block)
        by, bx = divmod(b, nbx)
        sl = (slice(by * 32, by * 32 + 32), slice(bx * 32, bx * 32 + 32))
        ref = key[sl] + x
        assert np.max(np.abs(fl[t][sl] - ref)) <= MAXABS_TOL, (t, b)


def test_bf16_serving_hd_camera_sampled_blocks(ctx):
    """A full-size GOP of the serving mix: one 1280x720 camera, GOP 32, B=16,
    M/n = 0.25 (M = 64), 31 x 3600 blocks decoded as one GOP.  The oracle
    recovers 17 sampled blocks one by one (spread over the GOP, plus the
    last blocks of the last frame) and the GPU's pixels must agree."""
    announce("bf16 full-size 1280x720 g32 b16 m64 sampled")
    spec = sv.serving_cameras(6)[5][0]
    assert (spec.width, spec.height, spec.gop, spec.block, spec.m) == (1280, 720, 32, 16, 64)
    frames = spec.video()
    p = _bf16(spec)
    gs = ctx.encode_gop(dev(frames), p)
    out, fl, _ = ctx.decode_gop(gs, p, want_float=True)
    fl = host(fl)
    key = host(out)[0].astype(np.float64)
    codes, exps = host(gs.codes), host(gs.exps)
    q = philox.measurement_matrix_q(spec.m, spec.n, spec.phi_seed, spec.stream_id)
    s_phi = philox.phi_scale(spec.m)
    a = cs.operator(q, s_phi, spec.block)
    L, _, _ = cs.lipschitz(q, s_phi)
    nb = codes.shape[1]
    rng = np.random.default_rng(1)
    picks = [(t, int(b)) for t in (0, 15, 30) for b in rng.choice(nb, 5, replace=False)]
    picks += [(30, nb - 1), (30, nb - 2)]
    bs = spec.block
    nbx = spec.width // bs
    for t, b in picks:
        y = cs.dequantise(codes[t, b][:, None], exps[t, b:b + 1], s_phi)
        lam = cs.lambdas(a, y)
        s_hat = cs.fista(a, y, lam, L, spec.iters)
        x = cs.synthesise(s_hat, bs)[:, 0].reshape(bs, bs)
        by, bx = divmod(b, nbx)
        sl = (slice(by * bs, by * bs + bs), slice(bx * bs, bx * bs + bs))
        ref = key[sl] + x
        assert np.max(np.abs(fl[t][sl] - ref)) <= MAXABS_TOL, (t, b)


@pytest.mark.parametrize("spec", [sv.qcif_tiny(), sv.vga_precision(0.25, gop=3)],
                         ids=["qcif-b16-m64", "vga-b32-m256"])
def test_decode_of_fp8_measured_gop(ctx, spec):
    """A GOP measured in the FP8 form decodes like the oracle's decode of
    the same FP8 codes (the BF16 bars), and within 0.25 dB of the GOP
    measured exactly (the FP8 operands perturb the measurements by a few
    percent; the oracle shows -0.04..+0.09 dB on these inputs)."""
    import paper_1311_1419_amd as P
    announce(f"decode of fp8-measured {spec.width}x{spec.height} B={spec.block}")
    frames = spec.video()
    op8 = codec.Params.from_spec(spec, measure_form="fp8")
    ref8 = codec.decode_gop(codec.encode_gop(frames, op8), op8)
    p8 = _bf16(spec, flags=P.CSV_FLAG_MEASURE_FP8)
    out8, fl8, _ = ctx.decode_gop(ctx.encode_gop(dev(frames), p8), p8, want_float=True)
    p = _bf16(spec)
    out, _, _ = ctx.decode_gop(ctx.encode_gop(dev(frames), p), p)
    out8, fl8, out = host(out8), host(fl8), host(out)
    for t in range(1, spec.gop):
        assert np.max(np.abs(fl8[t - 1].astype(np.float64) - ref8.cs_float[t - 1])) <= MAXABS_TOL
        assert abs(psnr(frames[t], out8[t]) - psnr(frames[t], ref8.frames[t])) <= PSNR_TOL
        assert abs(psnr(frames[t], out8[t]) - psnr(frames[t], out[t])) <= 0.25


def test_mixed64_batch_sampled_blocks(ctx):
    """The 64-stream mixed workload (176x144 / 352x288 / 640x480, GOP 4-32,
    B 16/32, M/n 0.05-0.4: seven fused classes running side by side) decoded
    as one batch; for one stream of every (B, M) pair the oracle recovers
    three sampled blocks one by one and the GPU's pixels must agree."""
    announce("bf16 mixed 64-stream batch, sampled blocks")
    specs = sv.mixed_streams(64)
    params = [_bf16(s) for s in specs]
    videos = [s.video() for s in specs]
    gss = [ctx.encode_gop(dev(v), p) for v, p in zip(videos, params)]
    outs = ctx.decode_batch(list(zip(gss, params)), want_float=True)
    first = {}
    for i, s in enumerate(specs):
        first.setdefault((s.block, s.m), i)
    rng = np.random.default_rng(64)
    for (bsz, m), i in sorted(first.items()):
        s = specs[i]
        fl = host(outs[i][1])
        key = host(outs[i][0])[0].astype(np.float64)
        codes, exps = host(gss[i].codes), host(gss[i].exps)
        q = philox.measurement_matrix_q(m, s.n, s.phi_seed, s.stream_id)
        s_phi = philox.phi_scale(m)
        a = cs.operator(q, s_phi, bsz)
        L, _, _ = cs.lipschitz(q, s_phi)
        nbx = (s.width + bsz - 1) // bsz
        nb = codes.shape[1]
        for _ in range(3):
            t, b = int(rng.integers(0, s.gop - 1)), int(rng.integers(0, nb))
            y = cs.dequantise(codes[t, b][:, None], exps[t, b:b + 1], s_phi)
            lam = cs.lambdas(a, y)
            x = cs.synthesise(cs.fista(a, y, lam, L, s.iters), bsz)[:, 0].reshape(bsz, bsz)
            by, bx = divmod(b, nbx)
            hh = min(bsz, s.height - by * bsz)
            ww = min(bsz, s.width - bx * bsz)
            sl = (slice(by * bsz, by * bsz + hh), slice(bx * bsz, bx * bsz + ww))
            ref = key[sl] + x[:hh, :ww]
            assert np.max(np.abs(fl[t][sl] - ref)) <= MAXABS_TOL, (i, t, b)


@pytest.fixture(scope="module")
def vga16_items(ctx):
    specs = [sv.vga_precision(0.25, stream=s) for s in range(16)]
    items = []
    for spec in specs:
        p = _bf16(spec)
        items.append((ctx.encode_gop(dev(spec.video()), p), p))
    return items


@pytest.mark.parametrize("variant", range(8))
def test_full_batch_equals_alone(ctx, vga16_items, variant):
    """The 16-camera 640x480 GOP-16 M=256 batch (2256 tiles of 32 blocks:
    persistent workgroups take several tiles and switch between the
    streams' operators) decodes every GOP bit for bit as it decodes alone
    (141 tiles, at most one per workgroup), with every kernel variant of
    the class."""
    import paper_1311_1419_amd as P
    name0, idx0, count = P.kernel_choice(32, 256)
    if variant >= count:
        pytest.skip(f"the class has {count} variants")
    P.set_kernel_choice(32, 256, variant)
    try:
        announce(f"bf16 16 x vga g16 m256 batch vs alone, variant {P.kernel_choice(32, 256)[0]}")
        batch = ctx.decode_batch(vga16_items, want_float=True)
        for i, (gs, p) in enumerate(vga16_items):
            fa = ctx.decode_gop(gs, p, want_float=True)[1]
            assert bool((fa == batch[i][1]).all()), f"stream {i}"
    finally:
        P.set_kernel_choice(32, 256, idx0)


def test_batched_objective_equals_alone(ctx):
    """The FP64 check of a batch runs one launch per (n, M) group; GOPs of
    one group with different block counts (sizes and GOP lengths) give the
    objectives, frames and relative residuals they give decoded alone."""
    announce("bf16 batched FP64 check vs alone")
    specs = [sv.vga_precision(0.25, gop=3, stream=40), sv.qcif_tiny().with_(block=32, m=256, gop=5),
             sv.cif_sweep(4, 0.25, stream=41).with_(block=32, m=256), sv.vga_precision(0.1, gop=2)]
    items = []
    for spec in specs:
        p = _bf16(spec)
        items.append((ctx.encode_gop(dev(spec.video()), p), p))
    batch = ctx.decode_batch(items, want_float=True, want_obj=True)
    for i, (gs, p) in enumerate(items):
        out, fl, obj = ctx.decode_gop(gs, p, want_float=True, want_obj=True)
        assert bool((out == batch[i][0]).all()), f"frames {i}"
        assert bool((obj == batch[i][2]).all()), f"objective {i}"
