"""Decoder parity of the plain FP32 path against the FP64 oracle.

Tolerances (FP32 arithmetic, 200-300 FISTA iterations): recovered float
frames within 0.05 grey levels, per-frame PSNR within 0.01 dB, uint8 frames
differing by at most one level (a rounding tie can fall either way), lambda
and the FP64 objective within 1e-5 relative, the relative residual within
2e-5 absolute.  The step constant is an FP64
power iteration on both sides: 1e-9 relative."""
import numpy as np
import pytest

import synthvid as sv
from oracle import codec, cs, philox
from tests.gpu_util import announce, ctx, dev, host, psnr  # noqa: F401

pytestmark = pytest.mark.gpu


def _gpu_params(spec, **kw):
    import paper_1311_1419_amd as P
    return P.Params.from_spec(spec, precision=P.CSV_FP32, **kw)


@pytest.mark.parametrize("m,b", [(64, 16), (13, 16), (51, 16), (128, 16), (200, 16), (256, 32),
                                 (410, 32), (1024, 32),
                                 # edges of the register-form tile sizes (32, 64, 128, 256 rows)
                                 (1, 16), (32, 16), (33, 16), (129, 16), (257, 32),
                                 # last one-workgroup memory form, first many-workgroup form
                                 (320, 32), (321, 32)])
def test_step_constant_and_operator(ctx, m, b):
    import paper_1311_1419_amd as P
    announce(f"operator/L m={m} B={b}")
    p = P.Params(width=64, height=64, gop=2, block=b, m=m, phi_seed=77 + m, stream_id=b)
    L, it = ctx.step_constant(p)
    q = philox.measurement_matrix_q(m, b * b, 77 + m, b)
    s_phi = philox.phi_scale(m)
    L_ref, _, it_ref = cs.lipschitz(q, s_phi)
    assert L == pytest.approx(L_ref, rel=1e-9)
    # the same iteration, summed in another order: the stopping test may flip
    # by a step where the relative change sits at the tolerance
    assert abs(it - it_ref) <= 2
    a = host(ctx.operator_matrix(p))
    assert np.max(np.abs(a - cs.operator(q, s_phi, b))) < 1e-12


def _decode_compare(ctx, spec, flags=0, max_abs=0.05, max_relres=2e-5, **okw):
    frames = spec.video()
    p = _gpu_params(spec, flags=flags)
    op = codec.Params.from_spec(spec, **okw)
    ref_stream = codec.encode_gop(frames, op)
    ref = codec.decode_gop(ref_stream, op)
    gs = ctx.encode_gop(dev(frames), p)
    out, fl, obj = ctx.decode_gop(gs, p, want_float=True, want_obj=True)
    out, fl, obj = host(out), host(fl), host(obj)
    assert np.array_equal(out[0], ref.frames[0])
    for t in range(1, spec.gop):
        err = np.max(np.abs(fl[t - 1].astype(np.float64) - ref.cs_float[t - 1]))
        assert err <= max_abs, f"frame {t}: max abs {err}"
        assert np.max(np.abs(out[t].astype(int) - ref.frames[t].astype(int))) <= 1
        assert abs(psnr(frames[t], out[t]) - psnr(frames[t], ref.frames[t])) <= 0.01
    rel = np.abs(obj[..., 0] - ref.objective) / np.maximum(ref.objective, 1e-300)
    assert np.max(rel) <= 1e-5
    # ||A s - y|| / ||y|| is a few percent: FP32 error in s shows up as an
    # absolute error of the order 1e-5 (in units of ||y||)
    assert np.max(np.abs(obj[..., 1] - ref.rel_residual)) <= max_relres
    return out, ref


@pytest.mark.parametrize("spec", [sv.qcif_tiny(), sv.cif_sweep(4, 0.1, iters=300),
                                  sv.cif_sweep(4, 0.5, iters=300),
                                  sv.qcif_tiny().with_(block=32, m=256, gop=3),
                                  sv.qcif_tiny().with_(m=150, gop=2),
                                  sv.qcif_tiny().with_(block=32, m=300, gop=2)],
                         ids=["qcif-tiny", "cif-m26", "cif-m128", "qcif-b32-padded",
                              "qcif-m150-mp160", "qcif-b32-m300-mp320"])
def test_decode_fp32_matches_oracle(ctx, spec):
    announce(f"decode fp32 {spec.width}x{spec.height} G={spec.gop} B={spec.block} M={spec.m}")
    _decode_compare(ctx, spec)


def test_decode_fp32_ista_and_pixel_lambda(ctx):
    import paper_1311_1419_amd as P
    announce("decode fp32 ISTA + pixel-domain lambda")
    spec = sv.qcif_tiny().with_(gop=2, iters=60)
    _decode_compare(ctx, spec, flags=P.CSV_FLAG_ISTA | P.CSV_FLAG_LAMBDA_PIXEL_DOMAIN,
                    solver="ista", pixel_domain_lambda=True)


def test_lambda_and_coefficients(ctx):
    announce("recover_blocks fp32 lambda/coefficients")
    spec = sv.qcif_tiny()
    frames = spec.video()
    op = codec.Params.from_spec(spec)
    st = codec.encode_gop(frames, op)
    p = _gpu_params(spec)
    codes = st.codes.reshape(-1, spec.m)
    exps = st.exps.reshape(-1)
    s, lam, obj = ctx.recover_blocks(p, dev(codes), dev(exps), want_obj=True)
    s, lam = host(s), host(lam)
    q = philox.measurement_matrix_q(spec.m, spec.n, spec.phi_seed, spec.stream_id)
    s_phi = philox.phi_scale(spec.m)
    a = cs.operator(q, s_phi, spec.block)
    y = cs.dequantise(codes.T, exps, s_phi)
    lam_ref = cs.lambdas(a, y)
    assert np.allclose(lam, lam_ref, rtol=1e-5, atol=1e-6)
    L, _, _ = cs.lipschitz(q, s_phi)
    s_ref = cs.fista(a, y, lam_ref, L, spec.iters).T
    scale = np.maximum(np.abs(s_ref).max(axis=1, keepdims=True), 1.0)
    assert np.max(np.abs(s - s_ref) / scale) < 1e-3


def test_zero_residual_and_key_only(ctx):
    announce("static video (zero residual) and key-only GOP")
    spec = sv.qcif_tiny()
    frames = spec.video(1)
    static = np.repeat(frames, 4, axis=0)
    p = _gpu_params(spec)
    gs = ctx.encode_gop(dev(static), p)
    out, fl, obj = ctx.decode_gop(gs, p, want_float=True, want_obj=True)
    out = host(out)
    key = out[0]
    # residual F_t - F^_key is the key coding error: not zero, but identical for every CS frame
    assert np.array_equal(host(gs.codes)[0], host(gs.codes)[1])
    assert np.array_equal(out[1], out[2]) and np.array_equal(out[2], out[3])
    # a frame equal to the decoded key has an all-zero residual -> codes 0, s = 0
    z = np.stack([frames[0], key, key])
    p3 = _gpu_params(spec.with_(gop=3))
    gs3 = ctx.encode_gop(dev(z), p3)
    assert not host(gs3.codes).any() and not host(gs3.exps).any()
    out3, fl3, obj3 = ctx.decode_gop(gs3, p3, want_float=True, want_obj=True)
    assert np.array_equal(host(out3)[1], key) and np.all(host(fl3)[0] == key)
    assert np.all(host(obj3) == 0)
    p1 = _gpu_params(spec.with_(gop=1))
    gs1 = ctx.encode_gop(dev(frames), p1)
    out1, _, _ = ctx.decode_gop(gs1, p1)
    assert np.array_equal(host(out1)[0], key)


def test_decode_deterministic(ctx):
    announce("decode fp32 determinism")
    spec = sv.cif_sweep(4, 0.2, iters=100)
    p = _gpu_params(spec)
    gs = ctx.encode_gop(dev(spec.video()), p)
    a = host(ctx.decode_gop(gs, p, want_float=True)[1])
    b = host(ctx.decode_gop(gs, p, want_float=True)[1])
    assert np.array_equal(a, b)


def test_bad_params_rejected(ctx):
    import paper_1311_1419_amd as P
    announce("bad params")
    spec = sv.qcif_tiny()
    frames = dev(spec.video())
    for bad in (dict(block=8), dict(m=257), dict(iters=0), dict(key_qstep=12)):
        with pytest.raises(P.CsvError):
            ctx.encode_gop(frames, _gpu_params(spec).with_(**bad))
    for bad in (dict(gop=0), dict(width=170), dict(m=0, rho=0.0), dict(lambda_frac=-1.0)):
        with pytest.raises(P.CsvError):
            _gpu_params(spec).with_(**bad).resolve()


def test_context_memory_budget(ctx):
    """A context whose budget cannot hold a stream's operator and working
    set refuses with CSV_ENOMEM instead of allocating past it, and stays
    usable for a GOP that fits."""
    import paper_1311_1419_amd as P
    from paper_1311_1419_amd import _native as N
    announce("context memory budget")
    big = sv.vga_precision(0.25, gop=2)
    small = sv.qcif_tiny()
    with P.Context(0, mem_budget=4 << 20) as c:
        with pytest.raises(P.CsvError) as ei:
            c.decode_gop(c.encode_gop(dev(big.video()), _gpu_params(big)), _gpu_params(big))
        assert ei.value.code == N.CSV_ENOMEM
        frames = small.video()
        op = codec.Params.from_spec(small)
        ref = codec.decode_gop(codec.encode_gop(frames, op), op)
        out, _, _ = c.decode_gop(c.encode_gop(dev(frames), _gpu_params(small)), _gpu_params(small))
        assert np.array_equal(host(out)[0], ref.frames[0])


def test_full_sampling_fp32_and_bf16_refusal(ctx):
    """M = n (B = 16, M = 256: A is square and invertible) decodes on the
    plain FP32 path to the FP32 bars; the fused BF16 path has no kernel for
    a padded M above 128 at n = 256 and refuses with CSV_EUNSUPPORTED
    before launching anything, leaving the context usable."""
    import paper_1311_1419_amd as P
    announce("full sampling M = n, fp32 decode and bf16 refusal")
    spec = sv.qcif_tiny().with_(m=256, gop=2)
    _decode_compare(ctx, spec)
    pb = P.Params.from_spec(spec, precision=P.CSV_BF16)
    gs = ctx.encode_gop(dev(spec.video()), pb)
    with pytest.raises(P.CsvError) as ei:
        ctx.decode_gop(gs, pb)
    assert ei.value.code == P._native.CSV_EUNSUPPORTED
    _decode_compare(ctx, sv.qcif_tiny().with_(gop=2))


def test_fp32_batch_equals_alone(ctx):
    """The plain FP32 path decodes a batch group by group (GOPs of one
    (n, M, T) shape share each product launch, every GOP with its own
    operator and block count) and prepares the GOPs on four streams; each
    GOP's frames, float frames and FP64 objectives equal those of the GOP
    decoded alone, bit for bit.  Five GOPs: two groups of two (different
    streams and sizes) and one alone, so the fifth wraps to the first
    stream."""
    announce("fp32 batch vs alone (5 GOPs, 3 shape groups)")
    specs = [sv.qcif_tiny(), sv.cif_sweep(4, 0.1, stream=1), sv.qcif_tiny(stream=3),
             sv.qcif_tiny().with_(block=32, m=102, stream_id=9, phi_seed=99),
             sv.cif_sweep(4, 0.1, stream=2).with_(width=176, height=144)]
    items = []
    for spec in specs:
        p = _gpu_params(spec)
        items.append((ctx.encode_gop(dev(spec.video()), p), p))
    batch = ctx.decode_batch(items, want_float=True, want_obj=True)
    for i, (gs, p) in enumerate(items):
        out, fl, obj = ctx.decode_gop(gs, p, want_float=True, want_obj=True)
        bo, bf, bj = batch[i]
        assert np.array_equal(host(out), host(bo)), f"frames {i}"
        assert np.array_equal(host(fl), host(bf)), f"float frames {i}"
        assert np.array_equal(host(obj), host(bj)), f"objective {i}"


@pytest.mark.parametrize("rho", [0.25, 0.1], ids=["m256", "m102"])
def test_fp32_full_vga_frames_vs_oracle(ctx, rho):
    """The benchmark's frame shape on the plain FP32 path: 640x480, B = 32
    (n = 1024), M = 256 or 102, two CS frames (600 blocks: four full
    128-row GEMM tiles and a ragged fifth) against the oracle at the FP32
    bars."""
    spec = sv.vga_precision(rho=rho, gop=3)
    announce(f"decode fp32 full VGA G=3 B=32 M={spec.m}")
    _decode_compare(ctx, spec)


@pytest.mark.parametrize("gop", [8, 16])
def test_fp32_cif_rho02_long_gops_vs_oracle(ctx, gop):
    """CIF at M/n = 0.2 (M = 51, padded to 64) with GOPs of 8 and 16 frames
    (2772 and 5940 blocks in one launch) against the oracle."""
    spec = sv.cif_sweep(gop, 0.2, iters=300)
    announce(f"decode fp32 CIF rho=0.2 G={gop}")
    _decode_compare(ctx, spec)


def test_fp32_monotone_matches_oracle_mfista(ctx):
    """CSV_FLAG_MONOTONE (MFISTA) against the oracle's monotone FISTA, on a
    QCIF GOP at M = 64 and a padded B = 32 GOP: objective (1e-5 relative),
    relative residual, PSNR (0.01 dB) and uint8 frames at the FP32 bars; the
    float frames within 0.5 grey levels.  MFISTA's per-block choice between
    z_k and s_{k-1} compares two objectives that differ by about 1e-6 near
    convergence, so FP32 and FP64 rounding take different branches and the
    iterates drift apart along the objective's flat directions: an FP32
    emulation of the same steps differs from the FP64 oracle by up to 0.10
    grey levels and 6.5e-5 in relative residual at T = 200 with the
    objective within 2.4e-6; the relative residual bar is 5e-4."""
    import paper_1311_1419_amd as P
    for spec in (sv.qcif_tiny(), sv.qcif_tiny().with_(block=32, m=256, gop=3)):
        announce(f"decode fp32 MONOTONE B={spec.block} M={spec.m}")
        _decode_compare(ctx, spec, flags=P.CSV_FLAG_MONOTONE, max_abs=0.5, max_relres=5e-4,
                        solver="mfista")


def test_fp32_monotone_objective_never_increases(ctx):
    """MFISTA's objective is non-increasing in the iteration count on the
    GPU too.  The oracle's plain FISTA history names an iteration k where
    plain FISTA's objective rises (by about 2e-4 relative on this clip); on
    the GPU plain FISTA rises there as well, while under CSV_FLAG_MONOTONE
    the FP64 objective of every block after T = 5, 10, 20, 40, k, k + 1, 160
    iterations never rises by more than the FP32 rounding of the decision
    (1e-6 relative)."""
    import paper_1311_1419_amd as P
    announce("fp32 MONOTONE objective sequence")
    spec = sv.qcif_tiny().with_(gop=2)
    frames = spec.video()
    op = codec.Params.from_spec(spec)
    st = codec.encode_gop(frames, op)
    q = philox.measurement_matrix_q(spec.m, spec.n, spec.phi_seed, spec.stream_id)
    s_phi = philox.phi_scale(spec.m)
    a = cs.operator(q, s_phi, spec.block)
    y = cs.dequantise(st.codes[0].T, st.exps[0], s_phi)
    lam = cs.lambdas(a, y)
    L, _, _ = cs.lipschitz(q, s_phi)
    _, hist = cs.fista(a, y, lam, L, 150, history=True)
    hist = np.stack(hist)
    rises = np.where(((hist[1:] - hist[:-1]) / hist[:-1] > 1e-4).any(axis=1))[0]
    assert rises.size, "the clip should show plain FISTA's objective rising"
    k = int(rises[0]) + 1   # F(s_k) < F(s_{k+1}) on some block

    def objective_after(T, flags):
        p = _gpu_params(spec.with_(iters=T), flags=flags)
        gs = ctx.encode_gop(dev(frames), p)
        _, _, obj = ctx.decode_gop(gs, p, want_obj=True)
        return host(obj)[0, :, 0]

    plain = np.stack([objective_after(T, 0) for T in (k, k + 1)])
    assert np.max((plain[1] - plain[0]) / plain[0]) > 1e-5
    mono = np.stack([objective_after(T, P.CSV_FLAG_MONOTONE)
                     for T in sorted({5, 10, 20, 40, k, k + 1, 160})])
    rise = np.max((mono[1:] - mono[:-1]) / np.maximum(mono[:-1], 1e-30))
    assert rise <= 1e-6, rise


def test_no_quant_closed_loop_cancels_key_error(ctx):
    """Eqs. (2)-(4) on the GPU: with CSV_FLAG_NO_QUANT (exact int32
    measurements), full sampling M = n and lambda = 0, the decoded CS frames
    equal the originals to within the solver's convergence (0.5 grey levels
    after 3000 iterations) although the decoded key frame they are built on
    is off by 10 or more levels: the key frame's coding error cancels.  The
    decoded floats also match the oracle's decode of the same measurements."""
    import paper_1311_1419_amd as P
    base = sv.qcif_tiny()
    frames = base.video(3)[:, :48, :48].copy()
    for qstep in (16, 64):
        spec = base.with_(height=48, width=48, gop=3, m=256, iters=3000, key_qstep=qstep,
                          lambda_frac=0.0)
        announce(f"fp32 NO_QUANT M=n lambda=0 key step {qstep}")
        p = _gpu_params(spec, flags=P.CSV_FLAG_NO_QUANT)
        gs = ctx.encode_gop(dev(frames), p)
        assert gs.codes.dtype == __import__("torch").int32
        out, fl, _ = ctx.decode_gop(gs, p, want_float=True)
        out, fl = host(out), host(fl)
        key_err = np.max(np.abs(out[0].astype(int) - frames[0].astype(int)))
        assert key_err >= 10
        cs_err = np.max(np.abs(fl - frames[1:].astype(np.float64)))
        assert cs_err <= 0.5, cs_err
        op = codec.Params.from_spec(spec, no_quant=True)
        ref_stream = codec.encode_gop(frames, op)
        assert np.array_equal(host(gs.codes), ref_stream.y_int.astype(np.int32))
        ref = codec.decode_gop(ref_stream, op)
        assert np.max(np.abs(fl - ref.cs_float)) <= 0.05


def test_batched_operator_setup_equals_single():
    """A batch decode that meets several new streams builds their operators
    together (their power iterations side by side in one launch); every
    step constant equals the one a fresh context computes for that stream
    alone, bit for bit (the same iteration in the same order), and equals
    the oracle's within 1e-9."""
    import paper_1311_1419_amd as P
    announce("batched operator setup vs single")
    specs = [sv.qcif_tiny().with_(stream_id=60 + k, phi_seed=600 + k, m=[26, 64, 13, 100, 64][k],
                                  gop=2, iters=20) for k in range(5)]
    specs.append(sv.vga_precision(0.25, gop=2, stream=7).with_(iters=20))
    specs.append(sv.vga_precision(0.3, gop=2, stream=8).with_(iters=20))   # M > 256: G from memory
    params = [_gpu_params(s) for s in specs]
    assert specs[-1].m > 256
    with P.Context(0) as c1:
        # one batch encode meets all the new streams at once: their operators
        # are built together (one power-iteration launch per register-form size)
        streams = c1.encode_batch([(dev(s.video()), p) for s, p in zip(specs, params)])
        c1.decode_batch(list(zip(streams, params)))
        batched = [c1.step_constant(p) for p in params]
    with P.Context(0) as c2:
        single = [c2.step_constant(p) for p in params]
    assert batched == single
    for s, (L, _) in zip(specs, batched):
        q = philox.measurement_matrix_q(s.m, s.n, s.phi_seed, s.stream_id)
        L_ref, _, _ = cs.lipschitz(q, philox.phi_scale(s.m))
        assert L == pytest.approx(L_ref, rel=1e-9)
