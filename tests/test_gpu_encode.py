"""Encoder parity on the GPU: measurement matrix, key-frame codec, integer
measurements, codes, exponents and bit counts must equal the FP64 oracle
bit for bit (all integer-defined: Sections 3.1-3.2, Table I)."""
import numpy as np
import pytest

import synthvid as sv
from oracle import codec, cs, keyframe, philox
from tests.gpu_util import announce, ctx, dev, host  # noqa: F401

pytestmark = pytest.mark.gpu


def _params(spec, **kw):
    import paper_1311_1419_amd as P
    return P.Params.from_spec(spec, precision=P.CSV_FP32, **kw)


@pytest.mark.parametrize("m,b,seed,sid", [(64, 16, 0x1311141900010000, 0), (13, 16, 5, 7),
                                         (256, 32, 0x1311141900030000, 0), (410, 32, 2**63 + 5, 2**32 - 1),
                                         (256, 16, 1, 1), (1, 16, 9, 9)])
def test_phi_matrix_bit_exact(ctx, m, b, seed, sid):
    import paper_1311_1419_amd as P
    announce(f"phi m={m} B={b}")
    p = P.Params(width=64, height=64, gop=2, block=b, m=m, phi_seed=seed, stream_id=sid)
    q = host(ctx.phi_matrix(p))
    assert np.array_equal(q.astype(np.int64), philox.measurement_matrix_q(m, b * b, seed, sid))


@pytest.mark.parametrize("h,w,step", [(144, 176, 16), (288, 352, 16), (480, 640, 16), (16, 8, 1),
                                      (144, 176, 64), (720, 1280, 16)])
def test_key_codec_bit_exact(ctx, h, w, step):
    announce(f"key codec {h}x{w} step {step}")
    rng = np.random.default_rng(h * w + step)
    if h >= 144:
        frame = sv.surveillance_video(sv.VideoSpec(h, w, 1, 3, h + w))[0]
    else:
        frame = rng.integers(0, 256, size=(h, w)).astype(np.uint8)
    lev, bits = ctx.key_encode(dev(frame), step)
    lev_ref = keyframe.encode_levels(frame, step)
    assert np.array_equal(host(lev).astype(np.int64), lev_ref)
    assert int(host(bits)[0]) == keyframe.frame_bits(lev_ref)
    dec = host(ctx.key_decode(lev, step))
    assert np.array_equal(dec, keyframe.decode_levels(lev_ref, step))


def test_key_codec_extreme_blocks(ctx):
    announce("key codec extremes")
    frame = np.zeros((16, 16), dtype=np.uint8)
    frame[:8, 8:] = 255
    frame[8:, :8] = np.indices((8, 8)).sum(0) * 18
    frame[8:, 8:] = (np.indices((8, 8))[0] % 2) * 255
    for step in (1, 2, 16, 256):
        lev, bits = ctx.key_encode(dev(frame), step)
        lev_ref = keyframe.encode_levels(frame, step)
        assert np.array_equal(host(lev).astype(np.int64), lev_ref)
        assert int(host(bits)[0]) == keyframe.frame_bits(lev_ref)
        assert np.array_equal(host(ctx.key_decode(lev, step)), keyframe.decode_levels(lev_ref, step))


@pytest.mark.parametrize("spec", [sv.qcif_tiny(), sv.cif_sweep(4, 0.1), sv.cif_sweep(4, 0.5),
                                  sv.vga_precision(0.25, gop=3), sv.vga_precision(0.1, gop=3),
                                  sv.qcif_tiny().with_(block=32, m=256),
                                  sv.qcif_tiny().with_(block=32, m=1024)],
                         ids=["qcif-b16-m64", "cif-m26", "cif-m128", "vga-m256", "vga-m102",
                              "qcif-b32-m256-padded", "qcif-b32-m1024-full"])
def test_measure_frame_bit_exact(ctx, spec):
    announce(f"measure {spec.width}x{spec.height} B={spec.block} M={spec.m}")
    frames = spec.video(2)
    p = _params(spec)
    key_dec = keyframe.decode_levels(keyframe.encode_levels(frames[0], 16), 16)
    y, codes, exps = ctx.measure_frame(p, dev(frames[1]), dev(key_dec))
    q = philox.measurement_matrix_q(spec.m, spec.n, spec.phi_seed, spec.stream_id)
    y_ref = cs.measure(q, cs.gather_blocks(frames[1].astype(np.int64) - key_dec, spec.block))
    c_ref, e_ref = cs.quantise(y_ref)
    assert np.array_equal(host(y).astype(np.int64), y_ref.T)
    assert np.array_equal(host(codes), c_ref.T)
    assert np.array_equal(host(exps), e_ref)


@pytest.mark.parametrize("spec", [sv.qcif_tiny(), sv.cif_sweep(8, 0.2), sv.vga_precision(0.25),
                                  sv.qcif_tiny().with_(block=32, m=102, gop=5),
                                  sv.qcif_tiny().with_(gop=1)],
                         ids=["qcif", "cif-g8", "vga-g16", "qcif-b32-padded", "key-only"])
def test_encode_gop_bit_exact(ctx, spec):
    announce(f"encode_gop {spec.width}x{spec.height} G={spec.gop} B={spec.block} M={spec.m}")
    frames = spec.video()
    p = _params(spec)
    gs = ctx.encode_gop(dev(frames), p)
    ref = codec.encode_gop(frames, codec.Params.from_spec(spec))
    assert np.array_equal(host(gs.key_levels).astype(np.int64), ref.key_levels)
    if spec.gop > 1:
        assert np.array_equal(host(gs.codes), ref.codes)
        assert np.array_equal(host(gs.exps), ref.exps)
    bits = host(gs.bits)
    assert int(bits[0]) == ref.bits_key and int(bits[1]) == ref.bits_cs
    cr = ctx.compression_ratio(p, int(bits[0]), int(bits[1])) if spec.gop > 1 else None
    if cr:
        ref_cr = codec.cr_from_bits(codec.Params.from_spec(spec), ref.bits_key, ref.bits_cs)
        assert cr["total"] == pytest.approx(ref_cr["total"], rel=1e-12)


def test_encode_deterministic(ctx):
    announce("encode determinism")
    spec = sv.cif_sweep(4, 0.3)
    frames = dev(spec.video())
    p = _params(spec)
    a = ctx.encode_gop(frames, p)
    b = ctx.encode_gop(frames, p)
    assert np.array_equal(host(a.codes), host(b.codes))
    assert np.array_equal(host(a.exps), host(b.exps))


def test_probe_ceilings_are_plausible(ctx):
    announce("probe_ceilings")
    held = ctx.bytes_held()
    c = ctx.probe_ceilings()
    assert ctx.bytes_held() == held            # probe buffers are freed again
    assert c["compute_units"] > 0
    # MI355X: 2.5 PF dense BF16, 8 TB/s HBM; the probes reach a large part
    # of those and L2/LDS stream faster than HBM
    assert 500.0 < c["mfma_bf16_tflops"] < 2600.0
    assert 1.0 < c["hbm_read_tbs"] < 8.5
    assert c["l2_read_tbs"] > c["hbm_read_tbs"]
    assert c["lds_read_tbs"] > c["l2_read_tbs"]


def test_encode_batch_equals_oracle_per_gop(ctx):
    """A batch of GOPs of different sizes, block sizes, M and GOP lengths
    (including a key-only GOP) encodes to exactly the oracle's streams."""
    specs = [sv.qcif_tiny(), sv.cif_sweep(4, 0.1, stream=1), sv.qcif_tiny().with_(gop=1),
             sv.qcif_tiny().with_(block=32, m=102, gop=3), sv.cif_sweep(4, 0.5, stream=2),
             sv.qcif_tiny(stream=3)]
    announce(f"encode_batch of {len(specs)} GOPs")
    vids = [s.video() for s in specs]
    items = [(dev(v), _params(s)) for v, s in zip(vids, specs)]
    outs = ctx.encode_batch(items)
    for spec, v, gs in zip(specs, vids, outs):
        ref = codec.encode_gop(v, codec.Params.from_spec(spec))
        assert np.array_equal(host(gs.key_levels).astype(np.int64), ref.key_levels)
        if spec.gop > 1:
            assert np.array_equal(host(gs.codes), ref.codes)
            assert np.array_equal(host(gs.exps), ref.exps)
        bits = host(gs.bits)
        assert int(bits[0]) == ref.bits_key and int(bits[1]) == ref.bits_cs


FORM_SPECS = [(sv.qcif_tiny(), "qcif-b16"), (sv.cif_sweep(4, 0.3), "cif-m77"),
              (sv.vga_precision(0.25, gop=3), "vga-b32-m256"),
              (sv.qcif_tiny().with_(block=32, m=410, gop=2), "qcif-b32-m410-padded")]


@pytest.mark.parametrize("form", ["int8", "fp8"])
@pytest.mark.parametrize("spec", [s for s, _ in FORM_SPECS], ids=[i for _, i in FORM_SPECS])
def test_measurement_forms_bit_exact(ctx, spec, form):
    """INT8 (split residual) and FP8 (E4M3) measurement forms equal the
    oracle's definition of each form bit for bit: measurements, codes,
    exponents and bit counts."""
    import paper_1311_1419_amd as P
    announce(f"measure form {form} {spec.width}x{spec.height} B={spec.block} M={spec.m}")
    flag = P.CSV_FLAG_MEASURE_INT8 if form == "int8" else P.CSV_FLAG_MEASURE_FP8
    frames = spec.video()
    p = _params(spec, flags=flag)
    gs = ctx.encode_gop(dev(frames), p)
    ref = codec.encode_gop(frames, codec.Params.from_spec(spec, measure_form=form))
    assert np.array_equal(host(gs.codes), ref.codes)
    assert np.array_equal(host(gs.exps), ref.exps)
    bits = host(gs.bits)
    assert int(bits[0]) == ref.bits_key and int(bits[1]) == ref.bits_cs
    # the raw integer measurements of one CS frame
    key = dev(ref.key_decoded)
    y, codes, exps = ctx.measure_frame(p, dev(frames[1]), key)
    assert np.array_equal(host(y).astype(np.int64), ref.y_int[0])
