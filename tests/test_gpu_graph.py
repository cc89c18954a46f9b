"""Graph replay of a captured batch decode: every replay, interleaved with
eager work (new GOPs encoded into the bound buffers, other decodes,
synchronisations), must equal an eager decode of the same inputs."""
import numpy as np
import pytest
import torch

import synthvid as sv
from tests.gpu_util import announce, ctx, dev, host  # noqa: F401

pytestmark = pytest.mark.gpu


def test_graph_replays_match_eager(ctx):
    import paper_1311_1419_amd as P
    announce("graph capture + replays")
    specs = [sv.qcif_tiny(), sv.cif_sweep(4, 0.1, stream=1), sv.vga_precision(0.25, gop=3, stream=2),
             sv.qcif_tiny().with_(block=32, m=102, stream_id=9, phi_seed=99)]
    params = [P.Params.from_spec(s, precision=P.CSV_BF16) for s in specs]
    bufs = [ctx.alloc_stream(p) for p in params]
    for s, p, b in zip(specs, params, bufs):
        ctx.encode_gop(dev(s.video()), p, out=b)
    st = torch.cuda.Stream()
    g = ctx.capture_batch(list(zip(bufs, params)), st, want_float=True)
    for rep in range(4):
        # new inputs in the bound buffers (eager encode of shifted videos)
        for k, (s, p, b) in enumerate(zip(specs, params, bufs)):
            vid = sv.surveillance_video(sv.VideoSpec(s.height, s.width, s.gop, s.n_objects,
                                                     s.video_seed + 17 * (rep + 1)))
            ctx.encode_gop(dev(vid), p, out=b)
        torch.cuda.synchronize()
        eager = ctx.decode_batch(list(zip(bufs, params)), want_float=True)
        eager = [(host(f), host(fl)) for f, fl, _ in eager]
        g.launch(st)
        st.synchronize()
        for (f, fl, _), (ef, efl) in zip(g.outputs, eager):
            assert np.array_equal(host(f), ef), f"replay {rep}"
            assert np.array_equal(host(fl), efl), f"replay {rep}"
    g.close()


def _replays_match(ctx, specs_params, make_video, reps=3):
    """Capture the decode of (spec, params) items, then replay it `reps`
    times with new GOPs encoded into the bound buffers in between; every
    replay must equal an eager decode of the same inputs."""
    bufs = [ctx.alloc_stream(p) for _, p in specs_params]
    for (s, p), b in zip(specs_params, bufs):
        ctx.encode_gop(dev(make_video(s, 0)), p, out=b)
    items = [(b, p) for b, (_, p) in zip(bufs, specs_params)]
    st = torch.cuda.Stream()
    g = ctx.capture_batch(items, st, want_float=True, want_obj=True)
    for rep in range(reps):
        for (s, p), b in zip(specs_params, bufs):
            ctx.encode_gop(dev(make_video(s, rep + 1)), p, out=b)
        torch.cuda.synchronize()
        eager = ctx.decode_batch(items, want_float=True, want_obj=True)
        eager = [(host(f), host(fl), host(ob)) for f, fl, ob in eager]
        g.launch(st)
        st.synchronize()
        for (f, fl, ob), (ef, efl, eob) in zip(g.outputs, eager):
            assert np.array_equal(host(f), ef), f"replay {rep}"
            assert np.array_equal(host(fl), efl), f"replay {rep}"
            assert np.array_equal(host(ob), eob), f"replay {rep}"
    g.close()


def _shifted(s, k):
    return sv.surveillance_video(sv.VideoSpec(s.height, s.width, s.gop, s.n_objects,
                                              s.video_seed + 17 * k))


def test_graph_replays_tv_bf16_batch(ctx):
    """The fused BF16 TV kernel and the fused l1 kernel in one captured batch."""
    import paper_1311_1419_amd as P
    announce("graph capture + replays: BF16 TV and l1")
    specs = [sv.qcif_tiny(), sv.cif_sweep(4, 0.3, stream=3)]
    items = [(specs[0], P.Params.from_spec(specs[0], precision=P.CSV_BF16, flags=P.CSV_FLAG_TV)),
             (specs[1], P.Params.from_spec(specs[1], precision=P.CSV_BF16, flags=P.CSV_FLAG_TV)),
             (specs[0], P.Params.from_spec(specs[0].with_(stream_id=11), precision=P.CSV_BF16))]
    _replays_match(ctx, items, _shifted)


def test_graph_replays_fp32_tv_and_whole_frame_batch(ctx):
    """FP32 batch: two whole-frame TV GOPs of one shape (shared launches), a
    block TV GOP and an l1 GOP."""
    import paper_1311_1419_amd as P
    announce("graph capture + replays: FP32 whole-frame TV, block TV, l1")
    spec = sv.qcif_tiny().with_(gop=3)
    whole = dict(precision=P.CSV_FP32, flags=P.CSV_FLAG_TV | P.CSV_FLAG_WHOLE_FRAME, m=300,
                 iters=40)
    items = [(spec, P.Params.from_spec(spec, **whole)),
             (spec, P.Params.from_spec(spec.with_(stream_id=21), **whole)),
             (spec, P.Params.from_spec(spec.with_(stream_id=22), precision=P.CSV_FP32,
                                       flags=P.CSV_FLAG_TV, iters=60)),
             (spec, P.Params.from_spec(spec.with_(stream_id=23), precision=P.CSV_FP32, iters=60))]
    _replays_match(ctx, items, _shifted)


def test_graph_launch_refuses_after_scratch_moved():
    """A larger eager decode on the graph's context moves scratch buffers
    the captured graph points into; the next launch must refuse with
    CSV_EINVAL before any GPU work instead of replaying into freed memory.
    A recaptured graph then replays correctly."""
    import paper_1311_1419_amd as P
    announce("graph launch after scratch growth")
    small = sv.qcif_tiny().with_(gop=2)
    big = sv.vga_precision(0.25, gop=3, stream=4)
    with P.Context(0) as c:
        ps = P.Params.from_spec(small, precision=P.CSV_BF16)
        pb = P.Params.from_spec(big, precision=P.CSV_BF16)
        bs, bb = c.alloc_stream(ps), c.alloc_stream(pb)
        c.encode_gop(dev(small.video()), ps, out=bs)
        c.encode_gop(dev(big.video()), pb, out=bb)
        st = torch.cuda.Stream()
        g = c.capture_batch([(bs, ps)], st)
        g.launch(st)
        st.synchronize()
        c.decode_batch([(bb, pb)])          # grows the context's scratch
        torch.cuda.synchronize()
        with pytest.raises(P.CsvError) as ei:
            g.launch(st)
        assert ei.value.code == -1 and "recapture" in str(ei.value)
        g.close()
        g2 = c.capture_batch([(bs, ps)], st)
        g2.launch(st)
        st.synchronize()
        eager = c.decode_batch([(bs, ps)])
        assert np.array_equal(host(g2.outputs[0][0]), host(eager[0][0]))
        g2.close()
