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
