"""Benchmark: recovered Mpixel/s of the CS video decoder on one MI355X.

Workload (one step): 16 synthetic 640x480 surveillance cameras, one GOP of
16 frames each (1 key + 15 CS frames), 32x32 blocks (n = 1024), M/n = 0.25
(M = 256), 300 FISTA iterations.  A step encodes the 16 GOPs as one batch
(key-frame codec, closed-loop residual, measurement, quantiser) and decodes
them as one batch (key frames, dequantisation, lambda, one fused recovery launch,
synthesis, FP64 final objective).  Frames are resident in HBM before the
timed region; per-stream measurement operators are built in the warm-up.

Prints one JSON line.  `value` is the fused BF16 path; the plain FP32 path
runs the same workload beside it for the BF16-vs-FP32 comparison and the
PSNR loss.  The roofline object covers the fused recovery kernel, timed
with HIP events on its own stream inside the timed region.
"""
from __future__ import annotations

import argparse
import collections
import json
import re
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "recovered Mpixel/s at M/n=0.25, BF16-MFMA vs FP32, ≤0.1dB PSNR loss; p99 ms"
KERNEL_SRC = [os.path.join(ROOT, "paper_1311_1419_amd", "csrc", f)
              for f in ("k_fista_bf16.hip", "fused_common.h")]


def kernel_source_digest():
    """sha256 of the profiled kernel's source: the fista_bf16_kernel template
    (k_fista_bf16.hip, up to its launcher) followed by fused_common.h, so the
    variant table can change without voiding the counters."""
    import hashlib
    txt = open(KERNEL_SRC[0]).read()
    a = txt.index("template <int N, int MP, int CT, int W, int kPF")
    b = txt.index("template <int N, int MP, int CT, int W, int PF,", a)
    return hashlib.sha256((txt[a:b] + open(KERNEL_SRC[1]).read()).encode()).hexdigest()
PMC_SUMMARY = os.path.join(ROOT, "profiles", "fista_bf16_vga640x480_m256_x16_pmc.md")
PEAK_BF16_TFLOPS = 2500.0      # MI355X dense BF16 MFMA
WORKLOAD = "vga640x480-g16-b32-m256-t300-x16streams"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--streams", type=int, default=16)
    ap.add_argument("--fp32-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the device-ceiling microbenchmarks")
    ap.add_argument("--cpu-blocks", type=int, default=3000,
                    help="blocks the oracle recovers for the CPU baseline")
    ap.add_argument("--cpu-blocks-1t", type=int, default=400,
                    help="blocks the oracle recovers on one thread for the CPU baseline")
    ap.add_argument("--variant", type=str, default="",
                    help="headline mode: run the (n=1024, M_p=256) class with this named kernel "
                         "variant instead of its default (e.g. q8_w8_pf2x2_pa2x2)")
    ap.add_argument("--headline-serve-load", type=float, default=0.16,
                    help="headline mode: one serving point at this fraction of the 256 "
                         "cameras' nominal GOP rates (0: none)")
    ap.add_argument("--headline-serve-window", type=float, default=1.0,
                    help="headline mode: seconds of Poisson arrivals in that point")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one device-to-device copy of this size (counter calibration)")
    ap.add_argument("--mode", choices=["headline", "mixed", "serve", "encode", "configure", "tv",
                                       "whole", "fp32", "b16", "setup"],
                    default="headline",
                    help="headline: the metric above; mixed: 64 mixed streams decoded by one "
                         "graph-captured batch; serve: 256 cameras under a Poisson load sweep; "
                         "encode: the headline cameras encoded in each measurement form; "
                         "configure: the (G, M) configurator sweep; tv: TV recovery vs l1; "
                         "whole: whole-frame measurement with Q regenerated on the fly; "
                         "fp32: the plain FP32 path alone on the headline workload; "
                         "b16: the fused path on 16 x 352x288 GOP-16 B=16 M=64 cameras; "
                         "setup: a new stream's operator and step constant per (M, n)")
    ap.add_argument("--psnr-floor", type=float, default=32.0,
                    help="configure mode: PSNR floor standing in for the tracking requirement")
    ap.add_argument("--serve-window", type=float, default=2.0, help="seconds per sweep point")
    ap.add_argument("--serve-streams", type=int, default=2,
                    help="HIP streams the server spreads consecutive batches over (1-4)")
    ap.add_argument("--serve-loads", type=str, default="0.01,0.02,0.04,0.08,0.16,0.24,0.32",
                    help="fractions of the cameras' nominal GOP rates")
    return ap.parse_args()


def make_streams(n_streams):
    import synthvid as sv
    return [sv.vga_precision(0.25, stream=s) for s in range(n_streams)]


def psnr(ref, test):
    d = ref.astype(np.float64) - test.astype(np.float64)
    mse = float(np.mean(d * d))
    return 99.99 if mse == 0 else 10.0 * np.log10(255.0 ** 2 / mse)


def run_path(ctx, P, torch, specs, frames_dev, precision, steps, warmup):
    params = [P.Params.from_spec(s, precision=precision) for s in specs]
    streams = [ctx.alloc_stream(p) for p in params]

    def step():
        ctx.encode_batch(list(zip(frames_dev, params)), outs=streams)
        return ctx.decode_batch(list(zip(streams, params)), want_obj=True)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile_reset()
    ctx.profile(True)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = None
    for a, b in evs:
        a.record()
        outs = step()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.profile(False)
    per_step = [a.elapsed_time(b) for a, b in evs]
    return wall, per_step, outs, streams


def measured_traffic(streams):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on this kernel source and this workload size; else None."""
    import hashlib
    import re
    if streams != 16 or not os.path.exists(PMC_SUMMARY):
        return None
    txt = open(PMC_SUMMARY).read()
    sha = re.search(r"kernel_source_sha256: (\w+)", txt)
    tb = re.search(r"traffic_bytes_per_launch: (\d+)", txt)
    cur = kernel_source_digest()
    if not sha or not tb or sha.group(1) != cur:
        return None
    return int(tb.group(1))


def host_cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_recovery(spec, codes, exps):
    """The FP64 oracle's recovery of the given blocks (host), timed."""
    from oracle import cs, philox
    t0 = time.perf_counter()
    q = philox.measurement_matrix_q(spec.m, spec.n, spec.phi_seed, spec.stream_id)
    s_phi = philox.phi_scale(spec.m)
    a = cs.operator(q, s_phi, spec.block)
    L, _, _ = cs.lipschitz(q, s_phi)
    y = cs.dequantise(codes.T, exps, s_phi)
    lam = cs.lambdas(a, y)
    s = cs.fista(a, y, lam, L, spec.iters)
    cs.synthesise(s, spec.block)
    return time.perf_counter() - t0


def cpu_baseline(spec, gs_host, n_blocks, n_blocks_1t):
    """Oracle recovery of the first CS blocks of one GOP on the host: with
    the BLAS pool at its default size (n_blocks) and at one thread
    (n_blocks_1t)."""
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    codes, exps = gs_host
    codes = codes.reshape(-1, spec.m)
    exps = exps.reshape(-1)
    dt = _oracle_recovery(spec, codes[:n_blocks], exps[:n_blocks])
    with threadpool_limits(limits=1):
        dt1 = _oracle_recovery(spec, codes[:n_blocks_1t], exps[:n_blocks_1t])
    px, px1 = n_blocks * spec.n, n_blocks_1t * spec.n
    return {"value": px / dt / 1e6, "unit": "Mpixel/s", "cores": int(threads), "kind": "oracle",
            "cpu_model": host_cpu_model(), "os_cpu_count": os.cpu_count(),
            "single_thread": {"value": px1 / dt1 / 1e6, "unit": "Mpixel/s", "cores": 1,
                              "blocks": n_blocks_1t, "seconds": round(dt1, 2)},
            "sample": f"FP64 oracle recovery (operator, step constant, lambda, {spec.iters} FISTA "
                      f"iterations, synthesis) of the first {n_blocks} blocks of 32x32 at M=256 "
                      f"of one 640x480 GOP on {threads} BLAS threads ({dt:.1f} s), and of "
                      f"{n_blocks_1t} blocks on one thread ({dt1:.1f} s)"}


def mixed_main(args):
    """64 mixed streams (176x144 / 352x288 / 640x480; GOP 4-32; M/n
    0.05-0.4; B 16 or 32): one batch decode captured in a HIP graph and
    replayed; every block of every stream goes through the persistent
    fused launches (one per tile class)."""
    import torch
    import paper_1311_1419_amd as P
    import synthvid as sv
    specs = sv.mixed_streams(64)
    with P.Context(0) as ctx:
        params = [P.Params.from_spec(s, precision=P.CSV_BF16) for s in specs]
        bufs = [ctx.alloc_stream(p) for p in params]
        for s, p, b in zip(specs, params, bufs):
            ctx.encode_gop(torch.from_numpy(s.video()).cuda(), p, out=b)
        torch.cuda.synchronize()
        items = list(zip(bufs, params))
        for _ in range(args.warmup):
            ctx.decode_batch(items)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.decode_batch(items)
        torch.cuda.synchronize()
        eager = (time.perf_counter() - t0) / args.steps
        st = torch.cuda.Stream()
        g = ctx.capture_batch(items, st)
        for _ in range(args.warmup):
            g.launch(st)
        st.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        t0 = time.perf_counter()
        for a, b in evs:
            a.record(st)
            g.launch(st)
            b.record(st)
        st.synchronize()
        wall = time.perf_counter() - t0
        per = [a.elapsed_time(b) for a, b in evs]
        g.close()
    px = sum((s.gop - 1) * s.height * s.width for s in specs)
    blocks = sum((s.gop - 1) * ((s.height + s.block - 1) // s.block)
                 * ((s.width + s.block - 1) // s.block) for s in specs)
    flops = sum((s.gop - 1) * ((s.height + s.block - 1) // s.block)
                * ((s.width + s.block - 1) // s.block) * 4.0 * s.m * s.n * s.iters for s in specs)
    # what the MFMA units execute: M padded to whole 32-row tiles
    flops_exec = sum((s.gop - 1) * ((s.height + s.block - 1) // s.block)
                     * ((s.width + s.block - 1) // s.block) * 4.0 * (-(-s.m // 32) * 32) * s.n
                     * s.iters for s in specs)
    ms = 1e3 * wall / args.steps
    print(json.dumps({
        "metric": "recovered Mpixel/s, 64 mixed streams, one graph-captured batch decode",
        "value": round(px * args.steps / wall / 1e6, 3), "unit": "Mpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "p50_ms": round(float(np.percentile(per, 50)), 4),
        "p99_ms": round(float(np.percentile(per, 99)), 4),
        "eager_ms_per_step": round(1e3 * eager, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "mixed64-qcif/cif/vga-g4..32-m/n0.05..0.4-b16/32-t300",
                   "recovered_px_per_step": px, "blocks_per_step": blocks},
        "algorithmic_tflops": round(flops / (ms / 1e3) / 1e12, 2),
        "executed_tflops": round(flops_exec / (ms / 1e3) / 1e12, 2),
        "executed_over_algorithmic": round(flops_exec / flops, 4),
    }), flush=True)


def serve_sweep(loads, window, on_point=None, hip_streams=2):
    """256 synthetic cameras (640x480 and 1280x720, B=16, M/n 0.1 or 0.25,
    GOP 8/16/32) served by the continuous-batching server under open-loop
    Poisson GOP arrivals at each fraction `load` of the cameras' nominal
    2-20 GOP/s, for `window` seconds of arrivals per point.  A fresh server
    per point; six warm-up requests are decoded and polled, then the
    statistics are reset, so latencies, counts and rates cover only the
    window's requests.  The served rate is the window's recovered pixels
    over max(window, last completion - window start), so it never exceeds
    the offered rate."""
    import torch
    import paper_1311_1419_amd as P
    import synthvid as sv
    cams = sv.serving_cameras(256)
    pool = {}
    for spec, _ in cams:
        key = (spec.height, spec.width, spec.gop)
        if key not in pool:
            pool[key] = torch.from_numpy(spec.video()).cuda()
    sweep = []
    with P.Context(0) as ctx:
        # one batch encode: the 256 cameras' operators are set up together
        params = [P.Params.from_spec(spec, precision=P.CSV_BF16) for spec, _ in cams]
        streams = ctx.encode_batch([(pool[(spec.height, spec.width, spec.gop)], p)
                                    for (spec, _), p in zip(cams, params)])
        enc = [(p, gs, rate) for p, gs, (_, rate) in zip(params, streams, cams)]
        torch.cuda.synchronize()
        rng = np.random.default_rng(7)
        for load in loads:
            with P.Server(0, mem_budget=48 << 30, hip_streams=hip_streams) as srv:
                sids = srv.register_streams([p for p, _, _ in enc])
                warm = [srv.submit(sids[i], enc[i][1]) for i in range(6)]
                srv.drain(120.0)
                for t in warm:
                    srv.poll(t)
                srv.reset_stats()
                arr = []
                for i, (p, gs, rate) in enumerate(enc):
                    t = float(rng.exponential(1.0 / (rate * load)))
                    while t < window:
                        arr.append((t, i))
                        t += float(rng.exponential(1.0 / (rate * load)))
                arr.sort()
                t0 = P.clock()
                pending = collections.deque()

                def collect():
                    # a client takes decoded GOPs as they finish (in order),
                    # which releases their frames from the server budget
                    while pending and srv.poll(pending[0]):
                        pending.popleft()

                for ta, i in arr:
                    while P.clock() < t0 + ta:
                        collect()
                        time.sleep(0.0002)
                    pending.append(srv.submit(sids[i], enc[i][1], t0 + ta))
                while pending:
                    collect()
                    time.sleep(0.0005)
                srv.drain(60.0)
                st = srv.stats()
            offered_px = sum((enc[i][0].gop - 1) * enc[i][0].width * enc[i][0].height
                             for _, i in arr)
            span = max(window, st["last_done_s"] - t0) if st["completed"] else window
            sweep.append({"load": load, "window_s": window, "requests": len(arr),
                          "offered_mpix_s": round(offered_px / window / 1e6, 1),
                          "completed": st["completed"],
                          "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                          "max_ms": round(st["max_ms"], 3),
                          "served_mpix_s": round(st["recovered_pixels"] / span / 1e6, 1),
                          "batches": st["batches"],
                          "max_concurrent_batches": st["max_concurrent"],
                          "server_device_gib": round(st["device_bytes"] / 2**30, 2)})
            if on_point:
                on_point(sweep[-1])
    return sweep


def serve_main(args):
    """The serving load sweep (serve_sweep over --serve-loads): latency and
    throughput per offered load, the highest stable load."""
    loads = [float(x) for x in args.serve_loads.split(",")]
    sweep = serve_sweep(loads, args.serve_window,
                        lambda pt: print(json.dumps({"sweep_point": pt}), flush=True),
                        hip_streams=args.serve_streams)
    best = max(sweep, key=lambda r: r["served_mpix_s"])
    # stable: the server keeps up with the offered load (served within 5% of
    # offered); the highest such point is the load the server sustains
    stable = [r for r in sweep if r["served_mpix_s"] >= 0.95 * r["offered_mpix_s"]]
    top = max(stable, key=lambda r: r["load"]) if stable else None
    print(json.dumps({
        "metric": "served Mpixel/s and p99 latency, 256 cameras, Poisson GOP arrivals",
        "value": best["served_mpix_s"], "unit": "Mpixel/s", "n_gpus": 1,
        "p99_ms": best["p99_ms"], "p50_ms": best["p50_ms"],
        "highest_stable_load": top,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "serve256-vga/720p-b16-m/n0.1,0.25-g8..32-t300",
                   "window_s": args.serve_window},
        "sweep": sweep}), flush=True)


def encode_main(args):
    """The headline cameras' GOPs encoded as one batch in each measurement
    form (exact integer product on BF16 MFMA, INT8 split-residual MFMA, FP8
    E4M3 MFMA); reports CS pixels encoded per second and the measurement
    kernel's algorithmic rate (2 M n operations per block)."""
    import torch
    import paper_1311_1419_amd as P
    specs = make_streams(args.streams)
    frames_dev = [torch.from_numpy(s.video()).cuda() for s in specs]
    px = sum((s.gop - 1) * s.height * s.width for s in specs)
    blocks = sum((s.gop - 1) * ((s.height + 31) // 32) * ((s.width + 31) // 32) for s in specs)
    ops_step = sum((s.gop - 1) * ((s.height + 31) // 32) * ((s.width + 31) // 32) * 2.0 * s.m * s.n
                   for s in specs)
    forms = {"exact_bf16": 0, "int8": P.CSV_FLAG_MEASURE_INT8, "fp8": P.CSV_FLAG_MEASURE_FP8}
    peaks = {"exact_bf16": 2500.0, "int8": 5000.0, "fp8": 5000.0}   # dense TFLOP/s or TOP/s
    res = {}
    with P.Context(0) as ctx:
        for name, flag in forms.items():
            params = [P.Params.from_spec(s, precision=P.CSV_BF16, flags=flag) for s in specs]
            outs = [ctx.alloc_stream(p) for p in params]
            items = list(zip(frames_dev, params))
            for _ in range(args.warmup):
                ctx.encode_batch(items, outs=outs)
            torch.cuda.synchronize()
            ctx.profile_reset()
            ctx.profile(True)
            t0 = time.perf_counter()
            for _ in range(args.steps):
                ctx.encode_batch(items, outs=outs)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            ctx.profile(False)
            m_ms, m_n = ctx.profile_query("measure")
            kernel_ms = m_ms / max(m_n, 1)                 # per GOP launch
            per_gop_ops = ops_step / len(specs)
            res[name] = {"mpix_per_s": round(px * args.steps / wall / 1e6, 1),
                         "ms_per_step": round(1e3 * wall / args.steps, 4),
                         "measure_kernel_us_per_gop": round(1e3 * kernel_ms, 2),
                         "measure_tops": round(per_gop_ops / (kernel_ms * 1e-3) / 1e12, 2),
                         "measure_frac_of_peak": round(per_gop_ops / (kernel_ms * 1e-3) / 1e12
                                                       / peaks[name], 4)}
    print(json.dumps({
        "metric": "encoded CS Mpixel/s per measurement form, 16 cameras 640x480 GOP 16, M/n=0.25",
        "value": res["exact_bf16"]["mpix_per_s"], "unit": "Mpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int8/fp8/bf16", "data": "synthetic",
        "config": {"workload": WORKLOAD + "-encode", "blocks_per_step": blocks,
                   "note": "measure kernel timed per GOP launch while the batch's GOPs overlap "
                           "on three streams"},
        "forms": res}), flush=True)


def configure_main(args):
    """The configurator's sweep (Fig. 6, Table I): a synthetic 352x288 clip
    of 105 frames, B = 32, GOP sizes 3/5/7 and M = 256/102/51/25/16/12 (CS
    frame CR 1024/(M+1) = 4.0 ... 78.8; 39.4/60.2/78.8 are the paper's
    40/60/80), every candidate coded and decoded on the GPU; the choice
    under a PSNR floor."""
    import torch
    import paper_1311_1419_amd as P
    import synthvid as sv
    spec = sv.cif_sweep(4, 0.25).with_(block=32, iters=300)
    clip = torch.from_numpy(spec.video(105)).cuda()
    gops, ms = [3, 5, 7], [256, 102, 51, 25, 16, 12]
    with P.Context(0) as ctx:
        base = P.Params.from_spec(spec, precision=P.CSV_BF16)
        ctx.configure(clip[:7], base, [3], [25], args.psnr_floor)   # warm-up: operators
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ctx.configure(clip, base, gops, ms, args.psnr_floor)
        wall = time.perf_counter() - t0
    pts = res["points"]
    # Fig. 6(a) with the paper's key-frame CR of 23 (Section 4), for comparison
    for p in pts:
        p["cr_total_at_key_cr_23"] = p["gop"] / (1.0 / 23.0 + (p["gop"] - 1) / p["cr_cs"])
        for k in ("cr_total", "cr_key", "cr_cs", "psnr_all", "psnr_cs", "cr_total_at_key_cr_23"):
            p[k] = round(p[k], 3)
    px = 105 * spec.height * spec.width * len(pts)
    print(json.dumps({
        "metric": "configurator sweep: (G, M) candidates coded and decoded per second, "
                  "352x288 clip of 105 frames",
        "value": round(len(pts) / wall, 3), "unit": "candidates/s", "n_gpus": 1,
        "ms_per_sweep": round(1e3 * wall, 2), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "cif352x288-f105-b32-g3,5,7-m256..12-t300",
                   "psnr_floor_db": args.psnr_floor, "pixels_coded_per_sweep": px},
        "best": res["best"], "chosen": pts[res["best"]] if res["best"] >= 0 else None,
        "points": pts}), flush=True)


def tv_main(args):
    """Total-variation recovery (the paper's TVAL3-style solver) against the
    l1-DCT path on the same GOPs: 4 synthetic 352x288 cameras, GOP 16, B =
    16, M/n = 0.25 (M = 64), T = 300; one step = decode the 4 GOPs as one
    batch.  Reports recovered Mpixel/s of each path and the PSNR each
    reaches on the same codes."""
    import torch
    import paper_1311_1419_amd as P
    import synthvid as sv
    specs = [sv.cif_sweep(16, 0.25, stream=s) for s in range(4)]
    videos = [s.video() for s in specs]
    px = sum((s.gop - 1) * s.height * s.width for s in specs)
    res = {}
    with P.Context(0) as ctx:
        for name, prec, flags in [("tv_bf16", P.CSV_BF16, P.CSV_FLAG_TV),
                                  ("tv_fp32", P.CSV_FP32, P.CSV_FLAG_TV),
                                  ("l1_fp32", P.CSV_FP32, 0), ("l1_bf16", P.CSV_BF16, 0)]:
            params = [P.Params.from_spec(s, precision=prec, flags=flags) for s in specs]
            items = [(ctx.encode_gop(torch.from_numpy(v).cuda(), p), p)
                     for v, p in zip(videos, params)]
            for _ in range(args.warmup):
                outs = ctx.decode_batch(items)
            torch.cuda.synchronize()
            ctx.profile_reset()
            ctx.profile(True)
            t0 = time.perf_counter()
            for _ in range(args.steps):
                outs = ctx.decode_batch(items)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / args.steps
            ctx.profile(False)
            ps = [psnr(v[t], o[0][t].cpu().numpy()) for v, o in zip(videos, outs)
                  for t in range(1, v.shape[0])]
            res[name] = {"mpix_per_s": round(px / wall / 1e6, 2), "ms_per_step": round(1e3 * wall, 3),
                         "mean_psnr_db": round(float(np.mean(ps)), 3)}
            kname = {"tv_bf16": "tv_bf16", "l1_bf16": "fista_bf16"}.get(name)
            if kname:
                k_ms, k_n = ctx.profile_query(kname)
                res[name]["kernel_ms"] = round(k_ms / max(k_n, 1), 4)
    # fused TV: the two Phi products are 4 M n flops per block per iteration
    # on BF16 MFMA; the stencil, shrinkage and step around them are VALU work
    blocks = sum((s.gop - 1) * (s.height // 16) * (s.width // 16) for s in specs)
    flops = blocks * 4.0 * 64 * 256 * 300
    ach = flops / (res["tv_bf16"]["kernel_ms"] * 1e-3) / 1e12
    # unfused FP32 TV moves about 72 bytes per pixel per iteration through HBM
    # (dual step: x, nu, w in, nu, w, P out; primal step: x, G, P in, x out;
    # the two products' x/R/G traffic): 8 TB/s / (72 B x T) pixels/s
    ceiling = 8.0e12 / (72.0 * 300) / 1e6
    print(json.dumps({
        "metric": "recovered Mpixel/s, TV recovery vs l1-DCT on the same codes, 4 cameras 352x288 "
                  "GOP 16, M/n=0.25, T=300",
        "value": res["tv_bf16"]["mpix_per_s"], "unit": "Mpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "cif352x288-g16-b16-m64-t300-x4streams-tv"},
        "roofline": {"bound": "mfma", "kernel": "tv_bf16_kernel<64>", "unit": "TFLOP/s",
                     "achieved": round(ach, 2), "peak": PEAK_BF16_TFLOPS,
                     "frac": round(ach / PEAK_BF16_TFLOPS, 4),
                     "note": "the Phi products' algorithmic flops; the stencil VALU work bounds "
                             "the kernel at this M"},
        "tv_fp32_roofline": {"bound": "hbm", "unit": "Mpixel/s", "peak": round(ceiling, 1),
                             "achieved": res["tv_fp32"]["mpix_per_s"],
                             "frac": round(res["tv_fp32"]["mpix_per_s"] / ceiling, 4)},
        "paths": res}), flush=True)


def whole_main(args):
    """Whole-frame measurement (eq. (1) literal): 8 synthetic 176x144
    cameras, GOP 5 (the paper's key frame + four CS frames), each CS frame
    measured as one 25 344-pixel vector by Q regenerated in the kernel; at
    the paper's CS compression ratio of 50 (M = 506) and at M/n = 0.25
    (M = 6336).  One step = the 8 GOPs encoded as one batch.  Then the
    same GOPs at M = 506 decoded by whole-frame TV recovery (reported
    beside the measurement rate, not as the headline value).  The kernel is
    integer-ALU bound: 332 VALU instructions per Philox block of four Q
    entries plus 7 per CS frame (counted in its gfx950 code), against
    256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s."""
    import torch
    import paper_1311_1419_amd as P
    import synthvid as sv
    specs = [sv.qcif_tiny(stream=s).with_(gop=5) for s in range(8)]
    frames = [torch.from_numpy(s.video()).cuda() for s in specs]
    n = 176 * 144
    peak = 256 * 4 * 16 * 2.4e9
    res = {}
    with P.Context(0) as ctx:
        for label, m in [("cr50_m506", 506), ("rho0.25_m6336", 6336)]:
            params = [P.Params.from_spec(s, m=m, precision=P.CSV_FP32,
                                         flags=P.CSV_FLAG_WHOLE_FRAME) for s in specs]
            outs = [ctx.alloc_stream(p) for p in params]
            items = list(zip(frames, params))
            for _ in range(args.warmup):
                ctx.encode_batch(items, outs=outs)
            torch.cuda.synchronize()
            ctx.profile_reset()
            ctx.profile(True)
            t0 = time.perf_counter()
            for _ in range(args.steps):
                ctx.encode_batch(items, outs=outs)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / args.steps
            ctx.profile(False)
            k_ms, k_n = ctx.profile_query("measure")
            k_s = k_ms / max(k_n, 1) / 1e3                      # per GOP launch
            entries = m * n                                     # Q entries per GOP
            ops = entries / 4 * (332 + 7 * 4)                   # VALU lane-ops per GOP
            px = len(specs) * 4 * n
            cr_cs = 8.0 * n / (8 * m + 8)
            res[label] = {"m": m, "cs_cr": round(cr_cs, 2),
                          "cs_mpix_per_s": round(px / wall / 1e6, 2),
                          "ms_per_step": round(1e3 * wall, 3),
                          "measure_ms_per_gop": round(1e3 * k_s, 4),
                          "q_entries_per_s": round(entries / k_s, 1),
                          "valu_tops": round(ops / k_s / 1e12, 2),
                          "valu_frac": round(ops / k_s / peak, 4)}
        # decode: each CS frame recovered as one 176x144 image by the TV
        # solver (FP32, T = 300) at CR 50, the 8 GOPs as one batch
        params = [P.Params.from_spec(s, m=506, precision=P.CSV_FP32, iters=300,
                                     flags=P.CSV_FLAG_WHOLE_FRAME | P.CSV_FLAG_TV) for s in specs]
        items = [(ctx.encode_gop(f, p), p) for f, p in zip(frames, params)]
        for _ in range(max(args.warmup, 1)):
            outs = ctx.decode_batch(items)
        torch.cuda.synchronize()
        ctx.profile_reset()
        ctx.profile(True)
        dsteps = max(1, min(args.steps, 5))
        t0 = time.perf_counter()
        for _ in range(dsteps):
            outs = ctx.decode_batch(items)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / dsteps
        ctx.profile(False)
        k_ms, k_n = ctx.profile_query("tv_whole")
        it_s = k_ms / max(k_n, 1) / 1e3 / 300               # one iteration, all 8 GOPs
        ps = [psnr(s.video()[t], o[0][t].cpu().numpy()) for s, o in zip(specs, outs)
              for t in range(1, 5)]
        # algorithmic HBM bytes per iteration and GOP: Q read by both
        # products (2 M n int8) and 16 FP32 words of state per pixel and CS
        # frame (dual step: x, nu, w in, nu, w, P out = 11; forward: x = 1;
        # primal step: x, P in, x out = 4)
        byt = len(specs) * (2.0 * 506 * n + 4 * n * 4 * 16)
        res["decode_tv_cr50_m506"] = {
            "cs_mpix_per_s": round(len(specs) * 4 * n / wall / 1e6, 3),
            "ms_per_step": round(1e3 * wall, 3), "iters": 300,
            "us_per_iteration_8gops": round(1e6 * it_s, 2),
            "algorithmic_tbs": round(byt / it_s / 1e12, 3),
            "hbm_frac": round(byt / it_s / 8e12, 4),
            "mean_psnr_db": round(float(np.mean(ps)), 3)}
    print(json.dumps({
        "metric": "whole-frame CS Mpixel/s encoded (Q regenerated on the fly), 8 cameras 176x144 "
                  "GOP 5",
        "value": res["cr50_m506"]["cs_mpix_per_s"], "unit": "Mpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32/int64", "data": "synthetic",
        "config": {"workload": "qcif176x144-g5-whole-frame-x8streams",
                   "note": "measure kernel timed per GOP while the batch's GOPs overlap"},
        "roofline": {"bound": "alu", "unit": "T lane-ops/s", "peak": round(peak / 1e12, 1),
                     "achieved": res["rho0.25_m6336"]["valu_tops"],
                     "frac": res["rho0.25_m6336"]["valu_frac"]},
        "rates": res}), flush=True)


def fp32_main(args):
    """The plain FP32 path alone on the headline workload (16 x 640x480
    GOP-16, B = 32, M = 256, T = 300): encode and decode as one batch per
    step, the two FP32-MFMA products of every iteration with the residual
    and the threshold/momentum step in their epilogues.  Per launch the
    forward product reads v (4 n B per block) and the operator and writes
    the residual (4 M_p B); the adjoint reads the residual and the operator
    and, in its epilogue, reads v and s_{k-1} and writes both (16 n B)."""
    import torch
    import paper_1311_1419_amd as P
    specs = make_streams(args.streams)
    frames_dev = [torch.from_numpy(s.video()).cuda() for s in specs]
    px = sum((s.gop - 1) * s.height * s.width for s in specs)
    blocks = sum((s.gop - 1) * ((s.height + 31) // 32) * ((s.width + 31) // 32) for s in specs)
    with P.Context(0) as ctx:
        wall, per_step, _, _ = run_path(ctx, P, torch, specs, frames_dev, P.CSV_FP32,
                                        args.steps, args.warmup)
        k_ms, k_n = ctx.profile_query("fista_fp32")
    it_s = k_ms / max(k_n, 1) / 1e3 / 300            # one iteration of the whole batch
    flops = blocks * 4.0 * 256 * 1024                 # both products, one iteration
    byts = blocks * (4 * 1024 + 4 * 256 + 4 * 256 + 16 * 1024 + 4 * 256)
    print(json.dumps({
        "metric": "recovered Mpixel/s, plain FP32 path, " + WORKLOAD,
        "value": round(px * args.steps / wall / 1e6, 3), "unit": "Mpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 4),
        "p50_ms": round(float(np.percentile(per_step, 50)), 4),
        "p99_ms": round(float(np.percentile(per_step, 99)), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32",
        "data": "synthetic", "config": {"workload": WORKLOAD + "-fp32", "blocks_per_step": blocks},
        "iteration_us": round(1e6 * it_s, 2),
        "fp32_mfma_tflops": round(flops / it_s / 1e12, 2),
        "algorithmic_hbm_tbs": round(byts / it_s / 1e12, 3)}), flush=True)


def b16_main(args):
    """The fused path on the 16 x 16-block class: 16 synthetic 352x288
    cameras, GOP 16, B = 16 (n = 256), M/n = 0.25 (M = 64), T = 300,
    encoded and decoded as one batch per step (23 760 x 4 recovery blocks
    in one launch of the (256, 64) class)."""
    import torch
    import paper_1311_1419_amd as P
    import synthvid as sv
    specs = [sv.cif_sweep(16, 0.25, stream=s) for s in range(args.streams)]
    frames_dev = [torch.from_numpy(s.video()).cuda() for s in specs]
    px = sum((s.gop - 1) * s.height * s.width for s in specs)
    blocks = sum((s.gop - 1) * (s.height // 16) * (s.width // 16) for s in specs)
    flops = sum((s.gop - 1) * (s.height // 16) * (s.width // 16) * 4.0 * s.m * s.n * s.iters
                for s in specs)
    with P.Context(0) as ctx:
        wall, per_step, _, _ = run_path(ctx, P, torch, specs, frames_dev, P.CSV_BF16,
                                        args.steps, args.warmup)
        k_ms, k_n = ctx.profile_query("fista_bf16")
    k_s = k_ms / max(k_n, 1) / 1e3
    ach = flops / k_s / 1e12
    print(json.dumps({
        "metric": "recovered Mpixel/s, fused BF16 path, 16 x 352x288 GOP-16 B=16 M=64 T=300",
        "value": round(px * args.steps / wall / 1e6, 3), "unit": "Mpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 4),
        "p50_ms": round(float(np.percentile(per_step, 50)), 4),
        "p99_ms": round(float(np.percentile(per_step, 99)), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "cif352x288-g16-b16-m64-t300-x%dstreams" % args.streams,
                   "blocks_per_step": blocks},
        "roofline": {"bound": "mfma", "kernel": "fista_bf16_kernel[n=256,Mp=64] variant "
                     + P.kernel_choice(16, 64)[0], "unit": "TFLOP/s",
                     "achieved": round(ach, 2), "peak": PEAK_BF16_TFLOPS,
                     "frac": round(ach / PEAK_BF16_TFLOPS, 4), "kernel_ms": round(1e3 * k_s, 4)}}),
        flush=True)


def setup_main(args):
    """Wall time of a new stream's setup (measurement matrix, operator, its
    fragment layouts, the exact Gram matrix and the FP64 power iteration for
    the step constant) per (M, n), each shape once in one context after a
    small warm-up stream; block operators at B = 32 and whole-frame ones."""
    import paper_1311_1419_amd as P
    cases = [("block", 32, m) for m in (256, 320, 352, 410, 512, 768, 1024)] + \
            [("whole", (48, 64), m) for m in (1500, 3000)]
    res = {}
    with P.Context(0) as ctx:
        ctx.step_constant(P.Params(width=64, height=64, gop=2, block=16, m=13, phi_seed=1,
                                   stream_id=1))
        for k, (kind, b, m) in enumerate(cases):
            if kind == "block":
                p = P.Params(width=64, height=64, gop=2, block=b, m=m, phi_seed=7000 + k,
                             stream_id=2)
                key, n = f"block_m{m}_n{b * b}", b * b
            else:
                h, w = b
                p = P.Params(width=w, height=h, gop=2, block=16, m=m, phi_seed=7000 + k,
                             stream_id=2, precision=P.CSV_FP32,
                             flags=P.CSV_FLAG_WHOLE_FRAME | P.CSV_FLAG_TV)
                key, n = f"whole_m{m}_n{h * w}", h * w
            t0 = time.perf_counter()
            _, it = ctx.step_constant(p)
            ms = 1e3 * (time.perf_counter() - t0)
            res[key] = {"ms": round(ms, 2), "power_iterations": int(it),
                        "us_per_iteration_upper": round(1e3 * ms / max(1, int(it)), 2)}
            print(json.dumps({"setup_point": {key: res[key]}}), flush=True)
    print(json.dumps({"metric": "new-stream setup ms (operator and step constant)",
                      "unit": "ms", "higher_is_better": False, "n_gpus": 1,
                      "data": "synthetic", "config": {"workload": "stream setup"},
                      "points": res}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by stream or GOP with no exchange between GPUs)",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_mib:
        import torch
        src = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.mode == "mixed":
        return mixed_main(args)
    if args.mode == "serve":
        return serve_main(args)
    if args.mode == "encode":
        return encode_main(args)
    if args.mode == "configure":
        return configure_main(args)
    if args.mode == "tv":
        return tv_main(args)
    if args.mode == "whole":
        return whole_main(args)
    if args.mode == "fp32":
        return fp32_main(args)
    if args.mode == "b16":
        return b16_main(args)
    if args.mode == "setup":
        return setup_main(args)
    import torch
    import paper_1311_1419_amd as P

    specs = make_streams(args.streams)
    videos = [s.video() for s in specs]
    frames_dev = [torch.from_numpy(v).cuda() for v in videos]
    px_per_step = sum((s.gop - 1) * s.height * s.width for s in specs)
    blocks = sum((s.gop - 1) * ((s.height + 31) // 32) * ((s.width + 31) // 32) for s in specs)
    flops_launch = sum((s.gop - 1) * ((s.height + 31) // 32) * ((s.width + 31) // 32)
                       * 4.0 * s.m * s.n * s.iters for s in specs)

    if args.variant:
        count = P.kernel_choice(32, 256)[2]
        names = []
        for i in range(count):
            P.set_kernel_choice(32, 256, i)
            names.append(P.kernel_choice(32, 256)[0])
        if args.variant not in names:
            sys.exit(f"no variant {args.variant!r} in the (1024, 256) class: {names}")
        P.set_kernel_choice(32, 256, names.index(args.variant))
    with P.Context(0) as ctx:
        wall, per_step, outs, streams = run_path(ctx, P, torch, specs, frames_dev, P.CSV_BF16,
                                                 args.steps, args.warmup)
        k_ms, k_n = ctx.profile_query("fista_bf16")
        torch.cuda.synchronize()
        bf16_frames = [o[0].cpu().numpy() for o in outs]
        codes_host = (streams[0].codes.cpu().numpy(), streams[0].exps.cpu().numpy())
        fp32 = None
        if not args.no_fp32:
            w32, ps32, outs32, _ = run_path(ctx, P, torch, specs, frames_dev, P.CSV_FP32,
                                            args.fp32_steps, 1)
            f32_frames = [o[0].cpu().numpy() for o in outs32]
            fp32 = {"value": px_per_step * args.fp32_steps / w32 / 1e6,
                    "ms_per_step": 1e3 * w32 / args.fp32_steps}
            loss = []
            for v, fb, ff in zip(videos, bf16_frames, f32_frames):
                for t in range(1, v.shape[0]):
                    loss.append(psnr(v[t], ff[t]) - psnr(v[t], fb[t]))
            fp32["psnr_loss_db_mean"] = float(np.mean(loss))
            fp32["psnr_loss_db_max"] = float(np.max(loss))
        mean_psnr = float(np.mean([psnr(v[t], fb[t]) for v, fb in zip(videos, bf16_frames)
                                   for t in range(1, v.shape[0])]))
        ceilings = None if args.no_ceilings else ctx.probe_ceilings()
    variant = P.kernel_choice(32, 256)[0]
    # L2 -> CU bytes of the fused launch: every tile of 32 blocks reads both
    # fragment layouts of its operator (2 x Mp x n bf16) once per iteration,
    # less the last `nl` forward K steps of each of the Mp / 32 forward tiles
    # (1 KiB fragments) that a variant named "..._lds<nl>" or "..._ldsi<nl>"
    # (optionally followed by "_pp") keeps in LDS
    nl_m = re.search(r"_ldsi?(\d+)(_pp)?$", variant)
    nl = int(nl_m.group(1)) if nl_m else 0
    tiles = sum(-(-((s.gop - 1) * ((s.height + 31) // 32) * ((s.width + 31) // 32)) // 32)
                for s in specs)
    l2_bytes = sum(-(-((s.gop - 1) * ((s.height + 31) // 32) * ((s.width + 31) // 32)) // 32)
                   * s.iters * (2 * (-(-s.m // 32) * 32) * s.n * 2
                                - (-(-s.m // 32)) * nl * 1024) for s in specs)

    value = px_per_step * args.steps / wall / 1e6
    avg_k_s = (k_ms / max(k_n, 1)) / 1e3
    achieved = flops_launch / avg_k_s / 1e12 if k_n else None
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 4),
        "p50_ms": round(float(np.percentile(per_step, 50)), 4),
        "p99_ms": round(float(np.percentile(per_step, 99)), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "frame": "640x480", "gop": 16, "block": 32, "m": 256,
                   "iters": 300, "streams_per_step": args.streams,
                   "recovered_px_per_step": px_per_step, "blocks_per_step": blocks},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2) if achieved else None,
                     "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_BF16_TFLOPS, 4) if achieved else None,
                     "traffic": None if args.variant else measured_traffic(args.streams),
                     "traffic_unit": "bytes/launch",
                     "kernel": f"fista_bf16_kernel[n=1024,Mp=256] variant {variant}",
                     "kernel_ms": round(1e3 * avg_k_s, 4), "flops_per_launch": flops_launch,
                     "tiles_per_launch": tiles, "l2_bytes_per_launch": l2_bytes,
                     "l2_tbs": round(l2_bytes / avg_k_s / 1e12, 2) if k_n else None},
        "fp32_path": fp32,
        "mean_psnr_db_bf16": round(mean_psnr, 3),
    }
    if ceilings and k_n:
        # the same kernel against what microbenchmarks reach on this device
        line["roofline"]["achievable"] = {
            "mfma_bf16_tflops": round(ceilings["mfma_bf16_tflops"], 1),
            "l2_read_tbs": round(ceilings["l2_read_tbs"], 2),
            "hbm_read_tbs": round(ceilings["hbm_read_tbs"], 2),
            "lds_read_tbs": round(ceilings["lds_read_tbs"], 2),
            "frac_mfma": round(achieved / ceilings["mfma_bf16_tflops"], 4),
            "frac_l2": round(l2_bytes / avg_k_s / 1e12 / ceilings["l2_read_tbs"], 4)}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(specs[0], codes_host, args.cpu_blocks,
                                            args.cpu_blocks_1t)
    if args.headline_serve_load > 0:
        # p50/p99 of the serving form in the same line: one short load point
        line["serving"] = serve_sweep([args.headline_serve_load],
                                      args.headline_serve_window)[0]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
