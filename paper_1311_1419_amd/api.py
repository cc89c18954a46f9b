"""Python face of the HIP coder: torch tensors for device memory and streams,
ctypes calls into libcsv.so for every step of the coder."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field, replace

import torch

from . import _native as N


@dataclass(frozen=True)
class Params:
    """One stream's coding parameters (mirrors csv_params)."""
    width: int
    height: int
    gop: int
    block: int = 16
    m: int = 0
    rho: float = 0.25
    phi_seed: int = 0
    stream_id: int = 0
    key_qstep: int = 16
    iters: int = 300
    lambda_frac: float = 0.01
    precision: int = N.CSV_BF16
    flags: int = 0

    def to_c(self) -> N.CsvParams:
        return N.CsvParams(self.width, self.height, self.gop, self.block, self.m,
                           self.rho, self.phi_seed & (2**64 - 1),
                           self.stream_id & 0xFFFFFFFF, self.key_qstep, self.iters,
                           self.lambda_frac, self.precision, self.flags)

    @property
    def n(self) -> int:
        """Pixels per measured vector: a B x B block, or the whole frame."""
        if self.flags & N.CSV_FLAG_WHOLE_FRAME:
            return self.width * self.height
        return self.block * self.block

    def resolve(self) -> tuple[int, int]:
        """(M, blocks per frame) as the library resolves them."""
        m = C.c_int32()
        nb = C.c_int32()
        N.check(N.lib().csv_resolve(C.byref(self.to_c()), C.byref(m), C.byref(nb)))
        return m.value, nb.value

    @staticmethod
    def from_spec(spec, **kw) -> "Params":
        base = dict(width=spec.width, height=spec.height, gop=spec.gop, block=spec.block,
                    m=spec.m, phi_seed=spec.phi_seed, stream_id=spec.stream_id,
                    key_qstep=spec.key_qstep, iters=spec.iters,
                    lambda_frac=spec.lambda_frac)
        base.update(kw)
        return Params(**base)

    def with_(self, **kw) -> "Params":
        return replace(self, **kw)


@dataclass
class GopStream:
    """Encoded GOP in device memory (mirrors csv_gop_stream)."""
    key_levels: torch.Tensor    # int16 H x W
    codes: torch.Tensor         # int8 (G-1) x N_b x M
    exps: torch.Tensor          # uint8 (G-1) x N_b
    bits: torch.Tensor = field(default=None)   # int64 [key bits, CS bits]

    def to_c(self) -> N.CsvGopStream:
        return N.CsvGopStream(self.key_levels.data_ptr(),
                              self.codes.data_ptr() if self.codes.numel() else None,
                              self.exps.data_ptr() if self.exps.numel() else None,
                              self.bits.data_ptr() if self.bits is not None else None)


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _require_cuda(t: torch.Tensor, dtype, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def kernel_choice(block: int, m: int) -> tuple[str, int, int]:
    """(variant name, index, number of variants) of the fused kernel class."""
    buf = C.create_string_buffer(128)
    idx, cnt = C.c_int32(), C.c_int32()
    N.check(N.lib().csv_autotune_choice(block, m, buf, 128, C.byref(idx), C.byref(cnt)))
    return buf.value.decode(), idx.value, cnt.value


def set_kernel_choice(block: int, m: int, index: int) -> None:
    N.check(N.lib().csv_autotune_set(block, m, index))


def load_kernel_choices(json_path: str) -> None:
    N.check(N.lib().csv_autotune_load(json_path.encode()))


class DecodeGraph:
    """A captured batch decode (csv_graph); keeps its bound buffers alive."""

    def __init__(self, handle, outputs, inputs):
        self._h = handle
        self.outputs = outputs
        self._inputs = inputs

    def launch(self, stream) -> None:
        N.check(N.lib().csv_graph_launch(self._h, stream.cuda_stream))

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            N.check(N.lib().csv_graph_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """A csv_ctx: per-stream operator caches and scratch on one device."""

    def __init__(self, device: int = 0, mem_budget: int = 0):
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        N.check(N.lib().csv_create(C.byref(h), device, mem_budget))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            N.check(N.lib().csv_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        return self._h

    def bytes_held(self) -> int:
        v = C.c_size_t()
        N.check(N.lib().csv_ctx_bytes(self._h, C.byref(v)))
        return v.value

    # ------------------------------------------------------------- sizes
    @staticmethod
    def encoded_size(p: Params):
        k, c, e, b = C.c_size_t(), C.c_size_t(), C.c_size_t(), C.c_uint64()
        N.check(N.lib().csv_encoded_size(C.byref(p.to_c()), C.byref(k), C.byref(c),
                                         C.byref(e), C.byref(b)))
        return k.value, c.value, e.value, b.value

    @staticmethod
    def compression_ratio(p: Params, bits_key: int, bits_cs: int):
        t, k, c = C.c_double(), C.c_double(), C.c_double()
        N.check(N.lib().csv_compression_ratio(C.byref(p.to_c()), bits_key, bits_cs,
                                              C.byref(t), C.byref(k), C.byref(c)))
        return {"total": t.value, "key": k.value, "cs": c.value}

    def alloc_stream(self, p: Params) -> GopStream:
        m, nb = p.resolve()
        g = p.gop
        dev = self.device
        # CSV_FLAG_NO_QUANT (test hook): exact int32 measurements instead of codes
        cdt = torch.int32 if p.flags & N.CSV_FLAG_NO_QUANT else torch.int8
        return GopStream(
            torch.empty((p.height, p.width), dtype=torch.int16, device=dev),
            torch.empty((g - 1, nb, m), dtype=cdt, device=dev),
            torch.empty((g - 1, nb), dtype=torch.uint8, device=dev),
            torch.zeros(2, dtype=torch.int64, device=dev))

    # ---------------------------------------------------------- hot path
    def encode_gop(self, frames: torch.Tensor, p: Params, out: GopStream | None = None) -> GopStream:
        _require_cuda(frames, torch.uint8, "frames")
        if tuple(frames.shape) != (p.gop, p.height, p.width):
            raise ValueError("frames must be G x H x W")
        out = out or self.alloc_stream(p)
        N.check(N.lib().csv_encode_gop(self._h, C.byref(p.to_c()), frames.data_ptr(),
                                       C.byref(out.to_c()), _stream(self.device)))
        return out

    def encode_batch(self, items, outs=None):
        """items: list of (frames G x H x W uint8 tensor, Params).  Encodes
        every GOP (same results as encode_gop per item) with overlapping
        kernels; returns the GopStreams (`outs`, if given, are filled)."""
        count = len(items)
        params = (N.CsvParams * max(count, 1))()
        fptr = (C.c_void_p * max(count, 1))()
        streams = (N.CsvGopStream * max(count, 1))()
        res = []
        for i, (frames, p) in enumerate(items):
            _require_cuda(frames, torch.uint8, "frames")
            if tuple(frames.shape) != (p.gop, p.height, p.width):
                raise ValueError("frames must be G x H x W")
            gs = outs[i] if outs is not None else self.alloc_stream(p)
            params[i] = p.to_c()
            fptr[i] = frames.data_ptr()
            streams[i] = gs.to_c()
            res.append(gs)
        N.check(N.lib().csv_encode_batch(self._h, count, params, fptr, streams,
                                         _stream(self.device)))
        return res

    def decode_gop(self, gs: GopStream, p: Params, want_float: bool = False,
                   want_obj: bool = False):
        m, nb = p.resolve()
        dev = self.device
        frames = torch.empty((p.gop, p.height, p.width), dtype=torch.uint8, device=dev)
        fl = (torch.empty((p.gop - 1, p.height, p.width), dtype=torch.float32, device=dev)
              if want_float else None)
        obj = (torch.empty((p.gop - 1, nb, 2), dtype=torch.float64, device=dev)
               if want_obj else None)
        N.check(N.lib().csv_decode_gop(self._h, C.byref(p.to_c()), C.byref(gs.to_c()),
                                       frames.data_ptr(), _ptr(fl), _ptr(obj),
                                       _stream(dev)))
        return frames, fl, obj

    def decode_batch(self, items, want_float: bool = False, want_obj: bool = False):
        """items: list of (GopStream, Params).  Returns a list of
        (frames, cs_float or None, obj or None)."""
        count = len(items)
        dev = self.device
        params = (N.CsvParams * max(count, 1))()
        streams = (N.CsvGopStream * max(count, 1))()
        fptr = (C.c_void_p * max(count, 1))()
        flptr = (C.c_void_p * max(count, 1))()
        optr = (C.c_void_p * max(count, 1))()
        outs = []
        for i, (gs, p) in enumerate(items):
            m, nb = p.resolve()
            frames = torch.empty((p.gop, p.height, p.width), dtype=torch.uint8, device=dev)
            fl = (torch.empty((p.gop - 1, p.height, p.width), dtype=torch.float32, device=dev)
                  if want_float else None)
            obj = (torch.empty((p.gop - 1, nb, 2), dtype=torch.float64, device=dev)
                   if want_obj else None)
            params[i] = p.to_c()
            streams[i] = gs.to_c()
            fptr[i] = frames.data_ptr()
            flptr[i] = _ptr(fl)
            optr[i] = _ptr(obj)
            outs.append((frames, fl, obj))
        N.check(N.lib().csv_decode_batch(self._h, count, params, streams, fptr,
                                         flptr if want_float else None,
                                         optr if want_obj else None, _stream(dev)))
        return outs

    def capture_batch(self, items, stream, want_float: bool = False, want_obj: bool = False):
        """Capture the decode of `items` (list of (GopStream, Params)) into a
        HIP graph on `stream` (a torch.cuda.Stream).  Returns a DecodeGraph
        whose launch() re-decodes whatever the bound GopStreams hold into
        the bound output tensors (graph.outputs)."""
        count = len(items)
        dev = self.device
        params = (N.CsvParams * count)()
        streams = (N.CsvGopStream * count)()
        fptr = (C.c_void_p * count)()
        flptr = (C.c_void_p * count)()
        optr = (C.c_void_p * count)()
        outs = []
        for i, (gs, p) in enumerate(items):
            m, nb = p.resolve()
            frames = torch.empty((p.gop, p.height, p.width), dtype=torch.uint8, device=dev)
            fl = (torch.empty((p.gop - 1, p.height, p.width), dtype=torch.float32, device=dev)
                  if want_float else None)
            obj = (torch.empty((p.gop - 1, nb, 2), dtype=torch.float64, device=dev)
                   if want_obj else None)
            params[i] = p.to_c()
            streams[i] = gs.to_c()
            fptr[i] = frames.data_ptr()
            flptr[i] = _ptr(fl)
            optr[i] = _ptr(obj)
            outs.append((frames, fl, obj))
        h = C.c_void_p()
        torch.cuda.synchronize(dev)
        N.check(N.lib().csv_graph_capture(self._h, count, params, streams, fptr,
                                          flptr if want_float else None,
                                          optr if want_obj else None, stream.cuda_stream,
                                          C.byref(h)))
        return DecodeGraph(h, outs, [gs for gs, _ in items])

    # ------------------------------------------------------------ autotuning
    def autotune(self, block: int, m: int, iters: int = 300, n_blocks: int = 8192,
                 json_path: str | None = None) -> dict:
        """Time every fused-kernel variant of the (block, m) class, make the
        fastest the choice; returns {"times_ms": [...], "best": i, "choice": name}."""
        ms = (C.c_double * 8)()
        cnt, best = C.c_int32(), C.c_int32()
        N.check(N.lib().csv_autotune(self._h, block, m, iters, n_blocks,
                                     json_path.encode() if json_path else None, ms,
                                     C.byref(cnt), C.byref(best)))
        return {"times_ms": list(ms[:cnt.value]), "best": best.value,
                "choice": kernel_choice(block, m)[0]}

    # ---------------------------------------------------------- profiling
    def profile(self, on: bool = True) -> None:
        N.check(N.lib().csv_profile_enable(self._h, 1 if on else 0))

    def profile_reset(self) -> None:
        N.check(N.lib().csv_profile_reset(self._h))

    def profile_query(self, name: str) -> tuple[float, int]:
        """(total milliseconds, number of ranges) of a named kernel range."""
        ms = C.c_double()
        cnt = C.c_int64()
        N.check(N.lib().csv_profile_query(self._h, name.encode(), C.byref(ms), C.byref(cnt)))
        return ms.value, cnt.value

    def configure(self, clip: torch.Tensor, base: Params, gops, ms, psnr_floor: float) -> dict:
        """Sweep (G, M) candidates over a calibration clip (F x H x W uint8
        device tensor) with the coder itself and choose the largest total CR
        whose mean PSNR meets the floor.  Returns {"points": [dict per
        candidate, G-major], "best": index or -1}."""
        _require_cuda(clip, torch.uint8, "clip")
        if clip.dim() != 3 or tuple(clip.shape[1:]) != (base.height, base.width):
            raise ValueError("clip must be F x H x W")
        ng, nm = len(gops), len(ms)
        g_arr = (C.c_int32 * ng)(*gops)
        m_arr = (C.c_int32 * nm)(*ms)
        pts = (N.CsvConfigPoint * (ng * nm))()
        best = C.c_int32()
        N.check(N.lib().csv_configure(self._h, C.byref(base.to_c()), clip.data_ptr(),
                                      clip.shape[0], g_arr, ng, m_arr, nm, psnr_floor, pts,
                                      C.byref(best), _stream(self.device)))
        return {"points": [{f: getattr(p, f) for f, _ in N.CsvConfigPoint._fields_} for p in pts],
                "best": best.value}

    def frame_sse(self, a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
        """Exact per-frame sums of squared differences of two F x H x W uint8
        device stacks (uint64 as int64)."""
        _require_cuda(a, torch.uint8, "a")
        _require_cuda(b, torch.uint8, "b")
        if a.shape != b.shape or a.dim() != 3:
            raise ValueError("a and b must both be F x H x W")
        out = torch.empty((a.shape[0],), dtype=torch.int64, device=self.device)
        N.check(N.lib().csv_frame_sse(self._h, a.data_ptr(), b.data_ptr(), a.shape[0],
                                      a.shape[2], a.shape[1], out.data_ptr(),
                                      _stream(self.device)))
        return out

    def probe_ceilings(self) -> dict:
        """Achievable MFMA BF16 TFLOP/s and L2 / HBM / LDS read TB/s of the
        device, from short microbenchmarks (synchronous)."""
        r = N.CsvCeilings()
        N.check(N.lib().csv_probe_ceilings(self._h, C.byref(r)))
        return {f: getattr(r, f) for f, _ in N.CsvCeilings._fields_}

    # ------------------------------------------------------ single steps
    def phi_matrix(self, p: Params) -> torch.Tensor:
        m, _ = p.resolve()
        q = torch.empty((m, p.n), dtype=torch.int8, device=self.device)
        N.check(N.lib().csv_phi_matrix(self._h, C.byref(p.to_c()), q.data_ptr(),
                                       _stream(self.device)))
        return q

    def operator_matrix(self, p: Params) -> torch.Tensor:
        m, _ = p.resolve()
        a = torch.empty((m, p.n), dtype=torch.float64, device=self.device)
        N.check(N.lib().csv_operator_matrix(self._h, C.byref(p.to_c()), a.data_ptr(),
                                            _stream(self.device)))
        return a

    def step_constant(self, p: Params) -> tuple[float, int]:
        torch.cuda.current_stream(self.device).synchronize()
        L = C.c_double()
        it = C.c_int32()
        N.check(N.lib().csv_step_constant(self._h, C.byref(p.to_c()), C.byref(L), C.byref(it)))
        return L.value, it.value

    def key_encode(self, frame: torch.Tensor, qstep: int = 16):
        _require_cuda(frame, torch.uint8, "frame")
        h, w = frame.shape
        lev = torch.empty((h, w), dtype=torch.int16, device=self.device)
        bits = torch.zeros(1, dtype=torch.int64, device=self.device)
        N.check(N.lib().csv_key_encode(self._h, w, h, qstep, frame.data_ptr(), lev.data_ptr(),
                                       bits.data_ptr(), _stream(self.device)))
        return lev, bits

    def key_decode(self, levels: torch.Tensor, qstep: int = 16) -> torch.Tensor:
        _require_cuda(levels, torch.int16, "levels")
        h, w = levels.shape
        out = torch.empty((h, w), dtype=torch.uint8, device=self.device)
        N.check(N.lib().csv_key_decode(self._h, w, h, qstep, levels.data_ptr(), out.data_ptr(),
                                       _stream(self.device)))
        return out

    def measure_frame(self, p: Params, frame: torch.Tensor, key_decoded: torch.Tensor):
        _require_cuda(frame, torch.uint8, "frame")
        _require_cuda(key_decoded, torch.uint8, "key_decoded")
        m, nb = p.resolve()
        y = torch.empty((nb, m), dtype=torch.int32, device=self.device)
        cdt = torch.int32 if p.flags & N.CSV_FLAG_NO_QUANT else torch.int8
        codes = torch.empty((nb, m), dtype=cdt, device=self.device)
        exps = torch.empty((nb,), dtype=torch.uint8, device=self.device)
        N.check(N.lib().csv_measure_frame(self._h, C.byref(p.to_c()), frame.data_ptr(),
                                          key_decoded.data_ptr(), y.data_ptr(), codes.data_ptr(),
                                          exps.data_ptr(), _stream(self.device)))
        return y, codes, exps

    def recover_blocks(self, p: Params, codes: torch.Tensor, exps: torch.Tensor,
                       want_obj: bool = False):
        _require_cuda(codes, torch.int8, "codes")
        _require_cuda(exps, torch.uint8, "exps")
        m, _ = p.resolve()
        nblk = exps.numel()
        if codes.numel() != nblk * m:
            raise ValueError("codes must hold n_blocks x M entries")
        s = torch.empty((nblk, p.n), dtype=torch.float32, device=self.device)
        lam = torch.empty((nblk,), dtype=torch.float32, device=self.device)
        obj = torch.empty((nblk, 2), dtype=torch.float64, device=self.device) if want_obj else None
        N.check(N.lib().csv_recover_blocks(self._h, C.byref(p.to_c()), nblk, codes.data_ptr(),
                                           exps.data_ptr(), s.data_ptr(), lam.data_ptr(),
                                           _ptr(obj), _stream(self.device)))
        return s, lam, obj


def measure_frame_noalloc(p: Params, q: torch.Tensor, frame: torch.Tensor,
                          key_decoded: torch.Tensor, y: torch.Tensor, codes: torch.Tensor,
                          exps: torch.Tensor) -> None:
    """csv_measure_frame_noalloc: the measurement of one CS frame into the
    caller's y (N_b x M int32, or None), codes (N_b x M int8; int32 with
    CSV_FLAG_NO_QUANT) and exps (N_b uint8), with the measurement matrix q
    (M x n int8, as Context.phi_matrix returns it); the library allocates no
    device memory (its working memory is a fixed device array), so every
    output is the caller's.  Runs on the current device and stream."""
    for t, dt, name in ((q, torch.int8, "q"), (frame, torch.uint8, "frame"),
                        (key_decoded, torch.uint8, "key_decoded"), (exps, torch.uint8, "exps")):
        _require_cuda(t, dt, name)
    _require_cuda(codes, torch.int32 if p.flags & N.CSV_FLAG_NO_QUANT else torch.int8, "codes")
    if y is not None:
        _require_cuda(y, torch.int32, "y")
    N.check(N.lib().csv_measure_frame_noalloc(
        C.byref(p.to_c()), q.data_ptr(), frame.data_ptr(), key_decoded.data_ptr(), _ptr(y),
        codes.data_ptr(), exps.data_ptr(), _stream(frame.device)))
