"""Python face of the continuous-batching decode server (csv_server.h)."""
from __future__ import annotations

import ctypes as C

from . import _native as N
from .api import GopStream, Params


def clock() -> float:
    """The server's latency clock (monotonic seconds)."""
    return N.lib().csv_clock()


class Server:
    """Decode server: register streams, submit GOPs as they arrive, poll."""

    def __init__(self, device: int = 0, mem_budget: int = 0, max_queue: int = 0,
                 max_batch_blocks: int = 0, precision: int = N.CSV_BF16, hip_streams: int = 0,
                 fake_executor: bool = False, fake_us_per_block: float = 0.0,
                 fake_fail_every: float = 0.0):
        opts = N.CsvServerOpts(mem_budget, max_queue, max_batch_blocks, precision, hip_streams,
                               N.CSV_SERVER_FAKE_EXECUTOR if fake_executor else 0,
                               fake_us_per_block, fake_fail_every)
        h = C.c_void_p()
        N.check(N.lib().csv_server_create(device, C.byref(opts), C.byref(h)))
        self._h = h
        self.fake = fake_executor
        self._keep = {}   # ticket -> stream buffers kept alive until completion

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            N.check(N.lib().csv_server_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def register_stream(self, p: Params) -> int:
        sid = C.c_uint32()
        N.check(N.lib().csv_server_register_stream(self._h, C.byref(p.to_c()), C.byref(sid)))
        return sid.value

    def register_streams(self, params) -> list[int]:
        """Register several streams at once (their operators' power
        iterations run side by side); returns their ids in order."""
        count = len(params)
        arr = (N.CsvParams * max(count, 1))()
        for i, p in enumerate(params):
            arr[i] = p.to_c()
        sids = (C.c_uint32 * max(count, 1))()
        N.check(N.lib().csv_server_register_streams(self._h, count, arr, sids))
        return list(sids[:count])

    def submit(self, sid: int, gs, t_arrival: float = 0.0) -> int:
        """gs: a GopStream of device tensors (or, with the fake executor, any
        object whose to_c() gives non-null pointers).  Inputs must be ready:
        the producing stream is synchronised here."""
        if not self.fake:
            import torch
            torch.cuda.current_stream().synchronize()
        t = C.c_uint64()
        N.check(N.lib().csv_submit(self._h, sid, C.byref(gs.to_c()), t_arrival, C.byref(t)))
        self._keep[t.value] = gs
        return t.value

    def poll(self, ticket: int, out=None):
        """Returns True once the frames were copied to `out` (a device
        tensor, or a host buffer with the fake executor; None discards)."""
        done = C.c_int32()
        ptr = None if out is None else (out.data_ptr() if hasattr(out, "data_ptr") else
                                        C.cast(out, C.c_void_p).value)
        rc = N.lib().csv_poll(self._h, ticket, ptr, C.byref(done))
        if rc != N.CSV_OK or done.value:
            self._keep.pop(ticket, None)
        N.check(rc)
        return bool(done.value)

    def cancel(self, ticket: int) -> None:
        N.check(N.lib().csv_cancel(self._h, ticket))

    def drain(self, timeout_s: float = 60.0) -> None:
        N.check(N.lib().csv_server_drain(self._h, timeout_s))

    def stats(self) -> dict:
        s = N.CsvStats()
        N.check(N.lib().csv_server_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in N.CsvStats._fields_}

    def reset_stats(self) -> None:
        """Start a new statistics window (requests already submitted are
        not counted when they finish)."""
        N.check(N.lib().csv_server_reset_stats(self._h))
