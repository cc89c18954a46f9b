"""Serving-loop logic on the CPU with the host-only fake executor:
admission by memory budget, queue limits, cancellation, injected batch
failures, latency bookkeeping and concurrent submitters."""
import ctypes
import threading
import time

import numpy as np
import pytest

import paper_1311_1419_amd as P
from paper_1311_1419_amd import _native as N


class FakeGop:
    """Non-null placeholders: the fake executor never dereferences them."""
    def to_c(self):
        return N.CsvGopStream(0x1000, 0x2000, 0x3000, None)


PARAMS = P.Params(width=176, height=144, gop=4, block=16, m=64)   # 297 blocks, 101 376 output bytes
OUT_BYTES = 4 * 176 * 144
# a BF16 request's charge: its frames plus, per recovery block, the
# coefficients and lambda's adjoint (4 n each), y^ (4 Mp) and lambda (4)
REQ_BYTES = OUT_BYTES + 3 * 99 * (2 * 256 * 4 + 64 * 4 + 4)


def _server(**kw):
    base = dict(fake_executor=True, fake_us_per_block=1.0, hip_streams=2)
    base.update(kw)
    return P.Server(**base)


def _out():
    return (ctypes.c_uint8 * (4 * 176 * 144))()


def _poll_until(srv, t, out=None, timeout=10.0):
    end = time.time() + timeout
    while time.time() < end:
        if srv.poll(t, out):
            return True
        time.sleep(0.001)
    raise AssertionError("request did not complete")


def test_submit_poll_and_stats():
    with _server() as srv:
        sid = srv.register_stream(PARAMS)
        tickets = [srv.submit(sid, FakeGop(), P.clock()) for _ in range(12)]
        srv.drain(10.0)
        for t in tickets:
            buf = _out()
            assert _poll_until(srv, t, buf)
            assert np.all(np.frombuffer(buf, dtype=np.uint8) == (t & 0xFF))
        st = srv.stats()
        assert st["submitted"] == st["admitted"] == st["completed"] == 12
        assert st["recovered_pixels"] == 12 * 3 * 176 * 144
        assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
        assert st["bytes_in_flight"] == 0 and st["batches"] >= 1


def test_memory_budget_limits_admission():
    # 297 blocks at 100 us each: a request runs for about 30 ms
    with _server(mem_budget=2 * REQ_BYTES, fake_us_per_block=100.0) as srv:
        sid = srv.register_stream(PARAMS)
        tickets = [srv.submit(sid, FakeGop()) for _ in range(5)]
        time.sleep(0.005)
        st = srv.stats()
        assert st["admitted"] == 2 and st["queue_depth"] == 3
        # finished requests keep only their frames charged, so all five fit
        # without any poll
        srv.drain(10.0)
        st = srv.stats()
        assert st["completed"] == 5 and st["peak_bytes"] <= 2 * REQ_BYTES
        assert st["bytes_in_flight"] == 5 * OUT_BYTES
        for t in tickets:
            _poll_until(srv, t)
        assert srv.stats()["bytes_in_flight"] == 0


def test_drain_reports_a_budget_held_by_unpolled_outputs():
    # room for one running request and one finished output: the third
    # request cannot be admitted until a finished one is polled
    with _server(mem_budget=REQ_BYTES + OUT_BYTES) as srv:
        sid = srv.register_stream(PARAMS)
        tickets = [srv.submit(sid, FakeGop()) for _ in range(3)]
        t0 = time.time()
        with pytest.raises(N.CsvError) as ei:
            srv.drain(30.0)
        assert ei.value.code == N.CSV_EAGAIN and "not polled" in str(ei.value)
        assert time.time() - t0 < 5.0                   # reported, not timed out
        st = srv.stats()
        assert st["completed"] == 2 and st["queue_depth"] == 1
        for t in tickets[:2]:
            _poll_until(srv, t)
        srv.drain(5.0)
        _poll_until(srv, tickets[2])
        assert srv.stats()["completed"] == 3


def test_queue_full_and_oversized_request():
    with _server(mem_budget=REQ_BYTES - 1, max_queue=3) as srv:
        sid = srv.register_stream(PARAMS)
        with pytest.raises(N.CsvError) as ei:
            srv.submit(sid, FakeGop())
        assert ei.value.code == N.CSV_ENOMEM
    with _server(mem_budget=REQ_BYTES, max_queue=3) as srv:
        sid = srv.register_stream(PARAMS)
        first = srv.submit(sid, FakeGop())
        time.sleep(0.02)                                # first admitted, holds the budget
        for _ in range(3):
            srv.submit(sid, FakeGop())
        with pytest.raises(N.CsvError) as ei:
            srv.submit(sid, FakeGop())
        assert ei.value.code == N.CSV_EAGAIN
        assert srv.stats()["rejected"] == 1
        _poll_until(srv, first)


def test_cancel_waiting_request():
    with _server(mem_budget=REQ_BYTES) as srv:
        sid = srv.register_stream(PARAMS)
        a = srv.submit(sid, FakeGop())
        b = srv.submit(sid, FakeGop())                  # waits: budget held by a
        srv.cancel(b)
        with pytest.raises(N.CsvError) as ei:
            srv.poll(b)
        assert ei.value.code == N.CSV_ECANCELED
        _poll_until(srv, a)
        assert srv.stats()["cancelled"] == 1


def test_injected_batch_failures_fail_only_their_requests():
    with _server(fake_fail_every=2, hip_streams=1, max_batch_blocks=297) as srv:
        sid = srv.register_stream(PARAMS)
        tickets = [srv.submit(sid, FakeGop()) for _ in range(6)]
        srv.drain(5.0)
        ok = failed = 0
        for t in tickets:
            try:
                _poll_until(srv, t)
                ok += 1
            except N.CsvError as e:
                assert e.code == N.CSV_EHIP and "injected" in str(e)
                failed += 1
        assert ok == 3 and failed == 3
        st = srv.stats()
        assert st["failed"] == 3 and st["completed"] == 3 and st["bytes_in_flight"] == 0


def test_latency_includes_service_time_and_unknown_ids():
    with _server(fake_us_per_block=200.0, hip_streams=1) as srv:
        sid = srv.register_stream(PARAMS)
        t = srv.submit(sid, FakeGop(), P.clock())
        _poll_until(srv, t)
        assert srv.stats()["max_ms"] >= 297 * 0.2 * 0.99
        with pytest.raises(N.CsvError) as ei:
            srv.submit(sid + 7, FakeGop())
        assert ei.value.code == N.CSV_ENOTFOUND
        with pytest.raises(N.CsvError) as ei:
            srv.poll(123456)
        assert ei.value.code == N.CSV_ENOTFOUND


def test_concurrent_submitters():
    with _server(fake_us_per_block=0.5) as srv:
        sid = srv.register_stream(PARAMS)
        tickets, lock = [], threading.Lock()

        def work():
            for _ in range(25):
                t = srv.submit(sid, FakeGop())
                with lock:
                    tickets.append(t)

        th = [threading.Thread(target=work) for _ in range(4)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        assert len(set(tickets)) == 100
        srv.drain(10.0)
        for t in tickets:
            _poll_until(srv, t)
        assert srv.stats()["completed"] == 100


def test_bad_server_options():
    with pytest.raises(N.CsvError):
        P.Server(fake_executor=True, hip_streams=9)
    with pytest.raises(N.CsvError):
        P.Server(fake_executor=True, precision=5)
    with _server() as srv:
        with pytest.raises(N.CsvError):
            srv.register_stream(PARAMS.with_(gop=1))


def test_working_set_charge_follows_the_path():
    """A request is charged the recovery working set of its path: the plain
    FP32 iteration adds v and the residual per block (4 n + 4 Mp), FP32 TV
    its seven state arrays and step on top of that."""
    per_bf16 = 2 * 256 * 4 + 64 * 4 + 4
    per_fp32 = per_bf16 + 256 * 4 + 64 * 4
    per_tv32 = per_fp32 + 7 * 256 * 4 + 4
    for prec, flags, per in ((N.CSV_BF16, 0, per_bf16), (N.CSV_FP32, 0, per_fp32),
                             (N.CSV_FP32, P.CSV_FLAG_TV, per_tv32)):
        need = OUT_BYTES + 297 * per
        with _server(mem_budget=need - 1, precision=prec) as srv:
            sid = srv.register_stream(PARAMS.with_(flags=flags))
            with pytest.raises(N.CsvError) as ei:
                srv.submit(sid, FakeGop())
            assert ei.value.code == N.CSV_ENOMEM
        with _server(mem_budget=need, precision=prec) as srv:
            sid = srv.register_stream(PARAMS.with_(flags=flags))
            t = srv.submit(sid, FakeGop())
            srv.drain(10.0)
            assert srv.stats()["peak_bytes"] == need
            _poll_until(srv, t)


def test_reset_stats_starts_a_new_window():
    """Requests submitted before csv_server_reset_stats (a warm-up) are left
    out of the counts, pixels and latencies; the window's first arrival and
    last completion bound the served rate."""
    with _server(fake_us_per_block=1.0) as srv:
        sid = srv.register_stream(PARAMS)
        warm = [srv.submit(sid, FakeGop()) for _ in range(3)]
        srv.drain(10.0)
        srv.reset_stats()
        st = srv.stats()
        assert st["completed"] == 0 and st["p99_ms"] == 0 and st["first_arrival_s"] == -1
        t0 = P.clock()
        tickets = [srv.submit(sid, FakeGop(), t0 + 0.001 * i) for i in range(4)]
        srv.drain(10.0)
        for t in warm + tickets:
            _poll_until(srv, t)
        st = srv.stats()
        assert st["submitted"] == 4 and st["completed"] == 4
        assert st["recovered_pixels"] == 4 * 3 * 176 * 144
        assert st["first_arrival_s"] == pytest.approx(t0)
        assert st["last_done_s"] >= t0
        span = st["last_done_s"] - st["first_arrival_s"]
        assert st["mpix_per_s"] == pytest.approx(st["recovered_pixels"] / span / 1e6, rel=1e-9)
