// Continuous-batching decode server (include/csv_server.h).
//
// A worker thread admits waiting requests in arrival order while the memory
// budget allows, groups admitted requests into batches of at most
// max_batch_blocks recovery blocks, and launches each batch on a free batch
// slot (one HIP stream and scratch set per slot).  Batches on different
// slots overlap on the device: the fused recovery launch of a new batch
// takes compute units as the tail of the running one frees them.  Device
// work goes through an Executor so that the admission and bookkeeping
// logic also runs with a host-only fake executor in tests.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <thread>

#include "csv_server.h"
#include "internal.h"

namespace csv {

double now_s() {
    using namespace std::chrono;
    return duration_cast<duration<double>>(steady_clock::now().time_since_epoch()).count();
}

enum ReqState { WAITING, ADMITTED, RUNNING, DONE, FAILED, CANCELLED };

struct StreamInfo {
    csv_params p;
    Shape s;
};

struct Request {
    uint64_t ticket = 0;
    uint32_t sid = 0;
    csv_gop_stream in{};
    double t_arr = 0, t_done = 0;
    size_t bytes = 0;
    size_t out_bytes = 0;
    int nblk = 0;
    uint8_t* out = nullptr;
    ReqState state = WAITING;
    bool cancel_requested = false;
    bool counted = true;   // submitted since the last statistics reset
    int err = CSV_OK;
    std::string msg;
};

class Executor {
  public:
    virtual ~Executor() = default;
    virtual int slots() const = 0;
    virtual void prepare(StreamInfo& si) = 0;
    // several streams' operators at once (their power iterations side by side)
    virtual void prepare_many(std::vector<StreamInfo>& sis) {
        for (auto& si : sis) prepare(si);
    }
    virtual uint8_t* alloc(size_t bytes) = 0;
    virtual void release(uint8_t* p, size_t bytes) = 0;
    virtual void launch(int slot, const std::vector<Request*>& batch,
                        const std::vector<StreamInfo>& streams) = 0;
    virtual bool done(int slot) = 0;
    virtual void copy_out(uint8_t* dst, const uint8_t* src, size_t bytes) = 0;
    // device bytes the executor holds: operators, slot scratch, output pool
    // (called on the worker thread, with the server lock held)
    virtual size_t device_bytes() = 0;
};

// ------------------------------------------------------------ HIP executor
class HipExecutor : public Executor {
  public:
    HipExecutor(int device, int nslots) : device_(device) {
        CSV_HIP(hipSetDevice(device));
        setup_.device = device;
        for (int i = 0; i < nslots; ++i) {
            auto c = std::make_unique<Ctx>();
            c->device = device;
            c->cache = setup_.cache;   // operators are shared by every slot
            hipStream_t st;
            CSV_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            hipEvent_t ev;
            CSV_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            slots_.push_back(Slot{std::move(c), st, ev});
        }
        CSV_HIP(hipStreamCreateWithFlags(&copy_, hipStreamNonBlocking));
    }
    ~HipExecutor() override {
        (void)hipSetDevice(device_);
        (void)hipDeviceSynchronize();
        for (auto& s : slots_) {
            release_ctx(s.ctx.get());
            (void)hipStreamDestroy(s.st);
            (void)hipEventDestroy(s.ev);
        }
        slots_.clear();
        release_ctx(&setup_);   // last owner of the operator cache
        for (auto& kv : pool_)
            for (void* p : kv.second) (void)hipFree(p);
        (void)hipStreamDestroy(copy_);
    }
    int slots() const override { return (int)slots_.size(); }
    // Builds the stream's operator in the shared cache (under the cache's
    // lock).  Nothing of the slot contexts is touched here: they belong to
    // the worker thread, which builds their momentum tables on first use.
    void prepare(StreamInfo& si) override {
        CSV_HIP(hipSetDevice(device_));
        get_operator(&setup_, si.s, copy_);
        CSV_HIP(hipStreamSynchronize(copy_));
    }
    void prepare_many(std::vector<StreamInfo>& sis) override {
        CSV_HIP(hipSetDevice(device_));
        std::vector<Shape> shapes;
        for (auto& si : sis) shapes.push_back(si.s);
        prepare_operators(&setup_, shapes.data(), (int)shapes.size(), copy_);
        for (auto& si : sis) get_operator(&setup_, si.s, copy_);   // any not batched
        CSV_HIP(hipStreamSynchronize(copy_));
    }
    uint8_t* alloc(size_t bytes) override {
        auto& fl = pool_[bytes];
        if (!fl.empty()) {
            void* p = fl.back();
            fl.pop_back();
            return static_cast<uint8_t*>(p);
        }
        void* p = nullptr;
        CSV_HIP(hipSetDevice(device_));
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            throw Error{CSV_ENOMEM, "server output allocation failed"};
        }
        pool_bytes_ += bytes;
        return static_cast<uint8_t*>(p);
    }
    void release(uint8_t* p, size_t bytes) override {
        if (p) pool_[bytes].push_back(p);
    }
    void launch(int slot, const std::vector<Request*>& batch,
                const std::vector<StreamInfo>& streams) override {
        CSV_HIP(hipSetDevice(device_));
        Slot& sl = slots_[slot];
        std::vector<Shape> shapes;
        std::vector<csv_gop_stream> ins;
        std::vector<uint8_t*> outs;
        for (Request* r : batch) {
            shapes.push_back(streams[r->sid].s);
            ins.push_back(r->in);
            outs.push_back(r->out);
        }
        decode_gops(sl.ctx.get(), (int)batch.size(), shapes.data(), ins.data(), outs.data(),
                    nullptr, nullptr, sl.st);
        CSV_HIP(hipEventRecord(sl.ev, sl.st));
    }
    bool done(int slot) override {
        const hipError_t e = hipEventQuery(slots_[slot].ev);
        if (e == hipSuccess) return true;
        if (e == hipErrorNotReady) return false;
        throw Error{CSV_EHIP, std::string("batch failed: ") + hipGetErrorString(e)};
    }
    void copy_out(uint8_t* dst, const uint8_t* src, size_t bytes) override {
        if (!dst) return;
        CSV_HIP(hipSetDevice(device_));
        CSV_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, copy_));
        CSV_HIP(hipStreamSynchronize(copy_));
    }
    size_t device_bytes() override {
        size_t b = pool_bytes_;
        for (auto& sl : slots_) b += sl.ctx->used;
        std::lock_guard<std::mutex> lk(setup_.cache->mu);   // register_stream may build
        return b + setup_.used;
    }

  private:
    struct Slot {
        std::unique_ptr<Ctx> ctx;
        hipStream_t st;
        hipEvent_t ev;
    };
    int device_;
    Ctx setup_;
    std::vector<Slot> slots_;
    hipStream_t copy_ = nullptr;
    std::map<size_t, std::vector<void*>> pool_;
    size_t pool_bytes_ = 0;   // every output buffer the pool holds, free or in use
};

// ----------------------------------------------------------- fake executor
// Host-only stand-in: one simulated device that serves batches in launch
// order at a fixed cost per recovery block; outputs are filled with the
// request's ticket (low byte) so a test can check which frames came back.
class FakeExecutor : public Executor {
  public:
    FakeExecutor(int nslots, double us_per_block, double fail_every)
        : us_(us_per_block), fail_every_(fail_every), until_(nslots, 0.0) {}
    int slots() const override { return (int)until_.size(); }
    void prepare(StreamInfo&) override {}
    uint8_t* alloc(size_t bytes) override { return static_cast<uint8_t*>(std::malloc(bytes)); }
    void release(uint8_t* p, size_t) override { std::free(p); }
    void launch(int slot, const std::vector<Request*>& batch,
                const std::vector<StreamInfo>&) override {
        ++launched_;
        if (fail_every_ > 0 && launched_ % (long)fail_every_ == 0)
            throw Error{CSV_EHIP, "injected batch failure"};
        int blocks = 0;
        for (Request* r : batch) {
            blocks += r->nblk;
            std::memset(r->out, (int)(r->ticket & 0xff), r->out_bytes);
        }
        const double start = std::max(now_s(), device_free_);
        device_free_ = start + us_ * 1e-6 * blocks;
        until_[slot] = device_free_;
    }
    bool done(int slot) override { return now_s() >= until_[slot]; }
    void copy_out(uint8_t* dst, const uint8_t* src, size_t bytes) override {
        if (dst) std::memcpy(dst, src, bytes);
    }
    size_t device_bytes() override { return 0; }

  private:
    double us_, fail_every_;
    std::vector<double> until_;
    double device_free_ = 0.0;
    long launched_ = 0;
};

// Device bytes of one request's recovery working set on the path its
// shape selects (the decode scratch of decode_gops): per block the
// coefficients S (4 n), lambda (4), y^ (4 Mp) and lambda's adjoint g0
// (4 n); the plain FP32 iteration adds v (4 n) and the residual (4 Mp);
// FP32 TV adds its multipliers, shrinkage variables, P, gradient and image
// (7 more arrays of 4 n) and its step (4); whole frames hold per CS frame
// the TV state (7 arrays of 4 n), y^ and the residual (4 M each), the
// forward product's partial sums (4 M per 512-pixel chunk), lambda and the
// step (8).
static size_t working_set_bytes(const Shape& s) {
    const size_t F = (size_t)(s.G - 1), n = (size_t)s.n, Mp = (size_t)s.Mp;
    if (s.flags & CSV_FLAG_WHOLE_FRAME)
        return F * (28 * n + 8 * (size_t)s.M + 4 * (size_t)s.M * whole_fwd_parts(s.n) + 8);
    const size_t nblk = F * s.nb;
    size_t per = 8 * n + 4 * Mp + 4;
    if (s.precision == CSV_FP32) {
        per += 4 * n + 4 * Mp;
        if (s.flags & CSV_FLAG_TV) per += 28 * n + 4;
    }
    return nblk * per;
}

// ------------------------------------------------------------------ server
struct Server {
    csv_server_opts o{};
    std::unique_ptr<Executor> ex;
    std::mutex mu;
    std::condition_variable cv;
    std::vector<StreamInfo> streams;
    std::deque<Request*> waiting, admitted;
    std::map<uint64_t, std::unique_ptr<Request>> reqs;
    std::vector<std::vector<Request*>> inflight;
    uint64_t next_ticket = 1;
    size_t bytes = 0, peak = 0;
    csv_stats st{};
    std::vector<double> lat_ms;
    double first_arrival = -1, last_done = 0;   // of requests counted since the last reset
    size_t dev_bytes = 0;                        // executor's device bytes, worker-updated
    bool stop = false;
    std::thread worker;

    int busy_slots() const {
        int b = 0;
        for (const auto& v : inflight) b += !v.empty();
        return b;
    }

    // Nothing runs or waits for a slot, yet the head request cannot be
    // admitted: only csv_poll (or csv_cancel) of finished requests frees
    // the budget it needs.
    bool stalled_locked() const {
        return !waiting.empty() && admitted.empty() && busy_slots() == 0 &&
               bytes + waiting.front()->bytes > o.mem_budget;
    }

    // Admit in arrival order while the budget allows (head-of-line).
    void admit_locked() {
        while (!waiting.empty()) {
            Request* r = waiting.front();
            if (bytes + r->bytes > o.mem_budget) break;
            r->out = ex->alloc(r->out_bytes);
            bytes += r->bytes;
            peak = std::max(peak, bytes);
            r->state = ADMITTED;
            waiting.pop_front();
            admitted.push_back(r);
            ++st.admitted;
        }
    }

    void release_locked(Request* r) {
        if (r->out) {
            ex->release(r->out, r->out_bytes);
            r->out = nullptr;
            bytes -= r->bytes;
        }
    }

    void finish_slot_locked(int slot, int err, const std::string& msg) {
        const double t = now_s();
        for (Request* r : inflight[slot]) {
            r->t_done = t;
            if (r->cancel_requested) {
                release_locked(r);
                r->state = CANCELLED;
                ++st.cancelled;
            } else if (err != CSV_OK) {
                release_locked(r);
                r->state = FAILED;
                r->err = err;
                r->msg = msg;
                ++st.failed;
            } else {
                // the recovery working set is free once the batch is done;
                // only the decoded frames stay charged until csv_poll
                bytes -= r->bytes - r->out_bytes;
                r->bytes = r->out_bytes;
                r->state = DONE;
                if (!r->counted) continue;   // submitted before the statistics reset
                ++st.completed;
                const StreamInfo& si = streams[r->sid];
                st.recovered_pixels += (uint64_t)(si.s.G - 1) * si.s.W * si.s.H;
                lat_ms.push_back(1e3 * (t - r->t_arr));
                last_done = t;
            }
        }
        inflight[slot].clear();
    }

    void run() {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            admit_locked();
            bool progressed = false;
            for (int s = 0; s < ex->slots(); ++s) {
                if (inflight[s].empty()) continue;
                bool fin = false;
                int err = CSV_OK;
                std::string msg;
                try {
                    fin = ex->done(s);
                } catch (const Error& e) {
                    fin = true;
                    err = e.code;
                    msg = e.msg;
                }
                if (fin) {
                    finish_slot_locked(s, err, msg);
                    progressed = true;
                }
            }
            if (progressed) {
                admit_locked();
                cv.notify_all();
            }
            int slot = -1;
            for (int s = 0; s < ex->slots(); ++s)
                if (inflight[s].empty()) {
                    slot = s;
                    break;
                }
            if (slot >= 0 && !admitted.empty()) {
                std::vector<Request*> batch;
                int blocks = 0;
                while (!admitted.empty()) {
                    Request* r = admitted.front();
                    if (!batch.empty() && blocks + r->nblk > o.max_batch_blocks) break;
                    admitted.pop_front();
                    if (r->cancel_requested) {
                        release_locked(r);
                        r->state = CANCELLED;
                        ++st.cancelled;
                        continue;
                    }
                    r->state = RUNNING;
                    blocks += r->nblk;
                    batch.push_back(r);
                }
                if (batch.empty()) continue;
                inflight[slot] = batch;
                ++st.batches;
                st.max_concurrent = std::max(st.max_concurrent, busy_slots());
                lk.unlock();
                int err = CSV_OK;
                std::string msg;
                try {
                    ex->launch(slot, batch, streams);
                } catch (const Error& e) {
                    err = e.code;
                    msg = e.msg;
                }
                lk.lock();
                dev_bytes = ex->device_bytes();
                if (err != CSV_OK) finish_slot_locked(slot, err, msg);
                continue;
            }
            if (stop && waiting.empty() && admitted.empty() && busy_slots() == 0) break;
            cv.wait_for(lk, std::chrono::microseconds(busy_slots() ? 100 : 5000));
        }
    }
};

}  // namespace csv

using namespace csv;

struct csv_server {
    Server impl;
};

static int guarded_s(const std::function<void()>& f) {
    try {
        f();
        return CSV_OK;
    } catch (const Error& e) {
        return fail(e.code, e.msg);
    } catch (const std::bad_alloc&) {
        return fail(CSV_ENOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(CSV_EINVAL, e.what());
    }
}

// Validate a stream for this server (its precision is the server's).
static StreamInfo stream_info(Server& s, const csv_params* p) {
    StreamInfo si;
    si.p = *p;
    si.p.precision = s.o.precision;
    si.s = resolve(&si.p);
    CSV_REQUIRE(si.s.G >= 2, CSV_EINVAL, "a served stream needs CS frames (gop >= 2)");
    const bool tv = (si.s.flags & CSV_FLAG_TV) != 0;
    if (si.s.flags & CSV_FLAG_WHOLE_FRAME)
        CSV_REQUIRE(tv && s.o.precision == CSV_FP32, CSV_EUNSUPPORTED,
                    "whole-frame streams are served in FP32 with CSV_FLAG_TV");
    else if (s.o.precision == CSV_BF16)
        CSV_REQUIRE(tv ? tv_class_supported(si.s.n, si.s.Mp)
                       : fused_class_supported(si.s.n, si.s.Mp),
                    CSV_EUNSUPPORTED, "no fused kernel for this block size and M");
    CSV_REQUIRE(!(si.s.flags & CSV_FLAG_MONOTONE) || s.o.precision == CSV_FP32,
                CSV_EUNSUPPORTED, "monotone FISTA runs on the plain FP32 path only");
    return si;
}

extern "C" {

double csv_clock(void) { return now_s(); }

int csv_server_create(int device, const csv_server_opts* opts, csv_server** out) {
    return guarded_s([&] {
        CSV_REQUIRE(out && opts, CSV_EINVAL, "NULL argument");
        auto* srv = new csv_server();
        Server& s = srv->impl;
        s.o = *opts;
        if (!s.o.mem_budget) s.o.mem_budget = (size_t)4 << 30;
        if (s.o.max_queue <= 0) s.o.max_queue = 4096;
        if (s.o.max_batch_blocks <= 0) s.o.max_batch_blocks = 262144;
        if (s.o.hip_streams <= 0) s.o.hip_streams = 2;
        try {
            CSV_REQUIRE(s.o.hip_streams <= 4, CSV_EINVAL, "hip_streams must be in 1..4");
            CSV_REQUIRE(s.o.precision == CSV_FP32 || s.o.precision == CSV_BF16, CSV_EINVAL,
                        "precision must be CSV_FP32 or CSV_BF16");
            if (s.o.flags & CSV_SERVER_FAKE_EXECUTOR)
                s.ex = std::make_unique<FakeExecutor>(s.o.hip_streams, s.o.fake_us_per_block,
                                                      s.o.fake_fail_every);
            else
                s.ex = std::make_unique<HipExecutor>(device, s.o.hip_streams);
        } catch (...) {
            delete srv;
            throw;
        }
        s.inflight.resize(s.ex->slots());
        s.worker = std::thread([&s] { s.run(); });
        *out = srv;
    });
}

int csv_server_destroy(csv_server* srv) {
    if (!srv) return CSV_OK;
    return guarded_s([&] {
        Server& s = srv->impl;
        {
            std::lock_guard<std::mutex> lk(s.mu);
            s.stop = true;
            for (Request* r : s.waiting) {
                r->state = CANCELLED;
            }
            s.waiting.clear();
        }
        s.cv.notify_all();
        if (s.worker.joinable()) s.worker.join();
        {
            std::lock_guard<std::mutex> lk(s.mu);
            for (auto& kv : s.reqs) s.release_locked(kv.second.get());
        }
        s.ex.reset();
        delete srv;
    });
}

int csv_server_register_stream(csv_server* srv, const csv_params* p, uint32_t* sid) {
    return guarded_s([&] {
        CSV_REQUIRE(srv && p && sid, CSV_EINVAL, "NULL argument");
        Server& s = srv->impl;
        StreamInfo si = stream_info(s, p);
        s.ex->prepare(si);   // operator setup outside the server lock
        std::lock_guard<std::mutex> lk(s.mu);
        s.streams.push_back(si);
        *sid = (uint32_t)(s.streams.size() - 1);
    });
}

int csv_server_register_streams(csv_server* srv, int32_t count, const csv_params* params,
                                uint32_t* sids) {
    return guarded_s([&] {
        CSV_REQUIRE(count >= 0, CSV_EINVAL, "negative count");
        if (count == 0) return;
        CSV_REQUIRE(srv && params && sids, CSV_EINVAL, "NULL argument");
        Server& s = srv->impl;
        std::vector<StreamInfo> sis;
        for (int i = 0; i < count; ++i) sis.push_back(stream_info(s, &params[i]));
        s.ex->prepare_many(sis);   // operator setup outside the server lock
        std::lock_guard<std::mutex> lk(s.mu);
        for (int i = 0; i < count; ++i) {
            s.streams.push_back(sis[i]);
            sids[i] = (uint32_t)(s.streams.size() - 1);
        }
    });
}

int csv_submit(csv_server* srv, uint32_t sid, const csv_gop_stream* in, double t_arrival,
               uint64_t* ticket) {
    return guarded_s([&] {
        CSV_REQUIRE(srv && in && ticket, CSV_EINVAL, "NULL argument");
        CSV_REQUIRE(in->key_levels && in->codes && in->exps, CSV_EINVAL, "NULL stream buffers");
        Server& s = srv->impl;
        std::lock_guard<std::mutex> lk(s.mu);
        CSV_REQUIRE(sid < s.streams.size(), CSV_ENOTFOUND, "unknown stream id");
        ++s.st.submitted;
        if ((int)s.waiting.size() >= s.o.max_queue) {
            ++s.st.rejected;
            throw Error{CSV_EAGAIN, "server queue full"};
        }
        const Shape& sh = s.streams[sid].s;
        auto r = std::make_unique<Request>();
        r->ticket = s.next_ticket++;
        r->sid = sid;
        r->in = *in;
        r->t_arr = t_arrival > 0 ? t_arrival : now_s();
        r->nblk = (sh.G - 1) * sh.nb;
        r->out_bytes = (size_t)sh.G * sh.W * sh.H;
        // output frames + the recovery working set of its blocks
        r->bytes = r->out_bytes + working_set_bytes(sh);
        r->counted = true;
        if (r->bytes > s.o.mem_budget) {
            ++s.st.rejected;
            throw Error{CSV_ENOMEM, "request larger than the server memory budget"};
        }
        if (s.first_arrival < 0 || r->t_arr < s.first_arrival) s.first_arrival = r->t_arr;
        *ticket = r->ticket;
        s.waiting.push_back(r.get());
        s.reqs.emplace(r->ticket, std::move(r));
        s.cv.notify_all();
    });
}

int csv_poll(csv_server* srv, uint64_t ticket, uint8_t* frames_out, int32_t* done) {
    int rc = CSV_OK;
    const int g = guarded_s([&] {
        CSV_REQUIRE(srv && done, CSV_EINVAL, "NULL argument");
        Server& s = srv->impl;
        std::unique_lock<std::mutex> lk(s.mu);
        auto it = s.reqs.find(ticket);
        CSV_REQUIRE(it != s.reqs.end(), CSV_ENOTFOUND, "unknown ticket");
        Request* r = it->second.get();
        *done = 0;
        if (r->state == DONE) {
            s.ex->copy_out(frames_out, r->out, r->out_bytes);
            s.release_locked(r);
            s.reqs.erase(it);
            *done = 1;
            s.cv.notify_all();
        } else if (r->state == FAILED) {
            rc = r->err;
            set_error(r->msg);
            s.reqs.erase(it);
        } else if (r->state == CANCELLED) {
            rc = CSV_ECANCELED;
            set_error("request was cancelled");
            s.reqs.erase(it);
        }
    });
    return g != CSV_OK ? g : rc;
}

int csv_cancel(csv_server* srv, uint64_t ticket) {
    return guarded_s([&] {
        CSV_REQUIRE(srv, CSV_EINVAL, "NULL argument");
        Server& s = srv->impl;
        std::lock_guard<std::mutex> lk(s.mu);
        auto it = s.reqs.find(ticket);
        CSV_REQUIRE(it != s.reqs.end(), CSV_ENOTFOUND, "unknown ticket");
        Request* r = it->second.get();
        switch (r->state) {
            case WAITING:
                s.waiting.erase(std::find(s.waiting.begin(), s.waiting.end(), r));
                r->state = CANCELLED;
                ++s.st.cancelled;
                break;
            case ADMITTED:
                s.admitted.erase(std::find(s.admitted.begin(), s.admitted.end(), r));
                s.release_locked(r);
                r->state = CANCELLED;
                ++s.st.cancelled;
                break;
            case RUNNING:
                r->cancel_requested = true;
                break;
            case DONE:
                s.release_locked(r);
                r->state = CANCELLED;
                ++s.st.cancelled;
                break;
            default:
                break;
        }
        s.cv.notify_all();
    });
}

int csv_server_drain(csv_server* srv, double timeout_s) {
    return guarded_s([&] {
        CSV_REQUIRE(srv, CSV_EINVAL, "NULL argument");
        Server& s = srv->impl;
        std::unique_lock<std::mutex> lk(s.mu);
        const auto until = std::chrono::steady_clock::now() +
                           std::chrono::microseconds((long long)(timeout_s * 1e6));
        while (!(s.waiting.empty() && s.admitted.empty() && s.busy_slots() == 0)) {
            CSV_REQUIRE(!s.stalled_locked(), CSV_EAGAIN,
                        "drain cannot finish: finished requests that were not polled hold the "
                        "memory budget the next request needs");
            if (s.cv.wait_until(lk, until) == std::cv_status::timeout &&
                !(s.waiting.empty() && s.admitted.empty() && s.busy_slots() == 0))
                throw Error{CSV_EAGAIN, "drain timed out"};
        }
    });
}

int csv_server_stats(csv_server* srv, csv_stats* out) {
    return guarded_s([&] {
        CSV_REQUIRE(srv && out, CSV_EINVAL, "NULL argument");
        Server& s = srv->impl;
        std::lock_guard<std::mutex> lk(s.mu);
        csv_stats r = s.st;
        r.bytes_in_flight = s.bytes;
        r.peak_bytes = s.peak;
        r.queue_depth = (int32_t)s.waiting.size();
        if (!s.lat_ms.empty()) {
            std::vector<double> v = s.lat_ms;
            std::sort(v.begin(), v.end());
            auto pct = [&](double q) {
                const double pos = q * (v.size() - 1);
                const size_t i = (size_t)pos;
                const double f = pos - i;
                return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
            };
            r.p50_ms = pct(0.50);
            r.p99_ms = pct(0.99);
            double sum = 0;
            for (double x : v) sum += x;
            r.mean_ms = sum / v.size();
            r.max_ms = v.back();
            const double span = s.last_done - s.first_arrival;
            r.mpix_per_s = span > 0 ? r.recovered_pixels / span / 1e6 : 0.0;
        }
        r.first_arrival_s = s.first_arrival;
        r.last_done_s = s.last_done;
        r.device_bytes = s.dev_bytes;
        *out = r;
    });
}

int csv_server_reset_stats(csv_server* srv) {
    return guarded_s([&] {
        CSV_REQUIRE(srv, CSV_EINVAL, "NULL argument");
        Server& s = srv->impl;
        std::lock_guard<std::mutex> lk(s.mu);
        for (auto& kv : s.reqs) kv.second->counted = false;
        s.st = csv_stats{};
        s.lat_ms.clear();
        s.first_arrival = -1;
        s.last_done = 0;
        s.peak = s.bytes;
    });
}

}  // extern "C"
