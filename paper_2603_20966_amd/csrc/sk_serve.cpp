// Request server: continuous batching of sketch requests of uneven shapes on
// one device.  The policy (queue, arena, admission, batching) is sk::Scheduler;
// this file is its executor: one worker thread per server stages A where
// needed, launches each batch as one persistent kernel plus one batched FP64
// strip sum on a stream of a small pool, and polls completion events.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/sketch_serve.h"
#include "sk_check.hpp"
#include "sk_internal.hpp"
#include "sk_sched.hpp"

namespace {

using namespace sk::check;

constexpr int kMaxQueue = 4096;
constexpr size_t kKeepFinished = 65536;
constexpr int kMaxStreams = 8;
constexpr int kMinFlights = 2;

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// Tiles, strips and memory of one request: exactly what a direct call on the
// same arguments would use.
struct Geometry {
    enum Path { kStream = 0, kMfma = 1, kMfmaLp = 2 };
    int path = kStream;
    int kclass = 0;          // streaming kernel: sketch-width class
    int nt = 0;              // matrix-core kernels: N-tiles of 16 columns
    int64_t strips = 0;      // contraction strips (partials when > 1)
    int64_t ncols = 0;       // column groups (streaming) or column blocks (matrix cores)
    int64_t rows = 0;        // rows per matrix-core tile
    size_t partial_bytes = 0;
    int64_t a_ld = 0;        // ld of a staged A (elements)
    size_t a_bytes = 0;      // staged A bytes (0 for device A)
    int tile_class = 0;
    size_t footprint = 0;
};

Geometry geometry(const sk_request& r) {
    Geometry g;
    const int64_t C = sk::strip_width_for(r.a_dtype, r.k);
    g.strips = (r.n + C - 1) / C;
    if (sk::use_mfma(r.a_dtype, r.k)) {
        g.path = Geometry::kMfma;
        g.nt = sk::mfma_ntiles(r.k);
        g.rows = sk::kMfmaRows;
        g.ncols = (r.k + 16 * g.nt - 1) / (16 * g.nt);
        g.tile_class = 1000 + g.nt;
    } else if (sk::use_mfma_lp(r.a_dtype, r.k)) {
        g.path = Geometry::kMfmaLp;
        g.nt = sk::lp_ntiles(r.k);
        g.rows = sk::kLpBatchRows;
        g.ncols = (r.k + 16 * g.nt - 1) / (16 * g.nt);
        g.tile_class = 2000 + 10 * r.a_dtype + g.nt;
    } else {
        g.kclass = sk::k_class((int)std::min<int64_t>(r.k, sk::kColGroup));
        g.ncols = (r.k + sk::kColGroup - 1) / sk::kColGroup;
        g.tile_class = 100 * r.a_dtype + g.kclass;
    }
    g.partial_bytes = sk::gemm_workspace_bytes(r.m, g.strips, r.k);
    if (r.a_source != SK_SRC_DEVICE) {
        const int es = elem_size(r.a_dtype);
        const int64_t q = 16 / es;
        g.a_ld = (r.n + q - 1) / q * q;
        g.a_bytes = (size_t)r.m * (size_t)g.a_ld * (size_t)es;
    }
    g.footprint = up256(g.a_bytes) + up256(g.partial_bytes);
    return g;
}

int validate(const sk_request* r) {
    if (r == nullptr) return SK_EINVAL;
    if (r->a_source != SK_SRC_DEVICE && r->a_source != SK_SRC_HOST && r->a_source != SK_SRC_SYNTH)
        return SK_EINVAL;
    int st = check_common(r->a_dtype, r->m, r->k, r->omega_col0, r->Y, r->y_dtype, r->ldy,
                          r->beta);
    if (st != SK_OK) return st;
    if (r->m < 1 || r->n < 1 || r->k < 1) return SK_EINVAL;
    if (!dist_ok(r->omega_dist)) return SK_EINVAL;
    if (r->a_source == SK_SRC_DEVICE)
        return check_block(r->A, r->a_dtype, r->m, r->n, r->lda, r->omega_row0, r->a_scales);
    if (r->omega_row0 < 0 || r->omega_row0 > kMaxRow - r->n) return SK_EINVAL;
    if (r->a_source == SK_SRC_HOST) {
        if (r->A == nullptr || r->lda < r->n) return SK_EINVAL;
    } else if (r->A != nullptr || r->a_dtype != SK_A_F32) {
        return SK_EINVAL;
    }
    if (r->a_dtype == SK_A_FP8_E4M3 && r->a_scales == nullptr) return SK_EINVAL;
    if (r->a_scales && ((uintptr_t)r->a_scales & 3u)) return SK_EALIGN;
    return SK_OK;
}

struct ServerReq {
    sk_request r{};
    Geometry g;
    void* a_dev = nullptr;       // A as the kernels read it
    int64_t a_ld = 0;
    float* partials = nullptr;
    int status = SK_OK;
    int batch_size = 0;
    double stage_us = 0, sketch_us = 0;
};

struct Flight {
    int64_t batch = 0;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};   // start, staged, done
    std::vector<int64_t> ids;
    int status = SK_OK;
};

}  // namespace

struct sk_server {
    int device = 0;
    char* arena = nullptr;
    size_t budget = 0;
    std::vector<hipStream_t> streams;
    size_t next_stream = 0;
    std::vector<hipEvent_t> event_pool;
    sk::Scheduler sched;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    std::map<int64_t, ServerReq> reqs;
    std::deque<int64_t> finished;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    sk_server(size_t budget_bytes, int slots, int batch)
        : budget(budget_bytes), sched(budget_bytes, slots, batch, kMaxQueue) {}

    double now() const {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0)
            .count();
    }
    hipEvent_t take_event() {
        if (!event_pool.empty()) {
            hipEvent_t e = event_pool.back();
            event_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

namespace {

// Enqueue one batch (worker thread, no lock held: the requests' records are
// only read, and no other thread changes an admitted request).
void launch_batch(sk_server* S, const sk::Batch& b, const std::vector<ServerReq*>& rq,
                  Flight& f) {
    f.batch = b.id;
    f.ids = b.reqs;
    for (hipEvent_t& e : f.ev) e = S->take_event();
    if (!f.ev[0] || !f.ev[1] || !f.ev[2]) {
        f.status = SK_EHIP;
        return;
    }
    hipStream_t st = S->streams[S->next_stream++ % S->streams.size()];
    hipError_t err = hipEventRecord(f.ev[0], st);
    for (ServerReq* q : rq) {
        if (err != hipSuccess) break;
        const sk_request& r = q->r;
        if (r.a_source == SK_SRC_HOST) {
            const size_t es = (size_t)elem_size(r.a_dtype);
            err = hipMemcpy2DAsync(q->a_dev, (size_t)q->a_ld * es, r.A, (size_t)r.lda * es,
                                   (size_t)r.n * es, (size_t)r.m, hipMemcpyHostToDevice, st);
        } else if (r.a_source == SK_SRC_SYNTH) {
            err = sk::launch_fill_normal(static_cast<float*>(q->a_dev), r.m, r.n, q->a_ld, r.a_seed,
                                         st);
        }
    }
    if (err == hipSuccess) err = hipEventRecord(f.ev[1], st);

    sk::BatchArgs a{};
    a.count = (int)rq.size();
    int64_t tiles = 0, outs = 0;
    for (size_t i = 0; i < rq.size(); ++i) {
        const ServerReq& q = *rq[i];
        const sk_request& r = q.r;
        sk::BatchReq& x = a.req[i];
        x.A = q.a_dev;
        x.n = r.n;
        x.lda = q.a_ld;
        x.row0 = r.omega_row0;
        x.scales = r.a_scales;
        x.m = r.m;
        x.k = r.k;
        x.Y = r.Y;
        x.ldy = r.ldy;
        x.partials = q.partials;
        x.seed = r.seed;
        x.col0 = (uint32_t)r.omega_col0;
        x.dist = r.omega_dist;
        x.y_f64 = r.y_dtype == SK_Y_F64;
        x.beta = r.beta;
        x.strips = (int32_t)q.g.strips;
        x.rows_per_wg = (int32_t)(q.g.path != Geometry::kStream
                                      ? q.g.rows
                                      : sk::rows_per_tile(r.m, q.g.strips, q.g.ncols,
                                                          sk::stream_max_rows(q.g.kclass)));
        x.rowblocks = (int32_t)((r.m + x.rows_per_wg - 1) / x.rows_per_wg);
        x.tile_begin = tiles;
        x.out_begin = outs;
        tiles += (int64_t)x.strips * x.rowblocks * q.g.ncols;
        if (x.strips > 1) outs += r.m * r.k;
    }
    a.total_tiles = tiles;
    a.total_outputs = outs;
    const ServerReq& q0 = *rq[0];
    if (err == hipSuccess) {
        switch (q0.g.path) {
        case Geometry::kMfma: err = sk::launch_gemm_mfma_batch(a, q0.g.nt, 0, st); break;
        case Geometry::kMfmaLp:
            err = sk::launch_gemm_mfma_lp_batch(a, q0.g.nt, q0.r.a_dtype, 0, st);
            break;
        default: err = sk::launch_gemm_batch(a, q0.g.kclass, q0.r.a_dtype, 0, st);
        }
    }
    if (err == hipSuccess) err = hipEventRecord(f.ev[2], st);
    if (err != hipSuccess) {
        f.status = SK_EHIP;
        (void)hipStreamSynchronize(st);   // nothing enqueued may outlive the memory it uses
    }
}

void worker_main(sk_server* S) {
    (void)hipSetDevice(S->device);
    std::vector<Flight> flights;
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        // ---- admit and assign arena memory ------------------------------------
        // While fewer than kMinFlights batches keep the device busy, admit what
        // fits at once; beyond that, wait until half the slots are free, so that
        // requests arriving under load share launches.
        const int min_free = (int)flights.size() < kMinFlights ? 1 : S->sched.max_running() / 2;
        std::vector<sk::Batch> batches = S->sched.admit(S->now(), min_free);
        std::vector<std::vector<ServerReq*>> members;
        for (const sk::Batch& b : batches) {
            std::vector<ServerReq*> v;
            for (int64_t id : b.reqs) {
                ServerReq& q = S->reqs[id];
                sk::Req rec;
                S->sched.get(id, &rec);
                char* base = rec.arena_offset >= 0 ? S->arena + rec.arena_offset : nullptr;
                if (q.r.a_source == SK_SRC_DEVICE) {
                    q.a_dev = const_cast<void*>(q.r.A);
                    q.a_ld = q.r.lda;
                } else {
                    q.a_dev = base;
                    q.a_ld = q.g.a_ld;
                }
                q.partials = q.g.partial_bytes
                                 ? reinterpret_cast<float*>(base + up256(q.g.a_bytes))
                                 : nullptr;
                q.batch_size = (int)b.reqs.size();
                v.push_back(&q);
            }
            members.push_back(v);
        }
        lk.unlock();

        // ---- launch ---------------------------------------------------------------
        std::vector<Flight> failed_now;
        for (size_t i = 0; i < batches.size(); ++i) {
            Flight f;
            launch_batch(S, batches[i], members[i], f);
            if (f.status == SK_OK) flights.push_back(f);
            else failed_now.push_back(f);
        }

        // ---- poll completions -----------------------------------------------------
        std::vector<Flight> done;
        for (size_t i = 0; i < flights.size();) {
            const hipError_t q = hipEventQuery(flights[i].ev[2]);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            if (q != hipSuccess) flights[i].status = SK_EHIP;
            done.push_back(flights[i]);
            flights.erase(flights.begin() + (ptrdiff_t)i);
        }
        for (Flight& f : failed_now) done.push_back(f);

        lk.lock();
        const double t = S->now();
        for (Flight& f : done) {
            float stage_ms = 0, sketch_ms = 0;
            if (f.status == SK_OK) {
                (void)hipEventElapsedTime(&stage_ms, f.ev[0], f.ev[1]);
                (void)hipEventElapsedTime(&sketch_ms, f.ev[1], f.ev[2]);
            }
            for (int64_t id : f.ids) {
                ServerReq& q = S->reqs[id];
                q.status = f.status;
                q.stage_us = 1e3 * stage_ms;
                q.sketch_us = 1e3 * sketch_ms;
                S->finished.push_back(id);
            }
            S->sched.finish_batch(f.batch, f.status == SK_OK, t);
            for (hipEvent_t e : f.ev)
                if (e) S->event_pool.push_back(e);
        }
        while (S->finished.size() > kKeepFinished) {
            const int64_t id = S->finished.front();
            S->finished.pop_front();
            S->sched.forget(id);
            S->reqs.erase(id);
        }
        if (!done.empty()) S->cv_done.notify_all();

        const sk::SchedStats st = S->sched.stats();
        if (S->stop && st.queued == 0 && flights.empty()) break;
        if (flights.empty()) {
            // nothing on the device: sleep until a submission (or stop)
            if (st.queued == 0)
                S->cv_work.wait(lk, [&] { return S->stop || S->sched.stats().queued > 0; });
        } else {
            // work in flight: poll its events again soon, admitting what arrives
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        }
    }
}

void fill_info(sk_server* S, int64_t id, sk_ticket_info* info) {
    sk::Req rec;
    S->sched.get(id, &rec);
    const ServerReq& q = S->reqs[id];
    sk_ticket_info x{};
    x.state = rec.state;
    x.status = q.status;
    x.batch = rec.batch > 0 ? rec.batch : 0;
    x.batch_size = q.batch_size;
    x.footprint = q.g.footprint;
    x.t_submit_us = rec.t_submit;
    x.t_admit_us = rec.t_start;
    x.t_done_us = rec.t_done;
    x.stage_us = q.stage_us;
    x.sketch_us = q.sketch_us;
    *info = x;
}

}  // namespace

extern "C" {

size_t sk_request_footprint(const sk_request* r) {
    if (validate(r) != SK_OK) return 0;
    return geometry(*r).footprint;
}

int sk_server_create(size_t budget_bytes, int max_slots, int max_batch, int n_streams,
                     sk_server** out) {
    if (out == nullptr) return SK_EINVAL;
    *out = nullptr;
    if (max_slots < 1 || max_batch < 1 || max_batch > sk::kMaxBatch || n_streams < 1 ||
        n_streams > kMaxStreams)
        return SK_EINVAL;
    sk_server* S = new (std::nothrow) sk_server(budget_bytes, max_slots, max_batch);
    if (S == nullptr) return SK_ENOMEM;
    int st = SK_OK;
    if (hipGetDevice(&S->device) != hipSuccess) st = SK_EHIP;
    if (st == SK_OK && budget_bytes > 0 &&
        hipMalloc(reinterpret_cast<void**>(&S->arena), budget_bytes) != hipSuccess) {
        (void)hipGetLastError();
        st = SK_ENOMEM;
    }
    for (int i = 0; st == SK_OK && i < n_streams; ++i) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) st = SK_EHIP;
        else S->streams.push_back(s);
    }
    if (st == SK_OK) {
        try {
            S->worker = std::thread(worker_main, S);
        } catch (...) {
            st = SK_EHIP;
        }
    }
    if (st != SK_OK) {
        for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
        if (S->arena) (void)hipFree(S->arena);
        delete S;
        return st;
    }
    *out = S;
    return SK_OK;
}

int sk_server_submit(sk_server* S, const sk_request* r, int64_t* ticket) {
    if (S == nullptr || ticket == nullptr) return SK_EINVAL;
    *ticket = 0;
    const int v = validate(r);
    if (v != SK_OK) return v;
    ServerReq q;
    q.r = *r;
    q.g = geometry(*r);
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return SK_EINVAL;
    const int64_t id = S->sched.submit(sk::ReqInfo{q.g.footprint, q.g.tile_class}, S->now());
    if (id == -1) return SK_EBUDGET;
    if (id < 0) return SK_EQUEUE;
    S->reqs[id] = q;
    *ticket = id;
    S->cv_work.notify_one();
    return SK_OK;
}

int sk_server_poll(sk_server* S, int64_t ticket, sk_ticket_info* info) {
    if (S == nullptr || info == nullptr) return SK_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->reqs.find(ticket) == S->reqs.end()) return SK_EQUEUE;
    fill_info(S, ticket, info);
    return SK_OK;
}

int sk_server_wait(sk_server* S, int64_t ticket, double timeout_s, sk_ticket_info* info) {
    if (S == nullptr || info == nullptr) return SK_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto finished = [&] {
        sk::Req rec;
        return !S->sched.get(ticket, &rec) || rec.state >= sk::kDone;
    };
    if (S->reqs.find(ticket) == S->reqs.end()) return SK_EQUEUE;
    if (timeout_s < 0) {
        S->cv_done.wait(lk, finished);
    } else if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), finished)) {
        fill_info(S, ticket, info);
        return SK_ETIMEOUT;
    }
    if (S->reqs.find(ticket) == S->reqs.end()) return SK_EQUEUE;
    fill_info(S, ticket, info);
    return SK_OK;
}

int sk_server_cancel(sk_server* S, int64_t ticket) {
    if (S == nullptr) return SK_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (!S->sched.cancel(ticket)) return SK_EQUEUE;
    S->finished.push_back(ticket);
    S->cv_done.notify_all();
    return SK_OK;
}

int sk_server_stats(sk_server* S, sk_serve_stats* out) {
    if (S == nullptr || out == nullptr) return SK_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    const sk::SchedStats st = S->sched.stats();
    sk_serve_stats x{};
    x.submitted = st.submitted;
    x.admitted = st.admitted;
    x.completed = st.completed;
    x.failed = st.failed;
    x.cancelled = st.cancelled;
    x.rejected = st.rejected;
    x.batches = st.batches;
    x.queued = st.queued;
    x.running = st.running;
    x.max_running = st.max_running;
    x.budget_bytes = S->budget;
    x.bytes_in_use = st.bytes_in_use;
    x.peak_bytes_in_use = st.peak_bytes_in_use;
    *out = x;
    return SK_OK;
}

double sk_server_now_us(sk_server* S) { return S ? S->now() : 0.0; }

int sk_server_destroy(sk_server* S) {
    if (S == nullptr) return SK_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (auto& kv : S->reqs) {
            sk::Req rec;
            if (S->sched.get(kv.first, &rec) && rec.state == sk::kQueued)
                S->sched.cancel(kv.first);
        }
        S->cv_work.notify_all();
        S->cv_done.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    int st = SK_OK;
    for (hipStream_t s : S->streams) {
        if (hipStreamSynchronize(s) != hipSuccess) st = SK_EHIP;
        (void)hipStreamDestroy(s);
    }
    for (hipEvent_t e : S->event_pool) (void)hipEventDestroy(e);
    if (S->arena && hipFree(S->arena) != hipSuccess) st = SK_EHIP;
    delete S;
    return st;
}

}  // extern "C"
