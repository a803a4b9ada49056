// Served path: continuous batching of assignment solves on one GPU.
//
// sk_submit copies a request's W to the device at once when its footprint
// (W plus the instance state) fits in the free part of the context arena and
// no earlier request is waiting for space; otherwise into pinned host staging.
// Copies run on a stream of their own, so they overlap the sweeps. A serving
// thread repeats a tick:
//   1. admit queued requests (FIFO) while their footprint fits (the policy
//      is in sk_sched.h); start the host-to-device copy of staged ones, and
//      take in those whose copy is complete; cold-start the new instances;
//   3. run a block of Sinkhorn iterations over every admitted instance at
//      once (one row-sweep launch and one column-sweep launch per iteration
//      cover all of them; each instance follows its own p ladder, tolerance
//      and cap on the device);
//   4. retire instances whose ladder finished: FP64 recheck and certificate,
//      reduction to CSR on the device, copy of the CSR to the host, release of
//      the device region; the exact solve of the reduced instance runs on a
//      host thread pool while the GPU keeps sweeping the others.
// Every per-instance computation depends only on that instance (work units,
// tile plan and reduction order are functions of n), so a request's result is
// the same alone and in any mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sk_alloc.h"
#include "sk_runtime.h"
#include "sk_sched.h"

namespace sk {

struct Request {
    uint64_t id = 0;
    int32_t n = 0;
    sk_params prm{};
    int16_t *staging = nullptr;  // host copy of W (in the pinned ring, or heap)
    size_t ring_off = 0;         // offset in the pinned ring
    bool in_ring = false;
    size_t off = 0, len = 0;     // device region in the arena
    Inst inst{};
    bool loaded = false;         // W is in its device region
    bool copying = false;        // placed, and its copy from the ring is in flight (ev)
    hipEvent_t ev = nullptr;     // completion of the host-to-device copy
    int phase = 0;               // 0 queued, 1 active, 2 solving, 3 done
    sk_status status = SK_OK;
    std::vector<int32_t> perm;
    int64_t weight = 0;
    sk_report rep{};
    std::vector<int64_t> rp;
    std::vector<int32_t> col;
    std::vector<int16_t> w;
    std::chrono::steady_clock::time_point t_submit;
};

struct Server {
    sk_ctx *ctx = nullptr;
    std::thread th;
    std::vector<std::thread> solvers;
    std::mutex mu;
    std::condition_variable cv, cv_solve;
    bool stop = false;
    uint64_t next_id = 1;
    std::deque<Request *> queue;
    std::deque<Request *> loading;  // admitted, copy in flight (serving thread only)
    int staged_waiting = 0;         // queued requests whose W is still on the host
    std::vector<Request *> active;
    std::unordered_map<uint64_t, Request *> reqs;
    std::deque<uint64_t> done_ids;  // finished requests in completion order (sk_completed)
    std::deque<Request *> solve_q;
    RangeAlloc ralloc;
    size_t tables_len = 0;
    Batch B;
    std::vector<RowUnit> init_units;
    std::vector<int> fresh_idx;  // host source of d_fresh (kept until the tick syncs)
    RowUnit *d_init_units = nullptr;
    std::string error;
    int iters_per_tick = 16;
    char *ring = nullptr;        // pinned staging for submitted W
    size_t ring_bytes = 0;
    RangeAlloc ring_alloc;
    int *d_fresh = nullptr;      // indices of admitted instances (device)
    hipStream_t copy_stream = nullptr;
};

static const size_t kRingBytes = size_t(512) << 20;

// Staged and device layout of a request's W: rows pad8(n) entries apart, so
// the kernels take 8-wide loads for every n.
static size_t wbytes_of(int32_t n) { return sizeof(int16_t) * (size_t)n * (size_t)pad8(n); }

static void release_staging(Server *S, Request *r) {
    if (!r->staging) return;
    if (r->in_ring) {
        S->ring_alloc.release(r->ring_off, wbytes_of(r->n));
    } else {
        free(r->staging);
    }
    r->staging = nullptr;
}

static const size_t kTablesBytes = size_t(64) << 20;

// Host copy of a submitted W into staging: one thread per kCopyChunk bytes,
// at most kCopyThreads (a single thread copies at about 25-30 GB/s).
static const size_t kCopyChunk = size_t(8) << 20;
static const int kCopyThreads = 4;

static void stage_copy(void *dst, const void *src, size_t bytes) {
    const int nt = (int)std::min<size_t>(kCopyThreads, std::max<size_t>(1, bytes / kCopyChunk));
    if (nt <= 1) {
        memcpy(dst, src, bytes);
        return;
    }
    const size_t part = (bytes / nt + 63) / 64 * 64;
    std::vector<std::thread> th;
    th.reserve(nt - 1);
    for (int k = 1; k < nt; ++k) {
        const size_t a = std::min(bytes, part * k), b = std::min(bytes, part * (k + 1));
        if (a < b)
            th.emplace_back([=] { memcpy((char *)dst + a, (const char *)src + a, b - a); });
    }
    memcpy(dst, src, std::min(bytes, part));
    for (auto &t : th) t.join();
}

// The caller's dense n x n W into that layout (padding columns set to 0),
// rows split over at most kCopyThreads threads as in stage_copy.
static void stage_rows(int16_t *dst, const int16_t *src, int32_t n) {
    const int32_t P = pad8(n);
    if (P == n) {
        stage_copy(dst, src, wbytes_of(n));
        return;
    }
    auto rows = [=](int32_t r0, int32_t r1) {
        for (int32_t r = r0; r < r1; ++r) {
            memcpy(dst + (size_t)r * P, src + (size_t)r * n, sizeof(int16_t) * n);
            memset(dst + (size_t)r * P + n, 0, sizeof(int16_t) * (P - n));
        }
    };
    const int nt = (int)std::min<size_t>(kCopyThreads, std::max<size_t>(1, wbytes_of(n) / kCopyChunk));
    const int32_t per = (n + nt - 1) / nt;
    std::vector<std::thread> th;
    th.reserve(nt - 1);
    for (int k = 1; k < nt; ++k) {
        const int32_t a = std::min(n, per * k), b = std::min(n, per * (k + 1));
        if (a < b) th.emplace_back(rows, a, b);
    }
    rows(0, std::min(n, per));
    for (auto &t : th) t.join();
}

static size_t footprint(int32_t n) {
    return align_up(wbytes_of(n), 256) + instance_bytes(n, 1, SK_W_I16) + 4096;
}

// Carves the request's device region at offset `off` (W first, then the
// instance state).
static void place(Server *S, Request *r, size_t off) {
    r->off = off;
    Bump bump{S->ctx->arena + off, r->len};
    int16_t *dW = bump.take<int16_t>((size_t)r->n * pad8(r->n));
    carve_instance(bump, dW, pad8(r->n), r->n, &r->prm, r->inst);
}

// Marks r finished (caller holds S->mu) and records it for sk_completed; the
// record keeps at most kMaxDoneIds entries (older tickets stay pollable).
static const size_t kMaxDoneIds = size_t(1) << 16;
static void mark_done(Server *S, Request *r) {
    r->phase = 3;
    S->done_ids.push_back(r->id);
    if (S->done_ids.size() > kMaxDoneIds) S->done_ids.pop_front();
}

static void drop_event(Request *r) {
    if (r->ev) (void)hipEventDestroy(r->ev);
    r->ev = nullptr;
}

static void solver_loop(Server *S) {
    for (;;) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> g(S->mu);
            S->cv_solve.wait(g, [&] { return S->stop || !S->solve_q.empty(); });
            if (S->solve_q.empty()) return;
            r = S->solve_q.front();
            S->solve_q.pop_front();
        }
        sk_csr csr{r->n, (int64_t)r->col.size(), r->rp.data(), r->col.data(), r->w.data()};
        r->perm.assign(r->n, -1);
        int64_t weight = 0;
        sk_status st = sk_solve_reduced(&csr, r->perm.data(), &weight);
        {
            std::lock_guard<std::mutex> g(S->mu);
            r->weight = weight;
            if (st != SK_OK) r->status = st;
            r->rep.stages_evaluated = 1;
            r->rep.threshold_used = r->prm.threshold;
            if (st == SK_OK) {
                // log gamma = ub - w(B) (eq. optratio); integer weights: < 1 proves optimality
                r->rep.log_gamma = r->rep.ub - (double)weight;
                r->rep.optimal_proved = r->rep.log_gamma < 1.0 - 1e-9 ? 1 : 0;
            } else {
                r->rep.log_gamma = NAN;
            }
            r->rep.seconds =
                std::chrono::duration<double>(std::chrono::steady_clock::now() - r->t_submit).count();
            r->rp.clear();
            r->rp.shrink_to_fit();
            r->col.clear();
            r->col.shrink_to_fit();
            r->w.clear();
            r->w.shrink_to_fit();
            mark_done(S, r);
        }
    }
}

// Rebuilds the batch tables for the active set (serving thread only).
static sk_status rebuild(Server *S) {
    sk_ctx *ctx = S->ctx;
    S->B.h_insts.clear();
    for (Request *r : S->active) S->B.h_insts.push_back(r->inst);
    Bump tb{ctx->arena, S->tables_len};
    // the first part of the tables region holds the init-unit table
    S->d_init_units = tb.take<RowUnit>(kLdsMaxN / kRowWaves * 64);
    S->d_fresh = tb.take<int>(kMaxBatch);
    sk_status st = finish_tables(ctx, tb, S->B);
    if (st != SK_OK) return st;
    return upload_batch(ctx, S->B);
}

// Retires the finished instances fin[] of the batch in two device phases:
// (1) FP64 checks and kept-entry counts of all of them, one copy + one sync;
// (2) CSR fills and copies to the host. Their device regions are released
// afterwards and the exact solves go to the host pool.
static sk_status retire_all(Server *S, const std::vector<int> &fin) {
    sk_ctx *ctx = S->ctx;
    Batch &B = S->B;
    const size_t m = fin.size();
    std::vector<size_t> rp_off(m, 0), rp_len(m, 0);
    std::vector<char> live(m, 0);
    hipError_t e = hipSuccess;
    sk_status st = SK_OK;
    for (size_t q = 0; q < m && st == SK_OK && e == hipSuccess; ++q) {
        const int k = fin[q];
        Request *r = S->active[k];
        const Ctl &c = ctx->h_ctl[k];
        memset(&r->rep, 0, sizeof r->rep);
        fill_report(c, &r->rep);
        if (c.err & (ERR_EMPTY_ROW | ERR_EMPTY_COL)) {
            r->status = SK_ENOSUPPORT;
            continue;
        }
        if (c.capped) r->status = SK_ENOCONV;
        rp_len[q] = sizeof(int64_t) * (r->n + 1);
        {
            std::lock_guard<std::mutex> g(S->mu);
            if (!S->ralloc.alloc(rp_len[q], rp_off[q])) {
                r->status = SK_ENOMEM;
                continue;
            }
        }
        live[q] = 1;
        st = enqueue_check(ctx, B, k);
        if (st != SK_OK) break;
        size_t first = 0;
        while (first < B.h_rows.size() && B.h_rows[first].inst != k) ++first;
        const int nunits = (r->n + kRowWaves - 1) / kRowWaves;
        const int grid = std::min(nunits, ctx->num_cus * 2);
        const double logt = std::log(r->prm.threshold);
        int64_t *d_rp = (int64_t *)(ctx->arena + rp_off[q]);
        e = launch_prune_count(B.d_insts, B.d_rows + first, nunits, grid, logt, B.d_counts,
                               gq_lds_bytes(r->n), B.h_insts[k].nt, 0, ctx->stream);
        if (e == hipSuccess) e = launch_scan(B.d_counts, d_rp, r->n, ctx->stream, B.d_nnz + k);
    }
    if (st == SK_OK && e == hipSuccess)
        e = hipMemcpyAsync(ctx->h_checkout, B.d_checkout, sizeof(double) * 4 * B.count,
                           hipMemcpyDeviceToHost, ctx->stream);
    if (st == SK_OK && e == hipSuccess)
        e = hipMemcpyAsync(ctx->h_nnz, B.d_nnz, sizeof(int64_t) * B.count, hipMemcpyDeviceToHost,
                           ctx->stream);
    if (st == SK_OK && e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    // phase 2: fills
    std::vector<size_t> cw_off(m, 0), cw_len(m, 0);
    for (size_t q = 0; q < m && st == SK_OK && e == hipSuccess; ++q) {
        if (!live[q]) continue;
        const int k = fin[q];
        Request *r = S->active[k];
        report_from_check(ctx->h_checkout + 4 * (size_t)k, ctx->h_ctl[k].p, &r->rep);
        const int64_t nnz = ctx->h_nnz[k];
        r->rep.nnz_kept = nnz;
        r->rp.resize(r->n + 1);
        int64_t *d_rp = (int64_t *)(ctx->arena + rp_off[q]);
        if (nnz > 0) {
            const size_t col_bytes = align_up(sizeof(int32_t) * (size_t)nnz, 256);
            cw_len[q] = col_bytes + sizeof(int16_t) * (size_t)nnz;
            bool ok;
            {
                std::lock_guard<std::mutex> g(S->mu);
                ok = S->ralloc.alloc(cw_len[q], cw_off[q]);
            }
            if (!ok) {
                cw_len[q] = 0;
                r->status = SK_ENOMEM;
                continue;
            }
            int32_t *d_col = (int32_t *)(ctx->arena + cw_off[q]);
            int16_t *d_w = (int16_t *)(ctx->arena + cw_off[q] + col_bytes);
            size_t first = 0;
            while (first < B.h_rows.size() && B.h_rows[first].inst != k) ++first;
            const int nunits = (r->n + kRowWaves - 1) / kRowWaves;
            const int grid = std::min(nunits, ctx->num_cus * 2);
            e = launch_prune_fill(B.d_insts, B.d_rows + first, nunits, grid,
                                  std::log(r->prm.threshold), d_rp, d_col, d_w,
                                  gq_lds_bytes(r->n), B.h_insts[k].nt, 0, ctx->stream);
            r->col.resize(nnz);
            r->w.resize(nnz);
            if (e == hipSuccess)
                e = hipMemcpyAsync(r->col.data(), d_col, sizeof(int32_t) * nnz,
                                   hipMemcpyDeviceToHost, ctx->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(r->w.data(), d_w, sizeof(int16_t) * nnz, hipMemcpyDeviceToHost,
                                   ctx->stream);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(r->rp.data(), d_rp, rp_len[q], hipMemcpyDeviceToHost, ctx->stream);
    }
    if (st == SK_OK && e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    {
        std::lock_guard<std::mutex> g(S->mu);
        for (size_t q = 0; q < m; ++q) {
            if (rp_len[q]) S->ralloc.release(rp_off[q], rp_len[q]);
            if (cw_len[q]) S->ralloc.release(cw_off[q], cw_len[q]);
        }
    }
    if (st != SK_OK) return st;
    if (e != hipSuccess) return fail(ctx, SK_EDEVICE, "retire: %s", hipGetErrorString(e));
    return SK_OK;
}

static void serve_loop(Server *S) {
    sk_ctx *ctx = S->ctx;
    (void)hipSetDevice(ctx->device);
    bool dirty = false;
    for (;;) {
        // to_copy: admitted in queue order, each either with its copy already
        // in flight (placed at submission) or to be copied from staging now
        std::vector<Request *> fresh, to_copy;
        {
            std::unique_lock<std::mutex> g(S->mu);
            if (S->stop) break;
            admit_fifo(S->queue, S->active.size() + S->loading.size(), (size_t)kMaxBatch, S->ralloc,
                       S->staged_waiting, fresh, to_copy,
                       [S](Request *r, size_t off) { place(S, r, off); });
        }
        hipError_t e = hipSuccess;
        for (Request *r : to_copy) {
            if (!r->copying) {
                if (e == hipSuccess)
                    e = hipMemcpyAsync((void *)r->inst.W, r->staging, wbytes_of(r->n),
                                       hipMemcpyHostToDevice, S->copy_stream);
                if (e == hipSuccess) e = hipEventCreateWithFlags(&r->ev, hipEventDisableTiming);
                if (e == hipSuccess) e = hipEventRecord(r->ev, S->copy_stream);
            }
            S->loading.push_back(r);
        }
        // take in the requests whose copy has completed, in admission order
        while (e == hipSuccess && !S->loading.empty()) {
            Request *r = S->loading.front();
            const hipError_t q = hipEventQuery(r->ev);
            if (q == hipErrorNotReady) break;
            e = q;
            drop_event(r);
            {
                std::lock_guard<std::mutex> g(S->mu);
                release_staging(S, r);
            }
            fresh.push_back(r);
            S->loading.pop_front();
        }
        if (e == hipSuccess && S->active.empty() && fresh.empty()) {
            if (!S->loading.empty()) {
                e = hipEventSynchronize(S->loading.front()->ev);
            } else {
                std::unique_lock<std::mutex> g(S->mu);
                if (S->queue.empty() && !S->stop) S->cv.wait_for(g, std::chrono::milliseconds(1));
            }
            if (e == hipSuccess) continue;
        }
        sk_status st = SK_OK;
        if (e == hipSuccess && !fresh.empty()) {
            const int base = (int)S->active.size();
            for (Request *r : fresh) S->active.push_back(r);
            st = rebuild(S);
            // cold start of the new instances only
            S->init_units.clear();
            std::vector<int> &idx = S->fresh_idx;
            idx.clear();
            for (size_t q = 0; q < fresh.size(); ++q) {
                const int k = base + (int)q;
                idx.push_back(k);
                for (int r0 = 0; r0 < fresh[q]->n; r0 += kRowWaves)
                    S->init_units.push_back(RowUnit{k, r0});
            }
            if (e == hipSuccess && st == SK_OK)
                e = hipMemcpyAsync(S->d_fresh, idx.data(), sizeof(int) * idx.size(),
                                   hipMemcpyHostToDevice, ctx->stream);
            if (e == hipSuccess && st == SK_OK)
                e = launch_reset_ctl(S->B.d_insts, S->d_fresh, (int)idx.size(), ctx->stream);
            size_t done = 0;
            while (e == hipSuccess && st == SK_OK && done < S->init_units.size()) {
                const size_t chunk = std::min<size_t>(S->init_units.size() - done,
                                                      (size_t)kLdsMaxN / kRowWaves * 64);
                e = hipMemcpyAsync(S->d_init_units, S->init_units.data() + done,
                                   sizeof(RowUnit) * chunk, hipMemcpyHostToDevice, ctx->stream);
                if (e == hipSuccess)
                    e = launch_init(S->B.d_insts, S->d_init_units, (int)chunk,
                                    (int)std::min<size_t>(chunk, (size_t)ctx->num_cus * 2), 1,
                                    ctx->stream);
                // the unit table is reused by the next chunk's copy, which the
                // stream orders after this launch; the host vector stays
                // untouched until the tick's read-back synchronises
                done += chunk;
            }
            dirty = false;
        } else if (dirty) {
            st = rebuild(S);
            dirty = false;
        }
        for (int it = 0; it < S->iters_per_tick && st == SK_OK && e == hipSuccess; ++it)
            st = iterate_i16(ctx, S->B);
        if (st == SK_OK && e == hipSuccess) st = read_ctl(ctx, S->B);
        if (st != SK_OK || e != hipSuccess) {
            std::lock_guard<std::mutex> g(S->mu);
            S->error = e != hipSuccess ? hipGetErrorString(e) : ctx->err;
            for (auto *list : {&S->active, &fresh}) {
                for (Request *r : *list) {
                    r->status = SK_EDEVICE;
                    mark_done(S, r);
                }
                list->clear();
            }
            for (Request *r : S->loading) {
                drop_event(r);
                r->status = SK_EDEVICE;
                mark_done(S, r);
            }
            S->loading.clear();
            break;
        }
        // retire finished instances
        std::vector<int> fin;
        std::vector<Request *> keep;
        for (int k = 0; k < (int)S->active.size(); ++k) {
            if (ctx->h_ctl[k].state == ST_RUNNING) keep.push_back(S->active[k]);
            else fin.push_back(k);
        }
        if (!fin.empty()) {
            st = retire_all(S, fin);
            std::lock_guard<std::mutex> g(S->mu);
            for (int k : fin) {
                Request *r = S->active[k];
                S->ralloc.release(r->off, r->len);
                if (st != SK_OK || r->status == SK_ENOSUPPORT || r->status == SK_ENOMEM) {
                    if (st != SK_OK) r->status = SK_EDEVICE;
                    mark_done(S, r);
                } else {
                    r->phase = 2;
                    S->solve_q.push_back(r);
                    S->cv_solve.notify_one();
                }
            }
            S->active.swap(keep);
            dirty = true;
        }
    }
}

static Server *ensure_server(sk_ctx *ctx) {
    if (ctx->server) return ctx->server;
    Server *S = new Server();
    S->ctx = ctx;
    S->tables_len = std::min(kTablesBytes, ctx->arena_bytes / 4);
    S->ralloc.init(align_up(S->tables_len, 256), ctx->arena_bytes);
    const char *env = getenv("SK_SERVE_ITERS_PER_TICK");
    if (env && atoi(env) > 0) S->iters_per_tick = atoi(env);
    if (hipHostMalloc((void **)&S->ring, kRingBytes, hipHostMallocDefault) == hipSuccess) {
        S->ring_bytes = kRingBytes;
        S->ring_alloc.init(0, kRingBytes);
    } else {
        S->ring = nullptr;
    }
    if (hipSetDevice(ctx->device) != hipSuccess ||
        hipStreamCreateWithFlags(&S->copy_stream, hipStreamNonBlocking) != hipSuccess) {
        if (S->ring) (void)hipHostFree(S->ring);
        delete S;
        return nullptr;
    }
    ctx->server = S;
    S->th = std::thread(serve_loop, S);
    for (int k = 0; k < 4; ++k) S->solvers.emplace_back(solver_loop, S);
    return S;
}

void serve_stop(sk_ctx *ctx) {
    Server *S = ctx->server;
    if (!S) return;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    S->cv_solve.notify_all();
    if (S->th.joinable()) S->th.join();
    for (auto &t : S->solvers)
        if (t.joinable()) t.join();
    for (Request *r : S->loading) drop_event(r);
    for (auto &kv : S->reqs) {
        release_staging(S, kv.second);
        drop_event(kv.second);
        delete kv.second;
    }
    if (S->copy_stream) (void)hipStreamSynchronize(S->copy_stream);
    if (S->copy_stream) (void)hipStreamDestroy(S->copy_stream);
    if (S->ring) (void)hipHostFree(S->ring);
    delete S;
    ctx->server = nullptr;
}

bool serving(const sk_ctx *ctx) { return ctx->server != nullptr; }

}  // namespace sk

using namespace sk;

extern "C" sk_status sk_submit(sk_ctx *ctx, const int16_t *W_host, int32_t n, const sk_params *params,
                               uint64_t *ticket) {
    if (!ctx) return SK_EINVAL;
    if (!W_host || !ticket) return fail(ctx, SK_EINVAL, "null argument");
    sk_status st = check_params(ctx, params);
    if (st != SK_OK) return st;
    if (params->storage != SK_W_I16) return fail(ctx, SK_EINVAL, "served path sweeps int16 W");
    if (n < 1 || n > kLdsMaxN) return fail(ctx, SK_EINVAL, "n = %d outside [1, %d]", n, kLdsMaxN);
    if (!(params->threshold > 0.0)) return fail(ctx, SK_EINVAL, "threshold must be > 0");
    std::lock_guard<std::mutex> call(ctx->mu);
    Server *S = ensure_server(ctx);
    if (!S) return fail(ctx, SK_EDEVICE, "could not start the serving thread");
    const size_t len = footprint(n);
    if (len + S->tables_len > ctx->arena_bytes)
        return fail(ctx, SK_ENOMEM, "n = %d can never fit in the arena", n);
    Request *r = new Request();
    r->n = n;
    r->prm = *params;
    r->len = len;
    r->t_submit = std::chrono::steady_clock::now();
    const size_t wbytes = wbytes_of(n);
    // W goes to the pinned ring when it has room (a parallel host copy; the
    // caller's buffer is free when this returns) and from there to the device
    // by an asynchronous copy started here if the device region is free too;
    // without ring room it is copied straight to a free device region
    // (waiting for the copy); with neither the call returns SK_EAGAIN (heap
    // staging only when the pinned ring could not be allocated); the
    // decision is plan_entry's (sk_sched.h)
    bool placed = false;
    {
        std::lock_guard<std::mutex> g(S->mu);
        if (!S->error.empty()) {
            delete r;
            return fail(ctx, SK_EDEVICE, "serving thread stopped: %s", S->error.c_str());
        }
        const EntryPlan ep = plan_entry(S->ring ? &S->ring_alloc : nullptr, S->ralloc, S->queue.size(),
                                        (size_t)kMaxBatch, S->staged_waiting, wbytes, len);
        if (ep.kind == Entry::Again) {
            delete r;
            return SK_EAGAIN;
        }
        if (ep.kind == Entry::RingAndDevice || ep.kind == Entry::RingOnly) {
            r->staging = (int16_t *)(S->ring + ep.ring_off);
            r->ring_off = ep.ring_off;
            r->in_ring = true;
        }
        if (ep.kind == Entry::RingAndDevice || ep.kind == Entry::DeviceOnly) {
            place(S, r, ep.dev_off);
            placed = true;
        }
    }
    auto undo = [&](const char *what, hipError_t e) {
        drop_event(r);
        {
            std::lock_guard<std::mutex> g(S->mu);
            if (placed) S->ralloc.release(r->off, r->len);
            release_staging(S, r);
        }
        delete r;
        return fail(ctx, SK_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    };
    if (r->in_ring) {
        stage_rows(r->staging, W_host, n);
        if (placed) {
            hipError_t e = hipSetDevice(ctx->device);
            if (e == hipSuccess)
                e = hipMemcpyAsync((void *)r->inst.W, r->staging, wbytes, hipMemcpyHostToDevice,
                                   S->copy_stream);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&r->ev, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventRecord(r->ev, S->copy_stream);
            if (e != hipSuccess) return undo("copy of W", e);
            r->copying = true;
        }
    } else if (placed) {
        hipError_t e = hipSetDevice(ctx->device);
        if (e == hipSuccess)
            e = hipMemcpy2DAsync((void *)r->inst.W, sizeof(int16_t) * pad8(n), W_host,
                                 sizeof(int16_t) * n, sizeof(int16_t) * n, n,
                                 hipMemcpyHostToDevice, S->copy_stream);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&r->ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(r->ev, S->copy_stream);
        if (e == hipSuccess) e = hipEventSynchronize(r->ev);
        if (e != hipSuccess) return undo("copy of W", e);
        drop_event(r);
        r->loaded = true;
    } else {
        // no ring at all (with a ring, neither ring room nor a free region was
        // refused above: heap staging would later need a pageable copy that
        // stalls the serving thread)
        r->staging = (int16_t *)malloc(wbytes);
        if (!r->staging) {
            delete r;
            return fail(ctx, SK_ENOMEM, "host staging allocation failed");
        }
        stage_rows(r->staging, W_host, n);
    }
    {
        std::lock_guard<std::mutex> g(S->mu);
        if (!r->loaded && !r->copying) ++S->staged_waiting;
        r->id = S->next_id++;
        S->queue.push_back(r);
        S->reqs[r->id] = r;
        *ticket = r->id;
    }
    S->cv.notify_one();
    return SK_OK;
}

extern "C" sk_status sk_poll(sk_ctx *ctx, uint64_t ticket, int32_t *perm, int64_t *weight,
                             sk_report *report) {
    if (!ctx) return SK_EINVAL;
    Server *S = ctx->server;
    if (!S) return fail(ctx, SK_EINVAL, "no request was submitted");
    Request *r = nullptr;
    {
        std::lock_guard<std::mutex> g(S->mu);
        auto it = S->reqs.find(ticket);
        if (it == S->reqs.end()) return SK_EINVAL;
        r = it->second;
        if (r->phase != 3) return SK_EAGAIN;
        S->reqs.erase(it);
    }
    if (perm && r->perm.size() == (size_t)r->n) memcpy(perm, r->perm.data(), sizeof(int32_t) * r->n);
    if (weight) *weight = r->weight;
    if (report) *report = r->rep;
    const sk_status st = r->status;
    delete r;
    return st;
}

extern "C" int32_t sk_completed(sk_ctx *ctx, uint64_t *tickets, int32_t max) {
    if (!ctx || max < 0 || (max > 0 && !tickets)) return -1;
    Server *S = ctx->server;
    if (!S) return 0;
    std::lock_guard<std::mutex> g(S->mu);
    int32_t k = 0;
    while (k < max && !S->done_ids.empty()) {
        const uint64_t id = S->done_ids.front();
        S->done_ids.pop_front();
        if (S->reqs.count(id)) tickets[k++] = id;  // not collected yet
    }
    return k;
}
