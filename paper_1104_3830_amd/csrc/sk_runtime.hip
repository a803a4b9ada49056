// Host runtime of libsk: contexts, arena planning, the stage controller that
// drives the sweep kernels, the FP64 recheck and certificate, pruning, and the
// C ABI entry points declared in include/sk.h.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "sk_internal.h"
#include "sk_runtime.h"

namespace sk {

// ---------------------------------------------------------------- planning

// Tuned segment heights (sk_set_tile_table); empty = built-in rule.
static std::vector<std::pair<int32_t, int32_t>> g_tile_table;

TilePlan plan_tiles(int32_t n, int vec8) {
    TilePlan t;
    t.tile_cols = vec8 ? kColTile8 : kColTile1;
    t.ntiles = (n + t.tile_cols - 1) / t.tile_cols;
    for (const auto &e : g_tile_table) {
        if (n <= e.first) {
            t.seg_rows = std::min(e.second, std::max(16, (n + 15) / 16 * 16));
            t.nseg = (n + t.seg_rows - 1) / t.seg_rows;
            return t;
        }
    }
    // Column-sweep segment height: aim for ~1024 work units per sweep, but
    // keep each unit at >= 128 rows so the fixed-slot partials stay a small
    // fraction of the matrix traffic.
    int64_t want = ((int64_t)n * t.ntiles + 1023) / 1024;
    int seg = (int)std::min<int64_t>(kMaxSegRows, std::max<int64_t>(128, (want + 15) / 16 * 16));
    seg = std::min(seg, std::max(16, (n + 15) / 16 * 16));
    t.seg_rows = seg;
    t.nseg = (n + seg - 1) / seg;
    return t;
}


size_t instance_bytes(int32_t n, int vec8, int storage, int fused) {
    TilePlan t = plan_tiles(n, vec8);
    size_t b = 0;
    b += align_up(sizeof(int32_t) * n, 256) * 3;  // F[2], G
    b += align_up(sizeof(float) * n, 256) * 3;    // phi[2], gam
    const size_t slots = fused ? std::max(t.nseg, kFusedSlots) : t.nseg;
    b += align_up(sizeof(float) * slots * n, 256);
    b += align_up(sizeof(uint32_t) * n, 256);
    b += align_up(sizeof(Ctl), 256);
    b += align_up(sizeof(float) * std::max((n + kRowWaves - 1) / kRowWaves, kFusedSlots), 256) * 2;
    b += align_up(sizeof(float) * n, 256);  // rres
    b += align_up(sizeof(uint32_t) * kRowResSlots * kRowResStride, 256);  // rowres
    if (n > kLdsMaxN) b += align_up(8 * (size_t)pad8(n), 256);  // colpack
    if (storage == SK_K_BF16 || storage == SK_K_F32) {
        const size_t es = storage == SK_K_BF16 ? 2 : 4;
        const size_t kp = (size_t)(n + 7) / 8 * 8;
        b += align_up(es * (size_t)n * kp, 256);
        b += align_up(sizeof(float) * n, 256) * 3;  // a[2], b
    }
    return b;
}

// The library's 8-wide copy of a W whose n is not a multiple of 8.
size_t pad_copy_bytes(int32_t n) {
    return (n % 8) ? align_up(sizeof(int16_t) * (size_t)n * (size_t)pad8(n), 256) : 0;
}

size_t shared_bytes(int32_t count, const int32_t *n) {
    int64_t rows = 0, cols = 0, nmax = 0, cpart = 0, fins = 0;
    for (int k = 0; k < count; ++k) {
        // an instance takes the 8-wide plan unless its W is misaligned
        // (then the 1-wide plan: no more slots, more column units)
        TilePlan t = plan_tiles(n[k], 1), t1 = plan_tiles(n[k], 0);
        cpart = std::max<int64_t>(cpart, (int64_t)t.nseg * n[k]);
        rows += (n[k] + kRowWaves - 1) / kRowWaves;
        cols += std::max<int64_t>((int64_t)t.ntiles * t.nseg, (int64_t)t1.ntiles * t1.nseg);
        fins += (n[k] + kFinCols - 1) / kFinCols;
        nmax = std::max<int64_t>(nmax, n[k]);
    }
    size_t b = 0;
    b += align_up(sizeof(Inst) * count, 256);
    b += align_up(sizeof(Ctl) * count, 256);
    b += align_up(sizeof(double) * 4 * count, 256) + align_up(sizeof(int64_t) * count, 256);
    b += align_up(sizeof(RowUnit) * rows, 256);
    b += align_up(sizeof(ColUnit) * cols, 256);
    b += align_up(sizeof(FinUnit) * fins, 256);
    b += align_up(sizeof(double) * nmax, 256) * 3;  // FP64 check: rsum, rmax, csum
    b += align_up(sizeof(double) * (size_t)cpart, 256);  // FP64 column partials
    b += align_up(sizeof(int64_t) * (nmax + 1), 256);  // prune row counts
    b += align_up(sizeof(int32_t) * (kMaxRowGrid + 1), 256);  // row-sweep workgroup bounds
    return b;
}



const char *kKernelNames[KID_COUNT] = {"init", "row_sweep", "col_sweep", "check_rows",
                                       "check_cols", "prune_count", "scan", "prune_fill",
                                       "absorb", "row_sweep_k", "col_sweep_k", "fold_k",
                                       "row_sweep:detect", "col_sweep:detect", "row_sweep:idle",
                                       "col_sweep:idle", "row_sweep_k:detect",
                                       "col_sweep_k:detect", "row_sweep_k:idle",
                                       "col_sweep_k:idle", "fused", "fused:detect", "fused:idle",
                                       "nt_product", "nt_step", "nt_product:idle",
                                       "nt_step:idle", "pad_copy"};

hipEvent_t Profiler::take() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}
hipEvent_t Profiler::kernel_stamp(int *idx) {
    *idx = -1;
    if (!on) return nullptr;
    hipEvent_t e = take();
    if (!e) return nullptr;
    stamps.push_back(e);
    *idx = (int)stamps.size() - 1;
    return e;
}
int Profiler::stamp(hipStream_t st) {
    if (!on) return -1;
    hipEvent_t e = take();
    if (!e) return -1;
    if (hipEventRecord(e, st) != hipSuccess) {
        pool.push_back(e);
        return -1;
    }
    stamps.push_back(e);
    return (int)stamps.size() - 1;
}
void Profiler::add(int id, int from, int to) {
    if (from >= 0 && to >= 0) pending.push_back({id, {from, to}});
}
void Profiler::begin(hipStream_t st, int id) {
    if (!on) return;
    cur_id = id;
    cur_start = stamp(st);
}
void Profiler::end(hipStream_t st) {
    if (!on || cur_start < 0) return;
    add(cur_id, cur_start, stamp(st));
    cur_start = -1;
}
void Profiler::drain() {
    for (auto &p : pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, stamps[p.second.first], stamps[p.second.second]) == hipSuccess) {
            launches[p.first] += 1;
            total_ms[p.first] += ms;
        }
    }
    for (hipEvent_t e : stamps) pool.push_back(e);
    stamps.clear();
    pending.clear();
    cur_start = -1;
    iter_end_stamp = -1;
}
void Profiler::reset() {
    drain();
    for (int k = 0; k < KID_COUNT; ++k) {
        launches[k] = 0;
        total_ms[k] = 0.0;
    }
}
Profiler::~Profiler() {
    for (auto e : stamps) (void)hipEventDestroy(e);
    for (auto e : pool) (void)hipEventDestroy(e);
}

}  // namespace sk

using namespace sk;

sk_status sk_set_tile_table(const int32_t *n_max, const int32_t *seg_rows, int32_t count) {
    if (count < 0 || (count > 0 && (!n_max || !seg_rows))) return SK_EINVAL;
    std::vector<std::pair<int32_t, int32_t>> t;
    for (int k = 0; k < count; ++k) {
        if (seg_rows[k] < 16 || seg_rows[k] > kMaxSegRows || seg_rows[k] % 16 != 0) return SK_EINVAL;
        if (k > 0 && n_max[k] <= n_max[k - 1]) return SK_EINVAL;
        t.push_back({n_max[k], seg_rows[k]});
    }
    g_tile_table = t;
    return SK_OK;
}

sk_status sk_profile_enable(sk_ctx *ctx, int enable) {
    if (!ctx) return SK_EINVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->prof.reset();
    ctx->prof.on = enable != 0;
    return SK_OK;
}

int32_t sk_profile_read(sk_ctx *ctx, sk_kernel_stat *out, int32_t max) {
    if (!ctx) return -1;
    std::lock_guard<std::mutex> g(ctx->mu);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->prof.drain();
    int32_t k = 0;
    for (int id = 0; id < KID_COUNT; ++id) {
        if (ctx->prof.launches[id] == 0) continue;
        if (out && k < max) {
            memset(&out[k], 0, sizeof out[k]);
            snprintf(out[k].name, sizeof out[k].name, "%s", kKernelNames[id]);
            out[k].launches = ctx->prof.launches[id];
            out[k].total_ms = ctx->prof.total_ms[id];
        }
        ++k;
    }
    return k;
}

// ---------------------------------------------------------------- context

static std::mutex g_attr_mu;
static bool g_attr_done = false;

size_t sk_potentials_bytes(int32_t n) { return n > 0 ? (size_t)16 * n : 0; }

size_t sk_arena_bytes(int32_t n, int32_t storage) {
    if (n <= 0 || n > kMaxN) return 0;
    return instance_bytes(n, 1, storage, 1) + pad_copy_bytes(n) + shared_bytes(1, &n) +
           newton_bytes(n) + 4096;
}

size_t sk_batch_arena_bytes(int32_t count, const int32_t *n, int32_t storage) {
    if (count <= 0 || !n) return 0;
    for (int k = 0; k < count; ++k)
        if (n[k] <= 0 || n[k] > (count == 1 ? kMaxN : kLdsMaxN)) return 0;
    size_t b = shared_bytes(count, n) + 4096;
    for (int k = 0; k < count; ++k) b += instance_bytes(n[k], 1, storage) + pad_copy_bytes(n[k]);
    return b;
}

sk_status sk_create(sk_ctx **out, int device, void *hip_stream, void *arena_dev_ptr,
                    size_t arena_bytes) {
    if (!out) return SK_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SK_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return SK_EDEVICE;
    // the static scratch of sk_scale_static: its address on this device
    if (static_scratch_init(device) != hipSuccess) return SK_EDEVICE;
    {
        std::lock_guard<std::mutex> g(g_attr_mu);
        if (!g_attr_done) {
            if (set_kernel_attributes() != hipSuccess) return SK_EDEVICE;
            if (set_k_attributes() != hipSuccess) return SK_EDEVICE;
            if (set_real_attributes() != hipSuccess) return SK_EDEVICE;
            g_attr_done = true;
        }
    }
    sk_ctx *c = new sk_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->arena = (char *)arena_dev_ptr;
    c->arena_bytes = arena_dev_ptr ? arena_bytes : 0;
    (void)hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, device);
    if (c->num_cus <= 0) c->num_cus = 256;
    if (hipHostMalloc((void **)&c->h_ctl, sizeof(Ctl) * kMaxBatch, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void **)&c->h_checkout, sizeof(double) * 4 * kMaxBatch,
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c->h_nnz, sizeof(int64_t) * kMaxBatch, hipHostMallocDefault) !=
            hipSuccess) {
        delete c;
        return SK_EDEVICE;
    }
    *out = c;
    return SK_OK;
}

sk_status sk_destroy(sk_ctx *ctx) {
    if (!ctx) return SK_EINVAL;
    serve_stop(ctx);
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->h_ctl) (void)hipHostFree(ctx->h_ctl);
    if (ctx->h_checkout) (void)hipHostFree(ctx->h_checkout);
    if (ctx->h_nnz) (void)hipHostFree(ctx->h_nnz);
    if (ctx->h_csr) (void)hipHostFree(ctx->h_csr);
    delete ctx;
    return SK_OK;
}

const char *sk_last_error(const sk_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

sk_status sk::fail(sk_ctx *ctx, sk_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
    return st;
}

sk_status sk::check_size(sk_ctx *ctx, int32_t n, const sk_params *p) {
    if (n < 1 || n > kMaxN) return fail(ctx, SK_EINVAL, "n = %d outside [1, %d]", n, kMaxN);
    if (n > kLdsMaxN && p && (p->storage != SK_W_I16 || p->fused || p->method != SK_SINKHORN))
        return fail(ctx, SK_EINVAL,
                    "n = %d above %d: only the two-sweep Sinkhorn iteration on int16 W (storage 0, not fused)",
                    n, kLdsMaxN);
    return SK_OK;
}

sk_status sk::check_params(sk_ctx *ctx, const sk_params *p, bool real) {
    if (!p) return fail(ctx, SK_EINVAL, "params is NULL");
    if (p->n_p < 1 || p->n_p > SK_MAX_LADDER)
        return fail(ctx, SK_EINVAL, "n_p must be in [1, %d]", SK_MAX_LADDER);
    for (int k = 0; k < p->n_p; ++k)
        if (p->p_ladder[k] < 1 || p->p_ladder[k] > 2048)
            return fail(ctx, SK_EINVAL, "p_ladder[%d] = %d outside [1, 2048]", k, p->p_ladder[k]);
    if (!(p->tol >= 0.0)) return fail(ctx, SK_EINVAL, "tol must be >= 0");
    if (p->max_iters_per_stage < 1) return fail(ctx, SK_EINVAL, "max_iters_per_stage must be >= 1");
    if (p->storage < SK_W_I16 || p->storage > SK_K_F32) return fail(ctx, SK_EINVAL, "bad storage");
    if (!(p->deform_a >= 0.0) || p->deform_a > 1e6)
        return fail(ctx, SK_EINVAL, "deform_a must be in [0, 1e6]");
    if (p->deform_a > 0.0 && p->storage != SK_W_I16)
        return fail(ctx, SK_EINVAL, "the deformed iteration sweeps int16 W");
    if (p->method != SK_SINKHORN && p->method != SK_NEWTON) return fail(ctx, SK_EINVAL, "bad method");
    if (p->method == SK_NEWTON && (p->storage != SK_W_I16 || p->fused || p->deform_a > 0.0))
        return fail(ctx, SK_EINVAL, "Newton scaling runs on int16 W, two-pass, undeformed");
    if (p->prescale != 0 && p->prescale != 1) return fail(ctx, SK_EINVAL, "prescale must be 0 or 1");
    if (!real && p->prescale)
        return fail(ctx, SK_EINVAL, "prescaling needs real-valued weights (sk_scale_real / sk_solve_real)");
    if (real && (p->storage != SK_W_I16 || p->fused || p->method != SK_SINKHORN))
        return fail(ctx, SK_EINVAL,
                    "real-valued weights run the two-sweep Sinkhorn iteration on W (storage 0, not fused)");
    return SK_OK;
}

// ---------------------------------------------------------------- batch plan

// Fills the descriptor of one instance and carves its buffers from `bump`.
bool sk::carve_instance(Bump &bump, const int16_t *W, int64_t pitch, int32_t nn,
                        const sk_params *prm, Inst &I, const float *Wr) {
    I = Inst{};
    I.W = W;
    I.pitch = pitch;
    I.n = nn;
    I.pscale = 1.0;
    // 8-wide loads read whole aligned 16-byte chunks up to column pad8(n):
    // inside each row when pitch >= pad8(n), and for the last row inside the
    // aligned chunk that holds its last entry
    I.vec8 = (pitch % 8 == 0) && (pitch >= pad8(nn)) && ((uintptr_t)W % 16 == 0);
    if (Wr) {
        // real-valued: 16-byte loads of 4 floats when every row is whole
        // 16-byte chunks
        I.W = nullptr;
        I.Wr = Wr;
        I.vec8 = (nn % 4 == 0) && (pitch % 4 == 0) && ((uintptr_t)Wr % 16 == 0);
    } else if (!I.vec8 && nn % 8 != 0) {
        // the library's padded copy (filled by k_pad_copy before the input scan)
        int16_t *cp = bump.take<int16_t>((size_t)nn * pad8(nn));
        if (!cp) return false;
        I.Wsrc = W;
        I.src_pitch = pitch;
        I.W = cp;
        I.pitch = pad8(nn);
        I.vec8 = 1;
    }
    TilePlan t = plan_tiles(nn, Wr ? 1 : I.vec8);
    if (Wr) {
        t.tile_cols = kRealTile;
        t.ntiles = (nn + kRealTile - 1) / kRealTile;
    }
    I.nseg = t.nseg;
    I.seg_rows = t.seg_rows;
    I.ntiles = t.ntiles;
    I.tile_cols = t.tile_cols;
    I.n_p = prm->n_p;
    for (int s = 0; s < prm->n_p; ++s) I.ladder[s] = prm->p_ladder[s];
    I.tol = (float)prm->tol;
    I.max_iters = prm->max_iters_per_stage;
    I.storage = prm->storage;
    I.fused = prm->fused ? 1 : 0;
    I.deform_a = prm->deform_a > 0.0 ? prm->deform_a : 0.0;
    I.fused_grid = std::min(kFusedSlots, std::max(1, nn / 2));
    for (int b = 0; b < 2; ++b) {
        I.F[b] = bump.take<int32_t>(nn);
        I.phi[b] = bump.take<float>(nn);
    }
    I.G = bump.take<int32_t>(nn);
    I.gam = bump.take<float>(nn);
    const size_t slots = I.fused ? std::max(t.nseg, kFusedSlots) : t.nseg;
    I.colpart = bump.take<float>(slots * nn);
    I.rescue = bump.take<uint32_t>(nn);
    I.ctl = bump.take<Ctl>(1);
    const int nrows_units = (nn + kRowWaves - 1) / kRowWaves;
    I.ncolslots = I.fused ? I.fused_grid : t.nseg;
    I.res_slots = bump.take<float>(std::max(nrows_units, kFusedSlots));
    I.drift_slots = bump.take<float>(std::max(nrows_units, kFusedSlots));
    I.rres = bump.take<float>(nn);
    I.rowres = bump.take<uint32_t>((size_t)kRowResSlots * kRowResStride);
    if (!I.res_slots || !I.drift_slots || !I.rres || !I.rowres) return false;
    if (nn > kLdsMaxN && !Wr) {
        I.colpack = bump.take<int2>((size_t)pad8(nn));
        if (!I.colpack) return false;
    }
    if (!I.F[0] || !I.F[1] || !I.phi[0] || !I.phi[1] || !I.G || !I.gam || !I.colpart ||
        !I.rescue || !I.ctl)
        return false;
    I.kpitch = (nn + 7) / 8 * 8;
    if (prm->storage != SK_W_I16) {
        const size_t es = prm->storage == SK_K_BF16 ? 2 : 4;
        I.K = bump.take<char>(es * (size_t)nn * I.kpitch);
        I.a[0] = bump.take<float>(nn);
        I.a[1] = bump.take<float>(nn);
        I.b = bump.take<float>(nn);
        if (!I.K || !I.a[0] || !I.a[1] || !I.b) return false;
    }
    return true;
}

// Work-unit tables, shared scratch and launch grids for the instances in B.h_insts.
sk_status sk::finish_tables(sk_ctx *ctx, Bump &bump, Batch &B) {
    B.count = (int)B.h_insts.size();
    // matrix loads take the non-temporal hint only when the batch's matrices
    // cannot stay in the last-level cache between passes
    size_t mbytes = 0;
    for (const Inst &I : B.h_insts) {
        const size_t es = (I.storage == SK_K_F32 || I.Wr) ? 4 : 2;
        mbytes += es * (size_t)I.n * (size_t)(I.storage == SK_W_I16 ? I.pitch : (I.n + 7) / 8 * 8);
    }
    for (Inst &I : B.h_insts) I.nt = mbytes > kNtBytes ? 1 : 0;
    B.h_rows.clear();
    B.h_cols.clear();
    B.h_fins.clear();
    B.nmax = 0;
    int64_t cpart = 0;
    for (int k = 0; k < B.count; ++k) {
        const Inst &I = B.h_insts[k];
        cpart = std::max<int64_t>(cpart, (int64_t)I.nseg * I.n);
        for (int r = 0; r < I.n; r += kRowWaves) B.h_rows.push_back(RowUnit{k, r});
        for (int s = 0; s < I.nseg; ++s)
            for (int tt = 0; tt < I.ntiles; ++tt) B.h_cols.push_back(ColUnit{k, tt, s, 0});
        for (int g = 0; g * kFinCols < I.n; ++g) B.h_fins.push_back(FinUnit{k, g});
        B.nmax = std::max(B.nmax, I.n);
    }
    B.d_insts = bump.take<Inst>(B.count);
    B.d_ctl_all = bump.take<Ctl>(B.count);
    B.d_checkout = bump.take<double>(4 * (size_t)B.count);
    B.d_nnz = bump.take<int64_t>(B.count);
    B.d_rows = bump.take<RowUnit>(B.h_rows.size());
    B.d_cols = bump.take<ColUnit>(B.h_cols.size());
    B.d_fins = bump.take<FinUnit>(B.h_fins.size());
    B.d_rsum = bump.take<double>(B.nmax);
    B.d_rmax = bump.take<double>(B.nmax);
    B.d_csum = bump.take<double>(B.nmax);
    B.d_counts = bump.take<int64_t>(B.nmax + 1);
    B.d_cpart = bump.take<double>(cpart);
    if (!B.d_insts || !B.d_rows || !B.d_cols || !B.d_fins || !B.d_rsum || !B.d_rmax || !B.d_csum ||
        !B.d_counts || !B.d_cpart || !B.d_ctl_all || !B.d_checkout || !B.d_nnz)
        return fail(ctx, SK_ENOMEM, "arena too small for the batch tables");
    // grids: row sweep stages pad8(n) columns of potentials (8 B each) in LDS
    // (above kLdsMaxN it reads them from the instance's packed buffer)
    const size_t lds = B.nmax > kLdsMaxN ? 0 : sizeof(float2) * (size_t)pad8(B.nmax);
    const int per_cu = lds <= 32768 ? 2 : 1;
    B.row_lds = lds;
    B.row_lds_k = sizeof(float) * (size_t)((B.nmax + 7) / 8 * 8);
    B.row_grid = (int)std::max<size_t>(
        1, std::min<size_t>({B.h_rows.size(), (size_t)ctx->num_cus * per_cu, (size_t)kMaxRowGrid}));
    // one workgroup per CU: with two (and four loads in flight per lane) the
    // BF16 row sweep at n = 16384 ran 99 us instead of 89 us, more
    // concurrent row streams than HBM serves well
    const int per_cu_k = 1;
    B.row_grid_k = (int)std::max<size_t>(1, std::min<size_t>(B.h_rows.size(), (size_t)ctx->num_cus * per_cu_k));
    for (Inst &I : B.h_insts) I.kres_slots = B.row_grid_k;
    // Row-sweep ranges: contiguous runs of row units of about equal cost, so
    // that a batch of mixed sizes does not wait on the workgroups that drew
    // the large instances (an even split by count ran the 512-instance batch
    // of n in [32, 1024] 24% slower). Costs in hundredths of a step: a unit
    // (one row per wave) takes one step per 512 columns of its rows (one
    // 16-byte load per lane covers 512); of five cost models timed on that
    // batch this was the best (charging the staging of an instance's column
    // data, or a constant per unit, did not help).
    // Integer costs: equal units split exactly evenly.
    constexpr int64_t kCostCols = 512;
    {
        const size_t nu = B.h_rows.size();
        const int g = B.row_grid;
        std::vector<int64_t> cost(nu);
        int64_t total = 0;
        for (size_t q = 0; q < nu; ++q) {
            const int64_t nn = B.h_insts[B.h_rows[q].inst].n;
            const int64_t c = 100 * ((nn + kCostCols - 1) / kCostCols);
            cost[q] = c;
            total += c;
        }
        B.h_row_bounds.assign((size_t)g + 1, (int32_t)nu);
        B.h_row_bounds[0] = 0;
        int b = 0;
        int64_t acc = 0;
        for (size_t q = 0; q < nu && b + 1 < g; ++q) {
            acc += cost[q];
            while (b + 1 < g && acc * g >= total * (b + 1)) B.h_row_bounds[++b] = (int32_t)(q + 1);
        }
        B.d_row_bounds = bump.take<int32_t>((size_t)g + 1);
        if (!B.d_row_bounds) return fail(ctx, SK_ENOMEM, "arena too small for the batch tables");
    }
    B.col_grid = (int)std::max<size_t>(1, std::min<size_t>(B.h_cols.size(), (size_t)ctx->num_cus * 8));
    B.fin_grid = (int)std::max<size_t>(1, std::min<size_t>(B.h_fins.size(), (size_t)ctx->num_cus * 4));
    return SK_OK;
}

sk_status sk::plan_batch(sk_ctx *ctx, Bump &bump, int count, const int16_t *const *W,
                         const int64_t *pitch, const int32_t *n, const sk_params *prm,
                         Batch &B) {
    B.h_insts.assign(count, Inst{});
    for (int k = 0; k < count; ++k)
        if (!carve_instance(bump, W[k], pitch[k], n[k], prm, B.h_insts[k]))
            return fail(ctx, SK_ENOMEM, "arena too small for instance %d (n=%d)", k, n[k]);
    return finish_tables(ctx, bump, B);
}

sk_status sk::upload_batch(sk_ctx *ctx, Batch &B) {
    HIPCHK(ctx, hipMemcpyAsync(B.d_insts, B.h_insts.data(), sizeof(Inst) * B.count,
                               hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(B.d_rows, B.h_rows.data(), sizeof(RowUnit) * B.h_rows.size(),
                               hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(B.d_row_bounds, B.h_row_bounds.data(),
                               sizeof(int32_t) * B.h_row_bounds.size(), hipMemcpyHostToDevice,
                               ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(B.d_cols, B.h_cols.data(), sizeof(ColUnit) * B.h_cols.size(),
                               hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(B.d_fins, B.h_fins.data(), sizeof(FinUnit) * B.h_fins.size(),
                               hipMemcpyHostToDevice, ctx->stream));
    bool pads = false;
    for (const Inst &I : B.h_insts) pads |= I.Wsrc != nullptr;
    if (pads)
        HIPCHK(ctx, PROF(ctx, KID_PAD_COPY, launch_pad_copy(B.d_insts, B.d_rows, (int)B.h_rows.size(),
                                                            B.row_grid, ctx->stream)));
    return SK_OK;
}

// Initial control blocks and the input scan (cold start or warm start).
sk_status sk::start_batch(sk_ctx *ctx, Batch &B, const sk_params *prm, void *const *pot_in) {
    HIPCHK(ctx, launch_reset_ctl(B.d_insts, nullptr, B.count, ctx->stream));
    if (prm->warm_start) {
        for (int k = 0; k < B.count; ++k) {
            const int nn = B.h_insts[k].n;
            const char *src = (const char *)pot_in[k];
            HIPCHK(ctx, hipMemcpyAsync(B.h_insts[k].F[0], src, 4 * (size_t)nn,
                                       hipMemcpyDeviceToDevice, ctx->stream));
            HIPCHK(ctx, hipMemcpyAsync(B.h_insts[k].phi[0], src + 4 * (size_t)nn, 4 * (size_t)nn,
                                       hipMemcpyDeviceToDevice, ctx->stream));
            HIPCHK(ctx, hipMemcpyAsync(B.h_insts[k].G, src + 8 * (size_t)nn, 4 * (size_t)nn,
                                       hipMemcpyDeviceToDevice, ctx->stream));
            HIPCHK(ctx, hipMemcpyAsync(B.h_insts[k].gam, src + 12 * (size_t)nn, 4 * (size_t)nn,
                                       hipMemcpyDeviceToDevice, ctx->stream));
        }
    }
    if (B.h_insts[0].Wr)
        HIPCHK(ctx, PROF(ctx, KID_INIT, launch_init_real(B.d_insts, B.d_rows, (int)B.h_rows.size(),
                                                         B.row_grid, prm->warm_start ? 0 : 1, ctx->stream)));
    else
        HIPCHK(ctx, PROF(ctx, KID_INIT, launch_init(B.d_insts, B.d_rows, (int)B.h_rows.size(), B.row_grid,
                                                    prm->warm_start ? 0 : 1, ctx->stream)));
    return SK_OK;
}

sk_status sk::read_ctl(sk_ctx *ctx, Batch &B) {
    if (B.count == 1) {
        HIPCHK(ctx, hipMemcpyAsync(&ctx->h_ctl[0], B.h_insts[0].ctl, sizeof(Ctl),
                                   hipMemcpyDeviceToHost, ctx->stream));
    } else {
        HIPCHK(ctx, launch_gather_ctl(B.d_insts, B.count, B.d_ctl_all, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(ctx->h_ctl, B.d_ctl_all, sizeof(Ctl) * B.count,
                                   hipMemcpyDeviceToHost, ctx->stream));
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return SK_OK;
}

// One Sinkhorn iteration over every running instance of the batch.
sk_status sk::iterate_i16(sk_ctx *ctx, Batch &B, bool chained) {
    Profiler &pf = ctx->prof;
    if (B.count == 1 && B.h_insts[0].fused) {
        const Inst &I = B.h_insts[0];
        HIPCHK(ctx, PROF(ctx, KID_FUSED, launch_fused(B.d_insts, 0, I.n, I.fused_grid, SK_W_I16,
                                                      I.nt, ctx->stream)));
        HIPCHK(ctx, launch_col_finalize(B.d_insts, B.d_fins, (int)B.h_fins.size(), B.fin_grid,
                                        kFinOnePass, ctx->stream));
        HIPCHK(ctx, launch_iter_end(B.d_insts, B.count, ctx->stream));
        pf.iter_end_stamp = -1;
        return SK_OK;
    }
    // timed: the two sweeps. Each sweep and the end-of-iteration launch
    // record their own end stamps; the row sweep is timed from the previous
    // iteration's end stamp when this call follows it directly, else from a
    // marker. The short finalise launch between is not stamped.
    const Inst &I0 = B.h_insts[0];
    // n > kLdsMaxN (one instance): the row sweep reads the column entries
    // packed here (timed with it)
    const int gcol = B.count == 1 && I0.colpack != nullptr;
    const int s0 = chained && !gcol && pf.iter_end_stamp >= 0 ? pf.iter_end_stamp : pf.stamp(ctx->stream);
    if (gcol) HIPCHK(ctx, launch_col_pack(B.d_insts, 0, I0.n, 0, ctx->stream));
    const int nt = B.count > 0 ? B.h_insts[0].nt : 0;  // the same for the whole batch
    int s1, s2, s3;
    hipEvent_t e1 = pf.kernel_stamp(&s1);
    if (I0.Wr)
        HIPCHK(ctx, launch_row_sweep_real(B.d_insts, B.d_rows, (int)B.h_rows.size(), B.row_grid,
                                          B.row_lds, nt, I0.vec8, ctx->stream, e1));
    else
        HIPCHK(ctx, launch_row_sweep(B.d_insts, B.d_rows, (int)B.h_rows.size(), B.d_row_bounds,
                                     B.row_grid, B.row_lds, nt, B.nmax <= kShortRowN, gcol, ctx->stream, e1));
    hipEvent_t e2 = pf.kernel_stamp(&s2);
    if (I0.Wr)
        HIPCHK(ctx, launch_col_sweep_real(B.d_insts, B.d_cols, (int)B.h_cols.size(), B.col_grid, nt,
                                          I0.vec8, ctx->stream, e2));
    else
        HIPCHK(ctx, launch_col_sweep(B.d_insts, B.d_cols, (int)B.h_cols.size(), B.col_grid, nt,
                                     B.nmax <= kShortRowN, ctx->stream, e2));
    pf.add(KID_ROW, s0, s1);
    pf.add(KID_COL, s1, s2);
    HIPCHK(ctx, launch_col_finalize(B.d_insts, B.d_fins, (int)B.h_fins.size(), B.fin_grid, 0,
                                    ctx->stream));
    hipEvent_t e3 = pf.kernel_stamp(&s3);
    HIPCHK(ctx, launch_iter_end(B.d_insts, B.count, ctx->stream, e3));
    pf.iter_end_stamp = s3;
    return SK_OK;
}

// Runs the ladder of every instance to completion (device-side stopping).
// With timing on, launches are tagged afterwards: a triple (row, column,
// end) either did an iteration, or only detected that a stage had converged
// (its column sweep does no sums), or came after every instance finished.
sk_status sk::run_batch_i16(sk_ctx *ctx, Batch &B, const sk_params *prm, int first_stage) {
    const int check = std::max(1, prm->check_every);
    const int64_t bound = (prm->max_iters_per_stage + 1) * prm->n_p + 1;
    const size_t pstart = ctx->prof.pending.size();
    int64_t launched = 0;
    // Launch blocks are check_every iterations long until the end is near:
    // once every running instance is in its last stage (or, for an instance
    // paused at each stage end, after the first block of the stage) they are
    // at most kTailBlock long, so fewer launches run after the end. The first
    // block of a paused stage is sized by the previous stage's iterations.
    constexpr int kTailBlock = 8;
    int blk = check;
    if (B.count == 1 && B.h_insts[0].pause && first_stage > 0)
        blk = (int)std::min<int64_t>(check, std::max<int64_t>(
                                                4, ctx->h_ctl[0].stage_iters[first_stage - 1] + 2));
    for (;;) {
        for (int k = 0; k < blk; ++k) {
            sk_status s = iterate_i16(ctx, B, k > 0);
            if (s != SK_OK) return s;
        }
        launched += blk;
        sk_status s = read_ctl(ctx, B);
        if (s != SK_OK) return s;
        bool running = false, tail = true;
        for (int k = 0; k < B.count; ++k) {
            const Ctl &c = ctx->h_ctl[k];
            if (c.state != ST_RUNNING) continue;
            running = true;
            const Inst &I = B.h_insts[k];
            // (the deformed iteration is one long stage: full blocks)
            const bool last = I.deform_a <= 0.0 && c.stage + 1 >= I.n_p;
            tail &= last || I.pause;
        }
        if (!running) break;
        if (launched > bound) return fail(ctx, SK_EDEVICE, "stage controller did not terminate");
        blk = tail ? std::min(check, kTailBlock) : check;
    }
    if (ctx->prof.on) {
        // triple index of each convergence detection, and the number of
        // triples that advanced some instance
        std::vector<int64_t> detect;
        int64_t working = 0;
        for (int k = 0; k < B.count; ++k) {
            const Ctl &c = ctx->h_ctl[k];
            int64_t t = 0;
            for (int s = first_stage; s <= std::min(c.stage, prm->n_p - 1); ++s) {
                t += c.stage_iters[s];
                const bool conv = c.stage_iters[s] < prm->max_iters_per_stage &&
                                  (s < c.stage || c.state == ST_DONE || c.state == ST_STAGE_END);
                if (conv) {
                    if (B.count == 1) detect.push_back(t);
                    t += 1;
                }
            }
            working = std::max(working, t);
        }
        if (B.count > 1) detect.clear();
        auto tagger = [&](int det, int idle) {
            return [&, det, idle](int64_t t) {
                if (t >= working) return idle;
                for (int64_t d : detect)
                    if (d == t) return det;
                return -1;
            };
        };
        ctx->prof.retag(pstart, KID_ROW, tagger(KID_ROW_DETECT, KID_ROW_IDLE));
        ctx->prof.retag(pstart, KID_COL, tagger(KID_COL_DETECT, KID_COL_IDLE));
        ctx->prof.retag(pstart, KID_FUSED, tagger(KID_FUSED_DETECT, KID_FUSED_IDLE));
    }
    return SK_OK;
}

// FP64 recheck of instance k (enqueued): row and column sums of the balanced
// matrix and the certificate terms, reduced on the device into B.d_checkout[k].
sk_status sk::enqueue_check(sk_ctx *ctx, Batch &B, int k, const CheckCounts *cc) {
    const Inst &I = B.h_insts[k];
    const int nn = I.n;
    size_t first = 0;
    while (first < B.h_rows.size() && B.h_rows[first].inst != k) ++first;
    const int nunits = (nn + kRowWaves - 1) / kRowWaves;
    const int grid = std::min(nunits, ctx->num_cus * 2);
    if (I.Wr) {
        HIPCHK(ctx, PROF(ctx, KID_CHECK_ROWS,
                         launch_check_real(B.d_insts, B.d_rows + first, nunits, grid, k, nn, I.nseg,
                                           B.d_rsum, B.d_rmax, cc ? cc->logt : 0.0,
                                           cc ? cc->counts : nullptr, cc ? cc->hint : nullptr,
                                           B.d_cpart, B.d_csum, ctx->stream)));
        HIPCHK(ctx, launch_check_reduce(B.d_insts, k, B.d_rsum, B.d_rmax, B.d_csum,
                                        B.d_checkout + 4 * (size_t)k, ctx->stream));
        return SK_OK;
    }
    // n > kLdsMaxN: the row pass reads (G_j, gam_j) packed in I.colpack
    const int gcol = I.colpack != nullptr;
    if (gcol) HIPCHK(ctx, launch_col_pack(B.d_insts, k, nn, 1, ctx->stream));
    HIPCHK(ctx, PROF(ctx, KID_CHECK_ROWS,
                     launch_check_rows(B.d_insts, B.d_rows + first, nunits, grid, B.d_rsum,
                                       B.d_rmax, cc ? cc->logt : 0.0, cc ? cc->counts : nullptr,
                                       cc ? cc->hint : nullptr, gq_lds_bytes(nn), I.nt, gcol,
                                       ctx->stream)));
    HIPCHK(ctx, PROF(ctx, KID_CHECK_COLS, launch_check_cols(B.d_insts, k, nn, I.nseg, I.vec8,
                                                            B.d_cpart, B.d_csum, I.nt, ctx->stream)));
    HIPCHK(ctx, launch_check_reduce(B.d_insts, k, B.d_rsum, B.d_rmax, B.d_csum,
                                    B.d_checkout + 4 * (size_t)k, ctx->stream));
    return SK_OK;
}

// Proposition prop:aoc with log d_r = log u, log d_c = log v: log u cancels,
// UB = p^-1 (sum_i max_j (p w_ij + log v_j) - sum_j log v_j).
void sk::report_from_check(const double *o, double p, sk_report *rep, int n, double wref) {
    rep->residual_fp64 = o[0];
    rep->col_residual_fp64 = o[1];
    rep->residual_exact_fp64 = o[0];
    rep->col_residual_exact_fp64 = o[1];
    rep->ub = (o[2] - o[3]) / p + (double)n * wref;
}

sk_status sk::check_fp64(sk_ctx *ctx, Batch &B, int k, sk_report *rep) {
    sk_status st = enqueue_check(ctx, B, k);
    if (st != SK_OK) return st;
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_checkout + 4 * (size_t)k, B.d_checkout + 4 * (size_t)k,
                               4 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    report_from_check(ctx->h_checkout + 4 * (size_t)k, ctx->h_ctl[k].p, rep);
    return SK_OK;
}

void sk::fill_report(const Ctl &c, sk_report *rep) {
    rep->residual_fp32 = c.last_res;
    rep->iters_total = c.iters_total;
    for (int s = 0; s < SK_MAX_LADDER; ++s) rep->iters_stage[s] = c.stage_iters[s];
    rep->p_final = c.p;
    rep->stages_capped = c.capped;
}

sk_status sk::copy_potentials_out(sk_ctx *ctx, Batch &B, int k, void *pot) {
    const Inst &I = B.h_insts[k];
    const int nn = I.n;
    const int par = ctx->h_ctl[k].iter & 1;
    char *dst = (char *)pot;
    HIPCHK(ctx, hipMemcpyAsync(dst, I.F[par], 4 * (size_t)nn, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(dst + 4 * (size_t)nn, I.phi[par], 4 * (size_t)nn,
                               hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(dst + 8 * (size_t)nn, I.G, 4 * (size_t)nn, hipMemcpyDeviceToDevice,
                               ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(dst + 12 * (size_t)nn, I.gam, 4 * (size_t)nn,
                               hipMemcpyDeviceToDevice, ctx->stream));
    return SK_OK;
}

sk_status sk::status_of(const Ctl &c) {
    if (c.err & (ERR_EMPTY_ROW | ERR_EMPTY_COL)) return SK_ENOSUPPORT;
    if (c.err & ERR_NEWTON) return SK_EDEVICE;
    if (c.capped) return SK_ENOCONV;
    return SK_OK;
}

// The sweeps form the exponent 4 (p w_ij + F_i + G_j) in int32 (the byte
// offset of exp(E) in the LDS table), with p w from v_mul_i32_i24. Valid
// weights lie in [-16384, 16383]; p <= 2048 keeps |4 p w| <= 2^27, so with
// the potentials' integer parts (a few p times the weight range) and the
// padding columns' kPadExp4 = -2^30 every sum stays inside int32 and every
// exponent is exact.
sk_status sk::check_range(sk_ctx *ctx, const sk_params *prm) {
    int pmax = 0;
    for (int s = 0; s < prm->n_p; ++s) pmax = std::max(pmax, prm->p_ladder[s]);
    if ((int64_t)pmax * 16384 > ((int64_t)1 << 25))
        return fail(ctx, SK_EINVAL, "p = %d: p * 16384 exceeds 2^25 (exact int32 exponents)", pmax);
    return SK_OK;
}

sk_status sk::scale_impl(sk_ctx *ctx, int count, const int16_t *const *W, const int32_t *n,
                         const sk_params *prm, void *const *pot, sk_report *reports, char *arena,
                         size_t arena_bytes) {
    auto t0 = std::chrono::steady_clock::now();
    if (serving(ctx)) return fail(ctx, SK_EINVAL, "context is serving; blocking calls are disabled");
    ctx->absorbs = 0;
    sk_status st = check_params(ctx, prm);
    if (st != SK_OK) return st;
    if (count < 1 || count > kMaxBatch) return fail(ctx, SK_EINVAL, "count must be in [1, %d]", kMaxBatch);
    std::vector<int64_t> pitch(count);
    for (int k = 0; k < count; ++k) {
        if (!W[k] || !pot[k]) return fail(ctx, SK_EINVAL, "null W or potentials for instance %d", k);
        if (count == 1) {
            if ((st = check_size(ctx, n[0], prm)) != SK_OK) return st;
        } else if (n[k] < 1 || n[k] > kLdsMaxN) {
            return fail(ctx, SK_EINVAL, "n[%d] = %d outside [1, %d] (a batch; one larger instance goes to sk_scale)",
                        k, n[k], kLdsMaxN);
        }
        pitch[k] = n[k];
    }
    if (prm->storage != SK_W_I16 && count != 1)
        return fail(ctx, SK_EINVAL, "stored-K storages are single-instance");
    if (prm->fused && count != 1)
        return fail(ctx, SK_EINVAL, "the single-pass iteration is single-instance");
    if (prm->fused && prm->storage == SK_W_I16 && (n[0] % 8 != 0 || (uintptr_t)W[0] % 16 != 0))
        return fail(ctx, SK_EINVAL, "the single-pass iteration over int16 W needs n %% 8 == 0");
    if ((st = check_range(ctx, prm)) != SK_OK) return st;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    Bump bump{arena, arena_bytes};
    Batch &B = ctx->scratch_batch;
    if ((st = plan_batch(ctx, bump, count, W, pitch.data(), n, prm, B)) != SK_OK) return st;
    if ((st = upload_batch(ctx, B)) != SK_OK) return st;
    if ((st = start_batch(ctx, B, prm, pot)) != SK_OK) return st;
    if (prm->method == SK_NEWTON) {
        if (count != 1) return fail(ctx, SK_EINVAL, "Newton scaling is single-instance");
        if ((st = run_newton_i16(ctx, B, prm, bump)) != SK_OK) return st;
        if ((st = read_ctl(ctx, B)) != SK_OK) return st;
    } else if (prm->storage == SK_W_I16) {
        if ((st = run_batch_i16(ctx, B, prm)) != SK_OK) return st;
    } else {
        if ((st = run_single_k(ctx, B, prm)) != SK_OK) return st;
    }
    sk_status result = SK_OK;
    // FP64 checks of every instance, reduced on the device; one copy back
    bool any_check = false;
    for (int k = 0; k < count; ++k) {
        if (ctx->h_ctl[k].err & (ERR_EMPTY_ROW | ERR_EMPTY_COL)) continue;
        if ((st = enqueue_check(ctx, B, k)) != SK_OK) return st;
        any_check = true;
    }
    if (any_check) {
        HIPCHK(ctx, hipMemcpyAsync(ctx->h_checkout, B.d_checkout, sizeof(double) * 4 * count,
                                   hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    for (int k = 0; k < count; ++k) {
        const Ctl &c = ctx->h_ctl[k];
        sk_report rep;
        memset(&rep, 0, sizeof rep);
        fill_report(c, &rep);
        rep.absorbs = ctx->absorbs;
        if (!(c.err & (ERR_EMPTY_ROW | ERR_EMPTY_COL))) {
            report_from_check(ctx->h_checkout + 4 * (size_t)k, c.p, &rep);
            if (prm->storage != SK_W_I16) {
                rep.residual_fp64 = ctx->k_res_rows;
                rep.col_residual_fp64 = ctx->k_res_cols;
            }
        }
        if ((st = copy_potentials_out(ctx, B, k, pot[k])) != SK_OK) return st;
        rep.seconds = 0;
        if (reports) reports[k] = rep;
        sk_status sk = status_of(c);
        if (sk == SK_ENOSUPPORT || sk == SK_EDEVICE) result = sk;
        else if (sk == SK_ENOCONV && result == SK_OK) result = SK_ENOCONV;
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (reports)
        for (int k = 0; k < count; ++k) reports[k].seconds = secs;
    if (result == SK_ENOSUPPORT) fail(ctx, result, "a row or column of A has no entry");
    else if (result == SK_EDEVICE) fail(ctx, result, "Newton scaling broke down");
    else if (result == SK_ENOCONV) fail(ctx, result, "a stage hit max_iters_per_stage");
    return result;
}

sk_status sk_scale(sk_ctx *ctx, const int16_t *W, int32_t n, const sk_params *params,
                   void *potentials, sk_report *report) {
    if (!ctx) return SK_EINVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    const int16_t *Ws[1] = {W};
    void *pots[1] = {potentials};
    return scale_impl(ctx, 1, Ws, &n, params, pots, report, ctx->arena, ctx->arena_bytes);
}

sk_status sk_scale_batch(sk_ctx *ctx, int32_t count, const int16_t *const *W, const int32_t *n,
                         const sk_params *params, void *const *potentials, sk_report *reports) {
    if (!ctx) return SK_EINVAL;
    if (!W || !n || !potentials) return fail(ctx, SK_EINVAL, "null array argument");
    std::lock_guard<std::mutex> g(ctx->mu);
    return scale_impl(ctx, count, W, n, params, potentials, reports, ctx->arena, ctx->arena_bytes);
}

// ---------------------------------------------------------------- prune

sk_status sk_prune(sk_ctx *ctx, const int16_t *W, int32_t n, const void *potentials,
                   const sk_params *params, sk_csr *csr) {
    if (!ctx) return SK_EINVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    if (serving(ctx)) return fail(ctx, SK_EINVAL, "context is serving; blocking calls are disabled");
    sk_status st = check_params(ctx, params);
    if (st != SK_OK) return st;
    if (!W || !potentials || !csr || !csr->row_ptr)
        return fail(ctx, SK_EINVAL, "null argument");
    if (n < 1 || n > kMaxN) return fail(ctx, SK_EINVAL, "n = %d outside [1, %d]", n, kMaxN);
    if (!(params->threshold > 0.0)) return fail(ctx, SK_EINVAL, "threshold must be > 0");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    Bump bump{ctx->arena, ctx->arena_bytes};
    Batch &B = ctx->scratch_batch;
    const int16_t *Ws[1] = {W};
    int64_t pitch = n;
    sk_params p1 = *params;
    p1.storage = SK_W_I16;
    if ((st = plan_batch(ctx, bump, 1, Ws, &pitch, &n, &p1, B)) != SK_OK) return st;
    // point the descriptor at the caller's potentials
    Inst &I = B.h_insts[0];
    char *pot = (char *)potentials;
    I.F[0] = I.F[1] = (int32_t *)pot;
    I.phi[0] = I.phi[1] = (float *)(pot + 4 * (size_t)n);
    I.G = (int32_t *)(pot + 8 * (size_t)n);
    I.gam = (float *)(pot + 12 * (size_t)n);
    if ((st = upload_batch(ctx, B)) != SK_OK) return st;
    Ctl c;
    memset(&c, 0, sizeof c);
    c.state = ST_DONE;
    c.p = params->p_ladder[params->n_p - 1];
    ctx->h_ctl[0] = c;
    HIPCHK(ctx, hipMemcpyAsync(I.ctl, &ctx->h_ctl[0], sizeof(Ctl), hipMemcpyHostToDevice,
                               ctx->stream));
    const double logt = std::log(params->threshold);
    const int nunits = (int)B.h_rows.size();
    const int gcol = I.colpack != nullptr;  // n > kLdsMaxN: (G_j, gam_j) packed
    if (gcol) HIPCHK(ctx, launch_col_pack(B.d_insts, 0, n, 1, ctx->stream));
    HIPCHK(ctx, PROF(ctx, KID_PRUNE_COUNT, launch_prune_count(B.d_insts, B.d_rows, nunits, B.row_grid, logt, B.d_counts,
                                   gq_lds_bytes(n), B.h_insts[0].nt, gcol, ctx->stream)));
    HIPCHK(ctx, PROF(ctx, KID_SCAN, launch_scan(B.d_counts, csr->row_ptr, n, ctx->stream)));
    int64_t total = 0;
    HIPCHK(ctx, hipMemcpyAsync(&total, csr->row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    const int64_t cap = csr->nnz;
    csr->n = n;
    csr->nnz = total;
    if (total > cap) return fail(ctx, SK_ENOMEM, "reduced matrix has %lld entries, capacity %lld",
                                 (long long)total, (long long)cap);
    if (total > 0) {
        if (!csr->col || !csr->w) return fail(ctx, SK_EINVAL, "null col/w buffers");
        HIPCHK(ctx, PROF(ctx, KID_PRUNE_FILL, launch_prune_fill(B.d_insts, B.d_rows, nunits, B.row_grid, logt, csr->row_ptr,
                                      csr->col, csr->w, gq_lds_bytes(n), B.h_insts[0].nt, gcol, ctx->stream)));
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return SK_OK;
}
