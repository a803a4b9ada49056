// Host-side runtime structures of libsk (not part of the ABI).
#pragma once

#include <cstdarg>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "sk_hostsolve.h"
#include "sk_internal.h"

namespace sk {

constexpr int kMaxBatch = 4096;

struct TilePlan {
    int tile_cols, ntiles, seg_rows, nseg;
};
TilePlan plan_tiles(int32_t n, int vec8);
size_t instance_bytes(int32_t n, int vec8, int storage, int fused = 0);
size_t shared_bytes(int32_t count, const int32_t *n);
size_t pad_copy_bytes(int32_t n);
// LDS of the kernels that stage (G_j, gam_j) per column (FP64 check,
// pruning); none above kLdsMaxN (the entries are read from I.colpack)
inline size_t gq_lds_bytes(int32_t n) { return n > kLdsMaxN ? 0 : 8 * (size_t)pad8(n); }

// A set of instances swept together, with its device tables.
struct Batch {
    int count = 0;
    int nmax = 0;
    std::vector<Inst> h_insts;
    std::vector<RowUnit> h_rows;
    std::vector<ColUnit> h_cols;
    std::vector<FinUnit> h_fins;
    Inst *d_insts = nullptr;
    RowUnit *d_rows = nullptr;
    std::vector<int32_t> h_row_bounds;  // row sweep: units of workgroup b are [b], [b + 1]
    int32_t *d_row_bounds = nullptr;
    ColUnit *d_cols = nullptr;
    FinUnit *d_fins = nullptr;
    double *d_rsum = nullptr, *d_rmax = nullptr, *d_csum = nullptr;
    double *d_cpart = nullptr;     // FP64 column partials [nseg][n] of the checked instance
    Ctl *d_ctl_all = nullptr;      // gathered control blocks (one copy per check)
    double *d_checkout = nullptr;  // [count][4] reduced FP64 checks
    int64_t *d_nnz = nullptr;      // [count] kept entries per instance
    int64_t *d_counts = nullptr;
    size_t row_lds = 0;
    size_t row_lds_k = 0;
    int row_grid = 1, col_grid = 1, row_grid_k = 1, fin_grid = 1;
};

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over a region of the caller's arena.
struct Bump {
    char *base;
    size_t cap, off = 0;
    template <class T>
    T *take(size_t count) {
        size_t o = align_up(off, 256);
        size_t need = sizeof(T) * count;
        if (o + need > cap) return nullptr;
        off = o + need;
        return reinterpret_cast<T *>(base + o);
    }
};
struct Server;

// Timed launch classes (the short finalise and end-of-iteration launches of
// an iteration are not timed). *_DETECT: a launch that only detected the end
// of a stage; *_IDLE: a launch after every instance finished.
enum KernelId {
    KID_INIT, KID_ROW, KID_COL, KID_CHECK_ROWS, KID_CHECK_COLS, KID_PRUNE_COUNT,
    KID_SCAN, KID_PRUNE_FILL, KID_ABSORB, KID_ROW_K, KID_COL_K, KID_FOLD_K,
    KID_ROW_DETECT, KID_COL_DETECT, KID_ROW_IDLE, KID_COL_IDLE,
    KID_ROW_K_DETECT, KID_COL_K_DETECT, KID_ROW_K_IDLE, KID_COL_K_IDLE,
    KID_FUSED, KID_FUSED_DETECT, KID_FUSED_IDLE,
    KID_NT_PRODUCT, KID_NT_STEP, KID_NT_PRODUCT_IDLE, KID_NT_STEP_IDLE,
    KID_PAD_COPY,
    KID_COUNT
};
extern const char *kKernelNames[KID_COUNT];

// HIP-event timing of launches on the context stream. Each event is a
// stamp; a timed launch is the interval between two stamps, and back-to-back
// launches share the stamp between them. A stamp is either a marker packet
// in the stream (stamp()) or an event that a launch records at its own end
// (kernel_stamp(), passed to launch_stamped): the latter adds no packet, so it
// costs the stream less and a launch timed from the previous launch's end
// stamp to its own is timed without any marker latency. Events are created
// without the system-scope fence (they time launches and order nothing).
struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> stamps;
    std::vector<std::pair<int, std::pair<int, int>>> pending;  // (kernel id, (stamp, stamp))
    std::vector<hipEvent_t> pool;
    int64_t launches[KID_COUNT] = {};
    double total_ms[KID_COUNT] = {};
    hipEvent_t take();
    int stamp(hipStream_t st);                // index of a new marker stamp, -1 when off
    // An event for a launch to record at its end (nullptr when off); its
    // stamp index goes to *idx (-1 when off).
    hipEvent_t kernel_stamp(int *idx);
    void add(int id, int from, int to);       // launch `id` ran between two stamps
    void begin(hipStream_t st, int id);
    void end(hipStream_t st);
    void drain();   // call after the stream is synchronised
    void reset();
    // Re-tags the pending launches of kernel `kid` recorded at or after
    // position `start`: occurrence t (0-based) gets tag(t) (or stays if -1).
    template <class F>
    void retag(size_t start, int kid, F tag) {
        int64_t t = 0;
        for (size_t q = start; q < pending.size(); ++q) {
            if (pending[q].first != kid) continue;
            const int nk = tag(t++);
            if (nk >= 0) pending[q].first = nk;
        }
    }
    ~Profiler();
    int cur_id = -1;
    int cur_start = -1;
    int iter_end_stamp = -1;  // end stamp of the last end-of-iteration launch
};

}  // namespace sk

struct sk_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    char *arena = nullptr;
    size_t arena_bytes = 0;
    int num_cus = 256;
    std::string err;
    std::mutex mu;                 // one blocking call at a time
    sk::Ctl *h_ctl = nullptr;      // pinned readback of control blocks
    double *h_checkout = nullptr;  // pinned readback of reduced checks [kMaxBatch][4]
    int64_t *h_nnz = nullptr;      // pinned readback of kept counts [kMaxBatch]
    char *h_csr = nullptr;         // pinned host copy of sk_solve's reduced matrix (grown on demand)
    size_t h_csr_bytes = 0;
    sk::Batch scratch_batch;
    int absorbs = 0;
    double k_res_rows = 0, k_res_cols = 0;
    sk::Profiler prof;
    sk::Server *server = nullptr;
};

namespace sk {

sk_status fail(sk_ctx *ctx, sk_status st, const char *fmt, ...);

// Returns SK_EDEVICE (with the HIP error text) from the enclosing function
// when `expr` fails.
#define HIPCHK(ctx, expr)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, SK_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

// Launch `call` between the profiler's begin/end events for kernel `id`.
#define PROF(ctx, id, call)                         \
    ([&]() {                                        \
        (ctx)->prof.begin((ctx)->stream, (id));     \
        hipError_t e__ = (call);                    \
        (ctx)->prof.end((ctx)->stream);             \
        return e__;                                 \
    }())
// real: the parameters of a real-valued entry point (prescale allowed; two
// sweeps, Sinkhorn, W read directly)
sk_status check_params(sk_ctx *ctx, const sk_params *p, bool real = false);
// n of one instance: [1, kMaxN]; above kLdsMaxN only the two-sweep Sinkhorn
// iteration on int16 W
sk_status check_size(sk_ctx *ctx, int32_t n, const sk_params *p);
sk_status check_range(sk_ctx *ctx, const sk_params *prm);  // p small enough for exact exponents
sk_status status_of(const Ctl &c);  // SK_OK, SK_ENOCONV (a stage capped) or SK_ENOSUPPORT
// Wr != nullptr: a real-valued instance (W unused; Wr read with pitch `pitch`).
bool carve_instance(Bump &bump, const int16_t *W, int64_t pitch, int32_t n, const sk_params *prm,
                    Inst &I, const float *Wr = nullptr);
sk_status finish_tables(sk_ctx *ctx, Bump &bump, Batch &B);
sk_status plan_batch(sk_ctx *ctx, Bump &bump, int count, const int16_t *const *W,
                     const int64_t *pitch, const int32_t *n, const sk_params *prm, Batch &B);
sk_status upload_batch(sk_ctx *ctx, Batch &B);
sk_status start_batch(sk_ctx *ctx, Batch &B, const sk_params *prm, void *const *pot_in);
sk_status read_ctl(sk_ctx *ctx, Batch &B);
// chained: the previous launch on the stream is the end-of-iteration launch
// of the previous call (timing then starts from that launch's end stamp).
sk_status iterate_i16(sk_ctx *ctx, Batch &B, bool chained = false);
// Iterates until no instance is running (done, error, or paused at a stage
// end); first_stage: the stage the instances start this call in (launch tags).
sk_status run_batch_i16(sk_ctx *ctx, Batch &B, const sk_params *prm, int first_stage = 0);
// Called at the end of every stage of the stored-K controller, after the
// scalings are folded into the potentials and before p moves on; setting
// `stop` ends the run there.
using StageHook = std::function<sk_status(bool &stop)>;
sk_status run_single_k(sk_ctx *ctx, Batch &B, const sk_params *prm,
                       const StageHook *hook = nullptr);
// Newton scaling stage by stage (one int16 instance); its vectors come from
// `bump` (the arena after the batch plan).
sk_status run_newton_i16(sk_ctx *ctx, Batch &B, const sk_params *prm, Bump &bump,
                         const StageHook *hook = nullptr);
// Arena bytes of the Newton vectors and state for size n.
inline size_t newton_bytes(int32_t n) {
    return 9 * align_up(sizeof(float) * 2 * (size_t)n, 256) +
           align_up(sizeof(double) * (kNtPhases + 1) * kNtMaxGroups * 4, 256) + 1024;
}
// Extra outputs of the FP64 row check: per row the number of entries with
// log x_ij >= logt (device int64[n]) and the first column of the largest x_ij
// (device int32[n]).
struct CheckCounts {
    double logt;
    int64_t *counts;
    int32_t *hint;
};
sk_status check_fp64(sk_ctx *ctx, Batch &B, int k, sk_report *rep);
// writes B.d_checkout[k] (and the counts when cc != nullptr)
sk_status enqueue_check(sk_ctx *ctx, Batch &B, int k, const CheckCounts *cc = nullptr);
// p: the stage's p (ctl.p * pscale); wref: the common shift of a real-valued
// instance's log-weights (0 for int16 W), added back to the certificate.
void report_from_check(const double *out4, double p, sk_report *rep, int n = 0, double wref = 0.0);
void fill_report(const Ctl &c, sk_report *rep);
sk_status copy_potentials_out(sk_ctx *ctx, Batch &B, int k, void *pot);
// Scales `count` instances with their working memory carved from
// [arena, arena + arena_bytes) (the context's arena, or the static scratch).
sk_status scale_impl(sk_ctx *ctx, int count, const int16_t *const *W, const int32_t *n,
                     const sk_params *prm, void *const *pot, sk_report *reports, char *arena,
                     size_t arena_bytes);
// Resolves the device address of the static scratch on `device` (the current
// device), once per device; sk_create calls it.
hipError_t static_scratch_init(int device);
void serve_stop(sk_ctx *ctx);
bool serving(const sk_ctx *ctx);
hipError_t set_k_attributes();

}  // namespace sk
