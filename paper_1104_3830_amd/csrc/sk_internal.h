// Internal data structures shared by the HIP kernels and the host runtime.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sk.h"

namespace sk {

constexpr int kWave = 64;
constexpr int kRowWaves = 16;    // waves per workgroup in the row sweep (one row per wave)
constexpr int kColWaves = 4;     // waves per workgroup in the column sweep
constexpr int kColTile8 = 512;   // columns per column tile, 8-wide vector loads
constexpr int kColTile1 = 64;    // columns per column tile, scalar loads
// Up to kLdsMaxN the kernels that need every column's data stage it in LDS
// (8 bytes per column); above it (int16 W, two sweeps, one instance, up to
// kMaxN) they read it from a packed per-instance buffer in global memory,
// which stays in the L2 cache (512 KiB at kMaxN).
constexpr int kLdsMaxN = 16384;
constexpr int kMaxN = 65536;
constexpr int kMaxSegRows = 1024;
constexpr int kShortRowN = 2048;  // batches up to this n take the short-row row sweep
constexpr int kFusedSlots = 256;  // workgroups (and column-partial slots) of the fused kernel
constexpr int kMaxRowGrid = 1024;  // row-sweep workgroups (bounds table sized for it)
constexpr int kRealTile = 256;     // columns per column tile of the real-weight sweeps

// Column count of the 8-wide layout: n rounded up to a multiple of 8.
__host__ __device__ constexpr int pad8(int n) { return (n + 7) & ~7; }
// Padding columns j in [n, pad8(n)) of the 8-wide kernels take these column
// potentials. With |4 p w| <= 2^28 (p <= 2048, int16 w) and row terms
// |B| = |4 (F_i - kTabLo)| < 2^29 (the potentials stay within a few p times
// the weight range, below 2^26), 4 p w + kPadExp4 + B lies in (-2^31, 0), so
// the exp-table read clamps to its zero entry and the column adds exactly 0;
// kPadG puts the exact exponent (with w read as SK_SENTINEL there, p w >=
// -2^26) below -2^27, far below every skip bound of the FP64 check and the
// kept test, which therefore need no explicit mask for these columns.
constexpr int kPadExp4 = -(1 << 30);
constexpr int kPadG = -(1 << 28);

enum : int32_t { ST_RUNNING = 0, ST_DONE = 1, ST_ERROR = 2, ST_STAGE_END = 3 };
enum : uint32_t { ERR_EMPTY_ROW = 1u, ERR_EMPTY_COL = 2u, ERR_RANGE = 4u, ERR_NEWTON = 8u };

// Per-instance control block, device memory. Written by the kernels only at
// the places documented on each field; read by the host between launches.
struct Ctl {
    uint32_t res_bits;      // max_i |r_i - 1| of the current iterate (float bits), from the finalise
    uint32_t rescue_cnt;    // columns whose sum left the safe range in the last column sweep
    uint32_t err;           // ERR_* flags
    uint32_t sent;          // 1: W holds the sentinel (set by the input scan)
    int32_t state;          // ST_*
    int32_t stage;          // index into the p ladder
    int32_t p;              // current p
    int32_t iter;           // completed iterations in this stage; parity selects the F/phi buffer
    int32_t capped;         // stages that hit the cap
    int64_t iters_total;
    float last_res;         // residual of the last measured iterate
    uint32_t need_absorb;   // stored K: K must be recomputed before the next K sweep
    uint32_t drift_bits;    // stored K: max |log2 a_i|, |log2 b_j| since the last absorb (float bits)
    int64_t stage_iters[SK_MAX_LADDER];
    // deformed iteration on real-valued weights: p of the current iteration
    // unrounded (p is its rounding, used by the integer path)
    double preal;
};

// Per-instance descriptor (device memory, constant during a launch).
struct Inst {
    const int16_t *W;       // n x n log-weights, row pitch `pitch` elements
    int64_t pitch;
    int32_t n;
    // 1: rows 16-byte aligned with pitch >= pad8(n) -> 8-wide loads over
    // pad8(n) columns; columns n..pad8(n)-1 are padding (any values)
    int32_t vec8;
    int32_t nt;             // 1: sweeps launched with non-temporal matrix loads (batch > kNtBytes)
    int32_t nseg;           // row segments of the column sweep
    int32_t seg_rows;
    int32_t ntiles;         // column tiles of the column sweep
    int32_t tile_cols;
    int32_t n_p;
    int32_t ladder[SK_MAX_LADDER];
    float tol;
    int32_t pad1;
    int64_t max_iters;
    int32_t *F[2];          // row potential, integer part (ping-pong by iteration parity)
    float *phi[2];          // row potential, fraction
    int32_t *G;             // column potential, integer part
    float *gam;             // column potential, fraction
    float *colpart;         // [nseg][n] partial column sums
    uint32_t *rescue;       // [n] list of flagged columns
    Ctl *ctl;
    // stored-K storages
    void *K;                // n x kpitch bf16 or f32 (kpitch = n rounded up to 8; pad = 0)
    float *a[2];            // row scalings of K (ping-pong by iteration parity)
    float *b;               // column scalings of K
    int32_t storage;
    int32_t kpitch;
    int32_t fused;          // single-pass iteration (colpart holds kFusedSlots rows)
    double deform_a;        // > 0: deformed iteration, p_m = round(a ln(m + 1)) in [ladder[0], ladder[n_p - 1]]
    int32_t fused_grid;
    int32_t ncolslots;      // rows of colpart in use: nseg (sweeps) or fused_grid (single pass)
    int32_t pause;          // end every stage in ST_STAGE_END (the host advances p)
    // max |r_i - 1| of the current iterate, per row segment (log-domain
    // sweeps), per row unit (stored-K sweeps) or per workgroup (single pass)
    float *res_slots;
    float *drift_slots;     // stored K: per row unit max |log2 a_i|
    float *rres;            // [n] |r_i - 1| from the log-domain row sweep
    // max |r_i - 1| of the log-domain row sweep spread over kRowResSlots
    // words kRowResStride apart (float bits, atomicMax by each wave; zero
    // between iterations); the column sweep reduces them
    uint32_t *rowres;
    // residual / drift slots the stored-K row sweep writes (one per workgroup)
    int32_t kres_slots;
    int32_t pad3;
    // the caller's W when W is the library's padded copy (n % 8 != 0),
    // else nullptr; copied once per batch before the input scan
    const int16_t *Wsrc;
    int64_t src_pitch;
    // real-valued log-weights (sk_scale_real / sk_solve_real): n x n float32,
    // row pitch `pitch` elements, -inf for a_ij = 0; nullptr for int16 W.
    // The sweeps use w_ij - wref (wref = the largest finite weight; a common
    // shift of the log-weights leaves X(p) unchanged), so the potentials stay
    // within a few p times the weight range.
    const float *Wr;
    float wref;
    int32_t pad2;
    // p of the current stage is ctl->p * pscale: 1 for int16 W; with the
    // prescaling of Section 4.1.1, 1 / (w_max - w_min) when that exceeds 1
    double pscale;
    // n > kLdsMaxN: pad8(n) 8-byte column entries in the layout the LDS
    // staging would use, rewritten before each kernel that reads them (row
    // sweep: (4 G_j, exp(gam_j)); FP64 check and CSR passes: (G_j, gam_j));
    // nullptr otherwise
    void *colpack;
};
constexpr int kRowResSlots = 64;    // = kWave: one wave reduces them
constexpr int kRowResStride = 32;   // one 128-byte line per slot

// p of iteration m (from 1) of the deformed iteration: the schedule
// a log(m + 1) of Theorem logconvergencepositive kept in [first, last ladder
// entry]; unrounded for real-valued weights, rounded for int16 W (whose
// exact exponents need an integer p).
__device__ __forceinline__ double deform_p_real(const Inst &I, int64_t m) {
    const double lo = (double)I.ladder[0], hi = (double)I.ladder[I.n_p - 1];
    return fmin(hi, fmax(lo, I.deform_a * log((double)(m + 1))));
}
__device__ __forceinline__ int deform_p(const Inst &I, int64_t m) {
    const double v = rint(I.deform_a * log((double)(m + 1)));
    const double lo = (double)I.ladder[0], hi = (double)I.ladder[I.n_p - 1];
    return (int)fmin(hi, fmax(lo, v));
}

// Loads through a global-address-space pointer, so the compiler emits
// global_load (counted by vmcnt only) instead of flat_load (also counted by
// lgkmcnt, which would make every LDS wait drain the outstanding HBM loads).
typedef int sk_gi4 __attribute__((ext_vector_type(4)));
typedef float sk_gf4 __attribute__((ext_vector_type(4)));
#define SK_GLOBAL __attribute__((address_space(1)))
// Matrix loads (W or K). With NT they carry the non-temporal hint: when the
// batch's matrices exceed the last-level cache a pass reads each entry once,
// and keeping the stream out of the caches' normal replacement made the
// n = 16384 sweeps 4-6% faster; a batch that fits (re-read every iteration
// from the cache) is slower with it. NT is a template parameter of the sweep
// kernels (the hint is an instruction bit; a run-time choice between two
// otherwise identical loads is merged by the compiler), chosen at launch from
// Inst::nt.
template <bool NT>
__device__ __forceinline__ int4 gload(const int4 *p) {
    sk_gi4 v;
    if constexpr (NT) v = __builtin_nontemporal_load((const SK_GLOBAL sk_gi4 *)p);
    else v = *(const SK_GLOBAL sk_gi4 *)p;
    return make_int4(v.x, v.y, v.z, v.w);
}
template <bool NT>
__device__ __forceinline__ float4 gload(const float4 *p) {
    sk_gf4 v;
    if constexpr (NT) v = __builtin_nontemporal_load((const SK_GLOBAL sk_gf4 *)p);
    else v = *(const SK_GLOBAL sk_gf4 *)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
template <bool NT>
__device__ __forceinline__ int16_t gload(const int16_t *p) {
    if constexpr (NT) return __builtin_nontemporal_load((const SK_GLOBAL int16_t *)p);
    else return *(const SK_GLOBAL int16_t *)p;
}
// Matrix bytes of a batch above which its loads take the non-temporal hint
// (three quarters of MI355X's 256 MiB last-level cache).
constexpr size_t kNtBytes = size_t(192) << 20;

// Newton scaling (Knight-Ruiz) of one instance: state of the device-side
// outer/inner (conjugate gradient) iteration on the 2n-vectors of the
// symmetric embedding S = [[0, X], [X^T, 0]].
enum : int32_t { NT_OUTER = 0, NT_INNER = 1 };
enum : int32_t { NT_RUN = 0, NT_CONVERGED = 1, NT_CAPPED = 2, NT_FAILED = 3 };
struct NtCtl {
    int32_t mode;          // NT_OUTER: sd = S x;  NT_INNER: sd = S (x o d)
    int32_t done;          // NT_RUN / NT_CONVERGED / NT_CAPPED / NT_FAILED
    int32_t first;         // the next NT_OUTER is the initial one
    int32_t pad;
    int64_t products, outer, max_products;
    double rout, rold, rho, rho_prev, eta, inner_tol, resinf;
    double tol, lo, hi, eta_max, g;
};
struct NtVec {
    float *q, *sd, *x, *v, *r, *z, *d, *y, *w;  // [2n] each
    double *parts;  // [kNtPhases + 1][kNtMaxGroups][4] per-workgroup partial reductions
};
constexpr int kNtPhases = 4, kNtMaxGroups = 64, kNtThreads = 256;

struct RowUnit { int32_t inst, row0; };
struct ColUnit { int32_t inst, tile, seg, pad; };
struct FinUnit { int32_t inst, group; };  // 64 columns of one instance
constexpr int kFinCols = 64;

// Launches `kernel` on `st`. With a non-null `stop` the launch itself
// records the event at the kernel's end (the dispatch carries the timestamp),
// so no separate marker packet enters the stream.
template <class F, class... Args>
inline void launch_stamped(F kernel, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                           hipEvent_t stop, Args... args) {
    if (stop)
        hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, st, nullptr, stop, 0u, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, st, args...);
}

// Kernel launchers (sk_kernels.hip). All enqueue on `st`; `stop` (optional)
// is recorded at the end of the launch (launch_stamped).
hipError_t launch_init(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid, int cold,
                       hipStream_t st);
hipError_t launch_pad_copy(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid,
                           hipStream_t st);
// short_rows: every instance of the batch has n <= kShortRowN (the row
// sweep compiled for two workgroups per CU, sk_rowshort.hip)
// bounds (device, grid + 1 entries, or nullptr for an even split by count):
// workgroup b sweeps the units [bounds[b], bounds[b + 1]).
// gcol: one instance with n > kLdsMaxN (column entries from I.colpack,
// packed by launch_col_pack mode 0 before the launch)
hipError_t launch_row_sweep(const Inst *d_insts, const RowUnit *d_units, int nunits,
                            const int32_t *bounds, int grid, size_t lds_bytes, int nt_loads,
                            int short_rows, int gcol, hipStream_t st, hipEvent_t stop = nullptr);
// Packs instance inst's column entries into its colpack buffer (n > kLdsMaxN):
// mode 0 for the row sweep, 1 for the FP64 check and the CSR passes.
hipError_t launch_col_pack(const Inst *d_insts, int inst, int n, int mode, hipStream_t st);
hipError_t launch_row_sweep_short(const Inst *d_insts, const RowUnit *d_units, int nunits,
                                  const int32_t *bounds, int grid, size_t lds_bytes, int nt_loads,
                                  hipStream_t st, hipEvent_t stop = nullptr);
hipError_t set_row_sweep_short_attributes();
hipError_t launch_col_sweep(const Inst *d_insts, const ColUnit *d_units, int nunits, int grid,
                            int nt_loads, int short_rows, hipStream_t st, hipEvent_t stop = nullptr);
hipError_t launch_nt_product(const Inst *d_insts, const RowUnit *d_rows, int nrows, int row_grid,
                             size_t row_lds, const ColUnit *d_cols, int ncols, int col_grid,
                             const NtCtl *nt, NtVec vec, int n, int nt_loads, hipStream_t st);
// nt: two control blocks (double-buffered by phase parity; nt[1] is current).
hipError_t launch_nt_step(const Inst *d_insts, NtCtl *nt, NtVec vec, int n, hipStream_t st);
hipError_t launch_nt_fold(const Inst *d_insts, const NtCtl *nt, NtVec vec, int n, int last,
                          hipStream_t st);
hipError_t launch_iter_end(const Inst *d_insts, int count, hipStream_t st,
                           hipEvent_t stop = nullptr);
enum : int { kFinOnePass = 1, kFinStoredK = 2 };
hipError_t launch_col_finalize(const Inst *d_insts, const FinUnit *d_units, int nunits, int grid,
                               int mode, hipStream_t st);
hipError_t launch_check_rows(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid,
                             double *rsum, double *rmax, double logt, int64_t *counts,
                             int32_t *hint, size_t lds_bytes, int nt_loads, int gcol, hipStream_t st);
hipError_t launch_check_cols(const Inst *d_insts, int inst, int n, int nseg, int vec8,
                             double *part, double *csum, int nt_loads, hipStream_t st);
hipError_t launch_prune_count(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid,
                              double logt, int64_t *counts, size_t lds_bytes, int nt_loads, int gcol,
                              hipStream_t st);
hipError_t launch_scan(const int64_t *counts, int64_t *row_ptr, int n, hipStream_t st,
                       int64_t *total_out = nullptr);
hipError_t launch_check_reduce(const Inst *d_insts, int inst, const double *rsum,
                               const double *rmax, const double *csum, double *out, hipStream_t st);
hipError_t launch_prune_fill(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid,
                             double logt, const int64_t *row_ptr, int32_t *col, int16_t *w,
                             size_t lds_bytes, int nt_loads, int gcol, hipStream_t st);
hipError_t launch_absorb(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid,
                         size_t lds_bytes, int storage, int nt, hipStream_t st);
hipError_t launch_row_sweep_k(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid,
                              size_t lds_bytes, int storage, int nt_loads,
                              hipStream_t st);
hipError_t launch_col_sweep_k(const Inst *d_insts, const ColUnit *d_units, int nunits, int grid,
                              int storage, int nt_loads,
                              hipStream_t st);
hipError_t launch_fold_k(const Inst *d_insts, int count, hipStream_t st);
hipError_t launch_advance(const Inst *d_insts, int count, hipStream_t st);
hipError_t launch_check_k(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid, int inst,
                          int n, int nseg, int storage, int nt, double *rsum, double *part, double *csum,
                          hipStream_t st);
hipError_t launch_fused(const Inst *d_insts, int inst, int n, int grid, int storage, int nt_loads,
                        hipStream_t st);
hipError_t launch_gather_ctl(const Inst *d_insts, int count, Ctl *out, hipStream_t st);
// real-valued log-weights (sk_real.hip)
hipError_t launch_real_minmax(const float *W, int n, int64_t pitch, int grid, float *part,
                              hipStream_t st);
hipError_t launch_init_real(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid, int cold,
                            hipStream_t st);
hipError_t launch_row_sweep_real(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid,
                                 size_t lds_bytes, int nt_loads, int vec4, hipStream_t st,
                                 hipEvent_t stop = nullptr);
hipError_t launch_col_sweep_real(const Inst *d_insts, const ColUnit *d_units, int nunits, int grid,
                                 int nt_loads, int vec4, hipStream_t st, hipEvent_t stop = nullptr);
hipError_t launch_check_real(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid, int inst,
                             int n, int nseg, double *rsum, double *rmax, double logt, int64_t *counts,
                             int32_t *hint, double *part, double *csum, hipStream_t st);
hipError_t launch_prune_fill_real(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid,
                                  double logt, const int64_t *row_ptr, int32_t *col, float *w, int n,
                                  hipStream_t st);
hipError_t set_real_attributes();
hipError_t launch_reset_ctl(const Inst *d_insts, const int *idx, int m, hipStream_t st);
hipError_t set_kernel_attributes();

}  // namespace sk
