// Device helpers shared by the HIP kernels, and the log-domain row sweep.
// The row sweep is a template on the waves per SIMD it is compiled for; each
// instantiation lives in a translation unit of its own (sk_kernels.hip: long
// rows; sk_rowshort.hip: batches of short rows), so that neither changes the
// other's code.
#pragma once

#include <type_traits>

#include "sk_exptab.h"

namespace sk {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr float kSafeLo = 5.421010862427522e-20f;  // 2^-64
constexpr float kSafeHi = 1.8446744073709552e19f;  // 2^64

__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float lg2(float x) { return __builtin_amdgcn_logf(x); }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// Contiguous range of work units owned by this workgroup.
__device__ __forceinline__ void unit_range(int nunits, int &u0, int &u1) {
    int per = (nunits + (int)gridDim.x - 1) / (int)gridDim.x;
    u0 = (int)blockIdx.x * per;
    u1 = min(nunits, u0 + per);
}

// LDS position of column j for 8-wide lanes: lane l owns columns
// l*8 + k*512 + c; storing column j at (j%8)*n8 + j/8, n8 = pad8(n)/8, makes
// the 64 lanes read 64 consecutive entries for each c (no bank conflicts).
__device__ __forceinline__ int swz8(int j, int n8) { return (j & 7) * n8 + (j >> 3); }

// In a row's last 8-wide chunk (columns jj..jj+7 with jj + 8 > n) the padding
// columns are marked absent, so the sentinel tests that follow skip them.
__device__ __forceinline__ void mask_pad8(int (&w)[8], int jj, int n) {
    if (jj + 8 > n) {
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if (jj + c >= n) w[c] = SK_SENTINEL;
    }
}

// ---------------------------------------------------------------- row sweep
// One wavefront per row; per column (4 G_j, exp(gam_j)) staged once per
// workgroup in LDS; W read with coalesced 16-byte loads. B = 4 (F_i - shift)
// - 4 kTabLo carries the row's integer part and the shift.

// Column data of the row sweep: a = 4 G_j, g = exp(gam_j).
struct alignas(8) ColPot {
    int a;
    float g;
};

// CP: the column entries' pointer type, an LDS array or (n > kLdsMaxN) a
// global-address-space pointer, so that each instantiation reads them with
// the matching instructions.
// Entry i of the column data, through either pointer type.
template <class CP>
__device__ __forceinline__ ColPot cp_at(CP cp, int i) {
    ColPot k;
    k.a = cp[i].a;
    k.g = cp[i].g;
    return k;
}

template <bool SENT, class CP>
__device__ __forceinline__ float chunk8(const int4 v, int q, int n8, int p4, int B, CP cp,
                                        const float *__restrict__ tab) {
    int w[8];
    unpack8i(v, w);
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const ColPot k = cp_at(cp, c * n8 + q);
        float e = tab_at(tab, tab_off(p4, w[c], k.a, B));
        if (SENT) e = (w[c] == SK_SENTINEL) ? 0.f : e;
        s = fmaf(e, k.g, s);
    }
    return s;
}

// 16-byte loads in flight per lane: the row sweep issues kRowLoads chunks of a
// row before using them; the column sweep double-buffers kColLoads rows (3
// and 4 row chunks, and a software-pipelined row sweep, measured no faster).
constexpr int kRowLoads = 2;
constexpr int kColLoads = 1;

// Row partial sum for one lane: chunks lane*8 + k*512, kRowLoads 16-byte
// loads in flight per lane.
template <bool SENT, bool NT, class CP>
__device__ __forceinline__ float row_partial_v8(const int16_t *__restrict__ wr, int n, int p4,
                                                int B, CP cp, const float *__restrict__ tab, int lane) {
    constexpr int U = kRowLoads;
    const int n8 = pad8(n) >> 3;
    float acc = 0.f;
    int j0 = lane * 8;
    for (; j0 + (U - 1) * 512 < n; j0 += U * 512) {
        int4 v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = gload<NT>(reinterpret_cast<const int4 *>(wr + j0 + k * 512));
        const int q = j0 >> 3;
#pragma unroll
        for (int k = 0; k < U; ++k) acc += chunk8<SENT>(v[k], q + 64 * k, n8, p4, B, cp, tab);
    }
    for (; j0 < n; j0 += 512) {
        const int4 v = gload<NT>(reinterpret_cast<const int4 *>(wr + j0));
        acc += chunk8<SENT>(v, j0 >> 3, n8, p4, B, cp, tab);
    }
    return acc;
}

// max_j of 4 (p w_ij + G_j) + B over the entries of the row (INT_MIN if none).
template <bool SENT, bool NT, class CP>
__device__ __forceinline__ int row_max_v8(const int16_t *__restrict__ wr, int n, int p4, int B, CP cp,
                                          int lane) {
    const int n8 = pad8(n) >> 3;
    int m = INT_MIN;
    for (int j0 = lane * 8; j0 < n; j0 += 512) {
        const int4 v = gload<NT>(reinterpret_cast<const int4 *>(wr + j0));
        int w[8];
        unpack8i(v, w);
        const int q = j0 >> 3;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int t = __mul24(p4, w[c]) + cp[c * n8 + q].a + B;
            if ((!SENT || w[c] != SK_SENTINEL) && j0 + c < n) m = max(m, t);
        }
    }
    return m;
}

template <bool SENT, bool NT, class CP>
__device__ __forceinline__ float row_partial_v1(const int16_t *__restrict__ wr, int n, int p4,
                                                int B, CP cp, const float *__restrict__ tab, int lane) {
    float acc = 0.f;
    for (int j = lane; j < n; j += kWave) {
        const int w = (int)gload<NT>(wr + j);
        const ColPot k = cp_at(cp, j);
        float e = tab_at(tab, tab_off(p4, w, k.a, B));
        if (SENT) e = (w == SK_SENTINEL) ? 0.f : e;
        acc = fmaf(e, k.g, acc);
    }
    return acc;
}

template <bool SENT, bool NT, class CP>
__device__ __forceinline__ int row_max_v1(const int16_t *__restrict__ wr, int n, int p4, int B, CP cp,
                                          int lane) {
    int m = INT_MIN;
    for (int j = lane; j < n; j += kWave) {
        const int w = (int)gload<NT>(wr + j);
        const int t = __mul24(p4, w) + cp[j].a + B;
        if (!SENT || w != SK_SENTINEL) m = max(m, t);
    }
    return m;
}

// What a row step reads from its instance besides W: none of it changes
// during a launch (the controller moves the iterate on between launches), so
// the row sweep loads it once per instance and a row's start waits on no
// chain of dependent loads (unit -> instance -> controller -> potentials).
// The potentials are global-address-space pointers: their loads then count
// only against the vector-memory counter (a flat load counts against the LDS
// counter too, and every LDS wait would include it).
struct RowCtx {
    const int16_t *W;
    int64_t pitch;
    const SK_GLOBAL int32_t *F;  // current iterate
    const SK_GLOBAL float *phi;
    SK_GLOBAL int32_t *Fn;       // next iterate
    SK_GLOBAL float *phin;
    SK_GLOBAL float *rres;
    Ctl *ctl;
    int n, p4;
};

__device__ __forceinline__ RowCtx row_ctx(const Inst &I, int par) {
    RowCtx c;
    c.W = I.W;
    c.pitch = I.pitch;
    c.F = (const SK_GLOBAL int32_t *)(par ? I.F[1] : I.F[0]);
    c.phi = (const SK_GLOBAL float *)(par ? I.phi[1] : I.phi[0]);
    c.Fn = (SK_GLOBAL int32_t *)(par ? I.F[0] : I.F[1]);
    c.phin = (SK_GLOBAL float *)(par ? I.phi[0] : I.phi[1]);
    c.rres = (SK_GLOBAL float *)I.rres;
    c.ctl = I.ctl;
    c.n = I.n;
    c.p4 = 4 * __builtin_amdgcn_readfirstlane(I.ctl->p);
    return c;
}

// Completes the row step of `row` from its sum S relative to the previous
// iterate (shift 0): the exact max-shifted recompute if S left the safe
// range, then the new potentials and the residual.
template <bool SENT, bool V8, bool NT, class CP>
__device__ __forceinline__ float row_finish(const RowCtx &I, int row, int lane, int Fi, float phi, float S,
                                            CP cp, const float *__restrict__ tab) {
    const int n = I.n;
    const int16_t *wr = I.W + (int64_t)row * I.pitch;
    const int p4 = I.p4;
    int M = 0;
    if (!(S >= kSafeLo && S <= kSafeHi)) {
        // exact max-shift (Section 4.1.2): M = max_j (p w_ij + F_i + G_j)
        int m4 = V8 ? row_max_v8<SENT, NT>(wr, n, p4, 4 * Fi, cp, lane)
                    : row_max_v1<SENT, NT>(wr, n, p4, 4 * Fi, cp, lane);
        m4 = wave_max_i(m4);
        if (m4 == INT_MIN) {
            if (lane == 0) atomicOr(&I.ctl->err, ERR_EMPTY_ROW);
            S = 1.f;
        } else {
            M = m4 >> 2;  // exact: m4 is a multiple of 4
            S = V8 ? row_partial_v8<SENT, NT>(wr, n, p4, 4 * (Fi - M - kTabLo), cp, tab, lane)
                   : row_partial_v1<SENT, NT>(wr, n, p4, 4 * (Fi - M - kTabLo), cp, tab, lane);
            S = wave_sum(S);
        }
    }
    if (lane == 0) {
        // log u_i <- F_i - M - log S
        const float l2S = lg2(S);
        const float phin = -l2S * kLn2;
        const float k = rintf(phin);
        I.Fn[row] = Fi - M + (int)k;
        I.phin[row] = phin - k;
        // r_i = exp(phi_i + M) S: row sum of the current iterate
        const float r = ex2(fmaf(phi + (float)M, kLog2e, l2S));
        const float res = fabsf(r - 1.f);
        I.rres[row] = res;
        return res;
    }
    return 0.f;
}

// Fi, phi: the row's potentials, loaded by the caller ahead of the row.
template <bool SENT, bool V8, bool NT, class CP>
__device__ __forceinline__ float row_step_one(const RowCtx &I, int row, int lane, int Fi, float phi, CP cp,
                                             const float *__restrict__ tab) {
    const int n = I.n;
    const int16_t *wr = I.W + (int64_t)row * I.pitch;
    float S = V8 ? row_partial_v8<SENT, NT>(wr, n, I.p4, 4 * (Fi - kTabLo), cp, tab, lane)
                 : row_partial_v1<SENT, NT>(wr, n, I.p4, 4 * (Fi - kTabLo), cp, tab, lane);
    S = wave_sum(S);
    return row_finish<SENT, V8, NT>(I, row, lane, Fi, phi, S, cp, tab);
}

// Rows above kLdsMaxN (column entries from the packed global buffer): a wave
// sweeps R rows at once, so that each chunk of column entries is loaded once
// for the R rows (its L2 traffic per matrix entry drops from 8 bytes to
// 8 / R). The sums of each row are formed exactly as row_partial_v8 forms
// them (the same chunks in the same order).
constexpr int kMultiRows = 4;

template <bool SENT, bool NT, int R, class CP>
__device__ __forceinline__ void row_partial_multi(const int16_t *const (&wr)[R], const bool (&act)[R], int n,
                                                  int p4, const int (&B)[R], CP cp,
                                                  const float *__restrict__ tab, int lane, float (&acc)[R]) {
    const int n8 = pad8(n) >> 3;
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = 0.f;
    for (int j0 = lane * 8; j0 < n; j0 += 512) {
        int4 v[R];
#pragma unroll
        for (int k = 0; k < R; ++k)
            v[k] = act[k] ? gload<NT>(reinterpret_cast<const int4 *>(wr[k] + j0)) : make_int4(0, 0, 0, 0);
        const int q = j0 >> 3;
        ColPot kc[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) kc[c] = cp_at(cp, c * n8 + q);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            int w[8];
            unpack8i(v[k], w);
            float s = 0.f;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                float e = tab_at(tab, tab_off(p4, w[c], kc[c].a, B[k]));
                if (SENT) e = (w[c] == SK_SENTINEL) ? 0.f : e;
                s = fmaf(e, kc[c].g, s);
            }
            acc[k] += s;
        }
    }
}

// Column potentials of the padding columns n..pad8(n)-1 of the 8-wide layout
// (a separate loop, so that the staging of the real columns keeps its loads
// unconditional and in flight together).
// Stages (4 G_j, exp(gam_j)) of every column of I into LDS (swizzled for the
// 8-wide loads when I.vec8). With WIDE, each thread takes 16 consecutive columns and
// issues all of their loads before it uses any, so the staging costs one
// memory round trip per thread rather than one per column; the columns past
// the last full group of 16 (all of them when the vectors are not 16-byte
// aligned) go one per thread. Every value is the one the per-column form
// computes.
// WIDE: the 16-column groups are compiled in (the long-row build; the
// short-row build, at 64 registers, stages one column per thread).
template <bool WIDE>
__device__ __forceinline__ void stage_col_pots(const Inst &I, ColPot *cp, int n8) {
    const int n = I.n;
    const int t = (int)threadIdx.x, nt = (int)blockDim.x;
    int tail = 0;
    if (WIDE && ((reinterpret_cast<uintptr_t>(I.G) | reinterpret_cast<uintptr_t>(I.gam)) & 15) == 0) {
        for (int j0 = 16 * t; j0 + 16 <= n; j0 += 16 * nt) {
            int4 g[4];
            float4 m[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                g[k] = *reinterpret_cast<const int4 *>(I.G + j0 + 4 * k);
                m[k] = *reinterpret_cast<const float4 *>(I.gam + j0 + 4 * k);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int gk[4] = {g[k].x, g[k].y, g[k].z, g[k].w};
                const float mk[4] = {m[k].x, m[k].y, m[k].z, m[k].w};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int j = j0 + 4 * k + c;
                    ColPot v;
                    v.a = 4 * gk[c];
                    v.g = ex2(mk[c] * kLog2e);
                    cp[I.vec8 ? swz8(j, n8) : j] = v;
                }
            }
        }
        tail = n & ~15;
    }
    for (int j = tail + t; j < n; j += nt) {
        ColPot v;
        v.a = 4 * I.G[j];
        v.g = ex2(I.gam[j] * kLog2e);
        cp[I.vec8 ? swz8(j, n8) : j] = v;
    }
}

__device__ __forceinline__ void stage_pad_cols(const Inst &I, ColPot *cp, int n8) {
    if (!I.vec8) return;
    for (int j = I.n + (int)threadIdx.x; j < 8 * n8; j += blockDim.x) {
        ColPot k;
        k.a = kPadExp4;
        k.g = 0.f;
        cp[swz8(j, n8)] = k;
    }
}

// Waves run their rows independently: the only barrier is the restaging of
// the column data when the instance changes. The residual |r_i - 1| goes to
// rres[i] (the column sweep reduces it per row segment for the finalise) and
// each wave's maximum to one of the instance's rowres slots (an exact
// maximum, so the column sweep's reduction of the slots equals the
// finalise's value; it uses it to skip a detection pass).
// MINW is the waves per SIMD the kernel is compiled for: 1 for long rows
// (registers hold loads in flight), 8 for batches of short rows (n <=
// kShortRowN; two workgroups per CU, at most 64 VGPRs). A short row is one or
// two passes of loads, so a wave's time goes to waiting for them, and twice
// the resident waves hide twice the latency.
// GCOL: one instance with n > kLdsMaxN; the column entries are read from
// I.colpack (k_col_pack, mode 0, in the same layout) instead of LDS, where
// the L2 cache holds them (8 bytes per column against 2 of W per entry).
template <bool NT, int MINW, bool GCOL = false>
__global__ __launch_bounds__(kRowWaves * kWave, MINW) void k_row_sweep(const Inst *__restrict__ insts,
                                                                   const RowUnit *__restrict__ units,
                                                                   int nunits,
                                                                   const int32_t *__restrict__ bounds) {
    extern __shared__ ColPot lds_cp[];
    __shared__ float tab[kTabN];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    // the workgroup's units: [bounds[b], bounds[b + 1]) (a split by cost
    // planned on the host), or an even split by count without bounds
    int u0, u1;
    if (bounds) {
        u0 = bounds[blockIdx.x];
        u1 = bounds[blockIdx.x + 1];
    } else {
        unit_range(nunits, u0, u1);
    }
    __shared__ unsigned wg_res, wg_done;
    if (threadIdx.x == 0) {
        wg_res = 0u;
        wg_done = 0u;
    }
    fill_exp_table(tab);
    __syncthreads();
    int cur = -1;
    // GCOL launches hold one instance: its packed entries, read as global
    using CP = std::conditional_t<GCOL, const SK_GLOBAL ColPot *, const ColPot *>;
    CP cp;
    if constexpr (GCOL) cp = (CP)insts[0].colpack;
    else cp = lds_cp;
    float wres = 0.f;  // this wave's residual maximum for instance `cur` (lane 0)
    const int slot = (int)((blockIdx.x * kRowWaves + wave) % kRowResSlots) * kRowResStride;
    auto flush = [&]() {
        if (cur >= 0 && lane == 0 && wres > 0.f)
            atomicMax(&insts[cur].rowres[slot], __float_as_uint(wres));
        wres = 0.f;
    };
    if constexpr (GCOL) {
        // one instance, 8-wide rows: kMultiRows units at a time, wave w taking
        // row w of each
        const Inst &I = insts[0];
        Ctl *ctl = I.ctl;
        if (ctl->state == ST_RUNNING && I.vec8) {
            const RowCtx rc = row_ctx(I, ctl->iter & 1);
            const int n = rc.n, p4 = rc.p4;
            const bool sent = ctl->sent != 0u;
            cur = 0;
            for (int u = u0; u < u1; u += kMultiRows) {
                constexpr int R = kMultiRows;
                const int16_t *wr[R];
                bool act[R];
                int row[R], Fi[R], B[R];
                float phi[R], acc[R];
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    row[k] = u + k < u1 ? units[u + k].row0 + wave : n;
                    act[k] = row[k] < n;
                    const int rr = act[k] ? row[k] : 0;
                    wr[k] = rc.W + (int64_t)rr * rc.pitch;
                    Fi[k] = rc.F[rr];
                    phi[k] = rc.phi[rr];
                    B[k] = 4 * (Fi[k] - kTabLo);
                }
                if (sent) row_partial_multi<true, NT, R>(wr, act, n, p4, B, cp, tab, lane, acc);
                else row_partial_multi<false, NT, R>(wr, act, n, p4, B, cp, tab, lane, acc);
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    if (!act[k]) continue;
                    const float S = wave_sum(acc[k]);
                    const float e = sent ? row_finish<true, true, NT>(rc, row[k], lane, Fi[k], phi[k], S, cp, tab)
                                         : row_finish<false, true, NT>(rc, row[k], lane, Fi[k], phi[k], S, cp, tab);
                    wres = fmaxf(wres, e);
                }
            }
            u0 = u1;  // the loop below has nothing left
        } else if (ctl->state == ST_RUNNING) {
            cur = 0;
        }
    }
    if constexpr (MINW == 1) {
        // The instance of the units in hand: whether it runs, and what its rows
        // read, loaded at each change of instance. With it, lane l of each wave
        // loads the potentials of the wave's row in unit ubase + l (up to 64
        // units ahead; the staging's wait covers these loads), and each row takes
        // its own from that lane with a register read.
        RowCtx rc{};
        bool run = false, sent = false, v8 = false;
        int ucur = -1, ubase = 0;
        int lF = 0;
        float lphi = 0.f;
        for (int u = u0; u < u1; ++u) {
            const RowUnit un = units[u];
            if (un.inst != ucur || u - ubase >= kWave) {
                if (un.inst != ucur) flush();
                const Inst &I = insts[un.inst];
                Ctl *ctl = I.ctl;
                // controller values are the same in every lane: read as
                // scalars, so that what depends on them stays in scalar
                // registers
                run = __builtin_amdgcn_readfirstlane(ctl->state) == ST_RUNNING;
                ucur = un.inst;
                ubase = u;
                if (run) {
                    rc = row_ctx(I, __builtin_amdgcn_readfirstlane(ctl->iter) & 1);
                    sent = __builtin_amdgcn_readfirstlane(ctl->sent) != 0u;
                    v8 = I.vec8 != 0;
                    const int ul = u + lane;
                    if (ul < u1) {
                        const RowUnit x = units[ul];
                        const int r = x.row0 + wave;
                        if (x.inst == un.inst && r < rc.n) {
                            lF = rc.F[r];
                            lphi = rc.phi[r];
                        }
                    }
                    if (!GCOL) {
                        __syncthreads();
                        const int n8 = pad8(rc.n) >> 3;
                        stage_col_pots<MINW == 1>(I, lds_cp, n8);
                        stage_pad_cols(I, lds_cp, n8);
                        __syncthreads();
                    }
                    // an empty use: the wait for these loads falls here, once per
                    // window, not before every row's register read
                    asm volatile("" : "+v"(lF), "+v"(lphi));
                }
                cur = run ? un.inst : -1;
            }
            if (!run) continue;
            const int ra = un.row0 + wave;
            if (ra >= rc.n) continue;
            const int k = u - ubase;
            const int Fi = __builtin_amdgcn_readlane(lF, k);
            const float phi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lphi), k));
            float e;
            if (v8) {
                e = sent ? row_step_one<true, true, NT>(rc, ra, lane, Fi, phi, cp, tab)
                         : row_step_one<false, true, NT>(rc, ra, lane, Fi, phi, cp, tab);
            } else {
                e = sent ? row_step_one<true, false, NT>(rc, ra, lane, Fi, phi, cp, tab)
                         : row_step_one<false, false, NT>(rc, ra, lane, Fi, phi, cp, tab);
            }
            wres = fmaxf(wres, e);
        }
    } else {
        // Short rows (batches of small instances; 64 registers): the unit's
        // values are loaded at the unit, which keeps the registers free.
        for (int u = u0; u < u1; ++u) {
            const RowUnit un = units[u];
            const Inst &I = insts[un.inst];
            Ctl *ctl = I.ctl;
            if (__builtin_amdgcn_readfirstlane(ctl->state) != ST_RUNNING) continue;
            const int n = I.n;
            if (un.inst != cur) {
                flush();
                __syncthreads();
                const int n8 = pad8(n) >> 3;
                stage_col_pots<false>(I, lds_cp, n8);
                stage_pad_cols(I, lds_cp, n8);
                __syncthreads();
                cur = un.inst;
            }
            const RowCtx rc = row_ctx(I, __builtin_amdgcn_readfirstlane(ctl->iter) & 1);
            const bool sent = __builtin_amdgcn_readfirstlane(ctl->sent) != 0u;
            const int ra = un.row0 + wave;
            if (ra >= n) continue;
            const int Fi = rc.F[ra];
            const float phi = rc.phi[ra];
            float e;
            if (I.vec8) {
                e = sent ? row_step_one<true, true, NT>(rc, ra, lane, Fi, phi, cp, tab)
                         : row_step_one<false, true, NT>(rc, ra, lane, Fi, phi, cp, tab);
            } else {
                e = sent ? row_step_one<true, false, NT>(rc, ra, lane, Fi, phi, cp, tab)
                         : row_step_one<false, false, NT>(rc, ra, lane, Fi, phi, cp, tab);
            }
            wres = fmaxf(wres, e);
        }
    }
    // every wave ends on the same instance: the waves' maxima meet in LDS and
    // the last wave to finish sends the workgroup's to the slot
    if (lane == 0) {
        if (wres > 0.f) atomicMax(&wg_res, __float_as_uint(wres));
        __threadfence_block();
        const unsigned k = atomicAdd(&wg_done, 1u);
        if (k == kRowWaves - 1) {
            __threadfence_block();
            const unsigned m = atomicMax(&wg_res, 0u);  // read after every wave's update
            if (cur >= 0 && m > 0u) atomicMax(&insts[cur].rowres[slot], m);
        }
    }
}

}  // namespace sk
