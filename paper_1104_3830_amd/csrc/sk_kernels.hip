// HIP kernels for gfx950 (MI355X): log-domain Sinkhorn sweeps over int16
// log-weights, the FP64 recheck, pruning to CSR, and the stored-K sweeps.
//
// Numerical scheme. With log u_i = F_i + phi_i and log v_j = G_j + gam_j
// (F, G int32; phi, gam float32 with |.| <= 1/2) and integer p and w_ij,
// the exponent p*w_ij + F_i + G_j is an integer below 2^24 in magnitude, so it
// is formed exactly in float32 arithmetic; only the small fractions are
// rounded. This is the max-shifted logarithmic iteration of Section 4.1.2
// with the shift taken from the previous iterate (and an exact two-pass
// max-shift whenever a sum leaves [2^-64, 2^64]).
//
// Row step (u = I(A^(p) v), eq. dad2):   S_i = sum_j exp(p w_ij + F_i + G_j + gam_j),
//                                        log u_i <- F_i - log S_i.
// Column step (v = I(A^(p)T u), eq. dad3): T_j = sum_i exp(p w_ij + F_i + phi_i + G_j),
//                                        log v_j <- G_j - log T_j.
// Row sums of the column-stochastic iterate (Section 4.2 stopping test):
//                                        r_i = exp(phi_i) S_i.
#include <algorithm>

#include "sk_real.h"
#include "sk_ring.h"
#include "sk_rowsweep.h"

namespace sk {

// Visits the entries of one row: lane-strided 8-wide chunks with 16-byte
// loads when the instance allows it, single entries otherwise. f(j, w); the
// padding columns j >= n of the 8-wide layout are passed as SK_SENTINEL.

template <class Fn>
__device__ __forceinline__ void visit_row(const Inst &I, const int16_t *wr, int lane, Fn f) {
    const int n = I.n;
    if (I.vec8) {
        // kVisitLoads 16-byte loads in flight per lane, then their entries in order
        constexpr int U = kVisitLoads;
        auto use = [&](const int4 v, int j0) {
            int w[8];
            unpack8i(v, w);
            mask_pad8(w, j0, n);
#pragma unroll
            for (int c = 0; c < 8; ++c) f(j0 + c, w[c]);
        };
        int j0 = lane * 8;
        for (; j0 + (U - 1) * 512 < n; j0 += U * 512) {
            int4 v[U];
#pragma unroll
            for (int k = 0; k < U; ++k) v[k] = gload<false>(reinterpret_cast<const int4 *>(wr + j0 + k * 512));
#pragma unroll
            for (int k = 0; k < U; ++k) use(v[k], j0 + k * 512);
        }
        for (; j0 < n; j0 += 512) use(gload<false>(reinterpret_cast<const int4 *>(wr + j0)), j0);
    } else {
        for (int j = lane; j < n; j += kWave) f(j, (int)gload<false>(wr + j));
    }
}

// ---------------------------------------------------------------- padded copy
// Copies the caller's W into the library's 8-wide layout (pitch pad8(n),
// columns n.. set to 0) for the instances that have one (Wsrc != nullptr):
// one wave per row, each lane writing 16-byte aligned chunks of 8 columns.
__global__ __launch_bounds__(kRowWaves * kWave) void k_pad_copy(const Inst *__restrict__ insts,
                                                                  const RowUnit *__restrict__ units,
                                                                  int nunits) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int u0, u1;
    unit_range(nunits, u0, u1);
    for (int u = u0; u < u1; ++u) {
        const RowUnit un = units[u];
        const Inst &I = insts[un.inst];
        const int n = I.n, row = un.row0 + wave;
        if (!I.Wsrc || row >= n) continue;
        const uint16_t *src = reinterpret_cast<const uint16_t *>(I.Wsrc) + (int64_t)row * I.src_pitch;
        int16_t *dst = const_cast<int16_t *>(I.W) + (int64_t)row * I.pitch;
        for (int j0 = lane * 8; j0 < n; j0 += 512) {
            unsigned h[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) h[c] = j0 + c < n ? (unsigned)src[j0 + c] : 0u;
            *reinterpret_cast<int4 *>(dst + j0) =
                make_int4((int)(h[0] | (h[1] << 16)), (int)(h[2] | (h[3] << 16)),
                          (int)(h[4] | (h[5] << 16)), (int)(h[6] | (h[7] << 16)));
        }
    }
}

// ---------------------------------------------------------------- input scan / cold start
// Marks instances whose W holds the sentinel and rows with no entry. With
// cold != 0 it also sets the first-stage start (v_0 = 1, eq. dad1) with the
// row shift of Section 4.1.2: F_i = -p*max_j w_ij, phi = 0, G = gam = 0.
__global__ __launch_bounds__(kRowWaves * kWave) void k_init(const Inst *__restrict__ insts,
                                                              const RowUnit *__restrict__ units,
                                                              int nunits, int cold) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int u0, u1;
    unit_range(nunits, u0, u1);
    for (int u = u0; u < u1; ++u) {
        const RowUnit un = units[u];
        const Inst &I = insts[un.inst];
        const int n = I.n, row = un.row0 + wave;
        if (cold && un.row0 == 0) {
            for (int j = threadIdx.x; j < n; j += blockDim.x) {
                I.G[j] = 0;
                I.gam[j] = 0.f;
            }
        }
        if (row >= n) continue;
        const int16_t *wr = I.W + (int64_t)row * I.pitch;
        int mx = -32768;
        int sent = 0;
        visit_row(I, wr, lane, [&](int j, int w) {
            sent |= (w == SK_SENTINEL) & (j < n);  // not the padding columns
            mx = max(mx, w);
        });
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            mx = max(mx, __shfl_xor(mx, o, kWave));
            sent |= __shfl_xor(sent, o, kWave);
        }
        if (lane == 0) {
            if (mx == SK_SENTINEL) atomicOr(&I.ctl->err, ERR_EMPTY_ROW);
            if (sent) atomicOr(&I.ctl->sent, 1u);
            if (cold) {
                I.F[0][row] = (mx == SK_SENTINEL) ? 0 : -I.ctl->p * mx;
                I.phi[0][row] = 0.f;
            }
        }
    }
}

// ---------------------------------------------------------------- column sweep
// Workgroup = column tile x row segment. Lanes own columns (8 per lane with
// 16-byte loads, coalesced along the row); waves split the segment's rows;
// per row (4 (F_i - kTabLo), exp(phi_i)) is staged in LDS; the four waves'
// partial sums are combined through LDS in a fixed order and written to the
// fixed slot colpart[seg][j], which the finalise kernel reduces in slot order.

// The deformed iteration may stop only at an iterate computed at the last p
// (its residual is then measured at that p too: the schedule stays there).
__device__ __forceinline__ bool deform_settled(const Inst &I, const Ctl *ctl) {
    if (I.deform_a <= 0.0) return true;
    if (I.Wr) return deform_p_real(I, ctl->iter) == (double)I.ladder[I.n_p - 1];
    return deform_p(I, ctl->iter) == I.ladder[I.n_p - 1];
}

__device__ __forceinline__ bool stage_converged(const Inst &I, const Ctl *ctl) {
    const float res = __uint_as_float(ctl->res_bits);
    return ctl->iter >= 1 && res < I.tol && deform_settled(I, ctl);
}

// Row data of the column sweep: b = 4 (F_i - kTabLo), r = exp(phi_i).
struct alignas(8) RowPot {
    int b;
    float r;
};

// Start of a lane's 8 columns of a tile (c0 < n): their 4 G_j in A
// (kPadExp4 for padding columns) and the wave's first row of the segment,
// requested now and used by col_partial_v8.
template <bool NT>
__device__ __forceinline__ void col_tile_start(const Inst &I, int c0, int r0, int r1, int wave, int (&A)[8],
                                               int4 &first) {
    const int n = I.n;
    first = make_int4(0, 0, 0, 0);
    if (r0 + wave < r1)
        first = gload<NT>(reinterpret_cast<const int4 *>(I.W + c0 + (int64_t)(r0 + wave) * I.pitch));
    if (c0 + 8 <= n) {
        const int4 g0 = *reinterpret_cast<const int4 *>(I.G + c0);
        const int4 g1 = *reinterpret_cast<const int4 *>(I.G + c0 + 4);
        A[0] = 4 * g0.x; A[1] = 4 * g0.y; A[2] = 4 * g0.z; A[3] = 4 * g0.w;
        A[4] = 4 * g1.x; A[5] = 4 * g1.y; A[6] = 4 * g1.z; A[7] = 4 * g1.w;
    } else {
#pragma unroll
        for (int c = 0; c < 8; ++c) A[c] = c0 + c < n ? 4 * I.G[c0 + c] : kPadExp4;
    }
}

// Column sums of one (512-column tile, row segment) unit over 8-wide rows.
// A: the lane's 4 G_j (kPadExp4 for padding columns); first: the wave's
// first row of the tile, already requested by the caller.
template <bool SENT, bool NT>
__device__ __forceinline__ void col_partial_v8(const Inst &I, int p4, int c0, int r0, int r1, int wave,
                                               const int (&A)[8], int4 first, const RowPot *__restrict__ rowpot,
                                               const float *__restrict__ tab, float (&acc)[8]) {
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.f;
    const int16_t *base = I.W + c0;
    const int64_t pitch = I.pitch;
    auto body = [&](const int4 v, const RowPot rp) {
        int w[8];
        unpack8i(v, w);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            float e = tab_at(tab, tab_off(p4, w[c], A[c], rp.b));
            if (SENT) e = (w[c] == SK_SENTINEL) ? 0.f : e;
            acc[c] = fmaf(e, rp.r, acc[c]);
        }
    };
    constexpr int S = kColWaves;
    int r = r0 + wave;
    if (r >= r1) return;
    // two register buffers: the next row is requested before the current one
    // is used, so a load stays in flight during the arithmetic (rows are
    // still added in order)
    int4 va = first, vb;
    for (;;) {
        const int r2 = r + S;
        const bool more = r2 < r1;
        if (more) vb = gload<NT>(reinterpret_cast<const int4 *>(base + (int64_t)r2 * pitch));
        body(va, rowpot[r - r0]);
        r = r2;
        if (!more) break;
        const int r3 = r + S;
        const bool more2 = r3 < r1;
        if (more2) va = gload<NT>(reinterpret_cast<const int4 *>(base + (int64_t)r3 * pitch));
        body(vb, rowpot[r - r0]);
        r = r3;
        if (!more2) break;
    }
}

// The same over a W without the 8-wide layout: one column per lane.
template <bool SENT, bool NT>
__device__ __forceinline__ void col_partial_v1(const Inst &I, int p4, int tile, int r0, int r1, int wave,
                                               int lane, const RowPot *__restrict__ rowpot,
                                               const float *__restrict__ tab, float &acc) {
    acc = 0.f;
    const int n = I.n;
    const int c0 = tile * kColTile1 + lane;
    if (c0 >= n) return;
    const int A = 4 * I.G[c0];
    for (int r = r0 + wave; r < r1; r += kColWaves) {
        const RowPot rp = rowpot[r - r0];
        const int w = (int)gload<NT>(I.W + (int64_t)r * I.pitch + c0);
        float e = tab_at(tab, tab_off(p4, w, A, rp.b));
        if (SENT) e = (w == SK_SENTINEL) ? 0.f : e;
        acc = fmaf(e, rp.r, acc);
    }
}

// Row potentials a workgroup thread stages per unit: seg_rows <= kMaxSegRows.
constexpr int kColStage = kMaxSegRows / (kColWaves * kWave);

// EARLY (launches whose largest instance has long rows): every load of a
// unit that does not depend on the controller goes out before it is read:
// the wave's first row of the tile, the tile's column potentials, and the
// segment's row potentials of both parities (the parity comes from the
// controller); so the unit's start costs one memory round trip instead of a
// chain of dependent ones. Batches of short rows keep the registers this
// takes (20 per thread) for resident waves, and load at the unit.
template <bool NT, bool EARLY>
__global__ __launch_bounds__(kColWaves * kWave, EARLY ? 1 : 6) void k_col_sweep(const Inst *__restrict__ insts,
                                                                   const ColUnit *__restrict__ units,
                                                                   int nunits) {
    __shared__ float red[kColWaves][kColTile8];
    __shared__ RowPot rowpot[kMaxSegRows];
    __shared__ float tab[kTabN];
    __shared__ float wmax[kColWaves];
    __shared__ float rowres_max;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    constexpr int NTH = kColWaves * kWave;
    int u0, u1;
    unit_range(nunits, u0, u1);
    fill_exp_table(tab);
    for (int u = u0; u < u1; ++u) {
        const ColUnit un = units[u];
        const Inst &I = insts[un.inst];
        Ctl *ctl = I.ctl;
        const int n = I.n;
        const int tc = I.tile_cols;
        const int ctile0 = un.tile * tc;
        const int ncols = min(tc, n - ctile0);
        const int r0 = un.seg * I.seg_rows, r1 = min(n, r0 + I.seg_rows);
        const bool v8 = I.vec8 != 0;
        const bool tile0 = un.tile == 0;
        const int c0 = un.tile * kColTile8 + lane * 8;
        int4 first;
        int A[8];
        int sF[2][kColStage];
        float sP[2][kColStage], sR[kColStage];
        if constexpr (EARLY) {
            if (v8 && c0 < n) col_tile_start<NT>(I, c0, r0, r1, wave, A, first);
#pragma unroll
            for (int k = 0; k < kColStage; ++k) {
                const int r = r0 + (int)threadIdx.x + k * NTH;
                if (r < r1) {
                    sF[0][k] = I.F[0][r];
                    sF[1][k] = I.F[1][r];
                    sP[0][k] = I.phi[0][r];
                    sP[1][k] = I.phi[1][r];
                    sR[k] = tile0 ? I.rres[r] : 0.f;
                }
            }
        }
        float rres_w = 0.f;
        if (EARLY && wave == 0) rres_w = __uint_as_float(I.rowres[lane * kRowResStride]);
        // controller values are the same in every lane: read as scalars
        if (__builtin_amdgcn_readfirstlane(ctl->state) != ST_RUNNING) continue;
        if (!EARLY && wave == 0) rres_w = __uint_as_float(I.rowres[lane * kRowResStride]);
        const int iter = __builtin_amdgcn_readfirstlane(ctl->iter);
        const int npar = (iter + 1) & 1;  // row potentials written by this iteration's row sweep
        const int p4 = 4 * __builtin_amdgcn_readfirstlane(ctl->p);
        const bool sent = __builtin_amdgcn_readfirstlane(ctl->sent) != 0u;
        __syncthreads();
        float rm = 0.f;
        if constexpr (EARLY) {
#pragma unroll
            for (int k = 0; k < kColStage; ++k) {
                const int r = r0 + (int)threadIdx.x + k * NTH;
                if (r < r1) {
                    RowPot kk;
                    kk.b = 4 * ((npar ? sF[1][k] : sF[0][k]) - kTabLo);
                    kk.r = ex2((npar ? sP[1][k] : sP[0][k]) * kLog2e);
                    rowpot[r - r0] = kk;
                    rm = fmaxf(rm, sR[k]);
                }
            }
        } else {
            for (int r = r0 + (int)threadIdx.x; r < r1; r += NTH) {
                RowPot kk;
                kk.b = 4 * (I.F[npar][r] - kTabLo);
                kk.r = ex2(I.phi[npar][r] * kLog2e);
                rowpot[r - r0] = kk;
                if (tile0) rm = fmaxf(rm, I.rres[r]);
            }
        }
        if (tile0) {
            // residual slot of this row segment (read by the finalise kernel)
            rm = wave_max(rm);
            if (lane == 0) wmax[wave] = rm;
        }
        if (wave == 0) {
            // the row sweep's residual (see k_row_sweep)
            const float rr = wave_max(rres_w);
            if (lane == 0) rowres_max = rr;
        }
        __syncthreads();
        if (tile0 && threadIdx.x == 0) {
            float m = wmax[0];
#pragma unroll
            for (int w2 = 1; w2 < kColWaves; ++w2) m = fmaxf(m, wmax[w2]);
            I.res_slots[un.seg] = m;
        }
        // the row sweep measured a converged iterate: the finalise will end
        // the stage without a column step, so no column sums are needed
        if (iter >= 1 && rowres_max < I.tol && deform_settled(I, ctl)) continue;
        if (v8) {
            float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (c0 < n) {
                if constexpr (!EARLY) col_tile_start<NT>(I, c0, r0, r1, wave, A, first);
                if (sent) col_partial_v8<true, NT>(I, p4, c0, r0, r1, wave, A, first, rowpot, tab, acc);
                else col_partial_v8<false, NT>(I, p4, c0, r0, r1, wave, A, first, rowpot, tab, acc);
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) red[wave][lane * 8 + c] = acc[c];
        } else {
            float acc;
            if (sent) col_partial_v1<true, NT>(I, p4, un.tile, r0, r1, wave, lane, rowpot, tab, acc);
            else col_partial_v1<false, NT>(I, p4, un.tile, r0, r1, wave, lane, rowpot, tab, acc);
            red[wave][lane] = acc;
        }
        __syncthreads();
        float *dst = I.colpart + (int64_t)un.seg * n + ctile0;
        for (int c = threadIdx.x; c < ncols; c += blockDim.x) {
            float s = red[0][c];
#pragma unroll
            for (int w2 = 1; w2 < kColWaves; ++w2) s += red[w2][c];
            dst[c] = s;
        }
    }
}

// ---------------------------------------------------------------- column step (finalise)
// Workgroup = 64 columns of one instance, four threads per column. It reduces
// the residual slots of the current iterate (stopping test; group 0 publishes
// the value for the end-of-iteration kernel), and unless the stage has
// converged adds each column's fixed slots in slot order and applies the
// column step (eq. dad3):
//   log-domain sweeps:   slots hold sum_i exp(p w_ij + log u_i + G_j):  gam_j <- -log C_j
//   log-domain 1 pass:   slots hold the column sum of the iterate:       gam_j <- gam_j - log C_j
//   stored K sweeps:     slots hold sum_i K_ij a_i:                      b_j <- 1 / C_j
//   stored K 1 pass:     slots hold b_j sum_i K_ij a_i:                  b_j <- b_j / C_j
// A log-domain column whose sum leaves [2^-64, 2^64] is queued for the exact
// recompute of the end-of-iteration kernel.
// Column slots a thread holds in registers (4 threads per column): up to
// 4 * kFinPre slots (the sweeps' row segments) are requested at the unit's
// start, before the controller is read, so that the unit costs one memory
// round trip; more slots (the single pass) are read in the loop.
constexpr int kFinPre = 8;

__global__ __launch_bounds__(256) void k_col_finalize(const Inst *__restrict__ insts,
                                                      const FinUnit *__restrict__ units, int nunits,
                                                      int mode) {
    __shared__ float part[4][kFinCols];
    __shared__ float rmax[4], dmax[4];
    const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
    const bool kpath = (mode & kFinStoredK) != 0;   // slots written by the stored-K kernels
    const bool onepass = (mode & kFinOnePass) != 0; // slots written by the single-pass kernel
    int u0, u1;
    unit_range(nunits, u0, u1);
    for (int u = u0; u < u1; ++u) {
        const FinUnit un = units[u];
        const Inst &I = insts[un.inst];
        Ctl *ctl = I.ctl;
        const int n = I.n;
        const int c = t & (kFinCols - 1), g = t / kFinCols;
        const int j = un.group * kFinCols + c;
        const int ns = I.ncolslots;
        const bool pre = ns <= 4 * kFinPre;
        float pv[kFinPre];
        if (pre && j < n) {
#pragma unroll
            for (int k = 0; k < kFinPre; ++k) {
                const int q = g + 4 * k;
                pv[k] = q < ns ? I.colpart[(int64_t)q * n + j] : 0.f;
            }
        }
        // residual (and drift) of this iteration's row step: one slot per
        // workgroup of the single pass and of the stored-K row sweep, per
        // row segment of the log-domain sweeps
        const int nres = onepass ? I.fused_grid : (kpath ? I.kres_slots : I.nseg);
        float m = 0.f, d = 0.f;
        for (int q = t; q < nres; q += 256) {
            m = fmaxf(m, I.res_slots[q]);
            if (kpath) d = fmaxf(d, I.drift_slots[q]);
        }
        if (ctl->state != ST_RUNNING) continue;
        if (kpath && ctl->need_absorb) continue;
        m = wave_max(m);
        d = wave_max(d);
        __syncthreads();  // the previous unit's readers of rmax, dmax and part are done
        if (lane == 0) {
            rmax[wave] = m;
            dmax[wave] = d;
        }
        __syncthreads();
        const float res = fmaxf(fmaxf(rmax[0], rmax[1]), fmaxf(rmax[2], rmax[3]));
        const float dm = fmaxf(fmaxf(dmax[0], dmax[1]), fmaxf(dmax[2], dmax[3]));
        const bool conv = ctl->iter >= 1 && res < I.tol && deform_settled(I, ctl);
        if (un.group == 0 && t == 0) {
            ctl->res_bits = __float_as_uint(res);
            if (kpath && dm > 0.f) atomicMax(&ctl->drift_bits, __float_as_uint(dm));
        }
        if (conv) continue;
        // each thread adds the slots g, g + 4, ... of its column, alternately
        // into two sums (fixed order)
        float s0 = 0.f, s1 = 0.f;
        if (j < n) {
            if (pre) {
#pragma unroll
                for (int k = 0; k < kFinPre; ++k) {
                    if (g + 4 * k >= ns) break;
                    if (k & 1) s1 += pv[k];
                    else s0 += pv[k];
                }
            } else {
                int q = g;
                for (; q + 4 < ns; q += 8) {
                    s0 += I.colpart[(int64_t)q * n + j];
                    s1 += I.colpart[(int64_t)(q + 4) * n + j];
                }
                for (; q < ns; q += 4) s0 += I.colpart[(int64_t)q * n + j];
            }
        }
        part[g][c] = s0 + s1;
        __syncthreads();
        float drift = 0.f;
        if (g == 0 && j < n) {
            const float C = (part[0][c] + part[1][c]) + (part[2][c] + part[3][c]);
            if (!kpath) {
                if (C >= kSafeLo && C <= kSafeHi) {
                    const float gn = (onepass ? I.gam[j] : 0.f) - lg2(C) * kLn2;
                    const float k = rintf(gn);
                    I.G[j] += (int)k;
                    I.gam[j] = gn - k;
                } else {
                    const unsigned slot = atomicAdd(&ctl->rescue_cnt, 1u);
                    I.rescue[slot] = (uint32_t)j;
                }
            } else {
                const float Cc = fminf(fmaxf(C, kSafeLo), kSafeHi);
                const float bn = fminf(fmaxf((onepass ? I.b[j] : 1.f) / Cc, kSafeLo), kSafeHi);
                I.b[j] = bn;
                drift = fabsf(lg2(bn));
            }
        }
        if (kpath) {
            drift = wave_max(drift);
            if ((t % kWave) == 0 && drift > 0.f) atomicMax(&ctl->drift_bits, __float_as_uint(drift));
        }
    }
}

// ---------------------------------------------------------------- end of iteration
// One workgroup per instance: exact recompute of flagged columns, commit of
// the iteration, stopping test, and the continuation to the next p with
// p^-1 log u and p^-1 log v held fixed (in FP64).
__device__ void stage_advance(const Inst &I, Ctl *ctl, int par) {
    const int n = I.n;
    const int s = ctl->stage;
    if (s + 1 < I.n_p) {
        const int p0 = I.ladder[s], p1 = I.ladder[s + 1];
        const double ratio = (double)p1 / (double)p0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const double f = ((double)I.F[par][i] + (double)I.phi[par][i]) * ratio;
            const double k = rint(f);
            I.F[0][i] = (int32_t)k;
            I.phi[0][i] = (float)(f - k);
            const double g = ((double)I.G[i] + (double)I.gam[i]) * ratio;
            const double kg = rint(g);
            I.G[i] = (int32_t)kg;
            I.gam[i] = (float)(g - kg);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            ctl->stage = s + 1;
            ctl->p = p1;
            ctl->iter = 0;
        }
    } else {
        // final stage: keep the committed buffer where the parity says
        if (threadIdx.x == 0) ctl->state = ST_DONE;
    }
}

// End of a stage: the log-domain path continues on the device; a stored-K
// path pauses (ST_STAGE_END) so the host can fold the scalings, move to the
// next p and recompute K; so does an instance whose host evaluates every
// stage (certificate, reduced matrix, ratio) before raising p.
__device__ void end_stage(const Inst &I, Ctl *ctl, int par) {
    if (I.deform_a > 0.0) {
        // the deformed iteration is a single stage
        __syncthreads();
        if (threadIdx.x == 0) ctl->state = ST_DONE;
        return;
    }
    if (I.storage == SK_W_I16 && !I.pause) {
        stage_advance(I, ctl, par);
    } else {
        __syncthreads();
        if (threadIdx.x == 0) ctl->state = ST_STAGE_END;
    }
}

// One workgroup of kIterEndThreads per instance (the FP64 rescaling of all
// potentials at a stage change is spread over all of them).
constexpr int kIterEndThreads = 1024;

__global__ __launch_bounds__(kIterEndThreads) void k_iter_end(const Inst *__restrict__ insts) {
    __shared__ int redi[kIterEndThreads];
    __shared__ float red[kIterEndThreads];
    __shared__ float tab[kTabN];
    const Inst &I = insts[blockIdx.x];
    Ctl *ctl = I.ctl;
    if (ctl->state != ST_RUNNING) return;
    const int n = I.n;
    const bool conv = stage_converged(I, ctl);
    const int iter = ctl->iter;
    const int npar = (iter + 1) & 1;
    const int p4 = 4 * ctl->p;
    unsigned nres = conv ? 0u : ctl->rescue_cnt;
    if (I.Wr) {
        // real-valued log-weights: the same recompute with FP64 exponents
        __shared__ double redd[kIterEndThreads];
        for (unsigned q = 0; q < nres; ++q) real_rescue_column(I, ctl, (int)I.rescue[q], npar, redd);
        nres = 0u;
    }
    if (nres > 0u) fill_exp_table(tab);
    // exact max-shifted recompute (Section 4.1.2) of the columns whose sum
    // left the safe range: M = max_i (p w_ij + F_i + G_j), then
    // T_j = e^M sum_i exp(p w_ij + F_i + G_j - M) exp(phi_i)
    for (unsigned q = 0; q < nres; ++q) {
        const int j = (int)I.rescue[q];
        const int A = 4 * I.G[j];
        int m = INT_MIN;
        for (int r = threadIdx.x; r < n; r += blockDim.x) {
            const int w = (int)I.W[(int64_t)r * I.pitch + j];
            if (w == SK_SENTINEL) continue;
            m = max(m, __mul24(p4, w) + A + 4 * I.F[npar][r]);
        }
        __syncthreads();
        redi[threadIdx.x] = m;
        __syncthreads();
        for (int o = kIterEndThreads / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) redi[threadIdx.x] = max(redi[threadIdx.x], redi[threadIdx.x + o]);
            __syncthreads();
        }
        const int m4 = redi[0];
        const int M = m4 >> 2;  // exact: m4 is a multiple of 4 (unused when m4 == INT_MIN)
        float sacc = 0.f;
        if (m4 != INT_MIN) {
            for (int r = threadIdx.x; r < n; r += blockDim.x) {
                const int w = (int)I.W[(int64_t)r * I.pitch + j];
                if (w == SK_SENTINEL) continue;
                const float e = tab_at(tab, tab_off(p4, w, A, 4 * (I.F[npar][r] - M - kTabLo)));
                sacc = fmaf(e, ex2(I.phi[npar][r] * kLog2e), sacc);
            }
        }
        red[threadIdx.x] = sacc;
        __syncthreads();
        if (threadIdx.x == 0) {
            if (m4 == INT_MIN) {
                atomicOr(&ctl->err, ERR_EMPTY_COL);
            } else {
                float S = 0.f;
                for (int t = 0; t < (int)blockDim.x; ++t) S += red[t];
                // log v_j <- G_j - M - log S
                const float gn = -lg2(S) * kLn2;
                const float k = rintf(gn);
                I.G[j] = I.G[j] - M + (int)k;
                I.gam[j] = gn - k;
            }
        }
        __syncthreads();
    }
    for (int q = threadIdx.x; q < kRowResSlots; q += blockDim.x) I.rowres[q * kRowResStride] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
        ctl->rescue_cnt = 0u;
        if (ctl->err & (ERR_EMPTY_ROW | ERR_EMPTY_COL)) ctl->state = ST_ERROR;
    }
    __syncthreads();
    if (ctl->state != ST_RUNNING) return;
    if (conv) {
        if (threadIdx.x == 0) {
            ctl->last_res = __uint_as_float(ctl->res_bits);
            ctl->res_bits = 0u;
        }
        end_stage(I, ctl, iter & 1);
        return;
    }
    // commit: the new row potentials are in buffer npar, i.e. (iter+1) & 1
    if (threadIdx.x == 0) {
        if (iter >= 1) ctl->last_res = __uint_as_float(ctl->res_bits);
        ctl->res_bits = 0u;
        ctl->iter = iter + 1;
        ctl->iters_total += 1;
        ctl->stage_iters[ctl->stage] += 1;
    }
    __syncthreads();
    if ((int64_t)(iter + 1) >= I.max_iters) {
        if (threadIdx.x == 0) ctl->capped += 1;
        end_stage(I, ctl, npar);
    } else if (I.deform_a > 0.0 && threadIdx.x == 0) {
        // deformed iteration: the next iteration's p, potentials unscaled
        ctl->p = deform_p(I, iter + 2);
        ctl->preal = deform_p_real(I, iter + 2);
    }
}

// ---------------------------------------------------------------- FP64 recheck
// Row sums r_i and m_i = max_j (p w_ij + log v_j) in FP64 from the committed
// potentials (Proposition prop:aoc needs sum_i m_i - sum_j log v_j).
// Entries with log x_ij below this contribute less than e^-48 each, i.e. at
// most n e^-48 < 2^-52 to a row or column sum of 1 for n <= 65536 (below one
// FP64 ulp of the sum); their exp is not evaluated.
constexpr double kNegligibleLog = -48.0;

// An entry whose exact integer exponent E = p w_ij + F_i + G_j is below
// kCheckSkip has log x_ij < kNegligibleLog: |phi_i|, |gam_j| <= 1/2.
constexpr int kCheckSkip = -50;

// Integer bound below which no entry can reach log x_ij >= logt (same
// argument: log x_ij <= E + 1).
__device__ __forceinline__ int kept_skip(double logt) {
    return (int)fmax(fmin(floor(logt), 1073741824.0), -1073741824.0) - 2;
}

// Stages the column potentials (G_j, bits of gam_j) for the instance in LDS;
// swizzled like the row sweep when 8-wide chunks are used. log v_j in FP64 is
// (double)G_j + (double)gam_j.
__device__ __forceinline__ void stage_gq(const Inst &I, int2 *gq) {
    const int n = I.n, n8 = pad8(n) >> 3;
    for (int j = threadIdx.x; j < n; j += blockDim.x)
        gq[I.vec8 ? swz8(j, n8) : j] = make_int2(I.G[j], __float_as_int(I.gam[j]));
    if (I.vec8)
        for (int j = n + (int)threadIdx.x; j < 8 * n8; j += blockDim.x) gq[swz8(j, n8)] = make_int2(kPadG, 0);
}
// Entry i of the (G_j, gam_j) column data, through either pointer type.
template <class GQ>
__device__ __forceinline__ int2 gq_ld(GQ gq, int i) {
    return make_int2(gq[i].x, gq[i].y);
}
template <class GQ>
__device__ __forceinline__ int2 gq_at(const Inst &I, GQ gq, int j) {
    return gq_ld(gq, I.vec8 ? swz8(j, pad8(I.n) >> 3) : j);
}
__device__ __forceinline__ double logv_of(int2 q) {
    return (double)q.x + (double)__int_as_float(q.y);
}

// n > kLdsMaxN: the column entries the LDS staging would hold, written to
// I.colpack in the same layout (mode 0: the row sweep's (4 G_j, exp(gam_j));
// mode 1: the FP64 check's and CSR passes' (G_j, bits of gam_j)).
__global__ __launch_bounds__(256) void k_col_pack(const Inst *__restrict__ insts, int inst, int mode) {
    const Inst &I = insts[inst];
    const int n = I.n, n8 = pad8(n) >> 3;
    const int ncols = I.vec8 ? 8 * n8 : n;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ncols) return;
    int2 v;
    if (mode == 0)
        v = j < n ? make_int2(4 * I.G[j], __float_as_int(ex2(I.gam[j] * kLog2e))) : make_int2(kPadExp4, 0);
    else
        v = j < n ? make_int2(I.G[j], __float_as_int(I.gam[j])) : make_int2(kPadG, 0);
    reinterpret_cast<int2 *>(I.colpack)[I.vec8 ? swz8(j, n8) : j] = v;
}

// With counts != nullptr it also counts the entries with log x_ij >= logt
// (the row lengths of B for the scan) and stores in hint[i] the first column
// of the row's largest x_ij (a starting matching for the exact solve).
//
// 8-wide rows: an entry goes through FP64 (its exp, the kept test, the row
// maximum) only when its exact integer exponent reaches eskip; such entries
// are few (about one per 512-column chunk at n = 16384) and scattered over
// the lanes, so they are queued per wave in LDS as (column, w) and evaluated
// 64 at a time, one per lane, instead of one lane at a time in every chunk.
// The queue order is fixed (chunk, then round, then lane), so the sums are
// the same on every run.
// The running state of one row's check: its FP64 sum, the row maximum of
// t = p w_ij + log v_j and its first column, the kept entries, the lane's
// largest p w + G_j, and the entries queued for FP64.
struct RowCheck {
    double s, m;
    int jm, cnt, Emax, qn;
};

// One entry in FP64 (t = p w_ij + log v_j, log x_ij = t + log u_i); gq in
// the full swizzled layout.
template <class GQ>
__device__ __forceinline__ void check_exact(GQ gq, int n8, int j, int w, double p, double f, double logt,
                                            RowCheck &a) {
    const int2 q = gq_ld(gq, (j & 7) * n8 + (j >> 3));
    const double pw = p * (double)w, lvj = logv_of(q);
    const double t = pw + lvj;
    const double lx = t + f;
    if (lx > kNegligibleLog) a.s += exp(lx);
    // the kept test in the exact arithmetic order of the fill kernel
    a.cnt += (pw + f + lvj >= logt);
    if (t > a.m || (t == a.m && j < a.jm)) {
        a.m = t;
        a.jm = j;
    }
}

template <class GQ>
__device__ __forceinline__ void check_flush(GQ gq, int n8, const int2 *qe, int lane, double p, double f,
                                            double logt, RowCheck &a) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (lane < a.qn) {
        const int2 e = qe[lane];
        check_exact(gq, n8, e.x, e.y, p, f, logt, a);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    a.qn = 0;
}

// Pass 1 over the row's columns [lo, hi) (lo a multiple of the step of
// kVisitLoads chunks): the exact integer exponents, with G_j from gs(c, jj)
// (column jj + c); the entries with E >= eskip (T = eskip - F_i) are queued
// for FP64 (check_exact through gq).
// Pass 1 takes in FP64 only the entries with E >= eskip (the others are
// negligible and below the threshold). The row maximum of t is at an
// entry with E >= E* - 1 (E* the largest E; |phi_i|, |gam_j| <= 1/2):
// when E* - 1 >= eskip pass 1 has seen it; otherwise (every entry
// negligible) pass 2 (check_row_finish) looks at the entries with E in
// [E* - 1, eskip).
template <bool SENT, bool NT, class GQ, class GS>
__device__ __forceinline__ void check_row_scan(const Inst &I, GQ gq, GS gs, int2 *qe, const int16_t *wr, int lane,
                                               int lo, int hi, int pi, double p, double f, int T, double logt,
                                               RowCheck &a) {
    const int n = I.n, n8 = pad8(n) >> 3;
    // The entries of one 8-wide chunk (columns jj..jj+7 of this lane).
    auto chunk = [&](int jj, int (&w)[8]) {
        int e8[8];
        bool hit = false;
        if (jj < n) {
            mask_pad8(w, jj, n);
            int m8 = INT_MIN;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                // 24-bit multiply-add, exact: |p w| <= 2048 * 32768 = 2^26
                e8[c] = (!SENT || w[c] != SK_SENTINEL) ? __mul24(pi, w[c]) + gs(c, jj) : INT_MIN;
                m8 = max(m8, e8[c]);
            }
            a.Emax = max(a.Emax, m8);
            hit = m8 >= T;
        }
        // the per-entry flags only where a lane's chunk reaches the
        // threshold (about one chunk in three has none in the wave)
        if (__ballot(hit) == 0ull) return;
        unsigned flag = 0;
        if (hit) {
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (e8[c] >= T) flag |= 1u << c;
        }
        // queue the flagged entries: per round, every lane with one left
        // appends its lowest, in lane order
        for (;;) {
            const uint64_t mask = __ballot(flag != 0u);
            if (mask == 0ull) break;
            const int nq = __popcll(mask);
            if (a.qn + nq > kWave) check_flush(gq, n8, qe, lane, p, f, logt, a);
            if (flag) {
                const int c = __ffs(flag) - 1;
                const int pos = a.qn + __popcll(mask & ((1ull << lane) - 1ull));
                qe[pos] = make_int2(jj + c, w[c]);
                flag &= flag - 1u;
            }
            a.qn += nq;
        }
    };
    ring_row_chunks<NT>(wr, n, lane, lo, hi, chunk);
}

// The rest of the row's check after its pass 1: the queued entries, pass 2
// when every entry was negligible, the wave reductions and the results.
template <bool SENT, class GQ>
__device__ __forceinline__ void check_row_finish(const Inst &I, GQ gq, const int2 *qe, const int16_t *wr, int row,
                                                 int lane, int eskip, int pi, double p, int Fi, double f,
                                                 double logt, double *rsum, double *rmax, int64_t *counts,
                                                 int32_t *hint, RowCheck &a) {
    const int n8 = pad8(I.n) >> 3;
    if (a.qn) check_flush(gq, n8, qe, lane, p, f, logt, a);
    double s = a.s, m = a.m;
    int jm = a.jm, cnt = a.cnt;
    const int Es = wave_max_i(a.Emax == INT_MIN ? INT_MIN : a.Emax + Fi);
    if (Es != INT_MIN && Es - 1 < eskip) {
        visit_row(I, wr, lane, [&](int j, int w) {
            if (w == SK_SENTINEL) return;
            const int2 q = gq_ld(gq, (j & 7) * n8 + (j >> 3));
            const int E = __mul24(pi, w) + q.x + Fi;
            if (E < Es - 1 || E >= eskip) return;
            const double t = p * (double)w + logv_of(q);
            if (t > m || (t == m && j < jm)) {
                m = t;
                jm = j;
            }
        });
    }
    s = wave_sum_d(s);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double m2 = __shfl_xor(m, o, kWave);
        const int j2 = __shfl_xor(jm, o, kWave);
        if (m2 > m || (m2 == m && (unsigned)j2 < (unsigned)jm)) {
            m = m2;
            jm = j2;
        }
        cnt += __shfl_xor(cnt, o, kWave);
    }
    if (lane == 0) {
        rsum[row] = s;
        rmax[row] = m;
        if (counts) {
            counts[row] = cnt;
            hint[row] = jm;
        }
    }
}

// A wave-uniform value moved to scalar registers (every lane holds it).
__device__ __forceinline__ float rfl_f(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ int64_t rfl_i64(int64_t x) {
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(x >> 32));
    return (int64_t)((hi << 32) | (uint32_t)__builtin_amdgcn_readfirstlane((int)x));
}

// n > kLdsMaxN: G_j of the row's columns staged in LDS kGTile at a time for
// the integer scan, column j of the tile starting at lo at
// (j mod 8) kGT8 + (j - lo) / 8 (the lanes of a wave read consecutive
// words). 128 KiB: one tile up to n = 32768.
constexpr int kGTile = 32768;
constexpr int kGT8 = kGTile / 8;

__device__ __forceinline__ void stage_g_tile(const Inst &I, int *gG, int lo) {
    const int n = I.n, hi = min(lo + kGTile, pad8(n));
    for (int j = lo + (int)threadIdx.x; j < hi; j += blockDim.x)
        gG[(j & 7) * kGT8 + ((j - lo) >> 3)] = j < n ? I.G[j] : kPadG;
}

// The whole row with its column entries in one layout (LDS, n <= kLdsMaxN).
template <bool SENT, bool NT, class GQ>
__device__ __forceinline__ void check_row_v8(const Inst &I, GQ gq, int2 *qe, int row, int lane,
                                             int eskip, double logt, double *rsum, double *rmax,
                                             int64_t *counts, int32_t *hint) {
    const int n = I.n, n8 = pad8(n) >> 3;
    const int par = I.ctl->iter & 1;
    const int pi = I.ctl->p, Fi = I.F[par][row];
    const double p = (double)pi;
    const double f = (double)Fi + (double)I.phi[par][row];
    const int16_t *wr = I.W + (int64_t)row * I.pitch;
    // Emax: the lane's largest p w + G_j (E = p w + F_i + G_j without the
    // row's F_i, which moves into the threshold: E >= eskip <=> p w + G_j >= T)
    RowCheck a{0.0, -INFINITY, -1, 0, INT_MIN, 0};
    auto gs = [&](int c, int jj) { return gq[c * n8 + (jj >> 3)].x; };
    check_row_scan<SENT, NT>(I, gq, gs, qe, wr, lane, 0, n, pi, p, f, eskip - Fi, logt, a);
    check_row_finish<SENT>(I, gq, qe, wr, row, lane, eskip, pi, p, Fi, f, logt, rsum, rmax, counts, hint, a);
}

// GCOL: one instance with n > kLdsMaxN, its column entries read from
// I.colpack (packed by k_col_pack, mode 1) instead of staged in LDS.
template <bool NT, bool GCOL>
__global__ __launch_bounds__(kRowWaves * kWave) void k_check_rows(const Inst *__restrict__ insts,
                                                                    const RowUnit *__restrict__ units,
                                                                    int nunits, double *rsum,
                                                                    double *rmax, double logt,
                                                                    int64_t *counts, int32_t *hint) {
    extern __shared__ int2 gq_lds[];
    __shared__ int2 queue[kRowWaves][kWave];
    // GCOL launches hold one instance: its packed entries, read as global
    using GQ = std::conditional_t<GCOL, const SK_GLOBAL int2 *, const int2 *>;
    GQ gq;
    if constexpr (GCOL) gq = (GQ)insts[0].colpack;
    else gq = gq_lds;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int u0, u1;
    unit_range(nunits, u0, u1);
    const int eskip = counts ? min(kCheckSkip, kept_skip(logt)) : kCheckSkip;
    if constexpr (GCOL) {
        if (insts[0].vec8) {
            // The integer scan reads G_j from LDS tiles (staged once when the
            // row fits one tile); the FP64 entries and pass 2 read (G_j,
            // gam_j) from the packed buffer, as the whole-row form does, so
            // the queue and the results are the same.
            __shared__ int gG[kGTile];
            const Inst &I = insts[0];
            const int n = I.n, ntile = (n + kGTile - 1) / kGTile;
            // the row's state is wave-uniform: kept in scalar registers
            const bool sent = __builtin_amdgcn_readfirstlane(I.ctl->sent) != 0u;
            const int par = __builtin_amdgcn_readfirstlane(I.ctl->iter) & 1;
            const int pi = __builtin_amdgcn_readfirstlane(I.ctl->p);
            const double p = (double)pi;
            for (int u = u0; u < u1; ++u) {
                const int row = __builtin_amdgcn_readfirstlane(units[u].row0 + wave);
                const bool on = row < n;
                const int Fi = on ? __builtin_amdgcn_readfirstlane(I.F[par][row]) : 0;
                const double f = (double)Fi + (double)(on ? rfl_f(I.phi[par][row]) : 0.0f);
                const int16_t *wr = I.W + (int64_t)(on ? row : 0) * I.pitch;
                RowCheck a{0.0, -INFINITY, -1, 0, INT_MIN, 0};
                for (int t = 0; t < ntile; ++t) {
                    const int lo = t * kGTile, hi = min(n, lo + kGTile);
                    if (ntile > 1 || u == u0) {
                        __syncthreads();
                        stage_g_tile(I, gG, lo);
                        __syncthreads();
                    }
                    if (!on) continue;
                    auto gs = [&](int c, int jj) { return gG[c * kGT8 + ((jj - lo) >> 3)]; };
                    if (sent)
                        check_row_scan<true, NT>(I, gq, gs, queue[wave], wr, lane, lo, hi, pi, p, f, eskip - Fi, logt,
                                                 a);
                    else
                        check_row_scan<false, NT>(I, gq, gs, queue[wave], wr, lane, lo, hi, pi, p, f, eskip - Fi, logt,
                                                  a);
                }
                if (!on) continue;
                if (sent)
                    check_row_finish<true>(I, gq, queue[wave], wr, row, lane, eskip, pi, p, Fi, f, logt, rsum, rmax,
                                           counts, hint, a);
                else
                    check_row_finish<false>(I, gq, queue[wave], wr, row, lane, eskip, pi, p, Fi, f, logt, rsum, rmax,
                                            counts, hint, a);
            }
            return;
        }
    }
    int cur = -1;
    for (int u = u0; u < u1; ++u) {
        const RowUnit un = units[u];
        const Inst &I = insts[un.inst];
        if (un.inst != cur) {
            if (!GCOL) {
                __syncthreads();
                stage_gq(I, gq_lds);
                __syncthreads();
            }
            cur = un.inst;
        }
        const int n = I.n, row = un.row0 + wave;
        if (row >= n) continue;
        if (I.vec8) {
            if (I.ctl->sent != 0u)
                check_row_v8<true, NT>(I, gq, queue[wave], row, lane, eskip, logt, rsum, rmax, counts, hint);
            else
                check_row_v8<false, NT>(I, gq, queue[wave], row, lane, eskip, logt, rsum, rmax, counts, hint);
            continue;
        }
        const int par = I.ctl->iter & 1;
        const int pi = I.ctl->p, Fi = I.F[par][row];
        const double p = (double)pi;
        const double f = (double)Fi + (double)I.phi[par][row];
        const int16_t *wr = I.W + (int64_t)row * I.pitch;
        double s = 0.0, m = -INFINITY;
        int jm = -1, cnt = 0;
        int Emax = INT_MIN;
        auto exact = [&](int j, int w, int2 q) {
            const double pw = p * (double)w, lvj = logv_of(q);
            const double t = pw + lvj;
            const double lx = t + f;
            if (lx > kNegligibleLog) s += exp(lx);
            cnt += (pw + f + lvj >= logt);
            if (t > m) {  // a lane visits its columns in increasing order
                m = t;
                jm = j;
            }
        };
        visit_row(I, wr, lane, [&](int j, int w) {
            if (w == SK_SENTINEL) return;
            const int2 q = gq_at(I, gq, j);
            const int E = __mul24(pi, w) + q.x + Fi;
            Emax = max(Emax, E);
            if (E >= eskip) exact(j, w, q);
        });
        const int Es = wave_max_i(Emax);
        if (Es != INT_MIN && Es - 1 < eskip) {
            visit_row(I, wr, lane, [&](int j, int w) {
                if (w == SK_SENTINEL) return;
                const int2 q = gq_at(I, gq, j);
                const int E = __mul24(pi, w) + q.x + Fi;
                if (E < Es - 1 || E >= eskip) return;
                const double t = p * (double)w + logv_of(q);
                if (t > m || (t == m && j < jm)) {
                    m = t;
                    jm = j;
                }
            });
        }
        s = wave_sum_d(s);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double m2 = __shfl_xor(m, o, kWave);
            const int j2 = __shfl_xor(jm, o, kWave);
            if (m2 > m || (m2 == m && (unsigned)j2 < (unsigned)jm)) {
                m = m2;
                jm = j2;
            }
            cnt += __shfl_xor(cnt, o, kWave);
        }
        if (lane == 0) {
            rsum[row] = s;
            rmax[row] = m;
            if (counts) {
                counts[row] = cnt;
                hint[row] = jm;
            }
        }
    }
}

// Column sums in FP64, two passes: workgroup (256-column tile, row segment)
// with one thread per column writes a partial to slot [segment][column]
// (coalesced along each row); then one thread per column adds its slots in
// segment order.
__global__ __launch_bounds__(256) void k_check_cols_part(const Inst *__restrict__ insts, int inst,
                                                         double *part) {
    const Inst &I = insts[inst];
    const int n = I.n;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int seg = blockIdx.y;
    if (j >= n) return;
    const int r0 = seg * I.seg_rows, r1 = min(n, r0 + I.seg_rows);
    const int par = I.ctl->iter & 1;
    const double p = (double)I.ctl->p;
    const double g = (double)I.G[j] + (double)I.gam[j];
    double s = 0.0;
    for (int r = r0; r < r1; ++r) {
        const int w = I.W[(int64_t)r * I.pitch + j];
        if (w == SK_SENTINEL) continue;
        const double lx = p * (double)w + g + ((double)I.F[par][r] + (double)I.phi[par][r]);
        if (lx > kNegligibleLog) s += exp(lx);
    }
    part[(int64_t)seg * n + j] = s;
}

__global__ __launch_bounds__(256) void k_check_cols_sum(const Inst *__restrict__ insts, int inst,
                                                        const double *part, double *csum) {
    const Inst &I = insts[inst];
    const int n = I.n;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int seg = 0; seg < I.nseg; ++seg) s += part[(int64_t)seg * n + j];
    csum[j] = s;
}

// The same slots from 8 columns per lane (16-byte loads along each row) with
// the segment's rows split over four waves and the waves' sums added in a
// fixed order. The exact integer part E = p w_ij + F_i + G_j decides first
// (E < kCheckSkip: negligible).

__device__ __forceinline__ void check_cols_add8(const int (&w)[8], int p, int2 rf, const int (&G)[8],
                                                const double (&gm)[8], double (&s)[8]) {
    // E = p w + F_i + G_j; the chunk's largest p w + G_j first: when it is
    // below kCheckSkip - F_i (the usual case) no entry is taken
    int e[8];
    int m8 = INT_MIN;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        e[c] = __mul24(p, w[c]) + G[c];
        m8 = max(m8, e[c]);
    }
    if (m8 < kCheckSkip - rf.x) return;
    const double ph = (double)__int_as_float(rf.y);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int E = e[c] + rf.x;
        if (w[c] != SK_SENTINEL && E >= kCheckSkip) {
            const double lx = (double)E + (ph + gm[c]);
            if (lx > kNegligibleLog) s[c] += exp(lx);
        }
    }
}

template <bool NT>
__global__ __launch_bounds__(kColWaves * kWave) void k_check_cols_part8(const Inst *__restrict__ insts,
                                                                        int inst, double *part) {
    __shared__ double red[kColWaves][kColTile8];
    __shared__ int2 rowf[kMaxSegRows];
    const Inst &I = insts[inst];
    const int n = I.n;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int ctile0 = blockIdx.x * kColTile8;
    const int seg = blockIdx.y;
    const int r0 = seg * I.seg_rows, r1 = min(n, r0 + I.seg_rows);
    const int par = I.ctl->iter & 1;
    const int p = I.ctl->p;
    for (int r = r0 + (int)threadIdx.x; r < r1; r += blockDim.x)
        rowf[r - r0] = make_int2(I.F[par][r], __float_as_int(I.phi[par][r]));
    __syncthreads();
    const int j0 = ctile0 + lane * 8;
    double s[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) s[c] = 0.0;
    if (j0 < n) {
        // padding columns (j0 + c >= n) fall below kCheckSkip and are not written
        int G[8];
        double gm[8];
        if (j0 + 8 <= n) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                G[c] = I.G[j0 + c];
                gm[c] = (double)I.gam[j0 + c];
            }
        } else {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                G[c] = j0 + c < n ? I.G[j0 + c] : kPadG;
                gm[c] = j0 + c < n ? (double)I.gam[j0 + c] : 0.0;
            }
        }
        // this wave's rows r0 + wave + m kColWaves of the segment, through the
        // load ring (loads past the segment read its last row, unused); the
        // row index is wave-uniform and kept in a scalar register
        const int ra = __builtin_amdgcn_readfirstlane(r0 + wave);
        ring_col_chunks<NT>(
            r1 > ra ? (r1 - ra + kColWaves - 1) / kColWaves : 0,
            [&](int m) {
                return reinterpret_cast<const int4 *>(I.W + (int64_t)min(ra + m * kColWaves, r1 - 1) * I.pitch + j0);
            },
            [&](int m, int (&w)[8]) { check_cols_add8(w, p, rowf[ra + m * kColWaves - r0], G, gm, s); });
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) red[wave][lane * 8 + c] = s[c];
    __syncthreads();
    double *dst = part + (int64_t)seg * n + ctile0;
    const int ncols = min(kColTile8, n - ctile0);
    for (int c = threadIdx.x; c < ncols; c += blockDim.x) {
        double t = red[0][c];
#pragma unroll
        for (int w2 = 1; w2 < kColWaves; ++w2) t += red[w2][c];
        dst[c] = t;
    }
}

// Reduces the FP64 check of one instance to four numbers, in a fixed order:
// out[0] = max_i |r_i - 1|, out[1] = max_j |c_j - 1|, out[2] = sum_i m_i,
// out[3] = sum_j log v_j (the certificate is (out[2] - out[3]) / p).
__global__ __launch_bounds__(256) void k_check_reduce(const Inst *__restrict__ insts, int inst,
                                                      const double *rsum, const double *rmax,
                                                      const double *csum, double *out) {
    __shared__ double a[256], b[256], c[256], d[256];
    const Inst &I = insts[inst];
    const int n = I.n, t = threadIdx.x;
    double ra = 0.0, ca = 0.0, sm = 0.0, sg = 0.0;
    for (int i = t; i < n; i += 256) {
        ra = fmax(ra, fabs(rsum[i] - 1.0));
        ca = fmax(ca, fabs(csum[i] - 1.0));
        sm += rmax[i];
        sg += (double)I.G[i] + (double)I.gam[i];
    }
    a[t] = ra;
    b[t] = ca;
    c[t] = sm;
    d[t] = sg;
    __syncthreads();
    if (t == 0) {
        double A = 0.0, Bm = 0.0, C = 0.0, D = 0.0;
        for (int k = 0; k < 256; ++k) {
            A = fmax(A, a[k]);
            Bm = fmax(Bm, b[k]);
            C += c[k];
            D += d[k];
        }
        out[0] = A;
        out[1] = Bm;
        out[2] = C;
        out[3] = D;
    }
}

// ---------------------------------------------------------------- prune
// B keeps (i, j) iff x_ij(p) >= t (eq. matrixred); the comparison is made on
// log x_ij = p w_ij + log u_i + log v_j in FP64.

// The kept entries (x_ij >= t) of one 8-wide chunk, columns j0..j0+7 with
// j0 < n, as a bit mask: the exact integer exponent first (below eskip an
// entry cannot reach t), FP64 only for the few that pass. G_j for the
// integer test from gs(c, j0), (G_j, gam_j) for FP64 from gq in the full
// layout. The CSR count and fill both decide through this function, so the
// fill places exactly the entries counted.
template <class GQ, class GS>
__device__ __forceinline__ unsigned kept8(GQ gq, GS gs, int (&wv)[8], int j0, int n, int n8, int pi, double p, int Fi,
                                          double f, int eskip, double logt, bool sent) {
    mask_pad8(wv, j0, n);
    const int base = j0 >> 3;
    // the chunk's largest p w + G_j first: below eskip - F_i (the usual
    // case) no entry is a candidate
    int e[8], m8 = INT_MIN;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        e[c] = __mul24(pi, wv[c]) + gs(c, j0);
        m8 = max(m8, e[c]);
    }
    if (m8 < eskip - Fi) return 0u;
    unsigned cand = 0, keep = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c)
        if (e[c] + Fi >= eskip) cand |= 1u << c;
    if (sent) {
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if (wv[c] == SK_SENTINEL) cand &= ~(1u << c);
    }
    if (cand) {
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if (cand & (1u << c)) {
                const double lx = p * (double)wv[c] + f + logv_of(gq_ld(gq, c * n8 + base));
                if (lx >= logt) keep |= 1u << c;
            }
    }
    return keep;
}

// The number of kept entries of one 8-wide row over its columns [lo, hi)
// (lo a multiple of the step of kVisitLoads chunks), added to cnt.
template <bool NT, class GQ, class GS>
__device__ __forceinline__ void count_row_range(const Inst &I, GQ gq, GS gs, const int16_t *wr, int lane, int lo,
                                                int hi, int pi, double p, int Fi, double f, int eskip,
                                                double logt, bool sent, int &cnt) {
    const int n = I.n, n8 = pad8(n) >> 3;
    ring_row_chunks<NT>(wr, n, lane, lo, hi, [&](int j0, int (&wv)[8]) {
        if (j0 < n) cnt += __popc(kept8(gq, gs, wv, j0, n, n8, pi, p, Fi, f, eskip, logt, sent));
    });
}

template <bool NT, bool GCOL>
__global__ __launch_bounds__(kRowWaves * kWave) void k_prune_count(const Inst *__restrict__ insts,
                                                                     const RowUnit *__restrict__ units,
                                                                     int nunits, double logt,
                                                                     int64_t *counts) {
    extern __shared__ int2 gq_lds[];
    // GCOL launches hold one instance: its packed entries, read as global
    using GQ = std::conditional_t<GCOL, const SK_GLOBAL int2 *, const int2 *>;
    GQ gq;
    if constexpr (GCOL) gq = (GQ)insts[0].colpack;
    else gq = gq_lds;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int u0, u1;
    unit_range(nunits, u0, u1);
    const int eskip = kept_skip(logt);
    if constexpr (GCOL) {
        if (insts[0].vec8) {
            // the integer test reads G_j from LDS tiles (as the CSR fill)
            __shared__ int gG[kGTile];
            const Inst &I = insts[0];
            const int n = I.n, ntile = (n + kGTile - 1) / kGTile;
            // the row's state is wave-uniform: kept in scalar registers
            const bool sent = __builtin_amdgcn_readfirstlane(I.ctl->sent) != 0u;
            const int par = __builtin_amdgcn_readfirstlane(I.ctl->iter) & 1;
            const int pi = __builtin_amdgcn_readfirstlane(I.ctl->p);
            const double p = (double)pi;
            for (int u = u0; u < u1; ++u) {
                const int row = __builtin_amdgcn_readfirstlane(units[u].row0 + wave);
                const bool on = row < n;
                const int Fi = on ? __builtin_amdgcn_readfirstlane(I.F[par][row]) : 0;
                const double f = (double)Fi + (double)(on ? rfl_f(I.phi[par][row]) : 0.0f);
                const int16_t *wr = I.W + (int64_t)(on ? row : 0) * I.pitch;
                int cnt = 0;
                for (int t = 0; t < ntile; ++t) {
                    const int lo = t * kGTile, hi = min(n, lo + kGTile);
                    if (ntile > 1 || u == u0) {
                        __syncthreads();
                        stage_g_tile(I, gG, lo);
                        __syncthreads();
                    }
                    if (!on) continue;
                    auto gs = [&](int c, int j0) { return gG[c * kGT8 + ((j0 - lo) >> 3)]; };
                    count_row_range<NT>(I, gq, gs, wr, lane, lo, hi, pi, p, Fi, f, eskip, logt, sent, cnt);
                }
                if (!on) continue;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, kWave);
                if (lane == 0) counts[row] = cnt;
            }
            return;
        }
    }
    int cur = -1;
    for (int u = u0; u < u1; ++u) {
        const RowUnit un = units[u];
        const Inst &I = insts[un.inst];
        if (un.inst != cur) {
            if (!GCOL) {
                __syncthreads();
                stage_gq(I, gq_lds);
                __syncthreads();
            }
            cur = un.inst;
        }
        const int n = I.n, row = un.row0 + wave;
        if (row >= n) continue;
        const int par = I.ctl->iter & 1;
        const int pi = I.ctl->p, Fi = I.F[par][row];
        const double p = (double)pi;
        const double f = (double)Fi + (double)I.phi[par][row];
        const int16_t *wr = I.W + (int64_t)row * I.pitch;
        int cnt = 0;
        if (I.vec8) {
            const int n8 = pad8(n) >> 3;
            auto gs = [&](int c, int j0) { return gq[c * n8 + (j0 >> 3)].x; };
            count_row_range<NT>(I, gq, gs, wr, lane, 0, n, pi, p, Fi, f, eskip, logt, I.ctl->sent != 0u, cnt);
        } else {
            visit_row(I, wr, lane, [&](int j, int w) {
                if (w == SK_SENTINEL) return;
                const int2 q = gq_at(I, gq, j);
                if (__mul24(pi, w) + q.x + Fi < eskip) return;  // cannot reach t
                const double lx = p * (double)w + f + logv_of(q);
                cnt += (lx >= logt);
            });
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, kWave);
        if (lane == 0) counts[row] = cnt;
    }
}

// Exclusive scan of n row counts into row_ptr[0..n] (one workgroup).
__global__ __launch_bounds__(1024) void k_scan(const int64_t *__restrict__ counts,
                                               int64_t *__restrict__ row_ptr, int n,
                                               int64_t *total_out) {
    // thread t sums a contiguous block (read kScanPer at a time, their loads
    // in flight together: one round for n <= 16384); the block sums are
    // scanned with shuffles within each wave and across the 16 wave totals
    constexpr int kScanPer = 16;
    __shared__ int64_t wsum[1024 / kWave];
    const int t = threadIdx.x, wave = t / kWave, lane = t % kWave;
    const int per = (n + 1023) / 1024;
    const int a = min(n, t * per), b = min(n, a + per);
    int64_t s = 0;
    for (int i0 = a; i0 < b; i0 += kScanPer) {
        int64_t c[kScanPer];
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) c[k] = i0 + k < b ? counts[i0 + k] : 0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) s += c[k];
    }
    int64_t x = s;  // inclusive scan within the wave
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int64_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wsum[wave] = x;
    __syncthreads();
    if (wave == 0) {
        int64_t v = lane < 1024 / kWave ? wsum[lane] : 0;
#pragma unroll
        for (int o = 1; o < 1024 / kWave; o <<= 1) {
            const int64_t y = __shfl_up(v, o, kWave);
            if (lane >= o) v += y;
        }
        if (lane < 1024 / kWave) wsum[lane] = v;
    }
    __syncthreads();
    int64_t run = x - s + (wave > 0 ? wsum[wave - 1] : 0);
    if (t == 1023) {
        const int64_t total = wsum[1024 / kWave - 1];
        row_ptr[n] = total;
        if (total_out) *total_out = total;
    }
    for (int i0 = a; i0 < b; i0 += kScanPer) {
        int64_t c[kScanPer];
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) c[k] = i0 + k < b ? counts[i0 + k] : 0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k)
            if (i0 + k < b) {
                row_ptr[i0 + k] = run;
                run += c[k];
            }
    }
}

// Writes the kept columns of each row in increasing order: each wave walks
// its row in 64-column chunks and places the kept ones with a ballot prefix.
// The CSR entries of one 8-wide row over its columns [lo, hi) (lo a
// multiple of the step of kVisitLoads chunks), placed from pos on: each lane
// tests 8 consecutive columns; kept entries are placed by a wave prefix sum
// of the per-lane counts (column order kept), skipped for the chunks where no
// lane keeps an entry. The kept test is kept8's.
template <bool NT, bool SPOS, class GQ, class GS>
__device__ __forceinline__ void fill_row_range(const Inst &I, GQ gq, GS gs, const int16_t *wr, int lane, int lo,
                                               int hi, int pi, double p, int Fi, double f, int eskip,
                                               double logt, bool sent, int64_t &pos, int32_t *__restrict__ col,
                                               int16_t *__restrict__ wout) {
    const int n = I.n, n8 = pad8(n) >> 3;
    ring_row_chunks<NT>(wr, n, lane, lo, hi, [&](int j0, int (&wv)[8]) {
        const unsigned keep = j0 < n ? kept8(gq, gs, wv, j0, n, n8, pi, p, Fi, f, eskip, logt, sent) : 0u;
        if (__ballot(keep != 0u) == 0ull) return;  // nothing kept in this chunk
        const int cnt = __popc(keep);
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int y = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += y;
        }
        // every lane is active here: with SPOS the wave's count is moved
        // to a scalar register, so pos stays scalar
        int total = __shfl(incl, kWave - 1, kWave);
        if constexpr (SPOS) total = __builtin_amdgcn_readfirstlane(total);
        int64_t q = pos + (incl - cnt);
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if (keep & (1u << c)) {
                col[q] = j0 + c;
                wout[q] = (int16_t)wv[c];
                ++q;
            }
        pos += total;
    });
}

template <bool NT, bool GCOL>
__global__ __launch_bounds__(kRowWaves * kWave) void k_prune_fill(const Inst *__restrict__ insts,
                                                                    const RowUnit *__restrict__ units,
                                                                    int nunits, double logt,
                                                                    const int64_t *__restrict__ row_ptr,
                                                                    int32_t *__restrict__ col,
                                                                    int16_t *__restrict__ wout) {
    extern __shared__ int2 gq_lds[];
    // GCOL launches hold one instance: its packed entries, read as global
    using GQ = std::conditional_t<GCOL, const SK_GLOBAL int2 *, const int2 *>;
    GQ gq;
    if constexpr (GCOL) gq = (GQ)insts[0].colpack;
    else gq = gq_lds;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int u0, u1;
    unit_range(nunits, u0, u1);
    const int eskip = kept_skip(logt);
    if constexpr (GCOL) {
        if (insts[0].vec8) {
            // the integer test reads G_j from LDS tiles (as the row check);
            // the FP64 test reads (G_j, gam_j) from the packed buffer
            __shared__ int gG[kGTile];
            const Inst &I = insts[0];
            const int n = I.n, ntile = (n + kGTile - 1) / kGTile;
            // the row's state is wave-uniform: kept in scalar registers
            const bool sent = __builtin_amdgcn_readfirstlane(I.ctl->sent) != 0u;
            const int par = __builtin_amdgcn_readfirstlane(I.ctl->iter) & 1;
            const int pi = __builtin_amdgcn_readfirstlane(I.ctl->p);
            const double p = (double)pi;
            for (int u = u0; u < u1; ++u) {
                const int row = __builtin_amdgcn_readfirstlane(units[u].row0 + wave);
                const bool on = row < n;
                const int Fi = on ? __builtin_amdgcn_readfirstlane(I.F[par][row]) : 0;
                const double f = (double)Fi + (double)(on ? rfl_f(I.phi[par][row]) : 0.0f);
                const int16_t *wr = I.W + (int64_t)(on ? row : 0) * I.pitch;
                int64_t pos = on ? rfl_i64(row_ptr[row]) : 0;
                for (int t = 0; t < ntile; ++t) {
                    const int lo = t * kGTile, hi = min(n, lo + kGTile);
                    if (ntile > 1 || u == u0) {
                        __syncthreads();
                        stage_g_tile(I, gG, lo);
                        __syncthreads();
                    }
                    if (!on) continue;
                    auto gs = [&](int c, int j0) { return gG[c * kGT8 + ((j0 - lo) >> 3)]; };
                    fill_row_range<NT, true>(I, gq, gs, wr, lane, lo, hi, pi, p, Fi, f, eskip, logt, sent, pos, col,
                                             wout);
                }
            }
            return;
        }
    }
    int cur = -1;
    for (int u = u0; u < u1; ++u) {
        const RowUnit un = units[u];
        const Inst &I = insts[un.inst];
        if (un.inst != cur) {
            if (!GCOL) {
                __syncthreads();
                stage_gq(I, gq_lds);
                __syncthreads();
            }
            cur = un.inst;
        }
        const int n = I.n, row = un.row0 + wave;
        if (row >= n) continue;
        const int par = I.ctl->iter & 1;
        const int pi = I.ctl->p, Fi = I.F[par][row];
        const double p = (double)pi;
        const double f = (double)Fi + (double)I.phi[par][row];
        const int16_t *wr = I.W + (int64_t)row * I.pitch;
        int64_t pos = row_ptr[row];
        if (I.vec8) {
            const int n8 = pad8(n) >> 3;
            auto gs = [&](int c, int j0) { return gq[c * n8 + (j0 >> 3)].x; };
            fill_row_range<NT, false>(I, gq, gs, wr, lane, 0, n, pi, p, Fi, f, eskip, logt, I.ctl->sent != 0u, pos,
                                      col, wout);
            continue;
        }
        for (int j0 = 0; j0 < n; j0 += kWave) {
            const int j = j0 + lane;
            bool keep = false;
            int w = SK_SENTINEL;
            if (j < n) {
                w = wr[j];
                if (w != SK_SENTINEL) {
                    const int2 q = gq_at(I, gq, j);
                    if (__mul24(pi, w) + q.x + Fi >= eskip) {
                        const double lx = p * (double)w + f + logv_of(q);
                        keep = lx >= logt;
                    }
                }
            }
            const uint64_t mask = __ballot(keep);
            if (keep) {
                const int before = __popcll(mask & ((1ull << lane) - 1ull));
                col[pos + before] = j;
                wout[pos + before] = (int16_t)w;
            }
            pos += __popcll(mask);
        }
    }
}

// ---------------------------------------------------------------- control blocks
// Copies every instance's control block into one contiguous array (one
// device-to-host copy per check instead of one per instance).
__global__ __launch_bounds__(256) void k_gather_ctl(const Inst *__restrict__ insts, int count,
                                                    Ctl *out) {
    const int words = (int)(sizeof(Ctl) / sizeof(uint32_t));
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < count * words;
         q += gridDim.x * blockDim.x) {
        const int k = q / words, w = q % words;
        reinterpret_cast<uint32_t *>(out + k)[w] =
            reinterpret_cast<const volatile uint32_t *>(insts[k].ctl)[w];
    }
}

// Resets the control blocks of instances idx[0..m) (all when idx is null) for a
// cold start at the first p of their ladders.
__global__ __launch_bounds__(256) void k_reset_ctl(const Inst *__restrict__ insts, const int *idx,
                                                   int m) {
    for (int q = blockIdx.x; q < m; q += gridDim.x) {
        const Inst &I = insts[idx ? idx[q] : q];
        for (int q = threadIdx.x; q < kRowResSlots; q += blockDim.x) I.rowres[q * kRowResStride] = 0u;
        if (threadIdx.x == 0) {
            Ctl c;
            memset(&c, 0, sizeof c);
            c.state = ST_RUNNING;
            c.p = I.deform_a > 0.0 ? deform_p(I, 1) : I.ladder[0];
            c.preal = I.deform_a > 0.0 ? deform_p_real(I, 1) : (double)I.ladder[0];
            c.last_res = INFINITY;
            *I.ctl = c;
        }
    }
}

// ---------------------------------------------------------------- Newton scaling
// Products with S = [[0, X], [X^T, 0]] for X = diag(u) A^(p) diag(v) at the
// instance's potentials (fixed during a Newton solve): sd[i] = (X q_c)_i and
// sd[n + j] = (X^T q_r)_j for q = (q_r, q_c), each term formed as in the
// sweeps, exp(E_ij) exp(phi_i) exp(gam_j). One instance (index 0).
template <bool NT>
__global__ __launch_bounds__(kRowWaves * kWave) void k_nt_rows(const Inst *__restrict__ insts,
                                                                 const RowUnit *__restrict__ units,
                                                                 int nunits,
                                                                 const NtCtl *__restrict__ nt,
                                                                 const float *__restrict__ q,
                                                                 float *__restrict__ sd) {
    extern __shared__ ColPot lds_cp[];
    __shared__ float tab[kTabN];
    if (nt->done != NT_RUN) return;
    const Inst &I = insts[0];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int n = I.n, n8 = pad8(n) >> 3;
    const int par = __builtin_amdgcn_readfirstlane(I.ctl->iter) & 1;
    const int p4 = 4 * __builtin_amdgcn_readfirstlane(I.ctl->p);
    const bool sent = __builtin_amdgcn_readfirstlane(I.ctl->sent) != 0u;
    int u0, u1;
    unit_range(nunits, u0, u1);
    // lane l holds F_i, phi_i of the wave's row in unit ubase + l, so that a
    // row starts and ends without waiting on a load of its own
    const SK_GLOBAL int32_t *Fp = (const SK_GLOBAL int32_t *)I.F[par];
    const SK_GLOBAL float *phip = (const SK_GLOBAL float *)I.phi[par];
    int lF = 0, ubase = u0;
    float lphi = 0.f;
    auto window = [&](int ub) {
        ubase = ub;
        const int ul = ub + lane;
        if (ul < u1) {
            const int r = units[ul].row0 + wave;
            if (r < n) {
                lF = Fp[r];
                lphi = phip[r];
            }
        }
    };
    window(u0);
    fill_exp_table(tab);
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        ColPot k;
        k.a = 4 * I.G[j];
        k.g = ex2(I.gam[j] * kLog2e) * q[n + j];
        lds_cp[I.vec8 ? swz8(j, n8) : j] = k;
    }
    stage_pad_cols(I, lds_cp, n8);
    __syncthreads();
    // an empty use: the wait for the window's loads falls here
    asm volatile("" : "+v"(lF), "+v"(lphi));
    for (int u = u0; u < u1; ++u) {
        if (u - ubase >= kWave) {
            window(u);
            asm volatile("" : "+v"(lF), "+v"(lphi));
        }
        const int row = units[u].row0 + wave;
        if (row >= n) continue;
        const int Fi = __builtin_amdgcn_readlane(lF, u - ubase);
        const float phi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lphi), u - ubase));
        const int16_t *wr = I.W + (int64_t)row * I.pitch;
        const int B = 4 * (Fi - kTabLo);
        float S;
        if (I.vec8) S = sent ? row_partial_v8<true, NT>(wr, n, p4, B, lds_cp, tab, lane)
                             : row_partial_v8<false, NT>(wr, n, p4, B, lds_cp, tab, lane);
        else S = sent ? row_partial_v1<true, NT>(wr, n, p4, B, lds_cp, tab, lane)
                      : row_partial_v1<false, NT>(wr, n, p4, B, lds_cp, tab, lane);
        S = wave_sum(S);
        if (lane == 0) sd[row] = ex2(phi * kLog2e) * S;
    }
}

template <bool NT>
__global__ __launch_bounds__(kColWaves * kWave) void k_nt_cols(const Inst *__restrict__ insts,
                                                                 const ColUnit *__restrict__ units,
                                                                 int nunits,
                                                                 const NtCtl *__restrict__ nt,
                                                                 const float *__restrict__ q) {
    __shared__ float red[kColWaves][kColTile8];
    __shared__ RowPot rowpot[kMaxSegRows];
    __shared__ float tab[kTabN];
    if (nt->done != NT_RUN) return;
    const Inst &I = insts[0];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int n = I.n;
    const int par = I.ctl->iter & 1;
    const bool sent = I.ctl->sent != 0u;
    int u0, u1;
    unit_range(nunits, u0, u1);
    fill_exp_table(tab);
    for (int u = u0; u < u1; ++u) {
        const ColUnit un = units[u];
        const int tc = I.tile_cols;
        const int ctile0 = un.tile * tc;
        const int ncols = min(tc, n - ctile0);
        const int r0 = un.seg * I.seg_rows, r1 = min(n, r0 + I.seg_rows);
        __syncthreads();
        for (int r = r0 + (int)threadIdx.x; r < r1; r += blockDim.x) {
            RowPot k;
            k.b = 4 * (I.F[par][r] - kTabLo);
            k.r = ex2(I.phi[par][r] * kLog2e) * q[r];
            rowpot[r - r0] = k;
        }
        __syncthreads();
        const int p4 = 4 * I.ctl->p;
        if (I.vec8) {
            float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            const int c0 = un.tile * kColTile8 + lane * 8;
            if (c0 < n) {
                int A[8];
                int4 first;
                col_tile_start<NT>(I, c0, r0, r1, wave, A, first);
                if (sent) col_partial_v8<true, NT>(I, p4, c0, r0, r1, wave, A, first, rowpot, tab, acc);
                else col_partial_v8<false, NT>(I, p4, c0, r0, r1, wave, A, first, rowpot, tab, acc);
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) red[wave][lane * 8 + c] = acc[c];
        } else {
            float acc;
            if (sent) col_partial_v1<true, NT>(I, p4, un.tile, r0, r1, wave, lane, rowpot, tab, acc);
            else col_partial_v1<false, NT>(I, p4, un.tile, r0, r1, wave, lane, rowpot, tab, acc);
            red[wave][lane] = acc;
        }
        __syncthreads();
        float *dst = I.colpart + (int64_t)un.seg * n + ctile0;
        for (int c = threadIdx.x; c < ncols; c += blockDim.x) {
            float v = red[0][c];
#pragma unroll
            for (int w2 = 1; w2 < kColWaves; ++w2) v += red[w2][c];
            dst[c] = v;
        }
    }
}

// sd[n + j] = exp(gam_j) * sum of the column's slots in segment order.
__global__ __launch_bounds__(256) void k_nt_cols_sum(const Inst *__restrict__ insts,
                                                     const NtCtl *__restrict__ nt,
                                                     float *__restrict__ sd) {
    if (nt->done != NT_RUN) return;
    const Inst &I = insts[0];
    const int n = I.n;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        float v = 0.f;
        for (int s = 0; s < I.nseg; ++s) v += I.colpart[(int64_t)s * n + j];
        sd[n + j] = ex2(I.gam[j] * kLog2e) * v;
    }
}

// Block reductions of the phase kernels (fixed order).
__device__ double nt_bsum(double v, double *sh) {
    v = wave_sum_d(v);
    const int wave = threadIdx.x / kWave;
    __syncthreads();
    if (threadIdx.x % kWave == 0) sh[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w2 = 0; w2 < (int)blockDim.x / kWave; ++w2) t += sh[w2];
    return t;
}
__device__ double nt_bmax(double v, double *sh) {
    v = wave_max_d(v);
    const int wave = threadIdx.x / kWave;
    __syncthreads();
    if (threadIdx.x % kWave == 0) sh[wave] = v;
    __syncthreads();
    double t = -INFINITY;
    for (int w2 = 0; w2 < (int)blockDim.x / kWave; ++w2) t = fmax(t, sh[w2]);
    return t;
}
// Reductions over the workgroups' partials of a phase: thread g loads the
// partial of workgroup g and the block reduces them in a fixed tree, the same
// in every workgroup, so all of them see the same scalars. Called by every
// thread of the block.
__device__ double nt_gsum(const double *part, int slot, double *sh) {
    const int g = threadIdx.x;
    return nt_bsum(g < (int)gridDim.x ? part[g * 4 + slot] : 0.0, sh);
}
__device__ double nt_gmax(const double *part, int slot, double *sh) {
    const int g = threadIdx.x;
    return nt_bmax(g < (int)gridDim.x ? part[g * 4 + slot] : -INFINITY, sh);
}
__device__ double nt_gmin(const double *part, int slot, double *sh) {
    return -nt_bmax(threadIdx.x < gridDim.x ? -part[threadIdx.x * 4 + slot] : -INFINITY, sh);
}

// One phase of a step of the Newton / conjugate-gradient iteration, after
// the product sd of the vector q it asked for. Four phases per step, each a
// grid-wide pass over the 2n-vectors that ends in per-workgroup partials;
// the next phase reduces them in a fixed order. Workgroup 0 alone writes
// the control block, which later phases (next launches) read.
//   NT_OUTER (sd = S x): 1. v = x o S x, r = 1 - v, |r|_2^2, max |r_i|;
//     2. stop if max |r_i| <= tol; forcing term eta; start an inner solve
//     of (D(x) S D(x) + D(v)) y = 1 + v at y = 1 with the preconditioner
//     D(v): z = r / v, d = z, q = x o d, r . z;  3. rho;  4. next product
//     S q (the mode changes only in phase 4, for every step).
//   NT_INNER (sd = S (x o d)): 1. w = x o sd + v o d, d . w;  2. alpha,
//     the extremes of y + alpha d;  3. a step that takes y to or past lo
//     (hi) is cut at that bound (its factor reduced here), else the CG
//     update of y, r, z and r . z;  4. cut: y += gamma alpha d and the
//     inner solve ends; else rho, and the solve ends below the inner
//     tolerance (x <- x o y, next product S x) or continues with
//     d = z + beta d (next product S (x o d)).
__device__ void nt_phase_body(const Inst *__restrict__ insts, const NtCtl &c, NtCtl &u, NtVec V,
                              int phase, double *sh) {
    const int n2 = 2 * insts[0].n;
    const int G = gridDim.x, gid = blockIdx.x, t = threadIdx.x;
    const int i0 = gid * kNtThreads + t, stride = G * kNtThreads;
    const double *prev = V.parts + (size_t)(phase - 1) * kNtMaxGroups * 4;
    double *mine = V.parts + (size_t)phase * kNtMaxGroups * 4 + gid * 4;
    const float lo = (float)c.lo, hi = (float)c.hi;
    if (c.mode == NT_OUTER) {
        if (phase == 1) {
            double rr = 0.0, rinf = 0.0;
            for (int i = i0; i < n2; i += stride) {
                const float v = V.x[i] * V.sd[i];
                const float r = 1.f - v;
                V.v[i] = v;
                V.r[i] = r;
                rr += (double)r * r;
                rinf = fmax(rinf, (double)fabsf(r));
            }
            rr = nt_bsum(rr, sh);
            rinf = nt_bmax(rinf, sh);
            if (t == 0) {
                mine[0] = rr;
                mine[1] = rinf;
            }
        } else if (phase == 2) {
            const double rout = nt_gsum(prev, 0, sh), resinf = nt_gmax(prev, 1, sh);
            const int64_t products = c.products + 1;
            double eta = c.eta;
            if (!c.first) {
                const double eta_prev = c.eta;
                eta = c.g * (rout / c.rold);
                if (c.g * eta_prev * eta_prev > 0.1) eta = fmax(eta, c.g * eta_prev * eta_prev);
                eta = fmax(fmin(eta, c.eta_max), 0.5 * c.tol / fmax(sqrt(rout), 1e-300));
            }
            int done = NT_RUN;
            if (resinf <= c.tol) done = NT_CONVERGED;
            else if (!(rout < INFINITY)) done = NT_FAILED;
            else if (products >= c.max_products) done = NT_CAPPED;
            u.products = products;
            u.eta = eta;
            u.first = 0;
            u.rold = rout;
            u.rout = rout;
            u.resinf = resinf;
            u.done = done;
            u.inner_tol = fmax(eta * eta * rout, c.tol * c.tol);
            if (done != NT_RUN) return;
            double rz = 0.0;
            for (int i = i0; i < n2; i += stride) {
                const float z = V.r[i] / V.v[i];
                V.y[i] = 1.f;
                V.z[i] = z;
                V.d[i] = z;
                V.q[i] = V.x[i] * z;
                rz += (double)V.r[i] * z;
            }
            rz = nt_bsum(rz, sh);
            if (t == 0) mine[0] = rz;
        } else if (phase == 3) {
            u.rho = nt_gsum(prev, 0, sh);
        } else {
            // the mode changes only in the last phase of a step
            u.mode = NT_INNER;
        }
        return;
    }
    // NT_INNER
    const double *p1 = V.parts + (size_t)1 * kNtMaxGroups * 4;
    const double *p2 = V.parts + (size_t)2 * kNtMaxGroups * 4;
    const double *p3 = V.parts + (size_t)3 * kNtMaxGroups * 4;
    if (phase == 1) {
        double dw = 0.0;
        for (int i = i0; i < n2; i += stride) {
            const float w = V.x[i] * V.sd[i] + V.v[i] * V.d[i];
            V.w[i] = w;
            dw += (double)V.d[i] * w;
        }
        dw = nt_bsum(dw, sh);
        if (t == 0) mine[0] = dw;
        return;
    }
    const double dsum = nt_gsum(p1, 0, sh);
    const float alpha = (float)(c.rho / dsum);
    if (phase == 2) {
        double mn = INFINITY, mx = -INFINITY;
        for (int i = i0; i < n2; i += stride) {
            const float yn = V.y[i] + alpha * V.d[i];
            mn = fmin(mn, (double)yn);
            mx = fmax(mx, (double)yn);
        }
        mn = -nt_bmax(-mn, sh);
        mx = nt_bmax(mx, sh);
        if (t == 0) {
            mine[0] = mn;
            mine[1] = mx;
        }
        return;
    }
    const double gmn = nt_gmin(p2, 0, sh);
    const double gmx = nt_gmax(p2, 1, sh);
    const bool failed = !(dsum > 0.0) || !(gmn == gmn);
    const bool cut = !failed && ((float)gmn <= lo || (float)gmx >= hi);
    if (phase == 3) {
        if (failed) {
            u.done = NT_FAILED;
            return;
        }
        if (cut) {
            // the step's largest fraction that keeps y inside (lo, hi)
            double gm = INFINITY;
            for (int i = i0; i < n2; i += stride) {
                const float st = alpha * V.d[i];
                if ((float)gmn <= lo) {
                    if (st < 0.f) gm = fmin(gm, (double)((lo - V.y[i]) / st));
                } else if (V.y[i] + st > hi) {
                    gm = fmin(gm, (double)((hi - V.y[i]) / st));
                }
            }
            gm = -nt_bmax(-gm, sh);
            if (t == 0) mine[0] = gm;
        } else {
            double rz = 0.0;
            for (int i = i0; i < n2; i += stride) {
                V.y[i] += alpha * V.d[i];
                const float r = V.r[i] - alpha * V.w[i];
                const float z = r / V.v[i];
                V.r[i] = r;
                V.z[i] = z;
                rz += (double)r * z;
            }
            rz = nt_bsum(rz, sh);
            if (t == 0) mine[0] = rz;
        }
        return;
    }
    // phase 4
    if (cut) {
        const double gm = nt_gmin(p3, 0, sh);
        const float f = gm < INFINITY ? (float)gm : 1.f;  // reached the bound exactly: full step
        for (int i = i0; i < n2; i += stride) {
            const float x = V.x[i] * (V.y[i] + f * alpha * V.d[i]);
            V.x[i] = x;
            V.q[i] = x;
        }
        u.products = c.products + 1;
        u.mode = NT_OUTER;
        u.outer = c.outer + 1;
        return;
    }
    const double rho = nt_gsum(p3, 0, sh);
    const bool end = !(rho > c.inner_tol) || c.products + 1 >= c.max_products;
    if (end) {
        for (int i = i0; i < n2; i += stride) {
            const float x = V.x[i] * V.y[i];
            V.x[i] = x;
            V.q[i] = x;
        }
    } else {
        const float beta = (float)(rho / c.rho);
        for (int i = i0; i < n2; i += stride) {
            const float d = V.z[i] + beta * V.d[i];
            V.d[i] = d;
            V.q[i] = V.x[i] * d;
        }
    }
    u.products = c.products + 1;
    u.rho_prev = c.rho;
    u.rho = rho;
    if (end) {
        u.mode = NT_OUTER;
        u.outer = c.outer + 1;
    }
}

// The control block is double-buffered by phase parity: a phase reads
// nt[phase & 1] and workgroup 0 writes the whole updated state to the other
// copy, so no workgroup of a launch can see a state written in that launch.
// After phase 4 (and for the product kernels and the host) the current state
// is nt[1].
__global__ __launch_bounds__(kNtThreads) void k_nt_phase(const Inst *__restrict__ insts, NtCtl *nt,
                                                         NtVec V, int phase) {
    __shared__ double sh[kNtThreads / kWave];
    const NtCtl c = nt[phase & 1];
    NtCtl u = c;
    if (c.done == NT_RUN) nt_phase_body(insts, c, u, V, phase, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) nt[(phase + 1) & 1] = u;
}

// Folds the Newton scalings into the potentials: log u_i += log x_i,
// log v_j += log x_{n+j} (FP64, re-split into integer and fraction), and
// ends the stage for the host.
__global__ __launch_bounds__(256) void k_nt_fold(const Inst *__restrict__ insts,
                                                 const NtCtl *__restrict__ nt,
                                                 const float *__restrict__ x, int last) {
    const Inst &I = insts[0];
    Ctl *ctl = I.ctl;
    const int n = I.n;
    const int par = ctl->iter & 1;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double f = (double)I.F[par][i] + (double)I.phi[par][i] + log((double)x[i]);
        const double k = rint(f);
        I.F[par][i] = (int32_t)k;
        I.phi[par][i] = (float)(f - k);
        const double g = (double)I.G[i] + (double)I.gam[i] + log((double)x[n + i]);
        const double kg = rint(g);
        I.G[i] = (int32_t)kg;
        I.gam[i] = (float)(g - kg);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const NtCtl c = *nt;
        ctl->stage_iters[ctl->stage] = c.products;
        ctl->iters_total += c.products;
        ctl->last_res = (float)c.resinf;
        if (c.done == NT_CAPPED) ctl->capped += 1;
        if (c.done == NT_FAILED) ctl->err |= ERR_NEWTON;
        ctl->state = c.done == NT_FAILED ? ST_ERROR : (last ? ST_DONE : ST_STAGE_END);
    }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_gather_ctl(const Inst *d_insts, int count, Ctl *out, hipStream_t st) {
    const int words = count * (int)(sizeof(Ctl) / sizeof(uint32_t));
    hipLaunchKernelGGL(k_gather_ctl, dim3(std::min(1024, (words + 255) / 256)), dim3(256), 0, st,
                       d_insts, count, out);
    return hipGetLastError();
}
hipError_t launch_reset_ctl(const Inst *d_insts, const int *idx, int m, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_ctl, dim3(std::min(m, 1024)), dim3(256), 0, st, d_insts, idx, m);
    return hipGetLastError();
}
hipError_t launch_init(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid, int cold,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_init, dim3(grid), dim3(kRowWaves * kWave), 0, st, d_insts, d_units,
                       nunits, cold);
    return hipGetLastError();
}
hipError_t launch_pad_copy(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_pad_copy, dim3(grid), dim3(kRowWaves * kWave), 0, st, d_insts, d_units,
                       nunits);
    return hipGetLastError();
}
hipError_t launch_row_sweep(const Inst *d_insts, const RowUnit *d_units, int nunits,
                            const int32_t *bounds, int grid, size_t lds_bytes, int nt_loads,
                            int short_rows, int gcol, hipStream_t st, hipEvent_t stop) {
    if (short_rows)
        return launch_row_sweep_short(d_insts, d_units, nunits, bounds, grid, lds_bytes, nt_loads, st,
                                      stop);
    if (gcol)
        launch_stamped(k_row_sweep<true, 1, true>, dim3(grid), dim3(kRowWaves * kWave), 0, st, stop, d_insts,
                       d_units, nunits, bounds);
    else if (nt_loads)
        launch_stamped(k_row_sweep<true, 1, false>, dim3(grid), dim3(kRowWaves * kWave), lds_bytes, st, stop,
                       d_insts, d_units, nunits, bounds);
    else
        launch_stamped(k_row_sweep<false, 1, false>, dim3(grid), dim3(kRowWaves * kWave), lds_bytes, st, stop,
                       d_insts, d_units, nunits, bounds);
    return hipGetLastError();
}
hipError_t launch_col_sweep(const Inst *d_insts, const ColUnit *d_units, int nunits, int grid,
                            int nt_loads, int short_rows, hipStream_t st, hipEvent_t stop) {
    if (short_rows) {
        if (nt_loads)
            launch_stamped(k_col_sweep<true, false>, dim3(grid), dim3(kColWaves * kWave), 0, st, stop, d_insts,
                           d_units, nunits);
        else
            launch_stamped(k_col_sweep<false, false>, dim3(grid), dim3(kColWaves * kWave), 0, st, stop, d_insts,
                           d_units, nunits);
    } else if (nt_loads) {
        launch_stamped(k_col_sweep<true, true>, dim3(grid), dim3(kColWaves * kWave), 0, st, stop, d_insts,
                       d_units, nunits);
    } else {
        launch_stamped(k_col_sweep<false, true>, dim3(grid), dim3(kColWaves * kWave), 0, st, stop, d_insts,
                       d_units, nunits);
    }
    return hipGetLastError();
}
hipError_t launch_col_finalize(const Inst *d_insts, const FinUnit *d_units, int nunits, int grid,
                               int mode, hipStream_t st) {
    hipLaunchKernelGGL(k_col_finalize, dim3(grid), dim3(256), 0, st, d_insts, d_units, nunits, mode);
    return hipGetLastError();
}
hipError_t launch_nt_product(const Inst *d_insts, const RowUnit *d_rows, int nrows, int row_grid,
                             size_t row_lds, const ColUnit *d_cols, int ncols, int col_grid,
                             const NtCtl *nt, NtVec vec, int n, int nt_loads, hipStream_t st) {
    const NtCtl *cur = nt + 1;  // the state after the last completed step
    if (nt_loads) {
        hipLaunchKernelGGL(k_nt_rows<true>, dim3(row_grid), dim3(kRowWaves * kWave), row_lds, st,
                           d_insts, d_rows, nrows, cur, vec.q, vec.sd);
        hipLaunchKernelGGL(k_nt_cols<true>, dim3(col_grid), dim3(kColWaves * kWave), 0, st, d_insts,
                           d_cols, ncols, cur, vec.q);
    } else {
        hipLaunchKernelGGL(k_nt_rows<false>, dim3(row_grid), dim3(kRowWaves * kWave), row_lds, st,
                           d_insts, d_rows, nrows, cur, vec.q, vec.sd);
        hipLaunchKernelGGL(k_nt_cols<false>, dim3(col_grid), dim3(kColWaves * kWave), 0, st, d_insts,
                           d_cols, ncols, cur, vec.q);
    }
    hipLaunchKernelGGL(k_nt_cols_sum, dim3((n + 255) / 256), dim3(256), 0, st, d_insts, cur, vec.sd);
    return hipGetLastError();
}
hipError_t launch_nt_step(const Inst *d_insts, NtCtl *nt, NtVec vec, int n, hipStream_t st) {
    const int groups = std::max(1, std::min(kNtMaxGroups, (2 * n + 2 * kNtThreads - 1) / (2 * kNtThreads)));
    for (int ph = 1; ph <= kNtPhases; ++ph)
        hipLaunchKernelGGL(k_nt_phase, dim3(groups), dim3(kNtThreads), 0, st, d_insts, nt, vec, ph);
    return hipGetLastError();
}
hipError_t launch_nt_fold(const Inst *d_insts, const NtCtl *nt, NtVec vec, int n, int last,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_nt_fold, dim3((n + 255) / 256), dim3(256), 0, st, d_insts, nt + 1, vec.x,
                       last);
    return hipGetLastError();
}
hipError_t launch_iter_end(const Inst *d_insts, int count, hipStream_t st, hipEvent_t stop) {
    launch_stamped(k_iter_end, dim3(count), dim3(kIterEndThreads), 0, st, stop, d_insts);
    return hipGetLastError();
}
hipError_t launch_check_rows(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid,
                             double *rsum, double *rmax, double logt, int64_t *counts,
                             int32_t *hint, size_t lds_bytes, int nt_loads, int gcol, hipStream_t st) {
    const dim3 g(grid), b(kRowWaves * kWave);
    if (gcol)
        hipLaunchKernelGGL((k_check_rows<true, true>), g, b, 0, st, d_insts, d_units, nunits, rsum, rmax, logt,
                           counts, hint);
    else if (nt_loads)
        hipLaunchKernelGGL((k_check_rows<true, false>), g, b, lds_bytes, st, d_insts, d_units, nunits, rsum,
                           rmax, logt, counts, hint);
    else
        hipLaunchKernelGGL((k_check_rows<false, false>), g, b, lds_bytes, st, d_insts, d_units, nunits, rsum,
                           rmax, logt, counts, hint);
    return hipGetLastError();
}
hipError_t launch_col_pack(const Inst *d_insts, int inst, int n, int mode, hipStream_t st) {
    hipLaunchKernelGGL(k_col_pack, dim3((pad8(n) + 255) / 256), dim3(256), 0, st, d_insts, inst, mode);
    return hipGetLastError();
}
hipError_t launch_check_reduce(const Inst *d_insts, int inst, const double *rsum,
                               const double *rmax, const double *csum, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_check_reduce, dim3(1), dim3(256), 0, st, d_insts, inst, rsum, rmax, csum, out);
    return hipGetLastError();
}
hipError_t launch_check_cols(const Inst *d_insts, int inst, int n, int nseg, int vec8,
                             double *part, double *csum, int nt_loads, hipStream_t st) {
    if (vec8 && nt_loads)
        hipLaunchKernelGGL(k_check_cols_part8<true>, dim3((n + kColTile8 - 1) / kColTile8, nseg),
                           dim3(kColWaves * kWave), 0, st, d_insts, inst, part);
    else if (vec8)
        hipLaunchKernelGGL(k_check_cols_part8<false>, dim3((n + kColTile8 - 1) / kColTile8, nseg),
                           dim3(kColWaves * kWave), 0, st, d_insts, inst, part);
    else
        hipLaunchKernelGGL(k_check_cols_part, dim3((n + 255) / 256, nseg), dim3(256), 0, st, d_insts,
                           inst, part);
    hipLaunchKernelGGL(k_check_cols_sum, dim3((n + 255) / 256), dim3(256), 0, st, d_insts, inst,
                       part, csum);
    return hipGetLastError();
}
hipError_t launch_prune_count(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid,
                              double logt, int64_t *counts, size_t lds_bytes, int nt_loads, int gcol,
                              hipStream_t st) {
    const dim3 g(grid), b(kRowWaves * kWave);
    if (gcol)
        hipLaunchKernelGGL((k_prune_count<true, true>), g, b, 0, st, d_insts, d_units, nunits, logt, counts);
    else if (nt_loads)
        hipLaunchKernelGGL((k_prune_count<true, false>), g, b, lds_bytes, st, d_insts, d_units, nunits, logt,
                           counts);
    else
        hipLaunchKernelGGL((k_prune_count<false, false>), g, b, lds_bytes, st, d_insts, d_units, nunits, logt,
                           counts);
    return hipGetLastError();
}
hipError_t launch_scan(const int64_t *counts, int64_t *row_ptr, int n, hipStream_t st,
                       int64_t *total_out) {
    if (n < 0 || n > kMaxN) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, counts, row_ptr, n, total_out);
    return hipGetLastError();
}
hipError_t launch_prune_fill(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid,
                             double logt, const int64_t *row_ptr, int32_t *col, int16_t *w,
                             size_t lds_bytes, int nt_loads, int gcol, hipStream_t st) {
    const dim3 g(grid), b(kRowWaves * kWave);
    if (gcol)
        hipLaunchKernelGGL((k_prune_fill<true, true>), g, b, 0, st, d_insts, d_units, nunits, logt, row_ptr,
                           col, w);
    else if (nt_loads)
        hipLaunchKernelGGL((k_prune_fill<true, false>), g, b, lds_bytes, st, d_insts, d_units, nunits, logt,
                           row_ptr, col, w);
    else
        hipLaunchKernelGGL((k_prune_fill<false, false>), g, b, lds_bytes, st, d_insts, d_units, nunits, logt,
                           row_ptr, col, w);
    return hipGetLastError();
}
hipError_t set_kernel_attributes() {
    const int lds = (int)(kLdsMaxN * sizeof(double));
    hipError_t e;
    if ((e = set_row_sweep_short_attributes()) != hipSuccess) return e;
    for (const void *f : {(const void *)k_row_sweep<true, 1, false>, (const void *)k_row_sweep<false, 1, false>,
                          (const void *)k_nt_rows<true>, (const void *)k_nt_rows<false>})
        if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds)) != hipSuccess)
            return e;
    for (const void *f : {(const void *)k_check_rows<true, false>, (const void *)k_check_rows<false, false>,
                          (const void *)k_prune_count<true, false>, (const void *)k_prune_count<false, false>,
                          (const void *)k_prune_fill<true, false>, (const void *)k_prune_fill<false, false>})
        if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds)) != hipSuccess)
            return e;
    return hipSuccess;
}

}  // namespace sk
