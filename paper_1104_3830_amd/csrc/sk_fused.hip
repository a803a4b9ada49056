// Single-pass Sinkhorn iteration: one read of the matrix per iteration.
//
// A workgroup of 1024 threads owns a contiguous block of rows and every
// column; thread t owns the 8-column chunks t, t + 1024 (n <= 16384). For
// each group of rows it
//   A. forms the terms of its columns and reduces the row sums S_i across the
//      workgroup (the row step, eq. dad2: log u_i <- F_i - log S_i, resp.
//      a_i <- 1 / S_i);
//   B. adds the terms divided by S_i into per-thread column accumulators: this
//      is the column sum of the new row-stochastic iterate.
// int16 W: the term is exp(E_ij) exp(gam_j) with the exact integer exponent
// E_ij = p w_ij + F_i + G_j read from the LDS table; exp(gam_j) is constant
// per column, so the accumulators hold sum_i exp(E_ij) / S_i and are scaled
// by exp(gam_j) once at the end. Stored K: the term is K_ij b_j.
// The accumulators go to fixed slots colpart[workgroup][j]; the finalise
// kernel adds the slots of each column in workgroup order (deterministic) and
// applies the column step (eq. dad3). The result equals a row sweep followed
// by a column sweep, with half the matrix traffic.
#include "sk_exptab.h"
#include "sk_runtime.h"

namespace sk {

constexpr int kFT = 1024;    // threads per workgroup
constexpr int kFR = 2;       // rows per group
// rows per workgroup at most: ceil(n / grid) with n <= kLdsMaxN (the single
// pass takes no larger instance) and a grid of
// min(kFusedSlots, max(1, n / 2)) workgroups (64 at n = 16384, at most 3 for
// n below 2 kFusedSlots)
constexpr int kFusedRows = (kLdsMaxN + kFusedSlots - 1) / kFusedSlots;
constexpr float kL2e = 1.4426950408889634f;
constexpr float kLn2f = 0.6931471805599453f;
constexpr float kLo = 5.421010862427522e-20f;  // 2^-64
constexpr float kHi = 1.8446744073709552e19f;  // 2^64

__device__ __forceinline__ float fex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float flg2(float x) { return __builtin_amdgcn_logf(x); }

// ---------------------------------------------------------------- int16 W
// Sums across lanes with DPP moves in a fixed order (deterministic, no LDS
// round trip): after dpp_sum16 every lane of a 16-lane row holds the row's
// sum, bitwise equal in all of them (each step adds two equal-shaped partial
// sums, and float addition is commutative); dpp_wave_sum leaves the
// wavefront's total in lane 63.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ float dppf(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWMASK, 0xf, false));
}
__device__ __forceinline__ float dpp_sum16(float x) {
    x += dppf<0xB1>(x);   // quad_perm [1,0,3,2]
    x += dppf<0x4E>(x);   // quad_perm [2,3,0,1]
    x += dppf<0x141>(x);  // row_half_mirror
    x += dppf<0x140>(x);  // row_mirror
    return x;
}
__device__ __forceinline__ float dpp_wave_sum(float x) {
    x = dpp_sum16(x);
    x += dppf<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
    x += dppf<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

__device__ __forceinline__ int gld(const int32_t *p) { return *(const SK_GLOBAL int32_t *)p; }
__device__ __forceinline__ float gld(const float *p) { return *(const SK_GLOBAL float *)p; }
__device__ __forceinline__ void gst(int32_t *p, int v) { *(SK_GLOBAL int32_t *)p = v; }
__device__ __forceinline__ void gst(float *p, float v) { *(SK_GLOBAL float *)p = v; }

// Sum of the NW per-wave partials in every lane, bitwise equal in all lanes:
// lane l passes partial l mod NW, and DPP adds equal-shaped partial sums.
template <int NW>
__device__ __forceinline__ float sum_partials(float x) {
    static_assert(NW == 8 || NW == 16, "8 or 16 waves per workgroup");
    x += dppf<0xB1>(x);   // quad_perm [1,0,3,2]
    x += dppf<0x4E>(x);   // quad_perm [2,3,0,1]
    x += dppf<0x141>(x);  // row_half_mirror
    if (NW == 16) x += dppf<0x140>(x);  // row_mirror
    return x;
}

// FT threads per workgroup (NW = FT / 64 waves), CPT 8-column chunks per
// thread (thread t owns chunks t, t + FT, ...), FR rows per group. Groups are
// loaded NB - 1 groups ahead into a ring of NB register buffers, so that many
// groups' loads are in flight while one is reduced. One barrier per group:
// the per-wave row partials are double-buffered by group parity and every
// lane forms S_i from the NW partials. The scalar work of row i (its new
// potentials and residual) is done by lane 0 of wave (i - r0) mod NW, so no
// single wave falls behind at every barrier.
template <int FT, int CPT, int FR, int NB, bool SENT, bool NT>
__device__ __forceinline__ void fused_i16_body(const Inst &I, Ctl *ctl, const float *tab,
                                               float (*red)[FT / kWave][kFR], int *redm,
                                               float *reds, float *wres, int2 *gc, int *sF,
                                               float *sphi) {
    constexpr int NW = FT / kWave;
    const int n = I.n;
    const int t = threadIdx.x, wave = t / kWave, lane = t % kWave;
    const int par = ctl->iter & 1;
    const int p4 = 4 * ctl->p;
    const int per = (n + (int)gridDim.x - 1) / (int)gridDim.x;
    const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
    const int16_t *W = I.W;
    const int64_t pitch = I.pitch;
    const int32_t *Fp = I.F[par];
    int32_t *Fn = I.F[par ^ 1];
    const float *phip = I.phi[par];
    float *phin_p = I.phi[par ^ 1];
    int c0[CPT];
    bool own[CPT];
    // per owned column (4 G_j, exp(gam_j)) in one 8-byte LDS word at
    // gc[(k * 8 + c) * FT + t] (the lanes of a wave read consecutive words),
    // which leaves the registers to the terms of FR rows
    float acc[CPT][8];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        c0[k] = (t + k * FT) * 8;
        own[k] = c0[k] < n;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            gc[(k * 8 + c) * FT + t] =
                own[k] ? make_int2(4 * gld(I.G + c0[k] + c), __float_as_int(fex2(gld(I.gam + c0[k] + c) * kL2e)))
                       : make_int2(0, 0);
            acc[k][c] = 0.f;
        }
    }
    // F_i and phi_i of the block's rows in LDS: read from LDS while the
    // rows' loads are in flight (a vector load here would be counted behind
    // them and wait for all of them)
    for (int r = r0 + t; r < r1; r += FT) {
        sF[r - r0] = gld(Fp + r);
        sphi[r - r0] = gld(phip + r);
    }
    __syncthreads();
    float resmax = 0.f;
    int4 buf[NB][FR][CPT];
    auto load_group = [&](int4 (&bf)[FR][CPT], int rb) {
#pragma unroll
        for (int rr = 0; rr < FR; ++rr)
#pragma unroll
            for (int k = 0; k < CPT; ++k)
                bf[rr][k] = (rb + rr < r1 && own[k])
                                ? gload<NT>(reinterpret_cast<const int4 *>(W + (int64_t)(rb + rr) * pitch + c0[k]))
                                : make_int4(0, 0, 0, 0);
    };
    int parity = 0;
    auto process = [&](const int4 (&cur)[FR][CPT], int rb) {
        // A: exp(E_ij) per owned column and the row partials
        float T[FR][CPT][8];
        float part[FR];
        int Fi[FR];
#pragma unroll
        for (int rr = 0; rr < FR; ++rr) {
            const int row = rb + rr;
            Fi[rr] = row < r1 ? sF[row - r0] : 0;
            const int B = 4 * (Fi[rr] - kTabLo);
            part[rr] = 0.f;
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                // T of rows past r1 or of columns past n is never read
                if (row < r1 && own[k]) {
                    int w[8];
                    unpack8i(cur[rr][k], w);
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const int2 ag = gc[(k * 8 + c) * FT + t];
                        float e = tab_at(tab, tab_off(p4, w[c], ag.x, B));
                        if (SENT) e = (w[c] == SK_SENTINEL) ? 0.f : e;
                        T[rr][k][c] = e;
                        part[rr] = fmaf(e, __int_as_float(ag.y), part[rr]);
                    }
                }
            }
        }
#pragma unroll
        for (int rr = 0; rr < FR; ++rr) {
            const float v = dpp_wave_sum(part[rr]);
            if (lane == 0) red[parity][wave][rr] = v;
        }
        __syncthreads();
        float inv[FR];
#pragma unroll
        for (int rr = 0; rr < FR; ++rr) {
            const int row = rb + rr;
            const float S = sum_partials<NW>(red[parity][lane & (NW - 1)][rr]);
            inv[rr] = 0.f;
            if (row >= r1) continue;  // uniform
            const bool writer = t == ((row - r0) % NW) * kWave;
            if (S >= kLo && S <= kHi) {
                inv[rr] = __builtin_amdgcn_rcpf(S);
                if (writer) {
                    // log u_i <- F_i - log S_i; r_i = exp(phi_i) S_i
                    const float l2S = flg2(S);
                    const float phin = -l2S * kLn2f;
                    const float kk = rintf(phin);
                    gst(Fn + row, Fi[rr] + (int)kk);
                    gst(phin_p + row, phin - kk);
                    const float r = fex2(fmaf(sphi[row - r0], kL2e, l2S));
                    resmax = fmaxf(resmax, fabsf(r - 1.f));
                }
                continue;
            }
            // exact max shift (Section 4.1.2), uniform across the workgroup:
            // M = max_j (p w_ij + F_i + G_j), then the sum with E - M
            int m4 = INT_MIN;
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                if (!own[k]) continue;
                int w[8];
                unpack8i(cur[rr][k], w);
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    if (!SENT || w[c] != SK_SENTINEL)
                        m4 = max(m4, __mul24(p4, w[c]) + gc[(k * 8 + c) * FT + t].x + 4 * Fi[rr]);
            }
            m4 = wave_max_i(m4);
            if (lane == 0) redm[wave] = m4;
            __syncthreads();
            int mm = INT_MIN;
            for (int w2 = 0; w2 < NW; ++w2) mm = max(mm, redm[w2]);
            const int M = mm >> 2;  // exact: a multiple of 4 (unused if mm == INT_MIN)
            float s2 = 0.f;
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                if (!own[k]) continue;
                int w[8];
                unpack8i(cur[rr][k], w);
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int2 ag = gc[(k * 8 + c) * FT + t];
                    float e = mm == INT_MIN ? 0.f
                                            : tab_at(tab, tab_off(p4, w[c], ag.x, 4 * (Fi[rr] - M - kTabLo)));
                    if (SENT) e = (w[c] == SK_SENTINEL) ? 0.f : e;
                    T[rr][k][c] = e;
                    s2 = fmaf(e, __int_as_float(ag.y), s2);
                }
            }
            s2 = dpp_wave_sum(s2);
            if (lane == 0) reds[wave] = s2;
            __syncthreads();
            float S2 = 0.f;
            for (int w2 = 0; w2 < NW; ++w2) S2 += reds[w2];
            if (mm == INT_MIN) {
                if (t == 0) atomicOr(&ctl->err, ERR_EMPTY_ROW);
            } else {
                inv[rr] = __builtin_amdgcn_rcpf(S2);
                if (writer) {
                    const float l2S = flg2(S2);
                    const float phin = -l2S * kLn2f;
                    const float kk = rintf(phin);
                    gst(Fn + row, Fi[rr] - M + (int)kk);
                    gst(phin_p + row, phin - kk);
                    const float r = fex2(fmaf(sphi[row - r0] + (float)M, kL2e, l2S));
                    resmax = fmaxf(resmax, fabsf(r - 1.f));
                }
            }
            __syncthreads();  // redm / reds are reused by the next such row
        }
        // B: column sums of the new row-stochastic iterate (times exp(-gam_j))
#pragma unroll
        for (int rr = 0; rr < FR; ++rr) {
            if (rb + rr >= r1) continue;  // uniform
#pragma unroll
            for (int k = 0; k < CPT; ++k)
                if (own[k]) {
#pragma unroll
                    for (int c = 0; c < 8; ++c) acc[k][c] = fmaf(T[rr][k][c], inv[rr], acc[k][c]);
                }
        }
        parity ^= 1;
    };
    // ring of NB buffers: group g lives in buf[g mod NB]; while group g is
    // reduced, groups g+1 .. g+NB-1 are loading
#pragma unroll
    for (int b = 0; b < NB - 1; ++b)
        if (r0 + b * FR < r1) load_group(buf[b], r0 + b * FR);
    for (int rb = r0; rb < r1; rb += NB * FR) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int rc = rb + b * FR;
            if (rc >= r1) break;  // uniform
            const int rn = rc + (NB - 1) * FR;
            if (rn < r1) load_group(buf[(b + NB - 1) % NB], rn);
            process(buf[b], rc);
        }
    }
    float *dst = I.colpart + (int64_t)blockIdx.x * n;
#pragma unroll
    for (int k = 0; k < CPT; ++k)
        if (own[k]) {
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (c0[k] + c < n) gst(dst + c0[k] + c, acc[k][c] * __int_as_float(gc[(k * 8 + c) * FT + t].y));
        }
    // residual slot of this workgroup: lane 0 of every wave formed the
    // residuals of its rows
    if (lane == 0) wres[wave] = resmax;
    __syncthreads();
    if (t == 0) {
        float m = 0.f;
        for (int w2 = 0; w2 < NW; ++w2) m = fmaxf(m, wres[w2]);
        I.res_slots[blockIdx.x] = m;
    }
}

// Two shapes, both 1024 threads (four waves per SIMD, 128 VGPRs): n <= 8192
// takes one chunk per thread and two rows per group, one group ahead; larger
// n two chunks per thread and one row per group, two rows ahead (12 bytes
// of spill). Measured at n = 16384: with the row potentials read from global
// memory per row instead of LDS, 150.5 us; one row ahead 143.0 us, two rows
// ahead 134.0 us; two rows per group (fewer barriers, more spill) 142.1 us;
// 512 threads with four chunks each (two waves per SIMD, 238 VGPRs, up to
// three rows ahead) 160-163 us at every depth.
constexpr int kFusedAhead = 2;
template <int FT, int CPT, int FR, int NB, bool NT>
__global__ __launch_bounds__(FT) void k_fused_i16(const Inst *__restrict__ insts, int inst) {
    __shared__ int sF[kFusedRows];
    __shared__ float sphi[kFusedRows];
    __shared__ float tab[kTabN];
    __shared__ float red[2][FT / kWave][kFR];
    __shared__ int redm[FT / kWave];
    __shared__ float reds[FT / kWave];
    __shared__ float wres[FT / kWave];
    __shared__ int2 gc[CPT * 8 * FT];
    const Inst &I = insts[inst];
    Ctl *ctl = I.ctl;
    if (ctl->state != ST_RUNNING) return;
    fill_exp_table(tab);
    __syncthreads();
    if (ctl->sent != 0u) fused_i16_body<FT, CPT, FR, NB, true, NT>(I, ctl, tab, red, redm, reds, wres, gc, sF, sphi);
    else fused_i16_body<FT, CPT, FR, NB, false, NT>(I, ctl, tab, red, redm, reds, wres, gc, sF, sphi);
}

// ---------------------------------------------------------------- stored K
// Raw words of one 8-entry chunk of K: BF16 (one 16-byte load) or F32 (two).
template <int ST>
struct KChunk {
    int4 v[ST == SK_K_F32 ? 2 : 1];
};
template <int ST, bool NT>
__device__ __forceinline__ KChunk<ST> kload(const void *K, int64_t off) {
    KChunk<ST> ch;
    if (ST == SK_K_BF16) {
        ch.v[0] = gload<NT>(reinterpret_cast<const int4 *>(reinterpret_cast<const uint16_t *>(K) + off));
    } else {
        const int4 *q = reinterpret_cast<const int4 *>(reinterpret_cast<const float *>(K) + off);
        ch.v[0] = gload<NT>(q);
        ch.v[1] = gload<NT>(q + 1);
    }
    return ch;
}
template <int ST>
__device__ __forceinline__ void kunpack(const KChunk<ST> &ch, float (&x)[8]) {
    if (ST == SK_K_BF16) {
        const uint32_t q[4] = {(uint32_t)ch.v[0].x, (uint32_t)ch.v[0].y, (uint32_t)ch.v[0].z, (uint32_t)ch.v[0].w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            x[2 * k] = __uint_as_float(q[k] << 16);
            x[2 * k + 1] = __uint_as_float(q[k] & 0xffff0000u);
        }
    } else {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            x[4 * h] = __int_as_float(ch.v[h].x);
            x[4 * h + 1] = __int_as_float(ch.v[h].y);
            x[4 * h + 2] = __int_as_float(ch.v[h].z);
            x[4 * h + 3] = __int_as_float(ch.v[h].w);
        }
    }
}

// Stored K: the row step a_i <- 1 / sum_j K_ij b_j (clamped to [2^-64, 2^64])
// and the column sums sum_i K_ij a_i of the new iterate, times b_j at the
// end. The raw K of a row stays in registers from its row sum to its column
// update (one unpack and one FMA per entry in each), so no terms are kept and
// NB - 1 rows are loading while one is reduced. a_i of the block's rows is
// staged in LDS (a vector load per row would wait behind the rows' loads).
template <int ST, int CPT, int FR, int NB, bool NT>
__global__ __launch_bounds__(kFT) void k_fused(const Inst *__restrict__ insts, int inst) {
    constexpr int NW = kFT / kWave;
    __shared__ float red[2][NW][FR];
    __shared__ float sa[kFusedRows];
    __shared__ float wres[2][NW];
    const Inst &I = insts[inst];
    Ctl *ctl = I.ctl;
    if (ctl->state != ST_RUNNING || ctl->need_absorb) return;
    const int n = I.n;
    const int t = threadIdx.x, wave = t / kWave, lane = t % kWave;
    const int par = ctl->iter & 1;
    const int64_t pitch = I.kpitch;
    const void *K = I.K;
    const int per = (n + (int)gridDim.x - 1) / (int)gridDim.x;
    const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
    int c0[CPT];
    bool own[CPT];
    float bj[CPT][8], acc[CPT][8];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        c0[k] = (t + k * kFT) * 8;
        own[k] = c0[k] < n;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            acc[k][c] = 0.f;
            bj[k][c] = own[k] && c0[k] + c < n ? gld(I.b + c0[k] + c) : 0.f;
        }
    }
    for (int r = r0 + t; r < r1; r += kFT) sa[r - r0] = gld(I.a[par] + r);
    __syncthreads();
    float resmax = 0.f, drift = 0.f;
    KChunk<ST> buf[NB][FR][CPT];
    auto load_group = [&](KChunk<ST> (&bf)[FR][CPT], int rb) {
#pragma unroll
        for (int rr = 0; rr < FR; ++rr)
#pragma unroll
            for (int k = 0; k < CPT; ++k)
                if (rb + rr < r1 && own[k]) bf[rr][k] = kload<ST, NT>(K, (int64_t)(rb + rr) * pitch + c0[k]);
    };
    int parity = 0;
    auto process = [&](const KChunk<ST> (&cur)[FR][CPT], int rb) {
#pragma unroll
        for (int rr = 0; rr < FR; ++rr) {
            float part = 0.f;
            if (rb + rr < r1) {
#pragma unroll
                for (int k = 0; k < CPT; ++k)
                    if (own[k]) {
                        float x[8];
                        kunpack<ST>(cur[rr][k], x);
#pragma unroll
                        for (int c = 0; c < 8; ++c) part = fmaf(x[c], bj[k][c], part);
                    }
            }
            const float v = dpp_wave_sum(part);
            if (lane == 0) red[parity][wave][rr] = v;
        }
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < FR; ++rr) {
            const int row = rb + rr;
            if (row >= r1) continue;  // uniform
            const float S = sum_partials<NW>(red[parity][lane & (NW - 1)][rr]);
            const float anew = 1.f / fminf(fmaxf(S, kLo), kHi);
            if (t == ((row - r0) % NW) * kWave) {
                gst(I.a[par ^ 1] + row, anew);
                resmax = fmaxf(resmax, fabsf(sa[row - r0] * S - 1.f));
                drift = fmaxf(drift, fabsf(flg2(anew)));
            }
#pragma unroll
            for (int k = 0; k < CPT; ++k)
                if (own[k]) {
                    float x[8];
                    kunpack<ST>(cur[rr][k], x);
#pragma unroll
                    for (int c = 0; c < 8; ++c) acc[k][c] = fmaf(x[c], anew, acc[k][c]);
                }
        }
        parity ^= 1;
    };
#pragma unroll
    for (int b = 0; b < NB - 1; ++b)
        if (r0 + b * FR < r1) load_group(buf[b], r0 + b * FR);
    for (int rb = r0; rb < r1; rb += NB * FR) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int rc = rb + b * FR;
            if (rc >= r1) break;  // uniform
            if (rc + (NB - 1) * FR < r1) load_group(buf[(b + NB - 1) % NB], rc + (NB - 1) * FR);
            process(buf[b], rc);
        }
    }
    // fixed-slot column partials of this workgroup
    float *dst = I.colpart + (int64_t)blockIdx.x * n;
#pragma unroll
    for (int k = 0; k < CPT; ++k)
        if (own[k]) {
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (c0[k] + c < n) gst(dst + c0[k] + c, acc[k][c] * bj[k][c]);
        }
    // residual and drift slots of this workgroup: lane 0 of every wave formed
    // those of its rows
    if (lane == 0) {
        wres[0][wave] = resmax;
        wres[1][wave] = drift;
    }
    __syncthreads();
    if (t == 0) {
        float m = 0.f, d = 0.f;
        for (int w2 = 0; w2 < NW; ++w2) {
            m = fmaxf(m, wres[0][w2]);
            d = fmaxf(d, wres[1][w2]);
        }
        I.res_slots[blockIdx.x] = m;
        I.drift_slots[blockIdx.x] = d;
    }
}

// Stored K: two rows per group. n <= 8192 (one chunk per thread) keeps two
// groups loading ahead; larger n two (BF16) or one (F32, whose rows are twice
// the registers). Measured at n = 16384, BF16 / F32: one row per group at
// depths 2-6 104-106 / 227-232 us; two rows per group 104 (two ahead) / 214
// (one ahead; two ahead spills, 307); the earlier kernel with no rows ahead
// and the row potentials read per row from global memory 143 / 219 us.
template <int ST, bool NT>
static hipError_t launch_fused_st(const Inst *d_insts, int inst, int n, int grid, hipStream_t st) {
    const int cpt = (n + 8 * kFT - 1) / (8 * kFT);
    if (cpt <= 1)
        hipLaunchKernelGGL((k_fused<ST, 1, 2, 3, NT>), dim3(grid), dim3(kFT), 0, st, d_insts, inst);
    else
        hipLaunchKernelGGL((k_fused<ST, 2, 2, ST == SK_K_BF16 ? 3 : 2, NT>), dim3(grid), dim3(kFT), 0, st,
                           d_insts, inst);
    return hipGetLastError();
}

template <bool NT>
static hipError_t launch_fused_nt(const Inst *d_insts, int inst, int n, int grid, int storage,
                                  hipStream_t st) {
    if (storage == SK_W_I16) {
        if ((n / 8 + kFT - 1) / kFT <= 1)
            hipLaunchKernelGGL((k_fused_i16<kFT, 1, 2, 2, NT>), dim3(grid), dim3(kFT), 0, st, d_insts, inst);
        else
            hipLaunchKernelGGL((k_fused_i16<kFT, 2, 1, kFusedAhead + 1, NT>), dim3(grid), dim3(kFT), 0, st,
                               d_insts, inst);
        return hipGetLastError();
    }
    if (storage == SK_K_BF16) return launch_fused_st<SK_K_BF16, NT>(d_insts, inst, n, grid, st);
    return launch_fused_st<SK_K_F32, NT>(d_insts, inst, n, grid, st);
}

hipError_t launch_fused(const Inst *d_insts, int inst, int n, int grid, int storage, int nt_loads,
                        hipStream_t st) {
    return nt_loads ? launch_fused_nt<true>(d_insts, inst, n, grid, storage, st)
                    : launch_fused_nt<false>(d_insts, inst, n, grid, storage, st);
}

}  // namespace sk
