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
constexpr float kL2e = 1.4426950408889634f;
constexpr float kLn2f = 0.6931471805599453f;
constexpr float kLo = 5.421010862427522e-20f;  // 2^-64
constexpr float kHi = 1.8446744073709552e19f;  // 2^64

__device__ __forceinline__ float fex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float flg2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float fwsum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ float fwmax(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
    return v;
}

// 8 values of one chunk as floats: int16 w (I16) or K (BF16 / F32).
template <int ST, bool NT>
__device__ __forceinline__ void fload(const void *base, int64_t off, float (&x)[8]) {
    if (ST == SK_W_I16) {
        const int4 v = gload<NT>(reinterpret_cast<const int4 *>(reinterpret_cast<const int16_t *>(base) + off));
        x[0] = (float)(short)(v.x & 0xffff); x[1] = (float)(v.x >> 16);
        x[2] = (float)(short)(v.y & 0xffff); x[3] = (float)(v.y >> 16);
        x[4] = (float)(short)(v.z & 0xffff); x[5] = (float)(v.z >> 16);
        x[6] = (float)(short)(v.w & 0xffff); x[7] = (float)(v.w >> 16);
    } else if (ST == SK_K_BF16) {
        const int4 v = gload<NT>(reinterpret_cast<const int4 *>(reinterpret_cast<const uint16_t *>(base) + off));
        const uint32_t q[4] = {(uint32_t)v.x, (uint32_t)v.y, (uint32_t)v.z, (uint32_t)v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            x[2 * k] = __uint_as_float(q[k] << 16);
            x[2 * k + 1] = __uint_as_float(q[k] & 0xffff0000u);
        }
    } else {
        const float4 *p = reinterpret_cast<const float4 *>(reinterpret_cast<const float *>(base) + off);
        const float4 a = gload<NT>(p), b = gload<NT>(p + 1);
        x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
        x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
    }
}

template <int ST, int CPT, bool NT>
__global__ __launch_bounds__(kFT) void k_fused(const Inst *__restrict__ insts, int inst) {
    __shared__ float red[kFT / kWave][kFR];
    __shared__ float rowinv[kFR];
    __shared__ int rowbad[kFR];
    const Inst &I = insts[inst];
    Ctl *ctl = I.ctl;
    if (ctl->state != ST_RUNNING) return;
    if (ST != SK_W_I16 && ctl->need_absorb) return;
    const int n = I.n;
    const int t = threadIdx.x, wave = t / kWave, lane = t % kWave;
    const int iter = ctl->iter;
    const int par = iter & 1;
    const bool sent = ST == SK_W_I16 && ctl->sent != 0u;
    const float pf = (float)ctl->p;
    const int64_t pitch = ST == SK_W_I16 ? I.pitch : I.kpitch;
    const void *base = ST == SK_W_I16 ? (const void *)I.W : (const void *)I.K;
    // rows of this workgroup
    const int per = (n + (int)gridDim.x - 1) / (int)gridDim.x;
    const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
    // owned columns and their potentials
    int c0[CPT];
    bool own[CPT];
    float gx[CPT][8], gy[CPT][8], acc[CPT][8];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        c0[k] = (t + k * kFT) * 8;
        own[k] = c0[k] < n;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            acc[k][c] = 0.f;
            if (ST == SK_W_I16) {
                gx[k][c] = own[k] ? (float)I.G[c0[k] + c] : 0.f;
                gy[k][c] = own[k] ? I.gam[c0[k] + c] * kL2e : 0.f;
            } else {
                gx[k][c] = own[k] && c0[k] + c < n ? I.b[c0[k] + c] : 0.f;
                gy[k][c] = 0.f;
            }
        }
    }
    float resmax = 0.f, drift = 0.f;
    for (int rb = r0; rb < r1; rb += kFR) {
        float s[kFR][CPT][8];
        float part[kFR];
        float Ff[kFR];
        // A: s_ij and row partials
#pragma unroll
        for (int rr = 0; rr < kFR; ++rr) {
            const int row = rb + rr;
            part[rr] = 0.f;
            Ff[rr] = (ST == SK_W_I16 && row < r1) ? (float)I.F[par][row] : 0.f;
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
#pragma unroll
                for (int c = 0; c < 8; ++c) s[rr][k][c] = 0.f;
                if (row < r1 && own[k]) {
                    float x[8];
                    fload<ST, NT>(base, (int64_t)row * pitch + c0[k], x);
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        float e;
                        if (ST == SK_W_I16) {
                            const float Iv = fmaf(x[c], pf, gx[k][c]) + Ff[rr];
                            e = fex2(fmaf(Iv, kL2e, gy[k][c]));
                            if (sent && x[c] == -32768.0f) e = 0.f;
                        } else {
                            e = x[c] * gx[k][c];
                        }
                        s[rr][k][c] = e;
                        part[rr] += e;
                    }
                }
            }
        }
#pragma unroll
        for (int rr = 0; rr < kFR; ++rr) {
            const float v = fwsum(part[rr]);
            if (lane == 0) red[wave][rr] = v;
        }
        __syncthreads();
        if (t < kFR) {
            const int row = rb + t;
            float S = 0.f;
            for (int w = 0; w < kFT / kWave; ++w) S += red[w][t];
            int bad = 0;
            if (row < r1) {
                if (ST == SK_W_I16) {
                    bad = !(S >= kLo && S <= kHi);
                    if (!bad) {
                        const float l2S = flg2(S);
                        float phin = -l2S * kLn2f;
                        const float kk = rintf(phin);
                        I.F[par ^ 1][row] = I.F[par][row] + (int)kk;
                        I.phi[par ^ 1][row] = phin - kk;
                        const float r = fex2(fmaf(I.phi[par][row], kL2e, l2S));
                        resmax = fmaxf(resmax, fabsf(r - 1.f));
                    }
                    rowinv[t] = bad ? 0.f : 1.f / S;
                } else {
                    const float Sc = fminf(fmaxf(S, kLo), kHi);
                    const float anew = 1.f / Sc;
                    I.a[par ^ 1][row] = anew;
                    resmax = fmaxf(resmax, fabsf(I.a[par][row] * S - 1.f));
                    drift = fmaxf(drift, fabsf(flg2(anew)));
                    rowinv[t] = anew;
                }
            } else {
                rowinv[t] = 0.f;
            }
            rowbad[t] = bad;
        }
        __syncthreads();
        // exact max shift for a row whose sum left the safe range (I16 only)
        if (ST == SK_W_I16) {
#pragma unroll
            for (int rr = 0; rr < kFR; ++rr) {
                if (!rowbad[rr]) continue;  // uniform across the workgroup
                const int row = rb + rr;
                float m = -INFINITY;
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    if (!own[k]) continue;
                    float x[8];
                    fload<ST, NT>(base, (int64_t)row * pitch + c0[k], x);
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const float Iv = fmaf(x[c], pf, gx[k][c]) + Ff[rr];
                        float y = fmaf(Iv, kL2e, gy[k][c]);
                        if (sent && x[c] == -32768.0f) y = -INFINITY;
                        m = fmaxf(m, y);
                        s[rr][k][c] = y;  // exponent, shifted below
                    }
                }
                m = fwmax(m);
                __syncthreads();
                if (lane == 0) red[wave][0] = m;
                __syncthreads();
                float M = -INFINITY;
                for (int w = 0; w < kFT / kWave; ++w) M = fmaxf(M, red[w][0]);
                float pp = 0.f;
#pragma unroll
                for (int k = 0; k < CPT; ++k)
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const float e = own[k] && M != -INFINITY ? fex2(s[rr][k][c] - M) : 0.f;
                        s[rr][k][c] = e;
                        pp += e;
                    }
                pp = fwsum(pp);
                __syncthreads();
                if (lane == 0) red[wave][1] = pp;
                __syncthreads();
                if (t == 0) {
                    float S2 = 0.f;
                    for (int w = 0; w < kFT / kWave; ++w) S2 += red[w][1];
                    if (M == -INFINITY) {
                        atomicOr(&ctl->err, ERR_EMPTY_ROW);
                        rowinv[rr] = 0.f;
                    } else {
                        const float l2S = M + flg2(S2);
                        const double phin = -(double)l2S * (double)kLn2f;
                        const double kk = rint(phin);
                        I.F[par ^ 1][row] = I.F[par][row] + (int)kk;
                        I.phi[par ^ 1][row] = (float)(phin - kk);
                        const float r = fex2(fmaf(I.phi[par][row], kL2e, l2S));
                        resmax = fmaxf(resmax, fabsf(r - 1.f));
                        rowinv[rr] = 1.f / S2;
                    }
                }
                __syncthreads();
            }
        }
        // B: column accumulation with the new row scalings
#pragma unroll
        for (int rr = 0; rr < kFR; ++rr) {
            const float inv = rowinv[rr];
#pragma unroll
            for (int k = 0; k < CPT; ++k)
#pragma unroll
                for (int c = 0; c < 8; ++c) acc[k][c] = fmaf(s[rr][k][c], inv, acc[k][c]);
        }
        __syncthreads();  // red / rowinv are reused by the next group
    }
    // fixed-slot column partials of this workgroup
    float *dst = I.colpart + (int64_t)blockIdx.x * n;
#pragma unroll
    for (int k = 0; k < CPT; ++k)
        if (own[k]) {
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (c0[k] + c < n) dst[c0[k] + c] = acc[k][c];
        }
    // residual (and drift) slot of this workgroup, reduced by the finaliser
    if (t < kFR) {
        red[0][t] = resmax;
        red[1][t] = drift;
    }
    __syncthreads();
    if (t == 0) {
        I.res_slots[blockIdx.x] = fmaxf(red[0][0], red[0][1]);
        if (ST != SK_W_I16) I.drift_slots[blockIdx.x] = fmaxf(red[1][0], red[1][1]);
    }
}

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

// Rows of a group (FR) are loaded one group ahead into the other of two
// register buffers, so the next group's loads are in flight while this one is
// reduced. One barrier per group: the per-wave row partials are
// double-buffered by group parity and every lane forms S_i from the 16
// partials with dpp_sum16. The scalar work of row i (its new potentials and
// residual) is done by lane 0 of wave (i - r0) mod 16, so no single wave falls
// behind at every barrier.
template <int CPT, int FR, bool SENT, bool NT>
__device__ __forceinline__ void fused_i16_body(const Inst &I, Ctl *ctl, const float *tab,
                                               float (*red)[kFT / kWave][kFR], int *redm,
                                               float *reds, float *wres, float *gl) {
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
    // per owned column: 4 G_j in registers, exp(gam_j) in LDS at
    // gl[(k * 8 + c) * kFT + t] (each lane reads consecutive words)
    int A[CPT][8];
    float acc[CPT][8];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        c0[k] = (t + k * kFT) * 8;
        own[k] = c0[k] < n;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            A[k][c] = own[k] ? 4 * gld(I.G + c0[k] + c) : 0;
            gl[(k * 8 + c) * kFT + t] = own[k] ? fex2(gld(I.gam + c0[k] + c) * kL2e) : 0.f;
            acc[k][c] = 0.f;
        }
    }
    float resmax = 0.f;
    int4 ba[FR][CPT], bb[FR][CPT];
    auto load_group = [&](int4 (&buf)[FR][CPT], int rb) {
#pragma unroll
        for (int rr = 0; rr < FR; ++rr)
#pragma unroll
            for (int k = 0; k < CPT; ++k)
                buf[rr][k] = (rb + rr < r1 && own[k])
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
            Fi[rr] = row < r1 ? gld(Fp + row) : 0;
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
                        float e = tab_at(tab, tab_off(p4, w[c], A[k][c], B));
                        if (SENT) e = (w[c] == SK_SENTINEL) ? 0.f : e;
                        T[rr][k][c] = e;
                        part[rr] = fmaf(e, gl[(k * 8 + c) * kFT + t], part[rr]);
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
            const float S = dpp_sum16(red[parity][lane & 15][rr]);
            inv[rr] = 0.f;
            if (row >= r1) continue;  // uniform
            const bool writer = t == ((row - r0) & 15) * kWave;
            if (S >= kLo && S <= kHi) {
                inv[rr] = __builtin_amdgcn_rcpf(S);
                if (writer) {
                    // log u_i <- F_i - log S_i; r_i = exp(phi_i) S_i
                    const float l2S = flg2(S);
                    const float phin = -l2S * kLn2f;
                    const float kk = rintf(phin);
                    gst(Fn + row, Fi[rr] + (int)kk);
                    gst(phin_p + row, phin - kk);
                    const float r = fex2(fmaf(gld(phip + row), kL2e, l2S));
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
                        m4 = max(m4, __mul24(p4, w[c]) + A[k][c] + 4 * Fi[rr]);
            }
            m4 = wave_max_i(m4);
            if (lane == 0) redm[wave] = m4;
            __syncthreads();
            int mm = INT_MIN;
            for (int w2 = 0; w2 < kFT / kWave; ++w2) mm = max(mm, redm[w2]);
            const int M = mm >> 2;  // exact: a multiple of 4 (unused if mm == INT_MIN)
            float s2 = 0.f;
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                if (!own[k]) continue;
                int w[8];
                unpack8i(cur[rr][k], w);
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    float e = mm == INT_MIN
                                  ? 0.f
                                  : tab_at(tab, tab_off(p4, w[c], A[k][c], 4 * (Fi[rr] - M - kTabLo)));
                    if (SENT) e = (w[c] == SK_SENTINEL) ? 0.f : e;
                    T[rr][k][c] = e;
                    s2 = fmaf(e, gl[(k * 8 + c) * kFT + t], s2);
                }
            }
            s2 = dpp_wave_sum(s2);
            if (lane == 0) reds[wave] = s2;
            __syncthreads();
            float S2 = 0.f;
            for (int w2 = 0; w2 < kFT / kWave; ++w2) S2 += reds[w2];
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
                    const float r = fex2(fmaf(gld(phip + row) + (float)M, kL2e, l2S));
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
    if (r0 < r1) load_group(ba, r0);
    for (int rb = r0; rb < r1; rb += 2 * FR) {
        if (rb + FR < r1) load_group(bb, rb + FR);
        process(ba, rb);
        if (rb + FR >= r1) break;
        if (rb + 2 * FR < r1) load_group(ba, rb + 2 * FR);
        process(bb, rb + FR);
    }
    float *dst = I.colpart + (int64_t)blockIdx.x * n;
#pragma unroll
    for (int k = 0; k < CPT; ++k)
        if (own[k]) {
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (c0[k] + c < n) gst(dst + c0[k] + c, acc[k][c] * gl[(k * 8 + c) * kFT + t]);
        }
    // residual slot of this workgroup: lane 0 of every wave formed the
    // residuals of its rows
    if (lane == 0) wres[wave] = resmax;
    __syncthreads();
    if (t == 0) {
        float m = 0.f;
        for (int w2 = 0; w2 < kFT / kWave; ++w2) m = fmaxf(m, wres[w2]);
        I.res_slots[blockIdx.x] = m;
    }
}

// Rows per group: two with 8 owned columns per thread, one with 16 (register
// budget of 128 VGPRs at 1024 threads).
template <int CPT, bool NT>
__global__ __launch_bounds__(kFT) void k_fused_i16(const Inst *__restrict__ insts, int inst) {
    constexpr int FR = CPT == 1 ? 2 : 1;
    __shared__ float tab[kTabN];
    __shared__ float red[2][kFT / kWave][kFR];
    __shared__ int redm[kFT / kWave];
    __shared__ float reds[kFT / kWave];
    __shared__ float wres[kFT / kWave];
    __shared__ float gl[CPT * 8 * kFT];
    const Inst &I = insts[inst];
    Ctl *ctl = I.ctl;
    if (ctl->state != ST_RUNNING) return;
    fill_exp_table(tab);
    __syncthreads();
    if (ctl->sent != 0u) fused_i16_body<CPT, FR, true, NT>(I, ctl, tab, red, redm, reds, wres, gl);
    else fused_i16_body<CPT, FR, false, NT>(I, ctl, tab, red, redm, reds, wres, gl);
}

template <int ST, bool NT>
static hipError_t launch_fused_st(const Inst *d_insts, int inst, int n, int grid, hipStream_t st) {
    const int cpt = (n / 8 + kFT - 1) / kFT;
    if (cpt <= 1)
        hipLaunchKernelGGL((k_fused<ST, 1, NT>), dim3(grid), dim3(kFT), 0, st, d_insts, inst);
    else
        hipLaunchKernelGGL((k_fused<ST, 2, NT>), dim3(grid), dim3(kFT), 0, st, d_insts, inst);
    return hipGetLastError();
}

template <bool NT>
static hipError_t launch_fused_nt(const Inst *d_insts, int inst, int n, int grid, int storage,
                                  hipStream_t st) {
    if (storage == SK_W_I16) {
        if ((n / 8 + kFT - 1) / kFT <= 1)
            hipLaunchKernelGGL((k_fused_i16<1, NT>), dim3(grid), dim3(kFT), 0, st, d_insts, inst);
        else
            hipLaunchKernelGGL((k_fused_i16<2, NT>), dim3(grid), dim3(kFT), 0, st, d_insts, inst);
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
