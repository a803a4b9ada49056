// Stored-K storages: the sweeps read K_ij = exp(p w_ij + log u_i + log v_j)
// (bfloat16 or float32), computed once from the log-domain potentials
// ("absorption"), and keep multiplicative row/column scalings a, b in FP32:
// x_ij = K_ij a_i b_j. A stage starts with one exact log-domain iteration
// (every column of the iterate then sums to one and every row holds an entry
// >= 1/n^2, so no sum of K can underflow), then absorbs and sweeps K. When the
// scalings drift by more than 2^20 since the last absorption, they are folded
// back into the potentials and K is recomputed, so an entry flushed to zero at
// absorption (< 2^-126) can never grow past ~2^-86.
//
// Row step (u = I(A^(p) v)):  a_i <- 1 / sum_j K_ij b_j,  r_i = a_i(old) * sum_j K_ij b_j.
// Column step (v = I(A^(p)T u)): b_j <- 1 / sum_i K_ij a_i.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "sk_exptab.h"
#include "sk_ring.h"
#include "sk_runtime.h"

namespace sk {

constexpr float kLog2eK = 1.4426950408889634f;
constexpr float kKLo = 5.421010862427522e-20f;  // 2^-64
constexpr float kKHi = 1.8446744073709552e19f;  // 2^64
constexpr float kDriftLimit = 20.0f;             // log2 of the scaling drift that triggers absorption

__device__ __forceinline__ float kex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float klg2(float x) { return __builtin_amdgcn_logf(x); }

__device__ __forceinline__ float kwave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ double kwave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ void krange(int nunits, int &u0, int &u1) {
    int per = (nunits + (int)gridDim.x - 1) / (int)gridDim.x;
    u0 = (int)blockIdx.x * per;
    u1 = min(nunits, u0 + per);
}

// float -> bfloat16 bits, round to nearest even (finite, non-negative inputs)
__device__ __forceinline__ uint32_t bf16_rne(float x) {
    uint32_t b = __float_as_uint(x);
    return (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;
}

// Loads 8 consecutive K values starting at a multiple of 8.
template <int ST, bool NT>
__device__ __forceinline__ void load8(const void *K, int64_t off, float (&k)[8]) {
    if (ST == SK_K_BF16) {
        const int4 v = gload<NT>(reinterpret_cast<const int4 *>(reinterpret_cast<const uint16_t *>(K) + off));
        const uint32_t x[4] = {(uint32_t)v.x, (uint32_t)v.y, (uint32_t)v.z, (uint32_t)v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            k[2 * q] = __uint_as_float(x[q] << 16);
            k[2 * q + 1] = __uint_as_float(x[q] & 0xffff0000u);
        }
    } else {
        const float4 *p = reinterpret_cast<const float4 *>(reinterpret_cast<const float *>(K) + off);
        const float4 a = gload<NT>(p), b = gload<NT>(p + 1);
        k[0] = a.x; k[1] = a.y; k[2] = a.z; k[3] = a.w;
        k[4] = b.x; k[5] = b.y; k[6] = b.z; k[7] = b.w;
    }
}

__device__ __forceinline__ int kswz(int j, int n8) { return (j & 7) * n8 + (j >> 3); }

// ---------------------------------------------------------------- absorption
// K_ij = exp(p w_ij + F_i + phi_i + G_j + gam_j) from the committed
// potentials: exp(E_ij) of the exact integer exponent E = p w + F_i + G_j
// from the LDS table (as in the log-domain sweeps), times exp(gam_j) and
// exp(phi_i); entries above 2^64 are clamped there, those with E <= -88 are
// 0. The committed F/phi are copied to both parity buffers, a = b = 1.
// 8-wide rows: two 16-byte loads of W in flight per lane, with the
// non-temporal hint above the cache size; K is stored without it (measured
// at n = 16384: 193.5 / 326 us for BF16 / F32 K, against 221 / 415 us with
// non-temporal stores and 212 / 353 us for the float exp2 of the assembled
// exponent with one load in flight).
template <int ST, bool NT>
__global__ __launch_bounds__(kRowWaves * kWave) void k_absorb(const Inst *__restrict__ insts,
                                                              const RowUnit *__restrict__ units,
                                                              int nunits) {
    extern __shared__ int2 pot[];  // (4 G_j, bits of exp(gam_j))
    __shared__ float tab[kTabN];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    fill_exp_table(tab);
    int u0, u1;
    krange(nunits, u0, u1);
    int cur = -1;
    for (int u = u0; u < u1; ++u) {
        const RowUnit un = units[u];
        const Inst &I = insts[un.inst];
        Ctl *ctl = I.ctl;
        if (ctl->state != ST_RUNNING || !ctl->need_absorb) continue;
        const int n = I.n, kp = I.kpitch;
        if (un.inst != cur) {
            __syncthreads();
            const int n8 = pad8(n) >> 3;
            for (int j = threadIdx.x; j < n; j += blockDim.x)
                pot[I.vec8 ? kswz(j, n8) : j] = make_int2(4 * I.G[j], __float_as_int(kex2(I.gam[j] * kLog2eK)));
            if (I.vec8)  // padding columns (their K entries are set to 0 below)
                for (int j = n + (int)threadIdx.x; j < 8 * n8; j += blockDim.x)
                    pot[kswz(j, n8)] = make_int2(0, 0);
            __syncthreads();
            cur = un.inst;
        }
        const int row = un.row0 + wave;
        if (row >= n) continue;
        const int par = ctl->iter & 1;
        const int p4 = 4 * ctl->p;
        const int B = 4 * (I.F[par][row] - kTabLo);
        const float eph = kex2(I.phi[par][row] * kLog2eK);
        const int16_t *wr = I.W + (int64_t)row * I.pitch;
        auto entry = [&](int w, int2 gp) {
            const float e = tab_at(tab, tab_off(p4, w, gp.x, B)) * __int_as_float(gp.y) * eph;
            return w == SK_SENTINEL ? 0.f : fminf(e, kKHi);
        };
        if (I.vec8) {
            // 8 columns per lane: the row of W through the load ring, one
            // 16/32-byte global store of K per chunk (K's padding columns,
            // j >= n, get 0 as in the 1-wide branch)
            const int n8 = pad8(n) >> 3;
            ring_row_chunks<NT>(wr, n, lane, 0, n, [&](int jj, int (&w)[8]) {
                if (jj >= n) return;
                float kv[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) kv[c] = jj + c < n ? entry(w[c], pot[c * n8 + (jj >> 3)]) : 0.f;
                if (ST == SK_K_BF16) {
                    sk_gi4 o;
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        o[c] = (int)(bf16_rne(kv[2 * c]) | (bf16_rne(kv[2 * c + 1]) << 16));
                    *(SK_GLOBAL sk_gi4 *)(reinterpret_cast<uint16_t *>(I.K) + (int64_t)row * kp + jj) = o;
                } else {
                    SK_GLOBAL sk_gf4 *dst =
                        (SK_GLOBAL sk_gf4 *)(reinterpret_cast<float *>(I.K) + (int64_t)row * kp + jj);
                    dst[0] = sk_gf4{kv[0], kv[1], kv[2], kv[3]};
                    dst[1] = sk_gf4{kv[4], kv[5], kv[6], kv[7]};
                }
            });
        } else {
            for (int j = lane; j < kp; j += kWave) {
                const float k = j < n ? entry(wr[j], pot[j]) : 0.f;
                if (ST == SK_K_BF16)
                    reinterpret_cast<uint16_t *>(I.K)[(int64_t)row * kp + j] = (uint16_t)bf16_rne(k);
                else
                    reinterpret_cast<float *>(I.K)[(int64_t)row * kp + j] = k;
            }
        }
        if (lane == 0) {
            I.F[par ^ 1][row] = I.F[par][row];
            I.phi[par ^ 1][row] = I.phi[par][row];
            I.a[0][row] = 1.f;
            I.a[1][row] = 1.f;
        }
    }
}

// Finishes an absorption: b = 1, flags cleared (one workgroup per instance).
__global__ __launch_bounds__(256) void k_absorb_done(const Inst *__restrict__ insts) {
    const Inst &I = insts[blockIdx.x];
    Ctl *ctl = I.ctl;
    if (ctl->state != ST_RUNNING || !ctl->need_absorb) return;
    for (int j = threadIdx.x; j < I.n; j += blockDim.x) I.b[j] = 1.f;
    __syncthreads();
    if (threadIdx.x == 0) {
        ctl->need_absorb = 0u;
        ctl->drift_bits = 0u;
    }
}

// ---------------------------------------------------------------- K row sweep
template <int ST, bool NT>
__global__ __launch_bounds__(kRowWaves * kWave) void k_row_sweep_k(const Inst *__restrict__ insts,
                                                                   const RowUnit *__restrict__ units,
                                                                   int nunits) {
    extern __shared__ float bsh[];
    __shared__ float wres[kRowWaves], wdrift[kRowWaves];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int u0, u1;
    krange(nunits, u0, u1);
    int cur = -1;
    // each wave's running maxima over its rows (lane 0); the workgroup's go to
    // its residual and drift slots at the end, so the waves run their rows
    // without a barrier
    float resmax = 0.f, drift = 0.f;
    // the controller is read once per instance (its values do not change
    // during a launch), as scalars
    bool run = false;
    int par = 0;
    for (int u = u0; u < u1; ++u) {
        const RowUnit un = units[u];
        const Inst &I = insts[un.inst];
        const int n = I.n, kp = I.kpitch, n8 = kp >> 3;
        if (un.inst != cur) {
            Ctl *ctl = I.ctl;
            run = __builtin_amdgcn_readfirstlane(ctl->state) == ST_RUNNING &&
                  !__builtin_amdgcn_readfirstlane(ctl->need_absorb);
            par = __builtin_amdgcn_readfirstlane(ctl->iter) & 1;
            cur = un.inst;
            if (run) {
                __syncthreads();
                for (int j = threadIdx.x; j < kp; j += blockDim.x) bsh[kswz(j, n8)] = j < n ? I.b[j] : 0.f;
                __syncthreads();
            }
        }
        if (!run) continue;
        const int row = un.row0 + wave;
        if (row < n) {
            // requested before the row's matrix loads, used at its end
            const float aold = I.a[par][row];
            float acc = 0.f;
            const int64_t rbase = (int64_t)row * kp;
            int j0 = lane * 8;
            // two 16-byte loads in flight per lane (as the int16 row sweep)
            for (; j0 + 512 < kp; j0 += 2 * 512) {
                float k0[8], k1[8];
                load8<ST, NT>(I.K, rbase + j0, k0);
                load8<ST, NT>(I.K, rbase + j0 + 512, k1);
                const int q = j0 >> 3;
                float s0 = 0.f, s1 = 0.f;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    s0 = fmaf(k0[c], bsh[c * n8 + q], s0);
                    s1 = fmaf(k1[c], bsh[c * n8 + q + 64], s1);
                }
                acc += s0 + s1;
            }
            for (; j0 < kp; j0 += 512) {
                float k[8];
                load8<ST, NT>(I.K, rbase + j0, k);
                const int q = j0 >> 3;
                float s = 0.f;
#pragma unroll
                for (int c = 0; c < 8; ++c) s = fmaf(k[c], bsh[c * n8 + q], s);
                acc += s;
            }
            const float S = kwave_sum(acc);
            if (lane == 0) {
                const float anew = 1.f / fminf(fmaxf(S, kKLo), kKHi);
                I.a[par ^ 1][row] = anew;
                resmax = fmaxf(resmax, fabsf(aold * S - 1.f));
                drift = fmaxf(drift, fabsf(klg2(anew)));
            }
        }
    }
    // stored K is single-instance: every workgroup writes its slot of
    // instance 0 (0 when it had no row), the finalise reduces kres_slots of them
    if (lane == 0) {
        wres[wave] = resmax;
        wdrift[wave] = drift;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = 0.f, d = 0.f;
        for (int w = 0; w < kRowWaves; ++w) {
            m = fmaxf(m, wres[w]);
            d = fmaxf(d, wdrift[w]);
        }
        const Inst &I = insts[0];
        I.res_slots[blockIdx.x] = m;
        I.drift_slots[blockIdx.x] = d;
    }
}

// ---------------------------------------------------------------- K column sweep
template <int ST, bool NT>
__global__ __launch_bounds__(kColWaves * kWave) void k_col_sweep_k(const Inst *__restrict__ insts,
                                                                   const ColUnit *__restrict__ units,
                                                                   int nunits) {
    __shared__ float red[kColWaves][kColTile8];
    __shared__ float ash[kMaxSegRows];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int u0, u1;
    krange(nunits, u0, u1);
    for (int u = u0; u < u1; ++u) {
        const ColUnit un = units[u];
        const Inst &I = insts[un.inst];
        Ctl *ctl = I.ctl;
        if (ctl->state != ST_RUNNING || ctl->need_absorb) continue;
        const int n = I.n, kp = I.kpitch;
        const int npar = (ctl->iter + 1) & 1;
        const int ctile0 = un.tile * kColTile8;
        const int ncols = min(kColTile8, n - ctile0);
        const int r0 = un.seg * I.seg_rows, r1 = min(n, r0 + I.seg_rows);
        __syncthreads();
        for (int r = r0 + (int)threadIdx.x; r < r1; r += blockDim.x) ash[r - r0] = I.a[npar][r];
        __syncthreads();
        float acc[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = 0.f;
        const int c0 = ctile0 + lane * 8;
        if (c0 < n) {
            constexpr int S = kColWaves;
            int r = r0 + wave;
            for (; r + 3 * S < r1; r += 4 * S) {
                float k0[8], k1[8], k2[8], k3[8];
                load8<ST, NT>(I.K, (int64_t)r * kp + c0, k0);
                load8<ST, NT>(I.K, (int64_t)(r + S) * kp + c0, k1);
                load8<ST, NT>(I.K, (int64_t)(r + 2 * S) * kp + c0, k2);
                load8<ST, NT>(I.K, (int64_t)(r + 3 * S) * kp + c0, k3);
                const float a0 = ash[r - r0], a1 = ash[r + S - r0];
                const float a2 = ash[r + 2 * S - r0], a3 = ash[r + 3 * S - r0];
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    acc[c] = fmaf(k3[c], a3, fmaf(k2[c], a2, fmaf(k1[c], a1, fmaf(k0[c], a0, acc[c]))));
            }
            for (; r < r1; r += S) {
                float k[8];
                load8<ST, NT>(I.K, (int64_t)r * kp + c0, k);
                const float ar = ash[r - r0];
#pragma unroll
                for (int c = 0; c < 8; ++c) acc[c] = fmaf(k[c], ar, acc[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) red[wave][lane * 8 + c] = acc[c];
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

// ---------------------------------------------------------------- fold, advance
// log u_i += log a_i, log v_j += log b_j; a = b = 1 (one workgroup per instance).
// Grids of (instances, kPotBlocks): the O(n) FP64 passes over the potentials
// are spread over many workgroups.
constexpr int kPotBlocks = 64;

__global__ __launch_bounds__(256) void k_fold(const Inst *__restrict__ insts) {
    const Inst &I = insts[blockIdx.x];
    Ctl *ctl = I.ctl;
    if (ctl->state == ST_ERROR || ctl->state == ST_DONE) return;
    const int par = ctl->iter & 1;
    for (int i = blockIdx.y * blockDim.x + threadIdx.x; i < I.n; i += gridDim.y * blockDim.x) {
        const double f = (double)I.F[par][i] + (double)I.phi[par][i] + log((double)I.a[par][i]);
        const double k = rint(f);
        I.F[0][i] = I.F[1][i] = (int32_t)k;
        I.phi[0][i] = I.phi[1][i] = (float)(f - k);
        I.a[0][i] = I.a[1][i] = 1.f;
        const double g = (double)I.G[i] + (double)I.gam[i] + log((double)I.b[i]);
        const double kg = rint(g);
        I.G[i] = (int32_t)kg;
        I.gam[i] = (float)(g - kg);
        I.b[i] = 1.f;
    }
}

// Next p of the ladder (p^-1 log u, p^-1 log v held fixed), or done; after a
// pause at the end of a stage (stored K, or a host that evaluates each stage).
// (1) the potentials: p^-1 log u and p^-1 log v held fixed across the step
// to the next p; (2) the control block (a kernel of its own, so that no
// workgroup of (1) can see the state already moved on).
__global__ __launch_bounds__(256) void k_advance_pot(const Inst *__restrict__ insts) {
    const Inst &I = insts[blockIdx.x];
    Ctl *ctl = I.ctl;
    if (ctl->state != ST_STAGE_END) return;
    const int n = I.n;
    const int s = ctl->stage;
    const int par = ctl->iter & 1;
    if (s + 1 >= I.n_p) return;
    const double ratio = (double)I.ladder[s + 1] / (double)I.ladder[s];
    for (int i = blockIdx.y * blockDim.x + threadIdx.x; i < n; i += gridDim.y * blockDim.x) {
        const double f = ((double)I.F[par][i] + (double)I.phi[par][i]) * ratio;
        const double k = rint(f);
        I.F[0][i] = (int32_t)k;
        I.phi[0][i] = (float)(f - k);
        const double g = ((double)I.G[i] + (double)I.gam[i]) * ratio;
        const double kg = rint(g);
        I.G[i] = (int32_t)kg;
        I.gam[i] = (float)(g - kg);
    }
}
__global__ void k_advance_state(const Inst *__restrict__ insts) {
    const Inst &I = insts[blockIdx.x];
    Ctl *ctl = I.ctl;
    if (ctl->state != ST_STAGE_END) return;
    const int s = ctl->stage;
    if (s + 1 < I.n_p) {
        ctl->stage = s + 1;
        ctl->p = I.ladder[s + 1];
        ctl->iter = 0;
        ctl->need_absorb = I.storage != SK_W_I16 ? 1u : 0u;
        ctl->state = ST_RUNNING;
    } else {
        ctl->state = ST_DONE;
    }
}

// FP64 row and column sums of the matrix the K sweeps balance, K_ij a_i b_j
// (each product exact in FP64). Rows: one wave per row, 8-wide loads of K,
// two in flight per lane, b staged in LDS as in the row sweep. Columns: a
// workgroup per (512-column tile, row segment) whose four waves split the
// segment's rows (eight columns per lane, the segment's a_i in LDS) and add
// their partials in wave order into part[segment][column].
template <int ST, bool NT>
__global__ __launch_bounds__(kRowWaves * kWave) void k_check_k_rows(const Inst *__restrict__ insts,
                                                                    const RowUnit *__restrict__ units,
                                                                    int nunits, double *rsum) {
    extern __shared__ float bsh[];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int u0, u1;
    krange(nunits, u0, u1);
    int cur = -1;
    for (int u = u0; u < u1; ++u) {
        const RowUnit un = units[u];
        const Inst &I = insts[un.inst];
        const int n = I.n, kp = I.kpitch, n8 = kp >> 3;
        if (un.inst != cur) {
            __syncthreads();
            for (int j = threadIdx.x; j < kp; j += blockDim.x) bsh[kswz(j, n8)] = j < n ? I.b[j] : 0.f;
            __syncthreads();
            cur = un.inst;
        }
        const int row = un.row0 + wave;
        if (row >= n) continue;
        const int par = I.ctl->iter & 1;
        const int64_t rbase = (int64_t)row * kp;
        double s = 0.0;
        int j0 = lane * 8;
        for (; j0 + 512 < kp; j0 += 2 * 512) {
            float k0[8], k1[8];
            load8<ST, NT>(I.K, rbase + j0, k0);
            load8<ST, NT>(I.K, rbase + j0 + 512, k1);
            const int q = j0 >> 3;
#pragma unroll
            for (int c = 0; c < 8; ++c) s = fma((double)k0[c], (double)bsh[c * n8 + q], s);
#pragma unroll
            for (int c = 0; c < 8; ++c) s = fma((double)k1[c], (double)bsh[c * n8 + q + 64], s);
        }
        for (; j0 < kp; j0 += 512) {
            float k0[8];
            load8<ST, NT>(I.K, rbase + j0, k0);
            const int q = j0 >> 3;
#pragma unroll
            for (int c = 0; c < 8; ++c) s = fma((double)k0[c], (double)bsh[c * n8 + q], s);
        }
        s = kwave_sum_d(s);
        if (lane == 0) rsum[row] = s * (double)I.a[par][row];
    }
}

constexpr int kCheckKWaves = 4;       // waves per workgroup of the column pass
constexpr int kCheckKTile = kWave * 8;  // columns per workgroup: 8 per lane

template <int ST, bool NT>
__global__ __launch_bounds__(kCheckKWaves * kWave) void k_check_k_cols(const Inst *__restrict__ insts,
                                                                       int inst, double *part) {
    __shared__ float ash[kMaxSegRows];
    __shared__ double red[kCheckKWaves][kCheckKTile];
    const Inst &I = insts[inst];
    const int n = I.n, kp = I.kpitch;
    const int seg = blockIdx.y;
    const int r0 = seg * I.seg_rows, r1 = min(n, r0 + I.seg_rows);
    const int par = I.ctl->iter & 1;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (int r = r0 + (int)threadIdx.x; r < r1; r += blockDim.x) ash[r - r0] = I.a[par][r];
    __syncthreads();
    const int j0 = blockIdx.x * kCheckKTile + lane * 8;
    double s[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) s[c] = 0.0;
    if (j0 < kp) {
        // wave w takes rows r0 + w, r0 + w + 4, ...; two rows in flight
        int r = r0 + wave;
        for (; r + kCheckKWaves < r1; r += 2 * kCheckKWaves) {
            float k0[8], k1[8];
            load8<ST, NT>(I.K, (int64_t)r * kp + j0, k0);
            load8<ST, NT>(I.K, (int64_t)(r + kCheckKWaves) * kp + j0, k1);
            const double a0 = (double)ash[r - r0], a1 = (double)ash[r + kCheckKWaves - r0];
#pragma unroll
            for (int c = 0; c < 8; ++c) s[c] = fma((double)k1[c], a1, fma((double)k0[c], a0, s[c]));
        }
        if (r < r1) {
            float k0[8];
            load8<ST, NT>(I.K, (int64_t)r * kp + j0, k0);
            const double a0 = (double)ash[r - r0];
#pragma unroll
            for (int c = 0; c < 8; ++c) s[c] = fma((double)k0[c], a0, s[c]);
        }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) red[wave][lane * 8 + c] = s[c];
    __syncthreads();
    // the waves' partials in wave order, two columns per thread
    for (int q = threadIdx.x; q < kCheckKTile; q += blockDim.x) {
        const int j = blockIdx.x * kCheckKTile + q;
        if (j >= n) continue;
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kCheckKWaves; ++w) t += red[w][q];
        part[(int64_t)seg * n + j] = t;
    }
}

__global__ __launch_bounds__(256) void k_check_k_cols_sum(const Inst *__restrict__ insts, int inst,
                                                          const double *part, double *csum) {
    const Inst &I = insts[inst];
    const int n = I.n;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int seg = 0; seg < I.nseg; ++seg) s += part[(int64_t)seg * n + j];
    csum[j] = s * (double)I.b[j];
}

// ---------------------------------------------------------------- launchers
template <int ST>
static hipError_t launch_absorb_st(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid,
                                   size_t lds_bytes, int nt, hipStream_t st) {
    if (nt)
        hipLaunchKernelGGL((k_absorb<ST, true>), dim3(grid), dim3(kRowWaves * kWave), lds_bytes, st, d_insts,
                           d_units, nunits);
    else
        hipLaunchKernelGGL((k_absorb<ST, false>), dim3(grid), dim3(kRowWaves * kWave), lds_bytes, st,
                           d_insts, d_units, nunits);
    return hipGetLastError();
}
hipError_t launch_absorb(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid,
                         size_t lds_bytes, int storage, int nt, hipStream_t st) {
    return storage == SK_K_BF16 ? launch_absorb_st<SK_K_BF16>(d_insts, d_units, nunits, grid, lds_bytes, nt, st)
                                : launch_absorb_st<SK_K_F32>(d_insts, d_units, nunits, grid, lds_bytes, nt, st);
}
template <int ST, bool NT>
static hipError_t launch_sweeps_k(bool rows, const Inst *d_insts, const void *d_units, int nunits,
                                  int grid, size_t lds_bytes, hipStream_t st) {
    if (rows)
        hipLaunchKernelGGL((k_row_sweep_k<ST, NT>), dim3(grid), dim3(kRowWaves * kWave), lds_bytes,
                           st, d_insts, (const RowUnit *)d_units, nunits);
    else
        hipLaunchKernelGGL((k_col_sweep_k<ST, NT>), dim3(grid), dim3(kColWaves * kWave), 0, st,
                           d_insts, (const ColUnit *)d_units, nunits);
    return hipGetLastError();
}
static hipError_t launch_sweep_k(bool rows, const Inst *d_insts, const void *d_units, int nunits,
                                 int grid, size_t lds_bytes, int storage, int nt_loads,
                                 hipStream_t st) {
    if (storage == SK_K_BF16)
        return nt_loads ? launch_sweeps_k<SK_K_BF16, true>(rows, d_insts, d_units, nunits, grid, lds_bytes, st)
                        : launch_sweeps_k<SK_K_BF16, false>(rows, d_insts, d_units, nunits, grid, lds_bytes, st);
    return nt_loads ? launch_sweeps_k<SK_K_F32, true>(rows, d_insts, d_units, nunits, grid, lds_bytes, st)
                    : launch_sweeps_k<SK_K_F32, false>(rows, d_insts, d_units, nunits, grid, lds_bytes, st);
}
hipError_t launch_row_sweep_k(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid,
                              size_t lds_bytes, int storage, int nt_loads, hipStream_t st) {
    return launch_sweep_k(true, d_insts, d_units, nunits, grid, lds_bytes, storage, nt_loads, st);
}
hipError_t launch_col_sweep_k(const Inst *d_insts, const ColUnit *d_units, int nunits, int grid,
                              int storage, int nt_loads, hipStream_t st) {
    return launch_sweep_k(false, d_insts, d_units, nunits, grid, 0, storage, nt_loads, st);
}
hipError_t launch_fold_k(const Inst *d_insts, int count, hipStream_t st) {
    hipLaunchKernelGGL(k_fold, dim3(count, kPotBlocks), dim3(256), 0, st, d_insts);
    return hipGetLastError();
}
hipError_t launch_advance(const Inst *d_insts, int count, hipStream_t st) {
    hipLaunchKernelGGL(k_advance_pot, dim3(count, kPotBlocks), dim3(256), 0, st, d_insts);
    hipLaunchKernelGGL(k_advance_state, dim3(count), dim3(1), 0, st, d_insts);
    return hipGetLastError();
}
static hipError_t launch_absorb_done(const Inst *d_insts, int count, hipStream_t st) {
    hipLaunchKernelGGL(k_absorb_done, dim3(count), dim3(256), 0, st, d_insts);
    return hipGetLastError();
}
template <int ST, bool NT>
static void launch_check_k_st(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid, int inst,
                              int n, int nseg, double *rsum, double *part, hipStream_t st) {
    const size_t lds = sizeof(float) * (size_t)pad8(n);
    hipLaunchKernelGGL((k_check_k_rows<ST, NT>), dim3(grid), dim3(kRowWaves * kWave), lds, st, d_insts,
                       d_units, nunits, rsum);
    hipLaunchKernelGGL((k_check_k_cols<ST, NT>), dim3((pad8(n) + kCheckKTile - 1) / kCheckKTile, nseg),
                       dim3(kCheckKWaves * kWave), 0, st, d_insts, inst, part);
}
hipError_t launch_check_k(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid, int inst,
                          int n, int nseg, int storage, int nt, double *rsum, double *part, double *csum,
                          hipStream_t st) {
    if (storage == SK_K_BF16) {
        if (nt) launch_check_k_st<SK_K_BF16, true>(d_insts, d_units, nunits, grid, inst, n, nseg, rsum, part, st);
        else launch_check_k_st<SK_K_BF16, false>(d_insts, d_units, nunits, grid, inst, n, nseg, rsum, part, st);
    } else {
        if (nt) launch_check_k_st<SK_K_F32, true>(d_insts, d_units, nunits, grid, inst, n, nseg, rsum, part, st);
        else launch_check_k_st<SK_K_F32, false>(d_insts, d_units, nunits, grid, inst, n, nseg, rsum, part, st);
    }
    hipLaunchKernelGGL(k_check_k_cols_sum, dim3((n + 255) / 256), dim3(256), 0, st, d_insts, inst,
                       part, csum);
    return hipGetLastError();
}

// ---------------------------------------------------------------- host controller
#define KCHK(expr)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, SK_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

static sk_status absorb(sk_ctx *ctx, Batch &B, int storage) {
    ctx->prof.begin(ctx->stream, KID_ABSORB);
    KCHK(launch_absorb(B.d_insts, B.d_rows, (int)B.h_rows.size(), B.row_grid, B.row_lds, storage,
                       B.h_insts[0].nt, ctx->stream));
    KCHK(launch_absorb_done(B.d_insts, B.count, ctx->stream));
    ctx->prof.end(ctx->stream);
    ctx->absorbs += 1;
    return SK_OK;
}

static sk_status fold(sk_ctx *ctx, Batch &B) {
    ctx->prof.begin(ctx->stream, KID_FOLD_K);
    KCHK(launch_fold_k(B.d_insts, B.count, ctx->stream));
    ctx->prof.end(ctx->stream);
    return SK_OK;
}

// Sets need_absorb on the device copy of the control block.
static sk_status request_absorb(sk_ctx *ctx, Batch &B) {
    static const uint32_t one = 1u;
    KCHK(hipMemcpyAsync(&B.h_insts[0].ctl->need_absorb, &one, sizeof one, hipMemcpyHostToDevice,
                        ctx->stream));
    KCHK(hipStreamSynchronize(ctx->stream));
    return SK_OK;
}

sk_status run_single_k(sk_ctx *ctx, Batch &B, const sk_params *prm, const StageHook *hook) {
    const int storage = prm->storage;
    const int check = std::max(1, prm->check_every);
    sk_status st;
    if ((st = request_absorb(ctx, B)) != SK_OK) return st;
    const int64_t bound = (prm->max_iters_per_stage + 2) * prm->n_p * 4 + 16;
    int64_t rounds = 0;
    ctx->k_res_rows = ctx->k_res_cols = NAN;
    for (;;) {
        if ((st = read_ctl(ctx, B)) != SK_OK) return st;
        const Ctl &c = ctx->h_ctl[0];
        if (++rounds > bound) return fail(ctx, SK_EDEVICE, "stored-K controller did not terminate");
        if (c.state == ST_ERROR || c.state == ST_DONE) break;
        if (c.state == ST_STAGE_END) {
            if (c.stage + 1 >= prm->n_p) {
                // FP64 sums of the balanced matrix K a b, before folding
                const Inst &I = B.h_insts[0];
                const int n = I.n;
                ctx->prof.begin(ctx->stream, KID_CHECK_ROWS);
                KCHK(launch_check_k(B.d_insts, B.d_rows, (int)B.h_rows.size(), B.row_grid, 0, n,
                                    I.nseg, storage, I.nt, B.d_rsum, B.d_cpart, B.d_csum, ctx->stream));
                ctx->prof.end(ctx->stream);
                std::vector<double> r(n), cs(n);
                KCHK(hipMemcpyAsync(r.data(), B.d_rsum, 8 * (size_t)n, hipMemcpyDeviceToHost,
                                    ctx->stream));
                KCHK(hipMemcpyAsync(cs.data(), B.d_csum, 8 * (size_t)n, hipMemcpyDeviceToHost,
                                    ctx->stream));
                KCHK(hipStreamSynchronize(ctx->stream));
                double rr = 0, cr = 0;
                for (int i = 0; i < n; ++i) {
                    rr = std::max(rr, std::fabs(r[i] - 1.0));
                    cr = std::max(cr, std::fabs(cs[i] - 1.0));
                }
                ctx->k_res_rows = rr;
                ctx->k_res_cols = cr;
            }
            if ((st = fold(ctx, B)) != SK_OK) return st;
            if (hook) {
                bool stop = false;
                if ((st = (*hook)(stop)) != SK_OK) return st;
                if (stop) return SK_OK;
            }
            KCHK(launch_advance(B.d_insts, B.count, ctx->stream));
            continue;
        }
        if (c.need_absorb) {
            // one exact log-domain iteration, then K from its potentials
            if ((st = iterate_i16(ctx, B)) != SK_OK) return st;
            if ((st = absorb(ctx, B, storage)) != SK_OK) return st;
            continue;
        }
        float drift;
        memcpy(&drift, &c.drift_bits, sizeof drift);
        if (drift > kDriftLimit) {
            if ((st = fold(ctx, B)) != SK_OK) return st;
            if ((st = request_absorb(ctx, B)) != SK_OK) return st;
            if ((st = absorb(ctx, B, storage)) != SK_OK) return st;
            continue;
        }
        // a block of K iterations; afterwards the launches past the point
        // where the stage ended are tagged (detection / idle). The stage's
        // first block is sized by the previous stage's iterations, later ones
        // are short, so few launches run after the stage has ended.
        const size_t pstart = ctx->prof.pending.size();
        const int64_t it0 = c.iters_total;
        const int stage0 = c.stage;
        const Inst &I0 = B.h_insts[0];
        const int64_t done = c.stage_iters[c.stage];
        int blk = std::min(check, 8);
        if (done <= 1)
            blk = c.stage == 0 ? check
                               : (int)std::min<int64_t>(
                                     check, std::max<int64_t>(4, c.stage_iters[c.stage - 1] + 2 - done));
        for (int k = 0; k < blk; ++k) {
            if (I0.fused) {
                ctx->prof.begin(ctx->stream, KID_FUSED);
                KCHK(launch_fused(B.d_insts, 0, I0.n, I0.fused_grid, storage, I0.nt, ctx->stream));
                ctx->prof.end(ctx->stream);

            } else {
                // the two sweeps share the stamp between them
                Profiler &pf = ctx->prof;
                const int s0 = pf.stamp(ctx->stream);
                KCHK(launch_row_sweep_k(B.d_insts, B.d_rows, (int)B.h_rows.size(), B.row_grid_k,
                                        B.row_lds_k, storage, I0.nt, ctx->stream));
                const int s1 = pf.stamp(ctx->stream);
                KCHK(launch_col_sweep_k(B.d_insts, B.d_cols, (int)B.h_cols.size(), B.col_grid,
                                        storage, I0.nt, ctx->stream));
                const int s2 = pf.stamp(ctx->stream);
                pf.add(KID_ROW_K, s0, s1);
                pf.add(KID_COL_K, s1, s2);
            }
            // finalise and end of iteration: short, not stamped
            KCHK(launch_col_finalize(B.d_insts, B.d_fins, (int)B.h_fins.size(), B.fin_grid,
                                     kFinStoredK | (I0.fused ? kFinOnePass : 0), ctx->stream));
            KCHK(launch_iter_end(B.d_insts, B.count, ctx->stream));
        }
        if (ctx->prof.on) {
            if ((st = read_ctl(ctx, B)) != SK_OK) return st;
            const Ctl &c2 = ctx->h_ctl[0];
            const int64_t did = c2.iters_total - it0;
            // the stage ended inside this block by convergence: one detection triple
            const bool ended = c2.state != ST_RUNNING || c2.stage != stage0;
            const bool conv = ended && c2.stage_iters[stage0] < prm->max_iters_per_stage;
            const int64_t det = conv ? did : -1;
            const int64_t work = did + (conv ? 1 : 0);
            auto tag = [&](int dk, int ik) {
                return [=](int64_t t) { return t == det ? dk : (t >= work ? ik : -1); };
            };
            ctx->prof.retag(pstart, KID_ROW_K, tag(KID_ROW_K_DETECT, KID_ROW_K_IDLE));
            ctx->prof.retag(pstart, KID_COL_K, tag(KID_COL_K_DETECT, KID_COL_K_IDLE));
            ctx->prof.retag(pstart, KID_FUSED, tag(KID_FUSED_DETECT, KID_FUSED_IDLE));
        }
    }
    return SK_OK;
}

hipError_t set_k_attributes() {
    hipError_t e;
    const int lds = (int)(kLdsMaxN * sizeof(float2));
    for (const void *f : {(const void *)k_absorb<SK_K_BF16, true>, (const void *)k_absorb<SK_K_BF16, false>,
                          (const void *)k_absorb<SK_K_F32, true>, (const void *)k_absorb<SK_K_F32, false>})
        if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds)) != hipSuccess)
            return e;
    for (const void *f : {(const void *)k_check_k_rows<SK_K_BF16, true>, (const void *)k_check_k_rows<SK_K_BF16, false>,
                          (const void *)k_check_k_rows<SK_K_F32, true>, (const void *)k_check_k_rows<SK_K_F32, false>})
        if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(kLdsMaxN * sizeof(float)))) != hipSuccess)
            return e;
    for (const void *f : {(const void *)k_row_sweep_k<SK_K_BF16, true>,
                          (const void *)k_row_sweep_k<SK_K_BF16, false>,
                          (const void *)k_row_sweep_k<SK_K_F32, true>,
                          (const void *)k_row_sweep_k<SK_K_F32, false>})
        if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds / 2)) !=
            hipSuccess)
            return e;
    return hipSuccess;
}

}  // namespace sk
