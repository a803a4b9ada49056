// Real-valued log-weights: input scan, Sinkhorn row and column sweeps, FP64
// recheck and reduced matrix for W = log A given as float32 (-inf for a zero
// entry). The terms are formed as described in sk_real.h; everything else
// (potentials layout, fixed-slot column partials, the finalise kernel's
// column step, residual slots, the end-of-iteration controller) is shared
// with the int16 path.
//
// Layout: W row-major with pitch I.pitch floats. With n % 4 == 0, a pitch
// that is a multiple of 4 and a 16-byte aligned W (Inst::vec8 set for a real
// instance) a lane reads 4 consecutive columns with one 16-byte load (lane l
// owns columns 4 l + 256 k + c); otherwise one column per load (lane l owns
// columns l + 64 k).
#include <climits>

#include "sk_real.h"
#include "sk_runtime.h"

namespace sk {

// Terms with log x below this are left out of the FP64 sums: each is below
// e^-46, so at most n e^-46 < 2^-52 of a row or column sum of 1 (n <= 16384).
constexpr double kRealNegligible = -46.0;

// LDS position of column j when lanes own 4 consecutive columns: column j at
// (j % 4) * n4 + j / 4 (n4 = ceil(n / 4)), so for each of the 4 columns the
// 64 lanes read 64 consecutive doubles.
__device__ __forceinline__ int swz4(int j, int n4) { return (j & 3) * n4 + (j >> 2); }

// ---------------------------------------------------------------- range scan
// Per workgroup: smallest and largest finite weight and whether W holds a NaN
// or +inf (not a log-weight). part[3 b + {0, 1, 2}].
__global__ __launch_bounds__(256) void k_real_minmax(const float *__restrict__ W, int n, int64_t pitch,
                                                     float *__restrict__ part) {
    __shared__ float smin[256], smax[256], sbad[256];
    float lo = INFINITY, hi = -INFINITY, bad = 0.f;
    for (int r = blockIdx.x; r < n; r += gridDim.x) {
        const float *wr = W + (int64_t)r * pitch;
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            const float w = wr[j];
            if (w == -INFINITY) continue;
            if (!(w < INFINITY)) {
                bad = 1.f;  // NaN or +inf
                continue;
            }
            lo = fminf(lo, w);
            hi = fmaxf(hi, w);
        }
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + o]);
            smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + o]);
            sbad[threadIdx.x] = fmaxf(sbad[threadIdx.x], sbad[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = smin[0];
        part[3 * blockIdx.x + 1] = smax[0];
        part[3 * blockIdx.x + 2] = sbad[0];
    }
}

// ---------------------------------------------------------------- input scan / cold start
// Marks instances whose W holds -inf and rows with no finite entry; with cold
// != 0 sets the first-stage start (v_0 = 1, eq. dad1) with the row shift of
// Section 4.1.2: log u_i = -p (max_j w_ij - wref), log v = 0.
__global__ __launch_bounds__(kRowWaves * kWave) void k_init_real(const Inst *__restrict__ insts,
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
        const float *wr = I.Wr + (int64_t)row * I.pitch;
        float mx = -INFINITY;
        int sent = 0;
        for (int j = lane; j < n; j += kWave) {
            const float w = wr[j];
            sent |= w == -INFINITY;
            mx = fmaxf(mx, w);
        }
        mx = wave_max(mx);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sent |= __shfl_xor(sent, o, kWave);
        if (lane == 0) {
            if (mx == -INFINITY) atomicOr(&I.ctl->err, ERR_EMPTY_ROW);
            if (sent) atomicOr(&I.ctl->sent, 1u);
            if (cold) {
                const double lu = mx == -INFINITY
                                      ? 0.0
                                      : -real_p(I, I.ctl) * ((double)mx - (double)I.wref);
                const double k = rint(lu);
                I.F[0][row] = (int32_t)k;
                I.phi[0][row] = (float)(lu - k);
            }
        }
    }
}

// ---------------------------------------------------------------- row sweep
// One wavefront per row; per column (G_j + gam_j) log2 e staged once per
// workgroup in LDS (FP64); the row's integer part F_i is the shift of the
// sum (as in the int16 path), the exact max shift is taken when the sum
// leaves [2^-64, 2^64].

template <bool SENT>
__device__ __forceinline__ float real_term(float w, double p2, double wref, double c) {
    float t = pow2_split(fma(p2, (double)w - wref, c));
    if (SENT) t = (w == -INFINITY) ? 0.f : t;
    return t;
}

template <bool SENT, bool NT, bool V4>
__device__ __forceinline__ float real_row_sum(const float *__restrict__ wr, int n, double p2,
                                              double wref, double f2, const double *__restrict__ lv2,
                                              int lane) {
    float acc = 0.f;
    if (V4) {
        const int n4 = (n + 3) >> 2;
        // two 16-byte loads in flight per lane
        for (int j0 = lane * 4; j0 < n; j0 += 512) {
            const bool two = j0 + 256 < n;
            const float4 a = gload<NT>(reinterpret_cast<const float4 *>(wr + j0));
            const float4 b = two ? gload<NT>(reinterpret_cast<const float4 *>(wr + j0 + 256))
                                 : make_float4(0.f, 0.f, 0.f, 0.f);
            const int q = j0 >> 2;
            float s = real_term<SENT>(a.x, p2, wref, f2 + lv2[q]);
            s += real_term<SENT>(a.y, p2, wref, f2 + lv2[n4 + q]);
            s += real_term<SENT>(a.z, p2, wref, f2 + lv2[2 * n4 + q]);
            s += real_term<SENT>(a.w, p2, wref, f2 + lv2[3 * n4 + q]);
            acc += s;
            if (two) {
                float s2 = real_term<SENT>(b.x, p2, wref, f2 + lv2[q + 64]);
                s2 += real_term<SENT>(b.y, p2, wref, f2 + lv2[n4 + q + 64]);
                s2 += real_term<SENT>(b.z, p2, wref, f2 + lv2[2 * n4 + q + 64]);
                s2 += real_term<SENT>(b.w, p2, wref, f2 + lv2[3 * n4 + q + 64]);
                acc += s2;
            }
        }
    } else {
        for (int j = lane; j < n; j += kWave) acc += real_term<SENT>(wr[j], p2, wref, f2 + lv2[j]);
    }
    return acc;
}

// max_j of E2 = (p w'_ij + F_i + log v_j) log2 e over the row (-inf if none).
template <bool V4>
__device__ __forceinline__ double real_row_max(const float *__restrict__ wr, int n, double p2,
                                               double wref, double f2, const double *__restrict__ lv2,
                                               int lane) {
    double m = -INFINITY;
    const int n4 = (n + 3) >> 2;
    for (int j = lane; j < n; j += kWave) {
        const float w = wr[j];
        if (w == -INFINITY) continue;
        const double l = V4 ? lv2[swz4(j, n4)] : lv2[j];
        m = fmax(m, fma(p2, (double)w - wref, f2 + l));
    }
    return m;
}

// A value that is the same in every lane, as a scalar.
__device__ __forceinline__ double rfl_d(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <bool NT, bool V4>
__global__ __launch_bounds__(kRowWaves * kWave) void k_row_sweep_real(const Inst *__restrict__ insts,
                                                                        const RowUnit *__restrict__ units,
                                                                        int nunits) {
    extern __shared__ double lv2[];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int u0, u1;
    unit_range(nunits, u0, u1);
    __shared__ unsigned wg_res, wg_done;
    if (threadIdx.x == 0) {
        wg_res = 0u;
        wg_done = 0u;
    }
    int cur = -1;  // running instance whose column data is staged
    float wres = 0.f;
    const int slot = (int)((blockIdx.x * kRowWaves + wave) % kRowResSlots) * kRowResStride;
    // What the rows of the instance in hand read, loaded at each change of
    // instance (none of it changes during a launch), and the potentials of
    // the wave's row in unit ubase + l in lane l (up to 64 units ahead): a
    // row then starts without a chain of dependent loads.
    bool run = false, sent = false;
    int ucur = -1, ubase = 0, n = 0;
    double p2 = 0.0, wref = 0.0;
    const float *Wr = nullptr;
    int64_t pitch = 0;
    const SK_GLOBAL int32_t *Fp = nullptr;
    SK_GLOBAL int32_t *Fn = nullptr;
    SK_GLOBAL float *phin_p = nullptr, *rres = nullptr;
    Ctl *cctl = nullptr;
    int lF = 0;
    float lphi = 0.f;
    for (int u = u0; u < u1; ++u) {
        const RowUnit un = units[u];
        if (un.inst != ucur || u - ubase >= kWave) {
            if (un.inst != ucur) {
                if (cur >= 0 && lane == 0 && wres > 0.f) atomicMax(&insts[cur].rowres[slot], __float_as_uint(wres));
                wres = 0.f;
            }
            const Inst &I = insts[un.inst];
            Ctl *ctl = I.ctl;
            // controller values are the same in every lane: read as scalars,
            // so that what depends on them stays in scalar registers
            run = __builtin_amdgcn_readfirstlane(ctl->state) == ST_RUNNING;
            ucur = un.inst;
            ubase = u;
            if (run) {
                n = I.n;
                const int par = __builtin_amdgcn_readfirstlane(ctl->iter) & 1;
                p2 = rfl_d(real_p(I, ctl) * kLog2eD);
                wref = (double)I.wref;
                Wr = I.Wr;
                pitch = I.pitch;
                sent = __builtin_amdgcn_readfirstlane(ctl->sent) != 0u;
                cctl = ctl;
                Fp = (const SK_GLOBAL int32_t *)(par ? I.F[1] : I.F[0]);
                const SK_GLOBAL float *phip = (const SK_GLOBAL float *)(par ? I.phi[1] : I.phi[0]);
                Fn = (SK_GLOBAL int32_t *)(par ? I.F[0] : I.F[1]);
                phin_p = (SK_GLOBAL float *)(par ? I.phi[0] : I.phi[1]);
                rres = (SK_GLOBAL float *)I.rres;
                const int ul = u + lane;
                if (ul < u1) {
                    const RowUnit x = units[ul];
                    const int r = x.row0 + wave;
                    if (x.inst == un.inst && r < n) {
                        lF = Fp[r];
                        lphi = phip[r];
                    }
                }
                __syncthreads();
                const int n4 = (n + 3) >> 2;
                for (int j = threadIdx.x; j < n; j += blockDim.x)
                    lv2[V4 ? swz4(j, n4) : j] = ((double)I.G[j] + (double)I.gam[j]) * kLog2eD;
                __syncthreads();
                // an empty use: the wait for these loads falls here, once per
                // window, not before every row's register read
                asm volatile("" : "+v"(lF), "+v"(lphi));
            }
            cur = run ? un.inst : -1;
        }
        if (!run) continue;
        const int row = un.row0 + wave;
        if (row >= n) continue;
        const int kk = u - ubase;
        const int Fi = __builtin_amdgcn_readlane(lF, kk);
        const float phi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lphi), kk));
        const float *wr = Wr + (int64_t)row * pitch;
        auto rsum = [&](int shift) {
            const double f2 = (double)(Fi - shift) * kLog2eD;
            return wave_sum(sent ? real_row_sum<true, NT, V4>(wr, n, p2, wref, f2, lv2, lane)
                                 : real_row_sum<false, NT, V4>(wr, n, p2, wref, f2, lv2, lane));
        };
        float S = rsum(0);
        int M = 0;
        if (!(S >= kSafeLo && S <= kSafeHi)) {
            // exact max shift (Section 4.1.2): M = rint(max_j (p w'_ij + F_i + log v_j))
            const double m2 = wave_max_d(real_row_max<V4>(wr, n, p2, wref, (double)Fi * kLog2eD, lv2, lane));
            if (m2 == -INFINITY) {
                if (lane == 0) atomicOr(&cctl->err, ERR_EMPTY_ROW);
                S = 1.f;
            } else {
                M = (int)rint(m2 * kLn2D);
                S = rsum(M);
            }
        }
        if (lane == 0) {
            // log u_i <- F_i - M - log S;  r_i = exp(phi_i + M) S
            const float l2S = lg2(S);
            const float phin = -l2S * kLn2;
            const float k = rintf(phin);
            Fn[row] = Fi - M + (int)k;
            phin_p[row] = phin - k;
            const float r = ex2(fmaf(phi + (float)M, kLog2e, l2S));
            const float res = fabsf(r - 1.f);
            rres[row] = res;
            wres = fmaxf(wres, res);
        }
    }
    // the waves' residual maxima meet in LDS; the last wave sends the
    // workgroup's to the instance's slot (read by the column sweep)
    if (lane == 0) {
        if (wres > 0.f) atomicMax(&wg_res, __float_as_uint(wres));
        __threadfence_block();
        const unsigned k = atomicAdd(&wg_done, 1u);
        if (k == kRowWaves - 1) {
            __threadfence_block();
            const unsigned m = atomicMax(&wg_res, 0u);
            if (cur >= 0 && m > 0u) atomicMax(&insts[cur].rowres[slot], m);
        }
    }
}

// ---------------------------------------------------------------- column sweep
// Workgroup = column tile (kRealTile columns) x row segment; the four waves
// split the segment's rows; per row (F_i + phi_i) log2 e of the new row
// potentials staged in LDS; the slots hold
// sum_i exp(p w'_ij + log u_i + G_j), added in a fixed order, as the
// finalise kernel expects of a log-domain column sweep.

__device__ __forceinline__ bool real_stage_converged_skip(const Inst &I, const Ctl *ctl, float rowres) {
    return ctl->iter >= 1 && rowres < I.tol;
}

template <bool SENT, bool NT, bool V4>
__device__ __forceinline__ void real_col_partial(const Inst &I, int r0, int r1, int wave, int n,
                                                 const int (&cols)[4], const double (&g2)[4], double p2,
                                                 double wref, const double *__restrict__ rowpot,
                                                 float (&acc)[4]) {
    const int64_t pitch = I.pitch;
    const float *base = I.Wr;
    auto row_vals = [&](int rr, float (&w)[4]) {
        if (V4) {
            const float4 v = gload<NT>(reinterpret_cast<const float4 *>(base + (int64_t)rr * pitch + cols[0]));
            w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) w[c] = cols[c] < n ? base[(int64_t)rr * pitch + cols[c]] : -INFINITY;
        }
    };
    // two rows in flight per lane; rows added in order
    int r = r0 + wave;
    for (; r + kColWaves < r1; r += 2 * kColWaves) {
        float wa[4], wb[4];
        row_vals(r, wa);
        row_vals(r + kColWaves, wb);
        const double fa = rowpot[r - r0], fb = rowpot[r + kColWaves - r0];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            acc[c] += real_term<SENT>(wa[c], p2, wref, fa + g2[c]);
            acc[c] += real_term<SENT>(wb[c], p2, wref, fb + g2[c]);
        }
    }
    if (r < r1) {
        float wa[4];
        row_vals(r, wa);
        const double fa = rowpot[r - r0];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] += real_term<SENT>(wa[c], p2, wref, fa + g2[c]);
    }
}

template <bool NT, bool V4>
__global__ __launch_bounds__(kColWaves * kWave) void k_col_sweep_real(const Inst *__restrict__ insts,
                                                                        const ColUnit *__restrict__ units,
                                                                        int nunits) {
    __shared__ float red[kColWaves][kRealTile];
    __shared__ double rowpot[kMaxSegRows];
    __shared__ float wmax[kColWaves];
    __shared__ float rowres_max;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int u0, u1;
    unit_range(nunits, u0, u1);
    for (int u = u0; u < u1; ++u) {
        const ColUnit un = units[u];
        const Inst &I = insts[un.inst];
        Ctl *ctl = I.ctl;
        if (ctl->state != ST_RUNNING) continue;
        const int n = I.n;
        const int npar = (ctl->iter + 1) & 1;
        const int ctile0 = un.tile * kRealTile;
        const int ncols = min(kRealTile, n - ctile0);
        const int r0 = un.seg * I.seg_rows, r1 = min(n, r0 + I.seg_rows);
        __syncthreads();
        float rm = 0.f;
        for (int r = r0 + (int)threadIdx.x; r < r1; r += blockDim.x) {
            rowpot[r - r0] = ((double)I.F[npar][r] + (double)I.phi[npar][r]) * kLog2eD;
            if (un.tile == 0) rm = fmaxf(rm, I.rres[r]);
        }
        if (un.tile == 0) {
            rm = wave_max(rm);
            if (lane == 0) wmax[wave] = rm;
        }
        if (wave == 0) {
            const float rr = wave_max(__uint_as_float(I.rowres[lane * kRowResStride]));
            if (lane == 0) rowres_max = rr;
        }
        __syncthreads();
        if (un.tile == 0 && threadIdx.x == 0) {
            float m = wmax[0];
#pragma unroll
            for (int w2 = 1; w2 < kColWaves; ++w2) m = fmaxf(m, wmax[w2]);
            I.res_slots[un.seg] = m;
        }
        // the row sweep measured a converged iterate: no column step follows
        if (real_stage_converged_skip(I, ctl, rowres_max)) continue;
        const double p2 = real_p(I, ctl) * kLog2eD;
        const double wref = (double)I.wref;
        // this lane's 4 columns and their integer parts G_j log2 e
        int cols[4];
        double g2[4];
        float acc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            cols[c] = V4 ? ctile0 + lane * 4 + c : ctile0 + lane + 64 * c;
            g2[c] = cols[c] < n ? (double)I.G[cols[c]] * kLog2eD : 0.0;
            acc[c] = 0.f;
        }
        if (cols[0] < n) {
            // padding columns of the 1-wide form read as -inf (masked)
            if (ctl->sent != 0u || !V4)
                real_col_partial<true, NT, V4>(I, r0, r1, wave, n, cols, g2, p2, wref, rowpot, acc);
            else
                real_col_partial<false, NT, V4>(I, r0, r1, wave, n, cols, g2, p2, wref, rowpot, acc);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) red[wave][V4 ? lane * 4 + c : lane + 64 * c] = acc[c];
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

// ---------------------------------------------------------------- FP64 recheck
// Row sums r_i and m_i = max_j (p w'_ij + log v_j) in FP64 (the certificate
// of Proposition prop:aoc needs sum_i m_i - sum_j log v_j); with counts the
// entries with log x_ij >= logt (the row lengths of B, in the arithmetic
// order of the fill kernel) and the first column of the row's largest x_ij.
__device__ __forceinline__ double real_logx_t(double p, float w, double wref, double lv) {
    return p * ((double)w - wref) + lv;  // t = p w' + log v_j; log x = t + log u_i
}

__global__ __launch_bounds__(kRowWaves * kWave) void k_check_rows_real(
    const Inst *__restrict__ insts, const RowUnit *__restrict__ units, int nunits, double *rsum,
    double *rmax, double logt, int64_t *counts, int32_t *hint) {
    extern __shared__ double lvd[];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int u0, u1;
    unit_range(nunits, u0, u1);
    int cur = -1;
    for (int u = u0; u < u1; ++u) {
        const RowUnit un = units[u];
        const Inst &I = insts[un.inst];
        const int n = I.n;
        if (un.inst != cur) {
            __syncthreads();
            for (int j = threadIdx.x; j < n; j += blockDim.x) lvd[j] = (double)I.G[j] + (double)I.gam[j];
            __syncthreads();
            cur = un.inst;
        }
        const int row = un.row0 + wave;
        if (row >= n) continue;
        const int par = I.ctl->iter & 1;
        const double p = real_p(I, I.ctl), wref = (double)I.wref;
        const double f = (double)I.F[par][row] + (double)I.phi[par][row];
        const float *wr = I.Wr + (int64_t)row * I.pitch;
        double s = 0.0, m = -INFINITY;
        int jm = -1, cnt = 0;
        for (int j = lane; j < n; j += kWave) {
            const float w = wr[j];
            if (w == -INFINITY) continue;
            const double t = real_logx_t(p, w, wref, lvd[j]);
            const double lx = t + f;
            if (lx > kRealNegligible) s += exp(lx);
            cnt += lx >= logt;
            if (t > m) {  // a lane visits its columns in increasing order
                m = t;
                jm = j;
            }
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

// FP64 column partials per row segment (one thread per column, rows of the
// segment in order), then their sum per column in segment order.
__global__ __launch_bounds__(256) void k_check_cols_real(const Inst *__restrict__ insts, int inst,
                                                         double *part) {
    const Inst &I = insts[inst];
    const int n = I.n;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int seg = blockIdx.y;
    if (j >= n) return;
    const int r0 = seg * I.seg_rows, r1 = min(n, r0 + I.seg_rows);
    const int par = I.ctl->iter & 1;
    const double p = real_p(I, I.ctl), wref = (double)I.wref;
    const double lv = (double)I.G[j] + (double)I.gam[j];
    double s = 0.0;
    for (int r = r0; r < r1; ++r) {
        const float w = I.Wr[(int64_t)r * I.pitch + j];
        if (w == -INFINITY) continue;
        const double lx = real_logx_t(p, w, wref, lv) + ((double)I.F[par][r] + (double)I.phi[par][r]);
        if (lx > kRealNegligible) s += exp(lx);
    }
    part[(int64_t)seg * n + j] = s;
}

__global__ __launch_bounds__(256) void k_check_cols_sum_real(const Inst *__restrict__ insts, int inst,
                                                             const double *part, double *csum) {
    const Inst &I = insts[inst];
    const int n = I.n;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int seg = 0; seg < I.nseg; ++seg) s += part[(int64_t)seg * n + j];
    csum[j] = s;
}

// ---------------------------------------------------------------- reduced matrix
// B keeps (i, j) iff x_ij(p) >= t (eq. matrixred), decided on log x_ij in FP64
// in the same arithmetic as the counts of k_check_rows_real. Each wave walks
// its row in 64-column chunks and places the kept entries with a ballot
// prefix (column order kept); w keeps the original log-weights.
__global__ __launch_bounds__(kRowWaves * kWave) void k_prune_fill_real(
    const Inst *__restrict__ insts, const RowUnit *__restrict__ units, int nunits, double logt,
    const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col, float *__restrict__ wout) {
    extern __shared__ double lvd[];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int u0, u1;
    unit_range(nunits, u0, u1);
    int cur = -1;
    for (int u = u0; u < u1; ++u) {
        const RowUnit un = units[u];
        const Inst &I = insts[un.inst];
        const int n = I.n;
        if (un.inst != cur) {
            __syncthreads();
            for (int j = threadIdx.x; j < n; j += blockDim.x) lvd[j] = (double)I.G[j] + (double)I.gam[j];
            __syncthreads();
            cur = un.inst;
        }
        const int row = un.row0 + wave;
        if (row >= n) continue;
        const int par = I.ctl->iter & 1;
        const double p = real_p(I, I.ctl), wref = (double)I.wref;
        const double f = (double)I.F[par][row] + (double)I.phi[par][row];
        const float *wr = I.Wr + (int64_t)row * I.pitch;
        int64_t pos = row_ptr[row];
        for (int jb = 0; jb < n; jb += kWave) {
            const int j = jb + lane;
            float w = -INFINITY;
            bool keep = false;
            if (j < n) {
                w = wr[j];
                if (w != -INFINITY) keep = real_logx_t(p, w, wref, lvd[j]) + f >= logt;
            }
            const unsigned long long mask = __ballot(keep);
            if (keep) {
                const int before = __popcll(mask & ((1ull << lane) - 1ull));
                col[pos + before] = j;
                wout[pos + before] = w;
            }
            pos += __popcll(mask);
        }
    }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_real_minmax(const float *W, int n, int64_t pitch, int grid, float *part,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_real_minmax, dim3(grid), dim3(256), 0, st, W, n, pitch, part);
    return hipGetLastError();
}
hipError_t launch_init_real(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid, int cold,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_init_real, dim3(grid), dim3(kRowWaves * kWave), 0, st, d_insts, d_units,
                       nunits, cold);
    return hipGetLastError();
}

template <bool NT>
static void row_real(int v4, const Inst *d, const RowUnit *u, int nu, int grid, size_t lds,
                     hipStream_t st, hipEvent_t stop) {
    if (v4)
        launch_stamped(k_row_sweep_real<NT, true>, dim3(grid), dim3(kRowWaves * kWave), lds, st, stop, d,
                       u, nu);
    else
        launch_stamped(k_row_sweep_real<NT, false>, dim3(grid), dim3(kRowWaves * kWave), lds, st, stop, d,
                       u, nu);
}
hipError_t launch_row_sweep_real(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid,
                                 size_t lds_bytes, int nt_loads, int vec4, hipStream_t st,
                                 hipEvent_t stop) {
    if (nt_loads) row_real<true>(vec4, d_insts, d_units, nunits, grid, lds_bytes, st, stop);
    else row_real<false>(vec4, d_insts, d_units, nunits, grid, lds_bytes, st, stop);
    return hipGetLastError();
}

template <bool NT>
static void col_real(int v4, const Inst *d, const ColUnit *u, int nu, int grid, hipStream_t st,
                     hipEvent_t stop) {
    if (v4)
        launch_stamped(k_col_sweep_real<NT, true>, dim3(grid), dim3(kColWaves * kWave), 0, st, stop, d, u,
                       nu);
    else
        launch_stamped(k_col_sweep_real<NT, false>, dim3(grid), dim3(kColWaves * kWave), 0, st, stop, d, u,
                       nu);
}
hipError_t launch_col_sweep_real(const Inst *d_insts, const ColUnit *d_units, int nunits, int grid,
                                 int nt_loads, int vec4, hipStream_t st, hipEvent_t stop) {
    if (nt_loads) col_real<true>(vec4, d_insts, d_units, nunits, grid, st, stop);
    else col_real<false>(vec4, d_insts, d_units, nunits, grid, st, stop);
    return hipGetLastError();
}

hipError_t launch_check_real(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid, int inst,
                             int n, int nseg, double *rsum, double *rmax, double logt, int64_t *counts,
                             int32_t *hint, double *part, double *csum, hipStream_t st) {
    hipLaunchKernelGGL(k_check_rows_real, dim3(grid), dim3(kRowWaves * kWave), sizeof(double) * (size_t)n,
                       st, d_insts, d_units, nunits, rsum, rmax, logt, counts, hint);
    hipLaunchKernelGGL(k_check_cols_real, dim3((n + 255) / 256, nseg), dim3(256), 0, st, d_insts, inst,
                       part);
    hipLaunchKernelGGL(k_check_cols_sum_real, dim3((n + 255) / 256), dim3(256), 0, st, d_insts, inst,
                       part, csum);
    return hipGetLastError();
}

hipError_t launch_prune_fill_real(const Inst *d_insts, const RowUnit *d_units, int nunits, int grid,
                                  double logt, const int64_t *row_ptr, int32_t *col, float *w, int n,
                                  hipStream_t st) {
    hipLaunchKernelGGL(k_prune_fill_real, dim3(grid), dim3(kRowWaves * kWave), sizeof(double) * (size_t)n,
                       st, d_insts, d_units, nunits, logt, row_ptr, col, w);
    return hipGetLastError();
}

hipError_t set_real_attributes() {
    const int lds = (int)(kLdsMaxN * sizeof(double));
    hipError_t e;
    for (const void *f :
         {(const void *)k_row_sweep_real<true, true>, (const void *)k_row_sweep_real<true, false>,
          (const void *)k_row_sweep_real<false, true>, (const void *)k_row_sweep_real<false, false>,
          (const void *)k_check_rows_real, (const void *)k_prune_fill_real})
        if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds)) != hipSuccess)
            return e;
    return hipSuccess;
}

}  // namespace sk
