// Device helpers of the real-valued log-weight path (W = log A as float32,
// -inf for a zero entry), shared by its kernels and the end-of-iteration
// kernel.
//
// A term exp(E), E = p (w_ij - wref) + log u_i + log v_j, is formed from the
// exponent in base 2 computed in FP64, E2 = E log2(e), split exactly into
// m = rint(E2) and f = E2 - m in [-1/2, 1/2]: exp(E) = ldexp(exp2(f), m),
// with exp2 of the fraction in FP32. f rounded to FP32 is within 2^-25 of
// itself and the hardware exp2 within ~1 ulp, so every term carries about 2
// FP32 ulp of relative error however large p w is (in FP64 the potentials
// cancel p w to 2^-53 of its magnitude).
#pragma once

#include "sk_rowsweep.h"

namespace sk {

constexpr double kLog2eD = 1.4426950408889634;
constexpr double kLn2D = 0.6931471805599453;

__device__ __forceinline__ float pow2_split(double e2) {
    const double m = rint(e2);
    const float f = (float)(e2 - m);
    // |m| > 400 is far outside the FP32 range either way (0 or +inf)
    const int mi = (int)fmin(fmax(m, -400.0), 400.0);
    return ldexpf(ex2(f), mi);
}

// p of the current stage (of the current iteration, deformed) of a
// real-weight instance.
__device__ __forceinline__ double real_p(const Inst &I, const Ctl *ctl) {
    return (I.deform_a > 0.0 ? ctl->preal : (double)ctl->p) * I.pscale;
}

// Exact max-shifted recompute (Section 4.1.2) of column j of a real-weight
// instance by one workgroup: M = max_i (p w'_ij + log u_i + G_j), shift by
// the integer Mi = rint(M), then log v_j <- G_j - Mi - log sum_i
// exp(p w'_ij + log u_i + G_j - Mi). red: blockDim.x doubles of LDS.
__device__ inline void real_rescue_column(const Inst &I, Ctl *ctl, int j, int npar, double *red) {
    const int n = I.n;
    const double p = real_p(I, ctl);
    const double wref = (double)I.wref;
    const double Gj = (double)I.G[j];
    double m = -INFINITY;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        const float w = I.Wr[(int64_t)r * I.pitch + j];
        if (w == -INFINITY) continue;
        const double lu = (double)I.F[npar][r] + (double)I.phi[npar][r];
        m = fmax(m, fma(p, (double)w - wref, lu + Gj));
    }
    __syncthreads();
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    const double M = red[0];
    __syncthreads();
    const double Mi = M == -INFINITY ? 0.0 : rint(M);
    double s = 0.0;
    if (M != -INFINITY) {
        const double p2 = p * kLog2eD;
        for (int r = threadIdx.x; r < n; r += blockDim.x) {
            const float w = I.Wr[(int64_t)r * I.pitch + j];
            if (w == -INFINITY) continue;
            const double lu = (double)I.F[npar][r] + (double)I.phi[npar][r];
            s += (double)pow2_split(fma(p2, (double)w - wref, (lu + Gj - Mi) * kLog2eD));
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        if (M == -INFINITY) {
            atomicOr(&ctl->err, ERR_EMPTY_COL);
        } else {
            double S = 0.0;
            for (int t = 0; t < (int)blockDim.x; ++t) S += red[t];
            const float gn = -lg2((float)S) * kLn2;
            const float k = rintf(gn);
            I.G[j] = I.G[j] - (int)Mi + (int)k;
            I.gam[j] = gn - k;
        }
    }
    __syncthreads();
}

}  // namespace sk
