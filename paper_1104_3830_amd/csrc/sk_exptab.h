// Exact integer exponents and the LDS table of exp(E) shared by the
// log-domain kernels (sweeps, single pass, exact recompute).
#pragma once

#include <climits>

#include "sk_internal.h"

namespace sk {

// Every exponent the sweeps evaluate splits exactly into an integer part
// E_ij = p w_ij + F_i + G_j and the fractions phi_i, gam_j:
//   x_ij = exp(E_ij) * exp(phi_i) * exp(gam_j).
// exp(E) for integer E is read from a table in LDS, correctly rounded to
// float32; the fraction factors are one value per row and per column. Entries
// with E <= kTabLo contribute exp(-88) < 2^-126 (dropped: a sum in the safe
// range [2^-64, 2^64] of at most 16384 such terms changes by less than one
// part in 2^40); E >= kTabHi reads +inf, which sends the row or column to the
// exact max-shifted recompute. Integer arithmetic is exact: with p <= 2048
// and |w| < 2^15, |4 E| < 2^31.
constexpr int kTabLo = -88;
constexpr int kTabHi = 80;
constexpr int kTabN = kTabHi - kTabLo + 1;  // 169 entries
constexpr int kTabMaxOff = 4 * (kTabN - 1);  // byte offset of the +inf entry

__device__ __forceinline__ void fill_exp_table(float *tab) {
    for (int k = threadIdx.x; k < kTabN; k += blockDim.x) {
        float v;
        if (k == 0) v = 0.f;
        else if (k == kTabN - 1) v = INFINITY;
        else v = (float)exp((double)(k + kTabLo));
        tab[k] = v;
    }
}

// Table read at a byte offset already clamped to [0, kTabMaxOff].
__device__ __forceinline__ float tab_at(const float *tab, int off) {
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(tab) + off);
}

// Byte offset of exp(E) with 4 E - 4 kTabLo = 4 p w + A + B (A, B prescaled).
__device__ __forceinline__ int tab_off(int p4, int w, int A, int B) {
    const int t = __mul24(p4, w) + A + B;
    return min(max(t, 0), kTabMaxOff);
}

// Unpacks 8 int16 from a 16-byte vector as int32.
__device__ __forceinline__ void unpack8i(const int4 v, int (&w)[8]) {
    w[0] = (int)(short)(v.x & 0xffff); w[1] = v.x >> 16;
    w[2] = (int)(short)(v.y & 0xffff); w[3] = v.y >> 16;
    w[4] = (int)(short)(v.z & 0xffff); w[5] = v.z >> 16;
    w[6] = (int)(short)(v.w & 0xffff); w[7] = v.w >> 16;
}

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
    return v;
}

}  // namespace sk
