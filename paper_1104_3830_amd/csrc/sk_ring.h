// Streaming 8-wide int16 chunks (16-byte loads, one chunk per lane) through
// a ring of loads: the row passes (FP64 row check, kept counts, CSR fill,
// absorb into stored K) and the FP64 column check's walk down its rows.
#pragma once

#include "sk_exptab.h"

namespace sk {

// 16-byte loads in flight per lane in the single-wave row passes (input
// scan, FP64 row check, kept counts, CSR fill).
constexpr int kVisitLoads = 4;

// Visits the 8-wide chunks of a row's columns [lo, hi) (lo a multiple of the
// step of kVisitLoads chunks) in column order: body(jj, w) with w the int16
// entries of columns jj..jj+7 of this lane (those past n unspecified; the
// loop bounds are uniform across the wave). The loads run as a ring of
// kVisitLoads per lane: slot k is refilled with the chunk kVisitLoads ahead
// once its own is unpacked; loads past the row's end read its last chunk
// (unused), so every load is issued and each chunk waits for its own load
// only. Slot 0 is unpacked a batch ahead (at the last chunk of the batch
// before), and the full batches run in a loop of their own with the partial
// last batch after it (from the slots already loaded): with either, the
// compiler's count of loads in flight stays exact at every wait.
template <bool NT, class Body>
__device__ __forceinline__ void ring_row_chunks(const int16_t *wr, int n, int lane, int lo, int hi, Body body) {
    constexpr int U = kVisitLoads;
    const int jlast = pad8(n) - 8;
    auto at = [&](int j) { return reinterpret_cast<const int4 *>(wr + min(j, jlast)); };
    int4 v[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        v[k] = gload<NT>(at(lo + k * 512 + lane * 8));
        // issued in slot order, as the loop refills them
        __builtin_amdgcn_sched_barrier(0);
    }
    int w0[8];
    unpack8i(v[0], w0);
    v[0] = gload<NT>(at(lo + U * 512 + lane * 8));
    int jb0 = lo;
    for (; jb0 + U * 512 <= hi; jb0 += U * 512) {
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int jj = jb0 + k * 512 + lane * 8;
            int w[8];
            if (k == 0) {
#pragma unroll
                for (int c = 0; c < 8; ++c) w[c] = w0[c];
            } else {
                unpack8i(v[k], w);
                v[k] = gload<NT>(at(jj + U * 512));
            }
            if (k == U - 1) {
                unpack8i(v[0], w0);
                // kept here, ahead of the refill of its slot (not sunk past it)
                asm volatile("" : "+v"(w0[0]), "+v"(w0[1]), "+v"(w0[2]), "+v"(w0[3]), "+v"(w0[4]), "+v"(w0[5]),
                             "+v"(w0[6]), "+v"(w0[7]));
                v[0] = gload<NT>(at(jj + (U + 1) * 512));
            }
            body(jj, w);
        }
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
        if (jb0 + k * 512 >= hi) break;
        const int jj = jb0 + k * 512 + lane * 8;
        int w[8];
        if (k == 0) {
#pragma unroll
            for (int c = 0; c < 8; ++c) w[c] = w0[c];
        } else {
            unpack8i(v[k], w);
        }
        body(jj, w);
    }
}

// The column check's walk down its rows: chunks m = 0..m_end-1 (m_end
// uniform across the wave) of 8 int16 entries per lane, loaded from at(m)
// (for m >= m_end a valid address whose entries are unused), handed to
// body(m, w) in order. The same ring as the row scans use (kVisitLoads
// loads per lane, each slot refilled once its chunk is unpacked, slot 0
// unpacked a batch ahead, the partial last batch after the loop); here
// scheduling barriers also keep each refill after its slot's unpack, which
// the compiler otherwise hoists, copying the slots at every batch.
template <bool NT, class At, class Body>
__device__ __forceinline__ void ring_col_chunks(int m_end, At at, Body body) {
    constexpr int U = kVisitLoads;
    int4 v[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        v[k] = gload<NT>(at(k));
        __builtin_amdgcn_sched_barrier(0);
    }
    int w0[8];
    unpack8i(v[0], w0);
    __builtin_amdgcn_sched_barrier(0);
    v[0] = gload<NT>(at(U));
    int mb = 0;
    for (; mb + U <= m_end; mb += U) {
#pragma unroll
        for (int k = 0; k < U; ++k) {
            int w[8];
            if (k == 0) {
#pragma unroll
                for (int c = 0; c < 8; ++c) w[c] = w0[c];
            } else {
                unpack8i(v[k], w);
                __builtin_amdgcn_sched_barrier(0);
                v[k] = gload<NT>(at(mb + k + U));
            }
            if (k == U - 1) {
                unpack8i(v[0], w0);
                asm volatile("" : "+v"(w0[0]), "+v"(w0[1]), "+v"(w0[2]), "+v"(w0[3]), "+v"(w0[4]), "+v"(w0[5]),
                             "+v"(w0[6]), "+v"(w0[7]));
                __builtin_amdgcn_sched_barrier(0);
                v[0] = gload<NT>(at(mb + 2 * U));
            }
            body(mb + k, w);
        }
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
        if (mb + k >= m_end) break;
        int w[8];
        if (k == 0) {
#pragma unroll
            for (int c = 0; c < 8; ++c) w[c] = w0[c];
        } else {
            unpack8i(v[k], w);
        }
        body(mb + k, w);
    }
}

}  // namespace sk
