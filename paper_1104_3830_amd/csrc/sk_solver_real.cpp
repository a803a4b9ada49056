// Exact maximum-weight perfect matching of a reduced instance with real
// (float) weights, the exact step of Section 4.2 for real-valued log-weights.
// Host code only, no device calls.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <functional>
#include <queue>
#include <vector>

#include "sk_hostsolve.h"

// Sparse shortest augmenting paths (Dijkstra with row and column potentials)
// minimising sum c with c = -w, i.e. maximising sum w. Invariant: reduced
// costs c_ij - u_i - v_j >= 0 on every entry and = 0 on matched ones. After a
// search from free row i0 that reaches a free column at distance d*, the
// potentials of the nodes it finalised move by (their distance - d*), which
// keeps the invariant and makes the augmenting path tight.
sk_status sk::solve_real_impl(int n, const int64_t *rp, const int32_t *col, const float *w,
                              const int32_t *hint, int32_t *perm, double *weight) {
    if (n <= 0) return SK_EINVAL;
    const double INF = INFINITY;
    std::vector<double> u((size_t)n), v((size_t)n, 0.0), dist((size_t)n, INF);
    std::vector<int32_t> row_of((size_t)n, -1), col_of((size_t)n, -1), pred((size_t)n, -1);
    std::vector<int64_t> edge_of((size_t)n, -1), pred_edge((size_t)n, -1);
    std::vector<char> done((size_t)n, 0);
    for (int i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) return SK_EINVAL;
        if (rp[i + 1] == rp[i]) return SK_EINFEASIBLE;
        double m = INF;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (col[e] < 0 || col[e] >= n || !(w[e] > -INFINITY && w[e] < INFINITY)) return SK_EINVAL;
            m = std::min(m, -(double)w[e]);
        }
        u[i] = m;
    }
    // greedy start on tight entries, the hinted column first
    for (int i = 0; i < n; ++i) {
        int64_t pick = -1;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (-(double)w[e] != u[i] || row_of[col[e]] >= 0) continue;
            if (pick < 0 || (hint && col[e] == hint[i])) pick = e;
        }
        if (pick >= 0) {
            col_of[i] = col[pick];
            row_of[col[pick]] = i;
            edge_of[i] = pick;
        }
    }
    using Item = std::pair<double, int32_t>;
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
    std::vector<int32_t> touched, finalized;
    for (int i0 = 0; i0 < n; ++i0) {
        if (col_of[i0] >= 0) continue;
        auto relax = [&](int i, double di) {
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
                const int j = col[e];
                if (done[j]) continue;
                const double r = std::max(0.0, -(double)w[e] - u[i] - v[j]);
                const double nd = di + r;
                if (nd < dist[j]) {
                    if (dist[j] == INF) touched.push_back(j);
                    dist[j] = nd;
                    pred[j] = i;
                    pred_edge[j] = e;
                    heap.push({nd, j});
                }
            }
        };
        relax(i0, 0.0);
        int sink = -1;
        double dsink = 0.0;
        while (!heap.empty()) {
            const Item it = heap.top();
            heap.pop();
            const int j = it.second;
            if (done[j] || it.first > dist[j]) continue;
            done[j] = 1;
            finalized.push_back(j);
            if (row_of[j] < 0) {
                sink = j;
                dsink = it.first;
                break;
            }
            relax(row_of[j], it.first);
        }
        if (sink < 0) return SK_EINFEASIBLE;
        for (int j : finalized) {
            if (j == sink) continue;
            const double delta = dist[j] - dsink;  // <= 0
            v[j] += delta;
            u[row_of[j]] -= delta;
        }
        u[i0] += dsink;
        // augment along the search tree
        for (int j = sink;;) {
            const int i = pred[j];
            const int jn = col_of[i];
            col_of[i] = j;
            row_of[j] = i;
            edge_of[i] = pred_edge[j];
            if (i == i0) break;
            j = jn;
        }
        for (int j : touched) dist[j] = INF;
        for (int j : finalized) done[j] = 0;
        touched.clear();
        finalized.clear();
        while (!heap.empty()) heap.pop();
    }
    double total = 0.0;
    for (int i = 0; i < n; ++i) {
        perm[i] = col_of[i];
        total += (double)w[edge_of[i]];
    }
    *weight = total;
    return SK_OK;
}

extern "C" sk_status sk_solve_reduced_real(const sk_csr_real *csr, int32_t *perm, double *weight) {
    if (!csr || !perm || !weight || !csr->row_ptr || csr->n < 1) return SK_EINVAL;
    if (csr->row_ptr[0] != 0 || csr->row_ptr[csr->n] != csr->nnz) return SK_EINVAL;
    if (csr->nnz > 0 && (!csr->col || !csr->w)) return SK_EINVAL;
    return sk::solve_real_impl(csr->n, csr->row_ptr, csr->col, csr->w, nullptr, perm, weight);
}
