// Exact maximum-weight perfect matching of the reduced sparse instance B
// (the sequential exact step of Section 4.2): successive shortest augmenting
// paths with row/column potentials and Dijkstra on a binary heap over the
// sparse bipartite graph, the O(n (m + n log n)) class cited in Section 1.
//
// Costs c_ij = -w_ij (integers, exact in int64). Invariant: reduced costs
// c_ij - u_i - v_j >= 0 on every edge and = 0 on matched edges.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <limits>
#include <queue>
#include <thread>
#include <vector>

#include "sk_hostsolve.h"

namespace {

// The row and column reductions of an instance with at least kParallelNnz
// entries run on up to kReduceThreads host threads.
constexpr int64_t kParallelNnz = int64_t(1) << 17;
constexpr unsigned kReduceThreads = 4;

struct HeapItem {
    int64_t d;
    int32_t col;
    bool operator>(const HeapItem &o) const { return d > o.d || (d == o.d && col > o.col); }
};

}  // namespace

extern "C" sk_status sk_solve_reduced(const sk_csr *csr, int32_t *perm, int64_t *weight) {
    return sk::solve_reduced_seeded(csr, nullptr, perm, weight);
}

// hint (optional, n entries): a column per row to try first when the greedy
// start of the matching is built; any values are accepted.
sk_status sk::solve_reduced_seeded(const sk_csr *csr, const int32_t *hint, int32_t *perm,
                                   int64_t *weight) {
    if (!csr || !perm || !weight || csr->n < 0) return SK_EINVAL;
    const int n = csr->n;
    if (n == 0) {
        *weight = 0;
        return SK_OK;
    }
    if (!csr->row_ptr || (csr->nnz > 0 && (!csr->col || !csr->w))) return SK_EINVAL;
    const int64_t *rp = csr->row_ptr;
    const int32_t *col = csr->col;
    const int16_t *w = csr->w;
    if (rp[0] != 0 || rp[n] != csr->nnz) return SK_EINVAL;
    for (int i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return SK_EINVAL;

    const int64_t INF = std::numeric_limits<int64_t>::max() / 4;
    std::vector<int64_t> u(n), v(n, INF);
    std::vector<int32_t> row_of(n, -1), col_of(n, -1);
    std::vector<int64_t> mpos(n, -1);  // CSR position of row i's matched edge
    // u_i = min_j c_ij makes every reduced cost non-negative with v = 0; the
    // column reduction v_j = min over edges into j of c_ij - u_i keeps them
    // non-negative and makes more edges tight. Both in one pass over the rows
    // (a row's second loop finds it in cache), the entries checked on the way;
    // large instances split the rows over a few threads, each with its own
    // column minima (merged after), and report the first bad row in row order.
    struct Part {
        int r0, r1;
        std::vector<int64_t> vmin;
        int bad_row = -1;
        sk_status bad = SK_OK;
    };
    auto reduce_rows = [&](Part &P, int64_t *vmin) {
        for (int i = P.r0; i < P.r1; ++i) {
            const int64_t e0 = rp[i], e1 = rp[i + 1];
            if (e1 == e0) {  // empty row
                P.bad_row = i;
                P.bad = SK_EINFEASIBLE;
                return;
            }
            int64_t m = INF;
            for (int64_t e = e0; e < e1; ++e) {
                if (col[e] < 0 || col[e] >= n || w[e] == SK_SENTINEL) {
                    P.bad_row = i;
                    P.bad = SK_EINVAL;
                    return;
                }
                m = std::min<int64_t>(m, -(int64_t)w[e]);
            }
            u[i] = m;
            for (int64_t e = e0; e < e1; ++e) {
                const int j = col[e];
                vmin[j] = std::min<int64_t>(vmin[j], -(int64_t)w[e] - m);
            }
        }
    };
    {
        const unsigned hc = std::thread::hardware_concurrency();
        const int T = csr->nnz >= kParallelNnz && hc >= 2 ? (int)std::min<unsigned>(kReduceThreads, hc) : 1;
        std::vector<Part> parts(T);
        for (int t = 0; t < T; ++t) {
            // rows split so that each part holds about nnz / T entries
            const int64_t lo = csr->nnz * t / T, hi = csr->nnz * (t + 1) / T;
            parts[t].r0 = t == 0 ? 0 : (int)(std::lower_bound(rp, rp + n, lo) - rp);
            parts[t].r1 = t == T - 1 ? n : (int)(std::lower_bound(rp, rp + n, hi) - rp);
            if (t > 0) parts[t].vmin.assign(n, INF);
        }
        std::vector<std::thread> th;
        for (int t = 1; t < T; ++t) th.emplace_back([&, t] { reduce_rows(parts[t], parts[t].vmin.data()); });
        reduce_rows(parts[0], v.data());
        for (auto &x : th) x.join();
        for (const Part &P : parts)
            if (P.bad != SK_OK) return P.bad;  // parts are in row order
        for (int t = 1; t < T; ++t)
            for (int j = 0; j < n; ++j) v[j] = std::min(v[j], parts[t].vmin[j]);
    }
    for (int j = 0; j < n; ++j)
        if (v[j] == INF) return SK_EINFEASIBLE;  // empty column
    // maximum matching on the tight edges (reduced cost 0), tested where an
    // edge is looked at: Hopcroft-Karp from a greedy start, in which each row
    // takes its hinted column if that edge is tight and the column still
    // free, else its first free tight column
    auto tight = [&](int i, int64_t e) { return -(int64_t)w[e] - u[i] - v[col[e]] == 0; };
    {
        const int64_t *tp = rp;
        const int32_t *tc = col;
        if (hint)
            for (int i = 0; i < n; ++i) {
                const int32_t h = hint[i];
                if (h < 0 || h >= n || row_of[h] >= 0) continue;
                for (int64_t e = tp[i]; e < tp[i + 1]; ++e)
                    if (tc[e] == h) {
                        if (tight(i, e)) {
                            row_of[h] = i;
                            col_of[i] = h;
                            mpos[i] = e;
                        }
                        break;
                    }
            }
        for (int i = 0; i < n; ++i) {
            if (col_of[i] >= 0) continue;
            for (int64_t e = tp[i]; e < tp[i + 1]; ++e)
                if (row_of[tc[e]] < 0 && tight(i, e)) {
                    row_of[tc[e]] = i;
                    col_of[i] = tc[e];
                    mpos[i] = e;
                    break;
                }
        }
        // Free rows one at a time: a breadth-first search over alternating
        // tight paths that stops at the first free column it reaches, then
        // flips that path. On sparse instances the paths are short and each
        // search looks at few edges; the searches share a budget of edge
        // visits, and whatever is still free when it runs out (or has no
        // tight augmenting path) goes to Hopcroft-Karp below, which keeps
        // the worst case at O(m sqrt(n)) plus the budget.
        {
            std::vector<int32_t> seen(n, -1);  // free row whose search reached column j
            std::vector<int32_t> via_row(n);   // row from which column j was reached
            std::vector<int64_t> via_e(n);     // and the CSR position of that edge
            std::vector<int32_t> fq;
            fq.reserve(n);
            int64_t budget = 4 * (csr->nnz + n);
            for (int s = 0; s < n && budget > 0; ++s) {
                if (col_of[s] >= 0) continue;
                fq.clear();
                fq.push_back(s);
                int found = -1;
                for (size_t h = 0; h < fq.size() && found < 0; ++h) {
                    const int i = fq[h];
                    budget -= tp[i + 1] - tp[i];
                    for (int64_t e = tp[i]; e < tp[i + 1]; ++e) {
                        const int j = tc[e];
                        if (seen[j] == s || !tight(i, e)) continue;
                        seen[j] = s;
                        via_row[j] = i;
                        via_e[j] = e;
                        if (row_of[j] < 0) {
                            found = j;
                            break;
                        }
                        fq.push_back(row_of[j]);
                    }
                }
                for (int j = found; j >= 0;) {  // flip the path back to s
                    const int i = via_row[j];
                    const int prev = col_of[i];
                    row_of[j] = i;
                    col_of[i] = j;
                    mpos[i] = via_e[j];
                    if (i == s) break;
                    j = prev;
                }
            }
        }
        const int NIL = std::numeric_limits<int>::max();
        std::vector<int> dist(n), q(n), stack;
        std::vector<int64_t> it(n);
        stack.reserve(n);
        for (;;) {
            // BFS layers from the free rows
            int qh = 0, qt = 0;
            for (int i = 0; i < n; ++i) {
                if (col_of[i] < 0) {
                    dist[i] = 0;
                    q[qt++] = i;
                } else {
                    dist[i] = NIL;
                }
            }
            // layers up to the first one that reaches a free column
            bool found = false;
            int limit = NIL;
            while (qh < qt) {
                const int i = q[qh++];
                if (dist[i] > limit) break;
                for (int64_t e = tp[i]; e < tp[i + 1]; ++e) {
                    if (!tight(i, e)) continue;
                    const int i2 = row_of[tc[e]];
                    if (i2 < 0) {
                        found = true;
                        limit = dist[i];
                    } else if (dist[i2] == NIL) {
                        dist[i2] = dist[i] + 1;
                        q[qt++] = i2;
                    }
                }
            }
            if (!found) break;
            // vertex-disjoint shortest augmenting paths, iterative DFS
            for (int i = 0; i < n; ++i) it[i] = tp[i];
            for (int s0 = 0; s0 < n; ++s0) {
                if (col_of[s0] >= 0 || dist[s0] != 0) continue;
                stack.clear();
                stack.push_back(s0);
                while (!stack.empty()) {
                    const int i = stack.back();
                    if (it[i] == tp[i + 1]) {
                        dist[i] = NIL;  // dead end
                        stack.pop_back();
                        continue;
                    }
                    if (!tight(i, it[i])) {
                        ++it[i];
                        continue;
                    }
                    const int j = tc[it[i]];
                    const int i2 = row_of[j];
                    if (i2 < 0) {
                        for (int r : stack) {
                            const int jj = tc[it[r]];
                            col_of[r] = jj;
                            row_of[jj] = r;
                            mpos[r] = it[r];
                        }
                        for (int r : stack) dist[r] = NIL;  // used this phase
                        stack.clear();
                        break;
                    }
                    if (dist[i2] != NIL && dist[i2] == dist[i] + 1) {
                        stack.push_back(i2);
                    } else {
                        ++it[i];
                    }
                }
            }
        }
    }

    std::vector<int64_t> dist(n, INF);
    std::vector<int32_t> pred(n, -1);  // row from which column j was reached
    std::vector<int64_t> pred_e(n, -1);  // and the CSR position of that edge
    std::vector<char> done(n, 0);
    std::vector<int32_t> touched, finalized;
    touched.reserve(n);
    finalized.reserve(n);
    std::priority_queue<HeapItem, std::vector<HeapItem>, std::greater<HeapItem>> heap;

    for (int s = 0; s < n; ++s) {
        if (col_of[s] >= 0) continue;
        for (int j : touched) {
            dist[j] = INF;
            pred[j] = -1;
            done[j] = 0;
        }
        touched.clear();
        finalized.clear();
        while (!heap.empty()) heap.pop();
        // relax the edges of row s (distance of s is 0)
        for (int64_t e = rp[s]; e < rp[s + 1]; ++e) {
            const int j = col[e];
            const int64_t d = -(int64_t)w[e] - u[s] - v[j];
            if (dist[j] == INF) touched.push_back(j);
            if (d < dist[j]) {
                dist[j] = d;
                pred[j] = s;
                pred_e[j] = e;
                heap.push({d, j});
            }
        }
        int target = -1;
        int64_t D = 0;
        while (!heap.empty()) {
            const HeapItem it = heap.top();
            heap.pop();
            const int j = it.col;
            if (done[j] || it.d != dist[j]) continue;
            done[j] = 1;
            finalized.push_back(j);
            if (row_of[j] < 0) {
                target = j;
                D = it.d;
                break;
            }
            const int i = row_of[j];
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
                const int k = col[e];
                if (done[k]) continue;
                const int64_t nd = it.d + (-(int64_t)w[e] - u[i] - v[k]);
                if (dist[k] == INF) touched.push_back(k);
                if (nd < dist[k]) {
                    dist[k] = nd;
                    pred[k] = i;
                    pred_e[k] = e;
                    heap.push({nd, k});
                }
            }
        }
        if (target < 0) return SK_EINFEASIBLE;
        // potential update keeps reduced costs >= 0 and the new path tight
        for (int j : finalized) {
            const int64_t delta = D - dist[j];
            if (delta == 0) continue;
            v[j] -= delta;
            const int i = row_of[j];
            if (i >= 0) u[i] += delta;
        }
        u[s] += D;
        // augment along pred
        int j = target;
        for (;;) {
            const int i = pred[j];
            const int prev = col_of[i];
            row_of[j] = i;
            col_of[i] = j;
            mpos[i] = pred_e[j];
            if (i == s) break;
            j = prev;
        }
    }
    // the weight from the matched edges themselves
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
        const int64_t e = mpos[i];
        if (e < rp[i] || e >= rp[i + 1] || col[e] != col_of[i]) return SK_EINVAL;
        perm[i] = col_of[i];
        total += w[e];
    }
    *weight = total;
    return SK_OK;
}
