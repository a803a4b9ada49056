// Host exact solvers (integer and real weights) driven on random and
// malformed reduced instances; built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitize.py. Prints "ok" and
// exits 0 when every check holds.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "../../include/sk.h"

namespace {

int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::printf("check failed at line %d: %s\n", __LINE__, #c);       \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

struct Inst {
    int n = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> col;
    std::vector<int16_t> w;
    std::vector<float> wf;
};

// Random sparse instance: each entry present with probability dens, weight
// uniform on [-wmax, wmax]; columns of a row in increasing order.
Inst random_inst(std::mt19937_64 &rng, int n, double dens, int wmax) {
    Inst I;
    I.n = n;
    I.rp.push_back(0);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    std::uniform_int_distribution<int> Wd(-wmax, wmax);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j)
            if (U(rng) < dens) {
                I.col.push_back(j);
                const int w = Wd(rng);
                I.w.push_back((int16_t)w);
                I.wf.push_back((float)w);
            }
        I.rp.push_back((int64_t)I.col.size());
    }
    return I;
}

// Largest sum of w over permutations inside the pattern; false if none.
bool brute(const Inst &I, int64_t &best) {
    const int n = I.n;
    std::vector<int64_t> dense((size_t)n * n, INT64_MIN);
    for (int i = 0; i < n; ++i)
        for (int64_t e = I.rp[i]; e < I.rp[i + 1]; ++e) dense[(size_t)i * n + I.col[e]] = I.w[e];
    std::vector<int> p(n);
    for (int i = 0; i < n; ++i) p[i] = i;
    bool any = false;
    best = INT64_MIN;
    do {
        int64_t s = 0;
        bool ok = true;
        for (int i = 0; i < n && ok; ++i) {
            const int64_t v = dense[(size_t)i * n + p[i]];
            if (v == INT64_MIN) ok = false;
            else s += v;
        }
        if (ok) {
            any = true;
            best = std::max(best, s);
        }
    } while (std::next_permutation(p.begin(), p.end()));
    return any;
}

// perm is a permutation whose entries lie in the pattern, and the weights
// of those entries add up to weight.
bool valid_perm(const Inst &I, const std::vector<int32_t> &perm, int64_t weight) {
    std::vector<char> seen(I.n, 0);
    int64_t s = 0;
    for (int i = 0; i < I.n; ++i) {
        const int j = perm[i];
        if (j < 0 || j >= I.n || seen[j]) return false;
        seen[j] = 1;
        bool found = false;
        for (int64_t e = I.rp[i]; e < I.rp[i + 1]; ++e)
            if (I.col[e] == j) {
                s += I.w[e];
                found = true;
            }
        if (!found) return false;
    }
    return s == weight;
}

sk_status solve_int(Inst &I, std::vector<int32_t> &perm, int64_t &weight) {
    sk_csr c{I.n, (int64_t)I.col.size(), I.rp.data(), I.col.data(), I.w.data()};
    perm.assign(std::max(I.n, 1), -1);
    return sk_solve_reduced(&c, perm.data(), &weight);
}

sk_status solve_real(Inst &I, std::vector<int32_t> &perm, double &weight) {
    sk_csr_real c{I.n, (int64_t)I.col.size(), I.rp.data(), I.col.data(), I.wf.data()};
    perm.assign(std::max(I.n, 1), -1);
    return sk_solve_reduced_real(&c, perm.data(), &weight);
}

void small_vs_brute_force() {
    std::mt19937_64 rng(11);
    for (int trial = 0; trial < 400; ++trial) {
        const int n = 1 + trial % 7;
        const double dens = 0.3 + 0.1 * (trial % 7);
        Inst I = random_inst(rng, n, dens, 1000);
        int64_t best = 0;
        const bool feasible = brute(I, best);
        std::vector<int32_t> perm;
        int64_t weight = 0;
        const sk_status st = solve_int(I, perm, weight);
        std::vector<int32_t> permr;
        double wr = 0;
        const sk_status str = solve_real(I, permr, wr);
        if (!feasible) {
            CHECK(st == SK_EINFEASIBLE);
            CHECK(str == SK_EINFEASIBLE);
            continue;
        }
        CHECK(st == SK_OK);
        CHECK(weight == best);
        CHECK(valid_perm(I, perm, weight));
        CHECK(str == SK_OK);
        CHECK(wr == (double)best);
        CHECK(valid_perm(I, permr, best));
    }
}

void malformed() {
    std::mt19937_64 rng(3);
    Inst good = random_inst(rng, 6, 0.7, 100);
    auto expect_inval = [&](Inst I) {
        std::vector<int32_t> perm;
        int64_t w = 0;
        double wr = 0;
        CHECK(solve_int(I, perm, w) == SK_EINVAL);
        CHECK(solve_real(I, perm, wr) == SK_EINVAL);
    };
    {
        Inst I = good;  // row pointers not starting at 0
        for (auto &x : I.rp) x += 1;
        expect_inval(I);
    }
    {
        Inst I = good;  // decreasing row pointers inside the range
        std::swap(I.rp[2], I.rp[3]);
        if (I.rp[2] != I.rp[3]) expect_inval(I);
    }
    {
        Inst I = good;  // column past n
        I.col[0] = I.n;
        expect_inval(I);
    }
    {
        Inst I = good;  // negative column
        I.col[I.col.size() - 1] = -1;
        expect_inval(I);
    }
    {
        // nnz that disagrees with the row pointers
        Inst I = good;
        sk_csr c{I.n, (int64_t)I.col.size() + 1, I.rp.data(), I.col.data(), I.w.data()};
        std::vector<int32_t> perm(I.n);
        int64_t w = 0;
        CHECK(sk_solve_reduced(&c, perm.data(), &w) == SK_EINVAL);
        sk_csr_real cr{I.n, (int64_t)I.col.size() + 1, I.rp.data(), I.col.data(), I.wf.data()};
        double wr = 0;
        CHECK(sk_solve_reduced_real(&cr, perm.data(), &wr) == SK_EINVAL);
    }
    {
        Inst I = good;  // sentinel weight (an absent entry listed as present)
        I.w[1] = SK_SENTINEL;
        std::vector<int32_t> perm;
        int64_t w = 0;
        CHECK(solve_int(I, perm, w) == SK_EINVAL);
    }
    for (float bad : {NAN, INFINITY, -INFINITY}) {
        Inst I = good;  // non-finite real weight
        I.wf[2] = bad;
        std::vector<int32_t> perm;
        double wr = 0;
        CHECK(solve_real(I, perm, wr) == SK_EINVAL);
    }
    {
        // null arrays
        std::vector<int32_t> perm(4);
        int64_t w = 0;
        double wr = 0;
        CHECK(sk_solve_reduced(nullptr, perm.data(), &w) == SK_EINVAL);
        CHECK(sk_solve_reduced_real(nullptr, perm.data(), &wr) == SK_EINVAL);
        Inst I = good;
        sk_csr c{I.n, (int64_t)I.col.size(), I.rp.data(), nullptr, I.w.data()};
        CHECK(sk_solve_reduced(&c, perm.data(), &w) == SK_EINVAL);
    }
    {
        // the empty instance: an empty matching of weight 0 (integer entry
        // point); the real entry point asks for n >= 1
        Inst I;
        I.rp.push_back(0);
        std::vector<int32_t> perm;
        int64_t w = 7;
        CHECK(solve_int(I, perm, w) == SK_OK && w == 0);
        double wr = 0;
        CHECK(solve_real(I, perm, wr) == SK_EINVAL);
    }
    {
        Inst I = good;  // a row with no entry
        const int64_t cut = I.rp[3] - I.rp[2];
        I.col.erase(I.col.begin() + I.rp[2], I.col.begin() + I.rp[3]);
        I.w.erase(I.w.begin() + I.rp[2], I.w.begin() + I.rp[3]);
        I.wf.erase(I.wf.begin() + I.rp[2], I.wf.begin() + I.rp[3]);
        for (int i = 3; i <= I.n; ++i) I.rp[i] -= cut;
        std::vector<int32_t> perm;
        int64_t w = 0;
        double wr = 0;
        CHECK(solve_int(I, perm, w) == SK_EINFEASIBLE);
        CHECK(solve_real(I, perm, wr) == SK_EINFEASIBLE);
    }
}

// Larger instances: a planted permutation (a perfect matching exists) plus
// random entries; enough entries that the row and column reductions split
// over host threads. The integer and real solvers must agree on the optimum.
void large_agree() {
    std::mt19937_64 rng(29);
    for (int trial = 0; trial < 3; ++trial) {
        const int n = 3000 + 500 * trial;
        const int per_row = 48;
        std::vector<int> sigma(n);
        for (int i = 0; i < n; ++i) sigma[i] = i;
        std::shuffle(sigma.begin(), sigma.end(), rng);
        Inst I;
        I.n = n;
        I.rp.push_back(0);
        std::uniform_int_distribution<int> C(0, n - 1), Wd(0, 1000);
        for (int i = 0; i < n; ++i) {
            std::vector<int> cs{sigma[i]};
            for (int k = 0; k < per_row; ++k) cs.push_back(C(rng));
            std::sort(cs.begin(), cs.end());
            cs.erase(std::unique(cs.begin(), cs.end()), cs.end());
            for (int j : cs) {
                const int w = trial == 2 ? 1000 : Wd(rng);  // the last: every entry tight
                I.col.push_back(j);
                I.w.push_back((int16_t)w);
                I.wf.push_back((float)w);
            }
            I.rp.push_back((int64_t)I.col.size());
        }
        CHECK(I.col.size() >= (size_t)1 << 17);
        std::vector<int32_t> perm, permr;
        int64_t weight = 0;
        double wr = 0;
        CHECK(solve_int(I, perm, weight) == SK_OK);
        CHECK(valid_perm(I, perm, weight));
        CHECK(solve_real(I, permr, wr) == SK_OK);
        CHECK(wr == (double)weight);
        CHECK(valid_perm(I, permr, weight));
        if (trial == 2) CHECK(weight == (int64_t)1000 * n);
    }
}

// Rows that leave most single-row searches without a free column, so their
// shared edge budget runs out and the rest of the matching takes the
// layered phase: block A (2k rows) complete onto k columns at weight 100,
// each A row also reaching a column of its own at weight 0; k rows B each
// reaching the own columns of two A rows at weight 50.
void budget_exhaustion() {
    const int k = 400, nA = 2 * k, n = nA + k;
    Inst I;
    I.n = n;
    I.rp.push_back(0);
    for (int i = 0; i < nA; ++i) {
        for (int j = 0; j < k; ++j) {
            I.col.push_back(j);
            I.w.push_back(100);
            I.wf.push_back(100.f);
        }
        I.col.push_back(k + i);
        I.w.push_back(0);
        I.wf.push_back(0.f);
        I.rp.push_back((int64_t)I.col.size());
    }
    for (int t = 0; t < k; ++t) {
        for (int c : {k + 2 * t, k + 2 * t + 1}) {
            I.col.push_back(c);
            I.w.push_back(50);
            I.wf.push_back(50.f);
        }
        I.rp.push_back((int64_t)I.col.size());
    }
    std::vector<int32_t> perm, permr;
    int64_t weight = 0;
    double wr = 0;
    CHECK(solve_int(I, perm, weight) == SK_OK);
    CHECK(weight == (int64_t)k * 100 + (int64_t)k * 50);
    CHECK(valid_perm(I, perm, weight));
    CHECK(solve_real(I, permr, wr) == SK_OK);
    CHECK(wr == (double)weight);
}

}  // namespace

int main() {
    small_vs_brute_force();
    malformed();
    large_agree();
    budget_exhaustion();
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
