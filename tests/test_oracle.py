"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each check is a value printed
in the paper, a closed form, an invariant, or brute force on a tiny input.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import skgen
from oracle import brute
from tests.golden import fixtures


# ---------------------------------------------------------------- worked examples

def test_example_3x3_stopping_rule():
    """Section 2.3 example: the printed X(10) is the first column-stochastic
    iterate with max_i |r_i - 1| < 1e-4 (rows first); it matches to within half
    a unit of the 7th printed decimal, and the iterate before does not stop."""
    fx = fixtures.load("example_3x3.txt")
    B = oracle.log_of(fx["A"])
    u, v, m, res = oracle.sinkhorn(B, fx["p"], 1e-4, 10**6)
    X = oracle.scaled_matrix(B, fx["p"], u, v)
    assert m == 106
    assert res < 1e-4
    assert np.abs(X - fx["X"]).max() <= 5e-8
    # one iteration fewer is not yet 1e-4-bistochastic
    u2, v2, m2, res2 = oracle.sinkhorn(B, fx["p"], 0.0, 105)
    assert m2 == 105 and res2 >= 1e-4


def test_example_3x3_limit_differs_from_printed():
    """The converged X(10) differs from the printed (stopped) iterate by ~5e-5,
    which is what makes the example pin the stopping rule."""
    fx = fixtures.load("example_3x3.txt")
    B = oracle.log_of(fx["A"])
    u, v, m, res = oracle.sinkhorn(B, fx["p"], 1e-13, 10**6)
    X = oracle.scaled_matrix(B, fx["p"], u, v)
    d = np.abs(X - fx["X"]).max()
    assert 1e-5 < d < 1e-4
    r, c = oracle.sums(B, fx["p"], u, v)
    assert np.abs(r - 1).max() < 1e-12 and np.abs(c - 1).max() < 1e-12


def test_example_5x5_scaled_matrix_and_support():
    """Section 4.2 example: X(50) printed to 2 digits from a matrix printed to
    3 decimals. With the same stopping rule at eps = 1e-2 the entries agree to
    within 0.2 decades everywhere (median 0.02) and 6% on entries >= 1e-3, the
    supports at t = 1/n and t = 1e-4 coincide, and the bold entries are the
    brute-force optimum."""
    fx = fixtures.load("example_5x5.txt")
    A, P = fx["A"], fx["X"]
    B = oracle.log_of(A)
    u, v, m, res = oracle.sinkhorn(B, fx["p"], 1e-2, 10**6)
    X = oracle.scaled_matrix(B, fx["p"], u, v)
    d = np.abs(np.log10(X) - np.log10(P))
    assert np.median(d) < 0.02 and d.max() < 0.2
    big = P >= 1e-3
    assert (np.abs(X - P)[big] / P[big]).max() < 0.06
    n = A.shape[0]
    for t in (1.0 / n, 1e-4):
        assert np.array_equal(oracle.prune(B, fx["p"], u, v, t), P >= t)
    opt = [int(k) - 1 for k in fx["opt"][0]]
    best, winners = brute.all_optima(B)
    assert winners == [tuple(opt)]
    assert all(X[i, opt[i]] > 0.9 for i in range(n))


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("p", [0.5, 1.0, 3.0, 10.0])
def test_2x2_closed_form(p):
    """For 2x2 the bistochastic X(p) is [[x,1-x],[1-x,x]] and ratio invariance
    gives x/(1-x) = (a11 a22 / (a12 a21))^(p/2)."""
    A = np.array([[2.0, 0.7], [1.3, 0.9]])
    B = oracle.log_of(A)
    u, v, m, res = oracle.sinkhorn(B, p, 1e-15, 10**5)
    X = oracle.scaled_matrix(B, p, u, v)
    R = (A[0, 0] * A[1, 1] / (A[0, 1] * A[1, 0])) ** (p / 2)
    x = R / (1 + R)
    assert np.allclose(X, [[x, 1 - x], [1 - x, x]], atol=1e-13, rtol=0)


def test_uniform_matrix_is_scaled_to_1_over_n():
    """A constant matrix scales to the uniform bistochastic matrix J/n in one step."""
    n = 7
    B = np.full((n, n), 0.3)
    u, v, m, res = oracle.sinkhorn(B, 4.0, 1e-14, 10)
    assert m == 1
    assert np.allclose(oracle.scaled_matrix(B, 4.0, u, v), 1.0 / n, atol=1e-15)


def test_permutation_ratio_invariance_any_iterate():
    """omega_sigma(X)/omega_pi(X) = (omega_sigma(A)/omega_pi(A))^p for every
    iterate (Section 3.3): it holds for any diagonal scaling of A^(p). Checked
    on all pairs of permutations of a 5x5 matrix after 1, 2 and 7 iterations,
    and on 2x2 minors of an 8x8 matrix."""
    rng = np.random.default_rng(3)
    A = rng.uniform(0.1, 1.0, (5, 5))
    B = oracle.log_of(A)
    p = 2.5
    bw = brute.permutation_weights(B)
    perms = list(bw)
    for iters in (1, 2, 7):
        u, v, m, res = oracle.sinkhorn(B, p, 0.0, iters)
        X = oracle.scaled_matrix(B, p, u, v)
        xw = brute.permutation_weights(np.log(X))
        for s, q in zip(perms[::7], perms[3::11]):
            assert math.isclose(xw[s] - xw[q], p * (bw[s] - bw[q]), rel_tol=0, abs_tol=1e-11)
    W = skgen.uniform_weights(8, 0, 9, seed=11)
    B = oracle.log_weights(W)
    u, v, m, res = oracle.sinkhorn(B, 1.5, 0.0, 3)
    L = np.log(oracle.scaled_matrix(B, 1.5, u, v))
    for (i, k), (j, l) in itertools.product(itertools.combinations(range(8), 2), repeat=2):
        lhs = L[i, j] + L[k, l] - L[i, l] - L[k, j]
        rhs = 1.5 * (B[i, j] + B[k, l] - B[i, l] - B[k, j])
        assert abs(lhs - rhs) < 1e-10


def test_uniqueness_of_scaling_start_independent():
    """X(p) is unique (Theorem prop-borweinlewisnussbaum): Sinkhorn from a cold
    start and from random scalings reaches the same matrix; the raw scalings
    differ only by a constant (Section 2.1 theorem)."""
    rng = np.random.default_rng(5)
    B = oracle.log_of(rng.uniform(0.05, 1.0, (9, 9)))
    p = 3.0
    u1, v1, _, r1 = oracle.sinkhorn(B, p, 1e-14, 10**5)
    u2, v2, _, r2 = oracle.sinkhorn(B, p, 1e-14, 10**5, ubar=rng.normal(size=9),
                                    vbar=rng.normal(size=9) * 5)
    X1 = oracle.scaled_matrix(B, p, u1, v1)
    X2 = oracle.scaled_matrix(B, p, u2, v2)
    assert np.abs(X1 - X2).max() < 1e-12
    d = u1 - u2
    assert np.ptp(d) < 1e-12 and np.abs((v1 - v2) + d[0]).max() < 1e-12


def test_entropy_maximality():
    """X(p) maximises J_p(X) = sum x_ij b_ij + p^-1 S(X) over bistochastic
    matrices (eq. pentropyopt): J_p(X(p)) >= J_p(Y) for random bistochastic Y
    (convex combinations of permutation matrices), and for small moves
    along directions that keep the row/column sums."""
    rng = np.random.default_rng(9)
    n, p = 5, 2.0
    B = oracle.log_of(rng.uniform(0.1, 1.0, (n, n)))

    def J(X):
        with np.errstate(divide="ignore", invalid="ignore"):
            ent = -np.where(X > 0, X * np.log(X), 0.0).sum()
        return (X * B).sum() + ent / p

    u, v, _, _ = oracle.sinkhorn(B, p, 1e-14, 10**5)
    X = oracle.scaled_matrix(B, p, u, v)
    jx = J(X)
    perms = list(itertools.permutations(range(n)))
    for _ in range(200):
        w = rng.dirichlet(np.ones(6))
        Y = np.zeros((n, n))
        for wk, k in zip(w, rng.choice(len(perms), 6, replace=False)):
            Y[np.arange(n), perms[k]] += wk
        assert J(Y) <= jx + 1e-12
    for _ in range(50):
        i, k = rng.choice(n, 2, replace=False)
        j, l = rng.choice(n, 2, replace=False)
        D = np.zeros((n, n))
        D[i, j] = D[k, l] = 1.0
        D[i, l] = D[k, j] = -1.0
        for h in (1e-3, -1e-3):
            assert J(X + h * D) < jx


# ---------------------------------------------------------------- convergence in p

def test_convergence_to_unique_optimum_along_p():
    """Corollary of Theorem thm:prop-converge1: with a unique optimal
    permutation, X(p) tends to its permutation matrix; the distance decreases
    along the ladder and the entries off the optimum decay."""
    W, sigma = skgen.planted(12, seed=2, lo=0, hi=10, bonus=1)
    B = oracle.log_weights(W)
    P = np.zeros((12, 12))
    P[np.arange(12), sigma] = 1.0
    dist = []
    ubar = vbar = None
    for p in (0.25, 0.5, 1, 2, 4, 8):
        ubar, vbar, m, res = oracle.sinkhorn(B, p, 1e-9, 2 * 10**5, ubar, vbar)
        dist.append(np.abs(oracle.scaled_matrix(B, p, ubar, vbar) - P).max())
    assert all(a > b for a, b in zip(dist, dist[1:]))
    assert dist[-1] < 1e-3


def test_limit_with_two_optima_is_their_average():
    """Theorem thm:prop-converge1: with exactly two optimal permutations that
    differ by a transposition, X(p) tends to the max-entropy point of their
    hull, which is their average."""
    b = np.array([[5.0, 5.0, 0.0], [5.0, 5.0, 1.0], [0.0, 2.0, 6.0]])
    best, winners = brute.all_optima(b)
    assert len(winners) == 2
    u, v, m, res = oracle.sinkhorn(b, 12.0, 1e-14, 10**6)
    X = oracle.scaled_matrix(b, 12.0, u, v)
    target = np.zeros((3, 3))
    for w in winners:
        target[np.arange(3), w] += 0.5
    assert np.abs(X - target).max() < 1e-4


def test_sums_reach_1e12_on_reachable_cases():
    """Row and column sums equal 1 within 1e-12 where Sinkhorn converges fast
    enough to reach it (small p on random weights; planted optimum)."""
    W = skgen.uniform_weights(64, 0, 100, seed=0)
    B = oracle.log_weights(W)
    u, v, m, res = oracle.sinkhorn(B, 0.05, 1e-13, 10**5)
    r, c = oracle.sums(B, 0.05, u, v)
    assert np.abs(r - 1).max() < 1e-12 and np.abs(c - 1).max() < 1e-12
    W, _ = skgen.planted(64, seed=1, lo=0, hi=100, bonus=20)
    B = oracle.log_weights(W)
    u, v, it, res = oracle.scale_ladder(B, [1, 2, 4], 1e-13, 10**5)
    r, c = oracle.sums(B, 4, u, v)
    assert np.abs(r - 1).max() < 1e-12 and np.abs(c - 1).max() < 1e-12


# ---------------------------------------------------------------- exact solver

@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 8])
def test_hungarian_vs_brute_force(n):
    rng = np.random.default_rng(n)
    for trial in range(6):
        w = rng.integers(-20, 21, (n, n))
        allowed = rng.random((n, n)) < (0.5 if trial % 2 else 1.0)
        b = np.where(allowed, w.astype(float), -np.inf)
        best, winners = brute.all_optima(b)
        if best == -math.inf:
            with pytest.raises(oracle.Infeasible):
                oracle.hungarian(w, allowed)
            continue
        perm, weight = oracle.hungarian(w, allowed)
        assert weight == best
        assert tuple(perm) in winners


def test_hungarian_vs_scipy():
    from scipy.optimize import linear_sum_assignment
    rng = np.random.default_rng(7)
    for n in (20, 100, 257):
        w = rng.integers(0, 1001, (n, n))
        perm, weight = oracle.hungarian(w)
        r, c = linear_sum_assignment(w, maximize=True)
        assert weight == int(w[r, c].sum())
        assert sorted(perm) == list(range(n))


def test_planted_closed_form_optimum():
    """w_i sigma(i) := hi + bonus makes sigma the unique optimum with weight n (hi + bonus)."""
    W, sigma = skgen.planted(300, seed=4)
    perm, weight = oracle.optimum_int(W)
    assert weight == 300 * 1050
    assert np.array_equal(perm, sigma)


def test_dominant_closed_form_optimum():
    """Diagonal weights >= 800 > 600 >= off-diagonal ones: the identity is optimal."""
    W = skgen.dominant(200, seed=3)
    perm, weight = oracle.optimum_int(W)
    assert np.array_equal(perm, np.arange(200))
    assert weight == int(np.diag(W).astype(np.int64).sum())


# ---------------------------------------------------------------- certificate

def test_certificate_is_an_upper_bound_at_any_iterate():
    """Proposition prop:aoc holds for any positive scalings: check against brute
    force after 0..6 iterations and for random scalings, with ties and zeros."""
    rng = np.random.default_rng(21)
    for trial in range(30):
        n = int(rng.integers(2, 8))
        w = rng.integers(0, 6, (n, n)).astype(float)
        w[rng.random((n, n)) < 0.2] = -np.inf
        best, winners = brute.all_optima(w)
        if best == -math.inf:
            continue
        p = float(rng.choice([0.5, 1.0, 3.0, 8.0]))
        ub_rand = oracle.certificate(w, p, rng.normal(size=n) * 3, rng.normal(size=n) * 3)
        assert ub_rand >= best - 1e-9
        for iters in range(0, 7):
            try:
                u, v, m, res = oracle.sinkhorn(w, p, 0.0, iters)
            except oracle.NoSupport:
                break
            assert oracle.certificate(w, p, u, v) >= best - 1e-9


def test_certificate_tight_at_convergence():
    """With a unique optimum and large p, UB tends to log omega_opt (gamma -> 1)."""
    W, sigma = skgen.planted(40, seed=8, lo=0, hi=20, bonus=1)
    B = oracle.log_weights(W)
    opt = float(W[np.arange(40), sigma].astype(np.int64).sum())
    gaps = []
    ubar = vbar = None
    for p in (0.25, 0.5, 1):
        ubar, vbar, m, res = oracle.sinkhorn(B, p, 1e-12, 10**6, ubar, vbar)
        gaps.append(oracle.certificate(B, p, ubar, vbar) - opt)
    assert all(g >= -1e-9 for g in gaps)
    assert gaps[-1] < 1e-3 and gaps[-1] < gaps[0]


# ---------------------------------------------------------------- prescaling

def test_prescale_range_and_power_invariance():
    """Section 4.1.1: after prescaling, nonzero entries lie in [1, e]; when
    max/min > e the result does not depend on an entrywise power A^(q); the
    step is idempotent (the result has max/min = e, so the branch is not taken)."""
    rng = np.random.default_rng(2)
    A = rng.uniform(0.01, 5.0, (6, 6))
    A[0, 3] = 0.0
    S = oracle.prescale(A)
    nz = S[A > 0]
    assert nz.min() == pytest.approx(1.0, abs=1e-14) and nz.max() == pytest.approx(math.e, abs=1e-13)
    assert S[0, 3] == 0.0
    for q in (2.0, 3.5):
        assert np.allclose(oracle.prescale(A ** q), S, atol=1e-13)
    assert np.allclose(oracle.prescale(S), S, atol=1e-13)
    C = rng.uniform(1.0, 2.0, (4, 4))
    assert np.allclose(oracle.prescale(C), C / C.min())


# ---------------------------------------------------------------- the whole path

def test_solve_config1_shape_recovers_optimum():
    """n = 64, w uniform on 0..100, ladder 1..64: the reduced instance at
    t = 1e-4 keeps a few percent of the entries and still contains an optimal
    permutation (its weight equals the dense optimum); the integer certificate
    UB - W_B < 1 proves optimality."""
    W = skgen.uniform_weights(64, 0, 100, seed=0)
    sol = oracle.solve(W, [1, 2, 4, 8, 16, 32, 64], 1e-9, 20000, 1e-4)
    perm_full, w_full = oracle.optimum_int(W)
    assert sol.weight == w_full
    assert sol.nnz < 0.1 * 64 * 64
    assert sol.ub >= w_full - 1e-9
    assert sol.log_gamma < 1.0


def test_solve_planted_and_dominant():
    W, sigma = skgen.planted(128, seed=3)
    sol = oracle.solve(W, [1, 2, 4, 8, 16, 32], 1e-5, 5000, 1e-4)
    assert sol.weight == 128 * 1050
    assert np.array_equal(sol.perm, sigma)
    assert sol.keep[np.arange(128), sigma].all()
    Wd = skgen.dominant(128, seed=1)
    sol = oracle.solve(Wd, [1, 2, 4, 8, 16, 32], 1e-5, 5000, 1e-4)
    assert np.array_equal(sol.perm, np.arange(128))
    assert sol.nnz == 128   # only the permutation survives


# ---------------------------------------------------------------- Algorithm alg:alg1

def test_adaptive_planted_closed_form():
    """Planted optimum (weight 1050 n, permutation sigma) at whatever p the
    loop returns; gamma >= 1 always (ub >= w_opt(A) >= w_opt(B))."""
    n = 24
    W, sigma = skgen.planted(n, 5)
    for ratio in (0.0, 1.5, 1e300):
        s, status = oracle.adaptive(W, [1, 2, 4, 8, 16], 1e-9, 5000, 1e-4, ratio)
        assert status == "ok"
        assert s.weight == 1050 * n and (s.perm == sigma).all()
        assert s.log_gamma >= -1e-9


def test_adaptive_certified_weight_is_brute_force_optimum():
    """Whenever log gamma < 1 the returned weight is the optimum of A over all
    n! permutations (integer weights), checked by enumeration."""
    for seed in range(6):
        W = skgen.uniform_weights(6, 0, 12, seed=seed)
        s, status = oracle.adaptive(W, [1, 2, 4, 8, 16, 32], 1e-10, 20000, 1e-4, math.e)
        assert status in ("ok", "ratio")
        best = max(int(W[np.arange(6), list(q)].astype(np.int64).sum())
                   for q in itertools.permutations(range(6)))
        assert s.log_gamma >= -1e-9 and s.ub >= best - 1e-9
        if s.log_gamma < 1.0:
            assert s.weight == best


def test_adaptive_stopping_rule():
    """A huge ratio stops at the first stage with a perfect matching; a ratio
    below 1 evaluates the last stage only; a ratio never reached returns the
    stage with the smallest gamma."""
    W = skgen.uniform_weights(64, 0, 100, seed=1)
    lad = [1, 2, 4, 8]
    s, status = oracle.adaptive(W, lad, 1e-6, 3000, 1e-4, 1e300)
    assert status == "ok" and s.p == 1.0 and s.extra["evaluated"] == 1
    s, status = oracle.adaptive(W, lad, 1e-6, 3000, 1e-4, 0.0)
    assert status == "ok" and s.p == 8.0 and s.extra["evaluated"] == 1
    s, status = oracle.adaptive(W, lad, 1e-6, 3000, 1e-4, 1.0 + 1e-12)
    assert status == "ratio" and s.extra["evaluated"] == 4
    gammas = [oracle.adaptive(W, lad[: k + 1], 1e-6, 3000, 1e-4, 0.0)[0].log_gamma
              for k in range(4)]
    assert s.log_gamma == min(gammas)


def test_adaptive_lowers_threshold_at_last_stage():
    """t = 0.99 leaves no perfect matching at p = 1; the loop lowers t tenfold
    until the reduced matrix has one, and the weight is then the optimum."""
    W = skgen.uniform_weights(64, 0, 100, seed=4)
    s, status = oracle.adaptive(W, [1], 1e-9, 5000, 0.99, 0.0)
    assert status == "ok" and s.extra["t"] < 0.99
    assert s.extra["t"] == pytest.approx(0.99 * 10.0 ** round(math.log10(s.extra["t"] / 0.99)))
    assert s.weight == oracle.optimum_int(W)[1]


# ---------------------------------------------------------------- deformed iteration

def test_deformed_constant_p_reproduces_worked_example():
    """With p_m held at 10 the deformed iteration is Sinkhorn iteration on
    A^(10): it stops at the same iteration (106) with the matrix printed in
    Section 2.3, to within half a unit of its 7th decimal."""
    fx = fixtures.load("example_3x3.txt")
    B = oracle.log_of(fx["A"])
    lu, lv, m, p, res = oracle.deformed(B, 1.0, 10, 10, 1e-4, 10**6)
    X = np.exp(p * B + lu[:, None] + lv[None, :])
    assert (m, p) == (106, 10) and res < 1e-4
    assert np.abs(X - fx["X"]).max() <= 5e-8


def _deformed_state(B, a, pmin, pmax, m, integer_p):
    lu, lv, m2, p, _ = oracle.deformed(B, a, pmin, pmax, 0.0, m, integer_p)
    assert m2 == m and p == oracle.deformed_p(a, pmin, pmax, m, integer_p)
    return lu, lv


def test_deformed_schedule():
    """p_m = a log(m + 1) kept in [p_min, p_max] (Theorem
    logconvergencepositive), unrounded; rounded half to even with integer_p."""
    assert oracle.deformed_p(3.0, 1, 16, 1) == pytest.approx(3.0 * math.log(2.0), abs=0.0)
    assert oracle.deformed_p(0.1, 1, 16, 1) == 1
    assert oracle.deformed_p(3.0, 1, 16, 10**6) == 16
    assert oracle.deformed_p(3.0, 1, 16, 1, integer_p=True) == 2  # round(2.079)
    assert oracle.deformed_p(2.0 / math.log(2.0), 1, 16, 1, integer_p=True) == 2


@pytest.mark.parametrize("integer_p", [False, True])
def test_deformed_hadamard_identity(integer_p):
    """Section 3.2, proposition on the iterates: with W_m = diag(u_m) A^(p_m)
    diag(v_m) and Z_m = diag(u_{m+1}) A^(p_{m+1}) diag(v_m),
    Z_m = ROWS(W_m o A^(p_{m+1} - p_m)), checked across steps where p changes."""
    rng = np.random.default_rng(3)
    A = rng.uniform(0.05, 1.0, size=(5, 5))
    B = oracle.log_of(A)
    a, pmin, pmax = 2.0, 1, 9
    changed = 0
    for m in range(1, 14):
        pm, pm1 = (oracle.deformed_p(a, pmin, pmax, k, integer_p) for k in (m, m + 1))
        changed += pm1 != pm
        lu_m, lv_m = _deformed_state(B, a, pmin, pmax, m, integer_p)
        lu_n, _ = _deformed_state(B, a, pmin, pmax, m + 1, integer_p)
        Wm = np.exp(pm * B + lu_m[:, None] + lv_m[None, :])
        Zm = np.exp(pm1 * B + lu_n[:, None] + lv_m[None, :])
        H = Wm * A ** (pm1 - pm)
        assert np.abs(Zm - H / H.sum(axis=1, keepdims=True)).max() < 1e-12
        assert np.abs(Zm.sum(axis=1) - 1).max() < 1e-12  # Z_m is row-stochastic
    assert changed >= 3


@pytest.mark.parametrize("integer_p", [False, True])
def test_deformed_permutation_ratio(integer_p):
    """Section 3.2: for permutations sigma, pi of A,
    w_sigma(Z_m) / w_pi(Z_m) = (w_sigma(A) / w_pi(A))^(p_{m+1}), by enumeration
    of all permutations of a 4 x 4 matrix."""
    rng = np.random.default_rng(5)
    A = rng.uniform(0.1, 1.0, size=(4, 4))
    B = oracle.log_of(A)
    a, pmin, pmax = 3.0, 1, 12
    perms = list(itertools.permutations(range(4)))
    for m in (1, 4, 9):
        pm1 = oracle.deformed_p(a, pmin, pmax, m + 1, integer_p)
        _, lv_m = _deformed_state(B, a, pmin, pmax, m, integer_p)
        lu_n, _ = _deformed_state(B, a, pmin, pmax, m + 1, integer_p)
        logZ = pm1 * B + lu_n[:, None] + lv_m[None, :]
        s0 = perms[0]
        for q in perms[1:]:
            lhs = sum(logZ[i, q[i]] - logZ[i, s0[i]] for i in range(4))
            rhs = pm1 * sum(B[i, q[i]] - B[i, s0[i]] for i in range(4))
            assert abs(lhs - rhs) < 1e-10


@pytest.mark.parametrize("integer_p", [False, True])
def test_deformed_planted_converges_to_permutation(integer_p):
    """Theorem optimalassign: the limit's support is the optimal permutation
    (planted, unique); its weight is the closed form 1050 n."""
    n = 32
    W, sigma = skgen.planted(n, 3)
    B = oracle.log_weights(W)
    lu, lv, m, p, res = oracle.deformed(B, 3.0, 1, 16, 1e-9, 5000, integer_p)
    X = np.exp(p * B + lu[:, None] + lv[None, :])
    assert p == 16 and res < 1e-9
    assert np.abs(X[np.arange(n), sigma] - 1.0).max() < 1e-6
    perm, weight = oracle.optimum_int(W, X >= 1e-4)
    assert weight == 1050 * n and (perm == sigma).all()


# ---------------------------------------------------------------- Newton scaling

def test_newton_2x2_closed_form():
    """X(p) of a positive 2 x 2 matrix is [[t, 1 - t], [1 - t, t]] with
    t / (1 - t) = (a d / (b c))^(p/2); the Newton iteration reaches it."""
    A = np.array([[3.0, 1.0], [0.5, 2.0]])
    B = oracle.log_of(A)
    for p in (1.0, 3.0):
        ub, vb, outer, prods, res = oracle.newton(B, p, 1e-13, 1000)
        X = oracle.scaled_matrix(B, p, ub, vb)
        t = 1.0 / (1.0 + (A[0, 1] * A[1, 0] / (A[0, 0] * A[1, 1])) ** (p / 2))
        assert np.abs(X - np.array([[t, 1 - t], [1 - t, t]])).max() < 1e-12
        assert res < 1e-12


def test_newton_worked_example():
    """Section 2.3's 3 x 3 matrix at p = 10: the Newton limit is the printed
    1e-4-bistochastic iterate to within 1e-4, and a bistochastic matrix to
    1e-12."""
    fx = fixtures.load("example_3x3.txt")
    B = oracle.log_of(fx["A"])
    ub, vb, outer, prods, res = oracle.newton(B, fx["p"], 1e-13, 5000)
    X = oracle.scaled_matrix(B, fx["p"], ub, vb)
    assert res < 1e-12
    assert np.abs(X - fx["X"]).max() < 1e-4


@pytest.mark.parametrize("norm", ["two", "inf"])
def test_newton_equals_sinkhorn_limit(norm):
    """X(p) is unique (Section 2.1): Newton and a converged Sinkhorn
    iteration give the same matrix; Newton needs far fewer products with A.
    Under either stopping norm (2-norm of the cited method, max-norm)."""
    W = skgen.uniform_weights(64, 0, 100, seed=2)
    B = oracle.log_weights(W)
    ub0 = -B.max(axis=1)
    ub, vb, outer, prods, res = oracle.newton(B, 1.0, 1e-11, 5000, ubar=ub0, norm=norm)
    us, vs, m, r2 = oracle.sinkhorn(B, 1.0, 1e-13, 200000, ub0, None)
    assert res < 1e-10 and r2 < 1e-13
    Xn, Xs = oracle.scaled_matrix(B, 1.0, ub, vb), oracle.scaled_matrix(B, 1.0, us, vs)
    assert np.abs(Xn - Xs).max() < 1e-10
    assert prods < m / 4


def test_newton_stopping_norms():
    """The 2-norm stop is the stricter one (|r|_inf <= |r|_2): at the same
    loose tolerance it takes at least as many products and ends with
    |1 - x o (S x)|_2 <= tol, while the max-norm stop ends with
    max |row or column sum - 1| <= tol."""
    W = skgen.uniform_weights(256, 0, 100, seed=4)
    B = oracle.log_weights(W)
    ub0 = -B.max(axis=1)
    tol = 1e-4
    u2, v2, _, prods2, _ = oracle.newton(B, 1.0, tol, 5000, ubar=ub0, norm="two")
    ui, vi, _, prodsi, resi = oracle.newton(B, 1.0, tol, 5000, ubar=ub0, norm="inf")
    assert prods2 >= prodsi and resi <= tol
    rs, cs = oracle.sums(B, 1.0, u2, v2)
    assert math.sqrt(float(((rs - 1) ** 2).sum() + ((cs - 1) ** 2).sum())) <= tol


# ---------------------------------------------------------------- real log-weights

@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_hungarian_real_vs_brute_force(n):
    rng = np.random.default_rng(100 + n)
    for trial in range(6):
        w = rng.standard_normal((n, n)) * 3.0
        allowed = rng.random((n, n)) < (0.5 if trial % 2 else 1.0)
        b = np.where(allowed, w, -np.inf)
        best, winners = brute.all_optima(b)
        if best == -math.inf:
            with pytest.raises(oracle.Infeasible):
                oracle.hungarian_real(b)
            continue
        perm, weight = oracle.hungarian_real(b)
        assert weight == pytest.approx(best, abs=1e-12)
        assert tuple(perm) in winners


def test_hungarian_real_vs_scipy_and_integer_solver():
    from scipy.optimize import linear_sum_assignment
    rng = np.random.default_rng(8)
    for n in (30, 120, 301):
        w = -rng.uniform(0.0, 1.7, (n, n))
        perm, weight = oracle.hungarian_real(w)
        r, c = linear_sum_assignment(w, maximize=True)
        assert weight == pytest.approx(w[r, c].sum(), abs=1e-9)
        assert sorted(perm) == list(range(n))
        wi = rng.integers(0, 1001, (n, n))
        assert oracle.hungarian_real(wi.astype(float))[1] == oracle.hungarian(wi)[1]


def test_prescale_log_matches_linear_prescale():
    """Section 4.1.1 on log-weights equals the linear prescaling (pinned
    above) entry by entry, maps the finite entries onto [0, 1] when
    max/min > e, and is invariant under entrywise powers A^(q)."""
    rng = np.random.default_rng(3)
    A = rng.uniform(0.01, 5.0, (7, 7))
    A[2, 4] = 0.0
    B = oracle.log_of(A)
    Bp, scale = oracle.prescale_log(B)
    assert scale == pytest.approx(1.0 / (np.log(A[A > 0].max()) - np.log(A[A > 0].min())))
    assert np.allclose(np.exp(Bp), oracle.prescale(A), atol=1e-13)
    fin = Bp[np.isfinite(Bp)]
    assert fin.min() == 0.0 and fin.max() == pytest.approx(1.0, abs=1e-15)
    for q in (2.0, 7.5):
        assert np.allclose(oracle.prescale_log(q * B)[0], Bp, atol=1e-13)
    C = rng.uniform(1.0, 2.0, (4, 4))
    Cp, s2 = oracle.prescale_log(np.log(C))
    assert s2 == 1.0 and np.allclose(np.exp(Cp), C / C.min())


def test_adaptive_real_equals_integer_loop_without_prescaling():
    """On integer weights with prescaling off, the real-weight loop takes the
    same decisions as the integer one (same p, t, weight and log gamma)."""
    W = skgen.uniform_weights(48, 0, 100, seed=2)
    lad = [1, 2, 4, 8]
    for ratio in (0.0, math.e, 1.0 + 1e-12):
        a, sa = oracle.adaptive(W, lad, 1e-7, 5000, 1e-4, ratio if ratio >= 1 else 1e300)
        b, sb = oracle.adaptive_real(oracle.log_weights(W), lad, 1e-7, 5000, 1e-4,
                                     ratio if ratio >= 1 else 1e300, prescale=False)
        assert sa == sb and a.p == b.p and a.extra["t"] == b.extra["t"]
        assert a.weight == b.weight and a.log_gamma == pytest.approx(b.log_gamma, abs=1e-9)
        assert np.array_equal(a.perm, b.perm)


def test_adaptive_real_paper_defaults_power_invariance_and_optimum():
    """Algorithm alg:alg1 with the paper's defaults (p0 = 100, p += 50 on the
    prescaled matrix, eps = t = 1/n, required ratio 2) on a Euclidean random
    assignment instance (real log-weights -d): the result does not change
    when A is replaced by an entrywise power A^(q) (the prescaled matrix is
    the same, Section 4.1.1); gamma >= 1; and when gamma is within the ratio
    the reduced matrix's optimum is within log gamma of the optimum of the
    whole matrix, in the prescaled units."""
    n = 40
    x, y = skgen.euclidean_points(n, 3)
    B = -np.sqrt(((x[:, None, :] - y[None, :, :]) ** 2).sum(axis=2))
    lad = [100 + 50 * k for k in range(8)]
    s, st = oracle.adaptive_real(B, lad, 1.0 / n, 20000, 1.0 / n, 2.0)
    s3, st3 = oracle.adaptive_real(3.0 * B, lad, 1.0 / n, 20000, 1.0 / n, 2.0)
    assert st == st3 and s.p == s3.p and np.array_equal(s.perm, s3.perm)
    assert s.log_gamma == pytest.approx(s3.log_gamma, abs=1e-9)
    assert s.log_gamma >= -1e-9
    Bp, scale = oracle.prescale_log(B)
    _, w_all = oracle.hungarian_real(Bp)
    assert s.weight <= w_all + 1e-12
    assert w_all - s.weight <= s.log_gamma + 1e-9
    assert s.extra["weight_orig"] == pytest.approx(B[np.arange(n), s.perm].sum())
