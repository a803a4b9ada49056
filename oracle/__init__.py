"""Oracle for the Sinkhorn-based preprocessing of the optimal assignment problem.

TEST INFRASTRUCTURE ONLY: a plain FP64 CPU statement of what the GPU library
computes, written from the paper (Sharify, Gaubert, Grigori, arXiv:1104.3830).
Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
it. It shares no code with the HIP library and never imports it.

Notation: b_ij = log a_ij (-inf where a_ij = 0); the scalings are held as
ubar = p^-1 log u, vbar = p^-1 log v (Section 4.1.2), so the scaled matrix is
x_ij(p) = exp(p (b_ij + ubar_i + vbar_j)).

Every function cites the passage it follows; parity status of each part:
  row/column step, Sinkhorn, ladder ... pinned (worked examples of Section 2.3
      and Section 4.2, 2x2 closed form, permutation-ratio invariance,
      brute-force limits)
  prune ............................... pinned (support of the 5x5 example)
  certificate ......................... pinned (upper bound vs brute force,
      tight at convergence)
  hungarian ........................... pinned (brute force n <= 8, scipy)
  hungarian_real ...................... pinned (brute force n <= 7, scipy, equality
      with hungarian on integer weights)
  prescale_log ........................ pinned (equal to the linear prescale; range
      [0, 1]; invariance under entrywise powers)
  adaptive_real ....................... pinned (equal to adaptive on integer weights
      without prescaling; invariance under entrywise powers with prescaling;
      optimum against the Hungarian of the whole matrix)
  prescale ............................ pinned (range [1, e], idempotence,
      invariance under entrywise powers, Section 4.1.1)
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        L.or_row_step.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]
        L.or_row_step.restype = ctypes.c_int
        L.or_col_step.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]
        L.or_col_step.restype = ctypes.c_int
        L.or_sums.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _dp, _dp]
        L.or_sums.restype = None
        L.or_row_residual.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]
        L.or_row_residual.restype = ctypes.c_double
        L.or_sinkhorn.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, ctypes.c_double,
                                  ctypes.c_long, ctypes.POINTER(ctypes.c_long), _dp]
        L.or_sinkhorn.restype = ctypes.c_int
        L.or_scale_ladder.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_long, _dp, _dp, ctypes.POINTER(ctypes.c_long), _dp]
        L.or_scale_ladder.restype = ctypes.c_int
        L.or_prune.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, ctypes.c_double, _u8p]
        L.or_prune.restype = ctypes.c_long
        L.or_certificate.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]
        L.or_certificate.restype = ctypes.c_double
        L.or_prescale.argtypes = [ctypes.c_int, _dp, _dp]
        L.or_prescale.restype = None
        L.or_hungarian.argtypes = [ctypes.c_int, _i64p, _u8p, _i32p, _i64p]
        L.or_hungarian.restype = ctypes.c_int
        L.or_hungarian_real.argtypes = [ctypes.c_int, _dp, _u8p, _i32p, _dp]
        L.or_hungarian_real.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


class NoSupport(RuntimeError):
    """A row or column of A has no positive entry (Section 2.1: A must have support)."""


class Infeasible(RuntimeError):
    """The (reduced) matrix has no perfect matching."""


SENTINEL = -32768


def log_weights(W: np.ndarray) -> np.ndarray:
    """b = log A from int16 log-weights: w as float64, the sentinel as -inf."""
    B = W.astype(np.float64)
    B[W == SENTINEL] = -np.inf
    return np.ascontiguousarray(B)


def log_of(A: np.ndarray) -> np.ndarray:
    """b = log A for a non-negative real matrix (log 0 = -inf)."""
    with np.errstate(divide="ignore"):
        return np.ascontiguousarray(np.log(np.asarray(A, dtype=np.float64)))


def row_step(B, p, vbar):
    """u = I(A^(p) v) in log coordinates (eq. dad2, Section 4.1.2). B may be a
    block of rows (rows x n); returns ubar for those rows."""
    B = np.ascontiguousarray(B, dtype=np.float64)
    rows, cols = B.shape
    vbar = np.ascontiguousarray(vbar, dtype=np.float64)
    ubar = np.empty(rows)
    if lib().or_row_step(rows, cols, float(p), _d(B), _d(vbar), _d(ubar)):
        raise NoSupport("a row has no finite entry")
    return ubar


def col_step(B, p, ubar):
    """v = I(A^(p)T u) in log coordinates (eq. dad3, Section 4.1.2). B may be a
    block of columns (n x cols); returns vbar for those columns."""
    B = np.ascontiguousarray(B, dtype=np.float64)
    rows, cols = B.shape
    ubar = np.ascontiguousarray(ubar, dtype=np.float64)
    vbar = np.empty(cols)
    if lib().or_col_step(rows, cols, float(p), _d(B), _d(ubar), _d(vbar)):
        raise NoSupport("a column has no finite entry")
    return vbar


def sums(B, p, ubar, vbar):
    """Row and column sums of X = diag(u) A^(p) diag(v)."""
    n = B.shape[0]
    r, c = np.empty(n), np.empty(n)
    lib().or_sums(n, float(p), _d(B), _d(np.ascontiguousarray(ubar, dtype=np.float64)),
                  _d(np.ascontiguousarray(vbar, dtype=np.float64)), _d(r), _d(c))
    return r, c


def row_residual(B, p, ubar, vbar):
    """max_i |r_i - 1| (Section 4.2, epsilon-bistochastic distance)."""
    n = B.shape[0]
    return lib().or_row_residual(n, float(p), _d(B),
                                 _d(np.ascontiguousarray(ubar, dtype=np.float64)),
                                 _d(np.ascontiguousarray(vbar, dtype=np.float64)))


def scaled_matrix(B, p, ubar, vbar):
    """X = diag(u) A^(p) diag(v), x_ij = exp(p (b_ij + ubar_i + vbar_j))."""
    with np.errstate(invalid="ignore", over="ignore"):
        X = np.exp(p * (B + ubar[:, None] + vbar[None, :]))
    X[np.isneginf(B)] = 0.0
    return X


def sinkhorn(B, p, eps, max_iters, ubar=None, vbar=None):
    """Sinkhorn iteration on A^(p) (Section 3.1, eqs. dad1-dad3, log form of
    Section 4.1.2). Rows first; stop when the column-stochastic iterate W_m
    has max_i |r_i - 1| < eps, or after max_iters iterations.
    Returns (ubar, vbar, iterations, residual)."""
    n = B.shape[0]
    ubar = np.zeros(n) if ubar is None else np.array(ubar, dtype=np.float64)
    vbar = np.zeros(n) if vbar is None else np.array(vbar, dtype=np.float64)
    it = ctypes.c_long(0)
    res = ctypes.c_double(0.0)
    bad = lib().or_sinkhorn(n, float(p), _d(B), _d(ubar), _d(vbar), float(eps), int(max_iters),
                            ctypes.byref(it), ctypes.byref(res))
    if bad:
        raise NoSupport("a row or column has no finite entry")
    return ubar, vbar, it.value, res.value


def scale_ladder(B, ladder, eps, max_iters, vbar=None):
    """Continuation in p over the ladder with (ubar, vbar) carried across
    stages. Returns (ubar, vbar, iterations per stage, residual per stage)."""
    n = B.shape[0]
    lad = np.ascontiguousarray(ladder, dtype=np.float64)
    ubar = np.zeros(n)
    vbar = np.zeros(n) if vbar is None else np.array(vbar, dtype=np.float64)
    iters = (ctypes.c_long * len(lad))()
    res = np.empty(len(lad))
    if lib().or_scale_ladder(n, _d(B), _d(lad), len(lad), float(eps), int(max_iters),
                             _d(ubar), _d(vbar), iters, _d(res)):
        raise NoSupport("a row or column has no finite entry")
    return ubar, vbar, list(iters), list(res)


def prune(B, p, ubar, vbar, t):
    """Support of the reduced matrix (eq. matrixred): keep (i, j) iff x_ij(p) >= t."""
    n = B.shape[0]
    keep = np.empty((n, n), dtype=np.uint8)
    lib().or_prune(n, float(p), _d(B), _d(np.ascontiguousarray(ubar, dtype=np.float64)),
                   _d(np.ascontiguousarray(vbar, dtype=np.float64)), float(t),
                   keep.ctypes.data_as(_u8p))
    return keep.astype(bool)


def certificate(B, p, ubar, vbar):
    """Upper bound on log omega_opt(A) (Proposition prop:aoc)."""
    n = B.shape[0]
    return lib().or_certificate(n, float(p), _d(B),
                                _d(np.ascontiguousarray(ubar, dtype=np.float64)),
                                _d(np.ascontiguousarray(vbar, dtype=np.float64)))


def prescale(A):
    """Prescaling into [1, e] (Section 4.1.1)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    out = np.empty_like(A)
    lib().or_prescale(A.shape[0], _d(A), _d(out))
    return out


def hungarian(w, allowed=None):
    """Exact maximum-weight perfect matching, dense O(n^3) (Section 1's
    Kuhn/Edmonds class). w: int64 n x n; allowed: bool mask (default: all).
    Returns (perm, weight) with perm[i] the column of row i."""
    w = np.ascontiguousarray(w, dtype=np.int64)
    n = w.shape[0]
    if allowed is None:
        allowed = np.ones((n, n), dtype=np.uint8)
    allowed = np.ascontiguousarray(allowed, dtype=np.uint8)
    perm = np.empty(n, dtype=np.int32)
    weight = ctypes.c_int64(0)
    if n == 0:
        return perm, 0
    st = lib().or_hungarian(n, w.ctypes.data_as(_i64p), allowed.ctypes.data_as(_u8p),
                            perm.ctypes.data_as(_i32p), ctypes.byref(weight))
    if st:
        raise Infeasible("no perfect matching on the allowed entries")
    return perm, weight.value


def hungarian_real(w, allowed=None):
    """Exact maximum-weight perfect matching for real weights, dense O(n^3)
    (the Hungarian method of Section 1's solver class) in FP64. w: n x n
    float64; allowed: bool mask (default: the finite entries). Returns
    (perm, weight)."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    n = w.shape[0]
    if allowed is None:
        allowed = np.isfinite(w)
    allowed = np.ascontiguousarray(allowed & np.isfinite(w), dtype=np.uint8)
    wz = np.where(allowed.astype(bool), w, 0.0)
    perm = np.empty(n, dtype=np.int32)
    weight = ctypes.c_double(0.0)
    if n == 0:
        return perm, 0.0
    st = lib().or_hungarian_real(n, _d(np.ascontiguousarray(wz)), allowed.ctypes.data_as(_u8p),
                                 perm.ctypes.data_as(_i32p), ctypes.byref(weight))
    if st:
        raise Infeasible("no perfect matching on the allowed entries")
    return perm, weight.value


def prescale_log(B):
    """The prescaling of Section 4.1.1 written on b = log a: with lo, hi the
    smallest and largest finite b, b' = (b - lo) / (hi - lo) when
    max(A)/min(A) > e (hi - lo > 1: A^(m)/c with m = 1/log(max/min)),
    otherwise b' = b - lo (A / min(A)). Returns (b', the factor applied to p:
    p on A' equals p / (hi - lo), resp. p, on A)."""
    B = np.asarray(B, dtype=np.float64)
    fin = B[np.isfinite(B)]
    lo, hi = float(fin.min()), float(fin.max())
    scale = 1.0 / (hi - lo) if hi - lo > 1.0 else 1.0
    with np.errstate(invalid="ignore"):
        out = (B - lo) * scale
    out[np.isneginf(B)] = -np.inf
    return np.ascontiguousarray(out), scale


def optimum_int(W, allowed=None):
    """Optimal assignment of int16 log-weights W (sentinel entries excluded)."""
    mask = W != SENTINEL
    if allowed is not None:
        mask = mask & allowed
    return hungarian(W.astype(np.int64), mask)


@dataclass
class Solution:
    """Result of the preprocessing pipeline for one instance."""
    p: float
    ubar: np.ndarray
    vbar: np.ndarray
    iters: list
    residuals: list
    keep: np.ndarray
    nnz: int
    ub: float
    perm: np.ndarray | None
    weight: int | None
    log_gamma: float | None
    extra: dict = field(default_factory=dict)


def solve(W, ladder, eps, max_iters, t):
    """The path for one int16 instance, step by step:
    continuation over the p ladder (Section 3.1 + 4.1.2), reduced matrix
    (eq. matrixred), exact solve of the reduced instance, certificate
    (Proposition prop:aoc) and log gamma (eq. optratio)."""
    B = log_weights(W)
    ubar, vbar, iters, res = scale_ladder(B, ladder, eps, max_iters)
    p = float(ladder[-1])
    keep = prune(B, p, ubar, vbar, t)
    ub = certificate(B, p, ubar, vbar)
    try:
        perm, weight = optimum_int(W, keep)
        log_gamma = ub - weight
    except Infeasible:
        perm, weight, log_gamma = None, None, None
    return Solution(p, ubar, vbar, iters, res, keep, int(keep.sum()), ub, perm, weight, log_gamma)


def adaptive(W, ladder, eps, max_iters, t, opt_ratio):
    """Algorithm alg:alg1 (Section 4.2) over a given ladder of p.

    Per p, in order: Sinkhorn scaling of A^(p) carried over from the previous
    p in the coordinates p^-1 log u, p^-1 log v (Section 4.1.2), the
    certificate (Proposition prop:aoc), the reduced matrix (eq. matrixred),
    an optimal assignment of it and log gamma = ub - w(B) (eq. optratio).
    The loop is read as "raise p while gamma exceeds opt_ratio": it stops at
    the first p with gamma <= opt_ratio; with opt_ratio < 1 only the last p is
    evaluated. gamma is undefined when the reduced matrix has no perfect
    matching; at the last p the threshold is then lowered tenfold, at most
    three times. Returns (Solution of the returned p, status) with status
    "ok", "ratio" (ladder ended first: the p with the smallest gamma is
    returned) or "infeasible"; Solution.extra holds t and the number of
    evaluated p."""
    Bw = log_weights(W)
    n = W.shape[0]
    ubar, vbar = np.zeros(n), np.zeros(n)
    evaluate_all = opt_ratio >= 1.0
    best, evaluated, iters_all, res_all = None, 0, [], []
    for k, p in enumerate(ladder):
        ubar, vbar, it, res = sinkhorn(Bw, p, eps, max_iters, ubar, vbar)
        iters_all.append(it)
        res_all.append(res)
        last = k + 1 == len(ladder)
        if not (evaluate_all or last):
            continue
        ub = certificate(Bw, p, ubar, vbar)
        tt = t
        for tries in range(4):
            keep = prune(Bw, p, ubar, vbar, tt)
            try:
                perm, weight = optimum_int(W, keep)
                break
            except Infeasible:
                perm, weight = None, None
                if not last or tries == 3:
                    break
                tt /= 10.0
        evaluated += 1
        if weight is not None:
            lg = ub - weight
            if best is None or lg < best.log_gamma:
                best = Solution(float(p), ubar.copy(), vbar.copy(), list(iters_all), list(res_all),
                                keep, int(keep.sum()), ub, perm, weight, lg, {"t": tt})
            if not evaluate_all or best.log_gamma <= np.log(opt_ratio):
                best.extra["evaluated"] = evaluated
                return best, "ok"
    if best is None:
        return None, "infeasible"
    best.extra["evaluated"] = evaluated
    return best, "ratio"


def adaptive_real(B, ladder, eps, max_iters, t, opt_ratio, prescale=True):
    """Algorithm alg:alg1 (Section 4.2) on real log-weights b = log a (-inf
    for a zero): with prescale, A is first replaced by its prescaled matrix
    (Section 4.1.1, prescale_log) and every quantity below refers to it, as
    in the algorithm; then, for each p of the ladder in order, Sinkhorn
    scaling of A^(p) to eps (carried from the previous p in the coordinates
    p^-1 log u, p^-1 log v), the certificate (Proposition prop:aoc), the
    reduced matrix at t (eq. matrixred), an optimal assignment of it and
    log gamma = ub - w(B) (eq. optratio). It stops at the first p with
    gamma <= opt_ratio (the loop condition read as "raise p while gamma
    exceeds the ratio"); when B has no perfect matching at the last p, t is
    lowered tenfold, at most three times. Returns (Solution, status) as
    adaptive(); Solution.weight is w(B) in the prescaled units and
    Solution.extra holds t, the number of evaluated p, the p factor of the
    prescaling, the weight in the original units and (p, log gamma) of every
    evaluated p."""
    B = np.asarray(B, dtype=np.float64)
    n = B.shape[0]
    Bp, scale = prescale_log(B) if prescale else (np.ascontiguousarray(B), 1.0)
    ubar, vbar = np.zeros(n), np.zeros(n)
    best, evaluated, iters_all, res_all, gammas = None, 0, [], [], []
    for k, p in enumerate(ladder):
        ubar, vbar, it, res = sinkhorn(Bp, p, eps, max_iters, ubar, vbar)
        iters_all.append(it)
        res_all.append(res)
        last = k + 1 == len(ladder)
        ub = certificate(Bp, p, ubar, vbar)
        tt = t
        for tries in range(4):
            keep = prune(Bp, p, ubar, vbar, tt)
            try:
                perm, weight = hungarian_real(Bp, keep)
                break
            except Infeasible:
                perm, weight = None, None
                if not last or tries == 3:
                    break
                tt /= 10.0
        evaluated += 1
        gammas.append((float(p), ub - weight if weight is not None else math.inf))
        if weight is not None:
            lg = ub - weight
            if best is None or lg < best.log_gamma:
                w_orig = float(B[np.arange(n), perm].sum())
                best = Solution(float(p), ubar.copy(), vbar.copy(), list(iters_all), list(res_all),
                                keep, int(keep.sum()), ub, perm, weight, lg,
                                {"t": tt, "p_scale": scale, "weight_orig": w_orig})
            if best.log_gamma <= np.log(opt_ratio):
                best.extra["evaluated"] = evaluated
                best.extra["gammas"] = gammas
                return best, "ok"
    if best is None:
        return None, "infeasible"
    best.extra["evaluated"] = evaluated
    best.extra["gammas"] = gammas
    return best, "ratio"


def deformed_p(a, p_min, p_max, m, integer_p=False):
    """p of iteration m (from 1) of the deformed iteration: the schedule
    p_m = a log(m + 1) of Theorem logconvergencepositive, kept in
    [p_min, p_max]. integer_p: rounded to an integer (half to even) first,
    the reading taken for integer log-weights, whose exact exponents need an
    integer p."""
    v = a * math.log(m + 1)
    if integer_p:
        return int(min(p_max, max(p_min, round(v))))
    return float(min(p_max, max(p_min, v)))


def deformed(B, a, p_min, p_max, eps, max_iters, integer_p=False):
    """Deformed Sinkhorn iteration (Section 3.2): v_0 = 1 and, for m = 1, 2, ...,
    u_m = I(A^(p_m) v_{m-1}), v_m = I(A^(p_m)T u_m) with u and v carried as they
    are from one p to the next (no rescaling), p_m from deformed_p (the
    paper's real schedule, or rounded with integer_p). Stops after iteration
    m when p_m = p_max and the column-stochastic iterate W_m has
    max_i |r_i - 1| < eps at that p, or after max_iters iterations.
    Returns (log u, log v, iterations, p of the last iteration, residual)."""
    n = B.shape[0]
    logu, logv = np.zeros(n), np.zeros(n)
    res = math.inf
    m = 0
    while m < max_iters:
        m += 1
        p = deformed_p(a, p_min, p_max, m, integer_p)
        logu = p * row_step(B, p, logv / p)
        logv = p * col_step(B, p, logu / p)
        if p == p_max:
            res = row_residual(B, p, logu / p, logv / p)
            if res < eps:
                break
    return logu, logv, m, deformed_p(a, p_min, p_max, m, integer_p), res


def newton(B, p, tol, max_products, ubar=None, vbar=None, lo=0.1, hi=3.0, eta_max=0.1,
           g=0.9, norm="two"):
    """Newton iteration for the diagonal scaling of A^(p) (Section 5.2, the
    method of Knight and Ruiz cited there).

    X = diag(u) A^(p) diag(v) for the starting scalings (u = v = 1 unless
    given) and S = [[0, X], [X^T, 0]] (the symmetric embedding of a
    nonsymmetric matrix). Find x > 0 with x o (S x) = 1. A Newton step for
    x o (S x) - 1 = 0, written multiplicatively as x <- x o y, solves
    (D(x) S D(x) + D(v)) y = 1 + v, v = x o (S x), by conjugate gradients
    preconditioned with D(v) and started at y = 1 (residual 1 - v); the matrix
    is symmetric positive semidefinite and the system consistent when A has
    support. A CG step that would take y to or past lo (or hi) is cut at that
    bound and ends the inner solve. The inner solve stops once the
    preconditioned residual falls below max(eta^2 |1 - v|^2, tol^2), with the
    forcing term eta updated after every outer step from the ratio of
    successive residuals (at most eta_max, at least tol / (2 |1 - v|)). The
    outer loop stops when |1 - v| <= tol, in the 2-norm of the cited method
    (norm="two") or the max-norm (norm="inf", the Sinkhorn stopping test's
    norm), or after max_products products with S. Returns (ubar, vbar, outer
    steps, products with S, max |row or column sum - 1| of the result)."""
    if norm not in ("two", "inf"):
        raise ValueError("norm is 'two' or 'inf'")

    def size(r):
        return math.sqrt(float(r @ r)) if norm == "two" else float(np.abs(r).max())
    n = B.shape[0]
    ubar = np.zeros(n) if ubar is None else np.array(ubar, dtype=np.float64)
    vbar = np.zeros(n) if vbar is None else np.array(vbar, dtype=np.float64)
    X = scaled_matrix(B, p, ubar, vbar)

    def Sx(z):
        return np.concatenate([X @ z[n:], X.T @ z[:n]])

    rt = tol * tol
    x = np.ones(2 * n)
    v = x * Sx(x)
    r = 1.0 - v
    rout = float(r @ r)
    rold = rout
    products, outer, eta = 1, 0, eta_max
    while size(r) > tol and products < max_products:
        outer += 1
        y = np.ones(2 * n)
        inner_tol = max(eta * eta * rout, rt)
        rho, rho_prev = rout, 1.0
        d = z = None
        while rho > inner_tol and products < max_products:
            if d is None:
                z = r / v
                rho = float(r @ z)
                d = z.copy()
            else:
                d = z + (rho / rho_prev) * d
            w = x * Sx(x * d) + v * d
            products += 1
            alpha = rho / float(d @ w)
            step = alpha * d
            ynew = y + step
            if ynew.min() <= lo:
                neg = step < 0
                y = y + ((lo - y[neg]) / step[neg]).min() * step
                break
            if ynew.max() >= hi:
                over = ynew > hi
                y = y + ((hi - y[over]) / step[over]).min() * step
                break
            y = ynew
            r = r - alpha * w
            rho_prev = rho
            z = r / v
            rho = float(r @ z)
        x = x * y
        v = x * Sx(x)
        products += 1
        r = 1.0 - v
        rout = float(r @ r)
        # forcing term for the next inner solve
        ratio, rold = rout / rold, rout
        eta_prev = eta
        eta = g * ratio
        if g * eta_prev * eta_prev > 0.1:
            eta = max(eta, g * eta_prev * eta_prev)
        eta = max(min(eta, eta_max), 0.5 * tol / max(math.sqrt(rout), 1e-300))
    rows, cols = x[:n], x[n:]
    ub = ubar + np.log(rows) / p
    vb = vbar + np.log(cols) / p
    rs, cs = sums(B, p, ub, vb)
    return ub, vb, outer, products, max(np.abs(rs - 1).max(), np.abs(cs - 1).max())
