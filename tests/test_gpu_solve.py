"""GPU parity of sk_solve, the path of Algorithm alg:alg1 run natively, against
the oracle's Algorithm alg:alg1 (oracle.adaptive) on the same inputs.

Integer results (optimal weight of the reduced matrix, the returned p, the
permutation where the optimum is unique) must match exactly. The certificate
ub is a sum over n rows of max_j (w_ij + log v_j / p) minus sum_j log v_j / p,
which only depends on the column potentials up to a common shift; with both
sides converged to 1e-6 its difference stays below n * 1e-6 / p per unit of
shift error, so 1e-2 at n <= 256 (the tests' inputs are chosen so that no
stage's log gamma lies within 0.05 of the stopping bound).
"""
import math

import numpy as np
import pytest

import oracle
import paper_1104_3830_amd as sk
import skgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    c = sk.Context(0)
    yield c
    c.close()


def dev(W):
    return torch.from_numpy(np.ascontiguousarray(W)).cuda()


def weight_of(W, perm):
    return int(W[np.arange(W.shape[0]), perm].astype(np.int64).sum())


def stage_gammas(W, ladder, tol, cap, t):
    """log gamma of the oracle at the end of every stage."""
    out = []
    for k in range(len(ladder)):
        s, _ = oracle.adaptive(W, ladder[: k + 1], tol, cap, t, 0.0)
        out.append(s.log_gamma if s is not None else math.inf)
    return out


@pytest.mark.parametrize("n,hi", [(64, 100), (256, 1000)])
def test_adaptive_stops_at_the_oracles_stage(ctx, n, hi):
    W = skgen.uniform_weights(n, 0, hi, seed=1)
    ladder, tol, cap, t, ratio = [1, 2, 4, 8, 16, 32], 1e-6, 3000, 1e-4, math.e
    gam = stage_gammas(W, ladder, tol, cap, t)
    assert all(abs(g - 1.0) > 0.05 for g in gam)  # no borderline decision
    want, status = oracle.adaptive(W, ladder, tol, cap, t, ratio)
    assert status == "ok"
    prm = sk.make_params(ladder, tol=tol, max_iters=cap, threshold=t, opt_ratio=ratio)
    out = ctx.solve(dev(W), prm)
    r = out["report"]
    assert out["status"] == sk.SK_OK
    assert r["p_final"] == want.p
    assert r["stages_evaluated"] == want.extra["evaluated"]
    assert out["weight"] == want.weight == weight_of(W, out["perm"])
    assert sorted(out["perm"].tolist()) == list(range(n))
    assert abs(r["ub"] - want.ub) < 1e-2
    assert abs(out["log_gamma"] - want.log_gamma) < 1e-2
    assert r["optimal_proved"] == 1  # log gamma < 1 with integer weights
    assert out["weight"] == oracle.optimum_int(W)[1]


def test_last_stage_only_matches_oracle(ctx):
    n = 256
    W = skgen.uniform_weights(n, 0, 100, seed=1)
    ladder, tol, cap, t = [1, 2, 4, 8, 16, 32], 1e-6, 3000, 1e-4
    want, status = oracle.adaptive(W, ladder, tol, cap, t, 0.0)
    prm = sk.make_params(ladder, tol=tol, max_iters=cap, threshold=t, opt_ratio=0.0)
    out = ctx.solve(dev(W), prm)
    r = out["report"]
    assert status == "ok" and out["status"] == sk.SK_OK
    assert r["p_final"] == 32 and r["stages_evaluated"] == 1
    assert out["weight"] == want.weight
    assert abs(r["ub"] - want.ub) < 1e-2
    # the potentials returned are those of the last stage
    lu, lv = sk.split_potentials(out["potentials"], n)
    Bw = oracle.log_weights(W)
    assert abs(oracle.certificate(Bw, 32.0, lu / 32.0, lv / 32.0) - r["ub"]) < 1e-6


def test_ratio_not_reached_returns_best_stage(ctx):
    n = 256
    W = skgen.uniform_weights(n, 0, 100, seed=1)
    ladder, tol, cap, t, ratio = [1, 2], 1e-6, 3000, 1e-4, 1.5
    want, status = oracle.adaptive(W, ladder, tol, cap, t, ratio)
    assert status == "ratio"
    prm = sk.make_params(ladder, tol=tol, max_iters=cap, threshold=t, opt_ratio=ratio)
    out = ctx.solve(dev(W), prm)
    assert out["status"] == sk.SK_ENOCONV
    assert out["report"]["p_final"] == want.p == 2
    assert out["weight"] == want.weight
    assert out["report"]["stages_evaluated"] == 2


def test_threshold_lowered_when_reduced_matrix_has_no_matching(ctx):
    n = 64
    W = skgen.uniform_weights(n, 0, 100, seed=4)
    ladder, tol, cap, t = [1], 1e-9, 5000, 0.99
    want, status = oracle.adaptive(W, ladder, tol, cap, t, 0.0)
    assert status == "ok" and want.extra["t"] < t
    prm = sk.make_params(ladder, tol=tol, max_iters=cap, threshold=t)
    out = ctx.solve(dev(W), prm)
    assert out["status"] == sk.SK_OK
    assert out["report"]["threshold_used"] == pytest.approx(want.extra["t"], rel=1e-12)
    assert out["weight"] == want.weight


def test_dominant_instance_proves_optimality(ctx):
    n = 512
    W = skgen.dominant(n, seed=7)
    prm = sk.make_params([1, 2, 4, 8, 16, 32], tol=1e-5, max_iters=2000, opt_ratio=math.e)
    out = ctx.solve(dev(W), prm)
    assert out["status"] == sk.SK_OK
    assert out["weight"] == int(np.diag(W).astype(np.int64).sum())  # closed form
    assert (out["perm"] == np.arange(n)).all()
    assert out["report"]["optimal_proved"] == 1


def test_dominant_full_size_recovers_identity(ctx):
    """The diagonally dominant 5% pattern at n = 16384 (sentinel-heavy, the
    largest size): the unique optimum is the identity (every diagonal weight
    exceeds every off-diagonal one), with the closed-form weight; the reduced
    matrix keeps the diagonal only and the certificate proves optimality."""
    n = 16384
    W = skgen.dominant(n, seed=5)
    diag = int(np.diag(W).astype(np.int64).sum())
    Wd = dev(W)
    del W
    prm = sk.make_params([1, 2, 4, 8, 16, 32], tol=1e-5, max_iters=60, check_every=32,
                         threshold=1e-4)
    out = ctx.solve(Wd, prm)
    assert out["status"] in (sk.SK_OK, sk.SK_ENOCONV)
    assert out["weight"] == diag
    assert (out["perm"] == np.arange(n)).all()
    assert out["nnz"] == n
    assert out["report"]["optimal_proved"] == 1


def test_planted_4096_full_path(ctx):
    n = 4096
    W, sigma = skgen.planted(n, seed=2)
    prm = sk.make_params([1, 2, 4, 8, 16, 32], tol=1e-5, max_iters=2000, threshold=1e-4)
    out = ctx.solve(dev(W), prm)
    assert out["status"] == sk.SK_OK
    assert out["weight"] == 1050 * n  # closed form of the planted optimum
    assert (out["perm"] == sigma).all()
    assert out["report"]["optimal_proved"] == 1


def test_euclidean_workload(ctx):
    """Euclidean random assignment (2n points in the unit cube, a_ij =
    exp(-d(x_i, y_j))) with distances quantised at 1/1000: same optimal
    weight and proof as the oracle; the permutation's real total distance is
    within n / 1000 of the real-valued optimum (each quantised weight is off
    by at most 1/2000)."""
    from scipy.optimize import linear_sum_assignment
    n = 256
    W, x, y = skgen.euclidean(n, 0)
    ladder, tol, cap, t = [1], 1e-5, 20000, 1e-4
    want, status = oracle.adaptive(W, ladder, tol, cap, t, math.e)
    assert status == "ok"
    prm = sk.make_params(ladder, tol=tol, max_iters=cap, threshold=t, opt_ratio=math.e)
    out = ctx.solve(dev(W), prm)
    assert out["status"] == sk.SK_OK
    assert out["weight"] == want.weight == oracle.optimum_int(W)[1]
    assert out["report"]["optimal_proved"] == 1
    d = np.sqrt(((x[:, None, :] - y[None, :, :]) ** 2).sum(axis=2))
    r, c = linear_sum_assignment(d)
    assert d[np.arange(n), out["perm"]].sum() - d[r, c].sum() <= n / 1000.0
