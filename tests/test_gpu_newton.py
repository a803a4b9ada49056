"""GPU parity of Newton scaling (Section 5.2, the Knight-Ruiz method cited
there) against the oracle.

X(p) is unique (Section 2.1), so the matrix the GPU's Newton iteration
converges to must be the oracle's converged Sinkhorn limit. The GPU works in
FP32 (terms as in the sweeps, vectors and products in FP32, scalars of the
conjugate-gradient iteration in FP64); it stops at max_i |1 - (x o S x)_i|
<= tol, so log x is within a few tol of the limit on entries that matter.
"""
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


@pytest.mark.parametrize("n,hi,p", [(64, 100, 1), (256, 100, 2), (1000, 1000, 1), (129, 50, 3)])
def test_newton_reaches_the_sinkhorn_limit(ctx, n, hi, p):
    W = skgen.uniform_weights(n, 0, hi, seed=n + hi)
    B = oracle.log_weights(W)
    prm = sk.make_params([p], tol=1e-5, max_iters=5000, check_every=8, method="newton")
    res = ctx.scale(dev(W), prm)
    assert res.status == sk.SK_OK
    r = res.report
    assert r["residual_fp64"] < 5e-5 and r["col_residual_fp64"] < 5e-5
    lu, lv = sk.split_potentials(res.potentials, n)
    ub, vb = lu / p, lv / p
    us, vs, m, r2 = oracle.sinkhorn(B, p, 1e-12, 400000, -B.max(axis=1), None)
    Lg = p * (B + ub[:, None] + vb[None, :])
    Lo = p * (B + us[:, None] + vs[None, :])
    big = Lo > np.log(1e-6)
    assert np.abs(Lg - Lo)[big].max() < 1e-3
    # Newton needs far fewer products with A than Sinkhorn iterations
    assert r["iters_total"] < max(m, 50)


def test_newton_planted_solve(ctx):
    n = 1024
    W, sigma = skgen.planted(n, seed=9)
    prm = sk.make_params([1, 2, 4], tol=1e-5, max_iters=5000, threshold=1e-4, method="newton")
    out = ctx.solve(dev(W), prm)
    assert out["status"] == sk.SK_OK
    assert out["weight"] == 1050 * n and (out["perm"] == sigma).all()
    assert out["report"]["optimal_proved"] == 1


def test_newton_rejects_unsupported_combinations(ctx):
    W = skgen.uniform_weights(64, 0, 100, seed=1)
    for kw in ({"storage": "bf16"}, {"fused": True}, {"deform_a": 2.0}):
        prm = sk.make_params([1], method="newton", **kw)
        with pytest.raises(sk.SkError):
            ctx.scale(dev(W), prm)


def test_newton_full_size(ctx):
    """Newton scaling at n = 16384 (w uniform on 0..1000, p = 32, cold start
    F = -p rowmax, G = 0; the product kernels' two-chunk, non-temporal form).
    One product with S at x = 1 gives the row and column sums of the
    starting matrix: its reported max |1 - (S x)_i| equals the oracle's FP64
    sums on the same potentials. Run to tol from the same start, the result
    is a fixed point of the oracle's row and column steps on sampled rows and
    columns, and the library's FP64 recheck is within a few tol."""
    n, p = 16384, 32
    W = skgen.uniform_weights(n, 0, 1000, seed=3)
    Wd = dev(W)
    one = ctx.scale(Wd, sk.make_params([p], tol=1e-5, max_iters=1, method="newton"))
    assert one.status == sk.SK_ENOCONV and one.report["iters_total"] == 1
    lu0, lv0 = sk.split_potentials(one.potentials, n)  # the start (x = 1 folds to it)
    # the oracle's sums of the starting matrix, in row blocks
    rmax, csum = 0.0, np.zeros(n)
    blk = 2048
    for r0 in range(0, n, blk):
        Bb = oracle.log_weights(W[r0:r0 + blk])
        X = np.exp(Bb * p + lu0[r0:r0 + blk, None] + lv0[None, :])
        rmax = max(rmax, np.abs(X.sum(axis=1) - 1).max())
        csum += X.sum(axis=0)
    want = max(rmax, np.abs(csum - 1).max())
    assert want > 1.0  # far from balanced: the product is a real test
    assert abs(one.report["residual_fp32"] - want) <= 2e-6 * want
    res = ctx.scale(Wd, sk.make_params([p], tol=1e-5, max_iters=2000, check_every=8,
                                       method="newton"))
    assert res.status == sk.SK_OK
    r = res.report
    assert r["residual_fp64"] < 5e-5 and r["col_residual_fp64"] < 5e-5
    lu, lv = sk.split_potentials(res.potentials, n)
    rng = np.random.default_rng(2)
    rows = np.sort(rng.choice(n, 64, replace=False))
    cols = np.sort(rng.choice(n, 64, replace=False))
    u_or = p * oracle.row_step(oracle.log_weights(W[rows]), p, lv / p)
    v_or = p * oracle.col_step(oracle.log_weights(np.ascontiguousarray(W[:, cols])), p, lu / p)
    assert np.abs(lu[rows] - u_or).max() < 1e-4
    assert np.abs(lv[cols] - v_or).max() < 1e-4
