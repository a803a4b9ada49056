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
