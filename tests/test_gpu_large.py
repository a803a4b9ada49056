"""Instances above 16384 (up to 65536): the int16 two-sweep path reads the
column entries from a packed per-instance buffer in global memory instead of
staging them in LDS (row sweep, FP64 check, CSR count and fill). Checked
against the oracle's row and column steps on sampled rows and columns, end
to end on a planted instance, and for the paths that keep the LDS limit, the
errors they return."""
import numpy as np
import pytest

import oracle
import paper_1104_3830_amd as sk
import skgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MARGIN = 1e-6  # the stopping test runs at tol - MARGIN (FP32 residual)


@pytest.fixture(scope="module")
def ctx():
    c = sk.Context(0)
    yield c
    c.close()


def dev(W):
    return torch.from_numpy(np.ascontiguousarray(W)).cuda()


def bars(pot, n, p):
    lu, lv = sk.split_potentials(pot, n)
    return lu / p, lv / p


@pytest.mark.parametrize("n", [16392, 20001])
def test_large_single_step_sampled(ctx, n):
    """One iteration from a warm start at p = 32 (w uniform on 0..1000): log u
    of sampled rows equals the oracle's row step on the starting v, log v of
    sampled columns the oracle's column step on the new u. 20001 runs on the
    library's padded 8-wide copy (a ragged last chunk)."""
    p = 32
    W = skgen.uniform_weights(n, 0, 1000, seed=7)
    Wd = dev(W)
    warm = ctx.scale(Wd, sk.make_params([p], tol=0.0, max_iters=20, check_every=20))
    _, vb0 = bars(warm.potentials, n, p)
    res = ctx.scale(Wd, sk.make_params([p], tol=0.0, max_iters=1, warm_start=True),
                    potentials=warm.potentials.clone())
    assert res.report["iters_total"] == 1
    ub1, vb1 = bars(res.potentials, n, p)
    rng = np.random.default_rng(1)
    rows = np.sort(np.r_[rng.choice(n - 8, 48, replace=False), np.arange(n - 4, n)])
    cols = np.sort(np.r_[rng.choice(n - 8, 48, replace=False), np.arange(n - 4, n)])
    u_or = oracle.row_step(oracle.log_weights(W[rows]), p, vb0)
    v_or = oracle.col_step(oracle.log_weights(np.ascontiguousarray(W[:, cols])), p, ub1)
    assert np.abs(p * (ub1[rows] - u_or)).max() < 2e-6 * np.log(n)
    assert np.abs(p * (vb1[cols] - v_or)).max() < 2e-6 * np.log(n)


def test_large_planted_solve(ctx):
    """n = 20000, w uniform on 0..1000 with w_i sigma(i) = 1050, ladder 1..32,
    tol 1e-5, t = 1e-4, through sk_solve: no stage capped, the FP64 recheck
    within 1e-5 in rows and columns, sigma recovered with weight 1050 n and
    the integer certificate proving it; sk_prune on the returned potentials
    (its own count pass) keeps as many entries as the solve's check counted,
    sigma among them, with the weights of W."""
    n = 20000
    W, sigma = skgen.planted(n, seed=21)
    Wd = dev(W)
    prm = sk.make_params([1, 2, 4, 8, 16, 32], tol=1e-5 - MARGIN, max_iters=5000, check_every=64,
                         threshold=1e-4)
    out = ctx.solve(Wd, prm)
    rep = out["report"]
    assert out["status"] == sk.SK_OK and rep["stages_capped"] == 0
    assert rep["residual_fp64"] <= 1e-5 and rep["col_residual_fp64"] <= 1e-5
    assert out["weight"] == 1050 * n
    assert np.array_equal(out["perm"], sigma)
    assert out["log_gamma"] < 1.0 and rep["optimal_proved"] == 1
    row_ptr, col, w = ctx.prune(Wd, out["potentials"], prm)
    rp, cc, ww = row_ptr.cpu().numpy(), col.cpu().numpy(), w.cpu().numpy()
    assert rp[-1] == out["nnz"] == len(cc)
    assert np.all(cc >= 0) and np.all(cc < n)
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert np.array_equal(ww, W[rows, cc])
    for i in np.r_[0, 1, 4999, 12345, n - 1]:
        seg = cc[rp[i]:rp[i + 1]]
        assert np.all(np.diff(seg) > 0) and sigma[i] in seg


def test_large_other_paths_refuse(ctx):
    """Above 16384 only the int16 two-sweep Sinkhorn path runs: stored K, the
    single pass, Newton, batches and real-valued weights return SK_EINVAL."""
    n = 16392
    Wd = dev(skgen.uniform_weights(n, 0, 1000, seed=2))
    for kw in (dict(storage="bf16"), dict(storage="f32"), dict(fused=True), dict(method="newton")):
        with pytest.raises(sk.SkError) as e:
            ctx.scale(Wd, sk.make_params([8], tol=1e-5, max_iters=10, **kw))
        assert e.value.status == sk.SK_EINVAL, kw
    with pytest.raises(sk.SkError) as e:
        ctx.scale_batch([Wd, dev(skgen.uniform_weights(64, 0, 1000, seed=3))],
                        sk.make_params([8], tol=1e-5, max_iters=10))
    assert e.value.status in (sk.SK_EINVAL, sk.SK_ENOMEM)
    Wr = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    with pytest.raises(sk.SkError) as e:
        ctx.scale_real(Wr, sk.make_params([8], tol=1e-5, max_iters=10))
    assert e.value.status in (sk.SK_EINVAL, sk.SK_ENOMEM)


def test_large_two_tile_rows_solve_and_prune(ctx):
    """n = 40000: in the row check and the CSR fill each row spans two LDS
    tiles of G_j (32768 columns each). The matrix: 4096 seeded rows uniform on
    0..1000, row i being row (i mod 4096) rotated right by 8 (i div 4096)
    columns. sk_solve (ladder 1..32, tol 1e-5, t = 1e-4; its counts and CSR
    from the tiled check and fill) returns a permutation whose weight is that
    of W and at most the certificate's bound (log gamma >= 0; with this many
    ties it proves nothing at p = 32); sk_prune on the same potentials
    (its own count pass) keeps as many entries as the solve counted, and the
    CSR of sampled rows is the oracle's kept set x_ij >= t (entries within
    1e-9 of log t aside) with the weights of W, in column order."""
    n, k, p, t = 40000, 4096, 32, 1e-4
    base = skgen.uniform_rows(k, n, 0, 1000, seed=31)

    def host_row(i):
        return np.roll(base[i % k], 8 * (i // k))

    bd = dev(base)
    Wd = torch.empty((n, n), dtype=torch.int16, device="cuda")
    for b in range((n + k - 1) // k):
        r0, r1 = b * k, min(n, (b + 1) * k)
        Wd[r0:r1] = torch.roll(bd[:r1 - r0], shifts=8 * b, dims=1)
    del bd
    prm = sk.make_params([1, 2, 4, 8, 16, p], tol=1e-5 - MARGIN, max_iters=5000, check_every=64,
                         threshold=t)
    out = ctx.solve(Wd, prm)
    rep = out["report"]
    assert out["status"] == sk.SK_OK and rep["stages_capped"] == 0
    perm = np.asarray(out["perm"])
    assert np.array_equal(np.sort(perm), np.arange(n))
    pd = torch.from_numpy(perm.astype(np.int64)).cuda()
    assert out["weight"] == int(Wd.gather(1, pd[:, None]).to(torch.int64).sum())
    assert out["log_gamma"] >= 0.0 and out["weight"] <= 1000 * n
    row_ptr, col, w = ctx.prune(Wd, out["potentials"], prm)
    rp, cc, ww = row_ptr.cpu().numpy(), col.cpu().numpy(), w.cpu().numpy()
    assert rp[-1] == out["nnz"] == len(cc)
    ub, vb = bars(out["potentials"], n, p)
    rng = np.random.default_rng(5)
    rows = np.sort(np.r_[0, 1, rng.choice(np.arange(2, n - 4), 60, replace=False), np.arange(n - 4, n)])
    Wr = np.stack([host_row(i) for i in rows])
    assert np.array_equal(Wr[:, :64], Wd[torch.from_numpy(rows).cuda(), :64].cpu().numpy())
    lx = p * (oracle.log_weights(Wr) + ub[rows][:, None] + vb[None, :])
    keep = oracle.scaled_matrix(oracle.log_weights(Wr), p, ub[rows], vb) >= t
    band = np.abs(lx - np.log(t)) < 1e-9
    beyond = 0
    for r, i in enumerate(rows):
        seg = cc[rp[i]:rp[i + 1]]
        assert np.all(np.diff(seg) > 0)
        assert np.array_equal(ww[rp[i]:rp[i + 1]], Wr[r, seg])
        got = np.zeros(n, dtype=bool)
        got[seg] = True
        assert np.array_equal(got[~band[r]], keep[r][~band[r]]), i
        beyond += int(np.sum(seg >= 32768))
    assert beyond > 0  # kept entries in the second tile were compared
