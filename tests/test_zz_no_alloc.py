"""GPU test of sk_scale_static (the entry point that allocates nothing: its
working memory is the library's static device scratch) against sk_scale
(the context's arena), through the C ABI."""
import numpy as np
import pytest

import paper_1104_3830_amd as sk
import skgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(W):
    return torch.from_numpy(np.ascontiguousarray(W)).cuda()


def same(a, b):
    assert a.status == b.status
    assert torch.equal(a.potentials, b.potentials)
    for k in ("iters_total", "iters_stage", "p_final", "stages_capped", "absorbs", "residual_fp32",
              "residual_fp64", "col_residual_fp64", "ub"):
        assert a.report[k] == b.report[k], k


@pytest.mark.parametrize("storage", ["i16", "bf16"])
def test_static_scratch_equals_arena(storage):
    """Two calls in a row, the second with a smaller (ragged) input: each
    result is bitwise the one sk_scale gives with the context's arena."""
    ctx = sk.Context(0)
    prm = sk.make_params([1, 2, 4, 8, 16, 32], tol=1e-5, max_iters=3000, check_every=32,
                         storage=storage)
    for n, seed in ((1024, 31), (300, 32)):
        W, _ = skgen.planted(n, seed=seed)
        Wd = dev(W)
        ref = ctx.scale(Wd, prm)
        got = ctx.scale_static(Wd, prm)
        same(got, ref)
    ctx.close()


def test_static_scratch_full_size_and_limit():
    """The benchmark's size (n = 16384, int16 W) fits the scratch and matches
    sk_scale; an instance whose working memory exceeds the scratch is refused
    with SK_ENOMEM before any work is queued."""
    ctx = sk.Context(0)
    n = 16384
    W = skgen.uniform_weights(n, 0, 1000, seed=3)
    Wd = dev(W)
    prm = sk.make_params([32], tol=0.0, max_iters=3, check_every=3)
    same(ctx.scale_static(Wd, prm), ctx.scale(Wd, prm))
    with pytest.raises(sk.SkError) as e:
        ctx.scale_static(Wd, sk.make_params([32], tol=0.0, max_iters=3, storage="bf16"))
    assert e.value.status == sk.SK_ENOMEM
    ctx.close()
