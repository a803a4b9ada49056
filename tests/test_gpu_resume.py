"""Checkpoint and resume: the potentials returned by a scaling call are the
whole state of the iteration within a stage (u and v in the log domain, as
Section 4.1.2 carries them), so a run of 20 iterations equals a run of 10
whose potentials are passed back with warm_start for 10 more, bit for bit.
This holds for every path that keeps the iterate in the potentials alone:
int16 W (two sweeps and the single pass), real-valued log-weights, and the
batched call."""
import numpy as np
import pytest

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


def split_run(run, total, first):
    """run(max_iters, warm_start, potentials) -> Result; returns the
    straight run and the checkpointed one."""
    straight = run(total, False, None)
    a = run(first, False, None)
    b = run(total - first, True, a.potentials.clone())
    return straight, a, b


@pytest.mark.parametrize("n,fused", [(1000, False), (4096, False), (16384, False), (4096, True)])
def test_resume_int16_bitwise(ctx, n, fused):
    W = dev(skgen.uniform_weights(n, 0, 1000, seed=11))

    def run(iters, warm, pot):
        return ctx.scale(W, sk.make_params([16], tol=0.0, max_iters=iters, check_every=8,
                                           warm_start=warm, fused=fused), potentials=pot)

    straight, a, b = split_run(run, 20, 10)
    assert straight.status == a.status == b.status in (sk.SK_OK, sk.SK_ENOCONV)
    assert straight.report["iters_total"] == 20
    assert a.report["iters_total"] == 10 and b.report["iters_total"] == 10
    assert torch.equal(straight.potentials, b.potentials)
    # the checkpoint is not already the end state (the run moved on)
    assert not torch.equal(a.potentials, b.potentials)


def test_resume_real_bitwise(ctx):
    W = skgen.euclidean_real(1000, seed=5)
    Wd = dev(W)

    def run(iters, warm, pot):
        return ctx.scale_real(Wd, sk.make_params([200], tol=0.0, max_iters=iters, check_every=8,
                                                 warm_start=warm, prescale=True), potentials=pot)

    straight, a, b = split_run(run, 30, 17)
    assert straight.status == a.status == b.status in (sk.SK_OK, sk.SK_ENOCONV)
    assert torch.equal(straight.potentials, b.potentials)
    assert not torch.equal(a.potentials, b.potentials)


def test_resume_batch_bitwise(ctx):
    ns = [37, 256, 1000]
    Ws = [dev(skgen.uniform_weights(n, 0, 1000, seed=40 + k)) for k, n in enumerate(ns)]

    def prm(iters, warm):
        return sk.make_params([8], tol=0.0, max_iters=iters, check_every=8, warm_start=warm)

    straight = ctx.scale_batch(Ws, prm(24, False))
    first = ctx.scale_batch(Ws, prm(9, False))
    rest = ctx.scale_batch(Ws, prm(15, True), potentials=[r.potentials.clone() for r in first])
    for s, r in zip(straight, rest):
        assert s.status == r.status in (sk.SK_OK, sk.SK_ENOCONV)
        assert torch.equal(s.potentials, r.potentials)
