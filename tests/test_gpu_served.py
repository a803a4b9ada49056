"""GPU tests of the served path (continuous batching through sk_submit/sk_poll)."""
import time

import numpy as np
import pytest

import oracle
import paper_1104_3830_amd as sk
import skgen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

LADDER = [1, 2, 4, 8, 16, 32]


def wait_all(ctx, tickets, ns, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t, n in zip(tickets, ns):
            if t in out:
                continue
            r = ctx.poll(t, n)
            if r is not None:
                out[t] = r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(out)}/{len(tickets)} requests finished")
        time.sleep(0.002)
    return [out[t] for t in tickets]


def test_served_results_equal_alone_and_in_the_mix():
    """Each request's result (permutation, weight, certificate, iteration
    counts) is bitwise the same when served in a mix as when solved alone."""
    ns = [64, 100, 256, 333, 512, 1000, 2048]
    insts = [skgen.planted(n, seed=500 + k) for k, n in enumerate(ns)]
    prm = sk.make_params(LADDER, tol=1e-5, max_iters=2000, threshold=1e-4)
    alone = sk.Context(0)
    ref = [alone.solve(torch.from_numpy(W).cuda(), prm) for W, _ in insts]
    alone.close()
    srv = sk.Context(0, arena_bytes=1 << 30)
    tickets = [srv.submit(W, prm) for W, _ in insts]
    res = wait_all(srv, tickets, ns)
    srv.close()
    for (W, sigma), r, (st, perm, weight, rep) in zip(insts, ref, res):
        assert st in (sk.SK_OK, sk.SK_ENOCONV)
        assert weight == r["weight"] == 1050 * W.shape[0]
        assert np.array_equal(perm, r["perm"]) and np.array_equal(perm, sigma)
        assert rep["ub"] == r["report"]["ub"]
        assert rep["iters_stage"] == r["report"]["iters_stage"]
        assert rep["residual_fp64"] == r["report"]["residual_fp64"]
        assert rep["nnz_kept"] == r["nnz"]


def test_served_admission_with_small_arena():
    """An arena that holds about one instance at a time still serves every
    request (admission waits for memory to free up), and each result is
    bitwise the one the instance gives alone and the planted optimum."""
    ns = [512, 512, 400, 512]
    insts = [skgen.planted(n, seed=20 + k) for k, n in enumerate(ns)]
    prm = sk.make_params(LADDER, tol=1e-5, max_iters=2000, threshold=1e-4)
    alone = sk.Context(0)
    ref = [alone.solve(torch.from_numpy(W).cuda(), prm) for W, _ in insts]
    alone.close()
    need = int(sk.lib().sk_arena_bytes(512, 0)) + 512 * 512 * 2
    srv = sk.Context(0, arena_bytes=(64 << 20) + 2 * need)
    tickets = [srv.submit(W, prm) for W, _ in insts]
    res = wait_all(srv, tickets, ns)
    srv.close()
    for (W, sigma), r, (st, perm, weight, rep) in zip(insts, ref, res):
        n = W.shape[0]
        assert st == sk.SK_OK == r["status"]
        assert weight == r["weight"] == 1050 * n == oracle.optimum_int(W)[1]
        assert np.array_equal(perm, sigma) and np.array_equal(perm, r["perm"])
        assert rep["ub"] == r["report"]["ub"]
        assert rep["iters_stage"] == r["report"]["iters_stage"]
        assert rep["residual_fp64"] == r["report"]["residual_fp64"]


def test_served_bad_request_does_not_block_others():
    good = [skgen.planted(128, seed=k)[0] for k in range(3)]
    bad = skgen.uniform_weights(128, 0, 10, seed=9)
    bad[5, :] = sk.SENTINEL
    prm = sk.make_params(LADDER, tol=1e-5, max_iters=2000, threshold=1e-4)
    srv = sk.Context(0, arena_bytes=256 << 20)
    tickets = [srv.submit(good[0], prm), srv.submit(bad, prm), srv.submit(good[1], prm),
               srv.submit(good[2], prm)]
    res = wait_all(srv, tickets, [128] * 4)
    srv.close()
    assert res[1][0] == sk.SK_ENOSUPPORT
    for r in (res[0], res[2], res[3]):
        assert r[0] in (sk.SK_OK, sk.SK_ENOCONV) and r[2] == 1050 * 128


def test_completion_queue_lists_each_finished_request_once():
    """sk_completed lists every finished request exactly once, in completion
    order, and the results collected through it equal direct polling; more
    requests than the pinned staging ring holds are taken in with SK_EAGAIN
    back-pressure."""
    ns = [64, 96, 200, 257, 512, 777, 1024, 64]
    insts = [skgen.planted(n, seed=900 + k) for k, n in enumerate(ns)]
    prm = sk.make_params(LADDER, tol=1e-5, max_iters=2000, threshold=1e-4)
    srv = sk.Context(0, arena_bytes=256 << 20)
    assert srv.completed() == []  # nothing submitted yet
    ticket_of = {}
    for k, (W, _) in enumerate(insts):
        ticket_of[srv.submit(W, prm)] = k
    got, seen = {}, []
    t0 = time.time()
    while len(got) < len(insts):
        for tk in srv.completed(max_tickets=3):
            assert tk in ticket_of and tk not in got
            seen.append(tk)
            got[tk] = srv.poll(tk, ns[ticket_of[tk]])
        assert time.time() - t0 < 120.0
        time.sleep(0.002)
    assert srv.completed() == []  # all collected
    # the same requests polled directly give the same answers
    again = [srv.submit(W, prm) for W, _ in insts]
    res = wait_all(srv, again, ns)
    srv.close()
    for tk, k in ticket_of.items():
        st, perm, weight, rep = got[tk]
        st2, perm2, weight2, rep2 = res[k]
        assert st == st2 and weight == weight2 and np.array_equal(perm, perm2)
        assert weight == 1050 * ns[k]
    # many large requests: the ring (512 MiB) fills, submit answers SK_EAGAIN
    big = skgen.planted(4096, seed=77)[0]  # 32 MiB each
    srv = sk.Context(0, arena_bytes=512 << 20)
    tickets, eagain = [], 0
    t0 = time.time()
    while len(tickets) < 40:
        try:
            tickets.append(srv.submit(big, prm))
        except sk.SkError as e:
            assert e.status == sk.SK_EAGAIN
            eagain += 1
            time.sleep(0.002)
        assert time.time() - t0 < 120.0
    res = wait_all(srv, tickets, [4096] * len(tickets))
    srv.close()
    assert all(r[2] == 1050 * 4096 for r in res)


def test_served_largest_request_with_small_ones():
    """The served workload's largest size, n = 8192 (planted, w uniform on
    0..1000 with w_i sigma(i) = 1050), submitted with small requests: every
    request returns its unique optimum sigma with the closed-form weight
    1050 n."""
    ns = [8192, 64, 257, 1000]
    insts = [skgen.planted(n, seed=700 + k) for k, n in enumerate(ns)]
    prm = sk.make_params(LADDER, tol=1e-5, max_iters=2000, check_every=32, threshold=1e-4)
    need = sum(int(sk.lib().sk_arena_bytes(n, 0)) + 2 * n * ((n + 7) // 8 * 8) for n in ns)
    srv = sk.Context(0, arena_bytes=need + (96 << 20))
    tickets = [srv.submit(W, prm) for W, _ in insts]
    res = wait_all(srv, tickets, ns)
    for (W, sigma), n, (st, perm, weight, rep) in zip(insts, ns, res):
        assert st == sk.SK_OK, (n, st)
        assert weight == 1050 * n
        assert np.array_equal(perm, sigma)
    srv.close()
