"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, the ctypes mirrors match the C layouts, and the host exact
solver (no GPU needed) agrees with the oracle and with brute force."""
import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import paper_1104_3830_amd as sk
from oracle import brute

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sk.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sk_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 10
    L = sk.lib()
    missing = [nm for nm in names if not hasattr(L, nm)]
    assert not missing, missing
    assert set(names) == set(sk.EXPORTS)


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(f'''#include <stdio.h>
#include <stddef.h>
#include "{HEADER}"
int main(void) {{
  printf("%zu %zu %zu\\n", sizeof(sk_params), sizeof(sk_report), sizeof(sk_csr));
  printf("%zu %zu %zu %zu %zu\\n", offsetof(sk_params, tol), offsetof(sk_params, storage),
         offsetof(sk_params, warm_start), offsetof(sk_params, fused), offsetof(sk_report, seconds));
  printf("%zu %zu\\n", offsetof(sk_report, nnz_kept), offsetof(sk_csr, w));
  printf("%zu %zu %zu %zu\\n", offsetof(sk_params, prescale), offsetof(sk_report, p_scale),
         sizeof(sk_csr_real), offsetof(sk_csr_real, w));
  return 0;
}}''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    got = [int(x) for x in out]
    want = [ctypes.sizeof(sk.Params), ctypes.sizeof(sk.Report), ctypes.sizeof(sk.CSR),
            sk.Params.tol.offset, sk.Params.storage.offset, sk.Params.warm_start.offset,
            sk.Params.fused.offset, sk.Report.seconds.offset, sk.Report.nnz_kept.offset, sk.CSR.w.offset,
            sk.Params.prescale.offset, sk.Report.p_scale.offset, ctypes.sizeof(sk.CSRReal),
            sk.CSRReal.w.offset]
    assert got == want


def test_potentials_pack_roundtrip():
    rng = np.random.default_rng(0)
    lu = rng.normal(size=37) * 3e4
    lv = rng.normal(size=37) * 50
    raw = sk.pack_potentials(lu, lv)
    assert raw.size == sk.potentials_bytes(37)
    u2, v2 = sk.split_potentials(raw, 37)
    assert np.abs(u2 - lu).max() < 1e-6 and np.abs(v2 - lv).max() < 1e-6


def _csr(mask, w):
    n = mask.shape[0]
    rp = np.concatenate([[0], np.cumsum(mask.sum(1))]).astype(np.int64)
    cols = np.nonzero(mask)[1].astype(np.int32)
    return rp, cols, w[mask].astype(np.int16)


@pytest.mark.parametrize("n", [1, 2, 5, 7])
def test_solve_reduced_vs_brute_force(n):
    rng = np.random.default_rng(100 + n)
    for trial in range(10):
        w = rng.integers(-50, 51, (n, n))
        mask = rng.random((n, n)) < 0.6
        rp, cols, ww = _csr(mask, w)
        b = np.where(mask, w.astype(float), -np.inf)
        best, winners = brute.all_optima(b)
        if best == -math.inf:
            with pytest.raises(sk.SkError) as e:
                sk.solve_reduced(rp, cols, ww, n)
            assert e.value.status == sk.SK_EINFEASIBLE
            continue
        perm, weight = sk.solve_reduced(rp, cols, ww, n)
        assert weight == best and tuple(perm) in winners


def test_solve_reduced_vs_oracle_hungarian():
    rng = np.random.default_rng(7)
    for n in (40, 200, 600):
        w = rng.integers(0, 1001, (n, n))
        mask = rng.random((n, n)) < 0.05
        mask[np.arange(n), rng.permutation(n)] = True
        rp, cols, ww = _csr(mask, w)
        perm, weight = sk.solve_reduced(rp, cols, ww, n)
        _, w_or = oracle.hungarian(w, mask)
        assert weight == w_or
        assert sorted(perm) == list(range(n))
        assert mask[np.arange(n), perm].all()


def test_solve_reduced_large_split_over_threads():
    """An instance with more than 2^17 entries: the reductions run on several
    host threads. The optimum equals the oracle's; an empty row or a bad
    column index late in the rows is still reported (the first bad row in row
    order decides the status)."""
    rng = np.random.default_rng(11)
    n = 1500
    w = rng.integers(0, 1001, (n, n))
    mask = rng.random((n, n)) < 0.07
    mask[np.arange(n), rng.permutation(n)] = True
    rp, cols, ww = _csr(mask, w)
    assert rp[-1] >= 1 << 17
    perm, weight = sk.solve_reduced(rp, cols, ww, n)
    _, w_or = oracle.hungarian(w, mask)
    assert weight == w_or
    assert sorted(perm) == list(range(n)) and mask[np.arange(n), perm].all()
    bad = cols.copy()
    bad[rp[n - 3]] = n + 5  # a column index out of range in one of the last rows
    with pytest.raises(sk.SkError) as e:
        sk.solve_reduced(rp, bad, ww, n)
    assert e.value.status == sk.SK_EINVAL
    m2 = mask.copy()
    m2[n - 2, :] = False  # an empty row late in the rows, before the bad index
    rp2, cols2, ww2 = _csr(m2, w)
    bad2 = cols2.copy()
    bad2[rp2[n - 1]] = -1
    with pytest.raises(sk.SkError) as e:
        sk.solve_reduced(rp2, bad2, ww2, n)
    assert e.value.status == sk.SK_EINFEASIBLE
    # the two faults in different threads' rows: the earlier row decides
    m3 = mask.copy()
    m3[10, :] = False
    rp3, cols3, ww3 = _csr(m3, w)
    bad3 = cols3.copy()
    bad3[rp3[n - 1]] = n
    with pytest.raises(sk.SkError) as e:
        sk.solve_reduced(rp3, bad3, ww3, n)
    assert e.value.status == sk.SK_EINFEASIBLE
    m4 = mask.copy()
    m4[n - 1, :] = False
    rp4, cols4, ww4 = _csr(m4, w)
    cols4[rp4[10]] = n
    with pytest.raises(sk.SkError) as e:
        sk.solve_reduced(rp4, cols4, ww4, n)
    assert e.value.status == sk.SK_EINVAL


def test_solve_reduced_errors():
    # empty row
    rp = np.array([0, 1, 1], dtype=np.int64)
    with pytest.raises(sk.SkError) as e:
        sk.solve_reduced(rp, np.array([0], np.int32), np.array([3], np.int16), 2)
    assert e.value.status == sk.SK_EINFEASIBLE
    # two rows, one column usable -> no perfect matching
    rp = np.array([0, 1, 2], dtype=np.int64)
    with pytest.raises(sk.SkError) as e:
        sk.solve_reduced(rp, np.array([1, 1], np.int32), np.array([3, 4], np.int16), 2)
    assert e.value.status == sk.SK_EINFEASIBLE
    # column index out of range
    with pytest.raises(sk.SkError) as e:
        sk.solve_reduced(rp, np.array([0, 5], np.int32), np.array([3, 4], np.int16), 2)
    assert e.value.status == sk.SK_EINVAL
    # n = 0
    perm, weight = sk.solve_reduced(np.array([0], np.int64), np.array([], np.int32),
                                    np.array([], np.int16), 0)
    assert weight == 0


def test_arena_sizes_include_the_padded_copy():
    """A W whose n is not a multiple of 8 is copied into the library's 8-wide
    layout (pitch rounded up to 8): the arena sizes grow by that copy, and
    only for such n."""
    L = sk.lib()
    copy = 2 * 1001 * 1008
    assert L.sk_arena_bytes(1001, 0) - L.sk_arena_bytes(1000, 0) >= copy
    assert L.sk_arena_bytes(1008, 0) - L.sk_arena_bytes(1000, 0) < copy // 4
    one = lambda n: L.sk_batch_arena_bytes(1, (ctypes.c_int32 * 1)(n), 0)
    assert one(1001) - one(1000) >= copy
    assert one(1008) - one(1000) < copy // 4
    two = L.sk_batch_arena_bytes(2, (ctypes.c_int32 * 2)(1001, 37), 0)
    assert two - L.sk_batch_arena_bytes(2, (ctypes.c_int32 * 2)(1000, 40), 0) >= copy + 2 * 37 * 40


def _budget_instance():
    """Row block A (1200 rows) complete onto 600 columns at weight 100, each
    A row also reaching a column of its own at weight 0; 600 rows B each
    reaching the own columns of two A rows at weight 50. After the row and
    column reductions the tight edges are A x (600 columns) and the B edges,
    so 600 A rows are left free and every search from one of them visits the
    whole A block without finding a free column."""
    k = 1200
    n = k + k // 2
    w = np.zeros((n, n), np.int64)
    mask = np.zeros((n, n), bool)
    mask[:k, : k // 2] = True
    w[:k, : k // 2] = 100
    own = k // 2 + np.arange(k)
    mask[np.arange(k), own] = True
    for t in range(k // 2):
        for c in (own[2 * t], own[2 * t + 1]):
            mask[k + t, c] = True
            w[k + t, c] = 50
    return n, w, mask


def test_solve_reduced_when_searches_exhaust_their_budget():
    """Single-row augmenting searches that fail on the tight graph use up
    their shared budget; the rest of the matching goes to Hopcroft-Karp and
    the shortest-path augmentations, and the optimum is still exact
    (600*100 + 600*50)."""
    n, w, mask = _budget_instance()
    rp, cols, ww = _csr(mask, w)
    perm, weight = sk.solve_reduced(rp, cols, ww, n)
    _, w_or = oracle.hungarian(w, mask)
    assert weight == w_or == 600 * 100 + 600 * 50
    assert sorted(perm) == list(range(n)) and mask[np.arange(n), perm].all()


def test_solve_reduced_all_tight_random_graph():
    """Every entry has the same weight, so every edge is tight and the
    matching is found by the augmenting searches alone: a random graph of 8
    entries per row plus a planted permutation (a perfect matching exists)."""
    rng = np.random.default_rng(5)
    n = 4000
    mask = np.zeros((n, n), bool)
    mask[np.repeat(np.arange(n), 8), rng.integers(0, n, 8 * n)] = True
    mask[np.arange(n), rng.permutation(n)] = True
    w = np.full((n, n), 1000, np.int64)
    rp, cols, ww = _csr(mask, w)
    perm, weight = sk.solve_reduced(rp, cols, ww, n)
    assert weight == 1000 * n
    assert sorted(perm) == list(range(n)) and mask[np.arange(n), perm].all()


# ---------------------------------------------------------------- real-weight exact solve

def _csr_of(b):
    """CSR (row_ptr, col, w float32) of the finite entries of b."""
    n = b.shape[0]
    rp, cols, ws = [0], [], []
    for i in range(n):
        js = np.nonzero(np.isfinite(b[i]))[0]
        cols.extend(js.tolist())
        ws.extend(b[i, js].tolist())
        rp.append(len(cols))
    return (np.array(rp, dtype=np.int64), np.array(cols, dtype=np.int32),
            np.array(ws, dtype=np.float32))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 8])
def test_real_solver_vs_brute_force(n):
    rng = np.random.default_rng(200 + n)
    for trial in range(8):
        w = (rng.standard_normal((n, n)) * 2.0).astype(np.float32).astype(np.float64)
        keep = rng.random((n, n)) < (0.45 if trial % 2 else 1.0)
        b = np.where(keep, w, -np.inf)
        best, _ = brute.all_optima(b)
        rp, col, ww = _csr_of(b)
        if best == -math.inf:
            with pytest.raises(sk.SkError) as e:
                sk.solve_reduced_real(rp, col, ww, n)
            assert e.value.status == sk.SK_EINFEASIBLE
            continue
        perm, weight = sk.solve_reduced_real(rp, col, ww, n)
        assert sorted(perm.tolist()) == list(range(n))
        assert np.isfinite(b[np.arange(n), perm]).all()
        assert weight == pytest.approx(best, abs=1e-9)
        assert weight == pytest.approx(b[np.arange(n), perm].sum(), abs=1e-9)


def test_real_solver_vs_oracle_on_sparse_instances():
    """Sparse random instances (about 8 entries per row plus a hidden perfect
    matching, so one exists) against the oracle's dense real Hungarian."""
    rng = np.random.default_rng(5)
    for n in (50, 300, 1000):
        w = -rng.uniform(0.0, 1.73, (n, n)).astype(np.float32).astype(np.float64)
        keep = rng.random((n, n)) < 8.0 / n
        keep[np.arange(n), rng.permutation(n)] = True
        b = np.where(keep, w, -np.inf)
        rp, col, ww = _csr_of(b)
        perm, weight = sk.solve_reduced_real(rp, col, ww, n)
        _, w_or = oracle.hungarian_real(b)
        assert weight == pytest.approx(w_or, abs=1e-7)
        assert np.isfinite(b[np.arange(n), perm]).all()


def test_real_solver_rejects_bad_csr():
    rp = np.array([0, 1, 2], dtype=np.int64)
    col = np.array([0, 5], dtype=np.int32)  # column out of range
    with pytest.raises(sk.SkError) as e:
        sk.solve_reduced_real(rp, col, np.array([1.0, 2.0], dtype=np.float32), 2)
    assert e.value.status == sk.SK_EINVAL
    col = np.array([0, 0], dtype=np.int32)  # both rows on column 0
    with pytest.raises(sk.SkError) as e:
        sk.solve_reduced_real(rp, col, np.array([1.0, 2.0], dtype=np.float32), 2)
    assert e.value.status == sk.SK_EINFEASIBLE


def test_tuned_tile_table_is_valid_and_loaded():
    """The autotuner's committed table (column-sweep segment heights per size
    bucket) is well formed, accepted by sk_set_tile_table and loaded by the
    binding at import."""
    import json
    if not os.path.exists(sk.TILE_TABLE):
        pytest.skip("no tuned table committed")
    tab = json.load(open(sk.TILE_TABLE))
    ent = [(e["n_max"], e["seg_rows"]) for e in tab["entries"]]
    assert ent and all(a < b for (a, _), (b, _) in zip(ent, ent[1:]))
    assert all(16 <= s <= 1024 and s % 16 == 0 for _, s in ent)
    sk.lib()
    if not os.environ.get("SK_NO_TILE_TABLE"):
        assert sk.loaded_tile_table == ent


def test_static_scratch_limits_documented_in_header():
    """The sizes include/sk.h gives for sk_scale_static are the largest whose
    sk_arena_bytes fit SK_STATIC_SCRATCH_BYTES (64 MiB): int16 W n = 44016
    (a multiple of 8), a ragged n = 5343, BF16 K n = 5336, FP32 K n = 3888."""
    L = sk.lib()
    lim = 64 << 20
    assert "SK_STATIC_SCRATCH_BYTES ((size_t)64 << 20)" in open(os.path.join(ROOT, "include", "sk.h")).read()
    for n, step, storage in ((44016, 8, 0), (5343, 1, 0), (5336, 8, 1), (3888, 8, 2)):
        assert L.sk_arena_bytes(n, storage) <= lim, (n, storage)
        nxt = n + step
        while storage == 0 and step == 1 and nxt % 8 == 0:
            nxt += 1  # the next ragged size
        assert L.sk_arena_bytes(nxt, storage) > lim, (nxt, storage)


def test_size_limits():
    """Single instances go up to n = 65536 (int16 W, two sweeps); 65537 has no
    arena size. Batches stay at n <= 16384."""
    L = sk.lib()
    assert L.sk_arena_bytes(65536, 0) > L.sk_arena_bytes(16384, 0) > 0
    assert L.sk_arena_bytes(65537, 0) == 0
