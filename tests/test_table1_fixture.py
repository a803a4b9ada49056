"""The Table 1 context fixture (tests/golden/table1_sinkhorn.txt, Section 5.1:
Algorithm 1 with Sinkhorn scaling at n = 1000) as the benchmark reads it,
checked against what Algorithm 1 fixes: p starts at 100 and rises by 50 per
round, gamma (the certificate's bound over the weight found) is at least 1,
and the kept entries are a percentage of the n^2 entries, at least the n of
a permutation."""
import bench


def test_table1_fixture_follows_algorithm1():
    rows = bench.table1_rows()
    assert len(rows) == 16 and "rand" in rows and "euclidean" in rows
    n = 1000
    for name, (gamma, p, iters, kept) in rows.items():
        assert gamma >= 1.0, name
        assert p >= 100 and (p - 100) % 50 == 0, name
        assert iters >= 1 and iters == int(iters), name
        assert 100.0 * n / n**2 <= kept <= 100.0, name
    assert rows["rand"] == (1.839, 100.0, 2.0, 25.87)
    assert rows["euclidean"] == (1.728, 200.0, 1416.0, 0.92)
