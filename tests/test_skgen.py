"""The seeded input generators: reproducible, in range, and the rectangular
form equal to the leading rows of the square one."""
import numpy as np

import skgen


def test_uniform_rows_are_leading_rows_of_uniform_weights():
    A = skgen.uniform_weights(300, 0, 1000, seed=5, chunk_rows=64)
    for k in (1, 63, 64, 120, 300):
        assert np.array_equal(skgen.uniform_rows(k, 300, 0, 1000, seed=5), A[:k])
    assert A.dtype == np.int16 and A.min() >= 0 and A.max() <= 1000
    # every value of a small range appears, and another seed differs
    assert np.array_equal(np.unique(skgen.uniform_rows(40, 50, -3, 3, seed=1)), np.arange(-3, 4))
    assert not np.array_equal(skgen.uniform_weights(300, 0, 1000, seed=6), A)
