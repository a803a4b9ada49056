"""Seeded synthetic inputs for the optimal-assignment workloads.

This module is shared by the tests, the benchmark and the oracle's checks. It
holds only random-number generation and the shapes of the workloads; none of
the scaling, pruning or assignment arithmetic lives here.

Generator: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) used in counter mode: draw number k of stream
(seed, tag) is mix(s0 + (k + 1) * GOLDEN) with s0 = mix(seed * GOLDEN ^ tag).
Bounded integers use Lemire's multiply-shift on the top 32 bits (no rejection
step; the bias is below range / 2**32).

Weights are log-weights w_ij = log a_ij stored as int16, row-major, pitch n.
The sentinel INT16_MIN stands for a_ij = 0 (w_ij = -inf); valid weights lie in
[-16384, 16383].
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
SENTINEL = -32768
W_MIN, W_MAX = -16384, 16383

# stream tags: one independent stream per purpose
TAG_W = 1
TAG_PERM = 2
TAG_MASK = 3
TAG_DIAG = 4
TAG_SIZES = 5
TAG_ARRIVALS = 6
TAG_OFFDIAG = 7
TAG_POINTS = 8
TAG_REAL = 9


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _seed_state(seed: int, tag: int) -> np.uint64:
    with np.errstate(over="ignore"):
        s = np.array([(int(seed) * int(GOLDEN) ^ int(tag)) & 0xFFFFFFFFFFFFFFFF],
                     dtype=np.uint64)
        return _mix(s)[0]


def stream(seed: int, tag: int, count: int, offset: int = 0) -> np.ndarray:
    """Draws offset .. offset+count-1 of stream (seed, tag) as uint64."""
    s0 = _seed_state(seed, tag)
    k = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(s0 + k * GOLDEN)


def bounded(z: np.ndarray, r: int) -> np.ndarray:
    """Integers in [0, r) from uint64 draws (multiply-shift on the top 32 bits)."""
    return ((z >> np.uint64(32)) * np.uint64(r)) >> np.uint64(32)


def unit(z: np.ndarray) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits."""
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def uniform_weights(n: int, lo: int, hi: int, seed: int, chunk_rows: int = 1024) -> np.ndarray:
    """n x n int16 matrix with entries uniform on the integers lo..hi."""
    return uniform_rows(n, n, lo, hi, seed, chunk_rows)


def uniform_rows(k: int, n: int, lo: int, hi: int, seed: int, chunk_rows: int = 1024) -> np.ndarray:
    """The first k rows of the n-column uniform matrix of (seed): k x n int16,
    entries uniform on the integers lo..hi (uniform_weights(n) for k = n)."""
    assert W_MIN <= lo <= hi <= W_MAX
    W = np.empty((k, n), dtype=np.int16)
    for r0 in range(0, k, chunk_rows):
        r1 = min(k, r0 + chunk_rows)
        z = stream(seed, TAG_W, (r1 - r0) * n, offset=r0 * n)
        W[r0:r1] = (bounded(z, hi - lo + 1).astype(np.int64) + lo).reshape(r1 - r0, n)
    return W


def permutation(n: int, seed: int) -> np.ndarray:
    """Fisher-Yates shuffle of 0..n-1 driven by stream (seed, TAG_PERM)."""
    z = stream(seed, TAG_PERM, max(n - 1, 0))
    perm = np.arange(n, dtype=np.int64)
    for k, i in enumerate(range(n - 1, 0, -1)):
        j = int(bounded(z[k:k + 1], i + 1)[0])
        perm[i], perm[j] = perm[j], perm[i]
    return perm


def planted(n: int, seed: int, lo: int = 0, hi: int = 1000, bonus: int = 50):
    """Uniform weights on lo..hi with w[i, sigma(i)] := hi + bonus.

    Every permutation other than sigma loses at least `bonus` per row where it
    differs, so sigma is the unique optimum and its weight is n * (hi + bonus).
    Returns (W, sigma).
    """
    W = uniform_weights(n, lo, hi, seed)
    sigma = permutation(n, seed)
    W[np.arange(n), sigma] = hi + bonus
    return W, sigma


def dominant(n: int, seed: int, density: float = 0.05, diag_lo: int = 800,
             diag_hi: int = 1000, off_hi: int = 600, chunk_rows: int = 1024) -> np.ndarray:
    """Diagonally dominant sparse pattern (pivoting-like workload).

    w_ii uniform on diag_lo..diag_hi; each off-diagonal entry present with
    probability `density`, value uniform on 0..off_hi; absent entries hold the
    sentinel. Since every diagonal weight exceeds every off-diagonal one, the
    identity is the unique optimal assignment.
    """
    W = np.empty((n, n), dtype=np.int16)
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        zm = stream(seed, TAG_MASK, (r1 - r0) * n, offset=r0 * n)
        zv = stream(seed, TAG_OFFDIAG, (r1 - r0) * n, offset=r0 * n)
        keep = unit(zm) < density
        vals = bounded(zv, off_hi + 1).astype(np.int16)
        W[r0:r1] = np.where(keep, vals, np.int16(SENTINEL)).reshape(r1 - r0, n)
    zd = stream(seed, TAG_DIAG, n)
    W[np.arange(n), np.arange(n)] = (bounded(zd, diag_hi - diag_lo + 1).astype(np.int64)
                                     + diag_lo).astype(np.int16)
    return W


def sizes_loguniform(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Instance sizes n = round(exp(U(ln lo, ln hi)))."""
    u = unit(stream(seed, TAG_SIZES, count))
    n = np.rint(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)
    return np.clip(n, lo, hi)


def poisson_arrivals(rate: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process with the given rate."""
    u = unit(stream(seed, TAG_ARRIVALS, count))
    gaps = -np.log1p(-u) / rate
    return np.cumsum(gaps)


def batch(count: int, lo: int, hi: int, seed: int, wlo: int = 0, whi: int = 1000):
    """A ragged batch: log-uniform sizes, uniform weights; instance k uses seed*100003+k."""
    ns = sizes_loguniform(count, lo, hi, seed)
    return [uniform_weights(int(n), wlo, whi, seed * 100003 + k) for k, n in enumerate(ns)]


def planted_batch(count: int, lo: int, hi: int, seed: int):
    """A ragged batch of planted instances: list of (W, sigma)."""
    ns = sizes_loguniform(count, lo, hi, seed)
    return [planted(int(n), seed * 100003 + k) for k, n in enumerate(ns)]


def euclidean_points(n: int, seed: int):
    """2n points uniform in the unit cube of R^3: (x, y), each of shape (n, 3)."""
    u = unit(stream(seed, TAG_POINTS, 6 * n)).reshape(2, n, 3)
    return u[0], u[1]


def euclidean(n: int, seed: int, scale: int = 1000, chunk_rows: int = 1024):
    """Euclidean random assignment workload: a_ij = exp(-d(x_i, y_j)) for the
    points of euclidean_points. The int16 log-weights are the distances
    quantised at 1/scale: w_ij = -round(scale * d(x_i, y_j)) (d <= sqrt 3, so
    |w| <= 1733 at scale 1000). Returns (W, x, y)."""
    x, y = euclidean_points(n, seed)
    W = np.empty((n, n), dtype=np.int16)
    for r in range(0, n, chunk_rows):
        d = np.sqrt(((x[r:r + chunk_rows, None, :] - y[None, :, :]) ** 2).sum(axis=2))
        W[r:r + chunk_rows] = -np.rint(scale * d).astype(np.int16)
    return W, x, y


def euclidean_real(n: int, seed: int, chunk_rows: int = 1024):
    """The Euclidean random assignment workload with real log-weights:
    w_ij = -d(x_i, y_j) as float32 (a_ij = exp(-d)), no quantisation.
    Returns W (the points are euclidean_points(n, seed))."""
    x, y = euclidean_points(n, seed)
    W = np.empty((n, n), dtype=np.float32)
    for r in range(0, n, chunk_rows):
        d = np.sqrt(((x[r:r + chunk_rows, None, :] - y[None, :, :]) ** 2).sum(axis=2))
        W[r:r + chunk_rows] = (-d).astype(np.float32)
    return W


def uniform_real(n: int, seed: int, chunk_rows: int = 1024):
    """A matrix with entries uniform on (0, 1] given by its log-weights
    w_ij = log a_ij (float32), the random matrix of Section 5's experiments."""
    W = np.empty((n, n), dtype=np.float32)
    for r in range(0, n, chunk_rows):
        rows = min(chunk_rows, n - r)
        u = unit(stream(seed, TAG_REAL, rows * n, offset=r * n)).reshape(rows, n)
        W[r:r + rows] = np.log1p(-u).astype(np.float32)
    return W
