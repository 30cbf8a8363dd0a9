"""Pins for the oracle's random-draw contract.

* Philox4x32-10 is checked block by block against rocRAND's own
  host-callable Philox4x32-10 engine, compiled here and run as a black box
  (an implementation the oracle shares nothing with).
* The uniform and bounded-integer maps are checked against the properties
  that define them (exact grid, symmetry, Lemire-style thresholds).
* The keyed subset permutation is checked to be a bijection by brute force
  and its m-subsets for uniformity (first and second order).
"""
import itertools
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    out = tmp_path_factory.mktemp("rr") / "rocrand_philox_ref"
    src = os.path.join(ROOT, "tests", "helpers", "rocrand_philox_ref.cpp")
    subprocess.run([hipcc, "-O1", "-o", str(out), src], check=True, cwd=str(out.parent),
                   capture_output=True)
    return str(out)


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(1234)
    queries = []
    for _ in range(300):
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        ctr = [int(v) for v in rng.integers(0, 2**32, size=4, dtype=np.uint64)]
        ctr[1] &= 2**30 - 1   # rocRAND addresses a block by a 64-bit word offset 4*block
        queries.append((seed, ctr))
    # structured counters of the draw contract: tag<<24|block, index, iteration, run
    for tag in (1, 2, 3, 4):
        for blk in (0, 1, 5):
            queries.append((7, [(tag << 24) | blk, 33, 17, 0]))
    queries.append((0, [0, 0, 0, 0]))
    queries.append((2**64 - 1, [2**32 - 1, 2**30 - 1, 2**32 - 1, 2**32 - 1]))
    lines = []
    for seed, c in queries:
        block = c[0] | (c[1] << 32)
        subseq = c[2] | (c[3] << 32)
        lines.append(f"{seed} {subseq} {block}")
    res = subprocess.run([rocrand_ref], input="\n".join(lines) + "\n", capture_output=True,
                         text=True, check=True)
    ref = [list(map(int, l.split())) for l in res.stdout.strip().splitlines()]
    assert len(ref) == len(queries)
    for (seed, c), r in zip(queries, ref):
        key = [seed & 0xFFFFFFFF, seed >> 32]
        got = [int(v) for v in O.philox4x32_10(c, key)]
        assert got == r, (seed, c)


def test_uniform_grid_properties():
    ws = [0, 1, 255, 256, 2**31 - 1, 2**31, 2**32 - 257, 2**32 - 1, 0xDEADBEEF, 0x12345678]
    for w in ws:
        u = O.uniform(w)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u                    # exact in binary32
        assert O.uniform(w | 0x1FF) == u                    # only the top 23 bits count
        assert O.uniform((~w) & 0xFFFFFFFF) + u == 1.0      # symmetric about 1/2
    assert O.uniform(0) == 2.0 ** -24                       # first grid point
    for w in (0, 12345 << 9, (2**23 - 2) << 9):
        assert O.uniform(w + 512) - O.uniform(w) == 2.0 ** -23
    # the sign draw "u < 1/2" is exactly the top bit being clear
    assert O.uniform(0x7FFFFFFF) < 0.5 <= O.uniform(0x80000000)


@pytest.mark.parametrize("n", [1, 2, 3, 7, 10, 100, 1000, 4095, 4096, 65537, 2**31 - 1])
def test_bounded_thresholds(n):
    # value k is produced exactly by w in [ceil(k 2^32 / n), ceil((k+1) 2^32 / n))
    for k in sorted({0, min(1, n - 1), n // 2, n - 1}):
        lo = -(-(k << 32) // n)
        assert O.bounded(lo, n) == k
        if lo > 0:
            assert O.bounded(lo - 1, n) == k - 1
    assert O.bounded(2**32 - 1, n) == n - 1
    assert O.bounded(0, n) == 0


def _keys(*words):
    c = [int(w) & 0xFFFFFFFF for w in words] + [0] * (4 - len(words))
    return np.concatenate([O.philox4x32_10(c[:4], [99, 5]),
                           O.philox4x32_10([c[0] ^ 1] + c[1:4], [99, 5])])


@pytest.mark.parametrize("n", list(range(1, 70)) + [100, 127, 128, 129, 255, 256, 257, 1000, 4096])
def test_subset_pi_is_bijection(n):
    for trial in range(3):
        keys = _keys(n, trial, 3)
        ys = [O.subset_pi(x, n, keys) for x in range(n)]
        assert sorted(ys) == list(range(n))


def _select(kind, n, m, keys):
    """The m-subset of [0, n): the Dr form {x : pi(x) < m} or the mask form."""
    if kind == "dr":
        return [x for x in range(n) if O.subset_pi(x, n, keys) < m]
    return O.subset_mask(n, m, keys)


@pytest.mark.parametrize("kind", ["dr", "mask"])
@pytest.mark.parametrize("n,m", [(10, 3), (100, 25), (100, 80), (32, 4), (7, 3), (1000, 333),
                                 (3, 1)])
def test_subset_inclusion_uniform(kind, n, m):
    trials = 3000 if n <= 100 else 600
    cnt = np.zeros(n)
    for t in range(trials):
        keys = _keys(t, n, m)
        sel = _select(kind, n, m, keys)
        assert len(sel) == m
        cnt[sel] += 1
    # inclusion counts of a uniform m-subset: hypergeometric margins; the
    # chi-square statistic over n cells has mean (n-1)(1-m/n)
    e = trials * m / n
    chi = ((cnt - e) ** 2 / e).sum() / (1 - m / n)
    p = stats.chi2.sf(chi, n - 1)
    assert p > 1e-4, (chi, p)


@pytest.mark.parametrize("kind", ["dr", "mask"])
@pytest.mark.parametrize("n,m", [(4, 2), (5, 2), (6, 3), (8, 1), (7, 3), (9, 4)])
def test_subset_second_order_uniform(kind, n, m):
    subsets = {s: i for i, s in enumerate(itertools.combinations(range(n), m))}
    cnt = np.zeros(len(subsets))
    trials = 400 * len(subsets)
    for t in range(trials):
        keys = _keys(t, 7 * n + m)
        sel = tuple(_select(kind, n, m, keys))
        cnt[subsets[sel]] += 1
    p = stats.chisquare(cnt).pvalue
    assert p > 1e-4, (cnt, p)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 31, 64, 100, 129, 1000])
def test_mask_subsets_are_exact_and_nested(n):
    """A mask of size m has exactly m distinct members in [0, n); for fixed
    keys the masks grow one element at a time (the first m of one order),
    m = 0 selects nothing and m = n everything."""
    for trial in range(3):
        keys = _keys(n, trial, 11)
        prev = set()
        for m in range(n + 1):
            sel = O.subset_mask(n, m, keys)
            assert len(sel) == m and len(set(sel)) == m
            assert all(0 <= x < n for x in sel)
            assert prev <= set(sel)
            prev = set(sel)
        assert sorted(prev) == list(range(n))
