"""The HIP library's device primitives, compiled for the host with stand-ins
that keep HIP's signatures, against the oracle: the subset permutation (a
bijection whose cycle walk ends, equal to the oracle's for every element),
Philox, and the fitness-order keys.  Regression guard for a signed shift of
__umul24's int result, which made the walk leave [0, 2^b) and never end."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    cxx = shutil.which("g++")
    if not cxx:
        pytest.skip("no host C++ compiler")
    out = tmp_path_factory.mktemp("dev") / "device_primitives_host"
    subprocess.run([cxx, "-O1", "-std=c++17", "-I",
                    os.path.join(ROOT, "paper_2510_14982_amd", "csrc"), "-o", str(out),
                    os.path.join(ROOT, "tests", "helpers", "device_primitives_host.cpp")],
                   check=True, capture_output=True)
    return str(out)


def _run(exe, mode, lines):
    r = subprocess.run([exe, mode], input="\n".join(lines) + "\n", capture_output=True,
                       text=True, check=True, timeout=120)
    return r.stdout.split("\n")


def test_subset_pi_matches_oracle_for_every_element(harness):
    rng = np.random.default_rng(7)
    lines, want = [], []
    for n in list(range(1, 300)) + [511, 512, 513, 1000, 1024, 4096, 65536]:
        keys = rng.integers(0, 2**32, size=8, dtype=np.uint64)
        xs = range(n) if n <= 1024 else rng.integers(0, n, size=300)
        for x in xs:
            lines.append(f"{n} {int(x)} " + " ".join(str(int(k)) for k in keys))
            want.append(O.subset_pi(int(x), n, keys))
    got = [int(v) for v in _run(harness, "pi", lines) if v]
    assert got == want


def test_mask_builder_equals_oracle_mask(harness):
    """The GPU builds each coordinate mask by scanning the pass order (from
    the end, clearing, when m > n / 2); the set must be exactly the
    oracle's mask subset, for every domain width and both scan directions
    (one lane here; the GPU parity tests cover the ballot across lanes)."""
    rng = np.random.default_rng(9)
    lines, want = [], []
    for n in list(range(1, 140)) + [255, 256, 1000, 1024]:
        for m in sorted({0, 1, n // 3, n // 2, (n + 1) // 2, n - 1, n} - {-1}):
            if m < 0:
                continue
            keys = rng.integers(0, 2**32, size=8, dtype=np.uint64)
            lines.append(f"{n} {m} " + " ".join(str(int(k)) for k in keys))
            want.append(O.subset_mask(n, m, keys))
    got = [[int(v) for v in l.split()] for l in _run(harness, "mask", lines)[:len(lines)]]
    assert got == want


def test_philox_matches_oracle(harness):
    rng = np.random.default_rng(8)
    q = rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64)
    got = [list(map(int, l.split())) for l in _run(harness, "philox",
                                                    [" ".join(map(str, r)) for r in q]) if l]
    for r, g in zip(q, got):
        assert g == [int(v) for v in O.philox4x32_10(r[:4], r[4:])]


def test_order_key_is_the_oracle_sort_order(harness):
    vals = [-np.inf, -3.5, -1e-30, -0.0, 0.0, 1e-30, 2.0, np.inf, np.nan, -np.nan]
    bits = [struct.unpack("<I", struct.pack("<f", v))[0] for v in vals]
    keys = [int(v) for v in _run(harness, "key32", [f"{b:08x}" for b in bits]) if v]
    F = np.array(vals, dtype=np.float64)
    order = np.lexsort((np.arange(len(keys)), np.array(keys)))
    assert np.array_equal(order, O.rank_order(F))

