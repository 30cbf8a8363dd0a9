"""Final best-fitness distributions over 30 seeds: GPU against the oracle,
each from its own initialisation (same Philox stream).  Whole trajectories
are parity-unpinned value by value (a near-tie selection flip makes them
diverge), so they are compared as distributions: two-sided Mann-Whitney U
with p > 0.01 and medians within 10 %.  The binary64 small run is expected
to reproduce the oracle seed by seed."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
from scipy import stats

import gen
import oracle as O
from gpu_common import need_gpu

pytestmark = pytest.mark.gpu
SEEDS = range(1, 31)


def _gpu_best(apo, w, precision, seed):
    with apo.APO(w.dim, w.lb, w.ub, w.pop, np_pairs=w.np_pairs, pf_max=w.pf_max, seed=seed,
                 max_iter=w.max_iter, precision=precision, kind=w.kind, shift=w.shift,
                 rot=w.rot, hist=w.hist) as g:
        g.run()
        return g.best()[1]


def _oracle_best(w, seed):
    p = O.Problem(dim=w.dim, pop=w.pop, lb=w.lb, ub=w.ub, np_pairs=w.np_pairs,
                  max_iter=w.max_iter, pf_max=w.pf_max, seed=seed, kind=w.kind, shift=w.shift,
                  rot=w.rot, hist=w.hist)
    return p.solve()[1]


def _host_threads():
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def _oracle_bests_parallel(make, seeds, tag):
    """The oracle's final best for every seed, the seeds spread over the
    host's threads (each a single-threaded oracle run; ctypes releases the
    interpreter lock during the oracle's calls)."""
    def one(s):
        O.set_threads(1)
        v = _oracle_best(make(s), s)
        print(f"[seeds] {tag} oracle seed {s}: {v:.6g}", flush=True)
        return v
    with ThreadPoolExecutor(max_workers=_host_threads()) as ex:
        return list(ex.map(one, seeds))


def _compare(gpu, ora, dtype=np.float64):
    """Distributions of final bests.  A binary32 run stores its fitness in
    binary32, so the oracle's binary64 values are rounded to binary32 first
    (runs that reach the same optimum then give equal values, rather than
    values one binary32 rounding apart)."""
    gpu, ora = np.asarray(gpu), np.asarray(ora, dtype=np.float64).astype(dtype)
    p = stats.mannwhitneyu(gpu, ora, alternative="two-sided").pvalue
    mg, mo = np.median(gpu), np.median(ora)
    assert p > 0.01, (p, mg, mo)
    assert abs(mg - mo) <= 0.10 * max(abs(mo), 1e-12), (mg, mo)
    return p


def test_small_fp64_run_30_seeds():
    apo = need_gpu()
    print("[seeds] ps32 D10 FP64 shifted Rastrigin, 200 iterations", flush=True)
    gpu, ora = [], []
    for s in SEEDS:
        w = gen.shifted_rastrigin_small(seed=s)
        gpu.append(_gpu_best(apo, w, "fp64", s))
        ora.append(_oracle_best(w, s))
    _compare(gpu, ora)
    same = np.isclose(gpu, ora, rtol=1e-9, atol=1e-9)
    assert same.mean() >= 0.9, np.c_[gpu, ora][~same]


def test_rotated_fp32_run_30_seeds():
    """Rotated Rastrigin FP32 at a reduced size (ps 256, D 20, 100
    iterations) so the oracle's 30 runs take seconds."""
    apo = need_gpu()
    print("[seeds] ps256 D20 FP32 rotated Rastrigin, 100 iterations", flush=True)
    gpu, ora = [], []
    for s in SEEDS:
        w = gen.rotated_rastrigin_large(seed=s, pop=256, dim=20, max_iter=100)
        gpu.append(_gpu_best(apo, w, "fp32", s))
        ora.append(_oracle_best(w, s))
    _compare(gpu, ora, np.float32)


def test_kapur_run_30_seeds():
    apo = need_gpu()
    print("[seeds] Kapur k=4 ps256, 60 iterations", flush=True)
    img = gen.blob_image(512, 512, seed=3)
    gpu, ora = [], []
    for s in SEEDS:
        w = gen.kapur_thresholds(k=4, seed=s, pop=256, max_iter=60, img=img)
        gpu.append(_gpu_best(apo, w, "fp32", s))
        ora.append(_oracle_best(w, s))
    _compare(gpu, ora, np.float32)


def test_rotated_fp32_full_size_30_seeds(golden_dir):
    """The single large run at its full size: ps 4096, D 100, 1000
    iterations of shifted-rotated Rastrigin in binary32 on the GPU against
    the binary64 oracle, 30 seeds each.  The oracle's 30 runs (about half
    an hour of CPU time) are read from the file tests/golden/make_seed_bests.py
    writes with the oracle alone."""
    apo = need_gpu()
    import json
    print("[seeds] ps4096 D100 FP32 rotated Rastrigin, 1000 iterations", flush=True)
    with open(os.path.join(golden_dir, "seed_bests_rotated_rastrigin_ps4096_d100.json")) as f:
        doc = json.load(f)
    assert doc["seeds"] == list(SEEDS)
    gpu = [_gpu_best(apo, gen.rotated_rastrigin_large(seed=s), "fp32", s) for s in SEEDS]
    print(f"[seeds] gpu bests {np.round(gpu, 2).tolist()}", flush=True)
    _compare(gpu, doc["best_f"], np.float32)


@pytest.mark.parametrize("k", [4, 8, 16])
def test_kapur_full_size_30_seeds(k):
    """The thresholding configuration at its full size: Kapur over k
    thresholds of a 4096 x 4096 blob image, ps 1024, 500 iterations."""
    apo = need_gpu()
    print(f"[seeds] Kapur k={k} ps1024 T500 4096x4096 image", flush=True)
    img = gen.blob_image(4096, 4096, seed=1)

    def make(s):
        return gen.kapur_thresholds(k=k, seed=s, img=img)
    gpu = [_gpu_best(apo, make(s), "fp32", s) for s in SEEDS]
    ora = _oracle_bests_parallel(make, SEEDS, f"kapur{k}")
    _compare(gpu, ora, np.float32)
