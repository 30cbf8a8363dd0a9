"""Final best-fitness distributions over 30 seeds: GPU against the oracle,
each from its own initialisation (same Philox stream).  Whole trajectories
are parity-unpinned value by value (a near-tie selection flip makes them
diverge), so they are compared as distributions: two-sided Mann-Whitney U
with p > 0.01 and medians within 10 %.  The binary64 small run is expected
to reproduce the oracle seed by seed."""
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


def _compare(gpu, ora):
    gpu, ora = np.asarray(gpu), np.asarray(ora)
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
    _compare(gpu, ora)


def test_kapur_run_30_seeds():
    apo = need_gpu()
    print("[seeds] Kapur k=4 ps256, 60 iterations", flush=True)
    img = gen.blob_image(512, 512, seed=3)
    gpu, ora = [], []
    for s in SEEDS:
        w = gen.kapur_thresholds(k=4, seed=s, pop=256, max_iter=60, img=img)
        gpu.append(_gpu_best(apo, w, "fp32", s))
        ora.append(_oracle_best(w, s))
    _compare(gpu, ora)
