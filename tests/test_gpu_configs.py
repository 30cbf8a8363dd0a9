"""GPU parity against the oracle for configurations the product runs beyond
the single-handle cases of test_gpu_parity.py: rotated Rosenbrock in binary32
at the batched workload's shapes, members of a mixed batch (stepped through
the batch launches), a BF16 handle, and the rank sort on fitness values
with ties, signed zeros, infinities and NaN (both sort forms, both
precisions).  Every case prints its name before it touches the GPU."""
import numpy as np
import pytest

import gen
import oracle as O
from gpu_common import check_step, compare_step, make_pair, need_gpu, random_state

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim,pop", [(20, 64), (50, 256), (100, 64), (100, 256)])
def test_rotated_rosenbrock_fp32(dim, pop):
    """Rosenbrock couples neighbouring coordinates of z = M (y - o), so the
    tiled step takes the transformed coordinates through LDS (not the
    per-tile sums of the separable objectives)."""
    apo = need_gpu()
    print(f"[configs] rotated rosenbrock fp32 D={dim} ps={pop}", flush=True)
    g, p = make_pair(apo, dim=dim, pop=pop, kind="rosenbrock", rotated=True, precision="fp32",
                     max_iter=1000, seed=31, pf_max=0.1)
    with g:
        for t, sseed in ((1, 3), (700, 4)):
            X, F = random_state(p, sseed, "fp32")
            compare_step(g, p, t, X, F, "fp32")


def _member_specs():
    """A mixed batch: binary32 rotated runs whose batch shapes differ from
    the standalone ones (4 lanes and 128-row tiles at D 50, 8 lanes and
    64-row tiles at D 100), rotated Rosenbrock (its own lanes), a binary64
    rotated run at D 40 (the reduced tile does not fit in binary64: its own
    lanes), an elementwise binary64 run with three pairs and a Kapur run."""
    specs = []
    for dim, pop, kind, prec, npairs in ((50, 130, "rastrigin", "fp32", 1),
                                         (100, 64, "ackley", "fp32", 1),
                                         (20, 256, "rosenbrock", "fp32", 1),
                                         (100, 70, "rosenbrock", "fp32", 2),
                                         (40, 90, "sphere", "fp64", 1),
                                         (33, 50, "ackley", "fp64", 3)):
        specs.append(dict(dim=dim, pop=pop, kind=kind, precision=prec, np_pairs=npairs,
                          rotated=kind != "ackley" or prec == "fp32"))
    return specs


def test_batch_members_match_the_oracle():
    apo = need_gpu()
    print("[configs] batch members against the oracle", flush=True)
    T = 30
    runs, probs = [], []
    for i, sp in enumerate(_member_specs()):
        dt = np.float32 if sp["precision"] == "fp32" else np.float64
        dim = sp["dim"]
        o = gen.shift_vector(dim, 40 + i, dtype=dt)
        M = gen.rotation_matrix(dim, 40 + i, dtype=dt) if sp["rotated"] else None
        runs.append(dict(dim=dim, lb=-100.0, ub=100.0, pop=sp["pop"], np_pairs=sp["np_pairs"],
                         pf_max=0.3, seed=50 + i, max_iter=T, precision=sp["precision"],
                         kind=sp["kind"], shift=o, rot=M, run_id=i, trace=True))
        probs.append(O.Problem(dim=dim, pop=sp["pop"], lb=-100.0, ub=100.0,
                               np_pairs=sp["np_pairs"], max_iter=T, pf_max=0.3, seed=50 + i,
                               run_id=i, kind=sp["kind"], shift=o, rot=M))
    img = gen.blob_image(128, 128, seed=2)
    hist = gen.histogram_of(img)
    runs.append(dict(dim=4, lb=0.0, ub=255.0, pop=70, seed=5, max_iter=T, precision="fp32",
                     kind="kapur", hist=hist, run_id=9, trace=True, pf_max=0.3))
    probs.append(O.Problem(dim=4, pop=70, lb=0.0, ub=255.0, max_iter=T, pf_max=0.3, seed=5,
                           run_id=9, kind="kapur", hist=hist))
    with apo.Batch(runs) as b:
        for t in (1, 17):
            states = []
            for i, p in enumerate(probs):
                X, F = random_state(p, 100 * t + i, runs[i]["precision"])
                b[i].set_state(X, F, t - 1)
                states.append((X, F))
            assert b.run(1) == 1
            for i, p in enumerate(probs):
                print(f"[configs] batch member {i} ({runs[i]['kind']} D={p.dim}) t={t}",
                      flush=True)
                X, F = states[i]
                check_step(b[i], p, t, X, F, runs[i]["precision"])


def test_bf16_handle_step_matches_the_oracle():
    """A BF16 handle stores the binary32 form's candidates and binary32
    fitness for every candidate it re-scores; the rejections its estimate
    settles must be rejections for the oracle too.  Sphere at D 520 (the
    GEMM form), where the bound settles part of the comparisons."""
    apo = need_gpu()
    print("[configs] bf16 handle, sphere D=520 ps=300", flush=True)
    g, p = make_pair(apo, dim=520, pop=300, kind="sphere", rotated=True, precision="bf16",
                     max_iter=100, seed=12, pf_max=0.2)
    with g:
        for t, sseed in ((1, 5), (60, 6)):
            X, F = random_state(p, sseed, "fp32")
            compare_step(g, p, t, X, F, "fp32", bf16=True)
        resc, _ = g.precision_stats()
        print(f"[configs] bf16 re-scored {resc} of {2 * p.pop}", flush=True)
        assert 0 < resc <= 2 * p.pop


SPECIAL = np.array([np.nan, -0.0, 0.0, 1.5, -np.inf, 1.5, np.inf, np.nan, -2.0, 1.5, 0.0, -0.0])


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("pop", [40, 300])
def test_rank_sort_special_values(precision, pop):
    """The sort: ascending, -0 equal to +0, NaN after +inf, ties by id.  pop
    40 runs the LDS form of the sort kernel, pop 300 the register form."""
    apo = need_gpu()
    print(f"[configs] rank sort special values {precision} ps={pop}", flush=True)
    g, p = make_pair(apo, dim=6, pop=pop, kind="sphere", precision=precision, max_iter=20,
                     seed=9, pf_max=0.5)
    rng = np.random.default_rng(pop)
    with g:
        X, _ = random_state(p, 2, precision)
        F = rng.choice(SPECIAL, size=pop)
        F[: len(SPECIAL)] = SPECIAL
        g.set_state(X, F, 4)
        assert g.step()
        _, _, opg, permg = g.get_trace()
        want = O.rank_order(F)
        assert np.array_equal(permg, want), (permg[:20], want[:20])
        _, _, tr = p.step(5, X, F)
        assert np.array_equal(opg, tr.op)
