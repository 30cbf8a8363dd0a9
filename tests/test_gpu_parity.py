"""GPU parity: the HIP path against the oracle, element by element, from
identical injected state, through the C ABI (every case prints its name
before it touches the GPU)."""
import numpy as np
import pytest

import gen
import oracle as O
from gpu_common import compare_step, make_pair, need_gpu, random_state

pytestmark = pytest.mark.gpu

STEP_CASES = [
    # name, kwargs, iteration t, max_iter
    ("c1_shape_rastrigin_fp64", dict(dim=10, pop=32, kind="rastrigin"), 1, 200),
    ("worked_example_shape_sphere", dict(dim=3, pop=4, kind="sphere", lb=0.0, ub=10.0), 1, 50),
    ("ragged_rosenbrock_np2", dict(dim=37, pop=50, kind="rosenbrock", np_pairs=2), 7, 40),
    ("ackley_g64", dict(dim=130, pop=64, kind="ackley", pf_max=0.5), 3, 30),
    ("rastrigin_two_chunks", dict(dim=300, pop=40, kind="rastrigin", pf_max=1.0), 2, 10),
    ("sphere_four_chunks_np3", dict(dim=1000, pop=24, kind="sphere", np_pairs=3), 5, 9),
    ("last_iteration", dict(dim=16, pop=33, kind="rastrigin", pf_max=0.3), 20, 20),
    ("no_dr", dict(dim=8, pop=17, kind="sphere", pf_max=0.0), 4, 10),
    ("all_dr", dict(dim=8, pop=17, kind="sphere", pf_max=1.0), 4, 10),
    ("pop2_dim1", dict(dim=1, pop=2, kind="rastrigin"), 1, 3),
    # Eq. (13) with the opposite sign (a variant of the printed formula)
    ("pdr_plus_variant", dict(dim=12, pop=40, kind="rastrigin", pf_max=1.0, pdr_plus=True), 3, 10),
    ("rotated_rastrigin_fp64", dict(dim=20, pop=70, kind="rastrigin", rotated=True), 3, 50),
    ("rotated_rosenbrock_np3_fp64", dict(dim=33, pop=40, kind="rosenbrock", rotated=True,
                                         np_pairs=3), 2, 20),
    ("elem_rastrigin_fp32", dict(dim=100, pop=300, kind="rastrigin", precision="fp32"), 5, 100),
    ("rotated_rastrigin_fp32", dict(dim=100, pop=300, kind="rastrigin", rotated=True,
                                    precision="fp32"), 5, 100),
    ("rotated_ackley_fp32", dict(dim=50, pop=100, kind="ackley", rotated=True,
                                 precision="fp32", pf_max=0.4), 9, 20),
    ("rotated_sphere_fp32_d200", dict(dim=200, pop=48, kind="sphere", rotated=True,
                                      precision="fp32"), 2, 10),
    # full benchmark size and launch configuration (ps 4096, D 100, FP32, rotated)
    ("c2_full_size_first", dict(dim=100, pop=4096, kind="rastrigin", rotated=True,
                                precision="fp32"), 1, 1000),
    ("c2_full_size_late", dict(dim=100, pop=4096, kind="rastrigin", rotated=True,
                               precision="fp32"), 640, 1000),
    # the GEMM form at its smallest: just above the dimension threshold, a
    # handful of protozoa (one partial row tile, ragged K and N padding)
    ("gemm_form_d513_pop5", dict(dim=513, pop=5, kind="rastrigin", rotated=True,
                                 precision="fp32", pf_max=0.5), 2, 10),
    ("gemm_form_d700_pop2_ackley", dict(dim=700, pop=2, kind="ackley", rotated=True,
                                        precision="fp32"), 1, 5),
    # the precision configuration's shape in binary32: the GEMM form as bench.py times it
    ("c5_full_size_fp32_gemm", dict(dim=1000, pop=8192, kind="ackley", rotated=True,
                                    precision="fp32"), 1, 2000),
    # many rank-sort splits with a ragged last block
    ("large_pop_ragged_fp64", dict(dim=10, pop=5000, kind="rastrigin"), 3, 10),
    ("large_pop_fp32_d3", dict(dim=3, pop=8192, kind="sphere", precision="fp32",
                               pf_max=0.3), 2, 10),
]


@pytest.mark.parametrize("name,kw,t,T", STEP_CASES, ids=[c[0] for c in STEP_CASES])
def test_step_parity(name, kw, t, T):
    apo = need_gpu()
    print(f"[parity] {name} t={t} T={T} {kw}", flush=True)
    prec = kw.get("precision", "fp64")
    g, p = make_pair(apo, max_iter=T, seed=11, **kw)
    with g:
        for rep, sseed in enumerate((3, 4)):
            X, F = random_state(p, sseed, prec)
            compare_step(g, p, t, X, F, prec)


@pytest.mark.parametrize("k", [1, 4, 8, 16])
@pytest.mark.parametrize("kind", ["kapur", "otsu"])
def test_threshold_step_parity(kind, k):
    apo = need_gpu()
    print(f"[parity] {kind} k={k}", flush=True)
    img = gen.blob_image(256, 256, seed=5)
    hist = gen.histogram_of(img)
    g, p = make_pair(apo, dim=k, pop=130, kind=kind, precision="fp32", lb=0.0, ub=255.0,
                     hist=hist, max_iter=50, seed=2)
    with g:
        X, F = random_state(p, 9, "fp32")
        compare_step(g, p, 4, X, F, "fp32")


def test_kapur_full_size_config():
    """Thresholding configuration: ps 1024, k = 16, 500 iterations."""
    apo = need_gpu()
    print("[parity] kapur ps1024 k16", flush=True)
    img = gen.blob_image(1024, 1024, seed=1)
    hist = gen.histogram_of(img)
    g, p = make_pair(apo, dim=16, pop=1024, kind="kapur", precision="fp32", lb=0.0, ub=255.0,
                     hist=hist, max_iter=500, seed=3)
    with g:
        for t in (1, 250, 500):
            X, F = random_state(p, t, "fp32")
            compare_step(g, p, t, X, F, "fp32")


@pytest.mark.parametrize("precision,rotated,dim", [("fp64", False, 10), ("fp64", True, 24),
                                                   ("fp32", False, 100), ("fp32", True, 100)])
def test_initial_population(precision, rotated, dim):
    apo = need_gpu()
    print(f"[init] {precision} rotated={rotated} dim={dim}", flush=True)
    g, p = make_pair(apo, dim=dim, pop=77, kind="rastrigin", precision=precision,
                     rotated=rotated, max_iter=5, seed=21)
    with g:
        X, F, t = g.get_state()
        Xo, Fo = p.init()
        assert t == 0
        if precision == "fp64":
            assert np.array_equal(X, Xo)
            assert np.allclose(F, Fo, rtol=1e-12, atol=0)
        else:
            assert np.allclose(X, Xo, rtol=1e-6, atol=1e-5)
            assert np.allclose(F, Fo, rtol=1e-5, atol=1e-4)


def test_c1_full_run_matches_oracle():
    """ps 32, D 10, 200 FP64 iterations of shifted Rastrigin from the GPU's
    own initialisation: the whole trajectory is reproduced (no near ties
    occur on this seed), checked every 25 iterations."""
    apo = need_gpu()
    print("[run] c1 full trajectory", flush=True)
    w = gen.shifted_rastrigin_small(seed=1)
    with apo.APO(w.dim, w.lb, w.ub, w.pop, seed=w.seed, max_iter=w.max_iter, precision="fp64",
                 kind=w.kind, shift=w.shift) as g:
        p = O.Problem(dim=w.dim, pop=w.pop, lb=w.lb, ub=w.ub, max_iter=w.max_iter, seed=w.seed,
                      kind=w.kind, shift=w.shift)
        Xo, Fo = p.init()
        t = 0
        while t < w.max_iter:
            n = g.run(25)
            Xo, Fo, t2 = p.run(Xo, Fo, t, n)
            t += n
            X, F, tg = g.get_state()
            assert tg == t == t2
            assert np.allclose(X, Xo, rtol=1e-9, atol=1e-9), t
            assert np.allclose(F, Fo, rtol=1e-9, atol=1e-9), t
        xb, fb, fes = g.best()
        assert fes == w.pop * (w.max_iter + 1)
        b = O.best(Fo)
        assert abs(fb - Fo[b]) <= 1e-9 * max(1.0, abs(Fo[b]))


def test_otsu_single_threshold_run_matches_oracle():
    """The thresholding application in the paper's table shape: one Otsu
    threshold, ps 100, D 1, 50 binary64 iterations from the GPU's own
    initialisation, on a 512 x 512 synthetic image.  Thresholds (rint of
    the coordinate) agree exactly at every checkpoint and the fitness to
    the prefix-table rounding; the final best threshold is the oracle's."""
    apo = need_gpu()
    import torch
    print("[run] otsu ps100 D1 T50 fp64", flush=True)
    w = gen.otsu_single(side=512, seed=4)
    img = torch.from_numpy(w.extra["image"]).cuda().reshape(-1)
    h = apo.histogram_u8(img)
    assert np.array_equal(h, w.hist)
    with apo.APO(w.dim, w.lb, w.ub, w.pop, seed=w.seed, max_iter=w.max_iter, precision="fp64",
                 kind=w.kind, hist=h) as g:
        p = O.Problem(dim=w.dim, pop=w.pop, lb=w.lb, ub=w.ub, max_iter=w.max_iter, seed=w.seed,
                      kind=w.kind, hist=w.hist)
        Xo, Fo = p.init()
        t = 0
        while t < w.max_iter:
            n = g.run(10)
            Xo, Fo, t2 = p.run(Xo, Fo, t, n)
            t += n
            X, F, tg = g.get_state()
            assert tg == t == t2
            assert np.array_equal(np.rint(X), np.rint(Xo)), t
            assert np.allclose(F, Fo, rtol=1e-9, atol=1e-12), t
        xb, fb, _ = g.best()
        b = O.best(Fo)
        assert np.rint(xb[0]) == np.rint(Xo[b][0])
        assert abs(fb - Fo[b]) <= 1e-9 * max(1.0, abs(Fo[b]))


def test_graph_replay_equals_single_steps_and_is_deterministic():
    apo = need_gpu()
    print("[run] graph replay vs steps", flush=True)
    kw = dict(dim=100, pop=500, kind="rastrigin", rotated=True, precision="fp32", max_iter=40)
    g1, _ = make_pair(apo, seed=5, **kw)
    g2, _ = make_pair(apo, seed=5, **kw)
    g3, _ = make_pair(apo, seed=5, **kw)
    with g1, g2, g3:
        assert g1.run(40) == 40
        for _ in range(40):
            assert g2.step()
        assert not g2.step()
        g3.run(13)
        g3.run(100)
        a, b, c = g1.get_state(), g2.get_state(), g3.get_state()
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
        assert a[2] == b[2] == c[2] == 40


_OTSU_HIST = gen.histogram_of(gen.blob_image(128, 128, seed=6))


@pytest.mark.parametrize("kw", [
    dict(dim=10, pop=32, kind="rastrigin", precision="fp64", max_iter=60),
    dict(dim=16, pop=64, kind="rosenbrock", precision="fp32", max_iter=40, pf_max=0.5),
    dict(dim=10, pop=50, kind="sphere", precision="fp64", max_iter=30, np_pairs=3),
    dict(dim=3, pop=4, kind="ackley", precision="fp32", max_iter=25, pf_max=1.0),
    # one protozoan a wavefront; the LDS image above 64 KiB (D 1000, binary64)
    dict(dim=1000, pop=4, kind="sphere", precision="fp64", max_iter=12),
    dict(dim=200, pop=4, kind="rastrigin", precision="fp32", max_iter=20, pf_max=0.5),
    # tiled runs one wide tile holds
    dict(dim=1, pop=100, kind="otsu", precision="fp64", max_iter=50, lb=0.0, ub=255.0,
         hist=_OTSU_HIST),
    dict(dim=4, pop=128, kind="kapur", precision="fp32", max_iter=20, lb=0.0, ub=255.0,
         hist=_OTSU_HIST, pf_max=0.5),
    dict(dim=12, pop=90, kind="rastrigin", rotated=True, precision="fp32", max_iter=30),
    dict(dim=10, pop=40, kind="rosenbrock", rotated=True, precision="fp64", max_iter=20,
         np_pairs=2),
], ids=["c1_fp64", "rosenbrock_fp32_full_wg", "sphere_np3", "tiny_all_dr", "d1000_lds_64k_plus",
        "d200_one_wave_each", "otsu_table_shape",
        "kapur_k4_full_tile", "rotated_rastrigin_fp32", "rotated_rosenbrock_fp64_np2"])
def test_persistent_run_equals_single_steps(kw):
    """Runs whose whole population fits one workgroup take the persistent
    form in apo_run (one launch for all iterations); the state after it is
    the two-kernel iteration's bit for bit, whatever the chunking of the
    calls, and every iteration count and the best agree."""
    apo = need_gpu()
    print(f"[run] persistent form vs single steps {kw}", flush=True)
    T = kw["max_iter"]
    g1, _ = make_pair(apo, seed=9, **kw)
    g2, _ = make_pair(apo, seed=9, **kw)
    g3, _ = make_pair(apo, seed=9, **kw)
    with g1, g2, g3:
        assert g1.run(T + 5) == T
        for _ in range(T):
            assert g2.step()
        assert g3.run(7) == 7 and g3.run(1) == 1 and g3.run(T) == T - 8
        a, b, c = g1.get_state(), g2.get_state(), g3.get_state()
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
        assert a[2] == b[2] == c[2] == T
        # the last iteration's trace (candidates, their fitness, operations, order)
        for u, v in zip(g1.get_trace(), g2.get_trace()):
            assert np.array_equal(u, v)
        assert g1.run(3) == 0
        x1, f1, e1 = g1.best()
        x2, f2, e2 = g2.best()
        assert np.array_equal(x1, x2) and f1 == f2 and e1 == e2 == kw["pop"] * (T + 1)


def test_checkpoint_resume_bit_identical():
    apo = need_gpu()
    print("[run] checkpoint resume", flush=True)
    kw = dict(dim=30, pop=64, kind="ackley", precision="fp32", max_iter=30)
    g1, _ = make_pair(apo, seed=8, **kw)
    g2, _ = make_pair(apo, seed=8, **kw)
    with g1, g2:
        g1.run(30)
        g2.run(11)
        X, F, t = g2.get_state()
        g2.set_state(X, F, t)
        g2.run(30)
        assert np.array_equal(g1.get_state()[0], g2.get_state()[0])
        assert np.array_equal(g1.get_state()[1], g2.get_state()[1])


def test_best_order_ties_and_nan():
    apo = need_gpu()
    print("[best] ties and NaN", flush=True)
    g, p = make_pair(apo, dim=5, pop=9, kind="sphere", max_iter=3)
    with g:
        X = gen.random_state(9, 5, p.lb, p.ub, 1)
        F = np.array([3.0, np.nan, 1.0, -0.0, 0.0, 1.0, np.nan, 7.0, 0.0])
        g.set_state(X, F, 0)
        x, f, fes = g.best()
        assert f == 0.0 and np.array_equal(x, X[3])        # -0 == +0, lowest id
        F2 = np.full(9, np.nan)
        F2[6] = 5.0
        g.set_state(X, F2, 1)
        x, f, fes = g.best()
        assert f == 5.0 and np.array_equal(x, X[6]) and fes == 9 * 2


def test_bounds_monotone_best_and_done():
    apo = need_gpu()
    print("[run] invariants", flush=True)
    g, p = make_pair(apo, dim=64, pop=256, kind="rastrigin", rotated=True, precision="fp32",
                     max_iter=60, pf_max=0.5)
    with g:
        last = np.inf
        for k in range(6):
            g.run(10)
            X, F, t = g.get_state()
            assert np.all(X >= p.lb) and np.all(X <= p.ub)
            assert F.min() <= last
            last = F.min()
        assert not g.step()
        assert g.run(5) == 0


@pytest.mark.parametrize("n", [0, 1, 15, 16, 17, 4096 * 3 + 5])
@pytest.mark.parametrize("offset", [0, 3])
def test_histogram_bit_exact(n, offset):
    apo = need_gpu()
    import torch
    print(f"[hist] n={n} offset={offset}", flush=True)
    rng = np.random.default_rng(n + offset)
    host = rng.integers(0, 256, size=n + offset, dtype=np.uint8)
    dev = torch.from_numpy(host).cuda()
    h = apo.histogram_u8(dev[offset:]).astype(np.int64)
    assert np.array_equal(h, np.bincount(host[offset:], minlength=256))


def test_histogram_blob_image_full_size():
    apo = need_gpu()
    import torch
    print("[hist] blob 4096x4096", flush=True)
    img = gen.blob_image(4096, 4096, seed=1)
    h = apo.histogram_u8(torch.from_numpy(img).cuda().reshape(-1))
    assert np.array_equal(h.astype(np.int64), np.bincount(img.reshape(-1), minlength=256))
    for const in (0, 255):
        im = torch.full((1 << 20,), const, dtype=torch.uint8, device="cuda")
        hc = apo.histogram_u8(im)
        assert hc[const] == 1 << 20 and hc.sum() == 1 << 20
