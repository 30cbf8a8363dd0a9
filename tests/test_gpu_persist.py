"""The persistent form of apo_run (APO_FLAG_PERSISTENT: every iteration of
a tiled run in one cooperative launch, sort and step separated by grid
barriers) against the graph-replayed two-kernel form: bit-identical states
after whole runs, after runs split into pieces, and after injected states;
the persistent form is engaged where the grid fits the device (timing
reports no separate sort kernel).  The two-kernel form is the one the
parity tests compare with the oracle step by step."""
import numpy as np
import pytest

from gpu_common import make_pair, need_gpu, random_state

pytestmark = pytest.mark.gpu

CASES = [
    ("c2_shape_fp32", dict(dim=100, pop=4096, kind="rastrigin", rotated=True, precision="fp32"), 60),
    ("rotated_fp64_small", dict(dim=20, pop=70, kind="rastrigin", rotated=True), 40),
    ("rosenbrock_np2_fp32", dict(dim=50, pop=256, kind="rosenbrock", rotated=True,
                                 precision="fp32", np_pairs=2), 30),
    ("ackley_ragged_fp32", dict(dim=37, pop=1000, kind="ackley", rotated=True,
                                precision="fp32", pf_max=0.5), 25),
]


def _pair(apo, seed, T, persistent, kw):
    g, p = make_pair(apo, max_iter=T, seed=seed, trace=False, **kw)
    if persistent:
        g.close()
        g = apo.APO(p.dim, p.lb, p.ub, p.pop, np_pairs=p.np_pairs, pf_max=p.pf_max, seed=seed,
                    max_iter=T, precision=kw.get("precision", "fp64"), kind=p.kind, shift=p.shift,
                    rot=p.rot, persistent=True)
    return g, p


@pytest.mark.parametrize("name,kw,T", CASES, ids=[c[0] for c in CASES])
def test_persistent_equals_graph_form(name, kw, T):
    apo = need_gpu()
    print(f"[persist] {name} T={T}", flush=True)
    a, p = _pair(apo, 17, T, True, kw)
    b, _ = _pair(apo, 17, T, False, kw)
    c, _ = _pair(apo, 17, T, True, kw)
    with a, b, c:
        assert a.run(T) == T
        assert b.run(T) == T
        for n in (7, 13, 1000):          # split into pieces: t0 handling
            c.run(n)
        sa, sb, sc = a.get_state(), b.get_state(), c.get_state()
        assert sa[2] == sb[2] == sc[2] == T
        assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1])
        assert np.array_equal(sa[0], sc[0]) and np.array_equal(sa[1], sc[1])
        assert a.best()[1] == b.best()[1]
        assert a.run(5) == 0


def test_persistent_form_is_engaged_and_resumes_injected_state():
    apo = need_gpu()
    print("[persist] engaged at the single-run shape; injected state", flush=True)
    kw = dict(dim=100, pop=4096, kind="rastrigin", rotated=True, precision="fp32")
    a, p = _pair(apo, 5, 100, True, kw)
    b, _ = _pair(apo, 5, 100, False, kw)
    with a, b:
        X, F = random_state(p, 3, "fp32")
        for g in (a, b):
            g.set_state(X, F, 40)
        na, ta = a.time_kernels(10)
        nb, tb = b.time_kernels(10)
        print(f"[persist] per-iteration us: persistent {ta}, graph form {tb}", flush=True)
        assert na == nb == 10
        assert ta["rank_us"] == 0.0 and ta["step_us"] > 0.0
        assert tb["rank_us"] > 0.0
        assert a.run(20) == b.run(20) == 20
        sa, sb = a.get_state(), b.get_state()
        assert sa[2] == sb[2] == 70
        assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1])
