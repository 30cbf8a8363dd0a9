"""Launch shapes of the step kernels, checked on the CPU against the header
the library itself uses (apo_shape.hpp): every lane count a policy can give
(4, 8, 16, 32, 64 lanes per protozoan, 16-row or wide tiles, binary32 and
binary64, every dimension up to 1024) either maps to a compiled kernel whose
LDS fits one workgroup, or is refused at creation; the shape key that groups
batched launches encodes each field without overlap; and the library's own
policies (single runs and batch members) only ever produce launchable
shapes.  Regression guard: a batch lane policy that produced (8 lanes,
2 chunks, 64 rows), a shape with no kernel, failed only at the first
launch, in the middle of a graph capture."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_14982_amd", "csrc")


@pytest.fixture(scope="module")
def table(tmp_path_factory):
    cxx = shutil.which("g++")
    if not cxx:
        pytest.skip("no host C++ compiler")
    exe = tmp_path_factory.mktemp("shape") / "shape_host"
    subprocess.run([cxx, "-O1", "-std=c++17", "-Wall", "-Werror", "-I", CSRC, "-o", str(exe),
                    os.path.join(ROOT, "tests", "helpers", "shape_host.cpp")],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    lines = out.splitlines()
    shapes = np.array([[int(v) for v in ln.split()[1:]] for ln in lines if ln.startswith("S ")])
    policy = np.array([[int(v) for v in ln.split()[1:]] for ln in lines if ln.startswith("P ")])
    image = np.array([[int(v) for v in ln.split()[1:]] for ln in lines if ln.startswith("I ")])
    return shapes, policy, image


def test_shape_key_round_trips(table):
    table = table[0]
    ok = table[:, 3] > 0
    t = table[ok]
    assert np.all(t[:, 7] >= 0)
    assert np.array_equal(t[:, 8], t[:, 2]) and np.array_equal(t[:, 9], t[:, 3])
    assert np.array_equal(t[:, 10], t[:, 4])


def test_built_shapes_fit_where_the_library_uses_them(table):
    table = table[0]
    es, dim, G, NCH, TM, built, fits = (table[:, i] for i in range(7))
    # a shape that fits is a compiled shape
    assert np.all(built[fits == 1] == 1)
    # single runs: the dimension's own lanes, 16-row or wide tiles, up to the
    # documented limits (512 in binary32, 256 in binary64)
    own = np.array([G[i] == _lanes_for_dim(dim[i]) for i in range(len(G))])
    lim = np.where(es == 8, 256, 512)
    single = own & (dim <= lim)
    assert np.all(fits[single] == 1), table[single & (fits == 0)][:5]


def test_batch_policy_shapes_fit(table):
    """The batch policy's shape for every dimension the tiled form takes
    (512 in binary32, 256 in binary64) is launchable; it is the documented
    reduced lane count (4 lanes for 17-64 dimensions, 8 for 65-128, wide
    tiles) for separable objectives in binary32, and falls back to the
    dimension's own lanes where the reduced tile does not fit (binary64
    above 32 dimensions) and for Rosenbrock."""
    es, dim, ros, G, NCH, TM, fits = (table[1][:, i] for i in range(7))
    inside = np.where(es == 8, dim <= 256, dim <= 512)
    assert np.all(fits[inside] == 1), table[1][inside & (fits == 0)][:5]
    assert np.array_equal(TM, np.maximum(16, 512 // G))
    own = np.array([_lanes_for_dim(d) for d in dim])
    reduced = np.where((dim > 16) & (dim <= 64), 4, np.where((dim > 64) & (dim <= 128), 8, own))
    sel = (es == 4) & (ros == 0)
    assert np.array_equal(G[sel], reduced[sel])
    assert np.array_equal(G[ros == 1], own[ros == 1])
    sel64 = (es == 8) & (ros == 0) & (dim > 32) & (dim <= 128)
    assert np.array_equal(G[sel64], own[sel64])


def _lanes_for_dim(d):
    g = 4
    while g < (d + 3) // 4 and g < 64:
        g *= 2
    return g


def test_unbuilt_shape_is_refused_not_launched(table):
    """(8 lanes, 2 chunks, 64 rows) has no kernel: the library must never
    pick it (the batch policy gives 4 lanes at 33-64 dimensions)."""
    es, dim, G, NCH, TM, built, fits = (table[0][:, i] for i in range(7))
    pol = table[1]
    assert not np.any((pol[:, 3] == 8) & (pol[:, 4] == 2) & (pol[:, 5] == 64))
    sel = (G == 8) & (NCH == 2) & (TM == 64)
    assert sel.any() and not built[sel].any()


def test_batch_layout_accepts_every_policy_dimension():
    """Through the C ABI (host-side sizing only, no GPU): a batch of rotated
    runs of every dimension 1..512 in binary32 and 1..256 in binary64 (and
    Rosenbrock, which keeps its own lanes) is sized, i.e. every member's
    shape is launchable."""
    from paper_2510_14982_amd import _lib
    L = _lib.lib()
    keep = []
    for prec, top in ((_lib.APO_FP32, 512), (_lib.APO_FP64, 256)):
      for kind in (_lib.KINDS["rastrigin"], _lib.KINDS["rosenbrock"]):
        for d in range(1, top + 1):
            lb, ub = np.full(d, -1.0), np.full(d, 1.0)
            rot = np.eye(d)
            keep += [lb, ub, rot]
            desc = (_lib.RunDesc * 1)()
            desc[0].dim = d
            desc[0].lb, desc[0].ub = _lib._dptr(lb), _lib._dptr(ub)
            desc[0].pop, desc[0].np, desc[0].pf_max, desc[0].seed = 64, 1, 0.1, 1
            desc[0].opt.max_iter = 10
            desc[0].opt.precision = prec
            desc[0].opt.objective.kind = kind
            desc[0].opt.objective.rot = _lib._dptr(rot)
            assert L.apo_batch_workspace_bytes(1, desc) > 0, (kind, d)


def test_persistent_lds_image_fits_and_is_disjoint(table):
    """The persistent elementwise form keeps a run's state in LDS: at the
    largest population it takes (256 / G protozoa) and every dimension up to
    1024, the image plus the sort's and masks' static LDS fits one workgroup,
    and its regions are 16-byte aligned, in order, and each as large as the
    array it holds."""
    image = table[2]
    limit, static = 163840, 16384
    for es, dim, G, pop, total, x0, x1, f, fs, perm, drf, pdr, lb, ub, sh in image:
        Dp = (dim + 64 // es - 1) // (64 // es) * (64 // es)
        offs = [x0, x1, f, fs, perm, drf, pdr, lb, ub, sh, total]
        sizes = [pop * Dp * es, pop * Dp * es, pop * es, pop * es, pop * 4, pop, pop * 8,
                 Dp * es, Dp * es, Dp * es]
        assert all(o % 16 == 0 for o in offs)
        assert all(offs[i] + sizes[i] <= offs[i + 1] for i in range(len(sizes)))
        assert total + static <= limit, (es, dim, total)
