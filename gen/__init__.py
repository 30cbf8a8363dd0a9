"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.  This module holds none of the optimiser's arithmetic: it only
makes the shift vectors, rotation matrices, grey-level images and workload
descriptions that both sides are then handed as inputs.

All randomness here comes from numpy's PCG64 (``numpy.random.default_rng``)
seeded with ``[seed, tag]``, independent of the Philox stream the optimiser
itself draws from.

Workload shapes follow the paper's experiments: CEC-style box-bounded
functions on [-100, 100]^D (Table 2 uses D = 1000, ps 1k-10k) and grey-level
image thresholding over [0, 255] (Table 3).  The CEC 2022 suite and the test
image are not reproduced; seeded shifted (and rotated) classic functions and
a seeded blob image stand in for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_TAG_SHIFT, _TAG_ROT, _TAG_IMAGE, _TAG_STATE = 11, 12, 13, 14


def shift_vector(dim: int, seed: int, lo: float = -80.0, hi: float = 80.0,
                 dtype=np.float64) -> np.ndarray:
    """o ~ U[lo, hi]^dim, rounded to ``dtype`` and returned as float64 (so
    the same values are exactly representable on both sides)."""
    rng = np.random.default_rng([seed, _TAG_SHIFT])
    o = rng.uniform(lo, hi, size=dim)
    return o.astype(dtype).astype(np.float64)


def rotation_matrix(dim: int, seed: int, dtype=np.float64) -> np.ndarray:
    """A Haar-distributed orthogonal matrix: QR of an N(0,1) matrix with the
    columns of Q multiplied by sign(diag R) (Mezzadri 2007).  Rounded to
    ``dtype`` and returned as float64."""
    rng = np.random.default_rng([seed, _TAG_ROT])
    A = rng.standard_normal((dim, dim))
    Q, R = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(R))[None, :]
    return np.ascontiguousarray(Q.astype(dtype).astype(np.float64))


def blob_image(height: int, width: int, seed: int, n_components: int = 5,
               n_blobs: int = 64, grid: int = 16) -> np.ndarray:
    """An 8-bit grey image: a mixture of ``n_components`` Gaussians
    (means U[20, 235], sigma U[5, 25]) laid out as seeded spatial blobs.

    Blobs are Voronoi cells of ``n_blobs`` seeded centres, computed on a
    coarse grid (one cell per ``grid`` x ``grid`` pixels) and each cell given
    one mixture component; pixel = clamp(rint(mu + sigma * N(0, 1)), 0, 255).
    """
    rng = np.random.default_rng([seed, _TAG_IMAGE])
    mu = rng.uniform(20.0, 235.0, size=n_components)
    sigma = rng.uniform(5.0, 25.0, size=n_components)
    cy = rng.uniform(0, height, size=n_blobs)
    cx = rng.uniform(0, width, size=n_blobs)
    comp = rng.integers(0, n_components, size=n_blobs)
    gh, gw = -(-height // grid), -(-width // grid)
    yy = (np.arange(gh) + 0.5) * grid
    xx = (np.arange(gw) + 0.5) * grid
    d2 = (yy[:, None, None] - cy[None, None, :]) ** 2 + (xx[None, :, None] - cx[None, None, :]) ** 2
    cell = np.argmin(d2, axis=2)                       # [gh, gw]
    label = comp[cell]
    label = np.repeat(np.repeat(label, grid, axis=0), grid, axis=1)[:height, :width]
    img = np.empty((height, width), dtype=np.uint8)
    rows = max(1, (1 << 22) // max(width, 1))          # bounded working set
    for r0 in range(0, height, rows):
        r1 = min(height, r0 + rows)
        lab = label[r0:r1]
        v = mu[lab] + sigma[lab] * rng.standard_normal(lab.shape)
        img[r0:r1] = np.clip(np.rint(v), 0, 255).astype(np.uint8)
    return img


def histogram_of(img: np.ndarray) -> np.ndarray:
    """256-bin grey-level histogram (numpy's exact integer bincount)."""
    return np.bincount(np.asarray(img, dtype=np.uint8).reshape(-1), minlength=256).astype(np.uint64)


def random_state(pop: int, dim: int, lb, ub, seed: int, dtype=np.float64) -> np.ndarray:
    """A population uniformly spread in the bounds (for injected-state
    parity cases), rounded to ``dtype`` and returned as float64."""
    rng = np.random.default_rng([seed, _TAG_STATE])
    lb = np.broadcast_to(np.asarray(lb, np.float64), (dim,))
    ub = np.broadcast_to(np.asarray(ub, np.float64), (dim,))
    X = lb + rng.random((pop, dim)) * (ub - lb)
    X = np.clip(X.astype(dtype).astype(np.float64), lb, ub)
    return np.ascontiguousarray(X)


@dataclass
class Workload:
    """One APO configuration: sizes, bounds, objective and its inputs."""
    name: str
    dim: int
    pop: int
    max_iter: int
    precision: str                    # "fp64" | "fp32"
    kind: str                         # objective
    lb: np.ndarray
    ub: np.ndarray
    np_pairs: int = 1
    pf_max: float = 0.1
    seed: int = 1
    run: int = 0
    shift: Optional[np.ndarray] = None
    rot: Optional[np.ndarray] = None
    hist: Optional[np.ndarray] = None
    note: str = ""
    extra: dict = field(default_factory=dict)


def _dt(precision: str):
    return np.float32 if precision == "fp32" else np.float64


def shifted_rastrigin_small(seed: int = 1) -> Workload:
    """Plain APO in FP64: ps 32, D 10, 200 iterations, np 1, pf_max 0.1,
    shifted Rastrigin on [-100, 100]^10 with o ~ U[-80, 80]^10."""
    D = 10
    return Workload("shifted_rastrigin_ps32_d10_fp64", D, 32, 200, "fp64", "rastrigin",
                    np.full(D, -100.0), np.full(D, 100.0), seed=seed,
                    shift=shift_vector(D, seed))


def rotated_rastrigin_large(seed: int = 1, pop: int = 4096, dim: int = 100,
                            max_iter: int = 1000) -> Workload:
    """Single large FP32 run: ps 4096, D 100, 1000 iterations, np 1,
    pf_max 0.1, shifted-rotated Rastrigin f(M(x - o)) on [-100, 100]^100,
    M Haar-orthogonal, o ~ U[-80, 80]^100 (both rounded to binary32)."""
    dt = np.float32
    return Workload(f"rotated_rastrigin_ps{pop}_d{dim}_fp32", dim, pop, max_iter, "fp32",
                    "rastrigin", np.full(dim, -100.0), np.full(dim, 100.0), seed=seed,
                    shift=shift_vector(dim, seed, dtype=dt),
                    rot=rotation_matrix(dim, seed, dtype=dt))


def kapur_thresholds(k: int = 4, seed: int = 1, side: int = 4096, pop: int = 1024,
                     max_iter: int = 500, img: Optional[np.ndarray] = None) -> Workload:
    """Multilevel thresholding: Kapur entropy over k integer thresholds of a
    synthetic side x side blob image; ps 1024, 500 iterations, bounds
    [0, 255].  The histogram is computed here with numpy for the oracle; the
    GPU path computes its own from the image."""
    if img is None:
        img = blob_image(side, side, seed)
    w = Workload(f"kapur_k{k}_img{side}_ps{pop}_fp32", k, pop, max_iter, "fp32", "kapur",
                 np.zeros(k), np.full(k, 255.0), seed=seed, hist=histogram_of(img))
    w.extra["image"] = img
    return w


def otsu_single(side: int = 512, seed: int = 1, pop: int = 100, max_iter: int = 50,
                precision: str = "fp64", img: Optional[np.ndarray] = None) -> Workload:
    """Single-threshold Otsu in the shape of the paper's thresholding table:
    ps 100, D 1, 50 iterations, bounds [0, 255], on a synthetic side x side
    blob image (standing in for the paper's colour test image)."""
    if img is None:
        img = blob_image(side, side, seed)
    w = Workload(f"otsu_k1_img{side}_ps{pop}_{precision}", 1, pop, max_iter, precision, "otsu",
                 np.zeros(1), np.full(1, 255.0), seed=seed, hist=histogram_of(img))
    w.extra["image"] = img
    return w


def batched_runs(n: int = 512, seed: int = 1, max_iter: int = 1000,
                 dims=(10, 20, 50, 100), pops=(64, 256, 1024),
                 kinds=("rastrigin", "rosenbrock", "ackley")) -> list:
    """Independent FP32 runs for the batched form: a balanced, seeded
    shuffle of dims x pops x kinds (each combination n // combos or one
    more times), every run shifted and rotated with its own o ~ U[-80, 80]
    and Haar M, bounds [-100, 100], np 1, pf_max 0.1, seed seed + i and
    run id i.  Returns a list of Workload."""
    combos = [(d, p, k) for d in dims for p in pops for k in kinds]
    reps = [n // len(combos) + (1 if i < n % len(combos) else 0) for i in range(len(combos))]
    plan = [c for c, r in zip(combos, reps) for _ in range(r)]
    order = np.random.default_rng(seed).permutation(len(plan))
    out = []
    for i, j in enumerate(order):
        d, p, k = plan[j]
        s = seed * 100003 + i
        w = Workload(f"batch_{i}_{k}_d{d}_ps{p}", d, p, max_iter, "fp32", k,
                     np.full(d, -100.0), np.full(d, 100.0), seed=seed + i, run=i,
                     shift=shift_vector(d, s), rot=rotation_matrix(d, s))
        out.append(w)
    return out


WORKLOADS = {
    "c1": shifted_rastrigin_small,
    "c2": rotated_rastrigin_large,
    "c3": kapur_thresholds,
}
