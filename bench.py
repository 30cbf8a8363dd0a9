"""Throughput of the APO population step on one MI355X.

Workload: a single large FP32 run -- population 4096, D = 100, 1000
iterations, np = 1, pf_max = 0.1, shifted-rotated Rastrigin f(M (x - o)) on
[-100, 100]^100 with M Haar-orthogonal and o ~ U[-80, 80]^100 (seeded,
synthetic).  A "step" is one APO iteration of the whole hot path: the rank
sort and the fused step kernel (candidates of Eqs. (1)-(10), clamp, the
rotated objective on the matrix cores, greedy selection), replayed as a HIP
graph.  Inputs and state are resident in HBM before the timed region.

Prints one JSON line: fitness evaluations per second (pop x iterations /
wall time), iterations per second, the roofline of the step kernel (HIP
events on the launch stream) and the plain CPU oracle timed on this host
on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP32_MFMA_TFLOPS = 157.3  # MI355X dense FP32 matrix
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_tile_f32_rotated_rastrigin_ps4096_d100_traffic.json")
KERNEL_SOURCES = ["apo_step.hpp", "apo_device.hpp", "apo_step_tile_f32.hip"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2510_14982_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the step kernel from the committed counter
    summary, only if it was taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(w, budget_s: float):
    """The oracle, as it stands, on this host: init + as many iterations of
    the same workload as fit in the budget (at least one)."""
    import oracle as O
    p = O.Problem(dim=w.dim, pop=w.pop, lb=w.lb, ub=w.ub, np_pairs=w.np_pairs,
                  max_iter=w.max_iter, pf_max=w.pf_max, seed=w.seed, kind=w.kind,
                  shift=w.shift, rot=w.rot)
    X, F = p.init()
    t0 = time.perf_counter()
    n = 0
    while n < w.max_iter:
        X, F, _ = p.step(n + 1, X, F, trace=False)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": w.pop * n / dt, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"iterations 1..{n} of the {w.pop}x{w.dim} rotated-Rastrigin FP32 "
                      f"workload, evaluated by the single-threaded FP64 oracle ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-iters", type=int, default=200)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path has no multi-GPU form in this build)", file=sys.stderr)
        sys.exit(2)

    import torch
    import gen
    import paper_2510_14982_amd as apo

    if args.copy_calibration:
        n = 256 << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "launches": 5}))
        return

    w = gen.rotated_rastrigin_large(seed=args.seed)

    def handle():
        return apo.APO(w.dim, w.lb, w.ub, w.pop, np_pairs=w.np_pairs, pf_max=w.pf_max,
                       seed=w.seed, max_iter=w.max_iter, precision="fp32", kind=w.kind,
                       shift=w.shift, rot=w.rot)

    # warm-up: graph capture, code-object load, clocks
    with handle() as g:
        g.run(max(1, min(args.warmup, w.max_iter)))
        g.best()
    torch.cuda.synchronize()

    # timed region: K iterations, fresh runs of the configured length chained
    # when K exceeds one run
    remaining = args.steps
    handles = []
    while remaining > 0:
        h = handle()
        handles.append((h, min(remaining, w.max_iter)))
        remaining -= w.max_iter
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for h, n in handles:
        h.run(n)
    for h, _ in handles:
        h.info()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _, best_f, fes = handles[-1][0].best()
    for h, _ in handles:
        h.close()

    # per-kernel durations with HIP events on the handle's stream
    with handle() as g:
        kn, kt = g.time_kernels(min(args.kernel_iters, w.max_iter))
    step_us = kt["step_us"]
    flops = 2.0 * w.pop * w.dim * w.dim            # z = M (y - o) for every candidate
    bytes_alg = 2.0 * w.pop * w.dim * 4            # read X once, write X' once (binary32)
    achieved = flops / (step_us * 1e-6) / 1e12
    traffic = measured_traffic()

    out = {
        "metric": "fitness evals/sec + APO iters/sec at pop x D; %HBM roofline / %MFMA peak",
        "value": w.pop * args.steps / dt,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "pop": w.pop, "dim": w.dim, "iterations": w.max_iter,
                   "np": w.np_pairs, "pf_max": w.pf_max, "objective": "shifted-rotated rastrigin",
                   "parallelism": "single GPU"},
        "iters_per_s": args.steps / dt,
        "final_best_f": best_f,
        "kernel_us": {"rank_sort": kt["rank_us"], "step": step_us, "iterations": kn},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_MFMA_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA_TFLOPS,
                     "traffic": traffic,
                     "kernel": "step_tile<float> (update + clamp + z = M(y-o) on MFMA + select)",
                     "algorithmic_flops_per_launch": flops,
                     "algorithmic_bytes_per_launch": bytes_alg,
                     "hbm_frac_at_algorithmic_bytes": bytes_alg / (step_us * 1e-6) / 1e9 / PEAK_HBM_GBS},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
