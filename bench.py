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
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP32_MFMA_TFLOPS = 157.3  # MI355X dense FP32 matrix
PEAK_BF16_MFMA_TFLOPS = 2500.0  # MI355X dense BF16 matrix
# The paper's own headline, on its hardware: context, not a target.
PAPER_CONTEXT = ("cuAPO reports up to 6.7x (average 4.87x) over its sequential CPU version: "
                 "NVIDIA Tesla T4, CUDA 12.2, against one core of an Intel Xeon at 2.20 GHz; "
                 "other hardware, quoted as context only")
# Counter summaries (HBM bytes per launch of a workload's dominant kernel)
# and the kernel sources they were taken on.
TRAFFIC = {
    "c2": ("traffic_step_tile_f32_rotated_rastrigin_ps4096_d100.md",
           ["apo_step.hpp", "apo_device.hpp", "apo_step_tile_f32.hip"]),
    "c5": ("traffic_gemm_obj_bf16_rotated_ackley_ps8192_d1000.md",
           ["apo_gemm.hip", "apo_step.hpp", "apo_device.hpp"]),
}


def kernel_source_hash(sources) -> str:
    """Hash of the kernel sources' code: comments and blank lines are left
    out, so a counter summary stays valid across comment-only edits."""
    h = hashlib.sha256()
    for name in sources:
        with open(os.path.join(ROOT, "paper_2510_14982_amd", "csrc", name)) as f:
            text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per launch of the workload's dominant kernel from the
    committed counter summary, only if it was taken on the current kernel
    source."""
    fname, sources = TRAFFIC[workload]
    fields = {}
    try:
        with open(os.path.join(ROOT, "profiles", fname)) as f:
            for line in f:
                if ":" in line and not line.startswith((" ", "|", "#")):
                    k, v = line.split(":", 1)
                    fields[k.strip()] = v.strip()
    except OSError:
        return None
    if fields.get("kernel_source_hash") != kernel_source_hash(sources):
        return None
    try:
        return int(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Threads this process may use: the affinity set, capped by
    OMP_NUM_THREADS when it is set (the share of the host given to it)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def _oracle_rate(O, w, budget_s: float):
    p = O.Problem(dim=w.dim, pop=w.pop, lb=w.lb, ub=w.ub, np_pairs=w.np_pairs,
                  max_iter=w.max_iter, pf_max=w.pf_max, seed=w.seed, kind=w.kind,
                  shift=w.shift, rot=w.rot, hist=w.hist)
    X, F = p.init()
    t0 = time.perf_counter()
    n = 0
    while n < w.max_iter:
        X, F, _ = p.step(n + 1, X, F, trace=False)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return w.pop * n / dt, n, dt


def cpu_baseline(w, budget_s: float):
    """The oracle, as it stands, on this host: init + as many iterations of
    the same workload as fit in half the budget, once on one thread and once
    with its loops over protozoa spread over every thread this process may
    use (bit-identical results)."""
    import oracle as O
    threads = host_threads()
    O.set_threads(1)
    v1, n1, dt1 = _oracle_rate(O, w, budget_s / 2)
    used = O.set_threads(threads)
    vn, nn, dtn = _oracle_rate(O, w, budget_s / 2)
    O.set_threads(1)
    return {"value": vn, "unit": "evals/s", "cores": used, "kind": "oracle",
            "sample": f"iterations 1..{nn} of {w.name} (from the oracle's own initial "
                      f"population), FP64 oracle on {used} threads, {dtn:.1f} s",
            "single_core": {"value": v1, "unit": "evals/s", "cores": 1,
                            "sample": f"iterations 1..{n1}, one thread, {dt1:.1f} s"},
            "nproc": os.cpu_count(), "threads_available": threads, "cpu_model": cpu_model()}


def make_handle(apo, w, precision):
    return apo.APO(w.dim, w.lb, w.ub, w.pop, np_pairs=w.np_pairs, pf_max=w.pf_max,
                   seed=w.seed, max_iter=w.max_iter, precision=precision, kind=w.kind,
                   shift=w.shift, rot=w.rot, hist=w.hist)


def timed_run(torch, apo, w, precision, steps, warmup):
    """`warmup` untimed iterations, then exactly `steps` timed iterations.
    Every handle the timed region uses is created and its replay graphs
    captured (apo_run(h, 0)) beforehand; the warm-up runs on the first of
    them, and runs of the configured length are chained when warm-up plus
    steps exceed one run."""
    warm = max(0, min(warmup, w.max_iter - 1))
    plan, left, first_room = [], steps, w.max_iter - warm
    while left > 0:
        room = first_room if not plan else w.max_iter
        plan.append(min(left, room))
        left -= plan[-1]
    handles = [make_handle(apo, w, precision) for _ in plan]
    for h in handles:
        h.run(0)
    if warm:
        handles[0].run(warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for h, n in zip(handles, plan):
        h.run(n)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    best_f = handles[-1].best()[1]
    for h in handles:
        h.close()
    return dt, best_f


def repeat_runs(torch, apo, w, precision, runs=5):
    """Whole runs of the configured length, each on a fresh handle whose
    graphs are captured before its timed run (the paper reports the average
    of 5 runs); evals/s of each."""
    out = []
    for _ in range(runs):
        with make_handle(apo, w, precision) as g:
            g.run(0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.run(w.max_iter)
            torch.cuda.synchronize()
            out.append(w.pop * w.max_iter / (time.perf_counter() - t0))
    return out


def measured_peaks(torch):
    """What this device reaches on plain library work: a device-to-device
    copy (read + write bytes) and large GEMMs through torch.matmul (the
    vendor BLAS, run as a black box)."""
    res = {}
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    res["copy_GB_per_s"] = 2 * n * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    for name, dt, m in (("bf16", torch.bfloat16, 8192), ("fp32", torch.float32, 8192)):
        x = torch.randn(m, m, device="cuda").to(dt)
        y = torch.randn(m, m, device="cuda").to(dt)
        for _ in range(3):
            torch.matmul(x, y)
        torch.cuda.synchronize()
        e0.record()
        reps = 20
        for _ in range(reps):
            torch.matmul(x, y)
        e1.record()
        torch.cuda.synchronize()
        res[f"gemm_{name}_TFLOP_per_s"] = 2 * m ** 3 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e12
    return res


def kernel_times(apo, w, precision, iters):
    with make_handle(apo, w, precision) as g:
        n, kt = g.time_kernels(min(iters, w.max_iter))
    return n, kt


def workload(name, seed):
    import gen
    if name == "c2":
        return gen.rotated_rastrigin_large(seed=seed), "fp32"
    if name == "c1":
        return gen.shifted_rastrigin_small(seed=seed), "fp64"
    if name == "c3":
        return gen.kapur_thresholds(k=16, seed=seed), "fp32"
    if name == "elem-large":
        w = gen.rotated_rastrigin_large(seed=seed, pop=8192, dim=1000, max_iter=200)
        w.rot = None
        w.name = "shifted_rastrigin_ps8192_d1000_fp32"
        return w, "fp32"
    raise SystemExit(f"unknown workload {name}")


# The paper's single-threshold Otsu timings (CUDA version, Tesla T4, 5-run
# average, seconds; the image is rescanned per evaluation there): context.
PAPER_OTSU_PAR_S = {512: 3.0, 1024: 13.0, 2048: 50.0, 4096: 199.0}


def otsu_table(torch, apo, args):
    """Histogram + 50 iterations of single-threshold Otsu (ps 100, D 1,
    binary64) per synthetic image size; one JSON line."""
    import gen
    rows = {}
    for side in (512, 1024, 2048, 4096):
        w = gen.otsu_single(side=side, seed=args.seed)
        img = torch.from_numpy(w.extra["image"]).cuda().reshape(-1)
        apo.histogram_u8(img)
        torch.cuda.synchronize()
        times = []
        for _ in range(5):
            t0 = time.perf_counter()
            h = apo.histogram_u8(img)
            with apo.APO(w.dim, w.lb, w.ub, w.pop, seed=w.seed, max_iter=w.max_iter,
                         precision="fp64", kind=w.kind, hist=h) as g:
                g.run(w.max_iter)
                xb, fb, _ = g.best()
            times.append(time.perf_counter() - t0)
        assert (h == w.hist).all(), "GPU histogram differs from numpy's"
        med = sorted(times)[2]
        rows[f"{side}x{side}"] = {"seconds_median_of_5": med, "best_threshold": float(round(xb[0])),
                                  "paper_cuda_seconds": PAPER_OTSU_PAR_S[side],
                                  "evals_per_s": w.pop * w.max_iter / med}
    big = rows["4096x4096"]
    print(json.dumps({
        "metric": "single-threshold Otsu: histogram + 50 APO iterations per image (ps 100, D 1)",
        "value": big["evals_per_s"], "unit": "evals/s", "n_gpus": 1, "steps": 50, "warmup": 1,
        "ms_per_step": 1000.0 * big["seconds_median_of_5"] / 50, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "otsu_k1_ps100_t50", "images": list(rows)},
        "per_image": rows,
        "note": "wall time per image includes the GPU histogram, handle creation, 50 iterations "
                "and the best read-back; the paper's times are context only (other hardware, "
                "image rescanned per evaluation)"}), flush=True)


def batched(torch, apo, args):
    """512 independent FP32 runs (D 10..100, ps 64..1024, rotated Rastrigin /
    Rosenbrock / Ackley) advanced together, against the same runs as plain
    handles one after another (timed on one run per combination and scaled
    by each combination's count)."""
    import collections
    import gen
    T = 1000
    ws = gen.batched_runs(n=512, seed=args.seed, max_iter=T)
    specs = [dict(dim=w.dim, lb=w.lb, ub=w.ub, pop=w.pop, seed=w.seed, max_iter=T,
                  precision="fp32", kind=w.kind, shift=w.shift, rot=w.rot, run_id=w.run)
             for w in ws]
    evals = sum(w.pop for w in ws) * T
    flops = sum(2.0 * w.pop * w.dim * w.dim for w in ws)
    # the first 16 iterations are the warm-up (they capture the graphs)
    steps = T - 16 if args.steps is None else max(1, min(args.steps, T - 16))
    with apo.Batch(specs) as b:
        sched, us = b.tune(16)          # the runs' state is restored after the trials
        w_n = T - steps
        b.run(w_n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    pop_sum = sum(w.pop for w in ws)
    value = pop_sum * steps / dt
    # the plain form: one handle per run, run to completion one after another
    combos = collections.Counter((w.dim, w.pop, w.kind) for w in ws)
    first = {}
    for i, w in enumerate(ws):
        first.setdefault((w.dim, w.pop, w.kind), i)
    seq_iters = 100
    seq_time = 0.0
    for key, cnt in combos.items():
        sp = dict(specs[first[key]], max_iter=seq_iters)
        with apo.APO(**sp) as g:
            g.run(5)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.run(seq_iters - 5)
            torch.cuda.synchronize()
            per_iter = (time.perf_counter() - t0) / (seq_iters - 5)
        seq_time += per_iter * cnt * steps
    seq_value = pop_sum * steps / seq_time
    it_s = steps / dt
    achieved = flops * it_s / 1e12
    print(json.dumps({
        "metric": "fitness evals/sec of 512 independent runs advanced together",
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": steps, "warmup": w_n,
        "ms_per_step": 1000.0 * dt / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch512_rotated_mixed_fp32", "runs": len(ws),
                   "dims": [10, 20, 50, 100], "pops": [64, 256, 1024],
                   "objectives": ["rastrigin", "rosenbrock", "ackley"], "iterations": T,
                   "parallelism": "single GPU"},
        "iters_per_s": it_s,
        "schedule": {"chosen": sched, "us_per_iteration": list(map(float, us)),
                     "candidates": ["serial, run order", "parallel branches, run order",
                                    "serial, interleaved", "parallel branches, interleaved"]},
        "sequential_plain": {"value": seq_value, "unit": "evals/s",
                             "speedup_of_batch": value / seq_value,
                             "sample": f"one run per combination ({len(combos)}), "
                                       f"{seq_iters - 5} timed iterations each, scaled by count"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_MFMA_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA_TFLOPS,
                     "traffic": None,
                     "kernel": "whole iteration (sort + all batched step launches)",
                     "algorithmic_flops_per_iteration": flops},
    }), flush=True)


def np_ablation(torch, apo, args):
    """Neighbour pairs np = 1, 2, 4, 8 on the single large run (ps 4096,
    D 100, rotated Rastrigin, FP32, 1000 iterations): throughput and the
    final best fitness over three seeds (np > 1 gathers 2 np rows per
    foraging protozoan and enlarges the weighted sums of Eqs. (6), (8))."""
    import gen
    rows = {}
    for npairs in (1, 2, 4, 8):
        rates, bests = [], []
        for seed in (1, 2, 3):
            w = gen.rotated_rastrigin_large(seed=seed)
            w.np_pairs = npairs
            with make_handle(apo, w, "fp32") as g:
                g.run(16)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                g.run(w.max_iter - 16)
                torch.cuda.synchronize()
                rates.append(w.pop * (w.max_iter - 16) / (time.perf_counter() - t0))
                bests.append(g.best()[1])
        rows[f"np{npairs}"] = {"evals_per_s_median": sorted(rates)[1],
                               "final_best_f": bests, "final_best_f_median": sorted(bests)[1]}
    print(json.dumps({
        "metric": "np ablation: fitness evals/sec and final best fitness, ps 4096 D 100",
        "value": rows["np1"]["evals_per_s_median"], "unit": "evals/s", "n_gpus": 1,
        "steps": 984, "warmup": 16, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "rotated_rastrigin_ps4096_d100_fp32", "np": [1, 2, 4, 8],
                   "seeds": [1, 2, 3]},
        "per_np": rows}), flush=True)


def precision_run(torch, apo, args):
    """ps 8192, D 1000, shifted-rotated Ackley (or --objective), 2000 iterations: the BF16
    form (estimate + binary32 re-score of every unsettled candidate and
    acceptance; it stores what the binary32 form stores) against the
    binary32 GEMM form, with the elite re-scored in binary64 and compared
    with the oracle's binary64 objective of the returned position."""
    import gen
    import oracle as O
    T = 2000
    w = gen.rotated_rastrigin_large(seed=args.seed, pop=8192, dim=1000, max_iter=T)
    w.kind = args.objective
    w.name = f"rotated_{args.objective}_ps8192_d1000"
    steps = T - 16 if args.steps is None else max(1, min(args.steps, T - 16))
    flops = 2.0 * w.pop * w.dim * w.dim
    forms = {}
    for prec in ("fp32", "bf16"):
        with make_handle(apo, w, prec) as g:
            g.run(16)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.run(steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            x, f, fes = g.best()
            resc, est = g.precision_stats()
        with make_handle(apo, w, prec) as h:
            _, st = h.time_gemm_stages(20)
        p = O.Problem(dim=w.dim, pop=w.pop, lb=w.lb, ub=w.ub, kind=w.kind, shift=w.shift,
                      rot=w.rot)
        fo = p.objective(x)
        forms[prec] = {"evals_per_s": w.pop * steps / dt, "ms_per_step": 1000.0 * dt / steps,
                       "final_best_f_fp64": f, "oracle_f_of_best_x": fo,
                       "abs_error_vs_oracle": abs(f - fo), "stage_us": st,
                       "rescored_fraction": (resc / est) if est else None,
                       "product_TFLOP_per_s": flops / (st["product"] * 1e-6) / 1e12}
    b, fp = forms["bf16"], forms["fp32"]
    ach = b["product_TFLOP_per_s"]
    out = {
        "metric": "fitness evals/sec, BF16 precision pipeline vs binary32 form (ps 8192, D 1000)",
        "value": b["evals_per_s"], "unit": "evals/s", "n_gpus": 1, "steps": steps, "warmup": 16,
        "ms_per_step": b["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": w.name, "pop": w.pop, "dim": w.dim, "iterations": T,
                   "objective": w.kind, "rotated": True, "parallelism": "single GPU"},
        "bf16_over_fp32": b["evals_per_s"] / fp["evals_per_s"],
        "equal_final_fitness": b["final_best_f_fp64"] == fp["final_best_f_fp64"],
        "forms": forms,
        "roofline": {"bound": "mfma", "achieved": ach, "peak": PEAK_BF16_MFMA_TFLOPS,
                     "unit": "TFLOP/s", "frac": ach / PEAK_BF16_MFMA_TFLOPS,
                     "traffic": measured_traffic("c5") if w.kind == "ackley" else None,
                     "kernel": f"gemm_obj_bf16<{w.kind.upper()}> (BF16 estimate of "
                               "z = M (y - o) with fused objective sums)",
                     "algorithmic_flops_per_launch": flops,
                     "algorithmic_bytes_per_launch": (w.pop + 1024) * 1024 * 2},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
        out["gpu_over_cpu_baseline"] = out["value"] / out["cpu_baseline"]["value"]
    out["context"] = PAPER_CONTEXT
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed iterations (default: the workload's configured run length)")
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--workload", default="c2",
                    choices=["c2", "c1", "c3", "elem-large", "otsu", "c4", "np-ablation", "c5"])
    ap.add_argument("--objective", default="ackley", choices=["ackley", "rastrigin", "sphere"],
                    help="objective of the precision workload (c5); its configuration is Ackley")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-iters", type=int, default=None,
                    help="iterations of the event-timed kernel run (default: the whole run, "
                         "so the operation mix matches the timed region's)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--peaks", action="store_true",
                    help="also measure the device's copy bandwidth and library GEMM rates")
    ap.add_argument("--no-repeats", action="store_true",
                    help="skip the five whole-run repeats")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the library runs on one GPU; it has no multi-GPU form)", file=sys.stderr)
        sys.exit(2)

    import torch
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

    if args.workload == "otsu":
        otsu_table(torch, apo, args)
        return
    if args.workload == "c4":
        batched(torch, apo, args)
        return
    if args.workload == "np-ablation":
        np_ablation(torch, apo, args)
        return
    if args.workload == "c5":
        precision_run(torch, apo, args)
        return
    w, precision = workload(args.workload, args.seed)
    steps = w.max_iter if args.steps is None else args.steps
    es = 8 if precision == "fp64" else 4
    extra = {}
    if args.workload == "c3":
        # the image is reduced once on the GPU: time the call (kernel, copy
        # of the 256 counts to the host and the synchronisation)
        img = torch.from_numpy(w.extra["image"]).cuda().reshape(-1)
        apo.histogram_u8(img)
        torch.cuda.synchronize()
        reps = 20
        t0 = time.perf_counter()
        for _ in range(reps):
            h = apo.histogram_u8(img)
        hist_us = (time.perf_counter() - t0) * 1e6 / reps
        assert (h == w.hist).all(), "GPU histogram differs from numpy's"
        extra["histogram"] = {"pixels": int(img.numel()), "us_per_call": hist_us,
                              "note": "whole call: kernels, copy of the counts to the host, "
                                      "stream synchronisation"}
    dt, best_f = timed_run(torch, apo, w, precision, steps, args.warmup)
    kn, kt = kernel_times(apo, w, precision,
                          w.max_iter if args.kernel_iters is None else args.kernel_iters)
    if not args.no_repeats:
        reps = repeat_runs(torch, apo, w, precision)
        extra["runs_evals_per_s"] = {"runs": reps, "median": sorted(reps)[len(reps) // 2],
                                     "iterations_each": w.max_iter}
    if args.peaks:
        extra["measured_peaks"] = measured_peaks(torch)
    step_us = kt["step_us"]
    bytes_alg = 2.0 * w.pop * w.dim * es          # read X once, write X' once
    out = {
        "metric": "fitness evals/sec + APO iters/sec at pop x D; %HBM roofline / %MFMA peak",
        "value": w.pop * steps / dt,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * dt / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "pop": w.pop, "dim": w.dim, "iterations": w.max_iter,
                   "np": w.np_pairs, "pf_max": w.pf_max, "objective": w.kind,
                   "rotated": w.rot is not None, "parallelism": "single GPU"},
        "iters_per_s": steps / dt,
        "final_best_f": best_f,
        "kernel_us": {"rank_sort": kt["rank_us"], "step": step_us, "iterations": kn},
    }
    out.update(extra)
    if w.rot is not None:
        flops = 2.0 * w.pop * w.dim * w.dim        # z = M (y - o) for every candidate
        achieved = flops / (step_us * 1e-6) / 1e12
        out["roofline"] = {
            "bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_MFMA_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA_TFLOPS,
            "traffic": measured_traffic("c2") if args.workload == "c2" else None,
            "kernel": "step_tile_sep<float> (update + clamp + z = M(y-o) on MFMA + select)",
            "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": bytes_alg,
            "hbm_frac_at_algorithmic_bytes": bytes_alg / (step_us * 1e-6) / 1e9 / PEAK_HBM_GBS}
    else:
        achieved = bytes_alg / (step_us * 1e-6) / 1e9
        out["roofline"] = {
            "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": None,
            "kernel": "step (update + clamp + objective + select)",
            "algorithmic_bytes_per_launch": bytes_alg}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
        out["gpu_over_cpu_baseline"] = out["value"] / out["cpu_baseline"]["value"]
    out["context"] = PAPER_CONTEXT
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
