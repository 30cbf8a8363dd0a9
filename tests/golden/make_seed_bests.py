"""Writes seed_bests_rotated_rastrigin_ps4096_d100.json: the oracle's final
best fitness for seeds 1..30 of the single large run (population 4096,
D = 100, 1000 iterations, np = 1, pf_max = 0.1, shifted-rotated Rastrigin
on [-100, 100]^100, binary32 bounds, shift and rotation as the generator
module builds them).  The 30 binary64 oracle runs take about half an hour
of CPU time, so the GPU test that compares distributions reads them from
this file instead of recomputing them.  Calls only the oracle and the
seeded input generators.

    python tests/golden/make_seed_bests.py [threads]
"""
import json
import os
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gen  # noqa: E402
import oracle as O  # noqa: E402

OUT = os.path.join(HERE, "seed_bests_rotated_rastrigin_ps4096_d100.json")
SEEDS = list(range(1, 31))


def best(seed):
    O.set_threads(1)
    w = gen.rotated_rastrigin_large(seed=seed)
    p = O.Problem(dim=w.dim, pop=w.pop, lb=w.lb, ub=w.ub, np_pairs=w.np_pairs,
                  max_iter=w.max_iter, pf_max=w.pf_max, seed=seed, kind=w.kind, shift=w.shift,
                  rot=w.rot)
    f = float(p.solve()[1])
    print(f"seed {seed}: {f!r}", flush=True)
    return f


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        bests = list(ex.map(best, SEEDS))
    doc = {"about": "Oracle (binary64) final best fitness of the single large run "
                    "(ps 4096, D 100, T 1000, np 1, pf_max 0.1, shifted-rotated Rastrigin, "
                    "binary32 inputs), one per seed; written by make_seed_bests.py.",
           "workload": "rotated_rastrigin_ps4096_d100", "seeds": SEEDS, "best_f": bests}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
