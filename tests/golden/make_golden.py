"""Writes the stored expected results of the whole-run parity tests.

Every value comes from the CPU oracle (``oracle/gao.c``) and nothing else:
the configurations are drawn by ``tests/inputs.py`` and each run is
``gao.run``.  The runs are too long to repeat inside a GPU test (tens of
minutes of CPU each), so their results are stored here:

* ``elite_m32_n200000.json``: the elitist plain GA at order 32, population
  200,000, seed 2, key SQ + NNZ, 2,000 elites, 1,000 generations, no stop on
  found: the result and SHA-256 digests of the final population (int8
  [n][m][m], C order) and keys (uint32, little-endian);
* ``batched_24runs.json``: the 24 runs of the batched workload (orders
  12..36, populations 2,000..60,000, 300 generations each): each run's
  result, best matrix and final-population digests;
* ``served_slice.json``: the first requests of the served stream whose order
  is at most 16 (the others need hours of oracle time): result and best
  matrix of each;
* ``paper_table2_m20.json``: the paper-mode runs of the Sec. 4.2 timing
  configuration at order 20 (40,000 matrices, crossover and mutation on every
  offspring, NC = 4, NR = 2, 10^4 generations, no stop on found, seed 9020),
  keys F1 and F2: result and final-population digests of each.

Usage: python tests/golden/make_golden.py {elite,batched,served,table2} [...]
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import gao  # noqa: E402
from tests import inputs  # noqa: E402

SERVED_REQUESTS = 200   # the slice of the served stream
SERVED_MAX_ORDER = 16   # orders the oracle finishes in minutes per request


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def matrix_rows(Q: np.ndarray) -> list:
    return ["".join("+" if x > 0 else "-" for x in row) for row in Q]


def run_record(fields: dict, with_digests: bool) -> dict:
    cfg = gao.Config(**fields)
    t = time.time()
    res, pop, keys = gao.run(cfg)
    rec = {"config": fields, **res, "matrix": matrix_rows(pop[res["index"]])}
    if with_digests:
        rec["population_sha256"] = digest(pop)
        rec["keys_sha256"] = digest(keys.astype("<u4"))
    print(f"  m={cfg.m} n={cfg.n} seed={cfg.seed}: {res} ({time.time() - t:.1f} s)", flush=True)
    return rec


def write(name: str, payload: dict) -> None:
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(payload, f, indent=1)
        f.write("\n")
    print("wrote", path, flush=True)


def elite() -> None:
    fields = dict(m=32, n=200_000, seed=2, fitness=gao.FIT_SQ_PLUS_NNZ, elite=2000,
                  max_generations=1000, stop_on_found=False)
    write("elite_m32_n200000.json", {"source": "oracle gao.run", "run": run_record(fields, True)})


def batched() -> None:
    runs = [run_record(f, True) for f in inputs.batched_workload()]
    write("batched_24runs.json", {"source": "oracle gao.run", "runs": runs})


def served() -> None:
    reqs, _ = inputs.served_workload()
    picked = [(i, f) for i, f in enumerate(reqs[:SERVED_REQUESTS]) if f["m"] <= SERVED_MAX_ORDER]
    runs = []
    for i, f in picked:
        rec = run_record(f, False)
        rec["request"] = i
        runs.append(rec)
    write("served_slice.json", {"source": "oracle gao.run", "requests": SERVED_REQUESTS,
                                "max_order": SERVED_MAX_ORDER, "runs": runs})


def table2() -> None:
    runs = [run_record(dict(m=20, n=40_000, seed=9020, fitness=kind, selection=gao.SEL_PAPER,
                            xo_threshold=1 << 32, mut_threshold=1 << 32, nc=4, nr=2,
                            max_generations=10_000, stop_on_found=False), True)
            for kind in (gao.FIT_F1, gao.FIT_F2)]
    write("paper_table2_m20.json", {"source": "oracle gao.run", "runs": runs})


if __name__ == "__main__":
    jobs = {"elite": elite, "batched": batched, "served": served, "table2": table2}
    for name in sys.argv[1:] or list(jobs):
        jobs[name]()
