"""Autotuner of the children kernel's tile shape: lanes per child.

For every order m = 4..128 (or those given by --orders) and a ladder of
population sizes, times each allowed lanes-per-child variant (2, 4, 8 up to
m = 32; 4, 8 up to 64; 8, 16 above) over a run of the plain GA (binary tournament, SQ key, the library's event-timed
generation loop) and writes the fastest per (order, size) as the tuning
table `csrc/ga_tuned.h` (or --out); rows of orders not timed are kept from
the library's current table.  The variants compute identical generations; only their speed
differs.  Needs a GPU; rebuild the library afterwards.

    python -m paper_2208_14961_amd.tune --out paper_2208_14961_amd/csrc/ga_tuned.h
    python -m paper_2208_14961_amd.tune --orders 68-128
"""
from __future__ import annotations

import argparse
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

# table columns: each entry is timed at the population size SIZES[j] and
# applies to launches of up to MAX_CHILDREN[j] children, the geometric
# midpoint to the next size (the last entry has no limit)
SIZES = [1024, 2048, 4096, 8192, 16384, 32768, 49152, 65536, 131072, 262144]
MAX_CHILDREN = [int((a * b) ** 0.5) for a, b in zip(SIZES, SIZES[1:])] + [None]
ORDERS = list(range(4, 129, 4))


def lanes_options(m: int):
    if m <= 32:
        return (2, 4, 8)
    return (4, 8) if m <= 64 else (8, 16)


def existing_rows(path: str) -> dict:
    """The row text of each order in a table written by this script."""
    rows = {}
    if os.path.exists(path):
        for line in open(path):
            mt = re.match(r"\s*\{[0-9, ]+\},\s*// m = (\d+):", line)
            if mt:
                rows[int(mt.group(1))] = line.rstrip("\n")
    return rows


def time_variant(m: int, n: int, lanes: int, gens: int) -> float:
    """Mean generation time (ms) of a `gens`-generation run."""
    import torch
    import paper_2208_14961_amd as ga
    cfg = ga.Config(m=m, n=n, seed=1, fitness=ga.FIT_SQ, max_generations=gens, flags=ga.lanes_flag(lanes))
    sh = ga.pop_shape(cfg)
    bufs = [torch.zeros(sh, dtype=torch.int32, device="cuda") for _ in range(2)]
    keys = [torch.zeros((n,), dtype=torch.int32, device="cuda") for _ in range(2)]
    ga.ga_run(cfg, bufs[0], bufs[1], keys[0], keys[1])  # warm
    best = None
    for _ in range(3):
        ga.ga_timing_enable(True)
        ga.ga_run(cfg, bufs[0], bufs[1], keys[0], keys[1])
        ms, _ = ga.ga_timing_read()
        ga.ga_timing_enable(False)
        best = ms if best is None else min(best, ms)
    return best


def header(table, times, kept) -> str:
    rows = []
    for i, m in enumerate(ORDERS):
        if m not in table:
            rows.append(kept[m])
            continue
        cells = ", ".join(str(table[m][j]) for j in range(len(SIZES)))
        detail = "; ".join(
            f"n={SIZES[j]}: " + " ".join(f"L{L} {times[m][j][L] * 1e3:.1f}us"
                                         for L in lanes_options(m))
            for j in range(len(SIZES)))
        rows.append(f"  {{{cells}}},  // m = {m}: {detail}")
    limits = ", ".join(str(c) if c is not None else "~0ull" for c in MAX_CHILDREN)
    return f"""// ga_tuned.h -- lanes per child of the children kernel, per order and
// launch size, as chosen by paper_2208_14961_amd/tune.py on one MI355X
// (mean generation time of a plain-GA run, binary tournament, SQ key; the
// times of every variant are in the comments).  Row i is order 4(i+1);
// entry j applies up to kTuneMaxChildren[j] children.  Regenerate with
// `python -m paper_2208_14961_amd.tune` on the GPU, then rebuild.
#pragma once
#include <stdint.h>

namespace ga {{

constexpr int kTuneSizes = {len(SIZES)};
constexpr uint64_t kTuneMaxChildren[kTuneSizes] = {{{limits}}};
constexpr uint8_t kTunedLanes[{len(ORDERS)}][kTuneSizes] = {{
{chr(10).join(rows)}
}};

}}  // namespace ga
"""


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "csrc", "ga_tuned.h"))
    ap.add_argument("--gens", type=int, default=128)
    ap.add_argument("--orders", default="4-128", help="first-last order to time")
    args = ap.parse_args()
    lo, hi = (int(x) for x in args.orders.split("-"))
    kept = existing_rows(os.path.join(HERE, "csrc", "ga_tuned.h"))
    todo = [m for m in ORDERS if lo <= m <= hi]
    missing = [m for m in ORDERS if m not in todo and m not in kept]
    if missing:
        sys.exit(f"no existing row for orders {missing}: time them too")
    table, times = {}, {}
    for m in todo:
        table[m], times[m] = [], []
        for n in SIZES:
            t = {L: time_variant(m, n, L, args.gens) for L in lanes_options(m)}
            best = min(t, key=t.get)
            table[m].append(best)
            times[m].append(t)
            print(f"m={m} n={n}: " + " ".join(f"L{L}={v * 1e3:.2f}us" for L, v in t.items())
                  + f" -> {best}", flush=True)
    text = header(table, times, kept)
    with open(args.out, "w") as f:
        f.write(text)
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
