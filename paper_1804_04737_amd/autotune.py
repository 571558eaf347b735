"""Autotuner for the batched schedule.  Stage 1 sweeps the team knobs -- a
fixed team size or per-LP team sizing (tableau bytes per workgroup), and the
team threshold (tableau bytes from which an LP is solved by a team of
workgroups instead of one workgroup) -- on a seeded batch.  Stage 2 sweeps the
wave-per-instance slots (LPs small enough for a wave's slice of LDS solved by
one wave each, versus one workgroup each).  The result goes to
`autotune.json` next to the library, where lp_solve_batch reads it.

Usage (on the GPU host):  python -m paper_1804_04737_amd.autotune [--out PATH]
"""
from __future__ import annotations

import argparse
import json
import os
import time

PKG = os.path.dirname(os.path.abspath(__file__))


def sweep(count=1024, seed=0, fixed_sizes=(2, 4, 8),
          per_wg=(1 << 18, 3 << 17, 1 << 19, 3 << 18, 1 << 20, 2 << 20, 4 << 20),
          thresholds=(1 << 18, 1 << 19, 1 << 20, 2 << 20, 4 << 20), reps=3, log=print):
    """Time lp_solve_batch for every knob setting; returns (best, all)."""
    import numpy as np
    import torch

    from . import lpdense, lpgen
    lps = lpgen.batch_lps(count, 32, 1024, seed)
    pb = lpdense.pack_batch(lps)
    torch.cuda.synchronize()
    settings = [dict(team_size=1, team_min_bytes=-1, team_bytes_per_wg=1 << 20)]
    settings += [dict(team_size=s, team_min_bytes=t, team_bytes_per_wg=1 << 20)
                 for s in fixed_sizes for t in thresholds]
    settings += [dict(team_size=0, team_min_bytes=t, team_bytes_per_wg=w) for w in per_wg for t in thresholds]
    results = []
    for kw in settings:
        times = []
        for _ in range(reps + 1):
            t0 = time.perf_counter()
            lpdense.solve_batch(pb, **kw)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        results.append(dict(kw, ms=round(float(np.median(times[1:])) * 1e3, 3)))
        log(json.dumps(results[-1]))
    best = min(results, key=lambda r: r["ms"])
    return best, results


def wave_sweep(team, count=1024, tiny_count=4096, seed=0, slots=(-1, 2, 4, 8, 16), reps=3, log=print):
    """Wave-per-instance stage: with the team knobs fixed, time every wave-slot
    count on the batched workload and on a batch of tiny LPs (m, n
    log-uniform in [4, 40]); the choice minimises the geometric mean of the
    two times relative to each workload's best."""
    import numpy as np
    import torch

    from . import lpdense, lpgen
    packs = {"batched": lpdense.pack_batch(lpgen.batch_lps(count, 32, 1024, seed)),
             "tiny": lpdense.pack_batch(lpgen.batch_lps(tiny_count, 4, 40, seed + 1))}
    torch.cuda.synchronize()
    rows = []
    for ws in slots:
        row = {"wave_slots": ws}
        for name, pb in packs.items():
            times = []
            for _ in range(reps + 1):
                t0 = time.perf_counter()
                lpdense.solve_batch(pb, wave_slots=ws, **team)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            row[f"ms_{name}"] = round(float(np.median(times[1:])) * 1e3, 3)
        rows.append(row)
        log(json.dumps(row))
    best = {name: min(r[f"ms_{name}"] for r in rows) for name in packs}
    for r in rows:
        r["score"] = round(float(np.sqrt(np.prod([r[f"ms_{k}"] / best[k] for k in packs]))), 4)
    return min(rows, key=lambda r: r["score"]), rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(PKG, "autotune.json"))
    ap.add_argument("--count", type=int, default=1024)
    args = ap.parse_args()
    best, results = sweep(count=args.count)
    team = {k: best[k] for k in ("team_size", "team_min_bytes", "team_bytes_per_wg")}
    wbest, wrows = wave_sweep(team, count=args.count)
    table = {"batch": {"team_size": best["team_size"], "team_min_bytes": best["team_min_bytes"],
                       "team_bytes_per_wg": best["team_bytes_per_wg"], "ms_per_batch": best["ms"],
                       "wave_slots": max(0, wbest["wave_slots"]),
                       "workload": f"{args.count} LPs, m and n log-uniform in [32, 1024], seed 0; wave slots "
                                   "also timed on 4096 LPs with m and n log-uniform in [4, 40], seed 1"},
             "sweep": results, "wave_sweep": wrows}
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps(table["batch"]))


if __name__ == "__main__":
    main()
