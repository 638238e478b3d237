"""Construct-schedule autotuner for the batched engine.

For each city-count bucket it builds a synthetic batch of that bucket's
sizes, times a few iterations under every construct schedule (lanes per ant,
live-block list), and keeps the fastest; it then times the number of
persistent construct wavefronts on a whole batch.  All schedules give the
same results bit for bit, so the choice is purely about speed.  The table is
written as JSON and loaded with load_table().

    python -m paper_2404_04895_amd.autotune [--out FILE] [--refine-on WORKLOAD]

With --refine-on the current table is refined on one mixed batch (coordinate
descent, each candidate timed on the whole batch), since a bucket's best
schedule alone need not be its best within a mix.
"""
import argparse
import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "schedules_gfx950.json")
BUCKETS = [64, 96, 128, 192, 256, 384, 512, 1024, 2048]


def _time_batch(dists, sched_table, waves, iters, reps, alpha=1.0, beta=2.0, rho=0.2):
    import torch

    from . import Batch
    stream = torch.cuda.Stream()
    best = float("inf")
    with torch.cuda.stream(stream):
        b = Batch(dists, alpha, beta, rho, 1.0, stream=stream)
        b.set_schedules(sched_table, waves)
        b.run(1)  # warm-up, builds the graph
        for _ in range(reps):
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record(stream)
            b.run(iters)
            t1.record(stream)
            t1.synchronize()
            best = min(best, t0.elapsed_time(t1) / iters)
        b.close()
    stream.synchronize()
    return best


def tune(out_path=DEFAULT_TABLE, per_bucket=48, iters=4, reps=2, seed=0, verbose=True):
    import aco_instances as inst

    from . import SCHEDULES
    rng = np.random.default_rng(seed)
    table, timings = [], {}
    lo = 3
    for hi in BUCKETS:
        ns = rng.integers(max(lo, 3), hi + 1, size=per_bucket)
        dists = [inst.distance_matrix(inst.uniform_cities(int(n), 10_000 + k))
                 for k, n in enumerate(ns)]
        ms_per_sched = {}
        for sched in SCHEDULES:
            ms_per_sched[sched] = _time_batch(dists, [(hi, sched)], 0, iters, reps)
        choice = min(ms_per_sched, key=ms_per_sched.get)
        table.append([int(hi), int(choice)])
        timings["n<=%d" % hi] = {str(k): v for k, v in ms_per_sched.items()}
        if verbose:
            print("bucket n in [%d, %d]: %s -> schedule %d" % (
                lo, hi, {k: round(v, 3) for k, v in ms_per_sched.items()}, choice), flush=True)
        lo = hi + 1
    w = inst.BATCH_WORKLOADS["batched-512-uniform-n50-500"]
    dists = w.dists()
    wave_ms = {}
    for waves in (1024, 2048, 4096, 8192):
        wave_ms[waves] = _time_batch(dists, table, waves, 3, reps, w.alpha, w.beta, w.rho)
        if verbose:
            print("persistent waves %d: %.3f ms/iteration" % (waves, wave_ms[waves]), flush=True)
    best_waves = min(wave_ms, key=wave_ms.get)
    result = {"arch": "gfx950", "table": table, "persistent_waves": int(best_waves),
              "timings_ms_per_iteration": timings,
              "waves_ms_per_iteration": {str(k): v for k, v in wave_ms.items()},
              "tuned_at": time.strftime("%Y-%m-%d %H:%M:%S")}
    with open(out_path, "w") as f:
        json.dump(result, f, indent=1)
    return result


def refine(workload="batched-512-uniform-n50-500", out_path=DEFAULT_TABLE, start=None, iters=3,
           reps=3, sweeps=2, gain=0.005, verbose=True):
    """Refine a table on one mixed batch instead of per bucket: coordinate
    descent over the buckets the batch uses, each schedule timed on the whole
    batch with the other buckets fixed; a change is kept when it is faster by
    more than `gain` (relative).  Then the persistent-wave count is chosen."""
    import aco_instances as inst

    from . import BATCH_SORTED_MAX_N, SCHEDULES, SORTED_SCHEDULES
    w = inst.BATCH_WORKLOADS[workload]
    dists = w.dists()
    table, waves = start if start is not None else load_table()
    table = [list(e) for e in table]
    waves = waves or 4096
    sizes = sorted({int(d.shape[0]) for d in dists})

    def timed(tab, wv):
        return _time_batch(dists, [tuple(e) for e in tab], wv, iters, reps, w.alpha, w.beta, w.rho)

    used, lo = [], 0
    for i, (hi, _) in enumerate(table):
        if any(lo < n <= hi for n in sizes):
            used.append(i)
        lo = hi
    best = timed(table, waves)
    if verbose:
        print("start: %s, %d waves: %.3f ms/iteration" % (table, waves, best), flush=True)
    for sweep in range(sweeps):
        changed = False
        for i in used:
            # the sorted walk is a candidate wherever the batch allows it
            candidates = SCHEDULES + (SORTED_SCHEDULES if table[i][0] <= BATCH_SORTED_MAX_N else ())
            for sched in candidates:
                if sched == table[i][1]:
                    continue
                trial = [list(e) for e in table]
                trial[i][1] = int(sched)
                ms = timed(trial, waves)
                if verbose:
                    print("  bucket n <= %d, schedule %d: %.3f ms" % (table[i][0], sched, ms), flush=True)
                if ms < best * (1.0 - gain):
                    best, table, changed = ms, trial, True
        if not changed:
            break
    wave_ms = {wv: timed(table, wv) for wv in (2048, 4096, 8192)}
    waves = min(wave_ms, key=wave_ms.get)
    result = {"arch": "gfx950", "table": table, "persistent_waves": int(waves),
              "refined_on": workload, "ms_per_iteration": wave_ms[waves],
              "waves_ms_per_iteration": {str(k): v for k, v in wave_ms.items()},
              "tuned_at": time.strftime("%Y-%m-%d %H:%M:%S")}
    if verbose:
        print("refined: %s, %d waves: %.3f ms/iteration" % (table, waves, wave_ms[waves]), flush=True)
    with open(out_path, "w") as f:
        json.dump(result, f, indent=1)
    return result


def load_table(path=DEFAULT_TABLE):
    """(schedule table as [(n_max, schedule)], persistent waves); ([], 0) if absent."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return [], 0
    return [tuple(e) for e in t["table"]], int(t.get("persistent_waves", 0))


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--per-bucket", type=int, default=48)
    ap.add_argument("--refine-on", default=None,
                    help="refine the current table on this batch workload instead of tuning "
                         "each bucket alone")
    args = ap.parse_args()
    if args.refine_on:
        refine(args.refine_on, args.out)
    else:
        tune(args.out, per_bucket=args.per_bucket)
