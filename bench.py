"""Throughput of the tensorized-ACO iteration on one MI355X.

A step is one whole iteration of the hot path over the workload: AdaIR tour
construction for every ant (with tour lengths and successor/predecessor
maps), best-so-far, elite weights, index-mapped deposit, evaporation and the
next transition matrix.  Inputs are resident in HBM before timing starts.

The construct runs the sorted walk by default on instances of 400 cities or
more (--selection adair-sorted).  It picks exactly the AdaIR argmax, bit for
bit, without scoring the cities that provably cannot win.  Its rows are
sorted in the update that builds P, which costs more than the walk saves on
smaller instances; there the default is the full scan (--selection adair),
which scores every unvisited city.

Prints one JSON line.  value = ant-steps per second over the whole iteration
(m * (n-1) per step).  roofline = the construct kernel's algorithmic HBM bytes
per launch over its measured average duration.  For the sorted walk these
bytes are what the kernel reports it read: 6 B per sorted entry, 16 B per
block of a fallback scan, 8 B per step.  roofline_full_scan
= the same for the full scan, timed on the same colony right after.
cpu_baseline = the CPU oracle on a bounded sample of the same workload.
roofline_issue = the same construct launches against the chip's VALU issue
capacity, from committed SQ_INSTS_VALU counts of the same kernel source
(omitted when the source has changed since they were taken).

On the default workload the line also carries the rest of the metric, each
object measured on its own workload after the headline:
  full_run  all 200 iterations of the 5000-city run, one gamma schedule
  batched   512 instances of 50..500 cities, graph replay (its own roofline
            and CPU baseline)
  learned   the learned heuristic against eta = 1/d at equal wall time on
            held-out clustered 2000-city instances (% shorter best tour)
--no-extras leaves them out.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published peak
COUNTERS_FILES = {"adair": os.path.join(ROOT, "profiles", "construct_counters.json"),
                  "adair-sorted": os.path.join(ROOT, "profiles", "construct_sorted_counters.json")}
SORTED_MIN_N = 400     # the sorted walk loses at 159 cities and wins at 442 (m = n)
DEFAULT_WORKLOAD = "clustered-n5000-m5000"
BATCH_WORKLOAD = "batched-512-uniform-n50-500"
# VALU issue capacity: 256 CUs x 4 SIMDs, one wave64 instruction per 4 cycles
# on a 16-lane SIMD, at 2.4 GHz
VALU_ISSUE_PEAK_G = 256 * 4 * 2.4 / 4
SQ_COUNTERS_FILES = {"adair-sorted": os.path.join(ROOT, "profiles",
                                                  "construct_sorted_sq_counters.json")}
KERNEL_SOURCES = ["paper_2404_04895_amd/csrc/construct.hip", "paper_2404_04895_amd/csrc/construct.hpp",
                  "paper_2404_04895_amd/csrc/philox.hpp"]


def default_selection(n):
    """The sorted walk from SORTED_MIN_N cities; below that the per-iteration
    row sort costs more than the scan it saves."""
    return "adair-sorted" if n >= SORTED_MIN_N else "adair"


def construct_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def construct_bytes(n, m):
    """Algorithmic bytes of one construct launch: per ant-step one FP32 row of
    P (4n), the tour entry written (4) and the distance gathered (4)."""
    return m * (n - 1) * (4 * n + 8)


def sorted_walk_bytes(stats, launches, n, m):
    """Algorithmic bytes of one sorted-walk construct launch from the kernel's
    own counts: each sorted entry read is an FP32 value + a uint16 city, each
    fallback block one float4 row slice, and every step writes its tour entry
    and gathers its distance."""
    entries, _, blocks = stats
    return (entries * 6 + blocks * 16) / launches + m * (n - 1) * 8


def counter_traffic(n, m, selection="adair"):
    """HBM traffic per construct launch from committed rocprofv3 counters, or
    None if they were taken on another workload or an older kernel."""
    path = COUNTERS_FILES.get(selection)
    if path is None:
        return None
    try:
        with open(path) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("source_hash") != construct_source_hash() or c.get("n") != n or c.get("m") != m:
        return None
    return c.get("bytes_per_launch")


def issue_rate(n, m, selection, avg_construct_s):
    """VALU issue rate of the construct against the chip's issue capacity,
    from committed SQ_INSTS_VALU counts of the same kernel source and
    workload (None otherwise)."""
    path = SQ_COUNTERS_FILES.get(selection)
    if path is None:
        return None
    try:
        with open(path) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("source_hash") != construct_source_hash() or c.get("n") != n or c.get("m") != m:
        return None
    valu = c["valu_insts_per_launch"]
    achieved = valu / avg_construct_s / 1e9
    return {"bound": "alu", "kernel": c["kernel"], "achieved": achieved,
            "peak": VALU_ISSUE_PEAK_G, "unit": "G VALU wave-instructions/s",
            "frac": achieved / VALU_ISSUE_PEAK_G, "valu_insts_per_launch": valu,
            "valu_insts_per_ant_step": valu / (m * (n - 1)),
            "counters": os.path.relpath(path, ROOT)}


def cpu_baseline(w, D, P, budget_s=15.0):
    """The oracle as it is, on this host: construct for a sample of ants from
    one P, plus one full update (deposit, evaporation, transition), scaled to
    ant-steps per second of a whole iteration.  The sample grows by four ants
    per thread at a time until about budget_s seconds of construction."""
    import numpy as np

    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    oracle.construct(P, D, 1, 0, np.arange(threads))   # first call: thread start-up
    chunk = 4 * threads
    parts_t, parts_l = [], []
    count, t_construct = 0, 0.0
    while count < w.m and t_construct < budget_s:
        ants = np.arange(count, min(w.m, count + chunk))
        t0 = time.perf_counter()
        tc, lc = oracle.construct(P, D, 1, 0, ants)
        t_construct += time.perf_counter() - t0
        parts_t.append(tc)
        parts_l.append(lc)
        count += len(ants)
    tours = np.concatenate(parts_t)
    lengths = np.concatenate(parts_l)
    # a full update on tours of the sample (the update's cost does not depend on which ants)
    reps = int(np.ceil(w.m / count))
    all_tours = np.tile(tours, (reps, 1))[:w.m]
    all_len = np.tile(lengths, reps)[:w.m]
    S = oracle.deposit_scale(D, w.m, w.Q)
    tau = np.where(np.eye(w.n, dtype=bool), 0, np.float32(w.tau0)).astype(np.float32)
    t0 = time.perf_counter()
    delta = oracle.deposit(all_tours, all_len, None, w.Q, S)
    tau = oracle.evaporate(tau, delta, w.rho, S)
    oracle.transition(tau, D, w.alpha, w.beta, 1.5)
    t_update = time.perf_counter() - t0
    t_iter = t_construct * (w.m / count) + t_update
    return {
        "value": w.m * (w.n - 1) / t_iter,
        "unit": "ant-steps/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "construct of %d of %d ants (%.1f s) from one P, plus one full update "
                  "(%.1f s), scaled to one whole iteration" % (count, w.m, t_construct, t_update),
    }


def cpu_baseline_batch(w, dists, budget_s=15.0):
    """The oracle on whole iterations of a sample of the batch's instances."""
    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    steps, spent, used = 0, 0.0, 0
    for i, D in enumerate(dists):
        n = D.shape[0]
        t0 = time.perf_counter()
        oracle.run(D, n, w.alpha, w.beta, w.rho, w.Q, i, 2)
        spent += time.perf_counter() - t0
        steps += 2 * n * (n - 1)
        used += 1
        if spent > budget_s:
            break
    return {
        "value": steps / spent,
        "unit": "ant-steps/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "2 whole iterations of each of the first %d of %d instances (%.1f s)" % (
            used, len(dists), spent),
    }


def bench_batch(args, w, cpu_budget_s=15.0):
    """The batched workload: `args.steps` iterations of every instance, graph
    replay, timed whole; then as many again with each construct launch timed."""
    import numpy as np
    import torch

    from paper_2404_04895_amd import SCHED_SORTED, Batch, autotune

    dists = w.dists()
    ns = np.array([d.shape[0] for d in dists], dtype=np.int64)
    table, waves = autotune.load_table()
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = Batch(dists, w.alpha, w.beta, w.rho, w.Q, stream=stream)
        b.set_schedules(table, waves)
        if args.warmup:
            b.run(args.warmup)
        stream.synchronize()
        t0 = time.perf_counter()
        b.run(args.steps, use_graph=True)
        stream.synchronize()
        elapsed = time.perf_counter() - t0
        lens, _, _ = b.best()
        sorted_member = np.array([b.view(i).schedule & SCHED_SORTED != 0 for i in range(len(ns))])
        b.sorted_walk_stats()  # reset the counts
        b.run(args.steps, use_graph=False, time_construct=True)
        construct_ms, launches = b.construct_time()
        walk = b.sorted_walk_stats()
        b.close()
    stream.synchronize()
    ant_steps = int((ns * (ns - 1)).sum())
    # full-scan members read whole rows; sorted-walk members what their walks
    # counted (as for one instance), plus their tour writes and distance gathers
    full = ~sorted_member
    entries, _, blocks = walk
    bytes_launch = int((ns[full] * (ns[full] - 1) * (4 * ns[full] + 8)).sum()) + int(
        (entries * 6 + blocks * 16) / launches) + int(
        (ns[sorted_member] * (ns[sorted_member] - 1) * 8).sum())
    avg_construct_s = construct_ms / launches / 1e3
    achieved = bytes_launch / avg_construct_s / 1e9
    line = {
        "metric": "ant-steps/sec & % HBM peak; learned-vs-plain best-tour gap at equal time",
        "value": ant_steps * args.steps / elapsed,
        "unit": "ant-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "instances": w.count, "n": [w.n_lo, w.n_hi],
                   "m": "n", "alpha": w.alpha, "beta": w.beta, "rho": w.rho, "Q": w.Q,
                   "cities": "uniform", "schedule_table": table, "persistent_waves": waves,
                   "graph": True},
        "roofline": {"bound": "hbm", "kernel": "batch_construct_kernel", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_launch": bytes_launch,
                     "avg_launch_ms": avg_construct_s * 1e3},
        "construct_ant_steps_per_s": ant_steps / avg_construct_s,
        "mean_best_len": float(np.mean(lens)),
        "sorted_walk_members": int(sorted_member.sum()),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_batch(w, dists, budget_s=cpu_budget_s)
    return line


def bench_learned(args, count):
    """Learned eta against eta = 1/d at equal wall time on held-out clustered
    n = 2000 instances (30 Gaussians, sigma 0.015), m = n, 300 iterations."""
    import numpy as np

    from paper_2404_04895_amd import learned

    master = learned.load_weights()
    if master is None:
        raise SystemExit("no trained weights")
    kappa, lam = learned.heuristic_config()
    count = max(1, count)
    rows = learned.equal_time_comparison(learned.evaluation_instances(count), [0], master,
                                         kappa=kappa, lam=lam, verbose=False)
    gaps = np.array([r["gap"] for r in rows])
    line = {
        "metric": "ant-steps/sec & % HBM peak; learned-vs-plain best-tour gap at equal time",
        "value": 100.0 * float(gaps.mean()),
        "unit": "% shorter best tour (learned vs plain, equal wall time)",
        "n_gpus": 1,
        "steps": count,
        "warmup": 0,
        "ms_per_step": 1e3 * float(np.mean([r["plain_s"] for r in rows])),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "learned-clustered-n2000", "instances": count, "n": 2000,
                   "m": 2000, "iters": 300, "alpha": 1.0, "beta": 2.0, "rho": 0.1,
                   "cities": "clustered, 30 Gaussians sigma 0.015", "kappa": kappa,
                   "lambda": lam},
        "min_gap_percent": 100.0 * float(gaps.min()),
        "better_runs": int((gaps > 0).sum()),
        "target_percent": 2.0,
        "runs": [{k: r[k] for k in ("instance", "plain_len", "learned_len", "gap", "plain_s",
                                    "learned_s", "learned_iters")} for r in rows],
    }
    return line


def bench_full_run(w, seed, selection):
    """All `w.iters` iterations of the workload on a fresh colony, as one run
    (the gamma schedule over the whole run): wall time per iteration, and the
    construct launches timed by HIP events on the colony's stream."""
    import torch

    from paper_2404_04895_amd import Colony, gamma_schedule

    D = w.dist(seed)
    dev = torch.device("cuda:0")
    col = Colony(torch.from_numpy(D).to(dev), w.alpha, w.beta, w.rho, w.Q, w.m, tau0=w.tau0,
                 elite_k=w.elite_k, gamma_max=w.gamma_max, gamma_min=w.gamma_min)
    col.set_selection(selection)
    stream = torch.cuda.current_stream()
    T = w.iters
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(T)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    col.transition(gamma_schedule(0, T, w.gamma_max, w.gamma_min))
    for t in range(T):
        events[t][0].record(stream)
        col.construct(w.m, seed, t)
        events[t][1].record(stream)
        col.update(gamma_schedule(t + 1, T, w.gamma_max, w.gamma_min))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    construct_ms = [a.elapsed_time(b) for a, b in events]
    _, best_len, best_iter = col.best()
    col.close()
    quarter = max(1, T // 4)
    return {
        "iterations": T,
        "selection": selection,
        "ms_per_iteration": elapsed / T * 1e3,
        "ant_steps_per_s": w.m * (w.n - 1) * T / elapsed,
        "construct_ms_mean": sum(construct_ms) / T,
        "construct_ms_by_quarter": [sum(construct_ms[q * quarter:(q + 1) * quarter]) / quarter
                                    for q in range(4)],
        "best_len": best_len,
        "best_iter": best_iter,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--selection", default=None,
                    choices=["adair", "adair-sorted", "roulette"],
                    help="per-step selection rule of the construct (default: adair-sorted "
                         "from %d cities, adair below)" % SORTED_MIN_N)
    ap.add_argument("--no-full-scan-reference", action="store_true",
                    help="skip the full-scan reference timing after the sorted walk")
    ap.add_argument("--schedule", type=int, default=None,
                    help="construct schedule code (ACO_SCHED_*); default: by size")
    ap.add_argument("--elite-k", type=int, default=None,
                    help="deposit from the k shortest tours only (the paper uses n/10)")
    ap.add_argument("--tau-min", type=float, default=0.0, help="MAX-MIN lower bound on tau")
    ap.add_argument("--tau-max", type=float, default=float("inf"),
                    help="MAX-MIN upper bound on tau")
    ap.add_argument("--walk", type=int, default=None,
                    help="sorted batches per step before the scan (adair-sorted)")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline workload: no full run, batched or learned objects")
    ap.add_argument("--learned-instances", type=int, default=10,
                    help="held-out instances of the learned-vs-plain comparison")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB before timing (a "
                         "reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the method is measured on one GPU's "
              "share; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import aco_instances as inst
    from paper_2404_04895_amd import Colony, gamma_schedule

    if args.workload in inst.BATCH_WORKLOADS:
        print(json.dumps(bench_batch(args, inst.BATCH_WORKLOADS[args.workload])), flush=True)
        return
    if args.workload == "learned-clustered-n2000":
        print(json.dumps(bench_learned(args, args.steps)), flush=True)
        return
    w = inst.WORKLOADS[args.workload]
    n, m, T = w.n, w.m, w.iters
    if args.selection is None:
        args.selection = default_selection(n)
    D = w.dist(args.seed)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    elite_k = w.elite_k if args.elite_k is None else args.elite_k
    col = Colony(torch.from_numpy(D).to(dev), w.alpha, w.beta, w.rho, w.Q, m, tau0=w.tau0,
                 elite_k=elite_k, gamma_max=w.gamma_max, gamma_min=w.gamma_min)
    col.set_tau_bounds(args.tau_min, args.tau_max)
    col.set_selection(args.selection)
    if args.walk is not None:
        col.set_sorted_walk(args.walk)
    if args.schedule is not None:
        col.set_schedule(args.schedule)
    stream = torch.cuda.current_stream()

    def step(t, ev=None):
        if ev is not None:
            ev[0].record(stream)
        col.construct(m, args.seed, t)
        if ev is not None:
            ev[1].record(stream)
        col.update(gamma_schedule(t + 1, T, w.gamma_max, w.gamma_min))

    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    col.transition(gamma_schedule(0, T, w.gamma_max, w.gamma_min))
    for t in range(args.warmup):
        step(t)
    torch.cuda.synchronize()

    sorted_walk = args.selection == "adair-sorted"
    if sorted_walk:
        col.sorted_walk_stats()  # reset the counts
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(args.warmup + k, events[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    construct_ms = [a.elapsed_time(b) for a, b in events]
    avg_construct_s = sum(construct_ms) / len(construct_ms) / 1e3
    ms_per_step = elapsed / args.steps * 1e3
    ant_steps = m * (n - 1)
    value = ant_steps * args.steps / elapsed
    walk = None
    if sorted_walk:
        stats = col.sorted_walk_stats()
        bytes_launch = sorted_walk_bytes(stats, args.steps, n, m)
        walk = {"entries_per_step": stats[0] / (args.steps * ant_steps),
                "scanned_step_fraction": stats[1] / (args.steps * ant_steps),
                "blocks_per_scanned_step": stats[2] / max(stats[1], 1)}
    else:
        bytes_launch = construct_bytes(n, m)
    achieved = bytes_launch / avg_construct_s / 1e9
    traffic = counter_traffic(n, m, args.selection)
    _, best_len, best_iter = col.best()

    reference = None
    if sorted_walk and not args.no_full_scan_reference:
        # the full scan on the same colony, continuing the same run, on the
        # schedule the library picks for it
        col.set_selection("adair")
        col.set_schedule(-1)
        k2 = min(args.steps, 5)
        ev2 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(k2)]
        for k in range(k2):
            step(args.warmup + args.steps + k, ev2[k])
        torch.cuda.synchronize()
        ref_s = sum(a.elapsed_time(b) for a, b in ev2) / k2 / 1e3
        ref_bytes = construct_bytes(n, m)
        reference = {"bound": "hbm", "kernel": "construct_kernel (full scan)",
                     "achieved": ref_bytes / ref_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ref_bytes / ref_s / 1e9 / HBM_PEAK_GBS,
                     "traffic": counter_traffic(n, m, "adair"), "bytes_per_launch": ref_bytes,
                     "avg_launch_ms": ref_s * 1e3, "launches": k2}

    line = {
        "metric": "ant-steps/sec & % HBM peak; learned-vs-plain best-tour gap at equal time",
        "value": value,
        "unit": "ant-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "m": m, "alpha": w.alpha, "beta": w.beta,
                   "rho": w.rho, "Q": w.Q, "cities": "%s, %d Gaussians sigma %g" % (
                       w.family, w.clusters, w.sigma) if w.family != "uniform" else "uniform",
                   "gamma": [w.gamma_max, w.gamma_min], "seed": args.seed,
                   "selection": args.selection, "elite_k": elite_k,
                   "tau_bounds": [args.tau_min, args.tau_max]},
        "roofline": {"bound": "hbm",
                     "kernel": "construct_kernel (sorted walk)" if sorted_walk else "construct_kernel",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": bytes_launch, "avg_launch_ms": avg_construct_s * 1e3},
        "construct_ant_steps_per_s": ant_steps / avg_construct_s,
        "best_len": best_len,
    }
    if walk is not None:
        line["sorted_walk"] = walk
    if reference is not None:
        line["roofline_full_scan"] = reference
    issue = issue_rate(n, m, args.selection, avg_construct_s)
    if issue is not None:
        line["roofline_issue"] = issue
    # the oracle's sample reads P from the host; copied only now, so that no
    # idle gap sits between the warm-up and the timed steps
    P_host = col.P().cpu().numpy() if not args.no_cpu_baseline else None
    col.close()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, D, P_host)
    if not args.no_extras and w.name == DEFAULT_WORKLOAD:
        # the rest of the metric, on the other workloads it is quoted on
        line["full_run"] = bench_full_run(w, args.seed, args.selection)
        print("full run done", file=sys.stderr, flush=True)
        line["batched"] = bench_batch(args, inst.BATCH_WORKLOADS[BATCH_WORKLOAD],
                                      cpu_budget_s=8.0)
        print("batched done", file=sys.stderr, flush=True)
        line["learned"] = bench_learned(args, args.learned_instances)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
