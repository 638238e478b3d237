"""Ablation of the selection rule: Roulette Wheel (RW), Independent Roulette
(IR, argmax of P * r with gamma = 1) and AdaIR (the cosine gamma schedule),
the comparison of Sec. 3's "Ablation Study on AdaIR".

Runtime: wall time per iteration (construct + update) for each rule on
uniform instances of the six sizes the paper's runtime figure uses (m = n).
The paper uses TSPLIB instances of these sizes, which are not available here;
uniform random cities of the same size stand in for them.

Convergence: best-so-far tour length per iteration over 1000 iterations,
five repeats (run seeds 0-4), m = 500 ants, on one uniform instance.  The
convergence generation of a run is the first iteration whose best-so-far is
within 0.1% of the run's final best.

The paper names cosine annealing for gamma but no constants, so the
convergence part also runs AdaIR under other schedules (gamma at the first
iteration -> gamma at the last), greedier than IR where gamma < 1: the
default 1.5 -> 1.0, 1.5 -> 0.5, 1.0 -> 0.5, the reverse 0.5 -> 1.0, and a
constant 1.5.  Every schedule runs the same kernels; only P's exponent 1/gamma
changes.

With TSPLIB files at hand, `--tsplib FILE...` times the runtime part on them
instead of the uniform stand-ins, and `--convergence-tsplib FILE` runs the
convergence part on that instance (the paper's has 442 cities).

    python -m paper_2404_04895_amd.ablation [--report FILE] [--quick] [--convergence-only]
        [--tsplib FILE_OR_DIR ...] [--convergence-tsplib FILE] [--tsplib-metric euclidean|tsplib]
"""
import argparse
import json
import time

import numpy as np

RULES = {
    "RW": dict(selection="roulette", gamma_max=1.0, gamma_min=1.0),
    "IR": dict(selection="adair", gamma_max=1.0, gamma_min=1.0),
    "AdaIR": dict(selection="adair", gamma_max=1.5, gamma_min=1.0),
}
# AdaIR under other gamma schedules (first -> last iteration): convergence only
SCHEDULE_VARIANTS = {
    "AdaIR 1.5->0.5": dict(selection="adair", gamma_max=1.5, gamma_min=0.5),
    "AdaIR 1.0->0.5": dict(selection="adair", gamma_max=1.0, gamma_min=0.5),
    "AdaIR 0.5->1.0": dict(selection="adair", gamma_max=0.5, gamma_min=1.0),
    "AdaIR 1.5 const": dict(selection="adair", gamma_max=1.5, gamma_min=1.5),
}
# AdaIR's exact sorted walk: the same tours as "AdaIR", so it is timed but its
# convergence is AdaIR's
TIMED_ONLY = {"AdaIR-sorted": dict(selection="adair-sorted", gamma_max=1.5, gamma_min=1.0)}
RUNTIME_SIZES = (159, 442, 654, 724, 1173, 2392)


def _colony(D, rule, m, alpha=1.0, beta=2.0, rho=0.1):
    import torch

    from . import Colony
    spec = RULES.get(rule) or SCHEDULE_VARIANTS.get(rule) or TIMED_ONLY[rule]
    col = Colony(torch.from_numpy(D).cuda(), alpha, beta, rho, 1.0, m,
                 gamma_max=spec["gamma_max"], gamma_min=spec["gamma_min"])
    col.set_selection(spec["selection"])
    return col


def iteration_times(D, m, iters=20, warmup=3, seed=0):
    """Mean ms per iteration (construct + update) for each rule."""
    import torch
    out = {}
    for rule in list(RULES) + list(TIMED_ONLY):
        col = _colony(D, rule, m)
        col.run(m, seed, warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        col.run(m, seed, iters)
        torch.cuda.synchronize()
        out[rule] = (time.perf_counter() - t0) / iters * 1e3
        col.close()
    return out


def best_so_far_curve(D, rule, m, iters, seed):
    """Best-so-far length after each iteration (one device sync at the end)."""
    import torch

    from . import gamma_schedule
    col = _colony(D, rule, m)
    spec = RULES.get(rule) or SCHEDULE_VARIANTS[rule]
    g = lambda t: gamma_schedule(t, iters, spec["gamma_max"], spec["gamma_min"])
    col.transition(g(0))
    mins = []
    for t in range(iters):
        col.construct(m, seed, t)
        mins.append(col.lengths(m).min())
        col.update(g(t + 1))
    curve = np.minimum.accumulate(torch.stack(mins).cpu().numpy().astype(np.float64))
    col.close()
    return curve


def convergence_generation(curve, tol=1e-3):
    return int(np.argmax(curve <= curve[-1] * (1 + tol)))


def main():
    import aco_instances as inst

    ap = argparse.ArgumentParser()
    ap.add_argument("--report", default=None)
    ap.add_argument("--quick", action="store_true", help="fewer iterations, for a smoke run")
    ap.add_argument("--convergence-only", action="store_true", help="skip the runtime part")
    ap.add_argument("--tsplib", nargs="+", default=None,
                    help="TSPLIB files (or directories of *.tsp) for the runtime part")
    ap.add_argument("--convergence-tsplib", default=None,
                    help="TSPLIB file for the convergence part")
    ap.add_argument("--tsplib-metric", default="euclidean", choices=["euclidean", "tsplib"],
                    help="distances of TSPLIB instances: plain Euclidean (default) or the "
                         "file's integer metric")
    args = ap.parse_args()
    iters, repeats = (200, 2) if args.quick else (1000, 5)
    report = {"runtime_ms_per_iteration": {}, "convergence": {}}
    if args.tsplib:
        from aco_instances import tsplib
        runtime = []
        for path in tsplib.instance_files(args.tsplib):
            t = tsplib.read_tsplib(path)
            runtime.append((t.name or path, tsplib.distance_matrix(t, args.tsplib_metric)))
    else:
        runtime = [(n, None) for n in RUNTIME_SIZES]
    for label, D in (() if args.convergence_only else runtime):
        if D is None:
            D = inst.distance_matrix(inst.uniform_cities(label, 5000 + label))
        n = D.shape[0]
        times = iteration_times(D, n)
        times["speedup_AdaIR_over_RW"] = times["RW"] / times["AdaIR"]
        times["speedup_AdaIR_sorted_over_RW"] = times["RW"] / times["AdaIR-sorted"]
        report["runtime_ms_per_iteration"][label] = times
        print("%s: n=%d m=%d: " % (label, n, n) + "  ".join(
            "%s %.3f ms" % (k, v) for k, v in times.items() if not k.startswith("speedup")) +
            "  RW/AdaIR %.2fx  RW/AdaIR-sorted %.2fx" % (
                times["speedup_AdaIR_over_RW"], times["speedup_AdaIR_sorted_over_RW"]), flush=True)
    if args.convergence_tsplib:
        from aco_instances import tsplib
        D = tsplib.distance_matrix(tsplib.read_tsplib(args.convergence_tsplib),
                                   args.tsplib_metric)
        report["convergence_instance"] = args.convergence_tsplib
    else:
        D = inst.distance_matrix(inst.uniform_cities(442, 5442))
    n_conv, m_conv = D.shape[0], 500
    for rule in list(RULES) + list(SCHEDULE_VARIANTS):
        curves = [best_so_far_curve(D, rule, m_conv, iters, s) for s in range(repeats)]
        gens = [convergence_generation(c) for c in curves]
        finals = [float(c[-1]) for c in curves]
        spec = RULES.get(rule) or SCHEDULE_VARIANTS[rule]
        report["convergence"][rule] = {
            "gamma_first": spec["gamma_max"], "gamma_last": spec["gamma_min"],
            "n": n_conv, "m": m_conv, "iterations": iters, "repeats": repeats,
            "generation": gens, "final_best": finals,
            "mean_generation": float(np.mean(gens)), "mean_final_best": float(np.mean(finals)),
            "curve_mean_every_50": [float(v) for v in np.mean(curves, axis=0)[::50]],
        }
        print("%s: converged at generation %.0f (mean of %s), final best %.4f (min %.4f max %.4f)"
              % (rule, np.mean(gens), gens, np.mean(finals), min(finals), max(finals)), flush=True)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)


if __name__ == "__main__":
    main()
