"""Runtime of one iteration (construct + update) as the colony and the
instance grow: the stand-in for the paper's runtime experiment (Sec. 3,
"Runtime over scaling population size and scaling city size").

The paper scales the population from 10^0 to 10^4 ants and the city count
over six TSPLIB instances (159 to 2392 cities, m = n), with the elitist
deposit k = n/10, and reports the mean time per iteration.  TSPLIB is not
available here: uniform random cities of the same sizes stand in for the
instances, and the population sweep runs on the 1173-city one.  Each point
is timed for both AdaIR constructs (the full scan and the sorted walk, which
give the same tours).

With TSPLIB files at hand, `--tsplib FILE...` runs the city-size sweep on
them (m = n) and the population sweep on the one closest to 1173 cities.

    python -m paper_2404_04895_amd.scaling [--report FILE] [--quick]
        [--tsplib FILE_OR_DIR ...] [--tsplib-metric euclidean|tsplib]
"""
import argparse
import json
import time

CITY_SIZES = (159, 442, 654, 724, 1173, 2392)
POPULATIONS = (1, 10, 100, 1000, 10000)
POPULATION_N = 1173
SELECTIONS = ("adair", "adair-sorted")


def elite_for(n, m):
    """The paper's k = n/10, or every ant when the colony is not larger."""
    k = n // 10
    return k if 0 < k < m else 0


def iteration_ms(D, m, selection, iters=20, warmup=3, seed=0, alpha=1.0, beta=2.0, rho=0.1):
    """Mean wall time of one iteration (construct + update), in ms."""
    import torch

    from . import Colony
    n = D.shape[0]
    col = Colony(torch.from_numpy(D).cuda(), alpha, beta, rho, 1.0, m,
                 elite_k=elite_for(n, m))
    col.set_selection(selection)
    col.run(m, seed, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    col.run(m, seed, iters)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / iters * 1e3
    col.close()
    return ms


def sweep(sizes=CITY_SIZES, populations=POPULATIONS, population_n=POPULATION_N, iters=20,
          instances=None):
    """{"cities": {n: {selection: {ms_per_iteration, ant_steps_per_s}}},
    "population": {m: ...}, "population_n": n}.  `instances`, a list of
    (label, distance matrix), replaces the uniform stand-ins: the city sweep
    runs on each, the population sweep on the one closest to population_n
    cities (labels key the city sweep then)."""
    import aco_instances as inst

    if instances is None:
        instances = [(n, inst.distance_matrix(inst.uniform_cities(n, 5000 + n))) for n in sizes]
        pop_D = inst.distance_matrix(inst.uniform_cities(population_n, 5000 + population_n))
    else:
        pop_D = min(instances, key=lambda e: abs(e[1].shape[0] - population_n))[1]
        population_n = pop_D.shape[0]
    out = {"cities": {}, "population": {}, "population_n": population_n}
    for label, D in instances:
        n = D.shape[0]
        row = {}
        for sel in SELECTIONS:
            ms = iteration_ms(D, n, sel, iters=iters)
            row[sel] = {"ms_per_iteration": ms, "ant_steps_per_s": n * (n - 1) / ms * 1e3}
        out["cities"][label] = row
    D = pop_D
    for m in populations:
        row = {}
        for sel in SELECTIONS:
            ms = iteration_ms(D, m, sel, iters=iters)
            row[sel] = {"ms_per_iteration": ms,
                        "ant_steps_per_s": m * (population_n - 1) / ms * 1e3}
        out["population"][m] = row
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--report", default=None)
    ap.add_argument("--quick", action="store_true", help="two small sizes, for a smoke run")
    ap.add_argument("--tsplib", nargs="+", default=None,
                    help="TSPLIB files (or directories of *.tsp) instead of the stand-ins")
    ap.add_argument("--tsplib-metric", default="euclidean", choices=["euclidean", "tsplib"],
                    help="distances of TSPLIB instances: plain Euclidean (default) or the "
                         "file's integer metric")
    args = ap.parse_args()
    instances = None
    if args.tsplib:
        from aco_instances import tsplib
        instances = []
        for path in tsplib.instance_files(args.tsplib):
            t = tsplib.read_tsplib(path)
            instances.append((t.name or path, tsplib.distance_matrix(t, args.tsplib_metric)))
    if args.quick:
        res = sweep(sizes=(159, 442), populations=(1, 100), population_n=442, iters=3,
                    instances=instances)
    else:
        res = sweep(instances=instances)
    for part, key in (("cities", "n = m"), ("population", "m (n = %d)" % res["population_n"])):
        for x, row in res[part].items():
            print("%s = %6s: " % (key, x) + "  ".join(
                "%s %.3f ms (%.3g ant-steps/s)" % (s, v["ms_per_iteration"], v["ant_steps_per_s"])
                for s, v in row.items()), flush=True)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
