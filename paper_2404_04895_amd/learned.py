"""Training and evaluation of the learned edge heuristic.

Training data: plain runs (eta = 1/d) of the method on clustered instances,
run together on the batched engine; the converged pheromone of each instance
gives the targets y_ij = tau_ij / max_k tau_ik of its edges, and the edge
features come from the distances and kNN ranks.  Training keeps the edges
within 32 nearest neighbours of either end plus 5% of the rest.  The edge MLP
is trained on the GPU (minibatch Adam, 20000 steps of 16384 edges) with the
library's own forward, backward and Adam kernels.  Evaluation: the plain method against the same method with the
learned eta, at equal wall time (the learned arm pays for ranks and inference
out of its iteration budget), judged by the best tour length.

    python -m paper_2404_04895_amd.learned train [--out FILE]
    python -m paper_2404_04895_amd.learned evaluate [--weights FILE]
    python -m paper_2404_04895_amd.learned profile [--reps K]
"""
import argparse
import json
import math
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "edge_mlp_clustered_n500.npy")


def init_params(seed=0):
    """He-style initial parameters (FP32, in the ABI's parameter order)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(4481, np.float32)
    p[0:192] = rng.standard_normal(192) * math.sqrt(2.0 / 3.0)
    p[256:4352] = rng.standard_normal(4096) * math.sqrt(2.0 / 64.0)
    p[4416:4480] = rng.standard_normal(64) * math.sqrt(1.0 / 64.0)
    p[4480] = -3.0  # most edges are not in a converged tour
    return p


def training_set(count=200, n=500, clusters=20, sigma=0.02, seed0=1000, iters=300, alpha=1.0,
                 beta=2.0, rho=0.1, runs=1, verbose=True):
    """Features (N x 3) and targets (N) on the device from plain batched runs.
    With runs > 1 each instance is run with `runs` generator seeds and its
    targets are the mean of the runs' targets."""
    import torch

    import aco_instances as inst
    from . import Batch, autotune, edge_ranks, mlp_features, mlp_targets

    seeds = list(range(seed0, seed0 + count))
    dists = [inst.distance_matrix(inst.clustered_cities(n, s, clusters, sigma)) for s in seeds]
    table, waves = autotune.load_table()
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        b = Batch(dists * runs, alpha, beta, rho, 1.0, ants=[n] * (count * runs),
                  seeds=[s + 100000 * r for r in range(runs) for s in seeds], stream=stream)
        b.set_schedules(table, waves)
        b.run(iters)
        feats, ys = [], []
        for i, D in enumerate(dists):
            rank, _, mean = edge_ranks(D, stream)
            feats.append(mlp_features(D, rank, mean, stream))
            y = None
            for r in range(runs):
                v = b.view(i + r * count)
                tau = b._dev(v.tau, torch.float32, (v.n, v.ld))
                yr = mlp_targets(tau, n, stream)
                y = yr if y is None else y + yr
            ys.append(y / runs)
        feats = torch.cat(feats)
        y = torch.cat(ys)
        b.close()
    stream.synchronize()
    if verbose:
        print("training set: %d instances x %d edges in %.1f s (plain runs of %d iterations)" % (
            count, n * (n - 1), time.perf_counter() - t0, iters), flush=True)
    return feats, y


def emphasise_near(feats, y, radius=32, far_fraction=0.05, seed=0):
    """The training edges that matter for construction: every edge within
    `radius` nearest neighbours of either end city, plus a random
    `far_fraction` of the rest (so the network still sees far edges).  An ant
    chooses almost always among near neighbours, and the converged targets
    are almost all zero beyond them."""
    import torch
    g = torch.Generator(device=feats.device)
    g.manual_seed(seed)
    thr = math.log2(1 + radius) + 1e-6
    near = (feats[:, 1] <= thr) | (feats[:, 2] <= thr)
    keep = near | (torch.rand(feats.shape[0], device=feats.device, generator=g) < far_fraction)
    return feats[keep].contiguous(), y[keep].contiguous()


def train(feats, y, steps=20000, batch=16384, lr=1e-3, seed=0, init_seed=0, verbose=True):
    import torch

    from . import MlpTrainer
    t = MlpTrainer(init_params(init_seed), batch)
    curve = []
    t0 = time.perf_counter()
    for k in range(steps):
        t.step(feats, y, seed, lr)
        if verbose and (k % 500 == 0 or k == steps - 1):
            curve.append((k, t.loss()))
            print("step %d: minibatch loss %.5f" % curve[-1], flush=True)
    torch.cuda.synchronize()
    master, eff = t.params()
    elapsed = time.perf_counter() - t0
    t.close()
    return master.cpu().numpy(), eff.cpu().numpy(), curve, elapsed


def save_weights(master, path=DEFAULT_WEIGHTS):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.save(path, np.asarray(master, np.float32), allow_pickle=False)


def load_weights(path=DEFAULT_WEIGHTS):
    """FP32 master parameters (ACO_MLP_PARAMS,), or None if there are none."""
    if not os.path.exists(path):
        return None
    p = np.load(path, allow_pickle=False)
    return p.astype(np.float32) if p.shape == (4481,) else None


DEFAULT_KAPPA, DEFAULT_LAMBDA = 1.4, 1.0


def heuristic_config(path=DEFAULT_WEIGHTS):
    """(kappa, lambda) stored beside the weights by the validation sweep."""
    cfg = path.replace(".npy", ".json")
    try:
        with open(cfg) as f:
            c = json.load(f)
        return float(c["kappa"]), float(c["lambda"])
    except (OSError, ValueError, KeyError):
        return DEFAULT_KAPPA, DEFAULT_LAMBDA


def learned_eta(dist, master, kappa=DEFAULT_KAPPA, lam=DEFAULT_LAMBDA, stream=None):
    """(eta = sigmoid(z)^kappa / (d/dNN)^lam from the network, count of bad outputs)."""
    from . import mlp_eta, mlp_round
    eta, bad = mlp_eta(mlp_round(master, stream), dist, stream=stream, kappa=kappa, lam=lam)
    return eta, int(bad.item())


def equal_time_comparison(dists, run_seeds, master, iters=300, alpha=1.0, beta=2.0, rho=0.1,
                          kappa=DEFAULT_KAPPA, lam=DEFAULT_LAMBDA, verbose=True):
    """Plain (eta = 1/d, `iters` iterations) against learned eta within the
    plain arm's wall time, per instance and run seed."""
    import torch

    from . import Colony
    rows = []
    for k, D in enumerate(dists):
        n = D.shape[0]
        dev = torch.from_numpy(D).cuda()
        for seed in run_seeds:
            col = Colony(dev, alpha, beta, rho, 1.0, n)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, L_plain = col.run(n, seed, iters)
            t_plain = time.perf_counter() - t0
            col.close()
            col = Colony(dev, alpha, beta, rho, 1.0, n)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            eta, bad = learned_eta(dev, master, kappa, lam)
            active = col.set_eta(eta)
            torch.cuda.synchronize()
            t_inf = time.perf_counter() - t0
            budget = max(1, int((t_plain - t_inf) / (t_plain / iters)))
            budget = min(budget, iters)
            _, L_learned = col.run(n, seed, budget)
            t_learned = time.perf_counter() - t0
            col.close()
            gap = (L_plain - L_learned) / L_plain
            rows.append({"instance": k, "seed": seed, "n": n, "plain_len": L_plain,
                         "learned_len": L_learned, "gap": gap, "plain_s": t_plain,
                         "learned_s": t_learned, "inference_s": t_inf,
                         "learned_iters": budget, "eta_active": bool(active),
                         "nonfinite": bad})
            if verbose:
                print("instance %d seed %d: plain %.4f (%.2f s)  learned %.4f (%.2f s, %d it)  "
                      "gap %+.2f%%" % (k, seed, L_plain, t_plain, L_learned, t_learned, budget,
                                       100 * gap), flush=True)
    return rows


def validate_heuristic(master, kappas=(0.7, 1.0, 1.4, 2.0, 2.8), lams=(DEFAULT_LAMBDA,),
                       count=6, seeds=(0, 1, 2), iters=300, verbose=True):
    """Choose (kappa, lambda) on validation instances (clustered n = 2000,
    instance seeds 3000 on, never the evaluation seeds) by the mean relative
    gap to the plain method over the same iteration count.  The runs use the
    sorted walk, which builds the same tours as the full scan, only faster."""
    import torch

    from . import Colony
    dists = evaluation_instances(count, seed0=3000)
    grid = [(k, l) for k in kappas for l in lams]
    gaps = {kl: [] for kl in grid}
    for i, D in enumerate(dists):
        dev = torch.from_numpy(D).cuda()
        n = D.shape[0]
        for seed in seeds:
            col = Colony(dev, 1.0, 2.0, 0.1, 1.0, n)
            col.set_selection("adair-sorted")
            _, L_plain = col.run(n, seed, iters)
            col.close()
            for k, l in grid:
                col = Colony(dev, 1.0, 2.0, 0.1, 1.0, n)
                col.set_selection("adair-sorted")
                eta, _ = learned_eta(dev, master, k, l)
                col.set_eta(eta)
                _, L = col.run(n, seed, iters)
                col.close()
                gaps[(k, l)].append((L_plain - L) / L_plain)
        if verbose:
            print("validation instance %d of %d done" % (i + 1, len(dists)), flush=True)
    means = {kl: float(np.mean(v)) for kl, v in gaps.items()}
    if verbose:
        for k, l in grid:
            print("validation kappa %.2f lambda %.2f: mean gap %+.2f%% over %d runs" % (
                k, l, 100 * means[(k, l)], len(gaps[(k, l)])), flush=True)
    return max(means, key=means.get), means


def evaluation_instances(count=10, n=2000, clusters=30, sigma=0.015, seed0=2000):
    import aco_instances as inst
    return [inst.distance_matrix(inst.clustered_cities(n, s, clusters, sigma))
            for s in range(seed0, seed0 + count)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["train", "validate", "evaluate", "profile"])
    ap.add_argument("--reps", type=int, default=6, help="inference repetitions (profile)")
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--weights", default=DEFAULT_WEIGHTS)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--radius", type=int, default=32,
                    help="train on edges within this many nearest neighbours (0: all edges)")
    ap.add_argument("--instances", type=int, default=10)
    ap.add_argument("--seeds", type=int, default=3)
    ap.add_argument("--report", default=None)
    ap.add_argument("--record", action="store_true",
                    help="evaluate: store the summary beside the weights")
    ap.add_argument("--train-iters", type=int, default=300)
    ap.add_argument("--runs", type=int, default=1)
    ap.add_argument("--kappas", default="0.7,1.0,1.4,2.0,2.8",
                    help="validate: exponents of the network's output to try")
    ap.add_argument("--lambdas", default="1.0",
                    help="validate: exponents of the scaled inverse distance to try")
    args = ap.parse_args()
    if args.mode == "train":
        feats, y = training_set(iters=args.train_iters, runs=args.runs)
        if args.radius > 0:
            feats, y = emphasise_near(feats, y, radius=args.radius)
        master, _, curve, secs = train(feats, y, steps=args.steps)
        save_weights(master, args.out)
        print("trained in %.1f s; weights -> %s" % (secs, args.out), flush=True)
        if args.report:
            with open(args.report, "w") as f:
                json.dump({"curve": curve, "seconds": secs, "edges": int(y.numel())}, f)
    elif args.mode == "validate":
        master = load_weights(args.weights)
        assert master is not None, "no weights at " + args.weights
        kappas = [float(x) for x in args.kappas.split(",")]
        lams = [float(x) for x in args.lambdas.split(",")]
        (kappa, lam), means = validate_heuristic(master, kappas, lams)
        # the choice and the grid go beside the weights; other records there stay
        cfg_path = args.weights.replace(".npy", ".json")
        try:
            with open(cfg_path) as f:
                cfg = json.load(f)
        except (OSError, ValueError):
            cfg = {}
        cfg.update({"kappa": kappa, "lambda": lam,
                    "validation_mean_gap": {"%g,%g" % kl: v for kl, v in means.items()}})
        with open(cfg_path, "w") as f:
            json.dump(cfg, f, indent=1)
        print("chose kappa %.2f lambda %.2f" % (kappa, lam), flush=True)
    elif args.mode == "profile":
        # inference alone (ranks, features, network, eta) on the first held-out instance
        import torch
        master = load_weights(args.weights)
        assert master is not None, "no weights at " + args.weights
        kappa, lam = heuristic_config(args.weights)
        dev = torch.from_numpy(evaluation_instances(1)[0]).cuda()
        for _ in range(args.reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, bad = learned_eta(dev, master, kappa, lam)
            torch.cuda.synchronize()
            print("inference %.3f ms, %d non-finite" % ((time.perf_counter() - t0) * 1e3, bad),
                  flush=True)
    else:
        master = load_weights(args.weights)
        assert master is not None, "no weights at " + args.weights
        kappa, lam = heuristic_config(args.weights)
        rows = equal_time_comparison(evaluation_instances(args.instances),
                                     list(range(args.seeds)), master, kappa=kappa, lam=lam)
        gaps = np.array([r["gap"] for r in rows])
        print("mean gap %+.2f%% (min %+.2f%%, max %+.2f%%) over %d runs" % (
            100 * gaps.mean(), 100 * gaps.min(), 100 * gaps.max(), len(rows)), flush=True)
        if args.report:
            with open(args.report, "w") as f:
                json.dump(rows, f, indent=1)
        if args.record:
            cfg_path = args.weights.replace(".npy", ".json")
            with open(cfg_path) as f:
                cfg = json.load(f)
            cfg["held_out_equal_time"] = {
                "mean_gap": float(gaps.mean()), "min_gap": float(gaps.min()),
                "max_gap": float(gaps.max()), "better": int((gaps > 0).sum()),
                "runs": len(rows), "kappa": kappa, "lambda": lam,
                "instances": "clustered n = 2000, seeds 2000-%d x run seeds 0-%d" % (
                    2000 + args.instances - 1, args.seeds - 1)}
            with open(cfg_path, "w") as f:
                json.dump(cfg, f, indent=1)


if __name__ == "__main__":
    main()
