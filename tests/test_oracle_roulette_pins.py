"""Pins of the oracle's Roulette Wheel (RW) selection, the proportional rule
that the Independent Roulette of Sec. 2.4 replaces and that the ablation of
Sec. 3 measures against.

What fixes the result independently of the oracle's code:
- the law: city j with probability p_j / (sum of p over the unvisited), checked by
  chi-square on one step and on whole 5-city tours (product of conditionals);
- the inverse CDF, recomputed with exact rationals from the deviate;
- the deviate's counter layout, against the Philox known-answer-tested routine;
- the degenerate cases: weight-0 and visited cities are never drawn, all-zero
  rows fall to the smallest unvisited city, one positive weight is always drawn;
- whole runs: permutations, lengths that agree with the tours, and never below the
  Held-Karp optimum.
"""
import itertools
from fractions import Fraction

import numpy as np
from scipy import stats

import aco_instances as inst


def test_roulette_deviate_counter_layout(oracle_lib):
    """Word 0 of Philox counter (0, s, a, t) under key (seed lo, seed hi)."""
    for seed, t, a, s in ((0, 0, 0, 1), (0x1234_5678_9ABC_DEF0, 7, 3, 11), (5, 2**31, 999, 4)):
        words = oracle_lib.philox4x32_10([0, s, a, t], [seed & 0xFFFFFFFF, seed >> 32])
        want = (2 * (int(words[0]) >> 9) + 1) * 2.0 ** -24
        assert oracle_lib.roulette_deviate(seed, t, a, s) == want


def test_roulette_inverse_cdf_exact(oracle_lib):
    """The city drawn is the first unvisited city, in ascending order, whose
    running sum exceeds v * total, computed here with exact rationals."""
    rng = np.random.default_rng(3)
    for trial in range(40):
        n = int(rng.integers(3, 12))
        row = rng.random(n).astype(np.float32)
        row[rng.random(n) < 0.2] = 0.0
        visited = (rng.random(n) < 0.3).astype(np.uint8)
        visited[int(rng.integers(n))] = 0
        free = [j for j in range(n) if not visited[j]]
        if sum(float(row[j]) for j in free) == 0.0:
            row[free[-1]] = 0.5
        total = sum(Fraction(float(row[j])) for j in free)
        for a in range(25):
            v = Fraction(oracle_lib.roulette_deviate(11, trial, a, 2))
            x = v * total
            run = Fraction(0)
            want = None
            for j in free:
                run += Fraction(float(row[j]))
                if run > x:
                    want = j
                    break
            assert oracle_lib.select_roulette(row, visited, 11, trial, a, 2) == want


def test_roulette_law_one_step(oracle_lib):
    row = np.array([0.30, 0.05, 0.9, 0.20, 0.0, 0.15, 0.10, 0.7], np.float32)
    visited = np.array([0, 0, 1, 0, 0, 0, 0, 1], np.uint8)
    trials = 150000
    picks = oracle_lib.select_roulette_many(row, visited, 21, 4, 6, trials)
    counts = np.bincount(picks, minlength=row.size)
    assert counts[2] == 0 and counts[7] == 0   # visited
    assert counts[4] == 0                      # weight 0
    cand = [0, 1, 3, 5, 6]
    w = row[cand].astype(np.float64)
    law = w / w.sum()
    assert stats.chisquare(counts[cand], law * trials).pvalue > 1e-4
    # the independent roulette (argmax of p * r) follows another law on the
    # same row; RW must not be mistaken for it
    ir = oracle_lib.select_many(row, visited, 21, 4, 6, trials)
    ir_counts = np.bincount(ir, minlength=row.size)[cand]
    assert stats.chisquare(ir_counts, law * trials).pvalue < 1e-6


def test_roulette_law_whole_tours(oracle_lib):
    """n = 5: the frequency of each tour from a given start equals the product
    of the step probabilities, each step using the row of the current city."""
    n = 5
    rng = np.random.default_rng(8)
    P = rng.random((n, n)).astype(np.float32) + 0.05
    np.fill_diagonal(P, 0.0)
    P[1, 3] = 0.0  # an edge that is never taken from city 1
    D = inst.distance_matrix(inst.uniform_cities(n, 4))
    ants = np.arange(120000)
    tours, lengths = oracle_lib.construct(P, D, 5, 1, ants, selection="roulette")
    for t in tours[:200]:
        assert sorted(t) == list(range(n))
    starts = tours[:, 0]
    for start in range(n):
        sel = tours[starts == start]
        perms = [p for p in itertools.permutations(range(n)) if p[0] == start]
        law = []
        for p in perms:
            prob, seen = 1.0, {start}
            for a, b in zip(p[:-1], p[1:]):
                free = [j for j in range(n) if j not in seen]
                total = sum(float(P[a, j]) for j in free)
                if total > 0:
                    prob *= float(P[a, b]) / total
                else:  # no positive weight left: the smallest free city
                    prob *= 1.0 if b == min(free) else 0.0
                seen.add(b)
            law.append(prob)
        law = np.array(law)
        key = {p: k for k, p in enumerate(perms)}
        counts = np.zeros(len(perms))
        for t in sel:
            counts[key[tuple(int(c) for c in t)]] += 1
        live = law > 0
        assert counts[~live].sum() == 0
        assert stats.chisquare(counts[live], law[live] / law[live].sum() * len(sel)).pvalue > 1e-4
    assert np.all(lengths == np.array([oracle_lib.tour_length(t, D) for t in tours[:len(lengths)]]))


def test_roulette_degenerate_rows(oracle_lib):
    vis = np.array([1, 0, 0, 1, 0, 0], np.uint8)
    zero = np.zeros(6, np.float32)
    one = np.array([0.0, 0.0, 0.0, 0.9, 0.4, 0.0], np.float32)  # only city 4 can be drawn
    tiny = np.array([0.0, 0.0, 0.0, 0.0, 1e-45, 0.0], np.float32)  # one subnormal weight
    for a in range(60):
        assert oracle_lib.select_roulette(zero, vis, 3, 0, a, 1) == 1
        assert oracle_lib.select_roulette(one, vis, 3, 0, a, 1) == 4
        assert oracle_lib.select_roulette(tiny, vis, 3, 0, a, 1) == 4  # not flushed to 0


def test_roulette_run_valid_and_above_optimum(oracle_lib):
    for seed in range(6):
        n = 8
        D = inst.distance_matrix(inst.uniform_cities(n, 300 + seed))
        opt, _ = oracle_lib.tsp_exact(D)
        res = oracle_lib.run(D, n, 1.0, 2.0, 0.5, 1.0, seed, 40, gamma_max=1.0, gamma_min=1.0,
                             selection="roulette")
        assert sorted(res["best_tour"]) == list(range(n))
        assert res["best_len"] == oracle_lib.tour_length(res["best_tour"], D)
        assert res["best_len"] >= np.float32(opt) * (1 - 1e-6)
        assert res["best_len"] <= 1.15 * opt
