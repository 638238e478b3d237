"""Pins for the CPU oracle: checks against things other than the oracle itself.

Each test fixes a part of the oracle to a published value, a closed form, a
library routine, an invariant or brute force, so that a plausible slip in the
oracle (a dropped term, a wrong sign or index, a transposed operand, gamma
applied the wrong way round) fails at least one of them.
"""
import itertools
import math
import os
import shutil
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import aco_instances as inst

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Philox4x32-10 (counter-based generator).
# --------------------------------------------------------------------------
def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            words = [int(w, 16) for w in line.split()]
            rows.append((words[0:4], words[4:6], words[6:10]))
    return rows


def test_philox_known_answers(oracle_lib):
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = oracle_lib.philox4x32_10(ctr, key)
        assert [int(x) for x in got] == want


def test_philox_matches_rocrand_header(oracle_lib, tmp_path):
    """Random (counter, key) pairs against rocRAND's open-source Philox header."""
    gxx = shutil.which("g++")
    inc = "/opt/rocm/include"
    if gxx is None or not os.path.exists(os.path.join(inc, "rocrand", "rocrand_philox4x32_10.h")):
        pytest.skip("rocRAND header or g++ not available")
    src = os.path.join(os.path.dirname(__file__), "rocrand_philox_check.cpp")
    exe = str(tmp_path / "rr")
    subprocess.run([gxx, "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I" + inc, src, "-o", exe],
                   check=True)
    rng = np.random.default_rng(7)
    cases = rng.integers(0, 2**32, size=(2000, 6), dtype=np.uint64)
    cases[:, 1] %= 2**30  # keeps the rocRAND offset (4 x words 0-1) inside 64 bits
    text = "\n".join(" ".join("%08x" % int(v) for v in row) for row in cases) + "\n"
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
    got_rr = [[int(w, 16) for w in line.split()] for line in out.strip().splitlines()]
    assert len(got_rr) == len(cases)
    for row, rr in zip(cases, got_rr):
        mine = oracle_lib.philox4x32_10([int(v) for v in row[:4]], [int(v) for v in row[4:]])
        assert [int(x) for x in mine] == rr


# --------------------------------------------------------------------------
# Uniform deviates r of Sec. 2.4 (open interval (0,1)).
# --------------------------------------------------------------------------
def test_to_unit_exhaustive(oracle_lib):
    """All 2^23 values of the top 23 bits: exact odd multiples of 2^-24 in (0,1),
    strictly increasing; the low 9 bits are ignored."""
    k = np.arange(1 << 23, dtype=np.uint64)
    words = (k << np.uint64(9)).astype(np.uint32)
    u = oracle_lib.to_unit_many(words)
    assert u.dtype == np.float32
    expect = (2.0 * k.astype(np.float64) + 1.0) / float(1 << 24)
    assert np.array_equal(u.astype(np.float64), expect)
    assert np.all(np.diff(u) > 0)
    assert u[0] > 0.0 and u[-1] < 1.0
    low = oracle_lib.to_unit_many(words | np.uint32(0x1FF))
    assert np.array_equal(low, u)


def test_uniforms_are_uniform(oracle_lib):
    us = np.array([oracle_lib.uniform(123, 4, a, s, j)
                   for a in range(20) for s in range(1, 11) for j in range(100)])
    res = stats.kstest(us, "uniform")
    assert res.pvalue > 1e-3


def test_uniform_keyed_by_city_block(oracle_lib):
    """r_j is word j mod 4 of counter (j/4, s, a, t)."""
    seed = (0xABCDEF << 32) | 0x12345
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for (t, a, s, j) in [(0, 0, 1, 0), (3, 17, 5, 6), (9, 2, 40, 13), (1, 99, 7, 31)]:
        words = oracle_lib.philox4x32_10([j // 4, s, a, t], key)
        assert oracle_lib.uniform(seed, t, a, s, j) == oracle_lib.to_unit(int(words[j % 4]))


def test_eq5_distribution_of_r_gamma(oracle_lib):
    """Eq. (5): Y = X^gamma has CDF y^(1/gamma) on (0,1)."""
    gamma = 1.5
    x = np.array([oracle_lib.uniform(5, 0, a, 1, j) for a in range(40) for j in range(500)],
                 dtype=np.float64)
    y = x ** gamma
    res = stats.kstest(y, lambda v: np.clip(v, 0, 1) ** (1.0 / gamma))
    assert res.pvalue > 1e-3
    # and it is not the law of X itself (the test has power)
    assert stats.kstest(y, "uniform").pvalue < 1e-6


def test_start_city_uniform(oracle_lib):
    n = 7
    starts = oracle_lib.start_cities(11, 3, n, 70000)
    assert starts.min() >= 0 and starts.max() < n
    counts = np.bincount(starts, minlength=n)
    assert stats.chisquare(counts).pvalue > 1e-3


# --------------------------------------------------------------------------
# Preprocessing, Eq. (1) with the AdaIR exponent folded in.
# --------------------------------------------------------------------------
def _triangle():
    xy = np.array([[0, 0], [3, 0], [0, 4]], np.float32)  # sides 3, 4, 5
    return inst.distance_matrix(xy)


def _golden_transition():
    cases = []
    cur = None
    with open(os.path.join(GOLDEN, "transition_triangle.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, val = line.partition("=")
            key = key.strip()
            val = val.strip()
            if key == "case":
                cur = {"name": val}
                cases.append(cur)
            elif key in ("alpha", "beta", "gamma"):
                cur[key] = float(val)
            elif key == "tau":
                cur["tau"] = np.array([[float(Fraction(x)) for x in r.split()]
                                       for r in val.split(";")], np.float32)
            elif key == "P":
                rows = []
                for r in val.split(";"):
                    row = []
                    for x in r.split():
                        if x.startswith("sqrt(") and x.endswith(")"):
                            row.append(math.sqrt(float(Fraction(x[5:-1]))))
                        else:
                            row.append(float(Fraction(x)))
                    rows.append(row)
                cur["P"] = np.array(rows, np.float64)
    return cases


def test_transition_triangle_golden(oracle_lib):
    D = _triangle()
    assert D[0, 1] == 3 and D[0, 2] == 4 and D[1, 2] == 5
    cases = _golden_transition()
    assert len(cases) >= 5
    for c in cases:
        P = oracle_lib.transition(c["tau"], D, c["alpha"], c["beta"], c["gamma"])
        np.testing.assert_allclose(P.astype(np.float64), c["P"], rtol=2e-7, atol=0,
                                   err_msg=c["name"])


def test_transition_uniform_when_exponents_zero(oracle_lib):
    D = inst.distance_matrix(inst.uniform_cities(37, 1))
    tau = np.random.default_rng(0).random((37, 37)).astype(np.float32) + 0.1
    P = oracle_lib.transition(tau, D, 0.0, 0.0, 1.0)
    off = ~np.eye(37, dtype=bool)
    np.testing.assert_allclose(P[off], np.float32(1.0 / 36), rtol=1e-7)
    assert np.all(np.diag(P) == 0)


def test_transition_row_sums_and_gamma(oracle_lib):
    """gamma = 1 rows sum to 1; for gamma != 1, P^gamma rows sum to 1 and the
    order of entries within a row is kept (x -> x^(1/gamma) is increasing)."""
    n = 60
    D = inst.distance_matrix(inst.clustered_cities(n, 3, 4, 0.05))
    rng = np.random.default_rng(1)
    tau = (rng.random((n, n)) * 3 + 0.01).astype(np.float32)
    P1 = oracle_lib.transition(tau, D, 1.0, 2.0, 1.0).astype(np.float64)
    np.testing.assert_allclose(P1.sum(1), 1.0, rtol=1e-5)
    for g in (1.5, 0.7):
        Pg = oracle_lib.transition(tau, D, 1.0, 2.0, g).astype(np.float64)
        np.testing.assert_allclose((Pg ** g).sum(1), 1.0, rtol=1e-5)
        np.testing.assert_allclose(Pg ** g, P1, rtol=2e-6, atol=1e-30)
    # explicit learned-heuristic input eta = 1/d gives the same matrix
    eta = np.where(np.eye(n, dtype=bool), 1.0, 1.0 / np.where(D > 0, D, 1)).astype(np.float32)
    Pe = oracle_lib.transition(tau, D, 1.0, 2.0, 1.0, eta=eta).astype(np.float64)
    np.testing.assert_allclose(Pe, P1, rtol=3e-7)


# --------------------------------------------------------------------------
# Selection, Sec. 2.4 (IR / AdaIR) against the closed-form selection law.
# --------------------------------------------------------------------------
def _win_probability(p, j, gamma):
    """P(candidate j wins) for score p_k * r_k^gamma with r_k i.i.d. U(0,1):
    integral over x in (0,1) of prod_{k != j} min(1, c_k x), c_k = (p_j/p_k)^(1/gamma).
    The integrand is a polynomial between the breakpoints 1/c_k; integrate
    each piece exactly."""
    c = [(p[j] / p[k]) ** (1.0 / gamma) for k in range(len(p)) if k != j]
    cuts = sorted({0.0, 1.0} | {1.0 / ck for ck in c if 1.0 / ck < 1.0})
    total = 0.0
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        mid = 0.5 * (lo + hi)
        poly = np.poly1d([1.0])
        for ck in c:
            poly = poly * (np.poly1d([ck, 0.0]) if ck * mid < 1.0 else np.poly1d([1.0]))
        integ = poly.integ()
        total += integ(hi) - integ(lo)
    return total


def test_win_probability_two_candidates_closed_form():
    for p1, p2, g in [(0.7, 0.3, 1.0), (0.7, 0.3, 1.5), (0.5, 0.5, 2.0), (0.9, 0.1, 1.5)]:
        want = 1.0 - 0.5 * (p2 / p1) ** (1.0 / g)
        assert abs(_win_probability([p1, p2], 0, g) - want) < 1e-12
    p = [0.5, 0.3, 0.15, 0.05]
    assert abs(sum(_win_probability(p, j, 1.5) for j in range(4)) - 1.0) < 1e-12


@pytest.mark.parametrize("gamma", [1.0, 1.5, 2.5])
def test_selection_law_matches_closed_form(oracle_lib, gamma):
    """Folded selection on P^(1/gamma) and the literal p*r^gamma of Eq. (4)
    both follow the closed-form law; the wrong exponent direction does not."""
    p = np.array([0.42, 0.25, 0.18, 0.10, 0.05])
    visited = np.array([0, 0, 1, 0, 0, 0, 0], np.uint8)
    row_p = np.array([p[0], p[1], 0.9, p[2], p[3], p[4], 0.0])
    row_p = np.where(visited == 1, 0.9, row_p)
    cand = [0, 1, 3, 4, 5, 6]
    weights = np.array([p[0], p[1], p[2], p[3], p[4], 0.0])
    trials = 120000
    folded_row = np.where(row_p > 0, row_p ** (1.0 / gamma), 0.0).astype(np.float32)
    folded = oracle_lib.select_many(folded_row, visited, 99, 2, 3, trials)
    literal = oracle_lib.select_many(row_p, visited, 99, 2, 3, trials, gamma=gamma, literal=True)
    live = [k for k in range(len(cand)) if weights[k] > 0]
    law = np.array([_win_probability(weights[live], i, gamma) for i in range(len(live))])
    for picks in (folded, literal):
        assert not np.any(picks == 2)          # visited city never chosen
        assert not np.any(picks == 6)          # zero-probability city never chosen
        counts = np.array([np.sum(picks == cand[k]) for k in live])
        assert counts.sum() == trials
        assert stats.chisquare(counts, law * trials).pvalue > 1e-4
    if gamma != 1.0:
        wrong = np.array([_win_probability(weights[live], i, 1.0 / gamma) for i in range(len(live))])
        counts = np.array([np.sum(folded == cand[k]) for k in live])
        assert stats.chisquare(counts, wrong * trials).pvalue < 1e-6


def test_selection_uniform_when_row_constant(oracle_lib):
    """alpha = beta = 0 makes every row constant: each step is a uniform draw
    over the unvisited cities."""
    n = 9
    row = np.full(n, 1.0 / (n - 1), np.float32)
    visited = np.zeros(n, np.uint8)
    visited[[2, 5]] = 1
    picks = oracle_lib.select_many(row, visited, 4, 0, 1, 70000)
    counts = np.bincount(picks, minlength=n)
    assert counts[2] == 0 and counts[5] == 0
    assert stats.chisquare(counts[[0, 1, 3, 4, 6, 7, 8]]).pvalue > 1e-3


def test_selection_ties_and_zero_rows(oracle_lib):
    """All-zero candidate scores fall to the smallest unvisited index."""
    row = np.zeros(6, np.float32)
    vis = np.array([1, 0, 0, 1, 0, 0], np.uint8)
    for a in range(50):
        assert oracle_lib.select(row, vis, 3, 0, a, 1) == 1


def test_construct_follows_deterministic_row(oracle_lib):
    """P[c, (c+1) mod n] = 1 and 0 elsewhere: every ant walks start, start+1, ...
    (reads row c, not column c: a transposed P would walk backwards)."""
    n = 11
    P = np.zeros((n, n), np.float32)
    for c in range(n):
        P[c, (c + 1) % n] = 1.0
    D = inst.distance_matrix(inst.uniform_cities(n, 2))
    tours, lengths = oracle_lib.construct(P, D, 77, 5, np.arange(8))
    for a in range(8):
        s0 = oracle_lib.start_city(77, 5, a, n)
        assert list(tours[a]) == [(s0 + k) % n for k in range(n)]
        want = sum(float(D[(s0 + k) % n, (s0 + k + 1) % n]) for k in range(n))
        assert abs(lengths[a] - want) <= 1e-6 * want


def test_construct_tours_are_permutations(oracle_lib):
    n = 40
    D = inst.distance_matrix(inst.uniform_cities(n, 5))
    tau = np.where(np.eye(n, dtype=bool), 0, 1).astype(np.float32)
    P = oracle_lib.transition(tau, D, 1.0, 2.0, 1.5)
    tours, lengths = oracle_lib.construct(P, D, 1, 0, np.arange(30))
    for a in range(30):
        assert sorted(tours[a]) == list(range(n))
        assert tours[a, 0] == oracle_lib.start_city(1, 0, a, n)
        assert lengths[a] == oracle_lib.tour_length(tours[a], D)


def test_tour_length_golden():
    import oracle
    xy = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], np.float32)
    D = inst.distance_matrix(xy)
    assert oracle.tour_length([0, 1, 2, 3], D) == 4.0
    assert oracle.tour_length([0, 2, 1, 3], D) == np.float32(2.0 + 2.0 * math.sqrt(2.0))


# --------------------------------------------------------------------------
# Ant path tensorization, Sec. 2.3 (Eq. 2, Eq. 3) and evaporation.
# --------------------------------------------------------------------------
def test_deposit_scale_square(oracle_lib):
    """Unit square: every nearest neighbour is at distance 1, so L_lb = 4.
    m_max = 2, Q = 1: x = 1/2, largest S with 2^(S-1) < 2^62 is S = 62."""
    xy = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], np.float32)
    D = inst.distance_matrix(xy)
    assert oracle_lib.length_lower_bound(D) == 4.0
    assert oracle_lib.deposit_scale(D, 2, 1.0) == 62
    assert oracle_lib.deposit_scale(D, 1, 1.0) == 63
    assert oracle_lib.deposit_scale(D, 3, 1.0) == 62
    assert oracle_lib.deposit_scale(D, 4, 1.0) == 61
    assert oracle_lib.deposit_weight(4.0, 1.0, 62) == 2 ** 60


def test_deposit_square_by_hand(oracle_lib):
    xy = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], np.float32)
    D = inst.distance_matrix(xy)
    tours = np.array([[0, 1, 2, 3], [0, 2, 1, 3]], np.int32)
    L = np.array([oracle_lib.tour_length(t, D) for t in tours], np.float32)
    S = oracle_lib.deposit_scale(D, 2, 1.0)
    q0 = 2 ** 60
    q1 = int(round(float(Fraction(2 ** S) / Fraction(float(L[1])))))
    assert oracle_lib.deposit_weight(L[1], 1.0, S) == q1
    delta = oracle_lib.deposit(tours, L, None, 1.0, S)
    want = np.zeros((4, 4), np.int64)
    for (i, j, v) in [(0, 1, q0), (1, 2, q0 + q1), (2, 3, q0), (3, 0, q0 + q1), (0, 2, q1),
                      (1, 3, q1)]:
        want[i, j] = want[j, i] = v
    assert np.array_equal(delta, want)
    only_best = oracle_lib.deposit(tours, L, oracle_lib.elite(L, 1), 1.0, S)
    assert only_best[0, 2] == 0 and only_best[0, 1] == q0


def test_deposit_equals_index_mapping_form(oracle_lib):
    """The oracle walks paths edge by edge; Eq. (2)-(3) build the index matrix
    of each path and its one-step shift and scatter 1/f symmetrically.  Both
    must give the same integer dTau."""
    n, m = 23, 17
    D = inst.distance_matrix(inst.uniform_cities(n, 9))
    rng = np.random.default_rng(3)
    tours = np.stack([rng.permutation(n) for _ in range(m)]).astype(np.int32)
    L = np.array([oracle_lib.tour_length(t, D) for t in tours], np.float32)
    S = oracle_lib.deposit_scale(D, m, 1.0)
    delta = oracle_lib.deposit(tours, L, None, 1.0, S)
    A_sum = np.zeros((n, n), dtype=object)
    for a in range(m):
        q = oracle_lib.deposit_weight(L[a], 1.0, S)
        I = np.stack([tours[a], np.roll(tours[a], 1)], 1)  # Eq. (2)
        A = np.zeros((n, n), bool)
        A[I[:, 0], I[:, 1]] = True
        A[I[:, 1], I[:, 0]] = True                          # Eq. (3): (i,j) or (j,i)
        A_sum = A_sum + A.astype(object) * q
    assert np.array_equal(delta.astype(object), A_sum)
    # invariants: symmetric, zero diagonal, total 2n * sum q
    assert np.array_equal(delta, delta.T)
    assert np.all(np.diag(delta) == 0)
    total_q = sum(oracle_lib.deposit_weight(L[a], 1.0, S) for a in range(m))
    assert int(delta.astype(object).sum()) == 2 * n * total_q
    approx = (delta.astype(np.float64) * D.astype(np.float64)).sum() / 2.0 ** S
    assert abs(approx - 2.0 * m * 1.0) < 1e-5 * 2 * m


def test_elite_top_k(oracle_lib):
    L = np.array([5.0, 3.0, 4.0, 3.0, 9.0], np.float32)
    assert list(oracle_lib.elite(L, 2)) == [0, 1, 0, 1, 0]
    assert list(oracle_lib.elite(L, 3)) == [0, 1, 1, 1, 0]
    assert list(oracle_lib.elite(L, 0)) == [1] * 5
    assert list(oracle_lib.elite(L, 5)) == [1] * 5


def test_evaporation_exact_powers(oracle_lib):
    """rho = 1/2 and no deposit: tau_t = 2^-t exactly; rho = 1 wipes tau to the deposit."""
    n = 5
    tau = np.where(np.eye(n, dtype=bool), 0, 1).astype(np.float32)
    for t in range(1, 60):
        tau = oracle_lib.evaporate(tau, None, 0.5, 0)
        off = tau[~np.eye(n, dtype=bool)]
        assert np.all(off == np.float32(2.0 ** -t))
    assert np.all(np.diag(tau) == 0)
    delta = np.full((n, n), 3 << 40, np.int64)
    t1 = oracle_lib.evaporate(tau, delta, 1.0, 40)
    assert np.all(t1[~np.eye(n, dtype=bool)] == 3.0)


def test_gamma_schedule(oracle_lib):
    T = 11
    g = [oracle_lib.gamma(t, T, 1.5, 1.0) for t in range(T)]
    assert g[0] == np.float32(1.5) and g[-1] == np.float32(1.0)
    assert abs(g[5] - 1.25) < 1e-7
    assert all(x >= y for x, y in zip(g, g[1:]))
    assert oracle_lib.gamma(3, 1, 1.5, 1.0) == np.float32(1.5)


# --------------------------------------------------------------------------
# Whole runs: exact optimum on tiny instances and invariants along the run.
# --------------------------------------------------------------------------
def _brute_force(D):
    n = D.shape[0]
    best = math.inf
    for perm in itertools.permutations(range(1, n)):
        tour = (0,) + perm
        L = sum(float(D[tour[k], tour[(k + 1) % n]]) for k in range(n))
        best = min(best, L)
    return best


def test_exact_solver_vs_brute_force(oracle_lib):
    for seed in range(6):
        n = 5 + seed % 4
        D = inst.distance_matrix(inst.uniform_cities(n, 100 + seed))
        L, tour = oracle_lib.tsp_exact(D)
        assert abs(L - _brute_force(D)) < 1e-9
        assert sorted(tour) == list(range(n))
        assert abs(sum(float(D[tour[k], tour[(k + 1) % n]]) for k in range(n)) - L) < 1e-9
        assert oracle_lib.length_lower_bound(D) <= L + 1e-12


def test_exact_solver_circle_polygon(oracle_lib):
    n, R = 12, 0.5
    D = inst.distance_matrix(inst.circle_cities(n, R))
    L, _ = oracle_lib.tsp_exact(D)
    assert abs(L - 2 * n * R * math.sin(math.pi / n)) < 1e-5


def test_run_reaches_optimum_on_tiny_instances(oracle_lib):
    hits, total = 0, 0
    for seed in range(20):
        n = 7 + seed % 2
        D = inst.distance_matrix(inst.uniform_cities(n, 200 + seed))
        opt, _ = oracle_lib.tsp_exact(D)
        res = oracle_lib.run(D, n, 1.0, 2.0, 0.5, 1.0, seed, 60)
        assert sorted(res["best_tour"]) == list(range(n))
        assert res["best_len"] >= np.float32(opt) * (1 - 1e-6)
        assert res["best_len"] == oracle_lib.tour_length(res["best_tour"], D)
        total += 1
        hits += int(abs(res["best_len"] - opt) <= 1e-5 * opt)
    assert hits >= 18, (hits, total)


def test_run_circle_finds_polygon(oracle_lib):
    n = 16
    D = inst.distance_matrix(inst.circle_cities(n, 0.5))
    res = oracle_lib.run(D, n, 1.0, 3.0, 0.3, 1.0, 0, 80)
    assert abs(res["best_len"] - 2 * n * 0.5 * math.sin(math.pi / n)) < 1e-5


def test_pheromone_bounds_along_run(oracle_lib):
    """lower_t = (1-rho)^t tau0 <= tau_ij <= (1-rho)^t tau0 + sum_s (1-rho)^(t-1-s) D_s,
    D_s = sum of Q/L over the ants that deposited at iteration s; tau stays
    symmetric with a zero diagonal."""
    n, m, rho, Q = 14, 10, 0.3, 1.0
    D = inst.distance_matrix(inst.uniform_cities(n, 4))
    tau = np.where(np.eye(n, dtype=bool), 0, 1).astype(np.float32)
    S = oracle_lib.deposit_scale(D, m, Q)
    lower, upper = 1.0, 1.0
    for t in range(25):
        P = oracle_lib.transition(tau, D, 1.0, 2.0, oracle_lib.gamma(t, 25, 1.5, 1.0))
        tours, L = oracle_lib.construct(P, D, 8, t, np.arange(m))
        elite = oracle_lib.elite(L, 4)
        delta = oracle_lib.deposit(tours, L, elite, Q, S)
        tau = oracle_lib.evaporate(tau, delta, rho, S)
        Ds = sum(Q / float(L[a]) for a in range(m) if elite[a])
        lower = (1 - rho) * lower
        upper = (1 - rho) * upper + Ds
        off = tau[~np.eye(n, dtype=bool)].astype(np.float64)
        slack = (t + 1) * 2.0 ** -23
        assert off.min() >= lower * (1 - slack)
        assert off.max() <= upper * (1 + slack)
        assert np.array_equal(tau, tau.T)
        assert np.all(np.diag(tau) == 0)


def test_transition_rows_subset(oracle_lib):
    """The row-subset entry point returns the full transition's rows."""
    n = 37
    D = inst.distance_matrix(inst.uniform_cities(n, 12))
    rng = np.random.default_rng(1)
    tau = (rng.random((n, n)) + 0.1).astype(np.float32)
    np.fill_diagonal(tau, 0.0)
    P = oracle_lib.transition(tau, D, 1.0, 2.0, 1.3)
    rows = [0, 5, 36, 5]
    assert np.array_equal(oracle_lib.transition_rows(tau, D, 1.0, 2.0, 1.3, rows), P[rows])
