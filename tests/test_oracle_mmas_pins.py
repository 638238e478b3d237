"""Pins of the oracle's MAX-MIN pheromone bounds (the MAX-MIN Ant System's
clamp of tau into [tau_min, tau_max] after each update; not in the paper).

What fixes the result:
- exact powers of two under evaporation only, where the closed form crosses
  the lower bound at a known iteration;
- the cap of a deposit larger than the upper bound;
- unbounded runs identical to runs without the clamp;
- a bounded run keeps every off-diagonal tau inside the bounds, symmetric,
  and with a zero diagonal;
- the clamp leaves the diagonal alone.
"""
import math

import numpy as np

import aco_instances as inst


def test_clamp_under_evaporation_closed_form(oracle_lib):
    """rho = 1/2, no deposit: tau halves each update, 1 -> 0.5, then 0.25
    falls below tau_min = 0.3 at the second update and is clamped to 0.3,
    where it stays (0.3 * 0.5 = 0.15 is clamped back each time)."""
    n = 5
    tau = np.where(np.eye(n, dtype=bool), 0, 1).astype(np.float32)
    want = [0.5, np.float32(0.3), np.float32(0.3), np.float32(0.3)]
    for t in range(4):
        tau = oracle_lib.evaporate(tau, None, 0.5, 0)
        tau = oracle_lib.clamp(tau, 0.3, math.inf)
        off = tau[~np.eye(n, dtype=bool)]
        assert np.all(off == np.float32(want[t])), (t, off[:3])
    assert np.all(np.diag(tau) == 0)


def test_clamp_caps_a_large_deposit(oracle_lib):
    n = 4
    tau = np.where(np.eye(n, dtype=bool), 0, 1).astype(np.float32)
    delta = np.zeros((n, n), np.int64)
    delta[0, 1] = delta[1, 0] = 3 << 20          # 3.0 at S = 20
    tau = oracle_lib.evaporate(tau, delta, 0.25, 20)
    assert tau[0, 1] == np.float32(0.75 + 3.0)
    capped = oracle_lib.clamp(tau, 0.0, 2.0)
    assert capped[0, 1] == 2.0 and capped[1, 0] == 2.0
    assert capped[0, 2] == np.float32(0.75)     # inside the bounds: untouched
    assert np.all(np.diag(capped) == 0)


def test_unbounded_run_equals_plain_run(oracle_lib):
    n, m = 12, 10
    D = inst.distance_matrix(inst.uniform_cities(n, 6))
    a = oracle_lib.run(D, m, 1.0, 2.0, 0.3, 1.0, 2, 15)
    b = oracle_lib.run(D, m, 1.0, 2.0, 0.3, 1.0, 2, 15, tau_min=0.0, tau_max=math.inf)
    assert np.array_equal(a["tau"], b["tau"]) and a["best_len"] == b["best_len"]


def test_bounded_run_stays_in_bounds(oracle_lib):
    n, m = 14, 12
    D = inst.distance_matrix(inst.uniform_cities(n, 9))
    lo, hi = 0.05, 0.6
    for iters in (1, 5, 30):
        r = oracle_lib.run(D, m, 1.0, 2.0, 0.2, 1.0, 4, iters, tau_min=lo, tau_max=hi)
        off = r["tau"][~np.eye(n, dtype=bool)]
        assert off.min() >= np.float32(lo) and off.max() <= np.float32(hi)
        assert np.array_equal(r["tau"], r["tau"].T)
        assert np.all(np.diag(r["tau"]) == 0)
    # after 30 iterations of rho = 0.2 both bounds are in use
    assert np.any(off == np.float32(lo)) and np.any(off == np.float32(hi))
    # and the bounds changed the run against the unbounded one
    free = oracle_lib.run(D, m, 1.0, 2.0, 0.2, 1.0, 4, 30)
    assert not np.array_equal(free["tau"], r["tau"])
