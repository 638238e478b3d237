"""MAX-MIN pheromone bounds and the paper's elitist deposit at scale (k = n/10),
on the GPU against the oracle, through the C ABI.

Bars: tau bit-exact (integer deposit, one FP64 fma, one rounding, an exact
clamp); P within 1e-5 relative; best lengths equal.
"""
import math

import numpy as np
import pytest

import aco_instances as inst
import oracle

pytestmark = pytest.mark.gpu

FLT_MIN = np.float32(1.1754944e-38)


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _colony(D, alpha, beta, rho, Q, m_max, **kw):
    torch = _torch()
    from paper_2404_04895_amd import Colony
    return Colony(torch.from_numpy(D).cuda(), alpha, beta, rho, Q, m_max, **kw)


def _assert_P_close(P_gpu, P_ref):
    P_gpu = np.asarray(P_gpu, np.float64)
    P_ref = np.asarray(P_ref, np.float64)
    bound = 1e-5 * np.maximum(np.abs(P_ref), float(FLT_MIN))
    assert not (np.abs(P_gpu - P_ref) > bound).any()


@pytest.mark.parametrize("bounds", [(0.05, 0.6), (0.0, 0.4), (0.2, math.inf)])
def test_bounded_run_matches_oracle(bounds):
    torch = _torch()
    n, m, T = 16, 16, 30
    D = inst.distance_matrix(inst.uniform_cities(n, 31))
    col = _colony(D, 1.0, 2.0, 0.2, 1.0, m)
    col.set_tau_bounds(*bounds)
    tour, L = col.run(m, 5, T)
    ref = oracle.run(D, m, 1.0, 2.0, 0.2, 1.0, 5, T, tau_min=bounds[0], tau_max=bounds[1])
    tau = col.tau().cpu().numpy()
    assert L == ref["best_len"]
    assert np.array_equal(tau, ref["tau"])
    off = tau[~np.eye(n, dtype=bool)]
    assert off.min() >= np.float32(bounds[0]) and off.max() <= np.float32(bounds[1])
    col.close()


def test_bounds_rejected_and_default_is_unbounded():
    torch = _torch()
    from paper_2404_04895_amd import AcoError
    n, m = 12, 8
    D = inst.distance_matrix(inst.uniform_cities(n, 2))
    col = _colony(D, 1.0, 2.0, 0.3, 1.0, m)
    for lo, hi in ((-0.1, 1.0), (0.5, 0.4), (0.0, 0.0), (math.inf, math.inf), (0.0, math.nan)):
        with pytest.raises(AcoError):
            col.set_tau_bounds(lo, hi)
    tour, L = col.run(m, 3, 10)
    ref = oracle.run(D, m, 1.0, 2.0, 0.3, 1.0, 3, 10)
    assert L == ref["best_len"] and np.array_equal(col.tau().cpu().numpy(), ref["tau"])
    col.close()


@pytest.mark.parametrize("selection", ["adair-sorted", "adair"])
def test_elite_tenth_with_bounds_full_size(selection):
    """The benchmark workload (5000 clustered cities, 5000 ants, beta 3) with
    the paper's elitist deposit, k = n/10 = 500, and MAX-MIN bounds: the
    tours of sampled ants, then the whole update, against the oracle."""
    torch = _torch()
    w = inst.WORKLOADS["clustered-n5000-m5000"]
    D = w.dist(0)
    n, m, k = w.n, w.m, w.n // 10
    col = _colony(D, w.alpha, w.beta, w.rho, w.Q, m, elite_k=k)
    col.set_selection(selection)
    lo, hi = 0.92, 1.0 + 1e-4
    col.set_tau_bounds(lo, hi)
    col.transition(1.5)
    col.construct(m, 3, 0)
    col.sync()
    P = col.P().cpu().numpy()
    tours = col.tours(m).cpu().numpy()
    lengths = col.lengths(m).cpu().numpy()
    tau_prev = col.tau().cpu().numpy()
    sample = np.array([0, 4999])
    o_tours, o_len = oracle.construct(P, D, 3, 0, sample)
    assert np.array_equal(tours[sample], o_tours)
    col.update(1.4)
    col.sync()
    S = col.deposit_scale
    elite = oracle.elite(lengths, k)
    assert int(elite.sum()) == k
    delta = oracle.deposit(tours, lengths, elite, w.Q, S)
    tau_ref = oracle.clamp(oracle.evaporate(tau_prev, delta, w.rho, S), lo, hi)
    del delta
    tau = col.tau().cpu().numpy()
    assert np.array_equal(tau.view(np.uint32), tau_ref.view(np.uint32))
    off = tau[~np.eye(n, dtype=bool)]
    # evaporation alone (0.9) falls below 0.92, the elite's deposit exceeds the cap
    assert np.any(off == np.float32(lo)) and np.any(off == np.float32(hi))
    _assert_P_close(col.P().cpu().numpy(), oracle.transition(tau_ref, D, w.alpha, w.beta, 1.4))
    col.close()
