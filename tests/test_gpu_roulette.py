"""Roulette Wheel selection on the GPU against the oracle, through the C ABI.

Bar: tours and FP32 lengths equal the oracle's for the same P.  The two sides
sum the wheel in FP64 with different associations (the oracle left to right,
the kernel per chunk of blocks), so a draw x that falls within rounding of a
boundary between two cities may legitimately go either way.  Such a step is
accepted only if exact rational arithmetic puts x within 1e-12 (relative to
the total) of the boundary the two sides disagree on.  Everything after the
first such step is not compared for that ant.  At these sizes such a step has
a probability of about 1e-5 per test.
"""
from fractions import Fraction

import numpy as np
import pytest

import aco_instances as inst
import oracle

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _colony(D, alpha, beta, rho, m_max, **kw):
    torch = _torch()
    from paper_2404_04895_amd import Colony
    col = Colony(torch.from_numpy(D).cuda(), alpha, beta, rho, 1.0, m_max, **kw)
    col.set_selection("roulette")
    return col


def _near_boundary(row, visited, x, a, b):
    """Whether exact x lies within 1e-12 of the total from the boundary
    between cities a and b (the cumulative sum up to the smaller of the two)."""
    free = [j for j in range(row.size) if not visited[j]]
    total = sum(Fraction(float(row[j])) for j in free)
    lo = min(a, b)
    cum = sum(Fraction(float(row[j])) for j in free if j <= lo)
    return abs(cum - x) <= Fraction(1, 10**12) * total


def assert_tours_match(P, D, tours, lengths, seed, it, ants):
    o_tours, o_len = oracle.construct(P, D, seed, it, ants, selection="roulette")
    n = D.shape[0]
    for k, a in enumerate(ants):
        t = tours[k]
        assert sorted(t) == list(range(n)), "ant %d: not a permutation" % a
        if np.array_equal(t, o_tours[k]):
            assert lengths[k].view(np.uint32) == o_len[k].view(np.uint32), "ant %d length" % a
            continue
        s = int(np.argmax(t != o_tours[k]))
        visited = np.zeros(n, np.uint8)
        visited[t[:s]] = 1
        row = P[t[s - 1]]
        free = [j for j in range(n) if not visited[j]]
        total = sum(Fraction(float(row[j])) for j in free)
        x = Fraction(oracle.roulette_deviate(seed, it, int(a), s)) * total
        assert _near_boundary(row, visited, x, int(t[s]), int(o_tours[k][s])), (
            "ant %d step %d: gpu %d oracle %d away from any boundary" % (a, s, t[s], o_tours[k][s]))


SCHEDS = ["auto", 0, 1, 2, 3, 4]


@pytest.mark.parametrize("n,m", [(3, 1), (4, 7), (5, 5), (31, 9), (64, 64), (67, 40), (257, 64),
                                 (1000, 24), (1100, 16)])
def test_roulette_construct_matches_oracle(n, m):
    torch = _torch()
    from paper_2404_04895_amd import AcoError
    D = inst.distance_matrix(inst.uniform_cities(n, 2000 + n))
    col = _colony(D, 1.0, 2.0, 0.2, max(m, 2))
    col.transition(1.0)
    col.sync()
    P = col.P().cpu().numpy()
    nblk = (n + 3) // 4
    seed, it = 777 + n, 3
    for sched in SCHEDS:
        if sched != "auto":
            G = {0: 16, 1: 32, 2: 32, 3: 64, 4: 64}[sched]
            col.set_schedule(sched)
            if -(-nblk // G) > G:
                with pytest.raises(AcoError):
                    col.construct(m, seed, it)
                continue
        col.construct(m, seed, it)
        col.sync()
        assert_tours_match(P, D, col.tours(m).cpu().numpy(), col.lengths(m).cpu().numpy(),
                           seed, it, np.arange(m))
    col.close()


def test_roulette_zero_and_subnormal_weights():
    """beta = 40 on clustered cities: P underflows to subnormals and exact
    zeros, so late steps meet rows whose remaining weights are all zero (the
    smallest unvisited city) or tiny."""
    torch = _torch()
    n, m = 300, 48
    D = inst.distance_matrix(inst.clustered_cities(n, 9, 4, 0.02))
    col = _colony(D, 1.0, 40.0, 0.2, m)
    col.transition(1.0)
    col.sync()
    P = col.P().cpu().numpy()
    off = ~np.eye(n, dtype=bool)
    assert np.sum(P[off] == 0) > 0.5 * off.sum()
    assert np.any((P > 0) & (P < np.float32(1.1754944e-38)))
    col.construct(m, 5, 1)
    col.sync()
    assert_tours_match(P, D, col.tours(m).cpu().numpy(), col.lengths(m).cpu().numpy(), 5, 1,
                       np.arange(m))
    col.close()


def test_roulette_free_run_matches_oracle_run():
    torch = _torch()
    n, m, T = 16, 16, 25
    D = inst.distance_matrix(inst.uniform_cities(n, 44))
    col = _colony(D, 1.0, 2.0, 0.3, m, gamma_max=1.0, gamma_min=1.0)
    tour, L = col.run(m, 8, T)
    ref = oracle.run(D, m, 1.0, 2.0, 0.3, 1.0, 8, T, gamma_max=1.0, gamma_min=1.0,
                     selection="roulette")
    assert L == ref["best_len"]
    assert np.array_equal(col.tau().cpu().numpy(), ref["tau"])
    col.close()


def test_selection_switch_and_bad_code():
    torch = _torch()
    from paper_2404_04895_amd import AcoError, _native
    n, m = 40, 8
    D = inst.distance_matrix(inst.uniform_cities(n, 3))
    col = _colony(D, 1.0, 2.0, 0.2, m)
    col.transition(1.0)
    col.sync()
    P = col.P().cpu().numpy()
    col.set_selection("adair")
    col.construct(m, 1, 0)
    col.sync()
    assert np.array_equal(col.tours(m).cpu().numpy(), oracle.construct(P, D, 1, 0, np.arange(m))[0])
    with pytest.raises(AcoError):
        _native.check(_native.lib().aco_set_selection(col._ctx, 7), "aco_set_selection")
    col.close()


def test_roulette_full_size_sampled_clustered_n5000():
    """The benchmark workload's size and launch shape (5000 clustered cities,
    5000 ants, beta 3) with the wheel at gamma = 1; sampled ants against the
    oracle."""
    torch = _torch()
    w = inst.WORKLOADS["clustered-n5000-m5000"]
    D = w.dist(0)
    n, m = w.n, w.m
    col = _colony(D, w.alpha, w.beta, w.rho, m)
    col.transition(1.0)
    col.construct(m, 2, 0)
    col.sync()
    P = col.P().cpu().numpy()
    tours = col.tours(m).cpu().numpy()
    lengths = col.lengths(m).cpu().numpy()
    srt = np.sort(tours, axis=1)
    assert np.array_equal(srt, np.broadcast_to(np.arange(n, dtype=np.int32), srt.shape))
    sample = np.array([0, 1, 2500, 4999])
    assert_tours_match(P, D, tours[sample], lengths[sample], 2, 0, sample)
    col.close()
