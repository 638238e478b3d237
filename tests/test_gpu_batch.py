"""Construct schedules and the batched engine, through the C ABI.

Every construct schedule (lanes per ant, live-block list) must give the same
tours bit for bit, and every member of a batch must evolve exactly as the same
instance run alone -- which the single-instance parity tests tie to the oracle.
"""
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


@pytest.mark.parametrize("n", [3, 5, 31, 64, 65, 128, 129, 300, 1030])
def test_every_schedule_builds_the_same_tours(n):
    torch = _torch()
    from paper_2404_04895_amd import SCHEDULES, Colony
    D = inst.distance_matrix(inst.uniform_cities(n, 40 + n))
    m = 37
    ref = None
    col = Colony(torch.from_numpy(D).cuda(), 1.0, 2.0, 0.3, 1.0, m)
    col.transition(1.5)
    P = col.P().cpu().numpy()
    for sched in SCHEDULES:
        col.set_schedule(sched)
        col.construct(m, 9 + n, 3)
        col.sync()
        got = (col.tours(m).cpu().numpy().copy(), col.lengths(m).cpu().numpy().copy())
        if ref is None:
            ref = got
            o_tours, o_len = oracle.construct(P, D, 9 + n, 3, np.arange(m))
            assert np.array_equal(got[0], o_tours) and np.array_equal(got[1], o_len)
        else:
            assert np.array_equal(got[0], ref[0]), "schedule %d" % sched
            assert np.array_equal(got[1], ref[1]), "schedule %d" % sched
    col.close()


def _batch_instances():
    ns = [3, 4, 7, 16, 50, 63, 64, 65, 100, 128, 129, 250, 257, 400]
    ms = [n if k % 3 else max(1, n // 2 + 3) for k, n in enumerate(ns)]
    seeds = [1000 + 7 * k for k in range(len(ns))]
    dists = [inst.distance_matrix(inst.uniform_cities(n, 500 + k)) for k, n in enumerate(ns)]
    return ns, ms, seeds, dists


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_independent_runs(use_graph):
    torch = _torch()
    from paper_2404_04895_amd import Batch, Colony
    ns, ms, seeds, dists = _batch_instances()
    T, alpha, beta, rho, elite_k = 9, 1.0, 2.0, 0.2, 5
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = Batch(dists, alpha, beta, rho, 1.0, ants=ms, seeds=seeds, elite_k=elite_k,
                  stream=stream)
        b.run(T, use_graph=use_graph)
        lens, its, tours = b.best()
        for i, n in enumerate(ns):
            col = Colony(torch.from_numpy(dists[i]).cuda(), alpha, beta, rho, 1.0, ms[i],
                         elite_k=min(elite_k, ms[i]), stream=stream)
            tour, L = col.run(ms[i], seeds[i], T)
            _, _, it = col.best()
            assert L == lens[i] and it == its[i], (i, n)
            assert np.array_equal(tour, tours[i]), (i, n)
            assert np.array_equal(col.tau().cpu().numpy(), b.tau(i).cpu().numpy()), (i, n)
            assert np.array_equal(col.P().cpu().numpy(), b.P(i).cpu().numpy()), (i, n)
            assert sorted(tours[i]) == list(range(n))
            assert oracle.tour_length(tours[i], dists[i]) == lens[i]
            col.close()
        b.close()
    stream.synchronize()


def test_batch_schedule_tables_do_not_change_results():
    """Every table gives the same results bit for bit, the sorted walk's
    (ACO_SCHED_SORTED: rows sorted in each update) included, with graph replay
    and with direct launches."""
    torch = _torch()
    from paper_2404_04895_amd import (Batch, SCHED_G16, SCHED_G32, SCHED_G32_LIVE, SCHED_G64,
                                      SCHED_G64_LIVE, SCHED_SORTED)
    ns, ms, seeds, dists = _batch_instances()
    stream = torch.cuda.Stream()
    outs = []
    with torch.cuda.stream(stream):
        for table, waves, graph in [
                ([], 0, True), ([(64, SCHED_G64), (10**6, SCHED_G64_LIVE)], 97, True),
                ([(400, SCHED_G32_LIVE)], 1, True), ([(10**6, SCHED_G16)], 4096, True),
                ([(1024, SCHED_G32 | SCHED_SORTED)], 0, True),
                ([(64, SCHED_G16 | SCHED_SORTED), (128, SCHED_G64),
                  (400, SCHED_G64 | SCHED_SORTED)], 200, False),
                ([(100, SCHED_G16), (1024, SCHED_G16 | SCHED_SORTED)], 4096, True)]:
            b = Batch(dists, 1.0, 3.0, 0.1, 1.0, ants=ms, seeds=seeds, stream=stream)
            b.set_schedules(table, waves)
            b.run(5, use_graph=graph)
            lens, its, tours = b.best()
            taus = [b.tau(i).cpu().numpy().copy() for i in range(len(ns))]
            outs.append((lens, its, tours, taus))
            b.close()
    for lens, its, tours, taus in outs[1:]:
        assert np.array_equal(lens, outs[0][0]) and np.array_equal(its, outs[0][1])
        for i in range(len(ns)):
            assert np.array_equal(tours[i], outs[0][2][i])
            assert np.array_equal(taus[i], outs[0][3][i])


def test_batch_sorted_flag_rejected_where_not_allowed():
    torch = _torch()
    from paper_2404_04895_amd import (AcoError, Batch, BATCH_SORTED_MAX_N, SCHED_G32_LIVE,
                                      SCHED_G64, SCHED_SORTED)
    ns, ms, seeds, dists = _batch_instances()
    b = Batch(dists[:4], 1.0, 2.0, 0.2, 1.0, ants=ms[:4], seeds=seeds[:4])
    for table in ([(64, SCHED_G32_LIVE | SCHED_SORTED)],
                  [(BATCH_SORTED_MAX_N + 1, SCHED_G64 | SCHED_SORTED)],
                  [(64, 5 | SCHED_SORTED)]):
        with pytest.raises(AcoError):
            b.set_schedules(table, 0)
    b.set_schedules([(BATCH_SORTED_MAX_N, SCHED_G64 | SCHED_SORTED)], 0)
    assert b.view(3).schedule == SCHED_G64 | SCHED_SORTED
    b.close()


def test_batch_sorted_walk_large_members():
    """Members of 513 to 1024 cities on the sorted walk (their rows are sorted
    with 16 entries per lane): the same results as the full scan, bit for bit."""
    torch = _torch()
    from paper_2404_04895_amd import (BATCH_SORTED_MAX_N, Batch, SCHED_G32, SCHED_G64_LIVE,
                                      SCHED_SORTED)
    ns = [700, BATCH_SORTED_MAX_N, 90]
    ms = [24, 16, 20]
    seeds = [11, 12, 13]
    dists = [inst.distance_matrix(inst.uniform_cities(n, 900 + k)) for k, n in enumerate(ns)]
    outs = []
    for table in ([(10**6, SCHED_G64_LIVE)], [(BATCH_SORTED_MAX_N, SCHED_G32 | SCHED_SORTED)]):
        b = Batch(dists, 1.0, 2.0, 0.2, 1.0, ants=ms, seeds=seeds)
        b.set_schedules(table, 0)
        b.run(3, use_graph=False)
        lens, its, tours = b.best()
        outs.append((lens, its, tours, [b.tau(i).cpu().numpy().copy() for i in range(3)]))
        b.close()
    (l0, i0, t0, tau0), (l1, i1, t1, tau1) = outs
    assert np.array_equal(l0, l1) and np.array_equal(i0, i1)
    for i in range(3):
        assert np.array_equal(t0[i], t1[i]) and np.array_equal(tau0[i], tau1[i]), i


def test_batch_sorted_walk_counts():
    """The members on the sorted walk report what their walks read: whole
    batches of their group width, at least one per step, reset by the read."""
    torch = _torch()
    from paper_2404_04895_amd import Batch, SCHED_G16, SCHED_G64, SCHED_SORTED
    ns, ms, seeds, dists = _batch_instances()
    b = Batch(dists, 1.0, 2.0, 0.2, 1.0, ants=ms, seeds=seeds)
    b.set_schedules([(100, SCHED_G16), (1024, SCHED_G64 | SCHED_SORTED)], 0)
    iters = 3
    b.run(iters, use_graph=False)
    entries, scanned, blocks = b.sorted_walk_stats()
    steps = sum(m * (n - 1) for n, m in zip(ns, ms) if n > 100) * iters
    assert entries % 64 == 0 and entries >= steps * 64
    assert 0 <= scanned <= steps and blocks >= scanned
    assert b.sorted_walk_stats() == (0, 0, 0)
    b.set_schedules([(10**6, SCHED_G16)], 0)
    b.run(1, use_graph=False)
    assert b.sorted_walk_stats() == (0, 0, 0)  # no member on the walk
    b.close()


def test_batch_consecutive_runs_continue_the_counter():
    """Two runs of 3 iterations continue the generator's iteration counter and
    the pheromone state: they equal a single-instance colony driven the same way."""
    torch = _torch()
    from paper_2404_04895_amd import Batch, Colony
    ns, ms, seeds, dists = _batch_instances()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = Batch(dists[:5], 1.0, 2.0, 0.3, 1.0, ants=ms[:5], seeds=seeds[:5], stream=stream)
        b.run(3)
        b.run(3)
        lens, _, _ = b.best()
        for i in range(5):
            col = Colony(torch.from_numpy(dists[i]).cuda(), 1.0, 2.0, 0.3, 1.0, ms[i],
                         stream=stream)
            col.run(ms[i], seeds[i], 3)
            _, L = col.run(ms[i], seeds[i], 3)
            assert L == lens[i]
            assert np.array_equal(col.tau().cpu().numpy(), b.tau(i).cpu().numpy())
            col.close()
        b.close()
    stream.synchronize()
