"""Every member of a batch against the oracle's whole run, through the C ABI.

A batch advances many instances in persistent launches, with its own row
update (64 threads per row) and a captured graph per iteration.  Each member
must still compute the paper's iteration exactly: transition (Sec. 2.1
Eq. (1) with the AdaIR exponent of Eq. (4)), AdaIR construction (Sec. 2.2,
Sec. 2.4), elite top-k and index-mapped deposit (Sec. 2.3 Eq. (2)-(3)),
evaporation.  So after T iterations each member's best length, best
iteration and best tour equal the oracle's, its pheromone equals the
oracle's bit for bit, and its P is within 1e-5 relative.
"""
import numpy as np
import pytest

import aco_instances as inst
import oracle

pytestmark = pytest.mark.gpu

T = 8
ALPHA, BETA, RHO, Q, ELITE_K = 1.0, 2.0, 0.2, 1.0, 5

# Members of uneven size: tiny, wavefront-ragged, and up to ~500 cities (the
# largest size of the batched workload).
NS = [3, 7, 50, 64, 65, 97, 130, 190, 257, 300, 420, 497]


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _members():
    ms = [n if k % 3 else max(1, n // 2 + 3) for k, n in enumerate(NS)]
    seeds = [3000 + 11 * k for k in range(len(NS))]
    dists = [inst.distance_matrix(inst.uniform_cities(n, 700 + k)) for k, n in enumerate(NS)]
    return ms, seeds, dists


def _tables():
    from paper_2404_04895_amd import (SCHED_G16, SCHED_G32, SCHED_G32_LIVE, SCHED_G64,
                                      SCHED_G64_LIVE, SCHED_SORTED)
    from paper_2404_04895_amd.autotune import load_table
    committed, waves = load_table()
    assert committed, "the committed schedule table is missing"
    every = [(7, SCHED_G16), (64, SCHED_G32), (97, SCHED_G64), (130, SCHED_G32_LIVE),
             (190, SCHED_G64_LIVE), (257, SCHED_G16 | SCHED_SORTED),
             (300, SCHED_G32 | SCHED_SORTED), (1024, SCHED_G64 | SCHED_SORTED)]
    return [("committed", committed, waves), ("every-schedule", every, 200)]


_ORACLE = {}


def _oracle_runs():
    if not _ORACLE:
        ms, seeds, dists = _members()
        for i, n in enumerate(NS):
            _ORACLE[i] = oracle.run(dists[i], ms[i], ALPHA, BETA, RHO, Q, seeds[i], T,
                                    elite_k=min(ELITE_K, ms[i]))
    return _ORACLE


@pytest.mark.parametrize("table_name", ["committed", "every-schedule"])
def test_batch_members_equal_oracle_run(table_name):
    torch = _torch()
    from paper_2404_04895_amd import Batch
    ms, seeds, dists = _members()
    name, table, waves = [t for t in _tables() if t[0] == table_name][0]
    ref = _oracle_runs()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = Batch(dists, ALPHA, BETA, RHO, Q, ants=ms, seeds=seeds, elite_k=ELITE_K,
                  stream=stream)
        b.set_schedules(table, waves)
        scheds = [b.view(i).schedule for i in range(len(NS))]
        b.run(T, use_graph=True)
        lens, its, tours = b.best()
        for i, n in enumerate(NS):
            o = ref[i]
            tag = "%s member %d (n=%d, m=%d, schedule %d)" % (name, i, n, ms[i], scheds[i])
            assert lens[i] == np.float32(o["best_len"]), tag
            assert its[i] == o["best_iter"], tag
            assert np.array_equal(tours[i], o["best_tour"]), tag
            assert np.array_equal(b.tau(i).cpu().numpy(), o["tau"]), tag
            P = b.P(i).cpu().numpy().astype(np.float64)
            Po = o["P"].astype(np.float64)
            assert np.all(np.abs(P - Po) <= 1e-5 * np.abs(Po)), tag
        b.close()
    stream.synchronize()
    if name == "every-schedule":
        # the table puts members on all five full-scan schedules and all three
        # sorted-walk widths
        assert len(set(scheds)) == 8, scheds


def test_batch_members_equal_oracle_run_under_the_greedier_schedule():
    """The same check under the alternative gamma schedule (cosine 1.0 ->
    0.5), for a few members spanning the schedule table (tiny, full scan,
    sorted walk)."""
    torch = _torch()
    from paper_2404_04895_amd import Batch
    from paper_2404_04895_amd.autotune import load_table
    pick = [0, 4, 8, 11]  # n = 3, 65, 257, 497
    ms, seeds, dists = _members()
    ms = [ms[i] for i in pick]
    seeds = [seeds[i] + 1 for i in pick]
    dists = [dists[i] for i in pick]
    table, waves = load_table()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = Batch(dists, ALPHA, BETA, RHO, Q, ants=ms, seeds=seeds, elite_k=ELITE_K,
                  gamma_max=1.0, gamma_min=0.5, stream=stream)
        b.set_schedules(table, waves)
        b.run(T, use_graph=True)
        lens, its, tours = b.best()
        for k, D in enumerate(dists):
            o = oracle.run(D, ms[k], ALPHA, BETA, RHO, Q, seeds[k], T,
                           elite_k=min(ELITE_K, ms[k]), gamma_max=1.0, gamma_min=0.5)
            tag = "member n=%d, m=%d, schedule %d" % (D.shape[0], ms[k], b.view(k).schedule)
            assert lens[k] == np.float32(o["best_len"]), tag
            assert its[k] == o["best_iter"], tag
            assert np.array_equal(tours[k], o["best_tour"]), tag
            assert np.array_equal(b.tau(k).cpu().numpy(), o["tau"]), tag
            P = b.P(k).cpu().numpy().astype(np.float64)
            Po = o["P"].astype(np.float64)
            assert np.all(np.abs(P - Po) <= 1e-5 * np.abs(Po)), tag
        b.close()
    stream.synchronize()
