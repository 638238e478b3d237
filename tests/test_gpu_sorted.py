"""The sorted walk (ACO_SELECT_ADAIR_SORTED) against the oracle, through the C ABI.

The walk must choose exactly the city the full AdaIR argmax chooses, so the
bar is the plain AdaIR bar: tours and FP32 lengths bit-exact against the
oracle's construct on the same P.  The cases cover the walk's exits:
- the walk decides the step;
- the walk runs out of batches and the scan decides;
- the walk is off (0 batches);
- rows where many entries are exactly 0 or subnormal.
They also cover pheromone that has converged over many iterations, where P is
steep.  The sorted rows themselves are checked as sorted permutations.
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


def _colony(D, alpha, beta, rho, m_max, **kw):
    torch = _torch()
    from paper_2404_04895_amd import Colony
    return Colony(torch.from_numpy(D).cuda(), alpha, beta, rho, 1.0, m_max, **kw)


def _check_sorted_rows(col, P, walk):
    """The kept prefix of every row equals the first K entries of the row
    sorted by (P descending, city ascending), K = 64 * walk rounded up to a
    power of two, at most n; nothing is kept at a walk of 0."""
    Ps, Js = col.sorted_rows()
    n = P.shape[0]
    K = 64
    while K < 64 * walk:
        K *= 2
    K = min(K, n) if walk > 0 else 0
    assert tuple(Ps.shape) == tuple(Js.shape) == (n, K)  # rows are K entries apart
    Ps = Ps.cpu().numpy()
    Js = Js.cpu().numpy().view(np.uint16).astype(np.int64)
    for c in range(n):
        want = np.lexsort((np.arange(n), -P[c].astype(np.float64)))[:K]
        assert np.array_equal(Js[c, :K], want), "row %d" % c
        assert np.array_equal(Ps[c, :K], P[c, want])


@pytest.mark.parametrize("n,m", [(3, 1), (5, 5), (31, 9), (64, 64), (67, 40), (257, 64),
                                 (1000, 24), (1100, 16)])
def test_sorted_walk_bit_exact(n, m):
    torch = _torch()
    D = inst.distance_matrix(inst.uniform_cities(n, 3000 + n))
    col = _colony(D, 1.0, 2.0, 0.2, max(m, 2))
    col.transition(1.5)
    col.sync()
    P = col.P().cpu().numpy()
    seed, it = 99 + n, 5
    o_tours, o_len = oracle.construct(P, D, seed, it, np.arange(m))
    col.set_selection("adair-sorted")
    steps = m * (n - 1)
    lanes = {0: 16, 1: 32, 2: 32, 3: 64, 4: 64}
    auto = 3  # 64 lanes below 4096 ants
    for sched, walk in (("auto", 4), (3, 2), (4, 2), (0, 2), (1, 3), (2, 2), (3, 0), (1, 0),
                        (4, 1), (0, 1), (3, 8), (1, 256)):
        if sched != "auto":
            col.set_schedule(sched)
        G = lanes[auto if sched == "auto" else sched]
        col.set_sorted_walk(walk)
        col.construct(m, seed, it)
        col.sync()
        assert np.array_equal(col.tours(m).cpu().numpy(), o_tours), (sched, walk)
        assert np.array_equal(col.lengths(m).cpu().numpy().view(np.uint32), o_len.view(np.uint32))
        entries, scanned, blocks = col.sorted_walk_stats()
        limit = min(64 * walk, n)
        most = -(-limit // G) * G  # whole batches up to the limit
        if walk == 0:
            assert (entries, scanned) == (0, steps)
        else:
            # every step reads at least one batch; a step that falls to the scan read all it may
            assert entries % G == 0
            assert steps * G <= entries <= steps * most
            assert entries >= steps * G + scanned * (most - G)
        assert 0 <= scanned <= steps
        assert scanned <= blocks <= scanned * ((n + 3) // 4)
        if n <= 300 or walk == 256:
            _check_sorted_rows(col, P, walk)
    col.close()


def test_sorted_walk_converged_pheromone():
    """After 60 iterations tau has concentrated: steep rows, where the walk
    decides early; the tours still equal the oracle's."""
    torch = _torch()
    n, m = 400, 64
    D = inst.distance_matrix(inst.clustered_cities(n, 12, 8, 0.03))
    col = _colony(D, 1.0, 3.0, 0.1, m)
    col.run(m, 3, 60)
    col.transition(1.2)
    col.sync()
    P = col.P().cpu().numpy()
    o_tours, o_len = oracle.construct(P, D, 7, 61, np.arange(m))
    col.set_selection("adair-sorted")
    col.construct(m, 7, 61)
    col.sync()
    assert np.array_equal(col.tours(m).cpu().numpy(), o_tours)
    assert np.array_equal(col.lengths(m).cpu().numpy().view(np.uint32), o_len.view(np.uint32))
    _check_sorted_rows(col, P, 8)  # the default walk
    col.close()


@pytest.mark.parametrize("beta", [2.0, 40.0])
def test_top_k_prefixes_every_size(beta):
    """Every row's kept prefix at K = 64 ... 2048 (one wavefront sorts the K
    selected entries in registers up to K = 1024, the LDS network above), on
    ordinary rows and on rows that are mostly zeros, where the K-th value is
    0 and many entries tie with it (ties go to the smaller city)."""
    torch = _torch()
    n = 2100
    D = inst.distance_matrix(inst.clustered_cities(n, 15, 11, 0.02))
    col = _colony(D, 1.0, beta, 0.2, 8)
    col.set_selection("adair-sorted")
    for walk in (1, 2, 4, 8, 16, 32):
        col.set_sorted_walk(walk)
        col.transition(1.0)
        col.sync()
        P = col.P().cpu().numpy()
        if beta > 2.0:
            assert np.mean(P == 0) > 0.9  # the K-th value is 0 in most rows
        _check_sorted_rows(col, P, walk)
    col.close()


def test_sorted_walk_zero_and_subnormal_rows():
    torch = _torch()
    n, m = 300, 48
    D = inst.distance_matrix(inst.clustered_cities(n, 9, 4, 0.02))
    col = _colony(D, 1.0, 40.0, 0.2, m)
    col.transition(1.0)
    col.sync()
    P = col.P().cpu().numpy()
    off = ~np.eye(n, dtype=bool)
    assert np.sum(P[off] == 0) > 0.5 * off.sum()
    o_tours, o_len = oracle.construct(P, D, 5, 1, np.arange(m))
    col.set_selection("adair-sorted")
    for walk in (2, 64):
        col.set_sorted_walk(walk)
        col.construct(m, 5, 1)
        col.sync()
        assert np.array_equal(col.tours(m).cpu().numpy(), o_tours)
    col.close()


def test_sorted_walk_free_run_and_rejections():
    torch = _torch()
    from paper_2404_04895_amd import AcoError
    n, m, T = 40, 40, 30
    D = inst.distance_matrix(inst.uniform_cities(n, 8))
    col = _colony(D, 1.0, 2.0, 0.3, m)
    col.set_selection("adair-sorted")
    tour, L = col.run(m, 4, T)
    ref = oracle.run(D, m, 1.0, 2.0, 0.3, 1.0, 4, T)
    assert L == ref["best_len"]
    assert np.array_equal(col.tau().cpu().numpy(), ref["tau"])
    with pytest.raises(AcoError):
        col.set_sorted_walk(-1)
    with pytest.raises(AcoError):
        col.set_sorted_walk(257)
    col.close()


def test_sorted_walk_full_size_clustered_n5000():
    """The benchmark workload and launch shape; sampled ants against the oracle."""
    torch = _torch()
    w = inst.WORKLOADS["clustered-n5000-m5000"]
    D = w.dist(0)
    n, m = w.n, w.m
    col = _colony(D, w.alpha, w.beta, w.rho, m)
    col.set_selection("adair-sorted")
    col.transition(1.5)
    col.construct(m, 1, 0)
    col.sync()
    P = col.P().cpu().numpy()
    tours = col.tours(m).cpu().numpy()
    lengths = col.lengths(m).cpu().numpy()
    srt = np.sort(tours, axis=1)
    assert np.array_equal(srt, np.broadcast_to(np.arange(n, dtype=np.int32), srt.shape))
    sample = np.array([0, 1, 2499, 4998, 4999])
    o_tours, o_len = oracle.construct(P, D, 1, 0, sample)
    assert np.array_equal(tours[sample], o_tours)
    assert np.array_equal(lengths[sample].view(np.uint32), o_len.view(np.uint32))
    col.close()


def test_sorted_walk_at_the_benchmarked_state_clustered_n5000():
    """The benchmark workload (5000 clustered cities, 5000 ants, beta 3) driven
    through its first 25 iterations of the 200-iteration gamma schedule, as
    the benchmark does, once on the sorted walk and once on the full scan.
    Every iteration's tours, lengths and pheromone agree bit for bit between
    the two, and 16 ants spread over the colony at iteration 25 (on pheromone
    the benchmark's timed iterations see) equal the oracle's AdaIR argmax
    (Sec. 2.4) on that iteration's P."""
    torch = _torch()
    from paper_2404_04895_amd import gamma_schedule
    w = inst.WORKLOADS["clustered-n5000-m5000"]
    D = w.dist(0)
    n, m, T, iters, seed = w.n, w.m, w.iters, 25, 0
    walk = _colony(D, w.alpha, w.beta, w.rho, m)
    walk.set_selection("adair-sorted")
    scan = _colony(D, w.alpha, w.beta, w.rho, m)
    scan.set_selection("adair")
    for col in (walk, scan):
        col.transition(gamma_schedule(0, T, w.gamma_max, w.gamma_min))
    P_last = None
    for t in range(iters):
        if t == iters - 1:
            walk.sync()
            P_last = walk.P().cpu().numpy()
            assert torch.equal(walk.P(), scan.P())
        for col in (walk, scan):
            col.construct(m, seed, t)
        walk.sync()
        scan.sync()
        assert torch.equal(walk.tours(m), scan.tours(m)), "tours differ at iteration %d" % t
        assert torch.equal(walk.lengths(m), scan.lengths(m)), "lengths differ at iteration %d" % t
        if t == iters - 1:
            tours = walk.tours(m).cpu().numpy()
            lengths = walk.lengths(m).cpu().numpy()
        for col in (walk, scan):
            col.update(gamma_schedule(t + 1, T, w.gamma_max, w.gamma_min))
        walk.sync()
        scan.sync()
        assert torch.equal(walk.tau(), scan.tau()), "tau differs after iteration %d" % t
    entries, scanned, _ = walk.sorted_walk_stats()
    # the walk really decided most steps (converging pheromone, steep rows)
    assert scanned < 0.05 * iters * m * (n - 1), scanned
    sample = np.linspace(0, m - 1, 16).astype(np.int64)
    o_tours, o_len = oracle.construct(P_last, D, seed, iters - 1, sample)
    assert np.array_equal(tours[sample], o_tours)
    assert np.array_equal(lengths[sample].view(np.uint32), o_len.view(np.uint32))
    _, best_walk, it_walk = walk.best()
    _, best_scan, it_scan = scan.best()
    assert best_walk == best_scan and it_walk == it_scan
    walk.close()
    scan.close()
