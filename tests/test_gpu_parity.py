"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: tours, start cities and FP32 tour lengths bit-exact given the same P;
pheromone bit-exact (integer deposit, one FP64 fma, one rounding); P within
1e-5 relative (FP64 exp/log of two different math libraries, one FP32
rounding), the tolerance the target states for FP32 matrices.
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


def assert_P_close(P_gpu, P_ref, what=""):
    P_gpu = np.asarray(P_gpu, np.float64)
    P_ref = np.asarray(P_ref, np.float64)
    bound = 1e-5 * np.maximum(np.abs(P_ref), float(FLT_MIN))
    bad = np.abs(P_gpu - P_ref) > bound
    assert not bad.any(), "%s: %d entries differ; worst %s" % (
        what, int(bad.sum()), np.max(np.abs(P_gpu - P_ref) / np.maximum(np.abs(P_ref), 1e-300)))


def _host(col, m):
    return (col.P().cpu().numpy(), col.tau().cpu().numpy(), col.tours(m).cpu().numpy(),
            col.lengths(m).cpu().numpy())


# --------------------------------------------------------------------------
def test_uniforms_bit_exact():
    torch = _torch()
    from paper_2404_04895_amd import uniforms
    for (seed, t, a, s, count) in [(0, 0, 0, 1, 64), (2**40 + 17, 3, 4999, 4998, 5003),
                                   (7, 2**31, 12, 1, 257), (0xFFFFFFFFFFFFFFFF, 9, 1, 2, 33)]:
        got = uniforms(seed, t, a, s, count).cpu().numpy()
        want = np.array([oracle.uniform(seed, t, a, s, j) for j in range(count)], np.float32)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), (seed, t, a, s)


@pytest.mark.parametrize("n", [3, 5, 64, 67, 300])
def test_transition_matches_oracle(n):
    torch = _torch()
    D = inst.distance_matrix(inst.uniform_cities(n, n))
    col = _colony(D, 1.0, 2.0, 0.3, 1.0, 4)
    for gamma in (1.0, 1.5, 0.8):
        col.transition(gamma)
        col.sync()
        P = col.P_padded().cpu().numpy()
        assert np.all(P[:, n:] == 0.0) and np.all(np.diag(P[:, :n]) == 0.0)
        ref = oracle.transition(col.tau().cpu().numpy(), D, 1.0, 2.0, gamma)
        assert_P_close(P[:, :n], ref, "n=%d gamma=%g" % (n, gamma))
    col.close()


@pytest.mark.parametrize("alpha,beta", [(1.0, 3.0), (0.0, 6.0), (2.0, 4.0), (6.0, 0.0),
                                        (1.0, 6.0), (1.5, 2.5), (0.5, 1.0)])
def test_transition_forms_match_oracle(alpha, beta):
    """The row update forms W by multiplication when alpha and beta are
    integers with alpha + beta <= 6 and through logarithms otherwise (the
    first four cases, then three of the other); both must give the oracle's P
    on pheromone spread over twelve decades, with an FP32 extreme (the largest
    finite value, the smallest normal or a subnormal) planted in every row."""
    torch = _torch()
    n = 131
    D = inst.distance_matrix(inst.uniform_cities(n, 7))
    col = _colony(D, alpha, beta, 0.3, 1.0, 4)
    rng = np.random.default_rng(11)
    tau = np.zeros((n, col.ld), np.float32)
    tau[:, :n] = (10.0 ** rng.uniform(-6.0, 6.0, (n, n))).astype(np.float32)
    for k, v in enumerate((np.finfo(np.float32).max, FLT_MIN, np.float32(1e-44))):
        rows = np.arange(k, n, 3)
        tau[rows, (rows + 1 + 17 * k) % n] = v
    tau[np.arange(n), np.arange(n)] = 0.0
    col.set_state(torch.from_numpy(tau), 0)
    for gamma in (1.0, 1.5, 0.7, 4.0):
        col.transition(gamma)
        col.sync()
        P = col.P_padded().cpu().numpy()
        assert np.all(P[:, n:] == 0.0) and np.all(np.diag(P[:, :n]) == 0.0)
        ref = oracle.transition(tau[:, :n].copy(), D, alpha, beta, gamma)
        assert_P_close(P[:, :n], ref, "alpha=%g beta=%g gamma=%g" % (alpha, beta, gamma))
    col.close()


@pytest.mark.parametrize("n,m", [(3, 1), (4, 7), (5, 5), (31, 9), (50, 50), (64, 64), (67, 40),
                                 (256, 33), (257, 64), (1000, 24)])
def test_construct_bit_exact(n, m):
    torch = _torch()
    D = inst.distance_matrix(inst.uniform_cities(n, 1000 + n))
    col = _colony(D, 1.0, 2.0, 0.2, 1.0, max(m, 2))
    col.transition(1.5)
    seed, it = 12345 + n, 7
    col.construct(m, seed, it)
    col.sync()
    P, _, tours, lengths = _host(col, m)
    o_tours, o_len = oracle.construct(P, D, seed, it, np.arange(m))
    for a in range(m):
        assert sorted(tours[a]) == list(range(n))
        assert tours[a, 0] == oracle.start_city(seed, it, a, n)
    assert np.array_equal(tours, o_tours)
    assert np.array_equal(lengths.view(np.uint32), o_len.view(np.uint32))
    col.close()


@pytest.mark.parametrize("elite_k", [0, 5])
def test_update_matches_oracle(elite_k):
    torch = _torch()
    n, m, rho, Q = 97, 29, 0.25, 2.0
    D = inst.distance_matrix(inst.clustered_cities(n, 5, 6, 0.05))
    col = _colony(D, 1.0, 3.0, rho, Q, m, elite_k=elite_k)
    S = oracle.deposit_scale(D, m, Q)
    assert col.deposit_scale == S
    col.transition(1.5)
    for it in range(4):
        col.construct(m, 99, it)
        col.sync()
        P, tau_prev, tours, lengths = _host(col, m)
        o_tours, o_len = oracle.construct(P, D, 99, it, np.arange(m))
        assert np.array_equal(tours, o_tours) and np.array_equal(lengths, o_len)
        col.update(1.25)
        col.sync()
        elite = oracle.elite(lengths, elite_k)
        delta = oracle.deposit(tours, lengths, elite, Q, S)
        tau_ref = oracle.evaporate(tau_prev, delta, rho, S)
        tau_gpu = col.tau().cpu().numpy()
        assert np.array_equal(tau_gpu.view(np.uint32), tau_ref.view(np.uint32)), it
        assert np.all(col.tau_padded().cpu().numpy()[:, n:] == 0)
        assert_P_close(col.P().cpu().numpy(), oracle.transition(tau_ref, D, 1.0, 3.0, 1.25),
                       "update it=%d" % it)
    col.close()


def _stepwise(D, w, m, T, seed, elite_k=0):
    from paper_2404_04895_amd import gamma_schedule
    n = D.shape[0]
    col = _colony(D, w.alpha, w.beta, w.rho, w.Q, m, elite_k=elite_k)
    S = oracle.deposit_scale(D, m, w.Q)
    col.transition(gamma_schedule(0, T, w.gamma_max, w.gamma_min))
    col.sync()
    P_cur = col.P().cpu().numpy()
    tau_cur = col.tau().cpu().numpy()
    assert_P_close(P_cur, oracle.transition(tau_cur, D, w.alpha, w.beta,
                                            oracle.gamma(0, T, w.gamma_max, w.gamma_min)), "P0")
    best = (math.inf, -1, None)
    for t in range(T):
        g_next = gamma_schedule(t + 1, T, w.gamma_max, w.gamma_min)
        assert g_next == oracle.gamma(t + 1, T, w.gamma_max, w.gamma_min)
        col.construct(m, seed, t)
        col.update(g_next)
        col.sync()
        tours = col.tours(m).cpu().numpy()
        lengths = col.lengths(m).cpu().numpy()
        o_tours, o_len = oracle.construct(P_cur, D, seed, t, np.arange(m))
        assert np.array_equal(tours, o_tours), "tours differ at iteration %d" % t
        assert np.array_equal(lengths, o_len), "lengths differ at iteration %d" % t
        a = int(np.lexsort((np.arange(m), lengths))[0])
        if lengths[a] < best[0]:
            best = (float(lengths[a]), t, tours[a].copy())
        delta = oracle.deposit(tours, lengths, oracle.elite(lengths, elite_k), w.Q, S)
        tau_ref = oracle.evaporate(tau_cur, delta, w.rho, S)
        tau_cur = col.tau().cpu().numpy()
        assert np.array_equal(tau_cur, tau_ref), "tau differs at iteration %d" % t
        P_cur = col.P().cpu().numpy()
        assert_P_close(P_cur, oracle.transition(tau_ref, D, w.alpha, w.beta, g_next),
                       "P at iteration %d" % t)
    tour_b, len_b, it_b = col.best()
    assert len_b == best[0] and it_b == best[1] and np.array_equal(tour_b, best[2])
    col.close()
    return best


def test_run_stepwise_small_workload():
    """50 uniform cities, 50 ants, rho 0.5, 100 iterations (the small workload),
    iteration by iteration against the oracle."""
    _torch()
    w = inst.WORKLOADS["uniform-n50-m50"]
    best = _stepwise(w.dist(0), w, w.m, w.iters, 0)
    opt_lb = oracle.length_lower_bound(w.dist(0))
    assert best[0] >= opt_lb


def test_run_stepwise_elite_ragged():
    _torch()
    w = inst.Workload("ragged", 77, 30, 1.0, 2.0, 0.2, 1.0, 12, elite_k=7)
    _stepwise(w.dist(3), w, 30, 12, 5, elite_k=7)


def test_free_run_matches_oracle_run():
    """aco_run against oracle_run end to end on a tiny instance (P computed
    independently on each side every iteration)."""
    torch = _torch()
    n, m, T = 12, 12, 30
    D = inst.distance_matrix(inst.uniform_cities(n, 21))
    col = _colony(D, 1.0, 2.0, 0.3, 1.0, m)
    tour, L = col.run(m, 4, T)
    ref = oracle.run(D, m, 1.0, 2.0, 0.3, 1.0, 4, T)
    assert L == ref["best_len"]
    assert np.array_equal(col.tau().cpu().numpy(), ref["tau"])
    exact, _ = oracle.tsp_exact(D)
    assert L >= np.float32(exact) * (1 - 1e-6)
    col.close()


def test_determinism_and_resume():
    """Two runs are bitwise identical; a run checkpointed after 5 iterations and
    resumed equals the uninterrupted run (the generator is stateless)."""
    torch = _torch()
    n, m = 130, 40
    D = inst.distance_matrix(inst.uniform_cities(n, 8))
    a = _colony(D, 1.0, 2.0, 0.1, 1.0, m)
    ta, La = a.run(m, 77, 12)
    tau_a = a.tau().cpu().numpy()
    b = _colony(D, 1.0, 2.0, 0.1, 1.0, m)
    tb, Lb = b.run(m, 77, 12)
    assert La == Lb and np.array_equal(ta, tb) and np.array_equal(tau_a, b.tau().cpu().numpy())
    # resume: 12 iterations as one schedule = construct/update driven by hand
    from paper_2404_04895_amd import gamma_schedule
    c = _colony(D, 1.0, 2.0, 0.1, 1.0, m)
    c.transition(gamma_schedule(0, 12, 1.5, 1.0))
    for t in range(5):
        c.construct(m, 77, t)
        c.update(gamma_schedule(t + 1, 12, 1.5, 1.0))
    state, it = c.get_state()
    c.close()
    d = _colony(D, 1.0, 2.0, 0.1, 1.0, m)
    d.set_state(state, 5)
    d.transition(gamma_schedule(5, 12, 1.5, 1.0))
    for t in range(5, 12):
        d.construct(m, 77, t)
        d.update(gamma_schedule(t + 1, 12, 1.5, 1.0))
    d.sync()
    assert np.array_equal(d.tau().cpu().numpy(), tau_a)
    for x in (a, b, d):
        x.close()


def test_exponents_zero_uniform_choice():
    """alpha = beta = 0: P is uniform, so step-1 choices are uniform over the
    unvisited cities (chi-square over many ants)."""
    torch = _torch()
    from scipy import stats
    n, m = 8, 4000
    D = inst.distance_matrix(inst.uniform_cities(n, 2))
    col = _colony(D, 0.0, 0.0, 0.5, 1.0, m)
    col.transition(1.0)
    col.construct(m, 3, 0)
    col.sync()
    assert_P_close(col.P().cpu().numpy(), np.where(np.eye(n, dtype=bool), 0, np.float32(1 / 7)))
    tours = col.tours(m).cpu().numpy()
    rel = (tours[:, 1] - tours[:, 0]) % n
    counts = np.bincount(rel, minlength=n)[1:]
    assert stats.chisquare(counts).pvalue > 1e-4
    col.close()


def test_eta_input_and_fallback():
    torch = _torch()
    n, m = 40, 10
    D = inst.distance_matrix(inst.uniform_cities(n, 6))
    eta = np.where(np.eye(n, dtype=bool), 0.0, 1.0 / np.where(D > 0, D, 1)).astype(np.float32)
    col = _colony(D, 1.0, 2.0, 0.3, 1.0, m)
    col.transition(1.0)
    P_plain = col.P().cpu().numpy()
    assert col.set_eta(eta) is True
    col.transition(1.0)
    assert_P_close(col.P().cpu().numpy(), oracle.transition(col.tau().cpu().numpy(), D, 1.0, 2.0,
                                                            1.0, eta=eta), "eta")
    assert_P_close(col.P().cpu().numpy(), P_plain, "eta=1/d vs plain")
    learned = (eta * np.random.default_rng(0).uniform(0.5, 2.0, eta.shape)).astype(np.float32)
    assert col.set_eta(learned) is True
    col.transition(1.0)
    assert_P_close(col.P().cpu().numpy(), oracle.transition(col.tau().cpu().numpy(), D, 1.0, 2.0,
                                                            1.0, eta=learned), "learned eta")
    bad = learned.copy()
    bad[3, 7] = np.nan
    assert col.set_eta(bad) is False
    col.transition(1.0)
    assert_P_close(col.P().cpu().numpy(), P_plain, "fallback")
    col.close()


def test_bad_inputs_rejected():
    torch = _torch()
    from paper_2404_04895_amd import AcoError
    n = 10
    D = inst.distance_matrix(inst.uniform_cities(n, 3))
    asym = D.copy(); asym[1, 2] *= 1.5
    nan = D.copy(); nan[4, 5] = nan[5, 4] = np.nan
    zero = D.copy(); zero[2, 3] = zero[3, 2] = 0.0
    diag = D.copy(); diag[6, 6] = 1.0
    for bad in (asym, nan, zero, diag):
        with pytest.raises(AcoError) as e:
            _colony(bad, 1.0, 2.0, 0.5, 1.0, 4)
        assert e.value.status == -1
    col = _colony(D, 1.0, 2.0, 0.5, 1.0, 4)
    with pytest.raises(AcoError) as e:
        col.construct(4, 0, 0)          # no P yet
    assert e.value.status == -4
    col.transition(1.0)
    with pytest.raises(AcoError) as e:
        col.update(1.0)                 # no construct yet
    assert e.value.status == -4
    with pytest.raises(AcoError) as e:
        col.construct(5, 0, 0)          # m > m_max
    assert e.value.status == -1
    col.close()


def test_full_size_sampled_clustered_n5000():
    """The benchmark's workload and launch shape (5000 clustered cities, 5000
    ants, beta 3): the oracle rebuilds sampled ants and rows one by one."""
    torch = _torch()
    w = inst.WORKLOADS["clustered-n5000-m5000"]
    D = w.dist(0)
    n, m = w.n, w.m
    col = _colony(D, w.alpha, w.beta, w.rho, w.Q, m)
    col.transition(1.5)
    col.construct(m, 1, 0)
    col.sync()
    P = col.P().cpu().numpy()
    tours = col.tours(m).cpu().numpy()
    lengths = col.lengths(m).cpu().numpy()
    tau_prev = col.tau().cpu().numpy()
    # every tour is a permutation
    srt = np.sort(tours, axis=1)
    assert np.array_equal(srt, np.broadcast_to(np.arange(n, dtype=np.int32), srt.shape))
    sample = np.array([0, 1, 2499, 4998, 4999])
    o_tours, o_len = oracle.construct(P, D, 1, 0, sample)
    assert np.array_equal(tours[sample], o_tours)
    assert np.array_equal(lengths[sample], o_len)
    col.update(1.4)
    col.sync()
    tau_gpu = col.tau().cpu().numpy()
    P_gpu = col.P().cpu().numpy()
    S = col.deposit_scale
    assert S == oracle.deposit_scale(D, m, w.Q)
    delta = oracle.deposit(tours, lengths, None, w.Q, S)
    total_q = sum(oracle.deposit_weight(L, w.Q, S) for L in lengths)
    assert int(delta.sum(dtype=object)) == 2 * n * total_q
    tau_ref = oracle.evaporate(tau_prev, delta, w.rho, S)
    del delta
    assert np.array_equal(tau_gpu.view(np.uint32), tau_ref.view(np.uint32))
    assert_P_close(P_gpu, oracle.transition(tau_ref, D, w.alpha, w.beta, 1.4), "P n=5000")
    col.close()


@pytest.mark.parametrize("selection", ["adair", "adair-sorted"])
def test_free_run_matches_oracle_under_the_greedier_schedule(selection):
    """The alternative gamma schedule the design discusses (cosine 1.0 -> 0.5,
    so P is raised to powers up to 2): aco_run against oracle_run, best tour,
    best length and pheromone bit for bit, under both AdaIR constructs."""
    torch = _torch()
    n, m, T = 60, 60, 24
    D = inst.distance_matrix(inst.clustered_cities(n, 31, 4, 0.05))
    col = _colony(D, 1.0, 2.0, 0.2, 1.0, m, gamma_max=1.0, gamma_min=0.5)
    col.set_selection(selection)
    tour, L = col.run(m, 9, T)
    ref = oracle.run(D, m, 1.0, 2.0, 0.2, 1.0, 9, T, gamma_max=1.0, gamma_min=0.5)
    assert L == np.float32(ref["best_len"])
    assert np.array_equal(tour, ref["best_tour"])
    assert np.array_equal(col.tau().cpu().numpy(), ref["tau"])
    assert_P_close(col.P().cpu().numpy(), ref["P"], "gamma 1.0 -> 0.5, " + selection)
    col.close()
