"""The largest supported instance, n = ACO_MAX_CITIES = 16384, through the C ABI.

At this size the update keeps a 131 KB FP64 row in LDS, the whole-row sort
uses 96 KB, and every construct schedule's per-ant lists are at their
longest.  Four ants; the oracle rebuilds two of them one by one.  The bars
are the usual ones: tours and lengths bit-exact given the same P (for the
Roulette Wheel, up to a draw within rounding of a boundary); τ bit-exact after
the update; sampled rows of the next P within 1e-5.
"""
import numpy as np
import pytest

import aco_instances as inst
import oracle

pytestmark = pytest.mark.gpu

FLT_MIN = np.float32(1.1754944e-38)


def test_max_size_n16384():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_04895_amd import MAX_CITIES, Colony
    from test_gpu_roulette import assert_tours_match
    n, m = MAX_CITIES, 4
    assert n == 16384
    D = inst.distance_matrix(inst.uniform_cities(n, 77))
    col = Colony(torch.from_numpy(D).cuda(), 1.0, 2.0, 0.1, 1.0, m)
    sample = np.array([0, 3])
    seed = 5
    # walk 8 keeps K = 512 entries per row (top-K from a row staged in LDS),
    # 128 keeps 8192 (top-K reading the row from global memory), 256 sorts
    # whole rows
    for selection, gamma, walk in (("adair", 1.5, None), ("adair-sorted", 1.5, 8),
                                   ("adair-sorted", 1.5, 128), ("adair-sorted", 1.5, 256),
                                   ("roulette", 1.0, None)):
        col.set_selection(selection)
        if walk is not None:
            col.set_sorted_walk(walk)
        col.transition(gamma)
        col.construct(m, seed, 0)
        col.sync()
        P = col.P().cpu().numpy()
        tours = col.tours(m).cpu().numpy()
        lengths = col.lengths(m).cpu().numpy()
        srt = np.sort(tours, axis=1)
        assert np.array_equal(srt, np.broadcast_to(np.arange(n, dtype=np.int32), srt.shape))
        if selection == "roulette":
            assert_tours_match(P, D, tours[sample], lengths[sample], seed, 0, sample)
        else:
            o_tours, o_len = oracle.construct(P, D, seed, 0, sample)
            assert np.array_equal(tours[sample], o_tours), (selection, walk)
            assert np.array_equal(lengths[sample].view(np.uint32), o_len.view(np.uint32))
        if walk is not None:
            # sampled rows' kept prefixes: the first K of (P descending, city ascending)
            K = min(max(64, 1 << (64 * walk - 1).bit_length()), n)
            Ps, Js = col.sorted_rows()
            for c in (0, 8191, n - 1):
                want = np.lexsort((np.arange(n), -P[c].astype(np.float64)))[:K]
                got_j = Js[c, :K].cpu().numpy().view(np.uint16).astype(np.int64)
                assert np.array_equal(got_j, want), (walk, c)
                assert np.array_equal(Ps[c, :K].cpu().numpy(), P[c, want]), (walk, c)
            del Ps, Js
        del P
    # the update at full size, from the last construct
    tau_prev = col.tau().cpu().numpy()
    col.update(1.4)
    col.sync()
    S = col.deposit_scale
    delta = oracle.deposit(tours, lengths, None, 1.0, S)
    tau_ref = oracle.evaporate(tau_prev, delta, 0.1, S)
    del delta, tau_prev
    assert np.array_equal(col.tau().cpu().numpy().view(np.uint32), tau_ref.view(np.uint32))
    rows = np.array([0, 8191, n - 1])
    ref = oracle.transition_rows(tau_ref, D, 1.0, 2.0, 1.4, rows).astype(np.float64)
    got = col.P().cpu().numpy()[rows].astype(np.float64)
    bound = 1e-5 * np.maximum(np.abs(ref), float(FLT_MIN))
    assert not (np.abs(got - ref) > bound).any()
    col.close()
