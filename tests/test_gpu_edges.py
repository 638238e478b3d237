"""Edge inputs on the GPU, through the C ABI: no ants, no iterations, the
smallest instance under every selection rule, and distances far from the
unit square's scale (TSPLIB-sized integer distances, and tiny ones)."""
import math

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


def test_no_ants_and_no_iterations():
    torch = _torch()
    from paper_2404_04895_amd import AcoError, Colony
    D = inst.distance_matrix(inst.uniform_cities(8, 1))
    col = Colony(torch.from_numpy(D).cuda(), 1.0, 2.0, 0.5, 1.0, 4)
    col.transition(1.0)
    for m in (0, -1):
        with pytest.raises(AcoError) as e:
            col.construct(m, 0, 0)
        assert e.value.status == -1
    tour, L = col.run(4, 0, 0)          # zero iterations: nothing recorded
    assert math.isinf(L) and L > 0
    _, L2, it = col.best()
    assert math.isinf(L2) and it == -1
    with pytest.raises(AcoError):
        col.run(4, 0, -1)
    col.close()


@pytest.mark.parametrize("selection", ["adair", "adair-sorted", "roulette"])
def test_smallest_instance_every_rule(selection):
    """n = 3: one tour up to direction and start; every rule runs, and each
    construct matches the oracle's on the same P."""
    torch = _torch()
    from paper_2404_04895_amd import Colony
    D = inst.distance_matrix(np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]], np.float32))
    m = 7
    col = Colony(torch.from_numpy(D).cuda(), 1.0, 2.0, 0.5, 1.0, m)
    col.set_selection(selection)
    for it in range(5):
        col.transition(1.0 if selection == "roulette" else 1.3)
        col.construct(m, 11, it)
        col.sync()
        P = col.P().cpu().numpy()
        want, wlen = oracle.construct(P, D, 11, it, np.arange(m),
                                      selection="roulette" if selection == "roulette" else "adair")
        assert np.array_equal(col.tours(m).cpu().numpy(), want)
        assert np.array_equal(col.lengths(m).cpu().numpy(), wlen)
        assert np.allclose(wlen, 2.0 + math.sqrt(2.0))
    col.close()


@pytest.mark.parametrize("scale,metric", [(1e4, "tsplib"), (1e-4, "euclidean")])
def test_distance_scales_match_oracle(scale, metric):
    """Tour lengths from about 1e-3 to 1e6: the deposit's fixed-point exponent
    follows the lower bound on a tour, so the run still equals the oracle's
    bit for bit.  The large case uses TSPLIB's integer metric, where equal
    tour lengths (ties broken by ant index) are common."""
    torch = _torch()
    from aco_instances import tsplib
    from paper_2404_04895_amd import Colony
    xy = inst.uniform_cities(40, 404).astype(np.float64) * scale
    D = tsplib.distance_matrix(tsplib.parse_tsplib(tsplib.format_tsplib("scaled", xy)), metric)
    n = m = D.shape[0]
    T = 15
    col = Colony(torch.from_numpy(D).cuda(), 1.0, 2.0, 0.3, 1.0, m)
    tour, L = col.run(m, 5, T)
    ref = oracle.run(D, m, 1.0, 2.0, 0.3, 1.0, 5, T)
    assert L == np.float32(ref["best_len"])
    assert np.array_equal(tour, ref["best_tour"])
    assert np.array_equal(col.tau().cpu().numpy(), ref["tau"])
    col.close()
