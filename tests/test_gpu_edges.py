"""Edge inputs on the GPU, through the C ABI: no ants, no iterations, the
smallest instance under every selection rule."""
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
