"""The runtime sweep over colony size and city count (the stand-in for the
paper's runtime experiment) runs on the GPU and reports every point."""
import pytest

pytestmark = pytest.mark.gpu


def test_scaling_sweep_small():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_04895_amd import scaling
    res = scaling.sweep(sizes=(159,), populations=(1, 20), population_n=159, iters=2)
    assert set(res["cities"]) == {159} and set(res["population"]) == {1, 20}
    for part in ("cities", "population"):
        for row in res[part].values():
            assert set(row) == set(scaling.SELECTIONS)
            for v in row.values():
                assert v["ms_per_iteration"] > 0 and v["ant_steps_per_s"] > 0
