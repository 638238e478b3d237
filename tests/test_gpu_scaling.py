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


def test_scaling_sweep_on_tsplib_files(tmp_path):
    """The sweep on instances read from TSPLIB files (synthetic ones, written
    here): the city sweep keys by instance name, and the population sweep
    runs on the instance closest to the population size asked for."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import aco_instances as inst
    from aco_instances import tsplib
    from paper_2404_04895_amd import scaling
    for n in (60, 130):
        text = tsplib.format_tsplib("s%d" % n, inst.uniform_cities(n, 70 + n) * 1000.0)
        (tmp_path / ("s%d.tsp" % n)).write_text(text)
    instances = []
    for path in tsplib.instance_files([str(tmp_path)]):
        t = tsplib.read_tsplib(path)
        instances.append((t.name, tsplib.distance_matrix(t)))
    res = scaling.sweep(populations=(1, 20), population_n=120, iters=2, instances=instances)
    assert set(res["cities"]) == {"s60", "s130"} and res["population_n"] == 130
    assert set(res["population"]) == {1, 20}
    for part in ("cities", "population"):
        for row in res[part].values():
            for v in row.values():
                assert v["ms_per_iteration"] > 0 and v["ant_steps_per_s"] > 0
