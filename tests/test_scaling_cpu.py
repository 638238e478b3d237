"""Host logic of the runtime sweep: the paper's elitist k = n/10, or every ant
when the colony is not larger than k."""
from paper_2404_04895_amd.scaling import elite_for


def test_elite_for():
    assert elite_for(1173, 10000) == 117
    assert elite_for(1173, 1173) == 117
    assert elite_for(1173, 117) == 0    # k >= m: every ant deposits
    assert elite_for(1173, 1) == 0
    assert elite_for(5, 100) == 0       # n/10 rounds to 0: every ant
