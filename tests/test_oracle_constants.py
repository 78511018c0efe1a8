"""The synthetic workloads use the paper's Earth parameters (Section 6)."""
import synth
from tests.golden.read import load

PAPER = load("paper_section6.txt")


def test_constants_match_paper():
    assert synth.EARTH_RADIUS == PAPER["radius"]
    assert synth.EARTH_OMEGA == PAPER["omega"]
    assert synth.GRAVITY == PAPER["gravity"]
    assert synth.MEAN_DEPTH == PAPER["mean_depth"]


def test_workload_sizes():
    w = synth.WORKLOADS
    assert [w[k].T for k in w] == [63, 63, 128, 128, 256]
    assert [2 * (w[k].M + w[k].L) + 1 for k in w] == [151, 279, 535, 407, 2071]
    for k in w:
        assert w[k].nlat * 2 == w[k].nlon
