"""Host checks of the seeded workload builders that have no oracle run of
their own: the paper-box pair arrangements (Secs. 3.2, 3.3)."""
import numpy as np
import pytest

from paper_2202_12147_amd import workloads as wl


@pytest.mark.parametrize("arrangement,axis", [("collinear", 0), ("side", 1)])
def test_paper_pair_geometry(arrangement, axis):
    single = wl.paper_run()["swimmers"][0]
    case = wl.paper_run(arrangement, 100.0)
    a, b = case["swimmers"]
    # middle beads the given distance apart along the arrangement's axis,
    # symmetric about the single swimmer's middle bead
    d = b["centres"][1] - a["centres"][1]
    expect = np.zeros(3)
    expect[axis] = 100.0
    np.testing.assert_array_equal(d, expect)
    np.testing.assert_array_equal(0.5 * (a["centres"][1] + b["centres"][1]), single["centres"][1])
    # otherwise identical, in-phase swimmers along x
    for sw in (a, b):
        np.testing.assert_array_equal(sw["centres"] - sw["centres"][1], single["centres"] - single["centres"][1])
        for key in ("radius", "k", "L0"):
            np.testing.assert_array_equal(sw[key], single[key])
        for key in ("A", "B", "T", "alpha", "phi0", "level"):
            assert sw[key] == single[key]
    assert case["shape"] == (1024, 256, 256) and case["forcing"] == wl.SHAN_CHEN


def test_paper_pair_rejects_unknown_arrangement():
    with pytest.raises(ValueError):
        wl.paper_run("diagonal", 50.0)
