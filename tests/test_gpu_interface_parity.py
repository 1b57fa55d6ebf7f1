"""One call sequence, two backends: the binding's Lattice and Batch over the
HIP library and over the oracle's implementation of the same interface
(oracle/orc_abi.c), compared at the coupled step's bars (velocity rel-L2 and
element-wise max error 1e-5 of the largest |u|; marker positions 1e-10 l.u.
per step; conserved sums to FP32 rounding of the populations, 1e-6 of the
mass)."""
import numpy as np
import pytest

from paper_2202_12147_amd import lbmib, workloads as wl
from tests.helpers import interface_batch, interface_lattice, max_rel, oracle_interface, rel_l2

pytestmark = pytest.mark.gpu

POS_PER_STEP = 1e-10


def _drive(lat, chunks):
    for n in chunks:
        lat.step(n)
    lat.sync()


@pytest.mark.parametrize("forcing", [wl.GUO, wl.SHAN_CHEN])
def test_lattice_through_both_backends(forcing):
    case = dict(wl.small_case(), forcing=forcing)
    print("small case, forcing", forcing, flush=True)
    hip = interface_lattice(lbmib.load_library(), case)
    ref = interface_lattice(oracle_interface(), case)
    chunks = (1, 6, 33, 60)
    for lat in (hip, ref):
        _drive(lat, chunks)
    steps = sum(chunks)
    assert hip.time == ref.time == steps
    u, uo = hip.velocity(), ref.velocity()
    print("rel-L2 u", rel_l2(u, uo), "max-rel u", max_rel(u, uo), flush=True)
    assert rel_l2(u, uo) < 1e-5 and max_rel(u, uo) < 1e-5
    assert np.abs(hip.markers() - ref.markers()).max() < POS_PER_STEP * steps
    assert np.abs(hip.swimmer_centres() - ref.swimmer_centres()).max() < POS_PER_STEP * steps
    c, co = hip.conserved(), ref.conserved()
    assert abs(c[0] - co[0]) < 1e-6 * co[0]
    assert np.abs(c[1:] - co[1:]).max() < 1e-6 * co[0]


def test_batch_through_both_backends():
    ens = wl.ensemble(seed=4, nboxes=2)
    boxes = [dict(bx, shape=tuple(bx["shape"])) for bx in ens["boxes"]]
    print("ensemble seed 4, 2 boxes", [bx["shape"] for bx in boxes], flush=True)
    hip = interface_batch(lbmib.load_library(), boxes, boxes[0]["width"])
    ref = interface_batch(oracle_interface(), boxes, boxes[0]["width"])
    for b in (hip, ref):
        _drive(b, (40,))
    for k in range(2):
        u, uo = hip.velocity(k), ref.velocity(k)
        assert rel_l2(u, uo) < 1e-5 and max_rel(u, uo) < 1e-5
    assert np.abs(hip.markers() - ref.markers()).max() < POS_PER_STEP * 40
