"""The library's calling interface served by the FP64 oracle (oracle/orc_abi.c,
built into liborc.so): the binding's Lattice and Batch drive it with the same
calls as the HIP library.  Pinned here against the oracle's own functions
(orc.Oracle) on the same workloads: FP64 observables bit for bit, float32
fields as the float32 rounding of the oracle's, deviations as f - w; and the
invalid calls of the interface fail with the same codes in both libraries
(the HIP library's checks run before any device call, so this runs on the
CPU)."""
import ctypes as C

import numpy as np
import pytest

from oracle import orc
from paper_2202_12147_amd import lbmib, workloads as wl
from tests.helpers import interface_batch, interface_lattice, oracle_from, oracle_interface


@pytest.fixture(scope="module")
def olib():
    return oracle_interface()


def test_every_symbol_is_served(olib):
    for name in lbmib.SYMBOLS:
        assert hasattr(olib, name), name


@pytest.mark.parametrize("forcing", [wl.GUO, wl.SHAN_CHEN])
def test_same_calls_same_results_as_the_oracle(olib, forcing):
    case = dict(wl.small_case(), forcing=forcing)
    lat = interface_lattice(olib, case)
    o = oracle_from(case)
    assert lat.n_markers == o.n_markers
    lat.step(12)
    lat.step(18)
    lat.sync()
    o.step(30)
    assert lat.time == 30
    assert np.array_equal(lat.markers(), o.markers())
    assert np.array_equal(lat.swimmer_centres(), o.swimmer_centres())
    assert np.array_equal(lat.bead_centres(), o.bead_centres())
    assert np.array_equal(lat.marker_velocities(), o.marker_velocities())
    assert np.array_equal(lat.marker_forces(), o.marker_forces())
    assert np.array_equal(lat.velocity(), o.velocity().astype(np.float32))
    assert np.array_equal(lat.density(), o.density().astype(np.float32))
    _, w = orc.lattice()
    assert np.array_equal(lat.populations().reshape(19, -1), o.pops().reshape(19, -1) - w[:, None])
    np.testing.assert_array_equal(lat.conserved(), o.conserved())
    lat.close()


def test_batch_matches_separate_oracles(olib):
    ens = wl.ensemble(seed=4, nboxes=2)
    boxes = [dict(bx, shape=tuple(bx["shape"])) for bx in ens["boxes"]]
    b = interface_batch(olib, boxes, boxes[0]["width"])
    ors = [oracle_from(dict(bx, width=boxes[0]["width"])) for bx in boxes]
    b.step(9)
    for o in ors:
        o.step(9)
    assert b.n_boxes == 2
    assert np.array_equal(b.markers(), np.concatenate([o.markers() for o in ors]))
    for k, o in enumerate(ors):
        assert np.array_equal(b.velocity(k), o.velocity().astype(np.float32))
        np.testing.assert_array_equal(b.conserved(k), o.conserved())
    np.testing.assert_allclose(b.conserved(-1), ors[0].conserved() + ors[1].conserved(), rtol=1e-15)


def test_calls_the_oracle_does_not_serve(olib):
    lat = interface_lattice(olib, wl.small_case())
    for call in (lambda: olib.lbm_average_begin(lat.h, 1), lambda: olib.lbm_save(lat.h, b"/nonexistent"),
                 lambda: olib.lbm_set_kernel_timing(lat.h, 1),
                 lambda: olib.lbm_swimmer_set_params(lat.h, 0, 1e-3, 1e-3, 1.0, 0.01)):
        assert call() == -4
        assert olib.lbm_last_error(lat.h) == b"not provided by the oracle"
    assert olib.lbm_set_stream_collide_launch(lat.h, 512, 0, 1) == 0
    assert olib.lbm_set_stream_collide_launch(lat.h, 300, 0, 1) == -1
    f = np.zeros(3 * lat.N, np.float32)
    assert olib.lbm_get_velocity(lat.h, f.ctypes.data_as(C.c_void_p), 1) == -1  # no device memory
    lat.step(1)
    assert lat.lib.lbm_set_populations(lat.h, np.zeros(19 * lat.N).ctypes.data_as(C.c_void_p)) == -4
    lat.close()


def _invalid_calls(lib):
    """Return codes of invalid calls, in a fixed order."""
    h = C.c_void_p()
    ok = lbmib.Grid(32, 32, 32)
    rc = [lib.lbm_create(C.byref(ok), 0.5, 0, None, C.byref(h)),
          lib.lbm_create(C.byref(ok), float("nan"), 0, None, C.byref(h)),
          lib.lbm_create(C.byref(lbmib.Grid(8, 32, 32)), 1.0, 0, None, C.byref(h)),
          lib.lbm_create(C.byref(ok), 1.0, 7, None, C.byref(h)),
          lib.lbm_create(None, 1.0, 0, None, C.byref(h))]
    for opts in ((0, 5, 1.0, 1, None, None, 0), (1, 3, 3.0, 1, None, None, 0), (9, 3, 1.0, 1, None, None, 0),
                 (0, 3, 1.0, 1, None, 0x10000 + 8, 1 << 30)):
        o = lbmib.Opts(*opts)
        rc.append(lib.lbm_create(C.byref(ok), 1.0, 0, C.byref(o), C.byref(h)))
    rc.append(lib.lbm_create(C.byref(lbmib.Grid(2048, 1024, 1024)), 1.0, 0, None, C.byref(h)))
    boxes = (lbmib.BoxDesc * 2)(lbmib.BoxDesc(lbmib.Grid(1024, 1024, 1024), 1.0, 0),
                                lbmib.BoxDesc(lbmib.Grid(1024, 1024, 1024), 1.0, 0))
    rc += [lib.lbm_batch_create(boxes, 2, None, C.byref(h)), lib.lbm_batch_create(boxes, 0, None, C.byref(h))]
    count = C.c_int64()
    desc = lbmib.AdjointDesc(10, 5, 0, 0)
    J, g = C.c_double(), (C.c_double * 4)()
    rc += [lib.lbm_step(None, 1), lib.lbm_average_begin(None, 1),
           lib.lbm_get_average_velocity(None, 0, None, 0, C.byref(count)),
           lib.lbm_adjoint(None, C.byref(desc), C.byref(J), g),
           lib.lbm_swimmer_set_params(None, 0, 1e-3, 1e-3, 1.0, 0.01), lib.lbm_autotune(None, 4, None, None, 0),
           lib.lbm_set_stream_collide_launch(None, 256, 0, 0), lib.lbm_destroy(None)]
    assert h.value is None
    return rc, [lib.lbm_strerror(c) for c in (0, -1, -2, -3, -4, -5, -6, -7, -8)]


def test_invalid_calls_fail_alike(olib):
    hip = lbmib.load_library()
    assert _invalid_calls(olib) == _invalid_calls(hip)


def test_launch_tuner_logic_on_the_oracle_interface(olib):
    """lbmib.tune_launch over the oracle's interface (which accepts launch
    shapes and ignores them): every candidate is timed in both passes, the
    best is the fastest of the table, and the scratch handle is destroyed;
    the caller's handle is never built or stepped by the tuner."""
    made = []

    def make():
        made.append(interface_lattice(olib, wl.small_case()))
        return made[-1]

    cands = ((512, True, 0), (256, False, 2), (128, True, 0))
    best, table = lbmib.tune_launch(make, cands, steps=2, warmup=1)
    assert len(made) == 1 and made[0].h is None  # closed
    assert set(table) == set(cands) and all(v > 0 for v in table.values())
    assert best == min(table, key=table.get)
