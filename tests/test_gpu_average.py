"""GPU time-averaged velocity (the period-averaged flow fields of the paper's
results, Sec. 3, Figs. 3, 6 and 9), summed by the stream-collide launches as
they compute u, against the FP64 oracle's mean of the u of the same steps.

Tolerances: each sampled u carries the FP32 error of the velocity field
(rel-L2 <= 1e-5, tests/test_gpu_swimmer.py); the FP64 sums add no error of
their own, so the mean meets the same bar.  FP16 storage: 5e-4 as its
velocity over long runs (tests/test_gpu_fp16.py)."""
import math

import numpy as np
import pytest

import bench
from paper_2202_12147_amd import lbmib, workloads as wl
from tests.helpers import oracle_from, rel_l2

pytestmark = pytest.mark.gpu


def _pair_average(case, t0, steps, every, storage=lbmib.FP32_SHIFTED, fp16_scale=1.0, launch=None,
                  use_graphs=True):
    o = oracle_from(case)
    lat = lbmib.from_workload(case, storage=storage, fp16_scale=fp16_scale, use_graphs=use_graphs)
    if launch is not None:
        lat.set_stream_collide_launch(*launch)
    o.step(t0)
    lat.step(t0)
    lat.average_begin(every)
    mo, no = o.average_velocity(steps, every)
    lat.step(steps)
    mg, ng = lat.average_velocity()
    assert ng == no == math.ceil(steps / every)
    return mo, mg, o, lat


@pytest.mark.parametrize("t0,steps,every", [(0, 200, 1), (40, 150, 7), (5, 70, 32)])
def test_small_case_average_matches_oracle(t0, steps, every):
    # 150..200 steps cross the 32-step graph chunks and the one-step graph
    print("average", t0, steps, every, flush=True)
    mo, mg, o, lat = _pair_average(wl.small_case(), t0, steps, every)
    err = rel_l2(mg, mo)
    print("rel-L2 mean u", err, flush=True)
    assert err < 1e-5
    assert rel_l2(lat.velocity(), o.velocity()) < 1e-5


def test_average_at_full_size_in_the_benchmark_launch():
    # the 128^3 swimmer workload in the benchmark's launch shape: a sampled
    # step every third step over one replayed 32-step graph and eight more
    case = wl.single_128(seed=0)
    mo, mg, _, _ = _pair_average(case, 0, 40, 3, launch=bench.MAIN_LAUNCH)
    err = rel_l2(mg, mo)
    print("rel-L2 mean u", err, flush=True)
    assert err < 1e-5


def test_batch_average_per_box():
    # ragged boxes at 128-node blocks (every box ends in a part block)
    shapes = [(39, 34, 39), (33, 37, 39), (34, 33, 34)]
    boxes = [dict(shape=s, tau=t, forcing=wl.GUO, width=3,
                  swimmers=[wl.swimmer(tuple(v // 2 for v in s), 9.0, A=1e-3, T=500.0)])
             for s, t in zip(shapes, [0.8, 1.0, 0.7])]
    b = lbmib.batch_from_ensemble(dict(boxes=boxes))
    b.set_stream_collide_launch(128, 0, 2)
    b.step(10)
    b.average_begin(2)
    b.step(51)
    for i, bx in enumerate(boxes):
        o = oracle_from(dict(bx))
        o.step(10)
        mo, no = o.average_velocity(51, 2)
        mg, ng = b.average_velocity(i)
        print("box", i, "rel-L2 mean u", rel_l2(mg, mo), flush=True)
        assert ng == no == 26
        assert rel_l2(mg, mo) < 1e-5
        # device output of one box of a batch (staged, then copied)
        t, nt = b.average_velocity(i, device="cuda:0")
        assert nt == ng and np.array_equal(t.cpu().numpy(), mg)


def test_launch_shape_change_keeps_the_average():
    # a new launch shape mid-average drops and recaptures the step graphs;
    # the sums, the schedule and every bit of the mean carry on
    case = wl.small_case()
    a = lbmib.from_workload(case)
    b = lbmib.from_workload(case)
    for x in (a, b):
        x.step(5)
        x.average_begin(3)
        x.step(40)
    b.set_stream_collide_launch(256, 1, 2)
    for x in (a, b):
        x.step(37)
    ma, na = a.average_velocity()
    mb, nb = b.average_velocity()
    assert na == nb == 26
    assert np.array_equal(ma, mb)


def test_fp16_storage_average():
    mo, mg, _, _ = _pair_average(wl.small_case(), 0, 200, 1, storage=lbmib.FP16_SHIFTED, fp16_scale=2.0 ** 27)
    err = rel_l2(mg, mo)
    print("rel-L2 mean u (fp16)", err, flush=True)
    assert err < 5e-4


@pytest.mark.parametrize("forcing", [wl.GUO, wl.SHAN_CHEN])
def test_uniform_acceleration_closed_form(forcing):
    # the velocity of step n is (n + 1/2) g under a uniform body force g
    g = np.array([2e-6, -1e-6, 5e-7])
    lat = lbmib.Lattice((24, 20, 18), 0.8, forcing)
    lat.set_body_force(g)
    lat.step(3)
    lat.average_begin(4)
    lat.step(21)
    mean, count = lat.average_velocity()
    K = 6
    assert count == K
    want = (3 + 4 * (K - 1) / 2 + 0.5) * g
    for a in range(3):
        np.testing.assert_allclose(mean[a], want[a], rtol=2e-6, atol=0)


def test_averaging_leaves_the_state_unchanged():
    case = wl.small_case()
    a = lbmib.from_workload(case)
    b = lbmib.from_workload(case)
    a.average_begin(1)
    for x in (a, b):
        x.step(77)
    assert np.array_equal(a.markers(), b.markers())
    assert np.array_equal(a.populations(), b.populations())


def test_graphs_direct_launches_and_device_output_agree():
    case = wl.small_case()
    _, ga, _, la = _pair_average(case, 3, 70, 5)
    _, gb, _, lb = _pair_average(case, 3, 70, 5, use_graphs=False)
    assert np.array_equal(ga, gb)
    import torch
    t, n = la.average_velocity(device="cuda:0")
    assert n == 14
    assert np.array_equal(t.cpu().numpy(), ga)


def test_restart_stop_checkpoint_and_adjoint(tmp_path):
    case = wl.small_case()
    lat = lbmib.from_workload(case)
    with pytest.raises(lbmib.LbmError) as e:
        lat.average_velocity()
    assert e.value.code == -4
    lat.average_begin(1)
    m0, n0 = lat.average_velocity()
    assert n0 == 0 and not m0.any()
    lat.step(10)
    lat.save(tmp_path / "c.bin")
    # restarting clears the sums and counts from the next step
    lat.average_begin(3)
    lat.step(7)
    ref = lbmib.from_workload(case)
    ref.step(10)
    ref.average_begin(3)
    ref.step(7)
    m1, n1 = lat.average_velocity()
    m2, n2 = ref.average_velocity()
    assert n1 == n2 == 3
    assert np.array_equal(m1, m2)
    # the adjoint refuses to run inside an average
    with pytest.raises(lbmib.LbmError) as e:
        lat.adjoint(5, checkpoint=5)
    assert e.value.code == -4
    # loading a checkpoint stops the average; so does every = 0
    lat.load(tmp_path / "c.bin")
    with pytest.raises(lbmib.LbmError):
        lat.average_velocity()
    lat.average_begin(1)
    lat.average_begin(0)
    with pytest.raises(lbmib.LbmError):
        lat.average_velocity()
    with pytest.raises(lbmib.LbmError):
        lat.average_begin(-1)
