"""GPU parity of FP16-shifted population storage (values g*S rounded to
nearest-even half precision, FP32 arithmetic) against the FP64 oracle.

Tolerances: each stored value carries a relative rounding error of at most
2^-11 (4.9e-4) once it is a normal half number.  With the scale chosen so
that the largest |g|*S sits ~16-32x below the half maximum (65504), the
O(1e-7..1e-5) deviations of these flows are all normal numbers.  One step
mixes ~19 rounded values per node: populations within 4e-3 of max |g|,
velocity rel-L2 within 2e-3.  Over the 1000-step small case the rounding
errors average out: velocity rel-L2 measured 1.1e-4 (bar 5e-4), swimmer
displacement within 1.4e-3 relative (bar 3e-3).  Unscaled storage (S = 1)
leaves every deviation subnormal (step 6e-8) and is shown to fail."""
import math
import os

import numpy as np
import pytest

import bench
from oracle import orc
from paper_2202_12147_amd import lbmib, workloads as wl
from tests.helpers import max_rel, oracle_from, rel_l2

pytestmark = pytest.mark.gpu

S27 = 2.0 ** 27
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_scale_rule():
    assert lbmib.fp16_scale_for(2e-5) == 2.0 ** 27
    assert lbmib.fp16_scale_for(1.0) == 2.0 ** 11


def test_fp16_rest_state_exact():
    lat = lbmib.Lattice((16, 16, 16), 0.8, storage=lbmib.FP16_SHIFTED, fp16_scale=S27)
    lat.step(5)
    assert np.array_equal(lat.populations(), np.zeros((19, 16, 16, 16)))


@pytest.mark.parametrize("forcing", [wl.GUO, wl.SHAN_CHEN])
def test_fp16_one_step(forcing):
    shape = (24, 20, 18)
    dev = wl.random_deviation(shape, 3, 1e-5)
    S = lbmib.fp16_scale_for(np.abs(dev).max())
    o = orc.Oracle(shape, 0.9, forcing, 3)
    o.set_deviation(dev)
    o.set_body_force((1e-7, 0, 0))
    lat = lbmib.Lattice(shape, 0.9, forcing, storage=lbmib.FP16_SHIFTED, fp16_scale=S)
    lat.set_populations(dev)
    lat.set_body_force((1e-7, 0, 0))
    o.step(1)
    lat.step(1)
    gref = o.pops() - orc.lattice()[1][:, None, None, None]
    assert np.abs(lat.populations() - gref).max() <= 4e-3 * np.abs(gref).max()
    assert rel_l2(lat.velocity(), o.velocity()) < 2e-3


def test_fp16_small_case_accuracy():
    case = wl.small_case()
    o = oracle_from(case)
    good = lbmib.from_workload(case, storage=lbmib.FP16_SHIFTED, fp16_scale=S27)
    bad = lbmib.from_workload(case, storage=lbmib.FP16_SHIFTED, fp16_scale=1.0)
    X0 = o.swimmer_centres().copy()
    o.step(1000)
    good.step(1000)
    bad.step(1000)
    eu = rel_l2(good.velocity(), o.velocity())
    d_o = (o.swimmer_centres() - X0)[0, 0]
    d_g = (good.swimmer_centres() - X0)[0, 0]
    print("fp16 S=2^27: u rel-L2", eu, "displacement", d_g, "oracle", d_o, flush=True)
    assert eu < 5e-4
    assert abs(d_g - d_o) <= 3e-3 * abs(d_o)
    assert rel_l2(bad.velocity(), o.velocity()) > 1e-2


@pytest.mark.parametrize("arrangement", ["collinear", "side"])
def test_pair_storage_forms_vs_oracle(arrangement):
    """Two swimmers in 256x128x128 (collinear gap 40 or side by side gap 20,
    random phase lag), FP32-shifted and FP16-shifted storage against the FP64
    oracle after 200 steps: velocity-field rel-L2 and the error of each
    swimmer's centre displacement.  FP32 bars as for one swimmer; FP16 as the
    small case's (rel-L2 5e-4, its per-value rounding 2^-11 averaging over
    nodes) with the centre displacement within 2e-3 of its size."""
    case = wl.pair_256(seed=0, arrangement=arrangement)
    steps = 200
    o = oracle_from(case)
    X0 = o.swimmer_centres().copy()
    o.step(steps)
    d_o = o.swimmer_centres() - X0
    res = {}
    for name, st, S, launch in (("fp32", lbmib.FP32_SHIFTED, 1.0, bench.MAIN_LAUNCH),
                                ("fp16", lbmib.FP16_SHIFTED, S27, bench.FP16_LAUNCH)):
        lat = lbmib.from_workload(case, storage=st, fp16_scale=S)
        lat.set_stream_collide_launch(*launch)
        lat.step(steps)
        d = lat.swimmer_centres() - X0
        res[name] = (rel_l2(lat.velocity(), o.velocity()), np.abs(d - d_o).max() / np.abs(d_o).max())
    print(arrangement, "u rel-L2 / centre displacement rel error:", res, flush=True)
    assert res["fp32"][0] < 1e-5 and res["fp32"][1] < 1e-4
    assert res["fp16"][0] < 5e-4 and res["fp16"][1] < 2e-3


@pytest.mark.parametrize("block,remap,resident", [(256, 0, 2), (256, 1, 2), (512, 0, 1), (128, 0, 0)])
def test_fp16_launch_shapes_bitwise_equal_with_swimmer(block, remap, resident):
    # FP16 storage walks the persistent bulk launch statically (in block
    # order or per XCD range); every launch shape gives the same bits as the
    # serial order
    case = wl.single_128(seed=1)
    case["shape"] = (48, 40, 40)
    case["swimmers"][0]["centres"] = case["swimmers"][0]["centres"] - (40, 24, 24)
    a = lbmib.from_workload(case, storage=lbmib.FP16_SHIFTED, fp16_scale=S27, use_graphs=False)
    a.set_stream_collide_launch(256, 0, -1)
    b = lbmib.from_workload(case, storage=lbmib.FP16_SHIFTED, fp16_scale=S27)
    b.set_stream_collide_launch(block, remap, resident)
    for x in (a, b):
        x.step(45)
        x.sync()
    assert np.array_equal(a.markers(), b.markers())
    assert np.array_equal(a.populations(), b.populations())


def test_fp16_above_the_write_through_size():
    # 256^3 with FP16 storage holds 1.27 GB of populations, above the 1 GiB
    # up to which stores are written through: the large-set store path of
    # FP16 against the oracle over ten steps (measured: velocity rel-L2
    # 1.0e-4, element-wise 1.3e-4 of max |u|; bars three times that; markers
    # move ~2.5e-5 per step with a 5e-4 relative FP16 error)
    case = wl.small_case()
    case["shape"] = (256, 256, 256)
    case["swimmers"] = [wl.swimmer((128, 128, 128), 10.0, A=1e-3, T=500.0, phi0=1.0)]
    o = oracle_from(case)
    lat = lbmib.from_workload(case, storage=lbmib.FP16_SHIFTED, fp16_scale=S27)
    o.step(10)
    lat.step(10)
    du = rel_l2(lat.velocity(), o.velocity())
    dmax = max_rel(lat.velocity(), o.velocity())
    dr = np.abs(lat.markers() - o.markers()).max()
    print("fp16 256^3: u rel-L2", du, "max-rel", dmax, "max |dr|", dr, flush=True)
    assert du < 3e-4 and dmax < 4e-4 and dr < 1e-6


@pytest.mark.parametrize("arrangement", ["collinear", "side"])
def test_pair_full_length_vs_stored_oracle(arrangement):
    """The two-swimmer 256x128x128 workload over its full 10000 steps in the
    benchmark's launch shapes, FP32- and FP16-shifted storage, against the
    FP64 oracle's run stored by tests/golden/make_trajectory_golden.py: both
    swimmer centres every 10 steps, every marker and the final velocity field
    on every fourth node per axis.  Reported: the largest centre error
    relative to the largest centre displacement, the final field's rel-L2 and
    element-wise error on the sampled nodes, the largest marker error."""
    ref = np.load(os.path.join(GOLDEN, f"pair256_{arrangement}_10000.npz"))
    Xr, every = ref["X"], int(ref["every"])
    case = wl.pair_256(seed=0, arrangement=arrangement)
    disp = np.abs(Xr - Xr[0]).max()
    res = {}
    for name, st, S, launch in (("fp32", lbmib.FP32_SHIFTED, 1.0, bench.MAIN_LAUNCH),
                                ("fp16", lbmib.FP16_SHIFTED, S27, bench.FP16_LAUNCH)):
        lat = lbmib.from_workload(case, storage=st, fp16_scale=S)
        lat.set_stream_collide_launch(*launch)
        np.testing.assert_allclose(lat.swimmer_centres(), Xr[0], rtol=0, atol=1e-12)
        worst = 0.0
        for k in range(1, len(Xr)):
            lat.step(every)
            worst = max(worst, float(np.abs(lat.swimmer_centres() - Xr[k]).max()))
        u = lat.velocity()[:, ::4, ::4, ::4]
        res[name] = dict(centre=worst / disp, u_l2=rel_l2(u, ref["u_sub"]), u_max=max_rel(u, ref["u_sub"]),
                         markers=float(np.abs(lat.markers() - ref["markers"]).max()))
        lat.close()
    print(arrangement, f"largest displacement {disp:.4e}:", res, flush=True)
    # measured (collinear / side by side): FP32 centre 1.4e-4 / 1.4e-4, field
    # rel-L2 3.2e-6 / 3.2e-6 and element-wise 8.5e-7 / 8.7e-7, markers
    # 9.5e-8 / 1.0e-7; FP16 centre 0.86e-3 / 0.77e-3 (1.1e-3 before the
    # force-free collision), field 2.4e-4 / 2.4e-4 and 1.3e-4 / 1.4e-4,
    # markers 6.0e-7 / 4.7e-7.  Bars about three times the largest.
    assert res["fp32"]["centre"] < 5e-4 and res["fp32"]["u_l2"] < 1e-5 and res["fp32"]["u_max"] < 5e-6
    assert res["fp32"]["markers"] < 5e-7
    assert res["fp16"]["centre"] < 4e-3 and res["fp16"]["u_l2"] < 1e-3 and res["fp16"]["u_max"] < 1e-3
    assert res["fp16"]["markers"] < 5e-6
