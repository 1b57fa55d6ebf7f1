"""GPU parity of the fused stream-collide against the FP64 oracle (paper Sec.
2.1): rest state, random smooth states under Guo and Shan-Chen forcing,
ragged grids, conservation, determinism, graphs and checkpoints.

Tolerances (FP32 storage of g = f - w, FP32 arithmetic): one step rounds each
g once (relative 6e-8) plus the collision's FP32 arithmetic on O(1e-4)
deviations, so per-step velocity errors are ~1e-7 relative; they grow at most
linearly with steps.  The bars are 1e-6 relative (one step) and 1e-5 (100
steps) on velocity, 1e-6 of max |g| on populations after one step."""
import numpy as np
import pytest

from oracle import orc
from paper_2202_12147_amd import lbmib, workloads as wl
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu

SHAPES = [(16, 16, 16), (20, 17, 19), (40, 24, 33)]


def _pair(shape, tau, forcing, seed=0, g=(0, 0, 0), eps=1e-4):
    dev = wl.random_deviation(shape, seed, eps)
    o = orc.Oracle(shape, tau, forcing, 3)
    o.set_deviation(dev)
    o.set_body_force(g)
    lat = lbmib.Lattice(shape, tau, forcing)
    lat.set_populations(dev)
    lat.set_body_force(g)
    return o, lat, dev


def test_rest_state_exact():
    lat = lbmib.Lattice((16, 16, 16), 0.8)
    lat.step(7)
    assert np.array_equal(lat.populations(), np.zeros((19, 16, 16, 16)))
    assert np.array_equal(lat.velocity(), np.zeros((3, 16, 16, 16), np.float32))
    c = lat.conserved()
    assert c[0] == 16 ** 3 and np.all(c[1:] == 0)


@pytest.mark.parametrize("forcing", [wl.GUO, wl.SHAN_CHEN])
@pytest.mark.parametrize("shape", SHAPES)
def test_one_step_parity(shape, forcing):
    print("case", shape, forcing, flush=True)
    o, lat, dev = _pair(shape, 0.8, forcing, seed=1, g=(2e-6, -1e-6, 5e-7))
    o.step(1)
    lat.step(1)
    gref = o.pops() - orc.lattice()[1][:, None, None, None]
    gg = lat.populations()
    assert np.abs(gg - gref).max() <= 1e-6 * np.abs(gref).max()
    assert rel_l2(lat.velocity(), o.velocity()) < 1e-6
    assert np.abs(lat.density() - o.density()).max() < 1e-6


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_hundred_steps_parity(tau):
    shape = (24, 20, 18)
    o, lat, _ = _pair(shape, tau, wl.GUO, seed=2, g=(1e-6, 0, 0))
    o.step(100)
    lat.step(100)
    assert rel_l2(lat.velocity(), o.velocity()) < 1e-5
    co, cg = o.conserved(), lat.conserved()
    assert abs(cg[0] - co[0]) < 1e-6
    np.testing.assert_allclose(cg[1:], co[1:], rtol=1e-5, atol=1e-9)


def test_graphs_and_direct_launches_bitwise_equal():
    shape = (32, 16, 24)
    dev = wl.random_deviation(shape, 3, 1e-4)
    a = lbmib.Lattice(shape, 0.9, use_graphs=True)
    b = lbmib.Lattice(shape, 0.9, use_graphs=False)
    for x in (a, b):
        x.set_populations(dev)
        x.step(37)
    assert np.array_equal(a.populations(), b.populations())
    assert a.time == b.time == 37


def test_checkpoint_restart_bitwise(tmp_path):
    shape = (16, 24, 16)
    dev = wl.random_deviation(shape, 4, 1e-4)
    a = lbmib.Lattice(shape, 0.9)
    a.set_populations(dev)
    a.step(10)
    a.save(tmp_path / "ck.bin")
    a.step(15)
    b = lbmib.Lattice(shape, 0.9)
    b.load(tmp_path / "ck.bin")
    assert b.time == 10
    b.step(15)
    assert np.array_equal(a.populations(), b.populations())
    assert np.array_equal(a.velocity(), b.velocity())


def test_velocity_on_device_matches_host():
    import torch
    shape = (16, 16, 32)
    dev = wl.random_deviation(shape, 5, 1e-4)
    a = lbmib.Lattice(shape, 0.9)
    a.set_populations(dev)
    a.step(3)
    t = a.velocity(device="cuda:0")
    assert np.array_equal(t.cpu().numpy(), a.velocity())


def test_shear_wave_viscosity_on_gpu():
    # nu = (tau - 1/2)/3 (Sec. 2.1) measured from the decay of a shear wave
    N, tau = 32, 0.8
    c, w = orc.lattice()
    y = np.arange(N)
    ux = 1e-5 * np.sin(2 * np.pi * y / N)
    dev = np.zeros((19, 16, N, 16))
    for i in range(19):
        cu = c[i, 0] * ux
        dev[i] = (w[i] * (3 * cu + 4.5 * cu * cu - 1.5 * ux * ux))[None, :, None]
    lat = lbmib.Lattice((16, N, 16), tau)
    lat.set_populations(dev)
    s = np.sin(2 * np.pi * y / N)
    lat.step(10)
    a0 = (lat.velocity()[0][0, :, 0].astype(np.float64) * s).sum()
    lat.step(256)
    a1 = (lat.velocity()[0][0, :, 0].astype(np.float64) * s).sum()
    nu = -np.log(a1 / a0) / ((2 * np.pi / N) ** 2 * 256)
    assert abs(nu / ((tau - 0.5) / 3) - 1) < 3e-3


@pytest.mark.parametrize("block,remap", [(128, 0), (512, 1), (256, 1)])
def test_launch_shapes_bitwise_equal(block, remap):
    shape = (40, 24, 33)
    dev = wl.random_deviation(shape, 6, 1e-4)
    a = lbmib.Lattice(shape, 0.9, use_graphs=False)
    b = lbmib.Lattice(shape, 0.9)
    b.set_stream_collide_launch(block, remap, 0)
    for x in (a, b):
        x.set_populations(dev)
        x.set_body_force((1e-6, 2e-6, 0))
        x.step(9)
    assert np.array_equal(a.populations(), b.populations())


def test_copy_probe_reports_bandwidth():
    gbs = lbmib.copy_bandwidth(1 << 28, 10)
    assert 500 < gbs < 20000
