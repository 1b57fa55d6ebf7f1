"""Pins of the oracle's lattice Boltzmann step and its coupling (paper Sec. 2.1
Eqs. lbe, lbm:equilibrium, sc; Sec. 2.3 Eqs. spreading, interpolation)."""
import os

import numpy as np
import pytest

from oracle import orc
from tests import brute_lbm

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_velocity_set_matches_paper_weights():
    c, w = orc.lattice()
    table = {}
    for line in open(os.path.join(GOLD, "d3q19_weights.txt")):
        if line.strip() and not line.startswith("#"):
            s, mult, num, den = (int(t) for t in line.split())
            table[s] = (mult, num / den)
    s2 = (c * c).sum(1)
    for s, (mult, wt) in table.items():
        assert (s2 == s).sum() == mult
        assert np.all(w[s2 == s] == wt)
    assert abs(w.sum() - 1) < 1e-15
    # isotropy: sum w c c = c_s^2 I with c_s^2 = 1/3, odd moments vanish
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, c, c), np.eye(3) / 3, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia->a", w, c), 0, atol=1e-17)
    # opposite pairs adjacent: c[2k] = -c[2k-1]
    for i in range(1, 19, 2):
        assert (c[i] == -c[i + 1]).all()


def _random_dev(shape, seed, eps=1e-3):
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    _, w = orc.lattice()
    return eps * rng.standard_normal((19, nz, ny, nx)) * w[:, None, None, None]


@pytest.mark.parametrize("forcing", [orc.GUO, orc.SHAN_CHEN])
def test_rest_state_is_fixed_point(forcing):
    o = orc.Oracle((8, 6, 5), 0.8, forcing, 3)
    o.step(3)
    _, w = orc.lattice()
    # unshifted FP64 populations: sum w_i = 1 only up to rounding, so the rest
    # state is a fixed point to within a few ulp
    np.testing.assert_allclose(o.pops(), np.broadcast_to(w[:, None, None, None], (19, 5, 6, 8)),
                               rtol=0, atol=2e-16)
    assert np.abs(o.velocity()).max() < 1e-16


@pytest.mark.parametrize("forcing", [orc.GUO, orc.SHAN_CHEN])
@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_mass_conserved_momentum_gains_force(forcing, tau):
    # collision conserves mass; momentum grows by exactly the applied force
    # (the total body force here is a uniform g plus point forces spread by IBM)
    shape = (9, 8, 7)
    o = orc.Oracle(shape, tau, forcing, 3)
    o.set_deviation(_random_dev(shape, 0))
    rng = np.random.default_rng(5)
    r = rng.uniform(0, 8, (4, 3))
    fm = 1e-4 * rng.standard_normal((4, 3))
    o.add_points(r, fm)
    g = np.array([1e-6, -2e-6, 5e-7])
    o.set_body_force(g)
    c0 = o.conserved()
    N = np.prod(shape)
    for n in range(1, 4):
        o.step(1)
        c1 = o.conserved()
        assert abs(c1[0] - c0[0]) < 1e-13 * N
        if forcing == orc.GUO:
            dp = fm.sum(0) + g * N
        else:
            # Shan-Chen: the equilibrium is shifted by tau F, so post-collision
            # momentum changes by (1/tau) * tau F = F per step as well
            dp = fm.sum(0) + g * N
        np.testing.assert_allclose(c1[1:] - c0[1:], dp, rtol=0, atol=1e-14 * N)
        c0 = c1


@pytest.mark.parametrize("forcing", ["guo", "sc"])
@pytest.mark.parametrize("width", [2, 3, 4])
@pytest.mark.parametrize("shape", [(4, 5, 6), (6, 6, 6)])
def test_bruteforce_tiny_grid(forcing, width, shape):
    tau = 0.9
    o = orc.Oracle(shape, tau, orc.GUO if forcing == "guo" else orc.SHAN_CHEN, width)
    dev = _random_dev(shape, 7)
    o.set_deviation(dev)
    rng = np.random.default_rng(11)
    r = rng.uniform(-1, 7, (2, 3))
    fm = 1e-3 * rng.standard_normal((2, 3))
    o.add_points(r, fm)
    g = np.array([2e-5, 0, -1e-5])
    o.set_body_force(g)
    # brute-force state in its own velocity ordering
    cb, wb = brute_lbm.velocity_set()
    co, wo = orc.lattice()
    perm = [int(np.where((cb == co[i]).all(1))[0][0]) for i in range(19)]
    f = np.zeros_like(dev)
    f[perm] = dev + wo[:, None, None, None]
    rb = r.copy()
    for _ in range(3):
        o.step(1)
        f, rb, u, rho, F = brute_lbm.step(f, rb, fm, shape, tau, width, forcing, g)
        np.testing.assert_allclose(o.velocity(), u, rtol=0, atol=1e-14)
        np.testing.assert_allclose(o.density(), rho, rtol=0, atol=1e-14)
        np.testing.assert_allclose(o.force(), F - g[:, None, None, None], rtol=0, atol=1e-15)
        np.testing.assert_allclose(o.pops(), f[perm], rtol=0, atol=1e-15)
        np.testing.assert_allclose(o.markers(), rb, rtol=0, atol=1e-14)


def _shear_nu(N, tau, steps):
    c, w = orc.lattice()
    o = orc.Oracle((N, N, 4), tau, orc.GUO, 3)
    y = np.arange(N)
    U0 = 1e-5
    ux = U0 * np.sin(2 * np.pi * y / N)
    dev = np.zeros((19, 4, N, N))
    for i in range(19):
        cu = c[i, 0] * ux
        dev[i] = (w[i] * (3 * cu + 4.5 * cu * cu - 1.5 * ux * ux))[None, :, None]
    o.set_deviation(dev)
    s = np.sin(2 * np.pi * y / N)
    o.step(10)
    a0 = (o.velocity()[0][0, :, 0] * s).sum()
    o.step(steps)
    a1 = (o.velocity()[0][0, :, 0] * s).sum()
    k = 2 * np.pi / N
    return -np.log(a1 / a0) / (k * k * steps)


def test_shear_wave_viscosity():
    # nu = c_s^2 (tau - 1/2) = (tau - 1/2)/3 (Sec. 2.1, with rho0 = 1), reached at
    # second order in the wavenumber
    tau = 0.8
    ex = (tau - 0.5) / 3
    errs = [abs(_shear_nu(N, tau, N * N // 4) / ex - 1) for N in (16, 32, 64)]
    assert errs[2] < 1e-3
    assert errs[0] / errs[1] > 3.2 and errs[1] / errs[2] > 3.2


def _poiseuille(ny, tau, forcing=orc.GUO, F=1e-6):
    nu = (tau - 0.5) / 3
    o = orc.Oracle((1, ny, 1), tau, forcing, 3)
    o.set_walls_y(True)
    o.set_body_force([F, 0, 0])
    o.step(int(35 * ny * ny / nu / np.pi ** 2) + 200)
    u = o.velocity()[0][0, :, 0]
    y = np.arange(ny)
    ex = F / (2 * nu) * (y + 0.5) * (ny - 0.5 - y)
    return np.abs(u - ex).max() / ex.max()


def test_poiseuille_exact_at_magic_tau():
    # Half-way bounce-back with Guo forcing reproduces the parabola exactly when
    # (tau - 1/2)^2 = 3/16 (wall at y = -1/2, ny - 1/2)
    assert _poiseuille(12, 0.5 + np.sqrt(3) / 4) < 1e-9


def test_poiseuille_second_order():
    e1, e2 = _poiseuille(8, 1.2), _poiseuille(16, 1.2)
    assert 3.5 < e1 / e2 < 4.5
