"""Pins of the coupled oracle: bead-spring swimmers and beads in the fluid
(paper Sec. 2.2-2.3; swimmer centre of Eq. vel_swim)."""
import math
import os

import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import orc
from paper_2202_12147_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _small(steps, **kw):
    c = wl.small_case()
    o = orc.Oracle(c["shape"], c["tau"], c["forcing"], c["width"])
    sw = wl.swimmer((16, 16, 16), 10.0, **kw)
    o.add_swimmer_desc(sw)
    X0 = o.swimmer_centres().copy()
    return o, X0


def test_mirror_symmetry_and_momentum():
    # the swimmer axis is a mirror axis of mesh and placement: no drift in y or z
    # (P12); all forces on the swimmer sum to zero, so fluid momentum stays 0 (P3)
    o, X0 = _small(0)
    o.step(300)
    X = o.swimmer_centres()
    assert abs(X[0, 1] - X0[0, 1]) < 1e-12 and abs(X[0, 2] - X0[0, 2]) < 1e-12
    assert abs(X[0, 0] - X0[0, 0]) > 1e-6
    c = o.conserved()
    assert np.abs(c[1:]).max() < 1e-9
    f = o.marker_forces()
    assert np.abs(f.sum(0)).max() < 1e-15


def test_no_actuation_nothing_moves():
    o, X0 = _small(0, A=0.0, B=0.0)
    r0 = o.markers().copy()
    o.step(50)
    assert np.abs(o.markers() - r0).max() < 1e-15
    assert np.abs(o.velocity()).max() < 1e-16


def test_driving_forces_sum_to_zero_and_follow_phase():
    # with stiff springs removed (k = 0) the bead forces are the driving forces:
    # f1 = A sin(w t), f3 = B sin(w t + alpha), f2 = -f1 - f3 (Sec. 2.2)
    o, _ = _small(0, k=0.0, A=1e-3, B=7e-4, T=40.0, alpha=1.1)
    nv = o.n_markers // 3
    for n in range(5):
        o.step(1)
        f = o.marker_forces().reshape(3, nv, 3).sum(1)
        t = n
        w = 2 * math.pi / 40.0
        ex1, ex3 = 1e-3 * math.sin(w * t), 7e-4 * math.sin(w * t + 1.1)
        # membrane forces add zero net force per bead
        assert abs(f[0, 0] - ex1) < 1e-15 and abs(f[2, 0] - ex3) < 1e-15
        assert abs(f[1, 0] + ex1 + ex3) < 1e-15
        assert np.abs(f[:, 1:]).max() < 1e-15


def test_spring_force_magnitude():
    # with no driving, stretched springs pull the outer beads inward with
    # k (|R1 - R2| - L) (Sec. 2.2)
    c = wl.small_case()
    o = orc.Oracle(c["shape"], 1.0, orc.GUO, 3)
    sw = wl.swimmer((16, 16, 16), 10.0, A=0.0)
    sw["L0"] = np.array([9.5, 9.0])
    o.add_swimmer_desc(sw)
    o.step(1)
    nv = o.n_markers // 3
    f = o.marker_forces().reshape(3, nv, 3).sum(1)
    np.testing.assert_allclose(f[0], [0.01 * 0.5, 0, 0], atol=1e-15)
    np.testing.assert_allclose(f[2], [-0.01 * 1.0, 0, 0], atol=1e-15)
    np.testing.assert_allclose(f[1], [0.01 * 0.5, 0, 0], atol=1e-15)


def _hasimoto():
    out = {}
    for line in open(os.path.join(GOLD, "hasimoto_1959.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def _drag_radius(L, tau=1.5, a=2.5, F0=1e-3, steps=1500):
    o = orc.Oracle((L, L, L), tau, orc.GUO, 3)
    c = L // 2
    o.add_bead((c, c, c), a, 2, 0.1, 4.5, 1.25e-3, 1.0, (F0, 0, 0))
    o.set_body_force([-F0 / L ** 3, 0, 0])
    o.step(steps - 100)
    R0 = o.bead_centres()[0].copy()
    o.step(100)
    U = (o.bead_centres()[0] - R0)[0] / 100
    mu = (tau - 0.5) / 3
    h = _hasimoto()

    def res(ae):
        x = ae / L
        return F0 * (1 - h["c1"] * x + h["c3"] * x ** 3 - h["c6"] * x ** 6) / (6 * math.pi * mu * ae) - U

    return brentq(res, 0.5, 6.0)


def test_stokes_drag_periodic_array():
    # A forced bead in a periodic box (compensating uniform body force) moves
    # at Hasimoto's periodic-array Stokes velocity with one effective radius
    # that does not depend on the box size.
    a16, a24 = _drag_radius(16), _drag_radius(24)
    assert abs(a16 - a24) < 0.05
    assert 0.9 < a24 / 2.5 < 1.3
