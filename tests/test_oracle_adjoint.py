"""Pins of the FP64 gradient oracle (oracle/adjoint.py).

Its forward model is an independent re-implementation of the method, checked
against the C oracle's trajectory; its gradient (reverse-mode differentiation
of that forward, checkpointed) is checked against central finite differences
of the C oracle's objective, which share no code with it.
"""
import copy
import math

import numpy as np
import pytest
import torch

from oracle import adjoint
from paper_2202_12147_amd import workloads
from tests.helpers import oracle_from


def _theta(case):
    sw = case["swimmers"][0]
    return (sw["A"], sw["B"], sw["alpha"], sw["k"][0])


def _c_objective(case, steps):
    o = oracle_from(case)
    x0 = o.markers()[:, 0].mean()
    o.step(steps)
    return o.markers()[:, 0].mean() - x0


def test_forward_matches_c_oracle():
    """Same markers and populations as the C oracle after 30 steps of the
    reduced adjoint workload (24^3, 3-point kernel, Guo forcing)."""
    case = workloads.adjoint_case(reduced=True)
    model = adjoint.SwimmerModel(case)
    th = [torch.tensor(v, dtype=torch.float64) for v in _theta(case)]
    with torch.no_grad():
        J, f, r = model.run(th, 30)
    o = oracle_from(case)
    o.step(30)
    assert np.abs(o.markers() - r.numpy()).max() < 1e-12
    assert np.abs(o.pops() - f.numpy()).max() < 1e-13
    assert abs(float(J) - (o.markers()[:, 0].mean() - model.r0[:, 0].mean().item())) < 1e-13


@pytest.mark.parametrize("width", [3, 4])
def test_forward_matches_c_oracle_other_kernels(width):
    case = workloads.adjoint_case(reduced=True)
    case["width"] = width
    case["tau"] = 0.8
    model = adjoint.SwimmerModel(case)
    th = [torch.tensor(v, dtype=torch.float64) for v in _theta(case)]
    with torch.no_grad():
        _, f, r = model.run(th, 10)
    o = oracle_from(case)
    o.step(10)
    assert np.abs(o.markers() - r.numpy()).max() < 1e-12
    assert np.abs(o.pops() - f.numpy()).max() < 1e-13


def test_forward_matches_c_oracle_shan_chen():
    """Shan-Chen forcing (Eq. sc: the equilibrium at (j + tau F)/rho, no
    source term; interpolation of (j + F/2)/rho): the same markers and
    populations as the C oracle after 30 steps, at tau 1 and 0.8."""
    for tau in (1.0, 0.8):
        case = workloads.adjoint_case(reduced=True)
        case["forcing"] = workloads.SHAN_CHEN
        case["tau"] = tau
        model = adjoint.SwimmerModel(case)
        th = [torch.tensor(v, dtype=torch.float64) for v in _theta(case)]
        with torch.no_grad():
            _, f, r = model.run(th, 30)
        o = oracle_from(case)
        o.step(30)
        assert np.abs(o.markers() - r.numpy()).max() < 1e-12
        assert np.abs(o.pops() - f.numpy()).max() < 1e-13


@pytest.mark.parametrize("forcing", [workloads.GUO, workloads.SHAN_CHEN])
def test_gradient_matches_finite_differences(forcing):
    """dJ/d(A, B, alpha, k) over 120 steps against central differences of the
    C oracle's J with relative step 1e-4 (truncation ~1e-8, rounding ~1e-6),
    for both forcing schemes."""
    case = workloads.adjoint_case(reduced=True)
    case["forcing"] = forcing
    steps = 120
    J, g = adjoint.displacement_gradient(case, steps, checkpoint_every=40)
    assert abs(J - _c_objective(case, steps)) < 1e-13
    base = _theta(case)
    fd = []
    for i, name in enumerate(["A", "B", "alpha", "k"]):
        h = 1e-4 * abs(base[i])
        vals = []
        for s in (1, -1):
            c = copy.deepcopy(case)
            sw = c["swimmers"][0]
            if name == "k":
                sw["k"] = sw["k"] + s * h
            else:
                sw[name] = base[i] + s * h
            vals.append(_c_objective(c, steps))
        fd.append((vals[0] - vals[1]) / (2 * h))
    fd = np.array(fd)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())


def test_checkpointed_equals_store_all():
    """Recomputing K-step segments gives the gradient of the stored run
    bitwise (the recompute repeats the same deterministic CPU arithmetic)."""
    case = workloads.adjoint_case(reduced=True)
    J1, g1 = adjoint.displacement_gradient(case, 48, checkpoint_every=16)
    J2, g2 = adjoint.displacement_gradient(case, 48, checkpoint_every=0)
    assert J1 == J2
    assert np.array_equal(g1, g2)


def test_unforced_sensitivities():
    """A = B = 0, alpha = 0: nothing moves (J = 0); dJ/dalpha (proportional
    to B) and dJ/dk (proportional to the spring stretch) vanish; and the
    mirror symmetry x -> 24 - x of the box and beads, which swaps the outer
    beads and reverses x, makes the linear responses to the two driving
    patterns equal: dJ/dA = dJ/dB != 0."""
    case = workloads.adjoint_case(reduced=True)
    J, g = adjoint.displacement_gradient(case, 20, checkpoint_every=0, theta=(0.0, 0.0, 0.0, 0.01))
    assert abs(J) < 1e-15
    assert abs(g[2]) < 1e-15 and abs(g[3]) < 1e-15
    assert abs(g[0]) > 1e-6
    assert abs(g[0] - g[1]) < 1e-9 * abs(g[0])
