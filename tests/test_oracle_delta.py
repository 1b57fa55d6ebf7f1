"""Pins of the oracle's discrete delta kernels, spreading and interpolation
(paper Sec. 2.3, Eqs. spreading and interpolation; kernel widths 2, 3, 4)."""
import numpy as np
import pytest

from oracle import orc

WIDTHS = (2, 3, 4)
SUPPORT = {2: 1.0, 3: 1.5, 4: 2.0}


def _moments(width, r):
    j = np.arange(np.floor(r) - 3, np.floor(r) + 4)
    p = np.array([orc.phi(width, x - r) for x in j])
    return p.sum(), ((j - r) * p).sum(), (p * p).sum()


@pytest.mark.parametrize("width", WIDTHS)
def test_partition_of_unity_and_first_moment(width):
    # A valid IB kernel sums to one and has zero first moment at every offset.
    for r in np.linspace(0.0, 1.0, 41):
        s0, s1, _ = _moments(width, r + 7.0)
        assert abs(s0 - 1.0) < 1e-15
        assert abs(s1) < 1e-15


@pytest.mark.parametrize("width,val", [(3, 0.5), (4, 0.375)])
def test_sum_of_squares(width, val):
    # Roma-Peskin-Berger (3-point) and Peskin (4-point) kernels are built so that
    # sum_j phi(r-j)^2 is independent of r: 1/2 and 3/8.
    for r in np.linspace(0.0, 1.0, 41):
        assert abs(_moments(width, r)[2] - val) < 1e-15


@pytest.mark.parametrize("width", WIDTHS)
def test_support_symmetry_continuity(width):
    a = SUPPORT[width]
    for r in np.linspace(-3, 3, 121):
        assert orc.phi(width, r) == orc.phi(width, -r)
        assert orc.phi(width, r) >= 0.0
        if abs(r) >= a:
            assert orc.phi(width, r) == 0.0
    # continuity at the piece boundaries and at the support edge
    eps = 1e-9
    for b in np.arange(0.5, a + 0.01, 0.5):
        assert abs(orc.phi(width, b - eps) - orc.phi(width, b + eps)) < 1e-6


def _random_markers(rng, m, shape):
    return rng.uniform(0, 1, (m, 3)) * np.array(shape)


@pytest.mark.parametrize("width", WIDTHS)
def test_spread_total_and_adjointness(width):
    rng = np.random.default_rng(1)
    shape = (7, 6, 5)  # smaller than a few stencils: every periodic image matters
    r = _random_markers(rng, 9, shape) + rng.integers(-2, 3, (9, 3)) * np.array(shape)
    f = rng.standard_normal((9, 3))
    F = orc.spread(shape, width, r, f)
    np.testing.assert_allclose(F.reshape(3, -1).sum(1), f.sum(0), rtol=0, atol=1e-14)
    u = rng.standard_normal((3,) + F.shape[1:])
    U = orc.interp(shape, width, r, u)
    lhs = (F * u).sum()
    rhs = (f * U).sum()
    assert abs(lhs - rhs) <= 1e-14 * max(1.0, abs(lhs))


@pytest.mark.parametrize("width", WIDTHS)
def test_interp_uniform_and_linear(width):
    rng = np.random.default_rng(2)
    shape = (16, 12, 10)
    nx, ny, nz = shape
    r = rng.uniform(4, 6, (20, 3))
    u = np.empty((3, nz, ny, nx))
    u[0], u[1], u[2] = 0.3, -1.2, 2.5
    U = orc.interp(shape, width, r, u)
    np.testing.assert_allclose(U, np.tile([0.3, -1.2, 2.5], (20, 1)), rtol=0, atol=1e-14)
    # linear field (markers far from the periodic seam): value at r
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u[0] = 0.5 * x - 0.25 * y + 0.125 * z
    u[1] = y.astype(float)
    u[2] = 2.0 - z
    U = orc.interp(shape, width, r, u)
    ex = np.stack([0.5 * r[:, 0] - 0.25 * r[:, 1] + 0.125 * r[:, 2], r[:, 1], 2.0 - r[:, 2]], 1)
    np.testing.assert_allclose(U, ex, rtol=0, atol=1e-13)
