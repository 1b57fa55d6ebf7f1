"""Hand-written discrete adjoint on the GPU (lbm_adjoint) against the FP64
gradient oracle (reverse-mode differentiation of an independent forward
model), on the reduced adjoint workload: 24^3 box, 3-point kernel, Guo
forcing (Shan-Chen in its own tests), spacing-7 swimmer, A = B = 1e-3,
alpha = pi/3, period 2000."""
import math
import os

import numpy as np
import pytest

from oracle import adjoint as oracle_adjoint
from paper_2202_12147_amd import lbmib, workloads
from tests.helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "adjoint_24.txt")

# FP32 grid arithmetic against FP64, per component of J and of the gradient:
# over tens of steps the FP32 rounding of the grid adjoint stays near 1e-6;
# over a 2000-step period the FP32 forward trajectory itself drifts by ~1e-5
# and the gradient by a few 1e-4, inside the 1e-3 bound for the full period
SHORT_RTOL = 2e-5
PERIOD_RTOL = 1e-3


def _case(width=3, tau=1.0):
    c = workloads.adjoint_case(reduced=True)
    c["width"] = width
    c["tau"] = tau
    return c


def _check(J, g, Jo, go, rtol):
    print(f"J gpu {J:.10e} oracle {Jo:.10e} rel {abs(J - Jo) / abs(Jo):.2e}; grad gpu {g} oracle {go} "
          f"rel {np.abs(g - go) / np.abs(go)}", flush=True)
    assert abs(J - Jo) <= rtol * abs(Jo)
    assert np.all(np.abs(g - go) <= rtol * np.abs(go)), (g, go)


def test_single_step_is_degenerate():
    """After one step only the self-interaction of each bead has acted: the
    middle and last beads carry opposite forces and identical meshes at the
    same lattice alignment, so the centre does not move and no parameter
    changes that to first order (J and grad vanish up to rounding)."""
    case = _case()
    J, g = lbmib.from_workload(case).adjoint(1, checkpoint=16)
    Jo, go = oracle_adjoint.displacement_gradient(case, 1, checkpoint_every=0)
    assert abs(J) < 1e-12 and abs(Jo) < 1e-12
    assert np.abs(g).max() < 1e-10 and np.abs(go).max() < 1e-10


@pytest.mark.parametrize("steps", [40, 120])
def test_short_horizons_match_oracle(steps):
    case = _case()
    lat = lbmib.from_workload(case)
    J, g = lat.adjoint(steps, checkpoint=16)
    Jo, go = oracle_adjoint.displacement_gradient(case, steps, checkpoint_every=0)
    _check(J, g, Jo, go, SHORT_RTOL)


@pytest.mark.parametrize("steps,tau", [(40, 1.0), (120, 1.0), (40, 0.8)])
def test_shan_chen_matches_oracle(steps, tau):
    """Shan-Chen forcing (Eq. sc): the collision's equilibrium at
    (j + tau F)/rho and no source term, interpolation of (j + F/2)/rho; the
    adjoint of that collision against the gradient oracle over short
    horizons, with the short-horizon bar."""
    case = _case(tau=tau)
    case["forcing"] = workloads.SHAN_CHEN
    lat = lbmib.from_workload(case)
    J, g = lat.adjoint(steps, checkpoint=16)
    Jo, go = oracle_adjoint.displacement_gradient(case, steps, checkpoint_every=0)
    _check(J, g, Jo, go, SHORT_RTOL)


@pytest.mark.parametrize("width,tau", [(2, 1.0), (4, 0.8)])
def test_other_kernels_match_oracle(width, tau):
    case = _case(width, tau)
    lat = lbmib.from_workload(case)
    J, g = lat.adjoint(24, checkpoint=10)
    Jo, go = oracle_adjoint.displacement_gradient(case, 24, checkpoint_every=0)
    _check(J, g, Jo, go, SHORT_RTOL)


def test_full_period_matches_golden():
    """One full 2000-step period, checkpoints every 100 steps, against the
    stored FP64 oracle gradient (tests/golden/make_adjoint_golden.py)."""
    vals = np.loadtxt(GOLDEN)
    Jo, go = vals[0], vals[1:]
    case = _case()
    lat = lbmib.from_workload(case)
    J, g = lat.adjoint(case["steps"], checkpoint=case["checkpoint"])
    _check(J, g, Jo, go, PERIOD_RTOL)


def test_checkpointed_equals_store_all():
    case = _case()
    a = lbmib.from_workload(case)
    b = lbmib.from_workload(case)
    Ja, ga = a.adjoint(150, checkpoint=40)
    Jb, gb = b.adjoint(150, checkpoint=150)
    assert Ja == Jb
    assert np.array_equal(ga, gb)


def test_direct_launches_equal_graphs():
    """Five segments (the recompute of each overlapping the reverse sweep of
    the next, the two segment buffers reused twice) issued directly and
    replayed from captured graphs give the same bits."""
    case = _case()
    a = lbmib.from_workload(case, use_graphs=False)
    b = lbmib.from_workload(case)
    Ja, ga = a.adjoint(90, checkpoint=20)
    Jb, gb = b.adjoint(90, checkpoint=20)
    assert Ja == Jb
    assert np.array_equal(ga, gb)


def test_full_size_gradient_matches_central_differences():
    """The 96^3 workload at full size, as the benchmark runs it (one 2000-step
    period, checkpoints every 100 steps, default launch shape): dJ/dA and
    dJ/dk of the adjoint against central differences of the GPU forward run
    at a 1 % step.  The displacement is, to leading order, bilinear in the two
    amplitudes, so the difference in A carries no truncation error (measured
    1e-5); in k it is O(h^2): 7e-4 measured at a 2 % step, so ~2e-4 at 1 %.
    The two FP32 forward runs of a difference agree to ~1e-5 of J, i.e. a
    few 1e-4 of the differenced J; the adjoint's own FP32 rounding over a
    period is ~1e-4 (reduced case).  Bar: 1e-3."""
    case = workloads.adjoint_case(reduced=False)
    T, K = case["steps"], case["checkpoint"]
    sw = case["swimmers"][0]
    theta = np.array([sw["A"], sw["B"], sw["alpha"], sw["k"][0]], dtype=np.float64)
    lat = lbmib.from_workload(case)
    J, g = lat.adjoint(T, checkpoint=K)

    def displacement(th):
        h = lbmib.from_workload(case)
        h.set_swimmer_params(0, *th)
        x0 = h.swimmer_centres()[0, 0]
        h.step(T)
        return h.swimmer_centres()[0, 0] - x0

    assert abs(displacement(theta) - J) <= 1e-12
    for i in (0, 3):
        d = 0.01 * theta[i]
        tp, tm = theta.copy(), theta.copy()
        tp[i] += d
        tm[i] -= d
        fd = (displacement(tp) - displacement(tm)) / (2.0 * d)
        print(f"parameter {i}: adjoint {g[i]:.8e} central difference {fd:.8e} "
              f"rel {abs(g[i] - fd) / abs(fd):.2e}", flush=True)
        assert abs(g[i] - fd) <= 1e-3 * abs(fd)


def test_state_after_adjoint():
    """Without rewind the handle ends exactly where lbm_step(T) takes it;
    with rewind it is back at its entry state."""
    case = _case()
    a = lbmib.from_workload(case)
    b = lbmib.from_workload(case)
    a.step(7)
    b.step(7)
    a.adjoint(50, checkpoint=20)
    b.step(50)
    assert a.time == b.time == 57
    assert np.array_equal(a.markers(), b.markers())
    assert np.array_equal(a.populations(), b.populations())
    m0, p0 = b.markers(), b.populations()
    b.adjoint(30, checkpoint=16, rewind=True)
    assert b.time == 57
    assert np.array_equal(b.markers(), m0)
    assert np.array_equal(b.populations(), p0)
    # stepping resumes identically after a rewind
    a.step(5)
    b.step(5)
    assert np.array_equal(a.markers(), b.markers())


def test_set_params_matches_construction():
    case = _case()
    other = _case()
    sw = other["swimmers"][0]
    sw.update(A=7e-4, B=1.3e-3, alpha=1.1)
    sw["k"] = np.array([0.02, 0.02])
    a = lbmib.from_workload(case)
    a.set_swimmer_params(0, 7e-4, 1.3e-3, 1.1, 0.02)
    b = lbmib.from_workload(other)
    a.step(20)
    b.step(20)
    assert np.array_equal(a.markers(), b.markers())


def test_autograd_function():
    import torch
    case = _case()
    sw = case["swimmers"][0]
    theta = torch.tensor([sw["A"], sw["B"], sw["alpha"], sw["k"][0]], dtype=torch.float64,
                         requires_grad=True)
    lat = lbmib.from_workload(case)
    J = lbmib.swimmer_displacement(lat, theta, 40, checkpoint=16)
    (2.0 * J).backward()
    ref = lbmib.from_workload(case)
    Jr, gr = ref.adjoint(40, checkpoint=16)
    assert float(J.detach()) == Jr
    assert np.array_equal(theta.grad.numpy(), 2.0 * gr)
    assert lat.time == 0  # rewound


def test_adjoint_rejects_unsupported():
    case = _case()
    fp16 = lbmib.from_workload(case, storage=lbmib.FP16_SHIFTED, fp16_scale=2.0 ** 20)
    with pytest.raises(lbmib.LbmError):
        fp16.adjoint(10)
    lat = lbmib.from_workload(case)
    for kw in (dict(steps=0), dict(steps=10, checkpoint=0), dict(steps=10, swimmer=1)):
        with pytest.raises(lbmib.LbmError):
            lat.adjoint(**kw)
    ens = workloads.ensemble(seed=0, nboxes=2)
    with pytest.raises(lbmib.LbmError):
        lbmib.batch_from_ensemble(ens).adjoint(10)
    assert not math.isnan(lat.adjoint(2)[0])


@pytest.mark.parametrize("shape", [(24, 24, 24), (25, 22, 23)])
def test_adjoint_across_periodic_seams(shape):
    """Swimmer straddling the x and y seams: the transposed spreading and
    interpolation wrap like the forward ones.  The 25x22x23 box has no edge
    that is a whole number of 8-node tiles."""
    case = _case()
    case["shape"] = shape
    mid = (shape[0] - 0.5, 0.4, shape[2] / 2)
    case["swimmers"] = [workloads.swimmer(mid, 7.0, A=1e-3, T=2000.0, alpha=math.pi / 3)]
    lat = lbmib.from_workload(case)
    J, g = lat.adjoint(40, checkpoint=16)
    Jo, go = oracle_adjoint.displacement_gradient(case, 40, checkpoint_every=0)
    _check(J, g, Jo, go, SHORT_RTOL)
