"""GPU test of the allocation-free conserved-sum entry point
(lbm_batch_get_conserved_noalloc): its partial sums live in the library's
static device scratch instead of handle memory, and it neither allocates nor
synchronises.  Checked against lbm_batch_get_conserved on the same states:
bitwise at the same partial count (same kernels, same summation order), and
within FP64 rounding at other counts, on two calls in a row, the second with
a smaller input."""
import numpy as np
import pytest

from paper_2202_12147_amd import lbmib, workloads as wl

pytestmark = pytest.mark.gpu


def _state(shape, seed, eps=1e-3):
    lat = lbmib.Lattice(shape, 0.9)
    lat.set_populations(wl.random_deviation(shape, seed, eps))
    lat.set_body_force((3e-6, -2e-6, 1e-6))
    lat.step(3)
    return lat


def _noalloc(lat, box=-1, parts=1024):
    import torch
    dst = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda:0")
    lat.conserved_noalloc(dst, box, parts)
    lat.sync()
    return dst.cpu().numpy()


def test_noalloc_conserved_matches_the_allocating_call():
    big = _state((48, 40, 36), seed=3)
    small = _state((20, 17, 19), seed=4)
    for lat in (big, small):  # second call: a smaller input, same scratch
        print("case", lat.shape, flush=True)
        ref = lat.conserved()
        got = _noalloc(lat)
        assert np.array_equal(got, ref), (got, ref)
        # another partial count changes only the FP64 summation order
        for parts in (1, 37, 4096):
            other = _noalloc(lat, parts=parts)
            assert np.allclose(other, ref, rtol=0, atol=1e-12 * lat.N), (parts, other, ref)
    # the first handle again, after the smaller one overwrote the scratch
    assert np.array_equal(_noalloc(big), big.conserved())


def test_noalloc_conserved_batch_boxes_and_limits():
    ens = wl.ensemble(seed=2, nboxes=3)
    b = lbmib.batch_from_ensemble(ens)
    b.step(20)
    for box in (-1, 0, 2, 1):
        assert np.array_equal(_noalloc(b, box), b.conserved(box)), box
    import torch
    dst = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    for parts in (0, 4097):
        with pytest.raises(lbmib.LbmError, match="LBM_EINVAL"):
            b.conserved_noalloc(dst, -1, parts)
    with pytest.raises(lbmib.LbmError, match="LBM_EINVAL"):
        b.conserved_noalloc(dst, 3, 1024)
