"""Seeded synthetic workloads shaped like the paper's runs.

This module holds parameter draws and placements only: no lattice Boltzmann,
immersed-boundary or membrane arithmetic.  Both the HIP path and the oracle
are fed from here, so the two sides start from the same numbers.

Unless stated, every swimmer uses the bead model of the small reference case:
radius 2.5 icosphere beads with 320 triangles (level 2), Skalak shear modulus
ks = 0.1, bending modulus 1.25e-3 and volume modulus 1 (paper Sec. 3),
harmonic springs k = 0.01, actuation B = A and alpha = pi/2.

Skalak C = 0 (area modulus equal to the shear modulus).  The paper's area
modulus ka = 1 (C = 4.5 at ks = 0.1) makes the explicit coupling unstable on
these meshes, whose edges (0.53-0.66 lattice units) are finer than the paper's
radius-5 beads: a membrane mode grows from rounding noise and the run diverges
after a few thousand steps.  C = 0 stays stable for tau in [0.6, 1.2].
"""
import math

import numpy as np

GUO, SHAN_CHEN = 0, 1

BEAD_DEFAULTS = dict(ks=0.1, C=0.0, kb=1.25e-3, kv=1.0)


def swimmer(middle, spacing, radius=2.5, level=2, k=0.01, A=1e-3, B=None, T=500.0,
            alpha=math.pi / 2, phi0=0.0, axis=0, **bead):
    """Three beads along ``axis`` with the middle one at ``middle``.

    ``spacing`` and ``radius`` may be scalars or per-spring / per-bead
    sequences."""
    sp = np.broadcast_to(np.asarray(spacing, float), (2,)).copy()
    rad = np.broadcast_to(np.asarray(radius, float), (3,)).copy()
    mid = np.asarray(middle, float)
    e = np.zeros(3)
    e[axis] = 1.0
    centres = np.stack([mid - sp[0] * e, mid, mid + sp[1] * e])
    p = dict(BEAD_DEFAULTS)
    p.update(bead)
    return dict(centres=centres, radius=rad, level=int(level), k=np.array([k, k], float),
                L0=sp, A=float(A), B=float(A if B is None else B), T=float(T),
                alpha=float(alpha), phi0=float(phi0), **p)


def small_case():
    """32^3 box, tau 1, Guo forcing, 3-point kernel, one swimmer with bead
    centres 10 apart, A = 1e-3, period 500, 1000 steps."""
    shape = (32, 32, 32)
    return dict(name="single swimmer 32^3 (FP64 reference case)", shape=shape, tau=1.0,
                forcing=GUO, width=3, steps=1000,
                swimmers=[swimmer((16, 16, 16), 10.0, radius=2.5, level=2, A=1e-3, T=500.0)])


def single_128(seed=0):
    """128^3 box, tau 0.8, 4-point kernel, radius-4 beads with 1280 triangles,
    spacing 16, A = 5e-4, period 2000, 20000 steps; random phase offset in
    [0, 2 pi) and independent +-1% jitter on each bead radius and spring rest
    length."""
    rng = np.random.default_rng(seed)
    phi0 = rng.uniform(0.0, 2 * math.pi)
    rad = 4.0 * (1 + rng.uniform(-0.01, 0.01, 3))
    sp = 16.0 * (1 + rng.uniform(-0.01, 0.01, 2))
    return dict(name="single swimmer 128^3", shape=(128, 128, 128), tau=0.8, forcing=GUO,
                width=4, steps=20000, seed=seed,
                swimmers=[swimmer((64, 64, 64), sp, radius=rad, level=3, A=5e-4, T=2000.0,
                                  phi0=phi0)])


def pair_256(seed=0, arrangement="collinear"):
    """256x128x128 box, two small-case swimmers, collinear (middle beads 40
    apart along x) or side by side (20 apart along y); the second swimmer's
    phase lags by a draw from [0, pi); 10000 steps."""
    rng = np.random.default_rng(seed)
    dphi = rng.uniform(0.0, math.pi)
    c = np.array([128.0, 64.0, 64.0])
    off = np.array([20.0, 0, 0]) if arrangement == "collinear" else np.array([0, 10.0, 0])
    sw = [swimmer(c - off, 10.0, T=500.0, phi0=0.0), swimmer(c + off, 10.0, T=500.0, phi0=dphi)]
    return dict(name=f"two swimmers 256x128x128 ({arrangement})", shape=(256, 128, 128),
                tau=1.0, forcing=GUO, width=3, steps=10000, seed=seed, swimmers=sw)


def ensemble(seed=0, nboxes=64):
    """Independent periodic boxes with edges drawn from {48, 64, 80, 96} per
    axis, tau in [0.6, 1.2], one swimmer each with spacing in [8, 16],
    amplitude in [2e-4, 1e-3], phase shift in [pi/4, 3 pi/4], period 1000;
    5000 steps."""
    rng = np.random.default_rng(seed)
    boxes = []
    for _ in range(nboxes):
        shape = tuple(int(v) for v in rng.choice([48, 64, 80, 96], 3))
        tau = float(rng.uniform(0.6, 1.2))
        sp = float(rng.uniform(8.0, 16.0))
        A = float(rng.uniform(2e-4, 1e-3))
        alpha = float(rng.uniform(math.pi / 4, 3 * math.pi / 4))
        mid = tuple(s // 2 for s in shape)
        boxes.append(dict(shape=shape, tau=tau, forcing=GUO, width=3,
                          swimmers=[swimmer(mid, sp, A=A, T=1000.0, alpha=alpha)]))
    return dict(name=f"{nboxes} independent boxes", boxes=boxes, steps=5000, seed=seed)


def adjoint_case(reduced=False):
    """Gradient of a swimmer's x-displacement over one 2000-step period with
    respect to (A, B, alpha, k); checkpoints every 100 steps.  The full case is
    96^3; the reduced case is 24^3 with bead spacing 7 so that the swimmer does
    not overlap its own periodic image."""
    if reduced:
        shape, sp = (24, 24, 24), 7.0
    else:
        shape, sp = (96, 96, 96), 10.0
    mid = tuple(s // 2 for s in shape)
    return dict(name=f"adjoint {shape[0]}^3", shape=shape, tau=1.0, forcing=GUO, width=3,
                steps=2000, checkpoint=100,
                swimmers=[swimmer(mid, sp, A=1e-3, T=2000.0, alpha=math.pi / 3)])


def paper_box():
    """The paper's box (Sec. 3): 1024x256x256, tau 1, 3-point kernel, one
    swimmer of radius-5 beads (1280 triangles) with rest length 36, spring
    constant 0.02, amplitudes A = B = 5e-3, alpha = pi/2, period 2e4; for
    throughput (a few hundred steps)."""
    return dict(name="paper box 1024x256x256", shape=(1024, 256, 256), tau=1.0, forcing=GUO, width=3,
                steps=500,
                swimmers=[swimmer((512, 128, 128), 36.0, radius=5.0, level=3, k=0.02, A=5e-3, T=2e4,
                                  alpha=math.pi / 2)])


PAPER_MODULI = dict(ks=0.05, C=9.5, kb=1.25e-3, kv=1.0)


def paper_moduli_case(adjoint=False):
    """The paper's membrane moduli (Sec. 3: ks = 0.05, ka = 1, i.e. C = 9.5,
    kb = 1.25e-3, kv = 1) on its radius-5 beads, refined twice (320
    triangles, mean edge ~1.3 l.u.: the paper does not give the refinement;
    with three refinements the explicit coupling diverges after ~1500 steps).
    Swimmer as in the paper (rest length 36, k = 0.02, A = B = 5e-3,
    alpha = pi/2) with the period shortened to 2000 steps so that the
    driving acts within a short comparison; 112x48x48 box, tau 1, Guo,
    3-point kernel.  adjoint=True: a 48x32x32 box, rest length 12,
    alpha = pi/3 (a gradient case small enough for the gradient oracle)."""
    if adjoint:
        return dict(name="paper moduli, adjoint 48x32x32", shape=(48, 32, 32), tau=1.0, forcing=GUO,
                    width=3, steps=2000, checkpoint=100,
                    swimmers=[swimmer((24, 16, 16), 12.0, radius=5.0, level=2, k=0.02, A=5e-3, T=2000.0,
                                      alpha=math.pi / 3, **PAPER_MODULI)])
    return dict(name="paper moduli 112x48x48", shape=(112, 48, 48), tau=1.0, forcing=GUO, width=3,
                steps=200,
                swimmers=[swimmer((56, 24, 24), 36.0, radius=5.0, level=2, k=0.02, A=5e-3, T=2000.0,
                                  **PAPER_MODULI)])


def paper_run(arrangement=None, distance=None, tau=1.0):
    """The paper's single-swimmer run (Sec. 3): 1024x256x256 fully periodic
    box, tau 1 (mu = 1/6; other tau for the paper's viscosity sweeps, mu =
    (tau - 1/2)/3 at rho0 = 1), Shan-Chen forcing as in the paper, radius-5 beads
    with the paper's moduli (refined twice, as in paper_moduli_case), rest
    length 36, k = 0.02, A = B = 5e-3 (the printed A = 1e-1 contradicts the
    bead Reynolds number the paper reports), T = 2e4, alpha = pi/2, 3-point
    kernel (the two-point kernel diverges within 500 steps with these
    moduli, also in the oracle); at least 12 periods to stationarity.

    arrangement "collinear" (Sec. 3.2) or "side" (Sec. 3.3): two identical,
    in-phase swimmers whose middle beads are `distance` apart along x (one
    behind the other) or along y (side by side), centred in the box."""
    def one(mid):
        return swimmer(mid, 36.0, radius=5.0, level=2, k=0.02, A=5e-3, T=2e4, alpha=math.pi / 2, **PAPER_MODULI)
    if arrangement is None:
        swimmers, name = [one((512, 128, 128))], "paper run 1024x256x256"
    else:
        h = 0.5 * float(distance)
        if arrangement == "collinear":
            mids = [(512 - h, 128, 128), (512 + h, 128, 128)]
        elif arrangement == "side":
            mids = [(512, 128 - h, 128), (512, 128 + h, 128)]
        else:
            raise ValueError(arrangement)
        swimmers, name = [one(m) for m in mids], f"paper pair run 1024x256x256, {arrangement}, d = {distance:g}"
    if tau != 1.0:
        name += f", tau = {tau:g}"
    return dict(name=name, shape=(1024, 256, 256), tau=float(tau), forcing=SHAN_CHEN, width=3, steps=12 * 20000,
                period=20000, swimmers=swimmers)


def random_deviation(shape, seed=0, eps=1e-4, modes=3):
    """Smooth random population deviations [19, z, y, x]: a few random Fourier
    modes per population, amplitude ``eps``."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros((19, nz, ny, nx))
    for i in range(19):
        for _ in range(modes):
            kx, ky, kz = rng.integers(0, 3, 3)
            ph = rng.uniform(0, 2 * math.pi)
            a = rng.uniform(-1, 1)
            out[i] += a * np.sin(2 * math.pi * (kx * x / nx + ky * y / ny + kz * z / nz) + ph)
    return eps * out / modes
