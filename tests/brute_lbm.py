"""Brute-force numpy model of one LBM + IBM step on tiny periodic grids.

Independent of the C oracle: its own velocity set (enumerated from the
definition of D3Q19), streaming by explicit array rolls, the delta kernel
summed over every node and every periodic image, moments and BGK collision
written from the paper's equations (Sec. 2.1, 2.3).  Markers are free points
with constant prescribed forces.  Test code only.
"""
import numpy as np


def velocity_set():
    c = [v for v in np.ndindex(3, 3, 3)]
    c = np.array(c) - 1
    c = c[(c * c).sum(1) <= 2]
    w = np.array([{0: 1 / 3, 1: 1 / 18, 2: 1 / 36}[int(s)] for s in (c * c).sum(1)])
    return c, w


def phi(width, r):
    r = np.abs(r)
    out = np.zeros_like(r)
    if width == 2:
        m = r < 1
        out[m] = 1 - r[m]
    elif width == 3:
        m1 = r <= 0.5
        m2 = (r > 0.5) & (r <= 1.5)
        out[m1] = (1 + np.sqrt(1 - 3 * r[m1] ** 2)) / 3
        out[m2] = (5 - 3 * r[m2] - np.sqrt(1 - 3 * (1 - r[m2]) ** 2)) / 6
    else:
        m1 = r <= 1
        m2 = (r > 1) & (r <= 2)
        out[m1] = (3 - 2 * r[m1] + np.sqrt(1 + 4 * r[m1] - 4 * r[m1] ** 2)) / 8
        out[m2] = (5 - 2 * r[m2] - np.sqrt(-7 + 12 * r[m2] - 4 * r[m2] ** 2)) / 8
    return out


def delta_matrix(shape, width, r):
    """D[m, z, y, x] = sum over images k of Delta(x + k N - r_m)."""
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    D = np.zeros((len(r),) + x.shape)
    for m, rm in enumerate(r):
        for kx in range(-3, 4):
            for ky in range(-3, 4):
                for kz in range(-3, 4):
                    D[m] += (phi(width, x + kx * nx - rm[0]) * phi(width, y + ky * ny - rm[1])
                             * phi(width, z + kz * nz - rm[2]))
    return D


def step(f, r, fm, shape, tau, width, forcing="guo", g=(0.0, 0.0, 0.0)):
    """One step from post-collision f* [19,z,y,x] and markers r [m,3] carrying
    forces fm [m,3].  Returns (f*_new, r_new, u, rho, F)."""
    c, w = velocity_set()
    D = delta_matrix(shape, width, r)
    F = np.einsum("mzyx,mk->kzyx", D, fm) + np.asarray(g)[:, None, None, None]
    fs = np.stack([np.roll(f[i], shift=(c[i, 2], c[i, 1], c[i, 0]), axis=(0, 1, 2)) for i in range(19)])
    rho = fs.sum(0)
    j = np.einsum("izyx,ik->kzyx", fs, c.astype(float))
    u = (j + F / 2) / rho
    ue = u if forcing == "guo" else (j + tau * F) / rho
    cu = np.einsum("ik,kzyx->izyx", c.astype(float), ue)
    uu = (ue * ue).sum(0)
    feq = w[:, None, None, None] * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)
    out = fs - (fs - feq) / tau
    if forcing == "guo":
        cuv = np.einsum("ik,kzyx->izyx", c.astype(float), u)
        cF = np.einsum("ik,kzyx->izyx", c.astype(float), F)
        uF = (u * F).sum(0)
        out = out + (1 - 0.5 / tau) * w[:, None, None, None] * (3 * (cF - uF) + 9 * cuv * cF)
    U = np.einsum("mzyx,kzyx->mk", D, u)
    return out, r + U, u, rho, F
