"""FP64 gradient oracle for a swimmer's displacement (test infrastructure only).

An independent, plain PyTorch (CPU, float64) implementation of the forward
step -- the same method and reading as the C oracle (see orc_sim.c): bead
centres, driving and spring forces (Sec. 2.2), Skalak / Kantor-Nelson /
volume membrane forces (Sec. 2.2), spreading (Eq. spreading), periodic
streaming and BGK collision with Guo or Shan-Chen forcing (Eqs. lbe,
lbm:equilibrium, sc; the physical velocity (j + F/2)/rho in both),
interpolation (Eq. interpolation) and forward-Euler advection -- written
as differentiable tensor expressions.  The gradient of

    J = x-displacement of the mean of all the swimmer's mesh nodes over T steps

with respect to theta = (A, B, alpha, k) (driving amplitudes of the outer
beads, their phase shift, the common spring constant) is reverse-mode
automatic differentiation of that forward model, with the step sequence
checkpointed every K steps and recomputed.  Pinned against the C oracle's
forward trajectory and against central finite differences of the C oracle's
J (tests/test_oracle_adjoint.py).

TEST INFRASTRUCTURE ONLY; the product never imports it.
"""
import ctypes
import math

import numpy as np
import torch
from torch.utils.checkpoint import checkpoint

from . import orc

DT = torch.float64


def _large_blocks_from_mmap():
    """Serve allocations of 1 MiB and more straight from mmap.  The step's
    many short-lived tensor temporaries otherwise fragment the glibc heap
    until a checkpointed 2000-step gradient holds tens of GB."""
    try:
        libc = ctypes.CDLL("libc.so.6")
        libc.mallopt(-3, 1 << 20)  # M_MMAP_THRESHOLD
    except OSError:
        pass


_large_blocks_from_mmap()


def _phi(width, r):
    """Delta kernels of Sec. 2.3.  Each branch is evaluated on a stand-in
    distance where it is not selected, so that no square root of a negative
    or zero argument enters the backward pass."""
    r = r.abs()
    zero = torch.zeros_like(r)
    if width == 2:
        return torch.clamp(1.0 - r, min=0.0)
    if width == 3:
        ri = torch.where(r <= 0.5, r, zero)
        ro = torch.where((r > 0.5) & (r <= 1.5), r, zero + 1.0)
        inner = (1.0 + torch.sqrt(1.0 - 3.0 * ri * ri)) / 3.0
        outer = (5.0 - 3.0 * ro - torch.sqrt(1.0 - 3.0 * (1.0 - ro) ** 2)) / 6.0
        return torch.where(r <= 0.5, inner, torch.where(r <= 1.5, outer, zero))
    ri = torch.where(r <= 1.0, r, zero)
    ro = torch.where((r > 1.0) & (r <= 2.0), r, zero + 1.5)
    inner = (3.0 - 2.0 * ri + torch.sqrt(1.0 + 4.0 * ri - 4.0 * ri * ri)) / 8.0
    outer = (5.0 - 2.0 * ro - torch.sqrt(-7.0 + 12.0 * ro - 4.0 * ro * ro)) / 8.0
    return torch.where(r <= 1.0, inner, torch.where(r <= 2.0, outer, zero))


def _dihedral(x1, x2, x3, x4):
    e = x2 - x1
    nA = torch.cross(e, x3 - x1, dim=-1)
    nB = torch.cross(x1 - x2, x4 - x2, dim=-1)
    E = torch.linalg.norm(e, dim=-1, keepdim=True)
    nAh = nA / torch.linalg.norm(nA, dim=-1, keepdim=True)
    nBh = nB / torch.linalg.norm(nB, dim=-1, keepdim=True)
    return torch.atan2((torch.cross(nAh, nBh, dim=-1) * (e / E)).sum(-1), (nAh * nBh).sum(-1))


class SwimmerModel:
    """One periodic box with one swimmer, stepped by differentiable torch ops."""

    def __init__(self, case):
        self.shape = tuple(case["shape"])
        nx, ny, nz = self.shape
        self.N = nx * ny * nz
        self.tau = float(case["tau"])
        self.forcing = int(case["forcing"])
        assert self.forcing in (0, 1), "Guo (0) or Shan-Chen (1) forcing"
        self.width = int(case["width"])
        sw = case["swimmers"][0]
        self.sw = sw
        c, w = orc.lattice()
        self.c = [tuple(int(v) for v in ci) for ci in c]
        self.cd = torch.tensor(c, dtype=DT)
        self.w = torch.tensor(w, dtype=DT)
        verts, tris, hinges, th0, first = [], [], [], [], []
        off = 0
        for b in range(3):
            v, t = orc.icosphere(sw["level"], sw["radius"][b], sw["centres"][b])
            first.append(off)
            verts.append(v)
            tris.append(t + off)
            h = self._hinges(t) + off
            hinges.append(h)
            off += len(v)
        self.nv = len(verts[0])
        self.first = first
        x0 = torch.tensor(np.concatenate(verts), dtype=DT)
        self.r0 = x0
        self.tri = torch.tensor(np.concatenate(tris), dtype=torch.long)
        self.hinge = torch.tensor(np.concatenate(hinges), dtype=torch.long)
        t = self.tri
        E1 = x0[t[:, 1]] - x0[t[:, 0]]
        E2 = x0[t[:, 2]] - x0[t[:, 0]]
        G11, G12, G22 = (E1 * E1).sum(1), (E1 * E2).sum(1), (E2 * E2).sum(1)
        self.detG0 = G11 * G22 - G12 * G12
        self.Gi = torch.stack([G22, -G12, G11], 1) / self.detG0[:, None]
        self.A0 = 0.5 * torch.sqrt(self.detG0)
        h = self.hinge
        self.th0 = _dihedral(x0[h[:, 0]], x0[h[:, 1]], x0[h[:, 2]], x0[h[:, 3]])
        self.V0 = torch.stack([self._volume(x0, b) for b in range(3)])
        self.bead_of_tri = torch.repeat_interleave(torch.arange(3), len(tris[0]))
        self.bead_of_hinge = torch.repeat_interleave(torch.arange(3), len(hinges[0]))

    @staticmethod
    def _hinges(t):
        opp = {}
        for f in t:
            for q in range(3):
                opp[(int(f[q]), int(f[(q + 1) % 3]))] = int(f[(q + 2) % 3])
        out = []
        for f in t:
            for q in range(3):
                a, b, c = int(f[q]), int(f[(q + 1) % 3]), int(f[(q + 2) % 3])
                if a < b:
                    out.append((a, b, c, opp[(b, a)]))
        return np.array(out, dtype=np.int64)

    def _bead(self, b):
        return slice(self.first[b], self.first[b] + self.nv)

    def _volume(self, x, b):
        xb = x[self._bead(b)]
        cb = xb.mean(0)
        nt = len(self.tri) // 3
        t = self.tri[b * nt:(b + 1) * nt]
        a, bb, cc = x[t[:, 0]] - cb, x[t[:, 1]] - cb, x[t[:, 2]] - cb
        return (a * torch.cross(bb, cc, dim=1)).sum() / 6.0

    # ---- forces (Sec. 2.2) -------------------------------------------------
    def forces(self, r, n, theta):
        A, B, alpha, k = theta
        sw = self.sw
        ks, C, kb, kv = sw["ks"], sw["C"], sw["kb"], sw["kv"]
        f = torch.zeros_like(r)
        t = self.tri
        e1 = r[t[:, 1]] - r[t[:, 0]]
        e2 = r[t[:, 2]] - r[t[:, 0]]
        g11, g12, g22 = (e1 * e1).sum(1), (e1 * e2).sum(1), (e2 * e2).sum(1)
        Gi = self.Gi
        I1 = Gi[:, 0] * g11 + 2.0 * Gi[:, 1] * g12 + Gi[:, 2] * g22 - 2.0
        I2 = (g11 * g22 - g12 * g12) / self.detG0 - 1.0
        dW1 = ks / 4.0 * self.A0 * (2.0 * I1 + 2.0)
        dW2 = ks / 4.0 * self.A0 * (-2.0 + 2.0 * C * I2)
        P11 = dW1 * Gi[:, 0] + dW2 * g22 / self.detG0
        P12 = dW1 * Gi[:, 1] - dW2 * g12 / self.detG0
        P22 = dW1 * Gi[:, 2] + dW2 * g11 / self.detG0
        dWde1 = 2.0 * (P11[:, None] * e1 + P12[:, None] * e2)
        dWde2 = 2.0 * (P12[:, None] * e1 + P22[:, None] * e2)
        f = f.index_add(0, t[:, 1], -dWde1).index_add(0, t[:, 2], -dWde2)
        f = f.index_add(0, t[:, 0], dWde1 + dWde2)
        # bending
        h = self.hinge
        x1, x2, x3, x4 = r[h[:, 0]], r[h[:, 1]], r[h[:, 2]], r[h[:, 3]]
        th = _dihedral(x1, x2, x3, x4)
        dWdth = 2.0 * kb / math.sqrt(3.0) * torch.sin(th - self.th0)
        e = x2 - x1
        nA = torch.cross(e, x3 - x1, dim=1)
        nB = torch.cross(x1 - x2, x4 - x2, dim=1)
        E = torch.linalg.norm(e, dim=1, keepdim=True)
        eh = e / E
        a = nA / (nA * nA).sum(1, keepdim=True)
        bq = nB / (nB * nB).sum(1, keepdim=True)
        g1 = -((x3 - x2) * eh).sum(1, keepdim=True) * a + ((x2 - x4) * eh).sum(1, keepdim=True) * bq
        g2 = -((x1 - x3) * eh).sum(1, keepdim=True) * a + ((x4 - x1) * eh).sum(1, keepdim=True) * bq
        g3 = -E * a
        g4 = -E * bq
        dw = dWdth[:, None]
        f = f.index_add(0, h[:, 0], -dw * g1).index_add(0, h[:, 1], -dw * g2)
        f = f.index_add(0, h[:, 2], -dw * g3).index_add(0, h[:, 3], -dw * g4)
        # volume, per bead
        nt = len(t) // 3
        R = []
        for b in range(3):
            sl = self._bead(b)
            cb = r[sl].mean(0)
            R.append(cb)
            tb = t[b * nt:(b + 1) * nt]
            p0, p1, p2 = r[tb[:, 0]] - cb, r[tb[:, 1]] - cb, r[tb[:, 2]] - cb
            V = (p0 * torch.cross(p1, p2, dim=1)).sum() / 6.0
            pref = kv * (V - self.V0[b]) / self.V0[b]
            f = f.index_add(0, tb[:, 0], -pref * torch.cross(p1, p2, dim=1) / 6.0)
            f = f.index_add(0, tb[:, 1], -pref * torch.cross(p2, p0, dim=1) / 6.0)
            f = f.index_add(0, tb[:, 2], -pref * torch.cross(p0, p1, dim=1) / 6.0)
        # driving and springs, shared equally by a bead's nodes
        om = 2.0 * math.pi / sw["T"]
        f1 = A * math.sin(om * n + sw["phi0"])
        f3 = B * torch.sin(om * n + sw["phi0"] + alpha)
        ex = torch.tensor([1.0, 0.0, 0.0], dtype=DT)
        fb = [f1 * ex, (-f1 - f3) * ex, f3 * ex]
        for sp, outer in ((0, 0), (1, 2)):
            d = R[outer] - R[1]
            ln = torch.linalg.norm(d)
            fs = -k * (ln - sw["L0"][sp]) * d / ln
            fb[outer] = fb[outer] + fs
            fb[1] = fb[1] - fs
        share = torch.cat([fb[b].expand(self.nv, 3) for b in range(3)]) / self.nv
        return f + share

    # ---- immersed boundary (Sec. 2.3) ----------------------------------------
    def _window(self, r):
        nx, ny, nz = self.shape
        # nodes floor(r) - 1 ... floor(r) + 2 hold every nonzero weight of the
        # three kernels (support |x - r| < 2)
        base = torch.floor(r.detach()).long() - 1
        o = torch.arange(4)
        ix = base[:, 0:1] + o
        iy = base[:, 1:2] + o
        iz = base[:, 2:3] + o
        wx = _phi(self.width, ix.to(DT) - r[:, 0:1])
        wy = _phi(self.width, iy.to(DT) - r[:, 1:2])
        wz = _phi(self.width, iz.to(DT) - r[:, 2:3])
        w = wz[:, :, None, None] * wy[:, None, :, None] * wx[:, None, None, :]
        idx = ((iz % nz)[:, :, None, None] * ny + (iy % ny)[:, None, :, None]) * nx + (ix % nx)[:, None, None, :]
        return w.reshape(len(r), -1), idx.reshape(len(r), -1)

    def spread(self, r, fm):
        w, idx = self._window(r)
        vals = w[:, :, None] * fm[:, None, :]
        F = torch.zeros(self.N, 3, dtype=DT).index_add(0, idx.reshape(-1), vals.reshape(-1, 3))
        return F

    def interp(self, r, u):
        w, idx = self._window(r)
        return (w[:, :, None] * u[idx]).sum(1)

    # ---- lattice Boltzmann (Sec. 2.1) ------------------------------------------
    def stream(self, f):
        return torch.stack([torch.roll(f[i], shifts=(c[2], c[1], c[0]), dims=(0, 1, 2))
                            for i, c in enumerate(self.c)])

    def step(self, f, r, n, theta):
        nx, ny, nz = self.shape
        F = self.spread(r, self.forces(r, n, theta))  # [N, 3]
        fs = self.stream(f).reshape(19, -1)
        rho = fs.sum(0)
        j = fs.t() @ self.cd  # [N, 3]
        u = (j + 0.5 * F) / rho[:, None]  # physical velocity, both forcings
        if self.forcing == 0:
            # Guo: the equilibrium at u plus the source term
            cu = u @ self.cd.t()  # [N, 19]
            uu = (u * u).sum(1, keepdim=True)
            feq = self.w * rho[:, None] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)
            cF = F @ self.cd.t()
            uF = (u * F).sum(1, keepdim=True)
            src = (1.0 - 0.5 / self.tau) * self.w * (3.0 * (cF - uF) + 9.0 * cu * cF)
            fo = fs.t() - (fs.t() - feq) / self.tau + src
        else:
            # Shan-Chen (Eq. sc): the equilibrium at (j + tau F)/rho, no source
            v = (j + self.tau * F) / rho[:, None]
            cv = v @ self.cd.t()
            vv = (v * v).sum(1, keepdim=True)
            feq = self.w * rho[:, None] * (1.0 + 3.0 * cv + 4.5 * cv * cv - 1.5 * vv)
            fo = fs.t() - (fs.t() - feq) / self.tau
        U = self.interp(r, u)
        return fo.t().reshape(19, nz, ny, nx), r + U

    def initial(self):
        nx, ny, nz = self.shape
        f = self.w[:, None, None, None].expand(19, nz, ny, nx).clone()
        return f, self.r0.clone()

    def run(self, theta, steps, checkpoint_every=0):
        """Advance from rest; return (J, final f, final r)."""
        f, r = self.initial()
        n = 0
        K = checkpoint_every if checkpoint_every > 0 else steps

        def segment(f, r, A, B, alpha, k, n0, m):
            th = (A, B, alpha, k)
            for i in range(m):
                f, r = self.step(f, r, float(n0 + i), th)
            return f, r

        while n < steps:
            m = min(K, steps - n)
            if checkpoint_every > 0:
                f, r = checkpoint(segment, f, r, *theta, n, m, use_reentrant=False)
            else:
                f, r = segment(f, r, *theta, n, m)
            n += m
        J = r[:, 0].mean() - self.r0[:, 0].mean()
        return J, f, r


def displacement_gradient(case, steps, checkpoint_every=100, theta=None):
    """J and dJ/d(A, B, alpha, k) for the first swimmer of `case`, FP64."""
    torch.set_num_threads(max(1, torch.get_num_threads()))
    model = SwimmerModel(case)
    sw = case["swimmers"][0]
    assert sw["k"][0] == sw["k"][1], "one spring constant shared by both springs"
    if theta is None:
        theta = (sw["A"], sw["B"], sw["alpha"], sw["k"][0])
    th = [torch.tensor(float(v), dtype=DT, requires_grad=True) for v in theta]
    J, _, _ = model.run(th, steps, checkpoint_every)
    J.backward()
    return float(J.detach()), np.array([float(t.grad) for t in th])
