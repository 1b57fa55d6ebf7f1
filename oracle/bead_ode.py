"""The paper's analytical comparison model (Sec. 2.4; Sec. 4, Eq. fit-eq):
point-like beads in unbounded Stokes flow.  Test infrastructure only (CPU,
numpy, float64): a physics-level comparator for the swimming speeds of the
lattice runs, not an oracle of the GPU path and not used by it.

Bead i moves with its own Stokes mobility times the force on it plus the flow
that the forces on the other beads induce at its position (Eq. EOM):

    dR_i/dt = f_i / (6 pi mu a) + sum_{j != i} T(R_i - R_j) . f_j

with T the Oseen tensor, (1 + r r / r^2) / (8 pi mu |r|), or the Rotne-Prager
tensor, which adds a^2 / (12 pi mu |r|^3) (1 - 3 r r / r^2) (Eqs. Oseen and
Rotne-Prager).  With a delay tau_d (Eq. fit-eq) the sum uses the other beads'
positions and forces at t - tau_d; before t = tau_d the initial state stands
in for the past.  The forces are the lattice model's (Sec. 2.2): driving
forces f1 = A sin(w t + phi0) x, f3 = B sin(w t + phi0 + alpha) x,
f2 = -(f1 + f3), and harmonic springs k (|d| - L0) d / |d| between each outer
bead and the middle one.  Time integration: classical fourth-order
Runge-Kutta with a fixed step; the delayed history is kept at every step and
interpolated linearly at the half steps.

Far-field limit used to pin the model (derived here for collinear beads,
a << L, small arm changes u_1 = L_1 - L, u_2 = L_2 - L): with the zeroth-order
forces that produce given arm rates and the first-order Oseen interactions,
the mean velocity of the three beads over a period is

    V = 7 a / (24 L^2) < u_1 du_2/dt - u_2 du_1/dt >,

the Golestanian-Ajdari result for the three-sphere swimmer; the mirror
symmetric stroke (B = -A, alpha = 0) does not move the centre at all.
"""
import math

import numpy as np


def oseen(r, mu):
    """Oseen tensors of separations r[..., 3]."""
    d = np.linalg.norm(r, axis=-1)[..., None, None]
    rr = r[..., :, None] * r[..., None, :] / d ** 2
    return (np.eye(3) + rr) / (8.0 * math.pi * mu * d)


def rotne_prager(r, mu, a):
    """Rotne-Prager tensors of separations r[..., 3] between beads of radius a."""
    d = np.linalg.norm(r, axis=-1)[..., None, None]
    rr = r[..., :, None] * r[..., None, :] / d ** 2
    return (np.eye(3) + rr) / (8.0 * math.pi * mu * d) + a ** 2 / (12.0 * math.pi * mu * d ** 3) * (np.eye(3) - 3.0 * rr)


class BeadSwimmers:
    """Three-bead swimmers (each a dict as made by workloads.swimmer: bead
    centres, radius, rest lengths L0, spring constants k, A, B, period T,
    alpha, phi0) in a fluid of dynamic viscosity mu."""

    def __init__(self, swimmers, mu, tensor="rotne_prager", delay=0.0):
        assert tensor in ("oseen", "rotne_prager")
        self.mu, self.tensor, self.delay = float(mu), tensor, float(delay)
        self.sw = swimmers
        self.R = np.concatenate([np.asarray(s["centres"], float) for s in swimmers])
        self.a = np.concatenate([np.broadcast_to(np.asarray(s["radius"], float), (3,)) for s in swimmers])
        # equal radii within a swimmer (the paper's beads); the tensor uses the
        # radius of the bead the flow acts on
        self.t = 0.0

    def forces(self, R, t):
        f = np.zeros_like(R)
        for s_i, s in enumerate(self.sw):
            b = 3 * s_i
            w = 2.0 * math.pi / s["T"]
            f1 = s["A"] * math.sin(w * t + s["phi0"])
            f3 = s["B"] * math.sin(w * t + s["phi0"] + s["alpha"])
            f[b, 0] += f1
            f[b + 2, 0] += f3
            f[b + 1, 0] -= f1 + f3
            for sp, outer in ((0, 0), (1, 2)):
                d = R[b + outer] - R[b + 1]
                ln = np.linalg.norm(d)
                fs = -s["k"][sp] * (ln - s["L0"][sp]) * d / ln
                f[b + outer] += fs
                f[b + 1] -= fs
        return f

    def _tensors(self, Ri, Rj):
        r = Ri[:, None, :] - Rj[None, :, :]
        n = len(Ri)
        r[np.arange(n), np.arange(n)] = 1.0  # placeholder on the diagonal, zeroed below
        if self.tensor == "oseen":
            T = oseen(r, self.mu)
        else:
            # radius of the bead the flow acts on (row i), one per tensor
            T = rotne_prager(r, self.mu, self.a[:, None, None, None])
        T[np.arange(n), np.arange(n)] = 0.0
        return T

    def velocity(self, R, t, Rd=None, fd=None):
        """Bead velocities at state R, time t; Rd, fd: the delayed positions
        and forces for the interaction sum (None: no delay)."""
        f = self.forces(R, t)
        own = f / (6.0 * math.pi * self.mu * self.a[:, None])
        if Rd is None:
            T = self._tensors(R, R)
            return own + np.einsum("ijab,jb->ia", T, f)
        T = self._tensors(R, Rd)
        return own + np.einsum("ijab,jb->ia", T, fd)

    def run(self, steps, dt=1.0, every=None, beads=False):
        """Advance `steps` steps of size dt; returns the swimmer centres
        [k, n_swimmers, 3] sampled every `every` steps (default: the end), or
        with beads=True the bead positions [k, n_beads, 3]."""
        every = every or steps
        ns = len(self.sw)
        out = []
        nd = int(round(self.delay / dt)) if self.delay > 0 else 0
        hist_R = [self.R.copy()]
        hist_f = [self.forces(self.R, self.t)]

        def delayed(tq):
            # positions and forces at tq - delay, linear between stored steps
            s = (tq - self.delay - self.t0) / dt
            if s <= 0:
                return hist_R[0], hist_f[0]
            i = int(math.floor(s))
            if i + 1 >= len(hist_R):
                return hist_R[-1], hist_f[-1]
            w = s - i
            return (1 - w) * hist_R[i] + w * hist_R[i + 1], (1 - w) * hist_f[i] + w * hist_f[i + 1]

        self.t0 = self.t
        for n in range(steps):
            t, R = self.t, self.R
            if nd:
                k1 = self.velocity(R, t, *delayed(t))
                k2 = self.velocity(R + 0.5 * dt * k1, t + 0.5 * dt, *delayed(t + 0.5 * dt))
                k3 = self.velocity(R + 0.5 * dt * k2, t + 0.5 * dt, *delayed(t + 0.5 * dt))
                k4 = self.velocity(R + dt * k3, t + dt, *delayed(t + dt))
            else:
                k1 = self.velocity(R, t)
                k2 = self.velocity(R + 0.5 * dt * k1, t + 0.5 * dt)
                k3 = self.velocity(R + 0.5 * dt * k2, t + 0.5 * dt)
                k4 = self.velocity(R + dt * k3, t + dt)
            self.R = R + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
            self.t = t + dt
            if nd:
                hist_R.append(self.R.copy())
                hist_f.append(self.forces(self.R, self.t))
            if (n + 1) % every == 0:
                out.append(self.R.copy() if beads else self.R.reshape(ns, 3, 3).mean(1))
        return np.array(out)

    def centres(self):
        return self.R.reshape(len(self.sw), 3, 3).mean(1)


def period_velocity(model, period, periods, dt=1.0):
    """x velocity of each swimmer's centre over each of `periods` periods
    (Eq. vel_swim: displacement over one period / period)."""
    steps = int(round(period / dt))
    X = [model.centres()]
    for _ in range(periods):
        X.append(model.run(steps, dt)[-1])
    X = np.array(X)
    return (X[1:, :, 0] - X[:-1, :, 0]) / period


def relative_changes(pair, single, mu, tensor="rotne_prager", delay=0.0, period=2e4, periods=4, dt=4.0):
    """v_Delta = (v - v_ref) / v_ref (Eq. inc) of each swimmer of `pair`
    against the lone swimmer `single`, both over the last of `periods`
    periods, in the same model."""
    v_ref = period_velocity(BeadSwimmers(single, mu, tensor, delay), period, periods, dt)[-1, 0]
    v = period_velocity(BeadSwimmers(pair, mu, tensor, delay), period, periods, dt)[-1]
    return v_ref, (v - v_ref) / v_ref


if __name__ == "__main__":
    # the paper-box runs' swimmers (Sec. 3) in the point-bead model, mu = 1/6
    from paper_2202_12147_amd import workloads as wl

    single = wl.paper_run()["swimmers"]
    for arrangement, d in (("collinear", 144.0), ("side", 72.0)):
        pair = wl.paper_run(arrangement, d)["swimmers"]
        for tensor in ("oseen", "rotne_prager"):
            for delay in ((0.0, 250.0, 500.0, 1000.0) if arrangement == "collinear" else (0.0,)):
                v_ref, vd = relative_changes(pair, single, 1.0 / 6.0, tensor, delay)
                print(f"{arrangement:9s} d={d:5.0f} {tensor:12s} delay {delay:6.0f}: v_ref {v_ref:.4e}, "
                      f"v_Delta {' '.join(f'{x:+.4f}' for x in vd)}", flush=True)
