"""ctypes binding of the FP64 C oracle (test infrastructure only).

Every array crossing this boundary is float64 (or int32 for meshes), laid out
as the C side documents: lattice fields [component][z][y][x], marker arrays
[marker][xyz].
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None

GUO, SHAN_CHEN = 0, 1

_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    vp = C.c_void_p
    sig = {
        "orc_phi": (C.c_double, [C.c_int, C.c_double]),
        "orc_lattice": (None, [_I, _I, _I, _D]),
        "orc_icosphere": (C.c_int, [C.c_int, C.c_double, _D, _D, _I]),
        "orc_icosphere_counts": (C.c_int, [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
        "orc_membrane_eval": (None, [C.c_int, C.c_int, _I, _D, _D, C.c_double, C.c_double,
                                     C.c_double, C.c_double, _D, _D]),
        "orc_spread": (None, [C.c_int] * 5 + [_D, _D, _D]),
        "orc_interp": (None, [C.c_int] * 5 + [_D, _D, _D]),
        "orc_new": (vp, [C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int]),
        "orc_free": (None, [vp]),
        "orc_set_walls_y": (None, [vp, C.c_int]),
        "orc_set_body_force": (None, [vp, _D]),
        "orc_set_threads": (None, [C.c_int]),
        "orc_get_threads": (C.c_int, []),
        "orc_set_deviation": (None, [vp, _D]),
        "orc_get_pops": (None, [vp, _D]),
        "orc_add_swimmer": (C.c_int, [vp, _D, _D, C.c_int, C.c_double, C.c_double, C.c_double,
                                      C.c_double, _D, _D, C.c_double, C.c_double, C.c_double,
                                      C.c_double, C.c_double]),
        "orc_add_points": (C.c_int, [vp, C.c_int, _D, _D]),
        "orc_add_bead": (C.c_int, [vp, _D, C.c_double, C.c_int, C.c_double, C.c_double,
                                   C.c_double, C.c_double, _D]),
        "orc_step": (None, [vp, C.c_long]),
        "orc_time": (C.c_long, [vp]),
        "orc_n_markers": (C.c_int, [vp]),
        "orc_n_beads": (C.c_int, [vp]),
        "orc_n_swimmers": (C.c_int, [vp]),
        "orc_get_markers": (None, [vp, _D]),
        "orc_get_marker_forces": (None, [vp, _D]),
        "orc_get_marker_velocities": (None, [vp, _D]),
        "orc_get_bead_centres": (None, [vp, _D]),
        "orc_get_swimmer_centres": (None, [vp, _D]),
        "orc_get_velocity": (None, [vp, _D]),
        "orc_get_density": (None, [vp, _D]),
        "orc_get_force": (None, [vp, _D]),
        "orc_conserved": (None, [vp, _D]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def phi(width, r):
    """1-D discrete delta kernel of the given support width (2, 3 or 4)."""
    lib = _load()
    return lib.orc_phi(int(width), float(r))


def lattice():
    """D3Q19 velocities (19x3 int) and weights (19 float64)."""
    lib = _load()
    cx, cy, cz = (np.zeros(19, np.int32) for _ in range(3))
    w = np.zeros(19)
    lib.orc_lattice(cx, cy, cz, w)
    return np.stack([cx, cy, cz], axis=1), w


def icosphere(level, radius=1.0, centre=(0.0, 0.0, 0.0)):
    lib = _load()
    nv, nt = C.c_int(), C.c_int()
    lib.orc_icosphere_counts(int(level), C.byref(nv), C.byref(nt))
    v = np.zeros((nv.value, 3))
    t = np.zeros((nt.value, 3), np.int32)
    lib.orc_icosphere(int(level), float(radius), _d(centre), v, t)
    return v, t


def membrane_eval(tris, xref, x, ks, C_, kb, kv):
    """Return (energies[3] = Skalak, bending, volume, forces[nv,3])."""
    lib = _load()
    tris = np.ascontiguousarray(tris, np.int32)
    xref, x = _d(xref), _d(x)
    e = np.zeros(3)
    f = np.zeros_like(x)
    lib.orc_membrane_eval(x.shape[0], tris.shape[0], tris, xref, x, ks, C_, kb, kv, e, f)
    return e, f


def spread(shape, width, r, f):
    nx, ny, nz = shape
    lib = _load()
    r, f = _d(r), _d(f)
    F = np.zeros((3, nz, ny, nx))
    lib.orc_spread(nx, ny, nz, int(width), r.shape[0], r, f, F)
    return F


def interp(shape, width, r, u):
    nx, ny, nz = shape
    lib = _load()
    r, u = _d(r), _d(u)
    U = np.zeros_like(r)
    lib.orc_interp(nx, ny, nz, int(width), r.shape[0], r, u, U)
    return U


def set_threads(n):
    _load().orc_set_threads(int(n))


class Oracle:
    """One periodic D3Q19 box with optional swimmers, stepped in FP64."""

    def __init__(self, shape, tau, forcing=GUO, width=3):
        self.lib = _load()
        self.shape = tuple(int(s) for s in shape)
        nx, ny, nz = self.shape
        self.N = nx * ny * nz
        self.h = self.lib.orc_new(nx, ny, nz, float(tau), int(forcing), int(width))
        if not self.h:
            raise RuntimeError("orc_new failed")

    def close(self):
        if self.h:
            self.lib.orc_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _fshape(self, c):
        nx, ny, nz = self.shape
        return (c, nz, ny, nx)

    def set_walls_y(self, on=True):
        self.lib.orc_set_walls_y(self.h, int(on))

    def set_body_force(self, g):
        self.lib.orc_set_body_force(self.h, _d(g))

    def set_deviation(self, dev):
        dev = _d(dev).reshape(self._fshape(19))
        self.lib.orc_set_deviation(self.h, dev)

    def pops(self):
        f = np.zeros(self._fshape(19))
        self.lib.orc_get_pops(self.h, f)
        return f

    def add_swimmer(self, centres, radius, level, ks, C_, kb, kv, k, L0, A, B, T, alpha,
                    phi0=0.0):
        radius = np.broadcast_to(np.asarray(radius, float), (3,))
        k = np.broadcast_to(np.asarray(k, float), (2,))
        L0 = np.broadcast_to(np.asarray(L0, float), (2,))
        return self.lib.orc_add_swimmer(self.h, _d(centres).reshape(9), _d(radius), int(level),
                                        ks, C_, kb, kv, _d(k), _d(L0), A, B, T, alpha, phi0)

    def add_bead(self, centre, radius, level, ks, C_, kb, kv, force):
        return self.lib.orc_add_bead(self.h, _d(centre), float(radius), int(level), ks, C_, kb,
                                     kv, _d(force))

    def add_swimmer_desc(self, sw):
        """Add a swimmer described by a ``workloads.swimmer`` dict."""
        return self.add_swimmer(sw["centres"], sw["radius"], sw["level"], sw["ks"], sw["C"],
                                sw["kb"], sw["kv"], sw["k"], sw["L0"], sw["A"], sw["B"],
                                sw["T"], sw["alpha"], sw["phi0"])

    def add_points(self, r, f):
        r, f = _d(r).reshape(-1, 3), _d(f).reshape(-1, 3)
        self.lib.orc_add_points(self.h, r.shape[0], r, f)

    def step(self, n=1):
        self.lib.orc_step(self.h, int(n))

    @property
    def time(self):
        return self.lib.orc_time(self.h)

    @property
    def n_markers(self):
        return self.lib.orc_n_markers(self.h)

    @property
    def n_beads(self):
        return self.lib.orc_n_beads(self.h)

    @property
    def n_swimmers(self):
        return self.lib.orc_n_swimmers(self.h)

    def markers(self):
        r = np.zeros((self.n_markers, 3))
        self.lib.orc_get_markers(self.h, r)
        return r

    def marker_forces(self):
        f = np.zeros((self.n_markers, 3))
        self.lib.orc_get_marker_forces(self.h, f)
        return f

    def marker_velocities(self):
        U = np.zeros((self.n_markers, 3))
        self.lib.orc_get_marker_velocities(self.h, U)
        return U

    def bead_centres(self):
        R = np.zeros((self.n_beads, 3))
        self.lib.orc_get_bead_centres(self.h, R)
        return R

    def swimmer_centres(self):
        X = np.zeros((self.n_swimmers, 3))
        self.lib.orc_get_swimmer_centres(self.h, X)
        return X

    def velocity(self):
        u = np.zeros(self._fshape(3))
        self.lib.orc_get_velocity(self.h, u)
        return u

    def average_velocity(self, steps, every=1):
        """Time-averaged fluid velocity, as in the period-averaged flow fields
        of the paper's results (Sec. 3, Figs. 3, 6 and 9, one swimming period):
        advance `steps` steps and return the mean, over the sampled steps, of
        the physical velocity u = (sum f c + F/2) / rho each of them computes
        (Sec. 2.1), with the number of samples.  The first of the steps is
        sampled and then every `every`-th one."""
        acc = np.zeros(self._fshape(3))
        count = 0
        for k in range(int(steps)):
            self.step(1)
            if k % int(every) == 0:
                acc += self.velocity()
                count += 1
        return (acc / count if count else acc), count

    def density(self):
        nx, ny, nz = self.shape
        r = np.zeros((nz, ny, nx))
        self.lib.orc_get_density(self.h, r)
        return r

    def force(self):
        F = np.zeros(self._fshape(3))
        self.lib.orc_get_force(self.h, F)
        return F

    def conserved(self):
        out = np.zeros(4)
        self.lib.orc_conserved(self.h, out)
        return out
