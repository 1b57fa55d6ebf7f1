"""Thin Python binding of the lbmib C-ABI (include/lbmib.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch supplies device memory (for on-device outputs) and the stream.  The
binding refuses to run without the compiled library: there is no fallback.
"""
import ctypes as C
import math
import os
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmib.so")

GUO, SHAN_CHEN = 0, 1
FP32_SHIFTED, FP16_SHIFTED, FP32_PLAIN, FP32_INPLACE = 0, 1, 2, 3

ERRORS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE", -4: "LBM_ESTATE",
          -5: "LBM_ENONFINITE", -6: "LBM_EIO", -7: "LBM_EOVERFLOW"}

# every symbol the header declares (checked by the CPU tests)
SYMBOLS = [
    "lbm_create", "lbm_destroy", "lbm_swimmer_add", "lbm_set_body_force", "lbm_step", "lbm_sync",
    "lbm_time", "lbm_n_markers", "lbm_n_swimmers", "lbm_get_swimmer_centres",
    "lbm_get_bead_centres", "lbm_get_markers", "lbm_get_marker_velocities",
    "lbm_get_marker_forces", "lbm_get_velocity",
    "lbm_get_density", "lbm_get_conserved", "lbm_set_populations", "lbm_get_populations",
    "lbm_average_begin", "lbm_get_average_velocity",
    "lbm_save", "lbm_load", "lbm_set_kernel_timing", "lbm_kernel_time", "lbm_bytes_per_step",
    "lbm_probe_copy_bandwidth", "lbm_set_stream_collide_launch",
    "lbm_batch_create", "lbm_batch_swimmer_add", "lbm_n_boxes", "lbm_batch_step", "lbm_batch_get_velocity",
    "lbm_batch_get_conserved", "lbm_batch_get_conserved_noalloc", "lbm_autotune",
    "lbm_swimmer_set_params", "lbm_adjoint", "lbm_field_bytes",
    "lbm_strerror", "lbm_last_error",
]


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32)]


class Opts(C.Structure):
    _fields_ = [("storage", C.c_int32), ("delta_width", C.c_int32), ("fp16_scale", C.c_float),
                ("use_graphs", C.c_int32), ("stream", C.c_void_p), ("field_memory", C.c_void_p),
                ("field_bytes", C.c_int64)]


class BoxDesc(C.Structure):
    _fields_ = [("grid", Grid), ("tau", C.c_double), ("forcing", C.c_int32)]


class BeadDesc(C.Structure):
    _fields_ = [("centre", C.c_double * 3), ("radius", C.c_double), ("level", C.c_int32),
                ("kappa_s", C.c_double), ("C", C.c_double), ("kappa_b", C.c_double),
                ("kappa_v", C.c_double)]


class SpringDesc(C.Structure):
    _fields_ = [("k", C.c_double), ("L0", C.c_double)]


class ActuationDesc(C.Structure):
    _fields_ = [("A", C.c_double), ("B", C.c_double), ("period", C.c_double),
                ("alpha", C.c_double), ("phi0", C.c_double)]


class AdjointDesc(C.Structure):
    _fields_ = [("steps", C.c_int64), ("checkpoint", C.c_int32), ("swimmer", C.c_int32),
                ("rewind", C.c_int32)]


_lib = None


def load_library():
    """Load liblbmib.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    # torch owns the process's HIP runtime: load it first so that the
    # library's libamdhip64.so.7 dependency resolves to torch's copy instead
    # of mapping a second runtime next to it
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    runtimes = _hip_runtimes()
    if len(runtimes) > 1:
        raise RuntimeError(f"two HIP runtimes are mapped in this process: {sorted(runtimes)}")
    _lib = bind(lib)
    return _lib


def bind(lib):
    """Declare the C signatures of every entry point on a loaded library."""
    vp, i32, i64, dp, fp = C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p
    sig = {
        "lbm_create": (C.c_int, [C.POINTER(Grid), C.c_double, C.c_int, C.POINTER(Opts),
                                 C.POINTER(C.c_void_p)]),
        "lbm_destroy": (C.c_int, [vp]),
        "lbm_swimmer_add": (C.c_int, [vp, C.POINTER(BeadDesc), C.POINTER(SpringDesc),
                                      C.POINTER(ActuationDesc), C.POINTER(i32)]),
        "lbm_set_body_force": (C.c_int, [vp, dp]),
        "lbm_step": (C.c_int, [vp, i64]),
        "lbm_sync": (C.c_int, [vp]),
        "lbm_time": (i64, [vp]),
        "lbm_n_markers": (i32, [vp]),
        "lbm_n_swimmers": (i32, [vp]),
        "lbm_get_swimmer_centres": (C.c_int, [vp, dp]),
        "lbm_get_bead_centres": (C.c_int, [vp, dp]),
        "lbm_get_markers": (C.c_int, [vp, dp]),
        "lbm_get_marker_velocities": (C.c_int, [vp, dp]),
        "lbm_get_marker_forces": (C.c_int, [vp, dp]),
        "lbm_get_velocity": (C.c_int, [vp, fp, C.c_int]),
        "lbm_get_density": (C.c_int, [vp, fp, C.c_int]),
        "lbm_get_conserved": (C.c_int, [vp, dp]),
        "lbm_set_populations": (C.c_int, [vp, dp]),
        "lbm_get_populations": (C.c_int, [vp, dp]),
        "lbm_average_begin": (C.c_int, [vp, i32]),
        "lbm_get_average_velocity": (C.c_int, [vp, i32, fp, C.c_int, C.POINTER(i64)]),
        "lbm_save": (C.c_int, [vp, C.c_char_p]),
        "lbm_load": (C.c_int, [vp, C.c_char_p]),
        "lbm_set_kernel_timing": (C.c_int, [vp, C.c_int]),
        "lbm_kernel_time": (C.c_int, [vp, C.POINTER(C.c_double), C.POINTER(i64)]),
        "lbm_bytes_per_step": (i64, [vp]),
        "lbm_probe_copy_bandwidth": (C.c_int, [i64, C.c_int, C.POINTER(C.c_double)]),
        "lbm_set_stream_collide_launch": (C.c_int, [vp, C.c_int, C.c_int, C.c_int]),
        "lbm_batch_create": (C.c_int, [C.POINTER(BoxDesc), i32, C.POINTER(Opts), C.POINTER(C.c_void_p)]),
        "lbm_batch_swimmer_add": (C.c_int, [vp, i32, C.POINTER(BeadDesc), C.POINTER(SpringDesc),
                                            C.POINTER(ActuationDesc), C.POINTER(i32)]),
        "lbm_n_boxes": (i32, [vp]),
        "lbm_batch_step": (C.c_int, [vp, i64]),
        "lbm_batch_get_velocity": (C.c_int, [vp, i32, fp, C.c_int]),
        "lbm_batch_get_conserved": (C.c_int, [vp, i32, dp]),
        "lbm_batch_get_conserved_noalloc": (C.c_int, [vp, i32, i32, dp]),
        "lbm_autotune": (C.c_int, [vp, i32, C.c_char_p, C.c_char_p, i32]),
        "lbm_swimmer_set_params": (C.c_int, [vp, i32, C.c_double, C.c_double, C.c_double, C.c_double]),
        "lbm_adjoint": (C.c_int, [vp, C.POINTER(AdjointDesc), C.POINTER(C.c_double), dp]),
        "lbm_field_bytes": (C.c_int, [C.POINTER(BoxDesc), i32, i32, C.POINTER(i64)]),
        "lbm_strerror": (C.c_char_p, [C.c_int]),
        "lbm_last_error": (C.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def _hip_runtimes():
    """Distinct libamdhip64 files mapped into this process."""
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return paths


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _swimmer_descs(sw):
    beads = (BeadDesc * 3)()
    for k in range(3):
        beads[k].centre[:] = [float(v) for v in sw["centres"][k]]
        beads[k].radius = float(sw["radius"][k])
        beads[k].level = int(sw["level"])
        beads[k].kappa_s = float(sw["ks"])
        beads[k].C = float(sw["C"])
        beads[k].kappa_b = float(sw["kb"])
        beads[k].kappa_v = float(sw["kv"])
    springs = (SpringDesc * 2)(SpringDesc(float(sw["k"][0]), float(sw["L0"][0])),
                               SpringDesc(float(sw["k"][1]), float(sw["L0"][1])))
    act = ActuationDesc(float(sw["A"]), float(sw["B"]), float(sw["T"]), float(sw["alpha"]),
                        float(sw["phi0"]))
    return beads, springs, act


def field_bytes(boxes, storage=FP32_SHIFTED):
    """Bytes of caller field memory a handle over ``boxes`` (list of (shape,
    tau, forcing)) needs (lbm_field_bytes; host only)."""
    lib = load_library()
    arr = _box_array(boxes)
    out = C.c_int64()
    rc = lib.lbm_field_bytes(arr, len(boxes), int(storage), C.byref(out))
    if rc:
        raise LbmError(rc, lib.lbm_strerror(rc).decode())
    return out.value


def _box_array(boxes):
    arr = (BoxDesc * len(boxes))()
    for i, (shape, tau, forcing) in enumerate(boxes):
        arr[i].grid = Grid(*[int(v) for v in shape])
        arr[i].tau = float(tau)
        arr[i].forcing = int(forcing)
    return arr


def _field_memory(boxes, storage, field_memory):
    """(tensor or None, pointer, bytes) for Opts: None lets the library
    allocate; "torch" allocates a uint8 tensor of the needed size on the
    current device; a contiguous device tensor is used as given."""
    if field_memory is None:
        return None, None, 0
    import torch
    need = field_bytes(boxes, storage)
    if isinstance(field_memory, str):
        if field_memory != "torch":
            raise ValueError("field_memory: None, 'torch' or a device tensor")
        t = torch.empty(need, dtype=torch.uint8, device=torch.device("cuda", torch.cuda.current_device()))
    else:
        t = field_memory
        if not (t.is_cuda and t.is_contiguous()):
            raise ValueError("field_memory must be a contiguous device tensor")
    return t, t.data_ptr(), t.numel() * t.element_size()


class Lattice:
    """One periodic D3Q19 box with swimmers, stepped by the HIP library.

    ``stream``: a ``torch.cuda.Stream`` (or raw hipStream_t int) to enqueue on;
    None lets the library create its own.  ``field_memory``: None (the
    library allocates the node fields), "torch" (a tensor allocated here) or
    a contiguous device tensor of at least ``field_bytes`` bytes; the handle
    keeps a reference for its lifetime (``self.field_tensor``)."""

    def __init__(self, shape, tau, forcing=GUO, storage=FP32_SHIFTED, width=3, fp16_scale=1.0,
                 use_graphs=True, stream=None, field_memory=None):
        self.lib = load_library()
        self.shape = tuple(int(s) for s in shape)
        self.storage = storage
        raw = None
        if stream is not None:
            raw = getattr(stream, "cuda_stream", stream)
            raw = int(raw) or None
        self.field_tensor, fptr, fbytes = _field_memory([(self.shape, tau, forcing)], storage, field_memory)
        g = Grid(*self.shape)
        o = Opts(int(storage), int(width), float(fp16_scale), int(bool(use_graphs)), raw, fptr, fbytes)
        h = C.c_void_p()
        rc = self.lib.lbm_create(C.byref(g), float(tau), int(forcing), C.byref(o), C.byref(h))
        if rc:
            raise LbmError(rc, self.lib.lbm_strerror(rc).decode())
        self.h = h

    # -- helpers
    def _check(self, rc):
        if rc:
            raise LbmError(rc, self.lib.lbm_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.lbm_destroy(self.h)  # waits for the handle's stream
            self.h = None
        self.field_tensor = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def N(self):
        nx, ny, nz = self.shape
        return nx * ny * nz

    # -- setup
    def add_swimmer(self, sw):
        """Add a swimmer described by a ``workloads.swimmer`` dict."""
        beads, springs, act = _swimmer_descs(sw)
        sid = C.c_int32()
        self._check(self.lib.lbm_swimmer_add(self.h, beads, springs, C.byref(act), C.byref(sid)))
        return sid.value

    def set_body_force(self, g):
        g = np.ascontiguousarray(g, np.float64)
        self._check(self.lib.lbm_set_body_force(self.h, _ptr(g)))

    def set_populations(self, dev):
        dev = np.ascontiguousarray(dev, np.float64)
        assert dev.size == 19 * self.N
        self._check(self.lib.lbm_set_populations(self.h, _ptr(dev)))

    # -- stepping
    def step(self, n=1):
        self._check(self.lib.lbm_step(self.h, int(n)))

    def sync(self):
        self._check(self.lib.lbm_sync(self.h))

    @property
    def time(self):
        return self.lib.lbm_time(self.h)

    @property
    def n_markers(self):
        return self.lib.lbm_n_markers(self.h)

    @property
    def n_swimmers(self):
        return self.lib.lbm_n_swimmers(self.h)

    # -- observables
    def swimmer_centres(self):
        out = np.zeros((self.n_swimmers, 3))
        self._check(self.lib.lbm_get_swimmer_centres(self.h, _ptr(out)))
        return out

    def bead_centres(self):
        out = np.zeros((3 * self.n_swimmers, 3))
        self._check(self.lib.lbm_get_bead_centres(self.h, _ptr(out)))
        return out

    def markers(self):
        out = np.zeros((self.n_markers, 3))
        self._check(self.lib.lbm_get_markers(self.h, _ptr(out)))
        return out

    def marker_velocities(self):
        out = np.zeros((self.n_markers, 3))
        self._check(self.lib.lbm_get_marker_velocities(self.h, _ptr(out)))
        return out

    def marker_forces(self):
        out = np.zeros((self.n_markers, 3))
        self._check(self.lib.lbm_get_marker_forces(self.h, _ptr(out)))
        return out

    def velocity(self, device=None):
        """u of the last step, [3, nz, ny, nx] float32: numpy on the host, or a
        torch tensor on ``device`` (e.g. "cuda:0")."""
        nx, ny, nz = self.shape
        if device is not None:
            import torch
            t = torch.empty((3, nz, ny, nx), dtype=torch.float32, device=device)
            self._check(self.lib.lbm_get_velocity(self.h, C.c_void_p(t.data_ptr()), 1))
            return t
        out = np.zeros((3, nz, ny, nx), np.float32)
        self._check(self.lib.lbm_get_velocity(self.h, _ptr(out), 0))
        return out

    def average_begin(self, every=1):
        """Start a new time average of u over this step and every `every`-th
        step after it (every = 0 stops it)."""
        self._check(self.lib.lbm_average_begin(self.h, int(every)))

    def average_velocity(self, box=0, device=None):
        """(mean u of the sampled steps [3, nz, ny, nx] float32, sample
        count): numpy on the host, or a torch tensor on ``device``."""
        nx, ny, nz = self._box_shape(box)
        count = C.c_int64()
        if device is not None:
            import torch
            t = torch.empty((3, nz, ny, nx), dtype=torch.float32, device=device)
            self._check(self.lib.lbm_get_average_velocity(self.h, int(box), C.c_void_p(t.data_ptr()), 1,
                                                          C.byref(count)))
            return t, count.value
        out = np.zeros((3, nz, ny, nx), np.float32)
        self._check(self.lib.lbm_get_average_velocity(self.h, int(box), _ptr(out), 0, C.byref(count)))
        return out, count.value

    def _box_shape(self, box):
        if box != 0:
            raise ValueError("a single-box handle has box 0 only")
        return self.shape

    def density(self):
        nx, ny, nz = self.shape
        out = np.zeros((nz, ny, nx), np.float32)
        self._check(self.lib.lbm_get_density(self.h, _ptr(out), 0))
        return out

    def conserved(self):
        out = np.zeros(4)
        self._check(self.lib.lbm_get_conserved(self.h, _ptr(out)))
        return out

    def conserved_noalloc(self, dst, box=-1, parts=1024):
        """Enqueue the conserved sums into ``dst`` (a float64 device tensor
        of at least 4 elements) without allocating or synchronising."""
        assert dst.dtype.itemsize == 8 and dst.numel() >= 4 and dst.is_cuda
        self._check(self.lib.lbm_batch_get_conserved_noalloc(self.h, int(box), int(parts),
                                                             C.c_void_p(dst.data_ptr())))

    def populations(self):
        nx, ny, nz = self.shape
        out = np.zeros((19, nz, ny, nx))
        self._check(self.lib.lbm_get_populations(self.h, _ptr(out)))
        return out

    def save(self, path):
        self._check(self.lib.lbm_save(self.h, str(path).encode()))

    def load(self, path):
        self._check(self.lib.lbm_load(self.h, str(path).encode()))

    # -- measurement
    def set_kernel_timing(self, on):
        self._check(self.lib.lbm_set_kernel_timing(self.h, int(bool(on))))

    def kernel_time(self):
        ms, n = C.c_double(), C.c_int64()
        self._check(self.lib.lbm_kernel_time(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def set_stream_collide_launch(self, block=256, xcd_remap=True, resident=0):
        self._check(self.lib.lbm_set_stream_collide_launch(self.h, int(block), int(bool(xcd_remap)),
                                                           int(resident)))

    def autotune(self, steps_per_candidate=64, cache_path=None):
        """The launch-shape tuner of the library, which is disabled: raises
        LbmError (LBM_ESTATE)."""
        buf = C.create_string_buffer(4096)
        cp = None if cache_path is None else str(cache_path).encode()
        self._check(self.lib.lbm_autotune(self.h, int(steps_per_candidate), cp, buf, 4096))
        return buf.value.decode()

    @property
    def bytes_per_step(self):
        return self.lib.lbm_bytes_per_step(self.h)

    def set_swimmer_params(self, swimmer, A, B, alpha, k):
        """Driving amplitudes, phase shift and spring constant (both springs)."""
        self._check(self.lib.lbm_swimmer_set_params(self.h, int(swimmer), float(A), float(B),
                                                    float(alpha), float(k)))

    def adjoint(self, steps, checkpoint=100, swimmer=0, rewind=False):
        """J = x displacement of the swimmer's centre over `steps` steps and
        dJ/d(A, B, alpha, k) from the hand-written discrete adjoint."""
        desc = AdjointDesc(int(steps), int(checkpoint), int(swimmer), int(bool(rewind)))
        J = C.c_double()
        grad = np.zeros(4)
        self._check(self.lib.lbm_adjoint(self.h, C.byref(desc), C.byref(J), _ptr(grad)))
        return J.value, grad


# Stream-collide launch shapes (block, xcd_remap, resident) the tuner tries:
# workgroups of 128 / 256 / 512 nodes, block order round robin over the XCDs
# or one contiguous range per XCD, one workgroup per block or 1-4 persistent
# workgroups per CU beside the immersed-boundary kernels, or (resident -1)
# the serial order: those kernels, then one full-grid launch.
LAUNCH_CANDIDATES = ((512, True, 0), (512, False, 0), (256, True, 0), (256, False, 0), (128, True, 0),
                     (512, False, 1), (512, True, 1), (512, False, 2), (256, False, 2), (256, False, 4),
                     (512, False, -1), (256, False, -1))


def tune_launch(make, candidates=LAUNCH_CANDIDATES, steps=200, warmup=50, rounds=2):
    """Pick the fastest stream-collide launch shape for a workload.

    ``make()`` builds a scratch handle over the same boxes and swimmers as
    the handle to be tuned (e.g. ``lambda: batch_from_ensemble(ens)``), so
    the caller's state is never touched.  Each candidate runs ``warmup``
    steps, then ``steps`` timed steps (host clock around synchronised
    stepping, graph replays as in use); ``rounds`` passes alternate the
    candidate order and each candidate keeps its best pass.  The scratch
    handle is destroyed before returning.  Returns (best shape,
    {shape: microseconds per step})."""
    lat = make()
    try:
        res = {}
        for r in range(rounds):
            for c in (candidates if r % 2 == 0 else candidates[::-1]):
                lat.set_stream_collide_launch(*c)
                lat.step(warmup)
                lat.sync()
                t0 = time.perf_counter()
                lat.step(steps)
                lat.sync()
                us = (time.perf_counter() - t0) / steps * 1e6
                res[c] = min(res.get(c, math.inf), us)
        return min(res, key=res.get), res
    finally:
        lat.close()


def fp16_scale_for(max_abs_dev, headroom=16.0):
    """Power-of-two scale S for FP16-shifted storage that puts the largest
    expected |f - w| a factor `headroom` below the half-precision maximum."""
    return 2.0 ** math.floor(math.log2(65504.0 / headroom / float(max_abs_dev)))


def copy_bandwidth(nbytes=1 << 30, iters=20):
    """Achievable device-memory bandwidth (GB/s, read + write) of a plain copy."""
    lib = load_library()
    out = C.c_double()
    rc = lib.lbm_probe_copy_bandwidth(int(nbytes), int(iters), C.byref(out))
    if rc:
        raise LbmError(rc, lib.lbm_strerror(rc).decode())
    return out.value


class Batch(Lattice):
    """Independent periodic boxes stepped together (one launch per kernel per
    step over all boxes).  ``boxes``: list of (shape, tau, forcing)."""

    def __init__(self, boxes, storage=FP32_SHIFTED, width=3, fp16_scale=1.0, use_graphs=True,
                 stream=None, field_memory=None):
        self.lib = load_library()
        self.shapes = [tuple(int(v) for v in b[0]) for b in boxes]
        self.shape = self.shapes[0]
        self.storage = storage
        raw = None
        if stream is not None:
            raw = int(getattr(stream, "cuda_stream", stream)) or None
        arr = _box_array(boxes)
        self.field_tensor, fptr, fbytes = _field_memory(boxes, storage, field_memory)
        o = Opts(int(storage), int(width), float(fp16_scale), int(bool(use_graphs)), raw, fptr, fbytes)
        h = C.c_void_p()
        rc = self.lib.lbm_batch_create(arr, len(boxes), C.byref(o), C.byref(h))
        if rc:
            raise LbmError(rc, self.lib.lbm_strerror(rc).decode())
        self.h = h

    @property
    def N(self):
        return sum(nx * ny * nz for nx, ny, nz in self.shapes)

    @property
    def n_boxes(self):
        return self.lib.lbm_n_boxes(self.h)

    def step(self, n=1):
        self._check(self.lib.lbm_batch_step(self.h, int(n)))

    def add_swimmer(self, sw, box=0):
        beads, springs, act = _swimmer_descs(sw)
        sid = C.c_int32()
        self._check(self.lib.lbm_batch_swimmer_add(self.h, int(box), beads, springs, C.byref(act),
                                                   C.byref(sid)))
        return sid.value

    def _box_shape(self, box):
        return self.shapes[box]

    def velocity(self, box=0):
        nx, ny, nz = self.shapes[box]
        out = np.zeros((3, nz, ny, nx), np.float32)
        self._check(self.lib.lbm_batch_get_velocity(self.h, int(box), _ptr(out), 0))
        return out

    def conserved(self, box=-1):
        out = np.zeros(4)
        self._check(self.lib.lbm_batch_get_conserved(self.h, int(box), _ptr(out)))
        return out

    def populations(self):
        out = np.zeros(19 * self.N)
        self._check(self.lib.lbm_get_populations(self.h, _ptr(out)))
        return out


def batch_from_ensemble(ens, storage=FP32_SHIFTED, use_graphs=True, stream=None, field_memory=None):
    """Build a Batch from a ``workloads.ensemble`` dict (boxes share the
    kernel width of the first box)."""
    boxes = ens["boxes"]
    b = Batch([(bx["shape"], bx["tau"], bx["forcing"]) for bx in boxes], storage,
              boxes[0]["width"], use_graphs=use_graphs, stream=stream, field_memory=field_memory)
    for i, bx in enumerate(boxes):
        for sw in bx["swimmers"]:
            b.add_swimmer(sw, box=i)
    return b


def from_workload(case, storage=FP32_SHIFTED, fp16_scale=1.0, use_graphs=True, stream=None,
                  field_memory=None):
    """Build a Lattice with the swimmers of a ``workloads`` case dict."""
    lat = Lattice(case["shape"], case["tau"], case["forcing"], storage, case["width"], fp16_scale,
                  use_graphs, stream, field_memory)
    for sw in case.get("swimmers", []):
        lat.add_swimmer(sw)
    return lat


def swimmer_displacement(lattice, theta, steps, checkpoint=100, swimmer=0, rewind=True):
    """Differentiable x displacement of a swimmer's centre over `steps` steps
    as a function of theta = (A, B, alpha, k) (float64 tensor of 4).  The
    forward pass sets the parameters, runs the checkpointed forward and the
    hand-written adjoint in one library call; backward returns the stored
    gradient times the incoming one."""
    import torch

    class _Displacement(torch.autograd.Function):
        @staticmethod
        def forward(ctx, th):
            A, B, alpha, k = (float(v) for v in th.detach().cpu().tolist())
            lattice.set_swimmer_params(swimmer, A, B, alpha, k)
            J, grad = lattice.adjoint(steps, checkpoint, swimmer, rewind)
            ctx.save_for_backward(torch.as_tensor(grad, dtype=th.dtype, device=th.device))
            return torch.as_tensor(J, dtype=th.dtype, device=th.device)

        @staticmethod
        def backward(ctx, gJ):
            (grad,) = ctx.saved_tensors
            return gJ * grad

    return _Displacement.apply(theta)


def mlups(nodes, steps, seconds):
    return nodes * steps / seconds / 1e6 if seconds > 0 else math.nan
