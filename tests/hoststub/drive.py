"""Drive the library's host code, built against the HIP stand-in of
hip_stub.cpp, through the call sequences of the GPU tests and the benchmark
(argument marshalling, handle lifetimes, launch-shape and graph changes, the
tuner, the adjoint's workspaces and graph caches, checkpoints, averages,
batches).  Run by tests/test_host_asan.py under AddressSanitizer; the
results are meaningless (no kernel runs), only memory errors matter, except
for the host's own population index map, which inplace_mapping checks.

    python tests/hoststub/drive.py <path of the stub-built library> <scratch dir>
"""
import ctypes as C
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_2202_12147_amd import lbmib, workloads as wl  # noqa: E402


def step_pattern(lat):
    for n in (1, 5, 20, 13, 32, 71, 0):
        lat.step(n)
    lat.sync()


def observables(lat, batch=False):
    lat.markers()
    lat.marker_velocities()
    lat.marker_forces()
    lat.bead_centres()
    lat.swimmer_centres()
    lat.populations()
    lat.conserved()
    lib = lat.lib
    boxes = lat.shapes if batch else [lat.shape]
    for b, (nx, ny, nz) in enumerate(boxes):
        u = np.zeros((3, nz, ny, nx), np.float32)
        if batch:
            assert lib.lbm_batch_get_velocity(lat.h, b, lbmib._ptr(u), 0) == 0
            assert lib.lbm_batch_get_velocity(lat.h, b, lbmib._ptr(u), 1) == 0
            lat.conserved(b)
        else:
            assert lib.lbm_get_velocity(lat.h, lbmib._ptr(u), 1) == 0
            lat.velocity()
            lat.density()
        dst = np.zeros(4)
        assert lib.lbm_batch_get_conserved_noalloc(lat.h, b, 4096, lbmib._ptr(dst)) == 0
        assert lib.lbm_batch_get_conserved_noalloc(lat.h, b, 4097, lbmib._ptr(dst)) == -1


def averages(lat, batch=False):
    lat.average_begin(3)
    lat.step(40)
    boxes = lat.shapes if batch else [lat.shape]
    for b, (nx, ny, nz) in enumerate(boxes):
        lat.average_velocity(b)
        u = np.zeros((3, nz, ny, nx), np.float32)
        cnt = C.c_int64()
        assert lat.lib.lbm_get_average_velocity(lat.h, b, lbmib._ptr(u), 1, C.byref(cnt)) == 0
    lat.set_stream_collide_launch(128, True, 2)
    lat.step(9)
    lat.average_begin(0)


def launch_shapes(lat):
    for block in (128, 256, 512):
        for remap in (0, 1):
            for res in (-1, 0, 1, 2, 3):
                lat.set_stream_collide_launch(block, remap, res)
                lat.step(3)
    lat.set_kernel_timing(True)
    lat.step(40)
    lat.kernel_time()
    lat.set_kernel_timing(False)


def single(case, tmp, storage=lbmib.FP32_SHIFTED, scale=1.0, graphs=True):
    lat = lbmib.from_workload(case, storage=storage, fp16_scale=scale, use_graphs=graphs)
    nx, ny, nz = lat.shape
    if not case.get("swimmers"):
        lat.set_populations(wl.random_deviation(lat.shape, 1, 1e-4))
    lat.set_body_force((1e-6, 0, 0))
    observables(lat)
    step_pattern(lat)
    observables(lat)
    averages(lat)
    launch_shapes(lat)
    path = os.path.join(tmp, "ck.bin")
    lat.save(path)
    lat.step(7)
    lat.load(path)
    step_pattern(lat)
    tuner_disabled(lat, tmp)
    observables(lat)
    lat.close()


def batch(ens, tmp, graphs=True, storage=lbmib.FP32_SHIFTED):
    b = lbmib.batch_from_ensemble(ens, storage=storage, use_graphs=graphs)
    observables(b, batch=True)
    step_pattern(b)
    averages(b, batch=True)
    launch_shapes(b)
    path = os.path.join(tmp, "bk.bin")
    b.save(path)
    b.load(path)
    observables(b, batch=True)
    b.close()


def caller_field_memory(case, storage):
    """A handle whose node fields live in a caller buffer (here host memory,
    which the stand-in's device memory is): every byte the library writes must
    stay inside the lbm_field_bytes it asked for."""
    lib = lbmib._lib
    need = lbmib.field_bytes([(case["shape"], case["tau"], case["forcing"])], storage)
    raw = np.zeros(need + 512, np.uint8)
    start = (-raw.ctypes.data) % 256
    buf = raw[start:start + need]  # exactly the asked-for bytes, 256-byte aligned
    o = lbmib.Opts(int(storage), int(case["width"]), 1.0, 1, None, buf.ctypes.data, need)
    h = C.c_void_p()
    assert lib.lbm_create(C.byref(lbmib.Grid(*case["shape"])), float(case["tau"]), int(case["forcing"]), C.byref(o),
                          C.byref(h)) == 0
    lat = object.__new__(lbmib.Lattice)
    lat.lib, lat.h, lat.shape, lat.storage, lat.field_tensor = lib, h, tuple(case["shape"]), storage, None
    for sw in case.get("swimmers", []):
        lat.add_swimmer(sw)
    step_pattern(lat)
    observables(lat)
    lat.close()
    assert raw[:start].max(initial=0) == 0 and raw[start + need:].max(initial=0) == 0


def inplace_mapping():
    """The host's map between the interface's population layout and the
    in-place set: with no kernel running (the stand-in's launches do
    nothing), what set_populations stores reads back unchanged at step 0,
    and after one (empty) step, whose parity moves every value to the other
    arrangement, reads back as a permutation of the same values."""
    shape = (20, 17, 19)
    lat = lbmib.Lattice(shape, 0.9, storage=lbmib.FP32_INPLACE)
    dev = np.random.default_rng(3).standard_normal(19 * 20 * 17 * 19) * 1e-3
    lat.set_populations(dev)
    stored = dev.astype(np.float32).astype(np.float64)
    assert np.array_equal(lat.populations().ravel(), stored)
    lat.step(1)
    lat.sync()
    got = lat.populations().ravel()
    assert not np.array_equal(got, stored)
    assert np.array_equal(np.sort(got), np.sort(stored))
    lat.close()


def tuner_disabled(lat, tmp):
    """The tuner returns LBM_ESTATE and an empty report."""
    for cache in (None, os.path.join(tmp, "tune.txt")):
        try:
            lat.autotune(4, cache)
        except lbmib.LbmError as e:
            assert e.code == -4
        else:
            raise AssertionError("the tuner ran")


def tuner_sequence(tmp):
    """The call sequence of the GPU test during which glibc reported a
    corrupted heap, with the tuner now refusing to run."""
    ens = wl.ensemble(seed=5, nboxes=4)
    a = lbmib.batch_from_ensemble(ens)
    b = lbmib.batch_from_ensemble(ens)
    a.step(40)
    b.step(40)
    tuner_disabled(a, tmp)
    a.step(25)
    b.step(25)
    a.markers()
    a.populations()
    a.close()
    b.close()


def adjoints():
    case = wl.adjoint_case(reduced=True)
    for graphs in (True, False):
        lat = lbmib.from_workload(case, use_graphs=graphs)
        lat.adjoint(1, checkpoint=16)
        lat.adjoint(40, checkpoint=16)
        lat.adjoint(150, checkpoint=40)
        lat.adjoint(150, checkpoint=150)
        lat.adjoint(90, checkpoint=20, rewind=True)
        lat.step(7)
        lat.adjoint(30, checkpoint=16, rewind=True)
        lat.set_swimmer_params(0, 7e-4, 1.3e-3, 1.1, 0.02)
        lat.set_stream_collide_launch(256, 1, 2)
        lat.adjoint(33, checkpoint=10)
        lat.close()
    for shape in ((24, 24, 24), (25, 22, 23)):
        c = dict(case, shape=shape)
        c["swimmers"] = [wl.swimmer((shape[0] - 0.5, 0.4, shape[2] / 2), 7.0, A=1e-3, T=2000.0,
                                    alpha=math.pi / 3)]
        lbmib.from_workload(c).adjoint(40, checkpoint=16)
    two = dict(case, shape=(48, 32, 32))
    two["swimmers"] = [wl.swimmer((24, 8, 16), 7.0, A=1e-3, T=2000.0),
                       wl.swimmer((24, 24, 16), 7.0, A=8e-4, T=2000.0)]
    lat = lbmib.from_workload(two)
    for sw in (0, 1, 0):
        lat.adjoint(40, checkpoint=16, swimmer=sw, rewind=True)
    for width in (2, 4):
        lbmib.from_workload(dict(case, width=width)).adjoint(24, checkpoint=10)


def main():
    lib_path, tmp = sys.argv[1], sys.argv[2]
    lbmib._lib = lbmib.bind(C.CDLL(lib_path))
    small = wl.small_case()
    single(dict(small, shape=(16, 16, 16), swimmers=[]), tmp)
    single(dict(small, shape=(20, 17, 19), swimmers=[]), tmp, graphs=False)
    single(small, tmp)
    single(small, tmp, storage=lbmib.FP16_SHIFTED, scale=2.0 ** 27)
    single(small, tmp, storage=lbmib.FP32_PLAIN)
    single(small, tmp, storage=lbmib.FP32_INPLACE)
    single(dict(small, shape=(20, 17, 19), swimmers=[]), tmp, storage=lbmib.FP32_INPLACE)
    inplace_mapping()
    caller_field_memory(small, lbmib.FP32_SHIFTED)
    caller_field_memory(small, lbmib.FP32_INPLACE)
    caller_field_memory(dict(small, shape=(20, 17, 19), swimmers=[]), lbmib.FP16_SHIFTED)
    single(dict(small, width=2), tmp, graphs=False)
    seams = dict(small, shape=(33, 30, 29))
    seams["swimmers"] = [wl.swimmer((31.5, 0.6, 28.2), 10.0, A=1e-3, T=500.0)]
    single(seams, tmp)
    single(wl.paper_moduli_case(), tmp)
    adjoints()
    tuner_sequence(tmp)
    batch(wl.ensemble(seed=2, nboxes=3), tmp)
    batch(wl.ensemble(seed=7, nboxes=5), tmp, graphs=False)
    batch(wl.ensemble(seed=7, nboxes=3), tmp, storage=lbmib.FP32_INPLACE)
    ragged = dict(boxes=[dict(wl.small_case(), shape=(20, 17, 19), swimmers=[]),
                         dict(wl.small_case(), shape=(33, 30, 29)),
                         dict(wl.small_case(), shape=(24, 20, 17), forcing=wl.SHAN_CHEN, swimmers=[])])
    batch(ragged, tmp)
    out = C.c_double()
    assert lbmib._lib.lbm_probe_copy_bandwidth(1 << 20, 3, C.byref(out)) == 0
    print("host sequences done", flush=True)


if __name__ == "__main__":
    main()
