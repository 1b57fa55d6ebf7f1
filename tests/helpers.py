"""Shared test helpers: build matched oracle / HIP runs from one workload."""
import numpy as np

from oracle import orc


def oracle_from(case):
    o = orc.Oracle(case["shape"], case["tau"], case["forcing"], case["width"])
    for sw in case.get("swimmers", []):
        o.add_swimmer_desc(sw)
    return o


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def max_rel(a, b):
    """Element-wise error of a against b, relative to the largest |b|:
    max |a - b| / max |b|."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def oracle_interface():
    """The library's calling interface served by the FP64 oracle (liborc.so,
    oracle/orc_abi.c), with the binding's signatures declared on it."""
    import ctypes as C

    from paper_2202_12147_amd import lbmib

    orc._load()  # builds liborc.so if it is missing
    return lbmib.bind(C.CDLL(orc._LIB_PATH))


def interface_lattice(lib, case, storage=0):
    """A binding Lattice over `lib` (the HIP library or the oracle's
    interface) with the swimmers of a workloads case: the same calls through
    either backend."""
    import ctypes as C

    from paper_2202_12147_amd import lbmib

    lat = object.__new__(lbmib.Lattice)
    lat.lib, lat.shape, lat.storage, lat.field_tensor = lib, tuple(case["shape"]), storage, None
    o = lbmib.Opts(int(storage), int(case["width"]), 1.0, 1, None, None, 0)
    h = C.c_void_p()
    rc = lib.lbm_create(C.byref(lbmib.Grid(*lat.shape)), float(case["tau"]), int(case["forcing"]), C.byref(o),
                        C.byref(h))
    assert rc == 0, rc
    lat.h = h
    for sw in case.get("swimmers", []):
        lat.add_swimmer(sw)
    return lat


def interface_batch(lib, boxes, width):
    """A binding Batch over `lib`: ``boxes`` a list of workloads box dicts
    (shape, tau, forcing, swimmers)."""
    import ctypes as C

    from paper_2202_12147_amd import lbmib

    b = object.__new__(lbmib.Batch)
    b.lib, b.storage, b.field_tensor = lib, 0, None
    b.shapes = [tuple(bx["shape"]) for bx in boxes]
    b.shape = b.shapes[0]
    arr = lbmib._box_array([(bx["shape"], bx["tau"], bx["forcing"]) for bx in boxes])
    o = lbmib.Opts(0, int(width), 1.0, 1, None, None, 0)
    h = C.c_void_p()
    assert lib.lbm_batch_create(arr, len(boxes), C.byref(o), C.byref(h)) == 0
    b.h = h
    for i, bx in enumerate(boxes):
        for sw in bx["swimmers"]:
            b.add_swimmer(sw, box=i)
    return b
