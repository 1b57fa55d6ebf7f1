"""CPU checks of the C-ABI boundary: the library loads, exports exactly what
include/lbmib.h declares, and rejects invalid arguments before touching the
GPU."""
import ctypes as C
import os
import re

import pytest

from paper_2202_12147_amd import lbmib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "lbmib.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert _declared() == sorted(lbmib.SYMBOLS)


def test_library_exports_every_symbol():
    lib = lbmib.load_library()
    for name in _declared():
        assert hasattr(lib, name), name


def test_invalid_arguments_rejected():
    lib = lbmib.load_library()
    h = C.c_void_p()
    ok = lbmib.Grid(32, 32, 32)
    assert lib.lbm_create(C.byref(ok), 0.5, 0, None, C.byref(h)) == -1  # tau <= 1/2
    assert lib.lbm_create(C.byref(ok), float("nan"), 0, None, C.byref(h)) == -1
    assert lib.lbm_create(C.byref(lbmib.Grid(8, 32, 32)), 1.0, 0, None, C.byref(h)) == -1
    assert lib.lbm_create(C.byref(ok), 1.0, 7, None, C.byref(h)) == -1  # bad forcing
    bad = lbmib.Opts(0, 5, 1.0, 1, None)
    assert lib.lbm_create(C.byref(ok), 1.0, 0, C.byref(bad), C.byref(h)) == -1  # width 5
    bad = lbmib.Opts(1, 3, 3.0, 1, None)
    assert lib.lbm_create(C.byref(ok), 1.0, 0, C.byref(bad), C.byref(h)) == -1  # scale not 2^k
    assert lib.lbm_create(None, 1.0, 0, None, C.byref(h)) == -1
    bad = lbmib.Opts(9, 3, 1.0, 1, None)
    assert lib.lbm_create(C.byref(ok), 1.0, 0, C.byref(bad), C.byref(h)) == -1  # bad storage
    # one box holds at most 2^31 - 2^16 nodes (32-bit node offsets in the kernels)
    assert lib.lbm_create(C.byref(lbmib.Grid(2048, 1024, 1024)), 1.0, 0, None, C.byref(h)) == -1
    assert lib.lbm_create(C.byref(lbmib.Grid(65535, 128, 256)), 1.0, 0, None, C.byref(h)) == -1
    # a batch holds fewer than 2^31 nodes in all, and at least one box
    boxes = (lbmib.BoxDesc * 2)(lbmib.BoxDesc(lbmib.Grid(1024, 1024, 1024), 1.0, 0),
                                lbmib.BoxDesc(lbmib.Grid(1024, 1024, 1024), 1.0, 0))
    assert lib.lbm_batch_create(boxes, 2, None, C.byref(h)) == -1
    assert lib.lbm_batch_create(boxes, 0, None, C.byref(h)) == -1
    assert h.value is None
    count = C.c_int64()
    assert lib.lbm_average_begin(None, 1) == -1
    assert lib.lbm_get_average_velocity(None, 0, None, 0, C.byref(count)) == -1
    desc = lbmib.AdjointDesc(10, 5, 0, 0)
    J, g = C.c_double(), (C.c_double * 4)()
    assert lib.lbm_adjoint(None, C.byref(desc), C.byref(J), g) == -1
    assert lib.lbm_swimmer_set_params(None, 0, 1e-3, 1e-3, 1.0, 0.01) == -1
    assert lib.lbm_autotune(None, 4, None, None, 0) == -1
    assert lib.lbm_strerror(-1) == b"invalid argument"
    assert lib.lbm_destroy(None) == 0


def test_field_bytes_and_caller_memory_checks():
    """lbm_field_bytes: two population sets (19 x 4 bytes per node, 19 x 2
    with FP16 storage) plus 3 + 3 float32 of force and velocity per node, the
    node count padded to whole 256-node population blocks (a batch: the sum
    of its boxes, padded once).  Caller memory that is misaligned or too small
    is refused before any device call."""
    lib = lbmib.load_library()
    out = C.c_int64()
    one = (lbmib.BoxDesc * 1)(lbmib.BoxDesc(lbmib.Grid(128, 128, 128), 0.8, 0))
    assert lib.lbm_field_bytes(one, 1, 0, C.byref(out)) == 0
    assert out.value == 128 ** 3 * (2 * 19 * 4 + 24)
    assert lbmib.field_bytes([((128, 128, 128), 0.8, 0)], lbmib.FP16_SHIFTED) == 128 ** 3 * (2 * 19 * 2 + 24)
    ragged = [((100, 20, 17), 1.0, 0), ((16, 16, 17), 0.7, 1)]
    padded = -(-(100 * 20 * 17 + 16 * 16 * 17) // 256) * 256
    assert lbmib.field_bytes(ragged) == padded * (2 * 19 * 4 + 24)
    assert lbmib.field_bytes(ragged, lbmib.FP32_PLAIN) == padded * (2 * 19 * 4 + 24)
    # the in-place storage keeps one population set
    assert lbmib.field_bytes([((128, 128, 128), 0.8, 0)], lbmib.FP32_INPLACE) == 128 ** 3 * (19 * 4 + 24)
    assert lib.lbm_field_bytes(one, 1, 9, C.byref(out)) == -1  # storage
    assert lib.lbm_field_bytes(one, 1, 0, None) == -1
    assert lib.lbm_field_bytes(one, 0, 0, C.byref(out)) == -1
    bad = (lbmib.BoxDesc * 1)(lbmib.BoxDesc(lbmib.Grid(8, 128, 128), 0.8, 0))
    assert lib.lbm_field_bytes(bad, 1, 0, C.byref(out)) == -1
    h = C.c_void_p()
    g = lbmib.Grid(128, 128, 128)
    need = 128 ** 3 * (2 * 19 * 4 + 24)
    o = lbmib.Opts(0, 3, 1.0, 1, None, 0x10000 + 8, need)  # not 256-byte aligned
    assert lib.lbm_create(C.byref(g), 1.0, 0, C.byref(o), C.byref(h)) == -1
    o = lbmib.Opts(0, 3, 1.0, 1, None, 0x10000, need - 1)  # too small
    assert lib.lbm_create(C.byref(g), 1.0, 0, C.byref(o), C.byref(h)) == -1
    assert lib.lbm_batch_create(one, 1, C.byref(o), C.byref(h)) == -1
    # one in-place set must stay below 4 GiB (32-bit byte offsets):
    # 1024 x 512 x 128 nodes x 76 bytes = 5.1 GB
    o = lbmib.Opts(3, 3, 1.0, 1, None, None, 0)
    assert lib.lbm_create(C.byref(lbmib.Grid(1024, 512, 128)), 1.0, 0, C.byref(o), C.byref(h)) == -1
    assert h.value is None


def test_binding_refuses_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(lbmib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(lbmib, "_lib", None)
    with pytest.raises(RuntimeError):
        lbmib.load_library()
