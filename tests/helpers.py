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
