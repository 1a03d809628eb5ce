"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import json
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def bandwidth(workload: str, kernel: str) -> float:
    with open(os.path.join(ROOT, "tests", "golden", "bandwidths.json")) as f:
        return float(json.load(f)[workload][kernel]["h"])


def device():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def rel_err(got, ref, floor=1e-16):
    """Relative error per query, ignoring queries whose exact KDE is below
    ``floor`` (the paper excludes KDE values under 1e-16)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    keep = ref >= floor
    return np.abs(got[keep] - ref[keep]) / ref[keep], int((~keep).sum())
