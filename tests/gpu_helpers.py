"""Shared helpers for the GPU tests: device gate and observed-data fixtures."""
import json
import os

import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "observed.json")


def observed():
    with open(GOLDEN) as f:
        return json.load(f)


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1902_09046_amd as P
    P.lib()  # raises if libpps.so is missing: no fallback path exists
    return torch


def rel_err(a, b, floor=0.0):
    import numpy as np
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), floor)
