"""Helpers for GPU tests: move seeded cases to the device and build handles."""
from __future__ import annotations

import sys

import numpy as np


def say(*a):
    """Name the case before each GPU step (flushed)."""
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def to_dev(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


class DevCase:
    """A fvcases.Case on the device with its Mesh and Matrix handles."""

    def __init__(self, case, symmetric=True, fp32_copy=False):
        import torch

        import paper_1505_07630_amd as fv

        self.case = case
        self.owner = to_dev(case.owner, torch.int32)
        self.nb = to_dev(case.neighbour, torch.int32)
        self.diag = to_dev(case.diag, torch.float64)
        self.upper = to_dev(case.upper, torch.float64)
        self.lower = None if symmetric else to_dev(case.lower, torch.float64)
        self.b = to_dev(case.b, torch.float64)
        self.mesh = fv.Mesh(case.n, self.owner, self.nb)
        self.A = fv.Matrix(self.mesh, self.diag, self.upper, self.lower, fp32_copy=fp32_copy)

    def close(self):
        self.A.close()
        self.mesh.close()


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
