"""Helpers shared by the GPU tests: device arrays, workload contexts, tolerances."""
import sys

import numpy as np

EPS = np.finfo(np.float64).eps


def torch_dev():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a visible MI355X")
    return torch


def to_dev(a):
    torch = torch_dev()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def to_host(t):
    torch = torch_dev()
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def empty_dev(*shape):
    torch = torch_dev()
    return torch.empty(*shape, dtype=torch.float64, device="cuda")


def say(msg):
    """Name the case before each GPU call so that a failure is attributable."""
    print(msg, flush=True)
    sys.stdout.flush()


def stencil_bound(op, X):
    """Rounding bound for one application of H to X: every output is a sum of
    at most 7 products, each bounded by (|d| + 2 sum c) |X|max."""
    c = op.kinetic * sum(1.0 / h ** 2 for h in op.h)
    dmax = np.max(np.abs(op.V + op.shift)) + 2.0 * c
    return 16.0 * EPS * (dmax + 2.0 * c) * np.max(np.abs(X))
