"""Helpers shared by the GPU tests (inputs to the device, error metrics)."""
import os
import sys

import numpy as np


def dev(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def col_err(got, ref):
    """max_k ||got_k - ref_k|| / ||ref_k|| over columns (first axis)."""
    g = np.asarray(got).reshape(np.shape(got)[0], -1).astype(np.complex128)
    r = np.asarray(ref).reshape(np.shape(ref)[0], -1).astype(np.complex128)
    return float(np.max(np.linalg.norm(g - r, axis=1) / np.linalg.norm(r, axis=1)))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def workers():
    return max(1, min(16, len(os.sched_getaffinity(0))))
