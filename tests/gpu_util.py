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


def _cols(a):
    return np.asarray(a).reshape(np.shape(a)[0], -1).astype(np.complex128)


def l2_err(got, ref):
    """max_k ||got_k - ref_k||_2 / ||ref_k||_2 over columns (first axis)."""
    g, r = _cols(got), _cols(ref)
    return float(np.max(np.linalg.norm(g - r, axis=1) / np.linalg.norm(r, axis=1)))


def elem_err(got, ref):
    """max_k max_i |got_ki - ref_ki| / max_i |ref_ki|: every element of a column is
    held to the tolerance times that column's largest magnitude."""
    g, r = _cols(got), _cols(ref)
    return float(np.max(np.abs(g - r).max(axis=1) / np.abs(r).max(axis=1)))


def rel_err(got, ref):
    """The grade of every parity test: the larger of the per-column relative L2
    error and the per-column element-wise error (elem_err), maximised over
    columns.  A defect confined to a few grid points fails the element-wise
    part even where the column norm hides it."""
    return max(l2_err(got, ref), elem_err(got, ref))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def workers():
    return max(1, min(16, len(os.sched_getaffinity(0))))
