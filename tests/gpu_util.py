"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import sys

import numpy as np
import torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return None if a is None else torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel_err(got, want):
    """max |got - want| / max |want| (field-scaled relative error)."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    scale = np.abs(want).max()
    if scale == 0:
        return float(np.abs(got).max())
    return float(np.abs(got - want).max() / scale)


def rel_err_pointwise(got, want, floor=1e-6):
    """max over cells of |got - want| / max(|want|, floor * max |want|): the
    relative error of every cell whose value is at least floor of the
    field's largest, and an absolute error at that level below it."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    scale = np.abs(want).max()
    if scale == 0:
        return float(np.abs(got).max())
    return float((np.abs(got - want) / np.maximum(np.abs(want), floor * scale)).max())


def gpu_problem(prob, x=None):
    """Device copy of an inputs.random_helmholtz-style problem dict."""
    return {
        "grid": prob["grid"], "bc": prob["bc"],
        "mask": dev(prob.get("mask"), torch.uint8),
        "alpha": dev(prob.get("alpha")), "alpha_c": prob.get("alpha_c", 0.0),
        "beta": dev(prob.get("beta")), "beta_c": prob.get("beta_c", 0.0),
        "rhs": dev(prob["rhs"]), "x": dev(prob["x0"] if x is None else x),
    }
