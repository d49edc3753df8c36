"""Shared helpers of the GPU parity tests (imported by test modules)."""

import math
import sys

import numpy as np

# Fields whose reference norm falls below this floor (times sqrt(P)) are
# reported but not compared with a relative measure: the relaxing workloads
# drive eta towards zero, where a relative error is meaningless.
NORM_FLOOR = 1e-30

# Kinetic coefficients that differ pairwise (M != L, kappa_c != kappa_eta):
# a kernel that used one coefficient in place of another fails a parity case
# run with them (the paper's own values have M = L and kappa_c = kappa_eta).
DISTINCT = {"M": 5.0, "kappa_c": 3.0, "L": 4.0, "kappa_eta": 2.0}


def rel_l2(got, ref):
    """Per-field ||got - ref||_2 / ||ref||_2 (None below the floor)."""
    P = ref[0].size
    out = []
    for f in range(ref.shape[0]):
        nb = float(np.linalg.norm(ref[f]))
        if nb < NORM_FLOOR * math.sqrt(P):
            out.append(None)
        else:
            out.append(float(np.linalg.norm(got[f] - ref[f])) / nb)
    return out


def max_rel(errs):
    vals = [e for e in errs if e is not None]
    return max(vals) if vals else 0.0


def gpu_or_fail():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X; none is visible"
    return torch


def announce(*what):
    """Print and flush the case name before a GPU step."""
    print("[gpu-case]", *what, flush=True)
    sys.stdout.flush()


def fp32_rounded(u):
    return np.asarray(u, dtype=np.float32).astype(np.float64)
