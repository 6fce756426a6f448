"""Shared helpers of the GPU tests."""
import os

import numpy as np
import pytest


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(msg):
    print("[gpu-test] " + msg, flush=True)


def rel_err(a, b, fluid):
    """max |a-b| over fluid cells / max |b| over fluid cells."""
    a = np.asarray(a)[..., fluid]
    b = np.asarray(b)[..., fluid]
    scale = np.abs(b).max()
    return float(np.abs(a - b).max() / (scale if scale > 0 else 1.0))


def compare_fields(gf, of, prob, keys=("u", "T", "Y", "Ph", "rho")):
    fluid = prob.mask == 0
    out = {}
    for k in keys:
        if k == "Y":
            out[k] = max(rel_err(gf[k][s], of[k][s], fluid) for s in range(of[k].shape[0]))
        elif k == "u":
            dims = 2 if prob.lattice == 9 else 3
            scale = max(np.abs(of["u"][d][fluid]).max() for d in range(dims))
            out[k] = max(float(np.abs(gf["u"][d][fluid] - of["u"][d][fluid]).max()) for d in range(dims)) / (
                scale if scale > 0 else 1.0)
        else:
            out[k] = rel_err(gf[k], of[k], fluid)
    return out


def oracle_threads():
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or None
