"""Shared set-up for the GPU tests: build a system on the device from a seeded
structure, and the matching oracle system on the host."""
from __future__ import annotations

import functools
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import gen  # noqa: E402


def log(*a):
    print(*a, flush=True)


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def gpu_context(struct, device_outputs=True):
    """Context with H, S built on the device from the structure's positions."""
    torch = torch_cuda()
    from paper_1210_1531_amd import Context, model
    ctx = Context(device_outputs=device_outputs)
    pos = torch.tensor(struct.pos, dtype=torch.float64, device="cuda")
    ctx.sk_build(model.sk_model(), pos, struct.cell)
    rowptr, colind, H, S = ctx.sk_get_csr()
    ctx.set_system(rowptr, colind, H, S, pos=pos, cell=struct.cell, r_cluster=struct.r_cluster)
    ctx._csr = (rowptr, colind, H, S)
    ctx._pos = pos
    return ctx


@functools.lru_cache(maxsize=8)
def oracle_system(key, nu=None):
    from oracle import solve
    s = gen.make(key, nu=nu)
    return s, solve.build_system(s)


@functools.lru_cache(maxsize=8)
def oracle_solution(key, nu=None, with_forces=False):
    from oracle import solve
    s, sysm = oracle_system(key, nu)
    workers = min(16, os.cpu_count() or 1)
    return solve.solve(sysm, workers=workers, with_forces=with_forces)


def np_(x):
    try:
        import torch
        if isinstance(x, torch.Tensor):
            return x.detach().cpu().numpy()
    except Exception:
        pass
    return np.asarray(x)
