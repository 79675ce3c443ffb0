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


def gpu_context(struct, device_outputs=True, sk=None):
    """Context with H, S built on the device from the structure's positions
    (sk: overrides of the Slater-Koster model, e.g. a shorter cutoff)."""
    torch = torch_cuda()
    from paper_1210_1531_amd import Context, model
    ctx = Context(device_outputs=device_outputs)
    pos = torch.tensor(struct.pos, dtype=torch.float64, device="cuda")
    ctx._sk = model.sk_model(**(sk or {}))
    ctx.sk_build(ctx._sk, pos, struct.cell)
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
    return solve.solve(sysm, with_forces=with_forces)


def torch_index(ix, like):
    """Index array for `like` (a torch tensor on the device, or NumPy)."""
    try:
        import torch
        if isinstance(like, torch.Tensor):
            return torch.as_tensor(np.asarray(ix, dtype=np.int64), device=like.device)
    except Exception:
        pass
    return np.asarray(ix, dtype=np.int64)


def np_(x):
    try:
        import torch
        if isinstance(x, torch.Tensor):
            return x.detach().cpu().numpy()
    except Exception:
        pass
    return np.asarray(x)


def stratified_atoms(sizes, n_pick, strata=8, seed=0):
    """n_pick atoms spread evenly over `strata` bands of cluster size (the
    atoms sorted by size, then cut into equal bands), drawn without
    replacement inside each band, plus the smallest and largest cluster."""
    rng = np.random.default_rng(seed)
    order = np.argsort(sizes, kind="stable")
    bands = np.array_split(order, strata)
    per = max(1, n_pick // strata)
    pick = [order[:1], order[-1:]]
    for b in bands:
        pick.append(rng.choice(b, size=min(per, b.size), replace=False))
    return np.unique(np.concatenate(pick))[:max(n_pick, 2)]


def sampled_parity(ctx, geo, atoms_pick, mu, kT):
    """The four columns of each picked atom: oracle mode K (fork-server
    workers) against the GPU's spectra and rho rows at the GPU's mu.  Returns
    a dict of the worst differences and the per-column electron counts of
    both sides."""
    from oracle import fermi, solve
    cols = (4 * np.asarray(atoms_pick)[:, None] + np.arange(4)[None, :]).ravel()
    cd = solve.column_data(geo, cols)
    eps_d, w_d, nu_d = ctx.spectra()
    rho_d, pi_d = ctx.density_matrix()
    rowptr = np_(ctx._csr[0])
    # only the sampled rows leave the device
    idx = np.concatenate([np.arange(rowptr[j], rowptr[j + 1]) for j in cols])
    take = (lambda a, ix: np_(a[torch_index(ix, a)]))
    eps, w, nu_eff = take(eps_d, cols), take(w_d, cols), take(nu_d, cols)
    rho, pi = take(rho_d, idx), take(pi_d, idx)
    out = dict(nu_mismatch=0, deps=0.0, dw=0.0, drho=0.0, dpi=0.0, n_gpu=[], n_ora=[])
    pos = 0
    for i, j in enumerate(cols):
        k = int(cd["nu_eff"][i])
        n_row = int(rowptr[j + 1] - rowptr[j])
        lo, hi = pos, pos + n_row
        pos += n_row
        if int(nu_eff[i]) != k:
            out["nu_mismatch"] += 1
            continue
        e_o, w_o = cd["eps"][i, :k], cd["w"][i, :k]
        out["deps"] = max(out["deps"], float(np.abs(eps[i, :k] - e_o).max()))
        out["dw"] = max(out["dw"], float(np.abs(w[i, :k] - w_o).max()))
        f = fermi.fermi((e_o - mu) / kT)
        r_o = 2.0 * (cd["ypd"][i] @ f)
        p_o = 2.0 * (cd["ypd"][i] @ (f * e_o))
        assert r_o.size == n_row
        out["drho"] = max(out["drho"], float(np.abs(rho[lo:hi] - r_o).max()))
        out["dpi"] = max(out["dpi"], float(np.abs(pi[lo:hi] - p_o).max()))
        out["n_ora"].append(float(np.sum(w_o * f)))
        out["n_gpu"].append(float(np.sum(w[i, :k] * fermi.fermi((eps[i, :k] - mu) / kT))))
    out["n_gpu"] = np.array(out["n_gpu"])
    out["n_ora"] = np.array(out["n_ora"])
    out["cols"] = cols
    return out
