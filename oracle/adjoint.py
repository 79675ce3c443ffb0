"""Exact gradient of the truncated-Krylov free energy (oracle; test
infrastructure).

The forces of the method are taken through the density matrix (the
Hellmann-Feynman form F = -sum [rho dH/dR - pi dS/dR]), which is the
derivative of the free energy only when the Krylov space of every column is
exact.  With nu below the cluster size each column's contribution depends on
H_C also through its Krylov space K_nu(H_C; e_l), and the exact derivative
needs the reverse pass through the Krylov construction as well.

Reading: the free energy at fixed electron number has the R-gradient of the
grand potential at fixed mu (the mu-dependence cancels through the electron
count constraint), and the grand potential is a sum over columns,
  Omega = sum_j Omega_j,  Omega_j = sum_k w_jk omega(eps_jk),
  omega(e) = -kT log(1 + exp(-(e - mu) / kT)),
with (eps_jk, w_jk) the Ritz data of column j (Rayleigh-Ritz of the pencil
(H_C, S_C) on K_nu(H_C; e_l), w = g_s d g).  Omega_j is written below with
plain PyTorch CPU operations in float64 (Gram-Schmidt against the whole
basis, the projected pencil, Cholesky reduction and a symmetric eigensolve),
and its gradient with respect to H_C and S_C is taken by reverse-mode
automatic differentiation; the chain rule through the Slater-Koster blocks
of the cluster gives the forces.  The basis here is Euclidean-orthonormal;
the Ritz data depend only on the span, so Omega_j is the mode-K value.
"""
from __future__ import annotations

import numpy as np
import torch

from . import neighbors as _nb
from . import sk as _sk

NORB = _nb.NORB
G_SPIN = 2.0


def column_omega(Hc, Sc, l, nu, mu, kT):
    """Omega_j of one column as a differentiable function of (H_C, S_C).

    Hc, Sc: float64 torch tensors (n, n); l: local orbital of the column.
    Raises if the Krylov space becomes invariant before nu (the derivative
    of a breakdown is not defined by this reading).
    """
    n = Hc.shape[0]
    nu = min(nu, n)
    q = torch.zeros(n, dtype=torch.float64)
    q[l] = 1.0
    basis = [q]
    for _ in range(1, nu):
        w = Hc @ basis[-1]
        norm0 = torch.linalg.norm(w)
        for _pass in range(2):
            B = torch.stack(basis, 1)
            w = w - B @ (B.T @ w)
        nw = torch.linalg.norm(w)
        if not float(nw.detach()) > 1e-10 * float(norm0.detach()):
            raise ValueError("Krylov breakdown before nu")
        basis.append(w / nw)
    Q = torch.stack(basis, 1)
    h = Q.T @ Hc @ Q
    s = Q.T @ Sc @ Q
    h = 0.5 * (h + h.T)
    s = 0.5 * (s + s.T)
    L = torch.linalg.cholesky(s)
    Li = torch.linalg.solve_triangular(L, torch.eye(nu, dtype=torch.float64), upper=False)
    C = Li @ h @ Li.T
    eps, U = torch.linalg.eigh(0.5 * (C + C.T))
    c = Li.T @ U  # c^T s c = I
    d = c[0, :]  # Y_l,k: row l of Q is e_1
    g = (s @ c)[0, :]  # Y_k^T S_C e_l = (s c)_{1k}
    w = G_SPIN * d * g
    om = -kT * torch.nn.functional.softplus(-(eps - mu) / kT)
    return torch.sum(w * om)


def column_gradient(Hc, Sc, l, nu, mu, kT):
    """(Omega_j, dOmega_j/dH_C, dOmega_j/dS_C) as NumPy arrays."""
    H = torch.tensor(Hc, dtype=torch.float64, requires_grad=True)
    S = torch.tensor(Sc, dtype=torch.float64, requires_grad=True)
    om = column_omega(H, S, l, nu, mu, kT)
    om.backward()
    return float(om.detach()), H.grad.numpy(), S.grad.numpy()


def atom_force_parts(sysm, J, mu, alphas=(0, 1, 2, 3)):
    """The contribution of the columns (J, alpha) to -dOmega/dR of every atom
    of J's cluster: (cluster atoms, parts of shape (atoms, 3)).

    Each column's gradient with respect to its cluster's H_C and S_C is
    contracted with the Slater-Koster block derivatives of every pair of
    cluster atoms closer than r_cut (the blocks H_AB(d), d = R_B - R_A, so
    dH_AB/dR_B = +dH/dd and dH_AB/dR_A = -dH/dd).  sysm: a System or a
    Geometry (positions, box, cluster radius, nu, kT, model).
    """
    p = sysm.params
    atoms = _nb.cluster_of(sysm.pos, sysm.cell, J, sysm.r_cluster)
    Hc, Sc = _nb.cluster_matrices(sysm.pos, sysm.cell, atoms, p)
    jl = int(np.searchsorted(atoms, J))
    gH = np.zeros_like(Hc)
    gS = np.zeros_like(Sc)
    for a in alphas:
        _, h, s = column_gradient(Hc, Sc, NORB * jl + a, sysm.nu, mu, sysm.kT)
        gH += h
        gS += s
    dOm = np.zeros((atoms.size, 3))
    P = sysm.pos[atoms]
    for A in range(atoms.size):
        d_all = _nb.min_image(P - P[A][None, :], sysm.cell[None, :])
        r2 = np.einsum("ij,ij->i", d_all, d_all)
        for B in np.nonzero(r2 < p.r_cut * p.r_cut)[0]:
            if B == A:
                continue
            dH, dS = _sk.pair_block_grads(d_all[B], p)  # (3, 4, 4) each, d/dd
            blkH = gH[NORB * A:NORB * A + NORB, NORB * B:NORB * B + NORB]
            blkS = gS[NORB * A:NORB * A + NORB, NORB * B:NORB * B + NORB]
            gvec = np.einsum("cab,ab->c", dH, blkH) + np.einsum("cab,ab->c", dS, blkS)
            dOm[B] += gvec
            dOm[A] -= gvec
    return atoms, -dOm


def exact_forces(sysm, mu, cols=None):
    """F_I = -dOmega/dR_I at fixed mu, summed over the given columns (all if
    None): the exact derivative of the truncated-Krylov free energy."""
    n = sysm.n_atoms
    cols = np.arange(NORB * n) if cols is None else np.asarray(cols)
    F = np.zeros((n, 3))
    by_atom = {}
    for j in cols:
        by_atom.setdefault(int(j) // NORB, []).append(int(j) % NORB)
    for J, alphas in sorted(by_atom.items()):
        atoms, parts = atom_force_parts(sysm, J, mu, alphas)
        F[atoms] += parts
    return F


_WORK = {}


def _init_worker(geo, mu):
    torch.set_num_threads(1)
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover - threadpoolctl is optional
        pass
    _WORK["geo"] = geo
    _WORK["mu"] = mu


def _parts_task(J):
    atoms, parts = atom_force_parts(_WORK["geo"], J, _WORK["mu"])
    return J, atoms, parts


def exact_forces_on(geo, targets, mu, workers=None):
    """Exact forces of the atoms `targets` only: every atom whose cluster
    holds a target contributes (the cluster relation is symmetric, so these
    are the atoms of the targets' own clusters), spread over fork-server
    workers.  Returns an array (len(targets), 3)."""
    from . import pool as _pool
    targets = np.asarray(targets, dtype=np.int64)
    need = np.unique(np.concatenate(
        [_nb.cluster_of(geo.pos, geo.cell, int(I), geo.r_cluster) for I in targets]))
    # these workers import torch, which opens the GPU driver in each of them
    # on a GPU host, where the processes holding it are limited: at most 12
    workers = min(workers or _pool.default_workers(), 12)
    if workers > 1 and need.size > 8:
        with _pool.executor(workers, initializer=_init_worker, initargs=(geo, mu)) as ex:
            res = list(ex.map(_parts_task, need.tolist(),
                              chunksize=max(1, need.size // (8 * workers))))
    else:
        res = [(int(J), *atom_force_parts(geo, int(J), mu)) for J in need]
    where = {int(I): i for i, I in enumerate(targets)}
    F = np.zeros((targets.size, 3))
    for J, atoms, parts in sorted(res, key=lambda t: t[0]):
        for a, I in enumerate(atoms):
            i = where.get(int(I))
            if i is not None:
                F[i] += parts[a]
    return F
