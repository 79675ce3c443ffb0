"""Green's-function columns by the conjugate orthogonal conjugate gradient
method (oracle; test infrastructure).

The letter lists the Krylov solvers of its family for the generalized shifted
equation (z S - H) x = b of Eq. 1, of which the multiple Arnoldi method is
the one used for MD; the conjugate-gradient-type members solve Eq. 1 itself
rather than a projection of it.  For real symmetric H and S and complex z the
matrix A = z S - H is complex symmetric (A^T = A, not Hermitian), and COCG
(van der Vorst and Melissen, IEEE Trans. Magn. 26, 706 (1990)) is conjugate
gradients with the bilinear form <u, v> = u^T v in place of the Hermitian
product:
  x_0 = 0, r_0 = b, p_0 = r_0, rho_0 = <r_0, r_0>
  k = 0, 1, ...:  v = A p_k;  alpha = rho_k / <p_k, v>
                  x_{k+1} = x_k + alpha p_k;  r_{k+1} = r_k - alpha v
                  stop when |r_{k+1}|_2 <= tol |b|_2
                  rho_{k+1} = <r_{k+1}, r_{k+1}>;  beta = rho_{k+1} / rho_k
                  p_{k+1} = r_{k+1} + beta p_k
The reading taken for the column problem (the same locality as the Arnoldi
columns): column j is solved on its atom's cluster, A = z S_C - H_C and
b = e_l, so the solution is the column of (z S_C - H_C)^-1, which for a
whole-cell cluster is the column of (z S - H)^-1 itself.
"""
from __future__ import annotations

import numpy as np

from . import neighbors as _nb

NORB = _nb.NORB


def cocg(A, b, tol, max_iter):
    """COCG on a complex symmetric A (dense or sparse, anything with @).

    Returns (x, iterations); iterations is -1 when tol was not reached within
    max_iter steps or the method broke down (<p, A p> = 0 or rho = 0).
    """
    b = np.asarray(b, np.complex128)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rho = r @ r
    bnorm = np.linalg.norm(b)
    for k in range(max_iter):
        v = A @ p
        d = p @ v
        if d == 0:
            return x, -1
        alpha = rho / d
        x = x + alpha * p
        r = r - alpha * v
        if np.linalg.norm(r) <= tol * bnorm:
            return x, k + 1
        rho_new = r @ r
        if rho_new == 0:
            return x, -1
        p = r + (rho_new / rho) * p
        rho = rho_new
    return x, -1


def cluster_problem(sysm, j):
    """(atoms, H_C, S_C, l) of column j's cluster (local orbital order)."""
    J, a = divmod(int(j), NORB)
    atoms = _nb.cluster_of(sysm.pos, sysm.cell, J, sysm.r_cluster)
    Hc, Sc = _nb.cluster_matrices(sysm.pos, sysm.cell, atoms, sysm.params)
    l = NORB * int(np.searchsorted(atoms, J)) + a
    return atoms, Hc, Sc, l


def green_columns_cocg(sysm, cols, z, tol=1e-10, max_iter=2000):
    """COCG solutions of (z_q S_C - H_C) x = e_l per column and energy.

    Returns (G, iters): G[i][q] is the cluster-ordered solution for column
    cols[i] at z[q], iters[i, q] its iteration count (-1: not converged).
    """
    z = np.atleast_1d(np.asarray(z, np.complex128))
    G, iters = [], np.zeros((len(cols), z.size), dtype=np.int64)
    for i, j in enumerate(cols):
        _, Hc, Sc, l = cluster_problem(sysm, j)
        b = np.zeros(Hc.shape[0], np.complex128)
        b[l] = 1.0
        row = []
        for q, zq in enumerate(z):
            x, it = cocg(zq * Sc - Hc, b, tol, max_iter)
            row.append(x)
            iters[i, q] = it
        G.append(row)
    return G, iters


def green_columns_dense(sysm, cols, z):
    """The same columns by dense solves of the cluster systems (the definition)."""
    z = np.atleast_1d(np.asarray(z, np.complex128))
    out = []
    for j in cols:
        _, Hc, Sc, l = cluster_problem(sysm, j)
        b = np.zeros(Hc.shape[0], np.complex128)
        b[l] = 1.0
        out.append([np.linalg.solve(zq * Sc - Hc, b) for zq in z])
    return out
