"""One Green's-function column by the multiple Arnoldi method (oracle, mode K).

The letter solves the generalized shifted equation (zS - H) x = b (Eq. 1) with
one Krylov subspace per column j of G = (zS - H)^-1, parallel over j, and takes
the density matrix from Eq. 2.  The algorithm itself is deferred to another
publication, so the steps below are the reading this project builds to:

  1. cluster C of the column's atom; dense principal submatrices H_C, S_C;
     l = local index of column j;
  2. v_1 = e_l / sqrt((S_C)_ll);
  3. for k = 1 .. nu-1: w = H_C v_k; S-orthogonalize w against v_1..v_k by
     modified Gram-Schmidt, twice; stop (nu_eff = k) if the orthogonalized w is
     at most 1e-12 of its length before; v_{k+1} = w / sqrt(w^T S_C w);
  4. h = V^T H_C V, s = V^T S_C V, each symmetrized;
  5. generalized symmetric eigenproblem h c = eps s c (LAPACK via SciPy),
     eps ascending, c^T s c = I;
  6. Y = V c, d = Y^T e_l, g = Y^T S_C e_l, weights w_k = g_s d_k g_k.

The Galerkin Green's function of the column is then
  G_ij(z) = sum_k Y_ik d_k / (z - eps_k),
and with Eq. 2 taken on this Ritz spectrum (the i0 limit is exact there)
  rho_ij = g_s sum_k f_k Y_ik d_k,     pi_ij = g_s sum_k f_k eps_k Y_ik d_k
(pi is the energy-density matrix).  g_s = 2 counts both spins.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from .fermi import fermi

G_SPIN = 2.0
BREAKDOWN = 1e-12


@dataclass
class ColumnResult:
    eps: np.ndarray  # (nu_eff,) Ritz values, ascending
    w: np.ndarray  # (nu_eff,) spectral weights g_s d g
    Y: np.ndarray  # (n_C, nu_eff) Ritz vectors in the cluster basis
    d: np.ndarray  # (nu_eff,) Y^T e_l
    nu_eff: int
    h: np.ndarray
    s: np.ndarray


def s_orthonormal_krylov(Hc: np.ndarray, Sc: np.ndarray, l: int, nu: int,
                         breakdown: float = BREAKDOWN):
    """Steps 2-3: S-orthonormal basis V of K_nu(H_C; e_l) by MGS2."""
    n = Hc.shape[0]
    nu = min(nu, n)
    V = np.zeros((n, nu))
    Z = np.zeros((n, nu))  # Z = S_C V, so that <v_i, w>_S = z_i^T w
    v = np.zeros(n)
    v[l] = 1.0 / np.sqrt(Sc[l, l])
    V[:, 0] = v
    Z[:, 0] = Sc @ v
    nu_eff = nu
    for k in range(1, nu):
        w = Hc @ V[:, k - 1]
        norm_before = np.linalg.norm(w)
        for _ in range(2):
            for i in range(k):
                w = w - (Z[:, i] @ w) * V[:, i]
        if np.linalg.norm(w) <= breakdown * norm_before:
            nu_eff = k
            break
        z = Sc @ w
        beta = np.sqrt(w @ z)
        V[:, k] = w / beta
        Z[:, k] = z / beta
    return V[:, :nu_eff], nu_eff


def project(Hc, Sc, V):
    """Step 4: projected pencil, symmetrized."""
    h = V.T @ Hc @ V
    s = V.T @ Sc @ V
    return 0.5 * (h + h.T), 0.5 * (s + s.T)


def ritz(Hc, Sc, l, V, g_spin=G_SPIN):
    """Steps 4-6 for a given basis V of the Krylov space."""
    h, s = project(Hc, Sc, V)
    eps, c = sla.eigh(h, s)
    Y = V @ c
    d = Y[l, :].copy()
    g = Y.T @ Sc[:, l]
    return ColumnResult(eps=eps, w=g_spin * d * g, Y=Y, d=d, nu_eff=V.shape[1], h=h, s=s)


def column_mode_k(Hc, Sc, l, nu, g_spin=G_SPIN, breakdown=BREAKDOWN) -> ColumnResult:
    V, _ = s_orthonormal_krylov(Hc, Sc, l, nu, breakdown)
    return ritz(Hc, Sc, l, V, g_spin)


def column_mode_d(Hc, Sc, l, g_spin=G_SPIN) -> ColumnResult:
    """Mode D: the whole cluster instead of a Krylov space (nu -> n_C limit)."""
    eps, Y = sla.eigh(Hc, Sc)
    d = Y[l, :].copy()
    g = Y.T @ Sc[:, l]
    n = Hc.shape[0]
    return ColumnResult(eps=eps, w=g_spin * d * g, Y=Y, d=d, nu_eff=n, h=Hc, s=Sc)


def density_column(res: ColumnResult, mu: float, kT: float, g_spin=G_SPIN):
    """rho_{i j} and pi_{i j} for every i of the cluster (Eq. 2 on the Ritz spectrum)."""
    f = fermi((res.eps - mu) / kT)
    yd = res.Y * res.d[None, :]
    return g_spin * (yd @ f), g_spin * (yd @ (f * res.eps))


def green_column(res: ColumnResult, z):
    """G_{i j}(z) = sum_k Y_ik d_k / (z - eps_k) for every i of the cluster.

    z may be an array of complex energies; the result has shape (n_C, len(z)).
    """
    z = np.atleast_1d(np.asarray(z, dtype=np.complex128))
    yd = res.Y * res.d[None, :]
    return yd @ (1.0 / (z[None, :] - res.eps[:, None]))
