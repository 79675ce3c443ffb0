"""Fermi-Dirac occupation, electronic entropy and the bisection for mu (oracle).

The density matrix is the Fermi-Dirac weighted spectral integral of Eq. 2 with
chemical potential mu; the memory-saving workflow of Eq. 3 finds mu between
the two Green's-function passes "by bisection".  The reading used here:

  N(mu) = sum_jk w_jk f((eps_jk - mu) / kT) over the valid Ritz pairs
          (k < nu_eff of column j), target N(mu) = N_e;
  bracket [min eps - 40 kT, max eps + 40 kT] over the same pairs;
  step    mid = lo + (hi - lo) / 2;  N(mid) < N_e -> lo = mid, else hi = mid;
  stop    when hi - lo <= tol (1e-12 eV) and return lo + (hi - lo) / 2.
"""
from __future__ import annotations

import numpy as np


def fermi(x):
    """f(x) = 1 / (1 + e^x), evaluated without overflow on either side."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    pos = x > 0
    e = np.exp(-x[pos])
    out[pos] = e / (1.0 + e)
    out[~pos] = 1.0 / (1.0 + np.exp(x[~pos]))
    return out


def entropy(x):
    """s(f) = -[f ln f + (1 - f) ln(1 - f)] at f = f(x).

    With f and 1 - f = f(-x) both taken from x directly, ln f = -ln(1 + e^x)
    and ln(1 - f) = -ln(1 + e^-x); each is written with log1p of a number
    <= 1 so that neither side overflows.
    """
    x = np.asarray(x, dtype=np.float64)
    f = fermi(x)
    g = fermi(-x)  # 1 - f
    lse = np.log1p(np.exp(-np.abs(x)))  # ln(1 + e^-|x|)
    ln_f = -(np.maximum(x, 0.0) + lse)  # -ln(1 + e^x)
    ln_g = -(np.maximum(-x, 0.0) + lse)  # -ln(1 + e^-x)
    return -(f * ln_f + g * ln_g)


def electron_count(mu, eps, w, kT):
    return float(np.sum(w * fermi((eps - mu) / kT)))


def bracket(eps, kT):
    return float(np.min(eps)) - 40.0 * kT, float(np.max(eps)) + 40.0 * kT


def bisect_mu(eps, w, kT, n_electrons, tol=1e-12, max_steps=400):
    """Plain bisection on the electron count over the given (valid) pairs.

    Returns (mu, number of halvings).
    """
    eps = np.asarray(eps, dtype=np.float64).ravel()
    w = np.asarray(w, dtype=np.float64).ravel()
    lo, hi = bracket(eps, kT)
    steps = 0
    while hi - lo > tol and steps < max_steps:
        mid = lo + (hi - lo) / 2.0
        if electron_count(mid, eps, w, kT) < n_electrons:
            lo = mid
        else:
            hi = mid
        steps += 1
    return lo + (hi - lo) / 2.0, steps


def band_energy(mu, eps, w, kT):
    """(E_band, S_ent, N): sums of w f eps, w s(f) and w f over all terms."""
    x = (eps - mu) / kT
    f = fermi(x)
    return (float(np.sum(w * f * eps)), float(np.sum(w * entropy(x))), float(np.sum(w * f)))
