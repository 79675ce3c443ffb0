"""Pins of the oracle's Krylov / Ritz / Green's-function / density steps.

Each test checks the multiple-Arnoldi oracle against something other than its
own formulas: the dense cluster limit (mode D) and the dense whole-system
inverse, the Lanczos-Gauss moment identity at S = I, invariants (weight
closure, basis independence), and the Lorentzian form of Eq. 2.
"""
import numpy as np
import pytest
import scipy.integrate as si
import scipy.linalg as sla

import gen
from oracle import fermi, krylov, neighbors as nb, sk, solve


def _small_cluster(r_small=3.2, k=2, atom=5, params=sk.CARBON):
    """A small cluster (the atoms within r_small of one atom) of config k."""
    s = gen.make(k)
    atoms = nb.cluster_of(s.pos, s.cell, atom, r_small)
    Hc, Sc = nb.cluster_matrices(s.pos, s.cell, atoms, params)
    l = 4 * int(np.searchsorted(atoms, atom))
    return Hc, Sc, l


def _cluster(k=2, atom=11, params=sk.CARBON):
    s = gen.make(k)
    atoms = nb.cluster_of(s.pos, s.cell, atom, s.r_cluster)
    Hc, Sc = nb.cluster_matrices(s.pos, s.cell, atoms, params)
    return Hc, Sc, 4 * int(np.searchsorted(atoms, atom))


def _euclidean_krylov(Hc, l, nu):
    """Independent basis of the same space: Euclidean Lanczos with full CGS2."""
    n = Hc.shape[0]
    Q = np.zeros((n, nu))
    Q[l, 0] = 1.0
    for k in range(1, nu):
        w = Hc @ Q[:, k - 1]
        for _ in range(2):
            w = w - Q[:, :k] @ (Q[:, :k].T @ w)
        Q[:, k] = w / np.linalg.norm(w)
    return Q


@pytest.mark.parametrize("beta", [0, 1, 2, 3])
def test_krylov_at_full_dimension_equals_dense_cluster(beta):
    Hc, Sc, l = _small_cluster()
    n = Hc.shape[0]
    rk = krylov.column_mode_k(Hc, Sc, l + beta, n)
    rd = krylov.column_mode_d(Hc, Sc, l + beta)
    for mu in (-1.0, 2.5, 6.0):
        a, pa = krylov.density_column(rk, mu, 0.1)
        b, pb = krylov.density_column(rd, mu, 0.1)
        np.testing.assert_allclose(a, b, atol=1e-10)
        np.testing.assert_allclose(pa, pb, atol=1e-9)
    z = np.array([0.3 + 0.7j, 5.0 - 0.2j, -12.0 + 1e-3j])
    np.testing.assert_allclose(krylov.green_column(rk, z), krylov.green_column(rd, z), atol=1e-8)


def test_galerkin_green_equals_dense_inverse():
    # cluster = whole cell and nu = M: the Galerkin column is (zS - H)^-1 e_j
    s = gen.make("tiny")
    sysm = solve.build_system(s)
    Hd, Sd = sysm.H.toarray(), sysm.S.toarray()
    cols = [0, 5, 101]
    z = [0.7 + 0.4j, -3.0 + 0.05j]
    ref = {zz: solve.green_exact(sysm, zz, cols) for zz in z}
    for i, j in enumerate(cols):
        res = krylov.column_mode_k(Hd, Sd, j, sysm.M)
        g = krylov.green_column(res, z)
        for iz, zz in enumerate(z):
            np.testing.assert_allclose(g[:, iz], ref[zz][:, i], atol=1e-9, rtol=1e-9)


def test_gauss_moments_at_unit_overlap():
    # S = I: the S-orthonormal Krylov process is plain Lanczos, h is
    # tridiagonal and the Ritz pairs are the nodes and weights of the Gauss
    # quadrature of the spectral measure of e_l:
    #   sum_k (w_k / g_s) eps_k^m = (H^m)_ll   for m <= 2 nu - 1.
    p = sk.SKParams(s_scale=0.0)
    Hc, Sc, l = _cluster(params=p)
    assert np.all(Sc == np.eye(Sc.shape[0]))
    nu = 12
    res = krylov.column_mode_k(Hc, Sc, l + 2, nu)
    assert res.nu_eff == nu
    off = np.triu(np.abs(res.h), 2)
    assert off.max() < 1e-12 * np.abs(res.h).max()
    norm = np.linalg.norm(Hc, 2)
    x = np.zeros(Hc.shape[0])
    x[l + 2] = 1.0
    v = x.copy()
    for m in range(2 * nu):
        moment = float(x @ v)
        quad = float(np.sum(res.w / krylov.G_SPIN * res.eps**m))
        assert abs(quad - moment) <= 1e-11 * norm**m, m
        v = Hc @ v
    # and one degree past exactness the identity fails, well above that tolerance
    miss = abs(float(np.sum(res.w / 2 * res.eps ** (2 * nu))) - float(x @ v))
    assert miss > 10 * 1e-11 * norm ** (2 * nu)


@pytest.mark.parametrize("atom,beta", [(11, 0), (11, 3), (200, 1)])
def test_weight_closure_and_basis_independence(atom, beta):
    Hc, Sc, l = _cluster(atom=atom)
    nu = 30
    rk = krylov.column_mode_k(Hc, Sc, l + beta, nu)
    # e_l lies in the Krylov space, so the weights add up to g_s
    assert abs(rk.w.sum() - krylov.G_SPIN) < 1e-12
    # another basis of the same space gives the same Ritz data
    Q = _euclidean_krylov(Hc, l + beta, nu)
    re = krylov.ritz(Hc, Sc, l + beta, Q)
    np.testing.assert_allclose(re.eps, rk.eps, atol=1e-12)
    np.testing.assert_allclose(re.w, rk.w, atol=1e-12)
    a, _ = krylov.density_column(rk, 3.0, 0.1)
    b, _ = krylov.density_column(re, 3.0, 0.1)
    np.testing.assert_allclose(a, b, atol=1e-13)
    # the projected overlap of the S-orthonormal basis is the identity
    np.testing.assert_allclose(rk.s, np.eye(nu), atol=1e-13)


def test_density_is_lorentzian_limit_of_eq2():
    # Eq. 2 with a finite broadening eta, integrated numerically, tends to the
    # Ritz-spectrum sum; the error is first order in eta.
    Hc, Sc, l = _small_cluster()
    res = krylov.column_mode_k(Hc, Sc, l, 14)
    mu, kT = 3.0, 0.4
    rho, _ = krylov.density_column(res, mu, kT)
    i = int(np.argmax(np.abs(rho)))
    i2 = int(np.argsort(np.abs(rho))[-3])
    errs = []
    for eta in (4e-2, 2e-2):
        def integrand(e, row):
            g = krylov.green_column(res, e + 1j * eta)[row, 0]
            return -krylov.G_SPIN / np.pi * fermi.fermi((e - mu) / kT) * g.imag
        lo, hi = res.eps.min() - 60.0, res.eps.max() + 60.0
        vals = []
        for row in (i, i2):
            v, _ = si.quad(integrand, lo, hi, args=(row,), points=list(res.eps), limit=2000,
                           epsabs=1e-12, epsrel=1e-12)
            vals.append(v)
        errs.append(max(abs(vals[0] - rho[i]), abs(vals[1] - rho[i2])))
    assert errs[0] < 0.05 and errs[1] < 0.6 * errs[0]


def test_fermi_and_entropy_identities():
    x = np.linspace(-800.0, 800.0, 4001)
    f = fermi.fermi(x)
    assert np.all(np.isfinite(f)) and f.min() >= 0.0 and f.max() <= 1.0
    np.testing.assert_allclose(f + fermi.fermi(-x), 1.0, atol=1e-15)
    s = fermi.entropy(x)
    assert np.all(np.isfinite(s)) and s.min() >= 0.0
    assert abs(fermi.entropy(np.array([0.0]))[0] - np.log(2.0)) < 1e-15
    np.testing.assert_allclose(s, fermi.entropy(-x), atol=1e-15)
    xm = np.linspace(-20, 20, 81)
    fm = fermi.fermi(xm)
    direct = -(fm * np.log(fm) + (1 - fm) * np.log(1 - fm))
    np.testing.assert_allclose(fermi.entropy(xm), direct, atol=1e-12)


def test_bisection_closed_form():
    # two levels symmetric about 0.5 holding half the electrons: mu = 0.5
    eps = np.array([0.0, 1.0])
    w = np.array([2.0, 2.0])
    mu, steps = fermi.bisect_mu(eps, w, 0.1, 2.0)
    assert abs(mu - 0.5) < 1e-12 and steps > 30
    # a single level with weight 2 holding n electrons: f(x) = n/2
    mu, _ = fermi.bisect_mu(np.array([1.3]), np.array([2.0]), 0.2, 0.5)
    assert abs(mu - (1.3 - 0.2 * np.log(2.0 / 0.5 - 1.0))) < 1e-11
