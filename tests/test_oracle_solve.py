"""System-level pins of the oracle: electron count, energy routes, the exact
regime against the whole-system solution, and forces against finite
differences of the free energy."""
import numpy as np
import pytest

import gen
from oracle import fermi, krylov, solve


def _half_filled_small():
    # 2x2x2 cell with half of the sites removed: 32 atoms, M = 128, so a
    # Krylov space of dimension M is affordable in the plain oracle.
    s = gen.make_structure(cells=(2, 2, 2), vacancy_frac=0.5, sigma=0.05, seed=4242,
                           nu=128, r_cluster=0.0)
    return s


@pytest.fixture(scope="module")
def cfg1():
    s = gen.make(1)
    sysm = solve.build_system(s)
    return sysm, solve.solve(sysm, workers=4)


def test_electron_count_and_two_energy_routes(cfg1):
    sysm, r = cfg1
    # N(mu) hits N_e; Tr(rho S) reproduces it on the pattern
    assert abs(r.N - sysm.n_electrons) < 1e-9
    assert abs(float(sysm.S.data @ r.rho) - sysm.n_electrons) < 1e-9
    # E_band = sum w f eps = Tr(rho H), because e_l^T H V = sqrt(S_ll) e_1^T h
    assert abs(float(sysm.H.data @ r.rho) - r.E_band) < 1e-9 * abs(r.E_band)
    # every column's weights close to g_s
    e, w = solve.valid_terms(r.cd)
    sums = np.array([r.cd["w"][i, :r.cd["nu_eff"][i]].sum() for i in range(sysm.M)])
    np.testing.assert_allclose(sums, krylov.G_SPIN, atol=1e-12)
    assert r.cd["nu_eff"].min() == sysm.nu


@pytest.fixture(scope="module")
def exact_small():
    s = _half_filled_small()
    sysm = solve.build_system(s)
    return sysm, solve.solve(sysm, workers=8, with_forces=True), solve.solve_exact(sysm)


def test_exact_regime_matches_whole_system(exact_small):
    sysm, rk, ex = exact_small
    assert abs(rk.mu - ex.mu) < 1e-8
    assert abs(rk.E_band - ex.E_band) < 1e-9 * sysm.n_atoms
    assert abs(rk.A_free - ex.A_free) < 1e-9 * sysm.n_atoms
    np.testing.assert_allclose(rk.rho, solve.pattern_of_dense(sysm, ex.rho), atol=1e-10)
    np.testing.assert_allclose(rk.pi, solve.pattern_of_dense(sysm, ex.pi), atol=1e-9)
    np.testing.assert_allclose(ex.rho, ex.rho.T, atol=1e-12)
    # Krylov-exact rho is symmetric on the pattern as well
    rho_t = solve.pattern_of_dense(sysm, ex.rho.T)
    np.testing.assert_allclose(rk.rho, rho_t, atol=1e-10)


def test_forces_match_finite_differences_in_exact_regime(exact_small):
    sysm, rk, ex = exact_small
    # F from rho and pi (Hellmann-Feynman + Pulay through S) against central
    # differences of the grand potential A - mu N at the fixed mu of the
    # reference state (its gradient equals that of the Mermin free energy A at
    # fixed electron number, and it carries no bisection noise)
    def free_energy(pos):
        s2 = gen.Structure(pos=pos, cell=sysm.cell, nu=sysm.nu, r_cluster=0.0)
        return solve.solve_exact(solve.build_system(s2), mu=ex.mu).omega
    h = 1e-5
    rng = np.random.default_rng(3)
    F_exact = solve.forces(sysm, solve.pattern_of_dense(sysm, ex.rho),
                           solve.pattern_of_dense(sysm, ex.pi))
    np.testing.assert_allclose(rk.F, F_exact, atol=1e-8)
    for _ in range(4):
        I = int(rng.integers(sysm.n_atoms))
        c = int(rng.integers(3))
        pp = sysm.pos.copy()
        pm = sysm.pos.copy()
        pp[I, c] += h
        pm[I, c] -= h
        fd = -(free_energy(pp) - free_energy(pm)) / (2 * h)
        assert abs(fd - F_exact[I, c]) < 1e-7, (I, c, fd, F_exact[I, c])


def test_forces_sum_to_zero_and_vanish_in_perfect_crystal():
    s = gen.make("tiny")
    sysm = solve.build_system(s)
    r = solve.solve(sysm, workers=4, with_forces=True)
    assert np.abs(r.F.sum(axis=0)).max() < 1e-10
    assert np.abs(r.F).max() > 1e-3
    # perfect diamond: every atom sits on a tetrahedral site, no force.  The
    # 2x2x2 cell has only 30 distinct levels, so nu is kept well below the
    # invariant dimension of each column; near it the Krylov tail is decided
    # by rounding and no longer respects the symmetry.
    p = gen.make_structure(cells=(2, 2, 2), sigma=0.0, seed=1, nu=10, r_cluster=0.0)
    sp = solve.build_system(p)
    rp = solve.solve(sp, workers=4, with_forces=True)
    assert np.abs(rp.F).max() < 1e-9


def test_mu_residual_small_and_bisection_steps(cfg1):
    sysm, r = cfg1
    e, w = solve.valid_terms(r.cd)
    n = fermi.electron_count(r.mu, e, w, sysm.kT)
    assert abs(n - sysm.n_electrons) < 1e-9
    lo, hi = fermi.bracket(e, sysm.kT)
    mu2, steps = fermi.bisect_mu(e, w, sysm.kT, sysm.n_electrons)
    assert mu2 == r.mu and steps == int(np.ceil(np.log2((hi - lo) / 1e-12)))
