"""Pins of the oracle's MD step (velocity Verlet on A_free + E_rep).

Energy conservation with the exact (mode W) forces ties the forces, the pair
repulsion, the integrator and the unit constant together: velocity Verlet's
energy error is second order in dt, so halving dt must divide the largest
excursion of the total energy by four, which fails for forces that are not
-grad E_pot (a wrong sign, scale or missing term) or for a wrong amu/eV
constant.
"""
from dataclasses import replace

import numpy as np
import pytest

from gen import structures as gs
from oracle import md
from oracle import solve as so

MASS_C = 12.011  # amu
KB = 8.617333262e-5  # eV / K


def _velocities(s, T, seed):
    return gs.random_velocities(s.n_atoms, np.sqrt(KB * T / (MASS_C * md.AMU_A2_FS2_IN_EV)), seed)


def test_unit_constant():
    # 1 amu (A/fs)^2 = 1.66053906660e-27 kg * 1e10 m^2 s^-2 in eV
    assert md.AMU_A2_FS2_IN_EV == pytest.approx(103.642696, rel=1e-8)


def test_pair_phi_closed_form_and_cutoff():
    p = so._sk.CARBON
    for r in (1.2, 1.54, 1.9):  # below r_on: no cutoff
        ph, dph = md.pair_phi(r, 2.0, 4.0, p)
        assert ph == pytest.approx(2.0 * (p.r0 / r) ** 4, rel=1e-14)
        assert dph == pytest.approx(-4.0 * 2.0 * p.r0**4 / r**5, rel=1e-14)
    assert md.pair_phi(p.r_cut + 1e-9, 2.0, 4.0, p) == (0.0, 0.0)
    # smooth through the cutoff region: derivative agrees with a difference quotient
    for r in (2.1, 2.3, 2.55):
        h = 1e-6
        fd = (md.pair_phi(r + h, 2.0, 4.0, p)[0] - md.pair_phi(r - h, 2.0, 4.0, p)[0]) / (2 * h)
        assert md.pair_phi(r, 2.0, 4.0, p)[1] == pytest.approx(fd, rel=1e-7, abs=1e-10)


def test_pair_repulsion_forces_are_minus_gradient():
    s = gs.make("tiny")
    E, e, F = md.pair_repulsion(s.pos, s.cell)
    assert E == pytest.approx(e.sum(), rel=1e-14)
    assert np.abs(F.sum(axis=0)).max() < 1e-10  # pair forces cancel
    rng = np.random.default_rng(3)
    h = 1e-6
    for I in rng.choice(s.n_atoms, 4, replace=False):
        for c in range(3):
            xp = s.pos.copy()
            xm = s.pos.copy()
            xp[I, c] += h
            xm[I, c] -= h
            fd = (md.pair_repulsion(xp, s.cell)[0] - md.pair_repulsion(xm, s.cell)[0]) / (2 * h)
            assert F[I, c] == pytest.approx(-fd, abs=1e-6)
    # the subset form returns the same rows
    sel = np.array([5, 0, 17])
    _, e2, F2 = md.pair_repulsion(s.pos, s.cell, atoms=sel)
    np.testing.assert_allclose(F2, F[sel], rtol=0, atol=0)
    np.testing.assert_allclose(e2, e[sel], rtol=0, atol=0)


def test_repulsion_calibration_zero_pressure():
    """REP_PHI0 puts perfect diamond at zero pressure in the mode-W total energy."""
    base = gs.make_structure(cells=(2, 2, 2), sigma=0.0, nu=30, r_cluster=0.0, seed=1,
                             name="perfect")

    def A_band(scale):
        s = replace(base, pos=base.pos * scale, cell=base.cell * scale)
        return so.solve_exact(so.build_system(s)).A_free

    def E_rep(scale, phi0):
        return md.pair_repulsion(base.pos * scale, base.cell * scale, phi0)[0]

    h = 1e-4
    dA = (A_band(1 + h) - A_band(1 - h)) / (2 * h)
    dR = (E_rep(1 + h, 1.0) - E_rep(1 - h, 1.0)) / (2 * h)
    assert md.REP_PHI0 == pytest.approx(-dA / dR, rel=1e-3)
    # and the lattice is a minimum of the total energy along the breathing mode
    E = [A_band(x) + E_rep(x, md.REP_PHI0) for x in (0.98, 1.0, 1.02)]
    assert E[1] < E[0] and E[1] < E[2]


@pytest.fixture(scope="module")
def tiny_runs():
    s = gs.make("tiny")
    v0 = _velocities(s, 300.0, 7)
    fn = md.exact_forces(s)
    runs = {dt: md.velocity_verlet(s.pos, v0, s.cell, fn, MASS_C, dt, int(round(4.0 / dt)))
            for dt in (0.5, 0.25)}
    return s, v0, fn, runs


def test_md_energy_error_is_second_order(tiny_runs):
    _, _, _, runs = tiny_runs
    dev = {}
    for dt, fr in runs.items():
        E = np.array([f.E_total for f in fr])
        dev[dt] = np.abs(E - E[0]).max()
    # the ions do work: the kinetic energy changes by far more than the error
    dK = abs(runs[0.25][-1].E_kin - runs[0.25][0].E_kin)
    assert dK > 100 * dev[0.25]
    assert 3.5 < dev[0.5] / dev[0.25] < 4.5
    assert dev[0.25] < 0.05


def test_md_momentum_and_first_step(tiny_runs):
    s, v0, _, runs = tiny_runs
    fr = runs[0.5]
    for f in fr:
        assert np.abs(f.vel.sum(axis=0)).max() < 1e-12
    # first drift: x1 = x0 + dt v0 + dt^2 F0 / (2 m)
    dt = 0.5
    expect = s.pos + dt * v0 + dt * dt * fr[0].F / (2 * MASS_C * md.AMU_A2_FS2_IN_EV)
    d = fr[1].pos - expect
    d -= s.cell * np.rint(d / s.cell)
    assert np.abs(d).max() < 1e-12


def test_md_time_reversible(tiny_runs):
    s, v0, fn, runs = tiny_runs
    fwd = runs[0.5][:7]  # six steps
    back = md.velocity_verlet(fwd[-1].pos, -fwd[-1].vel, s.cell, fn, MASS_C, 0.5, 6)
    d = back[-1].pos - s.pos
    d -= s.cell * np.rint(d / s.cell)
    assert np.abs(d).max() < 1e-9
    assert np.abs(back[-1].vel + v0).max() < 1e-9


def test_truncated_krylov_md_conserves_energy_only_with_exact_forces():
    # the 61-atom whole cell at nu = 12 (244 orbitals): with the exact
    # gradient of the truncated method the energy error of velocity Verlet is
    # second order in dt (ratio 4 on halving dt, compared at the common
    # times); with the forces through rho the missing part of the gradient
    # does work along the path, an error that does not shrink with dt.  The
    # steps are 0.25 and 0.125 fs: at 0.5 fs this cell is not yet in the
    # asymptotic range of the integrator
    s = gs.make("tiny")
    v0 = _velocities(s, 300.0, 7)
    rms = {}
    for kind, fn in (("exact", md.krylov_exact_forces(s)), ("rho", md.krylov_forces(s))):
        dE = {}
        for dt in (0.25, 0.125):
            fr = md.velocity_verlet(s.pos, v0, s.cell, fn, MASS_C, dt, int(round(1.0 / dt)))
            E = np.array([f.E_total for f in fr])
            dE[dt] = E - E[0]
        rms[kind] = (np.sqrt(np.mean(dE[0.25][1:] ** 2)), np.sqrt(np.mean(dE[0.125][2::2] ** 2)))
    ratio_exact = rms["exact"][0] / rms["exact"][1]
    ratio_rho = rms["rho"][0] / rms["rho"][1]
    assert 3.5 < ratio_exact < 4.8, ratio_exact
    assert 0.8 < ratio_rho < 1.25, ratio_rho
    assert rms["rho"][1] > 20 * rms["exact"][1]
