"""Molecular dynamics on the oracle's energies and forces (test infrastructure).

The letter's unit of work is one MD step: build H and S at the current
structure, compute the energy and the forces through the density matrix, and
move the atoms.  It runs only a couple of steps per benchmark and does not
name the integrator, so the reading taken here is velocity Verlet (Swope,
Andersen, Berens and Wilson, J. Chem. Phys. 76, 637 (1982)):
  v <- v + (dt / 2m) F(x);  x <- x + dt v;  F <- F(x);  v <- v + (dt / 2m) F(x)
with positions wrapped back into the box after each drift.

Units: Angstrom, fs, eV and amu.  One amu * (Angstrom / fs)^2 is
1.66053906660e-27 kg * 1e10 m^2/s^2 = 1.66053906660e-17 J, and one eV is
1.602176634e-19 J (CODATA 2018), hence AMU_A2_FS2_IN_EV below.

The forces come from the oracle's own solvers: the multiple Arnoldi columns
(mode K, with the Hellmann-Feynman reading of the density matrix) or the exact
eigendecomposition of the whole system (mode W).

Total energy.  A tight-binding total energy is the electronic (band) part plus
a short-range pair repulsion; the letter's models come with one, but their
parameters are not in it.  Without that term the band energy alone pulls
neighbouring atoms together without bound and a cell collapses within a few
fs, so the MD reading adds the form of Goodwin, Skinner and Pettifor
(Europhys. Lett. 9, 701 (1989)) that matches the (r0/r)^2 hoppings:
  E_rep = sum over pairs {I, K} closer than r_cut of
          phi(r) = phi0 (r0 / r)^m fc(r),   m = 4,
with the hoppings' r0 and smooth cutoff fc.  phi0 is the value that puts the
perfect diamond lattice (a = 3.567 A) at zero pressure in the mode-W total
energy at kT = 0.1 eV (derived in the tests from the oracle's own band energy).
The MD total energy is A_free + E_rep + E_kin.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

from . import neighbors as _nb
from . import sk as _sk
from . import solve as _solve

AMU_A2_FS2_IN_EV = 1.66053906660e-17 / 1.602176634e-19
REP_M = 4.0
REP_PHI0 = 13.18  # eV; zero-pressure value for perfect diamond (the tests re-derive it)


def pair_phi(r, phi0, m, p: _sk.SKParams):
    """phi(r) = phi0 (r0/r)^m fc(r) and dphi/dr."""
    fc, dfc = _sk.cutoff(r, p)
    g = phi0 * (p.r0 / r) ** m
    dg = -m * g / r
    return g * fc, dg * fc + g * dfc


def pair_repulsion(pos, cell, phi0=None, m=REP_M, p: _sk.SKParams = _sk.CARBON, atoms=None):
    """E_rep and the forces -dE_rep/dR_J of the given atoms (all if None).

    Each atom J sums phi over its neighbours K closer than r_cut (minimum
    image); a pair appears from both ends, so E_rep is half the sum over every
    atom.  With d = R_K - R_J, dphi(|d|)/dR_J = -phi'(r) d / r, so the force
    on J is sum_K phi'(r) d / r.  Returns (E_rep of all atoms, e, F) with e the
    per-atom halves and F the forces of `atoms` (rows in that order).
    """
    phi0 = REP_PHI0 if phi0 is None else phi0
    pos = np.asarray(pos, np.float64)
    cell = np.asarray(cell, np.float64)
    n = pos.shape[0]
    rows = np.arange(n) if atoms is None else np.asarray(atoms, np.int64)
    e_all = np.zeros(n)
    F = np.zeros((rows.size, 3))
    want = {int(J): i for i, J in enumerate(rows)}
    for J in range(n):
        if atoms is not None and J not in want:
            continue
        for K in _nb.neighbors_of(pos, cell, J, p.r_cut):
            d = _nb.min_image(pos[K] - pos[J], cell)
            r = float(np.sqrt(d @ d))
            ph, dph = pair_phi(r, phi0, m, p)
            e_all[J] += 0.5 * ph
            F[want[J]] += dph * d / r
    E = float(np.sum(e_all)) if atoms is None else None
    return E, e_all[rows], F


@dataclass
class Frame:
    pos: np.ndarray
    vel: np.ndarray
    F: np.ndarray
    E_pot: float  # A_free + E_rep
    E_kin: float
    mu: float
    E_band: float

    @property
    def E_total(self):
        return self.E_pot + self.E_kin


def kinetic_energy(vel, mass):
    """sum_I m |v_I|^2 / 2 in eV (vel in Angstrom/fs, mass in amu)."""
    return 0.5 * mass * float(np.sum(vel * vel)) * AMU_A2_FS2_IN_EV


def krylov_forces(struct, params=None, mode="K", workers=None, phi0=None):
    """Potential energy and forces from the multiple Arnoldi columns plus the
    pair repulsion: returns (A_free + E_rep, F, mu, E_band)."""
    p = _sk.CARBON if params is None else params

    def fn(pos):
        s = replace(struct, pos=np.asarray(pos, np.float64))
        sysm = _solve.build_system(s, params=p)
        r = _solve.solve(sysm, mode=mode, workers=workers, with_forces=True)
        E_rep, _, F_rep = pair_repulsion(s.pos, s.cell, phi0, p=p)
        return r.A_free + E_rep, r.F + F_rep, r.mu, r.E_band

    return fn


def krylov_exact_forces(struct, params=None, phi0=None, workers=None):
    """Potential energy and forces of the truncated multiple Arnoldi method
    with the forces as the exact derivative of its free energy (the reverse
    mode of the Krylov construction, oracle.adjoint) instead of the
    density-matrix reading, plus the pair repulsion: returns
    (A_free + E_rep, F, mu, E_band)."""
    from . import adjoint as _adj
    p = _sk.CARBON if params is None else params

    def fn(pos):
        s = replace(struct, pos=np.asarray(pos, np.float64))
        sysm = _solve.build_system(s, params=p)
        r = _solve.solve(sysm, workers=workers)
        geo = _solve.geometry(s, params=p)
        F = _adj.exact_forces_on(geo, np.arange(s.n_atoms), r.mu, workers=workers)
        E_rep, _, F_rep = pair_repulsion(s.pos, s.cell, phi0, p=p)
        return r.A_free + E_rep, F + F_rep, r.mu, r.E_band

    return fn


def exact_forces(struct, params=None, phi0=None):
    """The same from the exact solution of the whole system (mode W)."""
    p = _sk.CARBON if params is None else params

    def fn(pos):
        s = replace(struct, pos=np.asarray(pos, np.float64))
        sysm = _solve.build_system(s, params=p)
        ex = _solve.solve_exact(sysm)
        rho = _solve.pattern_of_dense(sysm, ex.rho)
        pi = _solve.pattern_of_dense(sysm, ex.pi)
        E_rep, _, F_rep = pair_repulsion(s.pos, s.cell, phi0, p=p)
        return ex.A_free + E_rep, _solve.forces(sysm, rho, pi) + F_rep, ex.mu, ex.E_band

    return fn


def wrap(pos, cell):
    return pos - cell[None, :] * np.floor(pos / cell[None, :])


def velocity_verlet(pos, vel, cell, force_fn, mass, dt, n_steps):
    """n_steps of velocity Verlet; returns the n_steps + 1 frames (frame 0: start)."""
    cell = np.asarray(cell, np.float64)
    x = np.array(pos, np.float64)
    v = np.array(vel, np.float64)
    A, F, mu, E = force_fn(x)
    frames = [Frame(x.copy(), v.copy(), F.copy(), A, kinetic_energy(v, mass), mu, E)]
    c = 0.5 * dt / (mass * AMU_A2_FS2_IN_EV)
    for _ in range(n_steps):
        v = v + c * F
        x = wrap(x + dt * v, cell)
        A, F, mu, E = force_fn(x)
        v = v + c * F
        frames.append(Frame(x.copy(), v.copy(), F.copy(), A, kinetic_energy(v, mass), mu, E))
    return frames
