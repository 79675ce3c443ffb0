"""Pins of the oracle's exact gradient of the truncated-Krylov free energy.

- one column's reverse-mode gradient against central differences of the same
  function along a random symmetric perturbation of the cluster pattern;
- the total forces against central differences of the oracle's own mode-K
  free energy (mu re-bisected at every displaced geometry, i.e. at fixed N),
  on the 61-atom whole-cell cell at nu = 12 < n_C = 244, where the
  Hellmann-Feynman forces differ from the difference quotients by a tenth of
  an eV/A or more, so the pin separates the two.
"""
from dataclasses import replace

import numpy as np
import pytest
import torch

from gen import structures as gs
from oracle import adjoint
from oracle import neighbors as nb
from oracle import solve as so


def test_column_gradient_matches_differences():
    s = gs.make("mini_vac")
    J = 17
    atoms = nb.cluster_of(s.pos, s.cell, J, s.r_cluster)
    Hc, Sc = nb.cluster_matrices(s.pos, s.cell, atoms)
    l = 4 * int(np.searchsorted(atoms, J)) + 1
    mu, kT, nu = 3.0, 0.1, 20
    _, gH, gS = adjoint.column_gradient(Hc, Sc, l, nu, mu, kT)
    rng = np.random.default_rng(1)
    E = rng.normal(size=Hc.shape) * (Hc != 0)
    E = 0.5 * (E + E.T)
    F = rng.normal(size=Sc.shape) * (Sc != 0)
    F = 0.5 * (F + F.T)
    ad = float((gH * E).sum() + (gS * F).sum())
    h = 1e-5
    with torch.no_grad():
        op = float(adjoint.column_omega(torch.tensor(Hc + h * E), torch.tensor(Sc + h * F), l, nu,
                                        mu, kT))
        om = float(adjoint.column_omega(torch.tensor(Hc - h * E), torch.tensor(Sc - h * F), l, nu,
                                        mu, kT))
    fd = (op - om) / (2 * h)
    assert abs(ad - fd) <= 1e-7 * abs(fd)


@pytest.fixture(scope="module")
def tiny():
    s = gs.make("tiny")  # whole-cell clusters, nu = 12
    sysm = so.build_system(s)
    r = so.solve(sysm, with_forces=True)
    return s, sysm, r, adjoint.exact_forces(sysm, r.mu)


def test_exact_forces_match_differences_of_the_free_energy(tiny):
    s, sysm, r, Fx = tiny
    assert s.nu < 4 * s.n_atoms
    h = 1e-5
    for I, c in ((3, 0), (17, 1), (40, 2)):
        xp, xm = s.pos.copy(), s.pos.copy()
        xp[I, c] += h
        xm[I, c] -= h
        Ap = so.solve(so.build_system(replace(s, pos=xp))).A_free
        Am = so.solve(so.build_system(replace(s, pos=xm))).A_free
        fd = -(Ap - Am) / (2 * h)
        assert abs(Fx[I, c] - fd) < 1e-5
        assert abs(r.F[I, c] - fd) > 0.1  # the Hellmann-Feynman reading is not the gradient here
    assert np.abs(Fx.sum(axis=0)).max() < 1e-9  # translation invariance


def test_forces_of_selected_atoms_equal_the_full_sum(tiny):
    # the pooled driver over the clusters that hold the chosen atoms gives
    # the same forces as the sum over every column
    s, sysm, r, Fx = tiny
    pick = np.array([0, 17, 40])
    Fp = adjoint.exact_forces_on(so.geometry(s), pick, r.mu, workers=4)
    np.testing.assert_allclose(Fp, Fx[pick], rtol=0, atol=1e-12)
