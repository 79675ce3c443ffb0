"""Pins of the oracle's COCG Green's-function columns.

- the converged columns equal dense solves of (z S_C - H_C) x = e_l;
- on a whole-cell cluster they are the columns of (z S - H)^-1 of Eq. 1 and
  the Green's function is complex symmetric, G_ij = G_ji;
- for real z below the spectrum A = z S - H is negative definite and real,
  and every COCG iterate is the textbook CG iterate (SciPy's cg on -A), which
  fixes the alpha and beta recurrences and the bilinear (unconjugated) form.
"""
import numpy as np
import pytest
from scipy.sparse.linalg import cg

from gen import structures as gs
from oracle import cocg
from oracle import solve as so

TOL = 1e-10


@pytest.fixture(scope="module")
def mini():
    s = gs.make("mini_vac")
    return s, so.build_system(s)


@pytest.fixture(scope="module")
def tiny():
    s = gs.make("tiny")
    return s, so.build_system(s)


def test_converged_columns_equal_dense_cluster_solves(mini):
    _, sysm = mini
    z = [-6.0 + 0.3j, 1.0 + 0.5j, 4.0 + 0.1j]
    cols = [3, 130]
    G, it = cocg.green_columns_cocg(sysm, cols, z, tol=TOL)
    D = cocg.green_columns_dense(sysm, cols, z)
    assert np.all(it > 0)
    for i in range(len(cols)):
        for q in range(len(z)):
            assert np.abs(G[i][q] - D[i][q]).max() < 1e-9


def test_whole_cell_columns_are_the_resolvent_and_symmetric(tiny):
    s, sysm = tiny
    z = np.array([0.5 + 0.2j, -3.0 + 0.05j])
    cols = [0, 7, 41]
    G, it = cocg.green_columns_cocg(sysm, cols, z, tol=1e-12, max_iter=5000)
    assert np.all(it > 0)
    for q, zq in enumerate(z):
        ex = so.green_exact(sysm, zq, cols)  # dense (z S - H)^-1 columns of the whole system
        for i in range(len(cols)):
            # whole-cell cluster: local order is the global order
            assert np.abs(G[i][q] - ex[:, i]).max() < 1e-9
        # G_ij = G_ji (A^T = A)
        for a in range(len(cols)):
            for b in range(len(cols)):
                assert abs(G[a][q][cols[b]] - G[b][q][cols[a]]) < 1e-9


def test_real_shift_below_spectrum_is_textbook_cg(mini):
    _, sysm = mini
    _, Hc, Sc, l = cocg.cluster_problem(sysm, 17)
    emin = np.linalg.eigvalsh(np.linalg.solve(Sc, Hc)).min()
    z = emin - 2.0
    A = z * Sc - Hc  # negative definite
    b = np.zeros(Hc.shape[0])
    b[l] = 1.0
    for k in (1, 2, 5, 12):
        xk, _ = cocg.cocg(A, b, tol=1e-300, max_iter=k)
        ref, _ = cg(-A, -b, x0=np.zeros_like(b), rtol=1e-300, atol=0.0, maxiter=k)
        assert np.abs(xk.imag).max() == 0.0
        np.testing.assert_allclose(xk.real, ref, rtol=1e-9, atol=1e-13)


def test_unconverged_and_breakdown_report_minus_one():
    A = np.diag([1.0, 2.0, 3.0, 4.0]).astype(np.complex128)
    b = np.ones(4)
    _, it = cocg.cocg(A, b, tol=1e-14, max_iter=2)
    assert it == -1
    # <b, b> = 0 for b = (1, i): rho vanishes at the start, <p, A p> = 0 for A = I
    _, it = cocg.cocg(np.eye(2, dtype=np.complex128), np.array([1.0, 1j]), tol=1e-12, max_iter=5)
    assert it == -1
