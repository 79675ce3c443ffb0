"""Pins of the oracle's crystal orbital Hamiltonian populations (Eqs. 4-8):
the sigma/pi split of the two-center blocks against the textbook forms, the
sum rule of Eq. 6, the decomposition of Eq. 8, pair symmetry in the exact
regime, the sign of the bond populations in perfect diamond, and the
energy-resolved COHP against the Galerkin column of the Krylov code and, in
the exact regime, against the dense resolvent (zS - H)^-1 of Eq. 1."""
import numpy as np
import pytest

import gen
from oracle import neighbors, sk, solve


def test_split_blocks_along_z_and_sum():
    p = sk.CARBON
    r = 1.5
    u = (p.r0 / r) ** 2  # fc = 1 below r_on
    hs, hp = sk.hopping_sigma_pi(np.array([0.0, 0.0, r]), p)
    # pi: only the px-px and py-py integrals, V_pp_pi each
    exp_p = np.zeros((4, 4))
    exp_p[1, 1] = exp_p[2, 2] = p.v_pp_pi * u
    np.testing.assert_allclose(hp, exp_p, rtol=1e-15, atol=0)
    # sigma: ss, s-pz, pz-s and pz-pz
    exp_s = np.zeros((4, 4))
    exp_s[0, 0] = p.v_ss_sigma * u
    exp_s[0, 3] = p.v_sp_sigma * u
    exp_s[3, 0] = -p.v_sp_sigma * u
    exp_s[3, 3] = p.v_pp_sigma * u
    np.testing.assert_allclose(hs, exp_s, rtol=1e-15, atol=0)
    # any direction: the parts add up to the full block
    rng = np.random.default_rng(3)
    for _ in range(5):
        d = rng.normal(size=3)
        d *= rng.uniform(1.3, 2.5) / np.linalg.norm(d)
        full, _ = sk.pair_blocks(d, p)
        hs, hp = sk.hopping_sigma_pi(d, p)
        np.testing.assert_allclose(hs + hp, full, rtol=0, atol=1e-14)


@pytest.fixture(scope="module")
def cfg1():
    s = gen.make(1)
    sysm = solve.build_system(s)
    return sysm, solve.solve(sysm, workers=4)


def test_sum_rule_and_decomposition(cfg1):
    sysm, r = cfg1
    B, Bs, Bp = solve.icohp(sysm, r.rho)
    nblk = sum(len(k) for k in sysm.rows)
    assert B.shape == (nblk,)
    # Eq. 6: the populations add up to the band energy
    assert abs(B.sum() - r.E_band) < 1e-10 * abs(r.E_band)
    # Eq. 8 on the off-diagonal blocks (the model's H is sigma + pi there)
    diag = np.concatenate([np.asarray(k) == J for J, k in enumerate(sysm.rows)])
    np.testing.assert_allclose((Bs + Bp)[~diag], B[~diag], rtol=0, atol=1e-12)
    assert np.all(Bs[diag] == 0.0) and np.all(Bp[diag] == 0.0)


def test_pair_symmetry_in_exact_regime():
    # whole-system rho is symmetric, so B_KJ = B_JK for every pair
    s = gen.make_structure(cells=(2, 2, 2), vacancy_frac=0.5, sigma=0.05, seed=4242,
                           nu=128, r_cluster=0.0)
    sysm = solve.build_system(s)
    ex = solve.solve_exact(sysm)
    B, Bs, Bp = solve.icohp(sysm, solve.pattern_of_dense(sysm, ex.rho))
    index = {}
    b = 0
    for J, ks in enumerate(sysm.rows):
        for K in ks:
            index[(J, int(K))] = b
            b += 1
    for (J, K), b in index.items():
        t = index[(K, J)]
        assert abs(B[b] - B[t]) < 1e-11
        assert abs(Bs[b] - Bs[t]) < 1e-11
        assert abs(Bp[b] - Bp[t]) < 1e-11
    assert abs(B.sum() - ex.E_band) < 1e-10 * abs(ex.E_band)


def test_bonds_of_perfect_diamond():
    # every nearest-neighbour pair is equivalent and bonding (negative
    # population, mostly sigma); second neighbours form one class as well
    s = gen.make_structure(cells=(2, 2, 2), sigma=0.0, seed=1, nu=10, r_cluster=0.0)
    sysm = solve.build_system(s)
    ex = solve.solve_exact(sysm)
    B, Bs, Bp = solve.icohp(sysm, solve.pattern_of_dense(sysm, ex.rho))
    dist = []
    for J, ks in enumerate(sysm.rows):
        for K in ks:
            d = neighbors.min_image(sysm.pos[int(K)] - sysm.pos[J], sysm.cell)
            dist.append(np.linalg.norm(d))
    dist = np.array(dist)
    nn = np.abs(dist - np.sqrt(3) / 4 * 3.567) < 1e-6
    assert nn.sum() == 4 * sysm.n_atoms
    np.testing.assert_allclose(B[nn], B[nn][0], rtol=0, atol=1e-10)
    np.testing.assert_allclose(Bs[nn], Bs[nn][0], rtol=0, atol=1e-10)
    # bonding, and sigma-dominated: the sp3 bond is a sigma bond
    assert B[nn][0] < -1.0
    assert Bs[nn][0] < 0.0 and abs(Bs[nn][0]) > 10.0 * abs(Bp[nn][0])
    nnn = np.abs(dist - np.sqrt(2) / 2 * 3.567) < 1e-6
    if nnn.any():
        np.testing.assert_allclose(B[nnn], B[nnn][0], rtol=0, atol=1e-10)


def test_cohp_against_galerkin_columns(cfg1):
    # the block-wise COHP against G taken column by column from the Krylov
    # code's own Galerkin column (a different indexing route: cluster rows of
    # the column atom instead of pattern rows)
    from oracle import krylov
    sysm, r = cfg1
    e = np.array([-8.0, -3.0, 0.5, 4.0])
    eta = 0.05
    C = solve.cohp(sysm, r.cd, e, eta)
    assert C.shape == (sum(len(k) for k in sysm.rows), e.size)
    atoms = neighbors.cluster_of(sysm.pos, sysm.cell, 0, sysm.r_cluster)
    Hc, Sc = neighbors.cluster_matrices(sysm.pos, sysm.cell, atoms, sysm.params)
    H = sysm.H.toarray()
    b = 0
    for J in range(3):
        for t, K in enumerate(sysm.rows[J]):
            ref = np.zeros(e.size)
            for a in range(4):
                res = krylov.column_mode_k(Hc, Sc, 4 * int(np.searchsorted(atoms, J)) + a, sysm.nu)
                G = krylov.green_column(res, e + 1j * eta)
                kl = int(np.searchsorted(atoms, K))
                for c in range(4):
                    ref += -(krylov.G_SPIN / np.pi) * H[4 * J + a, 4 * K + c] * G[4 * kl + c].imag
            np.testing.assert_allclose(C[b], ref, rtol=1e-11, atol=1e-11)
            b += 1


def test_cohp_exact_regime_equals_resolvent():
    # nu = M on the whole cell: the Galerkin G is (zS - H)^-1 itself (Eq. 1)
    s = gen.make_structure(cells=(2, 2, 2), vacancy_frac=0.5, sigma=0.05, seed=4242,
                           nu=128, r_cluster=0.0)
    sysm = solve.build_system(s)
    cd = solve.column_data(sysm, workers=8)
    e = np.array([-6.0, 1.0])
    eta = 0.1
    C = solve.cohp(sysm, cd, e, eta)
    H, S = sysm.H.toarray(), sysm.S.toarray()
    ref = []
    Gs = [np.linalg.solve(z * S - H, np.eye(H.shape[0])) for z in e + 1j * eta]
    for J in range(sysm.n_atoms):
        for K in sysm.rows[J]:
            row = []
            for G in Gs:
                blk = G[4 * int(K):4 * int(K) + 4, 4 * J:4 * J + 4]  # G_{Kb;Ja}
                hb = H[4 * J:4 * J + 4, 4 * int(K):4 * int(K) + 4]  # H_{Ja;Kb}
                row.append(-(2.0 / np.pi) * np.sum(hb * blk.T).imag)
            ref.append(row)
    np.testing.assert_allclose(C, np.array(ref), rtol=0, atol=1e-9)
