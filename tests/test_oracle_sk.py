"""Pins of the oracle's Slater-Koster model against closed forms and invariants.

The tight-binding H and S must be sparse, real-symmetric with S positive
definite (problem statement around Eq. 1).  None of these tests re-types the
block formulas: each checks a consequence that a sign, index or factor error
in them would break.
"""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.spatial.transform import Rotation

import gen
from oracle import neighbors as nb
from oracle import sk


def _dense(pos, cell, params=sk.CARBON):
    H, S, _ = nb.build_csr(pos, cell, params)
    return H.toarray(), S.toarray()


def _dimer(d, params=sk.CARBON):
    pos = np.array([[50.0, 50.0, 50.0], [50.0, 50.0, 50.0]]) + np.vstack([np.zeros(3), d])
    return _dense(pos, np.array([100.0, 100.0, 100.0]), params)


def _spectrum(H, S):
    return sla.eigh(H, S, eigvals_only=True)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dimer_pi_levels_closed_form(seed):
    # The two pi bonds of a dimer give the 2x2 pencil [[Ep, t], [t, Ep]] with
    # overlap [[1, s], [s, 1]]: levels (Ep + t)/(1 + s) and (Ep - t)/(1 - s),
    # each twice.
    rng = np.random.default_rng(seed)
    r = rng.uniform(1.3, 2.55)
    u = rng.normal(size=3)
    d = r * u / np.linalg.norm(u)
    H, S = _dimer(d)
    ev = _spectrum(H, S)
    p = sk.CARBON
    rad, _ = sk.radial(r, p)
    t = p.v_pp_pi * rad
    s = p.s_scale * p.s_signs[3] * rad
    for lev in [(p.ep + t) / (1 + s), (p.ep - t) / (1 - s)]:
        hits = np.sum(np.abs(ev - lev) < 1e-10)
        assert hits == 2, (lev, ev)


def test_dimer_sigma_levels_without_sp_coupling():
    # With the s-p bond integrals switched off the sigma system splits into an
    # s-s and a p-p(sigma) pencil with closed-form levels.
    p = sk.SKParams(v_sp_sigma=0.0, s_signs=(-1.0, 0.0, 1.0, -1.0))
    r = 1.7
    d = r * np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
    H, S = _dimer(d, p)
    ev = _spectrum(H, S)
    rad, _ = sk.radial(r, p)
    pairs = [(p.es, p.v_ss_sigma * rad, p.s_scale * p.s_signs[0] * rad),
             (p.ep, p.v_pp_sigma * rad, p.s_scale * p.s_signs[2] * rad)]
    for e0, t, s in pairs:
        for lev in [(e0 + t) / (1 + s), (e0 - t) / (1 - s)]:
            assert np.min(np.abs(ev - lev)) < 1e-10


def test_dimer_full_spectrum_is_rotation_invariant():
    base = np.array([1.62, 0.0, 0.0])
    ev0 = _spectrum(*_dimer(base))
    for seed in range(4):
        R = Rotation.random(random_state=seed).as_matrix()
        ev = _spectrum(*_dimer(R @ base))
        np.testing.assert_allclose(ev, ev0, atol=1e-12)


def test_cluster_spectrum_rotation_translation_invariant():
    # a noisy chunk of diamond in a large box, so that nothing wraps
    pos, _ = gen.diamond_sites(2, 2, 2)
    rng = np.random.default_rng(7)
    pos = pos[:30] + rng.normal(0.0, 0.05, size=(30, 3))
    cell = np.array([200.0, 200.0, 200.0])
    centre = pos.mean(axis=0)
    ev0 = _spectrum(*_dense(pos - centre + 100.0, cell))
    for seed in range(3):
        R = Rotation.random(random_state=10 + seed).as_matrix()
        shift = rng.uniform(60.0, 140.0, size=3)
        moved = (pos - centre) @ R.T + shift
        ev = _spectrum(*_dense(moved, cell))
        np.testing.assert_allclose(ev, ev0, atol=1e-11)


def test_diamond_gamma_point_closed_form():
    # Perfect diamond with nearest neighbours only (cutoff moved below the
    # second-neighbour shell).  At the Gamma point of the two-atom primitive
    # cell the four tetrahedral bonds decouple s from p and the p orbitals from
    # each other, leaving 2x2 pencils:
    #   s:  (Es +- 4 V_ss u) / (1 +- 4 S_ss u)
    #   p:  (Ep +- 4/3 (V_pps + 2 V_ppp) u) / (1 +- 4/3 (S_pps + 2 S_ppp) u)  (x3)
    # (Harrison's tetrahedral-solid Gamma levels, generalized to an overlap).
    # Gamma of the primitive cell folds onto Gamma of the 2x2x2 supercell.
    p = sk.SKParams(r_on=2.0, r_cut=2.2)
    pos, cell = gen.diamond_sites(2, 2, 2)
    H, S = _dense(pos, cell, p)
    ev = _spectrum(H, S)
    r = np.sqrt(3.0) / 4.0 * gen.structures.A_DIAMOND
    u, _ = sk.radial(r, p)
    sss, _, spps, sppp = p.overlap()
    levels = []
    for sg in (+1, -1):
        levels.append(((p.es + sg * 4 * p.v_ss_sigma * u) / (1 + sg * 4 * sss * u), 1))
        vp = 4.0 / 3.0 * (p.v_pp_sigma + 2 * p.v_pp_pi) * u
        spv = 4.0 / 3.0 * (spps + 2 * sppp) * u
        levels.append(((p.ep + sg * vp) / (1 + sg * spv), 3))
    for lev, mult in levels:
        assert np.sum(np.abs(ev - lev) < 1e-9) >= mult, (lev, mult)


@pytest.mark.parametrize("k", [1, 2])
def test_h_s_symmetric_and_s_positive_definite(k):
    s = gen.make(k)
    H, S, _ = nb.build_csr(s.pos, s.cell)
    assert abs(H - H.T).max() == 0.0
    assert abs(S - S.T).max() == 0.0
    if k == 1:
        Sd = S.toarray()
        sla.cholesky(Sd)  # raises if not positive definite
        assert sla.eigh(Sd, eigvals_only=True)[0] > 0.5


@pytest.mark.parametrize("r", [1.45, 1.9, 2.15, 2.45, 2.59])
def test_block_gradients_match_finite_differences(r):
    rng = np.random.default_rng(int(r * 100))
    u = rng.normal(size=3)
    d = r * u / np.linalg.norm(u)
    gH, gS = sk.pair_block_grads(d)
    h = 1e-6
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        Hp, Sp = sk.pair_blocks(d + e)
        Hm, Sm = sk.pair_blocks(d - e)
        np.testing.assert_allclose(gH[c], (Hp - Hm) / (2 * h), atol=2e-8)
        np.testing.assert_allclose(gS[c], (Sp - Sm) / (2 * h), atol=2e-9)


def test_cutoff_is_smooth_and_vanishes():
    p = sk.CARBON
    assert sk.cutoff(p.r_cut, p) == (0.0, 0.0)
    assert sk.cutoff(p.r_on, p)[0] == 1.0
    # continuity at both ends (the quintic step leaves only rounding there)
    f1, _ = sk.cutoff(p.r_cut - 1e-7, p)
    assert abs(f1) < 1e-14
    f0, _ = sk.cutoff(p.r_on + 1e-7, p)
    assert abs(f0 - 1.0) < 1e-14
