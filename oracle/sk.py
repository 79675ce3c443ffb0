"""Slater-Koster two-center carbon sp model (oracle copy; test infrastructure).

The paper works with tight-binding LCAO matrices H and S that are sparse,
real-symmetric, with S positive definite (problem statement around Eq. 1), and
runs a carbon sp model with four orbitals (s, px, py, pz) per atom.  Its own
parameter sets are in references that are not available, so the benchmark's
model is used:

  onsite        Es = -2.99 eV, Ep = 3.71 eV
  hoppings      V_ss_sigma = -5.0, V_sp_sigma = 4.7, V_pp_sigma = 5.5,
                V_pp_pi = -1.55 eV at r0 = 1.54 A
  radial form   (r0 / r)^2 * fc(r), fc = 1 - (10 t^3 - 15 t^4 + 6 t^5),
                t = (r - 2.0) / (2.6 - 2.0) clipped to [0, 1] (zero at 2.6 A)
  overlap       S = I + 0.08 * X, X the same two-center form with the four
                bond integrals replaced by their signs (-1, +1, +1, -1)
  pattern       atom pairs closer than 2.6 A (minimum image)

Block convention: for atoms I (rows) and K (columns) with displacement
d = R_K - R_I, direction cosines l = d / |d| and radial factor u(r):
  E_ss       = V_ss * u
  E_s,a      =  l_a * V_sp * u          (s on I, p_a on K)
  E_a,s      = -l_a * V_sp * u          (p_a on I, s on K)
  E_a,b      = (l_a l_b V_pp_sigma + (delta_ab - l_a l_b) V_pp_pi) * u
These are the standard two-center integrals of Slater and Koster (1954).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class SKParams:
    es: float = -2.99
    ep: float = 3.71
    v_ss_sigma: float = -5.0
    v_sp_sigma: float = 4.7
    v_pp_sigma: float = 5.5
    v_pp_pi: float = -1.55
    r0: float = 1.54
    r_on: float = 2.0
    r_cut: float = 2.6
    s_scale: float = 0.08
    s_signs: tuple = (-1.0, 1.0, 1.0, -1.0)

    def hopping(self):
        return (self.v_ss_sigma, self.v_sp_sigma, self.v_pp_sigma, self.v_pp_pi)

    def overlap(self):
        return tuple(self.s_scale * x for x in self.s_signs)


CARBON = SKParams()


def cutoff(r: float, p: SKParams):
    """fc(r) and dfc/dr for the quintic smooth step between r_on and r_cut."""
    width = p.r_cut - p.r_on
    t = (r - p.r_on) / width
    if t <= 0.0:
        return 1.0, 0.0
    if t >= 1.0:
        return 0.0, 0.0
    step = 10 * t**3 - 15 * t**4 + 6 * t**5
    dstep = (30 * t**2 - 60 * t**3 + 30 * t**4) / width
    return 1.0 - step, -dstep


def radial(r: float, p: SKParams):
    """u(r) = (r0/r)^2 fc(r) and du/dr."""
    fc, dfc = cutoff(r, p)
    g = (p.r0 / r) ** 2
    dg = -2.0 * p.r0**2 / r**3
    return g * fc, dg * fc + g * dfc


def two_center(d: np.ndarray, bonds, p: SKParams):
    """4x4 two-center block for displacement d (atom I -> atom K)."""
    r = float(np.sqrt(d @ d))
    l = d / r
    u, _ = radial(r, p)
    vss, vsp, vpps, vppp = bonds
    B = np.zeros((4, 4))
    B[0, 0] = vss * u
    for a in range(3):
        B[0, 1 + a] = l[a] * vsp * u
        B[1 + a, 0] = -l[a] * vsp * u
        for b in range(3):
            delta = 1.0 if a == b else 0.0
            B[1 + a, 1 + b] = (l[a] * l[b] * vpps + (delta - l[a] * l[b]) * vppp) * u
    return B


def two_center_grad(d: np.ndarray, bonds, p: SKParams):
    """d B / d d_c for c = x, y, z: array (3, 4, 4).

    Product rule on B = A(l) u(r) with dl_a/dd_c = (delta_ac - l_a l_c)/r and
    dr/dd_c = l_c.
    """
    r = float(np.sqrt(d @ d))
    l = d / r
    u, du = radial(r, p)
    vss, vsp, vpps, vppp = bonds
    G = np.zeros((3, 4, 4))
    dl = (np.eye(3) - np.outer(l, l)) / r  # dl[a, c] = dl_a / dd_c
    for c in range(3):
        dr = l[c]
        G[c, 0, 0] = vss * du * dr
        for a in range(3):
            val = l[a] * vsp
            dval = dl[a, c] * vsp
            G[c, 0, 1 + a] = dval * u + val * du * dr
            G[c, 1 + a, 0] = -(dval * u + val * du * dr)
            for b in range(3):
                delta = 1.0 if a == b else 0.0
                ang = l[a] * l[b] * vpps + (delta - l[a] * l[b]) * vppp
                dang = (dl[a, c] * l[b] + l[a] * dl[b, c]) * (vpps - vppp)
                G[c, 1 + a, 1 + b] = dang * u + ang * du * dr
    return G


def onsite_h(p: SKParams):
    return np.diag([p.es, p.ep, p.ep, p.ep])


def pair_blocks(d: np.ndarray, p: SKParams = CARBON):
    """(H block, S block) between two distinct atoms with displacement d."""
    return two_center(d, p.hopping(), p), two_center(d, p.overlap(), p)


def hopping_sigma_pi(d: np.ndarray, p: SKParams = CARBON):
    """(H_sigma, H_pi): the H block between distinct atoms split by bond type,
    as the sigma/pi crystal orbital Hamiltonian population needs it (the
    decomposition stated before Eq. 7).  The pi part is the V_pp_pi term of the
    p-p sub-block; the sigma part holds the V_ss, V_sp and V_pp_sigma terms.
    two_center is linear in the bond integrals, so the parts are the block with
    the other integrals set to zero."""
    vss, vsp, vpps, vppp = p.hopping()
    return (two_center(d, (vss, vsp, vpps, 0.0), p), two_center(d, (0.0, 0.0, 0.0, vppp), p))


def pair_block_grads(d: np.ndarray, p: SKParams = CARBON):
    """(dH/dd, dS/dd), each (3, 4, 4)."""
    return two_center_grad(d, p.hopping(), p), two_center_grad(d, p.overlap(), p)
