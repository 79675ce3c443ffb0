"""Tight-binding model of the benchmark workloads: two-center carbon sp.

Onsite Es = -2.99, Ep = 3.71 eV; bond integrals V_ss_sigma = -5.0,
V_sp_sigma = 4.7, V_pp_sigma = 5.5, V_pp_pi = -1.55 eV at r0 = 1.54 A, scaled by
(r0/r)^2 with a quintic smooth cutoff from 2.0 to 2.6 A; overlap S = I + 0.08 X
where X has the same form with the bond integrals replaced by their signs.

MD total energy: the band free energy plus a pair repulsion
phi(r) = phi0 (r0/r)^m fc(r) (Goodwin-Skinner-Pettifor form for (r0/r)^2
hoppings) with m = 4 and phi0 = 13.18 eV, the value that puts perfect diamond
(a = 3.567 A) at zero pressure at kT = 0.1 eV; carbon mass 12.011 amu.
"""
from __future__ import annotations

from ._lib import MagSKModel

CARBON_SP = dict(
    es=-2.99, ep=3.71,
    v_ss_sigma=-5.0, v_sp_sigma=4.7, v_pp_sigma=5.5, v_pp_pi=-1.55,
    s_ss_sigma=-0.08, s_sp_sigma=0.08, s_pp_sigma=0.08, s_pp_pi=-0.08,
    r0=1.54, r_on=2.0, r_cut=2.6,
)


PAIR_REPULSION = dict(phi0=13.18, m_rep=4.0)
MASS_CARBON = 12.011  # amu
KB_EV = 8.617333262e-5  # Boltzmann constant, eV/K
AMU_A2_FS2_EV = 1.66053906660e-17 / 1.602176634e-19  # amu (A/fs)^2 in eV


def thermal_sigma(T, mass=MASS_CARBON):
    """Standard deviation of one Maxwell-Boltzmann velocity component, A/fs."""
    return (KB_EV * T / (mass * AMU_A2_FS2_EV)) ** 0.5


def sk_model(**overrides) -> MagSKModel:
    p = dict(CARBON_SP)
    p.update(overrides)
    return MagSKModel(**p)
