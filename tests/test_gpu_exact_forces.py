"""The exact gradient of the truncated-Krylov grand potential on the GPU
(mag_forces_exact) against the oracle's reverse-mode gradient and against
central differences of the GPU's own grand potential.

The forces through rho and pi (mag_forces, the letter's reading after Eq. 1)
are the derivative only when every column's Krylov space is exact; the exact
gradient follows each column through its Krylov space as well.  Bars: 1e-8
eV/A against the oracle (the force bar), 1e-6 eV/A against differences at
h = 1e-5 A, and the exact and density-matrix forces equal in the exact
regime.
"""
import numpy as np
import pytest

from gpu_helpers import gpu_context, log, np_

pytestmark = pytest.mark.gpu

F_TOL = 1e-8


def _solve_both(s, sk=None):
    from paper_1210_1531_amd import model
    ctx = gpu_context(s, sk=sk)
    mu, E, A = ctx.solve(nu=s.nu, kT=s.kT, n_electrons=s.n_electrons)
    m = model.sk_model(**(sk or {}))
    Fx = np_(ctx.forces_exact(m))
    Fh = np_(ctx.forces(m))
    return ctx, mu, Fx, Fh


def test_exact_forces_whole_cell_against_oracle():
    # the 61-atom whole cell at nu = 12 (244 orbitals): every atom
    import gen
    from oracle import adjoint, solve
    s = gen.make("tiny")
    ctx, mu, Fx, Fh = _solve_both(s)
    Fo = adjoint.exact_forces_on(solve.geometry(s), np.arange(s.n_atoms), mu)
    d = np.abs(Fx - Fo).max()
    log(f"[exact tiny] max |F_exact - F_oracle| {d:.2e}; max |F_exact - F_rho| "
        f"{np.abs(Fx - Fh).max():.3f}; |sum F| {np.abs(Fx.sum(axis=0)).max():.1e}; "
        f"{ctx.stats()['t_forces_exact_ms']:.2f} ms")
    assert d <= F_TOL
    assert np.abs(Fx.sum(axis=0)).max() <= 1e-9


@pytest.mark.parametrize("key", ["mini_vac", 2])
def test_exact_forces_sampled_atoms_against_oracle(key):
    # 6 A clusters at nu = 30: the vacancy cell and the benchmark cell, three
    # atoms each (every column whose cluster holds them, on the oracle side)
    import gen
    from oracle import adjoint, solve
    s = gen.make(key)
    ctx, mu, Fx, Fh = _solve_both(s)
    pick = np.sort(np.random.default_rng(21).choice(s.n_atoms, 3, replace=False))
    Fo = adjoint.exact_forces_on(solve.geometry(s), pick, mu)
    d = np.abs(Fx[pick] - Fo).max()
    log(f"[exact {key}] atoms {pick.tolist()}: max |F_exact - F_oracle| {d:.2e}; "
        f"max |F_exact - F_rho| over all atoms {np.abs(Fx - Fh).max():.3f}; |sum F| "
        f"{np.abs(Fx.sum(axis=0)).max():.1e}; {ctx.stats()['t_forces_exact_ms']:.2f} ms")
    assert d <= F_TOL
    assert np.abs(Fx.sum(axis=0)).max() <= 1e-8


def test_exact_forces_against_differences_on_the_gradient_cell():
    # the gradient workload (3,892 atoms, nu = 30): eight atoms, central
    # differences of the GPU grand potential at fixed mu with h = 1e-5 and
    # 2e-5 A, and their Richardson combination (4 D(h) - D(2h)) / 3, whose
    # error is O(h^4) instead of O(h^2)
    import gen
    from test_gpu_grad import fd_forces
    s = gen.make(4)
    ctx, mu, Fx, Fh = _solve_both(s)
    atoms = np.sort(np.random.default_rng(4).choice(s.n_atoms, 32, replace=False))[:8]
    F1 = fd_forces(ctx, s, atoms, mu, h=1e-5)
    F2 = fd_forces(ctx, s, atoms, mu, h=2e-5)
    Fr = (4.0 * F1 - F2) / 3.0
    d1, d2, dr = (np.abs(Fx[atoms] - x).max() for x in (F1, F2, Fr))
    log(f"[exact config 4] 8 atoms: max |F_exact - F_FD| h=1e-5 {d1:.2e}, h=2e-5 {d2:.2e}, "
        f"Richardson {dr:.2e} eV/A; max |F_rho - F_FD| {np.abs(Fh[atoms] - Fr).max():.3f} eV/A")
    assert dr <= 1e-6


def test_exact_forces_equal_density_forces_in_the_exact_regime():
    # six atoms in one conventional cell (two vacancies, 24 orbitals), whole
    # cell, nu = 24: every Krylov space is the whole space, so the exact
    # gradient is the force through rho and pi
    from gen import structures as gs
    sk = dict(r_on=1.65, r_cut=1.75)
    s = gs.make_structure(cells=(1, 1, 1), vacancy_frac=0.25, sigma=0.05, seed=9, nu=24,
                          r_cluster=0.0, name="cell6_exact")
    assert s.n_atoms == 6
    ctx, mu, Fx, Fh = _solve_both(s, sk=sk)
    _, _, nu_eff = ctx.spectra()
    log(f"[exact regime] nu_eff {np.unique(np_(nu_eff)).tolist()}, max |F_exact - F_rho| "
        f"{np.abs(Fx - Fh).max():.2e}, max |F| {np.abs(Fh).max():.2e}")
    assert np.all(np_(nu_eff) == 24)
    assert np.abs(Fx - Fh).max() <= 1e-9


def test_exact_forces_errors():
    import gen
    from paper_1210_1531_amd import MagError, _lib as L, model
    s = gen.make("mini_vac")
    ctx = gpu_context(s)
    with pytest.raises(MagError) as e:
        ctx.forces_exact(model.sk_model())  # before a solve
    assert e.value.status == L.MAG_ESTATE
    ctx.solve(nu=40, kT=s.kT, n_electrons=s.n_electrons)
    with pytest.raises(MagError) as e:
        ctx.forces_exact(model.sk_model())  # nu above the kernel's capacity
    assert e.value.status == L.MAG_EUNSUPPORTED


def test_kept_pass_gives_the_same_forces_and_goes_stale():
    """keep_exact: the solve keeps every column's pass-1 data and
    mag_forces_exact skips its own pass; the forces are bitwise those of the
    second pass.  New values of H and S drop the kept data."""
    import torch
    import gen
    from paper_1210_1531_amd import model
    s = gen.make(2)
    m = model.sk_model()
    kw = dict(nu=s.nu, kT=s.kT, n_electrons=s.n_electrons)
    ctx = gpu_context(s)
    ctx.solve(**kw)
    F_ref = np_(ctx.forces_exact(m))
    t_ref = ctx.stats()["t_forces_exact_ms"]
    ctx.solve(keep_exact=True, **kw)
    F_kept = np_(ctx.forces_exact(m))
    t_kept = ctx.stats()["t_forces_exact_ms"]
    log(f"[exact kept] bitwise {np.array_equal(F_kept, F_ref)}; {t_ref:.1f} ms with the pass, "
        f"{t_kept:.1f} ms from the kept data")
    assert np.array_equal(F_kept, F_ref)
    # the kept data belong to the old values: after an update the next solve
    # (without keeping) and forces_exact use the new ones
    pos1 = torch.tensor(s.pos + np.random.default_rng(3).normal(0.0, 0.01, s.pos.shape),
                        dtype=torch.float64, device="cuda")
    ctx.solve(keep_exact=True, **kw)
    Hv, Sv = ctx.sk_values(pos1)
    ctx.update_values(Hv, Sv)
    ctx.solve(**kw)
    F_new = np_(ctx.forces_exact(m))
    fresh = gpu_context(s)
    fresh.update_values(*fresh.sk_values(pos1))
    fresh.solve(**kw)
    assert np.array_equal(F_new, np_(fresh.forces_exact(m)))
    assert not np.array_equal(F_new, F_ref)
