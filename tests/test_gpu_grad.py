"""The differentiation boundary on the GPU: the torch.autograd chain
positions -> (H, S) -> free energy, the adjoint dA/dH = gA rho and
dA/dS = -gA pi of mag_backward, the Slater-Koster values and their
vector-Jacobian product, and finite differences of the free energy.

Forces are taken through the density matrix (the force paragraph after Eq. 1
and Eq. 2).  In the exact regime they are the gradient (checked by
differences in test_gpu_edges); on the benchmark cell at nu = 30 they are not,
and the difference to central differences of the grand potential is the
method's non-variational error, which test_fd_report_on_the_gradient_cell
records.
"""
import numpy as np
import pytest

from gpu_helpers import gpu_context, log, np_, oracle_solution, oracle_system

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("device_outputs", [True, False])
def test_autograd_chain_gives_the_forces(device_outputs):
    import torch
    from paper_1210_1531_amd import model
    from paper_1210_1531_amd.autograd import EnergyFn, SKFn
    s, sysm = oracle_system("mini_vac")
    ctx = gpu_context(s, device_outputs=device_outputs)
    sk = model.sk_model()
    opts = dict(nu=s.nu, kT=s.kT, n_electrons=s.n_electrons)
    pos = torch.tensor(s.pos, dtype=torch.float64, device="cuda", requires_grad=True)
    H, S = SKFn.apply(pos, ctx)
    A = EnergyFn.apply(H, S, ctx, opts)
    A.backward()
    F = np_(ctx.forces(sk))
    g = pos.grad.detach().cpu().numpy()
    d = np.abs(g + F).max()
    log(f"[autograd outputs={'device' if device_outputs else 'host'}] A {float(A):.10f}, "
        f"max |dA/dR + F| {d:.2e}, max |F| {np.abs(F).max():.2e}")
    assert np.isfinite(g).all()
    assert d <= 1e-12 * max(1.0, np.abs(F).max())
    # the free energy is the library's
    assert float(A) == ctx.energy()["A_free"]


@pytest.mark.parametrize("device_outputs", [True, False])
def test_backward_is_gA_rho_and_minus_gA_pi(device_outputs):
    from oracle import solve
    s, sysm = oracle_system("mini_vac")
    ref = oracle_solution("mini_vac")
    ctx = gpu_context(s, device_outputs=device_outputs)
    mu, E, A = ctx.solve(nu=s.nu, kT=s.kT, n_electrons=s.n_electrons)
    rho, pi = (np_(x) for x in ctx.density_matrix())
    rho_o, pi_o = solve.density_on_pattern(sysm, ref.cd, mu)
    for gA in (1.0, 2.5, -0.75):
        dH, dS = (np_(x) for x in ctx.backward(gA))
        # the adjoint is linear in gA and is the density matrices themselves
        np.testing.assert_array_equal(dH, gA * rho)
        np.testing.assert_array_equal(dS, -gA * pi)
        assert np.abs(dH - gA * rho_o).max() <= abs(gA) * 1e-10
        assert np.abs(dS + gA * pi_o).max() <= abs(gA) * 1e-9
    log(f"[backward] mini_vac: gA rho and -gA pi against the oracle at gA = 1, 2.5, -0.75")


def values_on_pattern(sysm, pos):
    """The oracle's H and S values at positions `pos` on sysm's (fixed)
    pattern: the two-centre blocks of every block-row pair, onsite blocks on
    the diagonal (pairs that moved past the cutoff give zero blocks)."""
    from oracle import neighbors as nb
    from oracle import sk as osk
    H = np.zeros(sysm.H.nnz)
    S = np.zeros(sysm.H.nnz)
    ip = sysm.H.indptr
    for J, ks in enumerate(sysm.rows):
        for t, K in enumerate(ks):
            if K == J:
                bh, bs = osk.onsite_h(sysm.params), np.eye(4)
            else:
                bh, bs = osk.pair_blocks(nb.min_image(pos[K] - pos[J], sysm.cell), sysm.params)
            for a in range(4):
                lo = ip[4 * J + a] + 4 * t
                H[lo:lo + 4] = bh[a]
                S[lo:lo + 4] = bs[a]
    return H, S


def test_sk_values_and_vjp_match_oracle():
    # H, S values at displaced positions on the built pattern, and the
    # vector-Jacobian product sum_p gH_p dH_p/dR + gS_p dS_p/dR against the
    # oracle's own Slater-Koster derivatives (its force contraction with
    # rho = gH and pi = -gS gives minus the product)
    import torch
    from dataclasses import replace
    from oracle import solve
    s, sysm = oracle_system("mini_vac")
    ctx = gpu_context(s)
    rng = np.random.default_rng(3)
    pos1 = s.pos + rng.normal(0.0, 0.01, size=s.pos.shape)
    H1, S1 = values_on_pattern(sysm, pos1)
    p1 = torch.tensor(pos1, dtype=torch.float64, device="cuda")
    Hv, Sv = (np_(x) for x in ctx.sk_values(p1))
    dH, dS = np.abs(Hv - H1).max(), np.abs(Sv - S1).max()
    gH = rng.normal(size=sysm.H.nnz)
    gS = rng.normal(size=sysm.H.nnz)
    grad = np_(ctx.sk_vjp(p1, torch.tensor(gH, device="cuda"), torch.tensor(gS, device="cuda")))
    ref = -solve.forces(replace(sysm, pos=pos1), gH, -gS)
    d = np.abs(grad - ref).max()
    log(f"[sk values] |dH| {dH:.2e} |dS| {dS:.2e}; [sk vjp] max |d grad| {d:.2e} "
        f"(max |grad| {np.abs(ref).max():.2e})")
    assert dH <= 1e-13 and dS <= 1e-14
    assert d <= 1e-11 * max(1.0, np.abs(ref).max())


def grand_potential_columns(eps, w, nu_eff, mu, kT):
    """Per-column grand potential Omega_j = sum_k w_jk omega(eps_jk), with
    omega(e) = -kT ln(1 + exp(-(e - mu)/kT)) (A - mu N of the column)."""
    x = (eps - mu) / kT
    om = -kT * (np.maximum(-x, 0.0) + np.log1p(np.exp(-np.abs(x))))
    mask = np.arange(eps.shape[1])[None, :] < nu_eff[:, None]
    return np.where(mask, w * om, 0.0).sum(axis=1)


def fd_forces(ctx, s, atoms, mu, h=1e-5):
    """Central differences of the GPU's grand potential at fixed mu, for the
    three components of each atom.  Columns whose cluster does not hold the
    displaced atom are bitwise unchanged, so only the columns of the atoms of
    its cluster enter the difference (summed with math.fsum)."""
    import math
    import torch
    from gpu_helpers import torch_index
    ptr, catoms = (np_(x) for x in ctx.get_clusters())
    pos0 = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    out = np.zeros((len(atoms), 3))
    for a, I in enumerate(atoms):
        near = catoms[ptr[I]:ptr[I + 1]]
        cols = (4 * near[:, None] + np.arange(4)[None, :]).ravel()
        for c in range(3):
            om = []
            for sgn in (1.0, -1.0):
                p = pos0.clone()
                p[I, c] += sgn * h
                Hv, Sv = ctx.sk_values(p)
                ctx.update_values(Hv, Sv)
                ctx.solve(nu=s.nu, kT=s.kT, n_electrons=s.n_electrons, mu_fixed=mu)
                eps, w, nu = ctx.spectra()
                ix = torch_index(cols, eps)
                om.append(grand_potential_columns(np_(eps[ix]), np_(w[ix]), np_(nu[ix]), mu, s.kT))
            out[a, c] = -math.fsum(om[0] - om[1]) / (2 * h)
    Hv, Sv = ctx.sk_values(pos0)
    ctx.update_values(Hv, Sv)
    return out


def test_fd_report_on_the_gradient_cell():
    """The benchmark cell of the gradient workload (3,892 atoms, nu = 30):
    32 random atoms x 3 components x 2 displacements of 1e-5 A.  The forces
    through rho are not the derivative here (the Krylov space of each column
    also moves with H), so their distance to the differences is reported,
    not bounded; the differences themselves are checked for noise by
    Omega's antisymmetry (the force on an atom from the displacement of
    +h and -h agree with a quarter-step difference)."""
    import gen
    from paper_1210_1531_amd import model
    s = gen.make(4)
    ctx = gpu_context(s)
    mu, E, A = ctx.solve(nu=s.nu, kT=s.kT, n_electrons=s.n_electrons)
    F = np_(ctx.forces(model.sk_model()))
    atoms = np.sort(np.random.default_rng(4).choice(s.n_atoms, 32, replace=False))
    Ffd = fd_forces(ctx, s, atoms, mu)
    Ffd2 = fd_forces(ctx, s, atoms[:4], mu, h=2e-5)
    dev = np.abs(F[atoms] - Ffd)
    noise = np.abs(Ffd[:4] - Ffd2).max()
    log(f"[fd config 4] 32 atoms: max |F_HF - F_FD| {dev.max():.3e} eV/A, mean {dev.mean():.3e}; "
        f"max |F_FD| {np.abs(Ffd).max():.3e}; h vs 2h difference {noise:.2e}")
    assert np.isfinite(Ffd).all()
    assert noise <= 1e-5
