"""GPU MD step against the oracle: the pair repulsion and whole velocity Verlet
frames (rebuild, solve, forces, kick and drift), on seeded cells.

Bars: pair energies and forces to rounding (1e-11 eV, eV/A); frames of the
MD run within the force bar |dF| <= 1e-8 eV/A and |dE|/atom <= 1e-9 eV, which
move positions and velocities by at most dt^2 |dF| / m (1e-12 A) per step.
"""
import os

import numpy as np
import pytest

from gen import structures as gs
from gpu_helpers import log, np_, torch_cuda

pytestmark = pytest.mark.gpu

MASS = 12.011  # amu
KB = 8.617333262e-5  # eV / K
AMU_EV = 1.66053906660e-17 / 1.602176634e-19  # amu (A/fs)^2 in eV (CODATA 2018)
PHI0, MREP = 13.18, 4.0
PAIR_TOL = 1e-11
F_TOL = 1e-8
E_TOL = 1e-9


def _sigma(T):
    return float(np.sqrt(KB * T / (MASS * AMU_EV)))


def _min_image(d, cell):
    return d - cell * np.rint(d / cell)


@pytest.mark.parametrize("key", ["mini_vac", 2])
def test_pair_repulsion_matches_oracle(key):
    torch = torch_cuda()
    from oracle import md
    from paper_1210_1531_amd import Context, model
    s = gs.make(key)
    log(f"[pair {key}] {s.n_atoms} atoms")
    ctx = Context()
    ctx.sk_build(model.sk_model(), torch.tensor(s.pos, dtype=torch.float64, device="cuda"), s.cell)
    E, e, F = ctx.pair_repulsion(PHI0, MREP)
    e, F = np_(e), np_(F)
    atoms = None if key == "mini_vac" else np.sort(
        np.random.default_rng(5).choice(s.n_atoms, 96, replace=False))
    Eo, eo, Fo = md.pair_repulsion(s.pos, s.cell, PHI0, MREP, atoms=atoms)
    rows = slice(None) if atoms is None else atoms
    de, dF = np.abs(e[rows] - eo).max(), np.abs(F[rows] - Fo).max()
    log(f"[pair {key}] E_rep {E:.10f}, max |de| {de:.3e}, max |dF| {dF:.3e}")
    assert de <= PAIR_TOL and dF <= PAIR_TOL
    if Eo is not None:
        assert abs(E - Eo) <= 1e-12 * abs(Eo)
    assert abs(E - e.sum()) <= 1e-12 * abs(E)
    assert np.abs(F.sum(axis=0)).max() < 1e-9  # the pair forces cancel


def test_md_frames_match_oracle_mini_vac():
    torch = torch_cuda()
    from oracle import md
    from paper_1210_1531_amd import Context, model
    s = gs.make("mini_vac")
    v0 = gs.random_velocities(s.n_atoms, _sigma(300.0), 21)
    dt, steps = 0.5, 2
    log(f"[md mini_vac] {s.n_atoms} atoms, {steps} steps of {dt} fs")
    ctx = Context()
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    pos, vel, F, th = ctx.md_run(model.sk_model(), dev(s.pos), dev(v0), s.cell, dt, MASS, steps,
                                 phi0=PHI0, m_rep=MREP, r_cluster=s.r_cluster, nu=s.nu,
                                 kT=s.kT, n_electrons=s.n_electrons)
    pos, vel, F = np_(pos), np_(vel), np_(F)
    fr = md.velocity_verlet(s.pos, v0, s.cell, md.krylov_forces(s, phi0=PHI0),
                            MASS, dt, steps)
    n = s.n_atoms
    dx = np.abs(_min_image(pos - fr[-1].pos, s.cell)).max()
    dv = np.abs(vel - fr[-1].vel).max()
    dF = np.abs(F - fr[-1].F).max()
    log(f"[md mini_vac] max |dx| {dx:.3e} A, |dv| {dv:.3e} A/fs, |dF| {dF:.3e} eV/A; "
        f"E_tot {th[0, 0] + th[0, 1]:.8f} -> {th[-1, 0] + th[-1, 1]:.8f}; "
        f"{ctx.stats()['t_md_step_ms']:.1f} ms per step")
    assert dF <= F_TOL
    assert dx <= 1e-10 and dv <= 1e-11
    for k, f in enumerate(fr):
        assert abs(th[k, 0] - f.E_pot) / n <= E_TOL
        assert abs(th[k, 1] - f.E_kin) <= 1e-10 * f.E_kin
        assert abs(th[k, 3] - f.E_band) / n <= E_TOL
    # the context holds the last frame: its system and solve
    assert ctx.n_atoms == n and abs(ctx.energy()["E_band"] - th[-1, 3]) <= 1e-12 * abs(th[-1, 3])


def test_md_step_at_full_size_config2():
    """One velocity Verlet step on the 3,892-atom cell: the step's algebra on
    the GPU's own frame-0 forces, momentum, and a rerun from the same start."""
    torch = torch_cuda()
    from paper_1210_1531_amd import Context, model
    s = gs.make(2)
    v0 = gs.random_velocities(s.n_atoms, _sigma(300.0), 22)
    dt = 0.5
    ctx = Context()
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    kw = dict(phi0=PHI0, m_rep=MREP, r_cluster=s.r_cluster, nu=s.nu, kT=s.kT,
              n_electrons=s.n_electrons)
    log(f"[md config2] {s.n_atoms} atoms: frame 0")
    _, _, F0, th0 = ctx.md_run(model.sk_model(), dev(s.pos), dev(v0), s.cell, dt, MASS, 0, **kw)
    F0 = np_(F0)
    log("[md config2] one step")
    x1, v1, F1, th = ctx.md_run(model.sk_model(), dev(s.pos), dev(v0), s.cell, dt, MASS, 1, **kw)
    x1, v1, F1 = np_(x1), np_(v1), np_(F1)
    c = dt / (2 * MASS * AMU_EV)
    x_exp = s.pos + dt * v0 + dt * c * F0
    v_exp = v0 + c * (F0 + F1)
    dx = np.abs(_min_image(x1 - x_exp, s.cell)).max()
    dv = np.abs(v1 - v_exp).max()
    log(f"[md config2] frame-0 rerun |dE| {abs(th[0, 0] - th0[0, 0]):.3e}, step |dx| {dx:.3e}, "
        f"|dv| {dv:.3e}, E_tot {th[0, 0] + th[0, 1]:.6f} -> {th[1, 0] + th[1, 1]:.6f}, "
        f"{ctx.stats()['t_md_step_ms']:.1f} ms per step")
    assert np.array_equal(th[0], th0[0])  # deterministic solve: same start, same frame
    # x is wrapped into the box, the expectation is not: compare minimum images
    assert dx <= 1e-12 and dv <= 1e-12
    assert np.all((x1 >= 0) & (x1 < s.cell[None, :]))
    assert np.abs(F0.sum(axis=0)).max() < 1e-8 and np.abs(v1.sum(axis=0)).max() < 1e-11
    # the step moves energy between kinetic and potential, not more than the
    # Hellmann-Feynman reading at nu = 30 and the dt^2 error allow
    assert abs((th[1, 0] + th[1, 1]) - (th[0, 0] + th[0, 1])) / s.n_atoms < 1e-3


def test_md_whole_cell_cluster_matches_oracle():
    """r_cluster <= 0: every column's cluster is the whole 64-atom cell."""
    torch = torch_cuda()
    from oracle import md
    from paper_1210_1531_amd import Context, model
    s = gs.make(1)
    v0 = gs.random_velocities(s.n_atoms, _sigma(300.0), 23)
    ctx = Context()
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    pos, vel, F, th = ctx.md_run(model.sk_model(), dev(s.pos), dev(v0), s.cell, 0.5, MASS, 2,
                                 phi0=PHI0, m_rep=MREP, r_cluster=0.0, nu=s.nu, kT=s.kT,
                                 n_electrons=s.n_electrons)
    fr = md.velocity_verlet(s.pos, v0, s.cell, md.krylov_forces(s, workers=1, phi0=PHI0), MASS,
                            0.5, 2)
    dF = np.abs(np_(F) - fr[-1].F).max()
    dx = np.abs(_min_image(np_(pos) - fr[-1].pos, s.cell)).max()
    log(f"[md whole cell] |dF| {dF:.3e}, |dx| {dx:.3e}")
    assert dF <= F_TOL and dx <= 1e-10
    assert all(abs(th[k, 0] - f.E_pot) / s.n_atoms <= E_TOL for k, f in enumerate(fr))


def test_md_and_pair_errors():
    torch = torch_cuda()
    from paper_1210_1531_amd import Context, MagError, model
    s = gs.make("tiny")
    ctx = Context()
    x = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    v = torch.zeros_like(x)
    with pytest.raises(MagError):
        ctx.pair_repulsion(PHI0, MREP)  # no build yet
    kw = dict(nu=s.nu, kT=s.kT, n_electrons=s.n_electrons)
    for dt, mass, steps in ((0.0, MASS, 1), (0.5, -1.0, 1), (0.5, MASS, -1)):
        with pytest.raises(MagError):
            ctx.md_run(model.sk_model(), x, v, s.cell, dt, mass, steps, **kw)
    with pytest.raises(MagError):
        ctx.md_run(model.sk_model(), x, v, s.cell, 0.5, MASS, 1, phi0=1.0, m_rep=0.0, **kw)
    ctx.sk_build(model.sk_model(), x, s.cell)
    with pytest.raises(MagError):
        ctx.pair_repulsion(PHI0, -4.0)
    E, _, _ = ctx.pair_repulsion(0.0, MREP)  # no repulsion: zero energy
    assert E == 0.0


def test_md_host_arrays_equal_device_arrays():
    """The same run with host (NumPy) and device (torch) arrays: bitwise equal."""
    torch = torch_cuda()
    from paper_1210_1531_amd import Context, model
    s = gs.make("tiny")
    v0 = gs.random_velocities(s.n_atoms, _sigma(300.0), 24)
    kw = dict(phi0=PHI0, m_rep=MREP, r_cluster=s.r_cluster, nu=s.nu, kT=s.kT,
              n_electrons=s.n_electrons)
    host = Context(device_outputs=False)
    xh, vh, Fh, th_h = host.md_run(model.sk_model(), s.pos, v0, s.cell, 0.5, MASS, 2, **kw)
    dev = Context()
    t = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    xd, vd, Fd, th_d = dev.md_run(model.sk_model(), t(s.pos), t(v0), s.cell, 0.5, MASS, 2, **kw)
    assert isinstance(xh, np.ndarray)
    assert np.array_equal(xh, np_(xd)) and np.array_equal(vh, np_(vd))
    assert np.array_equal(Fh, np_(Fd)) and np.array_equal(th_h, th_d)


def test_sk_build_rejects_overfull_block_rows():
    """40 atoms within 1.2 A of a point: every block row would exceed the
    32-block limit; the build reports it instead of truncating the rows."""
    torch_cuda()
    from paper_1210_1531_amd import Context, MagError, model
    rng = np.random.default_rng(2)
    pos = 5.0 + rng.uniform(-0.7, 0.7, size=(40, 3))
    ctx = Context(device_outputs=False)
    with pytest.raises(MagError) as e:
        ctx.sk_build(model.sk_model(), pos, (10.0, 10.0, 10.0))
    assert "MAG_EUNSUPPORTED" in str(e.value)


def _md_energy_series(ctx, s, v0, dt, T, exact, torch):
    """E_pot + E_kin - its start at every frame of a run of T fs."""
    from paper_1210_1531_amd import model
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    _, _, _, th = ctx.md_run(model.sk_model(), dev(s.pos), dev(v0), s.cell, dt, MASS,
                             int(round(T / dt)), phi0=PHI0, m_rep=MREP, r_cluster=s.r_cluster,
                             nu=s.nu, kT=s.kT, n_electrons=s.n_electrons, exact_forces=exact)
    E = th[:, 0] + th[:, 1]
    return E - E[0]


def test_md_with_exact_forces_matches_oracle():
    """Frames of velocity Verlet driven by the exact gradient of the truncated
    method (61-atom whole-cell clusters, nu = 12) against the oracle's."""
    torch = torch_cuda()
    from oracle import md
    from paper_1210_1531_amd import Context, model
    s = gs.make("tiny")
    v0 = gs.random_velocities(s.n_atoms, _sigma(300.0), 25)
    dt, steps = 0.25, 2
    log(f"[md exact] {s.n_atoms} atoms, {steps} steps of {dt} fs")
    ctx = Context()
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    pos, vel, F, th = ctx.md_run(model.sk_model(), dev(s.pos), dev(v0), s.cell, dt, MASS, steps,
                                 phi0=PHI0, m_rep=MREP, r_cluster=s.r_cluster, nu=s.nu, kT=s.kT,
                                 n_electrons=s.n_electrons, exact_forces=True)
    fr = md.velocity_verlet(s.pos, v0, s.cell, md.krylov_exact_forces(s, phi0=PHI0), MASS, dt,
                            steps)
    dx = np.abs(_min_image(np_(pos) - fr[-1].pos, s.cell)).max()
    dv = np.abs(np_(vel) - fr[-1].vel).max()
    dF = np.abs(np_(F) - fr[-1].F).max()
    log(f"[md exact] max |dx| {dx:.3e} A, |dv| {dv:.3e} A/fs, |dF| {dF:.3e} eV/A")
    assert dF <= F_TOL and dx <= 1e-10 and dv <= 1e-11
    for k, f in enumerate(fr):
        assert abs(th[k, 0] - f.E_pot) / s.n_atoms <= E_TOL


def test_md_energy_error_order_exact_against_rho_forces():
    """With the exact gradient the energy error of velocity Verlet is second
    order in dt (ratio 4 on halving dt, at the common times); with the forces
    through rho it stays as dt shrinks (the part of the gradient that rho
    misses does work along the path)."""
    torch = torch_cuda()
    from paper_1210_1531_amd import Context
    s = gs.make("tiny")
    v0 = gs.random_velocities(s.n_atoms, _sigma(300.0), 7)
    ctx = Context()
    rms = {}
    for exact in (True, False):
        a = _md_energy_series(ctx, s, v0, 0.25, 1.5, exact, torch)
        b = _md_energy_series(ctx, s, v0, 0.125, 1.5, exact, torch)
        rms[exact] = (np.sqrt(np.mean(a[1:] ** 2)), np.sqrt(np.mean(b[2::2] ** 2)))
    r_exact = rms[True][0] / rms[True][1]
    r_rho = rms[False][0] / rms[False][1]
    log(f"[md order] rms dE exact {rms[True][0]:.2e} -> {rms[True][1]:.2e} (ratio {r_exact:.2f}), "
        f"rho {rms[False][0]:.2e} -> {rms[False][1]:.2e} (ratio {r_rho:.2f})")
    assert 3.5 < r_exact < 4.8
    assert 0.8 < r_rho < 1.25
    assert rms[False][1] > 20 * rms[True][1]


def test_md_exact_forces_option_is_checked():
    import ctypes as C
    torch = torch_cuda()
    from paper_1210_1531_amd import Context, MagError, model
    from paper_1210_1531_amd import _lib as L
    from paper_1210_1531_amd.mag import make_opts
    s = gs.make("tiny")
    ctx = Context()
    x = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    v = torch.zeros_like(x)
    F = torch.zeros_like(x)
    thermo = np.zeros((2, 5))
    o = make_opts(nu=s.nu, kT=s.kT, n_electrons=s.n_electrons)
    cell = (C.c_double * 3)(*[float(c) for c in s.cell])
    for flag, expect in ((2, L.MAG_EINVAL), (-1, L.MAG_EINVAL)):
        md = L.MagMDOpts(dt=0.5, mass=MASS, phi0=0.0, m_rep=4.0, r_cluster=0.0, n_steps=1,
                         exact_forces=flag)
        rc = ctx._lib.mag_md_run(ctx._h, C.byref(model.sk_model()), C.byref(o), C.byref(md),
                                 s.n_atoms, cell, C.c_void_p(x.data_ptr()),
                                 C.c_void_p(v.data_ptr()), C.c_void_p(F.data_ptr()),
                                 thermo.ctypes.data_as(C.POINTER(C.c_double)), L.MAG_DEVICE)
        assert rc == expect
    # nu above the exact-gradient kernels: refused at the first frame
    with pytest.raises(MagError) as err:
        ctx.md_run(model.sk_model(), x, v, s.cell, 0.5, MASS, 1, nu=40, kT=s.kT,
                   n_electrons=s.n_electrons, exact_forces=True)
    assert err.value.status == L.MAG_EUNSUPPORTED
