"""Drivers of the oracle: every column, mu, rho/pi, energies and forces.

Workflow of Eq. 3, read for the oracle: (H, S) => per-column Ritz data (G) =>
mu by bisection => rho (the oracle keeps Y d on the pattern between the two
steps instead of recomputing it; both workflows give the same numbers, the
letter says the memory savings do not change the physical quantities).

Layout of the density matrix on the H/S sparsity pattern: entry p of CSR row r
and column c holds rho_{c r} as computed from column r, which is exactly the
coefficient of H_{r c} in E_band = sum_j sum_i H_{j i} rho_{i j}.  Then
  E_band = sum_p H_p rho_p,   N = sum_p S_p rho_p,
  dA/dH_p = rho_p,            dA/dS_p = -pi_p  (Hellmann-Feynman reading),
and forces follow from the Slater-Koster derivatives:
  F_I = -sum_p [rho_p dH_p/dR_I - pi_p dS_p/dR_I].
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import fermi as _fermi
from . import krylov as _kry
from . import neighbors as _nb
from . import pool as _pool
from . import sk as _sk

NORB = _nb.NORB


@dataclass
class System:
    pos: np.ndarray
    cell: np.ndarray
    r_cluster: float
    nu: int
    kT: float
    n_electrons: float
    params: _sk.SKParams
    H: object  # scipy CSR
    S: object
    rows: list  # block rows (sorted atom ids incl. self)

    @property
    def n_atoms(self):
        return self.pos.shape[0]

    @property
    def M(self):
        return NORB * self.pos.shape[0]


def build_system(struct, params: _sk.SKParams = _sk.CARBON, nu=None, r_cluster=None,
                 kT=None, n_electrons=None) -> System:
    H, S, rows = _nb.build_csr(struct.pos, struct.cell, params)
    return System(
        pos=np.asarray(struct.pos, np.float64), cell=np.asarray(struct.cell, np.float64),
        r_cluster=struct.r_cluster if r_cluster is None else r_cluster,
        nu=struct.nu if nu is None else nu,
        kT=struct.kT if kT is None else kT,
        n_electrons=struct.n_electrons if n_electrons is None else n_electrons,
        params=params, H=H, S=S, rows=rows)


# --------------------------------------------------------------------------
# per-atom work (the four columns of an atom share its cluster)
# --------------------------------------------------------------------------
@dataclass
class Geometry:
    """What one column needs: positions, box, cluster radius, Krylov
    dimension and the model (no global matrices), so that sampled columns of
    cells far too large for the dense pattern build can be computed."""
    pos: np.ndarray
    cell: np.ndarray
    r_cluster: float
    nu: int
    params: _sk.SKParams
    kT: float = 0.1
    n_electrons: float = 0.0
    rows: list = None  # block rows of every atom, or None (found per column)

    @property
    def n_atoms(self):
        return self.pos.shape[0]

    @property
    def M(self):
        return NORB * self.pos.shape[0]


def geometry(struct, params: _sk.SKParams = _sk.CARBON, nu=None) -> Geometry:
    return Geometry(pos=np.asarray(struct.pos, np.float64), cell=np.asarray(struct.cell, np.float64),
                    r_cluster=struct.r_cluster, nu=struct.nu if nu is None else int(nu),
                    params=params, kT=struct.kT, n_electrons=struct.n_electrons)


_WORK = {}


def _block_row(geo, J):
    nb = _nb.neighbors_of(geo.pos, geo.cell, J, geo.params.r_cut)
    return np.sort(np.concatenate([nb, [J]])).astype(np.int64)


def _atom_columns(args):
    J, alphas, pat_atoms, mode, full = args
    geo = _WORK["geo"]
    breakdown = _WORK.get("breakdown", _kry.BREAKDOWN)
    atoms = _nb.cluster_of(geo.pos, geo.cell, J, geo.r_cluster)
    Hc, Sc = _nb.cluster_matrices(geo.pos, geo.cell, atoms, geo.params)
    jl = int(np.searchsorted(atoms, J))
    if pat_atoms is None:
        pat_atoms = _block_row(geo, J)
    pat_local = np.searchsorted(atoms, pat_atoms)
    pat_rows = (NORB * pat_local[:, None] + np.arange(NORB)[None, :]).ravel()
    out = []
    for a in alphas:
        l = NORB * jl + a
        if mode == "K":
            res = _kry.column_mode_k(Hc, Sc, l, geo.nu, breakdown=breakdown)
        else:
            res = _kry.column_mode_d(Hc, Sc, l)
        ypd = res.Y[pat_rows, :] * res.d[None, :]
        item = dict(j=NORB * J + a, eps=res.eps, w=res.w, nu_eff=res.nu_eff, ypd=ypd)
        if full:
            item["Y"] = res.Y
            item["d"] = res.d
            item["atoms"] = atoms
        out.append(item)
    return out


def _init_worker(geo, breakdown=_kry.BREAKDOWN):
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover - threadpoolctl is optional
        pass
    _WORK["geo"] = geo
    _WORK["breakdown"] = breakdown


def column_data(sysm, cols=None, mode="K", workers=None, full=False, breakdown=None):
    """Ritz data for the given global columns (all if None).

    sysm: a System or a Geometry.  Returns a dict with arrays eps, w (ncols x
    width, zero-padded), nu_eff, the column ids, and per-column lists ypd
    (pattern rows x nu_eff) and, if ``full``, the full Ritz vectors and
    cluster atoms.  With workers > 1 the atoms are spread over fork-server
    processes (oracle.pool); a worker that dies raises.  breakdown: the
    relative residual below which a Krylov space counts as invariant
    (default krylov.BREAKDOWN).
    """
    breakdown = _kry.BREAKDOWN if breakdown is None else float(breakdown)
    M = sysm.M
    cols = np.arange(M) if cols is None else np.asarray(cols, dtype=np.int64)
    by_atom = {}
    for j in cols:
        by_atom.setdefault(int(j) // NORB, []).append(int(j) % NORB)
    rows = getattr(sysm, "rows", None)
    tasks = [(J, sorted(a), None if rows is None else rows[J], mode, full)
             for J, a in sorted(by_atom.items())]
    geo = Geometry(pos=sysm.pos, cell=sysm.cell, r_cluster=sysm.r_cluster, nu=sysm.nu,
                   params=sysm.params)
    workers = workers or _pool.default_workers()
    if workers > 1 and len(tasks) > 8:
        with _pool.executor(workers, initializer=_init_worker, initargs=(geo, breakdown)) as ex:
            chunks = list(ex.map(_atom_columns, tasks,
                                 chunksize=max(1, len(tasks) // (8 * workers))))
    else:
        saved = dict(_WORK)
        _WORK["geo"] = geo
        _WORK["breakdown"] = breakdown
        try:
            chunks = [_atom_columns(t) for t in tasks]
        finally:
            _WORK.clear()
            _WORK.update(saved)
    items = {it["j"]: it for ch in chunks for it in ch}
    width = max([it["eps"].size for it in items.values()] + [1])
    n = cols.size
    eps = np.zeros((n, width))
    w = np.zeros((n, width))
    nu_eff = np.zeros(n, dtype=np.int64)
    ypd, extra = [], []
    for i, j in enumerate(cols):
        it = items[int(j)]
        k = it["eps"].size
        eps[i, :k] = it["eps"]
        w[i, :k] = it["w"]
        nu_eff[i] = it["nu_eff"]
        ypd.append(it["ypd"])
        extra.append(it if full else None)
    return dict(cols=cols, eps=eps, w=w, nu_eff=nu_eff, ypd=ypd, full=extra)


def valid_terms(cd):
    mask = np.arange(cd["eps"].shape[1])[None, :] < cd["nu_eff"][:, None]
    return cd["eps"][mask], cd["w"][mask]


def chemical_potential(sysm: System, cd, tol=1e-12):
    e, w = valid_terms(cd)
    mu, _ = _fermi.bisect_mu(e, w, sysm.kT, sysm.n_electrons, tol=tol)
    return mu


def density_on_pattern(sysm: System, cd, mu):
    """rho and pi in the CSR layout of H (requires every column)."""
    H = sysm.H
    rho = np.zeros(H.nnz)
    pi = np.zeros(H.nnz)
    for i, j in enumerate(cd["cols"]):
        k = cd["nu_eff"][i]
        e = cd["eps"][i, :k]
        f = _fermi.fermi((e - mu) / sysm.kT)
        lo, hi = H.indptr[j], H.indptr[j + 1]
        rho[lo:hi] = _kry.G_SPIN * (cd["ypd"][i] @ f)
        pi[lo:hi] = _kry.G_SPIN * (cd["ypd"][i] @ (f * e))
    return rho, pi


def energies(sysm: System, cd, mu):
    """(E_band, A_free, S_ent, N) from the spectral data."""
    e, w = valid_terms(cd)
    E, S_ent, N = _fermi.band_energy(mu, e, w, sysm.kT)
    return E, E - sysm.kT * S_ent, S_ent, N


def forces(sysm: System, rho, pi, rows=None):
    """F_I = -sum_p [rho_p dH_p/dR_I - pi_p dS_p/dR_I] over the CSR pattern.

    rows: block rows to contract (all if None).  F_I is complete when the
    rows of I and of every pattern neighbour of I are among them, and only
    their entries of rho and pi are read.
    """
    n = sysm.n_atoms
    dA = np.zeros((n, 3))
    H = sysm.H
    for J in (range(n) if rows is None else rows):
        ks = sysm.rows[J]
        nb = ks.size
        for t, K in enumerate(ks):
            if K == J:
                continue
            d = _nb.min_image(sysm.pos[K] - sysm.pos[J], sysm.cell)
            gH, gS = _sk.pair_block_grads(d, sysm.params)
            rb = np.zeros((NORB, NORB))
            pb = np.zeros((NORB, NORB))
            for a in range(NORB):
                base = H.indptr[NORB * J + a] + NORB * t
                rb[a] = rho[base:base + NORB]
                pb[a] = pi[base:base + NORB]
            g = np.einsum("cab,ab->c", gH, rb) - np.einsum("cab,ab->c", gS, pb)
            dA[K] += g
            dA[J] -= g
        assert nb == ks.size
    return -dA


def icohp(sysm: System, rho):
    """Integrated crystal orbital Hamiltonian populations, Eqs. 4-8.

    The COHP of Eq. 4 integrated against f (Eq. 5) is, through Eq. 2, a sum of
    H times rho over the orbitals of the atom pair.  For block t of block row J
    (column atom K): B = sum_ab H_{Ja;Kb} rho_{Kb;Ja}, with rho in the CSR
    layout of H (entry (Ja, Kb) holds rho_{Kb;Ja}, from column Ja).  B_sigma
    and B_pi replace H by its sigma and pi parts (Eq. 8); they are zero on the
    diagonal blocks, which carry on-site terms only.  Returns three arrays in
    block-CSR order.
    """
    H = sysm.H
    B, Bs, Bp = [], [], []
    for J in range(sysm.n_atoms):
        ks = sysm.rows[J]
        for t, K in enumerate(ks):
            hb = np.zeros((NORB, NORB))
            rb = np.zeros((NORB, NORB))
            for a in range(NORB):
                base = H.indptr[NORB * J + a] + NORB * t
                hb[a] = H.data[base:base + NORB]
                rb[a] = rho[base:base + NORB]
            B.append(float(np.sum(hb * rb)))
            if K == J:
                Bs.append(0.0)
                Bp.append(0.0)
            else:
                d = _nb.min_image(sysm.pos[K] - sysm.pos[J], sysm.cell)
                hs, hp = _sk.hopping_sigma_pi(d, sysm.params)
                Bs.append(float(np.sum(hs * rb)))
                Bp.append(float(np.sum(hp * rb)))
    return np.array(B), np.array(Bs), np.array(Bp)


def cohp(sysm: System, cd, energies, eta, atoms=None):
    """Energy-resolved crystal orbital Hamiltonian population, Eq. 4, at
    z = e + i eta (eta > 0 in place of the limit i0).

    For block t of block row J (column atom K):
      C(e) = -(g_s / pi) sum_ab H_{Ja;Kb} Im G_{Kb;Ja}(e + i eta),
    with the Galerkin column G_{Kb;j}(z) = sum_k Y_{Kb,k} d_k / (z - eps_k) of
    column j = (J, a) (its pattern rows are cd["ypd"]).  g_s = 2 as in rho, so
    that integrating against f(e - mu) gives the ICOHP of Eq. 5.  Returns an
    array (blocks in block-CSR order, energies); with `atoms`, the blocks of
    those block rows only, in the given order (cd needs their columns only).
    """
    H = sysm.H
    z = np.asarray(energies, dtype=np.float64) + 1j * eta
    where = {int(j): i for i, j in enumerate(cd["cols"])}
    out = []
    for J in (range(sysm.n_atoms) if atoms is None else atoms):
        for t, _ in enumerate(sysm.rows[J]):
            acc = np.zeros(z.size)
            for a in range(NORB):
                j = NORB * J + a
                i = where[j]
                k = cd["nu_eff"][i]
                G = cd["ypd"][i][NORB * t:NORB * t + NORB, :k] @ (
                    1.0 / (z[None, :] - cd["eps"][i, :k][:, None]))
                h = H.data[H.indptr[j] + NORB * t:H.indptr[j] + NORB * t + NORB]
                acc += -(_kry.G_SPIN / np.pi) * (h @ G).imag
            out.append(acc)
    return np.array(out)


@dataclass
class Result:
    mu: float
    E_band: float
    A_free: float
    S_ent: float
    N: float
    rho: np.ndarray
    pi: np.ndarray
    cd: dict
    F: np.ndarray = None


def solve(sysm: System, mode="K", workers=None, with_forces=False, mu=None,
          breakdown=None) -> Result:
    """Full forward (and optionally forces) over every column."""
    cd = column_data(sysm, None, mode=mode, workers=workers, breakdown=breakdown)
    if mu is None:
        mu = chemical_potential(sysm, cd)
    E, A, S_ent, N = energies(sysm, cd, mu)
    rho, pi = density_on_pattern(sysm, cd, mu)
    res = Result(mu=mu, E_band=E, A_free=A, S_ent=S_ent, N=N, rho=rho, pi=pi, cd=cd)
    if with_forces:
        res.F = forces(sysm, rho, pi)
    return res


# --------------------------------------------------------------------------
# mode W: the whole system, exactly (tiny cells only)
# --------------------------------------------------------------------------
@dataclass
class Exact:
    eps: np.ndarray
    Y: np.ndarray
    mu: float
    E_band: float
    A_free: float
    N: float
    rho: np.ndarray  # dense M x M
    pi: np.ndarray

    @property
    def omega(self):
        """Grand potential A - mu N (its R-gradient at fixed mu equals that of A at fixed N)."""
        return self.A_free - self.mu * self.N


def solve_exact(sysm: System, tol=1e-12, mu=None) -> Exact:
    Hd = sysm.H.toarray()
    Sd = sysm.S.toarray()
    eps, Y = sla.eigh(Hd, Sd)
    w = np.full(eps.size, _kry.G_SPIN)
    if mu is None:
        mu, _ = _fermi.bisect_mu(eps, w, sysm.kT, sysm.n_electrons, tol=tol)
    E, S_ent, N = _fermi.band_energy(mu, eps, w, sysm.kT)
    f = _fermi.fermi((eps - mu) / sysm.kT)
    rho = _kry.G_SPIN * (Y * f[None, :]) @ Y.T
    pi = _kry.G_SPIN * (Y * (f * eps)[None, :]) @ Y.T
    return Exact(eps=eps, Y=Y, mu=mu, E_band=E, A_free=E - sysm.kT * S_ent, N=N, rho=rho, pi=pi)


def green_exact(sysm: System, z, cols):
    """Columns of (zS - H)^-1 by dense solves."""
    Hd = sysm.H.toarray()
    Sd = sysm.S.toarray()
    B = np.zeros((sysm.M, len(cols)), dtype=np.complex128)
    for i, j in enumerate(cols):
        B[j, i] = 1.0
    return np.linalg.solve(z * Sd - Hd, B)


def pattern_of_dense(sysm: System, dense):
    """Gather a dense M x M matrix X onto the CSR layout: entry (r, c) -> X[c, r]."""
    H = sysm.H
    out = np.zeros(H.nnz)
    for r in range(sysm.M):
        lo, hi = H.indptr[r], H.indptr[r + 1]
        out[lo:hi] = dense[H.indices[lo:hi], r]
    return out
