"""Diamond-lattice carbon structures for the benchmark and parity workloads.

The paper's own systems (a ten-million-atom sp2-sp3 nano-composite carbon solid
and an amorphous polymer, described in its benchmark paragraph) are not
available, so synthetic carbon cells stand in for them: a diamond supercell
with random spherical voids, random vacancies and Gaussian displacements,
which gives the mixed local environments (bulk, surface, under-coordinated
sites) and uneven cluster sizes of the real workloads.

Draw order for a given seed (numpy PCG64):
  1. voids: centre ~ U(box), radius ~ U(rmin, rmax); remove every site within
     the radius (minimum image); repeat until the removed fraction reaches the
     target;
  2. vacancies: remove floor(p * N_remaining) distinct sites, uniformly;
  3. displacements: i.i.d. N(0, sigma^2) per Cartesian component.
Surviving atoms keep the site order (ix, iy, iz, basis).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

A_DIAMOND = 3.567  # conventional cubic lattice constant of diamond, Angstrom

# fractional coordinates of the 8 atoms of the conventional diamond cell
_BASIS = np.array(
    [
        [0.0, 0.0, 0.0],
        [0.0, 0.5, 0.5],
        [0.5, 0.0, 0.5],
        [0.5, 0.5, 0.0],
        [0.25, 0.25, 0.25],
        [0.25, 0.75, 0.75],
        [0.75, 0.25, 0.75],
        [0.75, 0.75, 0.25],
    ]
)


@dataclass
class Structure:
    """Atomic positions in an orthorhombic periodic box plus run settings."""

    pos: np.ndarray  # (N, 3) float64, Angstrom
    cell: np.ndarray  # (3,) float64, box lengths, Angstrom
    name: str = ""
    nu: int = 30  # Krylov dimension
    r_cluster: float = 6.0  # cluster radius, Angstrom (<= 0: whole cell)
    kT: float = 0.1  # electronic temperature, eV
    electrons_per_atom: float = 4.0
    meta: dict = field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_electrons(self) -> float:
        return self.electrons_per_atom * self.n_atoms


def diamond_sites(n1: int, n2: int, n3: int, a: float = A_DIAMOND):
    """All sites of an n1 x n2 x n3 diamond supercell, order (ix, iy, iz, basis)."""
    ix, iy, iz = np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij")
    origins = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    frac = origins[:, None, :] + _BASIS[None, :, :]
    pos = (frac.reshape(-1, 3) * a).astype(np.float64)
    cell = np.array([n1 * a, n2 * a, n3 * a], dtype=np.float64)
    return pos, cell


def _min_image_dist2(pos: np.ndarray, centre: np.ndarray, cell: np.ndarray) -> np.ndarray:
    d = pos - centre[None, :]
    d -= cell[None, :] * np.round(d / cell[None, :])
    return np.einsum("ij,ij->i", d, d)


def _void_candidates(centre: np.ndarray, radius: float, cells, a: float) -> np.ndarray:
    """Sites of the conventional cells that can lie within `radius` of `centre`
    (periodic wrap, two cells of margin); every other site is farther away."""
    axes = []
    for ax in range(3):
        n = int(cells[ax])
        lo = int(np.floor((centre[ax] - radius) / a)) - 2
        hi = int(np.floor((centre[ax] + radius) / a)) + 2
        axes.append(np.arange(n) if hi - lo + 1 >= n else np.unique(np.mod(np.arange(lo, hi + 1), n)))
    ix, iy, iz = np.meshgrid(*axes, indexing="ij")
    cell_id = ((ix * int(cells[1]) + iy) * int(cells[2]) + iz).ravel()
    return (cell_id[:, None] * _BASIS.shape[0] + np.arange(_BASIS.shape[0])[None, :]).ravel()


def make_structure(
    cells=(2, 2, 2),
    a: float = A_DIAMOND,
    void_frac: float = 0.0,
    void_radius=(3.0, 8.0),
    vacancy_frac: float = 0.0,
    sigma: float = 0.0,
    seed: int = 0,
    name: str = "",
    **settings,
) -> Structure:
    """Build a defective diamond cell following the draw order in the module doc."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos, cell = diamond_sites(*cells, a=a)
    n_sites = pos.shape[0]
    keep = np.ones(n_sites, dtype=bool)
    n_voids = 0
    if void_frac > 0.0:
        target = int(np.ceil(void_frac * n_sites))
        while n_sites - int(keep.sum()) < target:
            centre = rng.uniform(0.0, 1.0, size=3) * cell
            radius = rng.uniform(void_radius[0], void_radius[1])
            # only the sites near the void are tested (the same distance test,
            # so the structure is the one a test of every site gives)
            cand = _void_candidates(centre, radius, cells, a)
            keep[cand] &= _min_image_dist2(pos[cand], centre, cell) > radius * radius
            n_voids += 1
    idx = np.nonzero(keep)[0]
    n_vac = 0
    if vacancy_frac > 0.0:
        n_vac = int(np.floor(vacancy_frac * idx.size))
        drop = rng.choice(idx.size, size=n_vac, replace=False)
        mask = np.ones(idx.size, dtype=bool)
        mask[drop] = False
        idx = idx[mask]
    pos = pos[idx].copy()
    if sigma > 0.0:
        pos += rng.normal(0.0, sigma, size=pos.shape)
    pos = np.mod(pos, cell[None, :])
    meta = dict(
        cells=tuple(cells),
        a=a,
        n_sites=n_sites,
        n_voids=n_voids,
        n_vacancies=n_vac,
        sigma=sigma,
        seed=seed,
    )
    return Structure(pos=pos, cell=cell, name=name, meta=meta, **settings)


BASE_SEED = 12101531


def config_seed(k: int) -> int:
    return BASE_SEED + 100 * k


# Workload configurations (sizes, defects and settings of the five benchmark
# cases, plus small cells used by the parity tests).  Config 4 differentiates
# the cell of config 2, so it reuses config 2's structure seed.
CONFIGS = {
    1: dict(cells=(2, 2, 2), sigma=0.02, nu=30, r_cluster=0.0, seed_of=1,
            name="c64_perfect_noise"),
    2: dict(cells=(8, 8, 8), vacancy_frac=0.05, sigma=0.05, nu=30, r_cluster=6.0, seed_of=2,
            name="c4096_vac5"),
    3: dict(cells=(16, 16, 16), void_frac=0.10, sigma=0.1, nu=30, r_cluster=6.0, seed_of=3,
            name="c32768_voids"),
    4: dict(cells=(8, 8, 8), vacancy_frac=0.05, sigma=0.05, nu=30, r_cluster=6.0, seed_of=2,
            name="c4096_vac5_grad"),
    5: dict(cells=(64, 64, 32), void_frac=0.10, vacancy_frac=0.03, sigma=0.1, nu=30,
            r_cluster=6.0, seed_of=5, name="c1M_voids_vac3"),
    # small cells for exhaustive parity (not benchmark workloads)
    "mini_vac": dict(cells=(4, 4, 4), vacancy_frac=0.05, sigma=0.05, nu=30, r_cluster=6.0,
                     seed_of=11, name="c512_vac5"),
    "mini_void": dict(cells=(5, 5, 4), void_frac=0.10, void_radius=(3.0, 5.0), sigma=0.1,
                      nu=20, r_cluster=6.0, seed_of=12, name="c800_voids"),
    "tiny": dict(cells=(2, 2, 2), vacancy_frac=0.05, sigma=0.05, nu=12, r_cluster=0.0,
                 seed_of=13, name="c64_vac_tiny"),
}


def make(k, nu=None, seed=None) -> Structure:
    """Structure and settings of workload configuration ``k``."""
    spec = dict(CONFIGS[k])
    seed_of = spec.pop("seed_of")
    if seed is None:
        seed = config_seed(seed_of) if isinstance(seed_of, int) else BASE_SEED
    s = make_structure(seed=seed, **spec)
    if nu is not None:
        s.nu = int(nu)
    s.meta["config"] = k
    return s


def random_velocities(n_atoms: int, sigma: float, seed: int) -> np.ndarray:
    """(n_atoms, 3) normal velocity components of standard deviation sigma with
    the mean removed (zero total momentum for equal masses)."""
    v = np.random.default_rng(seed).normal(0.0, sigma, size=(n_atoms, 3))
    return v - v.mean(axis=0, keepdims=True)
