"""Brute-force pair lists, the H/S sparsity pattern and per-atom clusters (oracle).

Everything here is O(N) per atom with plain minimum-image distances in an
orthorhombic periodic box: no cell lists, no sorting tricks.

Cluster rule (a reading; the letter only says that G is generated column by
column in the LCAO basis, Eq. 1 and the paragraph after it): the cluster of
atom J holds every atom I with |R_I - R_J|_min-image <= r_c (inclusive), J
included, with all four orbitals of each atom, ordered by atom id then
orbital.  When r_c <= 0, or 2 r_c exceeds the shortest box length (so that
minimum images stop being unique), the cluster is the whole cell.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import sk as _sk

NORB = 4  # s, px, py, pz


def min_image(d: np.ndarray, cell: np.ndarray) -> np.ndarray:
    return d - cell * np.round(d / cell)


def dist2_from(pos: np.ndarray, cell: np.ndarray, j: int) -> np.ndarray:
    d = min_image(pos - pos[j][None, :], cell[None, :])
    return np.einsum("ij,ij->i", d, d)


def whole_cell(cell: np.ndarray, r_cluster: float) -> bool:
    return r_cluster <= 0.0 or 2.0 * r_cluster > float(np.min(cell))


def cluster_of(pos: np.ndarray, cell: np.ndarray, j: int, r_cluster: float) -> np.ndarray:
    """Sorted atom ids of the cluster of atom j."""
    if whole_cell(cell, r_cluster):
        return np.arange(pos.shape[0], dtype=np.int64)
    return np.nonzero(dist2_from(pos, cell, j) <= r_cluster * r_cluster)[0].astype(np.int64)


def all_clusters(pos: np.ndarray, cell: np.ndarray, r_cluster: float):
    """(clus_ptr, clus_atoms) for every atom, brute force."""
    n = pos.shape[0]
    lists = [cluster_of(pos, cell, j, r_cluster) for j in range(n)]
    ptr = np.zeros(n + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([x.size for x in lists])
    atoms = np.concatenate(lists).astype(np.int64) if n else np.zeros(0, np.int64)
    return ptr, atoms


def neighbors_of(pos: np.ndarray, cell: np.ndarray, j: int, r_cut: float) -> np.ndarray:
    """Sorted atom ids K != j with |R_K - R_j| < r_cut (the pattern of atom j)."""
    d2 = dist2_from(pos, cell, j)
    nb = np.nonzero(d2 < r_cut * r_cut)[0]
    return nb[nb != j].astype(np.int64)


def block_rows(pos: np.ndarray, cell: np.ndarray, r_cut: float):
    """For every atom J: sorted list of atoms K in its block row (J itself included)."""
    rows = []
    for j in range(pos.shape[0]):
        nb = neighbors_of(pos, cell, j, r_cut)
        rows.append(np.sort(np.concatenate([nb, [j]])).astype(np.int64))
    return rows


def build_csr(pos: np.ndarray, cell: np.ndarray, p: _sk.SKParams = _sk.CARBON):
    """Global H and S as scipy CSR matrices plus the block rows.

    Row (J, a) lists, for every atom K of the block row of J in ascending order,
    the four columns (K, 0..3).  Diagonal blocks are the onsite H and the
    identity S.
    """
    n = pos.shape[0]
    m = NORB * n
    rows = block_rows(pos, cell, p.r_cut)
    indptr = np.zeros(m + 1, dtype=np.int64)
    nnz_row = np.repeat([NORB * len(r) for r in rows], NORB)
    indptr[1:] = np.cumsum(nnz_row)
    nnz = int(indptr[-1])
    indices = np.zeros(nnz, dtype=np.int64)
    hv = np.zeros(nnz)
    sv = np.zeros(nnz)
    h_on = _sk.onsite_h(p)
    for j in range(n):
        ks = rows[j]
        blocks_h = []
        blocks_s = []
        for k in ks:
            if k == j:
                blocks_h.append(h_on)
                blocks_s.append(np.eye(NORB))
            else:
                d = min_image(pos[k] - pos[j], cell)
                bh, bs = _sk.pair_blocks(d, p)
                blocks_h.append(bh)
                blocks_s.append(bs)
        for a in range(NORB):
            r = NORB * j + a
            lo = indptr[r]
            cols = (NORB * ks[:, None] + np.arange(NORB)[None, :]).ravel()
            indices[lo:lo + cols.size] = cols
            hv[lo:lo + cols.size] = np.concatenate([b[a] for b in blocks_h])
            sv[lo:lo + cols.size] = np.concatenate([b[a] for b in blocks_s])
    H = sp.csr_matrix((hv, indices, indptr), shape=(m, m))
    S = sp.csr_matrix((sv, indices, indptr), shape=(m, m))
    return H, S, rows


def cluster_matrices(pos: np.ndarray, cell: np.ndarray, atoms: np.ndarray,
                     p: _sk.SKParams = _sk.CARBON):
    """Dense principal submatrices H[C, C] and S[C, C] of a cluster.

    Built straight from the positions of the cluster's atoms (pairs inside the
    cluster closer than r_cut), which is the same as cutting the rows and
    columns of C out of the global matrices.
    """
    na = atoms.size
    n = NORB * na
    Hc = np.zeros((n, n))
    Sc = np.zeros((n, n))
    h_on = _sk.onsite_h(p)
    P = pos[atoms]
    for a in range(na):
        Hc[NORB * a:NORB * a + NORB, NORB * a:NORB * a + NORB] = h_on
        Sc[NORB * a:NORB * a + NORB, NORB * a:NORB * a + NORB] = np.eye(NORB)
        d = min_image(P - P[a][None, :], cell[None, :])
        r2 = np.einsum("ij,ij->i", d, d)
        for b in np.nonzero(r2 < p.r_cut * p.r_cut)[0]:
            if b == a:
                continue
            bh, bs = _sk.pair_blocks(d[b], p)
            Hc[NORB * a:NORB * a + NORB, NORB * b:NORB * b + NORB] = bh
            Sc[NORB * a:NORB * a + NORB, NORB * b:NORB * b + NORB] = bs
    return Hc, Sc
