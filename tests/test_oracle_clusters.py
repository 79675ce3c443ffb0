"""Oracle pair lists and clusters against an independent library neighbour search."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import gen
from oracle import neighbors as nb


def _kdtree_lists(pos, cell, r):
    tree = cKDTree(np.mod(pos, cell), boxsize=cell)
    return [np.sort(np.asarray(x, dtype=np.int64)) for x in tree.query_ball_point(np.mod(pos, cell), r)]


@pytest.mark.parametrize("k", [2, "mini_void"])
def test_clusters_match_periodic_kdtree(k):
    s = gen.make(k)
    ptr, atoms = nb.all_clusters(s.pos, s.cell, s.r_cluster)
    ref = _kdtree_lists(s.pos, s.cell, s.r_cluster)
    for j in range(s.n_atoms):
        np.testing.assert_array_equal(atoms[ptr[j]:ptr[j + 1]], ref[j])
    sizes = np.diff(ptr)
    assert sizes.min() >= 1 and np.all(atoms[ptr[:-1]] <= atoms[ptr[1:] - 1])


def test_pattern_matches_periodic_kdtree():
    s = gen.make(2)
    rows = nb.block_rows(s.pos, s.cell, 2.6)
    ref = _kdtree_lists(s.pos, s.cell, 2.6)
    for j in range(s.n_atoms):
        np.testing.assert_array_equal(rows[j], ref[j])
    counts = np.array([r.size for r in rows])
    # bulk diamond: 1 + 4 first + 12 second neighbours inside 2.6 A
    assert counts.max() <= 19 and np.median(counts) >= 14


def test_whole_cell_rule():
    s = gen.make(1)
    assert nb.whole_cell(s.cell, s.r_cluster)
    assert nb.whole_cell(s.cell, 6.0)  # 12 A > 7.134 A box
    ptr, atoms = nb.all_clusters(s.pos, s.cell, 6.0)
    assert np.all(np.diff(ptr) == s.n_atoms)
    s2 = gen.make(2)
    assert not nb.whole_cell(s2.cell, 6.0)


def test_cluster_contains_pattern():
    s = gen.make("mini_vac")
    rows = nb.block_rows(s.pos, s.cell, 2.6)
    for j in range(0, s.n_atoms, 7):
        c = nb.cluster_of(s.pos, s.cell, j, s.r_cluster)
        assert np.all(np.isin(rows[j], c))
