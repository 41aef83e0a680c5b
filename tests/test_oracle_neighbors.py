"""Pins of the oracle neighbour list (CPU only).

The list is defined by exhaustive search (section "Allegro: Scalable
Equivariant Deep Learning": ordered pairs within the cutoff).  It is checked
against scipy's k-d tree (an independent library search), closed-form image
counts, the ordered-pair symmetry and the strict cutoff tie rule.  The
per-ordered-species-pair cutoffs (section "Species-dependent cutoffs") are
checked against a pure-Python loop over every atom pair and image.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import workloads as W
from oracle.neighbors import centre_neighbors, neighbor_list


def _as_set(i, j, s):
    return set(zip(i.tolist(), j.tolist(), map(tuple, s.tolist())))


@pytest.mark.parametrize("cfg", [1, 2])
def test_matches_scipy_kdtree(cfg):
    mc = W.model_config(cfg)
    s = W.system(cfg)
    i, j, sh = neighbor_list(s.pos, s.cell, s.pbc, mc.r_cut, method="brute")
    # scipy's own distance on the minimum image (box > 2 r_c here)
    tree = cKDTree(s.pos, boxsize=s.cell)
    pairs = tree.query_pairs(mc.r_cut, output_type="ndarray")
    d = s.pos[pairs[:, 1]] - s.pos[pairs[:, 0]]
    d -= np.round(d / s.cell) * s.cell
    dist = np.sqrt((d * d).sum(1))
    near_tie = np.abs(dist - mc.r_cut) < 1e-9
    assert not near_tie.any()
    ref = set()
    for (a, b) in pairs.tolist():
        ref.add((a, b)); ref.add((b, a))
    got = set(zip(i.tolist(), j.tolist()))
    assert got == ref
    assert len(got) == len(i)  # one image per pair when L > 2 r_c


def test_sorted_and_symmetric():
    mc = W.model_config(1)
    s = W.system(1)
    i, j, sh = neighbor_list(s.pos, s.cell, s.pbc, mc.r_cut)
    key = np.lexsort((sh[:, 2], sh[:, 1], sh[:, 0], j, i))
    assert np.array_equal(key, np.arange(len(i)))
    st = _as_set(i, j, sh)
    assert all((b, a, (-x, -y, -z)) in st for (a, b, (x, y, z)) in st)


def test_kdtree_candidates_equal_brute():
    mc = W.model_config(2)
    s = W.system(2)
    a = neighbor_list(s.pos, s.cell, s.pbc, mc.r_cut, method="brute")
    b = neighbor_list(s.pos, s.cell, s.pbc, mc.r_cut, method="kdtree")
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_single_atom_small_box_images():
    # one atom in a cube of side 3 with r_c = 4: images at |s| L < 4 -> the 6 face images
    pos = np.array([[0.5, 1.0, 2.0]])
    i, j, s = neighbor_list(pos, [3.0, 3.0, 3.0], [1, 1, 1], 4.0)
    assert len(i) == 6 and np.all(np.abs(s).sum(1) == 1)
    # r_c = 4.5: |s|^2 <= 2 -> 6 + 12 = 18 images
    i, j, s = neighbor_list(pos, [3.0, 3.0, 3.0], [1, 1, 1], 4.5)
    assert len(i) == 18


def test_cutoff_tie_is_excluded():
    pos = np.array([[1.0, 2.0, 3.0], [5.0, 2.0, 3.0], [1.0, 5.5, 3.0]])
    i, j, s = neighbor_list(pos, [0, 0, 0], [0, 0, 0], 4.0)
    got = _as_set(i, j, s)
    assert (0, 1, (0, 0, 0)) not in got          # d = 4 exactly
    assert (0, 2, (0, 0, 0)) in got              # d = 3.5
    # periodic tie: image across a 20 A box at exactly 4 A
    pos = np.array([[1.0, 1.0, 1.0], [17.0, 1.0, 1.0]])
    i, j, s = neighbor_list(pos, [20.0, 20.0, 20.0], [1, 1, 1], 4.0)
    assert len(i) == 0
    pos = np.array([[1.0, 1.0, 1.0], [17.25, 1.0, 1.0]])
    i, j, s = neighbor_list(pos, [20.0, 20.0, 20.0], [1, 1, 1], 4.0)
    assert _as_set(i, j, s) == {(0, 1, (-1, 0, 0)), (1, 0, (1, 0, 0))}


def test_ghost_shell_list_matches_periodic():
    """Centres of a non-periodic box plus its periodic-image ghost shell see
    exactly the neighbours of the periodic box (strict locality, section
    "Optimized LAMMPS-Kokkos implementation")."""
    mc = W.model_config(1)
    s = W.system(1)
    g = W.ghost_shell(s, mc.r_cut + 0.5)
    i0, j0, s0 = neighbor_list(s.pos, s.cell, s.pbc, mc.r_cut)
    i1, j1, s1 = neighbor_list(g.pos, g.cell, g.pbc, mc.r_cut, n_local=g.n_local)
    assert np.all(s1 == 0)
    own = np.concatenate([np.arange(s.n_local), g.ghost_owner])
    assert np.array_equal(i0, i1) or sorted(zip(i0, own[j1])) == sorted(zip(i0, j0))
    assert sorted(zip(i1.tolist(), own[j1].tolist())) == sorted(zip(i0.tolist(), j0.tolist()))


def test_centre_rows_equal_the_brute_force_rows():
    """Rows of chosen centres of a ghost-shell share (non-periodic, ghosts
    after the centres) equal the brute-force list's rows for them, including
    a centre whose neighbours are ghosts and an exact-cutoff tie."""
    mc = W.model_config(1)
    g = W.ghost_shell(W.system(1), mc.r_cut + 0.5)
    pos = g.pos.copy()
    # a pair at exactly r_c from centre 3 along x: excluded by the strict test
    pos[5] = pos[3] + np.array([mc.r_cut, 0.0, 0.0])
    i0, j0, s0 = neighbor_list(pos, g.cell, g.pbc, mc.r_cut, n_local=g.n_local, method="brute")
    cents = np.array([0, 3, 5, 17, g.n_local - 1])
    i1, j1, s1 = centre_neighbors(pos, mc.r_cut, cents[::-1])
    m = np.isin(i0, cents)
    assert np.array_equal(i1, i0[m]) and np.array_equal(j1, j0[m]) and np.array_equal(s1, s0[m])
    assert not np.any((i1 == 3) & (j1 == 5))
    assert np.any(j1 >= g.n_local)


def _loop_pairs(pos, cell, pbc, Z, table, r_max):
    """The definition, written out: every (i, j, image) with
    d2 < rc[Z_i][Z_j]^2 (d2 summed in the order the list fixes)."""
    n = len(pos)
    rng = [range(-(int(r_max // cell[a]) + 1), int(r_max // cell[a]) + 2) if pbc[a] else range(0, 1)
           for a in range(3)]
    out = set()
    for i in range(n):
        for j in range(n):
            rc = table[Z[i]][Z[j]]
            for sx in rng[0]:
                for sy in rng[1]:
                    for sz in rng[2]:
                        if i == j and sx == 0 and sy == 0 and sz == 0:
                            continue
                        dx = (pos[j][0] - pos[i][0]) + sx * cell[0]
                        dy = (pos[j][1] - pos[i][1]) + sy * cell[1]
                        dz = (pos[j][2] - pos[i][2]) + sz * cell[2]
                        if (dx * dx + dy * dy) + dz * dz < rc * rc:
                            out.add((i, j, (sx, sy, sz)))
    return out


def _water_like(n_side, spacing, seed):
    return W.jittered_lattice_box(n_side ** 3, n_side * spacing, 0.4, W.WATER_MIX, seed, sites_per_side=n_side)


def test_pair_cutoffs_match_loop_definition():
    s = _water_like(3, 2.9, 21)           # 27 atoms, 8.7 A box (< 2 r_c: several images)
    table = W.paper_pair_cutoffs(2, 4.0)   # H-H 3.0, H-O 1.25, O-H 3.0, O-O 4.0
    i, j, sh = neighbor_list(s.pos, s.cell, s.pbc, 4.0, species=s.species, pair_cutoffs=table)
    ref = _loop_pairs(s.pos.tolist(), [float(c) for c in s.cell], s.pbc, s.species.tolist(), table, 4.0)
    assert _as_set(i, j, sh) == ref and len(ref) == len(i) > 0
    full = neighbor_list(s.pos, s.cell, s.pbc, 4.0)
    assert len(i) < 0.7 * len(full[0])     # far fewer ordered pairs than with one 4 A cutoff


def test_pair_cutoffs_equal_to_r_cut_change_nothing():
    s = _water_like(4, 3.1, 5)
    a = neighbor_list(s.pos, s.cell, s.pbc, 4.0)
    b = neighbor_list(s.pos, s.cell, s.pbc, 4.0, species=s.species, pair_cutoffs=[[4.0, 4.0], [4.0, 4.0]])
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_pair_cutoffs_are_ordered():
    s = _water_like(4, 3.1, 8)
    table = W.paper_pair_cutoffs(2, 4.0)
    i, j, sh = neighbor_list(s.pos, s.cell, s.pbc, 4.0, species=s.species, pair_cutoffs=table)
    L = np.asarray(s.cell, dtype=np.float64)
    d = np.linalg.norm(s.pos[j] - s.pos[i] + sh * L, axis=1)
    Z = s.species
    h_o = (Z[i] == 0) & (Z[j] == 1)
    o_h = (Z[i] == 1) & (Z[j] == 0)
    assert np.all(d[h_o] < 1.25) and np.all(d[o_h] < 3.0)
    # O-H pairs between 1.25 and 3 A are kept from the O side only
    kept = _as_set(i, j, sh)
    one_sided = [(a, b, c) for (a, b, c), dd in zip(zip(i.tolist(), j.tolist(), map(tuple, sh.tolist())), d)
                 if Z[a] == 1 and Z[b] == 0 and dd >= 1.25]
    assert one_sided
    assert all((b, a, tuple(-x for x in c)) not in kept for (a, b, c) in one_sided)


def test_paper_pair_cutoff_table_matches_printed_values():
    """The table the code uses for the paper's cutoffs equals the printed one
    (tests/golden/pair_cutoffs_training_details.txt), ordering included."""
    import os
    names = ("H", "C", "N", "O")
    listed, default = {}, None
    with open(os.path.join(os.path.dirname(__file__), "golden", "pair_cutoffs_training_details.txt")) as f:
        for line in f:
            parts = line.split("#", 1)[0].split()
            if not parts:
                continue
            if parts[0] == "default":
                default = float(parts[1])
            else:
                listed[(parts[0], parts[1])] = float(parts[2])
    table = W.paper_pair_cutoffs(4, default)
    for a, za in enumerate(names):
        for b, zb in enumerate(names):
            assert table[a][b] == listed.get((za, zb), default), (za, zb)
    assert table[0][1] == 1.25 and table[1][0] == default       # H-C restricted, C-H not
    two = W.paper_pair_cutoffs(2, default)                       # (H, O) mix
    assert two == ((3.0, 1.25), (3.0, default))
