"""Ordered neighbour list: the definition, by exhaustive search.

Allegro decomposes each atomic energy into a sum over *ordered* neighbour pairs
(i, j) with j inside the cutoff sphere of i (section "Allegro: Scalable
Equivariant Deep Learning", the pair-energy decomposition), so the list is a
full list: (i, j, s) and (j, i, -s) both appear.  Only the first `n_local`
atoms are centres (one GPU's spatial-decomposition share: the strictly local
model needs only atoms within r_c of its own atoms, section "Optimized
LAMMPS-Kokkos implementation").

Distance test, fixed so that any implementation can reproduce it bit for bit:
  dx = (x_j - x_i) + s_x * L_x   (same for y, z; IEEE double, no fused ops)
  d2 = (dx*dx + dy*dy) + dz*dz
  keep iff d2 < r_c*r_c and not (i == j and s == 0).
With per-ordered-species-pair cutoffs (section "Species-dependent cutoffs":
an independent cutoff for each ordered pair, so that (Z_i, Z_j) and
(Z_j, Z_i) may differ) r_c is rc[Z_i][Z_j] of the centre's and the
neighbour's species; the global r_c then only bounds the search.
The result is sorted by (i, j, s_x, s_y, s_z).
"""
from __future__ import annotations

import math

import numpy as np


def _shift_ranges(dx0: np.ndarray, L: float, r_cut: float, periodic: bool):
    """Smallest/largest integer image shift that can bring |dx0 + s L| below r_c."""
    if not periodic:
        z = np.zeros_like(dx0, dtype=np.int64)
        return z, z
    # a 1e-9 slack on the quotient keeps the range conservative under rounding;
    # the exact test decides every candidate
    lo = np.ceil((-r_cut - dx0) / L - 1e-9).astype(np.int64)
    hi = np.floor((r_cut - dx0) / L + 1e-9).astype(np.int64)
    return lo, hi


def _d2(pos, cell, i, j, s):
    L = np.where(np.asarray(cell) > 0, np.asarray(cell, dtype=np.float64), 0.0)
    dx = (pos[j, 0] - pos[i, 0]) + s[:, 0].astype(np.float64) * L[0]
    dy = (pos[j, 1] - pos[i, 1]) + s[:, 1].astype(np.float64) * L[1]
    dz = (pos[j, 2] - pos[i, 2]) + s[:, 2].astype(np.float64) * L[2]
    return (dx * dx + dy * dy) + dz * dz


def _exact_test(pos, cell, i, j, s, r_cut):
    keep = _d2(pos, cell, i, j, s) < r_cut * r_cut
    keep &= ~((i == j) & np.all(s == 0, axis=1))
    return keep


def _expand_candidates(pos, cell, pbc, r_cut, ci, cj):
    """For candidate atom pairs (ci, cj), enumerate every image shift whose
    per-axis separation can be below r_c, then apply the exact test."""
    per_axis = []
    for ax in range(3):
        dx0 = pos[cj, ax] - pos[ci, ax]
        lo, hi = _shift_ranges(dx0, float(cell[ax]) if pbc[ax] else 1.0, r_cut, bool(pbc[ax]))
        per_axis.append((lo, hi))
    counts = np.ones(ci.shape[0], dtype=np.int64)
    for lo, hi in per_axis:
        counts *= (hi - lo + 1)
    rep_i = np.repeat(ci, counts)
    rep_j = np.repeat(cj, counts)
    # local running index inside each candidate's block of shifts
    starts = np.repeat(np.cumsum(counts) - counts, counts)
    k = np.arange(rep_i.shape[0], dtype=np.int64) - starts
    s = np.empty((rep_i.shape[0], 3), dtype=np.int64)
    rem = k
    for ax in (2, 1, 0):
        lo, hi = per_axis[ax]
        span = np.repeat(hi - lo + 1, counts)
        s[:, ax] = np.repeat(lo, counts) + rem % span
        rem = rem // span
    keep = _exact_test(pos, cell, rep_i, rep_j, s, r_cut)
    return rep_i[keep], rep_j[keep], s[keep]


def neighbor_list(pos, cell, pbc, r_cut, n_local=None, method="auto", species=None, pair_cutoffs=None):
    """Return (i, j, shift) int64 arrays, sorted by (i, j, sx, sy, sz).

    `pair_cutoffs` (with `species`): [S][S] ordered cutoffs rc[Z_centre][Z_neighbour],
    each at most r_cut; a pair is kept iff d2 < rc*rc for its own species pair.

    `method="brute"` tests every (i, j) atom pair with every image shift that
    can possibly be in range (the definition).  `method="kdtree"` only changes
    how candidate atom pairs are proposed (scipy's k-d tree with a slightly
    enlarged radius, valid when every periodic box length exceeds 2 r_c);
    the exact test above still decides every pair.  "auto" picks brute force
    for small systems.
    """
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    cell = np.asarray(cell, dtype=np.float64).reshape(-1)
    if cell.shape[0] == 9:
        cell = np.array([cell[0], cell[4], cell[8]])
    pbc = np.asarray(pbc, dtype=np.int64).reshape(3)
    n = pos.shape[0]
    n_local = n if n_local is None else int(n_local)
    if method == "auto":
        method = "brute" if n_local * n <= 4_000_000 else "kdtree"
    if method == "kdtree" and np.any((pbc != 0) & (cell <= 2.0 * r_cut * (1 + 1e-6) + 1e-6)):
        method = "brute"
    if method == "brute":
        out_i, out_j, out_s = [], [], []
        chunk = max(1, 2_000_000 // max(n, 1))
        for a in range(0, n_local, chunk):
            b = min(n_local, a + chunk)
            ci = np.repeat(np.arange(a, b, dtype=np.int64), n)
            cj = np.tile(np.arange(n, dtype=np.int64), b - a)
            ii, jj, ss = _expand_candidates(pos, cell, pbc, r_cut, ci, cj)
            out_i.append(ii); out_j.append(jj); out_s.append(ss)
        i = np.concatenate(out_i); j = np.concatenate(out_j); s = np.concatenate(out_s)
    elif method == "kdtree":
        from scipy.spatial import cKDTree
        rr = r_cut * (1.0 + 1e-9) + 1e-9
        if np.any(pbc):
            box = np.where(pbc != 0, cell, 0.0)
            lo = pos.min(0)
            # non-periodic axes: make the period large enough to never wrap
            span = pos.max(0) - lo + 4 * r_cut + 1.0
            boxsize = np.where(pbc != 0, box, span)
            shifted = np.where(pbc != 0, np.mod(pos, np.where(box > 0, box, 1.0)), pos - lo)
            shifted = np.where(shifted >= boxsize, shifted - boxsize, shifted)
            tree = cKDTree(shifted, boxsize=boxsize)
        else:
            shifted = pos
            tree = cKDTree(pos)
        pairs = tree.query_pairs(rr, output_type="ndarray").astype(np.int64)
        ci = np.concatenate([pairs[:, 0], pairs[:, 1]])
        cj = np.concatenate([pairs[:, 1], pairs[:, 0]])
        m = ci < n_local
        i, j, s = _expand_candidates(pos, cell, pbc, r_cut, ci[m], cj[m])
    else:
        raise ValueError(method)
    if pair_cutoffs is not None:
        rc = np.asarray(pair_cutoffs, dtype=np.float64)
        if np.any(rc > r_cut) or np.any(rc <= 0):
            raise ValueError("pair cutoffs must lie in (0, r_cut]")
        Z = np.asarray(species, dtype=np.int64)
        rcp = rc[Z[i], Z[j]]
        keep = _d2(pos, cell, i, j, s) < rcp * rcp
        i, j, s = i[keep], j[keep], s[keep]
    order = np.lexsort((s[:, 2], s[:, 1], s[:, 0], j, i))
    return i[order], j[order], s[order]


def centre_neighbors(pos, r_cut, centres):
    """The rows of the list above for the given centres only, in a
    non-periodic system (a spatial-decomposition share with its ghost shell):
    candidates from scipy's k-d tree over all atoms with a slightly enlarged
    radius, decided by the same exact test.  Returns (i, j, shift) sorted like
    neighbor_list; shifts are zero."""
    from scipy.spatial import cKDTree
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    centres = np.unique(np.asarray(centres, dtype=np.int64))
    rr = r_cut * (1.0 + 1e-9) + 1e-9
    cand = cKDTree(pos).query_ball_point(pos[centres], rr)
    ci = np.concatenate([np.full(len(c), a, dtype=np.int64) for a, c in zip(centres, cand)])
    cj = np.concatenate([np.asarray(c, dtype=np.int64) for c in cand])
    s = np.zeros((ci.shape[0], 3), dtype=np.int64)
    keep = _exact_test(pos, np.zeros(3), ci, cj, s, r_cut)
    i, j, s = ci[keep], cj[keep], s[keep]
    order = np.lexsort((s[:, 2], s[:, 1], s[:, 0], j, i))
    return i[order], j[order], s[order]


def row_ptr(i: np.ndarray, n_local: int) -> np.ndarray:
    counts = np.bincount(i, minlength=n_local)
    return np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)


def max_image_range(cell, r_cut):
    """K = ceil(r_c / L) per axis (documentation helper for tests)."""
    return [int(math.ceil(r_cut / float(L))) if L > 0 else 0 for L in cell]
