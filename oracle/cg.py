"""Tensor-product paths and their coupling tables.

Paths (section "Optimized tensor product"): every input pair of irreps
(l1, p1) x (l2, p2) couples to every output (l_out, p_out) with
|l1 - l2| <= l_out <= l1 + l2 and p_out = p1 p2; paths that can never
contribute to the final scalar outputs are omitted, and l_out is capped at
l_max.  Here every feature and every spherical harmonic carries natural parity
(-1)^l, which holds for models of at most two layers.

Coupling tensor of a path (the paper's w3j): for natural-parity real harmonics
the coupling is the real Gaunt coefficient
    C[m1, m2, m3] = (1 / 4 pi) \\int Y_{l1 m1} Y_{l2 m2} Y_{l3 m3} dOmega,
rescaled to unit Frobenius norm (reading: the paper fixes neither sign nor
normalisation; once Y is fixed the Gaunt form has no sign freedom).  The
integral is evaluated with a product rule exact for these polynomial degrees:
Gauss-Legendre in cos(theta) times the uniform trapezoid rule in phi.

Path fusion (section "Optimized tensor product"): the paths sharing an output
irrep are combined by a learned weighted sum that is pre-computed into one
constant tensor W[a, b, c] = sum_p alpha_p C_p[a, b, c] over the strided
component indices.  Reading for the weight scale: alpha_p = raw_p / sqrt(P_out)
with raw_p ~ N(0, 1) from the weight file and P_out the number of kept paths
into that output irrep.
In the final layer only scalar outputs remain, whose couplings are diagonal in
m (delta_{m1 m2} / sqrt(2l + 1)).
"""
from __future__ import annotations

import functools
import math
from typing import Dict, List, Tuple

import numpy as np

from .basis import spherical_harmonics_np


@functools.lru_cache(maxsize=None)
def _quadrature(n_theta: int = 16, n_phi: int = 32):
    ct, wt = np.polynomial.legendre.leggauss(n_theta)
    phi = 2.0 * math.pi * np.arange(n_phi) / n_phi
    st = np.sqrt(1.0 - ct * ct)
    pts = np.stack([np.outer(st, np.cos(phi)).ravel(), np.outer(st, np.sin(phi)).ravel(),
                    np.repeat(ct, n_phi)], axis=1)
    w = np.repeat(wt, n_phi) * (2.0 * math.pi / n_phi)
    return pts, w


def gaunt(l1: int, l2: int, l3: int) -> np.ndarray:
    """Unnormalised real Gaunt tensor [2l1+1, 2l2+1, 2l3+1] (mean over the sphere)."""
    pts, w = _quadrature()
    lm = max(l1, l2, l3)
    Y = spherical_harmonics_np(pts, lm)
    s = lambda l: Y[:, l * l:(l + 1) * (l + 1)]
    return np.einsum("q,qa,qb,qc->abc", w, s(l1), s(l2), s(l3)) / (4.0 * math.pi)


def coupling(l1: int, l2: int, l3: int) -> np.ndarray:
    """Gaunt tensor rescaled to unit Frobenius norm (zero tensor if it vanishes)."""
    g = gaunt(l1, l2, l3)
    g[np.abs(g) < 1e-13] = 0.0
    nrm = np.linalg.norm(g)
    return g / nrm if nrm > 0 else g


def _couples(l1, l2, lo):
    return abs(l1 - l2) <= lo <= l1 + l2 and (l1 + l2 + lo) % 2 == 0


def layer_paths(l_max: int, n_layers: int) -> List[List[Tuple[int, int, int]]]:
    """Kept paths (l1, l2, l_out) of each layer, after backward pruning.

    Features and harmonics hold irreps l = 0..l_max of natural parity; the
    last layer keeps only scalar outputs; an earlier layer keeps only outputs
    that some later layer can still couple into a kept input.
    """
    if n_layers > 2:
        raise NotImplementedError("more than two layers needs odd-parity paths")
    ls = range(l_max + 1)
    need = {0}
    kept: List[List[Tuple[int, int, int]]] = []
    for L in range(n_layers, 0, -1):
        paths = [(l1, l2, lo) for l1 in ls for l2 in ls for lo in ls
                 if lo in need and _couples(l1, l2, lo)]
        kept.append(paths)
        need = {l1 for (l1, _, _) in paths}
    return kept[::-1]


def fused_table(l_max: int, paths, alpha_raw: np.ndarray, final: bool) -> np.ndarray:
    """W[a, b, c] over strided components (a: feature, b: harmonic, c: output).

    `alpha_raw[l1, l2, l_out]` are the weight-file entries; the output axis has
    (l_max+1)^2 components, or 1 in the final layer.
    """
    dim = (l_max + 1) ** 2
    n_out = 1 if final else dim
    W = np.zeros((dim, dim, n_out))
    per_out: Dict[int, int] = {}
    for (_, _, lo) in paths:
        per_out[lo] = per_out.get(lo, 0) + 1
    for (l1, l2, lo) in paths:
        a = float(alpha_raw[l1, l2, lo]) / math.sqrt(per_out[lo])
        C = coupling(l1, l2, lo)
        W[l1 * l1:(l1 + 1) ** 2, l2 * l2:(l2 + 1) ** 2, lo * lo:lo * lo + (2 * lo + 1)] += a * C
    return W
