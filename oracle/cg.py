"""Tensor-product paths and their coupling tables.

Irreps are (l, p): rotation order l and parity p = +1 (even) or -1 (odd).  The
spherical harmonics Y_l, and so the first-layer features, carry natural parity
(-1)^l.  Paths (section "Optimized tensor product"): an input pair
(l1, p1) x (l2, p2) couples to every output (l_out, p_out) with
|l1 - l2| <= l_out <= l1 + l2 and p_out = p1 p2; l_out is capped at l_max, and
paths that can never contribute to the final scalar (0, +1) outputs are
omitted.  Products of two natural-parity irreps into an output whose l is one
off in parity, e.g. 1o x 1o -> 1e (the cross product), create unnatural-parity
features; these matter once a model has three or more layers.

Coupling tensor of a path (the paper's w3j).  For given (l1, l2, l3) the
rotation-invariant trilinear forms on the three real irreps span one
dimension, so the table is fixed up to scale and sign by (l1, l2, l3) alone;
parity only decides which paths exist.  Readings (the paper fixes neither the
sign nor the normalisation):
  * l1 + l2 + l3 even: the real Gaunt coefficient
        C[m1, m2, m3] = (1 / 4 pi) \\int Y_{l1 m1} Y_{l2 m2} Y_{l3 m3} dOmega;
  * l1 + l2 + l3 odd (the Gaunt integral vanishes): the triple-product form
        C[m1, m2, m3] = (1 / 4 pi) \\int rhat . (grad Y_{l1 m1} x grad Y_{l2 m2}) Y_{l3 m3} dOmega
    with the surface gradients of the harmonics; for (1, 1, 1) it is the
    Levi-Civita symbol;
and both are rescaled to unit Frobenius norm.  The integrals are evaluated with
a product rule exact for these polynomial degrees: Gauss-Legendre in
cos(theta) times the uniform trapezoid rule in phi.

Path fusion (section "Optimized tensor product"): the paths sharing an output
irrep are combined by a learned weighted sum that is pre-computed into one
constant tensor W[a, b, c] = sum_p alpha_p C_p[a, b, c] over the strided
component indices.  Reading for the weight scale: alpha_p = raw_p / sqrt(P_out)
with raw_p ~ N(0, 1) from the weight file and P_out the number of kept paths
into that output irrep.
In the final layer only scalar outputs remain, whose couplings are diagonal in
m (delta_{m1 m2} / sqrt(2l + 1)).

Strided layout (section "Optimized tensor product"): with D = (l_max + 1)^2,
natural-parity irrep (l, (-1)^l) occupies components l^2 .. l^2 + 2l and
unnatural-parity irrep (l, -(-1)^l) components D + l^2 .. D + l^2 + 2l; a
layer whose features are all natural stores D components, otherwise 2 D.
"""
from __future__ import annotations

import functools
import math
from typing import Dict, List, Tuple

import numpy as np
import torch

from .basis import spherical_harmonics, spherical_harmonics_np


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


def _triangle(l1, l2, lo):
    return abs(l1 - l2) <= lo <= l1 + l2


@functools.lru_cache(maxsize=None)
def _surface_grads(l_max: int):
    """Harmonics [Q, D] and their surface gradients [Q, D, 3] at the quadrature points."""
    pts, _ = _quadrature()
    r = torch.tensor(pts, dtype=torch.float64, requires_grad=True)
    Y = spherical_harmonics(r / torch.linalg.norm(r, dim=1, keepdim=True), l_max)
    grads = [torch.autograd.grad(Y[:, k].sum(), r, retain_graph=True)[0] for k in range(Y.shape[1])]
    return Y.detach().numpy(), torch.stack(grads, 1).numpy()


def triple_form(l1: int, l2: int, l3: int) -> np.ndarray:
    """Unnormalised (1/4pi) \\int rhat . (grad Y_a x grad Y_b) Y_c dOmega, [2l1+1, 2l2+1, 2l3+1]."""
    pts, w = _quadrature()
    lm = max(l1, l2, l3)
    Y, dY = _surface_grads(lm)
    s = lambda l: slice(l * l, (l + 1) * (l + 1))
    cross = np.cross(dY[:, s(l1), None, :], dY[:, None, s(l2), :])          # [Q, a, b, 3]
    trip = np.einsum("qabk,qk->qab", cross, pts)
    return np.einsum("q,qab,qc->abc", w, trip, Y[:, s(l3)]) / (4.0 * math.pi)


def coupling(l1: int, l2: int, l3: int) -> np.ndarray:
    """Coupling table of a path, unit Frobenius norm (zero tensor if the
    triangle condition fails)."""
    if not _triangle(l1, l2, l3):
        return np.zeros((2 * l1 + 1, 2 * l2 + 1, 2 * l3 + 1))
    g = gaunt(l1, l2, l3) if (l1 + l2 + l3) % 2 == 0 else triple_form(l1, l2, l3)
    g[np.abs(g) < 1e-13] = 0.0
    nrm = np.linalg.norm(g)
    return g / nrm if nrm > 0 else g


def natural(l: int) -> int:
    return 1 if l % 2 == 0 else -1


def layer_paths(l_max: int, n_layers: int) -> List[List[Tuple[int, int, int, int, int]]]:
    """Kept paths (l1, p1, l2, l_out, p_out) of each layer.

    Layer inputs are the irreps the previous layer can produce (natural
    parity for the first layer, whose features are built from the
    harmonics); the second operand is always a harmonic (l2, (-1)^l2); the
    last layer keeps only (0, +1) outputs and every earlier layer only the
    outputs that the next layer uses.
    """
    Yirr = [(l, natural(l)) for l in range(l_max + 1)]
    reach = [set(Yirr)]
    for _ in range(n_layers):
        reach.append({(lo, p1 * p2) for (l1, p1) in reach[-1] for (l2, p2) in Yirr
                      for lo in range(l_max + 1) if _triangle(l1, l2, lo)})
    need = {(0, 1)}
    kept = []
    for L in range(n_layers, 0, -1):
        paths = sorted((l1, p1, l2, lo, p1 * p2) for (l1, p1) in reach[L - 1] for (l2, p2) in Yirr
                       for lo in range(l_max + 1)
                       if _triangle(l1, l2, lo) and (lo, p1 * p2) in need)
        kept.append(paths)
        need = {(l1, p1) for (l1, p1, _, _, _) in paths}
    return kept[::-1]


def has_unnatural(l_max: int, n_layers: int) -> bool:
    """Whether any layer keeps an unnatural-parity irrep (then the weight file
    uses the parity-extended alpha and mixing layouts)."""
    return any(po != natural(lo) or p1 != natural(l1)
               for P in layer_paths(l_max, n_layers) for (l1, p1, _, lo, po) in P)


def comp_offset(l: int, p: int, l_max: int) -> int:
    """First strided component of irrep (l, p)."""
    return l * l + (0 if p == natural(l) else (l_max + 1) ** 2)


def irrep_slot(l: int, p: int, l_max: int) -> int:
    """Index of irrep (l, p) among natural l = 0..l_max then unnatural l = 0..l_max."""
    return l + (0 if p == natural(l) else l_max + 1)


def width(l_max: int, irreps) -> int:
    """Strided components of a feature holding `irreps`."""
    D = (l_max + 1) ** 2
    return 2 * D if any(p != natural(l) for (l, p) in irreps) else D


def layer_widths(l_max: int, n_layers: int):
    """(input components, output components) of each layer."""
    P = layer_paths(l_max, n_layers)
    out = []
    for L, paths in enumerate(P):
        ins = {(l1, p1) for (l1, p1, _, _, _) in paths}
        outs = {(lo, po) for (_, _, _, lo, po) in paths}
        final = L == len(P) - 1
        out.append((width(l_max, ins), 1 if final else width(l_max, outs)))
    return out


def fused_table(l_max: int, paths, alpha_raw: np.ndarray, final: bool, n_in: int = None,
                n_out: int = None) -> np.ndarray:
    """W[a, b, c] over strided components (a: feature, b: harmonic, c: output).

    `alpha_raw` holds the weight-file entries: indexed [l1][l2][l_out] when
    every irrep is natural, or [s1][l1][l2][l_out] with s1 = 0 for a natural
    and 1 for an unnatural input irrep (the output parity follows).  The
    output axis has `n_out` components (1 in the final layer).
    """
    D = (l_max + 1) ** 2
    n_in = D if n_in is None else n_in
    n_out = (1 if final else D) if n_out is None else n_out
    W = np.zeros((n_in, D, n_out))
    per_out: Dict[Tuple[int, int], int] = {}
    for (_, _, _, lo, po) in paths:
        per_out[(lo, po)] = per_out.get((lo, po), 0) + 1
    alpha_raw = np.asarray(alpha_raw)
    for (l1, p1, l2, lo, po) in paths:
        if alpha_raw.ndim == 4:
            raw = alpha_raw[0 if p1 == natural(l1) else 1, l1, l2, lo]
        else:
            raw = alpha_raw[l1, l2, lo]
        a = float(raw) / math.sqrt(per_out[(lo, po)])
        C = coupling(l1, l2, lo)
        o1, oo = comp_offset(l1, p1, l_max), comp_offset(lo, po, l_max)
        W[o1:o1 + 2 * l1 + 1, l2 * l2:(l2 + 1) ** 2, oo:oo + 2 * lo + 1] += a * C
    return W
