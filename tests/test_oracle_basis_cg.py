"""Pins of the oracle's edge basis and coupling tables (CPU only).

Envelope: closed-form boundary values.  Bessel: orthonormality on [0, r_c]
with weight r^2 (scipy quadrature).  Spherical harmonics: the addition theorem
with scipy's Legendre polynomials, parity, orthonormality on the sphere.
Couplings: sympy's exact real Gaunt coefficients, rotation equivariance, the final-layer diagonal form, and the
path/non-zero counts of the fused tables.  Odd (l1 + l2 + l3) couplings, which the Gaunt integral cannot
give: the Levi-Civita closed form of 1 x 1 -> 1, antisymmetry for l1 = l2, rotation equivariance (so each is
the unique invariant up to scale), and an independent adaptive-quadrature evaluation of the triple-product
form with finite-difference gradients.  Deeper models: the kept irreps of each layer, derived by hand.
"""
import math

import numpy as np
import pytest
import torch
from scipy import integrate
from scipy.special import eval_legendre

from oracle import basis, cg


def _rot(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q *= np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def _unit(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_envelope_boundary_values():
    t = torch.tensor([0.0, 1.0], dtype=torch.float64, requires_grad=True)
    u = basis.envelope(t, 6)
    assert u[0].item() == 1.0 and abs(u[1].item()) < 1e-14
    (g,) = torch.autograd.grad(u.sum(), t, create_graph=True)
    (h,) = torch.autograd.grad(g.sum(), t)
    assert abs(g[1].item()) < 1e-12 and abs(h[1].item()) < 1e-11
    ts = torch.linspace(0, 1, 101, dtype=torch.float64)
    assert torch.all(torch.diff(basis.envelope(ts, 6)) <= 1e-15)


def test_bessel_orthonormal():
    rc = 4.0
    def f(r, n, m):
        d = torch.tensor([r], dtype=torch.float64)
        B = basis.bessel(d, rc, 8)[0]
        return float(B[n] * B[m]) * r * r
    for n in range(8):
        for m in range(n, 8):
            val, _ = integrate.quad(f, 1e-9, rc, args=(n, m), limit=200)
            assert abs(val - (1.0 if n == m else 0.0)) < 1e-8


def test_sh_addition_theorem_and_parity():
    rng = np.random.default_rng(1)
    a, b = _unit(rng, 50), _unit(rng, 50)
    Ya, Yb = basis.spherical_harmonics_np(a, 3), basis.spherical_harmonics_np(b, 3)
    cos = (a * b).sum(1)
    for l in range(4):
        sl = slice(l * l, (l + 1) ** 2)
        lhs = (Ya[:, sl] * Yb[:, sl]).sum(1)
        assert np.allclose(lhs, (2 * l + 1) * eval_legendre(l, cos), atol=1e-12)
        assert np.allclose(basis.spherical_harmonics_np(-a, 3)[:, sl], (-1) ** l * Ya[:, sl])
    # component normalisation and orthogonality: mean over the sphere of Y Y^T = I
    pts, w = cg._quadrature()
    Y = basis.spherical_harmonics_np(pts, 3)
    G = (w[:, None] * Y).T @ Y / (4 * math.pi)
    assert np.allclose(G, np.eye(16), atol=1e-12)


def _wigner_D(R, l):
    rng = np.random.default_rng(7)
    x = _unit(rng, 40)
    sl = slice(l * l, (l + 1) ** 2)
    A = basis.spherical_harmonics_np(x, 3)[:, sl]
    B = basis.spherical_harmonics_np(x @ R.T, 3)[:, sl]
    D, *_ = np.linalg.lstsq(A, B, rcond=None)
    assert np.allclose(A @ D, B, atol=1e-10)
    return D.T  # Y(R x) = D Y(x)


@pytest.mark.parametrize("path", [(1, 1, 0), (1, 1, 2), (1, 2, 1), (2, 2, 2), (0, 2, 2), (2, 1, 1),
                                  (1, 1, 1), (1, 2, 2), (2, 2, 1), (2, 1, 2), (2, 2, 3), (3, 3, 3),
                                  (1, 3, 3), (3, 2, 2), (3, 3, 2), (2, 3, 1), (3, 3, 0), (1, 2, 3)])
def test_coupling_equivariant(path):
    rng = np.random.default_rng(3)
    R = _rot(rng)
    D = [_wigner_D(R, l) for l in range(4)]
    for l in range(4):
        assert np.allclose(D[l] @ D[l].T, np.eye(2 * l + 1), atol=1e-10)
    l1, l2, l3 = path
    C = cg.coupling(l1, l2, l3)
    lhs = np.einsum("abc,ax,by->xyc", C, D[l1], D[l2])
    rhs = np.einsum("xyc,zc->xyz", C, D[l3])
    assert np.allclose(lhs, rhs, atol=1e-10)
    assert abs(np.linalg.norm(C) - 1.0) < 1e-12


def test_sh_match_sympy_real_harmonics_up_to_sign():
    """Each Y_lm is sqrt(4 pi) times one of sympy's orthonormal real harmonics
    Z_lm (same l, m; sympy's sign convention for Z differs for some m)."""
    import sympy
    from sympy import Znm
    th, ph = sympy.symbols("theta phi", real=True)
    t0, p0 = 0.7, 0.4
    x = np.array([[math.sin(t0) * math.cos(p0), math.sin(t0) * math.sin(p0), math.cos(t0)]])
    ours = basis.spherical_harmonics_np(x, 3)[0]
    for l in range(4):
        for m in range(-l, l + 1):
            zc = complex(sympy.N(Znm(l, m, th, ph).expand(func=True).subs({th: t0, ph: p0})))
            assert abs(zc.imag) < 1e-12
            z = zc.real
            val = ours[l * l + m + l] / (math.sqrt(4 * math.pi) * z)
            assert abs(abs(val) - 1.0) < 1e-10, (l, m, val)


@pytest.mark.parametrize("path", [(1, 1, 0), (1, 1, 2), (1, 2, 1), (2, 2, 2), (0, 1, 1), (2, 2, 0),
                                  (3, 3, 0), (1, 2, 3), (3, 3, 2), (2, 3, 3)])
def test_coupling_matches_sympy_real_gaunt(path):
    """sympy's exact real Gaunt coefficients use the same real-harmonic
    convention as ours (no Condon-Shortley phase), so they agree entry by
    entry after the unit-norm rescaling."""
    from sympy.physics.wigner import real_gaunt
    l1, l2, l3 = path
    ref = np.zeros((2 * l1 + 1, 2 * l2 + 1, 2 * l3 + 1))
    for m1 in range(-l1, l1 + 1):
        for m2 in range(-l2, l2 + 1):
            for m3 in range(-l3, l3 + 1):
                g = float(real_gaunt(l1, l2, l3, m1, m2, m3))
                ref[m1 + l1, m2 + l2, m3 + l3] = g
    ref /= np.linalg.norm(ref)
    assert np.allclose(cg.coupling(l1, l2, l3), ref, atol=1e-12)


def test_final_layer_diagonal():
    for l in range(3):
        C = cg.coupling(l, l, 0)[:, :, 0]
        assert np.allclose(C, np.eye(2 * l + 1) / math.sqrt(2 * l + 1), atol=1e-13)


def test_path_counts_and_nonzeros():
    P = cg.layer_paths(2, 2)
    assert [len(p) for p in P] == [11, 3]
    assert sorted({p[3] for p in P[0]}) == [0, 1, 2] and {p[3] for p in P[1]} == {0}
    assert all(p[1] == (-1) ** p[0] and p[4] == (-1) ** p[3] for L in P for p in L)
    assert cg.layer_paths(1, 1) == [[(0, 1, 0, 0, 1), (1, -1, 1, 0, 1)]]
    assert not cg.has_unnatural(2, 2) and cg.has_unnatural(2, 3)
    rng = np.random.default_rng(0)
    W1 = cg.fused_table(2, P[0], rng.standard_normal((3, 3, 3)), False)
    W2 = cg.fused_table(2, P[1], rng.standard_normal((3, 3, 3)), True)
    assert np.count_nonzero(W1) == 83 and np.count_nonzero(W2) == 9


def test_three_layer_irreps_by_hand():
    """l_max 2, three layers.  Layer 1 takes the natural irreps 0e 1o 2e and
    keeps every triangle (l1, l2, l_out): its cross-parity outputs 1e, 2o are
    what layer 2 turns back into natural irreps through the odd-sum paths
    (1,1,1), (1,2,2), (2,1,2), (2,2,1).  The final layer reads natural irreps."""
    P = cg.layer_paths(2, 3)
    tri = [(l1, l2, lo) for l1 in range(3) for l2 in range(3) for lo in range(3) if abs(l1 - l2) <= lo <= l1 + l2]
    assert len(tri) == 15 and sorted((p[0], p[2], p[3]) for p in P[0]) == sorted(tri)
    out1 = {(p[3], p[4]) for p in P[0]}
    assert out1 == {(0, 1), (1, -1), (2, 1), (1, 1), (2, -1)}
    odd = {(1, 1, 1), (1, 2, 2), (2, 1, 2), (2, 2, 1)}
    assert {(p[0], p[2], p[3]) for p in P[1] if p[1] != (-1) ** p[0]} == odd
    assert {(p[3], p[4]) for p in P[1]} == {(0, 1), (1, -1), (2, 1)} and len(P[1]) == 15
    assert [(p[0], p[1]) for p in P[2]] == [(0, 1), (1, -1), (2, 1)]
    assert cg.layer_widths(2, 3) == [(9, 18), (18, 9), (9, 1)]


def test_odd_coupling_closed_form_and_symmetry():
    C = cg.coupling(1, 1, 1)
    # components (y, z, x): C[a, b, c] = eps_{sigma(a) sigma(b) sigma(c)} / sqrt(6)
    eps = np.zeros((3, 3, 3))
    for (i, j, k), s in {(0, 1, 2): 1, (1, 2, 0): 1, (2, 0, 1): 1, (0, 2, 1): -1, (2, 1, 0): -1,
                         (1, 0, 2): -1}.items():
        eps[i, j, k] = s
    assert np.allclose(C, eps / math.sqrt(6), atol=1e-13)
    for (l, lo) in ((2, 1), (2, 3), (3, 1), (3, 3), (3, 5 - 2)):
        Co = cg.coupling(l, l, lo)
        assert np.linalg.norm(Co) > 0.99 and np.allclose(Co, -Co.transpose(1, 0, 2), atol=1e-13)
    # the Gaunt integral vanishes on odd sums, the triple-product form on even ones
    assert np.abs(cg.gaunt(1, 2, 2)).max() < 1e-14 and np.abs(cg.triple_form(1, 1, 2)).max() < 1e-13


@pytest.mark.parametrize("entry", [((1, 2, 2), (1, 4, 0)), ((2, 3, 2), (2, 5, 0)), ((3, 2, 2), (5, 2, 0)),
                                   ((3, 3, 1), (0, 6, 1))])
def test_triple_form_adaptive_quadrature(entry):
    """(1/4pi) int rhat . (grad Y_a x grad Y_b) Y_c dOmega by scipy's adaptive
    double quadrature in (theta, phi) with central-difference surface
    gradients: independent of the product rule and of autograd."""
    (l1, l2, l3), (m1, m2, m3) = entry
    a, b, c = l1 * l1 + m1, l2 * l2 + m2, l3 * l3 + m3

    def Y(v):
        v = np.asarray(v, dtype=float)
        return basis.spherical_harmonics_np((v / np.linalg.norm(v))[None, :], 3)[0]

    def f(th, ph):
        r = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
        h = 1e-5
        g = np.zeros((16, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            g[:, k] = (Y(r + e) - Y(r - e)) / (2 * h)
        return float(np.dot(r, np.cross(g[a], g[b])) * Y(r)[c]) * math.sin(th)

    val, _ = integrate.dblquad(lambda ph, th: f(th, ph), 0, math.pi, 0, 2 * math.pi, epsabs=1e-9)
    ref = cg.triple_form(l1, l2, l3)[m1, m2, m3]
    assert abs(ref) > 1e-3 and abs(val / (4 * math.pi) - ref) < 1e-7


def test_path_fusion_equals_per_path_sum():
    """Fusing the weighted paths into one table (section "Optimized tensor
    product") equals applying the paths one by one."""
    rng = np.random.default_rng(5)
    P = cg.layer_paths(2, 2)[0]
    al = rng.standard_normal((3, 3, 3))
    W = cg.fused_table(2, P, al, False)
    x, y = rng.standard_normal(9), rng.standard_normal(9)
    fused = np.einsum("abc,a,b->c", W, x, y)
    per_out = {}
    for p in P:
        per_out[p[3]] = per_out.get(p[3], 0) + 1
    out = np.zeros(9)
    for (l1, _, l2, lo, _) in P:
        C = cg.coupling(l1, l2, lo)
        out[lo * lo:(lo + 1) ** 2] += al[l1, l2, lo] / math.sqrt(per_out[lo]) * np.einsum(
            "abc,a,b->c", C, x[l1 * l1:(l1 + 1) ** 2], y[l2 * l2:(l2 + 1) ** 2])
    assert np.allclose(fused, out, atol=1e-13)


# Number of kept paths into each output irrep (l_out, p_out), counted by hand
# from the selection rules (triangle, p_out = p1 p2, l_out <= l_max, pruning
# towards the final scalar), independently of the oracle's enumeration:
#   l_max 1, one layer: 0e <- (0,0), (1,1).
#   l_max 2, two layers: layer 1 (natural inputs, natural outputs) 0e <- (0,0),
#     (1,1), (2,2); 1o <- (0,1), (1,0), (1,2), (2,1); 2e <- (0,2), (2,0), (1,1),
#     (2,2); final 0e <- (0,0), (1,1), (2,2).
#   l_max 2, three layers: layer 1 also feeds the unnatural 1e <- (1,1), (2,2)
#     and 2o <- (1,2), (2,1); layer 2 adds to its natural outputs 1o <- (1e,1),
#     (2o,2) and 2e <- (1e,2), (2o,1).
HAND_PATHS_PER_OUTPUT = {
    (1, 1): [{(0, 1): 2}],
    (2, 2): [{(0, 1): 3, (1, -1): 4, (2, 1): 4}, {(0, 1): 3}],
    (2, 3): [{(0, 1): 3, (1, -1): 4, (2, 1): 4, (1, 1): 2, (2, -1): 2},
             {(0, 1): 3, (1, -1): 6, (2, 1): 6}, {(0, 1): 3}],
}


@pytest.mark.parametrize("model", sorted(HAND_PATHS_PER_OUTPUT), ids=lambda m: f"lmax{m[0]}_layers{m[1]}")
def test_path_weight_scale_by_hand_counts(model):
    """Reading of the path weights: alpha_p = raw_p / sqrt(P_out), P_out the
    number of kept paths into p's output irrep.  With a single unit raw weight
    the fused table is that path's unit-norm coupling divided by sqrt(P_out),
    so its Frobenius norm must be 1/sqrt of the hand-counted P_out (a wrong
    count in the oracle's fusion changes it)."""
    l_max, n_layers = model
    layers = cg.layer_paths(l_max, n_layers)
    widths = cg.layer_widths(l_max, n_layers)
    deep = cg.has_unnatural(l_max, n_layers)
    for L, paths in enumerate(layers):
        hand = HAND_PATHS_PER_OUTPUT[model][L]
        assert sum(hand.values()) == len(paths)
        final = L == len(layers) - 1
        for (l1, p1, l2, lo, po) in paths:
            raw = np.zeros((2, l_max + 1, l_max + 1, l_max + 1) if deep else (l_max + 1,) * 3)
            if deep:
                raw[0 if p1 == cg.natural(l1) else 1, l1, l2, lo] = 1.0
            else:
                raw[l1, l2, lo] = 1.0
            W = cg.fused_table(l_max, paths, raw, final, n_in=widths[L][0], n_out=widths[L][1])
            assert abs(np.linalg.norm(W) - 1.0 / math.sqrt(hand[(lo, po)])) < 1e-12, (L, l1, p1, l2, lo, po)
