"""Pins of the oracle's edge basis and coupling tables (CPU only).

Envelope: closed-form boundary values.  Bessel: orthonormality on [0, r_c]
with weight r^2 (scipy quadrature).  Spherical harmonics: the addition theorem
with scipy's Legendre polynomials, parity, orthonormality on the sphere.
Couplings: sympy's exact real Gaunt coefficients, rotation equivariance, the final-layer diagonal form, and the
path/non-zero counts of the fused tables.
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
    Ya, Yb = basis.spherical_harmonics_np(a, 2), basis.spherical_harmonics_np(b, 2)
    cos = (a * b).sum(1)
    for l in range(3):
        sl = slice(l * l, (l + 1) ** 2)
        lhs = (Ya[:, sl] * Yb[:, sl]).sum(1)
        assert np.allclose(lhs, (2 * l + 1) * eval_legendre(l, cos), atol=1e-12)
        assert np.allclose(basis.spherical_harmonics_np(-a, 2)[:, sl], (-1) ** l * Ya[:, sl])
    # component normalisation and orthogonality: mean over the sphere of Y Y^T = I
    pts, w = cg._quadrature()
    Y = basis.spherical_harmonics_np(pts, 2)
    G = (w[:, None] * Y).T @ Y / (4 * math.pi)
    assert np.allclose(G, np.eye(9), atol=1e-12)


def _wigner_D(R, l):
    rng = np.random.default_rng(7)
    x = _unit(rng, 40)
    sl = slice(l * l, (l + 1) ** 2)
    A = basis.spherical_harmonics_np(x, 2)[:, sl]
    B = basis.spherical_harmonics_np(x @ R.T, 2)[:, sl]
    D, *_ = np.linalg.lstsq(A, B, rcond=None)
    assert np.allclose(A @ D, B, atol=1e-10)
    return D.T  # Y(R x) = D Y(x)


@pytest.mark.parametrize("path", [(1, 1, 0), (1, 1, 2), (1, 2, 1), (2, 2, 2), (0, 2, 2), (2, 1, 1)])
def test_coupling_equivariant(path):
    rng = np.random.default_rng(3)
    R = _rot(rng)
    D = [_wigner_D(R, l) for l in range(3)]
    for l in range(3):
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
    ours = basis.spherical_harmonics_np(x, 2)[0]
    for l in range(3):
        for m in range(-l, l + 1):
            zc = complex(sympy.N(Znm(l, m, th, ph).expand(func=True).subs({th: t0, ph: p0})))
            assert abs(zc.imag) < 1e-12
            z = zc.real
            val = ours[l * l + m + l] / (math.sqrt(4 * math.pi) * z)
            assert abs(abs(val) - 1.0) < 1e-10, (l, m, val)


@pytest.mark.parametrize("path", [(1, 1, 0), (1, 1, 2), (1, 2, 1), (2, 2, 2), (0, 1, 1), (2, 2, 0)])
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
    assert sorted({p[2] for p in P[0]}) == [0, 1, 2] and {p[2] for p in P[1]} == {0}
    assert cg.layer_paths(1, 1) == [[(0, 0, 0), (1, 1, 0)]]
    rng = np.random.default_rng(0)
    W1 = cg.fused_table(2, P[0], rng.standard_normal((3, 3, 3)), False)
    W2 = cg.fused_table(2, P[1], rng.standard_normal((3, 3, 3)), True)
    assert np.count_nonzero(W1) == 83 and np.count_nonzero(W2) == 9


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
        per_out[p[2]] = per_out.get(p[2], 0) + 1
    out = np.zeros(9)
    for (l1, l2, lo) in P:
        C = cg.coupling(l1, l2, lo)
        out[lo * lo:(lo + 1) ** 2] += al[l1, l2, lo] / math.sqrt(per_out[lo]) * np.einsum(
            "abc,a,b->c", C, x[l1 * l1:(l1 + 1) ** 2], y[l2 * l2:(l2 + 1) ** 2])
    assert np.allclose(fused, out, atol=1e-13)
