"""Edge basis: polynomial cutoff envelope, Bessel radial basis, real spherical
harmonics (float64, torch so that autograd can differentiate them).

The paper embeds interatomic distances in a basis of 8 Bessel functions times a
polynomial cutoff envelope (section "Training details"), and the geometry of
each neighbour through spherical harmonics of the unit edge vector (section
"Allegro: Scalable Equivariant Deep Learning", the Y^{ik} of Eq. tp), with full
O(3) symmetry.  The exact forms are deferred there to the original Allegro
paper; the readings used are:

* envelope, p = 6:  u(t) = 1 - (p+1)(p+2)/2 t^p + p(p+2) t^(p+1) - p(p+1)/2 t^(p+2),
  t = d / r_c  (so u(0) = 1 and u, u', u'' vanish at t = 1);
* Bessel:  B_n(d) = sqrt(2 / r_c) sin(n pi d / r_c) / d, n = 1..n_bessel, with
  fixed frequencies;
* real spherical harmonics with "component" normalisation
  (sum_m Y_lm(r)^2 = 2l + 1 on the unit sphere), m ordered -l..l:
    Y_0 = 1
    Y_1 = sqrt(3) (y, z, x)
    Y_2 = (sqrt15 xy, sqrt15 yz, sqrt5/2 (3z^2 - 1), sqrt15 xz, sqrt15/2 (x^2 - y^2))
    Y_3 = (sqrt70/4 y(3x^2 - y^2), sqrt105 xyz, sqrt42/4 y(5z^2 - 1),
           sqrt7/2 z(5z^2 - 3), sqrt42/4 x(5z^2 - 1), sqrt105/2 z(x^2 - y^2),
           sqrt70/4 x(x^2 - 3y^2)).
  The parity of Y_l is (-1)^l.
"""
from __future__ import annotations

import math

import numpy as np
import torch


def envelope(t: torch.Tensor, p: int = 6) -> torch.Tensor:
    """Polynomial cutoff u(t) for t = d / r_c in [0, 1)."""
    return (1.0 - (p + 1) * (p + 2) / 2.0 * t ** p + p * (p + 2) * t ** (p + 1)
            - p * (p + 1) / 2.0 * t ** (p + 2))


def bessel(d: torch.Tensor, r_cut, n_bessel: int) -> torch.Tensor:
    """[E, n_bessel] Bessel basis B_n(d); `r_cut` is one radius or one per
    edge (per-ordered-species-pair cutoffs: each pair's basis is scaled to
    its own cutoff)."""
    n = torch.arange(1, n_bessel + 1, dtype=d.dtype)
    if isinstance(r_cut, torch.Tensor):
        rc = r_cut[:, None]
        return torch.sqrt(2.0 / rc) * torch.sin(n[None, :] * math.pi * d[:, None] / rc) / d[:, None]
    return math.sqrt(2.0 / r_cut) * torch.sin(n[None, :] * math.pi * d[:, None] / r_cut) / d[:, None]


def spherical_harmonics(rhat: torch.Tensor, l_max: int) -> torch.Tensor:
    """[E, (l_max+1)^2] real spherical harmonics of unit vectors."""
    if l_max > 3:
        raise NotImplementedError("l_max <= 3")
    x, y, z = rhat[:, 0], rhat[:, 1], rhat[:, 2]
    cols = [torch.ones_like(x)]
    if l_max >= 1:
        s3 = math.sqrt(3.0)
        cols += [s3 * y, s3 * z, s3 * x]
    if l_max >= 2:
        s15, s5 = math.sqrt(15.0), math.sqrt(5.0)
        cols += [s15 * x * y, s15 * y * z, s5 / 2.0 * (3.0 * z * z - 1.0), s15 * x * z,
                 s15 / 2.0 * (x * x - y * y)]
    if l_max >= 3:
        s70, s105, s42, s7 = math.sqrt(70.0), math.sqrt(105.0), math.sqrt(42.0), math.sqrt(7.0)
        zz = 5.0 * z * z
        cols += [s70 / 4.0 * y * (3.0 * x * x - y * y), s105 * x * y * z, s42 / 4.0 * y * (zz - 1.0),
                 s7 / 2.0 * z * (zz - 3.0), s42 / 4.0 * x * (zz - 1.0), s105 / 2.0 * z * (x * x - y * y),
                 s70 / 4.0 * x * (x * x - 3.0 * y * y)]
    return torch.stack(cols, dim=1)


def spherical_harmonics_np(rhat: np.ndarray, l_max: int) -> np.ndarray:
    return spherical_harmonics(torch.as_tensor(rhat, dtype=torch.float64), l_max).numpy()


def irrep_of_component(l_max: int):
    """l of each component index c = l^2 + (m + l)."""
    return [l for l in range(l_max + 1) for _ in range(2 * l + 1)]


# Ziegler-Biersack-Littmark universal screened Coulomb repulsion (the "ZBL
# term" the paper adds for stability, section "Training details"; the form and
# constants are those of the ZBL universal potential): k_e = e^2 / (4 pi eps0)
# in eV A, screening length a = 0.8854 a_0 / (Z_i^0.23 + Z_j^0.23), and the
# universal screening function phi as four exponentials with phi(0) = 1.
ZBL_KE = 14.399645
ZBL_A0 = 0.46850
ZBL_C = (0.18175, 0.50986, 0.28022, 0.02817)
ZBL_D = (3.19980, 0.94229, 0.40290, 0.20162)


def zbl_energy(d: torch.Tensor, zn_i: torch.Tensor, zn_j: torch.Tensor) -> torch.Tensor:
    """ZBL pair energy (eV) at distances d for atomic numbers zn_i, zn_j."""
    a = ZBL_A0 / (zn_i ** 0.23 + zn_j ** 0.23)
    x = d / a
    phi = sum(c * torch.exp(-k * x) for c, k in zip(ZBL_C, ZBL_D))
    return ZBL_KE * zn_i * zn_j / d * phi
