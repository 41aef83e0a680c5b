"""The Allegro network, energies, forces and virial in float64 (torch-CPU).

Follows the paper's description (section "Allegro: Scalable Equivariant Deep
Learning", Eq. tp and the two-track architecture; section "Optimized tensor
product"; section "Training details" for the MLP kinds) with these readings
where the paper defers to the original Allegro paper:

edge (i, j, s):  r = (x_j - x_i) + s L,  d = |r|,  rhat = r / d,  u = u(d / r_c)
  R_n = B_n(d) u                                    (Bessel x envelope)
  Y   = Y(rhat)                                     (strided components c = l^2 + m + l)
two-body latent:  x0 = u * MLP_2b([onehot(Z_i), onehot(Z_j), R])
initial tensor features:  V0[c, u] = (x0 @ W_embed)[l(c), u] * Y[c]
layer L = 1..N_l:
  w      = x^{L-1} @ W_env^L                        (the linear "embedding MLP")
  Gamma_i[b, u] = (1/sqrt(avg_nbrs)) sum_{k in N(i)} w^{ik}[l(b), u] Y^{ik}[b]
  T[c, u]       = sum_{a, b} W^L[a, b, c] V^{L-1}[a, u] Gamma_i[b, u]   (Eq. tp, factored)
  V^L[c, v]     = sum_u M^L_{irrep(c)}[v, u] T[c, u] / sqrt(n)   (linear channel mixing,
                  one matrix per output irrep (l, p))
  x^L    = (x^{L-1} + u * MLP_L([x^{L-1}, V^L[0, :]])) / sqrt(2)
edge energy:  E_ij = (x^{N_l} @ W_e1) @ W_e2        (one hidden layer, no nonlinearity)
atom energy:  A_i = sigma_{Z_i} sum_j E_ij + mu_{Z_i};  E = sum_i A_i
  (section "Allegro: Scalable Equivariant Deep Learning", first equation)

All MLPs are bias-free with SiLU after every layer but the last.  Forces are
F = -dE/dx; with g_e = dE/dr_e, F_i = sum_{e from i} g_e - sum_{e to i} g_e and
the virial is W = -sum_e r_e (x) g_e.

Each centre's energy depends only on its own edges, so the evaluation is
chunked over contiguous centre ranges to bound memory; nothing else is
reordered.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, Optional

import numpy as np
import torch

from . import basis, cg
from .neighbors import neighbor_list, row_ptr


@dataclass
class Result:
    energy: float
    atom_energy: np.ndarray   # [n_local]
    forces: np.ndarray        # [n_total, 3]
    virial: np.ndarray        # [3, 3]
    atom_virial: np.ndarray   # [n_total, 3, 3]
    edge_grad: np.ndarray     # [E, 3]  dE/dr_e
    edge_energy: np.ndarray   # [E]
    nbr: tuple                # (i, j, shift)


class Params:
    """Weights as float64 torch tensors plus the fused coupling tables."""

    def __init__(self, mc, weights: Dict[str, np.ndarray]):
        t = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64))
        self.mc = mc
        nb = len(mc.twobody_dims)
        nl = len(mc.latent_dims)
        self.twobody = [t(weights[f"twobody.W{k}"]) for k in range(nb)]
        self.embed0 = t(weights["embed0"])
        self.paths = cg.layer_paths(mc.l_max, mc.n_layers)
        self.widths = cg.layer_widths(mc.l_max, mc.n_layers)
        self.env, self.W, self.mix, self.mlp = [], [], [], []
        for L in range(1, mc.n_layers + 1):
            self.env.append(t(weights[f"layer{L}.env"]))
            final = L == mc.n_layers
            n_in, n_out = self.widths[L - 1]
            self.W.append(t(cg.fused_table(mc.l_max, self.paths[L - 1],
                                           np.asarray(weights[f"layer{L}.alpha"]), final, n_in, n_out)))
            self.mix.append(t(weights[f"layer{L}.mix"]))
            self.mlp.append([t(weights[f"layer{L}.mlp.W{k}"]) for k in range(nl)])
        ne = len(mc.edge_dims) + 1
        self.edge = [t(weights[f"edge.W{k}"]) for k in range(ne)]


def _mlp(x: torch.Tensor, Ws) -> torch.Tensor:
    for k, W in enumerate(Ws):
        x = x @ W
        if k < len(Ws) - 1:
            x = torch.nn.functional.silu(x)
    return x


def edge_energies(p: Params, r: torch.Tensor, ci: torch.Tensor, zi: torch.Tensor,
                  zj: torch.Tensor, n_centres: int) -> torch.Tensor:
    """Per-edge energies E_ij for edge vectors r [E, 3] whose centres are
    `ci` (0..n_centres-1, grouping edges by centre)."""
    mc = p.mc
    n, lm, S = mc.n_tensor, mc.l_max, mc.n_species
    lc = torch.as_tensor(basis.irrep_of_component(lm))
    dim = (lm + 1) ** 2
    # mixing-matrix slot of each strided component: natural (l, (-1)^l) -> l,
    # the other parity (components dim..2 dim) -> l_max + 1 + l
    slot = torch.cat([lc, lc + lm + 1])
    E = r.shape[0]

    d = torch.sqrt((r * r).sum(1))
    rhat = r / d[:, None]
    # cutoff of each edge: the global r_c, or its ordered species pair's own
    # (section "Species-dependent cutoffs"); envelope and basis scale with it
    if mc.pair_cutoffs is None:
        rc = mc.r_cut
    else:
        rc = torch.as_tensor(np.asarray(mc.pair_cutoffs, dtype=np.float64))[zi, zj]
    u = basis.envelope(d / rc, mc.envelope_p)
    R = basis.bessel(d, rc, mc.n_bessel) * u[:, None]
    Y = basis.spherical_harmonics(rhat, lm)

    onehot = torch.zeros(E, 2 * S, dtype=torch.float64)
    onehot[torch.arange(E), zi] = 1.0
    onehot[torch.arange(E), S + zj] = 1.0
    x = u[:, None] * _mlp(torch.cat([onehot, R], 1), p.twobody)

    a0 = (x @ p.embed0).view(E, lm + 1, n)
    V = a0[:, lc, :] * Y[:, :, None]                       # [E, dim, n]
    c_norm = 1.0 / math.sqrt(mc.avg_num_neighbors)
    for L in range(mc.n_layers):
        w = (x @ p.env[L]).view(E, lm + 1, n)
        wY = w[:, lc, :] * Y[:, :, None]                   # [E, dim, n]
        gam = torch.zeros(n_centres, dim, n, dtype=torch.float64).index_add(0, ci, wY) * c_norm
        T = torch.einsum("abc,eau,ebu->ecu", p.W[L], V, gam[ci])
        n_out = T.shape[1]
        if mc.channel_mix:
            M = p.mix[L][slot[:n_out]]                        # [n_out, v, u]
            V = torch.einsum("cvu,ecu->ecv", M, T) / math.sqrt(n)
        else:
            V = T
        s = V[:, 0, :]
        x = (x + u[:, None] * _mlp(torch.cat([x, s], 1), p.mlp[L])) / math.sqrt(2.0)
    return (x @ p.edge[0] @ p.edge[1] if len(p.edge) == 2 else _mlp_linear(x, p.edge)).view(E)


def pair_energies(mc, r: torch.Tensor, zi: torch.Tensor, zj: torch.Tensor) -> torch.Tensor:
    """Per-ordered-edge share of the ZBL repulsion, 1/2 E_ZBL(d) u(d / r_c,ij):
    each pair counts in full when both of its ordered edges are in the list,
    and the envelope of the edge takes it smoothly to zero at that edge's
    cutoff.  Zero when the model has no atomic numbers (no ZBL term)."""
    if getattr(mc, "atomic_numbers", None) is None:
        return torch.zeros(r.shape[0], dtype=torch.float64)
    d = torch.sqrt((r * r).sum(1))
    if mc.pair_cutoffs is None:
        rc = mc.r_cut
    else:
        rc = torch.as_tensor(np.asarray(mc.pair_cutoffs, dtype=np.float64))[zi, zj]
    zn = torch.as_tensor(np.asarray(mc.atomic_numbers, dtype=np.float64))
    u = basis.envelope(d / rc, mc.envelope_p)
    return 0.5 * basis.zbl_energy(d, zn[zi], zn[zj]) * u


def _mlp_linear(x, Ws):
    for W in Ws:
        x = x @ W
    return x


def evaluate(mc, weights, sysm, scale=None, shift=None, nbr=None, params=None,
             chunk_edges: int = 200_000, need_atom_virial: bool = True) -> Result:
    """Energy, per-atom energies, forces, virial of `sysm` (workloads.System)."""
    p = params or Params(mc, weights)
    pos = np.asarray(sysm.pos, dtype=np.float64)
    nl, nt = sysm.n_local, pos.shape[0]
    L = np.where(np.asarray(sysm.pbc) != 0, np.asarray(sysm.cell, dtype=np.float64), 0.0)
    if nbr is None:
        nbr = neighbor_list(pos, sysm.cell, sysm.pbc, mc.r_cut, n_local=nl, species=sysm.species,
                            pair_cutoffs=mc.pair_cutoffs)
    i, j, s = nbr
    rp = row_ptr(i, nl)
    sig = np.ones(mc.n_species) if scale is None else np.asarray(scale, dtype=np.float64)
    mu = np.zeros(mc.n_species) if shift is None else np.asarray(shift, dtype=np.float64)
    Z = np.asarray(sysm.species, dtype=np.int64)

    rvec = (pos[j] - pos[i]) + s.astype(np.float64) * L[None, :]
    E = rvec.shape[0]
    edge_e = np.zeros(E)
    edge_z = np.zeros(E)
    edge_g = np.zeros((E, 3))
    atom_e_raw = np.zeros(nl)
    # chunks of whole centre segments
    a = 0
    while a < nl:
        b = a
        while b < nl and (rp[b + 1] - rp[a] <= chunk_edges or b == a):
            b += 1
        e0, e1 = int(rp[a]), int(rp[b])
        if e1 > e0:
            r = torch.tensor(rvec[e0:e1], requires_grad=True)
            ci = torch.as_tensor(i[e0:e1] - a)
            zi_t, zj_t = torch.as_tensor(Z[i[e0:e1]]), torch.as_tensor(Z[j[e0:e1]])
            eij = edge_energies(p, r, ci, zi_t, zj_t, b - a)
            ez = pair_energies(mc, r, zi_t, zj_t)
            # dE/dE_ij = sigma_{Z_i}; the pair term is added unscaled
            w = torch.as_tensor(sig[Z[i[e0:e1]]])
            tot = (eij * w).sum() + ez.sum()
            (g,) = torch.autograd.grad(tot, r)
            edge_e[e0:e1] = eij.detach().numpy()
            edge_z[e0:e1] = ez.detach().numpy()
            edge_g[e0:e1] = g.numpy()
        a = b
    np.add.at(atom_e_raw, i, edge_e)
    atom_z = np.zeros(nl)
    np.add.at(atom_z, i, edge_z)
    atom_e = sig[Z[:nl]] * atom_e_raw + mu[Z[:nl]] + atom_z
    energy = float(atom_e.sum())
    F = np.zeros((nt, 3))
    np.add.at(F, i, edge_g)
    np.add.at(F, j, -edge_g)
    vir_e = -rvec[:, :, None] * edge_g[:, None, :]          # [E, 3, 3]
    virial = vir_e.sum(0)
    av = np.zeros((nt, 3, 3))
    if need_atom_virial:
        np.add.at(av, i, 0.5 * vir_e)
        np.add.at(av, j, 0.5 * vir_e)
    return Result(energy=energy, atom_energy=atom_e, forces=F, virial=virial, atom_virial=av,
                  edge_grad=edge_g, edge_energy=edge_e, nbr=nbr)


def energy_of_positions(mc, weights, sysm, pos, scale=None, shift=None, params=None) -> float:
    """Total energy for displaced positions (neighbour list rebuilt); used by
    finite-difference tests."""
    import copy
    s2 = copy.copy(sysm)
    s2.pos = np.asarray(pos, dtype=np.float64)
    return evaluate(mc, weights, s2, scale, shift, params=params, need_atom_virial=False).energy


def evaluate_centres(mc, weights, sysm, centres, nbr, scale=None, params=None):
    """Atom energies and edge gradients of a subset of centres only.

    Each centre's energy depends only on its own edges (strict locality), so a
    subset is evaluated exactly like the whole system restricted to those
    segments.  Returns (atom_energy[len(centres)], {edge index: dE/dr_e}).
    """
    if getattr(mc, "atomic_numbers", None) is not None:
        raise NotImplementedError("evaluate_centres returns network energies only (no ZBL term)")
    p = params or Params(mc, weights)
    pos = np.asarray(sysm.pos, dtype=np.float64)
    L = np.where(np.asarray(sysm.pbc) != 0, np.asarray(sysm.cell, dtype=np.float64), 0.0)
    i, j, s = nbr
    rp = row_ptr(i, sysm.n_local)
    sig = np.ones(mc.n_species) if scale is None else np.asarray(scale, dtype=np.float64)
    Z = np.asarray(sysm.species, dtype=np.int64)
    centres = np.asarray(centres, dtype=np.int64)
    idx = np.concatenate([np.arange(rp[c], rp[c + 1]) for c in centres]).astype(np.int64)
    local = np.repeat(np.arange(len(centres)), rp[centres + 1] - rp[centres])
    rvec = (pos[j[idx]] - pos[i[idx]]) + s[idx].astype(np.float64) * L[None, :]
    r = torch.tensor(rvec, requires_grad=True)
    eij = edge_energies(p, r, torch.as_tensor(local), torch.as_tensor(Z[i[idx]]),
                        torch.as_tensor(Z[j[idx]]), len(centres))
    w = torch.as_tensor(sig[Z[i[idx]]])
    (g,) = torch.autograd.grad((eij * w).sum(), r)
    e_raw = np.zeros(len(centres))
    np.add.at(e_raw, local, eij.detach().numpy())
    return e_raw, dict(zip(idx.tolist(), g.numpy()))
