"""Shared helpers of the GPU parity tests: run the HIP library through its
C interface (via the ctypes binding) on cuda:0."""
import numpy as np
import torch

import paper_2304_10061_amd as P
import workloads as W
from oracle import model as OM


def device():
    return torch.device("cuda", 0)


def to_dev(sysm):
    dev = device()
    pos = torch.as_tensor(np.ascontiguousarray(sysm.pos), dtype=torch.float64, device=dev)
    sp = torch.as_tensor(np.ascontiguousarray(sysm.species), dtype=torch.int32, device=dev)
    return pos, sp


def gpu_model(mc, w, precision, scale=None, shift=None, edge_chunk=0, mlp_tile=0):
    cfg = P.config_from(mc, precision=precision, edge_chunk=edge_chunk)
    m = P.Model(cfg, W.pack_weights(mc, w), scale, shift)
    if mlp_tile:
        m.set_tiles([mlp_tile] * 6 + [0, 0])
    return m


def gpu_eval(model, sysm, want_atom_virial=True):
    pos, sp = to_dev(sysm)
    out = model.evaluate(pos, sp, sysm.cell, sysm.pbc, sysm.n_local, want_atom_virial=want_atom_virial)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def gpu_edges(model, sysm):
    pos, sp = to_dev(sysm)
    model.neighbors(pos, sp, sysm.cell, sysm.pbc, sysm.n_local)
    ci, nj, sh = model.copy_edges()
    torch.cuda.synchronize()
    return ci.cpu().numpy().astype(np.int64), nj.cpu().numpy().astype(np.int64), sh.cpu().numpy().astype(np.int64)


def sampled_reference(mc, s, w, nbr, rng, n_centres=24, n_force_atoms=3):
    """Oracle energies of `n_centres` random centres and the forces on the
    first `n_force_atoms` of them (every edge touching those atoms is
    evaluated: their own segments and the segments of the centres that have
    them as neighbours)."""
    i, j, _ = nbr
    cents = np.sort(rng.choice(s.n_local, size=n_centres, replace=False))
    p = OM.Params(mc, w)
    e_raw, _ = OM.evaluate_centres(mc, w, s, cents, nbr, params=p)
    atoms = cents[:n_force_atoms]
    need = np.unique(np.concatenate([atoms, i[np.isin(j, atoms)]]))
    _, g = OM.evaluate_centres(mc, w, s, need, nbr, params=p)
    F = np.zeros((len(atoms), 3))
    for k, a in enumerate(atoms):
        for e in np.nonzero(i == a)[0]:
            F[k] += g[int(e)]
        for e in np.nonzero(j == a)[0]:
            F[k] -= g[int(e)]
    return cents, e_raw, atoms, F
