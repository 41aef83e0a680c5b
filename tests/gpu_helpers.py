"""Shared helpers of the GPU parity tests: run the HIP library through its
C interface (via the ctypes binding) on cuda:0."""
import numpy as np
import torch

import paper_2304_10061_amd as P
import workloads as W


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
