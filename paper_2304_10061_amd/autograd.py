"""Energy as a torch.autograd.Function.

forward(pos) runs the neighbour build and the library's energy/force
evaluation (which includes the hand-written adjoint) and returns the total
energy; backward(gE) returns -gE * F, i.e. gE * dE/dpos.
"""
from __future__ import annotations

import torch


class AllegroEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, model, species, cell, pbc, n_local=None):
        out = model.evaluate(pos.detach().contiguous(), species, cell, pbc, n_local)
        ctx.save_for_backward(out["forces"])
        return out["energy"][0].clone()

    @staticmethod
    def backward(ctx, gE):
        (F,) = ctx.saved_tensors
        return -gE * F, None, None, None, None, None


def energy(pos, model, species, cell, pbc, n_local=None):
    return AllegroEnergy.apply(pos, model, species, cell, pbc, n_local)
