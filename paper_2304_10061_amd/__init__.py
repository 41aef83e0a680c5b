"""MI355X (gfx950) Allegro energy-and-force library.

The compute path is the HIP library liballegro_mi355x.so (C interface in
include/allegro_mi355x.h); `binding` marshals arguments to it and `autograd`
exposes the energy as a torch.autograd.Function whose backward is the
library's hand-written adjoint.
"""
from .binding import (AllegroConfig, AllegroError, Model, PREC_BF16, PREC_BF16_MIXED, PREC_BF16_SINGLE, PREC_FP32,
                      config_from, describe, load_library, make_config, plan_chunks)

__all__ = ["AllegroConfig", "AllegroError", "Model", "PREC_BF16", "PREC_BF16_MIXED", "PREC_BF16_SINGLE", "PREC_FP32",
           "config_from", "describe", "load_library", "make_config", "plan_chunks"]
