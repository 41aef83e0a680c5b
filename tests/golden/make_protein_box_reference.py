"""Writes protein_box_reference.npz: the FP64 oracle's energy, virial, per-atom
energies and forces of the whole 23,558-atom protein-like box (the seeded
workload of `workloads.workload(3)`, sigma = 1, mu = 0).

Only `oracle/` computes anything here; `workloads/` draws the inputs.  The
file also stores a SHA-256 digest of those inputs so that a test can refuse a
fixture that no longer matches the generators.

    python tests/golden/make_protein_box_reference.py

takes a few minutes on a handful of cores (about 2 million edges evaluated in
chunks of whole centre segments).
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import model as OM  # noqa: E402
from oracle.neighbors import neighbor_list  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "protein_box_reference.npz")


def input_digest(mc, s, w) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(s.pos, dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(s.species, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(s.cell, dtype=np.float64).tobytes())
    h.update(W.pack_weights(mc, w).tobytes())
    return h.hexdigest()


def main():
    import torch
    torch.set_num_threads(len(os.sched_getaffinity(0)))
    mc, s, w = W.workload(3)
    t0 = time.time()
    nbr = neighbor_list(s.pos, s.cell, s.pbc, mc.r_cut, method="kdtree")
    ref = OM.evaluate(mc, w, s, nbr=nbr, chunk_edges=100_000, need_atom_virial=False)
    dt = time.time() - t0
    np.savez_compressed(
        OUT,
        energy=np.float64(ref.energy),
        virial=np.asarray(ref.virial, dtype=np.float64),
        atom_energy=np.asarray(ref.atom_energy, dtype=np.float32),
        forces=np.asarray(ref.forces, dtype=np.float32),
        n_edges=np.int64(len(nbr[0])),
        digest=np.array(input_digest(mc, s, w)),
    )
    print(f"wrote {OUT}: E = {ref.energy:.10f} eV, {len(nbr[0])} edges, {dt:.1f} s "
          f"on {torch.get_num_threads()} threads")


if __name__ == "__main__":
    main()
