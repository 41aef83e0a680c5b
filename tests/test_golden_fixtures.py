"""CPU checks of the stored oracle fixtures: each still matches the seeded
generators it was written from, and its contents are self-consistent."""
import importlib.util
import os

import numpy as np

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _maker():
    spec = importlib.util.spec_from_file_location(
        "make_protein_box_reference", os.path.join(HERE, "golden", "make_protein_box_reference.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_protein_box_fixture_matches_generators():
    ref = np.load(os.path.join(HERE, "golden", "protein_box_reference.npz"), allow_pickle=False)
    mc, s, w = W.workload(3)
    assert str(ref["digest"]) == _maker().input_digest(mc, s, w)
    assert ref["atom_energy"].shape == (s.n_local,)
    assert ref["forces"].shape == (s.n_total, 3)
    # sigma = 1, mu = 0: the total is the sum of the atom energies
    assert abs(float(ref["atom_energy"].astype(np.float64).sum()) - float(ref["energy"])) < 1e-3
    # periodic box: Newton's third law holds edge by edge in the oracle
    assert np.abs(ref["forces"].astype(np.float64).sum(0)).max() < 1e-2
    # the virial of a pair-decomposed force field is symmetric only for
    # central forces; here it is just finite and of the box's scale
    assert np.all(np.isfinite(ref["virial"]))
    assert int(ref["n_edges"]) == 2052690
