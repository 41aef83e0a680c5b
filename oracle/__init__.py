"""FP64 CPU oracle for the Allegro energy-and-force path.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
`cpu_baseline` leg of `bench.py` may import anything from this package.  The
product path (the HIP library and its Python binding) never imports, calls or
links it, and the oracle shares no code with that path: only the seeded input
generators in `workloads/` serve both.

Everything here is plain and slow on purpose: numpy / torch-CPU in float64,
each function citing the passage of the paper (arXiv 2304.10061, "Allegro at
scale") it follows.  Where the paper defers a formula to the original Allegro
paper, the reading used is stated in the docstring.

Modules:
  neighbors  - brute-force ordered neighbour list (the definition)
  basis      - polynomial envelope, Bessel radial basis, real spherical harmonics
  cg         - real Gaunt (Clebsch-Gordan) tables by quadrature, path enumeration
  model      - the network forward, per-atom energies, forces and virial
  md         - FP64 velocity Verlet

Parity status: no function here can be pinned to numbers printed in the paper
(the paper prints no model outputs, weights or worked example), so the whole
model is pinned by properties instead (finite differences, E(3) and permutation
invariance, locality, a loop-form re-evaluation on tiny inputs, a pair-potential
special case, NVE energy conservation).  Paper numbers: parity unpinned.
"""
