"""FP64 velocity Verlet (the time stepping of the paper's MD runs, section
"Systems and Environment for Measurement of Performance").

Units: positions in A, velocities in A/fs, masses in amu, forces in eV/A,
energies in eV.  1 eV/(A amu) = 1/103.6427 A/fs^2.
"""
from __future__ import annotations

import numpy as np

ACC = 1.0 / 103.642697  # (eV/A)/amu -> A/fs^2
KE = 103.642697         # amu A^2/fs^2 -> eV


def kinetic(masses, vel) -> float:
    return 0.5 * KE * float(np.sum(masses[:, None] * vel * vel))


def velocity_verlet(force_fn, pos, vel, masses, dt, n_steps, wrap_cell=None):
    """Integrate `n_steps`; `force_fn(pos) -> (energy, forces)`.
    Returns (pos, vel, [total energy per step incl. step 0])."""
    pos = np.array(pos, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    m = np.asarray(masses, dtype=np.float64)[:, None]
    e, f = force_fn(pos)
    etot = [e + kinetic(m[:, 0], vel)]
    for _ in range(n_steps):
        vel = vel + 0.5 * dt * ACC * f / m
        pos = pos + dt * vel
        if wrap_cell is not None:
            pos = np.mod(pos, wrap_cell)
        e, f = force_fn(pos)
        vel = vel + 0.5 * dt * ACC * f / m
        etot.append(e + kinetic(m[:, 0], vel))
    return pos, vel, np.asarray(etot)
