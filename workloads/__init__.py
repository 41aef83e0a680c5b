"""Seeded synthetic workloads shared by the oracle and the HIP path.

This module holds no arithmetic of the potential itself: it only draws random
numbers (lattice subsets, jitter, species labels, weights, velocities, cluster
sizes) and packages hyper-parameters.  Both the FP64 oracle and the GPU path
consume what it produces; neither side's numerics live here.

Stand-ins for the paper's structures: the paper measures on AMBER20 protein
boxes (DHFR 23k atoms, STMV 1M atoms) and replicated water (section "Scientific
applications used to measure performance").  Those structures are not
available, so the generators below make jittered-lattice boxes and random-packed
clusters with the same atom counts, the same liquid-water number density
(0.1 atoms per cubic Angstrom) and protein-like species mixes.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

DENSITY = 0.1  # atoms / A^3, liquid-water number density

# Species indices used throughout: 0 = H, 1 = C, 2 = N, 3 = O for 4-species
# mixes; 0 = H, 1 = O for the 2-species water-like mix.
MASSES_4 = (1.008, 12.011, 14.007, 15.999)
MASSES_2 = (1.008, 15.999)

# Ordered-pair cutoffs the paper used (section "Training details"): H-H 3.0,
# H-C 1.25, H-O 1.25, O-H 3.0 A, every other ordered pair the default cutoff.
PAPER_PAIR_CUTOFFS = {("H", "H"): 3.0, ("H", "C"): 1.25, ("H", "O"): 1.25, ("O", "H"): 3.0}


def atomic_numbers(n_species: int):
    """Atomic numbers of the 2-species (H, O) or 4-species (H, C, N, O) mixes."""
    return (1, 8) if n_species == 2 else (1, 6, 7, 8)


def paper_pair_cutoffs(n_species: int, r_cut: float):
    """[S][S] table of those cutoffs for the 2-species (H, O) or 4-species
    (H, C, N, O) mixes used here; pairs the paper does not list get r_cut."""
    names = ("H", "O") if n_species == 2 else ("H", "C", "N", "O")
    return tuple(tuple(min(r_cut, PAPER_PAIR_CUTOFFS.get((a, b), r_cut)) for b in names) for a in names)


@dataclasses.dataclass
class ModelConfig:
    """Hyper-parameters of one Allegro model (all bias-free MLPs)."""
    n_species: int
    r_cut: float
    n_bessel: int = 8
    envelope_p: int = 6
    l_max: int = 2
    n_layers: int = 2
    n_tensor: int = 32
    twobody_dims: Sequence[int] = (128, 128)
    latent_dims: Sequence[int] = (128, 128)
    edge_dims: Sequence[int] = (128,)
    avg_num_neighbors: Optional[float] = None
    channel_mix: bool = True
    # ordered per-species-pair cutoffs rc[Z_centre][Z_neighbour] (A), each at
    # most r_cut; None = r_cut for every pair
    pair_cutoffs: Optional[Sequence[Sequence[float]]] = None
    # atomic number of each species for the ZBL repulsion; None = no ZBL term
    atomic_numbers: Optional[Sequence[int]] = None

    def __post_init__(self):
        self.twobody_dims = tuple(int(v) for v in self.twobody_dims)
        self.latent_dims = tuple(int(v) for v in self.latent_dims)
        self.edge_dims = tuple(int(v) for v in self.edge_dims)
        if self.avg_num_neighbors is None:
            self.avg_num_neighbors = DENSITY * 4.0 / 3.0 * math.pi * self.r_cut ** 3
        if self.pair_cutoffs is not None:
            self.pair_cutoffs = tuple(tuple(float(v) for v in row) for row in self.pair_cutoffs)
            if len(self.pair_cutoffs) != self.n_species or any(len(r) != self.n_species for r in self.pair_cutoffs):
                raise ValueError("pair_cutoffs must be n_species x n_species")

    @property
    def latent(self) -> int:
        return self.latent_dims[-1]


@dataclasses.dataclass
class System:
    """Positions (FP64, [N][3]), species (int32, [N]) and an orthorhombic cell.

    `n_local` atoms are centres; atoms `[n_local, n_total)` are ghosts that only
    appear as neighbours.  `atom_offsets` (len n_systems+1) splits a batch of
    independent non-periodic systems.
    """
    pos: np.ndarray
    species: np.ndarray
    cell: np.ndarray          # [3] box lengths (orthorhombic); ignored where pbc is 0
    pbc: np.ndarray           # [3] int32
    n_local: int
    masses: Optional[np.ndarray] = None
    atom_offsets: Optional[np.ndarray] = None

    @property
    def n_total(self) -> int:
        return int(self.pos.shape[0])


def seeds(cfg_seed: int) -> List[np.random.Generator]:
    """[lattice subset, jitter, species, weights, velocities, cluster sizes]."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(cfg_seed).spawn(6)]


def largest_remainder(n: int, ratio: Sequence[float]) -> List[int]:
    r = np.asarray(ratio, dtype=np.float64)
    quota = n * r / r.sum()
    base = np.floor(quota).astype(np.int64)
    rest = n - int(base.sum())
    order = np.argsort(-(quota - base), kind="stable")
    base[order[:rest]] += 1
    return [int(v) for v in base]


def assign_species(n: int, ratio: Sequence[float], rng: np.random.Generator) -> np.ndarray:
    counts = largest_remainder(n, ratio)
    labels = np.concatenate([np.full(c, k, dtype=np.int32) for k, c in enumerate(counts)])
    return labels[rng.permutation(n)].astype(np.int32)


def jittered_lattice_box(n_atoms: int, box: float, jitter: float, ratio: Sequence[float],
                         cfg_seed: int, sites_per_side: Optional[int] = None) -> System:
    """`n_atoms` sites of an m^3 simple-cubic lattice (m = ceil(N^(1/3))) in a
    periodic cube of side `box`, jittered by U(-jitter, jitter) per coordinate
    and wrapped into [0, box)."""
    rs = seeds(cfg_seed)
    m = sites_per_side or int(math.ceil(round(n_atoms ** (1.0 / 3.0), 9)))
    while m ** 3 < n_atoms:
        m += 1
    a = box / m
    g = np.arange(m, dtype=np.float64)
    sites = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    if n_atoms < m ** 3:
        keep = np.sort(rs[0].choice(m ** 3, size=n_atoms, replace=False))
        sites = sites[keep]
    pos = (sites + 0.5) * a + rs[1].uniform(-jitter, jitter, size=(n_atoms, 3))
    pos = np.mod(pos, box)
    pos[pos >= box] -= box  # mod can return box for tiny negatives
    species = assign_species(n_atoms, ratio, rs[2])
    masses_tab = MASSES_4 if len(ratio) == 4 else MASSES_2
    return System(pos=pos, species=species, cell=np.full(3, float(box)),
                  pbc=np.ones(3, np.int32), n_local=n_atoms,
                  masses=np.asarray(masses_tab)[species])


def random_packed_cluster(n_atoms: int, rng: np.random.Generator, min_sep: float = 0.9) -> np.ndarray:
    """Random sequential insertion into a sphere of volume n/DENSITY."""
    radius = (3.0 * n_atoms / (4.0 * math.pi * DENSITY)) ** (1.0 / 3.0)
    pts = np.empty((n_atoms, 3))
    k = 0
    while k < n_atoms:
        cand = rng.uniform(-radius, radius, size=(4 * (n_atoms - k) + 16, 3))
        cand = cand[np.einsum("ij,ij->i", cand, cand) <= radius * radius]
        for c in cand:
            if k == n_atoms:
                break
            if k == 0 or np.min(np.sum((pts[:k] - c) ** 2, axis=1)) >= min_sep * min_sep:
                pts[k] = c
                k += 1
    return pts


def ghost_shell(sysm: System, shell: float) -> System:
    """Append periodic images of the local atoms that lie within `shell` of
    the box faces (outside the box); the result is non-periodic with
    `n_local` centres and ghosts after them."""
    L = sysm.cell
    imgs, owners = [], []
    rng3 = (-1, 0, 1)
    for sx in rng3:
        for sy in rng3:
            for sz in rng3:
                if sx == 0 and sy == 0 and sz == 0:
                    continue
                s = np.array([sx, sy, sz], dtype=np.float64)
                p = sysm.pos + s * L
                inside = np.all((p > -shell) & (p < L + shell), axis=1)
                idx = np.nonzero(inside)[0]
                imgs.append(p[idx])
                owners.append(idx)
    gpos = np.concatenate(imgs)
    gown = np.concatenate(owners).astype(np.int64)
    out = System(pos=np.concatenate([sysm.pos, gpos]),
                 species=np.concatenate([sysm.species, sysm.species[gown]]).astype(np.int32),
                 cell=L.copy(), pbc=np.zeros(3, np.int32), n_local=sysm.n_local,
                 masses=None if sysm.masses is None else np.concatenate([sysm.masses, sysm.masses[gown]]))
    out.ghost_owner = gown  # type: ignore[attr-defined]
    return out


# ----------------------------------------------------------------------------
# Workload configurations
# ----------------------------------------------------------------------------

PROTEIN_MIX = (50, 30, 8, 12)  # H:C:N:O
WATER_MIX = (2, 1)             # H:O


def model_config(cfg: int) -> ModelConfig:
    if cfg == 1:
        return ModelConfig(n_species=2, r_cut=4.0, l_max=1, n_layers=1, n_tensor=8,
                           twobody_dims=(32, 32), latent_dims=(32, 32), edge_dims=(128,))
    if cfg == 2:
        return ModelConfig(n_species=2, r_cut=4.0, l_max=2, n_layers=2, n_tensor=32,
                           twobody_dims=(128, 128), latent_dims=(128, 128), edge_dims=(128,))
    if cfg == 3:
        return ModelConfig(n_species=4, r_cut=6.0, l_max=2, n_layers=2, n_tensor=64,
                           twobody_dims=(256, 256, 256), latent_dims=(256, 256, 256),
                           edge_dims=(128,))
    if cfg in (4, 5):
        return ModelConfig(n_species=4, r_cut=4.0, l_max=2, n_layers=2, n_tensor=32,
                           twobody_dims=(128, 128), latent_dims=(128, 128), edge_dims=(128,))
    raise ValueError(cfg)


def deep_model_config() -> ModelConfig:
    """The water-box model deepened to three tensor-product layers with
    l_max = 3 (unnatural-parity irreps in the middle layer's input, l = 3
    harmonics); same MLP widths, channels and cutoff as the 3,000-atom model."""
    return ModelConfig(n_species=2, r_cut=4.0, l_max=3, n_layers=3, n_tensor=32,
                       twobody_dims=(128, 128), latent_dims=(128, 128), edge_dims=(128,))


def deep_workload():
    """(ModelConfig, System, weights): the deep model on the 3,000-atom water box."""
    mc = deep_model_config()
    sysm = system(2)
    w = make_weights(mc, np.random.default_rng(np.random.SeedSequence(6).spawn(6)[3]))
    return mc, sysm, w


def system(cfg: int) -> System:
    if cfg == 1:
        return jittered_lattice_box(64, 8.6, 0.3, WATER_MIX, 1, sites_per_side=4)
    if cfg == 2:
        return jittered_lattice_box(3000, 31.1, 0.4, WATER_MIX, 2, sites_per_side=15)
    if cfg == 3:
        box = (23558 / DENSITY) ** (1.0 / 3.0)
        return jittered_lattice_box(23558, box, 0.5, PROTEIN_MIX, 3, sites_per_side=29)
    if cfg == 4:
        base = jittered_lattice_box(1_000_000, 215.0, 0.5, PROTEIN_MIX, 4, sites_per_side=100)
        return ghost_shell(base, 6.0)
    if cfg == 5:
        return clusters(512, 5)
    raise ValueError(cfg)


def clusters(n_systems: int, cfg_seed: int, lo: int = 20, hi: int = 2000,
             ratio: Sequence[float] = PROTEIN_MIX, spacing: float = 0.0) -> System:
    """`n_systems` non-periodic clusters with log-uniform sizes in [lo, hi].

    Clusters are stacked along x with a gap larger than any cutoff when
    `spacing` > 0 (only useful for visual checks); batched evaluation never
    mixes systems regardless of their coordinates.
    """
    rs = seeds(cfg_seed)
    sizes = np.floor(np.exp(rs[5].uniform(math.log(lo), math.log(hi), size=n_systems))).astype(np.int64)
    sizes = np.clip(sizes, lo, hi)
    pos, spec = [], []
    for k, nk in enumerate(sizes):
        p = random_packed_cluster(int(nk), rs[0])
        if spacing:
            p[:, 0] += k * spacing
        pos.append(p)
        spec.append(assign_species(int(nk), ratio, rs[2]))
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    species = np.concatenate(spec).astype(np.int32)
    return System(pos=np.concatenate(pos), species=species, cell=np.zeros(3),
                  pbc=np.zeros(3, np.int32), n_local=int(offs[-1]),
                  masses=np.asarray(MASSES_4)[species], atom_offsets=offs)


# ----------------------------------------------------------------------------
# Weights
# ----------------------------------------------------------------------------

def _normal(rng: np.random.Generator, shape, var: float) -> np.ndarray:
    return (rng.standard_normal(shape) * math.sqrt(var)).astype(np.float32)


def weight_shapes(mc: ModelConfig) -> List[tuple]:
    """Ordered (name, shape) list: the flat weight format of the C interface.

    Every array is row-major float32.  MLP matrices are [fan_in, fan_out]
    (y = x @ W).  Columns of `embed0` and `layer*.env` are indexed l*n + u
    (irrep order l = 0..l_max, channel u).  `alpha` is indexed
    [l1][l2][l_out] over 0..l_max (entries of unused paths are ignored);
    `mix` is [l][v][u] (output channel v, input channel u).  Models of three
    or more layers, whose middle layers carry both parities, use
    [2][l1][l2][l_out] for `alpha` (leading index 0 for a natural-parity
    input irrep (l1, (-1)^l1), 1 for the other parity) and 2 (l_max + 1)
    mixing matrices (natural l = 0..l_max, then the other parity).
    """
    n, lm1, d = mc.n_tensor, mc.l_max + 1, mc.latent
    par = 2 if mc.n_layers >= 3 else 1
    out = []
    dims = [2 * mc.n_species + mc.n_bessel] + list(mc.twobody_dims)
    for k in range(len(dims) - 1):
        out.append((f"twobody.W{k}", (dims[k], dims[k + 1])))
    out.append(("embed0", (mc.twobody_dims[-1], lm1 * n)))
    prev = mc.twobody_dims[-1]
    for L in range(1, mc.n_layers + 1):
        out.append((f"layer{L}.env", (prev, lm1 * n)))
        out.append((f"layer{L}.alpha", (2, lm1, lm1, lm1) if par == 2 else (lm1, lm1, lm1)))
        out.append((f"layer{L}.mix", (par * lm1, n, n)))
        dims = [prev + n] + list(mc.latent_dims)
        for k in range(len(dims) - 1):
            out.append((f"layer{L}.mlp.W{k}", (dims[k], dims[k + 1])))
        prev = mc.latent_dims[-1]
    dims = [prev] + list(mc.edge_dims) + [1]
    for k in range(len(dims) - 1):
        out.append((f"edge.W{k}", (dims[k], dims[k + 1])))
    return out


def make_weights(mc: ModelConfig, rng: np.random.Generator) -> Dict[str, np.ndarray]:
    """MLP and linear weights ~ N(0, 1/fan_in); path weights alpha and channel
    mixing matrices ~ N(0, 1) (their normalisation belongs to the model)."""
    w = {}
    for name, shape in weight_shapes(mc):
        if name.endswith(".alpha") or name.endswith(".mix"):
            w[name] = _normal(rng, shape, 1.0)
        else:
            w[name] = _normal(rng, shape, 1.0 / shape[0])
    return w


def pack_weights(mc: ModelConfig, w: Dict[str, np.ndarray]) -> np.ndarray:
    parts = []
    for name, shape in weight_shapes(mc):
        a = np.asarray(w[name], dtype=np.float32)
        if a.shape != tuple(shape):
            raise ValueError(f"{name}: shape {a.shape} != {shape}")
        parts.append(a.reshape(-1))
    return np.concatenate(parts).astype(np.float32)


def species_scale_shift(mc: ModelConfig, rng: Optional[np.random.Generator] = None):
    """sigma = 1, mu = 0 by default; random positive scales/shifts if rng given."""
    if rng is None:
        return np.ones(mc.n_species), np.zeros(mc.n_species)
    return rng.uniform(0.5, 1.5, mc.n_species), rng.uniform(-3.0, 3.0, mc.n_species)


def workload(cfg: int):
    """(ModelConfig, System, weights) for one of the five configurations."""
    mc = model_config(cfg)
    sysm = system(cfg)
    w = make_weights(mc, seeds(cfg)[3])
    return mc, sysm, w


def maxwell_boltzmann(masses: np.ndarray, temperature: float, rng: np.random.Generator) -> np.ndarray:
    """Velocities in A/fs at `temperature` K with zero net momentum."""
    kB = 8.617333262e-5          # eV/K
    conv = 1.0 / 103.6427        # sqrt(eV/amu) -> A/fs is sqrt(1/103.6427)
    sig = np.sqrt(kB * temperature / masses * conv)
    v = rng.standard_normal((masses.shape[0], 3)) * sig[:, None]
    p = (masses[:, None] * v).sum(0) / masses.sum()
    return v - p[None, :]
