"""ctypes binding of liballegro_mi355x.so: argument marshalling only.

Every step of the energy/force path runs in the library's HIP kernels; this
module converts Python/torch arguments into the C interface declared in
include/allegro_mi355x.h and raises on any non-zero status.  There is no
fallback: if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liballegro_mi355x.so")

ALLEGRO_OK = 0
STATUS = {0: "ALLEGRO_OK", -1: "ALLEGRO_E_INVAL", -2: "ALLEGRO_E_NOMEM", -3: "ALLEGRO_E_CAPACITY",
          -4: "ALLEGRO_E_DEVICE", -5: "ALLEGRO_E_NONFINITE", -6: "ALLEGRO_E_STATE"}
PREC_FP32, PREC_BF16, PREC_BF16_SINGLE, PREC_BF16_MIXED = 0, 1, 2, 3
NOALLOC_SCRATCH_BYTES = 256 << 20   # ALLEGRO_NOALLOC_SCRATCH_BYTES

# Every symbol the header declares (checked by the CPU tests).
EXPORTS = ("allegro_describe", "allegro_plan_chunks", "allegro_create", "allegro_neighbors", "allegro_neighbors_batched",
           "allegro_system_energies", "allegro_energy_forces", "allegro_energy_forces_noalloc",
           "allegro_autotune", "allegro_set_tiles", "allegro_set_ghosts", "allegro_md_run", "allegro_md_stats", "allegro_check", "allegro_copy_edges", "allegro_num_edges", "allegro_set_timing", "allegro_kernel_times",
           "allegro_workspace_bytes", "allegro_destroy", "allegro_last_error", "allegro_status_string")


class AllegroConfig(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("n_bessel", ctypes.c_int32),
                ("envelope_p", ctypes.c_int32), ("l_max", ctypes.c_int32),
                ("n_layers", ctypes.c_int32), ("n_tensor", ctypes.c_int32),
                ("twobody_dims", ctypes.c_int32 * 4), ("n_twobody", ctypes.c_int32),
                ("latent_dims", ctypes.c_int32 * 4), ("n_latent", ctypes.c_int32),
                ("edge_dims", ctypes.c_int32 * 4), ("n_edge", ctypes.c_int32),
                ("r_cut", ctypes.c_double), ("avg_num_neighbors", ctypes.c_double),
                ("channel_mix", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("edge_chunk", ctypes.c_int64), ("neighbor_skin", ctypes.c_double),
                ("edge_capacity_hint", ctypes.c_int64),
                ("r_cut_pair", ctypes.POINTER(ctypes.c_double)),
                ("atomic_numbers", ctypes.POINTER(ctypes.c_int32))]


class AllegroInfo(ctypes.Structure):
    _fields_ = [("n_weights", ctypes.c_int64), ("n_paths", ctypes.c_int32 * 4),
                ("n_nonzero", ctypes.c_int32 * 4), ("width", ctypes.c_int32 * 4), ("dim", ctypes.c_int32),
                ("latent", ctypes.c_int32), ("widest_row", ctypes.c_int32),
                ("max_chunk_edges", ctypes.c_int64)]


class AllegroError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


_lib = None


def load_library(path: Optional[str] = None) -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} not found: build it with `python -m paper_2304_10061_amd.build`")
    # torch first: the library then binds to the HIP runtime torch has loaded,
    # rather than loading a second copy that torch's device setup would trip over
    import torch  # noqa: F401
    lib = ctypes.CDLL(p)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.allegro_describe.argtypes = [ctypes.POINTER(AllegroConfig), ctypes.POINTER(AllegroInfo)]
    lib.allegro_describe.restype = ctypes.c_int
    lib.allegro_plan_chunks.argtypes = [ctypes.POINTER(AllegroConfig), i64, vp, i64, vp, ctypes.POINTER(i64)]
    lib.allegro_plan_chunks.restype = ctypes.c_int
    lib.allegro_create.argtypes = [ctypes.POINTER(AllegroConfig), vp, i64, vp, vp, ctypes.POINTER(vp)]
    lib.allegro_create.restype = ctypes.c_int
    lib.allegro_neighbors.argtypes = [vp, i64, i64, dp, dp, vp, vp, vp, ctypes.POINTER(i64)]
    lib.allegro_neighbors.restype = ctypes.c_int
    lib.allegro_neighbors_batched.argtypes = [vp, i32, vp, dp, dp, vp, ctypes.POINTER(i64)]
    lib.allegro_neighbors_batched.restype = ctypes.c_int
    lib.allegro_system_energies.argtypes = [vp, dp, dp, vp]
    lib.allegro_system_energies.restype = ctypes.c_int
    lib.allegro_energy_forces.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp, vp]
    lib.allegro_energy_forces.restype = ctypes.c_int
    lib.allegro_energy_forces_noalloc.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp, vp]
    lib.allegro_energy_forces_noalloc.restype = ctypes.c_int
    lib.allegro_autotune.argtypes = [vp, dp, dp, vp, vp]
    lib.allegro_autotune.restype = ctypes.c_int
    lib.allegro_set_tiles.argtypes = [vp, vp]
    lib.allegro_set_tiles.restype = ctypes.c_int
    lib.allegro_set_ghosts.argtypes = [vp, i64, i64, vp, vp]
    lib.allegro_set_ghosts.restype = ctypes.c_int
    lib.allegro_md_run.argtypes = [vp, i32, ctypes.c_double, dp, dp, dp, dp, dp, dp, dp, i32, i32, vp,
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)]
    lib.allegro_md_run.restype = ctypes.c_int
    lib.allegro_md_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i64)]
    lib.allegro_md_stats.restype = ctypes.c_int
    lib.allegro_check.argtypes = [vp, vp]
    lib.allegro_check.restype = ctypes.c_int
    lib.allegro_copy_edges.argtypes = [vp, dp, dp, dp, vp]
    lib.allegro_copy_edges.restype = ctypes.c_int
    lib.allegro_num_edges.argtypes = [vp]
    lib.allegro_num_edges.restype = i64
    lib.allegro_set_timing.argtypes = [vp, i32]
    lib.allegro_set_timing.restype = ctypes.c_int
    lib.allegro_kernel_times.argtypes = [vp, i32, vp, vp, vp, ctypes.POINTER(i32)]
    lib.allegro_kernel_times.restype = ctypes.c_int
    lib.allegro_workspace_bytes.argtypes = [vp]
    lib.allegro_workspace_bytes.restype = i64
    lib.allegro_destroy.argtypes = [vp]
    lib.allegro_destroy.restype = None
    lib.allegro_last_error.argtypes = [vp]
    lib.allegro_last_error.restype = ctypes.c_char_p
    lib.allegro_status_string.argtypes = [ctypes.c_int]
    lib.allegro_status_string.restype = ctypes.c_char_p
    if path is None:
        _lib = lib
    return lib


def make_config(n_species: int, r_cut: float, *, n_bessel: int = 8, envelope_p: int = 6, l_max: int = 2,
                n_layers: int = 2, n_tensor: int = 32, twobody_dims: Sequence[int] = (128, 128),
                latent_dims: Sequence[int] = (128, 128), edge_dims: Sequence[int] = (128,),
                avg_num_neighbors: Optional[float] = None, channel_mix: bool = True,
                precision: int = PREC_BF16, edge_chunk: int = 0, neighbor_skin: float = 0.0,
                edge_capacity_hint: int = 0,
                r_cut_pair=None, atomic_numbers=None) -> AllegroConfig:
    """r_cut_pair: optional [n_species][n_species] ordered cutoffs (row = centre species);
    atomic_numbers: optional [n_species] (switches on the ZBL pair term)."""
    c = AllegroConfig()
    c.n_species, c.n_bessel, c.envelope_p, c.l_max = n_species, n_bessel, envelope_p, l_max
    c.n_layers, c.n_tensor = n_layers, n_tensor
    for name, dims in (("twobody", twobody_dims), ("latent", latent_dims), ("edge", edge_dims)):
        arr = getattr(c, f"{name}_dims")
        if len(dims) > 4:
            raise ValueError(f"{name}_dims has more than 4 entries")
        for k, v in enumerate(dims):
            arr[k] = int(v)
        setattr(c, f"n_{name}", len(dims))
    c.r_cut = float(r_cut)
    c.avg_num_neighbors = float(avg_num_neighbors if avg_num_neighbors is not None
                                else 0.1 * 4.0 / 3.0 * math.pi * r_cut ** 3)
    c.channel_mix = 1 if channel_mix else 0
    c.precision = int(precision)
    c.edge_chunk = int(edge_chunk)
    c.neighbor_skin = float(neighbor_skin)
    c.edge_capacity_hint = int(edge_capacity_hint)
    if r_cut_pair is not None:
        flat = [float(v) for row in r_cut_pair for v in row]
        if len(flat) != n_species * n_species:
            raise ValueError("r_cut_pair must be n_species x n_species")
        table = (ctypes.c_double * len(flat))(*flat)
        c.r_cut_pair = ctypes.cast(table, ctypes.POINTER(ctypes.c_double))
        c._r_cut_pair_table = table   # kept alive with the config; the library copies it
    if atomic_numbers is not None:
        if len(atomic_numbers) != n_species:
            raise ValueError("atomic_numbers must have n_species entries")
        zt = (ctypes.c_int32 * n_species)(*[int(z) for z in atomic_numbers])
        c.atomic_numbers = ctypes.cast(zt, ctypes.POINTER(ctypes.c_int32))
        c._atomic_numbers_table = zt
    return c


def config_from(mc, precision: int = PREC_BF16, edge_chunk: int = 0, neighbor_skin: float = 0.0,
                edge_capacity_hint: int = 0) -> AllegroConfig:
    """Config from any object with the ModelConfig attribute names."""
    return make_config(mc.n_species, mc.r_cut, n_bessel=mc.n_bessel, envelope_p=mc.envelope_p,
                       l_max=mc.l_max, n_layers=mc.n_layers, n_tensor=mc.n_tensor,
                       twobody_dims=mc.twobody_dims, latent_dims=mc.latent_dims, edge_dims=mc.edge_dims,
                       avg_num_neighbors=mc.avg_num_neighbors, channel_mix=mc.channel_mix,
                       precision=precision, edge_chunk=edge_chunk, neighbor_skin=neighbor_skin,
                       edge_capacity_hint=edge_capacity_hint, r_cut_pair=getattr(mc, "pair_cutoffs", None),
                       atomic_numbers=getattr(mc, "atomic_numbers", None))


def describe(cfg: AllegroConfig) -> AllegroInfo:
    lib = load_library()
    info = AllegroInfo()
    st = lib.allegro_describe(ctypes.byref(cfg), ctypes.byref(info))
    if st != ALLEGRO_OK:
        raise AllegroError(st, lib.allegro_last_error(None).decode())
    return info


def plan_chunks(cfg: AllegroConfig, edges_per_centre) -> np.ndarray:
    """Chunk boundaries (centre indices) that allegro_neighbors would use."""
    lib = load_library()
    cnt = np.ascontiguousarray(edges_per_centre, dtype=np.int32)
    n = ctypes.c_int64(0)
    st = lib.allegro_plan_chunks(ctypes.byref(cfg), cnt.size, cnt.ctypes.data, 0, None, ctypes.byref(n))
    if st != ALLEGRO_OK:
        raise AllegroError(st, lib.allegro_last_error(None).decode())
    out = np.zeros(n.value + 1, dtype=np.int64)
    st = lib.allegro_plan_chunks(ctypes.byref(cfg), cnt.size, cnt.ctypes.data, out.size, out.ctypes.data,
                                 ctypes.byref(n))
    if st != ALLEGRO_OK:
        raise AllegroError(st, lib.allegro_last_error(None).decode())
    return out


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream) or None
    return int(stream) or None


class Model:
    """One model on the current HIP device (wraps allegro_create/destroy)."""

    def __init__(self, cfg: AllegroConfig, weights: np.ndarray, species_scale=None, species_shift=None):
        self.lib = load_library()
        self.cfg = cfg
        w = np.ascontiguousarray(weights, dtype=np.float32)
        sc = None if species_scale is None else np.ascontiguousarray(species_scale, dtype=np.float64)
        sh = None if species_shift is None else np.ascontiguousarray(species_shift, dtype=np.float64)
        h = ctypes.c_void_p()
        st = self.lib.allegro_create(ctypes.byref(cfg), w.ctypes.data, w.size,
                                     None if sc is None else sc.ctypes.data,
                                     None if sh is None else sh.ctypes.data, ctypes.byref(h))
        if st != ALLEGRO_OK:
            raise AllegroError(st, self.lib.allegro_last_error(None).decode())
        self.handle = h
        self.n_local = None
        self.n_total = None

    def _check(self, st: int):
        if st != ALLEGRO_OK:
            raise AllegroError(st, self.lib.allegro_last_error(self.handle).decode())

    def close(self):
        if getattr(self, "handle", None):
            self.lib.allegro_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def neighbors(self, pos, species, cell, pbc, n_local: Optional[int] = None, stream=None) -> int:
        """Build the neighbour list (pos: cuda float64 [N][3], species: cuda int32 [N])."""
        n_total = int(pos.shape[0])
        n_local = n_total if n_local is None else int(n_local)
        cell9 = np.zeros(9, dtype=np.float64)
        c = np.asarray(cell, dtype=np.float64).reshape(-1)
        if c.size == 3:
            cell9[[0, 4, 8]] = c
        elif c.size == 9:
            cell9[:] = c
        pb = np.asarray(pbc, dtype=np.int32).reshape(3)
        ne = ctypes.c_int64(0)
        self._check(self.lib.allegro_neighbors(self.handle, n_local, n_total, _ptr(pos), _ptr(species),
                                               cell9.ctypes.data, pb.ctypes.data, _stream(stream),
                                               ctypes.byref(ne)))
        self.n_local, self.n_total = n_local, n_total
        return int(ne.value)

    def neighbors_batched(self, atom_offsets, pos, species, stream=None) -> int:
        """Neighbour list of independent non-periodic systems (host offsets)."""
        off = np.ascontiguousarray(atom_offsets, dtype=np.int64)
        ne = ctypes.c_int64(0)
        self._check(self.lib.allegro_neighbors_batched(self.handle, int(off.size - 1), off.ctypes.data, _ptr(pos),
                                                       _ptr(species), _stream(stream), ctypes.byref(ne)))
        self.n_local = self.n_total = int(off[-1])
        return int(ne.value)

    def system_energies(self, atom_energy, system_energy, stream=None):
        self._check(self.lib.allegro_system_energies(self.handle, _ptr(atom_energy), _ptr(system_energy),
                                                     _stream(stream)))

    def energy_forces(self, pos, species, forces, atom_energy=None, virial=None, atom_virial=None,
                      energy=None, stream=None):
        """Enqueue one evaluation; outputs are caller-owned cuda float64 tensors."""
        self._check(self.lib.allegro_energy_forces(self.handle, _ptr(pos), _ptr(species), _ptr(atom_energy),
                                                   _ptr(forces), _ptr(virial), _ptr(atom_virial),
                                                   _ptr(energy), _stream(stream)))

    def energy_forces_noalloc(self, pos, species, forces, atom_energy=None, virial=None, atom_virial=None,
                              energy=None, stream=None):
        """energy_forces on the library's static per-GPU workspace (allocates nothing)."""
        self._check(self.lib.allegro_energy_forces_noalloc(self.handle, _ptr(pos), _ptr(species),
                                                           _ptr(atom_energy), _ptr(forces), _ptr(virial),
                                                           _ptr(atom_virial), _ptr(energy), _stream(stream)))

    TILE_KINDS = ("mlp_fwd_twobody", "mlp_fwd_latent", "mlp_fwd_final", "mlp_bwd_final", "mlp_bwd_latent",
                  "mlp_bwd_twobody", "tp_mix", "mix_adjoint")

    def autotune(self, pos, species, stream=None):
        """Pick the fastest edge-tile shapes on the current neighbour list."""
        ch = (ctypes.c_int32 * 8)()
        self._check(self.lib.allegro_autotune(self.handle, _ptr(pos), _ptr(species), _stream(stream), ch))
        return dict(zip(self.TILE_KINDS, list(ch)))

    def set_tiles(self, tiles):
        """Set edge-tile shapes: a dict over TILE_KINDS (missing = 0, the default) or 8 ints."""
        if isinstance(tiles, dict):
            tiles = [int(tiles.get(k, 0)) for k in self.TILE_KINDS]
        arr = (ctypes.c_int32 * 8)(*[int(t) for t in tiles])
        self._check(self.lib.allegro_set_tiles(self.handle, arr))

    def set_ghosts(self, n_local: int, owner, offset):
        """Ghost g = atom n_local + g is owner[g]'s image at offset[g] (host arrays)."""
        ow = np.ascontiguousarray(owner, dtype=np.int32)
        of = np.ascontiguousarray(offset, dtype=np.float64).reshape(-1, 3)
        self._check(self.lib.allegro_set_ghosts(self.handle, int(n_local), int(ow.size),
                                                ow.ctypes.data if ow.size else None,
                                                of.ctypes.data if ow.size else None))

    def md_run(self, n_steps, dt_fs, masses, pos, vel, forces, species, thermo=None, init_forces=False,
               use_graph=True, stream=None, want_max_disp=True, virial=None):
        """Velocity Verlet on the device; returns the max displacement since the
        last neighbour build (or None).  thermo [n_steps][2] and virial
        [n_steps][9] (cuda float64, optional) receive (E_pot, E_kin) and the
        virial of each step.  Raises AllegroError (ALLEGRO_E_CAPACITY with
        .steps_done set) when an in-graph rebuild outgrew the capacity."""
        md = ctypes.c_double(0.0)
        done = ctypes.c_int32(0)
        st = self.lib.allegro_md_run(self.handle, int(n_steps), float(dt_fs), _ptr(masses), _ptr(pos),
                                     _ptr(vel), _ptr(forces), _ptr(species), _ptr(thermo), _ptr(virial),
                                     1 if init_forces else 0, 1 if use_graph else 0, _stream(stream),
                                     ctypes.byref(md) if want_max_disp else None, ctypes.byref(done))
        if st != ALLEGRO_OK:
            err = AllegroError(st, self.lib.allegro_last_error(self.handle).decode())
            err.steps_done = int(done.value)
            raise err
        return md.value if want_max_disp else None

    def md_run_all(self, n_steps, dt_fs, masses, pos, vel, forces, species, thermo=None, init_forces=False,
                   use_graph=True, stream=None, max_overflows=16, virial=None):
        """md_run for n_steps, resuming after each ALLEGRO_E_CAPACITY (the
        library has regrown the list by then); returns (max displacement since
        the last build, number of overflows)."""
        done, overflows = 0, 0
        while True:
            try:
                d = self.md_run(n_steps - done, dt_fs, masses, pos, vel, forces, species,
                                thermo=None if thermo is None else thermo[done:], init_forces=init_forces and done == 0,
                                use_graph=use_graph, stream=stream,
                                virial=None if virial is None else virial[done:])
                return d, overflows
            except AllegroError as e:
                if e.status != -3 or overflows >= max_overflows:
                    raise
                overflows += 1
                done += e.steps_done

    def md_stats(self):
        """(graph captures so far, edge capacity, 1 if rebuilds run on the device,
        list rebuilds during the last md_run)."""
        caps, cap, dev, nb = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int32(0), ctypes.c_int64(0)
        self._check(self.lib.allegro_md_stats(self.handle, ctypes.byref(caps), ctypes.byref(cap), ctypes.byref(dev),
                                              ctypes.byref(nb)))
        return int(caps.value), int(cap.value), int(dev.value), int(nb.value)

    def check(self, stream=None):
        """Synchronise and raise AllegroError if an evaluation since the last
        check produced non-finite energies or forces."""
        self._check(self.lib.allegro_check(self.handle, _stream(stream)))

    def num_edges(self) -> int:
        return int(self.lib.allegro_num_edges(self.handle))

    def workspace_bytes(self) -> int:
        return int(self.lib.allegro_workspace_bytes(self.handle))

    def set_timing(self, enable: bool):
        self._check(self.lib.allegro_set_timing(self.handle, 1 if enable else 0))

    def kernel_times(self):
        """{kernel kind: (total ms, launches)} since the last set_timing()."""
        n = ctypes.c_int32(0)
        self._check(self.lib.allegro_kernel_times(self.handle, 0, None, None, None, ctypes.byref(n)))
        k = n.value
        names = ctypes.create_string_buffer(48 * max(k, 1))
        ms = (ctypes.c_double * max(k, 1))()
        cnt = (ctypes.c_int64 * max(k, 1))()
        self._check(self.lib.allegro_kernel_times(self.handle, k, names, ms, cnt, ctypes.byref(n)))
        out = {}
        for q in range(k):
            nm = names.raw[48 * q:48 * q + 48].split(b"\0", 1)[0].decode()
            out[nm] = (float(ms[q]), int(cnt[q]))
        return out

    def copy_edges(self, stream=None):
        import torch
        E = self.num_edges()
        dev = torch.device("cuda", torch.cuda.current_device())
        ci = torch.empty(E, dtype=torch.int32, device=dev)
        nj = torch.empty(E, dtype=torch.int32, device=dev)
        sh = torch.empty((E, 3), dtype=torch.int32, device=dev)
        self._check(self.lib.allegro_copy_edges(self.handle, _ptr(ci), _ptr(nj), _ptr(sh), _stream(stream)))
        return ci, nj, sh

    def evaluate(self, pos, species, cell, pbc, n_local=None, want_atom_virial=False):
        """Convenience: neighbours + energy/forces, returns a dict of cuda tensors."""
        import torch
        self.neighbors(pos, species, cell, pbc, n_local)
        n_total = int(pos.shape[0])
        dev = pos.device
        out = dict(forces=torch.empty((n_total, 3), dtype=torch.float64, device=dev),
                   atom_energy=torch.empty(self.n_local, dtype=torch.float64, device=dev),
                   virial=torch.empty(9, dtype=torch.float64, device=dev),
                   energy=torch.empty(1, dtype=torch.float64, device=dev))
        if want_atom_virial:
            out["atom_virial"] = torch.empty((n_total, 9), dtype=torch.float64, device=dev)
        self.energy_forces(pos, species, out["forces"], out["atom_energy"], out["virial"],
                           out.get("atom_virial"), out["energy"])
        self.check()   # synchronises; raises on non-finite outputs
        return out
