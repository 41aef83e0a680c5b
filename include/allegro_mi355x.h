/*
 * allegro_mi355x.h - C interface of the MI355X (gfx950) Allegro energy-and-force
 * library.
 *
 * The method (arXiv 2304.10061, section "Allegro: Scalable Equivariant Deep
 * Learning"): the total energy is a sum of per-species scaled and shifted atomic
 * energies, E = sum_i sigma_{Z_i} E_i + mu_{Z_i}; each atomic energy is a sum of
 * ordered-pair energies E_i = sum_{j in N(i)} E_ij over the neighbours j of i
 * within the cutoff r_c; the pair energies come from a strictly local network
 * of scalar (latent MLP) and tensor (Clebsch-Gordan tensor product, Eq. tp)
 * tracks.  Molecular dynamics needs forces every step (section "Problem
 * overview"), returned here as F = -dE/dx together with per-atom energies and
 * the virial, as an MD engine's pair style consumes them (section "Optimized
 * LAMMPS-Kokkos implementation").  Units: eV and Angstrom (section "Training
 * details").
 *
 * Conventions for every entry point
 *  - Returns ALLEGRO_OK (0) or a negative status; never aborts and never lets a
 *    C++ exception escape.  allegro_last_error() describes the last failure.
 *  - "dev" pointers are device (HBM) pointers owned by the caller; "host"
 *    pointers are host memory owned by the caller.  The library owns the
 *    neighbour list, the coupling tables, the packed weights and its workspace.
 *  - All device work is ordered on `stream` (a hipStream_t; NULL = the default
 *    stream).  Functions that report a count to the host synchronise that
 *    stream.  A model handle is not thread-safe.
 *  - Atoms [0, n_local) are centres; atoms [n_local, n_total) are ghosts that
 *    only appear as neighbours (one GPU's spatial-decomposition share).
 */
#ifndef ALLEGRO_MI355X_H
#define ALLEGRO_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ALLEGRO_OK = 0,
  ALLEGRO_E_INVAL = -1,     /* bad argument, shape or unsupported configuration */
  ALLEGRO_E_NOMEM = -2,     /* device or host allocation failed */
  ALLEGRO_E_CAPACITY = -3,  /* a neighbour-list rebuild inside allegro_md_run
                               needed more edges than the list's capacity; the
                               capacity has been regrown, the steps before it are
                               complete, call again for the rest */
  ALLEGRO_E_DEVICE = -4,    /* a HIP runtime call failed */
  ALLEGRO_E_NONFINITE = -5, /* non-finite positions (allegro_neighbors), or a
                               non-finite atom energy or force was produced
                               (reported by allegro_check / allegro_md_run) */
  ALLEGRO_E_STATE = -6      /* call order violated (e.g. no neighbour list yet) */
};

/* Precision of the MLP GEMMs (everything else is the same in all modes):
 *   FP32         FP32 MFMA.
 *   BF16         BF16 MFMA with FP32 accumulation; activations rounded once to
 *                BF16, each weight held as a pair of BF16 numbers (w = hi + lo)
 *                and applied with two MFMAs, so the fixed rounding of the
 *                weights does not bias every pair energy the same way.
 *   BF16_SINGLE  BF16 MFMA with single-rounded weights (fastest; its energies
 *                carry a systematic error from the weight rounding).
 *   BF16_MIXED   weight pairs only where a fixed rounding adds up coherently
 *                over edges: every layer of the two-body MLP (its inputs are
 *                species one-hots and a smooth radial basis) and the first
 *                layer of each later latent MLP (it reads the residual stream);
 *                the other layers and the environment embedding single-rounded. */
enum {
  ALLEGRO_PREC_FP32 = 0,
  ALLEGRO_PREC_BF16 = 1,
  ALLEGRO_PREC_BF16_SINGLE = 2,
  ALLEGRO_PREC_BF16_MIXED = 3
};

typedef struct AllegroModel AllegroModel; /* opaque, library-owned */

/*
 * Model hyper-parameters (section "Training details" lists the kinds: two-body
 * latent MLP, later latent MLPs, a linear environment embedding, an edge-energy
 * MLP with one hidden layer and no nonlinearity, 8 Bessel functions with a
 * polynomial envelope, l_max = 2, full O(3)).
 *   n_species        number of atom types (one-hot width), 1..12, with 2 n_species + n_bessel <= 32
 *   n_bessel         radial basis size, 1..16 (1..8 with l_max = 3)
 *   envelope_p       polynomial envelope exponent p (u(r_c) = u' = u'' = 0)
 *   l_max            1, 2 or 3
 *   n_layers         1..4 Allegro (tensor product) layers.  With three or more
 *                    layers the features of all but the last two layers carry
 *                    both parities (section "Optimized tensor product": every
 *                    path with p_out = p1 p2 is kept when it can still reach the
 *                    scalar output), e.g. 1o x 1o -> 1e
 *   n_tensor         tensor feature channels n: 8, 16, 32 or 64 (32 or 64 with
 *                    l_max = 3 or three or more layers)
 *   twobody_dims     output widths of the two-body MLP (1..3 layers); the last
 *                    one is the latent width d
 *   latent_dims      output widths of each later latent MLP (1..3 layers); last = d
 *   edge_dims        hidden width(s) of the edge-energy MLP (exactly 1 entry)
 *   r_cut            cutoff radius (A)
 *   avg_num_neighbors  environment-sum normalisation, the sum is scaled by
 *                    1/sqrt(avg_num_neighbors)
 *   channel_mix      1 = per-irrep linear channel mixing after each tensor
 *                    product, 0 = none
 *   precision        one of the ALLEGRO_PREC_* modes above
 *   edge_chunk       0 = evaluate all edges at once; otherwise the largest
 *                    number of edges whose activations are held at a time
 *                    (whole centre segments; bounds workspace memory).  Either
 *                    way a chunk holds at most AllegroInfo.max_chunk_edges
 *                    edges (32-bit workspace offsets); larger edge sets are
 *                    split into chunks automatically, and a single centre with
 *                    more neighbours than that is rejected (ALLEGRO_E_INVAL)
 *   neighbor_skin    extra radius of the neighbour list (A), so that a list can
 *                    be reused over several MD steps; pairs beyond r_cut carry
 *                    a zero envelope and contribute exactly zero.  0 = the list
 *                    holds exactly the pairs inside r_cut.
 *   edge_capacity_hint  edges the neighbour-list buffers hold (fixed-shape
 *                    buffers for in-graph rebuilds in allegro_md_run, section
 *                    "Optimized LAMMPS-Kokkos implementation": preprocessing on
 *                    the device into padded buffers).  0 = 5 % more than the
 *                    list allegro_neighbors builds; otherwise at least this
 *                    many (never fewer than the list).  The capacity only
 *                    grows; a rebuild inside allegro_md_run that needs more
 *                    returns ALLEGRO_E_CAPACITY after regrowing it.
 *   r_cut_pair       host [n_species][n_species] cutoffs of ordered species pairs
 *                    (A), row = species of the centre, column = species of the
 *                    neighbour, each in (0, r_cut]; or NULL = r_cut for every
 *                    pair (section "Species-dependent cutoffs": a pair (i, j) is
 *                    a neighbour iff d_ij < r_cut_pair[Z_i][Z_j], and its radial
 *                    basis and envelope are scaled to that cutoff).  Read by
 *                    allegro_describe / allegro_create and copied; the skin is
 *                    added to every pair's radius.
 *   atomic_numbers   host [n_species] atomic number of each species (1..118), or
 *                    NULL = no pair term.  When given, the ZBL screened-Coulomb
 *                    repulsion the paper adds for stability (section "Training
 *                    details") enters every atom's energy unscaled:
 *                    A_i += sum_j 1/2 E_ZBL(d_ij) u(d_ij / r_c,ij), the ZBL
 *                    universal potential (k_e Z_i Z_j / d phi(d / a),
 *                    a = 0.4685 A / (Z_i^0.23 + Z_j^0.23)) under each edge's own
 *                    envelope; forces and virial include it.  Read at create and
 *                    copied.
 * MLP widths must be multiples of 16 and at most 512; the latent width d at most 256.
 */
typedef struct {
  int32_t n_species, n_bessel, envelope_p, l_max, n_layers, n_tensor;
  int32_t twobody_dims[4], n_twobody;
  int32_t latent_dims[4], n_latent;
  int32_t edge_dims[4], n_edge;
  double r_cut, avg_num_neighbors;
  int32_t channel_mix;
  int32_t precision;
  int64_t edge_chunk;
  double neighbor_skin;
  int64_t edge_capacity_hint;
  const double* r_cut_pair;
  const int32_t* atomic_numbers;
} AllegroConfig;

/* Host-side description of a configuration (no device work). */
typedef struct {
  int64_t n_weights;          /* floats expected by allegro_create */
  int32_t n_paths[4];         /* kept tensor-product paths per layer */
  int32_t n_nonzero[4];       /* non-zeros of each layer's fused coupling table */
  int32_t width[4];           /* strided components of each layer's output features
                                 ((l_max+1)^2, twice that with both parities, 1 for the last) */
  int32_t dim;                /* (l_max+1)^2 strided components */
  int32_t latent;             /* latent width d */
  int32_t widest_row;         /* widest per-edge (or per-centre) row of the
                                 evaluation's workspace, in floats */
  int64_t max_chunk_edges;    /* most edges evaluated at a time: the kernels
                                 address workspace rows with 32-bit element
                                 offsets, so a chunk holds at most
                                 (2^31 - 1) / widest_row edges; a larger
                                 edge_chunk (or 0) is reduced to this */
} AllegroInfo;

/*
 * allegro_describe: validate `cfg` and describe it (host only, no GPU needed).
 * Path selection and pruning follow section "Optimized tensor product": every
 * (l1,p1) x (l2,p2) -> (l_out,p_out) with |l1-l2| <= l_out <= l1+l2,
 * p_out = p1 p2, keeping only paths that can still reach the final scalars.
 * Returns ALLEGRO_E_INVAL for unsupported configurations.
 */
int allegro_describe(const AllegroConfig* cfg, AllegroInfo* info);

/*
 * allegro_plan_chunks: the split of the centres into evaluation chunks that
 * allegro_neighbors applies (host only, no GPU needed).  Centres [0, n_centres)
 * are cut into consecutive runs of whole centre segments (section "Allegro:
 * Scalable Equivariant Deep Learning": each atom's energy depends only on its
 * own neighbours, so a run of centres is evaluated exactly as in the whole
 * system) holding at most min(edge_chunk or unlimited, max_chunk_edges)
 * edges each (AllegroInfo.max_chunk_edges; 32-bit workspace offsets).
 *   edges_per_centre  host [n_centres] neighbour count of each centre
 *   max_bounds        capacity of `bounds`
 *   bounds            host, receives n_chunks + 1 ascending boundaries,
 *                     bounds[0] = 0 and bounds[n_chunks] = n_centres (may be
 *                     NULL to query the count)
 *   n_chunks          host, receives the number of chunks (may be NULL)
 * Returns ALLEGRO_E_INVAL when one centre has more edges than a chunk may
 * hold or `bounds` is too small.
 */
int allegro_plan_chunks(const AllegroConfig* cfg, int64_t n_centres, const int32_t* edges_per_centre,
                        int64_t max_bounds, int64_t* bounds, int64_t* n_chunks);

/*
 * allegro_create: build a model on the current HIP device.
 *   weights        host, n_weights floats in this order (row-major float32):
 *                  twobody.W0..Wk [fan_in][fan_out] (fan_in of W0 = 2 S + n_bessel:
 *                  one-hot(Z_i), one-hot(Z_j), radial basis);
 *                  embed0 [d][(l_max+1) n]  (column l*n + u);
 *                  per layer L: env [d][(l_max+1) n], alpha [l_max+1]^3 indexed
 *                  [l1][l2][l_out] (raw path weights; unused entries ignored),
 *                  mix [l_max+1][n][n] indexed [l][v][u], mlp.W0..Wk with
 *                  fan_in of W0 = d + n ([x, scalar tensor features]);
 *                  with three or more layers (both parities) alpha is
 *                  [2][l_max+1]^3 indexed [s1][l1][l2][l_out] (s1 = 0 for a
 *                  natural-parity input irrep (l1, (-1)^l1), 1 for the other
 *                  parity; the output parity follows) and mix is
 *                  [2 (l_max+1)][n][n] indexed [slot][v][u] (slot l for the
 *                  natural-parity irrep of order l, l_max + 1 + l for the other);
 *                  edge.W0 [d][h], edge.W1 [h][1].
 *   species_scale  host [n_species] sigma (NULL = 1)
 *   species_shift  host [n_species] mu (NULL = 0)
 *   out            receives the handle (NULL on failure)
 * The weights are copied; the caller may free them afterwards.
 */
int allegro_create(const AllegroConfig* cfg, const float* weights, int64_t n_weights,
                   const double* species_scale, const double* species_shift,
                   AllegroModel** out);

/*
 * allegro_neighbors: build the ordered neighbour list of the n_local centres
 * (every (i, j, s) with |x_j - x_i + s L| < r_c, i != j or s != 0; section
 * "Allegro: Scalable Equivariant Deep Learning").  The distance test is
 *   dx = (x_j - x_i) + s_x L_x (per axis, IEEE double, no fused operations),
 *   d2 = (dx dx + dy dy) + dz dz, kept iff d2 < r_c * r_c,
 * and each centre's neighbours are sorted by (j, s_x, s_y, s_z), so the list is
 * reproducible bit for bit.
 *   pos      dev [n_total][3] double (any coordinates; periodic axes need not
 *            be wrapped, within 500 box lengths of the box)
 *   species  dev [n_total] int32 in [0, n_species)
 *   cell     host [9] double, row vectors; must be diagonal (orthorhombic);
 *            entries of non-periodic axes are ignored
 *   pbc      host [3] int32, 1 = periodic axis
 *   n_edges  host, receives the edge count (may be NULL)
 * Synchronises `stream` (the edge count sizes the list).  The list stays valid
 * for allegro_energy_forces until the next call.
 */
int allegro_neighbors(AllegroModel* m, int64_t n_local, int64_t n_total, const double* pos,
                      const int32_t* species, const double* cell, const int32_t* pbc,
                      void* stream, int64_t* n_edges);

/*
 * allegro_neighbors_batched: neighbour list of many independent, non-periodic
 * systems evaluated together (every atom is a centre; pairs never cross
 * systems).  System k holds atoms [atom_offsets[k], atom_offsets[k+1]).
 *   atom_offsets  host [n_systems+1], ascending, atom_offsets[0] = 0
 *   pos, species  dev arrays over all atom_offsets[n_systems] atoms
 * Same distance test, ordering and synchronisation as allegro_neighbors.
 */
int allegro_neighbors_batched(AllegroModel* m, int32_t n_systems, const int64_t* atom_offsets,
                              const double* pos, const int32_t* species, void* stream,
                              int64_t* n_edges);

/*
 * allegro_system_energies: per-system totals (FP64) of per-atom energies after a
 * batched evaluation.
 *   atom_energy    dev [n_atoms] from allegro_energy_forces
 *   system_energy  dev [n_systems]
 */
int allegro_system_energies(AllegroModel* m, const double* atom_energy, double* system_energy,
                            void* stream);

/*
 * allegro_energy_forces: evaluate the network on the current neighbour list.
 *   pos, species  the arrays given to allegro_neighbors (same n_total)
 *   atom_energy   dev [n_local] double: sigma_Z E_i + mu_Z (may be NULL)
 *   forces        dev [n_total][3] double, overwritten; ghost rows hold the
 *                 forces on the ghost copies (fold them onto their owners)
 *   virial        dev [9] double, W = -sum_e r_e (x) dE/dr_e (may be NULL)
 *   atom_virial   dev [n_total][9] double, half of each edge term to each end
 *                 (may be NULL)
 *   energy        dev [1] double, total energy (may be NULL)
 * Energy reduction and virial are accumulated in FP64; everything else runs in
 * the model's precision.  Does not synchronise.
 */
int allegro_energy_forces(AllegroModel* m, const double* pos, const int32_t* species,
                          double* atom_energy, double* forces, double* virial,
                          double* atom_virial, double* energy, void* stream);

/* Size of the static workspace of allegro_energy_forces_noalloc (bytes, one
 * array per GPU the library runs on, held until the process ends). */
#define ALLEGRO_NOALLOC_SCRATCH_BYTES (256u << 20)

/*
 * allegro_energy_forces_noalloc: allegro_energy_forces for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, kernels and results; its
 * per-evaluation workspace (activations, gradients, per-edge dE/dr, partial
 * sums) lives in a static device array of ALLEGRO_NOALLOC_SCRATCH_BYTES per GPU
 * instead of the model's workspace, and it calls no allocator of any kind and
 * records no per-kernel timing.  The neighbour list must come from an earlier
 * allegro_neighbors call (which allocates) on the current device.
 *   Returns ALLEGRO_E_INVAL, with the required size in allegro_last_error,
 *   when the list's largest chunk needs more workspace than the static array
 *   holds (build the list with a smaller edge_chunk: whole centre segments are
 *   evaluated a chunk at a time, so any system fits with a small enough
 *   chunk); ALLEGRO_E_STATE without a neighbour list.
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * contents (no kernel expects it cleared): calls that overlap in time on one
 * GPU (two streams, two threads, two models) race and must be serialised by
 * the caller.  Does not synchronise.
 */
int allegro_energy_forces_noalloc(AllegroModel* m, const double* pos, const int32_t* species,
                                  double* atom_energy, double* forces, double* virial,
                                  double* atom_virial, double* energy, void* stream);

/*
 * allegro_autotune: time the candidate edge-tile shapes of the edge-batched
 * kernels (MLP chains: 128, 64 or 32 edges per tile in BF16, 32 or 16 in
 * FP32; tensor product / mixing: 32 or 16 edges) on the current neighbour list
 * and keep the fastest for each kernel kind.  Runs allegro_energy_forces three
 * times per candidate on internal buffers and synchronises the stream.
 *   choices  host [8] int32 receiving the chosen tiles, in the order
 *            mlp_fwd_twobody, mlp_fwd_latent, mlp_fwd_final, mlp_bwd_final,
 *            mlp_bwd_latent, mlp_bwd_twobody, tp_mix, mix_adjoint (may be NULL)
 */
int allegro_autotune(AllegroModel* m, const double* pos, const int32_t* species, void* stream,
                     int32_t* choices);

/*
 * allegro_set_tiles: set the edge-tile shapes directly (same order and values
 * as allegro_autotune's choices; 0 = the library's default: the largest
 * 64/32-edge (BF16) or 32/16-edge (FP32) MLP tile that fits in LDS, 32-edge
 * tensor tiles).  Host array of 8 int32, copied.  Returns ALLEGRO_E_INVAL for a value not available in the
 * model's precision.
 */
int allegro_set_tiles(AllegroModel* m, const int32_t* tiles);

/*
 * allegro_set_ghosts: declare ghosts as periodic images of local atoms, for
 * allegro_md_run: ghost g (atom n_local + g) sits at pos[owner[g]] + offset[g],
 * and its force is added to its owner's.  Pass n_ghost = 0 to clear.
 *   owner   host [n_ghost] int32 in [0, n_local)
 *   offset  host [n_ghost][3] double (A)
 */
int allegro_set_ghosts(AllegroModel* m, int64_t n_local, int64_t n_ghost, const int32_t* owner,
                       const double* offset);

/*
 * allegro_md_run: n_steps of FP64 velocity Verlet (section "Problem overview":
 * MD needs forces every step).  Per step: v += dt/2 F/m; x += dt v; ghosts
 * follow their owners; the neighbour list is rebuilt when some centre has
 * moved more than half the neighbor_skin since the last build; F = -dE/dx;
 * ghost forces fold onto owners; v += dt/2 F/m.
 * Lists that fit one evaluation chunk are rebuilt on the device, inside the
 * step (section "Optimized LAMMPS-Kokkos implementation": preprocessing on the
 * device into fixed-shape buffers): the list buffers keep their edge capacity
 * (edge_capacity_hint), the cell grid of the last allegro_neighbors call is
 * reused, and with use_graph one captured step (rebuild included) is replayed
 * n_steps times with no host round trip.  Larger lists are rebuilt by the host
 * between eager steps (use_graph is then ignored).
 *   n_steps      steps to run (>= 0); dt_fs the time step in fs
 *   masses       dev [n_local] double, amu
 *   pos, vel     dev [n_total][3] / [n_local][3] double, A and A/fs, updated
 *   forces       dev [n_total][3] double: on entry the (folded) forces at pos
 *                (or pass init_forces = 1 to compute them first); on exit the
 *                forces at the final positions
 *   species      dev [n_total] int32
 *   thermo       dev [2 n_steps] double or NULL: per step (E_pot, E_kin) in eV
 *   virial       dev [9 n_steps] double or NULL: per step the virial
 *                W = -sum_e r_e (x) dE/dr_e (row-major 3x3, eV) at that step's
 *                positions, in FP64 as allegro_energy_forces reports it
 *   use_graph    1 = run the steps as replays of one captured HIP graph
 *   max_disp     host, receives the largest centre displacement since the
 *                last neighbour build (may be NULL)
 *   steps_done   host, receives the number of completed steps (may be NULL)
 * Returns ALLEGRO_E_CAPACITY when a device-side rebuild needed more edges than
 * the capacity: pos, vel and forces then hold the state after *steps_done
 * steps, the capacity has been regrown and the list rebuilt there, and
 * calling again for the remaining steps continues the same trajectory (thermo
 * and virial rows from step *steps_done on are not valid).  Synchronises the stream at
 * the end and returns ALLEGRO_E_NONFINITE (as allegro_check) when a step
 * produced non-finite forces or energies.
 */
int allegro_md_run(AllegroModel* m, int32_t n_steps, double dt_fs, const double* masses, double* pos,
                   double* vel, double* forces, const int32_t* species, double* thermo, double* virial,
                   int32_t init_forces, int32_t use_graph, void* stream, double* max_disp,
                   int32_t* steps_done);

/*
 * allegro_md_stats: MD step graphs captured so far by allegro_md_run, the
 * neighbour list's edge capacity, whether its rebuilds run on the device (1)
 * or on the host (0), and how many of the last allegro_md_run call's
 * completed steps rebuilt the list (device rebuilds only; host rebuilds are
 * counted too when they run).  Host outputs, each may be NULL.
 */
int allegro_md_stats(const AllegroModel* m, int64_t* graph_captures, int64_t* edge_capacity,
                     int32_t* device_rebuild, int64_t* last_run_rebuilds);

/*
 * allegro_check: synchronise `stream` and report what the device recorded
 * since the last check (allegro_energy_forces itself does not synchronise).
 * Returns ALLEGRO_E_NONFINITE when an evaluation produced a non-finite atom
 * energy or force (e.g. two atoms at the same position: the pair direction is
 * undefined), else ALLEGRO_OK; the record is cleared either way.  Forces are
 * F = -dE/dx of a smooth energy (section "Problem overview"), so a non-finite
 * value means the input left the potential's domain.
 */
int allegro_check(AllegroModel* m, void* stream);

/*
 * allegro_copy_edges: copy the current neighbour list to caller buffers.
 *   centre    dev [E] int32 (i), neighbor dev [E] int32 (j),
 *   shift     dev [E][3] int32 (s); any of them may be NULL.
 */
int allegro_copy_edges(AllegroModel* m, int32_t* centre, int32_t* neighbor, int32_t* shift,
                       void* stream);

/* allegro_num_edges: edge count of the current neighbour list (host value). */
int64_t allegro_num_edges(const AllegroModel* m);

/*
 * allegro_set_timing: enable (1) or disable (0) per-kernel timing of
 * allegro_energy_forces and reset the accumulated times.  When enabled, every
 * kernel launch is bracketed by a pair of HIP events recorded on the caller's
 * stream (a small overhead; for measurement runs only).
 */
int allegro_set_timing(AllegroModel* m, int32_t enable);

/*
 * allegro_kernel_times: accumulated event times per kernel kind since the last
 * allegro_set_timing.  Synchronises the recorded events.
 *   max_entries  capacity of the output arrays
 *   names        host [max_entries][48] NUL-terminated kernel kind names (may be NULL)
 *   total_ms     host [max_entries] summed duration in milliseconds (may be NULL)
 *   launches     host [max_entries] number of timed launches (may be NULL)
 *   n_entries    host, number of kernel kinds recorded (may exceed max_entries)
 */
int allegro_kernel_times(AllegroModel* m, int32_t max_entries, char* names, double* total_ms,
                         int64_t* launches, int32_t* n_entries);

/* allegro_workspace_bytes: device bytes currently held by the model. */
int64_t allegro_workspace_bytes(const AllegroModel* m);

/* allegro_destroy: free the model (NULL is ignored). */
void allegro_destroy(AllegroModel* m);

/* allegro_last_error: message of the last failure of `m` (or of a failed
 * create when m is NULL); never NULL. */
const char* allegro_last_error(const AllegroModel* m);

/* allegro_status_string: name of a status code. */
const char* allegro_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* ALLEGRO_MI355X_H */
