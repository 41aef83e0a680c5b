// neighbors.hip - cell-list construction of the ordered neighbour list.
//
// The model sums over ordered neighbour pairs (i, j) inside the cutoff sphere
// of each centre i (section "Allegro: Scalable Equivariant Deep Learning"), so
// the list is a full list.  Building it on the device, from positions already
// resident there, follows section "Optimized LAMMPS-Kokkos implementation".
//
// Steps: bounding box (open axes) -> bin atoms into cells of side > r_c
// (counting sort) -> per centre, one wavefront scans the stencil of cells and
// counts hits -> exclusive scan (CSR row pointers) -> the same scan writes
// packed (j, shift) keys -> each centre's segment is sorted by rank, so the
// final order (j, s_x, s_y, s_z) does not depend on scheduling -> reverse CSR
// (edges grouped by neighbour j, ascending edge id) for the force gather.
//
// The distance test reproduces the FP64 definition exactly:
//   dx = (x_j - x_i) + s_x L_x,  d2 = (dx dx + dy dy) + dz dz,  keep d2 < r_c^2
// with explicitly rounded operations (no contraction into FMA).
#include "devutil.h"
#include "internal.h"

namespace allegro {

namespace {

constexpr int kShiftBias = 1024;  // shifts are stored in 11-bit fields

__device__ __forceinline__ unsigned long long pack_key(int j, int sx, int sy, int sz) {
  return ((unsigned long long)(unsigned)j << 33) |
         ((unsigned long long)(unsigned)(sx + kShiftBias) << 22) |
         ((unsigned long long)(unsigned)(sy + kShiftBias) << 11) |
         (unsigned long long)(unsigned)(sz + kShiftBias);
}

__device__ __forceinline__ int floor_div(int a, int b) {  // b > 0
  int q = a / b;
  return (a % b != 0 && (a < 0)) ? q - 1 : q;
}

__global__ void k_bbox(const double* __restrict__ pos, int64_t n, double* __restrict__ part) {
  __shared__ double red[6][256];
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < n;
       a += (int64_t)gridDim.x * blockDim.x) {
    for (int ax = 0; ax < 3; ++ax) {
      const double v = pos[3 * a + ax];
      mn[ax] = fmin(mn[ax], v);
      mx[ax] = fmax(mx[ax], v);
    }
  }
  for (int ax = 0; ax < 3; ++ax) { red[ax][threadIdx.x] = mn[ax]; red[3 + ax][threadIdx.x] = mx[ax]; }
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int ax = 0; ax < 3; ++ax) {
        red[ax][threadIdx.x] = fmin(red[ax][threadIdx.x], red[ax][threadIdx.x + s]);
        red[3 + ax][threadIdx.x] = fmax(red[3 + ax][threadIdx.x], red[3 + ax][threadIdx.x + s]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// Cell index and periodic image of every atom; counts atoms per cell.
__global__ void k_bin(NbrArgs a, int* __restrict__ err) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= a.n_total || (a.pred && !*a.pred)) return;
  int c[3];
  const int st = a.sys ? a.sys[t] : 0;
  for (int ax = 0; ax < 3; ++ax) {
    const double x = a.pos[3 * t + ax] + (a.sys ? a.sys_shift[3 * st + ax] : 0.0);
    int q = 0;
    double u;
    if (a.pbc[ax]) {
      const double fq = floor(x / a.L[ax]);
      u = x - fq * a.L[ax];
      if (!(fabs(fq) <= 500.0)) { atomicOr(err, 1); u = 0.0; q = 0; }
      else q = (int)fq;
      if (u < 0.0) u = 0.0;
    } else {
      u = x - a.lo[ax];
    }
    int ci = (int)floor(u / a.h[ax]);
    ci = ci < 0 ? 0 : (ci >= a.nc[ax] ? a.nc[ax] - 1 : ci);
    c[ax] = ci;
    a.img[3 * t + ax] = q;
  }
  if (!(isfinite(a.pos[3 * t]) && isfinite(a.pos[3 * t + 1]) && isfinite(a.pos[3 * t + 2])))
    atomicOr(err, 2);
  if (a.species[t] < 0 || a.species[t] >= a.n_species) atomicOr(err, 4);
  const int cell = (c[0] * a.nc[1] + c[1]) * a.nc[2] + c[2];
  a.cell_of[t] = cell;
  atomicAdd(&a.cell_count[cell], 1);
}

__global__ void k_fill_cells(NbrArgs a) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= a.n_total || (a.pred && !*a.pred)) return;
  const int cell = a.cell_of[t];
  const int slot = atomicAdd(&a.cell_cursor[cell], 1);
  a.cell_atoms[a.cell_start[cell] + slot] = (int32_t)t;
}

// One wavefront per centre walks the stencil of cells.  WRITE = false counts,
// WRITE = true stores packed keys at the centre's CSR offset.
template <bool WRITE>
__global__ __launch_bounds__(256) void k_scan_stencil(NbrArgs a) {
  const int lane = lane_id();
  const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= a.n_local || (a.pred && !*a.pred)) return;
  const double xi = a.pos[3 * i], yi = a.pos[3 * i + 1], zi = a.pos[3 * i + 2];
  // row of the centre's species in the ordered-pair radius table (species
  // are clamped: this pass may run before the host has seen their check)
  const int S = a.n_species;
  const int zc = min(max(a.species[i], 0), S - 1);
  const double* rc2_row = a.rc2_pair ? a.rc2_pair + zc * S : nullptr;
  const int ci = a.cell_of[i];
  const int cc[3] = {ci / (a.nc[1] * a.nc[2]), (ci / a.nc[2]) % a.nc[1], ci % a.nc[2]};
  const int qi[3] = {a.img[3 * i], a.img[3 * i + 1], a.img[3 * i + 2]};
  const int w[3] = {2 * a.R[0] + 1, 2 * a.R[1] + 1, 2 * a.R[2] + 1};
  const int nst = w[0] * w[1] * w[2];
  int hits = 0;
  int64_t out = WRITE ? a.row_ptr[i] : 0;
  // end of the centre's segment: a list clamped to its edge capacity may hold
  // fewer slots than candidates (its results are then discarded)
  const int64_t seg_end = WRITE ? a.row_ptr[i + 1] : 0;
  for (int sb = 0; sb < nst; sb += kWave) {
    const int sidx = sb + lane;
    int cnt = 0, start = 0, k0 = 0, k1 = 0, k2 = 0;
    if (sidx < nst) {
      const int o[3] = {sidx / (w[1] * w[2]) - a.R[0], (sidx / w[2]) % w[1] - a.R[1], sidx % w[2] - a.R[2]};
      int tcell[3], kk[3];
      bool ok = true;
      for (int ax = 0; ax < 3; ++ax) {
        const int tt = cc[ax] + o[ax];
        if (a.pbc[ax]) {
          kk[ax] = floor_div(tt, a.nc[ax]);
          tcell[ax] = tt - kk[ax] * a.nc[ax];
        } else {
          kk[ax] = 0;
          tcell[ax] = tt;
          ok = ok && tt >= 0 && tt < a.nc[ax];
        }
      }
      if (ok) {
        const int t = (tcell[0] * a.nc[1] + tcell[1]) * a.nc[2] + tcell[2];
        start = a.cell_start[t];
        cnt = a.cell_start[t + 1] - start;
        k0 = kk[0]; k1 = kk[1]; k2 = kk[2];
      }
    }
    const int incl = wave_incl_scan(cnt);
    const int excl = incl - cnt;
    const int total = __shfl(incl, kWave - 1, kWave);
    for (int fb = 0; fb < total; fb += kWave) {
      const int f = fb + lane;
      // stencil entry holding candidate f: first lane whose inclusive count exceeds f
      int lo = 0, hi = kWave - 1;
      for (int step = 0; step < 6; ++step) {
        const int mid = (lo + hi) >> 1;
        const int v = __shfl(incl, mid, kWave);
        if (v > f) hi = mid; else lo = mid + 1;
      }
      const int m = lo;
      const int st = __shfl(start, m, kWave);
      const int ex = __shfl(excl, m, kWave);
      const int m0 = __shfl(k0, m, kWave), m1 = __shfl(k1, m, kWave), m2 = __shfl(k2, m, kWave);
      bool hit = false;
      int j = 0, sx = 0, sy = 0, sz = 0;
      if (f < total) {
        j = a.cell_atoms[st + (f - ex)];
        const bool same_sys = a.sys == nullptr || a.sys[j] == a.sys[i];
        sx = a.pbc[0] ? m0 - a.img[3 * j] + qi[0] : 0;
        sy = a.pbc[1] ? m1 - a.img[3 * j + 1] + qi[1] : 0;
        sz = a.pbc[2] ? m2 - a.img[3 * j + 2] + qi[2] : 0;
        const double dx = __dadd_rn(__dsub_rn(a.pos[3 * j], xi), __dmul_rn((double)sx, a.L[0]));
        const double dy = __dadd_rn(__dsub_rn(a.pos[3 * j + 1], yi), __dmul_rn((double)sy, a.L[1]));
        const double dz = __dadd_rn(__dsub_rn(a.pos[3 * j + 2], zi), __dmul_rn((double)sz, a.L[2]));
        const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
        const double rc2 = rc2_row ? rc2_row[min(max(a.species[j], 0), S - 1)] : a.r_cut2;
        hit = same_sys && d2 < rc2 && !(j == i && sx == 0 && sy == 0 && sz == 0);
      }
      if (WRITE) {
        const unsigned long long mask = __ballot(hit);
        if (hit) {
          const int rank = __popcll(mask & ((1ull << lane) - 1ull));
          if (out + rank < seg_end) a.keys[out + rank] = pack_key(j, sx, sy, sz);
        }
        out += __popcll(mask);
      } else {
        hits += hit ? 1 : 0;
      }
    }
  }
  if (!WRITE) {
    hits = wave_sum_i(hits);
    if (lane == 0) a.count[i] = hits;
  }
}

// Rank sort of each centre's keys; writes (i, j, shift).
__global__ __launch_bounds__(256) void k_sort_segments(NbrArgs a) {
  const int lane = lane_id();
  const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= a.n_local || (a.pred && !*a.pred)) return;
  const int b = a.row_ptr[i], e = a.row_ptr[i + 1];
  for (int p = b + lane; p < e; p += kWave) {
    const unsigned long long kp = a.keys[p];
    int rank = 0;
    for (int q = b; q < e; ++q) rank += (a.keys[q] < kp) ? 1 : 0;
    const int dst = b + rank;
    a.ei[dst] = (int32_t)i;
    a.ej[dst] = (int32_t)(kp >> 33);
    a.es[3 * dst] = (int32_t)((kp >> 22) & 2047u) - kShiftBias;
    a.es[3 * dst + 1] = (int32_t)((kp >> 11) & 2047u) - kShiftBias;
    a.es[3 * dst + 2] = (int32_t)(kp & 2047u) - kShiftBias;
  }
}

// E: edges (or the capacity, with the live count in *e_dev); pred: run only
// when *pred != 0 (null: always).
__global__ void k_rcount(const int32_t* __restrict__ ej, int64_t E, const int32_t* __restrict__ e_dev,
                         const int32_t* __restrict__ pred, int32_t* __restrict__ rcount) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (pred && !*pred) return;
  if (e_dev && *e_dev < E) E = *e_dev;
  if (e < E) atomicAdd(&rcount[ej[e]], 1);
}

__global__ void k_rfill(const int32_t* __restrict__ ej, int64_t E, const int32_t* __restrict__ e_dev,
                        const int32_t* __restrict__ pred, const int32_t* __restrict__ rrow,
                        int32_t* __restrict__ rcursor, int32_t* __restrict__ unsorted) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (pred && !*pred) return;
  if (e_dev && *e_dev < E) E = *e_dev;
  if (e >= E) return;
  const int j = ej[e];
  const int slot = atomicAdd(&rcursor[j], 1);
  unsorted[rrow[j] + slot] = (int32_t)e;
}

__global__ __launch_bounds__(256) void k_rsort(const int32_t* __restrict__ rrow, int64_t n,
                                               const int32_t* __restrict__ unsorted,
                                               int32_t* __restrict__ redge, const int32_t* __restrict__ pred) {
  const int lane = lane_id();
  const int64_t a = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (a >= n || (pred && !*pred)) return;
  const int b = rrow[a], e = rrow[a + 1];
  for (int p = b + lane; p < e; p += kWave) {
    const int v = unsorted[p];
    int rank = 0;
    for (int q = b; q < e; ++q) rank += (unsorted[q] < v) ? 1 : 0;
    redge[b + rank] = v;
  }
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

// Exclusive scan, three passes over blocks of 1024 values.
constexpr int kScanBlock = 1024;

// pred (every kernel of the scan): run only when *pred != 0 (null: always);
// one value for the whole grid, so the early exits are block-uniform.
__global__ __launch_bounds__(1024) void k_scan_local(const int32_t* __restrict__ in, int64_t n,
                                                     int32_t* __restrict__ out,
                                                     int32_t* __restrict__ block_sum,
                                                     const int32_t* __restrict__ pred) {
  __shared__ int wsum[16];
  if (pred && !*pred) return;
  const int64_t t = blockIdx.x * (int64_t)kScanBlock + threadIdx.x;
  const int v = t < n ? in[t] : 0;
  const int incl = wave_incl_scan(v);
  const int w = threadIdx.x >> 6;
  if (lane_id() == kWave - 1) wsum[w] = incl;
  __syncthreads();
  int base = 0;
  for (int k = 0; k < w; ++k) base += wsum[k];
  if (t < n) out[t] = base + incl - v;
  if (threadIdx.x == kScanBlock - 1) block_sum[blockIdx.x] = base + incl;
}

__global__ __launch_bounds__(1024) void k_scan_blocks(int32_t* __restrict__ block_sum, int nb,
                                                      int32_t* __restrict__ total_out,
                                                      const int32_t* __restrict__ pred) {
  __shared__ int wsum[16];
  __shared__ int carry;
  if (pred && !*pred) return;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += kScanBlock) {
    const int t = base + threadIdx.x;
    const int v = t < nb ? block_sum[t] : 0;
    const int incl = wave_incl_scan(v);
    const int w = threadIdx.x >> 6;
    if (lane_id() == kWave - 1) wsum[w] = incl;
    __syncthreads();
    int off = carry;
    for (int k = 0; k < w; ++k) off += wsum[k];
    if (t < nb) block_sum[t] = off + incl - v;
    __syncthreads();
    if (threadIdx.x == kScanBlock - 1) carry = off + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total_out = carry;
}

__global__ void k_scan_add(int32_t* __restrict__ out, int64_t n, const int32_t* __restrict__ block_sum,
                           const int32_t* __restrict__ pred) {
  if (pred && !*pred) return;
  const int64_t t = blockIdx.x * (int64_t)kScanBlock + threadIdx.x;
  if (t < n) out[t] += block_sum[blockIdx.x];
}

// One block per system: min/max of its atoms' coordinates.
__global__ __launch_bounds__(256) void k_system_bbox(const double* __restrict__ pos,
                                                     const int64_t* __restrict__ off, double* __restrict__ out) {
  __shared__ double red[6][256];
  const int s = blockIdx.x;
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  for (int64_t a = off[s] + threadIdx.x; a < off[s + 1]; a += 256)
    for (int ax = 0; ax < 3; ++ax) {
      mn[ax] = fmin(mn[ax], pos[3 * a + ax]);
      mx[ax] = fmax(mx[ax], pos[3 * a + ax]);
    }
  for (int ax = 0; ax < 3; ++ax) { red[ax][threadIdx.x] = mn[ax]; red[3 + ax][threadIdx.x] = mx[ax]; }
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k)
      for (int ax = 0; ax < 3; ++ax) {
        red[ax][threadIdx.x] = fmin(red[ax][threadIdx.x], red[ax][threadIdx.x + k]);
        red[3 + ax][threadIdx.x] = fmax(red[3 + ax][threadIdx.x], red[3 + ax][threadIdx.x + k]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) out[6 * s + threadIdx.x] = red[threadIdx.x][0];
}

// One block per system: FP64 sum of a per-atom value (fixed tree order).
__global__ __launch_bounds__(256) void k_system_sums(const double* __restrict__ v,
                                                     const int64_t* __restrict__ off, double* __restrict__ out) {
  __shared__ double red[256];
  const int s = blockIdx.x;
  double acc = 0.0;
  for (int64_t a = off[s] + threadIdx.x; a < off[s + 1]; a += 256) acc += v[a];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[s] = red[0];
}

inline unsigned grid_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_system_bbox(const double* pos, const int64_t* offsets, int n_sys, double* out, hipStream_t s) {
  if (n_sys <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_system_bbox, dim3(n_sys), dim3(256), 0, s, pos, offsets, out);
  return hipGetLastError();
}

hipError_t launch_system_sums(const double* atom_value, const int64_t* offsets, int n_sys, double* out,
                              hipStream_t s) {
  if (n_sys <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_system_sums, dim3(n_sys), dim3(256), 0, s, atom_value, offsets, out);
  return hipGetLastError();
}

hipError_t launch_bbox(const NbrArgs& a, int* n_blocks, hipStream_t s) {
  int nb = (int)grid_for(a.n_total, 256);
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  *n_blocks = nb;
  hipLaunchKernelGGL(k_bbox, dim3(nb), dim3(256), 0, s, a.pos, a.n_total, a.bbox);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

size_t exclusive_scan_tmp_bytes(int64_t n) {
  return (size_t)(grid_for(n, kScanBlock) + 1) * sizeof(int32_t);
}

// out[0..n] = exclusive prefix sums of in[0..n), out[n] = total.
hipError_t launch_exclusive_scan(const int32_t* in, int32_t* out, int64_t n, void* tmp, hipStream_t s,
                                 const int32_t* pred) {
  if (n <= 0) return launch_fill_i32(out, 0, 1, s);
  const int nb = (int)grid_for(n, kScanBlock);
  int32_t* bs = (int32_t*)tmp;
  hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(kScanBlock), 0, s, in, n, out, bs, pred);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanBlock), 0, s, bs, nb, out + n, pred);
  hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kScanBlock), 0, s, out, n, (const int32_t*)bs, pred);
  return hipGetLastError();
}

hipError_t launch_bin_atoms_err(const NbrArgs& a, int* err, hipStream_t s) {
  hipLaunchKernelGGL(k_bin, dim3(grid_for(a.n_total, 256)), dim3(256), 0, s, a, err);
  return hipGetLastError();
}

hipError_t launch_fill_cells(const NbrArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_cells, dim3(grid_for(a.n_total, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_count_neighbors(const NbrArgs& a, hipStream_t s) {
  if (a.n_local <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan_stencil<false>, dim3(grid_for(a.n_local, 4)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fill_neighbors(const NbrArgs& a, hipStream_t s) {
  if (a.n_local <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan_stencil<true>, dim3(grid_for(a.n_local, 4)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sort_neighbors(const NbrArgs& a, hipStream_t s) {
  if (a.n_local <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sort_segments, dim3(grid_for(a.n_local, 4)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Reverse CSR: rcount/rcursor must be zeroed by the caller; `a.keys` is reused
// as scratch for the unsorted edge ids (E int32 fit in E uint64).
// With a.pred set (in-graph rebuild) E is the edge capacity and the live
// count is row_ptr[n_local].
hipError_t launch_reverse_csr(const NbrArgs& a, int64_t E, hipStream_t s) {
  const int32_t* e_dev = a.pred ? a.row_ptr + a.n_local : nullptr;
  if (E > 0)
    hipLaunchKernelGGL(k_rcount, dim3(grid_for(E, 256)), dim3(256), 0, s, a.ej, E, e_dev, a.pred, a.rcount);
  hipError_t st = launch_exclusive_scan(a.rcount, a.rrow_ptr, a.n_total, a.scan_tmp, s, a.pred);
  if (st != hipSuccess) return st;
  if (E <= 0) return hipGetLastError();
  int32_t* unsorted = (int32_t*)a.keys;
  hipLaunchKernelGGL(k_rfill, dim3(grid_for(E, 256)), dim3(256), 0, s, a.ej, E, e_dev, a.pred,
                     (const int32_t*)a.rrow_ptr, a.rcursor, unsorted);
  hipLaunchKernelGGL(k_rsort, dim3(grid_for(a.n_total, 4)), dim3(256), 0, s,
                     (const int32_t*)a.rrow_ptr, a.n_total, (const int32_t*)unsorted, a.redge, a.pred);
  return hipGetLastError();
}

}  // namespace allegro
