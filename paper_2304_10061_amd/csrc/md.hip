// md.hip - FP64 velocity Verlet for molecular dynamics on the device.
//
// The paper runs MD (section "Problem overview": forces every step; section
// "Measurement metrics": timesteps per second), integrated by the MD engine.
// Here one step is
//   v += dt/2 F/m;  x += dt v;  (ghost images follow their owners)
//   F = -dE/dx (energy/force path on the current neighbour list)
//   fold ghost forces onto owners;  v += dt/2 F/m
// with positions and velocities in FP64.  Units: A, fs, amu, eV;
// 1 eV/(A amu) = 1/103.642697 A/fs^2.
#include "devutil.h"
#include "internal.h"

namespace allegro {

namespace {

constexpr double kAcc = 1.0 / 103.642697;
constexpr double kKE = 103.642697;

__global__ void k_kick_drift(int64_t n, double dt, const double* __restrict__ m, double* __restrict__ x,
                             double* __restrict__ v, const double* __restrict__ f) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = 0.5 * dt * kAcc / m[i];
  for (int ax = 0; ax < 3; ++ax) {
    const double vv = v[3 * i + ax] + s * f[3 * i + ax];
    v[3 * i + ax] = vv;
    x[3 * i + ax] += dt * vv;
  }
}

__global__ void k_kick(int64_t n, double dt, const double* __restrict__ m, double* __restrict__ v,
                       const double* __restrict__ f) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = 0.5 * dt * kAcc / m[i];
  for (int ax = 0; ax < 3; ++ax) v[3 * i + ax] += s * f[3 * i + ax];
}

__global__ void k_ghost_refresh(int64_t n_ghost, int64_t n_local, const int32_t* __restrict__ owner,
                                const double* __restrict__ offset, double* __restrict__ x) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n_ghost) return;
  const int o = owner[g];
  for (int ax = 0; ax < 3; ++ax) x[3 * (n_local + g) + ax] = x[3 * o + ax] + offset[3 * g + ax];
}

// F[o] += sum of the forces on o's ghost images (CSR over owners, fixed order).
__global__ void k_fold(int64_t n_local, const int32_t* __restrict__ gptr, const int32_t* __restrict__ gidx,
                       double* __restrict__ f) {
  const int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (o >= n_local) return;
  for (int q = gptr[o]; q < gptr[o + 1]; ++q) {
    const int64_t g = n_local + gidx[q];
    for (int ax = 0; ax < 3; ++ax) f[3 * o + ax] += f[3 * g + ax];
  }
}

__global__ __launch_bounds__(256) void k_ke_partial(int64_t n, const double* __restrict__ m,
                                                    const double* __restrict__ v, double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double ke = 0.0;
  if (i < n) ke = m[i] * (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2]);
  red[threadIdx.x] = ke;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// rows[2 c] = potential energy, rows[2 c + 1] = kinetic energy, c = step
// counter; the destination lives in device memory so that a captured step
// does not depend on it.
__global__ __launch_bounds__(256) void k_thermo(const double* __restrict__ part, int nb,
                                                const double* __restrict__ epot, const double* __restrict__ vir,
                                                ThermoTarget* __restrict__ t) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) acc += part[b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t c = t->counter;
    if (t->rows && c < t->cap) {
      t->rows[2 * c] = *epot;
      t->rows[2 * c + 1] = 0.5 * kKE * red[0];
    }
    if (vir && t->vrows && c < t->cap)
      for (int k = 0; k < 9; ++k) t->vrows[9 * c + k] = vir[k];
    t->counter = c + 1;
  }
}

__global__ void k_set_thermo(ThermoTarget* t, double* rows, double* vrows, int64_t cap) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    t->rows = rows;
    t->vrows = vrows;
    t->cap = cap;
    t->counter = 0;
  }
}

__global__ __launch_bounds__(256) void k_max_disp(int64_t n, const double* __restrict__ x,
                                                  const double* __restrict__ x0, double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double d2 = 0.0;
  if (i < n)
    for (int ax = 0; ax < 3; ++ax) {
      const double dx = x[3 * i + ax] - x0[3 * i + ax];
      d2 += dx * dx;
    }
  red[threadIdx.x] = d2;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// In-graph neighbour rebuild (flags: kFlagRebuild, kFlagHalt, kFlagSteps).
// flags[kFlagRebuild] = 1 when some centre moved more than the half skin
// since the last build (r2 = (skin/2)^2) and the run has not halted; the
// caller clears it first.
__global__ void k_disp_check(int64_t n, const double* __restrict__ x, const double* __restrict__ x0, double r2,
                             int32_t* __restrict__ flags) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n || flags[kFlagHalt]) return;
  double d2 = 0.0;
  for (int ax = 0; ax < 3; ++ax) {
    const double dx = x[3 * i + ax] - x0[3 * i + ax];
    d2 += dx * dx;
  }
  if (!(d2 <= r2)) flags[kFlagRebuild] = 1;   // also for non-finite positions (the build reports them)
}

// dst[i] = src[i] for i < n when (flags[slot] != 0) == want.
__global__ void k_copy_f64_flag(double* __restrict__ dst, const double* __restrict__ src, int64_t n,
                                const int32_t* __restrict__ flags, int slot, int want) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n || (flags[slot] != 0) != (want != 0)) return;
  dst[i] = src[i];
}

// Edge capacity: when the rebuilt list holds more than `cap` edges, record
// it (sticky status bit, halt flag) ...
__global__ void k_cap_flag(const int32_t* __restrict__ row_ptr, int64_t n_local, int64_t cap,
                           int32_t* __restrict__ flags, int* __restrict__ status) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || !flags[kFlagRebuild]) return;
  if ((int64_t)row_ptr[n_local] > cap) {
    flags[kFlagHalt] = 1;
    flags[kFlagNeed] = row_ptr[n_local];
    atomicOr(status, kStatusCapacity);
  }
}
// ... and clamp the row pointers to it, so that every later kernel of the
// step stays inside the buffers (the run's results from here on are
// discarded).
__global__ void k_cap_clamp(int32_t* __restrict__ row_ptr, int64_t n_local, int64_t cap,
                            const int32_t* __restrict__ flags) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i > n_local || !flags[kFlagRebuild] || !flags[kFlagHalt]) return;
  if ((int64_t)row_ptr[i] > cap) row_ptr[i] = (int32_t)cap;
}

// One more completed step, and one more rebuild if it rebuilt the list (not
// counted after a halt).
__global__ void k_step_done(int32_t* __restrict__ flags) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && !flags[kFlagHalt]) {
    flags[kFlagSteps] += 1;
    flags[kFlagBuilds] += flags[kFlagRebuild];
  }
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_disp_check(int64_t n, const double* x, const double* x0, double r2, int32_t* flags,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_disp_check, dim3(blocks(n)), dim3(256), 0, s, n, x, x0, r2, flags);
  return hipGetLastError();
}

hipError_t launch_copy_f64_flag(double* dst, const double* src, int64_t n, const int32_t* flags, int slot, int want,
                                hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_f64_flag, dim3(blocks(n)), dim3(256), 0, s, dst, src, n, flags, slot, want);
  return hipGetLastError();
}

hipError_t launch_capacity_check(int32_t* row_ptr, int64_t n_local, int64_t cap, int32_t* flags, int* status,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_cap_flag, dim3(1), dim3(64), 0, s, (const int32_t*)row_ptr, n_local, cap, flags, status);
  hipLaunchKernelGGL(k_cap_clamp, dim3(blocks(n_local + 1)), dim3(256), 0, s, row_ptr, n_local, cap,
                     (const int32_t*)flags);
  return hipGetLastError();
}

hipError_t launch_step_done(int32_t* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_step_done, dim3(1), dim3(64), 0, s, flags);
  return hipGetLastError();
}

hipError_t launch_kick_drift(int64_t n, double dt, const double* m, double* x, double* v, const double* f,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kick_drift, dim3(blocks(n)), dim3(256), 0, s, n, dt, m, x, v, f);
  return hipGetLastError();
}

hipError_t launch_kick(int64_t n, double dt, const double* m, double* v, const double* f, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kick, dim3(blocks(n)), dim3(256), 0, s, n, dt, m, v, f);
  return hipGetLastError();
}

hipError_t launch_ghost_refresh(int64_t n_ghost, int64_t n_local, const int32_t* owner, const double* offset,
                                double* x, hipStream_t s) {
  if (n_ghost <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ghost_refresh, dim3(blocks(n_ghost)), dim3(256), 0, s, n_ghost, n_local, owner, offset, x);
  return hipGetLastError();
}

hipError_t launch_fold(int64_t n_local, const int32_t* gptr, const int32_t* gidx, double* f, hipStream_t s) {
  if (n_local <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fold, dim3(blocks(n_local)), dim3(256), 0, s, n_local, gptr, gidx, f);
  return hipGetLastError();
}

hipError_t launch_thermo(int64_t n, const double* m, const double* v, double* part, const double* epot,
                         const double* vir, ThermoTarget* target, hipStream_t s) {
  const int nb = (int)blocks(n > 0 ? n : 1);
  hipLaunchKernelGGL(k_ke_partial, dim3(nb), dim3(256), 0, s, n, m, v, part);
  hipLaunchKernelGGL(k_thermo, dim3(1), dim3(256), 0, s, (const double*)part, nb, epot, vir, target);
  return hipGetLastError();
}

hipError_t launch_set_thermo(ThermoTarget* target, double* rows, double* vrows, int64_t cap, hipStream_t s) {
  hipLaunchKernelGGL(k_set_thermo, dim3(1), dim3(64), 0, s, target, rows, vrows, cap);
  return hipGetLastError();
}

hipError_t launch_max_disp(int64_t n, const double* x, const double* x0, double* part, int* n_blocks,
                           hipStream_t s) {
  const int nb = (int)blocks(n > 0 ? n : 1);
  *n_blocks = nb;
  hipLaunchKernelGGL(k_max_disp, dim3(nb), dim3(256), 0, s, n, x, x0, part);
  return hipGetLastError();
}

}  // namespace allegro
