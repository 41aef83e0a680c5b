// edge.hip - per-edge basis and its adjoint, per-atom energies, forces and the
// virial.
//
// Edge basis (section "Training details": 8 Bessel functions times a
// polynomial cutoff envelope; section "Allegro: Scalable Equivariant Deep
// Learning": spherical harmonics of the edge direction, full O(3)).  Forms:
//   u(t) = 1 - (p+1)(p+2)/2 t^p + p(p+2) t^(p+1) - p(p+1)/2 t^(p+2),  t = d / r_c
//   R_n  = sqrt(2/r_c) sin(n pi d / r_c) / d * u,   n = 1..n_bessel
//   Y    = real harmonics with sum_m Y_lm^2 = 2l+1:
//          1;  sqrt3 (y, z, x);  sqrt15 xy, sqrt15 yz, sqrt5/2 (3z^2-1), sqrt15 xz, sqrt15/2 (x^2-y^2);
//          sqrt70/4 y(3x^2-y^2), sqrt105 xyz, sqrt42/4 y(5z^2-1), sqrt7/2 z(5z^2-3),
//          sqrt42/4 x(5z^2-1), sqrt105/2 z(x^2-y^2), sqrt70/4 x(x^2-3y^2)
// The edge vector r = (x_j - x_i) + s L is formed in FP64 and then rounded to
// FP32; the basis is FP32.
//
// Energies (section "Allegro: Scalable Equivariant Deep Learning", first
// equation; section "Mixed-precision calculations": shifting, scaling and
// summation of atomic energies in double precision): E_i is the FP32 sum of
// its pair energies, A_i = sigma_Z E_i + mu_Z and E = sum A_i in FP64.
//
// Forces from edge gradients g_e = dE/dr_e:  F_k = sum_{e from k} g_e -
// sum_{e to k} g_e, gathered per atom through the CSR and the reverse CSR (no
// atomics, so results are bit-reproducible); virial W = -sum_e r_e (x) g_e in
// FP64 with half of each edge term assigned to each end.
#include "devutil.h"
#include "internal.h"

namespace allegro {

namespace {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kS3 = 1.7320508075688772f;
constexpr float kS5 = 2.23606797749979f;
constexpr float kS15 = 3.872983346207417f;
constexpr float kS7 = 2.6457513110645907f;
constexpr float kS42 = 6.48074069840786f;
constexpr float kS70 = 8.366600265340756f;
constexpr float kS105 = 10.246950765959598f;

__device__ __forceinline__ void sh9(float x, float y, float z, float* Y) {
  Y[0] = 1.0f;
  Y[1] = kS3 * y; Y[2] = kS3 * z; Y[3] = kS3 * x;
  Y[4] = kS15 * x * y; Y[5] = kS15 * y * z; Y[6] = 0.5f * kS5 * (3.0f * z * z - 1.0f);
  Y[7] = kS15 * x * z; Y[8] = 0.5f * kS15 * (x * x - y * y);
}

__device__ __forceinline__ void sh3(float x, float y, float z, float* Y) {
  const float zz = 5.0f * z * z;
  Y[0] = 0.25f * kS70 * y * (3.0f * x * x - y * y);
  Y[1] = kS105 * x * y * z;
  Y[2] = 0.25f * kS42 * y * (zz - 1.0f);
  Y[3] = 0.5f * kS7 * z * (zz - 3.0f);
  Y[4] = 0.25f * kS42 * x * (zz - 1.0f);
  Y[5] = 0.5f * kS105 * z * (x * x - y * y);
  Y[6] = 0.25f * kS70 * x * (x * x - 3.0f * y * y);
}

__device__ __forceinline__ float ipow(float t, int p) {
  float r = 1.0f;
  for (int k = 0; k < p; ++k) r *= t;
  return r;
}

// ZBL universal screened Coulomb repulsion (the paper's stabilising pair
// term, section "Training details"): E(d) = k_e Z_i Z_j / d * phi(d / a_s),
// a_s = 0.46850 A / (Z_i^0.23 + Z_j^0.23), phi a sum of four exponentials
// with phi(0) = 1.  Returns E and dE/dd.
constexpr float kZblKe = 14.399645f;
__device__ __forceinline__ void zbl_pair(const float* zbl, int S, int zi, int zj, float d, float* E, float* dE) {
  const float zz = zbl[zi] * zbl[zj];
  const float as = 0.46850f / (zbl[S + zi] + zbl[S + zj]);
  const float x = d / as;
  const float c[4] = {0.18175f, 0.50986f, 0.28022f, 0.02817f};
  const float k[4] = {3.19980f, 0.94229f, 0.40290f, 0.20162f};
  float phi = 0.0f, dphi = 0.0f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float ex = c[q] * expf(-k[q] * x);
    phi += ex;
    dphi -= k[q] * ex;
  }
  const float pre = kZblKe * zz / d;
  *E = pre * phi;
  *dE = pre * (dphi / as - phi / d);
}

__device__ __forceinline__ void edge_vector(const EdgeArgs& a, int64_t e, double* r) {
  const int i = a.ei[e], j = a.ej[e];
  for (int ax = 0; ax < 3; ++ax)
    r[ax] = (a.pos[3 * j + ax] - a.pos[3 * i + ax]) + (double)a.es[3 * e + ax] * a.L[ax];
}

__global__ __launch_bounds__(256) void k_edge_basis(EdgeArgs a) {
  const int E = live_edges(a);
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= E) return;
  double r[3];
  edge_vector(a, e, r);
  const double dd = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  const float d = (float)dd;
  const float x = (float)(r[0] / dd), y = (float)(r[1] / dd), z = (float)(r[2] / dd);
  // species of the ordered pair (clamped into the table) and its cutoff
  const int S = a.n_species;
  const int zi = min(max(a.species[a.ei[e]], 0), S - 1), zj = min(max(a.species[a.ej[e]], 0), S - 1);
  const float rc = a.rc_pair ? a.rc_pair[zi * S + zj] : (float)a.r_cut;
  const float t = d / rc;
  const int p = a.p;
  const float tp = ipow(t, p);
  // zero beyond the cutoff, so that list entries in a neighbour skin contribute nothing
  const float u = t < 1.0f ? 1.0f - 0.5f * (p + 1) * (p + 2) * tp + (float)(p * (p + 2)) * tp * t -
                                 0.5f * p * (p + 1) * tp * t * t
                           : 0.0f;
  float* o = a.eb + e * kEB;
  float Y[9];
  sh9(x, y, z, Y);
  const int dim = (a.l_max + 1) * (a.l_max + 1);
  for (int c = 0; c < 9; ++c) o[c] = c < dim ? Y[c] : 0.0f;
  if (a.l_max >= 3) {
    float Y3[7];
    sh3(x, y, z, Y3);
    for (int c = 0; c < 7; ++c) o[eb_y(9 + c)] = Y3[c];
  }
  o[kEB_U] = u;
  o[kEB_D] = d;
  o[kEB_RHAT] = x; o[kEB_RHAT + 1] = y; o[kEB_RHAT + 2] = z;
  o[kEB_ZI] = (float)zi;
  o[kEB_ZJ] = (float)zj;
  if (a.zbl) {   // half of the pair's repulsion per ordered edge, under the edge's envelope
    float Ez, dEz;
    zbl_pair(a.zbl, S, zi, zj, d, &Ez, &dEz);
    a.e_pair[e] = 0.5f * Ez * u;
  }
  const float pref = sqrtf(2.0f / rc);
  const int nr = a.l_max >= 3 ? kEB_Y3 - kEB_R : 16;   // radial slots of the record
  for (int k = 0; k < nr; ++k) {
    float v = 0.0f;
    if (k < a.n_bessel) v = pref * sinf((float)(k + 1) * kPi * d / rc) / d * u;
    o[kEB_R + k] = v;
  }
}

__global__ __launch_bounds__(256) void k_edge_adjoint(EdgeArgs a) {
  const int E = live_edges(a);
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= E) return;
  const float* o = a.eb + e * kEB;
  const float d = o[kEB_D], u = o[kEB_U];
  const float x = o[kEB_RHAT], y = o[kEB_RHAT + 1], z = o[kEB_RHAT + 2];
  const float rc = a.rc_pair ? a.rc_pair[(int)o[kEB_ZI] * a.n_species + (int)o[kEB_ZJ]] : (float)a.r_cut;
  const float t = d / rc;
  const int p = a.p;
  // du/dd = -(p(p+1)(p+2)/2) t^(p-1) (1-t)^2 / r_c
  const float omt = 1.0f - t;
  const float du = t < 1.0f ? -0.5f * (float)(p * (p + 1) * (p + 2)) * ipow(t, p - 1) * omt * omt / rc : 0.0f;
  const float pref = sqrtf(2.0f / rc);
  float gu = a.g_u[e];
  float gd = 0.0f;
  for (int k = 0; k < a.n_bessel; ++k) {
    const float w = (float)(k + 1) * kPi / rc;
    float sn, cs;
    sincosf(w * d, &sn, &cs);
    const float B = pref * sn / d;
    const float dB = pref * (w * cs / d - sn / (d * d));
    const float gR = a.g_R[e * a.n_bessel + k];
    gu += gR * B;
    gd += gR * dB * u;
  }
  gd += gu * du;
  if (a.zbl) {
    const int zi = (int)o[kEB_ZI], zj = (int)o[kEB_ZJ];
    float Ez, dEz;
    zbl_pair(a.zbl, a.n_species, zi, zj, d, &Ez, &dEz);
    gd += 0.5f * (dEz * u + Ez * du);
  }
  const float* gY = a.g_Y + e * gy_width(a.l_max);
  float gx = 0.0f, gy = 0.0f, gz = 0.0f;
  if (a.l_max >= 1) {
    gx += kS3 * gY[3]; gy += kS3 * gY[1]; gz += kS3 * gY[2];
  }
  if (a.l_max >= 2) {
    gx += kS15 * (y * gY[4] + z * gY[7] + x * gY[8]);
    gy += kS15 * (x * gY[4] + z * gY[5] - y * gY[8]);
    gz += kS15 * (y * gY[5] + x * gY[7]) + 3.0f * kS5 * z * gY[6];
  }
  if (a.l_max >= 3) {   // Cartesian gradients of the l = 3 forms above
    const float* g3 = gY + 9;
    const float zz = 5.0f * z * z;
    const float a70 = 0.25f * kS70, a42 = 0.25f * kS42, a7 = 0.5f * kS7;
    gx += a70 * 6.0f * x * y * g3[0] + kS105 * y * z * g3[1] + a42 * (zz - 1.0f) * g3[4] +
          kS105 * x * z * g3[5] + a70 * 3.0f * (x * x - y * y) * g3[6];
    gy += a70 * 3.0f * (x * x - y * y) * g3[0] + kS105 * x * z * g3[1] + a42 * (zz - 1.0f) * g3[2] -
          kS105 * y * z * g3[5] - a70 * 6.0f * x * y * g3[6];
    gz += kS105 * x * y * g3[1] + a42 * 10.0f * y * z * g3[2] + a7 * (15.0f * z * z - 3.0f) * g3[3] +
          a42 * 10.0f * x * z * g3[4] + 0.5f * kS105 * (x * x - y * y) * g3[5];
  }
  const float dot = gx * x + gy * y + gz * z;
  const float inv = 1.0f / d;
  float* g = a.g_e + 3 * e;
  g[0] = gd * x + (gx - dot * x) * inv;
  g[1] = gd * y + (gy - dot * y) * inv;
  g[2] = gd * z + (gz - dot * z) * inv;
}

__global__ __launch_bounds__(256) void k_atom_energy(ReduceArgs a) {
  const int lane = lane_id();
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= a.n_centres) return;
  float s = 0.0f, sp = 0.0f;
  for (int e = a.row_ptr[c] + lane; e < a.row_ptr[c + 1]; e += kWave) {
    s += a.eij[e];
    if (a.e_pair) sp += a.e_pair[e];
  }
  s = wave_sum(s);
  sp = wave_sum(sp);
  if (lane == 0) {
    const int g = a.centre_base + c;
    // validated by the neighbour build; clamped like the edge records' species
    const int z = min(max(a.species[g], 0), a.n_species - 1);
    // the pair term is added after the species scale and shift
    a.atom_energy[g] = a.scale[z] * (double)s + a.shift[z] + (double)sp;
  }
}

__global__ __launch_bounds__(256) void k_forces(ForceArgs a) {
  __shared__ double red[10][256];
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double av[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double en = 0.0;
  if (k < a.n_total) {
    float f[3] = {0.0f, 0.0f, 0.0f};
    auto add_edge = [&](int e, float sign) {
      const float* g = a.g_e + 3 * (int64_t)e;
      const int i = a.ei[e], j = a.ej[e];
      double r[3];
      for (int ax = 0; ax < 3; ++ax) {
        f[ax] += sign * g[ax];
        r[ax] = (a.pos[3 * j + ax] - a.pos[3 * i + ax]) + (double)a.es[3 * (int64_t)e + ax] * a.L[ax];
      }
      for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) av[3 * p + q] -= 0.5 * r[p] * (double)g[q];
    };
    if (k < a.n_local)
      for (int e = a.row_ptr[k]; e < a.row_ptr[k + 1]; ++e) add_edge(e, 1.0f);
    for (int q = a.rrow_ptr[k]; q < a.rrow_ptr[k + 1]; ++q) add_edge(a.redge[q], -1.0f);
    for (int ax = 0; ax < 3; ++ax) a.forces[3 * k + ax] = (double)f[ax];
    if (a.atom_virial)
      for (int q = 0; q < 9; ++q) a.atom_virial[9 * k + q] = av[q];
    if (k < a.n_local) en = a.atom_energy[k];
    // sticky report of non-finite outputs (read and cleared by the host)
    if (a.status && !(isfinite(f[0]) && isfinite(f[1]) && isfinite(f[2]) && isfinite(en)))
      atomicOr(a.status, kStatusNonFinite);
  }
  for (int q = 0; q < 9; ++q) red[q][threadIdx.x] = av[q];
  red[9][threadIdx.x] = en;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int q = 0; q < 10; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 10) a.partial[blockIdx.x * 10 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_final_sums(const double* __restrict__ part, int nb,
                                                    double* __restrict__ virial,
                                                    double* __restrict__ energy) {
  __shared__ double red[10][256];
  double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nb; b += 256)
    for (int q = 0; q < 10; ++q) acc[q] += part[b * 10 + q];
  for (int q = 0; q < 10; ++q) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int q = 0; q < 10; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 9 && virial) virial[threadIdx.x] = red[threadIdx.x][0];
  if (threadIdx.x == 9 && energy) *energy = red[9][0];
}

inline unsigned blocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_edge_basis(const EdgeArgs& a, hipStream_t s) {
  if (a.E <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_edge_basis, dim3(blocks(a.E, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_edge_adjoint(const EdgeArgs& a, hipStream_t s) {
  if (a.E <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_edge_adjoint, dim3(blocks(a.E, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_atom_energy(const ReduceArgs& a, hipStream_t s) {
  if (a.n_centres <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_atom_energy, dim3(blocks(a.n_centres, 4)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_forces(const ForceArgs& a, int* n_blocks, hipStream_t s) {
  const int nb = (int)blocks(a.n_total > 0 ? a.n_total : 1, 256);
  *n_blocks = nb;
  hipLaunchKernelGGL(k_forces, dim3(nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_final_sums(const double* partial, int n_blocks, double* virial, double* energy,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_final_sums, dim3(1), dim3(256), 0, s, partial, n_blocks, virial, energy);
  return hipGetLastError();
}

}  // namespace allegro
