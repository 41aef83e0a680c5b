// coupling.h - tensor-product paths and the sparsity pattern of the fused
// coupling table, evaluated at compile time so that kernels can unroll the
// contraction over its non-zeros only.
//
// Paths (section "Optimized tensor product"): (l1, p1) x (l2, p2) -> (l_out,
// p_out) with |l1 - l2| <= l_out <= l1 + l2 and p_out = p1 p2; paths that cannot
// reach the final scalar outputs are dropped.  With at most two layers every
// kept irrep has natural parity (-1)^l, so the coupling of a path is the real
// Gaunt integral (1/4pi) \int Y_a Y_b Y_c dOmega, which is non-zero only when
// l1 + l2 + l_out is even.  The last layer keeps only l_out = 0 (so l1 = l2 and
// the coupling is diagonal in m).
//
// Strided components: c = l^2 + (m + l), l = 0..l_max, m = -l..l.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

namespace allegro {

// Real spherical harmonics (component normalisation, sum_m Y_lm^2 = 2l + 1) as
// polynomials in the unit-vector components (x, y, z):
//   Y_0 = 1; Y_1 = sqrt3 (y, z, x);
//   Y_2 = (sqrt15 xy, sqrt15 yz, sqrt5/2 (3 z^2 - 1), sqrt15 xz, sqrt15/2 (x^2 - y^2)).
struct Mono { double c; int i, j, k; };
struct Poly { int n; Mono t[3]; };

constexpr double kSqrt3 = 1.7320508075688772;
constexpr double kSqrt5 = 2.23606797749979;
constexpr double kSqrt15 = 3.872983346207417;

constexpr Poly sh_poly(int comp) {
  switch (comp) {
    case 0: return Poly{1, {{1.0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}}};
    case 1: return Poly{1, {{kSqrt3, 0, 1, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}}};
    case 2: return Poly{1, {{kSqrt3, 0, 0, 1}, {0, 0, 0, 0}, {0, 0, 0, 0}}};
    case 3: return Poly{1, {{kSqrt3, 1, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}}};
    case 4: return Poly{1, {{kSqrt15, 1, 1, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}}};
    case 5: return Poly{1, {{kSqrt15, 0, 1, 1}, {0, 0, 0, 0}, {0, 0, 0, 0}}};
    case 6: return Poly{2, {{1.5 * kSqrt5, 0, 0, 2}, {-0.5 * kSqrt5, 0, 0, 0}, {0, 0, 0, 0}}};
    case 7: return Poly{1, {{kSqrt15, 1, 0, 1}, {0, 0, 0, 0}, {0, 0, 0, 0}}};
    default: return Poly{2, {{0.5 * kSqrt15, 2, 0, 0}, {-0.5 * kSqrt15, 0, 2, 0}, {0, 0, 0, 0}}};
  }
}

constexpr int l_of(int comp) { return comp == 0 ? 0 : (comp < 4 ? 1 : 2); }

constexpr double dfact(int n) {  // n!! with (-1)!! = 1
  double r = 1.0;
  for (int v = n; v > 1; v -= 2) r *= v;
  return r;
}

// Mean of x^i y^j z^k over the unit sphere.
constexpr double sphere_mean(int i, int j, int k) {
  if ((i | j | k) & 1) return 0.0;
  return dfact(i - 1) * dfact(j - 1) * dfact(k - 1) / dfact(i + j + k + 1);
}

// Unnormalised real Gaunt coefficient of strided components (a, b, c).
constexpr double gaunt_raw(int a, int b, int c) {
  const Poly pa = sh_poly(a), pb = sh_poly(b), pc = sh_poly(c);
  double s = 0.0;
  for (int x = 0; x < pa.n; ++x)
    for (int y = 0; y < pb.n; ++y)
      for (int z = 0; z < pc.n; ++z)
        s += pa.t[x].c * pb.t[y].c * pc.t[z].c *
             sphere_mean(pa.t[x].i + pb.t[y].i + pc.t[z].i, pa.t[x].j + pb.t[y].j + pc.t[z].j,
                         pa.t[x].k + pb.t[y].k + pc.t[z].k);
  return s;
}

constexpr bool path_kept(int l1, int l2, int lo, int l_max, bool final_layer) {
  if (l1 > l_max || l2 > l_max || lo > l_max) return false;
  if (final_layer && lo != 0) return false;
  const int lo_min = l1 > l2 ? l1 - l2 : l2 - l1;
  return lo >= lo_min && lo <= l1 + l2 && ((l1 + l2 + lo) & 1) == 0;
}

constexpr double abs_c(double v) { return v < 0 ? -v : v; }

struct TpEntry { int a, b, c; };
struct TpList { int n; TpEntry e[729]; };

// Non-zeros of the fused table W[a, b, c] in a fixed order (a, b, c ascending).
constexpr TpList tp_list(int l_max, bool final_layer) {
  TpList L{};
  const int dim = (l_max + 1) * (l_max + 1);
  const int dout = final_layer ? 1 : dim;
  for (int a = 0; a < dim; ++a)
    for (int b = 0; b < dim; ++b)
      for (int c = 0; c < dout; ++c)
        if (path_kept(l_of(a), l_of(b), l_of(c), l_max, final_layer) &&
            abs_c(gaunt_raw(a, b, c)) > 1e-12) {
          L.e[L.n] = TpEntry{a, b, c};
          ++L.n;
        }
  return L;
}

template <int LMAX, bool FINAL>
struct TpPattern {
  static constexpr int DIM = (LMAX + 1) * (LMAX + 1);
  static constexpr int DOUT = FINAL ? 1 : DIM;
  static constexpr TpList list = tp_list(LMAX, FINAL);
  static constexpr int NNZ = list.n;
};

// T[c] += w_k V[a] G[b] over the non-zeros k of the pattern.
template <class Pat, std::size_t... K>
__device__ __forceinline__ void tp_forward(const float* V, const float* G, float* T, const float* w,
                                           std::index_sequence<K...>) {
  ((T[Pat::list.e[K].c] = fmaf(w[K] * V[Pat::list.e[K].a], G[Pat::list.e[K].b], T[Pat::list.e[K].c])), ...);
}

// gV[a] += w_k G[b] gT[c]   (adjoint with respect to the edge features)
template <class Pat, std::size_t... K>
__device__ __forceinline__ void tp_adjoint_v(const float* G, const float* gT, float* gV, const float* w,
                                             std::index_sequence<K...>) {
  ((gV[Pat::list.e[K].a] = fmaf(w[K] * G[Pat::list.e[K].b], gT[Pat::list.e[K].c], gV[Pat::list.e[K].a])), ...);
}

// gG[b] += w_k V[a] gT[c]   (adjoint with respect to the environment sum)
template <class Pat, std::size_t... K>
__device__ __forceinline__ void tp_adjoint_g(const float* V, const float* gT, float* gG, const float* w,
                                             std::index_sequence<K...>) {
  ((gG[Pat::list.e[K].b] = fmaf(w[K] * V[Pat::list.e[K].a], gT[Pat::list.e[K].c], gG[Pat::list.e[K].b])), ...);
}

}  // namespace allegro
