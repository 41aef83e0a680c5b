// coupling.h - tensor-product paths and the sparsity pattern of the fused
// coupling table, evaluated at compile time so that kernels can unroll the
// contraction over its non-zeros only.
//
// Irreps are (l, p), p the parity.  The harmonics Y_l carry natural parity
// (-1)^l.  Paths (section "Optimized tensor product"): (l1, p1) x (l2, p2) ->
// (l_out, p_out) with |l1 - l2| <= l_out <= l1 + l2 and p_out = p1 p2; paths
// that cannot reach the final scalar outputs are dropped.  The second operand
// is always a harmonic, so p2 = (-1)^l2.
//
// The invariant trilinear forms of three real irreps l1, l2, l3 span one
// dimension, so a path's coupling is fixed up to scale by (l1, l2, l3):
//   l1 + l2 + l3 even: the real Gaunt integral (1/4pi) \int Y_a Y_b Y_c dOmega;
//   l1 + l2 + l3 odd:  (1/4pi) \int rhat . (grad Y_a x grad Y_b) Y_c dOmega
//                      (the Gaunt integral vanishes; for 1 x 1 -> 1 this is
//                      the cross product),
// each path block rescaled to unit Frobenius norm.  Both are exact sphere
// means of polynomials: with every harmonic written as a homogeneous harmonic
// polynomial P of degree l, rhat . (grad P_a x grad P_b) on the unit sphere
// equals the triple product of the surface gradients (the radial parts of the
// full gradients are parallel to rhat and drop out).
//
// Strided components (section "Optimized tensor product"), D = (l_max+1)^2:
// c = l^2 + (m + l) holds natural-parity irrep (l, (-1)^l); c = D + l^2 + (m + l)
// holds unnatural-parity irrep (l, -(-1)^l).  A layer's operands are described
// by kinds: natural only (D components), both parities (2 D components, the
// unnatural l = 0 slot unused), or the scalar output of the last layer.  With
// at most four layers these kinds are exactly the pruned irrep sets: the
// unnatural scalar can first be produced by a second layer but is needed only
// by a layer that still keeps unnatural outputs two layers before the end.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

namespace allegro {

enum TpKind { kScalarOut = 0, kNatural = 1, kBothParities = 2 };

constexpr int kMaxLmax = 3;

// l of a natural-parity strided component c < 16.
constexpr int l_of(int comp) { return comp < 1 ? 0 : (comp < 4 ? 1 : (comp < 9 ? 2 : 3)); }

// Real spherical harmonics (component normalisation, sum_m Y_lm^2 = 2l + 1) as
// homogeneous harmonic polynomials in the unit-vector components (x, y, z):
//   Y_0 = 1; Y_1 = sqrt3 (y, z, x);
//   Y_2 = (sqrt15 xy, sqrt15 yz, sqrt5/2 (2z^2 - x^2 - y^2), sqrt15 xz, sqrt15/2 (x^2 - y^2));
//   Y_3 = (sqrt70/4 y(3x^2 - y^2), sqrt105 xyz, sqrt42/4 y(4z^2 - x^2 - y^2),
//          sqrt7/2 z(2z^2 - 3x^2 - 3y^2), sqrt42/4 x(4z^2 - x^2 - y^2),
//          sqrt105/2 z(x^2 - y^2), sqrt70/4 x(x^2 - 3y^2)).
struct Mono { double c; int i, j, k; };
struct Poly { int n; Mono t[3]; };

constexpr double kSqrt3 = 1.7320508075688772;
constexpr double kSqrt5 = 2.23606797749979;
constexpr double kSqrt7 = 2.6457513110645907;
constexpr double kSqrt15 = 3.872983346207417;
constexpr double kSqrt42 = 6.48074069840786;
constexpr double kSqrt70 = 8.366600265340756;
constexpr double kSqrt105 = 10.246950765959598;

constexpr Poly sh_poly(int comp) {
  switch (comp) {
    case 0: return Poly{1, {{1.0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}}};
    case 1: return Poly{1, {{kSqrt3, 0, 1, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}}};
    case 2: return Poly{1, {{kSqrt3, 0, 0, 1}, {0, 0, 0, 0}, {0, 0, 0, 0}}};
    case 3: return Poly{1, {{kSqrt3, 1, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}}};
    case 4: return Poly{1, {{kSqrt15, 1, 1, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}}};
    case 5: return Poly{1, {{kSqrt15, 0, 1, 1}, {0, 0, 0, 0}, {0, 0, 0, 0}}};
    case 6: return Poly{3, {{kSqrt5, 0, 0, 2}, {-0.5 * kSqrt5, 2, 0, 0}, {-0.5 * kSqrt5, 0, 2, 0}}};
    case 7: return Poly{1, {{kSqrt15, 1, 0, 1}, {0, 0, 0, 0}, {0, 0, 0, 0}}};
    case 8: return Poly{2, {{0.5 * kSqrt15, 2, 0, 0}, {-0.5 * kSqrt15, 0, 2, 0}, {0, 0, 0, 0}}};
    case 9: return Poly{2, {{0.75 * kSqrt70, 2, 1, 0}, {-0.25 * kSqrt70, 0, 3, 0}, {0, 0, 0, 0}}};
    case 10: return Poly{1, {{kSqrt105, 1, 1, 1}, {0, 0, 0, 0}, {0, 0, 0, 0}}};
    case 11: return Poly{3, {{kSqrt42, 0, 1, 2}, {-0.25 * kSqrt42, 2, 1, 0}, {-0.25 * kSqrt42, 0, 3, 0}}};
    case 12: return Poly{3, {{kSqrt7, 0, 0, 3}, {-1.5 * kSqrt7, 2, 0, 1}, {-1.5 * kSqrt7, 0, 2, 1}}};
    case 13: return Poly{3, {{kSqrt42, 1, 0, 2}, {-0.25 * kSqrt42, 3, 0, 0}, {-0.25 * kSqrt42, 1, 2, 0}}};
    case 14: return Poly{2, {{0.5 * kSqrt105, 2, 0, 1}, {-0.5 * kSqrt105, 0, 2, 1}, {0, 0, 0, 0}}};
    default: return Poly{2, {{0.25 * kSqrt70, 3, 0, 0}, {-0.75 * kSqrt70, 1, 2, 0}, {0, 0, 0, 0}}};
  }
}

// Means of x^i y^j z^k over the unit sphere: (i-1)!! (j-1)!! (k-1)!! / (i+j+k+1)!!
// for even i, j, k, else 0.
struct SphereMeans { double m[12][12][12]; };

constexpr SphereMeans make_sphere_means() {
  SphereMeans M{};
  for (int i = 0; i < 12; ++i)
    for (int j = 0; j < 12; ++j)
      for (int k = 0; k < 12; ++k) {
        if ((i | j | k) & 1) continue;
        double r = 1.0;
        for (int v = i - 1; v > 1; v -= 2) r *= v;
        for (int v = j - 1; v > 1; v -= 2) r *= v;
        for (int v = k - 1; v > 1; v -= 2) r *= v;
        for (int v = i + j + k + 1; v > 1; v -= 2) r /= v;
        M.m[i][j][k] = r;
      }
  return M;
}

inline constexpr SphereMeans kSphereMeans = make_sphere_means();

// Unnormalised real Gaunt coefficient of natural strided components (a, b, c).
constexpr double gaunt_raw(int a, int b, int c) {
  const Poly pa = sh_poly(a), pb = sh_poly(b), pc = sh_poly(c);
  double s = 0.0;
  for (int x = 0; x < pa.n; ++x)
    for (int y = 0; y < pb.n; ++y)
      for (int z = 0; z < pc.n; ++z)
        s += pa.t[x].c * pb.t[y].c * pc.t[z].c *
             kSphereMeans.m[pa.t[x].i + pb.t[y].i + pc.t[z].i][pa.t[x].j + pb.t[y].j + pc.t[z].j]
                           [pa.t[x].k + pb.t[y].k + pc.t[z].k];
  return s;
}

constexpr Poly deriv(const Poly& p, int ax) {
  Poly q{};
  for (int s = 0; s < p.n; ++s) {
    const int e = ax == 0 ? p.t[s].i : (ax == 1 ? p.t[s].j : p.t[s].k);
    if (e == 0) continue;
    Mono m = p.t[s];
    m.c *= e;
    if (ax == 0) --m.i;
    else if (ax == 1) --m.j;
    else --m.k;
    q.t[q.n] = m;
    ++q.n;
  }
  return q;
}

// Unnormalised triple-product form of natural strided components (a, b, c):
// the sphere mean of r . (grad P_a x grad P_b) P_c.
constexpr double triple_raw(int a, int b, int c) {
  const Poly pa = sh_poly(a), pb = sh_poly(b), pc = sh_poly(c);
  const Poly ga[3] = {deriv(pa, 0), deriv(pa, 1), deriv(pa, 2)};
  const Poly gb[3] = {deriv(pb, 0), deriv(pb, 1), deriv(pb, 2)};
  double s = 0.0;
  for (int x = 0; x < 3; ++x) {
    const int y = (x + 1) % 3, z = (x + 2) % 3;   // r_x (grad_y P_a grad_z P_b - grad_z P_a grad_y P_b)
    for (int sg = 0; sg < 2; ++sg) {
      const Poly& A = sg ? ga[z] : ga[y];
      const Poly& B = sg ? gb[y] : gb[z];
      const double sign = sg ? -1.0 : 1.0;
      for (int p = 0; p < A.n; ++p)
        for (int q = 0; q < B.n; ++q)
          for (int r = 0; r < pc.n; ++r)
            s += sign * A.t[p].c * B.t[q].c * pc.t[r].c *
                 kSphereMeans.m[A.t[p].i + B.t[q].i + pc.t[r].i + (x == 0)]
                               [A.t[p].j + B.t[q].j + pc.t[r].j + (x == 1)]
                               [A.t[p].k + B.t[q].k + pc.t[r].k + (x == 2)];
    }
  }
  return s;
}

// Unnormalised coupling of natural strided components (a, b, c).
constexpr double coupling_raw(int a, int b, int c) {
  return ((l_of(a) + l_of(b) + l_of(c)) & 1) ? triple_raw(a, b, c) : gaunt_raw(a, b, c);
}

constexpr bool triangle(int l1, int l2, int lo) {
  return lo >= (l1 > l2 ? l1 - l2 : l2 - l1) && lo <= l1 + l2;
}

constexpr double abs_c(double v) { return v < 0 ? -v : v; }

constexpr int kind_width(int kind, int l_max) {
  const int D = (l_max + 1) * (l_max + 1);
  return kind == kScalarOut ? 1 : (kind == kBothParities ? 2 * D : D);
}

// Whether strided component c (of a feature with D natural components) is a
// slot that can hold a kept irrep, and its l and parity class.
struct CompInfo { bool used; int l; bool natural; int base; };

constexpr CompInfo comp_info(int c, int D) {
  const bool nat = c < D;
  const int cc = nat ? c : c - D;
  return CompInfo{nat || cc > 0, l_of(cc), nat, cc};
}

// Whether the path (input component a, harmonic component b, output
// component c) is kept by a layer of the given kinds.
constexpr bool path_kept(int a, int b, int c, int l_max, int in_kind, int out_kind) {
  const int D = (l_max + 1) * (l_max + 1);
  if (a >= kind_width(in_kind, l_max) || b >= D || c >= kind_width(out_kind, l_max)) return false;
  const CompInfo ia = comp_info(a, D), io = comp_info(c, D);
  if (!ia.used || !io.used) return false;
  const int l2 = l_of(b);
  if (!triangle(ia.l, l2, io.l)) return false;
  // p1 p2 = s1 (-1)^(l1 + l2); the output is natural iff that equals (-1)^l_out
  const bool out_natural = ia.natural == (((ia.l + l2 + io.l) & 1) == 0);
  return out_natural == io.natural;
}

struct TpEntry { int a, b, c; };
struct TpList { int n; TpEntry e[1280]; };

// Non-zeros of the fused table W[a, b, c] in a fixed order (a, b, c ascending).
constexpr TpList tp_list(int l_max, int in_kind, int out_kind) {
  TpList L{};
  const int D = (l_max + 1) * (l_max + 1);
  const int din = kind_width(in_kind, l_max), dout = kind_width(out_kind, l_max);
  for (int a = 0; a < din; ++a)
    for (int b = 0; b < D; ++b)
      for (int c = 0; c < dout; ++c)
        if (path_kept(a, b, c, l_max, in_kind, out_kind) &&
            abs_c(coupling_raw(comp_info(a, D).base, b, comp_info(c, D).base)) > 1e-12) {
          L.e[L.n] = TpEntry{a, b, c};
          ++L.n;
        }
  return L;
}

template <int LMAX, int IN, int OUT>
struct TpPattern {
  static constexpr int Lmax = LMAX;
  static constexpr int In = IN, Out = OUT;
  static constexpr int DIM = (LMAX + 1) * (LMAX + 1);   // harmonic / environment-sum components
  static constexpr int DIN = kind_width(IN, LMAX);
  static constexpr int DOUT = kind_width(OUT, LMAX);
  static constexpr TpList list = tp_list(LMAX, IN, OUT);
  static constexpr int NNZ = list.n;
};

// The contractions take the non-zero weights through a pointer of type WP:
// the kernel-argument array, or a table in device memory seen through the
// constant address space, so that either way the wave-uniform weights are read
// with scalar loads instead of occupying vector registers.
//
// Three forms share one unrolled walk over the non-zeros k = (a, b, c):
//   kTpFwd:  T[c]  += w_k V[a] G[b]     (X = V, Y = G,  Z = T)
//   kTpAdjV: gV[a] += w_k G[b] gT[c]    (X = G, Y = gT, Z = gV)
//   kTpAdjG: gG[b] += w_k V[a] gT[c]    (X = V, Y = gT, Z = gG)
// Tables with more non-zeros than fit the kernel arguments are walked in
// blocks separated by scheduling barriers: the products w_k X[.] do not
// depend on the accumulators, and without the barriers the scheduler hoists
// hundreds of them at once and runs out of registers.
enum TpOp { kTpFwd = 0, kTpAdjV = 1, kTpAdjG = 2 };
constexpr int kTpBlock = 64;

template <class Pat, int OP, int K, class WP>
__device__ __forceinline__ void tp_term(const float* X, const float* Y, float* Z, WP w) {
  constexpr TpEntry e = Pat::list.e[K];
  if constexpr (OP == kTpFwd) Z[e.c] = fmaf(w[K] * X[e.a], Y[e.b], Z[e.c]);
  else if constexpr (OP == kTpAdjV) Z[e.a] = fmaf(w[K] * X[e.b], Y[e.c], Z[e.a]);
  else Z[e.b] = fmaf(w[K] * X[e.a], Y[e.c], Z[e.b]);
}

template <class Pat, int OP, int K0, class WP, std::size_t... K>
__device__ __forceinline__ void tp_run(const float* X, const float* Y, float* Z, WP w, std::index_sequence<K...>) {
  (tp_term<Pat, OP, K0 + (int)K>(X, Y, Z, w), ...);
}

template <class Pat, int J>
constexpr int tp_block_len() {
  return Pat::NNZ - J * kTpBlock < kTpBlock ? Pat::NNZ - J * kTpBlock : kTpBlock;
}

template <class Pat, int OP, class WP, std::size_t... J>
__device__ __forceinline__ void tp_blocks(const float* X, const float* Y, float* Z, WP w, std::index_sequence<J...>) {
  ((tp_run<Pat, OP, (int)J * kTpBlock>(X, Y, Z, w, std::make_index_sequence<tp_block_len<Pat, (int)J>()>{}),
    __builtin_amdgcn_sched_barrier(0)),
   ...);
}

template <class Pat, int OP, class WP>
__device__ __forceinline__ void tp_contract(const float* X, const float* Y, float* Z, WP w) {
  if constexpr (Pat::NNZ <= 83) {
    tp_run<Pat, OP, 0>(X, Y, Z, w, std::make_index_sequence<Pat::NNZ>{});
  } else {
    tp_blocks<Pat, OP>(X, Y, Z, w, std::make_index_sequence<(Pat::NNZ + kTpBlock - 1) / kTpBlock>{});
  }
}

// T[c] += w_k V[a] G[b] over the non-zeros k of the pattern.
template <class Pat, class WP>
__device__ __forceinline__ void tp_forward(const float* V, const float* G, float* T, WP w) {
  tp_contract<Pat, kTpFwd>(V, G, T, w);
}

// gV[a] += w_k G[b] gT[c]   (adjoint with respect to the edge features)
template <class Pat, class WP>
__device__ __forceinline__ void tp_adjoint_v(const float* G, const float* gT, float* gV, WP w) {
  tp_contract<Pat, kTpAdjV>(G, gT, gV, w);
}

// gG[b] += w_k V[a] gT[c]   (adjoint with respect to the environment sum)
template <class Pat, class WP>
__device__ __forceinline__ void tp_adjoint_g(const float* V, const float* gT, float* gG, WP w) {
  tp_contract<Pat, kTpAdjG>(V, gT, gG, w);
}

}  // namespace allegro
