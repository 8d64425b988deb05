// Compile-time lattice descriptions for the HIP kernels.
//
// D2Q9, D3Q19 and D3Q27 are the Gauss-Hermite quadratures the paper uses
// (Sec. II.A).  Directions follow the order documented in include/lbm.h:
// rest first, then opposite pairs (2k-1, 2k).  Velocities are generated from
// a single ordered list of the 26 non-rest unit-cube directions; D2Q9 takes
// the in-plane subset in the same pairing.
//
// The third-order Hermite terms each lattice can carry (Sec. II.A: D2Q9 and
// D3Q27 resolve the xxy-type and xyz polynomials; D3Q19 only resolves the
// sums and differences of the pairs xxy/yzz, xyy/xzz, xxz/yyz) are exposed
// as a short basis with compile-time values H_k(xi_i) and norms
// N_k = sum_i w_i H_k(xi_i)^2.
#pragma once

#include <cstdint>

namespace hrlbm {

constexpr double kCs2 = 1.0 / 3.0;

// 26 directions of the 3x3x3 stencil, paired as (+v, -v)
struct Dir {
  int x, y, z;
};
constexpr Dir kDirs3[27] = {
    {0, 0, 0},   {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},
    {0, 0, 1},   {0, 0, -1},  {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},
    {-1, 1, 0},  {1, 0, 1},   {-1, 0, -1}, {1, 0, -1},  {-1, 0, 1},
    {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1},  {1, 1, 1},
    {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1},  {-1, 1, -1},
    {-1, 1, 1},  {1, -1, -1}};
constexpr Dir kDirs2[9] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0},
                           {0, 1, 0},  {0, -1, 0},  {1, 1, 0},
                           {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};

// third-order Hermite polynomial H_abc at integer velocity v
constexpr double h3(const Dir& v, int a, int b, int c) {
  const int comp[3] = {v.x, v.y, v.z};
  const double xa = comp[a], xb = comp[b], xc = comp[c];
  return xa * xb * xc -
         kCs2 * (xa * (b == c ? 1 : 0) + xb * (a == c ? 1 : 0) +
                 xc * (a == b ? 1 : 0));
}

// Indices into the packed third-order coefficient set
//   {xxy, xyy, xxz, xzz, yyz, yzz, xyz}
enum A3 { kXXY = 0, kXYY, kXXZ, kXZZ, kYYZ, kYZZ, kXYZ };
constexpr int kA3Idx[7][3] = {{0, 0, 1}, {0, 1, 1}, {0, 0, 2}, {0, 2, 2},
                              {1, 1, 2}, {1, 2, 2}, {0, 1, 2}};

// A basis element: sum_j s_j H_{idx_j}, up to two packed components.
struct Basis3 {
  int n;
  int idx[2];
  int sgn[2];
};

// velocity set, weights and third-order basis of each lattice
template <int Q>
struct LatticeSet;

template <>
struct LatticeSet<9> {
  static constexpr int Q = 9, D = 2, K = 2;
  static constexpr Dir dir(int i) { return kDirs2[i]; }
  static constexpr double w(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
  static constexpr Basis3 basis(int k) {
    return k == 0 ? Basis3{1, {kXXY, 0}, {1, 0}} : Basis3{1, {kXYY, 0}, {1, 0}};
  }
};

template <>
struct LatticeSet<19> {
  static constexpr int Q = 19, D = 3, K = 6;
  static constexpr Dir dir(int i) { return kDirs3[i]; }
  static constexpr double w(int i) {
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
  // (xxy +- yzz), (xyy +- xzz), (xxz +- yyz)
  static constexpr Basis3 basis(int k) {
    return k == 0   ? Basis3{2, {kXXY, kYZZ}, {1, 1}}
           : k == 1 ? Basis3{2, {kXXY, kYZZ}, {1, -1}}
           : k == 2 ? Basis3{2, {kXYY, kXZZ}, {1, 1}}
           : k == 3 ? Basis3{2, {kXYY, kXZZ}, {1, -1}}
           : k == 4 ? Basis3{2, {kXXZ, kYYZ}, {1, 1}}
                    : Basis3{2, {kXXZ, kYYZ}, {1, -1}};
  }
};

template <>
struct LatticeSet<27> {
  static constexpr int Q = 27, D = 3, K = 7;
  static constexpr Dir dir(int i) { return kDirs3[i]; }
  static constexpr double w(int i) {
    return i == 0 ? 8.0 / 27.0
                  : (i < 7 ? 2.0 / 27.0 : (i < 19 ? 1.0 / 54.0 : 1.0 / 216.0));
  }
  static constexpr Basis3 basis(int k) { return Basis3{1, {k, 0}, {1, 0}}; }
};

// ------------------------------------------------------------------------
// Full recursive regularization (Sec. II.A, order n > 2).  D2Q9 and D3Q27
// are tensor products of the 1D three-velocity quadrature, on which the 1D
// Hermite polynomial of degree 3 vanishes (xi^3 = xi, 3 cs^2 = 1).  The
// polynomials they resolve are He_nx(xi_x) He_ny(xi_y) He_nz(xi_z) with every
// n_a <= 2.  Those of order 4 and above, in addition to the second- and
// third-order terms, are listed here by multi-index.
// ------------------------------------------------------------------------
struct MultiIndex {
  int n[3];
};
constexpr MultiIndex kHigh2[1] = {{{2, 2, 0}}};
constexpr MultiIndex kHigh3[10] = {
    {{2, 2, 0}}, {{2, 0, 2}}, {{0, 2, 2}}, {{2, 1, 1}}, {{1, 2, 1}},  // order 4
    {{1, 1, 2}}, {{2, 2, 1}}, {{2, 1, 2}}, {{1, 2, 2}},               // 4, 5
    {{2, 2, 2}}};                                                     // 6

// Collision of FLUID cells: the regularized operator, or the comparators
// the paper measures it against (Sec. II.A): LBM-BGK, and LBM-MRT on D2Q9.
enum : int { kCollRR = 0, kCollBGK = 1, kCollMRT = 2 };

// Lattice seen by the kernels: the velocity set, the regularization order
// (kFull: every resolved order; otherwise the third) and the collision.
template <int Q, bool F = false, int C = kCollRR>
struct Lattice : LatticeSet<Q> {
  static_assert(!F || Q != 19, "full-order regularization needs D2Q9 or D3Q27");
  static_assert(C != kCollMRT || Q == 9, "the MRT comparator is D2Q9 only");
  static_assert(C == kCollRR || !F, "comparators have no higher orders");
  static constexpr bool kFull = F;
  static constexpr int kColl = C;
  static constexpr int KH = !F ? 0 : (Q == 9 ? 1 : 10);
  static constexpr MultiIndex high(int k) { return Q == 9 ? kHigh2[k] : kHigh3[k]; }
};

// 1D Hermite polynomial of degree n <= 2 at an integer velocity component
constexpr double he1(int n, int v) {
  return n == 0 ? 1.0 : (n == 1 ? (double)v : (double)(v * v) - kCs2);
}

// value of high-order polynomial k at direction i, and its lattice norm
template <class L>
constexpr double high_h(int i, int k) {
  const MultiIndex m = L::high(k);
  const Dir v = L::dir(i);
  return he1(m.n[0], v.x) * he1(m.n[1], v.y) * he1(m.n[2], v.z);
}
template <class L>
constexpr double high_norm(int k) {
  double s = 0.0;
  for (int i = 0; i < L::Q; ++i) s += L::w(i) * high_h<L>(i, k) * high_h<L>(i, k);
  return s;
}
constexpr int high_order(const MultiIndex& m) { return m.n[0] + m.n[1] + m.n[2]; }

// value of basis element k at direction i
template <class L>
constexpr double basis_h(int i, int k) {
  const Basis3 b = L::basis(k);
  double s = 0.0;
  for (int j = 0; j < b.n; ++j)
    s += b.sgn[j] * h3(L::dir(i), kA3Idx[b.idx[j]][0], kA3Idx[b.idx[j]][1],
                       kA3Idx[b.idx[j]][2]);
  return s;
}

// lattice norm N_k = sum_i w_i H_k(xi_i)^2, evaluated at compile time
template <class L>
constexpr double basis_norm(int k) {
  double s = 0.0;
  for (int i = 0; i < L::Q; ++i) s += L::w(i) * basis_h<L>(i, k) * basis_h<L>(i, k);
  return s;
}

template <class L>
constexpr int opposite(int i) {
  return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1);
}

// direction index of velocity (x, y, z) in lattice L, -1 if absent
template <class L>
constexpr int find_dir(int x, int y, int z) {
  for (int i = 0; i < L::Q; ++i)
    if (L::dir(i).x == x && L::dir(i).y == y && L::dir(i).z == z) return i;
  return -1;
}

}  // namespace hrlbm
