/*
 * Plain FP64 CPU oracle for the Hermite-regularized lattice Boltzmann step
 * (Brogi, Malaspinas, Chopard & Bonadonna, "Hermite regularization of the
 * Lattice Boltzmann Method for open source computational aeroacoustics",
 * arXiv:1710.02065).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU library is checked against.  It shares no code, header, table or
 * constant generator with the HIP path; only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg load it.  It is written to be read
 * against the paper, not to be fast: every cell is handled one at a time,
 * with the full 3x3 and 3x3x3 moment tensors, in the order the paper states
 * the algorithm.  OpenMP over the outermost axis is the only concession to
 * speed; the update has no reductions, so results do not depend on threads.
 *
 * Readings of passages the paper leaves open (all listed in the design notes):
 *  - eq. (eqH): the first-order term is xi.u/cs^2 (the printed form lacks
 *    ".u"); third-order equilibrium coefficients are rho*u*u*u from
 *    eq. (recursive1).
 *  - eq. (neqH): no rho factor; a2_neq is an absolute moment.
 *  - a2 = Pi - rho*cs^2*I (the printed "a2 = P - rho(uu - delta)" is garbled);
 *    a2_neq = Pi - rho*cs^2*I - rho*u*u.
 *  - third-order basis per lattice (Sec. II.A singles out D2Q9 and D3Q27
 *    for it): D2Q9 {xxy, xyy}; D3Q27 {xxy, xyy, xxz, xzz, yyz, yzz, xyz};
 *    D3Q19 (not covered by that property) uses the lattice-orthogonal
 *    combinations (H_xxy +- H_yzz) and likewise for the x- and z-odd pairs.
 *    Each basis element k is rebuilt as w_i H_k,i c_k / N_k, with N_k the
 *    lattice norm sum_i w_i H_k,i^2, so the rebuilt populations carry the
 *    target third-order moment c_k exactly.
 *  - full recursive regularization (Sec. II.A, order n > 2): on D2Q9 and
 *    D3Q27 every Hermite polynomial the lattice resolves (degree <= 2 per
 *    axis: up to fourth order in 2D and sixth in 3D), coefficients
 *    rho u...u (eq. recursive1) and the eq. (recursive2) recursion.  D3Q19
 *    is refused: the paper names only D2Q9 and D3Q27 as carrying the
 *    property that makes this expansion exact.
 *  - sponge (Sec. II.C, eqs. spongeLB, dampingLBM, modifiedMoments): the
 *    unspecified factors n and m are 1/2, which makes the homogeneous decay
 *    rate of the BGK variant equal the effective damping sigma_eff the
 *    paper prints (eq. effectiveCoefficient).  rho* and j* are solved in
 *    closed form.  The force is added in full.
 *  - pull streaming of post-collision populations; halfway bounce-back
 *    (wall at rest); specular free-slip; zero-gradient outflow by clamping
 *    the source to the last interior row; equilibrium inlet cells.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_CS2 (1.0 / 3.0)

/* ------------------------------------------------------------------------ */
/* Lattices (Sec. II.A: D2Q9, D3Q19, D3Q27 Gauss-Hermite quadratures).       */
/* The paper cites the lattices without printing tables; these are the       */
/* textbook velocity sets and weights, in the direction order documented in  */
/* the library header: rest, then opposite pairs (odd i, i+1).               */
/* ------------------------------------------------------------------------ */

static const int ORA_D2Q9_XI[9][3] = {
    {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
static const double ORA_D2Q9_W[9] = {4.0 / 9,  1.0 / 9,  1.0 / 9,
                                     1.0 / 9,  1.0 / 9,  1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36};

static const int ORA_D3Q27_XI[27][3] = {
    {0, 0, 0},                                                 /* rest   */
    {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},         /* faces  */
    {0, 0, 1},   {0, 0, -1},                                   /*        */
    {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},         /* edges  */
    {1, 0, 1},   {-1, 0, -1}, {1, 0, -1},  {-1, 0, 1},         /*        */
    {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1},         /*        */
    {1, 1, 1},   {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},        /* corners*/
    {1, -1, 1},  {-1, 1, -1}, {-1, 1, 1},  {1, -1, -1}};

typedef struct {
  int q, d;
  int xi[27][3];
  double w[27];
  int opp[27];
  int full; /* 1: full recursive regularization (D2Q9 and D3Q27 only) */
} ora_lattice;

/* Fill *L for lattice id 9, 19 or 27; returns 0, or -1 for an unknown id. */
static int ora_make_lattice(int id, ora_lattice* L) {
  int i, a;
  memset(L, 0, sizeof(*L));
  if (id == 9) {
    L->q = 9;
    L->d = 2;
    for (i = 0; i < 9; ++i) {
      for (a = 0; a < 3; ++a) L->xi[i][a] = ORA_D2Q9_XI[i][a];
      L->w[i] = ORA_D2Q9_W[i];
    }
  } else if (id == 19 || id == 27) {
    L->q = id;
    L->d = 3;
    for (i = 0; i < id; ++i) {
      int n2 = 0;
      for (a = 0; a < 3; ++a) {
        L->xi[i][a] = ORA_D3Q27_XI[i][a];
        n2 += ORA_D3Q27_XI[i][a] * ORA_D3Q27_XI[i][a];
      }
      if (id == 19) /* D3Q19: 1/3 rest, 1/18 faces, 1/36 edges */
        L->w[i] = n2 == 0 ? 1.0 / 3 : (n2 == 1 ? 1.0 / 18 : 1.0 / 36);
      else /* D3Q27: 8/27, 2/27, 1/54, 1/216 */
        L->w[i] = n2 == 0 ? 8.0 / 27
                          : (n2 == 1 ? 2.0 / 27 : (n2 == 2 ? 1.0 / 54 : 1.0 / 216));
    }
  } else {
    return -1;
  }
  for (i = 0; i < L->q; ++i) {
    int j;
    for (j = 0; j < L->q; ++j)
      if (L->xi[j][0] == -L->xi[i][0] && L->xi[j][1] == -L->xi[i][1] &&
          L->xi[j][2] == -L->xi[i][2])
        L->opp[i] = j;
  }
  return 0;
}

int ora_lattice_info(int id, int* q, int* d, int* xi, double* w, int* opp) {
  ora_lattice L;
  int i, a;
  if (ora_make_lattice(id, &L)) return -1;
  if (q) *q = L.q;
  if (d) *d = L.d;
  for (i = 0; i < L.q; ++i) {
    if (xi)
      for (a = 0; a < 3; ++a) xi[3 * i + a] = L.xi[i][a];
    if (w) w[i] = L.w[i];
    if (opp) opp[i] = L.opp[i];
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Hermite polynomials on the lattice (eq. HE with the lattice weights).     */
/* ------------------------------------------------------------------------ */

/* Second-order Hermite polynomial H_ab(xi_i) = xi_a xi_b - cs^2 delta_ab. */
static double ora_h2(const ora_lattice* L, int i, int a, int b) {
  return (double)L->xi[i][a] * L->xi[i][b] - (a == b ? ORA_CS2 : 0.0);
}

/* Third-order Hermite polynomial
 * H_abc = xi_a xi_b xi_c - cs^2 (xi_a d_bc + xi_b d_ac + xi_c d_ab). */
static double ora_h3(const ora_lattice* L, int i, int a, int b, int c) {
  double xa = L->xi[i][a], xb = L->xi[i][b], xc = L->xi[i][c];
  return xa * xb * xc -
         ORA_CS2 * (xa * (b == c) + xb * (a == c) + xc * (a == b));
}

/* Third-order part of a regularized population:
 *   sum_k H_k,i c_k / N_k
 * over the basis the lattice supports (see header comment), with c_k the
 * matching combination of the symmetric 3rd-order tensor a3 and N_k the
 * lattice norm of H_k, both in closed form. */
static double ora_third_order(const ora_lattice* L, int i, double a3[3][3][3]) {
  const double cs6 = ORA_CS2 * ORA_CS2 * ORA_CS2;
  enum { X = 0, Y = 1, Z = 2 };
  if (L->q == 9) {
    return (ora_h3(L, i, X, X, Y) * a3[X][X][Y] +
            ora_h3(L, i, X, Y, Y) * a3[X][Y][Y]) /
           (2 * cs6);
  }
  if (L->q == 27) {
    double s = ora_h3(L, i, X, X, Y) * a3[X][X][Y] +
               ora_h3(L, i, X, Y, Y) * a3[X][Y][Y] +
               ora_h3(L, i, X, X, Z) * a3[X][X][Z] +
               ora_h3(L, i, X, Z, Z) * a3[X][Z][Z] +
               ora_h3(L, i, Y, Y, Z) * a3[Y][Y][Z] +
               ora_h3(L, i, Y, Z, Z) * a3[Y][Z][Z];
    return s / (2 * cs6) + ora_h3(L, i, X, Y, Z) * a3[X][Y][Z] / cs6;
  }
  /* D3Q19: for each odd axis the pair (P, Q) of third-order polynomials that
   * the lattice does not separate is replaced by (P + Q) with norm 2 cs^6 and
   * (P - Q) with norm 6 cs^6; coefficients a_P +- a_Q. */
  {
    double s = 0.0;
    /* pairs: (xxy, yzz) odd in y, (xyy, xzz) odd in x, (xxz, yyz) odd in z */
    const int pairs[3][2][3] = {{{X, X, Y}, {Y, Z, Z}},
                                {{X, Y, Y}, {X, Z, Z}},
                                {{X, X, Z}, {Y, Y, Z}}};
    int p;
    for (p = 0; p < 3; ++p) {
      const int* P = pairs[p][0];
      const int* Q = pairs[p][1];
      double hp = ora_h3(L, i, P[0], P[1], P[2]);
      double hq = ora_h3(L, i, Q[0], Q[1], Q[2]);
      double ap = a3[P[0]][P[1]][P[2]];
      double aq = a3[Q[0]][Q[1]][Q[2]];
      s += (hp + hq) * (ap + aq) / (2 * cs6) + (hp - hq) * (ap - aq) / (6 * cs6);
    }
    return s;
  }
}

/* ------------------------------------------------------------------------ */
/* Full recursive regularization (Sec. II.A, expansion to order n > 2 on the */
/* lattices Sec. II.A singles out, D2Q9 and D3Q27).  These are tensor       */
/* products of the 1D three-velocity quadrature, on which the 1D Hermite     */
/* polynomial of degree 3 vanishes (xi^3 = xi and 3 cs^2 = 1); the Hermite   */
/* polynomials they resolve are the products He_nx(xi_x) He_ny(xi_y)        */
/* He_nz(xi_z) with every n_a <= 2, mutually orthogonal under the weights,   */
/* with norms prod_a n_a! cs^(2 n_a).  A multi-index (nx, ny, nz) stands for */
/* the tensor component whose index list holds nx x's, ny y's and nz z's;    */
/* summing the contraction H^(n):a^(n)/(n! cs^2n) over the index lists that  */
/* share it gives H_k a_k / N_k.                                             */
/* ------------------------------------------------------------------------ */

/* 1D Hermite polynomial of degree n <= 2 for the weight of variance cs^2. */
static double ora_he(int n, double x) {
  return n == 0 ? 1.0 : (n == 1 ? x : x * x - ORA_CS2);
}

/* Non-equilibrium coefficient a^n_neq of the index list s[0..n-1] by
 * eq. (recursive2): a^n = a^(n-1) u_{s_n} plus, for every earlier index s_k,
 * a2_{s_k s_n} times the product of u over the remaining n - 2 indices;
 * a^0_neq = a^1_neq = 0 and a^2_neq is a2 itself. */
static double ora_aneq_rec(const int* s, int n, const double u[3],
                           double a2[3][3]) {
  double r;
  int k, j;
  if (n < 2) return 0.0;
  if (n == 2) return a2[s[0]][s[1]];
  r = ora_aneq_rec(s, n - 1, u, a2) * u[s[n - 1]];
  for (k = 0; k < n - 1; ++k) {
    double p = a2[s[k]][s[n - 1]];
    for (j = 0; j < n - 1; ++j)
      if (j != k) p *= u[s[j]];
    r += p;
  }
  return r;
}

/* sum over every resolved multi-index k of order >= min_order:
 *   w_i H_k(xi_i) A_k / N_k
 * with A_k = rho u_x^nx u_y^ny u_z^nz (eq. recursive1) when a2 is NULL, and
 * the eq. (recursive2) coefficient of a2 otherwise. */
static void ora_full_sum(const ora_lattice* L, double rho, const double u[3],
                         double a2[3][3], int min_order, double* out) {
  int n[3], i;
  const int top = 2;
  for (i = 0; i < L->q; ++i) out[i] = 0.0;
  for (n[2] = 0; n[2] <= (L->d == 3 ? top : 0); ++n[2])
    for (n[1] = 0; n[1] <= top; ++n[1])
      for (n[0] = 0; n[0] <= top; ++n[0]) {
        int seq[6], len = 0, a, r;
        double A, Nk = 1.0;
        for (a = 0; a < 3; ++a)
          for (r = 0; r < n[a]; ++r) seq[len++] = a;
        if (len < min_order) continue;
        if (a2) {
          A = ora_aneq_rec(seq, len, u, a2);
        } else {
          A = rho;
          for (r = 0; r < len; ++r) A *= u[seq[r]];
        }
        for (a = 0; a < 3; ++a)
          Nk *= (n[a] == 2 ? 2.0 * ORA_CS2 * ORA_CS2 : (n[a] == 1 ? ORA_CS2 : 1.0));
        for (i = 0; i < L->q; ++i) {
          double H = 1.0;
          for (a = 0; a < 3; ++a) H *= ora_he(n[a], (double)L->xi[i][a]);
          out[i] += L->w[i] * H * A / Nk;
        }
      }
}

/* Extended equilibrium f^{eqH}_i(rho, u) of eq. (eqH): the second-order
 * polynomial of eq. (truncatedEq) plus the third-order Hermite terms with the
 * equilibrium coefficients a3_eq = rho u u u of eq. (recursive1). */
static void ora_feq(const ora_lattice* L, double rho, const double u[3],
                    double* feq) {
  const double cs2 = ORA_CS2, cs4 = ORA_CS2 * ORA_CS2;
  double a3[3][3][3];
  int i, a, b, c;
  if (L->full) { /* every resolved order, coefficients rho u...u */
    ora_full_sum(L, rho, u, NULL, 0, feq);
    return;
  }
  for (a = 0; a < 3; ++a)
    for (b = 0; b < 3; ++b)
      for (c = 0; c < 3; ++c) a3[a][b][c] = rho * u[a] * u[b] * u[c];
  for (i = 0; i < L->q; ++i) {
    double xu = 0.0, h2uu = 0.0;
    for (a = 0; a < L->d; ++a) xu += L->xi[i][a] * u[a];
    for (a = 0; a < L->d; ++a)
      for (b = 0; b < L->d; ++b) h2uu += ora_h2(L, i, a, b) * u[a] * u[b];
    feq[i] = L->w[i] * (rho * (1.0 + xu / cs2 + h2uu / (2 * cs4)) +
                        ora_third_order(L, i, a3));
  }
}

/* Regularized non-equilibrium f^{neqH}_i of eq. (neqH): the second-order
 * term from a2_neq plus the third-order term whose coefficients come from the
 * recursion eq. (recursive2) at n = 3:
 *   a3_neq,abc = u_a a2_bc + u_b a2_ac + u_c a2_ab. */
static void ora_fneq(const ora_lattice* L, const double u[3],
                     double a2[3][3], double* fneq) {
  const double cs4 = ORA_CS2 * ORA_CS2;
  double a3[3][3][3];
  int i, a, b, c;
  if (L->full) { /* orders 2 ... 2d from the recursion */
    ora_full_sum(L, 0.0, u, a2, 2, fneq);
    return;
  }
  for (a = 0; a < 3; ++a)
    for (b = 0; b < 3; ++b)
      for (c = 0; c < 3; ++c)
        a3[a][b][c] = u[a] * a2[b][c] + u[b] * a2[a][c] + u[c] * a2[a][b];
  for (i = 0; i < L->q; ++i) {
    double h2a2 = 0.0;
    for (a = 0; a < L->d; ++a)
      for (b = 0; b < L->d; ++b) h2a2 += ora_h2(L, i, a, b) * a2[a][b];
    fneq[i] = L->w[i] * (h2a2 / (2 * cs4) + ora_third_order(L, i, a3));
  }
}

/* a2 in the packed order (xx, yy, zz, xy, xz, yz) -> full symmetric tensor */
static void ora_unpack6(const double* p, double t[3][3]) {
  t[0][0] = p[0];
  t[1][1] = p[1];
  t[2][2] = p[2];
  t[0][1] = t[1][0] = p[3];
  t[0][2] = t[2][0] = p[4];
  t[1][2] = t[2][1] = p[5];
}

/* Lattice of a grid: the velocity set plus the regularization order;
 * returns -1 for an unknown id or full order on D3Q19. */
static int ora_lattice_order(int id, int full, ora_lattice* L) {
  if (ora_make_lattice(id, L)) return -1;
  if (full && id == 19) return -1;
  L->full = full ? 1 : 0;
  return 0;
}

void ora_equilibrium_ex(int lattice, int full, double rho, const double* u,
                        double* feq) {
  ora_lattice L;
  if (ora_lattice_order(lattice, full, &L)) return;
  ora_feq(&L, rho, u, feq);
}

void ora_noneq_ex(int lattice, int full, const double* u,
                  const double* a2packed, double* fneq) {
  ora_lattice L;
  double a2[3][3];
  if (ora_lattice_order(lattice, full, &L)) return;
  ora_unpack6(a2packed, a2);
  ora_fneq(&L, u, a2, fneq);
}

void ora_equilibrium(int lattice, double rho, const double* u, double* feq) {
  ora_equilibrium_ex(lattice, 0, rho, u, feq);
}

void ora_noneq(int lattice, const double* u, const double* a2packed,
               double* fneq) {
  ora_noneq_ex(lattice, 0, u, a2packed, fneq);
}

/* ------------------------------------------------------------------------ */
/* One-cell collision: eq. (optimizedLB), with the damping force of          */
/* eqs. (spongeLB) and (dampingLBM) when chi > 0.                            */
/* f holds the pre-collision (streamed) populations; post receives the       */
/* populations to stream.  rho_star/u_star (may be NULL) receive the         */
/* moments used in the rebuild.                                              */
/* ------------------------------------------------------------------------ */
static void ora_collide_cell(const ora_lattice* L, const double* f, double tau,
                             double chi, double rho_ref, const double* u_ref,
                             double* post, double* rho_star, double* u_star,
                             double* a2_out) {
  const double cs2 = ORA_CS2;
  double rho = 0.0, j[3] = {0, 0, 0}, Pi[3][3] = {{0}};
  double rs, js[3], u[3], a2[3][3];
  double E[27], N[27], Eref[27];
  int i, a, b;

  /* eq. (moments) and the second-order moment Pi = sum f xi xi */
  for (i = 0; i < L->q; ++i) {
    rho += f[i];
    for (a = 0; a < 3; ++a) {
      j[a] += f[i] * L->xi[i][a];
      for (b = 0; b < 3; ++b) Pi[a][b] += f[i] * L->xi[i][a] * L->xi[i][b];
    }
  }
  /* eq. (modifiedMoments) with n = m = 1/2: rho* = rho + sum F / 2 and
   * rho* u* = j + sum F xi / 2, where sum F = chi (rho_ref - rho*) and
   * sum F xi = chi (rho_ref u_ref - rho* u*); solved for rho*, rho* u*.
   * With chi = 0 these are the plain moments of eq. (moments). */
  rs = (rho + 0.5 * chi * rho_ref) / (1.0 + 0.5 * chi);
  for (a = 0; a < 3; ++a)
    js[a] = (j[a] + 0.5 * chi * rho_ref * u_ref[a]) / (1.0 + 0.5 * chi);
  for (a = 0; a < 3; ++a) u[a] = js[a] / rs;

  /* non-equilibrium second-order Hermite coefficient (in the lattice's d
   * dimensions; the z row and column stay zero in 2D) */
  for (a = 0; a < 3; ++a)
    for (b = 0; b < 3; ++b)
      a2[a][b] = (a < L->d && b < L->d)
                     ? Pi[a][b] - rs * cs2 * (a == b) - rs * u[a] * u[b]
                     : 0.0;

  ora_feq(L, rs, u, E);
  ora_fneq(L, u, a2, N);
  if (chi != 0.0) ora_feq(L, rho_ref, u_ref, Eref);
  for (i = 0; i < L->q; ++i) {
    post[i] = E[i] + (1.0 - 1.0 / tau) * N[i];
    if (chi != 0.0) post[i] += chi * (Eref[i] - E[i]);
  }
  if (rho_star) *rho_star = rs;
  if (u_star)
    for (a = 0; a < 3; ++a) u_star[a] = u[a];
  if (a2_out) { /* packed (xx, yy, zz, xy, xz, yz) */
    a2_out[0] = a2[0][0];
    a2_out[1] = a2[1][1];
    a2_out[2] = a2[2][2];
    a2_out[3] = a2[0][1];
    a2_out[4] = a2[0][2];
    a2_out[5] = a2[1][2];
  }
}

void ora_collide_ex(int lattice, int full, const double* f, double tau,
                    double chi, double rho_ref, const double* u_ref,
                    double* post) {
  ora_lattice L;
  if (ora_lattice_order(lattice, full, &L)) return;
  ora_collide_cell(&L, f, tau, chi, rho_ref, u_ref, post, NULL, NULL, NULL);
}

void ora_collide(int lattice, const double* f, double tau, double chi,
                 double rho_ref, const double* u_ref, double* post) {
  ora_collide_ex(lattice, 0, f, tau, chi, rho_ref, u_ref, post);
}

/* Standard LBM-BGK collision, eq. (standardLB) with the second-order
 * equilibrium of eq. (truncatedEq), plus the same damping force and
 * modified moments as above.  Test mode only: it is the operator the paper's
 * 1D sponge analysis (eq. effectiveCoefficient) is stated for. */
void ora_collide_bgk(int lattice, const double* f, double tau, double chi,
                     double rho_ref, const double* u_ref, double* post) {
  ora_lattice L;
  const double cs2 = ORA_CS2, cs4 = ORA_CS2 * ORA_CS2;
  double rho = 0.0, j[3] = {0, 0, 0}, rs, u[3], uref_[3];
  int i, a;
  if (ora_make_lattice(lattice, &L)) return;
  for (i = 0; i < L.q; ++i) {
    rho += f[i];
    for (a = 0; a < 3; ++a) j[a] += f[i] * L.xi[i][a];
  }
  rs = (rho + 0.5 * chi * rho_ref) / (1.0 + 0.5 * chi);
  for (a = 0; a < 3; ++a) {
    u[a] = (j[a] + 0.5 * chi * rho_ref * u_ref[a]) / (1.0 + 0.5 * chi) / rs;
    uref_[a] = u_ref[a];
  }
  for (i = 0; i < L.q; ++i) {
    double xu = 0, uu = 0, xr = 0, rr = 0, feq, fref;
    for (a = 0; a < 3; ++a) {
      xu += L.xi[i][a] * u[a];
      uu += u[a] * u[a];
      xr += L.xi[i][a] * uref_[a];
      rr += uref_[a] * uref_[a];
    }
    feq = L.w[i] * rs * (1 + xu / cs2 + xu * xu / (2 * cs4) - uu / (2 * cs2));
    fref = L.w[i] * rho_ref *
           (1 + xr / cs2 + xr * xr / (2 * cs4) - rr / (2 * cs2));
    post[i] = f[i] - (f[i] - feq) / tau + chi * (fref - feq);
  }
}

/* Multiple-relaxation-time collision on D2Q9 (Lallemand & Luo, Phys. Rev. E
 * 61, 6546, 2000), one of the comparators of Sec. II.A.  The nine moments
 * are projections on the orthogonal polynomials of the velocity
 *   1, e = -4 + 3|xi|^2, eps = 4 - 21/2 |xi|^2 + 9/2 |xi|^4, xi_x,
 *   q_x = (-5 + 3|xi|^2) xi_x, xi_y, q_y, xi_x^2 - xi_y^2, xi_x xi_y;
 * their equilibria are those of the second-order equilibrium (e = -2 rho
 * + 3 |j|^2/rho, eps = rho - 3 |j|^2/rho, q = -j, p_xx = (jx^2 - jy^2)/rho,
 * p_xy = jx jy / rho); each relaxes at its own rate s[k] and the
 * populations follow from the orthogonal projection.  s: rates of
 * (e, eps, q, nu); s_nu = 1/tau sets the viscosity. */
void ora_collide_mrt(const double* f, const double* s4, double* post) {
  ora_lattice L;
  double m[9] = {0}, meq[9], rate[9], norm[9] = {0};
  double poly[9][9];
  double rho, jx, jy, jj;
  int i, k;
  if (ora_make_lattice(9, &L)) return;
  for (i = 0; i < 9; ++i) {
    double x = L.xi[i][0], y = L.xi[i][1], e2 = x * x + y * y;
    poly[0][i] = 1.0;
    poly[1][i] = -4.0 + 3.0 * e2;
    poly[2][i] = 4.0 - 10.5 * e2 + 4.5 * e2 * e2;
    poly[3][i] = x;
    poly[4][i] = (-5.0 + 3.0 * e2) * x;
    poly[5][i] = y;
    poly[6][i] = (-5.0 + 3.0 * e2) * y;
    poly[7][i] = x * x - y * y;
    poly[8][i] = x * y;
  }
  for (k = 0; k < 9; ++k)
    for (i = 0; i < 9; ++i) {
      m[k] += poly[k][i] * f[i];
      norm[k] += poly[k][i] * poly[k][i];
    }
  rho = m[0];
  jx = m[3];
  jy = m[5];
  jj = jx * jx + jy * jy;
  meq[0] = rho;
  meq[1] = -2.0 * rho + 3.0 * jj / rho;
  meq[2] = rho - 3.0 * jj / rho;
  meq[3] = jx;
  meq[4] = -jx;
  meq[5] = jy;
  meq[6] = -jy;
  meq[7] = (jx * jx - jy * jy) / rho;
  meq[8] = jx * jy / rho;
  rate[0] = rate[3] = rate[5] = 0.0;
  rate[1] = s4[0];
  rate[2] = s4[1];
  rate[4] = rate[6] = s4[2];
  rate[7] = rate[8] = s4[3];
  for (i = 0; i < 9; ++i) {
    double d = 0.0;
    for (k = 0; k < 9; ++k) d += poly[k][i] * rate[k] * (m[k] - meq[k]) / norm[k];
    post[i] = f[i] - d;
  }
}

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the k-th output (k >= 0) of */
/* the generator seeded with `seed`.  Used for the inlet perturbation.       */
/* ------------------------------------------------------------------------ */
uint64_t ora_splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* uniform in [-1, 1) with 2^-23 spacing from the top 24 bits */
static double ora_uniform_pm1(uint64_t z) {
  return (double)(z >> 40) * (1.0 / 8388608.0) - 1.0;
}

/* ------------------------------------------------------------------------ */
/* Grid update                                                               */
/* ------------------------------------------------------------------------ */

enum { ORA_PERIODIC = 0, ORA_FREESLIP = 1, ORA_OUTFLOW = 2 };
enum { ORA_FLUID = 0, ORA_SOLID = 1, ORA_INLET = 2 };

typedef struct {
  int lattice;              /* 9, 19, 27 */
  int level;                /* refinement level of this grid (0 = coarse) */
  int64_t nx, ny, nz;       /* nz = 1 in 2D */
  double tau, rho0;
  double u_in[3];           /* inlet velocity U * u_dir */
  int face_bc[6];           /* x-, x+, y-, y+, z-, z+ */
  int sponge_width[6];      /* cells, per face; 0 = none */
  double chi_max, rho_ref, u_ref[3];
  uint64_t seed;
  double inlet_noise;
  int full_order;           /* 1: full recursive regularization */
  int levels;               /* levels of the hierarchy this grid belongs to */
  /* absorbing layer given per cell (Sec. II.C with an arbitrary geometry,
   * e.g. circular, and spatially varying reference fields): when sp_chi is
   * set it replaces the face profile; sp_rho [N] and sp_u [3][N] (each may be
   * NULL: rho_ref, u_ref) give the reference state per cell */
  const double* sp_chi;
  const double* sp_rho;
  const double* sp_u;
  /* collision of FLUID cells: 0 the regularized operator (eq. optimizedLB);
   * 1 LBM-BGK (eq. standardLB); 2 LBM-MRT on D2Q9 (the comparators of
   * Sec. II.A); initial and inlet states are the regularized ones */
  int collision;
} ora_grid;

/* Sponge strength chi(x) = chi_max * max over faces of the polynomial
 * profile sigma of Sec. II.C,
 *   sigma(s) = 3125 (L - s)(s - s0)^4 / (256 (L - s0)^5),
 * with s the coordinate normal to the face, s0 = n - W the inner edge and
 * L = n one past the last node, for a face of width W on an axis of n nodes;
 * the low face uses the mirrored coordinate n - 1 - x. */
/* The profile itself, for a coordinate s across a layer from its inner
 * edge s0 to L (zero outside [s0, L]); used for other layer geometries
 * (e.g. circular, with s the distance from a centre). */
double ora_sponge_sigma(double s, double s0, double L) {
  if (s < s0 || s > L) return 0.0;
  return 3125.0 * (L - s) * pow(s - s0, 4) / (256.0 * pow(L - s0, 5));
}

double ora_sponge_chi(const ora_grid* g, int64_t x, int64_t y, int64_t z) {
  int64_t pos[3] = {x, y, z}, dims[3] = {g->nx, g->ny, g->nz};
  double best = 0.0;
  int face;
  if (g->chi_max == 0.0) return 0.0;
  for (face = 0; face < 6; ++face) {
    int axis = face / 2;
    int64_t n = dims[axis], W = g->sponge_width[face];
    double s, s0, Lend, sig;
    if (W <= 0) continue;
    s = (face % 2 == 1) ? (double)pos[axis] : (double)(n - 1 - pos[axis]);
    s0 = (double)(n - W);
    Lend = (double)n;
    if (s < s0) continue;
    sig = 3125.0 * (Lend - s) * pow(s - s0, 4) / (256.0 * pow(Lend - s0, 5));
    if (sig > best) best = sig;
  }
  return g->chi_max * best;
}

static int64_t ora_cell(const ora_grid* g, int64_t x, int64_t y, int64_t z) {
  return (z * g->ny + y) * g->nx + x;
}

/* Direction index with the component on `axis` reversed (specular mirror). */
static int ora_mirror(const ora_lattice* L, int i, int axis) {
  int j, a;
  for (j = 0; j < L->q; ++j) {
    int same = 1;
    for (a = 0; a < 3; ++a) {
      int want = (a == axis) ? -L->xi[i][a] : L->xi[i][a];
      if (L->xi[j][a] != want) same = 0;
    }
    if (same) return j;
  }
  return -1;
}

/* Source of population i pulled into cell (x, y, z): the cell x - xi_i,
 * mapped through the face rules axis by axis (periodic wrap; free-slip:
 * reflected back to the boundary row with the population mirrored;
 * outflow: the boundary row).  Returns 1 if that source is SOLID (the link
 * is bounced back), else 0 with *src_cell and *src_pop set. */
static int ora_source(const ora_grid* g, const ora_lattice* L,
                      const uint8_t* mask, int64_t x, int64_t y, int64_t z,
                      int i, int64_t* src_cell, int* src_pop) {
  int64_t s[3] = {x - L->xi[i][0], y - L->xi[i][1], z - L->xi[i][2]};
  int64_t dims[3] = {g->nx, g->ny, g->nz};
  int si = i, a;
  for (a = 0; a < L->d; ++a) {
    int64_t n = dims[a];
    int face;
    if (s[a] >= 0 && s[a] < n) continue;
    face = 2 * a + (s[a] >= n ? 1 : 0);
    switch (g->face_bc[face]) {
      case ORA_PERIODIC:
        s[a] = (s[a] % n + n) % n;
        break;
      case ORA_FREESLIP: /* the particle was reflected at the wall */
        s[a] = s[a] < 0 ? 0 : n - 1;
        si = ora_mirror(L, si, a);
        break;
      default: /* ORA_OUTFLOW: zero gradient, copy of the last row */
        s[a] = s[a] < 0 ? 0 : n - 1;
        break;
    }
  }
  *src_cell = ora_cell(g, s[0], s[1], s[2]);
  *src_pop = si;
  return mask && mask[*src_cell] == ORA_SOLID;
}

/* Pre-collision population i at cell (x, y, z), pulled from the
 * post-collision field fin (left side of eq. optimizedLB read backwards); a
 * link whose source is a SOLID cell is bounced back halfway: the population
 * that left this cell towards the wall returns reversed. */
static double ora_pull(const ora_grid* g, const ora_lattice* L,
                       const uint8_t* mask, const double* fin, int64_t x,
                       int64_t y, int64_t z, int i) {
  int64_t N = g->nx * g->ny * g->nz, sc;
  int sp;
  if (ora_source(g, L, mask, x, y, z, i, &sc, &sp))
    return fin[(int64_t)L->opp[i] * N + ora_cell(g, x, y, z)];
  return fin[(int64_t)sp * N + sc];
}

/* Inlet velocity at a cell for the state being produced at time index t:
 * u_in * (1 + noise * r), r uniform in [-1, 1) per component, drawn from
 * SplitMix64 with counter ((t * 2 + level) * N + cell) * 3 + component. */
static void ora_inlet_velocity(const ora_grid* g, int64_t cell, int64_t t,
                               double* u) {
  int64_t N = g->nx * g->ny * g->nz;
  /* one counter block per (time, level): time index times the level count
   * (at least 2) plus the level */
  uint64_t nl = g->levels > 2 ? (uint64_t)g->levels : 2u;
  int a;
  for (a = 0; a < 3; ++a) {
    uint64_t k = (((uint64_t)t * nl + (uint64_t)g->level) * (uint64_t)N +
                  (uint64_t)cell) * 3u + (uint64_t)a;
    double r = ora_uniform_pm1(ora_splitmix64(g->seed, k));
    u[a] = g->u_in[a] * (1.0 + g->inlet_noise * r);
  }
}

/* Initial post-collision state (the state streamed at t = 0):
 * f = f^{eqH}(rho, u) + (1 - 1/tau) f^{neqH}(a2_neq, u).
 * rho [N], u [3][N] (z ignored in 2D), pineq [6][N] (xx,yy,zz,xy,xz,yz);
 * a NULL field means rho0, the inlet velocity or zero. */
void ora_init(const ora_grid* g, const double* rho, const double* u,
              const double* pineq, double* f) {
  ora_lattice L;
  int64_t N = g->nx * g->ny * g->nz, c;
  if (ora_lattice_order(g->lattice, g->full_order, &L)) return;
#pragma omp parallel for schedule(static)
  for (c = 0; c < N; ++c) {
    double r = rho ? rho[c] : g->rho0, uu[3], p6[6] = {0, 0, 0, 0, 0, 0};
    double a2[3][3], E[27], Nq[27];
    int a, i;
    for (a = 0; a < 3; ++a) uu[a] = u ? u[(int64_t)a * N + c] : g->u_in[a];
    if (L.d == 2) uu[2] = 0.0;
    if (pineq)
      for (a = 0; a < 6; ++a) p6[a] = pineq[(int64_t)a * N + c];
    if (L.d == 2) p6[2] = p6[4] = p6[5] = 0.0;
    ora_unpack6(p6, a2);
    ora_feq(&L, r, uu, E);
    ora_fneq(&L, uu, a2, Nq);
    for (i = 0; i < L.q; ++i)
      f[(int64_t)i * N + c] = E[i] + (1.0 - 1.0 / g->tau) * Nq[i];
  }
}

/* Full update of the post-collision field from time t_new - 1 to t_new.
 * mask may be NULL (all fluid).  SOLID cells, and cells with skip[c] != 0
 * (skip may be NULL), are copied unchanged.  When rho_out / u_out / a2_out
 * are given, they receive the pre-collision moments rho*, u and a2_neq of
 * every collided cell (untouched elsewhere). */
void ora_step_ex(const ora_grid* g, const uint8_t* mask, const uint8_t* skip,
                 const double* fin, double* fout, int64_t t_new,
                 double* rho_out, double* u_out, double* a2_out) {
  ora_lattice L;
  int64_t N = g->nx * g->ny * g->nz, row;
  if (ora_lattice_order(g->lattice, g->full_order, &L)) return;
#pragma omp parallel for schedule(static)
  for (row = 0; row < g->ny * g->nz; ++row) {
    int64_t y = row % g->ny, z = row / g->ny, x;
    for (x = 0; x < g->nx; ++x) {
        int64_t c = ora_cell(g, x, y, z);
        uint8_t m = mask ? mask[c] : ORA_FLUID;
        double f[27], post[27];
        int i;
        if (m == ORA_SOLID || (skip && skip[c])) {
          for (i = 0; i < L.q; ++i)
            fout[(int64_t)i * N + c] = fin[(int64_t)i * N + c];
          continue;
        }
        if (m == ORA_INLET) {
          double uin[3];
          ora_inlet_velocity(g, c, t_new, uin);
          if (L.d == 2) uin[2] = 0.0;
          ora_feq(&L, g->rho0, uin, post);
        } else {
          double chi = g->sp_chi ? g->sp_chi[c] : ora_sponge_chi(g, x, y, z);
          double rref = g->sp_rho ? g->sp_rho[c] : g->rho_ref, uref[3];
          double rs, us[3], a2p[6];
          int a;
          for (a = 0; a < 3; ++a)
            uref[a] = g->sp_u ? g->sp_u[(int64_t)a * N + c] : g->u_ref[a];
          if (L.d == 2) uref[2] = 0.0;
          for (i = 0; i < L.q; ++i)
            f[i] = ora_pull(g, &L, mask, fin, x, y, z, i);
          if (g->collision == 1) {
            ora_collide_bgk(g->lattice, f, g->tau, chi, rref, uref, post);
            for (i = 0; i < L.q; ++i) fout[(int64_t)i * N + c] = post[i];
            continue; /* no moment record (comparators run unrefined) */
          }
          if (g->collision == 2) {
            /* Lallemand & Luo's rates for e, eps and q; s_nu = 1/tau */
            const double s4[4] = {1.64, 1.54, 1.9, 1.0 / g->tau};
            ora_collide_mrt(f, s4, post);
            for (i = 0; i < L.q; ++i) fout[(int64_t)i * N + c] = post[i];
            continue;
          }
          ora_collide_cell(&L, f, g->tau, chi, rref, uref, post, &rs, us, a2p);
          if (rho_out) rho_out[c] = rs;
          if (u_out)
            for (a = 0; a < 3; ++a) u_out[(int64_t)a * N + c] = us[a];
          if (a2_out)
            for (a = 0; a < 6; ++a) a2_out[(int64_t)a * N + c] = a2p[a];
        }
        for (i = 0; i < L.q; ++i) fout[(int64_t)i * N + c] = post[i];
    }
  }
}

void ora_step(const ora_grid* g, const uint8_t* mask, const double* fin,
              double* fout, int64_t t_new) {
  ora_step_ex(g, mask, NULL, fin, fout, t_new, NULL, NULL, NULL);
}

/* Force on all SOLID cells by momentum exchange (Ladd 1994; Mei, Yu, Shyy &
 * Luo 2002), from the post-collision state f at one time level: on every
 * bounced-back link of a FLUID cell x, the population f*_j(x) travelling
 * into the wall (xi_j = -xi_i for the pulled direction i) returns reversed
 * at the next step, so the wall receives 2 f*_j(x) xi_j.  F[3] receives the
 * sum over cells in index order and directions in lattice order. */
void ora_force(const ora_grid* g, const uint8_t* mask, const double* f,
               double* F) {
  ora_lattice L;
  int64_t N = g->nx * g->ny * g->nz, x, y, z;
  int a;
  F[0] = F[1] = F[2] = 0.0;
  if (!mask || ora_make_lattice(g->lattice, &L)) return;
  for (z = 0; z < g->nz; ++z)
    for (y = 0; y < g->ny; ++y)
      for (x = 0; x < g->nx; ++x) {
        int64_t c = ora_cell(g, x, y, z), sc;
        int i, sp;
        if (mask[c] != ORA_FLUID) continue;
        for (i = 1; i < L.q; ++i) {
          if (!ora_source(g, &L, mask, x, y, z, i, &sc, &sp)) continue;
          {
            int j = L.opp[i];
            double fj = f[(int64_t)j * N + c];
            for (a = 0; a < 3; ++a) F[a] += 2.0 * fj * L.xi[j][a];
          }
        }
      }
}

/* Density and velocity of the stored post-collision state at each cell:
 * rho = sum f, u = sum f xi / rho (eq. moments).  In cells without damping
 * the collision conserves both, so these equal the pre-collision moments of
 * the same time level.  SOLID cells report zero. */
void ora_moments(const ora_grid* g, const uint8_t* mask, const double* f,
                 double* rho_out, double* u_out) {
  ora_lattice L;
  int64_t N = g->nx * g->ny * g->nz, c;
  if (ora_make_lattice(g->lattice, &L)) return;
#pragma omp parallel for schedule(static)
  for (c = 0; c < N; ++c) {
    double r = 0, j[3] = {0, 0, 0};
    int i, a;
    if (mask && mask[c] == ORA_SOLID) {
      rho_out[c] = 0.0;
      for (a = 0; a < 3; ++a) u_out[(int64_t)a * N + c] = 0.0;
      continue;
    }
    for (i = 0; i < L.q; ++i) {
      double fi = f[(int64_t)i * N + c];
      r += fi;
      for (a = 0; a < 3; ++a) j[a] += fi * L.xi[i][a];
    }
    rho_out[c] = r;
    for (a = 0; a < 3; ++a) u_out[(int64_t)a * N + c] = j[a] / r;
  }
}

int ora_sizeof_grid(void) { return (int)sizeof(ora_grid); }

/* ------------------------------------------------------------------------ */
/* Two-level 2:1 multi-domain refinement (Sec. II.B).                        */
/*                                                                           */
/* Layout (the paper's Fig. 1 is not available; this is the reading used):   */
/* the fine grid covers the closed coarse-node box [lo, hi] with spacing 1/2 */
/* (eq. convective: dx_f = dx_c / 2, dt_f = dt_c / 2), so fine node k sits   */
/* at coarse coordinate lo + k/2 and an axis has 2 (hi - lo) + 1 fine nodes. */
/*   RING:    fine nodes on the outer shell; rebuilt from coarse data.       */
/*   IMPORT:  coarse nodes on the shell of [lo+1, hi-1]; rebuilt from fine   */
/*            data.                                                          */
/*   COVERED: coarse nodes strictly inside [lo+1, hi-1]; not updated.        */
/* ------------------------------------------------------------------------ */

typedef struct {
  ora_grid c; /* coarse grid (level 0) */
  ora_grid f; /* fine grid (level 1) */
  int64_t lo[3], hi[3];
} ora_refined;

enum { ORA_NORMAL = 0, ORA_IMPORT = 1, ORA_COVERED = 2 };

int ora_sizeof_refined(void) { return (int)sizeof(ora_refined); }

/* crole [Nc]: ORA_NORMAL / ORA_IMPORT / ORA_COVERED; fring [Nf]: 1 on RING */
void ora_ref_roles(const ora_refined* R, uint8_t* crole, uint8_t* fring) {
  const ora_grid* c = &R->c;
  const ora_grid* f = &R->f;
  int d = c->lattice == 9 ? 2 : 3;
  int64_t x, y, z;
  for (z = 0; z < c->nz; ++z)
    for (y = 0; y < c->ny; ++y)
      for (x = 0; x < c->nx; ++x) {
        int64_t p[3] = {x, y, z};
        int inside = 1, deep = 1, a;
        for (a = 0; a < d; ++a) {
          if (p[a] < R->lo[a] + 1 || p[a] > R->hi[a] - 1) inside = 0;
          if (p[a] < R->lo[a] + 2 || p[a] > R->hi[a] - 2) deep = 0;
        }
        crole[ora_cell(c, x, y, z)] =
            !inside ? ORA_NORMAL : (deep ? ORA_COVERED : ORA_IMPORT);
      }
  for (z = 0; z < f->nz; ++z)
    for (y = 0; y < f->ny; ++y)
      for (x = 0; x < f->nx; ++x) {
        int ring = (x == 0 || x == f->nx - 1 || y == 0 || y == f->ny - 1);
        if (d == 3) ring = ring || z == 0 || z == f->nz - 1;
        fring[ora_cell(f, x, y, z)] = (uint8_t)ring;
      }
}

/* Interpolation points along one axis for fine index k: the coincident
 * coarse node, or for a midpoint the local cubic (-1, 9, 9, -1)/16 over the
 * four nearest coarse nodes (Sec. II.B: at least cubic interpolation keeps
 * second order).  Returns the number of points. */
static int ora_axis_stencil(int64_t lo, int64_t k, int64_t n, int periodic,
                            int64_t* idx, double* wts) {
  if (k % 2 == 0) {
    idx[0] = lo + k / 2;
    wts[0] = 1.0;
    return 1;
  } else {
    const double w4[4] = {-1.0 / 16, 9.0 / 16, 9.0 / 16, -1.0 / 16};
    int64_t j = lo + (k - 1) / 2;
    int m;
    for (m = 0; m < 4; ++m) {
      int64_t s = j - 1 + m;
      if (periodic) s = (s % n + n) % n;
      idx[m] = s;
      wts[m] = w4[m];
    }
    return 4;
  }
}

/* Post-collision state of every RING node (eq. couplingFC): interpolated
 * rho~, u~ and Pi~_neq from the coarse pre-collision moments, blended in
 * time as wa * (level a) + wb * (level b) (linear interpolation in time,
 * Sec. II.B), then
 *   f = f^{eqH}(rho~, u~) + (1 - 1/tau_f) f^{neqH}(alpha_cf Pi~_neq, u~)
 * with alpha_cf = tau_f / (2 tau_c): the non-equilibrium stress scales
 * with tau * dt, the Chapman-Enskog leading order the paper invokes. */
void ora_ref_fill_ring(const ora_refined* R, const uint8_t* fring,
                       const double* rho_a, const double* u_a,
                       const double* a2_a, double wa, const double* rho_b,
                       const double* u_b, const double* a2_b, double wb,
                       double* ffine) {
  const ora_grid* c = &R->c;
  const ora_grid* f = &R->f;
  ora_lattice L;
  int64_t Nc = c->nx * c->ny * c->nz, Nf = f->nx * f->ny * f->nz, cf;
  const double alpha_cf = f->tau / (2.0 * c->tau);
  int d;
  if (ora_lattice_order(c->lattice, c->full_order, &L)) return;
  d = L.d;
#pragma omp parallel for schedule(static)
  for (cf = 0; cf < Nf; ++cf) {
    int64_t k[3], ix[3][4], cdims[3] = {c->nx, c->ny, c->nz};
    double wx[3][4], rho = 0, u[3] = {0, 0, 0}, p6[6] = {0, 0, 0, 0, 0, 0};
    double a2[3][3], E[27], Nq[27];
    int np[3], a, i, m0, m1, m2;
    if (!fring[cf]) continue;
    k[0] = cf % f->nx;
    k[1] = (cf / f->nx) % f->ny;
    k[2] = cf / (f->nx * f->ny);
    for (a = 0; a < 3; ++a) {
      if (a < d)
        np[a] = ora_axis_stencil(R->lo[a], k[a], cdims[a],
                                 c->face_bc[2 * a] == ORA_PERIODIC, ix[a], wx[a]);
      else {
        np[a] = 1;
        ix[a][0] = 0;
        wx[a][0] = 1.0;
      }
    }
    for (m2 = 0; m2 < np[2]; ++m2)
      for (m1 = 0; m1 < np[1]; ++m1)
        for (m0 = 0; m0 < np[0]; ++m0) {
          int64_t cc = ora_cell(c, ix[0][m0], ix[1][m1], ix[2][m2]);
          double w = wx[0][m0] * wx[1][m1] * wx[2][m2];
          rho += w * (wa * rho_a[cc] + wb * rho_b[cc]);
          for (a = 0; a < 3; ++a)
            u[a] += w * (wa * u_a[a * Nc + cc] + wb * u_b[a * Nc + cc]);
          for (a = 0; a < 6; ++a)
            p6[a] += w * (wa * a2_a[a * Nc + cc] + wb * a2_b[a * Nc + cc]);
        }
    for (a = 0; a < 6; ++a) p6[a] *= alpha_cf;
    if (d == 2) u[2] = p6[2] = p6[4] = p6[5] = 0.0;
    ora_unpack6(p6, a2);
    ora_feq(&L, rho, u, E);
    ora_fneq(&L, u, a2, Nq);
    for (i = 0; i < L.q; ++i)
      ffine[(int64_t)i * Nf + cf] = E[i] + (1.0 - 1.0 / f->tau) * Nq[i];
  }
}

/* Post-collision state of every IMPORT coarse node (eq. couplingCF): rho, u
 * copied from the coincident fine node; Pi_neq low-pass filtered with the
 * tensor weights (1/4, 1/2, 1/4) over the 3^D fine neighbours and rescaled
 * by alpha_fc = 2 tau_c / tau_f (only f_neq is filtered: Sec. II.B);
 *   f = f^{eqH}(rho, u) + (1 - 1/tau_c) f^{neqH}(alpha_fc Pi_neq, u).
 * rho_f, u_f, a2_f: fine pre-collision moments at the same time level. */
void ora_ref_import(const ora_refined* R, const uint8_t* crole,
                    const double* rho_f, const double* u_f, const double* a2_f,
                    double* fcoarse) {
  const ora_grid* c = &R->c;
  const ora_grid* f = &R->f;
  ora_lattice L;
  int64_t Nc = c->nx * c->ny * c->nz, Nf = f->nx * f->ny * f->nz, cc;
  const double alpha_fc = 2.0 * c->tau / f->tau;
  const double w1[3] = {0.25, 0.5, 0.25};
  if (ora_lattice_order(c->lattice, c->full_order, &L)) return;
#pragma omp parallel for schedule(static)
  for (cc = 0; cc < Nc; ++cc) {
    int64_t p[3], kc[3];
    double p6[6] = {0, 0, 0, 0, 0, 0}, u[3], rho, a2[3][3], E[27], Nq[27];
    int a, i, o0, o1, o2, oz = L.d == 3 ? 1 : 0;
    int64_t center;
    if (crole[cc] != ORA_IMPORT) continue;
    p[0] = cc % c->nx;
    p[1] = (cc / c->nx) % c->ny;
    p[2] = cc / (c->nx * c->ny);
    for (a = 0; a < 3; ++a) kc[a] = a < L.d ? 2 * (p[a] - R->lo[a]) : 0;
    center = ora_cell(f, kc[0], kc[1], kc[2]);
    rho = rho_f[center];
    for (a = 0; a < 3; ++a) u[a] = u_f[a * Nf + center];
    for (o2 = -oz; o2 <= oz; ++o2)
      for (o1 = -1; o1 <= 1; ++o1)
        for (o0 = -1; o0 <= 1; ++o0) {
          int64_t fc = ora_cell(f, kc[0] + o0, kc[1] + o1, kc[2] + o2);
          double w = w1[o0 + 1] * w1[o1 + 1] * (oz ? w1[o2 + 1] : 1.0);
          for (a = 0; a < 6; ++a) p6[a] += w * a2_f[a * Nf + fc];
        }
    for (a = 0; a < 6; ++a) p6[a] *= alpha_fc;
    if (L.d == 2) u[2] = p6[2] = p6[4] = p6[5] = 0.0;
    ora_unpack6(p6, a2);
    ora_feq(&L, rho, u, E);
    ora_fneq(&L, u, a2, Nq);
    for (i = 0; i < L.q; ++i)
      fcoarse[(int64_t)i * Nc + cc] = E[i] + (1.0 - 1.0 / c->tau) * Nq[i];
  }
}
