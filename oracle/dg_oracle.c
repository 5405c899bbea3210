/*
 * dg_oracle.c -- plain, slow, obviously correct CPU oracle for the matrix-free
 * weighted SIPG operator of Muething, Piatkowski & Bastian (arXiv 1711.10885).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only tests/, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or constant with the HIP
 * library.
 *
 * What it computes: y = A x with A_ij = a_h^Q(phi_j, phi_i), the bilinear form
 * of eq. (blf) in Sec. 2.2, with every volume and face integral replaced by the
 * tensor Gauss rule with m = k+1 points per direction (Problem A of Sec. 5.1
 * uses q = 2p, i.e. n = m = p+1).  Sum factorization (Sec. 3.5) is an exact
 * re-bracketing of these quadrature sums, so the oracle does NOT use it: at
 * every quadrature point the finite element function and its gradient are
 * evaluated by the full sum over all n^3 shape functions (eq. (evalfe) read
 * literally), and every test function is integrated point by point
 * (eq. (evalblf) read literally).  Cost O(n^3 m^3) per cell.
 *
 * Readings of the paper taken here (each listed in the design notes):
 *  - reference cube [0,1]^3, orthonormal Legendre basis
 *      theta_j(t) = sqrt(2j+1) P_j(2t-1)          (Sec. 2.2 "L2-orthogonal
 *      Legendre polynomials", Sec. 3.1 tensor product shape functions);
 *  - weighted average {v}_w = w- v- + w+ v+ (the printed minus sign in Sec. 2.2
 *    contradicts the convex weights given right after it);
 *  - penalty gamma_F = sigma * <delta-,delta+> / min(h_a-, h_a+) on interior
 *    faces (sigma absorbs alpha*p*(p+d-1); |F|/min|T| = 1/min h_a on a tensor
 *    grid), gamma_F = sigma * delta- / h_a- on boundary faces;
 *  - periodic axes (or_problem.periodic) join the first and last cells by an
 *    interior face, whose normal velocity is read at the axis' first node;
 *  - every other boundary face is homogeneous Dirichlet (g = 0), so the boundary
 *    upwind term is Phi(u,0,b_nu) (F^{DO} sum of eq. (blf)) and the boundary
 *    consistency/symmetry/penalty terms use [[v]] = {v} = v-;
 *  - D = kappa_T K with K constant SPD and kappa_T > 0 constant per cell;
 *  - b_r(x) = b_const[r] + b_sin[r] * sin(pi * x_{b_axis[r]}), or with
 *    or_problem.b_product the product form
 *    b_r(x) = b_amp[r] * prod_j sin(b_freq[3r+j] x_j + b_phase[3r+j]) (factors
 *    with b_freq == 0 are 1), which holds the Taylor-Green field of Sec. 5.4
 *    (eq. (2) of that section); b is evaluated at each quadrature point;
 *  - with or_problem.affine_on the mesh is the image x = A xi of the tensor
 *    grid of the nodes (affine geometry, Problem B of Sec. 5.1): gradients
 *    are A^{-T} times the tensor-grid gradients, volume and face measures
 *    scale by |det A| and |det A| |A^{-T} e_a|, face normals are
 *    A^{-T} e_a / |A^{-T} e_a|, d = nu^T D nu, and |F| / min|T| in gamma_F is
 *    |A^{-T} e_a| / min h_a; b is evaluated at physical points, the
 *    polynomial diffusion factor kp at the tensor-grid points xi (it is a
 *    polynomial in the grid coordinates of the affine cells);
 *  - every integral uses the tensor Gauss rule with m = k + 1 + quad_extra
 *    points per direction (quad_extra = 2 is the raised rule q = 2p + 4 of
 *    Problem B, Sec. 5.1; 0 the rule of Problem A);
 *  - with or_problem.multilinear_on the mesh is given by its vertices (a
 *    logically structured grid of (N1+1)(N2+1)(N3+1) points) and every cell
 *    is the image of [0,1]^3 under the trilinear (Q1) map through its eight
 *    vertices (multilinear geometry, Sec. 4 and Problem C of Sec. 5.1):
 *    gradients are J^{-T} times the reference gradients, with J the Jacobian
 *    of the map at the point; the volume weight is det J; a face xi_a = e has
 *    the area-weighted normal cof(J) e_a (|cof(J) e_a| is the surface measure,
 *    its direction the unit normal nu, both varying over the face); d = nu^T D
 *    nu, the weights and gamma_F are evaluated at each face point, with
 *    |F| / min(|T-|,|T+|) in gamma_F from the face area and the cell volumes
 *    (both integrated with the operator's rule); b and kp are evaluated at the
 *    physical point; no periodic axes;
 *  - with or_problem.kappa_poly_on the diffusion tensor is
 *    D(x) = kappa_T kp(x) K, kp(x) = prod_j (c_j0 + c_j1 x_j + c_j2 x_j^2)
 *    with c_ji = kappa_poly[3j+i] (coefficients polynomial in the
 *    coordinates, as in Problems B and C of Sec. 5.1); d = nu^T D nu, the
 *    weights and gamma_F are then evaluated at each face quadrature point.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXN 14 /* k <= 10; up to 13 Gauss points per direction */

typedef struct {
  int32_t ncell[3];
  const double *nodes[3]; /* length ncell[a]+1, strictly increasing */
  int32_t k;
  double K[9]; /* row-major, constant SPD */
  const double *kappa; /* per cell (axis-1 fastest) or NULL for 1 */
  double b_const[3];
  double b_sin[3];
  int32_t b_axis[3];
  double c;
  double sigma;
  int32_t periodic[3]; /* 1: axis a is periodic (first and last cells are neighbours) */
  int32_t b_product;   /* 1: b from b_amp, b_freq, b_phase below */
  double b_amp[3];
  double b_freq[9];
  double b_phase[9];
  int32_t kappa_poly_on; /* 1: D(x) = kappa_T kp(x) K, kp from kappa_poly */
  double kappa_poly[9];
  int32_t quad_extra;    /* Gauss points per direction m = k + 1 + quad_extra */
  int32_t affine_on;     /* 1: the mesh is the image x = A xi of the tensor grid xi */
  double affine[9];      /* A, row-major */
  int32_t multilinear_on; /* 1: trilinear cells through the vertices below */
  const double *vertices; /* (N1+1)(N2+1)(N3+1) x 3, vertex (v0,v1,v2) at v0 + (N1+1)(v1 + (N2+1) v2) */
} or_problem;

/* Geometry of the affine map x = A xi (identity unless affine_on): physical
 * gradients are A^{-T} times the gradients in xi; volumes scale by |det A|;
 * the face of a xi-cell normal to e_a has unit normal nu = A^{-T} e_a /
 * |A^{-T} e_a| and |det A| |A^{-T} e_a| area per unit xi-area, so that
 * |F| / |T| = |A^{-T} e_a| / h_a. */
typedef struct {
  double AiT[9]; /* A^{-T}, row-major */
  double det;    /* |det A| */
} or_geom;

static void geom_init(const or_problem *p, or_geom *G) {
  if (!p->affine_on) {
    for (int i = 0; i < 9; ++i) G->AiT[i] = (i % 4 == 0) ? 1.0 : 0.0;
    G->det = 1.0;
    return;
  }
  const double *A = p->affine;
  const double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8], c02 = A[3] * A[7] - A[4] * A[6];
  const double c10 = A[2] * A[7] - A[1] * A[8], c11 = A[0] * A[8] - A[2] * A[6], c12 = A[1] * A[6] - A[0] * A[7];
  const double c20 = A[1] * A[5] - A[2] * A[4], c21 = A[2] * A[3] - A[0] * A[5], c22 = A[0] * A[4] - A[1] * A[3];
  const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  /* A^{-1} = C^T / det (C the cofactor matrix), so A^{-T} = C / det */
  const double C[9] = {c00, c01, c02, c10, c11, c12, c20, c21, c22};
  for (int i = 0; i < 9; ++i) G->AiT[i] = C[i] / det;
  G->det = fabs(det);
}

/* g <- A^{-T} g */
static void geom_grad(const or_geom *G, double *g) {
  const double r0 = G->AiT[0] * g[0] + G->AiT[1] * g[1] + G->AiT[2] * g[2];
  const double r1 = G->AiT[3] * g[0] + G->AiT[4] * g[1] + G->AiT[5] * g[2];
  const double r2 = G->AiT[6] * g[0] + G->AiT[7] * g[1] + G->AiT[8] * g[2];
  g[0] = r0;
  g[1] = r1;
  g[2] = r2;
}

/* x <- A x (the physical point of a tensor-grid point) */
static void geom_point(const or_problem *p, double *x) {
  if (!p->affine_on) return;
  const double *A = p->affine;
  const double r0 = A[0] * x[0] + A[1] * x[1] + A[2] * x[2];
  const double r1 = A[3] * x[0] + A[4] * x[1] + A[5] * x[2];
  const double r2 = A[6] * x[0] + A[7] * x[1] + A[8] * x[2];
  x[0] = r0;
  x[1] = r1;
  x[2] = r2;
}

/* unit normal nu = A^{-T} e_a / |A^{-T} e_a|; returns |A^{-T} e_a| */
static double geom_normal(const or_geom *G, int a, double *nu) {
  const double v[3] = {G->AiT[a], G->AiT[3 + a], G->AiT[6 + a]};
  const double nrm = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  for (int r = 0; r < 3; ++r) nu[r] = v[r] / nrm;
  return nrm;
}

/* term mask for or_apply: which sums of eq. (blf) to include */
#define OR_VOLUME 1
#define OR_INTERIOR 2
#define OR_BOUNDARY 4

/* ------------------------------------------------------------------------ */
/* 1D building blocks                                                       */
/* ------------------------------------------------------------------------ */

/* Legendre polynomials P_0..P_k and their derivatives at s in [-1,1] by the
 * three-term recurrence (j+1) P_{j+1} = (2j+1) s P_j - j P_{j-1} and
 * P'_{j+1} = P'_{j-1} + (2j+1) P_j. */
static void legendre_all(int k, double s, double *P, double *dP) {
  P[0] = 1.0;
  dP[0] = 0.0;
  if (k >= 1) {
    P[1] = s;
    dP[1] = 1.0;
  }
  for (int j = 1; j < k; ++j) {
    P[j + 1] = ((2.0 * j + 1.0) * s * P[j] - j * P[j - 1]) / (j + 1.0);
    dP[j + 1] = dP[j - 1] + (2.0 * j + 1.0) * P[j];
  }
}

/* m-point Gauss-Legendre rule on [0,1] (Sec. 3.1, tensor Gauss quadrature):
 * nodes are the roots of P_m(2t-1), found by Newton's method; weights
 * 2/((1-s^2) P_m'(s)^2) on [-1,1], halved for [0,1].  Ascending order. */
int oracle_gauss(int m, double *xi, double *w) {
  if (m < 1 || m > 64) return -1;
  double P[66], dP[66];
  for (int i = 0; i < m; ++i) {
    /* root number i counted from s = +1 downwards */
    double s = cos(M_PI * (i + 0.75) / (m + 0.5));
    for (int it = 0; it < 100; ++it) {
      legendre_all(m, s, P, dP);
      double ds = P[m] / dP[m];
      s -= ds;
      if (fabs(ds) < 1e-16) break;
    }
    legendre_all(m, s, P, dP);
    double ws = 2.0 / ((1.0 - s * s) * dP[m] * dP[m]);
    /* store ascending in t = (1+s)/2 */
    xi[m - 1 - i] = 0.5 * (1.0 + s);
    w[m - 1 - i] = 0.5 * ws;
  }
  return 0;
}

/* Orthonormal Legendre basis on [0,1] and its derivative at t:
 * theta_j(t) = sqrt(2j+1) P_j(2t-1), theta_j'(t) = 2 sqrt(2j+1) P_j'(2t-1). */
void oracle_basis(int k, double t, double *val, double *der) {
  double P[OR_MAXN + 1], dP[OR_MAXN + 1];
  legendre_all(k, 2.0 * t - 1.0, P, dP);
  for (int j = 0; j <= k; ++j) {
    double sc = sqrt(2.0 * j + 1.0);
    val[j] = sc * P[j];
    der[j] = 2.0 * sc * dP[j];
  }
}

/* ------------------------------------------------------------------------ */
/* Per-problem tables                                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
  int n, m;
  double xi[OR_MAXN], w[OR_MAXN];
  double V[OR_MAXN][OR_MAXN]; /* V[q][j] = theta_j(xi_q)  */
  double D[OR_MAXN][OR_MAXN]; /* D[q][j] = theta_j'(xi_q) */
  double V0[OR_MAXN], V1[OR_MAXN]; /* theta_j(0), theta_j(1)   */
  double D0[OR_MAXN], D1[OR_MAXN]; /* theta_j'(0), theta_j'(1) */
} or_tables;

static void make_tables(int k, int extra, or_tables *t) {
  t->n = k + 1;
  t->m = k + 1 + extra;
  oracle_gauss(t->m, t->xi, t->w);
  for (int q = 0; q < t->m; ++q) oracle_basis(k, t->xi[q], t->V[q], t->D[q]);
  oracle_basis(k, 0.0, t->V0, t->D0);
  oracle_basis(k, 1.0, t->V1, t->D1);
}

static double coef_b(const or_problem *p, int r, const double *xp) {
  if (p->b_product) {
    double v = p->b_amp[r];
    for (int j = 0; j < 3; ++j)
      if (p->b_freq[3 * r + j] != 0.0) v *= sin(p->b_freq[3 * r + j] * xp[j] + p->b_phase[3 * r + j]);
    return v;
  }
  return p->b_const[r] + p->b_sin[r] * sin(M_PI * xp[p->b_axis[r]]);
}

/* The polynomial factor kp(x) of the diffusion tensor (1 when not used). */
static double coef_kp(const or_problem *p, const double *xp) {
  if (!p->kappa_poly_on) return 1.0;
  double v = 1.0;
  for (int j = 0; j < 3; ++j) {
    const double *c = p->kappa_poly + 3 * j;
    v *= c[0] + c[1] * xp[j] + c[2] * xp[j] * xp[j];
  }
  return v;
}

static double cell_kappa(const or_problem *p, int64_t c) {
  return p->kappa ? p->kappa[c] : 1.0;
}

static int64_t cell_id(const or_problem *p, const int *i) {
  return (int64_t)i[0] + (int64_t)p->ncell[0] * ((int64_t)i[1] + (int64_t)p->ncell[1] * i[2]);
}

static void cell_geom(const or_problem *p, const int *i, double *o, double *h) {
  for (int a = 0; a < 3; ++a) {
    o[a] = p->nodes[a][i[a]];
    h[a] = p->nodes[a][i[a] + 1] - p->nodes[a][i[a]];
  }
}

/* ------------------------------------------------------------------------ */
/* Volume term of eq. (blf):  (D grad u - b u, grad v)_T + (c u, v)_T       */
/* evaluated by the tensor Gauss rule (eq. (evalblf), eq. (gauss_points)).  */
/* ------------------------------------------------------------------------ */
static void volume_cell(const or_problem *p, const or_tables *t, const int *ic,
                        const double *xT, double *yT) {
  const int n = t->n, m = t->m;
  double o[3], h[3];
  cell_geom(p, ic, o, h);
  or_geom G;
  geom_init(p, &G);
  const double vol = h[0] * h[1] * h[2] * G.det;
  const double kap = cell_kappa(p, cell_id(p, ic));
  for (int q3 = 0; q3 < m; ++q3)
    for (int q2 = 0; q2 < m; ++q2)
      for (int q1 = 0; q1 < m; ++q1) {
        const int q[3] = {q1, q2, q3};
        /* u and its physical gradient at the point: full sum over shape
         * functions phi_j = theta_j1 theta_j2 theta_j3 (eq. (evalfe)). */
        double u = 0.0, g[3] = {0.0, 0.0, 0.0};
        for (int j3 = 0; j3 < n; ++j3)
          for (int j2 = 0; j2 < n; ++j2)
            for (int j1 = 0; j1 < n; ++j1) {
              const double xj = xT[j1 + n * (j2 + n * j3)];
              const double v1 = t->V[q1][j1], v2 = t->V[q2][j2], v3 = t->V[q3][j3];
              const double d1 = t->D[q1][j1], d2 = t->D[q2][j2], d3 = t->D[q3][j3];
              u += xj * v1 * v2 * v3;
              g[0] += xj * d1 * v2 * v3 / h[0];
              g[1] += xj * v1 * d2 * v3 / h[1];
              g[2] += xj * v1 * v2 * d3 / h[2];
            }
        geom_grad(&G, g);
        double xp[3];
        for (int a = 0; a < 3; ++a) xp[a] = o[a] + h[a] * t->xi[q[a]];
        /* kp is a polynomial in the tensor-grid coordinates (xi = x without an affine map) */
        const double kx = kap * coef_kp(p, xp); /* D = kx K at this point */
        geom_point(p, xp);
        double F[3];
        for (int r = 0; r < 3; ++r) {
          double s = 0.0;
          for (int c = 0; c < 3; ++c) s += kx * p->K[3 * r + c] * g[c];
          F[r] = s - coef_b(p, r, xp) * u;
        }
        const double W = t->w[q1] * t->w[q2] * t->w[q3] * vol;
        /* integrate against every test function */
        for (int j3 = 0; j3 < n; ++j3)
          for (int j2 = 0; j2 < n; ++j2)
            for (int j1 = 0; j1 < n; ++j1) {
              const double v1 = t->V[q1][j1], v2 = t->V[q2][j2], v3 = t->V[q3][j3];
              const double d1 = t->D[q1][j1], d2 = t->D[q2][j2], d3 = t->D[q3][j3];
              const double phi = v1 * v2 * v3;
              double gphi[3] = {d1 * v2 * v3 / h[0], v1 * d2 * v3 / h[1], v1 * v2 * d3 / h[2]};
              geom_grad(&G, gphi);
              yT[j1 + n * (j2 + n * j3)] +=
                  W * (F[0] * gphi[0] + F[1] * gphi[1] + F[2] * gphi[2] + p->c * u * phi);
            }
      }
}

/* Value and physical gradient of the shape function j of a cell at the face
 * point with reference coordinate e on axis a (e in {0,1}) and Gauss nodes
 * qt[0], qt[1] on the two tangential axes tb < tc. */
static void shape_on_face(const or_geom *G, const or_tables *t, int a, int e, int tb, int tc, int qb, int qc,
                          const int *j, const double *h, double *phi, double *gphi) {
  double val[3], der[3];
  val[a] = e ? t->V1[j[a]] : t->V0[j[a]];
  der[a] = e ? t->D1[j[a]] : t->D0[j[a]];
  val[tb] = t->V[qb][j[tb]];
  der[tb] = t->D[qb][j[tb]];
  val[tc] = t->V[qc][j[tc]];
  der[tc] = t->D[qc][j[tc]];
  *phi = val[0] * val[1] * val[2];
  gphi[0] = der[0] * val[1] * val[2] / h[0];
  gphi[1] = val[0] * der[1] * val[2] / h[1];
  gphi[2] = val[0] * val[1] * der[2] / h[2];
  geom_grad(G, gphi);
}

/* u and physical gradient of the FE function of one cell at a face point */
static void eval_on_face(const or_geom *G, const or_tables *t, int a, int e, int tb, int tc, int qb, int qc,
                         const double *h, const double *xT, double *u, double *g) {
  const int n = t->n;
  *u = 0.0;
  g[0] = g[1] = g[2] = 0.0;
  for (int j3 = 0; j3 < n; ++j3)
    for (int j2 = 0; j2 < n; ++j2)
      for (int j1 = 0; j1 < n; ++j1) {
        const int j[3] = {j1, j2, j3};
        double phi, gphi[3];
        shape_on_face(G, t, a, e, tb, tc, qb, qc, j, h, &phi, gphi);
        const double xj = xT[j1 + n * (j2 + n * j3)];
        *u += xj * phi;
        for (int r = 0; r < 3; ++r) g[r] += xj * gphi[r];
      }
}

/* ------------------------------------------------------------------------ */
/* Interior face F between Tm = T^-(F) (index i_a) and Tp = T^+(F) (index    */
/* i_a+1), normal nu = +e_a (Sec. 2.2).  Terms of eq. (blf):                 */
/*   (Phi(u-,u+,b.nu), [[v]])_F - (nu.{D grad u}_w, [[v]])_F                 */
/*   - (nu.{D grad v}_w, [[u]])_F + gamma_F ([[u]], [[v]])_F                 */
/* with [[v]] = v- - v+, {v}_w = w- v- + w+ v+, w- = d+/(d-+d+),              */
/* w+ = d-/(d-+d+), d = nu^T D nu, gamma_F = sigma <d-,d+> / min(h_a-,h_a+),  */
/* Phi = u- b.nu if b.nu >= 0 else u+ b.nu.                                  */
/* Contributions are added to ym (rows of Tm) if ym != NULL and to yp (rows  */
/* of Tp) if yp != NULL.                                                     */
/* ------------------------------------------------------------------------ */
static void interior_face(const or_problem *p, const or_tables *t, int a, const int *im,
                          const double *xm, const double *xp_, double *ym, double *yp) {
  const int n = t->n, m = t->m;
  const int tb = (a == 0) ? 1 : 0, tc = (a == 2) ? 1 : 2;
  int ip[3] = {im[0], im[1], im[2]};
  ip[a] += 1;
  if (ip[a] == p->ncell[a]) ip[a] = 0; /* periodic axis: the face across the domain boundary */
  double om[3], hm[3], op[3], hp[3];
  cell_geom(p, im, om, hm);
  cell_geom(p, ip, op, hp);
  const double km = cell_kappa(p, cell_id(p, im)), kp = cell_kappa(p, cell_id(p, ip));
  /* unit normal nu from T^- to T^+, nu^T K and nu^T K nu; |F| / |T| = nrm / h_a */
  or_geom G;
  geom_init(p, &G);
  double nu[3], nK[3];
  const double nrm = geom_normal(&G, a, nu);
  for (int s2 = 0; s2 < 3; ++s2) nK[s2] = nu[0] * p->K[s2] + nu[1] * p->K[3 + s2] + nu[2] * p->K[6 + s2];
  const double Knn = nK[0] * nu[0] + nK[1] * nu[1] + nK[2] * nu[2];
  const double hmin = hm[a] < hp[a] ? hm[a] : hp[a];
  const double area = hm[tb] * hm[tc] * G.det * nrm;
  for (int qc = 0; qc < m; ++qc)
    for (int qb = 0; qb < m; ++qb) {
      double um, gm[3], up, gp[3];
      eval_on_face(&G, t, a, 1, tb, tc, qb, qc, hm, xm, &um, gm);
      eval_on_face(&G, t, a, 0, tb, tc, qb, qc, hp, xp_, &up, gp);
      /* physical face point (on the plane x_a = node) */
      double X[3];
      X[a] = op[a];
      X[tb] = om[tb] + hm[tb] * t->xi[qb];
      X[tc] = om[tc] + hm[tc] * t->xi[qc];
      const double kpoly = coef_kp(p, X); /* at the tensor-grid point */
      geom_point(p, X);
      const double bnu = coef_b(p, 0, X) * nu[0] + coef_b(p, 1, X) * nu[1] + coef_b(p, 2, X) * nu[2];
      const double Phi = (bnu >= 0.0) ? bnu * um : bnu * up;
      const double J = um - up;
      /* D^- = kmx K, D^+ = kpx K at the point; d, the weights and gamma there */
      const double kmx = km * kpoly, kpx = kp * kpoly;
      const double dmx = kmx * Knn, dpx = kpx * Knn;
      const double wmx = dpx / (dmx + dpx), wpx = dmx / (dmx + dpx);
      const double gammax = p->sigma * (2.0 * dmx * dpx / (dmx + dpx)) * nrm / hmin;
      double Dgm = 0.0, Dgp = 0.0; /* nu . (D grad u^-), nu . (D grad u^+) */
      for (int s = 0; s < 3; ++s) {
        Dgm += kmx * nK[s] * gm[s];
        Dgp += kpx * nK[s] * gp[s];
      }
      const double avg = wmx * Dgm + wpx * Dgp;
      const double W = t->w[qb] * t->w[qc] * area;
      for (int j3 = 0; j3 < n; ++j3)
        for (int j2 = 0; j2 < n; ++j2)
          for (int j1 = 0; j1 < n; ++j1) {
            const int j[3] = {j1, j2, j3};
            const int jj = j1 + n * (j2 + n * j3);
            if (ym) {
              /* test function on T^-: [[v]] = v, {D grad v}_w = w- D- grad v */
              double phi, gphi[3];
              shape_on_face(&G, t, a, 1, tb, tc, qb, qc, j, hm, &phi, gphi);
              double Dgv = 0.0;
              for (int s = 0; s < 3; ++s) Dgv += kmx * nK[s] * gphi[s];
              ym[jj] += W * (Phi * phi - avg * phi - wmx * Dgv * J + gammax * J * phi);
            }
            if (yp) {
              /* test function on T^+: [[v]] = -v, {D grad v}_w = w+ D+ grad v */
              double phi, gphi[3];
              shape_on_face(&G, t, a, 0, tb, tc, qb, qc, j, hp, &phi, gphi);
              double Dgv = 0.0;
              for (int s = 0; s < 3; ++s) Dgv += kpx * nK[s] * gphi[s];
              yp[jj] += W * (-Phi * phi + avg * phi - wpx * Dgv * J - gammax * J * phi);
            }
          }
    }
}

/* ------------------------------------------------------------------------ */
/* Boundary face of cell T on the side e (0: x_a = lower end, 1: upper) of    */
/* axis a; outer normal nu = (2e-1) e_a.  Homogeneous Dirichlet: terms       */
/*   (Phi(u,0,b.nu), v)_F - (nu.D grad u, v)_F - (nu.D grad v, u)_F           */
/*   + gamma_F (u, v)_F,    gamma_F = sigma d- / h_a,  d- = nu^T D nu.        */
/* ------------------------------------------------------------------------ */
static void boundary_face(const or_problem *p, const or_tables *t, int a, int e, const int *ic,
                          const double *xT, double *yT) {
  const int n = t->n, m = t->m;
  const int tb = (a == 0) ? 1 : 0, tc = (a == 2) ? 1 : 2;
  double o[3], h[3];
  cell_geom(p, ic, o, h);
  const double kap = cell_kappa(p, cell_id(p, ic));
  const double nsign = e ? 1.0 : -1.0;
  /* nu = nsign A^{-T} e_a / |A^{-T} e_a| (outer); nK = nu^T K up to the sign */
  or_geom G;
  geom_init(p, &G);
  double nu[3], nK[3];
  const double nrm = geom_normal(&G, a, nu);
  for (int s2 = 0; s2 < 3; ++s2) nK[s2] = nu[0] * p->K[s2] + nu[1] * p->K[3 + s2] + nu[2] * p->K[6 + s2];
  const double Knn = nK[0] * nu[0] + nK[1] * nu[1] + nK[2] * nu[2];
  const double area = h[tb] * h[tc] * G.det * nrm;
  for (int qc = 0; qc < m; ++qc)
    for (int qb = 0; qb < m; ++qb) {
      double u, g[3];
      eval_on_face(&G, t, a, e, tb, tc, qb, qc, h, xT, &u, g);
      double X[3];
      X[a] = o[a] + (e ? h[a] : 0.0);
      X[tb] = o[tb] + h[tb] * t->xi[qb];
      X[tc] = o[tc] + h[tc] * t->xi[qc];
      const double kx = kap * coef_kp(p, X); /* D = kx K at the point (kp at the tensor-grid point) */
      geom_point(p, X);
      const double bnu = nsign * (coef_b(p, 0, X) * nu[0] + coef_b(p, 1, X) * nu[1] + coef_b(p, 2, X) * nu[2]);
      const double Phi = (bnu >= 0.0) ? bnu * u : 0.0;
      const double gammax = p->sigma * kx * Knn * nrm / h[a];
      double Dg = 0.0;
      for (int s = 0; s < 3; ++s) Dg += kx * nK[s] * g[s];
      Dg *= nsign;
      const double W = t->w[qb] * t->w[qc] * area;
      for (int j3 = 0; j3 < n; ++j3)
        for (int j2 = 0; j2 < n; ++j2)
          for (int j1 = 0; j1 < n; ++j1) {
            const int j[3] = {j1, j2, j3};
            double phi, gphi[3];
            shape_on_face(&G, t, a, e, tb, tc, qb, qc, j, h, &phi, gphi);
            double Dgv = 0.0;
            for (int s = 0; s < 3; ++s) Dgv += kx * nK[s] * gphi[s];
            Dgv *= nsign;
            yT[j1 + n * (j2 + n * j3)] += W * (Phi * phi - Dg * phi - Dgv * u + gammax * u * phi);
          }
    }
}

/* ------------------------------------------------------------------------ */
/* Multilinear geometry (Sec. 4: the map mu_T from the reference cube to the */
/* cell is a Q1 finite element function; Problem C of Sec. 5.1).  The same   */
/* terms of eq. (blf) as above, with the geometry taken point by point.      */
/* ------------------------------------------------------------------------ */

static const double *ml_vertex(const or_problem *p, int v0, int v1, int v2) {
  const int64_t V0 = p->ncell[0] + 1, V1 = p->ncell[1] + 1;
  return p->vertices + 3 * ((int64_t)v0 + V0 * ((int64_t)v1 + V1 * v2));
}

/* X = mu_T(xi) and J[3r+s] = d X_r / d xi_s for the cell ic:
 *   mu_T(xi) = sum over the corners c in {0,1}^3 of the vertex X_c times
 *   l_{c0}(xi_0) l_{c1}(xi_1) l_{c2}(xi_2),   l_0(t) = 1 - t,  l_1(t) = t. */
static void ml_map(const or_problem *p, const int *ic, const double *xi, double *X, double *J) {
  for (int r = 0; r < 3; ++r) {
    X[r] = 0.0;
    for (int s2 = 0; s2 < 3; ++s2) J[3 * r + s2] = 0.0;
  }
  for (int c = 0; c < 8; ++c) {
    const int cb[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
    const double *V = ml_vertex(p, ic[0] + cb[0], ic[1] + cb[1], ic[2] + cb[2]);
    double l[3], dl[3];
    for (int a = 0; a < 3; ++a) {
      l[a] = cb[a] ? xi[a] : 1.0 - xi[a];
      dl[a] = cb[a] ? 1.0 : -1.0;
    }
    const double wv = l[0] * l[1] * l[2];
    const double wd[3] = {dl[0] * l[1] * l[2], l[0] * dl[1] * l[2], l[0] * l[1] * dl[2]};
    for (int r = 0; r < 3; ++r) {
      X[r] += wv * V[r];
      for (int s2 = 0; s2 < 3; ++s2) J[3 * r + s2] += wd[s2] * V[r];
    }
  }
}

/* Cofactor matrix C = det(J) J^{-T} (row-major); returns det J.  Physical
 * gradients are C g_ref / det J; column a of C is the area-weighted normal of
 * the surfaces xi_a = const (pointing towards increasing xi_a when det J > 0). */
static double ml_cof(const double *J, double *C) {
  C[0] = J[4] * J[8] - J[5] * J[7];
  C[1] = J[5] * J[6] - J[3] * J[8];
  C[2] = J[3] * J[7] - J[4] * J[6];
  C[3] = J[2] * J[7] - J[1] * J[8];
  C[4] = J[0] * J[8] - J[2] * J[6];
  C[5] = J[1] * J[6] - J[0] * J[7];
  C[6] = J[1] * J[5] - J[2] * J[4];
  C[7] = J[2] * J[3] - J[0] * J[5];
  C[8] = J[0] * J[4] - J[1] * J[3];
  return J[0] * C[0] + J[1] * C[1] + J[2] * C[2];
}

/* g <- C g / det */
static void ml_grad(const double *C, double det, double *g) {
  const double r0 = (C[0] * g[0] + C[1] * g[1] + C[2] * g[2]) / det;
  const double r1 = (C[3] * g[0] + C[4] * g[1] + C[5] * g[2]) / det;
  const double r2 = (C[6] * g[0] + C[7] * g[1] + C[8] * g[2]) / det;
  g[0] = r0;
  g[1] = r1;
  g[2] = r2;
}

/* |T|: det J integrated over the reference cube with the operator's rule
 * (exact: det J is a polynomial of degree <= 2 in each coordinate). */
static double ml_cell_volume(const or_problem *p, const or_tables *t, const int *ic) {
  double v = 0.0;
  for (int q3 = 0; q3 < t->m; ++q3)
    for (int q2 = 0; q2 < t->m; ++q2)
      for (int q1 = 0; q1 < t->m; ++q1) {
        const double xi[3] = {t->xi[q1], t->xi[q2], t->xi[q3]};
        double X[3], J[9], C[9];
        ml_map(p, ic, xi, X, J);
        v += t->w[q1] * t->w[q2] * t->w[q3] * ml_cof(J, C);
      }
  return v;
}

/* |F| of the face xi_a = e of cell ic: |cof(J) e_a| integrated over the face
 * with the operator's rule on the tangential axes tb < tc. */
static double ml_face_area(const or_problem *p, const or_tables *t, const int *ic, int a, int e) {
  const int tb = (a == 0) ? 1 : 0, tc = (a == 2) ? 1 : 2;
  double A = 0.0;
  for (int qc = 0; qc < t->m; ++qc)
    for (int qb = 0; qb < t->m; ++qb) {
      double xi[3], X[3], J[9], C[9];
      xi[a] = e ? 1.0 : 0.0;
      xi[tb] = t->xi[qb];
      xi[tc] = t->xi[qc];
      ml_map(p, ic, xi, X, J);
      ml_cof(J, C);
      A += t->w[qb] * t->w[qc] * sqrt(C[a] * C[a] + C[3 + a] * C[3 + a] + C[6 + a] * C[6 + a]);
    }
  return A;
}

static void ml_volume_cell(const or_problem *p, const or_tables *t, const int *ic, const double *xT, double *yT) {
  const int n = t->n, m = t->m;
  const double kap = cell_kappa(p, cell_id(p, ic));
  for (int q3 = 0; q3 < m; ++q3)
    for (int q2 = 0; q2 < m; ++q2)
      for (int q1 = 0; q1 < m; ++q1) {
        const double xi[3] = {t->xi[q1], t->xi[q2], t->xi[q3]};
        double X[3], J[9], C[9];
        ml_map(p, ic, xi, X, J);
        const double det = ml_cof(J, C);
        /* u and its physical gradient: full sum over the shape functions */
        double u = 0.0, g[3] = {0.0, 0.0, 0.0};
        for (int j3 = 0; j3 < n; ++j3)
          for (int j2 = 0; j2 < n; ++j2)
            for (int j1 = 0; j1 < n; ++j1) {
              const double xj = xT[j1 + n * (j2 + n * j3)];
              const double v1 = t->V[q1][j1], v2 = t->V[q2][j2], v3 = t->V[q3][j3];
              u += xj * v1 * v2 * v3;
              g[0] += xj * t->D[q1][j1] * v2 * v3;
              g[1] += xj * v1 * t->D[q2][j2] * v3;
              g[2] += xj * v1 * v2 * t->D[q3][j3];
            }
        ml_grad(C, det, g);
        const double kx = kap * coef_kp(p, X);
        double F[3];
        for (int r = 0; r < 3; ++r) {
          double sum = 0.0;
          for (int c = 0; c < 3; ++c) sum += kx * p->K[3 * r + c] * g[c];
          F[r] = sum - coef_b(p, r, X) * u;
        }
        const double W = t->w[q1] * t->w[q2] * t->w[q3] * det;
        for (int j3 = 0; j3 < n; ++j3)
          for (int j2 = 0; j2 < n; ++j2)
            for (int j1 = 0; j1 < n; ++j1) {
              const double v1 = t->V[q1][j1], v2 = t->V[q2][j2], v3 = t->V[q3][j3];
              double gphi[3] = {t->D[q1][j1] * v2 * v3, v1 * t->D[q2][j2] * v3, v1 * v2 * t->D[q3][j3]};
              ml_grad(C, det, gphi);
              yT[j1 + n * (j2 + n * j3)] +=
                  W * (F[0] * gphi[0] + F[1] * gphi[1] + F[2] * gphi[2] + p->c * u * v1 * v2 * v3);
            }
      }
}

/* Value and physical gradient of shape function j of a cell at its face
 * point (xi_a = e, Gauss nodes qb, qc on the tangential axes tb < tc), from
 * the cell's cofactor matrix C and det J at that point. */
static void ml_shape_on_face(const or_tables *t, int a, int e, int tb, int tc, int qb, int qc, const int *j,
                             const double *C, double det, double *phi, double *gphi) {
  double val[3], der[3];
  val[a] = e ? t->V1[j[a]] : t->V0[j[a]];
  der[a] = e ? t->D1[j[a]] : t->D0[j[a]];
  val[tb] = t->V[qb][j[tb]];
  der[tb] = t->D[qb][j[tb]];
  val[tc] = t->V[qc][j[tc]];
  der[tc] = t->D[qc][j[tc]];
  *phi = val[0] * val[1] * val[2];
  gphi[0] = der[0] * val[1] * val[2];
  gphi[1] = val[0] * der[1] * val[2];
  gphi[2] = val[0] * val[1] * der[2];
  ml_grad(C, det, gphi);
}

static void ml_eval_on_face(const or_tables *t, int a, int e, int tb, int tc, int qb, int qc, const double *C,
                            double det, const double *xT, double *u, double *g) {
  const int n = t->n;
  *u = 0.0;
  g[0] = g[1] = g[2] = 0.0;
  for (int j3 = 0; j3 < n; ++j3)
    for (int j2 = 0; j2 < n; ++j2)
      for (int j1 = 0; j1 < n; ++j1) {
        const int j[3] = {j1, j2, j3};
        double phi, gphi[3];
        ml_shape_on_face(t, a, e, tb, tc, qb, qc, j, C, det, &phi, gphi);
        const double xj = xT[j1 + n * (j2 + n * j3)];
        *u += xj * phi;
        for (int r = 0; r < 3; ++r) g[r] += xj * gphi[r];
      }
}

/* Interior face between Tm (index i_a) and Tp (index i_a + 1): the face
 * xi_a = 1 of Tm and xi_a = 0 of Tp, with the same tangential coordinates
 * (the two trilinear maps agree on the shared face).  nu points from Tm to
 * Tp; the face point, b and kp are taken from Tm's map. */
static void ml_interior_face(const or_problem *p, const or_tables *t, int a, const int *im, const double *xm,
                             const double *xp_, double *ym, double *yp) {
  const int n = t->n, m = t->m;
  const int tb = (a == 0) ? 1 : 0, tc = (a == 2) ? 1 : 2;
  int ip[3] = {im[0], im[1], im[2]};
  ip[a] += 1;
  const double km = cell_kappa(p, cell_id(p, im)), kp = cell_kappa(p, cell_id(p, ip));
  const double volm = ml_cell_volume(p, t, im), volp = ml_cell_volume(p, t, ip);
  const double FoT = ml_face_area(p, t, im, a, 1) / (volm < volp ? volm : volp);
  for (int qc = 0; qc < m; ++qc)
    for (int qb = 0; qb < m; ++qb) {
      double xim[3], xip[3];
      xim[a] = 1.0;
      xip[a] = 0.0;
      xim[tb] = xip[tb] = t->xi[qb];
      xim[tc] = xip[tc] = t->xi[qc];
      double Xm[3], Jm[9], Cm[9], Xp[3], Jp[9], Cp[9];
      ml_map(p, im, xim, Xm, Jm);
      ml_map(p, ip, xip, Xp, Jp);
      const double detm = ml_cof(Jm, Cm), detp = ml_cof(Jp, Cp);
      const double nv[3] = {Cm[a], Cm[3 + a], Cm[6 + a]};
      const double nrm = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
      const double nu[3] = {nv[0] / nrm, nv[1] / nrm, nv[2] / nrm};
      double nK[3];
      for (int s2 = 0; s2 < 3; ++s2) nK[s2] = nu[0] * p->K[s2] + nu[1] * p->K[3 + s2] + nu[2] * p->K[6 + s2];
      const double Knn = nK[0] * nu[0] + nK[1] * nu[1] + nK[2] * nu[2];
      double um, gm[3], up, gp[3];
      ml_eval_on_face(t, a, 1, tb, tc, qb, qc, Cm, detm, xm, &um, gm);
      ml_eval_on_face(t, a, 0, tb, tc, qb, qc, Cp, detp, xp_, &up, gp);
      const double kpoly = coef_kp(p, Xm);
      const double bnu = coef_b(p, 0, Xm) * nu[0] + coef_b(p, 1, Xm) * nu[1] + coef_b(p, 2, Xm) * nu[2];
      const double Phi = (bnu >= 0.0) ? bnu * um : bnu * up;
      const double J = um - up;
      const double kmx = km * kpoly, kpx = kp * kpoly;
      const double dmx = kmx * Knn, dpx = kpx * Knn;
      const double wmx = dpx / (dmx + dpx), wpx = dmx / (dmx + dpx);
      const double gammax = p->sigma * (2.0 * dmx * dpx / (dmx + dpx)) * FoT;
      double Dgm = 0.0, Dgp = 0.0;
      for (int s2 = 0; s2 < 3; ++s2) {
        Dgm += kmx * nK[s2] * gm[s2];
        Dgp += kpx * nK[s2] * gp[s2];
      }
      const double avg = wmx * Dgm + wpx * Dgp;
      const double W = t->w[qb] * t->w[qc] * nrm;
      for (int j3 = 0; j3 < n; ++j3)
        for (int j2 = 0; j2 < n; ++j2)
          for (int j1 = 0; j1 < n; ++j1) {
            const int j[3] = {j1, j2, j3};
            const int jj = j1 + n * (j2 + n * j3);
            if (ym) {
              double phi, gphi[3];
              ml_shape_on_face(t, a, 1, tb, tc, qb, qc, j, Cm, detm, &phi, gphi);
              double Dgv = 0.0;
              for (int s2 = 0; s2 < 3; ++s2) Dgv += kmx * nK[s2] * gphi[s2];
              ym[jj] += W * (Phi * phi - avg * phi - wmx * Dgv * J + gammax * J * phi);
            }
            if (yp) {
              double phi, gphi[3];
              ml_shape_on_face(t, a, 0, tb, tc, qb, qc, j, Cp, detp, &phi, gphi);
              double Dgv = 0.0;
              for (int s2 = 0; s2 < 3; ++s2) Dgv += kpx * nK[s2] * gphi[s2];
              yp[jj] += W * (-Phi * phi + avg * phi - wpx * Dgv * J - gammax * J * phi);
            }
          }
    }
}

/* Boundary face xi_a = e of cell ic (homogeneous Dirichlet); outer
 * area-weighted normal (2e - 1) cof(J) e_a; gamma_F = sigma d |F| / |T|. */
static void ml_boundary_face(const or_problem *p, const or_tables *t, int a, int e, const int *ic, const double *xT,
                             double *yT) {
  const int n = t->n, m = t->m;
  const int tb = (a == 0) ? 1 : 0, tc = (a == 2) ? 1 : 2;
  const double kap = cell_kappa(p, cell_id(p, ic));
  const double nsign = e ? 1.0 : -1.0;
  const double FoT = ml_face_area(p, t, ic, a, e) / ml_cell_volume(p, t, ic);
  for (int qc = 0; qc < m; ++qc)
    for (int qb = 0; qb < m; ++qb) {
      double xi[3], X[3], J[9], C[9];
      xi[a] = e ? 1.0 : 0.0;
      xi[tb] = t->xi[qb];
      xi[tc] = t->xi[qc];
      ml_map(p, ic, xi, X, J);
      const double det = ml_cof(J, C);
      const double nv[3] = {nsign * C[a], nsign * C[3 + a], nsign * C[6 + a]};
      const double nrm = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
      const double nu[3] = {nv[0] / nrm, nv[1] / nrm, nv[2] / nrm};
      double nK[3];
      for (int s2 = 0; s2 < 3; ++s2) nK[s2] = nu[0] * p->K[s2] + nu[1] * p->K[3 + s2] + nu[2] * p->K[6 + s2];
      const double Knn = nK[0] * nu[0] + nK[1] * nu[1] + nK[2] * nu[2];
      double u, g[3];
      ml_eval_on_face(t, a, e, tb, tc, qb, qc, C, det, xT, &u, g);
      const double kx = kap * coef_kp(p, X);
      const double bnu = coef_b(p, 0, X) * nu[0] + coef_b(p, 1, X) * nu[1] + coef_b(p, 2, X) * nu[2];
      const double Phi = (bnu >= 0.0) ? bnu * u : 0.0;
      const double gammax = p->sigma * kx * Knn * FoT;
      double Dg = 0.0;
      for (int s2 = 0; s2 < 3; ++s2) Dg += kx * nK[s2] * g[s2];
      const double W = t->w[qb] * t->w[qc] * nrm;
      for (int j3 = 0; j3 < n; ++j3)
        for (int j2 = 0; j2 < n; ++j2)
          for (int j1 = 0; j1 < n; ++j1) {
            const int j[3] = {j1, j2, j3};
            double phi, gphi[3];
            ml_shape_on_face(t, a, e, tb, tc, qb, qc, j, C, det, &phi, gphi);
            double Dgv = 0.0;
            for (int s2 = 0; s2 < 3; ++s2) Dgv += kx * nK[s2] * gphi[s2];
            yT[j1 + n * (j2 + n * j3)] += W * (Phi * phi - Dg * phi - Dgv * u + gammax * u * phi);
          }
    }
}

static int check_problem(const or_problem *p) {
  if (!p || p->k < 1 || p->k > 10) return -1;
  if (p->quad_extra < 0 || p->k + 1 + p->quad_extra > OR_MAXN - 1) return -1;
  if (p->multilinear_on && (!p->vertices || p->affine_on)) return -1;
  for (int a = 0; a < 3; ++a) {
    if (p->ncell[a] < 1 || (!p->nodes[a] && !p->multilinear_on)) return -1;
    if (p->b_axis[a] < 0 || p->b_axis[a] > 2) return -1;
    if (p->multilinear_on && p->periodic[a]) return -1;
  }
  return 0;
}

int64_t oracle_ndof(const or_problem *p) {
  const int64_t n = p->k + 1;
  return (int64_t)p->ncell[0] * p->ncell[1] * p->ncell[2] * n * n * n;
}

/* ------------------------------------------------------------------------ */
/* y = A x, Algorithm 1 of Sec. 3.6: volume per cell, every interior face    */
/* once with its result scattered to both neighbours, every boundary face.   */
/* Faces are visited in two passes per axis (even and odd lower index), so   */
/* that faces processed concurrently never share a cell.                     */
/* ------------------------------------------------------------------------ */
typedef void (*or_iface_fn)(const or_problem *, const or_tables *, int, const int *, const double *,
                            const double *, double *, double *);
typedef void (*or_bface_fn)(const or_problem *, const or_tables *, int, int, const int *, const double *, double *);

int oracle_apply(const or_problem *p, const double *x, double *y, int terms, int nthreads) {
  if (check_problem(p)) return -1;
  const or_bface_fn bface = p->multilinear_on ? ml_boundary_face : boundary_face;
  or_tables t;
  make_tables(p->k, p->quad_extra, &t);
  const int64_t nb = (int64_t)t.n * t.n * t.n;
  const int N1 = p->ncell[0], N2 = p->ncell[1], N3 = p->ncell[2];
  const int64_t ncells = (int64_t)N1 * N2 * N3;
  if (nthreads <= 0) nthreads = 1;
  memset(y, 0, sizeof(double) * ncells * nb);
  if (terms & OR_VOLUME) {
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
    for (int64_t c = 0; c < ncells; ++c) {
      const int ic[3] = {(int)(c % N1), (int)((c / N1) % N2), (int)(c / ((int64_t)N1 * N2))};
      if (p->multilinear_on)
        ml_volume_cell(p, &t, ic, x + c * nb, y + c * nb);
      else
        volume_cell(p, &t, ic, x + c * nb, y + c * nb);
    }
  }
  if (terms & OR_INTERIOR) {
    /* pass 2 takes the faces across a periodic boundary (last cell to the
     * first); they would share cells with pass 0 or 1 when ncell is odd */
    for (int a = 0; a < 3; ++a)
      for (int parity = 0; parity < 3; ++parity) {
        if (parity == 2 && !p->periodic[a]) continue;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
        for (int64_t c = 0; c < ncells; ++c) {
          const int ic[3] = {(int)(c % N1), (int)((c / N1) % N2), (int)(c / ((int64_t)N1 * N2))};
          if (parity == 2) {
            if (ic[a] != p->ncell[a] - 1) continue;
          } else if (ic[a] % 2 != parity || ic[a] + 1 >= p->ncell[a]) {
            continue;
          }
          int jc[3] = {ic[0], ic[1], ic[2]};
          jc[a] = (ic[a] + 1) % p->ncell[a];
          const int64_t cp = cell_id(p, jc);
          if (p->multilinear_on)
            ml_interior_face(p, &t, a, ic, x + c * nb, x + cp * nb, y + c * nb, y + cp * nb);
          else
            interior_face(p, &t, a, ic, x + c * nb, x + cp * nb, y + c * nb, y + cp * nb);
        }
      }
  }
  if (terms & OR_BOUNDARY) {
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
    for (int64_t c = 0; c < ncells; ++c) {
      const int ic[3] = {(int)(c % N1), (int)((c / N1) % N2), (int)(c / ((int64_t)N1 * N2))};
      for (int a = 0; a < 3; ++a) {
        if (p->periodic[a]) continue;
        if (ic[a] == 0) bface(p, &t, a, 0, ic, x + c * nb, y + c * nb);
        if (ic[a] == p->ncell[a] - 1) bface(p, &t, a, 1, ic, x + c * nb, y + c * nb);
      }
    }
  }
  return 0;
}

/* Rows of y = A x belonging to selected cells only: for each listed cell T,
 * its volume term plus the contribution of each of its six faces to the test
 * functions of T (the same face terms as above, restricted to one side).
 * y_rows has ncsel * n^3 entries in the order of `cells`. */
int oracle_apply_rows(const or_problem *p, const double *x, const int64_t *cells, int64_t ncsel,
                      double *y_rows, int terms, int nthreads) {
  if (check_problem(p)) return -1;
  const or_iface_fn iface = p->multilinear_on ? ml_interior_face : interior_face;
  const or_bface_fn bface = p->multilinear_on ? ml_boundary_face : boundary_face;
  or_tables t;
  make_tables(p->k, p->quad_extra, &t);
  const int64_t nb = (int64_t)t.n * t.n * t.n;
  const int N1 = p->ncell[0], N2 = p->ncell[1], N3 = p->ncell[2];
  const int64_t ncells = (int64_t)N1 * N2 * N3;
  if (nthreads <= 0) nthreads = 1;
  for (int64_t s = 0; s < ncsel; ++s)
    if (cells[s] < 0 || cells[s] >= ncells) return -1;
  memset(y_rows, 0, sizeof(double) * ncsel * nb);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int64_t s = 0; s < ncsel; ++s) {
    const int64_t c = cells[s];
    const int ic[3] = {(int)(c % N1), (int)((c / N1) % N2), (int)(c / ((int64_t)N1 * N2))};
    double *yT = y_rows + s * nb;
    if (terms & OR_VOLUME) (p->multilinear_on ? ml_volume_cell : volume_cell)(p, &t, ic, x + c * nb, yT);
    for (int a = 0; a < 3; ++a) {
      /* lower face of T (across the domain boundary on a periodic axis) */
      if (ic[a] == 0 && !p->periodic[a]) {
        if (terms & OR_BOUNDARY) bface(p, &t, a, 0, ic, x + c * nb, yT);
      } else if (terms & OR_INTERIOR) {
        int jm[3] = {ic[0], ic[1], ic[2]};
        jm[a] = (ic[a] + p->ncell[a] - 1) % p->ncell[a];
        iface(p, &t, a, jm, x + cell_id(p, jm) * nb, x + c * nb, NULL, yT);
      }
      /* upper face of T */
      if (ic[a] == p->ncell[a] - 1 && !p->periodic[a]) {
        if (terms & OR_BOUNDARY) bface(p, &t, a, 1, ic, x + c * nb, yT);
      } else if (terms & OR_INTERIOR) {
        int jp[3] = {ic[0], ic[1], ic[2]};
        jp[a] = (ic[a] + 1) % p->ncell[a];
        iface(p, &t, a, ic, x + c * nb, x + cell_id(p, jp) * nb, yT, NULL);
      }
    }
  }
  (void)N3;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Right-hand side functional l_h(v) of Sec. 2.2 with g = 0 and no Neumann   */
/* faces: f_{T,j} = (f, phi_j)_T by the same Gauss rule.  The source f is a  */
/* sum of separable terms f(x) = sum_t alpha_t prod_r g_{t,r}(x_r) with      */
/* g(kind 0) = 1, g(kind 1) = sin(pi x), g(kind 2) = cos(pi x).              */
/* ------------------------------------------------------------------------ */
static double sep_fn(int kind, double x) {
  if (kind == 1) return sin(M_PI * x);
  if (kind == 2) return cos(M_PI * x);
  return 1.0;
}

static double sep_eval(int nterms, const double *alpha, const int32_t *kinds, const double *X) {
  double f = 0.0;
  for (int s = 0; s < nterms; ++s)
    f += alpha[s] * sep_fn(kinds[3 * s], X[0]) * sep_fn(kinds[3 * s + 1], X[1]) *
         sep_fn(kinds[3 * s + 2], X[2]);
  return f;
}

int oracle_rhs(const or_problem *p, int nterms, const double *alpha, const int32_t *kinds,
               double *f, int nthreads) {
  if (check_problem(p) || p->affine_on) return -1; /* tensor-grid sources only */
  or_tables t;
  make_tables(p->k, p->quad_extra, &t);
  const int n = t.n, m = t.m;
  const int64_t nb = (int64_t)n * n * n;
  const int N1 = p->ncell[0], N2 = p->ncell[1], N3 = p->ncell[2];
  const int64_t ncells = (int64_t)N1 * N2 * N3;
  if (nthreads <= 0) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
  for (int64_t c = 0; c < ncells; ++c) {
    const int ic[3] = {(int)(c % N1), (int)((c / N1) % N2), (int)(c / ((int64_t)N1 * N2))};
    double o[3] = {0.0, 0.0, 0.0}, h[3] = {1.0, 1.0, 1.0};
    if (!p->multilinear_on) cell_geom(p, ic, o, h);
    double *fT = f + c * nb;
    memset(fT, 0, sizeof(double) * nb);
    for (int q3 = 0; q3 < m; ++q3)
      for (int q2 = 0; q2 < m; ++q2)
        for (int q1 = 0; q1 < m; ++q1) {
          double X[3] = {o[0] + h[0] * t.xi[q1], o[1] + h[1] * t.xi[q2], o[2] + h[2] * t.xi[q3]};
          double W = t.w[q1] * t.w[q2] * t.w[q3] * h[0] * h[1] * h[2];
          if (p->multilinear_on) {
            const double xi[3] = {t.xi[q1], t.xi[q2], t.xi[q3]};
            double J[9], C[9];
            ml_map(p, ic, xi, X, J);
            W = t.w[q1] * t.w[q2] * t.w[q3] * ml_cof(J, C);
          }
          const double fx = sep_eval(nterms, alpha, kinds, X);
          for (int j3 = 0; j3 < n; ++j3)
            for (int j2 = 0; j2 < n; ++j2)
              for (int j1 = 0; j1 < n; ++j1)
                fT[j1 + n * (j2 + n * j3)] += W * fx * t.V[q1][j1] * t.V[q2][j2] * t.V[q3][j3];
        }
  }
  (void)N3;
  return 0;
}

/* L2 projection of the Gaussian g(x) = amp exp(-width |x - center|^2) onto
 * the DG space (the initial concentration of the transport example,
 * Sec. 5.4): u_{T,j} = (g, phi_j)_T / |T| (the mass matrix of the
 * orthonormal basis is |T| I), the inner product by the operator's tensor
 * Gauss rule; tensor-grid meshes (no affine or multilinear map); no
 * periodic images. */
int oracle_project_gaussian(const or_problem *p, double amp, double width, const double *center, double *u,
                            int nthreads) {
  if (check_problem(p) || p->affine_on || p->multilinear_on) return -1;
  or_tables t;
  make_tables(p->k, p->quad_extra, &t);
  const int n = t.n, m = t.m;
  const int64_t nb = (int64_t)n * n * n;
  const int N1 = p->ncell[0], N2 = p->ncell[1], N3 = p->ncell[2];
  const int64_t ncells = (int64_t)N1 * N2 * N3;
  if (nthreads <= 0) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
  for (int64_t c = 0; c < ncells; ++c) {
    const int ic[3] = {(int)(c % N1), (int)((c / N1) % N2), (int)(c / ((int64_t)N1 * N2))};
    double o[3], h[3];
    cell_geom(p, ic, o, h);
    double *uT = u + c * nb;
    memset(uT, 0, sizeof(double) * nb);
    for (int q3 = 0; q3 < m; ++q3)
      for (int q2 = 0; q2 < m; ++q2)
        for (int q1 = 0; q1 < m; ++q1) {
          const double X[3] = {o[0] + h[0] * t.xi[q1], o[1] + h[1] * t.xi[q2], o[2] + h[2] * t.xi[q3]};
          double r2 = 0.0;
          for (int a = 0; a < 3; ++a) r2 += (X[a] - center[a]) * (X[a] - center[a]);
          /* weight of the point with |T| divided out */
          const double gw = t.w[q1] * t.w[q2] * t.w[q3] * amp * exp(-width * r2);
          for (int j3 = 0; j3 < n; ++j3)
            for (int j2 = 0; j2 < n; ++j2)
              for (int j1 = 0; j1 < n; ++j1)
                uT[j1 + n * (j2 + n * j3)] += gw * t.V[q1][j1] * t.V[q2][j2] * t.V[q3][j3];
        }
  }
  (void)N3;
  return 0;
}

/* Squared L2 error ||u_h - u||^2 over the mesh for a separable-sum exact
 * solution u, with a (k+3)-point Gauss rule per direction (exact for the
 * polynomial part, accurate for the smooth part). */
double oracle_l2err2(const or_problem *p, const double *x, int nterms, const double *alpha,
                     const int32_t *kinds) {
  if (check_problem(p) || p->affine_on) return -1.0;
  const int n = p->k + 1, mq = p->k + 3;
  double xi[OR_MAXN + 2], w[OR_MAXN + 2];
  oracle_gauss(mq, xi, w);
  double V[OR_MAXN + 2][OR_MAXN], Dd[OR_MAXN];
  for (int q = 0; q < mq; ++q) oracle_basis(p->k, xi[q], V[q], Dd);
  const int64_t nb = (int64_t)n * n * n;
  const int N1 = p->ncell[0], N2 = p->ncell[1], N3 = p->ncell[2];
  const int64_t ncells = (int64_t)N1 * N2 * N3;
  double err = 0.0;
  for (int64_t c = 0; c < ncells; ++c) {
    const int ic[3] = {(int)(c % N1), (int)((c / N1) % N2), (int)(c / ((int64_t)N1 * N2))};
    double o[3] = {0.0, 0.0, 0.0}, h[3] = {1.0, 1.0, 1.0};
    if (!p->multilinear_on) cell_geom(p, ic, o, h);
    const double *xT = x + c * nb;
    for (int q3 = 0; q3 < mq; ++q3)
      for (int q2 = 0; q2 < mq; ++q2)
        for (int q1 = 0; q1 < mq; ++q1) {
          double uh = 0.0;
          for (int j3 = 0; j3 < n; ++j3)
            for (int j2 = 0; j2 < n; ++j2)
              for (int j1 = 0; j1 < n; ++j1)
                uh += xT[j1 + n * (j2 + n * j3)] * V[q1][j1] * V[q2][j2] * V[q3][j3];
          double X[3] = {o[0] + h[0] * xi[q1], o[1] + h[1] * xi[q2], o[2] + h[2] * xi[q3]};
          double W = w[q1] * w[q2] * w[q3] * h[0] * h[1] * h[2];
          if (p->multilinear_on) {
            const double xr[3] = {xi[q1], xi[q2], xi[q3]};
            double J[9], C[9];
            ml_map(p, ic, xr, X, J);
            W = w[q1] * w[q2] * w[q3] * ml_cof(J, C);
          }
          const double d = uh - sep_eval(nterms, alpha, kinds, X);
          err += W * d * d;
        }
  }
  (void)N3;
  return err;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
