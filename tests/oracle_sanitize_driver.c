/*
 * Driver for the sanitizer run of the CPU oracle: compiled together with
 * oracle/dg_oracle.c under -fsanitize=address,undefined by
 * tests/test_oracle_sanitizers.py, it calls every exported oracle routine
 * on small problems of every kind the oracle accepts (every degree, single
 * cells, periodic axes, product-form b, the polynomial diffusion factor, the
 * raised rule, affine and multilinear meshes) and checks that the whole-mesh apply and the
 * per-cell rows agree.  Any out-of-bounds access, use of uninitialised or
 * freed memory, or undefined arithmetic is reported by the sanitizers and
 * fails the run.  Test infrastructure only.
 */
#include <stdio.h>

#include "../oracle/dg_oracle.c"

static unsigned long long rng_state = 0x9e3779b97f4a7c15ull;

/* SplitMix64 (Steele, Lea & Flood): uniform in [-1, 1) */
static double urand(void) {
  unsigned long long z = (rng_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) / 4503599627370496.0 - 1.0;
}

/* multilinear: vertices of the nodes' tensor grid moved by up to 0.15 of a
 * cell in every coordinate (the cells stay valid hexahedra) */
static int run_case(int k, const int *ncell, int periodic, int bprod, int kpoly, int qx, int affine, int multilinear) {
  double *nodes[3];
  for (int a = 0; a < 3; ++a) {
    nodes[a] = malloc(sizeof(double) * (ncell[a] + 1));
    nodes[a][0] = 0.0;
    for (int i = 0; i < ncell[a]; ++i) nodes[a][i + 1] = nodes[a][i] + 1.0 + 0.4 * urand();
  }
  or_problem p;
  memset(&p, 0, sizeof(p));
  for (int a = 0; a < 3; ++a) {
    p.ncell[a] = ncell[a];
    p.nodes[a] = nodes[a];
    p.b_axis[a] = (a + 1) % 3;
    p.b_const[a] = 0.3 * urand();
    p.b_sin[a] = 0.5;
    p.periodic[a] = (periodic >> a) & 1;
  }
  p.k = k;
  const double K[9] = {1.0, 0.2, 0.1, 0.2, 0.8, -0.05, 0.1, -0.05, 0.6};
  memcpy(p.K, K, sizeof(K));
  const int64_t ncells = (int64_t)ncell[0] * ncell[1] * ncell[2];
  double *kap = malloc(sizeof(double) * ncells);
  for (int64_t c = 0; c < ncells; ++c) kap[c] = 1.0 + 0.5 * urand();
  p.kappa = kap;
  p.c = 0.7;
  p.sigma = 2.0 * k * (k + 2);
  p.b_product = bprod;
  for (int r = 0; r < 3; ++r) {
    p.b_amp[r] = urand();
    for (int j = 0; j < 3; ++j) {
      p.b_freq[3 * r + j] = (j == r) ? 0.0 : 1.0 + urand();
      p.b_phase[3 * r + j] = urand();
    }
  }
  p.kappa_poly_on = kpoly;
  for (int j = 0; j < 3; ++j) {
    p.kappa_poly[3 * j] = 1.0;
    p.kappa_poly[3 * j + 1] = 0.1 * urand();
    p.kappa_poly[3 * j + 2] = 0.05 * urand();
  }
  p.quad_extra = qx;
  p.affine_on = affine;
  const double A[9] = {1.2, 0.3, -0.1, 0.1, 0.8, 0.25, -0.2, 0.15, 1.1};
  memcpy(p.affine, A, sizeof(A));
  double *verts = NULL;
  if (multilinear) {
    const int64_t nv = (int64_t)(ncell[0] + 1) * (ncell[1] + 1) * (ncell[2] + 1);
    verts = malloc(sizeof(double) * 3 * nv);
    for (int v2 = 0; v2 <= ncell[2]; ++v2)
      for (int v1 = 0; v1 <= ncell[1]; ++v1)
        for (int v0 = 0; v0 <= ncell[0]; ++v0) {
          const int vi[3] = {v0, v1, v2};
          double *X = verts + 3 * (v0 + (int64_t)(ncell[0] + 1) * (v1 + (int64_t)(ncell[1] + 1) * v2));
          for (int a = 0; a < 3; ++a) X[a] = nodes[a][vi[a]] + 0.15 * urand();
        }
    p.multilinear_on = 1;
    p.vertices = verts;
    for (int a = 0; a < 3; ++a) p.periodic[a] = 0;
  }

  const int64_t nd = oracle_ndof(&p), nb = (int64_t)(k + 1) * (k + 1) * (k + 1);
  double *x = malloc(sizeof(double) * nd), *y = malloc(sizeof(double) * nd), *yr = malloc(sizeof(double) * nd);
  int64_t *cells = malloc(sizeof(int64_t) * ncells);
  for (int64_t i = 0; i < nd; ++i) x[i] = urand();
  for (int64_t c = 0; c < ncells; ++c) cells[c] = c;
  int bad = 0;
  if (oracle_apply(&p, x, y, OR_VOLUME | OR_INTERIOR | OR_BOUNDARY, 2) != 0) bad = 1;
  if (oracle_apply_rows(&p, x, cells, ncells, yr, OR_VOLUME | OR_INTERIOR | OR_BOUNDARY, 2) != 0) bad = 1;
  double mx = 0.0, dif = 0.0;
  for (int64_t i = 0; i < nd; ++i) {
    mx = fmax(mx, fabs(y[i]));
    dif = fmax(dif, fabs(y[i] - yr[i]));
  }
  if (!(dif <= 1e-12 * mx)) bad = 1;
  if (!affine) {
    const double alpha[2] = {1.0, -0.5};
    const int32_t kinds[6] = {1, 1, 1, 2, 0, 1};
    if (oracle_rhs(&p, 2, alpha, kinds, y, 2) != 0) bad = 1;
    const double e2 = oracle_l2err2(&p, x, 2, alpha, kinds);
    if (!(e2 > 0.0)) bad = 1;
  }
  printf("k=%d ncell=%dx%dx%d per=%d bprod=%d kpoly=%d qx=%d affine=%d multilinear=%d: apply/rows max diff %.2e of "
         "%.2e %s\n", k, ncell[0], ncell[1], ncell[2], periodic, bprod, kpoly, qx, affine, multilinear, dif, mx,
         bad ? "FAIL" : "ok");
  free(verts);
  free(cells);
  free(yr);
  free(y);
  free(x);
  free(kap);
  for (int a = 0; a < 3; ++a) free(nodes[a]);
  return bad;
}

int main(void) {
  int bad = 0;
  double xi[14], w[14], v[11], d[11];
  for (int m = 1; m <= 14; ++m) bad |= oracle_gauss(m, xi, w) != 0;
  for (int k = 1; k <= 10; ++k) oracle_basis(k, 0.3, v, d);
  const int meshes[4][3] = {{1, 1, 1}, {3, 2, 2}, {2, 1, 3}, {1, 3, 1}};
  for (int k = 1; k <= 10; ++k) {
    const int *nc = meshes[k % 4];
    bad |= run_case(k, nc, k % 8, 0, 0, 0, 0, 0);
  }
  bad |= run_case(3, meshes[1], 5, 1, 0, 0, 0, 0);
  bad |= run_case(4, meshes[2], 2, 1, 1, 0, 0, 0);
  bad |= run_case(2, meshes[1], 0, 0, 1, 2, 0, 0);
  bad |= run_case(8, meshes[0], 7, 1, 1, 2, 0, 0);
  bad |= run_case(3, meshes[1], 1, 0, 0, 0, 1, 0);
  bad |= run_case(2, meshes[3], 6, 0, 1, 2, 1, 0);
  bad |= run_case(1, meshes[1], 0, 0, 0, 0, 0, 1);
  bad |= run_case(2, meshes[2], 0, 1, 1, 2, 0, 1);
  bad |= run_case(7, meshes[0], 0, 0, 1, 5, 0, 1);
  printf(bad ? "SANITIZER DRIVER: FAIL\n" : "SANITIZER DRIVER: OK\n");
  return bad;
}
