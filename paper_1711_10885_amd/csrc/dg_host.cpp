// Host side of libdgmf: problem validation, 1D tables, device tables, errors.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "dg_internal.h"

namespace dgmf {

static thread_local std::string g_last_error;

dg_status set_error(dg_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

dg_status hip_error(hipError_t e, const char *what) {
  return set_error(e == hipErrorOutOfMemory ? DG_ENOMEM : DG_EHIP,
                   std::string(what) + ": " + hipGetErrorString(e));
}

// Legendre P_m and P_m' at s in [-1,1] (Bonnet recurrence).
static void legendre_pm(int m, double s, double &p, double &dp) {
  double p0 = 1.0, p1 = s;
  if (m == 0) {
    p = 1.0;
    dp = 0.0;
    return;
  }
  for (int j = 2; j <= m; ++j) {
    const double p2 = ((2 * j - 1) * s * p1 - (j - 1) * p0) / j;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  dp = m * (s * p1 - p0) / (s * s - 1.0);
}

// m-point Gauss-Legendre rule on [0,1] (tensor Gauss quadrature of Sec. 3.1),
// nodes ascending, weights summing to one.
static void gauss01(int m, double *xi, double *w) {
  for (int i = 0; i < (m + 1) / 2; ++i) {
    // Tricomi's initial guess for the i-th largest root
    double s = (1.0 - (m - 1.0) / (8.0 * m * m * m)) * std::cos(M_PI * (4.0 * i + 3.0) / (4.0 * m + 2.0));
    double p = 0, dp = 0;
    for (int it = 0; it < 64; ++it) {
      legendre_pm(m, s, p, dp);
      const double ds = p / dp;
      s -= ds;
      if (std::fabs(ds) <= 1e-17) break;
    }
    legendre_pm(m, s, p, dp);
    const double wt = 1.0 / ((1.0 - s * s) * dp * dp);  // 2/(...) on [-1,1], halved
    xi[m - 1 - i] = 0.5 + 0.5 * s;
    w[m - 1 - i] = wt;
    xi[i] = 0.5 - 0.5 * s;
    w[i] = wt;
  }
  if (m % 2 == 1) xi[m / 2] = 0.5;  // exact midpoint
}

// theta_j(t) = sqrt(2j+1) P_j(2t-1) and its derivative, j = 0..k.
static void legendre_basis(int k, double t, double *v, double *d) {
  const double s = 2.0 * t - 1.0;
  double P[kMaxN + 1], dP[kMaxN + 1];
  P[0] = 1.0;
  dP[0] = 0.0;
  if (k >= 1) {
    P[1] = s;
    dP[1] = 1.0;
  }
  for (int j = 2; j <= k; ++j) {
    P[j] = ((2 * j - 1) * s * P[j - 1] - (j - 1) * P[j - 2]) / j;
    dP[j] = j * P[j - 1] + s * dP[j - 1];  // P_j' = j P_{j-1} + s P_{j-1}'
  }
  for (int j = 0; j <= k; ++j) {
    const double sc = std::sqrt(2.0 * j + 1.0);
    v[j] = sc * P[j];
    d[j] = 2.0 * sc * dP[j];
  }
}

static void build_tables(int k, Tables &t, int m = 0) {
  std::memset(&t, 0, sizeof(t));
  t.n = k + 1;
  t.m = m > 0 ? m : k + 1;
  gauss01(t.m, t.xi, t.w);
  for (int q = 0; q < t.m; ++q) legendre_basis(k, t.xi[q], t.V[q], t.D[q]);
  legendre_basis(k, 0.0, t.e0v, t.e0d);
  legendre_basis(k, 1.0, t.e1v, t.e1d);
}

static bool is_spd(const double *K) {
  double mx = 0.0;
  for (int i = 0; i < 9; ++i) {
    if (!std::isfinite(K[i])) return false;
    mx = std::fmax(mx, std::fabs(K[i]));
  }
  if (mx == 0.0) return false;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < i; ++j)
      if (std::fabs(K[3 * i + j] - K[3 * j + i]) > 1e-12 * mx) return false;
  double L[9] = {0};
  for (int j = 0; j < 3; ++j) {
    double s = K[4 * j];
    for (int p = 0; p < j; ++p) s -= L[3 * j + p] * L[3 * j + p];
    if (!(s > 1e-14 * mx)) return false;
    L[4 * j] = std::sqrt(s);
    for (int i = j + 1; i < 3; ++i) {
      double t = K[3 * i + j];
      for (int p = 0; p < j; ++p) t -= L[3 * i + p] * L[3 * j + p];
      L[3 * i + j] = t / L[4 * j];
    }
  }
  return true;
}

}  // namespace dgmf

using namespace dgmf;

extern "C" const char *dg_last_error(void) { return g_last_error.c_str(); }

extern "C" int64_t dg_ndof(const dg_handle *h) { return h ? h->ndof : -1; }

extern "C" int32_t dg_degree(const dg_handle *h) { return h ? h->k : -1; }

extern "C" int64_t dg_bj_nblocks(const dg_handle *h) { return h ? (h->bj ? h->bj_nblocks : 0) : -1; }

extern "C" dg_status dg_set_kernel(dg_handle *h, int32_t variant) {
  if (!h) return set_error(DG_EINVAL, "dg_set_kernel: handle is NULL");
  if (variant != DG_KERNEL_AUTO && variant != DG_KERNEL_REFERENCE)
    return set_error(DG_EINVAL, "dg_set_kernel: unknown variant");
  h->variant = variant;
  return DG_OK;
}

extern "C" void dg_destroy(dg_handle *h) {
  if (!h) return;
  int cur = 0;
  if (hipGetDevice(&cur) == hipSuccess && cur != h->device) (void)hipSetDevice(h->device);
  release_solver(h);
  release_learned(h);
  if (h->bj) (void)hipFree(h->bj);
  if (h->bj16) (void)hipFree(h->bj16);
  if (h->bj16_scale) (void)hipFree(h->bj16_scale);
  if (h->bj_cells) (void)hipFree(h->bj_cells);
  if (h->bj_gblock) (void)hipFree(h->bj_gblock);
  if (h->ts) (void)hipFree(h->ts);
  if (h->dev_block) (void)hipFree(h->dev_block);
  if (h->geo_block) (void)hipFree(h->geo_block);
  if (cur != h->device) (void)hipSetDevice(cur);
  delete h;
}

// Affine map x = A xi of the tensor grid: the change of variables in every
// volume and face integral gives the tensor-grid operator with
// K' = |det A| A^-1 K A^-T, b' = |det A| A^-1 b, c' = |det A| c (normals,
// surface measures, d = nu^T D nu and |F|/|T| of the physical cells all
// fold into these), which p receives; *vol_scale = |det A|.
static dg_status fold_affine(dg_problem &p, double *vol_scale) {
  const double *A = p.affine;
  double mx = 0.0;
  for (int i = 0; i < 9; ++i) {
    if (!std::isfinite(A[i])) return set_error(DG_EINVAL, "dg_setup: the affine map must be finite");
    mx = std::fmax(mx, std::fabs(A[i]));
  }
  // a b varying in x would not stay separable in xi; the polynomial diffusion
  // factor is defined in the grid coordinates xi and passes through as a
  // scalar factor of K'
  if ((p.flags & DG_B_PRODUCT) || p.b_sin[0] != 0.0 || p.b_sin[1] != 0.0 || p.b_sin[2] != 0.0)
    return set_error(DG_EINVAL, "dg_setup: DG_AFFINE needs a constant b");
  const double C[9] = {A[4] * A[8] - A[5] * A[7], A[5] * A[6] - A[3] * A[8], A[3] * A[7] - A[4] * A[6],
                       A[2] * A[7] - A[1] * A[8], A[0] * A[8] - A[2] * A[6], A[1] * A[6] - A[0] * A[7],
                       A[1] * A[5] - A[2] * A[4], A[2] * A[3] - A[0] * A[5], A[0] * A[4] - A[1] * A[3]};
  const double det = A[0] * C[0] + A[1] * C[1] + A[2] * C[2];
  if (!(std::fabs(det) > 1e-12 * mx * mx * mx)) return set_error(DG_EINVAL, "dg_setup: the affine map must be invertible");
  double Ai[9];  // A^-1 = C^T / det
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Ai[3 * i + j] = C[3 * j + i] / det;
  const double s = std::fabs(det);
  double AK[9], Kp[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double t = 0.0;
      for (int l = 0; l < 3; ++l) t += Ai[3 * i + l] * p.K[3 * l + j];
      AK[3 * i + j] = t;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double t = 0.0;
      for (int l = 0; l < 3; ++l) t += AK[3 * i + l] * Ai[3 * j + l];
      Kp[3 * i + j] = s * t;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) p.K[3 * i + j] = 0.5 * (Kp[3 * i + j] + Kp[3 * j + i]);
  double bp[3];
  for (int i = 0; i < 3; ++i) bp[i] = s * (Ai[3 * i] * p.b_const[0] + Ai[3 * i + 1] * p.b_const[1] + Ai[3 * i + 2] * p.b_const[2]);
  for (int i = 0; i < 3; ++i) p.b_const[i] = bp[i];
  p.c *= s;
  p.flags &= ~DG_AFFINE;
  *vol_scale = s;
  return DG_OK;
}

// ---- multilinear meshes (DG_MULTILINEAR) ------------------------------------

// Trilinear map of cell (i0,i1,i2) through its eight vertices V at reference
// point s: point X and Jacobian J[3r + t] = dX_r / ds_t.
static void host_tri_map(const dg_problem &p, const int *ic, const double *s, double *X, double *J) {
  const int64_t V0 = p.ncell[0] + 1, V1 = p.ncell[1] + 1;
  for (int r = 0; r < 3; ++r) {
    X[r] = 0.0;
    for (int t = 0; t < 3; ++t) J[3 * r + t] = 0.0;
  }
  for (int c = 0; c < 8; ++c) {
    const int cb[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
    const double *v = p.vertices + 3 * ((ic[0] + cb[0]) + V0 * ((ic[1] + cb[1]) + V1 * int64_t(ic[2] + cb[2])));
    const double l[3] = {cb[0] ? s[0] : 1.0 - s[0], cb[1] ? s[1] : 1.0 - s[1], cb[2] ? s[2] : 1.0 - s[2]};
    const double dl[3] = {cb[0] ? 1.0 : -1.0, cb[1] ? 1.0 : -1.0, cb[2] ? 1.0 : -1.0};
    const double wv = l[0] * l[1] * l[2];
    const double wd[3] = {dl[0] * l[1] * l[2], l[0] * dl[1] * l[2], l[0] * l[1] * dl[2]};
    for (int r = 0; r < 3; ++r) {
      X[r] += wv * v[r];
      for (int t = 0; t < 3; ++t) J[3 * r + t] += wd[t] * v[r];
    }
  }
}

static double host_det3(const double *J) {
  return J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) + J[2] * (J[3] * J[7] - J[4] * J[6]);
}

// Validation of a vertex mesh: finite vertices, det J > 0 at the corners and
// the centre of every cell, the polynomial diffusion factor positive on the
// vertices' bounding box (every point of a trilinear cell is a convex
// combination of its vertices).
static dg_status check_vertex_mesh(const dg_problem &p) {
  if (!p.vertices) return set_error(DG_EINVAL, "dg_setup: DG_MULTILINEAR needs vertices");
  const int64_t nv = int64_t(p.ncell[0] + 1) * (p.ncell[1] + 1) * (p.ncell[2] + 1);
  double lo[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL}, hi[3] = {-HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
  for (int64_t i = 0; i < 3 * nv; ++i) {
    if (!std::isfinite(p.vertices[i])) return set_error(DG_EINVAL, "dg_setup: vertices must be finite");
    lo[i % 3] = std::fmin(lo[i % 3], p.vertices[i]);
    hi[i % 3] = std::fmax(hi[i % 3], p.vertices[i]);
  }
  for (int i2 = 0; i2 < p.ncell[2]; ++i2)
    for (int i1 = 0; i1 < p.ncell[1]; ++i1)
      for (int i0 = 0; i0 < p.ncell[0]; ++i0) {
        const int ic[3] = {i0, i1, i2};
        for (int c = 0; c < 9; ++c) {
          const double s[3] = {c == 8 ? 0.5 : double(c & 1), c == 8 ? 0.5 : double((c >> 1) & 1),
                               c == 8 ? 0.5 : double((c >> 2) & 1)};
          double X[3], J[9];
          host_tri_map(p, ic, s, X, J);
          if (!(host_det3(J) > 0.0))
            return set_error(DG_EINVAL, "dg_setup: every cell's Jacobian determinant must be positive");
        }
      }
  if (p.flags & DG_KAPPA_POLY)
    for (int j = 0; j < 3; ++j) {
      const double *c = p.kappa_poly + 3 * j;
      auto g = [&](double t) { return c[0] + c[1] * t + c[2] * t * t; };
      bool ok = g(lo[j]) > 0.0 && g(hi[j]) > 0.0;
      if (c[2] != 0.0) {
        const double tv = -c[1] / (2.0 * c[2]);
        if (tv > lo[j] && tv < hi[j]) ok = ok && g(tv) > 0.0;
      }
      if (!ok) return set_error(DG_EINVAL, "dg_setup: kappa_poly factors must be positive on the mesh");
    }
  return DG_OK;
}

// Cell volumes |T| (det J integrated with the 2-point Gauss rule, exact for
// the trilinear map: det J has degree <= 2 per direction) and face areas |F|
// (|cof(J) e_a| integrated with the operator's m-point rule over the face,
// from its four vertices), staged for the device.
static void vertex_mesh_tables(const dg_problem &p, const Tables &tq, std::vector<double> &cvol,
                               std::vector<double> farea[3]) {
  const int N[3] = {p.ncell[0], p.ncell[1], p.ncell[2]};
  const double g2[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  cvol.assign(size_t(N[0]) * N[1] * N[2], 0.0);
  for (int i2 = 0; i2 < N[2]; ++i2)
    for (int i1 = 0; i1 < N[1]; ++i1)
      for (int i0 = 0; i0 < N[0]; ++i0) {
        const int ic[3] = {i0, i1, i2};
        double v = 0.0;
        for (int q = 0; q < 8; ++q) {
          const double s[3] = {g2[q & 1], g2[(q >> 1) & 1], g2[(q >> 2) & 1]};
          double X[3], J[9];
          host_tri_map(p, ic, s, X, J);
          v += 0.125 * host_det3(J);
        }
        cvol[i0 + size_t(N[0]) * (i1 + size_t(N[1]) * i2)] = v;
      }
  for (int a = 0; a < 3; ++a) {
    const int b = (a == 0) ? 1 : 0, c = (a == 2) ? 1 : 2;
    farea[a].assign(size_t(N[a] + 1) * N[b] * N[c], 0.0);
    for (int icc = 0; icc < N[c]; ++icc)
      for (int ib = 0; ib < N[b]; ++ib)
        for (int pa = 0; pa <= N[a]; ++pa) {
          // the face as side e of the cell below it (e = 1), or above it on plane 0
          int ic[3];
          ic[a] = pa < N[a] ? pa : pa - 1;
          ic[b] = ib;
          ic[c] = icc;
          const double e = pa < N[a] ? 0.0 : 1.0;
          double A = 0.0;
          for (int qc = 0; qc < tq.m; ++qc)
            for (int qb = 0; qb < tq.m; ++qb) {
              double s[3], X[3], J[9];
              s[a] = e;
              s[b] = tq.xi[qb];
              s[c] = tq.xi[qc];
              host_tri_map(p, ic, s, X, J);
              // column a of cof(J): cross product of the tangent columns b, c
              const int t1 = (a + 1) % 3, t2 = (a + 2) % 3;
              const double n0 = J[3 + t1] * J[6 + t2] - J[6 + t1] * J[3 + t2];
              const double n1 = J[6 + t1] * J[t2] - J[t1] * J[6 + t2];
              const double n2 = J[t1] * J[3 + t2] - J[3 + t1] * J[t2];
              A += tq.w[qb] * tq.w[qc] * std::sqrt(n0 * n0 + n1 * n1 + n2 * n2);
            }
          farea[a][pa + size_t(N[a] + 1) * (ib + size_t(N[b]) * icc)] = A;
        }
  }
}

extern "C" dg_status dg_setup(const dg_problem *p_in, dg_handle **out) {
  if (!out) return set_error(DG_EINVAL, "dg_setup: out is NULL");
  *out = nullptr;
  if (!p_in) return set_error(DG_EINVAL, "dg_setup: problem is NULL");
  // the problem the kernels see: an affine map folds into the coefficients
  dg_problem pt = *p_in;
  double vol_scale = 1.0;
  if ((pt.flags & DG_MULTILINEAR) && (pt.flags & DG_AFFINE))
    return set_error(DG_EINVAL, "dg_setup: DG_MULTILINEAR excludes DG_AFFINE, periodic axes and block Jacobi");
  if (pt.flags & DG_AFFINE) {
    const dg_status st = fold_affine(pt, &vol_scale);
    if (st != DG_OK) return st;
  }
  // multilinear meshes: the tensor tables below are built on unit nodes
  // (the kernels take the geometry from the vertices)
  const bool multilinear = (pt.flags & DG_MULTILINEAR) != 0;
  std::vector<double> unit_nodes[3];
  if (multilinear) {
    if (pt.flags & (DG_AFFINE | DG_WITH_BLOCK_JACOBI | DG_PERIODIC_X | DG_PERIODIC_Y | DG_PERIODIC_Z))
      return set_error(DG_EINVAL, "dg_setup: DG_MULTILINEAR excludes DG_AFFINE, periodic axes and block Jacobi");
    if (pt.k < 1 || pt.k > 7) return set_error(DG_EINVAL, "dg_setup: multilinear meshes support k <= 7");
    if (pt.quad_extra != 0 && pt.quad_extra != 2 && pt.quad_extra != (pt.k + 4) / 2)
      return set_error(DG_EINVAL, "dg_setup: on multilinear meshes quad_extra must be 0, 2 or ceil((k+3)/2)");
    for (int a = 0; a < 3; ++a) {
      if (pt.ncell[a] < 1) return set_error(DG_EINVAL, "dg_setup: ncell must be >= 1");
      unit_nodes[a].resize(pt.ncell[a] + 1);
      for (int i = 0; i <= pt.ncell[a]; ++i) unit_nodes[a][i] = double(i) / pt.ncell[a];
      pt.nodes[a] = unit_nodes[a].data();
    }
    const dg_status st = check_vertex_mesh(pt);
    if (st != DG_OK) return st;
  }
  const dg_problem *p = &pt;
  if (p->k < 1 || p->k > 10) return set_error(DG_EINVAL, "dg_setup: k must be in 1..10");
  if (!multilinear && p->quad_extra != 0 && p->quad_extra != 2)
    return set_error(DG_EINVAL, "dg_setup: quad_extra must be 0 or 2");
  if (!multilinear && p->k + 1 + p->quad_extra > kMaxN)
    return set_error(DG_EINVAL, "dg_setup: raised quadrature supports k <= 8");
  int64_t ncells = 1;
  for (int a = 0; a < 3; ++a) {
    if (p->ncell[a] < 1) return set_error(DG_EINVAL, "dg_setup: ncell must be >= 1");
    if (!p->nodes[a]) return set_error(DG_EINVAL, "dg_setup: nodes pointer is NULL");
    for (int i = 0; i <= p->ncell[a]; ++i)
      if (!std::isfinite(p->nodes[a][i]))
        return set_error(DG_EINVAL, "dg_setup: nodes must be finite");
    for (int i = 0; i < p->ncell[a]; ++i)
      if (!(p->nodes[a][i + 1] > p->nodes[a][i]))
        return set_error(DG_EINVAL, "dg_setup: nodes must be strictly increasing");
    if (p->b_axis[a] < 0 || p->b_axis[a] > 2)
      return set_error(DG_EINVAL, "dg_setup: b_axis must be 0, 1 or 2");
    if (!std::isfinite(p->b_const[a]) || !std::isfinite(p->b_sin[a]))
      return set_error(DG_EINVAL, "dg_setup: b must be finite");
    ncells *= p->ncell[a];
  }
  if (!is_spd(p->K)) return set_error(DG_EINVAL, "dg_setup: K must be symmetric positive definite");
  if (!std::isfinite(p->c)) return set_error(DG_EINVAL, "dg_setup: c must be finite");
  if (!(p->sigma > 0.0) || !std::isfinite(p->sigma))
    return set_error(DG_EINVAL, "dg_setup: sigma must be positive");
  if (p->kappa)
    for (int64_t c = 0; c < ncells; ++c)
      if (!(p->kappa[c] > 0.0) || !std::isfinite(p->kappa[c]))
        return set_error(DG_EINVAL, "dg_setup: kappa must be positive and finite");
  const int n = p->k + 1;
  if (ncells > (int64_t(1) << 31) / 2) return set_error(DG_EINVAL, "dg_setup: too many cells");
  if (p->flags & ~(DG_WITH_BLOCK_JACOBI | DG_PERIODIC_X | DG_PERIODIC_Y | DG_PERIODIC_Z | DG_B_PRODUCT |
                   DG_KAPPA_POLY | DG_MULTILINEAR))
    return set_error(DG_EINVAL, "dg_setup: unknown flag bits");
  const bool bprod = (p->flags & DG_B_PRODUCT) != 0;
  const bool kpoly = (p->flags & DG_KAPPA_POLY) != 0;
  if (kpoly) {
    for (int t = 0; t < 9; ++t)
      if (!std::isfinite(p->kappa_poly[t])) return set_error(DG_EINVAL, "dg_setup: kappa_poly must be finite");
  }
  if (kpoly && !multilinear) {
    // every factor positive at the Gauss coordinates and nodes it is used at
    Tables tq;
    build_tables(p->k, tq, p->k + 1 + p->quad_extra);
    for (int j = 0; j < 3; ++j) {
      const double *c = p->kappa_poly + 3 * j;
      auto g = [&](double s) { return c[0] + c[1] * s + c[2] * s * s; };
      for (int i = 0; i < p->ncell[j]; ++i) {
        const double o = p->nodes[j][i], hh = p->nodes[j][i + 1] - p->nodes[j][i];
        bool ok = g(o) > 0.0 && g(o + hh) > 0.0;
        for (int q = 0; q < tq.m; ++q) ok = ok && g(o + hh * tq.xi[q]) > 0.0;
        if (!ok) return set_error(DG_EINVAL, "dg_setup: kappa_poly factors must be positive on the mesh");
      }
    }
  }
  if (bprod)
    for (int t = 0; t < 9; ++t)
      if (!std::isfinite(p->b_freq[t]) || !std::isfinite(p->b_phase[t]) || !std::isfinite(p->b_amp[t / 3]))
        return set_error(DG_EINVAL, "dg_setup: product-form b must be finite");
  const int periodic = (p->flags >> 2) & 7;  // bit a: axis a
  if ((p->flags & DG_WITH_BLOCK_JACOBI) && n * n * n > kMaxBjBlock)
    return set_error(DG_EINVAL, "dg_setup: block Jacobi supports k <= 7");
  for (int a = 0; a < 3; ++a)
    if ((p->flags & DG_WITH_BLOCK_JACOBI) && ((periodic >> a) & 1) && p->ncell[a] > 1 && p->ncell[a] % 2)
      return set_error(DG_EINVAL, "dg_setup: block Jacobi with a periodic axis needs an even number of cells");

  dg_handle *h = new dg_handle();
  std::memset(&h->prob, 0, sizeof(h->prob));
  h->prob = *p;
  for (int a = 0; a < 3; ++a) h->prob.nodes[a] = nullptr;
  h->prob.kappa = nullptr;
  h->prob.vertices = nullptr;
  h->k = p->k;
  h->ncells = ncells;
  h->ndof = ncells * n * n * n;
  h->dev_block = nullptr;
  h->geo_block = nullptr;
  h->variant = DG_KERNEL_AUTO;
  h->ws = nullptr;
  h->ts = nullptr;
  h->ws_bytes = 0;
  h->red = nullptr;
  h->bj = nullptr;
  h->bj16 = nullptr;
  h->bj16_scale = nullptr;
  h->bj_nb = 0;
  h->bj_nblocks = 0;
  h->bj_cells = nullptr;
  h->bj_gblock = nullptr;
  h->bj_ngroups = 0;
  h->mlp = nullptr;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return set_error(DG_EHIP, "dg_setup: no HIP device");
  }
  if (dg_status st = static_scratch_init(h->device); st != DG_OK) {
    delete h;
    return st;
  }
  build_tables(p->k, h->tab);
  build_tables(p->k, h->tabq, n + p->quad_extra);
  h->quad_extra = p->quad_extra;
  h->vol_scale = vol_scale;
  h->affine = (p_in->flags & DG_AFFINE) != 0;

  // host staging of every device table, then one allocation + one copy
  // (coefficients at the Gauss coordinates of the operator's rule)
  const int m = h->tabq.m;
  std::vector<double> host;
  size_t off_h[3], off_ih[3], off_nd[3], off_bv[3], off_bn[3], off_kappa = 0;
  for (int a = 0; a < 3; ++a) {
    off_h[a] = host.size();
    for (int i = 0; i < p->ncell[a]; ++i) host.push_back(p->nodes[a][i + 1] - p->nodes[a][i]);
    off_ih[a] = host.size();
    for (int i = 0; i < p->ncell[a]; ++i) host.push_back(1.0 / (p->nodes[a][i + 1] - p->nodes[a][i]));
    off_nd[a] = host.size();
    host.insert(host.end(), p->nodes[a], p->nodes[a] + p->ncell[a] + 1);
  }
  for (int r = 0; r < 3; ++r) {
    const int ax = p->b_axis[r];
    off_bv[r] = host.size();
    for (int i = 0; i < p->ncell[ax]; ++i) {
      const double o = p->nodes[ax][i], hh = p->nodes[ax][i + 1] - p->nodes[ax][i];
      for (int q = 0; q < m; ++q)
        host.push_back(p->b_const[r] + p->b_sin[r] * std::sin(M_PI * (o + hh * h->tabq.xi[q])));
    }
    off_bn[r] = host.size();
    for (int i = 0; i <= p->ncell[ax]; ++i)
      host.push_back(p->b_const[r] + p->b_sin[r] * std::sin(M_PI * p->nodes[ax][i]));
  }
  // product form: factor f_rj at the Gauss coordinates and nodes of axis j
  // (with the polynomial diffusion factor a sum-form b is tabulated this way
  // too: its one non-constant factor on axis b_axis[r], ones elsewhere)
  size_t off_bf[9] = {}, off_bfn[9] = {};
  const bool btab = bprod || kpoly;
  if (btab)
    for (int t = 0; t < 9; ++t) {
      const int r = t / 3, j = t % 3;
      const double amp = j == 0 ? p->b_amp[r] : 1.0;
      auto f = [&](double s) {
        if (!bprod) return j == p->b_axis[r] ? p->b_const[r] + p->b_sin[r] * std::sin(M_PI * s) : 1.0;
        return p->b_freq[t] == 0.0 ? amp : amp * std::sin(p->b_freq[t] * s + p->b_phase[t]);
      };
      off_bf[t] = host.size();
      for (int i = 0; i < p->ncell[j]; ++i) {
        const double o = p->nodes[j][i], hh = p->nodes[j][i + 1] - p->nodes[j][i];
        for (int q = 0; q < m; ++q) host.push_back(f(o + hh * h->tabq.xi[q]));
      }
      off_bfn[t] = host.size();
      for (int i = 0; i <= p->ncell[j]; ++i) host.push_back(f(p->nodes[j][i]));
    }
  // polynomial diffusion factor kp_j at the Gauss coordinates and nodes of axis j
  size_t off_kf[3] = {}, off_kfn[3] = {};
  if (kpoly) {
    for (int j = 0; j < 3; ++j) {
      const double *c = p->kappa_poly + 3 * j;
      auto g = [&](double s) { return c[0] + c[1] * s + c[2] * s * s; };
      off_kf[j] = host.size();
      for (int i = 0; i < p->ncell[j]; ++i) {
        const double o = p->nodes[j][i], hh = p->nodes[j][i + 1] - p->nodes[j][i];
        for (int q = 0; q < m; ++q) host.push_back(g(o + hh * h->tabq.xi[q]));
      }
      off_kfn[j] = host.size();
      for (int i = 0; i <= p->ncell[j]; ++i) host.push_back(g(p->nodes[j][i]));
    }
  }
  const size_t off_w = host.size();
  host.insert(host.end(), h->tabq.w, h->tabq.w + m);
  if (p->kappa) {
    off_kappa = host.size();
    host.insert(host.end(), p->kappa, p->kappa + ncells);
  }
  hipError_t e = hipMalloc(&h->dev_block, host.size() * sizeof(double));
  if (e != hipSuccess) {
    delete h;
    return hip_error(e, "dg_setup: hipMalloc");
  }
  e = hipMemcpy(h->dev_block, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    dg_destroy(h);
    return hip_error(e, "dg_setup: hipMemcpy");
  }
  double *base = static_cast<double *>(h->dev_block);
  DevMesh &M = h->mesh;
  for (int a = 0; a < 3; ++a) {
    M.ncell[a] = p->ncell[a];
    M.h[a] = base + off_h[a];
    M.ih[a] = base + off_ih[a];
    M.nodes[a] = base + off_nd[a];
    M.bvol[a] = base + off_bv[a];
    M.bnode[a] = base + off_bn[a];
    M.b_axis[a] = p->b_axis[a];
  }
  for (int t = 0; t < 9; ++t) {
    M.bf[t] = btab ? base + off_bf[t] : nullptr;
    M.bfn[t] = btab ? base + off_bfn[t] : nullptr;
  }
  M.bprod = btab ? 1 : 0;
  for (int j = 0; j < 3; ++j) {
    M.kf[j] = kpoly ? base + off_kf[j] : nullptr;
    M.kfn[j] = kpoly ? base + off_kfn[j] : nullptr;
  }
  M.kpoly = kpoly ? 1 : 0;
  M.kappa = p->kappa ? base + off_kappa : nullptr;
  M.periodic = periodic;
  M.w = base + off_w;
  std::memcpy(M.K, p->K, sizeof(M.K));
  M.c = p->c;
  M.sigma = p->sigma;
  M.verts = nullptr;
  M.cvol = nullptr;
  for (int a = 0; a < 3; ++a) M.farea[a] = nullptr;
  M.multilinear = multilinear ? 1 : 0;
  if (multilinear) {
    std::vector<double> cvol, farea[3];
    vertex_mesh_tables(*p, h->tabq, cvol, farea);
    const size_t nv3 = 3 * size_t(p->ncell[0] + 1) * (p->ncell[1] + 1) * (p->ncell[2] + 1);
    std::vector<double> g(p->vertices, p->vertices + nv3);
    const size_t off_cv = g.size();
    g.insert(g.end(), cvol.begin(), cvol.end());
    size_t off_fa[3];
    for (int a = 0; a < 3; ++a) {
      off_fa[a] = g.size();
      g.insert(g.end(), farea[a].begin(), farea[a].end());
    }
    e = hipMalloc(&h->geo_block, g.size() * sizeof(double));
    if (e != hipSuccess) {
      h->geo_block = nullptr;
      dg_destroy(h);
      return hip_error(e, "dg_setup: geometry tables");
    }
    e = hipMemcpy(h->geo_block, g.data(), g.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      dg_destroy(h);
      return hip_error(e, "dg_setup: hipMemcpy");
    }
    double *gb = static_cast<double *>(h->geo_block);
    M.verts = gb;
    M.cvol = gb + off_cv;
    for (int a = 0; a < 3; ++a) M.farea[a] = gb + off_fa[a];
  }
  if (p->flags & DG_WITH_BLOCK_JACOBI) {
    const dg_status ds = build_block_jacobi(h, p);
    if (ds != DG_OK) {
      const std::string msg = dg_last_error();
      dg_destroy(h);
      return set_error(ds, msg);
    }
  }
  *out = h;
  return DG_OK;
}

namespace dgmf {
hipError_t apply_f64(const dg_handle *h, const double *x, double *y, hipStream_t s) {
  if (h->mesh.multilinear) return launch_apply_geo_f64(h, x, y, s);
  if (h->variant == DG_KERNEL_REFERENCE) return launch_apply_ref_f64(h, x, y, s);
  return h->quad_extra ? apply_raised_f64(h, x, y, s) : launch_apply_fused_f64(h, x, y, s);
}

hipError_t apply_f32(const dg_handle *h, const float *x, float *y, hipStream_t s) {
  return h->quad_extra ? apply_raised_f32(h, x, y, s) : launch_apply_fused_f32(h, x, y, s);
}
}  // namespace dgmf

static bool overlaps(const void *a, const void *b, size_t bytes) {
  const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
  return pa < pb + bytes && pb < pa + bytes;
}

extern "C" dg_status dg_apply(dg_handle *h, const double *x, double *y, void *stream) {
  if (!h) return set_error(DG_EINVAL, "dg_apply: handle is NULL");
  if (!x || !y) return set_error(DG_EINVAL, "dg_apply: x or y is NULL");
  if (overlaps(x, y, size_t(h->ndof) * sizeof(double)))
    return set_error(DG_EINVAL, "dg_apply: x and y overlap");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != h->device) {
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_error(e, "dg_apply: hipSetDevice");
  }
  hipError_t e = apply_f64(h, x, y, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_error(e, "dg_apply: kernel launch");
  return DG_OK;
}

extern "C" dg_status dg_precond_apply(dg_handle *h, int32_t precond, const double *r, double *z, void *stream) {
  if (!h) return set_error(DG_EINVAL, "dg_precond_apply: handle is NULL");
  if (!r || !z) return set_error(DG_EINVAL, "dg_precond_apply: r or z is NULL");
  if (overlaps(r, z, size_t(h->ndof) * sizeof(double)))
    return set_error(DG_EINVAL, "dg_precond_apply: r and z overlap");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != h->device) {
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_error(e, "dg_precond_apply: hipSetDevice");
  }
  hipError_t e;
  if (precond == DG_PREC_BLOCK_JACOBI) {
    if (!h->bj) return set_error(DG_EINVAL, "dg_precond_apply: handle was set up without DG_WITH_BLOCK_JACOBI");
    e = bj_apply<double, double>(h, r, z, static_cast<hipStream_t>(stream));
  } else if (precond == DG_PREC_LEARNED) {
    if (!learned_ready(h))
      return set_error(DG_EINVAL, "dg_precond_apply: no trained or loaded network (or no block Jacobi)");
    e = learned_apply<double>(h, r, z, static_cast<hipStream_t>(stream));
  } else {
    return set_error(DG_EINVAL, "dg_precond_apply: unknown preconditioner");
  }
  if (e != hipSuccess) return hip_error(e, "dg_precond_apply: kernel launch");
  return DG_OK;
}

extern "C" dg_status dg_apply_f32(dg_handle *h, const float *x, float *y, void *stream) {
  if (!h) return set_error(DG_EINVAL, "dg_apply_f32: handle is NULL");
  if (!x || !y) return set_error(DG_EINVAL, "dg_apply_f32: x or y is NULL");
  if (overlaps(x, y, size_t(h->ndof) * sizeof(float)))
    return set_error(DG_EINVAL, "dg_apply_f32: x and y overlap");
  if (h->mesh.multilinear) return set_error(DG_EINVAL, "dg_apply_f32: not available on multilinear meshes");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != h->device) {
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_error(e, "dg_apply_f32: hipSetDevice");
  }
  hipError_t e = apply_f32(h, x, y, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_error(e, "dg_apply_f32: kernel launch");
  return DG_OK;
}
