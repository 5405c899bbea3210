// Load vector of a separable source (the right-hand-side functional of
// Sec. 2.2 with homogeneous Dirichlet data): f_{T,j} = (f, phi_j)_T by the
// tensor Gauss rule of the operator (Sec. 3.1): m = k + 1 points per
// direction, or k + 3 with the raised rule (q = 2p + 4, Problem B of Sec. 5.1).
//
// For f(x) = sum_t alpha_t g_t1(x_1) g_t2(x_2) g_t3(x_3) the cell integral
// factorises into 1D integrals (sum factorization of a rank-one integrand):
//   f_{T,j} = |T| sum_t alpha_t prod_a sum_q w_q g_ta(o_a + h_a xi_q) theta_{j_a}(xi_q).
// One thread per coefficient (cell, j).  The same kernel gives the L2
// projection of a Gaussian (the initial concentration of the transport
// example, Sec. 5.4): a product of 1D Gaussians, divided by |T| (the mass
// matrix of the orthonormal basis is |T| I).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "dg_internal.h"

namespace dgmf {

constexpr int kMaxTerms = 16;

struct LvArgs {
  int n, m, nterms;  // basis functions and Gauss points per direction
  double xi[kMaxN], w[kMaxN], V[kMaxN][kMaxN];
  double alpha[kMaxTerms];
  int kinds[kMaxTerms][3];
  // kind 3: the Gaussian factor exp(-gw (x_a - gc[a])^2) of axis a
  double gw, gc[3];
  int project;  // 1: divide by |T| (the L2 projection M^{-1} l), 0: the load vector l
};

__device__ __forceinline__ double sep_factor(const LvArgs &L, int kind, int a, double x) {
  if (kind == 3) {
    const double d = x - (a == 0 ? L.gc[0] : (a == 1 ? L.gc[1] : L.gc[2]));
    return exp(-L.gw * d * d);
  }
  return kind == 0 ? 1.0 : (kind == 1 ? sinpi(x) : cospi(x));
}

__global__ __launch_bounds__(256) void k_load_vector(DevMesh M, LvArgs L, int64_t ndof, double *__restrict__ f) {
  const int n = L.n, m = L.m, nb = n * n * n;
  for (int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; g < ndof; g += int64_t(gridDim.x) * blockDim.x) {
    const int64_t c = g / nb;
    const int j = int(g - c * nb);
    const int ja[3] = {j % n, (j / n) % n, j / (n * n)};
    const int ic[3] = {int(c % M.ncell[0]), int((c / M.ncell[0]) % M.ncell[1]),
                       int(c / (int64_t(M.ncell[0]) * M.ncell[1]))};
    double o[3], h[3];
    for (int a = 0; a < 3; ++a) {
      o[a] = M.nodes[a][ic[a]];
      h[a] = M.h[a][ic[a]];
    }
    double acc = 0.0;
    for (int t = 0; t < L.nterms; ++t) {
      double prod = L.alpha[t];
      for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int q = 0; q < m; ++q)
          s = fma(L.w[q] * sep_factor(L, L.kinds[t][a], a, o[a] + h[a] * L.xi[q]), L.V[q][ja[a]], s);
        prod *= s;
      }
      acc += prod;
    }
    f[g] = L.project ? acc : acc * h[0] * h[1] * h[2];
  }
}

// 1D tables of the operator's rule
static LvArgs lv_args(const dg_handle *h) {
  LvArgs L;
  std::memset(&L, 0, sizeof(L));
  L.n = h->tabq.n;
  L.m = h->tabq.m;
  for (int q = 0; q < L.m; ++q) {
    L.xi[q] = h->tabq.xi[q];
    L.w[q] = h->tabq.w[q];
    for (int jj = 0; jj < L.n; ++jj) L.V[q][jj] = h->tabq.V[q][jj];
  }
  return L;
}

static dg_status lv_launch(dg_handle *h, const LvArgs &L, double *f, void *stream, const char *who) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != h->device) {
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_error(e, who);
  }
  const int64_t blocks = std::min<int64_t>((h->ndof + 255) / 256, int64_t(1) << 20);
  hipLaunchKernelGGL(k_load_vector, dim3(unsigned(blocks)), dim3(256), 0, static_cast<hipStream_t>(stream), h->mesh, L,
                     int64_t(h->ndof), f);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, who);
  return DG_OK;
}

}  // namespace dgmf

using namespace dgmf;

extern "C" dg_status dg_load_vector(dg_handle *h, int32_t nterms, const double *alpha, const int32_t *kinds,
                                    double *f, void *stream) {
  if (!h) return set_error(DG_EINVAL, "dg_load_vector: handle is NULL");
  if (nterms < 1 || nterms > kMaxTerms) return set_error(DG_EINVAL, "dg_load_vector: nterms must be in 1..16");
  if (!alpha || !kinds || !f) return set_error(DG_EINVAL, "dg_load_vector: NULL argument");
  if (h->affine) return set_error(DG_EINVAL, "dg_load_vector: separable sources are tensor-grid only, not affine meshes");
  if (h->mesh.multilinear)
    return set_error(DG_EINVAL, "dg_load_vector: separable sources are tensor-grid only, not multilinear meshes");
  LvArgs L = lv_args(h);
  L.nterms = nterms;
  for (int t = 0; t < nterms; ++t) {
    if (!std::isfinite(alpha[t])) return set_error(DG_EINVAL, "dg_load_vector: alpha must be finite");
    L.alpha[t] = alpha[t];
    for (int a = 0; a < 3; ++a) {
      if (kinds[3 * t + a] < 0 || kinds[3 * t + a] > 2)
        return set_error(DG_EINVAL, "dg_load_vector: kinds must be 0, 1 or 2");
      L.kinds[t][a] = kinds[3 * t + a];
    }
  }
  return lv_launch(h, L, f, stream, "dg_load_vector");
}

extern "C" dg_status dg_project_gaussian(dg_handle *h, double amp, double width, const double *center, double *u,
                                         void *stream) {
  if (!h) return set_error(DG_EINVAL, "dg_project_gaussian: handle is NULL");
  if (!center || !u) return set_error(DG_EINVAL, "dg_project_gaussian: NULL argument");
  if (h->affine || h->mesh.multilinear)
    return set_error(DG_EINVAL, "dg_project_gaussian: tensor-grid meshes only");
  if (!std::isfinite(amp) || !(width > 0.0) || !std::isfinite(width))
    return set_error(DG_EINVAL, "dg_project_gaussian: amp must be finite and width positive");
  LvArgs L = lv_args(h);
  L.nterms = 1;
  L.alpha[0] = amp;
  L.gw = width;
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(center[a])) return set_error(DG_EINVAL, "dg_project_gaussian: center must be finite");
    L.kinds[0][a] = 3;
    L.gc[a] = center[a];
  }
  L.project = 1;
  return lv_launch(h, L, u, stream, "dg_project_gaussian");
}
