// dg_solve: restarted GMRES around the matrix-free operator.
//
// The operator application is the hot kernel; the solver adds HBM-bound
// vector passes (krylov.hip) and one host synchronisation per Arnoldi step
// (the Hessenberg column and the Givens rotations live on the host).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <string>

#include "dg_internal.h"
#include "krylov.h"

namespace dgmf {

void release_solver(dg_handle *h) {
  if (h->ws) (void)hipFree(h->ws);
  if (h->red) (void)hipFree(h->red);
  h->ws = nullptr;
  h->ws_bytes = 0;
  h->red = nullptr;
}

static dg_status ensure_workspace(dg_handle *h, size_t bytes) {
  if (!h->red) {
    hipError_t e = hipMalloc(&h->red, sizeof(double) * (size_t(kRedBlocks) * kMaxBasis + 3 * kMaxBasis));
    if (e != hipSuccess) {
      h->red = nullptr;
      return hip_error(e, "dg_solve: reduction buffer");
    }
  }
  if (bytes <= h->ws_bytes) return DG_OK;
  if (h->ws) (void)hipFree(h->ws);
  h->ws = nullptr;
  h->ws_bytes = 0;
  hipError_t e = hipMalloc(&h->ws, bytes);
  if (e != hipSuccess) {
    h->ws = nullptr;
    return hip_error(e, "dg_solve: Krylov workspace");
  }
  h->ws_bytes = bytes;
  return DG_OK;
}

// ||x||^2 of a device vector (synchronises s).
static hipError_t norm2_sync(dg_handle *h, const double *x, size_t n, hipStream_t s, double &out) {
  double *small = h->red + size_t(kRedBlocks) * kMaxBasis;
  hipError_t e = kr_norm2<double>(x, n, h->red, small, s);
  if (e != hipSuccess) return e;
  if ((e = hipMemcpyAsync(&out, small, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace dgmf

using namespace dgmf;

extern "C" dg_status dg_solve(dg_handle *h, const double *f, double *u, double tol, const dg_solve_opts *o,
                              dg_solve_stats *st, void *stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!h) return set_error(DG_EINVAL, "dg_solve: handle is NULL");
  if (!f || !u) return set_error(DG_EINVAL, "dg_solve: f or u is NULL");
  const size_t n = size_t(h->ndof);
  {
    const char *a = reinterpret_cast<const char *>(f), *b = reinterpret_cast<const char *>(u);
    if (a < b + n * sizeof(double) && b < a + n * sizeof(double))
      return set_error(DG_EINVAL, "dg_solve: f and u overlap");
  }
  if (!(tol > 0.0) || !std::isfinite(tol)) return set_error(DG_EINVAL, "dg_solve: tol must be positive");
  dg_solve_opts opt{DG_GMRES64, DG_PREC_NONE, 30, 20000, 1e-4};
  if (o) opt = *o;
  if (opt.restart < 1 || opt.restart > kMaxBasis - 1)
    return set_error(DG_EINVAL, "dg_solve: restart must be in 1..63");
  if (opt.maxit < 1) return set_error(DG_EINVAL, "dg_solve: maxit must be >= 1");
  if (opt.method != DG_GMRES64) return set_error(DG_EINVAL, "dg_solve: unknown method");
  if (opt.precond != DG_PREC_NONE && opt.precond != DG_PREC_BLOCK_JACOBI)
    return set_error(DG_EINVAL, "dg_solve: unknown preconditioner");
  if (opt.precond == DG_PREC_BLOCK_JACOBI && !h->bj)
    return set_error(DG_EINVAL, "dg_solve: handle was set up without DG_WITH_BLOCK_JACOBI");

  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != h->device) {
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_error(e, "dg_solve: hipSetDevice");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int m = opt.restart;

  const bool have_prec = opt.precond != DG_PREC_NONE;
  // workspace: V (m+1) n | w n | Z n (fixed preconditioner)
  const size_t vb = align256(sizeof(double) * n * (m + 1)), wb = align256(sizeof(double) * n);
  dg_status ds = ensure_workspace(h, vb + wb + (have_prec ? wb : 0));
  if (ds != DG_OK) return ds;
  char *base = static_cast<char *>(h->ws);
  KrylovBufs K;
  K.V = base;
  K.w = base + vb;
  K.Z = have_prec ? base + vb + wb : nullptr;
  K.n = n;
  K.restart = m;
  K.flex = false;
  double *scratch = h->red, *small = h->red + size_t(kRedBlocks) * kMaxBasis;

  dg_solve_stats stats{};
  double fn2 = 0.0, un2 = 0.0;
  hipError_t e = norm2_sync(h, f, n, s, fn2);
  if (e == hipSuccess) e = norm2_sync(h, u, n, s, un2);
  if (e != hipSuccess) return hip_error(e, "dg_solve: norm");
  if (!std::isfinite(fn2) || !std::isfinite(un2)) return set_error(DG_ENAN, "dg_solve: f or u is not finite");
  const double fnorm = std::sqrt(fn2);
  if (fnorm == 0.0) {
    // A u = 0 has the solution u = 0
    e = kr_scale<double, double>(u, u, 0.0, n, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_error(e, "dg_solve: zero solution");
    if (st) {
      *st = stats;
      st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return DG_OK;
  }
  auto op = [h, s](const double *x, double *y) { return apply_f64(h, x, y, s); };
  auto prec = [h, s](const double *v, double *z) { return bj_apply<double, double>(h, v, z, s); };
  GmresOut go;
  e = gmres<double>(K, op, prec, have_prec, f, u, fnorm, tol, opt.maxit, 0, un2 == 0.0, scratch, small, s, go);
  if (e != hipSuccess) return hip_error(e, "dg_solve: GMRES");
  stats.iters = go.iters;
  stats.outer = go.cycles;
  stats.applies = go.applies;
  stats.rel_resid = go.rel;
  stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = stats;
  if (go.nan) return set_error(DG_ENAN, "dg_solve: non-finite value in the iteration");
  if (!go.converged)
    return set_error(DG_ENOTCONV, "dg_solve: maxit reached at relative residual " + std::to_string(go.rel));
  return DG_OK;
}
