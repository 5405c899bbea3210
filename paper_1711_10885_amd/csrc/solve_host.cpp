// dg_solve: restarted GMRES around the matrix-free operator.
//
// The operator application is the hot kernel; the solver adds HBM-bound
// vector passes (krylov.hip) and one host synchronisation per Arnoldi step
// (the Hessenberg column and the Givens rotations live on the host).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "dg_internal.h"
#include "krylov.h"

namespace dgmf {

static std::string sci(double v) {
  char buf[32];
  std::snprintf(buf, sizeof buf, "%.3e", v);
  return buf;
}

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
  dg_solve_opts opt{DG_GMRES64, DG_PREC_NONE, 30, 20000, DG_ORTH_CGS1, 1e-4};
  if (o) opt = *o;
  if (opt.restart < 1 || opt.restart > kMaxBasis - 1)
    return set_error(DG_EINVAL, "dg_solve: restart must be in 1..63");
  if (opt.maxit < 1) return set_error(DG_EINVAL, "dg_solve: maxit must be >= 1");
  if (opt.orth != DG_ORTH_CGS1 && opt.orth != DG_ORTH_CGS2)
    return set_error(DG_EINVAL, "dg_solve: orth must be DG_ORTH_CGS1 or DG_ORTH_CGS2");
  if (opt.method != DG_GMRES64 && opt.method != DG_GMRES_IR && opt.method != DG_FGMRES)
    return set_error(DG_EINVAL, "dg_solve: unknown method");
  if (opt.method == DG_GMRES_IR && h->mesh.multilinear)
    return set_error(DG_EINVAL, "dg_solve: the FP32 tier is not available on multilinear meshes");
  if (opt.method == DG_GMRES_IR && !(opt.inner_tol > 0.0 && opt.inner_tol < 1.0))
    return set_error(DG_EINVAL, "dg_solve: inner_tol must be in (0, 1)");
  if (opt.precond != DG_PREC_NONE && opt.precond != DG_PREC_BLOCK_JACOBI && opt.precond != DG_PREC_LEARNED)
    return set_error(DG_EINVAL, "dg_solve: unknown preconditioner");
  if (opt.precond != DG_PREC_NONE && !h->bj)
    return set_error(DG_EINVAL, "dg_solve: handle was set up without DG_WITH_BLOCK_JACOBI");
  if (opt.precond == DG_PREC_LEARNED && opt.method != DG_FGMRES)
    return set_error(DG_EINVAL, "dg_solve: the learned preconditioner needs DG_FGMRES");
  if (opt.precond == DG_PREC_LEARNED && !learned_ready(h))
    return set_error(DG_EINVAL, "dg_solve: no trained or loaded network");

  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != h->device) {
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_error(e, "dg_solve: hipSetDevice");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int m = opt.restart;

  const bool have_prec = opt.precond != DG_PREC_NONE;
  const bool ir = opt.method == DG_GMRES_IR;
  const bool flex = opt.method == DG_FGMRES;
  // workspace, FP64 GMRES:  V (m+1) n | w n | Z n (fixed preconditioner)
  //            FGMRES:      V (m+1) n | w n | Z m n
  //            GMRES-IR:    r n (FP64) | V (m+1) n | w n | Z n | d n | r n (FP32)
  const size_t es = ir ? sizeof(float) : sizeof(double);
  const size_t ld = (n + kBasisAlign - 1) / kBasisAlign * kBasisAlign;
  const size_t vb = align256(es * ld * (m + 1)), wb = align256(es * n), rb = ir ? align256(sizeof(double) * n) : 0;
  const size_t zb = flex ? align256(es * ld * m) : (have_prec ? wb : 0);
  dg_status ds = ensure_workspace(h, rb + vb + wb + zb + (ir ? 2 * wb : 0));
  if (ds != DG_OK) return ds;
  char *base = static_cast<char *>(h->ws);
  double *r64 = ir ? reinterpret_cast<double *>(base) : nullptr;
  KrylovBufs K;
  K.V = base + rb;
  K.w = base + rb + vb;
  K.Z = (have_prec || flex) ? base + rb + vb + wb : nullptr;
  float *d32 = ir ? reinterpret_cast<float *>(base + rb + vb + wb + zb) : nullptr;
  float *r32 = ir ? reinterpret_cast<float *>(base + rb + vb + 2 * wb + zb) : nullptr;
  K.n = n;
  K.ld = ld;
  K.restart = m;
  K.flex = flex;
  K.reorth = opt.orth == DG_ORTH_CGS2;
  double *scratch = h->red, *small = h->red + size_t(kRedBlocks) * kMaxBasis;

  dg_solve_stats stats{};
  stats.fallback_step = stats.fallback_cycle = -1;
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
  GmresOut go;
  if (flex) {
    // FGMRES(m), one cycle per call so that the true residual of every cycle
    // can decide the fallback to block Jacobi
    bool learned = opt.precond == DG_PREC_LEARNED;
    auto op = [h, s](const double *x, double *y) { return apply_f64(h, x, y, s); };
    // after a fallback the learned preconditioner continues as block Jacobi
    auto prec = [h, s, &learned, &opt](const double *v, double *z) {
      if (learned) return learned_apply<double>(h, v, z, s);
      if (opt.precond != DG_PREC_NONE) return bj_apply<double, double>(h, v, z, s);
      return kr_scale<double, double>(v, z, 1.0, size_t(h->ndof), s);
    };
    bool zero = un2 == 0.0;
    std::vector<double> hist;  // true residual at the start of each cycle
    for (;;) {
      GmresOut gc;
      e = gmres<double>(K, op, prec, true, f, u, fnorm, tol, opt.maxit - stats.iters, 1, zero, scratch, small, s, gc);
      if (e != hipSuccess) return hip_error(e, "dg_solve: FGMRES");
      zero = false;
      stats.iters += gc.iters;
      stats.outer += gc.cycles;
      stats.applies += gc.applies;
      stats.rel_resid = gc.rel;
      if (gc.nan) {
        if (!learned) {
          go.nan = true;
          break;
        }
        learned = false;  // the cycle was abandoned before its update
        stats.fallback_used = 1;
        stats.fallback_step = stats.iters;
        stats.fallback_cycle = stats.outer;
        stats.fallback_resid = hist.empty() ? 1.0 : hist.back();
        continue;
      }
      if (gc.converged) {
        go.converged = true;
        break;
      }
      // at maxit the next call only measures the true residual (no cycle)
      if (gc.cycles == 0) break;
      hist.push_back(gc.rel);
      // stagnation of the learned preconditioner: less than 10 % over the
      // last 10 cycles -> block Jacobi alone from here on
      if (learned && hist.size() > 10 && hist.back() > 0.9 * hist[hist.size() - 11]) {
        learned = false;
        stats.fallback_used = 1;
        stats.fallback_step = stats.iters;
        stats.fallback_cycle = stats.outer;
        stats.fallback_resid = gc.rel;
      }
    }
  } else if (!ir) {
    auto op = [h, s](const double *x, double *y) { return apply_f64(h, x, y, s); };
    auto prec = [h, s](const double *v, double *z) { return bj_apply<double, double>(h, v, z, s); };
    e = gmres<double>(K, op, prec, have_prec, f, u, fnorm, tol, opt.maxit, 0, un2 == 0.0, scratch, small, s, go);
    if (e != hipSuccess) return hip_error(e, "dg_solve: GMRES");
    stats.iters = go.iters;
    stats.outer = go.cycles;
    stats.applies = go.applies;
    stats.rel_resid = go.rel;
  } else {
    // GMRES-IR: FP64 residual and update, FP32 correction by one inner cycle
    auto op = [h, s](const float *x, float *y) { return apply_f32(h, x, y, s); };
    // the inner FP32 solve reads the FP16 copy of the inverse blocks
    auto prec = [h, s](const float *v, float *z) { return bj_apply<float, float>(h, v, z, s, true); };
    go = GmresOut();
    bool first = true;
    for (;;) {
      double rn2 = 0.0;
      if (first && un2 == 0.0) {
        e = kr_scale<double, double>(f, r64, 1.0, n, s);
        rn2 = fn2;
      } else {
        e = apply_f64(h, u, r64, s);
        ++stats.applies;
        if (e == hipSuccess) e = kr_residual<double>(f, r64, n, scratch, small, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&rn2, small, sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
      }
      first = false;
      if (e != hipSuccess) return hip_error(e, "dg_solve: IR residual");
      const double rn = std::sqrt(rn2);
      if (!std::isfinite(rn)) {
        go.nan = true;
        break;
      }
      stats.rel_resid = rn / fnorm;
      if (stats.rel_resid <= tol) {
        go.converged = true;
        break;
      }
      if (stats.iters >= opt.maxit) break;
      ++stats.outer;
      // inner problem A d = r / ||r|| in FP32, zero initial guess
      e = kr_scale<double, float>(r64, r32, 1.0 / rn, n, s);
      if (e == hipSuccess) e = kr_scale<float, float>(r32, d32, 0.0, n, s);
      if (e != hipSuccess) return hip_error(e, "dg_solve: IR scaling");
      GmresOut gi;
      e = gmres<float>(K, op, prec, have_prec, r32, d32, 1.0, opt.inner_tol,
                       std::min(m, opt.maxit - stats.iters), 1, true, scratch, small, s, gi);
      if (e != hipSuccess) return hip_error(e, "dg_solve: inner GMRES");
      stats.iters += gi.iters;
      stats.applies_f32 += gi.applies;
      if (gi.nan) {
        go.nan = true;
        break;
      }
      // u += ||r|| d
      if ((e = kr_axpy<float, double>(d32, u, rn, n, s)) != hipSuccess) return hip_error(e, "dg_solve: IR update");
    }
  }
  stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = stats;
  if (go.nan) return set_error(DG_ENAN, "dg_solve: non-finite value in the iteration");
  if (!go.converged)
    return set_error(DG_ENOTCONV,
                     "dg_solve: maxit reached at relative residual " + sci(stats.rel_resid));
  return DG_OK;
}
