// Krylov kernels (krylov.hip) and the restarted, right-preconditioned GMRES
// template used by the solve entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "dg_internal.h"

namespace dgmf {

constexpr int kRedBlocks = 1024;  // fixed reduction grid (deterministic sums)
constexpr int kMaxBasis = 64;     // restart <= kMaxBasis - 1
constexpr size_t kBasisAlign = 64;  // basis vectors start 16-byte (and 256-byte) aligned

// out[0..nv) = V_k . w, out[nv] = w . w
template <typename T>
hipError_t kr_multidot(const T *V, size_t ld, int nv, const T *w, size_t n, double *partial,
                       double *out, hipStream_t s);
template <typename T, bool DOT, bool NORM>
hipError_t kr_orth(const T *V, size_t ld, int nv, const double *h, const T *w, T *wout, double scale,
                   size_t n, double *partial, double *out, hipStream_t s);
template <typename TI, typename TO>
hipError_t kr_scale(const TI *x, TO *y, double alpha, size_t n, hipStream_t s);
template <typename TZ, typename TO>
hipError_t kr_lincomb(TO *out, const TZ *Z, size_t ld, int nz, const double *c, double scale,
                      bool acc, size_t n, hipStream_t s);
template <typename TX, typename TY>
hipError_t kr_axpy(const TX *x, TY *y, double alpha, size_t n, hipStream_t s);
template <typename T>
hipError_t kr_residual(const T *b, T *r, size_t n, double *partial, double *out, hipStream_t s);
template <typename T>
hipError_t kr_norm2(const T *x, size_t n, double *partial, double *out, hipStream_t s);

// Device buffers of one GMRES instance (owned by the handle).
struct KrylovBufs {
  void *V = nullptr;   // (restart+1) x ld basis
  void *Z = nullptr;   // restart x ld (flexible) or n (fixed preconditioner)
  void *w = nullptr;   // n
  size_t n = 0;
  size_t ld = 0;       // basis stride: n rounded up to kBasisAlign entries
  int restart = 0;
  bool flex = false;
  bool reorth = false;  // CGS2 (second projection) instead of CGS1
};

struct GmresOut {
  int iters = 0;     // Arnoldi steps (= operator applications in the cycles)
  int cycles = 0;
  int applies = 0;   // every operator application, residuals included
  double rel = 0.0;  // true residual / bnorm at the last restart
  bool converged = false;
  bool nan = false;
};

// Restarted GMRES(m) for A u = b with right preconditioning M:
//   op(x, y):   y = A x            (vectors of T)
//   prec(v, z): z = M^{-1} v       (only called if have_prec)
// Each cycle starts from the true residual r = b - A u, and the solver only
// reports convergence on that true residual (||r|| <= tol * bnorm).  Inside a
// cycle the Givens estimate decides when to stop early.  Exits after maxit
// Arnoldi steps, after max_cycles cycles (0: no limit; the last cycle's update
// is then not followed by a residual), or on a non-finite value.
// zero_guess: u is zero on entry (the first residual is b, no apply).
// scratch: kRedBlocks*kMaxBasis doubles; small: 3*kMaxBasis doubles (device).
template <typename T, typename Op, typename Prec>
hipError_t gmres(KrylovBufs &K, Op &&op, Prec &&prec, bool have_prec, const T *b, T *u, double bnorm,
                 double tol, int maxit, int max_cycles, bool zero_guess, double *scratch, double *small,
                 hipStream_t s, GmresOut &out) {
  const size_t n = K.n, ld = K.ld;
  const int m = K.restart;
  T *V = static_cast<T *>(K.V);
  T *Z = static_cast<T *>(K.Z);
  T *w = static_cast<T *>(K.w);
  std::vector<double> H(size_t(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), y(m);
  std::vector<double> hb(2 * kMaxBasis);
  double *h1 = small, *h2 = small + kMaxBasis, *yd = small + 2 * kMaxBasis;
  hipError_t e;
  out = GmresOut();
  bool first = true;
  for (;;) {
    // V0 = b - A u, beta = ||V0||
    if (first && zero_guess) {
      if ((e = kr_scale<T, T>(b, V, 1.0, n, s)) != hipSuccess) return e;
      if ((e = kr_norm2<T>(V, n, scratch, small, s)) != hipSuccess) return e;
    } else {
      if ((e = op(u, V)) != hipSuccess) return e;
      ++out.applies;
      if ((e = kr_residual<T>(b, V, n, scratch, small, s)) != hipSuccess) return e;
    }
    first = false;
    if ((e = hipMemcpyAsync(hb.data(), small, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    const double beta = std::sqrt(hb[0]);
    if (!std::isfinite(beta)) {
      out.nan = true;
      return hipSuccess;
    }
    out.rel = beta / bnorm;
    if (out.rel <= tol || beta == 0.0) {
      out.converged = true;
      return hipSuccess;
    }
    if (out.iters >= maxit) return hipSuccess;
    ++out.cycles;
    if ((e = kr_scale<T, T>(V, V, 1.0 / beta, n, s)) != hipSuccess) return e;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jdone = 0;
    for (int j = 0; j < m && out.iters < maxit; ++j) {
      T *vj = V + size_t(j) * ld;
      T *zj = have_prec ? (K.flex ? Z + size_t(j) * ld : Z) : vj;
      if (have_prec && (e = prec(vj, zj)) != hipSuccess) return e;
      if ((e = op(zj, w)) != hipSuccess) return e;
      ++out.applies;
      const int nv = j + 1;
      // Classical Gram-Schmidt: pass 1 gives h1 = V^T w and ||w||^2, and the
      // norm of w - V h1 is ||w||^2 - ||h1||^2.  A second projection (CGS2:
      // w -= V h1; h2 = V^T w, ||w||^2) runs when K.reorth asks for it, or
      // when the first one cancels w below 1e-4 of its norm, where that
      // difference would have lost half its digits.  The last pass writes
      // v_{j+1} = (w - V h) / hn with the last projection h.
      double *Hj = H.data() + size_t(j) * (m + 1);
      bool bad = false;
      double wsq = 0.0;
      const double *hlast = h1;
      if ((e = kr_multidot<T>(V, ld, nv, w, n, scratch, h1, s)) != hipSuccess) return e;
      bool second = K.reorth;
      if (second) {
        if ((e = kr_orth<T, true, true>(V, ld, nv, h1, w, w, 1.0, n, scratch, h2, s)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(hb.data(), small, sizeof(double) * (kMaxBasis + nv + 1), hipMemcpyDeviceToHost,
                                s)) != hipSuccess)
          return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
      } else {
        if ((e = hipMemcpyAsync(hb.data(), h1, sizeof(double) * (nv + 1), hipMemcpyDeviceToHost, s)) != hipSuccess)
          return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        double h1sq = 0.0;
        for (int i = 0; i < nv; ++i) h1sq += hb[i] * hb[i];
        wsq = hb[nv] - h1sq;
        if (std::isfinite(wsq) && !(wsq > 1e-8 * hb[nv])) {
          second = true;
          if ((e = kr_orth<T, true, true>(V, ld, nv, h1, w, w, 1.0, n, scratch, h2, s)) != hipSuccess) return e;
          if ((e = hipMemcpyAsync(hb.data() + kMaxBasis, h2, sizeof(double) * (nv + 1), hipMemcpyDeviceToHost, s)) !=
              hipSuccess)
            return e;
          if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        }
      }
      double colsq = 0.0;
      if (second) {
        double h2sq = 0.0;
        for (int i = 0; i < nv; ++i) {
          Hj[i] = hb[i] + hb[kMaxBasis + i];
          h2sq += hb[kMaxBasis + i] * hb[kMaxBasis + i];
        }
        wsq = hb[kMaxBasis + nv] - h2sq;
        hlast = h2;
      } else {
        for (int i = 0; i < nv; ++i) Hj[i] = hb[i];
      }
      for (int i = 0; i < nv; ++i) {
        colsq += Hj[i] * Hj[i];
        bad = bad || !std::isfinite(Hj[i]);
      }
      const double hn = std::sqrt(std::max(wsq, 0.0));
      if (bad || !std::isfinite(hn)) {
        out.nan = true;
        return hipSuccess;
      }
      // invariant subspace (lucky breakdown) when the new direction vanishes
      const bool breakdown = !(hn > 1e-14 * std::sqrt(colsq + hn * hn));
      Hj[j + 1] = breakdown ? 0.0 : hn;
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * Hj[i] + sn[i] * Hj[i + 1];
        Hj[i + 1] = -sn[i] * Hj[i] + cs[i] * Hj[i + 1];
        Hj[i] = t;
      }
      const double den = std::hypot(Hj[j], Hj[j + 1]);
      cs[j] = den > 0 ? Hj[j] / den : 1.0;
      sn[j] = den > 0 ? Hj[j + 1] / den : 0.0;
      Hj[j] = den;
      Hj[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++out.iters;
      jdone = j + 1;
      if (std::fabs(g[j + 1]) <= tol * bnorm || breakdown) break;
      // v_{j+1} = (w - V h2) / hn  (not needed after the last step of a cycle)
      if (j + 1 < m && out.iters < maxit &&
          (e = kr_orth<T, false, false>(V, ld, nv, hlast, w, V + size_t(j + 1) * ld, 1.0 / hn, n, scratch,
                                        nullptr, s)) != hipSuccess)
        return e;
    }
    // y = R^{-1} g (back substitution on the rotated Hessenberg matrix)
    for (int i = jdone - 1; i >= 0; --i) {
      double t = g[i];
      for (int k = i + 1; k < jdone; ++k) t -= H[size_t(k) * (m + 1) + i] * y[k];
      const double d = H[size_t(i) * (m + 1) + i];
      y[i] = d != 0.0 ? t / d : 0.0;
    }
    if ((e = hipMemcpyAsync(yd, y.data(), sizeof(double) * jdone, hipMemcpyHostToDevice, s)) != hipSuccess)
      return e;
    if (have_prec && !K.flex) {
      // u += M^{-1} (V y)
      if ((e = kr_lincomb<T, T>(w, V, ld, jdone, yd, 1.0, false, n, s)) != hipSuccess) return e;
      if ((e = prec(w, Z)) != hipSuccess) return e;
      if ((e = kr_axpy<T, T>(Z, u, 1.0, n, s)) != hipSuccess) return e;
    } else {
      if ((e = kr_lincomb<T, T>(u, have_prec ? Z : V, ld, jdone, yd, 1.0, true, n, s)) != hipSuccess)
        return e;
    }
    // y is read by the update kernel: keep the host copy alive until then
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    if (max_cycles > 0 && out.cycles >= max_cycles) return hipSuccess;
  }
}

}  // namespace dgmf
