// Explicit time stepping of the semi-discrete system M du/dt + A u = f
// (Sec. 2.2, eq. (ODE_system)) by the strong-stability-preserving two-stage
// Runge-Kutta method (Heun), the scheme of the paper's transport example
// (Sec. 5.4).  The orthonormal tensor Legendre basis makes the mass matrix
// diagonal, M = |T| I on cell T, so each stage is one operator application
// and one elementwise update:
//   u1 = u + dt M^{-1} (f - A u)
//   u  <- (u + u1 + dt M^{-1} (f - A u1)) / 2.
// With the fused operator kernels each stage is a single launch: the kernel
// that produces (A x) at a point writes the stage value there instead, so
// A u is never stored (per step: read u, u1 and f twice or once, write u1
// and u once, on top of the operator's own reads).  The reference-variant
// kernels keep a separate elementwise pass over a stored A u (k_heun_stage).
// |T| comes from the per-axis spacing tables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "dg_internal.h"

namespace dgmf {

constexpr int kTsThreads = 256;

// STAGE 0: out = u + dt (f - Au) / |T|
// STAGE 1: out = (u + u1 + dt (f - Au) / |T|) / 2   (out may alias u)
template <int STAGE>
__global__ __launch_bounds__(kTsThreads) void k_heun_stage(const double *u, const double *__restrict__ u1,
                                                           const double *__restrict__ Au,
                                                           const double *__restrict__ f, DevMesh M, int nb,
                                                           int64_t ndof, double dt, double *out) {
  for (int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; g < ndof;
       g += int64_t(gridDim.x) * blockDim.x) {
    const int64_t c = g / nb;
    const int i0 = int(c % M.ncell[0]);
    const int64_t r = c / M.ncell[0];
    const int i1 = int(r % M.ncell[1]), i2 = int(r / M.ncell[1]);
    const double vol = M.h[0][i0] * M.h[1][i1] * M.h[2][i2];
    const double rhs = (f ? f[g] : 0.0) - Au[g];
    if (STAGE == 0)
      out[g] = fma(dt / vol, rhs, u[g]);
    else
      out[g] = 0.5 * (u[g] + u1[g] + dt / vol * rhs);
  }
}

static int ts_grid(int64_t n) { return int(std::min<int64_t>((n + kTsThreads - 1) / kTsThreads, 1 << 20)); }

}  // namespace dgmf

using namespace dgmf;

extern "C" dg_status dg_heun(dg_handle *h, double *u, const double *f, double dt, int32_t nsteps, void *stream) {
  if (!h) return set_error(DG_EINVAL, "dg_heun: handle is NULL");
  if (!u) return set_error(DG_EINVAL, "dg_heun: u is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(DG_EINVAL, "dg_heun: dt must be positive and finite");
  if (nsteps < 0) return set_error(DG_EINVAL, "dg_heun: nsteps must be >= 0");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != h->device) {
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_error(e, "dg_heun: hipSetDevice");
  }
  const size_t n = size_t(h->ndof);
  if (f && ((f < u + n && u < f + n))) return set_error(DG_EINVAL, "dg_heun: u and f overlap");
  // two vectors (u1 and, for the reference variant, A u) whatever the
  // variant, which dg_set_kernel may change between calls
  if (!h->ts) {
    hipError_t e = hipMalloc(&h->ts, 2 * n * sizeof(double));
    if (e != hipSuccess) {
      h->ts = nullptr;
      return hip_error(e, "dg_heun: workspace");
    }
  }
  const hipStream_t s = static_cast<hipStream_t>(stream);
  dt /= h->vol_scale;  // |T| of the physical cells: |det A| times the tensor-grid volumes
  if (h->variant != DG_KERNEL_REFERENCE && !h->quad_extra) {
    double *u1 = h->ts;
    for (int step = 0; step < nsteps; ++step) {
      hipError_t e = launch_heun_fused_f64(h, u, u1, f, dt, 0, s);
      if (e == hipSuccess) e = launch_heun_fused_f64(h, u1, u, f, dt, 1, s);
      if (e != hipSuccess) return hip_error(e, "dg_heun: stage");
    }
    return DG_OK;
  }
  double *u1 = h->ts, *Au = h->ts + n;
  const int nb = (h->k + 1) * (h->k + 1) * (h->k + 1);
  const int grid = ts_grid(int64_t(n));
  for (int step = 0; step < nsteps; ++step) {
    hipError_t e = apply_f64(h, u, Au, s);
    if (e != hipSuccess) return hip_error(e, "dg_heun: apply");
    hipLaunchKernelGGL(k_heun_stage<0>, dim3(grid), dim3(kTsThreads), 0, s, u, nullptr, Au, f, h->mesh, nb,
                       int64_t(n), dt, u1);
    if ((e = apply_f64(h, u1, Au, s)) != hipSuccess) return hip_error(e, "dg_heun: apply");
    hipLaunchKernelGGL(k_heun_stage<1>, dim3(grid), dim3(kTsThreads), 0, s, u, u1, Au, f, h->mesh, nb,
                       int64_t(n), dt, u);
    if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "dg_heun: stage update");
  }
  return DG_OK;
}
