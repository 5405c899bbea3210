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
#include <mutex>
#include <string>

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

// the stage update fused into the operator kernel's store (tuned kernels),
// else an apply into A u and a separate stage pass (reference kernel)
static bool heun_is_fused(const dg_handle *h) { return h->variant != DG_KERNEL_REFERENCE; }

}  // namespace dgmf

// Fixed workspace of dg_heun_noalloc: the stage vector u1 (and A u on the
// paths with a separate stage pass) for callers that cannot allocate.  One
// copy per device, resident while the library is loaded.  Host code never
// passes the array's name to a kernel (on the host it is a stand-in, not a
// device address): it uses the per-device address that
// dgmf::static_scratch_init resolves with hipGetSymbolAddress.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

namespace dgmf {

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxScratchDevices];

dg_status static_scratch_init(int device) {
  if (device < 0 || device >= kMaxScratchDevices)
    return set_error(DG_EINVAL, "dg_setup: device index beyond the static workspace table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return DG_OK;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                "dg_setup: address of the static workspace");
  g_scratch_ptr[device] = static_cast<double *>(ptr);
  return DG_OK;
}

// The Heun steps of dg_heun and dg_heun_noalloc on the given workspace: u1
// (ndof doubles) and, on the paths with a separate stage pass, Au (ndof
// doubles; may be null on the fused path).
static dg_status heun_steps(dg_handle *h, double *u, const double *f, double dt, int32_t nsteps, hipStream_t s,
                            double *u1, double *Au, const char *who) {
  const size_t n = size_t(h->ndof);
  dt /= h->vol_scale;  // |T| of the physical cells: |det A| times the tensor-grid volumes
  if (heun_is_fused(h)) {
    for (int step = 0; step < nsteps; ++step) {
      hipError_t e = launch_heun_fused_f64(h, u, u1, f, dt, 0, s);
      if (e == hipSuccess) e = launch_heun_fused_f64(h, u1, u, f, dt, 1, s);
      if (e != hipSuccess) return hip_error(e, who);
    }
    return DG_OK;
  }
  const int nb = (h->k + 1) * (h->k + 1) * (h->k + 1);
  const int grid = ts_grid(int64_t(n));
  for (int step = 0; step < nsteps; ++step) {
    hipError_t e = apply_f64(h, u, Au, s);
    if (e != hipSuccess) return hip_error(e, who);
    hipLaunchKernelGGL(k_heun_stage<0>, dim3(grid), dim3(kTsThreads), 0, s, u, nullptr, Au, f, h->mesh, nb,
                       int64_t(n), dt, u1);
    if ((e = apply_f64(h, u1, Au, s)) != hipSuccess) return hip_error(e, who);
    hipLaunchKernelGGL(k_heun_stage<1>, dim3(grid), dim3(kTsThreads), 0, s, u, u1, Au, f, h->mesh, nb,
                       int64_t(n), dt, u);
    if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, who);
  }
  return DG_OK;
}

static dg_status heun_check(dg_handle *h, double *u, const double *f, double dt, int32_t nsteps, const char *who) {
  if (!h) return set_error(DG_EINVAL, std::string(who) + ": handle is NULL");
  if (!u) return set_error(DG_EINVAL, std::string(who) + ": u is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt))
    return set_error(DG_EINVAL, std::string(who) + ": dt must be positive and finite");
  if (nsteps < 0) return set_error(DG_EINVAL, std::string(who) + ": nsteps must be >= 0");
  if (h->mesh.multilinear)
    return set_error(DG_EINVAL, std::string(who) + ": the mass matrix of multilinear cells is not diagonal");
  const size_t n = size_t(h->ndof);
  if (f && ((f < u + n && u < f + n))) return set_error(DG_EINVAL, std::string(who) + ": u and f overlap");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != h->device) {
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_error(e, who);
  }
  return DG_OK;
}

}  // namespace dgmf

using namespace dgmf;

extern "C" dg_status dg_heun(dg_handle *h, double *u, const double *f, double dt, int32_t nsteps, void *stream) {
  dg_status st = heun_check(h, u, f, dt, nsteps, "dg_heun");
  if (st != DG_OK) return st;
  const size_t n = size_t(h->ndof);
  // two vectors (u1 and, for the reference variant, A u) whatever the
  // variant, which dg_set_kernel may change between calls
  if (!h->ts) {
    hipError_t e = hipMalloc(&h->ts, 2 * n * sizeof(double));
    if (e != hipSuccess) {
      h->ts = nullptr;
      return hip_error(e, "dg_heun: workspace");
    }
  }
  return heun_steps(h, u, f, dt, nsteps, static_cast<hipStream_t>(stream), h->ts, h->ts + n, "dg_heun: stage");
}

extern "C" dg_status dg_heun_noalloc(dg_handle *h, double *u, const double *f, double dt, int32_t nsteps,
                                     void *stream) {
  dg_status st = heun_check(h, u, f, dt, nsteps, "dg_heun_noalloc");
  if (st != DG_OK) return st;
  double *ws = (h->device >= 0 && h->device < kMaxScratchDevices) ? g_scratch_ptr[h->device] : nullptr;
  if (!ws) return set_error(DG_EINVAL, "dg_heun_noalloc: the static workspace of this device is not set up");
  const size_t n = size_t(h->ndof);
  const size_t need = (heun_is_fused(h) ? 1 : 2) * n * sizeof(double);
  if (need > kStaticScratchBytes)
    return set_error(DG_EINVAL, "dg_heun_noalloc: needs " + std::to_string(need) + " bytes of workspace, above the " +
                                    std::to_string(kStaticScratchBytes) + "-byte static limit (use dg_heun)");
  return heun_steps(h, u, f, dt, nsteps, static_cast<hipStream_t>(stream), ws, heun_is_fused(h) ? nullptr : ws + n,
                    "dg_heun_noalloc: stage");
}
