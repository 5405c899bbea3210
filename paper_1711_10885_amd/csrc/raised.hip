// The operator with the raised Gauss rule (q = 2p + 4: k + 3 points per
// direction, Problem B of Sec. 5.1) on the tuned kernels.  The orthonormal
// Legendre basis is hierarchical, and the fused kernel of degree k + 2 uses
// exactly k + 3 Gauss points, so for x in the degree-k space
//   (A_raised x)_i = (A_{k+2} P x)_i  for every mode i <= k,
// with P the zero padding of the modes above k; the penalty sigma is the
// problem's own (it is a parameter of the form, not of the kernel degree) and
// the coefficient tables are already tabulated at the k + 3 points.  One
// apply = pad, the degree-(k+2) kernel, restriction; the two padded vectors
// live in a workspace the handle allocates at setup.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dg_internal.h"

namespace dgmf {

constexpr int kRqThreads = 256;

// xp[c][j1 + M j2 + M^2 j3] = x[c][j1 + N j2 + N^2 j3] for j < N, else 0
template <typename T>
__global__ __launch_bounds__(kRqThreads) void k_pad(const T *__restrict__ x, T *__restrict__ xp, int N, int M,
                                                    int64_t total) {
  for (int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; g < total; g += int64_t(gridDim.x) * blockDim.x) {
    const int MMM = M * M * M;
    const int64_t c = g / MMM;
    const int r = int(g - c * MMM);
    const int j1 = r % M, j2 = (r / M) % M, j3 = r / (M * M);
    xp[g] = (j1 < N && j2 < N && j3 < N) ? x[c * (N * N * N) + j1 + N * (j2 + N * j3)] : T(0);
  }
}

// y[c][j] = yp[c][j padded], j < N^3
template <typename T>
__global__ __launch_bounds__(kRqThreads) void k_restrict(const T *__restrict__ yp, T *__restrict__ y, int N, int M,
                                                         int64_t total) {
  for (int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; g < total; g += int64_t(gridDim.x) * blockDim.x) {
    const int NNN = N * N * N;
    const int64_t c = g / NNN;
    const int r = int(g - c * NNN);
    const int j1 = r % N, j2 = (r / N) % N, j3 = r / (N * N);
    y[g] = yp[c * (M * M * M) + j1 + M * (j2 + M * j3)];
  }
}

static unsigned rq_grid(int64_t n) { return unsigned(std::min<int64_t>((n + kRqThreads - 1) / kRqThreads, 1 << 20)); }

template <typename T>
static hipError_t apply_raised(const dg_handle *h, const T *x, T *y, hipStream_t s) {
  const int N = h->k + 1, M = N + h->quad_extra;
  const int64_t np = h->ncells * int64_t(M) * M * M;
  if (!h->rq || h->rq_bytes < 2 * size_t(np) * sizeof(T)) return hipErrorInvalidValue;
  T *xp = static_cast<T *>(h->rq), *yp = xp + np;
  hipLaunchKernelGGL(k_pad<T>, dim3(rq_grid(np)), dim3(kRqThreads), 0, s, x, xp, N, M, np);
  hipError_t e = (sizeof(T) == 8) ? launch_apply_fused_f64(h, reinterpret_cast<const double *>(xp),
                                                           reinterpret_cast<double *>(yp), s)
                                  : launch_apply_fused_f32(h, reinterpret_cast<const float *>(xp),
                                                           reinterpret_cast<float *>(yp), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_restrict<T>, dim3(rq_grid(h->ndof)), dim3(kRqThreads), 0, s, yp, y, N, M, int64_t(h->ndof));
  return hipGetLastError();
}

hipError_t apply_raised_f64(const dg_handle *h, const double *x, double *y, hipStream_t s) {
  return apply_raised<double>(h, x, y, s);
}

hipError_t apply_raised_f32(const dg_handle *h, const float *x, float *y, hipStream_t s) {
  return apply_raised<float>(h, x, y, s);
}

}  // namespace dgmf
