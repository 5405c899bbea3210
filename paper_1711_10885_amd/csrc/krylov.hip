// Krylov building blocks (HBM-bound vector kernels) and the restarted GMRES
// used by dg_solve.
//
// The paper stops at the operator application and motivates it as the core of
// iterative solvers (Sec. 1); the solver here is restarted GMRES (Saad &
// Schultz) with right preconditioning and classical Gram-Schmidt.  Every pass
// over the Krylov basis is one fused kernel that reads each basis vector once:
//   pass 1: h1 = V^T w and ||w||^2 (k_multidot)
//   [pass 2, CGS2 or heavy cancellation only: w <- w - V h1, then h2 = V^T w
//           and ||w||^2 on the updated w in the same sweep (k_orth)]
//   last:   v_{j+1} = (w - V h) / h_{j+1,j}, written straight into the basis,
//           h the last projection; h_{j+1,j}^2 = ||w||^2 - ||h||^2 since V is
//           orthonormal (k_orth).
// The host reads the projections and ||w||^2 after the dot-product passes.
// Reductions are two-stage and deterministic: fixed grid, per-block partial
// sums in a fixed order, then one block per output.
#include <cmath>
#include <vector>

#include "krylov.h"

namespace dgmf {

constexpr int kRedThreads = 256;

// Block-wide sums of NV per-thread values; result k in sm[R + k], R = waves*NV.
template <int NV>
__device__ __forceinline__ void block_sum(const double (&v)[NV], double *sm) {
  constexpr int NW = kRedThreads / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = v[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) sm[wave * NV + i] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += sm[w * NV + threadIdx.x];
    sm[NW * NV + threadIdx.x] = s;
  }
  __syncthreads();
}

#define GRID_STRIDE(i, n)                                                              \
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < (n); \
       i += size_t(gridDim.x) * blockDim.x)

// Vectors are streamed with 16-byte loads (VW = 16 / sizeof(T) entries per
// lane and load); the entries beyond the last full vector (n % VW) are done
// by a scalar tail.  V_k = V + k*ld, w and wout must be 16-byte aligned and
// ld a multiple of VW (the solver pads ld).
template <typename T>
struct Vec16 {
  static constexpr int VW = 16 / int(sizeof(T));
  typedef T type __attribute__((ext_vector_type(16 / sizeof(T))));
};

// Basis vectors are processed in chunks of KR_CH (all of them when NVMAX <= 32,
// else 16; a chunk is re-read for the dot products when there are several).
#define KR_CH(NVMAX) ((NVMAX) <= 32 ? (NVMAX) : 16)
#define KR_NC(NVMAX) ((NVMAX) / KR_CH(NVMAX))

// Loads are issued first for all basis vectors of a chunk (branch-free:
// slots k >= nv re-read V_{nv-1} with coefficient 0, a cache hit), then the
// arithmetic runs; with the loads behind per-slot branches the compiler
// serialises load and use and the passes fall to a fraction of the HBM rate.

// partial[b*(nv+1) + k] = sum over block b of V_k[i] w[i]   (V_k = V + k*ld),
// and slot nv: sum over block b of w[i]^2
template <typename T, int NVMAX>
__global__ __launch_bounds__(kRedThreads) void k_multidot(const T *__restrict__ V, size_t ld, int nv,
                                                           const T *__restrict__ w, size_t n,
                                                           double *__restrict__ partial) {
  using vec = typename Vec16<T>::type;
  constexpr int VW = Vec16<T>::VW;
  constexpr int NA = NVMAX + 1;
  __shared__ double sm[(kRedThreads / 64 + 1) * NA];
  double acc[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) acc[k] = 0.0;
  const size_t nvec = n / VW;
  GRID_STRIDE(i, nvec) {
    const vec wv = reinterpret_cast<const vec *>(w)[i];
#pragma unroll
    for (int c = 0; c < KR_NC(NVMAX); ++c)
      if (c * KR_CH(NVMAX) < nv) {
        vec vv[KR_CH(NVMAX)];
#pragma unroll
        for (int k = 0; k < KR_CH(NVMAX); ++k) {
          const int kk = c * KR_CH(NVMAX) + k;
          vv[k] = reinterpret_cast<const vec *>(V + (kk < nv ? kk : nv - 1) * ld)[i];
        }
#pragma unroll
        for (int k = 0; k < KR_CH(NVMAX); ++k)
#pragma unroll
          for (int e = 0; e < VW; ++e)
            acc[c * KR_CH(NVMAX) + k] = fma(double(vv[k][e]), double(wv[e]), acc[c * KR_CH(NVMAX) + k]);
      }
#pragma unroll
    for (int e = 0; e < VW; ++e) acc[NVMAX] = fma(double(wv[e]), double(wv[e]), acc[NVMAX]);
  }
  for (size_t i = nvec * VW + blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x) {
    const double wi = double(w[i]);
#pragma unroll
    for (int k = 0; k < NVMAX; ++k)
      if (k < nv) acc[k] = fma(double(V[k * ld + i]), wi, acc[k]);
    acc[NVMAX] = fma(wi, wi, acc[NVMAX]);
  }
  // drop the slots k >= nv (products with V_{nv-1}) and pack the norm right
  // after the nv dots (static indices only: no scratch)
#pragma unroll
  for (int k = 0; k < NVMAX; ++k)
    if (k >= nv) acc[k] = (k == nv) ? acc[NVMAX] : 0.0;
  block_sum<NA>(acc, sm);
  if (threadIdx.x <= nv) partial[blockIdx.x * (nv + 1) + threadIdx.x] = sm[(kRedThreads / 64) * NA + threadIdx.x];
}

// wout <- scale * (w - sum_k h_k V_k); then DOT: partial sums of V_k . wout;
// NORM: partial sum of wout . wout (stored after the nv dots).
template <typename T, int NVMAX, bool DOT, bool NORM>
__global__ __launch_bounds__(kRedThreads) void k_orth(const T *__restrict__ V, size_t ld, int nv,
                                                       const double *__restrict__ h, const T *w, T *wout,
                                                       double scale, size_t n, double *__restrict__ partial) {
  using vec = typename Vec16<T>::type;
  constexpr int VW = Vec16<T>::VW;
  constexpr int NA = NVMAX + 1;
  __shared__ double sm[(kRedThreads / 64 + 1) * NA];
  __shared__ double hs[NVMAX];
  if (threadIdx.x < NVMAX) hs[threadIdx.x] = threadIdx.x < nv ? h[threadIdx.x] : 0.0;
  __syncthreads();
  double acc[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) acc[k] = 0.0;
  const size_t nvec = n / VW;
  constexpr int CH = KR_CH(NVMAX), NC = KR_NC(NVMAX);
  GRID_STRIDE(i, nvec) {
    const vec wv = reinterpret_cast<const vec *>(w)[i];
    double wi[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) wi[e] = double(wv[e]);
    vec vv[CH];
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (c * CH < nv) {
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const int kk = c * CH + k;
          vv[k] = reinterpret_cast<const vec *>(V + (kk < nv ? kk : nv - 1) * ld)[i];
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          const double hk = hs[c * CH + k];
#pragma unroll
          for (int e = 0; e < VW; ++e) wi[e] = fma(-hk, double(vv[k][e]), wi[e]);
        }
      }
    vec ov;
#pragma unroll
    for (int e = 0; e < VW; ++e) ov[e] = T(wi[e] * scale);
    reinterpret_cast<vec *>(wout)[i] = ov;
    if (DOT) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (c * CH < nv) {
          if (NC > 1) {  // one chunk: its vectors are still in registers
#pragma unroll
            for (int k = 0; k < CH; ++k) {
              const int kk = c * CH + k;
              vv[k] = reinterpret_cast<const vec *>(V + (kk < nv ? kk : nv - 1) * ld)[i];
            }
          }
#pragma unroll
          for (int k = 0; k < CH; ++k)
#pragma unroll
            for (int e = 0; e < VW; ++e) acc[c * CH + k] = fma(double(vv[k][e]), double(ov[e]), acc[c * CH + k]);
        }
    }
    if (NORM) {
#pragma unroll
      for (int e = 0; e < VW; ++e) acc[NVMAX] = fma(double(ov[e]), double(ov[e]), acc[NVMAX]);
    }
  }
  for (size_t i = nvec * VW + blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x) {
    double v[NVMAX];
    double wi = double(w[i]);
#pragma unroll
    for (int k = 0; k < NVMAX; ++k)
      if (k < nv) {
        v[k] = double(V[k * ld + i]);
        wi = fma(-hs[k], v[k], wi);
      }
    const T wt = T(wi * scale);
    wout[i] = wt;
    const double wr = double(wt);
    if (DOT) {
#pragma unroll
      for (int k = 0; k < NVMAX; ++k)
        if (k < nv) acc[k] = fma(v[k], wr, acc[k]);
    }
    if (NORM) acc[NVMAX] = fma(wr, wr, acc[NVMAX]);
  }
  if (DOT || NORM) {
    // the slots k >= nv hold products with V_{nv-1}: drop them, then pack
    // the norm right after the nv dots (static indices only: no scratch)
#pragma unroll
    for (int k = 0; k < NVMAX; ++k)
      if (!DOT || k >= nv) acc[k] = 0.0;
    if (NORM) {
#pragma unroll
      for (int k = 0; k < NVMAX; ++k)
        if (k == (DOT ? nv : 0)) acc[k] = acc[NVMAX];
    }
    block_sum<NA>(acc, sm);
    const int nout = (DOT ? nv : 0) + (NORM ? 1 : 0);
    if (threadIdx.x < nout) partial[blockIdx.x * nout + threadIdx.x] = sm[(kRedThreads / 64) * NA + threadIdx.x];
  }
}

// out[k] = sum_b partial[b*nv + k]   (one block per k, fixed order)
__global__ __launch_bounds__(kRedThreads) void k_reduce(const double *__restrict__ partial, int nb,
                                                        int nv, double *__restrict__ out) {
  __shared__ double sm[kRedThreads / 64 + 1];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += kRedThreads) s += partial[b * nv + blockIdx.x];
  const double v[1] = {s};
  block_sum<1>(v, sm);
  if (threadIdx.x == 0) out[blockIdx.x] = sm[kRedThreads / 64];
}

// y = alpha x   (precision conversion allowed)
template <typename TI, typename TO>
__global__ void k_scale(const TI *__restrict__ x, TO *__restrict__ y, double alpha, size_t n) {
  GRID_STRIDE(i, n) y[i] = TO(alpha * double(x[i]));
}

// out (+)= sum_k c_k Z_k    (Z_k = Z + k*ld), c in device memory
template <typename TZ, typename TO, bool ACC>
__global__ void k_lincomb(TO *__restrict__ out, const TZ *__restrict__ Z, size_t ld, int nz,
                          const double *__restrict__ c, double scale, size_t n) {
  __shared__ double cs[kMaxBasis];
  if (threadIdx.x < kMaxBasis) cs[threadIdx.x] = threadIdx.x < nz ? c[threadIdx.x] * scale : 0.0;
  __syncthreads();
  GRID_STRIDE(i, n) {
    double s = ACC ? double(out[i]) : 0.0;
    for (int k = 0; k < nz; ++k) s = fma(cs[k], double(Z[k * ld + i]), s);
    out[i] = TO(s);
  }
}

// r <- b - r  (r holds A u on entry), partial ||r||^2
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_residual(const T *__restrict__ b, T *__restrict__ r,
                                                          size_t n, double *__restrict__ partial) {
  __shared__ double sm[kRedThreads / 64 + 1];
  double acc = 0.0;
  GRID_STRIDE(i, n) {
    const T v = T(double(b[i]) - double(r[i]));
    r[i] = v;
    acc = fma(double(v), double(v), acc);
  }
  const double a[1] = {acc};
  block_sum<1>(a, sm);
  if (threadIdx.x == 0) partial[blockIdx.x] = sm[kRedThreads / 64];
}

// y += alpha x   (precision conversion allowed)
template <typename TX, typename TY>
__global__ void k_axpy(const TX *__restrict__ x, TY *__restrict__ y, double alpha, size_t n) {
  GRID_STRIDE(i, n) y[i] = TY(fma(alpha, double(x[i]), double(y[i])));
}

// partial ||x||^2
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_norm2(const T *__restrict__ x, size_t n,
                                                       double *__restrict__ partial) {
  __shared__ double sm[kRedThreads / 64 + 1];
  double acc = 0.0;
  GRID_STRIDE(i, n) {
    const double v = double(x[i]);
    acc = fma(v, v, acc);
  }
  const double a[1] = {acc};
  block_sum<1>(a, sm);
  if (threadIdx.x == 0) partial[blockIdx.x] = sm[kRedThreads / 64];
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
#define KR_BUCKETS(X) X(8) X(16) X(24) X(32) X(40) X(48) X(56) X(64)

template <typename T>
hipError_t kr_multidot(const T *V, size_t ld, int nv, const T *w, size_t n, double *partial, double *out,
                       hipStream_t s) {
  const dim3 g(kRedBlocks), b(kRedThreads);
  if (nv < 1 || nv > 64) return hipErrorInvalidValue;
#define KR_MD(B)                                                                                \
  else if (nv <= B) hipLaunchKernelGGL((k_multidot<T, B>), g, b, 0, s, V, ld, nv, w, n, partial);
  if (false) {
  }
  KR_BUCKETS(KR_MD)
#undef KR_MD
  hipLaunchKernelGGL(k_reduce, dim3(nv + 1), b, 0, s, partial, kRedBlocks, nv + 1, out);
  return hipGetLastError();
}

template <typename T, bool DOT, bool NORM>
hipError_t kr_orth(const T *V, size_t ld, int nv, const double *h, const T *w, T *wout, double scale,
                   size_t n, double *partial, double *out, hipStream_t s) {
  const dim3 g(kRedBlocks), b(kRedThreads);
  if (nv < 1 || nv > 64) return hipErrorInvalidValue;
#define KR_OR(B)      \
  else if (nv <= B) \
    hipLaunchKernelGGL((k_orth<T, B, DOT, NORM>), g, b, 0, s, V, ld, nv, h, w, wout, scale, n, partial);
  if (false) {
  }
  KR_BUCKETS(KR_OR)
#undef KR_OR
  const int nout = (DOT ? nv : 0) + (NORM ? 1 : 0);
  if (nout) hipLaunchKernelGGL(k_reduce, dim3(nout), b, 0, s, partial, kRedBlocks, nout, out);
  return hipGetLastError();
}

template <typename TI, typename TO>
hipError_t kr_scale(const TI *x, TO *y, double alpha, size_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_scale<TI, TO>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, x, y, alpha, n);
  return hipGetLastError();
}

template <typename TZ, typename TO>
hipError_t kr_lincomb(TO *out, const TZ *Z, size_t ld, int nz, const double *c, double scale,
                      bool acc, size_t n, hipStream_t s) {
  if (acc)
    hipLaunchKernelGGL((k_lincomb<TZ, TO, true>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, out, Z,
                       ld, nz, c, scale, n);
  else
    hipLaunchKernelGGL((k_lincomb<TZ, TO, false>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, out,
                       Z, ld, nz, c, scale, n);
  return hipGetLastError();
}

template <typename TX, typename TY>
hipError_t kr_axpy(const TX *x, TY *y, double alpha, size_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_axpy<TX, TY>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, x, y, alpha, n);
  return hipGetLastError();
}

template <typename T>
hipError_t kr_residual(const T *b, T *r, size_t n, double *partial, double *out, hipStream_t s) {
  hipLaunchKernelGGL((k_residual<T>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, b, r, n, partial);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, s, partial, kRedBlocks, 1, out);
  return hipGetLastError();
}

template <typename T>
hipError_t kr_norm2(const T *x, size_t n, double *partial, double *out, hipStream_t s) {
  hipLaunchKernelGGL((k_norm2<T>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, x, n, partial);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, s, partial, kRedBlocks, 1, out);
  return hipGetLastError();
}

// explicit instantiations
template hipError_t kr_multidot<double>(const double *, size_t, int, const double *, size_t, double *, double *, hipStream_t);
template hipError_t kr_multidot<float>(const float *, size_t, int, const float *, size_t, double *, double *, hipStream_t);
template hipError_t kr_orth<double, true, true>(const double *, size_t, int, const double *, const double *, double *, double, size_t, double *, double *, hipStream_t);
template hipError_t kr_orth<double, false, false>(const double *, size_t, int, const double *, const double *, double *, double, size_t, double *, double *, hipStream_t);
template hipError_t kr_orth<float, true, true>(const float *, size_t, int, const double *, const float *, float *, double, size_t, double *, double *, hipStream_t);
template hipError_t kr_orth<float, false, false>(const float *, size_t, int, const double *, const float *, float *, double, size_t, double *, double *, hipStream_t);
template hipError_t kr_scale<double, double>(const double *, double *, double, size_t, hipStream_t);
template hipError_t kr_scale<float, float>(const float *, float *, double, size_t, hipStream_t);
template hipError_t kr_scale<double, float>(const double *, float *, double, size_t, hipStream_t);
template hipError_t kr_scale<float, double>(const float *, double *, double, size_t, hipStream_t);
template hipError_t kr_lincomb<double, double>(double *, const double *, size_t, int, const double *, double, bool, size_t, hipStream_t);
template hipError_t kr_lincomb<float, float>(float *, const float *, size_t, int, const double *, double, bool, size_t, hipStream_t);
template hipError_t kr_lincomb<float, double>(double *, const float *, size_t, int, const double *, double, bool, size_t, hipStream_t);
template hipError_t kr_axpy<double, double>(const double *, double *, double, size_t, hipStream_t);
template hipError_t kr_axpy<float, float>(const float *, float *, double, size_t, hipStream_t);
template hipError_t kr_axpy<float, double>(const float *, double *, double, size_t, hipStream_t);
template hipError_t kr_residual<double>(const double *, double *, size_t, double *, double *, hipStream_t);
template hipError_t kr_residual<float>(const float *, float *, size_t, double *, double *, hipStream_t);
template hipError_t kr_norm2<double>(const double *, size_t, double *, double *, hipStream_t);
template hipError_t kr_norm2<float>(const float *, size_t, double *, double *, hipStream_t);

}  // namespace dgmf
