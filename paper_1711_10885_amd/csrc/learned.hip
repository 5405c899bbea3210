// Learned cell-patch preconditioner: BF16 MLP inference and training kernels
// (gfx950 MFMA), data generation from the solver's own iterates, and the
// additive preconditioner
//   M^{-1} r = q + s_T (MLP(p_T / s_T) - MLP(-p_T / s_T)) / 2  per cell T,
// where q = BJ r is the block-Jacobi-preconditioned residual (the odd part
// of the network keeps M^{-1}(-r) = -M^{-1} r, as for a linear map).
//
// The paper stops at the operator (Sec. 1 motivates it as the core of
// iterative solvers); this network is an extension on top of the solver:
//   p_T   patch of q = BJ r: its coefficients on T and its six face
//         neighbours (order: T, -x, +x, -y, +y, -z, +z; zero outside the
//         domain), 7 (k+1)^3 values, padded with zeros to a multiple of 64.
//         Block Jacobi divides out the local coefficient (A_TT scales with
//         kappa_T), so the map from the patch to the correction depends on
//         the coefficient field only through neighbour ratios;
//   s_T   ||p_T||_2 (the correction is homogeneous of degree one in r);
//   MLP   in -> 256 -> 256 -> out, ReLU, biases; BF16 weights and
//         activations, FP32 accumulation (MFMA), FP32 biases and output.
// With the last layer at zero the preconditioner is block Jacobi exactly.
//
// GEMM convention: C[M x N] = A[M x K] * B[N x K]^T with both operands
// row-major and K contiguous, so every MFMA operand fragment is one 16-byte
// load.  Weights are kept as W^T (out x in, the forward operand) and W
// (in x out, the operand of the input gradient), both BF16, refreshed from
// the FP32 master copy after each optimiser step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include <cstdio>
#include <cstring>

#include "dg_internal.h"
#include "krylov.h"

namespace dgmf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kT = 256;  // threads per block of the elementwise kernels

// float -> bf16 bits, round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return uint16_t((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

static int blocks_for(int64_t work) {
  const int64_t g = (work + kT - 1) / kT;
  return int(g < 1 ? 1 : (g > (1 << 20) ? (1 << 20) : g));
}

#define GSTRIDE(i, n) \
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < (n); i += int64_t(gridDim.x) * blockDim.x)

// ---------------------------------------------------------------------------
// GEMM (MFMA 16x16x32 bf16).  Block tile 64 x 64, four waves of 32 x 32 (2 x 2
// MFMA tiles).  Requires M % 64 == N % 64 == 0, K % 32 == 0, lda, ldb % 8 == 0.
// Operand fragments (lane l): A row l%16, k = 8 (l/16) .. +7; B column l%16,
// same k; result lane l holds rows 4 (l/16) .. +3 of column l%16.
// ---------------------------------------------------------------------------
enum { EPI_F32 = 0, EPI_BIAS_RELU_BF16 = 1, EPI_BIAS_F32 = 2, EPI_MASK_BF16 = 3 };

template <int EPI, bool NEGA = false>
__global__ __launch_bounds__(256) void k_gemm_nt(const uint16_t *__restrict__ A, int lda,
                                                 const uint16_t *__restrict__ B, int ldb, int K,
                                                 float *__restrict__ Cf, uint16_t *__restrict__ Cb, int ldc,
                                                 const float *__restrict__ bias, const uint16_t *__restrict__ mask,
                                                 int ldm, float alpha) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int col0 = blockIdx.x * 64 + (wave & 1) * 32;
  const int lr = lane & 15, lk = (lane >> 4) * 8;
  const uint16_t *a0 = A + size_t(row0 + lr) * lda + lk;
  const uint16_t *a1 = a0 + size_t(16) * lda;
  const uint16_t *b0 = B + size_t(col0 + lr) * ldb + lk;
  const uint16_t *b1 = b0 + size_t(16) * ldb;
  f32x4 c00 = {0, 0, 0, 0}, c01 = c00, c10 = c00, c11 = c00;
  for (int k = 0; k < K; k += 32) {
    bf16x8 fa0 = *reinterpret_cast<const bf16x8 *>(a0 + k);
    bf16x8 fa1 = *reinterpret_cast<const bf16x8 *>(a1 + k);
    if (NEGA) {
      fa0 = -fa0;
      fa1 = -fa1;
    }
    const bf16x8 fb0 = *reinterpret_cast<const bf16x8 *>(b0 + k);
    const bf16x8 fb1 = *reinterpret_cast<const bf16x8 *>(b1 + k);
    c00 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa0, fb0, c00, 0, 0, 0);
    c01 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa0, fb1, c01, 0, 0, 0);
    c10 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa1, fb0, c10, 0, 0, 0);
    c11 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa1, fb1, c11, 0, 0, 0);
  }
  const f32x4 acc[2][2] = {{c00, c01}, {c10, c11}};
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = row0 + 16 * i + (lane >> 4) * 4 + t;
        const int n = col0 + 16 * j + lr;
        float v = alpha * acc[i][j][t];
        const size_t o = size_t(m) * ldc + n;
        if (EPI == EPI_F32) {
          Cf[o] = v;
        } else if (EPI == EPI_BIAS_F32) {
          Cf[o] = v + bias[n];
        } else if (EPI == EPI_BIAS_RELU_BF16) {
          Cb[o] = f2bf(fmaxf(v + bias[n], 0.0f));
        } else {
          Cb[o] = f2bf(bf2f(mask[size_t(m) * ldm + n]) > 0.0f ? v : 0.0f);
        }
      }
}

// Large-tile variant: block tile 128 x 128, K staged through LDS in steps of
// 32 (rows padded to 40 entries to spread the fragment reads over the banks),
// four waves of 64 x 64 (4 x 4 MFMA tiles); the next K tile is fetched into
// registers while the current one is multiplied.  Requires M % 128 == N % 128
// == 0, K % 32 == 0, lda, ldb % 8 == 0.
constexpr int kGBM = 128, kGBN = 128, kGBK = 32, kGLd = 40;

template <int EPI, bool NEGA = false>
__global__ __launch_bounds__(256) void k_gemm_nt_big(const uint16_t *__restrict__ A, int lda,
                                                     const uint16_t *__restrict__ B, int ldb, int K,
                                                     float *__restrict__ Cf, uint16_t *__restrict__ Cb, int ldc,
                                                     const float *__restrict__ bias, const uint16_t *__restrict__ mask,
                                                     int ldm, float alpha) {
  __shared__ __attribute__((aligned(16))) uint16_t As[kGBM * kGLd];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[kGBN * kGLd];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int bm = blockIdx.y * kGBM, bn = blockIdx.x * kGBN;
  // global -> LDS: thread t moves rows t/4 and t/4 + 64, 8 entries at k = 8 (t % 4)
  const int lrow = t >> 2, lk = (t & 3) * 8;
  const uint16_t *ga0 = A + size_t(bm + lrow) * lda + lk, *ga1 = ga0 + size_t(64) * lda;
  const uint16_t *gb0 = B + size_t(bn + lrow) * ldb + lk, *gb1 = gb0 + size_t(64) * ldb;
  typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
  // NEGA: the A operand enters with flipped signs (bf16 sign bit, exact)
  const u16x8 sgn = NEGA ? u16x8(uint16_t(0x8000)) : u16x8(uint16_t(0));
  u16x8 ra0 = *reinterpret_cast<const u16x8 *>(ga0) ^ sgn, ra1 = *reinterpret_cast<const u16x8 *>(ga1) ^ sgn;
  u16x8 rb0 = *reinterpret_cast<const u16x8 *>(gb0), rb1 = *reinterpret_cast<const u16x8 *>(gb1);
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
  for (int k0 = 0; k0 < K; k0 += kGBK) {
    *reinterpret_cast<u16x8 *>(As + lrow * kGLd + lk) = ra0;
    *reinterpret_cast<u16x8 *>(As + (lrow + 64) * kGLd + lk) = ra1;
    *reinterpret_cast<u16x8 *>(Bs + lrow * kGLd + lk) = rb0;
    *reinterpret_cast<u16x8 *>(Bs + (lrow + 64) * kGLd + lk) = rb1;
    __syncthreads();
    if (k0 + kGBK < K) {  // prefetch the next K tile while this one is multiplied
      ra0 = *reinterpret_cast<const u16x8 *>(ga0 + k0 + kGBK) ^ sgn;
      ra1 = *reinterpret_cast<const u16x8 *>(ga1 + k0 + kGBK) ^ sgn;
      rb0 = *reinterpret_cast<const u16x8 *>(gb0 + k0 + kGBK);
      rb1 = *reinterpret_cast<const u16x8 *>(gb1 + k0 + kGBK);
    }
    bf16x8 fa[4], fb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      fa[i] = *reinterpret_cast<const bf16x8 *>(As + (wm + 16 * i + fr) * kGLd + fk);
      fb[i] = *reinterpret_cast<const bf16x8 *>(Bs + (wn + 16 * i + fr) * kGLd + fk);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = bm + wm + 16 * i + (lane >> 4) * 4 + q;
        const int n = bn + wn + 16 * j + fr;
        const float v = alpha * acc[i][j][q];
        const size_t o = size_t(m) * ldc + n;
        if (EPI == EPI_F32) {
          Cf[o] = v;
        } else if (EPI == EPI_BIAS_F32) {
          Cf[o] = v + bias[n];
        } else if (EPI == EPI_BIAS_RELU_BF16) {
          Cb[o] = f2bf(fmaxf(v + bias[n], 0.0f));
        } else {
          Cb[o] = f2bf(bf2f(mask[size_t(m) * ldm + n]) > 0.0f ? v : 0.0f);
        }
      }
}

template <int EPI, bool NEGA = false>
static hipError_t gemm(const uint16_t *A, int lda, const uint16_t *B, int ldb, int M, int N, int K, float *Cf,
                       uint16_t *Cb, int ldc, const float *bias, const uint16_t *mask, int ldm, float alpha,
                       hipStream_t s) {
  if (M % 64 || N % 64 || K % 32 || lda % 8 || ldb % 8) return hipErrorInvalidValue;
  if (M % kGBM == 0 && N % kGBN == 0)
    hipLaunchKernelGGL((k_gemm_nt_big<EPI, NEGA>), dim3(N / kGBN, M / kGBM), dim3(256), 0, s, A, lda, B, ldb, K, Cf,
                       Cb, ldc, bias, mask, ldm, alpha);
  else
    hipLaunchKernelGGL((k_gemm_nt<EPI, NEGA>), dim3(N / 64, M / 64), dim3(256), 0, s, A, lda, B, ldb, K, Cf, Cb,
                       ldc, bias, mask, ldm, alpha);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Patches
// ---------------------------------------------------------------------------
// Row i of X (bf16, ld inp) = p_T / s_T for cell T = cells[i] (or first + i),
// s[i] = ||p_T||_2.  One wave per row; rows beyond nrows are zero.
template <typename TR>
__global__ __launch_bounds__(256) void k_gather(const TR *__restrict__ r, int n1, int n2, int n3, int nb, int inp,
                                                const int64_t *__restrict__ cells, int64_t first, int64_t nrows,
                                                int64_t rows_pad, uint16_t *__restrict__ X, float *__restrict__ s) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (blockIdx.x * int64_t(blockDim.x) + threadIdx.x) >> 6;
  if (row >= rows_pad) return;
  uint16_t *xr = X + row * inp;
  if (row >= nrows) {
    for (int t = lane; t < inp; t += 64) xr[t] = 0;
    if (lane == 0) s[row] = 0.0f;
    return;
  }
  const int64_t c = cells ? cells[row] : first + row;
  const int i1 = int(c % n1), i2 = int((c / n1) % n2), i3 = int(c / (int64_t(n1) * n2));
  auto nbr = [&](int q) -> int64_t {  // q = 0: T, 1..6: -x, +x, -y, +y, -z, +z
    if (q == 0) return c;
    const int a = (q - 1) >> 1, e = (q - 1) & 1;
    const int ia = a == 0 ? i1 : (a == 1 ? i2 : i3), na = a == 0 ? n1 : (a == 1 ? n2 : n3);
    const int64_t st = a == 0 ? 1 : (a == 1 ? n1 : int64_t(n1) * n2);
    if (e ? ia + 1 >= na : ia == 0) return -1;
    return e ? c + st : c - st;
  };
  if (nb <= 64) {
    // lane j owns coefficient j of each of the 7 patch cells (coalesced rows)
    double v[7];
    double ss = 0.0;
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      const int64_t cn = nbr(q);
      v[q] = (lane < nb && cn >= 0) ? double(r[cn * nb + lane]) : 0.0;
      ss = fma(v[q], v[q], ss);
    }
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
    const double sn = std::sqrt(ss);
    const double inv = sn > 0.0 ? 1.0 / sn : 0.0;
    if (lane < nb) {
#pragma unroll
      for (int q = 0; q < 7; ++q) xr[q * nb + lane] = f2bf(float(v[q] * inv));
    }
    for (int t = 7 * nb + lane; t < inp; t += 64) xr[t] = 0;
    if (lane == 0) s[row] = float(sn);
    return;
  }
  double ss = 0.0;
  for (int q = 0; q < 7; ++q) {
    const int64_t cn = nbr(q);
    if (cn < 0) continue;
    for (int j = lane; j < nb; j += 64) {
      const double v = double(r[cn * nb + j]);
      ss = fma(v, v, ss);
    }
  }
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
  const double sn = std::sqrt(ss);
  const double inv = sn > 0.0 ? 1.0 / sn : 0.0;
  for (int q = 0; q < 7; ++q) {
    const int64_t cn = nbr(q);
    for (int j = lane; j < nb; j += 64) xr[q * nb + j] = f2bf(cn >= 0 ? float(double(r[cn * nb + j]) * inv) : 0.0f);
  }
  for (int t = 7 * nb + lane; t < inp; t += 64) xr[t] = 0;
  if (lane == 0) s[row] = float(sn);
}

// training targets: T[i][j] = (e - z)_{T,j} / s[i] (zero where s = 0 and in the padding)
__global__ void k_targets(const double *__restrict__ e, const double *__restrict__ z, const int64_t *__restrict__ cells,
                          const float *__restrict__ s, int64_t nrows, int nb, int outp, float *__restrict__ T) {
  GSTRIDE(g, nrows * outp) {
    const int64_t i = g / outp;
    const int j = int(g - i * outp);
    float v = 0.0f;
    if (j < nb && s[i] > 0.0f) {
      const int64_t o = cells[i] * nb + j;
      v = float((e[o] - z[o]) / double(s[i]));
    }
    T[g] = v;
  }
}

// z_T += fac s_T Y_T  (the learned correction added to the block-Jacobi part)
template <typename TZ>
__global__ void k_scatter(const float *__restrict__ Y, const float *__restrict__ s, int64_t first, int64_t nrows,
                          int nb, int outp, double fac, TZ *__restrict__ z) {
  GSTRIDE(g, nrows * nb) {
    const int64_t i = g / nb;
    const int j = int(g - i * nb);
    const int64_t o = (first + i) * nb + j;
    z[o] = TZ(double(z[o]) + fac * double(s[i]) * double(Y[i * outp + j]));
  }
}


// ---------------------------------------------------------------------------
// Training kernels
// ---------------------------------------------------------------------------
// dY = 2 (Y - T) / (B out) on the first `out` columns (bf16, normal and
// transposed), per-block partial sums of (Y - T)^2
__global__ __launch_bounds__(kT) void k_loss(const float *__restrict__ Y, const float *__restrict__ T, int B, int out,
                                             int outp, float scale, uint16_t *__restrict__ dY,
                                             uint16_t *__restrict__ dYT, double *__restrict__ partial) {
  __shared__ double sm[kT / 64];
  double acc = 0.0;
  GSTRIDE(g, int64_t(B) * outp) {
    const int b = int(g / outp), j = int(g % outp);
    float d = 0.0f;
    if (j < out) {
      const float diff = Y[g] - T[g];
      acc = fma(double(diff), double(diff), acc);
      d = scale * diff;
    }
    const uint16_t h = f2bf(d);
    dY[g] = h;
    dYT[size_t(j) * B + b] = h;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kT / 64; ++w) t += sm[w];
    partial[blockIdx.x] = t;
  }
}

// sum of partials (one block, fixed order) -> out[0] * scale
__global__ __launch_bounds__(kT) void k_sum(const double *__restrict__ partial, int n, double scale,
                                            double *__restrict__ out) {
  __shared__ double sm[kT / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kT) acc += partial[i];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kT / 64; ++w) t += sm[w];
    out[0] = t * scale;
  }
}

// db[n] = sum_b G^T[n][b] (bf16 rows of length B), one wave per n
__global__ __launch_bounds__(kT) void k_bias_grad(const uint16_t *__restrict__ GT, int B, int N, float *__restrict__ db) {
  const int lane = threadIdx.x & 63;
  const int n = (blockIdx.x * kT + threadIdx.x) >> 6;
  if (n >= N) return;
  float acc = 0.0f;
  for (int b = lane; b < B; b += 64) acc += bf2f(GT[size_t(n) * B + b]);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) db[n] = acc;
}

// bf16 transpose, 64 x 64 tiles through LDS: out[c][r] = in[r][c]
__global__ __launch_bounds__(256) void k_transpose(const uint16_t *__restrict__ in, int R, int Cc,
                                                   uint16_t *__restrict__ out) {
  __shared__ uint16_t t[64][65];
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int i = e / 64, j = e % 64;
    t[i][j] = in[size_t(r0 + i) * Cc + c0 + j];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int i = e / 64, j = e % 64;
    out[size_t(c0 + i) * R + r0 + j] = t[j][i];
  }
}

// Adam (Kingma & Ba): m, v moments, bias-corrected step on the FP32 master copy
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  GSTRIDE(i, n) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// bf16 copies of one weight matrix Wt (O x I, FP32 master): wt = Wt, w = Wt^T
__global__ void k_refresh(const float *__restrict__ Wt, int O, int I, uint16_t *__restrict__ wt,
                          uint16_t *__restrict__ w) {
  GSTRIDE(g, int64_t(O) * I) {
    const int o = int(g / I), i = int(g % I);
    const uint16_t b = f2bf(Wt[g]);
    wt[g] = b;
    w[size_t(i) * O + o] = b;
  }
}

// rows of the data set into the batch buffers
__global__ void k_rows(const uint16_t *__restrict__ Xall, const float *__restrict__ Tall, const int32_t *__restrict__ idx,
                       int B, int inp, int outp, uint16_t *__restrict__ X, float *__restrict__ T) {
  GSTRIDE(g, int64_t(B) * (inp + outp)) {
    const int b = int(g / (inp + outp)), j = int(g % (inp + outp));
    const int64_t src = idx[b];
    if (j < inp)
      X[size_t(b) * inp + j] = Xall[src * inp + j];
    else
      T[size_t(b) * outp + (j - inp)] = Tall[src * outp + (j - inp)];
  }
}

// float rows (caller layout, width w) -> bf16 rows of width inp (zero padded)
__global__ void k_to_bf16_rows(const float *__restrict__ x, int rows, int w, int inp, uint16_t *__restrict__ X) {
  GSTRIDE(g, int64_t(rows) * inp) {
    const int i = int(g / inp), j = int(g % inp);
    X[g] = j < w ? f2bf(x[size_t(i) * w + j]) : uint16_t(0);
  }
}
__global__ void k_rows_f32(const float *__restrict__ x, int rows, int w, int wp, float *__restrict__ X) {
  GSTRIDE(g, int64_t(rows) * wp) {
    const int i = int(g / wp), j = int(g % wp);
    X[g] = j < w ? x[size_t(i) * w + j] : 0.0f;
  }
}
__global__ void k_rows_unpad(const float *__restrict__ X, int rows, int wp, int w, float *__restrict__ x) {
  GSTRIDE(g, int64_t(rows) * w) {
    const int i = int(g / w), j = int(g % w);
    x[g] = X[size_t(i) * wp + j];
  }
}

// SplitMix64 (Steele, Lea & Flood, 2014) as a counter-based generator:
// value i of stream `seed` is mix(seed * golden + (i + 1) * golden).
__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
__host__ __device__ __forceinline__ double u01(uint64_t seed, uint64_t i) {
  return (double(splitmix64(seed * 0x9e3779b97f4a7c15ull + i) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

// random exact solution: coefficient j of cell c is a centred uniform value
// damped by 1 / (1 + j1 + j2 + j3) (smoother than white noise)
__global__ void k_random_field(double *__restrict__ u, int64_t n, int nb, int np1, uint64_t seed, double sign) {
  GSTRIDE(g, n) {
    const int j = int(g % nb);
    const int j1 = j % np1, j2 = (j / np1) % np1, j3 = j / (np1 * np1);
    u[g] = sign * (2.0 * u01(seed, uint64_t(g)) - 1.0) / double(1 + j1 + j2 + j3);
  }
}

__global__ void k_sub(const double *__restrict__ a, const double *__restrict__ b, double *__restrict__ c, int64_t n) {
  GSTRIDE(i, n) c[i] = a[i] - b[i];
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct MlpDims {
  int nb, in, inp, out, outp, hid;
  int64_t oW1, ob1, oW2, ob2, oW3, ob3, np;  // padded master layout
  int64_t oc_W1, oc_W2, oc_W3;               // offsets into the bf16 copies
};

static MlpDims dims_for(int k) {
  MlpDims d;
  const int n = k + 1;
  d.nb = n * n * n;
  d.in = 7 * d.nb;
  d.inp = (d.in + 63) / 64 * 64;
  d.out = d.nb;
  d.outp = (d.out + 63) / 64 * 64;
  d.hid = kMlpHidden;
  d.oW1 = 0;
  d.ob1 = d.oW1 + int64_t(d.hid) * d.inp;
  d.oW2 = d.ob1 + d.hid;
  d.ob2 = d.oW2 + int64_t(d.hid) * d.hid;
  d.oW3 = d.ob2 + d.hid;
  d.ob3 = d.oW3 + int64_t(d.outp) * d.hid;
  d.np = d.ob3 + d.outp;
  d.oc_W1 = 0;
  d.oc_W2 = int64_t(d.hid) * d.inp;
  d.oc_W3 = d.oc_W2 + int64_t(d.hid) * d.hid;
  return d;
}

static int64_t public_nparams(const MlpDims &d) {
  return int64_t(d.hid) * d.in + d.hid + int64_t(d.hid) * d.hid + d.hid + int64_t(d.out) * d.hid + d.out;
}

struct Mlp {
  MlpDims d;
  double *q = nullptr;  // ndof: block-Jacobi output during an application
  float *master = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  uint16_t *wt = nullptr, *w = nullptr;  // bf16 copies (W^T and W)
  int64_t step = 0;
  bool trained = false;
  // work buffers (grown on demand): activations for `rows` rows
  void *buf = nullptr;
  size_t buf_bytes = 0;
};

void release_learned(dg_handle *h) {
  if (!h->mlp) return;
  Mlp *M = h->mlp;
  for (void *p : {(void *)M->master, (void *)M->grad, (void *)M->m, (void *)M->v, (void *)M->wt, (void *)M->w, M->buf,
                  (void *)M->q})
    if (p) (void)hipFree(p);
  delete M;
  h->mlp = nullptr;
}

static hipError_t refresh(Mlp *M, hipStream_t s) {
  const MlpDims &d = M->d;
  const int64_t ow[3] = {d.oW1, d.oW2, d.oW3}, oc[3] = {d.oc_W1, d.oc_W2, d.oc_W3};
  const int O[3] = {d.hid, d.hid, d.outp}, I[3] = {d.inp, d.hid, d.hid};
  for (int l = 0; l < 3; ++l)
    hipLaunchKernelGGL(k_refresh, dim3(blocks_for(int64_t(O[l]) * I[l])), dim3(kT), 0, s, M->master + ow[l], O[l],
                       I[l], M->wt + oc[l], M->w + oc[l]);
  return hipGetLastError();
}

static dg_status ensure_mlp(dg_handle *h) {
  if (h->mlp) return DG_OK;
  if (h->k + 1 > 8) return set_error(DG_EINVAL, "learned preconditioner: k <= 7");
  Mlp *M = new Mlp();
  M->d = dims_for(h->k);
  const int64_t np = M->d.np, nw = M->d.oc_W3 + int64_t(M->d.outp) * M->d.hid;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMalloc(&M->master, np * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&M->grad, np * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&M->m, np * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&M->v, np * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&M->wt, nw * sizeof(uint16_t));
  if (e == hipSuccess) e = hipMalloc(&M->w, nw * sizeof(uint16_t));
  if (e == hipSuccess) e = hipMemset(M->master, 0, np * sizeof(float));
  if (e == hipSuccess) e = hipMemset(M->grad, 0, np * sizeof(float));
  if (e == hipSuccess) e = hipMemset(M->m, 0, np * sizeof(float));
  if (e == hipSuccess) e = hipMemset(M->v, 0, np * sizeof(float));
  h->mlp = M;
  if (e == hipSuccess) e = refresh(M, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    release_learned(h);
    return hip_error(e, "learned preconditioner: allocation");
  }
  return DG_OK;
}

// activation buffers for `rows` rows (multiple of 64):
//   X bf16 rows x inp | H1, H2 bf16 rows x hid | Y f32 rows x outp | s f32 rows
//   training extras: XT bf16 inp x rows | H1T, H2T bf16 | T f32 rows x outp |
//   dY bf16 rows x outp | dYT bf16 outp x rows | dH bf16 rows x hid | dHT bf16
struct Acts {
  uint16_t *X, *H1, *H2, *XT, *H1T, *H2T, *dY, *dYT, *dH, *dH1, *dHT;
  float *Y, *s, *T;
  double *partial, *loss;
};

static size_t al(size_t b) { return (b + 255) & ~size_t(255); }

static dg_status acts_for(dg_handle *h, int64_t rows, bool train, Acts &A) {
  Mlp *M = h->mlp;
  const MlpDims &d = M->d;
  const size_t r = size_t(rows);
  size_t sz[15] = {al(r * d.inp * 2), al(r * d.hid * 2), al(r * d.hid * 2), al(r * d.outp * 4), al(r * 4),
                   al(1024 * 8 + 64)};
  size_t need = 0;
  for (int i = 0; i < 6; ++i) need += sz[i];
  if (train) {
    const size_t ex[9] = {al(r * d.inp * 2),  al(r * d.hid * 2),  al(r * d.hid * 2),
                          al(r * d.outp * 4), al(r * d.outp * 2), al(r * d.outp * 2),
                          al(r * d.hid * 2),  al(r * d.hid * 2),  al(r * d.hid * 2)};
    for (int i = 0; i < 9; ++i) need += ex[i];
  }
  if (need > M->buf_bytes) {
    if (M->buf) (void)hipFree(M->buf);
    M->buf = nullptr;
    M->buf_bytes = 0;
    hipError_t e = hipMalloc(&M->buf, need);
    if (e != hipSuccess) {
      M->buf = nullptr;
      return hip_error(e, "learned preconditioner: activation buffers");
    }
    M->buf_bytes = need;
  }
  char *p = static_cast<char *>(M->buf);
  auto take = [&](size_t b) {
    char *q = p;
    p += b;
    return q;
  };
  A.X = (uint16_t *)take(sz[0]);
  A.H1 = (uint16_t *)take(sz[1]);
  A.H2 = (uint16_t *)take(sz[2]);
  A.Y = (float *)take(sz[3]);
  A.s = (float *)take(sz[4]);
  A.partial = (double *)take(sz[5]);
  A.loss = A.partial + 1024;
  if (train) {
    A.XT = (uint16_t *)take(al(r * d.inp * 2));
    A.H1T = (uint16_t *)take(al(r * d.hid * 2));
    A.H2T = (uint16_t *)take(al(r * d.hid * 2));
    A.T = (float *)take(al(r * d.outp * 4));
    A.dY = (uint16_t *)take(al(r * d.outp * 2));
    A.dYT = (uint16_t *)take(al(r * d.outp * 2));
    A.dH = (uint16_t *)take(al(r * d.hid * 2));
    A.dH1 = (uint16_t *)take(al(r * d.hid * 2));
    A.dHT = (uint16_t *)take(al(r * d.hid * 2));
  } else {
    A.XT = A.H1T = A.H2T = A.dY = A.dYT = A.dH = A.dH1 = A.dHT = nullptr;
    A.T = nullptr;
  }
  return DG_OK;
}

// forward for rows (multiple of 64) of A.X (or -A.X) -> A.H1, A.H2, A.Y
static hipError_t forward(Mlp *M, const Acts &A, int rows, hipStream_t s, bool neg_x = false) {
  const MlpDims &d = M->d;
  hipError_t e;
  e = neg_x ? gemm<EPI_BIAS_RELU_BF16, true>(A.X, d.inp, M->wt + d.oc_W1, d.inp, rows, d.hid, d.inp, nullptr, A.H1,
                                             d.hid, M->master + d.ob1, nullptr, 0, 1.0f, s)
            : gemm<EPI_BIAS_RELU_BF16>(A.X, d.inp, M->wt + d.oc_W1, d.inp, rows, d.hid, d.inp, nullptr, A.H1, d.hid,
                                       M->master + d.ob1, nullptr, 0, 1.0f, s);
  if (e != hipSuccess) return e;
  if ((e = gemm<EPI_BIAS_RELU_BF16>(A.H1, d.hid, M->wt + d.oc_W2, d.hid, rows, d.hid, d.hid, nullptr, A.H2, d.hid,
                                    M->master + d.ob2, nullptr, 0, 1.0f, s)) != hipSuccess)
    return e;
  return gemm<EPI_BIAS_F32>(A.H2, d.hid, M->wt + d.oc_W3, d.hid, rows, d.outp, d.hid, A.Y, nullptr, d.outp,
                            M->master + d.ob3, nullptr, 0, 1.0f, s);
}

// forward + backward for B rows of A.X / A.T: gradients into M->grad, loss
// (mean over B * out squared errors) into A.loss[0]
static hipError_t backward(Mlp *M, const Acts &A, int B, hipStream_t s) {
  const MlpDims &d = M->d;
  hipError_t e;
  if ((e = forward(M, A, B, s)) != hipSuccess) return e;
  const float scale = 2.0f / (float(B) * float(d.out));
  const int nblk = 256;
  hipLaunchKernelGGL(k_loss, dim3(nblk), dim3(kT), 0, s, A.Y, A.T, B, d.out, d.outp, scale, A.dY, A.dYT, A.partial);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kT), 0, s, A.partial, nblk, 1.0 / (double(B) * d.out), A.loss);
  // transposed activations for the weight gradients
  hipLaunchKernelGGL(k_transpose, dim3(d.inp / 64, B / 64), dim3(256), 0, s, A.X, B, d.inp, A.XT);
  hipLaunchKernelGGL(k_transpose, dim3(d.hid / 64, B / 64), dim3(256), 0, s, A.H1, B, d.hid, A.H1T);
  hipLaunchKernelGGL(k_transpose, dim3(d.hid / 64, B / 64), dim3(256), 0, s, A.H2, B, d.hid, A.H2T);
  // layer 3: dW3^T = dY^T H2, db3 = sum dY, dH2 = (dY W3^T... ) masked by H2 > 0
  if ((e = gemm<EPI_F32>(A.dYT, B, A.H2T, B, d.outp, d.hid, B, M->grad + d.oW3, nullptr, d.hid, nullptr, nullptr, 0,
                         1.0f, s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_bias_grad, dim3((d.outp * 64 + kT - 1) / kT), dim3(kT), 0, s, A.dYT, B, d.outp,
                     M->grad + d.ob3);
  if ((e = gemm<EPI_MASK_BF16>(A.dY, d.outp, M->w + d.oc_W3, d.outp, B, d.hid, d.outp, nullptr, A.dH, d.hid, nullptr,
                               A.H2, d.hid, 1.0f, s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_transpose, dim3(d.hid / 64, B / 64), dim3(256), 0, s, A.dH, B, d.hid, A.dHT);
  // layer 2
  if ((e = gemm<EPI_F32>(A.dHT, B, A.H1T, B, d.hid, d.hid, B, M->grad + d.oW2, nullptr, d.hid, nullptr, nullptr, 0,
                         1.0f, s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_bias_grad, dim3((d.hid * 64 + kT - 1) / kT), dim3(kT), 0, s, A.dHT, B, d.hid, M->grad + d.ob2);
  if ((e = gemm<EPI_MASK_BF16>(A.dH, d.hid, M->w + d.oc_W2, d.hid, B, d.hid, d.hid, nullptr, A.dH1, d.hid, nullptr,
                               A.H1, d.hid, 1.0f, s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_transpose, dim3(d.hid / 64, B / 64), dim3(256), 0, s, A.dH1, B, d.hid, A.dHT);
  // layer 1
  if ((e = gemm<EPI_F32>(A.dHT, B, A.XT, B, d.hid, d.inp, B, M->grad + d.oW1, nullptr, d.inp, nullptr, nullptr, 0,
                         1.0f, s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_bias_grad, dim3((d.hid * 64 + kT - 1) / kT), dim3(kT), 0, s, A.dHT, B, d.hid, M->grad + d.ob1);
  return hipGetLastError();
}

static hipError_t adam_step(Mlp *M, float lr, hipStream_t s) {
  ++M->step;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = float(1.0 - std::pow(double(b1), double(M->step)));
  const float c2 = float(1.0 - std::pow(double(b2), double(M->step)));
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(M->d.np)), dim3(kT), 0, s, M->master, M->grad, M->m, M->v, M->d.np, lr,
                     b1, b2, eps, c1, c2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return refresh(M, s);
}

// z = q + learned correction (q = BJ r, the patches are read from q), in
// chunks of cells
template <typename TR>
hipError_t learned_apply(dg_handle *h, const TR *r, TR *z, hipStream_t s) {
  Mlp *M = h->mlp;
  const MlpDims &d = M->d;
  hipError_t e;
  if (!M->q && (e = hipMalloc(&M->q, size_t(h->ndof) * sizeof(double))) != hipSuccess) {
    M->q = nullptr;
    return e;
  }
  double *q = M->q;
  if ((e = bj_apply<TR, double>(h, r, q, s)) != hipSuccess) return e;
  if ((e = kr_scale<double, TR>(q, z, 1.0, size_t(h->ndof), s)) != hipSuccess) return e;
  const int64_t chunk = std::min<int64_t>((h->ncells + 63) / 64 * 64, kMlpChunk);
  Acts A;
  if (acts_for(h, chunk, false, A) != DG_OK) return hipErrorOutOfMemory;
  const int n1 = h->mesh.ncell[0], n2 = h->mesh.ncell[1], n3 = h->mesh.ncell[2];
  for (int64_t c0 = 0; c0 < h->ncells; c0 += chunk) {
    const int64_t rows = std::min<int64_t>(chunk, h->ncells - c0);
    const int64_t rp = (rows + 63) / 64 * 64;
    hipLaunchKernelGGL(k_gather<double>, dim3(unsigned((rp * 64 + 255) / 256)), dim3(256), 0, s, q, n1, n2, n3,
                       d.nb, d.inp, nullptr, c0, rows, rp, A.X, A.s);
    // odd part of the network: (N(x) - N(-x)) / 2, so the correction is
    // homogeneous of degree one in r (z(-r) = -z(r)) like a linear map
    if ((e = forward(M, A, int(rp), s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_scatter<TR>, dim3(blocks_for(rows * d.nb)), dim3(kT), 0, s, A.Y, A.s, c0, rows, d.nb, d.outp,
                       0.5, z);
    if ((e = forward(M, A, int(rp), s, true)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_scatter<TR>, dim3(blocks_for(rows * d.nb)), dim3(kT), 0, s, A.Y, A.s, c0, rows, d.nb, d.outp,
                       -0.5, z);
  }
  return hipGetLastError();
}
template hipError_t learned_apply<double>(dg_handle *, const double *, double *, hipStream_t);

bool learned_ready(const dg_handle *h) { return h->mlp != nullptr && h->mlp->trained && h->bj != nullptr; }

// ---------------------------------------------------------------------------
// Training data from the solver: for random exact solutions u*, f = A u*;
// block-Jacobi GMRES from u = 0 stopped after j steps gives u_j, and the
// pair (r_j = f - A u_j, e_j = u* - u_j) is exact.  Cells are sampled
// uniformly; inputs are the patches of q_j = BJ r_j, targets
// (e_j - q_j)_T / s_T.
// ---------------------------------------------------------------------------
static dg_status make_data(dg_handle *h, const dg_learn_opts &o, uint16_t *Xall, float *Tall, int64_t npairs,
                           hipStream_t s) {
  Mlp *M = h->mlp;
  const MlpDims &d = M->d;
  const size_t n = size_t(h->ndof);
  double *u_star = nullptr, *f = nullptr, *u = nullptr, *r = nullptr, *e = nullptr, *z = nullptr;
  int64_t *cells = nullptr;
  float *sv = nullptr;
  hipError_t err = hipSuccess;
  auto cleanup = [&]() {
    for (void *p : {(void *)u_star, (void *)f, (void *)u, (void *)r, (void *)e, (void *)z, (void *)cells, (void *)sv})
      if (p) (void)hipFree(p);
  };
  // GMRES step counts j = 0, 1, 2, 4, ..., max_steps (j = 0: e = u*, r = f)
  std::vector<int> js{0};
  for (int j = 1; j <= o.max_steps; j *= 2) js.push_back(j);
  const int nj = int(js.size());
  const int nsets = o.nrhs * nj;
  const int64_t per = (npairs + nsets - 1) / nsets;
  for (double **p : {&u_star, &f, &u, &r, &e, &z})
    if (err == hipSuccess) err = hipMalloc(p, n * sizeof(double));
  if (err == hipSuccess) err = hipMalloc(&cells, per * sizeof(int64_t));
  if (err == hipSuccess) err = hipMalloc(&sv, ((per + 63) / 64 * 64) * sizeof(float));
  if (err != hipSuccess) {
    cleanup();
    return hip_error(err, "dg_learned_train: data buffers");
  }
  std::vector<int64_t> hc(per);
  int64_t row = 0;
  dg_solve_opts so{DG_GMRES64, DG_PREC_BLOCK_JACOBI, 30, 1, DG_ORTH_CGS1, 1e-4};
  for (int q = 0; q < o.nrhs && row < npairs; ++q) {
    // fields come in sign pairs (u*, -u*): the pairs of -u* are exact too and
    // teach the network the odd symmetry the preconditioner imposes
    hipLaunchKernelGGL(k_random_field, dim3(blocks_for(int64_t(n))), dim3(kT), 0, s, u_star, int64_t(n), d.nb,
                       h->k + 1, o.seed * 1000003ull + uint64_t(q / 2), (q & 1) ? -1.0 : 1.0);
    if ((err = apply_f64(h, u_star, f, s)) != hipSuccess) break;
    for (int jj = 0; jj < nj && row < npairs; ++jj) {
      if ((err = hipMemsetAsync(u, 0, n * sizeof(double), s)) != hipSuccess) break;
      if (js[jj] > 0) {
        so.maxit = js[jj];
        dg_solve_stats st;
        const dg_status ds = dg_solve(h, f, u, 1e-300, &so, &st, s);
        if (ds != DG_OK && ds != DG_ENOTCONV) {
          cleanup();
          return ds;
        }
      }
      if ((err = apply_f64(h, u, r, s)) != hipSuccess) break;
      hipLaunchKernelGGL(k_sub, dim3(blocks_for(int64_t(n))), dim3(kT), 0, s, f, r, r, int64_t(n));
      hipLaunchKernelGGL(k_sub, dim3(blocks_for(int64_t(n))), dim3(kT), 0, s, u_star, u, e, int64_t(n));
      if ((err = bj_apply<double, double>(h, r, z, s)) != hipSuccess) break;
      const int64_t cnt = std::min<int64_t>(per, npairs - row);
      const uint64_t sseed = o.seed * 0x51ed27ull + uint64_t(q * nj + jj) + 7;
      for (int64_t i = 0; i < cnt; ++i)
        hc[i] = int64_t(u01(sseed, uint64_t(i)) * double(h->ncells)) % h->ncells;
      if ((err = hipMemcpyAsync(cells, hc.data(), cnt * sizeof(int64_t), hipMemcpyHostToDevice, s)) != hipSuccess) break;
      const int64_t cp = (cnt + 63) / 64 * 64;
      (void)cp;
      hipLaunchKernelGGL(k_gather<double>, dim3(unsigned((cnt * 64 + 255) / 256)), dim3(256), 0, s, z,
                         h->mesh.ncell[0], h->mesh.ncell[1], h->mesh.ncell[2], d.nb, d.inp, cells, 0, cnt, cnt,
                         Xall + row * d.inp, sv);
      hipLaunchKernelGGL(k_targets, dim3(blocks_for(cnt * d.outp)), dim3(kT), 0, s, e, z, cells, sv, cnt, d.nb,
                         d.outp, Tall + row * d.outp);
      if ((err = hipStreamSynchronize(s)) != hipSuccess) break;  // hc is reused
      row += cnt;
    }
    if (err != hipSuccess) break;
  }
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  cleanup();
  if (err != hipSuccess) return hip_error(err, "dg_learned_train: data generation");
  return DG_OK;
}

}  // namespace dgmf

using namespace dgmf;

static dg_status learned_prologue(dg_handle *h, const char *who) {
  if (!h) return set_error(DG_EINVAL, std::string(who) + ": handle is NULL");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != h->device) {
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_error(e, who);
  }
  return ensure_mlp(h);
}

extern "C" int64_t dg_learned_nparams(const dg_handle *h) {
  if (!h || h->k + 1 > 8) return -1;
  return public_nparams(dims_for(h->k));
}

// public layout (host) -> padded master layout (host), zero padding
static std::vector<float> padded_from_public(const MlpDims &d, const float *params) {
  std::vector<float> pad(size_t(d.np), 0.0f);
  const float *q = params;
  for (int o = 0; o < d.hid; ++o)
    for (int i = 0; i < d.in; ++i) pad[d.oW1 + int64_t(o) * d.inp + i] = *q++;
  for (int o = 0; o < d.hid; ++o) pad[d.ob1 + o] = *q++;
  for (int o = 0; o < d.hid; ++o)
    for (int i = 0; i < d.hid; ++i) pad[d.oW2 + int64_t(o) * d.hid + i] = *q++;
  for (int o = 0; o < d.hid; ++o) pad[d.ob2 + o] = *q++;
  for (int o = 0; o < d.out; ++o)
    for (int i = 0; i < d.hid; ++i) pad[d.oW3 + int64_t(o) * d.hid + i] = *q++;
  for (int o = 0; o < d.out; ++o) pad[d.ob3 + o] = *q++;
  return pad;
}

extern "C" dg_status dg_learned_set_params(dg_handle *h, const float *params, int64_t n) {
  dg_status ds = learned_prologue(h, "dg_learned_set_params");
  if (ds != DG_OK) return ds;
  if (!params) return set_error(DG_EINVAL, "dg_learned_set_params: params is NULL");
  Mlp *M = h->mlp;
  const MlpDims &d = M->d;
  if (n != public_nparams(d)) return set_error(DG_EINVAL, "dg_learned_set_params: wrong parameter count");
  const std::vector<float> pad = padded_from_public(d, params);
  hipError_t e = hipMemcpy(M->master, pad.data(), pad.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(M->m, 0, d.np * sizeof(float));
  if (e == hipSuccess) e = hipMemset(M->v, 0, d.np * sizeof(float));
  if (e == hipSuccess) e = refresh(M, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_error(e, "dg_learned_set_params");
  M->step = 0;
  M->trained = true;
  return DG_OK;
}

// padded device array (gradients or master) -> public layout on the host
static dg_status export_params(dg_handle *h, const float *dev, float *out, int64_t n, const char *who) {
  Mlp *M = h->mlp;
  const MlpDims &d = M->d;
  if (!out) return set_error(DG_EINVAL, std::string(who) + ": output is NULL");
  if (n != public_nparams(d)) return set_error(DG_EINVAL, std::string(who) + ": wrong parameter count");
  std::vector<float> pad(size_t(d.np));
  hipError_t e = hipMemcpy(pad.data(), dev, pad.size() * sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_error(e, who);
  float *q = out;
  for (int o = 0; o < d.hid; ++o)
    for (int i = 0; i < d.in; ++i) *q++ = pad[d.oW1 + int64_t(o) * d.inp + i];
  for (int o = 0; o < d.hid; ++o) *q++ = pad[d.ob1 + o];
  for (int o = 0; o < d.hid; ++o)
    for (int i = 0; i < d.hid; ++i) *q++ = pad[d.oW2 + int64_t(o) * d.hid + i];
  for (int o = 0; o < d.hid; ++o) *q++ = pad[d.ob2 + o];
  for (int o = 0; o < d.out; ++o)
    for (int i = 0; i < d.hid; ++i) *q++ = pad[d.oW3 + int64_t(o) * d.hid + i];
  for (int o = 0; o < d.out; ++o) *q++ = pad[d.ob3 + o];
  return DG_OK;
}

extern "C" dg_status dg_learned_get_params(dg_handle *h, float *params, int64_t n) {
  dg_status ds = learned_prologue(h, "dg_learned_get_params");
  if (ds != DG_OK) return ds;
  return export_params(h, h->mlp->master, params, n, "dg_learned_get_params");
}

// ---- checkpoint: parameters, Adam moments and step count -------------------
// File: 64-byte header {char magic[8] = "DGMFNET1"; int32 version = 1, k,
// in, hidden, out, 0; int64 n, step; uint64 checksum; 8 zero bytes}, then
// the parameters, the first and the second Adam moments, n FP32 values each
// in the public layout; checksum = FNV-1a (64-bit) of those 12 n bytes.
// Native byte order.
struct CkptHeader {
  char magic[8];
  int32_t version, k, in, hid, out, zero;
  int64_t n, step;
  uint64_t checksum, pad;
};
static_assert(sizeof(CkptHeader) == 64, "checkpoint header is 64 bytes");

static uint64_t fnv1a(const void *data, size_t bytes, uint64_t hsh = 1469598103934665603ull) {
  const unsigned char *p = static_cast<const unsigned char *>(data);
  for (size_t i = 0; i < bytes; ++i) hsh = (hsh ^ p[i]) * 1099511628211ull;
  return hsh;
}

extern "C" dg_status dg_learned_save(dg_handle *h, const char *path) {
  if (!h) return set_error(DG_EINVAL, "dg_learned_save: handle is NULL");
  if (!path) return set_error(DG_EINVAL, "dg_learned_save: path is NULL");
  if (!h->mlp || !h->mlp->trained) return set_error(DG_EINVAL, "dg_learned_save: no trained or loaded network");
  dg_status ds = learned_prologue(h, "dg_learned_save");
  if (ds != DG_OK) return ds;
  Mlp *M = h->mlp;
  const MlpDims &d = M->d;
  const int64_t n = public_nparams(d);
  std::vector<float> body(size_t(3 * n));
  const float *src[3] = {M->master, M->m, M->v};
  for (int t = 0; t < 3; ++t)
    if ((ds = export_params(h, src[t], body.data() + t * n, n, "dg_learned_save")) != DG_OK) return ds;
  CkptHeader hd;
  std::memset(&hd, 0, sizeof(hd));
  std::memcpy(hd.magic, "DGMFNET1", 8);
  hd.version = 1;
  hd.k = h->k;
  hd.in = d.in;
  hd.hid = d.hid;
  hd.out = d.out;
  hd.n = n;
  hd.step = M->step;
  hd.checksum = fnv1a(body.data(), body.size() * sizeof(float));
  FILE *f = std::fopen(path, "wb");
  if (!f) return set_error(DG_EIO, std::string("dg_learned_save: cannot open ") + path);
  const bool ok = std::fwrite(&hd, sizeof(hd), 1, f) == 1 &&
                  std::fwrite(body.data(), sizeof(float), body.size(), f) == body.size();
  if (std::fclose(f) != 0 || !ok) return set_error(DG_EIO, std::string("dg_learned_save: write failed: ") + path);
  return DG_OK;
}

extern "C" dg_status dg_learned_load(dg_handle *h, const char *path) {
  dg_status ds = learned_prologue(h, "dg_learned_load");
  if (ds != DG_OK) return ds;
  if (!path) return set_error(DG_EINVAL, "dg_learned_load: path is NULL");
  Mlp *M = h->mlp;
  const MlpDims &d = M->d;
  const int64_t n = public_nparams(d);
  FILE *f = std::fopen(path, "rb");
  if (!f) return set_error(DG_EIO, std::string("dg_learned_load: cannot open ") + path);
  CkptHeader hd;
  std::vector<float> body;
  bool ok = std::fread(&hd, sizeof(hd), 1, f) == 1;
  const bool shape = ok && std::memcmp(hd.magic, "DGMFNET1", 8) == 0 && hd.version == 1 && hd.k == h->k &&
                     hd.in == d.in && hd.hid == d.hid && hd.out == d.out && hd.n == n && hd.step >= 0;
  if (shape) {
    body.resize(size_t(3 * n));
    ok = std::fread(body.data(), sizeof(float), body.size(), f) == body.size();
    char extra;
    ok = ok && std::fread(&extra, 1, 1, f) == 0;  // nothing after the moments
  }
  std::fclose(f);
  if (!ok && !shape) return set_error(DG_EIO, std::string("dg_learned_load: cannot read ") + path);
  if (!shape) return set_error(DG_EINVAL, "dg_learned_load: not a network checkpoint of this degree");
  if (!ok) return set_error(DG_EIO, std::string("dg_learned_load: truncated or overlong file ") + path);
  if (fnv1a(body.data(), body.size() * sizeof(float)) != hd.checksum)
    return set_error(DG_EIO, "dg_learned_load: checksum mismatch");
  float *dst[3] = {M->master, M->m, M->v};
  hipError_t e = hipSuccess;
  for (int t = 0; t < 3 && e == hipSuccess; ++t) {
    const std::vector<float> pad = padded_from_public(d, body.data() + t * n);
    e = hipMemcpy(dst[t], pad.data(), pad.size() * sizeof(float), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = refresh(M, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_error(e, "dg_learned_load");
  M->step = hd.step;
  M->trained = true;
  return DG_OK;
}

// caller rows (B x in floats, B x out targets; device) into the activation buffers
static dg_status load_rows(dg_handle *h, const float *X, const float *T, int B, Acts &A, bool train,
                           hipStream_t s, const char *who) {
  if (!X || (train && !T)) return set_error(DG_EINVAL, std::string(who) + ": X or T is NULL");
  if (B < 64 || B % 64) return set_error(DG_EINVAL, std::string(who) + ": B must be a positive multiple of 64");
  dg_status ds = acts_for(h, B, train, A);
  if (ds != DG_OK) return ds;
  const MlpDims &d = h->mlp->d;
  hipLaunchKernelGGL(k_to_bf16_rows, dim3(blocks_for(int64_t(B) * d.inp)), dim3(kT), 0, s, X, B, d.in, d.inp, A.X);
  if (train)
    hipLaunchKernelGGL(k_rows_f32, dim3(blocks_for(int64_t(B) * d.outp)), dim3(kT), 0, s, T, B, d.out, d.outp, A.T);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, who);
  return DG_OK;
}

extern "C" dg_status dg_mlp_forward(dg_handle *h, const float *X, int32_t B, float *Y, void *stream) {
  dg_status ds = learned_prologue(h, "dg_mlp_forward");
  if (ds != DG_OK) return ds;
  if (!Y) return set_error(DG_EINVAL, "dg_mlp_forward: Y is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Acts A;
  if ((ds = load_rows(h, X, nullptr, B, A, false, s, "dg_mlp_forward")) != DG_OK) return ds;
  const MlpDims &d = h->mlp->d;
  hipError_t e = forward(h->mlp, A, B, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_rows_unpad, dim3(blocks_for(int64_t(B) * d.out)), dim3(kT), 0, s, A.Y, B, d.outp, d.out, Y);
    e = hipStreamSynchronize(s);
  }
  if (e != hipSuccess) return hip_error(e, "dg_mlp_forward");
  return DG_OK;
}

extern "C" dg_status dg_mlp_grad(dg_handle *h, const float *X, const float *T, int32_t B, float *grad_host,
                                 int64_t n, double *loss, void *stream) {
  dg_status ds = learned_prologue(h, "dg_mlp_grad");
  if (ds != DG_OK) return ds;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Acts A;
  if ((ds = load_rows(h, X, T, B, A, true, s, "dg_mlp_grad")) != DG_OK) return ds;
  hipError_t e = backward(h->mlp, A, B, s);
  if (e == hipSuccess && loss) e = hipMemcpyAsync(loss, A.loss, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_error(e, "dg_mlp_grad");
  return export_params(h, h->mlp->grad, grad_host, n, "dg_mlp_grad");
}

extern "C" dg_status dg_mlp_step(dg_handle *h, const float *X, const float *T, int32_t B, float lr, double *loss,
                                 void *stream) {
  dg_status ds = learned_prologue(h, "dg_mlp_step");
  if (ds != DG_OK) return ds;
  if (!(lr > 0.0f)) return set_error(DG_EINVAL, "dg_mlp_step: lr must be positive");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Acts A;
  if ((ds = load_rows(h, X, T, B, A, true, s, "dg_mlp_step")) != DG_OK) return ds;
  hipError_t e = backward(h->mlp, A, B, s);
  if (e == hipSuccess) e = adam_step(h->mlp, lr, s);
  if (e == hipSuccess && loss) e = hipMemcpyAsync(loss, A.loss, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_error(e, "dg_mlp_step");
  h->mlp->trained = true;
  return DG_OK;
}

extern "C" dg_status dg_learned_train(dg_handle *h, const dg_learn_opts *opts, dg_learn_stats *st, void *stream) {
  const auto t0 = std::chrono::steady_clock::now();
  dg_status ds = learned_prologue(h, "dg_learned_train");
  if (ds != DG_OK) return ds;
  if (!h->bj) return set_error(DG_EINVAL, "dg_learned_train: the handle needs DG_WITH_BLOCK_JACOBI");
  dg_learn_opts o{100000, 8, 20, 1024, 1e-3f, 6, 0};
  if (opts) o = *opts;
  if (o.npairs < 640 || o.nrhs < 1 || o.epochs < 0 || o.batch < 64 || o.batch % 64 || !(o.lr > 0.0f) ||
      o.max_steps < 0 || o.max_steps > 1024)
    return set_error(DG_EINVAL, "dg_learned_train: invalid options");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Mlp *M = h->mlp;
  const MlpDims &d = M->d;
  // He initialisation of W1, W2 (normal, variance 2 / fan-in, Box-Muller on
  // SplitMix64 draws); W3 and all biases zero, so the untrained network is
  // block Jacobi exactly
  {
    std::vector<float> pad(size_t(d.np), 0.0f);
    const uint64_t wseed = o.seed * 0x2545f4914f6cdd1dull + 11;
    uint64_t ctr = 0;
    auto normal = [&]() {
      const double a = u01(wseed, ctr++), b = u01(wseed, ctr++);
      return std::sqrt(-2.0 * std::log(a)) * std::cos(2.0 * M_PI * b);
    };
    const double s1 = std::sqrt(2.0 / d.in), s2 = std::sqrt(2.0 / d.hid);
    for (int oo = 0; oo < d.hid; ++oo)
      for (int i = 0; i < d.in; ++i) pad[d.oW1 + int64_t(oo) * d.inp + i] = float(s1 * normal());
    for (int oo = 0; oo < d.hid; ++oo)
      for (int i = 0; i < d.hid; ++i) pad[d.oW2 + int64_t(oo) * d.hid + i] = float(s2 * normal());
    hipError_t e = hipMemcpy(M->master, pad.data(), pad.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(M->m, 0, d.np * sizeof(float));
    if (e == hipSuccess) e = hipMemset(M->v, 0, d.np * sizeof(float));
    if (e == hipSuccess) e = refresh(M, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_error(e, "dg_learned_train: initialisation");
    M->step = 0;
  }
  // data set
  const int64_t np = o.npairs;
  uint16_t *Xall = nullptr;
  float *Tall = nullptr;
  int32_t *idx = nullptr;
  double *losses = nullptr;
  hipError_t e = hipMalloc(&Xall, size_t(np) * d.inp * sizeof(uint16_t));
  if (e == hipSuccess) e = hipMalloc(&Tall, size_t(np) * d.outp * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&idx, size_t(np) * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&losses, size_t(np / 64 + 16) * sizeof(double));
  auto cleanup = [&]() {
    for (void *p : {(void *)Xall, (void *)Tall, (void *)idx, (void *)losses})
      if (p) (void)hipFree(p);
  };
  if (e != hipSuccess) {
    cleanup();
    return hip_error(e, "dg_learned_train: data set");
  }
  if ((ds = make_data(h, o, Xall, Tall, np, s)) != DG_OK) {
    cleanup();
    return ds;
  }
  const double t_data = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  // 90 / 10 split of a shuffled order (Fisher-Yates on SplitMix64 draws)
  std::vector<int32_t> order(np);
  for (int64_t i = 0; i < np; ++i) order[i] = int32_t(i);
  uint64_t ctr = 0;
  const uint64_t sseed = o.seed * 0x9e3779b97f4a7c15ull + 3;
  auto shuffle = [&](int32_t *a, int64_t cnt) {
    for (int64_t i = cnt - 1; i > 0; --i) {
      const int64_t j = int64_t(u01(sseed, ctr++) * double(i + 1)) % (i + 1);
      std::swap(a[i], a[j]);
    }
  };
  shuffle(order.data(), np);
  const int B = o.batch;
  const int64_t nval = std::max<int64_t>(64, (np / 10) / 64 * 64);
  const int64_t ntrain = (np - nval) / B * B;
  if (ntrain < B) {
    cleanup();
    return set_error(DG_EINVAL, "dg_learned_train: npairs too small for the batch size");
  }
  Acts A;
  if ((ds = acts_for(h, std::max<int64_t>(B, 1024), true, A)) != DG_OK) {
    cleanup();
    return ds;
  }
  // validation loss: forward over the validation rows in blocks of 1024 (or B)
  auto val_loss = [&](double &out) -> hipError_t {
    const int vb = int(std::min<int64_t>(std::max<int64_t>(B, 1024), nval) / 64 * 64);
    double tot = 0.0;
    int64_t cnt = 0;
    hipError_t err;
    for (int64_t v0 = 0; v0 + vb <= nval; v0 += vb) {
      if ((err = hipMemcpyAsync(idx, order.data() + (np - nval) + v0, vb * sizeof(int32_t), hipMemcpyHostToDevice,
                                s)) != hipSuccess)
        return err;
      hipLaunchKernelGGL(k_rows, dim3(blocks_for(int64_t(vb) * (d.inp + d.outp))), dim3(kT), 0, s, Xall, Tall, idx,
                         vb, d.inp, d.outp, A.X, A.T);
      if ((err = forward(M, A, vb, s)) != hipSuccess) return err;
      hipLaunchKernelGGL(k_loss, dim3(256), dim3(kT), 0, s, A.Y, A.T, vb, d.out, d.outp, 0.0f, A.dY, A.dYT,
                         A.partial);
      hipLaunchKernelGGL(k_sum, dim3(1), dim3(kT), 0, s, A.partial, 256, 1.0 / (double(vb) * d.out), A.loss);
      double l = 0.0;
      if ((err = hipMemcpyAsync(&l, A.loss, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess) return err;
      if ((err = hipStreamSynchronize(s)) != hipSuccess) return err;
      tot += l * vb;
      cnt += vb;
    }
    out = cnt ? tot / double(cnt) : 0.0;
    return hipSuccess;
  };
  dg_learn_stats stats{};
  if ((e = val_loss(stats.val_loss_initial)) != hipSuccess) {
    cleanup();
    return hip_error(e, "dg_learned_train: validation");
  }
  const int nb_per_epoch = int(ntrain / B);
  for (int ep = 0; ep < o.epochs; ++ep) {
    shuffle(order.data(), np - nval);
    if ((e = hipMemcpyAsync(idx, order.data(), ntrain * sizeof(int32_t), hipMemcpyHostToDevice, s)) != hipSuccess)
      break;
    for (int bi = 0; bi < nb_per_epoch && e == hipSuccess; ++bi) {
      hipLaunchKernelGGL(k_rows, dim3(blocks_for(int64_t(B) * (d.inp + d.outp))), dim3(kT), 0, s, Xall, Tall,
                         idx + int64_t(bi) * B, B, d.inp, d.outp, A.X, A.T);
      if ((e = backward(M, A, B, s)) != hipSuccess) break;
      if ((e = adam_step(M, o.lr, s)) != hipSuccess) break;
      e = hipMemcpyAsync(losses + bi, A.loss, sizeof(double), hipMemcpyDeviceToDevice, s);
    }
    if (e != hipSuccess) break;
    std::vector<double> hl(nb_per_epoch);
    if ((e = hipMemcpyAsync(hl.data(), losses, nb_per_epoch * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess)
      break;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
    double tl = 0.0;
    for (double x : hl) tl += x;
    stats.train_loss = tl / nb_per_epoch;
    if (!std::isfinite(stats.train_loss)) {
      cleanup();
      return set_error(DG_ENAN, "dg_learned_train: non-finite training loss");
    }
  }
  if (e == hipSuccess) e = val_loss(stats.val_loss);
  cleanup();
  if (e != hipSuccess) return hip_error(e, "dg_learned_train: training");
  M->trained = true;
  stats.epochs = o.epochs;
  stats.steps = int32_t(M->step);
  stats.seconds_data = t_data;
  stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = stats;
  return DG_OK;
}
