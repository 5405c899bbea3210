// Block-Jacobi preconditioner: M = blockdiag(A_TT), the cell blocks of the
// WSIPG operator (volume term plus the self-coupling of the six faces: the
// operator applied to a function supported on T alone).
//
// Build (once, at setup):
//   1. Extraction by unit probing through the FP64 apply kernel.  Cells are
//      coloured by the parity of i1+i2+i3, so no two cells of one colour share
//      a face; x = e_j on every cell of one colour gives, on those cells,
//      column j of A_TT.  2 (k+1)^3 applications in total.  Column j of each
//      block is gathered into an FP64 store, column-major per cell.
//   2. In-place blocked Gauss-Jordan inversion in FP64, one workgroup per
//      cell, panels of BS rows/columns staged in LDS, without pivoting: the
//      form is coercive (x^T A x > 0 for x != 0, Sec. 2.2 with the upwind
//      flux and div b = 0), so every cell block and every Schur complement is
//      positive real and all pivots are positive.  A non-positive or
//      non-finite pivot is reported as an error.
//      Inverting the column-major store treated as row-major gives
//      (A^T)^{-1} = (A^{-1})^T row-major, i.e. A^{-1} column-major.
//   3. Conversion to FP32 (the store the FP64 solvers read) and to FP16 with
//      one scale per cell (max |entry|), the store of the FP32 inner solve of
//      GMRES-IR.
// Apply: z_T = A_TT^{-1} r_T with column-major blocks; each thread owns VR
// consecutive rows of one cell and reads VR entries of a column with one
// 16-byte load (VR = 4 in FP32, 8 in FP16; one row per thread when (k+1)^3
// is not a multiple of VR); FP64 accumulation.  HBM-bound: 4 (FP32) or 2
// (FP16) (k+1)^3 bytes of block store per DOF.
//
// Shared blocks: A_TT is a function of the cell's spacings, its face
// neighbours' spacings along each axis (the penalty), kappa on the cell and
// its neighbours (weights and penalty), which faces lie on the boundary, and
// b at the cell's quadrature points (Sec. 2.2).  Cells equal in all of these
// (to about 1e-11 relative) have equal blocks, so one block per class is
// probed, inverted and stored
// (on a uniform mesh with constant coefficients: 27 classes, one per
// combination of boundary faces).  The apply then walks groups of kBjGroup
// cells of one class: each block column is loaded once per group and used
// for all its cells, and the small class store stays in cache, so the apply
// moves little more than r and z.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "dg_internal.h"
#include "mesh_nb.h"

namespace dgmf {

constexpr int kBjThreads = 256;

// x[c*nb + j] = value on cells of the given colour
__global__ void k_bj_probe(double *__restrict__ x, int n1, int n2, int64_t ncells, int nb, int j,
                           int colour, double value) {
  for (int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; c < ncells;
       c += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i1 = c % n1, r = c / n1, i2 = r % n2, i3 = r / n2;
    if (int((i1 + i2 + i3) & 1) == colour) x[c * nb + j] = value;
  }
}

// B[slot][j*nb + i] = y[c*nb + i] on cells of the given colour (column j);
// slot = c, or slot[c] when blocks are shared (-1: not stored)
__global__ void k_bj_gather(const double *__restrict__ y, double *__restrict__ B, const int32_t *__restrict__ slot,
                            int n1, int n2, int64_t ncells, int nb, int j, int colour) {
  const int64_t total = ncells * nb;
  for (int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; g < total;
       g += int64_t(gridDim.x) * blockDim.x) {
    const int64_t c = g / nb;
    const int i = int(g - c * nb);
    const int64_t i1 = c % n1, r = c / n1, i2 = r % n2, i3 = r / n2;
    const int64_t b = slot ? int64_t(slot[c]) : c;
    if (int((i1 + i2 + i3) & 1) == colour && b >= 0) B[b * int64_t(nb) * nb + int64_t(j) * nb + i] = y[g];
  }
}

// In-place Gauss-Jordan inversion of one nb x nb block per workgroup (row-major
// view M[r*nb + c]).  For each pivot block P = [p0, p0+bs):
//   M_PP <- M_PP^{-1} =: I_P;        M_Pj <- I_P M_Pj            (j not in P)
//   M_ij <- M_ij - M_iP M_Pj(new);   M_iP <- -M_iP I_P           (i not in P)
// Dynamic LDS: Rp[BS][nb] (new row panel), Cp[nb][BS] (old column panel),
// Ip[BS][BS].
template <int BS>
__global__ __launch_bounds__(kBjThreads) void k_bj_invert(double *__restrict__ B, int nb, int *bad) {
  extern __shared__ double lds[];
  double *Rp = lds, *Cp = lds + BS * nb, *Ip = Cp + size_t(nb) * BS;
  __shared__ int s_bad;
  double *M = B + size_t(blockIdx.x) * nb * nb;
  const int t = threadIdx.x;
  if (t == 0) s_bad = 0;
  for (int p0 = 0; p0 < nb; p0 += BS) {
    const int bs = min(BS, nb - p0);
    // (a) pivot block into LDS
    for (int e = t; e < bs * bs; e += kBjThreads) Ip[(e / bs) * BS + e % bs] = M[size_t(p0 + e / bs) * nb + p0 + e % bs];
    // (d) old column panel (rows outside P)
    for (int e = t; e < nb * bs; e += kBjThreads) {
      const int i = e / bs, l = e % bs;
      Cp[i * BS + l] = M[size_t(i) * nb + p0 + l];
    }
    __syncthreads();
    // (b) invert the pivot block by scalar Gauss-Jordan (no pivoting)
    for (int k = 0; k < bs; ++k) {
      double a_rc = 0, a_rk = 0, a_kc = 0, piv = 1;
      const int r = t / bs, c = t % bs;
      const bool act = t < bs * bs;
      if (act) {
        a_rc = Ip[r * BS + c];
        a_rk = Ip[r * BS + k];
        a_kc = Ip[k * BS + c];
        piv = Ip[k * BS + k];
      }
      __syncthreads();
      if (act) {
        if (!(piv > 0.0) || !isfinite(piv)) s_bad = 1;
        const double d = 1.0 / piv;
        double v;
        if (r == k)
          v = (c == k) ? d : a_kc * d;
        else
          v = (c == k) ? -a_rk * d : fma(-a_rk * d, a_kc, a_rc);
        Ip[r * BS + c] = v;
      }
      __syncthreads();
    }
    // (c) new row panel R = I_P M_P,: for columns outside P (to LDS and memory)
    for (int e = t; e < bs * nb; e += kBjThreads) {
      const int k = e / nb, c = e % nb;
      if (c >= p0 && c < p0 + bs) continue;
      double s = 0.0;
      for (int l = 0; l < bs; ++l) s = fma(Ip[k * BS + l], M[size_t(p0 + l) * nb + c], s);
      Rp[k * nb + c] = s;
    }
    __syncthreads();
    for (int e = t; e < bs * nb; e += kBjThreads) {
      const int k = e / nb, c = e % nb;
      if (c >= p0 && c < p0 + bs) continue;
      M[size_t(p0 + k) * nb + c] = Rp[k * nb + c];
    }
    // (e) rank-bs update of the rest, (f) new column panel, (g) pivot block
    for (int e = t; e < nb * nb; e += kBjThreads) {
      const int i = e / nb, j = e % nb;
      if (i >= p0 && i < p0 + bs) continue;
      if (j >= p0 && j < p0 + bs) {
        const int l = j - p0;
        double s = 0.0;
        for (int m = 0; m < bs; ++m) s = fma(Cp[i * BS + m], Ip[m * BS + l], s);
        M[size_t(i) * nb + j] = -s;
      } else {
        double s = M[size_t(i) * nb + j];
        for (int l = 0; l < bs; ++l) s = fma(-Cp[i * BS + l], Rp[l * nb + j], s);
        M[size_t(i) * nb + j] = s;
      }
    }
    for (int e = t; e < bs * bs; e += kBjThreads) M[size_t(p0 + e / bs) * nb + p0 + e % bs] = Ip[(e / bs) * BS + e % bs];
    __syncthreads();
  }
  if (t == 0 && s_bad) atomicOr(bad, 1);
}

__global__ void k_to_f32(const double *__restrict__ a, float *__restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    b[i] = float(a[i]);
}

// z[c*nb + i] = sum_j Binv[c][j*nb + i] r[c*nb + j]
template <typename TR, typename TZ>
__global__ __launch_bounds__(kBjThreads) void k_bj_apply(const float *__restrict__ Binv, const TR *__restrict__ r,
                                                         TZ *__restrict__ z, int nb, int64_t total) {
  for (int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; g < total;
       g += int64_t(gridDim.x) * blockDim.x) {
    const int64_t c = g / nb;
    const int i = int(g - c * nb);
    const float *Bc = Binv + c * int64_t(nb) * nb + i;
    const TR *rc = r + c * nb;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int j = 0;
    for (; j + 4 <= nb; j += 4) {
      s0 = fma(double(Bc[size_t(j) * nb]), double(rc[j]), s0);
      s1 = fma(double(Bc[size_t(j + 1) * nb]), double(rc[j + 1]), s1);
      s2 = fma(double(Bc[size_t(j + 2) * nb]), double(rc[j + 2]), s2);
      s3 = fma(double(Bc[size_t(j + 3) * nb]), double(rc[j + 3]), s3);
    }
    for (; j < nb; ++j) s0 = fma(double(Bc[size_t(j) * nb]), double(rc[j]), s0);
    z[g] = TZ((s0 + s1) + (s2 + s3));
  }
}

// VR rows per thread, one 16-byte load per column; sc: per-cell scale or null
template <typename TR, typename TZ, typename TB, int VR>
__global__ __launch_bounds__(kBjThreads) void k_bj_apply_vec(const TB *__restrict__ Binv, const float *__restrict__ sc,
                                                             const TR *__restrict__ r, TZ *__restrict__ z, int nb,
                                                             int64_t ncells) {
  typedef TB bvec __attribute__((ext_vector_type(VR)));
  const int per = nb / VR;
  const int64_t total = ncells * per;
  for (int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; g < total;
       g += int64_t(gridDim.x) * blockDim.x) {
    const int64_t c = g / per;
    const int i0 = int(g - c * per) * VR;
    const TB *Bc = Binv + c * int64_t(nb) * nb + i0;
    const TR *rc = r + c * nb;
    double acc[VR];
#pragma unroll
    for (int e = 0; e < VR; ++e) acc[e] = 0.0;
    for (int j = 0; j < nb; ++j) {
      const bvec col = *reinterpret_cast<const bvec *>(Bc + size_t(j) * nb);
      const double rj = double(rc[j]);
#pragma unroll
      for (int e = 0; e < VR; ++e) acc[e] = fma(double(col[e]), rj, acc[e]);
    }
    const double s = sc ? double(sc[c]) : 1.0;
#pragma unroll
    for (int e = 0; e < VR; ++e) z[c * nb + i0 + e] = TZ(acc[e] * s);
  }
}

// shared blocks: thread (group, VR rows) applies the group's block to its
// kBjGroup cells; padding entries (-1) read the group's first cell and
// write nothing.  TA: accumulation type.  JU columns per step: with VR = 4
// the r values of JU consecutive columns come in one 16-byte load per cell
// (JU = 16 / sizeof(TR); nb is then a multiple of 4, hence of JU).
template <typename TR, typename TZ, typename TA, int VR>
__global__ __launch_bounds__(kBjThreads) void k_bj_apply_grp(const float *__restrict__ Binv,
                                                             const int32_t *__restrict__ cells,
                                                             const int32_t *__restrict__ gblock,
                                                             const TR *__restrict__ r, TZ *__restrict__ z, int nb,
                                                             int64_t ngroups) {
  constexpr int JU = (VR == 4) ? int(16 / sizeof(TR)) : 1;
  const int per = nb / VR;
  const int64_t total = ngroups * per;
  for (int64_t g = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; g < total;
       g += int64_t(gridDim.x) * blockDim.x) {
    const int64_t grp = g / per;
    const int i0 = int(g - grp * per) * VR;
    const float *Bc = Binv + int64_t(gblock[grp]) * nb * nb + i0;
    const int32_t *cg = cells + grp * kBjGroup;
    const int32_t c0 = cg[0];
    int64_t off[kBjGroup];
    bool live[kBjGroup];
#pragma unroll
    for (int q = 0; q < kBjGroup; ++q) {
      const int32_t c = cg[q];
      live[q] = c >= 0;
      off[q] = int64_t(c >= 0 ? c : c0) * nb;
    }
    TA acc[kBjGroup][VR];
#pragma unroll
    for (int q = 0; q < kBjGroup; ++q)
#pragma unroll
      for (int e = 0; e < VR; ++e) acc[q][e] = TA(0);
    for (int j = 0; j < nb; j += JU) {
      float col[JU][VR];
      TR rv[kBjGroup][JU];
      if constexpr (VR == 4) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        typedef TR rvec __attribute__((ext_vector_type(JU)));
#pragma unroll
        for (int u = 0; u < JU; ++u) {
          const f4 v = *reinterpret_cast<const f4 *>(Bc + size_t(j + u) * nb);
#pragma unroll
          for (int e = 0; e < 4; ++e) col[u][e] = v[e];
        }
#pragma unroll
        for (int q = 0; q < kBjGroup; ++q) {
          const rvec v = *reinterpret_cast<const rvec *>(r + off[q] + j);
#pragma unroll
          for (int u = 0; u < JU; ++u) rv[q][u] = v[u];
        }
      } else {
#pragma unroll
        for (int e = 0; e < VR; ++e) col[0][e] = Bc[size_t(j) * nb + e];
#pragma unroll
        for (int q = 0; q < kBjGroup; ++q) rv[q][0] = r[off[q] + j];
      }
#pragma unroll
      for (int u = 0; u < JU; ++u)
#pragma unroll
        for (int q = 0; q < kBjGroup; ++q) {
          const TA rj = TA(rv[q][u]);
#pragma unroll
          for (int e = 0; e < VR; ++e) acc[q][e] = fma(TA(col[u][e]), rj, acc[q][e]);
        }
    }
#pragma unroll
    for (int q = 0; q < kBjGroup; ++q)
      if (live[q])
#pragma unroll
        for (int e = 0; e < VR; ++e) z[off[q] + i0 + e] = TZ(acc[q][e]);
  }
}

// Shared blocks, 216 or 512 rows: a workgroup takes GPW = 256 / (nb / 4)
// groups (4 or 2, at most 32 cells) and stages their r values in LDS, 32
// columns at a time (lds[column][cell], coalesced loads of each cell's
// contiguous values).  A thread owns 4 rows of one group; per column it
// loads 16 bytes of the block from cache and reads its 8 cells' values as
// LDS broadcasts, instead of 8 global loads that every thread of the group
// repeats.
constexpr int kBjStageCols = 32;
constexpr int kBjStageCells = 32;
template <typename TR, typename TZ, typename TA>
__global__ __launch_bounds__(kBjThreads) void k_bj_apply_grp_lds(const float *__restrict__ Binv,
                                                                 const int32_t *__restrict__ cells,
                                                                 const int32_t *__restrict__ gblock,
                                                                 const TR *__restrict__ r, TZ *__restrict__ z,
                                                                 int nb, int64_t ngroups) {
  __shared__ TA rs[kBjStageCols * kBjStageCells];
  __shared__ int32_t cs[kBjStageCells];
  const int per = nb / 4;
  const int gpw = kBjThreads / per;  // groups per workgroup (<= 4)
  const int t = threadIdx.x;
  const int q = t / per;  // group of this thread within the workgroup
  const int64_t grp = int64_t(blockIdx.x) * gpw + q;
  const bool act = q < gpw && grp < ngroups;
  const int i0 = (t - q * per) * 4;
  const int ncl = gpw * kBjGroup;  // cells staged per workgroup
  // cell list of the workgroup; padding (-1, or groups past the end) reads
  // the first cell of the workgroup and is never written
  if (t < ncl) {
    const int64_t g = int64_t(blockIdx.x) * gpw + t / kBjGroup;
    const int32_t c = g < ngroups ? cells[g * kBjGroup + t % kBjGroup] : -1;
    cs[t] = c;
  }
  __syncthreads();
  const int32_t cfirst = cs[0];
  const float *Bc = Binv + (act ? int64_t(gblock[grp]) * nb * nb + i0 : 0);
  TA acc[kBjGroup][4];
#pragma unroll
  for (int c = 0; c < kBjGroup; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[c][e] = TA(0);
  for (int j0 = 0; j0 < nb; j0 += kBjStageCols) {
    const int jc = min(kBjStageCols, nb - j0);
    __syncthreads();  // the previous chunk has been consumed
    for (int e = t; e < ncl * jc; e += kBjThreads) {
      const int cl = e / jc, jj = e - cl * jc;
      const int32_t c = cs[cl] >= 0 ? cs[cl] : cfirst;
      rs[jj * kBjStageCells + cl] = TA(r[int64_t(c) * nb + j0 + jj]);
    }
    __syncthreads();
    if (act) {
      typedef float f4 __attribute__((ext_vector_type(4)));
      const TA *rq = rs + q * kBjGroup;
      for (int jj = 0; jj < jc; ++jj) {
        const f4 v = *reinterpret_cast<const f4 *>(Bc + size_t(j0 + jj) * nb);
        TA rv[kBjGroup];
#pragma unroll
        for (int c = 0; c < kBjGroup; ++c) rv[c] = rq[jj * kBjStageCells + c];
#pragma unroll
        for (int c = 0; c < kBjGroup; ++c)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[c][e] = fma(TA(v[e]), rv[c], acc[c][e]);
      }
    }
  }
  if (act) {
#pragma unroll
    for (int c = 0; c < kBjGroup; ++c) {
      const int32_t cell = cs[q * kBjGroup + c];
      if (cell >= 0)
#pragma unroll
        for (int e = 0; e < 4; ++e) z[int64_t(cell) * nb + i0 + e] = TZ(acc[c][e]);
    }
  }
}

// FP16 copy with one scale per cell: h = fp16(b / sc_c), sc_c = max |b| over the block
__global__ __launch_bounds__(kBjThreads) void k_to_f16_scaled(const double *__restrict__ B, int nb,
                                                              _Float16 *__restrict__ H, float *__restrict__ sc) {
  __shared__ double red[kBjThreads / 64];
  const size_t nn = size_t(nb) * nb;
  const double *Bc = B + blockIdx.x * nn;
  double mx = 0.0;
  for (size_t i = threadIdx.x; i < nn; i += kBjThreads) mx = fmax(mx, fabs(Bc[i]));
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  double m = 0.0;
  for (int w = 0; w < kBjThreads / 64; ++w) m = fmax(m, red[w]);
  const float s = m > 0.0 ? float(m) : 1.0f;
  const double inv = 1.0 / double(s);
  for (size_t i = threadIdx.x; i < nn; i += kBjThreads) H[blockIdx.x * nn + i] = _Float16(Bc[i] * inv);
  if (threadIdx.x == 0) sc[blockIdx.x] = s;
}

static int grid_for(int64_t work) {
  const int64_t g = (work + kBjThreads - 1) / kBjThreads;
  return int(g < 1 ? 1 : (g > (1 << 20) ? (1 << 20) : g));
}

// Key entry rounded to 36 significant bits: the node differences of a
// uniform mesh differ in their last bits from cell to cell, and blocks whose
// inputs agree to about 1e-11 agree far below the FP32 rounding of the
// stored inverse.  Negative values (-1 marks a boundary face) pass unchanged.
static double key_round(double v) {
  if (!(v > 0.0)) return v;
  int e = 0;
  const double m = std::frexp(v, &e);
  return std::ldexp(std::nearbyint(std::ldexp(m, 36)), e - 36);
}

// Classes of cells with equal blocks (see the top of this file); cls[c] is
// the class of cell c, rep[class] its first cell.
static void cell_classes(const dg_problem *p, std::vector<int32_t> &cls, std::vector<int64_t> &rep) {
  const int n1 = p->ncell[0], n2 = p->ncell[1], n3 = p->ncell[2];
  const int64_t ncells = int64_t(n1) * n2 * n3;
  const int64_t stride[3] = {1, n1, int64_t(n1) * n2};
  cls.resize(size_t(ncells));
  rep.clear();
  std::unordered_map<std::string, int32_t> ids;
  double key[22];
  const int periodic = (p->flags >> 2) & 7;
  for (int64_t c = 0; c < ncells; ++c) {
    const int i[3] = {int(c % n1), int((c / n1) % n2), int(c / stride[2])};
    FaceNb nb[3][2];
    for (int a = 0; a < 3; ++a)
      for (int e = 0; e < 2; ++e) nb[a][e] = face_nb(int(c), i[a], p->ncell[a], int(stride[a]), (periodic >> a) & 1, e);
    int nk = 0;
    for (int a = 0; a < 3; ++a) {
      const double *X = p->nodes[a];
      key[nk++] = nb[a][0].in ? X[nb[a][0].ja + 1] - X[nb[a][0].ja] : -1.0;
      key[nk++] = X[i[a] + 1] - X[i[a]];
      key[nk++] = nb[a][1].in ? X[nb[a][1].ja + 1] - X[nb[a][1].ja] : -1.0;
    }
    if (p->kappa) {
      key[nk++] = p->kappa[c];
      for (int a = 0; a < 3; ++a) {
        key[nk++] = nb[a][0].in ? p->kappa[nb[a][0].cell] : -1.0;
        key[nk++] = nb[a][1].in ? p->kappa[nb[a][1].cell] : -1.0;
      }
    }
    if (p->flags & DG_KAPPA_POLY) {
      // a non-constant diffusion factor along axis j: the cell's position along j
      for (int j = 0; j < 3; ++j)
        if (p->kappa_poly[3 * j + 1] != 0.0 || p->kappa_poly[3 * j + 2] != 0.0) key[nk++] = p->nodes[j][i[j]];
    }
    if (p->flags & DG_B_PRODUCT) {
      // a non-constant factor along axis j makes b depend on the cell's position along j
      for (int j = 0; j < 3; ++j)
        if (p->b_freq[j] != 0.0 || p->b_freq[3 + j] != 0.0 || p->b_freq[6 + j] != 0.0)
          key[nk++] = p->nodes[j][i[j]];
    } else {
      // a sine part of b_r makes it depend on the coordinate along b_axis[r]
      for (int r = 0; r < 3; ++r)
        if (p->b_sin[r] != 0.0) key[nk++] = p->nodes[p->b_axis[r]][i[p->b_axis[r]]];
    }
    for (int t = 0; t < nk; ++t) key[t] = key_round(key[t]);
    auto it = ids.emplace(std::string(reinterpret_cast<const char *>(key), size_t(nk) * sizeof(double)),
                          int32_t(rep.size()));
    if (it.second) rep.push_back(c);
    cls[size_t(c)] = it.first->second;
  }
}

dg_status build_block_jacobi(dg_handle *h, const dg_problem *p) {
  const int n = h->k + 1, nb = n * n * n;
  if (nb > kMaxBjBlock)
    return set_error(DG_EINVAL, "dg_setup: block Jacobi supports k <= 7 ((k+1)^3 <= 512)");
  std::vector<int32_t> cls;
  std::vector<int64_t> rep;
  cell_classes(p, cls, rep);
  const int64_t ncls = int64_t(rep.size());
  const bool share = 2 * ncls <= h->ncells;
  const int64_t nblocks = share ? ncls : h->ncells;
  const size_t ndof = size_t(h->ndof), nblk = size_t(nblocks) * nb * nb;
  double *x = nullptr, *y = nullptr, *B = nullptr;
  int *bad = nullptr;
  int32_t *slot = nullptr;
  hipError_t e;
  auto fail = [&](hipError_t err, const char *what) {
    for (void *q : {(void *)x, (void *)y, (void *)B, (void *)bad, (void *)slot})
      if (q) (void)hipFree(q);
    return hip_error(err, what);
  };
  if ((e = hipMalloc(&x, ndof * sizeof(double))) != hipSuccess) return fail(e, "block Jacobi: probe vector");
  if ((e = hipMalloc(&y, ndof * sizeof(double))) != hipSuccess) return fail(e, "block Jacobi: probe vector");
  if ((e = hipMalloc(&B, nblk * sizeof(double))) != hipSuccess) return fail(e, "block Jacobi: FP64 blocks");
  if ((e = hipMalloc(&bad, sizeof(int))) != hipSuccess) return fail(e, "block Jacobi: flag");
  if ((e = hipMalloc(&h->bj, nblk * sizeof(float))) != hipSuccess) {
    h->bj = nullptr;
    return fail(e, "block Jacobi: FP32 blocks");
  }
  if (share) {
    // probe store slot of each cell: its class for the class's first cell
    std::vector<int32_t> hs(static_cast<size_t>(h->ncells));
    for (int64_t c = 0; c < h->ncells; ++c) hs[size_t(c)] = rep[size_t(cls[size_t(c)])] == c ? cls[size_t(c)] : -1;
    // groups of kBjGroup cells of one class, cells in ascending order
    std::vector<int64_t> cnt(size_t(ncls), 0), first(size_t(ncls) + 1, 0);
    for (int32_t k : cls) ++cnt[size_t(k)];
    for (int64_t k = 0; k < ncls; ++k)
      first[size_t(k) + 1] = first[size_t(k)] + (cnt[size_t(k)] + kBjGroup - 1) / kBjGroup;
    const int64_t ngroups = first[size_t(ncls)];
    std::vector<int32_t> hc(static_cast<size_t>(ngroups) * kBjGroup, -1), hg(static_cast<size_t>(ngroups));
    std::vector<int64_t> fill(size_t(ncls), 0);
    for (int64_t c = 0; c < h->ncells; ++c) {
      const int32_t k = cls[size_t(c)];
      hc[size_t(first[size_t(k)] * kBjGroup + fill[size_t(k)]++)] = int32_t(c);
    }
    for (int64_t k = 0; k < ncls; ++k)
      for (int64_t g = first[size_t(k)]; g < first[size_t(k) + 1]; ++g) hg[size_t(g)] = int32_t(k);
    if ((e = hipMalloc(&slot, hs.size() * sizeof(int32_t))) != hipSuccess) return fail(e, "block Jacobi: slots");
    if ((e = hipMalloc(&h->bj_cells, hc.size() * sizeof(int32_t))) != hipSuccess) {
      h->bj_cells = nullptr;
      return fail(e, "block Jacobi: cell groups");
    }
    if ((e = hipMalloc(&h->bj_gblock, hg.size() * sizeof(int32_t))) != hipSuccess) {
      h->bj_gblock = nullptr;
      return fail(e, "block Jacobi: cell groups");
    }
    if ((e = hipMemcpy(slot, hs.data(), hs.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(h->bj_cells, hc.data(), hc.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(h->bj_gblock, hg.data(), hg.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess)
      return fail(e, "block Jacobi: cell groups");
    h->bj_ngroups = ngroups;
  }
  const hipStream_t s = nullptr;
  if ((e = hipMemsetAsync(x, 0, ndof * sizeof(double), s)) != hipSuccess) return fail(e, "block Jacobi: memset");
  if ((e = hipMemsetAsync(bad, 0, sizeof(int), s)) != hipSuccess) return fail(e, "block Jacobi: memset");
  const int n1 = h->mesh.ncell[0], n2 = h->mesh.ncell[1];
  const int gc = grid_for(h->ncells), gr = grid_for(int64_t(ndof));
  for (int colour = 0; colour < 2; ++colour)
    for (int j = 0; j < nb; ++j) {
      hipLaunchKernelGGL(k_bj_probe, dim3(gc), dim3(kBjThreads), 0, s, x, n1, n2, int64_t(h->ncells), nb, j,
                         colour, 1.0);
      if ((e = apply_f64(h, x, y, s)) != hipSuccess) return fail(e, "block Jacobi: probe apply");
      hipLaunchKernelGGL(k_bj_gather, dim3(gr), dim3(kBjThreads), 0, s, y, B, slot, n1, n2, int64_t(h->ncells), nb,
                         j, colour);
      hipLaunchKernelGGL(k_bj_probe, dim3(gc), dim3(kBjThreads), 0, s, x, n1, n2, int64_t(h->ncells), nb, j,
                         colour, 0.0);
    }
  if ((e = hipGetLastError()) != hipSuccess) return fail(e, "block Jacobi: probing");
  // panels stay under 64 KiB of LDS: BS = 16 up to (k+1)^3 = 216, else 4
  if (nb <= 216) {
    constexpr int BS = 16;
    const size_t lds = sizeof(double) * (2 * size_t(BS) * nb + BS * BS);
    hipLaunchKernelGGL((k_bj_invert<BS>), dim3(unsigned(nblocks)), dim3(kBjThreads), lds, s, B, nb, bad);
  } else {
    constexpr int BS = 4;
    const size_t lds = sizeof(double) * (2 * size_t(BS) * nb + BS * BS);
    hipLaunchKernelGGL((k_bj_invert<BS>), dim3(unsigned(nblocks)), dim3(kBjThreads), lds, s, B, nb, bad);
  }
  if ((e = hipGetLastError()) != hipSuccess) return fail(e, "block Jacobi: inversion");
  hipLaunchKernelGGL(k_to_f32, dim3(4096), dim3(kBjThreads), 0, s, B, h->bj, nblk);
  if (!share) {
    // FP16 store for the FP32 inner solves (shared blocks stay in FP32: the
    // class store is small and read from cache)
    if ((e = hipMalloc(&h->bj16, nblk * sizeof(_Float16))) != hipSuccess) {
      h->bj16 = nullptr;
      return fail(e, "block Jacobi: FP16 blocks");
    }
    if ((e = hipMalloc(&h->bj16_scale, size_t(nblocks) * sizeof(float))) != hipSuccess) {
      h->bj16_scale = nullptr;
      return fail(e, "block Jacobi: FP16 scales");
    }
    hipLaunchKernelGGL(k_to_f16_scaled, dim3(unsigned(nblocks)), dim3(kBjThreads), 0, s, B, nb, h->bj16,
                       h->bj16_scale);
  }
  int hbad = 0;
  if ((e = hipMemcpy(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost)) != hipSuccess)
    return fail(e, "block Jacobi: flag readback");
  for (void *q : {(void *)x, (void *)y, (void *)B, (void *)bad, (void *)slot})
    if (q) (void)hipFree(q);
  h->bj_nb = nb;
  h->bj_nblocks = nblocks;
  if (hbad) return set_error(DG_ENAN, "dg_setup: a cell block has a non-positive pivot (the form is not coercive)");
  return DG_OK;
}

template <typename TR, typename TZ>
hipError_t bj_apply(const dg_handle *h, const TR *r, TZ *z, hipStream_t s, bool half_store) {
  const int nb = h->bj_nb;
  if (h->bj_cells) {
    // shared blocks; FP32 accumulation for the FP32 inner solves
    using TA = typename std::conditional<std::is_same<TZ, float>::value, float, double>::type;
    if (nb == 216 || nb == 512)
      hipLaunchKernelGGL((k_bj_apply_grp_lds<TR, TZ, TA>), dim3(unsigned((h->bj_ngroups + kBjThreads / (nb / 4) - 1) /
                                                                       (kBjThreads / (nb / 4)))),
                         dim3(kBjThreads), 0, s, h->bj, h->bj_cells, h->bj_gblock, r, z, nb, h->bj_ngroups);
    else if (nb % 4 == 0)
      hipLaunchKernelGGL((k_bj_apply_grp<TR, TZ, TA, 4>), dim3(grid_for(h->bj_ngroups * (nb / 4))), dim3(kBjThreads),
                         0, s, h->bj, h->bj_cells, h->bj_gblock, r, z, nb, h->bj_ngroups);
    else
      hipLaunchKernelGGL((k_bj_apply_grp<TR, TZ, TA, 1>), dim3(grid_for(h->bj_ngroups * nb)), dim3(kBjThreads), 0, s,
                         h->bj, h->bj_cells, h->bj_gblock, r, z, nb, h->bj_ngroups);
  } else if (half_store && h->bj16 && nb % 8 == 0) {
    hipLaunchKernelGGL((k_bj_apply_vec<TR, TZ, _Float16, 8>), dim3(grid_for(h->ncells * (nb / 8))), dim3(kBjThreads),
                       0, s, h->bj16, h->bj16_scale, r, z, nb, int64_t(h->ncells));
  } else if (nb % 4 == 0) {
    hipLaunchKernelGGL((k_bj_apply_vec<TR, TZ, float, 4>), dim3(grid_for(h->ncells * (nb / 4))), dim3(kBjThreads), 0,
                       s, h->bj, nullptr, r, z, nb, int64_t(h->ncells));
  } else {
    const int64_t total = h->ndof;
    hipLaunchKernelGGL((k_bj_apply<TR, TZ>), dim3(grid_for(total)), dim3(kBjThreads), 0, s, h->bj, r, z, nb, total);
  }
  return hipGetLastError();
}

template hipError_t bj_apply<double, double>(const dg_handle *, const double *, double *, hipStream_t, bool);
template hipError_t bj_apply<float, float>(const dg_handle *, const float *, float *, hipStream_t, bool);

}  // namespace dgmf
