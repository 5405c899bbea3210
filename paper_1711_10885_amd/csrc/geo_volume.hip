// Volume term of the operator on multilinear cells (Sec. 4; Problem C of
// Sec. 5.1) in the pencil layout of the tuned kernel: sweeps A, B, C of the
// cell's coefficients to u and the reference gradient at the N^3 Gauss points
// (NI <= N modes per direction, rectangular contractions as for the raised
// rule), the pointwise flux with the geometry of the trilinear map at each
// point, and the transposed sweeps C', B', A' into y.  The face terms are
// added afterwards by the reference-layout kernel in its faces-only mode
// (apply_ref.hip), which starts from this y.
//
// Geometry per point.  Lane (q1, q2) streams the points along axis 3.  The
// trilinear map is bilinear in (s1, s2) at fixed s3 and linear in s3, so the
// lane folds its (s1, s2) into six numbers per coordinate once (the values,
// the s1- and s2-derivatives at s3 = 0 and their changes to s3 = 1) and gets
// the point X and the Jacobian J at each s3 from nine multiply-adds.  The
// flux is then as in the reference kernel: with C = cof(J) = det(J) J^{-T},
// x^(r) = w (C^T (D C grad_ref u / det J - b u))_r and x^(0) = w det J c u.
#include "fused_kernel.h"
#include "ref_geo.h"

namespace dgmf {

struct GeoVolArgs {
  double xi[kMaxQ], w[kMaxQ];  // the N-point Gauss rule on [0, 1]
  int groups;                  // workgroups per XCD slot (grid = 8 * groups)
  FastDiv fd_n1, fd_n2;
};

template <int N, int NI>
__global__ __launch_bounds__(FCfg<N>::THREADS) __attribute__((amdgpu_waves_per_eu(2))) void geo_volume_kernel(
    const double *__restrict__ x, double *__restrict__ y, RefMesh M, GeoVolArgs A) {
  using C = FCfg<N>;
  using TO = TabOff<N>;
  using T = double;
  constexpr int NN = C::NN, PS = C::PS;
  constexpr int NIII = NI * NI * NI;
  constexpr int H2 = N / 2;
  constexpr int EX = 3 * NN * PS;  // largest exchange: three pencil sets of stride PS
  __shared__ double lds[C::CPB * EX];
  __shared__ double vtx[C::CPB * 24];

  const int tid = threadIdx.x;
  const int cl = tid / C::LANES;
  const int p = tid - cl * C::LANES;
  const int alpha = p % N, beta = p / N;
  const bool slot = cl < C::CPB;
  const int wg = blockIdx.x;
  const int lblock = (wg & 7) * A.groups + (wg >> 3);
  const int L = lblock * C::CPB + (slot ? cl : 0);
  const bool active = slot && L < M.ncells;
  int cell = active ? L : 0;
  int i0, i1, i2;
  {
    const int r = fdiv(cell, A.fd_n1);
    i0 = cell - r * M.ncell[0];
    i2 = fdiv(r, A.fd_n2);
    i1 = r - i2 * M.ncell[1];
  }
  if constexpr (C::CPB == 1) {  // one cell per workgroup: cell values in scalar registers
    cell = wave_uniform(cell);
    i0 = wave_uniform(i0);
    i1 = wave_uniform(i1);
    i2 = wave_uniform(i2);
  }
  double *R = lds + (slot ? cl : 0) * EX;
  double *VT = vtx + (slot ? cl : 0) * 24;
  const CT<N, T> tab0{0};

  // prologue: the cell's x pencil along axis 1 and its eight vertices
  const bool lin = alpha < NI && beta < NI;
  T X[N];
  {
    const int al = min(alpha, NI - 1), be = min(beta, NI - 1);
    const T *xp = x + size_t(cell) * NIII + NI * NI * be + NI * al;
#pragma unroll
    for (int t = 0; t < N; ++t) X[t] = (t < NI && lin) ? xp[t < NI ? t : 0] : T(0);
  }
  if (slot)
    for (int i = p; i < 24; i += C::LANES) {
      const int v = i / 3, r = i - 3 * v;
      const int g0 = i0 + (v & 1), g1 = i1 + ((v >> 1) & 1), g2 = i2 + (v >> 2);
      VT[i] = M.verts[3 * (size_t(g0) + size_t(M.ncell[0] + 1) * (g1 + size_t(M.ncell[1] + 1) * g2)) + r];
    }
  // A (axis 1, lanes (j2, j3)): V1 x, D1 x as B-pencils (q1 + N j3) along j2
  {
    const cptr tb = fresh(tab0);
    T Tv[N], Td[N];
    eo_mv<N, false, T, NI>(tb + TO::V, X, Tv);
    eo_mv<N, true, T, NI>(tb + TO::D, X, Td);
    if (slot) {
#pragma unroll
      for (int q = 0; q < N; ++q) {
        R[(q + N * beta) * PS + alpha] = Tv[q];
        R[NN * PS + (q + N * beta) * PS + alpha] = Td[q];
      }
    }
  }
  __syncthreads();
  // B (axis 2, lanes (q1, j3))
  T vv[N], dv[N], vd[N];
  {
    const cptr tb = fresh(tab0);
    T P[N], Q[N];
#pragma unroll
    for (int t = 0; t < N; ++t) {
      P[t] = R[p * PS + t];
      Q[t] = R[NN * PS + p * PS + t];
    }
    eo_mv<N, false, T, NI>(tb + TO::V, P, vv);
    eo_mv<N, false, T, NI>(tb + TO::V, Q, dv);
    eo_mv<N, true, T, NI>(tb + TO::D, P, vd);
  }
  __syncthreads();
  if (slot) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
      R[(alpha + N * q) * PS + beta] = vv[q];
      R[NN * PS + (alpha + N * q) * PS + beta] = dv[q];
      R[2 * NN * PS + (alpha + N * q) * PS + beta] = vd[q];
    }
  }
  __syncthreads();
  // C (axis 3, lanes (q1, q2)) with the pointwise flux and C' streamed over
  // the point pairs (q3, N-1-q3)
  T Pc[N], Qc[N], Sc[N];
#pragma unroll
  for (int t = 0; t < N; ++t) {
    Pc[t] = R[p * PS + t];
    Qc[t] = R[NN * PS + p * PS + t];
    Sc[t] = R[2 * NN * PS + p * PS + t];
  }
  T Wvv[N], Wdv[N], Wvd[N];
#pragma unroll
  for (int j = 0; j < N; ++j) Wvv[j] = Wdv[j] = Wvd[j] = T(0);
  {
    const cptr tb = fresh(tab0);
    const cptr V = tb + TO::V, D = tb + TO::D, Wt = tb + TO::W;
    // the lane's fold of the trilinear map at (s1, s2) = (xi_q1, xi_q2)
    const double s0 = A.xi[alpha], s1 = A.xi[beta];
    double b0[3], db[3], e0[3], de[3], f0[3], df[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      auto v = [&](int c0, int c1, int c2) { return VT[3 * (c0 + 2 * c1 + 4 * c2) + r]; };
      const double v000 = v(0, 0, 0), v100 = v(1, 0, 0), v010 = v(0, 1, 0), v110 = v(1, 1, 0);
      const double v001 = v(0, 0, 1), v101 = v(1, 0, 1), v011 = v(0, 1, 1), v111 = v(1, 1, 1);
      const double d00 = v100 - v000, d10 = v110 - v010, d01 = v101 - v001, d11 = v111 - v011;
      const double a00 = fma(s0, d00, v000), a10 = fma(s0, d10, v010);
      const double a01 = fma(s0, d01, v001), a11 = fma(s0, d11, v011);
      const double g0 = a10 - a00, g1 = a11 - a01;
      const double c0 = fma(s1, g0, a00), c1 = fma(s1, g1, a01);
      const double h0 = fma(s1, d10 - d00, d00), h1 = fma(s1, d11 - d01, d01);
      b0[r] = c0;
      db[r] = c1 - c0;
      e0[r] = h0;
      de[r] = h1 - h0;
      f0[r] = g0;
      df[r] = g1 - g0;
    }
    const double kap = M.kappa ? M.kappa[cell] : 1.0;
    const double wab = A.w[alpha] * A.w[beta];
    auto flux = [&](T u, T g0, T g1, T g2, int q3, T W, T &x0, T &x1, T &x2, T &x3) {
      const double s2 = A.xi[q3];
      double Xp[3], J[9], Cm[9];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        Xp[r] = fma(s2, db[r], b0[r]);
        J[3 * r + 0] = fma(s2, de[r], e0[r]);
        J[3 * r + 1] = fma(s2, df[r], f0[r]);
        J[3 * r + 2] = db[r];
      }
      const double det = cof3(J, Cm), idet = 1.0 / det;
      double g[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) g[r] = (Cm[3 * r] * g0 + Cm[3 * r + 1] * g1 + Cm[3 * r + 2] * g2) * idet;
      const double kx = kap * geo_kp(M, Xp);
      double F[3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
        F[r] = kx * (M.K[3 * r] * g[0] + M.K[3 * r + 1] * g[1] + M.K[3 * r + 2] * g[2]) - geo_b(M, r, Xp) * u;
      x0 = W * det * M.c * u;
      x1 = W * (Cm[0] * F[0] + Cm[3] * F[1] + Cm[6] * F[2]);
      x2 = W * (Cm[1] * F[0] + Cm[4] * F[1] + Cm[7] * F[2]);
      x3 = W * (Cm[2] * F[0] + Cm[5] * F[1] + Cm[8] * F[2]);
    };
#pragma unroll
    for (int h = 0; h < H2; ++h) {
      T Eu = 0, Ou = 0, E0 = 0, O0 = 0, E1 = 0, O1 = 0, E2 = 0, O2 = 0;
#pragma unroll
      for (int t = 0; t < NI; t += 2) {
        Eu = fma(V[h * N + t], Pc[t], Eu);
        E0 = fma(V[h * N + t], Qc[t], E0);
        E1 = fma(V[h * N + t], Sc[t], E1);
        E2 = fma(D[h * N + t], Pc[t], E2);
      }
#pragma unroll
      for (int t = 1; t < NI; t += 2) {
        Ou = fma(V[h * N + t], Pc[t], Ou);
        O0 = fma(V[h * N + t], Qc[t], O0);
        O1 = fma(V[h * N + t], Sc[t], O1);
        O2 = fma(D[h * N + t], Pc[t], O2);
      }
      const T W = wab * Wt[h];
      T a0, a1, a2, a3, m0, m1, m2, m3;
      flux(Eu + Ou, E0 + O0, E1 + O1, E2 + O2, h, W, a0, a1, a2, a3);
      flux(Eu - Ou, E0 - O0, E1 - O1, O2 - E2, N - 1 - h, W, m0, m1, m2, m3);
      const T s0_ = a0 + m0, d0_ = a0 - m0, s1_ = a1 + m1, d1_ = a1 - m1;
      const T s2_ = a2 + m2, d2_ = a2 - m2, s3_ = a3 + m3, d3_ = a3 - m3;
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        const bool ev = (j & 1) == 0;
        Wvv[j] = fma(V[h * N + j], ev ? s0_ : d0_, Wvv[j]);
        Wvv[j] = fma(D[h * N + j], ev ? d3_ : s3_, Wvv[j]);
        Wdv[j] = fma(V[h * N + j], ev ? s1_ : d1_, Wdv[j]);
        Wvd[j] = fma(V[h * N + j], ev ? s2_ : d2_, Wvd[j]);
      }
    }
    if (N & 1) {
      constexpr int m = N / 2;
      T u = 0, g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
      for (int t = 0; t < NI; t += 2) {
        u = fma(V[m * N + t], Pc[t], u);
        g0 = fma(V[m * N + t], Qc[t], g0);
        g1 = fma(V[m * N + t], Sc[t], g1);
      }
#pragma unroll
      for (int t = 1; t < NI; t += 2) g2 = fma(D[m * N + t], Pc[t], g2);
      T x0, x1, x2, x3;
      flux(u, g0, g1, g2, m, wab * Wt[m], x0, x1, x2, x3);
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        if ((j & 1) == 0) {
          Wvv[j] = fma(V[m * N + j], x0, Wvv[j]);
          Wdv[j] = fma(V[m * N + j], x1, Wdv[j]);
          Wvd[j] = fma(V[m * N + j], x2, Wvd[j]);
        } else {
          Wvv[j] = fma(D[m * N + j], x3, Wvv[j]);
        }
      }
    }
  }
  // C' results as B'-pencils (q1 + N j3) along q2
  constexpr int BPS = NN * PL<N>::S;
  __syncthreads();
  if (slot) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int a = PL<N>::at(alpha + N * j, beta);
      R[a] = Wvv[j];
      R[BPS + a] = Wdv[j];
      R[2 * BPS + a] = Wvd[j];
    }
  }
  __syncthreads();
  // B' (axis 2, lanes (q1, j3))
  T Vv[N], Vd[N];
  {
    const cptr tb = fresh(tab0);
    T P[N], Q[N], S[N];
#pragma unroll
    for (int t = 0; t < N; ++t) {
      const int a = PL<N>::at(p, t);
      P[t] = R[a];
      Q[t] = R[BPS + a];
      S[t] = R[2 * BPS + a];
    }
    eo_mtv<N, false, false, T, NI>(tb + TO::V, P, Vv);
    eo_mtv<N, true, true, T, NI>(tb + TO::D, S, Vv);
    eo_mtv<N, false, false, T, NI>(tb + TO::V, Q, Vd);
  }
  __syncthreads();
  if (slot) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      R[(j + N * beta) * PS + alpha] = Vv[j];
      R[NN * PS + (j + N * beta) * PS + alpha] = Vd[j];
    }
  }
  __syncthreads();
  // A' (axis 1, lanes (j2, j3)) and the store of the cell's rows
  if (active && lin) {
    const cptr tb = fresh(tab0);
    T P[N], Q[N], Yv[N];
#pragma unroll
    for (int t = 0; t < N; ++t) {
      P[t] = R[p * PS + t];
      Q[t] = R[NN * PS + p * PS + t];
    }
    eo_mtv<N, false, false, T, NI>(tb + TO::V, P, Yv);
    eo_mtv<N, true, true, T, NI>(tb + TO::D, Q, Yv);
    const size_t off = size_t(cell) * NIII + NI * NI * beta + NI * alpha;
#pragma unroll
    for (int t = 0; t < NI; ++t) y[off + t] = Yv[t];
  }
}

template <int N, int NI>
static hipError_t launch_geo_volume_n(const dg_handle *h, const double *x, double *y, hipStream_t s) {
  using C = FCfg<N>;
  if (h->tabq.m != N || h->k + 1 != NI) return hipErrorInvalidValue;
  GeoVolArgs A;
  for (int q = 0; q < N; ++q) {
    A.xi[q] = h->tabq.xi[q];
    A.w[q] = h->tabq.w[q];
  }
  A.fd_n1 = make_fastdiv(h->mesh.ncell[0]);
  A.fd_n2 = make_fastdiv(h->mesh.ncell[1]);
  const int nblocks = int((h->ncells + C::CPB - 1) / C::CPB);
  A.groups = (nblocks + 7) / 8;
  const RefMesh M = make_ref_mesh(h, true);
  hipLaunchKernelGGL((geo_volume_kernel<N, NI>), dim3(unsigned(8 * A.groups)), dim3(C::THREADS), 0, s, x, y, M, A);
  return hipGetLastError();
}

// The rules of multilinear handles: k+1, k+3 and q = 3p + 4 (up to 13 points
// per direction at k = 7; at 12 and 13 points a workgroup holds one cell in
// three waves and the kernel spills 176 and 256 bytes per lane; with the
// faces-only reference kernel after it, the apply is still 1.13x faster than
// the reference kernel doing both terms).
template <int NI>
static hipError_t launch_geo_volume_ni(const dg_handle *h, const double *x, double *y, hipStream_t s) {
  constexpr int QC = (3 * (NI - 1) + 6) / 2;
  const int m = h->tabq.m;
  if (m == NI) return launch_geo_volume_n<NI, NI>(h, x, y, s);
  if constexpr (NI + 2 <= 11) {
    if (m == NI + 2) return launch_geo_volume_n<NI + 2, NI>(h, x, y, s);
  }
  if constexpr (QC <= 13 && QC != NI + 2 && QC != NI) {
    if (m == QC) return launch_geo_volume_n<QC, NI>(h, x, y, s);
  }
  return hipErrorNotSupported;
}

bool geo_volume_supported(const dg_handle *h) { return h->tabq.m <= 13 && h->k + 1 <= 8; }

hipError_t launch_geo_volume_f64(const dg_handle *h, const double *x, double *y, hipStream_t s) {
  switch (h->k + 1) {
    case 2: return launch_geo_volume_ni<2>(h, x, y, s);
    case 3: return launch_geo_volume_ni<3>(h, x, y, s);
    case 4: return launch_geo_volume_ni<4>(h, x, y, s);
    case 5: return launch_geo_volume_ni<5>(h, x, y, s);
    case 6: return launch_geo_volume_ni<6>(h, x, y, s);
    case 7: return launch_geo_volume_ni<7>(h, x, y, s);
    case 8: return launch_geo_volume_ni<8>(h, x, y, s);
    default: return hipErrorNotSupported;
  }
}

}  // namespace dgmf
