// Reference-layout FP64 apply kernel: one workgroup per cell, every tensor of
// the sum factorization staged in LDS, one thread per output entry of each 1D
// contraction.  Simple and general in k and in the number of Gauss points
// per direction Q (Q = k+1, or k+3 for the raised rule q = 2p + 4 of
// Problem B, Sec. 5.1, where every 1D contraction is rectangular, Q x (k+1));
// the tuned kernels are checked against the oracle exactly like this one.
//
// Per cell T (owner computes, so no two workgroups write the same entry):
//  * volume term of eq. (blf), Algorithm 1 steps 1-3: u and grad u at the
//    (k+1)^3 Gauss points by 1D contractions (eq. (evalfe), eq.
//    (sum_fact_kernel)), the pointwise flux x^(r) of eq. (gauss_points), and
//    the transposed contractions of eq. (evalblf);
//  * each of the six faces (steps 4-6 / 8-10): the normal direction is
//    contracted first (traces of u and d_a u, Sec. 3.4), then the two
//    tangential directions; the pointwise upwind, weighted-average and penalty
//    terms; the transposed tangential contractions; and the normal direction
//    last, into the test functions of T only.
//
// Multilinear meshes (GEO = true; Sec. 4, Problem C of Sec. 5.1): every cell
// is the trilinear image of the reference cube through its eight vertices.
// The map and its Jacobian J are evaluated at each quadrature point by one
// linear contraction per direction (the Q1 map is a degree-1 tensor
// polynomial, so this is sum factorization with 2-point factors), from the
// vertices of the cell and of its six face neighbours staged in LDS.  With
// C = cof(J) = det(J) J^{-T} the volume flux enters the transposed
// contractions as w C^T (D C grad_ref u / det J - b u) and the reaction as
// w det J c u; on the face xi_a = e the outer area-weighted normal is
// +-C e_a, and the symmetry term integrates against the reference gradient
// with the vector -W w_T [[u]] C^T D nu / det J.  Every face quantity of
// Sec. 2.2 (d = nu^T D nu, weights, gamma_F, b . nu) is taken per point;
// |F| and |T| in gamma_F come from per-face and per-cell tables.
#include "dg_internal.h"
#include "mesh_nb.h"
#include "ref_geo.h"

namespace dgmf {

constexpr int kRefThreads = 256;

// One 1D contraction along axis AX of a block in LDS with output dimensions
// (O0, O1, O2) (axis 0 fastest; O2 = 1 for a 2D block) and input length LI
// along AX (the other input dimensions are those of the output), all
// compile-time constants.  The TPC threads of one cell (local index lt) share
// the work:
//   out[.., q, ..] (+)= sum_{t < LI} A(q, t) in[.., t, ..],
// A(q, t) = Mat[q][t] (TRANS = false: evaluation, points from basis
// coefficients) or Mat[t][q] (TRANS = true: integration against the test
// functions); an optional second term with in2, Mat2.
// BLK = 1: one thread per output entry.  BLK > 1: a work item is one pencil
// along AX and BLK consecutive outputs q of it; the pencil's inputs are read
// from LDS once into registers and serve BLK outputs, and the pencils vary
// fastest across threads, so the threads of a group read the same matrix
// entries (LDS broadcasts).  Measured: faster for the multilinear cells at
// k >= 3, slower at k <= 2 and for the (k+1)-point rule, where the kernel is
// bound by latency rather than by LDS reads.
template <int LD, bool TRANS, int AX, int O0, int O1, int O2, int LI, int TPC, int BLK = 1>
__device__ inline void contract(int lt, double *out, const double *in, const double (*Mat)[LD],
                                const double *in2 = nullptr, const double (*Mat2)[LD] = nullptr) {
  constexpr int I0 = AX == 0 ? LI : O0, I1 = AX == 1 ? LI : O1;
  constexpr int IS[3] = {1, I0, I0 * I1};          // input strides
  if constexpr (BLK == 1) {
    constexpr int NT = O0 * O1 * O2;
    for (int i = lt; i < NT; i += TPC) {
      const int i0 = i % O0, i1 = (i / O0) % O1, i2 = i / (O0 * O1);
      const int q = AX == 0 ? i0 : (AX == 1 ? i1 : i2);
      const int base = (AX == 0 ? 0 : i0 * IS[0]) + (AX == 1 ? 0 : i1 * IS[1]) + (AX == 2 ? 0 : i2 * IS[2]);
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < LI; ++t) {
        const double a = TRANS ? Mat[t][q] : Mat[q][t];
        s = fma(a, in[base + t * IS[AX]], s);
      }
      if (in2) {
#pragma unroll
        for (int t = 0; t < LI; ++t) {
          const double a = TRANS ? Mat2[t][q] : Mat2[q][t];
          s = fma(a, in2[base + t * IS[AX]], s);
        }
      }
      out[i] = s;
    }
    return;
  }
  constexpr int OS[3] = {1, O0, O0 * O1};          // output strides
  constexpr int OA = AX == 0 ? O0 : (AX == 1 ? O1 : O2);  // outputs along AX
  constexpr int PA = AX == 0 ? O1 : O0, PB = AX == 2 ? O1 : O2;  // pencil grid (the other two axes)
  constexpr int NP = PA * PB;
  constexpr int RB = OA < BLK ? OA : BLK;
  constexpr int NC = (OA + RB - 1) / RB;
  for (int w = lt; w < NP * NC; w += TPC) {
    const int pp = w % NP, c = w / NP;
    const int pa = pp % PA, pb = pp / PA;
    // the two non-AX indices (pa on the lower axis, pb on the upper)
    const int ibase = AX == 0 ? (pa * IS[1] + pb * IS[2]) : (AX == 1 ? (pa * IS[0] + pb * IS[2]) : (pa * IS[0] + pb * IS[1]));
    const int obase = AX == 0 ? (pa * OS[1] + pb * OS[2]) : (AX == 1 ? (pa * OS[0] + pb * OS[2]) : (pa * OS[0] + pb * OS[1]));
    const int q0 = c * RB;
    double v[LI];
#pragma unroll
    for (int t = 0; t < LI; ++t) v[t] = in[ibase + t * IS[AX]];
    double s[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int q = q0 + r < OA ? q0 + r : OA - 1;
      double acc = 0.0;
#pragma unroll
      for (int t = 0; t < LI; ++t) acc = fma(TRANS ? Mat[t][q] : Mat[q][t], v[t], acc);
      s[r] = acc;
    }
    if (in2) {
#pragma unroll
      for (int t = 0; t < LI; ++t) v[t] = in2[ibase + t * IS[AX]];
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int q = q0 + r < OA ? q0 + r : OA - 1;
#pragma unroll
        for (int t = 0; t < LI; ++t) s[r] = fma(TRANS ? Mat2[t][q] : Mat2[q][t], v[t], s[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
      if (q0 + r < OA) out[obase + (q0 + r) * OS[AX]] = s[r];
  }
}

// CPB cells per workgroup, TPB / CPB threads and one LDS slice each
// (CPB = 1 for the (k+1)-point reference variant).  TPB = 512 where one
// cell's LDS exceeds half of a CU's (q = 3p + 4 at k = 6, 7): one workgroup
// per CU then still brings two waves per SIMD.
// Two waves per SIMD: without the cap some instantiations took more than 256
// registers and ran one wave per SIMD.
// VOL = false (multilinear cells with the volume already in y, from the
// pencil-layout volume kernel of geo_volume.hip): y is read as the start of the
// accumulation and only the face terms are added.
template <int N, int Q, int CPB, bool GEO, bool VOL = true, int TPB = kRefThreads>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(2))) void apply_ref_kernel(const double *__restrict__ x,
                                                                double *__restrict__ y,
                                                                RefMesh M, RefTab<N, Q> T) {
  constexpr int NB = N * N * N, NF = N * N, QB = Q * Q * Q, QF = Q * Q;
  constexpr int TPC = TPB / CPB;
  __shared__ double sV[Q][N], sD[Q][N], sw[Q], sxi[Q], sev[2][N], sed[2][N];
  // raised rule and multilinear cells: the six faces are processed together
  // (one pass per contraction over a (., ., 6) block); their 24 NF + 72 QF
  // doubles share the region of the volume tensors, which are dead by then
  constexpr bool BATCH = (Q != N) || GEO;
  constexpr int VBN = GEO ? 3 * kVB * kVB * kVB : 1;
  constexpr int BK = (GEO && N >= 4) ? 4 : 1;  // register blocking of the contractions (k >= 3)
  __shared__ double VBs[CPB][VBN];
  constexpr int FB = 24 * NF + 72 * QF;
  constexpr int RSZ = (BATCH && FB > 7 * QB) ? FB : 7 * QB;
  __shared__ double Xs[CPB][NB], Ys[CPB][NB], Rs[CPB][RSZ];
  constexpr int FQ = BATCH ? 1 : QF;  // per-face buffers of the face-by-face path
  __shared__ double Fs[CPB][16][FQ];
  const int tid = threadIdx.x;
  const int slot = tid / TPC, lt = tid % TPC;
  double *X = Xs[slot], *Y = Ys[slot];
  double *B0 = Rs[slot], *B1 = B0 + QB, *B2 = B0 + 2 * QB, *B3 = B0 + 3 * QB;
  double *B4 = B0 + 4 * QB, *B5 = B0 + 5 * QB, *B6 = B0 + 6 * QB;
  double(*F)[FQ] = Fs[slot];
  // a slot past the last cell repeats it (every thread reaches every barrier)
  // and does not store
  const bool active = int(blockIdx.x) * CPB + slot < M.ncells;
  const int cell = active ? int(blockIdx.x) * CPB + slot : M.ncells - 1;
  const int N1 = M.ncell[0], N2 = M.ncell[1];
  const int ic[3] = {cell % N1, (cell / N1) % N2, cell / (N1 * N2)};
  const int cstride[3] = {1, N1, N1 * N2};

  // the cell's x (and y) and the vertex block: every global load issued
  // before any of them is stored to LDS
  {
    constexpr int NXL = (NB + TPC - 1) / TPC, NVL = GEO ? (VBN + TPC - 1) / TPC : 1;
    const double *xT = x + size_t(cell) * NB;
    const double *yT = y + size_t(cell) * NB;
    double xv[NXL], yv[NXL], vv[NVL];
#pragma unroll
    for (int j = 0; j < NXL; ++j) {
      const int i = lt + j * TPC;
      xv[j] = i < NB ? xT[i] : 0.0;
      if constexpr (!VOL) yv[j] = i < NB ? yT[i] : 0.0;
    }
    if constexpr (GEO) {
      // vertices (i_a - 1 .. i_a + 2 per axis; zero where outside the vertex grid)
#pragma unroll
      for (int j = 0; j < NVL; ++j) {
        const int i = lt + j * TPC;
        const int v = i / 3, r = i - 3 * v;
        const int g0 = ic[0] - 1 + v % kVB, g1 = ic[1] - 1 + (v / kVB) % kVB, g2 = ic[2] - 1 + v / (kVB * kVB);
        const bool in = i < VBN && g0 >= 0 && g0 <= M.ncell[0] && g1 >= 0 && g1 <= M.ncell[1] && g2 >= 0 &&
                        g2 <= M.ncell[2];
        vv[j] = in ? M.verts[3 * (size_t(g0) + size_t(M.ncell[0] + 1) * (g1 + size_t(M.ncell[1] + 1) * g2)) + r]
                   : 0.0;
      }
    }
    // the 1D tables, while the loads above are in flight
    for (int i = tid; i < Q * N; i += TPB) {
      sV[i / N][i % N] = T.V[i / N][i % N];
      sD[i / N][i % N] = T.D[i / N][i % N];
    }
    if (tid < Q) {
      sw[tid] = T.w[tid];
      sxi[tid] = T.xi[tid];
    }
    if (tid < N) {
      sev[0][tid] = T.ev[0][tid];
      sev[1][tid] = T.ev[1][tid];
      sed[0][tid] = T.ed[0][tid];
      sed[1][tid] = T.ed[1][tid];
    }
#pragma unroll
    for (int j = 0; j < NXL; ++j) {
      const int i = lt + j * TPC;
      if (i < NB) {
        X[i] = xv[j];
        if constexpr (!VOL) Y[i] = yv[j];
      }
    }
    if constexpr (GEO) {
#pragma unroll
      for (int j = 0; j < NVL; ++j) {
        const int i = lt + j * TPC;
        if (i < VBN) VBs[slot][i] = vv[j];
      }
    }
  }
  __syncthreads();

  const double h[3] = {M.h[0][ic[0]], M.h[1][ic[1]], M.h[2][ic[2]]};
  const double kap = M.kappa ? M.kappa[cell] : 1.0;
  const double vol = h[0] * h[1] * h[2];

  if constexpr (VOL) {
  // ---------------- volume: forward (u, d1 u, d2 u, d3 u at points) --------
  contract<N, false, 0, Q, N, N, N, TPC, BK>(lt, B0, X, sV);  // V1 x
  contract<N, false, 0, Q, N, N, N, TPC, BK>(lt, B1, X, sD);  // D1 x
  __syncthreads();
  contract<N, false, 1, Q, Q, N, N, TPC, BK>(lt, B2, B0, sV);  // V2 V1 x
  contract<N, false, 1, Q, Q, N, N, TPC, BK>(lt, B3, B1, sV);  // V2 D1 x
  contract<N, false, 1, Q, Q, N, N, TPC, BK>(lt, B4, B0, sD);  // D2 V1 x
  __syncthreads();
  contract<N, false, 2, Q, Q, Q, N, TPC, BK>(lt, B0, B2, sV);  // u
  contract<N, false, 2, Q, Q, Q, N, TPC, BK>(lt, B1, B3, sV);  // d^1 u (reference)
  contract<N, false, 2, Q, Q, Q, N, TPC, BK>(lt, B5, B4, sV);  // d^2 u
  contract<N, false, 2, Q, Q, Q, N, TPC, BK>(lt, B6, B2, sD);  // d^3 u
  __syncthreads();
  // ---------------- volume: pointwise flux (eq. (gauss_points)) ------------
  if constexpr (GEO) {
    const double *VB = VBs[slot];
    for (int i = lt; i < QB; i += TPC) {
      const int q1 = i % Q, q2 = (i / Q) % Q, q3 = i / QF;
      double Xp[3], J[9], C[9];
      tri_map(VB, 1, 1, 1, sxi[q1], sxi[q2], sxi[q3], Xp, J);
      const double det = cof3(J, C), idet = 1.0 / det;
      const double u = B0[i];
      const double gr[3] = {B1[i], B5[i], B6[i]};  // reference gradient
      double g[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) g[r] = (C[3 * r] * gr[0] + C[3 * r + 1] * gr[1] + C[3 * r + 2] * gr[2]) * idet;
      const double kx = kap * geo_kp(M, Xp);
      double F[3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
        F[r] = kx * (M.K[3 * r] * g[0] + M.K[3 * r + 1] * g[1] + M.K[3 * r + 2] * g[2]) - geo_b(M, r, Xp) * u;
      const double W = sw[q1] * sw[q2] * sw[q3];
      B0[i] = W * det * M.c * u;
      B1[i] = W * (C[0] * F[0] + C[3] * F[1] + C[6] * F[2]);
      B5[i] = W * (C[1] * F[0] + C[4] * F[1] + C[7] * F[2]);
      B6[i] = W * (C[2] * F[0] + C[5] * F[1] + C[8] * F[2]);
    }
  } else
  for (int i = lt; i < QB; i += TPC) {
    const int q1 = i % Q, q2 = (i / Q) % Q, q3 = i / QF;
    const double u = B0[i];
    const double g[3] = {B1[i] / h[0], B5[i] / h[1], B6[i] / h[2]};
    const int qq[3] = {q1, q2, q3};
    const double W = sw[q1] * sw[q2] * sw[q3] * vol;
    double Fr[3];
    for (int r = 0; r < 3; ++r) {
      const int ax = M.b_axis[r];
      const double br = M.bprod ? M.bf[3 * r][ic[0] * Q + q1] * M.bf[3 * r + 1][ic[1] * Q + q2] *
                                      M.bf[3 * r + 2][ic[2] * Q + q3]
                                : M.bvol[r][ic[ax] * Q + qq[ax]];
      const double kx = M.kpoly ? kap * M.kf[0][ic[0] * Q + q1] * M.kf[1][ic[1] * Q + q2] * M.kf[2][ic[2] * Q + q3]
                                : kap;
      Fr[r] = kx * (M.K[3 * r] * g[0] + M.K[3 * r + 1] * g[1] + M.K[3 * r + 2] * g[2]) - br * u;
    }
    B0[i] = W * M.c * u;
    B1[i] = W * Fr[0] / h[0];
    B5[i] = W * Fr[1] / h[1];
    B6[i] = W * Fr[2] / h[2];
  }
  __syncthreads();
  // ---------------- volume: transposed contractions (eq. (evalblf)) --------
  contract<N, true, 2, Q, Q, N, Q, TPC, BK>(lt, B2, B0, sV, B6, sD);  // along 3: V^T x0 + D^T x3
  contract<N, true, 2, Q, Q, N, Q, TPC, BK>(lt, B3, B1, sV);          // V^T x1
  contract<N, true, 2, Q, Q, N, Q, TPC, BK>(lt, B4, B5, sV);          // V^T x2
  __syncthreads();
  contract<N, true, 1, Q, N, N, Q, TPC, BK>(lt, B0, B2, sV, B4, sD);  // along 2
  contract<N, true, 1, Q, N, N, Q, TPC, BK>(lt, B1, B3, sV);
  __syncthreads();
  contract<N, true, 0, N, N, N, Q, TPC, BK>(lt, Y, B0, sV, B1, sD);  // along 1
  __syncthreads();
  }

  // ---------------- faces --------------------------------------------------
  if constexpr (BATCH) {
    double *R = Rs[slot];
    double *TUo = R, *TDo = R + 6 * NF, *TUn = R + 12 * NF, *TDn = R + 18 * NF;  // (N, N, 6) each
    double *P = R + 24 * NF;                                                       // (Q, Q, 6) each
    double *S0 = P, *S1 = P + 6 * QF, *S2 = P + 12 * QF, *S3 = P + 18 * QF;
    double *uo = P + 24 * QF, *un = P + 30 * QF, *gao = P + 36 * QF, *gan = P + 42 * QF;
    double *gbo = P + 48 * QF, *gbn = P + 54 * QF, *gco = P + 60 * QF, *gcn = P + 66 * QF;
    // normal direction first: modal traces of face f on its (jb, jc) grid
    for (int i = lt; i < 6 * NF; i += TPC) {
      const int f = i / NF, ii = i - f * NF;
      const int a = f >> 1, e = f & 1;
      const int jb = ii % N, jc = ii / N;
      const int sa = sel3i(a, 1, N, NF), sb = (a == 0) ? N : 1, sc = (a == 2) ? N : NF;
      const int base = jb * sb + jc * sc;
      const FaceNb nb = face_nb(cell, sel3i(a, ic[0], ic[1], ic[2]), sel3i(a, M.ncell[0], M.ncell[1], M.ncell[2]),
                                sel3i(a, cstride[0], cstride[1], cstride[2]), (M.periodic >> a) & 1, e);
      double uo_ = 0, do_ = 0, un_ = 0, dn_ = 0;
      for (int ja = 0; ja < N; ++ja) {
        uo_ = fma(sev[e][ja], X[base + ja * sa], uo_);
        do_ = fma(sed[e][ja], X[base + ja * sa], do_);
      }
      if (nb.in) {
        const double *xN = x + size_t(nb.cell) * NB;
        for (int ja = 0; ja < N; ++ja) {
          const double v = xN[base + ja * sa];
          un_ = fma(sev[1 - e][ja], v, un_);
          dn_ = fma(sed[1 - e][ja], v, dn_);
        }
      }
      TUo[i] = uo_;
      TDo[i] = do_;
      TUn[i] = un_;
      TDn[i] = dn_;
    }
    __syncthreads();
    // tangential evaluation of all six faces: first b, then c
    contract<N, false, 0, Q, N, 6, N, TPC, BK>(lt, S0, TUo, sV);
    contract<N, false, 0, Q, N, 6, N, TPC, BK>(lt, S1, TUo, sD);
    contract<N, false, 0, Q, N, 6, N, TPC, BK>(lt, S2, TUn, sV);
    contract<N, false, 0, Q, N, 6, N, TPC, BK>(lt, S3, TUn, sD);
    __syncthreads();
    contract<N, false, 1, Q, Q, 6, N, TPC, BK>(lt, uo, S0, sV);
    contract<N, false, 1, Q, Q, 6, N, TPC, BK>(lt, gbo, S1, sV);
    contract<N, false, 1, Q, Q, 6, N, TPC, BK>(lt, gco, S0, sD);
    contract<N, false, 1, Q, Q, 6, N, TPC, BK>(lt, un, S2, sV);
    contract<N, false, 1, Q, Q, 6, N, TPC, BK>(lt, gbn, S3, sV);
    contract<N, false, 1, Q, Q, 6, N, TPC, BK>(lt, gcn, S2, sD);
    __syncthreads();
    contract<N, false, 0, Q, N, 6, N, TPC, BK>(lt, S0, TDo, sV);
    contract<N, false, 0, Q, N, 6, N, TPC, BK>(lt, S1, TDn, sV);
    __syncthreads();
    contract<N, false, 1, Q, Q, 6, N, TPC, BK>(lt, gao, S0, sV);
    contract<N, false, 1, Q, Q, 6, N, TPC, BK>(lt, gan, S1, sV);
    __syncthreads();
    // pointwise face terms of every face point (as in the per-face loop below)
    if constexpr (GEO) {
      const double *VB = VBs[slot];
      for (int i = lt; i < 6 * QF; i += TPC) {
        const int f = i / QF, ii = i - f * QF;
        const int a = f >> 1, e = f & 1;
        const int b = (a == 0) ? 1 : 0, c = (a == 2) ? 1 : 2;
        const int qb = ii % Q, qc = ii / Q;
        const FaceNb nb = face_nb(cell, sel3i(a, ic[0], ic[1], ic[2]), sel3i(a, M.ncell[0], M.ncell[1], M.ncell[2]),
                                  sel3i(a, cstride[0], cstride[1], cstride[2]), 0, e);
        const bool interior = nb.in;
        // reference coordinates of the point on the own side (s_a = e) and
        // on the neighbour's side (s_a = 1 - e)
        const double tb = sxi[qb], tc = sxi[qc], ee = double(e);
        const double s0 = a == 0 ? ee : tb, s1 = a == 1 ? ee : (a == 0 ? tb : tc), s2 = a == 2 ? ee : tc;
        double Xp[3], J[9], Co[9];
        tri_map(VB, 1, 1, 1, s0, s1, s2, Xp, J);
        const double deto = cof3(J, Co);
        const double sg = e ? 1.0 : -1.0;
        // outer area-weighted normal: column a of cof(J), signed
        const double nv0 = sg * sel3d(a, Co[0], Co[1], Co[2]);
        const double nv1 = sg * sel3d(a, Co[3], Co[4], Co[5]);
        const double nv2 = sg * sel3d(a, Co[6], Co[7], Co[8]);
        const double nrm = sqrt(nv0 * nv0 + nv1 * nv1 + nv2 * nv2);
        const double inrm = 1.0 / nrm, nu[3] = {nv0 * inrm, nv1 * inrm, nv2 * inrm};
        double Kn[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) Kn[r] = M.K[3 * r] * nu[0] + M.K[3 * r + 1] * nu[1] + M.K[3 * r + 2] * nu[2];
        const double nKn = nu[0] * Kn[0] + nu[1] * Kn[1] + nu[2] * Kn[2];
        // physical gradients from the reference gradients (axis order)
        const double gro[3] = {a == 0 ? gao[i] : gbo[i], a == 1 ? gao[i] : (a == 0 ? gbo[i] : gco[i]),
                               a == 2 ? gao[i] : gco[i]};
        double Kgo = 0.0;  // (K nu) . grad u_o
#pragma unroll
        for (int r = 0; r < 3; ++r)
          Kgo += Kn[r] * (Co[3 * r] * gro[0] + Co[3 * r + 1] * gro[1] + Co[3 * r + 2] * gro[2]);
        const double ideto = 1.0 / deto;
        Kgo *= ideto;
        const double kpx = geo_kp(M, Xp);
        const double kxo = kap * kpx;
        double kxn = 0.0, Kgn = 0.0;
        if (interior) {
          const int o = e ? 2 : 0;
          double Xn[3], Jn[9], Cn[9];
          tri_map(VB, a == 0 ? o : 1, a == 1 ? o : 1, a == 2 ? o : 1, a == 0 ? 1.0 - ee : s0, a == 1 ? 1.0 - ee : s1,
                  a == 2 ? 1.0 - ee : s2, Xn, Jn);
          const double detn = cof3(Jn, Cn);
          const double grn[3] = {a == 0 ? gan[i] : gbn[i], a == 1 ? gan[i] : (a == 0 ? gbn[i] : gcn[i]),
                                 a == 2 ? gan[i] : gcn[i]};
#pragma unroll
          for (int r = 0; r < 3; ++r)
            Kgn += Kn[r] * (Cn[3 * r] * grn[0] + Cn[3 * r + 1] * grn[1] + Cn[3 * r + 2] * grn[2]);
          Kgn /= detn;
          kxn = (M.kappa ? M.kappa[nb.cell] : 1.0) * kpx;
        }
        const double dT = kxo * nKn, dN = kxn * nKn;
        const double rs = 1.0 / (dT + dN);
        const double wT = interior ? dN * rs : 1.0;
        const double wN = interior ? dT * rs : 0.0;
        const int ia = sel3i(a, ic[0], ic[1], ic[2]), ib = sel3i(b, ic[0], ic[1], ic[2]);
        const int icc = sel3i(c, ic[0], ic[1], ic[2]);
        const int na = sel3i(a, M.ncell[0], M.ncell[1], M.ncell[2]), nbb = sel3i(b, M.ncell[0], M.ncell[1], M.ncell[2]);
        const double area = pickp<3>(M.farea, a)[(ia + e) + size_t(na + 1) * (ib + size_t(nbb) * icc)];
        const double gamma = M.sigma * dT * area * (interior ? 2.0 * dN * rs : 1.0) /
                             (interior ? fmin(M.cvol[cell], M.cvol[nb.cell]) : M.cvol[cell]);
        const double avg = wT * kxo * Kgo + wN * kxn * Kgn;
        const double Jmp = uo[i] - un[i];
        const double bout = geo_b(M, 0, Xp) * nu[0] + geo_b(M, 1, Xp) * nu[1] + geo_b(M, 2, Xp) * nu[2];
        const double Phi = bout >= 0.0 ? bout * uo[i] : bout * un[i];
        const double W = sw[qb] * sw[qc] * nrm;
        S0[i] = W * (Phi - avg + gamma * Jmp);
        // symmetry term against the reference gradient: t C^T (K nu)
        const double t = -W * wT * Jmp * kxo * ideto;
        const double Z0 = t * (Co[0] * Kn[0] + Co[3] * Kn[1] + Co[6] * Kn[2]);
        const double Z1 = t * (Co[1] * Kn[0] + Co[4] * Kn[1] + Co[7] * Kn[2]);
        const double Z2 = t * (Co[2] * Kn[0] + Co[5] * Kn[1] + Co[8] * Kn[2]);
        S1[i] = sel3d(b, Z0, Z1, Z2);
        S2[i] = sel3d(c, Z0, Z1, Z2);
        S3[i] = sel3d(a, Z0, Z1, Z2);
      }
    } else
    for (int i = lt; i < 6 * QF; i += TPC) {
      const int f = i / QF, ii = i - f * QF;
      const int a = f >> 1, e = f & 1;
      const int b = (a == 0) ? 1 : 0, c = (a == 2) ? 1 : 2;
      const int qb = ii % Q, qc = ii / Q;
      const int ia = sel3i(a, ic[0], ic[1], ic[2]), ib = sel3i(b, ic[0], ic[1], ic[2]), icc = sel3i(c, ic[0], ic[1], ic[2]);
      const FaceNb nb = face_nb(cell, ia, sel3i(a, M.ncell[0], M.ncell[1], M.ncell[2]),
                                sel3i(a, cstride[0], cstride[1], cstride[2]), (M.periodic >> a) & 1, e);
      const bool interior = nb.in;
      const double ha = sel3d(a, h[0], h[1], h[2]), hb = sel3d(b, h[0], h[1], h[2]), hc = sel3d(c, h[0], h[1], h[2]);
      const double sgn = e ? 1.0 : -1.0;
      const double hn = interior ? pickp<3>(M.h, a)[nb.ja] : ha;
      const double kn = interior ? (M.kappa ? M.kappa[nb.cell] : 1.0) : 0.0;
      const double Kaa = sel3d(a, M.K[0], M.K[4], M.K[8]);
      const double Kab = sel3d(a, M.K[1], M.K[3], M.K[6]), Kac = sel3d(a, M.K[2], M.K[5], M.K[7]);
      const double dT = kap * Kaa, dN = kn * Kaa;
      const double wT = interior ? dN / (dT + dN) : 1.0;
      const double wN = interior ? dT / (dT + dN) : 0.0;
      const double gamma = interior ? M.sigma * (2.0 * dT * dN / (dT + dN)) / fmin(ha, hn) : M.sigma * dT / ha;
      const double KgT = Kaa * gao[i] / ha + Kab * gbo[i] / hb + Kac * gco[i] / hc;
      const double KgN = Kaa * gan[i] / hn + Kab * gbn[i] / hb + Kac * gcn[i] / hc;
      const double avg = sgn * (wT * kap * KgT + wN * kn * KgN);
      const double J = uo[i] - un[i];
      const int fn = face_node(ia, e, nb.wrap);
      double ba;
      if (M.bprod) {
        ba = pickp<9>(M.bfn, 3 * a + a)[fn] * pickp<9>(M.bf, 3 * a + b)[ib * Q + qb] *
             pickp<9>(M.bf, 3 * a + c)[icc * Q + qc];
      } else {
        const int ax = sel3i(a, M.b_axis[0], M.b_axis[1], M.b_axis[2]);
        const double *bv = pickp<3>(M.bvol, a);
        ba = (ax == a) ? pickp<3>(M.bnode, a)[fn] : (ax == b) ? bv[ib * Q + qb] : bv[icc * Q + qc];
      }
      const double bout = sgn * ba;
      const double Phi = bout >= 0.0 ? bout * uo[i] : bout * un[i];
      const double W = sw[qb] * sw[qc] * hb * hc;
      const double kp = M.kpoly ? pickp<3>(M.kfn, a)[fn] * pickp<3>(M.kf, b)[ib * Q + qb] *
                                      pickp<3>(M.kf, c)[icc * Q + qc]
                                : 1.0;
      const double RV = W * (Phi - kp * avg + kp * gamma * J);
      const double RT = -W * wT * kap * kp * J * sgn;
      S0[i] = RV;
      S1[i] = RT * Kab / hb;
      S2[i] = RT * Kac / hc;
      S3[i] = RT * Kaa / ha;
    }
    __syncthreads();
    // transposed tangential contractions: along c, then b
    contract<N, true, 1, Q, N, 6, Q, TPC, BK>(lt, uo, S0, sV, S2, sD);
    contract<N, true, 1, Q, N, 6, Q, TPC, BK>(lt, un, S1, sV);
    contract<N, true, 1, Q, N, 6, Q, TPC, BK>(lt, gao, S3, sV);
    __syncthreads();
    contract<N, true, 0, N, N, 6, Q, TPC, BK>(lt, TUo, uo, sV, un, sD);  // R_v of every face
    contract<N, true, 0, N, N, 6, Q, TPC, BK>(lt, TDo, gao, sV);         // R_d
    __syncthreads();
    // normal direction last, all six faces into the own coefficients
    for (int i = lt; i < NB; i += TPC) {
      const int j0 = i % N, j1 = (i / N) % N, j2 = i / NF;
      double acc = 0.0;
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        const int a = f >> 1, e = f & 1;
        const int ja = sel3i(a, j0, j1, j2);
        const int i2 = (a == 0 ? j1 : j0) + N * (a == 2 ? j1 : j2);
        acc += sev[e][ja] * TUo[f * NF + i2] + sed[e][ja] * TDo[f * NF + i2];
      }
      Y[i] += acc;
    }
  } else {
  double *Uo = F[0], *Do = F[1], *Un = F[2], *Dn = F[3];
  double *S0 = F[4], *S1 = F[5], *S2 = F[6], *S3 = F[7];
  double *uo = F[8], *un = F[9], *gao = F[10], *gan = F[11];
  double *gbo = F[12], *gbn = F[13], *gco = F[14], *gcn = F[15];
  // raised rule: unrolled, so that the face's axes are compile-time and the
  // small per-cell arrays are not indexed per point from scratch (5-9 %
  // faster); the (k+1)-point variant keeps the loop (fewer registers)
  constexpr int FACE_UNROLL = (Q == N) ? 1 : 6;
#pragma unroll FACE_UNROLL
  for (int f = 0; f < 6; ++f) {
    const int a = f >> 1, e = f & 1;  // e = 1: upper face x_a = 1 (outer normal +e_a)
    const int b = (a == 0) ? 1 : 0, c = (a == 2) ? 1 : 2;
    const int st[3] = {1, N, NF};
    const int sa = st[a], sb = st[b], sc = st[c];
    const FaceNb nb = face_nb(cell, ic[a], M.ncell[a], cstride[a], (M.periodic >> a) & 1, e);
    const bool interior = nb.in;
    const int nbcell = nb.cell;
    const double *xN = x + size_t(nbcell) * NB;
    // normal direction first: modal traces on the 2D (jb, jc) grid
    for (int i = lt; i < NF; i += TPC) {
      const int jb = i % N, jc = i / N;
      const int base = jb * sb + jc * sc;
      double uo_ = 0, do_ = 0, un_ = 0, dn_ = 0;
      for (int ja = 0; ja < N; ++ja) {
        uo_ = fma(sev[e][ja], X[base + ja * sa], uo_);
        do_ = fma(sed[e][ja], X[base + ja * sa], do_);
      }
      if (interior)
        for (int ja = 0; ja < N; ++ja) {
          const double v = xN[base + ja * sa];
          un_ = fma(sev[1 - e][ja], v, un_);
          dn_ = fma(sed[1 - e][ja], v, dn_);
        }
      Uo[i] = uo_;
      Do[i] = do_;
      Un[i] = un_;
      Dn[i] = dn_;
    }
    __syncthreads();
    // tangential evaluation: first b (stride 1 in the 2D grid), then c
    contract<N, false, 0, Q, N, 1, N, TPC, BK>(lt, S0, Uo, sV);
    contract<N, false, 0, Q, N, 1, N, TPC, BK>(lt, S1, Uo, sD);
    contract<N, false, 0, Q, N, 1, N, TPC, BK>(lt, S2, Un, sV);
    contract<N, false, 0, Q, N, 1, N, TPC, BK>(lt, S3, Un, sD);
    __syncthreads();
    contract<N, false, 1, Q, Q, 1, N, TPC, BK>(lt, uo, S0, sV);
    contract<N, false, 1, Q, Q, 1, N, TPC, BK>(lt, gbo, S1, sV);
    contract<N, false, 1, Q, Q, 1, N, TPC, BK>(lt, gco, S0, sD);
    contract<N, false, 1, Q, Q, 1, N, TPC, BK>(lt, un, S2, sV);
    contract<N, false, 1, Q, Q, 1, N, TPC, BK>(lt, gbn, S3, sV);
    contract<N, false, 1, Q, Q, 1, N, TPC, BK>(lt, gcn, S2, sD);
    __syncthreads();
    contract<N, false, 0, Q, N, 1, N, TPC, BK>(lt, S0, Do, sV);
    contract<N, false, 0, Q, N, 1, N, TPC, BK>(lt, S1, Dn, sV);
    __syncthreads();
    contract<N, false, 1, Q, Q, 1, N, TPC, BK>(lt, gao, S0, sV);
    contract<N, false, 1, Q, Q, 1, N, TPC, BK>(lt, gan, S1, sV);
    __syncthreads();
    // pointwise face terms (Sec. 2.2): upwind flux, weighted average,
    // penalty, written with the outer normal n_T = sgn e_a of cell T
    {
      const double sgn = e ? 1.0 : -1.0;
      const double hn = interior ? (a == 0 ? M.h[0][nb.ja] : a == 1 ? M.h[1][nb.ja] : M.h[2][nb.ja]) : h[a];
      const double kn = interior ? (M.kappa ? M.kappa[nbcell] : 1.0) : 0.0;
      const double Kaa = M.K[4 * a];
      const double dT = kap * Kaa, dN = kn * Kaa;
      const double wT = interior ? dN / (dT + dN) : 1.0;
      const double wN = interior ? dT / (dT + dN) : 0.0;
      const double gamma = interior ? M.sigma * (2.0 * dT * dN / (dT + dN)) / fmin(h[a], hn)
                                    : M.sigma * dT / h[a];
      const double area = h[b] * h[c];
      const double Kab = M.K[3 * a + b], Kac = M.K[3 * a + c];
      for (int i = lt; i < QF; i += TPC) {
        const int qb = i % Q, qc = i / Q;
        // normal flux component (K grad u)_a of own / neighbour traces
        const double KgT = Kaa * gao[i] / h[a] + Kab * gbo[i] / h[b] + Kac * gco[i] / h[c];
        const double KgN = Kaa * gan[i] / hn + Kab * gbn[i] / h[b] + Kac * gcn[i] / h[c];
        const double avg = sgn * (wT * kap * KgT + wN * kn * KgN);  // {D grad u}_w . n_T
        const double J = uo[i] - un[i];
        // b_a at the face point: b_a depends on the coordinate b_axis[a]
        const int ax = M.b_axis[a];
        double ba;
        if (M.bprod)
          ba = M.bfn[3 * a + a][face_node(ic[a], e, nb.wrap)] * M.bf[3 * a + b][ic[b] * Q + qb] *
               M.bf[3 * a + c][ic[c] * Q + qc];
        else if (ax == a)
          ba = M.bnode[a][face_node(ic[a], e, nb.wrap)];
        else if (ax == b)
          ba = M.bvol[a][ic[b] * Q + qb];
        else
          ba = M.bvol[a][ic[c] * Q + qc];
        const double bout = sgn * ba;
        const double Phi = bout >= 0.0 ? bout * uo[i] : bout * un[i];
        const double W = sw[qb] * sw[qc] * area;
        // pointwise diffusion factor: scales the average, penalty and symmetry terms
        const double kp = M.kpoly ? M.kfn[a][face_node(ic[a], e, nb.wrap)] * M.kf[b][ic[b] * Q + qb] *
                                        M.kf[c][ic[c] * Q + qc]
                                  : 1.0;
        const double RV = W * (Phi - kp * avg + kp * gamma * J);
        const double RT = -W * wT * kap * kp * J * sgn;  // times (K grad phi)_a
        S0[i] = RV;
        S1[i] = RT * Kab / h[b];
        S2[i] = RT * Kac / h[c];
        S3[i] = RT * Kaa / h[a];
      }
    }
    __syncthreads();
    // transposed tangential contractions: along c, then b
    contract<N, true, 1, Q, N, 1, Q, TPC, BK>(lt, uo, S0, sV, S2, sD);  // value x V_c + (d_c part) x D_c
    contract<N, true, 1, Q, N, 1, Q, TPC, BK>(lt, un, S1, sV);          // d_b part
    contract<N, true, 1, Q, N, 1, Q, TPC, BK>(lt, gao, S3, sV);         // d_a part
    __syncthreads();
    contract<N, true, 0, N, N, 1, Q, TPC, BK>(lt, Uo, uo, sV, un, sD);  // R_v
    contract<N, true, 0, N, N, 1, Q, TPC, BK>(lt, Do, gao, sV);         // R_d
    __syncthreads();
    // normal direction last: y(ja,jb,jc) += theta_ja(e) R_v + theta'_ja(e) R_d
    for (int i = lt; i < NB; i += TPC) {
      const int j[3] = {i % N, (i / N) % N, i / NF};
      const int i2 = j[b] + N * j[c];
      Y[i] += sev[e][j[a]] * Uo[i2] + sed[e][j[a]] * Do[i2];
    }
    __syncthreads();
  }
  }
  if (active) {
    double *yT = y + size_t(cell) * NB;
    for (int i = lt; i < NB; i += TPC) yT[i] = Y[i];
  }
}

template <int N, int Q, bool GEO = false, bool VOL = true>
static hipError_t launch_ref_n(const dg_handle *h, const double *x, double *y, hipStream_t s) {
  if (h->tabq.m != Q) return hipErrorInvalidValue;
  RefTab<N, Q> T;
  for (int q = 0; q < Q; ++q) {
    for (int j = 0; j < N; ++j) {
      T.V[q][j] = h->tabq.V[q][j];
      T.D[q][j] = h->tabq.D[q][j];
    }
    T.w[q] = h->tabq.w[q];
    T.xi[q] = h->tabq.xi[q];
  }
  for (int j = 0; j < N; ++j) {
    T.ev[0][j] = h->tabq.e0v[j];
    T.ev[1][j] = h->tabq.e1v[j];
    T.ed[0][j] = h->tabq.e0d[j];
    T.ed[1][j] = h->tabq.e1d[j];
  }
  RefMesh M = make_ref_mesh(h, GEO);
  // raised rule and multilinear cells: as many cells per workgroup as keep
  // its LDS near 80 KB
  constexpr bool BATCH = (Q != N) || GEO;
  constexpr int NF_ = N * N, QF_ = Q * Q, QB_ = Q * Q * Q;
  constexpr int region = (BATCH && 24 * NF_ + 72 * QF_ > 7 * QB_) ? 24 * NF_ + 72 * QF_ : 7 * QB_;
  constexpr int per_cell = 8 * (2 * N * N * N + region + (BATCH ? 16 : 16 * QF_) + (GEO ? 3 * kVB * kVB * kVB : 1));
  constexpr int CPB = !BATCH ? 1 : (8 * per_cell <= 81920 ? 8 : 4 * per_cell <= 81920 ? 4 : 2 * per_cell <= 81920 ? 2 : 1);
  constexpr int TPB = (CPB == 1 && per_cell > 81920) ? 2 * kRefThreads : kRefThreads;
  const unsigned grid = unsigned((h->ncells + CPB - 1) / CPB);
  hipLaunchKernelGGL((apply_ref_kernel<N, Q, CPB, GEO, VOL, TPB>), dim3(grid), dim3(TPB), 0, s, x, y, M, T);
  return hipGetLastError();
}

// Multilinear meshes: the (k+1)-point rule, the raised rule (k+3 points) or
// the rule q = 3p + 4 of Problem C (ceil((3k+5)/2) points), k <= 7.  The
// volume runs on the pencil-layout kernel of geo_volume.hip (writing y) and
// this kernel adds the faces (VOL = false); where that kernel does not take
// the rule, this kernel does both.
template <int N, int Q>
static hipError_t launch_geo_rule(const dg_handle *h, const double *x, double *y, hipStream_t s) {
  if (geo_volume_supported(h)) {
    const hipError_t e = launch_geo_volume_f64(h, x, y, s);
    if (e != hipSuccess) return e;
    return launch_ref_n<N, Q, true, false>(h, x, y, s);
  }
  return launch_ref_n<N, Q, true>(h, x, y, s);
}

template <int N>
static hipError_t launch_geo_q(const dg_handle *h, const double *x, double *y, hipStream_t s) {
  constexpr int QC = (3 * (N - 1) + 6) / 2;
  if (h->tabq.m == N) return launch_geo_rule<N, N>(h, x, y, s);
  if (h->tabq.m == N + 2) return launch_geo_rule<N, N + 2>(h, x, y, s);
  if constexpr (QC != N + 2) {
    if (h->tabq.m == QC) return launch_geo_rule<N, QC>(h, x, y, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_apply_geo_f64(const dg_handle *h, const double *x, double *y, hipStream_t s) {
  switch (h->k + 1) {
    case 2: return launch_geo_q<2>(h, x, y, s);
    case 3: return launch_geo_q<3>(h, x, y, s);
    case 4: return launch_geo_q<4>(h, x, y, s);
    case 5: return launch_geo_q<5>(h, x, y, s);
    case 6: return launch_geo_q<6>(h, x, y, s);
    case 7: return launch_geo_q<7>(h, x, y, s);
    case 8: return launch_geo_q<8>(h, x, y, s);
    default: return hipErrorInvalidValue;
  }
}

// Q = N: the (k+1)-point rule; Q = N + 2: the raised rule (k <= 8).
template <int N>
static hipError_t launch_ref_q(const dg_handle *h, const double *x, double *y, hipStream_t s) {
  if (h->quad_extra == 0) return launch_ref_n<N, N>(h, x, y, s);
  if constexpr (N + 2 <= kMaxN) {
    if (h->quad_extra == 2) return launch_ref_n<N, N + 2>(h, x, y, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_apply_ref_f64(const dg_handle *h, const double *x, double *y, hipStream_t s) {
  switch (h->k + 1) {
    case 2: return launch_ref_q<2>(h, x, y, s);
    case 3: return launch_ref_q<3>(h, x, y, s);
    case 4: return launch_ref_q<4>(h, x, y, s);
    case 5: return launch_ref_q<5>(h, x, y, s);
    case 6: return launch_ref_q<6>(h, x, y, s);
    case 7: return launch_ref_q<7>(h, x, y, s);
    case 8: return launch_ref_q<8>(h, x, y, s);
    case 9: return launch_ref_q<9>(h, x, y, s);
    case 10: return launch_ref_q<10>(h, x, y, s);
    case 11: return launch_ref_q<11>(h, x, y, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dgmf
