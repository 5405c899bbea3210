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
#include "dg_internal.h"
#include "mesh_nb.h"

namespace dgmf {

template <int N, int Q>
struct RefTab {
  double V[Q][N], D[Q][N], w[Q], ev[2][N], ed[2][N];
};

struct RefMesh {
  int ncell[3];
  int periodic;  // bit a: axis a is periodic
  const double *h[3], *bvol[3], *bnode[3], *kappa;
  const double *bf[9], *bfn[9];  // product-form factors (bprod)
  const double *kf[3], *kfn[3];  // polynomial diffusion factor (kpoly)
  double K[9], c, sigma;
  int b_axis[3];
  int bprod, kpoly;
  int ncells;
};

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
template <int LD, bool TRANS, int AX, int O0, int O1, int O2, int LI, int TPC>
__device__ inline void contract(int lt, double *out, const double *in, const double (*Mat)[LD],
                                const double *in2 = nullptr, const double (*Mat2)[LD] = nullptr) {
  constexpr int I0 = AX == 0 ? LI : O0, I1 = AX == 1 ? LI : O1;
  constexpr int IS[3] = {1, I0, I0 * I1};  // input strides
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
}

// CPB cells per workgroup, kRefThreads / CPB threads and one LDS slice each
// (CPB = 1 for the (k+1)-point reference variant).
template <int N, int Q, int CPB>
__global__ __launch_bounds__(kRefThreads) void apply_ref_kernel(const double *__restrict__ x,
                                                                double *__restrict__ y,
                                                                RefMesh M, RefTab<N, Q> T) {
  constexpr int NB = N * N * N, NF = N * N, QB = Q * Q * Q, QF = Q * Q;
  constexpr int TPC = kRefThreads / CPB;
  __shared__ double sV[Q][N], sD[Q][N], sw[Q], sev[2][N], sed[2][N];
  __shared__ double Xs[CPB][NB], Ys[CPB][NB], Bs[CPB][7][QB];
  __shared__ double Fs[CPB][16][QF];
  const int tid = threadIdx.x;
  const int slot = tid / TPC, lt = tid % TPC;
  double *X = Xs[slot], *Y = Ys[slot];
  double *B0 = Bs[slot][0], *B1 = Bs[slot][1], *B2 = Bs[slot][2], *B3 = Bs[slot][3];
  double *B4 = Bs[slot][4], *B5 = Bs[slot][5], *B6 = Bs[slot][6];
  double(*F)[QF] = Fs[slot];
  // a slot past the last cell repeats it (every thread reaches every barrier)
  // and does not store
  const bool active = int(blockIdx.x) * CPB + slot < M.ncells;
  const int cell = active ? int(blockIdx.x) * CPB + slot : M.ncells - 1;
  const int N1 = M.ncell[0], N2 = M.ncell[1];
  const int ic[3] = {cell % N1, (cell / N1) % N2, cell / (N1 * N2)};
  const int cstride[3] = {1, N1, N1 * N2};

  for (int i = tid; i < Q * N; i += kRefThreads) {
    sV[i / N][i % N] = T.V[i / N][i % N];
    sD[i / N][i % N] = T.D[i / N][i % N];
  }
  if (tid < Q) sw[tid] = T.w[tid];
  if (tid < N) {
    sev[0][tid] = T.ev[0][tid];
    sev[1][tid] = T.ev[1][tid];
    sed[0][tid] = T.ed[0][tid];
    sed[1][tid] = T.ed[1][tid];
  }
  const double *xT = x + size_t(cell) * NB;
  for (int i = lt; i < NB; i += TPC) X[i] = xT[i];
  __syncthreads();

  const double h[3] = {M.h[0][ic[0]], M.h[1][ic[1]], M.h[2][ic[2]]};
  const double kap = M.kappa ? M.kappa[cell] : 1.0;
  const double vol = h[0] * h[1] * h[2];

  // ---------------- volume: forward (u, d1 u, d2 u, d3 u at points) --------
  contract<N, false, 0, Q, N, N, N, TPC>(lt, B0, X, sV);  // V1 x
  contract<N, false, 0, Q, N, N, N, TPC>(lt, B1, X, sD);  // D1 x
  __syncthreads();
  contract<N, false, 1, Q, Q, N, N, TPC>(lt, B2, B0, sV);  // V2 V1 x
  contract<N, false, 1, Q, Q, N, N, TPC>(lt, B3, B1, sV);  // V2 D1 x
  contract<N, false, 1, Q, Q, N, N, TPC>(lt, B4, B0, sD);  // D2 V1 x
  __syncthreads();
  contract<N, false, 2, Q, Q, Q, N, TPC>(lt, B0, B2, sV);  // u
  contract<N, false, 2, Q, Q, Q, N, TPC>(lt, B1, B3, sV);  // d^1 u (reference)
  contract<N, false, 2, Q, Q, Q, N, TPC>(lt, B5, B4, sV);  // d^2 u
  contract<N, false, 2, Q, Q, Q, N, TPC>(lt, B6, B2, sD);  // d^3 u
  __syncthreads();
  // ---------------- volume: pointwise flux (eq. (gauss_points)) ------------
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
  contract<N, true, 2, Q, Q, N, Q, TPC>(lt, B2, B0, sV, B6, sD);  // along 3: V^T x0 + D^T x3
  contract<N, true, 2, Q, Q, N, Q, TPC>(lt, B3, B1, sV);          // V^T x1
  contract<N, true, 2, Q, Q, N, Q, TPC>(lt, B4, B5, sV);          // V^T x2
  __syncthreads();
  contract<N, true, 1, Q, N, N, Q, TPC>(lt, B0, B2, sV, B4, sD);  // along 2
  contract<N, true, 1, Q, N, N, Q, TPC>(lt, B1, B3, sV);
  __syncthreads();
  contract<N, true, 0, N, N, N, Q, TPC>(lt, Y, B0, sV, B1, sD);  // along 1
  __syncthreads();

  // ---------------- faces --------------------------------------------------
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
    contract<N, false, 0, Q, N, 1, N, TPC>(lt, S0, Uo, sV);
    contract<N, false, 0, Q, N, 1, N, TPC>(lt, S1, Uo, sD);
    contract<N, false, 0, Q, N, 1, N, TPC>(lt, S2, Un, sV);
    contract<N, false, 0, Q, N, 1, N, TPC>(lt, S3, Un, sD);
    __syncthreads();
    contract<N, false, 1, Q, Q, 1, N, TPC>(lt, uo, S0, sV);
    contract<N, false, 1, Q, Q, 1, N, TPC>(lt, gbo, S1, sV);
    contract<N, false, 1, Q, Q, 1, N, TPC>(lt, gco, S0, sD);
    contract<N, false, 1, Q, Q, 1, N, TPC>(lt, un, S2, sV);
    contract<N, false, 1, Q, Q, 1, N, TPC>(lt, gbn, S3, sV);
    contract<N, false, 1, Q, Q, 1, N, TPC>(lt, gcn, S2, sD);
    __syncthreads();
    contract<N, false, 0, Q, N, 1, N, TPC>(lt, S0, Do, sV);
    contract<N, false, 0, Q, N, 1, N, TPC>(lt, S1, Dn, sV);
    __syncthreads();
    contract<N, false, 1, Q, Q, 1, N, TPC>(lt, gao, S0, sV);
    contract<N, false, 1, Q, Q, 1, N, TPC>(lt, gan, S1, sV);
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
    contract<N, true, 1, Q, N, 1, Q, TPC>(lt, uo, S0, sV, S2, sD);  // value x V_c + (d_c part) x D_c
    contract<N, true, 1, Q, N, 1, Q, TPC>(lt, un, S1, sV);          // d_b part
    contract<N, true, 1, Q, N, 1, Q, TPC>(lt, gao, S3, sV);         // d_a part
    __syncthreads();
    contract<N, true, 0, N, N, 1, Q, TPC>(lt, Uo, uo, sV, un, sD);  // R_v
    contract<N, true, 0, N, N, 1, Q, TPC>(lt, Do, gao, sV);         // R_d
    __syncthreads();
    // normal direction last: y(ja,jb,jc) += theta_ja(e) R_v + theta'_ja(e) R_d
    for (int i = lt; i < NB; i += TPC) {
      const int j[3] = {i % N, (i / N) % N, i / NF};
      const int i2 = j[b] + N * j[c];
      Y[i] += sev[e][j[a]] * Uo[i2] + sed[e][j[a]] * Do[i2];
    }
    __syncthreads();
  }
  if (active) {
    double *yT = y + size_t(cell) * NB;
    for (int i = lt; i < NB; i += TPC) yT[i] = Y[i];
  }
}

template <int N, int Q>
static hipError_t launch_ref_n(const dg_handle *h, const double *x, double *y, hipStream_t s) {
  if (h->tabq.m != Q) return hipErrorInvalidValue;
  RefTab<N, Q> T;
  for (int q = 0; q < Q; ++q) {
    for (int j = 0; j < N; ++j) {
      T.V[q][j] = h->tabq.V[q][j];
      T.D[q][j] = h->tabq.D[q][j];
    }
    T.w[q] = h->tabq.w[q];
  }
  for (int j = 0; j < N; ++j) {
    T.ev[0][j] = h->tabq.e0v[j];
    T.ev[1][j] = h->tabq.e1v[j];
    T.ed[0][j] = h->tabq.e0d[j];
    T.ed[1][j] = h->tabq.e1d[j];
  }
  RefMesh M;
  for (int a = 0; a < 3; ++a) {
    M.ncell[a] = h->mesh.ncell[a];
    M.h[a] = h->mesh.h[a];
    M.bvol[a] = h->mesh.bvol[a];
    M.bnode[a] = h->mesh.bnode[a];
    M.b_axis[a] = h->mesh.b_axis[a];
  }
  for (int t = 0; t < 9; ++t) {
    M.bf[t] = h->mesh.bf[t];
    M.bfn[t] = h->mesh.bfn[t];
  }
  M.bprod = h->mesh.bprod;
  M.kpoly = h->mesh.kpoly;
  for (int j = 0; j < 3; ++j) {
    M.kf[j] = h->mesh.kf[j];
    M.kfn[j] = h->mesh.kfn[j];
  }
  M.kappa = h->mesh.kappa;
  M.periodic = h->mesh.periodic;
  for (int i = 0; i < 9; ++i) M.K[i] = h->mesh.K[i];
  M.c = h->mesh.c;
  M.sigma = h->mesh.sigma;
  M.ncells = int(h->ncells);
  // raised rule: as many cells per workgroup as keep its LDS near 80 KB
  constexpr int per_cell = 8 * (2 * N * N * N + 7 * Q * Q * Q + 16 * Q * Q);
  constexpr int CPB = (Q == N) ? 1 : (8 * per_cell <= 81920 ? 8 : 4 * per_cell <= 81920 ? 4 : 2 * per_cell <= 81920 ? 2 : 1);
  const unsigned grid = unsigned((h->ncells + CPB - 1) / CPB);
  hipLaunchKernelGGL((apply_ref_kernel<N, Q, CPB>), dim3(grid), dim3(kRefThreads), 0, s, x, y, M, T);
  return hipGetLastError();
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
