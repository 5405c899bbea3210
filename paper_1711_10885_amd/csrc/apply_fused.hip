// Fused FP64 apply kernel for gfx950: volume and all six faces of each cell in
// one pass, owner-computes (each cell writes only its own rows, no atomics).
//
// Mapping.  A cell is handled by N^2 lanes ("pencil slots"); lane p = a + N b
// owns one 1D pencil of N values at a time and contracts it against the 1D
// matrices of Sec. 3.2 (eq. (gradient_matrices)) held in scalar registers
// (kernel-argument tables, compile-time indices), which is the sum
// factorization kernel of eq. (sum_fact_kernel) with the tensor rotation
// fused into the LDS exchange between directions.  Tensors pass through LDS
// only to change the pencil direction; each exchange uses pencils padded to
// N+1 doubles.
//
// Volume (Algorithm 1, steps 1-3), evaluation tree with a shared first sweep:
//   A  (axis 1, lanes (j2,j3)):  x -> V1 x, D1 x
//   B  (axis 2, lanes (q1,j3)):  -> V2V1x, V2D1x, D2V1x
//   C  (axis 3, lanes (q1,q2)):  -> u, d1u, d2u, d3u at the Gauss points
//   pointwise flux x^(r) of eq. (gauss_points), then the transposed sweeps
//   C' (axis 3), B' (axis 2), A' (axis 1) of eq. (evalblf).
//
// Faces (steps 4-6 / 8-10): the normal direction is contracted first on both
// sides (Sec. 3.4/3.5: traces of u and of d_a u), then the two tangential
// directions; pointwise flux; transposed tangential sweeps; normal direction
// last.  Own-side work is merged into the volume tensors where the normal
// axis is still modal there:
//   z faces: own traces come from the C-stage input pencils, own integration
//            is added to the C'-stage output pencils;
//   y faces: own traces come from the B-stage input pencils (already
//            evaluated along axis 1), own integration is added to the B'-stage
//            output (the A' sweep then does the axis-1 integration);
//   x faces: own traces from the x pencils, integration added to the A'
//            output.
// Neighbour traces are contracted in the normal direction straight from
// global memory (the pencil along the face normal is loaded by one lane).
#include "dg_internal.h"

namespace dgmf {

template <int N>
struct FTab {
  double V[N][N], D[N][N];  // V[q][j] = theta_j(xi_q), D[q][j] = theta_j'(xi_q)
  double ev[2][N], ed[2][N];  // theta_j(e), theta_j'(e) for e = 0, 1
};

struct FMesh {
  int ncell[3];
  const double *h[3], *bvol[3], *bnode[3], *kappa, *w;
  double K[9], c, sigma;
  int b_axis[3];
  int tz;          // depth (cells along axis 3) of the tiles of the cell order
  int ncells;
  int groups;      // workgroups per XCD slot (grid = 8 * groups)
};

template <int N>
struct FCfg {
  static constexpr int NN = N * N;
  static constexpr int PS = N + 1;  // padded pencil stride
  static constexpr int LANES = NN;
  static constexpr int CPB = (NN <= 64) ? (64 / NN) : 1;
  static constexpr int THREADS = ((CPB * LANES + 63) / 64) * 64;
  // per-cell LDS (doubles) of each exchange round
  static constexpr int R1 = 2 * NN * PS + 16 * N * PS;
  static constexpr int R2A = 3 * NN * PS + 6 * N * PS;
  static constexpr int R2B = 8 * NN + 24 * N * PS;
  static constexpr int R3 = 3 * NN * PS + 6 * NN + 6 * N * PS;
  static constexpr int R4 = 2 * NN * PS + 4 * NN;
  static constexpr int mx(int a, int b) { return a > b ? a : b; }
  static constexpr int REGION = mx(mx(mx(R1, R2A), mx(R2B, R3)), R4);
};

// out[q] = sum_t M[q][t] in[t]
template <int N>
__device__ __forceinline__ void mv(const double (&M)[N][N], const double *in, double *out) {
#pragma unroll
  for (int q = 0; q < N; ++q) {
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < N; ++t) s = fma(M[q][t], in[t], s);
    out[q] = s;
  }
}

// out[j] (+)= sum_q M[q][j] in[q]
template <int N, bool ACC>
__device__ __forceinline__ void mtv(const double (&M)[N][N], const double *in, double *out) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double s = ACC ? out[j] : 0.0;
#pragma unroll
    for (int q = 0; q < N; ++q) s = fma(M[q][j], in[q], s);
    out[j] = s;
  }
}

template <int N>
__device__ __forceinline__ double dotv(const double (&v)[N], const double *in) {
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < N; ++t) s = fma(v[t], in[t], s);
  return s;
}

// Per-cell geometry and coefficients used by the face terms.
struct FaceGeo {
  double h[3];
  double kap;
  int ic[3];
};

// Pointwise face terms of eq. (blf) seen from cell T with outer normal
// n_T = sgn e_a: upwind flux, weighted average of the normal diffusive flux,
// symmetry term and penalty.  Inputs are the reference-coordinate values
// (u, d_b u, d_c u, d_a u) of the own (o) and neighbour (n) traces at one
// face point; outputs the four test-function coefficients:
//   RV (times phi), Pb (times theta'_jb), Pc (times theta'_jc),
//   Pa (times theta'_ja(e)) -- all in reference scaling.
struct FaceCoef {
  double sgn, wT, wN, kT, kN, gamma, inv_ha, inv_hn, inv_hb, inv_hc, area, Kaa, Kab, Kac;
};

__device__ __forceinline__ void face_point(const FaceCoef &F, double uo, double gbo, double gco,
                                           double gao, double un, double gbn, double gcn,
                                           double gan, double ba, double W, double &RV,
                                           double &Pb, double &Pc, double &Pa) {
  const double KgT = F.Kaa * gao * F.inv_ha + F.Kab * gbo * F.inv_hb + F.Kac * gco * F.inv_hc;
  const double KgN = F.Kaa * gan * F.inv_hn + F.Kab * gbn * F.inv_hb + F.Kac * gcn * F.inv_hc;
  const double avg = F.sgn * (F.wT * F.kT * KgT + F.wN * F.kN * KgN);
  const double J = uo - un;
  const double bout = F.sgn * ba;
  const double Phi = bout >= 0.0 ? bout * uo : bout * un;
  RV = W * (Phi - avg + F.gamma * J);
  const double RT = -W * F.wT * F.kT * J * F.sgn;
  Pb = RT * F.Kab * F.inv_hb;
  Pc = RT * F.Kac * F.inv_hc;
  Pa = RT * F.Kaa * F.inv_ha;
}

__device__ __forceinline__ FaceCoef make_face(const FMesh &M, const FaceGeo &G, int a, int e,
                                              bool interior, double hn, double kn) {
  const int b = (a == 0) ? 1 : 0, c = (a == 2) ? 1 : 2;
  FaceCoef F;
  F.sgn = e ? 1.0 : -1.0;
  const double Kaa = M.K[4 * a];
  const double dT = G.kap * Kaa, dN = kn * Kaa;
  F.kT = G.kap;
  F.kN = interior ? kn : 0.0;
  F.wT = interior ? dN / (dT + dN) : 1.0;
  F.wN = interior ? dT / (dT + dN) : 0.0;
  F.gamma = interior ? M.sigma * (2.0 * dT * dN / (dT + dN)) / fmin(G.h[a], hn)
                     : M.sigma * dT / G.h[a];
  F.inv_ha = 1.0 / G.h[a];
  F.inv_hn = interior ? 1.0 / hn : 0.0;
  F.inv_hb = 1.0 / G.h[b];
  F.inv_hc = 1.0 / G.h[c];
  F.area = G.h[b] * G.h[c];
  F.Kaa = Kaa;
  F.Kab = M.K[3 * a + b];
  F.Kac = M.K[3 * a + c];
  return F;
}

// b_a at a point of the face normal to a (side e) with tangential Gauss
// indices qb, qc.
__device__ __forceinline__ double face_b(const FMesh &M, const FaceGeo &G, int N, int a, int e,
                                         int qb, int qc) {
  const int b = (a == 0) ? 1 : 0, c = (a == 2) ? 1 : 2;
  const int ax = M.b_axis[a];
  if (ax == a) return M.bnode[a][G.ic[a] + e];
  if (ax == b) return M.bvol[a][G.ic[b] * N + qb];
  return M.bvol[a][G.ic[c] * N + qc];
}

__device__ __forceinline__ int cell_of_logical(int L, const FMesh &M) {
  const int N1 = M.ncell[0], N2 = M.ncell[1], N3 = M.ncell[2];
  const int plane = N1 * N2;
  const int t = L / (plane * M.tz);
  const int r = L - t * plane * M.tz;
  const int z0 = t * M.tz;
  const int tzt = min(M.tz, N3 - z0);
  const int i3 = z0 + r % tzt;
  const int rr = r / tzt;
  const int i1 = rr % N1, i2 = rr / N1;
  return i1 + N1 * (i2 + N2 * i3);
}

template <int N>
__global__ __launch_bounds__(FCfg<N>::THREADS) void apply_fused_kernel(
    const double *__restrict__ x, double *__restrict__ y, FMesh M, FTab<N> T) {
  using C = FCfg<N>;
  constexpr int NN = C::NN, PS = C::PS, NNN = N * N * N;
  __shared__ double lds[C::CPB * C::REGION];

  const int tid = threadIdx.x;
  const int cl = tid / C::LANES;
  const int p = tid - cl * C::LANES;
  const int alpha = p % N, beta = p / N;
  const bool slot = cl < C::CPB;  // thread belongs to a cell slot
  const int wg = blockIdx.x;
  const int lblock = (wg & 7) * M.groups + (wg >> 3);
  const int L = lblock * C::CPB + (slot ? cl : 0);
  const bool active = slot && L < M.ncells;
  const int cell = active ? cell_of_logical(L, M) : 0;
  double *R = lds + (slot ? cl : 0) * C::REGION;

  FaceGeo G;
  G.ic[0] = cell % M.ncell[0];
  G.ic[1] = (cell / M.ncell[0]) % M.ncell[1];
  G.ic[2] = cell / (M.ncell[0] * M.ncell[1]);
  G.h[0] = M.h[0][G.ic[0]];
  G.h[1] = M.h[1][G.ic[1]];
  G.h[2] = M.h[2][G.ic[2]];
  G.kap = M.kappa ? M.kappa[cell] : 1.0;
  const int cstride[3] = {1, M.ncell[0], M.ncell[0] * M.ncell[1]};

  // neighbour data of the six faces f = 2a + e
  bool fin[6];
  double fh[6], fk[6];
  int fcell[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int a = f >> 1, e = f & 1;
    fin[f] = e ? (G.ic[a] + 1 < M.ncell[a]) : (G.ic[a] > 0);
    fcell[f] = fin[f] ? cell + (e ? cstride[a] : -cstride[a]) : cell;
    fh[f] = fin[f] ? M.h[a][G.ic[a] + (e ? 1 : -1)] : G.h[a];
    fk[f] = fin[f] ? (M.kappa ? M.kappa[fcell[f]] : 1.0) : 0.0;
  }

  // ------------------------------------------------------------------------
  // P0: global loads.  Lane (j2,j3) = (alpha,beta) owns the x pencil along 1.
  // ------------------------------------------------------------------------
  double X[N];
  {
    const double *xp = x + size_t(cell) * NNN + NN * beta + N * alpha;
#pragma unroll
    for (int t = 0; t < N; ++t) X[t] = xp[t];
  }
  // own x-face traces (e = 0, 1): value and normal derivative
  double uxo[2], dxo[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    uxo[e] = dotv<N>(T.ev[e], X);
    dxo[e] = dotv<N>(T.ed[e], X);
  }
  // neighbour traces, normal direction contracted from global memory
  double unb[6], dnb[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int a = f >> 1, e = f & 1;
    double v[N];
    if (fin[f]) {
      const double *xn = x + size_t(fcell[f]) * NNN;
      // pencil along the normal axis a; lane (alpha, beta) indexes the two
      // tangential axes in increasing order
      const int base = (a == 0) ? (N * alpha + NN * beta)
                       : (a == 1) ? (alpha + NN * beta) : (alpha + N * beta);
      const int st = (a == 0) ? 1 : (a == 1) ? N : NN;
#pragma unroll
      for (int t = 0; t < N; ++t) v[t] = xn[base + st * t];
    } else {
#pragma unroll
      for (int t = 0; t < N; ++t) v[t] = 0.0;
    }
    unb[f] = dotv<N>(T.ev[1 - e], v);
    dnb[f] = dotv<N>(T.ed[1 - e], v);
  }
  // volume step A
  double Tv[N], Td[N];
  mv<N>(T.V, X, Tv);
  mv<N>(T.D, X, Td);

  // ------------------------------------------------------------------------
  // R1: volume A->B exchange and first tangential sweep of the face traces.
  // Face field fid (16 of them) is stored as N pencils of the first
  // tangential axis; lane (alpha, beta) writes element alpha of pencil beta:
  //   x faces (a=0): grid (j2,j3), fid = 4e + 2s + {0:U,1:Dn}, s = 0 own, 1 nb
  //   y nb    (a=1): grid (j1,j3), fid = 8 + 2e + {U,Dn}
  //   z nb    (a=2): grid (j1,j2), fid = 12 + 2e + {U,Dn}
  // ------------------------------------------------------------------------
  constexpr int B_OFF = 0;                 // Tv, Td B-pencils (q1 + N j3) along j2
  constexpr int F1_OFF = 2 * NN * PS;
  if (slot) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
      R[B_OFF + (q + N * beta) * PS + alpha] = Tv[q];
      R[B_OFF + NN * PS + (q + N * beta) * PS + alpha] = Td[q];
    }
    const int w1 = beta * PS + alpha;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      R[F1_OFF + (4 * e + 0) * N * PS + w1] = uxo[e];
      R[F1_OFF + (4 * e + 1) * N * PS + w1] = dxo[e];
      R[F1_OFF + (4 * e + 2) * N * PS + w1] = unb[e];
      R[F1_OFF + (4 * e + 3) * N * PS + w1] = dnb[e];
      R[F1_OFF + (8 + 2 * e) * N * PS + w1] = unb[2 + e];
      R[F1_OFF + (9 + 2 * e) * N * PS + w1] = dnb[2 + e];
      R[F1_OFF + (12 + 2 * e) * N * PS + w1] = unb[4 + e];
      R[F1_OFF + (13 + 2 * e) * N * PS + w1] = dnb[4 + e];
    }
  }
  __syncthreads();
  // volume step B: lane (q1, j3) = (alpha, beta)
  double vv[N], dv[N], vd[N];
  double uyo[2], gyo[2], dyo[2];  // own y traces on (q1, j3)
  {
    double P[N], Q[N];
#pragma unroll
    for (int t = 0; t < N; ++t) {
      P[t] = R[B_OFF + p * PS + t];
      Q[t] = R[B_OFF + NN * PS + p * PS + t];
    }
    mv<N>(T.V, P, vv);
    mv<N>(T.V, Q, dv);
    mv<N>(T.D, P, vd);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      uyo[e] = dotv<N>(T.ev[e], P);
      gyo[e] = dotv<N>(T.ev[e], Q);
      dyo[e] = dotv<N>(T.ed[e], P);
    }
  }
  // face tasks of the first tangential sweep: 8 face-sides x N pencils.
  // face-side fs: 0..3 x faces (e = fs>>1, s = fs&1), 4..5 y nb (e), 6..7 z nb (e)
  constexpr int NT1 = 8 * N;
  constexpr int NR1 = (NT1 + C::LANES - 1) / C::LANES;
  double S1[NR1][3][N];
#pragma unroll
  for (int r = 0; r < NR1; ++r) {
    const int task = p + r * C::LANES;
    if (task < NT1) {
      const int fs = task / N, pi = task % N;
      const int fidU = (fs < 4) ? (2 * fs) : (fs < 6 ? 8 + 2 * (fs - 4) : 12 + 2 * (fs - 6));
      double U[N], Dn[N];
#pragma unroll
      for (int t = 0; t < N; ++t) {
        U[t] = R[F1_OFF + fidU * N * PS + pi * PS + t];
        Dn[t] = R[F1_OFF + (fidU + 1) * N * PS + pi * PS + t];
      }
      mv<N>(T.V, U, S1[r][0]);
      mv<N>(T.D, U, S1[r][1]);
      mv<N>(T.V, Dn, S1[r][2]);
    }
  }
  __syncthreads();

  // ------------------------------------------------------------------------
  // R2a: volume B->C exchange and z-neighbour second tangential sweep input.
  // ------------------------------------------------------------------------
  constexpr int C_OFF = 0;                    // vv, dv, vd C-pencils (q1 + N q2) along j3
  constexpr int Z2_OFF = 3 * NN * PS;         // z nb (e, {Sv,Sd,Sn}) pencils along j2, index q1
  if (slot) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
      R[C_OFF + (alpha + N * q) * PS + beta] = vv[q];
      R[C_OFF + NN * PS + (alpha + N * q) * PS + beta] = dv[q];
      R[C_OFF + 2 * NN * PS + (alpha + N * q) * PS + beta] = vd[q];
    }
#pragma unroll
    for (int r = 0; r < NR1; ++r) {
      const int task = p + r * C::LANES;
      if (task < NT1) {
        const int fs = task / N, pi = task % N;  // pi = j2 (second tangential)
        if (fs >= 6) {
          const int e = fs - 6;
#pragma unroll
          for (int g = 0; g < 3; ++g)
#pragma unroll
            for (int q = 0; q < N; ++q) R[Z2_OFF + (3 * e + g) * N * PS + q * PS + pi] = S1[r][g][q];
        }
      }
    }
  }
  __syncthreads();
  // volume step C: lane (q1, q2) = (alpha, beta)
  double U[N], G1[N], G2[N], G3[N];
  double zo[2][4];  // own z traces at (q1, q2): u, d1, d2, d3 (reference)
  {
    double P[N], Q[N], S[N];
#pragma unroll
    for (int t = 0; t < N; ++t) {
      P[t] = R[C_OFF + p * PS + t];
      Q[t] = R[C_OFF + NN * PS + p * PS + t];
      S[t] = R[C_OFF + 2 * NN * PS + p * PS + t];
    }
    mv<N>(T.V, P, U);
    mv<N>(T.V, Q, G1);
    mv<N>(T.V, S, G2);
    mv<N>(T.D, P, G3);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      zo[e][0] = dotv<N>(T.ev[e], P);
      zo[e][1] = dotv<N>(T.ev[e], Q);
      zo[e][2] = dotv<N>(T.ev[e], S);
      zo[e][3] = dotv<N>(T.ed[e], P);
    }
  }
  // z-neighbour second sweep tasks (e, q1): values at (q1, all q2)
  constexpr int NT2Z = 2 * N;
  constexpr int NR2Z = (NT2Z + C::LANES - 1) / C::LANES;
  double Zn[NR2Z][4][N];
#pragma unroll
  for (int r = 0; r < NR2Z; ++r) {
    const int task = p + r * C::LANES;
    if (task < NT2Z) {
      const int e = task / N, pi = task % N;  // pi = q1
      double Sv[N], Sd[N], Sn[N];
#pragma unroll
      for (int t = 0; t < N; ++t) {
        Sv[t] = R[Z2_OFF + (3 * e + 0) * N * PS + pi * PS + t];
        Sd[t] = R[Z2_OFF + (3 * e + 1) * N * PS + pi * PS + t];
        Sn[t] = R[Z2_OFF + (3 * e + 2) * N * PS + pi * PS + t];
      }
      mv<N>(T.V, Sv, Zn[r][0]);  // u
      mv<N>(T.V, Sd, Zn[r][1]);  // d1 (axis b = 0)
      mv<N>(T.D, Sv, Zn[r][2]);  // d2 (axis c = 1)
      mv<N>(T.V, Sn, Zn[r][3]);  // d3 (normal)
    }
  }
  __syncthreads();

  // ------------------------------------------------------------------------
  // R2b: z-neighbour point values to the volume lanes; x and y face second
  // tangential sweep inputs (pencils along j3 at fixed first tangential q).
  //   x: face-side fs = 2e + s, grid (q2, j3); y: fs = 4 + 2e + s, grid (q1, j3)
  // ------------------------------------------------------------------------
  constexpr int ZN_OFF = 0;                  // (e, g) on (q1 + N q2)
  constexpr int XY_OFF = 8 * NN;             // (fs, g) pencils along j3, index = first tangential q
  if (slot) {
#pragma unroll
    for (int r = 0; r < NR2Z; ++r) {
      const int task = p + r * C::LANES;
      if (task < NT2Z) {
        const int e = task / N, pi = task % N;
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
          for (int q = 0; q < N; ++q) R[ZN_OFF + (4 * e + g) * NN + pi + N * q] = Zn[r][g][q];
      }
    }
    // x faces (own and nb) and y nb from the first sweep tasks
#pragma unroll
    for (int r = 0; r < NR1; ++r) {
      const int task = p + r * C::LANES;
      if (task < NT1) {
        const int fs = task / N, pi = task % N;  // pi = j3
        if (fs < 6) {
          // x: fs 0..3 -> xy face-side fs; y nb: fs 4,5 -> e = fs-4, s = 1
          const int xs = (fs < 4) ? fs : (4 + 2 * (fs - 4) + 1);
#pragma unroll
          for (int g = 0; g < 3; ++g)
#pragma unroll
            for (int q = 0; q < N; ++q)
              R[XY_OFF + (3 * xs + g) * N * PS + q * PS + pi] = S1[r][g][q];
        }
      }
    }
    // own y traces from the volume lanes (q1, j3) = (alpha, beta)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int xs = 4 + 2 * e;
      R[XY_OFF + (3 * xs + 0) * N * PS + alpha * PS + beta] = uyo[e];
      R[XY_OFF + (3 * xs + 1) * N * PS + alpha * PS + beta] = gyo[e];
      R[XY_OFF + (3 * xs + 2) * N * PS + alpha * PS + beta] = dyo[e];
    }
  }
  __syncthreads();
  // volume lane (q1, q2): pointwise volume flux and z-face terms, then C'
  double Wvv[N], Wdv[N], Wvd[N];
  {
    const double vol = G.h[0] * G.h[1] * G.h[2];
    const double wa = M.w[alpha], wb = M.w[beta];
    const double ih0 = 1.0 / G.h[0], ih1 = 1.0 / G.h[1], ih2 = 1.0 / G.h[2];
    double x0[N], x1[N], x2[N], x3[N];
    const int bax0 = M.b_axis[0], bax1 = M.b_axis[1], bax2 = M.b_axis[2];
#pragma unroll
    for (int q3 = 0; q3 < N; ++q3) {
      const double u = U[q3];
      const double g0 = G1[q3] * ih0, g1 = G2[q3] * ih1, g2 = G3[q3] * ih2;
      const double W = wa * wb * M.w[q3] * vol;
      const int qq0 = bax0 == 0 ? alpha : (bax0 == 1 ? beta : q3);
      const int qq1 = bax1 == 0 ? alpha : (bax1 == 1 ? beta : q3);
      const int qq2 = bax2 == 0 ? alpha : (bax2 == 1 ? beta : q3);
      const double b0 = M.bvol[0][G.ic[bax0] * N + qq0];
      const double b1 = M.bvol[1][G.ic[bax1] * N + qq1];
      const double b2 = M.bvol[2][G.ic[bax2] * N + qq2];
      const double F0 = G.kap * (M.K[0] * g0 + M.K[1] * g1 + M.K[2] * g2) - b0 * u;
      const double F1 = G.kap * (M.K[3] * g0 + M.K[4] * g1 + M.K[5] * g2) - b1 * u;
      const double F2 = G.kap * (M.K[6] * g0 + M.K[7] * g1 + M.K[8] * g2) - b2 * u;
      x0[q3] = W * M.c * u;
      x1[q3] = W * F0 * ih0;
      x2[q3] = W * F1 * ih1;
      x3[q3] = W * F2 * ih2;
    }
    mtv<N, false>(T.V, x0, Wvv);
    mtv<N, true>(T.D, x3, Wvv);
    mtv<N, false>(T.V, x1, Wdv);
    mtv<N, false>(T.V, x2, Wvd);
    // z faces (a = 2, b = 0, c = 1) at the point (q1, q2)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int f = 4 + e;
      const FaceCoef F = make_face(M, G, 2, e, fin[f], fh[f], fk[f]);
      const double un = R[ZN_OFF + (4 * e + 0) * NN + p];
      const double gbn = R[ZN_OFF + (4 * e + 1) * NN + p];
      const double gcn = R[ZN_OFF + (4 * e + 2) * NN + p];
      const double gan = R[ZN_OFF + (4 * e + 3) * NN + p];
      const double ba = face_b(M, G, N, 2, e, alpha, beta);
      double RV, Pb, Pc, Pa;
      face_point(F, zo[e][0], zo[e][1], zo[e][2], zo[e][3], un, gbn, gcn, gan, ba,
                 wa * wb * F.area, RV, Pb, Pc, Pa);
#pragma unroll
      for (int j = 0; j < N; ++j) {
        Wvv[j] = fma(T.ev[e][j], RV, Wvv[j]);
        Wvv[j] = fma(T.ed[e][j], Pa, Wvv[j]);
        Wdv[j] = fma(T.ev[e][j], Pb, Wdv[j]);
        Wvd[j] = fma(T.ev[e][j], Pc, Wvd[j]);
      }
    }
  }
  // x and y face tasks: (face-pair fp = 0,1 x (e); 2,3 y (e)) x N pencils
  constexpr int NT2 = 4 * N;
  constexpr int NR2 = (NT2 + C::LANES - 1) / C::LANES;
  double Qf[NR2][3][N];
#pragma unroll
  for (int r = 0; r < NR2; ++r) {
    const int task = p + r * C::LANES;
    if (task < NT2) {
      const int fp = task / N, pi = task % N;  // pi = first tangential q (q2 for x, q1 for y)
      const int a = (fp < 2) ? 0 : 1, e = fp & 1;
      const int f = 2 * a + e;
      const int xso = (a == 0 ? 0 : 4) + 2 * e, xsn = xso + 1;
      double val[2][4][N];  // side, {u, gb, gc, ga}, q3
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int xs = s ? xsn : xso;
        double Sv[N], Sd[N], Sn[N];
#pragma unroll
        for (int t = 0; t < N; ++t) {
          Sv[t] = R[XY_OFF + (3 * xs + 0) * N * PS + pi * PS + t];
          Sd[t] = R[XY_OFF + (3 * xs + 1) * N * PS + pi * PS + t];
          Sn[t] = R[XY_OFF + (3 * xs + 2) * N * PS + pi * PS + t];
        }
        mv<N>(T.V, Sv, val[s][0]);
        mv<N>(T.V, Sd, val[s][1]);
        mv<N>(T.D, Sv, val[s][2]);
        mv<N>(T.V, Sn, val[s][3]);
      }
      const FaceCoef F = make_face(M, G, a, e, fin[f], fh[f], fk[f]);
      const double wp = M.w[pi] * F.area;
      double RVv[N], Pbv[N], Pcv[N], Pav[N];
#pragma unroll
      for (int q = 0; q < N; ++q) {
        const double ba = face_b(M, G, N, a, e, pi, q);
        face_point(F, val[0][0][q], val[0][1][q], val[0][2][q], val[0][3][q], val[1][0][q],
                   val[1][1][q], val[1][2][q], val[1][3][q], ba, wp * M.w[q], RVv[q], Pbv[q],
                   Pcv[q], Pav[q]);
      }
      // transposed sweep along q3 (the second tangential axis, c = 2)
      mtv<N, false>(T.V, RVv, Qf[r][0]);
      mtv<N, true>(T.D, Pcv, Qf[r][0]);
      mtv<N, false>(T.V, Pbv, Qf[r][1]);
      mtv<N, false>(T.V, Pav, Qf[r][2]);
    }
  }
  __syncthreads();

  // ------------------------------------------------------------------------
  // R3: volume C'->B' exchange; y-face results to the volume lanes (q1, j3);
  // x-face results as pencils along q2 at fixed j3.
  // ------------------------------------------------------------------------
  constexpr int BP_OFF = 0;                  // Wvv, Wdv, Wvd B'-pencils (q1 + N j3) along q2
  constexpr int Y3_OFF = 3 * NN * PS;        // (e, g) on (q1 + N j3)
  constexpr int X3_OFF = Y3_OFF + 6 * NN;    // (e, g) pencils along q2, index j3
  if (slot) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      R[BP_OFF + (alpha + N * j) * PS + beta] = Wvv[j];
      R[BP_OFF + NN * PS + (alpha + N * j) * PS + beta] = Wdv[j];
      R[BP_OFF + 2 * NN * PS + (alpha + N * j) * PS + beta] = Wvd[j];
    }
#pragma unroll
    for (int r = 0; r < NR2; ++r) {
      const int task = p + r * C::LANES;
      if (task < NT2) {
        const int fp = task / N, pi = task % N;
        const int e = fp & 1;
        if (fp >= 2) {
#pragma unroll
          for (int g = 0; g < 3; ++g)
#pragma unroll
            for (int j = 0; j < N; ++j) R[Y3_OFF + (3 * e + g) * NN + pi + N * j] = Qf[r][g][j];
        } else {
#pragma unroll
          for (int g = 0; g < 3; ++g)
#pragma unroll
            for (int j = 0; j < N; ++j)
              R[X3_OFF + (3 * e + g) * N * PS + j * PS + pi] = Qf[r][g][j];
        }
      }
    }
  }
  __syncthreads();
  // volume step B': lane (q1, j3) = (alpha, beta)
  double Vv[N], Vd[N];
  {
    double P[N], Q[N], S[N];
#pragma unroll
    for (int t = 0; t < N; ++t) {
      P[t] = R[BP_OFF + p * PS + t];
      Q[t] = R[BP_OFF + NN * PS + p * PS + t];
      S[t] = R[BP_OFF + 2 * NN * PS + p * PS + t];
    }
    mtv<N, false>(T.V, P, Vv);
    mtv<N, true>(T.D, S, Vv);
    mtv<N, false>(T.V, Q, Vd);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const double q1v = R[Y3_OFF + (3 * e + 0) * NN + p];
      const double qbv = R[Y3_OFF + (3 * e + 1) * NN + p];
      const double qav = R[Y3_OFF + (3 * e + 2) * NN + p];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        Vv[j] = fma(T.ev[e][j], q1v, Vv[j]);
        Vv[j] = fma(T.ed[e][j], qav, Vv[j]);
        Vd[j] = fma(T.ev[e][j], qbv, Vd[j]);
      }
    }
  }
  // x-face tasks: transposed sweep along q2 -> (R_v, R_d) on (j2, j3)
  constexpr int NT3 = 2 * N;
  constexpr int NR3 = (NT3 + C::LANES - 1) / C::LANES;
  double Rx[NR3][2][N];
#pragma unroll
  for (int r = 0; r < NR3; ++r) {
    const int task = p + r * C::LANES;
    if (task < NT3) {
      const int e = task / N, pi = task % N;  // pi = j3
      double Q1[N], Qb[N], Qa[N];
#pragma unroll
      for (int t = 0; t < N; ++t) {
        Q1[t] = R[X3_OFF + (3 * e + 0) * N * PS + pi * PS + t];
        Qb[t] = R[X3_OFF + (3 * e + 1) * N * PS + pi * PS + t];
        Qa[t] = R[X3_OFF + (3 * e + 2) * N * PS + pi * PS + t];
      }
      mtv<N, false>(T.V, Q1, Rx[r][0]);
      mtv<N, true>(T.D, Qb, Rx[r][0]);
      mtv<N, false>(T.V, Qa, Rx[r][1]);
    }
  }
  __syncthreads();

  // ------------------------------------------------------------------------
  // R4: volume B'->A' exchange; x-face results to the volume lanes (j2, j3).
  // ------------------------------------------------------------------------
  constexpr int AP_OFF = 0;                  // Vv, Vd A'-pencils (j2 + N j3) along q1
  constexpr int X4_OFF = 2 * NN * PS;        // (e, g) on (j2 + N j3)
  if (slot) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      R[AP_OFF + (j + N * beta) * PS + alpha] = Vv[j];
      R[AP_OFF + NN * PS + (j + N * beta) * PS + alpha] = Vd[j];
    }
#pragma unroll
    for (int r = 0; r < NR3; ++r) {
      const int task = p + r * C::LANES;
      if (task < NT3) {
        const int e = task / N, pi = task % N;
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
          for (int j = 0; j < N; ++j) R[X4_OFF + (2 * e + g) * NN + j + N * pi] = Rx[r][g][j];
      }
    }
  }
  __syncthreads();
  // volume step A': lane (j2, j3) = (alpha, beta)
  if (active) {
    double P[N], Q[N], Yv[N];
#pragma unroll
    for (int t = 0; t < N; ++t) {
      P[t] = R[AP_OFF + p * PS + t];
      Q[t] = R[AP_OFF + NN * PS + p * PS + t];
    }
    mtv<N, false>(T.V, P, Yv);
    mtv<N, true>(T.D, Q, Yv);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const double rv = R[X4_OFF + (2 * e + 0) * NN + p];
      const double rd = R[X4_OFF + (2 * e + 1) * NN + p];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        Yv[j] = fma(T.ev[e][j], rv, Yv[j]);
        Yv[j] = fma(T.ed[e][j], rd, Yv[j]);
      }
    }
    double *yp = y + size_t(cell) * NNN + NN * beta + N * alpha;
#pragma unroll
    for (int t = 0; t < N; ++t) yp[t] = Yv[t];
  }
}

template <int N>
static hipError_t launch_fused_n(const dg_handle *h, const double *x, double *y, hipStream_t s) {
  using C = FCfg<N>;
  FTab<N> T;
  for (int q = 0; q < N; ++q) {
    for (int j = 0; j < N; ++j) {
      T.V[q][j] = h->tab.V[q][j];
      T.D[q][j] = h->tab.D[q][j];
    }
    T.ev[0][q] = h->tab.e0v[q];
    T.ev[1][q] = h->tab.e1v[q];
    T.ed[0][q] = h->tab.e0d[q];
    T.ed[1][q] = h->tab.e1d[q];
  }
  FMesh M;
  for (int a = 0; a < 3; ++a) {
    M.ncell[a] = h->mesh.ncell[a];
    M.h[a] = h->mesh.h[a];
    M.bvol[a] = h->mesh.bvol[a];
    M.bnode[a] = h->mesh.bnode[a];
    M.b_axis[a] = h->mesh.b_axis[a];
  }
  M.kappa = h->mesh.kappa;
  M.w = h->mesh.w;
  for (int i = 0; i < 9; ++i) M.K[i] = h->mesh.K[i];
  M.c = h->mesh.c;
  M.sigma = h->mesh.sigma;
  M.ncells = int(h->ncells);
  // tiles of up to 4 cells along axis 3: z neighbours are adjacent in the
  // processing order, y neighbours 4*N1 cells apart
  M.tz = h->mesh.ncell[2] < 4 ? h->mesh.ncell[2] : 4;
  const int nblocks = int((h->ncells + C::CPB - 1) / C::CPB);
  M.groups = (nblocks + 7) / 8;
  hipLaunchKernelGGL(apply_fused_kernel<N>, dim3(unsigned(8 * M.groups)), dim3(C::THREADS), 0, s,
                     x, y, M, T);
  return hipGetLastError();
}

hipError_t launch_apply_fused_f64(const dg_handle *h, const double *x, double *y, hipStream_t s) {
  switch (h->k + 1) {
    case 2: return launch_fused_n<2>(h, x, y, s);
    case 3: return launch_fused_n<3>(h, x, y, s);
    case 4: return launch_fused_n<4>(h, x, y, s);
    case 5: return launch_fused_n<5>(h, x, y, s);
    case 6: return launch_fused_n<6>(h, x, y, s);
    case 7: return launch_fused_n<7>(h, x, y, s);
    case 8: return launch_fused_n<8>(h, x, y, s);
    case 9: return launch_fused_n<9>(h, x, y, s);
    case 10: return launch_fused_n<10>(h, x, y, s);
    case 11: return launch_fused_n<11>(h, x, y, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dgmf
