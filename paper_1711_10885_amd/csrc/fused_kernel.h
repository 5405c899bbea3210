// Fused FP64 apply kernel for gfx950: volume and all six faces of each cell in
// one pass, owner-computes (each cell writes only its own rows, no atomics).
//
// Mapping.  A cell is handled by N^2 lanes ("pencil slots"); lane p = a + N b
// owns one 1D pencil of N values at a time and contracts it against the 1D
// matrices of Sec. 3.2 (eq. (gradient_matrices)), which is the sum
// factorization kernel of eq. (sum_fact_kernel) with the tensor rotation fused
// into the LDS exchange between directions.  Tensors pass through LDS only to
// change the pencil direction (pencils stored with an odd stride).
//
// Each 1D contraction uses the point symmetry of the Gauss rule and the parity
// of the Legendre basis (theta_j(1-t) = (-1)^j theta_j(t)): only rows
// q < ceil(N/2) of V = theta(xi) and D = theta'(xi) are stored and every
// contraction splits into even and odd columns, halving its multiply-adds.
// The tables are compile-time constants (gl_tables.inc, correctly rounded),
// so the compiler materialises each coefficient into scalar registers where
// it is used instead of holding a whole table live.
//
// Volume (Algorithm 1, steps 1-3), evaluation tree with a shared first sweep:
//   A  (axis 1, lanes (j2,j3)):  x -> V1 x, D1 x
//   B  (axis 2, lanes (q1,j3)):  -> V2V1x, V2D1x, D2V1x
//   C  (axis 3, lanes (q1,q2)):  -> u, d1u, d2u, d3u at the Gauss points,
//   the pointwise flux x^(r) of eq. (gauss_points) and the transposed sweep
//   C' (axis 3) in one streamed loop, then B' (axis 2), A' (axis 1) of
//   eq. (evalblf).
//
// Faces (steps 4-6 / 8-10): the normal direction is contracted first on both
// sides (Sec. 3.4/3.5: traces of u and of d_a u), then the two tangential
// directions; pointwise flux; transposed tangential sweeps; normal direction
// last.  The averaged normal flux is linear in the traces with constants per
// face, so the traces are combined into one "flux pencil" before evaluation.
// Own-side work is merged into the volume tensors where the face normal axis
// is still modal:
//   z faces: own traces from the C-stage input pencils, integration added to
//            the C'-stage accumulators;
//   y faces: own traces from the B-stage input pencils (already evaluated
//            along axis 1), integration added to the B'-stage output;
//   x faces: own traces from the x pencils, integration added to the A'
//            output.
// Neighbour traces are contracted in the normal direction straight from
// global memory (the pencil along the face normal is loaded by one lane).
#pragma once

#include <vector>

#include "dg_internal.h"
#include "mesh_nb.h"
#include "fastdiv.h"
#include "gl_tables.inc"

namespace dgmf {

// View of the compile-time table GLTab<N> at an offset; indices are resolved
// at compile time after unrolling.
template <int N, typename T>
struct CT {
  int off;
  __device__ constexpr T operator[](int i) const { return T(GLTab<N>::v[off + i]); }
  __device__ constexpr CT operator+(int o) const { return CT{off + o}; }
};
#define cptr CT<N, T>

template <int N, typename T>
__device__ __forceinline__ CT<N, T> fresh(CT<N, T> p) {
  return p;
}

// Table layout (doubles), H = ceil(N/2):
//   V rows 0..H-1 [H*N] | D rows 0..H-1 [H*N] | theta(1) [N] | theta'(1) [N] | w 0..H-1 [H]
//   | g [N], g_j = sqrt(2(2j+1)): theta_j' = sum_{k<j, j-k odd} g_k g_j theta_k
template <int N>
struct TabOff {
  static constexpr int H = (N + 1) / 2;
  static constexpr int V = 0, D = H * N, E1 = 2 * H * N, F1 = 2 * H * N + N, W = 2 * H * N + 2 * N;
  static constexpr int G = W + H;
  static constexpr int SIZE = G + N;
};

// A value known to be equal on every lane of the wave, moved to scalar
// registers (the compiler then keeps it there and loads through it with
// scalar loads).
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double wave_uniform(double v) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readfirstlane(unsigned(b)), hi = __builtin_amdgcn_readfirstlane(unsigned(b >> 32));
  return __longlong_as_double((long long)((unsigned long long)hi << 32 | lo));
}
__device__ __forceinline__ float wave_uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

struct FMesh {
  int ncell[3];
  int periodic;    // bit a: axis a is periodic
  const double *h[3], *bvol[3], *bnode[3], *kappa, *w;
  const double *ih[3];             // 1 / h per axis
  FastDiv fd_n1, fd_n2;            // by ncell[0], ncell[1]
  FastDiv fd_tile, fd_tz, fd_tzl;  // by N1 N2 tz, tz, and the depth of the last tile
  const double *bf[9], *bfn[9];  // product-form factors (BP instantiations)
  const double *kf[3], *kfn[3];  // polynomial diffusion factor (KP instantiations)
  double K[9], c, sigma;
  int b_axis[3];
  int tz;          // depth (cells along axis 3) of the tiles of the cell order
  int ncells;
  int groups;      // workgroups per XCD slot (grid = 8 * groups)
  // Heun stage written in place of y = A x by the HEUN instantiations:
  //   stage 0: y = x + dt/|T| (f - A x)
  //   stage 1: y = (y + x + dt/|T| (f - A x)) / 2   (y holds the old u)
  const double *ts_f;  // load vector f, or nullptr for f = 0
  double ts_dt;
  int ts_stage;
};

// The stage update of n consecutive outputs y[off..off+n) of one cell, from
// their values Av of A x; dv = dt / |T|, |T| the product of the cell's three
// spacings.  xv holds x[off..off+n) and, in stage 1, yv the old y there
// (loaded by the caller ahead of the store).
template <int n, typename T>
__device__ __forceinline__ void heun_store(const FMesh &M, double dv, size_t off, const T *xv, const T *yv,
                                           T *__restrict__ y, const T *Av) {
#pragma unroll
  for (int t = 0; t < n; ++t) {
    const double r = (M.ts_f ? M.ts_f[off + t] : 0.0) - double(Av[t]);
    if (M.ts_stage == 0)
      y[off + t] = T(fma(dv, r, double(xv[t])));
    else
      y[off + t] = T(0.5 * (double(yv[t]) + double(xv[t]) + dv * r));
  }
}

// Pencil storage for the exchanges that dominate LDS size.  For N = 2, 4, 8 the
// pencils are unpadded and element t of pencil p is rotated by (p N)/16
// places, which keeps 16 consecutive lanes reading element t of 16
// consecutive pencils on distinct banks.  Other N store pencils with the odd
// stride N | 1 (N + 1 for even N, N itself for odd N): lanes reading element
// t of consecutive pencils then step through the banks with an odd stride
// (an even stride would repeat banks every 64 / gcd(2 stride, 64) lanes).
template <int N>
struct PL {
  static constexpr bool SW = (N == 2 || N == 4 || N == 8);
  static constexpr int S = SW ? N : (N | 1);  // doubles per pencil
  __device__ static __forceinline__ int at(int p, int t) {
    return SW ? p * N + ((t + (p * N) / 16) & (N - 1)) : p * S + t;
  }
};

template <int N>
struct FCfg {
  static constexpr int NN = N * N;
  static constexpr int PS = N | 1;  // pencil stride: odd (see PL)
  static constexpr int LANES = NN;
  // cells per workgroup: one 64-lane wave holds 64 / N^2 cells, which
  // leaves 22 % (N = 5), 44 % (N = 6), 23 % (N = 7) and 37 % (N = 9, two
  // waves per cell) of the lanes idle; larger workgroups pack 5 cells into
  // 128 lanes (N = 5) and 7, 5 and 3 cells into 256 lanes (N = 6, 7, 9;
  // 95-98 % busy) while two workgroups (five at N = 5) still fit in the
  // 160 KB of LDS of a CU.  At N = 5 the two-wave workgroup was 8-19 %
  // faster than 10 cells in 256 lanes (fewer waves per barrier); at N = 6, 7
  // the two-wave workgroups (3 and 2 cells) idle too many lanes and were slower
  static constexpr int CPB = (N == 5) ? 5 : (N == 6) ? 7 : (N == 7) ? 5 : (N == 9) ? 3 : (NN <= 64 ? 64 / NN : 1);
  static constexpr int THREADS = ((CPB * LANES + 63) / 64) * 64;
  // register budget: two waves per SIMD at every N.  At N >= 9 this caps the
  // kernel at 256 VGPRs and spills 28-404 bytes per lane, and is still
  // 1.04-1.62x faster than one wave per SIMD without spills (the kernel is
  // bound by latency, which the second wave hides)
  static constexpr int WAVES_PER_SIMD = 2;
  // N = 5 without the diffusion factor: three waves per SIMD (168 VGPRs, a
  // 92-byte spill) measured 4.5 % faster; with it the spill grows and the
  // kernel was 38 % slower
  static constexpr int waves(bool kp) { return (N == 5 && !kp) ? 3 : WAVES_PER_SIMD; }
  static constexpr int FCW = 8;  // doubles per face-constant record
  // per-cell LDS (doubles) of each exchange round
  static constexpr int mx(int a, int b) { return a > b ? a : b; }
  static constexpr int R1 = 2 * NN * PS + 16 * N * PS;
  static constexpr int R2 = 3 * NN * PS + 4 * N * PS;
  static constexpr int R2Z = 4 * NN;
  static constexpr int R3 = 14 * N * PL<N>::S + mx(4 * NN, 3 * NN * PL<N>::S);
  static constexpr int R4 = 4 * NN + 4 * N * PS;
  static constexpr int R5 = 2 * NN * PS + 4 * NN;
  static constexpr int EXCH = mx(mx(mx(R1, R2), mx(R2Z, R3)), mx(R4, R5));
  // Per-cell stride of the exchange regions in elements of T, padded to be
  // congruent to NN * PS modulo one row of the LDS banks (64 banks of 4
  // bytes: 32 doubles or 64 floats).  The B- and C-stage pencil of lane l of
  // the workgroup then starts at l * PS modulo the row, as if the cells'
  // regions were one array, and consecutive lanes keep the odd bank stride PS
  // across cell boundaries.  Against the unpadded stride: 3-4 % faster at
  // N = 3, 1 % at N = 5, within the run-to-run variation at N = 4, 6, 7.
  template <typename T>
  static constexpr int exch() {
    constexpr int row = 256 / int(sizeof(T));
    return CPB > 1 ? EXCH + (((NN * PS - EXCH) % row) + row) % row : EXCH;
  }
};

// ---- even-odd 1D contractions --------------------------------------------
// N Gauss points; NI <= N modes on the modal side of a contraction (NI < N:
// the degree-(NI-1) basis under the N-point rule, whose tables are the first
// NI columns of the degree-(N-1) tables: the Legendre basis is hierarchical).
// Modal outputs beyond NI are zero.

// out[q] = sum_{j < NI} M[q][j] in[j], M = V (ISD false) or D (ISD true)
template <int N, bool ISD, typename T, int NI = N>
__device__ __forceinline__ void eo_mv(cptr M, const T *in, T *out) {
#pragma unroll
  for (int q = 0; q < N / 2; ++q) {
    T E = T(0), O = T(0);
#pragma unroll
    for (int j = 0; j < NI; j += 2) E = fma(M[q * N + j], in[j], E);
#pragma unroll
    for (int j = 1; j < NI; j += 2) O = fma(M[q * N + j], in[j], O);
    out[q] = E + O;
    out[N - 1 - q] = ISD ? (O - E) : (E - O);
  }
  if (N & 1) {
    constexpr int m = N / 2;
    T S = T(0);
#pragma unroll
    for (int j = ISD ? 1 : 0; j < NI; j += 2) S = fma(M[m * N + j], in[j], S);
    out[m] = S;
  }
}

// out[j] (+)= sum_q M[q][j] in[q], j < NI
template <int N, bool ISD, bool ACC, typename T, int NI = N>
__device__ __forceinline__ void eo_mtv(cptr M, const T *in, T *out) {
  constexpr int H2 = N / 2;
  T s[H2 > 0 ? H2 : 1], d[H2 > 0 ? H2 : 1];
#pragma unroll
  for (int q = 0; q < H2; ++q) {
    s[q] = in[q] + in[N - 1 - q];
    d[q] = in[q] - in[N - 1 - q];
  }
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    const bool useS = ISD ? ((j & 1) != 0) : ((j & 1) == 0);
    T acc = ACC ? out[j] : T(0);
#pragma unroll
    for (int q = 0; q < H2; ++q) acc = fma(M[q * N + j], useS ? s[q] : d[q], acc);
    if ((N & 1) && useS) acc = fma(M[(N / 2) * N + j], in[N / 2], acc);
    out[j] = acc;
  }
  if (!ACC)
#pragma unroll
    for (int j = NI; j < N; ++j) out[j] = T(0);
}

// sum_{j < NI} theta_j(1) in[j] and sum_j theta_j(0) in[j]
template <int N, typename T, int NI = N>
__device__ __forceinline__ void tr_val(cptr E1, const T *in, T &v1, T &v0) {
  T E = T(0), O = T(0);
#pragma unroll
  for (int j = 0; j < NI; j += 2) E = fma(E1[j], in[j], E);
#pragma unroll
  for (int j = 1; j < NI; j += 2) O = fma(E1[j], in[j], O);
  v1 = E + O;
  v0 = E - O;
}

// sum_{j < NI} theta_j'(1) in[j] and sum_j theta_j'(0) in[j]
template <int N, typename T, int NI = N>
__device__ __forceinline__ void tr_der(cptr F1, const T *in, T &d1, T &d0) {
  T E = T(0), O = T(0);
#pragma unroll
  for (int j = 0; j < NI; j += 2) E = fma(F1[j], in[j], E);
#pragma unroll
  for (int j = 1; j < NI; j += 2) O = fma(F1[j], in[j], O);
  d1 = E + O;
  d0 = O - E;
}

// out[j] += theta_j(1) a1 + theta_j(0) a0 + theta_j'(1) b1 + theta_j'(0) b0, j < NI
template <int N, typename T, int NI = N>
__device__ __forceinline__ void tr_acc(cptr E1, cptr F1, T a1, T a0, T b1,
                                       T b0, T *out) {
  const T ap = a1 + a0, am = a1 - a0, bp = b1 + b0, bm = b1 - b0;
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    const bool ev = (j & 1) == 0;
    out[j] = fma(E1[j], ev ? ap : am, out[j]);
    out[j] = fma(F1[j], ev ? bm : bp, out[j]);
  }
}

// out[j] += theta_j(1) a1 + theta_j(0) a0, j < NI
template <int N, typename T, int NI = N>
__device__ __forceinline__ void tr_acc_v(cptr E1, T a1, T a0, T *out) {
  const T ap = a1 + a0, am = a1 - a0;
#pragma unroll
  for (int j = 0; j < NI; ++j) out[j] = fma(E1[j], (j & 1) == 0 ? ap : am, out[j]);
}

// Modal derivative of a coefficient pencil (Legendre derivative identity):
//   out_k = g_k sum_{j>k, j-k odd} g_j in_j      (coefficients of d/dt),
// so that D in = V (G in) and a sum V a + D b is one contraction V (a + G b).
// Entries j >= NI of the input are zero, so are those of the output.
template <int N, typename T, int NI = N>
__device__ __forceinline__ void gmod(cptr g, const T *in, T *out) {
  T se = T(0), so = T(0);  // suffix sums over even / odd j
#pragma unroll
  for (int k = NI - 1; k >= 0; --k) {
    out[k] = g[k] * ((k & 1) ? se : so);
    if (k & 1)
      so = fma(g[k], in[k], so);
    else
      se = fma(g[k], in[k], se);
  }
#pragma unroll
  for (int k = NI; k < N; ++k) out[k] = T(0);
}

// Transposed modal derivative: out_j = g_j sum_{k<j, j-k odd} g_k in_k, so
// that D^T r = G^T (V^T r); j < NI (zero beyond).
template <int N, typename T, int NI = N>
__device__ __forceinline__ void gmodT(cptr g, const T *in, T *out) {
  T pe = T(0), po = T(0);  // prefix sums over even / odd k
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    out[j] = g[j] * ((j & 1) ? pe : po);
    if (j & 1)
      po = fma(g[j], in[j], po);
    else
      pe = fma(g[j], in[j], pe);
  }
#pragma unroll
  for (int j = NI; j < N; ++j) out[j] = T(0);
}

// ---- per-cell geometry and face constants ---------------------------------

struct FaceGeo {
  double h0, h1, h2;
  double ih0, ih1, ih2;  // 1 / h (kernels that carry them, see face_coef)
  double kap;
  int i0, i1, i2;
};

__device__ __forceinline__ double sel3(int a, double v0, double v1, double v2) {
  return a == 0 ? v0 : (a == 1 ? v1 : v2);
}
__device__ __forceinline__ int seli3(int a, int v0, int v1, int v2) {
  return a == 0 ? v0 : (a == 1 ? v1 : v2);
}

// Constants of the face terms of eq. (blf) for the face of cell T normal to
// axis a on side e (outer normal n_T = sgn e_a), tangential axes b < c.
// With reference-coordinate traces of the own (o) and neighbour (n) side,
//   {D grad u}_w . n_T = cTa ga_o + cTb gb_o + cTc gc_o + cNa ga_n + cNb gb_n + cNc gc_n
// (weights: delta ratio of Sec. 2.2 with delta = kappa K_aa), and the
// symmetry term of a test function of T is
//   Z (cTa th'_a th_b th_c + cTb th_a th'_b th_c + cTc th_a th_b th'_c),  Z = -W [[u]].
// Boundary faces: w_T = 1, w_N = 0, neighbour traces zero (homogeneous
// Dirichlet), gamma = sigma delta / h_a.
struct FC {
  double cTa, cTb, cTc, cNa, cNb, cNc, gamma, sgn;
};

// IHG: G carries the reciprocal spacings (loaded once per cell); otherwise
// they are read from the tables where used, which keeps three fewer doubles
// live through the kernel (measured better for N >= 9, where it spills, and
// worse below).
template <bool IHG>
__device__ __forceinline__ FC face_coef(const FMesh &M, const FaceGeo &G, int cell, int a, int e) {
  const int b = (a == 0) ? 1 : 0, c = (a == 2) ? 1 : 2;
  const int ia = seli3(a, G.i0, G.i1, G.i2);
  const int na = seli3(a, M.ncell[0], M.ncell[1], M.ncell[2]);
  const int cst = seli3(a, 1, M.ncell[0], M.ncell[0] * M.ncell[1]);
  const FaceNb nb = face_nb(cell, ia, na, cst, (M.periodic >> a) & 1, e);
  const bool in = nb.in;
  const int ncl = nb.cell;
  const double *iha_tab = a == 0 ? M.ih[0] : (a == 1 ? M.ih[1] : M.ih[2]);
  const double iha = IHG ? sel3(a, G.ih0, G.ih1, G.ih2) : iha_tab[ia];
  const double ihb = IHG ? sel3(b, G.ih0, G.ih1, G.ih2) : (b == 0 ? M.ih[0][G.i0] : M.ih[1][G.i1]);
  const double ihc = IHG ? sel3(c, G.ih0, G.ih1, G.ih2) : (c == 1 ? M.ih[1][G.i1] : M.ih[2][G.i2]);
  const double ihn = in ? iha_tab[nb.ja] : iha;
  const double kn = in ? (M.kappa ? M.kappa[ncl] : 1.0) : 0.0;
  const double Kaa = sel3(a, M.K[0], M.K[4], M.K[8]);
  const double Kab = a == 0 ? M.K[1] : (a == 1 ? M.K[3] : M.K[6]);  // K[a][b]
  const double Kac = a == 0 ? M.K[2] : (a == 1 ? M.K[5] : M.K[7]);  // K[a][c]
  const double dT = G.kap * Kaa, dN = kn * Kaa;
  FC F;
  F.sgn = e ? 1.0 : -1.0;
  // the one division; 1 / min(h_T, h_N) = max(1 / h_T, 1 / h_N)
  const double rs = 1.0 / (dT + dN);
  const double wT = in ? dN * rs : 1.0;
  const double wN = in ? dT * rs : 0.0;
  F.gamma = in ? M.sigma * (2.0 * dT * dN * rs) * fmax(iha, ihn) : M.sigma * dT * iha;
  const double sT = F.sgn * wT * G.kap, sN = F.sgn * wN * kn;
  F.cTa = sT * Kaa * iha;
  F.cTb = sT * Kab * ihb;
  F.cTc = sT * Kac * ihc;
  F.cNa = in ? sN * Kaa * ihn : 0.0;
  F.cNb = sN * Kab * ihb;
  F.cNc = sN * Kac * ihc;
  return F;
}

__device__ __forceinline__ FC load_fc(const double *R, int f) {
  FC F;
  F.cTa = R[8 * f + 0];
  F.cTb = R[8 * f + 1];
  F.cTc = R[8 * f + 2];
  F.cNa = R[8 * f + 3];
  F.cNb = R[8 * f + 4];
  F.cNc = R[8 * f + 5];
  F.gamma = R[8 * f + 6];
  F.sgn = R[8 * f + 7];
  return F;
}

// Pointwise face flux at one face point: RV multiplies the test function,
// Z = -W [[u]] the symmetry-term combination above.  Upwind flux of Sec. 2.2
// with the outward normal velocity b . n_T.
// With a pointwise diffusion factor kp (KP) every diffusive term (average,
// penalty, symmetry) carries kp at the point; the weights do not (kp is
// continuous across the face and cancels in them).
template <bool KP>
__device__ __forceinline__ void face_flux(const FC &F, double uo, double un, double avg, double ba,
                                          double W, double &RV, double &Z, double kp) {
  const double J = uo - un;
  const double bout = F.sgn * ba;
  const double Phi = bout >= 0.0 ? bout * uo : bout * un;
  if constexpr (KP) {
    RV = W * (Phi - kp * avg + kp * F.gamma * J);
    Z = -W * kp * J;
  } else {
    RV = W * (Phi - avg + F.gamma * J);
    Z = -W * J;
  }
}

// Factor table 3 r + j of the product-form b (a select chain: no dynamic
// indexing of the kernel-argument array).
__device__ __forceinline__ const double *bfac(const double *const *t, int r, int j) {
  const int i = 3 * r + j;
  const double *p = t[0];
#pragma unroll
  for (int s = 1; s < 9; ++s)
    if (i == s) p = t[s];
  return p;
}

__device__ __forceinline__ const double *sel3p(int a, const double *const *t) {
  return a == 0 ? t[0] : (a == 1 ? t[1] : t[2]);
}

// Polynomial diffusion factor at a point of the face normal to a (side e)
// with tangential Gauss indices qb, qc; 1 unless KP.
template <bool KP>
__device__ __forceinline__ double face_kp(const FMesh &M, const FaceGeo &G, int N, int a, int e, int qb,
                                          int qc) {
  if constexpr (!KP) {
    return 1.0;
  } else {
    const int b = (a == 0) ? 1 : 0, c = (a == 2) ? 1 : 2;
    const int ia = seli3(a, G.i0, G.i1, G.i2);
    const bool wrap = ((M.periodic >> a) & 1) && e && ia + 1 == seli3(a, M.ncell[0], M.ncell[1], M.ncell[2]);
    return sel3p(a, M.kfn)[face_node(ia, e, wrap)] * sel3p(b, M.kf)[seli3(b, G.i0, G.i1, G.i2) * N + qb] *
           sel3p(c, M.kf)[seli3(c, G.i0, G.i1, G.i2) * N + qc];
  }
}

// b_a at a point of the face normal to a (side e) with tangential Gauss
// indices qb, qc (tangential axes b < c).
template <bool BP>
__device__ __forceinline__ double face_b(const FMesh &M, const FaceGeo &G, int N, int a, int e,
                                         int qb, int qc) {
  if (BP) {
    const int b = (a == 0) ? 1 : 0, c = (a == 2) ? 1 : 2;
    const int ia = seli3(a, G.i0, G.i1, G.i2);
    const bool wrap = ((M.periodic >> a) & 1) && e && ia + 1 == seli3(a, M.ncell[0], M.ncell[1], M.ncell[2]);
    return bfac(M.bfn, a, a)[face_node(ia, e, wrap)] * bfac(M.bf, a, b)[seli3(b, G.i0, G.i1, G.i2) * N + qb] *
           bfac(M.bf, a, c)[seli3(c, G.i0, G.i1, G.i2) * N + qc];
  }
  const int ax = M.b_axis[a];
  const double *bv = a == 0 ? M.bvol[0] : (a == 1 ? M.bvol[1] : M.bvol[2]);
  const double *bn = a == 0 ? M.bnode[0] : (a == 1 ? M.bnode[1] : M.bnode[2]);
  if (ax == a) {
    const int ia = seli3(a, G.i0, G.i1, G.i2);
    const bool wrap = ((M.periodic >> a) & 1) && e && ia + 1 == seli3(a, M.ncell[0], M.ncell[1], M.ncell[2]);
    return bn[face_node(ia, e, wrap)];
  }
  const int b = (a == 0) ? 1 : 0;
  if (ax == b) return bv[seli3(b, G.i0, G.i1, G.i2) * N + qb];
  const int c = (a == 2) ? 1 : 2;
  return bv[seli3(c, G.i0, G.i1, G.i2) * N + qc];
}

// Cell of processing position L: tiles of tz cells along axis 3 (fewer in
// the last tile), z fastest inside a tile, then axis 1, then axis 2.  Sets
// the cell's indices along the three axes.
__device__ __forceinline__ int cell_of_logical(int L, const FMesh &M, int &i0, int &i1, int &i2) {
  const int N1 = M.ncell[0], N2 = M.ncell[1], N3 = M.ncell[2];
  const int t = fdiv(L, M.fd_tile);
  const int r = L - t * (N1 * N2 * M.tz);
  const int z0 = t * M.tz;
  const bool full = N3 - z0 >= M.tz;
  const int tzt = full ? M.tz : N3 - z0;
  const int rr = fdiv(r, full ? M.fd_tz : M.fd_tzl);
  i2 = z0 + (r - rr * tzt);
  i1 = fdiv(rr, M.fd_n1);
  i0 = rr - i1 * N1;
  return i0 + N1 * (i1 + N2 * i2);
}

template <int N, typename T, bool HEUN, bool BP, bool KP, int NI = N>
__global__ __launch_bounds__(FCfg<N>::THREADS)
__attribute__((amdgpu_waves_per_eu(FCfg<N>::waves(KP)))) void apply_fused_kernel(
    const T *__restrict__ x, T *__restrict__ y, FMesh M) {
  using C = FCfg<N>;
  using TO = TabOff<N>;
  constexpr int NN = C::NN, PS = C::PS;
  constexpr int NIII = NI * NI * NI;  // coefficients per cell (NI modes per direction)
  constexpr int H2 = N / 2;
  constexpr int EX = C::template exch<T>();
  __shared__ T lds[C::CPB * EX];
  __shared__ double fcs[C::CPB * 6 * C::FCW];  // face constants stay FP64
  // axis-3 factors of b (and of the diffusion factor) at the cell's Gauss
  // points, staged in LDS (PWS) or read from the tables at every point.
  // Staging measured 3-6 % faster at N = 6, 7, 9..11 and 2-7 % slower at
  // N = 3, 4, 8.
  constexpr bool PWS = !(N == 3 || N == 4 || N == 8);
  constexpr int PWN = PWS ? (KP ? 4 : 3) * N : 1;
  __shared__ double pwc[C::CPB * PWN];

  const int tid = threadIdx.x;
  const int cl = tid / C::LANES;
  const int p = tid - cl * C::LANES;
  const int alpha = p % N, beta = p / N;
  const bool slot = cl < C::CPB;  // thread belongs to a cell slot
  const int wg = blockIdx.x;
  const int lblock = (wg & 7) * M.groups + (wg >> 3);
  const int L = lblock * C::CPB + (slot ? cl : 0);
  const bool active = slot && L < M.ncells;
  FaceGeo G;
  int cell = 0;
  G.i0 = G.i1 = G.i2 = 0;
  if (active) cell = cell_of_logical(L, M, G.i0, G.i1, G.i2);
  // One cell per workgroup (N = 8, 10, 11: a wave holds lanes of one cell
  // only): the cell and every per-cell constant derived from it are wave-
  // uniform, kept in scalar registers (fewer VGPRs where the kernel spills).
  // Lanes past the cell's pencil slots take the cell's values too; they
  // neither store nor write LDS.
  constexpr bool UNI = C::CPB == 1;
  if (UNI) {
    cell = wave_uniform(cell);
    G.i0 = wave_uniform(G.i0);
    G.i1 = wave_uniform(G.i1);
    G.i2 = wave_uniform(G.i2);
  }
  T *R = lds + (slot ? cl : 0) * EX;
  double *RFC = fcs + (slot ? cl : 0) * 6 * C::FCW;  // per-cell face constants
  double *PW = pwc + (slot ? cl : 0) * PWN;
  const CT<N, T> tab0{0};

  constexpr bool IHG = N <= 8;  // carry 1 / h in G (see face_coef)
  G.h0 = M.h[0][G.i0];
  G.h1 = M.h[1][G.i1];
  G.h2 = M.h[2][G.i2];
  if (IHG) {
    G.ih0 = M.ih[0][G.i0];
    G.ih1 = M.ih[1][G.i1];
    G.ih2 = M.ih[2][G.i2];
  }
  G.kap = M.kappa ? M.kappa[cell] : 1.0;

  // The prologue's global loads, all issued before any of them is used: the
  // cell's x pencil along axis 1 and, for each face, the neighbour's pencil
  // along the face normal (a boundary face loads the cell's own pencil, a
  // valid address, and uses zeros).  Lanes (j2, j3) with a mode >= NI hold a
  // zero pencil (indices clamped).  Issued face by face with a use in
  // between, the loads cost one memory round trip each.
  const bool lin = alpha < NI && beta < NI;
  T X[N], NV[6][N];
  bool fin[6];
  {
    const int al = min(alpha, NI - 1), be = min(beta, NI - 1);
    const T *xp = x + size_t(cell) * NIII + NI * NI * be + NI * al;
#pragma unroll
    for (int t = 0; t < N; ++t) X[t] = (t < NI && lin) ? xp[t < NI ? t : 0] : T(0);
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int a = f >> 1, e = f & 1;
      const int ia = a == 0 ? G.i0 : (a == 1 ? G.i1 : G.i2);
      const int cst = (a == 0) ? 1 : (a == 1) ? M.ncell[0] : M.ncell[0] * M.ncell[1];
      const FaceNb nb = face_nb(cell, ia, M.ncell[a], cst, (M.periodic >> a) & 1, e);
      fin[f] = nb.in;
      const T *xn = x + size_t(nb.cell) * NIII;
      const int base = (a == 0) ? (NI * al + NI * NI * be) : (a == 1) ? (al + NI * NI * be) : (al + NI * be);
      const int st = (a == 0) ? 1 : (a == 1) ? NI : NI * NI;
#pragma unroll
      for (int t = 0; t < N; ++t) NV[f][t] = (t < NI && lin) ? xn[base + st * (t < NI ? t : 0)] : T(0);
    }
  }

  // face constants of the six faces f = 2a + e
  if (slot)
    for (int f = p; f < 6; f += C::LANES) {
      const FC F = face_coef<IHG>(M, G, cell, f >> 1, f & 1);
      RFC[8 * f + 0] = F.cTa;
      RFC[8 * f + 1] = F.cTb;
      RFC[8 * f + 2] = F.cTc;
      RFC[8 * f + 3] = F.cNa;
      RFC[8 * f + 4] = F.cNb;
      RFC[8 * f + 5] = F.cNc;
      RFC[8 * f + 6] = F.gamma;
      RFC[8 * f + 7] = F.sgn;
    }
  // The volume flux reads, at every point, the axis-3 factor of each b_r that
  // varies along axis 3 (and of the diffusion factor): with PWS staged in
  // LDS here, where their load latency overlaps the loads above, instead of
  // one dependent global load per point in the volume loop.
  if (PWS && slot)
    for (int i = p; i < PWN; i += C::LANES) {
      const int r = i / N, q = i - r * N;
      double v;
      if (r == 3)
        v = M.kf[2][G.i2 * N + q];
      else if (BP)
        v = bfac(M.bf, r, 2)[G.i2 * N + q];
      else
        v = M.b_axis[r] == 2 ? M.bvol[r][G.i2 * N + q] : 0.0;
      PW[i] = v;
    }

  // ------------------------------------------------------------------------
  // Exchange 1.  Lane (j2,j3) = (alpha,beta) owns the x pencil along axis 1.
  // Writes: Tv, Td as B-pencils (q1 + N j3) along j2, and 16 modal face
  // trace fields, each N pencils of its first tangential axis (lane
  // (alpha,beta) writes element alpha of pencil beta):
  //   x faces (a=0): grid (j2,j3), fid = 4e + {0:U_o, 1:Dn_o, 2:U_n, 3:Dn_n}
  //   y nb    (a=1): grid (j1,j3), fid = 8 + 2e + {U_n, Dn_n}
  //   z nb    (a=2): grid (j1,j2), fid = 12 + 2e + {U_n, Dn_n}
  // U = trace of u, Dn = trace of d_a u (normal direction contracted first).
  // ------------------------------------------------------------------------
  constexpr int B_OFF = 0;
  constexpr int F1_OFF = 2 * NN * PS;
  const int w1 = beta * PS + alpha;
  {
    const cptr tb = fresh(tab0);
    T Tv[N], Td[N];
    eo_mv<N, false, T, NI>(tb + TO::V, X, Tv);
    eo_mv<N, true, T, NI>(tb + TO::D, X, Td);
    T u1, u0, d1, d0;
    tr_val<N, T, NI>(tb + TO::E1, X, u1, u0);
    tr_der<N, T, NI>(tb + TO::F1, X, d1, d0);
    if (slot) {
      R[F1_OFF + 0 * N * PS + w1] = u0;
      R[F1_OFF + 1 * N * PS + w1] = d0;
      R[F1_OFF + 4 * N * PS + w1] = u1;
      R[F1_OFF + 5 * N * PS + w1] = d1;
#pragma unroll
      for (int q = 0; q < N; ++q) {
        R[B_OFF + (q + N * beta) * PS + alpha] = Tv[q];
        R[B_OFF + NN * PS + (q + N * beta) * PS + alpha] = Td[q];
      }
    }
  }
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int a = f >> 1, e = f & 1;
    const cptr tb = fresh(tab0);
    T v[N];
#pragma unroll
    for (int t = 0; t < N; ++t) v[t] = fin[f] ? NV[f][t] : T(0);
    // neighbour trace at its reference coordinate 1 - e
    T u1, u0, d1, d0;
    tr_val<N, T, NI>(tb + TO::E1, v, u1, u0);
    tr_der<N, T, NI>(tb + TO::F1, v, d1, d0);
    const int fid = (a == 0) ? (4 * e + 2) : (a == 1 ? 8 + 2 * e : 12 + 2 * e);
    if (slot) {
      R[F1_OFF + fid * N * PS + w1] = e ? u0 : u1;
      R[F1_OFF + (fid + 1) * N * PS + w1] = e ? d0 : d1;
    }
  }
  __syncthreads();
  // volume step B: lane (q1, j3) = (alpha, beta)
  T vv[N], dv[N], vd[N];
  T yS[2], yA[2];  // own y-face value trace and flux part on (q1, j3)
  {
    const cptr tb = fresh(tab0);
    T P[N], Q[N];
#pragma unroll
    for (int t = 0; t < N; ++t) {
      P[t] = R[B_OFF + p * PS + t];
      Q[t] = R[B_OFF + NN * PS + p * PS + t];
    }
    eo_mv<N, false, T, NI>(tb + TO::V, P, vv);
    eo_mv<N, false, T, NI>(tb + TO::V, Q, dv);
    eo_mv<N, true, T, NI>(tb + TO::D, P, vd);
    T u1, u0, g1, g0, d1, d0;
    tr_val<N, T, NI>(tb + TO::E1, P, u1, u0);
    tr_val<N, T, NI>(tb + TO::E1, Q, g1, g0);
    tr_der<N, T, NI>(tb + TO::F1, P, d1, d0);
    const FC F0 = load_fc(RFC, 2), F1 = load_fc(RFC, 3);
    yS[0] = u0;
    yS[1] = u1;
    yA[0] = T(F0.cTb) * g0 + T(F0.cTa) * d0;
    yA[1] = T(F1.cTb) * g1 + T(F1.cTa) * d1;
  }
  // First tangential sweep of the face traces.  Tasks:
  //   t <  2N : x face e = t/N, pencil j3 = t%N  -> Sv_o, Sv_n, A1 (own + nb flux part)
  //   t <  4N : y nb  e, pencil j3               -> Sv_n, A1_n
  //   t <  6N : z nb  e, pencil j2               -> Sv_n, A1_n
  // with Sv = V U and A1 = V (cSa Dn) + D (cSb U) = V (cSa Dn + G cSb U) along
  // the first tangential axis (G the modal derivative).
  constexpr int NT1 = 6 * N;
  constexpr int NR1 = (NT1 + C::LANES - 1) / C::LANES;
  T S1[NR1][3][N];
#pragma unroll
  for (int r = 0; r < NR1; ++r) {
    const int task = p + r * C::LANES;
    if (task < NT1) {
      const cptr tb = fresh(tab0);
      const int kind = task / (2 * N), e = (task / N) & 1, pi = task % N;
      const FC F = load_fc(RFC, 2 * kind + e);
      const int fid = (kind == 0) ? (4 * e + 2) : (kind == 1 ? 8 + 2 * e : 12 + 2 * e);
      T U[N], Ub[N], Dc[N];
#pragma unroll
      for (int t = 0; t < N; ++t) {
        U[t] = R[F1_OFF + fid * N * PS + pi * PS + t];
        Ub[t] = T(F.cNb) * U[t];
        Dc[t] = T(F.cNa) * R[F1_OFF + (fid + 1) * N * PS + pi * PS + t];
      }
      eo_mv<N, false, T, NI>(tb + TO::V, U, S1[r][1]);  // Sv_n
      if (kind == 0) {
        T Uo[N];
#pragma unroll
        for (int t = 0; t < N; ++t) {
          Uo[t] = R[F1_OFF + (4 * e) * N * PS + pi * PS + t];
          const T Do = R[F1_OFF + (4 * e + 1) * N * PS + pi * PS + t];
          Ub[t] = fma(T(F.cTb), Uo[t], Ub[t]);
          Dc[t] = fma(T(F.cTa), Do, Dc[t]);
        }
        eo_mv<N, false, T, NI>(tb + TO::V, Uo, S1[r][0]);  // Sv_o
      }
      T GU[N];
      gmod<N, T, NI>(tb + TO::G, Ub, GU);
#pragma unroll
      for (int t = 0; t < N; ++t) Dc[t] += GU[t];
      eo_mv<N, false, T, NI>(tb + TO::V, Dc, S1[r][2]);  // A1
    }
  }
  __syncthreads();

  // ------------------------------------------------------------------------
  // Exchange 2.  Volume B->C exchange; z-neighbour second tangential sweep.
  // ------------------------------------------------------------------------
  constexpr int C_OFF = 0;                 // vv, dv, vd C-pencils (q1 + N q2) along j3
  constexpr int Z2_OFF = 3 * NN * PS;      // z nb (e, {Sv_n, A1_n}) pencils along j2, index q1
  constexpr int XY_OFF = 0;                // x/y second-sweep inputs, after the C reads
  constexpr int ZN_OFF = XY_OFF + 14 * N * PL<N>::S;  // (e, {u_n, avg_n}) on (q1 + N q2)
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
      if (task >= 4 * N && task < NT1) {
        const int e = (task / N) & 1, pi = task % N;  // pi = j2
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
          for (int q = 0; q < N; ++q)
            R[Z2_OFF + (2 * e + g) * N * PS + q * PS + pi] = S1[r][1 + g][q];
      }
    }
  }
  __syncthreads();
  T Pc[N], Qc[N], Sc[N];  // C-stage input pencils of lane (q1, q2)
#pragma unroll
  for (int t = 0; t < N; ++t) {
    Pc[t] = R[C_OFF + p * PS + t];
    Qc[t] = R[C_OFF + NN * PS + p * PS + t];
    Sc[t] = R[C_OFF + 2 * NN * PS + p * PS + t];
  }
  // z-neighbour second sweep tasks (e, q1): u_n and the neighbour part of the
  // averaged normal flux at (q1, all q2); c = axis 1
  constexpr int NT2Z = 2 * N;
  constexpr int NR2Z = (NT2Z + C::LANES - 1) / C::LANES;
  T Zn[NR2Z][2][N];
#pragma unroll
  for (int r = 0; r < NR2Z; ++r) {
    const int task = p + r * C::LANES;
    if (task < NT2Z) {
      const cptr tb = fresh(tab0);
      const int e = task / N, pi = task % N;  // pi = q1
      const FC F = load_fc(RFC, 4 + e);
      T Sv[N], A1[N], GS[N];
#pragma unroll
      for (int t = 0; t < N; ++t) {
        Sv[t] = R[Z2_OFF + (2 * e + 0) * N * PS + pi * PS + t];
        A1[t] = R[Z2_OFF + (2 * e + 1) * N * PS + pi * PS + t];
      }
      gmod<N, T, NI>(tb + TO::G, Sv, GS);
#pragma unroll
      for (int t = 0; t < N; ++t) A1[t] = fma(T(F.cNc), GS[t], A1[t]);
      eo_mv<N, false, T, NI>(tb + TO::V, Sv, Zn[r][0]);
      eo_mv<N, false, T, NI>(tb + TO::V, A1, Zn[r][1]);
    }
  }
  __syncthreads();
  if (slot) {
#pragma unroll
    for (int r = 0; r < NR2Z; ++r) {
      const int task = p + r * C::LANES;
      if (task < NT2Z) {
        const int e = task / N, pi = task % N;
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
          for (int q = 0; q < N; ++q) R[ZN_OFF + (2 * e + g) * NN + pi + N * q] = Zn[r][g][q];
      }
    }
  }
  // Second tangential sweep inputs of the x and y faces (pencils along j3 at
  // fixed first tangential q), written over the consumed C-stage pencils:
  //   x e: {Sv_o, Sv_n, A1} on (q2, j3), fields 3e + g
  //   y e: {Sv_o, A1_o, Sv_n, A1_n} on (q1, j3), fields 6 + 4e + g
  if (slot) {
#pragma unroll
    for (int r = 0; r < NR1; ++r) {
      const int task = p + r * C::LANES;
      if (task < 4 * N) {
        const int kind = task / (2 * N), e = (task / N) & 1, pi = task % N;  // pi = j3
        if (kind == 0) {
#pragma unroll
          for (int g = 0; g < 3; ++g)
#pragma unroll
            for (int q = 0; q < N; ++q)
              R[XY_OFF + (3 * e + g) * N * PL<N>::S + PL<N>::at(q, pi)] = S1[r][g][q];
        } else {
#pragma unroll
          for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int q = 0; q < N; ++q)
              R[XY_OFF + (6 + 4 * e + 2 + g) * N * PL<N>::S + PL<N>::at(q, pi)] = S1[r][1 + g][q];
        }
      }
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      R[XY_OFF + (6 + 4 * e + 0) * N * PL<N>::S + PL<N>::at(alpha, beta)] = yS[e];
      R[XY_OFF + (6 + 4 * e + 1) * N * PL<N>::S + PL<N>::at(alpha, beta)] = yA[e];
    }
  }
  __syncthreads();
  // volume pointwise flux (eq. (gauss_points)) streamed over the point pairs
  // (q3, N-1-q3) straight into the C'-stage accumulators (eq. (evalblf))
  T Wvv[N], Wdv[N], Wvd[N];
#pragma unroll
  for (int j = 0; j < N; ++j) Wvv[j] = Wdv[j] = Wvd[j] = T(0);
  {
    const cptr tb = fresh(tab0);
    const cptr V = tb + TO::V, D = tb + TO::D, Wt = tb + TO::W;
    const double vol = G.h0 * G.h1 * G.h2;
    const T wab = T(M.w[alpha] * M.w[beta] * vol);
    const double ihd[3] = {IHG ? G.ih0 : M.ih[0][G.i0], IHG ? G.ih1 : M.ih[1][G.i1], IHG ? G.ih2 : M.ih[2][G.i2]};
    const T ih0 = T(ihd[0]), ih1 = T(ihd[1]), ih2 = T(ihd[2]);
    const T cc = T(M.c);
    // Kh[r][s] = kappa K_rs / (h_r h_s): D acting on reference derivatives
    T Kh[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int s2 = 0; s2 < 3; ++s2) {
        Kh[3 * r + s2] = T(G.kap * M.K[3 * r + s2] * ihd[r] * ihd[s2]);
        if (UNI) Kh[3 * r + s2] = wave_uniform(Kh[3 * r + s2]);
      }
    // b_r / h_r: per-lane constant unless b_r varies along axis 3 (then its
    // values per point come from PW or the tables)
    T bh[3];
    bool bz[3];
    const int o2 = G.i2 * N;
    // the axis-3 factor of b_r (r < 3) or of the diffusion factor (r = 3) at point q3
    auto f3 = [&](int r, int q3) -> T {
      if constexpr (PWS) return T(PW[r * N + q3]);
      if (r == 3) return T(M.kf[2][o2 + q3]);
      if (BP) return T(M.bf[3 * r + 2][o2 + q3]);
      return T(M.bvol[r][o2 + q3]);
    };
    // product form: b_r / h_r = (f_r0(q1) f_r1(q2) / h_r) f_r2(q3), a lane factor
    // times the axis-3 factor in PW
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      if (BP) {
        bz[r] = true;
        bh[r] = T(bfac(M.bf, r, 0)[G.i0 * N + alpha] * bfac(M.bf, r, 1)[G.i1 * N + beta] * ihd[r]);
        continue;
      }
      const int ax = M.b_axis[r];
      bz[r] = (ax == 2);
      const int ia = ax == 0 ? G.i0 : (ax == 1 ? G.i1 : G.i2);
      const int qa = (ax == 0) ? alpha : beta;
      const double bv = M.bvol[r][ia * N + qa];  // a valid entry whatever bz (issued unconditionally)
      bh[r] = bz[r] ? T(0) : T(bv * ihd[r]);
    }
    // polynomial diffusion factor kp(q1, q2, q3) = (lane factor) * kf_2(q3)
    const T kpl = KP ? T(M.kf[0][G.i0 * N + alpha] * M.kf[1][G.i1 * N + beta]) : T(1);
    auto flux = [&](T u, T g0, T g1, T g2, int q3, T W, T &x0, T &x1, T &x2, T &x3) {
      const T b0 = BP ? bh[0] * f3(0, q3) : (bz[0] ? f3(0, q3) * ih0 : bh[0]);
      const T b1 = BP ? bh[1] * f3(1, q3) : (bz[1] ? f3(1, q3) * ih1 : bh[1]);
      const T b2 = BP ? bh[2] * f3(2, q3) : (bz[2] ? f3(2, q3) * ih2 : bh[2]);
      x0 = W * cc * u;
      if constexpr (KP) {
        const T kq = kpl * f3(3, q3);
        x1 = W * (kq * (Kh[0] * g0 + Kh[1] * g1 + Kh[2] * g2) - b0 * u);
        x2 = W * (kq * (Kh[3] * g0 + Kh[4] * g1 + Kh[5] * g2) - b1 * u);
        x3 = W * (kq * (Kh[6] * g0 + Kh[7] * g1 + Kh[8] * g2) - b2 * u);
      } else {
        x1 = W * (Kh[0] * g0 + Kh[1] * g1 + Kh[2] * g2 - b0 * u);
        x2 = W * (Kh[3] * g0 + Kh[4] * g1 + Kh[5] * g2 - b1 * u);
        x3 = W * (Kh[6] * g0 + Kh[7] * g1 + Kh[8] * g2 - b2 * u);
      }
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
      const T s0 = a0 + m0, d0 = a0 - m0, s1 = a1 + m1, d1 = a1 - m1;
      const T s2 = a2 + m2, d2 = a2 - m2, s3 = a3 + m3, d3 = a3 - m3;
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        const bool ev = (j & 1) == 0;
        Wvv[j] = fma(V[h * N + j], ev ? s0 : d0, Wvv[j]);
        Wvv[j] = fma(D[h * N + j], ev ? d3 : s3, Wvv[j]);
        Wdv[j] = fma(V[h * N + j], ev ? s1 : d1, Wdv[j]);
        Wvd[j] = fma(V[h * N + j], ev ? s2 : d2, Wvd[j]);
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
  __builtin_amdgcn_sched_barrier(0);
  // z faces (a = 2, b = 0, c = 1) at the point (q1, q2): own traces from the
  // C-stage input pencils; integration merged into the C'-stage accumulators
  {
    const cptr tb = fresh(tab0);
    const double wab = M.w[alpha] * M.w[beta] * G.h0 * G.h1;
    T u[2], gb[2], gc[2], ga[2];
    tr_val<N, T, NI>(tb + TO::E1, Pc, u[1], u[0]);
    tr_val<N, T, NI>(tb + TO::E1, Qc, gb[1], gb[0]);
    tr_val<N, T, NI>(tb + TO::E1, Sc, gc[1], gc[0]);
    tr_der<N, T, NI>(tb + TO::F1, Pc, ga[1], ga[0]);
    double RV[2], Za[2], Zb[2], Zc[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const FC F = load_fc(RFC, 4 + e);
      const double avg = F.cTb * double(gb[e]) + F.cTc * double(gc[e]) + F.cTa * double(ga[e]) +
                         double(R[ZN_OFF + (2 * e + 1) * NN + p]);
      const double un = R[ZN_OFF + (2 * e + 0) * NN + p];
      const double ba = face_b<BP>(M, G, N, 2, e, alpha, beta);
      double Z;
      face_flux<KP>(F, double(u[e]), un, avg, ba, wab, RV[e], Z, face_kp<KP>(M, G, N, 2, e, alpha, beta));
      Za[e] = F.cTa * Z;
      Zb[e] = F.cTb * Z;
      Zc[e] = F.cTc * Z;
    }
    tr_acc<N, T, NI>(tb + TO::E1, tb + TO::F1, T(RV[1]), T(RV[0]), T(Za[1]), T(Za[0]), Wvv);
    tr_acc_v<N, T, NI>(tb + TO::E1, T(Zb[1]), T(Zb[0]), Wdv);
    tr_acc_v<N, T, NI>(tb + TO::E1, T(Zc[1]), T(Zc[0]), Wvd);
  }

  // C'-stage results as B'-pencils (q1 + N j3) along q2, beyond the x/y
  // inputs and over the consumed z-neighbour values
  constexpr int BP_OFF = ZN_OFF;
  constexpr int BPS = NN * PL<N>::S;
  __syncthreads();
  if (slot) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int a = PL<N>::at(alpha + N * j, beta);
      R[BP_OFF + a] = Wvv[j];
      R[BP_OFF + BPS + a] = Wdv[j];
      R[BP_OFF + 2 * BPS + a] = Wvd[j];
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  // tasks (face pair fp: 0,1 x e; 2,3 y e) x N pencils; each produces the
  // transposed-sweep results Q1 = V^T RV + cTc D^T Z and VZ = V^T Z over j3
  constexpr int NT2 = 4 * N;
  constexpr int NR2 = (NT2 + C::LANES - 1) / C::LANES;
  T Qf[NR2][2][N];
#pragma unroll
  for (int r = 0; r < NR2; ++r) {
    const int task = p + r * C::LANES;
    if (task < NT2) {
      const cptr tb = fresh(tab0);
      const cptr V = tb + TO::V;
      const CT<N, double> Wt{TO::W};  // FP64 weights for the FP64 face flux
      const int fp = task / N, pi = task % N;  // pi = first tangential q (q2 for x, q1 for y)
      const int a = fp >> 1, e = fp & 1;
      const FC F = load_fc(RFC, fp);
      T So[N], Sn[N], A1[N], A2[N];
      if (a == 0) {
#pragma unroll
        for (int t = 0; t < N; ++t) {
          So[t] = R[XY_OFF + (3 * e + 0) * N * PL<N>::S + PL<N>::at(pi, t)];
          Sn[t] = R[XY_OFF + (3 * e + 1) * N * PL<N>::S + PL<N>::at(pi, t)];
          A1[t] = R[XY_OFF + (3 * e + 2) * N * PL<N>::S + PL<N>::at(pi, t)];
        }
      } else {
#pragma unroll
        for (int t = 0; t < N; ++t) {
          So[t] = R[XY_OFF + (6 + 4 * e + 0) * N * PL<N>::S + PL<N>::at(pi, t)];
          A1[t] = R[XY_OFF + (6 + 4 * e + 1) * N * PL<N>::S + PL<N>::at(pi, t)] +
                  R[XY_OFF + (6 + 4 * e + 3) * N * PL<N>::S + PL<N>::at(pi, t)];
          Sn[t] = R[XY_OFF + (6 + 4 * e + 2) * N * PL<N>::S + PL<N>::at(pi, t)];
        }
      }
      // averaged normal flux pencil: A1 + G (cTc Sv_o + cNc Sv_n)
#pragma unroll
      for (int t = 0; t < N; ++t) A2[t] = T(F.cTc) * So[t] + T(F.cNc) * Sn[t];
      {
        T GA[N];
        gmod<N, T, NI>(tb + TO::G, A2, GA);
#pragma unroll
        for (int t = 0; t < N; ++t) A1[t] += GA[t];
      }
      const double hb = a == 0 ? G.h1 : G.h0;
      const double wp = M.w[pi] * hb * G.h2;
      T VR[N], VZ[N];
#pragma unroll
      for (int j = 0; j < N; ++j) VR[j] = VZ[j] = T(0);
#pragma unroll
      for (int h = 0; h < H2; ++h) {
        T Eo = 0, Oo = 0, En = 0, On = 0, Ea = 0, Oa = 0;
#pragma unroll
        for (int t = 0; t < NI; t += 2) {
          Eo = fma(V[h * N + t], So[t], Eo);
          En = fma(V[h * N + t], Sn[t], En);
          Ea = fma(V[h * N + t], A1[t], Ea);
        }
#pragma unroll
        for (int t = 1; t < NI; t += 2) {
          Oo = fma(V[h * N + t], So[t], Oo);
          On = fma(V[h * N + t], Sn[t], On);
          Oa = fma(V[h * N + t], A1[t], Oa);
        }
        const double W = wp * Wt[h];
        double RVa, Za, RVm, Zm;
        face_flux<KP>(F, double(Eo + Oo), double(En + On), double(Ea + Oa), face_b<BP>(M, G, N, a, e, pi, h), W,
                      RVa, Za, face_kp<KP>(M, G, N, a, e, pi, h));
        face_flux<KP>(F, double(Eo - Oo), double(En - On), double(Ea - Oa),
                      face_b<BP>(M, G, N, a, e, pi, N - 1 - h), W, RVm, Zm, face_kp<KP>(M, G, N, a, e, pi, N - 1 - h));
        const T sr = T(RVa + RVm), dr = T(RVa - RVm), sz = T(Za + Zm), dz = T(Za - Zm);
#pragma unroll
        for (int j = 0; j < NI; ++j) {
          const bool ev = (j & 1) == 0;
          VR[j] = fma(V[h * N + j], ev ? sr : dr, VR[j]);
          VZ[j] = fma(V[h * N + j], ev ? sz : dz, VZ[j]);
        }
      }
      if (N & 1) {
        constexpr int m = N / 2;
        T uo = 0, un = 0, av = 0;
#pragma unroll
        for (int t = 0; t < NI; t += 2) {
          uo = fma(V[m * N + t], So[t], uo);
          un = fma(V[m * N + t], Sn[t], un);
          av = fma(V[m * N + t], A1[t], av);
        }
        double RVm, Zm;
        face_flux<KP>(F, double(uo), double(un), double(av), face_b<BP>(M, G, N, a, e, pi, m), wp * Wt[m], RVm, Zm,
                      face_kp<KP>(M, G, N, a, e, pi, m));
#pragma unroll
        for (int j = 0; j < NI; j += 2) {
          VR[j] = fma(V[m * N + j], T(RVm), VR[j]);
          VZ[j] = fma(V[m * N + j], T(Zm), VZ[j]);
        }
      }
      // D^T Z = G^T (V^T Z)
      T DZ[N];
      gmodT<N, T, NI>(tb + TO::G, VZ, DZ);
#pragma unroll
      for (int j = 0; j < N; ++j) {
        Qf[r][0][j] = fma(T(F.cTc), DZ[j], VR[j]);
        Qf[r][1][j] = VZ[j];
      }
    }
  }
  __syncthreads();

  // ------------------------------------------------------------------------
  // Exchange 4.  Volume C'->B' exchange; y-face results to the volume lanes
  // (q1, j3); x-face results as pencils along q2 at fixed j3.
  // ------------------------------------------------------------------------
  // (the B'-pencils were written before the x/y tasks, at BP_OFF)
  constexpr int Y3_OFF = 0;                  // y (e, {Q1, VZ}) on (q1 + N j3)
  constexpr int X3_OFF = Y3_OFF + 4 * NN;    // x (e, {Q1, VZ}) pencils along q2, index j3
  if (slot) {
#pragma unroll
    for (int r = 0; r < NR2; ++r) {
      const int task = p + r * C::LANES;
      if (task < NT2) {
        const int fp = task / N, pi = task % N;
        const int e = fp & 1;
        if (fp >= 2) {
#pragma unroll
          for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int j = 0; j < N; ++j) R[Y3_OFF + (2 * e + g) * NN + pi + N * j] = Qf[r][g][j];
        } else {
#pragma unroll
          for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int j = 0; j < N; ++j)
              R[X3_OFF + (2 * e + g) * N * PS + j * PS + pi] = Qf[r][g][j];
        }
      }
    }
  }
  __syncthreads();
  // volume step B': lane (q1, j3) = (alpha, beta), plus the y-face merge
  T Vv[N], Vd[N];
  {
    const cptr tb = fresh(tab0);
    T P[N], Q[N], S[N];
#pragma unroll
    for (int t = 0; t < N; ++t) {
      const int a = PL<N>::at(p, t);
      P[t] = R[BP_OFF + a];
      Q[t] = R[BP_OFF + BPS + a];
      S[t] = R[BP_OFF + 2 * BPS + a];
    }
    eo_mtv<N, false, false, T, NI>(tb + TO::V, P, Vv);
    eo_mtv<N, true, true, T, NI>(tb + TO::D, S, Vv);
    eo_mtv<N, false, false, T, NI>(tb + TO::V, Q, Vd);
    const FC F0 = load_fc(RFC, 2), F1 = load_fc(RFC, 3);
    const T q0 = R[Y3_OFF + 0 * NN + p], z0 = R[Y3_OFF + 1 * NN + p];
    const T q1 = R[Y3_OFF + 2 * NN + p], z1 = R[Y3_OFF + 3 * NN + p];
    tr_acc<N, T, NI>(tb + TO::E1, tb + TO::F1, q1, q0, T(F1.cTa) * z1, T(F0.cTa) * z0, Vv);
    tr_acc_v<N, T, NI>(tb + TO::E1, T(F1.cTb) * z1, T(F0.cTb) * z0, Vd);
  }
  // x-face tasks: transposed sweep along q2 -> (R_v, R_d) on (j2, j3)
  constexpr int NT3 = 2 * N;
  constexpr int NR3 = (NT3 + C::LANES - 1) / C::LANES;
  T Rx[NR3][2][N];
#pragma unroll
  for (int r = 0; r < NR3; ++r) {
    const int task = p + r * C::LANES;
    if (task < NT3) {
      const cptr tb = fresh(tab0);
      const int e = task / N, pi = task % N;  // pi = j3
      const FC F = load_fc(RFC, e);
      T Q1[N], VZ[N], VV[N], GV[N];
#pragma unroll
      for (int t = 0; t < N; ++t) {
        Q1[t] = R[X3_OFF + (2 * e + 0) * N * PS + pi * PS + t];
        VZ[t] = R[X3_OFF + (2 * e + 1) * N * PS + pi * PS + t];
      }
      // R_v = V^T Q1 + cTb D^T VZ = V^T Q1 + cTb G^T (V^T VZ),  R_d = cTa V^T VZ
      eo_mtv<N, false, false, T, NI>(tb + TO::V, VZ, VV);
      eo_mtv<N, false, false, T, NI>(tb + TO::V, Q1, Rx[r][0]);
      gmodT<N, T, NI>(tb + TO::G, VV, GV);
#pragma unroll
      for (int j = 0; j < N; ++j) {
        Rx[r][0][j] = fma(T(F.cTb), GV[j], Rx[r][0][j]);
        Rx[r][1][j] = T(F.cTa) * VV[j];
      }
    }
  }
  __syncthreads();

  // ------------------------------------------------------------------------
  // Exchange 5.  Volume B'->A' exchange; x-face results to the volume lanes.
  // ------------------------------------------------------------------------
  constexpr int AP_OFF = 0;                  // Vv, Vd A'-pencils (j2 + N j3) along q1
  constexpr int X4_OFF = 2 * NN * PS;        // (e, {R_v, R_d}) on (j2 + N j3)
  // Heun stage: the lane's x pencil and (stage 1) the old u it updates are
  // loaded here, so that their latency overlaps this exchange and step A'
  // instead of stalling the store (Heun stages 4.5-8.5 % faster).  Lanes that
  // store nothing load from the start of x and y, valid addresses.
  T hx[HEUN ? NI : 1], hy[HEUN ? NI : 1];
  if constexpr (HEUN) {
    const bool own = active && alpha < NI && beta < NI;
    const size_t off = size_t(own ? cell : 0) * NIII + (own ? NI * NI * beta + NI * alpha : 0);
#pragma unroll
    for (int t = 0; t < NI; ++t) {
      hx[t] = x[off + t];
      hy[t] = M.ts_stage ? y[off + t] : T(0);
    }
  }
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
  // volume step A': lane (j2, j3) = (alpha, beta), plus the x-face merge
  if (active && alpha < NI && beta < NI) {
    const cptr tb = fresh(tab0);
    T P[N], Q[N], Yv[N];
#pragma unroll
    for (int t = 0; t < N; ++t) {
      P[t] = R[AP_OFF + p * PS + t];
      Q[t] = R[AP_OFF + NN * PS + p * PS + t];
    }
    eo_mtv<N, false, false, T, NI>(tb + TO::V, P, Yv);
    eo_mtv<N, true, true, T, NI>(tb + TO::D, Q, Yv);
    const T rv0 = R[X4_OFF + 0 * NN + p], rd0 = R[X4_OFF + 1 * NN + p];
    const T rv1 = R[X4_OFF + 2 * NN + p], rd1 = R[X4_OFF + 3 * NN + p];
    tr_acc<N, T, NI>(tb + TO::E1, tb + TO::F1, rv1, rv0, rd1, rd0, Yv);
    const size_t off = size_t(cell) * NIII + NI * NI * beta + NI * alpha;
    if (HEUN) {
      const double ivol = IHG ? G.ih0 * G.ih1 * G.ih2 : M.ih[0][G.i0] * M.ih[1][G.i1] * M.ih[2][G.i2];
      heun_store<NI>(M, M.ts_dt * ivol, off, hx, hy, y, Yv);
    } else {
#pragma unroll
      for (int t = 0; t < NI; ++t) y[off + t] = Yv[t];
    }
  }
}

// ---------------------------------------------------------------------------
// One cell per lane (k = 1): the whole 2x2x2 cell lives in registers, so
// there is no LDS exchange and no barrier.  Same operator, same face
// constants and flux as the pencil kernel; the volume uses the direct tensor
// sums (N^3 terms per point value, which for N = 2 is no more work than the
// factorised sweeps) and the faces contract the normal direction first.
// Cells are taken in natural order inside contiguous per-XCD ranges, so the
// face neighbours of a range are mostly L2 hits.
// ---------------------------------------------------------------------------
template <int N, typename T>
struct LaneTab {
  static constexpr int H = (N + 1) / 2;
  static __device__ __forceinline__ T V(int q, int j) {
    const double v = GLTab<N>::v[TabOff<N>::V + (q < H ? q : N - 1 - q) * N + j];
    return T((q < H || (j & 1) == 0) ? v : -v);  // theta_j(1-t) = (-1)^j theta_j(t)
  }
  static __device__ __forceinline__ T D(int q, int j) {
    const double v = GLTab<N>::v[TabOff<N>::D + (q < H ? q : N - 1 - q) * N + j];
    return T((q < H || (j & 1) == 1) ? v : -v);  // theta_j'(1-t) = (-1)^(j+1) theta_j'(t)
  }
  static __device__ __forceinline__ T E(int e, int j) {  // theta_j(e), e = 0, 1
    const double v = GLTab<N>::v[TabOff<N>::E1 + j];
    return T((e == 1 || (j & 1) == 0) ? v : -v);
  }
  static __device__ __forceinline__ T F(int e, int j) {  // theta_j'(e)
    const double v = GLTab<N>::v[TabOff<N>::F1 + j];
    return T((e == 1 || (j & 1) == 1) ? v : -v);
  }
  static __device__ __forceinline__ double W(int q) { return GLTab<N>::v[TabOff<N>::W + (q < H ? q : N - 1 - q)]; }
};

template <int N, typename T, bool HEUN, bool BP, bool KP>
__global__ __launch_bounds__(256) void apply_lane_kernel(const T *__restrict__ x, T *__restrict__ y, FMesh M) {
  constexpr int NN = N * N, NNN = N * N * N;
  using TB = LaneTab<N, T>;
  const int wg = blockIdx.x;
  const int lblock = (wg & 7) * M.groups + (wg >> 3);
  const int cell = lblock * 256 + int(threadIdx.x);
  if (cell >= M.ncells) return;
  FaceGeo G;
  {
    const int r = fdiv(cell, M.fd_n1);
    G.i0 = cell - r * M.ncell[0];
    G.i2 = fdiv(r, M.fd_n2);
    G.i1 = r - G.i2 * M.ncell[1];
  }
  G.h0 = M.h[0][G.i0];
  G.h1 = M.h[1][G.i1];
  G.h2 = M.h[2][G.i2];
  G.ih0 = M.ih[0][G.i0];
  G.ih1 = M.ih[1][G.i1];
  G.ih2 = M.ih[2][G.i2];
  G.kap = M.kappa ? M.kappa[cell] : 1.0;
  T X[NNN], Y[NNN];
  {
    const T *xp = x + size_t(cell) * NNN;
#pragma unroll
    for (int j = 0; j < NNN; ++j) {
      X[j] = xp[j];
      Y[j] = T(0);
    }
  }
  // ---- volume (Alg. 1 steps 1-3) ----
  {
    const double vol = G.h0 * G.h1 * G.h2;
    const double ihd[3] = {G.ih0, G.ih1, G.ih2};
    const int ic[3] = {G.i0, G.i1, G.i2};
    T Kh[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) Kh[3 * r + c] = T(G.kap * M.K[3 * r + c] * ihd[r] * ihd[c]);
    const T cc = T(M.c);
#pragma unroll
    for (int q3 = 0; q3 < N; ++q3)
#pragma unroll
      for (int q2 = 0; q2 < N; ++q2)
#pragma unroll
        for (int q1 = 0; q1 < N; ++q1) {
          T u = 0, g1 = 0, g2 = 0, g3 = 0;
#pragma unroll
          for (int j3 = 0; j3 < N; ++j3)
#pragma unroll
            for (int j2 = 0; j2 < N; ++j2)
#pragma unroll
              for (int j1 = 0; j1 < N; ++j1) {
                const T xv = X[j1 + N * j2 + NN * j3];
                const T v1 = TB::V(q1, j1), v2 = TB::V(q2, j2), v3 = TB::V(q3, j3);
                u = fma(v1 * v2 * v3, xv, u);
                g1 = fma(TB::D(q1, j1) * v2 * v3, xv, g1);
                g2 = fma(v1 * TB::D(q2, j2) * v3, xv, g2);
                g3 = fma(v1 * v2 * TB::D(q3, j3), xv, g3);
              }
          const int qa[3] = {q1, q2, q3};
          T bh[3];
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            if (BP) {
              bh[r] = T(bfac(M.bf, r, 0)[ic[0] * N + q1] * bfac(M.bf, r, 1)[ic[1] * N + q2] *
                        bfac(M.bf, r, 2)[ic[2] * N + q3] * ihd[r]);
              continue;
            }
            const int ax = M.b_axis[r];
            const int qx = ax == 0 ? qa[0] : (ax == 1 ? qa[1] : qa[2]);
            const int ix = ax == 0 ? ic[0] : (ax == 1 ? ic[1] : ic[2]);
            bh[r] = T(M.bvol[r][ix * N + qx] * ihd[r]);
          }
          const T W = T(TB::W(q1) * TB::W(q2) * TB::W(q3) * vol);
          const T f0 = W * cc * u;
          T f1, f2, f3;
          if constexpr (KP) {
            const T kq = T(M.kf[0][ic[0] * N + q1] * M.kf[1][ic[1] * N + q2] * M.kf[2][ic[2] * N + q3]);
            f1 = W * (kq * (Kh[0] * g1 + Kh[1] * g2 + Kh[2] * g3) - bh[0] * u);
            f2 = W * (kq * (Kh[3] * g1 + Kh[4] * g2 + Kh[5] * g3) - bh[1] * u);
            f3 = W * (kq * (Kh[6] * g1 + Kh[7] * g2 + Kh[8] * g3) - bh[2] * u);
          } else {
            f1 = W * (Kh[0] * g1 + Kh[1] * g2 + Kh[2] * g3 - bh[0] * u);
            f2 = W * (Kh[3] * g1 + Kh[4] * g2 + Kh[5] * g3 - bh[1] * u);
            f3 = W * (Kh[6] * g1 + Kh[7] * g2 + Kh[8] * g3 - bh[2] * u);
          }
#pragma unroll
          for (int j3 = 0; j3 < N; ++j3)
#pragma unroll
            for (int j2 = 0; j2 < N; ++j2)
#pragma unroll
              for (int j1 = 0; j1 < N; ++j1) {
                const T v1 = TB::V(q1, j1), v2 = TB::V(q2, j2), v3 = TB::V(q3, j3);
                T acc = Y[j1 + N * j2 + NN * j3];
                acc = fma(v1 * v2 * v3, f0, acc);
                acc = fma(TB::D(q1, j1) * v2 * v3, f1, acc);
                acc = fma(v1 * TB::D(q2, j2) * v3, f2, acc);
                acc = fma(v1 * v2 * TB::D(q3, j3), f3, acc);
                Y[j1 + N * j2 + NN * j3] = acc;
              }
        }
  }
  // ---- faces (Alg. 1 steps 4-10), owner computes ----
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int a = f >> 1, e = f & 1;
    const int b = (a == 0) ? 1 : 0, c = (a == 2) ? 1 : 2;
    const FC F = face_coef<true>(M, G, cell, a, e);
    const int ia = a == 0 ? G.i0 : (a == 1 ? G.i1 : G.i2);
    const int cst = (a == 0) ? 1 : (a == 1) ? M.ncell[0] : M.ncell[0] * M.ncell[1];
    const FaceNb nb = face_nb(cell, ia, M.ncell[a], cst, (M.periodic >> a) & 1, e);
    const bool in = nb.in;
    T XN[NNN];
    {
      const T *xn = x + size_t(nb.cell) * NNN;
#pragma unroll
      for (int j = 0; j < NNN; ++j) XN[j] = in ? xn[j] : T(0);
    }
    const int sa = a == 0 ? 1 : (a == 1 ? N : NN), sb = b == 0 ? 1 : (b == 1 ? N : NN), sc = c == 1 ? N : NN;
    // normal direction first: traces of u and d_a u on the face, coefficients in (jb, jc)
    T To[NN], Tdo[NN], Tn[NN], Tdn[NN];
#pragma unroll
    for (int jc = 0; jc < N; ++jc)
#pragma unroll
      for (int jb = 0; jb < N; ++jb) {
        T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
        for (int ja = 0; ja < N; ++ja) {
          const int j = ja * sa + jb * sb + jc * sc;
          s0 = fma(TB::E(e, ja), X[j], s0);
          s1 = fma(TB::F(e, ja), X[j], s1);
          s2 = fma(TB::E(1 - e, ja), XN[j], s2);
          s3 = fma(TB::F(1 - e, ja), XN[j], s3);
        }
        To[jb + N * jc] = s0;
        Tdo[jb + N * jc] = s1;
        Tn[jb + N * jc] = s2;
        Tdn[jb + N * jc] = s3;
      }
    const double hb = b == 0 ? G.h0 : G.h1;
    const double hc = c == 1 ? G.h1 : G.h2;
    T Rv[NN], Rd[NN];
#pragma unroll
    for (int i = 0; i < NN; ++i) Rv[i] = Rd[i] = T(0);
    const T cTa = T(F.cTa), cTb = T(F.cTb), cTc = T(F.cTc);
#pragma unroll
    for (int qc = 0; qc < N; ++qc)
#pragma unroll
      for (int qb = 0; qb < N; ++qb) {
        T uo = 0, gao = 0, gbo = 0, gco = 0, un = 0, gan = 0, gbn = 0, gcn = 0;
#pragma unroll
        for (int jc = 0; jc < N; ++jc)
#pragma unroll
          for (int jb = 0; jb < N; ++jb) {
            const T vv = TB::V(qb, jb) * TB::V(qc, jc);
            const T dv = TB::D(qb, jb) * TB::V(qc, jc), vd = TB::V(qb, jb) * TB::D(qc, jc);
            const int i = jb + N * jc;
            uo = fma(vv, To[i], uo);
            gao = fma(vv, Tdo[i], gao);
            gbo = fma(dv, To[i], gbo);
            gco = fma(vd, To[i], gco);
            un = fma(vv, Tn[i], un);
            gan = fma(vv, Tdn[i], gan);
            gbn = fma(dv, Tn[i], gbn);
            gcn = fma(vd, Tn[i], gcn);
          }
        // pointwise face flux in FP64 (penalty, weighted average, upwind)
        const double avg = F.cTa * double(gao) + F.cTb * double(gbo) + F.cTc * double(gco) +
                           F.cNa * double(gan) + F.cNb * double(gbn) + F.cNc * double(gcn);
        const double W = TB::W(qb) * TB::W(qc) * hb * hc;
        double RV, Z;
        face_flux<KP>(F, double(uo), double(un), avg, face_b<BP>(M, G, N, a, e, qb, qc), W, RV, Z,
                      face_kp<KP>(M, G, N, a, e, qb, qc));
        const T rv = T(RV), z = T(Z);
#pragma unroll
        for (int jc = 0; jc < N; ++jc)
#pragma unroll
          for (int jb = 0; jb < N; ++jb) {
            const T vv = TB::V(qb, jb) * TB::V(qc, jc);
            const T dv = TB::D(qb, jb) * TB::V(qc, jc), vd = TB::V(qb, jb) * TB::D(qc, jc);
            const int i = jb + N * jc;
            Rv[i] = fma(vv, rv, Rv[i]);
            Rv[i] = fma(cTb * dv + cTc * vd, z, Rv[i]);
            Rd[i] = fma(cTa * vv, z, Rd[i]);
          }
      }
    // normal direction last: theta(e) for the value part, theta'(e) for d_a
#pragma unroll
    for (int jc = 0; jc < N; ++jc)
#pragma unroll
      for (int jb = 0; jb < N; ++jb)
#pragma unroll
        for (int ja = 0; ja < N; ++ja) {
          const int j = ja * sa + jb * sb + jc * sc;
          Y[j] = fma(TB::E(e, ja), Rv[jb + N * jc], Y[j]);
          Y[j] = fma(TB::F(e, ja), Rd[jb + N * jc], Y[j]);
        }
    // materialise Y here (no instruction is emitted), so that this face's
    // accumulators die before the next face instead of all six staying live
#pragma unroll
    for (int j = 0; j < NNN; ++j) asm volatile("" : "+v"(Y[j]));
  }
  if (HEUN) {
    // x is still in registers (X); the old u of stage 1 is loaded once
    T Yo[NNN];
#pragma unroll
    for (int j = 0; j < NNN; ++j) Yo[j] = M.ts_stage ? y[size_t(cell) * NNN + j] : T(0);
    heun_store<NNN>(M, M.ts_dt * (G.ih0 * G.ih1 * G.ih2), size_t(cell) * NNN, X, Yo, y, Y);
  } else {
    T *yp = y + size_t(cell) * NNN;
#pragma unroll
    for (int j = 0; j < NNN; ++j) yp[j] = Y[j];
  }
}

template <int N, typename T, bool HEUN, bool BP, bool KP, int NI = N>
static hipError_t launch_fused_n(const dg_handle *h, const T *x, T *y, hipStream_t s, const double *f = nullptr,
                                 double dt = 0.0, int stage = 0) {
  using C = FCfg<N>;
  FMesh M;
  for (int a = 0; a < 3; ++a) {
    M.ncell[a] = h->mesh.ncell[a];
    M.h[a] = h->mesh.h[a];
    M.ih[a] = h->mesh.ih[a];
    M.bvol[a] = h->mesh.bvol[a];
    M.bnode[a] = h->mesh.bnode[a];
    M.b_axis[a] = h->mesh.b_axis[a];
  }
  for (int t = 0; t < 9; ++t) {
    M.bf[t] = h->mesh.bf[t];
    M.bfn[t] = h->mesh.bfn[t];
  }
  for (int j = 0; j < 3; ++j) {
    M.kf[j] = h->mesh.kf[j];
    M.kfn[j] = h->mesh.kfn[j];
  }
  M.kappa = h->mesh.kappa;
  M.w = h->mesh.w;
  for (int i = 0; i < 9; ++i) M.K[i] = h->mesh.K[i];
  M.c = h->mesh.c;
  M.sigma = h->mesh.sigma;
  M.ncells = int(h->ncells);
  M.periodic = h->mesh.periodic;
  // tiles of up to 4 cells along axis 3: z neighbours are adjacent in the
  // processing order, y neighbours 4*N1 cells apart
  M.tz = h->mesh.ncell[2] < 4 ? h->mesh.ncell[2] : 4;
  {
    const int n1 = h->mesh.ncell[0], n2 = h->mesh.ncell[1], n3 = h->mesh.ncell[2];
    const int last = n3 - ((n3 - 1) / M.tz) * M.tz;  // depth of the last tile, 1..tz
    M.fd_n1 = make_fastdiv(n1);
    M.fd_n2 = make_fastdiv(n2);
    M.fd_tile = make_fastdiv(n1 * n2 * M.tz);
    M.fd_tz = make_fastdiv(M.tz);
    M.fd_tzl = make_fastdiv(last);
  }
  M.ts_f = f;
  M.ts_dt = dt;
  M.ts_stage = stage;
  if constexpr (N == 2 && NI == 2) {  // k = 1: one cell per lane
    const int nblocks = int((h->ncells + 255) / 256);
    M.groups = (nblocks + 7) / 8;
    hipLaunchKernelGGL((apply_lane_kernel<2, T, HEUN, BP, KP>), dim3(unsigned(8 * M.groups)), dim3(256), 0, s, x, y, M);
    return hipGetLastError();
  }
  const int nblocks = int((h->ncells + C::CPB - 1) / C::CPB);
  M.groups = (nblocks + 7) / 8;
  hipLaunchKernelGGL((apply_fused_kernel<N, T, HEUN, BP, KP, NI>), dim3(unsigned(8 * M.groups)), dim3(C::THREADS), 0,
                     s, x, y, M);
  return hipGetLastError();
}

}  // namespace dgmf
