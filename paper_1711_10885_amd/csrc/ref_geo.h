// Mesh arguments and multilinear-geometry helpers shared by the reference-
// layout kernel (apply_ref.hip) and the pencil-layout volume kernel of
// multilinear cells (geo_volume.hip).
#pragma once

#include "dg_internal.h"

namespace dgmf {

template <int N, int Q>
struct RefTab {
  double V[Q][N], D[Q][N], w[Q], xi[Q], ev[2][N], ed[2][N];
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
  // multilinear meshes (GEO kernels): vertex coordinates (N1+1)(N2+1)(N3+1) x 3,
  // |T| per cell, |F| per face normal to axis a indexed (i_a + e) + (N_a + 1)
  // (i_b + N_b i_c) (b < c the tangential axes); b and kp as formulas of the
  // physical point
  const double *verts, *cvol, *farea[3];
  double b_const[3], b_sin[3], b_amp[3], b_freq[9], b_phase[9], kpc[9];
};

// The mesh arguments of a handle; geo: evaluate b from the problem's own form
// at physical points (multilinear cells).
inline RefMesh make_ref_mesh(const dg_handle *h, bool geo) {
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
  M.verts = h->mesh.verts;
  M.cvol = h->mesh.cvol;
  for (int a = 0; a < 3; ++a) M.farea[a] = h->mesh.farea[a];
  for (int r = 0; r < 3; ++r) {
    M.b_const[r] = h->prob.b_const[r];
    M.b_sin[r] = h->prob.b_sin[r];
    M.b_amp[r] = h->prob.b_amp[r];
  }
  for (int t = 0; t < 9; ++t) {
    M.b_freq[t] = h->prob.b_freq[t];
    M.b_phase[t] = h->prob.b_phase[t];
    M.kpc[t] = h->prob.kappa_poly[t];
  }
  // the per-point path evaluates b from its formula: the problem's own form
  // (the tables above come in product form whenever kp is present)
  if (geo) M.bprod = (h->prob.flags & DG_B_PRODUCT) ? 1 : 0;
  return M;
}

__device__ __forceinline__ int sel3i(int a, int v0, int v1, int v2) { return a == 0 ? v0 : (a == 1 ? v1 : v2); }
__device__ __forceinline__ double sel3d(int a, double v0, double v1, double v2) {
  return a == 0 ? v0 : (a == 1 ? v1 : v2);
}
// Entry i of a kernel-argument pointer array by a select chain (a runtime
// index into the argument struct would copy it to scratch).
template <int L>
__device__ __forceinline__ const double *pickp(const double *const *t, int i) {
  const double *p = t[0];
#pragma unroll
  for (int s = 1; s < L; ++s)
    if (i == s) p = t[s];
  return p;
}

// ---- multilinear geometry --------------------------------------------------

constexpr int kVB = 4;  // vertex block 4 x 4 x 4 around a cell: planes i-1 .. i+2

// The trilinear map of the cell whose first vertex is block vertex
// (o0, o1, o2), at reference point (s0, s1, s2): point X and Jacobian
// J[3r + t] = d X_r / d s_t, by a linear contraction along each direction.
__device__ inline void tri_map(const double *VB, int o0, int o1, int o2, double s0, double s1, double s2, double *X,
                               double *J) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    auto v = [&](int c0, int c1, int c2) { return VB[3 * ((o0 + c0) + kVB * ((o1 + c1) + kVB * (o2 + c2))) + r]; };
    const double v000 = v(0, 0, 0), v100 = v(1, 0, 0), v010 = v(0, 1, 0), v110 = v(1, 1, 0);
    const double v001 = v(0, 0, 1), v101 = v(1, 0, 1), v011 = v(0, 1, 1), v111 = v(1, 1, 1);
    const double d00 = v100 - v000, d10 = v110 - v010, d01 = v101 - v001, d11 = v111 - v011;
    const double a00 = fma(s0, d00, v000), a10 = fma(s0, d10, v010);
    const double a01 = fma(s0, d01, v001), a11 = fma(s0, d11, v011);
    const double f0 = a10 - a00, f1 = a11 - a01;
    const double b0 = fma(s1, f0, a00), b1 = fma(s1, f1, a01);
    const double e0 = fma(s1, d10 - d00, d00), e1 = fma(s1, d11 - d01, d01);
    X[r] = fma(s2, b1 - b0, b0);
    J[3 * r + 0] = fma(s2, e1 - e0, e0);
    J[3 * r + 1] = fma(s2, f1 - f0, f0);
    J[3 * r + 2] = b1 - b0;
  }
}

// C = cof(J) = det(J) J^{-T} (row-major); returns det J
__device__ inline double cof3(const double *J, double *C) {
  C[0] = J[4] * J[8] - J[5] * J[7];
  C[1] = J[5] * J[6] - J[3] * J[8];
  C[2] = J[3] * J[7] - J[4] * J[6];
  C[3] = J[2] * J[7] - J[1] * J[8];
  C[4] = J[0] * J[8] - J[2] * J[6];
  C[5] = J[1] * J[6] - J[0] * J[7];
  C[6] = J[1] * J[5] - J[2] * J[4];
  C[7] = J[2] * J[3] - J[0] * J[5];
  C[8] = J[0] * J[4] - J[1] * J[3];
  return J[0] * C[0] + J[1] * C[1] + J[2] * C[2];
}

// component r of b at the physical point X (sum form with a sine part, or
// the product form); sin(pi x) as sinpi(x), whose argument reduction is
// exact and cheaper than that of sin (4-10 % on the multilinear kernels)
__device__ inline double geo_b(const RefMesh &M, int r, const double *X) {
  if (M.bprod) {
    double v = M.b_amp[r];
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (M.b_freq[3 * r + j] != 0.0) v *= sin(fma(M.b_freq[3 * r + j], X[j], M.b_phase[3 * r + j]));
    return v;
  }
  const int ax = M.b_axis[r];
  const double xa = ax == 0 ? X[0] : (ax == 1 ? X[1] : X[2]);
  return M.b_sin[r] != 0.0 ? fma(M.b_sin[r], sinpi(xa), M.b_const[r]) : M.b_const[r];
}

// polynomial diffusion factor at the physical point (1 without it)
__device__ inline double geo_kp(const RefMesh &M, const double *X) {
  if (!M.kpoly) return 1.0;
  double v = 1.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) v *= M.kpc[3 * j] + M.kpc[3 * j + 1] * X[j] + M.kpc[3 * j + 2] * X[j] * X[j];
  return v;
}

}  // namespace dgmf
