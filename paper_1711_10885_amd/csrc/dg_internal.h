// Internal declarations of libdgmf (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "dg.h"

namespace dgmf {

constexpr int kMaxN = 11;         // k <= 10
constexpr int kMaxQ = 13;         // Gauss points per direction (q = 3p + 4 at k = 7)
constexpr int kBjGroup = 8;  // cells per group of the shared-block apply
constexpr int kMaxBjBlock = 512;  // block Jacobi for (k+1)^3 <= 512
constexpr int kMlpHidden = 256;   // hidden width of the cell-patch network
constexpr int64_t kMlpChunk = 65536;  // cells per inference chunk
struct Mlp;

// 1D tables on the reference interval [0,1] for one degree (Sec. 3.2,
// eq. (gradient_matrices); face tables B^(q) of Sec. 3.4):
//   V[q][j] = theta_j(xi_q), D[q][j] = theta_j'(xi_q),
//   e0v/e1v = theta_j(0/1), e0d/e1d = theta_j'(0/1), w = Gauss weights.
struct Tables {
  int n;
  int m;  // quadrature points (rows of V, D; entries of xi, w)
  double xi[kMaxQ], w[kMaxQ];
  double V[kMaxQ][kMaxN], D[kMaxQ][kMaxN];
  double e0v[kMaxN], e1v[kMaxN], e0d[kMaxN], e1d[kMaxN];
};

// Geometry/coefficient tables in device memory, shared by all kernels.
struct DevMesh {
  int ncell[3];
  double *h[3];       // cell extents per axis, ncell[a]
  double *ih[3];      // their reciprocals 1 / h
  double *nodes[3];   // node coordinates per axis, ncell[a] + 1
  double *bvol[3];    // b_r at volume Gauss coordinates: [ncell[b_axis[r]] * m]
  double *bnode[3];   // b_r at nodes of axis b_axis[r]: [ncell[b_axis[r]] + 1]
  // product form (DG_B_PRODUCT; else null): factor f_rj of b_r along axis j,
  // b_amp[r] folded into j = 0, at the Gauss coordinates [ncell[j] * m] and
  // at the nodes [ncell[j] + 1] of axis j; index 3 r + j
  double *bf[9];
  double *bfn[9];
  int bprod;
  // polynomial diffusion factor (DG_KAPPA_POLY; else null): kp_j at the
  // Gauss coordinates [ncell[j] * m] and nodes [ncell[j] + 1] of axis j.
  // With it the b tables above are filled (product form) whatever form b has.
  double *kf[3];
  double *kfn[3];
  int kpoly;
  double *kappa;      // per cell or nullptr (= 1)
  int periodic;       // bit a: axis a is periodic (DG_PERIODIC_*)
  double *w;          // Gauss weights on [0,1] (for lane-dependent lookups)
  double K[9];
  double c, sigma;
  int b_axis[3];
  // multilinear meshes (DG_MULTILINEAR; else null): vertex coordinates
  // (N1+1)(N2+1)(N3+1) x 3, |T| per cell, |F| per face normal to axis a
  // indexed (i_a + e) + (N_a + 1) (i_b + N_b i_c), b < c the tangential axes
  double *verts;
  double *cvol;
  double *farea[3];
  int multilinear;
};

}  // namespace dgmf

struct dg_handle {
  int device;
  int k;
  int64_t ncells, ndof;
  dg_problem prob;  // host copy (pointers cleared)
  dgmf::Tables tab;   // (k+1)-point rule (load vector)
  dgmf::Tables tabq;  // the operator's rule, m = k + 1 + quad_extra points
  int quad_extra;
  int affine;         // the mesh is an affine image of the tensor grid (folded into the coefficients)
  double vol_scale;   // |det A|: physical cell volume over tensor-grid cell volume (1 if not affine)
  dgmf::DevMesh mesh;
  void *dev_block;  // single allocation backing the DevMesh arrays
  void *geo_block;  // multilinear meshes: vertices, cell volumes, face areas (or null)
  int variant;      // DG_KERNEL_*
  // solver workspace: grown on demand, freed by dg_destroy
  void *ws;
  size_t ws_bytes;
  double *red;      // reduction partials + small device vectors of the Krylov kernels
  double *ts;       // time-stepping workspace: 2 ndof doubles (or null)
  // block Jacobi: inverse cell blocks, FP32, column-major per cell (or null)
  float *bj;
  _Float16 *bj16;      // the same blocks in FP16, scaled per cell (inner FP32 solves)
  float *bj16_scale;
  int bj_nb;
  int64_t bj_nblocks;  // blocks stored: ncells, or the number of cell classes
  // cells grouped by class (shared blocks only, else null): kBjGroup cell
  // indices per group, -1 padding the last group of a class; block per group
  int32_t *bj_cells;
  int32_t *bj_gblock;
  int64_t bj_ngroups;
  // learned cell-patch preconditioner (or null)
  dgmf::Mlp *mlp;
};

namespace dgmf {

dg_status set_error(dg_status s, const std::string &msg);
dg_status hip_error(hipError_t e, const char *what);

// Kernel launchers, dispatching on k.
hipError_t launch_apply_ref_f64(const dg_handle *h, const double *x, double *y, hipStream_t s);
// multilinear meshes: the reference-layout kernel with per-point geometry
hipError_t launch_apply_geo_f64(const dg_handle *h, const double *x, double *y, hipStream_t s);
// volume of multilinear cells in the pencil layout (rules with <= 13 points per
// direction, geo_volume_supported); the faces then come from the reference kernel
bool geo_volume_supported(const dg_handle *h);
hipError_t launch_geo_volume_f64(const dg_handle *h, const double *x, double *y, hipStream_t s);
hipError_t launch_apply_fused_f64(const dg_handle *h, const double *x, double *y, hipStream_t s);
hipError_t launch_apply_fused_f32(const dg_handle *h, const float *x, float *y, hipStream_t s);
// One Heun stage fused into the apply's store: stage 0 y = x + dt/|T| (f - A x),
// stage 1 y = (y + x + dt/|T| (f - A x)) / 2; f may be nullptr (f = 0).
hipError_t launch_heun_fused_f64(const dg_handle *h, const double *x, double *y, const double *f, double dt,
                                 int stage, hipStream_t s);

// Operator application through the kernel the handle selects.
hipError_t apply_f64(const dg_handle *h, const double *x, double *y, hipStream_t s);
// the raised rule on the tuned kernels: k + 3 points, k + 1 modes
hipError_t apply_raised_f64(const dg_handle *h, const double *x, double *y, hipStream_t s);
hipError_t apply_raised_f32(const dg_handle *h, const float *x, float *y, hipStream_t s);
hipError_t launch_heun_raised_f64(const dg_handle *h, const double *x, double *y, const double *f, double dt,
                                  int stage, hipStream_t s);
// FP32 operator of the handle (raised rule included)
hipError_t apply_f32(const dg_handle *h, const float *x, float *y, hipStream_t s);

// Block Jacobi: build the inverse cell blocks (setup), z = M^{-1} r.
dg_status build_block_jacobi(dg_handle *h, const dg_problem *p);
template <typename TR, typename TZ>
hipError_t bj_apply(const dg_handle *h, const TR *r, TZ *z, hipStream_t s, bool half_store = false);

// Learned preconditioner: z = BJ r + s_T MLP(p_T / s_T); ready once trained
// or loaded (and block Jacobi is present).
template <typename TR>
hipError_t learned_apply(dg_handle *h, const TR *r, TR *z, hipStream_t s);
bool learned_ready(const dg_handle *h);

// Resolve, once per device (that device current), the address of the static
// workspace of dg_heun_noalloc (called by dg_setup).
dg_status static_scratch_init(int device);

// Free the solver / learned resources of a handle (called by dg_destroy).
void release_solver(dg_handle *h);
void release_learned(dg_handle *h);

}  // namespace dgmf
