/*
 * dg.h -- C ABI of libdgmf: matrix-free weighted symmetric interior penalty
 * discontinuous Galerkin (WSIPG) operator for stationary
 * convection-diffusion-reaction on axis-aligned cuboid meshes, on MI355X.
 *
 * Method: Muething, Piatkowski & Bastian, "High-performance Implementation of
 * Matrix-free High-order Discontinuous Galerkin Methods" (arXiv 1711.10885).
 *
 *   PDE (Sec. 2.1, stationary variant):   div(b u - D grad u) + c u = f
 *   with D = kappa_T K (K constant SPD, kappa_T > 0 per cell), homogeneous
 *   Dirichlet data on the whole boundary of the box [x0,x1]x[y0,y1]x[z0,z1].
 *
 *   Operator: (A x)_i = a_h(u_x, phi_i), the bilinear form eq. (blf) of
 *   Sec. 2.2 (volume term, upwind convection flux, weighted-average
 *   consistency and symmetry terms, interior penalty), with every integral
 *   evaluated by the tensor Gauss rule with k+1 points per direction
 *   (Sec. 3.1/3.2, eqs. (evalblf), (gauss_points); n = m = p+1 as in
 *   Problem A of Sec. 5.1) and computed by sum factorization (Sec. 3.5,
 *   eq. (sum_fact_kernel)) following Algorithm 1 of Sec. 3.6.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Vectors:  ndof = N1*N2*N3*(k+1)^3 contiguous values in cell-block order,
 *   entry g = c*(k+1)^3 + j,  c = i1 + N1*(i2 + N2*i3),
 *   j = j1 + (k+1)*(j2 + (k+1)*j3)  (axis 1 fastest in both).
 *   Coefficient j multiplies theta_j1(t1) theta_j2(t2) theta_j3(t3), with
 *   t_a in [0,1] the reference coordinate of the cell along axis a and
 *   theta_j(t) = sqrt(2j+1) P_j(2t-1) the orthonormal Legendre polynomials
 *   (Sec. 2.2 uses L2-orthogonal Legendre polynomials so that the mass matrix
 *   is diagonal; here it is diag(|T|)).
 * Device pointers: x, y, f, u are device memory of the handle's device,
 *   owned by the caller.  Host arrays in dg_problem are copied by dg_setup.
 * Streams: hip_stream is a hipStream_t (NULL = default stream).  Apply calls
 *   are stream-ordered and asynchronous; solve calls synchronise the stream.
 *   A handle may be used by one host thread/stream at a time.
 * Errors: no C++ exception crosses this interface.  Every dg_status < 0 comes
 *   with a message from dg_last_error() (thread-local, valid until the next
 *   call on the same thread).
 */
#ifndef DGMF_DG_H
#define DGMF_DG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_handle dg_handle; /* opaque; owns all device tables/workspace */

typedef enum {
  DG_OK = 0,
  DG_EINVAL = -1,    /* invalid argument (message says which)              */
  DG_ENOMEM = -2,    /* device allocation failed                           */
  DG_EHIP = -3,      /* HIP runtime error (message has hipGetErrorString)  */
  DG_ENOTCONV = -4,  /* solver hit maxit; u holds the best iterate          */
  DG_ENAN = -5       /* non-finite residual or input detected               */
} dg_status;

/* Problem description (all host memory, copied by dg_setup).
 *   ncell[a]   >= 1 cells along axis a (a = 0,1,2).
 *   nodes[a]   ncell[a]+1 strictly increasing coordinates (tensor grid).
 *   k          polynomial degree 1..10 (n = m = k+1).
 *   K          row-major constant diffusion tensor, symmetric positive
 *              definite (checked by Cholesky).
 *   kappa      NULL (all 1) or one value > 0 per cell (cell order as above):
 *              D = kappa_T K on cell T.
 *   b          b_r(x) = b_const[r] + b_sin[r] * sin(pi * x_{b_axis[r]}),
 *              b_axis[r] in {0,1,2}.  (b = (sin pi y, sin pi z, sin pi x) is
 *              b_sin = 1, b_axis = {1,2,0}.)
 *   c          constant reaction coefficient.
 *   sigma      penalty scale: gamma_F = sigma * <d-,d+> / min(h_a-, h_a+) on
 *              interior faces, sigma * d / h_a on boundary faces, with
 *              d = kappa K_aa and <.,.> the harmonic mean (Sec. 2.2:
 *              sigma = alpha p (p+d-1), alpha = 2, in the paper).
 *   flags      DG_WITH_FP32: also build the FP32 operator (dg_apply_f32);
 *              DG_WITH_BLOCK_JACOBI: factor the block-Jacobi preconditioner.
 */
typedef struct {
  int32_t ncell[3];
  const double *nodes[3];
  int32_t k;
  double K[9];
  const double *kappa;
  double b_const[3];
  double b_sin[3];
  int32_t b_axis[3];
  double c;
  double sigma;
  int32_t flags;
} dg_problem;

#define DG_WITH_FP32 1
#define DG_WITH_BLOCK_JACOBI 2

/* Create a handle on the current HIP device: validates the problem, builds
 * the 1D Gauss-Legendre/Legendre tables (Sec. 3.1/3.2, eq.
 * (gradient_matrices)) and uploads geometry and coefficient tables.
 * Returns DG_EINVAL (bad problem), DG_ENOMEM, DG_EHIP.  *out is set to NULL
 * on failure. */
dg_status dg_setup(const dg_problem *p, dg_handle **out);

/* y := A x (Algorithm 1 of Sec. 3.6, every cell computes its own rows: the
 * volume term and the six face terms restricted to its own test functions,
 * so no two cells write the same entry).  x, y: device, ndof doubles, must not
 * overlap.  Asynchronous on hip_stream. */
dg_status dg_apply(dg_handle *h, const double *x, double *y, void *hip_stream);

/* Kernel selection for dg_apply (both compute the same operator and are
 * checked against the same oracle):
 *   DG_KERNEL_AUTO       the tuned kernel for the handle's degree (default);
 *   DG_KERNEL_REFERENCE  one workgroup per cell, every tensor in LDS.
 * Returns DG_EINVAL for an unknown variant. */
#define DG_KERNEL_AUTO 0
#define DG_KERNEL_REFERENCE 1
dg_status dg_set_kernel(dg_handle *h, int32_t variant);

/* Number of degrees of freedom of the handle's space (or -1 for NULL). */
int64_t dg_ndof(const dg_handle *h);

/* Polynomial degree of the handle (or -1 for NULL). */
int32_t dg_degree(const dg_handle *h);

/* Message of the last failing call on this thread ("" if none). */
const char *dg_last_error(void);

/* Free every device resource of the handle.  NULL is a no-op. */
void dg_destroy(dg_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* DGMF_DG_H */
