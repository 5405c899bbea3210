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
  DG_ENAN = -5,      /* non-finite residual or input detected               */
  DG_EIO = -6        /* a file could not be opened, read, written or verified */
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
 *              b_sin = 1, b_axis = {1,2,0}.)  With DG_B_PRODUCT in flags the
 *              product form below replaces it.
 *   c          constant reaction coefficient.
 *   sigma      penalty scale: gamma_F = sigma * <d-,d+> / min(h_a-, h_a+) on
 *              interior (and periodic) faces, sigma * d / h_a on boundary
 *              faces, with
 *              d = kappa K_aa and <.,.> the harmonic mean (Sec. 2.2:
 *              sigma = alpha p (p+d-1), alpha = 2, in the paper).
 *   flags      DG_WITH_BLOCK_JACOBI: build the block-Jacobi preconditioner
 *              (k <= 7): the cell blocks A_TT of the operator (volume term
 *              and the self-coupling of the six faces) are extracted by
 *              probing, inverted in FP64 (Gauss-Jordan; coercivity makes every
 *              block positive real, so no pivoting) and stored in FP32:
 *              4 ncells (k+1)^6 bytes, plus 8 ncells (k+1)^6 bytes while
 *              building.  Cells whose blocks are equal by construction (the
 *              same spacings of the cell and of its face neighbours along
 *              each axis, the same kappa on the cell and its neighbours, all
 *              to about 1e-11 relative, the same boundary faces, and b
 *              without a sine part) share one stored block when that at
 *              least halves the store: a uniform mesh with constant
 *              coefficients has 27 blocks.  With a periodic axis of an odd
 *              number of cells > 1 the two-colour probing is not valid:
 *              DG_EINVAL.
 *              DG_PERIODIC_X, _Y, _Z: the axis is periodic (the first and
 *              last cells are face neighbours across the domain boundary,
 *              an interior face of the same form, with b_a read at node 0
 *              from both sides); other axes keep homogeneous Dirichlet
 *              faces.  b must then take the same value at both ends of a
 *              periodic axis for the scheme to be consistent (the sine part
 *              does when the axis spans an integer length).
 *              DG_B_PRODUCT: the flow field is the product form
 *                b_r(x) = b_amp[r] * prod_{j<3} f_rj(x_j),
 *                f_rj(s) = sin(b_freq[3r+j] s + b_phase[3r+j]), or 1 where
 *                b_freq[3r+j] == 0,
 *              evaluated at the Gauss points like the other form (the
 *              Taylor-Green field of the transport example of Sec. 5.4 is
 *              of this form); b_const and b_sin are then unused (b_axis
 *              must still be 0, 1 or 2).
 *              Block Jacobi classes then key on the cell position along
 *              every axis some factor depends on.
 *              DG_KAPPA_POLY: the diffusion tensor varies inside cells,
 *                D(x) = kappa_T kp(x) K,
 *                kp(x) = prod_{j<3} (c[3j] + c[3j+1] x_j + c[3j+2] x_j^2),
 *              c = kappa_poly (coefficients polynomial in the coordinates, as
 *              in Problems B and C of Sec. 5.1), evaluated at the Gauss
 *              points of cells and faces: d = nu^T D nu, the weights of the
 *              averages and gamma_F are taken at each face point (kp is
 *              continuous, so the weights reduce to those of kappa_T and
 *              gamma_F scales by kp).  Every factor must be positive at every
 *              Gauss coordinate and node of its axis: DG_EINVAL otherwise.
 *   quad_extra 0: the (k+1)-point Gauss rule per direction (q = 2p, Problem A
 *              of Sec. 5.1); 2: the raised rule with k+3 points (q = 2p + 4,
 *              Problem B), for k <= 8.  Every integral of the operator uses
 *              the rule, the load vector included.  With 2 the
 *              operator runs the tuned kernel with k+3 Gauss points and k+1
 *              modes per direction (rectangular 1D contractions; the tables
 *              of the hierarchical basis are the first k+1 columns of those
 *              of degree k+2), in FP64 and FP32, Heun stages fused;
 *              DG_KERNEL_REFERENCE selects the reference-layout kernel.
 *   affine     with DG_AFFINE the mesh is the image x = A xi of the tensor
 *              grid xi of the nodes (affine cells, Problem B of Sec. 5.1):
 *              gradients, normals, face and cell measures, d = nu^T D nu and
 *              |F| / min|T| in gamma_F are those of the physical cells.  The
 *              change of variables x = A xi turns every volume and face
 *              integral into the tensor-grid one with K' = |det A| A^-1 K A^-T,
 *              b' = |det A| A^-1 b, c' = |det A| c, which setup applies, so the
 *              tuned kernels run unchanged.  Requires A finite and invertible
 *              and b constant (b_sin = 0, no DG_B_PRODUCT: a b varying in x
 *              would not stay separable in xi): DG_EINVAL otherwise.  With
 *              DG_KAPPA_POLY the factor kp is a polynomial in the grid
 *              coordinates xi and passes through as a scalar factor of K'
 *              (affine cells, polynomial coefficients and the raised rule
 *              together are Problem B).  dg_load_vector rejects such
 *              handles; dg_heun uses the physical cell volumes.
 *   vertices   with DG_MULTILINEAR the mesh is given by its vertices, a
 *              logically structured grid of (N1+1)(N2+1)(N3+1) points (host
 *              array of 3 doubles each, vertex (v0,v1,v2) at index
 *              v0 + (N1+1)(v1 + (N2+1) v2)); cell (i0,i1,i2) is the image of
 *              the reference cube under the trilinear (Q1) map through the
 *              vertices (i0+c0, i1+c1, i2+c2), c in {0,1}^3 (multilinear
 *              geometry, Sec. 4; Problem C of Sec. 5.1; parallelepiped cells
 *              with different Jacobians are the affine cells of Problem B).
 *              The Jacobian J of the map is evaluated at every quadrature
 *              point: gradients J^{-T} grad_ref, volume weight det J, and on
 *              a face xi_a = e the area-weighted normal cof(J) e_a, so nu,
 *              d = nu^T D nu, the weights and gamma_F vary over a face; in
 *              gamma_F, |F| / min(|T-|,|T+|) is the face area over the
 *              smaller cell volume (integrated with the operator's rule).  b
 *              (either form) and the polynomial factor kp are evaluated at
 *              the physical point.  nodes are ignored (may be NULL).  The
 *              Gauss rule: quad_extra 0, 2, or ceil((k+3)/2) (the rule
 *              q = 3p + 4 of Problem C, ceil((3k+5)/2) points), k <= 7.
 *              Requires det J > 0 at the corners and centre of every cell,
 *              kp > 0 on the vertices' bounding box, no periodic axis, no
 *              DG_AFFINE and no DG_WITH_BLOCK_JACOBI: DG_EINVAL otherwise.
 *              Only dg_apply (always the multilinear reference-layout
 *              kernel) and dg_solve with DG_GMRES64 and DG_PREC_NONE run on
 *              such handles; the FP32 operator, dg_heun (the mass matrix is
 *              not diagonal on non-affine cells) and dg_load_vector return
 *              DG_EINVAL.  The handle keeps (N1+1)(N2+1)(N3+1) 3 + ncells +
 *              3 (N+1) N N doubles of geometry tables.
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
  double b_amp[3];    /* product-form flow field (DG_B_PRODUCT only) */
  double b_freq[9];
  double b_phase[9];
  double kappa_poly[9];  /* polynomial diffusion factor (DG_KAPPA_POLY only) */
  int32_t quad_extra;    /* Gauss points per direction m = k + 1 + quad_extra */
  double affine[9];      /* A of the affine map x = A xi (DG_AFFINE only), row-major */
  const double *vertices; /* vertex coordinates (DG_MULTILINEAR only), see above */
} dg_problem;

#define DG_WITH_BLOCK_JACOBI 2
#define DG_PERIODIC_X 4
#define DG_PERIODIC_Y 8
#define DG_PERIODIC_Z 16
#define DG_B_PRODUCT 32
#define DG_KAPPA_POLY 64
#define DG_AFFINE 128
#define DG_MULTILINEAR 256

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

/* Load vector f_{T,j} = (f, phi_j)_T of a separable source
 *   f(x) = sum_{t < nterms} alpha[t] g(kinds[3t], x_1) g(kinds[3t+1], x_2) g(kinds[3t+2], x_3),
 *   g(0, s) = 1, g(1, s) = sin(pi s), g(2, s) = cos(pi s),
 * the right-hand side of Sec. 2.2 for homogeneous Dirichlet data, by the
 * tensor Gauss rule of the operator (Sec. 3.1: k+1 points per direction, k+3
 * with quad_extra = 2), so that it matches the operator's rule.  alpha, kinds:
 * host arrays (nterms in 1..16); f: device, ndof doubles.  Asynchronous on
 * hip_stream.  DG_EINVAL on bad terms. */
dg_status dg_load_vector(dg_handle *h, int32_t nterms, const double *alpha, const int32_t *kinds, double *f,
                         void *hip_stream);

/* L2 projection onto the DG space of the Gaussian
 *   g(x) = amp exp(-width |x - center|^2)
 * (the initial concentration of the transport example, Sec. 5.4):
 * u = M^{-1} l with l_{T,j} = (g, phi_j)_T by the operator's Gauss rule (k+1
 * points per direction, k+3 with quad_extra = 2) and M = |T| I the mass
 * matrix of the orthonormal basis, so u_{T,j} = l_{T,j} / |T|.  No periodic
 * images are added on periodic axes.  center: host, 3 values; u: device, ndof
 * doubles.  Tensor-grid handles only (DG_EINVAL with DG_AFFINE or
 * DG_MULTILINEAR); DG_EINVAL for a non-finite amp or center or width <= 0.
 * Asynchronous on hip_stream. */
dg_status dg_project_gaussian(dg_handle *h, double amp, double width, const double *center, double *u,
                              void *hip_stream);

/* y := A x with FP32 vectors (the operator of the mixed-precision tier): the
 * 1D contractions, the LDS exchanges and the volume pointwise flux run in
 * FP32; the face constants (weights, penalty gamma_F) and the pointwise face
 * flux (jump, weighted average, upwind value, penalty term) are evaluated in
 * FP64 from the FP32 traces and rounded to FP32 before the transposed
 * contractions.  Same layout as dg_apply; always the tuned kernel.
 * x, y: device, ndof floats, must not overlap.  Asynchronous on hip_stream. */
dg_status dg_apply_f32(dg_handle *h, const float *x, float *y, void *hip_stream);

/* Kernel selection for dg_apply (both compute the same operator and are
 * checked against the same oracle):
 *   DG_KERNEL_AUTO       the tuned kernel for the handle's degree (default);
 *   DG_KERNEL_REFERENCE  one workgroup per cell, every tensor in LDS.
 * Returns DG_EINVAL for an unknown variant. */
#define DG_KERNEL_AUTO 0
#define DG_KERNEL_REFERENCE 1
dg_status dg_set_kernel(dg_handle *h, int32_t variant);

/* ---------------------------------------------------------------------------
 * Solvers.  The paper motivates the fast operator application as the core of
 * iterative solvers (Sec. 1) and stops there; dg_solve wraps the operator in
 * restarted GMRES (right preconditioning, classical Gram-Schmidt, Givens
 * rotations, the true residual recomputed at every restart) and its
 * variants below.
 * ------------------------------------------------------------------------- */
#define DG_GMRES64 0  /* GMRES(m): FP64 operator and FP64 Krylov basis.          */
#define DG_GMRES_IR 1 /* GMRES-IR: FP64 residual r = f - A u and update          *
                       * u += ||r|| d in FP64; the correction d solves           *
                       * A d = r/||r|| by one FP32 GMRES(m) cycle (FP32 operator *
                       * of dg_apply_f32, FP32 basis, FP32 preconditioner        *
                       * input/output) to inner_tol.                             */
#define DG_FGMRES 2   /* flexible GMRES(m) in FP64: the basis of preconditioned  *
                       * vectors Z is kept, so the preconditioner may change     *
                       * between applications (the learned one does).            */

#define DG_PREC_NONE 0
#define DG_PREC_BLOCK_JACOBI 1 /* inverse cell blocks A_TT (DG_WITH_BLOCK_JACOBI) */
#define DG_PREC_LEARNED 2      /* block Jacobi plus the cell-patch network        *
                                * (DG_FGMRES only); falls back to block Jacobi   *
                                * alone on a non-finite value in a cycle or when *
                                * the true residual falls by less than 10 % over *
                                * ten cycles                                      */

/* Orthogonalisation of each new Krylov direction w against the basis V:
 *   DG_ORTH_CGS1  classical Gram-Schmidt, one projection: h = V^T w (with
 *                 ||w||^2 in the same pass), v = (w - V h) / ||w - V h||,
 *                 the norm from ||w||^2 - ||h||^2; two passes over the basis;
 *   DG_ORTH_CGS2  the projection repeated once (orthogonal to working
 *                 precision): three passes over the basis. */
#define DG_ORTH_CGS1 0
#define DG_ORTH_CGS2 1

typedef struct {
  int32_t method;   /* DG_GMRES64 | DG_GMRES_IR | DG_FGMRES          (0)     */
  int32_t precond;  /* DG_PREC_*                                      (0)     */
  int32_t restart;  /* m, 1..63                                       (30)    */
  int32_t maxit;    /* cap on Arnoldi steps (inner steps for IR)      (20000) */
  int32_t orth;     /* DG_ORTH_CGS1 | DG_ORTH_CGS2                    (0)     */
  double inner_tol; /* GMRES-IR inner relative tolerance              (1e-4)  */
} dg_solve_opts;

typedef struct {
  int32_t iters;         /* Arnoldi steps (inner FP32 steps for GMRES-IR)     */
  int32_t outer;         /* restart cycles (refinement steps for GMRES-IR)    */
  int32_t applies;       /* FP64 operator applications                         */
  int32_t applies_f32;   /* FP32 operator applications                         */
  int32_t fallback_used; /* 1 if the learned preconditioner was replaced      */
  int32_t fallback_step; /* Arnoldi steps done when it was replaced (-1: not)  */
  int32_t fallback_cycle;/* restart cycles done when it was replaced (-1: not) */
  double fallback_resid; /* true relative residual when it was replaced       */
  double rel_resid;      /* ||f - A u||_2 / ||f||_2, FP64, at exit             */
  double seconds;        /* host wall time of the call                         */
} dg_solve_stats;

/* Solve A u = f to ||f - A u||_2 <= tol ||f||_2 (true FP64 residual).
 * f, u: device, ndof doubles, no overlap; u holds the initial guess on entry
 * and the last iterate on return.  o == NULL selects the defaults shown above;
 * st may be NULL.  The Krylov workspace ((m+1) ndof values, plus m ndof for
 * DG_FGMRES) is allocated on first use and kept by the handle.
 * Synchronises hip_stream.  Returns DG_EINVAL (bad options, or a tier the
 * handle was not set up for), DG_ENOMEM, DG_EHIP, DG_ENOTCONV (maxit reached;
 * u is the last iterate and st is filled), DG_ENAN (non-finite value). */
dg_status dg_solve(dg_handle *h, const double *f, double *u, double tol, const dg_solve_opts *o,
                   dg_solve_stats *st, void *hip_stream);

/* z := M^{-1} r for the handle's preconditioner precond:
 *   DG_PREC_BLOCK_JACOBI (needs DG_WITH_BLOCK_JACOBI): z_T = A_TT^{-1} r_T with
 *     the FP32 inverse cell blocks, FP64 accumulation;
 *   DG_PREC_LEARNED (needs block Jacobi and a trained or loaded network):
 *     z_T = q_T + s_T (N(p_T/s_T) - N(-p_T/s_T)) / 2, q = BJ r, see
 *     dg_learned_train.
 * r, z: device, ndof doubles, no overlap.  Asynchronous on hip_stream.
 * DG_EINVAL if the handle has no such preconditioner. */
dg_status dg_precond_apply(dg_handle *h, int32_t precond, const double *r, double *z, void *hip_stream);

/* ---------------------------------------------------------------------------
 * Learned cell-patch preconditioner (extension beyond the paper).
 *
 * With q = BJ r (q_T = A_TT^{-1} r_T), p_T is the patch of q: its
 * coefficients on T and on the six face neighbours in the order T, -x, +x,
 * -y, +y, -z, +z (zero where a neighbour is outside the domain), 7 (k+1)^3
 * values; s_T = ||p_T||_2.  The network N is an MLP
 * in = 7 (k+1)^3 -> 256 -> 256 -> out = (k+1)^3 with ReLU after the two
 * hidden layers and biases on all three, run with BF16 weights and
 * activations and FP32 accumulation (MFMA).  The preconditioner adds the odd
 * part of the network to block Jacobi:
 *   z_T = q_T + s_T (N(p_T / s_T) - N(-p_T / s_T)) / 2,
 * so that z(-r) = -z(r) and z(a r) = a z(r) for a > 0.
 *
 * Parameter layout (public, FP32, row-major, n = dg_learned_nparams):
 *   W1 [256 x in] | b1 [256] | W2 [256 x 256] | b2 [256] | W3 [out x 256] | b3 [out]
 * (layer l computes h_l = W_l h_{l-1} + b_l).  Supported for k <= 7.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t npairs; /* training patches                                    (100000) */
  int32_t nrhs;   /* random exact solutions u* the pairs come from       (8)      */
  int32_t epochs; /* passes over the training split (90 %)               (20)     */
  int32_t batch;  /* minibatch rows, multiple of 64                      (1024)   */
  float lr;       /* Adam step size (beta1 0.9, beta2 0.999, eps 1e-8)   (1e-3)   */
  uint64_t seed;  /* seeds initialisation, data and shuffling            (6)      */
  int32_t max_steps; /* largest GMRES step count j of the pairs         (0)      */
} dg_learn_opts;

typedef struct {
  int32_t epochs, steps;   /* epochs run, optimiser steps taken                  */
  double train_loss;       /* mean loss of the last epoch                        */
  double val_loss;         /* validation loss (10 % split) after training        */
  double val_loss_initial; /* validation loss of the initial network (= block    *
                            * Jacobi, the last layer starts at zero)             */
  double seconds;          /* total host wall time                               */
  double seconds_data;     /* of which: generating the training pairs            */
} dg_learn_stats;

/* Train the network on the GPU (needs DG_WITH_BLOCK_JACOBI).
 * Pairs come from the solver itself: for nrhs random exact solutions u*
 * (seeded counter-based draws), f = A u*; block-Jacobi GMRES from u = 0
 * stopped after j = 0, 1, 2, 4, ..., max_steps steps gives u_j (u_0 = 0), and
 * the exact pair (r_j = f - A u_j, e_j = u* - u_j) is sampled at uniformly
 * drawn cells, in equal numbers per (u*, j); the fields come in sign pairs
 * (u*, -u*).  With q_j = BJ r_j: input
 * p_T / s_T (patch of q_j), target (e_j - q_j)_T / s_T, loss: mean squared error
 * over the out outputs of each row.  W1, W2 start He-normal, W3 and biases
 * at zero (so the untrained preconditioner is block Jacobi).  Adam with FP32
 * master weights.  opts == NULL selects the defaults; st may be NULL.
 * Synchronises hip_stream.  DG_EINVAL, DG_ENOMEM, DG_EHIP, DG_ENAN (loss not
 * finite). */
dg_status dg_learned_train(dg_handle *h, const dg_learn_opts *opts, dg_learn_stats *st, void *hip_stream);

/* Parameter count of the public layout above (-1 for NULL or k > 7). */
int64_t dg_learned_nparams(const dg_handle *h);

/* Load / read the FP32 parameters (host arrays of n = dg_learned_nparams
 * values).  Loading resets the optimiser state and marks the network ready.
 * Synchronous.  DG_EINVAL on a wrong n. */
dg_status dg_learned_set_params(dg_handle *h, const float *params, int64_t n);
dg_status dg_learned_get_params(dg_handle *h, float *params, int64_t n);

/* Checkpoint of the network and its optimiser state (an extension beyond the
 * paper), so that training can stop and resume.  path: host string, a file
 * name.  dg_learned_save writes a 64-byte header (magic "DGMFNET1", format
 * version 1, k, input, hidden and output widths, the parameter count n of the
 * public layout, the Adam step count, an FNV-1a 64-bit checksum of the body),
 * then the parameters and the Adam first and second moments, n FP32 values
 * each in the public layout, in native byte order; it needs a trained or
 * loaded network (DG_EINVAL otherwise).  dg_learned_load reads such a file
 * into a handle of the same degree: parameters, moments and step count are
 * restored (the next dg_mlp_step continues the saved run exactly) and the
 * network is marked ready.  Synchronous.  DG_EINVAL (NULL arguments, a file
 * of another degree or format), DG_EIO (open, read or write failure,
 * truncated file, checksum mismatch), DG_EHIP. */
dg_status dg_learned_save(dg_handle *h, const char *path);
dg_status dg_learned_load(dg_handle *h, const char *path);

/* The network on caller rows (for checks and inference outside the solver).
 * X: device, B x in floats (rounded to BF16 on entry); T: device, B x out
 * targets; B a positive multiple of 64.
 *   dg_mlp_forward: Y (device, B x out floats) = N(X).
 *   dg_mlp_grad:    gradients of the loss (mean over B x out squared errors)
 *                   with respect to every parameter, in the public layout, to
 *                   the host array grad (n values); *loss (host) if non-NULL.
 *   dg_mlp_step:    forward, backward and one Adam step with step size lr.
 * Synchronise hip_stream. */
dg_status dg_mlp_forward(dg_handle *h, const float *X, int32_t B, float *Y, void *hip_stream);
dg_status dg_mlp_grad(dg_handle *h, const float *X, const float *T, int32_t B, float *grad, int64_t n,
                      double *loss, void *hip_stream);
dg_status dg_mlp_step(dg_handle *h, const float *X, const float *T, int32_t B, float lr, double *loss,
                      void *hip_stream);

/* ---------------------------------------------------------------------------
 * Explicit time stepping.  The semi-discrete system M du/dt + A u = f of
 * Sec. 2.2 (eq. (ODE_system)) with the diagonal mass matrix of the
 * orthonormal basis (M = |T| I on cell T), advanced by the two-stage
 * strong-stability-preserving Runge-Kutta method (Heun) of the paper's
 * transport example (Sec. 5.4):
 *   u1 = u + dt M^{-1} (f - A u),   u <- (u + u1 + dt M^{-1} (f - A u1)) / 2.
 * u: device, ndof doubles, advanced in place by nsteps steps of size dt.
 * f: device, ndof doubles (a load vector, constant in time; must not
 * overlap u) or NULL for f = 0.  Workspace of 2 ndof doubles is allocated
 * on first use and kept by the handle.  Asynchronous on hip_stream.
 * Returns DG_EINVAL (NULL u, dt not positive and finite, nsteps < 0,
 * overlapping u and f), DG_ENOMEM, DG_EHIP.
 * ------------------------------------------------------------------------- */
dg_status dg_heun(dg_handle *h, double *u, const double *f, double dt, int32_t nsteps, void *hip_stream);

/* dg_heun for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * steps and kernels, with the stage workspace taken from a fixed array of
 * 64 MiB in device memory that the library holds on every device it runs on
 * until the process ends, instead of the handle's workspace.  It calls no
 * allocating routine.  Needs ndof * 8 bytes on the fused path (the tuned
 * kernels, either rule) and 2 ndof * 8 bytes with DG_KERNEL_REFERENCE: at
 * most 8,388,608 or 4,194,304 DOF; larger handles get DG_EINVAL
 * (use dg_heun).  Every call on one device shares that array and it keeps
 * the last call's contents (nothing in it needs to start at zero): calls
 * that overlap in time on one device, from several streams or threads,
 * race and give wrong results.  Arguments, stream behaviour and the other
 * errors as dg_heun. */
dg_status dg_heun_noalloc(dg_handle *h, double *u, const double *f, double dt, int32_t nsteps, void *hip_stream);

/* Number of degrees of freedom of the handle's space (or -1 for NULL). */
int64_t dg_ndof(const dg_handle *h);

/* Polynomial degree of the handle (or -1 for NULL). */
int32_t dg_degree(const dg_handle *h);

/* Number of inverse cell blocks the block-Jacobi preconditioner stores: the
 * number of cells, or the number of cell classes when cells share their
 * block (see DG_WITH_BLOCK_JACOBI); 0 without block Jacobi, -1 for NULL. */
int64_t dg_bj_nblocks(const dg_handle *h);

/* Message of the last failing call on this thread ("" if none). */
const char *dg_last_error(void);

/* Free every device resource of the handle.  NULL is a no-op. */
void dg_destroy(dg_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* DGMF_DG_H */
