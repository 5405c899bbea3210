// The operator with the raised Gauss rule (q = 2p + 4: k + 3 points per
// direction, Problem B of Sec. 5.1) on the tuned kernels: the fused kernel
// with N = k + 3 Gauss points per direction and NI = k + 1 modes, i.e. with
// rectangular (k+3) x (k+1) 1D contractions.  The orthonormal Legendre basis
// is hierarchical, so the tables of the degree-k basis at the k + 3 points
// are the first k + 1 columns of the degree-(k+2) tables; the kernel reads x
// and writes y in the degree-k layout, runs every contraction only over the
// k + 1 modes of its modal side and keeps the pencils of the higher modes at
// zero.  The penalty sigma is the problem's own and the coefficient tables
// are tabulated at the k + 3 points.
#include "fused_kernel.h"

namespace dgmf {

template <typename T, bool HEUN, bool BP, bool KP>
static hipError_t launch_raised_bp(const dg_handle *h, const T *x, T *y, hipStream_t s, const double *f, double dt,
                                   int stage) {
  if (h->quad_extra != 2) return hipErrorInvalidValue;
  switch (h->k + 1) {
    case 2: return launch_fused_n<4, T, HEUN, BP, KP, 2>(h, x, y, s, f, dt, stage);
    case 3: return launch_fused_n<5, T, HEUN, BP, KP, 3>(h, x, y, s, f, dt, stage);
    case 4: return launch_fused_n<6, T, HEUN, BP, KP, 4>(h, x, y, s, f, dt, stage);
    case 5: return launch_fused_n<7, T, HEUN, BP, KP, 5>(h, x, y, s, f, dt, stage);
    case 6: return launch_fused_n<8, T, HEUN, BP, KP, 6>(h, x, y, s, f, dt, stage);
    case 7: return launch_fused_n<9, T, HEUN, BP, KP, 7>(h, x, y, s, f, dt, stage);
    case 8: return launch_fused_n<10, T, HEUN, BP, KP, 8>(h, x, y, s, f, dt, stage);
    case 9: return launch_fused_n<11, T, HEUN, BP, KP, 9>(h, x, y, s, f, dt, stage);
    default: return hipErrorInvalidValue;
  }
}

// coefficient variants as for the (k+1)-point rule
template <typename T, bool HEUN>
static hipError_t launch_raised(const dg_handle *h, const T *x, T *y, hipStream_t s, const double *f = nullptr,
                                double dt = 0.0, int stage = 0) {
  if (h->mesh.kpoly) return launch_raised_bp<T, HEUN, true, true>(h, x, y, s, f, dt, stage);
  return h->mesh.bprod ? launch_raised_bp<T, HEUN, true, false>(h, x, y, s, f, dt, stage)
                       : launch_raised_bp<T, HEUN, false, false>(h, x, y, s, f, dt, stage);
}

hipError_t apply_raised_f64(const dg_handle *h, const double *x, double *y, hipStream_t s) {
  return launch_raised<double, false>(h, x, y, s);
}

hipError_t apply_raised_f32(const dg_handle *h, const float *x, float *y, hipStream_t s) {
  return launch_raised<float, false>(h, x, y, s);
}

hipError_t launch_heun_raised_f64(const dg_handle *h, const double *x, double *y, const double *f, double dt,
                                  int stage, hipStream_t s) {
  return launch_raised<double, true>(h, x, y, s, f, dt, stage);
}

}  // namespace dgmf
