// Launchers of the fused apply kernels for the (k+1)-point rule (N = NI =
// k + 1; the kernels themselves are in fused_kernel.h, shared with the
// raised-rule launchers of raised.hip).
#include "fused_kernel.h"

namespace dgmf {

template <typename T, bool HEUN, bool BP, bool KP>
static hipError_t launch_fused_bp(const dg_handle *h, const T *x, T *y, hipStream_t s, const double *f, double dt,
                                  int stage) {
  if (h->quad_extra) return hipErrorInvalidValue;  // the raised rule: raised.hip
  switch (h->k + 1) {
    case 2: return launch_fused_n<2, T, HEUN, BP, KP>(h, x, y, s, f, dt, stage);
    case 3: return launch_fused_n<3, T, HEUN, BP, KP>(h, x, y, s, f, dt, stage);
    case 4: return launch_fused_n<4, T, HEUN, BP, KP>(h, x, y, s, f, dt, stage);
    case 5: return launch_fused_n<5, T, HEUN, BP, KP>(h, x, y, s, f, dt, stage);
    case 6: return launch_fused_n<6, T, HEUN, BP, KP>(h, x, y, s, f, dt, stage);
    case 7: return launch_fused_n<7, T, HEUN, BP, KP>(h, x, y, s, f, dt, stage);
    case 8: return launch_fused_n<8, T, HEUN, BP, KP>(h, x, y, s, f, dt, stage);
    case 9: return launch_fused_n<9, T, HEUN, BP, KP>(h, x, y, s, f, dt, stage);
    case 10: return launch_fused_n<10, T, HEUN, BP, KP>(h, x, y, s, f, dt, stage);
    case 11: return launch_fused_n<11, T, HEUN, BP, KP>(h, x, y, s, f, dt, stage);
    default: return hipErrorInvalidValue;
  }
}

// Coefficient variants: the sum-form b (the benchmarked kernels), tabulated
// product-form b, and tabulated b with the polynomial diffusion factor.
template <typename T, bool HEUN>
static hipError_t launch_fused(const dg_handle *h, const T *x, T *y, hipStream_t s, const double *f = nullptr,
                               double dt = 0.0, int stage = 0) {
  if (h->mesh.kpoly) return launch_fused_bp<T, HEUN, true, true>(h, x, y, s, f, dt, stage);
  return h->mesh.bprod ? launch_fused_bp<T, HEUN, true, false>(h, x, y, s, f, dt, stage)
                       : launch_fused_bp<T, HEUN, false, false>(h, x, y, s, f, dt, stage);
}

hipError_t launch_apply_fused_f64(const dg_handle *h, const double *x, double *y, hipStream_t s) {
  return launch_fused<double, false>(h, x, y, s);
}

hipError_t launch_heun_fused_f64(const dg_handle *h, const double *x, double *y, const double *f, double dt,
                                 int stage, hipStream_t s) {
  if (h->quad_extra) return launch_heun_raised_f64(h, x, y, f, dt, stage, s);
  return launch_fused<double, true>(h, x, y, s, f, dt, stage);
}

hipError_t launch_apply_fused_f32(const dg_handle *h, const float *x, float *y, hipStream_t s) {
  return launch_fused<float, false>(h, x, y, s);
}

}  // namespace dgmf
