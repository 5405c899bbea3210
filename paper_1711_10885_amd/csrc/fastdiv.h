// Division by a runtime-invariant divisor with a multiply and a shift, for
// the cell-index decomposition of the fused kernels (host and device).
#pragma once

#include <hip/hip_runtime.h>

namespace dgmf {

// Division by a divisor d >= 1 fixed for the launch, for 0 <= n < 2^31, by a
// multiply and a shift (Granlund and Montgomery, PLDI 1994, Thm. 4.2): with
// l = ceil(log2 d) and m = ceil(2^(31+l) / d) < 2^32, m d lies in
// [2^(31+l), 2^(31+l) + 2^l], so floor(n / d) = floor(n m / 2^(31+l)).  A
// hardware-less integer division costs about 25 instructions; this costs 3.
struct FastDiv {
  unsigned m;
  int s;  // 31 + l
};
inline FastDiv make_fastdiv(int d) {
  int l = 0;
  while ((1ull << l) < (unsigned long long)d) ++l;
  FastDiv f;
  f.s = 31 + l;
  f.m = unsigned(((1ull << f.s) + (unsigned long long)d - 1) / (unsigned long long)d);
  return f;
}
__host__ __device__ __forceinline__ int fdiv(int n, FastDiv f) {
  return int((unsigned long long)unsigned(n) * f.m >> f.s);
}

}  // namespace dgmf
