// Host check of the multiply-shift division used for the fused kernels' cell
// indices: fdiv(n, make_fastdiv(d)) == n / d for every divisor up to 4096 on
// the numerators around each multiple of d and on pseudo-random numerators,
// and for powers of two and their neighbours up to 2^30 against extreme
// numerators.  Prints the number of checked pairs, or the first mismatch.
#include <cstdio>
#include <cstdint>

#include "fastdiv.h"

int main() {
  using dgmf::fdiv;
  using dgmf::make_fastdiv;
  long long checked = 0;
  uint64_t state = 0x9e3779b97f4a7c15ull;
  auto next = [&]() {  // 64-bit LCG (Knuth's MMIX constants), top 31 bits
    state = state * 6364136223846793005ull + 1442695040888963407ull;
    return int(state >> 33);
  };
  auto check = [&](int n, int d) {
    const int q = fdiv(n, make_fastdiv(d));
    if (q != n / d) {
      std::printf("mismatch n=%d d=%d got %d want %d\n", n, d, q, n / d);
      return false;
    }
    ++checked;
    return true;
  };
  const int top = 2147483647;
  for (int d = 1; d <= 4096; ++d) {
    for (int k = 0; k <= 64; ++k)
      for (int r = -1; r <= 1; ++r) {
        const long long n = (long long)k * d + r;
        if (n >= 0 && n <= top && !check(int(n), d)) return 1;
      }
    for (int i = 0; i < 256; ++i)
      if (!check(next(), d)) return 1;
    if (!check(top, d) || !check(top - d, d)) return 1;
  }
  for (int e = 1; e <= 30; ++e)
    for (int dd = -1; dd <= 1; ++dd) {
      const int d = (1 << e) + dd;
      for (int i = 0; i < 4096; ++i)
        if (!check(next(), d)) return 1;
      if (!check(top, d) || !check(d - 1, d) || !check(d, d) || !check(0, d)) return 1;
    }
  std::printf("%lld\n", checked);
  return 0;
}
