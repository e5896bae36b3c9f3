// Host check of the multiply-high division constants the pass kernels use:
// for every tested divisor d and numerator x < 2^31, the device formula
// (mulhi(x, m) + x) >> s (evaluated here in 64-bit host arithmetic) equals
// x / d.  Prints "<cases> <mismatches>"; exits nonzero on a mismatch.
#include <cstdio>

#include "fft_engine.hpp"

int main() {
  using namespace lshom;
  unsigned long long bad = 0, checked = 0;
  for (uint32_t d = 1; d <= 70000; d = d < 4096 ? d + 1 : d * 3 + 1) {
    const FastDiv f = make_fastdiv(d);
    auto q = [&](uint32_t x) { return (uint32_t)(((((uint64_t)x * f.m) >> 32) + x) >> f.s); };
    for (uint32_t x = 0; x < 20000; ++x, ++checked) bad += q(x) != x / d;
    for (uint64_t x = 20000; x < (1ull << 31); x = x * 7 / 5 + 13, ++checked)
      bad += q((uint32_t)x) != (uint32_t)x / d;
    const uint32_t top = (1u << 31) - 1;
    ++checked;
    bad += q(top) != top / d;
  }
  std::printf("%llu %llu\n", checked, bad);
  return bad != 0;
}
