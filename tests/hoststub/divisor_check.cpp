// Exhaustive-in-divisor check of the library's invariant-divisor arithmetic
// (common.h make_divisor / divide) against the hardware division on the CPU:
// every divisor 1..65536 against a spread of dividends up to 2^32 - 1, and large
// divisors against random dividends.  Returns 0 when every quotient matches.
#include <cstdio>
#include <cstdint>

#include "../../paper_2202_12147_amd/csrc/common.h"

using lbmib::Divisor;

int main() {
  uint64_t bad = 0, checked = 0;
  uint32_t x = 12345;
  auto rnd = [&]() {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
  };
  for (uint32_t d = 1; d <= 65536; ++d) {
    const Divisor v = lbmib::make_divisor(d);
    const uint32_t edges[] = {0u, 1u, d - 1, d, d + 1, 2 * d - 1, 2 * d, 0x7fffffffu, 0x7ffeffffu, 0xffffffffu};
    for (uint32_t n : edges) {
      ++checked;
      if (lbmib::divide(n, v) != n / d) ++bad;
    }
    for (int i = 0; i < 64; ++i) {
      const uint32_t n = rnd();
      ++checked;
      if (lbmib::divide(n, v) != n / d) ++bad;
    }
  }
  for (int i = 0; i < 2000000; ++i) {
    const uint32_t d = rnd() | 1u, n = rnd();
    ++checked;
    if (lbmib::divide(n, lbmib::make_divisor(d)) != n / d) ++bad;
  }
  std::printf("checked %llu quotients, %llu wrong\n", (unsigned long long)checked, (unsigned long long)bad);
  return bad ? 1 : 0;
}
