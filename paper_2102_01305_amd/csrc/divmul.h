// Division by a per-solve constant as a multiply-high, for the wave indices
// the collide kernel splits (host side; plain C++).
#pragma once

namespace ibmk {

// Multiplier m with umulhi(n, m) = floor(n / d) for every 0 <= n < n_end:
// with m = floor(2^32 / d) + 1, n m / 2^32 = n / d + n (d - 2^32 mod d) / (d 2^32),
// and the second term stays below 1/d while n d < 2^32.  Returns 0 where that
// does not hold (or d < 2), and the kernel divides instead.
inline unsigned div_mul(unsigned long long d, unsigned long long n_end) {
  if (d < 2 || n_end * d >= (1ULL << 32)) return 0;
  return (unsigned)((1ULL << 32) / d + 1);
}

}  // namespace ibmk
