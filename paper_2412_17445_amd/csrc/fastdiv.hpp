// Division by a divisor that is fixed for a kernel launch, without the
// integer-division instruction sequence: q = (umulhi(n, m) + n) >> l with
// l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1 (round-up method
// of Granlund & Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994).  Exact for 0 <= n < 2^31 and 1 <= d < 2^31.
// The magic numbers are built on the host; the header also compiles as
// plain C++ so that the host test can check it against '/'.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define PFF_HD __host__ __device__
#else
#define PFF_HD
#endif

namespace pff {

struct FastDiv {
  uint32_t d, m, l;
};

inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while ((uint64_t(1) << l) < d) ++l;
  const uint64_t m = ((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1;
  return FastDiv{d, uint32_t(m), l};
}

PFF_HD inline uint32_t fdiv(uint32_t n, const FastDiv& f) {
  const uint32_t t = uint32_t((uint64_t(n) * f.m) >> 32);
  return (t + n) >> f.l;
}

// n mod d given the quotient q = n / d
PFF_HD inline uint32_t fmod_q(uint32_t n, uint32_t q, const FastDiv& f) { return n - q * f.d; }

}  // namespace pff
