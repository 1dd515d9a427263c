// Training order of the surrogate: a pseudo-random permutation of the pairs
// [0, n) for each (seed, epoch), evaluated independently per position on the
// host and on the device (no sort, no state).
//
// A four-round balanced Feistel network on words of 2h bits (2^(2h) >= n, so
// at most 4n) whose round function is SplitMix64's output mixer (Steele, Lea
// and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014)
// of the right half XOR a round key derived from seed, epoch and round.  A
// Feistel network is a bijection of its word space for any round function;
// positions whose image lies at or beyond n are passed through it again until
// they land in [0, n) (cycle walking: Black and Rogaway, "Ciphers with
// arbitrary finite domains", CT-RSA 2002), which restricts it to a bijection
// of [0, n).  Each walk step lands in [0, n) with probability at least 1/4, so
// the 1024-step cap is never reached in practice.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rwgt {

struct Shuffle {
  uint64_t key = 0;
  uint64_t mask = 0;      // 2^h - 1
  int64_t n = 0;          // domain size; 0 means identity order
  int half = 1;           // h
};

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

constexpr uint64_t kGolden64 = 0x9e3779b97f4a7c15ULL;   // 2^64 / golden ratio, SplitMix64's increment

inline Shuffle make_shuffle(uint64_t seed, int64_t epoch, int64_t n) {
  Shuffle s;
  int bits = 2;
  while (bits < 62 && (int64_t(1) << bits) < n) ++bits;
  if (bits & 1) ++bits;
  s.half = bits / 2;
  s.mask = (uint64_t(1) << s.half) - 1;
  s.n = n;
  s.key = mix64(seed ^ mix64(uint64_t(epoch) + kGolden64));
  return s;
}

__host__ __device__ inline uint64_t feistel(const Shuffle& s, uint64_t x) {
  uint64_t l = x >> s.half, r = x & s.mask;
  for (int k = 0; k < 4; ++k) {
    const uint64_t f = mix64(r ^ (s.key + uint64_t(k + 1) * kGolden64)) & s.mask;
    const uint64_t t = l ^ f;
    l = r;
    r = t;
  }
  return (l << s.half) | r;
}

// The pair at position pos (0 <= pos < n) of the epoch's order.
__host__ __device__ inline int64_t shuffled(const Shuffle& s, int64_t pos) {
  if (s.n == 0) return pos;
  uint64_t x = uint64_t(pos);
  for (int it = 0; it < 1024; ++it) {
    x = feistel(s, x);
    if (x < uint64_t(s.n)) return int64_t(x);
  }
  return pos;
}

}  // namespace rwgt
