// Bounds checks of the device code, compiled in by the check build
// (-DRWGT_CHECK, librwgt_check.so) and compiled away otherwise.
//
// RWGT_AT(p, i, n) is the element p[i] of an array of n elements.  In the
// check build an index outside [0, n) is counted in a device counter of the
// translation unit, and the access goes to a small sink array instead, so a
// wrong index is reported without touching memory outside the arrays (reads
// then return whatever the sink holds).  rwgt_bounds_check() adds and clears
// the counters of every translation unit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace rwgt {

// Host side: each checked translation unit registers a function that reads
// and clears its device counter (the registry is in rwgt_abi.cpp, which
// includes this header with RWGT_CHECK_REGISTRY_ONLY).
typedef unsigned long long (*BoundsReader)();
void register_bounds_reader(BoundsReader f);
std::vector<BoundsReader>& bounds_readers();

#if defined(RWGT_CHECK) && !defined(RWGT_CHECK_REGISTRY_ONLY)

namespace {
__device__ unsigned int g_bounds_miss;
constexpr int kBoundsSink = 4096;
__device__ __align__(256) unsigned char g_bounds_sink[kBoundsSink];

unsigned long long read_bounds_misses() {
  unsigned int v = 0;
  if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_bounds_miss), sizeof v) != hipSuccess) return ~0ull;
  const unsigned int zero = 0;
  if (hipMemcpyToSymbol(HIP_SYMBOL(g_bounds_miss), &zero, sizeof zero) != hipSuccess) return ~0ull;
  return v;
}

struct BoundsRegistration {
  BoundsRegistration() { register_bounds_reader(&read_bounds_misses); }
};
BoundsRegistration g_bounds_registration;
}  // namespace

template <class T>
__device__ __forceinline__ T& bounds_at(T* p, int64_t i, int64_t n) {
  static_assert(sizeof(T) <= kBoundsSink, "sink too small for the element type");
  if (i < 0 || i >= n) {
    atomicAdd(&g_bounds_miss, 1u);
    return *reinterpret_cast<T*>(g_bounds_sink);
  }
  return p[i];
}

#define RWGT_AT(p, i, n) (::rwgt::bounds_at((p), int64_t(i), int64_t(n)))
constexpr bool kBoundsChecked = true;

#else

#define RWGT_AT(p, i, n) ((p)[i])
constexpr bool kBoundsChecked = false;

#endif

}  // namespace rwgt
