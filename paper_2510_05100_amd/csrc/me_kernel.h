// One-event-per-lane matrix-element kernel, shared by the per-process
// translation units (each instantiates it for its generated process).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "card.h"
#include "kernels.h"

namespace rwgt {

#define RWGT_PROCESS_TRAITS(NAME)                                                              \
  struct Proc_##NAME {                                                                         \
    static constexpr int NPART = gen_##NAME::NPART;                                            \
    static constexpr int NCOL = gen_##NAME::NCOL;                                              \
    static constexpr int NGOOD = gen_##NAME::NGOOD;                                            \
    static constexpr double AVERAGE = gen_##NAME::AVERAGE;                                     \
    static __device__ __forceinline__ int good(int i) { return gen_##NAME::GOOD[i]; }         \
    template <class R>                                                                         \
    static __device__ __forceinline__ void jamps(const double (&P)[NPART][4], int hel,         \
                                                 const Card<R>& cd, cx<R> (&j)[NCOL]) {        \
      gen_##NAME::jamps<R, double>(P, hel, cd, j);                                                     \
    }                                                                                          \
    template <class R>                                                                         \
    static __device__ __forceinline__ R colour_sum(const cx<R> (&j)[NCOL]) {                   \
      return gen_##NAME::colour_sum<R>(j);                                                     \
    }                                                                                          \
  };

template <class R> __device__ __forceinline__ const Card<R>& pick(const CardPair& c);
template <> __device__ __forceinline__ const Card<double>& pick<double>(const CardPair& c) { return c.d; }
template <> __device__ __forceinline__ const Card<float>& pick<float>(const CardPair& c) { return c.f; }

template <class PROC, class R>
__global__ __launch_bounds__(kMeBlock) void me_kernel(const double* __restrict__ soa, int64_t nevt,
                                                      const CardPair* __restrict__ cards, int ncards,
                                                      const double* __restrict__ w_in, double* __restrict__ w_out,
                                                      double* __restrict__ me_out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nevt) return;
  double P[PROC::NPART][4];
#pragma unroll
  for (int a = 0; a < PROC::NPART; ++a)
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) P[a][mu] = soa[int64_t(a * 4 + mu) * nevt + i];

  double norm = 0.0;
  for (int k = 0; k < ncards; ++k) {
    const Card<R>& cd = pick<R>(cards[k]);
    double me = 0.0;
    for (int ih = 0; ih < PROC::NGOOD; ++ih) {
      // Momentum sums and propagator denominators do not depend on the
      // helicity; left to itself the compiler hoists all of them out of this
      // loop and keeps them live across it, which spills.  Re-defining the
      // momenta opaquely here keeps that algebra inside the iteration.
      double Ph[PROC::NPART][4];
#pragma unroll
      for (int a = 0; a < PROC::NPART; ++a)
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
          Ph[a][mu] = P[a][mu];
          asm volatile("" : "+v"(Ph[a][mu]));
        }
      cx<R> jamp[PROC::NCOL];
      PROC::template jamps<R>(Ph, PROC::good(ih), cd, jamp);
      me += double(PROC::template colour_sum<R>(jamp));
    }
    me *= PROC::AVERAGE;
    if (me_out) me_out[int64_t(k) * nevt + i] = me;
    if (w_out) {
      if (k == 0) {
        norm = (me == 0.0 ? 0.0 : 1.0 / me) * w_in[i];
      } else {
        w_out[int64_t(k - 1) * nevt + i] = norm * me;
      }
    }
  }
}

template <class PROC, class R>
inline hipError_t launch_me_t(const double* soa, int64_t nevt, const CardPair* cards, int ncards,
                              const double* w_in, double* w_out, double* me_out, hipStream_t s) {
  const int64_t blocks = (nevt + kMeBlock - 1) / kMeBlock;
  hipLaunchKernelGGL((me_kernel<PROC, R>), dim3(unsigned(blocks)), dim3(kMeBlock), 0, s, soa, nevt, cards, ncards,
                     w_in, w_out, me_out);
  return hipGetLastError();
}


}  // namespace rwgt
