// Batched form: many (process, card, event-range) segments in one persistent
// launch.  Workgroups claim fixed-size event tiles from a global counter until
// none are left (every workgroup exits once the counter passes the tile
// count), find the tile's segment by binary search over the segment table,
// and evaluate |M|^2 under the segment's original and new cards for each
// event of the tile: w' = (w * (1/|M|^2_orig)) * |M|^2_new.  Momenta are read
// in the caller's AoS layout ([nevt][npart][4]); no separate ingest pass.
#include <hip/hip_runtime.h>

#include "batch.h"
#include "check.h"
#include "generated/gen_ee_mumu.h"
#include "generated/gen_uu_eeg.h"
#include "me_kernel.h"

namespace rwgt {

RWGT_PROCESS_TRAITS(ee_mumu)
RWGT_PROCESS_TRAITS(uu_eeg)

template <class R, class PROC>
__device__ __forceinline__ void batch_event(const BatchSeg& sg, int64_t e, const CardPair& c0, const CardPair& c1) {
  constexpr int W = PROC::NPART * 4;
  double P[PROC::NPART][4];
#pragma unroll
  for (int a = 0; a < PROC::NPART; ++a)
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) P[a][mu] = RWGT_AT(sg.mom, e * W + a * 4 + mu, sg.nevt * W);
  const double m0 = me2_event<PROC, R>(P, pick<R>(c0));
  const double m1 = me2_event<PROC, R>(P, pick<R>(c1));
  RWGT_AT(sg.w_out, e, sg.nevt) = ((m0 == 0.0 ? 0.0 : 1.0 / m0) * RWGT_AT(sg.w_in, e, sg.nevt)) * m1;
}

template <class R, class... PROCS>
__device__ __forceinline__ void batch_dispatch(int proc, const BatchSeg& sg, int64_t e, const CardPair& c0,
                                               const CardPair& c1) {
  int idx = 0;
  ((proc == idx++ ? batch_event<R, PROCS>(sg, e, c0, c1) : void()), ...);
}

// One event on the 2 NGOOD consecutive lanes of a group (lane j of the
// group, the group's first lane at lane0 of the wave): lane j evaluates
// |M_h|^2 of helicity good(j % NGOOD) under c0 (j < NGOOD) or c1; the first
// lane gathers the group's values with shuffles, adds each card's in
// helicity order (the order of the one-lane-per-event kernels, so the result
// is the same to the bit) and writes w' = (w (1/|M|^2_0)) |M|^2_1.  Every lane
// of the group must call it.
template <class R, class PROC>
__device__ __forceinline__ void hel_group_event(const double* __restrict__ mom, int64_t e, int64_t nevt, int j,
                                                int lane0, const CardPair& c0, const CardPair& c1,
                                                const double* __restrict__ w_in, double* __restrict__ w_out) {
  constexpr int G = PROC::NGOOD;
  static_assert(PROC::NSUM == G, "every kept helicity is evaluated (no reversed-helicity weight)");
  double P[PROC::NPART][4];
#pragma unroll
  for (int a = 0; a < PROC::NPART; ++a)
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
      P[a][mu] = RWGT_AT(mom, e * (PROC::NPART * 4) + a * 4 + mu, nevt * (PROC::NPART * 4));
  cx<R> jamp[PROC::NCOL];
  PROC::template jamps<R>(P, PROC::good(j % G), pick<R>(j < G ? c0 : c1), jamp);
  const double hm = double(PROC::template colour_sum<R>(jamp));
  double m0 = 0.0, m1 = 0.0;
#pragma unroll
  for (int k = 0; k < G; ++k) {
    m0 += __shfl(hm, lane0 + k);
    m1 += __shfl(hm, lane0 + G + k);
  }
  if (j == 0) {
    m0 *= PROC::AVERAGE;
    m1 *= PROC::AVERAGE;
    RWGT_AT(w_out, e, nevt) = ((m0 == 0.0 ? 0.0 : 1.0 / m0) * RWGT_AT(w_in, e, nevt)) * m1;
  }
}

__global__ void batch_reset(unsigned long long* counter) { *counter = 0ull; }

template <class R, class... PROCS>
__global__ __launch_bounds__(256) void batch_kernel(const BatchSeg* __restrict__ segs, int nseg, int64_t ntiles,
                                                    int tile_events, const CardPair* __restrict__ cards,
                                                    unsigned long long* counter) {
  __shared__ long long s_tile;
  for (;;) {
    if (threadIdx.x == 0) s_tile = (long long)atomicAdd(counter, 1ull);
    __syncthreads();
    const int64_t tile = s_tile;
    __syncthreads();
    if (tile >= ntiles) return;
    int lo = 0, hi = nseg - 1;                 // last segment with tile0 <= tile
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (RWGT_AT(segs, mid, nseg).tile0 <= tile) lo = mid; else hi = mid - 1;
    }
    const BatchSeg sg = RWGT_AT(segs, lo, nseg);
    const int64_t e0 = (tile - sg.tile0) * tile_events;
    const int64_t e1 = e0 + tile_events < sg.nevt ? e0 + tile_events : sg.nevt;
    const CardPair& c0 = RWGT_AT(cards, 2 * lo, 2 * nseg);
    const CardPair& c1 = RWGT_AT(cards, 2 * lo + 1, 2 * nseg);
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) batch_dispatch<R, PROCS...>(sg.proc, sg, e, c0, c1);
  }
}

// The events of one tile of a segment of process PROC, one (event, card,
// helicity) per lane: 2 NGOOD lanes per event (the workgroup size is a
// multiple of 64, which 2 NGOOD divides).
template <class R, class PROC>
__device__ __forceinline__ void hel_tile(const BatchSeg& sg, int64_t e0, int64_t e1, const CardPair& c0,
                                         const CardPair& c1) {
  constexpr int G2 = 2 * PROC::NGOOD;
  static_assert(64 % G2 == 0, "event groups tile a wave");
  const int j = int(threadIdx.x) % G2;
  const int lane0 = int(threadIdx.x & 63) - j;
  for (int64_t e = e0 + threadIdx.x / G2; e < e1; e += blockDim.x / G2)
    hel_group_event<R, PROC>(sg.mom, e, sg.nevt, j, lane0, c0, c1, sg.w_in, sg.w_out);
}

// The persistent batch kernel with the helicity split: tiles claimed as in
// batch_kernel, each tile's events spread over (event, card, helicity) lanes.
template <class R, class... PROCS>
__global__ __launch_bounds__(256) void batch_hel_kernel(const BatchSeg* __restrict__ segs, int nseg, int64_t ntiles,
                                                        int tile_events, const CardPair* __restrict__ cards,
                                                        unsigned long long* counter) {
  __shared__ long long s_tile;
  for (;;) {
    if (threadIdx.x == 0) s_tile = (long long)atomicAdd(counter, 1ull);
    __syncthreads();
    const int64_t tile = s_tile;
    __syncthreads();
    if (tile >= ntiles) return;
    int lo = 0, hi = nseg - 1;                 // last segment with tile0 <= tile
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (RWGT_AT(segs, mid, nseg).tile0 <= tile) lo = mid; else hi = mid - 1;
    }
    const BatchSeg sg = RWGT_AT(segs, lo, nseg);
    const int64_t e0 = (tile - sg.tile0) * tile_events;
    const int64_t e1 = e0 + tile_events < sg.nevt ? e0 + tile_events : sg.nevt;
    const CardPair& c0 = RWGT_AT(cards, 2 * lo, 2 * nseg);
    const CardPair& c1 = RWGT_AT(cards, 2 * lo + 1, 2 * nseg);
    int idx = 0;
    ((sg.proc == idx++ ? hel_tile<R, PROCS>(sg, e0, e1, c0, c1) : void()), ...);
  }
}

template <class R, class... PROCS>
static hipError_t launch_batch_t(const BatchSeg* segs, int nseg, int64_t ntiles, const BatchSchedule& sc,
                                 const CardPair* cards, unsigned long long* counter, hipStream_t s) {
  hipLaunchKernelGGL(batch_reset, dim3(1), dim3(1), 0, s, counter);
  if (sc.hel_split)
    hipLaunchKernelGGL((batch_hel_kernel<R, PROCS...>), dim3(sc.grid), dim3(sc.block), 0, s, segs, nseg, ntiles,
                       sc.tile_events, cards, counter);
  else
    hipLaunchKernelGGL((batch_kernel<R, PROCS...>), dim3(sc.grid), dim3(sc.block), 0, s, segs, nseg, ntiles,
                       sc.tile_events, cards, counter);
  return hipGetLastError();
}

// Exact reweighting with a card per event (the surrogate's fallback list, or
// every event), one lane per (event, card, kept helicity): the 2 NGOOD lanes
// of an event are consecutive lanes of one wave; lane j evaluates |M_h|^2 of
// helicity good(j % NGOOD) under the original card cards[0] (j < NGOOD) or
// the event's card cards[1 + card_index[e]], and the group's first lane
// gathers them and adds each card's values in helicity order, the order of
// the one-lane-per-event kernels, so w' is the same to the bit.  One
// helicity and one card per lane keeps the registers to a few waves per
// SIMD, and a short fallback list still fills the chip.  Events
// list[0 .. *count) (the count stays on the device, at most n_all), or
// 0 .. n_all-1 without a list; grid-stride over events.  A card index
// outside [0, ncards) reads no card: the event's w' is NaN (the same
// decision on every lane of its group).
template <class R, class PROC>
__global__ __launch_bounds__(256) void exact_hel_kernel(const double* __restrict__ mom,
                                                        const int32_t* __restrict__ list,
                                                        const unsigned int* __restrict__ count, int64_t n_all,
                                                        const int32_t* __restrict__ card_index, int ncards,
                                                        const CardPair* __restrict__ cards,
                                                        const double* __restrict__ w_in, double* __restrict__ w_out) {
  constexpr int G2 = 2 * PROC::NGOOD;
  static_assert(64 % G2 == 0, "event groups tile a wave");
  const int64_t n = list ? (int64_t(*count) < n_all ? int64_t(*count) : n_all) : n_all;
  const int j = int(threadIdx.x) % G2;
  const int lane0 = int(threadIdx.x & 63) - j;             // the group's first lane in the wave
  const int64_t per_block = blockDim.x / G2;
  for (int64_t i = int64_t(blockIdx.x) * per_block + threadIdx.x / G2; i < n; i += int64_t(gridDim.x) * per_block) {
    const int64_t e = list ? int64_t(RWGT_AT(list, i, n_all)) : i;
    const int32_t k = RWGT_AT(card_index, e, n_all);
    if (k < 0 || k >= ncards) {
      if (j == 0) RWGT_AT(w_out, e, n_all) = __builtin_nan("");
      continue;
    }
    hel_group_event<R, PROC>(mom, e, n_all, j, lane0, RWGT_AT(cards, 0, ncards + 1), RWGT_AT(cards, 1 + k, ncards + 1),
                             w_in, w_out);
  }
}

template <class R>
static void launch_exact_hel(int proc, const double* mom, const int32_t* list, const unsigned int* count,
                             int64_t n_all, const int32_t* card_index, int ncards, const CardPair* cards,
                             const double* w_in, double* w_out, int max_blocks, hipStream_t s) {
  const int g = 2 * (proc == 0 ? Proc_ee_mumu::NGOOD : Proc_uu_eeg::NGOOD);   // lanes per event
  const int64_t need = (n_all * g + 255) / 256;
  const unsigned blocks = unsigned(need < max_blocks ? (need < 1 ? 1 : need) : max_blocks);
  if (proc == 0)
    hipLaunchKernelGGL((exact_hel_kernel<R, Proc_ee_mumu>), dim3(blocks), dim3(256), 0, s, mom, list, count, n_all,
                       card_index, ncards, cards, w_in, w_out);
  else
    hipLaunchKernelGGL((exact_hel_kernel<R, Proc_uu_eeg>), dim3(blocks), dim3(256), 0, s, mom, list, count, n_all,
                       card_index, ncards, cards, w_in, w_out);
}

hipError_t launch_exact_list(int family, int precision, int proc, const double* mom, const int32_t* list,
                             const unsigned int* count, int64_t n_all, const int32_t* card_index, int ncards,
                             const CardPair* cards, const double* w_in, double* w_out, int max_blocks,
                             hipStream_t s) {
  if (family != kFamilyElectroweak || (proc != 0 && proc != 1)) return hipErrorInvalidValue;
  if (n_all <= 0) return hipSuccess;
  if (precision == kPrecFP64)
    launch_exact_hel<double>(proc, mom, list, count, n_all, card_index, ncards, cards, w_in, w_out, max_blocks, s);
  else
    launch_exact_hel<float>(proc, mom, list, count, n_all, card_index, ncards, cards, w_in, w_out, max_blocks, s);
  return hipGetLastError();
}

hipError_t launch_batch(int family, int precision, const BatchSeg* segs, int nseg, int64_t ntiles,
                        const BatchSchedule& sc, const CardPair* cards, unsigned long long* counter,
                        hipStream_t s) {
  const bool f64 = precision == kPrecFP64;
  if (family == kFamilyElectroweak)
    return f64 ? launch_batch_t<double, Proc_ee_mumu, Proc_uu_eeg>(segs, nseg, ntiles, sc, cards, counter, s)
               : launch_batch_t<float, Proc_ee_mumu, Proc_uu_eeg>(segs, nseg, ntiles, sc, cards, counter, s);
  return hipErrorInvalidValue;
}

}  // namespace rwgt
