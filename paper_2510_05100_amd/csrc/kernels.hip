// Device kernels of the reweighting path (gfx950, wave64):
//   ingest_kernel  AoS [nevt][npart][4] -> SoA [npart*4][nevt] through LDS
//   launch_me      dispatch to the per-process matrix-element kernels
//                  (me_kernel.h, proc_<name>.hip)
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace rwgt {

constexpr int kIngestEvents = 64;

// One block moves kIngestEvents events: a coalesced read of their contiguous
// AoS rows into LDS, then one coalesced row write per SoA component.
template <int NPART>
__global__ __launch_bounds__(256) void ingest_kernel(const double* __restrict__ aos, double* __restrict__ soa,
                                                     int64_t nevt) {
  constexpr int W = NPART * 4;
  __shared__ double tile[kIngestEvents][W + 1];
  const int64_t e0 = int64_t(blockIdx.x) * kIngestEvents;
  const int64_t nloc = (nevt - e0) < kIngestEvents ? (nevt - e0) : kIngestEvents;
  const double* src = aos + e0 * W;
  for (int t = threadIdx.x; t < nloc * W; t += blockDim.x) tile[t / W][t % W] = src[t];
  __syncthreads();
  for (int t = threadIdx.x; t < kIngestEvents * W; t += blockDim.x) {
    const int c = t / kIngestEvents, e = t % kIngestEvents;
    if (e < nloc) soa[int64_t(c) * nevt + e0 + e] = tile[e][c];
  }
}

hipError_t launch_ingest(int npart, const double* aos, double* soa, int64_t nevt, hipStream_t s) {
  const int64_t blocks = (nevt + kIngestEvents - 1) / kIngestEvents;
  switch (npart) {
    case 4: hipLaunchKernelGGL(ingest_kernel<4>, dim3(unsigned(blocks)), dim3(256), 0, s, aos, soa, nevt); break;
    case 5: hipLaunchKernelGGL(ingest_kernel<5>, dim3(unsigned(blocks)), dim3(256), 0, s, aos, soa, nevt); break;
    case 6: hipLaunchKernelGGL(ingest_kernel<6>, dim3(unsigned(blocks)), dim3(256), 0, s, aos, soa, nevt); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_me(int proc, int precision, const double* soa, int64_t nevt, const CardPair* cards, int ncards,
                     const double* w_in, double* w_out, double* me_out, hipStream_t s) {
  switch (proc) {
    case kProcEeMumu: return launch_me_ee_mumu(precision, soa, nevt, cards, ncards, w_in, w_out, me_out, s);
    case kProcUuEeg: return launch_me_uu_eeg(precision, soa, nevt, cards, ncards, w_in, w_out, me_out, s);
    case kProcGgTtgg: return launch_me_gg_ttgg(precision, soa, nevt, cards, ncards, w_in, w_out, me_out, s);
  }
  return hipErrorInvalidValue;
}

void process_constants(int proc, int* npart, int* ngood, int* ncol, int* ndiag) {
  switch (proc) {
    case kProcEeMumu: constants_ee_mumu(npart, ngood, ncol, ndiag); break;
    case kProcUuEeg: constants_uu_eeg(npart, ngood, ncol, ndiag); break;
    case kProcGgTtgg: constants_gg_ttgg(npart, ngood, ncol, ndiag); break;
    default: *npart = *ngood = *ncol = *ndiag = 0;
  }
}

double process_flops(int proc) {
  switch (proc) {
    case kProcEeMumu: return flops_ee_mumu();
    case kProcUuEeg: return flops_uu_eeg();
    case kProcGgTtgg: return flops_gg_ttgg();
  }
  return 0.0;
}

}  // namespace rwgt
