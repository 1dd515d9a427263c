// Device kernels of the reweighting path (gfx950, wave64):
//   ingest_kernel  AoS [nevt][npart][4] -> SoA [npart*4][nevt] through LDS
//   launch_me      dispatch to the per-process matrix-element kernels
//                  (me_kernel.h, proc_<name>.hip)
//   xsec_*         reweighted cross sections and errors per card
//   factored       coupling-factored reweighting of many cards
#include <hip/hip_runtime.h>

#include <cstdint>

#include "check.h"
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
  for (int t = threadIdx.x; t < nloc * W; t += blockDim.x) tile[t / W][t % W] = RWGT_AT(aos, e0 * W + t, nevt * W);
  __syncthreads();
  for (int t = threadIdx.x; t < kIngestEvents * W; t += blockDim.x) {
    const int c = t / kIngestEvents, e = t % kIngestEvents;
    if (e < nloc) RWGT_AT(soa, int64_t(c) * nevt + e0 + e, nevt * W) = tile[e][c];
  }
}

// Reweighted cross sections (teaRex section): per card the sums
// S1 = sum w' and R = sum w'/w (terms with w = 0 count 0), then, around the
// mean m = S1/N, S2 = sum (w' - m)^2, each reduced in a fixed order (block
// partials, then one lane per card), so results are deterministic:
//   sigma' = C S1,  dsigma' = dsigma R/N + sigma std(w'),  std = sqrt(S2/N),
// and, when dsigma' is infinite, NaN or not positive, dsigma' = dsigma max(sigma'/sigma, sigma/sigma').
// The variance is taken about the mean (two passes) because for near-constant
// w' (a pure alpha_s change) S2/N - m^2 cancels to noise of order 1e-16 m^2.
constexpr int kXsecBlock = 256;

template <int Q>
__device__ void block_sum(double (&sh)[Q][kXsecBlock], const double (&v)[Q], double* __restrict__ dst) {
#pragma unroll
  for (int q = 0; q < Q; ++q) sh[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int w = kXsecBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int q = 0; q < Q; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < Q) dst[threadIdx.x] = sh[threadIdx.x][0];
}

// Pass 1: block partials of S1 and R -> part[k][block][2].
__global__ __launch_bounds__(kXsecBlock) void xsec_pass1(const double* __restrict__ w_in,
                                                         const double* __restrict__ w_out, int64_t nevt,
                                                         double* __restrict__ part) {
  __shared__ double sh[2][kXsecBlock];
  const int k = blockIdx.y;
  const int64_t nw = int64_t(gridDim.y) * nevt;            // w_out: [nsets][nevt], nsets = gridDim.y
  double v[2] = {0.0, 0.0};
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nevt; i += int64_t(gridDim.x) * blockDim.x) {
    const double x = RWGT_AT(w_out, int64_t(k) * nevt + i, nw);
    const double wi = RWGT_AT(w_in, i, nevt);
    v[0] += x;
    v[1] += wi != 0.0 ? x / wi : 0.0;
  }
  block_sum<2>(sh, v, part + (int64_t(k) * gridDim.x + blockIdx.x) * 2);
}

// One lane per card: S1, R from pass 1 -> sums[k] = {S1, R, S1/N}.
__global__ __launch_bounds__(64) void xsec_mean(const double* __restrict__ part, int nblocks, int64_t nevt,
                                                int nsets, double* __restrict__ sums) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nsets) return;
  double s1 = 0.0, r = 0.0;
  const int64_t np = int64_t(nsets) * nblocks * 2;
  for (int b = 0; b < nblocks; ++b) {
    s1 += RWGT_AT(part, (int64_t(k) * nblocks + b) * 2, np);
    r += RWGT_AT(part, (int64_t(k) * nblocks + b) * 2 + 1, np);
  }
  RWGT_AT(sums, k * 3 + 0, nsets * 3) = s1;
  RWGT_AT(sums, k * 3 + 1, nsets * 3) = r;
  RWGT_AT(sums, k * 3 + 2, nsets * 3) = s1 / double(nevt);
}

// Pass 2: block partials of sum (w' - m)^2 -> part2[k][block].
__global__ __launch_bounds__(kXsecBlock) void xsec_pass2(const double* __restrict__ w_out, int64_t nevt,
                                                         const double* __restrict__ sums,
                                                         double* __restrict__ part2) {
  __shared__ double sh[1][kXsecBlock];
  const int k = blockIdx.y;
  const int64_t nw = int64_t(gridDim.y) * nevt;
  const double m = RWGT_AT(sums, k * 3 + 2, int64_t(gridDim.y) * 3);
  double v[1] = {0.0};
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nevt; i += int64_t(gridDim.x) * blockDim.x) {
    const double d = RWGT_AT(w_out, int64_t(k) * nevt + i, nw) - m;
    v[0] += d * d;
  }
  block_sum<1>(sh, v, part2 + int64_t(k) * gridDim.x + blockIdx.x);
}

__global__ __launch_bounds__(64) void xsec_final(const double* __restrict__ sums, const double* __restrict__ part2,
                                                 int nblocks, int64_t nevt, int nsets, double sigma, double dsigma,
                                                 double norm, double* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nsets) return;
  double s2 = 0.0;
  for (int b = 0; b < nblocks; ++b) s2 += RWGT_AT(part2, int64_t(k) * nblocks + b, int64_t(nsets) * nblocks);
  const double n = double(nevt);
  const double xs = norm * RWGT_AT(sums, k * 3 + 0, nsets * 3);
  double err = dsigma * (RWGT_AT(sums, k * 3 + 1, nsets * 3) / n) + sigma * sqrt(s2 / n);
  double fallback = 0.0;
  if (!(err > 0.0) || isinf(err)) {
    const double a = xs / sigma, b = sigma / xs;
    err = dsigma * (a > b ? a : b);
    fallback = 1.0;
  }
  RWGT_AT(out, k * 3 + 0, nsets * 3) = xs;
  RWGT_AT(out, k * 3 + 1, nsets * 3) = err;
  RWGT_AT(out, k * 3 + 2, nsets * 3) = fallback;
}

hipError_t launch_xsec(const double* w_in, const double* w_out, int64_t nevt, int nsets, double sigma, double dsigma,
                       double norm, double* part, int nblocks, double* out, hipStream_t s) {
  // part: [nsets][nblocks][2] pass-1 partials, then [nsets][3] sums, then [nsets][nblocks] pass-2 partials.
  double* sums = part + size_t(nsets) * nblocks * 2;
  double* part2 = sums + size_t(nsets) * 3;
  const int lanes = (nsets + 63) / 64;
  hipLaunchKernelGGL(xsec_pass1, dim3(nblocks, nsets), dim3(kXsecBlock), 0, s, w_in, w_out, nevt, part);
  hipLaunchKernelGGL(xsec_mean, dim3(lanes), dim3(64), 0, s, part, nblocks, nevt, nsets, sums);
  hipLaunchKernelGGL(xsec_pass2, dim3(nblocks, nsets), dim3(kXsecBlock), 0, s, w_out, nevt, sums, part2);
  hipLaunchKernelGGL(xsec_final, dim3(lanes), dim3(64), 0, s, sums, part2, nblocks, nevt, nsets, sigma, dsigma, norm,
                     out);
  return hipGetLastError();
}

// Coupling-factored reweighting.  Electroweak family: every kept helicity
// amplitude is K_h(p) F_chi(card, s), chi the chirality class (LL, LR, RL, RR)
// of the two fermion lines, s the invariant mass of the resonant pair and
//   F_chi = A / s + B_chi / (s - M_Z^2 + i M_Z Gamma_Z)
// (A: product of the lines' photon couplings, B_chi: of their Z couplings),
// so |M|^2 = g sum_chi W_chi |F_chi|^2.  The class weights W_chi of an event
// come from four probe cards (Z couplings 1 on one class, all others 0):
// W_chi = |M|^2_probe,chi |s - M_p^2 + i M_p Gamma_p|^2.  QCD family (cards
// change alpha_s only): |M|^2 = g |M|^2_probe with g = (g_s / g_s,0)^8.
// Card 0 is the original card; w_out[k-1][i] = (w_in[i] / |M|^2_0) |M|^2_k.
template <bool EW>
__global__ __launch_bounds__(256) void factored_kernel(const double* __restrict__ soa, int64_t nsoa, int64_t nevt,
                                                       int ia, int ib,
                                                       const double* __restrict__ probe, double mzp, double wzp,
                                                       const FactorCard* __restrict__ fc, int ncards,
                                                       const double* __restrict__ w_in, double* __restrict__ w_out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nevt) return;
  double W[4] = {0.0, 0.0, 0.0, 0.0};
  double s = 0.0;
  if constexpr (EW) {
    double pa[4], pb[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      pa[mu] = RWGT_AT(soa, int64_t(ia * 4 + mu) * nevt + i, nsoa);
      pb[mu] = RWGT_AT(soa, int64_t(ib * 4 + mu) * nevt + i, nsoa);
    }
    s = 2.0 * (pa[0] * pb[0] - pa[1] * pb[1] - pa[2] * pb[2] - pa[3] * pb[3]);
    const double xp = s - mzp * mzp, yp = mzp * wzp;
    const double dp = xp * xp + yp * yp;
#pragma unroll
    for (int c = 0; c < 4; ++c) W[c] = RWGT_AT(probe, int64_t(c) * nevt + i, 4 * nevt) * dp;
  } else {
    W[0] = RWGT_AT(probe, i, nevt);
  }
  auto me2 = [&](const FactorCard& k) {
    if constexpr (EW) {
      const double x = s - k.mz * k.mz, y = k.mz * k.wz;
      const double d = x * x + y * y;
      const double ga = k.A / s, gr = x / d, gi = -y / d;
      double sum = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double re = ga + k.B[c] * gr, im = k.B[c] * gi;
        sum += W[c] * (re * re + im * im);
      }
      return k.g * sum;
    } else {
      return k.g * W[0];
    }
  };
  const double m0 = me2(RWGT_AT(fc, 0, ncards));
  const double norm = m0 != 0.0 ? RWGT_AT(w_in, i, nevt) * (1.0 / m0) : 0.0;
  for (int k = 1; k < ncards; ++k)
    RWGT_AT(w_out, int64_t(k - 1) * nevt + i, int64_t(ncards - 1) * nevt) = norm * me2(RWGT_AT(fc, k, ncards));
}

hipError_t launch_factored(bool ew, const double* soa, int npart, int64_t nevt, int ia, int ib, const double* probe,
                           double mzp, double wzp, const FactorCard* fc, int ncards, const double* w_in,
                           double* w_out, hipStream_t s) {
  if (nevt <= 0) return hipSuccess;
  const unsigned blocks = unsigned((nevt + 255) / 256);
  const int64_t nsoa = int64_t(npart) * 4 * nevt;
  if (ew)
    hipLaunchKernelGGL(factored_kernel<true>, dim3(blocks), dim3(256), 0, s, soa, nsoa, nevt, ia, ib, probe, mzp, wzp,
                       fc, ncards, w_in, w_out);
  else
    hipLaunchKernelGGL(factored_kernel<false>, dim3(blocks), dim3(256), 0, s, soa, nsoa, nevt, ia, ib, probe, mzp, wzp,
                       fc, ncards, w_in, w_out);
  return hipGetLastError();
}

// Per-event strong coupling on top of the fixed-coupling weights: every
// diagram of these processes carries the same power p of g_s, so |M|^2 under
// alpha_s(event) is |M|^2 under the card's alpha_s times (alpha_s(event) /
// alpha_s(card))^p.  The original uses the event's own alpha_s (or the
// original card's run to the event scale); card k its alpha_s run to the
// event scale at one loop: a(mu) = a / (1 + a b0 ln(mu^2 / m_ref^2)).
__device__ __forceinline__ double run_alphas(double a, double mu, double b0, double mref2) {
  return a / (1.0 + a * b0 * log(mu * mu / mref2));
}

__global__ __launch_bounds__(256) void alphas_kernel(double* __restrict__ w_out, int64_t nevt, int nsets,
                                                     const double* __restrict__ alphas_orig,
                                                     const double* __restrict__ scales, double as0,
                                                     const double* __restrict__ as_cards, int p, double b0,
                                                     double mref2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nevt) return;
  const double mu = RWGT_AT(scales, i, nevt);
  const double a0 = alphas_orig ? RWGT_AT(alphas_orig, i, nevt) : run_alphas(as0, mu, b0, mref2);
  const bool zero = a0 == 0.0;             // |M|^2 of the original is 0: w' = 0
  const double r0 = zero ? 0.0 : as0 / a0;
  for (int k = 0; k < nsets; ++k) {
    const double ak = RWGT_AT(as_cards, k, nsets);
    const double rk = ak != 0.0 ? run_alphas(ak, mu, b0, mref2) / ak : 1.0;
    double f = 1.0, x = rk * r0;
    for (int q = 0; q < p; ++q) f *= x;
    double& w = RWGT_AT(w_out, int64_t(k) * nevt + i, int64_t(nsets) * nevt);
    w = zero ? 0.0 : w * f;
  }
}

hipError_t launch_alphas(double* w_out, int64_t nevt, int nsets, const double* alphas_orig, const double* scales,
                         double as0, const double* as_cards, int p, double b0, double mref2, hipStream_t s) {
  if (nevt <= 0) return hipSuccess;
  hipLaunchKernelGGL(alphas_kernel, dim3(unsigned((nevt + 255) / 256)), dim3(256), 0, s, w_out, nevt, nsets,
                     alphas_orig, scales, as0, as_cards, p, b0, mref2);
  return hipGetLastError();
}

// Count of the non-finite outputs of a call: a grid-stride pass, each wave
// sums its lanes' counts with shuffles, the block's four wave sums meet in
// LDS and thread 0 writes the block total (no atomics, nothing to clear).
__global__ __launch_bounds__(256) void nonfinite_kernel(const double* __restrict__ x, int64_t n,
                                                        unsigned long long* __restrict__ part) {
  __shared__ unsigned long long wsum[4];
  unsigned long long c = 0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    c += isfinite(RWGT_AT(x, i, n)) ? 0 : 1;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) RWGT_AT(part, blockIdx.x, gridDim.x) = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

int nonfinite_blocks(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return int(b < kNonfiniteBlocks ? (b < 1 ? 1 : b) : kNonfiniteBlocks);
}

hipError_t launch_nonfinite(const double* x, int64_t n, unsigned long long* part, hipStream_t s) {
  hipLaunchKernelGGL(nonfinite_kernel, dim3(unsigned(nonfinite_blocks(n))), dim3(256), 0, s, x, n, part);
  return hipGetLastError();
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
    case kProcGgTttt: return launch_me_gg_tttt(precision, soa, nevt, cards, ncards, w_in, w_out, me_out, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_me_guarded(int proc, int precision, const double* soa, int64_t nevt, const CardPair* cards,
                             int ncards, const double* w_in, double* w_out, double* me_out, const GuardArgs& g,
                             hipStream_t s) {
  switch (proc) {
    case kProcEeMumu: return launch_me_guarded_ee_mumu(precision, soa, nevt, cards, ncards, w_in, w_out, me_out, g, s);
    case kProcUuEeg: return launch_me_guarded_uu_eeg(precision, soa, nevt, cards, ncards, w_in, w_out, me_out, g, s);
    case kProcGgTtgg:
      return launch_me_guarded_gg_ttgg(precision, soa, nevt, cards, ncards, w_in, w_out, me_out, g, s);
    case kProcGgTttt:
      return launch_me_guarded_gg_tttt(precision, soa, nevt, cards, ncards, w_in, w_out, me_out, g, s);
  }
  return hipErrorInvalidValue;
}

void process_constants(int proc, int* npart, int* ngood, int* ncol, int* ndiag) {
  switch (proc) {
    case kProcEeMumu: constants_ee_mumu(npart, ngood, ncol, ndiag); break;
    case kProcUuEeg: constants_uu_eeg(npart, ngood, ncol, ndiag); break;
    case kProcGgTtgg: constants_gg_ttgg(npart, ngood, ncol, ndiag); break;
    case kProcGgTttt: constants_gg_tttt(npart, ngood, ncol, ndiag); break;
    default: *npart = *ngood = *ncol = *ndiag = 0;
  }
}

double process_flops(int proc, bool executed) {
  switch (proc) {
    case kProcEeMumu: return flops_ee_mumu(executed);
    case kProcUuEeg: return flops_uu_eeg(executed);
    case kProcGgTtgg: return flops_gg_ttgg(executed);
    case kProcGgTttt: return flops_gg_tttt(executed);
  }
  return 0.0;
}

}  // namespace rwgt
