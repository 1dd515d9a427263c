// One-event-per-lane matrix-element kernel, shared by the per-process
// translation units (each instantiates it for its generated process).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include <type_traits>

#include "card.h"
#include "check.h"
#include "colour_mfma.h"
#include "kernels.h"

namespace rwgt {

#define RWGT_PROCESS_TRAITS(NAME)                                                              \
  struct Proc_##NAME {                                                                         \
    static constexpr int NPART = gen_##NAME::NPART;                                            \
    static constexpr int NCOL = gen_##NAME::NCOL;                                              \
    static constexpr int NGOOD = gen_##NAME::NGOOD;                                            \
    static constexpr double AVERAGE = gen_##NAME::AVERAGE;                                     \
    static constexpr int NSUM = gen_##NAME::NSUM;                                              \
    static constexpr double SCALE = gen_##NAME::AVERAGE * gen_##NAME::HELW;                    \
    static constexpr int CDEN = gen_##NAME::CDEN;                                              \
    static __device__ __forceinline__ const int (&cnum())[NCOL][NCOL] { return gen_##NAME::CNUM; } \
    static __device__ __forceinline__ int good(int i) { return gen_##NAME::GOOD[i]; }         \
    template <class R, class J>                                                                \
    static __device__ __forceinline__ void jamps(const double (&P)[NPART][4], int hel,         \
                                                 const Card<R>& cd, J& j) {                    \
      gen_##NAME::jamps<R, double>(P, hel, cd, j);                                             \
    }                                                                                          \
    template <class R, class J>                                                                \
    static __device__ __forceinline__ void jamps_grouped(const double (&P)[NPART][4], int hel, \
                                                         const Card<R>& cd, J& j) {            \
      gen_##NAME::jamps_grouped<R, double>(P, hel, cd, j);                                     \
    }                                                                                          \
    template <class R, class J>                                                                \
    static __device__ __forceinline__ R colour_sum(const J& j) {                               \
      return gen_##NAME::colour_sum<R>(j);                                                     \
    }                                                                                          \
  };

template <class R> __device__ __forceinline__ const Card<R>& pick(const CardPair& c);
template <> __device__ __forceinline__ const Card<double>& pick<double>(const CardPair& c) { return c.d; }
template <> __device__ __forceinline__ const Card<float>& pick<float>(const CardPair& c) { return c.f; }

// Colour-flow amplitudes of one lane kept in LDS, [NCOL][kMeBlock] so that
// the lanes of a wave touch consecutive addresses.
template <class R, int NCOL, int STRIDE = kMeBlock>
struct LdsJamp {
  cx<R>* base;
  __device__ __forceinline__ cx<R>& operator[](int c) { return base[c * STRIDE]; }
  __device__ __forceinline__ const cx<R>& operator[](int c) const { return base[c * STRIDE]; }
};

// Where a lane keeps its colour-flow amplitudes: registers, unless the
// process has many flows and the amplitudes are double (then LDS, which frees
// 4 * NCOL registers for the currents).
template <class PROC, class R>
constexpr bool jamp_in_lds() { return PROC::NCOL >= 8 && sizeof(R) == 8; }

// Colour-flow amplitudes of the guarded mixed path: the flows and the
// incoherent sum of the amplitude terms, sum_t m_t |amp_t|^2 (m_t: the number
// of flows term t enters).  Its ratio to the coherent sum_c |J_c|^2 measures
// how much the terms cancel in the flows, which is what amplifies their
// single-precision rounding.
template <class R, int NCOL>
struct GuardJamp {
  cx<R> j[NCOL];
  R inco;
  __device__ __forceinline__ cx<R>& operator[](int c) { return j[c]; }
  __device__ __forceinline__ const cx<R>& operator[](int c) const { return j[c]; }
};
template <class R, int NCOL>
__device__ __forceinline__ void note_reset(GuardJamp<R, NCOL>& g) { g.inco = R(0); }
template <class R, int NCOL>
__device__ __forceinline__ void note_amp(GuardJamp<R, NCOL>& g, const cx<R>& a, int m) {
  g.inco += R(m) * (a.re * a.re + a.im * a.im);
}
template <class R, int NCOL>
__device__ __forceinline__ cx<R> (&flows(GuardJamp<R, NCOL>& g))[NCOL] { return g.j; }
template <class R, int NCOL>
__device__ __forceinline__ cx<R> (&flows(cx<R> (&j)[NCOL]))[NCOL] { return j; }

// |M|^2 of one event under one card with the colour flows in registers and
// the colour sum on the VALU (the form of few-flow processes).
template <class PROC, class R>
__device__ __forceinline__ double me2_event(const double (&P)[PROC::NPART][4], const Card<R>& cd) {
  double me = 0.0;
  for (int ih = 0; ih < PROC::NSUM; ++ih) {
    cx<R> jamp[PROC::NCOL];
    PROC::template jamps<R>(P, PROC::good(ih), cd, jamp);
    me += double(PROC::template colour_sum<R>(jamp));
  }
  return me * PROC::SCALE;
}

// LDS of the matrix-core colour sum (one region per wave), or nothing.
template <class CT> struct ColourLdsOf { typedef ColourLds<CT> type; };
template <> struct ColourLdsOf<void> { typedef char type; };

// Helicities: the first NSUM of the kept ones, weighted by HELW (for pure QCD
// one of each pair with every helicity reversed, whose |M_h|^2 are equal,
// weight 2; otherwise all of them, weight 1); SCALE = AVERAGE * HELW.
// Waves per event group: the helicity sum of a many-flow process is split
// between the HS waves of a 64 HS-lane workgroup (consecutive blocks of
// helicities, each wave-uniform, added through LDS per card): HS times the
// waves, each HS times shorter, so the last round of waves leaves fewer
// SIMDs idle, and with wave-uniform loop bounds fewer registers spill.
// Few-flow processes keep one lane per event in 256-lane workgroups and the
// one-lane summation order, which their card-per-event and batched kernels
// reproduce bit for bit.  g g -> t t~ g g, 1e6 events: 161.4 ms with one
// wave, 152.9 ms with two (24 spilled registers instead of 54), 155.6 ms
// with four (56 spilled).
constexpr int kHelSplit = 2;
template <class PROC>
constexpr int hel_split() { return PROC::NCOL >= 8 ? kHelSplit : 1; }
template <class PROC>
constexpr int me_block() { return hel_split<PROC>() > 1 ? 64 * hel_split<PROC>() : kMeBlock; }

// One event per lane (of each wave of the helicity split).  R: amplitude
// precision.  CT: 16-bit type of the matrix-core colour sum (_Float16 or
// __bf16), or void for the VALU form.  GUARD (float amplitudes): also the
// cancellation measure kappa of each event, the largest over its cards of
// sum_hel sum_t m_t |amp_t|^2 / sum_hel sum_c |J_c|^2; events with kappa above
// g.kmax are appended to g.flagged.  INDEXED: row r of the launch is event
// g.rows[r] of the nevt-event arrays, for r < *g.nrows (the re-evaluation of
// flagged events in double precision).
template <class PROC, class R, class CT, bool GUARD = false, bool INDEXED = false>
__global__ __launch_bounds__(kMeBlock) void me_kernel(const double* __restrict__ soa, int64_t nevt,
                                                      const CardPair* __restrict__ cards, int ncards,
                                                      const double* __restrict__ w_in, double* __restrict__ w_out,
                                                      double* __restrict__ me_out, const GuardArgs g) {
  constexpr bool kMfma = !std::is_void<CT>::value;
  constexpr int HS = hel_split<PROC>(), B = me_block<PROC>();
  constexpr int EPB = HS > 1 ? 64 : B;                        // events per workgroup
  constexpr int NH = PROC::NSUM / HS;                         // helicities per wave
  static_assert(PROC::NSUM % HS == 0 && EPB % 64 == 0, "helicity split");
  static_assert(!GUARD || sizeof(R) == 4, "the guard watches single-precision amplitudes");
  // which helicities: wave-uniform, kept in a scalar register so that the
  // helicity of each loop trip stays uniform too
  const int half = HS > 1 ? __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6)) : 0;
  const int64_t r = int64_t(blockIdx.x) * EPB + (HS > 1 ? int(threadIdx.x & 63) : int(threadIdx.x));
  const int64_t nrows = INDEXED ? int64_t(*g.nrows) : nevt;
  // whole waves (split: whole workgroups) past the end leave together; inside
  // the last wave the lanes past the end recompute the last event (the
  // matrix-core colour sum needs every lane) and write nothing
  if constexpr (HS > 1) {
    if (int64_t(blockIdx.x) * EPB >= nrows) return;
  } else {
    if (int64_t(blockIdx.x) * B + (threadIdx.x & ~63) >= nrows) return;
  }
  const bool valid = r < nrows;
  const int64_t rr = valid ? r : nrows - 1;
  const int64_t i = INDEXED ? int64_t(RWGT_AT(g.rows, rr, nevt)) : rr;   // the event of this lane
  const int64_t ie = i;
  double P[PROC::NPART][4];
#pragma unroll
  for (int a = 0; a < PROC::NPART; ++a)
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) P[a][mu] = RWGT_AT(soa, int64_t(a * 4 + mu) * nevt + ie, PROC::NPART * 4 * nevt);

  [[maybe_unused]] __shared__ cx<R> lds_jamp[jamp_in_lds<PROC, R>() ? PROC::NCOL * B : 1];
  [[maybe_unused]] __shared__ typename ColourLdsOf<CT>::type lds_colour[kMfma ? B / 64 : 1];
  [[maybe_unused]] __shared__ double lds_half[HS > 1 ? 64 * (HS - 1) : 1];   // the other waves' partial sums
  [[maybe_unused]] __shared__ double lds_guard[GUARD && HS > 1 ? 2 * 64 * (HS - 1) : 1];
  [[maybe_unused]] std::conditional_t<kMfma, ColourMfma<PROC::NCOL, std::conditional_t<kMfma, CT, _Float16>>, char> cm;
  if constexpr (kMfma) cm.init(PROC::cnum(), lds_colour[threadIdx.x >> 6]);

  double norm = 0.0;
  [[maybe_unused]] double kappa = 0.0;
  for (int k = 0; k < ncards; ++k) {
    const Card<R>& cd = pick<R>(RWGT_AT(cards, k, ncards));
    double me = 0.0;
    [[maybe_unused]] double inco = 0.0, coh = 0.0;
    for (int ih = half * NH; ih < (half + 1) * NH; ++ih) {
      // The generated code reads the momenta through opq() at every use, so
      // none of the helicity-independent algebra is hoisted out of this loop.
      if constexpr (jamp_in_lds<PROC, R>()) {
        LdsJamp<R, PROC::NCOL, B> jamp{lds_jamp + threadIdx.x};
        PROC::template jamps_grouped<R>(P, PROC::good(ih), cd, jamp);
        me += double(PROC::template colour_sum<R>(jamp));
      } else {
        std::conditional_t<GUARD, GuardJamp<R, PROC::NCOL>, cx<R>[PROC::NCOL]> jamp;
        PROC::template jamps<R>(P, PROC::good(ih), cd, jamp);
        if constexpr (kMfma) {
          me += cm.sum(flows(jamp), lds_colour[threadIdx.x >> 6]) * (1.0 / PROC::CDEN);
        } else {
          me += double(PROC::template colour_sum<R>(jamp));
        }
        if constexpr (GUARD) {
          R c2 = R(0);
#pragma unroll
          for (int c = 0; c < PROC::NCOL; ++c) c2 += jamp[c].re * jamp[c].re + jamp[c].im * jamp[c].im;
          coh += double(c2);
          inco += double(jamp.inco);
        }
      }
    }
    if constexpr (HS > 1) {                      // the waves' partial sums in order, on the first wave
      if (half > 0) lds_half[(half - 1) * 64 + (threadIdx.x & 63)] = me;
      if constexpr (GUARD) {
        if (half > 0) {
          lds_guard[(half - 1) * 128 + (threadIdx.x & 63)] = inco;
          lds_guard[(half - 1) * 128 + 64 + (threadIdx.x & 63)] = coh;
        }
      }
      __syncthreads();
      if (half == 0)
        for (int w = 1; w < HS; ++w) me += lds_half[(w - 1) * 64 + threadIdx.x];
      if constexpr (GUARD) {
        if (half == 0)
          for (int w = 1; w < HS; ++w) {
            inco += lds_guard[(w - 1) * 128 + threadIdx.x];
            coh += lds_guard[(w - 1) * 128 + 64 + threadIdx.x];
          }
      }
      __syncthreads();                           // before the next card's partial sums
    }
    if constexpr (GUARD) {
      const double kk = coh > 0.0 ? inco / coh : (inco > 0.0 ? __builtin_inf() : 0.0);
      kappa = kk > kappa || !(kk == kk) ? kk : kappa;
    }
    me *= PROC::SCALE;                           // average (and the reversed helicities)
    if (!valid || half != 0) continue;
    if (me_out) RWGT_AT(me_out, int64_t(k) * nevt + i, int64_t(ncards) * nevt) = me;
    if (w_out) {
      if (k == 0) {
        norm = (me == 0.0 ? 0.0 : 1.0 / me) * RWGT_AT(w_in, i, nevt);
      } else {
        RWGT_AT(w_out, int64_t(k - 1) * nevt + i, int64_t(ncards - 1) * nevt) = norm * me;
      }
    }
  }
  if constexpr (GUARD) {
    if (valid && half == 0) {
      if (g.kappa) RWGT_AT(g.kappa, i, nevt) = kappa;
      if (g.flagged && !(kappa <= g.kmax)) RWGT_AT(g.flagged, atomicAdd(g.nflagged, 1u), nevt) = int32_t(i);
    }
  }
}

static __global__ void zero_count_kernel(unsigned int* c) { *c = 0u; }

// Double-precision re-evaluation of the events rows[0 .. *nrows) of a
// many-flow process, one wave per event (grid-stride over the list), one lane
// per evaluated helicity (the first NSUM kept ones): each lane evaluates its
// helicity's |M_h|^2 (flows in LDS) under every card, and lane 0 adds the
// lanes' values in me_kernel's order (the first half of the helicities in
// sequence, the second half in sequence, then their sum).  The per-helicity
// code is me_kernel's, but with the helicity per lane instead of per wave the
// compiler may round a last bit differently (measured: within 1 ulp of
// me_kernel's result).
// A short list keeps the chip busy for one helicity's evaluation per card,
// where one lane per event would take a whole helicity loop.
template <class PROC>
__global__ __launch_bounds__(64) void me_wave_kernel(const double* __restrict__ soa, int64_t nevt,
                                                     const CardPair* __restrict__ cards, int ncards,
                                                     const double* __restrict__ w_in, double* __restrict__ w_out,
                                                     double* __restrict__ me_out, const int32_t* __restrict__ rows,
                                                     const unsigned int* __restrict__ nrows) {
  constexpr int NG = PROC::NSUM;
  static_assert(NG <= 64 && hel_split<PROC>() == 2 && NG % 2 == 0, "one wave holds an event's helicities");
  __shared__ cx<double> lds_jamp[PROC::NCOL * 64];
  const int lane = int(threadIdx.x);
  const int ih = lane < NG ? lane : NG - 1;
  const int64_t n = int64_t(*nrows);
  for (int64_t r = blockIdx.x; r < n; r += gridDim.x) {
    const int64_t i = int64_t(RWGT_AT(rows, r, nevt));
    double P[PROC::NPART][4];
#pragma unroll
    for (int a = 0; a < PROC::NPART; ++a)
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) P[a][mu] = RWGT_AT(soa, int64_t(a * 4 + mu) * nevt + i, PROC::NPART * 4 * nevt);
    double norm = 0.0;
    for (int k = 0; k < ncards; ++k) {
      LdsJamp<double, PROC::NCOL, 64> jamp{lds_jamp + lane};
      PROC::template jamps_grouped<double>(P, PROC::good(ih), RWGT_AT(cards, k, ncards).d, jamp);
      const double hm = double(PROC::template colour_sum<double>(jamp));
      double m0 = 0.0, m1 = 0.0;
      for (int h = 0; h < NG / 2; ++h) m0 += __shfl(hm, h);
      for (int h = NG / 2; h < NG; ++h) m1 += __shfl(hm, h);
      double me = m0;
      me += m1;
      me *= PROC::SCALE;
      if (lane == 0) {
        if (me_out) RWGT_AT(me_out, int64_t(k) * nevt + i, int64_t(ncards) * nevt) = me;
        if (w_out) {
          if (k == 0) {
            norm = (me == 0.0 ? 0.0 : 1.0 / me) * RWGT_AT(w_in, i, nevt);
          } else {
            RWGT_AT(w_out, int64_t(k - 1) * nevt + i, int64_t(ncards - 1) * nevt) = norm * me;
          }
        }
      }
    }
  }
}

template <class PROC, class R, class CT, bool GUARD = false, bool INDEXED = false>
inline hipError_t launch_me_t(const double* soa, int64_t nevt, const CardPair* cards, int ncards,
                              const double* w_in, double* w_out, double* me_out, hipStream_t s,
                              const GuardArgs& g = GuardArgs{}) {
  constexpr int B = me_block<PROC>(), EPB = hel_split<PROC>() > 1 ? 64 : B;
  const int64_t blocks = (nevt + EPB - 1) / EPB;
  hipLaunchKernelGGL((me_kernel<PROC, R, CT, GUARD, INDEXED>), dim3(unsigned(blocks)), dim3(B), 0, s, soa, nevt,
                     cards, ncards, w_in, w_out, me_out, g);
  return hipGetLastError();
}

// Mixed precision with the cancellation guard: the float-amplitude kernel
// flags the events whose kappa exceeds g.kmax (g.kmax < 0: none, kappa only),
// then double precision re-evaluates the flagged events in place: one wave
// per event and a lane per helicity for many-flow processes (me_wave_kernel),
// else the one-lane-per-event kernel over the list (groups past the flagged
// count leave at once).
template <class PROC>
inline hipError_t launch_me_guarded_t(int precision, const double* soa, int64_t nevt, const CardPair* cards,
                                      int ncards, const double* w_in, double* w_out, double* me_out, GuardArgs g,
                                      hipStream_t s) {
  constexpr bool many = PROC::NCOL >= 8;
  if (g.nflagged) hipLaunchKernelGGL(zero_count_kernel, dim3(1), dim3(1), 0, s, g.nflagged);
  hipError_t e = precision == kPrecMixedBF16
      ? launch_me_t<PROC, float, std::conditional_t<many, __bf16, void>, true>(soa, nevt, cards, ncards, w_in, w_out,
                                                                               me_out, s, g)
      : launch_me_t<PROC, float, std::conditional_t<many, _Float16, void>, true>(soa, nevt, cards, ncards, w_in,
                                                                                 w_out, me_out, s, g);
  if (e != hipSuccess || g.kmax < 0.0 || !g.flagged || !g.nflagged) return e;
  if constexpr (hel_split<PROC>() > 1) {
    const int64_t blocks = nevt < 4096 ? nevt : 4096;
    hipLaunchKernelGGL(me_wave_kernel<PROC>, dim3(unsigned(blocks)), dim3(64), 0, s, soa, nevt, cards, ncards, w_in,
                       w_out, me_out, g.flagged, g.nflagged);
    return hipGetLastError();
  } else {
    GuardArgs gi;
    gi.rows = g.flagged;
    gi.nrows = g.nflagged;
    return launch_me_t<PROC, double, void, false, true>(soa, nevt, cards, ncards, w_in, w_out, me_out, s, gi);
  }
}

// Precision dispatch: FP64; or float amplitudes with the colour sum on the
// matrix cores (FP16 or BF16 split) for many-flow processes, on the VALU
// otherwise.
template <class PROC>
inline hipError_t launch_me_prec(int precision, const double* soa, int64_t nevt, const CardPair* cards, int ncards,
                                 const double* w_in, double* w_out, double* me_out, hipStream_t s) {
  constexpr bool many = PROC::NCOL >= 8;
  if (precision == kPrecFP64)
    return launch_me_t<PROC, double, void>(soa, nevt, cards, ncards, w_in, w_out, me_out, s);
  if (precision == kPrecMixedBF16)
    return launch_me_t<PROC, float, std::conditional_t<many, __bf16, void>>(soa, nevt, cards, ncards, w_in, w_out,
                                                                             me_out, s);
  return launch_me_t<PROC, float, std::conditional_t<many, _Float16, void>>(soa, nevt, cards, ncards, w_in, w_out,
                                                                             me_out, s);
}


}  // namespace rwgt
