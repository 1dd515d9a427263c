// Internal launch interface between the C-ABI host code and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "card.h"

namespace rwgt {

enum { kProcEeMumu = 0, kProcUuEeg = 1, kProcGgTtgg = 2, kProcGgTttt = 3 };
enum { kPrecFP64 = 0, kPrecMixedFP16 = 1, kPrecMixedBF16 = 2 };
constexpr int kMeBlock = 256;

hipError_t launch_ingest(int npart, const double* aos, double* soa, int64_t nevt, hipStream_t s);

// cards[0..ncards): |M|^2 per card -> me_out[k][nevt] (if non-null); when
// w_out is non-null, card 0 is the original card and
// w_out[k-1][i] = (w_in[i] * (1/|M|^2_0)) * |M|^2_k for k >= 1.
hipError_t launch_me(int proc, int precision, const double* soa, int64_t nevt, const CardPair* cards, int ncards,
                     const double* w_in, double* w_out, double* me_out, hipStream_t s);

// Default threshold of the mixed path's cancellation guard: measured on 4e6
// g g -> t t~ g g events (FP16 colour sum), it re-evaluates 0.10 % of them and
// leaves a largest w' error of 3.6e-6 (none: 6.9e-6); on 1e6 u u~ -> e+ e- g
// events 0.13 % and 2.3e-6 on w', 4.1e-6 on |M|^2 (none: 6.0e-5).
constexpr double kGuardKappaDefault = 300.0;

// Cancellation guard of the mixed path (me_kernel.h, launch_me_guarded).
struct GuardArgs {
  const int32_t* rows = nullptr;          // re-evaluation: the event of each row
  const unsigned int* nrows = nullptr;    // re-evaluation: number of rows (device)
  int32_t* flagged = nullptr;             // guard: events to re-evaluate (capacity nevt)
  unsigned int* nflagged = nullptr;       // guard: their count (device)
  double kmax = 0.0;                      // guard: kappa above this is flagged (< 0: flag nothing)
  double* kappa = nullptr;                // guard (optional): kappa of each event
};

// Mixed-precision |M|^2 / w' (precision RWGT_MIXED_*) with the events whose
// cancellation measure exceeds g.kmax re-evaluated in double precision.
hipError_t launch_me_guarded(int proc, int precision, const double* soa, int64_t nevt, const CardPair* cards,
                             int ncards, const double* w_in, double* w_out, double* me_out, const GuardArgs& g,
                             hipStream_t s);

// Reweighted cross sections and errors per card: out[k] = {sigma', dsigma', fallback flag};
// part must hold nsets * (3 * nblocks + 3) doubles (two-pass scratch).
hipError_t launch_xsec(const double* w_in, const double* w_out, int64_t nevt, int nsets, double sigma, double dsigma,
                       double norm, double* part, int nblocks, double* out, hipStream_t s);

// One card of the coupling-factored path (kernels.hip, factored_kernel).
struct FactorCard {
  double A;        // product of the two fermion lines' photon couplings
  double B[4];     // products of their Z couplings: LL, LR, RL, RR
  double mz, wz;   // Z mass and width
  double g;        // overall factor relative to the probe cards
};

// w_out[k-1][i] for cards fc[1..ncards) against fc[0] from the probe |M|^2
// (ew: [4][nevt] class probes and the resonant pair (ia, ib); else [1][nevt]).
// soa: [npart * 4][nevt].
hipError_t launch_factored(bool ew, const double* soa, int npart, int64_t nevt, int ia, int ib, const double* probe,
                           double mzp, double wzp, const FactorCard* fc, int ncards, const double* w_in,
                           double* w_out, hipStream_t s);

// w_out[k][i] *= (alpha_k(mu_i)/alpha_k)^p (alpha_0/alpha_0(i))^p (per-event strong coupling).
hipError_t launch_alphas(double* w_out, int64_t nevt, int nsets, const double* alphas_orig, const double* scales,
                         double as0, const double* as_cards, int p, double b0, double mref2, hipStream_t s);

// Non-finite entries (NaN, +-inf) of x[0..n): block b of the launch writes
// its count to part[b]; the launch uses nonfinite_blocks(n) blocks (at most
// kNonfiniteBlocks), so part needs that many entries.
constexpr int kNonfiniteBlocks = 1024;
int nonfinite_blocks(int64_t n);
hipError_t launch_nonfinite(const double* x, int64_t n, unsigned long long* part, hipStream_t s);

void process_constants(int proc, int* npart, int* ngood, int* ncol, int* ndiag);
double process_flops(int proc, bool executed);

#define RWGT_DECLARE_PROCESS(NAME)                                                                        \
  hipError_t launch_me_##NAME(int precision, const double* soa, int64_t nevt, const CardPair* cards,     \
                              int ncards, const double* w_in, double* w_out, double* me_out, hipStream_t s); \
  hipError_t launch_me_guarded_##NAME(int precision, const double* soa, int64_t nevt, const CardPair* cards, \
                                      int ncards, const double* w_in, double* w_out, double* me_out,          \
                                      const GuardArgs& g, hipStream_t s);                                     \
  void constants_##NAME(int* npart, int* ngood, int* ncol, int* ndiag);                                 \
  double flops_##NAME(bool executed);
RWGT_DECLARE_PROCESS(ee_mumu)
RWGT_DECLARE_PROCESS(uu_eeg)
RWGT_DECLARE_PROCESS(gg_ttgg)
RWGT_DECLARE_PROCESS(gg_tttt)
#undef RWGT_DECLARE_PROCESS

}  // namespace rwgt
