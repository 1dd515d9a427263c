// Matrix-element kernels for the generated process ee_mumu (FP64 and mixed).
#include "generated/gen_ee_mumu.h"
#include "me_kernel.h"
#include "opcount.h"

namespace rwgt {

RWGT_PROCESS_TRAITS(ee_mumu)

hipError_t launch_me_ee_mumu(int precision, const double* soa, int64_t nevt, const CardPair* cards, int ncards,
                            const double* w_in, double* w_out, double* me_out, hipStream_t s) {
  return launch_me_prec<Proc_ee_mumu>(precision, soa, nevt, cards, ncards, w_in, w_out, me_out, s);
}

hipError_t launch_me_guarded_ee_mumu(int precision, const double* soa, int64_t nevt, const CardPair* cards,
                                    int ncards, const double* w_in, double* w_out, double* me_out,
                                    const GuardArgs& g, hipStream_t s) {
  return launch_me_guarded_t<Proc_ee_mumu>(precision, soa, nevt, cards, ncards, w_in, w_out, me_out, g, s);
}

void constants_ee_mumu(int* npart, int* ngood, int* ncol, int* ndiag) {
  *npart = gen_ee_mumu::NPART;
  *ngood = gen_ee_mumu::NGOOD;
  *ncol = gen_ee_mumu::NCOL;
  *ndiag = gen_ee_mumu::NDIAG;
}

// Floating-point operations of one |M|^2 (helicities, colour sums, average),
// counted by running the generated code on the host with OpCnt at a
// representative point (beams along +-z, final state in generic directions):
// executed = false, the plain sum over every kept helicity; true, the
// helicities the kernels evaluate (NSUM, with the reversed ones as a weight).
double flops_ee_mumu(bool executed) {
  constexpr int N = gen_ee_mumu::NPART;
  static const double pts[6][4] = {{500.0, 0.0, 0.0, 500.0}, {500.0, 0.0, 0.0, -500.0},
                                   {300.0, 110.0, -150.0, 90.0}, {250.0, -60.0, 120.0, -170.0},
                                   {260.0, -30.0, 20.0, 90.0}, {190.0, -20.0, 10.0, -10.0}};
  OpCnt P[N][4];
  for (int a = 0; a < N; ++a)
    for (int mu = 0; mu < 4; ++mu) P[a][mu] = pts[a][mu];
  Card<OpCnt, OpCnt> cd;
  cd.gqq = 1.2;
  cd.g3 = 1.2;
  cd.g4 = 1.44;
  for (int f = 0; f < 4; ++f) {
    cd.a[f] = 0.3;
    cd.zL[f] = 0.2;
    cd.zR[f] = 0.1;
  }
  cd.mz = 91.0;
  cd.wz = 2.5;
  cd.mt = 173.0;
  OpCounter::flops = 0;
  cx<OpCnt> j[gen_ee_mumu::NCOL];
  gen_ee_mumu::jamps<OpCnt, OpCnt>(P, gen_ee_mumu::GOOD_HOST[0], cd, j);
  (void)gen_ee_mumu::colour_sum<OpCnt>(j);
  const double per_hel = double(OpCounter::flops) + 1.0;   // + accumulate into the sum
  return per_hel * (executed ? gen_ee_mumu::NSUM : gen_ee_mumu::NGOOD) + 1.0;   // + average factor
}

}  // namespace rwgt
