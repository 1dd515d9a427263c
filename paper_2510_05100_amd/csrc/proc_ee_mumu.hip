// Matrix-element kernels for the generated process ee_mumu (FP64 and mixed).
#include "generated/gen_ee_mumu.h"
#include "me_kernel.h"

namespace rwgt {

RWGT_PROCESS_TRAITS(ee_mumu)

hipError_t launch_me_ee_mumu(int precision, const double* soa, int64_t nevt, const CardPair* cards, int ncards,
                            const double* w_in, double* w_out, double* me_out, hipStream_t s) {
  if (precision == kPrecFP64)
    return launch_me_t<Proc_ee_mumu, double>(soa, nevt, cards, ncards, w_in, w_out, me_out, s);
  return launch_me_t<Proc_ee_mumu, float>(soa, nevt, cards, ncards, w_in, w_out, me_out, s);
}

void constants_ee_mumu(int* npart, int* ngood, int* ncol, int* ndiag) {
  *npart = gen_ee_mumu::NPART;
  *ngood = gen_ee_mumu::NGOOD;
  *ncol = gen_ee_mumu::NCOL;
  *ndiag = gen_ee_mumu::NDIAG;
}

}  // namespace rwgt
