// Matrix-element kernels for the generated process uu_eeg (FP64 and mixed).
#include "generated/gen_uu_eeg.h"
#include "me_kernel.h"

namespace rwgt {

RWGT_PROCESS_TRAITS(uu_eeg)

hipError_t launch_me_uu_eeg(int precision, const double* soa, int64_t nevt, const CardPair* cards, int ncards,
                            const double* w_in, double* w_out, double* me_out, hipStream_t s) {
  if (precision == kPrecFP64)
    return launch_me_t<Proc_uu_eeg, double>(soa, nevt, cards, ncards, w_in, w_out, me_out, s);
  return launch_me_t<Proc_uu_eeg, float>(soa, nevt, cards, ncards, w_in, w_out, me_out, s);
}

void constants_uu_eeg(int* npart, int* ngood, int* ncol, int* ndiag) {
  *npart = gen_uu_eeg::NPART;
  *ngood = gen_uu_eeg::NGOOD;
  *ncol = gen_uu_eeg::NCOL;
  *ndiag = gen_uu_eeg::NDIAG;
}

}  // namespace rwgt
