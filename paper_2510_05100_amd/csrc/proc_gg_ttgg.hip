// Matrix-element kernels for the generated process gg_ttgg (FP64 and mixed).
#include "generated/gen_gg_ttgg.h"
#include "me_kernel.h"

namespace rwgt {

RWGT_PROCESS_TRAITS(gg_ttgg)

hipError_t launch_me_gg_ttgg(int precision, const double* soa, int64_t nevt, const CardPair* cards, int ncards,
                            const double* w_in, double* w_out, double* me_out, hipStream_t s) {
  if (precision == kPrecFP64)
    return launch_me_t<Proc_gg_ttgg, double>(soa, nevt, cards, ncards, w_in, w_out, me_out, s);
  return launch_me_t<Proc_gg_ttgg, float>(soa, nevt, cards, ncards, w_in, w_out, me_out, s);
}

void constants_gg_ttgg(int* npart, int* ngood, int* ncol, int* ndiag) {
  *npart = gen_gg_ttgg::NPART;
  *ngood = gen_gg_ttgg::NGOOD;
  *ncol = gen_gg_ttgg::NCOL;
  *ndiag = gen_gg_ttgg::NDIAG;
}

}  // namespace rwgt
