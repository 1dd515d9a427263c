// Internal interface of the batched persistent launch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "card.h"

namespace rwgt {

// Process families a batch kernel is compiled for; the process index of a
// segment is its position in the family.
enum { kFamilyElectroweak = 0 };   // 0: e+e- -> mu+mu-, 1: u u~ -> e+e- g

struct BatchSeg {
  int32_t proc;          // index within the family
  int32_t pad;
  int64_t nevt;
  int64_t tile0;         // first global tile of the segment
  const double* mom;     // [nevt][npart][4]
  const double* w_in;    // [nevt]
  double* w_out;         // [nevt]
};

struct BatchSchedule {
  int tile_events;       // events per tile
  int block;             // threads per workgroup
  int grid;              // persistent workgroups
  int hel_split;         // 0: one lane per event; 1: one lane per (event, card, helicity)
};

hipError_t launch_batch(int family, int precision, const BatchSeg* segs, int nseg, int64_t ntiles,
                        const BatchSchedule& sc, const CardPair* cards, unsigned long long* counter,
                        hipStream_t s);

// Exact reweighting with a card per event: the events list[0 .. *count) (device
// list and count, at most n_all of them), or every event 0 .. n_all-1 when
// list is NULL.  One lane per (event, kept helicity), at most max_blocks
// workgroups of 256 lanes (grid-stride beyond).  Event e uses cards[0] and
// cards[1 + card_index[e]]; an index outside [0, ncards) gives w' = NaN.
hipError_t launch_exact_list(int family, int precision, int proc, const double* mom, const int32_t* list,
                             const unsigned int* count, int64_t n_all, const int32_t* card_index, int ncards,
                             const CardPair* cards, const double* w_in, double* w_out, int max_blocks,
                             hipStream_t s);

}  // namespace rwgt
