// Per-card couplings as the device sees them (uniform across a launch).
//
// Vertex factors follow the textbook rules (quark-gluon i g_s gamma^mu t^a,
// three-gluon g_s f^{abc}[...], four-gluon -i g_s^2 [...], photon -i e Q,
// Z -i e/(s_W c_W)((T3 - Q s_W^2) P_L - Q s_W^2 P_R)).  Species index: 0 e,
// 1 mu, 2 u, 3 t.
#pragma once

#include "helas.h"

namespace rwgt {

// Fermion-boson couplings are c = i kappa; the real kappa is stored.
template <class R, class D = double>
struct Card {
  R gqq;                 // kappa = g_s           (quark-gluon, vector)
  R g3;                  // g_s                   (three-gluon vertex g f^{abc} [...])
  R g4;                  // g_s^2                 (four-gluon, the -i is in vvvv_vec)
  R a[4];                // kappa = -e Q          (photon, vector)
  R zL[4], zR[4];        // kappa = -e/(s_W c_W) g_{L,R}   (Z, chiral)
  D mz, wz, mt;          // double on the device: resonant and mass terms
};

// Both precisions of one card, filled on the host.
struct CardPair {
  Card<double> d;
  Card<float> f;
};

}  // namespace rwgt
