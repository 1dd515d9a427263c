// Per-card couplings as the device sees them (uniform across a launch).
//
// Vertex factors follow the textbook rules (quark-gluon i g_s gamma^mu t^a,
// three-gluon g_s f^{abc}[...], four-gluon -i g_s^2 [...], photon -i e Q,
// Z -i e/(s_W c_W)(T3 - Q s_W^2) P_L + ...); the complex ones are stored with
// their factor of i.  Species index: 0 e, 1 mu, 2 u, 3 t.
#pragma once

#include "helas.h"

namespace rwgt {

template <class R, class D = double>
struct Card {
  cx<R> gqq;             // i g_s   (quark-gluon, both chiralities)
  R g3;                  // g_s     (three-gluon)
  R g4;                  // g_s^2   (four-gluon, the -i is in vvvv_vec)
  cx<R> aL[4], aR[4];    // photon: -i e Q
  cx<R> zL[4], zR[4];    // Z: -i e/(s_W c_W) g_{L,R}
  D mz, wz, mt;          // double on the device: resonant and mass terms
};

// Both precisions of one card, filled on the host.
struct CardPair {
  Card<double> d;
  Card<float> f;
};

}  // namespace rwgt
