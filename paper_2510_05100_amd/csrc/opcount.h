// Operation-counting scalar for the host instantiation of the device code.
//
// Instantiating the generated amplitude code with R = D = OpCnt evaluates it
// once on the host and counts every floating-point operation it performs:
// +, -, * and / count one each, sqrt counts one, a fused multiply-add in the
// compiled kernel is the multiply and the add counted here (two).  Negation,
// conjugation and multiplication by i are sign/swap moves and count zero.
// The count is the algorithmic work per evaluation, independent of how the
// compiler schedules it.
#pragma once

#include <cmath>

namespace rwgt {

struct OpCounter {
  static inline thread_local long long flops = 0;
};

struct OpCnt {
  double v = 0.0;
  OpCnt() = default;
  template <class T>
  OpCnt(T x) : v(double(x)) {}  // NOLINT: implicit, like a built-in scalar
};

inline OpCnt operator+(OpCnt a, OpCnt b) { ++OpCounter::flops; return OpCnt(a.v + b.v); }
inline OpCnt operator-(OpCnt a, OpCnt b) { ++OpCounter::flops; return OpCnt(a.v - b.v); }
inline OpCnt operator*(OpCnt a, OpCnt b) { ++OpCounter::flops; return OpCnt(a.v * b.v); }
inline OpCnt operator/(OpCnt a, OpCnt b) { ++OpCounter::flops; return OpCnt(a.v / b.v); }
inline OpCnt operator-(OpCnt a) { return OpCnt(-a.v); }
inline OpCnt& operator+=(OpCnt& a, OpCnt b) { a = a + b; return a; }
inline OpCnt sqrt(OpCnt a) { ++OpCounter::flops; return OpCnt(std::sqrt(a.v)); }
inline bool operator>(OpCnt a, double b) { return a.v > b; }
inline bool operator>=(OpCnt a, double b) { return a.v >= b; }
inline bool operator<(OpCnt a, double b) { return a.v < b; }

#define RWGT_OPCNT_MIXED(OP)                                                     \
  inline OpCnt operator OP(OpCnt a, double b) { return a OP OpCnt(b); }         \
  inline OpCnt operator OP(double a, OpCnt b) { return OpCnt(a) OP b; }
RWGT_OPCNT_MIXED(+)
RWGT_OPCNT_MIXED(-)
RWGT_OPCNT_MIXED(*)
RWGT_OPCNT_MIXED(/)
#undef RWGT_OPCNT_MIXED

}  // namespace rwgt
