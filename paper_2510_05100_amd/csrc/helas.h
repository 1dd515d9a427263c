// Per-lane helicity-amplitude building blocks for gfx950 (one event per lane).
//
// The paper names the roles of these routines only (external wavefunctions
// ixxxxx / oxxxxx / vxxxxx, vertex amplitude FFV1_0, off-shell currents such as
// VVV1P0_1); what they compute here is written from the textbook Feynman rules:
//
//   metric diag(+,-,-,-), chiral Dirac basis psi = (psi_L, psi_R),
//   gamma^mu V_mu = [[0, V.sigma], [V.sigmabar, 0]],
//     V.sigma    = [[V0 - V3, -(V1 - i V2)], [-(V1 + i V2), V0 + V3]],
//     V.sigmabar = [[V0 + V3,   V1 - i V2 ], [  V1 + i V2,  V0 - V3]],
//   fermion-boson vertex  Gamma(V) = V-slash (cL P_L + cR P_R)  (vertex factors
//   i g_s, -i e Q, -i e/(s_W c_W) g_{L,R} are folded into the complex cL, cR),
//   fermion propagator    i (q-slash + m) / (q^2 - m^2),
//   massless vector       -i g_{mu nu} / q^2,
//   massive vector        -i (g_{mu nu} - q_mu q_nu / M^2) / (q^2 - M^2 + i M W),
//   three-gluon vertex    g f^{abc} [g^{mn}(k-p)^r + g^{nr}(p-q)^m + g^{rm}(q-k)^n],
//   four-gluon vertex     -i g^2 [f^{abe} f^{cde} (g^{mr} g^{ns} - g^{ms} g^{nr}) + 2 more].
//
// R is the amplitude precision (double, or float in the mixed mode).  Momenta,
// propagator denominators and the resonant Z denominator are always formed in
// double and only their reciprocals are rounded to R.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace rwgt {

// Mass argument of a massless line: the mass terms are dropped at compile
// time (without fast-math the compiler may not fold x + y * 0).
struct Massless {};
template <class M> constexpr bool is_massless = std::is_same<M, Massless>::value;

// a / b for the propagator denominators and polarisation angles.  On the
// device, in double: b's hardware reciprocal refined by two Newton steps,
// times a (within about an ulp of the rounded quotient, 6 instructions
// against about 10 for the correctly rounded division); elsewhere (the host,
// and the operation-counting type) the division itself.
template <class D>
__host__ __device__ __forceinline__ D quot(D a, D b) {
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (std::is_same<D, double>::value) {
    double r = __builtin_amdgcn_rcp(b);
    r = fma(r, fma(-b, r, 1.0), r);
    r = fma(r, fma(-b, r, 1.0), r);
    return a * r;
  } else {
    return a / b;
  }
#else
  return a / b;
#endif
}

template <class R> struct cx { R re, im; };

template <class R> __host__ __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R> __host__ __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R> __host__ __device__ __forceinline__ cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <class R> __host__ __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R> __host__ __device__ __forceinline__ cx<R> operator*(cx<R> a, R s) { return {a.re * s, a.im * s}; }
template <class R> __host__ __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {a.re * s, a.im * s}; }
template <class R> __host__ __device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
template <class R> __host__ __device__ __forceinline__ cx<R> times_i(cx<R> a) { return {-a.im, a.re}; }
template <class R> __host__ __device__ __forceinline__ cx<R> times_minus_i(cx<R> a) { return {a.im, -a.re}; }

template <class R> struct Spinor { cx<R> c[4]; };   // column (flowing in) or row (flowing out)
template <class R> struct Vec { cx<R> c[4]; };      // vector field, upper index

template <class R> __host__ __device__ __forceinline__ cx<R> mdot(const Vec<R>& a, const Vec<R>& b) {
  return a.c[0] * b.c[0] - a.c[1] * b.c[1] - a.c[2] * b.c[2] - a.c[3] * b.c[3];
}
template <class R, class D> __host__ __device__ __forceinline__ cx<R> mdot(const D* k, const Vec<R>& a) {
  return a.c[0] * R(k[0]) - a.c[1] * R(k[1]) - a.c[2] * R(k[2]) - a.c[3] * R(k[3]);
}
// A momentum component re-read at each use: opaque to value numbering on the
// device, so the sums below are recomputed where they are needed instead of
// being computed once and kept live across the whole helicity iteration.
template <class D> __host__ __device__ __forceinline__ D opq(D x) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(x));
#endif
  return x;
}
// Fence between amplitude terms: the instruction scheduler may not move work
// across it, so the evaluation order chosen by the process compiler (which
// keeps few currents live) is the order executed.
__host__ __device__ __forceinline__ void term_fence() {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_sched_barrier(0);
#endif
}
// Hooks of the mixed path's cancellation guard (me_kernel.h), called by the
// generated amplitude code at the start of a helicity and after each
// amplitude term (with the number of colour flows the term enters).  No-ops
// for plain amplitude storage; the guard's storage overloads them.
template <class J> __host__ __device__ __forceinline__ void note_reset(J&) {}
template <class J, class R> __host__ __device__ __forceinline__ void note_amp(J&, const cx<R>&, int) {}

template <class D> __host__ __device__ __forceinline__ D msq(const D* k) {
  return k[0] * k[0] - k[1] * k[1] - k[2] * k[2] - k[3] * k[3];
}

// ------------------------------------------------------------ external states
// Helicity 2-spinors along p: chi_+ = (cos t/2, e^{if} sin t/2),
// chi_- = (-e^{-if} sin t/2, cos t/2), written with |p| + pz instead of angles.
template <class R, class D>
__host__ __device__ __forceinline__ void helicity_basis(const D* p, D pabs, cx<R>& a0, cx<R>& a1, int lam) {
  const D pt2 = p[1] * p[1] + p[2] * p[2];
  // |p| + pz without cancellation when pz < 0
  const D ppz = p[3] >= 0.0 ? pabs + p[3] : (pt2 > 0.0 ? pt2 / (pabs - p[3]) : D(0.0));
  if (ppz > 0.0) {
    const D nrm = 1.0 / sqrt(2.0 * pabs * ppz);
    if (lam > 0) {
      a0 = {R(ppz * nrm), R(0)};
      a1 = {R(p[1] * nrm), R(p[2] * nrm)};
    } else {
      a0 = {R(-p[1] * nrm), R(p[2] * nrm)};
      a1 = {R(ppz * nrm), R(0)};
    }
  } else {  // along -z
    if (lam > 0) { a0 = {R(0), R(0)}; a1 = {R(1), R(0)}; }
    else         { a0 = {R(-1), R(0)}; a1 = {R(0), R(0)}; }
  }
}

// ixxxxx role: spinor flowing into the diagram.  nsf = +1: u(p, h) of an
// incoming fermion; nsf = -1: v(p, h) of an outgoing antifermion.
//   u = (sqrt(E - h|p|) chi_h, sqrt(E + h|p|) chi_h)
//   v = (sqrt(E + h|p|) chi_-h, -sqrt(E - h|p|) chi_-h)
template <class R, class D, class M>
__host__ __device__ __forceinline__ Spinor<R> ixx(const D* p, M m, int h, int nsf) {
  const D pabs = sqrt(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
  const D big = sqrt(p[0] + pabs);
  D small;                                // sqrt(E - |p|) = m / sqrt(E + |p|)
  if constexpr (is_massless<M>) small = D(0.0); else small = m / big;
  Spinor<R> s;
  cx<R> x0, x1;
  if (nsf > 0) {
    helicity_basis<R>(p, pabs, x0, x1, h);
    const R lo = R(h > 0 ? small : big), hi = R(h > 0 ? big : small);
    s.c[0] = x0 * lo; s.c[1] = x1 * lo; s.c[2] = x0 * hi; s.c[3] = x1 * hi;
  } else {
    helicity_basis<R>(p, pabs, x0, x1, -h);
    const R lo = R(h > 0 ? big : small), hi = R(h > 0 ? small : big);
    s.c[0] = x0 * lo; s.c[1] = x1 * lo; s.c[2] = -(x0 * hi); s.c[3] = -(x1 * hi);
  }
  return s;
}

// oxxxxx role: row spinor flowing out of the diagram, psi^dagger gamma^0.
// nsf = +1: ubar(p, h) of an outgoing fermion; nsf = -1: vbar(p, h) of an
// incoming antifermion.  gamma^0 swaps the chiral halves.
template <class R, class D, class M>
__host__ __device__ __forceinline__ Spinor<R> oxx(const D* p, M m, int h, int nsf) {
  const Spinor<R> col = ixx<R>(p, m, h, nsf);
  Spinor<R> s;
  s.c[0] = conj(col.c[2]); s.c[1] = conj(col.c[3]);
  s.c[2] = conj(col.c[0]); s.c[3] = conj(col.c[1]);
  return s;
}

// vxxxxx role: massless vector polarisation eps(k, h) = (-h e1 - i e2)/sqrt 2,
// e1 = (0, cos t cos f, cos t sin f, -sin t), e2 = (0, -sin f, cos f, 0);
// nsv = -1 (outgoing) returns eps*.
template <class R, class D>
__host__ __device__ __forceinline__ Vec<R> vxx(const D* k, int h, int nsv) {
  const D pt = sqrt(k[1] * k[1] + k[2] * k[2]);
  const D pabs = sqrt(pt * pt + k[3] * k[3]);
  D cf = 1.0, sf = 0.0, ct = k[3] >= 0.0 ? 1.0 : -1.0, st = 0.0;
  if (pt > 0.0) { cf = quot(k[1], pt); sf = quot(k[2], pt); ct = quot(k[3], pabs); st = quot(pt, pabs); }
  const double r = 0.70710678118654752440;
  const double hr = -h * r;                 // constants: folded at compile time
  const double im_sign = nsv > 0 ? -r : r;  // -i e2 for eps, +i e2 for eps*
  Vec<R> e;
  e.c[0] = {R(0), R(0)};
  e.c[1] = {R(hr * ct * cf), R(im_sign * -sf)};
  e.c[2] = {R(hr * ct * sf), R(im_sign * cf)};
  e.c[3] = {R(hr * -st), R(0)};
  return e;
}

// ------------------------------------------------------------- chiral blocks
// (V.sigma) x and (V.sigmabar) x for a complex vector V and 2-spinor x.
template <class R>
__host__ __device__ __forceinline__ void vsigma(const Vec<R>& v, cx<R> x0, cx<R> x1, cx<R>& y0, cx<R>& y1) {
  const cx<R> d = v.c[0] - v.c[3], u = v.c[0] + v.c[3];
  const cx<R> m = v.c[1] - times_i(v.c[2]), p = v.c[1] + times_i(v.c[2]);
  y0 = d * x0 - m * x1;
  y1 = u * x1 - p * x0;
}
template <class R>
__host__ __device__ __forceinline__ void vsigmabar(const Vec<R>& v, cx<R> x0, cx<R> x1, cx<R>& y0, cx<R>& y1) {
  const cx<R> d = v.c[0] - v.c[3], u = v.c[0] + v.c[3];
  const cx<R> m = v.c[1] - times_i(v.c[2]), p = v.c[1] + times_i(v.c[2]);
  y0 = u * x0 + m * x1;
  y1 = p * x0 + d * x1;
}
// row x times (V.sigma) and (V.sigmabar)
template <class R>
__host__ __device__ __forceinline__ void row_vsigma(const Vec<R>& v, cx<R> x0, cx<R> x1, cx<R>& y0, cx<R>& y1) {
  const cx<R> d = v.c[0] - v.c[3], u = v.c[0] + v.c[3];
  const cx<R> m = v.c[1] - times_i(v.c[2]), p = v.c[1] + times_i(v.c[2]);
  y0 = x0 * d - x1 * p;
  y1 = x1 * u - x0 * m;
}
template <class R>
__host__ __device__ __forceinline__ void row_vsigmabar(const Vec<R>& v, cx<R> x0, cx<R> x1, cx<R>& y0, cx<R>& y1) {
  const cx<R> d = v.c[0] - v.c[3], u = v.c[0] + v.c[3];
  const cx<R> m = v.c[1] - times_i(v.c[2]), p = v.c[1] + times_i(v.c[2]);
  y0 = x0 * u + x1 * p;
  y1 = x0 * m + x1 * d;
}
// Same blocks for a real momentum q.
template <class R>
__host__ __device__ __forceinline__ void qsigma(const R* q, cx<R> x0, cx<R> x1, cx<R>& y0, cx<R>& y1) {
  const R d = q[0] - q[3], u = q[0] + q[3];
  const cx<R> m = {q[1], -q[2]}, p = {q[1], q[2]};
  y0 = x0 * d - m * x1;
  y1 = x1 * u - p * x0;
}
template <class R>
__host__ __device__ __forceinline__ void qsigmabar(const R* q, cx<R> x0, cx<R> x1, cx<R>& y0, cx<R>& y1) {
  const R d = q[0] - q[3], u = q[0] + q[3];
  const cx<R> m = {q[1], -q[2]}, p = {q[1], q[2]};
  y0 = x0 * u + m * x1;
  y1 = p * x0 + x1 * d;
}
template <class R>
__host__ __device__ __forceinline__ void row_qsigma(const R* q, cx<R> x0, cx<R> x1, cx<R>& y0, cx<R>& y1) {
  const R d = q[0] - q[3], u = q[0] + q[3];
  const cx<R> m = {q[1], -q[2]}, p = {q[1], q[2]};
  y0 = x0 * d - x1 * p;
  y1 = x1 * u - x0 * m;
}
template <class R>
__host__ __device__ __forceinline__ void row_qsigmabar(const R* q, cx<R> x0, cx<R> x1, cx<R>& y0, cx<R>& y1) {
  const R d = q[0] - q[3], u = q[0] + q[3];
  const cx<R> m = {q[1], -q[2]}, p = {q[1], q[2]};
  y0 = x0 * u + x1 * p;
  y1 = x0 * m + x1 * d;
}

// ------------------------------------------------------------------ vertices
// Every vertex coupling of these processes is purely imaginary, c = i kappa
// (quark-gluon i g_s, photon -i e Q, Z -i e/(s_W c_W) g_{L,R}); the routines
// take the real kappa and fold the i into the propagator factors.  "_v"
// routines take one kappa (vector coupling), "_c" ones kappa_L and kappa_R.

// (V.sigma) psi_R and (V.sigmabar) psi_L of Gamma(V) psi.
template <class R>
__host__ __device__ __forceinline__ void gamma_v(const Vec<R>& v, const Spinor<R>& fi, cx<R>& u0, cx<R>& u1,
                                                 cx<R>& d0, cx<R>& d1) {
  vsigma(v, fi.c[2], fi.c[3], u0, u1);
  vsigmabar(v, fi.c[0], fi.c[1], d0, d1);
}
// Row versions: (b V.sigmabar, a V.sigma) of fo Gamma(V), fo = (a, b).
template <class R>
__host__ __device__ __forceinline__ void row_gamma_v(const Vec<R>& v, const Spinor<R>& fo, cx<R>& u0, cx<R>& u1,
                                                     cx<R>& d0, cx<R>& d1) {
  row_vsigmabar(v, fo.c[2], fo.c[3], u0, u1);
  row_vsigma(v, fo.c[0], fo.c[1], d0, d1);
}

// Fermion-pair vectors X^mu = a sigma^mu psi_R, Y^mu = b sigmabar^mu psi_L
// (fo = (a, b), fi = (psi_L, psi_R)); fo gamma^mu (cL P_L + cR P_R) fi =
// i (kR X + kL Y).  pair_w returns W = X + Y (vector coupling).
template <class R>
__host__ __device__ __forceinline__ void pair_xy(const Spinor<R>& fo, const Spinor<R>& fi, Vec<R>& x, Vec<R>& y) {
  const cx<R> a0 = fo.c[0], a1 = fo.c[1], b0 = fo.c[2], b1 = fo.c[3];
  const cx<R> r0 = fi.c[2], r1 = fi.c[3], l0 = fi.c[0], l1 = fi.c[1];
  const cx<R> s00 = a0 * r0, s01 = a0 * r1, s10 = a1 * r0, s11 = a1 * r1;
  const cx<R> t00 = b0 * l0, t01 = b0 * l1, t10 = b1 * l0, t11 = b1 * l1;
  x.c[0] = s00 + s11; x.c[1] = s01 + s10; x.c[2] = times_i(s10 - s01); x.c[3] = s00 - s11;
  y.c[0] = t00 + t11; y.c[1] = -(t01 + t10); y.c[2] = times_i(t01 - t10); y.c[3] = t11 - t00;
}
template <class R>
__host__ __device__ __forceinline__ Vec<R> pair_w(const Spinor<R>& fo, const Spinor<R>& fi) {
  const cx<R> a0 = fo.c[0], a1 = fo.c[1], b0 = fo.c[2], b1 = fo.c[3];
  const cx<R> r0 = fi.c[2], r1 = fi.c[3], l0 = fi.c[0], l1 = fi.c[1];
  const cx<R> s00 = a0 * r0, s01 = a0 * r1, s10 = a1 * r0, s11 = a1 * r1;
  const cx<R> t00 = b0 * l0, t01 = b0 * l1, t10 = b1 * l0, t11 = b1 * l1;
  Vec<R> w;
  w.c[0] = (s00 + s11) + (t00 + t11);
  w.c[1] = (s01 + s10) - (t01 + t10);
  w.c[2] = times_i((s10 - s01) - (t10 - t01));
  w.c[3] = (s00 - s11) - (t00 - t11);
  return w;
}

// FFV1_0 role, vector coupling: fo Gamma(V) fi = i k V.W(fo, fi).
template <class R>
__host__ __device__ __forceinline__ cx<R> ffv_amp_v(const Spinor<R>& fo, const Spinor<R>& fi, const Vec<R>& v, R k) {
  return times_i(mdot(v, pair_w(fo, fi))) * k;
}
// Same with a precomputed W of the (fo, fi) pair.
template <class R>
__host__ __device__ __forceinline__ cx<R> pair_amp_v(const Vec<R>& w, const Vec<R>& v, R k) {
  return times_i(mdot(v, w)) * k;
}
// FFV1_0 role, chiral coupling: i (kR V.X + kL V.Y).
template <class R>
__host__ __device__ __forceinline__ cx<R> ffv_amp_c(const Spinor<R>& fo, const Spinor<R>& fi, const Vec<R>& v, R kl, R kr) {
  Vec<R> x, y;
  pair_xy(fo, fi, x, y);
  return times_i(mdot(v, x) * kr + mdot(v, y) * kl);
}

// (q-slash + m) applied to a column (u, d) / a row (u, d), then scaled by s.
template <class R, class D, class M>
__host__ __device__ __forceinline__ Spinor<R> qslash_col(cx<R> u0, cx<R> u1, cx<R> d0, cx<R> d1, const D* qd, M m, R s) {
  const R q[4] = {R(qd[0]), R(qd[1]), R(qd[2]), R(qd[3])};
  Spinor<R> o;
  qsigma(q, d0, d1, o.c[0], o.c[1]);          // upper = (q.sigma) d + m u
  qsigmabar(q, u0, u1, o.c[2], o.c[3]);       // lower = (q.sigmabar) u + m d
  if constexpr (!is_massless<M>) {
    const R rm = R(m);
    o.c[0] = o.c[0] + u0 * rm; o.c[1] = o.c[1] + u1 * rm;
    o.c[2] = o.c[2] + d0 * rm; o.c[3] = o.c[3] + d1 * rm;
  }
  for (int i = 0; i < 4; ++i) o.c[i] = o.c[i] * s;
  return o;
}
template <class R, class D, class M>
__host__ __device__ __forceinline__ Spinor<R> qslash_row(cx<R> u0, cx<R> u1, cx<R> d0, cx<R> d1, const D* qd, M m, R s) {
  const R q[4] = {R(qd[0]), R(qd[1]), R(qd[2]), R(qd[3])};
  Spinor<R> o;
  row_qsigmabar(q, d0, d1, o.c[0], o.c[1]);   // first half = m u + d (q.sigmabar)
  row_qsigma(q, u0, u1, o.c[2], o.c[3]);      // second half = u (q.sigma) + m d
  if constexpr (!is_massless<M>) {
    const R rm = R(m);
    o.c[0] = o.c[0] + u0 * rm; o.c[1] = o.c[1] + u1 * rm;
    o.c[2] = o.c[2] + d0 * rm; o.c[3] = o.c[3] + d1 * rm;
  }
  for (int i = 0; i < 4; ++i) o.c[i] = o.c[i] * s;
  return o;
}
// 1/(q^2 - m^2) in double (the momentum type), then rounded
template <class D, class M>
__host__ __device__ __forceinline__ D inv_den(const D* q, M m) {
  if constexpr (is_massless<M>) return quot(D(1.0), msq(q));
  else return quot(D(1.0), msq(q) - m * m);
}

// Off-shell fermion flowing in, i (q-slash + m)/(q^2 - m^2) Gamma(V) fi, with
// Gamma = i kappa V-slash: -kappa (q-slash + m)/(q^2 - m^2) V-slash fi.
template <class R, class D, class M>
__host__ __device__ __forceinline__ Spinor<R> ffv_in_v(const Spinor<R>& fi, const Vec<R>& v, R k, const D* q, M m) {
  cx<R> u0, u1, d0, d1;
  gamma_v(v, fi, u0, u1, d0, d1);
  return qslash_col(u0, u1, d0, d1, q, m, R(-k * inv_den(q, m)));
}
template <class R, class D, class M>
__host__ __device__ __forceinline__ Spinor<R> ffv_in_c(const Spinor<R>& fi, const Vec<R>& v, R kl, R kr, const D* q, M m) {
  cx<R> u0, u1, d0, d1;
  gamma_v(v, fi, u0, u1, d0, d1);
  u0 = u0 * kr; u1 = u1 * kr; d0 = d0 * kl; d1 = d1 * kl;
  return qslash_col(u0, u1, d0, d1, q, m, R(-inv_den(q, m)));
}
// Off-shell fermion flowing out (row): fo Gamma(V) i (q-slash + m)/(q^2 - m^2).
template <class R, class D, class M>
__host__ __device__ __forceinline__ Spinor<R> ffv_out_v(const Spinor<R>& fo, const Vec<R>& v, R k, const D* q, M m) {
  cx<R> u0, u1, d0, d1;
  row_gamma_v(v, fo, u0, u1, d0, d1);
  return qslash_row(u0, u1, d0, d1, q, m, R(-k * inv_den(q, m)));
}
template <class R, class D, class M>
__host__ __device__ __forceinline__ Spinor<R> ffv_out_c(const Spinor<R>& fo, const Vec<R>& v, R kl, R kr, const D* q, M m) {
  cx<R> u0, u1, d0, d1;
  row_gamma_v(v, fo, u0, u1, d0, d1);
  u0 = u0 * kl; u1 = u1 * kl; d0 = d0 * kr; d1 = d1 * kr;
  return qslash_row(u0, u1, d0, d1, q, m, R(-inv_den(q, m)));
}

// Off-shell massless vector from a fermion pair, vector coupling:
// (-i/q^2) (i k W) = k W / q^2.
template <class R, class D>
__host__ __device__ __forceinline__ Vec<R> ffv_vec0_v(const Spinor<R>& fo, const Spinor<R>& fi, R k, const D* q) {
  Vec<R> w = pair_w(fo, fi);
  const R s = R(quot(D(k), msq(q)));
  for (int i = 0; i < 4; ++i) w.c[i] = w.c[i] * s;
  return w;
}

// Off-shell massive vector from a fermion pair, chiral coupling, unitary
// gauge and fixed width: (-i)(i j')... = (j' - q (q.j')/M^2) / (q^2 - M^2 + i M W)
// with j' = kR X + kL Y; the denominator is formed and inverted in double.
template <class R, class D, class M>
__host__ __device__ __forceinline__ Vec<R> ffv_vecm_c(const Spinor<R>& fo, const Spinor<R>& fi, R kl, R kr,
                                                      const D* q, M mass, M width) {
  Vec<R> x, y, j;
  pair_xy(fo, fi, x, y);
  for (int i = 0; i < 4; ++i) j.c[i] = x.c[i] * kr + y.c[i] * kl;
  const D dre = msq(q) - mass * mass, dim = mass * width;
  const D inv = quot(D(1.0), dre * dre + dim * dim);
  const cx<R> f = {R(dre * inv), R(-dim * inv)};      // 1 / (dre + i dim)
  const cx<R> qj = mdot(q, j) * R(1.0 / (mass * mass));
  for (int i = 0; i < 4; ++i) j.c[i] = f * (j.c[i] - qj * R(q[i]));
  return j;
}

// VVV1P0_1 role: off-shell gluon from two gluon currents, (-i/K^2) g V3 with
// V3 = (J1.J2)(k1 - k2) + ((k1 + 2 k2).J1) J2 - ((2 k1 + k2).J2) J1.
template <class R, class D>
__host__ __device__ __forceinline__ Vec<R> vvv_vec(const Vec<R>& j1, const D* k1, const Vec<R>& j2, const D* k2, R g) {
  D kk[4], a[4], b[4], d[4];
  for (int i = 0; i < 4; ++i) {
    kk[i] = k1[i] + k2[i];
    a[i] = k1[i] + 2.0 * k2[i];
    b[i] = 2.0 * k1[i] + k2[i];
    d[i] = k1[i] - k2[i];
  }
  const cx<R> j12 = mdot(j1, j2), aj1 = mdot(a, j1), bj2 = mdot(b, j2);
  const R s = R(quot(D(g), msq(kk)));
  Vec<R> out;
  for (int i = 0; i < 4; ++i) {
    const cx<R> v = j12 * R(d[i]) + aj1 * j2.c[i] - bj2 * j1.c[i];
    out.c[i] = times_minus_i(v) * s;
  }
  return out;
}

// Off-shell gluon from three gluon currents through one of the three colour
// structures of the four-gluon vertex: (-i/K^2)(-i g^2) L_t,
//   L_0 = J2 (J1.J3) - J3 (J1.J2),  L_1 = J1 (J2.J3) - J3 (J1.J2),
//   L_2 = J1 (J2.J3) - J2 (J1.J3).
template <int TERM, class R, class D>
__host__ __device__ __forceinline__ Vec<R> vvvv_vec(const Vec<R>& j1, const Vec<R>& j2, const Vec<R>& j3, const D* kk, R g2) {
  const R s = R(quot(D(g2), msq(kk)));      // (-i)(-i) = -1 folded below
  Vec<R> out;
  if (TERM == 0) {
    const cx<R> x = mdot(j1, j3), y = mdot(j1, j2);
    for (int i = 0; i < 4; ++i) out.c[i] = (j3.c[i] * y - j2.c[i] * x) * s;
  } else if (TERM == 1) {
    const cx<R> x = mdot(j2, j3), y = mdot(j1, j2);
    for (int i = 0; i < 4; ++i) out.c[i] = (j3.c[i] * y - j1.c[i] * x) * s;
  } else {
    const cx<R> x = mdot(j2, j3), y = mdot(j1, j3);
    for (int i = 0; i < 4; ++i) out.c[i] = (j2.c[i] * y - j1.c[i] * x) * s;
  }
  return out;
}

}  // namespace rwgt
