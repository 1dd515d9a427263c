// Colour quadratic form J^dagger C J on the matrix cores, one wave of 64
// events at a time (mixed precision).
//
// C is real and symmetric, so J^dagger C J = Jr.C.Jr + Ji.C.Ji.  Per lane
// (event) the float amplitudes are scaled by a power of two s (largest
// component near 2^14) and split into NT terms of the 16-bit type T
// (FP16: hi + lo; BF16: hi + mid + lo), each term exact in T, their sum
// equal to J s to ~2^-22 (FP16) / ~2^-24 (BF16) relative.  The terms are
// written to LDS as the K x N operand of v_mfma_f32_32x32x16 (K = colour flow,
// N = event); the integer colour numerators (exact in FP16 and BF16) form the
// constant M x K operand held in registers.  With FP32 accumulation the
// products give Z = C (J s) per event; each lane then forms (J s).Z for one
// event over its 16 output rows, the two half-waves holding the rest of the
// rows are summed with one lane swap, and the result is divided by s^2.
#pragma once

#include <hip/hip_runtime.h>

#include "helas.h"

namespace rwgt {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

template <class T> struct MfmaT;
template <> struct MfmaT<_Float16> {
  typedef f16x8 vec;
  static constexpr int terms = 2;
  static __device__ __forceinline__ f32x16 mfma(vec a, vec b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};
template <> struct MfmaT<__bf16> {
  typedef bf16x8 vec;
  static constexpr int terms = 3;
  static __device__ __forceinline__ f32x16 mfma(vec a, vec b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

// LDS of one wave: [part re/im][term][event 0..63][flow 0..31] of T.
template <class T>
struct ColourLds {
  static constexpr int kTerms = MfmaT<T>::terms;
  T v[2][kTerms][64][32];
};

template <int NCOL, class T>
struct ColourMfma {
  static_assert(NCOL <= 32, "one 32-row tile of colour flows");
  static constexpr int KSTEPS = (NCOL + 15) / 16;
  typedef typename MfmaT<T>::vec vec;
  vec a[KSTEPS];

  // A operand: lane l holds row l%32, columns 16 ks + 8 (l/32) + 0..7 of the
  // zero-padded numerator matrix.  Also zeroes the padding flows in LDS.
  __device__ __forceinline__ void init(const int (&cnum)[NCOL][NCOL], ColourLds<T>& lds) {
    const int l = threadIdx.x & 63;
    const int m = l & 31;
    for (int ks = 0; ks < KSTEPS; ++ks)
      for (int i = 0; i < 8; ++i) {
        const int k = 16 * ks + 8 * (l >> 5) + i;
        a[ks][i] = T((m < NCOL && k < NCOL) ? float(cnum[m][k]) : 0.0f);
      }
    for (int p = 0; p < 2; ++p)
      for (int t = 0; t < ColourLds<T>::kTerms; ++t)
        for (int c = NCOL; c < 32; ++c) lds.v[p][t][l][c] = T(0.0f);
  }

  // Sum over flows of the numerators, sum_ij conj(J_i) CNUM_ij J_j, for this
  // lane's event (in double, after removing the scale).  Every lane of the
  // wave must call it.
  template <class J>
  __device__ __forceinline__ double sum(const J& jamp, ColourLds<T>& lds) {
    constexpr int NT = ColourLds<T>::kTerms;
    const int l = threadIdx.x & 63;
    float mx = 0.0f;
    for (int c = 0; c < NCOL; ++c) mx = fmaxf(mx, fmaxf(fabsf(jamp[c].re), fabsf(jamp[c].im)));
    const int e = mx > 0.0f ? 14 - ilogbf(mx) : 0;
    const float s = ldexpf(1.0f, e);
#pragma unroll
    for (int c = 0; c < NCOL; ++c) {
      float x[2] = {jamp[c].re * s, jamp[c].im * s};
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        float r = x[p];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const T q = T(r);
          lds.v[p][t][l][c] = q;
          r -= float(q);
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // every loop unrolled: with the three BF16 terms the compiler otherwise
    // keeps a loop here, and the guarded kernel spilled 175 registers (2 now)
    float part[2] = {0.0f, 0.0f};
#pragma unroll
    for (int p = 0; p < 2; ++p) {
#pragma unroll
      for (int tile = 0; tile < 2; ++tile) {
        f32x16 acc = {};
        const int ev = 32 * tile + (l & 31);
#pragma unroll
        for (int ks = 0; ks < KSTEPS; ++ks)
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const vec b = *reinterpret_cast<const vec*>(&lds.v[p][t][ev][16 * ks + 8 * (l >> 5)]);
            acc = MfmaT<T>::mfma(a[ks], b, acc);
          }
        // lane l holds Z[row][ev] for row = 8 (i/4) + 4 (l/32) + i%4
        float dot = 0.0f;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int row = 8 * (i >> 2) + 4 * (l >> 5) + (i & 3);
          if (row < NCOL) {
            float xr = 0.0f;
#pragma unroll
            for (int t = 0; t < NT; ++t) xr += float(lds.v[p][t][ev][row]);
            dot += xr * acc[i];
          }
        }
        dot += __shfl_xor(dot, 32);
        if ((l >> 5) == tile) part[p] = dot;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return ldexp(double(part[0] + part[1]), -2 * e);
  }
};

}  // namespace rwgt
