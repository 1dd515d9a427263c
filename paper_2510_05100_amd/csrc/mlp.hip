// Kernels of the learned surrogate: a multilayer perceptron (SiLU hidden
// layers) predicting the log of the reweighting ratio and the log of its own
// error, trained and evaluated on the GPU.
//
// Training runs layer by layer; each layer has its own operand type.  In a
// BF16 network the first layer (whose inputs locate the Z resonance) and the
// two-row head are FP32 on the VALU and the width x width hidden layers are
// BF16 on the matrix cores, all with FP32 accumulation and FP32 master
// weights.
//
//   gemm_nt    C[M x N] = A[M x K] . B[N x K]^T (row-major, K contiguous).
//              BF16 operands on v_mfma_f32_32x32x16_bf16 (one wave per
//              32 x 32 tile) or FP32 operands on the VALU.  Epilogue: + bias,
//              the FP32 result and/or the SiLU (or identity) in the next
//              layer's operand type.
//   silu_bwd   G = dH * silu'(Z)
//   colsum     db = sum over rows of G (two coalesced passes over a
//              workspace, else one workgroup per column)
//   loss_grad  Gaussian-error loss of the two heads and its gradient
//   adam       FP32 master weights, moments, and the operand-type copies W, W^T
//   features   standardised input rows (raw or physics feature map)
//   gate       w' = w exp(mu) where the predicted error is small; the others
//              are listed for the exact path
//   pack       weights in the per-lane order of the fused kernel's A operands
//   infer      the fused inference pass: features, every layer, the heads and
//              the gate for 32 rows per wave, activations kept in registers,
//              weights read from L2 (staging them in LDS per compute unit
//              measured slower: 0.45 against 0.39 ms per 1e6 rows)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "mlp.h"
#include "shuffle.h"

namespace rwgt {

typedef __bf16 bf16;
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

// SiLU and its derivative with the hardware reciprocal (1 ulp) instead of a
// correctly rounded division: the same function in training and inference.
__device__ __forceinline__ float sigmoid(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigmoid(z); }
__device__ __forceinline__ float silu_grad(float z) {
  const float s = sigmoid(z);
  return s * (1.0f + z * (1.0f - s));
}

// asinh x = sign(x) log(|x| + sqrt(x^2 + 1)) with the hardware logarithm:
// absolute error about 1e-7 for the |x| < 1e3 of the propagator features.
__device__ __forceinline__ float fast_asinh(float x) {
  return copysignf(__logf(fabsf(x) + sqrtf(fmaf(x, x, 1.0f))), x);
}

// ------------------------------------------------------------ feature maps
// Raw map: [momenta (NPART x 4), M_Z, Gamma_Z, sin^2 theta_W].
// Physics map: with s_hat = 2 p0.p1 and s_ij = 2 pi.pj,
//   [log s_hat, log(|s_ij| / s_hat) for i < j, M_Z, Gamma_Z, sin^2 theta_W,
//    asinh Re chi, asinh Im chi, asinh Re chi0, asinh Im chi0]
// where chi = s / (s - M^2 + i M Gamma) at s = s_ab of the resonant pair,
// under the card (chi) and under the original card (chi0).  Invariants and
// propagator ratios in FP64 from the FP64 momenta (they cancel near collinear
// limits and the pole), their logarithms and asinh in FP32 with the hardware
// logarithm; unused slots are zero.
template <int NPART, int KIND>
__device__ __forceinline__ void feature_row(const FeatureMap& fm, const double (&p)[NPART * 4], const float (&card)[3],
                                            float (&f)[kMlpMaxIn]) {
#pragma unroll
  for (int k = 0; k < kMlpMaxIn; ++k) f[k] = 0.0f;
  if constexpr (KIND == kFeatRaw) {
#pragma unroll
    for (int k = 0; k < NPART * 4; ++k) f[k] = float(p[k]);
#pragma unroll
    for (int j = 0; j < kMlpCardParams; ++j) f[NPART * 4 + j] = card[j];
  } else {
    auto dot2 = [&](int i, int j) {
      return 2.0 * (p[4 * i] * p[4 * j] - p[4 * i + 1] * p[4 * j + 1] - p[4 * i + 2] * p[4 * j + 2] -
                    p[4 * i + 3] * p[4 * j + 3]);
    };
    const double shat = dot2(0, 1);
    const double ishat = 1.0 / shat;
    f[0] = __logf(float(shat));
    double s_res = 0.0;
    int k = 1;
#pragma unroll
    for (int i = 0; i < NPART; ++i)
#pragma unroll
      for (int j = i + 1; j < NPART; ++j) {
        const double sij = dot2(i, j);
        f[k++] = __logf(fmaxf(float(fabs(sij) * ishat), 1e-37f));
        if ((i == fm.res_a && j == fm.res_b) || (i == fm.res_b && j == fm.res_a)) s_res = sij;
      }
#pragma unroll
    for (int j = 0; j < kMlpCardParams; ++j) f[k++] = card[j];
    auto chi = [&](double m, double w, float& re, float& im) {
      const double x = s_res - m * m, y = m * w;
      const double t = s_res / (x * x + y * y);
      re = fast_asinh(float(t * x));
      im = fast_asinh(float(-t * y));
    };
    chi(double(card[0]), double(card[1]), f[k], f[k + 1]);
    chi(fm.mz0, fm.wz0, f[k + 2], f[k + 3]);
  }
}

// (f - mean) / std as a product with the reciprocals istd (computed once on
// the host per normalisation).
__device__ __forceinline__ void standardise(float (&f)[kMlpMaxIn], const float* __restrict__ mean,
                                            const float* __restrict__ istd) {
#pragma unroll
  for (int k = 0; k < kMlpMaxIn; ++k) f[k] = (f[k] - mean[k]) * istd[k];
}

template <int NPART>
__device__ __forceinline__ void load_event(const double* __restrict__ mom, int64_t e, double (&p)[NPART * 4]) {
#pragma unroll
  for (int k = 0; k < NPART * 4; ++k) p[k] = mom[e * (NPART * 4) + k];
}

// ------------------------------------------------------------------ GEMMs
// Epilogue of a 32 x 32 tile held in the standard accumulator layout (lane
// l, element i: row 8 (i/4) + 4 (l/32) + i%4, column l%32): the raw sums to
// this K chunk's slice of part, or bias, activation and the outputs.
template <class TO>
__device__ __forceinline__ void tile_out(const f32x16_t& acc, int tm, int tn, int M, int N,
                                         const float* __restrict__ bias, float* __restrict__ Cf,
                                         TO* __restrict__ Ct, int act, float* __restrict__ part) {
  const int l = threadIdx.x;
  const int col = tn * 32 + (l & 31);
  if (part) {
    float* p = part + size_t(blockIdx.y) * M * N;
#pragma unroll
    for (int i = 0; i < 16; ++i) p[size_t(tm * 32 + 8 * (i >> 2) + 4 * (l >> 5) + (i & 3)) * N + col] = acc[i];
    return;
  }
  const float bb = bias ? bias[col] : 0.0f;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int row = tm * 32 + 8 * (i >> 2) + 4 * (l >> 5) + (i & 3);
    const float v = acc[i] + bb;
    if (Cf) Cf[size_t(row) * N + col] = v;
    if (Ct) Ct[size_t(row) * N + col] = TO(act ? silu(v) : v);
  }
}

// C = A B^T (A [M][K], B [N][K], K contiguous): one wave per 32 x 32 tile
// (blockIdx.x) and K chunk [kchunk y, kchunk (y+1)) (blockIdx.y).  With more
// than one chunk the partial tiles go to part [chunks][M][N] and ksum_k adds
// them in chunk order (deterministic): long-K products (weight gradients,
// K = batch rows) then fill the chip instead of a few waves.
template <class TO>
__global__ __launch_bounds__(64) void gemm_nt_bf16(const bf16* __restrict__ A, const bf16* __restrict__ B, int M,
                                                   int N, int K, int kchunk, const float* __restrict__ bias,
                                                   float* __restrict__ Cf, TO* __restrict__ Ct, int act,
                                                   float* __restrict__ part) {
  const int ntn = N / 32;
  const int tm = blockIdx.x / ntn, tn = blockIdx.x % ntn;
  const int l = threadIdx.x;
  const bf16* a_row = A + size_t(tm * 32 + (l & 31)) * K + 8 * (l >> 5);
  const bf16* b_row = B + size_t(tn * 32 + (l & 31)) * K + 8 * (l >> 5);
  const int kb = int(blockIdx.y) * kchunk, ke = min(K, kb + kchunk);
  f32x16_t acc = {};
  int k0 = kb;
  // four K steps at a time: their loads in flight together, then the products
  // in K order
  for (; k0 + 64 <= ke; k0 += 64) {
    bf16x8_t a[4], b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      a[j] = *reinterpret_cast<const bf16x8_t*>(a_row + k0 + 16 * j);
      b[j] = *reinterpret_cast<const bf16x8_t*>(b_row + k0 + 16 * j);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[j], b[j], acc, 0, 0, 0);
  }
  for (; k0 < ke; k0 += 16) {
    const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(a_row + k0);
    const bf16x8_t b = *reinterpret_cast<const bf16x8_t*>(b_row + k0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  tile_out<TO>(acc, tm, tn, M, N, bias, Cf, Ct, act, part);
}

// FP32 operands through the matrix cores as high and low BF16 parts: three
// products hi.hi + hi.lo + lo.hi per step (relative error about 2^-16), the
// same arithmetic as the fused kernel's first layer.
template <class TO>
__global__ __launch_bounds__(64) void gemm_nt_split(const float* __restrict__ A, const float* __restrict__ B, int M,
                                                    int N, int K, int kchunk, const float* __restrict__ bias,
                                                    float* __restrict__ Cf, TO* __restrict__ Ct, int act,
                                                    float* __restrict__ part) {
  const int ntn = N / 32;
  const int tm = blockIdx.x / ntn, tn = blockIdx.x % ntn;
  const int l = threadIdx.x;
  const float* a_row = A + size_t(tm * 32 + (l & 31)) * K + 8 * (l >> 5);
  const float* b_row = B + size_t(tn * 32 + (l & 31)) * K + 8 * (l >> 5);
  const int kb = int(blockIdx.y) * kchunk, ke = min(K, kb + kchunk);
  f32x16_t acc = {};
  for (int k0 = kb; k0 < ke; k0 += 16) {
    bf16x8_t ah, al, bh, bl;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const float a = a_row[k0 + s], b = b_row[k0 + s];
      ah[s] = bf16(a);
      al[s] = bf16(a - float(ah[s]));
      bh[s] = bf16(b);
      bl[s] = bf16(b - float(bh[s]));
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
  }
  tile_out<TO>(acc, tm, tn, M, N, bias, Cf, Ct, act, part);
}

// FP32 C = A B^T on the matrix cores (v_mfma_f32_32x32x2_f32: FP32 products,
// FP32 accumulation), tiles and K chunks as gemm_nt_bf16.  Lane l reads 4
// consecutive K values of row l%32 of each operand, half-wave h = l/32 the
// four after half 0's; product step j pairs element j of both halves, so
// step j covers K = {k0 + j, k0 + 4 + j}: the same indices on A and B, every
// index of the 8-wide block once.
template <class TO>
__global__ __launch_bounds__(64) void gemm_nt_f32m(const float* __restrict__ A, const float* __restrict__ B, int M,
                                                   int N, int K, int kchunk, const float* __restrict__ bias,
                                                   float* __restrict__ Cf, TO* __restrict__ Ct, int act,
                                                   float* __restrict__ part) {
  const int ntn = N / 32;
  const int tm = blockIdx.x / ntn, tn = blockIdx.x % ntn;
  const int l = threadIdx.x;
  const float* a_row = A + size_t(tm * 32 + (l & 31)) * K + 4 * (l >> 5);
  const float* b_row = B + size_t(tn * 32 + (l & 31)) * K + 4 * (l >> 5);
  const int kb = int(blockIdx.y) * kchunk, ke = min(K, kb + kchunk);
  f32x16_t acc = {};
  int k0 = kb;
  // four 8-wide K blocks at a time: loads first, products in K order
  for (; k0 + 32 <= ke; k0 += 32) {
    float4 a[4], b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      a[j] = *reinterpret_cast<const float4*>(a_row + k0 + 8 * j);
      b[j] = *reinterpret_cast<const float4*>(b_row + k0 + 8 * j);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[j].x, b[j].x, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[j].y, b[j].y, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[j].z, b[j].z, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[j].w, b[j].w, acc, 0, 0, 0);
    }
  }
  for (; k0 < ke; k0 += 8) {
    const float4 a = *reinterpret_cast<const float4*>(a_row + k0);
    const float4 b = *reinterpret_cast<const float4*>(b_row + k0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b.w, acc, 0, 0, 0);
  }
  tile_out<TO>(acc, tm, tn, M, N, bias, Cf, Ct, act, part);
}

// C[i] = sum over chunks c (in order) of part[c][i], then bias / activation.
template <class TO>
__global__ __launch_bounds__(256) void ksum_k(const float* __restrict__ part, int chunks, int M, int N,
                                              const float* __restrict__ bias, float* __restrict__ Cf,
                                              TO* __restrict__ Ct, int act) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t mn = int64_t(M) * N;
  if (i >= mn) return;
  // loads in groups of eight ahead of their additions (independent loads in
  // flight instead of one per trip); the additions keep chunk order
  float v = 0.0f;
  int c = 0;
  for (; c + 8 <= chunks; c += 8) {
    float p[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) p[k] = part[(c + k) * mn + i];
#pragma unroll
    for (int k = 0; k < 8; ++k) v += p[k];
  }
  for (; c < chunks; ++c) v += part[c * mn + i];
  v += bias ? bias[i % N] : 0.0f;
  if (Cf) Cf[i] = v;
  if (Ct) Ct[i] = TO(act ? silu(v) : v);
}

template <class TO>
__global__ __launch_bounds__(256) void gemm_nt_f32(const float* __restrict__ A, const float* __restrict__ B, int M,
                                                   int N, int K, const float* __restrict__ bias,
                                                   float* __restrict__ Cf, TO* __restrict__ Ct, int act) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(M) * N) return;
  const int row = int(idx / N), col = int(idx % N);
  const float* a = A + size_t(row) * K;
  const float* b = B + size_t(col) * K;
  float s = 0.0f;
  for (int k = 0; k < K; ++k) s = fmaf(a[k], b[k], s);
  const float v = s + (bias ? bias[col] : 0.0f);
  if (Cf) Cf[idx] = v;
  if (Ct) Ct[idx] = TO(act ? silu(v) : v);
}

// out[c][r] = in[r][c] converted to TO
template <class TI, class TO>
__global__ __launch_bounds__(256) void transpose_k(const TI* __restrict__ in, TO* __restrict__ out, int R, int C) {
  __shared__ float tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int j = ty; j < 32; j += 8) {
    const int r = by + j, c = bx + tx;
    if (r < R && c < C) tile[j][tx] = float(in[size_t(r) * C + c]);
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int c = bx + j, r = by + tx;
    if (r < R && c < C) out[size_t(c) * R + r] = TO(tile[tx][j]);
  }
}

template <class T>
__global__ __launch_bounds__(256) void silu_bwd(const float* __restrict__ dh, const float* __restrict__ z,
                                                float* __restrict__ g, T* __restrict__ gt, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float v = dh[i] * silu_grad(z[i]);
  g[i] = v;
  gt[i] = T(v);
}

// db[c] = sum_r g[r][c]: one workgroup per column
__global__ __launch_bounds__(256) void colsum(const float* __restrict__ g, float* __restrict__ db, int R, int C) {
  __shared__ float part[256];
  const int c = blockIdx.x;
  float s = 0.0f;
  for (int r = threadIdx.x; r < R; r += blockDim.x) s += g[size_t(r) * C + c];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[c] = part[0];
}

// The same sum in two passes over a workspace of ceil(R/64) x C partials,
// coalesced and deterministic.  colsum_part: workgroup (x, y) takes the 64
// columns from 64x and the 64 rows from 64y; lane = column, so each row's
// columns are one contiguous load; each wave loads its 16 rows (every fourth)
// before adding them, and the four waves add in wave order.  colsum_fin: one
// wave per column adds the slab partials (lane k takes slabs k, k+64, ...)
// and reduces the lanes with a fixed shuffle tree.
constexpr int kColsumSlabRows = 64;

__global__ __launch_bounds__(256) void colsum_part(const float* __restrict__ g, float* __restrict__ part, int R, int C) {
  __shared__ float ws[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  const int r0 = blockIdx.y * kColsumSlabRows + w;
  float v[kColsumSlabRows / 4];
#pragma unroll
  for (int k = 0; k < kColsumSlabRows / 4; ++k) {
    const int r = r0 + 4 * k;
    v[k] = (c < C && r < R) ? g[size_t(r) * C + c] : 0.0f;
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kColsumSlabRows / 4; ++k) s += v[k];
  ws[w][lane] = s;
  __syncthreads();
  if (w == 0 && c < C) part[size_t(blockIdx.y) * C + c] = ((ws[0][lane] + ws[1][lane]) + ws[2][lane]) + ws[3][lane];
}

__global__ __launch_bounds__(64) void colsum_fin(const float* __restrict__ part, float* __restrict__ db, int C,
                                                 int slabs) {
  const int c = blockIdx.x;
  float s = 0.0f;
  for (int k = threadIdx.x; k < slabs; k += 64) s += part[size_t(k) * C + c];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
  if (threadIdx.x == 0) db[c] = s;
}

// Heads: mu = z[r][0], s = z[r][1] in standardised target units
// (y' = (y - ym) / ys).  Per row
//   loss = 1/2 (y' - mu)^2 + lambda (1/2 r^2 exp(-2 s) + s),  r = y' - mu held fixed
// averaged over the n_valid rows; the gradient goes to g (FP32) and gt (the
// head's operand type), the loss sum to *loss.
template <class T>
__global__ __launch_bounds__(256) void loss_grad(const float* __restrict__ z, const float* __restrict__ y, int n_valid,
                                                 int rows, int ld, float lambda, float ym, float ys,
                                                 float* __restrict__ g, T* __restrict__ gt,
                                                 float* __restrict__ loss) {
  // the block's rows [r0, r0 + nr) are zeroed first with consecutive lanes on
  // consecutive addresses, then the two head columns of the valid rows are set
  const int r0 = blockIdx.x * blockDim.x;
  const int nr = min(int(blockDim.x), rows - r0);
  for (int k = threadIdx.x; k < nr * ld; k += blockDim.x) {
    g[size_t(r0) * ld + k] = 0.0f;
    gt[size_t(r0) * ld + k] = T(0.0f);
  }
  __syncthreads();
  const int r = r0 + threadIdx.x;
  float l = 0.0f;
  if (r < n_valid) {
    // log-error head clamped at -15 (its gradient is zero below)
    const float mu = z[size_t(r) * ld], s_raw = z[size_t(r) * ld + 1], s = fmaxf(s_raw, -15.0f);
    const float res = (y[r] - ym) / ys - mu;
    const float e2 = __expf(-2.0f * s);
    const float inv = 1.0f / float(n_valid);
    const float g0 = -res * inv;
    const float g1 = s_raw > -15.0f ? lambda * (1.0f - res * res * e2) * inv : 0.0f;
    g[size_t(r) * ld] = g0;
    g[size_t(r) * ld + 1] = g1;
    gt[size_t(r) * ld] = T(g0);
    gt[size_t(r) * ld + 1] = T(g1);
    l = 0.5f * res * res + lambda * (0.5f * res * res * e2 + s);
  }
  // wave reduction then one atomic per wave
  for (int off = 32; off > 0; off >>= 1) l += __shfl_down(l, off);
  if ((threadIdx.x & 63) == 0) atomicAdd(loss, l);
}

// Adam on FP32 master weights w [rows][cols]; writes the operand-type copy wt
// and its transpose wtt [cols][rows] (if non-null).  mask_rows/mask_cols:
// entries beyond them are padding and stay zero.
template <class T>
__global__ __launch_bounds__(256) void adam(float* __restrict__ w, const float* __restrict__ grad,
                                            float* __restrict__ m, float* __restrict__ v, T* __restrict__ wt,
                                            T* __restrict__ wtt, int rows, int cols, int mask_rows, int mask_cols,
                                            float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(rows) * cols) return;
  const int r = int(i / cols), c = int(i % cols);
  float wi = 0.0f;
  if (r < mask_rows && c < mask_cols) {
    const float gi = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    w[i] = wi;
  }
  if (wt) wt[i] = T(wi);
  if (wtt) wtt[size_t(c) * rows + r] = T(wi);
}

// Adam over a table of parameter tensors: element gi belongs to the last
// segment whose begin is at most gi (a few segments: a linear scan).
__global__ __launch_bounds__(256) void adam_all(const AdamSeg* __restrict__ segs, int nseg, int64_t total, float lr,
                                                float b1, float b2, float eps, float c1, float c2) {
  const int64_t gi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gi >= total) return;
  int k = 0;
  while (k + 1 < nseg && gi >= segs[k + 1].begin) ++k;
  const AdamSeg sg = segs[k];
  const int64_t i = gi - sg.begin;
  const int r = int(i / sg.cols), c = int(i % sg.cols);
  float wi = 0.0f;
  if (r < sg.mask_rows && c < sg.mask_cols) {
    const float gv = sg.grad[i];
    const float mi = b1 * sg.m[i] + (1.0f - b1) * gv;
    const float vi = b2 * sg.v[i] + (1.0f - b2) * gv * gv;
    sg.m[i] = mi;
    sg.v[i] = vi;
    wi = sg.w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    sg.w[i] = wi;
  }
  if (sg.bf16_out) {
    if (sg.wt) static_cast<bf16*>(sg.wt)[i] = bf16(wi);
    if (sg.wtt) static_cast<bf16*>(sg.wtt)[size_t(c) * sg.rows + r] = bf16(wi);
  } else {
    if (sg.wt) static_cast<float*>(sg.wt)[i] = wi;
    if (sg.wtt) static_cast<float*>(sg.wtt)[size_t(c) * sg.rows + r] = wi;
  }
}

template <class T>
__global__ __launch_bounds__(256) void convert_k(const float* __restrict__ in, T* __restrict__ out,
                                                 T* __restrict__ outt, int rows, int cols) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(rows) * cols) return;
  out[i] = T(in[i]);
  if (outt) outt[size_t(i % cols) * rows + i / cols] = T(in[i]);
}

// x[r][0..ld) = standardised feature row of (event ev[r] (NULL: r), card
// cidx[r]); rows >= n are zero.
template <int NPART, int KIND>
__global__ __launch_bounds__(256) void features_k(const FeatureMap fm, const double* __restrict__ mom,
                                                  const int32_t* __restrict__ ev, const int32_t* __restrict__ cidx,
                                                  const float* __restrict__ cpar, const float* __restrict__ mean,
                                                  const float* __restrict__ istd, float* __restrict__ x, int64_t n,
                                                  int64_t rows, int ld) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  float f[kMlpMaxIn];
  if (r < n) {
    const int64_t e = ev ? int64_t(ev[r]) : r;
    const int c0 = cidx[r];
    const bool ok = c0 >= 0 && c0 < fm.ncards;           // an index out of range reads card 0, gives NaN
    const int c = ok ? c0 : 0;
    double p[NPART * 4];
    load_event<NPART>(mom, e, p);
    const float card[3] = {cpar[3 * c], cpar[3 * c + 1], cpar[3 * c + 2]};
    feature_row<NPART, KIND>(fm, p, card, f);
    standardise(f, mean, istd);
    if (!ok)
#pragma unroll
      for (int k = 0; k < kMlpMaxIn; ++k) f[k] = __builtin_nanf("");
  } else {
#pragma unroll
    for (int k = 0; k < kMlpMaxIn; ++k) f[k] = 0.0f;
  }
#pragma unroll
  for (int k = 0; k < kMlpMaxIn; ++k)
    if (k < ld) x[size_t(r) * ld + k] = f[k];
}

// Heads in target units: out[r][0] = z0 ys + ym, out[r][1] = z1 + log ys,
// further columns (ld_out > 2) copied.
__global__ __launch_bounds__(256) void heads_k(const float* __restrict__ z, int ld, int64_t n, float ym, float ys,
                                               float* __restrict__ out, int ld_out) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n) return;
  out[size_t(r) * ld_out] = z[size_t(r) * ld] * ys + ym;
  out[size_t(r) * ld_out + 1] = z[size_t(r) * ld + 1] + logf(ys);
  for (int c = 2; c < ld_out; ++c) out[size_t(r) * ld_out + c] = z[size_t(r) * ld + c];
}

// Surrogate weights where k exp(s) <= threshold; the other events are listed.
__global__ __launch_bounds__(256) void gate_k(const float* __restrict__ z, int ld, int64_t n, float ym, float ys,
                                              float k_cal, float threshold, const double* __restrict__ w_in,
                                              double* __restrict__ w_out, int32_t* __restrict__ list,
                                              unsigned int* __restrict__ count) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const float mu = z[size_t(r) * ld] * ys + ym, s = z[size_t(r) * ld + 1] + logf(ys);
  if (k_cal * __expf(s) <= threshold && isfinite(mu)) {
    w_out[r] = w_in[r] * exp(double(mu));
  } else {
    const unsigned int slot = atomicAdd(count, 1u);
    list[slot] = int32_t(r);
  }
}

// Rows [pos0, pos0 + n) of an epoch's order over the pairs of a card-major
// grid (pair j: event j % nevt, card j / nevt): each row's event and card
// index and, when y is given, its target y[j].  s.n = 0: pairs in order.
__global__ __launch_bounds__(256) void gather_pairs_k(const Shuffle s, int64_t pos0, int64_t n, int64_t nevt,
                                                      const float* __restrict__ y, int32_t* __restrict__ ev,
                                                      int32_t* __restrict__ cd, float* __restrict__ yb) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t j = shuffled(s, pos0 + r);
  ev[r] = int32_t(j % nevt);
  cd[r] = int32_t(j / nevt);
  if (y) yb[r] = y[j];
}

// Training targets y = log(w_new / w_old) (w_old = 0: y = 0).
__global__ __launch_bounds__(256) void log_ratio_k(const double* __restrict__ w_new, const double* __restrict__ w_old,
                                                   float* __restrict__ y, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double o = w_old ? w_old[i] : 1.0;
  y[i] = o != 0.0 ? float(log(w_new[i] / o)) : 0.0f;
}

// A-operand order of the fused kernels: block b of 32 output rows, chunk c
// of 16 inputs, lane l, slot s holds W[32 b + l % 32][16 c + 8 (s / 4) + 4 (l / 32) + s % 4]
// (the order in which a wave's accumulators come out, so one layer's output
// is the next layer's B operand without moving data between lanes).  hi is
// the BF16 rounding of W, lo (optional) the BF16 rounding of the remainder.
// transposed: the matrix packed is W^T (element (row, col) = w[col][row]).
__host__ __device__ __forceinline__ int64_t pack_pos(int row, int col, int nchunks) {
  const int o = col & 15;
  const int lane = (row & 31) + 32 * ((o & 7) >> 2), slot = 4 * (o >> 3) + (o & 3);
  return ((int64_t(row >> 5) * nchunks + (col >> 4)) * 64 + lane) * 8 + slot;
}

__global__ __launch_bounds__(256) void pack_k(const float* __restrict__ w, int ld, int rows_used, int cols_used,
                                              int nblocks, int nchunks, bf16* __restrict__ hi, bf16* __restrict__ lo,
                                              int transposed) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(nblocks) * nchunks * 512) return;
  const int s = int(t & 7), l = int((t >> 3) & 63);
  const int64_t q = t >> 9;
  const int c = int(q % nchunks), b = int(q / nchunks);
  const int row = 32 * b + (l & 31);
  const int col = 16 * c + 8 * (s >> 2) + 4 * (l >> 5) + (s & 3);
  float v = 0.0f;
  if (row < rows_used && col < cols_used) v = transposed ? w[size_t(col) * ld + row] : w[size_t(row) * ld + col];
  const bf16 vh = bf16(v);
  hi[t] = vh;
  if (lo) lo[t] = bf16(v - float(vh));
}

// Column sums of x and x^2 (FP64) over n rows of ld columns, added to
// sums[0..ld) and sums[ld..2 ld).
__global__ __launch_bounds__(256) void moments_k(const float* __restrict__ x, int64_t n, int ld,
                                                 double* __restrict__ sums) {
  __shared__ double part[2][kMlpMaxIn][8];
  const int c = threadIdx.x % kMlpMaxIn, q = threadIdx.x / kMlpMaxIn;   // 32 columns x 8 row groups
  double s1 = 0.0, s2 = 0.0;
  if (c < ld)
    for (int64_t r = int64_t(blockIdx.x) * 8 + q; r < n; r += int64_t(gridDim.x) * 8) {
      const double v = x[r * ld + c];
      s1 += v;
      s2 += v * v;
    }
  part[0][c][q] = s1;
  part[1][c][q] = s2;
  __syncthreads();
  if (q == 0 && c < ld) {
    double t1 = 0.0, t2 = 0.0;
    for (int k = 0; k < 8; ++k) {
      t1 += part[0][c][k];
      t2 += part[1][c][k];
    }
    atomicAdd(&sums[c], t1);
    atomicAdd(&sums[ld + c], t2);
  }
}

__global__ void zero_f64(double* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

__global__ void zero_u32(unsigned int* p) { *p = 0u; }
__global__ void zero_f32(float* p) { *p = 0.0f; }

__device__ __forceinline__ f32x16_t mfma_bf16(bf16x8_t a, bf16x8_t b, f32x16_t c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Fused inference for the 32 rows e0 .. e0+31 of one wave.  Lanes l and
// l + 32 share row l % 32 and hold complementary halves of its features.
// Transposed products H'^T = W H^T: A = packed weights, B = this wave's
// activations, so the accumulators of output block b are chunks 2b and 2b+1
// of the next B operand.  The first layer runs on the high and low BF16 parts
// of its FP32 weights and inputs (three products: hi.hi + hi.lo + lo.hi); the
// hidden layers on BF16 weights and activations as in training; the head in
// FP32 on the VALU.
struct InferWeights {
  const bf16x8_t *w0h, *w0l;
  const float* b0;
  const bf16x8_t* wh;
  const float* bh;
  const float* whead;   // rows 0 and 1, width floats each
};

template <int W, int NPART, int KIND>
__device__ __forceinline__ void infer_rows(const InferArgs& a, const InferWeights& q, int64_t e0) {
  constexpr int NB = W / 32, NC = W / 16;
  const int lane = threadIdx.x & 63, h = lane >> 5;
  const int64_t r = e0 + (lane & 31);
  const int64_t rr = r < a.n ? r : a.n - 1;

  float f[kMlpMaxIn];
  {
    const int64_t e = a.ev ? int64_t(a.ev[rr]) : rr;
    const int c0 = a.cidx[rr];
    const bool ok = c0 >= 0 && c0 < a.fm.ncards;         // an index out of range reads card 0, gives NaN
    const int c = ok ? c0 : 0;
    double p[NPART * 4];
    load_event<NPART>(a.mom, e, p);
    const float card[3] = {a.cpar[3 * c], a.cpar[3 * c + 1], a.cpar[3 * c + 2]};
    feature_row<NPART, KIND>(a.fm, p, card, f);
    standardise(f, a.mean, a.istd);
    if (!ok)
#pragma unroll
      for (int k = 0; k < kMlpMaxIn; ++k) f[k] = __builtin_nanf("");
  }
  // this lane's half of the inputs (a bitwise blend, so that the choice does
  // not become a lane-dependent index into f)
  const unsigned int pick = h ? ~0u : 0u;
  bf16x8_t xh[2], xl[2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int k = 16 * c + 8 * (s >> 2) + (s & 3);
      const unsigned int u0 = __float_as_uint(f[k]), u1 = __float_as_uint(f[k + 4]);
      const float v = __uint_as_float(u0 ^ ((u0 ^ u1) & pick));
      const bf16 vh = bf16(v);
      xh[c][s] = vh;
      xl[c][s] = bf16(v - float(vh));
    }

  bf16x8_t act[NC];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    f32x16_t acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = q.b0[32 * b + 8 * (i >> 2) + 4 * h + (i & 3)];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const bf16x8_t ah = q.w0h[(b * 2 + c) * 64 + lane];
      const bf16x8_t al = q.w0l[(b * 2 + c) * 64 + lane];
      acc = mfma_bf16(ah, xh[c], acc);
      acc = mfma_bf16(ah, xl[c], acc);
      acc = mfma_bf16(al, xh[c], acc);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) act[2 * b + (i >> 3)][i & 7] = bf16(silu(acc[i]));
  }
  for (int l = 0; l + 1 < a.nh; ++l) {
    const bf16x8_t* wl = q.wh + size_t(l) * NB * NC * 64;
    const float* bl = q.bh + size_t(l) * W;
    bf16x8_t nxt[NC];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      f32x16_t acc;
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[i] = bl[32 * b + 8 * (i >> 2) + 4 * h + (i & 3)];
#pragma unroll
      for (int c = 0; c < NC; ++c) acc = mfma_bf16(wl[(b * NC + c) * 64 + lane], act[c], acc);
#pragma unroll
      for (int i = 0; i < 16; ++i) nxt[2 * b + (i >> 3)][i & 7] = bf16(silu(acc[i]));
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) act[c] = nxt[c];
  }
  // last hidden layer, straight into the two FP32 heads
  float mu = 0.0f, sg = 0.0f;
  {
    const bf16x8_t* wl = q.wh + size_t(a.nh - 1) * NB * NC * 64;
    const float* bl = q.bh + size_t(a.nh - 1) * W;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      f32x16_t acc;
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[i] = bl[32 * b + 8 * (i >> 2) + 4 * h + (i & 3)];
#pragma unroll
      for (int c = 0; c < NC; ++c) acc = mfma_bf16(wl[(b * NC + c) * 64 + lane], act[c], acc);
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int fo = 32 * b + 8 * (i >> 2) + 4 * h + (i & 3);
        const float v = silu(acc[i]);
        mu = fmaf(v, q.whead[fo], mu);
        sg = fmaf(v, q.whead[W + fo], sg);
      }
    }
  }
  mu += __shfl_xor(mu, 32);
  sg += __shfl_xor(sg, 32);
  mu = (mu + a.bhead[0]) * a.ys + a.ym;
  sg = sg + a.bhead[1] + logf(a.ys);

  const bool mine = lane < 32 && r < a.n;
  if (a.heads && mine) {
    a.heads[2 * r] = mu;
    a.heads[2 * r + 1] = sg;
  }
  if (a.w_out) {
    bool fb = false;
    if (mine) {
      if (a.k_cal * __expf(sg) <= a.threshold && isfinite(mu))
        a.w_out[r] = a.w_in[r] * exp(double(mu));
      else
        fb = true;
    }
    if constexpr (W == 256) {
      // width 256 (one wave per SIMD): one atomic per wave with a fallback
      // row (the block-count form below measured 1.09 against 0.86 ms per 1e6
      // rows for this kernel's code generation)
      const uint64_t m = __ballot(fb);
      if (m) {                                        // wave-uniform
        unsigned int base = 0;
        if (lane == 0) base = atomicAdd(a.count, unsigned(__popcll(m)));
        base = __shfl(base, 0);
        if (fb) a.list[base + __popcll(m & ((uint64_t(1) << lane) - 1))] = int32_t(r);
      }
    } else {
      // fallback rows join the device list: the workgroup's waves count theirs
      // in LDS and one lane reserves the block's slots with a single atomic
      // (one atomic per wave contends on the counter when most waves have a
      // fallback row: 0.49 against 0.32 ms for the gated path at 8.6%)
      __shared__ unsigned int s_cnt[4];
      __shared__ unsigned int s_base;
      const uint64_t m = __ballot(fb);
      const int wid = int(threadIdx.x >> 6), nw = int(blockDim.x >> 6);
      if (lane == 0) s_cnt[wid] = unsigned(__popcll(m));
      __syncthreads();
      if (threadIdx.x == 0) {
        unsigned int tot = 0;
        for (int w = 0; w < nw; ++w) tot += s_cnt[w];
        s_base = tot ? atomicAdd(a.count, tot) : 0u;
      }
      __syncthreads();
      if (fb) {
        unsigned int off = s_base;
        for (int w = 0; w < wid; ++w) off += s_cnt[w];
        a.list[off + __popcll(m & ((uint64_t(1) << lane) - 1))] = int32_t(r);
      }
    }
  }
}

// Weights from global memory (L2-resident): one wave per 32 rows, 4 waves per
// workgroup.  Width 128 is held to 128 registers (4 waves per SIMD, no
// spills): the kernel is bound by its vector instructions, and the extra
// waves hide the weight loads (0.207 against 0.242 ms per 1e6 rows at 3
// waves).  Width 128: waves past the last row run on the clamped last row
// and write nothing (every wave reaches the gate's barriers).
template <int W, int NPART, int KIND>
__global__ __launch_bounds__(256, W == 128 ? 4 : 1) void infer_k(const InferArgs a) {
  const int64_t e0 = ((int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6) * 32;
  if constexpr (W == 256) {
    if (e0 >= a.n) return;                            // whole waves; this width's gate has no barrier
  }
  const InferWeights q{static_cast<const bf16x8_t*>(a.w0hi), static_cast<const bf16x8_t*>(a.w0lo), a.b0,
                       static_cast<const bf16x8_t*>(a.wh), a.bh, a.whead};
  infer_rows<W, NPART, KIND>(a, q, e0);
}

// ------------------------------------------------------- fused training step
// One step in two launches instead of several per layer.  train_k: per
// workgroup, row tiles of R rows in groups of 32 (lanes l and l + 32 on row
// l % 32, as in the fused inference kernel); the NF waves of a row group
// split every layer's 32-feature output blocks between them (FB blocks
// each), so that each wave's chain of dependent steps is a fraction of the
// whole network's.  Per tile:
//   - the rows' inputs: the epoch's pairs (shuffled position -> event and
//     card -> standardised features) or given input rows, and their targets;
//   - forward: each wave its blocks of each layer (the fused inference
//     kernel's arithmetic), the layer's activations exchanged through LDS,
//     the pre-activations kept in a per-wave workspace; the heads summed
//     over the waves in a fixed order;
//   - the heads' loss gradient (the loss of loss_grad), then backward: each
//     wave its blocks of each layer's input gradient, a transposed product
//     on the packed W^T with BF16 gradients (as the layered path rounds
//     them), times SiLU'(z);
//   - each layer's weight gradient G^T H over the tile's rows on the matrix
//     cores, both operands staged in LDS with rows contiguous (the K order of
//     the product): BF16 G and H for the hidden layers, as the layered path;
//     split BF16 (hi.hi + hi.lo + lo.hi, about 2^-16) for the first layer's
//     FP32 inputs.  Biases and the two FP32 heads: sums over rows on the VALU
//     of FP32 values (gradients as hi + lo BF16 parts, 2^-17).
// The sums go to this workgroup's slot of part (added over its tiles in tile
// order).  train_update_k adds the slots in workgroup order: deterministic.
template <int W>
struct TrainShape {
  static constexpr int NB = W / 32, NC = W / 16;
  static constexpr int FB = W == 128 ? 1 : 2;       // 32-feature blocks per wave
  static constexpr int NF = NB / FB;                // waves per row group
  static constexpr int RG = W == 128 ? 4 : 2;       // row groups per workgroup
  static constexpr int NWV = NF * RG;               // waves per workgroup (16 or 8)
  static constexpr int R = 32 * RG;                 // rows per tile
  static constexpr int S = R + 8;                   // LDS row stride: consecutive rows start 4 banks apart
};

int train_tile_rows(int width) { return width == 128 ? TrainShape<128>::R : TrainShape<256>::R; }
// per workgroup: each wave's pre-activations of its blocks, every layer
int64_t train_zws_floats(int width, int nh) {
  const int per = width == 128 ? TrainShape<128>::NWV * TrainShape<128>::FB : TrainShape<256>::NWV * TrainShape<256>::FB;
  return int64_t(per) * (nh + 2) * 16 * 64;              // + the first layer's inputs (16 words per lane)
}

// feature of accumulator element i of block b in lane half h
__device__ __forceinline__ int acc_feat(int b, int i, int h) { return 32 * b + 8 * (i >> 2) + 4 * h + (i & 3); }

__device__ __forceinline__ void split_bf16(float v, bf16& hi, bf16& lo) {
  hi = bf16(v);
  lo = bf16(v - float(hi));
}

// Sums over the R rows of nout outputs, by every thread of the workgroup: G
// consecutive threads per output (G a power of two up to 8, as many as the
// threads allow), each over R / G consecutive rows in order, combined by a
// fixed butterfly over the G lanes.  part8(o, r0) is output o's sum over
// rows r0 .. r0 + 7; emit(o, s) receives each total once.
template <int R, int NT, class P, class E>
__device__ __forceinline__ void group_sums(int nout, P part8, E emit) {
  int G = 1;
  while (G < 8 && G * 8 < R && nout * G * 2 <= NT) G *= 2;
  const int span = R / G;
  for (int base = 0; base < nout * G; base += NT) {       // uniform over the workgroup
    const int t = base + int(threadIdx.x), o = t / G, g = t % G;
    float s = 0.0f;
    if (o < nout)
      for (int r0 = g * span; r0 < (g + 1) * span; r0 += 8) s += part8(o, r0);
    for (int m = 1; m < G; m <<= 1) s += __shfl_xor(s, m);
    if (o < nout && g == 0) emit(o, s);
  }
}

// sum over 8 rows from r0 of hi + lo (a non-NULL: weighted by a[r])
__device__ __forceinline__ float sum8(const float* a, const bf16* hi, const bf16* lo, int r0) {
  const bf16x8_t vh = *reinterpret_cast<const bf16x8_t*>(hi + r0);
  const bf16x8_t vl = *reinterpret_cast<const bf16x8_t*>(lo + r0);
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float v = float(vh[k]) + float(vl[k]);
    s = a ? fmaf(a[r0 + k], v, s) : s + v;
  }
  return s;
}

// chunk c of a row's features (LDS [feature][row] layout) as a B operand:
// slot s holds feature 16 c + 8 (s / 4) + 4 h + s % 4, the order in which
// the accumulators of the producing layer come out
template <int S>
__device__ __forceinline__ bf16x8_t gather_chunk(const bf16 (*m)[S], int c, int h, int rl) {
  bf16x8_t v;
#pragma unroll
  for (int s = 0; s < 8; ++s) v[s] = m[16 * c + 8 * (s >> 2) + 4 * h + (s & 3)][rl];
  return v;
}

// A pointer (launder: wave-uniform; vlaunder: any value) the compiler must
// take as changed here: loads through it, and per-lane address arithmetic on
// it, stay inside the row-tile loop instead of being hoisted out of it (every
// layer's weights and addresses held across the loop would not fit in
// registers).
template <class P>
__device__ __forceinline__ P launder(P p) {
  asm volatile("" : "+s"(p));
  return p;
}
template <class V>
__device__ __forceinline__ V vlaunder(V v) {
  asm volatile("" : "+v"(v));
  return v;
}

// two BF16 values in one 32-bit word (a in the low half) and back
__device__ __forceinline__ unsigned int pack_bf16x2(bf16 a, bf16 b) {
  return unsigned(__builtin_bit_cast(unsigned short, a)) | (unsigned(__builtin_bit_cast(unsigned short, b)) << 16);
}
__device__ __forceinline__ bf16 bf16_lo(unsigned int v) { return __builtin_bit_cast(bf16, (unsigned short)(v & 0xffffu)); }
__device__ __forceinline__ bf16 bf16_hi(unsigned int v) { return __builtin_bit_cast(bf16, (unsigned short)(v >> 16)); }

// this workgroup's first tile writes its slot, later tiles add to it
__device__ __forceinline__ void put(float* p, float v, bool first) { *p = first ? v : *p + v; }

template <int W, int NPART, int KIND, bool XROWS>
__global__ __launch_bounds__(64 * TrainShape<W>::NWV, 1) void train_k(const TrainArgs a) {
  using T = TrainShape<W>;
  constexpr int NB = T::NB, NC = T::NC, FB = T::FB, NF = T::NF, NWV = T::NWV, R = T::R, S = T::S;
  __shared__ __attribute__((aligned(16))) bf16 ah_s[W][S];   // layer inputs (hi) [feature][row]
  __shared__ __attribute__((aligned(16))) bf16 al_s[W][S];   // their low parts (first layer, heads)
  __shared__ __attribute__((aligned(16))) bf16 gh_s[W][S];   // gradients (hi)
  __shared__ __attribute__((aligned(16))) bf16 gl_s[W][S];   // their low parts
  __shared__ float hpart[NF][R][2];                         // the waves' partial heads
  __shared__ float ghead[2][R];
  __shared__ float wloss[T::RG];
  const int lane = threadIdx.x & 63, h = lane >> 5;
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));   // wave-uniform
  const int rg = wv / NF, fw = wv % NF;                     // row group, feature wave
  const int rl = 32 * rg + (lane & 31);
  const int nh = a.nh;
  const bf16x8_t* w0h_ = static_cast<const bf16x8_t*>(a.w0hi);
  const bf16x8_t* w0l_ = static_cast<const bf16x8_t*>(a.w0lo);
  const bf16x8_t* wh_ = static_cast<const bf16x8_t*>(a.wh);
  const bf16x8_t* wht_ = static_cast<const bf16x8_t*>(a.wht);
  float* const zw_ = a.zws + (size_t(blockIdx.x) * NWV + wv) * size_t(nh + 2) * FB * 16 * 64;
  float* part = a.part + size_t(blockIdx.x) * a.pstride;
  const int head = nh + 1;
  float loss_acc = 0.0f;

  for (int tile = int(blockIdx.x); tile < a.tiles; tile += int(gridDim.x)) {
    const bool first = tile == int(blockIdx.x);
    const int lv = vlaunder(lane);
    const bf16x8_t* w0h = launder(w0h_) + lv;          // per-lane pointers (packed slots)
    const bf16x8_t* w0l = launder(w0l_) + lv;
    const bf16x8_t* wh = launder(wh_) + lv;
    const bf16x8_t* wht = launder(wht_) + lv;
    const float* b0 = launder(a.b0);
    const float* bh = launder(a.bh);
    const float* whead = launder(a.whead);
    const float* bhead = launder(a.bhead);
    float* zw = launder(zw_) + lv;                        // this lane's column of the workspace
    const int64_t r = int64_t(tile) * R + rl;
    const bool valid = r < a.n;
    float f[kMlpMaxIn];
    float yv;
    if constexpr (XROWS) {
      const int64_t rr = r < a.rows ? r : a.rows - 1;
#pragma unroll
      for (int k = 0; k < kMlpMaxIn; ++k) f[k] = a.x[rr * kMlpMaxIn + k];
      yv = a.y[rr];
    } else {
      const int64_t rr = valid ? r : a.n - 1;
      const int64_t j = shuffled(a.sh, a.pos0 + rr);
      const int64_t e = j % a.nevt;
      const int c = int(j / a.nevt);
      double p[NPART * 4];
      load_event<NPART>(a.mom, e, p);
      const float card[3] = {a.cpar[3 * c], a.cpar[3 * c + 1], a.cpar[3 * c + 2]};
      feature_row<NPART, KIND>(a.fm, p, card, f);
      standardise(f, a.mean, a.istd);
      yv = a.ygrid[j];
    }
    // this lane's half of the inputs, as the fused inference kernel takes it
    const unsigned int pick = h ? ~0u : 0u;
    bf16x8_t xh[2], xl[2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int k = 16 * c + 8 * (s >> 2) + (s & 3);
        const unsigned int u0 = __float_as_uint(f[k]), u1 = __float_as_uint(f[k + 4]);
        bf16 vh, vl;
        split_bf16(__uint_as_float(u0 ^ ((u0 ^ u1) & pick)), vh, vl);
        xh[c][s] = vh;
        xl[c][s] = vl;
      }

    if (fw == 0) {                                        // kept for the first layer's weight gradient
      float* xs = zw + size_t(nh + 1) * FB * 16 * 64;
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int s = 0; s < 8; s += 2) {
          xs[(c * 8 + s) * 64] = __uint_as_float(pack_bf16x2(xh[c][s], xh[c][s + 1]));
          xs[(c * 8 + s + 1) * 64] = __uint_as_float(pack_bf16x2(xl[c][s], xl[c][s + 1]));
        }
    }

    // ---------------------------------------------------------- forward
#pragma unroll
    for (int u = 0; u < FB; ++u) {
      const int b = fw * FB + u;
      f32x16_t acc;
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[i] = b0[acc_feat(b, i, h)];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const bf16x8_t wa = w0h[(b * 2 + c) * 64];
        const bf16x8_t wb = w0l[(b * 2 + c) * 64];
        acc = mfma_bf16(wa, xh[c], acc);
        acc = mfma_bf16(wa, xl[c], acc);
        acc = mfma_bf16(wb, xh[c], acc);
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        zw[(u * 16 + i) * 64] = acc[i];
        ah_s[acc_feat(b, i, h)][rl] = bf16(silu(acc[i]));
      }
    }
    __syncthreads();
    float mu = 0.0f, sg = 0.0f;
    float zl[FB][16];                                     // the last hidden layer's pre-activations
    for (int q = 0; q < nh; ++q) {
      const bool last = q + 1 == nh;
      const bf16x8_t* wl = wh + size_t(q) * NB * NC * 64;
      const float* bl = bh + size_t(q) * W;
      float* zq = zw + size_t(q + 1) * FB * 16 * 64;
      f32x16_t acc[FB];
#pragma unroll
      for (int u = 0; u < FB; ++u)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[u][i] = bl[acc_feat(fw * FB + u, i, h)];
#pragma unroll
      for (int c = 0; c < NC; ++c) {                      // input chunk by chunk from LDS
        const bf16x8_t xc = gather_chunk<S>(ah_s, c, h, rl);
#pragma unroll
        for (int u = 0; u < FB; ++u) acc[u] = mfma_bf16(wl[((fw * FB + u) * NC + c) * 64], xc, acc[u]);
      }
      bf16x8_t nxt[FB][2];
#pragma unroll
      for (int u = 0; u < FB; ++u)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          zq[(u * 16 + i) * 64] = acc[u][i];
          zl[u][i] = acc[u][i];
          nxt[u][i >> 3][i & 7] = bf16(silu(acc[u][i]));
        }
      if (last) {                                         // the last hidden layer feeds the FP32 heads
#pragma unroll
        for (int u = 0; u < FB; ++u)
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int fo = acc_feat(fw * FB + u, i, h);
            const float v = silu(zl[u][i]);
            mu = fmaf(v, whead[fo], mu);
            sg = fmaf(v, whead[W + fo], sg);
          }
        break;
      }
      __syncthreads();                                    // every wave has read this layer's inputs
#pragma unroll
      for (int u = 0; u < FB; ++u)
#pragma unroll
        for (int i = 0; i < 16; ++i) ah_s[acc_feat(fw * FB + u, i, h)][rl] = nxt[u][i >> 3][i & 7];
      __syncthreads();
    }
    mu += __shfl_xor(mu, 32);
    sg += __shfl_xor(sg, 32);
    if (lane < 32) {
      hpart[fw][rl][0] = mu;
      hpart[fw][rl][1] = sg;
    }
    __syncthreads();                                      // partial heads written; the inputs read
    mu = 0.0f;
    sg = 0.0f;
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      mu += hpart[k][rl][0];
      sg += hpart[k][rl][1];
    }
    mu += bhead[0];
    sg += bhead[1];

    // ------------------------------------------------ loss and its gradient
    float g0 = 0.0f, g1 = 0.0f, lrow = 0.0f;
    if (valid) {
      const float s = fmaxf(sg, -15.0f);               // log-error head clamped as loss_grad does
      const float res = (yv - a.ym) / a.ys - mu;
      const float e2 = __expf(-2.0f * s);
      const float inv = 1.0f / float(a.n);
      g0 = -res * inv;
      g1 = sg > -15.0f ? a.lambda * (1.0f - res * res * e2) * inv : 0.0f;
      lrow = 0.5f * res * res + a.lambda * (0.5f * res * res * e2 + s);
    }
    if (fw == 0) {
      float lw = lane < 32 ? lrow : 0.0f;
      for (int off = 32; off > 0; off >>= 1) lw += __shfl_down(lw, off);
      if (lane == 0) wloss[rg] = lw;
      if (lane < 32) {
        ghead[0][rl] = g0;
        ghead[1][rl] = g1;
      }
    }
    // the heads' FP32 input (hi / lo) and the gradient of the last hidden
    // layer's pre-activation (hi / lo), this wave's blocks
#pragma unroll
    for (int u = 0; u < FB; ++u)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int fo = acc_feat(fw * FB + u, i, h);
        const float z = zl[u][i];
        split_bf16(silu(z), ah_s[fo][rl], al_s[fo][rl]);
        split_bf16((g0 * whead[fo] + g1 * whead[W + fo]) * silu_grad(z), gh_s[fo][rl], gl_s[fo][rl]);
      }
    __syncthreads();
    if (threadIdx.x == 0) {
      float t = 0.0f;
      for (int k = 0; k < T::RG; ++k) t += wloss[k];
      loss_acc += t;
    }
    // heads: dW[j][f] = sum_r g_j h_f (outputs 0 .. 2W-1), db[j] = sum_r g_j (outputs 2W, 2W+1)
    group_sums<R, NWV * 64>(
        2 * W + 2,
        [&](int o, int r0) {
          if (o >= 2 * W) {
            float s = 0.0f;
#pragma unroll
            for (int k = 0; k < 8; ++k) s += ghead[o - 2 * W][r0 + k];
            return s;
          }
          return sum8(ghead[o / W], ah_s[o % W], al_s[o % W], r0);
        },
        [&](int o, float v) {
          put(part + (o < 2 * W ? a.off_w[head] + o : a.off_b[head] + (o - 2 * W)), v, first);
        });

    // ------------------------------------------------- hidden layers, backward
    // LDS holds G of layer l (hi / lo); per layer: H of its input to LDS, the
    // weight-gradient tiles and bias sums, then this wave's blocks of the
    // input gradient (bf16(G) W) SiLU'(z), a transposed product on W^T, into
    // LDS as the next layer's G.
    unsigned int xs_w[16];                                      // the first layer's inputs, packed
    for (int l = nh; l >= 1; --l) {
      const float* zp = zw + size_t(l - 1) * FB * 16 * 64;     // pre-activation entering layer l
      float zv[FB][16];
#pragma unroll
      for (int u = 0; u < FB; ++u)
#pragma unroll
        for (int i = 0; i < 16; ++i) zv[u][i] = zp[(u * 16 + i) * 64];
      __syncthreads();                                          // the previous sums are done with LDS
#pragma unroll
      for (int u = 0; u < FB; ++u)
#pragma unroll
        for (int i = 0; i < 16; ++i) ah_s[acc_feat(fw * FB + u, i, h)][rl] = bf16(silu(zv[u][i]));
      __syncthreads();
      for (int t = wv; t < NB * NB; t += NWV) {
        const int ob = t / NB, ib = t % NB;
        f32x16_t acc = {};
#pragma unroll
        for (int k0 = 0; k0 < R; k0 += 16) {
          const bf16x8_t av = *reinterpret_cast<const bf16x8_t*>(&gh_s[32 * ob + (lane & 31)][k0 + 8 * h]);
          const bf16x8_t bv = *reinterpret_cast<const bf16x8_t*>(&ah_s[32 * ib + (lane & 31)][k0 + 8 * h]);
          acc = mfma_bf16(av, bv, acc);
        }
        float* pw = part + a.off_w[l] + size_t(32 * ib + (lane & 31));
#pragma unroll
        for (int i = 0; i < 16; ++i) put(pw + size_t(32 * ob + 8 * (i >> 2) + 4 * h + (i & 3)) * W, acc[i], first);
      }
      group_sums<R, NWV * 64>(
          W, [&](int o, int r0) { return sum8(nullptr, gh_s[o], gl_s[o], r0); },
          [&](int o, float v) { put(part + a.off_b[l] + o, v, first); });
      float gn[FB][16];
      {
        const bf16x8_t* wt = wht + size_t(l - 1) * NB * NC * 64;
        f32x16_t acc[FB] = {};
#pragma unroll
        for (int c = 0; c < NC; ++c) {                    // this row's G chunk by chunk from LDS
          const bf16x8_t gc = gather_chunk<S>(gh_s, c, h, rl);
#pragma unroll
          for (int u = 0; u < FB; ++u) acc[u] = mfma_bf16(wt[((fw * FB + u) * NC + c) * 64], gc, acc[u]);
        }
#pragma unroll
        for (int u = 0; u < FB; ++u)
#pragma unroll
          for (int i = 0; i < 16; ++i) gn[u][i] = acc[u][i] * silu_grad(zv[u][i]);
      }
      if (l == 1 && fw == 0) {                                  // loaded early for the first layer
        const float* xs = zw + size_t(nh + 1) * FB * 16 * 64;
#pragma unroll
        for (int k = 0; k < 16; ++k) xs_w[k] = __float_as_uint(xs[k * 64]);
      }
      __syncthreads();                                          // every read of this layer's G is done
#pragma unroll
      for (int u = 0; u < FB; ++u)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int fo = acc_feat(fw * FB + u, i, h);
          split_bf16(gn[u][i], gh_s[fo][rl], gl_s[fo][rl]);
        }
    }

    // --------------------------------------------------------- first layer
    if (fw == 0) {
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int s = 0; s < 8; s += 2) {
          const unsigned int ph = xs_w[c * 8 + s], pl = xs_w[c * 8 + s + 1];
          const int k = 16 * c + 8 * (s >> 2) + 4 * h + (s & 3);
          ah_s[k][rl] = bf16_lo(ph);
          ah_s[k + 1][rl] = bf16_hi(ph);
          al_s[k][rl] = bf16_lo(pl);
          al_s[k + 1][rl] = bf16_hi(pl);
        }
    }
    __syncthreads();
    for (int ob = wv; ob < NB; ob += NWV) {
      f32x16_t acc = {};
#pragma unroll
      for (int k0 = 0; k0 < R; k0 += 16) {
        const bf16x8_t ga = *reinterpret_cast<const bf16x8_t*>(&gh_s[32 * ob + (lane & 31)][k0 + 8 * h]);
        const bf16x8_t gb = *reinterpret_cast<const bf16x8_t*>(&gl_s[32 * ob + (lane & 31)][k0 + 8 * h]);
        const bf16x8_t xa = *reinterpret_cast<const bf16x8_t*>(&ah_s[lane & 31][k0 + 8 * h]);
        const bf16x8_t xb = *reinterpret_cast<const bf16x8_t*>(&al_s[lane & 31][k0 + 8 * h]);
        acc = mfma_bf16(ga, xa, acc);
        acc = mfma_bf16(ga, xb, acc);
        acc = mfma_bf16(gb, xa, acc);
      }
      float* pw = part + a.off_w[0] + (lane & 31);
#pragma unroll
      for (int i = 0; i < 16; ++i) put(pw + size_t(32 * ob + 8 * (i >> 2) + 4 * h + (i & 3)) * kMlpMaxIn, acc[i], first);
    }
    group_sums<R, NWV * 64>(
        W, [&](int o, int r0) { return sum8(nullptr, gh_s[o], gl_s[o], r0); },
        [&](int o, float v) { put(part + a.off_b[0] + o, v, first); });
    __syncthreads();                                            // LDS free for the next tile
  }
  if (threadIdx.x == 0) part[a.total] = loss_acc;
}

// Per parameter element: the workgroups' sums in workgroup order into the
// gradient buffer; with adam, the step of adam_all and every copy of the new
// value (operand copies, packed forward and transposed orders, contiguous
// hidden biases).  Element total: the loss sum.  Padding elements get a zero
// gradient and stay zero.
__global__ __launch_bounds__(256) void train_update_k(const AdamSeg* __restrict__ segs, const PackSeg* __restrict__ pk,
                                                      int nseg, int64_t total, const float* __restrict__ part,
                                                      int groups, int64_t pstride, float* __restrict__ loss, int adam,
                                                      float lr, float b1, float b2, float eps, float c1, float c2) {
  // the segment tables in LDS: the lookup below reads them in a dependent
  // chain, which from global memory costs a round trip per segment
  __shared__ AdamSeg s_seg[2 * kTrainMaxLayers];
  __shared__ PackSeg s_pk[2 * kTrainMaxLayers];
  for (int k = int(threadIdx.x); k < nseg; k += int(blockDim.x)) {
    s_seg[k] = segs[k];
    s_pk[k] = pk[k];
  }
  __syncthreads();
  const int64_t gi = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gi > total) return;
  if (gi == total) {
    float s = 0.0f;
    for (int g = 0; g < groups; ++g) s += part[size_t(g) * pstride + total];
    *loss = s;
    return;
  }
  int k = 0;
  while (k + 1 < nseg && gi >= s_seg[k + 1].begin) ++k;
  const AdamSeg sg = s_seg[k];
  const PackSeg pq = s_pk[k];
  const int64_t i = gi - sg.begin;
  const int r = int(i / sg.cols), c = int(i % sg.cols);
  const bool used = r < sg.mask_rows && c < sg.mask_cols;
  // the slots' loads in batches of 32 ahead of their additions (in slot order)
  float gv = 0.0f;
  if (used) {
    for (int g = 0; g < groups; g += 32) {
      float v[32];
#pragma unroll
      for (int k = 0; k < 32; ++k) v[k] = g + k < groups ? part[size_t(g + k) * pstride + gi] : 0.0f;
#pragma unroll
      for (int k = 0; k < 32; ++k) gv += v[k];
    }
  }
  pq.grad[i] = gv;
  if (!adam) return;
  float wi = 0.0f;
  if (used) {
    const float mi = b1 * sg.m[i] + (1.0f - b1) * gv;
    const float vi = b2 * sg.v[i] + (1.0f - b2) * gv * gv;
    sg.m[i] = mi;
    sg.v[i] = vi;
    wi = sg.w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    sg.w[i] = wi;
  }
  if (sg.bf16_out) {
    if (sg.wt) static_cast<bf16*>(sg.wt)[i] = bf16(wi);
    if (sg.wtt) static_cast<bf16*>(sg.wtt)[size_t(c) * sg.rows + r] = bf16(wi);
  } else {
    if (sg.wt) static_cast<float*>(sg.wt)[i] = wi;
    if (sg.wtt) static_cast<float*>(sg.wtt)[size_t(c) * sg.rows + r] = wi;
  }
  if (pq.hi) {
    const int64_t t = pack_pos(r, c, pq.nchunks);
    bf16 vh, vl;
    split_bf16(wi, vh, vl);
    static_cast<bf16*>(pq.hi)[t] = vh;
    if (pq.lo) static_cast<bf16*>(pq.lo)[t] = vl;
  }
  if (pq.tr) static_cast<bf16*>(pq.tr)[pack_pos(c, r, pq.tchunks)] = bf16(wi);
  if (pq.bias) pq.bias[c] = wi;
}

// ----------------------------------------------------------------- launchers
static unsigned blocks_for(int64_t n, int b = 256) { return unsigned((n + b - 1) / b); }

// K chunks of one product: one unless K is long (weight gradients, K = batch
// rows) and a workspace of chunks x M x N floats is given; then enough
// chunks of at least 128 K values each (a multiple of kstep) to bring the
// waves near 1024, at most 32.
static int k_chunk(int tiles, int M, int N, int K, int kstep, int64_t work_elems, int* chunks) {
  int c = 1;
  if (work_elems > 0 && K >= 1024) {
    c = std::min(32, std::min(K / 128, std::max(1, 1024 / tiles)));
    while (c > 1 && int64_t(c) * M * N > work_elems) c /= 2;
  }
  int kc = (K + c - 1) / c;
  kc = (kc + kstep - 1) / kstep * kstep;
  *chunks = (K + kc - 1) / kc;
  return kc;
}

template <class TO>
static void gemm_launch(int tin, const void* A, const void* B, int M, int N, int K, const float* bias, float* Cf,
                        void* Ct, int act, float* work, int64_t work_elems, hipStream_t s) {
  const bool mfma = M % 32 == 0 && N % 32 == 0 && K % (tin == kMlpFP32 ? 8 : 16) == 0;
  if (!mfma) {                      // FP32 of any shape (BF16 shapes are checked by the caller)
    hipLaunchKernelGGL(gemm_nt_f32<TO>, dim3(blocks_for(int64_t(M) * N)), dim3(256), 0, s,
                       static_cast<const float*>(A), static_cast<const float*>(B), M, N, K, bias, Cf,
                       static_cast<TO*>(Ct), act);
    return;
  }
  const int tiles = (M / 32) * (N / 32);
  int chunks = 1;
  const int kc = k_chunk(tiles, M, N, K, tin == kMlpFP32 ? 8 : 16, work_elems, &chunks);
  float* part = chunks > 1 ? work : nullptr;
  const dim3 grid{unsigned(tiles), unsigned(chunks), 1u};
  if (tin == kMlpSplit)
    hipLaunchKernelGGL(gemm_nt_split<TO>, grid, dim3(64), 0, s, static_cast<const float*>(A),
                       static_cast<const float*>(B), M, N, K, kc, bias, Cf, static_cast<TO*>(Ct), act, part);
  else if (tin == kMlpBF16)
    hipLaunchKernelGGL(gemm_nt_bf16<TO>, grid, dim3(64), 0, s, static_cast<const bf16*>(A),
                       static_cast<const bf16*>(B), M, N, K, kc, bias, Cf, static_cast<TO*>(Ct), act, part);
  else
    hipLaunchKernelGGL(gemm_nt_f32m<TO>, grid, dim3(64), 0, s, static_cast<const float*>(A),
                       static_cast<const float*>(B), M, N, K, kc, bias, Cf, static_cast<TO*>(Ct), act, part);
  if (part)
    hipLaunchKernelGGL(ksum_k<TO>, dim3(blocks_for(int64_t(M) * N)), dim3(256), 0, s, part, chunks, M, N, bias, Cf,
                       static_cast<TO*>(Ct), act);
}

hipError_t mlp_gemm(int tin, int tout, const void* A, const void* B, int M, int N, int K, const float* bias,
                    float* Cf, void* Ct, int act, float* work, int64_t work_elems, hipStream_t s) {
  if (tin != kMlpFP32 && (M % 32 || N % 32 || K % 16)) return hipErrorInvalidValue;
  if (tout == kMlpBF16)
    gemm_launch<bf16>(tin, A, B, M, N, K, bias, Cf, Ct, act, work, work_elems, s);
  else
    gemm_launch<float>(tin, A, B, M, N, K, bias, Cf, Ct, act, work, work_elems, s);
  return hipGetLastError();
}

hipError_t mlp_transpose(int tin, int tout, const void* in, void* out, int R, int C, hipStream_t s) {
  const dim3 grid((C + 31) / 32, (R + 31) / 32);
  if (tin == kMlpFP32 && tout == kMlpBF16)
    hipLaunchKernelGGL((transpose_k<float, bf16>), grid, dim3(256), 0, s, static_cast<const float*>(in),
                       static_cast<bf16*>(out), R, C);
  else if (tin == kMlpFP32)
    hipLaunchKernelGGL((transpose_k<float, float>), grid, dim3(256), 0, s, static_cast<const float*>(in),
                       static_cast<float*>(out), R, C);
  else if (tout == kMlpBF16)
    hipLaunchKernelGGL((transpose_k<bf16, bf16>), grid, dim3(256), 0, s, static_cast<const bf16*>(in),
                       static_cast<bf16*>(out), R, C);
  else
    hipLaunchKernelGGL((transpose_k<bf16, float>), grid, dim3(256), 0, s, static_cast<const bf16*>(in),
                       static_cast<float*>(out), R, C);
  return hipGetLastError();
}

hipError_t mlp_silu_bwd(int tout, const float* dh, const float* z, float* g, void* gt, int64_t n, hipStream_t s) {
  if (tout == kMlpBF16)
    hipLaunchKernelGGL(silu_bwd<bf16>, dim3(blocks_for(n)), dim3(256), 0, s, dh, z, g, static_cast<bf16*>(gt), n);
  else
    hipLaunchKernelGGL(silu_bwd<float>, dim3(blocks_for(n)), dim3(256), 0, s, dh, z, g, static_cast<float*>(gt), n);
  return hipGetLastError();
}

hipError_t mlp_colsum(const float* g, float* db, int R, int C, float* work, int64_t work_elems, hipStream_t s) {
  const int64_t slabs = (int64_t(R) + kColsumSlabRows - 1) / kColsumSlabRows;
  if (work && slabs >= 1 && slabs <= 65535 && slabs * C <= work_elems) {
    hipLaunchKernelGGL(colsum_part, dim3((C + 63) / 64, unsigned(slabs)), dim3(256), 0, s, g, work, R, C);
    hipLaunchKernelGGL(colsum_fin, dim3(C), dim3(64), 0, s, work, db, C, int(slabs));
  } else {
    hipLaunchKernelGGL(colsum, dim3(C), dim3(256), 0, s, g, db, R, C);
  }
  return hipGetLastError();
}

hipError_t mlp_loss_grad(int tout, const float* z, const float* y, int n_valid, int rows, int ld, float lambda,
                         float ym, float ys, float* g, void* gt, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(zero_f32, dim3(1), dim3(1), 0, s, loss);
  if (tout == kMlpBF16)
    hipLaunchKernelGGL(loss_grad<bf16>, dim3(blocks_for(rows)), dim3(256), 0, s, z, y, n_valid, rows, ld, lambda, ym,
                       ys, g, static_cast<bf16*>(gt), loss);
  else
    hipLaunchKernelGGL(loss_grad<float>, dim3(blocks_for(rows)), dim3(256), 0, s, z, y, n_valid, rows, ld, lambda, ym,
                       ys, g, static_cast<float*>(gt), loss);
  return hipGetLastError();
}

hipError_t mlp_adam(int tout, float* w, const float* grad, float* m, float* v, void* wt, void* wtt, int rows,
                    int cols, int mask_rows, int mask_cols, float lr, float b1, float b2, float eps, float c1,
                    float c2, hipStream_t s) {
  const int64_t n = int64_t(rows) * cols;
  if (tout == kMlpBF16)
    hipLaunchKernelGGL(adam<bf16>, dim3(blocks_for(n)), dim3(256), 0, s, w, grad, m, v, static_cast<bf16*>(wt),
                       static_cast<bf16*>(wtt), rows, cols, mask_rows, mask_cols, lr, b1, b2, eps, c1, c2);
  else
    hipLaunchKernelGGL(adam<float>, dim3(blocks_for(n)), dim3(256), 0, s, w, grad, m, v, static_cast<float*>(wt),
                       static_cast<float*>(wtt), rows, cols, mask_rows, mask_cols, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t mlp_adam_all(const AdamSeg* segs, int nseg, int64_t total, float lr, float b1, float b2, float eps, float c1,
                        float c2, hipStream_t s) {
  if (!segs || nseg < 1 || total < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(adam_all, dim3(blocks_for(total)), dim3(256), 0, s, segs, nseg, total, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t mlp_convert(int tout, const float* in, void* out, void* outt, int rows, int cols, hipStream_t s) {
  const int64_t n = int64_t(rows) * cols;
  if (tout == kMlpBF16)
    hipLaunchKernelGGL(convert_k<bf16>, dim3(blocks_for(n)), dim3(256), 0, s, in, static_cast<bf16*>(out),
                       static_cast<bf16*>(outt), rows, cols);
  else
    hipLaunchKernelGGL(convert_k<float>, dim3(blocks_for(n)), dim3(256), 0, s, in, static_cast<float*>(out),
                       static_cast<float*>(outt), rows, cols);
  return hipGetLastError();
}

hipError_t mlp_features(const FeatureMap& fm, const double* mom, const int32_t* ev, const int32_t* cidx,
                        const float* cpar, const float* mean, const float* istd, float* x, int64_t n, int64_t rows,
                        int ld, hipStream_t s) {
  const dim3 g(blocks_for(rows)), b(256);
  if (fm.npart == 4 && fm.kind == kFeatRaw)
    hipLaunchKernelGGL((features_k<4, kFeatRaw>), g, b, 0, s, fm, mom, ev, cidx, cpar, mean, istd, x, n, rows, ld);
  else if (fm.npart == 4)
    hipLaunchKernelGGL((features_k<4, kFeatPhys>), g, b, 0, s, fm, mom, ev, cidx, cpar, mean, istd, x, n, rows, ld);
  else if (fm.npart == 5 && fm.kind == kFeatRaw)
    hipLaunchKernelGGL((features_k<5, kFeatRaw>), g, b, 0, s, fm, mom, ev, cidx, cpar, mean, istd, x, n, rows, ld);
  else if (fm.npart == 5)
    hipLaunchKernelGGL((features_k<5, kFeatPhys>), g, b, 0, s, fm, mom, ev, cidx, cpar, mean, istd, x, n, rows, ld);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t mlp_heads(const float* z, int ld, int64_t n, float ym, float ys, float* out, int ld_out, hipStream_t s) {
  hipLaunchKernelGGL(heads_k, dim3(blocks_for(n)), dim3(256), 0, s, z, ld, n, ym, ys, out, ld_out);
  return hipGetLastError();
}

hipError_t mlp_gather_pairs(const Shuffle& sh, int64_t pos0, int64_t n, int64_t nevt, const float* y, int32_t* ev,
                            int32_t* cd, float* yb, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_pairs_k, dim3(blocks_for(n)), dim3(256), 0, s, sh, pos0, n, nevt, y, ev, cd, yb);
  return hipGetLastError();
}

hipError_t mlp_log_ratio(const double* w_new, const double* w_old, float* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(log_ratio_k, dim3(blocks_for(n)), dim3(256), 0, s, w_new, w_old, y, n);
  return hipGetLastError();
}

hipError_t mlp_gate(const float* z, int ld, int64_t n, float ym, float ys, float k_cal, float threshold,
                    const double* w_in, double* w_out, int32_t* list, unsigned int* count, hipStream_t s) {
  hipLaunchKernelGGL(zero_u32, dim3(1), dim3(1), 0, s, count);
  hipLaunchKernelGGL(gate_k, dim3(blocks_for(n)), dim3(256), 0, s, z, ld, n, ym, ys, k_cal, threshold, w_in, w_out,
                     list, count);
  return hipGetLastError();
}

hipError_t mlp_pack(const float* w, int ld, int rows_used, int cols_used, int nblocks, int nchunks, void* hi,
                    void* lo, hipStream_t s, bool transposed) {
  hipLaunchKernelGGL(pack_k, dim3(blocks_for(int64_t(nblocks) * nchunks * 512)), dim3(256), 0, s, w, ld, rows_used,
                     cols_used, nblocks, nchunks, static_cast<bf16*>(hi), static_cast<bf16*>(lo), int(transposed));
  return hipGetLastError();
}

hipError_t mlp_moments(const float* x, int64_t n, int ld, double* sums, bool clear, hipStream_t s) {
  if (ld < 1 || ld > kMlpMaxIn) return hipErrorInvalidValue;
  if (clear) hipLaunchKernelGGL(zero_f64, dim3(1), dim3(64), 0, s, sums, 2 * ld);
  if (n > 0) {
    const int64_t groups = (n + 7) / 8;
    const unsigned grid = unsigned(groups < 4096 ? groups : 4096);
    hipLaunchKernelGGL(moments_k, dim3(grid), dim3(256), 0, s, x, n, ld, sums);
  }
  return hipGetLastError();
}

template <int W>
static hipError_t infer_launch(const InferArgs& a, hipStream_t s) {
  const dim3 g(blocks_for(a.n, 4 * 32)), b(256);      // 4 waves x 32 rows per workgroup
  if (a.fm.npart == 4 && a.fm.kind == kFeatRaw)
    hipLaunchKernelGGL((infer_k<W, 4, kFeatRaw>), g, b, 0, s, a);
  else if (a.fm.npart == 4)
    hipLaunchKernelGGL((infer_k<W, 4, kFeatPhys>), g, b, 0, s, a);
  else if (a.fm.npart == 5 && a.fm.kind == kFeatRaw)
    hipLaunchKernelGGL((infer_k<W, 5, kFeatRaw>), g, b, 0, s, a);
  else if (a.fm.npart == 5)
    hipLaunchKernelGGL((infer_k<W, 5, kFeatPhys>), g, b, 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t mlp_infer(int width, const InferArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (a.nh < 1 || a.nh > kMlpMaxHidden) return hipErrorInvalidValue;
  if (a.w_out) hipLaunchKernelGGL(zero_u32, dim3(1), dim3(1), 0, s, a.count);
  if (width == 128) return infer_launch<128>(a, s);
  if (width == 256) return infer_launch<256>(a, s);
  return hipErrorInvalidValue;
}

template <int W>
static hipError_t train_launch(const TrainArgs& a, hipStream_t s) {
  const dim3 g(unsigned(a.groups)), b(64 * TrainShape<W>::NWV);
  if (a.x)
    hipLaunchKernelGGL((train_k<W, 4, kFeatRaw, true>), g, b, 0, s, a);
  else if (a.fm.npart == 4 && a.fm.kind == kFeatRaw)
    hipLaunchKernelGGL((train_k<W, 4, kFeatRaw, false>), g, b, 0, s, a);
  else if (a.fm.npart == 4)
    hipLaunchKernelGGL((train_k<W, 4, kFeatPhys, false>), g, b, 0, s, a);
  else if (a.fm.npart == 5 && a.fm.kind == kFeatRaw)
    hipLaunchKernelGGL((train_k<W, 5, kFeatRaw, false>), g, b, 0, s, a);
  else if (a.fm.npart == 5)
    hipLaunchKernelGGL((train_k<W, 5, kFeatPhys, false>), g, b, 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t mlp_train_grads(int width, const TrainArgs& a, hipStream_t s) {
  if (a.n <= 0 || a.nh < 1 || a.nh > kMlpMaxHidden || a.groups < 1 || a.groups > kTrainMaxGroups ||
      a.tiles < a.groups || int64_t(a.tiles) * train_tile_rows(width) < a.n || (a.x && (!a.y || a.rows < 1)) ||
      (!a.x && (!a.mom || !a.cpar || !a.ygrid || a.nevt < 1)))
    return hipErrorInvalidValue;
  if (width == 128) return train_launch<128>(a, s);
  if (width == 256) return train_launch<256>(a, s);
  return hipErrorInvalidValue;
}

hipError_t mlp_train_update(const AdamSeg* segs, const PackSeg* pk, int nseg, int64_t total, const float* part,
                            int groups, int64_t pstride, float* loss, int adam, float lr, float b1, float b2,
                            float eps, float c1, float c2, hipStream_t s) {
  if (!segs || !pk || nseg < 1 || nseg > 2 * kTrainMaxLayers || total < 1 || groups < 1 || pstride <= total)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(train_update_k, dim3(blocks_for(total + 1)), dim3(256), 0, s, segs, pk, nseg, total, part, groups,
                     pstride, loss, adam, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace rwgt
