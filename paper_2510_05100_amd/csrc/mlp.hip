// Kernels of the learned surrogate: a multilayer perceptron (SiLU hidden
// layers) predicting the log of the reweighting ratio and the log of its own
// error, trained and evaluated on the GPU.
//
//   gemm_nt    C[M x N] = A[M x K] . B[N x K]^T (row-major, K contiguous), FP32
//              accumulation; BF16 operands on v_mfma_f32_32x32x16_bf16 (one
//              wave per 32 x 32 tile) or FP32 operands on the VALU (the
//              gradient-check form).  Epilogue: + bias, the FP32 result and/or
//              the SiLU (or identity) in the operand type for the next layer.
//   silu_bwd   G = dH * silu'(Z)
//   colsum     db = sum over rows of G
//   loss_grad  Gaussian-error loss of the two heads and its gradient
//   adam       FP32 master weights, moments, and the operand-type copies W, W^T
//   features   standardised [momenta, card parameters] rows
//   gate       w' = w exp(mu) where the predicted error is small; the others
//              are listed for the exact path
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mlp.h"

namespace rwgt {

typedef __bf16 bf16;
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_grad(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

__global__ __launch_bounds__(64) void gemm_nt_bf16(const bf16* __restrict__ A, const bf16* __restrict__ B, int M,
                                                   int N, int K, const float* __restrict__ bias,
                                                   float* __restrict__ Cf, bf16* __restrict__ Ct, int act) {
  const int ntn = N / 32;
  const int tm = blockIdx.x / ntn, tn = blockIdx.x % ntn;
  const int l = threadIdx.x;
  const bf16* a_row = A + size_t(tm * 32 + (l & 31)) * K + 8 * (l >> 5);
  const bf16* b_row = B + size_t(tn * 32 + (l & 31)) * K + 8 * (l >> 5);
  f32x16_t acc = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(a_row + k0);
    const bf16x8_t b = *reinterpret_cast<const bf16x8_t*>(b_row + k0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  const int col = tn * 32 + (l & 31);
  const float bb = bias ? bias[col] : 0.0f;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int row = tm * 32 + 8 * (i >> 2) + 4 * (l >> 5) + (i & 3);
    const float v = acc[i] + bb;
    if (Cf) Cf[size_t(row) * N + col] = v;
    if (Ct) Ct[size_t(row) * N + col] = bf16(act ? silu(v) : v);
  }
}

__global__ __launch_bounds__(256) void gemm_nt_f32(const float* __restrict__ A, const float* __restrict__ B, int M,
                                                   int N, int K, const float* __restrict__ bias,
                                                   float* __restrict__ Cf, float* __restrict__ Ct, int act) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(M) * N) return;
  const int row = int(idx / N), col = int(idx % N);
  const float* a = A + size_t(row) * K;
  const float* b = B + size_t(col) * K;
  float s = 0.0f;
  for (int k = 0; k < K; ++k) s = fmaf(a[k], b[k], s);
  const float v = s + (bias ? bias[col] : 0.0f);
  if (Cf) Cf[idx] = v;
  if (Ct) Ct[idx] = act ? silu(v) : v;
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

// Heads: mu = z[r][0] (log ratio), s = z[r][1] (log of its error).  Per row
//   loss = 1/2 (y - mu)^2 + lambda (1/2 r^2 exp(-2 s) + s),  r = y - mu held fixed
// averaged over the n_valid rows; the gradient goes to g (both as FP32 and in
// the operand type), the loss sum to *loss.
template <class T>
__global__ __launch_bounds__(256) void loss_grad(const float* __restrict__ z, const float* __restrict__ y, int n_valid,
                                                 int rows, int ld, float lambda, float* __restrict__ g,
                                                 T* __restrict__ gt, float* __restrict__ loss) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  float l = 0.0f;
  for (int c = 0; c < ld; ++c) {
    g[size_t(r) * ld + c] = 0.0f;
    gt[size_t(r) * ld + c] = T(0.0f);
  }
  if (r < n_valid) {
    // log-error head clamped at -15 (its gradient is zero below)
    const float mu = z[size_t(r) * ld], s_raw = z[size_t(r) * ld + 1], s = fmaxf(s_raw, -15.0f);
    const float res = y[r] - mu;
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
// and its transpose wtt [cols][rows] (if non-null).  mask_rows: rows beyond it
// are padding and stay zero.
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

template <class T>
__global__ __launch_bounds__(256) void convert_k(const float* __restrict__ in, T* __restrict__ out,
                                                 T* __restrict__ outt, int rows, int cols) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(rows) * cols) return;
  out[i] = T(in[i]);
  if (outt) outt[size_t(i % cols) * rows + i / cols] = T(in[i]);
}

// x[r][0..n_in) = (raw - mean) / std, raw = [momenta of event ev[r] (npart*4),
// params of card cidx[r] (nparam)], padded with zeros to ld columns; rows
// >= n are zero.
template <class T>
__global__ __launch_bounds__(256) void features_k(const double* __restrict__ mom, int npart,
                                                  const int32_t* __restrict__ ev, const int32_t* __restrict__ cidx,
                                                  const float* __restrict__ cpar, int nparam,
                                                  const float* __restrict__ mean, const float* __restrict__ stdv,
                                                  T* __restrict__ x, int64_t n, int64_t rows, int ld) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int nin = npart * 4 + nparam;
  for (int c = 0; c < ld; ++c) {
    float v = 0.0f;
    if (r < n && c < nin) {
      const int64_t e = ev ? ev[r] : r;
      const float raw = c < npart * 4 ? float(mom[e * npart * 4 + c]) : cpar[size_t(cidx[r]) * nparam + c - npart * 4];
      v = (raw - mean[c]) / stdv[c];
    }
    x[size_t(r) * ld + c] = T(v);
  }
}

// Surrogate weights where k exp(s) <= threshold; the other events are listed.
__global__ __launch_bounds__(256) void gate_k(const float* __restrict__ z, int ld, int64_t n, float k_cal,
                                              float threshold, const double* __restrict__ w_in,
                                              double* __restrict__ w_out, int32_t* __restrict__ list,
                                              unsigned int* __restrict__ count) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const float mu = z[size_t(r) * ld], s = z[size_t(r) * ld + 1];
  if (k_cal * __expf(s) <= threshold && isfinite(mu)) {
    w_out[r] = w_in[r] * exp(double(mu));
  } else {
    const unsigned int slot = atomicAdd(count, 1u);
    list[slot] = int32_t(r);
  }
}

// Training targets y = log(w_new / w_old) (w_old = 0: y = 0).
__global__ __launch_bounds__(256) void log_ratio_k(const double* __restrict__ w_new, const double* __restrict__ w_old,
                                                   float* __restrict__ y, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double o = w_old ? w_old[i] : 1.0;
  y[i] = o != 0.0 ? float(log(w_new[i] / o)) : 0.0f;
}

__global__ void zero_u32(unsigned int* p) { *p = 0u; }
__global__ void zero_f32(float* p) { *p = 0.0f; }

// ----------------------------------------------------------------- launchers
static unsigned blocks_for(int64_t n, int b = 256) { return unsigned((n + b - 1) / b); }

hipError_t mlp_gemm(int mode, const void* A, const void* B, int M, int N, int K, const float* bias, float* Cf,
                    void* Ct, int act, hipStream_t s) {
  if (M % 32 || N % 32 || K % 16) return hipErrorInvalidValue;
  if (mode == kMlpBF16) {
    hipLaunchKernelGGL(gemm_nt_bf16, dim3((M / 32) * (N / 32)), dim3(64), 0, s, static_cast<const bf16*>(A),
                       static_cast<const bf16*>(B), M, N, K, bias, Cf, static_cast<bf16*>(Ct), act);
  } else {
    hipLaunchKernelGGL(gemm_nt_f32, dim3(blocks_for(int64_t(M) * N)), dim3(256), 0, s,
                       static_cast<const float*>(A), static_cast<const float*>(B), M, N, K, bias, Cf,
                       static_cast<float*>(Ct), act);
  }
  return hipGetLastError();
}

hipError_t mlp_transpose(int mode, const void* in, bool in_f32, void* out, int R, int C, hipStream_t s) {
  const dim3 grid((C + 31) / 32, (R + 31) / 32);
  if (mode == kMlpBF16) {
    if (in_f32)
      hipLaunchKernelGGL((transpose_k<float, bf16>), grid, dim3(256), 0, s, static_cast<const float*>(in),
                         static_cast<bf16*>(out), R, C);
    else
      hipLaunchKernelGGL((transpose_k<bf16, bf16>), grid, dim3(256), 0, s, static_cast<const bf16*>(in),
                         static_cast<bf16*>(out), R, C);
  } else {
    hipLaunchKernelGGL((transpose_k<float, float>), grid, dim3(256), 0, s, static_cast<const float*>(in),
                       static_cast<float*>(out), R, C);
  }
  return hipGetLastError();
}

hipError_t mlp_silu_bwd(int mode, const float* dh, const float* z, float* g, void* gt, int64_t n, hipStream_t s) {
  if (mode == kMlpBF16)
    hipLaunchKernelGGL(silu_bwd<bf16>, dim3(blocks_for(n)), dim3(256), 0, s, dh, z, g, static_cast<bf16*>(gt), n);
  else
    hipLaunchKernelGGL(silu_bwd<float>, dim3(blocks_for(n)), dim3(256), 0, s, dh, z, g, static_cast<float*>(gt), n);
  return hipGetLastError();
}

hipError_t mlp_colsum(const float* g, float* db, int R, int C, hipStream_t s) {
  hipLaunchKernelGGL(colsum, dim3(C), dim3(256), 0, s, g, db, R, C);
  return hipGetLastError();
}

hipError_t mlp_loss_grad(int mode, const float* z, const float* y, int n_valid, int rows, int ld, float lambda,
                         float* g, void* gt, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(zero_f32, dim3(1), dim3(1), 0, s, loss);
  if (mode == kMlpBF16)
    hipLaunchKernelGGL(loss_grad<bf16>, dim3(blocks_for(rows)), dim3(256), 0, s, z, y, n_valid, rows, ld, lambda, g,
                       static_cast<bf16*>(gt), loss);
  else
    hipLaunchKernelGGL(loss_grad<float>, dim3(blocks_for(rows)), dim3(256), 0, s, z, y, n_valid, rows, ld, lambda, g,
                       static_cast<float*>(gt), loss);
  return hipGetLastError();
}

hipError_t mlp_adam(int mode, float* w, const float* grad, float* m, float* v, void* wt, void* wtt, int rows,
                    int cols, int mask_rows, int mask_cols, float lr, float b1, float b2, float eps, float c1,
                    float c2, hipStream_t s) {
  const int64_t n = int64_t(rows) * cols;
  if (mode == kMlpBF16)
    hipLaunchKernelGGL(adam<bf16>, dim3(blocks_for(n)), dim3(256), 0, s, w, grad, m, v, static_cast<bf16*>(wt),
                       static_cast<bf16*>(wtt), rows, cols, mask_rows, mask_cols, lr, b1, b2, eps, c1, c2);
  else
    hipLaunchKernelGGL(adam<float>, dim3(blocks_for(n)), dim3(256), 0, s, w, grad, m, v, static_cast<float*>(wt),
                       static_cast<float*>(wtt), rows, cols, mask_rows, mask_cols, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t mlp_convert(int mode, const float* in, void* out, void* outt, int rows, int cols, hipStream_t s) {
  const int64_t n = int64_t(rows) * cols;
  if (mode == kMlpBF16)
    hipLaunchKernelGGL(convert_k<bf16>, dim3(blocks_for(n)), dim3(256), 0, s, in, static_cast<bf16*>(out),
                       static_cast<bf16*>(outt), rows, cols);
  else
    hipLaunchKernelGGL(convert_k<float>, dim3(blocks_for(n)), dim3(256), 0, s, in, static_cast<float*>(out),
                       static_cast<float*>(outt), rows, cols);
  return hipGetLastError();
}

hipError_t mlp_features(int mode, const double* mom, int npart, const int32_t* ev, const int32_t* cidx,
                        const float* cpar, int nparam, const float* mean, const float* stdv, void* x, int64_t n,
                        int64_t rows, int ld, hipStream_t s) {
  if (mode == kMlpBF16)
    hipLaunchKernelGGL(features_k<bf16>, dim3(blocks_for(rows)), dim3(256), 0, s, mom, npart, ev, cidx, cpar, nparam,
                       mean, stdv, static_cast<bf16*>(x), n, rows, ld);
  else
    hipLaunchKernelGGL(features_k<float>, dim3(blocks_for(rows)), dim3(256), 0, s, mom, npart, ev, cidx, cpar,
                       nparam, mean, stdv, static_cast<float*>(x), n, rows, ld);
  return hipGetLastError();
}

hipError_t mlp_log_ratio(const double* w_new, const double* w_old, float* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(log_ratio_k, dim3(blocks_for(n)), dim3(256), 0, s, w_new, w_old, y, n);
  return hipGetLastError();
}

hipError_t mlp_gate(const float* z, int ld, int64_t n, float k_cal, float threshold, const double* w_in,
                    double* w_out, int32_t* list, unsigned int* count, hipStream_t s) {
  hipLaunchKernelGGL(zero_u32, dim3(1), dim3(1), 0, s, count);
  hipLaunchKernelGGL(gate_k, dim3(blocks_for(n)), dim3(256), 0, s, z, ld, n, k_cal, threshold, w_in, w_out, list,
                     count);
  return hipGetLastError();
}

}  // namespace rwgt
