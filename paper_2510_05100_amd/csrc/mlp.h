// Internal launch interface of the surrogate kernels (mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rwgt {

enum { kMlpBF16 = 0, kMlpFP32 = 1 };   // operand type: BF16 on the matrix cores, or FP32 on the VALU

hipError_t mlp_gemm(int mode, const void* A, const void* B, int M, int N, int K, const float* bias, float* Cf,
                    void* Ct, int act, hipStream_t s);
hipError_t mlp_transpose(int mode, const void* in, bool in_f32, void* out, int R, int C, hipStream_t s);
hipError_t mlp_silu_bwd(int mode, const float* dh, const float* z, float* g, void* gt, int64_t n, hipStream_t s);
hipError_t mlp_colsum(const float* g, float* db, int R, int C, hipStream_t s);
hipError_t mlp_loss_grad(int mode, const float* z, const float* y, int n_valid, int rows, int ld, float lambda,
                         float* g, void* gt, float* loss, hipStream_t s);
hipError_t mlp_adam(int mode, float* w, const float* grad, float* m, float* v, void* wt, void* wtt, int rows,
                    int cols, int mask_rows, int mask_cols, float lr, float b1, float b2, float eps, float c1,
                    float c2, hipStream_t s);
hipError_t mlp_convert(int mode, const float* in, void* out, void* outt, int rows, int cols, hipStream_t s);
hipError_t mlp_features(int mode, const double* mom, int npart, const int32_t* ev, const int32_t* cidx,
                        const float* cpar, int nparam, const float* mean, const float* stdv, void* x, int64_t n,
                        int64_t rows, int ld, hipStream_t s);
hipError_t mlp_log_ratio(const double* w_new, const double* w_old, float* y, int64_t n, hipStream_t s);
hipError_t mlp_gate(const float* z, int ld, int64_t n, float k_cal, float threshold, const double* w_in,
                    double* w_out, int32_t* list, unsigned int* count, hipStream_t s);

}  // namespace rwgt
