// The surrogate network object shared by mlp_abi.cpp and rwgt_abi.cpp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

struct rwgt_mlp {
  struct Layer {
    int in = 0, out = 0, in_used = 0, out_used = 0;      // padded and used shapes
    float *w = nullptr, *b = nullptr;                     // FP32 master parameters
    float *gw = nullptr, *gb = nullptr;                   // gradients
    float *mw = nullptr, *vw = nullptr, *mb = nullptr, *vb = nullptr;   // Adam moments
    void *wc = nullptr, *wct = nullptr;                   // operand-type W [out][in] and W^T [in][out]
  };
  int mode = 0;
  int device = 0;
  int n_in = 0, n_out = 0;
  std::vector<Layer> layers;
  float *mean = nullptr, *stdv = nullptr, *loss = nullptr;
  float lambda = 0.1f, b1 = 0.9f, b2 = 0.999f, eps = 1e-8f, k_cal = 3.3f;
  long long t = 0;
  hipStream_t stream = nullptr;
  // batch workspace
  int64_t bcap = 0;
  std::vector<void*> h, ht, gt, gtt;
  std::vector<float*> z, g, dh;
  std::vector<void*> work, params;
  std::string err;

  int fail(int code, const std::string& msg) { err = msg; return code; }
  int hip_fail(hipError_t e, const char* what) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? -5 : -4;
  }
  int ensure_batch(int64_t rows);
  int refresh_copies();
  int forward(const void* x, int64_t rows);
  int backward(const float* y, int64_t n_valid, int64_t rows);
  int update(float lr);
  ~rwgt_mlp();
};
