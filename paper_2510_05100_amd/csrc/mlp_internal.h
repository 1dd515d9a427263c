// The surrogate network object shared by mlp_abi.cpp and rwgt_abi.cpp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mlp.h"

struct rwgt_mlp {
  enum { kCopyParams = 0, kCopyGrads = 1, kCopyFirst = 2, kCopySecond = 3 };   // pack_params selections
  struct Layer {
    int mode = 0;                                         // operand type (rwgt::kMlpBF16 / kMlpFP32)
    bool split = false;                                   // FP32 forward product as split BF16 (kMlpSplit)
    int in = 0, out = 0, in_used = 0, out_used = 0;      // padded and used shapes
    float *w = nullptr, *b = nullptr;                     // FP32 master parameters
    float *gw = nullptr, *gb = nullptr;                   // gradients
    float *mw = nullptr, *vw = nullptr, *mb = nullptr, *vb = nullptr;   // Adam moments
    void *wc = nullptr, *wct = nullptr;                   // operand-type W [out][in] and W^T [in][out]
  };
  int mode = 0;                                           // network precision (RWGT_MLP_*)
  int device = 0;
  int n_in = 0, n_out = 0, width = 0;
  std::vector<Layer> layers;
  rwgt::FeatureMap fm;
  float *mean = nullptr, *stdv = nullptr, *istd = nullptr, *loss = nullptr;   // istd = 1 / stdv
  float lambda = 0.1f, b1 = 0.9f, b2 = 0.999f, eps = 1e-8f, k_cal = 3.3f;
  float ym = 0.0f, ys = 1.0f;                             // target standardisation
  long long t = 0;
  hipStream_t stream = nullptr;
  // fused inference: packed weights (valid while !pack_dirty)
  void *p0hi = nullptr, *p0lo = nullptr, *phid = nullptr;
  void* phid_t = nullptr;                                 // hidden layers' W^T, packed (fused training)
  float* pbias = nullptr;
  bool pack_dirty = true;
  // fused training step: per-segment packed copies, per-workgroup gradient
  // sums and pre-activation workspace
  rwgt::PackSeg* pack_segs = nullptr;
  float *tr_part = nullptr, *tr_zws = nullptr;
  int tr_groups = 0;                                      // workgroup slots allocated
  int64_t tr_pstride = 0;
  // batch workspace
  int64_t bcap = 0;
  const void* x_in = nullptr;                             // the current batch's input rows (FP32)
  std::vector<void*> h, ht, gt, gtt;
  std::vector<float*> z, g, dh;
  float* kpart = nullptr;                                 // K-chunk partial tiles of the weight gradients
  rwgt::AdamSeg* adam_segs = nullptr;                     // device table of every parameter tensor (one Adam launch)
  int adam_nseg = 0;
  int64_t adam_total = 0;
  int64_t kpart_elems = 0;
  std::vector<void*> work, params;
  // training schedule and progress (rwgt_mlp_train; saved in checkpoints)
  struct Schedule {
    int64_t batch = 0;
    int32_t epochs = 0;
    float lr = 0.0f, lr_final = 0.0f;
    uint64_t seed = 0;
  } sched;
  bool has_sched = false;
  int64_t epoch = 0;                                      // epochs completed
  int64_t step = 0;                                       // steps of the schedule taken
  // training-batch workspace (rwgt_mlp_train)
  int64_t tcap = 0;
  int32_t *tr_ev = nullptr, *tr_cd = nullptr;
  float *tr_y = nullptr, *tr_x = nullptr, *tr_loss = nullptr;
  int64_t tr_loss_cap = 0;
  std::vector<void*> twork;
  std::string err;

  int fail(int code, const std::string& msg) { err = msg; return code; }
  int hip_fail(hipError_t e, const char* what) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? -5 : -4;
  }
  const void* input(int l) const { return l == 0 ? x_in : h[l]; }
  bool fused() const;                                     // eligible for the fused inference kernel
  int pack();                                             // refresh the packed weights if stale
  // fused pass over n rows (see rwgt::InferArgs); gate when w_out is non-NULL
  int infer(const double* mom, const int32_t* ev, const int32_t* cidx, const float* cpar, int64_t n,
            float* heads, const double* w_in, double* w_out, int32_t* list, unsigned int* count, float threshold);
  int ensure_batch(int64_t rows);
  int refresh_copies();
  int forward(const void* x, int64_t rows);
  int backward(const float* y, int64_t n_valid, int64_t rows);
  int update(float lr);
  int ensure_train(int64_t batch, int64_t probes);
  // eligible for the fused training step (fused inference weights, two heads)
  bool fused_train() const { return phid_t && pack_segs && n_out == 2; }
  // one fused step over the rows described by rows_in (x / y, or the pairs
  // of a grid); lr > 0: with the Adam step, else gradients and loss only
  int train_fused(const rwgt::TrainArgs& rows_in, float lr);
  // heads (mu_y, s_y) [n][2] of rows (ev, cd), fused kernel or layer by layer
  int predict_rows(const double* mom, const int32_t* ev, const int32_t* cd, const float* cpar, int64_t n,
                   float* heads);
  ~rwgt_mlp();
};

// Host <-> device copy of the parameters, gradients or Adam moments (which:
// rwgt_mlp::kCopy*) packed layer by layer as W[out_used][in_used], b[out_used];
// waits for the network's stream.  Setting parameters refreshes the operand
// copies.
int pack_params(rwgt_mlp* m, bool to_host, float* host, int which);
// The feature map of a network that has none yet becomes the raw map of
// npart particles; errors when the map and the network's width or npart
// disagree.
int resolve_map(rwgt_mlp* m, int32_t npart);
