// Internal launch interface of the surrogate kernels (mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "shuffle.h"

namespace rwgt {

// Operand type of one layer: BF16 on the matrix cores, or FP32 on the VALU.
// kMlpSplit (forward GEMM only): FP32 operands on the matrix cores as high
// and low BF16 parts.
enum { kMlpBF16 = 0, kMlpFP32 = 1, kMlpSplit = 2 };
// Input feature maps (rwgt_mlp_set_features).
enum { kFeatRaw = 0, kFeatPhys = 1 };
constexpr int kMlpMaxIn = 32;          // inputs are padded to one 32-wide block
constexpr int kMlpCardParams = 3;      // M_Z, Gamma_Z, sin^2 theta_W
constexpr int kMlpMaxHidden = 8;       // width x width layers of the fused inference kernel

struct FeatureMap {
  int kind = kFeatRaw;
  int npart = 0;
  int res_a = 2, res_b = 3;            // the resonant pair of the propagator features
  double mz0 = 0.0, wz0 = 0.0;         // original card's Z mass and width
  int ncards = 0x7fffffff;             // card indices at or beyond this (or < 0) give NaN features
};

inline int feature_count(int kind, int npart) {
  return kind == kFeatRaw ? npart * 4 + kMlpCardParams : 1 + npart * (npart - 1) / 2 + kMlpCardParams + 4;
}

// Arguments of the fused inference kernel (features, every layer, heads and
// the gate in one pass; hidden width 128 or 256, BF16 hidden layers).
struct InferArgs {
  const double* mom = nullptr;         // [nevt][npart][4]
  const int32_t* ev = nullptr;         // row -> event (NULL: identity)
  const int32_t* cidx = nullptr;       // row -> card
  const float* cpar = nullptr;         // [ncards][3]
  int64_t n = 0;                       // rows
  FeatureMap fm;
  const float* mean = nullptr;         // [32] standardisation (padded: 0 / 1)
  const float* istd = nullptr;       // 1 / standard deviation per input
  const void* w0hi = nullptr;          // first layer, packed BF16 high and low parts
  const void* w0lo = nullptr;
  const float* b0 = nullptr;
  const void* wh = nullptr;            // hidden layers, packed BF16, one after the other
  const float* bh = nullptr;           // their biases, [nh][width]
  int nh = 0;                          // number of width x width layers
  const float* whead = nullptr;        // head layer FP32 [32][width] (rows 0, 1 used)
  const float* bhead = nullptr;
  float ym = 0.0f, ys = 1.0f;          // target scale: mu = mu' ys + ym, s = s' + log ys
  float k_cal = 1.0f, threshold = 0.0f;
  const double* w_in = nullptr;        // gate (w_out non-NULL)
  double* w_out = nullptr;
  int32_t* list = nullptr;
  unsigned int* count = nullptr;
  float* heads = nullptr;              // [n][2] (nullable)
};

// C = A B^T with optional bias and SiLU (act) into FP32 Cf and / or Ct of
// type tout.  work (work_elems floats, may be NULL): space for the partial
// tiles of long-K products, which then run in K chunks on more waves.
hipError_t mlp_gemm(int tin, int tout, const void* A, const void* B, int M, int N, int K, const float* bias,
                    float* Cf, void* Ct, int act, float* work, int64_t work_elems, hipStream_t s);
hipError_t mlp_transpose(int tin, int tout, const void* in, void* out, int R, int C, hipStream_t s);
hipError_t mlp_silu_bwd(int tout, const float* dh, const float* z, float* g, void* gt, int64_t n, hipStream_t s);
// db[c] = sum over the R rows of g[r][c], deterministic.  work (may be NULL):
// ceil(R/64) C floats for row-slab partials; without enough of it the sum
// runs in one pass (one workgroup per column).
hipError_t mlp_colsum(const float* g, float* db, int R, int C, float* work, int64_t work_elems, hipStream_t s);
hipError_t mlp_loss_grad(int tout, const float* z, const float* y, int n_valid, int rows, int ld, float lambda,
                         float ym, float ys, float* g, void* gt, float* loss, hipStream_t s);
hipError_t mlp_adam(int tout, float* w, const float* grad, float* m, float* v, void* wt, void* wtt, int rows,
                    int cols, int mask_rows, int mask_cols, float lr, float b1, float b2, float eps, float c1,
                    float c2, hipStream_t s);
// One Adam step over every parameter tensor of a network in one launch: a
// device table of segments (each a tensor as mlp_adam takes it, at element
// offset begin of the concatenation, begins ascending from 0) and the total
// element count.  Per element the same arithmetic as mlp_adam.
struct AdamSeg {
  float* w;
  const float* grad;
  float* m;
  float* v;
  void* wt;
  void* wtt;
  int64_t begin;
  int rows, cols, mask_rows, mask_cols, bf16_out;
};
hipError_t mlp_adam_all(const AdamSeg* segs, int nseg, int64_t total, float lr, float b1, float b2, float eps, float c1,
                        float c2, hipStream_t s);
hipError_t mlp_convert(int tout, const float* in, void* out, void* outt, int rows, int cols, hipStream_t s);
hipError_t mlp_features(const FeatureMap& fm, const double* mom, const int32_t* ev, const int32_t* cidx,
                        const float* cpar, const float* mean, const float* istd, float* x, int64_t n, int64_t rows,
                        int ld, hipStream_t s);
hipError_t mlp_heads(const float* z, int ld, int64_t n, float ym, float ys, float* out, int ld_out, hipStream_t s);
// Rows [pos0, pos0 + n) of the order sh over a card-major (event, card) grid
// of nevt events: event and card index per row, and y[pair] into yb when y
// is non-NULL (shuffle.h).
hipError_t mlp_gather_pairs(const Shuffle& sh, int64_t pos0, int64_t n, int64_t nevt, const float* y, int32_t* ev,
                            int32_t* cd, float* yb, hipStream_t s);
hipError_t mlp_log_ratio(const double* w_new, const double* w_old, float* y, int64_t n, hipStream_t s);
hipError_t mlp_gate(const float* z, int ld, int64_t n, float ym, float ys, float k_cal, float threshold,
                    const double* w_in, double* w_out, int32_t* list, unsigned int* count, hipStream_t s);
// Packed operand order of the fused kernels (pack_pos in mlp.hip); with
// transposed, W^T is packed: rows_used / cols_used then count rows and
// columns of W^T (element (row, col) = w[col * ld + row]).
hipError_t mlp_pack(const float* w, int ld, int rows_used, int cols_used, int nblocks, int nchunks, void* hi,
                    void* lo, hipStream_t s, bool transposed = false);
hipError_t mlp_infer(int width, const InferArgs& a, hipStream_t s);

// Fused training step of the networks the fused inference kernel runs (two
// heads).  mlp_train_grads: every row tile's inputs, forward and backward
// pass, and per workgroup the sums over its rows of every gradient (and of
// the loss) into its slot of part; mlp_train_update: those sums added in
// workgroup order into the gradient buffers, then (adam) the Adam step and
// every copy of each new parameter.
constexpr int kTrainMaxLayers = kMlpMaxHidden + 2;
constexpr int kTrainMaxGroups = 256;   // workgroups of one step (more tiles: each takes several)
struct TrainArgs {
  const float* x = nullptr;            // input rows [rows][32] (NULL: pairs of a card-major grid)
  const float* y = nullptr;            // their targets [rows]
  Shuffle sh;                          // pairs: positions pos0 .. pos0 + n - 1 of this order
  int64_t pos0 = 0;
  int64_t nevt = 0;                    // events of the grid (pair j: event j % nevt, card j / nevt)
  const double* mom = nullptr;
  const float* cpar = nullptr;
  const float* ygrid = nullptr;        // targets per pair
  FeatureMap fm;
  const float* mean = nullptr;
  const float* istd = nullptr;
  int64_t n = 0;                       // rows of the step (the loss averages over them)
  int64_t rows = 0;                    // readable rows of x
  const void* w0hi = nullptr;          // packed weights as InferArgs
  const void* w0lo = nullptr;
  const float* b0 = nullptr;
  const void* wh = nullptr;
  const void* wht = nullptr;           // the hidden layers' W^T in the same packed order
  const float* bh = nullptr;
  int nh = 0;
  const float* whead = nullptr;        // FP32 [32][width], rows 0 and 1 used
  const float* bhead = nullptr;
  float lambda = 0.0f, ym = 0.0f, ys = 1.0f;
  float* zws = nullptr;                // pre-activations, train_zws_floats(width, nh) per workgroup
  float* part = nullptr;               // [workgroups][pstride]: gradient sums, then the loss at [total]
  int64_t pstride = 0;
  int64_t total = 0;                   // parameters (the Adam segments concatenated)
  int64_t off_w[kTrainMaxLayers] = {}; // begin of each layer's W and b segment
  int64_t off_b[kTrainMaxLayers] = {};
  int tiles = 0;                       // row tiles (train_tile_rows(width) rows each)
  int groups = 0;                      // workgroups (at most kTrainMaxGroups)
};
int train_tile_rows(int width);
int64_t train_zws_floats(int width, int nh);
hipError_t mlp_train_grads(int width, const TrainArgs& a, hipStream_t s);
// Per Adam segment: the packed copies of the parameter to refresh (NULL: none).
// Plain data (copied to LDS by the update kernel); value-initialise on the host.
struct PackSeg {
  float* grad;                         // the gradient buffer (written with the sums)
  void* hi;                            // packed forward order (BF16), nchunks of 16 columns
  void* lo;                            // its low parts (first layer)
  void* tr;                            // packed transposed order
  int nchunks, tchunks;
  float* bias;                         // contiguous hidden-layer biases
};
hipError_t mlp_train_update(const AdamSeg* segs, const PackSeg* pk, int nseg, int64_t total, const float* part,
                            int groups, int64_t pstride, float* loss, int adam, float lr, float b1, float b2,
                            float eps, float c1, float c2, hipStream_t s);
// sums[0..ld) += column sums of x [n][ld], sums[ld..2ld) += sums of squares
// (FP64); clear: zero sums first.
hipError_t mlp_moments(const float* x, int64_t n, int ld, double* sums, bool clear, hipStream_t s);

}  // namespace rwgt
