// Host side of the surrogate network (rwgt_mlp_* in include/rwgt.h): FP32
// master parameters and Adam moments on the device, operand-type copies
// (BF16 or FP32) of every weight matrix and of its transpose, and the
// forward / backward / update sequence of kernel launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "../../include/rwgt.h"
#include "mlp.h"
#include "mlp_internal.h"

using rwgt::kMlpBF16;
using rwgt::kMlpFP32;

namespace {

size_t esize(int mode) { return mode == kMlpBF16 ? 2 : 4; }
int pad32(int x) { return (x + 31) / 32 * 32; }

}  // namespace


int rwgt_mlp::ensure_batch(int64_t rows) {
  if (rows <= bcap) return RWGT_OK;
  for (void* p : work) hipFree(p);
  work.clear();
  const int L = int(layers.size());
  h.assign(L + 1, nullptr);
  ht.assign(L + 1, nullptr);
  z.assign(L, nullptr);
  g.assign(L, nullptr);
  gt.assign(L, nullptr);
  gtt.assign(L, nullptr);
  dh.assign(L, nullptr);
  auto alloc = [&](size_t bytes, void** out) {
    hipError_t e = hipMalloc(out, bytes);
    if (e == hipSuccess) work.push_back(*out);
    return e;
  };
  hipError_t e = hipSuccess;
  for (int l = 0; l <= L && e == hipSuccess; ++l) {
    const int width = l < L ? layers[l].in : layers[L - 1].out;
    e = alloc(size_t(rows) * width * esize(mode), &h[l]);
    if (e == hipSuccess) e = alloc(size_t(rows) * width * esize(mode), &ht[l]);
  }
  for (int l = 0; l < L && e == hipSuccess; ++l) {
    const size_t n = size_t(rows) * layers[l].out;
    e = alloc(n * 4, reinterpret_cast<void**>(&z[l]));
    if (e == hipSuccess) e = alloc(n * 4, reinterpret_cast<void**>(&g[l]));
    if (e == hipSuccess) e = alloc(n * esize(mode), &gt[l]);
    if (e == hipSuccess) e = alloc(n * esize(mode), &gtt[l]);
    if (e == hipSuccess) e = alloc(size_t(rows) * layers[l].in * 4, reinterpret_cast<void**>(&dh[l]));
  }
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(mlp workspace)");
  bcap = rows;
  return RWGT_OK;
}

int rwgt_mlp::refresh_copies() {
  for (auto& ly : layers) {
    hipError_t e = rwgt::mlp_convert(mode, ly.w, ly.wc, ly.wct, ly.out, ly.in, stream);
    if (e != hipSuccess) return hip_fail(e, "convert");
  }
  return RWGT_OK;
}

// Forward over rows (multiple of 64) of x (operand type, [rows][in0]); the
// output head z[L-1] stays in FP32.
int rwgt_mlp::forward(const void* x, int64_t rows) {
  const int L = int(layers.size());
  int rc = ensure_batch(rows);
  if (rc != RWGT_OK) return rc;
  hipError_t e = hipMemcpyAsync(h[0], x, size_t(rows) * layers[0].in * esize(mode), hipMemcpyDeviceToDevice, stream);
  for (int l = 0; l < L && e == hipSuccess; ++l) {
    const bool last = l == L - 1;
    e = rwgt::mlp_gemm(mode, h[l], layers[l].wc, int(rows), layers[l].out, layers[l].in, layers[l].b, z[l],
                       last ? nullptr : h[l + 1], last ? 0 : 1, stream);
  }
  if (e != hipSuccess) return hip_fail(e, "mlp forward");
  return RWGT_OK;
}

// Gradients of the loss into the per-layer gw/gb buffers (after forward).
int rwgt_mlp::backward(const float* y, int64_t n_valid, int64_t rows) {
  const int L = int(layers.size());
  const int ld = layers[L - 1].out;
  hipError_t e = rwgt::mlp_loss_grad(mode, z[L - 1], y, int(n_valid), int(rows), ld, lambda, g[L - 1], gt[L - 1],
                                     loss, stream);
  for (int l = L - 1; l >= 0 && e == hipSuccess; --l) {
    const auto& ly = layers[l];
    // dW = G^T H: operands G^T [out][rows], H^T [in][rows]
    e = rwgt::mlp_transpose(mode, g[l], true, gtt[l], int(rows), ly.out, stream);
    if (e == hipSuccess) e = rwgt::mlp_transpose(mode, h[l], false, ht[l], int(rows), ly.in, stream);
    if (e == hipSuccess) e = rwgt::mlp_gemm(mode, gtt[l], ht[l], ly.out, ly.in, int(rows), nullptr, ly.gw, nullptr, 0, stream);
    if (e == hipSuccess) e = rwgt::mlp_colsum(g[l], ly.gb, int(rows), ly.out, stream);
    if (l == 0 || e != hipSuccess) continue;
    // dH = G W: operands G [rows][out], W^T [in][out]; then through SiLU
    e = rwgt::mlp_gemm(mode, gt[l], ly.wct, int(rows), ly.in, ly.out, nullptr, dh[l], nullptr, 0, stream);
    if (e == hipSuccess) e = rwgt::mlp_silu_bwd(mode, dh[l], z[l - 1], g[l - 1], gt[l - 1], rows * layers[l - 1].out, stream);
  }
  if (e != hipSuccess) return hip_fail(e, "mlp backward");
  return RWGT_OK;
}

int rwgt_mlp::update(float lr) {
  ++t;
  const float c1 = 1.0f / (1.0f - std::pow(b1, float(t)));
  const float c2 = 1.0f / (1.0f - std::pow(b2, float(t)));
  for (auto& ly : layers) {
    hipError_t e = rwgt::mlp_adam(mode, ly.w, ly.gw, ly.mw, ly.vw, ly.wc, ly.wct, ly.out, ly.in, ly.out_used, ly.in_used,
                                  lr, b1, b2, eps, c1, c2, stream);
    if (e == hipSuccess)
      e = rwgt::mlp_adam(kMlpFP32, ly.b, ly.gb, ly.mb, ly.vb, nullptr, nullptr, 1, ly.out, 1, ly.out_used, lr, b1, b2,
                         eps, c1, c2, stream);
    if (e != hipSuccess) return hip_fail(e, "adam");
  }
  return RWGT_OK;
}

rwgt_mlp::~rwgt_mlp() {
  if (stream) hipStreamSynchronize(stream); else hipDeviceSynchronize();
  for (void* p : work) hipFree(p);
  for (void* p : params) hipFree(p);
}

extern "C" {

int rwgt_mlp_create(int32_t n_in, int32_t width, int32_t depth, int32_t n_out, int32_t precision, uint64_t seed,
                    rwgt_mlp** out) {
  if (!out) return RWGT_EINVAL;
  *out = nullptr;
  if (n_in < 1 || width < 32 || width % 32 || depth < 1 || n_out < 2 || n_out > 32 ||
      (precision != RWGT_MLP_BF16 && precision != RWGT_MLP_FP32))
    return RWGT_EINVAL;
  rwgt_mlp* m = new (std::nothrow) rwgt_mlp;
  if (!m) return RWGT_ENOMEM;
  m->mode = precision == RWGT_MLP_BF16 ? kMlpBF16 : rwgt::kMlpFP32;
  m->n_in = n_in;
  m->n_out = n_out;
  // layer shapes: in0 = n_in padded to 32; hidden width; head padded to 32
  std::vector<std::pair<int, int>> shape;   // (in, out), padded
  std::vector<std::pair<int, int>> used;
  shape.push_back({pad32(n_in), width});
  used.push_back({n_in, width});
  for (int d = 1; d < depth; ++d) { shape.push_back({width, width}); used.push_back({width, width}); }
  shape.push_back({width, 32});
  used.push_back({width, n_out});
  std::mt19937_64 rng(seed);
  hipError_t e = hipGetDevice(&m->device);
  for (size_t l = 0; l < shape.size() && e == hipSuccess; ++l) {
    rwgt_mlp::Layer ly;
    ly.in = shape[l].first;
    ly.out = shape[l].second;
    ly.in_used = used[l].first;
    ly.out_used = used[l].second;
    const size_t nw = size_t(ly.in) * ly.out;
    // uniform(-a, a) with a = sqrt(6 / fan_in) on the used block (He-uniform),
    // zero biases and zero padding
    std::vector<float> w(nw, 0.0f);
    const float a = std::sqrt(6.0f / float(ly.in_used));
    std::uniform_real_distribution<float> U(-a, a);
    for (int r = 0; r < ly.out_used; ++r)
      for (int c = 0; c < ly.in_used; ++c) w[size_t(r) * ly.in + c] = U(rng) * (l + 1 == shape.size() ? 0.1f : 1.0f);
    float** f32[] = {&ly.w, &ly.gw, &ly.mw, &ly.vw};
    for (float** p : f32) {
      if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(p), nw * 4);
      if (e == hipSuccess) { m->params.push_back(*p); e = hipMemset(*p, 0, nw * 4); }
    }
    float** bias[] = {&ly.b, &ly.gb, &ly.mb, &ly.vb};
    for (float** p : bias) {
      if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(p), ly.out * 4);
      if (e == hipSuccess) { m->params.push_back(*p); e = hipMemset(*p, 0, ly.out * 4); }
    }
    if (e == hipSuccess) e = hipMalloc(&ly.wc, nw * esize(m->mode));
    if (e == hipSuccess) { m->params.push_back(ly.wc); e = hipMalloc(&ly.wct, nw * esize(m->mode)); }
    if (e == hipSuccess) { m->params.push_back(ly.wct); e = hipMemcpy(ly.w, w.data(), nw * 4, hipMemcpyHostToDevice); }
    m->layers.push_back(ly);
  }
  std::vector<float> ones(32 * ((n_in + 31) / 32), 1.0f), zeros(ones.size(), 0.0f);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&m->mean), ones.size() * 4);
  if (e == hipSuccess) { m->params.push_back(m->mean); e = hipMalloc(reinterpret_cast<void**>(&m->stdv), ones.size() * 4); }
  if (e == hipSuccess) { m->params.push_back(m->stdv); e = hipMalloc(reinterpret_cast<void**>(&m->loss), 4); }
  if (e == hipSuccess) { m->params.push_back(m->loss); e = hipMemcpy(m->mean, zeros.data(), zeros.size() * 4, hipMemcpyHostToDevice); }
  if (e == hipSuccess) e = hipMemcpy(m->stdv, ones.data(), ones.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess && m->refresh_copies() != RWGT_OK) e = hipErrorUnknown;
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) { delete m; return e == hipErrorOutOfMemory ? RWGT_ENOMEM : RWGT_EDEVICE; }
  *out = m;
  return RWGT_OK;
}

void rwgt_mlp_destroy(rwgt_mlp* m) { delete m; }

int rwgt_mlp_set_stream(rwgt_mlp* m, void* stream) {
  if (!m) return RWGT_EINVAL;
  m->stream = static_cast<hipStream_t>(stream);
  return RWGT_OK;
}

int rwgt_mlp_num_params(const rwgt_mlp* m, int64_t* n) {
  if (!m || !n) return RWGT_EINVAL;
  int64_t s = 0;
  for (const auto& ly : m->layers) s += int64_t(ly.in_used) * ly.out_used + ly.out_used;
  *n = s;
  return RWGT_OK;
}

// Parameters packed layer by layer as W[out_used][in_used] then b[out_used].
static int pack(rwgt_mlp* m, bool to_host, float* host, bool grads) {
  hipError_t e = hipStreamSynchronize(m->stream);
  size_t off = 0;
  for (auto& ly : m->layers) {
    float* w = grads ? ly.gw : ly.w;
    float* b = grads ? ly.gb : ly.b;
    std::vector<float> full(size_t(ly.in) * ly.out);
    if (e == hipSuccess && to_host) e = hipMemcpy(full.data(), w, full.size() * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && !to_host) {
      e = hipMemcpy(full.data(), w, full.size() * 4, hipMemcpyDeviceToHost);
      for (int r = 0; r < ly.out_used; ++r)
        std::memcpy(&full[size_t(r) * ly.in], host + off + size_t(r) * ly.in_used, ly.in_used * 4);
      if (e == hipSuccess) e = hipMemcpy(w, full.data(), full.size() * 4, hipMemcpyHostToDevice);
    }
    if (to_host)
      for (int r = 0; r < ly.out_used; ++r)
        std::memcpy(host + off + size_t(r) * ly.in_used, &full[size_t(r) * ly.in], ly.in_used * 4);
    off += size_t(ly.in_used) * ly.out_used;
    if (e == hipSuccess)
      e = to_host ? hipMemcpy(host + off, b, ly.out_used * 4, hipMemcpyDeviceToHost)
                  : hipMemcpy(b, host + off, ly.out_used * 4, hipMemcpyHostToDevice);
    off += ly.out_used;
  }
  if (e != hipSuccess) return m->hip_fail(e, "parameter copy");
  if (!to_host && !grads) return m->refresh_copies();
  return RWGT_OK;
}

int rwgt_mlp_get_params(rwgt_mlp* m, float* host) { return (m && host) ? pack(m, true, host, false) : RWGT_EINVAL; }
int rwgt_mlp_set_params(rwgt_mlp* m, const float* host) {
  return (m && host) ? pack(m, false, const_cast<float*>(host), false) : RWGT_EINVAL;
}
int rwgt_mlp_get_grads(rwgt_mlp* m, float* host) { return (m && host) ? pack(m, true, host, true) : RWGT_EINVAL; }

int rwgt_mlp_set_normalisation(rwgt_mlp* m, const float* mean, const float* stdv) {
  if (!m || !mean || !stdv) return RWGT_EINVAL;
  hipError_t e = hipMemcpy(m->mean, mean, m->n_in * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->stdv, stdv, m->n_in * 4, hipMemcpyHostToDevice);
  return e == hipSuccess ? RWGT_OK : m->hip_fail(e, "normalisation");
}

int rwgt_mlp_set_training(rwgt_mlp* m, float lambda, float beta1, float beta2, float eps) {
  if (!m) return RWGT_EINVAL;
  m->lambda = lambda;
  m->b1 = beta1;
  m->b2 = beta2;
  m->eps = eps;
  return RWGT_OK;
}

int rwgt_mlp_set_calibration(rwgt_mlp* m, float k) {
  if (!m || !(k > 0.0f)) return RWGT_EINVAL;
  m->k_cal = k;
  return RWGT_OK;
}

int rwgt_mlp_features(rwgt_mlp* m, const double* momenta, int32_t npart, const int32_t* event_index,
                      const int32_t* card_index, const float* card_params, int32_t nparam, int64_t n, void* x_out) {
  if (!m || !momenta || !card_index || !card_params || !x_out || n < 0) return RWGT_EINVAL;
  if (npart * 4 + nparam != m->n_in) return m->fail(RWGT_EINVAL, "feature count differs from the input width");
  const int64_t rows = (n + 63) / 64 * 64;
  hipError_t e = rwgt::mlp_features(m->mode, momenta, npart, event_index, card_index, card_params, nparam, m->mean,
                                    m->stdv, x_out, n, rows, m->layers[0].in, m->stream);
  return e == hipSuccess ? RWGT_OK : m->hip_fail(e, "features");
}

int rwgt_mlp_forward(rwgt_mlp* m, const void* x, int64_t n, float* heads_out) {
  if (!m || !x || n < 1) return RWGT_EINVAL;
  const int64_t rows = (n + 63) / 64 * 64;
  int rc = m->forward(x, rows);
  if (rc != RWGT_OK) return rc;
  if (heads_out) {
    hipError_t e = hipMemcpyAsync(heads_out, m->z.back(), size_t(n) * 32 * 4, hipMemcpyDeviceToDevice, m->stream);
    if (e != hipSuccess) return m->hip_fail(e, "copy heads");
  }
  return RWGT_OK;
}

int rwgt_mlp_train_step(rwgt_mlp* m, const void* x, const float* y, int64_t n, float lr, float* loss_out) {
  if (!m || !x || !y || n < 1) return RWGT_EINVAL;
  const int64_t rows = (n + 63) / 64 * 64;
  int rc = m->forward(x, rows);
  if (rc == RWGT_OK) rc = m->backward(y, n, rows);
  if (rc == RWGT_OK && lr > 0.0f) rc = m->update(lr);
  if (rc == RWGT_OK && loss_out) {
    hipError_t e = hipMemcpyAsync(loss_out, m->loss, 4, hipMemcpyDeviceToDevice, m->stream);
    if (e != hipSuccess) return m->hip_fail(e, "copy loss");
  }
  return rc;
}

int rwgt_mlp_input_bytes(const rwgt_mlp* m, int64_t n, int64_t* bytes) {
  if (!m || !bytes) return RWGT_EINVAL;
  *bytes = (n + 63) / 64 * 64 * m->layers[0].in * int64_t(esize(m->mode));
  return RWGT_OK;
}

int rwgt_mlp_targets(rwgt_mlp* m, const double* w_new, const double* w_old, int64_t n, float* y) {
  if (!m || !w_new || !y || n < 0) return RWGT_EINVAL;
  if (n == 0) return RWGT_OK;
  hipError_t e = rwgt::mlp_log_ratio(w_new, w_old, y, n, m->stream);
  return e == hipSuccess ? RWGT_OK : m->hip_fail(e, "targets");
}

const char* rwgt_mlp_last_error(const rwgt_mlp* m) { return m ? m->err.c_str() : "mlp is NULL"; }

}  // extern "C"
