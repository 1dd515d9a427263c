// Host side of the surrogate network (rwgt_mlp_* in include/rwgt.h): FP32
// master parameters and Adam moments on the device, operand-type copies of
// every weight matrix and of its transpose, the forward / backward / update
// sequence of kernel launches, and the packed weights of the fused inference
// kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
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
int64_t pad64(int64_t x) { return (x + 63) / 64 * 64; }
constexpr size_t kPackBytes = 512 * 2;      // one packed (block, chunk): 64 lanes x 8 BF16

}  // namespace

int rwgt_mlp::ensure_batch(int64_t rows) {
  if (rows <= bcap) return RWGT_OK;
  for (void* p : work) hipFree(p);
  work.clear();
  const int L = int(layers.size());
  h.assign(L, nullptr);
  ht.assign(L, nullptr);
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
  for (int l = 0; l < L && e == hipSuccess; ++l) {
    const Layer& ly = layers[l];
    const size_t es = esize(ly.mode);
    if (l > 0) e = alloc(size_t(rows) * ly.in * es, &h[l]);     // h[0]: the caller's input rows
    if (e == hipSuccess) e = alloc(size_t(rows) * ly.in * es, &ht[l]);
    const size_t n = size_t(rows) * ly.out;
    if (e == hipSuccess) e = alloc(n * 4, reinterpret_cast<void**>(&z[l]));
    if (e == hipSuccess) e = alloc(n * 4, reinterpret_cast<void**>(&g[l]));
    if (e == hipSuccess) e = alloc(n * es, &gt[l]);
    if (e == hipSuccess) e = alloc(n * es, &gtt[l]);
    if (e == hipSuccess && l > 0) e = alloc(size_t(rows) * ly.in * 4, reinterpret_cast<void**>(&dh[l]));
  }
  // partial tiles of the chunked weight-gradient products: 32 chunks of the
  // largest layer
  int64_t most = 0;
  for (const Layer& ly : layers) most = std::max(most, int64_t(ly.out) * ly.in);
  kpart = nullptr;
  kpart_elems = 0;
  if (e == hipSuccess) e = alloc(size_t(32 * most) * 4, reinterpret_cast<void**>(&kpart));
  if (e == hipSuccess) kpart_elems = 32 * most;
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(mlp workspace)");
  bcap = rows;
  return RWGT_OK;
}

int rwgt_mlp::refresh_copies() {
  for (auto& ly : layers) {
    hipError_t e = rwgt::mlp_convert(ly.mode, ly.w, ly.wc, ly.wct, ly.out, ly.in, stream);
    if (e != hipSuccess) return hip_fail(e, "convert");
  }
  pack_dirty = true;
  return RWGT_OK;
}

// Forward over rows (multiple of 64) of x (FP32, [rows][in0]); z[l] holds
// each layer's FP32 pre-activation, the head's output stays in z[L-1].
int rwgt_mlp::forward(const void* x, int64_t rows) {
  const int L = int(layers.size());
  int rc = ensure_batch(rows);
  if (rc != RWGT_OK) return rc;
  x_in = x;
  hipError_t e = hipSuccess;
  for (int l = 0; l < L && e == hipSuccess; ++l) {
    const bool last = l == L - 1;
    const Layer& ly = layers[l];
    e = rwgt::mlp_gemm(ly.split ? rwgt::kMlpSplit : ly.mode, last ? ly.mode : layers[l + 1].mode, input(l), ly.wc,
                       int(rows), ly.out, ly.in, ly.b, z[l], last ? nullptr : h[l + 1], last ? 0 : 1, nullptr, 0,
                       stream);
  }
  if (e != hipSuccess) return hip_fail(e, "mlp forward");
  return RWGT_OK;
}

// Gradients of the loss into the per-layer gw/gb buffers (after forward).
int rwgt_mlp::backward(const float* y, int64_t n_valid, int64_t rows) {
  const int L = int(layers.size());
  const Layer& head = layers[L - 1];
  hipError_t e = rwgt::mlp_loss_grad(head.mode, z[L - 1], y, int(n_valid), int(rows), head.out, lambda, ym, ys,
                                     g[L - 1], gt[L - 1], loss, stream);
  for (int l = L - 1; l >= 0 && e == hipSuccess; --l) {
    const Layer& ly = layers[l];
    // dW = G^T H: operands G^T [out][rows], H^T [in][rows] in this layer's type
    e = rwgt::mlp_transpose(kMlpFP32, ly.mode, g[l], gtt[l], int(rows), ly.out, stream);
    if (e == hipSuccess) e = rwgt::mlp_transpose(ly.mode, ly.mode, input(l), ht[l], int(rows), ly.in, stream);
    if (e == hipSuccess)
      e = rwgt::mlp_gemm(ly.mode, ly.mode, gtt[l], ht[l], ly.out, ly.in, int(rows), nullptr, ly.gw, nullptr, 0, kpart,
                         kpart_elems, stream);
    // the bias gradient's slab partials reuse kpart, free again once the
    // weight-gradient product above has summed its chunks (stream order)
    if (e == hipSuccess) e = rwgt::mlp_colsum(g[l], ly.gb, int(rows), ly.out, kpart, kpart_elems, stream);
    if (l == 0 || e != hipSuccess) continue;
    // dH = G W: operands G [rows][out], W^T [in][out]; then through SiLU into
    // the previous layer's gradient (FP32 and its operand type)
    e = rwgt::mlp_gemm(ly.mode, ly.mode, gt[l], ly.wct, int(rows), ly.in, ly.out, nullptr, dh[l], nullptr, 0, nullptr, 0,
                       stream);
    if (e == hipSuccess)
      e = rwgt::mlp_silu_bwd(layers[l - 1].mode, dh[l], z[l - 1], g[l - 1], gt[l - 1], rows * layers[l - 1].out,
                             stream);
  }
  if (e != hipSuccess) return hip_fail(e, "mlp backward");
  return RWGT_OK;
}

int rwgt_mlp::update(float lr) {
  ++t;
  const float c1 = 1.0f / (1.0f - std::pow(b1, float(t)));
  const float c2 = 1.0f / (1.0f - std::pow(b2, float(t)));
  if (adam_segs) {
    hipError_t e = rwgt::mlp_adam_all(adam_segs, adam_nseg, adam_total, lr, b1, b2, eps, c1, c2, stream);
    if (e != hipSuccess) return hip_fail(e, "adam");
    pack_dirty = true;
    return RWGT_OK;
  }
  for (auto& ly : layers) {
    hipError_t e = rwgt::mlp_adam(ly.mode, ly.w, ly.gw, ly.mw, ly.vw, ly.wc, ly.wct, ly.out, ly.in, ly.out_used,
                                  ly.in_used, lr, b1, b2, eps, c1, c2, stream);
    if (e == hipSuccess)
      e = rwgt::mlp_adam(kMlpFP32, ly.b, ly.gb, ly.mb, ly.vb, nullptr, nullptr, 1, ly.out, 1, ly.out_used, lr, b1, b2,
                         eps, c1, c2, stream);
    if (e != hipSuccess) return hip_fail(e, "adam");
  }
  pack_dirty = true;
  return RWGT_OK;
}

bool rwgt_mlp::fused() const {
  const int L = int(layers.size());
  return p0hi && L >= 3 && fm.npart >= 4 && fm.npart <= 5 && n_in == rwgt::feature_count(fm.kind, fm.npart);
}

int rwgt_mlp::pack() {
  if (!pack_dirty) return RWGT_OK;
  const int L = int(layers.size());
  const int nb = width / 32, nc = width / 16;
  const Layer& l0 = layers[0];
  hipError_t e = rwgt::mlp_pack(l0.w, l0.in, l0.out_used, l0.in_used, nb, 2, p0hi, p0lo, stream);
  for (int l = 1; l + 1 < L && e == hipSuccess; ++l) {
    const Layer& ly = layers[l];
    char* dst = static_cast<char*>(phid) + size_t(l - 1) * nb * nc * kPackBytes;
    e = rwgt::mlp_pack(ly.w, ly.in, ly.out_used, ly.in_used, nb, nc, dst, nullptr, stream);
    if (e == hipSuccess && phid_t) {
      char* dst_t = static_cast<char*>(phid_t) + size_t(l - 1) * nb * nc * kPackBytes;
      e = rwgt::mlp_pack(ly.w, ly.in, ly.in_used, ly.out_used, nb, nc, dst_t, nullptr, stream, true);
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(pbias + size_t(l - 1) * width, ly.b, size_t(width) * 4, hipMemcpyDeviceToDevice, stream);
  }
  if (e != hipSuccess) return hip_fail(e, "pack");
  pack_dirty = false;
  return RWGT_OK;
}

int rwgt_mlp::infer(const double* mom, const int32_t* ev, const int32_t* cidx, const float* cpar, int64_t n,
                    float* heads, const double* w_in, double* w_out, int32_t* list, unsigned int* count,
                    float threshold) {
  int rc = pack();
  if (rc != RWGT_OK) return rc;
  const int L = int(layers.size());
  rwgt::InferArgs a;
  a.mom = mom;
  a.ev = ev;
  a.cidx = cidx;
  a.cpar = cpar;
  a.n = n;
  a.fm = fm;
  a.mean = mean;
  a.istd = istd;
  a.w0hi = p0hi;
  a.w0lo = p0lo;
  a.b0 = layers[0].b;
  a.wh = phid;
  a.bh = pbias;
  a.nh = L - 2;
  a.whead = layers[L - 1].w;
  a.bhead = layers[L - 1].b;
  a.ym = ym;
  a.ys = ys;
  a.k_cal = k_cal;
  a.threshold = threshold;
  a.w_in = w_in;
  a.w_out = w_out;
  a.list = list;
  a.count = count;
  a.heads = heads;
  hipError_t e = rwgt::mlp_infer(width, a, stream);
  return e == hipSuccess ? RWGT_OK : hip_fail(e, "fused inference");
}

rwgt_mlp::~rwgt_mlp() {
  if (stream) hipStreamSynchronize(stream); else hipDeviceSynchronize();
  for (void* p : work) hipFree(p);
  for (void* p : twork) hipFree(p);
  for (void* p : params) hipFree(p);
  if (tr_part) hipFree(tr_part);
  if (tr_zws) hipFree(tr_zws);
}

extern "C" {

int rwgt_mlp_create(int32_t n_in, int32_t width, int32_t depth, int32_t n_out, int32_t precision, uint64_t seed,
                    rwgt_mlp** out) {
  if (!out) return RWGT_EINVAL;
  *out = nullptr;
  if (n_in < 1 || n_in > rwgt::kMlpMaxIn || width < 32 || width % 32 || depth < 1 || n_out < 2 || n_out > 32 ||
      (precision != RWGT_MLP_BF16 && precision != RWGT_MLP_FP32))
    return RWGT_EINVAL;
  rwgt_mlp* m = new (std::nothrow) rwgt_mlp;
  if (!m) return RWGT_ENOMEM;
  m->mode = precision == RWGT_MLP_BF16 ? kMlpBF16 : kMlpFP32;
  m->n_in = n_in;
  m->n_out = n_out;
  m->width = width;
  // layer shapes: in0 = n_in padded to 32; hidden width; head padded to 32.
  // BF16 networks: FP32 first layer (forward product as split BF16, the
  // arithmetic of the fused inference kernel) and head, BF16 hidden layers.
  struct Shape { int in, out, in_used, out_used, mode; };
  std::vector<Shape> shape;
  const int hidden_mode = m->mode;
  shape.push_back({pad32(n_in), width, n_in, width, kMlpFP32});
  for (int d = 1; d < depth; ++d) shape.push_back({width, width, width, width, hidden_mode});
  shape.push_back({width, 32, width, n_out, kMlpFP32});
  std::mt19937_64 rng(seed);
  hipError_t e = hipGetDevice(&m->device);
  auto dalloc = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes);
    if (e == hipSuccess) m->params.push_back(*p);
  };
  for (size_t l = 0; l < shape.size() && e == hipSuccess; ++l) {
    rwgt_mlp::Layer ly;
    ly.mode = shape[l].mode;
    ly.split = l == 0 && m->mode == kMlpBF16;
    ly.in = shape[l].in;
    ly.out = shape[l].out;
    ly.in_used = shape[l].in_used;
    ly.out_used = shape[l].out_used;
    const size_t nw = size_t(ly.in) * ly.out;
    // uniform(-a, a) with a = sqrt(6 / fan_in) on the used block (He-uniform),
    // zero biases and zero padding
    std::vector<float> w(nw, 0.0f);
    const float a = std::sqrt(6.0f / float(ly.in_used));
    std::uniform_real_distribution<float> U(-a, a);
    for (int r = 0; r < ly.out_used; ++r)
      for (int c = 0; c < ly.in_used; ++c) w[size_t(r) * ly.in + c] = U(rng) * (l + 1 == shape.size() ? 0.1f : 1.0f);
    for (float** p : {&ly.w, &ly.gw, &ly.mw, &ly.vw}) {
      dalloc(reinterpret_cast<void**>(p), nw * 4);
      if (e == hipSuccess) e = hipMemset(*p, 0, nw * 4);
    }
    for (float** p : {&ly.b, &ly.gb, &ly.mb, &ly.vb}) {
      dalloc(reinterpret_cast<void**>(p), size_t(ly.out) * 4);
      if (e == hipSuccess) e = hipMemset(*p, 0, size_t(ly.out) * 4);
    }
    dalloc(&ly.wc, nw * esize(ly.mode));
    dalloc(&ly.wct, nw * esize(ly.mode));
    if (e == hipSuccess) e = hipMemcpy(ly.w, w.data(), nw * 4, hipMemcpyHostToDevice);
    m->layers.push_back(ly);
  }
  std::vector<float> ones(rwgt::kMlpMaxIn, 1.0f), zeros(rwgt::kMlpMaxIn, 0.0f);
  dalloc(reinterpret_cast<void**>(&m->mean), ones.size() * 4);
  dalloc(reinterpret_cast<void**>(&m->stdv), ones.size() * 4);
  dalloc(reinterpret_cast<void**>(&m->istd), ones.size() * 4);
  dalloc(reinterpret_cast<void**>(&m->loss), 4);
  if (e == hipSuccess) e = hipMemcpy(m->mean, zeros.data(), zeros.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->stdv, ones.data(), ones.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->istd, ones.data(), ones.size() * 4, hipMemcpyHostToDevice);
  // packed weights of the fused inference kernel (BF16 networks of width 128
  // or 256 with 1..kMlpMaxHidden hidden width x width layers)
  const int nh = depth - 1;
  if (m->mode == kMlpBF16 && (width == 128 || width == 256) && nh >= 1 && nh <= rwgt::kMlpMaxHidden) {
    const size_t nb = width / 32, nc = width / 16;
    dalloc(&m->p0hi, nb * 2 * kPackBytes);
    dalloc(&m->p0lo, nb * 2 * kPackBytes);
    dalloc(&m->phid, size_t(nh) * nb * nc * kPackBytes);
    dalloc(reinterpret_cast<void**>(&m->pbias), size_t(nh) * width * 4);
    if (n_out == 2) dalloc(&m->phid_t, size_t(nh) * nb * nc * kPackBytes);   // fused training
  }
  // the Adam segment table: each layer's W (operand-type copies W, W^T) and
  // bias, in layer order, as the per-tensor calls take them
  if (e == hipSuccess) {
    std::vector<rwgt::AdamSeg> segs;
    int64_t begin = 0;
    for (const auto& ly : m->layers) {
      segs.push_back({ly.w, ly.gw, ly.mw, ly.vw, ly.wc, ly.wct, begin, ly.out, ly.in, ly.out_used, ly.in_used,
                      ly.mode == kMlpBF16 ? 1 : 0});
      begin += int64_t(ly.out) * ly.in;
      segs.push_back({ly.b, ly.gb, ly.mb, ly.vb, nullptr, nullptr, begin, 1, ly.out, 1, ly.out_used, 0});
      begin += ly.out;
    }
    void* tab = nullptr;
    dalloc(&tab, segs.size() * sizeof(rwgt::AdamSeg));
    if (e == hipSuccess) e = hipMemcpy(tab, segs.data(), segs.size() * sizeof(rwgt::AdamSeg), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
      m->adam_segs = static_cast<rwgt::AdamSeg*>(tab);
      m->adam_nseg = int(segs.size());
      m->adam_total = begin;
    }
    // the fused training step's copies of each segment: packed first layer
    // (hi / lo), packed hidden W and W^T, contiguous hidden biases
    if (e == hipSuccess && m->phid_t) {
      const int L = int(m->layers.size()), nb = width / 32, nc = width / 16;
      std::vector<rwgt::PackSeg> pk(segs.size());
      for (int l = 0; l < L; ++l) {
        rwgt::PackSeg& pw = pk[size_t(2 * l)];
        rwgt::PackSeg& pb = pk[size_t(2 * l + 1)];
        pw.grad = m->layers[size_t(l)].gw;
        pb.grad = m->layers[size_t(l)].gb;
        if (l == 0) {
          pw.hi = m->p0hi;
          pw.lo = m->p0lo;
          pw.nchunks = 2;
        } else if (l + 1 < L) {
          const size_t off = size_t(l - 1) * nb * nc * kPackBytes;
          pw.hi = static_cast<char*>(m->phid) + off;
          pw.tr = static_cast<char*>(m->phid_t) + off;
          pw.nchunks = pw.tchunks = nc;
          pb.bias = m->pbias + size_t(l - 1) * width;
        }
      }
      void* ptab = nullptr;
      dalloc(&ptab, pk.size() * sizeof(rwgt::PackSeg));
      if (e == hipSuccess) e = hipMemcpy(ptab, pk.data(), pk.size() * sizeof(rwgt::PackSeg), hipMemcpyHostToDevice);
      if (e == hipSuccess) m->pack_segs = static_cast<rwgt::PackSeg*>(ptab);
    }
  }
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

}  // extern "C"

// Parameters (or gradients, or Adam moments: rwgt_mlp::kCopy*) packed layer
// by layer as W[out_used][in_used] then b[out_used]; padding stays as it is.
int pack_params(rwgt_mlp* m, bool to_host, float* host, int which) {
  hipError_t e = hipStreamSynchronize(m->stream);
  size_t off = 0;
  for (auto& ly : m->layers) {
    float* const ws[4] = {ly.w, ly.gw, ly.mw, ly.vw};
    float* const bs[4] = {ly.b, ly.gb, ly.mb, ly.vb};
    float* w = ws[which];
    float* b = bs[which];
    std::vector<float> full(size_t(ly.in) * ly.out);
    if (e == hipSuccess) e = hipMemcpy(full.data(), w, full.size() * 4, hipMemcpyDeviceToHost);
    if (to_host) {
      for (int r = 0; r < ly.out_used; ++r)
        std::memcpy(host + off + size_t(r) * ly.in_used, &full[size_t(r) * ly.in], ly.in_used * 4);
    } else {
      for (int r = 0; r < ly.out_used; ++r)
        std::memcpy(&full[size_t(r) * ly.in], host + off + size_t(r) * ly.in_used, ly.in_used * 4);
      if (e == hipSuccess) e = hipMemcpy(w, full.data(), full.size() * 4, hipMemcpyHostToDevice);
    }
    off += size_t(ly.in_used) * ly.out_used;
    if (e == hipSuccess)
      e = to_host ? hipMemcpy(host + off, b, ly.out_used * 4, hipMemcpyDeviceToHost)
                  : hipMemcpy(b, host + off, ly.out_used * 4, hipMemcpyHostToDevice);
    off += ly.out_used;
  }
  if (e != hipSuccess) return m->hip_fail(e, "parameter copy");
  if (!to_host && which == rwgt_mlp::kCopyParams) return m->refresh_copies();
  return RWGT_OK;
}

extern "C" {

int rwgt_mlp_get_params(rwgt_mlp* m, float* host) {
  return (m && host) ? pack_params(m, true, host, rwgt_mlp::kCopyParams) : RWGT_EINVAL;
}
int rwgt_mlp_set_params(rwgt_mlp* m, const float* host) {
  return (m && host) ? pack_params(m, false, const_cast<float*>(host), rwgt_mlp::kCopyParams) : RWGT_EINVAL;
}
int rwgt_mlp_get_grads(rwgt_mlp* m, float* host) {
  return (m && host) ? pack_params(m, true, host, rwgt_mlp::kCopyGrads) : RWGT_EINVAL;
}
int rwgt_mlp_get_adam(rwgt_mlp* m, float* first, float* second, int64_t* steps) {
  if (!m || !first || !second || !steps) return RWGT_EINVAL;
  int rc = pack_params(m, true, first, rwgt_mlp::kCopyFirst);
  if (rc == RWGT_OK) rc = pack_params(m, true, second, rwgt_mlp::kCopySecond);
  *steps = m->t;
  return rc;
}

int rwgt_mlp_set_normalisation(rwgt_mlp* m, const float* mean, const float* stdv) {
  if (!m || !mean || !stdv) return RWGT_EINVAL;
  for (int k = 0; k < m->n_in; ++k)
    if (!(stdv[k] > 0.0f) || !std::isfinite(stdv[k]) || !std::isfinite(mean[k]))
      return m->fail(RWGT_EINVAL, "standard deviations must be positive and finite");
  std::vector<float> inv(size_t(m->n_in));
  for (int k = 0; k < m->n_in; ++k) inv[size_t(k)] = 1.0f / stdv[k];
  hipError_t e = hipMemcpy(m->mean, mean, m->n_in * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->stdv, stdv, m->n_in * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->istd, inv.data(), m->n_in * 4, hipMemcpyHostToDevice);
  return e == hipSuccess ? RWGT_OK : m->hip_fail(e, "normalisation");
}

int rwgt_mlp_set_features(rwgt_mlp* m, int32_t kind, int32_t npart, int32_t res_a, int32_t res_b, double mz0,
                          double wz0) {
  if (!m) return RWGT_EINVAL;
  if (kind != RWGT_FEAT_RAW && kind != RWGT_FEAT_PHYS) return m->fail(RWGT_EINVAL, "unknown feature map");
  if (npart < 4 || npart > 5) return m->fail(RWGT_EINVAL, "feature maps cover 4 or 5 external particles");
  if (m->n_in != rwgt::feature_count(kind, npart))
    return m->fail(RWGT_EINVAL, "the feature map's width differs from the network's n_in");
  if (kind == RWGT_FEAT_PHYS &&
      (res_a < 0 || res_b < 0 || res_a >= npart || res_b >= npart || res_a == res_b || !(mz0 > 0.0) || !(wz0 > 0.0)))
    return m->fail(RWGT_EINVAL, "bad resonant pair or original Z mass / width");
  m->fm.kind = kind;
  m->fm.npart = npart;
  m->fm.res_a = res_a;
  m->fm.res_b = res_b;
  m->fm.mz0 = mz0;
  m->fm.wz0 = wz0;
  return RWGT_OK;
}

int rwgt_mlp_get_normalisation(rwgt_mlp* m, float* mean, float* stdv, float* y_scale) {
  if (!m || !mean || !stdv || !y_scale) return RWGT_EINVAL;
  hipError_t e = hipStreamSynchronize(m->stream);
  if (e == hipSuccess) e = hipMemcpy(mean, m->mean, m->n_in * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(stdv, m->stdv, m->n_in * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return m->hip_fail(e, "normalisation");
  y_scale[0] = m->ym;
  y_scale[1] = m->ys;
  return RWGT_OK;
}

int rwgt_mlp_set_target_scale(rwgt_mlp* m, float mean, float stdv) {
  if (!m || !(stdv > 0.0f) || !std::isfinite(stdv) || !std::isfinite(mean)) return RWGT_EINVAL;
  m->ym = mean;
  m->ys = stdv;
  return RWGT_OK;
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

}  // extern "C"

// The feature map of a network that has none yet: the raw map of npart
// particles.  Errors when the map and the network's width disagree.
int resolve_map(rwgt_mlp* m, int32_t npart) {
  if (m->fm.npart == 0) {
    if (m->n_in != rwgt::feature_count(RWGT_FEAT_RAW, npart))
      return m->fail(RWGT_EINVAL, "feature count differs from the input width");
    m->fm.kind = RWGT_FEAT_RAW;
    m->fm.npart = npart;
  }
  if (npart != m->fm.npart) return m->fail(RWGT_EINVAL, "particle count differs from the feature map");
  return RWGT_OK;
}

extern "C" {

int rwgt_mlp_features(rwgt_mlp* m, const double* momenta, int32_t npart, const int32_t* event_index,
                      const int32_t* card_index, const float* card_params, int32_t nparam, int64_t n, void* x_out) {
  if (!m || !momenta || !card_index || !card_params || !x_out || n < 0) return RWGT_EINVAL;
  if (nparam != rwgt::kMlpCardParams) return m->fail(RWGT_EINVAL, "cards carry (M_Z, Gamma_Z, sin^2 theta_W)");
  int rc = resolve_map(m, npart);
  if (rc != RWGT_OK) return rc;
  const int64_t rows = pad64(n);
  hipError_t e = rwgt::mlp_features(m->fm, momenta, event_index, card_index, card_params, m->mean, m->istd,
                                    static_cast<float*>(x_out), n, rows, m->layers[0].in, m->stream);
  return e == hipSuccess ? RWGT_OK : m->hip_fail(e, "features");
}

}  // extern "C"

// Mean and population standard deviation of columns [0, ncol) of FP32 rows
// produced chunk by chunk by fill(a, b, buffer) (rows a..b), FP64 sums on the
// device.  Constant columns get standard deviation 1.
template <class Fill>
static int column_stats(rwgt_mlp* m, int64_t n, int ld, int ncol, Fill fill, std::vector<float>& mean,
                        std::vector<float>& stdv) {
  const int64_t chunk = int64_t(1) << 18;
  void* x = nullptr;
  double* sums = nullptr;
  hipError_t e = hipMalloc(&x, size_t(std::min(n, chunk)) * ld * 4);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&sums), size_t(2 * ld) * 8);
  for (int64_t a = 0; a < n && e == hipSuccess; a += chunk) {
    const int64_t b = std::min(n, a + chunk);
    e = fill(a, b, static_cast<float*>(x));
    if (e == hipSuccess) e = rwgt::mlp_moments(static_cast<float*>(x), b - a, ld, sums, a == 0, m->stream);
  }
  std::vector<double> h(size_t(2 * ld), 0.0);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), sums, h.size() * 8, hipMemcpyDeviceToHost, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (x) (void)hipFree(x);
  if (sums) (void)hipFree(sums);
  if (e != hipSuccess) return m->hip_fail(e, "column statistics");
  mean.assign(ncol, 0.0f);
  stdv.assign(ncol, 1.0f);
  for (int c = 0; c < ncol; ++c) {
    const double mu = h[c] / double(n);
    const double var = std::max(h[ld + c] / double(n) - mu * mu, 0.0);
    const double sd = std::sqrt(var);
    mean[c] = float(mu);
    stdv[c] = sd > 1e-12 * std::max(1.0, std::fabs(mu)) ? float(sd) : 1.0f;
  }
  return RWGT_OK;
}

extern "C" {

int rwgt_mlp_fit_normalisation(rwgt_mlp* m, const double* momenta, int32_t npart, const int32_t* event_index,
                               const int32_t* card_index, const float* card_params, int64_t n) {
  if (!m || !momenta || !card_index || !card_params || n < 1) return RWGT_EINVAL;
  int rc = resolve_map(m, npart);
  if (rc != RWGT_OK) return rc;
  const std::vector<float> zeros(rwgt::kMlpMaxIn, 0.0f), ones(rwgt::kMlpMaxIn, 1.0f);
  hipError_t e = hipMemcpy(m->mean, zeros.data(), zeros.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->stdv, ones.data(), ones.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->istd, ones.data(), ones.size() * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) return m->hip_fail(e, "normalisation");
  const int ld = m->layers[0].in;
  auto fill = [&](int64_t a, int64_t b, float* x) {
    const double* mom = event_index ? momenta : momenta + a * npart * 4;
    return rwgt::mlp_features(m->fm, mom, event_index ? event_index + a : nullptr, card_index + a, card_params,
                              m->mean, m->istd, x, b - a, b - a, ld, m->stream);
  };
  std::vector<float> mean, stdv;
  rc = column_stats(m, n, ld, m->n_in, fill, mean, stdv);
  if (rc != RWGT_OK) return rc;
  return rwgt_mlp_set_normalisation(m, mean.data(), stdv.data());
}

int rwgt_mlp_fit_target_scale(rwgt_mlp* m, const float* y, int64_t n) {
  if (!m || !y || n < 1) return RWGT_EINVAL;
  auto fill = [&](int64_t a, int64_t b, float* x) {
    return hipMemcpyAsync(x, y + a, size_t(b - a) * 4, hipMemcpyDeviceToDevice, m->stream);
  };
  std::vector<float> mean, stdv;
  int rc = column_stats(m, n, 1, 1, fill, mean, stdv);
  if (rc != RWGT_OK) return rc;
  return rwgt_mlp_set_target_scale(m, mean[0], stdv[0]);
}

int rwgt_mlp_fit_grid(rwgt_mlp* m, const double* momenta, int32_t npart, int64_t nevt, const float* card_params,
                      int32_t ncards, const float* y) {
  if (!m || !momenta || !card_params || !y || nevt < 1 || ncards < 1) return RWGT_EINVAL;
  const int64_t total = nevt * ncards;
  if (nevt > INT32_MAX || total > (int64_t(1) << 40)) return m->fail(RWGT_EINVAL, "grid too large");
  int rc = resolve_map(m, npart);
  if (rc != RWGT_OK) return rc;
  const std::vector<float> zeros(rwgt::kMlpMaxIn, 0.0f), ones(rwgt::kMlpMaxIn, 1.0f);
  hipError_t e = hipMemcpy(m->mean, zeros.data(), zeros.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->stdv, ones.data(), ones.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->istd, ones.data(), ones.size() * 4, hipMemcpyHostToDevice);
  int32_t* idx = nullptr;
  const int64_t chunk = int64_t(1) << 18;
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&idx), size_t(2 * chunk) * 4);
  if (e != hipSuccess) {
    if (idx) (void)hipFree(idx);
    return m->hip_fail(e, "normalisation");
  }
  const int ld = m->layers[0].in;
  const rwgt::Shuffle in_order;                          // n = 0: pairs in order
  auto fill = [&](int64_t a, int64_t b, float* x) {
    hipError_t r = rwgt::mlp_gather_pairs(in_order, a, b - a, nevt, nullptr, idx, idx + chunk, nullptr, m->stream);
    if (r == hipSuccess)
      r = rwgt::mlp_features(m->fm, momenta, idx, idx + chunk, card_params, m->mean, m->istd, x, b - a, b - a, ld,
                             m->stream);
    return r;
  };
  std::vector<float> mean, stdv;
  rc = column_stats(m, total, ld, m->n_in, fill, mean, stdv);
  (void)hipFree(idx);
  if (rc == RWGT_OK) rc = rwgt_mlp_set_normalisation(m, mean.data(), stdv.data());
  if (rc == RWGT_OK) rc = rwgt_mlp_fit_target_scale(m, y, total);
  return rc;
}

int rwgt_mlp_forward(rwgt_mlp* m, const void* x, int64_t n, float* heads_out) {
  if (!m || !x || n < 1) return RWGT_EINVAL;
  int rc = m->forward(x, pad64(n));
  if (rc != RWGT_OK) return rc;
  if (heads_out) {
    hipError_t e = rwgt::mlp_heads(m->z.back(), 32, n, m->ym, m->ys, heads_out, 32, m->stream);
    if (e != hipSuccess) return m->hip_fail(e, "heads");
  }
  return RWGT_OK;
}

int rwgt_mlp_predict(rwgt_mlp* m, const double* momenta, int32_t npart, const int32_t* event_index,
                     const int32_t* card_index, const float* card_params, int64_t n, float* heads_out) {
  if (!m || !momenta || !card_index || !card_params || !heads_out || n < 0) return RWGT_EINVAL;
  int rc = resolve_map(m, npart);
  if (rc != RWGT_OK) return rc;
  if (!m->fused()) return m->fail(RWGT_EINVAL, "network not eligible for the fused kernel (BF16, width 128 or 256, "
                                               "depth 2..9, 4 or 5 particles)");
  if (n == 0) return RWGT_OK;
  return m->infer(momenta, event_index, card_index, card_params, n, heads_out, nullptr, nullptr, nullptr, nullptr,
                  0.0f);
}

int rwgt_mlp_train_step(rwgt_mlp* m, const void* x, const float* y, int64_t n, float lr, float* loss_out) {
  if (!m || !x || !y || n < 1) return RWGT_EINVAL;
  const int64_t rows = pad64(n);
  int rc = RWGT_OK;
  if (m->fused_train()) {
    rwgt::TrainArgs a;
    a.x = static_cast<const float*>(x);
    a.y = y;
    a.n = n;
    a.rows = rows;
    rc = m->train_fused(a, lr);
  } else {
    rc = m->forward(x, rows);
    if (rc == RWGT_OK) rc = m->backward(y, n, rows);
    if (rc == RWGT_OK && lr > 0.0f) rc = m->update(lr);
  }
  if (rc == RWGT_OK && loss_out) {
    hipError_t e = hipMemcpyAsync(loss_out, m->loss, 4, hipMemcpyDeviceToDevice, m->stream);
    if (e != hipSuccess) return m->hip_fail(e, "copy loss");
  }
  return rc;
}

int rwgt_mlp_input_bytes(const rwgt_mlp* m, int64_t n, int64_t* bytes) {
  if (!m || !bytes || n < 0) return RWGT_EINVAL;
  *bytes = pad64(n) * m->layers[0].in * 4;
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
