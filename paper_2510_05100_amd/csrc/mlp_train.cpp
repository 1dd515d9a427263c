// Surrogate training, calibration and checkpoints behind the C ABI
// (rwgt_mlp_train, rwgt_mlp_calibrate, rwgt_mlp_save / rwgt_mlp_load in
// include/rwgt.h): the epoch loop over a shuffled (event, card) grid with its
// learning-rate schedule, the calibration quantile of the error head, and a
// binary checkpoint holding everything a resumed run needs (FP32 master
// parameters, both Adam moments and their step count, the schedule, the
// epoch reached, normalisations and the calibration factor).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rwgt.h"
#include "mlp.h"
#include "mlp_internal.h"
#include "shuffle.h"

namespace {

int64_t pad64(int64_t x) { return (x + 63) / 64 * 64; }
constexpr int kProbeEvery = 64;          // the loss is read on every 64th step of an epoch
constexpr int64_t kPredictChunk = int64_t(1) << 18;

// Linear-interpolation quantile of v at q (position (n - 1) q between the
// neighbouring order statistics); reorders v.
double quantile(std::vector<double>& v, double q) {
  const double h = double(v.size() - 1) * q;
  const size_t lo = size_t(std::floor(h));
  std::nth_element(v.begin(), v.begin() + lo, v.end());
  const double a = v[lo];
  if (lo + 1 >= v.size()) return a;
  const double b = *std::min_element(v.begin() + lo + 1, v.end());
  return a + (h - double(lo)) * (b - a);
}

}  // namespace

int rwgt_mlp::ensure_train(int64_t batch, int64_t probes) {
  if (batch <= tcap && probes <= tr_loss_cap) return RWGT_OK;
  for (void* p : twork) hipFree(p);
  twork.clear();
  tcap = tr_loss_cap = 0;
  const int64_t rows = pad64(batch);
  void *a = nullptr, *b = nullptr, *c = nullptr, *d = nullptr, *l = nullptr;
  hipError_t e = hipMalloc(&a, size_t(rows) * 4);
  if (e == hipSuccess) twork.push_back(a), e = hipMalloc(&b, size_t(rows) * 4);
  if (e == hipSuccess) twork.push_back(b), e = hipMalloc(&c, size_t(rows) * 4);
  if (e == hipSuccess) twork.push_back(c), e = hipMalloc(&d, size_t(rows) * layers[0].in * 4);
  if (e == hipSuccess) twork.push_back(d), e = hipMalloc(&l, size_t(std::max<int64_t>(probes, 1)) * 4);
  if (e == hipSuccess) twork.push_back(l);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(training batch)");
  tr_ev = static_cast<int32_t*>(a);
  tr_cd = static_cast<int32_t*>(b);
  tr_y = static_cast<float*>(c);
  tr_x = static_cast<float*>(d);
  tr_loss = static_cast<float*>(l);
  tcap = batch;
  tr_loss_cap = std::max<int64_t>(probes, 1);
  // padded target rows stay defined (the loss reads n_valid rows only)
  e = hipMemsetAsync(tr_y, 0, size_t(rows) * 4, stream);
  return e == hipSuccess ? RWGT_OK : hip_fail(e, "clear training batch");
}

int rwgt_mlp::train_fused(const rwgt::TrainArgs& rows_in, float lr) {
  int rc = pack();
  if (rc != RWGT_OK) return rc;
  const int L = int(layers.size()), nh = L - 2;
  const int R = rwgt::train_tile_rows(width);
  const int64_t tiles = (rows_in.n + R - 1) / R;
  if (rows_in.n < 1 || tiles > INT32_MAX) return fail(RWGT_EINVAL, "bad row count");
  const int groups = int(std::min<int64_t>(tiles, rwgt::kTrainMaxGroups));
  const int64_t pstride = (adam_total + 1 + 63) / 64 * 64;
  if (groups > tr_groups || pstride != tr_pstride) {
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (tr_part) hipFree(tr_part);
    if (tr_zws) hipFree(tr_zws);
    tr_part = tr_zws = nullptr;
    tr_groups = 0;
    e = hipMalloc(&tr_part, size_t(groups) * size_t(pstride) * 4);
    if (e == hipSuccess) e = hipMalloc(&tr_zws, size_t(groups) * size_t(rwgt::train_zws_floats(width, nh)) * 4);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(fused training workspace)");
    tr_groups = groups;
    tr_pstride = pstride;
  }
  rwgt::TrainArgs a = rows_in;
  a.fm = fm;
  a.mean = mean;
  a.istd = istd;
  a.w0hi = p0hi;
  a.w0lo = p0lo;
  a.b0 = layers[0].b;
  a.wh = phid;
  a.wht = phid_t;
  a.bh = pbias;
  a.nh = nh;
  a.whead = layers[size_t(L - 1)].w;
  a.bhead = layers[size_t(L - 1)].b;
  a.lambda = lambda;
  a.ym = ym;
  a.ys = ys;
  a.zws = tr_zws;
  a.part = tr_part;
  a.pstride = pstride;
  a.total = adam_total;
  int64_t begin = 0;                     // segment order of the Adam table: W then b per layer
  for (int l = 0; l < L; ++l) {
    a.off_w[l] = begin;
    begin += int64_t(layers[size_t(l)].out) * layers[size_t(l)].in;
    a.off_b[l] = begin;
    begin += layers[size_t(l)].out;
  }
  a.tiles = int(tiles);
  a.groups = groups;
  hipError_t e = rwgt::mlp_train_grads(width, a, stream);
  if (e != hipSuccess) return hip_fail(e, "fused training step");
  const int adam = lr > 0.0f ? 1 : 0;
  float c1 = 0.0f, c2 = 0.0f;
  if (adam) {
    ++t;
    c1 = 1.0f / (1.0f - std::pow(b1, float(t)));
    c2 = 1.0f / (1.0f - std::pow(b2, float(t)));
  }
  e = rwgt::mlp_train_update(adam_segs, pack_segs, adam_nseg, adam_total, tr_part, groups, pstride, loss, adam, lr,
                             b1, b2, eps, c1, c2, stream);
  if (e != hipSuccess) return hip_fail(e, "fused training update");
  return RWGT_OK;                        // the packed copies were refreshed with the parameters
}

int rwgt_mlp::predict_rows(const double* mom, const int32_t* ev, const int32_t* cd, const float* cpar, int64_t n,
                           float* heads) {
  if (fused()) return infer(mom, ev, cd, cpar, n, heads, nullptr, nullptr, nullptr, nullptr, 0.0f);
  const int64_t rows = pad64(n);
  int rc = ensure_train(std::max(n, tcap), tr_loss_cap);
  if (rc != RWGT_OK) return rc;
  hipError_t e =
      rwgt::mlp_features(fm, mom, ev, cd, cpar, mean, istd, tr_x, n, rows, layers[0].in, stream);
  if (e != hipSuccess) return hip_fail(e, "features");
  rc = forward(tr_x, rows);
  if (rc != RWGT_OK) return rc;
  e = rwgt::mlp_heads(z.back(), 32, n, ym, ys, heads, 2, stream);
  return e == hipSuccess ? RWGT_OK : hip_fail(e, "heads");
}

extern "C" {

int rwgt_train_order(uint64_t seed, int64_t epoch, int64_t n, int64_t pos0, int64_t count, int64_t* out) {
  if (!out || n < 1 || epoch < 0 || pos0 < 0 || count < 0 || pos0 + count > n) return RWGT_EINVAL;
  const rwgt::Shuffle s = rwgt::make_shuffle(seed, epoch, n);
  for (int64_t i = 0; i < count; ++i) out[i] = rwgt::shuffled(s, pos0 + i);
  return RWGT_OK;
}

int rwgt_mlp_get_progress(const rwgt_mlp* m, int64_t* epoch, int64_t* steps, int64_t* adam_steps) {
  if (!m || !epoch || !steps || !adam_steps) return RWGT_EINVAL;
  *epoch = m->epoch;
  *steps = m->step;
  *adam_steps = m->t;
  return RWGT_OK;
}

int rwgt_mlp_train(rwgt_mlp* m, const double* momenta, int32_t npart, int64_t nevt, const float* card_params,
                   int32_t ncards, const float* y, const rwgt_train_cfg* cfg, int32_t epoch_end, float* epoch_loss) {
  if (!m) return RWGT_EINVAL;
  if (!momenta || !card_params || !y || !cfg || nevt < 1 || ncards < 1)
    return m->fail(RWGT_EINVAL, "bad arguments");
  const int64_t total = nevt * ncards;
  if (nevt > INT32_MAX || total > (int64_t(1) << 40)) return m->fail(RWGT_EINVAL, "grid too large");
  if (cfg->batch < 1 || cfg->batch > total || cfg->batch > INT32_MAX / 2 || cfg->epochs < 1 || !(cfg->lr > 0.0f) ||
      !(cfg->lr_final > 0.0f) || !std::isfinite(cfg->lr) || !std::isfinite(cfg->lr_final))
    return m->fail(RWGT_EINVAL, "bad schedule (batch in [1, pairs], epochs >= 1, learning rates > 0)");
  if (m->has_sched) {
    const auto& s = m->sched;
    if (s.batch != cfg->batch || s.epochs != cfg->epochs || s.lr != cfg->lr || s.lr_final != cfg->lr_final ||
        s.seed != cfg->seed)
      return m->fail(RWGT_EINVAL, "a resumed run must keep the schedule it started with");
  }
  if (epoch_end <= m->epoch || epoch_end > cfg->epochs)
    return m->fail(RWGT_EINVAL, "epoch_end must lie in (epochs done, schedule epochs]");
  int rc = resolve_map(m, npart);
  if (rc != RWGT_OK) return rc;
  const int64_t batch = cfg->batch, rows = pad64(batch);
  const int64_t per_epoch = total / batch;
  const int64_t nsteps = per_epoch * cfg->epochs;
  const int64_t probes = (per_epoch + kProbeEvery - 1) / kProbeEvery;
  rc = m->ensure_train(batch, probes);
  if (rc != RWGT_OK) return rc;
  if (!m->has_sched) {
    m->sched.batch = batch;
    m->sched.epochs = cfg->epochs;
    m->sched.lr = cfg->lr;
    m->sched.lr_final = cfg->lr_final;
    m->sched.seed = cfg->seed;
    m->has_sched = true;
  }
  const int ld = m->layers[0].in;
  // one fused step per batch (rows straight from the grid) where the network
  // and feature map allow it; else the layered step on gathered rows
  const bool fused = m->fused_train() && m->fused();
  std::vector<float> probe(static_cast<size_t>(probes));
  const int64_t first = m->epoch;
  for (int64_t ep = first; ep < epoch_end; ++ep) {
    const rwgt::Shuffle sh = rwgt::make_shuffle(cfg->seed, ep, total);
    hipError_t e = hipSuccess;
    int64_t np = 0;
    for (int64_t b = 0; b < per_epoch; ++b) {
      const double frac = double(m->step) / double(std::max<int64_t>(1, nsteps - 1));
      const float lr = float(double(cfg->lr) * std::pow(double(cfg->lr_final) / double(cfg->lr), frac));
      if (fused) {
        rwgt::TrainArgs a;
        a.sh = sh;
        a.pos0 = b * batch;
        a.nevt = nevt;
        a.mom = momenta;
        a.cpar = card_params;
        a.ygrid = y;
        a.n = batch;
        rc = m->train_fused(a, lr);
      } else {
        e = rwgt::mlp_gather_pairs(sh, b * batch, batch, nevt, y, m->tr_ev, m->tr_cd, m->tr_y, m->stream);
        if (e == hipSuccess)
          e = rwgt::mlp_features(m->fm, momenta, m->tr_ev, m->tr_cd, card_params, m->mean, m->istd, m->tr_x, batch,
                                 rows, ld, m->stream);
        if (e != hipSuccess) return m->hip_fail(e, "training batch");
        rc = m->forward(m->tr_x, rows);
        if (rc == RWGT_OK) rc = m->backward(m->tr_y, batch, rows);
        if (rc == RWGT_OK) rc = m->update(lr);
      }
      if (rc != RWGT_OK) return rc;
      if (b % kProbeEvery == 0) {
        e = hipMemcpyAsync(m->tr_loss + np, m->loss, 4, hipMemcpyDeviceToDevice, m->stream);
        if (e != hipSuccess) return m->hip_fail(e, "loss probe");
        ++np;
      }
      ++m->step;
    }
    if (epoch_loss) {
      e = hipMemcpyAsync(probe.data(), m->tr_loss, size_t(np) * 4, hipMemcpyDeviceToHost, m->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
      if (e != hipSuccess) return m->hip_fail(e, "loss probe");
      double acc = 0.0;
      for (int64_t k = 0; k < np; ++k) acc += double(probe[size_t(k)]) / double(batch);
      epoch_loss[ep - first] = float(acc / double(std::max<int64_t>(np, 1)));
    }
    m->epoch = ep + 1;
  }
  return RWGT_OK;
}

int rwgt_mlp_calibrate(rwgt_mlp* m, const double* momenta, int32_t npart, int64_t nevt, const float* card_params,
                       int32_t ncards, const float* y, double coverage, double* stats) {
  if (!m) return RWGT_EINVAL;
  if (!momenta || !card_params || !y || !stats || nevt < 1 || ncards < 1 || !(coverage > 0.0) || !(coverage < 1.0))
    return m->fail(RWGT_EINVAL, "bad arguments (coverage in (0, 1))");
  const int64_t total = nevt * ncards;
  if (nevt > INT32_MAX || total > (int64_t(1) << 34)) return m->fail(RWGT_EINVAL, "grid too large");
  int rc = resolve_map(m, npart);
  if (rc != RWGT_OK) return rc;
  const int64_t chunk = std::min(total, kPredictChunk);
  void* buf = nullptr;          // ev, cd, y of a chunk, then its heads
  hipError_t e = hipMalloc(&buf, size_t(chunk) * 5 * 4);
  if (e != hipSuccess) return m->hip_fail(e, "hipMalloc(calibration)");
  int32_t* ev = static_cast<int32_t*>(buf);
  int32_t* cd = ev + chunk;
  float* yb = reinterpret_cast<float*>(cd + chunk);
  float* heads = yb + chunk;
  const size_t ntot = static_cast<size_t>(total);
  std::vector<float> hy(ntot), hh(ntot * 2);
  const rwgt::Shuffle in_order;
  for (int64_t a = 0; a < total && rc == RWGT_OK; a += chunk) {
    const int64_t n = std::min(chunk, total - a);
    e = rwgt::mlp_gather_pairs(in_order, a, n, nevt, y, ev, cd, yb, m->stream);
    if (e != hipSuccess) { rc = m->hip_fail(e, "calibration rows"); break; }
    rc = m->predict_rows(momenta, ev, cd, card_params, n, heads);
    if (rc != RWGT_OK) break;
    e = hipMemcpyAsync(hy.data() + a, yb, size_t(n) * 4, hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(hh.data() + 2 * a, heads, size_t(n) * 8, hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) rc = m->hip_fail(e, "calibration copy");
  }
  (void)hipFree(buf);
  if (rc != RWGT_OK) return rc;
  // residual r = |y - mu| and its size in units of the predicted error, |r| / exp(s), in FP64
  std::vector<double> r(ntot), zq(ntot);
  for (int64_t i = 0; i < total; ++i) {
    r[size_t(i)] = std::fabs(double(hy[size_t(i)]) - double(hh[size_t(2 * i)]));
    zq[size_t(i)] = r[size_t(i)] / std::exp(double(hh[size_t(2 * i + 1)]));
  }
  for (double v : zq)
    if (!std::isfinite(v)) return m->fail(RWGT_EINVAL, "non-finite residual in the calibration set");
  const double k = quantile(zq, coverage);
  if (!(k > 0.0) || !std::isfinite(k)) return m->fail(RWGT_EINVAL, "calibration factor not positive");
  stats[0] = k;
  stats[1] = quantile(r, 0.5);
  stats[2] = quantile(r, 0.9);
  stats[3] = quantile(r, 0.999);
  m->k_cal = float(k);
  return RWGT_OK;
}

}  // extern "C"

// ------------------------------------------------------------ checkpoints
// File: "RWGTMLP\0", format version, then the fields written by put() below in
// order (little-endian, as the host stores them), then an FNV-1a 64-bit hash
// of every preceding byte.
namespace {

constexpr char kMagic[8] = {'R', 'W', 'G', 'T', 'M', 'L', 'P', '\0'};
constexpr uint32_t kVersion = 1;

uint64_t fnv1a(const std::string& s) {
  uint64_t h = 0xcbf29ce484222325ULL;
  for (unsigned char c : s) h = (h ^ c) * 0x100000001b3ULL;
  return h;
}

struct Writer {
  std::string out;
  template <class T>
  void put(const T& v) { out.append(reinterpret_cast<const char*>(&v), sizeof(T)); }
  void put_floats(const std::vector<float>& v) { out.append(reinterpret_cast<const char*>(v.data()), v.size() * 4); }
};

struct Reader {
  const std::string& in;
  size_t pos = 0;
  bool ok = true;
  template <class T>
  T get() {
    T v{};
    if (pos + sizeof(T) > in.size()) { ok = false; return v; }
    std::memcpy(&v, in.data() + pos, sizeof(T));
    pos += sizeof(T);
    return v;
  }
  std::vector<float> get_floats(int64_t n) {
    std::vector<float> v;
    if (n < 0 || pos + size_t(n) * 4 > in.size()) { ok = false; return v; }
    v.resize(size_t(n));
    std::memcpy(v.data(), in.data() + pos, size_t(n) * 4);
    pos += size_t(n) * 4;
    return v;
  }
};

struct Header {
  int32_t n_in = 0, width = 0, depth = 0, n_out = 0, precision = 0;
  int32_t fm_kind = 0, fm_npart = 0, fm_res_a = 0, fm_res_b = 0;
  double mz0 = 0.0, wz0 = 0.0;
  float ym = 0.0f, ys = 1.0f, k_cal = 0.0f, lambda = 0.0f, b1 = 0.0f, b2 = 0.0f, eps = 0.0f;
  int64_t t = 0, epoch = 0, step = 0;
  int32_t has_sched = 0;
  int64_t batch = 0;
  int32_t epochs = 0;
  float lr = 0.0f, lr_final = 0.0f;
  uint64_t seed = 0;
  int64_t nparams = 0;
};

thread_local std::string g_ckpt_error;

// Reads and checks a checkpoint file: magic, version, hash, sizes.
int read_checkpoint(const char* path, Header& h, std::vector<float>& mean, std::vector<float>& stdv,
                    std::vector<float>& params, std::vector<float>& first, std::vector<float>& second) {
  if (!path) return RWGT_EINVAL;
  FILE* f = std::fopen(path, "rb");
  if (!f) { g_ckpt_error = std::string("cannot open ") + path; return RWGT_EINVAL; }
  std::string data;
  char chunk[1 << 16];
  size_t got;
  while ((got = std::fread(chunk, 1, sizeof(chunk), f)) > 0) data.append(chunk, got);
  std::fclose(f);
  if (data.size() < sizeof(kMagic) + 4 + 8 || std::memcmp(data.data(), kMagic, sizeof(kMagic)) != 0) {
    g_ckpt_error = "not a surrogate checkpoint";
    return RWGT_ECARD;
  }
  uint64_t stored;
  std::memcpy(&stored, data.data() + data.size() - 8, 8);
  const std::string body = data.substr(0, data.size() - 8);
  if (fnv1a(body) != stored) { g_ckpt_error = "checkpoint hash mismatch (truncated or corrupted)"; return RWGT_ECARD; }
  Reader r{body};
  r.pos = sizeof(kMagic);
  if (r.get<uint32_t>() != kVersion) { g_ckpt_error = "unsupported checkpoint version"; return RWGT_ECARD; }
  h.n_in = r.get<int32_t>(); h.width = r.get<int32_t>(); h.depth = r.get<int32_t>(); h.n_out = r.get<int32_t>();
  h.precision = r.get<int32_t>();
  h.fm_kind = r.get<int32_t>(); h.fm_npart = r.get<int32_t>(); h.fm_res_a = r.get<int32_t>();
  h.fm_res_b = r.get<int32_t>();
  h.mz0 = r.get<double>(); h.wz0 = r.get<double>();
  h.ym = r.get<float>(); h.ys = r.get<float>(); h.k_cal = r.get<float>(); h.lambda = r.get<float>();
  h.b1 = r.get<float>(); h.b2 = r.get<float>(); h.eps = r.get<float>();
  h.t = r.get<int64_t>(); h.epoch = r.get<int64_t>(); h.step = r.get<int64_t>();
  h.has_sched = r.get<int32_t>(); h.batch = r.get<int64_t>(); h.epochs = r.get<int32_t>();
  h.lr = r.get<float>(); h.lr_final = r.get<float>(); h.seed = r.get<uint64_t>();
  h.nparams = r.get<int64_t>();
  if (!r.ok || h.n_in < 1 || h.n_in > 32 || h.width < 32 || h.depth < 1 || h.n_out < 2 || h.nparams < 1) {
    g_ckpt_error = "checkpoint header out of range";
    return RWGT_ECARD;
  }
  mean = r.get_floats(h.n_in);
  stdv = r.get_floats(h.n_in);
  params = r.get_floats(h.nparams);
  first = r.get_floats(h.nparams);
  second = r.get_floats(h.nparams);
  if (!r.ok || r.pos != body.size()) { g_ckpt_error = "checkpoint size does not match its header"; return RWGT_ECARD; }
  return RWGT_OK;
}

}  // namespace

extern "C" {

int rwgt_mlp_save(rwgt_mlp* m, const char* path) {
  if (!m || !path) return RWGT_EINVAL;
  int64_t np = 0;
  rwgt_mlp_num_params(m, &np);
  const size_t nps = static_cast<size_t>(np);
  std::vector<float> params(nps), first(nps), second(nps);
  int rc = pack_params(m, true, params.data(), rwgt_mlp::kCopyParams);
  if (rc == RWGT_OK) rc = pack_params(m, true, first.data(), rwgt_mlp::kCopyFirst);
  if (rc == RWGT_OK) rc = pack_params(m, true, second.data(), rwgt_mlp::kCopySecond);
  std::vector<float> mean(size_t(m->n_in)), stdv(size_t(m->n_in));
  hipError_t e = hipSuccess;
  if (rc == RWGT_OK) e = hipMemcpy(mean.data(), m->mean, size_t(m->n_in) * 4, hipMemcpyDeviceToHost);
  if (rc == RWGT_OK && e == hipSuccess) e = hipMemcpy(stdv.data(), m->stdv, size_t(m->n_in) * 4, hipMemcpyDeviceToHost);
  if (rc != RWGT_OK) return rc;
  if (e != hipSuccess) return m->hip_fail(e, "checkpoint copy");
  Writer w;
  w.out.append(kMagic, sizeof(kMagic));
  w.put(kVersion);
  w.put(int32_t(m->n_in)); w.put(int32_t(m->width)); w.put(int32_t(m->layers.size() - 1)); w.put(int32_t(m->n_out));
  w.put(int32_t(m->mode));
  w.put(int32_t(m->fm.kind)); w.put(int32_t(m->fm.npart)); w.put(int32_t(m->fm.res_a)); w.put(int32_t(m->fm.res_b));
  w.put(m->fm.mz0); w.put(m->fm.wz0);
  w.put(m->ym); w.put(m->ys); w.put(m->k_cal); w.put(m->lambda); w.put(m->b1); w.put(m->b2); w.put(m->eps);
  w.put(int64_t(m->t)); w.put(m->epoch); w.put(m->step);
  w.put(int32_t(m->has_sched)); w.put(m->sched.batch); w.put(m->sched.epochs); w.put(m->sched.lr);
  w.put(m->sched.lr_final); w.put(m->sched.seed);
  w.put(np);
  w.put_floats(mean); w.put_floats(stdv); w.put_floats(params); w.put_floats(first); w.put_floats(second);
  w.put(fnv1a(w.out));
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return m->fail(RWGT_EINVAL, std::string("cannot write ") + tmp);
  const bool ok = std::fwrite(w.out.data(), 1, w.out.size(), f) == w.out.size();
  if (std::fclose(f) != 0 || !ok || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return m->fail(RWGT_EINVAL, std::string("cannot write ") + path);
  }
  return RWGT_OK;
}

int rwgt_mlp_checkpoint_info(const char* path, int32_t* shape, int64_t* epoch, int64_t* adam_steps) {
  Header h;
  std::vector<float> a, b, c, d, e;
  const int rc = read_checkpoint(path, h, a, b, c, d, e);
  if (rc != RWGT_OK) return rc;
  if (shape) {
    shape[0] = h.n_in; shape[1] = h.width; shape[2] = h.depth; shape[3] = h.n_out; shape[4] = h.precision;
  }
  if (epoch) *epoch = h.epoch;
  if (adam_steps) *adam_steps = h.t;
  return RWGT_OK;
}

const char* rwgt_mlp_checkpoint_error(void) { return g_ckpt_error.c_str(); }

int rwgt_mlp_load(const char* path, rwgt_mlp** out) {
  if (!out) return RWGT_EINVAL;
  *out = nullptr;
  Header h;
  std::vector<float> mean, stdv, params, first, second;
  int rc = read_checkpoint(path, h, mean, stdv, params, first, second);
  if (rc != RWGT_OK) return rc;
  rwgt_mlp* m = nullptr;
  rc = rwgt_mlp_create(h.n_in, h.width, h.depth, h.n_out, h.precision, 0, &m);
  if (rc != RWGT_OK) { g_ckpt_error = "cannot create the checkpoint's network"; return rc; }
  int64_t np = 0;
  rwgt_mlp_num_params(m, &np);
  if (np != h.nparams) {
    rwgt_mlp_destroy(m);
    g_ckpt_error = "parameter count does not match the network shape";
    return RWGT_ECARD;
  }
  if (h.fm_npart != 0) {
    rc = rwgt_mlp_set_features(m, h.fm_kind, h.fm_npart, h.fm_res_a, h.fm_res_b, h.mz0, h.wz0);
    if (rc != RWGT_OK && h.fm_kind == RWGT_FEAT_RAW) {   // a raw map carries no resonance data
      m->fm.kind = RWGT_FEAT_RAW;
      m->fm.npart = h.fm_npart;
      rc = RWGT_OK;
    }
  }
  if (rc == RWGT_OK) rc = rwgt_mlp_set_normalisation(m, mean.data(), stdv.data());
  if (rc == RWGT_OK) rc = rwgt_mlp_set_target_scale(m, h.ym, h.ys);
  if (rc == RWGT_OK) rc = rwgt_mlp_set_training(m, h.lambda, h.b1, h.b2, h.eps);
  if (rc == RWGT_OK) rc = pack_params(m, false, params.data(), rwgt_mlp::kCopyParams);
  if (rc == RWGT_OK) rc = pack_params(m, false, first.data(), rwgt_mlp::kCopyFirst);
  if (rc == RWGT_OK) rc = pack_params(m, false, second.data(), rwgt_mlp::kCopySecond);
  if (rc == RWGT_OK) rc = m->refresh_copies();
  if (rc == RWGT_OK && hipDeviceSynchronize() != hipSuccess) rc = RWGT_EDEVICE;
  if (rc != RWGT_OK) {
    g_ckpt_error = "restoring the checkpoint: " + m->err;
    rwgt_mlp_destroy(m);
    return rc;
  }
  m->k_cal = h.k_cal;
  m->t = h.t;
  m->epoch = h.epoch;
  m->step = h.step;
  m->has_sched = h.has_sched != 0;
  m->sched.batch = h.batch;
  m->sched.epochs = h.epochs;
  m->sched.lr = h.lr;
  m->sched.lr_final = h.lr_final;
  m->sched.seed = h.seed;
  *out = m;
  return RWGT_OK;
}

}  // extern "C"
