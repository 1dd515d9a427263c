// Host side of the C ABI declared in include/rwgt.h: process and SLHA
// parsing, per-card couplings, device buffers and kernel launches.
#include <hip/hip_runtime.h>

#include <cctype>
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include <chrono>
#include <cstdlib>
#include <fstream>

#include "../../include/rwgt.h"
#include "batch.h"
#define RWGT_CHECK_REGISTRY_ONLY
#include "check.h"
#undef RWGT_CHECK_REGISTRY_ONLY
#include "kernels.h"
#include "mlp.h"
#include "mlp_internal.h"

using rwgt::Card;
using rwgt::CardPair;

namespace {

thread_local std::string g_create_error;

struct ProcessDef {
  const char* text;
  int id;
  int npart;
  std::vector<std::string> layout;   // param_sets columns
  std::vector<std::string> required; // entries the original card must have
  std::vector<std::string> fixed;    // entries a new card may not change
};

const std::vector<ProcessDef>& processes() {
  static const std::vector<ProcessDef> defs = {
      {"e+ e- > mu+ mu-", rwgt::kProcEeMumu, 4,
       {"SMINPUTS 1", "RWGTEW 1", "MASS 23", "DECAY 23"},
       {"SMINPUTS 1", "RWGTEW 1", "MASS 23", "DECAY 23"}, {}},
      {"u u~ > e+ e- g", rwgt::kProcUuEeg, 5,
       {"SMINPUTS 1", "SMINPUTS 3", "RWGTEW 1", "MASS 23", "DECAY 23"},
       {"SMINPUTS 1", "SMINPUTS 3", "RWGTEW 1", "MASS 23", "DECAY 23"}, {}},
      {"g g > t t~ g g", rwgt::kProcGgTtgg, 6,
       {"SMINPUTS 3", "MASS 6"}, {"SMINPUTS 3", "MASS 6"}, {"MASS 6"}},
      {"g g > t t~ t t~", rwgt::kProcGgTttt, 6,
       {"SMINPUTS 3", "MASS 6"}, {"SMINPUTS 3", "MASS 6"}, {"MASS 6"}},
  };
  return defs;
}

std::string normalise_ws(const char* s) {
  std::istringstream in(s);
  std::string tok, out;
  while (in >> tok) out += (out.empty() ? "" : " ") + tok;
  return out;
}

std::string upper(std::string s) {
  for (auto& c : s) c = char(std::toupper(static_cast<unsigned char>(c)));
  return s;
}

// Minimal SLHA reader: "BLOCK NAME" opens a block whose lines are "id value";
// "DECAY pdg width" sets "DECAY pdg".  '#' starts a comment.
bool parse_slha(const char* text, std::map<std::string, double>& out, std::string& err) {
  std::istringstream in(text);
  std::string line, block;
  int lineno = 0;
  while (std::getline(in, line)) {
    ++lineno;
    const auto hash = line.find('#');
    if (hash != std::string::npos) line.resize(hash);
    std::istringstream ls(line);
    std::string first;
    if (!(ls >> first)) continue;
    const std::string kw = upper(first);
    if (kw == "BLOCK") {
      if (!(ls >> block)) { err = "line " + std::to_string(lineno) + ": BLOCK without a name"; return false; }
      block = upper(block);
      continue;
    }
    if (kw == "DECAY") {
      std::string pdg;
      double w;
      if (!(ls >> pdg >> w)) { err = "line " + std::to_string(lineno) + ": malformed DECAY"; return false; }
      out["DECAY " + pdg] = w;
      block.clear();
      continue;
    }
    if (block.empty()) { err = "line " + std::to_string(lineno) + ": entry outside a block"; return false; }
    double v;
    if (!(ls >> v)) { err = "line " + std::to_string(lineno) + ": malformed entry in block " + block; return false; }
    out[block + " " + first] = v;
  }
  return true;
}

// Fermion (charge, weak isospin) in species order e, mu, u, t.
constexpr double kQ[4] = {-1.0, -1.0, 2.0 / 3.0, 2.0 / 3.0};
constexpr double kT3[4] = {-0.5, -0.5, 0.5, 0.5};

double get(const std::map<std::string, double>& m, const char* key, double fallback) {
  auto it = m.find(key);
  return it == m.end() ? fallback : it->second;
}

// Couplings of one card (textbook electroweak and QCD vertex factors).
template <class R>
Card<R> couplings(const std::map<std::string, double>& m) {
  const double pi = 3.14159265358979323846;
  const double inv_alpha = get(m, "SMINPUTS 1", 0.0);
  const double as = get(m, "SMINPUTS 3", 0.0);
  const double sw2 = get(m, "RWGTEW 1", 0.0);
  const double e = inv_alpha > 0.0 ? std::sqrt(4.0 * pi / inv_alpha) : 0.0;
  const double gs = std::sqrt(4.0 * pi * as);
  const double sw = std::sqrt(sw2), cw = std::sqrt(1.0 - sw2);
  const double gz = (sw > 0.0 && cw > 0.0) ? e / (sw * cw) : 0.0;
  Card<R> c;
  c.gqq = R(gs);                    // i g_s gamma^mu t^a
  c.g3 = R(gs);
  c.g4 = R(gs * gs);
  for (int f = 0; f < 4; ++f) {
    c.a[f] = R(-e * kQ[f]);                      // -i e Q gamma^mu
    c.zL[f] = R(-gz * (kT3[f] - kQ[f] * sw2));   // -i gZ gL gamma^mu P_L
    c.zR[f] = R(-gz * (-kQ[f] * sw2));           // -i gZ gR gamma^mu P_R
  }
  c.mz = get(m, "MASS 23", 0.0);
  c.wz = get(m, "DECAY 23", 0.0);
  c.mt = get(m, "MASS 6", 0.0);
  return c;
}

CardPair card_pair(const std::map<std::string, double>& m) {
  CardPair p;
  p.d = couplings<double>(m);
  p.f = couplings<float>(m);
  return p;
}

}  // namespace

struct rwgt_ctx {
  const ProcessDef* def = nullptr;
  int precision = 0;
  int device = 0;
  std::map<std::string, double> card;
  hipStream_t stream = nullptr;
  double* soa = nullptr;
  int64_t soa_events = 0;
  CardPair* dcards = nullptr;
  int dcards_cap = 0;
  CardPair* hcards = nullptr;   // pinned staging for the card upload
  int hcards_cap = 0;
  hipEvent_t upload_done = nullptr;
  bool upload_pending = false;
  bool profiling = false;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};   // before ingest, after ingest, after ME
  // surrogate path workspace
  void* sur_x = nullptr;
  int32_t* sur_list = nullptr;
  unsigned int* sur_count = nullptr;
  float* sur_heads = nullptr;
  CardPair* sur_cards = nullptr;
  float* sur_cpar = nullptr;
  int64_t sur_cap = 0;
  int sur_card_cap = 0;
  std::vector<double> sur_table;   // the param_table the device tables were built from
  // coupling-factored path: probe |M|^2 and per-card factors
  double* fac_probe = nullptr;
  int64_t fac_probe_cap = 0;
  rwgt::FactorCard* fac_cards = nullptr;
  int fac_cards_cap = 0;
  // per-event strong coupling: alpha_s of each card
  double* as_cards = nullptr;
  int as_cards_cap = 0;
  // cancellation guard of the mixed path: events whose kappa exceeds
  // guard_kmax are re-evaluated in double precision (guard_kmax <= 0: off)
  double guard_kmax = rwgt::kGuardKappaDefault;
  int32_t* guard_list = nullptr;
  unsigned int* guard_count = nullptr;
  int64_t guard_cap = 0;
  bool guard_ran = false;                  // the last evaluation ran the guard
  // device copies of caller arrays that live in host memory (rwgt_eval,
  // rwgt_me2): momenta, then weights in, then outputs
  double* stage = nullptr;
  size_t stage_bytes = 0;
  // non-finite outputs of the last evaluation: per-block counts on the device
  unsigned long long* nf_part = nullptr;
  unsigned long long* nf_host = nullptr;   // pinned
  int nf_blocks = 0;                       // blocks of the last count (0: nothing counted)
  std::string err;

  int fail(int code, const std::string& msg) {
    err = msg;
    return code;
  }
  int hip_fail(hipError_t e, const char* what) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? RWGT_ENOMEM : RWGT_EDEVICE;
  }
  ~rwgt_ctx() {
    if (upload_done) { hipEventSynchronize(upload_done); hipEventDestroy(upload_done); }
    for (auto& e : ev)
      if (e) hipEventDestroy(e);
    if (stream) hipStreamSynchronize(stream); else hipDeviceSynchronize();
    if (soa) hipFree(soa);
    if (dcards) hipFree(dcards);
    if (hcards) hipHostFree(hcards);
    for (void* p : {sur_x, static_cast<void*>(sur_list), static_cast<void*>(sur_count), static_cast<void*>(sur_heads),
                    static_cast<void*>(sur_cards), static_cast<void*>(sur_cpar), static_cast<void*>(fac_probe),
                    static_cast<void*>(fac_cards), static_cast<void*>(as_cards), static_cast<void*>(nf_part),
                    static_cast<void*>(guard_list), static_cast<void*>(guard_count), static_cast<void*>(stage)})
      if (p) hipFree(p);
    if (nf_host) hipHostFree(nf_host);
  }
};

namespace {

int ensure_buffers(rwgt_ctx* c, int64_t nevt, int ncards) {
  if (nevt > c->soa_events) {
    if (c->soa) {
      hipStreamSynchronize(c->stream);
      hipFree(c->soa);
      c->soa = nullptr;
      c->soa_events = 0;
    }
    const size_t bytes = size_t(nevt) * size_t(c->def->npart) * 4 * sizeof(double);
    hipError_t e = hipMalloc(&c->soa, bytes);
    if (e != hipSuccess) return c->hip_fail(e, "hipMalloc(momenta SoA)");
    c->soa_events = nevt;
  }
  if (ncards > c->dcards_cap) {
    if (c->dcards) { hipStreamSynchronize(c->stream); hipFree(c->dcards); c->dcards = nullptr; }
    if (c->upload_pending) { hipEventSynchronize(c->upload_done); c->upload_pending = false; }
    if (c->hcards) { hipHostFree(c->hcards); c->hcards = nullptr; }
    c->dcards_cap = c->hcards_cap = 0;
    const int cap = ncards < 16 ? 16 : ncards;
    hipError_t e = hipMalloc(&c->dcards, size_t(cap) * sizeof(CardPair));
    if (e != hipSuccess) return c->hip_fail(e, "hipMalloc(cards)");
    e = hipHostMalloc(&c->hcards, size_t(cap) * sizeof(CardPair), hipHostMallocDefault);
    if (e != hipSuccess) return c->hip_fail(e, "hipHostMalloc(cards)");
    c->dcards_cap = c->hcards_cap = cap;
  }
  return RWGT_OK;
}

// Card list [original, param_sets rows...] (with_original) or just the rows.
int build_cards(rwgt_ctx* c, const double* param_sets, int32_t nsets, bool with_original,
                std::vector<CardPair>& out) {
  const auto& layout = c->def->layout;
  out.clear();
  if (with_original) out.push_back(card_pair(c->card));
  for (int32_t k = 0; k < nsets; ++k) {
    std::map<std::string, double> m = c->card;
    for (size_t j = 0; j < layout.size(); ++j) {
      const double v = param_sets[size_t(k) * layout.size() + j];
      for (const auto& f : c->def->fixed) {
        if (f == layout[j] && v != c->card[f]) {
          return c->fail(RWGT_EPARAM, "param set " + std::to_string(k) + " changes " + f +
                                          ", an external mass fixed by the momenta");
        }
      }
      m[layout[j]] = v;
    }
    out.push_back(card_pair(m));
  }
  return RWGT_OK;
}

// Device list and count of the guard's flagged events, for nevt events.
int ensure_guard(rwgt_ctx* c, int64_t nevt) {
  if (nevt <= c->guard_cap && c->guard_count) return RWGT_OK;
  if (c->guard_list) { hipStreamSynchronize(c->stream); hipFree(c->guard_list); c->guard_list = nullptr; }
  c->guard_cap = 0;
  hipError_t e = hipSuccess;
  if (!c->guard_count) e = hipMalloc(&c->guard_count, sizeof(unsigned int));
  if (e == hipSuccess) e = hipMalloc(&c->guard_list, size_t(nevt) * sizeof(int32_t));
  if (e != hipSuccess) return c->hip_fail(e, "hipMalloc(guard list)");
  c->guard_cap = nevt;
  return RWGT_OK;
}

int run(rwgt_ctx* c, bool reweight, const double* momenta, int64_t nevt, const double* w_in,
        const double* param_sets, int32_t nsets, double* w_out, double* me_out, double* kappa_out = nullptr) {
  if (nevt < 0) return c->fail(RWGT_EINVAL, "nevt < 0");
  if (nsets < 1) return c->fail(RWGT_EINVAL, "nsets < 1");
  if (!param_sets) return c->fail(RWGT_EINVAL, "param_sets is NULL");
  std::vector<CardPair> cards;
  int rc = build_cards(c, param_sets, nsets, reweight, cards);
  if (rc != RWGT_OK) return rc;
  if (nevt == 0) return RWGT_OK;
  if (!momenta) return c->fail(RWGT_EINVAL, "momenta is NULL");
  if (reweight && !w_in) return c->fail(RWGT_EINVAL, "weights_in is NULL");
  if (reweight && !w_out) return c->fail(RWGT_EINVAL, "weights_out is NULL");
  if (!reweight && !me_out && !kappa_out) return c->fail(RWGT_EINVAL, "me2_out is NULL");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return c->hip_fail(e, "hipSetDevice");
  rc = ensure_buffers(c, nevt, int(cards.size()));
  if (rc != RWGT_OK) return rc;
  if (c->upload_pending) {
    e = hipEventSynchronize(c->upload_done);
    if (e != hipSuccess) return c->hip_fail(e, "hipEventSynchronize");
    c->upload_pending = false;
  }
  std::memcpy(c->hcards, cards.data(), cards.size() * sizeof(CardPair));
  e = hipMemcpyAsync(c->dcards, c->hcards, cards.size() * sizeof(CardPair), hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "hipMemcpyAsync(cards)");
  e = hipEventRecord(c->upload_done, c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "hipEventRecord");
  c->upload_pending = true;
  if (c->profiling) hipEventRecord(c->ev[0], c->stream);
  e = rwgt::launch_ingest(c->def->npart, momenta, c->soa, nevt, c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "ingest kernel");
  if (c->profiling) hipEventRecord(c->ev[1], c->stream);
  c->guard_ran = false;
  if (c->precision != RWGT_FP64 && (kappa_out || c->guard_kmax > 0.0)) {
    rwgt::GuardArgs g;
    if (kappa_out) {                             // kappa only: nothing flagged or re-evaluated
      g.kmax = -1.0;
      g.kappa = kappa_out;
    } else {
      rc = ensure_guard(c, nevt);
      if (rc != RWGT_OK) return rc;
      g.kmax = c->guard_kmax;
      g.flagged = c->guard_list;
      g.nflagged = c->guard_count;
      c->guard_ran = true;
    }
    e = rwgt::launch_me_guarded(c->def->id, c->precision, c->soa, nevt, c->dcards, int(cards.size()), w_in, w_out,
                                me_out, g, c->stream);
  } else {
    e = rwgt::launch_me(c->def->id, c->precision, c->soa, nevt, c->dcards, int(cards.size()), w_in, w_out, me_out,
                        c->stream);
  }
  if (e != hipSuccess) return c->hip_fail(e, "matrix-element kernel");
  if (c->profiling) hipEventRecord(c->ev[2], c->stream);
  return RWGT_OK;
}

// Queue the count of non-finite entries of out[0..n) (the outputs of the call
// that just enqueued its kernels); rwgt_nonfinite reads it back.
int count_nonfinite(rwgt_ctx* c, const double* out, int64_t n) {
  c->nf_blocks = 0;
  if (n <= 0) return RWGT_OK;
  hipError_t e = hipSuccess;
  if (!c->nf_part) {
    e = hipMalloc(&c->nf_part, rwgt::kNonfiniteBlocks * sizeof(unsigned long long));
    if (e != hipSuccess) return c->hip_fail(e, "hipMalloc(non-finite counts)");
  }
  e = rwgt::launch_nonfinite(out, n, c->nf_part, c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "non-finite count kernel");
  c->nf_blocks = rwgt::nonfinite_blocks(n);
  return RWGT_OK;
}

// Where a caller array lives.  Memory of this context's device (device or
// managed allocations) is used in place (kHere); anything else is copied
// through the context's staging buffer: pinned host memory and other devices'
// memory asynchronously on the stream (kCopy), pageable host memory the same
// way but with the call waiting for its stream before it returns (kCopyWait).
enum class Mem { kHere, kCopy, kCopyWait };

Mem where(const rwgt_ctx* c, const void* p) {
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();                     // older runtimes reject unregistered host memory
    return Mem::kCopyWait;
  }
  const bool dev = a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
  if (dev && a.device == c->device) return Mem::kHere;
  return dev || a.type == hipMemoryTypeHost ? Mem::kCopy : Mem::kCopyWait;
}

// The caller's momenta, input weights and output of one rwgt_eval / rwgt_me2
// call, replaced by staging-buffer addresses where they are not device memory
// of this context; finish() copies the output back.
struct Staged {
  const double* mom;
  const double* w_in;
  double* out;
  double* out_host = nullptr;                    // caller's output, when staged
  size_t out_bytes = 0;
  bool wait = false;                             // some array is pageable host memory

  int begin(rwgt_ctx* c, int64_t nevt, int64_t nout) {
    if (nevt <= 0 || !mom || !out) return RWGT_OK;   // run() reports the errors
    const size_t mbytes = size_t(nevt) * size_t(c->def->npart) * 4 * sizeof(double);
    const size_t wbytes = size_t(nevt) * sizeof(double);
    const size_t obytes = size_t(nout) * sizeof(double);
    const Mem wm = where(c, mom), ww = w_in ? where(c, w_in) : Mem::kHere, wo = where(c, out);
    if (wm == Mem::kHere && ww == Mem::kHere && wo == Mem::kHere) return RWGT_OK;
    wait = wm == Mem::kCopyWait || ww == Mem::kCopyWait || wo == Mem::kCopyWait;
    const size_t need = (wm != Mem::kHere ? mbytes : 0) + (ww != Mem::kHere ? wbytes : 0) +
                        (wo != Mem::kHere ? obytes : 0);
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return c->hip_fail(e, "hipSetDevice");
    if (need > c->stage_bytes) {
      if (c->stage) {
        e = hipStreamSynchronize(c->stream);   // earlier calls may still read it
        if (e != hipSuccess) return c->hip_fail(e, "hipStreamSynchronize");
        hipFree(c->stage);
        c->stage = nullptr;
        c->stage_bytes = 0;
      }
      e = hipMalloc(&c->stage, need);
      if (e != hipSuccess) return c->hip_fail(e, "hipMalloc(staging)");
      c->stage_bytes = need;
    }
    char* at = reinterpret_cast<char*>(c->stage);
    if (wm != Mem::kHere) {
      e = hipMemcpyAsync(at, mom, mbytes, hipMemcpyDefault, c->stream);
      if (e != hipSuccess) return c->hip_fail(e, "hipMemcpyAsync(momenta)");
      mom = reinterpret_cast<const double*>(at);
      at += mbytes;
    }
    if (ww != Mem::kHere) {
      e = hipMemcpyAsync(at, w_in, wbytes, hipMemcpyDefault, c->stream);
      if (e != hipSuccess) return c->hip_fail(e, "hipMemcpyAsync(weights_in)");
      w_in = reinterpret_cast<const double*>(at);
      at += wbytes;
    }
    if (wo != Mem::kHere) {
      out_host = out;
      out_bytes = obytes;
      out = reinterpret_cast<double*>(at);
    }
    return RWGT_OK;
  }

  int finish(rwgt_ctx* c) {
    hipError_t e = hipSuccess;
    if (out_host) e = hipMemcpyAsync(out_host, out, out_bytes, hipMemcpyDefault, c->stream);
    if (e == hipSuccess && wait) e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? RWGT_OK : c->hip_fail(e, "copy of the output to host memory");
  }
};

}  // namespace

namespace rwgt {

// Readers of the device bounds-check counters (check build only: every
// checked translation unit registers one while the library loads).
std::vector<BoundsReader>& bounds_readers() {
  static std::vector<BoundsReader> readers;
  return readers;
}

void register_bounds_reader(BoundsReader f) { bounds_readers().push_back(f); }

}  // namespace rwgt

extern "C" {

int rwgt_create(const char* process, const char* param_card, int precision, rwgt_ctx** out) {
  g_create_error.clear();
  if (!out) { g_create_error = "out is NULL"; return RWGT_EINVAL; }
  *out = nullptr;
  if (!process || !param_card) { g_create_error = "process or param_card is NULL"; return RWGT_EINVAL; }
  if (precision < RWGT_FP64 || precision > RWGT_MIXED_BF16) { g_create_error = "unknown precision"; return RWGT_EINVAL; }
  const std::string want = normalise_ws(process);
  const ProcessDef* def = nullptr;
  for (const auto& d : processes())
    if (want == d.text) def = &d;
  if (!def) { g_create_error = "unsupported process '" + want + "'"; return RWGT_EPROCESS; }
  std::map<std::string, double> card;
  std::string err;
  if (!parse_slha(param_card, card, err)) { g_create_error = "param card: " + err; return RWGT_ECARD; }
  for (const auto& r : def->required) {
    if (!card.count(r)) { g_create_error = "param card lacks " + r; return RWGT_ECARD; }
  }
  rwgt_ctx* c = new (std::nothrow) rwgt_ctx;
  if (!c) { g_create_error = "out of host memory"; return RWGT_ENOMEM; }
  c->def = def;
  c->precision = precision;
  c->card = card;
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->upload_done, hipEventDisableTiming);
  if (e != hipSuccess) {
    g_create_error = std::string("HIP: ") + hipGetErrorString(e);
    delete c;
    return RWGT_EDEVICE;
  }
  *out = c;
  return RWGT_OK;
}

void rwgt_destroy(rwgt_ctx* ctx) { delete ctx; }

int rwgt_param_layout(const rwgt_ctx* ctx, int32_t* npar, const char** names) {
  if (!ctx || !npar) return RWGT_EINVAL;
  *npar = int32_t(ctx->def->layout.size());
  if (names)
    for (size_t j = 0; j < ctx->def->layout.size(); ++j) names[j] = ctx->def->layout[j].c_str();
  return RWGT_OK;
}

int rwgt_original_params(const rwgt_ctx* ctx, double* values) {
  if (!ctx || !values) return RWGT_EINVAL;
  for (size_t j = 0; j < ctx->def->layout.size(); ++j) values[j] = ctx->card.at(ctx->def->layout[j]);
  return RWGT_OK;
}

int rwgt_set_stream(rwgt_ctx* ctx, void* stream) {
  if (!ctx) return RWGT_EINVAL;
  ctx->stream = static_cast<hipStream_t>(stream);
  return RWGT_OK;
}

int rwgt_eval(rwgt_ctx* ctx, const double* momenta, int64_t nevt, const double* weights_in,
              const double* param_sets, int32_t nsets, double* weights_out) {
  if (!ctx) return RWGT_EINVAL;
  ctx->err.clear();
  try {
    ctx->nf_blocks = 0;
    if (nsets < 1) return ctx->fail(RWGT_EINVAL, "nsets < 1");
    Staged st{momenta, weights_in, weights_out};
    int rc = st.begin(ctx, nevt, int64_t(nsets) * nevt);
    if (rc == RWGT_OK) rc = run(ctx, true, st.mom, nevt, st.w_in, param_sets, nsets, st.out, nullptr);
    if (rc == RWGT_OK) rc = count_nonfinite(ctx, st.out, int64_t(nsets) * nevt);
    return rc == RWGT_OK ? st.finish(ctx) : rc;
  } catch (const std::exception& ex) {
    return ctx->fail(RWGT_ENOMEM, ex.what());
  }
}

// Reweighting with the strong coupling per event (one-loop running from
// alpha_s(91.1876 GeV) with five flavours for the new cards; the event's own
// alpha_s, or the original card's run to the event scale, for the original).
int rwgt_eval_alphas(rwgt_ctx* c, const double* momenta, int64_t nevt, const double* w_in, const double* alphas_orig,
                     const double* scales, const double* param_sets, int32_t nsets, double* w_out) {
  if (!c) return RWGT_EINVAL;
  c->err.clear();
  c->nf_blocks = 0;
  if (nevt > 0 && !scales) return c->fail(RWGT_EINVAL, "scales is NULL");
  int rc = run(c, true, momenta, nevt, w_in, param_sets, nsets, w_out, nullptr);
  if (rc != RWGT_OK || nevt == 0) return rc;
  const int id = c->def->id;
  const int p = id == rwgt::kProcEeMumu ? 0 : id == rwgt::kProcUuEeg ? 1 : 4;   // power of alpha_s in |M|^2
  if (p == 0) return count_nonfinite(c, w_out, int64_t(nsets) * nevt);
  const auto& layout = c->def->layout;
  int ja = -1;
  for (size_t j = 0; j < layout.size(); ++j)
    if (layout[j] == "SMINPUTS 3") ja = int(j);
  std::vector<double> as(static_cast<size_t>(nsets));
  for (int k = 0; k < nsets; ++k) as[size_t(k)] = param_sets[size_t(k) * layout.size() + size_t(ja)];
  hipError_t e = hipSuccess;
  if (nsets > c->as_cards_cap) {
    if (c->as_cards) { (void)hipStreamSynchronize(c->stream); (void)hipFree(c->as_cards); c->as_cards = nullptr; }
    c->as_cards_cap = 0;
    e = hipMalloc(&c->as_cards, size_t(nsets) * sizeof(double));
    if (e != hipSuccess) return c->hip_fail(e, "hipMalloc(alpha_s per card)");
    c->as_cards_cap = nsets;
  }
  // pageable source: wait for the copy
  e = hipMemcpyAsync(c->as_cards, as.data(), as.size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "alpha_s upload");
  const double pi = 3.14159265358979323846;
  const double b0 = (33.0 - 2.0 * 5.0) / (12.0 * pi), mref = 91.1876;
  e = rwgt::launch_alphas(w_out, nevt, nsets, alphas_orig, scales, c->card.at("SMINPUTS 3"), c->as_cards, p, b0,
                          mref * mref, c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "per-event alpha_s");
  return count_nonfinite(c, w_out, int64_t(nsets) * nevt);
}

// Coupling-factored reweighting (same result as rwgt_eval).  Electroweak
// processes: the two fermion lines (species f1, f2 of the card's coupling
// arrays) and the resonant pair (ia, ib); four probe cards give each event's
// chirality-class weights, then every card costs a few operations per event.
// QCD process: cards change alpha_s only and |M|^2 scales as g_s^8.
int rwgt_eval_factored(rwgt_ctx* c, const double* momenta, int64_t nevt, const double* w_in,
                       const double* param_sets, int32_t nsets, double* w_out) {
  if (!c) return RWGT_EINVAL;
  c->err.clear();
  c->nf_blocks = 0;
  if (nevt < 0) return c->fail(RWGT_EINVAL, "nevt < 0");
  if (nsets < 1) return c->fail(RWGT_EINVAL, "nsets < 1");
  if (!param_sets) return c->fail(RWGT_EINVAL, "param_sets is NULL");
  try {
    std::vector<CardPair> cards;
    int rc = build_cards(c, param_sets, nsets, true, cards);
    if (rc != RWGT_OK) return rc;
    if (nevt == 0) return RWGT_OK;
    if (!momenta || !w_in || !w_out) return c->fail(RWGT_EINVAL, "NULL device pointer");
    const int id = c->def->id;
    const bool ew = id == rwgt::kProcEeMumu || id == rwgt::kProcUuEeg;
    const int f1 = id == rwgt::kProcUuEeg ? 2 : 0;         // u or e line
    const int f2 = id == rwgt::kProcUuEeg ? 0 : 1;         // e or mu line
    const int ia = 2, ib = 3;                              // the outgoing lepton pair
    const Card<double>& o = cards[0].d;
    std::vector<rwgt::FactorCard> fc(cards.size());
    for (size_t k = 0; k < cards.size(); ++k) {
      const Card<double>& q = cards[k].d;
      rwgt::FactorCard& f = fc[k];
      f.A = q.a[f1] * q.a[f2];
      f.B[0] = q.zL[f1] * q.zL[f2];
      f.B[1] = q.zL[f1] * q.zR[f2];
      f.B[2] = q.zR[f1] * q.zL[f2];
      f.B[3] = q.zR[f1] * q.zR[f2];
      f.mz = q.mz;
      f.wz = q.wz;
      const double r = o.gqq != 0.0 ? q.gqq / o.gqq : 0.0;
      f.g = id == rwgt::kProcEeMumu ? 1.0 : id == rwgt::kProcUuEeg ? r * r : std::pow(r, 8);
    }
    // probe cards: EW, the original with every photon and Z coupling zero but
    // the Z couplings of one chirality class (1 x 1); QCD, the original card
    std::vector<CardPair> probes;
    if (ew) {
      for (int cl = 0; cl < 4; ++cl) {
        CardPair p = cards[0];
        for (int f = 0; f < 4; ++f) {
          p.d.a[f] = p.d.zL[f] = p.d.zR[f] = 0.0;
          p.f.a[f] = p.f.zL[f] = p.f.zR[f] = 0.0f;
        }
        (cl & 2 ? p.d.zR : p.d.zL)[f1] = 1.0;
        (cl & 1 ? p.d.zR : p.d.zL)[f2] = 1.0;
        (cl & 2 ? p.f.zR : p.f.zL)[f1] = 1.0f;
        (cl & 1 ? p.f.zR : p.f.zL)[f2] = 1.0f;
        probes.push_back(p);
      }
    } else {
      probes.push_back(cards[0]);
    }
    const int nprobe = int(probes.size());
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return c->hip_fail(e, "hipSetDevice");
    rc = ensure_buffers(c, nevt, nprobe);
    if (rc != RWGT_OK) return rc;
    if (int64_t(nprobe) * nevt > c->fac_probe_cap) {
      if (c->fac_probe) { (void)hipStreamSynchronize(c->stream); (void)hipFree(c->fac_probe); c->fac_probe = nullptr; }
      c->fac_probe_cap = 0;
      e = hipMalloc(&c->fac_probe, size_t(nprobe) * nevt * sizeof(double));
      if (e != hipSuccess) return c->hip_fail(e, "hipMalloc(probe |M|^2)");
      c->fac_probe_cap = int64_t(nprobe) * nevt;
    }
    if (int(fc.size()) > c->fac_cards_cap) {
      if (c->fac_cards) { (void)hipStreamSynchronize(c->stream); (void)hipFree(c->fac_cards); c->fac_cards = nullptr; }
      c->fac_cards_cap = 0;
      e = hipMalloc(&c->fac_cards, fc.size() * sizeof(rwgt::FactorCard));
      if (e != hipSuccess) return c->hip_fail(e, "hipMalloc(factor cards)");
      c->fac_cards_cap = int(fc.size());
    }
    if (c->upload_pending) {
      e = hipEventSynchronize(c->upload_done);
      if (e != hipSuccess) return c->hip_fail(e, "hipEventSynchronize");
      c->upload_pending = false;
    }
    std::memcpy(c->hcards, probes.data(), probes.size() * sizeof(CardPair));
    e = hipMemcpyAsync(c->dcards, c->hcards, probes.size() * sizeof(CardPair), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->upload_done, c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "probe card upload");
    c->upload_pending = true;
    // the factor table comes from pageable memory: wait for that copy
    e = hipMemcpyAsync(c->fac_cards, fc.data(), fc.size() * sizeof(rwgt::FactorCard), hipMemcpyHostToDevice,
                       c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "factor card upload");
    e = rwgt::launch_ingest(c->def->npart, momenta, c->soa, nevt, c->stream);
    if (e == hipSuccess)
      e = rwgt::launch_me(id, c->precision, c->soa, nevt, c->dcards, nprobe, nullptr, nullptr, c->fac_probe,
                          c->stream);
    if (e == hipSuccess)
      e = rwgt::launch_factored(ew, c->soa, c->def->npart, nevt, ia, ib, c->fac_probe, o.mz, o.wz, c->fac_cards,
                                int(fc.size()), w_in, w_out, c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "factored evaluation");
    return count_nonfinite(c, w_out, int64_t(nsets) * nevt);
  } catch (const std::exception& ex) {
    return c->fail(RWGT_ENOMEM, ex.what());
  }
}

int rwgt_me2(rwgt_ctx* ctx, const double* momenta, int64_t nevt, const double* param_sets, int32_t nsets,
             double* me2_out) {
  if (!ctx) return RWGT_EINVAL;
  ctx->err.clear();
  try {
    ctx->nf_blocks = 0;
    if (nsets < 1) return ctx->fail(RWGT_EINVAL, "nsets < 1");
    Staged st{momenta, nullptr, me2_out};
    int rc = st.begin(ctx, nevt, int64_t(nsets) * nevt);
    if (rc == RWGT_OK) rc = run(ctx, false, st.mom, nevt, nullptr, param_sets, nsets, nullptr, st.out);
    if (rc == RWGT_OK) rc = count_nonfinite(ctx, st.out, int64_t(nsets) * nevt);
    return rc == RWGT_OK ? st.finish(ctx) : rc;
  } catch (const std::exception& ex) {
    return ctx->fail(RWGT_ENOMEM, ex.what());
  }
}

int rwgt_nonfinite(rwgt_ctx* c, int64_t* count) {
  if (!c || !count) return RWGT_EINVAL;
  *count = 0;
  if (c->nf_blocks == 0) return RWGT_OK;
  hipError_t e = hipSuccess;
  if (!c->nf_host) {
    e = hipHostMalloc(&c->nf_host, rwgt::kNonfiniteBlocks * sizeof(unsigned long long), hipHostMallocDefault);
    if (e != hipSuccess) return c->hip_fail(e, "hipHostMalloc(non-finite counts)");
  }
  e = hipMemcpyAsync(c->nf_host, c->nf_part, size_t(c->nf_blocks) * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                     c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "non-finite count read-back");
  unsigned long long s = 0;
  for (int b = 0; b < c->nf_blocks; ++b) s += c->nf_host[b];
  *count = int64_t(s);
  return RWGT_OK;
}

const char* rwgt_last_error(const rwgt_ctx* ctx) { return ctx ? ctx->err.c_str() : "context is NULL"; }

const char* rwgt_create_error(void) { return g_create_error.c_str(); }

int rwgt_process_layout(const char* process, int32_t* npar, const char** names) {
  if (!process || !npar) return RWGT_EINVAL;
  const std::string want = normalise_ws(process);
  for (const auto& d : processes())
    if (want == d.text) {
      *npar = int32_t(d.layout.size());
      if (names)
        for (size_t j = 0; j < d.layout.size(); ++j) names[j] = d.layout[j].c_str();
      return RWGT_OK;
    }
  return RWGT_EPROCESS;
}

// Reweighting card (MadtRex / teaRex SLHA reweighting): "launch
// [--]rwgt_name=NAME" opens a parameter set initialised to the original
// card, "set BLOCK ID VALUE" (or "set DECAY PDG VALUE") overrides one entry,
// "change fptype X" records the requested precision, other "change" lines
// and '#' comments are ignored.  Entries outside the process's layout do not
// affect its |M|^2 and are skipped.
int rwgt_reweight_card(const char* process, const char* param_card, const char* rwgt_card, int32_t cap,
                       double* param_sets, int32_t* nsets, char* names, int32_t name_len, char* fptype) {
  g_create_error.clear();
  if (!process || !param_card || !rwgt_card || !nsets || cap < 0 || (cap > 0 && !param_sets) ||
      (names && name_len < 2)) {
    g_create_error = "NULL argument or bad size";
    return RWGT_EINVAL;
  }
  *nsets = 0;
  const std::string want = normalise_ws(process);
  const ProcessDef* def = nullptr;
  for (const auto& d : processes())
    if (want == d.text) def = &d;
  if (!def) { g_create_error = "unsupported process '" + want + "'"; return RWGT_EPROCESS; }
  std::map<std::string, double> card;
  std::string err;
  if (!parse_slha(param_card, card, err)) { g_create_error = "param card: " + err; return RWGT_ECARD; }
  const size_t npar = def->layout.size();
  std::vector<double> orig(npar);
  for (size_t j = 0; j < npar; ++j) {
    auto it = card.find(def->layout[j]);
    if (it == card.end()) { g_create_error = "param card lacks " + def->layout[j]; return RWGT_ECARD; }
    orig[j] = it->second;
  }
  std::istringstream in(rwgt_card);
  std::string line;
  int lineno = 0;
  int32_t n = 0;
  std::vector<double> cur;
  auto flush = [&]() {
    if (!cur.empty() && n <= cap && n > 0) std::copy(cur.begin(), cur.end(), param_sets + size_t(n - 1) * npar);
  };
  while (std::getline(in, line)) {
    ++lineno;
    const auto hash = line.find('#');
    if (hash != std::string::npos) line.resize(hash);
    std::istringstream ls(line);
    std::string cmd;
    if (!(ls >> cmd)) continue;
    cmd = upper(cmd);
    const std::string where = "reweight card line " + std::to_string(lineno) + ": ";
    if (cmd == "LAUNCH") {
      flush();
      cur = orig;
      ++n;
      std::string name = "rwgt_" + std::to_string(n), opt;
      while (ls >> opt) {
        const auto eq = opt.find('=');
        std::string key = opt.substr(0, eq);
        while (!key.empty() && key[0] == '-') key.erase(0, 1);
        if (eq != std::string::npos && key == "rwgt_name") name = opt.substr(eq + 1);
      }
      if (names && n <= cap) {
        char* dst = names + size_t(n - 1) * size_t(name_len);
        std::snprintf(dst, size_t(name_len), "%s", name.c_str());
      }
    } else if (cmd == "SET") {
      if (cur.empty()) { g_create_error = where + "'set' before the first 'launch'"; return RWGT_ECARD; }
      std::string block, id, val;
      if (!(ls >> block >> id >> val)) {
        g_create_error = where + "expected 'set BLOCK ID VALUE'";
        return RWGT_ECARD;
      }
      char* endp = nullptr;
      const double v = std::strtod(val.c_str(), &endp);
      char* endi = nullptr;
      (void)std::strtol(id.c_str(), &endi, 10);
      if (!endp || *endp != '\0' || !endi || *endi != '\0') {
        g_create_error = where + "expected 'set BLOCK ID VALUE' with a numeric id and value";
        return RWGT_ECARD;
      }
      const std::string key = upper(block) + " " + id;
      for (size_t j = 0; j < npar; ++j)
        if (def->layout[j] == key) cur[j] = v;
    } else if (cmd == "CHANGE") {
      std::string what, val;
      ls >> what >> val;
      if (fptype && upper(what) == "FPTYPE" && !val.empty()) {
        fptype[0] = val[0];
        fptype[1] = '\0';
      }
    } else {
      g_create_error = where + "unknown command '" + cmd + "'";
      return RWGT_ECARD;
    }
  }
  flush();
  *nsets = n;
  return RWGT_OK;
}

int rwgt_process_info(const rwgt_ctx* ctx, int32_t* npart, int32_t* nhel_kept, int32_t* ncol, int32_t* ndiag) {
  if (!ctx) return RWGT_EINVAL;
  int np = 0, ng = 0, nc = 0, nd = 0;
  rwgt::process_constants(ctx->def->id, &np, &ng, &nc, &nd);
  if (npart) *npart = np;
  if (nhel_kept) *nhel_kept = ng;
  if (ncol) *ncol = nc;
  if (ndiag) *ndiag = nd;
  return RWGT_OK;
}

int rwgt_set_profiling(rwgt_ctx* ctx, int enable) {
  if (!ctx) return RWGT_EINVAL;
  if (enable && !ctx->ev[0]) {
    for (auto& e : ctx->ev) {
      const hipError_t rc = hipEventCreate(&e);
      if (rc != hipSuccess) return ctx->hip_fail(rc, "hipEventCreate");
    }
  }
  ctx->profiling = enable != 0;
  return RWGT_OK;
}

int rwgt_kernel_times(rwgt_ctx* ctx, float* ingest_ms, float* me_ms) {
  if (!ctx || !ingest_ms || !me_ms) return RWGT_EINVAL;
  if (!ctx->profiling) return ctx->fail(RWGT_EINVAL, "profiling is off");
  hipError_t e = hipEventSynchronize(ctx->ev[2]);
  if (e == hipSuccess) e = hipEventElapsedTime(ingest_ms, ctx->ev[0], ctx->ev[1]);
  if (e == hipSuccess) e = hipEventElapsedTime(me_ms, ctx->ev[1], ctx->ev[2]);
  if (e != hipSuccess) return ctx->hip_fail(e, "kernel timing");
  return RWGT_OK;
}

int rwgt_xsec(rwgt_ctx* ctx, const double* weights_in, const double* weights_out, int64_t nevt, int32_t nsets,
              double sigma, double dsigma, double norm, double* xsec, double* xerr, int32_t* fallback) {
  if (!ctx) return RWGT_EINVAL;
  ctx->err.clear();
  if (nevt < 1 || nsets < 1 || !weights_in || !weights_out || !xsec || !xerr)
    return ctx->fail(RWGT_EINVAL, "bad arguments");
  constexpr int kBlocks = 512;
  double *part = nullptr, *out = nullptr;
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = hipMalloc(&part, size_t(nsets) * (3 * kBlocks + 3) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&out, size_t(nsets) * 3 * sizeof(double));
  if (e == hipSuccess)
    e = rwgt::launch_xsec(weights_in, weights_out, nevt, nsets, sigma, dsigma, norm, part, kBlocks, out, ctx->stream);
  std::vector<double> host(size_t(nsets) * 3);
  if (e == hipSuccess) e = hipMemcpyAsync(host.data(), out, host.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (part) hipFree(part);
  if (out) hipFree(out);
  if (e != hipSuccess) return ctx->hip_fail(e, "cross-section reduction");
  for (int32_t k = 0; k < nsets; ++k) {
    xsec[k] = host[k * 3];
    xerr[k] = host[k * 3 + 1];
    if (fallback) fallback[k] = host[k * 3 + 2] != 0.0;
    if (host[k * 3 + 2] != 0.0)
      std::fprintf(stderr, "rwgt: error propagation for card %d gave no positive finite value; "
                           "using dsigma * max(sigma'/sigma, sigma/sigma')\n", int(k));
  }
  return RWGT_OK;
}

}  // extern "C"

// ------------------------------------------------ rwgt_xsec without allocation
// Scratch of rwgt_xsec_noalloc: the two passes' block partials and the
// per-card sums and results for up to kXsecStaticSets cards, in a static
// device array (each GPU holds its own copy until the process ends).  Host
// code reaches it only through the address hipGetSymbolAddress returns on
// that device (the array's name is a host-side stand-in there).
namespace {
constexpr int kXsecStaticBlocks = 512;
constexpr int kXsecStaticSets = 64;
constexpr size_t kXsecStaticDoubles = size_t(kXsecStaticSets) * (3 * kXsecStaticBlocks + 3) + 3 * kXsecStaticSets;
__device__ __align__(256) double scratch[kXsecStaticDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's device address on the current device (looked up once
// per device).
hipError_t static_scratch(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}
}  // namespace

extern "C" {

int rwgt_xsec_noalloc(rwgt_ctx* ctx, const double* weights_in, const double* weights_out, int64_t nevt,
                      int32_t nsets, double sigma, double dsigma, double norm, double* xsec, double* xerr,
                      int32_t* fallback) {
  if (!ctx) return RWGT_EINVAL;
  ctx->err.clear();
  if (nevt < 1 || nsets < 1 || !weights_in || !weights_out || !xsec || !xerr)
    return ctx->fail(RWGT_EINVAL, "bad arguments");
  if (nsets > kXsecStaticSets)
    return ctx->fail(RWGT_EINVAL, "nsets exceeds the static scratch of rwgt_xsec_noalloc (64 cards)");
  double* base = nullptr;
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = static_scratch(ctx->device, &base);
  if (e != hipSuccess) return ctx->hip_fail(e, "static scratch address");
  double* part = base;                                                  // nsets * (3 nblocks + 3)
  double* out = base + size_t(nsets) * (3 * kXsecStaticBlocks + 3);     // nsets * 3
  e = rwgt::launch_xsec(weights_in, weights_out, nevt, nsets, sigma, dsigma, norm, part, kXsecStaticBlocks, out,
                        ctx->stream);
  double host[3 * kXsecStaticSets];
  if (e == hipSuccess)
    e = hipMemcpyAsync(host, out, size_t(nsets) * 3 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return ctx->hip_fail(e, "cross-section reduction");
  for (int32_t k = 0; k < nsets; ++k) {
    xsec[k] = host[k * 3];
    xerr[k] = host[k * 3 + 1];
    if (fallback) fallback[k] = host[k * 3 + 2] != 0.0;
    if (host[k * 3 + 2] != 0.0)
      std::fprintf(stderr, "rwgt: error propagation for card %d gave no positive finite value; "
                           "using dsigma * max(sigma'/sigma, sigma/sigma')\n", int(k));
  }
  return RWGT_OK;
}

int rwgt_set_mixed_guard(rwgt_ctx* ctx, double kappa_max) {
  if (!ctx) return RWGT_EINVAL;
  if (!(kappa_max == kappa_max)) return ctx->fail(RWGT_EINVAL, "kappa_max is NaN");
  ctx->guard_kmax = kappa_max;
  return RWGT_OK;
}

int rwgt_mixed_guard_count(rwgt_ctx* ctx, int64_t* n_reevaluated) {
  if (!ctx || !n_reevaluated) return RWGT_EINVAL;
  *n_reevaluated = 0;
  if (!ctx->guard_ran) return RWGT_OK;
  unsigned int h = 0;
  hipError_t e = hipMemcpyAsync(&h, ctx->guard_count, sizeof(h), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return ctx->hip_fail(e, "guard count");
  *n_reevaluated = int64_t(h);
  return RWGT_OK;
}

int rwgt_cancellation(rwgt_ctx* ctx, const double* momenta, int64_t nevt, const double* param_sets, int32_t nsets,
                      double* me2_out, double* kappa_out) {
  if (!ctx) return RWGT_EINVAL;
  ctx->err.clear();
  if (ctx->precision == RWGT_FP64) return ctx->fail(RWGT_EINVAL, "the cancellation measure is of the mixed path");
  if (!kappa_out && nevt > 0) return ctx->fail(RWGT_EINVAL, "kappa_out is NULL");
  try {
    ctx->nf_blocks = 0;
    return run(ctx, false, momenta, nevt, nullptr, param_sets, nsets, nullptr, me2_out, kappa_out);
  } catch (const std::exception& ex) {
    return ctx->fail(RWGT_ENOMEM, ex.what());
  }
}

int rwgt_flops(const rwgt_ctx* ctx, double* flops_per_me2) {
  if (!ctx || !flops_per_me2) return RWGT_EINVAL;
  *flops_per_me2 = rwgt::process_flops(ctx->def->id, false);
  return RWGT_OK;
}

int rwgt_bounds_check(int32_t* enabled, uint64_t* misses) {
  if (!enabled || !misses) return RWGT_EINVAL;
  const auto& readers = rwgt::bounds_readers();
  *enabled = readers.empty() ? 0 : 1;
  uint64_t total = 0;
  for (rwgt::BoundsReader f : readers) {
    const unsigned long long v = f();
    if (v == ~0ull) return RWGT_EDEVICE;
    total += v;
  }
  *misses = total;
  return RWGT_OK;
}

int rwgt_flops_executed(const rwgt_ctx* ctx, double* flops_per_me2) {
  if (!ctx || !flops_per_me2) return RWGT_EINVAL;
  *flops_per_me2 = rwgt::process_flops(ctx->def->id, true);
  return RWGT_OK;
}

}  // extern "C"

// ------------------------------------------------------------ batched form
struct rwgt_batch {
  std::vector<rwgt_ctx*> ctxs;
  int precision = 0;
  int family = rwgt::kFamilyElectroweak;
  int device = 0;
  int ncu = 256;
  hipStream_t user_stream = nullptr;
  hipStream_t own_stream = nullptr;    // capture needs a non-null stream
  rwgt::BatchSeg* dsegs = nullptr;
  CardPair* dcards = nullptr;
  rwgt::BatchSeg* hsegs = nullptr;     // pinned staging
  CardPair* hcards = nullptr;
  int cap = 0;
  unsigned long long* counter = nullptr;
  hipEvent_t staged = nullptr, t0 = nullptr, t1 = nullptr;
  bool staged_pending = false;
  rwgt::BatchSchedule sched{256, 256, 0, 0};
  bool tuned = false;
  // captured graph and the launch shape it was captured for
  hipGraphExec_t exec = nullptr;
  int g_nseg = -1, g_tile = 0, g_block = 0, g_grid = 0, g_hel = 0;
  int64_t g_ntiles = -1;
  std::string err;

  int fail(int code, const std::string& m) { err = m; return code; }
  int hip_fail(hipError_t e, const char* what) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? RWGT_ENOMEM : RWGT_EDEVICE;
  }
  hipStream_t stream() const { return user_stream ? user_stream : own_stream; }
  ~rwgt_batch() {
    if (own_stream) hipStreamSynchronize(own_stream);
    if (user_stream) hipStreamSynchronize(user_stream);
    if (exec) hipGraphExecDestroy(exec);
    if (dsegs) hipFree(dsegs);
    if (dcards) hipFree(dcards);
    if (counter) hipFree(counter);
    if (hsegs) hipHostFree(hsegs);
    if (hcards) hipHostFree(hcards);
    for (hipEvent_t e : {staged, t0, t1})
      if (e) hipEventDestroy(e);
    if (own_stream) hipStreamDestroy(own_stream);
  }
};

namespace {

int family_index(int proc) {
  if (proc == rwgt::kProcEeMumu) return 0;
  if (proc == rwgt::kProcUuEeg) return 1;
  return -1;
}

std::string tune_cache_path() {
  if (const char* p = std::getenv("RWGT_TUNE_CACHE")) return p;
  const char* home = std::getenv("HOME");
  return std::string(home ? home : "/tmp") + "/.rwgt_autotune";
}

// Key of a tuned schedule: the target, the HIP runtime version (a new ROCm
// may schedule the same kernels differently), the family, precision, segment
// count and event count (log2).
std::string tune_key(const rwgt_batch* b, int nseg, int64_t events) {
  int lg = 0;
  while ((int64_t(1) << (lg + 1)) <= events) ++lg;
  int rt = 0;
  if (hipRuntimeGetVersion(&rt) != hipSuccess) rt = 0;
  return "gfx950 hip=" + std::to_string(rt) + " family=" + std::to_string(b->family) +
         " prec=" + std::to_string(b->precision) + " nseg=" + std::to_string(nseg) + " log2events=" + std::to_string(lg);
}

bool tune_lookup(const std::string& key, rwgt::BatchSchedule& out) {
  std::ifstream in(tune_cache_path());
  std::string line;
  while (std::getline(in, line)) {
    const auto bar = line.find('|');
    if (bar == std::string::npos || line.substr(0, bar) != key) continue;
    std::istringstream v(line.substr(bar + 1));
    rwgt::BatchSchedule s{};
    if (v >> s.tile_events >> s.block >> s.grid) {
      if (!(v >> s.hel_split)) s.hel_split = 0;               // entries written before the helicity split
      out = s;
      return true;
    }
  }
  return false;
}

void tune_store(const std::string& key, const rwgt::BatchSchedule& s) {
  std::ofstream outf(tune_cache_path(), std::ios::app);
  if (outf) outf << key << "|" << s.tile_events << " " << s.block << " " << s.grid << " " << s.hel_split << "\n";
}

int batch_stage(rwgt_batch* b, const rwgt_segment* segs, int32_t nseg, int& nlive, int64_t& ntiles,
                int64_t& events) {
  // host tables: segments with events, two cards each
  std::vector<rwgt::BatchSeg> hs;
  std::vector<CardPair> hc;
  ntiles = 0;
  events = 0;
  for (int32_t k = 0; k < nseg; ++k) {
    const rwgt_segment& s = segs[k];
    if (s.ctx < 0 || s.ctx >= int32_t(b->ctxs.size())) return b->fail(RWGT_EINVAL, "segment ctx out of range");
    if (s.nevt < 0) return b->fail(RWGT_EINVAL, "segment nevt < 0");
    if (!s.params) return b->fail(RWGT_EINVAL, "segment params is NULL");
    rwgt_ctx* c = b->ctxs[s.ctx];
    std::vector<CardPair> cards;
    int rc = build_cards(c, s.params, 1, true, cards);
    if (rc != RWGT_OK) return b->fail(rc, c->err);
    if (s.nevt == 0) continue;
    if (!s.momenta || !s.weights_in || !s.weights_out) return b->fail(RWGT_EINVAL, "segment pointer is NULL");
    rwgt::BatchSeg d{};
    d.proc = family_index(c->def->id);
    d.nevt = s.nevt;
    d.tile0 = ntiles;
    d.mom = s.momenta;
    d.w_in = s.weights_in;
    d.w_out = s.weights_out;
    hs.push_back(d);
    hc.push_back(cards[0]);
    hc.push_back(cards[1]);
    ntiles += (s.nevt + b->sched.tile_events - 1) / b->sched.tile_events;
    events += s.nevt;
  }
  nlive = int(hs.size());
  if (nlive == 0) return RWGT_OK;
  hipError_t e;
  if (nlive > b->cap) {
    if (b->staged_pending) { hipEventSynchronize(b->staged); b->staged_pending = false; }
    hipStreamSynchronize(b->stream());
    if (b->dsegs) hipFree(b->dsegs);
    if (b->dcards) hipFree(b->dcards);
    if (b->hsegs) hipHostFree(b->hsegs);
    if (b->hcards) hipHostFree(b->hcards);
    b->dsegs = nullptr; b->dcards = nullptr; b->hsegs = nullptr; b->hcards = nullptr; b->cap = 0;
    const int cap = nlive < 64 ? 64 : nlive;
    if ((e = hipMalloc(&b->dsegs, cap * sizeof(rwgt::BatchSeg))) != hipSuccess) return b->hip_fail(e, "hipMalloc");
    if ((e = hipMalloc(&b->dcards, 2 * cap * sizeof(CardPair))) != hipSuccess) return b->hip_fail(e, "hipMalloc");
    if ((e = hipHostMalloc(&b->hsegs, cap * sizeof(rwgt::BatchSeg), hipHostMallocDefault)) != hipSuccess)
      return b->hip_fail(e, "hipHostMalloc");
    if ((e = hipHostMalloc(&b->hcards, 2 * cap * sizeof(CardPair), hipHostMallocDefault)) != hipSuccess)
      return b->hip_fail(e, "hipHostMalloc");
    b->cap = cap;
    if (b->exec) { hipGraphExecDestroy(b->exec); b->exec = nullptr; b->g_nseg = -1; }
  }
  if (b->staged_pending) {
    if ((e = hipEventSynchronize(b->staged)) != hipSuccess) return b->hip_fail(e, "hipEventSynchronize");
    b->staged_pending = false;
  }
  std::memcpy(b->hsegs, hs.data(), hs.size() * sizeof(rwgt::BatchSeg));
  std::memcpy(b->hcards, hc.data(), hc.size() * sizeof(CardPair));
  hipStream_t st = b->stream();
  if ((e = hipMemcpyAsync(b->dsegs, b->hsegs, hs.size() * sizeof(rwgt::BatchSeg), hipMemcpyHostToDevice, st)) !=
      hipSuccess)
    return b->hip_fail(e, "hipMemcpyAsync(segments)");
  if ((e = hipMemcpyAsync(b->dcards, b->hcards, hc.size() * sizeof(CardPair), hipMemcpyHostToDevice, st)) !=
      hipSuccess)
    return b->hip_fail(e, "hipMemcpyAsync(cards)");
  if ((e = hipEventRecord(b->staged, st)) != hipSuccess) return b->hip_fail(e, "hipEventRecord");
  b->staged_pending = true;
  return RWGT_OK;
}

// One launch of the staged tables: replay the captured graph when the launch
// shape is unchanged, otherwise capture it again.
int batch_launch(rwgt_batch* b, int nlive, int64_t ntiles) {
  hipStream_t st = b->stream();
  hipError_t e;
  rwgt::BatchSchedule sc = b->sched;
  if (sc.grid <= 0) sc.grid = 2 * b->ncu;
  const bool same = b->exec && b->g_nseg == nlive && b->g_ntiles == ntiles && b->g_tile == sc.tile_events &&
                    b->g_block == sc.block && b->g_grid == sc.grid && b->g_hel == sc.hel_split;
  if (!same) {
    if (b->exec) { hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    hipGraph_t g = nullptr;
    if ((e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed)) != hipSuccess)
      return b->hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = rwgt::launch_batch(b->family, b->precision, b->dsegs, nlive, ntiles, sc, b->dcards, b->counter,
                                       st);
    e = hipStreamEndCapture(st, &g);
    if (le != hipSuccess) { if (g) hipGraphDestroy(g); return b->hip_fail(le, "batch kernel"); }
    if (e != hipSuccess) return b->hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) { b->exec = nullptr; return b->hip_fail(e, "hipGraphInstantiate"); }
    b->g_nseg = nlive; b->g_ntiles = ntiles; b->g_tile = sc.tile_events; b->g_block = sc.block; b->g_grid = sc.grid;
    b->g_hel = sc.hel_split;
  }
  hipEventRecord(b->t0, st);
  if ((e = hipGraphLaunch(b->exec, st)) != hipSuccess) return b->hip_fail(e, "hipGraphLaunch");
  hipEventRecord(b->t1, st);
  return RWGT_OK;
}

}  // namespace

extern "C" {

int rwgt_batch_create(rwgt_ctx* const* ctxs, int32_t nctx, rwgt_batch** out) {
  if (!out) return RWGT_EINVAL;
  *out = nullptr;
  if (!ctxs || nctx < 1) return RWGT_EINVAL;
  for (int32_t i = 0; i < nctx; ++i) {
    if (!ctxs[i]) return RWGT_EINVAL;
    if (family_index(ctxs[i]->def->id) < 0) {
      ctxs[i]->err = "the batched form covers the electroweak family (e+ e- > mu+ mu-, u u~ > e+ e- g)";
      return RWGT_EPROCESS;
    }
    if (ctxs[i]->precision != ctxs[0]->precision) return RWGT_EINVAL;
  }
  rwgt_batch* b = new (std::nothrow) rwgt_batch;
  if (!b) return RWGT_ENOMEM;
  b->ctxs.assign(ctxs, ctxs + nctx);
  b->precision = ctxs[0]->precision == RWGT_FP64 ? rwgt::kPrecFP64 : rwgt::kPrecMixedFP16;
  b->device = ctxs[0]->device;
  hipError_t e = hipSetDevice(b->device);
  hipDeviceProp_t prop;
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, b->device);
  if (e == hipSuccess) b->ncu = prop.multiProcessorCount;
  if (e == hipSuccess) e = hipStreamCreate(&b->own_stream);
  if (e == hipSuccess) e = hipMalloc(&b->counter, sizeof(unsigned long long));
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreate(&b->t0);
  if (e == hipSuccess) e = hipEventCreate(&b->t1);
  if (e != hipSuccess) { delete b; return e == hipErrorOutOfMemory ? RWGT_ENOMEM : RWGT_EDEVICE; }
  *out = b;
  return RWGT_OK;
}

void rwgt_batch_destroy(rwgt_batch* b) { delete b; }

int rwgt_batch_set_stream(rwgt_batch* b, void* stream) {
  if (!b) return RWGT_EINVAL;
  b->user_stream = static_cast<hipStream_t>(stream);
  if (b->exec) { hipGraphExecDestroy(b->exec); b->exec = nullptr; b->g_nseg = -1; }
  return RWGT_OK;
}

int rwgt_batch_set_schedule(rwgt_batch* b, int32_t tile_events, int32_t block, int32_t blocks_per_cu,
                            int32_t hel_split) {
  if (!b || tile_events < 1 || block < 64 || block > 256 || block % 64 || blocks_per_cu < 1 ||
      (hel_split != 0 && hel_split != 1))
    return RWGT_EINVAL;
  b->sched = rwgt::BatchSchedule{tile_events, block, blocks_per_cu * b->ncu, hel_split};
  b->tuned = true;
  return RWGT_OK;
}

int rwgt_batch_get_schedule(const rwgt_batch* b, int32_t* tile_events, int32_t* block, int32_t* grid,
                            int32_t* hel_split) {
  if (!b || !tile_events || !block || !grid) return RWGT_EINVAL;
  *tile_events = b->sched.tile_events;
  *block = b->sched.block;
  *grid = b->sched.grid > 0 ? b->sched.grid : 2 * b->ncu;
  if (hel_split) *hel_split = b->sched.hel_split;
  return RWGT_OK;
}

int rwgt_batch_eval(rwgt_batch* b, const rwgt_segment* segs, int32_t nseg) {
  if (!b) return RWGT_EINVAL;
  b->err.clear();
  if (nseg < 0 || (nseg > 0 && !segs)) return b->fail(RWGT_EINVAL, "bad segment list");
  if (nseg == 0) return RWGT_OK;
  try {
    hipError_t e = hipSetDevice(b->device);
    if (e != hipSuccess) return b->hip_fail(e, "hipSetDevice");
    if (!b->tuned) {
      int64_t total = 0;
      for (int32_t k = 0; k < nseg; ++k) total += segs[k].nevt > 0 ? segs[k].nevt : 0;
      rwgt::BatchSchedule s{};
      if (tune_lookup(tune_key(b, nseg, total), s)) b->sched = s;
      b->tuned = true;
    }
    int nlive = 0;
    int64_t ntiles = 0, events = 0;
    int rc = batch_stage(b, segs, nseg, nlive, ntiles, events);
    if (rc != RWGT_OK || nlive == 0) return rc;
    return batch_launch(b, nlive, ntiles);
  } catch (const std::exception& ex) {
    return b->fail(RWGT_ENOMEM, ex.what());
  }
}

int rwgt_batch_time(rwgt_batch* b, float* ms) {
  if (!b || !ms) return RWGT_EINVAL;
  hipError_t e = hipEventSynchronize(b->t1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, b->t0, b->t1);
  if (e != hipSuccess) return b->hip_fail(e, "batch timing");
  return RWGT_OK;
}

// Grid search over (tile events, workgroup size, workgroups per CU, helicity
// split) on the given segments, timing each candidate with HIP events; the
// fastest is kept and appended to the tuning cache (RWGT_TUNE_CACHE, default
// ~/.rwgt_autotune).
int rwgt_batch_tune(rwgt_batch* b, const rwgt_segment* segs, int32_t nseg, int32_t reps) {
  if (!b || !segs || nseg < 1) return RWGT_EINVAL;
  if (reps < 1) reps = 2;
  static const int tiles[] = {64, 128, 256, 512, 1024, 2048};
  static const int blocks[] = {64, 128, 256};
  static const int per_cu[] = {1, 2, 4, 8};
  float best = 1e30f;
  rwgt::BatchSchedule best_s = b->sched;
  int64_t total = 0;
  for (int32_t k = 0; k < nseg; ++k) total += segs[k].nevt > 0 ? segs[k].nevt : 0;
  for (int hs = 0; hs <= 1; ++hs)
    for (int t : tiles)
      for (int bl : blocks)
        for (int pc : per_cu) {
          if (!hs && bl > t) continue;             // more lanes than the tile's events
          b->sched = rwgt::BatchSchedule{t, bl, pc * b->ncu, hs};
          b->tuned = true;
          float acc = 0.0f;
          for (int r = 0; r <= reps; ++r) {
            int rc = rwgt_batch_eval(b, segs, nseg);
            if (rc != RWGT_OK) return rc;
            float ms = 0.0f;
            rc = rwgt_batch_time(b, &ms);
            if (rc != RWGT_OK) return rc;
            if (r > 0) acc += ms;   // the first run captures the graph
          }
          if (acc / reps < best) { best = acc / reps; best_s = b->sched; }
        }
  b->sched = best_s;
  b->tuned = true;
  tune_store(tune_key(b, nseg, total), best_s);
  return RWGT_OK;
}

const char* rwgt_batch_last_error(const rwgt_batch* b) { return b ? b->err.c_str() : "batch is NULL"; }

// Device tables of the card-per-event paths: cards[0] = original, cards[1 + k]
// = param_table row k; the network's card inputs (M_Z, Gamma_Z,
// sin^2 theta_W) per row; the gate list and count for up to rows events, and
// (need_x) the input rows of a layered network.
static int per_event_tables(rwgt_ctx* c, const rwgt_mlp* m, const double* param_table, int32_t ncards, int64_t rows,
                            bool need_x) {
  constexpr int kNparam = rwgt::kMlpCardParams;
  // the same table as last time and room for the rows: nothing to rebuild
  const size_t nval = size_t(ncards) * c->def->layout.size();
  if (rows <= c->sur_cap && (!need_x || c->sur_x) && c->sur_cards && c->sur_table.size() == nval &&
      std::memcmp(c->sur_table.data(), param_table, nval * sizeof(double)) == 0)
    return RWGT_OK;
  c->sur_table.clear();
  std::vector<CardPair> cards;
  int rc = build_cards(c, param_table, ncards, true, cards);
  if (rc != RWGT_OK) return rc;
  const auto& layout = c->def->layout;
  auto col = [&](const char* name) {
    for (size_t j = 0; j < layout.size(); ++j)
      if (layout[j] == name) return int(j);
    return -1;
  };
  const int jm = col("MASS 23"), jw = col("DECAY 23"), js = col("RWGTEW 1");
  std::vector<float> cpar(size_t(ncards) * kNparam);
  for (int k = 0; k < ncards; ++k) {
    const double* row = param_table + size_t(k) * layout.size();
    cpar[k * kNparam + 0] = float(row[jm]);
    cpar[k * kNparam + 1] = float(row[jw]);
    cpar[k * kNparam + 2] = float(row[js]);
  }
  hipError_t e = hipSetDevice(c->device);
  hipStream_t st = c->stream;
  if (e == hipSuccess && (rows > c->sur_cap || ncards + 1 > c->sur_card_cap || (need_x && !c->sur_x))) {
    e = hipStreamSynchronize(st);
    for (void* p : {c->sur_x, static_cast<void*>(c->sur_list), static_cast<void*>(c->sur_count),
                    static_cast<void*>(c->sur_heads), static_cast<void*>(c->sur_cards), static_cast<void*>(c->sur_cpar)})
      if (p) (void)hipFree(p);
    c->sur_x = nullptr; c->sur_list = nullptr; c->sur_count = nullptr; c->sur_heads = nullptr;
    c->sur_cards = nullptr; c->sur_cpar = nullptr; c->sur_cap = 0; c->sur_card_cap = 0;
    const int64_t cap = std::max<int64_t>(rows, 64);
    const int cc = std::max(ncards + 1, 64);
    int64_t xbytes = 0;
    if (need_x) rwgt_mlp_input_bytes(m, cap, &xbytes);
    if (e == hipSuccess && need_x) e = hipMalloc(&c->sur_x, size_t(xbytes));
    if (e == hipSuccess) e = hipMalloc(&c->sur_list, size_t(cap) * 4);
    if (e == hipSuccess) e = hipMalloc(&c->sur_count, 4);
    if (e == hipSuccess) e = hipMalloc(&c->sur_cards, size_t(cc) * sizeof(CardPair));
    if (e == hipSuccess) e = hipMalloc(&c->sur_cpar, size_t(cc) * kNparam * 4);
    if (e == hipSuccess) { c->sur_cap = cap; c->sur_card_cap = cc; }
  }
  if (e != hipSuccess) return c->hip_fail(e, "per-event workspace");
  // small tables: synchronous copies (pageable host memory)
  e = hipMemcpyAsync(c->sur_cards, cards.data(), cards.size() * sizeof(CardPair), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(c->sur_cpar, cpar.data(), cpar.size() * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return c->hip_fail(e, "per-event tables");
  c->sur_table.assign(param_table, param_table + nval);
  return RWGT_OK;
}

static int compute_units(int device) {
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || ncu < 1) ncu = 256;
  return ncu;
}

int rwgt_eval_cards(rwgt_ctx* c, const double* momenta, int64_t nevt, const double* w_in, const double* param_table,
                    int32_t ncards, const int32_t* card_index, double* w_out) {
  if (!c) return RWGT_EINVAL;
  c->err.clear();
  if (nevt < 0 || ncards < 1 || !param_table) return c->fail(RWGT_EINVAL, "bad sizes or NULL param_table");
  const int proc = family_index(c->def->id);
  if (proc < 0) return c->fail(RWGT_EPROCESS, "the card-per-event path covers the electroweak family");
  if (nevt == 0) return RWGT_OK;
  if (!momenta || !w_in || !w_out || !card_index) return c->fail(RWGT_EINVAL, "NULL device pointer");
  try {
    int rc = per_event_tables(c, nullptr, param_table, ncards, 0, false);
    if (rc != RWGT_OK) return rc;
    hipError_t e = rwgt::launch_exact_list(rwgt::kFamilyElectroweak,
                                           c->precision == RWGT_FP64 ? rwgt::kPrecFP64 : rwgt::kPrecMixedFP16, proc,
                                           momenta, nullptr, nullptr, nevt, card_index, ncards, c->sur_cards, w_in,
                                           w_out, 16 * compute_units(c->device), c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "card-per-event evaluation");
    return count_nonfinite(c, w_out, nevt);
  } catch (const std::exception& ex) {
    return c->fail(RWGT_ENOMEM, ex.what());
  }
}

int rwgt_sur_eval(rwgt_ctx* c, rwgt_mlp* m, const double* momenta, int64_t nevt, const double* w_in,
                  const double* param_table, int32_t ncards, const int32_t* card_index, double threshold,
                  double* w_out, int64_t* n_fallback) {
  if (!c || !m) return RWGT_EINVAL;
  c->err.clear();
  if (n_fallback) *n_fallback = 0;
  if (nevt < 0 || ncards < 1 || !param_table) return c->fail(RWGT_EINVAL, "bad sizes or NULL param_table");
  const int proc = family_index(c->def->id);
  if (proc < 0) return c->fail(RWGT_EPROCESS, "the surrogate path covers the electroweak family");
  const int npart = c->def->npart;
  if (m->fm.npart != 0 ? m->fm.npart != npart : m->n_in != rwgt::feature_count(rwgt::kFeatRaw, npart))
    return c->fail(RWGT_EINVAL, "the network's feature map does not fit this process");
  if (nevt == 0) return RWGT_OK;
  if (!momenta || !w_in || !w_out || !card_index) return c->fail(RWGT_EINVAL, "NULL device pointer");
  try {
    const int64_t rows = (nevt + 63) / 64 * 64;
    int rc = per_event_tables(c, m, param_table, ncards, rows, !m->fused());
    if (rc != RWGT_OK) return rc;
    hipStream_t st = c->stream;
    hipError_t e = hipSuccess;
    rwgt_mlp_set_stream(m, st);
    // card indices outside [0, ncards) give NaN features, so the gate sends
    // those events to the exact path, which writes NaN for them
    const rwgt::FeatureMap fm_network = m->fm;
    if (m->fm.npart == 0) {                                   // the raw map of this process
      m->fm.kind = rwgt::kFeatRaw;
      m->fm.npart = npart;
    }
    rwgt::FeatureMap fm = m->fm;
    fm.ncards = ncards;
    if (m->fused()) {
      // one pass: features, layers, heads, gate (w' or an entry in the list)
      m->fm = fm;
      rc = m->infer(momenta, nullptr, card_index, c->sur_cpar, nevt, nullptr, w_in, w_out, c->sur_list, c->sur_count,
                    float(threshold));
      m->fm = fm_network;
      if (rc != RWGT_OK) return c->fail(rc, m->err);
    } else {
      m->fm = fm_network;
      e = rwgt::mlp_features(fm, momenta, nullptr, card_index, c->sur_cpar, m->mean, m->istd,
                             static_cast<float*>(c->sur_x), nevt, rows, m->layers[0].in, st);
      if (e != hipSuccess) return c->hip_fail(e, "surrogate features");
      rc = rwgt_mlp_forward(m, c->sur_x, nevt, nullptr);
      if (rc != RWGT_OK) return c->fail(rc, m->err);
      e = rwgt::mlp_gate(m->z.back(), 32, nevt, m->ym, m->ys, m->k_cal, float(threshold), w_in, w_out, c->sur_list,
                         c->sur_count, st);
    }
    if (e == hipSuccess)
      e = rwgt::launch_exact_list(rwgt::kFamilyElectroweak,
                                  c->precision == RWGT_FP64 ? rwgt::kPrecFP64 : rwgt::kPrecMixedFP16, proc, momenta,
                                  c->sur_list, c->sur_count, nevt, card_index, ncards, c->sur_cards, w_in, w_out,
                                  16 * compute_units(c->device), st);
    if (e != hipSuccess) return c->hip_fail(e, "surrogate gate / exact fallback");
    rc = count_nonfinite(c, w_out, nevt);
    if (rc != RWGT_OK) return rc;
    if (n_fallback) {
      unsigned int cnt = 0;
      e = hipMemcpyAsync(&cnt, c->sur_count, 4, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return c->hip_fail(e, "fallback count");
      *n_fallback = cnt;
    }
    return RWGT_OK;
  } catch (const std::exception& ex) {
    return c->fail(RWGT_ENOMEM, ex.what());
  }
}

}  // extern "C"
