// Exercises the host-side code of the whole library under the sanitizers, on
// a machine without a GPU: the process and SLHA-card parsers behind
// rwgt_create (which then fails cleanly with RWGT_EDEVICE where it needs the
// device), the reweighting-card parser (valid cards and damaged copies),
// rwgt_process_layout, the training order, and the checkpoint reader on
// damaged files.  Exit status 0 when every check holds; the sanitizers abort
// on any memory error or undefined behaviour.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <string>
#include <vector>

#include "../../include/rwgt.h"

static int fails = 0;
#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++fails;                                                            \
    }                                                                     \
  } while (0)

static const char* kProcesses[] = {"e+ e- > mu+ mu-", "u u~ > e+ e- g", "g g > t t~ g g"};

static const char* kCard =
    "BLOCK SMINPUTS\n  1 1.325070e+02 # 1/alpha\n  3 1.180000e-01 # alpha_s\n"
    "BLOCK RWGTEW\n  1 2.222000e-01\nBLOCK MASS\n  6 1.730000e+02\n 23 9.118800e+01\n"
    "DECAY 23 2.441000e+00\nDECAY 6 0.0\n";

static const char* kRwgtCard =
    "# reweighting card\nchange backend hip\nchange fptype m\n"
    "launch --rwgt_name=mz_up\nset MASS 23 91.5\nset decay 23 2.6\n"
    "launch rwgt_name=alpha_s\nset SMINPUTS 3 0.130\nset MASS 6 180.0\n"
    "launch\nset RWGTEW 1 0.2312\n";

int main() {
  // process layouts
  for (const char* p : kProcesses) {
    int32_t npar = 0;
    const char* names[16] = {};
    CHECK(rwgt_process_layout(p, &npar, names) == RWGT_OK && npar > 0 && npar <= 16);
    for (int32_t k = 0; k < npar; ++k) CHECK(names[k] && std::strlen(names[k]) > 0);
  }
  int32_t npar = 0;
  CHECK(rwgt_process_layout("d d~ > e+ e-", &npar, nullptr) == RWGT_EPROCESS);
  // rwgt_create: argument and card errors before any device work; a valid
  // card reaches the device and fails there without a GPU
  rwgt_ctx* ctx = nullptr;
  CHECK(rwgt_create(nullptr, kCard, RWGT_FP64, &ctx) == RWGT_EINVAL && !ctx);
  CHECK(rwgt_create("g g > t t~", kCard, RWGT_FP64, &ctx) == RWGT_EPROCESS && !ctx);
  CHECK(rwgt_create("g g > t t~ g g", "BLOCK MASS\n 6 173\n", RWGT_FP64, &ctx) == RWGT_ECARD && !ctx);
  CHECK(rwgt_create("e+ e- > mu+ mu-", "BLOCK SMINPUTS\n 1 x\n", RWGT_FP64, &ctx) == RWGT_ECARD && !ctx);
  for (const char* p : kProcesses) {
    const int rc = rwgt_create(p, kCard, RWGT_MIXED_FP16, &ctx);
    CHECK((rc == RWGT_OK) == (ctx != nullptr));
    rwgt_destroy(ctx);
    ctx = nullptr;
  }
  // the SLHA parser on every truncation and on overwritten bytes of a valid card
  const std::string card(kCard);
  for (size_t cut = 0; cut <= card.size(); ++cut) {
    const std::string t = card.substr(0, cut);
    if (rwgt_create("g g > t t~ g g", t.c_str(), RWGT_FP64, &ctx) == RWGT_OK) rwgt_destroy(ctx);
    ctx = nullptr;
  }
  for (size_t pos = 0; pos < card.size(); ++pos) {
    std::string t = card;
    t[pos] = "x<#\n.-e9"[pos % 8];
    if (rwgt_create("u u~ > e+ e- g", t.c_str(), RWGT_FP64, &ctx) == RWGT_OK) rwgt_destroy(ctx);
    ctx = nullptr;
  }
  // reweighting cards: the valid one, then damaged copies
  double sets[16 * 8];
  char names[16 * 32];
  char fptype[2] = {0, 0};
  int32_t nsets = 0;
  for (const char* p : kProcesses) {
    CHECK(rwgt_reweight_card(p, kCard, kRwgtCard, 16, sets, &nsets, names, 32, fptype) == RWGT_OK && nsets == 3);
    CHECK(fptype[0] == 'm');
  }
  const std::string rc(kRwgtCard);
  int accepted = 0, rejected = 0;
  for (size_t cut = 0; cut <= rc.size(); ++cut) {
    const std::string t = rc.substr(0, cut);
    (rwgt_reweight_card(kProcesses[1], kCard, t.c_str(), 2, sets, &nsets, names, 8, fptype) == RWGT_OK ? accepted
                                                                                                      : rejected)++;
  }
  for (size_t pos = 0; pos < rc.size(); ++pos) {
    std::string t = rc;
    t[pos] = "x \n=#9"[pos % 6];
    rwgt_reweight_card(kProcesses[2], kCard, t.c_str(), 16, sets, &nsets, nullptr, 0, nullptr);
  }
  CHECK(accepted > 0 && rejected > 0);
  // training order: a bijection for a few sizes
  for (int64_t n : {1, 5, 1000, 65537}) {
    std::vector<int64_t> o(static_cast<size_t>(n));
    CHECK(rwgt_train_order(42, 3, n, 0, n, o.data()) == RWGT_OK);
    std::vector<char> seen(static_cast<size_t>(n), 0);
    for (int64_t v : o) {
      CHECK(v >= 0 && v < n);
      if (v >= 0 && v < n) seen[static_cast<size_t>(v)]++;
    }
    for (char s : seen) CHECK(s == 1);
  }
  CHECK(rwgt_train_order(1, 0, 10, 5, 6, nullptr) == RWGT_EINVAL);
  // the checkpoint reader on damaged files
  const char* path = "/tmp/rwgt_sanitize.ckpt";
  int32_t shape[5];
  int64_t ep = 0, steps = 0;
  for (int variant = 0; variant < 4; ++variant) {
    std::ofstream f(path, std::ios::binary);
    std::string body = "RWGTMLP";
    body.push_back('\0');
    if (variant == 1) body += std::string(7, 'x');
    if (variant == 2) body += std::string(300, '\0');
    if (variant == 3) body = "not a checkpoint";
    f.write(body.data(), static_cast<std::streamsize>(body.size()));
    f.close();
    CHECK(rwgt_mlp_checkpoint_info(path, shape, &ep, &steps) != RWGT_OK);
    CHECK(std::strlen(rwgt_mlp_checkpoint_error()) > 0);
  }
  CHECK(rwgt_mlp_checkpoint_info("/nonexistent/dir/x.ckpt", shape, &ep, &steps) == RWGT_EINVAL);
  std::remove(path);
  std::printf("reweighting-card truncations accepted %d rejected %d, failures %d\n", accepted, rejected, fails);
  return fails == 0 ? 0 : 1;
}
