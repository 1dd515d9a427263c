// Exercises the library's host-side event-file code (rwgt_lhe_* of
// include/rwgt.h) for the sanitizer builds: reads a file given on the command
// line (the threaded parse), sorts it into each supported process, exports
// momenta and event info, appends weights, writes and re-reads the result,
// and feeds the in-memory parser damaged copies (truncated at many points,
// bytes overwritten), which must fail with an error code, never crash.
// Exit status 0 when every check holds; the sanitizers abort on any fault.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
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
static const int kNpart[] = {4, 5, 6};

static int64_t exercise(rwgt_lhe* lhe, const char* out_path) {
  int64_t n = 0;
  CHECK(rwgt_lhe_num_events(lhe, &n) == RWGT_OK && n > 0);
  int64_t matched = 0;
  for (int p = 0; p < 3; ++p) {
    int64_t count = 0;
    CHECK(rwgt_lhe_select(lhe, kProcesses[p], nullptr, 0, &count) == RWGT_OK);
    std::vector<int64_t> idx(static_cast<size_t>(count));
    int64_t again = 0;
    CHECK(rwgt_lhe_select(lhe, kProcesses[p], idx.data(), count, &again) == RWGT_OK && again == count);
    matched += count;
    if (count == 0) continue;
    std::vector<double> mom(static_cast<size_t>(count) * kNpart[p] * 4), w(static_cast<size_t>(count));
    std::vector<double> info(static_cast<size_t>(count) * 4);
    CHECK(rwgt_lhe_momenta(lhe, kProcesses[p], idx.data(), count, mom.data(), w.data()) == RWGT_OK);
    CHECK(rwgt_lhe_info(lhe, idx.data(), count, info.data()) == RWGT_OK);
    for (int64_t i = 0; i < count; ++i) CHECK(w[static_cast<size_t>(i)] == info[static_cast<size_t>(i) * 4]);
    std::vector<double> nw(w);
    for (double& x : nw) x *= 1.5;
    const std::string id = std::string("san_") + std::to_string(p);
    CHECK(rwgt_lhe_add_weights(lhe, id.c_str(), "sanitizer pass", idx.data(), count, nw.data()) == RWGT_OK);
    // an event outside the process is refused
    if (count < n) {
      int64_t other = -1;
      for (int64_t e = 0; e < n && other < 0; ++e) {
        bool in = false;
        for (int64_t j : idx) in = in || j == e;
        if (!in) other = e;
      }
      CHECK(rwgt_lhe_momenta(lhe, kProcesses[p], &other, 1, mom.data(), nullptr) != RWGT_OK);
    }
  }
  CHECK(rwgt_lhe_select(lhe, "d d~ > x y", nullptr, 0, &matched) != RWGT_OK);
  CHECK(rwgt_lhe_write(lhe, out_path) == RWGT_OK);
  return n;
}

int main(int argc, char** argv) {
  if (argc < 3) {
    std::fprintf(stderr, "usage: %s in.lhe out.lhe\n", argv[0]);
    return 2;
  }
  rwgt_lhe* lhe = nullptr;
  CHECK(rwgt_lhe_read(argv[1], &lhe) == RWGT_OK && lhe);
  if (!lhe) return 1;
  const int64_t n = exercise(lhe, argv[2]);
  rwgt_lhe_destroy(lhe);
  // the written file reads back with the same events and the new weights
  rwgt_lhe* back = nullptr;
  CHECK(rwgt_lhe_read(argv[2], &back) == RWGT_OK && back);
  if (back) {
    int64_t m = 0;
    CHECK(rwgt_lhe_num_events(back, &m) == RWGT_OK && m == n);
    const std::string out2 = std::string(argv[2]) + ".2";
    exercise(back, out2.c_str());
    rwgt_lhe_destroy(back);
  }
  // damaged copies of the input through the in-memory parser
  std::ifstream f(argv[1], std::ios::binary);
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  int rejected = 0, accepted = 0;
  for (size_t cut = 1; cut < text.size(); cut += text.size() / 97 + 1) {
    rwgt_lhe* t = nullptr;
    const int rc = rwgt_lhe_parse(text.data(), static_cast<int64_t>(cut), &t);
    (rc == RWGT_OK ? accepted : rejected)++;
    if (t) {
      int64_t k = 0;
      rwgt_lhe_num_events(t, &k);
      rwgt_lhe_select(t, kProcesses[2], nullptr, 0, &k);
      rwgt_lhe_destroy(t);
    }
  }
  std::string bad = text;
  for (size_t pos = 200; pos < bad.size(); pos += bad.size() / 53 + 1) {
    std::string b2 = bad;
    b2[pos] = (pos % 3 == 0) ? 'x' : (pos % 3 == 1 ? '<' : '\n');
    rwgt_lhe* t = nullptr;
    if (rwgt_lhe_parse(b2.data(), static_cast<int64_t>(b2.size()), &t) == RWGT_OK && t) {
      int64_t k = 0;
      for (const char* pr : kProcesses) rwgt_lhe_select(t, pr, nullptr, 0, &k);
      rwgt_lhe_destroy(t);
    }
  }
  CHECK(rejected > 0);
  CHECK(rwgt_lhe_parse(nullptr, 10, &lhe) != RWGT_OK);
  std::printf("events %lld, truncations rejected %d accepted %d, failures %d\n", static_cast<long long>(n), rejected,
              accepted, fails);
  return fails == 0 ? 0 : 1;
}
