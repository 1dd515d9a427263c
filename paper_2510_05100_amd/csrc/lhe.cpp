// Les Houches event files (LHE v3) on the host: the reader, the sort of
// mixed-process events into one process's particle order, and the writer
// that appends reweighting weights (rwgt_lhe_* in include/rwgt.h).
//
// The file is kept in memory as read; events are located in one pass and
// parsed in parallel threads (contiguous event ranges, merged in order).
// Writing copies every byte of the input except where weights are added:
// a <weightgroup> in the header's <initrwgt> (created if absent) and one
// <wgt> per new weight in each event's <rwgt> block (created if absent).
// This follows the Rex section of the paper: events stored object-wise,
// sorted into processes by their external partons, transposed into
// contiguous per-process arrays, and written back with the new weights
// listed in <initrwgt>.
#include <algorithm>
#include <charconv>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "../../include/rwgt.h"

namespace {

struct Particle {
  int id = 0, status = 0, moth1 = 0, moth2 = 0, col1 = 0, col2 = 0;
  double p[5] = {0, 0, 0, 0, 0};          // px, py, pz, E, m as in the file
  double vtim = 0.0, spin = 0.0;
};

struct Event {
  size_t begin = 0, end = 0;              // text of "<event ...>" .. "</event>" (end: at "</event>")
  size_t tail = 0;                        // first byte after the particle lines
  int nup = 0, idprup = 0;
  double xwgt = 0.0, scale = 0.0, aqed = 0.0, aqcd = 0.0;
  size_t first = 0;                       // index of its first particle
};

struct Weight {
  std::string id, description;
  std::vector<double> value;              // per event (0 where not set)
};

// Skip blanks (not newlines when stop_at_eol).
inline const char* skip_ws(const char* p, const char* end, bool stop_at_eol = false) {
  while (p < end && (*p == ' ' || *p == '\t' || *p == '\r' || (!stop_at_eol && *p == '\n'))) ++p;
  return p;
}

// One number token; accepts a leading '+' and Fortran 'D' exponents.
bool read_double(const char*& p, const char* end, double& v) {
  p = skip_ws(p, end, true);
  const char* q = p;
  while (q < end && *q != ' ' && *q != '\t' && *q != '\n' && *q != '\r') ++q;
  if (q == p) return false;
  const char* s = p;
  if (*s == '+') ++s;
  if (std::memchr(s, 'D', q - s) || std::memchr(s, 'd', q - s)) {
    std::string t(s, q);
    for (auto& c : t)
      if (c == 'D' || c == 'd') c = 'e';
    auto r = std::from_chars(t.data(), t.data() + t.size(), v);
    if (r.ec != std::errc() || r.ptr != t.data() + t.size()) return false;
  } else {
    auto r = std::from_chars(s, q, v);
    if (r.ec != std::errc() || r.ptr != q) return false;
  }
  p = q;
  return true;
}

bool read_int(const char*& p, const char* end, int& v) {
  p = skip_ws(p, end, true);
  const char* s = p;
  if (s < end && *s == '+') ++s;
  auto r = std::from_chars(s, end, v);
  if (r.ec != std::errc()) return false;
  p = r.ptr;
  return p == end || *p == ' ' || *p == '\t' || *p == '\n' || *p == '\r';
}

const char* next_line(const char* p, const char* end) {
  while (p < end && *p != '\n') ++p;
  return p < end ? p + 1 : end;
}

// PDG code of a particle name in a process string.
bool pdg_of(const std::string& name, int& code) {
  static const std::map<std::string, int> table = {
      {"d", 1},    {"u", 2},     {"s", 3},     {"c", 4},     {"b", 5},     {"t", 6},     {"d~", -1},
      {"u~", -2},  {"s~", -3},   {"c~", -4},   {"b~", -5},   {"t~", -6},   {"e-", 11},   {"e+", -11},
      {"ve", 12},  {"ve~", -12}, {"mu-", 13},  {"mu+", -13}, {"vm", 14},   {"vm~", -14}, {"ta-", 15},
      {"ta+", -15}, {"vt", 16},  {"vt~", -16}, {"g", 21},    {"a", 22},    {"z", 23},    {"w+", 24},
      {"w-", -24}, {"h", 25}};
  auto it = table.find(name);
  if (it == table.end()) return false;
  code = it->second;
  return true;
}

}  // namespace

struct rwgt_lhe {
  std::string text;
  size_t init_begin = 0;                  // "<init"
  size_t events_end = 0;                  // just after the last "</event>"
  std::vector<Event> events;
  std::vector<Particle> parts;
  std::vector<Weight> weights;
  std::string err;

  int fail(int code, const std::string& m) { err = m; return code; }
  int parse();
  int parse_event(Event& ev, std::vector<Particle>& out, std::string& why) const;
  int process_slots(const char* process, std::vector<std::pair<int, int>>& slots);
  bool match(const Event& ev, const std::vector<std::pair<int, int>>& slots, int* map) const;
};

int rwgt_lhe::parse_event(Event& ev, std::vector<Particle>& out, std::string& why) const {
  const char* base = text.data();
  const char* p = base + ev.begin;
  const char* end = base + ev.end;
  p = next_line(p, end);                  // past the "<event ...>" line
  // skip blank lines and comments before the event line
  while (p < end) {
    const char* q = skip_ws(p, end);
    if (q < end && *q == '#') { p = next_line(q, end); continue; }
    p = q;
    break;
  }
  if (!read_int(p, end, ev.nup) || !read_int(p, end, ev.idprup) || !read_double(p, end, ev.xwgt) ||
      !read_double(p, end, ev.scale) || !read_double(p, end, ev.aqed) || !read_double(p, end, ev.aqcd)) {
    why = "malformed event line";
    return RWGT_ECARD;
  }
  if (ev.nup < 1 || ev.nup > 1000) { why = "bad particle count"; return RWGT_ECARD; }
  p = next_line(p, end);
  ev.first = out.size();
  for (int k = 0; k < ev.nup; ++k) {
    Particle q;
    if (!read_int(p, end, q.id) || !read_int(p, end, q.status) || !read_int(p, end, q.moth1) ||
        !read_int(p, end, q.moth2) || !read_int(p, end, q.col1) || !read_int(p, end, q.col2)) {
      why = "malformed particle line " + std::to_string(k + 1);
      return RWGT_ECARD;
    }
    for (double& x : q.p)
      if (!read_double(p, end, x)) { why = "malformed momentum on particle line " + std::to_string(k + 1); return RWGT_ECARD; }
    if (!read_double(p, end, q.vtim) || !read_double(p, end, q.spin)) {
      why = "malformed particle line " + std::to_string(k + 1);
      return RWGT_ECARD;
    }
    out.push_back(q);
    p = next_line(p, end);
  }
  ev.tail = size_t(p - base);
  return RWGT_OK;
}

// Position of the opening tag "<name>" or "<name ...>" (not "<name...>" of a
// longer tag name such as <initrwgt>) at or after from.
static size_t find_tag(const std::string& t, const char* name, size_t from) {
  const size_t len = std::strlen(name);
  for (size_t p = t.find(name, from); p != std::string::npos; p = t.find(name, p + len)) {
    const char c = p + len < t.size() ? t[p + len] : '\0';
    if (c == '>' || c == ' ' || c == '\t' || c == '\n' || c == '\r') return p;
  }
  return std::string::npos;
}

int rwgt_lhe::parse() {
  const size_t ib = find_tag(text, "<init", 0);
  if (ib == std::string::npos) return fail(RWGT_ECARD, "no <init> block");
  init_begin = ib;
  // pass 1: event boundaries
  size_t pos = text.find("</init>", ib);
  if (pos == std::string::npos) return fail(RWGT_ECARD, "unterminated <init> block");
  events_end = pos + 7;
  for (;;) {
    const size_t b = find_tag(text, "<event", pos);       // not <eventgroup>
    if (b == std::string::npos) break;
    const size_t e = text.find("</event>", b);
    if (e == std::string::npos) return fail(RWGT_ECARD, "unterminated <event> at byte " + std::to_string(b));
    Event ev;
    ev.begin = b;
    ev.end = e;
    events.push_back(ev);
    pos = e + 8;
    events_end = pos;
  }
  // pass 2: parse event ranges in parallel, merge in order
  const size_t n = events.size();
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 4096) nt = 1;
  std::vector<std::vector<Particle>> chunk(nt);
  std::vector<int> rc(nt, RWGT_OK);
  std::vector<std::string> why(nt);
  std::vector<size_t> bad(nt, 0);
  auto work = [&](unsigned t) {
    const size_t a = n * t / nt, b = n * (t + 1) / nt;
    for (size_t i = a; i < b; ++i) {
      const int r = parse_event(events[i], chunk[t], why[t]);
      if (r != RWGT_OK) { rc[t] = r; bad[t] = i; return; }
    }
  };
  std::vector<std::thread> pool;
  for (unsigned t = 1; t < nt; ++t) pool.emplace_back(work, t);
  work(0);
  for (auto& th : pool) th.join();
  for (unsigned t = 0; t < nt; ++t)
    if (rc[t] != RWGT_OK) return fail(rc[t], "event " + std::to_string(bad[t]) + ": " + why[t]);
  size_t total = 0;
  for (auto& c : chunk) total += c.size();
  parts.reserve(total);
  size_t off = 0;
  for (unsigned t = 0; t < nt; ++t) {
    const size_t a = n * t / nt, b = n * (t + 1) / nt;
    for (size_t i = a; i < b; ++i) events[i].first += off;
    off += chunk[t].size();
    parts.insert(parts.end(), chunk[t].begin(), chunk[t].end());
  }
  return RWGT_OK;
}

// Process string -> (status, pdg) per slot in process order: incoming -1, outgoing +1.
int rwgt_lhe::process_slots(const char* process, std::vector<std::pair<int, int>>& slots) {
  slots.clear();
  if (!process) return fail(RWGT_EINVAL, "process is NULL");
  std::istringstream in(process);
  std::string tok;
  int status = -1;
  while (in >> tok) {
    if (tok == ">") {
      if (status == 1) return fail(RWGT_EPROCESS, "two '>' in the process string");
      status = 1;
      continue;
    }
    int code = 0;
    if (!pdg_of(tok, code)) return fail(RWGT_EPROCESS, "unknown particle '" + tok + "'");
    slots.push_back({status, code});
  }
  if (status != 1 || slots.empty()) return fail(RWGT_EPROCESS, "process string needs 'a b > c ...'");
  return RWGT_OK;
}

// Slot s takes the first unused external particle (file order) with the
// slot's status and PDG code; map[s] = particle index within the event.
bool rwgt_lhe::match(const Event& ev, const std::vector<std::pair<int, int>>& slots, int* map) const {
  int next = 0;
  for (int k = 0; k < ev.nup; ++k) {
    const int st = parts[ev.first + k].status;
    if (st == -1 || st == 1) ++next;
  }
  if (next != int(slots.size())) return false;
  std::vector<char> used(size_t(ev.nup), 0);
  for (size_t s = 0; s < slots.size(); ++s) {
    int found = -1;
    for (int k = 0; k < ev.nup && found < 0; ++k) {
      const Particle& q = parts[ev.first + k];
      if (!used[size_t(k)] && q.status == slots[s].first && q.id == slots[s].second) found = k;
    }
    if (found < 0) return false;
    used[size_t(found)] = 1;
    map[s] = found;
  }
  return true;
}

namespace {
thread_local std::string g_read_error;

int finish_read(rwgt_lhe* l, rwgt_lhe** out) {
  const int rc = l->parse();
  if (rc != RWGT_OK) {
    g_read_error = l->err;
    delete l;
    return rc;
  }
  *out = l;
  return RWGT_OK;
}

void fmt_double(std::string& s, double v) {
  char buf[40];
  std::snprintf(buf, sizeof buf, "%.17g", v);
  s += buf;
}
}  // namespace

extern "C" {

int rwgt_lhe_read(const char* path, rwgt_lhe** out) {
  g_read_error.clear();
  if (!path || !out) { g_read_error = "NULL argument"; return RWGT_EINVAL; }
  *out = nullptr;
  std::ifstream f(path, std::ios::binary);
  if (!f) { g_read_error = std::string("cannot open ") + path; return RWGT_EINVAL; }
  rwgt_lhe* l = new (std::nothrow) rwgt_lhe;
  if (!l) return RWGT_ENOMEM;
  try {
    std::ostringstream ss;
    ss << f.rdbuf();
    l->text = ss.str();
    return finish_read(l, out);
  } catch (const std::exception& ex) {
    g_read_error = ex.what();
    delete l;
    return RWGT_ENOMEM;
  }
}

int rwgt_lhe_parse(const char* text, int64_t len, rwgt_lhe** out) {
  g_read_error.clear();
  if (!text || !out || len < 0) { g_read_error = "NULL argument or negative length"; return RWGT_EINVAL; }
  *out = nullptr;
  rwgt_lhe* l = new (std::nothrow) rwgt_lhe;
  if (!l) return RWGT_ENOMEM;
  try {
    l->text.assign(text, size_t(len));
    return finish_read(l, out);
  } catch (const std::exception& ex) {
    g_read_error = ex.what();
    delete l;
    return RWGT_ENOMEM;
  }
}

const char* rwgt_lhe_read_error(void) { return g_read_error.c_str(); }

void rwgt_lhe_destroy(rwgt_lhe* l) { delete l; }

const char* rwgt_lhe_last_error(const rwgt_lhe* l) { return l ? l->err.c_str() : "lhe is NULL"; }

int rwgt_lhe_num_events(const rwgt_lhe* l, int64_t* n) {
  if (!l || !n) return RWGT_EINVAL;
  *n = int64_t(l->events.size());
  return RWGT_OK;
}

int rwgt_lhe_event_info(const rwgt_lhe* l, int64_t i, int32_t* nup, int32_t* idprup, double* info) {
  if (!l || i < 0 || i >= int64_t(l->events.size())) return RWGT_EINVAL;
  const Event& ev = l->events[size_t(i)];
  if (nup) *nup = ev.nup;
  if (idprup) *idprup = ev.idprup;
  if (info) {
    info[0] = ev.xwgt;
    info[1] = ev.scale;
    info[2] = ev.aqed;
    info[3] = ev.aqcd;
  }
  return RWGT_OK;
}

int rwgt_lhe_info(const rwgt_lhe* l, const int64_t* index, int64_t n, double* info) {
  if (!l || n < 0 || (n > 0 && (!index || !info))) return RWGT_EINVAL;
  for (int64_t r = 0; r < n; ++r) {
    if (index[r] < 0 || index[r] >= int64_t(l->events.size())) return RWGT_EINVAL;
    const Event& ev = l->events[size_t(index[r])];
    info[4 * r] = ev.xwgt;
    info[4 * r + 1] = ev.scale;
    info[4 * r + 2] = ev.aqed;
    info[4 * r + 3] = ev.aqcd;
  }
  return RWGT_OK;
}

int rwgt_lhe_select(rwgt_lhe* l, const char* process, int64_t* index_out, int64_t cap, int64_t* n_match) {
  if (!l || !n_match || cap < 0 || (cap > 0 && !index_out)) return RWGT_EINVAL;
  l->err.clear();
  std::vector<std::pair<int, int>> slots;
  int rc = l->process_slots(process, slots);
  if (rc != RWGT_OK) return rc;
  std::vector<int> map(slots.size());
  int64_t n = 0;
  for (size_t i = 0; i < l->events.size(); ++i) {
    if (!l->match(l->events[i], slots, map.data())) continue;
    if (n < cap) index_out[n] = int64_t(i);
    ++n;
  }
  *n_match = n;
  return RWGT_OK;
}

int rwgt_lhe_momenta(rwgt_lhe* l, const char* process, const int64_t* index, int64_t n, double* momenta,
                     double* weights) {
  if (!l || n < 0 || (n > 0 && (!index || !momenta))) return RWGT_EINVAL;
  l->err.clear();
  std::vector<std::pair<int, int>> slots;
  int rc = l->process_slots(process, slots);
  if (rc != RWGT_OK) return rc;
  const size_t np = slots.size();
  std::vector<int> map(np);
  for (int64_t r = 0; r < n; ++r) {
    const int64_t i = index[r];
    if (i < 0 || i >= int64_t(l->events.size())) return l->fail(RWGT_EINVAL, "event index out of range");
    const Event& ev = l->events[size_t(i)];
    if (!l->match(ev, slots, map.data()))
      return l->fail(RWGT_EPROCESS, "event " + std::to_string(i) + " does not belong to the process");
    for (size_t s = 0; s < np; ++s) {
      const Particle& q = l->parts[ev.first + size_t(map[s])];
      double* o = momenta + (size_t(r) * np + s) * 4;
      o[0] = q.p[3];                      // E
      o[1] = q.p[0];
      o[2] = q.p[1];
      o[3] = q.p[2];
    }
    if (weights) weights[r] = ev.xwgt;
  }
  return RWGT_OK;
}

int rwgt_lhe_add_weights(rwgt_lhe* l, const char* id, const char* description, const int64_t* index, int64_t n,
                         const double* w) {
  if (!l || !id || !*id || n < 0 || (n > 0 && (!index || !w))) return RWGT_EINVAL;
  l->err.clear();
  for (const char* c = id; *c; ++c)
    if (*c == '\'' || *c == '"' || *c == '<' || *c == '>' || *c == '&' || *c == ' ')
      return l->fail(RWGT_EINVAL, "weight id must not contain quotes, spaces, '<', '>' or '&'");
  Weight* wt = nullptr;
  for (auto& x : l->weights)
    if (x.id == id) wt = &x;
  if (!wt) {
    l->weights.push_back(Weight{id, description ? description : "", std::vector<double>(l->events.size(), 0.0)});
    wt = &l->weights.back();
  }
  for (int64_t r = 0; r < n; ++r) {
    if (index[r] < 0 || index[r] >= int64_t(l->events.size())) return l->fail(RWGT_EINVAL, "event index out of range");
    wt->value[size_t(index[r])] = w[r];
  }
  return RWGT_OK;
}

int rwgt_lhe_write(rwgt_lhe* l, const char* path) {
  if (!l || !path) return RWGT_EINVAL;
  l->err.clear();
  try {
    const std::string& t = l->text;
    std::string out;
    out.reserve(t.size() + l->events.size() * (l->weights.size() * 48 + 16) + 4096);
    // header: the new weightgroup inside <initrwgt>, created if absent
    std::string group;
    if (!l->weights.empty()) {
      group = "<weightgroup name='rwgt_amd' weight_name_strategy='includeIdInWeightName'>\n";
      for (const auto& w : l->weights) group += "<weight id='" + w.id + "'>" + w.description + "</weight>\n";
      group += "</weightgroup>\n";
    }
    const std::string head = t.substr(0, l->init_begin);
    if (group.empty()) {
      out += head;
    } else if (size_t p = head.rfind("</initrwgt>"); p != std::string::npos) {
      out += head.substr(0, p) + group + head.substr(p);
    } else if (size_t q = head.rfind("</header>"); q != std::string::npos) {
      out += head.substr(0, q) + "<initrwgt>\n" + group + "</initrwgt>\n" + head.substr(q);
    } else {
      out += head + "<header>\n<initrwgt>\n" + group + "</initrwgt>\n</header>\n";
    }
    size_t pos = l->init_begin;
    for (size_t i = 0; i < l->events.size(); ++i) {
      const Event& ev = l->events[i];
      out.append(t, pos, ev.end - pos);   // up to "</event>"
      if (!l->weights.empty()) {
        std::string wl;
        for (const auto& w : l->weights) {
          wl += "<wgt id='" + w.id + "'> ";
          fmt_double(wl, w.value[i]);
          wl += " </wgt>\n";
        }
        const std::string body = t.substr(ev.tail, ev.end - ev.tail);
        const size_t r = body.rfind("</rwgt>");
        if (r != std::string::npos) {
          // insert before the existing block's end
          out.resize(out.size() - (ev.end - ev.tail - r));
          out += wl;
          out.append(body, r, std::string::npos);
        } else {
          if (!out.empty() && out.back() != '\n') out += '\n';
          out += "<rwgt>\n" + wl + "</rwgt>\n";
        }
      }
      pos = ev.end;
    }
    out.append(t, pos, std::string::npos);
    std::ofstream f(path, std::ios::binary);
    if (!f) return l->fail(RWGT_EINVAL, std::string("cannot open ") + path + " for writing");
    f.write(out.data(), std::streamsize(out.size()));
    if (!f) return l->fail(RWGT_EDEVICE, "write failed");
    return RWGT_OK;
  } catch (const std::exception& ex) {
    return l->fail(RWGT_ENOMEM, ex.what());
  }
}

}  // extern "C"
