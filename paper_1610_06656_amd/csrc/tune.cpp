// Launch-shape table of the sketch pass: for a pass shape (operand precision,
// SRHT or Gaussian, k, n1, n2 with n2 = 0 when B is A, and the rows one launch
// covers) the sketch-row chunk cap of the BF16 stored-Pi pass and the number
// of row splits that smp_tune_sketch measured fastest. The table is shared by
// every context of the process (the choice is a function of the job's own
// shape only) and is kept in a JSON file between processes:
//
//   {"format": "smp-sketch-tuning", "version": 1, "entries": [
//     {"prec": 1, "srht": 0, "k": 1024, "n1": 4096, "n2": 4096, "rows": 32768,
//      "cap": 16, "splits": 2, "ms": 0.7012}, ...]}
//
// The reader accepts exactly what the writer produces (any whitespace, the
// keys of an entry in any order); anything else is an error and leaves the
// table as it was.
#include <cctype>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "smp_internal.hpp"

namespace smp {
namespace {

using Key = std::tuple<int, int, int, int64_t, int64_t, int64_t>;

std::mutex g_mu;
std::map<Key, TuneChoice> g_table;

Key key_of(const TuneKey &k) { return Key(k.prec, k.srht, k.k, k.n1, k.n2, k.rows); }

bool parse_int(const std::string &obj, const char *name, int64_t &out) {
  const std::string pat = std::string("\"") + name + "\"";
  const size_t at = obj.find(pat);
  if (at == std::string::npos) return false;
  size_t i = obj.find(':', at + pat.size());
  if (i == std::string::npos) return false;
  ++i;
  while (i < obj.size() && std::isspace((unsigned char)obj[i])) ++i;
  char *end = nullptr;
  const long long v = std::strtoll(obj.c_str() + i, &end, 10);
  if (end == obj.c_str() + i) return false;
  out = v;
  return true;
}

bool parse_double(const std::string &obj, const char *name, double &out) {
  const std::string pat = std::string("\"") + name + "\"";
  const size_t at = obj.find(pat);
  if (at == std::string::npos) return false;
  size_t i = obj.find(':', at + pat.size());
  if (i == std::string::npos) return false;
  char *end = nullptr;
  out = std::strtod(obj.c_str() + i + 1, &end);
  return end != obj.c_str() + i + 1;
}

}  // namespace

bool tune_lookup(const TuneKey &k, TuneChoice &out) {
  std::lock_guard<std::mutex> g(g_mu);
  const auto it = g_table.find(key_of(k));
  if (it == g_table.end()) return false;
  out = it->second;
  return true;
}

void tune_store(const TuneKey &k, const TuneChoice &c) {
  std::lock_guard<std::mutex> g(g_mu);
  g_table[key_of(k)] = c;
}

void tune_clear() {
  std::lock_guard<std::mutex> g(g_mu);
  g_table.clear();
}

size_t tune_count() {
  std::lock_guard<std::mutex> g(g_mu);
  return g_table.size();
}

std::string tune_save(const char *path) {
  std::lock_guard<std::mutex> g(g_mu);
  std::string s = "{\"format\": \"smp-sketch-tuning\", \"version\": 1, \"entries\": [";
  bool first = true;
  for (const auto &kv : g_table) {
    char buf[320];
    std::snprintf(buf, sizeof buf,
                  "%s\n  {\"prec\": %d, \"srht\": %d, \"k\": %d, \"n1\": %lld, \"n2\": %lld, \"rows\": %lld, "
                  "\"cap\": %d, \"splits\": %d, \"ms\": %.6f}",
                  first ? "" : ",", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                  (long long)std::get<3>(kv.first), (long long)std::get<4>(kv.first),
                  (long long)std::get<5>(kv.first), kv.second.cap, kv.second.splits, kv.second.ms);
    s += buf;
    first = false;
  }
  s += "\n]}\n";
  FILE *f = std::fopen(path, "wb");
  if (!f) return std::string("cannot open ") + path + " for writing";
  const bool ok = std::fwrite(s.data(), 1, s.size(), f) == s.size();
  if (std::fclose(f) != 0 || !ok) return std::string("cannot write ") + path;
  return "";
}

std::string tune_load(const char *path) {
  FILE *f = std::fopen(path, "rb");
  if (!f) return std::string("cannot open ") + path;
  std::string s;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, got);
  std::fclose(f);
  if (s.find("\"smp-sketch-tuning\"") == std::string::npos) return "not a sketch tuning file";
  int64_t version = 0;
  if (!parse_int(s, "version", version) || version != 1) return "unsupported tuning file version";
  const size_t lb = s.find('[', s.find("\"entries\""));
  const size_t rb = s.rfind(']');
  if (lb == std::string::npos || rb == std::string::npos || rb < lb) return "no entries list";
  std::vector<std::pair<TuneKey, TuneChoice>> got_entries;
  size_t i = lb + 1;
  while (true) {
    const size_t ob = s.find('{', i);
    if (ob == std::string::npos || ob > rb) break;
    const size_t cb = s.find('}', ob);
    if (cb == std::string::npos || cb > rb) return "unterminated entry";
    const std::string obj = s.substr(ob, cb - ob + 1);
    int64_t v[8];
    const char *names[8] = {"prec", "srht", "k", "n1", "n2", "rows", "cap", "splits"};
    for (int j = 0; j < 8; ++j)
      if (!parse_int(obj, names[j], v[j])) return std::string("entry without \"") + names[j] + "\"";
    if (v[0] < 0 || v[0] > 2 || v[1] < 0 || v[1] > 1 || v[2] < 1 || v[3] < 1 || v[4] < 0 || v[5] < 1 || v[6] < 0 ||
        v[7] < 1)
      return "entry out of range";
    double ms = 0.0;
    parse_double(obj, "ms", ms);
    TuneKey k{(int)v[0], (int)v[1], (int)v[2], v[3], v[4], v[5]};
    TuneChoice c{(int)v[6], (int)v[7], ms};
    got_entries.emplace_back(k, c);
    i = cb + 1;
  }
  std::lock_guard<std::mutex> g(g_mu);
  for (const auto &e : got_entries) g_table[key_of(e.first)] = e.second;
  return "";
}

}  // namespace smp
