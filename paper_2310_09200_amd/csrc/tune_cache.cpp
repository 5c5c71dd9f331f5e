// Autotune cache: the tile chosen per K class by bb_synth_autotune_batched,
// kept in the file named by the environment variable BB_TUNE_CACHE so that
// later handles (in this or another process) start from it.
//
// One JSON object per line, written and read by this file only:
//   {"arch": "gfx950", "precision": 2, "k_class": 2, "pix_log2": 18, "tile": 11, "ms": 565.8}
// keyed by the device architecture, the contraction mode, the K class and
// floor(log2(n_pix)) (the pixel count sets how many tiles a launch has per
// workgroup, which the best shape depends on).  Lines in another form are
// left alone: skipped on reading, kept on rewriting.  A rewrite goes to a
// temporary file beside the cache, then replaces it (rename), so a reader
// never sees a half-written file; two processes tuning at once keep the
// entries of whichever renames last.

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "tune_cache.h"

namespace bb_host {
namespace {

struct Entry {
  std::string arch;
  int precision = -1, k_class = -1, pix_log2 = -1, tile = -1;
  double ms = 0.0;
};

// The value after "key": in a line, as text up to the next ',' or '}'.
bool field(const std::string& line, const char* key, std::string& out) {
  const std::string k = std::string("\"") + key + "\":";
  const size_t p = line.find(k);
  if (p == std::string::npos) return false;
  size_t a = p + k.size();
  while (a < line.size() && line[a] == ' ') ++a;
  size_t b = a;
  while (b < line.size() && line[b] != ',' && line[b] != '}') ++b;
  if (b == a) return false;
  out = line.substr(a, b - a);
  while (!out.empty() && out.back() == ' ') out.pop_back();
  return true;
}

bool parse_int(const std::string& s, int& v) {
  char* end = nullptr;
  const long x = std::strtol(s.c_str(), &end, 10);
  if (end == s.c_str() || *end != 0 || x < -1000000 || x > 1000000) return false;
  v = (int)x;
  return true;
}

bool parse(const std::string& line, Entry& e) {
  std::string v;
  if (!field(line, "arch", v) || v.size() < 2 || v.front() != '"' || v.back() != '"') return false;
  e.arch = v.substr(1, v.size() - 2);
  if (!field(line, "precision", v) || !parse_int(v, e.precision)) return false;
  if (!field(line, "k_class", v) || !parse_int(v, e.k_class)) return false;
  if (!field(line, "pix_log2", v) || !parse_int(v, e.pix_log2)) return false;
  if (!field(line, "tile", v) || !parse_int(v, e.tile)) return false;
  if (field(line, "ms", v)) e.ms = std::strtod(v.c_str(), nullptr);
  return true;
}

std::string format(const Entry& e) {
  char buf[256];
  std::snprintf(buf, sizeof buf,
                "{\"arch\": \"%s\", \"precision\": %d, \"k_class\": %d, \"pix_log2\": %d, \"tile\": %d, \"ms\": %.3f}",
                e.arch.c_str(), e.precision, e.k_class, e.pix_log2, e.tile, e.ms);
  return buf;
}

std::vector<std::string> read_lines(const char* path) {
  std::vector<std::string> out;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line))
    if (!line.empty()) out.push_back(line);
  return out;
}

}  // namespace

const char* tune_cache_path() {
  const char* p = std::getenv("BB_TUNE_CACHE");
  return (p && p[0]) ? p : nullptr;
}

int pix_log2(int64_t n_pix) {
  int l = 0;
  while (l < 62 && ((int64_t)1 << (l + 1)) <= n_pix) ++l;
  return l;
}

void tune_cache_lookup(const std::string& arch, int precision, int64_t n_pix, int tiles[kTuneClasses]) {
  for (int c = 0; c < kTuneClasses; ++c) tiles[c] = -1;
  const char* path = tune_cache_path();
  if (!path) return;
  const int pl = pix_log2(n_pix);
  for (const std::string& line : read_lines(path)) {
    Entry e;
    if (!parse(line, e)) continue;
    if (e.arch == arch && e.precision == precision && e.pix_log2 == pl && e.k_class >= 0 && e.k_class < kTuneClasses)
      tiles[e.k_class] = e.tile;  // the last matching line wins
  }
}

bool tune_cache_store(const std::string& arch, int precision, int64_t n_pix, const int tiles[kTuneClasses],
                      const double ms[kTuneClasses], const bool tuned[kTuneClasses], std::string& err) {
  const char* path = tune_cache_path();
  if (!path) return true;
  const int pl = pix_log2(n_pix);
  std::vector<std::string> keep;
  for (const std::string& line : read_lines(path)) {
    Entry e;
    const bool same = parse(line, e) && e.arch == arch && e.precision == precision && e.pix_log2 == pl &&
                      e.k_class >= 0 && e.k_class < kTuneClasses && tuned[e.k_class];
    if (!same) keep.push_back(line);
  }
  for (int c = 0; c < kTuneClasses; ++c) {
    if (!tuned[c]) continue;
    Entry e;
    e.arch = arch;
    e.precision = precision;
    e.k_class = c;
    e.pix_log2 = pl;
    e.tile = tiles[c];
    e.ms = ms[c];
    keep.push_back(format(e));
  }
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) {
      err = "cannot write the tune cache " + tmp;
      return false;
    }
    for (const std::string& line : keep) f << line << '\n';
    f.flush();
    if (!f) {
      err = "cannot write the tune cache " + tmp;
      return false;
    }
  }
  if (std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    err = std::string("cannot replace the tune cache ") + path;
    return false;
  }
  return true;
}

}  // namespace bb_host
