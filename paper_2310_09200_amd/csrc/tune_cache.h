// Autotune cache (BB_TUNE_CACHE): tile per K class, kept in a file between
// handles and processes (tune_cache.cpp).
#pragma once

#include <stdint.h>

#include <string>

namespace bb_host {

constexpr int kTuneClasses = 4;

// Path from BB_TUNE_CACHE, or null when the variable is unset or empty.
const char* tune_cache_path();
// floor(log2(n_pix)) for n_pix >= 1: the pixel-count key of an entry.
int pix_log2(int64_t n_pix);
// tiles[c]: the cached tile of K class c for (arch, precision, pix_log2(n_pix)), -1 where none.
void tune_cache_lookup(const std::string& arch, int precision, int64_t n_pix, int tiles[kTuneClasses]);
// Replace the entries of the classes with tuned[c] for this key by tiles[c] (time ms[c]);
// false with a message when the file cannot be written.
bool tune_cache_store(const std::string& arch, int precision, int64_t n_pix, const int tiles[kTuneClasses],
                      const double ms[kTuneClasses], const bool tuned[kTuneClasses], std::string& err);

}  // namespace bb_host
