// Level determination and image weighting, on the device.
//
// k-means levels (Section 2.6; the positive/negative split of Section 4.2):
// exact one-dimensional k-means of the positive eigenvalues, i.e. the cut of
// the sorted values into k contiguous runs with the least total within-run sum
// of squared deviations, found by dynamic programming over the last cut.  One
// workgroup does it all in LDS: bitonic sort, k DP sweeps (thread j extends a
// Welford mean / sum of squares from v[j] down to v[m], so every run's cost is
// formed directly from its values), back-tracking, interval bounds at the gap
// midpoints and the level id of every eigenvalue.
//
// Uniform weighting (Section 3.5): every visibility V_pq is divided by the
// number of ordered antenna pairs whose baseline falls in the same uv cell,
// cells 1/FoV wide.  Cells are counted in an open-addressing hash table
// (64-bit keys, linear probing, global atomics) at least twice as large as the
// number of pairs, so that every probe sequence ends.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bb_internal.h"

namespace bb {

// ---------------------------------------------------------------------------
// k-means levels

constexpr int kKmThreads = 1024;  // = kMaxEig: one value per thread

__global__ __launch_bounds__(kKmThreads) void kmeans_levels_kernel(const double* __restrict__ lam, int n, int k,
                                                                   int negative_level, int n_levels,
                                                                   double* __restrict__ intervals,
                                                                   int* __restrict__ level_of,
                                                                   int* __restrict__ err) {
  __shared__ double s_v[kKmThreads];        // positive eigenvalues, sorted ascending (+inf padding)
  __shared__ double s_prev[kKmThreads];     // best cost of v[0..j] in m runs
  __shared__ double s_cur[kKmThreads];      // ... in m + 1 runs
  __shared__ int16_t s_cut[kMaxLevels][kKmThreads];  // start of the last run
  __shared__ double s_lo[kMaxLevels], s_hi[kMaxLevels];
  __shared__ double s_maxneg;
  __shared__ int s_npos, s_nneg;

  const int t = threadIdx.x;
  if (t == 0) {
    s_npos = 0;
    s_nneg = 0;
    s_maxneg = -INFINITY;
  }
  __syncthreads();
  const double x = t < n ? lam[t] : 0.0;
  const bool pos = t < n && x > 0.0;
  s_v[t] = pos ? x : INFINITY;
  if (pos) atomicAdd(&s_npos, 1);
  if (t < n && !pos) atomicAdd(&s_nneg, 1);
  __syncthreads();
  // largest non-positive eigenvalue (tree reduction over s_cur as scratch)
  s_cur[t] = (t < n && !pos) ? x : -INFINITY;
  __syncthreads();
  for (int w = kKmThreads / 2; w > 0; w >>= 1) {
    if (t < w) s_cur[t] = fmax(s_cur[t], s_cur[t + w]);
    __syncthreads();
  }
  if (t == 0) s_maxneg = s_cur[0];
  __syncthreads();

  // bitonic sort, ascending
  for (int size = 2; size <= kKmThreads; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const int partner = t ^ stride;
      if (partner > t) {
        const bool up = (t & size) == 0;
        const double a = s_v[t], b = s_v[partner];
        if ((a > b) == up) {
          s_v[t] = b;
          s_v[partner] = a;
        }
      }
      __syncthreads();
    }
  }

  const int np = s_npos;
  if (np < k) {  // fewer positive eigenvalues than positive levels
    if (t == 0) atomicOr(err, kErrKmeansTooFew);
    if (t < n_levels) {
      intervals[t] = NAN;
      intervals[n_levels + t] = NAN;
    }
    if (t < n) level_of[t] = -1;
    return;
  }

  // dynamic programme: s_cur[j] = min over i of s_prev[i - 1] + cost(v[i..j])
  for (int m = 0; m < k; ++m) {
    if (t >= m && t < np) {
      double mean = 0.0, m2 = 0.0, best = INFINITY;
      int arg = m;
      const int lowest = m;  // run start i >= m (m runs before it need m values)
      for (int i = t, c = 1; i >= lowest; --i, ++c) {
        const double v = s_v[i];
        const double delta = v - mean;
        mean += delta / (double)c;
        m2 += delta * (v - mean);
        if (m == 0) {
          if (i == 0) {
            best = m2;
            arg = 0;
          }
        } else {
          const double cand = s_prev[i - 1] + m2;
          if (cand <= best) {  // going down in i: ties keep the smallest start
            best = cand;
            arg = i;
          }
        }
      }
      s_cur[t] = best;
      s_cut[m][t] = (int16_t)arg;
    }
    __syncthreads();
    if (t < np) s_prev[t] = s_cur[t];
    __syncthreads();
  }

  if (t == 0) {
    int starts[kMaxLevels];
    int j = np - 1;
    for (int m = k - 1; m > 0; --m) {
      starts[m] = s_cut[m][j];
      j = starts[m] - 1;
    }
    starts[0] = 0;
    const double low = 0.5 * (s_v[0] + (s_nneg > 0 ? s_maxneg : 0.0));
    // run g (ascending) -> level k - 1 - g
    for (int g = 0; g < k; ++g) {
      const double lo = g == 0 ? low : 0.5 * (s_v[starts[g] - 1] + s_v[starts[g]]);
      const double hi = g + 1 < k ? 0.5 * (s_v[starts[g + 1] - 1] + s_v[starts[g + 1]]) : INFINITY;
      s_lo[k - 1 - g] = lo;
      s_hi[k - 1 - g] = hi;
    }
    if (negative_level) {
      s_lo[k] = -INFINITY;
      s_hi[k] = nextafter(low, -INFINITY);
    }
  }
  __syncthreads();
  if (t < n_levels) {
    intervals[t] = s_lo[t];
    intervals[n_levels + t] = s_hi[t];
  }
  if (t < n) {
    int lev = -1;
    for (int l = 0; l < n_levels; ++l) {
      if (s_lo[l] <= x && x <= s_hi[l]) {
        lev = l;
        break;
      }
    }
    level_of[t] = lev;
  }
}

hipError_t launch_kmeans_levels(const double* lam, int n, int k, int negative_level, double* intervals,
                                int* level_of, int* err, hipStream_t s) {
  if (n < 1 || n > kKmThreads || k < 1 || k + (negative_level ? 1 : 0) > kMaxLevels) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kmeans_levels_kernel, dim3(1), dim3(kKmThreads), 0, s, lam, n, k, negative_level,
                     k + (negative_level ? 1 : 0), intervals, level_of, err);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Uniform weighting

constexpr uint64_t kEmptyKey = 0x8000000080000000ull;  // cell (INT_MIN, INT_MIN): never a real cell
constexpr double kMaxCell = 1073741824.0;              // |cell| < 2^30

__device__ __forceinline__ uint64_t mix64(uint64_t z) {  // splitmix64 finaliser
  z ^= z >> 30;
  z *= 0xbf58476d1ce4e5b9ull;
  z ^= z >> 27;
  z *= 0x94d049bb133111ebull;
  z ^= z >> 31;
  return z;
}

// uv cell of the ordered pair (p, q); false when it is out of range.  The
// operation order is part of the definition (a coordinate on a cell edge is
// decided by it), so no multiply-add is fused here.
__device__ bool uv_cell_key(const double* __restrict__ ant, int64_t ld, int p, int q, const UvFrame& f,
                            uint64_t& key) {
#pragma clang fp contract(off)
  const double d0 = ant[p] - ant[q];
  const double d1 = ant[p + ld] - ant[q + ld];
  const double d2 = ant[p + 2 * ld] - ant[q + 2 * ld];
  const double au = ((d0 * f.eu[0] + d1 * f.eu[1]) + d2 * f.eu[2]) * f.scale;
  const double av = ((d0 * f.ev[0] + d1 * f.ev[1]) + d2 * f.ev[2]) * f.scale;
  const double cu = round(au), cv = round(av);  // halves away from zero
  if (!(fabs(cu) < kMaxCell) || !(fabs(cv) < kMaxCell)) return false;
  key = ((uint64_t)(uint32_t)(int32_t)cu << 32) | (uint64_t)(uint32_t)(int32_t)cv;
  return true;
}

__global__ __launch_bounds__(256) void uv_clear_kernel(uint64_t* __restrict__ keys, uint32_t* __restrict__ counts,
                                                       int64_t slots) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= slots) return;
  keys[i] = kEmptyKey;
  counts[i] = 0u;
}

__global__ __launch_bounds__(256) void uv_count_kernel(const double* __restrict__ ant, int64_t ld, int L, UvFrame f,
                                                       uint64_t* __restrict__ keys, uint32_t* __restrict__ counts,
                                                       int64_t slots, int* __restrict__ err) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)L * L) return;
  const int p = (int)(idx % L), q = (int)(idx / L);
  uint64_t key;
  if (!uv_cell_key(ant, ld, p, q, f, key)) {
    atomicOr(err, kErrUvRange);
    return;
  }
  const uint64_t mask = (uint64_t)slots - 1;
  uint64_t h = mix64(key) & mask;
  for (int64_t probe = 0; probe < slots; ++probe) {
    const unsigned long long prev =
        atomicCAS((unsigned long long*)&keys[h], (unsigned long long)kEmptyKey, (unsigned long long)key);
    if (prev == kEmptyKey || prev == key) {
      atomicAdd(&counts[h], 1u);
      return;
    }
    h = (h + 1) & mask;
  }
}

__global__ __launch_bounds__(256) void uv_apply_kernel(const double* __restrict__ ant, int64_t ld, int L, UvFrame f,
                                                       const uint64_t* __restrict__ keys,
                                                       const uint32_t* __restrict__ counts, int64_t slots,
                                                       double* __restrict__ vis) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)L * L) return;
  const int p = (int)(idx % L), q = (int)(idx / L);
  uint64_t key;
  if (!uv_cell_key(ant, ld, p, q, f, key)) return;  // flagged by the count pass
  const uint64_t mask = (uint64_t)slots - 1;
  uint64_t h = mix64(key) & mask;
  for (int64_t probe = 0; probe < slots; ++probe) {
    const uint64_t kk = keys[h];
    if (kk == key) {
      const double c = (double)counts[h];
      double* v = vis + 2 * ((int64_t)q * L + p);
      v[0] = v[0] / c;
      v[1] = v[1] / c;
      return;
    }
    if (kk == kEmptyKey) return;  // not reached: every pair's key was inserted
    h = (h + 1) & mask;
  }
}

int64_t uv_table_slots(int L) {
  int64_t slots = 1;
  while (slots < 2 * (int64_t)L * L) slots <<= 1;
  return slots;
}

hipError_t launch_uniform_weighting(const double* ant, int64_t ld, int L, const UvFrame& f, void* table,
                                    double* vis, int* err, hipStream_t s) {
  const int64_t slots = uv_table_slots(L);
  uint64_t* keys = (uint64_t*)table;
  uint32_t* counts = (uint32_t*)(keys + slots);
  const int64_t pairs = (int64_t)L * L;
  hipLaunchKernelGGL(uv_clear_kernel, dim3((unsigned)((slots + 255) / 256)), dim3(256), 0, s, keys, counts, slots);
  hipLaunchKernelGGL(uv_count_kernel, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s, ant, ld, L, f, keys,
                     counts, slots, err);
  hipLaunchKernelGGL(uv_apply_kernel, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s, ant, ld, L, f, keys,
                     counts, slots, vis);
  return hipGetLastError();
}

// Byte fill with 0xFF: the workspace poison of the BB_DEBUG_FILL debug mode.
__global__ void fill_poison_kernel(unsigned char* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0xFF;
}

hipError_t launch_fill_poison(void* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_poison_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (unsigned char*)p, n);
  return hipGetLastError();
}

}  // namespace bb
