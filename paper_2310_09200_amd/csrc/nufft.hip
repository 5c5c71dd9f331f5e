// NUFFT synthesis kernels for gfx950 (Section 2.5; Section 3.4, Algorithm 3).
//
// The level image is the type-3 Fourier sum over baselines
//     I_l(p) = sum_q V'_l[q, q] + 2 Re sum_{q < r} V'_l[r, q] exp(+2 pi i <b_qr, p>),
//     V'_l = W_l diag(d_l) W_l^H,   b_qr = (x_q - x_r) / lambda_w,
// evaluated in an image frame (e_u, e_v, p0) as
//   1. spread: every baseline of every collected instance deposits
//      V'_l[r, q] exp(2 pi i <b, D>) times the tensor-product
//      exponential-of-semicircle kernel on the w^3 nearest points of the
//      periodic N0 x N1 x N2 grid (spacing h_d turns), one channel per level.
//      Grids thin along axis 2 are spread from the grid's side
//      (nufft_gather.hip); thicker ones with LDS tiles or global atomics (here);
//   2. deconvolve and zero-pad: each level's grid, divided by the type-2
//      kernel's transform, placed in an M = 2N grid;
//   3. inverse FFT (unnormalised, e^{+i}), pruned to the lines that hold data
//      and the outputs the pixels reach (nufft_fft.hip: LDS line FFTs, a
//      direct DFT on MFMA for lines of at most 64 points; rocFFT for long lines);
//   4. interpolate at each pixel's rescaled position with the same kernel,
//      divide by the spreading kernel's transform there, and add
//      2 Re(.) + the diagonal term into the image.
// The grid is the accumulator over instances: instances collected before one
// emit share steps 2-4 (the sum is linear).  Where grid points are added with
// FP32 atomics (split column blocks, tiles, the global-atomic path) their
// order, and so the last bits, vary between runs.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "bb_internal.h"
#include "nufft_device.h"

namespace bb {

typedef float f32x2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Per instance: eigenpair order grouped by level (stable), level starts, and
// the diagonal term sum_{k in l} d_k ||w_k||^2 added into diag[l].
__global__ __launch_bounds__(256) void nufft_prep_kernel(const NufftInst* __restrict__ insts, const float2* __restrict__ W,
                                                         const float* __restrict__ dw, const int* __restrict__ lev,
                                                         int n_levels, int* __restrict__ order, int* __restrict__ lstart,
                                                         double* __restrict__ diag, int* __restrict__ err) {
  const NufftInst I = insts[blockIdx.x];
  __shared__ int s_count[kMaxLevels + 1];
  __shared__ double s_sum[kMaxLevels][256 / 64];
  const int tid = threadIdx.x;
  int* ord = order + I.ord_off;
  int* ls = lstart + I.ls_off;
  if (tid == 0) {
    for (int l = 0; l <= n_levels; ++l) s_count[l] = 0;
    for (int k = 0; k < I.n_eig; ++k) {
      int lv = lev[I.eig_off + k];
      if (lv < -1 || lv >= n_levels) {
        atomicOr(err, kErrLevelId);
        lv = -1;
      }
      if (lv >= 0) s_count[lv + 1] += 1;
    }
    for (int l = 0; l < n_levels; ++l) s_count[l + 1] += s_count[l];
    for (int l = 0; l <= n_levels; ++l) ls[l] = s_count[l];
    for (int k = 0; k < I.n_eig; ++k) {  // stable placement
      const int lv = lev[I.eig_off + k];
      if (lv >= 0 && lv < n_levels) ord[s_count[lv]++] = k;
    }
  }
  __syncthreads();
  // diagonal term: thread t sums d_k ||w_k||^2 over the eigenpairs k = t, t + 256, ...
  double part[kMaxLevels];
#pragma unroll
  for (int l = 0; l < kMaxLevels; ++l) part[l] = 0.0;
  for (int k = tid; k < I.n_eig; k += 256) {
    const int lv = lev[I.eig_off + k];
    if (lv < 0 || lv >= n_levels) continue;
    const float2* col = W + I.w_off + (int64_t)k * I.n_ant;
    double nrm = 0.0;
    for (int q = 0; q < I.n_ant; ++q) nrm += (double)col[q].x * col[q].x + (double)col[q].y * col[q].y;
    const double v = (double)dw[I.eig_off + k] * nrm;
#pragma unroll
    for (int l = 0; l < kMaxLevels; ++l)
      if (l == lv) part[l] += v;
  }
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int l = 0; l < kMaxLevels; ++l) {
    double v = part[l];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) s_sum[l][wave] = v;
  }
  __syncthreads();
  if (tid < n_levels) {
    const double v = ((s_sum[tid][0] + s_sum[tid][1]) + s_sum[tid][2]) + s_sum[tid][3];
    if (v != 0.0) unsafeAtomicAdd(&diag[tid], v);
  }
}

// ---------------------------------------------------------------------------
// Spreading: one thread per antenna pair (q, r), q < r, of one instance.
template <int W>
__global__ __launch_bounds__(256) void nufft_spread_kernel(NufftGeom g, const NufftInst* __restrict__ insts,
                                                           const double* __restrict__ ant, int64_t ant_ld,
                                                           const float2* __restrict__ Wp, const float* __restrict__ dw,
                                                           const int* __restrict__ order, const int* __restrict__ lstart,
                                                           int n_levels, float* __restrict__ grid, int64_t n_cell,
                                                           int* __restrict__ err) {
  const NufftInst I = insts[blockIdx.y];
  const int L = I.n_ant;
  const int64_t pair = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pair >= (int64_t)L * L) return;
  const int q = (int)(pair % L), r = (int)(pair / L);  // consecutive lanes: consecutive q, same r
  if (q >= r) return;

  double xi[3], t;
  const int where = source_coords(g, I, ant, ant_ld, q, r, xi, t);
  if (where != 0) {
    if (where == 1) atomicOr(err, kErrNufftExtent);
    return;
  }
  // pre-phase exp(2 pi i <b, D>) centres the targets; turns reduced exactly in FP64
  const float f = (float)(t - rint(t));
  const float pc = __builtin_amdgcn_cosf(f), ps = __builtin_amdgcn_sinf(f);

  // axis 0 is walked at run time (its kernel value computed per step), axes 1
  // and 2 are unrolled from precomputed rows: keeps the w^2 addresses of a
  // step in registers without spilling
  const double xi0 = xi[0];
  const double first0 = ceil(xi0 - 0.5 * W);
  int64_t j0 = (int64_t)first0 % g.N[0];
  if (j0 < 0) j0 += g.N[0];
  float k1[W], k2[W];
  int i1[W], i2[W];
  kernel_row<W>(xi[1], g.N[1], g.beta, k1, i1);
  kernel_row<W>(xi[2], g.N[2], g.beta, k2, i2);
  const float inv_half = 2.0f / (float)W;

  const float2* Wi = Wp + I.w_off;
  const int* ord = order + I.ord_off;
  const int* ls = lstart + I.ls_off;
  const int64_t n12 = (int64_t)g.N[1] * g.N[2];
  for (int lv = 0; lv < n_levels; ++lv) {
    const int k_lo = ls[lv], k_hi = ls[lv + 1];
    if (k_lo == k_hi) continue;
    // V'[r, q] = sum_k d_k W_rk conj(W_qk)
    float cr = 0.0f, ci = 0.0f;
    for (int t2 = k_lo; t2 < k_hi; ++t2) {
      const int k = ord[t2];
      const float2 wq = Wi[q + (int64_t)k * L];
      const float2 wr = Wi[r + (int64_t)k * L];
      const float dk = dw[I.eig_off + k];
      cr += dk * (wr.x * wq.x + wr.y * wq.y);
      ci += dk * (wr.y * wq.x - wr.x * wq.y);
    }
    const float vr = cr * pc - ci * ps, vi = cr * ps + ci * pc;
    float* G = grid + 2 * (int64_t)lv * n_cell;
#pragma unroll 1
    for (int a = 0; a < W; ++a) {
      const float ka = es_kernel((float)((first0 + a) - xi0) * inv_half, g.beta);
      int64_t ia = j0 + a;
      if (ia >= g.N[0]) ia -= g.N[0];
      const float ar = vr * ka, ai = vi * ka;
      const int64_t row = ia * n12;
#pragma unroll
      for (int c = 0; c < W; ++c) {
        const float br = ar * k1[c], bi = ai * k1[c];
        float* line = G + 2 * (row + (int64_t)i1[c] * g.N[2]);
#pragma unroll
        for (int e = 0; e < W; ++e) {
          unsafeAtomicAdd(line + 2 * i2[e], br * k2[e]);
          unsafeAtomicAdd(line + 2 * i2[e] + 1, bi * k2[e]);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Tiled spreading (the default): V' is formed once per pair and level, the
// baselines are sorted into bins by the first grid point of their support on
// axes 0 and 1, and one workgroup per (tile, level) accumulates every baseline
// that reaches its tile in LDS, then adds the tile into the grid.  Tiles
// cover disjoint cells (the whole of axis 2), so the grid is written with
// plain loads and stores; only LDS sees atomics.

// V'_l[r, q] = sum_{k in l} d_k W_rk conj(W_qk) for q < r, at vp[vp_off + l L^2 + q + r L].
// One workgroup per 32 x 32 block of (q, r) with q-block <= r-block: the two
// blocks of W rows (the r side times d_k) go through LDS kVpK eigenpairs at a
// time, level by level in the level-grouped order; each thread keeps 2 x 2
// pairs.
constexpr int kVpK = 64;

__global__ __launch_bounds__(256) void nufft_vprime_kernel(const NufftInst* __restrict__ insts,
                                                           const float2* __restrict__ Wp, const float* __restrict__ dw,
                                                           const int* __restrict__ order, const int* __restrict__ lstart,
                                                           int n_levels, float2* __restrict__ vp) {
  __shared__ float2 s_q[kVpK][32], s_r[kVpK][32];
  const NufftInst I = insts[blockIdx.y];
  const int L = I.n_ant;
  const int nb = (L + 31) / 32;
  // upper-triangular block (bq <= br) number blockIdx.x
  int br = 0, rest = blockIdx.x;
  while (br < nb && rest > br) rest -= br + 1, ++br;
  if (br >= nb) return;
  const int bq = rest;
  const int tid = threadIdx.x, tq = tid & 15, tr = tid >> 4;
  const float2* Wi = Wp + I.w_off;
  const int* ord = order + I.ord_off;
  const int* ls = lstart + I.ls_off;
  const int q0 = bq * 32, r0 = br * 32;
  for (int lv = 0; lv < n_levels; ++lv) {
    float2 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = make_float2(0.0f, 0.0f);
    const int k_lo = ls[lv], k_hi = ls[lv + 1];
    for (int k0 = k_lo; k0 < k_hi; k0 += kVpK) {
      const int nk = min(kVpK, k_hi - k0);
      __syncthreads();  // the previous chunk is consumed
      for (int i = tid; i < nk * 32; i += 256) {
        const int row = i & 31, kk = i >> 5;
        const int k = ord[k0 + kk];
        const int64_t col = (int64_t)k * L;
        const float dk = dw[I.eig_off + k];
        const float2 wq = q0 + row < L ? Wi[q0 + row + col] : make_float2(0.0f, 0.0f);
        const float2 wr = r0 + row < L ? Wi[r0 + row + col] : make_float2(0.0f, 0.0f);
        s_q[kk][row] = wq;
        s_r[kk][row] = make_float2(dk * wr.x, dk * wr.y);
      }
      __syncthreads();
      for (int kk = 0; kk < nk; ++kk) {
        const float2 wq[2] = {s_q[kk][tq], s_q[kk][tq + 16]};
        const float2 wr[2] = {s_r[kk][tr], s_r[kk][tr + 16]};
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {  // wr conj(wq)
            acc[a][b].x += wr[b].x * wq[a].x + wr[b].y * wq[a].y;
            acc[a][b].y += wr[b].y * wq[a].x - wr[b].x * wq[a].y;
          }
      }
    }
    float2* out = vp + I.vp_off + (int64_t)lv * L * L;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int q = q0 + tq + 16 * a, r = r0 + tr + 16 * b;
        if (q < r && r < L) out[q + (int64_t)r * L] = acc[a][b];
      }
  }
}

// pass 0: count baselines per bin; pass 1: place them (cursor = bin starts).
__global__ __launch_bounds__(256) void nufft_bin_kernel(NufftGeom g, const NufftInst* __restrict__ insts,
                                                        const double* __restrict__ ant, int64_t ld, int bin, int nb1,
                                                        int pass, int* __restrict__ count_or_cursor,
                                                        uint64_t* __restrict__ list, int* __restrict__ err) {
  const NufftInst I = insts[blockIdx.y];
  const int L = I.n_ant;
  const int64_t pair = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pair >= (int64_t)L * L) return;
  const int q = (int)(pair % L), r = (int)(pair / L);
  if (q >= r) return;
  double xi[3], td;
  const int where = source_coords(g, I, ant, ld, q, r, xi, td);
  if (where != 0) {  // beyond the extent (reported once), or another uvw cell's
    if (where == 1 && pass == 0) atomicOr(err, kErrNufftExtent);
    return;
  }
  const int b = (first_cell(xi[0], g.w, g.N[0]) / bin) * nb1 + first_cell(xi[1], g.w, g.N[1]) / bin;
  const int pos = atomicAdd(&count_or_cursor[b], 1);
  if (pass == 1) list[pos] = ((uint64_t)blockIdx.y << 32) | ((uint64_t)q << 16) | (uint64_t)r;
}

// Exclusive prefix sum of n counts into offset[0..n] and cursor[0..n-1] (one workgroup).
__global__ __launch_bounds__(1024) void nufft_scan_kernel(const int* __restrict__ count, int n, int* __restrict__ offset,
                                                          int* __restrict__ cursor) {
  __shared__ int s[1024];
  __shared__ int carry;
  const int tid = threadIdx.x;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < n; base += 1024) {
    const int v = base + tid < n ? count[base + tid] : 0;
    s[tid] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int t = tid >= off ? s[tid - off] : 0;
      __syncthreads();
      s[tid] += t;
      __syncthreads();
    }
    if (base + tid < n) {
      offset[base + tid] = carry + s[tid] - v;
      if (cursor) cursor[base + tid] = carry + s[tid] - v;
    }
    __syncthreads();
    if (tid == 1023) carry += s[1023];
    __syncthreads();
  }
  if (tid == 0) offset[n] = carry;
}

// Exclusive prefix sums of long arrays in three steps: the sum of each chunk
// of kScanChunk counts, a one-workgroup scan of those sums, and a scan inside
// each chunk started at its chunk's offset.
constexpr int kScanChunk = 4096;

__global__ __launch_bounds__(1024) void scan_chunk_sums_kernel(const int* __restrict__ count, int n,
                                                               int* __restrict__ sums) {
  __shared__ int s[1024];
  const int base = blockIdx.x * kScanChunk, t = threadIdx.x;
  int v = 0;
  for (int i = t; i < kScanChunk; i += 1024)
    if (base + i < n) v += count[base + i];
  s[t] = v;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) s[t] += s[t + off];
    __syncthreads();
  }
  if (t == 0) sums[blockIdx.x] = s[0];
}

// Each thread scans 4 consecutive counts; cursor may alias count (every count
// is read before the barrier that precedes the writes).
__global__ __launch_bounds__(1024) void scan_chunks_kernel(const int* count, int n, const int* __restrict__ chunk_off,
                                                           int* __restrict__ offset, int* cursor) {
  __shared__ int s[1024];
  const int base = blockIdx.x * kScanChunk, t = threadIdx.x;
  int v[4], sum = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int idx = base + 4 * t + i;
    v[i] = idx < n ? count[idx] : 0;
    sum += v[i];
  }
  s[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int x = t >= off ? s[t - off] : 0;
    __syncthreads();
    s[t] += x;
    __syncthreads();
  }
  int run = chunk_off[blockIdx.x] + s[t] - sum;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int idx = base + 4 * t + i;
    if (idx < n) {
      offset[idx] = run;
      if (cursor) cursor[idx] = run;
    }
    run += v[i];
  }
  if (blockIdx.x == gridDim.x - 1 && t == 0) offset[n] = chunk_off[gridDim.x];
}

// Bins holding the first cells x0 - (w - 1) .. x0 + t - 1 (mod n) of an axis:
// every baseline that reaches cells x0 .. x0 + t - 1 starts in one of them.
__device__ int tile_bins(int x0, int t, int n, int bin, int w, int (&out)[8]) {
  int len = t + w - 1;
  if (len > n) len = n;
  int c = ((x0 - (w - 1)) % n + n) % n;
  int cnt = 0, covered = 0;
  while (covered < len) {
    const int b = c / bin;
    bool seen = false;
    for (int k = 0; k < cnt; ++k) seen |= out[k] == b;
    if (!seen && cnt < 8) out[cnt++] = b;
    const int next = min((b + 1) * bin, n);
    covered += next - c;
    c = next == n ? 0 : next;
  }
  return cnt;
}

// Chunks of a tile's candidate baselines: nch[t] = ceil(candidates / chunk).
__global__ __launch_bounds__(256) void nufft_tile_chunks_kernel(NufftGeom g, const int* __restrict__ offset, int bin,
                                                                int nb0, int nb1, int chunk, int* __restrict__ nch) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb0 * nb1) return;
  const int bx = t / nb1, by = t % nb1;
  const int x0 = bx * bin, y0 = by * bin;
  int cb0[8], cb1[8];
  const int nc0 = tile_bins(x0, min(bin, g.N[0] - x0), g.N[0], bin, g.w, cb0);
  const int nc1 = tile_bins(y0, min(bin, g.N[1] - y0), g.N[1], bin, g.w, cb1);
  int cnt = 0;
  for (int i = 0; i < nc0; ++i)
    for (int j = 0; j < nc1; ++j) {
      const int b = cb0[i] * nb1 + cb1[j];
      cnt += offset[b + 1] - offset[b];
    }
  nch[t] = (cnt + chunk - 1) / chunk;
}

// One workgroup per (chunk, level), grid-strided over the chunks of every tile
// (chunk c belongs to the tile t with choff[t] <= c < choff[t + 1]).  A tile of
// one chunk adds its LDS tile into the grid with plain loads and stores (it is
// the only writer of those cells); the chunks of a busier tile use atomics.
template <int W>
__global__ __launch_bounds__(256) void nufft_spread_tile_kernel(NufftGeom g, const NufftInst* __restrict__ insts,
                                                                const double* __restrict__ ant, int64_t ld,
                                                                const float2* __restrict__ vp,
                                                                const int* __restrict__ offset,
                                                                const uint64_t* __restrict__ list, int bin, int nb0,
                                                                int nb1, int chunk, const int* __restrict__ choff,
                                                                float* __restrict__ grid, int64_t n_cell) {
  extern __shared__ float2 s_tile[];  // t0 x t1 x N2
  __shared__ int s_tile_id;
  const int tid = threadIdx.x;
  const int lv = blockIdx.y;
  const int n_tiles = nb0 * nb1;
  const int n_chunks = choff[n_tiles];
  const int n2 = g.N[2];
  float* G = grid + 2 * (int64_t)lv * n_cell;
  for (int c = blockIdx.x; c < n_chunks; c += gridDim.x) {
    if (tid == 0) {  // tile of chunk c: last t with choff[t] <= c
      int lo = 0, hi = n_tiles;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (choff[mid] <= c) lo = mid; else hi = mid;
      }
      s_tile_id = lo;
    }
    __syncthreads();
    const int t = s_tile_id;
    const int k = c - choff[t];
    const bool shared_tile = choff[t + 1] - choff[t] > 1;
    const int bx = t / nb1, by = t % nb1;
    const int x0 = bx * bin, y0 = by * bin;
    const int t0 = min(bin, g.N[0] - x0), t1 = min(bin, g.N[1] - y0);
    const int n_tile = t0 * t1 * n2;
    for (int i = tid; i < n_tile; i += blockDim.x) s_tile[i] = make_float2(0.0f, 0.0f);
    __syncthreads();
    int cb0[8], cb1[8];
    const int nc0 = tile_bins(x0, t0, g.N[0], bin, W, cb0);
    const int nc1 = tile_bins(y0, t1, g.N[1], bin, W, cb1);
    // candidates [k chunk, (k + 1) chunk) of the tile's bins taken in order
    const int c_lo = k * chunk, c_hi = c_lo + chunk;
    int before = 0;
    for (int i = 0; i < nc0; ++i) {
      for (int j = 0; j < nc1; ++j) {
        const int b = cb0[i] * nb1 + cb1[j];
        const int beg = offset[b], cnt = offset[b + 1] - beg;
        const int lo = max(c_lo - before, 0), hi = min(c_hi - before, cnt);
        before += cnt;
        for (int s = lo + tid; s < hi; s += blockDim.x) {
          const uint64_t key = list[beg + s];
          const int inst = (int)(key >> 32), q = (int)((key >> 16) & 0xffff), r = (int)(key & 0xffff);
          const NufftInst I = insts[inst];
          double xi[3], td;
          if (source_coords(g, I, ant, ld, q, r, xi, td) != 0) continue;
          const int L = I.n_ant;
          const float2 v = vp[I.vp_off + (int64_t)lv * L * L + q + (int64_t)r * L];
          const float f = (float)(td - rint(td));
          const float pc = __builtin_amdgcn_cosf(f), ps = __builtin_amdgcn_sinf(f);
          const float vr = v.x * pc - v.y * ps, vi = v.x * ps + v.y * pc;
          float k0[W], k1[W], k2[W];
          int j0[W], j1[W], j2[W];
          kernel_row<W>(xi[0], g.N[0], g.beta, k0, j0);
          kernel_row<W>(xi[1], g.N[1], g.beta, k1, j1);
          kernel_row<W>(xi[2], g.N[2], g.beta, k2, j2);
#pragma unroll
          for (int a = 0; a < W; ++a) {
            int x = j0[a] - x0;
            if (x < 0) x += g.N[0];
            if (x >= t0) continue;
            const float ar = vr * k0[a], ai = vi * k0[a];
#pragma unroll
            for (int cc = 0; cc < W; ++cc) {
              int y = j1[cc] - y0;
              if (y < 0) y += g.N[1];
              if (y >= t1) continue;
              const float br = ar * k1[cc], bi = ai * k1[cc];
              float2* line = s_tile + (x * t1 + y) * n2;
#pragma unroll
              for (int e = 0; e < W; ++e) {
                atomicAdd(&line[j2[e]].x, br * k2[e]);
                atomicAdd(&line[j2[e]].y, bi * k2[e]);
              }
            }
          }
        }
      }
    }
    __syncthreads();
    for (int i = tid; i < n_tile; i += blockDim.x) {
      const int z = i % n2;
      const int rest = i / n2;
      const int y = rest % t1, x = rest / t1;
      const int64_t cell = ((int64_t)(x0 + x) * g.N[1] + (y0 + y)) * n2 + z;
      const float2 v = s_tile[i];
      if (v.x != 0.0f || v.y != 0.0f) {
        if (shared_tile) {
          unsafeAtomicAdd(&G[2 * cell], v.x);
          unsafeAtomicAdd(&G[2 * cell + 1], v.y);
        } else {
          G[2 * cell] += v.x;
          G[2 * cell + 1] += v.y;
        }
      }
    }
    __syncthreads();  // s_tile and s_tile_id are reused by the next chunk
  }
}

// ---------------------------------------------------------------------------
// The type-2 transform of one level's grid, pruned: an inverse 3-D FFT of the
// grid zero-padded from N to M points per axis, done as three batched 1-D
// FFTs (rocFFT) so that only lines holding data are transformed and only the
// outputs the pixels need (a window of win_len points per axis) are kept.
// Each gather places one axis's frequencies -N/2 .. N/2-1 at m = g mod M,
// divides by that axis's kernel transform and zero-fills the rest:
//   A [i0][i1][m2]   (N0 x N1 x M2)   from the grid        -> FFT along m2
//   B [i0][w2][m1]   (N0 x W2 x M1)   from A, m2 in window -> FFT along m1
//   C [w1][w2][m0]   (W1 x W2 x M0)   from B, m1 in window -> FFT along m0

// stored index of the frequency at position m of an M-point axis (-1 = zero padding)
__device__ __forceinline__ int freq_index(int m, int n, int M) {
  const int half = n / 2;
  if (m < half) return m;
  if (m >= M - half) return m - M + n;
  return -1;
}

__global__ __launch_bounds__(256) void nufft_gather_a_kernel(NufftGeom g, const float2* __restrict__ grid,
                                                             const float* __restrict__ inv_psi2,
                                                             float2* __restrict__ A, int64_t n_out) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n_out;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int m2 = (int)(idx % g.M[2]);
    const int64_t line = idx / g.M[2];  // i0 N1 + i1
    const int i2 = freq_index(m2, g.N[2], g.M[2]);
    float2 v = make_float2(0.0f, 0.0f);
    if (i2 >= 0) {
      const float2 x = grid[line * g.N[2] + i2];
      const float s = inv_psi2[i2];
      v = make_float2(x.x * s, x.y * s);
    }
    A[idx] = v;
  }
}

__global__ __launch_bounds__(256) void nufft_gather_b_kernel(NufftGeom g, const float2* __restrict__ A,
                                                             const float* __restrict__ inv_psi1,
                                                             float2* __restrict__ B, int64_t n_out) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n_out;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int m1 = (int)(idx % g.M[1]);
    const int64_t rest = idx / g.M[1];
    const int w2 = (int)(rest % g.win_len[2]);
    const int i0 = (int)(rest / g.win_len[2]);
    int m2 = g.win_lo[2] + w2;
    if (m2 >= g.M[2]) m2 -= g.M[2];
    const int i1 = freq_index(m1, g.N[1], g.M[1]);
    float2 v = make_float2(0.0f, 0.0f);
    if (i1 >= 0) {
      const float2 x = A[((int64_t)i0 * g.N[1] + i1) * g.M[2] + m2];
      const float s = inv_psi1[i1];
      v = make_float2(x.x * s, x.y * s);
    }
    B[idx] = v;
  }
}

__global__ __launch_bounds__(256) void nufft_gather_c_kernel(NufftGeom g, const float2* __restrict__ B,
                                                             const float* __restrict__ inv_psi0,
                                                             float2* __restrict__ C, int64_t n_out) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n_out;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int m0 = (int)(idx % g.M[0]);
    const int64_t rest = idx / g.M[0];
    const int w2 = (int)(rest % g.win_len[2]);
    const int w1 = (int)(rest / g.win_len[2]);
    int m1 = g.win_lo[1] + w1;
    if (m1 >= g.M[1]) m1 -= g.M[1];
    const int i0 = freq_index(m0, g.N[0], g.M[0]);
    float2 v = make_float2(0.0f, 0.0f);
    if (i0 >= 0) {
      const float2 x = B[((int64_t)i0 * g.win_len[2] + w2) * g.M[1] + m1];
      const float s = inv_psi0[i0];
      v = make_float2(x.x * s, x.y * s);
    }
    C[idx] = v;
  }
}

// ---------------------------------------------------------------------------
// Interpolation at the pixels, correction and accumulation into one level's image.
template <int W, bool SHIFT>
__global__ __launch_bounds__(256) void nufft_interp_kernel(NufftGeom g, InterpLayout lay,
                                                           const double* __restrict__ pix, int64_t pix_ld,
                                                           int64_t n_pix, const float* __restrict__ u,
                                                           const double* __restrict__ corr,
                                                           const double* __restrict__ diag, int lv,
                                                           float* __restrict__ image) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pix) return;
  const double a0 = pix[p], a1 = pix[p + pix_ld], a2 = pix[p + 2 * pix_ld];
  const double s0 = frame_coord(g, 0, a0, a1, a2), s1 = frame_coord(g, 1, a0, a1, a2),
               s2 = frame_coord(g, 2, a0, a1, a2);
  float k0[W], k1[W], k2[W];
  int i0[W], i1[W], i2[W];
  kernel_row<W>((s0 - g.D[0]) * g.hM[0], g.M[0], g.beta, k0, i0);
  kernel_row<W>((s1 - g.D[1]) * g.hM[1], g.M[1], g.beta, k1, i1);
  kernel_row<W>((s2 - g.D[2]) * g.hM[2], g.M[2], g.beta, k2, i2);
  // window offsets; points outside the windows (pixels other than the ones
  // planned for) contribute nothing
  int w0[W], w1[W], w2[W];
#pragma unroll
  for (int t = 0; t < W; ++t) {
    w0[t] = i0[t] - lay.lo0;
    if (w0[t] < 0) w0[t] += g.M[0];
    w1[t] = i1[t] - g.win_lo[1];
    if (w1[t] < 0) w1[t] += g.M[1];
    w2[t] = i2[t] - g.win_lo[2];
    if (w2[t] < 0) w2[t] += g.M[2];
  }
  float fr = 0.0f, fi = 0.0f;
#pragma unroll
  for (int c = 0; c < W; ++c) {
    if (w1[c] >= g.win_len[1]) continue;
#pragma unroll
    for (int e = 0; e < W; ++e) {
      if (w2[e] >= g.win_len[2]) continue;
      const int64_t base = (int64_t)w1[c] * lay.s1 + (int64_t)w2[e] * lay.s2;
      float sr = 0.0f, si = 0.0f;
#pragma unroll
      for (int a = 0; a < W; ++a)
        if (w0[a] < lay.len0) {
          sr += u[2 * (base + w0[a])] * k0[a];
          if (SHIFT) si += u[2 * (base + w0[a]) + 1] * k0[a];
        }
      fr += sr * k1[c] * k2[e];
      if (SHIFT) fi += si * k1[c] * k2[e];
    }
  }
  // the image is 2 Re(.); a uvw cell's sources were shifted by C, which the
  // factor exp(2 pi i <s, C>) restores (turns reduced exactly in FP64)
  double val = fr;
  if (SHIFT) {
    const double t = s0 * g.C[0] + s1 * g.C[1] + s2 * g.C[2];
    const float f = (float)(t - rint(t));
    val = (double)fr * (double)__builtin_amdgcn_cosf(f) - (double)fi * (double)__builtin_amdgcn_sinf(f);
  }
  image[p] += (float)(2.0 * val * corr[p] + (g.use_diag ? diag[lv] : 0.0));
}

// Per-pixel correction 1 / prod_d (phi_hat_d(2 pi s_d) / h_d), by quadrature:
// phi_hat(k) = a sum_j w_j phi(t_j) cos(k a t_j), a = w h / 2.
__global__ __launch_bounds__(256) void nufft_corr_kernel(NufftGeom g, const double* __restrict__ pix, int64_t pix_ld,
                                                         int64_t n_pix, const double* __restrict__ quad_t,
                                                         const double* __restrict__ quad_wphi, int n_quad,
                                                         double* __restrict__ corr) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pix) return;
  const double a0 = pix[p], a1 = pix[p + pix_ld], a2 = pix[p + 2 * pix_ld];
  double prod = 1.0;
  for (int d = 0; d < 3; ++d) {
    const double s = frame_coord(g, d, a0, a1, a2) - g.D[d];
    const double a = 0.5 * g.w * g.h[d];
    const double k = 2.0 * M_PI * s;
    double acc = 0.0;
    for (int j = 0; j < n_quad; ++j) acc += quad_wphi[j] * cos(k * a * quad_t[j]);
    prod *= a * acc / g.h[d];
  }
  corr[p] = 1.0 / prod;
}

__global__ __launch_bounds__(256) void fill_zero_f64_kernel(double* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// ---------------------------------------------------------------------------
hipError_t launch_nufft_prep(const NufftInst* insts, int n_inst, const void* W, const float* d, const int* lev,
                             int n_levels, int* order, int* lstart, double* diag, int* err, hipStream_t s) {
  hipLaunchKernelGGL(nufft_prep_kernel, dim3(n_inst), dim3(256), 0, s, insts, (const float2*)W, d, lev, n_levels,
                     order, lstart, diag, err);
  return hipGetLastError();
}

hipError_t launch_nufft_spread(const NufftGeom& g, const NufftInst* insts, int n_inst, int max_ant,
                               const double* ant, int64_t ant_ld, const void* Wmat, const float* d, const int* order,
                               const int* lstart, int n_levels, float* grid, int64_t n_cell, int* err, hipStream_t s) {
  const int64_t pairs = (int64_t)max_ant * max_ant;
  const dim3 grd((unsigned)((pairs + 255) / 256), (unsigned)n_inst);
  const float2* Wc = static_cast<const float2*>(Wmat);
  return with_width(g.w, [&](auto wc) {
    constexpr int KW = decltype(wc)::value;
    hipLaunchKernelGGL(nufft_spread_kernel<KW>, grd, dim3(256), 0, s, g, insts, ant, ant_ld, Wc, d, order, lstart,
                       n_levels, grid, n_cell, err);
    return hipGetLastError();
  });
}

hipError_t launch_nufft_vprime(const NufftInst* insts, int n_inst, int max_ant, const void* Wmat, const float* d,
                               const int* order, const int* lstart, int n_levels, void* vp, hipStream_t s) {
  const int nb = (max_ant + 31) / 32;
  hipLaunchKernelGGL(nufft_vprime_kernel, dim3((unsigned)(nb * (nb + 1) / 2), (unsigned)n_inst), dim3(256), 0, s,
                     insts, static_cast<const float2*>(Wmat), d, order, lstart, n_levels, static_cast<float2*>(vp));
  return hipGetLastError();
}

constexpr int kNufftChunk = 2048;  // candidate baselines per workgroup of the tiled spread

int nufft_tile_size(const NufftGeom& g) {
  for (int b : {16, 8})
    if ((int64_t)b * b * g.N[2] * 8 <= 65536) return b;
  return 0;  // too thick along axis 2 for an LDS tile: spread with global atomics
}

int scan_tmp_ints(int n) { return 2 * ((n + kScanChunk - 1) / kScanChunk) + 2; }

hipError_t launch_scan_i32(const int* count, int n, int* offset, int* cursor, int* tmp, hipStream_t s) {
  if (n <= 1 << 16 || !tmp) {
    hipLaunchKernelGGL(nufft_scan_kernel, dim3(1), dim3(1024), 0, s, count, n, offset, cursor);
    return hipGetLastError();
  }
  const int nc = (n + kScanChunk - 1) / kScanChunk;
  int* sums = tmp;
  int* chunk_off = tmp + nc;  // nc + 1 entries
  hipLaunchKernelGGL(scan_chunk_sums_kernel, dim3((unsigned)nc), dim3(1024), 0, s, count, n, sums);
  hipLaunchKernelGGL(nufft_scan_kernel, dim3(1), dim3(1024), 0, s, sums, nc, chunk_off, static_cast<int*>(nullptr));
  hipLaunchKernelGGL(scan_chunks_kernel, dim3((unsigned)nc), dim3(1024), 0, s, count, n, chunk_off, offset, cursor);
  return hipGetLastError();
}

hipError_t launch_nufft_bin(const NufftGeom& g, const NufftInst* insts, int n_inst, int max_ant, const double* ant,
                            int64_t ld, int bin, int* count, int* offset, int* cursor, uint64_t* list, int* err,
                            int* scan_tmp, hipStream_t s) {
  const int nb0 = (g.N[0] + bin - 1) / bin, nb1 = (g.N[1] + bin - 1) / bin;
  const int n_bins = nb0 * nb1;
  const int64_t pairs = (int64_t)max_ant * max_ant;
  const dim3 grd((unsigned)((pairs + 255) / 256), (unsigned)n_inst);
  hipError_t e = launch_fill_zero(reinterpret_cast<float*>(count), n_bins, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(nufft_bin_kernel, grd, dim3(256), 0, s, g, insts, ant, ld, bin, nb1, 0, count, list, err);
  e = launch_scan_i32(count, n_bins, offset, cursor, scan_tmp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(nufft_bin_kernel, grd, dim3(256), 0, s, g, insts, ant, ld, bin, nb1, 1, cursor, list, err);
  return hipGetLastError();
}

hipError_t launch_nufft_spread_tiles(const NufftGeom& g, const NufftInst* insts, const double* ant, int64_t ld,
                                     const void* vp, const int* offset, const uint64_t* list, int bin, int n_levels,
                                     int* nch, int* choff, float* grid, int64_t n_cell, hipStream_t s) {
  const int nb0 = (g.N[0] + bin - 1) / bin, nb1 = (g.N[1] + bin - 1) / bin;
  const int n_tiles = nb0 * nb1;
  const int chunk = kNufftChunk;
  hipLaunchKernelGGL(nufft_tile_chunks_kernel, dim3((unsigned)((n_tiles + 255) / 256)), dim3(256), 0, s, g, offset,
                     bin, nb0, nb1, chunk, nch);
  // exclusive offsets of the chunks (the scan's cursor output may overwrite nch: each
  // entry is read before it is written, and nch is not needed afterwards)
  hipLaunchKernelGGL(nufft_scan_kernel, dim3(1), dim3(1024), 0, s, nch, n_tiles, choff, nch);
  const size_t lds = (size_t)bin * bin * g.N[2] * sizeof(float2);
  const dim3 grd(4096u, (unsigned)n_levels);
  return with_width(g.w, [&](auto wc) {
    constexpr int KW = decltype(wc)::value;
    hipLaunchKernelGGL(nufft_spread_tile_kernel<KW>, grd, dim3(256), lds, s, g, insts, ant, ld,
                       static_cast<const float2*>(vp), offset, list, bin, nb0, nb1, chunk, choff, grid, n_cell);
    return hipGetLastError();
  });
}

static unsigned grid_blocks(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 65536); }

// Image-domain partitions: the pixels of one partition gathered into their own
// column-major array, and its level images added into the plan's images (each
// pixel belongs to one partition) and cleared.
__global__ __launch_bounds__(256) void nufft_gather_pix_kernel(const double* __restrict__ pix, int64_t ld,
                                                               const int64_t* __restrict__ idx, int64_t n,
                                                               double* __restrict__ out) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx[p];
#pragma unroll
    for (int d = 0; d < 3; ++d) out[p + d * n] = pix[i + d * ld];
  }
}

__global__ __launch_bounds__(256) void nufft_scatter_images_kernel(float* __restrict__ part_img, int64_t n,
                                                                   int n_levels, const int64_t* __restrict__ idx,
                                                                   float* __restrict__ images, int64_t ld) {
  const int64_t total = n * n_levels;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = e / n, p = e - l * n;
    images[l * ld + idx[p]] += part_img[e];
    part_img[e] = 0.0f;
  }
}

hipError_t launch_nufft_gather_pix(const double* pix, int64_t ld, const int64_t* idx, int64_t n, double* out,
                                   hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(nufft_gather_pix_kernel, dim3(grid_blocks(n)), dim3(256), 0, s, pix, ld, idx, n, out);
  return hipGetLastError();
}

hipError_t launch_nufft_scatter_images(float* part_img, int64_t n, int n_levels, const int64_t* idx, float* images,
                                       int64_t ld, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(nufft_scatter_images_kernel, dim3(grid_blocks(n * n_levels)), dim3(256), 0, s, part_img, n,
                     n_levels, idx, images, ld);
  return hipGetLastError();
}

hipError_t launch_nufft_gather(int axis, const NufftGeom& g, const void* src, const float* inv_psi, void* dst,
                               hipStream_t s) {
  if (axis == 2) {
    const int64_t n = (int64_t)g.N[0] * g.N[1] * g.M[2];
    hipLaunchKernelGGL(nufft_gather_a_kernel, dim3(grid_blocks(n)), dim3(256), 0, s, g,
                       static_cast<const float2*>(src), inv_psi, static_cast<float2*>(dst), n);
  } else if (axis == 1) {
    const int64_t n = (int64_t)g.N[0] * g.win_len[2] * g.M[1];
    hipLaunchKernelGGL(nufft_gather_b_kernel, dim3(grid_blocks(n)), dim3(256), 0, s, g,
                       static_cast<const float2*>(src), inv_psi, static_cast<float2*>(dst), n);
  } else {
    const int64_t n = (int64_t)g.win_len[1] * g.win_len[2] * g.M[0];
    hipLaunchKernelGGL(nufft_gather_c_kernel, dim3(grid_blocks(n)), dim3(256), 0, s, g,
                       static_cast<const float2*>(src), inv_psi, static_cast<float2*>(dst), n);
  }
  return hipGetLastError();
}

hipError_t launch_nufft_interp(const NufftGeom& g, const InterpLayout& lay, const double* pix, int64_t pix_ld,
                               int64_t n_pix, const float* u, const double* corr, const double* diag, int lv,
                               float* image, hipStream_t s) {
  const dim3 grd((unsigned)((n_pix + 255) / 256));
  return with_width(g.w, [&](auto wc) {
    constexpr int KW = decltype(wc)::value;
    if (g.cell_q > 1)
      hipLaunchKernelGGL((nufft_interp_kernel<KW, true>), grd, dim3(256), 0, s, g, lay, pix, pix_ld, n_pix, u, corr,
                         diag, lv, image);
    else
      hipLaunchKernelGGL((nufft_interp_kernel<KW, false>), grd, dim3(256), 0, s, g, lay, pix, pix_ld, n_pix, u, corr,
                         diag, lv, image);
    return hipGetLastError();
  });
}

hipError_t launch_nufft_corr(const NufftGeom& g, const double* pix, int64_t pix_ld, int64_t n_pix, const double* quad_t,
                             const double* quad_wphi, int n_quad, double* corr, hipStream_t s) {
  hipLaunchKernelGGL(nufft_corr_kernel, dim3((unsigned)((n_pix + 255) / 256)), dim3(256), 0, s, g, pix, pix_ld, n_pix,
                     quad_t, quad_wphi, n_quad, corr);
  return hipGetLastError();
}

hipError_t launch_fill_zero_f64(double* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(fill_zero_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace bb
