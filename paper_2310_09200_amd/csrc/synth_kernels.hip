// Staging and fused standard-synthesis kernels for gfx950 (CDNA4).
//
// Per (time step, channel) instance the image of each energy level is
//     I_l(p) += sum_{k in l} d_k |E_kp|^2,   E = W^H B,   B_lp = exp(+j 2 pi <x_l, p> / lambda_w)
// (standard synthesis, Section 2.4; levels and filters, Section 2.6 and
// Algorithm 1).  The complex product is done as a real GEMM on the embedding
//     [Er; Ei] = [[Wr^T, Wi^T], [-Wi^T, Wr^T]] [Br; Bi]
// with antennas interleaved (re, im) along the contraction axis.
//
// Kernel structure (one workgroup = one pixel tile of one image slot):
//   for each instance of the slot (its scaled positions copied to LDS once),
//   for each K pass, for each 32-antenna chunk:
//     MFMA: real-embedded W^H operand streamed from HBM/L2 in operand order
//       and prefetched one MFMA group ahead, B operand from LDS, accumulators
//       for [Er; Ei] in registers
//     phase generation of the next chunk, a slice per MFMA group: FP64
//       <x_l, p> in turns, exact FP64 reduction to [-1/2, 1/2], hardware FP32
//       sin/cos in turns -> the other B buffer in LDS (double-buffered)
//   epilogue of a pass: d_k (Er^2 + Ei^2) reduced over k in-lane, across the
//     two half-waves, and into per-level partial sums in LDS
//   end of the tile: sum over waves in a fixed order, one read-modify-write of
//     the images (one writer per pixel and launch: deterministic, no atomics).
// Neither B (L x N_pix) nor E (K x N_pix) is ever written to HBM.
// synth_fwd16_kernel is the same structure for the three-product FP32 form on
// 16-row eigenpair blocks (16x16x4 MFMAs), for instances with few eigenpairs.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "bb_internal.h"

namespace bb {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Pointers read out of an instance descriptor are generic to the compiler, and
// generic (flat) loads count against the LDS wait counter too, so every wait
// for an LDS read would also wait for the prefetched W operand.  Casting them
// to the global address space makes those loads vector-memory loads only.
#define BB_GLOBAL __attribute__((address_space(1)))
#define BB_LDS __attribute__((address_space(3)))
template <class T>
__device__ __forceinline__ const BB_GLOBAL T* as_global(const void* p) {
  return (const BB_GLOBAL T*)p;
}

// Phase of one (antenna, pixel) pair: xs = position / wavelength, so t is the
// phase in turns.  The reduction t - rint(t) is exact in FP64 and leaves
// f in [-1/2, 1/2]; gfx950's transcendental unit takes its sine and cosine
// argument in turns (sin(2 pi f)), with an absolute error near 1.3e-7 there.
// xs points into the workgroup's LDS copy of the instance's positions.
__device__ __forceinline__ void phase_pair(const BB_LDS double* __restrict__ xs, double px, double py, double pz,
                                           float& c, float& s) {
  const double t = fma(xs[2], pz, fma(xs[1], py, xs[0] * px));
  const float f = (float)(t - rint(t));
  s = __builtin_amdgcn_sinf(f);
  c = __builtin_amdgcn_cosf(f);
}

// ---------------------------------------------------------------------------
// Staging, part 1 (one workgroup per instance): sort eigenpairs by level
// (stable, dropping level -1), scaled positions, per-32-block level ranges.
__global__ __launch_bounds__(256) void stage_meta_kernel(const InstDesc* __restrict__ descs,
                                                         InstDyn* __restrict__ dyn, int n_levels,
                                                         int* __restrict__ err) {
  const InstDesc D = descs[blockIdx.x];
  __shared__ int s_lev[kMaxEig];
  __shared__ int s_cnt[kMaxLevels + 1];
  __shared__ int s_base[kMaxLevels + 1];
  const int tid = threadIdx.x;
  if (tid <= kMaxLevels) s_cnt[tid] = 0;
  __syncthreads();
  for (int k = tid; k < D.K; k += blockDim.x) {
    int lv = D.lev_in[k];
    if (lv < -1 || lv >= n_levels) {
      atomicOr(err, kErrLevelId);
      lv = -1;
    }
    s_lev[k] = lv;
    if (lv >= 0) atomicAdd(&s_cnt[lv], 1);
  }
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int l = 0; l < n_levels; ++l) {
      s_base[l] = acc;
      acc += s_cnt[l];
    }
    s_base[n_levels] = acc;
    InstDyn o;
    o.K_eff = acc;
    o.K_pad = round_up(acc, 32);
    dyn[blockIdx.x] = o;
  }
  __syncthreads();
  const int K_eff = s_base[n_levels];
  for (int k = tid; k < D.K; k += blockDim.x) {
    const int lv = s_lev[k];
    if (lv < 0) continue;
    int r = 0;
    for (int j = 0; j < k; ++j) r += (s_lev[j] == lv);
    const int pos = s_base[lv] + r;
    D.perm[pos] = k;
    D.wts[pos] = D.d[k];
    D.levs[pos] = lv;
  }
  for (int pos = K_eff + tid; pos < D.K_alloc; pos += blockDim.x) {
    D.perm[pos] = -1;
    D.wts[pos] = 0.0f;
    D.levs[pos] = -1;
  }
  __syncthreads();
  // level range of each 32-block, then of each 16-block, of sorted positions
  // (levels are non-decreasing; (1, 0) for a block with no kept eigenpair)
  const int nb32 = D.K_alloc / 32;
  for (int i = tid; i < nb32 + D.K_alloc / 16; i += blockDim.x) {
    const int rows = i < nb32 ? 32 : 16;
    const int p0 = (i < nb32 ? i : i - nb32) * rows;
    int lo = 1, hi = 0;
    if (p0 < K_eff) {
      const int p1 = min(p0 + rows - 1, K_eff - 1);
      // sorted positions: find their levels through the base offsets
      int l0 = 0, l1 = 0;
      for (int l = 0; l < n_levels; ++l) {
        if (s_base[l] <= p0 && p0 < s_base[l + 1]) l0 = l;
        if (s_base[l] <= p1 && p1 < s_base[l + 1]) l1 = l;
      }
      lo = l0;
      hi = l1;
    }
    D.kbr[i] = make_int2(lo, hi);
  }
  for (int l = tid; l < D.L_pad; l += blockDim.x) {
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;
    if (l < D.L) {
      v0 = D.ant[l] * D.scale;
      v1 = D.ant[l + D.ant_ld] * D.scale;
      v2 = D.ant[l + 2 * D.ant_ld] * D.scale;
    }
    D.xs[4 * l + 0] = v0;
    D.xs[4 * l + 1] = v1;
    D.xs[4 * l + 2] = v2;
    D.xs[4 * l + 3] = 0.0;
  }
}

__device__ __forceinline__ void load_w(const InstDesc& D, int l, int col, float& wr, float& wi) {
  if (D.W_c128) {
    const double* w = (const double*)D.W + 2 * ((int64_t)col * D.W_ld + l);
    wr = (float)w[0];
    wi = (float)w[1];
  } else {
    const float* w = (const float*)D.W + 2 * ((int64_t)col * D.W_ld + l);
    wr = w[0];
    wi = w[1];
  }
}

// Staging, part 2, FP32: one float4 = 4 consecutive antennas of one lane of
// one MFMA A-operand fragment (32x32x2: lane = row + 32 * (re/im)).
__global__ __launch_bounds__(256) void stage_pack_f32_kernel(const InstDesc* __restrict__ descs) {
  const InstDesc D = descs[blockIdx.y];
  const int G4 = D.L_pad / 4;
  const int64_t total = (int64_t)(D.K_alloc / 32) * 2 * G4 * 64;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int lane = (int)(idx % 64);
  int64_t rest = idx / 64;
  const int g = (int)(rest % G4);
  rest /= G4;
  const int ri = (int)(rest % 2);
  const int kb = (int)(rest / 2);
  const int k = kb * 32 + (lane & 31);
  const int h = lane >> 5;
  const int src = D.perm[k];
  f32x4 out;
  for (int s = 0; s < 4; ++s) {
    const int l = 4 * g + s;
    float wr = 0.0f, wi = 0.0f;
    if (src >= 0 && l < D.L) load_w(D, l, D.wcol ? D.wcol[src] : src, wr, wi);
    // Er row: (Wr, Wi) pairs with (Br, Bi); Ei row: (-Wi, Wr)
    out[s] = ri == 0 ? (h == 0 ? wr : wi) : (h == 0 ? -wi : wr);
  }
  ((f32x4*)D.apack)[idx] = out;
}

// Staging, part 2, BF16 x3: hi = bf16(a), lo = bf16(a - hi) of the real
// embedding, 8 contraction rows per lane (32x32x16: lane = row + 32 * (k / 8)).
__global__ __launch_bounds__(256) void stage_pack_bf16_kernel(const InstDesc* __restrict__ descs) {
  const InstDesc D = descs[blockIdx.y];
  const int G8 = D.L_pad / 8;
  const int64_t total = (int64_t)(D.K_alloc / 32) * 2 * G8 * 64;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int lane = (int)(idx % 64);
  int64_t rest = idx / 64;
  const int g = (int)(rest % G8);
  rest /= G8;
  const int ri = (int)(rest % 2);
  const int kb = (int)(rest / 2);
  const int k = kb * 32 + (lane & 31);
  const int h = lane >> 5;
  const int src = D.perm[k];
  bf16x8 hi, lo;
  for (int a = 0; a < 4; ++a) {
    const int l = 8 * g + 4 * h + a;
    float wr = 0.0f, wi = 0.0f;
    if (src >= 0 && l < D.L) load_w(D, l, D.wcol ? D.wcol[src] : src, wr, wi);
    const float v0 = ri == 0 ? wr : -wi;  // multiplies Br
    const float v1 = ri == 0 ? wi : wr;   // multiplies Bi
    const __bf16 h0 = (__bf16)v0, h1 = (__bf16)v1;
    hi[2 * a] = h0;
    hi[2 * a + 1] = h1;
    lo[2 * a] = (__bf16)(v0 - (float)h0);
    lo[2 * a + 1] = (__bf16)(v1 - (float)h1);
  }
  const int64_t base = (((int64_t)(kb * 2 + ri) * G8 + g) * 2) * 64 + lane;
  ((bf16x8*)D.apack)[base] = hi;
  ((bf16x8*)D.apack)[base + 64] = lo;
}

// Staging, part 2, FP32 with three real products per complex product (Gauss):
// conj(W) B = (k1 - k3) + j (k1 + k2) with k1 = (Wr - Wi) Br, k2 = Wr (Bi - Br),
// k3 = -Wi (Br + Bi).  Three planes (Wr - Wi, Wr, -Wi), 12 bytes per
// (eigenpair, antenna) in either operand order:
//  - 32-row blocks (32x32x2 operands, the two contraction rows of an MFMA step
//    being two antennas): lane = row + 32 * (antenna parity), float4 = 4 steps
//    = 8 antennas, vectors ordered (32-block, plane, 8-antenna group, lane);
//  - 16-row blocks (16x16x4 operands, four antennas per step): lane = row +
//    16 * (antenna mod 4), float2 = 2 steps = 8 antennas, vectors ordered
//    (16-block, 8-antenna group, plane, lane).
__global__ __launch_bounds__(256) void stage_pack_f32g_kernel(const InstDesc* __restrict__ descs) {
  const InstDesc D = descs[blockIdx.y];
  const int64_t total = (int64_t)D.K_alloc * 3 * D.L_pad / 4;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int lane = (int)(idx % 64);
  int64_t rest = idx / 64;
  if (D.rows16) {  // two float2 vectors: 8-antenna groups 2 gg and 2 gg + 1
    const int q = (int)(rest % 3);
    rest /= 3;
    const int G16 = D.L_pad / 16;
    const int gg = (int)(rest % G16);
    const int blk = (int)(rest / G16);
    const int k = blk * 16 + (lane & 15);
    const int src = D.perm[k];
    for (int h = 0; h < 2; ++h) {
      const int g8 = 2 * gg + h;
      f32x2 out;
      for (int s = 0; s < 2; ++s) {
        const int l = 8 * g8 + 4 * s + (lane >> 4);
        float wr = 0.0f, wi = 0.0f;
        if (src >= 0 && l < D.L) load_w(D, l, D.wcol ? D.wcol[src] : src, wr, wi);
        out[s] = q == 0 ? wr - wi : (q == 1 ? wr : -wi);
      }
      ((f32x2*)D.apack)[(((int64_t)blk * (D.L_pad / 8) + g8) * 3 + q) * 64 + lane] = out;
    }
    return;
  }
  const int G8 = D.L_pad / 8;
  const int g = (int)(rest % G8);
  rest /= G8;
  const int q = (int)(rest % 3);
  const int kb = (int)(rest / 3);
  const int k = kb * 32 + (lane & 31);
  const int src = D.perm[k];
  f32x4 out;
  for (int s = 0; s < 4; ++s) {
    const int l = 8 * g + 2 * s + (lane >> 5);
    float wr = 0.0f, wi = 0.0f;
    if (src >= 0 && l < D.L) load_w(D, l, D.wcol ? D.wcol[src] : src, wr, wi);
    out[s] = q == 0 ? wr - wi : (q == 1 ? wr : -wi);
  }
  ((f32x4*)D.apack)[idx] = out;
}

// Staging, part 2, BF16 x3 with three real products per complex product: the
// three planes of the FP32 three-product form, each split hi = bf16(a),
// lo = bf16(a - hi); 32x32x16 operand order with the 16 contraction rows of an
// MFMA step being 16 antennas: lane = row + 32 * (antenna / 8), 8 antennas per lane.
__global__ __launch_bounds__(256) void stage_pack_bf16g_kernel(const InstDesc* __restrict__ descs) {
  const InstDesc D = descs[blockIdx.y];
  const int G16 = D.L_pad / 16;
  const int64_t total = (int64_t)(D.K_alloc / 32) * 3 * G16 * 64;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int lane = (int)(idx % 64);
  int64_t rest = idx / 64;
  const int g = (int)(rest % G16);
  rest /= G16;
  const int q = (int)(rest % 3);
  const int kb = (int)(rest / 3);
  const int k = kb * 32 + (lane & 31);
  const int h = lane >> 5;
  const int src = D.perm[k];
  bf16x8 hi, lo;
  for (int e = 0; e < 8; ++e) {
    const int l = 16 * g + 8 * h + e;
    float wr = 0.0f, wi = 0.0f;
    if (src >= 0 && l < D.L) load_w(D, l, D.wcol ? D.wcol[src] : src, wr, wi);
    const float v = q == 0 ? wr - wi : (q == 1 ? wr : -wi);
    const __bf16 vh = (__bf16)v;
    hi[e] = vh;
    lo[e] = (__bf16)(v - (float)vh);
  }
  const int64_t base = (((int64_t)(kb * 3 + q) * G16 + g) * 2) * 64 + lane;
  ((bf16x8*)D.apack)[base] = hi;
  ((bf16x8*)D.apack)[base + 64] = lo;
}

hipError_t launch_stage(const InstDesc* d_descs, InstDyn* d_dyn, int n_inst, int max_K_alloc, int max_L_pad,
                        int n_levels, int precision, int* d_err, hipStream_t s) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(stage_meta_kernel, dim3(n_inst), dim3(256), 0, s, d_descs, d_dyn, n_levels, d_err);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t per = (int64_t)(max_K_alloc / 32) * 2 * (max_L_pad / 4) * 64;
  if (precision == 1) per = (int64_t)(max_K_alloc / 32) * 2 * (max_L_pad / 8) * 64;
  if (precision == 2) per = (int64_t)(max_K_alloc / 32) * 3 * (max_L_pad / 8) * 64;
  if (precision == 3) per = (int64_t)(max_K_alloc / 32) * 3 * (max_L_pad / 16) * 64;
  const unsigned gx = (unsigned)((per + 255) / 256);
  if (precision == 3)
    hipLaunchKernelGGL(stage_pack_bf16g_kernel, dim3(gx, n_inst), dim3(256), 0, s, d_descs);
  else if (precision == 1)
    hipLaunchKernelGGL(stage_pack_bf16_kernel, dim3(gx, n_inst), dim3(256), 0, s, d_descs);
  else if (precision == 2)
    hipLaunchKernelGGL(stage_pack_f32g_kernel, dim3(gx, n_inst), dim3(256), 0, s, d_descs);
  else
    hipLaunchKernelGGL(stage_pack_f32_kernel, dim3(gx, n_inst), dim3(256), 0, s, d_descs);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Synthesis kernel.
//   PREC:    0 = FP32, four real products per complex product (accumulators Er, Ei)
//            1 = BF16 x3 (hi/lo split, three bf16 MFMAs per real product; Er, Ei)
//            2 = FP32, three real products (Gauss; accumulators k1, k2, k3)
//            3 = BF16 x3 of the three-product form (k1, k2, k3)
//   MB x NB: 32x32 output blocks per wave (k-blocks x pixel blocks);
//   WK x WN: waves along k and along pixels.
template <int MB, int NB, int WK, int WN>
struct TileCfg {
  static constexpr int ROWS = 32;
  static constexpr int WAVES = WK * WN;
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int KC = 32 * MB * WK;      // eigenpairs per pass
  static constexpr int NT = 32 * NB * WN;      // pixels per tile
  static constexpr int NCB = NT / 32;
  static constexpr int LCH = NT <= 128 ? 32 : 16;  // antennas per LDS chunk
  static constexpr int G4 = LCH / 4;
  static constexpr int G8 = LCH / 8;
  static constexpr int G16 = LCH / 16;
  static constexpr int CHUNK_VEC = LCH * NT / 2;   // 16-byte vectors per chunk buffer
  static constexpr int TASKS = NT * G4;           // (pixel, 4-antenna) phase tasks per chunk
  static constexpr int JT = (TASKS + THREADS - 1) / THREADS;
  static_assert(THREADS % NT == 0, "a thread keeps one pixel");
  static_assert(TASKS % THREADS == 0, "task split");
  static_assert(kAntChunk % LCH == 0, "antenna padding covers the chunk");
};

template <int PREC>
struct Acc {
  static constexpr int N = PREC >= 2 ? 3 : 2;  // accumulator tiles per output block
};

template <class C, int PREC>
struct ChunkVec {  // 16-byte vectors per LDS phase chunk
  static constexpr int N = PREC >= 2 ? 3 * C::LCH * C::NT / 4 : C::CHUNK_VEC;
};

// A thread's share of a phase chunk: JT tasks of 4 (antenna, pixel) pairs, one
// pixel per task.  The pairs of a task are laid out so that each task fills
// whole 16-byte vectors of the chunk's MFMA operand layout.
template <class C>
__device__ __forceinline__ int gen_group(int tid, int j) {  // antenna group of task j
  const int t = tid + j * C::THREADS;
  // wave-uniform when a wave's 64 lanes share one antenna group
  return C::NT % 64 == 0 ? __builtin_amdgcn_readfirstlane(t / C::NT) : t / C::NT;
}

// Antenna (within the chunk) of pair s of a task in antenna group g4.
template <int PREC>
__device__ __forceinline__ int gen_antenna(int g4, int s) {
  if (PREC == 3) {
    // lane (h, jj) of a plane holds antennas 16 g16 + 8 h + e, e = 0..7; a task
    // fills e = 4 half .. 4 half + 3 (8 bytes of each 16-byte operand)
    const int g16 = g4 >> 2, h = (g4 >> 1) & 1, half = g4 & 1;
    return 16 * g16 + 8 * h + 4 * half + s;
  }
  if (PREC == 2) return 8 * (g4 >> 1) + 2 * s + (g4 & 1);  // one lane of each of the three B planes
  return 4 * g4 + s;
}

// Phase pairs first .. first + count - 1 (pair q = pair q % 4 of task q / 4) of
// this thread's share of a chunk, into registers.
template <class C, int PREC>
__device__ __forceinline__ void gen_pairs(float (&cr)[4 * C::JT], float (&ci)[4 * C::JT],
                                          const BB_LDS double* __restrict__ xs_chunk, double px, double py,
                                          double pz, int tid, int first, int count) {
#pragma unroll
  for (int q = 0; q < 4 * C::JT; ++q)
    if (q >= first && q < first + count)
      phase_pair(xs_chunk + 4 * gen_antenna<PREC>(gen_group<C>(tid, q >> 2), q & 3), px, py, pz, cr[q], ci[q]);
}

// This thread's share of a chunk from its phase pairs into the LDS operand
// layout of the precision: (Br, Bi) vectors (FP32), interleaved BF16 hi / lo
// vectors (BF16 x3), or the three planes Br, Bi - Br, Br + Bi (three products).
template <class C, int PREC>
__device__ __forceinline__ void gen_store(f32x4* __restrict__ buf, const float (&pr)[4 * C::JT],
                                          const float (&pi)[4 * C::JT], int tid) {
  static_assert(C::TASKS % C::THREADS == 0, "whole tasks per thread");
#pragma unroll
  for (int j = 0; j < C::JT; ++j) {
    const int pl = (tid + j * C::THREADS) % C::NT;
    const int g4 = gen_group<C>(tid, j);
    const int cb = pl >> 5, jj = pl & 31;
    const float* cr = pr + 4 * j;
    const float* ci = pi + 4 * j;
    if (PREC == 3) {
      const int g16 = g4 >> 2, h = (g4 >> 1) & 1, half = g4 & 1;
      bf16x4* b4 = (bf16x4*)buf;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        bf16x4 hi, lo;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const float v = q == 0 ? cr[s] : (q == 1 ? ci[s] - cr[s] : cr[s] + ci[s]);
          const __bf16 vh = (__bf16)v;
          hi[s] = vh;
          lo[s] = (__bf16)(v - (float)vh);
        }
        const int o = ((((g16 * 3 + q) * C::NCB + cb) * 2) * 64 + h * 32 + jj) * 2 + half;
        b4[o] = hi;
        b4[o + 128] = lo;
      }
    } else if (PREC == 2) {
      const int g8 = g4 >> 1, h = g4 & 1;
      f32x4 vr = {cr[0], cr[1], cr[2], cr[3]};
      f32x4 vd = {ci[0] - cr[0], ci[1] - cr[1], ci[2] - cr[2], ci[3] - cr[3]};
      f32x4 vs = {cr[0] + ci[0], cr[1] + ci[1], cr[2] + ci[2], cr[3] + ci[3]};
      buf[((g8 * 3 + 0) * C::NCB + cb) * 64 + h * 32 + jj] = vr;
      buf[((g8 * 3 + 1) * C::NCB + cb) * 64 + h * 32 + jj] = vd;
      buf[((g8 * 3 + 2) * C::NCB + cb) * 64 + h * 32 + jj] = vs;
    } else if (PREC == 0) {
      f32x4 vr = {cr[0], cr[1], cr[2], cr[3]};
      f32x4 vi = {ci[0], ci[1], ci[2], ci[3]};
      buf[(g4 * C::NCB + cb) * 64 + jj] = vr;
      buf[(g4 * C::NCB + cb) * 64 + 32 + jj] = vi;
    } else {
      bf16x8 hi, lo;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const __bf16 hr = (__bf16)cr[s], hiv = (__bf16)ci[s];
        hi[2 * s] = hr;
        hi[2 * s + 1] = hiv;
        lo[2 * s] = (__bf16)(cr[s] - (float)hr);
        lo[2 * s + 1] = (__bf16)(ci[s] - (float)hiv);
      }
      const int g8 = g4 >> 1, h = g4 & 1;
      bf16x8* b16 = (bf16x8*)buf;
      b16[((g8 * C::NCB + cb) * 2 + 0) * 64 + h * 32 + jj] = hi;
      b16[((g8 * C::NCB + cb) * 2 + 1) * 64 + h * 32 + jj] = lo;
    }
  }
}

template <class C, int PREC>
__device__ __forceinline__ void gen_chunk(f32x4* __restrict__ buf, const BB_LDS double* __restrict__ xs_chunk,
                                          double px, double py, double pz, int tid) {
  float cr[4 * C::JT], ci[4 * C::JT];
  gen_pairs<C, PREC>(cr, ci, xs_chunk, px, py, pz, tid, 0, 4 * C::JT);
  gen_store<C, PREC>(buf, cr, ci, tid);
}

// A operand (the W^H side) of one MFMA group: 4 contraction steps of the
// wave's k-block.  It is loaded from L2 / HBM one group ahead of its use, so
// the load latency is covered by the previous group's MFMAs.
template <int PREC>
struct AFrag;
template <>
struct AFrag<0> {  // Er / Ei rows, 4 antennas
  f32x4 v[2];
};
template <>
struct AFrag<1> {  // Er / Ei rows, hi / lo, 8 antennas
  bf16x8 h[2], l[2];
};
template <>
struct AFrag<2> {  // three planes, 8 antennas
  f32x4 v[3];
};
template <>
struct AFrag<3> {  // three planes, hi / lo, 16 antennas
  bf16x8 h[3], l[3];
};

template <class C, int PREC>
struct NGroups {  // MFMA groups per LDS chunk
  static constexpr int N = PREC == 0 ? C::G4 : (PREC == 3 ? C::G16 : C::G8);
};

// base: first vector of this wave's k-block; stride: vectors per row tile (PREC 0/1)
// or per plane (PREC 2/3); group g of chunk c.
template <class C, int PREC>
__device__ __forceinline__ void load_a(AFrag<PREC>& a, const void* apack, int64_t base, int64_t stride,
                                       int c, int g, int lane) {
  if constexpr (PREC == 0) {
    const BB_GLOBAL f32x4* __restrict__ A = as_global<f32x4>(apack);
    const int64_t o = base + (int64_t)(c * C::G4 + g) * 64 + lane;
    a.v[0] = A[o];
    a.v[1] = A[o + stride];
  } else if constexpr (PREC == 1) {
    const BB_GLOBAL bf16x8* __restrict__ A = as_global<bf16x8>(apack);
    const int64_t o = base + (int64_t)(c * C::G8 + g) * 128 + lane;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      a.h[rt] = A[o + rt * stride];
      a.l[rt] = A[o + rt * stride + 64];
    }
  } else if constexpr (PREC == 2) {
    const BB_GLOBAL f32x4* __restrict__ A = as_global<f32x4>(apack);
    const int64_t o = base + (int64_t)(c * C::G8 + g) * 64 + lane;
#pragma unroll
    for (int q = 0; q < 3; ++q) a.v[q] = A[o + q * stride];
  } else {
    const BB_GLOBAL bf16x8* __restrict__ A = as_global<bf16x8>(apack);
    const int64_t o = base + (int64_t)(c * C::G16 + g) * 128 + lane;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      a.h[q] = A[o + q * stride];
      a.l[q] = A[o + q * stride + 64];
    }
  }
}

// MFMAs of group g of an LDS chunk for this wave's k-block and NB pixel blocks.
template <class C, int PREC, int NB>
__device__ __forceinline__ void mma_group(f32x16 (&acc)[Acc<PREC>::N][NB], const AFrag<PREC>& a,
                                          const f32x4* __restrict__ buf, int g, int cb0, int lane) {
  if constexpr (PREC == 0) {
    f32x4 b[NB];
#pragma unroll
    for (int n = 0; n < NB; ++n) b[n] = buf[(g * C::NCB + cb0 + n) * 64 + lane];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int n = 0; n < NB; ++n)
          acc[rt][n] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.v[rt][s], b[n][s], acc[rt][n], 0, 0, 0);
  } else if constexpr (PREC == 1) {
    const bf16x8* Bb = (const bf16x8*)buf;
    bf16x8 bh[NB], bl[NB];
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      const int o = ((g * C::NCB + cb0 + n) * 2) * 64 + lane;
      bh[n] = Bb[o];
      bl[n] = Bb[o + 64];
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int n = 0; n < NB; ++n) {
        acc[rt][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.l[rt], bh[n], acc[rt][n], 0, 0, 0);
        acc[rt][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.h[rt], bl[n], acc[rt][n], 0, 0, 0);
        acc[rt][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.h[rt], bh[n], acc[rt][n], 0, 0, 0);
      }
  } else if constexpr (PREC == 2) {
    // planes q = 0, 1, 2 pair with Br, Bi - Br, Br + Bi
    f32x4 b[3 * NB];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int n = 0; n < NB; ++n) b[3 * n + q] = buf[((g * 3 + q) * C::NCB + cb0 + n) * 64 + lane];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int n = 0; n < NB; ++n)
#pragma unroll
        for (int q = 0; q < 3; ++q)
          acc[q][n] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.v[q][s], b[3 * n + q][s], acc[q][n], 0, 0, 0);
  } else {
    const bf16x8* Bb = (const bf16x8*)buf;
    bf16x8 bh[3 * NB], bl[3 * NB];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int n = 0; n < NB; ++n) {
        const int o = (((g * 3 + q) * C::NCB + cb0 + n) * 2) * 64 + lane;
        bh[3 * n + q] = Bb[o];
        bl[3 * n + q] = Bb[o + 64];
      }
#pragma unroll
    for (int n = 0; n < NB; ++n)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        f32x16& c = acc[q][n];
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.l[q], bh[3 * n + q], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.h[q], bl[3 * n + q], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.h[q], bh[3 * n + q], c, 0, 0, 0);
      }
  }
}

// (Er, Ei) of accumulator register r of pixel block n.
template <int PREC, int NB>
__device__ __forceinline__ void fields(const f32x16 (&acc)[Acc<PREC>::N][NB], int n, int r, float& er, float& ei) {
  if constexpr (PREC >= 2) {
    er = acc[0][n][r] - acc[2][n][r];
    ei = acc[0][n][r] + acc[1][n][r];
  } else {
    er = acc[0][n][r];
    ei = acc[1][n][r];
  }
}

// MODE 0: level images (the product).  MODE 1: write E itself (two planes,
// re and im, [K_alloc][n_pix] each) for the backward pass; one instance only.
template <int MB, int NB, int WK, int WN, int PREC, int MODE>
__global__ __launch_bounds__(64 * WK * WN) void synth_fwd_kernel(const FwdParams P) {
  static_assert(MB == 1, "one k-block of 32 eigenpairs per wave");
  using C = TileCfg<MB, NB, WK, WN>;
  __shared__ f32x4 s_buf[2][ChunkVec<C, PREC>::N];
  constexpr int NA = Acc<PREC>::N;
  constexpr int NG = NGroups<C, PREC>::N;
  __shared__ float s_part[WK][kMaxLevels][C::NT];
  // scaled positions of the current instance, (x, y, z, 0) per antenna: every
  // phase chunk reads them from here (a broadcast LDS read per antenna) rather
  // than through L2, whose latency would otherwise open each chunk
  __shared__ __align__(16) double s_xs[4 * kMaxAnt];
  const BB_LDS double* const xs = (const BB_LDS double*)s_xs;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  // k-block of a wave = wave / WN: the waves of one SIMD (wave mod 4) cover the
  // k-blocks evenly, so an instance whose K fills only part of the tile leaves
  // no SIMD idle
  const int wk = wave / WN;
  const int wn = wave % WN;
  const int cb0 = wn * NB;
  const int n_levels = P.n_levels;
  // Phases of the next chunk are spread over the MFMA groups of the current
  // one.  A SIMD issues few vector instructions while another of its waves
  // streams MFMAs, so phases generated in one burst per chunk left the matrix
  // pipe idle at the chunk's barrier; in slices, each wave's phase work sits
  // between its own MFMA groups while the other wave keeps multiplying.
  constexpr int PPG = 4 * C::JT / NG;  // phase pairs per MFMA group
  static_assert(PPG * NG == 4 * C::JT, "pairs split evenly over the groups");

  // Persistent grid: workgroup b owns pixel tiles b, b + gridDim.x, ...; every
  // workgroup walks the groups (slots) and their instances in the same order,
  // so the workgroups running at one time stream the same instance's W operand
  // through L2.  Each image tile has exactly one writer (its owner).
  for (int grp = 0; grp < P.n_groups; ++grp) {
    const int slot = __builtin_amdgcn_readfirstlane(P.group_slot[grp]);
    for (int ii = P.group_begin[grp]; ii < P.group_begin[grp + 1]; ++ii) {
      // Instance fields are copied into (wave-uniform) locals once: read
      // through the descriptor pointer they would be reloaded after every LDS
      // store, which the compiler cannot prove does not alias them.
      const int inst = __builtin_amdgcn_readfirstlane(P.inst_list[ii]);
      const InstDesc& Dg = P.descs[inst];
      const void* const apack = Dg.apack;
      const BB_GLOBAL double* const xs_g = as_global<double>(Dg.xs);
      const BB_GLOBAL float* const wts = as_global<float>(Dg.wts);
      const BB_GLOBAL int* const levs = as_global<int>(Dg.levs);
      const BB_GLOBAL int* const kbr = as_global<int>(Dg.kbr);  // (lo, hi) pairs
      const int K_pad = __builtin_amdgcn_readfirstlane(P.dyn[inst].K_pad);
      const int L_pad = __builtin_amdgcn_readfirstlane(Dg.L_pad);
      const int n_chunks = L_pad / C::LCH;
      const int n_pass = (K_pad + C::KC - 1) / C::KC;
      // 16-byte vectors per A row tile (PREC 0/1) or per plane (PREC 2/3)
      const int64_t a_stride = PREC >= 2 ? (int64_t)(L_pad / 8) * 64 : (int64_t)(L_pad / 4) * 64;
      if (blockIdx.x < P.n_tiles) {  // workgroup-uniform: this workgroup owns a tile
        __syncthreads();  // the previous instance's phase chunks are done with s_xs
        for (int i = tid; i < 2 * L_pad; i += C::THREADS)
          ((f64x2*)s_xs)[i] = ((const BB_GLOBAL f64x2*)xs_g)[i];
        __syncthreads();
      }
      for (int64_t tile = blockIdx.x; tile < P.n_tiles; tile += gridDim.x) {
        const int64_t p0 = tile * C::NT;
        for (int i = tid; i < WK * kMaxLevels * C::NT; i += C::THREADS) (&s_part[0][0][0])[i] = 0.0f;
        // this thread's pixel (phase generation); clamp the ragged tail
        int64_t pg = p0 + (tid % C::NT);
        if (pg >= P.n_pix) pg = P.n_pix - 1;
        const double px = P.pix[pg], py = P.pix[pg + P.pix_ld], pz = P.pix[pg + 2 * P.pix_ld];
        for (int pass = 0; pass < n_pass; ++pass) {
          const int kb = pass * (C::KC / 32) + wk;   // this wave's k-block
          const bool active = kb < K_pad / 32;        // wave-uniform
          const int64_t a_base = (int64_t)kb * (PREC >= 2 ? 3 : 2) * a_stride;
          f32x16 acc[NA][NB];
#pragma unroll
          for (int t = 0; t < NA; ++t)
#pragma unroll
            for (int n = 0; n < NB; ++n)
#pragma unroll
              for (int r = 0; r < 16; ++r) acc[t][n][r] = 0.0f;
          AFrag<PREC> a_cur;
          if (active) load_a<C, PREC>(a_cur, apack, a_base, a_stride, 0, 0, lane);

          __syncthreads();  // previous users of s_buf are done
          gen_chunk<C, PREC>(s_buf[0], xs, px, py, pz, tid);
          __syncthreads();
          for (int c = 0; c < n_chunks; ++c) {
            // the last chunk regenerates itself into the idle buffer (read by
            // nobody), so that no branch splits the MFMA stream
            const int c_next = min(c + 1, n_chunks - 1);
            const BB_LDS double* const xs_next = xs + 4 * c_next * C::LCH;
            float cr[4 * C::JT], ci[4 * C::JT];
            if (active) {
              // FP32 three products: the second wave of each SIMD multiplies at a
              // higher priority, which staggers the two waves' phase slices
              if (PREC == 2 && wave >= C::WAVES / 2) __builtin_amdgcn_s_setprio(1);
#pragma unroll
              for (int g = 0; g < NG; ++g) {
                AFrag<PREC> a_nxt;  // next group's operand (past the end: reloads the last chunk's)
                load_a<C, PREC>(a_nxt, apack, a_base, a_stride, g + 1 < NG ? c : c_next, g + 1 < NG ? g + 1 : 0,
                                lane);
                gen_pairs<C, PREC>(cr, ci, xs_next, px, py, pz, tid, g * PPG, PPG);
                mma_group<C, PREC, NB>(acc, a_cur, s_buf[c & 1], g, cb0, lane);
                a_cur = a_nxt;
                // keep each group's phase pairs among its own MFMAs (left to
                // itself the scheduler sinks them all behind the last group)
                __builtin_amdgcn_sched_barrier(0);
              }
              if (PREC == 2 && wave >= C::WAVES / 2) __builtin_amdgcn_s_setprio(0);
            } else {
              gen_pairs<C, PREC>(cr, ci, xs_next, px, py, pz, tid, 0, 4 * C::JT);
            }
            gen_store<C, PREC>(s_buf[(c + 1) & 1], cr, ci, tid);
            __syncthreads();
          }
          if (!active) continue;

          if (MODE == 1) {
#pragma unroll
            for (int n = 0; n < NB; ++n) {
              const int64_t p = p0 + (cb0 + n) * 32 + (lane & 31);
              if (p < P.n_pix) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                  const int k = kb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                  float er, ei;
                  fields<PREC, NB>(acc, n, r, er, ei);
                  P.e_out[(int64_t)k * P.e_ld + p] = er;
                  P.e_out[(int64_t)(P.e_rows + k) * P.e_ld + p] = ei;
                }
              }
            }
            continue;
          }
          // epilogue: weighted |E|^2 into per-level partial sums
          const int lev_lo = kbr[2 * kb], lev_hi = kbr[2 * kb + 1];
          if (lev_lo > lev_hi) continue;  // no kept eigenvalue in this k-block
          float w[16];
          int lv[16];
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int k = kb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            w[r] = wts[k];
            lv[r] = levs[k];
          }
#pragma unroll
          for (int n = 0; n < NB; ++n) {
            float e2[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              float er, ei;
              fields<PREC, NB>(acc, n, r, er, ei);
              e2[r] = w[r] * fmaf(er, er, ei * ei);
            }
            for (int l = lev_lo; l <= lev_hi; ++l) {
              float sum = 0.0f;
#pragma unroll
              for (int r = 0; r < 16; ++r) sum += (lv[r] == l) ? e2[r] : 0.0f;
              sum += __shfl_xor(sum, 32);
              if (lane < 32) s_part[wk][l][(cb0 + n) * 32 + lane] += sum;
            }
          }
        }
        __syncthreads();
        if (MODE == 1) continue;
        for (int i = tid; i < n_levels * C::NT; i += C::THREADS) {
          const int l = i / C::NT, pl = i % C::NT;
          const int64_t p = p0 + pl;
          if (p < P.n_pix) {
            float sum = 0.0f;
#pragma unroll
            for (int q = 0; q < WK; ++q) sum += s_part[q][l][pl];
            float* dst = P.img + ((int64_t)slot * n_levels + l) * P.img_ld + p;
            *dst += sum;
          }
        }
        __syncthreads();
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Tiles of 16-row eigenpair blocks for the three-product FP32 form, on
// v_mfma_f32_16x16x4f32 (the same matrix rate as 32x32x2): kept eigenpairs are
// padded to 16 rather than 32, which is what small K loses most to.
//   MR x NP: 16x16 output blocks per wave (eigenpair blocks x pixel blocks);
//   WK x WN: waves along eigenpairs and along pixels.  Eigenpair block m of
//   k-group wk in pass p is block p * MR * WK + m * WK + wk (interleaved), so the
//   blocks that exist at a given K fall evenly on the k-groups, and with WN a
//   multiple of 4 each SIMD holds one wave of every k-group.
// MFMA operand order (64 lanes): A lane l = row l % 16 of antenna l / 16 of the
// step, B lane l = pixel l % 16 of antenna l / 16; result register r of lane l
// = row 4 (l / 16) + r, pixel l % 16.  Operand vectors are float2 (two steps,
// 8 antennas): a group of MFMAs covers 8 antennas, which keeps the A operand
// and its prefetch within the register budget (256 VGPRs at two waves per
// SIMD, 128 at four).
template <int MR, int NP, int WK, int WN>
struct Tile16 {
  static constexpr int ROWS = 16;
  static constexpr int WAVES = WK * WN;
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int KC = 16 * MR * WK;       // eigenpairs per pass
  static constexpr int NT = 16 * NP * WN;       // pixels per tile
  static constexpr int NPB = NT / 16;           // 16-pixel blocks per tile
  static constexpr int LCH = 32;                // antennas per LDS chunk
  static constexpr int NG = LCH / 8;            // MFMA groups (2 steps of 4 antennas) per chunk
  static constexpr int TASKS = NT * (LCH / 4);  // (pixel, 4-antenna) phase tasks per chunk
  static constexpr int JT = TASKS / THREADS;
  static constexpr int CHUNK_VEC = 3 * LCH * NT / 2;  // float2 vectors per chunk buffer
  static constexpr int PPG = 4 * JT / NG;       // phase pairs per MFMA group
  static_assert(WN % 4 == 0, "every SIMD holds one wave of each k-group");
  static_assert(THREADS % NT == 0, "a thread keeps one pixel");
  static_assert(JT >= 1 && TASKS % THREADS == 0, "whole tasks per thread");
  static_assert(PPG * NG == 4 * JT, "pairs split evenly over the groups");
  static_assert(kAntChunk % LCH == 0, "antenna padding covers the chunk");
};

// Task j of a thread: pixel (tid + j THREADS) mod NT and antenna group
// gk = t / NT = 2 g8 + h; its four pairs are antennas 8 g8 + 4 s + kk for
// s = 0, 1 and kk = 2 h, 2 h + 1: two float2 operand vectors.
template <class C>
__device__ __forceinline__ int gen_antenna16(int gk, int q) {
  return 8 * (gk >> 1) + 4 * (q & 1) + 2 * (gk & 1) + ((q >> 1) & 1);
}

template <class C>
__device__ __forceinline__ void gen_pairs16(float (&cr)[4 * C::JT], float (&ci)[4 * C::JT],
                                            const BB_LDS double* __restrict__ xs_chunk, double px, double py,
                                            double pz, int tid, int first, int count) {
#pragma unroll
  for (int q = 0; q < 4 * C::JT; ++q)
    if (q >= first && q < first + count)
      phase_pair(xs_chunk + 4 * gen_antenna16<C>(gen_group<C>(tid, q >> 2), q & 3), px, py, pz, cr[q], ci[q]);
}

// B planes Br, Bi - Br, Br + Bi of this thread's tasks into the chunk buffer,
// float2 vectors ordered (8-antenna group, plane, pixel block, lane).
template <class C>
__device__ __forceinline__ void gen_store16(f32x2* __restrict__ buf, const float (&pr)[4 * C::JT],
                                            const float (&pi)[4 * C::JT], int tid) {
#pragma unroll
  for (int j = 0; j < C::JT; ++j) {
    const int pl = (tid + j * C::THREADS) % C::NT;
    const int gk = gen_group<C>(tid, j);
    const int g8 = gk >> 1, h = gk & 1;
#pragma unroll
    for (int e = 0; e < 2; ++e) {  // kk = 2 h + e: pairs 2 e (s = 0) and 2 e + 1 (s = 1)
      const int o = (g8 * 3 * C::NPB + (pl >> 4)) * 64 + (2 * h + e) * 16 + (pl & 15);
      const float r0 = pr[4 * j + 2 * e], r1 = pr[4 * j + 2 * e + 1];
      const float i0 = pi[4 * j + 2 * e], i1 = pi[4 * j + 2 * e + 1];
      buf[o] = f32x2{r0, r1};
      buf[o + C::NPB * 64] = f32x2{i0 - r0, i1 - r1};
      buf[o + 2 * C::NPB * 64] = f32x2{r0 + i0, r1 + i1};
    }
  }
}

template <int NV>
struct AFrag16 {  // three planes of NV eigenpair blocks, 8 antennas
  f32x2 v[3][NV];
};

// A operand of group g of chunk c for NV blocks: block m's vectors start at
// a_base + m * a_mstep (wave-uniform, so the address stays scalar and each
// lane adds only its own offset), 8-antenna groups 3 x 64 vectors apart.
template <class C, int NV>
__device__ __forceinline__ void load_a16(AFrag16<NV>& a, const BB_GLOBAL f32x2* a_base, int64_t a_mstep, int c,
                                         int g, int lane) {
#pragma unroll
  for (int m = 0; m < NV; ++m) {
    const BB_GLOBAL f32x2* const blk = a_base + (m * a_mstep + (int64_t)(c * C::NG + g) * 3 * 64);
#pragma unroll
    for (int q = 0; q < 3; ++q) a.v[q][m] = blk[lane + q * 64];
  }
}

template <class C, int MR, int NP, int NV>
__device__ __forceinline__ void mma_group16(f32x4 (&acc)[3][MR][NP], const AFrag16<NV>& a,
                                            const f32x2* __restrict__ buf, int g, int pb0, int lane) {
  f32x2 b[3][NP];
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int n = 0; n < NP; ++n) b[q][n] = buf[((g * 3 + q) * C::NPB + pb0 + n) * 64 + lane];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int m = 0; m < NV; ++m)
#pragma unroll
      for (int n = 0; n < NP; ++n)
#pragma unroll
        for (int q = 0; q < 3; ++q)
          acc[q][m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[q][m][s], b[q][n][s], acc[q][m][n], 0, 0, 0);
}

template <int MR, int NP, int WK, int WN>
__global__ __launch_bounds__(64 * WK * WN) void synth_fwd16_kernel(const FwdParams P) {
  using C = Tile16<MR, NP, WK, WN>;
  __shared__ f32x2 s_buf[2][C::CHUNK_VEC];
  __shared__ float s_part[WK][kMaxLevels][C::NT];
  __shared__ __align__(16) double s_xs[4 * kMaxAnt];
  const BB_LDS double* const xs = (const BB_LDS double*)s_xs;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wk = __builtin_amdgcn_readfirstlane(wave / WN);
  const int pb0 = __builtin_amdgcn_readfirstlane((wave % WN) * NP);
  const int n_levels = P.n_levels;

  // persistent grid over pixel tiles; groups and instances in the same order
  // in every workgroup; one writer per image tile (as synth_fwd_kernel)
  for (int grp = 0; grp < P.n_groups; ++grp) {
    const int slot = __builtin_amdgcn_readfirstlane(P.group_slot[grp]);
    for (int ii = P.group_begin[grp]; ii < P.group_begin[grp + 1]; ++ii) {
      const int inst = __builtin_amdgcn_readfirstlane(P.inst_list[ii]);
      const InstDesc& Dg = P.descs[inst];
      const void* const apack = Dg.apack;
      const BB_GLOBAL double* const xs_g = as_global<double>(Dg.xs);
      const BB_GLOBAL float* const wts = as_global<float>(Dg.wts);
      const BB_GLOBAL int* const levs = as_global<int>(Dg.levs);
      const int K_alloc = __builtin_amdgcn_readfirstlane(Dg.K_alloc);
      const BB_GLOBAL int* const kbr16 = as_global<int>(Dg.kbr) + 2 * (K_alloc / 32);
      const int nb16 = __builtin_amdgcn_readfirstlane((P.dyn[inst].K_eff + 15) / 16);
      const int L_pad = __builtin_amdgcn_readfirstlane(Dg.L_pad);
      const int n_chunks = L_pad / C::LCH;
      const int n_pass = (nb16 * 16 + C::KC - 1) / C::KC;
      const int64_t a_blk_vec = (int64_t)(L_pad / 8) * 3 * 64;  // float2 vectors per 16-block
      if (blockIdx.x < P.n_tiles) {
        __syncthreads();
        for (int i = tid; i < 2 * L_pad; i += C::THREADS) ((f64x2*)s_xs)[i] = ((const BB_GLOBAL f64x2*)xs_g)[i];
        __syncthreads();
      }
      for (int64_t tile = blockIdx.x; tile < P.n_tiles; tile += gridDim.x) {
        const int64_t p0 = tile * C::NT;
        for (int i = tid; i < WK * kMaxLevels * C::NT; i += C::THREADS) (&s_part[0][0][0])[i] = 0.0f;
        int64_t pg = p0 + (tid % C::NT);
        if (pg >= P.n_pix) pg = P.n_pix - 1;
        const double px = P.pix[pg], py = P.pix[pg + P.pix_ld], pz = P.pix[pg + 2 * P.pix_ld];
        for (int pass = 0; pass < n_pass; ++pass) {
          const int b0 = pass * MR * WK + wk;  // this wave's first block; block m is b0 + m WK
          int nv = nb16 > b0 ? (nb16 - b0 + WK - 1) / WK : 0;
          nv = __builtin_amdgcn_readfirstlane(nv < MR ? nv : MR);
          f32x4 acc[3][MR][NP];
#pragma unroll
          for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int m = 0; m < MR; ++m)
#pragma unroll
              for (int n = 0; n < NP; ++n) acc[q][m][n] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

          // the chunk loop for NV existing blocks of this wave (NV = 0: phases only)
          auto chunks = [&](auto nv_c) {
            constexpr int NV = decltype(nv_c)::value;
            const BB_GLOBAL f32x2* const a_base = as_global<f32x2>(apack) + (int64_t)b0 * a_blk_vec;
            const int64_t a_mstep = (int64_t)WK * a_blk_vec;
            AFrag16<NV> a_cur;
            if constexpr (NV > 0) load_a16<C, NV>(a_cur, a_base, a_mstep, 0, 0, lane);
            __syncthreads();  // previous users of s_buf are done
            {
              float cr[4 * C::JT], ci[4 * C::JT];
              gen_pairs16<C>(cr, ci, xs, px, py, pz, tid, 0, 4 * C::JT);
              gen_store16<C>(s_buf[0], cr, ci, tid);
            }
            __syncthreads();
            for (int c = 0; c < n_chunks; ++c) {
              const int c_next = min(c + 1, n_chunks - 1);
              const BB_LDS double* const xs_next = xs + 4 * c_next * C::LCH;
              float cr[4 * C::JT], ci[4 * C::JT];
              if constexpr (NV > 0) {
                // waves of odd k-groups multiply at a higher priority, which
                // staggers the phase slices of the waves sharing a SIMD
                if (wk & 1) __builtin_amdgcn_s_setprio(1);
#pragma unroll
                for (int g = 0; g < C::NG; ++g) {
                  AFrag16<NV> a_nxt;
                  load_a16<C, NV>(a_nxt, a_base, a_mstep, g + 1 < C::NG ? c : c_next, g + 1 < C::NG ? g + 1 : 0,
                                  lane);
                  gen_pairs16<C>(cr, ci, xs_next, px, py, pz, tid, g * C::PPG, C::PPG);
                  mma_group16<C, MR, NP, NV>(acc, a_cur, s_buf[c & 1], g, pb0, lane);
                  a_cur = a_nxt;
                  __builtin_amdgcn_sched_barrier(0);
                }
                if (wk & 1) __builtin_amdgcn_s_setprio(0);
              } else {
                gen_pairs16<C>(cr, ci, xs_next, px, py, pz, tid, 0, 4 * C::JT);
              }
              gen_store16<C>(s_buf[(c + 1) & 1], cr, ci, tid);
              __syncthreads();
            }
          };
          if (nv == MR)
            chunks(std::integral_constant<int, MR>{});
          else if (MR > 3 && nv == 3)
            chunks(std::integral_constant<int, (MR > 3 ? 3 : 1)>{});
          else if (MR > 2 && nv == 2)
            chunks(std::integral_constant<int, (MR > 2 ? 2 : 1)>{});
          else if (MR > 1 && nv == 1)
            chunks(std::integral_constant<int, 1>{});
          else
            chunks(std::integral_constant<int, 0>{});

          // epilogue: weighted |E|^2 of each existing block into per-level sums
#pragma unroll
          for (int m = 0; m < MR; ++m) {
            if (m >= nv) continue;
            const int b = b0 + m * WK;
            const int lev_lo = kbr16[2 * b], lev_hi = kbr16[2 * b + 1];
            if (lev_lo > lev_hi) continue;
            float w[4];
            int lv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int k = b * 16 + 4 * (lane >> 4) + r;
              w[r] = wts[k];
              lv[r] = levs[k];
            }
#pragma unroll
            for (int n = 0; n < NP; ++n) {
              float e2[4];
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const float er = acc[0][m][n][r] - acc[2][m][n][r];
                const float ei = acc[0][m][n][r] + acc[1][m][n][r];
                e2[r] = w[r] * fmaf(er, er, ei * ei);
              }
              for (int l = lev_lo; l <= lev_hi; ++l) {
                float sum = 0.0f;
#pragma unroll
                for (int r = 0; r < 4; ++r) sum += (lv[r] == l) ? e2[r] : 0.0f;
                sum += __shfl_xor(sum, 16);
                sum += __shfl_xor(sum, 32);
                if (lane < 16) s_part[wk][l][(pb0 + n) * 16 + lane] += sum;
              }
            }
          }
        }
        __syncthreads();
        for (int i = tid; i < n_levels * C::NT; i += C::THREADS) {
          const int l = i / C::NT, pl = i % C::NT;
          const int64_t p = p0 + pl;
          if (p < P.n_pix) {
            float sum = 0.0f;
#pragma unroll
            for (int q = 0; q < WK; ++q) sum += s_part[q][l][pl];
            float* dst = P.img + ((int64_t)slot * n_levels + l) * P.img_ld + p;
            *dst += sum;
          }
        }
        __syncthreads();
      }
    }
  }
}

// Resident workgroups of a kernel on the current device (persistent grid size).
template <class K>
static int resident_blocks(K kernel, int threads) {
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess) return 0;
  return ncu * (per_cu > 0 ? per_cu : 1);
}

template <int MB, int NB, int WK, int WN, int PREC, int MODE = 0>
static hipError_t launch_cfg(const FwdParams& p, hipStream_t s) {
  using C = TileCfg<MB, NB, WK, WN>;
  if (p.n_tiles <= 0 || p.n_groups <= 0) return hipSuccess;
  auto kern = synth_fwd_kernel<MB, NB, WK, WN, PREC, MODE>;
  static int resident = 0;  // per instantiation; one device type per process
  if (resident <= 0) resident = resident_blocks(kern, C::THREADS);
  int64_t grid = resident > 0 ? resident : 1024;
  if (grid > p.n_tiles) grid = p.n_tiles;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(C::THREADS), 0, s, p);
  return hipGetLastError();
}

template <int PREC, int MODE, int MB, int NB, int WK, int WN>
static hipError_t launch_tc(const FwdParams& p, TileCfg<MB, NB, WK, WN>, hipStream_t s) {
  return launch_cfg<MB, NB, WK, WN, PREC, MODE>(p, s);
}

// 16-row tiles: the three-product FP32 form's level images only.
template <int PREC, int MODE, int MR, int NP, int WK, int WN>
static hipError_t launch_tc(const FwdParams& p, Tile16<MR, NP, WK, WN>, hipStream_t s) {
  using C = Tile16<MR, NP, WK, WN>;
  if constexpr (PREC != 2 || MODE != 0) {
    return hipErrorInvalidValue;
  } else {
    if (p.n_tiles <= 0 || p.n_groups <= 0) return hipSuccess;
    auto kern = synth_fwd16_kernel<MR, NP, WK, WN>;
    static int resident = 0;  // per instantiation; one device type per process
    if (resident <= 0) resident = resident_blocks(kern, C::THREADS);
    int64_t grid = resident > 0 ? resident : 1024;
    if (grid > p.n_tiles) grid = p.n_tiles;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(C::THREADS), 0, s, p);
    return hipGetLastError();
  }
}

// ---------------------------------------------------------------------------
// Tile candidates.  Each precision has a list of tile shapes (kernel
// instantiations); a launch names one by its index in the list.  Instances
// fall in K classes by their kept eigenpairs rounded up to 32: at most 32, 64,
// 128, or more.  Each class has a default shape (the measured best on this
// GPU) and may use every shape of the list whose eigenpairs per pass do not
// exceed the class's largest K (so that no wave of a tile is idle at that K).
// Register budget: 8-wave tiles run two waves per SIMD (<= 256 VGPRs each),
// 16-wave tiles four (<= 128).
template <class... T>
struct TileList {};

template <int PREC>
struct Cands;
template <>
struct Cands<0> {  // 4 products: Er/Ei accumulators, 32 regs per output block
  using L = TileList<TileCfg<1, 4, 8, 1>,   // 0: 256 x 128  (2 x 2 blocks per wave measured slower)
                     TileCfg<1, 4, 4, 2>,   // 1: 128 x 256
                     TileCfg<1, 2, 2, 4>,   // 2: 64 x 256
                     TileCfg<1, 2, 1, 4>,   // 3: 32 x 256, 4 waves
                     TileCfg<1, 2, 4, 2>>;  // 4: 128 x 128
  static constexpr int dflt[4] = {3, 2, 1, 0};
};
template <>
struct Cands<1> {  // BF16 x3, 4 products: the shapes of the FP32 form, and narrower pixel tiles
  using L = TileList<TileCfg<1, 4, 8, 1>,   // 0: 256 x 128
                     TileCfg<1, 4, 4, 2>,   // 1: 128 x 256
                     TileCfg<1, 2, 2, 4>,   // 2: 64 x 256
                     TileCfg<1, 2, 1, 4>,   // 3: 32 x 256, 4 waves
                     TileCfg<1, 2, 4, 2>,   // 4: 128 x 128
                     TileCfg<1, 2, 8, 1>>;  // 5: 256 x 64
  static constexpr int dflt[4] = {3, 2, 1, 0};
};
template <>
struct Cands<2> {  // 3 products: k1/k2/k3 accumulators, 48 regs per 32x32 output block
  using L = TileList<TileCfg<1, 2, 8, 1>,    // 0: 256 x 64
                     TileCfg<1, 1, 4, 4>,    // 1: 128 x 128, 16 waves: 3 active k-blocks (K <= 96) still
                                             //    spread evenly over the four SIMDs
                     TileCfg<1, 2, 2, 4>,    // 2: 64 x 256
                     TileCfg<1, 1, 1, 8>,    // 3: 32 x 256, one pixel block per wave, two waves per SIMD
                     TileCfg<1, 2, 4, 2>,    // 4: 128 x 128
                     TileCfg<1, 1, 2, 8>,    // 5: 64 x 256, 16 waves
                     Tile16<4, 2, 2, 4>,     // 6: 128 x 128 in 16-row blocks, 8 waves
                     Tile16<2, 2, 2, 4>,     // 7: 64 x 128 in 16-row blocks
                     Tile16<1, 1, 2, 8>,     // 8: 32 x 128 in 16-row blocks, 16 waves
                     Tile16<2, 1, 2, 8>,     // 9: 64 x 128 in 16-row blocks, 16 waves
                     Tile16<1, 2, 4, 4>,     // 10: 64 x 128 in 16-row blocks, 16 waves
                     Tile16<2, 2, 4, 4>>;    // 11: 128 x 128 in 16-row blocks, 16 waves
  static constexpr int dflt[4] = {3, 9, 11, 0};
};
template <>
struct Cands<3> {  // BF16 three products: in 16 waves its operand fragments would spill
  using L = TileList<TileCfg<1, 2, 8, 1>,   // 0: 256 x 64
                     TileCfg<1, 2, 4, 2>,   // 1: 128 x 128
                     TileCfg<1, 2, 2, 4>,   // 2: 64 x 256
                     TileCfg<1, 1, 1, 8>,   // 3: 32 x 256
                     TileCfg<1, 1, 4, 2>>;  // 4: 128 x 64
  static constexpr int dflt[4] = {3, 2, 1, 0};
};

template <int I, class F, class T0, class... Ts>
static hipError_t tile_at(int id, F&& f, TileList<T0, Ts...>) {
  if (id == I) return f(T0{});
  if constexpr (sizeof...(Ts) > 0)
    return tile_at<I + 1>(id, f, TileList<Ts...>{});
  else
    return hipErrorInvalidValue;
}

template <class... Ts>
static constexpr int list_len(TileList<Ts...>) {
  return (int)sizeof...(Ts);
}

// f(cfg) for tile `id` of `precision`; hipErrorInvalidValue for an unknown id.
template <class F>
static hipError_t with_tile(int precision, int id, F&& f) {
  switch (precision) {
    case 1: return tile_at<0>(id, f, Cands<1>::L{});
    case 2: return tile_at<0>(id, f, Cands<2>::L{});
    case 3: return tile_at<0>(id, f, Cands<3>::L{});
    default: return tile_at<0>(id, f, Cands<0>::L{});
  }
}

int synth_k_class(int K_alloc) { return K_alloc <= 32 ? 0 : (K_alloc <= 64 ? 1 : (K_alloc <= 128 ? 2 : 3)); }

int synth_n_tiles(int precision) {
  switch (precision) {
    case 1: return list_len(Cands<1>::L{});
    case 2: return list_len(Cands<2>::L{});
    case 3: return list_len(Cands<3>::L{});
    default: return list_len(Cands<0>::L{});
  }
}

int synth_default_tile(int precision, int k_class) {
  if (k_class < 0 || k_class > 3) return -1;
  switch (precision) {
    case 1: return Cands<1>::dflt[k_class];
    case 2: return Cands<2>::dflt[k_class];
    case 3: return Cands<3>::dflt[k_class];
    default: return Cands<0>::dflt[k_class];
  }
}

bool synth_tile_info(int precision, int id, int* kc, int* nt, int* waves) {
  int a = 0, b = 0, c = 0;
  const hipError_t e = with_tile(precision, id, [&](auto cfg) {
    using C = decltype(cfg);
    a = C::KC;
    b = C::NT;
    c = C::WAVES;
    return hipSuccess;
  });
  if (e != hipSuccess) return false;
  if (kc) *kc = a;
  if (nt) *nt = b;
  if (waves) *waves = c;
  return true;
}

int synth_tile_rows(int precision, int id) {
  int rows = 32;
  (void)with_tile(precision, id, [&](auto cfg) {
    rows = decltype(cfg)::ROWS;
    return hipSuccess;
  });
  return rows;
}

bool synth_tile_allowed(int precision, int id, int k_class) {
  static const int kmax[4] = {32, 64, 128, kMaxEig};
  int kc = 0;
  if (k_class < 0 || k_class > 3 || !synth_tile_info(precision, id, &kc, nullptr, nullptr)) return false;
  return kc <= kmax[k_class];
}

template <int PREC>
static hipError_t launch_prec_tile(const FwdParams& p, int id, hipStream_t s) {
  return tile_at<0>(id, [&](auto cfg) { return launch_tc<PREC, 0>(p, cfg, s); }, typename Cands<PREC>::L{});
}

hipError_t launch_synth_tile(const FwdParams& p, int precision, int id, hipStream_t s) {
  switch (precision) {
    case 1: return launch_prec_tile<1>(p, id, s);
    case 2: return launch_prec_tile<2>(p, id, s);
    case 3: return launch_prec_tile<3>(p, id, s);
    default: return launch_prec_tile<0>(p, id, s);
  }
}

int synth_tile_pixels(int max_K_alloc, int precision) {
  int nt = 0;
  synth_tile_info(precision, synth_default_tile(precision, synth_k_class(max_K_alloc)), nullptr, &nt, nullptr);
  return nt;
}

hipError_t launch_synth(const FwdParams& p, int max_K_alloc, int precision, int tile_pixels_out[1],
                        hipStream_t s) {
  if (tile_pixels_out) tile_pixels_out[0] = synth_tile_pixels(max_K_alloc, precision);
  return launch_synth_tile(p, precision, synth_default_tile(precision, synth_k_class(max_K_alloc)), s);
}

// FP32 recompute of E for the backward pass, in the three-product form
// whatever the handle's precision (the instance is staged as three planes), on
// 32-row tiles (the 16-row kernel writes no E), one per K class so that no
// k-block wave idles: K <= 32: 32 x 256, <= 64: 64 x 256, <= 128: 128 x 128,
// above: 256 x 64.
using FieldsL = TileList<TileCfg<1, 1, 1, 8>, TileCfg<1, 2, 2, 4>, TileCfg<1, 2, 4, 2>, TileCfg<1, 2, 8, 1>>;

int fields_tile_pixels(int K_alloc) {
  int nt = 0;
  tile_at<0>(synth_k_class(K_alloc), [&](auto cfg) { nt = decltype(cfg)::NT; return hipSuccess; }, FieldsL{});
  return nt;
}

hipError_t launch_fields(const FwdParams& p, int K_alloc, hipStream_t s) {
  return tile_at<0>(synth_k_class(K_alloc), [&](auto cfg) { return launch_tc<2, 1>(p, cfg, s); }, FieldsL{});
}

// Phase-generation throughput probe (measurement only): every thread takes one
// pixel and evaluates the phases of all antennas `reps` times with the
// synthesis kernel's own arithmetic (positions from LDS, FP64 argument and
// reduction, hardware sine and cosine), summing cos + sin so that nothing is
// dropped.  No MFMA work runs beside it: its rate is the device's peak for
// phase generation alone.
__global__ __launch_bounds__(256) void phase_probe_kernel(const double* __restrict__ ant, int n_ant, double inv_wl,
                                                          const double* __restrict__ pix, int64_t n_pix, int reps,
                                                          float* __restrict__ out) {
  __shared__ __align__(16) double s_xs[4 * kMaxAnt];
  for (int l = threadIdx.x; l < n_ant; l += blockDim.x) {
    s_xs[4 * l + 0] = ant[l] * inv_wl;
    s_xs[4 * l + 1] = ant[l + n_ant] * inv_wl;
    s_xs[4 * l + 2] = ant[l + 2 * n_ant] * inv_wl;
    s_xs[4 * l + 3] = 0.0;
  }
  __syncthreads();
  const BB_LDS double* const xs = (const BB_LDS double*)s_xs;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_pix; p += (int64_t)gridDim.x * blockDim.x) {
    const double px = pix[p], py = pix[p + n_pix], pz = pix[p + 2 * n_pix];
    float acc = 0.0f;
    for (int r = 0; r < reps; ++r)
      for (int l = 0; l < n_ant; ++l) {
        float c, sn;
        phase_pair(xs + 4 * l, px, py, pz, c, sn);
        acc += c + sn;
      }
    out[p] = acc;
  }
}

hipError_t launch_phase_probe(const double* ant, int n_ant, double inv_wl, const double* pix, int64_t n_pix, int reps,
                              float* out, hipStream_t s) {
  int64_t blocks = (n_pix + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(phase_probe_kernel, dim3((unsigned)blocks), dim3(256), 0, s, ant, n_ant, inv_wl, pix, n_pix, reps,
                     out);
  return hipGetLastError();
}

__global__ void fill_zero_kernel(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace bb
