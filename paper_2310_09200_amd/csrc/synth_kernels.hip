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
//   for each instance of the slot, for each K pass, for each 32-antenna chunk:
//     phase generation: FP64 <x_l, p> in quarter turns, exact FP64 reduction to
//       [-1/2, 1/2] plus a quadrant, FP32 sin/cos series -> B chunk in LDS
//       (double-buffered: the next chunk is generated while this one is used)
//     MFMA: real-embedded W^H operand streamed from HBM/L2 in operand order,
//       B operand from LDS, accumulators for [Er; Ei] in registers
//   epilogue of a pass: d_k (Er^2 + Ei^2) reduced over k in-lane, across the
//     two half-waves, and into per-level partial sums in LDS
//   end of the tile: sum over waves in a fixed order, one read-modify-write of
//     the images (one writer per pixel and launch: deterministic, no atomics).
// Neither B (L x N_pix) nor E (K x N_pix) is ever written to HBM.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bb_internal.h"

namespace bb {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// Phase: (cos, sin) of (q + f) * pi/2 for f in [-1/2, 1/2], q any integer.
// Taylor series of sin and cos about 0 (terms to theta^9 and theta^10; the
// truncation error on |theta| <= pi/4 is below 2e-9), then a rotation by q
// quarter turns.
__device__ __forceinline__ void cis_quarter(float f, int q, float& c, float& s) {
  const float th = f * 1.57079632679489662f;
  const float t2 = th * th;
  float sp = fmaf(t2, 2.7557319224e-6f, -1.9841269841e-4f);
  sp = fmaf(t2, sp, 8.3333333333e-3f);
  sp = fmaf(t2, sp, -1.6666666667e-1f);
  const float sn = fmaf(th * t2, sp, th);
  float cp = fmaf(t2, -2.7557319224e-7f, 2.4801587302e-5f);
  cp = fmaf(t2, cp, -1.3888888889e-3f);
  cp = fmaf(t2, cp, 4.1666666667e-2f);
  cp = fmaf(t2, cp, -0.5f);
  const float cs = fmaf(t2, cp, 1.0f);
  const bool swap = (q & 1) != 0;
  const float cc = swap ? sn : cs;
  const float ss = swap ? cs : sn;
  c = ((q + 1) & 2) ? -cc : cc;
  s = (q & 2) ? -ss : ss;
}

// Phase of one (antenna, pixel) pair; xs = position * 4 / wavelength.
__device__ __forceinline__ void phase_pair(const double* __restrict__ xs, double px, double py, double pz,
                                           float& c, float& s) {
  const double t = fma(xs[2], pz, fma(xs[1], py, xs[0] * px));
  const double q = rint(t);
  const float f = (float)(t - q);
  cis_quarter(f, (int)q, c, s);
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
      atomicOr(err, 1);
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
  // level range of each 32-block of sorted positions (levels are non-decreasing)
  for (int kb = tid; kb < D.K_alloc / 32; kb += blockDim.x) {
    int lo = 1, hi = 0;
    const int p0 = kb * 32;
    if (p0 < K_eff) {
      const int p1 = min(p0 + 31, K_eff - 1);
      // sorted positions: find their levels through the base offsets
      int l0 = 0, l1 = 0;
      for (int l = 0; l < n_levels; ++l) {
        if (s_base[l] <= p0 && p0 < s_base[l + 1]) l0 = l;
        if (s_base[l] <= p1 && p1 < s_base[l + 1]) l1 = l;
      }
      lo = l0;
      hi = l1;
    }
    D.kbr[kb] = make_int2(lo, hi);
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

hipError_t launch_stage(const InstDesc* d_descs, InstDyn* d_dyn, int n_inst, int max_K_alloc, int max_L_pad,
                        int n_levels, int precision, int* d_err, hipStream_t s) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(stage_meta_kernel, dim3(n_inst), dim3(256), 0, s, d_descs, d_dyn, n_levels, d_err);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t per = (int64_t)(max_K_alloc / 32) * 2 * (max_L_pad / (precision ? 8 : 4)) * 64;
  const unsigned gx = (unsigned)((per + 255) / 256);
  if (precision)
    hipLaunchKernelGGL(stage_pack_bf16_kernel, dim3(gx, n_inst), dim3(256), 0, s, d_descs);
  else
    hipLaunchKernelGGL(stage_pack_f32_kernel, dim3(gx, n_inst), dim3(256), 0, s, d_descs);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Synthesis kernel.
//   MB x NB: 32x32 output blocks per wave (k-blocks x pixel blocks), each
//            k-block holding an Er and an Ei accumulator;
//   WK x WN: waves along k and along pixels.
template <int MB, int NB, int WK, int WN>
struct TileCfg {
  static constexpr int WAVES = WK * WN;
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int KC = 32 * MB * WK;      // eigenpairs per pass
  static constexpr int NT = 32 * NB * WN;      // pixels per tile
  static constexpr int NCB = NT / 32;
  static constexpr int LCH = NT <= 128 ? 32 : 16;  // antennas per LDS chunk
  static constexpr int G4 = LCH / 4;
  static constexpr int G8 = LCH / 8;
  static constexpr int CHUNK_VEC = LCH * NT / 2;   // 16-byte vectors per chunk buffer
  static constexpr int JT = NT * G4 / THREADS;     // (pixel, 4-antenna) tasks per thread
  static_assert(THREADS % NT == 0, "a thread keeps one pixel");
  static_assert(JT >= 1 && NT * G4 % THREADS == 0, "task split");
  static_assert(kAntChunk % LCH == 0, "antenna padding covers the chunk");
};

template <class C, int PREC>
__device__ __forceinline__ void gen_chunk(f32x4* __restrict__ buf, const double* __restrict__ xs_chunk,
                                          double px, double py, double pz, int tid) {
#pragma unroll
  for (int j = 0; j < C::JT; ++j) {
    const int t = tid + j * C::THREADS;
    const int pl = t % C::NT;
    const int g4 = __builtin_amdgcn_readfirstlane(t / C::NT);
    const int cb = pl >> 5, jj = pl & 31;
    float cr[4], ci[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) phase_pair(xs_chunk + 4 * (4 * g4 + s), px, py, pz, cr[s], ci[s]);
    if (PREC == 0) {
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

// MFMA over one LDS chunk for the first M (<= MB) k-blocks of this wave.
template <class C, int PREC, int M, int MB, int NB>
__device__ __forceinline__ void mfma_chunk(f32x16 (&acc)[2 * MB][NB], const f32x4* __restrict__ buf,
                                           const void* __restrict__ apack, int64_t a_rt_stride_vec,
                                           int64_t a_base_vec, int cb0, int lane) {
  if (PREC == 0) {
    const f32x4* A = (const f32x4*)apack;
#pragma unroll
    for (int g = 0; g < C::G4; ++g) {
      f32x4 a[2 * M], b[NB];
#pragma unroll
      for (int rt = 0; rt < 2 * M; ++rt) a[rt] = A[a_base_vec + rt * a_rt_stride_vec + (int64_t)g * 64 + lane];
#pragma unroll
      for (int n = 0; n < NB; ++n) b[n] = buf[(g * C::NCB + cb0 + n) * 64 + lane];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int rt = 0; rt < 2 * M; ++rt)
#pragma unroll
          for (int n = 0; n < NB; ++n)
            acc[rt][n] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rt][s], b[n][s], acc[rt][n], 0, 0, 0);
    }
  } else {
    const bf16x8* A = (const bf16x8*)apack;
    const bf16x8* Bb = (const bf16x8*)buf;
#pragma unroll
    for (int g = 0; g < C::G8; ++g) {
      bf16x8 ah[2 * M], al[2 * M], bh[NB], bl[NB];
#pragma unroll
      for (int rt = 0; rt < 2 * M; ++rt) {
        const int64_t o = a_base_vec + rt * a_rt_stride_vec + (int64_t)g * 128 + lane;
        ah[rt] = A[o];
        al[rt] = A[o + 64];
      }
#pragma unroll
      for (int n = 0; n < NB; ++n) {
        const int o = ((g * C::NCB + cb0 + n) * 2) * 64 + lane;
        bh[n] = Bb[o];
        bl[n] = Bb[o + 64];
      }
#pragma unroll
      for (int rt = 0; rt < 2 * M; ++rt)
#pragma unroll
        for (int n = 0; n < NB; ++n) {
          acc[rt][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[rt], bh[n], acc[rt][n], 0, 0, 0);
          acc[rt][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[rt], bl[n], acc[rt][n], 0, 0, 0);
          acc[rt][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[rt], bh[n], acc[rt][n], 0, 0, 0);
        }
    }
  }
}

// MODE 0: level images (the product).  MODE 1: write E itself (two planes,
// re and im, [K_alloc][n_pix] each) for the backward pass; one instance only.
template <int MB, int NB, int WK, int WN, int PREC, int MODE>
__global__ __launch_bounds__(64 * WK * WN) void synth_fwd_kernel(const FwdParams P) {
  using C = TileCfg<MB, NB, WK, WN>;
  __shared__ f32x4 s_buf[2][C::CHUNK_VEC];
  __shared__ float s_part[WK][kMaxLevels][C::NT];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wk = wave % WK;
  const int wn = wave / WK;
  const int cb0 = wn * NB;
  const int n_levels = P.n_levels;

  for (int64_t item = blockIdx.x; item < P.n_items; item += gridDim.x) {
    const int grp = (int)(item / P.n_tiles);
    const int slot = P.group_slot[grp];
    const int64_t tile = item % P.n_tiles;
    const int64_t p0 = tile * C::NT;

    for (int i = tid; i < WK * kMaxLevels * C::NT; i += C::THREADS) (&s_part[0][0][0])[i] = 0.0f;

    // this thread's pixel (phase generation); clamp the ragged tail
    int64_t pg = p0 + (tid % C::NT);
    if (pg >= P.n_pix) pg = P.n_pix - 1;
    const double px = P.pix[pg], py = P.pix[pg + P.pix_ld], pz = P.pix[pg + 2 * P.pix_ld];

    const int ib = P.group_begin[grp], ie = P.group_begin[grp + 1];
    for (int ii = ib; ii < ie; ++ii) {
      const int inst = P.inst_list[ii];
      const InstDesc& D = P.descs[inst];
      const int K_pad = P.dyn[inst].K_pad;
      const int L_pad = D.L_pad;
      const int n_chunks = L_pad / C::LCH;
      const int n_pass = (K_pad + C::KC - 1) / C::KC;
      const double* xs = D.xs;
      const int64_t a_rt_stride = (int64_t)(L_pad / 4) * 64;  // 16-byte vectors per A row tile (both precisions)
      for (int pass = 0; pass < n_pass; ++pass) {
        const int kb0 = pass * (C::KC / 32) + wk * MB;
        int mact = K_pad / 32 - kb0;
        mact = mact < 0 ? 0 : (mact > MB ? MB : mact);
        f32x16 acc[2 * MB][NB];
#pragma unroll
        for (int rt = 0; rt < 2 * MB; ++rt)
#pragma unroll
          for (int n = 0; n < NB; ++n)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[rt][n][r] = 0.0f;

        __syncthreads();  // previous users of s_buf are done
        gen_chunk<C, PREC>(s_buf[0], xs, px, py, pz, tid);
        __syncthreads();
        for (int c = 0; c < n_chunks; ++c) {
          if (c + 1 < n_chunks)
            gen_chunk<C, PREC>(s_buf[(c + 1) & 1], xs + 4 * (c + 1) * C::LCH, px, py, pz, tid);
          const int64_t a_base = (int64_t)(kb0 * 2) * a_rt_stride + (int64_t)c * (C::LCH / 4) * 64;
          if (mact == MB)
            mfma_chunk<C, PREC, MB, MB, NB>(acc, s_buf[c & 1], D.apack, a_rt_stride, a_base, cb0, lane);
          else if (MB > 1 && mact == 1)
            mfma_chunk<C, PREC, 1, MB, NB>(acc, s_buf[c & 1], D.apack, a_rt_stride, a_base, cb0, lane);
          __syncthreads();
        }

        if (MODE == 1) {
#pragma unroll
          for (int m = 0; m < MB; ++m) {
            if (m >= mact) break;
            const int kb = kb0 + m;
#pragma unroll
            for (int n = 0; n < NB; ++n) {
              const int64_t p = p0 + (cb0 + n) * 32 + (lane & 31);
              if (p < P.n_pix) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                  const int k = kb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                  P.e_out[(int64_t)k * P.e_ld + p] = acc[2 * m][n][r];
                  P.e_out[(int64_t)(P.e_rows + k) * P.e_ld + p] = acc[2 * m + 1][n][r];
                }
              }
            }
          }
          continue;
        }
        // epilogue: weighted |E|^2 into per-level partial sums
#pragma unroll
        for (int m = 0; m < MB; ++m) {
          if (m >= mact) break;
          const int kb = kb0 + m;
          const int2 lr = D.kbr[kb];
          if (lr.x > lr.y) continue;
          float w[16];
          int lv[16];
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int k = kb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            w[r] = D.wts[k];
            lv[r] = D.levs[k];
          }
#pragma unroll
          for (int n = 0; n < NB; ++n) {
            float e2[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const float er = acc[2 * m][n][r], ei = acc[2 * m + 1][n][r];
              e2[r] = w[r] * fmaf(er, er, ei * ei);
            }
            for (int l = lr.x; l <= lr.y; ++l) {
              float sum = 0.0f;
#pragma unroll
              for (int r = 0; r < 16; ++r) sum += (lv[r] == l) ? e2[r] : 0.0f;
              sum += __shfl_xor(sum, 32);
              if (lane < 32) s_part[wk][l][(cb0 + n) * 32 + lane] += sum;
            }
          }
        }
      }
    }
    __syncthreads();
    if (MODE == 1) continue;
    for (int i = tid; i < n_levels * C::NT; i += C::THREADS) {
      const int l = i / C::NT, pl = i % C::NT;
      const int64_t p = p0 + pl;
      if (p < P.n_pix) {
        float s = 0.0f;
#pragma unroll
        for (int q = 0; q < WK; ++q) s += s_part[q][l][pl];
        float* dst = P.img + ((int64_t)slot * n_levels + l) * P.img_ld + p;
        *dst += s;
      }
    }
    __syncthreads();
  }
}

template <int MB, int NB, int WK, int WN, int PREC, int MODE = 0>
static hipError_t launch_cfg(const FwdParams& p, hipStream_t s) {
  using C = TileCfg<MB, NB, WK, WN>;
  const int64_t grid = p.n_items;
  if (grid <= 0) return hipSuccess;
  const unsigned g = (unsigned)(grid > 0x7fffffff ? 0x7fffffff : grid);
  hipLaunchKernelGGL((synth_fwd_kernel<MB, NB, WK, WN, PREC, MODE>), dim3(g), dim3(C::THREADS), 0, s, p);
  return hipGetLastError();
}

int synth_tile_pixels(int max_K_alloc) {
  if (max_K_alloc > 256) return TileCfg<2, 2, 8, 1>::NT;
  if (max_K_alloc > 128) return TileCfg<1, 4, 8, 1>::NT;
  if (max_K_alloc > 64) return TileCfg<1, 4, 4, 2>::NT;
  if (max_K_alloc > 32) return TileCfg<1, 2, 2, 4>::NT;
  return TileCfg<1, 2, 1, 4>::NT;
}

template <int PREC>
static hipError_t launch_prec(const FwdParams& p, int max_K_alloc, hipStream_t s) {
  if (max_K_alloc > 256) return launch_cfg<2, 2, 8, 1, PREC>(p, s);
  if (max_K_alloc > 128) return launch_cfg<1, 4, 8, 1, PREC>(p, s);
  if (max_K_alloc > 64) return launch_cfg<1, 4, 4, 2, PREC>(p, s);
  if (max_K_alloc > 32) return launch_cfg<1, 2, 2, 4, PREC>(p, s);
  return launch_cfg<1, 2, 1, 4, PREC>(p, s);
}

hipError_t launch_synth(const FwdParams& p, int max_K_alloc, int precision, int tile_pixels_out[1],
                        hipStream_t s) {
  if (tile_pixels_out) tile_pixels_out[0] = synth_tile_pixels(max_K_alloc);
  return precision ? launch_prec<1>(p, max_K_alloc, s) : launch_prec<0>(p, max_K_alloc, s);
}

int fields_tile_pixels(int K_alloc) {
  if (K_alloc > 256) return TileCfg<2, 2, 8, 1>::NT;
  if (K_alloc > 128) return TileCfg<1, 4, 8, 1>::NT;
  return TileCfg<1, 4, 4, 2>::NT;
}

hipError_t launch_fields(const FwdParams& p, int K_alloc, hipStream_t s) {
  // FP32 recompute of E for the backward pass (the handle's precision does not apply)
  if (K_alloc > 256) return launch_cfg<2, 2, 8, 1, 0, 1>(p, s);
  if (K_alloc > 128) return launch_cfg<1, 4, 8, 1, 0, 1>(p, s);
  return launch_cfg<1, 4, 4, 2, 0, 1>(p, s);
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
