// Line FFTs of the NUFFT's pruned type-2 transform (gfx950).  Lines of at
// most 64 points (the thin axis of a grid) are instead a direct pruned DFT on
// MFMA (line_dft_kernel, at the end of this file).
//
// Each workgroup transforms one or more lines of L = M points held in LDS
// (L 2,3,5-smooth, at most 16384).  A line's N stored inputs are placed at
// their frequencies' positions (index i holds frequency i for i < N/2, else
// i - N) and divided by the axis's kernel transform on load; the other M - N
// positions are zero.  The inverse DFT X[m] = sum_n x[n] exp(+2 pi i n m / M)
// (unnormalised) is done in place by mixed-radix decimation in time (radix 8,
// 4, 2, 3, 5 in the order R_0, R_1, ...): pass s combines R_s transforms of
// length Ns = R_0 ... R_{s-1} that sit Ns apart into one of length P = Ns R_s,
// each butterfly reading and writing the same R_s points (twiddles
// exp(2 pi i k r / P)).  For that the load puts input n at the digit-reversed
// position sum_s r_s Ns_s, where n = r_{S-1} + R_{S-1} (r_{S-2} + R_{S-2} (...)),
// from a table made on the host.  Only a window of outputs, positions
// (lo + w) mod M for w < len, is stored.  One LDS buffer of L x 8 bytes per
// line.  Twiddles come from a table made in FP64 on the host: pass s keeps
// its Ns (R_s - 1) values exp(2 pi i k r / P), k < Ns, 1 <= r < R_s, at
// offset Ns - 1 (the earlier passes hold sum (P - Ns) = Ns - 1 of them), so
// a butterfly reads its R - 1 twiddles as one contiguous run.  Index
// quotients use an FP32 reciprocal: for j, d <= 16384, (j + 1/2) / d is at
// least 1/(2d) from an integer and the rounding error stays below that.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "bb_internal.h"

namespace bb {

namespace {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 mul_i(float2 a) { return make_float2(-a.y, a.x); }  // i a

// Inverse DFTs of size R in place: y[q] = sum_r v[r] exp(+2 pi i r q / R).
template <int R>
__device__ __forceinline__ void small_dft(float2 (&v)[R]);

template <>
__device__ __forceinline__ void small_dft<2>(float2 (&v)[2]) {
  const float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <>
__device__ __forceinline__ void small_dft<4>(float2 (&v)[4]) {
  const float2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
  const float2 s13 = cadd(v[1], v[3]), d13 = mul_i(csub(v[1], v[3]));
  v[0] = cadd(s02, s13);
  v[1] = cadd(d02, d13);
  v[2] = csub(s02, s13);
  v[3] = csub(d02, d13);
}

template <>
__device__ __forceinline__ void small_dft<8>(float2 (&v)[8]) {
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  small_dft<4>(e);
  small_dft<4>(o);
  constexpr float h = 0.70710678118654752440f;  // 1 / sqrt(2)
  const float2 o1 = make_float2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y));    // (1 + i)/sqrt2
  const float2 o2 = mul_i(o[2]);                                                   // i
  const float2 o3 = make_float2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y));   // (-1 + i)/sqrt2
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

template <>
__device__ __forceinline__ void small_dft<3>(float2 (&v)[3]) {
  constexpr float s = 0.86602540378443864676f;  // sin(2 pi / 3)
  const float2 a = v[0], p = cadd(v[1], v[2]), m = csub(v[1], v[2]);
  const float2 t = make_float2(a.x - 0.5f * p.x, a.y - 0.5f * p.y);
  const float2 u = make_float2(-s * m.y, s * m.x);  // i s (b - c)
  v[0] = cadd(a, p);
  v[1] = cadd(t, u);
  v[2] = csub(t, u);
}

template <>
__device__ __forceinline__ void small_dft<5>(float2 (&v)[5]) {
  constexpr float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
  constexpr float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
  constexpr float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
  constexpr float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
  const float2 a = v[0];
  const float2 p14 = cadd(v[1], v[4]), m14 = csub(v[1], v[4]);
  const float2 p23 = cadd(v[2], v[3]), m23 = csub(v[2], v[3]);
  const float2 r1 = make_float2(a.x + c1 * p14.x + c2 * p23.x, a.y + c1 * p14.y + c2 * p23.y);
  const float2 r2 = make_float2(a.x + c2 * p14.x + c1 * p23.x, a.y + c2 * p14.y + c1 * p23.y);
  // i (s1 m14 + s2 m23) and i (s2 m14 - s1 m23)
  const float2 j1 = mul_i(make_float2(s1 * m14.x + s2 * m23.x, s1 * m14.y + s2 * m23.y));
  const float2 j2 = mul_i(make_float2(s2 * m14.x - s1 * m23.x, s2 * m14.y - s1 * m23.y));
  v[0] = make_float2(a.x + p14.x + p23.x, a.y + p14.y + p23.y);
  v[1] = cadd(r1, j1);
  v[4] = csub(r1, j1);
  v[2] = cadd(r2, j2);
  v[3] = csub(r2, j2);
}

// floor(j / d) for 0 <= j, 1 <= d <= 16384, given inv_d = 1 / d in FP32.
__device__ __forceinline__ int quot(int j, float inv_d) { return (int)(((float)j + 0.5f) * inv_d); }

// One in-place decimation-in-time pass of radix R over nl lines of L points
// (nl = 1 unless MULTI); tw holds this pass's twiddles, [k][r - 1].
// LDS position of point i of the lines: with PAD one spare point after every
// 32, which spreads the power-of-two strides of the early radix-8 passes of
// a line with many factors of 2 over the banks (one long line per workgroup).
template <bool PAD>
__device__ __forceinline__ int padi(int i) { return PAD ? i + (i >> 5) : i; }

template <int R, int T, bool MULTI, bool PAD>
__device__ __forceinline__ void dit_pass(float2* s, int L, int nl, int Ns, const float2* __restrict__ tw) {
  const int per_line = L / R;
  const int nb = nl * per_line;
  const int P = Ns * R;
  const float inv_pl = 1.0f / (float)per_line, inv_ns = 1.0f / (float)Ns;
  for (int j = threadIdx.x; j < nb; j += T) {
    const int line = MULTI ? quot(j, inv_pl) : 0, jj = j - line * per_line;
    const int g = quot(jj, inv_ns), k = jj - g * Ns;
    const int base = line * L + g * P + k;
    const float2* const w = tw + k * (R - 1);
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s[padi<PAD>(base + r * Ns)];
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], w[r - 1]);
    small_dft<R>(v);
#pragma unroll
    for (int r = 0; r < R; ++r) s[padi<PAD>(base + r * Ns)] = v[r];
  }
  __syncthreads();
}

// nl lines of L points per workgroup (nl = 1 unless MULTI), T threads.
template <int T, bool MULTI, bool PAD>
__global__ __launch_bounds__(T) void line_fft_kernel(LineFft p, const float2* __restrict__ in,
                                                     const float* __restrict__ inv_psi, const int* __restrict__ perm,
                                                     const float2* __restrict__ tw, float2* __restrict__ out) {
  extern __shared__ float2 s_line[];  // nl x L points
  const int L = p.L, nl = MULTI ? p.nl : 1;
  const int n_in = p.n_in, half = n_in / 2, gap = L - n_in;
  const int in_stride = (int)p.in_stride;
  const int tid = threadIdx.x;
  const float inv_nin = 1.0f / (float)n_in;
  for (int64_t l0 = (int64_t)blockIdx.x * nl; l0 < p.n_lines; l0 += (int64_t)gridDim.x * nl) {
    const int nh = MULTI ? (int)min<int64_t>(nl, p.n_lines - l0) : 1;
    // zero the lines (L is even), then place the stored inputs: input i of a
    // line holds the frequency at position m (i, or i + M - N for the
    // negative half), which the passes want at perm[m]
    float4* const z = reinterpret_cast<float4*>(s_line);
    for (int e = tid; e < (padi<PAD>(nl * L) + 1) / 2; e += T) z[e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    __syncthreads();
    const float2* const src = in + l0 * p.in_stride;
#pragma unroll 4
    for (int e = tid; e < nh * n_in; e += T) {
      const int l = MULTI ? quot(e, inv_nin) : 0;
      const int i = e - l * n_in;
      const int m = i < half ? i : i + gap;
      const float2 x = src[l * in_stride + i];
      const float sc = inv_psi[i];
      s_line[padi<PAD>(l * L + perm[m])] = make_float2(x.x * sc, x.y * sc);
    }
    __syncthreads();
    int Ns = 1;
    for (int ps = 0; ps < p.n_pass; ++ps) {
      const int R = (int)((p.radix_codes >> (4 * ps)) & 15);
      switch (R) {
        case 8: dit_pass<8, T, MULTI, PAD>(s_line, L, nl, Ns, tw + (Ns - 1)); break;
        case 4: dit_pass<4, T, MULTI, PAD>(s_line, L, nl, Ns, tw + (Ns - 1)); break;
        case 2: dit_pass<2, T, MULTI, PAD>(s_line, L, nl, Ns, tw + (Ns - 1)); break;
        case 3: dit_pass<3, T, MULTI, PAD>(s_line, L, nl, Ns, tw + (Ns - 1)); break;
        default: dit_pass<5, T, MULTI, PAD>(s_line, L, nl, Ns, tw + (Ns - 1)); break;
      }
      Ns *= R;
    }
    const int wl = p.win_len, lo = p.win_lo;
    if (p.out_mode == 0) {  // out[line][w]
      float2* const dst = out + l0 * p.out_stride;
      const int os = (int)p.out_stride;
      const float inv_wl = 1.0f / (float)wl;
      for (int e = tid; e < nh * wl; e += T) {
        const int l = MULTI ? quot(e, inv_wl) : 0, w = e - l * wl;
        const int m = lo + w < L ? lo + w : lo + w - L;
        dst[l * os + w] = s_line[padi<PAD>(l * L + m)];
      }
    } else {  // lines are (outer, inner), inner < t_inner: out[outer][w][inner]
      const int64_t outer0 = l0 / p.t_inner;
      const int inner0 = (int)(l0 - outer0 * p.t_inner);
      const int ti = (int)p.t_inner;
      float2* const dst = out + outer0 * wl * p.t_inner + inner0;
      const float inv_nh = 1.0f / (float)nh, inv_ti = 1.0f / (float)ti;
      for (int e = tid; e < nh * wl; e += T) {
        const int w = quot(e, inv_nh), l = e - w * nh;
        const int q = quot(inner0 + l, inv_ti);  // (inner0 + l) / t_inner
        const int m = lo + w < L ? lo + w : lo + w - L;
        dst[(q * wl + w) * ti + l - q * ti] = s_line[padi<PAD>(l * L + m)];
      }
    }
    __syncthreads();  // the lines are reused by the next group
  }
}

// out[c][r] = in[r][c] for an rows x cols matrix of complex64, 32 x 32 tiles.
__global__ __launch_bounds__(256) void transpose_c64_kernel(const float2* __restrict__ in, int64_t rows, int64_t cols,
                                                            float2* __restrict__ out) {
  __shared__ float2 tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
#pragma unroll
  for (int k = 0; k < 32; k += 8) {
    const int64_t r = r0 + ty + k, c = c0 + tx;
    if (r < rows && c < cols) tile[ty + k][tx] = in[r * cols + c];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 32; k += 8) {
    const int64_t c = c0 + ty + k, r = r0 + tx;
    if (r < rows && c < cols) out[c * rows + r] = tile[tx][ty + k];
  }
}

// Lines of at most kLineDftMax points as a direct pruned DFT on MFMA: the
// kept outputs of a block of 16 lines are one small dense product,
//   D[n][line] = sum_k A[n][k] B[k][line],
// B the lines' stored inputs as floats (k <-> float f of the line: re / im of
// input f / 2), A the real form of the table T (complex64, n_in x win_len,
// exp(+2 pi i f_i m_w / L) / psi_i): row n = 2 w + c gives the real (c = 0) or
// imaginary (c = 1) part of output w, A[2w][2i] = Re T, A[2w][2i+1] = -Im T,
// A[2w+1][2i] = Im T, A[2w+1][2i+1] = Re T.  One wave per 16-line block on
// v_mfma_f32_16x16x4f32 (A lane l = row l % 16 of k = 4 s + l / 16; B lane l
// = line l % 16; D register r of lane l = row 4 (l / 16) + r); K index
// k = 4 s + q is float q STEPS + s of the line, so lane (line, q) reads STEPS
// consecutive floats of its line and the table fragments stay in registers
// for the whole kernel.  D registers r, r + 1 are the real and imaginary part
// of one output: each lane stores whole complex values, 16 consecutive lines
// at a time.  STEPS = 2 n_in / 4; at most 8 blocks of 16 output rows.
template <int STEPS, int NBMAX>
__global__ __launch_bounds__(256) void line_dft_kernel(LineFft p, const float2* __restrict__ in,
                                                       const float2* __restrict__ tab, float2* __restrict__ out) {
  typedef float f32x4_t __attribute__((ext_vector_type(4)));
  // blocks of 16 lines per wave and step: all their inputs are requested
  // before the first product, so that a wave keeps G x 2 KB of reads in flight
  constexpr int G = 4;
  const int lane = threadIdx.x & 63, q = lane >> 4, r16 = lane & 15;
  const int wl = p.win_len, n_in = p.n_in;
  const int nb = (2 * wl + 15) / 16;  // blocks of 16 output rows (wave-uniform, <= NBMAX)
  float a[NBMAX][STEPS];
#pragma unroll
  for (int b = 0; b < NBMAX; ++b)
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
      const int n = 16 * b + r16, w = n >> 1, cn = n & 1;
      const int f = q * STEPS + s, i = f >> 1, cf = f & 1;
      float v = 0.0f;
      if (b < nb && w < wl && i < n_in) {
        const float2 t = tab[i * wl + w];
        v = cn == 0 ? (cf == 0 ? t.x : -t.y) : (cf == 0 ? t.y : t.x);
      }
      a[b][s] = v;
    }
  const int64_t n_blocks = (p.n_lines + 15) / 16;
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t blk0 = wave0 * G; blk0 < n_blocks; blk0 += n_waves * G) {
    float x[G][STEPS];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t line = (blk0 + g) * 16 + r16;
      const bool live = line < p.n_lines;
      const float* const src = reinterpret_cast<const float*>(in + (live ? line : 0) * p.in_stride) + q * STEPS;
      if constexpr (STEPS % 4 == 0) {  // 16-byte aligned runs: vector loads
#pragma unroll
        for (int s = 0; s < STEPS; s += 4) {
          const float4 v = live ? *reinterpret_cast<const float4*>(src + s) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
          x[g][s] = v.x;
          x[g][s + 1] = v.y;
          x[g][s + 2] = v.z;
          x[g][s + 3] = v.w;
        }
      } else {
#pragma unroll
        for (int s = 0; s < STEPS; ++s) x[g][s] = live ? src[s] : 0.0f;
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t line = (blk0 + g) * 16 + r16;
      f32x4_t d[NBMAX];
#pragma unroll
      for (int b = 0; b < NBMAX; ++b) {
        d[b] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
        if (b < nb)
#pragma unroll
          for (int s = 0; s < STEPS; ++s)
            d[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b][s], x[g][s], d[b], 0, 0, 0);
      }
      if (line >= p.n_lines) continue;
      float2* dst;
      int64_t wstride;
      if (p.out_mode == 0) {
        dst = out + line * p.out_stride;
        wstride = 1;
      } else {  // line = outer * t_inner + inner, stored at [outer][w][inner]
        const int64_t outer = line / p.t_inner, inner = line - outer * p.t_inner;
        dst = out + outer * wl * p.t_inner + inner;
        wstride = p.t_inner;
      }
#pragma unroll
      for (int b = 0; b < NBMAX; ++b)
#pragma unroll
        for (int h = 0; h < 2; ++h) {  // registers 2 h, 2 h + 1: output w = 8 b + 2 q + h
          const int w = 8 * b + 2 * q + h;
          if (b < nb && w < wl) dst[w * wstride] = make_float2(d[b][2 * h], d[b][2 * h + 1]);
        }
    }
  }
}

}  // namespace

void line_dft_table(const LineFft& p, const float* inv_psi, float* tab) {
  const int half = p.n_in / 2;
  for (int i = 0; i < p.n_in; ++i) {
    const int f = i < half ? i : i - p.n_in;
    for (int w = 0; w < p.win_len; ++w) {
      const int m = (p.win_lo + w) % p.L;
      // the angle's numerator reduced mod L first: exact in integers
      const int64_t fm = (((int64_t)f * m) % p.L + p.L) % p.L;
      const double a = 2.0 * M_PI * (double)fm / p.L;
      tab[2 * ((size_t)i * p.win_len + w)] = (float)(std::cos(a) * inv_psi[i]);
      tab[2 * ((size_t)i * p.win_len + w) + 1] = (float)(std::sin(a) * inv_psi[i]);
    }
  }
}

bool line_dft_fits(const LineFft& p) {
  // 2 n_in floats per line in 4 lane groups (2 <= STEPS <= 16), at most 8 blocks of 16 output rows
  return p.L <= kLineDftMax && p.n_in % 2 == 0 && p.n_in >= 4 && p.n_in <= 32 && p.win_len >= 1 &&
         2 * p.win_len <= 128;
}

hipError_t launch_line_dft(const LineFft& p, const void* in, const float2* tab, void* out, hipStream_t s) {
  if (p.n_lines <= 0) return hipSuccess;
  if (!line_dft_fits(p)) return hipErrorInvalidValue;
  // the vector loads of runs of 4 floats need 16-byte aligned lines
  if ((p.n_in / 2) % 4 == 0 && ((p.in_stride * 8) % 16 != 0 || reinterpret_cast<uintptr_t>(in) % 16 != 0))
    return hipErrorInvalidValue;
  const int64_t waves = (p.n_lines + 63) / 64;  // four 16-line blocks per wave and step
  const unsigned grid = (unsigned)std::min<int64_t>((waves + 3) / 4, 1 << 16);
  const float2* const x = static_cast<const float2*>(in);
  float2* const y = static_cast<float2*>(out);
  const bool narrow = 2 * p.win_len <= 64;  // at most 4 blocks of 16 output rows
#define BB_DFT_CASE(S)                                                                                  \
  case S:                                                                                               \
    if (narrow)                                                                                         \
      hipLaunchKernelGGL((line_dft_kernel<S, 4>), dim3(grid), dim3(256), 0, s, p, x, tab, y);           \
    else                                                                                                \
      hipLaunchKernelGGL((line_dft_kernel<S, 8>), dim3(grid), dim3(256), 0, s, p, x, tab, y);           \
    break;
  switch (p.n_in / 2) {
    BB_DFT_CASE(2) BB_DFT_CASE(3) BB_DFT_CASE(4) BB_DFT_CASE(5) BB_DFT_CASE(6) BB_DFT_CASE(7) BB_DFT_CASE(8)
    BB_DFT_CASE(9) BB_DFT_CASE(10) BB_DFT_CASE(11) BB_DFT_CASE(12) BB_DFT_CASE(13) BB_DFT_CASE(14)
    BB_DFT_CASE(15) BB_DFT_CASE(16)
    default: return hipErrorInvalidValue;
  }
#undef BB_DFT_CASE
  return hipGetLastError();
}

int line_fft_plan(int L, LineFft& p) {
  if (L < 2 || L > kLineFftMax) return -1;
  int m = L, n2 = 0, n3 = 0, n5 = 0;
  while (m % 2 == 0) m /= 2, ++n2;
  while (m % 3 == 0) m /= 3, ++n3;
  while (m % 5 == 0) m /= 5, ++n5;
  if (m != 1) return -1;
  int rad[32], n = 0;
  while (n2 > 4 || n2 == 3) rad[n++] = 8, n2 -= 3;
  if (n2 == 4) rad[n++] = 4, rad[n++] = 4;
  if (n2 == 2) rad[n++] = 4;
  if (n2 == 1) rad[n++] = 2;
  for (int i = 0; i < n3; ++i) rad[n++] = 3;
  for (int i = 0; i < n5; ++i) rad[n++] = 5;
  if (n > 16) return -1;
  p.L = L;
  p.n_pass = n;
  p.radix_codes = 0;
  for (int i = 0; i < n; ++i) p.radix_codes |= (uint64_t)rad[i] << (4 * i);
  p.nl = std::max(1, 4096 / L);
  return 0;
}

// Padding pays for long lines with at least 2^6 in their length (4608: 0.92
// against 1.02 ms per call on the 1024^2 benchmark grid); for the others
// (4500 = 2^2 3^2 5^3) the extra index work outweighs it.
static bool fft_pad(const LineFft& p) { return p.nl == 1 && p.L % 64 == 0; }
size_t line_fft_lds_bytes(const LineFft& p) {
  const size_t n = (size_t)p.nl * p.L;
  return (fft_pad(p) ? n + (n >> 5) + 2 : n) * sizeof(float2);
}

void line_fft_twiddles(const LineFft& p, float* tw) {
  int ns = 1;
  for (int s = 0; s < p.n_pass; ++s) {
    const int R = (int)((p.radix_codes >> (4 * s)) & 15), P = ns * R;
    float* t = tw + 2 * (size_t)(ns - 1);
    for (int k = 0; k < ns; ++k)
      for (int r = 1; r < R; ++r) {
        const double a = 2.0 * M_PI * (double)(k * r) / P;
        t[2 * (k * (R - 1) + r - 1)] = (float)std::cos(a);
        t[2 * (k * (R - 1) + r - 1) + 1] = (float)std::sin(a);
      }
    ns = P;
  }
}

void line_fft_perm(const LineFft& p, int* perm) {
  int rad[16], span[16];
  int ns = 1;
  for (int s = 0; s < p.n_pass; ++s) {
    rad[s] = (int)((p.radix_codes >> (4 * s)) & 15);
    span[s] = ns;
    ns *= rad[s];
  }
  for (int n = 0; n < p.L; ++n) {
    int rem = n, pos = 0;
    for (int s = p.n_pass - 1; s >= 0; --s) {
      pos += (rem % rad[s]) * span[s];
      rem /= rad[s];
    }
    perm[n] = pos;
  }
}

hipError_t launch_line_fft(const LineFft& p, const void* in, const float* inv_psi, const int* perm, const float2* tw,
                           void* out, hipStream_t s) {
  if (p.n_lines <= 0) return hipSuccess;
  const int64_t groups = (p.n_lines + p.nl - 1) / p.nl;
  const unsigned grid = (unsigned)std::min<int64_t>(groups, 1 << 16);
  const size_t lds = line_fft_lds_bytes(p);
  const bool pad = fft_pad(p);
  const void* const fn = p.nl > 1 ? reinterpret_cast<const void*>(&line_fft_kernel<512, true, false>)
                                  : (pad ? reinterpret_cast<const void*>(&line_fft_kernel<512, false, true>)
                                         : reinterpret_cast<const void*>(&line_fft_kernel<512, false, false>));
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (p.nl > 1)
    hipLaunchKernelGGL((line_fft_kernel<512, true, false>), dim3(grid), dim3(512), lds, s, p, static_cast<const float2*>(in),
                       inv_psi, perm, tw, static_cast<float2*>(out));
  else if (pad)
    hipLaunchKernelGGL((line_fft_kernel<512, false, true>), dim3(grid), dim3(512), lds, s, p,
                       static_cast<const float2*>(in), inv_psi, perm, tw, static_cast<float2*>(out));
  else
    hipLaunchKernelGGL((line_fft_kernel<512, false, false>), dim3(grid), dim3(512), lds, s, p,
                       static_cast<const float2*>(in), inv_psi, perm, tw, static_cast<float2*>(out));
  return hipGetLastError();
}

hipError_t launch_transpose_c64(const void* in, int64_t rows, int64_t cols, void* out, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
  hipLaunchKernelGGL(transpose_c64_kernel, grid, dim3(256), 0, s, static_cast<const float2*>(in), rows, cols,
                     static_cast<float2*>(out));
  return hipGetLastError();
}

}  // namespace bb
