// Backward of the level images of one instance.
//
// Loss = sum_l sum_p g_lp I_lp with I_lp = sum_{k in l} d_k |E_kp|^2, E = W^H B,
// B_lp = exp(+j 2 pi <x_l, p> / lambda_w) (Sections 2.4 and 2.6).  With
// c_kp = g_{level(k), p}:
//   dd_k  = sum_p c_kp |E_kp|^2
//   M_kp  = d_k c_kp conj(E_kp)
//   dW_lk = 2 sum_p B_lp M_kp            (d/dRe W + j d/dIm W)
//   H_lp  = sum_k conj(W_lk) M_kp
//   dx_l  = -(4 pi / lambda_w) sum_p Im(H_lp B_lp) p
// E is recomputed by the forward MFMA kernel (FP32, three products) into HBM; the
// contractions dW and H run on FP32 MFMA (32x32x2), in one kernel sharing its
// staged phases and M when every eigenpair fits one 64-wide slice, in two
// otherwise.  The kernels work in level-sorted eigenpair order (the staging
// permutation) and
// the reduction writes results back in the caller's order.  Contractions over
// pixels are split into fixed pixel ranges whose FP64 partials are summed in a
// fixed order: the result is deterministic.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bb_internal.h"

namespace bb {

// Same phase evaluation as the forward kernels: xs = position / wavelength,
// exact FP64 reduction to [-1/2, 1/2] turns, hardware sine and cosine in turns.
__device__ __forceinline__ void phase_b(const double* __restrict__ xs, double px, double py, double pz, float& c,
                                        float& s) {
  const double t = fma(xs[2], pz, fma(xs[1], py, xs[0] * px));
  const float f = (float)(t - rint(t));
  s = __builtin_amdgcn_sinf(f);
  c = __builtin_amdgcn_cosf(f);
}

template <int N>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < N / 64; ++i) t += sh[i];
  __syncthreads();
  return t;
}

// M = d c conj(E) in place, dd partial sums; grid (K_alloc, n_split), 256 threads.
__global__ __launch_bounds__(256) void bwd_m_kernel(const BwdParams P) {
  __shared__ double sh[4];
  const int k = blockIdx.x;
  const int s = blockIdx.y;
  const InstDesc& D = *P.desc;
  const int lev = D.levs[k];
  const float w = D.wts[k];
  float* er = P.E + (int64_t)k * P.n_pix;
  float* ei = P.E + (int64_t)(P.K_alloc + k) * P.n_pix;
  const int64_t p0 = (int64_t)s * P.split_len;
  int64_t p1 = p0 + P.split_len;
  if (p1 > P.n_pix) p1 = P.n_pix;
  double acc = 0.0;
  if (lev < 0) {
    // padding / unused rows (the recompute leaves rows past K_pad unwritten)
    for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
      er[p] = 0.0f;
      ei[p] = 0.0f;
    }
  } else {
    for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
      const float c = P.gimg[(int64_t)lev * P.gimg_ld + p];
      const float a = er[p], b = ei[p];
      acc += (double)(c * fmaf(a, a, b * b));
      er[p] = w * c * a;
      ei[p] = -w * c * b;
    }
  }
  const double t = block_sum<256>(acc, sh);
  if (threadIdx.x == 0) P.dd_part[(int64_t)k * P.n_split + s] = t;
}

// dW partial: sum over the split's pixels of B_lp M_kp for a 32 x 64 (l, k)
// tile of two 32-eigenpair blocks, on MFMA.  grid (L_pad/32,
// ceil(K_alloc/64), n_split), 256 threads.  Each 64-pixel chunk stages
// phases [64 px][32 l] and M [64 px][64 k] in LDS; wave w contracts pixels
// 16 w .. 16 w + 15 of it as 8 steps of 32x32x2 MFMAs per block (A = B
// phases, rows l; B = M, columns k):
//   Re += Br Mr - Bi Mi,  Im += Br Mi + Bi Mr.
// Two blocks per workgroup share each phase evaluation; the second is absent
// (workgroup-uniform) when K_alloc is an odd multiple of 32.  The next
// chunk's M and pixel coordinates are loaded into registers while the
// current chunk is processed.  The four waves' partial tiles are summed in a
// fixed order at the end.
typedef float bwd_f32x16 __attribute__((ext_vector_type(16)));

// One chunk's H block of a wave: H[l][p] += sum over 64 eigenpairs of
// conj(W)[l][k] M[k][p] for pixels 32 blk .. 32 blk + 31, real part (PART 0:
// Wr' Mr - Wi' Mi) or imaginary part (PART 1: Wr' Mi + Wi' Mr), W' = conj W.
// PART is a template argument and the loop is unrolled whole, so that it holds
// no branch: its LDS reads then run ahead of the MFMAs instead of each step
// waiting for its own.
// The real part takes -Wi' from the staged plane sWn (no negation per step).
template <int PART>
__device__ __forceinline__ void h_chunk(bwd_f32x16& h, const float2 (*sW)[65], const float (*sWn)[65],
                                        const float2 (*sM)[65], int blk, int lane) {
#pragma unroll
  for (int st = 0; st < 32; ++st) {
    const int kk = 2 * st + (lane >> 5);              // this lane's contraction row (eigenpair)
    const float2 w = sW[lane & 31][kk];               // A operand: row l = lane % 32
    const float2 m = sM[kk][32 * blk + (lane & 31)];  // B operand: column p = lane % 32 of the half
    if (PART == 0) {
      h = __builtin_amdgcn_mfma_f32_32x32x2f32(w.x, m.x, h, 0, 0, 0);
      h = __builtin_amdgcn_mfma_f32_32x32x2f32(sWn[lane & 31][kk], m.y, h, 0, 0, 0);
    } else {
      h = __builtin_amdgcn_mfma_f32_32x32x2f32(w.x, m.y, h, 0, 0, 0);
      h = __builtin_amdgcn_mfma_f32_32x32x2f32(w.y, m.x, h, 0, 0, 0);
    }
  }
}

// h_chunk for a W that stays the same over the chunks: the real part takes
// -Wi' from registers (wny[st] for this lane's row of step st), loaded once.
template <int PART>
__device__ __forceinline__ void h_chunk_w(bwd_f32x16& h, const float2 (*sW)[65], const float (&wny)[32],
                                          const float2 (*sM)[65], int blk, int lane) {
#pragma unroll
  for (int st = 0; st < 32; ++st) {
    const int kk = 2 * st + (lane >> 5);
    const float2 m = sM[kk][32 * blk + (lane & 31)];
    if (PART == 0) {
      h = __builtin_amdgcn_mfma_f32_32x32x2f32(sW[lane & 31][kk].x, m.x, h, 0, 0, 0);
      h = __builtin_amdgcn_mfma_f32_32x32x2f32(wny[st], m.y, h, 0, 0, 0);
    } else {
      const float2 w = sW[lane & 31][kk];
      h = __builtin_amdgcn_mfma_f32_32x32x2f32(w.x, m.y, h, 0, 0, 0);
      h = __builtin_amdgcn_mfma_f32_32x32x2f32(w.y, m.x, h, 0, 0, 0);
    }
  }
}

// h_chunk over conj(W) staged once for every eigenpair of the instance (rows
// of WS, this slice's columns kc .. kc + 63); the real part negates Wi' per
// step.
template <int PART, int WS>
__device__ __forceinline__ void h_chunk_all(bwd_f32x16& h, const float2 (*sW)[WS], int kc, const float2 (*sM)[65],
                                            int blk, int lane) {
#pragma unroll
  for (int st = 0; st < 32; ++st) {
    const int kk = 2 * st + (lane >> 5);
    const float2 w = sW[lane & 31][kc + kk];
    const float2 m = sM[kk][32 * blk + (lane & 31)];
    if (PART == 0) {
      h = __builtin_amdgcn_mfma_f32_32x32x2f32(w.x, m.x, h, 0, 0, 0);
      h = __builtin_amdgcn_mfma_f32_32x32x2f32(-w.y, m.y, h, 0, 0, 0);
    } else {
      h = __builtin_amdgcn_mfma_f32_32x32x2f32(w.x, m.y, h, 0, 0, 0);
      h = __builtin_amdgcn_mfma_f32_32x32x2f32(w.y, m.x, h, 0, 0, 0);
    }
  }
}

// One chunk's dW block of a wave: dW[l][k] += sum over the chunk's 64 pixels
// of B[p][l] M[k][p] for eigenpairs 32 blk .. 32 blk + 31, real part (PART 0:
// Br Mr - Bi Mi) or imaginary part (PART 1: Br Mi + Bi Mr).
// The real part takes -Bi from the staged plane sBn (no negation per step).
template <int PART>
__device__ __forceinline__ void dw_chunk(bwd_f32x16& dw, const float2 (*sB)[32], const float (*sBn)[32],
                                         const float2 (*sM)[65], int blk, int lane) {
#pragma unroll
  for (int st = 0; st < 32; ++st) {
    const int pp = 2 * st + (lane >> 5);
    const float2 b = sB[pp][lane & 31];
    const float2 m = sM[32 * blk + (lane & 31)][pp];
    if (PART == 0) {
      dw = __builtin_amdgcn_mfma_f32_32x32x2f32(b.x, m.x, dw, 0, 0, 0);
      dw = __builtin_amdgcn_mfma_f32_32x32x2f32(sBn[pp][lane & 31], m.y, dw, 0, 0, 0);
    } else {
      dw = __builtin_amdgcn_mfma_f32_32x32x2f32(b.x, m.y, dw, 0, 0, 0);
      dw = __builtin_amdgcn_mfma_f32_32x32x2f32(b.y, m.x, dw, 0, 0, 0);
    }
  }
}

// One chunk's dW steps of a wave for both eigenpair blocks.
__device__ __forceinline__ void dw2_chunk(bwd_f32x16 (&are)[2], bwd_f32x16 (&aim)[2], const float2 (*sB)[32],
                                          const float2 (*sM)[65], int wave, int lane) {
#pragma unroll
  for (int st = 0; st < 8; ++st) {
    const int pp = 16 * wave + 2 * st + (lane >> 5);  // this lane's contraction row (pixel)
    const float2 b = sB[pp][lane & 31];               // A operand: row l = lane % 32
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const float2 m = sM[pp][32 * q + (lane & 31)];  // B operand: column k = lane % 32 of block q
      are[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(b.x, m.x, are[q], 0, 0, 0);
      are[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(-b.y, m.y, are[q], 0, 0, 0);
      aim[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(b.x, m.y, aim[q], 0, 0, 0);
      aim[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(b.y, m.x, aim[q], 0, 0, 0);
    }
  }
}

__global__ __launch_bounds__(256) void bwd_dw_kernel(const BwdParams P) {
  __shared__ float2 sB[64][32];
  __shared__ float2 sM[64][65];  // [pixel][eigenpair] (+1 pad: the staging writes run along pixels)
  __shared__ double sP[3][64];   // the chunk's pixel coordinates
  __shared__ double sX[32][4];   // the tile's scaled antenna positions
  const InstDesc& D = *P.desc;
  const int l0 = blockIdx.x * 32, k0 = blockIdx.y * 64, s = blockIdx.z;
  const bool two = k0 + 32 < P.K_alloc;  // the second eigenpair block exists
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if (t < 128) (&sX[0][0])[t] = D.xs[4 * l0 + t];  // rows l0 .. l0 + 31 < L_pad
  const int64_t p0 = (int64_t)s * P.split_len;
  int64_t p1 = p0 + P.split_len;
  if (p1 > P.n_pix) p1 = P.n_pix;
  const float* Er = P.E;
  const float* Ei = P.E + (int64_t)P.K_alloc * P.n_pix;
  // the next chunk's M (16 values per thread: eigenpair k0 + 4 j + t / 64,
  // pixel t % 64; rows up to K_alloc hold M or zeros, an absent second block
  // reads row k0 and keeps zeros) and pixel coordinates (threads < 192: axis
  // t / 64); lanes past the split load the split's last pixel and keep zeros
  float2 mnext[16];
  double pnext = 0.0;
  auto load_chunk = [&](int64_t pc) {
    const int64_t p = pc + (t & 63);
    const bool p_ok = p < p1;
    const int64_t pq = p_ok ? p : p1 - 1;
    const int64_t r0 = (int64_t)(k0 + (t >> 6)) * P.n_pix + pq, st4 = 4 * P.n_pix;  // rows advance by 4 per j
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const bool k_ok = j < 8 || two;
      const int64_t e = k_ok ? r0 + j * st4 : pq;
      const float er = Er[e], ei = Ei[e];
      mnext[j] = (p_ok && k_ok) ? make_float2(er, ei) : make_float2(0.0f, 0.0f);
    }
    if (t < 192) pnext = p_ok ? P.pix[pq + (t >> 6) * P.pix_ld] : 0.0;
  };
  load_chunk(p0);
  bwd_f32x16 are[2], aim[2];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) are[q][r] = aim[q][r] = 0.0f;
  for (int64_t pc = p0; pc < p1; pc += 64) {
#pragma unroll
    for (int j = 0; j < 16; ++j) sM[t & 63][4 * j + (t >> 6)] = mnext[j];
    if (t < 192) sP[t >> 6][t & 63] = pnext;
    __syncthreads();
    if (pc + 64 < p1) load_chunk(pc + 64);  // workgroup-uniform
    // phases: 32 antennas x 64 pixels, 8 per thread (zero past the split)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = t + 256 * j;
      const int pp = i >> 5, ll = i & 31;
      float c, sn;
      phase_b(&sX[ll][0], sP[0][pp], sP[1][pp], sP[2][pp], c, sn);
      sB[pp][ll] = pc + pp < p1 ? make_float2(c, sn) : make_float2(0.0f, 0.0f);
    }
    __syncthreads();
    dw2_chunk(are, aim, sB, sM, wave, lane);  // an absent second block multiplies zeros
    __syncthreads();
  }
  // fixed-order sum of the four waves' tiles, one block at a time: wave w's
  // register r of lane q holds (l, k) = (8 (r / 4) + 4 (q / 32) + r % 4, q % 32)
  float* const red = reinterpret_cast<float*>(&sB[0][0]);  // [4 waves][16 regs][64 lanes] re, then im in sM
  float* const redi = reinterpret_cast<float*>(&sM[0][0]);
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    if (b == 1 && !two) break;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      red[(wave * 16 + r) * 64 + lane] = are[b][r];
      redi[(wave * 16 + r) * 64 + lane] = aim[b][r];
    }
    __syncthreads();
    for (int i = t; i < 16 * 64; i += 256) {
      const int r = i >> 6, q = i & 63;
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        re += red[(w * 16 + r) * 64 + q];
        im += redi[(w * 16 + r) * 64 + q];
      }
      const int l = 8 * (r >> 2) + 4 * (q >> 5) + (r & 3), k = 32 * b + (q & 31);
      double* out = P.dW_part + (((int64_t)s * P.L_pad + (l0 + l)) * P.K_alloc + k0 + k) * 2;
      out[0] = re;
      out[1] = im;
    }
    __syncthreads();
  }
}

// dx partial: H_lp = sum_k conj(W_lk) M_kp on MFMA, then Im(H_lp B_lp) p
// summed over the split's pixels.  grid (L_pad/32, n_split), 256 threads.  The
// work runs in steps (64-pixel chunk, 64-eigenpair slice); each step stages
// conj(W) [32 l][64 k] and M [64 k][64 p] in LDS from registers loaded during
// the step before.  Wave w computes one real 32 x 32 block of H: pixel half
// w / 2, real part (w even: Wr Mr - Wi' Mi with W' = conj W) or imaginary part
// (w odd: Wr' Mi + Wi' Mr).  After a chunk's last slice the blocks go through
// LDS (pixel-major, rows padded to 33) to the threads that own (antenna t % 32,
// pixels t / 32 + 8 j), which evaluate the phases.  WONCE (K_alloc <= 128):
// conj(W) of all the instance's eigenpairs is staged once, and the steps
// stage only M.
template <bool WONCE>
__global__ __launch_bounds__(256) void bwd_dx_kernel(const BwdParams P) {
  __shared__ float2 sW[32][65];   // conj(W) for 32 antennas x 64 eigenpairs (+1 pad: column reads)
  __shared__ float sWn[32][65];   // its negated imaginary parts
  __shared__ float2 sM[64][65];   // M for 64 eigenpairs x 64 pixels; then H re / im [2][64 p][33] floats
  __shared__ double sP[3][64];    // the chunk's pixel coordinates
  __shared__ double sX[32][4];    // the tile's scaled antenna positions
  __shared__ double sh[3][256];
  __shared__ int sOff[kMaxEig];   // staged eigenpair -> offset of its column of W (src * L), -1 if none
  __shared__ float2 sWall[32][129];  // WONCE: conj(W) for 32 antennas x 128 eigenpairs (+1 pad)
  const InstDesc& D = *P.desc;
  const int l0 = blockIdx.x * 32, s = blockIdx.y;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int tl = t & 31, tp = t >> 5;
  const int l = l0 + tl;
  if (t < 128) (&sX[0][0])[t] = D.xs[4 * l0 + t];  // rows l0 .. l0 + 31 < L_pad
  // this wave's H block: pixel half, re / im (wave-uniform, held in scalar registers)
  const int blk = __builtin_amdgcn_readfirstlane(wave >> 1), part = __builtin_amdgcn_readfirstlane(wave & 1);
  const int64_t p0 = (int64_t)s * P.split_len;
  int64_t p1 = p0 + P.split_len;
  if (p1 > P.n_pix) p1 = P.n_pix;
  const int K_pad = P.dyn->K_pad;
  const int n_kc = K_pad > 64 ? (K_pad + 63) / 64 : 1;  // slices per chunk (one of zeros if K_pad = 0)
  const float* Er = P.E;
  const float* Ei = P.E + (int64_t)P.K_alloc * P.n_pix;
  const float* Wf = (const float*)P.W;
  float* const sH = reinterpret_cast<float*>(&sM[0][0]);  // [2 parts][64 p][33]
  // The next step's M (16 values per thread: eigenpair 4 j + t / 64 of the
  // slice, pixel t % 64), conj(W) (8 per thread: antenna t % 32, eigenpair
  // t / 32 + 8 j of the slice, so that a wave reads 32 consecutive antennas
  // of a column of W) and, for a new chunk, pixel coordinates.  Lanes outside
  // the split, K_pad or the antennas load a valid address and keep zeros.
  float2 mnext[16], wnext[8];
  double pnext = 0.0;
  auto load_step = [&](int64_t pc, int kc) {
    const int64_t p = pc + (t & 63);
    const bool p_ok = p < p1;
    const int64_t pq = p_ok ? p : p1 - 1;
    const int64_t r0 = (int64_t)(kc + (t >> 6)) * P.n_pix + pq, st4 = 4 * P.n_pix;  // rows advance by 4 per j
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int k = kc + 4 * j + (t >> 6);
      const int64_t e = k < K_pad ? r0 + j * st4 : pq;
      const float er = Er[e], ei = Ei[e];
      mnext[j] = (p_ok && k < K_pad) ? make_float2(er, ei) : make_float2(0.0f, 0.0f);
    }
    const bool l_ok = l0 + tl < P.L;
#pragma unroll
    for (int j = 0; j < 8 && !WONCE; ++j) {
      const int k = kc + tp + 8 * j;
      const int off = sOff[k];
      const bool ok = l_ok && off >= 0;
      const float* w = Wf + 2 * ((int64_t)(ok ? off : 0) + (l_ok ? l0 + tl : 0));
      float wr = w[0], wi = w[1];
      // keep the loads unconditional (a load the compiler moves under `ok`
      // becomes a branch per element)
      asm volatile("" : "+v"(wr), "+v"(wi));
      wnext[j] = ok ? make_float2(wr, -wi) : make_float2(0.0f, 0.0f);
    }
    if (kc == 0 && t < 192) pnext = p_ok ? P.pix[pq + (t >> 6) * P.pix_ld] : 0.0;
  };
  if constexpr (WONCE) {
    for (int i = t; i < 32 * 128; i += 256) {
      const int ll = i & 31, kk = i >> 5;  // a wave reads 32 consecutive antennas of two columns of W
      const int src = kk < K_pad ? D.perm[kk] : -1;
      float2 wv = make_float2(0.0f, 0.0f);
      if (l0 + ll < P.L && src >= 0) {
        const float* w = Wf + 2 * ((int64_t)src * P.L + l0 + ll);
        wv = make_float2(w[0], -w[1]);
      }
      sWall[ll][kk] = wv;
    }
  } else {
    for (int k = t; k < 64 * n_kc; k += 256) {  // 64 n_kc <= kMaxEig
      const int src = k < K_pad ? D.perm[k] : -1;
      sOff[k] = src >= 0 ? src * P.L : -1;
    }
  }
  __syncthreads();
  load_step(p0, 0);
  double gx = 0.0, gy = 0.0, gz = 0.0;
  for (int64_t pc = p0; pc < p1; pc += 64) {
    bwd_f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    for (int kq = 0; kq < n_kc; ++kq) {
#pragma unroll
      for (int j = 0; j < 16; ++j) sM[4 * j + (t >> 6)][t & 63] = mnext[j];
      if constexpr (!WONCE) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          sW[tl][tp + 8 * j] = wnext[j];
          sWn[tl][tp + 8 * j] = -wnext[j].y;
        }
      }
      if (kq == 0 && t < 192) sP[t >> 6][t & 63] = pnext;
      __syncthreads();
      // the next step: the chunk's next slice, else the next chunk's first
      const bool last = kq + 1 == n_kc;
      const int64_t npc = last ? pc + 64 : pc;
      if (npc < p1) load_step(npc, last ? 0 : 64 * (kq + 1));  // workgroup-uniform
      if constexpr (WONCE) {
        if (part == 0)
          h_chunk_all<0, 129>(acc, sWall, 64 * kq, sM, blk, lane);
        else
          h_chunk_all<1, 129>(acc, sWall, 64 * kq, sM, blk, lane);
      } else {
        if (part == 0)
          h_chunk<0>(acc, sW, sWn, sM, blk, lane);
        else
          h_chunk<1>(acc, sW, sWn, sM, blk, lane);
      }
      __syncthreads();
    }
    // register r of lane q holds H at (l, p) = (8 (r / 4) + 4 (q / 32) + r % 4, 32 blk + q % 32)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int ll = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      sH[(part * 64 + 32 * blk + (lane & 31)) * 33 + ll] = acc[r];
    }
    __syncthreads();
    if (l < P.L) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        // pixels past the split add exact zeros (their M and hence H, and
        // coordinates are 0)
        const int pp = tp + 8 * j;
        const double px = sP[0][pp], py = sP[1][pp], pz = sP[2][pp];
        float c, sn;
        phase_b(&sX[tl][0], px, py, pz, c, sn);
        const float hr = sH[pp * 33 + tl], hi = sH[(64 + pp) * 33 + tl];
        const double v = (double)fmaf(hr, sn, hi * c);  // Im(H B)
        gx += v * px;
        gy += v * py;
        gz += v * pz;
      }
    }
    __syncthreads();  // sH (in sM) and sP are restaged by the next chunk
  }
  sh[0][t] = gx;
  sh[1][t] = gy;
  sh[2][t] = gz;
  __syncthreads();
  if (tp == 0 && l < P.L_pad) {
    double a = 0, b = 0, c = 0;
    for (int j = 0; j < 8; ++j) {
      a += sh[0][t + 32 * j];
      b += sh[1][t + 32 * j];
      c += sh[2][t + 32 * j];
    }
    double* o = P.dx_part + ((int64_t)s * P.L_pad + l) * 3;
    o[0] = a;
    o[1] = b;
    o[2] = c;
  }
}

// dW and dx partials together when every eigenpair fits one 64-wide slice
// (K_alloc <= 64): each 64-pixel chunk's phases [64 p][32 l] and M [64 k][64 p]
// are staged once and serve both contractions.  grid (L_pad/32, n_split), 256
// threads; wave w owns
//   the dW block of eigenpairs 32 (w / 2) .. + 31, part w % 2 (re / im),
//     accumulated over the split (A = phases, rows l; B = M, columns k);
//   the H block of pixels 32 (w / 2) .. + 31 of the chunk, part w % 2
//     (A = conj(W), rows l; B = M, columns p).
// H goes through LDS to the threads that own (antenna t % 32, pixels t / 32 + 8 j),
// which form Im(H B) p with the staged phases.  The next chunk's M and pixel
// coordinates are loaded into registers while the current chunk is processed.
__global__ __launch_bounds__(256) void bwd_fused_kernel(const BwdParams P) {
  __shared__ float2 sW[32][65];   // conj(W) [32 l][64 k], staged once (+1 pad: column reads)
  __shared__ float2 sM[64][65];   // M [64 k][64 p] (+1 pad: column reads); then H re / im [2][64 p][33] floats
  __shared__ float2 sB[64][32];   // phases [64 p][32 l]
  __shared__ float sBn[64][32];   // their negated sines
  __shared__ double sP[3][64];    // the chunk's pixel coordinates
  __shared__ double sX[32][4];    // the tile's scaled antenna positions, staged once
  const InstDesc& D = *P.desc;
  const int l0 = blockIdx.x * 32, s = blockIdx.y;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  // Im(H B) p: consecutive lanes take consecutive antennas, so the reads of
  // the phases and of H (stored pixel-major, rows padded to 33) are free of
  // bank conflicts
  const int tl = t & 31, tp = t >> 5;
  const int l = l0 + tl;
  const int blk = __builtin_amdgcn_readfirstlane(wave >> 1), part = __builtin_amdgcn_readfirstlane(wave & 1);
  const bool dw_active = 32 * blk < P.K_alloc;  // this wave's dW block exists
  const int64_t p0 = (int64_t)s * P.split_len;
  int64_t p1 = p0 + P.split_len;
  if (p1 > P.n_pix) p1 = P.n_pix;
  const int K_pad = P.dyn->K_pad;
  const float* Er = P.E;
  const float* Ei = P.E + (int64_t)P.K_alloc * P.n_pix;
  const float* Wf = (const float*)P.W;
  float* const sH = reinterpret_cast<float*>(&sM[0][0]);  // [2 parts][64 p][33]
  if (t < 128) (&sX[0][0])[t] = D.xs[4 * l0 + t];            // rows l0 .. l0 + 31 < L_pad
  for (int i = t; i < 32 * 64; i += 256) {
    const int ll = i & 31, kk = i >> 5;  // a wave reads 32 consecutive antennas of two columns of W
    float2 wv = make_float2(0.0f, 0.0f);
    if (l0 + ll < P.L && kk < K_pad) {
      const int src = D.perm[kk];
      if (src >= 0) {
        const float* w = Wf + 2 * ((int64_t)src * P.L + l0 + ll);
        wv = make_float2(w[0], -w[1]);
      }
    }
    sW[ll][kk] = wv;
  }
  // the next chunk's M (16 values per thread: eigenpair 4 j + t / 64, pixel
  // t % 64) and pixel coordinates (threads < 192: axis t / 64, pixel t % 64)
  // are loaded into registers while the current chunk is processed
  float2 mnext[16];
  double pnext = 0.0;
  // Every lane loads (pixels past the split and eigenpairs past K_pad from
  // row 0 and the split's last pixel) and then zeroes what lies outside, so
  // the loads carry no branches.
  auto load_chunk = [&](int64_t pc) {
    const int pp = t & 63;
    const int64_t p = pc + pp;
    const bool p_ok = p < p1;
    const int64_t pq = p_ok ? p : p1 - 1;
    const int64_t r0 = (int64_t)(t >> 6) * P.n_pix + pq, st4 = 4 * P.n_pix;  // rows advance by 4 per j
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int kk = 4 * j + (t >> 6);
      const int64_t e = kk < K_pad ? r0 + j * st4 : pq;
      const float er = Er[e], ei = Ei[e];
      mnext[j] = (p_ok && kk < K_pad) ? make_float2(er, ei) : make_float2(0.0f, 0.0f);
    }
    if (t < 192) pnext = p_ok ? P.pix[pq + (t >> 6) * P.pix_ld] : 0.0;
  };
  load_chunk(p0);
  // -Im conj(W) of this lane's rows, for the real part of H (waves of part 0)
  float wny[32];
  __syncthreads();  // conj(W) is staged
  if (part == 0)
#pragma unroll
    for (int st = 0; st < 32; ++st) wny[st] = -sW[lane & 31][2 * st + (lane >> 5)].y;
  bwd_f32x16 dw;
#pragma unroll
  for (int r = 0; r < 16; ++r) dw[r] = 0.0f;
  double gx = 0.0, gy = 0.0, gz = 0.0;
  for (int64_t pc = p0; pc < p1; pc += 64) {
#pragma unroll
    for (int j = 0; j < 16; ++j) sM[4 * j + (t >> 6)][t & 63] = mnext[j];
    if (t < 192) sP[t >> 6][t & 63] = pnext;
    __syncthreads();
    if (pc + 64 < p1) load_chunk(pc + 64);  // workgroup-uniform
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = t + 256 * j;
      const int pp = i >> 5, ll = i & 31;
      float c, sn;  // pixels past the split have coordinates 0 and get phases 0
      phase_b(&sX[ll][0], sP[0][pp], sP[1][pp], sP[2][pp], c, sn);
      const bool ok = pc + pp < p1;
      sB[pp][ll] = ok ? make_float2(c, sn) : make_float2(0.0f, 0.0f);
      sBn[pp][ll] = ok ? -sn : 0.0f;
    }
    __syncthreads();
    // dW += B M^T over the chunk's pixels, then H = conj(W) M for this wave's
    // pixel half
    bwd_f32x16 h;
#pragma unroll
    for (int r = 0; r < 16; ++r) h[r] = 0.0f;
    if (part == 0) {
      if (dw_active) dw_chunk<0>(dw, sB, sBn, sM, blk, lane);
      h_chunk_w<0>(h, sW, wny, sM, blk, lane);
    } else {
      if (dw_active) dw_chunk<1>(dw, sB, sBn, sM, blk, lane);
      h_chunk_w<1>(h, sW, wny, sM, blk, lane);
    }
    __syncthreads();  // every wave is done with sM
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int ll = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      sH[(part * 64 + 32 * blk + (lane & 31)) * 33 + ll] = h[r];
    }
    __syncthreads();
    if (l < P.L) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        // pixels past the split add exact zeros (their phases, M and hence
        // H, and coordinates are all 0)
        const int pp = tp + 8 * j;
        const float2 b = sB[pp][tl];
        const float hr = sH[pp * 33 + tl], hi = sH[(64 + pp) * 33 + tl];
        const double v = (double)fmaf(hr, b.y, hi * b.x);  // Im(H B)
        gx += v * sP[0][pp];
        gy += v * sP[1][pp];
        gz += v * sP[2][pp];
      }
    }
    __syncthreads();  // sB, sP and sM (holding H) are restaged by the next chunk
  }
  if (dw_active) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int ll = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), k = 32 * blk + (lane & 31);
      P.dW_part[(((int64_t)s * P.L_pad + (l0 + ll)) * P.K_alloc + k) * 2 + part] = dw[r];
    }
  }
  double* const sh = reinterpret_cast<double*>(&sM[0][0]);  // [3][256]; sM is free after the loop
  sh[t] = gx;
  sh[256 + t] = gy;
  sh[512 + t] = gz;
  __syncthreads();
  if (tp == 0 && l < P.L_pad) {
    double a = 0, b = 0, c = 0;
    for (int j = 0; j < 8; ++j) {
      a += sh[t + 32 * j];
      b += sh[256 + t + 32 * j];
      c += sh[512 + t + 32 * j];
    }
    double* o = P.dx_part + ((int64_t)s * P.L_pad + l) * 3;
    o[0] = a;
    o[1] = b;
    o[2] = c;
  }
}

// dW and dd of eigenpairs outside every level are zero.
__global__ __launch_bounds__(256) void bwd_zero_kernel(int64_t n_w, int K, float* __restrict__ dW,
                                                       float* __restrict__ dd) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n_w) {
    dW[2 * idx] = 0.0f;
    dW[2 * idx + 1] = 0.0f;
  }
  if (idx < K) dd[idx] = 0.0f;
}

// Fixed-order sums over splits, scattered back to the caller's eigenpair order.
__global__ __launch_bounds__(256) void bwd_reduce_kernel(const BwdParams P, float* __restrict__ dW,
                                                         float* __restrict__ dd, double* __restrict__ dx) {
  const InstDesc& D = *P.desc;
  const int K_pad = P.dyn->K_pad;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (int64_t)P.L * K_pad) {
    // consecutive threads take consecutive eigenpairs: their partials are adjacent
    const int k = (int)(idx % K_pad), l = (int)(idx / K_pad);
    const int src = D.perm[k];
    if (src >= 0) {
      double re = 0.0, im = 0.0;
      for (int s = 0; s < P.n_split; ++s) {
        const double* q = P.dW_part + (((int64_t)s * P.L_pad + l) * P.K_alloc + k) * 2;
        re += q[0];
        im += q[1];
      }
      dW[2 * ((int64_t)src * P.L + l)] = (float)(2.0 * re);
      dW[2 * ((int64_t)src * P.L + l) + 1] = (float)(2.0 * im);
      if (l == 0) {
        double a = 0.0;
        for (int s = 0; s < P.n_split; ++s) a += P.dd_part[(int64_t)k * P.n_split + s];
        dd[src] = (float)a;
      }
    }
  }
  if (idx < (int64_t)P.L * 3) {
    const int l = (int)(idx % P.L), c = (int)(idx / P.L);
    double a = 0.0;
    for (int s = 0; s < P.n_split; ++s) a += P.dx_part[((int64_t)s * P.L_pad + l) * 3 + c];
    dx[(int64_t)c * P.L + l] = P.scale_x * a;
  }
}

hipError_t launch_backward(const BwdParams& p, hipStream_t s) {
  hipLaunchKernelGGL(bwd_m_kernel, dim3(p.K_alloc, p.n_split), dim3(256), 0, s, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (p.K_alloc <= 64) {  // one eigenpair slice: both contractions share their staged tiles
    hipLaunchKernelGGL(bwd_fused_kernel, dim3(p.L_pad / 32, p.n_split), dim3(256), 0, s, p);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(bwd_dw_kernel, dim3(p.L_pad / 32, (p.K_alloc + 63) / 64, p.n_split), dim3(256), 0, s, p);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (p.K_alloc <= 128)
    hipLaunchKernelGGL(bwd_dx_kernel<true>, dim3(p.L_pad / 32, p.n_split), dim3(256), 0, s, p);
  else
    hipLaunchKernelGGL(bwd_dx_kernel<false>, dim3(p.L_pad / 32, p.n_split), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_backward_reduce(const BwdParams& p, void* dW, float* dd, double* dx, hipStream_t s) {
  const int64_t n_w = (int64_t)p.L * p.K;
  int64_t n = n_w > p.K ? n_w : p.K;
  hipLaunchKernelGGL(bwd_zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n_w, p.K,
                     static_cast<float*>(dW), dd);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  n = (int64_t)p.L * p.K_alloc;
  if (n < (int64_t)p.L * 3) n = (int64_t)p.L * 3;
  hipLaunchKernelGGL(bwd_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p,
                     static_cast<float*>(dW), dd, dx);
  return hipGetLastError();
}

}  // namespace bb
