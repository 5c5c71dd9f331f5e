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
// E is recomputed by the forward MFMA kernel (FP32) into HBM; the kernels
// below work in level-sorted eigenpair order (the staging permutation) and
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

// dW partial: sum over the split's pixels of B_lp M_kp for a 32 x 32 (l, k)
// tile.  grid (L_pad/32, K_alloc/32, n_split), 256 threads; each thread owns
// one antenna and four eigenpairs.  LDS: phases [64 px][32 l] and M [64 px][32 k].
__global__ __launch_bounds__(256) void bwd_dw_kernel(const BwdParams P) {
  __shared__ float2 sB[64][32];
  __shared__ float2 sM[64][32];
  const InstDesc& D = *P.desc;
  const int l0 = blockIdx.x * 32, k0 = blockIdx.y * 32, s = blockIdx.z;
  const int t = threadIdx.x;
  const int tl = t >> 3, tk = (t & 7) * 4;
  const int64_t p0 = (int64_t)s * P.split_len;
  int64_t p1 = p0 + P.split_len;
  if (p1 > P.n_pix) p1 = P.n_pix;
  float ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
  const float* Er = P.E;
  const float* Ei = P.E + (int64_t)P.K_alloc * P.n_pix;
  for (int64_t pc = p0; pc < p1; pc += 64) {
    // phases: 32 antennas x 64 pixels, 8 per thread
    for (int i = t; i < 64 * 32; i += 256) {
      const int pp = i >> 5, ll = i & 31;
      const int64_t p = pc + pp;
      float c = 0.0f, sn = 0.0f;
      if (p < p1) {
        phase_b(D.xs + 4 * (l0 + ll), P.pix[p], P.pix[p + P.pix_ld], P.pix[p + 2 * P.pix_ld], c, sn);
      }
      sB[pp][ll] = make_float2(c, sn);
    }
    for (int i = t; i < 64 * 32; i += 256) {
      const int kk = i >> 6, pp = i & 63;
      const int64_t p = pc + pp;
      float2 m = make_float2(0.0f, 0.0f);
      if (p < p1) m = make_float2(Er[(int64_t)(k0 + kk) * P.n_pix + p], Ei[(int64_t)(k0 + kk) * P.n_pix + p]);
      sM[pp][kk] = m;
    }
    __syncthreads();
#pragma unroll 4
    for (int pp = 0; pp < 64; ++pp) {
      const float2 b = sB[pp][tl];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float2 m = sM[pp][tk + j];
        ar[j] = fmaf(b.x, m.x, fmaf(-b.y, m.y, ar[j]));
        ai[j] = fmaf(b.x, m.y, fmaf(b.y, m.x, ai[j]));
      }
    }
    __syncthreads();
  }
  double* out = P.dW_part + (((int64_t)s * P.L_pad + (l0 + tl)) * P.K_alloc + k0 + tk) * 2;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    out[2 * j] = ar[j];
    out[2 * j + 1] = ai[j];
  }
}

// dx partial: H_lp = sum_k conj(W_lk) M_kp, then Im(H_lp B_lp) p summed over
// the split's pixels.  grid (L_pad/32, n_split), 256 threads; each thread owns
// one antenna and 8 pixels of every 64-pixel chunk.
__global__ __launch_bounds__(256) void bwd_dx_kernel(const BwdParams P) {
  __shared__ float2 sW[32][65];   // conj(W) for 32 antennas x 64 eigenpairs (+1 pad)
  __shared__ float2 sM[64][65];   // M for 64 eigenpairs x 64 pixels (+1 pad)
  __shared__ double sh[3][256];
  const InstDesc& D = *P.desc;
  const int l0 = blockIdx.x * 32, s = blockIdx.y;
  const int t = threadIdx.x;
  const int tl = t >> 3, tp = (t & 7);
  const int l = l0 + tl;
  const int64_t p0 = (int64_t)s * P.split_len;
  int64_t p1 = p0 + P.split_len;
  if (p1 > P.n_pix) p1 = P.n_pix;
  const int K_pad = P.dyn->K_pad;
  const float* Er = P.E;
  const float* Ei = P.E + (int64_t)P.K_alloc * P.n_pix;
  const float* Wf = (const float*)P.W;
  double gx = 0.0, gy = 0.0, gz = 0.0;
  for (int64_t pc = p0; pc < p1; pc += 64) {
    float hr[8], hi[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) hr[j] = hi[j] = 0.0f;
    for (int kc = 0; kc < K_pad; kc += 64) {
      for (int i = t; i < 32 * 64; i += 256) {
        const int ll = i >> 6, kk = i & 63;
        const int k = kc + kk;
        float2 wv = make_float2(0.0f, 0.0f);
        if (l0 + ll < P.L && k < K_pad) {
          const int src = D.perm[k];
          if (src >= 0) {
            const float* w = Wf + 2 * ((int64_t)src * P.L + l0 + ll);
            wv = make_float2(w[0], -w[1]);
          }
        }
        sW[ll][kk] = wv;
      }
      for (int i = t; i < 64 * 64; i += 256) {
        const int kk = i >> 6, pp = i & 63;
        const int k = kc + kk;
        const int64_t p = pc + pp;
        float2 m = make_float2(0.0f, 0.0f);
        if (p < p1 && k < K_pad) m = make_float2(Er[(int64_t)k * P.n_pix + p], Ei[(int64_t)k * P.n_pix + p]);
        sM[kk][pp] = m;
      }
      __syncthreads();
      for (int kk = 0; kk < 64; ++kk) {
        const float2 w = sW[tl][kk];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const float2 m = sM[kk][tp + 8 * j];
          hr[j] = fmaf(w.x, m.x, fmaf(-w.y, m.y, hr[j]));
          hi[j] = fmaf(w.x, m.y, fmaf(w.y, m.x, hi[j]));
        }
      }
      __syncthreads();
    }
    if (l < P.L) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t p = pc + tp + 8 * j;
        if (p < p1) {
          const double px = P.pix[p], py = P.pix[p + P.pix_ld], pz = P.pix[p + 2 * P.pix_ld];
          float c, sn;
          phase_b(D.xs + 4 * l, px, py, pz, c, sn);
          const double v = (double)fmaf(hr[j], sn, hi[j] * c);  // Im(H B)
          gx += v * px;
          gy += v * py;
          gz += v * pz;
        }
      }
    }
  }
  sh[0][t] = gx;
  sh[1][t] = gy;
  sh[2][t] = gz;
  __syncthreads();
  if (tp == 0 && l < P.L_pad) {
    double a = 0, b = 0, c = 0;
    for (int j = 0; j < 8; ++j) {
      a += sh[0][t + j];
      b += sh[1][t + j];
      c += sh[2][t + j];
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
    const int l = (int)(idx % P.L), k = (int)(idx / P.L);
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
  hipLaunchKernelGGL(bwd_dw_kernel, dim3(p.L_pad / 32, p.K_alloc / 32, p.n_split), dim3(256), 0, s, p);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bwd_dx_kernel, dim3(p.L_pad / 32, p.n_split), dim3(256), 0, s, p);
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
