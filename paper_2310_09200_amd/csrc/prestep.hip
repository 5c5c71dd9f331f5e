// FP64 pre-step of one instance (Algorithm 1 up to the synthesis call):
// Gram matrix, copy of V for the in-place eigensolver, and selection of the
// kept eigenpairs with their filter weights and level ids.  The generalized
// eigensolve itself is rocSOLVER's zhegvd, called from the host API.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bb_internal.h"

namespace bb {

// G_pq = sinc(2 ||x_p - x_q|| / lambda_w), sinc(u) = sin(pi u) / (pi u)
// (Section 2.2, Eq. gram), stored complex128 column-major for zhegvd.
// With `identity`, G = I: the eigen-decomposition is then that of V itself and
// the image is the back-projected (dirty) image of Section 2.8.
// Instance blockIdx.y: antennas at ant + y * ant_step (rows of a shared
// column-major array), 1 / wavelength inv_wl[y] (or inv_wl0 without an array),
// G at G + y * g_step doubles.
__global__ __launch_bounds__(256) void gram_kernel(const double* __restrict__ ant, int64_t ant_ld, int64_t ant_step,
                                                   int L, double inv_wl0, const double* __restrict__ inv_wl,
                                                   double* __restrict__ G, int ldg, int64_t g_step, int identity) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)L * L) return;
  const int y = blockIdx.y;
  ant += y * ant_step;
  G += y * g_step;
  const int p = (int)(idx % L), q = (int)(idx / L);
  if (identity) {
    double* g = G + 2 * ((int64_t)q * ldg + p);
    g[0] = p == q ? 1.0 : 0.0;
    g[1] = 0.0;
    return;
  }
  const double iw = inv_wl ? inv_wl[y] : inv_wl0;
  const double dx = ant[p] - ant[q];
  const double dy = ant[p + ant_ld] - ant[q + ant_ld];
  const double dz = ant[p + 2 * ant_ld] - ant[q + 2 * ant_ld];
  const double u = 2.0 * sqrt(dx * dx + dy * dy + dz * dz) * iw;
  const double v = (u == 0.0) ? 1.0 : sinpi(u) / (M_PI * u);
  double* g = G + 2 * ((int64_t)q * ldg + p);
  g[0] = v;
  g[1] = 0.0;
}

// Instance blockIdx.y: src + y * step, dst + y * step doubles (step 0 for one instance).
__global__ __launch_bounds__(256) void copy_c128_kernel(const double* __restrict__ src, int L,
                                                        double* __restrict__ dst, int ldd, int64_t step) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)L * L) return;
  src += blockIdx.y * step;
  dst += blockIdx.y * step;
  const int p = (int)(idx % L), q = (int)(idx / L);
  const double* s = src + 2 * ((int64_t)q * L + p);
  double* d = dst + 2 * ((int64_t)q * ldd + p);
  d[0] = s[0];
  d[1] = s[1];
}

// Hermiticity of the visibility matrix (Section 2.1: V is a correlation
// matrix): out[0] = ||V - V^H||_F^2, out[1] = ||V||_F^2, one workgroup, fixed
// summation order.  The eigensolver reads one triangle only, so without this
// check a non-Hermitian V would be imaged as if symmetrised.  Workgroup y
// checks the matrix at V + y * step doubles into out[2 y], out[2 y + 1].
__global__ __launch_bounds__(256) void herm_check_kernel(const double* __restrict__ V, int L, int64_t step,
                                                         double* __restrict__ out) {
  __shared__ double s_d[256], s_n[256];
  const int tid = threadIdx.x;
  V += blockIdx.x * step;
  out += 2 * blockIdx.x;
  double dsum = 0.0, nsum = 0.0;
  for (int64_t i = tid; i < (int64_t)L * L; i += 256) {
    const int p = (int)(i % L), q = (int)(i / L);
    const double* a = V + 2 * ((int64_t)q * L + p);  // V_pq
    const double* b = V + 2 * ((int64_t)p * L + q);  // V_qp
    const double dr = a[0] - b[0], di = a[1] + b[1];  // V_pq - conj(V_qp)
    dsum += dr * dr + di * di;
    nsum += a[0] * a[0] + a[1] * a[1];
  }
  s_d[tid] = dsum;
  s_n[tid] = nsum;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      s_d[tid] += s_d[tid + w];
      s_n[tid] += s_n[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = s_d[0];
    out[1] = s_n[0];
  }
}

hipError_t launch_herm_check(const double* V, int L, double* out, hipStream_t s) {
  hipLaunchKernelGGL(herm_check_kernel, dim3(1), dim3(256), 0, s, V, L, (int64_t)0, out);
  return hipGetLastError();
}

// zhegvd returns eigenvalues ascending; keep the K largest, descending
// (Section 2.6 truncation; Algorithm 1 selection).  Weight: lambda (LSQ
// filter) or 1 (standardized filter).  Level: first closed interval that
// contains lambda, else -1.  wcol maps kept position k to its eigenvector column.
// Instance blockIdx.y: evals + y * L, outputs + y * K.
__global__ __launch_bounds__(256) void select_kernel(const double* __restrict__ evals, int L, int K,
                                                     Intervals iv, int n_levels, int filter,
                                                     float* __restrict__ d_out, int* __restrict__ lev_out,
                                                     int* __restrict__ wcol_out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  evals += (int64_t)blockIdx.y * L;
  d_out += (int64_t)blockIdx.y * K;
  lev_out += (int64_t)blockIdx.y * K;
  wcol_out += (int64_t)blockIdx.y * K;
  const int col = L - 1 - k;
  const double lam = evals[col];
  int lv = -1;
  for (int l = n_levels - 1; l >= 0; --l)
    if (lam >= iv.lo[l] && lam <= iv.hi[l]) lv = l;
  d_out[k] = filter == 0 ? (float)lam : 1.0f;
  lev_out[k] = lv;
  wcol_out[k] = col;
}

hipError_t launch_gram(const double* ant, int64_t ant_ld, int L, double wl, double* G, int ldg, bool identity,
                       hipStream_t s) {
  const int64_t n = (int64_t)L * L;
  hipLaunchKernelGGL(gram_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ant, ant_ld, (int64_t)0, L,
                     1.0 / wl, (const double*)nullptr, G, ldg, (int64_t)0, identity ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_copy_c128(const double* src, int L, double* dst, int ldd, hipStream_t s) {
  const int64_t n = (int64_t)L * L;
  hipLaunchKernelGGL(copy_c128_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, L, dst, ldd,
                     (int64_t)0);
  return hipGetLastError();
}

hipError_t launch_select(const double* evals, int L, int K, Intervals iv, int n_levels, int filter, float* d_out,
                         int* lev_out, int* wcol_out, hipStream_t s) {
  hipLaunchKernelGGL(select_kernel, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, evals, L, K, iv, n_levels,
                     filter, d_out, lev_out, wcol_out);
  return hipGetLastError();
}

hipError_t launch_prestep_inputs_batched(const double* ant, int64_t ant_ld, int L, const double* inv_wl, int n_inst,
                                         bool identity, const double* vis, double* A, double* G, double* herm,
                                         hipStream_t s) {
  const int64_t n = (int64_t)L * L;
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)n_inst);
  hipLaunchKernelGGL(gram_kernel, grid, dim3(256), 0, s, ant, ant_ld, (int64_t)L, L, 0.0, inv_wl, G, L, 2 * n,
                     identity ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(copy_c128_kernel, grid, dim3(256), 0, s, vis, L, A, L, 2 * n);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(herm_check_kernel, dim3((unsigned)n_inst), dim3(256), 0, s, vis, L, 2 * n, herm);
  return hipGetLastError();
}

// Copy the kept eigenpairs out: W (complex64, L x K column-major), lambda,
// weights and level ids.  Instance blockIdx.y: A + y * 2 L^2, evals + y * L,
// selection and outputs + y * K (W_out + y * 2 L K).
__global__ __launch_bounds__(256) void export_eig_kernel(const double* __restrict__ A, const double* __restrict__ evals,
                                                         int L, int K, const int* __restrict__ wcol,
                                                         const float* __restrict__ dsel, const int* __restrict__ lsel,
                                                         float* __restrict__ W_out, double* __restrict__ lam_out,
                                                         float* __restrict__ d_out, int* __restrict__ lev_out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)L * K) return;
  const int64_t y = blockIdx.y;
  A += y * 2 * (int64_t)L * L;
  evals += y * L;
  wcol += y * K;
  dsel += y * K;
  lsel += y * K;
  W_out += y * 2 * (int64_t)L * K;
  lam_out += y * K;
  d_out += y * K;
  lev_out += y * K;
  const int l = (int)(idx % L), k = (int)(idx / L);
  const int col = wcol[k];
  const double* a = A + 2 * ((int64_t)col * L + l);
  W_out[2 * idx] = (float)a[0];
  W_out[2 * idx + 1] = (float)a[1];
  if (l == 0) {
    lam_out[k] = evals[col];
    d_out[k] = dsel[k];
    lev_out[k] = lsel[k];
  }
}

hipError_t launch_export_eig(const double* A, const double* evals, int L, int K, const int* wcol, const float* dsel,
                             const int* lsel, float* W_out, double* lam_out, float* d_out, int* lev_out,
                             hipStream_t s) {
  const int64_t n = (int64_t)L * K;
  hipLaunchKernelGGL(export_eig_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, evals, L, K, wcol,
                     dsel, lsel, W_out, lam_out, d_out, lev_out);
  return hipGetLastError();
}

hipError_t launch_select_export_batched(const double* A, const double* evals, int L, int K, int n_inst, Intervals iv,
                                        int n_levels, int filter, float* dsel, int* lsel, int* wcol, float* W_out,
                                        double* lam_out, float* d_out, int* lev_out, hipStream_t s) {
  hipLaunchKernelGGL(select_kernel, dim3((unsigned)((K + 255) / 256), (unsigned)n_inst), dim3(256), 0, s, evals, L,
                     K, iv, n_levels, filter, dsel, lsel, wcol);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = (int64_t)L * K;
  hipLaunchKernelGGL(export_eig_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)n_inst), dim3(256), 0, s, A,
                     evals, L, K, wcol, dsel, lsel, W_out, lam_out, d_out, lev_out);
  return hipGetLastError();
}

}  // namespace bb
