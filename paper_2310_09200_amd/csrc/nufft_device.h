// Device helpers shared by the NUFFT kernels (internal; not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "bb_internal.h"

namespace bb {

__device__ __forceinline__ float es_kernel(float z, float beta) {
  const float t = fmaxf(1.0f - z * z, 0.0f);
  return __expf(beta * (sqrtf(t) - 1.0f));
}

// Kernel values and wrapped grid indices of the W points nearest to xi
// (grid units) on a periodic axis of n points.
template <int W>
__device__ __forceinline__ void kernel_row(double xi, int n, float beta, float (&k)[W], int (&idx)[W]) {
  const double first = ceil(xi - 0.5 * W);
  const float inv_half = 2.0f / (float)W;
  int j = (int)first % n;
  if (j < 0) j += n;
#pragma unroll
  for (int t = 0; t < W; ++t) {
    k[t] = es_kernel((float)((first + t) - xi) * inv_half, beta);
    idx[t] = j;
    j = (j + 1 == n) ? 0 : j + 1;
  }
}

__device__ __forceinline__ double frame_coord(const NufftGeom& g, int d, double a0, double a1, double a2) {
#pragma clang fp contract(off)
  return (a0 * g.R[d][0] + a1 * g.R[d][1]) + a2 * g.R[d][2];
}

// Baseline (q, r) of an instance in spread-grid units of the plan: returns
// 0 when the plan transforms it, 1 when it lies beyond the planned extent (an
// error), 2 when it belongs to another uvw cell (shifted by the cell centre
// when cells are in use).
__device__ __forceinline__ int source_coords(const NufftGeom& g, const NufftInst& I, const double* __restrict__ ant,
                                             int64_t ld, int q, int r, double (&xi)[3], double& turns_d) {
  const double* A = ant + I.ant_off;
  double b[3];
  {
#pragma clang fp contract(off)
    const double d0 = A[q] - A[r];
    const double d1 = A[q + ld] - A[r + ld];
    const double d2 = A[q + 2 * ld] - A[r + 2 * ld];
    for (int d = 0; d < 3; ++d) b[d] = frame_coord(g, d, d0, d1, d2) / I.wavelength_m;
  }
  if (!(fabs(b[0]) <= g.Xf[0]) || !(fabs(b[1]) <= g.Xf[1]) || !(fabs(b[2]) <= g.Xf[2])) return 1;
  if (g.cell_q > 1) {
    if (uvw_cell(b[0], g.Xf[0], g.cell_q) != g.cell_i[0] || uvw_cell(b[1], g.Xf[1], g.cell_q) != g.cell_i[1]) return 2;
    for (int d = 0; d < 3; ++d) b[d] -= g.C[d];
  }
  for (int d = 0; d < 3; ++d) xi[d] = b[d] * g.inv_h[d];
  turns_d = b[0] * g.D[0] + b[1] * g.D[1] + b[2] * g.D[2];
  return 0;
}

__device__ __forceinline__ int first_cell(double xi, int w, int n) {
  const int j = (int)ceil(xi - 0.5 * w) % n;
  return j < 0 ? j + n : j;
}

// Calls f with the kernel support w (3 .. 8) as a compile-time constant.
template <class F>
inline hipError_t with_width(int w, F f) {
  switch (w) {
    case 3: return f(std::integral_constant<int, 3>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 5: return f(std::integral_constant<int, 5>{});
    case 6: return f(std::integral_constant<int, 6>{});
    case 7: return f(std::integral_constant<int, 7>{});
    case 8: return f(std::integral_constant<int, 8>{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bb
