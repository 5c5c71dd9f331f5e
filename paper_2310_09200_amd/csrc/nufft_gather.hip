// Output-driven spreading of the NUFFT (gfx950) for grids of at most 64 points
// along axis 2.
//
// The spread is the same sum as in nufft.hip (every baseline adds its value
// times the tensor-product kernel on the w^3 grid points nearest to it), but
// taken from the side of the grid: each thread owns one grid point (x, y, z)
// and adds, for every level at once, the baselines whose kernel reaches it.
// No two threads write the same point, so there are no LDS atomics.
//
//   1. baselines are sorted by their first grid point on axes 0 and 1
//      (counting sort over N0 x N1 bins);
//   2. one record per sorted baseline: its three kernel rows, its first point
//      on axis 2, and V'_l[r, q] exp(2 pi i <b, D>) for every level;
//   3. a workgroup takes a block of columns (x, y) times the Z >= N2 points of
//      axis 2; the baselines reaching column (x, y) are exactly those of the
//      w x w bins (x - a, y - c), a, c < w, and for such a baseline the kernel
//      weight of point (x, y, z) is k0[a] k1[c] k2[(z - f2) mod N2].
//      A column's points sit in rows of 16 lanes: each lane of a row loads
//      one word of the baseline's record and the value pair of one level,
//      and the row shares them with DPP row broadcasts (and one permute for
//      k2), so every word crosses the texture path once per row instead of
//      once per lane.
// Columns near the centre of the uv plane see up to ~1e5 baselines, so a
// block is split into up to w^2 parts (each a range of the (a, c) offsets)
// sized from its busiest column; a block of one part writes its points with
// plain stores, the parts of a split block add theirs with atomics.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>
#include <utility>

#include "bb_internal.h"
#include "nufft_device.h"

namespace bb {

namespace {

constexpr int kPartLoad = 4096;  // target baselines per column and part
constexpr int kXcds = 8;         // XCDs of the device (workgroups are dealt to them round-robin)
constexpr int kRun = 64;         // consecutive parts an XCD takes at a time

// f(integral_constant<int, I>) for I = B .. E - 1
template <int B, int E, class F>
void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

struct SrcRec {  // one sorted baseline (128 bytes); k2 and f2 share the first 48
  float k2[8];
  int f2;
  int pad0[3];
  float k0[8], k1[8];
  int pad1[4];
};
static_assert(sizeof(SrcRec) == kGatherRecBytes, "record size");

// Columns of a workgroup: 256 threads = (256 / Z) columns x Z points of axis 2
// (Z = 16, 32 or 64: whole rows of 16 lanes per column).
template <int Z>
struct ColBlock {
  static constexpr int COLS = 256 / Z;
  static constexpr int CX = 4;
  static constexpr int CY = COLS / CX;
};

// Word n (0..15) of each row of 16 lanes, to every lane of that row.  The
// empty asm keeps the broadcast a v_mov_b32_dpp of its own.  Left alone, the
// compiler folds the broadcast into its consumer as a DPP operand, among
// others into v_subrev_u32_dpp for the integer grid index; on gfx950 that
// opcode applies the DPP lane control to src1 instead of src0 (measured with
// one-wave checks: v_subrev_u32_dpp with row_newbcast or row_shr selects the
// lanes of src1, while v_sub_u32_dpp, v_sub_f32_dpp, v_subrev_f32_dpp and
// v_mul_f32_dpp select those of src0), so the folded code read the wrong
// lanes.  A plain v_mov_b32_dpp behaves as documented.
template <int N>
__device__ __forceinline__ float row_bcast(int v) {
  int r = __builtin_amdgcn_mov_dpp(v, 0x150 + N, 0xF, 0xF, true);
  asm volatile("" : "+v"(r));
  return __builtin_bit_cast(float, r);
}

// acc[L] += wgt * level value L, held (re, im) by lane L of the row (levels
// past the plan's count carry zeros).  All values are broadcast first, each
// into a register of its own, and then multiplied in: a broadcast into the
// register a multiply-add has just read costs wait states.
template <size_t... L>
__device__ __forceinline__ void add_levels(float2 (&acc)[kMaxLevels], float wgt, int cr, int ci,
                                           std::index_sequence<L...>) {
  const float vr[] = {row_bcast<(int)L>(cr)...};
  const float vi[] = {row_bcast<(int)L>(ci)...};
  ((acc[L].x += wgt * vr[L], acc[L].y += wgt * vi[L]), ...);
}

template <int W>
__global__ __launch_bounds__(256) void nufft_records_kernel(NufftGeom g, const NufftInst* __restrict__ insts,
                                                            const double* __restrict__ ant, int64_t ld,
                                                            const float2* __restrict__ vp,
                                                            const uint64_t* __restrict__ list,
                                                            const int* __restrict__ n_src_dev, int n_levels,
                                                            int cv_stride, SrcRec* __restrict__ rec,
                                                            float2* __restrict__ cv) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= *n_src_dev) return;
  const uint64_t key = list[p];
  const int inst = (int)(key >> 32), q = (int)((key >> 16) & 0xffff), r = (int)(key & 0xffff);
  const NufftInst I = insts[inst];
  double xi[3], td;
  source_coords(g, I, ant, ld, q, r, xi, td);  // in range: the sort kept only such baselines
  float k0[W], k1[W], k2[W];
  int j0[W], j1[W], j2[W];
  kernel_row<W>(xi[0], g.N[0], g.beta, k0, j0);
  kernel_row<W>(xi[1], g.N[1], g.beta, k1, j1);
  kernel_row<W>(xi[2], g.N[2], g.beta, k2, j2);
  SrcRec R = {};
#pragma unroll
  for (int t = 0; t < W; ++t) {
    R.k0[t] = k0[t];
    R.k1[t] = k1[t];
    R.k2[t] = k2[t];
  }
  R.f2 = j2[0];
  rec[p] = R;
  const float f = (float)(td - rint(td));
  const float pc = __builtin_amdgcn_cosf(f), ps = __builtin_amdgcn_sinf(f);
  const int L = I.n_ant;
  float2* out = cv + p * cv_stride;
  for (int lv = 0; lv < n_levels; ++lv) {
    const float2 v = vp[I.vp_off + (int64_t)lv * L * L + q + (int64_t)r * L];
    out[lv] = make_float2(v.x * pc - v.y * ps, v.x * ps + v.y * pc);
  }
  if (cv_stride > n_levels) out[n_levels] = make_float2(0.0f, 0.0f);
}

// Parts of each column block: ceil(busiest column's baselines / kPartLoad), 1 .. W^2.
template <int W, int Z>
__global__ __launch_bounds__(256) void nufft_block_parts_kernel(NufftGeom g, const int* __restrict__ offset, int nbx,
                                                                int nby, int* __restrict__ nparts) {
  using B = ColBlock<Z>;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbx * nby) return;
  const int bx = b / nby, by = b - bx * nby;
  const int N0 = g.N[0], N1 = g.N[1];
  int busiest = 0;
  for (int cx = 0; cx < B::CX; ++cx) {
    const int x = bx * B::CX + cx;
    if (x >= N0) break;
    for (int cy = 0; cy < B::CY; ++cy) {
      const int y = by * B::CY + cy;
      if (y >= N1) break;
      int load = 0;
      for (int a = 0; a < W; ++a) {
        const int xb = x - a < 0 ? x - a + N0 : x - a;
        for (int c = 0; c < W; ++c) {
          const int yb = y - c < 0 ? y - c + N1 : y - c;
          const int bin = xb * N1 + yb;
          load += offset[bin + 1] - offset[bin];
        }
      }
      busiest = max(busiest, load);
    }
  }
  nparts[b] = min(max((busiest + kPartLoad - 1) / kPartLoad, 1), W * W);
}

// Persistent over the parts of every column block (part k of block b for
// part_off[b] <= k < part_off[b + 1]); see the file comment.  LV: the level
// count.
template <int Z, int LV>
__global__ __launch_bounds__(256) void nufft_gather_spread_kernel(NufftGeom g, const int* __restrict__ offset,
                                                                  const SrcRec* __restrict__ rec,
                                                                  const float2* __restrict__ cv, int n_levels,
                                                                  int cv_stride, const int* __restrict__ part_off,
                                                                  int nbx, int nby, float* __restrict__ grid,
                                                                  int64_t n_cell) {
  using B = ColBlock<Z>;
  __shared__ int s_block;
  const int tid = threadIdx.x;
  const int n_blocks = nbx * nby;
  const int n_parts = part_off[n_blocks];
  const int N0 = g.N[0], N1 = g.N[1], N2 = g.N[2], W = g.w;
  const int z = tid % Z, col = tid / Z;
  // Workgroups are dealt to the 8 XCDs round-robin (XCD = blockIdx.x mod 8);
  // each XCD takes runs of kRun consecutive parts (neighbouring column
  // blocks, which read many of the same records through its L2), the runs
  // dealt round-robin too so that the busy centre of the uv plane is shared.
  const int xcd = blockIdx.x % kXcds, slot = blockIdx.x / kXcds, n_slot = gridDim.x / kXcds;
  for (int t = slot;; t += n_slot) {
    const int w = ((t / kRun) * kXcds + xcd) * kRun + t % kRun;
    if (w >= n_parts) break;
    if (tid == 0) {  // block of part w: last b with part_off[b] <= w
      int lo = 0, hi = n_blocks;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (part_off[mid] <= w) lo = mid; else hi = mid;
      }
      s_block = lo;
    }
    __syncthreads();
    const int b = s_block;
    const int k = w - part_off[b], K = part_off[b + 1] - part_off[b];
    const int bx = b / nby, by = b - bx * nby;
    const int x = bx * B::CX + col % B::CX, y = by * B::CY + col / B::CX;
    const bool col_active = x < N0 && y < N1;  // the same for the 16 lanes of a row
    const int row_lane = tid & 15, row_base = (tid & 63) & ~15;
    const int o_lo = k * (W * W) / K, o_hi = (k + 1) * (W * W) / K;
    float2 acc[kMaxLevels];
#pragma unroll
    for (int l = 0; l < kMaxLevels; ++l) acc[l] = make_float2(0.0f, 0.0f);
    if (col_active) {
      for (int o = o_lo; o < o_hi; ++o) {
        const int a = o / W, c = o - a * W;
        const int xb = x - a < 0 ? x - a + N0 : x - a;
        const int yb = y - c < 0 ? y - c + N1 : y - c;
        const int bin = xb * N1 + yb;
        const int beg = offset[bin], end = offset[bin + 1];
        // record word of this lane: k2[0..7] (lanes 0-7), f2 (8), k0[a] (9), k1[c] (10)
        const int rw = row_lane < 9 ? row_lane : row_lane == 9 ? 12 + a : row_lane == 10 ? 20 + c : 0;
        const bool lv_ok = row_lane < n_levels;  // this lane holds level row_lane's value
        for (int p = beg; p < end; ++p) {
          const int m = reinterpret_cast<const int*>(rec + p)[rw];
          const float2 c = lv_ok ? cv[(int64_t)p * cv_stride + row_lane] : make_float2(0.0f, 0.0f);
          const int cr = __builtin_bit_cast(int, c.x), ci = __builtin_bit_cast(int, c.y);
          const int f2 = __builtin_bit_cast(int, row_bcast<8>(m));
          const float k01 = row_bcast<9>(m) * row_bcast<10>(m);
          int d = z - f2;
          if (d < 0) d += N2;
          const bool in = d < W;
          const float k2d =
              __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute((row_base + (in ? d : 0)) * 4, m));
          const float wgt = in ? k01 * k2d : 0.0f;
          add_levels(acc, wgt, cr, ci, std::make_index_sequence<LV>{});
        }
      }
      if (z < N2) {
        const int64_t cell = ((int64_t)x * N1 + y) * N2 + z;
#pragma unroll
        for (int l = 0; l < kMaxLevels; ++l) {
          if (l < n_levels && (acc[l].x != 0.0f || acc[l].y != 0.0f)) {
            float* G = grid + 2 * ((int64_t)l * n_cell + cell);
            if (K == 1) {
              G[0] += acc[l].x;
              G[1] += acc[l].y;
            } else {
              unsafeAtomicAdd(G, acc[l].x);
              unsafeAtomicAdd(G + 1, acc[l].y);
            }
          }
        }
      }
    }
    __syncthreads();  // s_block is reused by the next part
  }
}

}  // namespace

int nufft_gather_z(const NufftGeom& g) {
  for (int z : {16, 32, 64})
    if (g.N[2] <= z) return z;
  return 0;
}

void nufft_gather_blocks(const NufftGeom& g, int& nbx, int& nby) {
  const int z = nufft_gather_z(g);
  const int cx = 4, cy = (256 / z) / cx;
  nbx = (g.N[0] + cx - 1) / cx;
  nby = (g.N[1] + cy - 1) / cy;
}

hipError_t launch_nufft_spread_gather(const NufftGeom& g, const NufftInst* insts, int64_t max_src, const double* ant,
                                      int64_t ld, const void* vp, const int* offset, const uint64_t* list,
                                      int n_levels, void* rec, void* cv, int* nparts, int* part_off, int* scan_tmp,
                                      float* grid, int64_t n_cell, hipStream_t s) {
  const int Zc = nufft_gather_z(g);
  if (Zc == 0) return hipErrorInvalidValue;
  int nbx, nby;
  nufft_gather_blocks(g, nbx, nby);
  const int n_blocks = nbx * nby;
  const int cv_stride = (n_levels + 1) & ~1;
  const int* n_src_dev = offset + (int64_t)g.N[0] * g.N[1];
  hipError_t e = with_width(g.w, [&](auto wc) -> hipError_t {
    constexpr int KW = decltype(wc)::value;
    if (max_src > 0)
      hipLaunchKernelGGL(nufft_records_kernel<KW>, dim3((unsigned)((max_src + 255) / 256)), dim3(256), 0, s, g,
                         insts, ant, ld, static_cast<const float2*>(vp), list, n_src_dev, n_levels, cv_stride,
                         static_cast<SrcRec*>(rec), static_cast<float2*>(cv));
    const unsigned pb = (unsigned)((n_blocks + 255) / 256);
    if (Zc == 16)
      hipLaunchKernelGGL((nufft_block_parts_kernel<KW, 16>), dim3(pb), dim3(256), 0, s, g, offset, nbx, nby, nparts);
    else if (Zc == 32)
      hipLaunchKernelGGL((nufft_block_parts_kernel<KW, 32>), dim3(pb), dim3(256), 0, s, g, offset, nbx, nby, nparts);
    else
      hipLaunchKernelGGL((nufft_block_parts_kernel<KW, 64>), dim3(pb), dim3(256), 0, s, g, offset, nbx, nby, nparts);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  e = launch_scan_i32(nparts, n_blocks, part_off, nullptr, scan_tmp, s);
  if (e != hipSuccess) return e;
  auto run = [&](auto zc, auto lc) -> hipError_t {
    constexpr int ZZ = decltype(zc)::value, LL = decltype(lc)::value;
    hipLaunchKernelGGL((nufft_gather_spread_kernel<ZZ, LL>), dim3(8192u), dim3(256), 0, s, g, offset,
                       static_cast<const SrcRec*>(rec), static_cast<const float2*>(cv), n_levels, cv_stride, part_off,
                       nbx, nby, grid, n_cell);
    return hipGetLastError();
  };
  auto by_levels = [&](auto zc) -> hipError_t {
    hipError_t r = hipErrorInvalidValue;
    static_for<1, kMaxLevels + 1>([&](auto lc) {
      if (decltype(lc)::value == n_levels) r = run(zc, lc);
    });
    return r;
  };
  if (Zc == 16) return by_levels(std::integral_constant<int, 16>{});
  if (Zc == 32) return by_levels(std::integral_constant<int, 32>{});
  return by_levels(std::integral_constant<int, 64>{});
}

}  // namespace bb
