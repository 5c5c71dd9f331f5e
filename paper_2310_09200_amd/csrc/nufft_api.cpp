// Host side of NUFFT synthesis (Section 2.5; Section 3.4, Algorithm 3): plan
// geometry from the options and the pixels, workspace carving, the pruned
// transform's line-FFT tables (or rocFFT plans), and the spread / emit calls
// declared in include/bluebild.h.

#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "api_common.h"
#include "bb_internal.h"
#include "bluebild.h"

using bb_host::align_up;
using bb_host::fail;
using bb_host::finite_pos;

namespace {

constexpr int kSigma = 2;        // type-2 grid upsampling
constexpr int kQuadNodes = 100;  // Gauss-Legendre nodes for kernel transforms

// Byte offsets of a plan's two regions.  The transient region (grid, the
// pruned transform's stages, rocFFT's work area) holds data only from a spread
// to the end of the next emit, so the plans of a partitioned plan, run one
// after another, share one; the persistent region (tables, corrections, level
// diagonals, error word) is each plan's own.  A single plan's workspace is the
// transient region followed by the persistent one.
struct NufftLayout {
  size_t grid, stage_ac, stage_b, work, work_bytes, t_total;  // from the transient base
  size_t perm[3];  // line FFTs: digit-reversed load position per input index (int32, M_d)
  size_t tw[3];    // line FFTs: the passes' twiddles (complex64, M_d - 1)
  size_t dft[3];   // lines of at most kLineDftMax points: direct DFT table (complex64, N_d x window_d)
  size_t psi0, psi1, psi2, corr, quad_t, quad_wphi, diag, err, p_total;  // from the persistent base
  size_t total;    // t_total + p_total
};

// Which uvw cell a plan transforms (cells of 1: every baseline, no shift), and
// whether its interpolation adds the level diagonals.
struct CellSpec {
  int q = 1, iu = 0, iv = 0;
  bool use_diag = true;
};

// The pruned type-2 transform runs as the library's own LDS line FFTs when
// every axis fits one workgroup's LDS on this device (and the caller did not
// ask for rocFFT).
bool use_line_fft(const bb::NufftGeom& g, int transform, int device) {
  if (transform != 0) return false;
  int lds_limit = 0;
  if (hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) return false;
  for (int d = 0; d < 3; ++d) {
    bb::LineFft p{};
    if (bb::line_fft_plan(g.M[d], p) != 0 || bb::line_fft_lds_bytes(p) > (size_t)lds_limit) return false;
  }
  return true;
}

// Complex points of the stages of the pruned type-2 transform.
//   rocFFT:     A [i0][i1][m2], B [i0][w2][m1], C [w1][w2][m0] (A and C share a region)
//   line FFTs:  A'[i0][w2][i1], B [i0][w2][w1], B'[w2][w1][i0], C [w2][w1][w0]
//               (A' and B' share one region, B and C the other)
struct StageSizes {
  size_t a, b, c;
};
StageSizes stage_sizes(const bb::NufftGeom& g) {
  return {(size_t)g.N[0] * g.N[1] * g.M[2], (size_t)g.N[0] * g.win_len[2] * g.M[1],
          (size_t)g.win_len[1] * g.win_len[2] * g.M[0]};
}
StageSizes line_stage_sizes(const bb::NufftGeom& g) {
  const size_t w0 = g.win_len[0], w1 = g.win_len[1], w2 = g.win_len[2];
  return {(size_t)g.N[0] * w2 * g.N[1], (size_t)g.N[0] * w2 * w1, w2 * w1 * w0};
}

// Gauss-Legendre nodes and weights on [-1, 1]: Newton's method on P_n,
// evaluated by the three-term recurrence.
void gauss_legendre(int n, std::vector<double>& t, std::vector<double>& wt) {
  t.assign(n, 0.0);
  wt.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (x * p1 - p0) / (x * x - 1.0);
    t[i] = -x;
    t[n - 1 - i] = x;
    wt[i] = wt[n - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
}

double es_kernel_host(double z, double beta) {
  return std::fabs(z) <= 1.0 ? std::exp(beta * (std::sqrt(1.0 - z * z) - 1.0)) : 0.0;
}

int kernel_width(double eps) { return (int)std::ceil(std::log10(1.0 / eps) - 1e-9) + 1; }

int smooth_size(int64_t n) {
  n = std::max<int64_t>(n, 2);
  for (;; ++n) {
    if (n % 2) continue;
    int64_t m = n;
    for (int p : {2, 3, 5})
      while (m % p == 0) m /= p;
    if (m == 1) return (int)n;
  }
}

// Plan geometry (the same rules, in the same arithmetic order, as the
// grid-size rules documented in the header).
bb_status nufft_geometry(bb_context ctx, const bb_nufft_options* o, int64_t n_pix, const double* pix_host,
                         bb::NufftGeom& g, const CellSpec& cell = CellSpec{}) {
#pragma clang fp contract(off)
  if (!o) return fail(ctx, BB_ERR_INVALID_ARG, "options is NULL");
  if (o->n_levels < 1 || o->n_levels > bb::kMaxLevels)
    return fail(ctx, BB_ERR_INVALID_ARG, "n_levels must be in [1, %d]", bb::kMaxLevels);
  if (o->n_ant_max < 2 || o->n_ant_max > bb::kMaxAnt)
    return fail(ctx, BB_ERR_INVALID_ARG, "n_ant_max must be in [2, %d]", bb::kMaxAnt);
  if (o->k_max < 1 || o->k_max > bb::kMaxEig) return fail(ctx, BB_ERR_INVALID_ARG, "k_max must be in [1, %d]", bb::kMaxEig);
  if (o->transform != 0 && o->transform != 1) return fail(ctx, BB_ERR_INVALID_ARG, "transform must be 0 or 1");
  if (o->partitions < 0 || o->partitions > 8) return fail(ctx, BB_ERR_INVALID_ARG, "partitions must be in [0, 8]");
  if (o->uvw_partitions < 0 || o->uvw_partitions > 16)
    return fail(ctx, BB_ERR_INVALID_ARG, "uvw_partitions must be in [0, 16]");
  if (!(o->epsilon >= 1e-7 && o->epsilon <= 1e-2)) return fail(ctx, BB_ERR_INVALID_ARG, "epsilon must be in [1e-7, 1e-2]");
  for (int i = 0; i < 3; ++i)
    if (!finite_pos(o->uvw_max[i])) return fail(ctx, BB_ERR_INVALID_ARG, "uvw_max must be finite and > 0");
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(o->frame[i])) return fail(ctx, BB_ERR_INVALID_ARG, "frame must be finite");
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const double dot = o->frame[3 * a] * o->frame[3 * b] + o->frame[3 * a + 1] * o->frame[3 * b + 1] +
                         o->frame[3 * a + 2] * o->frame[3 * b + 2];
      if (std::fabs(dot - (a == b ? 1.0 : 0.0)) > 1e-9) return fail(ctx, BB_ERR_INVALID_ARG, "frame rows must be orthonormal");
    }
  if (n_pix < 1 || !pix_host) return fail(ctx, BB_ERR_INVALID_ARG, "need pixels (host copy) for planning");
  std::memset(&g, 0, sizeof g);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) g.R[a][b] = o->frame[3 * a + b];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t p = 0; p < n_pix; ++p) {
    const double a0 = pix_host[p], a1 = pix_host[p + n_pix], a2 = pix_host[p + 2 * n_pix];
    if (!std::isfinite(a0) || !std::isfinite(a1) || !std::isfinite(a2))
      return fail(ctx, BB_ERR_INVALID_ARG, "pixel %lld is not finite", (long long)p);
    for (int d = 0; d < 3; ++d) {
      const double r = (a0 * g.R[d][0] + a1 * g.R[d][1]) + a2 * g.R[d][2];
      lo[d] = std::min(lo[d], r);
      hi[d] = std::max(hi[d], r);
    }
  }
  g.w = kernel_width(o->epsilon);
  g.beta = (float)(2.30 * g.w);
  g.cell_q = cell.q;
  g.cell_i[0] = cell.iu;
  g.cell_i[1] = cell.iv;
  g.use_diag = cell.use_diag ? 1 : 0;
  for (int d = 0; d < 3; ++d) {
    g.D[d] = 0.5 * (lo[d] + hi[d]);
    const double S = std::max(0.5 * (hi[d] - lo[d]), 1e-12);
    g.Xf[d] = o->uvw_max[d];
    g.X[d] = o->uvw_max[d];
    g.C[d] = 0.0;
    if (cell.q > 1 && d < 2) {  // a cell of the uvw split: its half-width, and its centre as the source shift
      const int i = d == 0 ? cell.iu : cell.iv;
      g.X[d] = (g.Xf[d] / cell.q) * (1.0 + 1e-9);
      g.C[d] = (i + 0.5) * (2.0 * g.Xf[d] / cell.q) - g.Xf[d];
    }
    g.h[d] = 1.0 / (2.0 * kSigma * S);
    g.inv_h[d] = 1.0 / g.h[d];
    const double need = std::ceil(8.0 * g.X[d] * S) + g.w;
    if (!(need < 1.0e6)) return fail(ctx, BB_ERR_SHAPE, "grid axis %d would need %.3g points", d, need);
    g.N[d] = smooth_size(std::max<int64_t>(2 * g.w, (int64_t)need));
    g.M[d] = kSigma * g.N[d];
    g.hM[d] = g.h[d] * g.M[d];
    // The pixels sit at |eta| <= M/4 type-2 grid points from the centre (eta =
    // (s - D) h M, |s - D| <= S, h = 1/(4 S)); their kernels reach from
    // ceil(eta - w/2) to that plus w - 1.  One point of slack each side covers
    // the rounding of eta.
    const int lo = (int)std::ceil(-0.25 * g.M[d] - 0.5 * g.w) - 1;
    const int hi = (int)std::ceil(0.25 * g.M[d] - 0.5 * g.w) + g.w;
    if (hi - lo + 1 >= g.M[d]) {
      g.win_lo[d] = 0;
      g.win_len[d] = g.M[d];
    } else {
      g.win_lo[d] = ((lo % g.M[d]) + g.M[d]) % g.M[d];
      g.win_len[d] = hi - lo + 1;
    }
  }
  return BB_OK;
}

// The three batched 1-D inverse transforms of the pruned type-2 transform,
// in place on contiguous lines: A along axis 2, B along axis 1, C along axis 0.
struct FftPlans {
  rocfft_plan p[3] = {nullptr, nullptr, nullptr};
  void destroy() {
    for (rocfft_plan& q : p)
      if (q) {
        rocfft_plan_destroy(q);
        q = nullptr;
      }
  }
};

// Work-buffer bytes of the plans (max over the three), or (size_t)-1 on failure.
// With keep, the plans are handed over; otherwise destroyed.
size_t rocfft_work_bytes(const bb::NufftGeom& g, FftPlans* keep) {
  const StageSizes st = stage_sizes(g);
  const size_t len[3] = {(size_t)g.M[2], (size_t)g.M[1], (size_t)g.M[0]};
  const size_t batch[3] = {st.a / len[0], st.b / len[1], st.c / len[2]};
  FftPlans plans;
  size_t bytes = 0;
  for (int i = 0; i < 3; ++i) {
    if (rocfft_plan_create(&plans.p[i], rocfft_placement_inplace, rocfft_transform_type_complex_inverse,
                           rocfft_precision_single, 1, &len[i], batch[i], nullptr) != rocfft_status_success) {
      plans.p[i] = nullptr;
      plans.destroy();
      return (size_t)-1;
    }
    size_t b = 0;
    rocfft_plan_get_work_buffer_size(plans.p[i], &b);
    bytes = std::max(bytes, b);
  }
  if (keep)
    *keep = plans;
  else
    plans.destroy();
  return bytes;
}

NufftLayout nufft_layout(const bb::NufftGeom& g, int n_levels, int64_t n_pix, size_t work_bytes, bool line_fft) {
  NufftLayout l{};
  const size_t n_cell = (size_t)g.N[0] * g.N[1] * g.N[2];
  size_t p = 0;  // transient region
  l.grid = p;
  p += align_up(8 * n_cell * (size_t)n_levels);
  if (line_fft) {
    const StageSizes st = line_stage_sizes(g);
    l.stage_ac = p;
    p += align_up(8 * std::max(st.a, st.b));
    l.stage_b = p;
    p += align_up(8 * std::max(st.b, st.c));
  } else {
    const StageSizes st = stage_sizes(g);
    l.stage_ac = p;
    p += align_up(8 * std::max(st.a, st.c));
    l.stage_b = p;
    p += align_up(8 * st.b);
  }
  l.work = p;
  l.work_bytes = work_bytes;
  p += align_up(std::max<size_t>(work_bytes, 1));
  l.t_total = p;
  p = 0;  // persistent region
  if (line_fft)
    for (int d = 0; d < 3; ++d) {
      l.perm[d] = p;
      p += align_up(4 * (size_t)g.M[d]);
      l.tw[d] = p;
      p += align_up(8 * (size_t)g.M[d]);
      l.dft[d] = p;
      if (g.M[d] <= bb::kLineDftMax) p += align_up(8 * (size_t)g.N[d] * g.win_len[d]);
    }
  l.psi0 = p;
  p += align_up(4 * (size_t)g.N[0]);
  l.psi1 = p;
  p += align_up(4 * (size_t)g.N[1]);
  l.psi2 = p;
  p += align_up(4 * (size_t)g.N[2]);
  l.corr = p;
  p += align_up(8 * (size_t)n_pix);
  l.quad_t = p;
  p += align_up(8 * kQuadNodes);
  l.quad_wphi = p;
  p += align_up(8 * kQuadNodes);
  l.diag = p;
  p += align_up(8 * bb::kMaxLevels);
  l.err = p;
  p += bb_host::kAlign;
  l.p_total = p;
  l.total = l.t_total + l.p_total;
  return l;
}

std::once_flag g_rocfft_once;
rocfft_status g_rocfft_setup = rocfft_status_success;

}  // namespace

// A tile of a partitioned plan's pixels (image-domain partition): its own
// plan (grid sized to the tile), whose images are moved into the partitioned
// plan's images after each call.
struct NufftPart {
  bb_nufft sub = nullptr;
  int64_t n = 0;    // pixels
  int64_t* idx;     // device: indices of its pixels in the plan's pixel list
  float* img;       // device: its level images [n_levels][n]
};

struct bb_nufft_ {
  bb_context ctx = nullptr;
  std::vector<NufftPart> parts;  // non-empty: a partitioned plan (the fields below describe its largest part)
  int cells = 1;                 // uvw cells per axis of every part's plan
  bb_nufft_options opt{};
  bb::NufftGeom g{};
  int64_t n_pix = 0;
  const double* pix = nullptr;
  float* images = nullptr;
  char* tws = nullptr;  // transient region (shared by the parts of a partitioned plan)
  char* pws = nullptr;  // persistent region
  NufftLayout lay{};
  bool line_fft = false;
  bb::LineFft lf[3]{};  // line-FFT stages: axis 2, axis 1, axis 0
  FftPlans plans;
  rocfft_execution_info info = nullptr;
  int64_t count = 0;  // instances spread since the last emit
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool spread_timed = false, emit_timed = false;
};

namespace {

template <class T>
T* tnat(bb_nufft h, size_t off) {
  return reinterpret_cast<T*>(h->tws + off);
}
template <class T>
T* pnat(bb_nufft h, size_t off) {
  return reinterpret_cast<T*>(h->pws + off);
}

// Point a plan made for uvw cells at cell (iu, iv): its source shift and
// whether its interpolation adds the level diagonals (the first cell does).
void set_cell(bb::NufftGeom& g, int iu, int iv) {
#pragma clang fp contract(off)
  const int idx[2] = {iu, iv};
  for (int d = 0; d < 2; ++d) g.C[d] = (idx[d] + 0.5) * (2.0 * g.Xf[d] / g.cell_q) - g.Xf[d];
  g.C[2] = 0.0;
  g.cell_i[0] = iu;
  g.cell_i[1] = iv;
  g.use_diag = (iu == 0 && iv == 0) ? 1 : 0;
}

bb_status plan_size(bb_context ctx, const bb_nufft_options* o, int64_t n_pix, const double* pix_host,
                    const CellSpec& cell, bb::NufftGeom& g, bool& line_fft, NufftLayout& lay) {
  bb_status st = nufft_geometry(ctx, o, n_pix, pix_host, g, cell);
  if (st != BB_OK) return st;
  line_fft = use_line_fft(g, o->transform, ctx->device);
  size_t work = 0;
  if (!line_fft) {
    std::call_once(g_rocfft_once, [] { g_rocfft_setup = rocfft_setup(); });
    if (g_rocfft_setup != rocfft_status_success) return fail(ctx, BB_ERR_DEVICE, "rocfft_setup failed");
    work = rocfft_work_bytes(g, nullptr);
    if (work == (size_t)-1) return fail(ctx, BB_ERR_DEVICE, "rocfft_plan_create failed");
  }
  lay = nufft_layout(g, o->n_levels, n_pix, work, line_fft);
  return BB_OK;
}

bb_status create_one(bb_context ctx, const bb_nufft_options* opt, int64_t n_pix, const double* pix_host,
                     const double* pix_xyz, float* images, char* tws, char* pws, const CellSpec& cell,
                     bb_nufft* out);

// ---- partitions (Section 3.4.1) ----------------------------------------------
// The pixels are split into P x P tiles of their extent along e_u and e_v;
// each nonempty tile gets a plan (grid sized to the tile, and to one uvw cell
// when the baselines are split too) with its own pixel array, images and
// persistent region, carved from the caller's workspace after one transient
// region sized for the largest tile, which every tile's plan uses in turn.
struct PartLayout {
  std::vector<std::vector<int64_t>> tiles;  // pixel indices per nonempty tile
  std::vector<std::vector<double>> pix;     // host copy of each tile's pixels (column-major)
  std::vector<size_t> idx, px, img, pers;
  size_t trans_bytes = 0, total = 0;
};

bb_status part_layout(bb_context ctx, const bb_nufft_options* o, int64_t n_pix, const double* pix_host,
                      PartLayout& L) {
#pragma clang fp contract(off)
  bb_nufft_options one = *o;
  one.partitions = 1;
  one.uvw_partitions = 1;
  bb::NufftGeom g;
  bb_status st = nufft_geometry(ctx, &one, n_pix, pix_host, g);  // validates the options and every pixel
  if (st != BB_OK) return st;
  if (o->partitions < 0 || o->partitions > 8) return fail(ctx, BB_ERR_INVALID_ARG, "partitions must be in [0, 8]");
  if (o->uvw_partitions < 0 || o->uvw_partitions > 16)
    return fail(ctx, BB_ERR_INVALID_ARG, "uvw_partitions must be in [0, 16]");
  const int P = std::max(1, o->partitions);
  CellSpec cell;
  cell.q = std::max(1, o->uvw_partitions);
  std::vector<double> u(n_pix), v(n_pix);
  double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
  for (int64_t p = 0; p < n_pix; ++p) {
    const double a0 = pix_host[p], a1 = pix_host[p + n_pix], a2 = pix_host[p + 2 * n_pix];
    u[p] = (a0 * o->frame[0] + a1 * o->frame[1]) + a2 * o->frame[2];
    v[p] = (a0 * o->frame[3] + a1 * o->frame[4]) + a2 * o->frame[5];
    lo[0] = std::min(lo[0], u[p]);
    hi[0] = std::max(hi[0], u[p]);
    lo[1] = std::min(lo[1], v[p]);
    hi[1] = std::max(hi[1], v[p]);
  }
  auto tile_of = [&](double x, int d) {
    const double span = hi[d] - lo[d];
    if (!(span > 0.0)) return 0;
    return std::min(P - 1, std::max(0, (int)((x - lo[d]) / span * P)));
  };
  std::vector<std::vector<int64_t>> t(P * P);
  for (int64_t p = 0; p < n_pix; ++p) t[tile_of(u[p], 0) * P + tile_of(v[p], 1)].push_back(p);
  std::vector<NufftLayout> lays;
  for (auto& tile : t) {
    if (tile.empty()) continue;
    const int64_t n = (int64_t)tile.size();
    std::vector<double> px(3 * n);
    for (int64_t i = 0; i < n; ++i)
      for (int d = 0; d < 3; ++d) px[i + d * n] = pix_host[tile[i] + d * n_pix];
    bb::NufftGeom gt;
    bool line = false;
    NufftLayout lay;
    st = plan_size(ctx, &one, n, px.data(), cell, gt, line, lay);
    if (st != BB_OK) return st;
    L.trans_bytes = std::max(L.trans_bytes, lay.t_total);
    lays.push_back(lay);
    L.tiles.push_back(std::move(tile));
    L.pix.push_back(std::move(px));
  }
  size_t off = align_up(L.trans_bytes);
  for (size_t k = 0; k < L.tiles.size(); ++k) {
    const int64_t n = (int64_t)L.tiles[k].size();
    L.idx.push_back(off);
    off += align_up(8 * (size_t)n);
    L.px.push_back(off);
    off += align_up(24 * (size_t)n);
    L.img.push_back(off);
    off += align_up(4 * (size_t)o->n_levels * n);
    L.pers.push_back(off);
    off += align_up(lays[k].p_total);
  }
  L.total = off;
  return BB_OK;
}

bb_status part_destroy(bb_nufft h) {
  bb_context ctx = h->ctx;
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  for (NufftPart& q : h->parts)
    if (q.sub) bb_nufft_destroy(q.sub);
  for (hipEvent_t& e : h->ev)
    if (e) hipEventDestroy(e);
  delete h;
  return BB_OK;
}

bb_status part_create(bb_context ctx, const bb_nufft_options* opt, int64_t n_pix, const double* pix_host,
                      const double* pix_xyz, float* images, void* workspace, size_t ws_bytes, bb_nufft* out) {
  PartLayout L;
  bb_status st = part_layout(ctx, opt, n_pix, pix_host, L);
  if (st != BB_OK) return st;
  if (!pix_xyz || !images || !workspace) return fail(ctx, BB_ERR_INVALID_ARG, "null device pointer");
  if (reinterpret_cast<uintptr_t>(workspace) % bb_host::kAlign)
    return fail(ctx, BB_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total) return fail(ctx, BB_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.total);
  BB_HIP(ctx, hipSetDevice(ctx->device));
  bb_nufft h = new (std::nothrow) bb_nufft_;
  if (!h) return fail(ctx, BB_ERR_DEVICE, "out of host memory");
  h->ctx = ctx;
  h->opt = *opt;
  h->n_pix = n_pix;
  h->pix = pix_xyz;
  h->images = images;
  h->cells = std::max(1, opt->uvw_partitions);
  h->tws = static_cast<char*>(workspace);
  h->pws = static_cast<char*>(workspace);
  for (hipEvent_t& e : h->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      part_destroy(h);
      return fail(ctx, BB_ERR_DEVICE, "hipEventCreate failed");
    }
  bb_nufft_options one = *opt;
  one.partitions = 1;
  one.uvw_partitions = 1;
  CellSpec cell;
  cell.q = h->cells;
  hipStream_t s = ctx->stream;
  int64_t biggest = -1;
  for (size_t t = 0; t < L.tiles.size(); ++t) {
    NufftPart q;
    q.n = (int64_t)L.tiles[t].size();
    q.idx = pnat<int64_t>(h, L.idx[t]);
    q.img = pnat<float>(h, L.img[t]);
    double* px = pnat<double>(h, L.px[t]);
    // pageable source: the copy is staged before the call returns
    if (hipMemcpyAsync(q.idx, L.tiles[t].data(), 8 * (size_t)q.n, hipMemcpyHostToDevice, s) != hipSuccess ||
        bb::launch_nufft_gather_pix(pix_xyz, n_pix, q.idx, q.n, px, s) != hipSuccess ||
        bb::launch_fill_zero(q.img, (int64_t)opt->n_levels * q.n, s) != hipSuccess) {
      part_destroy(h);
      return fail(ctx, BB_ERR_DEVICE, "partition set-up failed");
    }
    st = create_one(ctx, &one, q.n, L.pix[t].data(), px, q.img, h->tws, h->pws + L.pers[t], cell, &q.sub);
    if (st != BB_OK) {
      part_destroy(h);
      return st;
    }
    const int64_t cells = (int64_t)q.sub->g.N[0] * q.sub->g.N[1] * q.sub->g.N[2];
    if (cells > biggest) {
      biggest = cells;
      h->g = q.sub->g;
    }
    h->parts.push_back(q);
  }
  ctx->live += 1;
  *out = h;
  return BB_OK;
}

// A plan over the given pixels whose transient region is at tws and
// persistent region at pws (sized by plan_size for the same arguments).
bb_status create_one(bb_context ctx, const bb_nufft_options* opt, int64_t n_pix, const double* pix_host,
                     const double* pix_xyz, float* images, char* tws, char* pws, const CellSpec& cell,
                     bb_nufft* out) {
  *out = nullptr;
  bb::NufftGeom g;
  bb_status st = nufft_geometry(ctx, opt, n_pix, pix_host, g, cell);
  if (st != BB_OK) return st;
  const bool line_fft = use_line_fft(g, opt->transform, ctx->device);
  BB_HIP(ctx, hipSetDevice(ctx->device));
  FftPlans plans;
  size_t work = 0;
  if (!line_fft) {
    std::call_once(g_rocfft_once, [] { g_rocfft_setup = rocfft_setup(); });
    if (g_rocfft_setup != rocfft_status_success) return fail(ctx, BB_ERR_DEVICE, "rocfft_setup failed");
    work = rocfft_work_bytes(g, &plans);
    if (work == (size_t)-1) return fail(ctx, BB_ERR_DEVICE, "rocfft_plan_create failed");
  }
  const NufftLayout lay = nufft_layout(g, opt->n_levels, n_pix, work, line_fft);
  bb_nufft h = new (std::nothrow) bb_nufft_;
  if (!h) {
    plans.destroy();
    return fail(ctx, BB_ERR_DEVICE, "out of host memory");
  }
  h->ctx = ctx;
  h->opt = *opt;
  h->g = g;
  h->n_pix = n_pix;
  h->pix = pix_xyz;
  h->images = images;
  h->tws = tws;
  h->pws = pws;
  h->lay = lay;
  h->plans = plans;
  h->line_fft = line_fft;
  if (line_fft) {
    const int64_t w0 = g.win_len[0], w1 = g.win_len[1], w2 = g.win_len[2];
    for (int st = 0; st < 3; ++st) {
      const int d = 2 - st;
      bb::LineFft& p = h->lf[st];
      bb::line_fft_plan(g.M[d], p);
      p.n_in = g.N[d];
      p.win_lo = g.win_lo[d];
      p.win_len = g.win_len[d];
      p.direct = bb::line_dft_fits(p) ? 1 : 0;
    }
    h->lf[0].n_lines = (int64_t)g.N[0] * g.N[1];  // grid lines along axis 2 -> A'[i0][w2][i1]
    h->lf[0].in_stride = g.N[2];
    h->lf[0].out_mode = 1;
    h->lf[0].t_inner = g.N[1];
    h->lf[1].n_lines = (int64_t)g.N[0] * w2;  // A' lines along axis 1 -> B[i0][w2][w1]
    h->lf[1].in_stride = g.N[1];
    h->lf[1].out_stride = w1;
    h->lf[2].n_lines = w2 * w1;  // B' lines along axis 0 -> C[w2][w1][w0]
    h->lf[2].in_stride = g.N[0];
    h->lf[2].out_stride = w0;
  }
  auto bail = [&](const char* what) {
    if (h->info) rocfft_execution_info_destroy(h->info);
    h->plans.destroy();
    for (hipEvent_t& e : h->ev)
      if (e) hipEventDestroy(e);
    delete h;
    return fail(ctx, BB_ERR_DEVICE, "%s", what);
  };
  if (!line_fft) {
    if (rocfft_execution_info_create(&h->info) != rocfft_status_success)
      return bail("rocfft_execution_info_create failed");
    if (work > 0 && rocfft_execution_info_set_work_buffer(h->info, h->tws + lay.work, work) != rocfft_status_success)
      return bail("rocfft_execution_info_set_work_buffer failed");
    if (rocfft_execution_info_set_stream(h->info, ctx->stream) != rocfft_status_success)
      return bail("rocfft_execution_info_set_stream failed");
  }
  for (hipEvent_t& e : h->ev)
    if (hipEventCreate(&e) != hipSuccess) return bail("hipEventCreate failed");

  // host tables: 1 / type-2 kernel transform per stored grid index, quadrature
  std::vector<double> qt, qw;
  gauss_legendre(kQuadNodes, qt, qw);
  std::vector<double> wphi(kQuadNodes);
  for (int j = 0; j < kQuadNodes; ++j) wphi[j] = qw[j] * es_kernel_host(qt[j], (double)g.beta);
  std::vector<float> psi[3];
  for (int d = 0; d < 3; ++d) {
    psi[d].resize(g.N[d]);
    const double a = 0.5 * g.w;
    for (int i = 0; i < g.N[d]; ++i) {
      const int freq = i < g.N[d] / 2 ? i : i - g.N[d];
      const double k = freq * (2.0 * M_PI / g.M[d]);
      double acc = 0.0;
      for (int j = 0; j < kQuadNodes; ++j) acc += wphi[j] * std::cos(k * a * qt[j]);
      psi[d][i] = (float)(1.0 / (a * acc));  // psi_hat(g) M / (2 pi), inverted
    }
  }
  std::vector<int> perm[3];
  std::vector<float> tw[3], dft[3];
  if (line_fft)
    for (int d = 0; d < 3; ++d) {
      perm[d].resize(g.M[d]);
      bb::line_fft_perm(h->lf[2 - d], perm[d].data());
      tw[d].assign(2 * (size_t)g.M[d], 0.0f);
      bb::line_fft_twiddles(h->lf[2 - d], tw[d].data());
      if (h->lf[2 - d].direct) {
        dft[d].assign(2 * (size_t)g.N[d] * g.win_len[d], 0.0f);
        bb::line_dft_table(h->lf[2 - d], psi[d].data(), dft[d].data());
      }
    }
  hipStream_t s = ctx->stream;
  if (bb_host::debug_fill() && (bb::launch_fill_poison(h->tws, lay.t_total, s) != hipSuccess ||
                                bb::launch_fill_poison(h->pws, lay.p_total, s) != hipSuccess))
    return bail("debug fill failed");
  for (int d = 0; d < 3 && line_fft; ++d)
    if (hipMemcpyAsync(pnat<int>(h, lay.perm[d]), perm[d].data(), 4 * perm[d].size(), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(pnat<float>(h, lay.tw[d]), tw[d].data(), 4 * tw[d].size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        (!dft[d].empty() && hipMemcpyAsync(pnat<float>(h, lay.dft[d]), dft[d].data(), 4 * dft[d].size(),
                                           hipMemcpyHostToDevice, s) != hipSuccess))
      return bail("table upload failed");
  // pageable sources: each copy is staged before the call returns
  if (hipMemcpyAsync(pnat<float>(h, lay.psi0), psi[0].data(), 4 * psi[0].size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(pnat<float>(h, lay.psi1), psi[1].data(), 4 * psi[1].size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(pnat<float>(h, lay.psi2), psi[2].data(), 4 * psi[2].size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(pnat<double>(h, lay.quad_t), qt.data(), 8 * kQuadNodes, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(pnat<double>(h, lay.quad_wphi), wphi.data(), 8 * kQuadNodes, hipMemcpyHostToDevice, s) != hipSuccess)
    return bail("table upload failed");
  if (bb::launch_nufft_corr(g, pix_xyz, n_pix, n_pix, pnat<double>(h, lay.quad_t), pnat<double>(h, lay.quad_wphi),
                            kQuadNodes, pnat<double>(h, lay.corr), s) != hipSuccess ||
      bb::launch_fill_zero(tnat<float>(h, lay.grid), (int64_t)2 * g.N[0] * g.N[1] * g.N[2] * opt->n_levels, s) !=
          hipSuccess ||
      bb::launch_fill_zero_f64(pnat<double>(h, lay.diag), bb::kMaxLevels, s) != hipSuccess ||
      bb::launch_fill_zero(pnat<float>(h, lay.err), 1, s) != hipSuccess)
    return bail("plan set-up launch failed");
  if (hipStreamSynchronize(s) != hipSuccess) return bail("plan set-up failed on the device");
  ctx->live += 1;
  *out = h;
  return BB_OK;
}

}  // namespace

extern "C" {

bb_status bb_nufft_workspace_size(bb_context ctx, const bb_nufft_options* opt, int64_t n_pix, const double* pix_host,
                                  size_t* bytes) {
  if (!ctx || !bytes) return BB_ERR_INVALID_ARG;
  if (opt && (opt->partitions > 1 || opt->uvw_partitions > 1)) {
    PartLayout L;
    const bb_status st = part_layout(ctx, opt, n_pix, pix_host, L);
    if (st == BB_OK) *bytes = L.total;
    return st;
  }
  bb::NufftGeom g;
  bool line_fft = false;
  NufftLayout lay;
  const bb_status st = plan_size(ctx, opt, n_pix, pix_host, CellSpec{}, g, line_fft, lay);
  if (st == BB_OK) *bytes = lay.total;
  return st;
}

bb_status bb_nufft_create(bb_context ctx, const bb_nufft_options* opt, int64_t n_pix, const double* pix_host,
                          const double* pix_xyz, float* images, void* workspace, size_t ws_bytes, bb_nufft* out) {
  if (!ctx || !out) return BB_ERR_INVALID_ARG;
  *out = nullptr;
  if (opt && (opt->partitions > 1 || opt->uvw_partitions > 1))
    return part_create(ctx, opt, n_pix, pix_host, pix_xyz, images, workspace, ws_bytes, out);
  bb::NufftGeom g;
  bool line_fft = false;
  NufftLayout lay;
  bb_status st = plan_size(ctx, opt, n_pix, pix_host, CellSpec{}, g, line_fft, lay);
  if (st != BB_OK) return st;
  if (!pix_xyz || !images || !workspace) return fail(ctx, BB_ERR_INVALID_ARG, "null device pointer");
  if (reinterpret_cast<uintptr_t>(workspace) % bb_host::kAlign)
    return fail(ctx, BB_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < lay.total) return fail(ctx, BB_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, lay.total);
  char* ws = static_cast<char*>(workspace);
  return create_one(ctx, opt, n_pix, pix_host, pix_xyz, images, ws, ws + lay.t_total, CellSpec{}, out);
}

bb_status bb_nufft_shape(bb_nufft h, int32_t* spread_grid, int32_t* fft_grid, int32_t* kernel_width_out) {
  if (!h) return BB_ERR_INVALID_ARG;
  for (int d = 0; d < 3; ++d) {
    if (spread_grid) spread_grid[d] = h->g.N[d];
    if (fft_grid) fft_grid[d] = h->g.M[d];
  }
  if (kernel_width_out) *kernel_width_out = h->g.w;
  return BB_OK;
}

}  // extern "C"

namespace {

// Per-call workspace of a spread call (byte offsets).
struct CallLayout {
  size_t inst, order, lstart, vp, count, offset, cursor, list, nch, choff, scan_tmp, rec, cv, nparts, part_off, total;
  int mode = 0;  // 2: output-driven spread, 1: LDS tiles, 0: global atomics
  int bin = 0, n_bins = 0, n_blocks = 0;
  int64_t pairs = 0;
};

CallLayout call_layout(bb_nufft h, int32_t n_inst, const bb_instance* inst) {
  CallLayout c{};
  size_t n_eig = 0, vp = 0, pairs = 0;
  for (int i = 0; i < n_inst; ++i) {
    const size_t L = (size_t)std::max(inst[i].n_ant, 0);
    n_eig += (size_t)std::max(inst[i].n_eig, 0);
    vp += (size_t)h->opt.n_levels * L * L;
    pairs += L * (L > 0 ? L - 1 : 0) / 2;
  }
  c.pairs = (int64_t)pairs;
  c.mode = bb::nufft_gather_z(h->g) > 0 ? 2 : bb::nufft_tile_size(h->g) > 0 ? 1 : 0;
  c.bin = c.mode == 2 ? 1 : c.mode == 1 ? bb::nufft_tile_size(h->g) : 0;
  size_t p = 0;
  c.inst = p;
  p += align_up(sizeof(bb::NufftInst) * n_inst);
  c.order = p;
  p += align_up(4 * n_eig);
  c.lstart = p;
  p += align_up(4 * (size_t)n_inst * (h->opt.n_levels + 1));
  if (c.mode > 0) {
    c.n_bins = ((h->g.N[0] + c.bin - 1) / c.bin) * ((h->g.N[1] + c.bin - 1) / c.bin);
    int scan_n = c.n_bins;
    if (c.mode == 2) {
      int nbx, nby;
      bb::nufft_gather_blocks(h->g, nbx, nby);
      c.n_blocks = nbx * nby;
      scan_n = std::max(scan_n, c.n_blocks);
      const size_t lv_pad = (size_t)((h->opt.n_levels + 1) & ~1);
      c.rec = p;
      p += align_up((size_t)bb::kGatherRecBytes * std::max<size_t>(pairs, 1));
      c.cv = p;
      p += align_up(8 * lv_pad * std::max<size_t>(pairs, 1));
      c.nparts = p;
      p += align_up(4 * (size_t)c.n_blocks);
      c.part_off = p;
      p += align_up(4 * ((size_t)c.n_blocks + 1));
    }
    c.scan_tmp = p;
    p += align_up(4 * (size_t)bb::scan_tmp_ints(scan_n));
    c.vp = p;
    p += align_up(8 * vp);
    c.count = p;
    p += align_up(4 * (size_t)c.n_bins);
    c.offset = p;
    p += align_up(4 * ((size_t)c.n_bins + 1));
    c.cursor = p;
    p += align_up(4 * (size_t)c.n_bins);
    c.list = p;
    p += align_up(8 * std::max<size_t>(pairs, 1));
    c.nch = p;  // tiles and bins share one grid
    p += align_up(4 * (size_t)c.n_bins);
    c.choff = p;
    p += align_up(4 * ((size_t)c.n_bins + 1));
  }
  c.total = p;
  return c;
}

}  // namespace

extern "C" {

bb_status bb_nufft_batched_workspace_size(bb_nufft h, int32_t n_inst, const bb_instance* inst, size_t* bytes) {
  if (!h || !bytes || n_inst < 1 || !inst) return BB_ERR_INVALID_ARG;
  if (!h->parts.empty()) {  // the parts run one after another on the stream: the largest need
    size_t most = 0;
    for (NufftPart& q : h->parts) most = std::max(most, call_layout(q.sub, n_inst, inst).total);
    *bytes = most;
    return BB_OK;
  }
  *bytes = call_layout(h, n_inst, inst).total;
  return BB_OK;
}

bb_status bb_nufft_collect_eig_batched(bb_nufft h, int32_t n_inst, const bb_instance* inst, int64_t n_ant_rows,
                                       int64_t n_w_elems, int64_t n_eig_elems, const double* ant_xyz_packed,
                                       const void* W_packed, const float* d_packed, const int32_t* level_packed,
                                       void* workspace, size_t ws_bytes) {
  if (!h) return BB_ERR_INVALID_ARG;
  bb_context ctx = h->ctx;
  if (!h->parts.empty()) {
    // one NUFFT per (tile, uvw cell), one after another on the shared grid:
    // spread the cell's baselines, transform, interpolate into the tile's
    // images; then move the tile's images into the plan's
    BB_HIP(ctx, hipSetDevice(ctx->device));
    BB_HIP(ctx, hipEventRecord(h->ev[0], ctx->stream));
    for (NufftPart& q : h->parts) {
      const bb::NufftGeom& gq = q.sub->g;
      const int64_t grid_floats = 2 * (int64_t)gq.N[0] * gq.N[1] * gq.N[2] * h->opt.n_levels;
      for (int iu = 0; iu < h->cells; ++iu)
        for (int iv = 0; iv < h->cells; ++iv) {
          if (h->cells > 1) set_cell(q.sub->g, iu, iv);
          // the other tiles' transform stages share this region: clear the grid first
          BB_HIP(ctx, bb::launch_fill_zero(tnat<float>(q.sub, q.sub->lay.grid), grid_floats, ctx->stream));
          bb_status st = bb_nufft_collect_eig_batched(q.sub, n_inst, inst, n_ant_rows, n_w_elems, n_eig_elems,
                                                      ant_xyz_packed, W_packed, d_packed, level_packed, workspace,
                                                      ws_bytes);
          if (st == BB_OK) st = bb_nufft_emit(q.sub);
          if (st != BB_OK) return st;
        }
      BB_HIP(ctx, bb::launch_nufft_scatter_images(q.img, q.n, h->opt.n_levels, q.idx, h->images, h->n_pix,
                                                  ctx->stream));
    }
    BB_HIP(ctx, hipEventRecord(h->ev[1], ctx->stream));
    h->spread_timed = true;
    h->count += n_inst;
    return BB_OK;
  }
  if (n_inst < 1 || n_inst > 65535 || !inst) return fail(ctx, BB_ERR_INVALID_ARG, "n_inst must be in [1, 65535]");
  if (!ant_xyz_packed || !W_packed || !d_packed || !level_packed || !workspace)
    return fail(ctx, BB_ERR_INVALID_ARG, "null device pointer");
  if (reinterpret_cast<uintptr_t>(workspace) % bb_host::kAlign)
    return fail(ctx, BB_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  const int n_levels = h->opt.n_levels;
  std::vector<bb::NufftInst> ni(n_inst);
  int64_t ord_off = 0, vp_off = 0;
  int max_ant = 0;
  for (int i = 0; i < n_inst; ++i) {
    const bb_instance& b = inst[i];
    if (b.n_ant < 2 || b.n_ant > h->opt.n_ant_max)
      return fail(ctx, BB_ERR_SHAPE, "instance %d: n_ant %d outside [2, %d]", i, b.n_ant, h->opt.n_ant_max);
    if (b.n_eig < 1 || b.n_eig > h->opt.k_max)
      return fail(ctx, BB_ERR_SHAPE, "instance %d: n_eig %d outside [1, %d]", i, b.n_eig, h->opt.k_max);
    if (b.slot != 0) return fail(ctx, BB_ERR_INVALID_ARG, "instance %d: slot must be 0", i);
    if (!finite_pos(b.wavelength_m)) return fail(ctx, BB_ERR_INVALID_ARG, "instance %d: bad wavelength", i);
    if (b.ant_off < 0 || b.ant_off + b.n_ant > n_ant_rows || b.w_off < 0 || b.eig_off < 0)
      return fail(ctx, BB_ERR_INVALID_ARG, "instance %d: offsets out of range", i);
    if (b.w_off + (int64_t)b.n_ant * b.n_eig > n_w_elems || b.eig_off + b.n_eig > n_eig_elems)
      return fail(ctx, BB_ERR_INVALID_ARG, "instance %d: W block or eigenpairs beyond the packed arrays", i);
    bb::NufftInst& d = ni[i];
    d.n_ant = b.n_ant;
    d.n_eig = b.n_eig;
    d.wavelength_m = b.wavelength_m;
    d.ant_off = b.ant_off;
    d.w_off = b.w_off;
    d.eig_off = b.eig_off;
    d.ord_off = ord_off;
    d.ls_off = (int64_t)i * (n_levels + 1);
    d.vp_off = vp_off;
    ord_off += b.n_eig;
    vp_off += (int64_t)n_levels * b.n_ant * b.n_ant;
    max_ant = std::max(max_ant, b.n_ant);
  }
  const CallLayout cl = call_layout(h, n_inst, inst);
  if (ws_bytes < cl.total) return fail(ctx, BB_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, cl.total);
  char* ws = static_cast<char*>(workspace);
  bb::NufftInst* d_inst = reinterpret_cast<bb::NufftInst*>(ws + cl.inst);
  int* d_order = reinterpret_cast<int*>(ws + cl.order);
  int* d_lstart = reinterpret_cast<int*>(ws + cl.lstart);
  BB_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  if (bb_host::debug_fill()) BB_HIP(ctx, bb::launch_fill_poison(ws, cl.total, s));
  BB_HIP(ctx, hipEventRecord(h->ev[0], s));
  // pageable source: the copy is staged before the call returns
  BB_HIP(ctx, hipMemcpyAsync(d_inst, ni.data(), sizeof(bb::NufftInst) * n_inst, hipMemcpyHostToDevice, s));
  BB_HIP(ctx, bb::launch_nufft_prep(d_inst, n_inst, W_packed, d_packed, level_packed, n_levels, d_order, d_lstart,
                                    pnat<double>(h, h->lay.diag), pnat<int>(h, h->lay.err), s));
  const int64_t n_cell = (int64_t)h->g.N[0] * h->g.N[1] * h->g.N[2];
  if (cl.mode > 0) {
    BB_HIP(ctx, bb::launch_nufft_vprime(d_inst, n_inst, max_ant, W_packed, d_packed, d_order, d_lstart, n_levels,
                                        ws + cl.vp, s));
    int* count = reinterpret_cast<int*>(ws + cl.count);
    int* offset = reinterpret_cast<int*>(ws + cl.offset);
    int* cursor = reinterpret_cast<int*>(ws + cl.cursor);
    uint64_t* list = reinterpret_cast<uint64_t*>(ws + cl.list);
    int* scan_tmp = reinterpret_cast<int*>(ws + cl.scan_tmp);
    BB_HIP(ctx, bb::launch_nufft_bin(h->g, d_inst, n_inst, max_ant, ant_xyz_packed, n_ant_rows, cl.bin, count, offset,
                                     cursor, list, pnat<int>(h, h->lay.err), scan_tmp, s));
  }
  if (cl.mode == 2) {
    BB_HIP(ctx, bb::launch_nufft_spread_gather(h->g, d_inst, cl.pairs, ant_xyz_packed, n_ant_rows, ws + cl.vp,
                                               reinterpret_cast<int*>(ws + cl.offset),
                                               reinterpret_cast<uint64_t*>(ws + cl.list), n_levels, ws + cl.rec,
                                               ws + cl.cv, reinterpret_cast<int*>(ws + cl.nparts),
                                               reinterpret_cast<int*>(ws + cl.part_off),
                                               reinterpret_cast<int*>(ws + cl.scan_tmp), tnat<float>(h, h->lay.grid),
                                               n_cell, s));
  } else if (cl.mode == 1) {
    const int* offset = reinterpret_cast<int*>(ws + cl.offset);
    const uint64_t* list = reinterpret_cast<uint64_t*>(ws + cl.list);
    BB_HIP(ctx, bb::launch_nufft_spread_tiles(h->g, d_inst, ant_xyz_packed, n_ant_rows, ws + cl.vp, offset, list,
                                              cl.bin, n_levels, reinterpret_cast<int*>(ws + cl.nch),
                                              reinterpret_cast<int*>(ws + cl.choff), tnat<float>(h, h->lay.grid), n_cell,
                                              s));
  } else {
    BB_HIP(ctx, bb::launch_nufft_spread(h->g, d_inst, n_inst, max_ant, ant_xyz_packed, n_ant_rows, W_packed, d_packed,
                                        d_order, d_lstart, n_levels, tnat<float>(h, h->lay.grid), n_cell,
                                        pnat<int>(h, h->lay.err), s));
  }
  BB_HIP(ctx, hipEventRecord(h->ev[1], s));
  h->spread_timed = true;
  h->count += n_inst;
  return BB_OK;
}

bb_status bb_nufft_emit(bb_nufft h) {
  if (!h) return BB_ERR_INVALID_ARG;
  bb_context ctx = h->ctx;
  if (!h->parts.empty()) {  // each collect call already transformed its instances
    BB_HIP(ctx, hipSetDevice(ctx->device));
    BB_HIP(ctx, hipEventRecord(h->ev[2], ctx->stream));
    BB_HIP(ctx, hipEventRecord(h->ev[3], ctx->stream));
    h->emit_timed = true;
    h->count = 0;
    return BB_OK;
  }
  BB_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const bb::NufftGeom& g = h->g;
  const int64_t n_cell = (int64_t)g.N[0] * g.N[1] * g.N[2];
  void* ac = h->tws + h->lay.stage_ac;
  void* b = h->tws + h->lay.stage_b;
  const float* psi[3] = {pnat<float>(h, h->lay.psi0), pnat<float>(h, h->lay.psi1), pnat<float>(h, h->lay.psi2)};
  // the context's stream may have been rebound since the plan was made
  if (!h->line_fft && rocfft_execution_info_set_stream(h->info, s) != rocfft_status_success)
    return fail(ctx, BB_ERR_DEVICE, "rocfft_execution_info_set_stream failed");
  BB_HIP(ctx, hipEventRecord(h->ev[2], s));
  for (int lv = 0; lv < h->opt.n_levels; ++lv) {
    const float* level_grid = tnat<float>(h, h->lay.grid) + 2 * (int64_t)lv * n_cell;
    bb::InterpLayout il;
    const void* u;
    if (h->line_fft) {
      // axis 2: grid -> A'; axis 1: A' -> B; B -> B' (transpose); axis 0: B' -> C
      const int64_t w1 = g.win_len[1], w2 = g.win_len[2];
      auto line = [&](int st, const void* in, void* out) {
        const int d = 2 - st;
        return h->lf[st].direct
                   ? bb::launch_line_dft(h->lf[st], in, pnat<float2>(h, h->lay.dft[d]), out, s)
                   : bb::launch_line_fft(h->lf[st], in, psi[d], pnat<int>(h, h->lay.perm[d]),
                                         pnat<float2>(h, h->lay.tw[d]), out, s);
      };
      BB_HIP(ctx, line(0, level_grid, ac));
      BB_HIP(ctx, line(1, ac, b));
      BB_HIP(ctx, bb::launch_transpose_c64(b, g.N[0], w2 * w1, ac, s));
      BB_HIP(ctx, line(2, ac, b));
      il = {(int64_t)g.win_len[0], w1 * g.win_len[0], g.win_lo[0], g.win_len[0]};
      u = b;
    } else {
      // grid -> A (FFT along axis 2) -> B (axis 1) -> C (axis 0)
      void* const stage_in[3] = {const_cast<float*>(level_grid), ac, b};
      void* const stage_out[3] = {ac, b, ac};
      for (int st = 0; st < 3; ++st) {
        BB_HIP(ctx, bb::launch_nufft_gather(2 - st, g, stage_in[st], psi[2 - st], stage_out[st], s));
        void* buf[1] = {stage_out[st]};
        if (rocfft_execute(h->plans.p[st], buf, nullptr, h->info) != rocfft_status_success)
          return fail(ctx, BB_ERR_DEVICE, "rocfft_execute failed");
      }
      il = {(int64_t)g.win_len[2] * g.M[0], (int64_t)g.M[0], 0, g.M[0]};
      u = ac;
    }
    BB_HIP(ctx, bb::launch_nufft_interp(g, il, h->pix, h->n_pix, h->n_pix, static_cast<const float*>(u),
                                        pnat<double>(h, h->lay.corr), pnat<double>(h, h->lay.diag), lv,
                                        h->images + (int64_t)lv * h->n_pix, s));
  }
  BB_HIP(ctx, bb::launch_fill_zero(tnat<float>(h, h->lay.grid), 2 * n_cell * h->opt.n_levels, s));
  BB_HIP(ctx, bb::launch_fill_zero_f64(pnat<double>(h, h->lay.diag), bb::kMaxLevels, s));
  BB_HIP(ctx, hipEventRecord(h->ev[3], s));
  h->emit_timed = true;
  h->count = 0;
  return BB_OK;
}

bb_status bb_nufft_sync(bb_nufft h) {
  if (!h) return BB_ERR_INVALID_ARG;
  bb_context ctx = h->ctx;
  if (!h->parts.empty()) {  // every part's error word is read and cleared
    bb_status first = BB_OK;
    for (NufftPart& q : h->parts) {
      const bb_status st = bb_nufft_sync(q.sub);
      if (first == BB_OK) first = st;
    }
    return first;
  }
  BB_HIP(ctx, hipSetDevice(ctx->device));
  BB_HIP(ctx, hipStreamSynchronize(ctx->stream));
  int err = 0;
  BB_HIP(ctx, hipMemcpy(&err, pnat<int>(h, h->lay.err), sizeof err, hipMemcpyDeviceToHost));
  if (err) {
    BB_HIP(ctx, bb::launch_fill_zero(pnat<float>(h, h->lay.err), 1, ctx->stream));
    BB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::string msg;
    if (err & bb::kErrLevelId) msg += "a level id outside [-1, n_levels) was treated as -1; ";
    if (err & bb::kErrNufftExtent) msg += "a baseline beyond uvw_max was skipped; ";
    if (msg.size() >= 2) msg.resize(msg.size() - 2);
    return fail(ctx, BB_ERR_INVALID_ARG, "%s", msg.c_str());
  }
  return BB_OK;
}

bb_status bb_nufft_timings(bb_nufft h, double* ms_out, int32_t n) {
  if (!h || !ms_out || n < 1) return BB_ERR_INVALID_ARG;
  bb_context ctx = h->ctx;
  BB_HIP(ctx, hipSetDevice(ctx->device));
  BB_HIP(ctx, hipStreamSynchronize(ctx->stream));
  float a = 0.0f, b = 0.0f;
  if (h->spread_timed) BB_HIP(ctx, hipEventElapsedTime(&a, h->ev[0], h->ev[1]));
  if (h->emit_timed) BB_HIP(ctx, hipEventElapsedTime(&b, h->ev[2], h->ev[3]));
  ms_out[0] = a;
  if (n > 1) ms_out[1] = b;
  return BB_OK;
}

bb_status bb_nufft_destroy(bb_nufft h) {
  if (!h) return BB_ERR_INVALID_ARG;
  bb_context ctx = h->ctx;
  if (!h->parts.empty()) {
    ctx->live -= 1;
    return part_destroy(h);
  }
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  if (h->info) rocfft_execution_info_destroy(h->info);
  h->plans.destroy();
  for (hipEvent_t& e : h->ev)
    if (e) hipEventDestroy(e);
  ctx->live -= 1;
  delete h;
  return BB_OK;
}

}  // extern "C"
