// Host side of the C ABI declared in include/bluebild.h: argument validation,
// workspace carving, stream-ordered launches, the rocSOLVER eigensolve of the
// FP64 pre-step, status codes.  No exception crosses the ABI.

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "api_common.h"
#include "tune_cache.h"
#include "bb_internal.h"
#include "bluebild.h"

using bb::InstDesc;
using bb::InstDyn;


namespace {

using bb_host::align_up;
using bb_host::kAlign;

// Device metadata block for single-instance calls (written by a kernel from
// its arguments, so no host buffer has to outlive the call).
struct SingleMeta {
  InstDesc desc;
  InstDyn dyn;
  int group_slot;
  int group_begin[2];
  int inst_list;
};

struct Layout {  // byte offsets into a handle's workspace
  size_t meta, err, apack, xs, wts, levs, kbr, perm;
  size_t A, G, T, U, evals, E, info, dsel, lsel, wcol, solver, solver_bytes;
  size_t total;
};

size_t staging_bytes(int L_pad, int K_alloc, size_t* off_xs = nullptr, size_t* off_wts = nullptr,
                     size_t* off_levs = nullptr, size_t* off_kbr = nullptr, size_t* off_perm = nullptr) {
  size_t o = 0;
  o += align_up((size_t)2 * K_alloc * 2 * L_pad * 4);  // apack (fp32; bf16 hi+lo has the same size)
  if (off_xs) *off_xs = o;
  o += align_up((size_t)L_pad * 4 * 8);
  if (off_wts) *off_wts = o;
  o += align_up((size_t)K_alloc * 4);
  if (off_levs) *off_levs = o;
  o += align_up((size_t)K_alloc * 4);
  if (off_kbr) *off_kbr = o;
  o += align_up((size_t)(K_alloc / 32 + K_alloc / 16) * 8);
  if (off_perm) *off_perm = o;
  o += align_up((size_t)K_alloc * 4);
  return o;
}

Layout make_layout(const bb_options& o, size_t solver_bytes) {
  Layout l{};
  const int L_pad = bb::round_up(o.n_ant_max, bb::kAntChunk);
  const int K_alloc = bb::round_up(o.k_max, 32);
  const size_t Lm = (size_t)o.n_ant_max;
  size_t p = 0;
  l.meta = p;
  p += align_up(sizeof(SingleMeta));
  l.err = p;
  p += kAlign;
  l.apack = p;
  size_t xs, wts, levs, kbr, perm;
  const size_t st = staging_bytes(L_pad, K_alloc, &xs, &wts, &levs, &kbr, &perm);
  l.xs = p + xs;
  l.wts = p + wts;
  l.levs = p + levs;
  l.kbr = p + kbr;
  l.perm = p + perm;
  p += st;
  l.A = p;
  p += align_up(16 * Lm * Lm);
  l.G = p;
  p += align_up(16 * Lm * Lm);
  l.T = p;  // beamforming: G W_bf
  p += align_up(16 * Lm * Lm);
  l.U = p;  // beamforming: W_bf alpha
  p += align_up(16 * Lm * Lm);
  l.evals = p;
  p += align_up(8 * Lm);
  l.E = p;
  p += align_up(8 * Lm);
  l.info = p;
  p += kAlign;
  l.dsel = p;
  p += align_up(4 * Lm);
  l.lsel = p;
  p += align_up(4 * Lm);
  l.wcol = p;
  p += align_up(4 * Lm);
  l.solver = p;
  l.solver_bytes = solver_bytes;
  p += align_up(solver_bytes);
  l.total = p;
  return l;
}

}  // namespace

struct bb_synth_ {
  bb_context ctx = nullptr;
  bb_options opt{};
  int64_t n_pix = 0;
  const double* pix = nullptr;
  float* images = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  Layout lay{};
  int64_t count = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool timed = false;
  int tiles[bb::kKClasses] = {-1, -1, -1, -1};  // tile id per K class (set to the defaults at creation)
};

namespace {

using bb_host::fail;
using bb_host::finite_pos;

bb_status check_options(bb_context ctx, const bb_options* o) {
  if (!o) return fail(ctx, BB_ERR_INVALID_ARG, "options is NULL");
  if (o->n_levels < 1 || o->n_levels > bb::kMaxLevels)
    return fail(ctx, BB_ERR_INVALID_ARG, "n_levels must be in [1, %d]", bb::kMaxLevels);
  if (o->n_slots < 1) return fail(ctx, BB_ERR_INVALID_ARG, "n_slots must be >= 1");
  if (o->n_ant_max < 1 || o->n_ant_max > bb::kMaxAnt)
    return fail(ctx, BB_ERR_INVALID_ARG, "n_ant_max must be in [1, %d]", bb::kMaxAnt);
  if (o->k_max < 1 || o->k_max > bb::kMaxEig)
    return fail(ctx, BB_ERR_INVALID_ARG, "k_max must be in [1, %d]", bb::kMaxEig);
  if (o->precision < BB_PREC_FP32 || o->precision > BB_PREC_BF16X3_3M)
    return fail(ctx, BB_ERR_INVALID_ARG, "unknown precision %d", o->precision);
  if (o->filter != BB_FILTER_LSQ && o->filter != BB_FILTER_STD)
    return fail(ctx, BB_ERR_INVALID_ARG, "unknown filter %d", o->filter);
  if (o->gram != BB_GRAM_SINC && o->gram != BB_GRAM_IDENTITY)
    return fail(ctx, BB_ERR_INVALID_ARG, "unknown gram mode %d", o->gram);
  if (o->reserved != 0) return fail(ctx, BB_ERR_INVALID_ARG, "reserved option field must be 0");
  return BB_OK;
}

size_t solver_query(bb_context ctx, int n) {
  // Size query mode: rocSOLVER returns its workspace need without computing.
  // Null pointers make a call that is not honoured as a query fail its
  // argument check instead of launching.
  size_t sz = 0;
  if (rocblas_start_device_memory_size_query(ctx->rb) != rocblas_status_success) return 0;
  rocsolver_zhegvd(ctx->rb, rocblas_eform_ax, rocblas_evect_original, rocblas_fill_lower, n, nullptr, n, nullptr, n,
                   nullptr, nullptr, nullptr);
  if (rocblas_stop_device_memory_size_query(ctx->rb, &sz) != rocblas_status_success) return 0;
  return sz;
}

__global__ void write_meta_kernel(SingleMeta* dst, InstDesc d, int slot) {
  dst->desc = d;
  dst->group_slot = slot;
  dst->group_begin[0] = 0;
  dst->group_begin[1] = 1;
  dst->inst_list = 0;
}

__global__ void zero_int_kernel(int* p) { *p = 0; }

template <class T>
T* at(bb_synth h, size_t off) {
  return reinterpret_cast<T*>(h->ws + off);
}

InstDesc staging_desc(bb_synth h, char* base, int L, int K, double wl, int slot) {
  InstDesc d{};
  d.L = L;
  d.K = K;
  d.L_pad = bb::round_up(L, bb::kAntChunk);
  d.K_alloc = bb::round_up(K, 32);
  d.scale = 1.0 / wl;
  d.slot = slot;
  size_t xs, wts, levs, kbr, perm;
  staging_bytes(d.L_pad, d.K_alloc, &xs, &wts, &levs, &kbr, &perm);
  d.apack = base;
  d.xs = reinterpret_cast<double*>(base + xs);
  d.wts = reinterpret_cast<float*>(base + wts);
  d.levs = reinterpret_cast<int*>(base + levs);
  d.kbr = reinterpret_cast<int2*>(base + kbr);
  d.perm = reinterpret_cast<int*>(base + perm);
  (void)h;
  return d;
}

// Stage + synthesize one instance whose descriptor is `d` (its staging
// regions already point into `stage`'s owner), with the metadata block at
// `meta` and the device error word at `err`; ev_staged / ev_done (may be
// null) are recorded after staging and after the synthesis.
bb_status launch_single(bb_context ctx, SingleMeta* meta, int* err, const InstDesc& d, const double* pix,
                        int64_t n_pix, float* images, int n_levels, int precision, int tile, hipEvent_t ev_staged,
                        hipEvent_t ev_done) {
  hipStream_t s = ctx->stream;
  int nt = 0;
  if (!bb::synth_tile_info(precision, tile, nullptr, &nt, nullptr))
    return fail(ctx, BB_ERR_INVALID_ARG, "unknown tile %d", tile);
  InstDesc dd = d;
  dd.rows16 = bb::synth_tile_rows(precision, tile) == 16 ? 1 : 0;  // operand order of the tile
  hipLaunchKernelGGL(write_meta_kernel, dim3(1), dim3(1), 0, s, meta, dd, dd.slot);
  BB_HIP(ctx, hipGetLastError());
  BB_HIP(ctx, bb::launch_stage(&meta->desc, &meta->dyn, 1, d.K_alloc, d.L_pad, n_levels, precision, err, s));
  if (ev_staged) BB_HIP(ctx, hipEventRecord(ev_staged, s));
  bb::FwdParams p{};
  p.pix = pix;
  p.pix_ld = n_pix;
  p.n_pix = n_pix;
  p.descs = &meta->desc;
  p.dyn = &meta->dyn;
  p.group_slot = &meta->group_slot;
  p.group_begin = meta->group_begin;
  p.inst_list = &meta->inst_list;
  p.img = images;
  p.img_ld = n_pix;
  p.n_levels = n_levels;
  p.n_tiles = (n_pix + nt - 1) / nt;
  p.n_groups = 1;
  BB_HIP(ctx, bb::launch_synth_tile(p, precision, tile, s));
  if (ev_done) BB_HIP(ctx, hipEventRecord(ev_done, s));
  return BB_OK;
}

// Single-instance calls on a handle: staging in the handle's workspace.
bb_status run_single(bb_synth h, const InstDesc& d) {
  bb_status st = launch_single(h->ctx, at<SingleMeta>(h, h->lay.meta), at<int>(h, h->lay.err), d, h->pix, h->n_pix,
                               h->images, h->opt.n_levels, h->opt.precision, h->tiles[bb::synth_k_class(d.K_alloc)],
                               h->ev[2], h->ev[3]);
  if (st != BB_OK) return st;
  h->timed = true;
  h->count += 1;
  return BB_OK;
}

// Fixed scratch of the no-allocation entry point: metadata, error word, staging.
static_assert(BB_NOALLOC_SCRATCH_BYTES == bb::kNoallocScratchBytes, "header and library agree on the scratch size");
static_assert(BB_K_CLASSES == bb::kKClasses, "header and library agree on the K classes");
static_assert(bb_host::kTuneClasses == bb::kKClasses, "the tune cache keys the K classes");
constexpr size_t kNoallocMeta = 0;
constexpr size_t kNoallocErr = (sizeof(SingleMeta) + kAlign - 1) / kAlign * kAlign;
constexpr size_t kNoallocStage = kNoallocErr + kAlign;

// The scratch address of `device`, looked up once per device with that device
// current (each device holds its own copy of the array).
bb_status noalloc_lookup(bb_context ctx, int device, void** out) {
  static std::mutex mu;
  static void* addr[64] = {};
  if (device < 0 || device >= 64) return fail(ctx, BB_ERR_DEVICE, "device %d beyond the scratch table", device);
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    hipError_t e = bb::noalloc_scratch_address(&p);
    if (e != hipSuccess || !p)
      return fail(ctx, BB_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    addr[device] = p;
  }
  *out = addr[device];
  return BB_OK;
}

}  // namespace

extern "C" {

const char* bb_status_string(bb_status s) {
  switch (s) {
    case BB_OK: return "BB_OK";
    case BB_ERR_INVALID_ARG: return "BB_ERR_INVALID_ARG";
    case BB_ERR_SHAPE: return "BB_ERR_SHAPE";
    case BB_ERR_NOT_POSDEF: return "BB_ERR_NOT_POSDEF";
    case BB_ERR_EIGEN: return "BB_ERR_EIGEN";
    case BB_ERR_WORKSPACE: return "BB_ERR_WORKSPACE";
    case BB_ERR_DEVICE: return "BB_ERR_DEVICE";
    case BB_ERR_STATE: return "BB_ERR_STATE";
  }
  return "BB_ERR_UNKNOWN";
}

bb_status bb_context_create(int device, void* hip_stream, bb_context* out) {
  if (!out) return BB_ERR_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return BB_ERR_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return BB_ERR_DEVICE;
  bb_context c = new (std::nothrow) bb_context_;
  if (!c) return BB_ERR_DEVICE;
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (rocblas_create_handle(&c->rb) != rocblas_status_success) {
    delete c;
    return BB_ERR_DEVICE;
  }
  rocblas_set_stream(c->rb, c->stream);
  hipDeviceProp_t prop{};
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    c->arch = prop.gcnArchName;
    const size_t colon = c->arch.find(':');
    if (colon != std::string::npos) c->arch.resize(colon);
  }
  bb_status st = noalloc_lookup(c, device, &c->noalloc_scratch);
  if (st != BB_OK) {
    rocblas_destroy_handle(c->rb);
    delete c;
    return st;
  }
  *out = c;
  return BB_OK;
}

bb_status bb_context_set_stream(bb_context ctx, void* hip_stream) {
  if (!ctx) return BB_ERR_INVALID_ARG;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  rocblas_set_stream(ctx->rb, ctx->stream);
  return BB_OK;
}

bb_status bb_context_destroy(bb_context ctx) {
  if (!ctx) return BB_ERR_INVALID_ARG;
  if (ctx->live > 0) return fail(ctx, BB_ERR_STATE, "%d synthesis handle(s) still alive", ctx->live);
  rocblas_destroy_handle(ctx->rb);
  delete ctx;
  return BB_OK;
}

const char* bb_last_error(bb_context ctx) { return ctx ? ctx->err.c_str() : "null context"; }

bb_status bb_workspace_size(bb_context ctx, const bb_options* opt, int64_t n_pix, size_t* bytes) {
  if (!ctx || !bytes) return BB_ERR_INVALID_ARG;
  bb_status st = check_options(ctx, opt);
  if (st != BB_OK) return st;
  if (n_pix < 1) return fail(ctx, BB_ERR_INVALID_ARG, "n_pix must be >= 1");
  if (hipSetDevice(ctx->device) != hipSuccess) return BB_ERR_DEVICE;
  *bytes = make_layout(*opt, solver_query(ctx, opt->n_ant_max)).total;
  return BB_OK;
}

bb_status bb_synth_create(bb_context ctx, const bb_options* opt, int64_t n_pix, const double* pix_xyz,
                          float* images, void* workspace, size_t ws_bytes, bb_synth* out) {
  if (!ctx || !out) return BB_ERR_INVALID_ARG;
  *out = nullptr;
  bb_status st = check_options(ctx, opt);
  if (st != BB_OK) return st;
  if (n_pix < 1) return fail(ctx, BB_ERR_INVALID_ARG, "n_pix must be >= 1");
  if (!pix_xyz || !images || !workspace) return fail(ctx, BB_ERR_INVALID_ARG, "null device pointer");
  if (hipSetDevice(ctx->device) != hipSuccess) return BB_ERR_DEVICE;
  const Layout lay = make_layout(*opt, solver_query(ctx, opt->n_ant_max));
  if (ws_bytes < lay.total)
    return fail(ctx, BB_ERR_WORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, lay.total);
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return fail(ctx, BB_ERR_INVALID_ARG, "workspace must be %zu-byte aligned", kAlign);
  bb_synth h = new (std::nothrow) bb_synth_;
  if (!h) return BB_ERR_DEVICE;
  h->ctx = ctx;
  h->opt = *opt;
  h->n_pix = n_pix;
  h->pix = pix_xyz;
  h->images = images;
  h->ws = static_cast<char*>(workspace);
  h->ws_bytes = ws_bytes;
  h->lay = lay;
  int cached[bb::kKClasses];
  bb_host::tune_cache_lookup(ctx->arch, opt->precision, n_pix, cached);
  for (int c = 0; c < bb::kKClasses; ++c)
    h->tiles[c] = (cached[c] >= 0 && bb::synth_tile_allowed(opt->precision, cached[c], c))
                      ? cached[c]
                      : bb::synth_default_tile(opt->precision, c);
  for (auto& e : h->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      delete h;
      return fail(ctx, BB_ERR_DEVICE, "hipEventCreate failed");
    }
  if (bb_host::debug_fill() && bb::launch_fill_poison(h->ws, lay.total, ctx->stream) != hipSuccess) {
    for (auto& e : h->ev) (void)hipEventDestroy(e);
    delete h;
    return fail(ctx, BB_ERR_DEVICE, "launch failed");
  }
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, ctx->stream, at<int>(h, h->lay.err));
  if (hipGetLastError() != hipSuccess) {
    for (auto& e : h->ev) (void)hipEventDestroy(e);
    delete h;
    return fail(ctx, BB_ERR_DEVICE, "launch failed");
  }
  ctx->live += 1;
  *out = h;
  return BB_OK;
}

bb_status bb_synth_destroy(bb_synth h) {
  if (!h) return BB_ERR_INVALID_ARG;
  (void)hipStreamSynchronize(h->ctx->stream);
  for (auto& e : h->ev) (void)hipEventDestroy(e);
  h->ctx->live -= 1;
  delete h;
  return BB_OK;
}

static bb_status check_instance_args(bb_synth h, int32_t slot, int32_t n_ant, int32_t n_eig, double wl) {
  bb_context ctx = h->ctx;
  if (slot < 0 || slot >= h->opt.n_slots) return fail(ctx, BB_ERR_INVALID_ARG, "slot %d out of range", slot);
  if (n_ant < 1) return fail(ctx, BB_ERR_INVALID_ARG, "n_ant must be >= 1");
  if (n_ant > h->opt.n_ant_max) return fail(ctx, BB_ERR_SHAPE, "n_ant %d > n_ant_max %d", n_ant, h->opt.n_ant_max);
  if (n_eig < 1) return fail(ctx, BB_ERR_INVALID_ARG, "n_eig must be >= 1");
  if (n_eig > h->opt.k_max) return fail(ctx, BB_ERR_SHAPE, "n_eig %d > k_max %d", n_eig, h->opt.k_max);
  if (!finite_pos(wl)) return fail(ctx, BB_ERR_INVALID_ARG, "wavelength must be finite and > 0");
  return BB_OK;
}

bb_status bb_synth_collect_eig(bb_synth h, int32_t slot, int32_t n_ant, int32_t n_eig, double wavelength_m,
                               const double* ant_xyz, const void* W, const float* d, const int32_t* level_of) {
  if (!h) return BB_ERR_INVALID_ARG;
  bb_context ctx = h->ctx;
  bb_status st = check_instance_args(h, slot, n_ant, n_eig, wavelength_m);
  if (st != BB_OK) return st;
  if (!ant_xyz || !W || !d || !level_of) return fail(ctx, BB_ERR_INVALID_ARG, "null device pointer");
  BB_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  BB_HIP(ctx, hipEventRecord(h->ev[0], s));
  BB_HIP(ctx, hipEventRecord(h->ev[1], s));
  InstDesc dsc = staging_desc(h, h->ws + h->lay.apack, n_ant, n_eig, wavelength_m, slot);
  dsc.ant = ant_xyz;
  dsc.ant_ld = n_ant;
  dsc.W = W;
  dsc.W_ld = n_ant;
  dsc.W_c128 = 0;
  dsc.wcol = nullptr;
  dsc.d = d;
  dsc.lev_in = level_of;
  return run_single(h, dsc);
}

bb_status bb_synth_collect_eig_noalloc(bb_context ctx, int32_t precision, int32_t n_levels, int64_t n_pix,
                                       const double* pix_xyz, float* images, int32_t n_ant, int32_t n_eig,
                                       double wavelength_m, const double* ant_xyz, const void* W, const float* d,
                                       const int32_t* level_of) {
  if (!ctx) return BB_ERR_INVALID_ARG;
  if (precision < BB_PREC_FP32 || precision > BB_PREC_BF16X3_3M)
    return fail(ctx, BB_ERR_INVALID_ARG, "unknown precision %d", precision);
  if (n_levels < 1 || n_levels > bb::kMaxLevels)
    return fail(ctx, BB_ERR_INVALID_ARG, "n_levels must be in [1, %d]", bb::kMaxLevels);
  if (n_pix < 1) return fail(ctx, BB_ERR_INVALID_ARG, "n_pix must be >= 1");
  if (n_ant < 1 || n_ant > bb::kMaxAnt) return fail(ctx, BB_ERR_SHAPE, "n_ant must be in [1, %d]", bb::kMaxAnt);
  if (n_eig < 1 || n_eig > bb::kMaxEig) return fail(ctx, BB_ERR_SHAPE, "n_eig must be in [1, %d]", bb::kMaxEig);
  if (!finite_pos(wavelength_m)) return fail(ctx, BB_ERR_INVALID_ARG, "wavelength must be finite and > 0");
  if (!pix_xyz || !images || !ant_xyz || !W || !d || !level_of)
    return fail(ctx, BB_ERR_INVALID_ARG, "null device pointer");
  if (!ctx->noalloc_scratch) return fail(ctx, BB_ERR_STATE, "context has no scratch address");
  const int L_pad = bb::round_up(n_ant, bb::kAntChunk), K_alloc = bb::round_up(n_eig, 32);
  const size_t need = kNoallocStage + staging_bytes(L_pad, K_alloc);
  if (need > bb::kNoallocScratchBytes)
    return fail(ctx, BB_ERR_WORKSPACE, "n_ant %d x n_eig %d needs %zu bytes of scratch, more than the fixed %zu",
                n_ant, n_eig, need, bb::kNoallocScratchBytes);
  BB_HIP(ctx, hipSetDevice(ctx->device));
  char* base = static_cast<char*>(ctx->noalloc_scratch);
  int* err = reinterpret_cast<int*>(base + kNoallocErr);
  // the error word keeps the previous call's bits: clear it (a kernel, not a memset node)
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, ctx->stream, err);
  BB_HIP(ctx, hipGetLastError());
  InstDesc dsc = staging_desc(nullptr, base + kNoallocStage, n_ant, n_eig, wavelength_m, 0);
  dsc.ant = ant_xyz;
  dsc.ant_ld = n_ant;
  dsc.W = W;
  dsc.W_ld = n_ant;
  dsc.W_c128 = 0;
  dsc.wcol = nullptr;
  dsc.d = d;
  dsc.lev_in = level_of;
  return launch_single(ctx, reinterpret_cast<SingleMeta*>(base + kNoallocMeta), err, dsc, pix_xyz, n_pix, images,
                       n_levels, precision, bb::synth_default_tile(precision, bb::synth_k_class(dsc.K_alloc)), nullptr,
                       nullptr);
}

// Host intervals (n_levels x 2, column-major [min, max]) into the kernels' form.
// Intervals may touch (k-means bounds are shared); a positive-length overlap
// is rejected.  A value on a shared bound goes to the first such level.
static bb_status parse_intervals(bb_context ctx, const double* intervals, int nl, bb::Intervals& iv) {
  for (int l = 0; l < nl; ++l) {
    iv.lo[l] = intervals[l];
    iv.hi[l] = intervals[l + nl];
    if (std::isnan(iv.lo[l]) || std::isnan(iv.hi[l]) || iv.lo[l] > iv.hi[l])
      return fail(ctx, BB_ERR_INVALID_ARG, "interval %d is not [min <= max]", l);
  }
  for (int a = 0; a < nl; ++a)
    for (int b = a + 1; b < nl; ++b)
      if (std::max(iv.lo[a], iv.lo[b]) < std::min(iv.hi[a], iv.hi[b]))
        return fail(ctx, BB_ERR_INVALID_ARG, "intervals %d and %d overlap", a, b);
  return BB_OK;
}

// FP64 pre-step shared by bb_synth_collect and bb_synth_prestep: Gram,
// generalized eigensolve, selection; leaves weights / level ids / column map
// in the workspace.  Waits for the eigensolver status.
// With energy_fraction > 0, n_eig is chosen from the eigenvalues (fewest
// leading eigenpairs reaching that fraction of the positive eigenvalues' sum,
// at most k_max) and returned through n_eig_used.
// With a beamforming matrix W_bf (n_ant x n_beam), the eigenproblem is the
// beamformed one (V^W, W_bf^H G W_bf) of size n_beam and the eigenvectors
// are mapped back to antennas, U = W_bf alpha (left in the U region).
static bb_status run_prestep(bb_synth h, int32_t n_ant, double wavelength_m, const double* ant_xyz,
                             const double* vis, int32_t n_eig, const double* intervals,
                             double energy_fraction = 0.0, int32_t* n_eig_used = nullptr,
                             const double* W_bf = nullptr, int32_t n_beam = 0) {
  bb_context ctx = h->ctx;
  const int n_sys = W_bf ? n_beam : n_ant;  // size of the eigenproblem
  if (energy_fraction <= 0.0 && n_eig > n_ant) return fail(ctx, BB_ERR_INVALID_ARG, "n_eig %d > n_ant %d", n_eig, n_ant);
  if (!ant_xyz || !vis || !intervals) return fail(ctx, BB_ERR_INVALID_ARG, "null pointer");
  const int nl = h->opt.n_levels;
  bb::Intervals iv{};
  bb_status ist = parse_intervals(ctx, intervals, nl, iv);
  if (ist != BB_OK) return ist;
  BB_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const Layout& L = h->lay;
  double* A = at<double>(h, L.A);
  double* G = at<double>(h, L.G);
  BB_HIP(ctx, hipEventRecord(h->ev[0], s));
  BB_HIP(ctx, bb::launch_gram(ant_xyz, n_ant, n_ant, wavelength_m, G, n_ant, h->opt.gram == BB_GRAM_IDENTITY, s));
  BB_HIP(ctx, bb::launch_copy_c128(vis, n_sys, A, n_sys, s));
  double* herm = reinterpret_cast<double*>(h->ws + L.info + 16);  // two doubles beside the solver status
  BB_HIP(ctx, bb::launch_herm_check(vis, n_sys, herm, s));
  rocblas_set_stream(ctx->rb, s);
  if (L.solver_bytes > 0 && rocblas_set_workspace(ctx->rb, h->ws + L.solver, L.solver_bytes) != rocblas_status_success)
    return fail(ctx, BB_ERR_DEVICE, "rocblas_set_workspace failed");
  using cplx = rocblas_double_complex;
  const cplx one = {1.0, 0.0}, zero = {0.0, 0.0};
  cplx* Gc = reinterpret_cast<cplx*>(G);
  if (W_bf) {
    // G^W = W_bf^H (G W_bf), written over G's leading n_beam x n_beam block (ld n_beam)
    cplx* T = at<cplx>(h, L.T);
    const cplx* Wb = reinterpret_cast<const cplx*>(W_bf);
    rocblas_status gs = rocblas_zgemm(ctx->rb, rocblas_operation_none, rocblas_operation_none, n_ant, n_beam, n_ant,
                                      &one, Gc, n_ant, Wb, n_ant, &zero, T, n_ant);
    if (gs == rocblas_status_success)
      gs = rocblas_zgemm(ctx->rb, rocblas_operation_conjugate_transpose, rocblas_operation_none, n_beam, n_beam, n_ant,
                         &one, Wb, n_ant, T, n_ant, &zero, Gc, n_beam);
    if (gs != rocblas_status_success) {
      if (L.solver_bytes > 0) rocblas_set_workspace(ctx->rb, nullptr, 0);
      return fail(ctx, BB_ERR_DEVICE, "rocblas_zgemm status %d", (int)gs);
    }
  }
  rocblas_status rs = rocsolver_zhegvd(ctx->rb, rocblas_eform_ax, rocblas_evect_original, rocblas_fill_lower, n_sys,
                                       reinterpret_cast<cplx*>(A), n_sys, Gc, n_sys, at<double>(h, L.evals),
                                       at<double>(h, L.E), at<rocblas_int>(h, L.info));
  if (rs == rocblas_status_success && W_bf)
    rs = rocblas_zgemm(ctx->rb, rocblas_operation_none, rocblas_operation_none, n_ant, n_beam, n_beam, &one,
                       reinterpret_cast<const cplx*>(W_bf), n_ant, reinterpret_cast<cplx*>(A), n_beam, &zero,
                       at<cplx>(h, L.U), n_ant);
  if (L.solver_bytes > 0) rocblas_set_workspace(ctx->rb, nullptr, 0);
  if (rs == rocblas_status_memory_error) return fail(ctx, BB_ERR_WORKSPACE, "rocSOLVER workspace too small");
  if (rs != rocblas_status_success) return fail(ctx, BB_ERR_DEVICE, "rocsolver_zhegvd / zgemm status %d", (int)rs);
  BB_HIP(ctx, hipEventRecord(h->ev[1], s));
  rocblas_int info = 0;
  double herm_host[2] = {0.0, 0.0};
  std::vector<double> ev;
  BB_HIP(ctx, hipMemcpyAsync(&info, at<rocblas_int>(h, L.info), sizeof info, hipMemcpyDeviceToHost, s));
  BB_HIP(ctx, hipMemcpyAsync(herm_host, herm, sizeof herm_host, hipMemcpyDeviceToHost, s));
  if (energy_fraction > 0.0) {
    ev.resize(n_sys);
    BB_HIP(ctx, hipMemcpyAsync(ev.data(), at<double>(h, L.evals), sizeof(double) * n_sys, hipMemcpyDeviceToHost, s));
  }
  BB_HIP(ctx, hipStreamSynchronize(s));
  // ||V - V^H||_F <= 1e-12 ||V||_F, squared; NaN fails too
  if (!(herm_host[0] <= 1e-24 * herm_host[1]))
    return fail(ctx, BB_ERR_INVALID_ARG, "visibility matrix is not Hermitian (||V - V^H|| / ||V|| = %.3g)",
                std::sqrt(herm_host[0] / herm_host[1]));
  if (info > n_sys) return fail(ctx, BB_ERR_NOT_POSDEF, "Gram matrix not positive definite (leading minor %d)", info - n_sys);
  if (info != 0) return fail(ctx, BB_ERR_EIGEN, "eigensolver did not converge (info %d)", info);
  if (energy_fraction > 0.0) {
    // eigenvalues ascending: walk from the largest (Section 2.6 truncation by energy)
    double total = 0.0;
    for (double v : ev)
      if (v > 0.0) total += v;
    int k = 1;
    if (total > 0.0) {
      double acc = 0.0;
      int npos = 0;
      for (double v : ev) npos += v > 0.0;
      k = npos;
      for (int i = 0; i < n_sys; ++i) {
        acc += ev[n_sys - 1 - i];
        if (acc >= energy_fraction * total) {
          k = i + 1;
          break;
        }
      }
    }
    n_eig = std::min(std::min(k, h->opt.k_max), n_sys);
    if (n_eig_used) *n_eig_used = n_eig;
  }
  BB_HIP(ctx, bb::launch_select(at<double>(h, L.evals), n_sys, n_eig, iv, nl, h->opt.filter, at<float>(h, L.dsel),
                                at<int>(h, L.lsel), at<int>(h, L.wcol), s));
  return BB_OK;
}

bb_status bb_synth_collect(bb_synth h, int32_t slot, int32_t n_ant, double wavelength_m, const double* ant_xyz,
                           const double* vis, int32_t n_eig, const double* intervals) {
  if (!h) return BB_ERR_INVALID_ARG;
  bb_status st = check_instance_args(h, slot, n_ant, n_eig, wavelength_m);
  if (st != BB_OK) return st;
  st = run_prestep(h, n_ant, wavelength_m, ant_xyz, vis, n_eig, intervals);
  if (st != BB_OK) return st;
  const Layout& L = h->lay;
  InstDesc dsc = staging_desc(h, h->ws + L.apack, n_ant, n_eig, wavelength_m, slot);
  dsc.ant = ant_xyz;
  dsc.ant_ld = n_ant;
  dsc.W = at<double>(h, L.A);
  dsc.W_ld = n_ant;
  dsc.W_c128 = 1;
  dsc.wcol = at<int>(h, L.wcol);
  dsc.d = at<float>(h, L.dsel);
  dsc.lev_in = at<int>(h, L.lsel);
  return run_single(h, dsc);
}

bb_status bb_synth_collect_energy(bb_synth h, int32_t slot, int32_t n_ant, double wavelength_m,
                                  const double* ant_xyz, const double* vis, double energy_fraction,
                                  const double* intervals, int32_t* n_eig_out) {
  if (!h) return BB_ERR_INVALID_ARG;
  bb_context ctx = h->ctx;
  bb_status st = check_instance_args(h, slot, n_ant, 1, wavelength_m);
  if (st != BB_OK) return st;
  if (!(energy_fraction > 0.0 && energy_fraction <= 1.0))
    return fail(ctx, BB_ERR_INVALID_ARG, "energy_fraction must be in (0, 1]");
  if (!n_eig_out) return fail(ctx, BB_ERR_INVALID_ARG, "n_eig_out is NULL");
  int32_t k = 0;
  st = run_prestep(h, n_ant, wavelength_m, ant_xyz, vis, 0, intervals, energy_fraction, &k);
  if (st != BB_OK) return st;
  *n_eig_out = k;
  const Layout& L = h->lay;
  InstDesc dsc = staging_desc(h, h->ws + L.apack, n_ant, k, wavelength_m, slot);
  dsc.ant = ant_xyz;
  dsc.ant_ld = n_ant;
  dsc.W = at<double>(h, L.A);
  dsc.W_ld = n_ant;
  dsc.W_c128 = 1;
  dsc.wcol = at<int>(h, L.wcol);
  dsc.d = at<float>(h, L.dsel);
  dsc.lev_in = at<int>(h, L.lsel);
  return run_single(h, dsc);
}

bb_status bb_synth_collect_beamformed(bb_synth h, int32_t slot, int32_t n_ant, int32_t n_beam,
                                      double wavelength_m, const double* ant_xyz, const double* W_bf,
                                      const double* vis_bf, int32_t n_eig, const double* intervals) {
  if (!h) return BB_ERR_INVALID_ARG;
  bb_context ctx = h->ctx;
  bb_status st = check_instance_args(h, slot, n_ant, n_eig, wavelength_m);
  if (st != BB_OK) return st;
  if (n_beam < 1 || n_beam > n_ant) return fail(ctx, BB_ERR_INVALID_ARG, "n_beam must be in [1, n_ant]");
  if (n_eig > n_beam) return fail(ctx, BB_ERR_INVALID_ARG, "n_eig %d > n_beam %d", n_eig, n_beam);
  if (!W_bf) return fail(ctx, BB_ERR_INVALID_ARG, "W_bf is NULL");
  st = run_prestep(h, n_ant, wavelength_m, ant_xyz, vis_bf, n_eig, intervals, 0.0, nullptr, W_bf, n_beam);
  if (st != BB_OK) return st;
  const Layout& L = h->lay;
  InstDesc dsc = staging_desc(h, h->ws + L.apack, n_ant, n_eig, wavelength_m, slot);
  dsc.ant = ant_xyz;
  dsc.ant_ld = n_ant;
  dsc.W = at<double>(h, L.U);  // U = W_bf alpha, n_ant x n_beam
  dsc.W_ld = n_ant;
  dsc.W_c128 = 1;
  dsc.wcol = at<int>(h, L.wcol);
  dsc.d = at<float>(h, L.dsel);
  dsc.lev_in = at<int>(h, L.lsel);
  return run_single(h, dsc);
}

bb_status bb_synth_prestep(bb_synth h, int32_t n_ant, double wavelength_m, const double* ant_xyz,
                           const double* vis, int32_t n_eig, const double* intervals, void* W_out,
                           double* lam_out, float* d_out, int32_t* level_out) {
  if (!h) return BB_ERR_INVALID_ARG;
  bb_context ctx = h->ctx;
  bb_status st = check_instance_args(h, 0, n_ant, n_eig, wavelength_m);
  if (st != BB_OK) return st;
  if (!W_out || !lam_out || !d_out || !level_out) return fail(ctx, BB_ERR_INVALID_ARG, "null output pointer");
  st = run_prestep(h, n_ant, wavelength_m, ant_xyz, vis, n_eig, intervals);
  if (st != BB_OK) return st;
  const Layout& L = h->lay;
  BB_HIP(ctx, bb::launch_export_eig(at<double>(h, L.A), at<double>(h, L.evals), n_ant, n_eig, at<int>(h, L.wcol),
                                    at<float>(h, L.dsel), at<int>(h, L.lsel), static_cast<float*>(W_out), lam_out,
                                    d_out, level_out, ctx->stream));
  BB_HIP(ctx, hipEventRecord(h->ev[2], ctx->stream));
  BB_HIP(ctx, hipEventRecord(h->ev[3], ctx->stream));
  h->timed = true;
  return BB_OK;
}

// ---- batched pre-step ---------------------------------------------------------
namespace {

struct PrestepBatchLayout {  // byte offsets into the caller's workspace
  size_t inv_wl, A, G, evals, E, info, herm, dsel, lsel, wcol, solver, solver_bytes, total;
};

size_t solver_query_batched(bb_context ctx, int n, int n_inst) {
  size_t sz = 0;
  if (rocblas_start_device_memory_size_query(ctx->rb) != rocblas_status_success) return 0;
  rocsolver_zhegvd_strided_batched(ctx->rb, rocblas_eform_ax, rocblas_evect_original, rocblas_fill_lower, n, nullptr,
                                   n, (rocblas_stride)n * n, nullptr, n, (rocblas_stride)n * n, nullptr, n, nullptr,
                                   n, nullptr, n_inst);
  if (rocblas_stop_device_memory_size_query(ctx->rb, &sz) != rocblas_status_success) return 0;
  return sz;
}

PrestepBatchLayout prestep_batch_layout(int n_inst, int L, int K, size_t solver_bytes) {
  PrestepBatchLayout b{};
  const size_t n = (size_t)n_inst, Lm = (size_t)L;
  size_t p = 0;
  b.inv_wl = p;
  p += align_up(8 * n);
  b.A = p;
  p += align_up(16 * Lm * Lm * n);
  b.G = p;
  p += align_up(16 * Lm * Lm * n);
  b.evals = p;
  p += align_up(8 * Lm * n);
  b.E = p;
  p += align_up(8 * Lm * n);
  b.info = p;
  p += align_up(4 * n);
  b.herm = p;
  p += align_up(16 * n);
  b.dsel = p;
  p += align_up(4 * (size_t)K * n);
  b.lsel = p;
  p += align_up(4 * (size_t)K * n);
  b.wcol = p;
  p += align_up(4 * (size_t)K * n);
  b.solver = p;
  b.solver_bytes = solver_bytes;
  p += align_up(solver_bytes);
  b.total = p;
  return b;
}

bb_status check_prestep_batch(bb_synth h, int32_t n_inst, int32_t n_ant, int32_t n_eig) {
  bb_context ctx = h->ctx;
  if (n_inst < 1) return fail(ctx, BB_ERR_INVALID_ARG, "n_inst must be >= 1");
  if (n_ant < 1) return fail(ctx, BB_ERR_INVALID_ARG, "n_ant must be >= 1");
  if (n_ant > h->opt.n_ant_max) return fail(ctx, BB_ERR_SHAPE, "n_ant %d > n_ant_max %d", n_ant, h->opt.n_ant_max);
  if (n_eig < 1 || n_eig > n_ant) return fail(ctx, BB_ERR_INVALID_ARG, "n_eig must be in [1, n_ant]");
  if (n_eig > h->opt.k_max) return fail(ctx, BB_ERR_SHAPE, "n_eig %d > k_max %d", n_eig, h->opt.k_max);
  return BB_OK;
}

}  // namespace

bb_status bb_prestep_batched_workspace_size(bb_synth h, int32_t n_inst, int32_t n_ant, int32_t n_eig,
                                            size_t* bytes) {
  if (!h || !bytes) return BB_ERR_INVALID_ARG;
  bb_status st = check_prestep_batch(h, n_inst, n_ant, n_eig);
  if (st != BB_OK) return st;
  if (hipSetDevice(h->ctx->device) != hipSuccess) return BB_ERR_DEVICE;
  *bytes = prestep_batch_layout(n_inst, n_ant, n_eig, solver_query_batched(h->ctx, n_ant, n_inst)).total;
  return BB_OK;
}

bb_status bb_synth_prestep_batched(bb_synth h, int32_t n_inst, int32_t n_ant, int32_t n_eig,
                                   const double* wavelengths_m, const double* ant_xyz_packed, const double* vis_packed,
                                   const double* intervals, void* W_out, double* lam_out, float* d_out,
                                   int32_t* level_out, void* workspace, size_t ws_bytes) {
  if (!h) return BB_ERR_INVALID_ARG;
  bb_context ctx = h->ctx;
  bb_status st = check_prestep_batch(h, n_inst, n_ant, n_eig);
  if (st != BB_OK) return st;
  if (!wavelengths_m || !intervals) return fail(ctx, BB_ERR_INVALID_ARG, "null host pointer");
  if (!ant_xyz_packed || !vis_packed || !W_out || !lam_out || !d_out || !level_out || !workspace)
    return fail(ctx, BB_ERR_INVALID_ARG, "null device pointer");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return fail(ctx, BB_ERR_INVALID_ARG, "workspace must be %zu-byte aligned", kAlign);
  std::vector<double> inv_wl(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    if (!finite_pos(wavelengths_m[i]))
      return fail(ctx, BB_ERR_INVALID_ARG, "instance %d: wavelength must be finite and > 0", i);
    inv_wl[i] = 1.0 / wavelengths_m[i];
  }
  const int nl = h->opt.n_levels;
  bb::Intervals iv{};
  st = parse_intervals(ctx, intervals, nl, iv);
  if (st != BB_OK) return st;
  BB_HIP(ctx, hipSetDevice(ctx->device));
  const PrestepBatchLayout B = prestep_batch_layout(n_inst, n_ant, n_eig, solver_query_batched(ctx, n_ant, n_inst));
  if (ws_bytes < B.total) return fail(ctx, BB_ERR_WORKSPACE, "workspace %zu < required %zu", ws_bytes, B.total);
  char* ws = static_cast<char*>(workspace);
  hipStream_t s = ctx->stream;
  if (bb_host::debug_fill()) BB_HIP(ctx, bb::launch_fill_poison(ws, B.total, s));
  BB_HIP(ctx, hipEventRecord(h->ev[0], s));
  // pageable source: the copy is staged before the call returns
  BB_HIP(ctx, hipMemcpyAsync(ws + B.inv_wl, inv_wl.data(), sizeof(double) * n_inst, hipMemcpyHostToDevice, s));
  double* A = reinterpret_cast<double*>(ws + B.A);
  double* G = reinterpret_cast<double*>(ws + B.G);
  double* herm = reinterpret_cast<double*>(ws + B.herm);
  BB_HIP(ctx, bb::launch_prestep_inputs_batched(ant_xyz_packed, (int64_t)n_inst * n_ant, n_ant,
                                                reinterpret_cast<const double*>(ws + B.inv_wl), n_inst,
                                                h->opt.gram == BB_GRAM_IDENTITY, vis_packed, A, G, herm, s));
  rocblas_set_stream(ctx->rb, s);
  if (B.solver_bytes > 0 && rocblas_set_workspace(ctx->rb, ws + B.solver, B.solver_bytes) != rocblas_status_success)
    return fail(ctx, BB_ERR_DEVICE, "rocblas_set_workspace failed");
  using cplx = rocblas_double_complex;
  const rocblas_stride mstride = (rocblas_stride)n_ant * n_ant;
  rocblas_status rs = rocsolver_zhegvd_strided_batched(
      ctx->rb, rocblas_eform_ax, rocblas_evect_original, rocblas_fill_lower, n_ant, reinterpret_cast<cplx*>(A), n_ant,
      mstride, reinterpret_cast<cplx*>(G), n_ant, mstride, reinterpret_cast<double*>(ws + B.evals), n_ant,
      reinterpret_cast<double*>(ws + B.E), n_ant, reinterpret_cast<rocblas_int*>(ws + B.info), n_inst);
  if (B.solver_bytes > 0) rocblas_set_workspace(ctx->rb, nullptr, 0);
  if (rs == rocblas_status_memory_error) return fail(ctx, BB_ERR_WORKSPACE, "rocSOLVER workspace too small");
  if (rs != rocblas_status_success) return fail(ctx, BB_ERR_DEVICE, "rocsolver_zhegvd_strided_batched status %d", (int)rs);
  BB_HIP(ctx, hipEventRecord(h->ev[1], s));
  // one wait per call: every instance's solver status and Hermiticity sums
  std::vector<rocblas_int> info(n_inst);
  std::vector<double> hs(2 * (size_t)n_inst);
  BB_HIP(ctx, hipMemcpyAsync(info.data(), ws + B.info, sizeof(rocblas_int) * n_inst, hipMemcpyDeviceToHost, s));
  BB_HIP(ctx, hipMemcpyAsync(hs.data(), herm, sizeof(double) * 2 * n_inst, hipMemcpyDeviceToHost, s));
  BB_HIP(ctx, hipStreamSynchronize(s));
  for (int i = 0; i < n_inst; ++i) {
    if (!(hs[2 * i] <= 1e-24 * hs[2 * i + 1]))
      return fail(ctx, BB_ERR_INVALID_ARG, "instance %d: visibility matrix is not Hermitian (||V - V^H|| / ||V|| = %.3g)",
                  i, std::sqrt(hs[2 * i] / hs[2 * i + 1]));
    if (info[i] > n_ant)
      return fail(ctx, BB_ERR_NOT_POSDEF, "instance %d: Gram matrix not positive definite (leading minor %d)", i,
                  info[i] - n_ant);
    if (info[i] != 0) return fail(ctx, BB_ERR_EIGEN, "instance %d: eigensolver did not converge (info %d)", i, info[i]);
  }
  BB_HIP(ctx, bb::launch_select_export_batched(A, reinterpret_cast<double*>(ws + B.evals), n_ant, n_eig, n_inst, iv,
                                               nl, h->opt.filter, reinterpret_cast<float*>(ws + B.dsel),
                                               reinterpret_cast<int*>(ws + B.lsel), reinterpret_cast<int*>(ws + B.wcol),
                                               static_cast<float*>(W_out), lam_out, d_out, level_out, s));
  BB_HIP(ctx, hipEventRecord(h->ev[2], s));
  BB_HIP(ctx, hipEventRecord(h->ev[3], s));
  h->timed = true;
  return BB_OK;
}

// ---- level determination and weighting ---------------------------------------
bb_status bb_synth_levels_kmeans(bb_synth h, int32_t n, const double* lam, int32_t negative_level,
                                 double* intervals, int32_t* level_of) {
  if (!h) return BB_ERR_INVALID_ARG;
  bb_context ctx = h->ctx;
  if (n < 1 || n > bb::kMaxEig) return fail(ctx, BB_ERR_SHAPE, "n %d outside [1, %d]", n, bb::kMaxEig);
  if (negative_level != 0 && negative_level != 1) return fail(ctx, BB_ERR_INVALID_ARG, "negative_level must be 0 or 1");
  const int k = h->opt.n_levels - negative_level;
  if (k < 1) return fail(ctx, BB_ERR_INVALID_ARG, "no positive level left (n_levels %d)", h->opt.n_levels);
  if (!lam || !intervals || !level_of) return fail(ctx, BB_ERR_INVALID_ARG, "null device pointer");
  BB_HIP(ctx, hipSetDevice(ctx->device));
  BB_HIP(ctx, bb::launch_kmeans_levels(lam, n, k, negative_level, intervals, level_of, at<int>(h, h->lay.err),
                                       ctx->stream));
  return BB_OK;
}

bb_status bb_synth_uniform_weighting(bb_synth h, int32_t n_ant, double wavelength_m, const double* ant_xyz,
                                     const double* e_u, const double* e_v, double fov_rad, double* vis) {
  if (!h) return BB_ERR_INVALID_ARG;
  bb_context ctx = h->ctx;
  if (n_ant < 1) return fail(ctx, BB_ERR_INVALID_ARG, "n_ant must be >= 1");
  if (n_ant > h->opt.n_ant_max) return fail(ctx, BB_ERR_SHAPE, "n_ant %d > n_ant_max %d", n_ant, h->opt.n_ant_max);
  if (!finite_pos(wavelength_m)) return fail(ctx, BB_ERR_INVALID_ARG, "wavelength must be finite and > 0");
  if (!finite_pos(fov_rad)) return fail(ctx, BB_ERR_INVALID_ARG, "fov must be finite and > 0");
  if (!ant_xyz || !vis) return fail(ctx, BB_ERR_INVALID_ARG, "null device pointer");
  if (!e_u || !e_v) return fail(ctx, BB_ERR_INVALID_ARG, "null uv axis");
  bb::UvFrame f{};
  for (int i = 0; i < 3; ++i) {
    if (!std::isfinite(e_u[i]) || !std::isfinite(e_v[i])) return fail(ctx, BB_ERR_INVALID_ARG, "uv axes must be finite");
    f.eu[i] = e_u[i];
    f.ev[i] = e_v[i];
  }
  f.scale = fov_rad / wavelength_m;
  // the hash table lives in the pre-step matrices' region (free between calls)
  const size_t need = (size_t)bb::uv_table_slots(n_ant) * 12;
  if (need > h->lay.evals - h->lay.A) return fail(ctx, BB_ERR_WORKSPACE, "uv table does not fit");
  BB_HIP(ctx, hipSetDevice(ctx->device));
  BB_HIP(ctx, bb::launch_uniform_weighting(ant_xyz, n_ant, n_ant, f, h->ws + h->lay.A, vis, at<int>(h, h->lay.err),
                                           ctx->stream));
  return BB_OK;
}

// ---- batched ----------------------------------------------------------------
namespace {

// Instances are grouped by the tile shape of their K class (the handle's tile
// table: one persistent launch per shape, the costliest shape first); inside a
// shape, by image slot (slots in decreasing cost order).  Launches are
// stream-ordered, each has one writer per image tile: the result is
// deterministic.
struct Bucket {
  int tile = 0, max_K_alloc = 0, n_groups = 0;
  double cost = 0.0;
  size_t gslot_idx = 0, gbegin_idx = 0;
};

struct BatchPlan {
  std::vector<InstDesc> descs;
  std::vector<Bucket> buckets;
  std::vector<int> group_slot, group_begin, inst_list;
  size_t off_descs, off_dyn, off_gslot, off_gbegin, off_ilist, off_stage, total;
  int max_K_alloc = 0, max_L_pad = 0;
};

// n_w_elems / n_eig_elems: lengths of the packed W (complex elements) and of
// the packed weights and level ids; negative skips those two checks (the
// workspace-size query, which sees no arrays).  tiles: tile id per K class;
// only_class >= 0 puts only that class's instances into the groups (the
// workspace layout does not depend on it: group arrays are sized for n_inst).
bb_status plan_batch(bb_synth h, int32_t n_inst, const bb_instance* inst, int64_t n_ant_rows, int64_t n_w_elems,
                     int64_t n_eig_elems, const int* tiles, int only_class, BatchPlan& bp) {
  bb_context ctx = h->ctx;
  if (n_inst < 1 || !inst) return fail(ctx, BB_ERR_INVALID_ARG, "empty instance table");
  std::vector<Bucket> bks;
  std::vector<int> tile_of(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    const bb_instance& b = inst[i];
    bb_status st = check_instance_args(h, b.slot, b.n_ant, b.n_eig, b.wavelength_m);
    if (st != BB_OK) return st;
    if (b.ant_off < 0 || b.w_off < 0 || b.eig_off < 0 || b.ant_off + b.n_ant > n_ant_rows)
      return fail(ctx, BB_ERR_INVALID_ARG, "instance %d: offsets out of range", i);
    if (n_w_elems >= 0 && b.w_off + (int64_t)b.n_ant * b.n_eig > n_w_elems)
      return fail(ctx, BB_ERR_INVALID_ARG, "instance %d: W block [%lld, %lld) beyond the %lld packed elements", i,
                  (long long)b.w_off, (long long)(b.w_off + (int64_t)b.n_ant * b.n_eig), (long long)n_w_elems);
    if (n_eig_elems >= 0 && b.eig_off + b.n_eig > n_eig_elems)
      return fail(ctx, BB_ERR_INVALID_ARG, "instance %d: eigenpairs [%lld, %lld) beyond the %lld packed elements", i,
                  (long long)b.eig_off, (long long)(b.eig_off + b.n_eig), (long long)n_eig_elems);
    const int L_pad = bb::round_up(b.n_ant, bb::kAntChunk), K_alloc = bb::round_up(b.n_eig, 32);
    bp.max_K_alloc = std::max(bp.max_K_alloc, K_alloc);
    bp.max_L_pad = std::max(bp.max_L_pad, L_pad);
    const int kcl = bb::synth_k_class(K_alloc);
    tile_of[i] = (only_class >= 0 && kcl != only_class) ? -1 : tiles[kcl];
    if (tile_of[i] < 0) continue;
    auto it = std::find_if(bks.begin(), bks.end(), [&](const Bucket& x) { return x.tile == tile_of[i]; });
    if (it == bks.end()) {
      bks.push_back(Bucket{});
      it = bks.end() - 1;
      it->tile = tile_of[i];
    }
    it->max_K_alloc = std::max(it->max_K_alloc, K_alloc);
    it->cost += (double)L_pad * K_alloc;
  }
  std::stable_sort(bks.begin(), bks.end(), [](const Bucket& a, const Bucket& b) { return a.cost > b.cost; });
  for (Bucket bk : bks) {
    std::vector<double> cost(h->opt.n_slots, 0.0);
    std::vector<std::vector<int>> by_slot(h->opt.n_slots);
    for (int i = 0; i < n_inst; ++i) {
      if (tile_of[i] != bk.tile) continue;
      const bb_instance& b = inst[i];
      cost[b.slot] += (double)bb::round_up(b.n_ant, bb::kAntChunk) * bb::round_up(b.n_eig, 32);
      by_slot[b.slot].push_back(i);
    }
    std::vector<int> slots;
    for (int sl = 0; sl < h->opt.n_slots; ++sl)
      if (!by_slot[sl].empty()) slots.push_back(sl);
    std::stable_sort(slots.begin(), slots.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    bk.gslot_idx = bp.group_slot.size();
    bk.gbegin_idx = bp.group_begin.size();
    bp.group_begin.push_back((int)bp.inst_list.size());
    for (int sl : slots) {
      bp.group_slot.push_back(sl);
      for (int i : by_slot[sl]) bp.inst_list.push_back(i);
      bp.group_begin.push_back((int)bp.inst_list.size());
    }
    bk.n_groups = (int)slots.size();
    bp.buckets.push_back(bk);
  }
  // group arrays sized for the worst case (one group per instance, one more
  // begin entry per bucket), so that the layout depends on n_inst only
  size_t p = 0;
  bp.off_descs = p;
  p += align_up(sizeof(InstDesc) * n_inst);
  bp.off_dyn = p;
  p += align_up(sizeof(InstDyn) * n_inst);
  bp.off_gslot = p;
  p += align_up(sizeof(int) * n_inst);
  bp.off_gbegin = p;
  p += align_up(sizeof(int) * ((size_t)n_inst + bb::kKClasses));
  bp.off_ilist = p;
  p += align_up(sizeof(int) * n_inst);
  bp.off_stage = p;
  for (int i = 0; i < n_inst; ++i)
    p += staging_bytes(bb::round_up(inst[i].n_ant, bb::kAntChunk), bb::round_up(inst[i].n_eig, 32));
  bp.total = p;
  return BB_OK;
}

// Descriptors of every instance of a planned batch, their staging regions in
// `ws`, each staged in the operand order of its K class's tile in `tiles`.
void batch_descs(bb_synth h, const bb_instance* inst, int32_t n_inst, int64_t n_ant_rows, const double* ant,
                 const void* W, const float* d, const int32_t* lev, char* ws, const int* tiles, BatchPlan& bp) {
  size_t stage = bp.off_stage;
  bp.descs.resize(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    const bb_instance& b = inst[i];
    InstDesc dd = staging_desc(h, ws + stage, b.n_ant, b.n_eig, b.wavelength_m, b.slot);
    stage += staging_bytes(dd.L_pad, dd.K_alloc);
    dd.ant = ant + b.ant_off;
    dd.ant_ld = n_ant_rows;
    dd.W = static_cast<const float*>(W) + 2 * b.w_off;
    dd.W_ld = b.n_ant;
    dd.W_c128 = 0;
    dd.wcol = nullptr;
    dd.d = d + b.eig_off;
    dd.lev_in = lev + b.eig_off;
    dd.rows16 = bb::synth_tile_rows(h->opt.precision, tiles[bb::synth_k_class(dd.K_alloc)]) == 16 ? 1 : 0;
    bp.descs[i] = dd;
  }
}

// Upload the group arrays of a plan and, with `descs`, the instance
// descriptors.  The kept-eigenpair counts between the two regions (written by
// the staging kernel) are left alone, so a plan of already staged instances
// can be swapped in.
bb_status upload_plan(bb_context ctx, const BatchPlan& bp, char* ws, int32_t n_inst, bool descs) {
  std::vector<char> meta(bp.off_stage, 0);
  std::memcpy(meta.data() + bp.off_descs, bp.descs.data(), sizeof(InstDesc) * n_inst);
  std::memcpy(meta.data() + bp.off_gslot, bp.group_slot.data(), sizeof(int) * bp.group_slot.size());
  std::memcpy(meta.data() + bp.off_gbegin, bp.group_begin.data(), sizeof(int) * bp.group_begin.size());
  std::memcpy(meta.data() + bp.off_ilist, bp.inst_list.data(), sizeof(int) * bp.inst_list.size());
  // pageable source: the copies are staged before the call returns
  if (descs)
    BB_HIP(ctx, hipMemcpyAsync(ws + bp.off_descs, meta.data() + bp.off_descs, bp.off_dyn - bp.off_descs,
                               hipMemcpyHostToDevice, ctx->stream));
  BB_HIP(ctx, hipMemcpyAsync(ws + bp.off_gslot, meta.data() + bp.off_gslot, bp.off_stage - bp.off_gslot,
                             hipMemcpyHostToDevice, ctx->stream));
  return BB_OK;
}

// One synthesis launch per bucket of a planned, staged batch into `images`.
bb_status launch_buckets(bb_synth h, const BatchPlan& bp, char* ws, float* images) {
  bb_context ctx = h->ctx;
  for (const Bucket& bk : bp.buckets) {
    bb::FwdParams p{};
    p.pix = h->pix;
    p.pix_ld = h->n_pix;
    p.n_pix = h->n_pix;
    p.descs = reinterpret_cast<InstDesc*>(ws + bp.off_descs);
    p.dyn = reinterpret_cast<InstDyn*>(ws + bp.off_dyn);
    p.group_slot = reinterpret_cast<int*>(ws + bp.off_gslot) + bk.gslot_idx;
    p.group_begin = reinterpret_cast<int*>(ws + bp.off_gbegin) + bk.gbegin_idx;
    p.inst_list = reinterpret_cast<int*>(ws + bp.off_ilist);
    p.img = images;
    p.img_ld = h->n_pix;
    p.n_levels = h->opt.n_levels;
    int nt = 0;
    if (!bb::synth_tile_info(h->opt.precision, bk.tile, nullptr, &nt, nullptr))
      return fail(ctx, BB_ERR_INVALID_ARG, "unknown tile %d", bk.tile);
    p.n_tiles = (h->n_pix + nt - 1) / nt;
    p.n_groups = bk.n_groups;
    BB_HIP(ctx, bb::launch_synth_tile(p, h->opt.precision, bk.tile, ctx->stream));
  }
  return BB_OK;
}

}  // namespace

bb_status bb_batched_workspace_size(bb_synth h, int32_t n_inst, const bb_instance* inst, size_t* bytes) {
  if (!h || !bytes) return BB_ERR_INVALID_ARG;
  BatchPlan bp;
  int64_t rows = 0;
  for (int i = 0; inst && i < n_inst; ++i) rows = std::max<int64_t>(rows, inst[i].ant_off + inst[i].n_ant);
  bb_status st = plan_batch(h, n_inst, inst, rows, -1, -1, h->tiles, -1, bp);
  if (st != BB_OK) return st;
  *bytes = bp.total;
  return BB_OK;
}

bb_status bb_synth_collect_eig_batched(bb_synth h, int32_t n_inst, const bb_instance* inst, int64_t n_ant_rows,
                                       int64_t n_w_elems, int64_t n_eig_elems, const double* ant_xyz_packed,
                                       const void* W_packed, const float* d_packed, const int32_t* level_packed,
                                       void* workspace, size_t ws_bytes) {
  if (!h) return BB_ERR_INVALID_ARG;
  bb_context ctx = h->ctx;
  if (!ant_xyz_packed || !W_packed || !d_packed || !level_packed || !workspace)
    return fail(ctx, BB_ERR_INVALID_ARG, "null device pointer");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return fail(ctx, BB_ERR_INVALID_ARG, "workspace must be %zu-byte aligned", kAlign);
  BatchPlan bp;
  if (n_w_elems < 0 || n_eig_elems < 0) return fail(ctx, BB_ERR_INVALID_ARG, "packed array lengths must be >= 0");
  bb_status st = plan_batch(h, n_inst, inst, n_ant_rows, n_w_elems, n_eig_elems, h->tiles, -1, bp);
  if (st != BB_OK) return st;
  if (ws_bytes < bp.total) return fail(ctx, BB_ERR_WORKSPACE, "workspace %zu < required %zu", ws_bytes, bp.total);
  BB_HIP(ctx, hipSetDevice(ctx->device));
  char* ws = static_cast<char*>(workspace);
  batch_descs(h, inst, n_inst, n_ant_rows, ant_xyz_packed, W_packed, d_packed, level_packed, ws, h->tiles, bp);
  hipStream_t s = ctx->stream;
  if (bb_host::debug_fill()) BB_HIP(ctx, bb::launch_fill_poison(ws, bp.total, s));
  BB_HIP(ctx, hipEventRecord(h->ev[0], s));
  BB_HIP(ctx, hipEventRecord(h->ev[1], s));
  st = upload_plan(ctx, bp, ws, n_inst, true);
  if (st != BB_OK) return st;
  BB_HIP(ctx, bb::launch_stage(reinterpret_cast<InstDesc*>(ws + bp.off_descs), reinterpret_cast<InstDyn*>(ws + bp.off_dyn),
                               n_inst, bp.max_K_alloc, bp.max_L_pad, h->opt.n_levels, h->opt.precision,
                               at<int>(h, h->lay.err), s));
  BB_HIP(ctx, hipEventRecord(h->ev[2], s));
  st = launch_buckets(h, bp, ws, h->images);
  if (st != BB_OK) return st;
  BB_HIP(ctx, hipEventRecord(h->ev[3], s));
  h->timed = true;
  h->count += n_inst;
  return BB_OK;
}

bb_status bb_tile_info(int32_t precision, int32_t tile, int32_t* eig_per_pass, int32_t* pix_per_tile, int32_t* waves,
                       int32_t* class_mask) {
  if (precision < BB_PREC_FP32 || precision > BB_PREC_BF16X3_3M) return BB_ERR_INVALID_ARG;
  int kc = 0, nt = 0, wv = 0;
  if (tile < 0 || !bb::synth_tile_info(precision, tile, &kc, &nt, &wv)) return BB_ERR_INVALID_ARG;
  int mask = 0;
  for (int c = 0; c < bb::kKClasses; ++c)
    if (bb::synth_tile_allowed(precision, tile, c)) mask |= 1 << c;
  if (eig_per_pass) *eig_per_pass = kc;
  if (pix_per_tile) *pix_per_tile = nt;
  if (waves) *waves = wv;
  if (class_mask) *class_mask = mask;
  return BB_OK;
}

bb_status bb_tune_cache_lookup(const char* arch, int32_t precision, int64_t n_pix, int32_t* tiles) {
  if (!arch || !tiles || n_pix < 1 || precision < BB_PREC_FP32 || precision > BB_PREC_BF16X3_3M)
    return BB_ERR_INVALID_ARG;
  int cached[bb::kKClasses];
  bb_host::tune_cache_lookup(arch, precision, n_pix, cached);
  for (int c = 0; c < bb::kKClasses; ++c)
    tiles[c] = (cached[c] >= 0 && bb::synth_tile_allowed(precision, cached[c], c)) ? cached[c] : -1;
  return BB_OK;
}

bb_status bb_synth_get_tiles(bb_synth h, int32_t* tiles) {
  if (!h || !tiles) return BB_ERR_INVALID_ARG;
  for (int c = 0; c < bb::kKClasses; ++c) tiles[c] = h->tiles[c];
  return BB_OK;
}

bb_status bb_synth_set_tiles(bb_synth h, const int32_t* tiles) {
  if (!h || !tiles) return BB_ERR_INVALID_ARG;
  int next[bb::kKClasses];
  for (int c = 0; c < bb::kKClasses; ++c) {
    next[c] = tiles[c] < 0 ? bb::synth_default_tile(h->opt.precision, c) : tiles[c];
    if (!bb::synth_tile_allowed(h->opt.precision, next[c], c))
      return fail(h->ctx, BB_ERR_INVALID_ARG, "tile %d is not a candidate for K class %d", tiles[c], c);
  }
  for (int c = 0; c < bb::kKClasses; ++c) h->tiles[c] = next[c];
  return BB_OK;
}

bb_status bb_synth_autotune_batched(bb_synth h, int32_t n_inst, const bb_instance* inst, int64_t n_ant_rows,
                                    int64_t n_w_elems, int64_t n_eig_elems, const double* ant_xyz_packed,
                                    const void* W_packed, const float* d_packed, const int32_t* level_packed,
                                    void* workspace, size_t ws_bytes, float* scratch_images, int32_t reps,
                                    double* ms_out) {
  if (!h) return BB_ERR_INVALID_ARG;
  bb_context ctx = h->ctx;
  if (!ant_xyz_packed || !W_packed || !d_packed || !level_packed || !workspace || !scratch_images)
    return fail(ctx, BB_ERR_INVALID_ARG, "null device pointer");
  if (!ms_out) return fail(ctx, BB_ERR_INVALID_ARG, "ms_out is NULL");
  if (reps < 1 || reps > 100) return fail(ctx, BB_ERR_INVALID_ARG, "reps must be in [1, 100]");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return fail(ctx, BB_ERR_INVALID_ARG, "workspace must be %zu-byte aligned", kAlign);
  if (n_w_elems < 0 || n_eig_elems < 0) return fail(ctx, BB_ERR_INVALID_ARG, "packed array lengths must be >= 0");
  BatchPlan full;
  bb_status st = plan_batch(h, n_inst, inst, n_ant_rows, n_w_elems, n_eig_elems, h->tiles, -1, full);
  if (st != BB_OK) return st;
  if (ws_bytes < full.total) return fail(ctx, BB_ERR_WORKSPACE, "workspace %zu < required %zu", ws_bytes, full.total);
  const int n_tiles = bb::synth_n_tiles(h->opt.precision);
  if (n_tiles > BB_MAX_TILES) return fail(ctx, BB_ERR_STATE, "more tile candidates than BB_MAX_TILES");
  for (int i = 0; i < bb::kKClasses * BB_MAX_TILES; ++i) ms_out[i] = -1.0;
  BB_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  char* ws = static_cast<char*>(workspace);
  batch_descs(h, inst, n_inst, n_ant_rows, ant_xyz_packed, W_packed, d_packed, level_packed, ws, h->tiles, full);
  if (bb_host::debug_fill()) BB_HIP(ctx, bb::launch_fill_poison(ws, full.total, s));
  st = upload_plan(ctx, full, ws, n_inst, true);
  if (st != BB_OK) return st;
  BB_HIP(ctx, bb::launch_stage(reinterpret_cast<InstDesc*>(ws + full.off_descs),
                               reinterpret_cast<InstDyn*>(ws + full.off_dyn), n_inst, full.max_K_alloc,
                               full.max_L_pad, h->opt.n_levels, h->opt.precision, at<int>(h, h->lay.err), s));
  BB_HIP(ctx, bb::launch_fill_zero(scratch_images, (int64_t)h->opt.n_slots * h->opt.n_levels * h->n_pix, s));
  bool present[bb::kKClasses] = {false, false, false, false};
  for (int i = 0; i < n_inst; ++i) present[bb::synth_k_class(bb::round_up(inst[i].n_eig, 32))] = true;
  int best[bb::kKClasses];
  for (int c = 0; c < bb::kKClasses; ++c) best[c] = h->tiles[c];
  for (int c = 0; c < bb::kKClasses; ++c) {
    if (!present[c]) continue;
    double best_ms = 0.0;
    for (int t = 0; t < n_tiles; ++t) {
      if (!bb::synth_tile_allowed(h->opt.precision, t, c)) continue;
      int tiles[bb::kKClasses];
      for (int q = 0; q < bb::kKClasses; ++q) tiles[q] = h->tiles[q];
      tiles[c] = t;
      BatchPlan bp;
      st = plan_batch(h, n_inst, inst, n_ant_rows, n_w_elems, n_eig_elems, tiles, c, bp);
      if (st != BB_OK) return st;
      // restage this class's instances when the tile takes the other operand order
      const int rows16 = bb::synth_tile_rows(h->opt.precision, t) == 16 ? 1 : 0;
      bool restage = false;
      for (int i = 0; i < n_inst; ++i)
        if (bb::synth_k_class(full.descs[i].K_alloc) == c && full.descs[i].rows16 != rows16) {
          full.descs[i].rows16 = rows16;
          restage = true;
        }
      bp.descs = full.descs;
      st = upload_plan(ctx, bp, ws, n_inst, restage);
      if (st != BB_OK) return st;
      if (restage)
        BB_HIP(ctx, bb::launch_stage(reinterpret_cast<InstDesc*>(ws + full.off_descs),
                                     reinterpret_cast<InstDyn*>(ws + full.off_dyn), n_inst, full.max_K_alloc,
                                     full.max_L_pad, h->opt.n_levels, h->opt.precision, at<int>(h, h->lay.err), s));
      st = launch_buckets(h, bp, ws, scratch_images);  // warm-up
      if (st != BB_OK) return st;
      BB_HIP(ctx, hipEventRecord(h->ev[0], s));
      for (int r = 0; r < reps; ++r) {
        st = launch_buckets(h, bp, ws, scratch_images);
        if (st != BB_OK) return st;
      }
      BB_HIP(ctx, hipEventRecord(h->ev[1], s));
      BB_HIP(ctx, hipEventSynchronize(h->ev[1]));
      float ms = 0.0f;
      BB_HIP(ctx, hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
      const double per = ms / reps;
      ms_out[c * BB_MAX_TILES + t] = per;
      if (best_ms == 0.0 || per < best_ms) {
        best_ms = per;
        best[c] = t;
      }
    }
  }
  for (int c = 0; c < bb::kKClasses; ++c) h->tiles[c] = best[c];
  h->timed = false;
  double best_ms[bb::kKClasses];
  for (int c = 0; c < bb::kKClasses; ++c) best_ms[c] = present[c] ? ms_out[c * BB_MAX_TILES + best[c]] : 0.0;
  std::string cache_err;
  if (!bb_host::tune_cache_store(ctx->arch, h->opt.precision, h->n_pix, best, best_ms, present, cache_err))
    return fail(ctx, BB_ERR_STATE, "%s (the handle keeps the tuned tiles)", cache_err.c_str());
  return BB_OK;
}

// ---- backward -------------------------------------------------------------
namespace {

struct BwdPlan {
  int L_pad, K_alloc, n_split;
  int64_t split_len;
  size_t off_E, off_dd, off_dW, off_dx, total;
};

BwdPlan plan_backward(int64_t n_pix, int n_ant, int n_eig) {
  BwdPlan b{};
  b.L_pad = bb::round_up(n_ant, bb::kAntChunk);
  b.K_alloc = bb::round_up(n_eig, 32);
  // pixel splits: the fused and dx kernels run (L_pad / 32) x n_split
  // workgroups, two of which fit a CU; 512 of them fill the 256 CUs
  const int64_t lblocks = b.L_pad / 32;
  int64_t want = (512 + lblocks - 1) / lblocks;
  const int64_t max_split = (n_pix + 63) / 64;
  if (want > max_split) want = max_split;
  if (want < 1) want = 1;
  b.split_len = ((n_pix + want - 1) / want + 63) / 64 * 64;
  b.n_split = (int)((n_pix + b.split_len - 1) / b.split_len);
  size_t p = 0;
  b.off_E = p;
  p += align_up((size_t)2 * b.K_alloc * n_pix * 4);
  b.off_dd = p;
  p += align_up((size_t)b.K_alloc * b.n_split * 8);
  b.off_dW = p;
  p += align_up((size_t)b.n_split * b.L_pad * b.K_alloc * 2 * 8);
  b.off_dx = p;
  p += align_up((size_t)b.n_split * b.L_pad * 3 * 8);
  b.total = p;
  return b;
}

}  // namespace

bb_status bb_backward_workspace_size(bb_synth h, int32_t n_ant, int32_t n_eig, size_t* bytes) {
  if (!h || !bytes) return BB_ERR_INVALID_ARG;
  bb_status st = check_instance_args(h, 0, n_ant, n_eig, 1.0);
  if (st != BB_OK) return st;
  *bytes = plan_backward(h->n_pix, n_ant, n_eig).total;
  return BB_OK;
}

bb_status bb_synth_eig_backward(bb_synth h, int32_t n_ant, int32_t n_eig, double wavelength_m,
                                const double* ant_xyz, const void* W, const float* d, const int32_t* level_of,
                                const float* grad_images, void* dW, float* dd, double* dx, void* workspace,
                                size_t ws_bytes) {
  if (!h) return BB_ERR_INVALID_ARG;
  bb_context ctx = h->ctx;
  bb_status st = check_instance_args(h, 0, n_ant, n_eig, wavelength_m);
  if (st != BB_OK) return st;
  if (!ant_xyz || !W || !d || !level_of || !grad_images || !dW || !dd || !dx || !workspace)
    return fail(ctx, BB_ERR_INVALID_ARG, "null device pointer");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return fail(ctx, BB_ERR_INVALID_ARG, "workspace must be %zu-byte aligned", kAlign);
  const BwdPlan bp = plan_backward(h->n_pix, n_ant, n_eig);
  if (ws_bytes < bp.total) return fail(ctx, BB_ERR_WORKSPACE, "workspace %zu < required %zu", ws_bytes, bp.total);
  BB_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  char* ws = static_cast<char*>(workspace);
  if (bb_host::debug_fill()) BB_HIP(ctx, bb::launch_fill_poison(ws, bp.total, s));
  InstDesc dsc = staging_desc(h, h->ws + h->lay.apack, n_ant, n_eig, wavelength_m, 0);
  dsc.ant = ant_xyz;
  dsc.ant_ld = n_ant;
  dsc.W = W;
  dsc.W_ld = n_ant;
  dsc.W_c128 = 0;
  dsc.wcol = nullptr;
  dsc.d = d;
  dsc.lev_in = level_of;
  SingleMeta* meta = at<SingleMeta>(h, h->lay.meta);
  BB_HIP(ctx, hipEventRecord(h->ev[0], s));
  BB_HIP(ctx, hipEventRecord(h->ev[1], s));
  hipLaunchKernelGGL(write_meta_kernel, dim3(1), dim3(1), 0, s, meta, dsc, 0);
  BB_HIP(ctx, hipGetLastError());
  // three planes: the recompute of E runs the three-product FP32 form
  BB_HIP(ctx, bb::launch_stage(&meta->desc, &meta->dyn, 1, dsc.K_alloc, dsc.L_pad, h->opt.n_levels, 2,
                               at<int>(h, h->lay.err), s));
  BB_HIP(ctx, hipEventRecord(h->ev[2], s));
  bb::FwdParams p{};
  p.pix = h->pix;
  p.pix_ld = h->n_pix;
  p.n_pix = h->n_pix;
  p.descs = &meta->desc;
  p.dyn = &meta->dyn;
  p.group_slot = &meta->group_slot;
  p.group_begin = meta->group_begin;
  p.inst_list = &meta->inst_list;
  p.img = nullptr;
  p.img_ld = h->n_pix;
  p.n_levels = h->opt.n_levels;
  const int nt = bb::fields_tile_pixels(dsc.K_alloc);
  p.n_tiles = (h->n_pix + nt - 1) / nt;
  p.n_groups = 1;
  p.e_out = reinterpret_cast<float*>(ws + bp.off_E);
  p.e_ld = h->n_pix;
  p.e_rows = dsc.K_alloc;
  BB_HIP(ctx, bb::launch_fields(p, dsc.K_alloc, s));
  bb::BwdParams b{};
  b.pix = h->pix;
  b.pix_ld = h->n_pix;
  b.n_pix = h->n_pix;
  b.desc = &meta->desc;
  b.dyn = &meta->dyn;
  b.gimg = grad_images;
  b.gimg_ld = h->n_pix;
  b.E = p.e_out;
  b.K_alloc = dsc.K_alloc;
  b.L_pad = dsc.L_pad;
  b.L = n_ant;
  b.K = n_eig;
  b.W = W;
  b.n_split = bp.n_split;
  b.split_len = bp.split_len;
  b.dd_part = reinterpret_cast<double*>(ws + bp.off_dd);
  b.dW_part = reinterpret_cast<double*>(ws + bp.off_dW);
  b.dx_part = reinterpret_cast<double*>(ws + bp.off_dx);
  b.scale_x = -4.0 * M_PI / wavelength_m;
  BB_HIP(ctx, bb::launch_backward(b, s));
  BB_HIP(ctx, bb::launch_backward_reduce(b, dW, dd, dx, s));
  BB_HIP(ctx, hipEventRecord(h->ev[3], s));
  h->timed = true;
  return BB_OK;
}

// ---- misc -------------------------------------------------------------------
bb_status bb_synth_sync(bb_synth h) {
  if (!h) return BB_ERR_INVALID_ARG;
  bb_context ctx = h->ctx;
  BB_HIP(ctx, hipSetDevice(ctx->device));
  BB_HIP(ctx, hipStreamSynchronize(ctx->stream));
  int err = 0;
  BB_HIP(ctx, hipMemcpy(&err, at<int>(h, h->lay.err), sizeof err, hipMemcpyDeviceToHost));
  if (err) {
    hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, ctx->stream, at<int>(h, h->lay.err));
    BB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::string msg;
    if (err & bb::kErrLevelId) msg += "a level id outside [-1, n_levels) was treated as -1; ";
    if (err & bb::kErrKmeansTooFew) msg += "k-means: fewer positive eigenvalues than positive levels; ";
    if (err & bb::kErrUvRange) msg += "uniform weighting: a uv cell index out of range or not finite; ";
    msg.resize(msg.size() - 2);
    return fail(ctx, BB_ERR_INVALID_ARG, "%s", msg.c_str());
  }
  return BB_OK;
}

bb_status bb_synth_reset(bb_synth h) {
  if (!h) return BB_ERR_INVALID_ARG;
  bb_context ctx = h->ctx;
  BB_HIP(ctx, hipSetDevice(ctx->device));
  const int64_t n = (int64_t)h->opt.n_slots * h->opt.n_levels * h->n_pix;
  BB_HIP(ctx, bb::launch_fill_zero(h->images, n, ctx->stream));
  h->count = 0;
  return BB_OK;
}

bb_status bb_synth_get_count(bb_synth h, int64_t* count) {
  if (!h || !count) return BB_ERR_INVALID_ARG;
  *count = h->count;
  return BB_OK;
}

bb_status bb_synth_set_count(bb_synth h, int64_t count) {
  if (!h || count < 0) return BB_ERR_INVALID_ARG;
  h->count = count;
  return BB_OK;
}

bb_status bb_phase_probe(bb_context ctx, int32_t n_ant, double wavelength_m, const double* ant_xyz, int64_t n_pix,
                         const double* pix, int32_t reps, float* out) {
  if (!ctx) return BB_ERR_INVALID_ARG;
  if (!ant_xyz || !pix || !out) return fail(ctx, BB_ERR_INVALID_ARG, "null pointer");
  if (n_ant < 1 || n_ant > bb::kMaxAnt) return fail(ctx, BB_ERR_INVALID_ARG, "n_ant must be in [1, %d]", bb::kMaxAnt);
  if (n_pix < 1 || reps < 1) return fail(ctx, BB_ERR_INVALID_ARG, "n_pix and reps must be >= 1");
  if (!(wavelength_m > 0.0) || !std::isfinite(wavelength_m))
    return fail(ctx, BB_ERR_INVALID_ARG, "wavelength must be positive and finite");
  BB_HIP(ctx, hipSetDevice(ctx->device));
  BB_HIP(ctx, bb::launch_phase_probe(ant_xyz, n_ant, 1.0 / wavelength_m, pix, n_pix, reps, out, ctx->stream));
  return BB_OK;
}

bb_status bb_synth_timings(bb_synth h, double* ms_out, int32_t n) {
  if (!h || !ms_out || n < 0) return BB_ERR_INVALID_ARG;
  bb_context ctx = h->ctx;
  if (!h->timed) return fail(ctx, BB_ERR_STATE, "no timed call yet");
  BB_HIP(ctx, hipEventSynchronize(h->ev[3]));
  for (int i = 0; i < n && i < 3; ++i) {
    float ms = 0.0f;
    BB_HIP(ctx, hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]));
    ms_out[i] = ms;
  }
  return BB_OK;
}

}  // extern "C"
