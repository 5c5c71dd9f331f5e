/*
 * bluebild.h -- C ABI of the MI355X (gfx950) Bluebild standard-synthesis library.
 *
 * What it computes (Tolley et al., "BIPP: An efficient HPC implementation of
 * the Bluebild algorithm for radio astronomy"):
 *
 *   For one (time step, channel) instance with L antennas at positions x_l,
 *   visibility matrix V (L x L) and pixel directions p (unit vectors):
 *     G_pq  = sinc(2 ||x_p - x_q|| / lambda_w)              Section 2.2, Eq. gram
 *     V a   = lambda G a,  a^H G a = 1                      Section 2.3, Eq. eigenvaleq
 *     keep the K largest eigenpairs (by signed value)       Section 2.6, Algorithm 1
 *     B_lp  = exp(+j 2 pi <x_l, p> / lambda_w)              Section 2.1 (Psi*, g = 1)
 *     E     = W^H B   (W = kept eigenvectors, L x K)        Section 2.4, Eq. standard_synthesis
 *     I_l(p) += sum_{k in level l} d_k |E_kp|^2             Section 2.6 level equation; Algorithm 1
 *   with d_k = lambda_k (least-squares filter) or d_k = 1 (standardized
 *   filter), and images summed over instances (Section 2.3).
 *
 * Sign convention: V_pq = sum_s I_s exp(+j 2 pi <x_p - x_q, r_s> / lambda_w).
 * Visibilities in the usual radio convention must be passed conjugated.
 * Scale convention: G_pp = 1 exactly (the continuous Gram of Eq. gram).
 *
 * Conventions for every call:
 *  - Device pointers are HIP device memory on the context's device; "host"
 *    marks the few host pointers.  All matrices are column-major (Table 1).
 *  - The caller owns every buffer, including the images and the workspace.
 *    The library keeps the pixel, image and workspace pointers given to
 *    bb_synth_create until bb_synth_destroy; it keeps no other pointer.
 *  - Work is enqueued on the context's HIP stream, in call order.  Inputs
 *    must stay valid and unmodified until the stream has reached the work;
 *    inputs are never written (except the visibilities given to
 *    bb_synth_uniform_weighting).  bb_synth_sync waits for the stream.
 *  - Arguments are validated on the host before anything is enqueued; a call
 *    that returns an error has enqueued nothing and left the images as they
 *    were.  Asynchronous device faults surface as BB_ERR_DEVICE from
 *    bb_synth_sync.  No C++ exception crosses this interface.
 *  - Calls on one handle, or on handles sharing a context, must not be made
 *    concurrently from several host threads.
 *  - Checkpoint / resume: the accumulated images and the instance count
 *    (bb_synth_get_count / bb_synth_set_count) are the whole state of a run;
 *    a handle created over restored images, with the count set, continues it
 *    bitwise (standard synthesis adds in a fixed order, with no atomics).
 *  - Debug aid: with the environment variable BB_DEBUG_FILL set to a value
 *    other than "0", every workspace handed to the library is filled with
 *    0xFF bytes (NaN as float32 / float64) before use, at handle or plan
 *    creation and at each call that takes a workspace, so that a read of
 *    unwritten workspace memory shows in the results.
 */
#ifndef BLUEBILD_H
#define BLUEBILD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BB_OK = 0,
  BB_ERR_INVALID_ARG = 1, /* null pointer, bad size, NaN input, bad interval, bad level id */
  BB_ERR_SHAPE = 2,       /* size beyond the maxima fixed at handle creation */
  BB_ERR_NOT_POSDEF = 3,  /* Cholesky of G failed (e.g. coincident antennas) */
  BB_ERR_EIGEN = 4,       /* eigensolver did not converge */
  BB_ERR_WORKSPACE = 5,   /* workspace smaller than bb_workspace_size() */
  BB_ERR_DEVICE = 6,      /* HIP runtime / library error */
  BB_ERR_STATE = 7        /* wrong object state (e.g. destroying a context with live handles) */
} bb_status;

/* Contraction arithmetic of the synthesis (FP64 phase arguments in every mode):
 *  BB_PREC_FP32     FP32 MFMA, four real products per complex product
 *  BB_PREC_BF16X3   BF16 hi/lo split of both operands, hi*hi + hi*lo + lo*hi in FP32 accumulators
 *  BB_PREC_FP32_3M  FP32 MFMA, three real products per complex product (Gauss):
 *                   conj(w) b = (k1 - k3) + j (k1 + k2), k1 = (wr - wi) br,
 *                   k2 = wr (bi - br), k3 = -wi (br + bi)
 *  BB_PREC_BF16X3_3M  the three-product form with BF16 hi/lo operands and three
 *                   compensating products each, FP32 accumulators */
typedef enum { BB_PREC_FP32 = 0, BB_PREC_BF16X3 = 1, BB_PREC_FP32_3M = 2, BB_PREC_BF16X3_3M = 3 } bb_precision;
typedef enum { BB_FILTER_LSQ = 0, BB_FILTER_STD = 1 } bb_filter;

typedef struct bb_context_* bb_context;
typedef struct bb_synth_* bb_synth;

/* Options fixed when a synthesis handle is created.
 *  n_levels   number of energy levels (images per slot), 1..16
 *  n_slots    number of image slots (e.g. channels), >= 1
 *  n_ant_max  largest antenna count of any instance, 1..1024
 *  k_max      largest number of kept eigenpairs, 1..1024, <= n_ant_max for bb_synth_collect
 *  precision  bb_precision of the contraction (see above)
 *  filter     bb_filter applied by bb_synth_collect (collect_eig takes weights directly)
 *  gram       bb_gram used by the pre-step: the instrument's Gram matrix (least-squares
 *             image), or the identity, which makes the image the back-projected
 *             (dirty) image diag(Psi V Psi*) of Section 2.8
 *  reserved   must be 0 */
typedef enum { BB_GRAM_SINC = 0, BB_GRAM_IDENTITY = 1 } bb_gram;
typedef struct {
  int32_t n_levels;
  int32_t n_slots;
  int32_t n_ant_max;
  int32_t k_max;
  int32_t precision;
  int32_t filter;
  int32_t gram;
  int32_t reserved;
} bb_options;

/* One instance of a batched call.  Offsets index the packed arrays passed to
 * bb_synth_collect_eig_batched:
 *  ant_off  first row of this instance in ant_xyz_packed (n_ant rows)
 *  w_off    first element of this instance's W block (n_ant x n_eig, column-major,
 *           leading dimension n_ant) in W_packed
 *  eig_off  first element of this instance's n_eig weights / level ids */
typedef struct {
  int32_t n_ant;
  int32_t n_eig;
  int32_t slot;
  int32_t reserved;
  double wavelength_m;
  int64_t ant_off;
  int64_t w_off;
  int64_t eig_off;
} bb_instance;

/* ---- context -------------------------------------------------------------
 * A context binds a HIP device and stream and holds the eigensolver library
 * handle (Section 3.1 "Context").  hip_stream may be NULL (default stream). */
bb_status bb_context_create(int device, void* hip_stream, bb_context* out);
bb_status bb_context_set_stream(bb_context ctx, void* hip_stream);
/* BB_ERR_STATE if synthesis handles created on it are still alive. */
bb_status bb_context_destroy(bb_context ctx);
const char* bb_status_string(bb_status s);
/* Message of the last failed call on this context; valid until the next call. */
const char* bb_last_error(bb_context ctx);

/* ---- synthesis handle ----------------------------------------------------
 * Bytes of device workspace a handle needs for these options and pixel count
 * (staging of one instance plus the FP64 pre-step of one instance). */
bb_status bb_workspace_size(bb_context ctx, const bb_options* opt, int64_t n_pix, size_t* bytes);

/* Create a StandardSynthesis handle (Section 3.1).
 *  pix_xyz    device, n_pix x 3 float64, column-major, unit vectors (X_pix of Table 1)
 *  images     device, float32 [n_slots][n_levels][n_pix]; accumulated into, never cleared
 *             except by bb_synth_reset
 *  workspace  device, ws_bytes >= bb_workspace_size(...) */
bb_status bb_synth_create(bb_context ctx, const bb_options* opt, int64_t n_pix, const double* pix_xyz,
                          float* images, void* workspace, size_t ws_bytes, bb_synth* out);

/* Full step of Algorithm 1 for one instance: Gram (FP64), generalized
 * eigensolve (FP64), selection of the n_eig largest eigenpairs, filter,
 * levels from intervals, synthesis, accumulation into images[slot].
 *  ant_xyz    device, n_ant x 3 float64 column-major, metres (P_icrs of Table 1)
 *  vis        device, complex128 n_ant x n_ant column-major, Hermitian (S of Table 1)
 *  n_eig      1..min(n_ant, k_max)
 *  intervals  host, n_levels x 2 float64 column-major [min, max] (I of Table 1),
 *             closed, min <= max, +-inf allowed; intervals may share an endpoint but
 *             must not overlap on more than that (a value on a shared endpoint
 *             goes to the lower-numbered level)
 * Returns BB_ERR_NOT_POSDEF if the Cholesky factorisation of G fails and
 * BB_ERR_EIGEN if the eigensolver fails; this status is read back from the
 * device, so the call waits for its own pre-step.  On those errors the images
 * are unchanged. */
bb_status bb_synth_collect(bb_synth h, int32_t slot, int32_t n_ant, double wavelength_m,
                           const double* ant_xyz, const double* vis, int32_t n_eig,
                           const double* intervals);

/* Full step with beamforming (Section 2.7): the n_ant antenna voltages are
 * combined into n_beam beams by W_bf, so the data are V^W = W_bf^H V W_bf and
 * the sampling operator is Phi* = W_bf^H Psi*.  The pre-step solves
 * V^W a = lambda (W_bf^H G W_bf) a (n_beam x n_beam, FP64), keeps the n_eig
 * largest, and synthesizes over the n_ant antennas with U = W_bf a.
 *  W_bf    device, complex128 n_ant x n_beam column-major, 1 <= n_beam <= n_ant
 *  vis_bf  device, complex128 n_beam x n_beam column-major, Hermitian
 *  n_eig   1..min(n_beam, k_max)
 * Otherwise as bb_synth_collect. */
bb_status bb_synth_collect_beamformed(bb_synth h, int32_t slot, int32_t n_ant, int32_t n_beam,
                                      double wavelength_m, const double* ant_xyz, const double* W_bf,
                                      const double* vis_bf, int32_t n_eig, const double* intervals);

/* Full step with N_eig chosen from the eigenvalues (Section 2.6 truncation):
 * the fewest leading eigenpairs whose eigenvalues add up to at least
 * energy_fraction (0 < f <= 1) of the sum of the positive eigenvalues, at most
 * k_max.  n_eig_out (host) receives the count used.  Otherwise as
 * bb_synth_collect. */
bb_status bb_synth_collect_energy(bb_synth h, int32_t slot, int32_t n_ant, double wavelength_m,
                                  const double* ant_xyz, const double* vis, double energy_fraction,
                                  const double* intervals, int32_t* n_eig_out);

/* The FP64 pre-step of bb_synth_collect alone (Algorithm 1 up to the
 * synthesis call), for callers that keep the eigenpairs, e.g. to image them
 * again or to differentiate the synthesis with respect to them.  Arguments as
 * for bb_synth_collect; outputs (device, overwritten):
 *  W_out      complex64 n_ant x n_eig column-major, kept eigenvectors (a^H G a = 1),
 *             in descending eigenvalue order
 *  lam_out    float64 n_eig eigenvalues, descending
 *  d_out      float32 n_eig filter weights of the handle's filter
 *  level_out  int32 n_eig level ids from the intervals (-1 = in none)
 * Waits for the eigensolver status like bb_synth_collect; images untouched. */
bb_status bb_synth_prestep(bb_synth h, int32_t n_ant, double wavelength_m, const double* ant_xyz,
                           const double* vis, int32_t n_eig, const double* intervals, void* W_out,
                           double* lam_out, float* d_out, int32_t* level_out);

/* The FP64 pre-step of bb_synth_prestep for n_inst instances of one antenna
 * count at once (Algorithm 1's per-step Gram, eigensolve and selection, over
 * many time steps or channels): the Gram matrices, one strided-batched
 * generalized eigensolve and the selections are enqueued together, and the
 * call waits once for all solver statuses instead of once per instance.
 *  n_inst          >= 1
 *  n_ant, n_eig    as bb_synth_prestep (1 <= n_eig <= n_ant, n_eig <= k_max)
 *  wavelengths_m   host, float64 n_inst
 *  ant_xyz_packed  device, float64 (n_inst n_ant) x 3 column-major (leading
 *                  dimension n_inst n_ant); instance i at rows i n_ant ..
 *  vis_packed      device, complex128, n_inst column-major n_ant x n_ant
 *                  matrices one after the other, each Hermitian
 *  intervals       host, as bb_synth_collect (one partition for all instances)
 *  W_out, lam_out, d_out, level_out  device, as bb_synth_prestep per instance,
 *                  instance i at element i n_ant n_eig of W_out and i n_eig of
 *                  the others: the packed layout bb_synth_collect_eig_batched
 *                  takes (ant_off = i n_ant, w_off = i n_ant n_eig, eig_off = i n_eig)
 *  workspace       device, 256-byte aligned,
 *                  ws_bytes >= bb_prestep_batched_workspace_size(...)
 *                  (two n_ant^2 complex128 matrices per instance plus the solver's area)
 * Errors as bb_synth_prestep, naming the first failing instance; the outputs
 * are then not written.  Images untouched. */
bb_status bb_prestep_batched_workspace_size(bb_synth h, int32_t n_inst, int32_t n_ant, int32_t n_eig, size_t* bytes);
bb_status bb_synth_prestep_batched(bb_synth h, int32_t n_inst, int32_t n_ant, int32_t n_eig,
                                   const double* wavelengths_m, const double* ant_xyz_packed, const double* vis_packed,
                                   const double* intervals, void* W_out, double* lam_out, float* d_out,
                                   int32_t* level_out, void* workspace, size_t ws_bytes);

/* Energy levels by k-means on the eigenvalues (Section 2.6; the split of the
 * positive eigenvalues into levels plus one level for every negative
 * eigenvalue follows Section 4.2).  The positive eigenvalues are cut into
 * k = n_levels - negative_level groups by exact one-dimensional k-means (the
 * partition into contiguous runs of the sorted values with the least total
 * within-group sum of squared deviations; on equal cost the highest cut is
 * the lowest possible).  Level 0 holds the largest group; the bound between
 * two groups is the midpoint of the gap between them, the top bound +inf,
 * the lowest positive bound b the midpoint between the smallest positive and
 * the largest non-positive eigenvalue (0 if none); with negative_level = 1
 * the last level is [-inf, nextafter(b, -inf)].
 *  n           number of eigenvalues, 1 <= n <= 1024
 *  lam         device, float64 n eigenvalues, any order
 *  intervals   device out, float64 n_levels x 2 column-major [min, max]
 *              (the layout bb_synth_collect takes on the host)
 *  level_of    device out, int32 n: first interval holding lam[i], else -1
 * Stream-ordered; images untouched.  Fewer positive eigenvalues than k is
 * found on the device: intervals become NaN, level_of -1, and the next
 * bb_synth_sync returns BB_ERR_INVALID_ARG. */
bb_status bb_synth_levels_kmeans(bb_synth h, int32_t n, const double* lam, int32_t negative_level,
                                 double* intervals, int32_t* level_of);

/* Uniform image weighting of a visibility matrix, in place (Section 3.5),
 * for use before bb_synth_collect.  The uv coordinate of baseline (p, q) is
 * a_pq = <x_p - x_q, e> / lambda_w * fov_rad for e = e_u, e_v, evaluated as
 * ((d0 e0 + d1 e1) + d2 e2) * (fov_rad / wavelength_m) with no fused
 * multiply-add; its cell is round(a) with halves away from zero, so cells
 * are 1/FoV wide and (p, q), (q, p) fall in mirrored cells.  Every V_pq is
 * divided (real and imaginary parts separately) by the number of ordered
 * pairs (p', q'), autocorrelations included, in the cell of (p, q).
 *  ant_xyz     device, float64 n_ant x 3 column-major, metres
 *  e_u, e_v    host, float64 3 each: image-plane axes at the phase centre
 *              (same frame as ant_xyz)
 *  fov_rad     field of view, radians
 *  vis         device, complex128 n_ant x n_ant column-major, read and
 *              overwritten (the one input this library writes)
 * Uses the handle's pre-step workspace (free between calls), so it is
 * stream-ordered with the handle's other calls.  A cell index beyond +-2^30
 * (or not finite) leaves that visibility unweighted and makes the next
 * bb_synth_sync return BB_ERR_INVALID_ARG. */
bb_status bb_synth_uniform_weighting(bb_synth h, int32_t n_ant, double wavelength_m, const double* ant_xyz,
                                     const double* e_u, const double* e_v, double fov_rad, double* vis);

/* Hot path only (Section 2.4 and Algorithm 2, given the eigenpairs):
 *  W          device, complex64 n_ant x n_eig column-major (interleaved re, im float32)
 *  d          device, float32 n_eig filter weights (lambda_k for the LSQ filter)
 *  level_of   device, int32 n_eig level ids in [0, n_levels) or -1 (eigenpair unused)
 * Accumulates images[slot][l] += sum_{k: level_of[k] = l} d_k |(W^H B)_kp|^2. */
bb_status bb_synth_collect_eig(bb_synth h, int32_t slot, int32_t n_ant, int32_t n_eig, double wavelength_m,
                               const double* ant_xyz, const void* W, const float* d,
                               const int32_t* level_of);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): the hot path
 * of bb_synth_collect_eig without a synthesis handle or a workspace.  The
 * instance's metadata and staged operands go to a fixed scratch array inside
 * the library, BB_NOALLOC_SCRATCH_BYTES per device, which each device holds
 * from the first context created on it until the process ends.  The call
 * itself makes no hipMalloc, hipFree or allocating library call.
 *  precision  bb_precision of the contraction
 *  n_levels   1..16, images per call
 *  n_pix, pix_xyz  as bb_synth_create (device, n_pix x 3 float64 column-major)
 *  images     device, float32 [n_levels][n_pix], accumulated into
 *  n_ant, n_eig, wavelength_m, ant_xyz, W, d, level_of  as bb_synth_collect_eig
 * The images equal those of bb_synth_collect_eig on a handle of the same
 * precision and level count (same kernels).  Returns BB_ERR_WORKSPACE, having
 * enqueued nothing, when the instance's staging (16 round_up(n_eig, 32)
 * round_up(n_ant, 32) bytes plus about 1 KB) exceeds the scratch: for
 * example n_ant = n_eig = 512 fits, n_ant = n_eig = 1024 does not.  Level
 * ids outside [-1, n_levels) are treated as -1 without a report.
 * Every call on one device shares that device's scratch and leaves its
 * contents behind: calls ordered on one stream are safe; calls that can run
 * at the same time on one device (several streams or host threads) race and
 * give wrong images. */
#define BB_NOALLOC_SCRATCH_BYTES ((size_t)8 << 20)
bb_status bb_synth_collect_eig_noalloc(bb_context ctx, int32_t precision, int32_t n_levels, int64_t n_pix,
                                       const double* pix_xyz, float* images, int32_t n_ant, int32_t n_eig,
                                       double wavelength_m, const double* ant_xyz, const void* W, const float* d,
                                       const int32_t* level_of);

/* ---- tile shapes of the synthesis kernel (not in the paper) ----------------
 * An instance's K class is its kept eigenpair count rounded up to 32: class
 * 0, 1, 2, 3 for at most 32, 64, 128, or more.  Each precision has a list of
 * tile shapes (ids 0 .. at most BB_MAX_TILES - 1): eigenpairs per pass x
 * pixels per tile, with a wave count.  A handle holds one tile id per K class,
 * initially the measured default; the batched call launches one persistent
 * kernel per distinct tile among its instances.
 * bb_tile_info: shape of tile `tile` of `precision` (BB_ERR_INVALID_ARG past the
 *   end of the list); class_mask bit c is set when K class c may use it (its
 *   eigenpairs per pass do not exceed the class's largest K).  Any out pointer may be NULL.
 * bb_synth_get_tiles / bb_synth_set_tiles: the handle's table, BB_K_CLASSES
 *   ids (host); -1 on set restores a class's default; a tile the class may not
 *   use is rejected and the table left unchanged.
 * bb_synth_autotune_batched: times every tile each K class present in the
 *   batch may use, on that class's instances over the handle's pixels (one
 *   warm-up, then `reps` launches, 1..100), and keeps the fastest in the
 *   handle's table.  Arguments as bb_synth_collect_eig_batched, plus
 *   scratch_images (device, float32 n_slots x n_levels x n_pix, overwritten;
 *   the handle's images are not touched) and ms_out (host, BB_K_CLASSES x
 *   BB_MAX_TILES doubles, row per class: mean milliseconds per launch, -1 where
 *   not timed).  Waits for the device.
 * Autotune cache: with the environment variable BB_TUNE_CACHE naming a file,
 *   bb_synth_autotune_batched records the tile it kept for each K class it
 *   timed, keyed by (device architecture, precision, K class,
 *   floor(log2(n_pix))), one JSON object per line (the file is replaced
 *   whole through a temporary file beside it; lines in another form are
 *   kept), and bb_synth_create starts a handle from the cached tiles of its
 *   key (a cached tile its class may not use is ignored).  A cache that
 *   cannot be written makes the autotune call return BB_ERR_STATE; the
 *   handle keeps the tuned tiles.
 * bb_tune_cache_lookup: the tiles a new handle of device architecture `arch`
 *   (e.g. "gfx950"), `precision` and `n_pix` pixels would take from the
 *   cache: tiles (host, BB_K_CLASSES ints) gets each class's cached tile, or
 *   -1 where there is none (or BB_TUNE_CACHE is unset).  Host only: touches
 *   no device. */
#define BB_K_CLASSES 4
#define BB_MAX_TILES 12
bb_status bb_tile_info(int32_t precision, int32_t tile, int32_t* eig_per_pass, int32_t* pix_per_tile, int32_t* waves,
                       int32_t* class_mask);
bb_status bb_tune_cache_lookup(const char* arch, int32_t precision, int64_t n_pix, int32_t* tiles);
bb_status bb_synth_get_tiles(bb_synth h, int32_t* tiles);
bb_status bb_synth_set_tiles(bb_synth h, const int32_t* tiles);
bb_status bb_synth_autotune_batched(bb_synth h, int32_t n_inst, const bb_instance* inst, int64_t n_ant_rows,
                                    int64_t n_w_elems, int64_t n_eig_elems, const double* ant_xyz_packed,
                                    const void* W_packed, const float* d_packed, const int32_t* level_packed,
                                    void* workspace, size_t ws_bytes, float* scratch_images, int32_t reps,
                                    double* ms_out);

/* Many uneven instances in one launch (not in the paper, which takes one
 * instance per call).  inst is a host array of n_inst descriptors; the packed
 * device arrays hold every instance's data at the descriptor offsets:
 *  ant_xyz_packed  device, float64 n_ant_rows x 3 column-major (leading dim n_ant_rows)
 *  W_packed        device, complex64, n_w_elems elements
 *  d_packed        device, float32, n_eig_elems elements
 *  level_packed    device, int32, n_eig_elems elements
 *  workspace       device, 256-byte aligned, ws_bytes >= bb_batched_workspace_size(...)
 * Every instance's rows, W block and eigenpairs must lie inside these lengths
 * (BB_ERR_INVALID_ARG otherwise, found on the host before anything is enqueued).
 * Results equal calling bb_synth_collect_eig once per instance, up to the
 * order of floating-point summation across instances of one slot. */
bb_status bb_batched_workspace_size(bb_synth h, int32_t n_inst, const bb_instance* inst, size_t* bytes);
bb_status bb_synth_collect_eig_batched(bb_synth h, int32_t n_inst, const bb_instance* inst,
                                       int64_t n_ant_rows, int64_t n_w_elems, int64_t n_eig_elems,
                                       const double* ant_xyz_packed, const void* W_packed, const float* d_packed,
                                       const int32_t* level_packed, void* workspace, size_t ws_bytes);

/* Backward of collect_eig for the loss sum_l sum_p grad_images[l][p] * I_l(p)
 * (images of this one instance, before accumulation).  Outputs (overwritten):
 *  dW    device, complex64 n_ant x n_eig: dLoss/dRe(W) + j dLoss/dIm(W)
 *  dd    device, float32 n_eig
 *  dx    device, float64 n_ant x 3 column-major
 *  grad_images  device, float32 [n_levels][n_pix]
 *  workspace    device, ws_bytes >= bb_backward_workspace_size(...) */
bb_status bb_backward_workspace_size(bb_synth h, int32_t n_ant, int32_t n_eig, size_t* bytes);
bb_status bb_synth_eig_backward(bb_synth h, int32_t n_ant, int32_t n_eig, double wavelength_m,
                                const double* ant_xyz, const void* W, const float* d,
                                const int32_t* level_of, const float* grad_images,
                                void* dW, float* dd, double* dx, void* workspace, size_t ws_bytes);

/* ---- NUFFT synthesis ------------------------------------------------------
 * The level images again, evaluated as the type-3 Fourier sum over baselines
 * (Section 2.5; Section 3.4 and Algorithm 3):
 *   I_l(p) = sum_q V'_l[q, q] + 2 Re sum_{q < r} V'_l[r, q] exp(+2 pi i <b_qr, p>),
 *   V'_l = W_l diag(d_l) W_l^H (the eigenpairs of level l),  b_qr = (x_q - x_r) / lambda_w,
 * which equals standard synthesis of the same eigenpairs up to the NUFFT
 * tolerance.  In the image frame (e_u, e_v, p0) each baseline is spread onto a
 * periodic N0 x N1 x N2 grid with the exponential-of-semicircle kernel
 * phi(z) = exp(beta (sqrt(1 - z^2) - 1)), w = ceil(log10(1 / epsilon) - 1e-9) + 1
 * points of support, beta = 2.30 w; the grid is deconvolved, zero-padded to
 * M = 2 N, transformed (e^{+i}) one axis at a time over only the lines that
 * hold data and only the outputs the pixels reach, interpolated at the pixels
 * and divided by the kernel's transform.  Per frame axis d, with pixel half-width
 * S_d (floored at 1e-12) about the centre D_d and baseline bound X_d = uvw_max[d]:
 *   spacing h_d = 1 / (4 S_d) turns, N_d = the least even 2^a 3^b 5^c
 *   >= max(2 w, ceil(8 X_d S_d) + w).
 * Instances collected before one bb_nufft_emit share the grid: the transform,
 * interpolation and correction run once per emit and level.  Where grid
 * points are added with FP32 atomics (the busiest parts of the uv plane, and
 * grids thicker than 32 points along p0) the last bits of a result vary
 * between runs.  Memory: n_levels N0 N1 N2 complex64 grid cells plus two stage
 * buffers of about N0 M1 M2 / 2 cells each (bb_nufft_workspace_size).
 * Allocation: the plan and its calls use only the caller's workspace, except
 * on the rocFFT transform, whose plans (made at bb_nufft_create, released at
 * bb_nufft_destroy) keep device tables that rocFFT allocates itself. */
typedef struct bb_nufft_* bb_nufft;
typedef struct {
  int32_t n_levels;   /* images, 1..16 */
  int32_t n_ant_max;  /* largest antenna count of an instance, 2..1024 */
  int32_t k_max;      /* largest eigenpair count of an instance, 1..1024 */
  int32_t transform;  /* type-2 transform: 0 = automatic (the library's own LDS line
                         FFTs when every M_d <= 16384 and fits the device's LDS, else rocFFT), 1 = rocFFT */
  double epsilon;     /* requested accuracy, 1e-7 .. 1e-2 */
  double frame[9];    /* rows e_u, e_v, p0: orthonormal, in the frame of ant_xyz and pix_xyz */
  double uvw_max[3];  /* bound on |<x_q - x_r, frame row d>| / lambda_w over every baseline
                         to be collected (wavelengths); a baseline beyond it is skipped and
                         reported by bb_nufft_sync */
  int32_t partitions; /* image-domain partitions per axis, 0..8 (0 and 1: one tile).  With
                         P > 1 the pixels are split into P x P tiles of the (e_u, e_v)
                         extent, each imaged by its own NUFFTs (grids sized to the tile) */
  int32_t uvw_partitions; /* uvw-domain partitions per axis, 0..16 (0 and 1: one cell).  With
                         Q > 1 the baselines are split into Q x Q cells of
                         [-uvw_max[0], uvw_max[0]] x [-uvw_max[1], uvw_max[1]] along e_u and e_v
                         (cell of b: floor((b + X) Q / (2 X)), clamped to [0, Q - 1]); each
                         cell's baselines are shifted by the cell centre C and transformed on a
                         grid sized by the cell's half-width (X / Q) (1 + 1e-9), and the result
                         multiplied by exp(2 pi i <p, C>) */
} bb_nufft_options;
/* Partitioned plans (partitions > 1 or uvw_partitions > 1; Section 3.4.1) run one
 * NUFFT per (image tile, uvw cell) pair, one after another on the stream, all on
 * one grid and one set of transform buffers sized for the largest pair: memory
 * is bounded by the largest pair, not the sum.  Each bb_nufft_collect_eig_batched
 * call of a partitioned plan spreads, transforms and interpolates right away
 * (Algorithm 3 adds one NUFFT per step), so its bb_nufft_emit has nothing left to
 * do; the images are the same up to rounding. */

/* Workspace bytes of a plan.  pix_host: host, n_pix x 3 float64 column-major,
 * the pixels the plan will be created with (their extents fix the grid). */
bb_status bb_nufft_workspace_size(bb_context ctx, const bb_nufft_options* opt, int64_t n_pix, const double* pix_host,
                                  size_t* bytes);
/* Create a plan.  pix_host as above (read during the call only); pix_xyz: the
 * same pixels on the device (kept; the transform keeps only the grid points
 * that the planned pixels reach, and treats any other point a differing
 * device pixel would read as zero); images: device, float32 [n_levels][n_pix],
 * accumulated into by bb_nufft_emit; workspace: device, 256-byte aligned,
 * ws_bytes >= bb_nufft_workspace_size(...).  Waits for its set-up work. */
bb_status bb_nufft_create(bb_context ctx, const bb_nufft_options* opt, int64_t n_pix, const double* pix_host,
                          const double* pix_xyz, float* images, void* workspace, size_t ws_bytes, bb_nufft* out);
/* Grid sizes (N, M, 3 values each) and kernel support of a plan (of its largest
 * partition when partitioned); NULL outputs are skipped. */
bb_status bb_nufft_shape(bb_nufft h, int32_t* spread_grid, int32_t* fft_grid, int32_t* kernel_width);
/* Spread instances onto the grid; packed arrays and descriptors as for
 * bb_synth_collect_eig_batched (slot must be 0, n_ant >= 2).  workspace:
 * device, 256-byte aligned, >= bb_nufft_batched_workspace_size(...) bytes,
 * in use until the stream reaches the work. */
bb_status bb_nufft_batched_workspace_size(bb_nufft h, int32_t n_inst, const bb_instance* inst, size_t* bytes);
bb_status bb_nufft_collect_eig_batched(bb_nufft h, int32_t n_inst, const bb_instance* inst, int64_t n_ant_rows,
                                       int64_t n_w_elems, int64_t n_eig_elems, const double* ant_xyz_packed,
                                       const void* W_packed, const float* d_packed, const int32_t* level_packed,
                                       void* workspace, size_t ws_bytes);
/* Transform what has been spread since the last emit, add it to the images,
 * and clear the grid. */
bb_status bb_nufft_emit(bb_nufft h);
/* Wait; BB_ERR_INVALID_ARG (cleared) if a kernel skipped a baseline beyond
 * uvw_max or treated an out-of-range level id as -1. */
bb_status bb_nufft_sync(bb_nufft h);
/* Device ms of the last spread call [0] and the last emit [1]; waits. */
bb_status bb_nufft_timings(bb_nufft h, double* ms_out, int32_t n);
bb_status bb_nufft_destroy(bb_nufft h);

/* Wait for all enqueued work; BB_ERR_DEVICE on an asynchronous device error,
 * BB_ERR_INVALID_ARG (and clear it) when a kernel found an input error: a level
 * id out of range, too few positive eigenvalues for k-means, a uv cell out of
 * range; bb_last_error names which. */
bb_status bb_synth_sync(bb_synth h);
/* Zero every image (stream-ordered) and set the instance count to 0. */
bb_status bb_synth_reset(bb_synth h);
/* Number of instances accumulated since creation / reset; settable for resume. */
bb_status bb_synth_get_count(bb_synth h, int64_t* count);
bb_status bb_synth_set_count(bb_synth h, int64_t count);
/* Device time (ms) of the last call's stages: [0] pre-step (Gram + eigensolve),
 * [1] selection and staging, [2] synthesis.  Waits for the stream.  At most
 * 3 values are written. */
bb_status bb_synth_timings(bb_synth h, double* ms_out, int32_t n);
bb_status bb_synth_destroy(bb_synth h);

/* Phase-generation throughput probe, for measurement only.  Standard synthesis
 * evaluates the phase exp(+j 2 pi <x_l, p> / lambda) of every (antenna, pixel)
 * pair (Section 2.4, Eq. standard_synthesis; Algorithm 2); this call does that
 * work alone, with the synthesis kernel's arithmetic (FP64 argument and exact
 * reduction in turns, hardware FP32 sine and cosine), and no contraction, so
 * that timing it gives the device's peak rate of phase generation.  For each
 * pixel p it writes out[p] = reps * sum_l (cos + sin)(2 pi <x_l, p> / lambda),
 * summed in FP32 (every antenna's phase evaluated reps times).
 *  n_ant         antennas, 1 .. 1024
 *  wavelength_m  > 0
 *  ant_xyz       device, n_ant x 3 column-major, metres
 *  n_pix         pixels, >= 1
 *  pix           device, n_pix x 3 column-major unit vectors
 *  reps          repetitions over the antennas, >= 1
 *  out           device, n_pix floats (written)
 * Enqueued on the context's stream (time it with events there); the caller
 * owns every buffer.  BB_ERR_INVALID_ARG for null pointers or sizes out of
 * range, BB_ERR_DEVICE if the launch fails. */
bb_status bb_phase_probe(bb_context ctx, int32_t n_ant, double wavelength_m, const double* ant_xyz, int64_t n_pix,
                         const double* pix, int32_t reps, float* out);

#ifdef __cplusplus
}
#endif

#endif /* BLUEBILD_H */
