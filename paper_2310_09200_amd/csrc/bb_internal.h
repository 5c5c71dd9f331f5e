// Internal declarations shared by the host API and the kernels (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bb {

// Antennas per LDS phase chunk; every instance's antenna count is padded to it.
constexpr int kAntChunk = 32;
// Largest level count a handle may use (sizes the per-tile level accumulators in LDS).
constexpr int kMaxLevels = 16;
// Largest antenna / eigenpair counts.
constexpr int kMaxAnt = 1024;
constexpr int kMaxEig = 1024;

// Bytes of the fixed device scratch used by bb_synth_collect_eig_noalloc
// (one instance's metadata, error word and staging; noalloc.hip).
constexpr size_t kNoallocScratchBytes = (size_t)8 << 20;  // BB_NOALLOC_SCRATCH_BYTES
// Device address of that scratch on the current device (hipGetSymbolAddress).
hipError_t noalloc_scratch_address(void** out);

// Bits of a handle's device error word (read and cleared by bb_synth_sync).
constexpr int kErrLevelId = 1;        // a level id outside [-1, n_levels) was treated as -1
constexpr int kErrKmeansTooFew = 2;   // k-means: fewer positive eigenvalues than positive levels
constexpr int kErrUvRange = 4;        // uniform weighting: a uv cell index beyond +-2^30 or not finite
constexpr int kErrNufftExtent = 8;    // NUFFT synthesis: a baseline beyond the planned extent (skipped)

__host__ __device__ inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

// One instance as seen by the staging and synthesis kernels.  Built on the
// host; the device-computed part (kept eigenpair count) lives in InstDyn.
struct InstDesc {
  const double* ant;     // antenna x column; y at ant + ant_ld, z at ant + 2*ant_ld
  int64_t ant_ld;
  const void* W;         // eigenvectors, column-major, leading dim W_ld
  int64_t W_ld;
  const int* wcol;       // optional column map (nullptr = identity)
  const float* d;        // filter weights, one per eigenpair
  const int* lev_in;     // level id per eigenpair, -1 = unused
  double scale;          // 1 / wavelength: positions in turns per unit direction
  int L, K, L_pad, K_alloc;
  int slot, W_c128;
  int rows16;            // staged operand order: 1 = 16-row blocks (tiles on 16x16x4 MFMAs), 0 = 32-row
  int pad1;
  // workspace regions owned by this instance
  void* apack;           // packed real-embedded W^H, MFMA operand order
  double* xs;            // [L_pad][4] scaled positions
  float* wts;            // [K_alloc] weights after level sort (0 beyond K_eff)
  int* levs;             // [K_alloc] level ids after sort (-1 beyond K_eff)
  int2* kbr;             // [K_alloc/32] (lowest, highest) level of each 32-block, then
                         // [K_alloc/16] the same for each 16-block
  int* perm;             // [K_alloc] source eigenpair of each sorted position (-1 = pad)
};

struct InstDyn {
  int K_pad;             // kept eigenpairs rounded up to 32
  int K_eff;
};

struct FwdParams {
  const double* pix;     // x column; y at pix + pix_ld, z at pix + 2*pix_ld
  int64_t pix_ld;
  int64_t n_pix;
  const InstDesc* descs;
  const InstDyn* dyn;
  const int* group_slot;   // image slot of group g (groups in processing order)
  const int* group_begin;  // instances of group g: inst_list[group_begin[g] .. group_begin[g+1])
  const int* inst_list;
  int n_groups;
  float* img;              // [n_slots][n_levels][img_ld]
  int64_t img_ld;
  int n_levels;
  int64_t n_tiles;
  float* e_out;            // backward only: E planes [2][e_rows][e_ld]
  int64_t e_ld;
  int e_rows;
};

// Staging (launchers in synth_kernels.hip).
hipError_t launch_stage(const InstDesc* d_descs, InstDyn* d_dyn, int n_inst, int max_K_alloc, int max_L_pad,
                        int n_levels, int precision, int* d_err, hipStream_t s);

// Synthesis tiles.  K class of an instance: 0..3 for kept eigenpairs rounded
// up to 32 of at most 32, 64, 128, or more.  Each precision has a list of
// tile shapes (ids 0 .. synth_n_tiles - 1) and a default per class.
constexpr int kKClasses = 4;
int synth_k_class(int K_alloc);
int synth_n_tiles(int precision);
int synth_default_tile(int precision, int k_class);
// Eigenpairs per pass, pixels per tile and waves of a tile; false for an unknown id.
bool synth_tile_info(int precision, int id, int* kc, int* nt, int* waves);
// Whether a class may use a tile (its eigenpairs per pass do not exceed the class's largest K).
bool synth_tile_allowed(int precision, int id, int k_class);
// Rows of a tile's eigenpair blocks (32, or 16 for tiles on 16x16x4 MFMAs); the
// instances a tile runs must be staged in that order (InstDesc::rows16).
int synth_tile_rows(int precision, int id);
hipError_t launch_synth_tile(const FwdParams& p, int precision, int id, hipStream_t s);
// The default tile for the largest K_alloc of the call.
hipError_t launch_synth(const FwdParams& p, int max_K_alloc, int precision, int tile_pixels_out[1],
                        hipStream_t s);
int synth_tile_pixels(int max_K_alloc, int precision);

// Zero-fill of a float buffer (graph-capture safe, no memset nodes).
hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s);
// Fill n bytes with 0xFF (the workspace poison of BB_DEBUG_FILL).
hipError_t launch_fill_poison(void* p, size_t n, hipStream_t s);
hipError_t launch_phase_probe(const double* ant, int n_ant, double inv_wl, const double* pix, int64_t n_pix, int reps,
                              float* out, hipStream_t s);

// Pre-step kernels (prestep.hip).
hipError_t launch_gram(const double* ant, int64_t ant_ld, int L, double wl, double* G_c128, int ldg, bool identity,
                       hipStream_t s);
hipError_t launch_copy_c128(const double* src, int L, double* dst, int ldd, hipStream_t s);
// out[0] = ||V - V^H||_F^2, out[1] = ||V||_F^2 of an L x L complex128 matrix.
hipError_t launch_herm_check(const double* V, int L, double* out, hipStream_t s);
struct Intervals {
  double lo[kMaxLevels];
  double hi[kMaxLevels];
};
hipError_t launch_select(const double* evals, int L, int K, Intervals iv, int n_levels, int filter,
                         float* d_out, int* lev_out, int* wcol_out, hipStream_t s);
// Batched pre-step of n_inst instances with L antennas each: Gram matrices
// (antennas of instance i at rows i L of a column-major array with leading
// dimension ant_ld; 1/wavelength inv_wl[i], device), copies of the
// visibilities into A, Hermiticity sums into herm[2 i, 2 i + 1]; then the
// selection and export of each instance's K kept eigenpairs.  Matrices are
// packed one after the other (2 L^2 doubles each).
hipError_t launch_prestep_inputs_batched(const double* ant, int64_t ant_ld, int L, const double* inv_wl, int n_inst,
                                         bool identity, const double* vis, double* A, double* G, double* herm,
                                         hipStream_t s);
hipError_t launch_select_export_batched(const double* A, const double* evals, int L, int K, int n_inst, Intervals iv,
                                        int n_levels, int filter, float* dsel, int* lsel, int* wcol, float* W_out,
                                        double* lam_out, float* d_out, int* lev_out, hipStream_t s);
hipError_t launch_export_eig(const double* A_c128, const double* evals, int L, int K, const int* wcol,
                             const float* dsel, const int* lsel, float* W_out_c64, double* lam_out, float* d_out,
                             int* lev_out, hipStream_t s);

// Level determination and weighting (levels_weighting.hip).
hipError_t launch_kmeans_levels(const double* lam, int n, int k, int negative_level, double* intervals,
                                int* level_of, int* err, hipStream_t s);
struct UvFrame {
  double eu[3], ev[3];  // image-plane axes at the phase centre
  double scale;         // FoV / wavelength: cells per metre of baseline
};
int64_t uv_table_slots(int L);  // hash slots for L^2 pairs (power of two >= 2 L^2); 12 bytes each
hipError_t launch_uniform_weighting(const double* ant, int64_t ld, int L, const UvFrame& f, void* table,
                                    double* vis, int* err, hipStream_t s);

// NUFFT synthesis (nufft.hip).
struct NufftGeom {
  double R[3][3];   // image frame, rows e_u, e_v, p0
  double D[3];      // centre of the pixels in the frame
  double X[3];      // bound on |baseline| per frame axis, wavelengths
  double h[3];      // spread-grid spacing, turns
  double inv_h[3];  // 1 / h
  double hM[3];     // h * M: type-2 grid points per unit of pixel offset
  int N[3];         // spread grid
  int M[3];         // type-2 (FFT) grid, 2 N
  int win_lo[3];    // first type-2 grid point the pixels need per axis (mod M)
  int win_len[3];   // number of type-2 grid points the pixels need per axis
  int w;            // kernel support in grid points
  float beta;       // kernel shape
  // uvw-domain partitions (Section 3.4.1): a plan may transform only the
  // baselines of one cell of a cell_q x cell_q split of [-Xf, Xf] along e_u
  // and e_v, shifted by the cell's centre C (its grid is sized by the cell's
  // half-width X); the interpolation multiplies by exp(2 pi i <s, C>).
  double C[3];      // source shift, wavelengths (zero without cells)
  double Xf[3];     // bound on |baseline| of every source (the plan's uvw_max)
  int cell_q;       // cells per axis along e_u and e_v (<= 1: a single cell, no shift)
  int cell_i[2];    // this plan's cell along e_u and e_v
  int use_diag;     // the interpolation adds sum_q V'_qq (one plan per set of pixels)
};

// uvw cell of a baseline coordinate b along one axis: floor((b + X) q / (2 X)),
// clamped to [0, q - 1] (so b = X falls in the last cell).
__host__ __device__ inline int uvw_cell(double b, double X, int q) {
  const int c = (int)floor((b + X) * (q / (2.0 * X)));
  return c < 0 ? 0 : (c >= q ? q - 1 : c);
}
struct NufftInst {
  int n_ant, n_eig;
  double wavelength_m;
  int64_t ant_off, w_off, eig_off;
  int64_t ord_off, ls_off;  // this instance's level-grouped order and level starts
  int64_t vp_off;           // this instance's V' block (n_levels x n_ant^2 complex64)
};
hipError_t launch_nufft_prep(const NufftInst* insts, int n_inst, const void* W, const float* d, const int* lev,
                             int n_levels, int* order, int* lstart, double* diag, int* err, hipStream_t s);
hipError_t launch_nufft_spread(const NufftGeom& g, const NufftInst* insts, int n_inst, int max_ant,
                               const double* ant, int64_t ant_ld, const void* Wmat, const float* d, const int* order,
                               const int* lstart, int n_levels, float* grid, int64_t n_cell, int* err, hipStream_t s);
// One gather of the pruned type-2 transform: axis 2 (grid -> A), 1 (A -> B) or 0 (B -> C).
hipError_t launch_nufft_gather(int axis, const NufftGeom& g, const void* src, const float* inv_psi, void* dst,
                               hipStream_t s);
// Where the interpolation finds type-2 point (m0, m1, m2): at w1 s1 + w2 s2 + w0
// (complex64 elements), w_d = (m_d - win_lo[d]) mod M_d; axis 0 is windowed
// by (lo0, len0) (0 and M0 for an unwindowed axis).  Points outside read as 0.
struct InterpLayout {
  int64_t s1, s2;
  int lo0, len0;
};
// Adds 2 Re(exp(2 pi i <s, C>) interpolated value) * corr (+ diag[lv] when
// g.use_diag) to each pixel's level image.
hipError_t launch_nufft_interp(const NufftGeom& g, const InterpLayout& lay, const double* pix, int64_t pix_ld,
                               int64_t n_pix, const float* u, const double* corr, const double* diag, int lv,
                               float* image, hipStream_t s);
// Line FFTs of the pruned transform (nufft_fft.hip).
constexpr int kLineFftMax = 16384;  // longest line held in LDS (128 KB)
constexpr int kLineDftMax = 64;     // lines up to this length may be a direct pruned DFT instead
struct LineFft {
  int L;                 // transform length (M of the axis)
  int n_in;              // stored inputs per line (N of the axis)
  int win_lo, win_len;   // outputs kept: positions (win_lo + w) mod L, w < win_len
  int n_pass, nl;        // Stockham passes; lines per workgroup
  uint64_t radix_codes;  // radix of pass i in bits [4i, 4i + 4)
  int64_t n_lines, in_stride, out_stride;
  int64_t t_inner;       // out_mode 1: line = outer * t_inner + inner, stored at [outer][w][inner]
  int out_mode;          // 0: out[line * out_stride + w]
  int direct;            // 1: a direct pruned DFT per line (L <= kLineDftMax) from a table
};
// Fills L, n_pass, radix_codes and nl; -1 if L is not 2,3,5-smooth or exceeds kLineFftMax.
int line_fft_plan(int L, LineFft& p);
size_t line_fft_lds_bytes(const LineFft& p);  // dynamic LDS of a launch
// Load position of each input index of a planned length (p.L ints): the digit
// reversal the in-place passes need.
void line_fft_perm(const LineFft& p, int* perm);
// The passes' twiddles of a planned length (2 (p.L - 1) floats, complex64).
void line_fft_twiddles(const LineFft& p, float* tw);
hipError_t launch_line_fft(const LineFft& p, const void* in, const float* inv_psi, const int* perm, const float2* tw,
                           void* out, hipStream_t s);
hipError_t launch_transpose_c64(const void* in, int64_t rows, int64_t cols, void* out, hipStream_t s);
// Table of the direct pruned DFT of a line of p.L points from p.n_in stored
// inputs to the p.win_len kept outputs (complex64 [n_in][win_len], host):
// exp(+2 pi i f m / L) times inv_psi[i], f the input's frequency, m the output position.
void line_dft_table(const LineFft& p, const float* inv_psi, float* tab);
// Whether a planned line (with n_in and the window set) fits the direct DFT kernel.
bool line_dft_fits(const LineFft& p);
hipError_t launch_line_dft(const LineFft& p, const void* in, const float2* tab, void* out, hipStream_t s);
hipError_t launch_nufft_corr(const NufftGeom& g, const double* pix, int64_t pix_ld, int64_t n_pix, const double* quad_t,
                             const double* quad_wphi, int n_quad, double* corr, hipStream_t s);
hipError_t launch_fill_zero_f64(double* p, int n, hipStream_t s);
// Image-domain partitions of a NUFFT plan: out[p + d n] = pix[idx[p] + d ld];
// images[l ld + idx[p]] += part_img[l n + p], then part_img = 0.
hipError_t launch_nufft_gather_pix(const double* pix, int64_t ld, const int64_t* idx, int64_t n, double* out,
                                   hipStream_t s);
hipError_t launch_nufft_scatter_images(float* part_img, int64_t n, int n_levels, const int64_t* idx, float* images,
                                       int64_t ld, hipStream_t s);
hipError_t launch_nufft_vprime(const NufftInst* insts, int n_inst, int max_ant, const void* Wmat, const float* d,
                               const int* order, const int* lstart, int n_levels, void* vp, hipStream_t s);
int nufft_tile_size(const NufftGeom& g);  // 16 or 8 grid points per tile side, 0 = no tiled path
// Exclusive prefix sum of n ints into offset[0..n] (and cursor[0..n-1] unless
// null); tmp: scan_tmp_ints(n) ints (may be null for n <= 65536).
int scan_tmp_ints(int n);
hipError_t launch_scan_i32(const int* count, int n, int* offset, int* cursor, int* tmp, hipStream_t s);
hipError_t launch_nufft_bin(const NufftGeom& g, const NufftInst* insts, int n_inst, int max_ant, const double* ant,
                            int64_t ld, int bin, int* count, int* offset, int* cursor, uint64_t* list, int* err,
                            int* scan_tmp, hipStream_t s);
// Output-driven spread (nufft_gather.hip) for grids with N2 <= 64: points of
// axis 2 per column (16, 32 or 64; 0 = not applicable) and column blocks.
int nufft_gather_z(const NufftGeom& g);
void nufft_gather_blocks(const NufftGeom& g, int& nbx, int& nby);
constexpr int kGatherRecBytes = 128;  // per sorted baseline
// After launch_nufft_bin with bin 1: records (max_src x 128 bytes), level values
// (max_src x ((n_levels + 1) & ~1) complex64), nparts and part_off (blocks,
// blocks + 1 ints), scan_tmp (scan_tmp_ints(blocks)).
hipError_t launch_nufft_spread_gather(const NufftGeom& g, const NufftInst* insts, int64_t max_src, const double* ant,
                                      int64_t ld, const void* vp, const int* offset, const uint64_t* list,
                                      int n_levels, void* rec, void* cv, int* nparts, int* part_off, int* scan_tmp,
                                      float* grid, int64_t n_cell, hipStream_t s);
// nch, choff: n_tiles and n_tiles + 1 ints of scratch (chunks per tile and their offsets).
hipError_t launch_nufft_spread_tiles(const NufftGeom& g, const NufftInst* insts, const double* ant, int64_t ld,
                                     const void* vp, const int* offset, const uint64_t* list, int bin, int n_levels,
                                     int* nch, int* choff, float* grid, int64_t n_cell, hipStream_t s);

// Backward.
// E recompute (FP32 MFMA, three-product form, one instance staged as three
// planes) into two planes [2][K_alloc][n_pix].
hipError_t launch_fields(const FwdParams& p, int K_alloc, hipStream_t s);
int fields_tile_pixels(int K_alloc);

struct BwdParams {
  const double* pix; int64_t pix_ld; int64_t n_pix;
  const InstDesc* desc; const InstDyn* dyn;
  const float* gimg; int64_t gimg_ld;   // upstream gradient [n_levels][gimg_ld]
  float* E;                             // [2][K_alloc][n_pix], overwritten by M = d c conj(E)
  int K_alloc, L_pad, L, K;
  const void* W;                        // caller's W (complex64, L x K column-major)
  int n_split;                          // pixel splits of the contractions over pixels
  int64_t split_len;                    // pixels per split (multiple of 64)
  double* dd_part;                      // [K_alloc][n_split]
  double* dW_part;                      // [n_split][L_pad][K_alloc][2]
  double* dx_part;                      // [n_split][L_pad][3]
  double scale_x;                       // -(4 pi / wavelength)
};
hipError_t launch_backward(const BwdParams& p, hipStream_t s);
hipError_t launch_backward_reduce(const BwdParams& p, void* dW, float* dd, double* dx, hipStream_t s);

}  // namespace bb
