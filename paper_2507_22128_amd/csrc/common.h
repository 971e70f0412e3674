// Shared definitions of the HIP imager library (internal header).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/imager.h"

namespace imgr {

// ----------------------------------------------------------------- complex

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// real type of a complex vector type, and a constructor
template <class C> struct Real;
template <> struct Real<float2> { typedef float T; };
template <> struct Real<double2> { typedef double T; };
template <class C>
__device__ __forceinline__ C mkc(typename Real<C>::T re, typename Real<C>::T im) {
  C c;
  c.x = re;
  c.y = im;
  return c;
}

// twiddle table: tw[m] = exp(-2 pi i m / kTwMax), FP64-computed, f32-stored
constexpr int kTwMax = 16384;

// ----------------------------------------------------------------- handle

// Visibilities of one partition binned for one grid: sorted by the
// blk x blk block of grid cells that holds the first tap of their footprint
// shifted by W/2 - 1, then by the row and column of that tap inside the
// block, and cut into chunks of at most C visibilities of one block.  Every footprint of a
// block lies in a 16 x 16 window of the grid whose origin is the block origin
// minus W/2 - 1.
// Grid cells the chunk windows of a partition cover: columns [x0, x1)
// (multiples of 64), rows [y0, y1) (multiples of 16).  The de/gridding reads
// and the flush writes nothing outside, so the transforms skip the rest.
// The whole grid when some window wraps around the grid's edge.
struct Box {
  int x0 = 0, x1 = 0, y0 = 0, y1 = 0;
};

struct Bins {
  int64_t n = 0;               // members
  int n_chunks = 0;
  int ng = 0;                  // grid side the positions refer to
  int nb = 0;                  // blocks per grid side (ng / blk)
  float4 *posvis = nullptr;    // [n] {dx, dy, re, im}: offsets from the block origin, visibility
  float *w = nullptr;          // [n] imaging weight
  int32_t *orig = nullptr;     // [n] original index
  int32_t *outpos = nullptr;   // [n] member rank (position in member order)
  int32_t *chunk_block = nullptr;  // [n_chunks] block of each chunk
  int32_t *chunk_begin = nullptr;  // [n_chunks + 1]
  int32_t *chunk_rows = nullptr;   // [n_chunks][8] visibilities of the chunk with row <= j
  int32_t *block_chunk = nullptr;  // [nb * nb + 1] first chunk of each block
  int32_t *order = nullptr;        // [n_chunks] launch order: largest chunk first
  Box box;                         // cells the chunk windows cover
};

// work buffers of one node's major cycle
struct Work {
  float2 *grid_a = nullptr;   // Ng^2 (model grid, residual grid)
  float2 *grid_b = nullptr;   // Ng^2 (transform scratch)
  float2 *rows = nullptr;     // N x Ng (row-pass intermediate)
  float2 *scratch = nullptr;  // [n_chunks][16][16] chunk windows
  float *img = nullptr;       // N^2 (node-local residual)
};

// device work area of one node's multi-scale CLEAN (kept between calls)
struct CleanWork {
  double *R = nullptr;       // [n_int][N^2] smoothed residuals
  double *B = nullptr;       // [n_pairs][(2N)^2] cross PSFs
  double *kern = nullptr;    // scale kernels and their pairwise convolutions
  double *model = nullptr;   // N^2
  void *state = nullptr;     // loop state
  void *slots = nullptr;     // per-block peak candidates
  size_t R_elems = 0, B_elems = 0, k_elems = 0;
};

// device work area of one node's FISTA (kept between calls; FP64)
struct FistaWork {
  double *alpha_prev = nullptr, *y = nullptr, *coef = nullptr;   // P N^2 coefficients
  double *tmp = nullptr, *xb = nullptr;  // P N^2 transform work (xb: dictionaries only)
  double *x = nullptr, *u1 = nullptr, *u2 = nullptr, *u3 = nullptr;  // N^2 images
  double *cst = nullptr;                                         // N^2
  double *d64 = nullptr, *r64 = nullptr;                         // inputs in FP64
  double2 *work64 = nullptr, *tmp64 = nullptr;                   // transform buffers
  double2 *psf_ext = nullptr;  // spectrum of a caller's PSF (4 N^2, on first use)
  double *scal = nullptr;    // device scalars (L_hat, lambda, norms)
  double *part = nullptr;    // reduction partials
  double *hlo = nullptr;     // wavelet filters (low, high) of every basis, concatenated
  std::vector<int> taps, hoff;  // per basis: filter length, offset in hlo
  int vanishing = 0, n_bases = 0;
  size_t n = 0;
};

struct Partition {
  double sum_w = 0.0;
  Bins bins;                   // on the Ng grid (major cycle, degrid, grid)
  Bins psf_bins;               // on the 2 Ng grid of the 2N x 2N PSF (freed after create)
  float *psf = nullptr;        // (2N)^2 normalised PSF, centre (N, N)
  float2 *psf_hat = nullptr;   // (2N)^2 plain DFT of psf
  double2 *psf_hat64 = nullptr;  // the same in FP64 (built on first use)
};

}  // namespace imgr

struct imgr_s {
  // geometry
  int N = 0, Ng = 0, W = 8, blk = 8, n_parts = 1, C = 1024;
  int device = 0;  // the device current at imager_create
  double cell = 0, beta = 0, ell = 0, delta = 1;
  int weighting = 0;
  int64_t n_valid = 0;
  hipStream_t stream = nullptr;
  imgr::Partition part[2];
  // tables
  float *cinv = nullptr;       // [N]  1 / psi_hat, N image on the Ng grid
  float *cinv2 = nullptr;      // [2N] 1 / psi_hat, 2N image on the 2 Ng grid
  float2 *tw = nullptr;        // [kTwMax]
  double2 *tw64 = nullptr;     // [kTwMax], FP64
  float2 *twrow = nullptr;     // [2 kTwMax]: entry L + m = w_L^m (row passes)
  double2 *twrow64 = nullptr;  // the same in FP64
  // per-node work buffers and streams: the two nodes' major cycles may run
  // concurrently (imager_major_cycle_nodes)
  imgr::Work work[2];
  imgr::CleanWork clean[2];
  imgr::FistaWork fista[2];
  // per-node images of the reconstruction loop: composed dirty (N^2),
  // composed PSF ((2N)^2), deconvolved residual (N^2)
  float *loop_dirty[2] = {nullptr, nullptr};
  float *loop_psf[2] = {nullptr, nullptr};
  float *loop_delta[2] = {nullptr, nullptr};
  hipStream_t node_stream[2] = {nullptr, nullptr};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[2] = {nullptr, nullptr};
  // the PSF terms of Eq. 7 of both nodes depend only on the cycle's inputs:
  // imager_major_cycle_nodes runs their fronts on a stream of their own,
  // into psf_work[p] (N x 2N complex, tmp (2N)^2)
  hipStream_t psf_stream = nullptr;
  hipEvent_t ev_psf[2] = {nullptr, nullptr};
  hipEvent_t ev_win = nullptr;  // end of node V_L's de/gridding
  hipEvent_t ev_psf_join = nullptr;
  float2 *psf_work[2] = {nullptr, nullptr};
  float2 *psf_tmp = nullptr;
  // stage timing (imager_set_timing): one set of events per recorded cycle
  bool timing = false;
  std::vector<std::vector<hipEvent_t>> ev_sets;
  std::vector<hipEvent_t> ev_pool;
  // work layout autotuner (create time): candidates tried and their times
  bool tune = false;
  int tile_fixed = 0, chunk_fixed = 0;  // nonzero: not tuned
  struct TuneEntry {
    int blk, C;
    float ms;
  };
  std::vector<TuneEntry> tune_log;
  size_t scratch_chunks[2] = {0, 0};  // capacity of work[p].scratch in chunk windows
  uint64_t layout_version = 0;        // bumped whenever chunk tables or scratch change
  // bookkeeping
  std::vector<void *> allocs;
  std::vector<size_t> alloc_sizes;
  size_t bytes = 0, budget = 0, peak_bytes = 0;
  // during imager_create: freed blocks kept for reuse (pointer, bytes)
  bool caching = false;
  std::vector<std::pair<void *, size_t>> cache;
  size_t cached_bytes = 0;
  double create_ms = 0;
  bool broken = false;
  std::string err;
};

namespace imgr {

// ----------------------------------------------------------------- errors

struct Error {
  imgr_status code;
  std::string msg;
};

#define IMGR_HIP(expr)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::imgr::Error{IMGR_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define IMGR_CHECK(cond, msg)                                   \
  do {                                                          \
    if (!(cond)) throw ::imgr::Error{IMGR_EINVAL, (msg)};       \
  } while (0)

// device allocation accounted against the handle's budget
void *dev_alloc(imgr_s *h, size_t bytes);
void dev_free(imgr_s *h, void *p);

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// ----------------------------------------------------------------- prep (a0)
void prep_build(imgr_s *h, const imgr_vis *vis);
void free_bins(imgr_s *h, Bins &B);
// rechunk every partition of h for cap C (imager_set_chunk)
void set_chunk(imgr_s *h, int C);
// one node's major cycle: its arguments, and the index of its stage-event set
// (-1 without timing)
struct NodeCall {
  int part;
  const float *model, *rho_other;
  double gamma, mu;
  float *residual_out, *local;
  int flags;
  hipStream_t s;
  int ev_set;
  bool psf_pre;  // the PSF term's front already enqueued (compose_psf_front)
};
NodeCall node_begin(imgr_s *h, int part, const float *model, const float *rho_other,
                    double gamma, double mu, float *residual_out, float *residual_local_out,
                    int flags, hipStream_t s);
// enqueue stage 0 .. IMGR_N_STAGES - 1 of the cycle (model transform,
// de/gridding, flush, inverse transform, composition)
void node_stage(imgr_s *h, const NodeCall &c, int stage);
// one node's major cycle enqueued on s (imager_major_cycle)
void node_cycle(imgr_s *h, int part, const float *model, const float *rho_other, double gamma,
                double mu, float *residual_out, float *residual_local_out, int flags,
                hipStream_t s);
// device time (ms) of one degrid / grid launch plus flush over bins B
float time_layout(imgr_s *h, const Bins &B, float2 *grid, float2 *scr, int reps, hipStream_t s);
// chunk indices in decreasing chunk size, ties in index order (cb: chunk
// starts with the closing entry)
std::vector<int32_t> largest_first(const std::vector<int32_t> &cb);
// support W for a target relative accuracy on a 2x padded grid: the
// smallest built support with 3 x 10^(1 - W) <= tol, or 0 if none
int support_for_tolerance(double tol);

// ----------------------------------------------------------------- FFT
// centred forward transform of an N x N real image (times 1/psi_hat on both
// axes, plus optional second image) into the Ng x Ng grid `out`
// (box: the grid cells the following de/gridding reads; nothing else is formed)
void fft_model_to_grid(imgr_s *h, const float *model, const float *model_add, const float *cinv,
                       int n, int ng, float2 *rows, float2 *tmp, float2 *out, const Box &box,
                       hipStream_t s);
// centred inverse transform of the Ng x Ng grid `in` (already multiplied by
// (-1)^(gx+gy)) cropped to N x N, times (-1)^(px+py)/psi_hat^2 * scale, real part
// One member's model and residual transforms in a batched launch (members of
// one grid side Ng and image side N): model -> rows -> tmp -> grid on the
// model side, grid -> tmp -> rows -> image on the residual side, over the
// member's covered box.
struct FftMember {
  const float *model;  // N x N model image
  float *image;        // N x N residual image
  float2 *rows, *tmp, *grid;
  const float *cinv;   // gridding correction (N)
  float scale;         // residual image scale (1 / sum of weights)
  int x0, x1, y0, y1;  // covered box
};
// the model / residual transforms of `count` members (device table) in one
// launch per pass; max_cb: the most 64-column blocks of any member's box;
// h supplies the twiddle tables (equal for every handle)
void fft_model_to_grid_batch(const imgr_s *h, int ng, int n, const FftMember *members, int count,
                             int max_cb, hipStream_t s);
void fft_grid_to_image_batch(const imgr_s *h, int ng, int n, const FftMember *members, int count,
                             int max_cb, hipStream_t s);
// (box: the cells of `in` that the flush wrote; the rest is taken as zero)
void fft_grid_to_image(imgr_s *h, const float2 *in, const float *cinv, int n, int ng, float scale,
                       float2 *rows, float2 *tmp, float *out, const Box &box, hipStream_t s);
// out (+)= Re F_N^-1 (Gamma_own . F_N (a - b)) * coef for N x N images
// (b may be NULL; plain DFTs; own_low: bit 0 set = Gamma_L, else Gamma_H;
// bit 1 set = the filter squared);
// work holds N x L and tmp L x L complex values (L = N here, 2N below)
void image_gamma(imgr_s *h, const float *a, const float *b, int own_low, float coef, float *out,
                 int accumulate, float2 *work, float2 *tmp, hipStream_t s);
// out (+)= coef * (psf * a), the linear convolution of the N x N image a by
// the 2N x 2N PSF with spectrum psf_hat (centre (N, N)), cropped to N x N
void image_psf_conv(imgr_s *h, const float *a, const float2 *psf_hat, float coef, float *out,
                    int accumulate, float2 *work, float2 *tmp, hipStream_t s);
// out = gamma Gamma_own a (own_low as in image_gamma, bit 0 only): Gamma_H a
// is formed as gamma a - gamma Gamma_L a, whose spectral factor vanishes
// beyond (ell + delta), so only those column blocks are transformed
void image_gamma_scaled(imgr_s *h, const float *a, int own_low, float gamma, float *out,
                        float2 *work, float2 *tmp, hipStream_t s);
// its two parts, for callers that run them on different streams: the front
// leaves N rows of 2N complex values in work (tmp: (2N)^2 complex), the back
// (+)= them into out
void image_psf_conv_front(imgr_s *h, const float *a, const float2 *psf_hat, float coef,
                          float2 *work, float2 *tmp, hipStream_t s);
void image_psf_conv_back(imgr_s *h, const float2 *work, float *out, int accumulate,
                         hipStream_t s);
// FP64 versions of the two filters (work: N x 2N, tmp: (2N)^2 double2)
void image_gamma64(imgr_s *h, const double *a, const double *b, int own_low, double coef,
                   double *out, int accumulate, double2 *work, double2 *tmp, hipStream_t s);
void image_psf_conv64(imgr_s *h, const double *a, const double2 *psf_hat, double coef, double *out,
                      int accumulate, double2 *work, double2 *tmp, hipStream_t s);
// two FP64 Gamma filters (own_low, coef, accumulate as in image_gamma64) of
// different images in one launch per pass; work: 2 N^2, tmp: 2 N^2 double2
void image_gamma64_pair(imgr_s *h, const double *a0, int own0, double coef0, double *out0,
                        int acc0, const double *a1, int own1, double coef1, double *out1,
                        int acc1, double2 *work, double2 *tmp, hipStream_t s);
// plain FP64 2-D DFT of an n x n complex buffer in place
void fft2_plain64(imgr_s *h, double2 *buf, double2 *tmp, int n, int dir, hipStream_t s);
// the partition's FP64 PSF spectrum (built on first use, kept)
const double2 *psf_spectrum64(imgr_s *h, int p, hipStream_t s);
// FP64 spectrum of a caller's 2N x 2N float32 PSF into out (4 N^2), tmp of the same size
void psf_spectrum64_of(imgr_s *h, const float *psf, double2 *out, double2 *tmp, hipStream_t s);
// plain 2-D DFT of an n x n complex buffer in place (dir -1 forward, +1 inverse, unnormalised)
void fft2_plain(imgr_s *h, float2 *buf, float2 *tmp, int n, int dir, hipStream_t s);

// ----------------------------------------------------------------- de/gridding
enum GridMode { MODE_DEGRID_GRID = 0, MODE_GRID = 1, MODE_DEGRID = 2, MODE_PSF = 3 };
constexpr int kWin = 16;  // window side (cells) of a block's footprints
// one chunk pass over bins b: grid_in is the model grid (modes 0, 2),
// vis_in member-order visibilities (mode 1), vis_out member-order
// predictions (mode 2); every gridding mode writes one window per chunk
// to scratch ([n_chunks][16][16])
void degrid_grid(imgr_s *h, const Bins &b, int mode, const float2 *grid_in, const float2 *vis_in,
                 float2 *vis_out, float2 *scratch, hipStream_t s);
// deterministic flush of the chunk windows into the b.ng x b.ng grid, with (-1)^(x+y)
void flush_chunks(imgr_s *h, const Bins &b, const float2 *scratch, float2 *grid_out,
                  hipStream_t s);
// whether kernels exist for support W with blocks of blk cells
bool window_supported(int W, int blk);

// arguments of the window kernel for one grid (one partition's bins)
struct WinArgs {
  const float4 *posvis;
  const float *wts;
  const int32_t *outpos;
  const int32_t *chunk_block;
  const int32_t *chunk_begin;
  const int32_t *chunk_rows;
  int n;  // visibilities in the stream
  int nb, ng;
  float bl2e;
  const float2 *grid_in;
  const float2 *vis_in;
  float2 *vis_out;
  float2 *scratch;
};
// arguments of the flush of one grid
struct FlushArgs {
  const float2 *scratch;
  const int32_t *block_chunk;
  int nb, ng;
  float2 *grid_out;
  int gx0, gy0, gnx;  // 16 x 16 cell groups of the box: first column, first row, per row
};
FlushArgs flush_args(const Bins &B, const float2 *scratch, float2 *grid_out);
// 16 x 16 cell groups of the flush of bins B
inline int flush_groups(const Bins &B) {
  return ((B.box.x1 - B.box.x0) / 16) * ((B.box.y1 - B.box.y0) / 16);
}
WinArgs win_args(const imgr_s *h, const Bins &B, const float2 *grid_in, const float2 *vis_in,
                 float2 *vis_out, float2 *scratch);
// fused degrid / residual / grid over the chunks of many grids: order[i] =
// (grid, chunk) with grids[] device descriptors; all grids share W and blk
void degrid_grid_batch(int W, int blk, const WinArgs *grids, const int2 *order, int n_slots,
                       hipStream_t s);
// flush of many grids: grid g owns workgroups [group_start[g], group_start[g+1])
void flush_batch(int W, int blk, const FlushArgs *grids, const int32_t *group_start, int n_grids,
                 int n_groups, hipStream_t s);
// rebuild the chunk tables of bins B for a new chunk cap C (the sort stays)
void rechunk(imgr_s *h, Bins &B, int C, hipStream_t s);

// ----------------------------------------------------------------- composition
// Eq. 7 for node p on stream s; with psf_pre, the PSF term's front was
// enqueued by compose_psf_front and only its back runs here (after ev_psf[p])
void compose(imgr_s *h, int p, const float *resid, const float *rho_other, double gamma, double mu,
             float *out, bool psf_pre, hipStream_t s);
// the front of node p's PSF term, mu H_other rho_other, into psf_work[p] on
// stream s, then ev_psf[p] recorded on s
void compose_psf_front(imgr_s *h, int p, const float *rho_other, double mu, hipStream_t s);
void composed_psf(imgr_s *h, int p, double gamma, double mu, float *out, hipStream_t s);
void exchange(imgr_s *h, const float *a, const float *b, float *rho_a, float *rho_b, hipStream_t s);
void combine_final(imgr_s *h, const float *a, const float *b, double wa, double wb, double *out,
                   hipStream_t s);
void psf_spectrum(imgr_s *h, int p, hipStream_t s);

// ----------------------------------------------------------------- minor cycles
// multi-scale CLEAN of node `part`, enqueued on stream s; msclean_count
// (after s has completed) returns the number of components it took
void msclean_enqueue(imgr_s *h, int part, const imgr_msclean_params &prm, const float *dirty,
                     const float *psf, float *model_delta, float *model_accum, float *resid_out,
                     imgr_component *comps, hipStream_t s);
int msclean_count(imgr_s *h, int part);
// bytes of the static work area a call with these parameters needs
size_t msclean_static_bytes(const imgr_s *h, const imgr_msclean_params &prm);
// the same minor cycle on the device's static work area (nothing is
// allocated); synchronises s and returns the number of components
int msclean_enqueue_static(imgr_s *h, const imgr_msclean_params &prm, const float *dirty,
                           const float *psf, float *model_delta, float *model_accum,
                           float *resid_out, imgr_component *comps, hipStream_t s);
uint32_t msclean_own_scales(const imgr_s *h, int part, const imgr_msclean_params &prm);
void msclean_release(imgr_s *h, int part);

// sparsity-regularised minor cycle of node `part` (Eqs. 4, 5), enqueued on s
// (psf: a caller's 2N x 2N PSF for H, or NULL for the node's own)
void fista_enqueue(imgr_s *h, int part, const imgr_fista_params &prm, const float *dirty,
                   const float *psf, const float *rho_other, const float *power_start,
                   float *model_delta, float *model_accum, double *objective, hipStream_t s);
// (after s has completed) the step constant L_hat and lambda of the last run
void fista_scalars(imgr_s *h, int part, double *lipschitz, double *lambda);

// ----------------------------------------------------------------- misc kernels
void add_images(const float *a, const float *b, float *out, int64_t n, hipStream_t s);

}  // namespace imgr
