/*
 * imager.h - C-ABI of the MI355X (gfx950) major-cycle imager.
 *
 * Hot path of the spatial-frequency-decentralized reconstruction of
 * Wang et al., "A Decentralized Framework for Radio-Interferometric Image
 * Reconstruction" (arXiv 2507.22128): for one node (visibility partition)
 * the major-cycle residual of Eq. 2, i~ = F^dagger G (v - G^dagger F i^),
 * its PSF H, and the pseudo-full-resolution composition of Eq. 7
 * (Section 4.2), with the partition of Fig. 3 (Section 3), uniform
 * weighting (Section 5.1), the aggregate update of Eq. 5 (Section 4.1) and
 * the final combination (Section 5.2).
 *
 * Conventions used by every call (they are readings of passages the paper
 * leaves silent):
 *   - images are N x N float32, row-major [iy][ix]; pixel (ix, iy) has
 *     direction cosines l = (ix - N/2) cell, m = (iy - N/2) cell;
 *   - the forward operator is (A x)_k = sum_p x_p exp(-2 pi i (u_k l_p +
 *     v_k m_p)) (Eq. 1 with the C, D, w and 1/n terms dropped, as the text
 *     after Eq. 1 allows), approximated by gridding with the
 *     exponential-of-semicircle kernel of support W on a 2x padded grid;
 *   - residual / dirty images are Re A^H (w . r) / sum(w); the PSF is
 *     Re A'^H (w) / sum(w) on a 2N x 2N image with the same pixel size,
 *     centred at pixel (N, N);
 *   - "members" of a partition are its visibilities in increasing order of
 *     their index in the array given to imager_create.
 *
 * Memory and streams: every pointer argument documented "device" must be
 * device memory of the handle's device (e.g. a torch tensor's data
 * pointer); "host" pointers are ordinary host memory.  The caller owns all
 * memory it passes; the library never frees it.  imager_create copies,
 * sorts and bins the visibilities into library-owned device memory, so the
 * caller may free its arrays when it returns.  All library allocations are
 * released by imager_destroy.  Calls other than create, destroy, info and
 * last_error only enqueue work on the handle's stream and return; results
 * are valid after imager_sync or any later synchronisation of that stream.
 *
 * Errors: every call returns an imgr_status.  EINVAL: bad arguments,
 * nothing enqueued.  ENOMEM: the device footprint would exceed
 * hbm_budget, or hipMalloc failed; the handle is unchanged.  EDEVICE: a HIP
 * runtime error; the handle then refuses further work with ESTATE until it
 * is destroyed.  imager_last_error returns a message for the last failure.
 * A handle must not be used by two host threads at once; different handles
 * are independent.
 */
#ifndef IMAGER_H
#define IMAGER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct imgr_s *imgr_t;

typedef enum {
  IMGR_OK = 0,
  IMGR_EINVAL = 1,
  IMGR_ENOMEM = 2,
  IMGR_EDEVICE = 3,
  IMGR_ESTATE = 4,
  IMGR_ENOTIMPL = 5
} imgr_status;

/* visibility element types (interleaved re, im) */
enum { IMGR_C64 = 0, IMGR_C128 = 1 };

/* imgr_config.weighting */
enum { IMGR_WEIGHT_NATURAL = 0, IMGR_WEIGHT_UNIFORM = 1 };

/* partition indices; with n_partitions == 1 only IMGR_PART_LOW (= all) exists */
enum { IMGR_PART_LOW = 0, IMGR_PART_HIGH = 1 };

/* imgr_config.flags and imager_major_cycle flags */
enum {
  /* degrid model + rho_other instead of model (the "local model plus the
     other partition's previous image" form); default degrids model alone */
  IMGR_DEGRID_COMPOSITE = 1
};

/* imager_grid modes */
enum { IMGR_GRID_DIRTY = 0, IMGR_GRID_UNNORMALIZED = 1 };

/* imager_combine_partitions modes */
enum { IMGR_COMBINE_EXCHANGE = 0, IMGR_COMBINE_FINAL = 1 };

typedef struct {
  int32_t n_pix;        /* N: power of two, 64 <= N <= 2048 */
  double cell_rad;      /* pixel size in radians (> 0) */
  int32_t support;      /* W: 4, 6, 8, 10 or 12; 0 selects 8 */
  double es_beta;       /* ES kernel beta; <= 0 selects 2.30 W */
  int32_t weighting;    /* IMGR_WEIGHT_* */
  int32_t n_partitions; /* 1 (serial) or 2 (V_L, V_H) */
  double ell_pix;       /* partition radius ell in Fourier pixels; < 0: lower median */
  double delta_pix;     /* half-width of the overlap ring; <= 0 selects 1 */
  int32_t tile;         /* block side in grid cells, 4 or 8, with tile + support - 1
                           <= 16; 0 selects 8 for support <= 8, else 4 */
  int32_t chunk;        /* max visibilities per work chunk, >= 16; 0 selects 1024 */
  int32_t flags;        /* reserved, 0 */
  size_t hbm_budget;    /* bytes of device memory the handle may hold; 0 = no cap */
  void *stream;         /* hipStream_t for all work; NULL = the null stream */
  int32_t autotune;     /* 1: choose tile and chunk (those left 0) at create by
                           timing one degrid / grid launch plus flush of the
                           first partition for every candidate (imager_tune_log) */
  double tolerance;     /* > 0 with support == 0: support = the smallest built W
                           with 3 x 10^(1 - W) <= tolerance.  The relative error
                           of the exponential-of-semicircle kernel with beta =
                           2.30 W on a 2x padded grid falls by about a decade per
                           tap (Barnett, Magland and af Klinteberg 2019), and is
                           1.0 - 2.3 x 10^(1 - W) for W = 4 .. 12 against the
                           direct sum; EINVAL if no built support reaches it */
} imgr_config;

typedef struct {
  int64_t n_vis;        /* number of visibilities */
  double freq_hz;       /* observing frequency; u = uvw * freq / c */
  const double *uvw;    /* [n_vis][3] metres */
  const void *vis;      /* [n_vis] complex, element type vis_dtype */
  int32_t vis_dtype;    /* IMGR_C64 or IMGR_C128 */
  const float *weight;  /* [n_vis] natural weights, or NULL for all ones */
  const uint8_t *flag;  /* [n_vis], nonzero = flagged (dropped), or NULL */
  int32_t on_device;    /* 0: the five arrays are host memory; 1: device */
} imgr_vis;

typedef struct {
  int32_t n_pix, n_grid, support, tile, n_partitions;
  double cell_rad, es_beta, ell_pix, delta_pix;
  int64_t n_valid;      /* unflagged visibilities */
  int64_t n_vis[2];     /* members per partition (overlap counted in both) */
  int64_t n_chunks[2];  /* work chunks per partition */
  double sum_w[2];      /* summed imaging weights per partition (FP64) */
  size_t device_bytes;  /* device memory held by the handle */
  double create_ms;     /* wall time of imager_create */
  int32_t chunk;        /* max visibilities per work chunk (after tuning) */
  size_t device_peak_bytes; /* most device memory the handle has held at once */
} imgr_info;

/* Device-memory footprint of a handle before it is built, for admission
 * control: *resident (host) receives an upper estimate of device_bytes after
 * imager_create plus the reconstruction loop's buffers and the minor-cycle
 * work areas (multi-scale CLEAN with n_scales scales if n_scales > 0, FISTA
 * over a dictionary of `fista` bases if fista > 0), *peak (host, may be
 * NULL) one of device_peak_bytes, which
 * adds the temporaries of imager_create (host-staged inputs if vis_on_host,
 * sort and binning buffers, the PSF grid, the autotuner's trials).  With
 * two partitions and ell_pix < 0 (median split) each partition is taken to
 * hold at most 60 % of the visibilities, with ell_pix >= 0 all of them. */
imgr_status imager_footprint(const imgr_config *cfg, int64_t n_vis, int32_t vis_on_host,
                             int32_t n_scales, int32_t fista, size_t *resident, size_t *peak);

/* Build a handle: scale (u, v) in FP64, drop flagged visibilities, apply the
 * weighting, split into V_L = {rho <= ell + delta} and V_H = {rho >= ell -
 * delta} (Fig. 3; rho = |uv| in Fourier pixels), sort each partition by uv
 * block, and grid each partition's PSF once.  Synchronous.  *out receives
 * the handle (NULL on error). */
imgr_status imager_create(const imgr_config *cfg, const imgr_vis *vis, imgr_t *out);

imgr_status imager_destroy(imgr_t h);

imgr_status imager_info(imgr_t h, imgr_info *out);

/* Original indices (int64, host) of the members of partition part, in
 * member order: idx[n_vis[part]].  Synchronous. */
imgr_status imager_vis_index(imgr_t h, int32_t part, int64_t *idx);

/* Imaging weights (float32, host) of the members in member order. Synchronous. */
imgr_status imager_vis_weight(imgr_t h, int32_t part, float *w);

/* Degridding G^dagger F of Eq. 2: predicted visibilities of the N x N
 * model (device float32) at the members of partition part, written as
 * complex64 (device, [n_vis[part]], member order). */
imgr_status imager_degrid(imgr_t h, int32_t part, const float *model, void *vis_out);

/* Gridding F^dagger G of Eq. 2 of member visibilities vis_in (device
 * complex64, member order): image_out (device N x N float32) receives
 * Re A^H (w . vis) / sum(w) (IMGR_GRID_DIRTY) or without the division
 * (IMGR_GRID_UNNORMALIZED). */
imgr_status imager_grid(imgr_t h, int32_t part, const void *vis_in, float *image_out,
                        int32_t mode);

/* The partition's PSF (Section 2, operator H of Eqs. 4, 5, 7): 2N x 2N
 * float32 (device), normalised to peak 1 at pixel (N, N). */
imgr_status imager_psf(imgr_t h, int32_t part, float *psf_out);

/* One major cycle of node `part` (Eq. 2 then Eq. 7):
 *   residual_local = Re A^H (w . (v - A model)) / sum(w)      (Eq. 2)
 *   residual_out   = gamma Gamma_own residual_local + mu H_other rho_other
 * with Gamma_own the node's filter (Gamma_L for IMGR_PART_LOW) and H_other
 * the other partition's PSF.  With one partition residual_out =
 * residual_local.  rho_other may be NULL (then the mu term is dropped).
 * model, rho_other: device N x N float32; residual_out: device N x N
 * float32; residual_local_out: device N x N float32 or NULL.
 * flags: IMGR_DEGRID_COMPOSITE degrids model + rho_other. */
imgr_status imager_major_cycle(imgr_t h, int32_t part, const float *model,
                               const float *rho_other, double gamma, double mu,
                               float *residual_out, float *residual_local_out,
                               int32_t flags);

/* The major cycles of all nodes at once (Section 4: the nodes of the
 * decentralized framework work concurrently between exchanges).  Each
 * array has one entry per partition (n_partitions entries); entry p has
 * the meaning of the same argument of imager_major_cycle for part = p, and
 * rho_other / residual_local_out may be NULL (all entries absent).  The
 * nodes run concurrently on library-owned streams with their own work
 * buffers (the PSF terms mu H_other rho_other of Eq. 7, which read only the
 * inputs, on a third one), forked from and joined back into the handle's
 * stream, so the call is ordered on that stream like any other.  Results equal those of
 * imager_major_cycle for each node, bit for bit.  Output buffers of
 * different nodes must not overlap. */
imgr_status imager_major_cycle_nodes(imgr_t h, const float *const *model,
                                     const float *const *rho_other, const double *gamma,
                                     const double *mu, float *const *residual_out,
                                     float *const *residual_local_out, int32_t flags);

/* Composed PSF of Eq. 7, gamma Gamma_own H_own + mu Gamma_other H_other,
 * 2N x 2N float32 (device). */
imgr_status imager_composed_psf(imgr_t h, int32_t part, double gamma, double mu,
                                float *psf_out);

/* Multi-scale CLEAN minor cycle (Eq. 6; Eq. 7 for a node of the
 * decentralized loop), after Cornwell's multi-scale CLEAN as the paper uses
 * it.  Scale functions phi_s: a unit impulse for s = 0, else the truncated
 * paraboloid 1 - (r/s)^2 on r < s normalised to unit sum.  With R_s =
 * phi_s * dirty and B_ab = phi_a * phi_b * psf (linear convolutions, zero
 * outside the image), each of at most max_iter iterations
 *   - stops if max |R_0| < threshold (R_0 the unsmoothed residual),
 *   - picks (s*, p*) = argmax of bias_s |R_s(p)| over the selectable scales,
 *     bias_s = 1 - bias_slope s / max(S); ties go to the smaller scale
 *     index, then the smaller flat pixel index iy N + ix,
 *   - takes alpha = gain R_{s*}(p*) / B_{s*s*}(0), adds alpha phi_{s*}
 *     centred at p* to the model, and subtracts alpha B_{s*t} shifted to p*
 *     from every R_t.
 * Everything that decides a peak is evaluated in FP64 on the device.
 * dirty: device N x N float32 (e.g. the composed residual of
 * imager_major_cycle); psf: device 2N x 2N float32 centred at (N, N)
 * (e.g. imager_composed_psf).  Outputs (device float32 N x N, each may be
 * NULL): model_delta = the deconvolved residual ibar of Eqs. 6 / 7;
 * model_accum += model_delta (the update of Eq. 3); residual_out = R_0
 * after the last component.  comps (device, max_iter entries, or NULL)
 * receives the components in order; *n_comps (host) their number.
 * The call keeps an FP64 work area per node in the handle (grown on
 * demand) and synchronises the handle's stream before it returns. */
#define IMGR_MAX_SCALES 8
typedef struct {
  int32_t n_scales;                /* |S|, 1 .. IMGR_MAX_SCALES */
  double scales[IMGR_MAX_SCALES];  /* scale radii in pixels, >= 0 (0: point) */
  uint32_t active_mask;            /* bit i: scale i selectable (psi^n); 0 = all */
  double gain;                     /* loop gain in (0, 1] */
  int32_t max_iter;                /* K >= 0 */
  double threshold;                /* absolute threshold on max |R_0| */
  double bias_slope;               /* small-scale bias slope, e.g. 0.6 */
  int32_t own_scales_only;         /* 1: further restrict to the scales present in
                                      the node's own domain (psi^1 of Eq. 7, reading:
                                      V_L: s >= N / (2 (ell + delta)), V_H:
                                      s <= N / (ell - delta), else the nearest) */
  int32_t first_cycle;             /* imager_reconstruct_msclean only: number of the
                                      first cycle it runs (0 or 1: a fresh loop);
                                      k > 1 continues a loop from the models and
                                      rho of its cycle k - 1, so cycles may be run
                                      one call at a time with the same results */
} imgr_msclean_params;

typedef struct {
  int32_t scale;                   /* index into imgr_msclean_params.scales */
  int32_t iy, ix;                  /* pixel of the component's centre */
  int32_t reserved;
  double amp;                      /* flux: the model gets amp * phi_scale there */
} imgr_component;

imgr_status imager_minor_cycle_msclean(imgr_t h, int32_t part, const imgr_msclean_params *params,
                                       const float *dirty, const float *psf, float *model_delta,
                                       float *model_accum, float *residual_out,
                                       imgr_component *comps, int32_t *n_comps);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * minor cycle of imager_minor_cycle_msclean, same arguments and same
 * results bit for bit, with its FP64 work area (smoothed residuals, cross
 * PSFs, model, kernels, peak candidates, loop state) taken from a fixed
 * device array of IMGR_MSCLEAN_STATIC_BYTES that the library holds on
 * every device it runs on until the process ends, instead of the handle's
 * work area grown on first use.  The call allocates nothing (no hipMalloc,
 * no hipFree).  It needs 8 (N^2 (n_int + 1) + 4 N^2 n_int (n_int + 1) / 2)
 * bytes plus about 80 KB, n_int = |S| (+ 1 if 0 is not in S): N = 512 with
 * 3 scales, or N = 256 with up to 5, fits; larger needs are refused with
 * EINVAL and nothing enqueued.  The handle's device must be current.
 * Every call on one device shares that device's array and leaves its
 * contents behind (each call clears what it needs): calls that overlap on
 * one device, from different threads or streams, race.  Synchronises the
 * handle's stream before returning. */
#define IMGR_MSCLEAN_STATIC_BYTES (64u << 20)
imgr_status imager_minor_cycle_msclean_static(imgr_t h, int32_t part,
                                              const imgr_msclean_params *params,
                                              const float *dirty, const float *psf,
                                              float *model_delta, float *model_accum,
                                              float *residual_out, imgr_component *comps,
                                              int32_t *n_comps);

/* The whole major/minor loop with multi-scale CLEAN (Section 4.2): for
 * cycle n = 1 .. n_cycles and every node k, concurrently,
 *   i~ = residual of model[k] on the node's visibilities            (Eq. 2)
 *   D, P = the composed dirty image and PSF with the other node's
 *          rho[k] and PSF, gamma = 1, mu = 0 at n = 1, else the
 *          partitions' shares of the summed imaging weights (reading) (Eq. 7)
 *   ibar = ms-CLEAN(D, P, psi^n, K), psi^1 = the node's own scales
 *   model[k] += ibar                                                 (Eq. 3)
 * then the exchange rho[0] += Gamma_H (ibar_H - ibar_L), rho[1] +=
 * Gamma_L (ibar_L - ibar_H) (Section 4.1), and finally final_image =
 * 0.5 model[0] + 0.5 model[1] in FP64 (Section 5.2).  With one partition
 * the loop is Eq. 2 -> ms-CLEAN(i~, H, S, K) -> Eq. 3 and final_image =
 * model[0].  model[k], rho[k]: device N x N float32, read and updated in
 * place (start from zeros for a fresh reconstruction; rho may be NULL with
 * one partition); final_image: device N x N float64.  n_comps (host,
 * n_cycles x n_partitions, row-major, or NULL) receives the components
 * taken per cycle and node.  params->active_mask limits every cycle's
 * scales; own_scales_only is ignored (psi is applied as above).
 * Synchronises the handle's stream before returning. */
imgr_status imager_reconstruct_msclean(imgr_t h, int32_t n_cycles,
                                       const imgr_msclean_params *params, float *const *model,
                                       float *const *rho, double *final_image,
                                       int32_t *n_comps);

/* Sparsity-regularised minor cycle of node `part` (Eq. 5; Eq. 4 with
 * serial = 1): with W the orthonormal periodized Daubechies synthesis
 * (vanishing moments p, 2p taps, `levels` levels, every coefficient in the
 * l1 term), H the node's PSF convolution and Gamma_own / Gamma_other the
 * filters of Section 4.1,
 *   min_alpha ||Gamma_own (dirty - H W alpha)||^2
 *             + gamma_n ||rho_other - Gamma_other W alpha||^2 + lambda ||alpha||_1
 * by n_iter FISTA iterations from alpha = 0 with the constant step 1 / L_hat,
 * L_hat = 2 x the largest eigenvalue of H Gamma_own^2 H + gamma_n
 * Gamma_other^2 estimated by power_iters power iterations from the image
 * power_start (any nonzero N x N image; Beck and Teboulle's method as the
 * paper uses it).  lambda = params->lambda if > 0, else lambda_frac *
 * max |dirty|.  dirty: the node's residual i~ of Eq. 2 (device N x N
 * float32); psf: the 2N x 2N PSF whose convolution is H (device float32,
 * centre (N, N), the layout imager_psf writes), or NULL for the node's own
 * PSF from imager_create; rho_other: the node's aggregate rho of Eq. 5
 * (device N x N float32, ignored when gamma_n = 0 or serial).  Outputs (device, each may
 * be NULL): model_delta (N x N float32) = W alpha, model_accum += it,
 * objective (float64 [n_iter]) = the objective after every iteration.
 * *lipschitz and *lambda_used (host, may be NULL) receive L_hat and lambda.
 * Synchronises the handle's stream before returning. */
typedef struct {
  int32_t vanishing;     /* Daubechies p, 1 .. 10 (8: the 16-tap db8) */
  int32_t levels;        /* wavelet levels, N >> levels >= 2 p */
  int32_t n_iter;        /* FISTA iterations >= 0 */
  int32_t power_iters;   /* power iterations >= 1 */
  double lambda;         /* > 0: absolute weight of the l1 term */
  double lambda_frac;    /* lambda <= 0: lambda = lambda_frac * max |dirty| */
  double gamma_n;        /* weight of the rho term (Eq. 5: 0 at the first cycle, else 1) */
  int32_t serial;        /* 1: Eq. 4 (Gamma_own = identity, no rho term) */
  int32_t first_cycle;   /* imager_reconstruct_fista only: as in imgr_msclean_params */
  int32_t dictionary;    /* 0: W is the one basis db_vanishing; 1: W is the concatenation of
                            the first `vanishing` Daubechies bases db_1 .. db_vanishing, each
                            scaled by 1 / sqrt(vanishing) (a tight frame, W W^T = I; the
                            dictionary of Section 5.1), alpha then has vanishing x N^2
                            coefficients */
} imgr_fista_params;

imgr_status imager_minor_cycle_fista(imgr_t h, int32_t part, const imgr_fista_params *params,
                                     const float *dirty, const float *psf,
                                     const float *rho_other, const float *power_start,
                                     float *model_delta, float *model_accum, double *objective,
                                     double *lipschitz, double *lambda_used);

/* The whole major/minor loop with the sparsity-regularised minor cycle
 * (Section 4.1): for cycle n = 1 .. n_cycles and every node k,
 * concurrently, i~ = the residual of model[k] (Eq. 2), lambda =
 * lambda_frac * max |i~| (or params->lambda if > 0), gamma_n = 0 at n = 1
 * and 1 afterwards (Eq. 5; params->gamma_n is ignored), ibar = W alpha
 * from imager_minor_cycle_fista with power_start[k], model[k] += ibar
 * (Eq. 3); then the exchange rho[0] += Gamma_H (ibar_H - ibar_L), rho[1]
 * += Gamma_L (ibar_L - ibar_H), and final_image = 0.5 model[0] + 0.5
 * model[1] in FP64 (Section 5.2).  With one partition: Eq. 4 every cycle
 * and final_image = model[0].  model, rho (device N x N float32, updated in
 * place; rho may be NULL with one partition), final_image (device N x N
 * float64); lipschitz, lambdas (host, n_cycles x n_partitions, or NULL).
 * Synchronises the handle's stream before returning. */
imgr_status imager_reconstruct_fista(imgr_t h, int32_t n_cycles, const imgr_fista_params *params,
                                     const float *const *power_start, float *const *model,
                                     float *const *rho, double *final_image, double *lipschitz,
                                     double *lambdas);

/* Exchange and combination between the two partitions (Section 4.1,
 * Fig. 2, Section 5.2).
 * IMGR_COMBINE_EXCHANGE: a = ibar_L^n, b = ibar_H^n (device N x N float32,
 *   the nodes' latest deconvolved residuals); out_a, out_b (device N x N
 *   float32) are the aggregates rho_H held by node L and rho_L held by node
 *   H, updated in place:
 *     out_a += Gamma_H (b - a)     (Phi_H - Gamma_H ibar_L)
 *     out_b += Gamma_L (a - b)     (Phi_L - Gamma_L ibar_H)
 * IMGR_COMBINE_FINAL: out_a (device N x N float64) = w_a a + w_b b computed
 *   in FP64 (the paper uses w_a = w_b = 0.5); out_b unused. */
imgr_status imager_combine_partitions(imgr_t h, int32_t mode, const float *a, const float *b,
                                      double w_a, double w_b, void *out_a, void *out_b);

/* Device-time accounting of imager_major_cycle, for benchmarks.  While
 * enabled, every major cycle records HIP events on the handle's stream
 * around its stages; imager_get_timing synchronises the stream, returns the
 * summed milliseconds per stage and the number of cycles since the last
 * get (or enable), and clears the sums.  Stages:
 *   0 model -> model grid (gridding correction, padding, forward FFT)
 *   1 fused degrid / residual / grid over the uv-block chunks
 *   2 flush of the chunk sub-grids into the residual grid
 *   3 residual grid -> residual image (inverse FFT, crop, correction)
 *   4 composition of Eq. 7 (or the copy for one partition) */
#define IMGR_N_STAGES 5
typedef struct {
  int64_t cycles;
  double ms[IMGR_N_STAGES];
} imgr_timing;

imgr_status imager_set_timing(imgr_t h, int32_t enable);
imgr_status imager_get_timing(imgr_t h, imgr_timing *out);

/* Candidates timed by the create-time autotuner (imgr_config.autotune):
 * entry i < *n has tile[i], chunk[i] and ms[i], the least device time in
 * milliseconds of one fused degrid / grid launch plus its flush on the
 * first partition with a zero model.  At most cap entries are written; *n
 * receives the number of candidates (0 without autotune).  Host arrays. */
imgr_status imager_tune_log(imgr_t h, int32_t cap, int32_t *tile, int32_t *chunk, float *ms,
                            int32_t *n);

/* Cut the work chunks of every partition again for cap `chunk` (>= 16)
 * from the existing sort: the same tables as imager_create with that
 * chunk, so results equal such a handle's bit for bit.  Synchronous. */
imgr_status imager_set_chunk(imgr_t h, int32_t chunk);

/* ------------------------------------------------------------------ batches
 * Frequency channels are the axis along which imaging work is usually
 * spread (Section 1); a batch runs the major cycles (Eq. 2) of many
 * single-partition handles, e.g. one per channel with its own image size,
 * cell and flags, with the de/gridding of many of them as one fused launch
 * over their chunks (largest chunks first across channels), one fused
 * flush, and the model / residual transforms of the members with one image
 * size as one launch per pass (imager_batch_set_bytes can split the members
 * into cache-sized sets, one fused launch each; imgr_batch_info.n_sets).  Members must have one partition, equal support and tile, and
 * one stream, on which the batch enqueues its work.  The caller owns the
 * members; they must outlive the batch.  The batch uses the members' work
 * buffers, so a member's own calls and batch calls must be ordered (they
 * are when issued from one thread: all go to the shared stream). */
typedef struct imgr_batch_s *imgr_batch_t;

/* imager_batch_major_cycle flags */
enum {
  IMGR_BATCH_GRAPH = 1, /* capture the cycle into a HIP graph once per distinct set of
                           model / residual pointers (or after a re-chunk) and replay it */
  IMGR_BATCH_LOOP = 2   /* per-member launches, one member after another (the
                           per-channel loop the fused form is compared with) */
};

typedef struct {
  int32_t n_members, support, tile, chunk;
  int64_t n_vis;        /* member visibilities over all members */
  int64_t n_chunks;     /* chunks of the fused launches */
  int32_t graph_ready;  /* 1 if a captured graph is held */
  int32_t n_sets;       /* consecutive member sets, one fused launch each (1 unless
                           imager_batch_set_bytes set a cache budget) */
} imgr_batch_info;

/* members: host array of n >= 1 handles.  Synchronous. */
imgr_status imager_batch_create(const imgr_t *members, int32_t n, imgr_batch_t *out);
imgr_status imager_batch_destroy(imgr_batch_t b);
imgr_status imager_batch_info(imgr_batch_t b, imgr_batch_info *out);

/* residual[i] (device N_i x N_i float32) = the residual image of Eq. 2 for
 * member i and model[i] (device N_i x N_i float32), equal bit for bit to
 * imager_major_cycle of that member alone, in every mode.  model, residual:
 * host arrays of n_members device pointers; residual buffers must not
 * overlap each other or any model. */
imgr_status imager_batch_major_cycle(imgr_batch_t b, const float *const *model,
                                     float *const *residual, int32_t flags);

/* Chunk-cap autotuner of the fused launch: for each caps[i] (>= 16) every
 * member is re-chunked (imager_set_chunk) and the fused degrid / grid
 * launch plus flush is timed (least of reps >= 1 runs, zero models);
 * ms[i] (host, may be NULL) receives the times, and the fastest cap is
 * applied to all members and returned in *chosen.  Synchronous. */
imgr_status imager_batch_autotune(imgr_batch_t b, const int32_t *caps, int32_t n_caps,
                                  int32_t reps, float *ms, int32_t *chosen);

/* Cache budget of a member set (imgr_batch_info.n_sets).  By default (and
 * with bytes = 0) all members form one set: one fused de/gridding launch and
 * one flush per major cycle for all of them.  With bytes > 0 members are
 * taken in consecutive sets whose model grids and chunk windows stay within
 * `bytes`, each set's stages running back to back.  Results are unchanged
 * bit for bit.  Rebuilds the batch's tables; synchronous. */
imgr_status imager_batch_set_bytes(imgr_batch_t b, uint64_t bytes);

/* Message for the last failure on b.  Never NULL. */
const char *imager_batch_last_error(imgr_batch_t b);

/* Wait for all work enqueued on the handle's stream. */
imgr_status imager_sync(imgr_t h);

/* Message for the last failure on h (or, for h == NULL, of the calling
 * thread's last imager_create).  Never NULL. */
const char *imager_last_error(imgr_t h);

#ifdef __cplusplus
}
#endif

#endif /* IMAGER_H */
