// C-ABI entry points of the imager library: argument checks, handle
// lifetime, device-memory accounting, and the order in which each call
// enqueues its kernels on the handle's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"

namespace imgr {

void *dev_alloc(imgr_s *h, size_t bytes) {
  bytes = std::max<size_t>(bytes, 16);
  if (h->caching) bytes = (bytes + 4095) & ~(size_t)4095;
  void *p = nullptr;
  if (h->caching) {
    // a block freed earlier during handle creation, of the same size: its last user
    // was enqueued on the same stream, so reuse is ordered after it
    for (size_t i = 0; i < h->cache.size(); ++i) {
      if (h->cache[i].second == bytes) {
        p = h->cache[i].first;
        h->cache.erase(h->cache.begin() + i);
        h->cached_bytes -= bytes;
        break;
      }
    }
  }
  if (!p) {
    if (h->budget && h->bytes + h->cached_bytes + bytes > h->budget)
      throw Error{IMGR_ENOMEM, "device footprint would exceed hbm_budget (" +
                                   std::to_string(h->bytes + h->cached_bytes + bytes) + " > " +
                                   std::to_string(h->budget) + " bytes)"};
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error{IMGR_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e)};
    }
  }
  h->bytes += bytes;
  h->peak_bytes = std::max(h->peak_bytes, h->bytes + h->cached_bytes);
  h->allocs.push_back(p);
  // remember the size in a parallel list for accounting on free
  h->alloc_sizes.push_back(bytes);
  return p;
}

void dev_free(imgr_s *h, void *p) {
  if (!p) return;
  for (size_t i = 0; i < h->allocs.size(); ++i) {
    if (h->allocs[i] == p) {
      const size_t bytes = h->alloc_sizes[i];
      h->bytes -= bytes;
      h->allocs.erase(h->allocs.begin() + i);
      h->alloc_sizes.erase(h->alloc_sizes.begin() + i);
      if (h->caching) {
        h->cache.emplace_back(p, bytes);
        h->cached_bytes += bytes;
      } else {
        (void)hipFree(p);
      }
      return;
    }
  }
}

// end of a build: release the blocks kept for reuse (the stream is idle)
static void drop_cache(imgr_s *h) {
  h->caching = false;
  for (auto &c : h->cache) (void)hipFree(c.first);
  h->cache.clear();
  h->cached_bytes = 0;
}

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on P_n.
static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// 1 / psi_hat(p), p = ix - n/2, for an n-pixel image axis on an ng-cell grid:
// psi_hat(p) = (W/2) int_{-1}^{1} phi(z) cos(pi W z p / ng) dz (FP64).
static std::vector<float> correction_inv(int n, int ng, int W, double beta) {
  std::vector<double> z, wq;
  gauss_legendre(128, z, wq);
  std::vector<double> phi(z.size());
  for (size_t k = 0; k < z.size(); ++k) phi[k] = std::exp(beta * (std::sqrt(1.0 - z[k] * z[k]) - 1.0));
  std::vector<float> out(n);
  for (int ix = 0; ix < n; ++ix) {
    const double p = (double)(ix - n / 2);
    double acc = 0.0;
    for (size_t k = 0; k < z.size(); ++k) acc += wq[k] * phi[k] * std::cos(M_PI * W * z[k] * p / ng);
    out[ix] = (float)(1.0 / (0.5 * W * acc));
  }
  return out;
}

static bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

static void fail(imgr_s *h, const Error &e) {
  h->err = e.msg;
  if (e.code == IMGR_EDEVICE) h->broken = true;
}

// PSF of partition p: unit visibilities gridded on the 2 Ng grid (same cell
// size), transformed to the 2N x 2N image and normalised by sum(w); then
// its plain DFT for the H x products of Eq. 7
static void build_psf(imgr_s *h, int p) {
  hipStream_t s = h->stream;
  Partition &P = h->part[p];
  const int n2 = 2 * h->N, ng2 = 2 * h->Ng;
  P.psf = (float *)dev_alloc(h, (size_t)n2 * n2 * sizeof(float));
  P.psf_hat = (float2 *)dev_alloc(h, (size_t)n2 * n2 * sizeof(float2));
  float2 *grid = (float2 *)dev_alloc(h, (size_t)ng2 * ng2 * sizeof(float2));
  float2 *tmp = (float2 *)dev_alloc(h, (size_t)ng2 * ng2 * sizeof(float2));
  float2 *rows = (float2 *)dev_alloc(h, (size_t)n2 * ng2 * sizeof(float2));
  float2 *scr = (float2 *)dev_alloc(
      h, (size_t)std::max(P.psf_bins.n_chunks, 1) * kWin * kWin * sizeof(float2));
  degrid_grid(h, P.psf_bins, MODE_PSF, nullptr, nullptr, nullptr, scr, s);
  flush_chunks(h, P.psf_bins, scr, grid, s);
  fft_grid_to_image(h, grid, h->cinv2, n2, ng2, (float)(1.0 / P.sum_w), rows, tmp, P.psf,
                    P.psf_bins.box, s);
  IMGR_HIP(hipStreamSynchronize(s));
  dev_free(h, scr);
  dev_free(h, rows);
  dev_free(h, tmp);
  dev_free(h, grid);
  free_bins(h, P.psf_bins);
  psf_spectrum(h, p, s);
  IMGR_HIP(hipStreamSynchronize(s));
}

static hipEvent_t take_event(imgr_s *h) {
  if (!h->ev_pool.empty()) {
    hipEvent_t e = h->ev_pool.back();
    h->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  IMGR_HIP(hipEventCreate(&e));
  return e;
}

static void recycle_events(imgr_s *h) {
  for (auto &set : h->ev_sets)
    for (hipEvent_t e : set) h->ev_pool.push_back(e);
  h->ev_sets.clear();
}

// frees everything the handle holds (streams, events, device memory) and the handle
static void release(imgr_s *h) {
  (void)hipStreamSynchronize(h->stream);
  for (int p = 0; p < 2; ++p)
    if (h->node_stream[p]) (void)hipStreamSynchronize(h->node_stream[p]);
  if (h->psf_stream) (void)hipStreamSynchronize(h->psf_stream);
  recycle_events(h);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  for (int p = 0; p < 2; ++p) {
    if (h->ev_join[p]) (void)hipEventDestroy(h->ev_join[p]);
    if (h->node_stream[p]) (void)hipStreamDestroy(h->node_stream[p]);
    if (h->ev_psf[p]) (void)hipEventDestroy(h->ev_psf[p]);
  }
  if (h->ev_psf_join) (void)hipEventDestroy(h->ev_psf_join);
  if (h->ev_win) (void)hipEventDestroy(h->ev_win);
  if (h->psf_stream) (void)hipStreamDestroy(h->psf_stream);
  for (void *q : h->allocs) (void)hipFree(q);
  for (auto &c : h->cache) (void)hipFree(c.first);
  delete h;
}


static void check_cycle_args(imgr_s *h, int part, const float *model, const float *rho_other,
                             const float *residual_out, int flags) {
  IMGR_CHECK(part >= 0 && part < h->n_parts, "partition index out of range");
  IMGR_CHECK(model && residual_out, "null pointer");
  IMGR_CHECK(!(flags & IMGR_DEGRID_COMPOSITE) || rho_other, "composite degrid needs rho_other");
}

// One node's major cycle (Eq. 2 then Eq. 7) enqueued on stream s with the
// node's own work buffers, stage by stage (node_stage); stage events are
// recorded on s when timing is on.
NodeCall node_begin(imgr_s *h, int part, const float *model, const float *rho_other,
                    double gamma, double mu, float *residual_out, float *residual_local_out,
                    int flags, hipStream_t s) {
  NodeCall c{part, model, rho_other, gamma, mu, residual_out,
             residual_local_out ? residual_local_out : h->work[part].img, flags, s, -1, false};
  if (h->timing) {
    c.ev_set = (int)h->ev_sets.size();
    h->ev_sets.emplace_back();
    for (int k = 0; k <= IMGR_N_STAGES; ++k) h->ev_sets.back().push_back(take_event(h));
    IMGR_HIP(hipEventRecord(h->ev_sets[c.ev_set][0], s));
  }
  return c;
}

void node_stage(imgr_s *h, const NodeCall &c, int stage) {
  const Partition &P = h->part[c.part];
  Work &wk = h->work[c.part];
  hipStream_t s = c.s;
  switch (stage) {
    case 0:  // a1: model -> model grid
      fft_model_to_grid(h, c.model, (c.flags & IMGR_DEGRID_COMPOSITE) ? c.rho_other : nullptr,
                        h->cinv, h->N, h->Ng, wk.rows, wk.grid_b, wk.grid_a, P.bins.box, s);
      break;
    case 1:  // a2 + a3: degrid, residual, grid (one pass per chunk)
      degrid_grid(h, P.bins, MODE_DEGRID_GRID, wk.grid_a, nullptr, nullptr, wk.scratch, s);
      break;
    case 2:  // flush of the chunk windows
      flush_chunks(h, P.bins, wk.scratch, wk.grid_a, s);
      break;
    case 3:  // a4: residual grid -> residual image
      fft_grid_to_image(h, wk.grid_a, h->cinv, h->N, h->Ng, (float)(1.0 / P.sum_w), wk.rows,
                        wk.grid_b, c.local, P.bins.box, s);
      break;
    case 4:  // a6: pseudo-full-resolution composition (none without an output)
      if (!c.residual_out) break;
      if (h->n_parts == 2) {
        compose(h, c.part, c.local, c.rho_other, c.gamma, c.mu, c.residual_out, c.psf_pre, s);
      } else if (c.residual_out != c.local) {
        IMGR_HIP(hipMemcpyAsync(c.residual_out, c.local, (size_t)h->N * h->N * sizeof(float),
                                hipMemcpyDeviceToDevice, s));
      }
      break;
    default:
      throw Error{IMGR_EINVAL, "unknown cycle stage"};
  }
  if (c.ev_set >= 0) IMGR_HIP(hipEventRecord(h->ev_sets[c.ev_set][stage + 1], s));
}

void node_cycle(imgr_s *h, int part, const float *model, const float *rho_other,
                       double gamma, double mu, float *residual_out, float *residual_local_out,
                       int flags, hipStream_t s) {
  const NodeCall c = node_begin(h, part, model, rho_other, gamma, mu, residual_out,
                                residual_local_out, flags, s);
  for (int stage = 0; stage < IMGR_N_STAGES; ++stage) node_stage(h, c, stage);
}

// re-cut every partition's chunks for cap C and grow the chunk-window
// scratch when needed
void set_chunk(imgr_s *h, int C) {
  hipStream_t s = h->stream;
  IMGR_HIP(hipStreamSynchronize(s));
  for (int p = 0; p < h->n_parts; ++p) {
    Bins &B = h->part[p].bins;
    rechunk(h, B, C, s);
    const size_t nc = (size_t)std::max(B.n_chunks, 1);
    if (nc > h->scratch_chunks[p]) {
      dev_free(h, h->work[p].scratch);
      h->work[p].scratch = nullptr;
      h->scratch_chunks[p] = 0;
      h->work[p].scratch = (float2 *)dev_alloc(h, nc * kWin * kWin * sizeof(float2));
      h->scratch_chunks[p] = nc;
    }
  }
  h->C = C;
  ++h->layout_version;
}

}  // namespace imgr

using namespace imgr;

static thread_local std::string g_create_error;

#define API_BEGIN(h)                                                  \
  if (!(h)) return IMGR_EINVAL;                                       \
  if ((h)->broken) {                                                  \
    (h)->err = "handle is unusable after an earlier device error";    \
    return IMGR_ESTATE;                                               \
  }                                                                   \
  try {
#define API_END(h)          \
  }                         \
  catch (const Error &e) {  \
    fail((h), e);           \
    return e.code;          \
  }                         \
  catch (const std::exception &e) { \
    (h)->err = e.what();    \
    return IMGR_EINVAL;     \
  }                         \
  return IMGR_OK;

extern "C" {

imgr_status imager_create(const imgr_config *cfg, const imgr_vis *vis, imgr_t *out) {
  if (out) *out = nullptr;
  if (!cfg || !vis || !out) {
    g_create_error = "null argument";
    return IMGR_EINVAL;
  }
  auto t0 = std::chrono::steady_clock::now();
  imgr_s *h = new imgr_s();
  try {
    IMGR_CHECK(pow2(cfg->n_pix) && cfg->n_pix >= 64 && cfg->n_pix <= 2048,
               "n_pix must be a power of two in [64, 2048]");
    h->N = cfg->n_pix;
    h->Ng = 2 * h->N;
    IMGR_HIP(hipGetDevice(&h->device));
    if (cfg->support == 0 && cfg->tolerance > 0) {
      h->W = support_for_tolerance(cfg->tolerance);
      IMGR_CHECK(h->W > 0, "no built support reaches the requested tolerance");
    } else {
      h->W = cfg->support ? cfg->support : 8;
    }
    IMGR_CHECK(h->W == 4 || h->W == 6 || h->W == 8 || h->W == 10 || h->W == 12,
               "support must be 4, 6, 8, 10 or 12");
    h->beta = cfg->es_beta > 0 ? cfg->es_beta : 2.30 * h->W;
    h->blk = cfg->tile ? cfg->tile : (h->W <= 8 ? 8 : 4);
    IMGR_CHECK(h->blk == 4 || h->blk == 8, "tile (block side) must be 4 or 8");
    IMGR_CHECK(window_supported(h->W, h->blk),
               "tile + support - 1 must not exceed 16 (the footprint window)");
    h->C = cfg->chunk ? cfg->chunk : 1024;
    IMGR_CHECK(h->C >= 16 && h->C <= (1 << 20), "chunk must be in [16, 2^20]");
    h->tune = cfg->autotune != 0 && (cfg->tile == 0 || cfg->chunk == 0);
    h->tile_fixed = cfg->tile;
    h->chunk_fixed = cfg->chunk;
    IMGR_CHECK(cfg->n_partitions == 1 || cfg->n_partitions == 2, "n_partitions must be 1 or 2");
    h->n_parts = cfg->n_partitions;
    IMGR_CHECK(cfg->weighting == IMGR_WEIGHT_NATURAL || cfg->weighting == IMGR_WEIGHT_UNIFORM,
               "weighting must be natural or uniform");
    h->weighting = cfg->weighting;
    h->ell = cfg->ell_pix;
    h->delta = cfg->delta_pix > 0 ? cfg->delta_pix : 1.0;
    h->budget = cfg->hbm_budget;
    h->stream = (hipStream_t)cfg->stream;
    IMGR_CHECK(vis->n_vis > 0 && vis->n_vis < (int64_t)INT32_MAX, "n_vis must be in [1, 2^31)");
    IMGR_CHECK(vis->uvw && vis->vis, "uvw and vis are required");
    IMGR_CHECK(vis->vis_dtype == IMGR_C64 || vis->vis_dtype == IMGR_C128, "vis_dtype");
    IMGR_CHECK(vis->freq_hz > 0, "freq_hz must be positive");
    IMGR_CHECK(cfg->cell_rad > 0, "cell_rad must be given (> 0)");
    h->cell = cfg->cell_rad;

    // tables
    {
      std::vector<float> c1 = correction_inv(h->N, h->Ng, h->W, h->beta);
      std::vector<float> c2 = correction_inv(2 * h->N, 2 * h->Ng, h->W, h->beta);
      h->cinv = (float *)dev_alloc(h, c1.size() * sizeof(float));
      h->cinv2 = (float *)dev_alloc(h, c2.size() * sizeof(float));
      IMGR_HIP(hipMemcpy(h->cinv, c1.data(), c1.size() * sizeof(float), hipMemcpyHostToDevice));
      IMGR_HIP(hipMemcpy(h->cinv2, c2.data(), c2.size() * sizeof(float), hipMemcpyHostToDevice));
      std::vector<float2> tw(kTwMax);
      for (int m = 0; m < kTwMax; ++m) {
        const double a = 2.0 * M_PI * (double)m / (double)kTwMax;
        tw[m] = make_float2((float)std::cos(a), (float)-std::sin(a));
      }
      h->tw = (float2 *)dev_alloc(h, kTwMax * sizeof(float2));
      IMGR_HIP(hipMemcpy(h->tw, tw.data(), kTwMax * sizeof(float2), hipMemcpyHostToDevice));
      std::vector<double2> tw64(kTwMax);
      for (int m = 0; m < kTwMax; ++m) {
        const double a = 2.0 * M_PI * (double)m / (double)kTwMax;
        tw64[m] = make_double2(std::cos(a), -std::sin(a));
      }
      h->tw64 = (double2 *)dev_alloc(h, kTwMax * sizeof(double2));
      IMGR_HIP(hipMemcpy(h->tw64, tw64.data(), kTwMax * sizeof(double2), hipMemcpyHostToDevice));
      // per-length tables: entry L + m = w_L^m = the entry m kTwMax / L above
      std::vector<float2> twr(2 * kTwMax, make_float2(0.f, 0.f));
      std::vector<double2> twr64(2 * kTwMax, make_double2(0.0, 0.0));
      for (int L = 2; L <= kTwMax; L *= 2)
        for (int m = 0; m < L; ++m) {
          twr[L + m] = tw[m * (kTwMax / L)];
          twr64[L + m] = tw64[m * (kTwMax / L)];
        }
      h->twrow = (float2 *)dev_alloc(h, twr.size() * sizeof(float2));
      h->twrow64 = (double2 *)dev_alloc(h, twr64.size() * sizeof(double2));
      IMGR_HIP(hipMemcpy(h->twrow, twr.data(), twr.size() * sizeof(float2),
                         hipMemcpyHostToDevice));
      IMGR_HIP(hipMemcpy(h->twrow64, twr64.data(), twr64.size() * sizeof(double2),
                         hipMemcpyHostToDevice));
    }
    const size_t ng2 = (size_t)h->Ng * h->Ng;
    for (int p = 0; p < h->n_parts; ++p) {
      Work &wk = h->work[p];
      wk.grid_a = (float2 *)dev_alloc(h, ng2 * sizeof(float2));
      wk.grid_b = (float2 *)dev_alloc(h, ng2 * sizeof(float2));
      wk.rows = (float2 *)dev_alloc(h, (size_t)h->N * h->Ng * sizeof(float2));
      wk.img = (float *)dev_alloc(h, (size_t)h->N * h->N * sizeof(float));
    }

    // the build frees and re-requests many temporaries of equal size: keep
    // freed blocks for reuse until it ends, instead of a hipFree (which
    // waits for the device) and a hipMalloc each time
    h->caching = true;
    prep_build(h, vis);

    for (int p = 0; p < h->n_parts; ++p) {
      const size_t nc = (size_t)std::max(h->part[p].bins.n_chunks, 1);
      h->work[p].scratch = (float2 *)dev_alloc(h, nc * kWin * kWin * sizeof(float2));
      h->scratch_chunks[p] = nc;
    }
    if (h->n_parts == 2) {
      IMGR_HIP(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
      for (int p = 0; p < 2; ++p) {
        IMGR_HIP(hipStreamCreateWithFlags(&h->node_stream[p], hipStreamNonBlocking));
        IMGR_HIP(hipEventCreateWithFlags(&h->ev_join[p], hipEventDisableTiming));
        IMGR_HIP(hipEventCreateWithFlags(&h->ev_psf[p], hipEventDisableTiming));
        h->psf_work[p] = (float2 *)dev_alloc(h, (size_t)h->N * h->Ng * sizeof(float2));
      }
      IMGR_HIP(hipStreamCreateWithFlags(&h->psf_stream, hipStreamNonBlocking));
      IMGR_HIP(hipEventCreateWithFlags(&h->ev_psf_join, hipEventDisableTiming));
      IMGR_HIP(hipEventCreateWithFlags(&h->ev_win, hipEventDisableTiming));
      h->psf_tmp = (float2 *)dev_alloc(h, (size_t)h->Ng * h->Ng * sizeof(float2));
    }
    for (int p = 0; p < h->n_parts; ++p) {
      IMGR_CHECK(h->part[p].bins.n > 0, "a partition is empty (check ell / delta)");
      build_psf(h, p);
    }
    IMGR_HIP(hipStreamSynchronize(h->stream));
    drop_cache(h);
  } catch (const Error &e) {
    g_create_error = e.msg;
    release(h);
    (void)hipGetLastError();
    return e.code;
  } catch (const std::exception &e) {
    g_create_error = e.what();
    release(h);
    return IMGR_EINVAL;
  }
  h->create_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = h;
  return IMGR_OK;
}

imgr_status imager_destroy(imgr_t h) {
  if (!h) return IMGR_EINVAL;
  (void)hipStreamSynchronize(h->stream);
  release(h);
  return IMGR_OK;
}

imgr_status imager_info(imgr_t h, imgr_info *o) {
  if (!h || !o) return IMGR_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->n_pix = h->N;
  o->n_grid = h->Ng;
  o->support = h->W;
  o->tile = h->blk;
  o->n_partitions = h->n_parts;
  o->cell_rad = h->cell;
  o->es_beta = h->beta;
  o->ell_pix = h->ell;
  o->delta_pix = h->delta;
  o->n_valid = h->n_valid;
  for (int p = 0; p < h->n_parts; ++p) {
    o->n_vis[p] = h->part[p].bins.n;
    o->n_chunks[p] = h->part[p].bins.n_chunks;
    o->sum_w[p] = h->part[p].sum_w;
  }
  o->device_bytes = h->bytes;
  o->create_ms = h->create_ms;
  o->chunk = h->C;
  o->device_peak_bytes = h->peak_bytes;
  return IMGR_OK;
}

imgr_status imager_footprint(const imgr_config *cfg, int64_t n_vis, int32_t vis_on_host,
                             int32_t n_scales, int32_t fista, size_t *resident, size_t *peak) {
  if (!cfg || !resident || n_vis < 0 || n_scales < 0 || n_scales > IMGR_MAX_SCALES)
    return IMGR_EINVAL;
  if (!pow2(cfg->n_pix) || cfg->n_pix < 64 || cfg->n_pix > 2048) return IMGR_EINVAL;
  if (cfg->n_partitions != 1 && cfg->n_partitions != 2) return IMGR_EINVAL;
  const double N = cfg->n_pix, Ng = 2.0 * N, nn = N * N;
  int W = cfg->support;
  if (W == 0) W = cfg->tolerance > 0 ? support_for_tolerance(cfg->tolerance) : 8;
  if (W <= 0) return IMGR_EINVAL;
  // the smaller tile (more blocks) bounds both candidates
  const int blk = cfg->tile ? cfg->tile : 4;
  const int C = cfg->chunk ? cfg->chunk : (cfg->autotune ? 256 : 1024);
  const int parts = cfg->n_partitions;
  const double m = (double)n_vis;
  const double np_ = parts == 2 ? (cfg->ell_pix < 0 ? 0.6 * m : m) : m;
  auto chunks = [&](double ng) { return np_ / C + (ng / blk) * (ng / blk); };
  auto tables = [&](double ng) {  // posvis, w, orig, outpos + chunk tables (with row counts)
    const double nb2 = (ng / blk) * (ng / blk);
    return 28.0 * np_ + 4.0 * (11.0 * chunks(ng) + nb2 + 2.0);
  };
  const double fixed = 4.0 * (N + 2 * N) + 3 * 24.0 * kTwMax + 4096.0;
  double per = 2 * 8.0 * Ng * Ng + 8.0 * N * Ng + 4.0 * nn   // work grids, rows, image
               + tables(Ng) + 2048.0 * chunks(Ng)             // bins, chunk windows
               + 12.0 * 4 * nn;                               // PSF and its spectrum
  double loop = 0.0;
  if (n_scales > 0 || fista) loop += 6.0 * 4 * nn;            // loop dirty, psf, delta
  double minor = 0.0;
  if (n_scales > 0) {
    const double ni = n_scales + 1, npair = ni * (ni + 1) / 2;
    minor = std::max(minor, 8.0 * (ni * nn + npair * 4 * nn + nn) + 65536.0);
  }
  // FISTA: 11 FP64 images, 6 complex FP64 images of work, the FP64 PSF
  // spectrum and the temporary it is built in
  if (fista > 0)  // 4 coefficient-sized arrays per basis (+1 for a dictionary), 7 images,
                  // transform work, the FP64 PSF spectrum and its temporary
    minor = std::max(minor, 8.0 * (7.0 + 4.0 * fista + (fista > 1 ? fista : 0)) * nn +
                                16.0 * 6 * nn + 2 * 16.0 * 4 * nn + 65536.0);
  // two partitions: the PSF terms' work (N x 2N complex per node) and their
  // shared (2N)^2 complex temporary
  const double psf_terms = parts == 2 ? 2 * 8.0 * N * Ng + 8.0 * Ng * Ng : 0.0;
  const double res = fixed + parts * (per + loop + minor) + psf_terms;
  // create-time temporaries on top of the handle's work buffers and tables
  const double staged = vis_on_host ? (24.0 + 16.0 + 4.0 + 1.0) * m : 0.0;
  const double prep = 45.0 * m + 4.0 * nn;                   // coordinates, weights, keys
  const double sortb = 8.0 * m + 16.0 * m + 12.0 * (Ng / blk) * (Ng / blk) * 4;
  const double psf_build = tables(2 * Ng) + 2 * 8.0 * 4 * Ng * Ng + 8.0 * 2 * N * 2 * Ng +
                           2048.0 * chunks(2 * Ng) + 16.0 * 4 * nn;
  const double tune = cfg->autotune ? 2 * 8.0 * Ng * Ng + tables(Ng) + 2048.0 * chunks(Ng) : 0.0;
  const double create_peak = fixed + psf_terms + parts * (per - 12.0 * 4 * nn) + staged + prep +
                             sortb + std::max(psf_build + 12.0 * 4 * nn, tune);
  *resident = (size_t)res;
  if (peak) *peak = (size_t)std::max(res, create_peak + parts * 12.0 * 4 * nn);
  return IMGR_OK;
}

imgr_status imager_tune_log(imgr_t h, int32_t cap, int32_t *tile, int32_t *chunk, float *ms,
                            int32_t *n) {
  API_BEGIN(h)
  IMGR_CHECK(n != nullptr && cap >= 0, "bad arguments");
  IMGR_CHECK(cap == 0 || (tile && chunk && ms), "null output array");
  const int k = (int)h->tune_log.size();
  for (int i = 0; i < k && i < cap; ++i) {
    tile[i] = h->tune_log[i].blk;
    chunk[i] = h->tune_log[i].C;
    ms[i] = h->tune_log[i].ms;
  }
  *n = k;
  API_END(h)
}

imgr_status imager_set_chunk(imgr_t h, int32_t chunk) {
  API_BEGIN(h)
  IMGR_CHECK(chunk >= 16 && chunk <= (1 << 20), "chunk must be in [16, 2^20]");
  set_chunk(h, chunk);
  API_END(h)
}

static void check_part(imgr_s *h, int part) {
  IMGR_CHECK(part >= 0 && part < h->n_parts, "partition index out of range");
}

// the minor cycle's parameters checked, with psi^1's scale subset applied
static imgr_msclean_params checked_msclean_params(imgr_s *h, int part,
                                                  const imgr_msclean_params &p) {
  IMGR_CHECK(p.n_scales >= 1 && p.n_scales <= IMGR_MAX_SCALES, "n_scales must be in [1, 8]");
  for (int i = 0; i < p.n_scales; ++i)
    IMGR_CHECK(p.scales[i] >= 0.0 && p.scales[i] <= 64.0 && std::isfinite(p.scales[i]),
               "scales must be in [0, 64] pixels");
  IMGR_CHECK(p.gain > 0.0 && p.gain <= 1.0, "gain must be in (0, 1]");
  IMGR_CHECK(p.max_iter >= 0, "max_iter must be >= 0");
  IMGR_CHECK(std::isfinite(p.threshold) && std::isfinite(p.bias_slope), "threshold / bias");
  IMGR_CHECK(p.active_mask == 0u || (p.active_mask & ((1u << p.n_scales) - 1u)) != 0u,
             "active_mask selects no scale");
  imgr_msclean_params q = p;
  if (p.own_scales_only) q.active_mask = (p.active_mask ? p.active_mask : ~0u) &
                                         msclean_own_scales(h, part, p);
  return q;
}

imgr_status imager_vis_index(imgr_t h, int32_t part, int64_t *idx) {
  API_BEGIN(h)
  check_part(h, part);
  IMGR_CHECK(idx != nullptr, "idx is NULL");
  const Bins &P = h->part[part].bins;
  std::vector<int32_t> orig(P.n), pos(P.n);
  IMGR_HIP(hipMemcpyAsync(orig.data(), P.orig, P.n * 4, hipMemcpyDeviceToHost, h->stream));
  IMGR_HIP(hipMemcpyAsync(pos.data(), P.outpos, P.n * 4, hipMemcpyDeviceToHost, h->stream));
  IMGR_HIP(hipStreamSynchronize(h->stream));
  for (int64_t s = 0; s < P.n; ++s) idx[pos[s]] = orig[s];
  API_END(h)
}

imgr_status imager_vis_weight(imgr_t h, int32_t part, float *w) {
  API_BEGIN(h)
  check_part(h, part);
  IMGR_CHECK(w != nullptr, "w is NULL");
  const Bins &P = h->part[part].bins;
  std::vector<float> ws(P.n);
  std::vector<int32_t> pos(P.n);
  IMGR_HIP(hipMemcpyAsync(ws.data(), P.w, P.n * 4, hipMemcpyDeviceToHost, h->stream));
  IMGR_HIP(hipMemcpyAsync(pos.data(), P.outpos, P.n * 4, hipMemcpyDeviceToHost, h->stream));
  IMGR_HIP(hipStreamSynchronize(h->stream));
  for (int64_t s = 0; s < P.n; ++s) w[pos[s]] = ws[s];
  API_END(h)
}

imgr_status imager_degrid(imgr_t h, int32_t part, const float *model, void *vis_out) {
  API_BEGIN(h)
  check_part(h, part);
  IMGR_CHECK(model && vis_out, "null pointer");
  hipStream_t s = h->stream;
  Work &wk = h->work[part];
  fft_model_to_grid(h, model, nullptr, h->cinv, h->N, h->Ng, wk.rows, wk.grid_b, wk.grid_a,
                    h->part[part].bins.box, s);
  degrid_grid(h, h->part[part].bins, MODE_DEGRID, wk.grid_a, nullptr, (float2 *)vis_out, nullptr,
              s);
  API_END(h)
}

imgr_status imager_grid(imgr_t h, int32_t part, const void *vis_in, float *image_out,
                        int32_t mode) {
  API_BEGIN(h)
  check_part(h, part);
  IMGR_CHECK(vis_in && image_out, "null pointer");
  IMGR_CHECK(mode == IMGR_GRID_DIRTY || mode == IMGR_GRID_UNNORMALIZED, "mode");
  hipStream_t s = h->stream;
  const Bins &B = h->part[part].bins;
  Work &wk = h->work[part];
  degrid_grid(h, B, MODE_GRID, nullptr, (const float2 *)vis_in, nullptr, wk.scratch, s);
  flush_chunks(h, B, wk.scratch, wk.grid_a, s);
  const float scale = mode == IMGR_GRID_DIRTY ? (float)(1.0 / h->part[part].sum_w) : 1.f;
  fft_grid_to_image(h, wk.grid_a, h->cinv, h->N, h->Ng, scale, wk.rows, wk.grid_b, image_out,
                    B.box, s);
  API_END(h)
}

imgr_status imager_psf(imgr_t h, int32_t part, float *psf_out) {
  API_BEGIN(h)
  check_part(h, part);
  IMGR_CHECK(psf_out, "null pointer");
  const size_t n2 = (size_t)2 * h->N;
  IMGR_HIP(hipMemcpyAsync(psf_out, h->part[part].psf, n2 * n2 * sizeof(float),
                          hipMemcpyDeviceToDevice, h->stream));
  API_END(h)
}

imgr_status imager_major_cycle(imgr_t h, int32_t part, const float *model, const float *rho_other,
                               double gamma, double mu, float *residual_out,
                               float *residual_local_out, int32_t flags) {
  API_BEGIN(h)
  check_cycle_args(h, part, model, rho_other, residual_out, flags);
  node_cycle(h, part, model, rho_other, gamma, mu, residual_out, residual_local_out, flags,
             h->stream);
  API_END(h)
}

imgr_status imager_major_cycle_nodes(imgr_t h, const float *const *model,
                                     const float *const *rho_other, const double *gamma,
                                     const double *mu, float *const *residual_out,
                                     float *const *residual_local_out, int32_t flags) {
  API_BEGIN(h)
  IMGR_CHECK(model && gamma && mu && residual_out, "null pointer");
  for (int p = 0; p < h->n_parts; ++p)
    check_cycle_args(h, p, model[p], rho_other ? rho_other[p] : nullptr, residual_out[p], flags);
  auto ro = [&](int p) { return rho_other ? rho_other[p] : nullptr; };
  auto lo = [&](int p) { return residual_local_out ? residual_local_out[p] : nullptr; };
  if (h->n_parts == 1) {
    node_cycle(h, 0, model[0], ro(0), gamma[0], mu[0], residual_out[0], lo(0), flags, h->stream);
  } else {
    // fork both nodes off the caller's stream, join them back into it
    // the two nodes' stages are enqueued alternately, so both streams have
    // work from the start (enqueueing one node's whole cycle first would hold
    // the other back by the host's launch time)
    IMGR_HIP(hipEventRecord(h->ev_fork, h->stream));
    NodeCall c[2];
    for (int p = 0; p < 2; ++p) {
      IMGR_HIP(hipStreamWaitEvent(h->node_stream[p], h->ev_fork, 0));
      c[p] = node_begin(h, p, model[p], ro(p), gamma[p], mu[p], residual_out[p], lo(p), flags,
                        h->node_stream[p]);
    }
    // the PSF terms of Eq. 7 read only the cycle's inputs: their fronts run
    // on the PSF stream, one after the other, from the end of node V_L's
    // de/gridding on (the smaller partition's, which ends first; earlier,
    // they take the de/gridding's compute units), beside the memory-bound
    // stages; each node's composition waits for its own before its last pass
    bool pre[2];
    for (int p = 0; p < 2; ++p) c[p].psf_pre = pre[p] = residual_out[p] && mu[p] != 0.0 && ro(p);
    for (int stage = 0; stage < IMGR_N_STAGES; ++stage)
      for (int p = 0; p < 2; ++p) {
        node_stage(h, c[p], stage);
        if (stage == 1 && p == IMGR_PART_LOW && (pre[0] || pre[1])) {
          IMGR_HIP(hipEventRecord(h->ev_win, h->node_stream[p]));
          IMGR_HIP(hipStreamWaitEvent(h->psf_stream, h->ev_win, 0));
          for (int k = 0; k < 2; ++k)
            if (pre[k]) compose_psf_front(h, k, ro(k), mu[k], h->psf_stream);
        }
      }
    for (int p = 0; p < 2; ++p) {
      IMGR_HIP(hipEventRecord(h->ev_join[p], h->node_stream[p]));
      IMGR_HIP(hipStreamWaitEvent(h->stream, h->ev_join[p], 0));
    }
    if (pre[0] || pre[1]) {
      IMGR_HIP(hipEventRecord(h->ev_psf_join, h->psf_stream));
      IMGR_HIP(hipStreamWaitEvent(h->stream, h->ev_psf_join, 0));
    }
  }
  API_END(h)
}

imgr_status imager_composed_psf(imgr_t h, int32_t part, double gamma, double mu, float *psf_out) {
  API_BEGIN(h)
  check_part(h, part);
  IMGR_CHECK(psf_out, "null pointer");
  if (h->n_parts == 1) {
    const size_t n2 = (size_t)2 * h->N;
    IMGR_HIP(hipMemcpyAsync(psf_out, h->part[part].psf, n2 * n2 * sizeof(float),
                            hipMemcpyDeviceToDevice, h->stream));
  } else {
    composed_psf(h, part, gamma, mu, psf_out, h->stream);
  }
  API_END(h)
}

imgr_status imager_minor_cycle_msclean(imgr_t h, int32_t part, const imgr_msclean_params *params,
                                       const float *dirty, const float *psf, float *model_delta,
                                       float *model_accum, float *residual_out,
                                       imgr_component *comps, int32_t *n_comps) {
  API_BEGIN(h)
  check_part(h, part);
  IMGR_CHECK(params && dirty && psf && n_comps, "null pointer");
  const imgr_msclean_params q = checked_msclean_params(h, part, *params);
  msclean_enqueue(h, part, q, dirty, psf, model_delta, model_accum, residual_out, comps,
                  h->stream);
  IMGR_HIP(hipStreamSynchronize(h->stream));
  *n_comps = msclean_count(h, part);
  API_END(h)
}

imgr_status imager_minor_cycle_msclean_static(imgr_t h, int32_t part,
                                              const imgr_msclean_params *params,
                                              const float *dirty, const float *psf,
                                              float *model_delta, float *model_accum,
                                              float *residual_out, imgr_component *comps,
                                              int32_t *n_comps) {
  API_BEGIN(h)
  check_part(h, part);
  IMGR_CHECK(params && dirty && psf && n_comps, "null pointer");
  const imgr_msclean_params q = checked_msclean_params(h, part, *params);
  *n_comps = msclean_enqueue_static(h, q, dirty, psf, model_delta, model_accum, residual_out,
                                    comps, h->stream);
  API_END(h)
}

imgr_status imager_reconstruct_msclean(imgr_t h, int32_t n_cycles,
                                       const imgr_msclean_params *params, float *const *model,
                                       float *const *rho, double *final_image,
                                       int32_t *n_comps) {
  API_BEGIN(h)
  IMGR_CHECK(params && model && final_image, "null pointer");
  IMGR_CHECK(n_cycles >= 1, "n_cycles must be >= 1");
  IMGR_CHECK(h->n_parts == 1 || rho, "rho is required with two partitions");
  const imgr_msclean_params &p = *params;
  IMGR_CHECK(p.n_scales >= 1 && p.n_scales <= IMGR_MAX_SCALES, "n_scales must be in [1, 8]");
  IMGR_CHECK(p.gain > 0.0 && p.gain <= 1.0 && p.max_iter >= 0, "gain / max_iter");
  for (int k = 0; k < h->n_parts; ++k) IMGR_CHECK(model[k] && (!rho || rho[k]), "null pointer");
  const int n = h->N;
  const size_t nn = (size_t)n * n;
  for (int k = 0; k < h->n_parts; ++k) {
    if (!h->loop_dirty[k]) {
      h->loop_dirty[k] = (float *)dev_alloc(h, nn * sizeof(float));
      h->loop_psf[k] = (float *)dev_alloc(h, 4 * nn * sizeof(float));
      h->loop_delta[k] = (float *)dev_alloc(h, nn * sizeof(float));
    }
  }
  const double wsum = h->part[0].sum_w + (h->n_parts == 2 ? h->part[1].sum_w : 0.0);
  IMGR_CHECK(p.first_cycle >= 0, "first_cycle must be >= 0");
  const int c0 = std::max(p.first_cycle, 1);
  for (int cyc = c0; cyc < c0 + n_cycles; ++cyc) {
    if (h->n_parts == 1) {
      hipStream_t s = h->stream;
      node_cycle(h, 0, model[0], nullptr, 1.0, 0.0, h->loop_dirty[0], nullptr, 0, s);
      IMGR_HIP(hipMemcpyAsync(h->loop_psf[0], h->part[0].psf, 4 * nn * sizeof(float),
                              hipMemcpyDeviceToDevice, s));
      msclean_enqueue(h, 0, p, h->loop_dirty[0], h->loop_psf[0], h->loop_delta[0], model[0],
                      nullptr, nullptr, s);
    } else {
      IMGR_HIP(hipEventRecord(h->ev_fork, h->stream));
      // the major cycles of both nodes, their stages enqueued alternately
      NodeCall nc[2];
      for (int k = 0; k < 2; ++k) {
        hipStream_t s = h->node_stream[k];
        IMGR_HIP(hipStreamWaitEvent(s, h->ev_fork, 0));
        // Eq. 7 weights (reading): gamma = 1, mu = 0 at the first cycle,
        // then the partitions' shares of the summed imaging weights
        const double gamma = (cyc == 1) ? 1.0 : h->part[k].sum_w / wsum;
        const double mu = (cyc == 1) ? 0.0 : h->part[1 - k].sum_w / wsum;
        nc[k] = node_begin(h, k, model[k], rho[k], gamma, mu, h->loop_dirty[k], nullptr, 0, s);
      }
      for (int stage = 0; stage < IMGR_N_STAGES; ++stage)
        for (int k = 0; k < 2; ++k) node_stage(h, nc[k], stage);
      for (int k = 0; k < 2; ++k) {
        hipStream_t s = h->node_stream[k];
        const double gamma = nc[k].gamma, mu = nc[k].mu;
        composed_psf(h, k, gamma, mu, h->loop_psf[k], s);
        imgr_msclean_params q = p;
        if (cyc == 1) q.active_mask = (p.active_mask ? p.active_mask : ~0u) &
                                      msclean_own_scales(h, k, p);
        msclean_enqueue(h, k, q, h->loop_dirty[k], h->loop_psf[k], h->loop_delta[k], model[k],
                        nullptr, nullptr, s);
        IMGR_HIP(hipEventRecord(h->ev_join[k], s));
      }
      for (int k = 0; k < 2; ++k) IMGR_HIP(hipStreamWaitEvent(h->stream, h->ev_join[k], 0));
      // Phi / rho exchange (Section 4.1): rho_H at node L, rho_L at node H
      exchange(h, h->loop_delta[0], h->loop_delta[1], rho[0], rho[1], h->stream);
    }
    if (n_comps) {
      IMGR_HIP(hipStreamSynchronize(h->stream));
      for (int k = 0; k < h->n_parts; ++k)
        n_comps[(size_t)(cyc - c0) * h->n_parts + k] = msclean_count(h, k);
    }
  }
  // final image: equal-weight average of the nodes' models in FP64 (Section 5.2)
  if (h->n_parts == 2)
    combine_final(h, model[0], model[1], 0.5, 0.5, final_image, h->stream);
  else
    combine_final(h, model[0], model[0], 1.0, 0.0, final_image, h->stream);
  IMGR_HIP(hipStreamSynchronize(h->stream));
  API_END(h)
}

static void check_fista(imgr_s *h, const imgr_fista_params &p) {
  IMGR_CHECK(p.vanishing >= 1 && p.vanishing <= 10, "vanishing must be in [1, 10]");
  IMGR_CHECK(p.levels >= 1 && (h->N >> p.levels) >= 1, "levels must be in [1, log2 N]");
  IMGR_CHECK(p.n_iter >= 0 && p.power_iters >= 1, "n_iter >= 0 and power_iters >= 1");
  IMGR_CHECK(std::isfinite(p.lambda) && std::isfinite(p.lambda_frac) && std::isfinite(p.gamma_n),
             "lambda / gamma_n");
  IMGR_CHECK(p.lambda > 0.0 || p.lambda_frac >= 0.0, "lambda_frac must be >= 0");
  IMGR_CHECK(p.dictionary == 0 || p.dictionary == 1, "dictionary must be 0 or 1");
}

imgr_status imager_minor_cycle_fista(imgr_t h, int32_t part, const imgr_fista_params *params,
                                     const float *dirty, const float *psf,
                                     const float *rho_other, const float *power_start,
                                     float *model_delta, float *model_accum, double *objective,
                                     double *lipschitz, double *lambda_used) {
  API_BEGIN(h)
  check_part(h, part);
  IMGR_CHECK(params && dirty && power_start, "null pointer");
  check_fista(h, *params);
  IMGR_CHECK(params->serial || params->gamma_n == 0.0 || rho_other || h->n_parts == 1,
             "gamma_n != 0 needs rho_other");
  fista_enqueue(h, part, *params, dirty, psf, rho_other, power_start, model_delta,
                model_accum, objective, h->stream);
  IMGR_HIP(hipStreamSynchronize(h->stream));
  fista_scalars(h, part, lipschitz, lambda_used);
  API_END(h)
}

imgr_status imager_reconstruct_fista(imgr_t h, int32_t n_cycles, const imgr_fista_params *params,
                                     const float *const *power_start, float *const *model,
                                     float *const *rho, double *final_image, double *lipschitz,
                                     double *lambdas) {
  API_BEGIN(h)
  IMGR_CHECK(params && power_start && model && final_image, "null pointer");
  IMGR_CHECK(n_cycles >= 1, "n_cycles must be >= 1");
  IMGR_CHECK(h->n_parts == 1 || rho, "rho is required with two partitions");
  check_fista(h, *params);
  for (int k = 0; k < h->n_parts; ++k)
    IMGR_CHECK(power_start[k] && model[k] && (!rho || rho[k]), "null pointer");
  const size_t nn = (size_t)h->N * h->N;
  for (int k = 0; k < h->n_parts; ++k) {
    if (!h->loop_dirty[k]) {
      h->loop_dirty[k] = (float *)dev_alloc(h, nn * sizeof(float));
      h->loop_psf[k] = (float *)dev_alloc(h, 4 * nn * sizeof(float));
      h->loop_delta[k] = (float *)dev_alloc(h, nn * sizeof(float));
    }
  }
  IMGR_CHECK(params->first_cycle >= 0, "first_cycle must be >= 0");
  const int c0 = std::max(params->first_cycle, 1);
  for (int cyc = c0; cyc < c0 + n_cycles; ++cyc) {
    imgr_fista_params q = *params;
    if (h->n_parts == 1) {
      hipStream_t s = h->stream;
      q.serial = 1;
      q.gamma_n = 0.0;
      node_cycle(h, 0, model[0], nullptr, 1.0, 0.0, h->loop_dirty[0], nullptr, 0, s);
      fista_enqueue(h, 0, q, h->loop_dirty[0], nullptr, nullptr, power_start[0],
                    h->loop_delta[0], model[0], nullptr, s);
    } else {
      q.serial = 0;
      q.gamma_n = (cyc == 1) ? 0.0 : 1.0;  // Eq. 5
      IMGR_HIP(hipEventRecord(h->ev_fork, h->stream));
      // the node's own residual i~ (Eq. 2) on both nodes, stages enqueued
      // alternately; the composition is not used here
      NodeCall nc[2];
      for (int k = 0; k < 2; ++k) {
        IMGR_HIP(hipStreamWaitEvent(h->node_stream[k], h->ev_fork, 0));
        nc[k] = node_begin(h, k, model[k], nullptr, 1.0, 0.0, nullptr, h->loop_dirty[k], 0,
                           h->node_stream[k]);
      }
      for (int stage = 0; stage < IMGR_N_STAGES; ++stage)
        for (int k = 0; k < 2; ++k) node_stage(h, nc[k], stage);
      for (int k = 0; k < 2; ++k) {
        hipStream_t s = h->node_stream[k];
        fista_enqueue(h, k, q, h->loop_dirty[k], nullptr, rho[k], power_start[k],
                      h->loop_delta[k], model[k], nullptr, s);
        IMGR_HIP(hipEventRecord(h->ev_join[k], s));
      }
      for (int k = 0; k < 2; ++k) IMGR_HIP(hipStreamWaitEvent(h->stream, h->ev_join[k], 0));
      exchange(h, h->loop_delta[0], h->loop_delta[1], rho[0], rho[1], h->stream);
    }
    if (lipschitz || lambdas) {
      IMGR_HIP(hipStreamSynchronize(h->stream));
      for (int k = 0; k < h->n_parts; ++k) {
        const size_t at = (size_t)(cyc - c0) * h->n_parts + k;
        fista_scalars(h, k, lipschitz ? lipschitz + at : nullptr, lambdas ? lambdas + at : nullptr);
      }
    }
  }
  if (h->n_parts == 2)
    combine_final(h, model[0], model[1], 0.5, 0.5, final_image, h->stream);
  else
    combine_final(h, model[0], model[0], 1.0, 0.0, final_image, h->stream);
  IMGR_HIP(hipStreamSynchronize(h->stream));
  API_END(h)
}

imgr_status imager_combine_partitions(imgr_t h, int32_t mode, const float *a, const float *b,
                                      double w_a, double w_b, void *out_a, void *out_b) {
  API_BEGIN(h)
  IMGR_CHECK(a && b && out_a, "null pointer");
  if (mode == IMGR_COMBINE_EXCHANGE) {
    IMGR_CHECK(h->n_parts == 2, "exchange needs two partitions");
    IMGR_CHECK(out_b, "null pointer");
    exchange(h, a, b, (float *)out_a, (float *)out_b, h->stream);
  } else if (mode == IMGR_COMBINE_FINAL) {
    combine_final(h, a, b, w_a, w_b, (double *)out_a, h->stream);
  } else {
    throw Error{IMGR_EINVAL, "mode"};
  }
  API_END(h)
}

imgr_status imager_set_timing(imgr_t h, int32_t enable) {
  API_BEGIN(h)
  IMGR_HIP(hipStreamSynchronize(h->stream));
  recycle_events(h);
  h->timing = enable != 0;
  API_END(h)
}

imgr_status imager_get_timing(imgr_t h, imgr_timing *out) {
  API_BEGIN(h)
  IMGR_CHECK(out, "null pointer");
  IMGR_HIP(hipStreamSynchronize(h->stream));
  std::memset(out, 0, sizeof(*out));
  for (auto &set : h->ev_sets) {
    for (int k = 0; k < IMGR_N_STAGES; ++k) {
      float ms = 0.f;
      IMGR_HIP(hipEventElapsedTime(&ms, set[k], set[k + 1]));
      out->ms[k] += ms;
    }
    out->cycles += 1;
  }
  recycle_events(h);
  API_END(h)
}

imgr_status imager_sync(imgr_t h) {
  API_BEGIN(h)
  IMGR_HIP(hipStreamSynchronize(h->stream));
  API_END(h)
}

const char *imager_last_error(imgr_t h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}

}  // extern "C"
