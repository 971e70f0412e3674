// Multi-scale CLEAN minor cycle (Eq. 6 and Eq. 7, Section 4.2) in FP64.
//
// For the scale set S (scale 0 added internally, not selectable, when S
// lacks it, so the unsmoothed residual R_0 is always tracked):
//   R_s  = phi_s * D               (N x N, linear convolution, zero outside)
//   B_ab = phi_a * phi_b * P       (2N x 2N, a <= b, centre (N, N))
// then per iteration k < K:
//   step:   apply the previous component's update R_t -= alpha B_{s*t}
//           (shifted to p*), and find the block-local peak of
//           bias_s |R_s(p)| over the selectable scales (ties: smaller scale,
//           then smaller flat index) and the block-local max |R_0|;
//   select: one workgroup reduces the block results; stops (for good) if
//           max |R_0| < threshold, else alpha = gain R_{s*}(p*) / B_{s*s*}(0),
//           records the component and adds alpha phi_{s*} at p* to the model.
// Every operation that can decide an argmax is done in FP64 with separate
// multiply / subtract roundings, in the order of the plain definition, so
// the decisions are those of an FP64 evaluation.  The host launches the K
// step/select pairs without waiting; once stopped, every later kernel
// returns at once.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

// The work area of imager_minor_cycle_msclean_static: one array per device
// (each GPU the library runs on holds its own copy until the process ends),
// shared by every call on that device.  Host code never passes `scratch`
// itself to a kernel or copy: in host code that name is a stand-in, not a
// device address.  The address comes from hipGetSymbolAddress
// (imgr::static_area) and only that address is used.
static __device__ __align__(256) unsigned char scratch[IMGR_MSCLEAN_STATIC_BYTES];

namespace imgr {
namespace {

constexpr int kMaxInt = IMGR_MAX_SCALES + 1;  // internal scales (scale 0 may be added)
constexpr int kStepThreads = 256;
constexpr int kStepBlocks = 1024;

struct CleanState {
  int stop;     // no more components
  int pend;     // the last component's update is not yet applied
  int s, p;     // last component: internal scale, flat pixel
  double alpha;
  int n_comps;
  int pad;
};

struct Cand {
  double v;     // bias_s |R_s(p)|
  int s, p;     // internal scale, flat pixel
  double peak0; // max |R_0|
  double rv;    // R_s(p) itself
};

__device__ __forceinline__ bool better(double v1, int s1, int p1, double v2, int s2, int p2) {
  return v1 > v2 || (v1 == v2 && (s1 < s2 || (s1 == s2 && p1 < p2)));
}

struct StepArgs {
  double *R;            // [n_int][N*N]
  const double *B;      // [n_pairs][(2N)^2]
  int pair[kMaxInt][kMaxInt];
  double bias[kMaxInt];
  int selectable[kMaxInt];
  int n_int, n, r0;     // internal scales, image side, internal index of scale 0
};

__device__ __forceinline__ void reduce_cand(Cand &c, Cand *sh) {
  // wave then workgroup reduction under the total order of `better`
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(c.v, off);
    const int os = __shfl_xor(c.s, off), op = __shfl_xor(c.p, off);
    const double o0 = __shfl_xor(c.peak0, off);
    const double orv = __shfl_xor(c.rv, off);
    if (better(ov, os, op, c.v, c.s, c.p)) {
      c.v = ov;
      c.s = os;
      c.p = op;
      c.rv = orv;
    }
    c.peak0 = fmax(c.peak0, o0);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      if (better(sh[w].v, sh[w].s, sh[w].p, c.v, c.s, c.p)) {
        c.v = sh[w].v;
        c.s = sh[w].s;
        c.p = sh[w].p;
        c.rv = sh[w].rv;
      }
      c.peak0 = fmax(c.peak0, sh[w].peak0);
    }
  }
}

struct SelectArgs {
  const double *B;
  int pair[kMaxInt][kMaxInt];
  const double *kern;   // scale kernels, concatenated
  int koff[kMaxInt], krad[kMaxInt];
  int user[kMaxInt];    // internal -> user scale index
  int n, n_int;
  double gain, threshold;
};

// One iteration.  Every workgroup reduces the previous iteration's
// per-workgroup candidates itself (the same values in the same order, so
// all reach the same decision): stop for good if max |R_0| < threshold, else
// alpha = gain R_{s*}(p*) / B_{s*s*}(0).  Workgroup 0 records the component
// and adds alpha phi_{s*} at p* to the model.  Then every workgroup applies
// R_t -= alpha B_{s*t} (shifted to p*) to its pixels and posts its candidate
// for the next iteration.  With first != 0 there is no previous candidate
// set: the launch only posts the candidates of the initial residuals.
// NI = a.n_int (internal scales), a template argument so the per-pixel
// arrays hold exactly the scales in use.
template <int NI>
__global__ __launch_bounds__(kStepThreads) void k_clean_iter(StepArgs a, SelectArgs se,
                                                              CleanState *st, const Cand *prev,
                                                              int n_prev, Cand *next, int first,
                                                              imgr_component *comps,
                                                              double *model) {
  __shared__ Cand sh[kStepThreads / 64];
  __shared__ int go, s_s, s_p;
  __shared__ double s_alpha;
  if (st->stop) return;
  const int n = a.n, nn = n * n, n2 = 2 * n;
  bool upd = false;
  int ps = 0, pp = 0;
  double alpha = 0.0;
  if (!first) {
    Cand c{-1.0, 0x7fffffff, 0x7fffffff, 0.0, 0.0};
    for (int i = threadIdx.x; i < n_prev; i += kStepThreads) {
      const Cand o = prev[i];
      if (better(o.v, o.s, o.p, c.v, c.s, c.p)) {
        c.v = o.v;
        c.s = o.s;
        c.p = o.p;
        c.rv = o.rv;
      }
      c.peak0 = fmax(c.peak0, o.peak0);
    }
    reduce_cand(c, sh);
    if (threadIdx.x == 0) {
      go = 0;
      if (!(c.peak0 >= se.threshold) || c.s >= se.n_int) {
        if (blockIdx.x == 0) st->stop = 1;
      } else {
        const double bc = se.B[(size_t)se.pair[c.s][c.s] * n2 * n2 + (size_t)n * n2 + n];
        const double al = __ddiv_rn(__dmul_rn(se.gain, c.rv), bc);
        if (blockIdx.x == 0) {
          const int k = st->n_comps;
          imgr_component cp;
          cp.scale = se.user[c.s];
          cp.iy = c.p / n;
          cp.ix = c.p % n;
          cp.reserved = 0;
          cp.amp = al;
          if (comps) comps[k] = cp;
          st->n_comps = k + 1;
        }
        s_alpha = al;
        s_s = c.s;
        s_p = c.p;
        go = 1;
      }
    }
    __syncthreads();
    if (!go) return;
    upd = true;
    ps = s_s;
    pp = s_p;
    alpha = s_alpha;
    if (blockIdx.x == 0) {
      // model += alpha phi_s centred at p (clipped to the image)
      const int r = se.krad[ps], w = 2 * r + 1;
      const double *k = se.kern + se.koff[ps];
      const int cy = pp / n, cx = pp % n;
      for (int j = threadIdx.x; j < w * w; j += kStepThreads) {
        const int y = cy + j / w - r, x = cx + j % w - r;
        if (y >= 0 && y < n && x >= 0 && x < n) {
          double *m = model + (size_t)y * n + x;
          *m = __dadd_rn(*m, __dmul_rn(alpha, k[j]));
        }
      }
    }
  }
  const int py = pp / n, px = pp % n;
  Cand c{-1.0, 0x7fffffff, 0x7fffffff, 0.0, 0.0};
  // two pixels per pass, every load of both issued before the first use;
  // the candidate order (`better`) is total and peak0 a maximum, so the
  // result does not depend on the order pixels and scales are visited in
  const int lg = 31 - __clz(n);  // n is a power of two
  double *__restrict__ R = a.R;
  const double *__restrict__ Bs[NI];
#pragma unroll
  for (int t = 0; t < NI; ++t) Bs[t] = a.B + (size_t)a.pair[upd ? ps : 0][t] * n2 * n2;
  const int stride = gridDim.x * kStepThreads;
  for (int i0 = blockIdx.x * kStepThreads + threadIdx.x; i0 < nn; i0 += 2 * stride) {
    const int i1 = i0 + stride;
    const bool has1 = i1 < nn;
    double v0[NI], v1[NI], b0[NI], b1[NI];
    const size_t bi0 = (size_t)(n + (i0 >> lg) - py) * n2 + (n + (i0 & (n - 1)) - px);
    const size_t bi1 = (size_t)(n + (i1 >> lg) - py) * n2 + (n + (i1 & (n - 1)) - px);
#pragma unroll
    for (int t = 0; t < NI; ++t) {
      v0[t] = R[(size_t)t * nn + i0];
      if (has1) v1[t] = R[(size_t)t * nn + i1];
      if (upd) {
        b0[t] = Bs[t][bi0];
        if (has1) b1[t] = Bs[t][bi1];
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h == 1 && !has1) break;
      const int i = h ? i1 : i0;
#pragma unroll
      for (int t = 0; t < NI; ++t) {
        double v = h ? v1[t] : v0[t];
        if (upd) {
          v = __dsub_rn(v, __dmul_rn(alpha, h ? b1[t] : b0[t]));
          R[(size_t)t * nn + i] = v;
        }
        if (a.selectable[t]) {
          const double bv = __dmul_rn(a.bias[t], fabs(v));
          if (better(bv, t, i, c.v, c.s, c.p)) {
            c.v = bv;
            c.s = t;
            c.p = i;
            c.rv = v;
          }
        }
        if (t == a.r0) c.peak0 = fmax(c.peak0, fabs(v));
      }
    }
  }
  reduce_cand(c, sh);
  if (threadIdx.x == 0) next[blockIdx.x] = c;
}

// out (n x n) = in * k (linear, zero outside), k of side 2r+1, centred
template <typename T>
__global__ __launch_bounds__(256) void k_conv_same(const T *__restrict__ in, int n,
                                                   const double *__restrict__ k, int r,
                                                   double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * n) return;
  const int y = (int)(i / n), x = (int)(i % n);
  const int w = 2 * r + 1;
  double acc = 0.0;
  for (int a = -r; a <= r; ++a) {
    const int yy = y - a;
    if (yy < 0 || yy >= n) continue;
    const T *row = in + (size_t)yy * n;
    const double *kr = k + (size_t)(a + r) * w + r;
    for (int b = -r; b <= r; ++b) {
      const int xx = x - b;
      if (xx < 0 || xx >= n) continue;
      acc = fma(kr[b], (double)row[xx], acc);
    }
  }
  out[i] = acc;
}

// The same convolution on 16 x 64 output tiles: the workgroup stages the
// input tile with its halo (zero outside the image) and the kernel, padded
// with zero columns to a multiple of 4, in LDS; each thread forms 4
// neighbouring outputs of one row, taking the kernel columns in groups of 4
// (7 staged values serve the 16 products of a group).  Every output adds
// k[a][b] in[y - a][x - b] in the order of k_conv_same (a, then b,
// ascending); the extra products with padded zeros add nothing.
constexpr int kConvTY = 16, kConvTX = 64;

inline size_t conv_tile_lds(int r) {
  const int wp = (2 * r + 1 + 3) / 4 * 4, pad = wp - (2 * r + 1);
  return (size_t)(kConvTY + 2 * r) * (kConvTX + 2 * r + pad) * sizeof(float) +
         (size_t)(2 * r + 1) * wp * sizeof(double);
}

__global__ __launch_bounds__(256) void k_conv_tile(const float *__restrict__ in, int n,
                                                   const double *__restrict__ k, int r,
                                                   double *__restrict__ out) {
  extern __shared__ double conv_lds[];
  const int w = 2 * r + 1;
  const int wp = (w + 3) / 4 * 4, pad = wp - w;
  const int th = kConvTY + 2 * r, tw = kConvTX + 2 * r + pad;
  double *kw = conv_lds;                          // [w][wp]
  float *tile = reinterpret_cast<float *>(kw + (size_t)w * wp);  // [th][tw]
  const int x0 = blockIdx.x * kConvTX, y0 = blockIdx.y * kConvTY;
  for (int i = threadIdx.x; i < w * wp; i += 256) {
    const int a = i / wp, b = i % wp;
    kw[i] = (b < w) ? k[a * w + b] : 0.0;
  }
  for (int i = threadIdx.x; i < th * tw; i += 256) {
    const int ty = i / tw, tx = i % tw;
    const int yy = y0 - r + ty, xx = x0 - r - pad + tx;
    tile[i] = (yy >= 0 && yy < n && xx >= 0 && xx < n) ? in[(size_t)yy * n + xx] : 0.f;
  }
  __syncthreads();
  const int ly = threadIdx.x >> 4, lx = (threadIdx.x & 15) * 4;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int a = 0; a < w; ++a) {
    const float *row = tile + (size_t)(ly + 2 * r - a) * tw;
    const double *kr = kw + (size_t)a * wp;
    for (int g = 0; g < wp; g += 4) {
      // columns lx + (2 r + pad - g) - 3 .. + 3 of the tile
      const float *c = row + lx + (2 * r + pad - g) - 3;
      float v[7];
#pragma unroll
      for (int m = 0; m < 7; ++m) v[m] = c[m];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double kq = kr[g + q];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = fma(kq, (double)v[j - q + 3], acc[j]);
      }
    }
  }
  const int y = y0 + ly;
  if (y < n) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int x = x0 + lx + j;
      if (x < n) out[(size_t)y * n + x] = acc[j];
    }
  }
}

// out = in * k (same as k_conv_same), tiled when the tile fits in LDS
void conv_same(const float *in, int n, const double *k, int r, double *out, hipStream_t s) {
  const size_t lds = conv_tile_lds(r);
  if (lds <= 64 * 1024) {
    hipLaunchKernelGGL(k_conv_tile, dim3(cdiv(n, kConvTX), cdiv(n, kConvTY)), dim3(256), lds, s,
                       in, n, k, r, out);
  } else {
    hipLaunchKernelGGL(k_conv_same<float>, dim3(cdiv((int64_t)n * n, 256)), dim3(256), 0, s, in,
                       n, k, r, out);
  }
}

// pending update on R_0 only, then the f32 outputs
struct FinishArgs {
  int pair_r0[kMaxInt];  // pair index of (t, r0) for each internal scale t
};

__global__ void k_clean_finish(double *R0, const double *B, FinishArgs fa, const CleanState *st,
                               int n, const double *model, float *model_delta,
                               float *model_accum, float *resid_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nn = n * n, n2 = 2 * n;
  if (i >= nn) return;
  double v = R0[i];
  if (st->pend) {
    const int y = (int)(i / n), x = (int)(i % n);
    const int py = st->p / n, px = st->p % n;
    const double *b = B + (size_t)fa.pair_r0[st->s] * n2 * n2;
    v = __dsub_rn(v, __dmul_rn(st->alpha, b[(size_t)(n + y - py) * n2 + (n + x - px)]));
    R0[i] = v;
  }
  const float m = (float)model[i];
  if (model_delta) model_delta[i] = m;
  if (model_accum) model_accum[i] += m;
  if (resid_out) resid_out[i] = (float)v;
}

// phi_s: 1 at s = 0; else 1 - (x^2 + y^2) / s^2 on r = ceil(s) - 1, unit sum
std::vector<double> scale_kernel(double s, int &r) {
  if (s == 0.0) {
    r = 0;
    return {1.0};
  }
  r = (int)std::ceil(s) - 1;
  const int w = 2 * r + 1;
  std::vector<double> k(w * w);
  double sum = 0.0;
  for (int y = -r; y <= r; ++y)
    for (int x = -r; x <= r; ++x) {
      double v = 1.0 - (double)(x * x + y * y) / (s * s);
      if (v < 0.0) v = 0.0;
      k[(y + r) * w + (x + r)] = v;
      sum += v;
    }
  for (double &v : k) v /= sum;
  return k;
}

// full 2-D convolution of two centred odd kernels
std::vector<double> conv_full(const std::vector<double> &a, int ra, const std::vector<double> &b,
                              int rb, int &r) {
  r = ra + rb;
  const int wa = 2 * ra + 1, wb = 2 * rb + 1, w = 2 * r + 1;
  std::vector<double> out(w * w, 0.0);
  for (int y1 = 0; y1 < wa; ++y1)
    for (int x1 = 0; x1 < wa; ++x1)
      for (int y2 = 0; y2 < wb; ++y2)
        for (int x2 = 0; x2 < wb; ++x2)
          out[(y1 + y2) * w + (x1 + x2)] += a[y1 * wa + x1] * b[y2 * wb + x2];
  return out;
}

}  // namespace

void msclean_release(imgr_s *h, int part) {
  CleanWork &cw = h->clean[part];
  for (void *q : {(void *)cw.R, (void *)cw.B, (void *)cw.kern, (void *)cw.model, cw.state,
                  cw.slots})
    dev_free(h, q);
  cw = CleanWork();
}

// mask of the scales of S present in the node's own spatial-frequency
// domain (psi^1 of Eq. 7; reading): V_L keeps s >= N / (2 (ell + delta)),
// V_H keeps s <= N / (ell - delta); if none qualifies, the scale nearest to
// the bound.  With one partition: every scale.
uint32_t msclean_own_scales(const imgr_s *h, int part, const imgr_msclean_params &prm) {
  const int ns = prm.n_scales;
  if (h->n_parts == 1) return (1u << ns) - 1u;
  const double bound = (part == IMGR_PART_LOW) ? h->N / (2.0 * (h->ell + h->delta))
                                               : h->N / (h->ell - h->delta);
  uint32_t m = 0;
  for (int i = 0; i < ns; ++i) {
    const double sv = prm.scales[i];
    if ((part == IMGR_PART_LOW) ? (sv >= bound) : (sv <= bound)) m |= 1u << i;
  }
  if (m == 0) {
    int best = 0;
    for (int i = 1; i < ns; ++i)
      if (std::fabs(prm.scales[i] - bound) < std::fabs(prm.scales[best] - bound)) best = i;
    m = 1u << best;
  }
  return m;
}

int msclean_count(imgr_s *h, int part) {
  CleanState hs;
  IMGR_HIP(hipMemcpy(&hs, h->clean[part].state, sizeof(CleanState), hipMemcpyDeviceToHost));
  return hs.n_comps;
}

namespace {

// Everything the host derives from the parameters before any device work:
// internal scales, the scale kernels and their pairwise convolutions
// (concatenated in kall), and the device work area's size.
struct CleanPlan {
  int n_int = 0, n_pairs = 0, r0 = 0;
  double smax = 0.0;
  std::vector<double> sc, kall;
  std::vector<int> user, selectable, rad, koff, poff, prad;
  int pair[kMaxInt][kMaxInt];
};

CleanPlan make_plan(const imgr_msclean_params &prm) {
  CleanPlan P;
  const int ns = prm.n_scales;
  // internal scales: scale 0 first when S lacks it (tracked, not selectable)
  int r0_user = -1;
  for (int i = 0; i < ns; ++i)
    if (prm.scales[i] == 0.0) {
      r0_user = i;
      break;
    }
  const int shift = (r0_user < 0) ? 1 : 0;
  P.n_int = ns + shift;
  P.sc.assign(P.n_int, 0.0);
  P.user.assign(P.n_int, -1);
  P.selectable.assign(P.n_int, 0);
  for (int i = 0; i < ns; ++i) P.smax = std::max(P.smax, prm.scales[i]);
  for (int i = 0; i < ns; ++i) {
    P.sc[i + shift] = prm.scales[i];
    P.user[i + shift] = i;
    P.selectable[i + shift] = (prm.active_mask == 0u || ((prm.active_mask >> i) & 1u)) ? 1 : 0;
  }
  P.r0 = shift ? 0 : r0_user;
  // kernels phi_s and phi_a * phi_b
  std::vector<std::vector<double>> ph(P.n_int);
  P.rad.assign(P.n_int, 0);
  for (int i = 0; i < P.n_int; ++i) ph[i] = scale_kernel(P.sc[i], P.rad[i]);
  P.koff.assign(P.n_int, 0);
  for (int i = 0; i < P.n_int; ++i) {
    P.koff[i] = (int)P.kall.size();
    P.kall.insert(P.kall.end(), ph[i].begin(), ph[i].end());
  }
  for (int a = 0; a < P.n_int; ++a)
    for (int b = a; b < P.n_int; ++b) {
      int r;
      std::vector<double> c = conv_full(ph[a], P.rad[a], ph[b], P.rad[b], r);
      P.poff.push_back((int)P.kall.size());
      P.prad.push_back(r);
      P.kall.insert(P.kall.end(), c.begin(), c.end());
      P.pair[a][b] = P.pair[b][a] = P.n_pairs++;
    }
  return P;
}

// the minor cycle on a given work area (nothing is allocated here)
void enqueue_plan(imgr_s *h, const CleanPlan &P, const imgr_msclean_params &prm,
                  const float *dirty, const float *psf, float *model_delta, float *model_accum,
                  float *resid_out, imgr_component *comps, const CleanWork &cw, hipStream_t s) {
  const int n = h->N, nn = n * n, n2 = 2 * n;
  const int n_int = P.n_int, n_pairs = P.n_pairs;
  IMGR_HIP(hipMemcpyAsync(cw.kern, P.kall.data(), P.kall.size() * sizeof(double),
                          hipMemcpyHostToDevice, s));
  IMGR_HIP(hipMemsetAsync(cw.model, 0, (size_t)nn * sizeof(double), s));
  IMGR_HIP(hipMemsetAsync(cw.state, 0, sizeof(CleanState), s));
  // R_s = phi_s * D, B_ab = phi_a phi_b * P
  for (int i = 0; i < n_int; ++i)
    conv_same(dirty, n, cw.kern + P.koff[i], P.rad[i], cw.R + (size_t)i * nn, s);
  for (int q = 0; q < n_pairs; ++q)
    conv_same(psf, n2, cw.kern + P.poff[q], P.prad[q], cw.B + (size_t)q * n2 * n2, s);
  IMGR_HIP(hipGetLastError());

  StepArgs sa;
  sa.R = cw.R;
  sa.B = cw.B;
  SelectArgs se;
  se.B = cw.B;
  se.kern = cw.kern;
  for (int a = 0; a < kMaxInt; ++a) {
    for (int b = 0; b < kMaxInt; ++b)
      sa.pair[a][b] = se.pair[a][b] = (a < n_int && b < n_int) ? P.pair[a][b] : 0;
    sa.bias[a] = 0.0;
    sa.selectable[a] = 0;
    se.koff[a] = se.krad[a] = 0;
    se.user[a] = -1;
  }
  for (int i = 0; i < n_int; ++i) {
    sa.bias[i] = (P.smax == 0.0) ? 1.0 : 1.0 - prm.bias_slope * P.sc[i] / P.smax;
    sa.selectable[i] = P.selectable[i];
    se.koff[i] = P.koff[i];
    se.krad[i] = P.rad[i];
    se.user[i] = P.user[i];
  }
  sa.n_int = se.n_int = n_int;
  sa.n = se.n = n;
  sa.r0 = P.r0;
  se.gain = prm.gain;
  se.threshold = prm.threshold;
  const int nblk = std::min(kStepBlocks, (int)cdiv(nn, kStepThreads));
  CleanState *st = (CleanState *)cw.state;
  Cand *slots = (Cand *)cw.slots;
  // candidates of iteration k live in slots[(k % 2) * kStepBlocks ...]: an
  // iteration reads one half and writes the other
  static_assert(kMaxInt == 9, "one instantiation per internal scale count");
  void (*iter)(StepArgs, SelectArgs, CleanState *, const Cand *, int, Cand *, int,
               imgr_component *, double *) = nullptr;
  switch (n_int) {
    case 1: iter = k_clean_iter<1>; break;
    case 2: iter = k_clean_iter<2>; break;
    case 3: iter = k_clean_iter<3>; break;
    case 4: iter = k_clean_iter<4>; break;
    case 5: iter = k_clean_iter<5>; break;
    case 6: iter = k_clean_iter<6>; break;
    case 7: iter = k_clean_iter<7>; break;
    case 8: iter = k_clean_iter<8>; break;
    case 9: iter = k_clean_iter<9>; break;
    default: throw Error{IMGR_EINVAL, "internal scale count out of range"};
  }
  hipLaunchKernelGGL(iter, dim3(nblk), dim3(kStepThreads), 0, s, sa, se, st,
                     (const Cand *)nullptr, 0, slots, 1, comps, cw.model);
  for (int k = 0; k < prm.max_iter; ++k)
    hipLaunchKernelGGL(iter, dim3(nblk), dim3(kStepThreads), 0, s, sa, se, st,
                       (const Cand *)(slots + (k % 2) * kStepBlocks), nblk,
                       slots + ((k + 1) % 2) * kStepBlocks, 0, comps, cw.model);
  IMGR_HIP(hipGetLastError());
  FinishArgs fa;
  for (int t = 0; t < kMaxInt; ++t) fa.pair_r0[t] = (t < n_int) ? P.pair[t][P.r0] : 0;
  hipLaunchKernelGGL(k_clean_finish, dim3(cdiv(nn, 256)), dim3(256), 0, s,
                     cw.R + (size_t)P.r0 * nn, cw.B, fa, st, n, cw.model, model_delta,
                     model_accum, resid_out);
  IMGR_HIP(hipGetLastError());
}

// Device addresses of `scratch` (below), one per device, taken once per
// device with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices] = {};

void *static_area(int device) {
  IMGR_CHECK(device >= 0 && device < kMaxDevices, "device index out of range");
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[device]) {
    void *p = nullptr;
    IMGR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    IMGR_CHECK(p != nullptr, "hipGetSymbolAddress returned no address for the work area");
    g_static_ptr[device] = p;
  }
  return g_static_ptr[device];
}

inline size_t up256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

void msclean_enqueue(imgr_s *h, int part, const imgr_msclean_params &prm, const float *dirty,
                     const float *psf, float *model_delta, float *model_accum, float *resid_out,
                     imgr_component *comps, hipStream_t s) {
  const int n = h->N, nn = n * n, n2 = 2 * n;
  const CleanPlan P = make_plan(prm);
  // device work area of this node (grown on demand, kept for later calls)
  CleanWork &cw = h->clean[part];
  const size_t need_R = (size_t)P.n_int * nn, need_B = (size_t)P.n_pairs * n2 * n2;
  if (cw.R_elems < need_R || cw.B_elems < need_B || cw.k_elems < P.kall.size()) {
    msclean_release(h, part);
    cw.R = (double *)dev_alloc(h, need_R * sizeof(double));
    cw.B = (double *)dev_alloc(h, need_B * sizeof(double));
    cw.kern = (double *)dev_alloc(h, P.kall.size() * sizeof(double));
    cw.model = (double *)dev_alloc(h, (size_t)nn * sizeof(double));
    cw.state = dev_alloc(h, sizeof(CleanState));
    cw.slots = dev_alloc(h, (size_t)2 * kStepBlocks * sizeof(Cand));
    cw.R_elems = need_R;
    cw.B_elems = need_B;
    cw.k_elems = P.kall.size();
  }
  enqueue_plan(h, P, prm, dirty, psf, model_delta, model_accum, resid_out, comps, cw, s);
}

size_t msclean_static_bytes(const imgr_s *h, const imgr_msclean_params &prm) {
  const CleanPlan P = make_plan(prm);
  const size_t nn = (size_t)h->N * h->N;
  return up256(sizeof(CleanState)) + up256((size_t)2 * kStepBlocks * sizeof(Cand)) +
         up256(nn * sizeof(double)) + up256(P.kall.size() * sizeof(double)) +
         up256((size_t)P.n_int * nn * sizeof(double)) +
         up256((size_t)P.n_pairs * 4 * nn * sizeof(double));
}

int msclean_enqueue_static(imgr_s *h, const imgr_msclean_params &prm, const float *dirty,
                           const float *psf, float *model_delta, float *model_accum,
                           float *resid_out, imgr_component *comps, hipStream_t s) {
  const CleanPlan P = make_plan(prm);
  const size_t need = msclean_static_bytes(h, prm);
  if (need > (size_t)IMGR_MSCLEAN_STATIC_BYTES)
    throw Error{IMGR_EINVAL, "the static msCLEAN work area holds " +
                                 std::to_string((size_t)IMGR_MSCLEAN_STATIC_BYTES) +
                                 " bytes; this image size and scale set need " +
                                 std::to_string(need)};
  int dev = -1;
  IMGR_HIP(hipGetDevice(&dev));
  IMGR_CHECK(dev == h->device, "the handle's device must be current");
  unsigned char *base = (unsigned char *)static_area(dev);
  const size_t nn = (size_t)h->N * h->N;
  CleanWork cw;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    void *p = base + off;
    off += up256(bytes);
    return p;
  };
  cw.state = take(sizeof(CleanState));
  cw.slots = take((size_t)2 * kStepBlocks * sizeof(Cand));
  cw.model = (double *)take(nn * sizeof(double));
  cw.kern = (double *)take(P.kall.size() * sizeof(double));
  cw.R = (double *)take((size_t)P.n_int * nn * sizeof(double));
  cw.B = (double *)take((size_t)P.n_pairs * 4 * nn * sizeof(double));
  enqueue_plan(h, P, prm, dirty, psf, model_delta, model_accum, resid_out, comps, cw, s);
  IMGR_HIP(hipStreamSynchronize(s));
  CleanState hs;
  IMGR_HIP(hipMemcpy(&hs, cw.state, sizeof(CleanState), hipMemcpyDeviceToHost));
  return hs.n_comps;
}

}  // namespace imgr
