// Image-domain pieces of the decentralized framework (Sections 3 and 4):
// the filters Gamma_L / Gamma_H, the pseudo-full-resolution composition of
// Eq. 7, the composed PSF, the aggregate update of Eq. 5 and the final
// combination of Section 5.2.  Filtering and PSF convolution are products
// in the plain 2-D DFT domain of the image's own grid (N x N for Gamma,
// 2N x 2N zero-padded for the linear convolution by the 2N x 2N PSF).
#include "common.h"

namespace imgr {
namespace {

// dst (nd x nd complex) = 0 except dst[r][c] = a[r][c] (- b[r][c])
__global__ void k_pad_real(const float *__restrict__ a, const float *__restrict__ b, int n,
                           float2 *__restrict__ dst, int nd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nd * nd) return;
  const int r = (int)(i / nd), c = (int)(i % nd);
  float v = 0.f;
  if (r < n && c < n) {
    v = a[(int64_t)r * n + c];
    if (b) v -= b[(int64_t)r * n + c];
  }
  dst[i] = make_float2(v, 0.f);
}

// Gamma_L(kappa) = clip((ell + delta - kappa) / (2 delta), 0, 1), kappa the
// radius of the plain-DFT frequency index divided by `scale` (1 on the N
// grid, 2 on the 2N grid); Gamma_H = 1 - Gamma_L.
__device__ __forceinline__ float gamma_low(int kx, int ky, int nd, double ell, double delta,
                                           double scale) {
  const int fx = (kx < nd / 2) ? kx : kx - nd;
  const int fy = (ky < nd / 2) ? ky : ky - nd;
  const double kappa = sqrt((double)fx * fx + (double)fy * fy) / scale;
  const double g = (ell + delta - kappa) / (2.0 * delta);
  return (float)fmin(fmax(g, 0.0), 1.0);
}

// out = gamma Gamma_own a + mu Gamma_other b, per frequency
__global__ void k_spec_combine(float2 *__restrict__ out, const float2 *__restrict__ a,
                               const float2 *__restrict__ b, int nd, double ell, double delta,
                               double scale, int own_low, float gamma, float mu, float coef) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nd * nd) return;
  const int ky = (int)(i / nd), kx = (int)(i % nd);
  const float gl = gamma_low(kx, ky, nd, ell, delta, scale);
  const float g_own = own_low ? gl : 1.f - gl;
  const float g_oth = 1.f - g_own;
  float2 v = cscale(a[i], gamma * g_own);
  if (b) v = cadd(v, cscale(b[i], mu * g_oth));
  out[i] = cscale(v, coef);
}

// out[r][c] (+)= scale * Re buf[row0 + r][col0 + c], r, c < n
__global__ void k_crop_real(const float2 *__restrict__ buf, int nd, int row0, int col0, int n,
                            float scale, float *__restrict__ out, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * n) return;
  const int r = (int)(i / n), c = (int)(i % n);
  const float v = scale * buf[(int64_t)(row0 + r) * nd + col0 + c].x;
  out[i] = accumulate ? out[i] + v : v;
}

__global__ void k_combine_final(const float *__restrict__ a, const float *__restrict__ b,
                                double wa, double wb, int64_t n, double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = wa * (double)a[i] + wb * (double)b[i];
}

__global__ void k_add(const float *__restrict__ a, const float *__restrict__ b,
                      float *__restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] + b[i];
}

inline dim3 g1(int64_t n) { return dim3(cdiv(n, 256)); }

}  // namespace

void add_images(const float *a, const float *b, float *out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_add, g1(n), dim3(256), 0, s, a, b, out, n);
  IMGR_HIP(hipGetLastError());
}

// spectrum of the partition's 2N x 2N PSF (plain DFT), kept for H x products
void psf_spectrum(imgr_s *h, int p, hipStream_t s) {
  const int nd = 2 * h->N;
  Partition &P = h->part[p];
  hipLaunchKernelGGL(k_pad_real, g1((int64_t)nd * nd), dim3(256), 0, s, P.psf, nullptr, nd,
                     P.psf_hat, nd);
  IMGR_HIP(hipGetLastError());
  fft2_plain(h, P.psf_hat, h->work[p].grid_b, nd, -1, s);
}

__global__ void k_pad_real64(const float *__restrict__ a, int n, double2 *__restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)n * n) dst[i] = make_double2((double)a[i], 0.0);
}

// FP64 spectrum (plain DFT) of a 2N x 2N float32 PSF
void psf_spectrum64_of(imgr_s *h, const float *psf, double2 *out, double2 *tmp, hipStream_t s) {
  const int nd = 2 * h->N;
  const size_t m = (size_t)nd * nd;
  hipLaunchKernelGGL(k_pad_real64, g1((int64_t)m), dim3(256), 0, s, psf, nd, out);
  IMGR_HIP(hipGetLastError());
  fft2_plain64(h, out, tmp, nd, -1, s);
}

// FP64 spectrum of the partition's 2N x 2N PSF, built once
const double2 *psf_spectrum64(imgr_s *h, int p, hipStream_t s) {
  Partition &P = h->part[p];
  if (P.psf_hat64) return P.psf_hat64;
  const size_t m = (size_t)4 * h->N * h->N;
  P.psf_hat64 = (double2 *)dev_alloc(h, m * sizeof(double2));
  double2 *tmp = (double2 *)dev_alloc(h, m * sizeof(double2));
  psf_spectrum64_of(h, P.psf, P.psf_hat64, tmp, s);
  IMGR_HIP(hipStreamSynchronize(s));
  dev_free(h, tmp);
  return P.psf_hat64;
}

// Eq. 7: out = gamma Gamma_own resid + mu H_other rho_other
void compose(imgr_s *h, int p, const float *resid, const float *rho_other, double gamma,
             double mu, float *out, bool psf_pre, hipStream_t s) {
  const int n = h->N, nd = 2 * n;
  // both grids are free once the residual image is out
  float2 *work = h->work[p].grid_a, *tmp = h->work[p].grid_b;
  image_gamma_scaled(h, resid, p == IMGR_PART_LOW ? 1 : 0, (float)gamma, out, work, tmp, s);
  if (mu == 0.0 || !rho_other) return;
  if (psf_pre) {
    IMGR_HIP(hipStreamWaitEvent(s, h->ev_psf[p], 0));
    image_psf_conv_back(h, h->psf_work[p], out, 1, s);
  } else {
    image_psf_conv_front(h, rho_other, h->part[1 - p].psf_hat, (float)(mu / ((double)nd * nd)),
                         work, tmp, s);
    image_psf_conv_back(h, work, out, 1, s);
  }
}

void compose_psf_front(imgr_s *h, int p, const float *rho_other, double mu, hipStream_t s) {
  const int nd = 2 * h->N;
  image_psf_conv_front(h, rho_other, h->part[1 - p].psf_hat, (float)(mu / ((double)nd * nd)),
                       h->psf_work[p], h->psf_tmp, s);
  IMGR_HIP(hipEventRecord(h->ev_psf[p], s));
}

void composed_psf(imgr_s *h, int p, double gamma, double mu, float *out, hipStream_t s) {
  const int nd = 2 * h->N;
  const Partition &P = h->part[p];
  const float2 *other = (h->n_parts == 2 && mu != 0.0) ? h->part[1 - p].psf_hat : nullptr;
  float2 *buf = h->work[p].grid_a, *tmp = h->work[p].grid_b;
  hipLaunchKernelGGL(k_spec_combine, g1((int64_t)nd * nd), dim3(256), 0, s, buf, P.psf_hat, other,
                     nd, h->ell, h->delta, 2.0, p == IMGR_PART_LOW ? 1 : 0, (float)gamma,
                     (float)mu, (float)(1.0 / ((double)nd * nd)));
  fft2_plain(h, buf, tmp, nd, 1, s);
  hipLaunchKernelGGL(k_crop_real, g1((int64_t)nd * nd), dim3(256), 0, s, buf, nd, 0, 0, nd, 1.f,
                     out, 0);
  IMGR_HIP(hipGetLastError());
}

// rho_a += Gamma_H (b - a), rho_b += Gamma_L (a - b)
void exchange(imgr_s *h, const float *a, const float *b, float *rho_a, float *rho_b,
              hipStream_t s) {
  const int n = h->N;
  const float inv = (float)(1.0 / ((double)n * n));
  image_gamma(h, b, a, 0, inv, rho_a, 1, h->work[0].grid_a, h->work[0].grid_b, s);
  image_gamma(h, a, b, 1, inv, rho_b, 1, h->work[0].grid_a, h->work[0].grid_b, s);
}

void combine_final(imgr_s *h, const float *a, const float *b, double wa, double wb, double *out,
                   hipStream_t s) {
  const int64_t nn = (int64_t)h->N * h->N;
  hipLaunchKernelGGL(k_combine_final, g1(nn), dim3(256), 0, s, a, b, wa, wb, nn, out);
  IMGR_HIP(hipGetLastError());
}

}  // namespace imgr
