// Sparsity-regularised minor cycle (Eqs. 4 and 5, Section 4.1): FISTA on
// the coefficients of an orthonormal periodized Daubechies wavelet basis.
//
//   f(alpha) = ||Gamma_own (d - H W alpha)||^2 + gamma_n ||rho - Gamma_other W alpha||^2
//   grad f   = -2 W^T (c - H Gamma_own^2 H x - gamma_n Gamma_other^2 x),  x = W alpha,
//   c        = H Gamma_own^2 d + gamma_n Gamma_other rho  (once per minor cycle)
//
// H (the node's 2N x 2N PSF) and Gamma are applied with the fused transform
// pipelines of fft.hip (H and Gamma are self-adjoint: the PSF is even, the
// filters real and radial).  The wavelet transforms are level-by-level
// gather kernels over the Mallat layout.  Everything runs in FP64 (the
// transforms with the FP64 twiddle table and PSF spectrum): FISTA's
// momentum amplifies operator rounding by about ten per fifty iterations
// on these deconvolution problems, which FP32 transforms cannot absorb over
// a few hundred iterations.  lambda and the step constant L_hat live on the
// device, so the iterations run without host synchronisation.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "common.h"

namespace imgr {
namespace {

constexpr int kRedBlocks = 512;

// ------------------------------------------------------------------ filters

// Daubechies low-pass filter with p vanishing moments by spectral
// factorisation: the roots of z^(p-1) P((2 - z - 1/z) / 4), P(y) =
// sum_{k<p} C(p-1+k, k) y^k, come in pairs (r, 1/conj r); h(z) is
// proportional to (1 + z)^p prod_{|r| > 1} (z - r) with sum h = sqrt 2
// (the convention whose p = 2 filter is (1 + sqrt3, 3 + sqrt3, 3 - sqrt3,
// 1 - sqrt3) / (4 sqrt2)).  Roots by Durand-Kerner iteration, polished by
// Newton's method, in long double.
std::vector<double> daubechies(int p) {
  if (p == 1) return {1.0 / std::sqrt(2.0), 1.0 / std::sqrt(2.0)};
  typedef long double R;
  typedef std::complex<R> C;
  const int deg = 2 * (p - 1);
  std::vector<R> poly(deg + 1, 0.0L);  // increasing powers
  // (z y)^k z^(p-1-k) with z y = (-1 + 2 z - z^2) / 4
  for (int k = 0; k < p; ++k) {
    std::vector<R> t(1, 1.0L);
    for (int i = 0; i < k; ++i) {
      std::vector<R> u(t.size() + 2, 0.0L);
      for (size_t a = 0; a < t.size(); ++a) {
        u[a] += -0.25L * t[a];
        u[a + 1] += 0.5L * t[a];
        u[a + 2] += -0.25L * t[a];
      }
      t.swap(u);
    }
    R binom = 1.0L;  // C(p-1+k, k)
    for (int i = 1; i <= k; ++i) binom = binom * (R)(p - 1 + i) / (R)i;
    for (size_t a = 0; a < t.size(); ++a) poly[a + (p - 1 - k)] += binom * t[a];
  }
  auto eval = [&](C z, C &dp) {
    C v = 0, d = 0;
    for (int a = deg; a >= 0; --a) {
      d = d * z + v;
      v = v * z + poly[a];
    }
    dp = d;
    return v;
  };
  std::vector<C> r(deg);
  const C seed(0.4L, 0.9L);
  C pw(1.0L, 0.0L);
  for (int i = 0; i < deg; ++i) {
    r[i] = pw;
    pw *= seed;
  }
  const R lead = poly[deg];
  for (int it = 0; it < 2000; ++it) {
    R move = 0;
    for (int i = 0; i < deg; ++i) {
      C dp;
      C num = eval(r[i], dp) / lead;
      C den = 1;
      for (int j = 0; j < deg; ++j)
        if (j != i) den *= (r[i] - r[j]);
      const C step = num / den;
      r[i] -= step;
      move = std::max(move, std::abs(step));
    }
    if (move < 1e-19L) break;
  }
  for (auto &z : r)
    for (int it = 0; it < 10; ++it) {
      C dp;
      const C v = eval(z, dp);
      if (std::abs(dp) == 0) break;
      z -= v / dp;
    }
  std::vector<C> hz(1, C(1.0L));
  auto mul = [&](C a0, C a1) {  // hz *= (a0 + a1 z)
    std::vector<C> u(hz.size() + 1, C(0));
    for (size_t i = 0; i < hz.size(); ++i) {
      u[i] += a0 * hz[i];
      u[i + 1] += a1 * hz[i];
    }
    hz.swap(u);
  };
  for (int i = 0; i < p; ++i) mul(C(1), C(1));
  for (const C &z : r)
    if (std::abs(z) > 1.0L) mul(-z, C(1));
  R sum = 0;
  for (const C &c : hz) sum += c.real();
  std::vector<double> h(hz.size());
  for (size_t i = 0; i < hz.size(); ++i) h[i] = (double)(hz[i].real() * std::sqrt(2.0L) / sum);
  return h;
}

// ------------------------------------------------------------------ wavelet kernels
// hg: taps low-pass h then taps high-pass g, g_j = (-1)^j h_{L-1-j}

// analysis of the top-left n x n block along the rows (AXIS 1) or the
// columns (AXIS 0): a[k] = sum_j h_j x[(2k + j) mod n], d[k] likewise with g;
// the input is a - b (b may be NULL)
constexpr int kMaxBases = 10;  // dictionary bases: db1 .. db10 at most

// filters of the dictionary's bases (blockIdx.y = basis)
struct Bases {
  int hoff[kMaxBases], taps[kMaxBases];
};

// The tap count T is a template argument (each basis' launch dispatches on
// it), so every tap's load is issued before the first product: the sums
// themselves run in the same order as a plain loop over the taps.
__device__ __forceinline__ int wrap_hi(int m, int n) {  // m mod n for m >= 0
  while (m >= n) m -= n;
  return m;
}

template <int AXIS, int T>
__device__ __forceinline__ void dwt_body(const double *__restrict__ a,
                                         const double *__restrict__ b, int in_stride,
                                         double *__restrict__ out, int out_stride, int n,
                                         const double *__restrict__ hg, double sc, int line,
                                         int k) {
  const int half = n / 2;
  double v[T];
#pragma unroll
  for (int j = 0; j < T; ++j) {
    const int m = wrap_hi(2 * k + j, n);
    const size_t off = (AXIS == 1) ? (size_t)line * in_stride + m : (size_t)m * in_stride + line;
    v[j] = a[off];
    if (b) v[j] -= b[off];
  }
  double lo = 0.0, hi = 0.0;
#pragma unroll
  for (int j = 0; j < T; ++j) {
    double x = v[j];
    if (sc != 1.0) x *= sc;
    lo = fma(hg[j], x, lo);
    hi = fma(hg[T + j], x, hi);
  }
  if (AXIS == 1) {
    out[(size_t)line * out_stride + k] = lo;
    out[(size_t)line * out_stride + half + k] = hi;
  } else {
    out[(size_t)k * out_stride + line] = lo;
    out[(size_t)(half + k) * out_stride + line] = hi;
  }
}

template <int AXIS>
__global__ void k_dwt(const double *__restrict__ a, size_t a_bstride, const double *__restrict__ b,
                      int in_stride, double *__restrict__ out, size_t out_bstride, int out_stride,
                      int n, const double *__restrict__ hlo, Bases bs, double sc) {
  const int p = blockIdx.y;
  const double *__restrict__ hg = hlo + bs.hoff[p];
  const int taps = bs.taps[p];
  a += p * a_bstride;
  out += p * out_bstride;
  const int half = n / 2;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * half) return;
  int line, k;
  if (AXIS == 1) {
    line = (int)(idx / half);
    k = (int)(idx % half);
  } else {
    line = (int)(idx % n);
    k = (int)(idx / n);
  }
  switch (taps) {
#define TAPS_(T) \
  case T: dwt_body<AXIS, T>(a, b, in_stride, out, out_stride, n, hg, sc, line, k); break;
    TAPS_(2) TAPS_(4) TAPS_(6) TAPS_(8) TAPS_(10) TAPS_(12) TAPS_(14) TAPS_(16) TAPS_(18)
    TAPS_(20)
#undef TAPS_
    default: break;  // the host admits db1 .. db10 only
  }
}

// synthesis (the transpose): x[m] = sum over j with m - j even of
// h_j a[k] + g_j d[k], k = ((m - j) mod n) / 2
template <int AXIS, int T>
__device__ __forceinline__ void idwt_body(const double *__restrict__ in,
                                          const double *__restrict__ ll, int in_stride,
                                          double *__restrict__ out, int out_stride, int n,
                                          const double *__restrict__ hg, int line, int m) {
  const int half = n / 2;
  // the approximation quadrant (rows and columns below half) comes from ll
  // when given; the detail quadrants always come from in
  const double *__restrict__ lo_src = (ll && line < half) ? ll : in;
  const int j0 = m & 1;
  double va[T / 2], vd[T / 2];
#pragma unroll
  for (int i = 0; i < T / 2; ++i) {
    const int j = j0 + 2 * i;
    int t = m - j;
    while (t < 0) t += n;
    const int k = t / 2;
    size_t oa, od;
    if (AXIS == 1) {
      oa = (size_t)line * in_stride + k;
      od = oa + half;
    } else {
      oa = (size_t)k * in_stride + line;
      od = (size_t)(half + k) * in_stride + line;
    }
    va[i] = lo_src[oa];
    vd[i] = in[od];
  }
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < T / 2; ++i) {
    const int j = j0 + 2 * i;
    acc = fma(hg[j], va[i], acc);
    acc = fma(hg[T + j], vd[i], acc);
  }
  if (AXIS == 1)
    out[(size_t)line * out_stride + m] = acc;
  else
    out[(size_t)m * out_stride + line] = acc;
}

// (AXIS 0 only: ll, when given, holds the approximation quadrant in place of
// in, with in's layout)
template <int AXIS>
__global__ void k_idwt(const double *__restrict__ in, const double *__restrict__ ll,
                       int in_stride, double *__restrict__ out, int out_stride, size_t bstride,
                       int n, const double *__restrict__ hlo, Bases bs) {
  const int p = blockIdx.y;
  const double *__restrict__ hg = hlo + bs.hoff[p];
  const int taps = bs.taps[p];
  in += p * bstride;
  if (ll) ll += p * bstride;
  out += p * bstride;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  int line, m;
  if (AXIS == 1) {
    line = (int)(idx / n);
    m = (int)(idx % n);
  } else {
    line = (int)(idx % n);
    m = (int)(idx / n);
  }
  switch (taps) {
#define TAPS_(T) \
  case T: idwt_body<AXIS, T>(in, ll, in_stride, out, out_stride, n, hg, line, m); break;
    TAPS_(2) TAPS_(4) TAPS_(6) TAPS_(8) TAPS_(10) TAPS_(12) TAPS_(14) TAPS_(16) TAPS_(18)
    TAPS_(20)
#undef TAPS_
    default: break;
  }
}

// ------------------------------------------------------------------ elementwise / reductions

__global__ void k_f64_to_f32(const double *__restrict__ a, float *__restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

__global__ void k_f32_to_f64(const float *__restrict__ a, double *__restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

__global__ void k_copy_f64(const double *__restrict__ a, double *__restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

// out = sum over the nb blocks of a (stride n) of k a_p, in block order
__global__ void k_sum_bases(const double *__restrict__ a, int nb, double k,
                            double *__restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = k * a[i];
  for (int p = 1; p < nb; ++p) acc = acc + k * a[(size_t)p * n + i];
  out[i] = acc;
}

__global__ void k_add_to_f32(const double *__restrict__ a, float *__restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] += (float)a[i];
}

// per-block partials of: mode 0 sum (a - b)^2, mode 1 max |a|, mode 2 sum |alpha|
__global__ __launch_bounds__(256) void k_reduce(const double *__restrict__ a,
                                                const double *__restrict__ b,
                                                const double *__restrict__ al, int64_t n,
                                                int mode, double *__restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    if (mode == 0) {
      const double v = a[i] - (b ? b[i] : 0.0);
      acc += v * v;
    } else if (mode == 1) {
      acc = fmax(acc, fabs(a[i]));
    } else {
      acc += fabs(al[i]);
    }
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off)
      sh[threadIdx.x] = (mode == 1) ? fmax(sh[threadIdx.x], sh[threadIdx.x + off])
                                    : sh[threadIdx.x] + sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// scal[dst] = op(partials): op 0 sum, 1 max, 2 sqrt(sum); then
// scal[dst] *= mul (and, for op 3 = sqrt(sum) as the power-iteration norm,
// also scal[0] = 2 * norm)
__global__ __launch_bounds__(256) void k_finish(const double *__restrict__ part, int nb, int op,
                                                double mul, double *__restrict__ scal, int dst) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256)
    acc = (op == 1) ? fmax(acc, part[i]) : acc + part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off)
      sh[threadIdx.x] = (op == 1) ? fmax(sh[threadIdx.x], sh[threadIdx.x + off])
                                  : sh[threadIdx.x] + sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double v = sh[0];
    if (op >= 2) v = sqrt(v);
    scal[dst] = v * mul;
    if (op == 3) scal[0] = 2.0 * v;
  }
}

// x *= 1 / scal[k]
__global__ void k_scale_inv(double *__restrict__ x, const double *__restrict__ scal, int k,
                            int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = x[i] / scal[k];
}

// scal[1] = lambda (absolute, or frac * max|dirty| already in scal[1])
__global__ void k_set_lambda(double *scal, double lam) {
  if (threadIdx.x == 0 && lam > 0.0) scal[1] = lam;
}

// a_new = soft(y + 2 v / L, lambda / L); y = a_new + beta (a_new - a_prev); a_prev = a_new
__global__ void k_fista_update(double *__restrict__ a_prev, double *__restrict__ y,
                               const double *__restrict__ v, const double *__restrict__ scal,
                               double beta, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double L = scal[0], thr = scal[1] / L;
  const double z = y[i] + 2.0 * v[i] / L;
  const double m = fabs(z) - thr;
  const double a = (m > 0.0) ? copysign(m, z) : 0.0;
  y[i] = a + beta * (a - a_prev[i]);
  a_prev[i] = a;
}

// objective[k] = scal[4] + gamma_n scal[5] + lambda scal[6]
__global__ void k_objective(const double *scal, double gamma_n, double *obj, int k) {
  if (threadIdx.x == 0) obj[k] = scal[4] + gamma_n * scal[5] + scal[1] * scal[6];
}

inline dim3 g1(int64_t n) { return dim3(cdiv(n, 256)); }

struct Ctx {
  imgr_s *h;
  int part, n, levels, nb;  // nb: bases of the dictionary
  Bases bases;
  size_t nn;
  FistaWork *fw;
  const double2 *psf_hat;
  hipStream_t s;
  bool serial;
  double gamma_n;
};

// W^T (a - b) -> out (coefficients, nb stacked N^2 blocks), via fw->tmp (nb
// blocks); all bases in one launch per pass, each seeing the input scaled
// by 1 / sqrt(nb) for a dictionary
void dwt2(Ctx &c, const double *a, const double *b, double *out) {
  const int N = c.n;
  const double sc = c.nb > 1 ? 1.0 / std::sqrt((double)c.nb) : 1.0;
  int n = N;
  for (int lev = 0; lev < c.levels; ++lev) {
    const double *src = lev == 0 ? a : out;
    const size_t sstride = lev == 0 ? 0 : c.nn;
    const double *sb = lev == 0 ? b : nullptr;
    const dim3 grid(cdiv((int64_t)n * (n / 2), 256), c.nb);
    hipLaunchKernelGGL(k_dwt<1>, grid, dim3(256), 0, c.s, src, sstride, sb, N, c.fw->tmp, c.nn,
                       N, n, c.fw->hlo, c.bases, lev == 0 ? sc : 1.0);
    hipLaunchKernelGGL(k_dwt<0>, grid, dim3(256), 0, c.s, (const double *)c.fw->tmp, c.nn,
                       (const double *)nullptr, N, out, c.nn, N, n, c.fw->hlo, c.bases, 1.0);
    n /= 2;
  }
}

// W alpha -> out image: each basis' synthesis (all in one launch per pass),
// then for a dictionary the sum over the bases times 1 / sqrt(nb)
void idwt2(Ctx &c, const double *alpha, double *out) {
  const int N = c.n;
  double *xs = c.nb > 1 ? c.fw->xb : out;
  // the detail quadrants are read from alpha itself; the approximation of
  // each finer level is the previous level's synthesis in xs (the coarsest
  // level's is alpha's own)
  int n = N >> (c.levels - 1);
  for (int lev = 0; lev < c.levels; ++lev) {
    const dim3 grid(cdiv((int64_t)n * n, 256), c.nb);
    hipLaunchKernelGGL(k_idwt<0>, grid, dim3(256), 0, c.s, alpha,
                       lev == 0 ? (const double *)nullptr : (const double *)xs, N, c.fw->tmp, N,
                       c.nn, n, c.fw->hlo, c.bases);
    hipLaunchKernelGGL(k_idwt<1>, grid, dim3(256), 0, c.s, (const double *)c.fw->tmp,
                       (const double *)nullptr, N, xs, N, c.nn, n, c.fw->hlo, c.bases);
    n *= 2;
  }
  if (c.nb > 1)
    hipLaunchKernelGGL(k_sum_bases, g1((int64_t)c.nn), dim3(256), 0, c.s, (const double *)xs,
                       c.nb, 1.0 / std::sqrt((double)c.nb), out, (int64_t)c.nn);
}

void psf_conv(Ctx &c, const double *a, double coef, double *out, int acc) {
  const double nd = 2.0 * c.n;
  image_psf_conv64(c.h, a, c.psf_hat, coef / (nd * nd), out, acc, c.fw->work64, c.fw->tmp64, c.s);
}

// out (+)= coef Gamma^(pow) (a - b); own selects Gamma_own, else Gamma_other
void gam(Ctx &c, const double *a, const double *b, bool own, bool squared, double coef,
         double *out, int acc) {
  const bool low = (c.part == IMGR_PART_LOW) == own;
  const int flags = (low ? 1 : 0) | (squared ? 2 : 0);
  image_gamma64(c.h, a, b, flags, coef / ((double)c.n * c.n), out, acc, c.fw->work64, c.fw->tmp64,
                c.s);
}

// u3 = H Gamma_own^2 H x + gamma_n Gamma_other^2 x
void normal_map(Ctx &c, const double *x, double *u3) {
  FistaWork &f = *c.fw;
  psf_conv(c, x, 1.0, f.u1, 0);
  if (c.serial) {
    psf_conv(c, f.u1, 1.0, u3, 0);
  } else if (c.gamma_n == 0.0) {
    gam(c, f.u1, nullptr, true, true, 1.0, f.u2, 0);
    psf_conv(c, f.u2, 1.0, u3, 0);
  } else {
    // Gamma_own^2 H x -> u2 and gamma_n Gamma_other^2 x -> u3 as one pair of
    // filters (one launch per pass), then u3 += H u2: the same sum, term for
    // term, as H u2 + gamma_n Gamma_other^2 x
    const bool low = c.part == IMGR_PART_LOW;  // Gamma_own = Gamma_L at node L
    const double nn = (double)c.n * c.n;
    image_gamma64_pair(c.h, f.u1, (low ? 1 : 0) | 2, 1.0 / nn, f.u2, 0, x, (low ? 0 : 1) | 2,
                       c.gamma_n / nn, u3, 0, c.fw->work64, c.fw->tmp64, c.s);
    psf_conv(c, f.u2, 1.0, u3, 1);
  }
}

void reduce(Ctx &c, const double *a, const double *b, const double *al, int mode, int op,
            double mul, int dst, int64_t count = 0) {
  if (count == 0) count = (int64_t)c.nn;
  const int nb = std::min<int64_t>(kRedBlocks, cdiv(count, 256));
  hipLaunchKernelGGL(k_reduce, dim3(nb), dim3(256), 0, c.s, a, b, al, count, mode, c.fw->part);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, c.s, c.fw->part, nb, op, mul, c.fw->scal,
                     dst);
}

}  // namespace

void fista_enqueue(imgr_s *h, int part, const imgr_fista_params &prm, const float *dirty,
                   const float *rho_other, const float *power_start, float *model_delta,
                   float *model_accum, double *objective, hipStream_t s) {
  const int n = h->N;
  const size_t nn = (size_t)n * n;
  FistaWork &f = h->fista[part];
  // bases: db_p alone, or the dictionary db_1 .. db_p
  const int nbases = prm.dictionary ? prm.vanishing : 1;
  if (f.n != nn || f.vanishing != prm.vanishing || f.n_bases != nbases) {
    for (void *q : {(void *)f.alpha_prev, (void *)f.y, (void *)f.x, (void *)f.u1, (void *)f.u2,
                    (void *)f.u3, (void *)f.cst, (void *)f.tmp, (void *)f.coef, (void *)f.xb,
                    (void *)f.d64, (void *)f.r64, (void *)f.scal, (void *)f.part, (void *)f.hlo,
                    (void *)f.work64, (void *)f.tmp64})
      dev_free(h, q);
    f = FistaWork();
    for (double **b : {&f.alpha_prev, &f.y, &f.coef, &f.tmp})
      *b = (double *)dev_alloc(h, (size_t)nbases * nn * sizeof(double));
    for (double **b : {&f.x, &f.u1, &f.u2, &f.u3, &f.cst, &f.d64, &f.r64})
      *b = (double *)dev_alloc(h, nn * sizeof(double));
    if (nbases > 1) f.xb = (double *)dev_alloc(h, (size_t)nbases * nn * sizeof(double));
    f.work64 = (double2 *)dev_alloc(h, 2 * nn * sizeof(double2));
    f.tmp64 = (double2 *)dev_alloc(h, 4 * nn * sizeof(double2));
    f.scal = (double *)dev_alloc(h, 16 * sizeof(double));
    f.part = (double *)dev_alloc(h, kRedBlocks * sizeof(double));
    std::vector<double> hg;
    for (int b = 0; b < nbases; ++b) {
      const std::vector<double> lo = daubechies(prm.dictionary ? b + 1 : prm.vanishing);
      const int L = (int)lo.size();
      f.hoff.push_back((int)hg.size());
      f.taps.push_back(L);
      for (int j = 0; j < L; ++j) hg.push_back(lo[j]);
      for (int j = 0; j < L; ++j) hg.push_back(((j & 1) ? -1.0 : 1.0) * lo[L - 1 - j]);
    }
    f.hlo = (double *)dev_alloc(h, hg.size() * sizeof(double));
    IMGR_HIP(hipMemcpy(f.hlo, hg.data(), hg.size() * sizeof(double), hipMemcpyHostToDevice));
    f.vanishing = prm.vanishing;
    f.n_bases = nbases;
    f.n = nn;
  }
  const double2 *spec = psf_spectrum64(h, part, s);
  Bases bs{};
  for (int b = 0; b < nbases; ++b) {
    bs.hoff[b] = f.hoff[b];
    bs.taps[b] = f.taps[b];
  }
  Ctx c{h, part, n, prm.levels, nbases, bs, nn, &f, spec, s,
        prm.serial != 0 || h->n_parts == 1, prm.gamma_n};
  const int64_t NC = (int64_t)nbases * (int64_t)nn;  // coefficients
  if (c.serial) c.gamma_n = 0.0;
  const int64_t N2 = (int64_t)nn;
  IMGR_HIP(hipMemsetAsync(f.scal, 0, 16 * sizeof(double), s));
  hipLaunchKernelGGL(k_f32_to_f64, g1(N2), dim3(256), 0, s, dirty, f.d64, N2);
  const bool use_rho = !c.serial && c.gamma_n != 0.0 && rho_other;
  if (use_rho) hipLaunchKernelGGL(k_f32_to_f64, g1(N2), dim3(256), 0, s, rho_other, f.r64, N2);
  // lambda: absolute, or frac * max |dirty|
  if (prm.lambda > 0.0) {
    hipLaunchKernelGGL(k_set_lambda, dim3(1), dim3(64), 0, s, f.scal, prm.lambda);
  } else {
    reduce(c, f.d64, nullptr, nullptr, 1, 1, prm.lambda_frac, 1);
  }
  // L_hat: power iteration on the normal map from power_start
  hipLaunchKernelGGL(k_f32_to_f64, g1(N2), dim3(256), 0, s, power_start, f.x, N2);
  reduce(c, f.x, nullptr, nullptr, 0, 2, 1.0, 2);
  hipLaunchKernelGGL(k_scale_inv, g1(N2), dim3(256), 0, s, f.x, f.scal, 2, N2);
  for (int it = 0; it < prm.power_iters; ++it) {
    normal_map(c, f.x, f.u3);
    reduce(c, f.u3, nullptr, nullptr, 0, 3, 1.0, 2);  // scal[2] = norm, scal[0] = 2 norm
    hipLaunchKernelGGL(k_copy_f64, g1(N2), dim3(256), 0, s, f.u3, f.x, N2);
    hipLaunchKernelGGL(k_scale_inv, g1(N2), dim3(256), 0, s, f.x, f.scal, 2, N2);
  }
  // constant part of the gradient: c = H Gamma_own^2 d + gamma_n Gamma_other rho
  if (c.serial) {
    psf_conv(c, f.d64, 1.0, f.cst, 0);
  } else {
    gam(c, f.d64, nullptr, true, true, 1.0, f.u2, 0);
    psf_conv(c, f.u2, 1.0, f.cst, 0);
    if (use_rho) gam(c, f.r64, nullptr, false, false, c.gamma_n, f.cst, 1);
  }
  // FISTA from alpha = y = 0, t = 1
  IMGR_HIP(hipMemsetAsync(f.alpha_prev, 0, NC * sizeof(double), s));
  IMGR_HIP(hipMemsetAsync(f.y, 0, NC * sizeof(double), s));
  double t = 1.0;
  for (int k = 0; k < prm.n_iter; ++k) {
    idwt2(c, f.y, f.x);                 // x = W y
    normal_map(c, f.x, f.u3);           // u3 = (H Gamma^2 H + gamma Gamma_o^2) x
    dwt2(c, f.cst, f.u3, f.coef);       // v = W^T (c - u3) = -grad / 2
    const double t_next = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
    hipLaunchKernelGGL(k_fista_update, g1(NC), dim3(256), 0, s, f.alpha_prev, f.y, f.coef,
                       f.scal, (t - 1.0) / t_next, NC);
    t = t_next;
    if (objective) {
      idwt2(c, f.alpha_prev, f.x);
      psf_conv(c, f.x, 1.0, f.u1, 0);
      if (c.serial) {
        reduce(c, f.d64, f.u1, nullptr, 0, 0, 1.0, 4);
      } else {
        gam(c, f.d64, f.u1, true, false, 1.0, f.u2, 0);
        reduce(c, f.u2, nullptr, nullptr, 0, 0, 1.0, 4);
        if (use_rho) {
          hipLaunchKernelGGL(k_copy_f64, g1(N2), dim3(256), 0, s, f.r64, f.u2, N2);
          gam(c, f.x, nullptr, false, false, -1.0, f.u2, 1);
          reduce(c, f.u2, nullptr, nullptr, 0, 0, 1.0, 5);
        }
      }
      reduce(c, nullptr, nullptr, f.alpha_prev, 2, 0, 1.0, 6, NC);
      hipLaunchKernelGGL(k_objective, dim3(1), dim3(64), 0, s, f.scal, c.gamma_n, objective, k);
    }
  }
  // ibar = W alpha
  idwt2(c, f.alpha_prev, f.x);
  if (model_delta)
    hipLaunchKernelGGL(k_f64_to_f32, g1(N2), dim3(256), 0, s, f.x, model_delta, N2);
  if (model_accum)
    hipLaunchKernelGGL(k_add_to_f32, g1(N2), dim3(256), 0, s, f.x, model_accum, N2);
  IMGR_HIP(hipGetLastError());
}

void fista_scalars(imgr_s *h, int part, double *lipschitz, double *lambda) {
  double sc[2];
  IMGR_HIP(hipMemcpy(sc, h->fista[part].scal, sizeof(sc), hipMemcpyDeviceToHost));
  if (lipschitz) *lipschitz = sc[0];
  if (lambda) *lambda = sc[1];
}

}  // namespace imgr
