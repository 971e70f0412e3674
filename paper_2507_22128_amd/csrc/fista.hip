// Sparsity-regularised minor cycle (Eqs. 4 and 5, Section 4.1): FISTA on
// the coefficients of an orthonormal periodized Daubechies wavelet basis.
//
//   f(alpha) = ||Gamma_own (d - H W alpha)||^2 + gamma_n ||rho - Gamma_other W alpha||^2
//   grad f   = -2 W^T (c - H Gamma_own^2 H x - gamma_n Gamma_other^2 x),  x = W alpha,
//   c        = H Gamma_own^2 d + gamma_n Gamma_other rho  (once per minor cycle)
//
// H (the node's 2N x 2N PSF) and Gamma are applied with the fused transform
// pipelines of fft.hip (H and Gamma are self-adjoint: the PSF is even, the
// filters real and radial).  The wavelet transforms run one fused
// launch per level (both axes through LDS).  Everything runs in FP64 (the
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
//
// One launch per level and transform, both axes fused through LDS: a
// workgroup stages the input patch its outputs need (periodic wrap), filters
// it along the rows into LDS, then along the columns.  Every sum runs over
// the taps in increasing order with one FMA per tap, as a plain loop would.
// Block sizes are powers of two (N is one), so the wrap is a mask.

constexpr int kMaxBases = 10;  // dictionary bases: db1 .. db10 at most
constexpr int kMaxTaps = 20;   // db10

// filters of the dictionary's bases (blockIdx.z = basis)
struct Bases {
  int hoff[kMaxBases], taps[kMaxBases];
};

// analysis: a workgroup makes kAnaK x kAnaK outputs of each of the four
// subbands from an input patch of (2 kAnaK + T - 2)^2 samples
constexpr int kAnaK = 16;
constexpr int kAnaS = 2 * kAnaK + kMaxTaps - 2;  // patch side, 50 at most
// synthesis: a workgroup makes kSynM x kSynM outputs from patches of
// (kSynM / 2 + T / 2 - 1)^2 coefficients of each subband
constexpr int kSynM = 32;
constexpr int kSynC = kSynM / 2 + kMaxTaps / 2 - 1;  // patch side, 25 at most
constexpr int kAnaLds = kAnaS * kAnaS + kAnaS * 2 * kAnaK;
constexpr int kSynLds = 4 * kSynC * kSynC + kSynM * 2 * kSynC;
constexpr int kWavLds = kAnaLds > kSynLds ? kAnaLds : kSynLds;  // doubles
// one work item per thread in the single-pass stages
static_assert(kAnaS * (kAnaK / 4) <= 256 && (kAnaK / 2) * 2 * kAnaK == 256, "analysis tiling");
static_assert(kSynM * (kSynM / 4) == 256, "synthesis tiling");

// W^T, one level: the top-left n x n block of src (minus b, times sc) ->
// the detail subbands at their Mallat places in out (row stride out_ld)
// and the approximation into ll (row stride ll_ld):
//   a[k] = sum_j h_j x[(2k + j) mod n],  d[k] = sum_j g_j x[(2k + j) mod n]
// along the rows first, then along the columns.
template <int T>
__device__ __forceinline__ void dwt_level_body(const double *__restrict__ src, int src_ld,
                                               const double *__restrict__ b, double sc,
                                               double *__restrict__ out, int out_ld,
                                               double *__restrict__ ll, int ll_ld, int n,
                                               const double *__restrict__ hg, double *lds) {
  constexpr int S = 2 * kAnaK + T - 2;
  double *x = lds;                    // [S][kAnaS] input patch
  double *mid = lds + kAnaS * kAnaS;  // [S][2 kAnaK] row-filtered: a | d
  const int tid = threadIdx.x;
  const int half = n >> 1, mask = n - 1;
  const int ky0 = blockIdx.y * kAnaK, kx0 = blockIdx.x * kAnaK;
  {
    // every load of the patch is issued before the first LDS store
    constexpr int R = (S + 3) / 4;
    const int c = tid & 63;
    const int gx = (2 * kx0 + c) & mask;
    double v[R], w[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int r = (tid >> 6) + 4 * i;
      const size_t off = (size_t)((2 * ky0 + r) & mask) * src_ld + gx;
      if (c < S && r < S) {
        v[i] = src[off];
        if (b) w[i] = b[off];
      }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int r = (tid >> 6) + 4 * i;
      if (c < S && r < S) {
        double y = v[i];
        if (b) y -= w[i];
        if (sc != 1.0) y *= sc;
        x[r * kAnaS + c] = y;
      }
    }
  }
  __syncthreads();
  // along the rows: a thread makes 4 adjacent outputs of one patch row from
  // the T + 6 samples they span (read once from LDS)
  if (tid < S * (kAnaK / 4)) {
    const int r = tid >> 2, kg = tid & 3;
    const double *xr = x + r * kAnaS + 8 * kg;
    double v[T + 6];
#pragma unroll
    for (int m = 0; m < T + 6; ++m) v[m] = xr[m];
    double lo[4], hi[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      lo[e] = 0.0;
      hi[e] = 0.0;
#pragma unroll
      for (int j = 0; j < T; ++j) {
        lo[e] = fma(hg[j], v[2 * e + j], lo[e]);
        hi[e] = fma(hg[T + j], v[2 * e + j], hi[e]);
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      mid[r * 2 * kAnaK + 4 * kg + e] = lo[e];
      mid[r * 2 * kAnaK + kAnaK + 4 * kg + e] = hi[e];
    }
  }
  __syncthreads();
  // along the columns: a thread makes 2 adjacent outputs of one column
  {
    const int k = tid & (kAnaK - 1), hx = (tid / kAnaK) & 1, kyp = tid / (2 * kAnaK);
    const double *mc = mid + 4 * kyp * 2 * kAnaK + hx * kAnaK + k;
    double v[T + 2];
#pragma unroll
    for (int m = 0; m < T + 2; ++m) v[m] = mc[m * 2 * kAnaK];
    const int gx = kx0 + k;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      double lo = 0.0, hi = 0.0;
#pragma unroll
      for (int j = 0; j < T; ++j) {
        lo = fma(hg[j], v[2 * e + j], lo);
        hi = fma(hg[T + j], v[2 * e + j], hi);
      }
      const int gy = ky0 + 2 * kyp + e;
      if (gy < half && gx < half) {
        if (hx == 0)
          ll[(size_t)gy * ll_ld + gx] = lo;
        else
          out[(size_t)gy * out_ld + half + gx] = lo;
        out[(size_t)(half + gy) * out_ld + hx * half + gx] = hi;
      }
    }
  }
}

// src, ll, out: basis p at + p * bstride (src_bs 0: one input for all bases)
__global__ __launch_bounds__(256) void k_dwt_level(const double *__restrict__ src, size_t src_bs,
                                                   int src_ld, const double *__restrict__ b,
                                                   double sc, double *__restrict__ out,
                                                   int out_ld, double *__restrict__ ll,
                                                   int ll_ld, size_t bstride, int n,
                                                   const double *__restrict__ hlo, Bases bs) {
  __shared__ double lds[kWavLds];
  const int p = blockIdx.z;
  const double *__restrict__ hg = hlo + bs.hoff[p];
  src += p * src_bs;
  out += p * bstride;
  ll += p * bstride;
  switch (bs.taps[p]) {
#define TAPS_(T) \
  case T: dwt_level_body<T>(src, src_ld, b, sc, out, out_ld, ll, ll_ld, n, hg, lds); break;
    TAPS_(2) TAPS_(4) TAPS_(6) TAPS_(8) TAPS_(10) TAPS_(12) TAPS_(14) TAPS_(16) TAPS_(18)
    TAPS_(20)
#undef TAPS_
    default: break;  // the host admits db1 .. db10 only
  }
}

// W, one level (the transpose of the analysis level): the n x n block of
// out from the n/2 x n/2 approximation ll (row stride ll_ld) and the three
// detail subbands of the coefficient array c (row stride c_ld):
//   x[m] = sum over j with m - j even of h_j a[k] + g_j d[k],  k = ((m - j) mod n) / 2
// along the columns first, then along the rows.
template <int T>
__device__ __forceinline__ void idwt_level_body(const double *__restrict__ c, int c_ld,
                                                const double *__restrict__ ll, int ll_ld,
                                                double *__restrict__ out, int out_ld, int n,
                                                const double *__restrict__ hg, double *lds) {
  constexpr int C = kSynM / 2 + T / 2 - 1;
  double *q = lds;                        // [2 (a|d along y)][2 (a|d along x)][C][kSynC]
  double *t = lds + 4 * kSynC * kSynC;    // [kSynM][2][kSynC] column-synthesised
  const int tid = threadIdx.x;
  const int half = n >> 1, hmask = half - 1;
  const int my0 = blockIdx.y * kSynM, mx0 = blockIdx.x * kSynM;
  // coefficient k' = (m - j) / 2 spans my0 / 2 - T / 2 + 1 ... my0 / 2 + kSynM / 2 - 1
  const int kyb = my0 / 2 - T / 2 + 1, kxb = mx0 / 2 - T / 2 + 1;
  {
    // every load of the four patches is issued before the first LDS store
    constexpr int R = (4 * C + 7) / 8;
    const int ix = tid & 31;
    const int kx = (kxb + ix) & hmask;
    double v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int row = (tid >> 5) + 8 * i;
      const int quad = row / C, iy = row % C;
      const int hy = quad >> 1, hx = quad & 1;
      const int ky = (kyb + iy) & hmask;
      if (ix < C && row < 4 * C)
        v[i] = (hy == 0 && hx == 0) ? ll[(size_t)ky * ll_ld + kx]
                                    : c[(size_t)(hy * half + ky) * c_ld + hx * half + kx];
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int row = (tid >> 5) + 8 * i;
      if (ix < C && row < 4 * C) q[((row / C) * kSynC + row % C) * kSynC + ix] = v[i];
    }
  }
  __syncthreads();
  // Output rows (columns) 2p and 2p + 1 take the same coefficients k = p - i
  // (i < T / 2), with the even and the odd taps.  A thread makes two such
  // pairs, from the T / 2 + 1 coefficients of each half that they span.
  // along y: 16 row pairs x 2 halves along x x 32 patch columns (25 used)
  for (int it = tid; it < (kSynM / 4) * 2 * 32; it += 256) {
    const int ix = it & 31, hx = (it >> 5) & 1, pg = it >> 6;
    if (ix < C) {
      const double *qa = q + (hx * kSynC + 2 * pg) * kSynC + ix;        // a along y
      const double *qd = q + ((2 + hx) * kSynC + 2 * pg) * kSynC + ix;  // d along y
      double va[T / 2 + 1], vd[T / 2 + 1];
#pragma unroll
      for (int m = 0; m <= T / 2; ++m) {
        va[m] = qa[m * kSynC];
        vd[m] = qd[m * kSynC];
      }
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        double ev = 0.0, od = 0.0;
#pragma unroll
        for (int i = 0; i < T / 2; ++i) {
          const int m = e + T / 2 - 1 - i;
          ev = fma(hg[2 * i], va[m], ev);
          ev = fma(hg[T + 2 * i], vd[m], ev);
          od = fma(hg[2 * i + 1], va[m], od);
          od = fma(hg[T + 2 * i + 1], vd[m], od);
        }
        const int my = 2 * (2 * pg + e);
        t[(my * 2 + hx) * kSynC + ix] = ev;
        t[((my + 1) * 2 + hx) * kSynC + ix] = od;
      }
    }
  }
  __syncthreads();
  // along x: 32 rows x 8 groups of 4 adjacent outputs
  {
    const int g = tid & 7, my = tid >> 3;
    const double *ta = t + (my * 2) * kSynC + 2 * g, *td = ta + kSynC;
    double ua[T / 2 + 1], ud[T / 2 + 1];
#pragma unroll
    for (int m = 0; m <= T / 2; ++m) {
      ua[m] = ta[m];
      ud[m] = td[m];
    }
    double r[4];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      double ev = 0.0, od = 0.0;
#pragma unroll
      for (int i = 0; i < T / 2; ++i) {
        const int m = e + T / 2 - 1 - i;
        ev = fma(hg[2 * i], ua[m], ev);
        ev = fma(hg[T + 2 * i], ud[m], ev);
        od = fma(hg[2 * i + 1], ua[m], od);
        od = fma(hg[T + 2 * i + 1], ud[m], od);
      }
      r[2 * e] = ev;
      r[2 * e + 1] = od;
    }
    if (my0 + my < n) {
      double *o = out + (size_t)(my0 + my) * out_ld + mx0 + 4 * g;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (mx0 + 4 * g + e < n) o[e] = r[e];
    }
  }
}

// c, ll, out: basis p at + p * bstride
__global__ __launch_bounds__(256) void k_idwt_level(const double *__restrict__ c, int c_ld,
                                                    const double *__restrict__ ll, int ll_ld,
                                                    double *__restrict__ out, int out_ld,
                                                    size_t bstride, int n,
                                                    const double *__restrict__ hlo, Bases bs) {
  __shared__ double lds[kWavLds];
  const int p = blockIdx.z;
  const double *__restrict__ hg = hlo + bs.hoff[p];
  c += p * bstride;
  ll += p * bstride;
  out += p * bstride;
  switch (bs.taps[p]) {
#define TAPS_(T) \
  case T: idwt_level_body<T>(c, c_ld, ll, ll_ld, out, out_ld, n, hg, lds); break;
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

// W^T (a - b) -> out (coefficients, nb stacked N^2 blocks): one launch per
// level for all bases, each seeing the input scaled by 1 / sqrt(nb) for a
// dictionary.  The approximation of every level but the last goes to
// fw->tmp (halves 0 and N^2 / 2 of each basis' block, alternately, so a
// level never overwrites its own input); the details go to out.
void dwt2(Ctx &c, const double *a, const double *b, double *out) {
  const int N = c.n;
  const double sc = c.nb > 1 ? 1.0 / std::sqrt((double)c.nb) : 1.0;
  const double *src = a;
  size_t src_bs = 0;  // one image for every basis
  int src_ld = N, n = N;
  for (int lev = 0; lev < c.levels; ++lev) {
    const bool last = lev == c.levels - 1;
    double *ll = last ? out : c.fw->tmp + ((lev & 1) ? c.nn / 2 : 0);
    const int ll_ld = last ? N : n / 2;
    const int tiles = (int)cdiv(n / 2, kAnaK);
    hipLaunchKernelGGL(k_dwt_level, dim3(tiles, tiles, c.nb), dim3(256), 0, c.s, src, src_bs,
                       src_ld, lev == 0 ? b : (const double *)nullptr, lev == 0 ? sc : 1.0, out,
                       N, ll, ll_ld, c.nn, n, (const double *)c.fw->hlo, c.bases);
    src = ll;
    src_bs = c.nn;
    src_ld = ll_ld;
    n /= 2;
  }
}

// W alpha -> out image: each basis' synthesis (all in one launch per level),
// then for a dictionary the sum over the bases times 1 / sqrt(nb).  The
// coarsest level takes its approximation from alpha; each finer level takes
// the previous level's output, kept in fw->tmp (alternate halves).
void idwt2(Ctx &c, const double *alpha, double *out) {
  const int N = c.n;
  double *xs = c.nb > 1 ? c.fw->xb : out;
  const double *ll = alpha;
  int ll_ld = N;
  int n = N >> (c.levels - 1);
  for (int lev = 0; lev < c.levels; ++lev) {
    const bool last = lev == c.levels - 1;
    double *dst = last ? xs : c.fw->tmp + ((lev & 1) ? c.nn / 2 : 0);
    const int dst_ld = last ? N : n;
    const int tiles = (int)cdiv(n, kSynM);
    hipLaunchKernelGGL(k_idwt_level, dim3(tiles, tiles, c.nb), dim3(256), 0, c.s, alpha, N, ll,
                       ll_ld, dst, dst_ld, c.nn, n, (const double *)c.fw->hlo, c.bases);
    ll = dst;
    ll_ld = dst_ld;
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
                   const float *psf, const float *rho_other, const float *power_start,
                   float *model_delta, float *model_accum, double *objective, hipStream_t s) {
  const int n = h->N;
  const size_t nn = (size_t)n * n;
  FistaWork &f = h->fista[part];
  // bases: db_p alone, or the dictionary db_1 .. db_p
  const int nbases = prm.dictionary ? prm.vanishing : 1;
  if (f.n != nn || f.vanishing != prm.vanishing || f.n_bases != nbases) {
    for (void *q : {(void *)f.alpha_prev, (void *)f.y, (void *)f.x, (void *)f.u1, (void *)f.u2,
                    (void *)f.u3, (void *)f.cst, (void *)f.tmp, (void *)f.coef, (void *)f.xb,
                    (void *)f.d64, (void *)f.r64, (void *)f.scal, (void *)f.part, (void *)f.hlo,
                    (void *)f.work64, (void *)f.tmp64, (void *)f.psf_ext})
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
  const double2 *spec;
  if (psf) {
    if (!f.psf_ext) f.psf_ext = (double2 *)dev_alloc(h, 4 * nn * sizeof(double2));
    psf_spectrum64_of(h, psf, f.psf_ext, f.tmp64, s);
    spec = f.psf_ext;
  } else {
    spec = psf_spectrum64(h, part, s);
  }
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
