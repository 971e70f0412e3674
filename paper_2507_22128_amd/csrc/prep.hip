// Preparation of a handle (once per imager_create): FP64 coordinate chain,
// uniform weighting (Section 5.1), spatial-frequency partition of Fig. 3
// with ell at the lower median of rho unless given, stable sort of each
// partition by uv block (on the Ng grid of the major cycle and on the 2 Ng
// grid of the PSF), chunk tables, and packing into the 20-byte
// per-visibility stream the de/gridding kernels read.
//
// Every decision that turns a floating-point value into an integer (tap
// cell, block, uniform-weight cell, partition membership) is taken in FP64
// with plain multiply / add / sqrt (no contraction), the same operation
// sequence the CPU oracle uses, so the integer results agree bit for bit.
#pragma clang fp contract(off)

#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"

namespace imgr {
namespace {

constexpr double kC = 299792458.0;

// ---------------------------------------------------------------- coordinates

__global__ void k_coords(int64_t m, const double *__restrict__ uvw,
                         const uint8_t *__restrict__ flag, double lam_scale, double g_scale,
                         double g_half, double p_scale, int n_img, int ng,
                         double *__restrict__ gx, double *__restrict__ gy,
                         double *__restrict__ rho, int32_t *__restrict__ cellkey,
                         uint8_t *__restrict__ valid) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double u = uvw[3 * i] * lam_scale;
  double v = uvw[3 * i + 1] * lam_scale;
  bool ok = flag ? (flag[i] == 0) : true;
  if (!isfinite(u) || !isfinite(v)) {  // unusable coordinates are dropped like flags
    ok = false;
    u = 0.0;
    v = 0.0;
  }
  double x = u * g_scale + g_half;
  double y = v * g_scale + g_half;
  // periodic grid: bring coordinates into [0, Ng) (x == Ng after rounding is cell 0)
  if (x < 0.0 || x >= (double)ng) x = x - (double)ng * floor(x / (double)ng);
  if (y < 0.0 || y >= (double)ng) y = y - (double)ng * floor(y / (double)ng);
  if (!(x < (double)ng)) x = 0.0;
  if (!(y < (double)ng)) y = 0.0;
  gx[i] = x;
  gy[i] = y;
  const double pu = u * p_scale, pv = v * p_scale;
  rho[i] = sqrt(pu * pu + pv * pv);
  long long cu = (long long)floor(pu + 0.5) % n_img;
  long long cv = (long long)floor(pv + 0.5) % n_img;
  if (cu < 0) cu += n_img;
  if (cv < 0) cv += n_img;
  cellkey[i] = (int32_t)(cv * n_img + cu);
  valid[i] = ok ? 1 : 0;
}

__global__ void k_cell_hist(int64_t m, const int32_t *__restrict__ cellkey,
                            const uint8_t *__restrict__ valid, int32_t *__restrict__ counts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m && valid[i]) atomicAdd(&counts[cellkey[i]], 1);
}

__global__ void k_weights(int64_t m, const float *__restrict__ w_in,
                          const int32_t *__restrict__ cellkey, const uint8_t *__restrict__ valid,
                          const int32_t *__restrict__ counts, int uniform,
                          double *__restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double wi = w_in ? (double)w_in[i] : 1.0;
  double r = 0.0;
  if (valid[i]) r = uniform ? wi / (double)counts[cellkey[i]] : wi;
  w[i] = r;
}

__global__ void k_valid_int(int64_t m, const uint8_t *__restrict__ valid,
                            int32_t *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[i] = valid[i] ? 1 : 0;
}

// ---------------------------------------------------------------- radix select

__global__ void k_select_hist(int64_t m, const double *__restrict__ rho,
                              const uint8_t *__restrict__ valid, unsigned long long pmask,
                              unsigned long long pval, int shift, int32_t *__restrict__ hist) {
  __shared__ int32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
    if (!valid[i]) continue;
    const unsigned long long b = (unsigned long long)__double_as_longlong(rho[i]);
    if ((b & pmask) != pval) continue;
    atomicAdd(&h[(b >> shift) & 255], 1);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// ---------------------------------------------------------------- membership, block keys

// which: 0 = V_L (rho <= lo_max), 1 = V_H (rho >= hi_min), 2 = all valid
__global__ void k_member(int64_t m, const double *__restrict__ rho,
                         const uint8_t *__restrict__ valid, int which, double lo_max,
                         double hi_min, int32_t *__restrict__ member) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  bool in = valid[i];
  if (which == 0) in = in && (rho[i] <= lo_max);
  if (which == 1) in = in && (rho[i] >= hi_min);
  member[i] = in ? 1 : 0;
}

// row (column) of the first tap inside its block, from the FP32 offset the
// packed stream stores (so the window kernel, which reads that offset, agrees)
__device__ __forceinline__ int row_in_block(float d, int blk) {
  return min(max((int)d, 0), blk - 1);
}

// sort key: block of the first tap, floor(scale * g) / blk (scale 1 or 2 is
// exact), then the tap's row and column in the block: 64 block + 8 row +
// column; non-members get key 64 nb^2 and sort last
__global__ void k_block_keys(int64_t m, const double *__restrict__ gx,
                             const double *__restrict__ gy, const int32_t *__restrict__ member,
                             double scale, int blk, int nb, uint32_t *__restrict__ keys,
                             int32_t *__restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  uint32_t key = (uint32_t)nb * (uint32_t)nb * 64u;
  if (member[i]) {
    const int cx = (int)floor(gx[i] * scale), cy = (int)floor(gy[i] * scale);
    const int bx = cx / blk, by = cy / blk;
    const int row = row_in_block((float)(gy[i] * scale - (double)(by * blk)), blk);
    const int col = row_in_block((float)(gx[i] * scale - (double)(bx * blk)), blk);
    key = (uint32_t)(by * nb + bx) * 64u + (uint32_t)(row * 8 + col);
  }
  keys[i] = key;
  vals[i] = (int32_t)i;
}

// ---------------------------------------------------------------- scan (int32)

constexpr int kScanBlock = 1024;  // elements per block, 256 threads x 4

__device__ int block_excl_scan(int v, int *sh) {
  // inclusive scan of 256 values in LDS (Hillis-Steele), returns exclusive
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int a = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  const int incl = sh[t];
  __syncthreads();
  return incl - v;
}

__global__ void k_scan_sums(const int32_t *__restrict__ in, int64_t n, int32_t *__restrict__ sums) {
  __shared__ int sh[256];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
  int s = 0;
  for (int k = 0; k < 4; ++k)
    if (base + k < n) s += in[base + k];
  const int ex = block_excl_scan(s, sh);
  if (threadIdx.x == 255) sums[blockIdx.x] = ex + s;
}

__global__ void k_scan_apply(const int32_t *__restrict__ in, int64_t n,
                             const int32_t *__restrict__ offs, int32_t *__restrict__ out) {
  __shared__ int sh[256];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
  int v[4], s = 0;
  for (int k = 0; k < 4; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    s += v[k];
  }
  int run = block_excl_scan(s, sh) + offs[blockIdx.x];
  for (int k = 0; k < 4; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
}

// exclusive scan of n int32 values (in and out may alias); returns the total
int64_t scan_exclusive(imgr_s *h, const int32_t *in, int32_t *out, int64_t n, hipStream_t s) {
  if (n == 0) return 0;
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  int32_t *sums = (int32_t *)dev_alloc(h, (nb + 1) * sizeof(int32_t));
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(256), 0, s, in, n, sums);
  IMGR_HIP(hipGetLastError());
  int64_t total;
  if (nb == 1) {
    int32_t t;
    IMGR_HIP(hipMemcpyAsync(&t, sums, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    IMGR_HIP(hipStreamSynchronize(s));
    total = t;
    IMGR_HIP(hipMemsetAsync(sums, 0, sizeof(int32_t), s));
  } else {
    total = scan_exclusive(h, sums, sums, nb, s);
  }
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, s, in, n, sums, out);
  IMGR_HIP(hipGetLastError());
  IMGR_HIP(hipStreamSynchronize(s));
  dev_free(h, sums);
  return total;
}

// ---------------------------------------------------------------- radix sort
// Stable LSD radix sort of (uint32 key, int32 value) pairs, 8-bit digits.
// Block b owns elements [b * 4096, (b + 1) * 4096) in both kernels.

constexpr int kSortItems = 4096;

__global__ void k_radix_hist(const uint32_t *__restrict__ keys, int64_t n, int shift, int nb,
                             int32_t *__restrict__ counts) {
  __shared__ int32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortItems;
  for (int k = threadIdx.x; k < kSortItems; k += 256) {
    const int64_t i = base + k;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255], 1);
  }
  __syncthreads();
  counts[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

__global__ void k_radix_scatter(const uint32_t *__restrict__ kin, const int32_t *__restrict__ vin,
                                int64_t n, int shift, int nb, const int32_t *__restrict__ offs,
                                uint32_t *__restrict__ kout, int32_t *__restrict__ vout) {
  __shared__ int32_t base[256];
  __shared__ int32_t wcnt[4][256];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  base[t] = offs[(int64_t)t * nb + blockIdx.x];
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int round = 0; round < kSortItems / 256; ++round) {
    const int64_t i = (int64_t)blockIdx.x * kSortItems + round * 256 + t;
    const bool ok = i < n;
    const uint32_t key = ok ? kin[i] : 0u;
    const int d = (key >> shift) & 255;
    for (int w = 0; w < 4; ++w) wcnt[w][t] = 0;
    __syncthreads();
    unsigned long long same = __ballot(ok);
    for (int bit = 0; bit < 8; ++bit) {
      const unsigned long long bb = __ballot(ok && ((d >> bit) & 1));
      same &= ((d >> bit) & 1) ? bb : ~bb;
    }
    const int rank = __popcll(same & below);
    const int cnt = __popcll(same);
    if (ok && rank == cnt - 1) wcnt[wv][d] = cnt;
    __syncthreads();
    if (ok) {
      int pos = base[d] + rank;
      for (int w = 0; w < wv; ++w) pos += wcnt[w][d];
      kout[pos] = key;
      vout[pos] = vin[i];
    }
    __syncthreads();
    base[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
    __syncthreads();
  }
}

void radix_sort(imgr_s *h, uint32_t *&keys, int32_t *&vals, uint32_t *&ktmp, int32_t *&vtmp,
                int64_t n, int key_bits, hipStream_t s) {
  const int nb = (int)((n + kSortItems - 1) / kSortItems);
  int32_t *counts = (int32_t *)dev_alloc(h, (size_t)256 * nb * sizeof(int32_t));
  for (int shift = 0; shift < key_bits; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(256), 0, s, keys, n, shift, nb, counts);
    IMGR_HIP(hipGetLastError());
    scan_exclusive(h, counts, counts, (int64_t)256 * nb, s);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(256), 0, s, keys, vals, n, shift, nb,
                       counts, ktmp, vtmp);
    IMGR_HIP(hipGetLastError());
    std::swap(keys, ktmp);
    std::swap(vals, vtmp);
  }
  IMGR_HIP(hipStreamSynchronize(s));
  dev_free(h, counts);
}

// ---------------------------------------------------------------- blocks, chunks, pack

// first index of the sorted keys[0, n) with key >= k
__device__ __forceinline__ int64_t lower_bound_key(const uint32_t *keys, int64_t n, uint32_t k) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (keys[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// visibilities per block from the sorted keys (block = key / 64); entry
// n_blocks is 0.  Binary searches instead of a histogram: sorted keys would
// send every atomic of a run to one counter
__global__ void k_block_count(int64_t n, const uint32_t *__restrict__ keys, int n_blocks,
                              int32_t *__restrict__ cnt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > n_blocks) return;
  if (t == n_blocks) {
    cnt[t] = 0;
    return;
  }
  const uint32_t k0 = (uint32_t)t * 64u;
  cnt[t] = (int32_t)(lower_bound_key(keys, n, k0 + 64u) - lower_bound_key(keys, n, k0));
}

__global__ void k_chunk_count(int n_blocks, const int32_t *__restrict__ cnt, int cap,
                              int32_t *__restrict__ nch) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n_blocks) nch[t] = (cnt[t] + cap - 1) / cap;
}

// chunks of block t split its cnt[t] visibilities evenly:
// chunk q covers [start + cnt*q/k, start + cnt*(q+1)/k)
__global__ void k_make_chunks(int n_blocks, const int32_t *__restrict__ cnt,
                              const int32_t *__restrict__ bstart,
                              const int32_t *__restrict__ bchunk, int32_t *__restrict__ cblock,
                              int32_t *__restrict__ cbegin) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_blocks) return;
  const int k = bchunk[t + 1] - bchunk[t];
  for (int q = 0; q < k; ++q) {
    cblock[bchunk[t] + q] = t;
    cbegin[bchunk[t] + q] = bstart[t] + (int)(((int64_t)cnt[t] * q) / k);
  }
}

// rows[8 c + j]: visibilities of chunk c whose first tap lies in rows
// 0 .. j of the block (the sort keeps them first); binary search over the
// chunk's packed offsets
__global__ void k_chunk_rows(int n_chunks, const int32_t *__restrict__ cbegin,
                             const float4 *__restrict__ posvis, int blk,
                             int32_t *__restrict__ rows) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_chunks * 8) return;
  const int c = t >> 3, j = t & 7;
  const int b = cbegin[c], e = cbegin[c + 1];
  int lo = b, hi = e;  // first index with row > j
  while (lo < hi) {
    const int mid = lo + ((hi - lo) >> 1);
    if (row_in_block(posvis[mid].y, blk) <= j) lo = mid + 1;
    else hi = mid;
  }
  rows[t] = lo - b;
}

__global__ void k_pack(int64_t n, const uint32_t *__restrict__ keys,
                       const int32_t *__restrict__ idx, const double *__restrict__ gx,
                       const double *__restrict__ gy, double scale, const void *__restrict__ vis,
                       int c128, const double *__restrict__ w64, const int32_t *__restrict__ rank,
                       int blk, int nb, float4 *__restrict__ posvis, float *__restrict__ w,
                       int32_t *__restrict__ orig, int32_t *__restrict__ outpos) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int i = idx[s];
  const int t = (int)(keys[s] >> 6);
  const int bx = t % nb, by = t / nb;
  float re, im;
  if (c128) {
    const double2 z = ((const double2 *)vis)[i];
    re = (float)z.x;
    im = (float)z.y;
  } else {
    const float2 z = ((const float2 *)vis)[i];
    re = z.x;
    im = z.y;
  }
  posvis[s] = make_float4((float)(gx[i] * scale - (double)(bx * blk)),
                          (float)(gy[i] * scale - (double)(by * blk)), re, im);
  w[s] = (float)w64[i];
  orig[s] = i;
  outpos[s] = rank[i];
}

__global__ void k_sum_members(int64_t m, const double *__restrict__ w,
                              const int32_t *__restrict__ member, double *__restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  const int64_t per = (m + gridDim.x - 1) / gridDim.x;
  const int64_t b = (int64_t)blockIdx.x * per, e = min(m, b + per);
  for (int64_t i = b + threadIdx.x; i < e; i += 256)
    if (member[i]) acc += w[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

template <typename T>
T *alloc_n(imgr_s *h, int64_t n) {
  return (T *)dev_alloc(h, (size_t)std::max<int64_t>(n, 1) * sizeof(T));
}

double lower_median_rho(imgr_s *h, int64_t m, const double *rho, const uint8_t *valid,
                        int64_t n_valid, hipStream_t s) {
  int32_t *hist = alloc_n<int32_t>(h, 256);
  unsigned long long pmask = 0, pval = 0;
  int64_t rank = (n_valid - 1) / 2;
  std::vector<int32_t> hh(256);
  for (int shift = 56; shift >= 0; shift -= 8) {
    IMGR_HIP(hipMemsetAsync(hist, 0, 256 * sizeof(int32_t), s));
    hipLaunchKernelGGL(k_select_hist, dim3(1024), dim3(256), 0, s, m, rho, valid, pmask, pval,
                       shift, hist);
    IMGR_HIP(hipGetLastError());
    IMGR_HIP(hipMemcpyAsync(hh.data(), hist, 256 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    IMGR_HIP(hipStreamSynchronize(s));
    int d = 0;
    for (; d < 256; ++d) {
      if (rank < hh[d]) break;
      rank -= hh[d];
    }
    if (d == 256) throw Error{IMGR_EDEVICE, "median selection lost its rank"};
    pmask |= 255ull << shift;
    pval |= (unsigned long long)d << shift;
  }
  dev_free(h, hist);
  double med;
  memcpy(&med, &pval, sizeof(double));
  return med;
}

// B.box from the blocks that hold visibilities: the union of their 16 x 16
// windows (origin block origin - (W/2 - 1)), columns widened to multiples of
// 64 and rows to multiples of 16; the whole grid when a window wraps
void cover_box(imgr_s *h, Bins &B, hipStream_t s) {
  const int n_blocks = B.nb * B.nb, blk = h->blk, H = h->W / 2 - 1, ng = B.ng;
  std::vector<int32_t> bc(n_blocks + 1);
  IMGR_HIP(hipMemcpyAsync(bc.data(), B.block_chunk, (n_blocks + 1) * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
  IMGR_HIP(hipStreamSynchronize(s));
  int x0 = ng, x1 = 0, y0 = ng, y1 = 0;
  bool wraps = false;
  for (int b = 0; b < n_blocks; ++b) {
    if (bc[b + 1] == bc[b]) continue;
    const int wx = (b % B.nb) * blk - H, wy = (b / B.nb) * blk - H;
    if (wx < 0 || wy < 0 || wx + kWin > ng || wy + kWin > ng) wraps = true;
    x0 = std::min(x0, wx);
    x1 = std::max(x1, wx + kWin);
    y0 = std::min(y0, wy);
    y1 = std::max(y1, wy + kWin);
  }
  Box box;
  if (wraps) {
    box = Box{0, ng, 0, ng};
  } else if (x1 > x0) {
    box.x0 = x0 / 64 * 64;
    box.x1 = std::min(ng, (x1 + 63) / 64 * 64);
    box.y0 = y0 / 16 * 16;
    box.y1 = std::min(ng, (y1 + 15) / 16 * 16);
  }
  B.box = box;
}

// (re)build B.chunk_rows from the chunk table and the packed stream
void chunk_rows(imgr_s *h, Bins &B, hipStream_t s) {
  dev_free(h, B.chunk_rows);
  B.chunk_rows = alloc_n<int32_t>(h, 8 * (int64_t)B.n_chunks);
  if (B.n_chunks > 0)
    hipLaunchKernelGGL(k_chunk_rows, dim3(cdiv(8 * (int64_t)B.n_chunks, 256)), dim3(256), 0, s,
                       B.n_chunks, B.chunk_begin, B.posvis, h->blk, B.chunk_rows);
  IMGR_HIP(hipGetLastError());
}

// Sort the members of a partition by block of the (scale * g) grid of side
// ng, cut chunks, and pack the 20-byte per-visibility stream.
void bin_members(imgr_s *h, Bins &B, int64_t m, int64_t n, const int32_t *member,
                 const int32_t *rank, const double *gx, const double *gy, double scale, int ng,
                 const double *w64, const void *vis_dev, int c128, hipStream_t s) {
  const int blk = h->blk;
  B.n = n;
  B.ng = ng;
  B.nb = ng / blk;
  const int n_blocks = B.nb * B.nb;
  const unsigned nbk = cdiv(m, 256);
  uint32_t *keys = alloc_n<uint32_t>(h, m), *ktmp = alloc_n<uint32_t>(h, m);
  int32_t *vals = alloc_n<int32_t>(h, m), *vtmp = alloc_n<int32_t>(h, m);
  hipLaunchKernelGGL(k_block_keys, dim3(nbk), dim3(256), 0, s, m, gx, gy, member, scale, blk,
                     B.nb, keys, vals);
  IMGR_HIP(hipGetLastError());
  // stable sort by block, row and column; non-members (key 64 n_blocks) go last
  IMGR_CHECK(n_blocks < (1 << 25), "grid too large for the 32-bit sort key");
  int key_bits = 0;
  while ((1ll << key_bits) <= 64ll * n_blocks) key_bits += 8;
  radix_sort(h, keys, vals, ktmp, vtmp, m, key_bits, s);
  // block counts, starts, chunks
  int32_t *cnt = alloc_n<int32_t>(h, n_blocks + 1);
  int32_t *bstart = alloc_n<int32_t>(h, n_blocks + 1);
  int32_t *nch = alloc_n<int32_t>(h, n_blocks + 1);
  hipLaunchKernelGGL(k_block_count, dim3(cdiv(n_blocks + 1, 256)), dim3(256), 0, s, n, keys,
                     n_blocks, cnt);
  IMGR_HIP(hipGetLastError());
  scan_exclusive(h, cnt, bstart, n_blocks + 1, s);
  hipLaunchKernelGGL(k_chunk_count, dim3(cdiv(n_blocks + 1, 256)), dim3(256), 0, s, n_blocks + 1,
                     cnt, h->C, nch);
  IMGR_HIP(hipGetLastError());
  B.block_chunk = alloc_n<int32_t>(h, n_blocks + 1);
  // nch[n_blocks] is 0 (cnt[n_blocks] == 0), so the scan's last entry is the total
  B.n_chunks = (int)scan_exclusive(h, nch, B.block_chunk, n_blocks + 1, s);
  B.chunk_block = alloc_n<int32_t>(h, B.n_chunks);
  B.chunk_begin = alloc_n<int32_t>(h, B.n_chunks + 1);
  hipLaunchKernelGGL(k_make_chunks, dim3(cdiv(n_blocks, 256)), dim3(256), 0, s, n_blocks, cnt,
                     bstart, B.block_chunk, B.chunk_block, B.chunk_begin);
  IMGR_HIP(hipGetLastError());
  // launch order: largest chunk first (stable), so the heavy blocks of the
  // dense uv core start early and the tail of the launch is short
  {
    std::vector<int32_t> cb(B.n_chunks + 1);
    if (B.n_chunks > 0)
      IMGR_HIP(hipMemcpyAsync(cb.data(), B.chunk_begin, B.n_chunks * sizeof(int32_t),
                              hipMemcpyDeviceToHost, s));
    IMGR_HIP(hipStreamSynchronize(s));
    cb[B.n_chunks] = (int32_t)n;
    const std::vector<int32_t> ord = largest_first(cb);
    B.order = alloc_n<int32_t>(h, B.n_chunks);
    if (B.n_chunks > 0)
      IMGR_HIP(hipMemcpyAsync(B.order, ord.data(), B.n_chunks * sizeof(int32_t),
                              hipMemcpyHostToDevice, s));
    const int32_t nn = (int32_t)n;
    IMGR_HIP(hipMemcpyAsync(B.chunk_begin + B.n_chunks, &nn, sizeof(int32_t),
                            hipMemcpyHostToDevice, s));
    IMGR_HIP(hipStreamSynchronize(s));
  }
  // pack the per-visibility stream
  B.posvis = alloc_n<float4>(h, n);
  B.w = alloc_n<float>(h, n);
  B.orig = alloc_n<int32_t>(h, n);
  B.outpos = alloc_n<int32_t>(h, n);
  if (n > 0)
    hipLaunchKernelGGL(k_pack, dim3(cdiv(n, 256)), dim3(256), 0, s, n, keys, vals, gx, gy, scale,
                       vis_dev, c128, w64, rank, blk, B.nb, B.posvis, B.w, B.orig, B.outpos);
  IMGR_HIP(hipGetLastError());
  chunk_rows(h, B, s);
  cover_box(h, B, s);
  IMGR_HIP(hipStreamSynchronize(s));
  for (void *q : {(void *)keys, (void *)ktmp, (void *)vals, (void *)vtmp, (void *)cnt,
                  (void *)bstart, (void *)nch})
    dev_free(h, q);
}

// Create-time autotuner of the work layout: for each candidate block side
// (tile) the members of the first partition are binned, and for each
// candidate chunk cap the chunk tables are cut again from the same sort;
// the pair with the least device time of one degrid / grid launch plus its
// flush wins and is kept in h->blk, h->C.  Results of every candidate are
// the same operator up to the FP32 summation order inside a chunk.
void tune_layout(imgr_s *h, int64_t m, int64_t n, const int32_t *member, const int32_t *rank,
                 const double *gx, const double *gy, const double *w64, const void *vis_dev,
                 int c128, hipStream_t s) {
  std::vector<int> blks, caps;
  for (int b : {8, 4})
    if ((h->tile_fixed == 0 || h->tile_fixed == b) && window_supported(h->W, b)) blks.push_back(b);
  if (h->chunk_fixed) caps.push_back(h->chunk_fixed);
  else caps = {4096, 2048, 1024, 512, 256};
  IMGR_CHECK(!blks.empty(), "no tile fits the support");
  const size_t ng2 = (size_t)h->Ng * h->Ng;
  float2 *grid = alloc_n<float2>(h, 2 * ng2);  // zero model grid, then the flush target
  IMGR_HIP(hipMemsetAsync(grid, 0, ng2 * sizeof(float2), s));
  h->tune_log.clear();
  float best = 1e30f;
  int best_blk = blks[0], best_c = caps[0];
  for (int b : blks) {
    h->blk = b;
    h->C = caps[0];
    Bins T;
    bin_members(h, T, m, n, member, rank, gx, gy, 1.0, h->Ng, w64, vis_dev, c128, s);
    for (int c : caps) {
      if (c != h->C) rechunk(h, T, c, s);
      h->C = c;
      float2 *scr = alloc_n<float2>(h, (int64_t)std::max(T.n_chunks, 1) * kWin * kWin);
      const float ms = time_layout(h, T, grid, scr, 3, s);
      dev_free(h, scr);
      h->tune_log.push_back({b, c, ms});
      if (ms < best) {
        best = ms;
        best_blk = b;
        best_c = c;
      }
    }
    free_bins(h, T);
  }
  dev_free(h, grid);
  h->blk = best_blk;
  h->C = best_c;
}

void build_partition(imgr_s *h, int p, int which, int64_t m, const double *gx, const double *gy,
                     const double *rho, const uint8_t *valid, const double *w64,
                     const void *vis_dev, int c128, hipStream_t s) {
  Partition &P = h->part[p];
  const unsigned nbk = cdiv(m, 256);
  int32_t *member = alloc_n<int32_t>(h, m);
  hipLaunchKernelGGL(k_member, dim3(nbk), dim3(256), 0, s, m, rho, valid, which,
                     h->ell + h->delta, h->ell - h->delta, member);
  IMGR_HIP(hipGetLastError());
  // member rank in original order, and the member count
  int32_t *rank = alloc_n<int32_t>(h, m);
  const int64_t n = scan_exclusive(h, member, rank, m, s);
  // summed weight (FP64, fixed order: 256 block partials summed on the host)
  {
    double *part = alloc_n<double>(h, 256);
    hipLaunchKernelGGL(k_sum_members, dim3(256), dim3(256), 0, s, m, w64, member, part);
    IMGR_HIP(hipGetLastError());
    std::vector<double> hp(256);
    IMGR_HIP(hipMemcpyAsync(hp.data(), part, 256 * sizeof(double), hipMemcpyDeviceToHost, s));
    IMGR_HIP(hipStreamSynchronize(s));
    double acc = 0.0;
    for (double v : hp) acc += v;
    P.sum_w = acc;
    dev_free(h, part);
  }
  if (h->tune && p == 0) tune_layout(h, m, n, member, rank, gx, gy, w64, vis_dev, c128, s);
  // the Ng grid of the major cycle, and the 2 Ng grid of the 2N x 2N PSF
  // (same cell size, so grid coordinates double exactly)
  bin_members(h, P.bins, m, n, member, rank, gx, gy, 1.0, h->Ng, w64, vis_dev, c128, s);
  bin_members(h, P.psf_bins, m, n, member, rank, gx, gy, 2.0, 2 * h->Ng, w64, vis_dev, c128, s);
  dev_free(h, member);
  dev_free(h, rank);
}

}  // namespace

// chunks in decreasing size, ties in index order; cb = chunk_begin with
// its closing entry
std::vector<int32_t> largest_first(const std::vector<int32_t> &cb) {
  const int nc = (int)cb.size() - 1;
  std::vector<int32_t> ord(nc);
  for (int c = 0; c < nc; ++c) ord[c] = c;
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
    return cb[a + 1] - cb[a] > cb[b + 1] - cb[b];
  });
  return ord;
}

// Device time of the fused degrid / residual / grid launch plus its flush
// over bins B (zero model grid), the least of `reps` timed repetitions
// after one untimed one.
float time_layout(imgr_s *h, const Bins &B, float2 *grid, float2 *scr, int reps, hipStream_t s) {
  hipEvent_t e0, e1;
  IMGR_HIP(hipEventCreate(&e0));
  IMGR_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  for (int r = 0; r <= reps; ++r) {
    IMGR_HIP(hipEventRecord(e0, s));
    degrid_grid(h, B, MODE_DEGRID_GRID, grid, nullptr, nullptr, scr, s);
    flush_chunks(h, B, scr, grid + (size_t)B.ng * B.ng, s);
    IMGR_HIP(hipEventRecord(e1, s));
    IMGR_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    IMGR_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (r > 0) best = std::min(best, ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

int support_for_tolerance(double tol) {
  if (!(tol > 0.0) || tol >= 1.0) return 0;
  // the kernel's relative error on a 2x padded grid is about
  // 1.0 - 2.3 x 10^(1 - W) at beta = 2.30 W (W = 4 .. 12); a margin of 3
  const int w = (int)std::ceil(1.0 + std::log10(3.0 / tol) - 1e-12);
  for (int c : {4, 6, 8, 10, 12})
    if (c >= w) return c;
  return 0;
}

void free_bins(imgr_s *h, Bins &B) {
  for (void *q : {(void *)B.posvis, (void *)B.w, (void *)B.orig, (void *)B.outpos,
                  (void *)B.chunk_block, (void *)B.chunk_begin, (void *)B.chunk_rows,
                  (void *)B.block_chunk, (void *)B.order})
    dev_free(h, q);
  B = Bins();
}

// Cut the chunk tables of B again for cap C: block b keeps its visibilities
// [start_b, start_b + cnt_b) and is split into ceil(cnt_b / C) near-equal
// chunks, exactly as at create with chunk = C.
void rechunk(imgr_s *h, Bins &B, int C, hipStream_t s) {
  IMGR_CHECK(C >= 16, "chunk cap must be >= 16");
  const int n_blocks = B.nb * B.nb;
  std::vector<int32_t> bc(n_blocks + 1), cb(B.n_chunks + 1);
  IMGR_HIP(hipMemcpyAsync(bc.data(), B.block_chunk, (n_blocks + 1) * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
  IMGR_HIP(hipMemcpyAsync(cb.data(), B.chunk_begin, (B.n_chunks + 1) * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
  IMGR_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> nbc(n_blocks + 1), ncb, ncblk;
  for (int b = 0; b < n_blocks; ++b) {
    nbc[b] = (int32_t)ncblk.size();
    const int32_t c0 = bc[b], c1 = bc[b + 1];
    if (c0 == c1) continue;
    const int32_t start = cb[c0], cnt = cb[c1] - start;
    const int k = (cnt + C - 1) / C;
    for (int q = 0; q < k; ++q) {
      ncblk.push_back(b);
      ncb.push_back(start + (int32_t)(((int64_t)cnt * q) / k));
    }
  }
  const int nc = (int)ncblk.size();
  nbc[n_blocks] = nc;
  ncb.push_back((int32_t)B.n);
  const std::vector<int32_t> ord = largest_first(ncb);
  for (void *q : {(void *)B.chunk_block, (void *)B.chunk_begin, (void *)B.order}) dev_free(h, q);
  B.n_chunks = nc;
  B.chunk_block = alloc_n<int32_t>(h, nc);
  B.chunk_begin = alloc_n<int32_t>(h, nc + 1);
  B.order = alloc_n<int32_t>(h, nc);
  IMGR_HIP(hipMemcpyAsync(B.block_chunk, nbc.data(), (n_blocks + 1) * sizeof(int32_t),
                          hipMemcpyHostToDevice, s));
  if (nc > 0) {
    IMGR_HIP(hipMemcpyAsync(B.chunk_block, ncblk.data(), nc * sizeof(int32_t),
                            hipMemcpyHostToDevice, s));
    IMGR_HIP(hipMemcpyAsync(B.order, ord.data(), nc * sizeof(int32_t), hipMemcpyHostToDevice, s));
  }
  IMGR_HIP(hipMemcpyAsync(B.chunk_begin, ncb.data(), (nc + 1) * sizeof(int32_t),
                          hipMemcpyHostToDevice, s));
  chunk_rows(h, B, s);
  IMGR_HIP(hipStreamSynchronize(s));
}

void prep_build(imgr_s *h, const imgr_vis *vis) {
  hipStream_t s = h->stream;
  const int64_t m = vis->n_vis;
  const int c128 = vis->vis_dtype == IMGR_C128;
  const size_t vbytes = (size_t)m * (c128 ? 16 : 8);
  // inputs on the device
  const double *uvw = vis->uvw;
  const void *vdev = vis->vis;
  const float *wdev = vis->weight;
  const uint8_t *fdev = vis->flag;
  std::vector<void *> staged;
  if (!vis->on_device) {
    double *a = alloc_n<double>(h, 3 * m);
    IMGR_HIP(hipMemcpyAsync(a, vis->uvw, (size_t)m * 24, hipMemcpyHostToDevice, s));
    uvw = a;
    void *b = dev_alloc(h, std::max<size_t>(vbytes, 1));
    IMGR_HIP(hipMemcpyAsync(b, vis->vis, vbytes, hipMemcpyHostToDevice, s));
    vdev = b;
    staged.push_back(a);
    staged.push_back(b);
    if (vis->weight) {
      float *c = alloc_n<float>(h, m);
      IMGR_HIP(hipMemcpyAsync(c, vis->weight, (size_t)m * 4, hipMemcpyHostToDevice, s));
      wdev = c;
      staged.push_back(c);
    }
    if (vis->flag) {
      uint8_t *d = alloc_n<uint8_t>(h, m);
      IMGR_HIP(hipMemcpyAsync(d, vis->flag, (size_t)m, hipMemcpyHostToDevice, s));
      fdev = d;
      staged.push_back(d);
    }
  }
  double *gx = alloc_n<double>(h, m), *gy = alloc_n<double>(h, m), *rho = alloc_n<double>(h, m);
  double *w64 = alloc_n<double>(h, m);
  int32_t *cellkey = alloc_n<int32_t>(h, m);
  uint8_t *valid = alloc_n<uint8_t>(h, m);
  const unsigned nbk = cdiv(m, 256);
  const double lam_scale = vis->freq_hz / kC;
  const double g_scale = (double)h->Ng * h->cell;
  const double p_scale = (double)h->N * h->cell;
  if (m > 0)
    hipLaunchKernelGGL(k_coords, dim3(nbk), dim3(256), 0, s, m, uvw, fdev, lam_scale, g_scale,
                       (double)(h->Ng / 2), p_scale, h->N, h->Ng, gx, gy, rho, cellkey, valid);
  IMGR_HIP(hipGetLastError());
  // uniform weighting: per-cell counts of unflagged visibilities
  int32_t *counts = alloc_n<int32_t>(h, (int64_t)h->N * h->N);
  IMGR_HIP(hipMemsetAsync(counts, 0, (size_t)h->N * h->N * sizeof(int32_t), s));
  if (m > 0) {
    hipLaunchKernelGGL(k_cell_hist, dim3(nbk), dim3(256), 0, s, m, cellkey, valid, counts);
    hipLaunchKernelGGL(k_weights, dim3(nbk), dim3(256), 0, s, m, wdev, cellkey, valid, counts,
                       h->weighting == IMGR_WEIGHT_UNIFORM ? 1 : 0, w64);
  }
  IMGR_HIP(hipGetLastError());
  // number of unflagged visibilities
  {
    int32_t *vi = alloc_n<int32_t>(h, m);
    if (m > 0)
      hipLaunchKernelGGL(k_valid_int, dim3(nbk), dim3(256), 0, s, m, valid, vi);
    IMGR_HIP(hipGetLastError());
    h->n_valid = scan_exclusive(h, vi, vi, m, s);
    dev_free(h, vi);
  }
  if (h->n_valid == 0) throw Error{IMGR_EINVAL, "no unflagged visibilities"};
  // partition radius
  if (h->n_parts == 2 && h->ell < 0) h->ell = lower_median_rho(h, m, rho, valid, h->n_valid, s);
  for (int p = 0; p < h->n_parts; ++p)
    build_partition(h, p, h->n_parts == 1 ? 2 : p, m, gx, gy, rho, valid, w64, vdev, c128, s);
  IMGR_HIP(hipStreamSynchronize(s));
  for (void *q : {(void *)gx, (void *)gy, (void *)rho, (void *)w64, (void *)cellkey,
                  (void *)valid, (void *)counts})
    dev_free(h, q);
  for (void *q : staged) dev_free(h, q);
}

}  // namespace imgr
