// De/gridding of Eq. 2 on the matrix cores (gfx950 MFMA, FP32 in and out).
//
// The visibilities of a partition are binned by the blk x blk block of grid
// cells that holds the first tap of their W x W footprint shifted by
// W/2 - 1, so every footprint of a block lies in one 16 x 16 window of the
// grid (window origin = block origin - (W/2 - 1)).  For the visibilities k
// of one block both halves of Eq. 2 are dense products over that window:
//   degridding (G^dagger F)  v_hat_k = ky_k^T  G  kx_k       (G: model window)
//   gridding   (F^dagger G)  A       = sum_k (r_k ky_k) kx_k^T
// with kx_k, ky_k the separable exponential-of-semicircle tap weights placed
// at the visibility's offset in the window (zero elsewhere).  Both products
// run as v_mfma_f32_16x16x4f32 on batches of 16 visibilities: G kx with the
// window column as inner index for the prediction, and the sum of outer
// products with the visibility as inner index for the accumulation.  The
// residual window therefore stays in accumulator registers for the whole
// chunk; there are no LDS or global atomics.  One wave owns one chunk (at
// most C visibilities of one block), evaluates each of its 2W tap weights
// once per visibility and shares them between the two products through
// LDS, forms the weighted residual w (v - v_hat) in registers, and writes
// its window once.  The flush then adds, for every grid cell, the windows of
// the chunks of the neighbouring blocks in a fixed order in FP64, so the
// grid is reproducible bit for bit.
//
// For W <= 8 the kernel uses a row-group form with half the matrix work: the
// visibilities of a chunk are sorted by the row oy (then the column) of their
// first tap in the block, and a batch of 16 visibilities of one row group
// touches only the W rows oy .. oy + W - 1 of the window.  Eight of those rows (padded with
// zero weights) times {real, imaginary} make the 16 rows of both operands:
//   T[8 c + y][k]   = sum_x G_c[oy + y][x] kx_k[x]          (c = 0 re, 1 im)
//   v_hat_k         = sum_y ky_k[y] (T[y][k] + i T[8 + y][k])
//   A_oy[8 c + y][x] += sum_k part_c(r_k) ky_k[y] kx_k[x]
// so each product is 4 MFMAs per batch instead of 8 (the first one skips the
// K-steps of window columns no footprint of the batch reaches); A_oy is
// added into the residual window (LDS) at row offset oy when the group ends.
#include "common.h"

namespace imgr {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
// word 3 of a raw (untyped) buffer descriptor on gfx9-family chips
constexpr int kBufferWord3 = 0x00020000;

#ifndef IMGR_WIN_WAVES
#define IMGR_WIN_WAVES 4
#endif
// independent waves per workgroup (each owns one chunk and an LDS slice)
constexpr int kWaves = IMGR_WIN_WAVES;

// Address-space views of the argument pointers.  The batched kernels read
// their arguments from a device table, and pointers loaded from memory are
// generic to the compiler: flat accesses, which also count against the LDS
// wait counter and may alias LDS.  Global (1) and constant (4) views give
// plain global and, for wave-uniform table reads, scalar loads.
// (The host pass only parses device code, so the qualifiers are empty there.)
#if defined(__HIP_DEVICE_COMPILE__)
#define AS_GLOBAL __attribute__((address_space(1)))
#define AS_CONST __attribute__((address_space(4)))
#else
#define AS_GLOBAL
#define AS_CONST
#endif
template <class T>
__device__ __forceinline__ AS_GLOBAL T *glb(T *p) {
  return (AS_GLOBAL T *)p;
}
template <class T>
__device__ __forceinline__ const AS_CONST T *cst(const T *p) {
  return (const AS_CONST T *)p;
}
// complex values through the global view (as native two-float vectors)
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld2(const float2 *p, size_t i) {
  const f32x2 v = ((const AS_GLOBAL f32x2 *)p)[i];
  return make_float2(v.x, v.y);
}
// element index below 2^32 (the chunk-window arrays hold fewer than 2^24 windows)
__device__ __forceinline__ float2 ld2u(const float2 *p, unsigned i) {
  const f32x2 v = ((const AS_GLOBAL f32x2 *)p)[i];
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void st2(float2 *p, size_t i, float2 v) {
  ((AS_GLOBAL f32x2 *)p)[i] = f32x2{v.x, v.y};
}

// orders the LDS traffic of one wave around a point where its lanes
// exchange data (no other wave shares the data)
__device__ __forceinline__ void wave_sync() {
  // A wave's LDS instructions are executed in the order it issues them, so
  // a lane reads what another lane of the same wave wrote by an earlier
  // instruction without waiting for the write to complete; only the
  // compiler must not move LDS accesses across this point.
  __asm__ volatile("" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

// sums over the four lanes c16 + 16 g (g = 0..3) of a wave: lanes with
// even g receive (a_0 + a_1) + (a_2 + a_3), lanes with odd g the same sum of
// b.  The first swap exchanges row 1 of a with row 0 of b and row 3 of a
// with row 2 of b, so one add forms the row-pair sums of a in rows 0, 2 and
// of b in rows 1, 3; the second swap adds the two halves.
__device__ __forceinline__ float sum_rows2(float a, float b) {
  auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  const float u = __uint_as_float(p[0]) + __uint_as_float(p[1]);
  auto q = __builtin_amdgcn_permlane32_swap(__float_as_uint(u), __float_as_uint(u), false, false);
  return __uint_as_float(q[0]) + __uint_as_float(q[1]);
}

template <int W, int BLK, int MODE>
__device__ __forceinline__ void window_chunk(const WinArgs &a, int chunk, float *kx_t, float *ky_t,
                                             float2 *r_t) {
  static_assert(BLK + W - 1 <= kWin, "footprints of a block must fit the window");
  constexpr int H = W / 2 - 1;
  constexpr int TPL = (W + 3) / 4;  // taps per lane and axis
  constexpr float kC = 2.0f / W;    // z = (t - H - f) * kC for tap t at fraction f
  constexpr bool kDegrid = (MODE == MODE_DEGRID_GRID || MODE == MODE_DEGRID);
  constexpr bool kGrid = (MODE != MODE_DEGRID);
  constexpr bool kCplx = (MODE != MODE_PSF);
  const float4 *__restrict__ posvis = a.posvis;
  const float *__restrict__ wts = a.wts;
  const int32_t *__restrict__ outpos = a.outpos;
  const float2 *__restrict__ grid_in = a.grid_in;
  const float2 *__restrict__ vis_in = a.vis_in;
  float2 *__restrict__ vis_out = a.vis_out;
  float2 *__restrict__ scratch = a.scratch;
  const int nb = a.nb, ng = a.ng;
  const float bl2e = a.bl2e;

  const int l = threadIdx.x & 63, c16 = l & 15, g = l >> 4;
  const int blk = a.chunk_block[chunk];
  const int wx0 = (blk % nb) * BLK - H, wy0 = (blk / nb) * BLK - H;

  // 1 - z^2 of this lane's taps as quadratics in the fraction f:
  // alpha + beta f - kC^2 f^2 with t0 = t - H
  float qa[TPL], qb[TPL];
#pragma unroll
  for (int q = 0; q < TPL; ++q) {
    const float t0 = (float)(g * TPL + q - H);
    qa[q] = 1.0f - kC * kC * t0 * t0;
    qb[q] = 2.0f * kC * kC * t0;
  }
  constexpr float qc = -kC * kC;

  // model window as the A operand of G kx.  The contraction over the 16
  // window columns runs as 4 K-steps of 4; K-step s of lane group g takes
  // column x = 4 g + s, so lane (c16, g) holds G[y = c16][x = 4 g + s] and
  // feeds the weights of columns 4 g .. 4 g + 3, one 16-byte table read
  float gre[4], gim[4];
  if constexpr (kDegrid) {
    const int gy = (wy0 + c16) & (ng - 1);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int gx = (wx0 + 4 * g + s) & (ng - 1);
      const float2 v = grid_in[(size_t)gy * ng + gx];
      gre[s] = v.x;
      gim[s] = v.y;
    }
  }
  floatx4 acc_re = {0.f, 0.f, 0.f, 0.f}, acc_im = {0.f, 0.f, 0.f, 0.f};

  const int b = a.chunk_begin[chunk], e = a.chunk_begin[chunk + 1];
  // lane (c16, g) works on visibility c16 of each batch; the record of the
  // next batch is loaded while the current one is processed (indices past
  // the chunk are clamped to its last visibility and masked by `valid`)
  float4 pv_next = posvis[min(b + c16, e - 1)];
  float w_next = 0.f;
  if constexpr (kGrid) w_next = wts[min(b + c16, e - 1)];
  for (int base = b; base < e; base += 16) {
    const int v = base + c16;
    const bool valid = v < e;
    const float4 pv = pv_next;
    const float w = valid ? w_next : 0.f;
    pv_next = posvis[min(v + 16, e - 1)];
    if constexpr (kGrid) w_next = wts[min(v + 16, e - 1)];
    // offsets are >= 0, so truncation is the floor
    const int ox = min(max((int)pv.x, 0), BLK - 1);
    const int oy = min(max((int)pv.y, 0), BLK - 1);
    const float fx = pv.x - (float)ox, fy = pv.y - (float)oy;

    // tap weights: clear this lane's quarter of the two table rows of its
    // visibility, then write taps g*TPL .. g*TPL + TPL - 1 of each axis
    // (both tables in natural window order):
    // phi = exp2(beta log2(e) (sqrt(1 - z^2) - 1))
    *(floatx4 *)&kx_t[c16 * 16 + 4 * g] = floatx4{0.f, 0.f, 0.f, 0.f};
    *(floatx4 *)&ky_t[c16 * 16 + 4 * g] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < TPL; ++q) {
      const int t = g * TPL + q;
      if (t < W) {
        const float sx = fmaxf(fmaf(fmaf(qc, fx, qb[q]), fx, qa[q]), 0.0f);
        const float sy = fmaxf(fmaf(fmaf(qc, fy, qb[q]), fy, qa[q]), 0.0f);
        kx_t[c16 * 16 + ox + t] =
            __builtin_amdgcn_exp2f(fmaf(bl2e, __builtin_amdgcn_sqrtf(sx), -bl2e));
        ky_t[c16 * 16 + oy + t] =
            __builtin_amdgcn_exp2f(fmaf(bl2e, __builtin_amdgcn_sqrtf(sy), -bl2e));
      }
    }
    wave_sync();

    float val = 0.f;  // predicted visibility: real part in lanes of even g, imaginary in odd
    if constexpr (kDegrid) {
      float pr = 0.f, pi = 0.f;
      // T[y][k] = sum_x G[y][x] kx_k[x]: B[x = 4 g + s][k = c16]
      const floatx4 bx = *(const floatx4 *)&kx_t[c16 * 16 + 4 * g];
      floatx4 tre = {0.f, 0.f, 0.f, 0.f}, tim = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        tre = __builtin_amdgcn_mfma_f32_16x16x4f32(gre[s], bx[s], tre, 0, 0, 0);
        tim = __builtin_amdgcn_mfma_f32_16x16x4f32(gim[s], bx[s], tim, 0, 0, 0);
      }
      // lane (c16, g) holds T[4 g + r][c16]; v_hat_k = sum_y ky_k[y] T[y][k]
      const floatx4 by = *(const floatx4 *)&ky_t[c16 * 16 + 4 * g];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        pr = fmaf(by[r], tre[r], pr);
        pi = fmaf(by[r], tim[r], pi);
      }
      val = sum_rows2(pr, pi);
    }
    if constexpr (MODE == MODE_DEGRID) {
      if (valid && g < 2) reinterpret_cast<float *>(vis_out)[2 * (size_t)outpos[v] + g] = val;
    }
    if constexpr (kGrid) {
      if constexpr (MODE == MODE_DEGRID_GRID) {
        // lane g = 0 forms the real part of w (v - v_hat), lane g = 1 the imaginary
        if (g < 2) reinterpret_cast<float *>(r_t)[2 * c16 + g] = w * ((g ? pv.w : pv.z) - val);
      } else if (g == 0) {
        float2 r;
        if constexpr (MODE == MODE_GRID) {
          const float2 x = valid ? vis_in[outpos[v]] : make_float2(0.f, 0.f);
          r = make_float2(w * x.x, w * x.y);
        } else {  // MODE_PSF: unit visibilities
          r = make_float2(w, 0.f);
        }
        r_t[c16] = r;
      }
      wave_sync();
      // A[y][x] += sum_k (r_k ky_k[y]) kx_k[x]; K-step s covers k = 4 s + g
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = 4 * s + g;
        const float kyv = ky_t[k * 16 + c16];
        const float kxv = kx_t[k * 16 + c16];
        const float2 rk = r_t[k];
        acc_re = __builtin_amdgcn_mfma_f32_16x16x4f32(rk.x * kyv, kxv, acc_re, 0, 0, 0);
        if constexpr (kCplx)
          acc_im = __builtin_amdgcn_mfma_f32_16x16x4f32(rk.y * kyv, kxv, acc_im, 0, 0, 0);
      }
    }
    wave_sync();  // the tables are rewritten by the next batch
  }

  if constexpr (kGrid) {
    // lane (c16, g) holds A[4 g + r][c16]
    float2 *out = scratch + (size_t)chunk * (kWin * kWin);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      out[(4 * g + r) * kWin + c16] = make_float2(acc_re[r], kCplx ? acc_im[r] : 0.f);
  }
}

// LDS of one wave in the row-group form.  Per batch of 16 visibilities:
//   kxT[x][k]      column weight of visibility k at window column x,
//   ky[k][t]       row weight of visibility k at footprint row t,
//   pT[m][k]       part_c(r_k) ky_k[y] for m = 8 c + y (the gridding product's
//                  left operand), written over ky once ky has been read.
// Row strides: 20 floats for the transposed tables (the 16-byte reads of
// eight consecutive lanes, rows m .. m + 7, land on distinct banks) and 12
// for ky (the same for its 16-byte reads).
constexpr int kS = 20, kKy = 12;
struct RowsLds {
  float kxT[16 * kS];
  union {
    float ky[16 * kKy];
    float pT[16 * kS];
  };
  float g[2][16 * 16];   // model window: real, imaginary planes [row][column]
  float acc[2][16 * 16]; // residual window: real, imaginary planes
};

template <int W, int BLK, int MODE>
__device__ __forceinline__ void window_chunk_rows(const WinArgs &a, int chunk, RowsLds &s) {
  static_assert(W <= 8 && BLK + 7 <= kWin, "the row groups must fit the window");
  constexpr int H = W / 2 - 1;
  constexpr float kC = 2.0f / W;    // z = (t - H - f) * kC for tap t at fraction f
  constexpr bool kDegrid = (MODE == MODE_DEGRID_GRID || MODE == MODE_DEGRID);
  constexpr bool kGrid = (MODE != MODE_DEGRID);
  const float4 *__restrict__ posvis = a.posvis;
  const float *__restrict__ wts = a.wts;
  const int nb = a.nb, ng = a.ng;
  const float bl2e = a.bl2e;

  const int l = threadIdx.x & 63, c16 = l & 15, g = l >> 4;
  chunk = __builtin_amdgcn_readfirstlane(chunk);
  const int blk = cst(a.chunk_block)[chunk];
  const int wx0 = (blk % nb) * BLK - H, wy0 = (blk / nb) * BLK - H;
  const int b = cst(a.chunk_begin)[chunk];
  const AS_CONST int32_t *__restrict__ rows = cst(a.chunk_rows) + 8 * chunk;

  // this lane's taps t = 2 g, 2 g + 1 of each axis (those >= W have zero
  // weight); 1 - z^2 = qa + qb f + qc f^2 with t0 = t - H
  float qa[2], qb[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const float t0 = (float)(2 * g + q - H);
    qa[q] = 1.0f - kC * kC * t0 * t0;
    qb[q] = 2.0f * kC * kC * t0;
  }
  constexpr float qc = -kC * kC;

  // chunk set-up: the model window in LDS (two planes) and a zero residual
  // window
  wave_sync();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int y = 4 * g + r;
    if constexpr (kDegrid) {
      const float2 v = ld2(a.grid_in, (size_t)((wy0 + y) & (ng - 1)) * ng + ((wx0 + c16) & (ng - 1)));
      s.g[0][y * 16 + c16] = v.x;
      s.g[1][y * 16 + c16] = v.y;
    }
    if constexpr (kGrid) {
      s.acc[0][y * 16 + c16] = 0.f;
      s.acc[1][y * 16 + c16] = 0.f;
    }
  }
  // the column-weight table starts clear (lane l: row l / 4, columns
  // 4 (l % 4) ..); each batch writes its taps and takes them out again
  *(floatx4 *)&s.kxT[(l >> 2) * kS + 4 * (l & 3)] = floatx4{0.f, 0.f, 0.f, 0.f};
  wave_sync();

  // row groups: group j holds the chunk's visibilities [b + rows[j-1], b + rows[j])
  int oy = 0, ge = b + rows[0];
  while (ge == b && oy < BLK - 1) ge = b + rows[++oy];
  float foy = (float)oy;
  // A operand of the degridding: in K-step q lane (c16, g) holds
  // G_c[oy + y][4 q + g], c16 = 8 c + y
  floatx4 ga = {0.f, 0.f, 0.f, 0.f};
  auto load_ga = [&]() {
    const float *row = &s.g[c16 >> 3][(oy + (c16 & 7)) * 16 + g];
#pragma unroll
    for (int q = 0; q < 4; ++q) ga[q] = row[4 * q];
  };
  if constexpr (kDegrid) load_ga();
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};

  // lane (c16, g) works on visibility c16 of each batch; the record of the
  // next batch is loaded while the current one is processed.  The stream is
  // read through buffer descriptors with 32-bit offsets.  The record index
  // of a lane past the batch's group is clamped to the group's last
  // visibility; its weight is read through a descriptor that ends at the
  // group, so the hardware returns 0 for it and masks its residual
  const __amdgpu_buffer_rsrc_t pv_rs =
      __builtin_amdgcn_make_buffer_rsrc((void *)posvis, (short)0, a.n * 16, kBufferWord3);
  auto load_pv = [&](int first, int end) {  // record first + c16 (clamped to end - 1)
    const u32x4 r = __builtin_amdgcn_raw_buffer_load_b128(
        pv_rs, (unsigned)min(first + c16, end - 1) * 16u, 0, 0);
    return make_float4(__uint_as_float(r[0]), __uint_as_float(r[1]), __uint_as_float(r[2]),
                       __uint_as_float(r[3]));
  };
  auto load_w = [&](int first, int end) {  // weight of record first + c16, 0 from end on
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)wts, (short)0, end * 4, kBufferWord3);
    return __uint_as_float(
        __builtin_amdgcn_raw_buffer_load_b32(rs, (unsigned)(first + c16) * 4u, 0, 0));
  };
  // two record sets in turn (ping-pong): a batch loads the next batch's
  // records into the other set, so no register copy (which would wait for
  // the load) closes an iteration
  float4 pvA = make_float4(0.f, 0.f, 0.f, 0.f), pvB = pvA;
  float wA = 0.f, wB = 0.f;
  if (ge > b) {
    pvA = load_pv(b, ge);
    if constexpr (kGrid) wA = load_w(b, ge);
  }
  int base = b;
  // one batch on records (pv, w); loads the next batch's into (pvn, wn);
  // false once the chunk is done
  auto batch = [&](const float4 pv, const float w, float4 &pvn, float &wn) -> bool {
    const int v = base + c16;
    const bool valid = c16 < ge - base;
    // the next batch: the rest of this group, else the next nonempty group
    int nbase = base + 16, nge = ge, noy = oy;
    const bool group_end = nbase >= ge;
    if (group_end) {
      nbase = ge;
      while (nge == ge && noy < BLK - 1) nge = b + rows[++noy];
    }
    // (without a next batch, nbase == nge: the loads re-read the last record
    // and return zero weights, which keeps them unconditional)
    const bool more = nbase < nge;
    pvn = load_pv(nbase, nge);
    if constexpr (kGrid) wn = load_w(nbase, nge);
    // offsets are >= 0, so truncation is the floor; the row is the group's
    const int ox = min(max((int)pv.x, 0), BLK - 1);
    const float fx = pv.x - (float)ox, fy = pv.y - foy;

    // tap weights phi = exp2(beta log2(e) (sqrt(1 - z^2) - 1)); every lane
    // writes its column taps at window columns ox + t of the (clear) column
    // table and its row taps t (zero for t >= W)
    float wy2[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int t = 2 * g + q;
      // 1 - z^2 >= 0 on the support; rounding can leave -1e-8 at |z| = 1,
      // so the root takes the magnitude (a free source modifier)
      const float sx = fmaf(fmaf(qc, fx, qb[q]), fx, qa[q]);
      const float sy = fmaf(fmaf(qc, fy, qb[q]), fy, qa[q]);
      const float wx = __builtin_amdgcn_exp2f(fmaf(bl2e, __builtin_amdgcn_sqrtf(fabsf(sx)), -bl2e));
      const float wyv = __builtin_amdgcn_exp2f(fmaf(bl2e, __builtin_amdgcn_sqrtf(fabsf(sy)), -bl2e));
      if (W == 8 || t < W) s.kxT[(ox + t) * kS + c16] = wx;
      wy2[q] = (W == 8 || t < W) ? wyv : 0.f;
    }
    *(float2 *)&s.ky[c16 * kKy + 2 * g] = make_float2(wy2[0], wy2[1]);
    wave_sync();

    // row weights of this lane's footprint rows 4 (g & 1) .. + 3
    const floatx4 by = *(const floatx4 *)&s.ky[c16 * kKy + 4 * (g & 1)];
    float val = 0.f;  // predicted visibility: real part in lanes g = 0, 1, imaginary in g = 2, 3
    if constexpr (kDegrid) {
      // T[m][k] = sum_x Gs[m][x] kx_k[x]: K-step q takes window columns
      // 4 q .. 4 q + 3, B[x = 4 q + g][k = c16].  The stream is sorted by
      // column inside a row group, so lane 0 holds the batch's first column
      // and lane 15 (the last visibility, or a copy of it) the last: K-steps
      // whose four columns no footprint reaches have all-zero weights and
      // are skipped, which leaves the sums unchanged
      const int s_lo = __builtin_amdgcn_readfirstlane(ox) >> 2;
      const int s_hi = (__builtin_amdgcn_readlane(ox, 15) + W - 1) >> 2;
      const float *kxr = &s.kxT[g * kS + c16];
      const floatx4 kq = {kxr[0], kxr[4 * kS], kxr[8 * kS], kxr[12 * kS]};
      floatx4 t = {0.f, 0.f, 0.f, 0.f};
#define MF_(q) t = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[q], kq[q], t, 0, 0, 0)
      switch (s_lo * 4 + s_hi) {  // (first, last) K-step
        case 0: MF_(0); break;
        case 1: MF_(0); MF_(1); break;
        case 2: MF_(0); MF_(1); MF_(2); break;
        case 5: MF_(1); break;
        case 6: MF_(1); MF_(2); break;
        case 7: MF_(1); MF_(2); MF_(3); break;
        case 10: MF_(2); break;
        case 11: MF_(2); MF_(3); break;
        case 15: MF_(3); break;
        default: MF_(0); MF_(1); MF_(2); MF_(3); break;
      }
#undef MF_
      // lane (c16, g) holds T[4 g + r][c16]: part g >> 1, rows 4 (g & 1) + r
      float p = by[0] * t[0];
#pragma unroll
      for (int r = 1; r < 4; ++r) p = fmaf(by[r], t[r], p);
      // rows 0 + 1 and 2 + 3 of the wave: both lanes of a pair get the same sum
      auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(p), __float_as_uint(p), false,
                                                false);
      val = __uint_as_float(q[0]) + __uint_as_float(q[1]);
    }
    if constexpr (MODE == MODE_DEGRID) {
      if (valid && !(g & 1))
        glb(reinterpret_cast<float *>(a.vis_out))[2 * (size_t)glb(a.outpos)[v] + (g >> 1)] = val;
    }
    if constexpr (kGrid) {
      // part c = g >> 1 of the weighted residual (or visibility) r_k of this
      // lane's visibility k = c16
      float rc;
      if constexpr (MODE == MODE_DEGRID_GRID) {
        rc = w * ((g >> 1 ? pv.w : pv.z) - val);
      } else if constexpr (MODE == MODE_GRID) {
        float2 x = make_float2(0.f, 0.f);
        if (valid) x = ld2(a.vis_in, glb(a.outpos)[v]);
        rc = w * (g >> 1 ? x.y : x.x);
      } else {  // MODE_PSF: unit visibilities
        rc = (g >> 1) ? 0.f : w;
      }
      // pT[m][k] = part_c(r_k) ky_k[y] for m = 8 c + y = 4 g + r (over ky:
      // this wave has read it)
#pragma unroll
      for (int r = 0; r < 4; ++r) s.pT[(4 * g + r) * kS + c16] = rc * by[r];
      wave_sync();
      // A_oy[m][x] += sum_k pT[m][k] kxT[x][k]; K-step q covers k = 4 g + q
      const floatx4 pa = *(const floatx4 *)&s.pT[c16 * kS + 4 * g];
      const floatx4 kb = *(const floatx4 *)&s.kxT[c16 * kS + 4 * g];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(pa[q], kb[q], acc, 0, 0, 0);
    }
    wave_sync();  // the tables are rewritten by the next batch
    // clear this lane's column taps again (the wave's LDS accesses execute in
    // issue order, so the next batch's taps land after these zeros)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int t = 2 * g + q;
      if (W == 8 || t < W) s.kxT[(ox + t) * kS + c16] = 0.f;
    }

    if (group_end) {
      if constexpr (kGrid) {
        // lane (c16, g) holds A_oy[4 g + r][c16]: part g >> 1, window row oy + 4 (g & 1) + r
#pragma unroll
        for (int r = 0; r < 4; ++r) s.acc[g >> 1][(oy + 4 * (g & 1) + r) * 16 + c16] += acc[r];
        acc = floatx4{0.f, 0.f, 0.f, 0.f};
        wave_sync();
      }
      if (!more) return false;
      oy = noy;
      foy = (float)oy;
      if constexpr (kDegrid) load_ga();
    }
    base = nbase;
    ge = nge;
    return true;
  };
  if (ge > b) {
    for (;;) {
      if (!batch(pvA, wA, pvB, wB)) break;
      if (!batch(pvB, wB, pvA, wA)) break;
    }
  }

  if constexpr (kGrid) {
    // lane (c16, g) writes window rows 4 g .. 4 g + 3 of column c16
    float2 *out = a.scratch + (size_t)chunk * (kWin * kWin);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int y = 4 * g + r;
      st2(out, y * kWin + c16, make_float2(s.acc[0][y * 16 + c16], s.acc[1][y * 16 + c16]));
    }
  }
}

// one partition's chunks, launch order `order` (largest first)
template <int W, int BLK, int MODE>
__global__ __launch_bounds__(64 * kWaves) void k_window(WinArgs a, const int32_t *__restrict__ order,
                                                       int n_chunks) {
  const int wave = threadIdx.x >> 6;
  // with fewer workgroups than chunk groups each wave takes every
  // (gridDim.x * kWaves)-th chunk of the order; no wave waits for another
  if constexpr (W <= 8) {
    __shared__ __attribute__((aligned(16))) RowsLds lds[kWaves];
    for (int slot = blockIdx.x * kWaves + wave; slot < n_chunks; slot += gridDim.x * kWaves)
      window_chunk_rows<W, BLK, MODE>(a, order[slot], lds[wave]);
  } else {
    // per wave and batch: tap weights of the 16 visibilities over the 16
    // window positions (natural order), and their residuals
    __shared__ __attribute__((aligned(16))) float kx_s[kWaves][16 * 16];
    __shared__ __attribute__((aligned(16))) float ky_s[kWaves][16 * 16];
    __shared__ float2 r_s[kWaves][16];
    for (int slot = blockIdx.x * kWaves + wave; slot < n_chunks; slot += gridDim.x * kWaves)
      window_chunk<W, BLK, MODE>(a, order[slot], kx_s[wave], ky_s[wave], r_s[wave]);
  }
}

// the chunks of many grids (channels) in one launch: order[slot] = (grid,
// chunk), largest chunks of all grids first
template <int W, int BLK, int MODE>
__global__ __launch_bounds__(64 * kWaves) void k_window_batch(const WinArgs *__restrict__ grids,
                                                             const int2 *__restrict__ order,
                                                             int n_slots) {
  const int wave = threadIdx.x >> 6;
  // wave-uniform, so the descriptor is read through scalar loads
  const int slot = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + wave);
  if (slot >= n_slots) return;
  const int2 gc = order[slot];
  const WinArgs a = grids[gc.x];
  if constexpr (W <= 8) {
    __shared__ __attribute__((aligned(16))) RowsLds lds[kWaves];
    window_chunk_rows<W, BLK, MODE>(a, gc.y, lds[wave]);
  } else {
    __shared__ __attribute__((aligned(16))) float kx_s[kWaves][16 * 16];
    __shared__ __attribute__((aligned(16))) float ky_s[kWaves][16 * 16];
    __shared__ float2 r_s[kWaves][16];
    window_chunk<W, BLK, MODE>(a, gc.y, kx_s[wave], ky_s[wave], r_s[wave]);
  }
}

// s + c += x with the rounding error of every FP64 addition kept in c
// (Knuth's TwoSum, exact in IEEE arithmetic): a compensated sum
__device__ __forceinline__ void add_compensated(double &s, double &c, double x) {
  const double t = s + x;
  const double z = t - s;
  c += (s - (t - z)) + (x - z);
  s = t;
}

// One thread per grid cell, 16 x 16 cells per workgroup: compensated FP64
// sum over the chunk windows of the blocks whose window covers the cell
// (fixed order: block row offset, block column offset, chunk), times
// (-1)^(x + y) for the centred inverse DFT that follows.  The workgroup first stages the chunk
// ranges of the blocks around its 16 x 16 cells in LDS; each thread then
// issues the loads of the first chunk of every covering block at once (the
// common case is one chunk per block) and adds the values, and any further
// chunks, in the fixed order.
template <int W, int BLK>
__device__ __forceinline__ void flush_group(const FlushArgs &a, int group) {
  constexpr int H = W / 2 - 1;
  constexpr int R = kWin / BLK;       // block offsets -R .. R can cover a cell
  constexpr int SB = kWin / BLK + 2 * R;  // staged blocks per axis
  constexpr int KA = kWin / BLK;  // covering blocks per axis: exactly KA
  __shared__ int2 rng[SB * SB];
  const int nb = a.nb, ng = a.ng;
  const int gx0 = (a.gx0 + group % a.gnx) * 16, gy0 = (a.gy0 + group / a.gnx) * 16;
  const int bx0 = gx0 / BLK - R, by0 = gy0 / BLK - R;
  for (int i = threadIdx.x; i < SB * SB; i += 256) {
    const int sy = i / SB, sx = i % SB;
    const int n = ((by0 + sy + nb) % nb) * nb + (bx0 + sx + nb) % nb;
    rng[i] = make_int2(glb(a.block_chunk)[n], glb(a.block_chunk)[n + 1]);
  }
  __syncthreads();
  const int cx = gx0 + (threadIdx.x & 15);
  const int cy = gy0 + (threadIdx.x >> 4);
  const int lx = cx % BLK, ly = cy % BLK;
  // the blocks whose window holds the cell: offsets d_lo .. d_lo + KA - 1
  // per axis, d_lo = floor((l + H - 16) / BLK) + 1 (the shift by 8 BLK keeps
  // the division on non-negative values)
  const int dy_lo = (ly + H - kWin + 8 * BLK) / BLK - 8 + 1;
  const int dx_lo = (lx + H - kWin + 8 * BLK) / BLK - 8 + 1;
  const int sy0 = cy / BLK + dy_lo - by0, sx0 = cx / BLK + dx_lo - bx0;
  const int wy0 = ly + H - dy_lo * BLK, wx0 = lx + H - dx_lo * BLK;
  float2 first[KA * KA];
#pragma unroll
  for (int i = 0; i < KA; ++i)
#pragma unroll
    for (int j = 0; j < KA; ++j) {
      const int2 r = rng[(sy0 + i) * SB + sx0 + j];
      const int off = (wy0 - i * BLK) * kWin + wx0 - j * BLK;
      first[i * KA + j] = make_float2(0.f, 0.f);
      if (r.x < r.y) first[i * KA + j] = ld2u(a.scratch, (unsigned)(r.x * (kWin * kWin) + off));
    }
  double re = 0.0, im = 0.0, cre = 0.0, cim = 0.0;
#pragma unroll
  for (int i = 0; i < KA; ++i)
#pragma unroll
    for (int j = 0; j < KA; ++j) {
      const int2 r = rng[(sy0 + i) * SB + sx0 + j];
      if (r.x < r.y) {
        add_compensated(re, cre, (double)first[i * KA + j].x);
        add_compensated(im, cim, (double)first[i * KA + j].y);
        const int off = (wy0 - i * BLK) * kWin + wx0 - j * BLK;
        for (int c = r.x + 1; c < r.y; ++c) {
          const float2 v = ld2u(a.scratch, (unsigned)(c * (kWin * kWin) + off));
          add_compensated(re, cre, (double)v.x);
          add_compensated(im, cim, (double)v.y);
        }
      }
    }
  const float sg = ((cx + cy) & 1) ? -1.f : 1.f;
  st2(a.grid_out, (size_t)cy * ng + cx,
      make_float2(sg * (float)(re + cre), sg * (float)(im + cim)));
}

template <int W, int BLK>
__global__ __launch_bounds__(256) void k_flush(FlushArgs a) {
  flush_group<W, BLK>(a, blockIdx.x);
}

// the flushes of many grids in one launch: grid g owns the workgroups
// [group_start[g], group_start[g + 1])
template <int W, int BLK>
__global__ __launch_bounds__(256) void k_flush_batch(const FlushArgs *__restrict__ grids,
                                                     const int32_t *__restrict__ group_start,
                                                     int n_grids) {
  // the last g with group_start[g] <= blockIdx.x (binary search)
  int lo = 0, hi = n_grids - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (group_start[mid] <= (int)blockIdx.x) lo = mid;
    else hi = mid - 1;
  }
  flush_group<W, BLK>(grids[lo], blockIdx.x - group_start[lo]);
}

template <int W, int BLK>
void launch_window(imgr_s *h, const Bins &B, int mode, const float2 *grid_in,
                   const float2 *vis_in, float2 *vis_out, float2 *scratch, hipStream_t s) {
  const WinArgs a = win_args(h, B, grid_in, vis_in, vis_out, scratch);
  dim3 grid(cdiv(B.n_chunks, kWaves)), block(64 * kWaves);
#define L_(M) hipLaunchKernelGGL((k_window<W, BLK, M>), grid, block, 0, s, a, B.order, B.n_chunks)
  switch (mode) {
    case MODE_DEGRID_GRID: L_(MODE_DEGRID_GRID); break;
    case MODE_GRID: L_(MODE_GRID); break;
    case MODE_DEGRID: L_(MODE_DEGRID); break;
    case MODE_PSF: L_(MODE_PSF); break;
    default: throw Error{IMGR_EINVAL, "unknown de/gridding mode"};
  }
#undef L_
}

template <int W, int BLK>
void launch_flush(const Bins &B, const float2 *scratch, float2 *out, hipStream_t s) {
  const int n_groups = flush_groups(B);
  if (n_groups == 0) return;
  hipLaunchKernelGGL((k_flush<W, BLK>), dim3(n_groups), dim3(256), 0, s, flush_args(B, scratch, out));
}

template <int W, int BLK>
void launch_window_batch(const WinArgs *grids, const int2 *order, int n_slots, hipStream_t s) {
  dim3 grid(cdiv(n_slots, kWaves)), block(64 * kWaves);
  hipLaunchKernelGGL((k_window_batch<W, BLK, MODE_DEGRID_GRID>), grid, block, 0, s, grids, order,
                     n_slots);
}

template <int W, int BLK>
void launch_flush_batch(const FlushArgs *grids, const int32_t *group_start, int n_grids,
                        int n_groups, hipStream_t s) {
  hipLaunchKernelGGL((k_flush_batch<W, BLK>), dim3(n_groups), dim3(256), 0, s, grids, group_start,
                     n_grids);
}

// (W, blk) pairs the library is built for: blk + W - 1 <= 16
#define IMGR_WB_CASES(X) \
  X(4, 8) X(6, 8) X(8, 8) X(4, 4) X(6, 4) X(8, 4) X(10, 4) X(12, 4)

}  // namespace

bool window_supported(int W, int blk) {
#define C_(w, b) if (W == w && blk == b) return true;
  IMGR_WB_CASES(C_)
#undef C_
  return false;
}

void degrid_grid(imgr_s *h, const Bins &B, int mode, const float2 *grid_in, const float2 *vis_in,
                 float2 *vis_out, float2 *scratch, hipStream_t s) {
  if (B.n_chunks == 0) return;
  IMGR_CHECK(B.ng >= 16 && (B.ng & (B.ng - 1)) == 0 && B.nb * h->blk == B.ng, "bin geometry");
#define C_(w, b)                                                                         \
  if (h->W == w && h->blk == b) {                                                        \
    launch_window<w, b>(h, B, mode, grid_in, vis_in, vis_out, scratch, s);               \
    IMGR_HIP(hipGetLastError());                                                         \
    return;                                                                              \
  }
  IMGR_WB_CASES(C_)
#undef C_
  throw Error{IMGR_EINVAL, "unsupported support / block combination"};
}

FlushArgs flush_args(const Bins &B, const float2 *scratch, float2 *grid_out) {
  IMGR_CHECK(B.n_chunks < (1 << 24), "too many chunk windows for 32-bit element offsets");
  FlushArgs a{scratch, B.block_chunk, B.nb, B.ng, grid_out, B.box.x0 / 16, B.box.y0 / 16,
              (B.box.x1 - B.box.x0) / 16};
  return a;
}

WinArgs win_args(const imgr_s *h, const Bins &B, const float2 *grid_in, const float2 *vis_in,
                 float2 *vis_out, float2 *scratch) {
  WinArgs a;
  a.posvis = B.posvis;
  a.wts = B.w;
  a.outpos = B.outpos;
  a.chunk_block = B.chunk_block;
  a.chunk_begin = B.chunk_begin;
  a.chunk_rows = B.chunk_rows;
  // buffer descriptors address the stream with 32-bit byte offsets
  IMGR_CHECK(B.n < (int64_t)1 << 27, "a partition holds at most 2^27 visibilities");
  a.n = (int)B.n;
  a.nb = B.nb;
  a.ng = B.ng;
  a.bl2e = (float)(h->beta * 1.4426950408889634);
  a.grid_in = grid_in;
  a.vis_in = vis_in;
  a.vis_out = vis_out;
  a.scratch = scratch;
  return a;
}

void degrid_grid_batch(int W, int blk, const WinArgs *grids, const int2 *order, int n_slots,
                       hipStream_t s) {
  if (n_slots == 0) return;
#define C_(w, b)                                                 \
  if (W == w && blk == b) {                                      \
    launch_window_batch<w, b>(grids, order, n_slots, s);         \
    IMGR_HIP(hipGetLastError());                                 \
    return;                                                      \
  }
  IMGR_WB_CASES(C_)
#undef C_
  throw Error{IMGR_EINVAL, "unsupported support / block combination"};
}

void flush_batch(int W, int blk, const FlushArgs *grids, const int32_t *group_start, int n_grids,
                 int n_groups, hipStream_t s) {
  if (n_groups == 0) return;
#define C_(w, b)                                                              \
  if (W == w && blk == b) {                                                   \
    launch_flush_batch<w, b>(grids, group_start, n_grids, n_groups, s);       \
    IMGR_HIP(hipGetLastError());                                              \
    return;                                                                   \
  }
  IMGR_WB_CASES(C_)
#undef C_
  throw Error{IMGR_EINVAL, "unsupported support / block combination"};
}

void flush_chunks(imgr_s *h, const Bins &B, const float2 *scratch, float2 *grid_out,
                  hipStream_t s) {
  IMGR_CHECK(B.ng >= 16 && (B.ng & (B.ng - 1)) == 0 && B.nb * h->blk == B.ng, "bin geometry");
#define C_(w, b)                                    \
  if (h->W == w && h->blk == b) {                   \
    launch_flush<w, b>(B, scratch, grid_out, s);    \
    IMGR_HIP(hipGetLastError());                    \
    return;                                         \
  }
  IMGR_WB_CASES(C_)
#undef C_
  throw Error{IMGR_EINVAL, "unsupported support / block combination"};
}

}  // namespace imgr
