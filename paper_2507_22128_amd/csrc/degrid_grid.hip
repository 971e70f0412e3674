// Tile-binned de/gridding with the exponential-of-semicircle kernel.
//
// Visibilities of a partition are sorted by uv tile (T x T grid cells) and
// split into chunks of at most C visibilities.  One workgroup owns one
// chunk: it stages the (T+W-1)^2 model sub-grid of its tile in LDS
// (degridding, G^dagger F of Eq. 2), forms the weighted residual
// w (v - v_hat) in registers, and accumulates it with the same tap weights
// into an LDS sub-grid (gridding, F^dagger G of Eq. 2).  The sub-grid is
// written once per chunk; a separate flush sums, for every grid cell, the
// sub-grids of the chunks of the 3 x 3 neighbouring tiles in a fixed order
// in FP64, so there are no global atomics and the grid is reproducible bit
// for bit.  Tap weights are evaluated in FP32 from the offset of the
// visibility inside its tile, which the prep step derives from FP64
// coordinates.
#include "common.h"

namespace imgr {
namespace {

// ES kernel phi(z) = exp(beta (sqrt(1 - z^2) - 1)), here as
// exp2(beta log2(e) (sqrt(max(1 - z^2, 0)) - 1)).
template <int W>
__device__ __forceinline__ void es_taps(float f, float bl2e, float *k) {
  constexpr int H = W / 2 - 1;
  constexpr float inv_half = 2.0f / W;
#pragma unroll
  for (int i = 0; i < W; ++i) {
    const float z = ((float)(i - H) - f) * inv_half;
    const float t = fmaxf(1.0f - z * z, 0.0f);
    k[i] = __builtin_amdgcn_exp2f(bl2e * (__builtin_amdgcn_sqrtf(t) - 1.0f));
  }
}

template <int T, int W, int MODE>
struct ChunkLds {
  static constexpr int S = T + W - 1;
  static constexpr bool kDegrid = (MODE == MODE_DEGRID_GRID || MODE == MODE_DEGRID);
  static constexpr bool kGrid = (MODE != MODE_DEGRID);
  static constexpr bool kIm = kGrid && (MODE != MODE_PSF);
};

// posvis: {dx, dy, re, im} with dx, dy the offsets (cells) of the
// visibility from its tile origin on the grid the prep step binned for;
// `pos_scale` = 2 grids on the twice finer PSF grid with tiles of 2T.
template <int T, int W, int MODE>
__global__ __launch_bounds__(256) void k_chunk(
    const float4 *__restrict__ posvis, const float *__restrict__ wts,
    const int32_t *__restrict__ outpos, const int32_t *__restrict__ chunk_tile,
    const int32_t *__restrict__ chunk_begin, int ntx, int ng, float pos_scale, float bl2e,
    const float2 *__restrict__ grid_in, const float2 *__restrict__ vis_in,
    float2 *__restrict__ vis_out, float2 *__restrict__ scratch) {
  using L = ChunkLds<T, W, MODE>;
  constexpr int S = L::S;
  constexpr int H = W / 2 - 1;
  __shared__ float2 sub[L::kDegrid ? S * S : 1];
  __shared__ float acc_re[L::kGrid ? S * S : 1];
  __shared__ float acc_im[L::kIm ? S * S : 1];

  const int chunk = blockIdx.x;
  const int tile = chunk_tile[chunk];
  const int tx = tile % ntx, ty = tile / ntx;
  const int gx0 = tx * T - H, gy0 = ty * T - H;
  const int t = threadIdx.x;

  if constexpr (L::kDegrid) {
    for (int i = t; i < S * S; i += 256) {
      const int sy = i / S, sx = i - sy * S;
      const int gx = (gx0 + sx) & (ng - 1), gy = (gy0 + sy) & (ng - 1);
      sub[i] = grid_in[(size_t)gy * ng + gx];
    }
  }
  if constexpr (L::kGrid) {
    for (int i = t; i < S * S; i += 256) {
      acc_re[i] = 0.f;
      if constexpr (L::kIm) acc_im[i] = 0.f;
    }
  }
  __syncthreads();

  const int b = chunk_begin[chunk], e = chunk_begin[chunk + 1];
  for (int v = b + t; v < e; v += 256) {
    const float4 pv = posvis[v];
    const float dx = pv.x * pos_scale, dy = pv.y * pos_scale;
    const int cx = min(max((int)floorf(dx), 0), T - 1);
    const int cy = min(max((int)floorf(dy), 0), T - 1);
    float kx[W], ky[W];
    es_taps<W>(dx - (float)cx, bl2e, kx);
    es_taps<W>(dy - (float)cy, bl2e, ky);

    float2 pred = make_float2(0.f, 0.f);
    if constexpr (L::kDegrid) {
#pragma unroll
      for (int j = 0; j < W; ++j) {
        const float2 *srow = sub + (cy + j) * S + cx;
        float rx = 0.f, ry = 0.f;
#pragma unroll
        for (int i = 0; i < W; ++i) {
          const float2 g = srow[i];
          rx = fmaf(kx[i], g.x, rx);
          ry = fmaf(kx[i], g.y, ry);
        }
        pred.x = fmaf(ky[j], rx, pred.x);
        pred.y = fmaf(ky[j], ry, pred.y);
      }
    }
    if constexpr (MODE == MODE_DEGRID) {
      vis_out[outpos[v]] = pred;
    } else {
      const float w = wts[v];
      float2 r;
      if constexpr (MODE == MODE_DEGRID_GRID) {
        r = make_float2(w * (pv.z - pred.x), w * (pv.w - pred.y));
      } else if constexpr (MODE == MODE_GRID) {
        const float2 x = vis_in[outpos[v]];
        r = make_float2(w * x.x, w * x.y);
      } else {  // MODE_PSF
        r = make_float2(w, 0.f);
      }
#pragma unroll
      for (int j = 0; j < W; ++j) {
        const float rx = r.x * ky[j], ry = r.y * ky[j];
        const int base = (cy + j) * S + cx;
#pragma unroll
        for (int i = 0; i < W; ++i) {
          atomicAdd(&acc_re[base + i], rx * kx[i]);
          if constexpr (MODE != MODE_PSF) atomicAdd(&acc_im[base + i], ry * kx[i]);
        }
      }
    }
  }

  if constexpr (L::kGrid) {
    __syncthreads();
    float2 *out = scratch + (size_t)chunk * S * S;
    for (int i = t; i < S * S; i += 256)
      out[i] = make_float2(acc_re[i], L::kIm ? acc_im[i] : 0.f);
  }
}

// For every cell of output tile blockIdx.x: FP64 sum over the chunks of the
// 3 x 3 neighbouring tiles (fixed order: row offset, column offset, chunk),
// times (-1)^(x + y) for the centred inverse DFT that follows.
template <int T, int W>
__global__ __launch_bounds__(256) void k_flush(const float2 *__restrict__ scratch,
                                               const int32_t *__restrict__ tile_chunk, int ntx,
                                               int ng, float2 *__restrict__ grid_out) {
  constexpr int S = T + W - 1;
  constexpr int H = W / 2 - 1;
  const int tile = blockIdx.x;
  const int tx = tile % ntx, ty = tile / ntx;
  for (int i = threadIdx.x; i < T * T; i += 256) {
    const int lx = i % T, ly = i / T;
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int dty = -1; dty <= 1; ++dty) {
      const int sy = ly + H - dty * T;
      if (sy < 0 || sy >= S) continue;
      const int nty = (ty + dty + ntx) % ntx;
#pragma unroll
      for (int dtx = -1; dtx <= 1; ++dtx) {
        const int sx = lx + H - dtx * T;
        if (sx < 0 || sx >= S) continue;
        const int ntxx = (tx + dtx + ntx) % ntx;
        const int n = nty * ntx + ntxx;
        const int c0 = tile_chunk[n], c1 = tile_chunk[n + 1];
        for (int c = c0; c < c1; ++c) {
          const float2 v = scratch[(size_t)c * S * S + sy * S + sx];
          re += (double)v.x;
          im += (double)v.y;
        }
      }
    }
    const int gx = tx * T + lx, gy = ty * T + ly;
    const float sg = ((gx + gy) & 1) ? -1.f : 1.f;
    grid_out[(size_t)gy * ng + gx] = make_float2(sg * (float)re, sg * (float)im);
  }
}

template <int T, int W>
void chunk_launch(imgr_s *h, const Partition &P, int mode, float pos_scale, int ng,
                  const float2 *grid_in, const float2 *vis_in, float2 *vis_out, float2 *scratch,
                  hipStream_t s) {
  const float bl2e = (float)(h->beta * 1.4426950408889634);
  const int ntx = ng / T;
  dim3 grid(P.n_chunks), block(256);
  if constexpr (T > 32) {
    // tiles of 64 cells only serve the PSF grid (2T for T = 32): the fused
    // modes would need more LDS than a workgroup may hold
    if (mode != MODE_PSF) throw Error{IMGR_EINVAL, "tile 64 is PSF-only"};
    hipLaunchKernelGGL((k_chunk<T, W, MODE_PSF>), grid, block, 0, s, P.posvis, P.w, P.outpos,
                       P.chunk_tile, P.chunk_begin, ntx, ng, pos_scale, bl2e, grid_in, vis_in,
                       vis_out, scratch);
    return;
  } else {
  switch (mode) {
    case MODE_DEGRID_GRID:
      hipLaunchKernelGGL((k_chunk<T, W, MODE_DEGRID_GRID>), grid, block, 0, s, P.posvis, P.w,
                         P.outpos, P.chunk_tile, P.chunk_begin, ntx, ng, pos_scale, bl2e, grid_in,
                         vis_in, vis_out, scratch);
      break;
    case MODE_GRID:
      hipLaunchKernelGGL((k_chunk<T, W, MODE_GRID>), grid, block, 0, s, P.posvis, P.w, P.outpos,
                         P.chunk_tile, P.chunk_begin, ntx, ng, pos_scale, bl2e, grid_in, vis_in,
                         vis_out, scratch);
      break;
    case MODE_DEGRID:
      hipLaunchKernelGGL((k_chunk<T, W, MODE_DEGRID>), grid, block, 0, s, P.posvis, P.w,
                         P.outpos, P.chunk_tile, P.chunk_begin, ntx, ng, pos_scale, bl2e, grid_in,
                         vis_in, vis_out, scratch);
      break;
    case MODE_PSF:
      hipLaunchKernelGGL((k_chunk<T, W, MODE_PSF>), grid, block, 0, s, P.posvis, P.w, P.outpos,
                         P.chunk_tile, P.chunk_begin, ntx, ng, pos_scale, bl2e, grid_in, vis_in,
                         vis_out, scratch);
      break;
  }
  }
}

template <int W>
void chunk_dispatch_t(imgr_s *h, const Partition &P, int mode, int tile, float pos_scale, int ng,
                      const float2 *grid_in, const float2 *vis_in, float2 *vis_out,
                      float2 *scratch, hipStream_t s) {
  switch (tile) {
    case 16: chunk_launch<16, W>(h, P, mode, pos_scale, ng, grid_in, vis_in, vis_out, scratch, s); break;
    case 32: chunk_launch<32, W>(h, P, mode, pos_scale, ng, grid_in, vis_in, vis_out, scratch, s); break;
    case 64: chunk_launch<64, W>(h, P, mode, pos_scale, ng, grid_in, vis_in, vis_out, scratch, s); break;
    default: throw Error{IMGR_EINVAL, "unsupported tile"};
  }
}

}  // namespace

void degrid_grid(imgr_s *h, int p, int mode, const float2 *grid_in, const float2 *vis_in,
                 float2 *vis_out, int tile, int ng, float2 *scratch, hipStream_t s) {
  const Partition &P = h->part[p];
  if (P.n_chunks == 0) return;
  const float pos_scale = (float)tile / (float)h->T;
  switch (h->W) {
    case 4: chunk_dispatch_t<4>(h, P, mode, tile, pos_scale, ng, grid_in, vis_in, vis_out, scratch, s); break;
    case 6: chunk_dispatch_t<6>(h, P, mode, tile, pos_scale, ng, grid_in, vis_in, vis_out, scratch, s); break;
    case 8: chunk_dispatch_t<8>(h, P, mode, tile, pos_scale, ng, grid_in, vis_in, vis_out, scratch, s); break;
    case 10: chunk_dispatch_t<10>(h, P, mode, tile, pos_scale, ng, grid_in, vis_in, vis_out, scratch, s); break;
    case 12: chunk_dispatch_t<12>(h, P, mode, tile, pos_scale, ng, grid_in, vis_in, vis_out, scratch, s); break;
    default: throw Error{IMGR_EINVAL, "unsupported support W"};
  }
  IMGR_HIP(hipGetLastError());
}

template <int W>
static void flush_t(int tile, const int32_t *tile_chunk, int ntx, int ng, const float2 *scratch,
                    float2 *out, hipStream_t s) {
  dim3 grid(ntx * ntx), block(256);
  switch (tile) {
    case 16: hipLaunchKernelGGL((k_flush<16, W>), grid, block, 0, s, scratch, tile_chunk, ntx, ng, out); break;
    case 32: hipLaunchKernelGGL((k_flush<32, W>), grid, block, 0, s, scratch, tile_chunk, ntx, ng, out); break;
    case 64: hipLaunchKernelGGL((k_flush<64, W>), grid, block, 0, s, scratch, tile_chunk, ntx, ng, out); break;
    default: throw Error{IMGR_EINVAL, "unsupported tile"};
  }
}

void flush_chunks(imgr_s *h, int p, int tile, int ng, const float2 *scratch, float2 *grid_out,
                  hipStream_t s) {
  const Partition &P = h->part[p];
  const int ntx = ng / tile;
  switch (h->W) {
    case 4: flush_t<4>(tile, P.tile_chunk, ntx, ng, scratch, grid_out, s); break;
    case 6: flush_t<6>(tile, P.tile_chunk, ntx, ng, scratch, grid_out, s); break;
    case 8: flush_t<8>(tile, P.tile_chunk, ntx, ng, scratch, grid_out, s); break;
    case 10: flush_t<10>(tile, P.tile_chunk, ntx, ng, scratch, grid_out, s); break;
    case 12: flush_t<12>(tile, P.tile_chunk, ntx, ng, scratch, grid_out, s); break;
    default: throw Error{IMGR_EINVAL, "unsupported support W"};
  }
  IMGR_HIP(hipGetLastError());
}

}  // namespace imgr
