// Hand-written radix-8/4/2 Stockham FFTs for gfx950.
//
// The 2-D transforms of Eq. 2 (F and F^dagger, Section 2) are split into
//   * row passes: one workgroup per row, the whole row in LDS (<= 8192
//     points, padded one slot per 32 against bank conflicts of the
//     strided Stockham stores);
//   * column passes: a four-step split L = P * Q done in two kernels over
//     blocks of CW = 32 adjacent columns (256-byte coalesced row segments in
//     FP32; 64 columns halve the workgroup count, which leaves much of the
//     chip idle at these sizes, and 16 columns measured slower); in LDS each
//     group of CW threads owns the block's columns, one lane per column.
//     Transforms of 64 points keep both radix-8 passes in registers and
//     exchange through LDS once (col64_regs).
// Zero rows of a padded input are never read and rows outside a crop are
// never written.  The centred transform of the gridder (grid cell g holds
// frequency g - Ng/2) is the plain DFT with (-1)^index modulation on both
// sides, which the load and store of the passes apply.
#include "common.h"

namespace imgr {
namespace {

__device__ __forceinline__ int padi(int i) { return i + (i >> 5); }

// width of the column passes' blocks where the split allows it (ColWidth)
constexpr int kColWant = 32;

template <int DIR, class C>
__device__ __forceinline__ C tw_get(const C *__restrict__ tw, int idx) {
  C t = tw[idx];
  if (DIR > 0) t.y = -t.y;
  return t;
}

// multiply by -i (forward, DIR < 0) or +i (inverse)
template <int DIR, class C>
__device__ __forceinline__ C mul_mi(C a) {
  return DIR < 0 ? mkc<C>(a.y, -a.x) : mkc<C>(-a.y, a.x);
}

template <int DIR, class C>
__device__ __forceinline__ void dft4(C &y0, C &y1, C &y2, C &y3) {
  C t0 = cadd(y0, y2), t1 = csub(y0, y2), t2 = cadd(y1, y3), t3 = mul_mi<DIR>(csub(y1, y3));
  y0 = cadd(t0, t2);
  y2 = csub(t0, t2);
  y1 = cadd(t1, t3);
  y3 = csub(t1, t3);
}

template <int R, int DIR, class C>
__device__ __forceinline__ void dft(C *x) {
  typedef typename Real<C>::T RT;
  if constexpr (R == 2) {
    C a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  } else if constexpr (R == 4) {
    dft4<DIR>(x[0], x[1], x[2], x[3]);
  } else {
    static_assert(R == 8, "radix");
    const RT h = (RT)0.70710678118654752440L;
    C a0 = cadd(x[0], x[4]), a1 = cadd(x[1], x[5]), a2 = cadd(x[2], x[6]), a3 = cadd(x[3], x[7]);
    C b0 = csub(x[0], x[4]), b1 = csub(x[1], x[5]), b2 = csub(x[2], x[6]), b3 = csub(x[3], x[7]);
    // b_n *= W8^n, W8 = exp(DIR * 2 pi i / 8)
    if (DIR < 0) {
      b1 = mkc<C>((b1.x + b1.y) * h, (b1.y - b1.x) * h);
      b3 = mkc<C>((b3.y - b3.x) * h, -(b3.x + b3.y) * h);
    } else {
      b1 = mkc<C>((b1.x - b1.y) * h, (b1.x + b1.y) * h);
      b3 = mkc<C>(-(b3.x + b3.y) * h, (b3.x - b3.y) * h);
    }
    b2 = mul_mi<DIR>(b2);
    dft4<DIR>(a0, a1, a2, a3);
    dft4<DIR>(b0, b1, b2, b3);
    x[0] = a0; x[2] = a1; x[4] = a2; x[6] = a3;
    x[1] = b0; x[3] = b1; x[5] = b2; x[7] = b3;
  }
}

// Row twiddles w_L^m = exp(-2 pi i m / L), m < L, as the product of two
// short tables staged in LDS: w_L^m = w_L^(B floor(m / B)) w_L^(m mod B),
// B the power of two nearest sqrt L from above.  Every index of the first
// passes is a multiple of B and takes w_L^0 = 1 from the second table, an
// exact product; the tables take B + L / B entries instead of L, which
// leaves the LDS to the rows (twice the resident rows per CU at L = 4096).
template <int L>
struct RowTw {
  static constexpr int log2l() {
    int k = 0;
    while ((1 << k) < L) ++k;
    return k;
  }
  static constexpr int B = 1 << ((log2l() + 1) / 2), H = L / B, SIZE = B + H;
};
template <int B, class C>
struct TwoLevel {
  const C *lo, *hi;  // lo[m] = w_L^m (m < B), hi[h] = w_L^(B h)
};
template <int DIR, int B, class C>
__device__ __forceinline__ C tw_get(const TwoLevel<B, C> &tw, int idx) {
  C t = cmul(tw.hi[idx / B], tw.lo[idx & (B - 1)]);
  if (DIR > 0) t.y = -t.y;
  return t;
}

// One sequence of length L in padded LDS, NT threads, Stockham passes from
// sub-length NS upward (radix 8 while possible, then 4 or 2).  tw gives
// w_L^m, m < L (a table pointer or a TwoLevel view).
template <int L, int NT, int NS, int DIR, class C, class TW>
__device__ __forceinline__ void stockham_seq(C *s, const TW &tw, int t) {
  if constexpr (NS < L) {
    constexpr int R = (L / NS >= 8) ? 8 : (L / NS);
    constexpr int NB = L / R;
    constexpr int PER = (NB + NT - 1) / NT;
    C x[PER][R];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = t + q * NT;
      if ((NB % NT) == 0 || j < NB) {
#pragma unroll
        for (int r = 0; r < R; ++r) x[q][r] = s[padi(j + r * NB)];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = t + q * NT;
      if ((NB % NT) == 0 || j < NB) {
        const int k = j & (NS - 1);
        if constexpr (NS > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r)
            x[q][r] = cmul(x[q][r], tw_get<DIR>(tw, r * k * (L / (NS * R))));
        }
        dft<R, DIR>(x[q]);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) s[padi(base + r * NS)] = x[q][r];
      }
    }
    __syncthreads();
    stockham_seq<L, NT, NS * R, DIR, C, TW>(s, tw, t);
  }
}

// The last Stockham pass of a length-L sequence: its sub-length NS and radix R.
template <int L>
struct LastPass {
  static constexpr int ns() {
    int n = 1;
    while (true) {
      const int r = (L / n >= 8) ? 8 : L / n;
      if (n * r >= L) return n;
      n *= r;
    }
  }
  static constexpr int NS = ns(), R = L / NS;
};

// Stockham passes from sub-length NS on, with the last pass left in
// registers instead of LDS: after the call, o[q][r] holds element
// j + r * LastPass<L>::NS of the transform, j = t + q * NT (for j below
// LastPass<L>::NS).  The same arithmetic as stockham_seq, one LDS store and
// load of the whole sequence fewer.
template <int L, int NT, int NS, int DIR, class C, class TW, int PO, int RO>
__device__ __forceinline__ void stockham_out(C *s, const TW &tw, int t, C (&o)[PO][RO]) {
  constexpr int R = (L / NS >= 8) ? 8 : (L / NS);
  constexpr int NB = L / R;
  constexpr int PER = (NB + NT - 1) / NT;
  C x[PER][R];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = t + q * NT;
    if ((NB % NT) == 0 || j < NB) {
#pragma unroll
      for (int r = 0; r < R; ++r) x[q][r] = s[padi(j + r * NB)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = t + q * NT;
    if ((NB % NT) == 0 || j < NB) {
      const int k = j & (NS - 1);
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r)
          x[q][r] = cmul(x[q][r], tw_get<DIR>(tw, r * k * (L / (NS * R))));
      }
      dft<R, DIR>(x[q]);
    }
  }
  if constexpr (NS * R == L) {
    static_assert(PER == PO && R == RO, "last pass shape");
#pragma unroll
    for (int q = 0; q < PER; ++q)
#pragma unroll
      for (int r = 0; r < R; ++r) o[q][r] = x[q][r];
  } else {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = t + q * NT;
      if ((NB % NT) == 0 || j < NB) {
        const int k = j & (NS - 1);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) s[padi(base + r * NS)] = x[q][r];
      }
    }
    __syncthreads();
    stockham_out<L, NT, NS * R, DIR, C, TW, PO, RO>(s, tw, t, o);
  }
}

// Rows with L / 8 threads: thread t loads elements t + q L/8, exactly the
// inputs of its butterfly in the first pass (sub-length 1, radix 8, no
// twiddles), which then runs on the loaded registers.
template <int L, int NT>
constexpr bool first_pass_in_regs() {
  return NT * 8 == L;
}

template <int L, int DIR, class C>
__device__ __forceinline__ void first_pass_regs(C *s, C (&v)[8], int t) {
  dft<8, DIR>(v);
#pragma unroll
  for (int r = 0; r < 8; ++r) s[padi(8 * t + r)] = v[r];
}

// CW sequences of length LEN stored as s[pos][CW] (column c = t % CW), 256
// threads in G = 256 / CW groups: group g does butterflies j = g, g + G, ...
// (with CW = 64 a group is a wave, and its row index and twiddles are
// wave-uniform)
template <int LEN, int NS, int DIR, class C, int CW>
__device__ __forceinline__ void stockham_cols(C *s, const C *__restrict__ tw, int t) {
  if constexpr (NS < LEN) {
    constexpr int R = (LEN / NS >= 8) ? 8 : (LEN / NS);
    constexpr int NB = LEN / R;
    constexpr int G = 256 / CW;
    constexpr int PER = (NB + G - 1) / G;
    const int c = t % CW;
    const int wv = CW == 64 ? __builtin_amdgcn_readfirstlane(t >> 6) : t / CW;
    C x[PER][R];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = wv + G * q;
      if (j < NB) {
#pragma unroll
        for (int r = 0; r < R; ++r) x[q][r] = s[(j + r * NB) * CW + c];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = wv + G * q;
      if (j < NB) {
        const int k = j & (NS - 1);
        if constexpr (NS > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r)
            x[q][r] = cmul(x[q][r], tw_get<DIR>(tw, r * k * (kTwMax / (NS * R))));
        }
        dft<R, DIR>(x[q]);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) s[(base + r * NS) * CW + c] = x[q][r];
      }
    }
    __syncthreads();
    stockham_cols<LEN, NS * R, DIR, C, CW>(s, tw, t);
  }
}

// Column DFTs of length 64 over CW = 32 columns with 256 threads, the two
// radix-8 passes of stockham_cols kept in registers: group g = t / 32 owns
// butterfly g of each pass and lane c = t % 32 its column.  On entry v[r]
// holds row g + 8 r of column c (as the column passes load their tile), on
// exit output row g + 8 r; one LDS round trip between the passes instead of
// the tile's store, two round trips and reload.  The same arithmetic as
// stockham_cols<64, 1, DIR, C, 32>.
template <int DIR, class C>
__device__ __forceinline__ void col64_regs(C *s, const C *__restrict__ tw, int t, C (&v)[8]) {
  constexpr int CW = 32;
  const int g = t / CW, c = t % CW;
  dft<8, DIR>(v);
#pragma unroll
  for (int r = 0; r < 8; ++r) s[(8 * g + r) * CW + c] = v[r];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 8; ++r) v[r] = s[(g + 8 * r) * CW + c];
#pragma unroll
  for (int r = 1; r < 8; ++r) v[r] = cmul(v[r], tw_get<DIR>(tw, r * g * (kTwMax / 64)));
  dft<8, DIR>(v);
}

// stage the two tables of RowTw<L> into twl (lo then hi) from the per-length
// tables (entry L + m of twr holds w_L^m)
template <int L, int NT, class C>
__device__ __forceinline__ void stage_twiddles(C *twl, const C *__restrict__ twr) {
  constexpr int B = RowTw<L>::B, H = RowTw<L>::H;
  static_assert(B + H <= NT, "one entry per thread");
  const int t = threadIdx.x;
  if (t < B + H) twl[t] = twr[L + (t < B ? t : (t - B) * B)];
}

// the view of the staged tables that stockham_seq takes
template <int L, class C>
__device__ __forceinline__ TwoLevel<RowTw<L>::B, C> row_tw(const C *twl) {
  return TwoLevel<RowTw<L>::B, C>{twl, twl + RowTw<L>::B};
}

template <int L>
struct RowThreads {
  static constexpr int v = (L / 8 < 64) ? 64 : ((L / 8 > 1024) ? 1024 : L / 8);
};

// ---------------------------------------------------------------- row kernels

// model (n x n f32) [+ model_add] -> rows (n x L complex): correction 1/psi on
// both axes, centred zero-padding, (-1)^(x+y) modulation, forward row DFT.
// The rows are real, so one workgroup transforms rows 2p and 2p + 1 at
// once as the real and imaginary parts of one complex sequence z = a + i b,
// and separates them by the symmetry of real spectra:
// A[k] = (Z[k] + conj Z[L-k]) / 2, B[k] = (Z[k] - conj Z[L-k]) / 2i.
template <int L>
__device__ __forceinline__ void rows_model_body(const float *__restrict__ model,
                                                const float *__restrict__ model_add,
                                                const float *__restrict__ cinv, int n,
                                                float2 *__restrict__ rows,
                                                const float2 *__restrict__ twr, int c_lo,
                                                int c_hi, int pair) {
  constexpr int NT = RowThreads<L>::v;
  __shared__ float2 s[L + L / 32];
  __shared__ float2 twl[RowTw<L>::SIZE];
  const int o = (L - n) / 2;
  const int ra = 2 * pair, rb = ra + 1;
  const int ya = o + ra;
  const float cya = cinv[ra], cyb = cinv[rb];
  constexpr int PER = L / NT;
  float va[PER], vb[PER], c[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int x = threadIdx.x + q * NT;
    va[q] = vb[q] = c[q] = 0.f;
    if (x >= o && x < o + n) {
      va[q] = model[(size_t)ra * n + x - o];
      vb[q] = model[(size_t)rb * n + x - o];
      c[q] = cinv[x - o];
    }
  }
  if (model_add) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int x = threadIdx.x + q * NT;
      if (x >= o && x < o + n) {
        va[q] += model_add[(size_t)ra * n + x - o];
        vb[q] += model_add[(size_t)rb * n + x - o];
      }
    }
  }
  // the twiddle loads go out behind the row loads: one wait covers both
  stage_twiddles<L, NT, float2>(twl, twr);
  float2 w[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int x = threadIdx.x + q * NT;
    float wa = va[q] * (c[q] * cya), wb = vb[q] * (c[q] * cyb);
    // (-1)^(x + y): rows ra and rb = ra + 1 have opposite signs
    if ((x + ya) & 1) wa = -wa;
    else wb = -wb;
    w[q] = make_float2(wa, wb);
  }
  if constexpr (first_pass_in_regs<L, NT>()) {
    first_pass_regs<L, -1>(s, w, threadIdx.x);
    __syncthreads();
    stockham_seq<L, NT, 8, -1>(s, row_tw<L>(twl), threadIdx.x);
  } else {
#pragma unroll
    for (int q = 0; q < PER; ++q) s[padi(threadIdx.x + q * NT)] = w[q];
    __syncthreads();
    stockham_seq<L, NT, 1, -1>(s, row_tw<L>(twl), threadIdx.x);
  }
  // only the columns [c_lo, c_hi) are ever read
  for (int x = c_lo + threadIdx.x; x < c_hi; x += NT) {
    const float2 zx = s[padi(x)], zm = s[padi((L - x) & (L - 1))];
    rows[(size_t)ra * L + x] = make_float2(0.5f * (zx.x + zm.x), 0.5f * (zx.y - zm.y));
    rows[(size_t)rb * L + x] = make_float2(0.5f * (zx.y + zm.y), 0.5f * (zm.x - zx.x));
  }
}

template <int L>
__global__ __launch_bounds__(RowThreads<L>::v) void k_rows_model(
    const float *__restrict__ model, const float *__restrict__ model_add,
    const float *__restrict__ cinv, int n, float2 *__restrict__ rows,
    const float2 *__restrict__ twr, int c_lo, int c_hi) {
  rows_model_body<L>(model, model_add, cinv, n, rows, twr, c_lo, c_hi, blockIdx.x);
}

// rows (n x L complex) -> image (n x n f32): inverse row DFT, crop of the
// centre, (-1)^(x+y), correction 1/psi on both axes, real part, scale.
// Columns outside [c_lo, c_hi) are zero and not read.
template <int L>
__device__ __forceinline__ void rows_image_body(const float2 *__restrict__ rows,
                                                const float *__restrict__ cinv, int n,
                                                float scale, float *__restrict__ out,
                                                const float2 *__restrict__ twr, int c_lo,
                                                int c_hi, int r) {
  constexpr int NT = RowThreads<L>::v;
  __shared__ float2 s[L + L / 32];
  __shared__ float2 twl[RowTw<L>::SIZE];
  const int o = (L - n) / 2;
  const int y = o + r;
  constexpr int PER = L / NT;
  float2 v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int x = threadIdx.x + q * NT;
    v[q] = (x >= c_lo && x < c_hi) ? rows[(size_t)r * L + x] : make_float2(0.f, 0.f);
  }
  stage_twiddles<L, NT, float2>(twl, twr);
  const float cy = cinv[r] * scale;
  if constexpr (first_pass_in_regs<L, NT>()) {
    // first and last passes in registers: the loaded values feed the first
    // pass, the last pass's outputs go straight to the image
    constexpr int NS = LastPass<L>::NS, RL = LastPass<L>::R, PL = (NS + NT - 1) / NT;
    first_pass_regs<L, 1>(s, v, threadIdx.x);
    __syncthreads();
    float2 z[PL][RL];
    stockham_out<L, NT, 8, 1>(s, row_tw<L>(twl), threadIdx.x, z);
#pragma unroll
    for (int q = 0; q < PL; ++q) {
      const int j = threadIdx.x + q * NT;
#pragma unroll
      for (int k = 0; k < RL; ++k) {
        const int x = j + k * NS, ix = x - o;
        if (j < NS && ix >= 0 && ix < n) {
          float w = z[q][k].x;
          if ((x + y) & 1) w = -w;
          out[(size_t)r * n + ix] = w * cinv[ix] * cy;
        }
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < PER; ++q) s[padi(threadIdx.x + q * NT)] = v[q];
    __syncthreads();
    stockham_seq<L, NT, 1, 1>(s, row_tw<L>(twl), threadIdx.x);
    for (int ix = threadIdx.x; ix < n; ix += NT) {
      const int x = o + ix;
      float w = s[padi(x)].x;
      if ((x + y) & 1) w = -w;
      out[(size_t)r * n + ix] = w * cinv[ix] * cy;
    }
  }
}

template <int L>
__global__ __launch_bounds__(RowThreads<L>::v) void k_rows_image(
    const float2 *__restrict__ rows, const float *__restrict__ cinv, int n, float scale,
    float *__restrict__ out, const float2 *__restrict__ twr, int c_lo, int c_hi) {
  rows_image_body<L>(rows, cinv, n, scale, out, twr, c_lo, c_hi, blockIdx.x);
}

// plain in-place complex row DFTs of an L x L buffer
template <int L, int DIR, class C>
__global__ __launch_bounds__(RowThreads<L>::v) void k_rows_plain(C *__restrict__ buf,
                                                                 const C *__restrict__ twr) {
  constexpr int NT = RowThreads<L>::v;
  __shared__ C s[L + L / 32];
  __shared__ C twl[RowTw<L>::SIZE];
  C *row = buf + (size_t)blockIdx.x * L;
  constexpr int PER = L / NT;
  C v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) v[q] = row[threadIdx.x + q * NT];
  stage_twiddles<L, NT, C>(twl, twr);
  if constexpr (first_pass_in_regs<L, NT>()) {
    constexpr int NS = LastPass<L>::NS, RL = LastPass<L>::R, PL = (NS + NT - 1) / NT;
    first_pass_regs<L, DIR>(s, v, threadIdx.x);
    __syncthreads();
    C z[PL][RL];
    stockham_out<L, NT, 8, DIR>(s, row_tw<L>(twl), threadIdx.x, z);
#pragma unroll
    for (int q = 0; q < PL; ++q) {
      const int j = threadIdx.x + q * NT;
#pragma unroll
      for (int k = 0; k < RL; ++k)
        if (j < NS) row[j + k * NS] = z[q][k];
    }
  } else {
#pragma unroll
    for (int q = 0; q < PER; ++q) s[padi(threadIdx.x + q * NT)] = v[q];
    __syncthreads();
    stockham_seq<L, NT, 1, DIR, C>(s, row_tw<L>(twl), threadIdx.x);
    for (int x = threadIdx.x; x < L; x += NT) row[x] = s[padi(x)];
  }
}

// ---------------------------------------------------------------- column kernels
// Width of the column blocks for a transform of length L = P * Q: every
// pass keeps P or Q rows of CW columns in LDS, 256 threads, at least one
// element each.  Narrower blocks give more workgroups for the same data.
template <int P, int Q, class C>
struct ColWidth {
  static constexpr int lo = 256 / (P < Q ? P : Q);  // one element per thread
  // FP64 elements are twice as wide: the same bytes per row segment, except
  // for 64-point columns, whose two radix-8 passes stay in registers when
  // each of the 256 threads holds eight elements (32 columns)
  static constexpr int want =
      sizeof(C) > 8 ? ((P == 64 || Q == 64) && P <= 64 && Q <= 64 ? kColWant : kColWant / 2)
                    : kColWant;
  static constexpr int v = want > lo ? want : lo;
};
// Column DFT of length L = P * Q over an L x L array (row stride L):
//   pass 1 (block (cb, y2)): A[k1] = sum_y1 x[Q y1 + y2] w_P^(y1 k1), times
//          w_L^(y2 k1), stored at row Q k1 + y2 of dst;
//   pass 2 (block (cb, k1)): X[k1 + P k2] = sum_y2 A[Q k1 + y2] w_Q^(y2 k2).
// Pass 1 reads source row y from src row (y - src_row0) and treats rows
// outside [y_lo, y_hi) as zero.  Pass 2 keeps output rows k in [k_lo, k_hi),
// stored at dst row (k - dst_row0), optionally times (-1)^(k + x).

template <int P, int Q, int DIR, class C>
__device__ __forceinline__ void cols_p1_body(const C *__restrict__ src, int src_row0, int y_lo,
                                             int y_hi, C *__restrict__ dst,
                                             const C *__restrict__ tw, int x0, int y2) {
  constexpr int L = P * Q, CW = ColWidth<P, Q, C>::v;
  __shared__ C s[P * CW];
  const int t = threadIdx.x;
  // every load of the thread goes out before the first is used
  constexpr int PER = P * CW / 256;
  C v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int i = t + q * 256, y1 = i / CW, c = i % CW;
    const int y = Q * y1 + y2;
    v[q] = (y >= y_lo && y < y_hi) ? src[(size_t)(y - src_row0) * L + x0 + c] : mkc<C>(0, 0);
  }
  // the twiddles of the store, loaded while the transform runs
  C w[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int k1 = (t + q * 256) / CW;
    w[q] = tw_get<DIR>(tw, ((y2 * k1) & (L - 1)) * (kTwMax / L));
  }
  if constexpr (P == 64 && CW == 32) {
    // thread t holds rows t / 32 + 8 q of column t % 32: the transform runs
    // on them, and output row k1 = t / 32 + 8 q is v[q]
    col64_regs<DIR>(s, tw, t, v);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int i = t + q * 256, k1 = i / CW, c = i % CW;
      dst[(size_t)(Q * k1 + y2) * L + x0 + c] = cmul(v[q], w[q]);
    }
  } else {
#pragma unroll
    for (int q = 0; q < PER; ++q) s[t + q * 256] = v[q];
    __syncthreads();
    stockham_cols<P, 1, DIR, C, CW>(s, tw, t);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int i = t + q * 256, k1 = i / CW, c = i % CW;
      dst[(size_t)(Q * k1 + y2) * L + x0 + c] = cmul(s[i], w[q]);
    }
  }
}

template <int P, int Q, int DIR, class C>
__global__ __launch_bounds__(256) void k_cols_p1(const C *__restrict__ src, int src_row0,
                                                 int y_lo, int y_hi, C *__restrict__ dst,
                                                 const C *__restrict__ tw, int cb0) {
  cols_p1_body<P, Q, DIR, C>(src, src_row0, y_lo, y_hi, dst, tw,
                             (blockIdx.x + cb0) * ColWidth<P, Q, C>::v, blockIdx.y);
}

template <int P, int Q, int DIR, class C>
__device__ __forceinline__ void cols_p2_body(const C *__restrict__ src, C *__restrict__ dst,
                                             int dst_row0, int k_lo, int k_hi, int modulate,
                                             const C *__restrict__ tw, int x0, int k1) {
  constexpr int L = P * Q, CW = ColWidth<P, Q, C>::v;
  __shared__ C s[Q * CW];
  const int t = threadIdx.x;
  constexpr int PER = Q * CW / 256;
  C v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int i = t + q * 256, y2 = i / CW, c = i % CW;
    v[q] = src[(size_t)(Q * k1 + y2) * L + x0 + c];
  }
  if constexpr (Q == 64 && CW == 32) {
    // output row k2 = t / 32 + 8 q of column t % 32 is v[q] after the transform
    col64_regs<DIR>(s, tw, t, v);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int i = t + q * 256, k2 = i / CW, c = i % CW;
      const int k = k1 + P * k2;
      if (k >= k_lo && k < k_hi) {
        C z = v[q];
        if (modulate && ((k + x0 + c) & 1)) z = mkc<C>(-z.x, -z.y);
        dst[(size_t)(k - dst_row0) * L + x0 + c] = z;
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < PER; ++q) s[t + q * 256] = v[q];
    __syncthreads();
    stockham_cols<Q, 1, DIR, C, CW>(s, tw, t);
    for (int i = t; i < Q * CW; i += 256) {
      const int k2 = i / CW, c = i % CW;
      const int k = k1 + P * k2;
      if (k >= k_lo && k < k_hi) {
        C z = s[i];
        if (modulate && ((k + x0 + c) & 1)) z = mkc<C>(-z.x, -z.y);
        dst[(size_t)(k - dst_row0) * L + x0 + c] = z;
      }
    }
  }
}

template <int P, int Q, int DIR, class C>
__global__ __launch_bounds__(256) void k_cols_p2(const C *__restrict__ src,
                                                 C *__restrict__ dst, int dst_row0, int k_lo,
                                                 int k_hi, int modulate,
                                                 const C *__restrict__ tw, int cb0) {
  cols_p2_body<P, Q, DIR, C>(src, dst, dst_row0, k_lo, k_hi, modulate, tw,
                             (blockIdx.x + cb0) * ColWidth<P, Q, C>::v, blockIdx.y);
}

// ---------------------------------------------------------------- batched transforms
// The model / residual transforms of many members (same L and N) per launch:
// the member is the last grid dimension; blocks past a member's own row or
// column-block count return at once.

template <int L>
__global__ __launch_bounds__(RowThreads<L>::v) void k_rows_model_batch(
    const FftMember *__restrict__ m, int n, const float2 *__restrict__ twr) {
  const FftMember &a = m[blockIdx.y];
  rows_model_body<L>(a.model, nullptr, a.cinv, n, a.rows, twr, a.x0, a.x1, blockIdx.x);
}

template <int L>
__global__ __launch_bounds__(RowThreads<L>::v) void k_rows_image_batch(
    const FftMember *__restrict__ m, int n, const float2 *__restrict__ twr) {
  const FftMember &a = m[blockIdx.y];
  rows_image_body<L>(a.rows, a.cinv, n, a.scale, a.image, twr, a.x0, a.x1, blockIdx.x);
}

// SIDE 0: model side (rows -> tmp), 1: residual side (grid -> tmp)
template <int P, int Q, int DIR, int SIDE>
__global__ __launch_bounds__(256) void k_cols_p1_batch(const FftMember *__restrict__ m, int n,
                                                       const float2 *__restrict__ tw) {
  constexpr int L = P * Q;
  const FftMember &a = m[blockIdx.z];
  constexpr int CW = ColWidth<P, Q, float2>::v;
  if ((int)blockIdx.x >= (a.x1 - a.x0) / CW) return;
  const int x0 = a.x0 + blockIdx.x * CW;
  const int o = (L - n) / 2;
  if constexpr (SIDE == 0)
    cols_p1_body<P, Q, DIR, float2>(a.rows, o, o, o + n, a.tmp, tw, x0, blockIdx.y);
  else
    cols_p1_body<P, Q, DIR, float2>(a.grid, 0, a.y0, a.y1, a.tmp, tw, x0, blockIdx.y);
}

// SIDE 0: model side (tmp -> grid rows of the box, modulated), 1: residual
// side (tmp -> rows of the crop)
template <int P, int Q, int DIR, int SIDE>
__global__ __launch_bounds__(256) void k_cols_p2_batch(const FftMember *__restrict__ m, int n,
                                                       const float2 *__restrict__ tw) {
  constexpr int L = P * Q;
  const FftMember &a = m[blockIdx.z];
  constexpr int CW = ColWidth<P, Q, float2>::v;
  if ((int)blockIdx.x >= (a.x1 - a.x0) / CW) return;
  const int x0 = a.x0 + blockIdx.x * CW;
  const int o = (L - n) / 2;
  if constexpr (SIDE == 0)
    cols_p2_body<P, Q, DIR, float2>(a.tmp, a.grid, 0, a.y0, a.y1, 1, tw, x0, blockIdx.y);
  else
    cols_p2_body<P, Q, DIR, float2>(a.tmp, a.rows, o, o, o + n, 0, tw, x0, blockIdx.y);
}

// ---------------------------------------------------------------- image-domain filters
// Products in the plain 2-D DFT domain of an image (Gamma filters of
// Section 4.1 on the N x N grid; linear convolution by a 2N x 2N PSF on the
// zero-padded 2N x 2N grid, Eq. 7): a real-input row pass, one column pass
// that transforms, multiplies and transforms back with whole columns in LDS,
// and a real-output row pass.

// rows r < 2 gridDim.x (two per workgroup): (a - b) (n_in real values, zero
// padded to L) -> plain forward row DFT -> out[r][0..c_hi): the column passes
// that follow read
// only the column blocks holding frequencies 0 .. L / 2 (the row is
// Hermitian), fewer when the spectral factor vanishes beyond a frequency
template <int L>
constexpr int half_spectrum_cols() {
  return ((L / 2) / 64 + 1) * 64 < L ? ((L / 2) / 64 + 1) * 64 : L;
}
template <int L, class C>
__device__ __forceinline__ void rows_real_fwd_body(const typename Real<C>::T *__restrict__ a,
                                                   const typename Real<C>::T *__restrict__ b,
                                                   int n_in, C *__restrict__ out,
                                                   const C *__restrict__ twr, int c_hi,
                                                   int pair) {
  typedef typename Real<C>::T RT;
  constexpr int NT = RowThreads<L>::v;
  __shared__ C s[L + L / 32];
  __shared__ C twl[RowTw<L>::SIZE];
  // rows 2 pair and 2 pair + 1 as the real and imaginary parts of one
  // complex sequence z = u + i v; their spectra are separated below by the
  // symmetry of real spectra: U[k] = (Z[k] + conj Z[L-k]) / 2,
  // V[k] = (Z[k] - conj Z[L-k]) / 2i
  const int ra = 2 * pair, rb = ra + 1;
  {
    constexpr int PER = L / NT;
    RT u[PER], v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int x = threadIdx.x + q * NT;
      u[q] = (x < n_in) ? a[(size_t)ra * n_in + x] : RT(0);
      v[q] = (x < n_in) ? a[(size_t)rb * n_in + x] : RT(0);
    }
    if (b) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int x = threadIdx.x + q * NT;
        if (x < n_in) {
          u[q] -= b[(size_t)ra * n_in + x];
          v[q] -= b[(size_t)rb * n_in + x];
        }
      }
    }
    stage_twiddles<L, NT, C>(twl, twr);
    if constexpr (first_pass_in_regs<L, NT>()) {
      C w[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) w[q] = mkc<C>(u[q], v[q]);
      first_pass_regs<L, -1>(s, w, threadIdx.x);
    } else {
#pragma unroll
      for (int q = 0; q < PER; ++q) s[padi(threadIdx.x + q * NT)] = mkc<C>(u[q], v[q]);
    }
  }
  __syncthreads();
  stockham_seq<L, NT, first_pass_in_regs<L, NT>() ? 8 : 1, -1, C>(s, row_tw<L>(twl),
                                                                  threadIdx.x);
  const RT h = RT(0.5);
  for (int x = threadIdx.x; x < c_hi; x += NT) {
    const C zx = s[padi(x)], zm = s[padi((L - x) & (L - 1))];
    out[(size_t)ra * L + x] = mkc<C>(h * (zx.x + zm.x), h * (zx.y - zm.y));
    out[(size_t)rb * L + x] = mkc<C>(h * (zx.y + zm.y), h * (zm.x - zx.x));
  }
}

template <int L, class C>
__global__ __launch_bounds__(RowThreads<L>::v) void k_rows_real_fwd(
    const typename Real<C>::T *__restrict__ a, const typename Real<C>::T *__restrict__ b,
    int n_in, C *__restrict__ out, const C *__restrict__ twr, int c_hi) {
  rows_real_fwd_body<L, C>(a, b, n_in, out, twr, c_hi, blockIdx.x);
}

// rows r < 2 gridDim.x (two per workgroup): inverse plain row DFT of
// in[r][0..L) (columns x and L - x at or above c_hi zero), then
// out[r][c] (+)= Re s[col0 + c], c < n_out
template <int L, class C>
__device__ __forceinline__ void rows_inv_real_body(const C *__restrict__ in, int col0, int n_out,
                                                   typename Real<C>::T *__restrict__ out,
                                                   int accumulate, const C *__restrict__ twr,
                                                   int c_hi, int pair,
                                                   const typename Real<C>::T *__restrict__ add =
                                                       nullptr,
                                                   typename Real<C>::T add_scale = 0) {
  typedef typename Real<C>::T RT;
  constexpr int NT = RowThreads<L>::v;
  __shared__ C s[L + L / 32];
  __shared__ C twl[RowTw<L>::SIZE];
  // rows 2 pair and 2 pair + 1 in one transform: each row is Hermitian (the
  // 2-D spectrum it came from belongs to a real image), columns above L / 2
  // being the conjugates of those below, so the inverse DFT of
  // Z = U + i V is u + i v with both u and v real.  The imaginary parts at
  // columns 0 and L / 2, which do not reach the real part of a row's own
  // inverse, are dropped so that they do not reach the other row's.
  const int ra = 2 * pair, rb = ra + 1;
  {
    constexpr int PER = L / NT;
    C u[PER], v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int x = threadIdx.x + q * NT;
      const int xs = x <= L / 2 ? x : L - x;  // columns from c_hi on are zero
      u[q] = xs < c_hi ? in[(size_t)ra * L + xs] : mkc<C>(0, 0);
      v[q] = xs < c_hi ? in[(size_t)rb * L + xs] : mkc<C>(0, 0);
    }
    stage_twiddles<L, NT, C>(twl, twr);
    C w[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int x = threadIdx.x + q * NT;
      if (x > L / 2) {
        u[q].y = -u[q].y;
        v[q].y = -v[q].y;
      } else if (x == 0 || x == L / 2) {
        u[q].y = 0;
        v[q].y = 0;
      }
      w[q] = mkc<C>(u[q].x - v[q].y, u[q].y + v[q].x);
    }
    if constexpr (first_pass_in_regs<L, NT>()) {
      first_pass_regs<L, 1>(s, w, threadIdx.x);
    } else {
#pragma unroll
      for (int q = 0; q < PER; ++q) s[padi(threadIdx.x + q * NT)] = w[q];
    }
  }
  __syncthreads();
  if constexpr (first_pass_in_regs<L, NT>()) {
    // last pass in registers: thread t holds columns j + k NS of both rows
    constexpr int NS = LastPass<L>::NS, RL = LastPass<L>::R, PL = (NS + NT - 1) / NT;
    C z[PL][RL];
    stockham_out<L, NT, 8, 1>(s, row_tw<L>(twl), threadIdx.x, z);
    RT pa[PL][RL], pb[PL][RL];
    if (accumulate) {
#pragma unroll
      for (int q = 0; q < PL; ++q)
#pragma unroll
        for (int k = 0; k < RL; ++k) {
          const int c = threadIdx.x + q * NT + k * NS - col0;
          pa[q][k] = pb[q][k] = RT(0);
          if (threadIdx.x + q * NT < NS && c >= 0 && c < n_out) {
            pa[q][k] = out[(size_t)ra * n_out + c];
            pb[q][k] = out[(size_t)rb * n_out + c];
          }
        }
    }
#pragma unroll
    for (int q = 0; q < PL; ++q)
#pragma unroll
      for (int k = 0; k < RL; ++k) {
        const int c = threadIdx.x + q * NT + k * NS - col0;
        if (threadIdx.x + q * NT < NS && c >= 0 && c < n_out) {
          const C zz = z[q][k];
          if (accumulate) {
            out[(size_t)ra * n_out + c] = pa[q][k] + zz.x;
            out[(size_t)rb * n_out + c] = pb[q][k] + zz.y;
          } else if (add) {
            out[(size_t)ra * n_out + c] = add_scale * add[(size_t)ra * n_out + c] + zz.x;
            out[(size_t)rb * n_out + c] = add_scale * add[(size_t)rb * n_out + c] + zz.y;
          } else {
            out[(size_t)ra * n_out + c] = zz.x;
            out[(size_t)rb * n_out + c] = zz.y;
          }
        }
      }
    return;
  }
  stockham_seq<L, NT, 1, 1, C>(s, row_tw<L>(twl), threadIdx.x);
  if (accumulate) {
    constexpr int PO = (L + NT - 1) / NT;  // n_out <= L
    RT pa[PO], pb[PO];
#pragma unroll
    for (int q = 0; q < PO; ++q) {
      const int c = threadIdx.x + q * NT;
      pa[q] = (c < n_out) ? out[(size_t)ra * n_out + c] : RT(0);
      pb[q] = (c < n_out) ? out[(size_t)rb * n_out + c] : RT(0);
    }
#pragma unroll
    for (int q = 0; q < PO; ++q) {
      const int c = threadIdx.x + q * NT;
      if (c < n_out) {
        const C z = s[padi(col0 + c)];
        out[(size_t)ra * n_out + c] = pa[q] + z.x;
        out[(size_t)rb * n_out + c] = pb[q] + z.y;
      }
    }
  } else if (add) {
    // out = add_scale add + the row (add: n_out columns per row, like out)
    for (int c = threadIdx.x; c < n_out; c += NT) {
      const C z = s[padi(col0 + c)];
      out[(size_t)ra * n_out + c] = add_scale * add[(size_t)ra * n_out + c] + z.x;
      out[(size_t)rb * n_out + c] = add_scale * add[(size_t)rb * n_out + c] + z.y;
    }
  } else {
    for (int c = threadIdx.x; c < n_out; c += NT) {
      const C z = s[padi(col0 + c)];
      out[(size_t)ra * n_out + c] = z.x;
      out[(size_t)rb * n_out + c] = z.y;
    }
  }
}

template <int L, class C>
__global__ __launch_bounds__(RowThreads<L>::v) void k_rows_inv_real(
    const C *__restrict__ in, int col0, int n_out, typename Real<C>::T *__restrict__ out,
    int accumulate, const C *__restrict__ twr, int c_hi,
    const typename Real<C>::T *__restrict__ add = nullptr, typename Real<C>::T add_scale = 0) {
  rows_inv_real_body<L, C>(in, col0, n_out, out, accumulate, twr, c_hi, blockIdx.x, add,
                           add_scale);
}

// Spectral product between a forward and an inverse column DFT, four-step
// form (L = P * Q, blocks of CW columns):
//   forward pass 1 (k_cols_p1) leaves A[Q k1 + y2];
//   mid (block (cb, k1)): X[k1 + P k2] = sum_y2 A[Q k1 + y2] w_Q^(y2 k2)
//          (forward), times the spectral factor, then
//          B[y2] = sum_k2 X[k1 + P k2] w_Q^(-y2 k2) w_L^(-y2 k1), stored back
//          at row Q k1 + y2 (in place);
//   fin (block (cb, y2)): x[y2 + Q y1] = sum_k1 B[Q k1 + y2] w_P^(-y1 k1),
//          rows y in [k_lo, k_hi) stored at dst row y - k_lo.
enum { FILT_GAMMA = 0, FILT_SPEC = 1 };

// Gamma_L(kappa) = clip((ell + delta - kappa) / (2 delta), 0, 1) at the
// plain-DFT frequency (kx, ky) of an nd-point grid, kappa = |k| / scale
__device__ __forceinline__ double gamma_low_at(int kx, int ky, int nd, double ell, double delta,
                                               double scale) {
  const int fx = (kx < nd / 2) ? kx : kx - nd;
  const int fy = (ky < nd / 2) ? ky : ky - nd;
  const double kappa = sqrt((double)fx * fx + (double)fy * fy) / scale;
  const double g = (ell + delta - kappa) / (2.0 * delta);
  return fmin(fmax(g, 0.0), 1.0);
}

template <int P, int Q, int MODE, class C>
__device__ __forceinline__ void cols_mid_body(C *__restrict__ buf, const C *__restrict__ spec,
                                              double ell, double delta, double gscale,
                                              int own_low, typename Real<C>::T coef,
                                              const C *__restrict__ tw, int x0, int k1) {
  typedef typename Real<C>::T RT;
  constexpr int L = P * Q, CW = ColWidth<P, Q, C>::v;
  __shared__ C s[Q * CW];
  const int t = threadIdx.x;
  constexpr int PER = Q * CW / 256;
  // the column block and (for a spectral factor) the factors it is
  // multiplied by: all loads issued before the first is used
  C sp[MODE == FILT_SPEC ? PER : 1];
  {
    C v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int i = t + q * 256, y2 = i / CW, c = i % CW;
      v[q] = buf[(size_t)(Q * k1 + y2) * L + x0 + c];
    }
    if constexpr (MODE == FILT_SPEC) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int i = t + q * 256, k2 = i / CW, c = i % CW;
        sp[q] = spec[(size_t)(k1 + P * k2) * L + x0 + c];
      }
    }
    // the factor applied at frequency row k = k1 + P k2 of column c
    auto filt = [&](C z, int q) {
      const int i = t + q * 256, k2 = i / CW, c = i % CW;
      const int k = k1 + P * k2;
      if constexpr (MODE == FILT_GAMMA) {
        RT g = (RT)gamma_low_at(x0 + c, k, L, ell, delta, gscale);
        if (!(own_low & 1)) g = (RT)1 - g;
        if (own_low & 2) g = g * g;
        if (own_low & 4) g = g * ((RT)2 - g);  // 1 - (1 - Gamma_L)^2
        return cscale(z, g * coef);
      } else {
        return cscale(cmul(z, sp[q]), coef);
      }
    };
    if constexpr (Q == 64 && CW == 32) {
      // thread t holds rows t / 32 + 8 q of column t % 32 throughout: the
      // inverse transform, the factor and the forward transform run on them
      col64_regs<-1>(s, tw, t, v);
#pragma unroll
      for (int q = 0; q < PER; ++q) v[q] = filt(v[q], q);
      C w[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int y2 = (t + q * 256) / CW;
        w[q] = tw_get<1>(tw, ((y2 * k1) & (L - 1)) * (kTwMax / L));
      }
      __syncthreads();  // the first transform's reads of s are done
      col64_regs<1>(s, tw, t, v);
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int i = t + q * 256, y2 = i / CW, c = i % CW;
        buf[(size_t)(Q * k1 + y2) * L + x0 + c] = cmul(v[q], w[q]);
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) s[t + q * 256] = v[q];
    __syncthreads();
    stockham_cols<Q, 1, -1, C, CW>(s, tw, t);
#pragma unroll
    for (int q = 0; q < PER; ++q) s[t + q * 256] = filt(s[t + q * 256], q);
  }
  C w[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int y2 = (t + q * 256) / CW;
    w[q] = tw_get<1>(tw, ((y2 * k1) & (L - 1)) * (kTwMax / L));
  }
  __syncthreads();
  stockham_cols<Q, 1, 1, C, CW>(s, tw, t);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int i = t + q * 256, y2 = i / CW, c = i % CW;
    buf[(size_t)(Q * k1 + y2) * L + x0 + c] = cmul(s[i], w[q]);
  }
}

template <int P, int Q, int MODE, class C>
__global__ __launch_bounds__(256) void k_cols_mid(C *__restrict__ buf, const C *__restrict__ spec,
                                                  double ell, double delta, double gscale,
                                                  int own_low, typename Real<C>::T coef,
                                                  const C *__restrict__ tw) {
  cols_mid_body<P, Q, MODE, C>(buf, spec, ell, delta, gscale, own_low, coef, tw,
                               blockIdx.x * ColWidth<P, Q, C>::v, blockIdx.y);
}

template <int P, int Q, class C>
__device__ __forceinline__ void cols_fin_body(const C *__restrict__ src, C *__restrict__ dst,
                                              int k_lo, int k_hi, const C *__restrict__ tw,
                                              int x0, int y2) {
  constexpr int L = P * Q, CW = ColWidth<P, Q, C>::v;
  __shared__ C s[P * CW];
  const int t = threadIdx.x;
  {
    constexpr int PER = P * CW / 256;
    C v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int i = t + q * 256, k1 = i / CW, c = i % CW;
      v[q] = src[(size_t)(Q * k1 + y2) * L + x0 + c];
    }
    if constexpr (P == 64 && CW == 32) {
      // output row y1 = t / 32 + 8 q of column t % 32 is v[q] after the transform
      col64_regs<1>(s, tw, t, v);
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int i = t + q * 256, y1 = i / CW, c = i % CW;
        const int y = y2 + Q * y1;
        if (y >= k_lo && y < k_hi) dst[(size_t)(y - k_lo) * L + x0 + c] = v[q];
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) s[t + q * 256] = v[q];
  }
  __syncthreads();
  stockham_cols<P, 1, 1, C, CW>(s, tw, t);
  for (int i = t; i < P * CW; i += 256) {
    const int y1 = i / CW, c = i % CW;
    const int y = y2 + Q * y1;
    if (y >= k_lo && y < k_hi) dst[(size_t)(y - k_lo) * L + x0 + c] = s[i];
  }
}

template <int P, int Q, class C>
__global__ __launch_bounds__(256) void k_cols_fin(const C *__restrict__ src, C *__restrict__ dst,
                                                  int k_lo, int k_hi, const C *__restrict__ tw) {
  cols_fin_body<P, Q, C>(src, dst, k_lo, k_hi, tw, blockIdx.x * ColWidth<P, Q, C>::v,
                         blockIdx.y);
}

template <int L>
struct Split;
template <> struct Split<64> { static constexpr int P = 8, Q = 8; };
template <> struct Split<128> { static constexpr int P = 8, Q = 16; };
template <> struct Split<256> { static constexpr int P = 16, Q = 16; };
template <> struct Split<512> { static constexpr int P = 16, Q = 32; };
template <> struct Split<1024> { static constexpr int P = 32, Q = 32; };
template <> struct Split<2048> { static constexpr int P = 32, Q = 64; };
template <> struct Split<4096> { static constexpr int P = 64, Q = 64; };
template <> struct Split<8192> { static constexpr int P = 64, Q = 128; };

template <class C> const C *twiddles(const imgr_s *h);
template <> const float2 *twiddles<float2>(const imgr_s *h) { return h->tw; }
template <> const double2 *twiddles<double2>(const imgr_s *h) { return h->tw64; }
template <class C> const C *row_twiddles(const imgr_s *h);
template <> const float2 *row_twiddles<float2>(const imgr_s *h) { return h->twrow; }
template <> const double2 *row_twiddles<double2>(const imgr_s *h) { return h->twrow64; }

// column blocks [cb0, cb1) of 64 columns (F = 64 / CW launch blocks each)
template <int L, int DIR, class C>
void cols(const C *src, int src_row0, int y_lo, int y_hi, C *tmp, C *dst, int dst_row0, int k_lo,
          int k_hi, int modulate, const C *tw, hipStream_t s, int cb0 = 0, int cb1 = L / 64) {
  constexpr int P = Split<L>::P, Q = Split<L>::Q, F = 64 / ColWidth<P, Q, C>::v;
  if (cb1 <= cb0) return;
  hipLaunchKernelGGL((k_cols_p1<P, Q, DIR, C>), dim3((cb1 - cb0) * F, Q), dim3(256), 0, s, src,
                     src_row0, y_lo, y_hi, tmp, tw, cb0 * F);
  hipLaunchKernelGGL((k_cols_p2<P, Q, DIR, C>), dim3((cb1 - cb0) * F, P), dim3(256), 0, s, tmp,
                     dst, dst_row0, k_lo, k_hi, modulate, tw, cb0 * F);
}

// the transforms touch only the box of grid cells the partition's chunk
// windows cover: the de/gridding reads and the flush writes nothing else,
// so the rest of the grid is never formed (model side) and is zero (residual
// side)
template <int L>
void model_to_grid_t(imgr_s *h, const float *model, const float *model_add, const float *cinv,
                     int n, float2 *rows, float2 *tmp, float2 *out, const Box &b, hipStream_t s) {
  const int o = (L - n) / 2;
  // one workgroup per pair of rows (n is even)
  hipLaunchKernelGGL((k_rows_model<L>), dim3(n / 2), dim3(RowThreads<L>::v), 0, s, model,
                     model_add, cinv, n, rows, h->twrow, b.x0, b.x1);
  cols<L, -1, float2>(rows, o, o, o + n, tmp, out, 0, b.y0, b.y1, 1, h->tw, s, b.x0 / 64,
                      b.x1 / 64);
}

template <int L>
void grid_to_image_t(imgr_s *h, const float2 *in, const float *cinv, int n, float scale,
                     float2 *rows, float2 *tmp, float *out, const Box &b, hipStream_t s) {
  const int o = (L - n) / 2;
  cols<L, 1, float2>(in, 0, b.y0, b.y1, tmp, rows, o, o, o + n, 0, h->tw, s, b.x0 / 64,
                     b.x1 / 64);
  hipLaunchKernelGGL((k_rows_image<L>), dim3(n), dim3(RowThreads<L>::v), 0, s, rows, cinv, n,
                     scale, out, h->twrow, b.x0, b.x1);
}

template <int L, class C>
void plain_t(imgr_s *h, C *buf, C *tmp, int dir, hipStream_t s) {
  const C *tw = twiddles<C>(h);
  const C *twr = row_twiddles<C>(h);
  if (dir < 0) {
    hipLaunchKernelGGL((k_rows_plain<L, -1, C>), dim3(L), dim3(RowThreads<L>::v), 0, s, buf, twr);
    cols<L, -1, C>(buf, 0, 0, L, tmp, buf, 0, 0, L, 0, tw, s);
  } else {
    hipLaunchKernelGGL((k_rows_plain<L, 1, C>), dim3(L), dim3(RowThreads<L>::v), 0, s, buf, twr);
    cols<L, 1, C>(buf, 0, 0, L, tmp, buf, 0, 0, L, 0, tw, s);
  }
}

// n_in rows of n_in pixels in (zero padded to L x L), rows [k_lo, k_hi) x
// cols [col0, col0 + n_out) out; work: n_in x L, tmp: L x L.
// The filter is two parts: the front (real-input row pass and the three
// column passes) leaves rows [k_lo, k_hi) of the filtered spectrum's inverse
// column transform in work; the back (real-output row pass) turns them into
// the output.  Either part may run on its own stream.
template <int L>
int filter_cols(const imgr_s *h, int mode, int own_low, double gscale) {
  // the input is real, so its 2-D spectrum is Hermitian and the real
  // spectral factors keep it so: the column passes only need the column
  // blocks that hold frequencies 0 .. L / 2; the final row pass rebuilds
  // the rest by conjugate symmetry
  int CB = half_spectrum_cols<L>() / 64;
  // Gamma_L (own_low odd) vanishes for |kx| >= (ell + delta) scale: the column
  // blocks from there on are zero after the product, so they are never formed
  if (mode == FILT_GAMMA && (own_low & 1))
    CB = std::min(CB, std::max(1, (int)std::ceil((h->ell + h->delta) * gscale / 64.0)));
  return CB * 64;
}

template <int L, class C>
void filter_front_t(imgr_s *h, const typename Real<C>::T *a, const typename Real<C>::T *b,
                    int n_in, int mode, const C *spec, int own_low, double gscale,
                    typename Real<C>::T coef, int k_lo, int k_hi, C *work, C *tmp,
                    hipStream_t s) {
  constexpr int P = Split<L>::P, Q = Split<L>::Q;
  const int c_hi = filter_cols<L>(h, mode, own_low, gscale);
  const int CB = c_hi / ColWidth<P, Q, C>::v;  // launch blocks
  const C *tw = twiddles<C>(h);
  const C *twr = row_twiddles<C>(h);
  hipLaunchKernelGGL((k_rows_real_fwd<L, C>), dim3(n_in / 2), dim3(RowThreads<L>::v), 0, s, a, b,
                     n_in, work, twr, c_hi);
  hipLaunchKernelGGL((k_cols_p1<P, Q, -1, C>), dim3(CB, Q), dim3(256), 0, s, work, 0, 0, n_in,
                     tmp, tw, 0);
  if (mode == FILT_GAMMA)
    hipLaunchKernelGGL((k_cols_mid<P, Q, FILT_GAMMA, C>), dim3(CB, P), dim3(256), 0, s, tmp,
                       spec, h->ell, h->delta, gscale, own_low, coef, tw);
  else
    hipLaunchKernelGGL((k_cols_mid<P, Q, FILT_SPEC, C>), dim3(CB, P), dim3(256), 0, s, tmp,
                       spec, h->ell, h->delta, gscale, own_low, coef, tw);
  hipLaunchKernelGGL((k_cols_fin<P, Q, C>), dim3(CB, Q), dim3(256), 0, s, tmp, work, k_lo,
                     k_hi, tw);
}

template <int L, class C>
void filter_back_t(imgr_s *h, int mode, int own_low, double gscale, int k_lo, int k_hi, int col0,
                   int n_out, typename Real<C>::T *out, int accumulate, const C *work,
                   hipStream_t s) {
  const int c_hi = filter_cols<L>(h, mode, own_low, gscale);
  hipLaunchKernelGGL((k_rows_inv_real<L, C>), dim3((k_hi - k_lo) / 2), dim3(RowThreads<L>::v),
                     0, s, work, col0, n_out, out, accumulate, row_twiddles<C>(h), c_hi);
}

// Two Gamma filters of the same length L = N in one launch per pass: the
// member is the last grid dimension; column blocks past a member's own
// column count return at once.  Each member computes exactly what filter_t
// computes for it alone.
template <class C>
struct GammaMember {
  const typename Real<C>::T *a;
  typename Real<C>::T *out;
  C *work, *tmp;
  typename Real<C>::T coef;
  int own_low, accumulate, c_hi;
  // out = add_scale add + the filtered image (add may be null)
  const typename Real<C>::T *add;
  typename Real<C>::T add_scale;
};
template <class C>
struct GammaPair {
  GammaMember<C> m[2];
};
template <class C>
__device__ __forceinline__ GammaMember<C> pick(const GammaPair<C> &g, unsigned k) {
  GammaMember<C> m = g.m[0];  // a select, not an indexed copy of the arguments
  if (k) m = g.m[1];
  return m;
}

template <int L, class C>
__global__ __launch_bounds__(RowThreads<L>::v) void k_gamma_pair_rows_fwd(GammaPair<C> g,
                                                                          const C *twr) {
  const GammaMember<C> m = pick(g, blockIdx.y);
  rows_real_fwd_body<L, C>(m.a, nullptr, L, m.work, twr, m.c_hi, blockIdx.x);
}
template <int P, int Q, class C>
__global__ __launch_bounds__(256) void k_gamma_pair_p1(GammaPair<C> g, const C *tw) {
  constexpr int CW = ColWidth<P, Q, C>::v;
  const GammaMember<C> m = pick(g, blockIdx.z);
  if ((int)blockIdx.x * CW >= m.c_hi) return;
  cols_p1_body<P, Q, -1, C>(m.work, 0, 0, P * Q, m.tmp, tw, blockIdx.x * CW, blockIdx.y);
}
template <int P, int Q, class C>
__global__ __launch_bounds__(256) void k_gamma_pair_mid(GammaPair<C> g, double ell, double delta,
                                                        const C *tw) {
  constexpr int CW = ColWidth<P, Q, C>::v;
  const GammaMember<C> m = pick(g, blockIdx.z);
  if ((int)blockIdx.x * CW >= m.c_hi) return;
  cols_mid_body<P, Q, FILT_GAMMA, C>(m.tmp, nullptr, ell, delta, 1.0, m.own_low, m.coef, tw,
                                     blockIdx.x * CW, blockIdx.y);
}
template <int P, int Q, class C>
__global__ __launch_bounds__(256) void k_gamma_pair_fin(GammaPair<C> g, const C *tw) {
  constexpr int CW = ColWidth<P, Q, C>::v;
  const GammaMember<C> m = pick(g, blockIdx.z);
  if ((int)blockIdx.x * CW >= m.c_hi) return;
  cols_fin_body<P, Q, C>(m.tmp, m.work, 0, P * Q, tw, blockIdx.x * CW, blockIdx.y);
}
template <int L, class C>
__global__ __launch_bounds__(RowThreads<L>::v) void k_gamma_pair_rows_inv(GammaPair<C> g,
                                                                          const C *twr) {
  const GammaMember<C> m = pick(g, blockIdx.y);
  rows_inv_real_body<L, C>(m.work, 0, L, m.out, m.accumulate, twr, m.c_hi, blockIdx.x, m.add,
                           m.add_scale);
}

template <int L, class C>
void gamma_pair_t(imgr_s *h, GammaPair<C> g, hipStream_t s) {
  typedef typename Real<C>::T RT;
  constexpr int P = Split<L>::P, Q = Split<L>::Q, CW = ColWidth<P, Q, C>::v;
  for (int k = 0; k < 2; ++k) {
    GammaMember<C> &m = g.m[k];
    // a high-pass member as a minus its complement: Gamma_H a = a - Gamma_L a
    // and Gamma_H^2 a = a - Gamma_L (2 - Gamma_L) a, whose factors vanish
    // beyond ell + delta like Gamma_L, so the member needs only the low
    // column blocks (the subtraction cancels at low frequencies, which the
    // FP64 transforms of these filters absorb)
    if (!(m.own_low & 1) && !m.accumulate && !m.add) {
      m.add = m.a;
      m.add_scale = m.coef * (RT)L * (RT)L;
      m.coef = -m.coef;
      m.own_low = 1 | ((m.own_low & 2) ? 4 : 0);
    }
    m.c_hi = filter_cols<L>(h, FILT_GAMMA, m.own_low, 1.0);
  }
  const int cb = std::max(g.m[0].c_hi, g.m[1].c_hi) / CW;
  const C *tw = twiddles<C>(h);
  const C *twr = row_twiddles<C>(h);
  hipLaunchKernelGGL((k_gamma_pair_rows_fwd<L, C>), dim3(L / 2, 2), dim3(RowThreads<L>::v), 0, s,
                     g, twr);
  hipLaunchKernelGGL((k_gamma_pair_p1<P, Q, C>), dim3(cb, Q, 2), dim3(256), 0, s, g, tw);
  hipLaunchKernelGGL((k_gamma_pair_mid<P, Q, C>), dim3(cb, P, 2), dim3(256), 0, s, g, h->ell,
                     h->delta, tw);
  hipLaunchKernelGGL((k_gamma_pair_fin<P, Q, C>), dim3(cb, Q, 2), dim3(256), 0, s, g, tw);
  hipLaunchKernelGGL((k_gamma_pair_rows_inv<L, C>), dim3(L / 2, 2), dim3(RowThreads<L>::v), 0, s,
                     g, twr);
}

template <int L, class C>
void filter_t(imgr_s *h, const typename Real<C>::T *a, const typename Real<C>::T *b, int n_in,
              int mode, const C *spec, int own_low, double gscale, typename Real<C>::T coef,
              int k_lo, int k_hi, int col0, int n_out, typename Real<C>::T *out, int accumulate,
              C *work, C *tmp, hipStream_t s) {
  filter_front_t<L, C>(h, a, b, n_in, mode, spec, own_low, gscale, coef, k_lo, k_hi, work, tmp,
                       s);
  filter_back_t<L, C>(h, mode, own_low, gscale, k_lo, k_hi, col0, n_out, out, accumulate, work,
                      s);
}

}  // namespace

#define IMGR_FFT_SIZES(X) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(8192)

static void check_box(const Box &b, int ng) {
  IMGR_CHECK(b.x0 >= 0 && b.x0 <= b.x1 && b.x1 <= ng && b.x0 % 64 == 0 && b.x1 % 64 == 0 &&
                 b.y0 >= 0 && b.y0 <= b.y1 && b.y1 <= ng,
             "transform box outside the grid");
}

namespace {
template <int L>
void model_to_grid_batch_t(const imgr_s *h, int n, const FftMember *m, int count, int max_cb,
                           hipStream_t s) {
  constexpr int P = Split<L>::P, Q = Split<L>::Q, F = 64 / ColWidth<P, Q, float2>::v;
  hipLaunchKernelGGL((k_rows_model_batch<L>), dim3(n / 2, count), dim3(RowThreads<L>::v), 0, s,
                     m, n, h->twrow);
  if (max_cb == 0) return;
  hipLaunchKernelGGL((k_cols_p1_batch<P, Q, -1, 0>), dim3(max_cb * F, Q, count), dim3(256), 0, s,
                     m, n, h->tw);
  hipLaunchKernelGGL((k_cols_p2_batch<P, Q, -1, 0>), dim3(max_cb * F, P, count), dim3(256), 0, s,
                     m, n, h->tw);
}

template <int L>
void grid_to_image_batch_t(const imgr_s *h, int n, const FftMember *m, int count, int max_cb,
                           hipStream_t s) {
  constexpr int P = Split<L>::P, Q = Split<L>::Q, F = 64 / ColWidth<P, Q, float2>::v;
  if (max_cb > 0) {
    hipLaunchKernelGGL((k_cols_p1_batch<P, Q, 1, 1>), dim3(max_cb * F, Q, count), dim3(256), 0, s,
                       m, n, h->tw);
    hipLaunchKernelGGL((k_cols_p2_batch<P, Q, 1, 1>), dim3(max_cb * F, P, count), dim3(256), 0, s,
                       m, n, h->tw);
  }
  hipLaunchKernelGGL((k_rows_image_batch<L>), dim3(n, count), dim3(RowThreads<L>::v), 0, s, m, n,
                     h->twrow);
}
}  // namespace

void fft_model_to_grid_batch(const imgr_s *h, int ng, int n, const FftMember *members, int count,
                             int max_cb, hipStream_t s) {
  if (count == 0) return;
  IMGR_CHECK(count <= 65535 && max_cb >= 0 && max_cb <= ng / 64, "batched transform shape");
  switch (ng) {
#define X(L) \
  case L: model_to_grid_batch_t<L>(h, n, members, count, max_cb, s); break;
    IMGR_FFT_SIZES(X)
#undef X
    default: throw Error{IMGR_EINVAL, "unsupported FFT size"};
  }
  IMGR_HIP(hipGetLastError());
}

void fft_grid_to_image_batch(const imgr_s *h, int ng, int n, const FftMember *members, int count,
                             int max_cb, hipStream_t s) {
  if (count == 0) return;
  IMGR_CHECK(count <= 65535 && max_cb >= 0 && max_cb <= ng / 64, "batched transform shape");
  switch (ng) {
#define X(L) \
  case L: grid_to_image_batch_t<L>(h, n, members, count, max_cb, s); break;
    IMGR_FFT_SIZES(X)
#undef X
    default: throw Error{IMGR_EINVAL, "unsupported FFT size"};
  }
  IMGR_HIP(hipGetLastError());
}

void fft_model_to_grid(imgr_s *h, const float *model, const float *model_add, const float *cinv,
                       int n, int ng, float2 *rows, float2 *tmp, float2 *out, const Box &box,
                       hipStream_t s) {
  check_box(box, ng);
  switch (ng) {
#define X(L) \
  case L: model_to_grid_t<L>(h, model, model_add, cinv, n, rows, tmp, out, box, s); break;
    IMGR_FFT_SIZES(X)
#undef X
    default: throw Error{IMGR_EINVAL, "unsupported FFT size"};
  }
  IMGR_HIP(hipGetLastError());
}

void fft_grid_to_image(imgr_s *h, const float2 *in, const float *cinv, int n, int ng, float scale,
                       float2 *rows, float2 *tmp, float *out, const Box &box, hipStream_t s) {
  check_box(box, ng);
  switch (ng) {
#define X(L) \
  case L: grid_to_image_t<L>(h, in, cinv, n, scale, rows, tmp, out, box, s); break;
    IMGR_FFT_SIZES(X)
#undef X
    default: throw Error{IMGR_EINVAL, "unsupported FFT size"};
  }
  IMGR_HIP(hipGetLastError());
}

void image_gamma(imgr_s *h, const float *a, const float *b, int own_low, float coef, float *out,
                 int accumulate, float2 *work, float2 *tmp, hipStream_t s) {
  const int n = h->N;
  switch (n) {
#define X(L)                                                                                   \
  case L:                                                                                      \
    filter_t<L, float2>(h, a, b, n, FILT_GAMMA, nullptr, own_low, 1.0, coef, 0, n, 0, n, out,  \
                        accumulate, work, tmp, s);                                             \
    break;
    IMGR_FFT_SIZES(X)
#undef X
    default: throw Error{IMGR_EINVAL, "unsupported FFT size"};
  }
  IMGR_HIP(hipGetLastError());
}

void image_psf_conv(imgr_s *h, const float *a, const float2 *psf_hat, float coef, float *out,
                    int accumulate, float2 *work, float2 *tmp, hipStream_t s) {
  const int n = h->N, nd = 2 * n;
  switch (nd) {
#define X(L)                                                                                   \
  case L:                                                                                      \
    filter_t<L, float2>(h, a, nullptr, n, FILT_SPEC, psf_hat, 1, 1.0, coef, n, nd, n, n, out,  \
                        accumulate, work, tmp, s);                                             \
    break;
    IMGR_FFT_SIZES(X)
#undef X
    default: throw Error{IMGR_EINVAL, "unsupported FFT size"};
  }
  IMGR_HIP(hipGetLastError());
}

// the two parts of image_psf_conv: the front leaves N rows of 2N complex
// values in work (tmp: (2N)^2 complex), the back (+)= them into out
void image_psf_conv_front(imgr_s *h, const float *a, const float2 *psf_hat, float coef,
                          float2 *work, float2 *tmp, hipStream_t s) {
  const int n = h->N, nd = 2 * n;
  switch (nd) {
#define X(L)                                                                                  \
  case L:                                                                                     \
    filter_front_t<L, float2>(h, a, nullptr, n, FILT_SPEC, psf_hat, 1, 1.0, coef, n, nd, work, \
                              tmp, s);                                                        \
    break;
    IMGR_FFT_SIZES(X)
#undef X
    default: throw Error{IMGR_EINVAL, "unsupported FFT size"};
  }
  IMGR_HIP(hipGetLastError());
}

void image_psf_conv_back(imgr_s *h, const float2 *work, float *out, int accumulate,
                         hipStream_t s) {
  const int n = h->N, nd = 2 * n;
  switch (nd) {
#define X(L)                                                                              \
  case L:                                                                                 \
    filter_back_t<L, float2>(h, FILT_SPEC, 1, 1.0, n, nd, n, n, out, accumulate, work, s); \
    break;
    IMGR_FFT_SIZES(X)
#undef X
    default: throw Error{IMGR_EINVAL, "unsupported FFT size"};
  }
  IMGR_HIP(hipGetLastError());
}

void image_gamma_scaled(imgr_s *h, const float *a, int own_low, float gamma, float *out,
                        float2 *work, float2 *tmp, hipStream_t s) {
  const int n = h->N;
  const float inv = (float)(1.0 / ((double)n * n));
  switch (n) {
#define X(L)                                                                                 \
  case L:                                                                                    \
    if (own_low & 1) {                                                                       \
      filter_t<L, float2>(h, a, nullptr, n, FILT_GAMMA, nullptr, own_low, 1.0, gamma * inv, \
                          0, n, 0, n, out, 0, work, tmp, s);                                 \
    } else {                                                                                 \
      filter_front_t<L, float2>(h, a, nullptr, n, FILT_GAMMA, nullptr, 1, 1.0, -gamma * inv, \
                                0, n, work, tmp, s);                                         \
      hipLaunchKernelGGL((k_rows_inv_real<L, float2>), dim3(n / 2), dim3(RowThreads<L>::v), 0, \
                         s, work, 0, n, out, 0, h->twrow,                                   \
                         filter_cols<L>(h, FILT_GAMMA, 1, 1.0), a, gamma);                  \
    }                                                                                        \
    break;
    IMGR_FFT_SIZES(X)
#undef X
    default: throw Error{IMGR_EINVAL, "unsupported FFT size"};
  }
  IMGR_HIP(hipGetLastError());
}

void fft2_plain(imgr_s *h, float2 *buf, float2 *tmp, int n, int dir, hipStream_t s) {
  switch (n) {
#define X(L) \
  case L: plain_t<L, float2>(h, buf, tmp, dir, s); break;
    IMGR_FFT_SIZES(X)
#undef X
    default: throw Error{IMGR_EINVAL, "unsupported FFT size"};
  }
  IMGR_HIP(hipGetLastError());
}

// sizes of the FP64 transforms (images up to 2048, their 2N grids)
#define IMGR_FFT64_SIZES(X) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

void image_gamma64(imgr_s *h, const double *a, const double *b, int own_low, double coef,
                   double *out, int accumulate, double2 *work, double2 *tmp, hipStream_t s) {
  const int n = h->N;
  switch (n) {
#define X(L)                                                                                   \
  case L:                                                                                      \
    filter_t<L, double2>(h, a, b, n, FILT_GAMMA, nullptr, own_low, 1.0, coef, 0, n, 0, n, out, \
                         accumulate, work, tmp, s);                                            \
    break;
    IMGR_FFT64_SIZES(X)
#undef X
    default: throw Error{IMGR_EINVAL, "unsupported FFT size"};
  }
  IMGR_HIP(hipGetLastError());
}

void image_psf_conv64(imgr_s *h, const double *a, const double2 *psf_hat, double coef, double *out,
                      int accumulate, double2 *work, double2 *tmp, hipStream_t s) {
  const int n = h->N, nd = 2 * n;
  switch (nd) {
#define X(L)                                                                                   \
  case L:                                                                                      \
    filter_t<L, double2>(h, a, nullptr, n, FILT_SPEC, psf_hat, 1, 1.0, coef, n, nd, n, n, out, \
                         accumulate, work, tmp, s);                                            \
    break;
    IMGR_FFT64_SIZES(X)
#undef X
    default: throw Error{IMGR_EINVAL, "unsupported FFT size"};
  }
  IMGR_HIP(hipGetLastError());
}

void image_gamma64_pair(imgr_s *h, const double *a0, int own0, double coef0, double *out0,
                        int acc0, const double *a1, int own1, double coef1, double *out1,
                        int acc1, double2 *work, double2 *tmp, hipStream_t s) {
  const int n = h->N;
  const size_t nn = (size_t)n * n;
  GammaPair<double2> g;
  g.m[0] = GammaMember<double2>{a0, out0, work, tmp, coef0, own0, acc0, 0};
  g.m[1] = GammaMember<double2>{a1, out1, work + nn, tmp + nn, coef1, own1, acc1, 0};
  switch (n) {
#define X(L) \
  case L: gamma_pair_t<L, double2>(h, g, s); break;
    IMGR_FFT64_SIZES(X)
#undef X
    default: throw Error{IMGR_EINVAL, "unsupported FFT size"};
  }
  IMGR_HIP(hipGetLastError());
}

void fft2_plain64(imgr_s *h, double2 *buf, double2 *tmp, int n, int dir, hipStream_t s) {
  switch (n) {
#define X(L) \
  case L: plain_t<L, double2>(h, buf, tmp, dir, s); break;
    IMGR_FFT64_SIZES(X)
#undef X
    default: throw Error{IMGR_EINVAL, "unsupported FFT size"};
  }
  IMGR_HIP(hipGetLastError());
}

}  // namespace imgr
