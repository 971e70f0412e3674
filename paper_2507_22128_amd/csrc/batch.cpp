// Batched channels: the major cycles (Eq. 2) of many single-partition
// handles with the de/gridding of many of them in one fused launch.
//
// Frequency channels share the array but not their uv coordinates, flags,
// cell or image size, so their visibility counts and chunk counts differ
// widely; launched one by one, each small channel leaves most of the 256
// compute units idle at the head and tail of its launch.  The batch keeps
// one device table of per-grid kernel arguments (bins, model grid, chunk
// windows) and, per member set, one (grid, chunk) list in decreasing chunk
// size, so a single k_window_batch launch spreads the set's chunks over the
// whole chip, and a single k_flush_batch covers the set's grids.  The
// members of a set with one image size also run each pass of their model
// and residual transforms as one launch (k_*_batch in the FFT source).  The
// per-chunk, per-cell, per-row and per-column-block arithmetic is the same
// device code as the single-handle path, so results match it bit for bit.
// The whole cycle can be captured into a HIP graph and replayed; it holds no
// memset nodes.
//
// By default all members form one set: one fused de/gridding launch and one
// fused flush per major cycle for every channel, and one launch per
// transform pass per image size.  imager_batch_set_bytes can split the
// members into consecutive sets whose model grids and chunk windows stay
// within a cache budget, each set running its stages back to back so a grid
// written by one stage is still cached when the next reads it; measured on
// 64 channels of 3.8 - 14.9M visibilities (images 512 - 2048), one set
// takes 16.4 ms per cycle against 17.4 ms for sets of 128 MB (half of the
// last-level cache), and 4.8 against 5.7 ms on 256 small channels: the
// longer launches keep the chip fuller than the cache saves.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "common.h"

struct imgr_batch_s {
  std::vector<imgr_s *> m;
  int W = 0, blk = 0;
  size_t set_bytes = 0;              // cache budget of a member set (0: one set)
  hipStream_t stream = nullptr;      // the members' stream
  hipStream_t cap_stream = nullptr;  // private stream used only for graph capture
  // device tables of the fused launches
  imgr::WinArgs *d_win = nullptr;
  imgr::FlushArgs *d_flush = nullptr;
  int2 *d_order = nullptr;
  int32_t *d_gstart = nullptr;
  int n_slots = 0, n_groups = 0;
  // consecutive member sets: members [g0, g1), slots [slot0, slot0 + n_slots)
  // of d_order, flush-group offsets d_gstart[gs0 .. gs0 + g1 - g0] (relative)
  struct Set {
    int g0, g1, slot0, n_slots, gs0, n_groups;
  };
  std::vector<Set> sets;
  // members of one set with one grid and image side: their model / residual
  // transforms run as one batched launch per pass, arguments in
  // d_fft[off .. off + count) (member pointers of the last call)
  struct FftGroup {
    int set, ng, n, off, count, max_cb;
    std::vector<int> members;
  };
  std::vector<FftGroup> fft_groups;
  imgr::FftMember *d_fft = nullptr;
  std::vector<const void *> fft_key;  // model / residual pointers d_fft was filled for
  int64_t n_vis = 0;
  std::vector<uint64_t> versions;  // member layout versions the tables were built for
  // captured graph and the pointers it was captured with
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void *> key;
  bool broken = false;
  std::string err;
};

namespace imgr {
namespace {

void free_graph(imgr_batch_s *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->key.clear();
}

void free_tables(imgr_batch_s *b) {
  for (void *q : {(void *)b->d_win, (void *)b->d_flush, (void *)b->d_order, (void *)b->d_gstart,
                  (void *)b->d_fft})
    if (q) (void)hipFree(q);
  b->d_win = nullptr;
  b->d_flush = nullptr;
  b->d_order = nullptr;
  b->d_gstart = nullptr;
  b->d_fft = nullptr;
  b->fft_key.clear();
}

template <typename T>
T *upload(const std::vector<T> &v, hipStream_t s) {
  T *d = nullptr;
  IMGR_HIP(hipMalloc((void **)&d, std::max<size_t>(v.size(), 1) * sizeof(T)));
  if (!v.empty()) IMGR_HIP(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return d;
}

// (Re)build the device tables from the members' current bins and buffers.
void build_tables(imgr_batch_s *b) {
  hipStream_t s = b->stream;
  IMGR_HIP(hipStreamSynchronize(s));
  free_graph(b);
  free_tables(b);
  const int n = (int)b->m.size();
  std::vector<WinArgs> win(n);
  std::vector<FlushArgs> fl(n);
  std::vector<int32_t> gstart;
  // (size, grid, chunk) of every chunk of a set, grids in member order
  struct Item {
    int32_t size, grid, chunk;
  };
  std::vector<Item> items;
  std::vector<int2> order;
  b->sets.clear();
  b->n_vis = 0;
  b->versions.resize(n);
  size_t set_bytes = 0;
  auto close_set = [&](int g1) {
    imgr_batch_s::Set &st = b->sets.back();
    st.g1 = g1;
    std::stable_sort(items.begin(), items.end(),
                     [](const Item &x, const Item &y) { return x.size > y.size; });
    for (const Item &it : items) order.push_back(make_int2(it.grid, it.chunk));
    st.n_slots = (int)items.size();
    st.n_groups = gstart.back();
    items.clear();
  };
  for (int g = 0; g < n; ++g) {
    imgr_s *h = b->m[g];
    const Bins &B = h->part[0].bins;
    Work &wk = h->work[0];
    const size_t bytes = (size_t)B.ng * B.ng * sizeof(float2) + (size_t)B.n_chunks * kWin * kWin *
                                                                   sizeof(float2);
    if (g == 0 || (b->set_bytes && set_bytes + bytes > b->set_bytes)) {
      if (g > 0) close_set(g);
      b->sets.push_back({g, g, (int)order.size(), 0, (int)gstart.size(), 0});
      gstart.push_back(0);
      set_bytes = 0;
    }
    set_bytes += bytes;
    win[g] = win_args(h, B, wk.grid_a, nullptr, nullptr, wk.scratch);
    fl[g] = flush_args(B, wk.scratch, wk.grid_a);
    gstart.push_back(gstart.back() + flush_groups(B));
    std::vector<int32_t> cb(B.n_chunks + 1);
    IMGR_HIP(hipMemcpyAsync(cb.data(), B.chunk_begin, (B.n_chunks + 1) * sizeof(int32_t),
                            hipMemcpyDeviceToHost, s));
    IMGR_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < B.n_chunks; ++c) items.push_back({cb[c + 1] - cb[c], g, c});
    b->n_vis += B.n;
    b->versions[g] = h->layout_version;
  }
  if (n > 0) close_set(n);
  IMGR_CHECK(order.size() < (size_t)INT32_MAX, "too many chunks for one launch");
  b->n_slots = (int)order.size();
  b->n_groups = 0;
  for (const imgr_batch_s::Set &st : b->sets) b->n_groups += st.n_groups;
  // transform groups: per set, members of equal (Ng, N) in member order
  b->fft_groups.clear();
  int off = 0;
  for (int si = 0; si < (int)b->sets.size(); ++si) {
    const imgr_batch_s::Set &st = b->sets[si];
    const size_t first = b->fft_groups.size();
    for (int g = st.g0; g < st.g1; ++g) {
      imgr_s *h = b->m[g];
      const Box &box = h->part[0].bins.box;
      imgr_batch_s::FftGroup *grp = nullptr;
      for (size_t k = first; k < b->fft_groups.size(); ++k)
        if (b->fft_groups[k].ng == h->Ng && b->fft_groups[k].n == h->N) grp = &b->fft_groups[k];
      if (!grp) {
        b->fft_groups.push_back({si, h->Ng, h->N, 0, 0, 0, {}});
        grp = &b->fft_groups.back();
      }
      grp->members.push_back(g);
      grp->max_cb = std::max(grp->max_cb, (box.x1 - box.x0) / 64);
    }
    for (size_t k = first; k < b->fft_groups.size(); ++k) {
      b->fft_groups[k].off = off;
      b->fft_groups[k].count = (int)b->fft_groups[k].members.size();
      off += b->fft_groups[k].count;
    }
  }
  IMGR_HIP(hipMalloc((void **)&b->d_fft, std::max(off, 1) * sizeof(FftMember)));
  b->fft_key.clear();
  b->d_win = upload(win, s);
  b->d_flush = upload(fl, s);
  b->d_order = upload(order, s);
  b->d_gstart = upload(gstart, s);
  IMGR_HIP(hipStreamSynchronize(s));
}

void refresh(imgr_batch_s *b) {
  for (size_t g = 0; g < b->m.size(); ++g)
    if (b->m[g]->broken) throw Error{IMGR_ESTATE, "a member handle is unusable"};
  bool stale = b->versions.size() != b->m.size();
  for (size_t g = 0; !stale && g < b->m.size(); ++g)
    stale = b->versions[g] != b->m[g]->layout_version;
  if (stale) build_tables(b);
}

// fused de/gridding and flush of the members of one set (model grids
// already in work[0].grid_a; residual grids left there)
void fused_set(imgr_batch_s *b, const imgr_batch_s::Set &st, hipStream_t s) {
  degrid_grid_batch(b->W, b->blk, b->d_win, b->d_order + st.slot0, st.n_slots, s);
  flush_batch(b->W, b->blk, b->d_flush + st.g0, b->d_gstart + st.gs0, st.g1 - st.g0,
              st.n_groups, s);
}

void fused_window(imgr_batch_s *b, hipStream_t s) {
  for (const imgr_batch_s::Set &st : b->sets) fused_set(b, st, s);
}

// the transform arguments of every member for the model / residual
// pointers of this call (uploaded when they change; the stream is drained
// first, since earlier cycles may still read the table)
void fill_fft_table(imgr_batch_s *b, const float *const *model, float *const *residual) {
  const int n = (int)b->m.size();
  std::vector<const void *> key(2 * n);
  for (int g = 0; g < n; ++g) {
    key[g] = model[g];
    key[n + g] = residual[g];
  }
  if (key == b->fft_key) return;
  std::vector<FftMember> tab;
  for (const imgr_batch_s::FftGroup &grp : b->fft_groups)
    for (int g : grp.members) {
      imgr_s *h = b->m[g];
      Work &wk = h->work[0];
      const Box &box = h->part[0].bins.box;
      tab.push_back(FftMember{model[g], residual[g], wk.rows, wk.grid_b, wk.grid_a, h->cinv,
                              (float)(1.0 / h->part[0].sum_w), box.x0, box.x1, box.y0, box.y1});
    }
  IMGR_HIP(hipStreamSynchronize(b->stream));
  if (!tab.empty())
    IMGR_HIP(hipMemcpy(b->d_fft, tab.data(), tab.size() * sizeof(FftMember),
                       hipMemcpyHostToDevice));
  b->fft_key = key;
}

void enqueue_cycle(imgr_batch_s *b, hipStream_t s) {
  for (int si = 0; si < (int)b->sets.size(); ++si) {
    for (const imgr_batch_s::FftGroup &grp : b->fft_groups)
      if (grp.set == si)
        fft_model_to_grid_batch(b->m[grp.members[0]], grp.ng, grp.n, b->d_fft + grp.off,
                                grp.count, grp.max_cb, s);
    fused_set(b, b->sets[si], s);
    for (const imgr_batch_s::FftGroup &grp : b->fft_groups)
      if (grp.set == si)
        fft_grid_to_image_batch(b->m[grp.members[0]], grp.ng, grp.n, b->d_fft + grp.off,
                                grp.count, grp.max_cb, s);
  }
}

void check_cycle(imgr_batch_s *b, const float *const *model, float *const *residual) {
  IMGR_CHECK(model && residual, "null pointer array");
  for (size_t g = 0; g < b->m.size(); ++g) IMGR_CHECK(model[g] && residual[g], "null image");
}

}  // namespace
}  // namespace imgr

using namespace imgr;

#define BATCH_BEGIN(b)                                                \
  if (!(b)) return IMGR_EINVAL;                                       \
  if ((b)->broken) {                                                  \
    (b)->err = "batch is unusable after an earlier device error";     \
    return IMGR_ESTATE;                                               \
  }                                                                   \
  try {
#define BATCH_END(b)                 \
  }                                  \
  catch (const Error &e) {           \
    (b)->err = e.msg;                \
    if (e.code == IMGR_EDEVICE) (b)->broken = true; \
    return e.code;                   \
  }                                  \
  catch (const std::exception &e) {  \
    (b)->err = e.what();             \
    return IMGR_EINVAL;              \
  }                                  \
  return IMGR_OK;

static void release_batch(imgr_batch_s *b) {
  if (b->stream || b->cap_stream) (void)hipStreamSynchronize(b->stream);
  free_graph(b);
  free_tables(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
}

static thread_local std::string g_batch_create_error;

extern "C" {

imgr_status imager_batch_create(const imgr_t *members, int32_t n, imgr_batch_t *out) {
  if (out) *out = nullptr;
  if (!members || n < 1 || !out) {
    g_batch_create_error = "bad arguments";
    return IMGR_EINVAL;
  }
  imgr_batch_s *b = new imgr_batch_s();
  try {
    for (int g = 0; g < n; ++g) {
      imgr_s *h = members[g];
      IMGR_CHECK(h != nullptr, "null member");
      IMGR_CHECK(!h->broken, "a member handle is unusable");
      IMGR_CHECK(h->n_parts == 1, "batch members must have one partition");
      for (int q = 0; q < g; ++q) IMGR_CHECK(members[q] != h, "a member appears twice");
      if (g == 0) {
        b->W = h->W;
        b->blk = h->blk;
        b->stream = h->stream;
      }
      IMGR_CHECK(h->W == b->W && h->blk == b->blk, "members must share support and tile");
      IMGR_CHECK(h->stream == b->stream, "members must share one stream");
      b->m.push_back(h);
    }
    IMGR_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    build_tables(b);
  } catch (const Error &e) {
    g_batch_create_error = e.msg;
    release_batch(b);
    return e.code;
  } catch (const std::exception &e) {
    g_batch_create_error = e.what();
    release_batch(b);
    return IMGR_EINVAL;
  }
  *out = b;
  return IMGR_OK;
}

imgr_status imager_batch_set_bytes(imgr_batch_t b, uint64_t bytes) {
  BATCH_BEGIN(b)
  b->set_bytes = (size_t)bytes;
  build_tables(b);
  BATCH_END(b)
}

imgr_status imager_batch_destroy(imgr_batch_t b) {
  if (!b) return IMGR_EINVAL;
  release_batch(b);
  return IMGR_OK;
}

imgr_status imager_batch_info(imgr_batch_t b, imgr_batch_info *o) {
  if (!b || !o) return IMGR_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->n_members = (int32_t)b->m.size();
  o->support = b->W;
  o->tile = b->blk;
  o->chunk = b->m.empty() ? 0 : b->m[0]->C;
  for (imgr_s *h : b->m)
    if (h->C != o->chunk) o->chunk = -1;  // members differ
  o->n_vis = b->n_vis;
  o->n_chunks = b->n_slots;
  o->graph_ready = b->exec != nullptr;
  o->n_sets = (int32_t)b->sets.size();
  return IMGR_OK;
}

imgr_status imager_batch_major_cycle(imgr_batch_t b, const float *const *model,
                                     float *const *residual, int32_t flags) {
  BATCH_BEGIN(b)
  check_cycle(b, model, residual);
  IMGR_CHECK((flags & ~(IMGR_BATCH_GRAPH | IMGR_BATCH_LOOP)) == 0, "unknown flags");
  IMGR_CHECK(!((flags & IMGR_BATCH_GRAPH) && (flags & IMGR_BATCH_LOOP)),
             "GRAPH and LOOP are exclusive");
  refresh(b);
  const int n = (int)b->m.size();
  if (flags & IMGR_BATCH_LOOP) {
    for (int g = 0; g < n; ++g)
      node_cycle(b->m[g], 0, model[g], nullptr, 1.0, 0.0, residual[g], residual[g], 0, b->stream);
    return IMGR_OK;
  }
  fill_fft_table(b, model, residual);
  if (!(flags & IMGR_BATCH_GRAPH)) {
    enqueue_cycle(b, b->stream);
    return IMGR_OK;
  }
  std::vector<const void *> key(2 * n);
  for (int g = 0; g < n; ++g) {
    key[g] = model[g];
    key[n + g] = residual[g];
  }
  if (!b->exec || key != b->key) {
    free_graph(b);
    IMGR_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    try {
      enqueue_cycle(b, b->cap_stream);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(b->cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    IMGR_HIP(hipStreamEndCapture(b->cap_stream, &b->graph));
    IMGR_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->key = key;
  }
  IMGR_HIP(hipGraphLaunch(b->exec, b->stream));
  BATCH_END(b)
}

imgr_status imager_batch_autotune(imgr_batch_t b, const int32_t *caps, int32_t n_caps,
                                  int32_t reps, float *ms, int32_t *chosen) {
  BATCH_BEGIN(b)
  IMGR_CHECK(caps && n_caps >= 1 && reps >= 1, "bad arguments");
  for (int i = 0; i < n_caps; ++i)
    IMGR_CHECK(caps[i] >= 16 && caps[i] <= (1 << 20), "chunk caps must be in [16, 2^20]");
  refresh(b);
  hipStream_t s = b->stream;
  // zero model grids: the timing must not depend on a previous cycle's data
  hipEvent_t e0, e1;
  IMGR_HIP(hipEventCreate(&e0));
  IMGR_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int best_cap = caps[0];
  try {
    for (int i = 0; i < n_caps; ++i) {
      for (imgr_s *h : b->m)
        if (h->C != caps[i]) set_chunk(h, caps[i]);
      refresh(b);
      for (imgr_s *h : b->m)
        IMGR_HIP(hipMemsetAsync(h->work[0].grid_a, 0, (size_t)h->Ng * h->Ng * sizeof(float2), s));
      float t = 1e30f;
      for (int r = 0; r <= reps; ++r) {
        IMGR_HIP(hipEventRecord(e0, s));
        fused_window(b, s);
        IMGR_HIP(hipEventRecord(e1, s));
        IMGR_HIP(hipEventSynchronize(e1));
        float x = 0.f;
        IMGR_HIP(hipEventElapsedTime(&x, e0, e1));
        if (r > 0) t = std::min(t, x);
        // the flush overwrote the model grids; zero them again
        for (imgr_s *h : b->m)
          IMGR_HIP(hipMemsetAsync(h->work[0].grid_a, 0, (size_t)h->Ng * h->Ng * sizeof(float2), s));
      }
      if (ms) ms[i] = t;
      if (t < best) {
        best = t;
        best_cap = caps[i];
      }
    }
    for (imgr_s *h : b->m)
      if (h->C != best_cap) set_chunk(h, best_cap);
    refresh(b);
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (chosen) *chosen = best_cap;
  BATCH_END(b)
}

const char *imager_batch_last_error(imgr_batch_t b) {
  if (!b) return g_batch_create_error.c_str();
  return b->err.c_str();
}

}  // extern "C"
