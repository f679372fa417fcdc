// sw_runtime.hip -- host side of the gfx950 word sort: the C ABI declared in
// include/sort_words.h, workspace layout, launch sequence, graph-captured
// plans, the per-bucket-launch form and kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "sort_words.h"
#include "sw_kernels.hpp"
#include "sw_text.hpp"

namespace {

using sw::Header;
using sw::RunDesc;
using sw::TileWork;
using sw::Ws;

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(SW_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr int kNT = 256;         // threads per workgroup of the streaming kernels
constexpr int kScatterNT = 512;  // threads per workgroup of k_scatter_pack

// ------------------------------------------------------------------ variants
// A variant fixes, for one key class, the chunk-sort tile (NTS threads x ES
// items) and the merge tile (NTM threads x EM items).
struct Variant {
  void (*sort)(const Ws&, int, TileWork, unsigned, hipStream_t);
  void (*packed)(const Ws&, int, unsigned, hipStream_t);
  void (*partition)(const Ws&, int, int, TileWork, unsigned, hipStream_t);
  void (*merge)(const Ws&, int, int, TileWork, unsigned, hipStream_t);
  const void* sort_fn;
  const void* merge_fn;
  uint32_t T, P;
  int nts, ntm;
};

constexpr int kPartNT = 256;

template <int NL, int NTS, int ES, int NTM, int EM, int MM = 0>
struct V {
  static void sort(const Ws& w, int c, TileWork tw, unsigned grid, hipStream_t s) {
    sw::k_sort_tiles<NL, NTS, ES, MM><<<grid, NTS, 0, s>>>(w, c, tw);
  }
  static void packed(const Ws& w, int c, unsigned grid, hipStream_t s) {
    sw::k_sort_packed<NL, 8, 0><<<grid, sw::kPackTile / 8, 0, s>>>(w, c);
  }
  static void partition(const Ws& w, int c, int l, TileWork tw, unsigned grid, hipStream_t s) {
    sw::k_partition<NL, kPartNT><<<grid, kPartNT, 0, s>>>(w, c, l, tw, (uint32_t)(NTM * EM));
  }
  static void merge(const Ws& w, int c, int l, TileWork tw, unsigned grid, hipStream_t s) {
    sw::k_merge<NL, NTM, EM, MM><<<grid, NTM, 0, s>>>(w, c, l, tw);
  }
  static Variant get() {
    static_assert(NTM * EM >= (int)sw::kMinMergeTile, "merge tile below the split-array sizing");
    static_assert(NTM * EM <= 2 * NTS * ES, "merge tile must divide a pair of sorted tiles");
    return Variant{sort, packed, partition, merge, (const void*)sw::k_sort_tiles<NL, NTS, ES, MM>,
                   (const void*)sw::k_merge<NL, NTM, EM, MM>, (uint32_t)(NTS * ES), (uint32_t)(NTM * EM), NTS, NTM};
  }
};

// The last template argument picks the register merge: 0 serial, 1 bitonic.
constexpr int kMaxVariants = 8;
const Variant* variants(int c, int* count) {
  static const Variant v0[] = {V<0, 256, 16, 256, 16, 0>::get(), V<0, 256, 8, 256, 8, 0>::get(),
                               V<0, 512, 16, 256, 16, 0>::get(), V<0, 512, 16, 256, 8, 0>::get(),
                               V<0, 512, 16, 256, 16, 1>::get(), V<0, 512, 16, 256, 8, 1>::get(),
                               V<0, 1024, 16, 256, 16, 0>::get()};
  static const Variant v1[] = {V<1, 256, 16, 256, 16, 0>::get(), V<1, 256, 8, 256, 8, 0>::get(),
                               V<1, 512, 16, 256, 8, 0>::get(), V<1, 512, 16, 256, 16, 0>::get(),
                               V<1, 512, 16, 256, 8, 1>::get(), V<1, 256, 8, 256, 8, 1>::get(),
                               V<1, 1024, 8, 256, 16, 0>::get()};
  static const Variant v2[] = {V<2, 256, 16, 256, 16, 0>::get(), V<2, 256, 8, 256, 8, 0>::get(),
                               V<2, 256, 8, 256, 16, 0>::get(), V<2, 256, 8, 256, 8, 1>::get(),
                               V<2, 512, 8, 256, 8, 1>::get(), V<2, 512, 8, 256, 16, 0>::get()};
  static const Variant v3[] = {V<4, 256, 8, 256, 8, 0>::get(), V<4, 128, 16, 128, 16, 0>::get(),
                               V<4, 128, 16, 256, 8, 0>::get()};
  static const Variant* all[] = {v0, v1, v2, v3};
  static const int counts[] = {7, 7, 6, 3};
  *count = counts[c];
  return all[c];
}

// ------------------------------------------------------------------ config
std::mutex g_cfg_mu;
sw_config g_cfg = {{16, 16, 16, 16}, {0, 0, 0, 0}, 0};

sw_config current_config() {
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  return g_cfg;
}

// ------------------------------------------------------------------ device info
struct DevInfo {
  bool ready = false;
  int cus = 0;
  int occ_hist = 1, occ_scatter = 1;
  int occ_sort[sw::kNClass][kMaxVariants] = {};
  int occ_merge[sw::kNClass][kMaxVariants] = {};
};
std::mutex g_dev_mu;
DevInfo g_dev[64];

int device_info(DevInfo** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(SW_ERR_HIP, "device id %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_dev_mu);
  DevInfo& d = g_dev[dev];
  if (!d.ready) {
    HIP_TRY(hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&d.occ_hist, (const void*)sw::k_hist<kNT>, kNT, 0));
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&d.occ_scatter, (const void*)sw::k_scatter_pack<kScatterNT>,
                                                         kScatterNT, 0));
    for (int c = 0; c < sw::kNClass; ++c) {
      int nv;
      const Variant* vs = variants(c, &nv);
      for (int v = 0; v < nv; ++v) {
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&d.occ_sort[c][v], vs[v].sort_fn, vs[v].nts, 0));
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&d.occ_merge[c][v], vs[v].merge_fn, vs[v].ntm, 0));
        d.occ_sort[c][v] = std::max(d.occ_sort[c][v], 1);
        d.occ_merge[c][v] = std::max(d.occ_merge[c][v], 1);
      }
    }
    d.occ_hist = std::max(d.occ_hist, 1);
    d.occ_scatter = std::max(d.occ_scatter, 1);
    d.ready = true;
  }
  *out = &d;
  return SW_OK;
}

// ------------------------------------------------------------------ layout
struct Layout {
  uint64_t Nmax = 0, Dmax = 0, Bmax = 0, Smax = 0, SBmax = 0, rec_stride = 0;
  size_t o_hdr, o_doc_off, o_doc_blk, o_cnt, o_seg_n, o_seg_base, o_segcnt, o_sorted, o_st, o_mt, o_vpre, o_rec;
  size_t o_a[4], o_ai, o_b[4], o_bi;
  size_t total = 0;
};

bool make_layout(uint64_t Nmax, uint64_t Dmax, Layout& L) {
  if (Dmax == 0) Dmax = 1;
  if (Nmax > 0xFFFFFFFFull || Dmax > 0xFFFFFFFFull / sw::kNB) return false;
  L.Nmax = Nmax;
  L.Dmax = Dmax;
  L.Bmax = (Nmax + sw::kWordsPerBlock - 1) / sw::kWordsPerBlock + Dmax;
  L.Smax = Dmax * sw::kNB;
  L.SBmax = (L.Smax + sw::kSegsPerBlock - 1) / sw::kSegsPerBlock;
  const uint64_t N1 = Nmax ? Nmax : 1;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    const size_t o = at;
    at += (bytes + 255) & ~(size_t)255;
    return o;
  };
  L.o_hdr = take(sizeof(Header));
  L.o_doc_off = take(4 * (Dmax + 1));
  L.o_doc_blk = take(4 * (Dmax + 1));
  L.o_cnt = take(4 * (size_t)sw::kNB * (L.Bmax + 1));
  L.o_seg_n = take(4 * L.Smax);
  L.o_seg_base = take(4 * L.Smax);
  L.o_segcnt = take(4 * (size_t)sw::kNKeys * (L.SBmax + 1));
  L.o_sorted = take(4 * L.Smax);
  L.o_st = take(4 * (L.Smax + sw::kNClass));
  L.o_mt = take(4 * (L.Smax + sw::kNClass));
  L.o_vpre = take(4 * (L.Smax + sw::kNClass));
  L.rec_stride = Nmax / sw::kMinMergeTile + L.Smax + 2;
  L.o_rec = take(16 * sw::kNClass * L.rec_stride);
  for (int q = 0; q < 4; ++q) L.o_a[q] = take(8 * N1);
  L.o_ai = take(4 * N1);
  for (int q = 0; q < 4; ++q) L.o_b[q] = take(8 * N1);
  L.o_bi = take(4 * N1);
  L.total = at;
  return true;
}

// Largest word capacity whose layout (with Dmax documents) fits in `bytes`.
uint64_t capacity_for(size_t bytes, uint64_t Dmax) {
  Layout L;
  if (!make_layout(0, Dmax, L) || L.total > bytes) return 0;
  uint64_t lo = 0, hi = 0xFFFFFFFFull;
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo + 1) / 2;
    if (make_layout(mid, Dmax, L) && L.total <= bytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

Ws make_ws(void* base, const Layout& L, const sw_config& cfg) {
  char* p = (char*)base;
  Ws w;
  w.h = (Header*)(p + L.o_hdr);
  w.doc_off = (uint32_t*)(p + L.o_doc_off);
  w.doc_blk = (uint32_t*)(p + L.o_doc_blk);
  w.cnt = (uint32_t*)(p + L.o_cnt);
  w.seg_n = (uint32_t*)(p + L.o_seg_n);
  w.seg_base = (uint32_t*)(p + L.o_seg_base);
  w.segcnt = (uint32_t*)(p + L.o_segcnt);
  w.sorted = (uint32_t*)(p + L.o_sorted);
  w.st = (uint32_t*)(p + L.o_st);
  w.mt = (uint32_t*)(p + L.o_mt);
  w.vpre = (uint32_t*)(p + L.o_vpre);
  w.rec = (uint4*)(p + L.o_rec);
  w.rec_stride = (uint32_t)L.rec_stride;
  for (int q = 0; q < 4; ++q) {
    w.a.k[q] = (uint64_t*)(p + L.o_a[q]);
    w.b.k[q] = (uint64_t*)(p + L.o_b[q]);
  }
  w.a.idx = (uint32_t*)(p + L.o_ai);
  w.b.idx = (uint32_t*)(p + L.o_bi);
  w.Nmax = (uint32_t)L.Nmax;
  w.Dmax = (uint32_t)L.Dmax;
  w.Bmax = (uint32_t)L.Bmax;
  w.Smax = (uint32_t)L.Smax;
  w.SBmax = (uint32_t)L.SBmax;
  for (int c = 0; c < sw::kNClass; ++c) {
    int nv;
    const Variant& v = variants(c, &nv)[cfg.variant[c]];
    w.T[c] = v.T;
    w.P[c] = v.P;
    w.chunk[c] = cfg.chunk[c];
  }
  return w;
}

// ------------------------------------------------------------------ profiling
enum KernelId {
  K_BEGIN, K_DOC_PLAN, K_HIST, K_SCAN, K_SEGMENTS, K_SEG_COUNT, K_SEG_SCATTER, K_TILE_PREFIX, K_SCATTER,
  K_SORT0, K_SORT1, K_SORT2, K_SORT3, K_MERGE0, K_MERGE1, K_MERGE2, K_MERGE3,
  K_PART0, K_PART1, K_PART2, K_PART3, K_PACK0, K_PACK1, K_PACK2, K_PACK3, K_COUNT
};
const char* const kKernelNames[K_COUNT] = {
    "begin", "doc_plan", "hist", "scan_rows", "segments", "seg_count", "seg_scatter", "tile_prefix",
    "scatter_pack", "sort_tiles_c0", "sort_tiles_c1", "sort_tiles_c2", "sort_tiles_c3",
    "merge_c0", "merge_c1", "merge_c2", "merge_c3",
    "partition_c0", "partition_c1", "partition_c2", "partition_c3",
    "sort_packed_c0", "sort_packed_c1", "sort_packed_c2", "sort_packed_c3"};

struct ProfRec {
  int kid;
  hipEvent_t e0, e1;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_recs;
std::vector<hipEvent_t> g_prof_pool;
double g_prof_ms[K_COUNT];
uint32_t g_prof_n[K_COUNT];

hipEvent_t prof_event() {
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch with events when profiling is on (never inside capture).
struct ProfScope {
  bool on;
  int kid;
  hipStream_t s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ProfScope(int k, hipStream_t st, bool capture) : on(false), kid(k), s(st) {
    if (capture) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return;
    e0 = prof_event();
    e1 = prof_event();
    if (!e0 || !e1) return;
    on = hipEventRecord(e0, s) == hipSuccess;
  }
  ~ProfScope() {
    if (!on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (hipEventRecord(e1, s) == hipSuccess) g_prof_recs.push_back(ProfRec{kid, e0, e1});
  }
};

// ------------------------------------------------------------------ launch sequence
struct Grids {
  uint32_t flags;
  unsigned words, scatter, docs, segs;
  unsigned sort[sw::kNClass], merge[sw::kNClass], part[sw::kNClass], packed;
  int levels[sw::kNClass];
  const Variant* var[sw::kNClass];
};

int make_grids(const Ws& w, const sw_config& cfg, Grids& g) {
  DevInfo* d;
  int rc = device_info(&d);
  if (rc) return rc;
  const uint64_t cus = (uint64_t)d->cus;
  auto clampg = [](uint64_t want, uint64_t cap) { return (unsigned)std::max<uint64_t>(1, std::min(want, cap)); };
  g.flags = cfg.flags;
  g.words = clampg(w.Bmax, cus * (uint64_t)d->occ_hist);
  g.scatter = clampg(w.Bmax, cus * (uint64_t)d->occ_scatter);
  g.docs = clampg((w.Dmax + 3) / 4, cus * 4);
  g.packed = clampg((uint64_t)w.Nmax / sw::kPackMax + 1, cus * 4);
  g.segs = clampg(w.SBmax, cus * 2);
  for (int c = 0; c < sw::kNClass; ++c) {
    int nv;
    const Variant* vs = variants(c, &nv);
    const int v = (int)cfg.variant[c];
    g.var[c] = &vs[v];
    const uint64_t maxtiles_s = (uint64_t)w.Nmax / vs[v].T + w.Smax;
    const uint64_t maxtiles_m = (uint64_t)w.Nmax / vs[v].P + w.Smax;
    g.sort[c] = clampg(maxtiles_s, cus * (uint64_t)d->occ_sort[c][v]);
    g.merge[c] = clampg(maxtiles_m, cus * (uint64_t)d->occ_merge[c][v]);
    const uint64_t tiles_per_wg = (uint64_t)(kPartNT / 64) * (64 / sw::kPartLanes);
    g.part[c] = clampg((maxtiles_m + tiles_per_wg - 1) / tiles_per_wg, cus * 8);
    g.levels[c] = (int)sw::levels_for(w.Nmax, vs[v].T);
  }
  return SW_OK;
}

// Side streams and events for running the four key classes concurrently:
// after the scatter the classes share nothing, so each class's chain (chunk
// sort, then partition + merge per level) goes on its own stream, forked
// from and joined back into the caller's stream.  Under graph capture the
// chains become parallel branches of the graph.
struct Fork {
  hipStream_t side[sw::kNClass] = {};   // side[0] unused: class 0 stays on the main stream
  hipEvent_t fork = nullptr;
  hipEvent_t join[sw::kNClass] = {};
  bool ready = false;
};

int fork_init(Fork& f) {
  if (f.ready) return SW_OK;
  for (int c = 1; c < sw::kNClass; ++c) HIP_TRY(hipStreamCreateWithFlags(&f.side[c], hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&f.fork, hipEventDisableTiming));
  for (int c = 1; c < sw::kNClass; ++c) HIP_TRY(hipEventCreateWithFlags(&f.join[c], hipEventDisableTiming));
  f.ready = true;
  return SW_OK;
}

void fork_free(Fork& f) {
  if (!f.ready) return;
  for (int c = 1; c < sw::kNClass; ++c) {
    if (f.side[c]) (void)hipStreamSynchronize(f.side[c]);
  }
  for (int c = 1; c < sw::kNClass; ++c) {
    if (f.side[c]) (void)hipStreamDestroy(f.side[c]);
    if (f.join[c]) (void)hipEventDestroy(f.join[c]);
  }
  if (f.fork) (void)hipEventDestroy(f.fork);
  f = Fork();
}

bool profiling_on() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  return g_prof_on;
}

// Everything after k_begin.  With `through_scatter` only the pre-pass and the
// scatter are enqueued (the per-bucket-launch form continues on the host).
// With a Fork the key classes run on parallel streams; without one (or while
// profiling, so that every kernel is timed alone) they run one after another.
int enqueue_body(const Ws& w, const Grids& g, hipStream_t s, bool capture, bool through_scatter,
                 Fork* fork = nullptr) {
  {
    ProfScope p(K_DOC_PLAN, s, capture);
    sw::k_doc_plan<1024><<<1, 1024, 0, s>>>(w);
  }
  {
    ProfScope p(K_HIST, s, capture);
    sw::k_hist<kNT><<<g.words, kNT, 0, s>>>(w);
  }
  {
    ProfScope p(K_SCAN, s, capture);
    sw::k_scan_rows<1024, 4><<<sw::kNB, 1024, 0, s>>>(w, w.cnt, sw::kNB, w.Bmax + 1, 0);
  }
  {
    ProfScope p(K_SEGMENTS, s, capture);
    sw::k_segments<kNT><<<g.docs, kNT, 0, s>>>(w);
  }
  if (!through_scatter) {
    {
      ProfScope p(K_SEG_COUNT, s, capture);
      sw::k_seg_count<kNT><<<g.segs, kNT, 0, s>>>(w);
    }
    {
      ProfScope p(K_SCAN, s, capture);
      sw::k_scan_rows<1024, 4><<<sw::kNKeys, 1024, 0, s>>>(w, w.segcnt, sw::kNKeys, w.SBmax + 1, 1);
    }
    {
      ProfScope p(K_SEG_SCATTER, s, capture);
      sw::k_seg_scatter<kNT><<<g.segs, kNT, 0, s>>>(w);
    }
    {
      ProfScope p(K_TILE_PREFIX, s, capture);
      sw::k_tile_prefix<1024><<<3 * sw::kNClass, 1024, 0, s>>>(w);
    }
  }
  {
    ProfScope p(K_SCATTER, s, capture);
    sw::k_scatter_pack<kScatterNT><<<g.scatter, kScatterNT, 0, s>>>(w);
  }
  if (through_scatter) return SW_OK;
  const bool par = fork && fork->ready && !(!capture && profiling_on()) && !(g.flags & SW_FLAG_SERIAL_CLASSES);
  if (par) {
    HIP_TRY(hipEventRecord(fork->fork, s));
    for (int c = 1; c < sw::kNClass; ++c) HIP_TRY(hipStreamWaitEvent(fork->side[c], fork->fork, 0));
  }
  const TileWork none{0, 0, 0, 0};
  // Each class keeps its own order on its own stream; across classes the work
  // is enqueued stage by stage (all chunk sorts, then merge level 0 of every
  // class, level 1, ...), so that a runtime which maps the parallel chains
  // onto fewer hardware queues still finds every class's next kernel early.
  auto cstream = [&](int c) { return (par && c > 0) ? fork->side[c] : s; };
  int max_levels = 0;
  for (int c = 0; c < sw::kNClass; ++c) {
    hipStream_t cs = cstream(c);
    {
      ProfScope p(K_SORT0 + c, cs, capture);
      g.var[c]->sort(w, c, none, g.sort[c], cs);
    }
    {
      ProfScope p(K_PACK0 + c, cs, capture);
      g.var[c]->packed(w, c, g.packed, cs);
    }
    max_levels = std::max(max_levels, g.levels[c]);
  }
  for (int l = 0; l < max_levels; ++l) {
    for (int c = 0; c < sw::kNClass; ++c) {
      if (l >= g.levels[c]) continue;
      hipStream_t cs = cstream(c);
      {
        ProfScope p(K_PART0 + c, cs, capture);
        g.var[c]->partition(w, c, l, none, g.part[c], cs);
      }
      ProfScope p(K_MERGE0 + c, cs, capture);
      g.var[c]->merge(w, c, l, none, g.merge[c], cs);
    }
  }
  if (par) {
    for (int c = 1; c < sw::kNClass; ++c) {
      HIP_TRY(hipEventRecord(fork->join[c], fork->side[c]));
      HIP_TRY(hipStreamWaitEvent(s, fork->join[c], 0));
    }
  }
  HIP_TRY(hipGetLastError());
  return SW_OK;
}

int enqueue_begin(const Ws& w, const RunDesc& d, hipStream_t s) {
  ProfScope p(K_BEGIN, s, false);
  sw::k_begin<<<1, 64, 0, s>>>(w, d);
  return SW_OK;
}

int status_to_code(uint32_t st) {
  if (st & sw::ST_INVALID) return fail(SW_ERR_INVALID_ARG, "device: offsets or document offsets invalid");
  if (st & sw::ST_WORKSPACE) return fail(SW_ERR_WORKSPACE, "device: word count exceeds workspace capacity");
  if (st & sw::ST_TOO_LONG) return fail(SW_ERR_WORD_TOO_LONG, "device: a word is longer than %d bytes", SW_MAX_LEN);
  return SW_OK;
}

int read_status(const void* ws, hipStream_t s) {
  HIP_TRY(hipStreamSynchronize(s));
  uint32_t st = 0;
  HIP_TRY(hipMemcpy(&st, &((const Header*)ws)->status, sizeof st, hipMemcpyDeviceToHost));
  return status_to_code(st);
}

// Side streams of the eager path, one set per device; the mutex keeps each
// fork (event record + waits) of concurrent callers consistent.
std::mutex g_fork_mu;
Fork g_fork[64];

int run_eager(const uint8_t* chars, const uint32_t* offsets, const uint32_t* doc_offsets, uint32_t n_docs,
              uint32_t n_words, uint32_t* out_perm, uint32_t* out_boff, void* ws, const Layout& L,
              hipStream_t s) {
  const sw_config cfg = current_config();
  const Ws w = make_ws(ws, L, cfg);
  Grids g;
  int rc = make_grids(w, cfg, g);
  if (rc) return rc;
  RunDesc d{chars, offsets, doc_offsets, out_perm, out_boff, n_words, n_docs};
  rc = enqueue_begin(w, d, s);
  if (rc) return rc;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_fork_mu);
  Fork& f = g_fork[dev & 63];
  if ((rc = fork_init(f))) return rc;
  return enqueue_body(w, g, s, false, false, &f);
}

// Library-owned workspace of the simple form, one per device.
struct Cache {
  void* p = nullptr;
  size_t bytes = 0;
};
std::mutex g_cache_mu;
Cache g_cache[64];

}  // namespace

// =================================================================== C ABI
extern "C" {

const char* sort_words_last_error(void) { return g_err.c_str(); }
const char* sort_words_version(void) { return "sortwords-gfx950 0.6"; }

size_t sort_words_workspace_size(uint32_t max_words, uint32_t max_docs) {
  Layout L;
  if (!make_layout(max_words, max_docs, L)) return 0;
  return L.total;
}

int sort_words_ex(const uint8_t* chars, const uint32_t* offsets, uint32_t n, uint32_t* out_perm,
                  uint32_t* out_bucket_offsets, void* workspace, size_t workspace_bytes, void* stream) {
  if (!offsets || !out_bucket_offsets || (n && !out_perm) || !workspace)
    return fail(SW_ERR_INVALID_ARG, "sort_words_ex: null pointer argument");
  Layout L;
  if (!make_layout(n, 1, L)) return fail(SW_ERR_INVALID_ARG, "sort_words_ex: n out of range");
  if (L.total > workspace_bytes)
    return fail(SW_ERR_WORKSPACE, "sort_words_ex: workspace of %zu bytes, need %zu", workspace_bytes, L.total);
  return run_eager(chars, offsets, nullptr, 1, n, out_perm, out_bucket_offsets, workspace, L, (hipStream_t)stream);
}

int sort_words(const uint8_t* chars, const uint32_t* offsets, uint32_t n, uint32_t* out_perm,
               uint32_t* out_bucket_offsets) {
  if (!offsets || !out_bucket_offsets || (n && !out_perm))
    return fail(SW_ERR_INVALID_ARG, "sort_words: null pointer argument");
  Layout L;
  if (!make_layout(n, 1, L)) return fail(SW_ERR_INVALID_ARG, "sort_words: n out of range");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(SW_ERR_HIP, "device id out of range");
  std::lock_guard<std::mutex> lk(g_cache_mu);
  Cache& c = g_cache[dev];
  if (c.bytes < L.total) {
    if (c.p) {
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipFree(c.p));
      c.p = nullptr;
      c.bytes = 0;
    }
    if (hipMalloc(&c.p, L.total) != hipSuccess) {
      (void)hipGetLastError();
      c.p = nullptr;
      return fail(SW_ERR_OOM, "sort_words: cannot allocate %zu bytes of workspace", L.total);
    }
    c.bytes = L.total;
  }
  int rc = run_eager(chars, offsets, nullptr, 1, n, out_perm, out_bucket_offsets, c.p, L, nullptr);
  if (rc) return rc;
  return read_status(c.p, nullptr);
}

int sort_words_batch(const uint8_t* chars, const uint32_t* offsets, const uint32_t* doc_offsets, uint32_t n_docs,
                     uint32_t* out_perm, uint32_t* out_bucket_offsets, void* workspace, size_t workspace_bytes,
                     void* stream) {
  if (!offsets || !doc_offsets || !out_bucket_offsets || !out_perm || !workspace)
    return fail(SW_ERR_INVALID_ARG, "sort_words_batch: null pointer argument");
  const uint64_t cap = capacity_for(workspace_bytes, n_docs);
  Layout L;
  if (!make_layout(cap, n_docs, L) || L.total > workspace_bytes)
    return fail(SW_ERR_WORKSPACE, "sort_words_batch: workspace of %zu bytes too small for %u documents",
                workspace_bytes, n_docs);
  return run_eager(chars, offsets, doc_offsets, n_docs, 0, out_perm, out_bucket_offsets, workspace, L,
                   (hipStream_t)stream);
}

int sort_words_status_async(const void* workspace, uint32_t* status_dst, void* stream) {
  if (!workspace || !status_dst) return fail(SW_ERR_INVALID_ARG, "sort_words_status_async: null argument");
  HIP_TRY(hipMemcpyAsync(status_dst, &((const Header*)workspace)->status, sizeof(uint32_t), hipMemcpyDefault,
                         (hipStream_t)stream));
  return SW_OK;
}

int sort_words_decode_status(uint32_t status_word) { return status_to_code(status_word); }

int sort_words_status(const void* workspace, void* stream) {
  if (!workspace) return fail(SW_ERR_INVALID_ARG, "sort_words_status: null workspace");
  return read_status(workspace, (hipStream_t)stream);
}

int sort_words_plain(const uint8_t* chars, const uint32_t* offsets, const uint32_t* doc_offsets, uint32_t n_docs,
                     uint32_t* out_perm, uint32_t* out_bucket_offsets, void* workspace, size_t workspace_bytes,
                     void* stream) {
  if (!offsets || !doc_offsets || !out_bucket_offsets || !out_perm || !workspace)
    return fail(SW_ERR_INVALID_ARG, "sort_words_plain: null pointer argument");
  const uint64_t cap = capacity_for(workspace_bytes, n_docs);
  Layout L;
  if (!make_layout(cap, n_docs, L) || L.total > workspace_bytes)
    return fail(SW_ERR_WORKSPACE, "sort_words_plain: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  const sw_config cfg = current_config();
  const Ws w = make_ws(workspace, L, cfg);
  Grids g;
  int rc = make_grids(w, cfg, g);
  if (rc) return rc;
  RunDesc d{chars, offsets, doc_offsets, out_perm, out_bucket_offsets, 0, n_docs};
  if ((rc = enqueue_begin(w, d, s))) return rc;
  if ((rc = enqueue_body(w, g, s, false, true))) return rc;
  // the host reads the segment table (the length histogram of every document)
  if ((rc = read_status(workspace, s))) return rc;
  const size_t S = (size_t)n_docs * sw::kNB;
  std::vector<uint32_t> seg_n(S), seg_base(S);
  if (S) {
    HIP_TRY(hipMemcpy(seg_n.data(), w.seg_n, 4 * S, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(seg_base.data(), w.seg_base, 4 * S, hipMemcpyDeviceToHost));
  }
  for (size_t sidx = 0; sidx < S; ++sidx) {
    const uint32_t n = seg_n[sidx];
    if (!n) continue;
    const int c = sw::class_of_len((uint32_t)(sidx % sw::kNB));
    const Variant& v = *g.var[c];
    const uint32_t m = sw::levels_for(n, v.T);
    const TileWork tw{1, seg_base[sidx], n, m};
    {
      ProfScope p(K_SORT0 + c, s, false);
      v.sort(w, c, tw, (n + v.T - 1) / v.T, s);
    }
    const uint32_t mtiles = (n + v.P - 1) / v.P;
    for (uint32_t l = 0; l < m; ++l) {
      {
        ProfScope p(K_PART0 + c, s, false);
        const uint32_t tiles_per_wg = (kPartNT / 64) * (64 / sw::kPartLanes);
        v.partition(w, c, (int)l, tw, (mtiles + tiles_per_wg - 1) / tiles_per_wg, s);
      }
      ProfScope p(K_MERGE0 + c, s, false);
      v.merge(w, c, (int)l, tw, mtiles, s);
    }
  }
  HIP_TRY(hipGetLastError());
  return read_status(workspace, s);
}

int sort_words_unbucketed(const uint8_t* chars, const uint32_t* offsets, uint32_t n, uint32_t* out_perm,
                          uint32_t* out_bucket_offsets, void* workspace, size_t workspace_bytes, void* stream) {
  if (!offsets || !out_bucket_offsets || !workspace || (n && !out_perm))
    return fail(SW_ERR_INVALID_ARG, "sort_words_unbucketed: null pointer argument");
  Layout L;
  if (!make_layout(capacity_for(workspace_bytes, 1), 1, L) || L.total > workspace_bytes || n > L.Nmax)
    return fail(SW_ERR_WORKSPACE, "sort_words_unbucketed: workspace too small for %u words", n);
  hipStream_t s = (hipStream_t)stream;
  const sw_config cfg = current_config();
  const Ws w = make_ws(workspace, L, cfg);
  Grids g;
  int rc = make_grids(w, cfg, g);
  if (rc) return rc;
  DevInfo* di;
  if ((rc = device_info(&di))) return rc;
  RunDesc d{chars, offsets, nullptr, out_perm, out_bucket_offsets, n, 1};
  if ((rc = enqueue_begin(w, d, s))) return rc;
  // the pre-pass of the bucketed sort: validation, length counts, bucket offsets
  sw::k_doc_plan<1024><<<1, 1024, 0, s>>>(w);
  sw::k_hist<kNT><<<g.words, kNT, 0, s>>>(w);
  sw::k_scan_rows<1024, 4><<<sw::kNB, 1024, 0, s>>>(w, w.cnt, sw::kNB, w.Bmax + 1, 0);
  sw::k_segments<kNT><<<g.docs, kNT, 0, s>>>(w);
  if (n) {
    const unsigned pgrid = (unsigned)std::min<uint64_t>((n + kNT - 1) / kNT, (uint64_t)di->cus * 8);
    sw::k_pack_full<kNT><<<pgrid, kNT, 0, s>>>(w);
    // one segment of n four-lane keys: chunk sort, then every merge level
    constexpr int c = sw::kNClass - 1;
    const Variant& v = *g.var[c];
    const uint32_t m = sw::levels_for(n, v.T);
    const TileWork tw{1, 0, n, m};
    v.sort(w, c, tw, (n + v.T - 1) / v.T, s);
    const uint32_t mtiles = (n + v.P - 1) / v.P;
    const uint32_t tiles_per_wg = (kPartNT / 64) * (64 / sw::kPartLanes);
    for (uint32_t l = 0; l < m; ++l) {
      v.partition(w, c, (int)l, tw, (mtiles + tiles_per_wg - 1) / tiles_per_wg, s);
      v.merge(w, c, (int)l, tw, std::min<uint32_t>(mtiles, (uint32_t)(di->cus * di->occ_merge[c][cfg.variant[c]])), s);
    }
  }
  HIP_TRY(hipGetLastError());
  return SW_OK;
}

// ------------------------------------------------------------------ plans
struct sw_plan {
  void* ws = nullptr;
  Layout L;
  Ws w;
  Grids g;
  hipStream_t s = nullptr;
  bool own_stream = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  Fork fork;
};

static void plan_free(sw_plan* p) {
  if (!p) return;
  if (p->s) (void)hipStreamSynchronize(p->s);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  fork_free(p->fork);
  if (p->ws) (void)hipFree(p->ws);
  if (p->own_stream && p->s) (void)hipStreamDestroy(p->s);
  delete p;
}

int sw_plan_create(uint32_t max_words, uint32_t max_docs, void* stream, sw_plan** out) {
  if (!out) return fail(SW_ERR_INVALID_ARG, "sw_plan_create: null out");
  *out = nullptr;
  sw_plan* p = new sw_plan();
  if (!make_layout(max_words, max_docs, p->L)) {
    delete p;
    return fail(SW_ERR_INVALID_ARG, "sw_plan_create: sizes out of range");
  }
  if (stream) {
    p->s = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&p->s, hipStreamNonBlocking) != hipSuccess) {
      delete p;
      return fail(SW_ERR_HIP, "sw_plan_create: cannot create a stream");
    }
    p->own_stream = true;
  }
  if (hipMalloc(&p->ws, p->L.total) != hipSuccess) {
    (void)hipGetLastError();
    p->ws = nullptr;
    plan_free(p);
    return fail(SW_ERR_OOM, "sw_plan_create: cannot allocate %zu bytes", p->L.total);
  }
  const sw_config cfg = current_config();
  p->w = make_ws(p->ws, p->L, cfg);
  int rc = make_grids(p->w, cfg, p->g);
  if (rc) {
    plan_free(p);
    return rc;
  }
  if ((rc = fork_init(p->fork))) {
    plan_free(p);
    return rc;
  }
  if (hipStreamBeginCapture(p->s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    plan_free(p);
    return fail(SW_ERR_HIP, "sw_plan_create: stream capture failed to begin");
  }
  rc = enqueue_body(p->w, p->g, p->s, true, false, &p->fork);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(p->s, &graph);
  p->graph = graph;
  if (rc || ec != hipSuccess || !graph) {
    plan_free(p);
    return rc ? rc : fail(SW_ERR_HIP, "sw_plan_create: capture failed: %s", hipGetErrorString(ec));
  }
  if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) {
    p->exec = nullptr;
    plan_free(p);
    return fail(SW_ERR_HIP, "sw_plan_create: graph instantiation failed");
  }
  *out = p;
  return SW_OK;
}

int sw_plan_run(sw_plan* p, const uint8_t* chars, const uint32_t* offsets, const uint32_t* doc_offsets,
                uint32_t n_docs, uint32_t n_words, uint32_t* out_perm, uint32_t* out_bucket_offsets) {
  if (!p || !offsets || !out_bucket_offsets) return fail(SW_ERR_INVALID_ARG, "sw_plan_run: null argument");
  if (doc_offsets) {
    if (n_docs > p->L.Dmax) return fail(SW_ERR_WORKSPACE, "sw_plan_run: %u documents, plan holds %llu", n_docs,
                                        (unsigned long long)p->L.Dmax);
    if (!out_perm) return fail(SW_ERR_INVALID_ARG, "sw_plan_run: null out_perm");
  } else {
    if (n_words > p->L.Nmax)
      return fail(SW_ERR_WORKSPACE, "sw_plan_run: %u words, plan holds %llu", n_words,
                  (unsigned long long)p->L.Nmax);
    if (n_words && !out_perm) return fail(SW_ERR_INVALID_ARG, "sw_plan_run: null out_perm");
  }
  RunDesc d{chars, offsets, doc_offsets, out_perm, out_bucket_offsets, n_words, doc_offsets ? n_docs : 1u};
  int rc = enqueue_begin(p->w, d, p->s);
  if (rc) return rc;
  HIP_TRY(hipGraphLaunch(p->exec, p->s));
  return SW_OK;
}

int sw_plan_status_async(sw_plan* p, uint32_t* status_dst) {
  if (!p || !status_dst) return fail(SW_ERR_INVALID_ARG, "sw_plan_status_async: null argument");
  HIP_TRY(hipMemcpyAsync(status_dst, &((const Header*)p->ws)->status, sizeof(uint32_t), hipMemcpyDefault, p->s));
  return SW_OK;
}

int sw_plan_status(sw_plan* p) {
  if (!p) return fail(SW_ERR_INVALID_ARG, "sw_plan_status: null plan");
  return read_status(p->ws, p->s);
}

void sw_plan_destroy(sw_plan* p) { plan_free(p); }

// ------------------------------------------------------------------ config
int sw_get_config(sw_config* out) {
  if (!out) return fail(SW_ERR_INVALID_ARG, "sw_get_config: null");
  *out = current_config();
  return SW_OK;
}

int sw_set_config(const sw_config* cfg) {
  if (!cfg) return fail(SW_ERR_INVALID_ARG, "sw_set_config: null");
  for (int c = 0; c < sw::kNClass; ++c) {
    const uint32_t C = cfg->chunk[c];
    if (C < 2 || C > 1024 || (C & (C - 1)))
      return fail(SW_ERR_INVALID_ARG, "sw_set_config: chunk[%d]=%u is not a power of two in [2,1024]", c, C);
    int nv;
    variants(c, &nv);
    if (cfg->variant[c] >= (uint32_t)nv)
      return fail(SW_ERR_INVALID_ARG, "sw_set_config: variant[%d]=%u out of range", c, cfg->variant[c]);
  }
  if (cfg->flags & ~SW_FLAG_SERIAL_CLASSES) return fail(SW_ERR_INVALID_ARG, "sw_set_config: unknown flags");
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  g_cfg = *cfg;
  return SW_OK;
}

int sw_num_variants(int cls) {
  if (cls < 0 || cls >= sw::kNClass) return 0;
  int nv;
  variants(cls, &nv);
  return nv;
}

int sw_variant_tiles(int cls, int variant, uint32_t* sort_tile, uint32_t* merge_tile) {
  if (cls < 0 || cls >= sw::kNClass || variant < 0 || variant >= sw_num_variants(cls))
    return fail(SW_ERR_INVALID_ARG, "sw_variant_tiles: out of range");
  int nv;
  const Variant& v = variants(cls, &nv)[variant];
  if (sort_tile) *sort_tile = v.T;
  if (merge_tile) *merge_tile = v.P;
  return SW_OK;
}

// ------------------------------------------------------------------ profiling
int sw_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return SW_OK;
}

int sw_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_prof_recs) {
    g_prof_pool.push_back(r.e0);
    g_prof_pool.push_back(r.e1);
  }
  g_prof_recs.clear();
  for (int k = 0; k < K_COUNT; ++k) {
    g_prof_ms[k] = 0;
    g_prof_n[k] = 0;
  }
  return SW_OK;
}

int sw_profile_read(int max_entries, const char** names, uint32_t* launches, double* ms) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_prof_recs) {
    HIP_TRY(hipEventSynchronize(r.e1));
    float t = 0;
    HIP_TRY(hipEventElapsedTime(&t, r.e0, r.e1));
    g_prof_ms[r.kid] += t;
    g_prof_n[r.kid] += 1;
    g_prof_pool.push_back(r.e0);
    g_prof_pool.push_back(r.e1);
  }
  g_prof_recs.clear();
  int n = 0;
  for (int k = 0; k < K_COUNT && n < max_entries; ++k, ++n) {
    if (names) names[n] = kKernelNames[k];
    if (launches) launches[n] = g_prof_n[k];
    if (ms) ms[n] = g_prof_ms[k];
  }
  return n;
}

// ------------------------------------------------------------------ around the sort
static uint64_t tok_blocks(uint64_t n_bytes) { return (n_bytes + sw::kTokBlock - 1) / sw::kTokBlock; }
static size_t tok_header_bytes() { return (sizeof(Header) + 255) & ~(size_t)255; }

size_t sort_words_tokenize_workspace_size(uint64_t n_bytes) {
  if (n_bytes >= (1ull << 32)) return 0;
  return tok_header_bytes() + 2 * tok_blocks(n_bytes) * sizeof(uint4) + 256;
}

int sort_words_tokenize(const uint8_t* text, uint64_t n_bytes, uint32_t flags, uint8_t* out_chars,
                        uint32_t* out_offsets, uint32_t max_words, uint32_t* out_n_words, void* workspace,
                        size_t workspace_bytes, void* stream) {
  if (!out_offsets || !out_n_words || !workspace || (n_bytes && (!text || !out_chars)))
    return fail(SW_ERR_INVALID_ARG, "sort_words_tokenize: null pointer argument");
  if (n_bytes >= (1ull << 32)) return fail(SW_ERR_INVALID_ARG, "sort_words_tokenize: text of 2^32 bytes or more");
  if (flags & ~SW_TOK_LOWER) return fail(SW_ERR_INVALID_ARG, "sort_words_tokenize: unknown flags 0x%x", flags);
  if (workspace_bytes < sort_words_tokenize_workspace_size(n_bytes))
    return fail(SW_ERR_WORKSPACE, "sort_words_tokenize: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  Header* h = (Header*)workspace;
  const uint32_t nblk = (uint32_t)tok_blocks(n_bytes);
  uint4* sums = (uint4*)((char*)workspace + tok_header_bytes());
  uint4* pre = sums + nblk;
  sw::k_tok_begin<<<1, 64, 0, s>>>(h);
  if (nblk) sw::k_tok_sum<<<nblk, sw::kTokNT, 0, s>>>(text, n_bytes, sums);
  sw::k_tok_scan<1024><<<1, 1024, 0, s>>>(h, sums, pre, nblk, max_words, out_offsets, out_n_words);
  if (nblk) sw::k_tok_write<<<nblk, sw::kTokNT, 0, s>>>(h, text, n_bytes, pre, flags, out_chars, out_offsets);
  HIP_TRY(hipGetLastError());
  return SW_OK;
}

int sort_words_materialize(const uint8_t* chars, const uint32_t* offsets, const uint32_t* doc_offsets,
                           uint32_t n_docs, uint32_t n_words, const uint32_t* perm, const uint32_t* bucket_offsets,
                           int sep, uint8_t* out_text, uint32_t* out_status, void* stream) {
  if (!offsets || !bucket_offsets || !out_status || (n_words && (!chars || !perm || !out_text)))
    return fail(SW_ERR_INVALID_ARG, "sort_words_materialize: null pointer argument");
  if (sep > 255) return fail(SW_ERR_INVALID_ARG, "sort_words_materialize: separator %d is not a byte", sep);
  if (doc_offsets ? n_docs == 0 : n_docs != 1)
    return fail(SW_ERR_INVALID_ARG, "sort_words_materialize: n_docs must be 1 without doc_offsets, >= 1 with");
  hipStream_t s = (hipStream_t)stream;
  sw::k_mat_begin<<<1, 64, 0, s>>>(out_status);
  if (n_words) {
    DevInfo* d;
    int rc = device_info(&d);
    if (rc) return rc;
    constexpr int NT = 256;
    const unsigned grid =
        (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n_words + NT - 1) / NT, (uint64_t)d->cus * 8));
    sw::k_materialize<NT><<<grid, NT, 0, s>>>(chars, offsets, doc_offsets, n_docs, n_words, perm, bucket_offsets,
                                              sep, out_text, out_status);
  }
  HIP_TRY(hipGetLastError());
  return SW_OK;
}

}  // extern "C"
