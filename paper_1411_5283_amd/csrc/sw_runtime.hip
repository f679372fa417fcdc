// sw_runtime.hip -- host side of the gfx950 word sort: the C ABI declared in
// include/sort_words.h, workspace layout, launch sequence, graph-captured
// plans, the per-bucket-launch form and kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sort_words.h"
#include "sw_kernels.hpp"
#include "sw_text.hpp"
#include "sw_gather.hpp"
#include "sw_sched.hpp"

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
constexpr int kTextNT = 256, kTextIPT = 8, kTextKTB = 12;   // k_keys_text: threads, words per thread, LDS bytes per word

// ------------------------------------------------------------------ variants
// A variant fixes, for one key class, the chunk-sort tile (NTS threads x ES
// items) and the merge tile (NTM threads x EM items).
struct Variant {
  void (*sort)(const Ws&, int, TileWork, unsigned, hipStream_t);
  void (*packed)(const Ws&, int, unsigned, hipStream_t);
  void (*merge)(const Ws&, int, int, TileWork, unsigned, hipStream_t);
  const void* sort_fn;
  const void* merge_fn;
  uint32_t T, P;
  int nts, ntm;
};


template <int NL, int NTS, int ES, int NTM, int EM, int MM = 0, int PE = 8>
struct V {
  static void sort(const Ws& w, int c, TileWork tw, unsigned grid, hipStream_t s) {
    sw::k_sort_tiles<NL, NTS, ES, MM><<<grid, NTS, 0, s>>>(w, c, tw);
  }
  static void packed(const Ws& w, int c, unsigned grid, hipStream_t s) {
    sw::k_sort_packed<NL, PE, 0><<<grid, sw::kPackTile / PE, 0, s>>>(w, c);
  }
  static void merge(const Ws& w, int c, int l, TileWork tw, unsigned grid, hipStream_t s) {
    sw::k_merge<NL, NTM, EM, MM><<<grid, NTM, 0, s>>>(w, c, l, tw);
  }
  static Variant get() {
    static_assert(NTM * EM <= 2 * NTS * ES, "merge tile must divide a pair of sorted tiles");
    static_assert(NTS * ES >= 1024 && sw::kPackTile >= 1024, "a chunk of up to 1024 items fits every tile");
    return Variant{sort, packed, merge, (const void*)sw::k_sort_tiles<NL, NTS, ES, MM>,
                   (const void*)sw::k_merge<NL, NTM, EM, MM>, (uint32_t)(NTS * ES), (uint32_t)(NTM * EM), NTS, NTM};
  }
};

// MM picks the register merge: 0 serial, 1 bitonic; PE is the items per
// thread of the short segments' tiles.  The last variant of every class
// spreads a chunk of 1024 over 512 threads (2 items each, short segments
// too): for the chunk of 1024 the paper's second dataset fixes, where a
// chunk's 1024 phases, not the work, set the time.  For classes 1 and 2 one
// variant keeps variant 1's tiles but sorts the short segments with 4 items
// a thread (twice the waves of 8 for those wider keys: thousands of short
// documents sort faster).
constexpr int kMaxVariants = 8;
const Variant* variants(int c, int* count) {
  static const Variant v0[] = {V<0, 256, 16, 256, 16, 0>::get(), V<0, 256, 8, 256, 8, 0>::get(),
                               V<0, 512, 16, 256, 16, 0>::get(), V<0, 512, 16, 512, 4, 0>::get(),
                               V<0, 512, 16, 256, 16, 1>::get(), V<0, 512, 16, 256, 8, 1>::get(),
                               V<0, 1024, 16, 256, 16, 0>::get(), V<0, 512, 2, 256, 4, 0, 2>::get()};
  static const Variant v1[] = {V<1, 256, 16, 256, 16, 0>::get(), V<1, 256, 8, 256, 8, 0>::get(),
                               V<1, 512, 16, 256, 8, 0>::get(), V<1, 512, 16, 256, 16, 0>::get(),
                               V<1, 512, 16, 256, 8, 1>::get(), V<1, 256, 8, 256, 8, 0, 4>::get(),
                               V<1, 1024, 8, 256, 16, 0>::get(), V<1, 512, 2, 256, 4, 0, 2>::get()};
  static const Variant v2[] = {V<2, 256, 16, 256, 16, 0>::get(), V<2, 256, 8, 256, 8, 0>::get(),
                               V<2, 256, 8, 256, 16, 0>::get(), V<2, 256, 8, 256, 8, 0, 4>::get(),
                               V<2, 512, 8, 256, 8, 1>::get(), V<2, 512, 8, 256, 16, 0>::get(),
                               V<2, 512, 2, 256, 4, 0, 2>::get()};
  static const Variant v3[] = {V<3, 256, 8, 256, 8, 0>::get(), V<3, 128, 16, 128, 16, 0>::get(),
                               V<3, 128, 16, 256, 8, 0>::get(), V<3, 512, 2, 256, 4, 0, 2>::get()};
  static const Variant v4[] = {V<4, 256, 8, 256, 8, 0>::get(), V<4, 128, 16, 128, 16, 0>::get(),
                               V<4, 128, 16, 256, 8, 0>::get(), V<4, 512, 2, 256, 4, 0, 2>::get()};
  static const Variant* all[] = {v0, v1, v2, v3, v4};
  static const int counts[] = {8, 8, 7, 4, 4};
  *count = counts[c];
  return all[c];
}

// Four-way merge configurations of a class (k_merge4w, passes by bounded
// windows): NT threads, E outputs a thread, windows of NT*E/4 items.
struct Merge4 {
  void (*merge)(const Ws&, int, int, TileWork, unsigned, hipStream_t);
  const void* fn;
  int nt;
  uint32_t ps;   // outputs per step at most: four windows
};
template <int NL, int NT, int E>
struct V4W {
  static void merge(const Ws& w, int c, int l, TileWork tw, unsigned grid, hipStream_t s) {
    sw::k_merge4w<NL, NT, E><<<grid, NT, 0, s>>>(w, c, l, tw);
  }
  static Merge4 get() { return Merge4{merge, (const void*)sw::k_merge4w<NL, NT, E>, NT, (uint32_t)(NT * E)}; }
};
constexpr int kMaxMerge4 = 2;
const Merge4* merges4(int c, int* count) {
  static const Merge4 m0[] = {V4W<0, 256, 4>::get(), V4W<0, 256, 2>::get()};
  static const Merge4 m1[] = {V4W<1, 256, 4>::get(), V4W<1, 256, 2>::get()};
  static const Merge4 m2[] = {V4W<2, 256, 4>::get(), V4W<2, 256, 2>::get()};
  static const Merge4 m3[] = {V4W<3, 256, 2>::get()};
  static const Merge4 m4[] = {V4W<4, 256, 2>::get()};
  static const Merge4* all[] = {m0, m1, m2, m3, m4};
  static const int counts[] = {2, 2, 2, 1, 1};
  *count = counts[c];
  return all[c];
}

// ------------------------------------------------------------------ config
std::mutex g_cfg_mu;
sw_config g_cfg = {{16, 16, 16, 16, 16}, {0, 0, 0, 0, 0}, 0, {0, 0, 0, 0, 0}};

sw_config current_config() {
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  return g_cfg;
}

// ------------------------------------------------------------------ device info
struct DevInfo {
  bool ready = false;
  int cus = 0;
  int occ_hist = 1, occ_scatter = 1, occ_text = 1;
  int occ_sort[sw::kNClass][kMaxVariants] = {};
  int occ_merge[sw::kNClass][kMaxVariants] = {};
  int occ_merge4[sw::kNClass][kMaxMerge4] = {};
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
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&d.occ_text, (const void*)sw::k_keys_text<kTextNT, kTextIPT, kTextKTB>,
                                                         kTextNT, 0));
    for (int c = 0; c < sw::kNClass; ++c) {
      int nv;
      const Variant* vs = variants(c, &nv);
      for (int v = 0; v < nv; ++v) {
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&d.occ_sort[c][v], vs[v].sort_fn, vs[v].nts, 0));
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&d.occ_merge[c][v], vs[v].merge_fn, vs[v].ntm, 0));
        d.occ_sort[c][v] = std::max(d.occ_sort[c][v], 1);
        d.occ_merge[c][v] = std::max(d.occ_merge[c][v], 1);
      }
      int nm;
      const Merge4* ms = merges4(c, &nm);
      for (int k = 0; k < nm; ++k) {
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&d.occ_merge4[c][k], ms[k].fn, ms[k].nt, 0));
        d.occ_merge4[c][k] = std::max(d.occ_merge4[c][k], 1);
      }
    }
    d.occ_hist = std::max(d.occ_hist, 1);
    d.occ_scatter = std::max(d.occ_scatter, 1);
    d.occ_text = std::max(d.occ_text, 1);
    d.ready = true;
  }
  *out = &d;
  return SW_OK;
}

// ------------------------------------------------------------------ layout
struct Layout {
  uint64_t Nmax = 0, Dmax = 0, Bmax = 0, Smax = 0, SBmax = 0;
  size_t o_hdr, o_doc_off, o_doc_blk, o_cnt, o_seg_n, o_seg_base, o_segcnt, o_sorted, o_st, o_mt, o_vpre, o_wpre;
  size_t o_a[4], o_ai, o_b[4], o_bi;
  size_t total = 0;
};

bool make_layout(uint64_t Nmax, uint64_t Dmax, Layout& L) {
  if (Dmax == 0) Dmax = 1;
  // at most 2^32 - 2 words: every index then lies below the chunk sort's fill
  // key (index 2^32 - 2) and its sentinel (2^32 - 1)
  if (Nmax > 0xFFFFFFFEull || Dmax > 0xFFFFFFFFull / sw::kNB) return false;
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
  L.o_wpre = take(4 * (L.Smax + sw::kNClass));
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

Ws make_ws(void* base, const Layout& L, const sw_config& cfg, uint64_t max_chars = ~0ull) {
  char* p = (char*)base;
  Ws w;
  w.Cmax = max_chars;
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
  w.wpre = (uint32_t*)(p + L.o_wpre);
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
    w.fan[c] = cfg.merge[c] ? 4u : 2u;
  }
  return w;
}

// ------------------------------------------------------------------ profiling
enum KernelId {
  K_BEGIN, K_DOC_PLAN, K_HIST, K_SCAN, K_SEGMENTS, K_SEG_COUNT, K_SEG_SCATTER, K_TILE_PREFIX, K_SCATTER,
  K_SORT0, K_SORT1, K_SORT2, K_SORT3, K_SORT4, K_MERGE0, K_MERGE1, K_MERGE2, K_MERGE3, K_MERGE4,
  K_PACK0, K_PACK1, K_PACK2, K_PACK3, K_PACK4, K_KEYS_TEXT, K_COUNT
};
static_assert(K_MERGE0 - K_SORT0 == sw::kNClass && K_PACK0 - K_MERGE0 == sw::kNClass &&
              K_KEYS_TEXT - K_PACK0 == sw::kNClass, "one kernel id per class");
const char* const kKernelNames[K_COUNT] = {
    "begin", "doc_plan", "hist", "scan_rows", "segments", "seg_count", "seg_scatter", "tile_prefix",
    "scatter_pack", "sort_tiles_c0", "sort_tiles_c1", "sort_tiles_c2", "sort_tiles_c3", "sort_tiles_c4",
    "merge_c0", "merge_c1", "merge_c2", "merge_c3", "merge_c4",
    "sort_packed_c0", "sort_packed_c1", "sort_packed_c2", "sort_packed_c3", "sort_packed_c4", "keys_text"};

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
  unsigned sort[sw::kNClass], merge[sw::kNClass], packed, text;
  int passes[sw::kNClass];             // HBM merge passes of the longest possible segment
  const Variant* var[sw::kNClass];
  const Merge4* m4[sw::kNClass];       // four-way merge, or null for two-way levels
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
  g.text = clampg(((uint64_t)w.Nmax + kTextNT * kTextIPT - 1) / (kTextNT * kTextIPT), cus * (uint64_t)d->occ_text);
  for (int c = 0; c < sw::kNClass; ++c) {
    int nv;
    const Variant* vs = variants(c, &nv);
    const int v = (int)cfg.variant[c];
    g.var[c] = &vs[v];
    const uint64_t maxtiles_s = (uint64_t)w.Nmax / vs[v].T + w.Smax;
    const uint64_t maxtiles_m = (uint64_t)w.Nmax / vs[v].P + w.Smax;
    g.sort[c] = clampg(maxtiles_s, cus * (uint64_t)d->occ_sort[c][v]);
    const int mk = (int)cfg.merge[c];
    g.m4[c] = nullptr;
    if (mk) {
      int nm;
      g.m4[c] = &merges4(c, &nm)[mk - 1];
      g.merge[c] = clampg(((uint64_t)w.Nmax + 4095) / 4096, cus * (uint64_t)d->occ_merge4[c][mk - 1]);
    } else {
      g.merge[c] = clampg(maxtiles_m, cus * (uint64_t)d->occ_merge[c][v]);
    }
    g.passes[c] = (int)sw::merge_passes(w.Nmax, vs[v].T, mk ? 4u : 2u);
  }
  return SW_OK;
}

// The k-th order of the five classes in lexicographic order (k < 120): the
// factorial number system picks each position's class among those left.
constexpr uint32_t kNOrders = 120;   // kNClass!
void class_order(uint32_t k, int (&order)[sw::kNClass]) {
  static_assert(sw::kNClass == 5, "120 orders of five classes");
  int left[sw::kNClass];
  for (int c = 0; c < sw::kNClass; ++c) left[c] = c;
  int n = sw::kNClass;
  uint32_t f = 24;   // (kNClass - 1)!
  for (int i = 0; i < sw::kNClass; ++i) {
    const int j = (int)(k / f);
    order[i] = left[j];
    for (int t = j; t + 1 < n; ++t) left[t] = left[t + 1];
    --n;
    k %= f;
    if (n > 0) f /= (uint32_t)n;
  }
}

// Side streams and events for running the key classes concurrently: after
// the scatter the classes share nothing, so each class's chain (chunk sort,
// then one merge per level) goes on a stream of its own, forked from and
// joined back into the caller's stream; under graph capture the chains become
// parallel branches of the graph.  The two long classes (17-24 and 25-32
// bytes, the fewest words in text) share one stream, so that the chains fit
// the four hardware queues a process gets by default: a fifth stream would
// share a queue with another class and serialize behind it.
constexpr int kNStreams = 4;
inline int stream_of_class(int c) { return c < kNStreams ? c : kNStreams - 1; }
struct Fork {
  hipStream_t side[kNStreams] = {};   // side[0] unused: class 0 stays on the main stream
  hipEvent_t fork = nullptr;
  hipEvent_t join[kNStreams] = {};
  hipEvent_t seg_fork = nullptr, seg_join = nullptr;
  bool ready = false;
};

int fork_init(Fork& f) {
  if (f.ready) return SW_OK;
  for (int c = 1; c < kNStreams; ++c) HIP_TRY(hipStreamCreateWithFlags(&f.side[c], hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&f.fork, hipEventDisableTiming));
  for (int c = 1; c < kNStreams; ++c) HIP_TRY(hipEventCreateWithFlags(&f.join[c], hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&f.seg_fork, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&f.seg_join, hipEventDisableTiming));
  f.ready = true;
  return SW_OK;
}

void fork_free(Fork& f) {
  if (!f.ready) return;
  for (int c = 1; c < kNStreams; ++c) {
    if (f.side[c]) (void)hipStreamSynchronize(f.side[c]);
  }
  for (int c = 1; c < kNStreams; ++c) {
    if (f.side[c]) (void)hipStreamDestroy(f.side[c]);
    if (f.join[c]) (void)hipEventDestroy(f.join[c]);
  }
  if (f.fork) (void)hipEventDestroy(f.fork);
  if (f.seg_fork) (void)hipEventDestroy(f.seg_fork);
  if (f.seg_join) (void)hipEventDestroy(f.seg_join);
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
// With `text` the sorted text is written from the sorted keys at the end.
int enqueue_body(const Ws& w, const Grids& g, hipStream_t s, bool capture, bool through_scatter,
                 Fork* fork = nullptr, bool text = false) {
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
  const bool par = !through_scatter && fork && fork->ready && !(!capture && profiling_on()) &&
                   !(g.flags & SW_FLAG_SERIAL_CLASSES);
  // the segment scheduling reads only the segment table, so it may run
  // beside the scatter (on class 1's side stream, joined before the classes fork)
  const bool beside = par && (g.flags & SW_FLAG_SCHEDULE_BESIDE_SCATTER);
  if (!through_scatter) {
    hipStream_t ss = s;
    if (beside) {
      ss = fork->side[1];
      HIP_TRY(hipEventRecord(fork->seg_fork, s));
      HIP_TRY(hipStreamWaitEvent(ss, fork->seg_fork, 0));
    }
    {
      ProfScope p(K_SEG_COUNT, ss, capture);
      sw::k_seg_count<kNT><<<g.segs, kNT, 0, ss>>>(w);
    }
    {
      ProfScope p(K_SCAN, ss, capture);
      sw::k_scan_rows<1024, 4><<<sw::kNKeys, 1024, 0, ss>>>(w, w.segcnt, sw::kNKeys, w.SBmax + 1, 1);
    }
    {
      ProfScope p(K_SEG_SCATTER, ss, capture);
      sw::k_seg_scatter<kNT><<<g.segs, kNT, 0, ss>>>(w);
    }
    {
      ProfScope p(K_TILE_PREFIX, ss, capture);
      sw::k_tile_prefix<1024><<<4 * sw::kNClass, 1024, 0, ss>>>(w);
    }
    if (beside) HIP_TRY(hipEventRecord(fork->seg_join, ss));
  }
  {
    ProfScope p(K_SCATTER, s, capture);
    sw::k_scatter_pack<kScatterNT><<<g.scatter, kScatterNT, 0, s>>>(w);
  }
  if (through_scatter) return SW_OK;
  if (beside) HIP_TRY(hipStreamWaitEvent(s, fork->seg_join, 0));
  if (par) {
    HIP_TRY(hipEventRecord(fork->fork, s));
    for (int c = 1; c < kNStreams; ++c) HIP_TRY(hipStreamWaitEvent(fork->side[c], fork->fork, 0));
  }
  const TileWork none{0, 0, 0, 0, 0};
  // Each class keeps its own order on its own stream; across classes the work
  // is enqueued stage by stage (all chunk sorts, then merge level 0 of every
  // class, level 1, ...), so that a runtime which maps the parallel chains
  // onto fewer hardware queues still finds every class's next kernel early.
  auto cstream = [&](int c) { return (par && c > 0) ? fork->side[stream_of_class(c)] : s; };
  int order[sw::kNClass];
  class_order((g.flags & SW_FLAG_ORDER_MASK) >> SW_FLAG_ORDER_SHIFT, order);
  int max_levels = 0;
  for (int k = 0; k < sw::kNClass; ++k) {
    const int c = order[k];
    hipStream_t cs = cstream(c);
    // the short segments are disjoint from the chunk-sorted ones, so the two
    // kernels may go in either order (which is faster depends on the workload)
    const bool packed_first = (g.flags & SW_FLAG_PACKED_FIRST) != 0;
    for (int step = 0; step < 2; ++step) {
      if ((step == 0) == packed_first) {
        ProfScope p(K_PACK0 + c, cs, capture);
        g.var[c]->packed(w, c, g.packed, cs);
      } else {
        ProfScope p(K_SORT0 + c, cs, capture);
        g.var[c]->sort(w, c, none, g.sort[c], cs);
      }
    }
    max_levels = std::max(max_levels, g.passes[c]);
  }
  for (int l = 0; l < max_levels; ++l) {
    for (int k = 0; k < sw::kNClass; ++k) {
      const int c = order[k];
      if (l >= g.passes[c]) continue;
      hipStream_t cs = cstream(c);
      ProfScope p(K_MERGE0 + c, cs, capture);
      if (g.m4[c])
        g.m4[c]->merge(w, c, l, none, g.merge[c], cs);
      else
        g.var[c]->merge(w, c, l, none, g.merge[c], cs);
    }
  }
  if (par) {
    for (int c = 1; c < kNStreams; ++c) {
      HIP_TRY(hipEventRecord(fork->join[c], fork->side[c]));
      HIP_TRY(hipStreamWaitEvent(s, fork->join[c], 0));
    }
  }
  if (text) {
    ProfScope p(K_KEYS_TEXT, s, capture);
    sw::k_keys_text<kTextNT, kTextIPT, kTextKTB><<<g.text, kTextNT, 0, s>>>(w);
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

// Workspace of sort_words_noalloc: a fixed array in device memory, one copy
// per GPU, held until the process ends.  Host code never uses its name as an
// address (on the host the name is only a stand-in): the device address comes
// from hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) uint8_t scratch[SW_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[64];

int scratch_address(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(SW_ERR_HIP, "device id %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SW_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SW_OK;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

const char* sort_words_last_error(void) { return g_err.c_str(); }
const char* sort_words_version(void) { return "sortwords-gfx950 0.8"; }

size_t sort_words_workspace_size(uint32_t max_words, uint32_t max_docs) {
  Layout L;
  if (!make_layout(max_words, max_docs, L)) return 0;
  return L.total;
}

// Device offset arrays are read with 16-byte loads from the 16-byte aligned
// address below them, which assumes a 4-byte aligned start (as any uint32_t
// array has); a misaligned one is rejected rather than read shifted.
bool misaligned(const void* p) { return ((uintptr_t)p & 3) != 0; }

int sort_words_noalloc(const uint8_t* chars, const uint32_t* offsets, uint32_t n, uint32_t* out_perm,
                       uint32_t* out_bucket_offsets, uint32_t* out_status, void* stream) {
  if (!offsets || !out_bucket_offsets || !out_status || (n && !out_perm))
    return fail(SW_ERR_INVALID_ARG, "sort_words_noalloc: null pointer argument");
  if (misaligned(offsets))
    return fail(SW_ERR_INVALID_ARG, "sort_words_noalloc: offsets not 4-byte aligned");
  Layout L;
  if (!make_layout(n, 1, L)) return fail(SW_ERR_INVALID_ARG, "sort_words_noalloc: n out of range");
  if (L.total > SW_NOALLOC_SCRATCH_BYTES)
    return fail(SW_ERR_WORKSPACE, "sort_words_noalloc: %u words need %zu bytes of workspace; the scratch holds %u "
                "(at most %llu words)", n, L.total, (unsigned)SW_NOALLOC_SCRATCH_BYTES,
                (unsigned long long)capacity_for(SW_NOALLOC_SCRATCH_BYTES, 1));
  void* ws = nullptr;
  int rc = scratch_address(&ws);
  if (rc) return rc;
  const sw_config cfg = current_config();
  const Ws w = make_ws(ws, L, cfg);
  Grids g;
  if ((rc = make_grids(w, cfg, g))) return rc;
  hipStream_t s = (hipStream_t)stream;
  const RunDesc d{chars, offsets, nullptr, out_perm, out_bucket_offsets, n, 1};
  sw::k_begin<<<1, 64, 0, s>>>(w, d);
  // every kernel on the caller's stream, in order (no side streams, no events,
  // no timing), so the call may also be captured into a graph
  if ((rc = enqueue_body(w, g, s, true, false, nullptr))) return rc;
  sw::k_status_out<<<1, 64, 0, s>>>(w, out_status);
  HIP_TRY(hipGetLastError());
  return SW_OK;
}

int sort_words_ex(const uint8_t* chars, const uint32_t* offsets, uint32_t n, uint32_t* out_perm,
                  uint32_t* out_bucket_offsets, void* workspace, size_t workspace_bytes, void* stream) {
  if (!offsets || !out_bucket_offsets || (n && !out_perm) || !workspace)
    return fail(SW_ERR_INVALID_ARG, "sort_words_ex: null pointer argument");
  if (misaligned(offsets))
    return fail(SW_ERR_INVALID_ARG, "sort_words_ex: offsets not 4-byte aligned");
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
  if (misaligned(offsets))
    return fail(SW_ERR_INVALID_ARG, "sort_words: offsets not 4-byte aligned");
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
  if (misaligned(offsets) || misaligned(doc_offsets))
    return fail(SW_ERR_INVALID_ARG, "sort_words_batch: offsets not 4-byte aligned");
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
  if (misaligned(offsets) || misaligned(doc_offsets))
    return fail(SW_ERR_INVALID_ARG, "sort_words_plain: offsets not 4-byte aligned");
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
    const uint32_t m = sw::merge_passes(n, v.T, g.m4[c] ? 4u : 2u);
    const TileWork tw{1, seg_base[sidx], n, m, 0};
    {
      ProfScope p(K_SORT0 + c, s, false);
      v.sort(w, c, tw, (n + v.T - 1) / v.T, s);
    }
    for (uint32_t l = 0; l < m; ++l) {
      ProfScope p(K_MERGE0 + c, s, false);
      if (g.m4[c])
        g.m4[c]->merge(w, c, (int)l, tw, std::min<unsigned>((n + 4095) / 4096, g.merge[c]), s);
      else
        v.merge(w, c, (int)l, tw, (n + v.P - 1) / v.P, s);
    }
  }
  HIP_TRY(hipGetLastError());
  return read_status(workspace, s);
}

int sort_words_chunks(const uint8_t* chars, const uint32_t* offsets, uint32_t n, uint32_t chunk,
                      uint32_t* out_perm, uint32_t* out_bucket_offsets, void* workspace, size_t workspace_bytes,
                      void* stream) {
  if (!offsets || !out_bucket_offsets || !workspace || (n && !out_perm))
    return fail(SW_ERR_INVALID_ARG, "sort_words_chunks: null pointer argument");
  if (misaligned(offsets))
    return fail(SW_ERR_INVALID_ARG, "sort_words_chunks: offsets not 4-byte aligned");
  if (chunk < 2 || chunk > 1024 || (chunk & (chunk - 1)))
    return fail(SW_ERR_INVALID_ARG, "sort_words_chunks: chunk %u is not a power of two in [2,1024]", chunk);
  Layout L;
  if (!make_layout(n, 1, L)) return fail(SW_ERR_INVALID_ARG, "sort_words_chunks: n out of range");
  if (L.total > workspace_bytes)
    return fail(SW_ERR_WORKSPACE, "sort_words_chunks: workspace of %zu bytes, need %zu", workspace_bytes, L.total);
  hipStream_t s = (hipStream_t)stream;
  sw_config cfg = current_config();
  for (int c = 0; c < sw::kNClass; ++c) cfg.chunk[c] = chunk;
  const Ws w = make_ws(workspace, L, cfg);
  Grids g;
  int rc = make_grids(w, cfg, g);
  if (rc) return rc;
  RunDesc d{chars, offsets, nullptr, out_perm, out_bucket_offsets, n, 1};
  if ((rc = enqueue_begin(w, d, s))) return rc;
  if ((rc = enqueue_body(w, g, s, false, true))) return rc;
  if ((rc = read_status(workspace, s))) return rc;
  std::vector<uint32_t> seg_n(sw::kNB), seg_base(sw::kNB);
  HIP_TRY(hipMemcpy(seg_n.data(), w.seg_n, 4 * sw::kNB, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(seg_base.data(), w.seg_base, 4 * sw::kNB, hipMemcpyDeviceToHost));
  for (int len = 0; len < sw::kNB; ++len) {
    const uint32_t m = seg_n[len];
    if (!m) continue;
    const int c = sw::class_of_len((uint32_t)len);
    const Variant& v = *g.var[c];
    const TileWork tw{1, seg_base[len], m, 0, 1};
    v.sort(w, c, tw, (m + v.T - 1) / v.T, s);
  }
  HIP_TRY(hipGetLastError());
  return read_status(workspace, s);
}

int sort_words_unbucketed(const uint8_t* chars, const uint32_t* offsets, uint32_t n, uint32_t* out_perm,
                          uint32_t* out_bucket_offsets, void* workspace, size_t workspace_bytes, void* stream) {
  if (!offsets || !out_bucket_offsets || !workspace || (n && !out_perm))
    return fail(SW_ERR_INVALID_ARG, "sort_words_unbucketed: null pointer argument");
  if (misaligned(offsets))
    return fail(SW_ERR_INVALID_ARG, "sort_words_unbucketed: offsets not 4-byte aligned");
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
    const uint32_t m = sw::merge_passes(n, v.T, g.m4[c] ? 4u : 2u);
    const TileWork tw{1, 0, n, m, 0};
    v.sort(w, c, tw, (n + v.T - 1) / v.T, s);
    const uint32_t mtiles = (n + v.P - 1) / v.P;
    for (uint32_t l = 0; l < m; ++l) {
      if (g.m4[c])
        g.m4[c]->merge(w, c, (int)l, tw, std::min<unsigned>((n + 4095) / 4096, g.merge[c]), s);
      else
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
  hipGraph_t graph_text = nullptr;     // the same pass plus the sorted text, captured on first use
  hipGraphExec_t exec_text = nullptr;
  Fork fork;
};

static void plan_free(sw_plan* p) {
  if (!p) return;
  if (p->s) (void)hipStreamSynchronize(p->s);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->exec_text) (void)hipGraphExecDestroy(p->exec_text);
  if (p->graph_text) (void)hipGraphDestroy(p->graph_text);
  fork_free(p->fork);
  if (p->ws) (void)hipFree(p->ws);
  if (p->own_stream && p->s) (void)hipStreamDestroy(p->s);
  delete p;
}

// Captures the whole pass (with the sorted text or without) into a graph on
// the plan's stream.
static int plan_capture(sw_plan* p, bool text, hipGraph_t* graph_out, hipGraphExec_t* exec_out) {
  if (hipStreamBeginCapture(p->s, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return fail(SW_ERR_HIP, "sw_plan: stream capture failed to begin");
  const int rc = enqueue_body(p->w, p->g, p->s, true, false, &p->fork, text);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(p->s, &graph);
  if (rc || ec != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc ? rc : fail(SW_ERR_HIP, "sw_plan: capture failed: %s", hipGetErrorString(ec));
  }
  hipGraphExec_t exec = nullptr;
  if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(SW_ERR_HIP, "sw_plan: graph instantiation failed");
  }
  *graph_out = graph;
  *exec_out = exec;
  return SW_OK;
}

int sw_plan_create(uint32_t max_words, uint32_t max_docs, uint64_t max_chars, void* stream, sw_plan** out) {
  if (!out) return fail(SW_ERR_INVALID_ARG, "sw_plan_create: null out");
  *out = nullptr;
  if (max_chars >= (1ull << 32)) return fail(SW_ERR_INVALID_ARG, "sw_plan_create: max_chars must be below 2^32");
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
  p->w = make_ws(p->ws, p->L, cfg, max_chars);
  int rc = make_grids(p->w, cfg, p->g);
  if (!rc) rc = fork_init(p->fork);
  if (!rc) rc = plan_capture(p, false, &p->graph, &p->exec);
  if (rc) {
    plan_free(p);
    return rc;
  }
  *out = p;
  return SW_OK;
}

static int plan_check(const sw_plan* p, const char* what, const uint32_t* offsets, const uint32_t* doc_offsets,
                      uint32_t n_docs, uint32_t n_words, const uint32_t* out_perm,
                      const uint32_t* out_bucket_offsets) {
  if (!p || !offsets || !out_bucket_offsets) return fail(SW_ERR_INVALID_ARG, "%s: null argument", what);
  if (misaligned(offsets) || misaligned(doc_offsets))
    return fail(SW_ERR_INVALID_ARG, "%s: offsets not 4-byte aligned", what);
  if (doc_offsets) {
    if (n_docs > p->L.Dmax)
      return fail(SW_ERR_WORKSPACE, "%s: %u documents, plan holds %llu", what, n_docs, (unsigned long long)p->L.Dmax);
    if (!out_perm) return fail(SW_ERR_INVALID_ARG, "%s: null out_perm", what);
  } else {
    if (n_words > p->L.Nmax)
      return fail(SW_ERR_WORKSPACE, "%s: %u words, plan holds %llu", what, n_words, (unsigned long long)p->L.Nmax);
    if (n_words && !out_perm) return fail(SW_ERR_INVALID_ARG, "%s: null out_perm", what);
  }
  return SW_OK;
}

int sw_plan_run(sw_plan* p, const uint8_t* chars, const uint32_t* offsets, const uint32_t* doc_offsets,
                uint32_t n_docs, uint32_t n_words, uint32_t* out_perm, uint32_t* out_bucket_offsets) {
  int rc = plan_check(p, "sw_plan_run", offsets, doc_offsets, n_docs, n_words, out_perm, out_bucket_offsets);
  if (rc) return rc;
  RunDesc d{chars, offsets, doc_offsets, out_perm, out_bucket_offsets, n_words, doc_offsets ? n_docs : 1u};
  if ((rc = enqueue_begin(p->w, d, p->s))) return rc;
  HIP_TRY(hipGraphLaunch(p->exec, p->s));
  return SW_OK;
}

int sw_plan_run_text(sw_plan* p, const uint8_t* chars, const uint32_t* offsets, const uint32_t* doc_offsets,
                     uint32_t n_docs, uint32_t n_words, uint32_t* out_perm, uint32_t* out_bucket_offsets, int sep,
                     uint8_t* out_text) {
  int rc = plan_check(p, "sw_plan_run_text", offsets, doc_offsets, n_docs, n_words, out_perm, out_bucket_offsets);
  if (rc) return rc;
  if (!out_text) return fail(SW_ERR_INVALID_ARG, "sw_plan_run_text: null out_text");
  if (sep > 255) return fail(SW_ERR_INVALID_ARG, "sw_plan_run_text: separator %d is not a byte", sep);
  if (!p->exec_text && (rc = plan_capture(p, true, &p->graph_text, &p->exec_text))) return rc;
  RunDesc d{chars, offsets, doc_offsets, out_perm, out_bucket_offsets, n_words, doc_offsets ? n_docs : 1u,
            out_text, sep < 0 ? -1 : sep};
  if ((rc = enqueue_begin(p->w, d, p->s))) return rc;
  HIP_TRY(hipGraphLaunch(p->exec_text, p->s));
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
    int nm;
    merges4(c, &nm);
    if (cfg->merge[c] > (uint32_t)nm)
      return fail(SW_ERR_INVALID_ARG, "sw_set_config: merge[%d]=%u out of range", c, cfg->merge[c]);
  }
  if (cfg->flags &
      ~(SW_FLAG_SERIAL_CLASSES | SW_FLAG_PACKED_FIRST | SW_FLAG_SCHEDULE_BESIDE_SCATTER | SW_FLAG_ORDER_MASK))
    return fail(SW_ERR_INVALID_ARG, "sw_set_config: unknown flags");
  if (((cfg->flags & SW_FLAG_ORDER_MASK) >> SW_FLAG_ORDER_SHIFT) >= kNOrders)
    return fail(SW_ERR_INVALID_ARG, "sw_set_config: class order index %u is not below 120",
                (cfg->flags & SW_FLAG_ORDER_MASK) >> SW_FLAG_ORDER_SHIFT);
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

int sw_num_merges(int cls) {
  if (cls < 0 || cls >= sw::kNClass) return 0;
  int nm;
  merges4(cls, &nm);
  return nm + 1;
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
  if (misaligned(offsets) || misaligned(doc_offsets))
    return fail(SW_ERR_INVALID_ARG, "sort_words_materialize: offsets not 4-byte aligned");
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

// ------------------------------------------------------------------ serving
// The serving loop (continuous batching): the scheduling rules are in
// sw_sched.hpp; here are the GPU executor (a device pool of the budget's
// size that holds every admitted request, upload threads that copy each
// request into its block as soon as it is admitted, and per slot a stream, a
// graph-captured plan and the batch's buffers, packed on the device), the
// host threads that copy results out, and the scheduler thread.
namespace {

// A few host threads for the copies of a batch; the calling thread takes the
// first part.
class CopyPool {
 public:
  explicit CopyPool(unsigned n) {
    for (unsigned i = 0; i < n; ++i) th_.emplace_back([this] { loop(); });
  }
  ~CopyPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  unsigned threads() const { return (unsigned)th_.size() + 1; }
  // fn(part) for part = 0..parts-1, spread over the pool and the caller
  void run(unsigned parts, const std::function<void(unsigned)>& fn) {
    if (parts <= 1 || th_.empty()) {
      for (unsigned i = 0; i < parts; ++i) fn(i);
      return;
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      fn_ = &fn;
      next_ = 1;
      parts_ = parts;
      left_ = parts - 1;
      ++gen_;
    }
    cv_.notify_all();
    fn(0);
    std::unique_lock<std::mutex> lk(mu_);
    done_cv_.wait(lk, [this] { return left_ == 0; });
    fn_ = nullptr;
  }

 private:
  void loop() {
    uint64_t seen = 0;
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      cv_.wait(lk, [&] { return stop_ || (gen_ != seen && next_ < parts_); });
      if (stop_) return;
      seen = gen_;
      while (next_ < parts_) {
        const unsigned part = next_++;
        const std::function<void(unsigned)>* f = fn_;
        lk.unlock();
        (*f)(part);
        lk.lock();
        if (--left_ == 0) done_cv_.notify_all();
      }
    }
  }
  std::vector<std::thread> th_;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(unsigned)>* fn_ = nullptr;
  unsigned next_ = 0, parts_ = 0, left_ = 0;
  uint64_t gen_ = 0;
  bool stop_ = false;
};

// Upload of admitted requests into their device blocks: worker threads copy
// requests through two pinned staging buffers of their own and issue the
// device copies on one upload stream, in one order for all workers (so the
// upload event of the latest request of a batch covers the whole batch).
// Requests admitted one after another usually get neighbouring blocks (the
// pool hands out the lowest free block), so a worker takes as many queued
// requests as lie back to back in device memory and fit its staging buffer,
// lays them out there as in the pool, and moves them with one copy: a copy
// has a fixed cost of its own that per-request copies of small requests
// would pay thousands of times.  A request larger than the staging buffer
// goes alone, in pieces.  A request's upload event is its staging buffer's;
// the buffer's next use records it again, later on the same stream, so a
// wait on it may wait longer but never too little.
class Uploader {
 public:
  static constexpr uint64_t kStage = 4u << 20;
  // host-to-device copies go out on this many streams (worker i on stream
  // i % kStreams), so that several copy engines can carry them
  static constexpr int kStreams = 4;

  int init(unsigned workers, uint8_t* base, std::function<void()> notify) {
    base_ = base;
    notify_ = std::move(notify);
    for (int k = 0; k < kStreams; ++k)
      if (hipStreamCreateWithFlags(&s_[k], hipStreamNonBlocking) != hipSuccess) return SW_ERR_HIP;
    stage_.resize(std::max(1u, workers));
    for (size_t i = 0; i < stage_.size(); ++i) {
      Stage& st = stage_[i];
      st.stream = (int)(i % kStreams);
      for (int b = 0; b < 2; ++b) {
        if (hipHostMalloc(&st.buf[b], kStage, 0) != hipSuccess) return SW_ERR_OOM;
        if (hipEventCreateWithFlags(&st.ev[b], hipEventDisableTiming) != hipSuccess) return SW_ERR_HIP;
      }
    }
    for (Stage& st : stage_) th_.emplace_back([this, &st] { loop(st); });
    return SW_OK;
  }
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
    th_.clear();
    for (int k = 0; k < kStreams; ++k)
      if (s_[k]) (void)hipStreamSynchronize(s_[k]);
  }
  void free_all() {
    for (Stage& st : stage_)
      for (int b = 0; b < 2; ++b) {
        if (st.buf[b]) (void)hipHostFree(st.buf[b]);
        if (st.ev[b]) (void)hipEventDestroy(st.ev[b]);
      }
    stage_.clear();
    for (int k = 0; k < kStreams; ++k) {
      if (s_[k]) (void)hipStreamDestroy(s_[k]);
      s_[k] = nullptr;
    }
  }
  void push(swsrv::Request* r) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      q_.push_back(r);
    }
    cv_.notify_one();
  }

 private:
  struct Stage {
    uint8_t* buf[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    int next = 0;
    int stream = 0;
  };

  void loop(Stage& st) {
    std::vector<swsrv::Request*> group;
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [this] { return stop_ || !q_.empty(); });
        if (q_.empty()) return;
        // the queue's head and the requests right behind it in device memory
        group.assign(1, q_.front());
        q_.pop_front();
        uint64_t end = group[0]->dev_off + group[0]->bytes;
        while (group[0]->bytes <= kStage && !q_.empty() && q_.front()->dev_off == end &&
               end + q_.front()->bytes - group[0]->dev_off <= kStage) {
          end += q_.front()->bytes;
          group.push_back(q_.front());
          q_.pop_front();
        }
      }
      const int rc = group[0]->bytes > kStage ? upload_large(st, group[0]) : upload_group(st, group);
      for (swsrv::Request* r : group) {
        r->upload_error = rc;
        r->uploaded.store(true, std::memory_order_release);
      }
      notify_();
    }
  }

  // the requests' blocks as laid out in the pool: characters, then the
  // offsets at the next 256-byte boundary
  static void layout(const swsrv::Request* r, const uint8_t** src, uint64_t* len, uint64_t* at) {
    src[0] = r->nchars ? r->chars + r->offsets[0] : nullptr;
    src[1] = (const uint8_t*)r->offsets;
    len[0] = r->nchars;
    len[1] = 4ull * (r->n + 1);
    at[0] = 0;
    at[1] = swsrv::DevicePool::rounded(r->nchars);
  }

  int next_buffer(Stage& st, int* b) {
    *b = st.next;
    st.next ^= 1;
    return hipEventSynchronize(st.ev[*b]) == hipSuccess ? SW_OK : SW_ERR_HIP;   // its previous copy is done
  }

  int upload_group(Stage& st, const std::vector<swsrv::Request*>& group) {
    const uint64_t start = group[0]->dev_off;
    const uint64_t total = group.back()->dev_off + group.back()->bytes - start;
    int b;
    if (next_buffer(st, &b)) return SW_ERR_HIP;
    for (const swsrv::Request* r : group) {
      const uint8_t* src[2];
      uint64_t len[2], at[2];
      layout(r, src, len, at);
      for (int part = 0; part < 2; ++part)
        if (len[part]) memcpy(st.buf[b] + (r->dev_off - start) + at[part], src[part], len[part]);
    }
    std::lock_guard<std::mutex> lk(issue_mu_[st.stream]);
    if (hipMemcpyAsync(base_ + start, st.buf[b], total, hipMemcpyHostToDevice, s_[st.stream]) != hipSuccess ||
        hipEventRecord(st.ev[b], s_[st.stream]) != hipSuccess)
      return SW_ERR_HIP;
    const uint64_t q = ++seq_[st.stream];
    for (swsrv::Request* r : group) {
      r->upload_event = st.ev[b];
      r->upload_seq = q;
      r->upload_stream = st.stream;
    }
    return SW_OK;
  }

  int upload_large(Stage& st, swsrv::Request* r) {
    const uint8_t* src[2];
    uint64_t len[2], at[2];
    layout(r, src, len, at);
    uint8_t* dst = base_ + r->dev_off;
    for (int part = 0; part < 2; ++part) {
      for (uint64_t pos = 0; pos < len[part]; pos += kStage) {
        const uint64_t n = std::min(kStage, len[part] - pos);
        int b;
        if (next_buffer(st, &b)) return SW_ERR_HIP;
        memcpy(st.buf[b], src[part] + pos, n);
        std::lock_guard<std::mutex> lk(issue_mu_[st.stream]);
        if (hipMemcpyAsync(dst + at[part] + pos, st.buf[b], n, hipMemcpyHostToDevice, s_[st.stream]) != hipSuccess ||
            hipEventRecord(st.ev[b], s_[st.stream]) != hipSuccess)
          return SW_ERR_HIP;
        r->upload_event = st.ev[b];
        r->upload_seq = ++seq_[st.stream];
        r->upload_stream = st.stream;
      }
    }
    return SW_OK;
  }

  hipStream_t s_[kStreams] = {};
  uint8_t* base_ = nullptr;
  std::function<void()> notify_;
  std::vector<Stage> stage_;
  std::vector<std::thread> th_;
  std::mutex mu_, issue_mu_[kStreams];
  std::condition_variable cv_;
  std::deque<swsrv::Request*> q_;
  uint64_t seq_[kStreams] = {};   // uploads issued on each stream
  bool stop_ = false;
};

struct SrvSlot {
  hipStream_t s = nullptr;
  sw_plan* plan = nullptr;
  uint8_t* d_chars = nullptr;
  uint32_t *d_offsets = nullptr, *d_docs = nullptr, *d_perm = nullptr, *d_boff = nullptr;
  sw::GatherPiece *d_pieces = nullptr, *h_pieces = nullptr;
  uint32_t *h_docs = nullptr, *h_perm = nullptr, *h_boff = nullptr, *h_status = nullptr;
  hipEvent_t ev = nullptr;
  std::vector<uint64_t> wpos, cpos;   // per request: first word and first char in the batch
};

class HipExec {
 public:
  uint64_t max_words = 0, max_docs = 0, max_chars = 0, max_pieces = 0;
  std::vector<SrvSlot> slot;
  CopyPool* pool = nullptr;
  // the budget: one device allocation, handed out in blocks
  uint8_t* d_pool = nullptr;
  swsrv::DevicePool blocks;
  Uploader up;

  uint32_t slots() const { return (uint32_t)slot.size(); }
  bool capacity(uint64_t words, uint64_t docs, uint64_t chars) const {
    return words <= max_words && docs <= max_docs && chars <= max_chars;
  }

  // Called by the scheduler thread only.
  bool reserve(swsrv::Request& r) {
    if (!blocks.alloc(r.bytes, &r.dev_off)) return false;
    up.push(&r);
    return true;
  }
  bool uploaded(const swsrv::Request& r) { return r.uploaded.load(std::memory_order_acquire); }
  void release(swsrv::Request& r) { blocks.release(r.dev_off, r.bytes); }

  // On an error the slot's stream is drained first, so the slot's buffers
  // are free again when the batch is closed.
  int launch(swsrv::Batch& b) {
    const int rc = enqueue(b);
    if (rc) (void)hipStreamSynchronize(slot[(size_t)b.slot].s);
    return rc;
  }

  int enqueue(swsrv::Batch& b) {
    SrvSlot& sl = slot[(size_t)b.slot];
    const size_t nr = b.reqs.size();
    sl.wpos.resize(nr + 1);
    sl.cpos.resize(nr + 1);
    sl.wpos[0] = sl.cpos[0] = 0;
    sl.h_docs[0] = 0;
    // per upload stream, the batch's request uploaded last on it
    const swsrv::Request* latest[Uploader::kStreams] = {};
    uint32_t np = 0;
    for (size_t i = 0; i < nr; ++i) {
      const swsrv::Request* r = b.reqs[i];
      if (r->upload_error) return r->upload_error;
      const swsrv::Request*& l = latest[r->upload_stream];
      if (!l || r->upload_seq > l->upload_seq) l = r;
      sl.wpos[i + 1] = sl.wpos[i] + r->n;
      sl.cpos[i + 1] = sl.cpos[i] + r->nchars;
      sl.h_docs[i + 1] = (uint32_t)sl.wpos[i + 1];
      const uint8_t* blk = d_pool + r->dev_off;
      for (uint32_t k0 = 0; k0 == 0 || k0 < r->n; k0 += sw::kGatherWords) {
        if (np >= max_pieces) return fail(SW_ERR_WORKSPACE, "server: batch pieces over capacity");
        sl.h_pieces[np++] = sw::GatherPiece{blk, (const uint32_t*)(blk + swsrv::DevicePool::rounded(r->nchars)), k0,
                                            std::min(r->n, k0 + sw::kGatherWords), r->n, (uint32_t)sl.wpos[i],
                                            (uint32_t)sl.cpos[i]};
      }
    }
    const uint64_t W = sl.wpos[nr];
    HIP_TRY(hipMemcpyAsync(sl.d_pieces, sl.h_pieces, sizeof(sw::GatherPiece) * np, hipMemcpyHostToDevice, sl.s));
    HIP_TRY(hipMemcpyAsync(sl.d_docs, sl.h_docs, 4 * (nr + 1), hipMemcpyHostToDevice, sl.s));
    // each upload stream carries its copies in issue order: the batch's latest
    // on a stream covers its other requests there
    for (const swsrv::Request* l : latest)
      if (l) HIP_TRY(hipStreamWaitEvent(sl.s, (hipEvent_t)l->upload_event, 0));
    sw::k_gather<256><<<np, 256, 0, sl.s>>>(sl.d_pieces, sl.d_chars, sl.d_offsets);
    HIP_TRY(hipGetLastError());
    int rc = sw_plan_run(sl.plan, sl.d_chars, sl.d_offsets, sl.d_docs, (uint32_t)nr, (uint32_t)W, sl.d_perm,
                         sl.d_boff);
    if (rc) return rc;
    if (W) HIP_TRY(hipMemcpyAsync(sl.h_perm, sl.d_perm, 4 * W, hipMemcpyDeviceToHost, sl.s));
    HIP_TRY(hipMemcpyAsync(sl.h_boff, sl.d_boff, 4 * nr * SW_NUM_OFFSETS, hipMemcpyDeviceToHost, sl.s));
    if ((rc = sw_plan_status_async(sl.plan, sl.h_status))) return rc;
    HIP_TRY(hipEventRecord(sl.ev, sl.s));
    return SW_OK;
  }

  bool poll(const swsrv::Batch& b) { return hipEventQuery(slot[(size_t)b.slot].ev) != hipErrorNotReady; }

  int finish(swsrv::Batch& b) {
    SrvSlot& sl = slot[(size_t)b.slot];
    HIP_TRY(hipEventSynchronize(sl.ev));
    const int st = sort_words_decode_status(*sl.h_status);
    if (st) return st;
    const size_t nr = b.reqs.size();
    const unsigned parts = std::min<unsigned>(pool->threads(), (unsigned)nr);
    auto out = [&](unsigned part) {
      const size_t lo = nr * part / parts, hi = nr * (part + 1) / parts;
      for (size_t i = lo; i < hi; ++i) {
        swsrv::Request* r = b.reqs[i];
        if (r->n) memcpy(r->out_perm, sl.h_perm + sl.wpos[i], 4 * (size_t)r->n);
        memcpy(r->out_boff, sl.h_boff + i * SW_NUM_OFFSETS, 4 * SW_NUM_OFFSETS);
      }
    };
    pool->run(parts, out);
    return SW_OK;
  }
};

// Pieces of k_gather a batch can need: every request at least one, and one
// more per kGatherWords words.
uint64_t max_gather_pieces(uint64_t max_words, uint64_t max_docs) {
  return max_words / sw::kGatherWords + max_docs + 1;
}

double srv_now() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct sw_server {
  int device = 0;
  HipExec ex;
  std::unique_ptr<CopyPool> pool;
  std::unique_ptr<swsrv::Scheduler<HipExec>> sched;
  swsrv::Limits lim;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv_in, cv_done;
  std::deque<swsrv::Request*> intake;
  swsrv::TicketBook live;
  swsrv::Counters counters;
  uint64_t next_ticket = 1;
  bool stop = false;
  bool wake = false;        // an upload was issued: the scheduler looks again
  int thread_error = 0;
};

static void server_loop(sw_server* sv) {
  (void)hipSetDevice(sv->device);
  std::vector<swsrv::Request*> done;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      if (!sv->sched->busy() && sv->intake.empty()) {
        if (sv->stop) return;
        sv->cv_in.wait(lk, [sv] { return sv->stop || !sv->intake.empty(); });
        if (sv->stop && sv->intake.empty()) return;
      }
      while (!sv->intake.empty()) {
        sv->sched->enqueue(sv->intake.front());
        sv->intake.pop_front();
      }
    }
    done.clear();
    const uint64_t batches0 = sv->sched->counters().batches;
    sv->sched->step(srv_now(), done);
    const bool launched = sv->sched->counters().batches != batches0;
    if (!done.empty() || launched) {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->counters = sv->sched->counters();
      for (swsrv::Request* r : done) r->finished = true;
      if (!done.empty()) sv->cv_done.notify_all();
    }
    if (done.empty() && !launched) {
      // batches on the device or uploads in flight, nothing to do: look again
      // on the next submission or issued upload, or shortly
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_in.wait_for(lk, std::chrono::microseconds(20), [sv] { return !sv->intake.empty() || sv->wake; });
      sv->wake = false;
    }
  }
}

static void server_free(sw_server* sv) {
  if (!sv) return;
  (void)hipSetDevice(sv->device);
  sv->ex.up.stop();
  for (SrvSlot& sl : sv->ex.slot) {
    if (sl.s) (void)hipStreamSynchronize(sl.s);
    if (sl.plan) sw_plan_destroy(sl.plan);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    for (void* d : {(void*)sl.d_chars, (void*)sl.d_offsets, (void*)sl.d_docs, (void*)sl.d_perm, (void*)sl.d_boff,
                    (void*)sl.d_pieces})
      if (d) (void)hipFree(d);
    for (void* h : {(void*)sl.h_pieces, (void*)sl.h_docs, (void*)sl.h_perm, (void*)sl.h_boff, (void*)sl.h_status})
      if (h) (void)hipHostFree(h);
    if (sl.s) (void)hipStreamDestroy(sl.s);
  }
  sv->ex.up.free_all();
  if (sv->ex.d_pool) (void)hipFree(sv->ex.d_pool);
  delete sv;   // the ticket book frees the requests never waited for
}

extern "C" {

int sw_server_create(const sw_server_config* cfg, sw_server** out) {
  if (!cfg || !out) return fail(SW_ERR_INVALID_ARG, "sw_server_create: null argument");
  *out = nullptr;
  if (cfg->slots < 1 || cfg->slots > 8 || cfg->max_batch_words < 1 || cfg->max_batch_docs < 1 ||
      cfg->max_batch_chars < 1 || cfg->copy_threads > 64)
    return fail(SW_ERR_INVALID_ARG, "sw_server_create: slots 1..8, batch limits >= 1, copy_threads <= 64");
  if (cfg->max_batch_chars >= (1ull << 32))
    return fail(SW_ERR_INVALID_ARG, "sw_server_create: a batch's characters must stay below 2^32");
  int device = 0;
  HIP_TRY(hipGetDevice(&device));
  sw_server* sv = new sw_server();
  sv->device = device;
  sv->lim.budget_bytes = cfg->budget_bytes;
  sv->lim.max_batch_words = cfg->max_batch_words;
  sv->lim.max_batch_docs = cfg->max_batch_docs;
  sv->lim.max_batch_chars = cfg->max_batch_chars;
  sv->lim.min_batch_words = cfg->min_batch_words;
  sv->lim.max_wait_s = cfg->max_wait_us * 1e-6;
  HipExec& ex = sv->ex;
  ex.max_words = cfg->max_batch_words;
  ex.max_docs = cfg->max_batch_docs;
  ex.max_chars = cfg->max_batch_chars;
  ex.max_pieces = max_gather_pieces(cfg->max_batch_words, cfg->max_batch_docs);
  sv->pool.reset(new CopyPool(cfg->copy_threads));
  ex.pool = sv->pool.get();
  ex.slot.resize(cfg->slots);
  const uint64_t W = cfg->max_batch_words, D = cfg->max_batch_docs, C = cfg->max_batch_chars;
  auto cleanup = [&](int rc) {
    server_free(sv);
    return rc;
  };
  // the budget is device memory held from the start; admitted requests live in it
  ex.blocks.reset(cfg->budget_bytes);
  if (ex.blocks.capacity() && hipMalloc(&ex.d_pool, ex.blocks.capacity()) != hipSuccess)
    return cleanup(fail(SW_ERR_OOM, "sw_server_create: device pool of %llu bytes",
                        (unsigned long long)ex.blocks.capacity()));
  for (SrvSlot& sl : ex.slot) {
    if (hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess)
      return cleanup(fail(SW_ERR_HIP, "sw_server_create: stream or event creation failed"));
    int rc = sw_plan_create((uint32_t)W, (uint32_t)D, C, sl.s, &sl.plan);
    if (rc) return cleanup(rc);
    if (hipMalloc(&sl.d_chars, C) != hipSuccess || hipMalloc(&sl.d_offsets, 4 * (W + 1)) != hipSuccess ||
        hipMalloc(&sl.d_docs, 4 * (D + 1)) != hipSuccess || hipMalloc(&sl.d_perm, 4 * W) != hipSuccess ||
        hipMalloc(&sl.d_boff, 4 * D * SW_NUM_OFFSETS) != hipSuccess ||
        hipMalloc(&sl.d_pieces, sizeof(sw::GatherPiece) * ex.max_pieces) != hipSuccess)
      return cleanup(fail(SW_ERR_OOM, "sw_server_create: device buffers"));
    if (hipHostMalloc(&sl.h_pieces, sizeof(sw::GatherPiece) * ex.max_pieces, 0) != hipSuccess ||
        hipHostMalloc(&sl.h_docs, 4 * (D + 1), 0) != hipSuccess || hipHostMalloc(&sl.h_perm, 4 * W, 0) != hipSuccess ||
        hipHostMalloc(&sl.h_boff, 4 * D * SW_NUM_OFFSETS, 0) != hipSuccess ||
        hipHostMalloc(&sl.h_status, 4, 0) != hipSuccess)
      return cleanup(fail(SW_ERR_OOM, "sw_server_create: pinned staging"));
  }
  {
    const int rc = ex.up.init(std::max(1u, cfg->copy_threads), ex.d_pool, [sv] {
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->wake = true;
      }
      sv->cv_in.notify_one();
    });
    if (rc) return cleanup(fail(rc, "sw_server_create: upload threads"));
  }
  sv->sched.reset(new swsrv::Scheduler<HipExec>(ex, sv->lim));
  sv->th = std::thread(server_loop, sv);
  *out = sv;
  return SW_OK;
}

int sw_server_submit(sw_server* sv, const uint8_t* chars, const uint32_t* offsets, uint32_t n_words,
                     uint32_t* out_perm, uint32_t* out_bucket_offsets, uint64_t* out_ticket) {
  if (!sv || !offsets || !out_bucket_offsets || !out_ticket || (n_words && !out_perm))
    return fail(SW_ERR_INVALID_ARG, "sw_server_submit: null argument");
  const int chk = swsrv::check_request(offsets, n_words, SW_MAX_LEN);
  if (chk) return fail(chk, "sw_server_submit: %s", chk == SW_ERR_INVALID_ARG ? "offsets decrease" : "a word is too long");
  const uint64_t nchars = (uint64_t)offsets[n_words] - offsets[0];
  if (nchars && !chars) return fail(SW_ERR_INVALID_ARG, "sw_server_submit: null characters");
  swsrv::Request* r = new swsrv::Request();
  r->chars = chars;
  r->offsets = offsets;
  r->n = n_words;
  r->nchars = nchars;
  r->bytes = swsrv::footprint(n_words, nchars);
  r->out_perm = out_perm;
  r->out_boff = out_bucket_offsets;
  r->status = 1;   // pending
  if (!sv->sched->acceptable(*r)) {
    delete r;
    return fail(SW_ERR_WORKSPACE, "sw_server_submit: a request of %u words can never fit", n_words);
  }
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    r->ticket = sv->next_ticket++;
    r->arrival = srv_now();
    sv->live.add(r);
    sv->intake.push_back(r);
    *out_ticket = r->ticket;
  }
  sv->cv_in.notify_one();
  return SW_OK;
}

int sw_server_wait(sw_server* sv, uint64_t ticket, double* latency_s) {
  if (!sv) return fail(SW_ERR_INVALID_ARG, "sw_server_wait: null server");
  std::unique_lock<std::mutex> lk(sv->mu);
  swsrv::Request* r = nullptr;
  if (sv->live.claim(ticket, &r))
    return fail(SW_ERR_INVALID_ARG, "sw_server_wait: ticket %llu is unknown or already waited for",
                (unsigned long long)ticket);
  sv->cv_done.wait(lk, [r] { return r->finished; });
  const int st = r->status;
  if (latency_s) *latency_s = r->done - r->arrival;
  sv->live.release(ticket);
  return st ? fail(st, "sw_server_wait: the request's batch failed") : SW_OK;
}

int sw_server_stats(sw_server* sv, sw_server_counts* out) {
  if (!sv || !out) return fail(SW_ERR_INVALID_ARG, "sw_server_stats: null argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  out->completed = sv->counters.completed;
  out->failed = sv->counters.failed;
  out->words = sv->counters.words;
  out->batches = sv->counters.batches;
  out->bytes_in_use = sv->counters.in_use;
  out->max_bytes_in_use = sv->counters.max_in_use;
  return SW_OK;
}

size_t sw_server_fixed_bytes(const sw_server_config* cfg) {
  if (!cfg) return 0;
  const uint64_t W = cfg->max_batch_words, D = cfg->max_batch_docs;
  return (size_t)cfg->slots * (sort_words_workspace_size((uint32_t)W, (uint32_t)D) + cfg->max_batch_chars +
                               8 * (W + 1) + 4 * (D + 1) + 4 * D * SW_NUM_OFFSETS +
                               sizeof(sw::GatherPiece) * max_gather_pieces(W, D));
}

uint64_t sw_server_request_bytes(uint32_t n_words, uint64_t n_chars) { return swsrv::footprint(n_words, n_chars); }

void sw_server_destroy(sw_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_in.notify_all();
  if (sv->th.joinable()) sv->th.join();
  server_free(sv);
}

}  // extern "C"
