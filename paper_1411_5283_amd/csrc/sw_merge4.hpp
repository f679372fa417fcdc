// sw_merge4.hpp -- the streamed four-way merge of one merge level, as plain
// code built for the device (k_merge4 in sw_kernels.hpp calls these phases
// with barriers between them) and, by its test, for the host (the same
// phases run thread by thread).
//
// A four-way level merges groups of four consecutive sorted runs of R items
// (the last group of a segment may hold fewer or shorter runs) into runs of
// 4R: one HBM read and one write of every item for two doublings of the run
// length, where a two-way level spends them on one.  The merge is done as the
// tree merge(merge(A, B), merge(C, D)) inside the workgroup: A..D stream
// through rings in LDS, the first level keeps X = merge(A, B) and
// Y = merge(C, D) topped up in two small LDS rings, and the final level
// merges X and Y into the output, PS items a step.  A workgroup takes one
// contiguous range of the level's output; where the range starts inside a
// group, the four co-ranks of its first output come from the split search of
// sw_split.hpp, and from there every step's consumption follows from the
// merges themselves, so no tile placement is searched for in HBM.
//
// A step:
//   A  the items loaded last step go into their ring slots; loads are issued
//      for every ring slot now free (they land at the next step's A, so a
//      whole step hides their latency);
//   B  X and Y are topped up to PS items (or to their end) from the rings;
//   C  PS outputs (or fewer at the range's end) are merged from X and Y;
//   D  the outputs are stored from registers.
// With rings of RC >= 2 PS, a run has at least RC - PS >= PS items in its
// ring at every B (or all it has left), so the top-up never needs an item that
// is not there; every merge path below reads a missing item as the sentinel,
// which is exact at a run's end and never decides an output elsewhere.
#pragma once

#include "sw_keys.hpp"
#include "sw_split.hpp"

namespace sw {

// Keys in LDS as structure of arrays, N slots.
template <int NL, int N>
struct SlotArr {
  uint64_t k[NL][N];
  uint32_t idx[N];
  __host__ __device__ Key<NL> get(uint32_t i) const {
    Key<NL> v;
#pragma unroll
    for (int q = 0; q < NL; ++q) v.k[q] = k[q][i];
    v.idx = idx[i];
    return v;
  }
  __host__ __device__ void put(uint32_t i, const Key<NL>& v) {
#pragma unroll
    for (int q = 0; q < NL; ++q) k[q][i] = v.k[q];
    idx[i] = v.idx;
  }
};
template <int N>
struct SlotArr<0, N> {
  uint64_t k[N];
  __host__ __device__ Key<0> get(uint32_t i) const {
    Key<0> v;
    v.k = k[i];
    return v;
  }
  __host__ __device__ void put(uint32_t i, const Key<0>& v) { k[i] = v.k; }
};

__host__ __device__ __attribute__((always_inline)) inline int m4_bitlen(uint32_t x) {
  int b = 0;
  while (x) {
    ++b;
    x >>= 1;
  }
  return b;
}

// a + b modulo m, for a, b < m
__host__ __device__ __attribute__((always_inline)) inline uint32_t m4_wrap(uint32_t a, uint32_t b, uint32_t m) {
  const uint32_t s = a + b;
  return s >= m ? s - m : s;
}

// Four-way level geometry of a segment of n items: the group holding segment
// position s, its four runs (start inside the segment, length) and the rank
// of s inside the group.
struct M4Group {
  uint64_t start;       // group's first position in the segment
  uint32_t run_off[4];  // runs' first positions relative to the group
  uint32_t len[4];
  uint32_t size;        // items in the group
  uint32_t d;           // rank of s inside the group
};
__host__ __device__ __attribute__((always_inline)) inline M4Group m4_group(uint32_t n, uint64_t s, uint64_t R) {
  M4Group g;
  const uint64_t G = 4 * R;
  g.start = (s / G) * G;
  g.d = (uint32_t)(s - g.start);
  uint64_t at = g.start;
  for (int i = 0; i < 4; ++i) {
    g.run_off[i] = (uint32_t)(at - g.start);
    const uint64_t e = at + R < n ? at + R : (uint64_t)n;
    g.len[i] = e > at ? (uint32_t)(e - at) : 0u;
    at = e > at ? e : at;
  }
  g.size = (uint32_t)(at - g.start);
  return g;
}

template <int NL, int NT, int E, int PS, int RC>
struct M4 {
  static_assert(PS <= NT * E, "one step's outputs fit the threads");
  static_assert(RC >= 2 * PS, "a ring keeps a step of items while the next step's loads are in flight");
  static_assert((PS & (PS - 1)) == 0 && (RC & (RC - 1)) == 0, "ring sizes are powers of two");
  static constexpr int FE = (PS + NT - 1) / NT;   // in-flight items per thread
  static constexpr uint32_t RM = RC - 1, XM = PS - 1;
  using K = Key<NL>;

  struct Lds {
    SlotArr<NL, RC> ring[4];
    union {
      SlotArr<NL, PS> xy[2];
      SplitScratch<K> sp;
    } u;
    uint32_t end[2][2];   // items of each input taken by the last top-up of X (0) and Y (1)
    uint32_t xsplit;      // X items among the last step's outputs
    uint32_t seg;         // broadcast of a segment index
  };

  // Uniform stream state, held by every thread.
  struct State {
    uint64_t start[4];                 // HBM position of each run's first item
    uint32_t len[4], cons[4], valid[4], fly[4], hs[4];   // hs: ring slot of the next item
    uint32_t px[2], cx[2], hx[2];      // X/Y: items produced, consumed, slot of the next one
    uint32_t sealed;                   // bits 0-3: run's end marked; bits 4-5: X's, Y's
  };

  struct Less {
    __host__ __device__ __attribute__((always_inline)) bool operator()(const K& a, const K& b) const {
      return key_less<NL>(a, b);
    }
  };

  // ---------------------------------------------------------------- views
  // A run (or X, Y) as seen from its next unconsumed item: item j sits in
  // slot (head + j) mod CAP.  A read is one masked LDS load, never a branch:
  // past the valid items a ring holds either later items, stale ones or --
  // once everything of that run (or side) is in the ring and there is room --
  // a sentinel right after its last item.  The merges below read an item
  // past the valid ones only where it cannot decide an output they keep:
  // while a run has items beyond its ring it holds at least PS of them, more
  // than one step takes, and at its end the sentinel is in place.
  template <int CAP>
  struct View {
    const SlotArr<NL, CAP>* r;
    uint32_t head;
    __host__ __device__ __attribute__((always_inline)) K operator()(uint32_t j) const {
      return r->get((head + j) & (uint32_t)(CAP - 1));
    }
  };
  using RunView = View<RC>;
  using XyView = View<PS>;

  // Merge path (Odeh et al., IPDPSW 2012): items of A among the first d of
  // merge(A, B), by ksteps halvings (2^ksteps - 1 >= the search range).  A
  // probe out of range reads some slot and is not counted.
  template <class V>
  __host__ __device__ __attribute__((always_inline)) static uint32_t path(const V& A, uint32_t la, const V& B,
                                                                        uint32_t lb, uint32_t d, int ksteps) {
    uint32_t lo = d > lb ? d - lb : 0u;
    const uint32_t hi = d < la ? d : la;
    for (int k = ksteps - 1; k >= 0; --k) {
      const uint32_t a = lo + (1u << k) - 1;
      const bool take = a < hi && !Less()(B(d - 1 - a), A(a));
      lo = take ? lo + (1u << k) : lo;
    }
    return lo;
  }

  // E outputs of merge(A, B) from A[pa], B[pb]; pa, pb end past the first n
  // of them.  One LDS read an output: the next item of whichever run gave it.
  template <int CAP>
  __host__ __device__ __attribute__((always_inline)) static void serial(const View<CAP>& A, const View<CAP>& B,
                                                                      uint32_t& pa, uint32_t& pb, K (&out)[E],
                                                                      uint32_t n) {
    K ha = A(pa), hb = B(pb);
    uint32_t qa = pa, qb = pb;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const bool takeB = Less()(hb, ha);
      out[j] = key_select<NL>(takeB, hb, ha);
      qa += takeB ? 0u : 1u;
      qb += takeB ? 1u : 0u;
      const SlotArr<NL, CAP>* from = takeB ? B.r : A.r;
      const K nv = from->get(((takeB ? B.head + qb : A.head + qa)) & (uint32_t)(CAP - 1));
      ha = key_select<NL>(takeB, ha, nv);
      hb = key_select<NL>(takeB, nv, hb);
      if ((uint32_t)j + 1 == n) {
        pa = qa;
        pb = qb;
      }
    }
  }

  // ---------------------------------------------------------------- start
  // State of a stream whose first output has co-ranks sp[] in the runs.
  __host__ __device__ __attribute__((always_inline)) static void begin(State& s, const uint64_t (&start)[4],
                                                                     const uint32_t (&len)[4],
                                                                     const uint32_t (&sp)[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      s.start[r] = start[r];
      s.len[r] = len[r];
      s.cons[r] = sp[r];
      s.valid[r] = 0;
      s.fly[r] = 0;
      s.hs[r] = 0;
    }
#pragma unroll
    for (int x = 0; x < 2; ++x) s.px[x] = s.cx[x] = s.hx[x] = 0;
    s.sealed = 0;
  }

  // Loads for the ring slots now free (at most `cap` items in all, runs in
  // order); true if the cap cut them short.  At a stream's start the cap is
  // 4 RC and the loads are done at once; in the stream's steps it is what the
  // threads can hold in registers, which the consumption of one top-up
  // (at most PS items) never exceeds.
  __host__ __device__ __attribute__((always_inline)) static bool fill_amounts(State& s, uint32_t cap) {
    uint32_t tot = 0;
    bool cut = false;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t left = s.len[r] - s.cons[r] - s.valid[r];
      const uint32_t room = (uint32_t)RC - s.valid[r];
      uint32_t f = left < room ? left : room;
      if (f > cap - tot) {
        f = cap - tot;
        cut = true;
      }
      s.fly[r] = f;
      tot += f;
    }
    return cut;
  }
  // Item q of the refill list (runs one after another, each run's items past
  // its valid ones): loads it from HBM (false when q is past the list).  The
  // runs are walked with compile-time indices, so the state stays in registers.
  __host__ __device__ __attribute__((always_inline)) static uint32_t refill_total(const State& s) {
    return s.fly[0] + s.fly[1] + s.fly[2] + s.fly[3];
  }
  __host__ __device__ __attribute__((always_inline)) static bool refill_load(const State& s, const KeyBuf& src,
                                                                           uint32_t q, K& v) {
    bool found = false;
    uint64_t at = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool here = !found && q < s.fly[r];
      at = here ? s.start[r] + s.cons[r] + s.valid[r] + q : at;
      if (!found && !here) q -= s.fly[r];
      found = found || here;
    }
    if (found) v = gload<NL>(src, (size_t)at);
    return found;
  }
  // Stores item q of the refill list into its ring slot.
  __host__ __device__ __attribute__((always_inline)) static void refill_put(Lds& L, const State& s, uint32_t q,
                                                                          const K& v) {
    bool found = false;
    uint32_t ring = 0, slot = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool here = !found && q < s.fly[r];
      ring = here ? (uint32_t)r : ring;
      slot = here ? (s.hs[r] + s.valid[r] + q) & RM : slot;
      if (!found && !here) q -= s.fly[r];
      found = found || here;
    }
    if (found) L.ring[ring].put(slot, v);
  }
  // After the refill items are in their slots (every thread, same values).
  __host__ __device__ __attribute__((always_inline)) static void refill_done(State& s) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      s.valid[r] += s.fly[r];
      s.fly[r] = 0;
    }
  }
  // A run whose every remaining item is in its ring gets a sentinel right
  // after its last one, as soon as there is a free slot (thread r writes run
  // r's; every thread notes it).
  __host__ __device__ __attribute__((always_inline)) static void seal_runs(Lds& L, State& s, uint32_t tid) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool now = !(s.sealed & (1u << r)) && s.cons[r] + s.valid[r] == s.len[r] && s.valid[r] < (uint32_t)RC;
      if (now && tid == (uint32_t)r) L.ring[r].put((s.hs[r] + s.valid[r]) & RM, key_sentinel<NL>());
      s.sealed |= now ? 1u << r : 0u;
    }
  }

  // ---------------------------------------------------------------- B: top-up
  // Items of A and B (C and D) not yet taken into X (Y).
  __host__ __device__ __attribute__((always_inline)) static uint32_t left(const State& s, int side) {
    return side ? (s.len[2] - s.cons[2]) + (s.len[3] - s.cons[3]) : (s.len[0] - s.cons[0]) + (s.len[1] - s.cons[1]);
  }
  __host__ __device__ __attribute__((always_inline)) static uint32_t want(const State& s, int side) {
    const uint32_t have = side ? s.px[1] - s.cx[1] : s.px[0] - s.cx[0];
    const uint32_t l = left(s, side), room = (uint32_t)PS - have;
    return l < room ? l : room;
  }
  // Work items of the top-up per side: thread t merges X's item t and Y's
  // item t (E outputs each); one thread count covers both, since want <= PS
  // = NT * E items.
  __host__ __device__ __attribute__((always_inline)) static uint32_t topup_items(const State& s) {
    const uint32_t nx = (want(s, 0) + E - 1) / E, ny = (want(s, 1) + E - 1) / E;
    return nx > ny ? nx : ny;
  }
  // The E outputs at diagonal dd of one side's top-up (n of them real), into
  // out[]; the input positions after them in pa, pb.  Computed for every
  // thread, real work or not, so that the two sides' searches interleave.
  template <int SIDE>
  __host__ __device__ __attribute__((always_inline)) static uint32_t topup_merge(const Lds& L, const State& s,
                                                                               uint32_t dd, uint32_t wnt,
                                                                               uint32_t& pa, uint32_t& pb,
                                                                               K (&out)[E]) {
    constexpr int RA = 2 * SIDE, RB = RA + 1;
    const RunView A{&L.ring[RA], s.hs[RA]}, B{&L.ring[RB], s.hs[RB]};
    pa = path(A, s.valid[RA], B, s.valid[RB], dd, m4_bitlen((uint32_t)PS));
    pb = dd - pa;
    const uint32_t n = dd < wnt ? (wnt - dd < (uint32_t)E ? wnt - dd : (uint32_t)E) : 0u;
    serial(A, B, pa, pb, out, n);
    return n;
  }
  template <int SIDE>
  __host__ __device__ __attribute__((always_inline)) static void topup_store(Lds& L, const State& s, uint32_t dd,
                                                                           uint32_t wnt, uint32_t n, uint32_t pa,
                                                                           uint32_t pb, const K (&out)[E]) {
    const uint32_t at = s.hx[SIDE] + (s.px[SIDE] - s.cx[SIDE]) + dd;
#pragma unroll
    for (int j = 0; j < E; ++j)
      if ((uint32_t)j < n) L.u.xy[SIDE].put((at + j) & XM, out[j]);
    if (n && dd + n == wnt) {
      L.end[SIDE][0] = pa;
      L.end[SIDE][1] = pb;
    }
  }
  // Thread w's share of the top-up: X's work item w and Y's work item w.
  __host__ __device__ __attribute__((always_inline)) static void topup(Lds& L, const State& s, uint32_t w) {
    const uint32_t wx = want(s, 0), wy = want(s, 1);
    uint32_t xa, xb, ya, yb;
    K xo[E], yo[E];
    const uint32_t nx = topup_merge<0>(L, s, w * E, wx, xa, xb, xo);
    const uint32_t ny = topup_merge<1>(L, s, w * E, wy, ya, yb, yo);
    topup_store<0>(L, s, w * E, wx, nx, xa, xb, xo);
    topup_store<1>(L, s, w * E, wy, ny, ya, yb, yo);
  }
  // A side whose inputs this top-up exhausts gets a sentinel after its last
  // item once there is a free slot (thread SIDE writes it, beside the top-up,
  // in a slot the top-up does not write).
  __host__ __device__ __attribute__((always_inline)) static void seal_xy(Lds& L, State& s, uint32_t tid,
                                                                       uint32_t wx, uint32_t wy) {
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const uint32_t w = x ? wy : wx;
      const uint32_t have = s.px[x] - s.cx[x] + w;
      const bool now = !(s.sealed & (16u << x)) && left(s, x) == w && have < (uint32_t)PS;
      if (now && tid == (uint32_t)x) L.u.xy[x].put((s.hx[x] + have) & XM, key_sentinel<NL>());
      s.sealed |= now ? 16u << x : 0u;
    }
  }
  // After the top-up (every thread): inputs consumed, X and Y grown.
  __host__ __device__ __attribute__((always_inline)) static void topup_done(State& s, const Lds& L, uint32_t wx,
                                                                          uint32_t wy) {
#pragma unroll
    for (int side = 0; side < 2; ++side) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = 2 * side + h;
        const uint32_t c = L.end[side][h];
        s.cons[r] += c;
        s.valid[r] -= c;
        s.hs[r] = (s.hs[r] + c) & RM;
      }
      s.px[side] += side ? wy : wx;
    }
  }

  // ---------------------------------------------------------------- C: final
  // Thread t's outputs dd = tE .. of this step's cnt: n of them into out[];
  // the thread holding the step's last output records the X items taken.
  __host__ __device__ __attribute__((always_inline)) static uint32_t final_merge(Lds& L, const State& s, uint32_t t,
                                                                               uint32_t cnt, K (&out)[E]) {
    const uint32_t dd = t * E;
    if (dd >= cnt) return 0;
    const XyView X{&L.u.xy[0], s.hx[0]}, Y{&L.u.xy[1], s.hx[1]};
    const uint32_t vx = s.px[0] - s.cx[0], vy = s.px[1] - s.cx[1];
    uint32_t pa = path(X, vx, Y, vy, dd, m4_bitlen((uint32_t)PS));
    uint32_t pb = dd - pa;
    const uint32_t n = cnt - dd < (uint32_t)E ? cnt - dd : (uint32_t)E;
    serial(X, Y, pa, pb, out, n);
    if (dd + n == cnt) L.xsplit = pa;
    return n;
  }
  __host__ __device__ __attribute__((always_inline)) static void final_done(State& s, const Lds& L, uint32_t cnt) {
    const uint32_t tx = L.xsplit;
    s.cx[0] += tx;
    s.hx[0] = (s.hx[0] + tx) & XM;
    s.cx[1] += cnt - tx;
    s.hx[1] = (s.hx[1] + cnt - tx) & XM;
  }
};

}  // namespace sw
