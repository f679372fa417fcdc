// CPU test of the serving scheduler's rules (sw_sched.hpp) with a stand-in
// executor and a simulated clock.  Prints "OK" and exits 0, or names the
// broken rule and exits 1.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "sw_sched.hpp"

using swsrv::Batch;
using swsrv::Request;

#define CHECK(cond, ...)                                 \
  do {                                                   \
    if (!(cond)) {                                       \
      std::printf("FAIL line %d: ", __LINE__);           \
      std::printf(__VA_ARGS__);                          \
      std::printf("\n");                                 \
      std::exit(1);                                      \
    }                                                    \
  } while (0)

struct FakeExec {
  uint32_t nslots = 2;
  uint64_t max_words = 1000, max_docs = 8, max_chars = 1 << 20;
  double* clock = nullptr;
  double per_word = 1e-6;                 // simulated device time
  uint64_t poison = ~0ull;                // a batch holding this ticket fails on the "device"
  std::vector<std::vector<uint64_t>> launched;   // tickets of every batch, in launch order
  std::vector<double> finish_at;
  std::vector<int> running_per_launch;
  int running = 0, max_running = 0;
  // device memory: a pool as large as the budget; uploads take upload_s
  swsrv::DevicePool pool{1ull << 40};
  double upload_s = 0;
  std::map<uint64_t, double> upload_done;   // ticket -> when its upload is issued
  uint64_t reserve_refused = 0, seq = 0;

  uint32_t slots() const { return nslots; }
  bool capacity(uint64_t w, uint64_t d, uint64_t c) const { return w <= max_words && d <= max_docs && c <= max_chars; }
  bool reserve(Request& r) {
    if (!pool.alloc(r.bytes, &r.dev_off)) {
      ++reserve_refused;
      return false;
    }
    upload_done[r.ticket] = *clock + upload_s;
    return true;
  }
  bool uploaded(const Request& r) { return *clock >= upload_done.at(r.ticket); }
  void release(Request& r) { pool.release(r.dev_off, r.bytes); }
  int launch(Batch& b) {
    std::vector<uint64_t> t;
    for (Request* r : b.reqs) {
      t.push_back(r->ticket);
      CHECK(uploaded(*r), "request %llu launched before its upload", (unsigned long long)r->ticket);
    }
    launched.push_back(t);
    finish_at.resize((size_t)b.slot + 1 > finish_at.size() ? (size_t)b.slot + 1 : finish_at.size());
    finish_at[(size_t)b.slot] = *clock + 1e-5 + per_word * (double)b.words;
    ++running;
    if (running > max_running) max_running = running;
    return 0;
  }
  bool poll(const Batch& b) { return *clock >= finish_at[(size_t)b.slot]; }
  int finish(Batch& b) {
    --running;
    for (Request* r : b.reqs)
      if (r->ticket == poison) return -5;
    for (Request* r : b.reqs)
      for (uint32_t i = 0; i < r->n; ++i) r->out_perm[i] = i;
    return 0;
  }
};

static Request* make(uint64_t ticket, uint32_t n, double t, std::vector<uint32_t>& store) {
  Request* r = new Request();
  r->ticket = ticket;
  r->n = n;
  r->nchars = 4ull * n;
  r->bytes = swsrv::footprint(n, r->nchars);
  r->arrival = t;
  store.assign(n ? n : 1, 0xFFFFFFFFu);
  r->out_perm = store.data();
  return r;
}

int main() {
  // 1. FIFO admission under the budget: a large head request is not overtaken
  {
    double clock = 0;
    FakeExec ex;
    ex.clock = &clock;
    swsrv::Limits lim;
    lim.budget_bytes = swsrv::footprint(600, 2400) + swsrv::footprint(100, 400);
    lim.max_batch_words = 1000;
    lim.max_batch_docs = 8;
    swsrv::Scheduler<FakeExec> s(ex, lim);
    std::vector<std::vector<uint32_t>> store(4);
    std::vector<Request*> reqs = {make(1, 600, 0, store[0]), make(2, 500, 0, store[1]), make(3, 50, 0, store[2]),
                                  make(4, 100, 0, store[3])};
    for (Request* r : reqs) {
      CHECK(s.acceptable(*r), "request %llu refused", (unsigned long long)r->ticket);
      s.enqueue(r);
    }
    std::vector<Request*> done;
    std::set<uint64_t> seen;
    for (int it = 0; it < 100000 && s.busy(); ++it) {
      s.step(clock, done);
      CHECK(s.counters().in_use <= lim.budget_bytes, "budget exceeded: %llu", (unsigned long long)s.counters().in_use);
      clock += 1e-5;
    }
    CHECK(!s.busy(), "did not drain");
    for (Request* r : done) {
      CHECK(seen.insert(r->ticket).second, "request %llu finished twice", (unsigned long long)r->ticket);
      CHECK(r->status == 0 && r->out_perm[0] == 0, "request %llu has no result", (unsigned long long)r->ticket);
    }
    CHECK(seen.size() == 4, "%zu of 4 finished", seen.size());
    // request 1 (600 words) fits alone; 2 (500) does not fit beside it, and 3
    // and 4 must not overtake 2: the first batch is {1}, the second starts
    // with 2
    CHECK(ex.launched[0].size() == 1 && ex.launched[0][0] == 1, "first batch is not {1}");
    CHECK(ex.launched[1][0] == 2, "request 2 was overtaken");
    CHECK(s.counters().max_in_use <= lim.budget_bytes, "max in use above budget");
    for (Request* r : reqs) delete r;
  }
  // 2. batch limits and order; slots overlap; min batch words while busy
  {
    double clock = 0;
    FakeExec ex;
    ex.clock = &clock;
    ex.per_word = 2e-6;
    swsrv::Limits lim;
    lim.max_batch_words = 1000;
    lim.max_batch_docs = 4;
    lim.min_batch_words = 300;
    lim.max_wait_s = 1e-3;
    swsrv::Scheduler<FakeExec> s(ex, lim);
    const int N = 60;
    std::vector<std::vector<uint32_t>> store(N);
    std::vector<Request*> reqs;
    std::vector<Request*> done;
    for (int i = 0; i < N; ++i) {
      reqs.push_back(make((uint64_t)i + 1, (uint32_t)(20 + (i * 37) % 200), clock, store[(size_t)i]));
      s.enqueue(reqs.back());
      s.step(clock, done);
      clock += 2e-5;
    }
    for (int it = 0; it < 1000000 && s.busy(); ++it) {
      s.step(clock, done);
      clock += 1e-5;
    }
    CHECK(!s.busy() && done.size() == (size_t)N, "did not drain (%zu of %d)", done.size(), N);
    uint64_t expect = 1;
    for (size_t b = 0; b < ex.launched.size(); ++b) {
      uint64_t words = 0;
      for (uint64_t t : ex.launched[b]) {
        CHECK(t == expect, "batch %zu takes request %llu out of order", b, (unsigned long long)t);
        ++expect;
        words += reqs[(size_t)t - 1]->n;
      }
      CHECK(ex.launched[b].size() <= lim.max_batch_docs && words <= lim.max_batch_words, "batch %zu over limits", b);
    }
    CHECK(ex.max_running == 2, "the two slots never overlapped (max running %d)", ex.max_running);
    CHECK(ex.launched.size() < (size_t)N, "no batching happened");
    for (Request* r : reqs) delete r;
  }
  // 3. a batch that fails on the device fails its requests only
  {
    double clock = 0;
    FakeExec ex;
    ex.clock = &clock;
    ex.nslots = 1;
    ex.poison = 2;
    swsrv::Limits lim;
    lim.max_batch_docs = 1;
    swsrv::Scheduler<FakeExec> s(ex, lim);
    std::vector<std::vector<uint32_t>> store(3);
    std::vector<Request*> reqs = {make(1, 10, 0, store[0]), make(2, 10, 0, store[1]), make(3, 10, 0, store[2])};
    for (Request* r : reqs) s.enqueue(r);
    std::vector<Request*> done;
    for (int it = 0; it < 10000 && s.busy(); ++it) {
      s.step(clock, done);
      clock += 1e-4;
    }
    CHECK(done.size() == 3, "not all finished");
    CHECK(reqs[0]->status == 0 && reqs[1]->status == -5 && reqs[2]->status == 0, "failure not isolated");
    CHECK(s.counters().failed == 1 && s.counters().completed == 2, "counters wrong");
    CHECK(s.counters().in_use == 0, "bytes not released");
    for (Request* r : reqs) delete r;
  }
  // 4. intake checks
  {
    uint32_t ok[] = {0, 3, 3, 35};
    uint32_t dec[] = {0, 3, 2};
    uint32_t lng[] = {5, 10, 43};
    CHECK(swsrv::check_request(ok, 3, 32) == 0, "good request refused");
    CHECK(swsrv::check_request(dec, 2, 32) == -1, "decreasing offsets accepted");
    CHECK(swsrv::check_request(lng, 2, 32) == -2, "33-byte word accepted");
    CHECK(swsrv::check_request(ok, 0, 32) == 0, "empty request refused");
  }
  // 5. tickets: one waiter per ticket; a second claim, or a claim after the
  // wait, is refused; requests never waited for are freed with the book
  {
    swsrv::TicketBook book;
    std::vector<uint32_t> st;
    for (uint64_t t = 1; t <= 3; ++t) book.add(make(t, 4, 0, st));
    Request* r = nullptr;
    CHECK(book.claim(2, &r) == 0 && r && r->ticket == 2, "first claim refused");
    Request* r2 = nullptr;
    CHECK(book.claim(2, &r2) != 0 && r2 == nullptr, "second waiter of one ticket accepted");
    CHECK(book.claim(9, &r2) != 0, "unknown ticket accepted");
    book.release(2);
    CHECK(book.claim(2, &r2) != 0, "a ticket waited for twice");
    CHECK(book.size() == 2, "book holds %zu requests, expected 2", book.size());
    // a claim keeps the request alive until its release, whatever else is added
    CHECK(book.claim(3, &r) == 0, "claim of ticket 3 refused");
    for (uint64_t t = 10; t < 2000; ++t) book.add(make(t, 1, 0, st));
    CHECK(r->ticket == 3 && r->claimed, "claimed request changed");
    book.release(3);
  }
  // 6. the device pool: first fit, no overlap, freed neighbours merge;
  // random allocations and frees against a map of every 256-byte unit
  {
    const uint64_t units = 4096;
    swsrv::DevicePool pool(units * 256 + 100);   // the odd tail is not used
    CHECK(pool.capacity() == units * 256, "capacity %llu", (unsigned long long)pool.capacity());
    std::vector<int> owner(units, -1);
    std::map<int, std::pair<uint64_t, uint64_t>> live;   // id -> (offset, bytes)
    std::mt19937_64 rng(5);
    int next_id = 0;
    uint64_t refused = 0;
    for (int it = 0; it < 200000; ++it) {
      if (live.empty() || rng() % 100 < 55) {
        const uint64_t bytes = rng() % 4 == 0 ? rng() % 300 : rng() % 40000;
        uint64_t off = 0;
        const uint64_t need = swsrv::DevicePool::rounded(bytes) / 256;
        // the lowest run of `need` free units, from the map
        uint64_t want = ~0ull;
        for (uint64_t u = 0, run = 0; u < units; ++u) {
          run = owner[u] < 0 ? run + 1 : 0;
          if (run == need) {
            want = u + 1 - need;
            break;
          }
        }
        const bool ok = pool.alloc(bytes, &off);
        CHECK(ok == (want != ~0ull), "alloc of %llu bytes: pool says %d, map says %d", (unsigned long long)bytes,
              (int)ok, (int)(want != ~0ull));
        if (!ok) {
          ++refused;
          continue;
        }
        CHECK(off == want * 256, "first fit: got %llu, lowest fit %llu", (unsigned long long)off,
              (unsigned long long)(want * 256));
        for (uint64_t u = off / 256; u < off / 256 + need; ++u) owner[u] = next_id;
        live[next_id++] = {off, bytes};
      } else {
        auto itl = live.begin();
        std::advance(itl, (long)(rng() % live.size()));
        const uint64_t off = itl->second.first, bytes = itl->second.second;
        pool.release(off, bytes);
        for (uint64_t u = off / 256; u < off / 256 + swsrv::DevicePool::rounded(bytes) / 256; ++u) owner[u] = -1;
        live.erase(itl);
      }
      uint64_t used = 0;
      for (int o : owner) used += o >= 0 ? 256 : 0;
      CHECK(pool.used() == used, "used %llu, map %llu", (unsigned long long)pool.used(), (unsigned long long)used);
    }
    CHECK(refused > 0, "the pool never filled up");
    for (auto& kv : live) pool.release(kv.second.first, kv.second.second);
    CHECK(pool.used() == 0 && pool.free_blocks() == 1 && pool.largest_free() == pool.capacity(),
          "free blocks did not merge back into one");
  }
  // 7. admission on real blocks: a small pool, requests of mixed sizes,
  // uploads that take time; the budget binds, nothing overlaps, no request
  // runs before its upload, all finish in order
  {
    double clock = 0;
    FakeExec ex;
    ex.clock = &clock;
    ex.upload_s = 3e-5;
    ex.max_words = 4000;
    ex.max_chars = 1 << 20;
    swsrv::Limits lim;
    lim.budget_bytes = 60 * 1024;
    lim.max_batch_words = 4000;
    lim.max_batch_docs = 8;
    ex.pool.reset(lim.budget_bytes);
    swsrv::Scheduler<FakeExec> s(ex, lim);
    std::mt19937_64 rng(9);
    const int N = 400;
    std::vector<std::vector<uint32_t>> store(N);
    std::vector<Request*> reqs, done;
    uint64_t total = 0;
    for (int i = 0; i < N; ++i) {
      reqs.push_back(make((uint64_t)i + 1, (uint32_t)(rng() % 3 ? rng() % 300 : 1000 + rng() % 2000), clock,
                          store[(size_t)i]));
      CHECK(s.acceptable(*reqs.back()), "request %d refused", i);
      total += reqs.back()->bytes;
      s.enqueue(reqs.back());
    }
    uint64_t max_used = 0;
    for (int it = 0; it < 1000000 && s.busy(); ++it) {
      s.step(clock, done);
      CHECK(ex.pool.used() <= lim.budget_bytes && s.counters().in_use == ex.pool.used(),
            "pool %llu, counted %llu", (unsigned long long)ex.pool.used(), (unsigned long long)s.counters().in_use);
      max_used = std::max(max_used, ex.pool.used());
      clock += 1e-5;
    }
    CHECK(!s.busy() && done.size() == (size_t)N, "did not drain (%zu of %d)", done.size(), N);
    CHECK(total > 10 * lim.budget_bytes && max_used > lim.budget_bytes / 2, "the budget never bound");
    CHECK(ex.pool.used() == 0 && ex.pool.free_blocks() == 1, "device memory not returned");
    uint64_t expect = 1;
    for (const auto& b : ex.launched)
      for (uint64_t t : b) CHECK(t == expect++, "request %llu out of order", (unsigned long long)t);
    std::printf("pool refusals under the budget (fragmentation): %llu\n", (unsigned long long)ex.reserve_refused);
    for (Request* r : reqs) delete r;
  }
  std::printf("OK\n");
  return 0;
}
