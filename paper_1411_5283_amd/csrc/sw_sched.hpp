// sw_sched.hpp -- continuous-batching scheduler of the serving loop, host
// code only (no HIP): the device side is an executor type with
//   uint32_t slots() const;                       concurrent batches
//   bool capacity(uint64_t words, uint64_t docs, uint64_t chars) const;
//   int  launch(Batch&);                          0, or an sw_status for the whole batch
//   bool poll(const Batch&);                      true once the batch has completed
//   int  finish(Batch&);                          results into the requests' buffers; 0 or an sw_status
// so that the same rules run under the HIP executor in the library and under
// a stand-in executor in a CPU test.
//
// Rules: requests are admitted in arrival order while the device bytes of
// every admitted request stay within the budget (the head of the queue is
// never overtaken); every admitted request that is not running is packed,
// in order, into the next batch up to the batch limits; while another batch
// is running, a new one starts only once it holds min_batch_words words, or
// max_batch_docs documents, or its oldest request has waited max_wait_s; a
// request's bytes are released when its batch completes.  A batch that fails
// on the device fails all its requests; a request rejected at intake fails
// alone.
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <unordered_map>
#include <vector>

namespace swsrv {

struct Request {
  uint64_t ticket = 0;
  const uint8_t* chars = nullptr;   // the caller's, valid until completion
  const uint32_t* offsets = nullptr;
  uint32_t n = 0;                   // words
  uint64_t nchars = 0;
  uint64_t bytes = 0;               // device footprint while admitted
  uint32_t* out_perm = nullptr;     // the caller's result buffers
  uint32_t* out_boff = nullptr;
  double arrival = 0, start = 0, done = 0;
  int status = 0;
  bool finished = false;            // set by the serving thread under its lock
  bool claimed = false;             // a caller is waiting for it
};

// The requests that have a ticket and have not been waited for.  A ticket is
// claimed by one waiter; a second claim, or a claim of an unknown ticket, is
// refused (the caller's lock guards every call).
class TicketBook {
 public:
  ~TicketBook() {
    for (auto& kv : live_) delete kv.second;
  }
  void add(Request* r) { live_[r->ticket] = r; }
  // 0 and the request on success; -1 for an unknown or already claimed ticket
  int claim(uint64_t ticket, Request** out) {
    auto it = live_.find(ticket);
    if (it == live_.end() || it->second->claimed) return -1;
    it->second->claimed = true;
    *out = it->second;
    return 0;
  }
  // the claimed request is done with: forgotten and freed
  void release(uint64_t ticket) {
    auto it = live_.find(ticket);
    if (it == live_.end()) return;
    delete it->second;
    live_.erase(it);
  }
  size_t size() const { return live_.size(); }

 private:
  std::unordered_map<uint64_t, Request*> live_;
};

struct Batch {
  std::vector<Request*> reqs;
  uint64_t words = 0, chars = 0;
  int slot = -1;
  double launched = 0;
};

struct Limits {
  uint64_t budget_bytes = 8ull << 30;
  uint64_t max_batch_words = 1u << 22;
  uint64_t max_batch_docs = 256;
  uint64_t max_batch_chars = 32ull << 20;
  uint64_t min_batch_words = 0;
  double max_wait_s = 0.0;
};

struct Counters {
  uint64_t completed = 0, failed = 0, words = 0, batches = 0;
  uint64_t in_use = 0, max_in_use = 0;
};

// Device bytes a request holds while admitted: characters, offsets, the
// output permutation and its bucket-offset row.
inline uint64_t footprint(uint64_t n_words, uint64_t n_chars) {
  return n_chars + 4 * (n_words + 1) + 4 * n_words + 4 * 34;
}

template <class Exec>
class Scheduler {
 public:
  Scheduler(Exec& ex, const Limits& lim) : ex_(ex), lim_(lim) {
    for (uint32_t sl = ex_.slots(); sl > 0; --sl) free_slots_.push_back((int)(sl - 1));
  }

  // A request that can never run (larger than the budget or a batch) is
  // refused here; otherwise it joins the queue.
  bool acceptable(const Request& r) const {
    return r.bytes <= lim_.budget_bytes && r.n <= lim_.max_batch_words && r.nchars <= lim_.max_batch_chars &&
           ex_.capacity(r.n, 1, r.nchars);
  }
  void enqueue(Request* r) { queue_.push_back(r); }

  // One pass: reap finished batches, admit, launch.  `now` is the caller's
  // clock; `done` receives every request that completed or failed.
  void step(double now, std::vector<Request*>& done) {
    reap(now, done);
    admit();
    launch(now, done);
  }

  bool busy() const { return !queue_.empty() || !ready_.empty() || !running_.empty(); }
  bool running() const { return !running_.empty(); }
  const Counters& counters() const { return c_; }

 private:
  void reap(double now, std::vector<Request*>& done) {
    for (size_t i = 0; i < running_.size();) {
      Batch& b = running_[i];
      if (!ex_.poll(b)) {
        ++i;
        continue;
      }
      const int st = ex_.finish(b);
      close(b, st, now, done);
      free_slots_.push_back(b.slot);
      running_.erase(running_.begin() + (long)i);
    }
  }

  void admit() {
    while (!queue_.empty()) {
      Request* r = queue_.front();
      if (c_.in_use + r->bytes > lim_.budget_bytes) break;
      queue_.pop_front();
      c_.in_use += r->bytes;
      c_.max_in_use = std::max(c_.max_in_use, c_.in_use);
      ready_.push_back(r);
    }
  }

  bool worth_launching(double now) const {
    if (running_.empty()) return true;
    uint64_t words = 0;
    for (const Request* r : ready_) words += r->n;
    if (words >= lim_.min_batch_words || ready_.size() >= lim_.max_batch_docs) return true;
    return now - ready_.front()->arrival >= lim_.max_wait_s;
  }

  void launch(double now, std::vector<Request*>& done) {
    while (!ready_.empty() && !free_slots_.empty() && worth_launching(now)) {
      Batch b;
      size_t k = 0;
      for (; k < ready_.size(); ++k) {
        Request* r = ready_[k];
        if (k && (b.words + r->n > lim_.max_batch_words || b.reqs.size() >= lim_.max_batch_docs ||
                  b.chars + r->nchars > lim_.max_batch_chars ||
                  !ex_.capacity(b.words + r->n, b.reqs.size() + 1, b.chars + r->nchars)))
          break;
        b.reqs.push_back(r);
        b.words += r->n;
        b.chars += r->nchars;
      }
      ready_.erase(ready_.begin(), ready_.begin() + (long)k);
      b.slot = free_slots_.back();
      free_slots_.pop_back();
      b.launched = now;
      for (Request* r : b.reqs) r->start = now;
      const int st = ex_.launch(b);
      if (st) {
        close(b, st, now, done);
        free_slots_.push_back(b.slot);
        continue;
      }
      running_.push_back(b);
      ++c_.batches;
    }
  }

  void close(Batch& b, int st, double now, std::vector<Request*>& done) {
    for (Request* r : b.reqs) {
      r->done = now;
      r->status = st;
      c_.in_use -= r->bytes;
      if (st) {
        ++c_.failed;
      } else {
        ++c_.completed;
        c_.words += r->n;
      }
      done.push_back(r);
    }
  }

  Exec& ex_;
  Limits lim_;
  std::deque<Request*> queue_;    // arrived, not admitted
  std::vector<Request*> ready_;   // admitted, not launched
  std::vector<Batch> running_;
  std::vector<int> free_slots_;
  Counters c_;
};

// Intake check of one request on the host: offsets that decrease are
// SW_ERR_INVALID_ARG, a word longer than max_len is SW_ERR_WORD_TOO_LONG;
// returns 0 when the request is well formed.
inline int check_request(const uint32_t* offsets, uint32_t n, uint32_t max_len) {
  if (!offsets) return -1;
  uint32_t bad_order = 0, too_long = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t a = offsets[i], e = offsets[i + 1];
    bad_order |= (uint32_t)(e < a);
    too_long |= (uint32_t)(e - a > max_len);
  }
  return bad_order ? -1 : (too_long ? -2 : 0);
}

}  // namespace swsrv
