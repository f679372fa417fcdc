// sw_sched.hpp -- continuous-batching scheduler of the serving loop, host
// code only (no HIP): the device side is an executor type with
//   uint32_t slots() const;                       concurrent batches
//   bool capacity(uint64_t words, uint64_t docs, uint64_t chars) const;
//   bool reserve(Request&);                       device memory for an admitted request
//                                                 (its upload starts); false: none free yet
//   bool uploaded(const Request&);                its upload has been issued
//   void release(Request&);                       its device memory is free again
//   int  launch(Batch&);                          0, or an sw_status for the whole batch
//   bool poll(const Batch&);                      true once the batch has completed
//   int  finish(Batch&);                          results into the requests' buffers; 0 or an sw_status
// so that the same rules run under the HIP executor in the library and under
// a stand-in executor in a CPU test.
//
// Rules: requests are admitted in arrival order while the device bytes of
// every admitted request stay within the budget and the executor finds them
// a block of device memory (the head of the queue is never overtaken); an
// admitted request is uploaded into its block at once, so queued requests
// wait on the device; every admitted request whose upload has been issued
// and that is not running is packed, in order, into the next batch up to the
// batch limits; while another batch is running, a new one starts only once
// it holds min_batch_words words, or max_batch_docs documents, or its oldest
// request has waited max_wait_s; a request's device memory is released when
// its batch completes.  A batch that fails on the device fails all its
// requests; a request rejected at intake fails alone.
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
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
  // the executor's: where the request lies in device memory, and its upload
  uint64_t dev_off = 0;
  std::atomic<bool> uploaded{false};
  uint64_t upload_seq = 0;          // issue order of the upload on its stream (valid once uploaded)
  int upload_stream = 0;            // which upload stream carried it
  int upload_error = 0;
  void* upload_event = nullptr;
};

// Device memory of the admitted requests: one region of `capacity` bytes
// handed out first fit in 256-byte units; a freed block merges with its free
// neighbours.  Bookkeeping only (offsets into the region).
class DevicePool {
 public:
  static constexpr uint64_t kAlign = 256;
  static uint64_t rounded(uint64_t bytes) { return (std::max<uint64_t>(bytes, 1) + kAlign - 1) / kAlign * kAlign; }

  explicit DevicePool(uint64_t capacity = 0) { reset(capacity); }
  void reset(uint64_t capacity) {
    cap_ = capacity / kAlign * kAlign;
    used_ = 0;
    free_.clear();
    if (cap_) free_[0] = cap_;
  }
  // the lowest free block that holds `bytes` (rounded up), or false
  bool alloc(uint64_t bytes, uint64_t* off) {
    const uint64_t b = rounded(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < b) continue;
      *off = it->first;
      const uint64_t at = it->first + b, rest = it->second - b;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += b;
      return true;
    }
    return false;
  }
  // a block handed out by alloc(bytes), back to the free list
  void release(uint64_t off, uint64_t bytes) {
    const uint64_t b = rounded(bytes);
    used_ -= b;
    uint64_t start = off, len = b;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && next->first == off + b) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
  }
  uint64_t capacity() const { return cap_; }
  uint64_t used() const { return used_; }
  size_t free_blocks() const { return free_.size(); }
  uint64_t largest_free() const {
    uint64_t m = 0;
    for (const auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }

 private:
  std::map<uint64_t, uint64_t> free_;   // offset -> length of every free block
  uint64_t cap_ = 0, used_ = 0;
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

// Device bytes a request holds from admission until its batch completes:
// its characters, then its n+1 offsets, each part in whole 256-byte units
// (the results go to the batch slot's own buffers).
inline uint64_t footprint(uint64_t n_words, uint64_t n_chars) {
  return DevicePool::rounded(n_chars) + DevicePool::rounded(4 * (n_words + 1));
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
      if (!ex_.reserve(*r)) break;   // no free block large enough until a batch completes
      queue_.pop_front();
      c_.in_use += r->bytes;
      c_.max_in_use = std::max(c_.max_in_use, c_.in_use);
      ready_.push_back(r);
    }
  }

  // the first `up` ready requests (those uploaded) make a batch worth starting
  bool worth_launching(double now, size_t up) const {
    if (running_.empty()) return true;
    uint64_t words = 0;
    for (size_t i = 0; i < up; ++i) words += ready_[i]->n;
    if (words >= lim_.min_batch_words || up >= lim_.max_batch_docs) return true;
    return now - ready_.front()->arrival >= lim_.max_wait_s;
  }

  void launch(double now, std::vector<Request*>& done) {
    size_t up = 0;   // ready requests, in order, whose upload has been issued
    while (up < ready_.size() && ex_.uploaded(*ready_[up])) ++up;
    while (up > 0 && !free_slots_.empty() && worth_launching(now, up)) {
      Batch b;
      size_t k = 0;
      for (; k < up; ++k) {
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
      up -= k;
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
      ex_.release(*r);
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
