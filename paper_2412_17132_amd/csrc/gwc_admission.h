// Admission of requests to the device by predicted footprint (host C++ only,
// no HIP): the request server's scheduling policy, kept apart from execution
// so that it can be exercised with a fake executor.
//
// Policy: requests are served in arrival order (FIFO).  A free worker takes
// the oldest queued request as soon as its footprint fits in the budget next
// to the footprints of the requests already running; a later, smaller request
// never overtakes an earlier one.  A request larger than the whole budget is
// refused at submission.  A finished request may leave part of its footprint
// allocated (device memory it built for a resident system): that part stays
// counted as in use ("kept") for the life of the policy, and a queued request
// that can then never fit is handed out as refused instead of blocking the
// queue.  After stop() the workers drain the queue and then receive nullptr.
#pragma once

#include <algorithm>
#include <condition_variable>
#include <cstddef>
#include <deque>
#include <mutex>

namespace gwc {

template <class Item>
class Admission {
 public:
  explicit Admission(size_t budget) : budget_(budget) {}

  size_t budget() const { return budget_; }

  // Queues `item` with its footprint; false (not queued) when it exceeds the
  // budget left beside the kept bytes.
  bool submit(Item *item, size_t footprint) {
    {
      std::lock_guard<std::mutex> lock(mu_);
      if (footprint > budget_ - kept_) return false;
      queue_.push_back(Entry{item, footprint});
    }
    cv_.notify_all();
    return true;
  }

  // Blocks until the oldest request fits (returns it and its footprint, now
  // counted as in use) or the server stops with an empty queue (nullptr).
  // When the oldest request can never fit beside the kept bytes it is
  // returned at once with *refused = true (not counted as in use: the caller
  // fails it and does not release it).  `ticket`, when given, receives the
  // request's admission number (0, 1, ... in the order requests are handed out).
  Item *acquire(size_t &footprint, long long *ticket = nullptr, bool *refused = nullptr) {
    std::unique_lock<std::mutex> lock(mu_);
    cv_.wait(lock, [&] { return fits_locked() || never_fits_locked() || (stop_ && queue_.empty()); });
    if (queue_.empty()) return nullptr;
    const Entry e = queue_.front();
    queue_.pop_front();
    footprint = e.footprint;
    if (ticket) *ticket = admitted_;
    admitted_ += 1;
    if (never_fits(e.footprint)) {
      completed_ += 1;
      refused_ += 1;
      if (refused) *refused = true;
      lock.unlock();
      cv_.notify_all();
      return e.item;
    }
    if (refused) *refused = false;
    in_use_ += e.footprint;
    peak_in_use_ = std::max(peak_in_use_, in_use_);
    active_ += 1;
    peak_active_ = std::max(peak_active_, active_);
    return e.item;
  }

  // Returns a finished request's footprint to the budget, except `keep`
  // bytes of it that stay allocated (kept, and counted, from now on).
  void release(size_t footprint, size_t keep = 0) {
    {
      std::lock_guard<std::mutex> lock(mu_);
      keep = std::min(keep, footprint);
      in_use_ -= footprint - keep;
      kept_ += keep;
      active_ -= 1;
      completed_ += 1;
    }
    cv_.notify_all();
  }

  void stop() {
    {
      std::lock_guard<std::mutex> lock(mu_);
      stop_ = true;
    }
    cv_.notify_all();
  }

  struct Stats {
    size_t queued, in_use, peak_in_use, kept;
    int active, peak_active;
    long long completed, refused;
  };
  Stats stats() const {
    std::lock_guard<std::mutex> lock(mu_);
    return Stats{queue_.size(), in_use_, peak_in_use_, kept_, active_, peak_active_, completed_, refused_};
  }

 private:
  struct Entry {
    Item *item;
    size_t footprint;
  };
  bool fits_locked() const {
    return !queue_.empty() && in_use_ + queue_.front().footprint <= budget_;
  }
  bool never_fits(size_t footprint) const { return footprint > budget_ - kept_; }
  bool never_fits_locked() const { return !queue_.empty() && never_fits(queue_.front().footprint); }

  const size_t budget_;
  mutable std::mutex mu_;
  std::condition_variable cv_;
  std::deque<Entry> queue_;
  size_t in_use_ = 0, peak_in_use_ = 0, kept_ = 0;  // kept_ is part of in_use_
  int active_ = 0, peak_active_ = 0;
  long long completed_ = 0, admitted_ = 0, refused_ = 0;
  bool stop_ = false;
};

}  // namespace gwc
