// Scheduling core of the serving loop, free of device calls.  Events are
// admitted in arrival order while their result blocks (and, while running,
// a staging block) fit a first-fit pool and an in-flight slot is free; an
// executor starts admitted events and reports when they finish; results
// stay in the pool until released; events still queued can be cancelled.
// The library's executor runs host -> device transfers on HIP streams; the
// host tests plug in an executor that finishes events on host threads.
//
// Executor interface (Exec, with events of type CoreEvent<Payload>):
//   void thread_init();          on the scheduler thread, before its loop
//   uint64_t start(Event& e);    enqueue an admitted event's work (no lock
//                                held; the event is the scheduler's alone
//                                until it is RUNNING); returns bytes moved
//   bool poll(Event& e);         lock held: true once e has finished (e's
//                                status set from what the work reported)
//   void retire(Event& e);       lock held: e leaves the server (released,
//                                cancelled, or the server is destroyed)
#pragma once

#include <stdint.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/relayout.h"
#include "pool.h"

namespace rl {

enum class EvState { QUEUED, ADMITTED, RUNNING, DONE };

template <class Payload>
struct CoreEvent {
  using Clock = std::chrono::steady_clock;
  uint64_t ticket = 0;
  Clock::time_point submitted, done_at;
  std::vector<uint64_t> block_bytes;   // result blocks, in the executor's order (0: no block)
  std::vector<uint64_t> block_off;     // their pool offsets once admitted (UINT64_MAX: none)
  uint64_t stage_bytes = 0;            // staging held while running
  uint64_t stage_off = UINT64_MAX;
  uint64_t bytes = 0;                  // result bytes as the pool places them
  EvState state = EvState::QUEUED;
  uint32_t stream = 0, slot = 0;
  rl_status status = RL_OK;
  Payload p;
};

template <class Exec, class Payload>
class ServeCore {
 public:
  using Event = CoreEvent<Payload>;
  using Clock = std::chrono::steady_clock;

  ServeCore(Exec& exec, uint64_t pool_bytes, uint32_t max_in_flight, uint32_t n_streams)
      : exec_(exec), max_in_flight_(max_in_flight), n_streams_(n_streams) {
    pool_.reset(pool_bytes, 256);
    usable_ = pool_.capacity();
    for (uint32_t k = max_in_flight; k-- > 0;) free_slots_.push_back(k);
  }
  ~ServeCore() { stop(); }
  ServeCore(const ServeCore&) = delete;
  ServeCore& operator=(const ServeCore&) = delete;

  // A block kept for the server's own use (before start); UINT64_MAX if it
  // does not fit.  Events can never use it.
  uint64_t reserve(uint64_t bytes) {
    const uint64_t off = pool_.alloc(bytes);
    if (off != UINT64_MAX) usable_ -= pool_.round(bytes);
    return off;
  }

  void start() { thread_ = std::thread([this] { loop(); }); }

  // Stop the scheduler; events still held are retired.
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stopped_) return;
      stop_ = true;
    }
    cv_work_.notify_all();
    if (thread_.joinable()) thread_.join();
    std::lock_guard<std::mutex> lk(mu_);
    for (auto& kv : events_) exec_.retire(*kv.second);
    events_.clear();
    queue_.clear();
    stopped_ = true;
    cv_done_.notify_all();
  }

  // Queue an event (its block_bytes and stage_bytes set).
  rl_status submit(std::unique_ptr<Event> e, uint64_t* ticket) {
    uint64_t bytes = 0;
    for (uint64_t b : e->block_bytes) bytes += b ? pool_.round(b) : 0;
    e->bytes = bytes;
    const uint64_t need = bytes + (e->stage_bytes ? pool_.round(e->stage_bytes) : 0);
    std::lock_guard<std::mutex> lk(mu_);
    if (stop_) return RL_EINVAL;
    if (need > usable_) return RL_EBUDGET;
    e->ticket = next_ticket_++;
    e->submitted = Clock::now();
    if (!any_) {
      first_submit_ = e->submitted;
      any_ = true;
    }
    *ticket = e->ticket;
    queue_.push_back(e->ticket);
    events_[e->ticket] = std::move(e);
    ++submitted_;
    cv_work_.notify_one();
    return RL_OK;
  }

  // Block until the event is done (timeout_ms < 0: forever), then call
  // fill(event) with the lock held.  RL_EBUSY on timeout, RL_ECANCELED if
  // the event was cancelled (or the server stopped) while waiting,
  // RL_EINVAL for an unknown ticket; else the event's status.
  template <class F>
  rl_status wait(uint64_t ticket, int64_t timeout_ms, F&& fill) {
    std::unique_lock<std::mutex> lk(mu_);
    if (events_.find(ticket) == events_.end()) return RL_EINVAL;
    // the event is looked up again on every wake-up: another thread may
    // cancel or release it meanwhile
    auto ready = [&] {
      auto it = events_.find(ticket);
      return it == events_.end() || it->second->state == EvState::DONE;
    };
    if (timeout_ms < 0) cv_done_.wait(lk, ready);
    else if (!cv_done_.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) return RL_EBUSY;
    auto it = events_.find(ticket);
    if (it == events_.end()) return RL_ECANCELED;
    fill(*it->second);
    return it->second->status;
  }

  // Free a finished event's results.  RL_EBUSY if not finished.
  rl_status release(uint64_t ticket) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = events_.find(ticket);
    if (it == events_.end()) return RL_EINVAL;
    Event& e = *it->second;
    if (e.state != EvState::DONE) return RL_EBUSY;
    for (uint64_t off : e.block_off)
      if (off != UINT64_MAX) pool_.release(off);
    exec_.retire(e);
    events_.erase(it);
    cv_work_.notify_one();
    cv_done_.notify_all();
    return RL_OK;
  }

  // Withdraw an event that has not been admitted yet.  RL_EBUSY once it is
  // admitted (it then runs to completion and is released as usual).
  rl_status cancel(uint64_t ticket) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = events_.find(ticket);
    if (it == events_.end()) return RL_EINVAL;
    if (it->second->state != EvState::QUEUED) return RL_EBUSY;
    for (auto q = queue_.begin(); q != queue_.end(); ++q)
      if (*q == ticket) {
        queue_.erase(q);
        break;
      }
    exec_.retire(*it->second);
    events_.erase(it);
    ++cancelled_;
    cv_work_.notify_one();   // the next event may now be at the head
    cv_done_.notify_all();   // waiters on it return RL_ECANCELED
    return RL_OK;
  }

  void stats(rl_server_stats* out) {
    std::lock_guard<std::mutex> lk(mu_);
    out->completed = completed_;
    out->submitted = submitted_;
    out->p50_ms = percentile(lat_ms_, 50);
    out->p99_ms = percentile(lat_ms_, 99);
    out->max_ms = percentile(lat_ms_, 100);
    out->events_per_s = 0.0;
    if (completed_ && any_) {
      const double sec = std::chrono::duration<double>(last_done_ - first_submit_).count();
      out->events_per_s = sec > 0 ? (double)completed_ / sec : 0.0;
    }
    out->peak_bytes = peak_;
    out->h2d_bytes = moved_;
  }

  uint64_t cancelled() {
    std::lock_guard<std::mutex> lk(mu_);
    return cancelled_;
  }
  uint64_t usable() const { return usable_; }
  // Pool bytes held right now (results, staging and reserved blocks).
  uint64_t in_use() {
    std::lock_guard<std::mutex> lk(mu_);
    return pool_.in_use();
  }

 private:
  // Queued events in arrival order while their blocks fit and a slot is
  // free (lock held).  The head of the queue waits for releases: later
  // events never overtake it.
  std::vector<Event*> admit() {
    std::vector<Event*> out;
    while (!queue_.empty() && running_ < max_in_flight_ && !free_slots_.empty()) {
      Event& e = *events_[queue_.front()];
      std::vector<uint64_t> sizes;
      for (uint64_t b : e.block_bytes)
        if (b) sizes.push_back(b);
      if (e.stage_bytes) sizes.push_back(e.stage_bytes);
      if (!pool_.fits(sizes)) break;
      e.block_off.clear();
      for (uint64_t b : e.block_bytes) e.block_off.push_back(b ? pool_.alloc(b) : UINT64_MAX);
      e.stage_off = e.stage_bytes ? pool_.alloc(e.stage_bytes) : UINT64_MAX;
      e.slot = free_slots_.back();
      free_slots_.pop_back();
      peak_ = std::max<uint64_t>(peak_, pool_.in_use());
      queue_.pop_front();
      e.stream = next_stream_;
      next_stream_ = (next_stream_ + 1) % n_streams_;
      e.state = EvState::ADMITTED;
      ++running_;
      out.push_back(&e);
    }
    return out;
  }

  // Finished events (lock held); true if any.
  bool reap() {
    bool any = false;
    for (auto& kv : events_) {
      Event& e = *kv.second;
      if (e.state != EvState::RUNNING || !exec_.poll(e)) continue;
      free_slots_.push_back(e.slot);
      if (e.stage_off != UINT64_MAX) {
        pool_.release(e.stage_off);
        e.stage_off = UINT64_MAX;
      }
      e.state = EvState::DONE;
      e.done_at = Clock::now();
      lat_ms_.push_back(std::chrono::duration<double, std::milli>(e.done_at - e.submitted).count());
      ++completed_;
      last_done_ = e.done_at;
      --running_;
      any = true;
    }
    return any;
  }

  void loop() {
    exec_.thread_init();
    std::unique_lock<std::mutex> lk(mu_);
    while (!stop_) {
      const bool finished = reap();
      std::vector<Event*> admitted = admit();
      if (finished) cv_done_.notify_all();
      if (!admitted.empty()) {
        lk.unlock();
        uint64_t moved = 0;
        for (Event* e : admitted) moved += exec_.start(*e);
        lk.lock();
        moved_ += moved;
        for (Event* e : admitted) e->state = EvState::RUNNING;
        continue;
      }
      if (running_ == 0 && (queue_.empty() || !finished)) {
        cv_work_.wait_for(lk, std::chrono::microseconds(2000));
      } else {
        // poll completions at a short period while work is running
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(10));
        lk.lock();
      }
    }
    // events admitted but not yet marked running are the scheduler's own;
    // let their work finish before the executor retires them
    for (auto& kv : events_)
      if (kv.second->state == EvState::ADMITTED) kv.second->state = EvState::RUNNING;
  }

  Exec& exec_;
  const uint32_t max_in_flight_, n_streams_;
  SlabAllocator pool_;
  uint64_t usable_ = 0;
  std::vector<uint32_t> free_slots_;
  std::mutex mu_;
  std::condition_variable cv_done_, cv_work_;
  std::deque<uint64_t> queue_;
  std::map<uint64_t, std::unique_ptr<Event>> events_;
  uint64_t next_ticket_ = 1;
  uint32_t running_ = 0, next_stream_ = 0;
  bool stop_ = false, stopped_ = false;
  std::thread thread_;
  std::vector<double> lat_ms_;
  uint64_t submitted_ = 0, completed_ = 0, cancelled_ = 0, peak_ = 0, moved_ = 0;
  Clock::time_point first_submit_, last_done_;
  bool any_ = false;
};

}  // namespace rl
