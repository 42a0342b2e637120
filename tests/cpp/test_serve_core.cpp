// Host-side checks of the serving core with a fake executor (no device):
// FIFO admission by budget and slots, a consumer that holds its results,
// head-of-line waiting, cancellation (also of an event someone waits on),
// timeouts, per-event statuses, staging held only while running, shutdown
// with events outstanding, and a multi-threaded stress run.  Built plain,
// with ThreadSanitizer and with AddressSanitizer by the test driver.
#if defined(__SANITIZE_THREAD__)
// GCC 11's ThreadSanitizer does not intercept pthread_cond_clockwait, which
// libstdc++ uses for steady-clock waits, and then reports races on data the
// waiting mutex guards; without it the waits go through
// pthread_cond_timedwait, which it does intercept.
#include <bits/c++config.h>
#undef _GLIBCXX_USE_PTHREAD_COND_CLOCKWAIT
#endif
#include <assert.h>
#include <stdio.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "../../paper_2511_04853_amd/csrc/serve_core.h"

using namespace std::chrono_literals;
using Clock = std::chrono::steady_clock;

#define CHECK(c)                                                    \
  do {                                                              \
    if (!(c)) {                                                     \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      abort();                                                      \
    }                                                               \
  } while (0)

struct FakePayload {
  int tag = 0;
};
using Event = rl::CoreEvent<FakePayload>;

// Events finish when the test allows them (finish()), or, in automatic
// mode, a random short time after they start (a worker thread).
struct Fake {
  std::mutex m;
  std::condition_variable cv;
  std::vector<uint64_t> started;
  std::map<uint64_t, rl_status> finished;
  std::set<uint64_t> retired;
  bool automatic = false, quit = false;
  std::deque<std::pair<uint64_t, Clock::time_point>> pending;
  std::thread worker;
  std::mt19937_64 rng{11};

  void thread_init() {}
  uint64_t start(Event& e) {
    std::lock_guard<std::mutex> lk(m);
    started.push_back(e.ticket);
    if (automatic) {
      pending.emplace_back(e.ticket, Clock::now() + std::chrono::microseconds(rng() % 300));
      cv.notify_one();
    }
    return 1;
  }
  bool poll(Event& e) {
    std::lock_guard<std::mutex> lk(m);
    auto it = finished.find(e.ticket);
    if (it == finished.end()) return false;
    e.status = it->second;
    return true;
  }
  void retire(Event& e) {
    std::lock_guard<std::mutex> lk(m);
    retired.insert(e.ticket);
  }
  void finish(uint64_t t, rl_status st = RL_OK) {
    std::lock_guard<std::mutex> lk(m);
    finished[t] = st;
  }
  std::vector<uint64_t> started_now() {
    std::lock_guard<std::mutex> lk(m);
    return started;
  }
  void run_automatic() {
    automatic = true;
    worker = std::thread([this] {
      std::unique_lock<std::mutex> lk(m);
      while (!quit) {
        const auto now = Clock::now();
        while (!pending.empty() && pending.front().second <= now) {
          finished[pending.front().first] = RL_OK;
          pending.pop_front();
        }
        cv.wait_for(lk, 50us);
      }
    });
  }
  void stop() {
    {
      std::lock_guard<std::mutex> lk(m);
      quit = true;
    }
    cv.notify_all();
    if (worker.joinable()) worker.join();
  }
};

using Core = rl::ServeCore<Fake, FakePayload>;

static std::unique_ptr<Event> event(std::vector<uint64_t> blocks, uint64_t stage = 0) {
  auto e = std::make_unique<Event>();
  e->block_bytes = std::move(blocks);
  e->stage_bytes = stage;
  return e;
}

// Wait (bounded) until the fake has started `k` events.
static std::vector<uint64_t> started(Fake& f, size_t k) {
  for (int i = 0; i < 4000; ++i) {
    auto s = f.started_now();
    if (s.size() >= k) return s;
    std::this_thread::sleep_for(500us);
  }
  return f.started_now();
}

static void settle() { std::this_thread::sleep_for(20ms); }

static void admission_budget_release_cancel() {
  Fake f;
  Core c(f, 10240, 8, 2);
  c.start();
  uint64_t t[6];
  for (int k = 0; k < 5; ++k) CHECK(c.submit(event({1000, 2000, 0}), &t[k]) == RL_OK);   // 3 KiB each
  auto s = started(f, 3);
  settle();
  s = f.started_now();
  CHECK(s.size() == 3 && s[0] == t[0] && s[1] == t[1] && s[2] == t[2]);   // FIFO, 3 fit
  CHECK(c.in_use() == 3 * 3072);
  CHECK(c.wait(t[0], 5, [](Event&) {}) == RL_EBUSY);   // not finished: timeout
  for (int k = 0; k < 3; ++k) f.finish(t[k]);
  for (int k = 0; k < 3; ++k) CHECK(c.wait(t[k], -1, [](Event& e) { CHECK(e.state == rl::EvState::DONE); }) == RL_OK);
  settle();
  CHECK(f.started_now().size() == 3);   // results held: the fourth still waits
  CHECK(c.cancel(t[0]) == RL_EBUSY);    // done events are released, not cancelled
  CHECK(c.release(t[3]) == RL_EBUSY);   // queued: nothing to release
  CHECK(c.release(t[0]) == RL_OK);
  s = started(f, 4);
  CHECK(s.size() == 4 && s[3] == t[3]);
  settle();
  CHECK(f.started_now().size() == 4);   // one release makes room for one event
  CHECK(c.cancel(t[4]) == RL_OK);       // still queued
  CHECK(c.wait(t[4], 0, [](Event&) {}) == RL_EINVAL);
  CHECK(c.cancel(t[4]) == RL_EINVAL);
  CHECK(c.cancel(t[3]) == RL_EBUSY);    // admitted: runs to completion
  f.finish(t[3], RL_EBOUNDS);
  CHECK(c.wait(t[3], -1, [](Event&) {}) == RL_EBOUNDS);   // its own status
  CHECK(c.wait(t[1], -1, [](Event&) {}) == RL_OK);        // others unaffected
  CHECK(c.release(t[1]) == RL_OK && c.release(t[2]) == RL_OK && c.release(t[3]) == RL_OK);
  CHECK(c.in_use() == 0);
  CHECK(c.submit(event({10240 + 1}), &t[5]) == RL_EBUDGET);
  CHECK(c.cancelled() == 1);
  rl_server_stats st;
  c.stats(&st);
  CHECK(st.submitted == 5 && st.completed == 4 && st.peak_bytes == 3 * 3072);
  c.stop();
  {
    std::lock_guard<std::mutex> lk(f.m);
    CHECK(f.retired.size() == 5);   // four released, one cancelled
  }
}

static void head_of_line_and_cancelled_waiter() {
  Fake f;
  Core c(f, 8192, 8, 1);
  c.start();
  uint64_t a, big, s1, s2;
  CHECK(c.submit(event({4096}), &a) == RL_OK);
  started(f, 1);
  CHECK(c.submit(event({6144}), &big) == RL_OK);   // does not fit while a is held
  CHECK(c.submit(event({1024}), &s1) == RL_OK);    // would fit, but must not overtake
  CHECK(c.submit(event({1024}), &s2) == RL_OK);
  settle();
  CHECK(f.started_now().size() == 1);
  std::atomic<int> got{-1};
  std::thread waiter([&] { got = c.wait(big, -1, [](Event&) {}); });
  settle();
  CHECK(c.cancel(big) == RL_OK);
  waiter.join();
  CHECK(got == RL_ECANCELED);
  auto s = started(f, 3);
  CHECK(s.size() == 3 && s[1] == s1 && s[2] == s2);
  // a waiter on an event that is released by another thread returns
  f.finish(a);
  CHECK(c.wait(a, -1, [](Event&) {}) == RL_OK);
  CHECK(c.release(a) == RL_OK);
  CHECK(c.wait(a, 0, [](Event&) {}) == RL_EINVAL);
  c.stop();
  std::lock_guard<std::mutex> lk(f.m);
  CHECK(f.retired.count(big) && f.retired.count(s1) && f.retired.count(s2));
}

static void slots_staging_and_reserve() {
  Fake f;
  Core c(f, 1 << 20, 2, 2);
  const uint64_t r = c.reserve(256 << 10);   // the server's own block
  CHECK(r != UINT64_MAX && c.usable() == (1 << 20) - (256 << 10));
  c.start();
  uint64_t t[4];
  for (int k = 0; k < 4; ++k) CHECK(c.submit(event({1000}, 100000), &t[k]) == RL_OK);
  started(f, 2);
  settle();
  CHECK(f.started_now().size() == 2);   // two slots
  const uint64_t held = c.in_use();
  CHECK(held == (256 << 10) + 2 * (1024 + 100096));
  f.finish(t[0]);
  CHECK(c.wait(t[0], -1, [](Event&) {}) == RL_OK);
  started(f, 3);
  settle();
  // t[0]'s staging went back at completion, its result stays; t[2] took a slot
  CHECK(c.in_use() == (256 << 10) + 3 * 1024 + 2 * 100096);
  uint64_t x;
  CHECK(c.submit(event({(768 << 10) + 1}), &x) == RL_EBUDGET);   // beyond what events may use
  c.stop();   // events running and queued are retired
  std::lock_guard<std::mutex> lk(f.m);
  CHECK(f.retired.size() == 4);
}

static void stress() {
  Fake f;
  f.run_automatic();
  const uint64_t cap = 256 << 10;
  Core c(f, cap, 16, 4);
  c.start();
  std::atomic<uint64_t> ok{0}, cancelled{0}, busy_cancels{0};
  std::vector<std::thread> th;
  for (int w = 0; w < 4; ++w)
    th.emplace_back([&, w] {
      std::mt19937_64 rng(100 + w);
      std::vector<uint64_t> mine;
      for (int k = 0; k < 250; ++k) {
        uint64_t t;
        const uint64_t sz = 1 + rng() % (24 << 10);
        const uint64_t extra = rng() % 2 ? 4096 : 0, stage = rng() % 4 ? 0 : 8192;
        CHECK(c.submit(event({sz, extra}, stage), &t) == RL_OK);
        mine.push_back(t);
        if (rng() % 5 == 0) {
          const rl_status st = c.cancel(t);
          CHECK(st == RL_OK || st == RL_EBUSY);
          if (st == RL_OK) {
            ++cancelled;
            mine.pop_back();
          } else {
            ++busy_cancels;
          }
        }
        // keep at most a few results per thread: a consumer that releases
        while (mine.size() > 3) {
          CHECK(c.wait(mine.front(), -1, [](Event&) {}) == RL_OK);
          CHECK(c.release(mine.front()) == RL_OK);
          mine.erase(mine.begin());
          ++ok;
        }
      }
      for (auto t : mine) {
        CHECK(c.wait(t, -1, [](Event&) {}) == RL_OK);
        CHECK(c.release(t) == RL_OK);
        ++ok;
      }
    });
  std::thread stats_reader([&] {
    for (int k = 0; k < 200; ++k) {
      rl_server_stats s;
      c.stats(&s);
      CHECK(s.peak_bytes <= cap);
      CHECK(c.in_use() <= cap);
      std::this_thread::sleep_for(200us);
    }
  });
  for (auto& t : th) t.join();
  stats_reader.join();
  CHECK(ok + cancelled == 1000);
  CHECK(c.cancelled() == cancelled);
  CHECK(c.in_use() == 0);
  // admission never reorders: started tickets increase
  auto s = f.started_now();
  for (size_t k = 1; k < s.size(); ++k) CHECK(s[k] > s[k - 1]);
  CHECK(s.size() == ok);
  c.stop();
  f.stop();
  printf("stress: %llu served, %llu cancelled, %llu cancels refused (admitted)\n", (unsigned long long)ok.load(),
         (unsigned long long)cancelled.load(), (unsigned long long)busy_cancels.load());
}

int main() {
  admission_budget_release_cancel();
  head_of_line_and_cancelled_waiter();
  slots_staging_and_reserve();
  stress();
  printf("serve core ok\n");
  return 0;
}
