// Serving loop: events (one or more collections each, in pinned host
// memory) arrive at any time; a scheduler thread admits them in arrival
// order while their result bytes fit a device-memory budget and an
// in-flight slot is free, converts them with host -> device transfers on
// the server's streams (events overlap on the device), and keeps the
// converted collections resident in a pool carved from one device slab
// until the client releases them.  Completion is observed by polling
// events; latency is submit -> last conversion done.
#include <math.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "plan.h"
#include "pool.h"
#include "rl_internal.h"

using namespace rl;

namespace {

using Clock = std::chrono::steady_clock;

enum class EvState { QUEUED, ADMITTED, RUNNING, DONE, RELEASED };

struct ItemCopy {
  const rl_layout* src_layout;
  const rl_layout* dst_layout;
  uint64_t n, src_cap;
  std::vector<void*> src_bufs;
  std::vector<uint64_t> src_mcap;
  std::vector<uint64_t> dst_mcap;      // member capacity of the result
  std::vector<uint64_t> dst_bytes;     // bytes of each result buffer
  std::vector<uint64_t> dst_offsets;   // pool offsets of the result buffers
  std::vector<void*> dst_bufs;
};

struct Event {
  uint64_t ticket;
  Clock::time_point submitted, done_at;
  std::vector<ItemCopy> items;
  uint64_t bytes = 0;
  EvState state = EvState::QUEUED;
  hipEvent_t done = nullptr;
  uint32_t stream = 0;
  uint32_t slot = 0;                  // in-flight slot (status word) while admitted
  uint64_t stage_need = 0;            // device staging bytes while converting
  uint64_t stage_off = UINT64_MAX;    // pool offset of the staging block
  rl_status status = RL_OK;
  // result views handed to the client
  std::vector<void* const*> buf_ptrs;
  std::vector<uint64_t> mcaps;
};

}  // namespace

// Look-back bytes per server stream: single-pass jagged conversions of up
// to 32,768 tiles; larger collections take the multi-kernel path.
constexpr uint64_t kServerLookbackBytes = 256 << 10;

struct rl_server {
  rl_server_opts opts{};
  int device = 0;
  std::vector<hipStream_t> streams;
  // per stream: look-back state of single-pass jagged conversions, carved
  // from the slab at creation and zeroed once (reused in stream order)
  std::vector<uint64_t*> lookback;
  uint8_t* slab = nullptr;
  SlabAllocator pool;
  // one pinned word per in-flight slot: the device status flags of the
  // event in that slot, handed over in stream order when it completes
  uint32_t* slot_words = nullptr;
  uint32_t* slot_words_dev = nullptr;
  std::vector<uint32_t> free_slots;
  std::mutex mu;
  std::condition_variable cv_done;   // events finished
  std::condition_variable cv_work;   // new submissions or releases
  std::deque<uint64_t> queue;
  std::map<uint64_t, std::unique_ptr<Event>> events;
  uint64_t next_ticket = 1;
  uint32_t running = 0;
  uint32_t next_stream = 0;
  bool stop = false;
  std::thread scheduler;
  // statistics
  std::vector<double> lat_ms;
  uint64_t submitted = 0, completed = 0, peak = 0, h2d_bytes = 0;
  Clock::time_point first_submit, last_done;
  bool any = false;
};

namespace {

// Result bytes of an event as the pool places them (buffers of 0 bytes
// take no block).
uint64_t event_bytes(Event& e) {
  uint64_t total = 0;
  for (auto& it : e.items)
    for (auto b : it.dst_bytes) total += (b + 255) / 256 * 256;
  return total;
}

// Take queued events in arrival order while their results fit the pool and
// a slot is free, placing their result buffers (caller holds mu).
std::vector<Event*> admit(rl_server* s) {
  std::vector<Event*> out;
  while (!s->queue.empty() && s->running < s->opts.max_in_flight && !s->free_slots.empty()) {
    Event& e = *s->events[s->queue.front()];
    std::vector<uint64_t> sizes;
    for (auto& it : e.items)
      for (auto b : it.dst_bytes)
        if (b) sizes.push_back(b);
    if (e.stage_need) sizes.push_back(e.stage_need);
    if (!s->pool.fits(sizes)) break;   // head of line waits for releases
    for (auto& it : e.items) {
      it.dst_offsets.clear();
      it.dst_bufs.clear();
      for (auto b : it.dst_bytes) {
        const uint64_t off = b ? s->pool.alloc(b) : UINT64_MAX;
        it.dst_offsets.push_back(off);
        it.dst_bufs.push_back(b ? s->slab + off : nullptr);
      }
    }
    e.stage_off = e.stage_need ? s->pool.alloc(e.stage_need) : UINT64_MAX;
    e.slot = s->free_slots.back();
    s->free_slots.pop_back();
    s->slot_words[e.slot] = 0;
    s->peak = std::max<uint64_t>(s->peak, s->pool.in_use());
    s->queue.pop_front();
    e.stream = s->next_stream;
    s->next_stream = (s->next_stream + 1) % (uint32_t)s->streams.size();
    e.state = EvState::ADMITTED;
    ++s->running;
    out.push_back(&e);
  }
  return out;
}

// Enqueue the transfers of admitted events (without the lock: an admitted
// event is touched only by the scheduler thread until it is RUNNING).
uint64_t launch(rl_server* s, Event& e) {
  uint64_t h2d = 0;
  hipStream_t st = s->streams[e.stream];
  uint8_t* stage = e.stage_need ? s->slab + e.stage_off : nullptr;
  for (auto& it : e.items) {
    rl_view sv{it.src_layout, it.src_cap, it.src_mcap.empty() ? nullptr : it.src_mcap.data(), it.src_bufs.data()};
    rl_view dv{it.dst_layout, it.n, it.dst_mcap.empty() ? nullptr : it.dst_mcap.data(), it.dst_bufs.data()};
    rl_xfer_opts o{RL_XFER_AUTO};
    // items of an event run one after another on its stream, so they share
    // the event's staging block
    const rl_status r = transfer_impl(&sv, &dv, it.n, st, &o, stage, e.stage_need, s->lookback[e.stream],
                                      kServerLookbackBytes);
    if (r != RL_OK && e.status == RL_OK) e.status = r;
    std::vector<uint64_t> hb(layout_n_buffers(it.src_layout));
    layout_buffer_bytes(it.src_layout, it.n, it.src_mcap.empty() ? nullptr : it.src_mcap.data(), hb.data());
    for (auto b : hb) h2d += b;
  }
  // the stream's device status flags (this event's alone: the stream runs
  // events in order and each hand-over clears them) go to the slot's word
  uint32_t* word = stream_status(st);
  if (!word || launch_take_status(word, s->slot_words_dev + e.slot, st) != hipSuccess) {
    if (e.status == RL_OK) e.status = RL_EHIP;
  }
  if (hipEventRecord(e.done, st) != hipSuccess && e.status == RL_OK) e.status = RL_EHIP;
  return h2d;
}

// Mark finished events (caller holds mu); true if any finished.
bool reap(rl_server* s) {
  bool any = false;
  for (auto& kv : s->events) {
    Event& e = *kv.second;
    if (e.state != EvState::RUNNING) continue;
    const hipError_t q = hipEventQuery(e.done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess && e.status == RL_OK) e.status = RL_EHIP;
    if (e.status == RL_OK) e.status = status_of_flags(((volatile uint32_t*)s->slot_words)[e.slot]);
    s->free_slots.push_back(e.slot);
    if (e.stage_off != UINT64_MAX) {
      s->pool.release(e.stage_off);
      e.stage_off = UINT64_MAX;
    }
    e.state = EvState::DONE;
    e.done_at = Clock::now();
    const double ms = std::chrono::duration<double, std::milli>(e.done_at - e.submitted).count();
    s->lat_ms.push_back(ms);
    ++s->completed;
    s->last_done = e.done_at;
    --s->running;
    any = true;
  }
  return any;
}

void scheduler_loop(rl_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    const bool finished = reap(s);
    std::vector<Event*> admitted = admit(s);
    if (finished) s->cv_done.notify_all();
    if (!admitted.empty()) {
      lk.unlock();
      uint64_t h2d = 0;
      for (Event* e : admitted) h2d += launch(s, *e);
      lk.lock();
      s->h2d_bytes += h2d;
      for (Event* e : admitted) e->state = EvState::RUNNING;
      continue;
    }
    if (s->running == 0 && (s->queue.empty() || !finished))
      s->cv_work.wait_for(lk, std::chrono::microseconds(s->running ? 20 : 2000));
    else {
      // poll completions at a short period while work is on the device
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(10));
      lk.lock();
    }
  }
}

}  // namespace

extern "C" rl_status rl_server_create(const rl_server_opts* opts, rl_server** out) {
  if (!opts || !out) return fail(RL_EINVAL, "rl_server_create: NULL argument");
  *out = nullptr;
  if (!opts->budget_bytes || !opts->max_in_flight || !opts->n_streams || opts->n_streams > 64 ||
      opts->max_in_flight > 65536)
    return fail(RL_EINVAL, "budget, 1..65536 slots and 1..64 streams are required");
  auto s = std::make_unique<rl_server>();
  s->opts = *opts;
  hipError_t e = hipGetDevice(&s->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if ((e = hipMalloc(&s->slab, opts->budget_bytes)) != hipSuccess)
    return fail(RL_ENOMEM, "serving pool of %llu bytes: %s", (unsigned long long)opts->budget_bytes,
                hipGetErrorString(e));
  s->pool.reset(opts->budget_bytes, 256);
  if ((e = hipHostMalloc((void**)&s->slot_words, opts->max_in_flight * sizeof(uint32_t), hipHostMallocDefault)) !=
      hipSuccess) {
    (void)hipFree(s->slab);
    return hip_fail(e, "hipHostMalloc(status words)");
  }
  if ((e = hipHostGetDevicePointer((void**)&s->slot_words_dev, s->slot_words, 0)) != hipSuccess) {
    (void)hipHostFree(s->slot_words);
    (void)hipFree(s->slab);
    return hip_fail(e, "hipHostGetDevicePointer(status words)");
  }
  for (uint32_t k = opts->max_in_flight; k-- > 0;) s->free_slots.push_back(k);
  for (uint32_t k = 0; k < opts->n_streams; ++k) {
    hipStream_t st;
    if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) {
      for (auto x : s->streams) (void)hipStreamDestroy(x);
      (void)hipHostFree(s->slot_words);
      (void)hipFree(s->slab);
      return hip_fail(e, "hipStreamCreate");
    }
    s->streams.push_back(st);
  }
  for (uint32_t k = 0; k < opts->n_streams; ++k) {
    const uint64_t off = s->pool.alloc(kServerLookbackBytes);
    uint64_t* lb = off == UINT64_MAX ? nullptr : reinterpret_cast<uint64_t*>(s->slab + off);
    if (lb && (e = launch_zero(lb, kServerLookbackBytes, s->streams[k])) != hipSuccess) lb = nullptr;
    s->lookback.push_back(lb);   // null (budget too small): the library's per-stream buffer
  }
  for (auto x : s->streams)
    if ((e = hipStreamSynchronize(x)) != hipSuccess) {
      for (auto y : s->streams) (void)hipStreamDestroy(y);
      (void)hipHostFree(s->slot_words);
      (void)hipFree(s->slab);
      return hip_fail(e, "hipStreamSynchronize");
    }
  rl_server* raw = s.release();
  raw->scheduler = std::thread(scheduler_loop, raw);
  *out = raw;
  return RL_OK;
}

extern "C" rl_status rl_server_submit(rl_server* s, const rl_event* ev, uint64_t* ticket) {
  if (!s || !ev || !ticket || (ev->n_items && !ev->items)) return fail(RL_EINVAL, "rl_server_submit: NULL argument");
  auto e = std::make_unique<Event>();
  for (uint32_t k = 0; k < ev->n_items; ++k) {
    const rl_event_item& it = ev->items[k];
    std::vector<Range> rs;
    rl_status st = validate_view(&it.src, it.n, "src", &rs, false);
    if (st) return st;
    if (!it.dst_layout || it.dst_layout->schema != it.src.layout->schema)
      return fail(RL_EINVAL, "item %u: destination layout of another schema", k);
    if (it.src.layout->space != RL_SPACE_HOST_PINNED && it.src.layout->space != RL_SPACE_HOST)
      return fail(RL_EINVAL, "item %u: sources are host collections", k);
    if (it.dst_layout->space != RL_SPACE_DEVICE) return fail(RL_EINVAL, "item %u: results live on the device", k);
    if (it.dst_layout->kind == RL_AOSOA && it.dst_layout->width == 0)
      return fail(RL_EINVAL, "item %u: auto block width is for batches", k);
    ItemCopy c;
    c.src_layout = it.src.layout;
    c.dst_layout = it.dst_layout;
    c.n = it.n;
    c.src_cap = it.src.capacity;
    c.src_bufs.assign(it.src.buffers, it.src.buffers + layout_n_buffers(it.src.layout));
    const size_t ng = it.src.layout->schema->members.size();
    if (ng) {
      c.src_mcap.assign(it.src.member_capacity, it.src.member_capacity + ng);
      // results hold at most the source's members
      c.dst_mcap = c.src_mcap;
    }
    c.dst_bytes.resize(layout_n_buffers(it.dst_layout));
    layout_buffer_bytes(it.dst_layout, it.n, c.dst_mcap.empty() ? nullptr : c.dst_mcap.data(), c.dst_bytes.data());
    rl_xfer_opts o{RL_XFER_AUTO};
    if (it.n && transfer_is_staged(it.src, &o))
      e->stage_need = std::max<uint64_t>(e->stage_need, staging_bytes(it.src, it.n));
    e->items.push_back(std::move(c));
  }
  e->bytes = event_bytes(*e);
  const uint64_t need = e->bytes + (e->stage_need + 255) / 256 * 256;
  // the slab less the look-back regions is what events can ever use
  uint64_t usable = s->pool.capacity();
  for (auto* lb : s->lookback)
    if (lb) usable -= kServerLookbackBytes;
  if (need > usable)
    return fail(RL_EBUDGET, "event needs %llu bytes (results and staging), %llu of the budget hold events",
                (unsigned long long)need, (unsigned long long)usable);
  hipError_t he = hipEventCreateWithFlags(&e->done, hipEventDisableTiming);
  if (he != hipSuccess) return hip_fail(he, "hipEventCreate");
  std::lock_guard<std::mutex> lk(s->mu);
  e->ticket = s->next_ticket++;
  e->submitted = Clock::now();
  if (!s->any) {
    s->first_submit = e->submitted;
    s->any = true;
  }
  *ticket = e->ticket;
  s->queue.push_back(e->ticket);
  s->events[e->ticket] = std::move(e);
  ++s->submitted;
  s->cv_work.notify_one();
  return RL_OK;
}

extern "C" rl_status rl_server_wait(rl_server* s, uint64_t ticket, int64_t timeout_ms, rl_event_result* res) {
  if (!s) return fail(RL_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->events.find(ticket);
  if (it == s->events.end()) return fail(RL_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  Event* e = it->second.get();
  auto done = [&] { return e->state == EvState::DONE || e->state == EvState::RELEASED; };
  if (timeout_ms < 0) s->cv_done.wait(lk, done);
  else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done))
    return fail(RL_EBUSY, "event %llu not done", (unsigned long long)ticket);
  if (e->state == EvState::RELEASED) return fail(RL_EINVAL, "event %llu already released", (unsigned long long)ticket);
  if (res) {
    e->buf_ptrs.clear();
    e->mcaps.clear();
    for (auto& c : e->items) {
      e->buf_ptrs.push_back(c.dst_bufs.data());
      for (auto m : c.dst_mcap) e->mcaps.push_back(m);
    }
    res->n_items = (uint32_t)e->items.size();
    res->latency_ns = (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(e->done_at - e->submitted).count();
    res->bytes = e->bytes;
    res->buffers = e->buf_ptrs.data();
    res->member_capacity = e->mcaps.empty() ? nullptr : e->mcaps.data();
    res->status = e->status;
  }
  return e->status;
}

extern "C" rl_status rl_server_release(rl_server* s, uint64_t ticket) {
  if (!s) return fail(RL_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->events.find(ticket);
  if (it == s->events.end()) return fail(RL_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  Event* e = it->second.get();
  if (e->state != EvState::DONE) return fail(RL_EBUSY, "event %llu not done", (unsigned long long)ticket);
  for (auto& c : e->items)
    for (size_t b = 0; b < c.dst_offsets.size(); ++b)
      if (c.dst_offsets[b] != UINT64_MAX) s->pool.release(c.dst_offsets[b]);
  (void)hipEventDestroy(e->done);
  s->events.erase(it);
  s->cv_work.notify_one();
  return RL_OK;
}

extern "C" rl_status rl_server_stats_get(rl_server* s, rl_server_stats* out) {
  if (!s || !out) return fail(RL_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  memset(out, 0, sizeof *out);
  out->completed = s->completed;
  out->submitted = s->submitted;
  out->p50_ms = percentile(s->lat_ms, 50);
  out->p99_ms = percentile(s->lat_ms, 99);
  out->max_ms = percentile(s->lat_ms, 100);
  if (s->completed && s->any) {
    const double sec = std::chrono::duration<double>(s->last_done - s->first_submit).count();
    out->events_per_s = sec > 0 ? (double)s->completed / sec : 0.0;
  }
  out->peak_bytes = s->peak;
  out->h2d_bytes = s->h2d_bytes;
  return RL_OK;
}

extern "C" void rl_server_destroy(rl_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->scheduler.joinable()) s->scheduler.join();
  for (auto st : s->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (auto& kv : s->events)
    if (kv.second->done) (void)hipEventDestroy(kv.second->done);
  if (s->slab) (void)hipFree(s->slab);
  if (s->slot_words) (void)hipHostFree(s->slot_words);
  delete s;
}
