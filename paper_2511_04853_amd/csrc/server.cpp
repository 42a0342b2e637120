// Serving loop: events (one or more collections each, in pinned host
// memory) arrive at any time; a scheduler thread admits them in arrival
// order while their result bytes fit a device-memory budget and an
// in-flight slot is free, converts them with host -> device transfers on
// the server's streams (events overlap on the device), and keeps the
// converted collections resident in a pool carved from one device slab
// until the client releases them.  The scheduling itself (admission,
// completion, release, cancellation, statistics) is the device-free core
// in serve_core.h; this file is its HIP executor.  Completion is observed
// by polling events; latency is submit -> last conversion done.
#include <string.h>

#include <memory>
#include <vector>

#include "plan.h"
#include "rl_internal.h"
#include "serve_core.h"

using namespace rl;

namespace {

struct ItemCopy {
  const rl_layout* src_layout;
  const rl_layout* dst_layout;
  uint64_t n, src_cap;
  std::vector<void*> src_bufs;
  std::vector<uint64_t> src_mcap;
  std::vector<uint64_t> dst_mcap;      // member capacity of the result
  std::vector<uint64_t> dst_bytes;     // bytes of each result buffer
  std::vector<void*> dst_bufs;         // set when the event starts
};

struct Payload {
  std::vector<ItemCopy> items;
  hipEvent_t done = nullptr;
  bool recorded = false;
  // result views handed to the client
  std::vector<void* const*> buf_ptrs;
  std::vector<uint64_t> mcaps;
};

using Event = CoreEvent<Payload>;

struct HipExec {
  rl_server* s = nullptr;
  void thread_init();
  uint64_t start(Event& e);
  bool poll(Event& e);
  void retire(Event& e);
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
  // one pinned word per in-flight slot: the device status flags of the
  // event in that slot, handed over in stream order when it completes
  uint32_t* slot_words = nullptr;
  uint32_t* slot_words_dev = nullptr;
  HipExec exec;
  std::unique_ptr<ServeCore<HipExec, Payload>> core;
};

namespace {

void HipExec::thread_init() { (void)hipSetDevice(s->device); }

// Enqueue the transfers of an admitted event on its stream (no lock held).
uint64_t HipExec::start(Event& e) {
  uint64_t h2d = 0;
  hipStream_t st = s->streams[e.stream];
  uint8_t* stage = e.stage_bytes ? s->slab + e.stage_off : nullptr;
  s->slot_words[e.slot] = 0;
  size_t k = 0;
  for (auto& it : e.p.items) {
    it.dst_bufs.clear();
    for (size_t b = 0; b < it.dst_bytes.size(); ++b, ++k)
      it.dst_bufs.push_back(e.block_off[k] == UINT64_MAX ? nullptr : s->slab + e.block_off[k]);
  }
  for (auto& it : e.p.items) {
    rl_view sv{it.src_layout, it.src_cap, it.src_mcap.empty() ? nullptr : it.src_mcap.data(), it.src_bufs.data()};
    rl_view dv{it.dst_layout, it.n, it.dst_mcap.empty() ? nullptr : it.dst_mcap.data(), it.dst_bufs.data()};
    rl_xfer_opts o{RL_XFER_AUTO};
    // items of an event run one after another on its stream, so they share
    // the event's staging block
    const rl_status r = transfer_impl(&sv, &dv, it.n, st, &o, stage, e.stage_bytes, s->lookback[e.stream],
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
  if (hipEventRecord(e.p.done, st) != hipSuccess) {
    if (e.status == RL_OK) e.status = RL_EHIP;
  } else {
    e.p.recorded = true;
  }
  return h2d;
}

bool HipExec::poll(Event& e) {
  if (e.p.recorded) {
    const hipError_t q = hipEventQuery(e.p.done);
    if (q == hipErrorNotReady) return false;
    if (q != hipSuccess && e.status == RL_OK) e.status = RL_EHIP;
  }
  if (e.status == RL_OK) e.status = status_of_flags(((volatile uint32_t*)s->slot_words)[e.slot]);
  return true;
}

void HipExec::retire(Event& e) {
  if (!e.p.done) return;
  if (e.p.recorded) (void)hipEventSynchronize(e.p.done);
  (void)hipEventDestroy(e.p.done);
  e.p.done = nullptr;
}

void free_device_state(rl_server* s) {
  for (auto x : s->streams) (void)hipStreamDestroy(x);
  if (s->slot_words) (void)hipHostFree(s->slot_words);
  if (s->slab) (void)hipFree(s->slab);
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
  s->exec.s = s.get();
  hipError_t e = hipGetDevice(&s->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if ((e = hipMalloc(&s->slab, opts->budget_bytes)) != hipSuccess)
    return fail(RL_ENOMEM, "serving pool of %llu bytes: %s", (unsigned long long)opts->budget_bytes,
                hipGetErrorString(e));
  if ((e = hipHostMalloc((void**)&s->slot_words, opts->max_in_flight * sizeof(uint32_t), hipHostMallocDefault)) !=
      hipSuccess) {
    free_device_state(s.get());
    return hip_fail(e, "hipHostMalloc(status words)");
  }
  if ((e = hipHostGetDevicePointer((void**)&s->slot_words_dev, s->slot_words, 0)) != hipSuccess) {
    free_device_state(s.get());
    return hip_fail(e, "hipHostGetDevicePointer(status words)");
  }
  for (uint32_t k = 0; k < opts->n_streams; ++k) {
    hipStream_t st;
    if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) {
      free_device_state(s.get());
      return hip_fail(e, "hipStreamCreate");
    }
    s->streams.push_back(st);
  }
  s->core = std::make_unique<ServeCore<HipExec, Payload>>(s->exec, opts->budget_bytes, opts->max_in_flight,
                                                          opts->n_streams);
  for (uint32_t k = 0; k < opts->n_streams; ++k) {
    const uint64_t off = s->core->reserve(kServerLookbackBytes);
    uint64_t* lb = off == UINT64_MAX ? nullptr : reinterpret_cast<uint64_t*>(s->slab + off);
    if (lb && (e = launch_zero(lb, kServerLookbackBytes, s->streams[k])) != hipSuccess) lb = nullptr;
    s->lookback.push_back(lb);   // null (budget too small): the library's per-stream buffer
  }
  for (auto x : s->streams)
    if ((e = hipStreamSynchronize(x)) != hipSuccess) {
      s->core.reset();
      free_device_state(s.get());
      return hip_fail(e, "hipStreamSynchronize");
    }
  s->core->start();
  *out = s.release();
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
    if (it.src.layout->kind == RL_STRIDED || it.dst_layout->kind == RL_STRIDED)
      return fail(RL_EUNSUPPORTED, "item %u: strided layouts are not served", k);
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
    for (auto b : c.dst_bytes) e->block_bytes.push_back(b);
    rl_xfer_opts o{RL_XFER_AUTO};
    if (it.n && transfer_is_staged(it.src, &o))
      e->stage_bytes = std::max<uint64_t>(e->stage_bytes, staging_bytes(it.src, it.n));
    e->p.items.push_back(std::move(c));
  }
  hipError_t he = hipEventCreateWithFlags(&e->p.done, hipEventDisableTiming);
  if (he != hipSuccess) return hip_fail(he, "hipEventCreate");
  hipEvent_t done = e->p.done;
  const rl_status st = s->core->submit(std::move(e), ticket);
  if (st == RL_EBUDGET) {
    (void)hipEventDestroy(done);
    return fail(RL_EBUDGET, "event needs more than the %llu bytes of the budget that hold events (results and staging)",
                (unsigned long long)s->core->usable());
  }
  if (st) {
    (void)hipEventDestroy(done);
    return fail(st, "server is stopping");
  }
  return RL_OK;
}

extern "C" rl_status rl_server_wait(rl_server* s, uint64_t ticket, int64_t timeout_ms, rl_event_result* res) {
  if (!s) return fail(RL_EINVAL, "server is NULL");
  const rl_status st = s->core->wait(ticket, timeout_ms, [&](Event& e) {
    if (!res) return;
    e.p.buf_ptrs.clear();
    e.p.mcaps.clear();
    for (auto& c : e.p.items) {
      e.p.buf_ptrs.push_back(c.dst_bufs.data());
      for (auto m : c.dst_mcap) e.p.mcaps.push_back(m);
    }
    res->n_items = (uint32_t)e.p.items.size();
    res->latency_ns = (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(e.done_at - e.submitted).count();
    res->bytes = e.bytes;
    res->buffers = e.p.buf_ptrs.data();
    res->member_capacity = e.p.mcaps.empty() ? nullptr : e.p.mcaps.data();
    res->status = e.status;
  });
  switch (st) {
    case RL_EINVAL: return fail(st, "unknown ticket %llu", (unsigned long long)ticket);
    case RL_EBUSY: return fail(st, "event %llu not done", (unsigned long long)ticket);
    case RL_ECANCELED: return fail(st, "event %llu was cancelled", (unsigned long long)ticket);
    default: return st;
  }
}

extern "C" rl_status rl_server_release(rl_server* s, uint64_t ticket) {
  if (!s) return fail(RL_EINVAL, "server is NULL");
  const rl_status st = s->core->release(ticket);
  if (st == RL_EINVAL) return fail(st, "unknown ticket %llu", (unsigned long long)ticket);
  if (st == RL_EBUSY) return fail(st, "event %llu not done", (unsigned long long)ticket);
  return st;
}

extern "C" rl_status rl_server_cancel(rl_server* s, uint64_t ticket) {
  if (!s) return fail(RL_EINVAL, "server is NULL");
  const rl_status st = s->core->cancel(ticket);
  if (st == RL_EINVAL) return fail(st, "unknown ticket %llu", (unsigned long long)ticket);
  if (st == RL_EBUSY) return fail(st, "event %llu already admitted", (unsigned long long)ticket);
  return st;
}

extern "C" rl_status rl_server_stats_get(rl_server* s, rl_server_stats* out) {
  if (!s || !out) return fail(RL_EINVAL, "NULL argument");
  memset(out, 0, sizeof *out);
  s->core->stats(out);
  return RL_OK;
}

extern "C" void rl_server_destroy(rl_server* s) {
  if (!s) return;
  s->core->stop();   // joins the scheduler, waits for and retires held events
  for (auto st : s->streams) (void)hipStreamSynchronize(st);
  s->core.reset();
  free_device_state(s);
  delete s;
}
