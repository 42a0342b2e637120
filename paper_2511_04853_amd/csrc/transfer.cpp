// Host <-> device transfers that carry a conversion (Sec. VII-A: copies
// between memory contexts with extra arguments controlling the copy;
// Sec. VII-B: copy between layouts).
//
// Staged mode, host -> device: the source is cut into chunks of whole
// objects; a copy stream moves chunk k into staging slot k mod S with the
// DMA engines while the caller's stream converts chunk k - 1 out of its
// slot into the destination.  Events order slot reuse across the two
// streams.  Device -> host runs the same ring the other way (convert into
// a slot on the caller's stream, copy the slot out on the copy stream).
// Collections with jagged groups are staged whole (their members can sit
// anywhere in the pool), in stream-ordered allocations.
//
// Zero-copy mode: the conversion kernels read (or write) the pinned host
// buffers directly through their device mapping; one pass, no staging.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <numeric>

#include "plan.h"
#include "rl_internal.h"

namespace rl {

namespace {

constexpr uint32_t kMaxSlots = 8;
constexpr uint64_t kDefaultChunk = 4ull << 20;

struct DevXfer {
  std::mutex mu;
  bool ready = false;
  hipStream_t copy = nullptr;
  uint8_t* staging = nullptr;
  uint64_t slot_bytes = 0;
  uint32_t n_slots = 0;
  hipEvent_t slot_free[kMaxSlots] = {};
  hipEvent_t filled[kMaxSlots] = {};
  hipEvent_t tail = nullptr;
  uint32_t next = 0;
};

DevXfer g_xfer[64];

rl_status ensure(DevXfer& x, uint64_t slot_bytes, uint32_t n_slots) {
  hipError_t e;
  if (!x.ready) {
    if ((e = hipStreamCreateWithFlags(&x.copy, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "copy stream");
    for (uint32_t k = 0; k < kMaxSlots; ++k) {
      if ((e = hipEventCreateWithFlags(&x.slot_free[k], hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "event");
      if ((e = hipEventCreateWithFlags(&x.filled[k], hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "event");
    }
    if ((e = hipEventCreateWithFlags(&x.tail, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "event");
    x.ready = true;
  }
  if (x.slot_bytes < slot_bytes || x.n_slots < n_slots) {
    // wait for every use of the old ring before freeing it
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    if (x.staging) (void)hipFree(x.staging);
    x.staging = nullptr;
    const uint64_t sb = std::max<uint64_t>(x.slot_bytes, (slot_bytes + 255) & ~255ull);
    const uint32_t ns = std::max(x.n_slots, n_slots);
    if ((e = hipMalloc(&x.staging, sb * ns)) != hipSuccess) {
      x.slot_bytes = 0;
      x.n_slots = 0;
      return fail(RL_ENOMEM, "staging ring of %llu bytes: %s", (unsigned long long)(sb * ns), hipGetErrorString(e));
    }
    x.slot_bytes = sb;
    x.n_slots = ns;
  }
  return RL_OK;
}

bool is_host(rl_space s) { return s == RL_SPACE_HOST || s == RL_SPACE_HOST_PINNED; }

// Device address of pinned host memory (or nullptr if not pinned).
void* device_alias(void* p) {
  if (!p) return nullptr;
  hipPointerAttribute_t a;
  memset(&a, 0, sizeof a);
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (a.type != hipMemoryTypeHost || !a.devicePointer) return nullptr;
  const intptr_t off = (intptr_t)((uint8_t*)p - (uint8_t*)a.hostPointer);
  return (uint8_t*)a.devicePointer + (a.hostPointer ? off : 0);
}

// Buffers of `view` shifted to start at object i0 (dense layouts only).
std::vector<void*> shifted(const rl_view& v, uint64_t i0) {
  const rl_layout* L = v.layout;
  const uint32_t nb = layout_n_buffers(L);
  std::vector<void*> out(v.buffers, v.buffers + nb);
  if (L->kind == RL_AOS) out[0] = (uint8_t*)out[0] + i0 * L->stride;
  else if (L->kind == RL_AOSOA) out[0] = (uint8_t*)out[0] + i0 * (uint64_t)L->obj_bytes;
  else
    for (size_t c = 0; c < L->storage.size(); ++c) out[c] = (uint8_t*)out[c] + i0 * type_size(L->storage[c]);
  return out;
}

// Bytes per object of a dense layout (for chunking), and the byte runs of
// objects [i0, i0 + cnt) as (buffer, offset, length).
uint64_t bytes_per_object(const rl_layout* L) {
  return L->kind == RL_AOS ? L->stride : L->obj_bytes;
}

uint32_t chunk_unit(const rl_layout* a, const rl_layout* b) {
  uint32_t u = 16;
  for (const rl_layout* L : {a, b})
    if (L->kind == RL_AOSOA) u = u / std::gcd(u, L->width) * L->width;
  return u;
}

// A view of the staging slot holding `cnt` objects of layout L (dense).
struct SlotView {
  std::vector<void*> bufs;
  rl_view view;
};

void make_slot_view(const rl_layout* L, uint8_t* slot, uint64_t cnt, SlotView* sv) {
  const uint32_t nb = layout_n_buffers(L);
  std::vector<uint64_t> bytes(nb);
  layout_buffer_bytes(L, cnt, nullptr, bytes.data());
  sv->bufs.resize(nb);
  uint64_t pos = 0;
  for (uint32_t b = 0; b < nb; ++b) {
    sv->bufs[b] = slot + pos;
    pos += (bytes[b] + 255) & ~255ull;
  }
  sv->view = rl_view{L, cnt, nullptr, sv->bufs.data()};
}

uint64_t slot_bytes_for(const rl_layout* L, uint64_t cnt) {
  const uint32_t nb = layout_n_buffers(L);
  std::vector<uint64_t> bytes(nb);
  layout_buffer_bytes(L, cnt, nullptr, bytes.data());
  uint64_t pos = 0;
  for (auto b : bytes) pos += (b + 255) & ~255ull;
  return pos;
}

// Copy objects [i0, i0 + cnt) of a dense layout between two buffer sets
// (host view <-> staging slot), one async copy per buffer run.
hipError_t copy_objects(const rl_layout* L, void* const* from, uint64_t from_i0, void* const* to,
                        uint64_t to_i0, uint64_t cnt, hipMemcpyKind kind, hipStream_t s) {
  if (L->kind == RL_SOA) {
    for (size_t c = 0; c < L->storage.size(); ++c) {
      const uint64_t sz = type_size(L->storage[c]);
      hipError_t e = hipMemcpyAsync((uint8_t*)to[c] + to_i0 * sz, (const uint8_t*)from[c] + from_i0 * sz,
                                    cnt * sz, kind, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  uint64_t per = bytes_per_object(L), len = cnt * per;
  if (L->kind == RL_AOSOA) len = (cnt + L->width - 1) / L->width * L->width * per;
  return hipMemcpyAsync((uint8_t*)to[0] + to_i0 * per, (const uint8_t*)from[0] + from_i0 * per, len, kind, s);
}

rl_status staged_dense(const rl_view& src, const rl_view& dst, uint64_t n, hipStream_t stream,
                       const rl_xfer_opts& o, bool h2d, DevXfer& x) {
  const rl_layout* SL = src.layout;
  const rl_layout* DL = dst.layout;
  const rl_layout* HL = h2d ? SL : DL;   // the host side's layout, staged as is
  const uint64_t per = std::max<uint64_t>(1, bytes_per_object(HL));
  const uint32_t unit = chunk_unit(SL, DL);
  uint64_t chunk_bytes = o.chunk_bytes ? o.chunk_bytes : kDefaultChunk;
  uint64_t cnt = std::max<uint64_t>(unit, chunk_bytes / per / unit * unit);
  if (cnt > n) cnt = (n + unit - 1) / unit * unit;
  const uint32_t ns = std::min<uint32_t>(o.n_slots ? o.n_slots : 3, kMaxSlots);
  rl_status st = ensure(x, slot_bytes_for(HL, cnt), ns);
  if (st) return st;
  hipError_t e;
  // The copy stream must not touch a host destination before earlier work
  // on the caller's stream is done, nor may conversions overtake it.
  if ((e = hipEventRecord(x.tail, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
  if ((e = hipStreamWaitEvent(x.copy, x.tail, 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  for (uint64_t i0 = 0; i0 < n; i0 += cnt) {
    const uint64_t c = std::min(cnt, n - i0);
    const uint32_t slot = x.next;
    x.next = (x.next + 1) % ns;
    uint8_t* sp = x.staging + (uint64_t)slot * x.slot_bytes;
    SlotView sv;
    make_slot_view(HL, sp, c, &sv);
    if (h2d) {
      // host chunk -> slot (copy stream), then slot -> destination (caller stream)
      if ((e = hipStreamWaitEvent(x.copy, x.slot_free[slot], 0)) != hipSuccess) return hip_fail(e, "wait");
      if ((e = copy_objects(HL, src.buffers, i0, sv.bufs.data(), 0, c, hipMemcpyHostToDevice, x.copy)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync H2D");
      if ((e = hipEventRecord(x.filled[slot], x.copy)) != hipSuccess) return hip_fail(e, "record");
      if ((e = hipStreamWaitEvent(stream, x.filled[slot], 0)) != hipSuccess) return hip_fail(e, "wait");
      std::vector<void*> db = shifted(dst, i0);
      rl_view dv{DL, c, dst.member_capacity, db.data()};
      Plan plan;
      if ((st = make_plan(sv.view, dv, c, PlanShape{}, &plan))) return st;
      if ((st = enqueue_plan(plan, stream))) return st;
      if ((e = hipEventRecord(x.slot_free[slot], stream)) != hipSuccess) return hip_fail(e, "record");
    } else {
      // source -> slot (caller stream), then slot -> host chunk (copy stream)
      if ((e = hipStreamWaitEvent(stream, x.slot_free[slot], 0)) != hipSuccess) return hip_fail(e, "wait");
      std::vector<void*> sb = shifted(src, i0);
      rl_view s2{SL, c, src.member_capacity, sb.data()};
      Plan plan;
      if ((st = make_plan(s2, sv.view, c, PlanShape{}, &plan))) return st;
      if ((st = enqueue_plan(plan, stream))) return st;
      if ((e = hipEventRecord(x.filled[slot], stream)) != hipSuccess) return hip_fail(e, "record");
      if ((e = hipStreamWaitEvent(x.copy, x.filled[slot], 0)) != hipSuccess) return hip_fail(e, "wait");
      if ((e = copy_objects(HL, sv.bufs.data(), 0, dst.buffers, i0, c, hipMemcpyDeviceToHost, x.copy)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync D2H");
      if ((e = hipEventRecord(x.slot_free[slot], x.copy)) != hipSuccess) return hip_fail(e, "record");
    }
  }
  // later work on the caller's stream comes after the last copy
  if ((e = hipEventRecord(x.tail, x.copy)) != hipSuccess) return hip_fail(e, "record");
  if ((e = hipStreamWaitEvent(stream, x.tail, 0)) != hipSuccess) return hip_fail(e, "wait");
  return RL_OK;
}

// Jagged collections: stage every buffer of the host side whole.
rl_status staged_whole(const rl_view& src, const rl_view& dst, uint64_t n, hipStream_t stream, bool h2d) {
  const rl_view& hv = h2d ? src : dst;
  const rl_layout* HL = hv.layout;
  const uint32_t nb = layout_n_buffers(HL);
  std::vector<uint64_t> bytes(nb);
  layout_buffer_bytes(HL, n, hv.member_capacity, bytes.data());
  uint64_t total = 0;
  std::vector<uint64_t> at(nb);
  for (uint32_t b = 0; b < nb; ++b) {
    at[b] = total;
    total += (bytes[b] + 255) & ~255ull;
  }
  uint8_t* stage = nullptr;
  hipError_t e = hipMallocAsync((void**)&stage, std::max<uint64_t>(total, 256), stream);
  if (e != hipSuccess) return fail(RL_ENOMEM, "staging %llu bytes: %s", (unsigned long long)total, hipGetErrorString(e));
  std::vector<void*> sb(nb);
  for (uint32_t b = 0; b < nb; ++b) sb[b] = stage + at[b];
  rl_view staged{HL, hv.capacity, hv.member_capacity, sb.data()};
  rl_status st = RL_OK;
  if (h2d) {
    for (uint32_t b = 0; b < nb && !st; ++b)
      if (bytes[b] && (e = hipMemcpyAsync(sb[b], hv.buffers[b], bytes[b], hipMemcpyHostToDevice, stream)) != hipSuccess)
        st = hip_fail(e, "hipMemcpyAsync H2D");
    Plan plan;
    if (!st) st = make_plan(staged, dst, n, PlanShape{}, &plan);
    if (!st) st = enqueue_plan(plan, stream);
  } else {
    Plan plan;
    st = make_plan(src, staged, n, PlanShape{}, &plan);
    if (!st) st = enqueue_plan(plan, stream);
    for (uint32_t b = 0; b < nb && !st; ++b)
      if (bytes[b] && (e = hipMemcpyAsync(hv.buffers[b], sb[b], bytes[b], hipMemcpyDeviceToHost, stream)) != hipSuccess)
        st = hip_fail(e, "hipMemcpyAsync D2H");
  }
  e = hipFreeAsync(stage, stream);
  if (!st && e != hipSuccess) st = hip_fail(e, "hipFreeAsync");
  return st;
}

}  // namespace

rl_status transfer_impl(const rl_view* src, const rl_view* dst, uint64_t n, hipStream_t stream,
                        const rl_xfer_opts* opts) {
  std::vector<Range> rs, rd;
  rl_status st = validate_view(src, n, "src", &rs, false);
  if (st) return st;
  if ((st = validate_view(dst, n, "dst", &rd, false))) return st;
  const rl_layout* SL = src->layout;
  const rl_layout* DL = dst->layout;
  if (SL->schema != DL->schema) return fail(RL_EINVAL, "src and dst use different schemas");
  if (auto_width(src) || auto_width(dst)) return fail(RL_EINVAL, "block width 0 (auto) is only for batches");
  const bool sh = is_host(SL->space), dh = is_host(DL->space);
  if (sh == dh) return fail(RL_EUNSUPPORTED, "rl_transfer needs one host and one device view (use rl_convert on device)");
  if (n == 0) return RL_OK;
  const bool h2d = sh;
  const bool jagged = !SL->schema->members.empty();
  if (jagged && SL->kind == RL_AOS && DL->kind == RL_AOS)
    return fail(RL_EUNSUPPORTED, "AoS -> AoS conversion of a schema with jagged groups");
  rl_xfer_opts o{RL_XFER_AUTO, 0, 0};
  if (opts) o = *opts;
  if (o.mode < RL_XFER_AUTO || o.mode > RL_XFER_ZERO_COPY) return fail(RL_EINVAL, "bad transfer mode");
  if (o.n_slots > kMaxSlots) return fail(RL_EINVAL, "at most %u staging slots", kMaxSlots);
  const rl_layout* HL = h2d ? SL : DL;
  const rl_view& hv = h2d ? *src : *dst;
  // auto: dense collections in pinned memory are read (or written) in place
  // by the conversion kernels; others go through device staging
  if (o.mode == RL_XFER_AUTO) o.mode = (!jagged && HL->space == RL_SPACE_HOST_PINNED) ? RL_XFER_ZERO_COPY : RL_XFER_STAGED;
  if (o.mode == RL_XFER_ZERO_COPY) {
    if (HL->space != RL_SPACE_HOST_PINNED) return fail(RL_EUNSUPPORTED, "zero-copy needs pinned host memory");
    const uint32_t nb = layout_n_buffers(HL);
    std::vector<uint64_t> bytes(nb);
    layout_buffer_bytes(HL, n, hv.member_capacity, bytes.data());
    std::vector<void*> alias(nb, nullptr);
    for (uint32_t b = 0; b < nb; ++b) {
      if (!bytes[b]) continue;
      alias[b] = device_alias(hv.buffers[b]);
      if (!alias[b]) return fail(RL_EUNSUPPORTED, "host buffer %u is not pinned memory mapped to the device", b);
      // the whole run must belong to one pinned allocation mapped linearly
      uint8_t* last = (uint8_t*)device_alias((uint8_t*)hv.buffers[b] + bytes[b] - 1);
      if (last != (uint8_t*)alias[b] + bytes[b] - 1)
        return fail(RL_EUNSUPPORTED, "host buffer %u is not one linearly mapped pinned allocation", b);
    }
    rl_view hv2{HL, hv.capacity, hv.member_capacity, alias.data()};
    Plan plan;
    st = h2d ? make_plan(hv2, *dst, n, PlanShape{}, &plan) : make_plan(*src, hv2, n, PlanShape{}, &plan);
    if (st) return st;
    return enqueue_plan(plan, stream);
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(RL_EUNSUPPORTED, "device index");
  if (jagged) return staged_whole(*src, *dst, n, stream, h2d);
  DevXfer& x = g_xfer[dev];
  std::lock_guard<std::mutex> lk(x.mu);
  return staged_dense(*src, *dst, n, stream, o, h2d, x);
}

}  // namespace rl

extern "C" rl_status rl_transfer(const rl_view* src, const rl_view* dst, uint64_t n, void* stream,
                                 const rl_xfer_opts* opts) {
  return rl::transfer_impl(src, dst, n, (hipStream_t)stream, opts);
}
