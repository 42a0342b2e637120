// Host <-> device transfers that carry a conversion (Sec. VII-A: copies
// between memory contexts with extra arguments controlling the copy;
// Sec. VII-B: copy between layouts).
//
// Zero-copy mode: the conversion kernels read (or write) the pinned host
// buffers directly through their device mapping, so the PCIe transfer and
// the layout change are one pass with no staging.
//
// Staged mode: the host side's buffers are copied whole by the DMA engines
// into a device staging buffer kept per stream (reuse is ordered by the
// stream), then converted from there (or converted into it, then copied
// out), all on the caller's stream.  Copies
// and conversions of different calls on different streams overlap.  (A
// split into chunks on a second copy stream was measured slower: every
// cross-stream event dependency between the DMA queue and the compute queue
// cost tens of microseconds, more than the overlap it bought.)
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <numeric>

#include "plan.h"
#include "rl_internal.h"

namespace rl {

bool is_host(rl_space s) { return s == RL_SPACE_HOST || s == RL_SPACE_HOST_PINNED; }

namespace {

struct StageBuf {
  uint8_t* ptr = nullptr;
  uint64_t bytes = 0;
};
std::mutex g_stage_mu;
std::map<std::pair<int, hipStream_t>, StageBuf> g_stage;   // held until the process ends

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

// Stage every buffer of the host side whole, in `given` (device memory of
// at least staging_bytes(), owned by the caller) or else in the staging
// buffer of (device, stream).
rl_status staged(const rl_view& src, const rl_view& dst, uint64_t n, hipStream_t stream, bool h2d,
                 uint8_t* given, uint64_t given_bytes, const PlanShape& shape) {
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
  // one staging buffer per (device, stream), reused in stream order; the
  // lock keeps the enqueue of one call from interleaving with another's
  std::unique_lock<std::mutex> lk(g_stage_mu, std::defer_lock);
  uint8_t* stage = nullptr;
  hipError_t e;
  if (given) {
    if (given_bytes < total) return fail(RL_EINVAL, "staging block too small");
    stage = given;
  } else {
    lk.lock();
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
    StageBuf& sbuf = g_stage[{dev, stream}];
    if (sbuf.bytes < total) {
      if (sbuf.ptr) {
        // earlier work on this stream may still read the old buffer
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        (void)hipFree(sbuf.ptr);
        sbuf.ptr = nullptr;
        sbuf.bytes = 0;
      }
      const uint64_t want = std::max<uint64_t>(total + total / 4, 1 << 20);
      if ((e = hipMalloc(&sbuf.ptr, want)) != hipSuccess)
        return fail(RL_ENOMEM, "staging %llu bytes: %s", (unsigned long long)want, hipGetErrorString(e));
      sbuf.bytes = want;
    }
    stage = sbuf.ptr;
  }
  std::vector<void*> sb(nb);
  for (uint32_t b = 0; b < nb; ++b) sb[b] = stage + at[b];
  rl_view staged{HL, hv.capacity, hv.member_capacity, sb.data()};
  rl_status st = RL_OK;
  if (h2d) {
    for (uint32_t b = 0; b < nb && !st; ++b)
      if (bytes[b] && (e = hipMemcpyAsync(sb[b], hv.buffers[b], bytes[b], hipMemcpyHostToDevice, stream)) != hipSuccess)
        st = hip_fail(e, "hipMemcpyAsync H2D");
    Plan plan;
    if (!st) st = make_plan(staged, dst, n, shape, &plan);
    if (!st) st = enqueue_plan(plan, stream);
  } else {
    Plan plan;
    st = make_plan(src, staged, n, shape, &plan);
    if (!st) st = enqueue_plan(plan, stream);
    for (uint32_t b = 0; b < nb && !st; ++b)
      if (bytes[b] && (e = hipMemcpyAsync(hv.buffers[b], sb[b], bytes[b], hipMemcpyDeviceToHost, stream)) != hipSuccess)
        st = hip_fail(e, "hipMemcpyAsync D2H");
  }
  return st;
}

}  // namespace

uint64_t staging_bytes(const rl_view& hv, uint64_t n) {
  const uint32_t nb = layout_n_buffers(hv.layout);
  std::vector<uint64_t> bytes(nb);
  layout_buffer_bytes(hv.layout, n, hv.member_capacity, bytes.data());
  uint64_t total = 0;
  for (auto b : bytes) total += (b + 255) & ~255ull;
  return total;
}

bool transfer_is_staged(const rl_view& hv, const rl_xfer_opts* opts) {
  const rl_xfer_mode m = opts ? opts->mode : RL_XFER_AUTO;
  if (m == RL_XFER_STAGED) return true;
  if (m == RL_XFER_ZERO_COPY) return false;
  return hv.layout->space != RL_SPACE_HOST_PINNED;
}

rl_status transfer_impl(const rl_view* src, const rl_view* dst, uint64_t n, hipStream_t stream,
                        const rl_xfer_opts* opts, uint8_t* stage, uint64_t stage_bytes,
                        uint64_t* lookback, uint64_t lookback_bytes) {
  std::vector<Range> rs, rd;
  rl_status st = validate_view(src, n, "src", &rs, false);
  if (st) return st;
  if ((st = validate_view(dst, n, "dst", &rd, false))) return st;
  const rl_layout* SL = src->layout;
  const rl_layout* DL = dst->layout;
  if (SL->schema != DL->schema) return fail(RL_EINVAL, "src and dst use different schemas");
  if (auto_width(src) || auto_width(dst)) return fail(RL_EINVAL, "block width 0 (auto) is only for batches");
  if (SL->kind == RL_STRIDED || DL->kind == RL_STRIDED)
    return fail(RL_EUNSUPPORTED, "transfers of strided layouts (convert on the device, or register a user transfer)");
  const bool sh = is_host(SL->space), dh = is_host(DL->space);
  if (sh == dh) return fail(RL_EUNSUPPORTED, "rl_transfer needs one host and one device view (use rl_convert on device)");
  if (n == 0) return RL_OK;
  const bool h2d = sh;
  const bool jagged = !SL->schema->members.empty();
  if (jagged && SL->kind == RL_AOS && DL->kind == RL_AOS)
    return fail(RL_EUNSUPPORTED, "AoS -> AoS conversion of a schema with jagged groups");
  rl_xfer_opts o{RL_XFER_AUTO};
  if (opts) o = *opts;
  if (o.mode < RL_XFER_AUTO || o.mode > RL_XFER_ZERO_COPY) return fail(RL_EINVAL, "bad transfer mode");
  const rl_layout* HL = h2d ? SL : DL;
  const rl_view& hv = h2d ? *src : *dst;
  // auto: collections in pinned memory are read (or written) in place by
  // the conversion kernels (measured at the link rate, jagged ones too);
  // pageable ones go through device staging
  if (o.mode == RL_XFER_AUTO) o.mode = transfer_is_staged(hv, &o) ? RL_XFER_STAGED : RL_XFER_ZERO_COPY;
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
    // kernels write host memory only in whole 16-byte vectors of an image,
    // and read it through registers
    PlanShape to_host, from_host;
    to_host.direct = 0;
    from_host.dma = 0;
    to_host.lookback = from_host.lookback = lookback;
    to_host.lookback_bytes = from_host.lookback_bytes = lookback_bytes;
    if (stream_capturing(stream)) to_host.fused = from_host.fused = 0;
    st = h2d ? make_plan(hv2, *dst, n, from_host, &plan) : make_plan(*src, hv2, n, to_host, &plan);
    if (st) return st;
    return enqueue_plan(plan, stream);
  }
  PlanShape shape;
  shape.lookback = lookback;
  shape.lookback_bytes = lookback_bytes;
  if (stream_capturing(stream)) shape.fused = 0;
  return staged(*src, *dst, n, stream, h2d, stage, stage_bytes, shape);
}

}  // namespace rl

extern "C" rl_status rl_transfer(const rl_view* src, const rl_view* dst, uint64_t n, void* stream,
                                 const rl_xfer_opts* opts) {
  if (n && src && dst && src->layout && dst->layout && src->layout->schema == dst->layout->schema) {
    std::vector<rl::Range> rs, rd;
    rl_status st = rl::validate_view(src, n, "src", &rs, false);
    if (st) return st;
    if ((st = rl::validate_view(dst, n, "dst", &rd, false))) return st;
    bool handled = false;
    st = rl::run_specialisations(src, dst, n, stream, &handled);
    if (handled) return st;
  }
  return rl::transfer_impl(src, dst, n, (hipStream_t)stream, opts, nullptr, 0);
}

// ------------------------------------------------------------------ no-allocation variant
//
// Staging memory of rl_transfer_noalloc: a fixed array in the code object.
// Every device the library is loaded on holds its own copy until the
// process ends.  In host code `scratch` only names the symbol; its device
// address on the current device comes from hipGetSymbolAddress and is the
// only form passed to copies and kernels.
namespace {
constexpr uint64_t kNoAllocStageBytes = RL_TRANSFER_NOALLOC_LIMIT;
// after the staging bytes: look-back words of single-pass jagged
// conversions (zero at load)
constexpr uint64_t kNoAllocLookbackBytes = 1ull << 20;
__device__ __align__(256) uint8_t scratch[kNoAllocStageBytes + kNoAllocLookbackBytes];

std::mutex g_scratch_mu;
std::map<int, uint8_t*> g_scratch_ptr;   // device -> address of that device's scratch

rl_status scratch_on_current_device(uint8_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return rl::hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess)
      return rl::hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return rl::fail(RL_EHIP, "hipGetSymbolAddress(scratch) gave a null address");
    it = g_scratch_ptr.emplace(dev, (uint8_t*)p).first;
  }
  *out = it->second;
  return RL_OK;
}
}  // namespace

extern "C" rl_status rl_transfer_noalloc(const rl_view* src, const rl_view* dst, uint64_t n, void* stream,
                                         const rl_xfer_opts* opts) {
  // staging and the look-back state of jagged conversions are the memory
  // the library would otherwise allocate; the staging limit is checked
  // before anything is enqueued
  const bool one_host = src && dst && src->layout && dst->layout &&
                        rl::is_host(src->layout->space) != rl::is_host(dst->layout->space);
  const bool strided = src && dst && src->layout && dst->layout &&
                       (src->layout->kind == RL_STRIDED || dst->layout->kind == RL_STRIDED);
  if (!one_host || n == 0 || strided) return rl::transfer_impl(src, dst, n, (hipStream_t)stream, opts, nullptr, 0);
  const rl_view& hv = rl::is_host(src->layout->space) ? *src : *dst;
  uint8_t* base = nullptr;
  if (!rl::transfer_is_staged(hv, opts)) {
    rl_status st = scratch_on_current_device(&base);
    if (st) return st;
    return rl::transfer_impl(src, dst, n, (hipStream_t)stream, opts, nullptr, 0,
                             reinterpret_cast<uint64_t*>(base + kNoAllocStageBytes), kNoAllocLookbackBytes);
  }
  if (n > hv.capacity) return rl::fail(RL_EINVAL, "n %llu over the host view's capacity", (unsigned long long)n);
  if (!hv.layout->schema->members.empty() && !hv.member_capacity)
    return rl::fail(RL_EINVAL, "member capacities of the host view are NULL");
  const uint64_t need = rl::staging_bytes(hv, n);
  if (need > kNoAllocStageBytes)
    return rl::fail(RL_ELIMIT, "rl_transfer_noalloc stages at most %llu bytes; this transfer needs %llu",
                    (unsigned long long)kNoAllocStageBytes, (unsigned long long)need);
  rl_status st = scratch_on_current_device(&base);
  if (st) return st;
  return rl::transfer_impl(src, dst, n, (hipStream_t)stream, opts, base, kNoAllocStageBytes,
                           reinterpret_cast<uint64_t*>(base + kNoAllocStageBytes), kNoAllocLookbackBytes);
}
