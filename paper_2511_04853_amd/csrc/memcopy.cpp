// Copies between memory contexts (Sec. VII-A: memcopy_with_context and its
// variants for partially overlapping arrays, which insertion and deletion
// use).
//
// Device to device: the library's copy kernel (16-byte vectors).  Ranges
// that overlap are moved with memmove semantics in bands taken in the order
// that keeps every band's source intact (from the start when the data moves
// down, from the end when it moves up); a band whose source and destination
// overlap goes through the stream's scratch buffer (two copies), a band
// that does not is copied directly.  Host <-> device: the DMA engines
// (hipMemcpyAsync).  Host <-> host: memmove once the stream is idle.
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "plan.h"
#include "rl_internal.h"

namespace rl {

namespace {

constexpr uint64_t kMoveBand = 64ull << 20;   // bytes per band through scratch

std::mutex g_move_mu;
std::map<std::pair<int, hipStream_t>, uint8_t*> g_move_scratch;   // kMoveBand bytes each, held until exit

rl_status move_scratch(hipStream_t s, uint8_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  uint8_t*& p = g_move_scratch[{dev, s}];
  if (!p && (e = hipMalloc((void**)&p, kMoveBand)) != hipSuccess) {
    p = nullptr;
    return fail(RL_ENOMEM, "move scratch of %llu bytes: %s", (unsigned long long)kMoveBand, hipGetErrorString(e));
  }
  *out = p;
  return RL_OK;
}

}  // namespace

rl_status device_move(uint8_t* dst, const uint8_t* src, uint64_t bytes, hipStream_t s) {
  if (!bytes || dst == src) return RL_OK;
  hipError_t e;
  const bool up = dst > src;
  const uint64_t d = up ? (uint64_t)(dst - src) : (uint64_t)(src - dst);
  if (d >= bytes) {   // disjoint
    if ((e = launch_copy(dst, src, bytes, s)) != hipSuccess) return hip_fail(e, "copy");
    return RL_OK;
  }
  // bands of d bytes never overlap their own destination: direct copies
  // when there are few of them, else bands through scratch
  const bool direct = d >= kMoveBand;
  const uint64_t band = direct ? d : kMoveBand;
  uint8_t* tmp = nullptr;
  std::unique_lock<std::mutex> lk(g_move_mu, std::defer_lock);
  if (!direct) {
    lk.lock();   // held until the bands are enqueued
    rl_status st = move_scratch(s, &tmp);
    if (st) return st;
  }
  for (uint64_t done = 0; done < bytes;) {
    const uint64_t len = std::min(band, bytes - done);
    const uint64_t at = up ? bytes - done - len : done;
    if (direct) {
      e = launch_copy(dst + at, src + at, len, s);
    } else {
      e = launch_copy(tmp, src + at, len, s);
      if (e == hipSuccess) e = launch_copy(dst + at, tmp, len, s);
    }
    if (e != hipSuccess) return hip_fail(e, "copy");
    done += len;
  }
  return RL_OK;
}

}  // namespace rl

using namespace rl;

extern "C" rl_status rl_memcopy(void* dst, rl_space dst_space, const void* src, rl_space src_space, uint64_t bytes,
                                void* stream) {
  if (dst_space < RL_SPACE_DEVICE || dst_space > RL_SPACE_HOST_PINNED || src_space < RL_SPACE_DEVICE ||
      src_space > RL_SPACE_HOST_PINNED)
    return fail(RL_EINVAL, "rl_memcopy: bad memory context");
  if (!bytes) return RL_OK;
  if (!dst || !src) return fail(RL_EINVAL, "rl_memcopy: NULL pointer");
  hipStream_t s = (hipStream_t)stream;
  const bool dh = is_host(dst_space), sh = is_host(src_space);
  hipError_t e;
  if (!dh && !sh) return device_move((uint8_t*)dst, (const uint8_t*)src, bytes, s);
  if (dh && sh) {
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    memmove(dst, src, bytes);
    return RL_OK;
  }
  e = hipMemcpyAsync(dst, src, bytes, dh ? hipMemcpyDeviceToHost : hipMemcpyHostToDevice, s);
  return e == hipSuccess ? RL_OK : hip_fail(e, "hipMemcpyAsync");
}
