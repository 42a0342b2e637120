// Collections that own their buffers in a memory context (Sec. VII-A: every
// collection has a memory context that says how memory is allocated,
// deallocated and set; update_memory_context_info allocates with the new
// context information, copies from the old memory and frees it).  The
// context here is the layout's space: device memory (hipMalloc), pinned
// host memory (hipHostMalloc) or pageable host memory (malloc).
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "plan.h"
#include "rl_internal.h"

struct rl_collection {
  const rl_layout* layout = nullptr;
  uint64_t capacity = 0;
  std::vector<uint64_t> member_capacity;
  std::vector<void*> buffers;
  std::vector<uint64_t> bytes;
};

namespace rl {

namespace {

void free_buffers(rl_space space, std::vector<void*>& bufs) {
  for (void*& p : bufs) {
    if (!p) continue;
    if (space == RL_SPACE_DEVICE) (void)hipFree(p);
    else if (space == RL_SPACE_HOST_PINNED) (void)hipHostFree(p);
    else free(p);
    p = nullptr;
  }
}

// Buffers of `layout` for the given capacities, zero-filled (device memory
// by a kernel on `stream`, host memory at once).
rl_status alloc_buffers(const rl_layout* L, uint64_t capacity, const uint64_t* mcap, hipStream_t s,
                        std::vector<void*>* bufs, std::vector<uint64_t>* bytes) {
  const uint32_t nb = layout_n_buffers(L);
  bytes->assign(nb, 0);
  layout_buffer_bytes(L, capacity, mcap, bytes->data());
  bufs->assign(nb, nullptr);
  for (uint32_t b = 0; b < nb; ++b) {
    const uint64_t sz = std::max<uint64_t>((*bytes)[b], 1);   // every buffer distinct and non-null
    hipError_t e = hipSuccess;
    void* p = nullptr;
    if (L->space == RL_SPACE_DEVICE) e = hipMalloc(&p, sz);
    else if (L->space == RL_SPACE_HOST_PINNED) e = hipHostMalloc(&p, sz, hipHostMallocDefault);
    else p = aligned_alloc(256, (sz + 255) & ~255ull);
    if (e != hipSuccess || !p) {
      free_buffers(L->space, *bufs);
      return fail(RL_ENOMEM, "buffer %u of %llu bytes: %s", b, (unsigned long long)sz,
                  e != hipSuccess ? hipGetErrorString(e) : "out of host memory");
    }
    (*bufs)[b] = p;
    if (L->space == RL_SPACE_DEVICE) {
      if ((e = launch_zero_bytes(p, sz, s)) != hipSuccess) {
        free_buffers(L->space, *bufs);
        return hip_fail(e, "zero");
      }
    } else {
      memset(p, 0, sz);
    }
  }
  return RL_OK;
}

rl_view view_of(const rl_collection* c) {
  return rl_view{c->layout, c->capacity, c->member_capacity.empty() ? nullptr : c->member_capacity.data(),
                 c->buffers.data()};
}

}  // namespace

}  // namespace rl

using namespace rl;

extern "C" rl_status rl_collection_create(const rl_layout* layout, uint64_t capacity, const uint64_t* member_capacity,
                                          void* stream, rl_collection** out) {
  if (!layout || !out) return fail(RL_EINVAL, "rl_collection_create: NULL argument");
  *out = nullptr;
  if (layout->kind == RL_AOSOA && layout->width == 0)
    return fail(RL_EINVAL, "block width 0 (auto) is only for batches");
  if (layout->kind == RL_STRIDED) return fail(RL_EUNSUPPORTED, "a strided layout's memory belongs to its user");
  const size_t ng = layout->schema->members.size();
  if (ng && !member_capacity) return fail(RL_EINVAL, "member capacities needed");
  auto c = new rl_collection();
  c->layout = layout;
  c->capacity = capacity;
  if (ng) c->member_capacity.assign(member_capacity, member_capacity + ng);
  rl_status st = alloc_buffers(layout, capacity, c->member_capacity.empty() ? nullptr : c->member_capacity.data(),
                               (hipStream_t)stream, &c->buffers, &c->bytes);
  if (st) {
    delete c;
    return st;
  }
  *out = c;
  return RL_OK;
}

extern "C" rl_status rl_collection_view(const rl_collection* c, rl_view* out) {
  if (!c || !out) return fail(RL_EINVAL, "rl_collection_view: NULL argument");
  *out = view_of(c);
  return RL_OK;
}

extern "C" rl_status rl_collection_rehome(rl_collection* c, const rl_layout* layout, uint64_t n, void* stream) {
  if (!c || !layout) return fail(RL_EINVAL, "rl_collection_rehome: NULL argument");
  if (layout->schema != c->layout->schema) return fail(RL_EINVAL, "a layout of another schema");
  if (layout->kind == RL_AOSOA && layout->width == 0) return fail(RL_EINVAL, "block width 0 (auto) is only for batches");
  if (layout->kind == RL_STRIDED) return fail(RL_EUNSUPPORTED, "a strided layout's memory belongs to its user");
  if (n > c->capacity) return fail(RL_EINVAL, "n %llu over the capacity %llu", (unsigned long long)n,
                                   (unsigned long long)c->capacity);
  if (!c->layout->schema->members.empty() && c->layout->kind == RL_AOS && layout->kind == RL_AOS)
    return fail(RL_EUNSUPPORTED, "AoS -> AoS conversion of a schema with jagged groups");
  hipStream_t s = (hipStream_t)stream;
  std::vector<void*> nb;
  std::vector<uint64_t> bytes;
  const uint64_t* mcap = c->member_capacity.empty() ? nullptr : c->member_capacity.data();
  rl_status st = alloc_buffers(layout, c->capacity, mcap, s, &nb, &bytes);
  if (st) return st;
  const rl_view src = view_of(c);
  const rl_view dst{layout, c->capacity, mcap, nb.data()};
  const bool sh = is_host(c->layout->space), dh = is_host(layout->space);
  std::vector<void*> tmp;
  if (n) {
    if (!sh && !dh) {
      st = rl_convert(&src, &dst, n, stream);
    } else if (sh != dh) {
      st = rl_transfer(&src, &dst, n, stream, nullptr);
    } else {
      // host to host: through a device copy of the new layout
      rl_layout dl = *layout;
      dl.space = RL_SPACE_DEVICE;
      std::vector<uint64_t> tb;
      st = alloc_buffers(&dl, c->capacity, mcap, s, &tmp, &tb);
      const rl_view mid{&dl, c->capacity, mcap, tmp.data()};
      if (!st) st = rl_transfer(&src, &mid, n, stream, nullptr);
      for (size_t b = 0; b < nb.size() && !st; ++b) {
        hipError_t e = hipMemcpyAsync(nb[b], tmp[b], bytes[b], hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) st = hip_fail(e, "hipMemcpyAsync");
      }
    }
  }
  // the old memory (and any temporary) may be freed once the copy is done
  hipError_t e = hipStreamSynchronize(s);
  if (!st && e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
  free_buffers(RL_SPACE_DEVICE, tmp);
  if (st) {
    free_buffers(layout->space, nb);
    return st;
  }
  free_buffers(c->layout->space, c->buffers);
  c->layout = layout;
  c->buffers = nb;
  c->bytes = bytes;
  return RL_OK;
}

extern "C" void rl_collection_destroy(rl_collection* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();   // kernels may still use device buffers
  free_buffers(c->layout->space, c->buffers);
  delete c;
}
