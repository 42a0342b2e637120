// Schema and layout descriptors, validation, conversion planning and the
// synchronous entry points of librelayout.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "plan.h"
#include "rl_internal.h"

namespace rl {

// ------------------------------------------------------------------ errors

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

rl_status fail(rl_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return st;
}

rl_status hip_fail(hipError_t e, const char* what) {
  return fail(RL_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// ------------------------------------------------------------------ device state

// Status words: slot k of a device's array belongs to the k-th stream that
// ran a conversion on that device in this process (slots are never
// reused; beyond kStatusSlots - 1 streams, the later ones share the last
// slot).  A slot is written only by kernels of its stream, so rl_sync can
// read and clear it on that stream without racing other streams.
static std::mutex g_dev_mu;
struct DeviceSlots {
  uint32_t* words = nullptr;                 // device address of the array
  std::map<hipStream_t, uint32_t> slot;      // stream -> slot
  uint32_t next = 0;
};
static std::map<int, DeviceSlots> g_slots;

static uint32_t* stream_status_on(int dev, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_dev_mu);
  DeviceSlots& d = g_slots[dev];
  if (!d.words) {
    uint32_t* w = nullptr;
    if (status_words(&w) != hipSuccess || !w) {
      (void)hipGetLastError();
      return nullptr;
    }
    d.words = w;
  }
  auto it = d.slot.find(s);
  if (it == d.slot.end()) {
    const uint32_t k = d.next < kStatusSlots - 1 ? d.next++ : kStatusSlots - 1;
    it = d.slot.emplace(s, k).first;
  }
  return d.words + it->second;
}

uint32_t* stream_status(hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  return stream_status_on(dev, s);
}

uint32_t type_size(rl_type t) {
  switch (t) {
    case RL_U8: case RL_I8: return 1;
    case RL_U16: case RL_I16: return 2;
    case RL_U32: case RL_I32: case RL_F32: return 4;
    default: return 8;
  }
}

static bool valid_type(int t) { return t >= RL_U8 && t <= RL_F64; }

static uint64_t round_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

}  // namespace rl

using namespace rl;

// ------------------------------------------------------------------ layouts

extern "C" rl_status rl_layout_create(const rl_schema* schema, const rl_layout_desc* desc,
                                      rl_layout** out) {
  if (!schema || !desc || !out) return fail(RL_EINVAL, "rl_layout_create: NULL argument");
  *out = nullptr;
  if (desc->kind < RL_AOS || desc->kind > RL_STRIDED) return fail(RL_EINVAL, "bad layout kind %d", (int)desc->kind);
  if (desc->space < RL_SPACE_DEVICE || desc->space > RL_SPACE_HOST_PINNED)
    return fail(RL_EINVAL, "bad memory space %d", (int)desc->space);
  auto* L = new rl_layout();
  L->schema = schema;
  L->kind = desc->kind;
  L->space = desc->space;
  L->width = desc->block_width;
  L->stride = 0;
  L->record_align = 1;
  L->has_gaps = false;
  L->indexed = false;
  const size_t nl = schema->leaves.size();
  for (size_t c = 0; c < nl; ++c) {
    const rl_type st = desc->storage_type ? desc->storage_type[c] : schema->leaves[c].type;
    const rl_type t = schema->leaves[c].type;
    if (!valid_type(st)) { delete L; return fail(RL_EINVAL, "leaf %zu: bad storage type", c); }
    if (st != t && !((t == RL_F64 && st == RL_F32) || (t == RL_F32 && st == RL_F64))) {
      delete L; return fail(RL_EINVAL, "leaf %zu: storage type may only change f64<->f32", c);
    }
    L->storage.push_back(st);
  }
  uint32_t acc = 0;
  for (size_t c = 0; c < nl; ++c) {
    L->prefix.push_back(acc);
    acc += type_size(L->storage[c]);
  }
  L->obj_bytes = acc;
  if (acc > (uint32_t)kMaxObjBytes) { delete L; return fail(RL_EINVAL, "more than %d bytes per object", kMaxObjBytes); }
  if (L->kind == RL_STRIDED) {
    if (!schema->members.empty()) {
      delete L;
      return fail(RL_EUNSUPPORTED, "strided layouts hold per-object leaves only (the schema has jagged groups)");
    }
    for (size_t c = 0; c < nl; ++c) {
      const uint64_t sz = type_size(L->storage[c]);
      const uint64_t st = desc->leaf_strides ? desc->leaf_strides[c] : sz;
      if (st == 0 || st % sz || st >= (1ull << 31)) {
        delete L;
        return fail(RL_EINVAL, "leaf %zu: stride %llu is not a non-zero multiple of %llu below 2^31", c,
                    (unsigned long long)st, (unsigned long long)sz);
      }
      L->leaf_stride.push_back(st);
    }
    L->indexed = desc->indexed != 0;
  }
  if (L->kind == RL_AOSOA) {
    // width 0: chosen by a batch ("auto"); buffers are sized for the widest candidate
    if (L->width >= 65536) { delete L; return fail(RL_EINVAL, "AoSoA block width must be 0..65535"); }
  }
  if (L->kind == RL_AOS) {
    std::vector<uint64_t> nat;
    uint64_t nat_stride;
    natural_record(schema, L->storage, nat, nat_stride);
    if (desc->slot_offsets) {
      L->slot_offsets.assign(desc->slot_offsets, desc->slot_offsets + schema->slots.size());
      L->stride = desc->record_stride;
    } else {
      L->slot_offsets = nat;
      L->stride = desc->record_stride ? desc->record_stride : nat_stride;
    }
    if (L->stride >= (1ull << 31)) { delete L; return fail(RL_EINVAL, "record stride too large"); }
    if (!schema->members.empty() && L->stride % 8)
      { delete L; return fail(RL_EINVAL, "records with jagged groups need a stride that is a multiple of 8"); }
    // slots inside the stride, not overlapping
    std::vector<std::pair<uint64_t, uint64_t>> spans;
    uint64_t covered = 0;
    for (size_t k = 0; k < schema->slots.size(); ++k) {
      const auto& sl = schema->slots[k];
      const uint64_t sz = sl.kind == 0 ? type_size(L->storage[sl.index]) : (sl.kind == 1 ? 8 : 4);
      const uint64_t o = L->slot_offsets[k];
      if (o + sz > L->stride) { delete L; return fail(RL_EINVAL, "slot %zu does not fit the record stride", k); }
      spans.push_back({o, o + sz});
      covered += sz;
      if (o % sz == 0) L->record_align = std::max<uint32_t>(L->record_align, (uint32_t)sz);
      if (sl.kind == 1 && o % 8) { delete L; return fail(RL_EINVAL, "group pointer slot must be 8-byte aligned"); }
      if (sl.kind == 2 && o % 4) { delete L; return fail(RL_EINVAL, "group count slot must be 4-byte aligned"); }
    }
    std::sort(spans.begin(), spans.end());
    for (size_t k = 1; k < spans.size(); ++k)
      if (spans[k].first < spans[k - 1].second) { delete L; return fail(RL_EINVAL, "record slots overlap"); }
    L->has_gaps = covered < L->stride;
    L->leaf_offset.assign(nl, 0);
    L->ptr_off.assign(schema->offset_types.size(), 0);
    L->len_off.assign(schema->offset_types.size(), 0);
    for (size_t k = 0; k < schema->slots.size(); ++k) {
      const auto& sl = schema->slots[k];
      if (sl.kind == 0) L->leaf_offset[sl.index] = (uint32_t)L->slot_offsets[k];
      else if (sl.kind == 1) L->ptr_off[sl.index] = (uint32_t)L->slot_offsets[k];
      else L->len_off[sl.index] = (uint32_t)L->slot_offsets[k];
    }
    for (uint32_t g = 0; g < (uint32_t)schema->members.size(); ++g) {
      std::vector<uint32_t> mo;
      uint32_t ms = 0, ma = 1;
      natural_member_record(schema, g, mo, ms, ma);
      L->moff.push_back(mo);
      L->mstride.push_back(ms);
      L->malign.push_back(ma);
    }
  }
  *out = L;
  return RL_OK;
}

extern "C" void rl_layout_destroy(rl_layout* layout) { delete layout; }

namespace rl {

uint32_t layout_n_buffers(const rl_layout* L) {
  const rl_schema* s = L->schema;
  uint32_t n = 0;
  if (L->kind == RL_AOS) return 1 + (uint32_t)s->members.size();
  if (L->kind == RL_STRIDED) return (uint32_t)s->leaves.size() + (L->indexed ? 1 : 0);
  n = L->kind == RL_SOA ? (uint32_t)s->leaves.size() : 1;
  for (const auto& m : s->members) n += 1 + (uint32_t)m.size();
  return n;
}

void layout_buffer_bytes(const rl_layout* L, uint64_t n, const uint64_t* members, uint64_t* bytes) {
  const rl_schema* s = L->schema;
  uint32_t k = 0;
  if (L->kind == RL_AOS) {
    bytes[k++] = n * L->stride;
    for (size_t g = 0; g < s->members.size(); ++g) bytes[k++] = (members ? members[g] : 0) * L->mstride[g];
    return;
  }
  if (L->kind == RL_STRIDED) {
    for (size_t c = 0; c < s->leaves.size(); ++c)
      bytes[k++] = n ? (n - 1) * L->leaf_stride[c] + type_size(L->storage[c]) : 0;
    if (L->indexed) bytes[k++] = n * 8;
    return;
  }
  if (L->kind == RL_SOA) {
    for (size_t c = 0; c < s->leaves.size(); ++c) bytes[k++] = n * type_size(L->storage[c]);
  } else {
    const uint64_t w = L->width ? L->width : kAutoWidthMax;
    bytes[k++] = (n + w - 1) / w * w * (uint64_t)L->obj_bytes;
  }
  for (size_t g = 0; g < s->members.size(); ++g) {
    bytes[k++] = (n + 1) * type_size(s->offset_types[g]);
    for (const auto& m : s->members[g]) bytes[k++] = (members ? members[g] : 0) * m.size;
  }
}

// Alignment each buffer needs.
void layout_buffer_align(const rl_layout* L, uint64_t* align) {
  const rl_schema* s = L->schema;
  uint32_t k = 0;
  if (L->kind == RL_AOS) {
    align[k++] = L->record_align;
    for (size_t g = 0; g < s->members.size(); ++g) align[k++] = L->malign[g];
    return;
  }
  if (L->kind == RL_STRIDED) {
    for (size_t c = 0; c < s->leaves.size(); ++c) align[k++] = type_size(L->storage[c]);
    if (L->indexed) align[k++] = 8;
    return;
  }
  if (L->kind == RL_SOA) {
    for (size_t c = 0; c < s->leaves.size(); ++c) align[k++] = type_size(L->storage[c]);
  } else {
    uint64_t a = 1;
    for (auto t : L->storage) a = std::max<uint64_t>(a, type_size(t));
    align[k++] = a;
  }
  for (size_t g = 0; g < s->members.size(); ++g) {
    align[k++] = type_size(s->offset_types[g]);
    for (const auto& m : s->members[g]) align[k++] = m.size;
  }
}

// First buffer index of group g's storage.
uint32_t group_buffer(const rl_layout* L, uint32_t g) {
  const rl_schema* s = L->schema;
  if (L->kind == RL_AOS) return 1 + g;
  uint32_t k = L->kind == RL_SOA ? (uint32_t)s->leaves.size() : 1;
  for (uint32_t h = 0; h < g; ++h) k += 1 + (uint32_t)s->members[h].size();
  return k;
}

}  // namespace rl

extern "C" rl_status rl_layout_buffers(const rl_layout* L, uint64_t n, const uint64_t* n_members,
                                       uint32_t* n_buffers, uint64_t* bytes) {
  if (!L || !n_buffers) return fail(RL_EINVAL, "rl_layout_buffers: NULL argument");
  if (!L->schema->members.empty() && !n_members && bytes)
    return fail(RL_EINVAL, "rl_layout_buffers: n_members needed for jagged groups");
  *n_buffers = layout_n_buffers(L);
  if (bytes) layout_buffer_bytes(L, n, n_members, bytes);
  return RL_OK;
}

extern "C" rl_status rl_layout_info(const rl_layout* L, uint64_t* slot_offsets, uint64_t* stride,
                                    uint32_t* max_buffers) {
  if (!L) return fail(RL_EINVAL, "layout is NULL");
  if (slot_offsets && L->kind == RL_AOS)
    std::copy(L->slot_offsets.begin(), L->slot_offsets.end(), slot_offsets);
  if (stride) *stride = L->stride;
  if (max_buffers) *max_buffers = layout_n_buffers(L);
  return RL_OK;
}

// ------------------------------------------------------------------ validation

namespace rl {

rl_status validate_view(const rl_view* v, uint64_t n, const char* which, std::vector<Range>* ranges,
                        bool want_device) {
  if (!v || !v->layout) return fail(RL_EINVAL, "%s: view or layout is NULL", which);
  const rl_layout* L = v->layout;
  const size_t ng = L->schema->members.size();
  if (ng && !v->member_capacity) return fail(RL_EINVAL, "%s: member_capacity needed", which);
  if (n > v->capacity) return fail(RL_EINVAL, "%s: n = %llu exceeds capacity %llu", which,
                                   (unsigned long long)n, (unsigned long long)v->capacity);
  if (want_device && L->space != RL_SPACE_DEVICE)
    return fail(RL_EUNSUPPORTED, "%s: expected device memory", which);
  const uint32_t nb = layout_n_buffers(L);
  if (nb && !v->buffers) return fail(RL_EINVAL, "%s: buffers is NULL", which);
  std::vector<uint64_t> bytes(nb), align(nb);
  // an indexed strided view's objects may reach any of its `capacity`
  // elements
  const uint64_t reach = L->kind == RL_STRIDED && L->indexed ? v->capacity : n;
  layout_buffer_bytes(L, reach, v->member_capacity, bytes.data());
  layout_buffer_align(L, align.data());
  for (uint32_t b = 0; b < nb; ++b) {
    const uintptr_t p = (uintptr_t)v->buffers[b];
    if (bytes[b] == 0) continue;
    if (!p) return fail(RL_EINVAL, "%s: buffer %u is NULL", which, b);
    if (p % align[b]) return fail(RL_EALIGN, "%s: buffer %u not aligned to %llu bytes", which, b,
                                  (unsigned long long)align[b]);
    if (ranges) ranges->push_back({p, p + bytes[b]});
  }
  return RL_OK;
}

rl_status check_overlap(const std::vector<Range>& src, const std::vector<Range>& dst, bool dst_shared) {
  for (size_t i = 0; i < dst.size(); ++i) {
    for (const auto& s : src)
      if (dst[i].lo < s.hi && s.lo < dst[i].hi) return fail(RL_EOVERLAP, "a destination buffer overlaps a source buffer");
    if (dst_shared) continue;
    for (size_t j = 0; j < i; ++j)
      if (dst[i].lo < dst[j].hi && dst[j].lo < dst[i].hi) return fail(RL_EOVERLAP, "destination buffers overlap");
  }
  return RL_OK;
}

}  // namespace rl

// ------------------------------------------------------------------ convert

namespace rl {
// Tile shape override for experiments and the tile-independence tests:
// RL_TILE_OBJECTS (objects per tile), RL_BLOCK_THREADS, RL_GRID_BLOCKS;
// RL_DST_DIRECT, RL_SOURCE_DMA, RL_JAGGED_FUSED and RL_PIPELINE (0 turns a path off;
// RL_PIPELINE=1 double-buffers every dense step where two tile slots fit;
// RL_JAGGED_FUSED=2 makes a jagged records conversion fail with
// RL_EUNSUPPORTED where the single-pass kernel does not apply).
PlanShape shape_from_env() {
  PlanShape s;
  if (const char* v = getenv("RL_TILE_OBJECTS")) s.tile = (uint32_t)strtoul(v, nullptr, 10);
  if (const char* v = getenv("RL_BLOCK_THREADS")) {
    const uint32_t t = (uint32_t)strtoul(v, nullptr, 10);
    if (t >= 64 && t <= 1024 && t % 64 == 0) s.threads = t;
  }
  if (const char* v = getenv("RL_GRID_BLOCKS")) s.grid = (uint32_t)strtoul(v, nullptr, 10);
  if (const char* v = getenv("RL_DST_DIRECT")) s.direct = atoi(v) ? -1 : 0;
  if (const char* v = getenv("RL_SOURCE_DMA")) s.dma = atoi(v) ? -1 : 0;
  if (const char* v = getenv("RL_JAGGED_FUSED")) s.fused = atoi(v) == 2 ? 2 : atoi(v) ? -1 : 0;
  if (const char* v = getenv("RL_PIPELINE")) s.pipe = atoi(v) == 1 ? 1 : atoi(v) ? -1 : 0;
  if (const char* v = getenv("RL_STREAM_STORES")) s.stream = atoi(v) ? 1 : 0;
  return s;
}
}  // namespace rl

namespace rl {
bool auto_width(const rl_view* v) {
  return v && v->layout && v->layout->kind == RL_AOSOA && v->layout->width == 0;
}
}  // namespace rl

extern "C" rl_status rl_convert(const rl_view* src, const rl_view* dst, uint64_t n, void* stream) {
  std::vector<Range> rs, rd;
  rl_status st = validate_view(src, n, "src", &rs, true);
  if (st) return st;
  st = validate_view(dst, n, "dst", &rd, true);
  if (st) return st;
  if (auto_width(src) || auto_width(dst)) return fail(RL_EINVAL, "block width 0 (auto) is only for batches");
  if (src->layout->schema != dst->layout->schema) return fail(RL_EINVAL, "src and dst use different schemas");
  if ((st = check_overlap(rs, rd, dst->layout->kind == RL_STRIDED))) return st;
  if (!src->layout->schema->members.empty() && src->layout->kind == RL_AOS && dst->layout->kind == RL_AOS)
    return fail(RL_EUNSUPPORTED, "AoS -> AoS conversion of a schema with jagged groups");
  if (n == 0) return RL_OK;
  bool handled = false;
  st = run_specialisations(src, dst, n, stream, &handled);
  if (handled) return st;
  if (src->layout->kind == RL_STRIDED || dst->layout->kind == RL_STRIDED)
    return convert_general(*src, *dst, n, (hipStream_t)stream);
  Plan plan;
  PlanShape shape = shape_from_env();
  if (stream_capturing((hipStream_t)stream)) shape.fused = 0;
  if ((st = make_plan(*src, *dst, n, shape, &plan))) return st;
  return enqueue_plan(plan, (hipStream_t)stream);
}

extern "C" rl_status rl_offsets(const rl_view* src, const rl_view* dst, uint32_t group, uint64_t n,
                                uint64_t* total_host, void* stream) {
  std::vector<Range> rs, rd;
  rl_status st = validate_view(src, n, "src", &rs, true);
  if (st) return st;
  st = validate_view(dst, n, "dst", &rd, true);
  if (st) return st;
  if (src->layout->schema != dst->layout->schema) return fail(RL_EINVAL, "src and dst use different schemas");
  if (group >= src->layout->schema->members.size()) return fail(RL_EINVAL, "no jagged group %u", group);
  if (auto_width(src) || auto_width(dst)) return fail(RL_EINVAL, "block width 0 (auto) is only for batches");
  if (dst->layout->kind == RL_AOS) return fail(RL_EUNSUPPORTED, "rl_offsets writes an offsets column (SoA/AoSoA dst)");
  // only the offsets column of dst is written
  const uint32_t ob = group_buffer(dst->layout, group);
  std::vector<Range> rd1;
  for (const auto& r : rd)
    if (r.lo == (uintptr_t)dst->buffers[ob]) rd1.push_back(r);
  if ((st = check_overlap(rs, rd1))) return st;
  Plan plan;
  if ((st = make_offsets_plan(*src, *dst, group, n, shape_from_env(), &plan))) return st;
  if ((st = enqueue_plan(plan, (hipStream_t)stream))) return st;
  if (total_host) {
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    const rl_type ot = src->layout->schema->offset_types[group];
    uint64_t v = 0;
    e = hipMemcpy(&v, (const uint8_t*)dst->buffers[ob] + n * type_size(ot), type_size(ot), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    if (ot == RL_I32) v = (uint64_t)(int64_t)(int32_t)(uint32_t)v;
    *total_host = v;
  }
  return RL_OK;
}

namespace rl {
rl_status status_of_flags(uint32_t f) {
  if (f & ST_FLAG_OVERFLOW) return fail(RL_EOVERFLOW, "a member total does not fit the offset type");
  if (f & ST_FLAG_CAPACITY) return fail(RL_ECAPACITY, "members exceed the destination capacity");
  if (f & ST_FLAG_BOUNDS) return fail(RL_EBOUNDS, "a source member block lies outside its storage or is misaligned");
  return RL_OK;
}
}  // namespace rl

// Per-thread pinned word that rl_sync receives a stream's flags in.
static thread_local uint32_t* t_sync_word = nullptr;

extern "C" rl_status rl_sync(void* stream) {
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  uint32_t* ds = stream_status(s);
  if (!ds) return fail(RL_EHIP, "status words of the current device");
  if (!t_sync_word) {
    // leaked at thread exit (4 bytes of pinned memory per thread that syncs)
    if ((e = hipHostMalloc((void**)&t_sync_word, 64, hipHostMallocDefault)) != hipSuccess)
      return hip_fail(e, "hipHostMalloc(status)");
  }
  uint32_t* dev_alias = nullptr;
  if ((e = hipHostGetDevicePointer((void**)&dev_alias, t_sync_word, 0)) != hipSuccess)
    return hip_fail(e, "hipHostGetDevicePointer(status)");
  *t_sync_word = 0;
  if ((e = launch_take_status(ds, dev_alias, s)) != hipSuccess) return hip_fail(e, "take status");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return status_of_flags(*(volatile uint32_t*)t_sync_word);
}

extern "C" const char* rl_last_error(void) { return g_err; }
