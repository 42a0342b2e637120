// Insertion, deletion and compaction on collections in device memory
// (Sec. VII-B: the layout holder's insert and erase act on the arrays of
// every property; a filtered collection is compacted).  Each is a gather of
// existing objects into new positions:
//  - rl_select: the flagged objects, in order, into another view (a scan of
//    the flags gives every kept object its place; members of jagged groups
//    follow, their offsets from a second scan);
//  - rl_erase / rl_insert: in place; the objects after the gap move with
//    memmove semantics (AoS records and SoA columns as overlapping byte
//    ranges; AoSoA blocks object by object through a scratch band), the
//    inserted objects are converted into the opened slots.
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "plan.h"
#include "rl_internal.h"

namespace rl {

namespace {

constexpr uint64_t kBandBytes = 64ull << 20;

struct ScratchBuf {
  uint8_t* ptr = nullptr;
  uint64_t bytes = 0;
};
std::mutex g_edit_mu;
std::map<std::pair<int, hipStream_t>, ScratchBuf> g_edit;   // held until the process ends

// The stream's scratch with room for `need` bytes (caller holds g_edit_mu
// until its work is enqueued).
rl_status edit_scratch(hipStream_t s, uint64_t need, uint8_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  ScratchBuf& b = g_edit[{dev, s}];
  if (b.bytes < need) {
    if (b.ptr) {
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
      (void)hipFree(b.ptr);
      b.ptr = nullptr;
      b.bytes = 0;
    }
    const uint64_t want = std::max<uint64_t>((need + 255) & ~255ull, 1 << 20);
    if ((e = hipMalloc((void**)&b.ptr, want)) != hipSuccess)
      return fail(RL_ENOMEM, "scratch of %llu bytes: %s", (unsigned long long)want, hipGetErrorString(e));
    b.bytes = want;
  }
  *out = b.ptr;
  return RL_OK;
}

// `capacity`: the view's capacity (the elements of an indexed strided side).
GenSide gen_side(const rl_layout* L, void* const* bufs, uint64_t capacity = 0) {
  GenSide s;
  memset(&s, 0, sizeof s);
  s.kind = (uint32_t)L->kind;
  const size_t nl = L->storage.size();
  if (L->kind == RL_STRIDED) {
    for (size_t c = 0; c < nl; ++c) {
      s.col[c] = (uint8_t*)bufs[c];
      s.off[c] = (uint32_t)L->leaf_stride[c];
    }
    if (L->indexed) {
      s.index = (const uint64_t*)bufs[nl];
      s.elements = capacity;
    }
  } else if (L->kind == RL_AOS) {
    s.base = (uint8_t*)bufs[0];
    s.stride = (uint32_t)L->stride;
    for (size_t c = 0; c < nl; ++c) s.off[c] = L->leaf_offset[c];
  } else if (L->kind == RL_SOA) {
    for (size_t c = 0; c < nl; ++c) s.col[c] = (uint8_t*)bufs[c];
  } else {
    s.base = (uint8_t*)bufs[0];
    s.width = L->width;
    s.obj_bytes = L->obj_bytes;
    for (size_t c = 0; c < nl; ++c) s.off[c] = L->prefix[c];
  }
  return s;
}

// SoA columns of `cap` objects packed one after the other in `base` (a
// scratch band for the leaves of layout L).
GenSide scratch_side(const rl_layout* L, uint8_t* base, uint64_t cap) {
  GenSide s;
  memset(&s, 0, sizeof s);
  s.kind = KIND_SOA;
  uint64_t at = 0;
  for (size_t c = 0; c < L->storage.size(); ++c) {
    s.col[c] = base + at;
    at += (cap * type_size(L->storage[c]) + 15) & ~15ull;
  }
  return s;
}

uint64_t scratch_side_bytes(const rl_layout* L, uint64_t cap) {
  uint64_t at = 0;
  for (size_t c = 0; c < L->storage.size(); ++c) at += (cap * type_size(L->storage[c]) + 15) & ~15ull;
  return at;
}

rl_status move_desc(const rl_layout* SL, const GenSide& s, const rl_layout* DL, const GenSide& d, MoveDesc* out) {
  MoveDesc& m = *out;
  memset(&m, 0, sizeof m);
  m.src = s;
  m.dst = d;
  m.n_leaves = (uint32_t)SL->storage.size();
  for (uint32_t c = 0; c < m.n_leaves; ++c) {
    const rl_type a = SL->storage[c], b = DL->storage[c];
    m.src_size[c] = (uint8_t)type_size(a);
    m.dst_size[c] = (uint8_t)type_size(b);
    if (a == b) m.op[c] = OP_COPY;
    else if (a == RL_F64 && b == RL_F32) m.op[c] = OP_NARROW;
    else if (a == RL_F32 && b == RL_F64) m.op[c] = OP_WIDEN;
    else return fail(RL_EUNSUPPORTED, "leaf %u: storage types %d -> %d", c, (int)a, (int)b);
  }
  return RL_OK;
}

GenGroup gen_group(const rl_layout* L, void* const* bufs, uint32_t g, uint64_t capacity) {
  GenGroup G;
  memset(&G, 0, sizeof G);
  const rl_schema* sc = L->schema;
  const uint32_t gb = group_buffer(L, g);
  G.n_members = (uint32_t)sc->members[g].size();
  G.capacity = capacity;
  for (uint32_t m = 0; m < G.n_members; ++m) G.msize[m] = (uint8_t)sc->members[g][m].size;
  if (L->kind == RL_AOS) {
    G.form = 0;
    G.records = (uint8_t*)bufs[0];
    G.rec_stride = (uint32_t)L->stride;
    G.ptr_off = L->ptr_off[g];
    G.len_off = L->len_off[g];
    G.mstride = L->mstride[g];
    G.malign = L->malign[g];
    G.pool = (uint8_t*)bufs[gb];
    for (uint32_t m = 0; m < G.n_members; ++m) G.moff[m] = L->moff[g][m];
  } else {
    G.form = 1;
    G.offsets = (uint8_t*)bufs[gb];
    G.off_type = (uint32_t)sc->offset_types[g];
    for (uint32_t m = 0; m < G.n_members; ++m) G.mcol[m] = (uint8_t*)bufs[gb + 1 + m];
  }
  return G;
}

rl_status launch_or_fail(hipError_t e, const char* what) { return e == hipSuccess ? RL_OK : hip_fail(e, what); }

// Zero the unused slots of the last block of an AoSoA view holding n objects.
rl_status zero_block_tail(const rl_layout* L, void* const* bufs, uint64_t n, hipStream_t s) {
  if (L->kind != RL_AOSOA) return RL_OK;
  const uint64_t end = (n + L->width - 1) / L->width * L->width;
  if (end == n) return RL_OK;
  MoveDesc m;
  GenSide d = gen_side(L, bufs);
  rl_status st = move_desc(L, d, L, d, &m);
  if (st) return st;
  m.zero_only = 1;
  m.count = end - n;
  m.dst0 = n;
  return launch_or_fail(launch_move(m, m.count, s), "zero block tail");
}

// Objects [from, from + count) of a view move to [to, to + count), as if
// through a separate buffer (memmove semantics).
rl_status shift_objects(const rl_view& v, uint64_t from, uint64_t to, uint64_t count, hipStream_t s) {
  if (!count || from == to) return RL_OK;
  const rl_layout* L = v.layout;
  if (L->kind == RL_AOS) {
    uint8_t* rec = (uint8_t*)v.buffers[0];
    return device_move(rec + to * L->stride, rec + from * L->stride, count * L->stride, s);
  }
  if (L->kind == RL_SOA) {
    for (size_t c = 0; c < L->storage.size(); ++c) {
      uint8_t* col = (uint8_t*)v.buffers[c];
      const uint64_t sz = type_size(L->storage[c]);
      rl_status st = device_move(col + to * sz, col + from * sz, count * sz, s);
      if (st) return st;
    }
    return RL_OK;
  }
  // AoSoA: bands of objects through scratch, in the order that keeps every
  // band's source intact (from the front when moving down)
  const uint64_t per = std::max<uint64_t>(1, kBandBytes / std::max<uint32_t>(1, L->obj_bytes));
  const uint64_t band = std::min(per, count);
  std::lock_guard<std::mutex> lk(g_edit_mu);
  uint8_t* tmp = nullptr;
  rl_status st = edit_scratch(s, scratch_side_bytes(L, band), &tmp);
  if (st) return st;
  const GenSide view = gen_side(L, v.buffers), sc = scratch_side(L, tmp, band);
  const bool down = to < from;
  for (uint64_t done = 0; done < count;) {
    const uint64_t len = std::min(band, count - done);
    const uint64_t at = down ? done : count - done - len;
    MoveDesc a, b;
    if ((st = move_desc(L, view, L, sc, &a)) || (st = move_desc(L, sc, L, view, &b))) return st;
    a.count = b.count = len;
    a.src0 = from + at;
    b.dst0 = to + at;
    if ((st = launch_or_fail(launch_move(a, len, s), "move")) || (st = launch_or_fail(launch_move(b, len, s), "move")))
      return st;
    done += len;
  }
  return RL_OK;
}

}  // namespace

}  // namespace rl

using namespace rl;

extern "C" rl_status rl_select(const rl_view* src, const rl_view* dst, uint64_t n, const uint8_t* keep,
                               uint64_t* n_kept, void* stream) {
  std::vector<Range> rs, rd;
  rl_status st = validate_view(src, n, "src", &rs, true);
  if (st) return st;
  if ((st = validate_view(dst, n, "dst", &rd, true))) return st;
  if (src->layout->schema != dst->layout->schema) return fail(RL_EINVAL, "src and dst use different schemas");
  if (auto_width(src) || auto_width(dst)) return fail(RL_EINVAL, "block width 0 (auto) is only for batches");
  if ((st = check_overlap(rs, rd, dst->layout->kind == RL_STRIDED))) return st;
  if (n && !keep) return fail(RL_EINVAL, "rl_select: keep is NULL");
  hipStream_t s = (hipStream_t)stream;
  const rl_layout* SL = src->layout;
  const rl_layout* DL = dst->layout;
  const uint32_t ng = (uint32_t)SL->schema->members.size();
  const uint64_t tiles = (n + kSelectTile - 1) / kSelectTile;
  // scratch: tile totals, kept indices, kept count, member offsets
  const uint64_t need = std::max<uint64_t>(1, tiles) * 8 + n * 8 + 64 + (n + 1) * 8;
  std::lock_guard<std::mutex> lk(g_edit_mu);
  uint8_t* tmp = nullptr;
  if ((st = edit_scratch(s, need, &tmp))) return st;
  uint32_t* status = stream_status(s);
  if (!status) return fail(RL_EHIP, "status words of the current device");
  SelectDesc sd;
  memset(&sd, 0, sizeof sd);
  sd.keep = keep;
  sd.n = n;
  sd.tile_tot = (uint64_t*)tmp;
  sd.map = sd.tile_tot + std::max<uint64_t>(1, tiles);
  sd.count = sd.map + n;
  sd.count_out = n_kept;
  sd.lens = sd.count + 8;
  sd.status = status;
  if ((st = launch_or_fail(launch_select(sd, s), "select"))) return st;
  // destination slots that no kept object fills stay zero (record padding,
  // unused block slots)
  if (DL->kind == RL_AOSOA) {
    const uint64_t bytes = (n + DL->width - 1) / DL->width * DL->width * (uint64_t)DL->obj_bytes;
    if ((st = launch_or_fail(launch_zero_bytes(dst->buffers[0], bytes, s), "zero"))) return st;
  } else if (DL->kind == RL_AOS && DL->has_gaps) {
    if ((st = launch_or_fail(launch_zero_bytes(dst->buffers[0], n * DL->stride, s), "zero"))) return st;
  }
  MoveDesc m;
  if ((st = move_desc(SL, gen_side(SL, src->buffers, src->capacity), DL, gen_side(DL, dst->buffers, dst->capacity),
                      &m)))
    return st;
  m.count_dev = sd.count;
  m.map = sd.map;
  m.status = status;
  if ((st = launch_or_fail(launch_move(m, n, s), "move"))) return st;
  for (uint32_t g = 0; g < ng; ++g) {
    sd.src = gen_group(SL, src->buffers, g, src->member_capacity[g]);
    if ((st = launch_or_fail(launch_select_members(sd, s), "select members"))) return st;
    MemberMoveDesc mm;
    memset(&mm, 0, sizeof mm);
    mm.src = sd.src;
    mm.dst = gen_group(DL, dst->buffers, g, dst->member_capacity[g]);
    mm.map = sd.map;
    mm.count_dev = sd.count;
    mm.out_off = sd.lens;
    mm.n_max = n;
    mm.status = status;
    if ((st = launch_or_fail(launch_member_move(mm, s), "member move"))) return st;
  }
  return RL_OK;
}

namespace rl {

rl_status convert_general(const rl_view& src, const rl_view& dst, uint64_t n, hipStream_t s) {
  const rl_layout* SL = src.layout;
  const rl_layout* DL = dst.layout;
  uint32_t* status = stream_status(s);
  if (!status) return fail(RL_EHIP, "status words of the current device");
  rl_status st;
  // the padding bytes of destination records are zero, as in every conversion
  if (DL->kind == RL_AOS && DL->has_gaps &&
      (st = launch_or_fail(launch_zero_bytes(dst.buffers[0], n * DL->stride, s), "zero")))
    return st;
  MoveDesc m;
  if ((st = move_desc(SL, gen_side(SL, src.buffers, src.capacity), DL, gen_side(DL, dst.buffers, dst.capacity), &m)))
    return st;
  m.count = n;
  m.status = status;
  if ((st = launch_or_fail(launch_move(m, n, s), "move"))) return st;
  return zero_block_tail(DL, dst.buffers, n, s);
}

}  // namespace rl

extern "C" rl_status rl_erase(const rl_view* view, uint64_t n, uint64_t at, uint64_t count, void* stream) {
  std::vector<Range> rv;
  rl_status st = validate_view(view, n, "view", &rv, true);
  if (st) return st;
  if (auto_width(view)) return fail(RL_EINVAL, "block width 0 (auto) is only for batches");
  if (view->layout->kind == RL_STRIDED) return fail(RL_EUNSUPPORTED, "erase on a strided view");
  if (at > n || count > n - at) return fail(RL_EINVAL, "erase [%llu, %llu) outside %llu objects",
                                            (unsigned long long)at, (unsigned long long)(at + count),
                                            (unsigned long long)n);
  if (!count) return RL_OK;
  hipStream_t s = (hipStream_t)stream;
  const bool jagged = !view->layout->schema->members.empty();
  if (jagged && at + count != n)
    return fail(RL_EUNSUPPORTED, "erasing objects before the end of a collection with jagged groups");
  if ((st = shift_objects(*view, at + count, at, n - at - count, s))) return st;
  return zero_block_tail(view->layout, view->buffers, n - count, s);
}

extern "C" rl_status rl_insert(const rl_view* view, uint64_t n, uint64_t at, const rl_view* src, uint64_t count,
                               void* stream) {
  std::vector<Range> rv, rs;
  rl_status st = validate_view(view, n, "view", &rv, true);
  if (st) return st;
  if ((st = validate_view(src, count, "src", &rs, true))) return st;
  if (view->layout->schema != src->layout->schema) return fail(RL_EINVAL, "view and src use different schemas");
  if (auto_width(view) || auto_width(src)) return fail(RL_EINVAL, "block width 0 (auto) is only for batches");
  if (view->layout->kind == RL_STRIDED) return fail(RL_EUNSUPPORTED, "insert into a strided view");
  if (at > n) return fail(RL_EINVAL, "insert position %llu beyond %llu objects", (unsigned long long)at,
                          (unsigned long long)n);
  if (n + count > view->capacity)
    return fail(RL_EINVAL, "%llu objects do not fit the view's capacity %llu", (unsigned long long)(n + count),
                (unsigned long long)view->capacity);
  if (!count) return RL_OK;
  rv.clear();
  if ((st = validate_view(view, n + count, "view", &rv, true))) return st;
  if ((st = check_overlap(rs, rv))) return st;
  hipStream_t s = (hipStream_t)stream;
  const rl_layout* L = view->layout;
  const rl_layout* SL = src->layout;
  const uint32_t ng = (uint32_t)L->schema->members.size();
  if (ng && (at != n || L->kind == RL_AOS || SL->kind == RL_AOS))
    return fail(RL_EUNSUPPORTED, "jagged groups: only appends between offsets layouts (SoA / AoSoA)");
  if ((st = shift_objects(*view, at, at + count, n - at, s))) return st;
  if (L->kind == RL_AOS && L->has_gaps) {
    // the opened records' padding bytes are zero
    uint8_t* rec = (uint8_t*)view->buffers[0];
    if ((st = launch_or_fail(launch_zero_bytes(rec + at * L->stride, count * L->stride, s), "zero"))) return st;
  }
  uint32_t* status = stream_status(s);
  if (!status) return fail(RL_EHIP, "status words of the current device");
  MoveDesc m;
  if ((st = move_desc(SL, gen_side(SL, src->buffers, src->capacity), L, gen_side(L, view->buffers), &m))) return st;
  m.count = count;
  m.dst0 = at;
  m.status = status;
  if ((st = launch_or_fail(launch_move(m, count, s), "move"))) return st;
  if ((st = zero_block_tail(L, view->buffers, n + count, s))) return st;
  for (uint32_t g = 0; g < ng; ++g) {
    AppendDesc ad;
    memset(&ad, 0, sizeof ad);
    ad.src = gen_group(SL, src->buffers, g, src->member_capacity[g]);
    ad.dst = gen_group(L, view->buffers, g, view->member_capacity[g]);
    ad.at = n;
    ad.count = count;
    ad.status = status;
    if ((st = launch_or_fail(launch_append(ad, s), "append"))) return st;
  }
  return RL_OK;
}
