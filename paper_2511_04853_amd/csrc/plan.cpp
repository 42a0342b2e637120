// Planning of conversions: descriptors of the dense, scan, gather and
// rebase kernels for one collection.
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <numeric>

#include "plan.h"

namespace rl {

static constexpr uint32_t kLdsBudget = 64 * 1024;
static constexpr uint32_t kDefaultTile = 512;
static constexpr uint32_t kMaxTile = 4096;
// single-pass jagged conversions of at most this many tiles store member
// columns non-temporally
static constexpr uint64_t kStreamMembersTiles = 1024;

SideSpec object_side(const rl_layout* L, void* const* bufs, uint64_t index0) {
  SideSpec s;
  s.kind = (uint32_t)L->kind;
  s.types = L->storage;
  if (L->kind == RL_AOS) {
    s.base = (uint8_t*)bufs[0] + index0 * L->stride;
    s.stride = (uint32_t)L->stride;
    s.off = L->leaf_offset;
  } else if (L->kind == RL_SOA) {
    for (size_t c = 0; c < L->storage.size(); ++c)
      s.cols.push_back((uint8_t*)bufs[c] + index0 * type_size(L->storage[c]));
  } else {
    s.base = (uint8_t*)bufs[0] + index0 * (uint64_t)L->obj_bytes;  // index0 is a multiple of W
    s.width = L->width;
  }
  return s;
}

SideSpec member_side(const rl_layout* L, void* const* bufs, uint32_t g) {
  SideSpec s;
  const rl_schema* sc = L->schema;
  const uint32_t gb = group_buffer(L, g);
  for (const auto& m : sc->members[g]) s.types.push_back(m.type);
  if (L->kind == RL_AOS) {
    s.kind = KIND_AOS;
    s.base = (uint8_t*)bufs[gb];
    s.stride = L->mstride[g];
    s.off = L->moff[g];
  } else {
    s.kind = KIND_SOA;
    for (size_t m = 0; m < sc->members[g].size(); ++m) s.cols.push_back((uint8_t*)bufs[gb + 1 + m]);
  }
  return s;
}

static uint32_t side_obj_bytes(const SideSpec& s) {
  uint32_t b = 0;
  for (auto t : s.types) b += type_size(t);
  return b;
}

static uint64_t image_bytes(const SideSpec& s, uint32_t tile) {
  if (s.kind == KIND_AOS) return (uint64_t)tile * s.stride;
  return (uint64_t)tile * side_obj_bytes(s);
}

static uint32_t lcm32(uint32_t a, uint32_t b) { return a / std::gcd(a, b) * b; }

uint32_t choose_tile(const SideSpec& s, const SideSpec& d, uint32_t target, uint64_t n) {
  uint32_t unit = 16;
  if (s.kind == KIND_AOSOA) unit = lcm32(unit, s.width);
  if (d.kind == KIND_AOSOA) unit = lcm32(unit, d.width);
  if (unit > kMaxTile) return 0;
  // Tile targets are object counts for objects of about 32 bytes: a tile
  // carries a fixed cost (descriptor, DMA issue, barriers), so smaller
  // objects (member records of a few bytes) get proportionally more of them.
  const uint64_t per = std::max<uint64_t>(1, std::max(image_bytes(s, 1), image_bytes(d, 1)));
  const uint32_t scale = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(16, 32 / per));
  if (!target) {
    // long column runs favour large tiles; small collections need enough
    // tiles to spread over the 256 compute units.  Records written from an
    // LDS image of columns or blocks take half the tile: the two images
    // then fit twice as many work-groups (SoA -> AoS at 2^22 - 2^24
    // objects: 3-7% faster, AoSoA -> AoS about even)
    target = (d.kind == KIND_AOS && s.kind != KIND_AOS ? kDefaultTile / 2 : kDefaultTile) * scale;
    while (target > 128 && n && (n + target - 1) / target < 1024) target /= 2;
  } else {
    target *= scale;
  }
  target = std::min<uint32_t>(target, kMaxTile);
  uint32_t t = std::max(unit, target / unit * unit);
  while (t >= unit) {
    const uint64_t lds = ((image_bytes(s, t) + 15) & ~15ull) + ((image_bytes(d, t) + 15) & ~15ull) + 144;
    if (lds <= kLdsBudget) return t;
    t -= unit;
  }
  return 0;
}

static bool side_aligned(const SideSpec& s, uint32_t c, uint32_t size, uint32_t prefix, uint32_t obj_bytes) {
  if (s.kind == KIND_AOS) return s.stride % size == 0 && s.off[c] % size == 0;
  if (s.kind == KIND_SOA) return true;
  return ((uint64_t)s.width * obj_bytes) % size == 0 && ((uint64_t)s.width * prefix) % size == 0;
}

static bool cols_aligned16(const SideSpec& s) {
  for (auto* p : s.cols)
    if ((uintptr_t)p & 15) return false;
  return true;
}

// ceil(2^32 / w): umulhi(i, magic) == i / w for i < 2^17 and 2 <= w <= 4096
// (the rounding error i * (magic - 2^32 / w) / 2^32 stays below 1 / w).
// Width 1 is handled without the multiplier.
static uint32_t width_magic(uint32_t w) {
  if (w <= 1) return 0;
  return (uint32_t)(((1ull << 32) + w - 1) / w);
}

rl_status build_dense(const SideSpec& s, const SideSpec& d, uint64_t n, uint32_t tile, DenseDesc* out) {
  DenseDesc& k = *out;
  memset(&k, 0, sizeof k);
  const uint32_t nl = (uint32_t)s.types.size();
  if (nl != d.types.size()) return fail(RL_EINVAL, "internal: leaf count mismatch");
  if (nl > (uint32_t)kMaxLeaves) return fail(RL_EUNSUPPORTED, "too many leaves");
  const uint32_t sb = side_obj_bytes(s), db = side_obj_bytes(d);
  auto fill_side = [&](const SideSpec& x, uint32_t obj_bytes, SideDesc& o) {
    o.base = x.base;
    o.kind = x.kind;
    o.stride = x.stride;
    o.width = x.kind == KIND_AOSOA ? x.width : 1;
    o.obj_bytes = obj_bytes;
    o.width_magic = width_magic(o.width);
    o.image_bytes = (uint32_t)image_bytes(x, tile);
  };
  fill_side(s, sb, k.src);
  fill_side(d, db, k.dst);
  k.n = n;
  k.tile = tile;
  // umulhi(v, magic) == v / (tile / 16) for v < 2^17, 2 <= tile / 16 <= 256
  // (tile == 16 is handled without it)
  k.vt_magic = tile <= 16 ? 0 : (uint32_t)(((1ull << 32) + tile / 16 - 1) / (tile / 16));
  k.n_leaves = nl;
  uint32_t sp = 0, dp = 0;
  for (uint32_t c = 0; c < nl; ++c) {
    LeafDesc& L = k.leaf[c];
    const uint32_t ss = type_size(s.types[c]), dsz = type_size(d.types[c]);
    L.src_size = (uint8_t)ss;
    L.dst_size = (uint8_t)dsz;
    if (s.types[c] == d.types[c]) L.op = OP_COPY;
    else if (s.types[c] == RL_F64 && d.types[c] == RL_F32) L.op = OP_NARROW;
    else if (s.types[c] == RL_F32 && d.types[c] == RL_F64) L.op = OP_WIDEN;
    else return fail(RL_EUNSUPPORTED, "leaf %u: storage types %d -> %d", c, (int)s.types[c], (int)d.types[c]);
    auto image_off = [&](const SideSpec& x, uint32_t prefix) -> uint32_t {
      if (x.kind == KIND_AOS) return x.off[c];
      if (x.kind == KIND_SOA) return tile * prefix;
      return x.width * prefix;
    };
    L.src_off = image_off(s, sp);
    L.dst_off = image_off(d, dp);
    L.byte_wise = !(side_aligned(s, c, ss, sp, sb) && side_aligned(d, c, dsz, dp, db));
    if (L.byte_wise) L.code = CODE_BYTES;
    else if (L.op == OP_NARROW) L.code = CODE_NARROW;
    else if (L.op == OP_WIDEN) L.code = CODE_WIDEN;
    else L.code = ss == 1 ? CODE_COPY1 : ss == 2 ? CODE_COPY2 : ss == 4 ? CODE_COPY4 : CODE_COPY8;
    L.src_col = s.kind == KIND_SOA ? s.cols[c] : nullptr;
    L.dst_col = d.kind == KIND_SOA ? d.cols[c] : nullptr;
    if (L.code >= CODE_BYTES) k.slow_leaves = 1;
    else ++k.fast_leaves;
    sp += ss;
    dp += dsz;
  }
  if (s.kind == KIND_SOA && sb <= (uint32_t)kMaxUnits && sb > 0 && cols_aligned16(s)) {
    k.units_src = 1;
    uint32_t u = 0;
    for (uint32_t c = 0; c < nl; ++c)
      for (uint32_t b = 0; b < k.leaf[c].src_size; ++b) k.unit_src[u++] = (uint8_t)c;
  }
  // source runs go to LDS by DMA when 16-byte aligned: SoA columns must
  // be (tiles hold a multiple of 16 objects); record and block runs are
  // checked per tile
  if (s.kind == KIND_SOA) k.dma = cols_aligned16(s) ? 1 : 0;
  else k.dma = 1;
  if (d.kind == KIND_SOA && db <= (uint32_t)kMaxUnits && db > 0 && cols_aligned16(d)) {
    k.units_dst = 1;
    uint32_t u = 0;
    for (uint32_t c = 0; c < nl; ++c)
      for (uint32_t b = 0; b < k.leaf[c].dst_size; ++b) k.unit_dst[u++] = (uint8_t)c;
  }
  return RL_OK;
}

static uint32_t default_grid(uint64_t tiles, const PlanShape& shape) {
  if (shape.grid) return (uint32_t)std::min<uint64_t>(tiles ? tiles : 1, shape.grid);
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(tiles, 256ull * 16));
}

// Threads of a dense work-group: two objects per thread per pass.
static uint32_t dense_threads(uint32_t tile, const PlanShape& shape) {
  uint32_t t = shape.threads ? shape.threads : (tile / 2 + 63) / 64 * 64;
  return std::min<uint32_t>(kDenseMaxThreads, std::max<uint32_t>(64, t));
}

// Whether a dense step can store its values straight into the destination:
// SoA columns or AoSoA blocks in device memory, every leaf on a fast path
// (aligned, no record pointers), no padding to zero.
static bool direct_ok(const DenseDesc& d) {
  const SideDesc& o = d.dst;
  if (d.slow_leaves || d.zero_dst) return false;
  // records of at most 8 bytes without gaps (member records of a pool):
  // each store of a wave covers a contiguous 256-512 byte run, and leaving
  // out the destination image frees LDS for more work-groups (measured:
  // 8-byte records from SoA / AoSoA 64, 3.8 -> 4.3-4.4 TB/s; 32-byte
  // records lose, 2.9 -> 2.3 TB/s)
  if (o.kind == KIND_AOS) return d.src.kind != KIND_AOS && o.stride <= 8 && ((uintptr_t)o.base & 15) == 0;
  if (o.kind == KIND_AOSOA) return ((uintptr_t)o.base & 15) == 0;
  for (uint32_t c = 0; c < d.n_leaves; ++c)
    if ((uintptr_t)d.leaf[c].dst_col % d.leaf[c].dst_size) return false;
  return true;
}

static rl_status push_dense(Plan* plan, const DenseDesc& d, const PlanShape& shape) {
  Step st;
  st.kind = Step::DENSE;
  st.dense = d;
  st.dense.dst_direct = shape.direct != 0 && direct_ok(d) ? 1u : 0u;
  if (shape.dma == 0) st.dense.dma = 0;
  st.threads = dense_threads(d.tile, shape);
  st.grid = default_grid(dense_tiles(d), shape);
  // double-buffered only where asked for (RL_PIPELINE=1, a batch tuner
  // candidate): with records read and values stored non-temporally the
  // single-slot kernel is faster at every length measured (AoS -> SoA at
  // 2^24 - 2^25 objects: 5.25-5.50 double-buffered, 5.57-5.86 TB/s single
  // slot); before those cache policies two slots had won by 2-4% there
  const uint32_t slot = (dense_lds_bytes(st.dense) + 15u) & ~15u;
  if (shape.pipe == 1 && 2 * slot <= kLdsBudget) st.dense.pipe_slot = slot;
  st.dense.stream_stores = shape.stream ? 1u : 0u;
  plan->steps.push_back(st);
  return RL_OK;
}

// Objects per gather work-group: a power of two dividing the scan tile,
// sized for one staging pass of members at the destination's mean members
// per object (the capacity bounds the total), at least 16.
static uint32_t gather_sub_objects(uint32_t tile, uint64_t n, uint64_t capacity) {
  if (!capacity || !n) return tile;
  const uint64_t per = std::max<uint64_t>(1, (capacity + n - 1) / n);
  uint32_t sub = 16;
  while (sub * 2 <= tile && tile % (sub * 2) == 0 && (uint64_t)sub * 2 * per <= kGatherStage) sub *= 2;
  return sub;
}

// Scan + gather steps for group g of an AoS record source into an offsets
// destination.  `fused` says the first pass already ran inside the objects'
// dense step.
static rl_status push_scan_gather(Plan* plan, const rl_view& src, const rl_view& dst, uint32_t g,
                                  uint64_t n, uint32_t tile, bool fused, bool gather,
                                  const PlanShape& shape, uint32_t* status) {
  const rl_layout* SL = src.layout;
  const rl_layout* DL = dst.layout;
  const rl_schema* sc = SL->schema;
  const rl_type ot = sc->offset_types[g];
  uint8_t* offs = (uint8_t*)dst.buffers[group_buffer(DL, g)];
  if (!fused) {
    // counts-only pass: a dense step with no leaves that scans group g
    SideSpec s = object_side(SL, src.buffers, 0);
    s.types.clear();
    s.off.clear();
    SideSpec d;
    d.kind = KIND_SOA;
    DenseDesc dd;
    rl_status st = build_dense(s, d, n, tile, &dd);
    if (st) return st;
    dd.scan_offsets = offs;
    dd.scan_len_off = SL->len_off[g];
    dd.scan_off_type = ot;
    dd.status = status;
    push_dense(plan, dd, shape);
  }
  Step t;
  t.kind = Step::SCAN_TOTALS;
  t.totals = ScanTotalsDesc{offs, n, tile, (uint32_t)ot, gather ? dst.member_capacity[g] : ~0ull, status};
  plan->steps.push_back(t);
  Step ga;
  ga.kind = Step::GATHER;
  GatherDesc& G = ga.gather;
  memset(&G, 0, sizeof G);
  G.offsets = offs;
  G.n = n;
  G.tile = tile;
  G.off_type = ot;
  G.capacity = gather ? dst.member_capacity[g] : 0;
  G.records = (const uint8_t*)src.buffers[0];
  G.rec_stride = (uint32_t)SL->stride;
  G.ptr_off = SL->ptr_off[g];
  G.len_off = SL->len_off[g];
  G.mstride = SL->mstride[g];
  G.malign = SL->malign[g];
  G.pool = (const uint8_t*)src.buffers[group_buffer(SL, g)];
  G.pool_bytes = src.member_capacity[g] * SL->mstride[g];
  G.status = status;
  if (gather) {
    const uint32_t mb = group_buffer(DL, g) + 1;
    G.n_members = (uint32_t)sc->members[g].size();
    for (uint32_t m = 0; m < G.n_members; ++m) {
      G.moff[m] = SL->moff[g][m];
      G.msize[m] = sc->members[g][m].size;
      G.mcol[m] = (uint8_t*)dst.buffers[mb + m];
    }
    // fast path: packed 4-byte member words into 16-byte aligned columns
    bool packed = G.n_members >= 1 && G.n_members <= 4 && G.mstride == 4 * G.n_members;
    for (uint32_t m = 0; m < G.n_members && packed; ++m)
      packed = G.msize[m] == 4 && G.moff[m] == 4 * m && ((uintptr_t)G.mcol[m] & 15) == 0;
    G.packed_words = packed ? G.n_members : 0;
  }
  G.sub = gather_sub_objects(tile, n, gather ? G.capacity : 0);
  ga.threads = kGatherThreads;
  plan->steps.push_back(ga);
  return RL_OK;
}

// The single-pass jagged kernel: one jagged group read from AoS records
// (pointer, count) into an offsets destination whose per-object leaves are
// stored directly, member records of 1..4 packed 4-byte words into 16-byte
// aligned member columns, a destination capacity below 2^39 (look-back
// values saturate at 2^40).  Objects per tile are sized so that a tile's
// members fill about three quarters of one LDS staging pass at the
// destination's mean members per object.  Returns false (and leaves *out
// unspecified) where it does not apply.
static bool build_jagged(const rl_view& src, const rl_view& dst, uint64_t n, const PlanShape& shape,
                         JaggedDesc* out) {
  const rl_layout* SL = src.layout;
  const rl_layout* DL = dst.layout;
  const rl_schema* sc = SL->schema;
  if (shape.fused == 0 || shape.direct == 0 || sc->members.size() != 1 || SL->kind != RL_AOS ||
      DL->kind == RL_AOS || n == 0)
    return false;
  const uint64_t cap = dst.member_capacity[0];
  if (cap >= (1ull << 39) || src.member_capacity[0] >= (1ull << 39)) return false;
  const uint32_t nw = (uint32_t)sc->members[0].size();
  if (nw < 1 || nw > 4 || SL->mstride[0] != 4 * nw) return false;
  const uint32_t mb = group_buffer(DL, 0) + 1;
  for (uint32_t m = 0; m < nw; ++m)
    if (sc->members[0][m].size != 4 || SL->moff[0][m] != 4 * m || ((uintptr_t)dst.buffers[mb + m] & 15))
      return false;
  if (SL->ptr_off[0] % 8 || SL->len_off[0] % 4 || SL->stride % 8) return false;
  SideSpec s = object_side(SL, src.buffers, 0);
  SideSpec d = object_side(DL, dst.buffers, 0);
  uint32_t unit = 16;
  if (d.kind == KIND_AOSOA) unit = lcm32(unit, d.width);
  if (unit > 512) return false;
  const uint32_t S = jagged_stage_members(nw);
  const uint64_t mean = std::max<uint64_t>(1, (cap + n - 1) / n);
  uint32_t target = 512;
  while (target > 16 && (uint64_t)target * mean > (uint64_t)S * 3 / 4) target /= 2;
  if (shape.tile) target = std::min<uint32_t>(shape.tile, 512);
  const uint32_t tile = std::max(unit, target / unit * unit);
  JaggedDesc& j = *out;
  memset(&j, 0, sizeof j);
  if (build_dense(s, d, n, tile, &j.dense) != RL_OK) return false;
  j.dense.dst_direct = 1;
  if (!direct_ok(j.dense)) return false;
  if (shape.dma == 0) j.dense.dma = 0;
  j.offsets = (uint8_t*)dst.buffers[group_buffer(DL, 0)];
  j.capacity = cap;
  j.pool = (const uint8_t*)src.buffers[group_buffer(SL, 0)];
  j.pool_bytes = src.member_capacity[0] * SL->mstride[0];
  for (uint32_t m = 0; m < nw; ++m) j.mcol[m] = (uint8_t*)dst.buffers[mb + m];
  j.ptr_off = SL->ptr_off[0];
  j.len_off = SL->len_off[0];
  j.mstride = SL->mstride[0];
  j.malign = SL->malign[0];
  j.words = nw;
  j.off_type = (uint32_t)sc->offset_types[0];
  j.stage = S;
  // four work-groups per compute unit: members per staging pass shrink to
  // fit 40 KB of LDS (a tile then takes more passes)
  while (jagged_lds_bytes(j) > 40 * 1024 && j.stage > 256) j.stage -= 64;
  if (jagged_lds_bytes(j) > kLdsBudget) return false;
  const uint64_t need = lookback_bytes((n + tile - 1) / tile);
  // non-temporal member stores pay while the tiles fit one round of
  // resident work-groups and cost beyond it
  j.stream_members = shape.stream && (n + tile - 1) / tile <= kStreamMembersTiles ? 1u : 0u;
  j.dense.stream_stores = j.stream_members;
  if (shape.lookback) {
    if (need > shape.lookback_bytes) return false;
    j.lookback = shape.lookback;
  }
  return true;
}

rl_status make_plan(const rl_view& src, const rl_view& dst, uint64_t n, const PlanShape& shape,
                    Plan* plan) {
  const rl_layout* SL = src.layout;
  const rl_layout* DL = dst.layout;
  if (SL->kind == RL_STRIDED || DL->kind == RL_STRIDED)
    return fail(RL_EUNSUPPORTED, "strided layouts take the general mover, not a tiled plan");
  const rl_schema* sc = SL->schema;
  const uint32_t ng = (uint32_t)sc->members.size();
  uint32_t* const status = nullptr;   // stamped with the stream's word at enqueue
  if (ng && SL->kind == RL_AOS && DL->kind == RL_AOS)
    return fail(RL_EUNSUPPORTED, "AoS -> AoS conversion of a schema with jagged groups");

  {
    Step js;
    js.kind = Step::JAGGED;
    if (build_jagged(src, dst, n, shape, &js.jagged)) {
      js.threads = shape.threads ? std::min<uint32_t>(shape.threads, 256) : 256;
      plan->steps.push_back(js);
      return RL_OK;
    }
    if (shape.fused == 2 && ng && SL->kind == RL_AOS && n)
      return fail(RL_EUNSUPPORTED, "the single-pass jagged kernel does not apply to this conversion");
  }

  SideSpec s = object_side(SL, src.buffers, 0);
  SideSpec d = object_side(DL, dst.buffers, 0);
  const uint32_t tile = choose_tile(s, d, shape.tile, n);
  if (!tile) return fail(RL_EUNSUPPORTED, "no tile shape fits these layouts (block widths or record size)");
  DenseDesc dd;
  rl_status st = build_dense(s, d, n, tile, &dd);
  if (st) return st;
  dd.status = status;
  dd.zero_dst = DL->kind == RL_AOS && DL->has_gaps;
  // destination records of a jagged schema get (ptr, len) from the source
  // offsets (staged in LDS per tile when there is one group)
  if (ng && DL->kind == RL_AOS) {
    if (ng == 1) {
      dd.stage_offsets = (const uint8_t*)src.buffers[group_buffer(SL, 0)];
      dd.stage_type = (uint32_t)sc->offset_types[0];
      dd.stage_src_capacity = src.member_capacity[0];
      dd.stage_dst_capacity = dst.member_capacity[0];
    }
    for (uint32_t g = 0; g < ng; ++g) {
      const rl_type ot = sc->offset_types[g];
      const uint8_t* so = (const uint8_t*)src.buffers[group_buffer(SL, g)];
      for (int which = 0; which < 2; ++which) {
        if (dd.n_leaves >= (uint32_t)kMaxLeaves) return fail(RL_EUNSUPPORTED, "too many leaves");
        LeafDesc& L = dd.leaf[dd.n_leaves++];
        memset(&L, 0, sizeof L);
        L.op = which == 0 ? OP_PTR : OP_LEN;
        L.dst_off = which == 0 ? DL->ptr_off[g] : DL->len_off[g];
        L.dst_size = which == 0 ? 8 : 4;
        L.src_size = 0;
        L.byte_wise = (DL->stride % L.dst_size) != 0;
        L.mstride = (uint16_t)(which == 0 ? DL->mstride[g] : 0);
        L.off_type = (uint8_t)ot;
        L.code = which == 0 ? CODE_PTR : CODE_LEN;
        dd.slow_leaves = 1;
        L.src_col = so;
      }
    }
  }
  const bool scan_src = ng && SL->kind == RL_AOS;
  if (scan_src) {
    dd.scan_offsets = (uint8_t*)dst.buffers[group_buffer(DL, 0)];
    dd.scan_len_off = SL->len_off[0];
    dd.scan_off_type = sc->offset_types[0];
  }
  push_dense(plan, dd, shape);

  for (uint32_t g = 0; g < ng; ++g) {
    const rl_type ot = sc->offset_types[g];
    if (SL->kind == RL_AOS) {
      if ((st = push_scan_gather(plan, src, dst, g, n, tile, g == 0, true, shape, status))) return st;
      continue;
    }
    // offsets-column source: check (and, for an offsets destination, copy
    // rebased), then move the member values.  The records kernel checks
    // the offsets it stages, so a single group into records needs no pass.
    if (!dd.stage_offsets) {
      Step r;
      r.kind = Step::REBASE;
      r.rebase = RebaseDesc{(const uint8_t*)src.buffers[group_buffer(SL, g)],
                            DL->kind == RL_AOS ? nullptr : (uint8_t*)dst.buffers[group_buffer(DL, g)],
                            n, (uint32_t)ot, src.member_capacity[g], dst.member_capacity[g], status};
      plan->steps.push_back(r);
    }
    SideSpec ms = member_side(SL, src.buffers, g);
    SideSpec md = member_side(DL, dst.buffers, g);
    const uint32_t mt = choose_tile(ms, md, shape.tile, dst.member_capacity[g]);
    if (!mt) return fail(RL_EUNSUPPORTED, "no tile shape fits the member records");
    DenseDesc m;
    if ((st = build_dense(ms, md, dst.member_capacity[g], mt, &m))) return st;
    m.status = status;
    m.count_offsets = (const uint8_t*)src.buffers[group_buffer(SL, g)];
    m.count_index = n;
    m.count_off_type = (uint32_t)ot;
    m.src_capacity = src.member_capacity[g];
    m.zero_dst = md.kind == KIND_AOS && (side_obj_bytes(md) < md.stride);
    push_dense(plan, m, shape);
  }
  return RL_OK;
}

rl_status make_offsets_plan(const rl_view& src, const rl_view& dst, uint32_t g, uint64_t n,
                            const PlanShape& shape, Plan* plan) {
  const rl_layout* SL = src.layout;
  const rl_schema* sc = SL->schema;
  uint32_t* const status = nullptr;   // stamped with the stream's word at enqueue
  if (SL->kind == RL_AOS) {
    SideSpec s = object_side(SL, src.buffers, 0);
    s.types.clear();
    SideSpec d;
    d.kind = KIND_SOA;
    const uint32_t tile = choose_tile(s, d, shape.tile ? shape.tile : 1024, n);
    if (!tile) return fail(RL_EUNSUPPORTED, "record too large for a tile");
    return push_scan_gather(plan, src, dst, g, n, tile, false, false, shape, status);
  }
  Step r;
  r.kind = Step::REBASE;
  r.rebase = RebaseDesc{(const uint8_t*)src.buffers[group_buffer(SL, g)],
                        (uint8_t*)dst.buffers[group_buffer(dst.layout, g)], n,
                        (uint32_t)sc->offset_types[g], src.member_capacity[g], ~0ull, status};
  plan->steps.push_back(r);
  return RL_OK;
}

// Look-back memory of single-pass jagged steps, one buffer per (device,
// stream), zeroed when allocated and reused in stream order; held until
// the process ends.  Every buffer (these and those callers give) has a
// launch counter that numbers the launches on it.
namespace {
struct LookbackBuf {
  uint64_t* ptr = nullptr;
  uint64_t bytes = 0;
};
std::mutex g_lb_mu;
std::map<std::pair<int, hipStream_t>, LookbackBuf> g_lb;
std::map<const uint64_t*, uint32_t> g_lb_launches;
}  // namespace

// The stream's look-back buffer with room for `need` bytes (caller holds g_lb_mu).
static rl_status stream_lookback(hipStream_t s, uint64_t need, uint64_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  LookbackBuf& b = g_lb[{dev, s}];
  if (b.bytes < need) {
    if (b.ptr) {
      // earlier work on this stream may still use the old buffer
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
      (void)hipFree(b.ptr);
      g_lb_launches.erase(b.ptr);
      b.ptr = nullptr;
      b.bytes = 0;
    }
    const uint64_t want = std::max<uint64_t>((need * 2 + 255) & ~255ull, 64 << 10);
    if ((e = hipMalloc((void**)&b.ptr, want)) != hipSuccess)
      return fail(RL_ENOMEM, "look-back buffer of %llu bytes: %s", (unsigned long long)want, hipGetErrorString(e));
    if ((e = launch_zero(b.ptr, want, s)) != hipSuccess) return hip_fail(e, "zero look-back buffer");
    b.bytes = want;
  }
  *out = b.ptr;
  return RL_OK;
}

bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus c = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &c) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return c != hipStreamCaptureStatusNone;
}

rl_status enqueue_plan(const Plan& plan, hipStream_t stream) {
  // device-detected errors go to the status word of the launching stream
  uint32_t* const status = stream_status(stream);
  if (!status) return fail(RL_EHIP, "status words of the current device");
  for (const Step& s0 : plan.steps) {
    Step s = s0;
    hipError_t e = hipSuccess;
    switch (s.kind) {
      case Step::DENSE: s.dense.status = status; e = launch_dense(s.dense, s.threads, s.grid, stream); break;
      case Step::SCAN_TOTALS: s.totals.status = status; e = launch_scan_totals(s.totals, stream); break;
      case Step::GATHER: s.gather.status = status; e = launch_gather(s.gather, s.threads, stream); break;
      case Step::REBASE: s.rebase.status = status; e = launch_rebase(s.rebase, stream); break;
      case Step::JAGGED: {
        s.jagged.dense.status = status;
        const uint64_t tiles = (s.jagged.dense.n + s.jagged.dense.tile - 1) / s.jagged.dense.tile;
        // the buffer and its launch counter stay locked until the kernel is
        // enqueued (another thread may grow the buffer)
        std::lock_guard<std::mutex> lk(g_lb_mu);
        if (!s.jagged.lookback) {
          rl_status st = stream_lookback(stream, lookback_bytes(tiles), &s.jagged.lookback);
          if (st) return st;
        }
        s.jagged.epoch = ++g_lb_launches[s.jagged.lookback];
        e = launch_jagged(s.jagged, s.threads, stream);
        break;
      }
    }
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
  }
  return RL_OK;
}

}  // namespace rl
