// HIP kernels of librelayout for gfx950 (CDNA4, wave64).
//
// Dense conversion (every per-object leaf value moves from the source
// address map to the destination address map, Sec. VII-B default transfer):
// a work-group takes a tile of T objects, copies the source bytes of the
// tile into an LDS image with 16-byte global loads, moves every
// (object, leaf) value from the source image to the destination image
// inside LDS, then writes the destination image out with 16-byte global
// stores.  Both global sides are contiguous runs per tile (AoS: one run of
// T records; AoSoA: T/W whole blocks; SoA: one run per column), so both
// reads and writes coalesce whatever the field widths.
//
// Jagged groups (Sec. VI, prefix sum of member counts): the counts of an AoS
// record source are scanned per tile inside the dense kernel (wave prefix
// sums + an LDS pass over waves), a one-work-group pass scans the tile
// totals, and a third pass adds tile prefixes and gathers each tile's
// members from the member pool.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "rl_internal.h"

namespace rl {

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ helpers

// Global memory.  Pointers that kernels read out of descriptors held in
// memory (batches) are generic to the compiler, which would then use flat
// instructions; those also count on the LDS counter, so every later LDS
// wait would wait for them too.  Kernels reach global memory (device or
// pinned host) through address space 1.
#define RL_G __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ RL_G T* gp(T* p) { return (RL_G T*)p; }

// Descriptor tables of batches: written by the host before a launch and
// never by kernels, so they are read as constant memory (address space 4),
// through scalar loads.  Read through a generic pointer they would be
// vector loads, each of which the in-order vector-memory counter makes
// wait behind every store issued before it.
#define RL_C __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const RL_C T& cdesc(const T* table, uint64_t i) {
  return ((const RL_C T*)table)[i];
}

// A kernel's only argument, read in place in the kernel-argument segment
// like a descriptor table entry.  The empty asm hides that every call
// yields the same address: the compiler otherwise loads every field the
// kernel uses into scalar registers at entry and keeps them live across
// the whole kernel, spilling registers once the code grows.
template <class T>
__device__ __forceinline__ const RL_C T& kernel_arg() {
  const RL_C T* p = (const RL_C T*)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(p));
  return *p;
}

__device__ __forceinline__ uint64_t load_off(const uint8_t* p, uint32_t type, uint64_t i) {
  if (type == RL_U64) return gp(reinterpret_cast<const uint64_t*>(p))[i];
  if (type == RL_I32) return (uint64_t)(int64_t)gp(reinterpret_cast<const int32_t*>(p))[i];
  return gp(reinterpret_cast<const uint32_t*>(p))[i];
}

__device__ __forceinline__ void store_off(uint8_t* p, uint32_t type, uint64_t i, uint64_t v) {
  if (type == RL_U64) gp(reinterpret_cast<uint64_t*>(p))[i] = v;
  else if (type == RL_I32) gp(reinterpret_cast<int32_t*>(p))[i] = (int32_t)v;
  else gp(reinterpret_cast<uint32_t*>(p))[i] = (uint32_t)v;
}

__device__ __forceinline__ uint64_t off_limit(uint32_t type) {
  if (type == RL_U64) return ~0ull;
  if (type == RL_I32) return 0x7fffffffull;
  return 0xffffffffull;
}

__device__ __forceinline__ void flag(uint32_t* status, uint32_t f) {
  if (status) __hip_atomic_fetch_or(gp(status), f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Copy `bytes` from global memory to LDS (the LDS side is 16-byte aligned).
// All threads of the work-group take part.
__device__ __forceinline__ void g2l(uint8_t* lds, const uint8_t* g, uint32_t bytes,
                                    uint32_t tid, uint32_t nt) {
  if ((reinterpret_cast<uintptr_t>(g) & 15) == 0) {
    const uint32_t nv = bytes >> 4;
    const RL_G v4u* gv = gp(reinterpret_cast<const v4u*>(g));
    v4u* lv = reinterpret_cast<v4u*>(lds);
    for (uint32_t v = tid; v < nv; v += nt) lv[v] = gv[v];
    for (uint32_t b = (nv << 4) + tid; b < bytes; b += nt) lds[b] = gp(g)[b];
  } else if ((reinterpret_cast<uintptr_t>(g) & 3) == 0) {
    const uint32_t nw = bytes >> 2;
    const RL_G uint32_t* gw = gp(reinterpret_cast<const uint32_t*>(g));
    uint32_t* lw = reinterpret_cast<uint32_t*>(lds);
    for (uint32_t v = tid; v < nw; v += nt) lw[v] = gw[v];
    for (uint32_t b = (nw << 2) + tid; b < bytes; b += nt) lds[b] = gp(g)[b];
  } else {
    for (uint32_t b = tid; b < bytes; b += nt) lds[b] = gp(g)[b];
  }
}

// Values stored straight from the transform can be non-temporal
// (DenseDesc::stream_stores): a conversion streams its destination out and
// never reads it back, and such stores leave the caches to the data still
// to be read (measured: the benchmark step of four conversions 10.7 ->
// 8.4 us, AoS -> SoA at 2^22 - 2^24 objects 4.8 -> 5.1 and 5.2 -> 5.4 TB/s,
// single conversions 7-9% faster; but the 512-collection batch 1.29 ->
// 1.35 ms, so batches leave the choice to their tuner).  Destination images copied out of LDS (records, host
// memory) keep ordinary stores: non-temporal there, AoSoA -> AoS lost 6%
// and zero-copy writes into pinned host memory up to 13%.  Member columns
// of the single-pass jagged kernel are non-temporal only for conversions
// of at most one round of work-groups (50,000 clusters: 15.3 -> 13.6 us;
// at 2^21 objects, 32,768 tiles, 460 -> 520 us).
template <class T>
__device__ __forceinline__ void st_nt(RL_G T* p, T v) {
  __builtin_nontemporal_store(v, p);
}

// Copy `bytes` from LDS (16-byte aligned) to global memory.
__device__ __forceinline__ void l2g(uint8_t* g, const uint8_t* lds, uint32_t bytes,
                                    uint32_t tid, uint32_t nt) {
  if ((reinterpret_cast<uintptr_t>(g) & 15) == 0) {
    const uint32_t nv = bytes >> 4;
    RL_G v4u* gv = gp(reinterpret_cast<v4u*>(g));
    const v4u* lv = reinterpret_cast<const v4u*>(lds);
    for (uint32_t v = tid; v < nv; v += nt) gv[v] = lv[v];
    for (uint32_t b = (nv << 4) + tid; b < bytes; b += nt) gp(g)[b] = lds[b];
  } else if ((reinterpret_cast<uintptr_t>(g) & 3) == 0) {
    const uint32_t nw = bytes >> 2;
    RL_G uint32_t* gw = gp(reinterpret_cast<uint32_t*>(g));
    const uint32_t* lw = reinterpret_cast<const uint32_t*>(lds);
    for (uint32_t v = tid; v < nw; v += nt) gw[v] = lw[v];
    for (uint32_t b = (nw << 2) + tid; b < bytes; b += nt) gp(g)[b] = lds[b];
  } else {
    for (uint32_t b = tid; b < bytes; b += nt) gp(g)[b] = lds[b];
  }
}

// Bytes of a side's image that hold `cnt` objects (runs are contiguous for
// AoS and AoSoA; for SoA this is only used for zeroing).
template <class SD>
__device__ __forceinline__ uint32_t image_used(const SD& s, uint32_t cnt) {
  if (s.kind == KIND_AOS) return cnt * s.stride;
  if (s.kind == KIND_AOSOA) {
    const uint32_t nblk = s.width == 1 ? cnt : __umulhi(cnt + s.width - 1, s.width_magic);
    return nblk * s.width * s.obj_bytes;
  }
  return s.image_bytes;
}

__device__ __forceinline__ void copy_bytes(uint8_t* d, const uint8_t* s, uint32_t n) {
  for (uint32_t k = 0; k < n; ++k) d[k] = s[k];
}

// Change of precision of one value.  Numbers: IEEE round to nearest even
// (v_cvt_f32_f64; overflow to infinity, subnormal results kept) and exact
// widening (v_cvt_f64_f32).  NaNs: the result is a quiet NaN with the
// input's sign and the leading bits of its payload (as many as the
// destination holds), assembled from the bit fields so that it does not
// depend on how the conversion instructions treat NaN operands.
__device__ __forceinline__ float narrow_value(double x) {
  const float y = (float)x;
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t q = (uint32_t)((b >> 63) << 31) | 0x7FC00000u | (uint32_t)((b & 0x000FFFFFFFFFFFFFull) >> 29);
  return __builtin_isnan(x) ? __uint_as_float(q) : y;
}

__device__ __forceinline__ double widen_value(float x) {
  const double y = (double)x;
  const uint32_t b = __float_as_uint(x);
  const uint64_t q = ((uint64_t)(b >> 31) << 63) | 0x7FF8000000000000ull | ((uint64_t)(b & 0x007FFFFFu) << 29);
  return __builtin_isnan(x) ? __longlong_as_double((long long)q) : y;
}

// Move one value inside LDS.
template <class LD>
__device__ __forceinline__ void move_value(uint8_t* dst, const uint8_t* src, const LD& L) {
  if (L.op == OP_COPY) {
    if (L.byte_wise) { copy_bytes(dst, src, L.src_size); return; }
    switch (L.src_size) {
      case 1: *dst = *src; break;
      case 2: *reinterpret_cast<uint16_t*>(dst) = *reinterpret_cast<const uint16_t*>(src); break;
      case 4: *reinterpret_cast<uint32_t*>(dst) = *reinterpret_cast<const uint32_t*>(src); break;
      default: *reinterpret_cast<uint64_t*>(dst) = *reinterpret_cast<const uint64_t*>(src); break;
    }
  } else if (L.op == OP_NARROW) {
    double x;
    if (L.byte_wise) copy_bytes(reinterpret_cast<uint8_t*>(&x), src, 8);
    else x = *reinterpret_cast<const double*>(src);
    const float y = narrow_value(x);
    if (L.byte_wise) copy_bytes(dst, reinterpret_cast<const uint8_t*>(&y), 4);
    else *reinterpret_cast<float*>(dst) = y;
  } else {  // OP_WIDEN
    float x;
    if (L.byte_wise) copy_bytes(reinterpret_cast<uint8_t*>(&x), src, 4);
    else x = *reinterpret_cast<const float*>(src);
    const double y = widen_value(x);
    if (L.byte_wise) copy_bytes(dst, reinterpret_cast<const uint8_t*>(&y), 8);
    else *reinterpret_cast<double*>(dst) = y;
  }
}

// Block-wide exclusive scan of one u64 per thread (wave64 prefix with
// cross-lane shuffles, then an LDS pass over the wave totals).  Returns the
// exclusive prefix; *total receives the block total.  `wsum` has room for
// one u64 per wave.  Must be called by every thread of the block.
__device__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* wsum, uint64_t* total) {
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t nwaves = (blockDim.x + 63) >> 6;
  uint64_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t o = __shfl_up(inc, d, 64);
    if (lane >= (uint32_t)d) inc += o;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t run = 0;
    for (uint32_t w = 0; w < nwaves; ++w) {
      const uint64_t t = wsum[w];
      wsum[w] = run;
      run += t;
    }
    wsum[nwaves] = run;
  }
  __syncthreads();
  const uint64_t r = wsum[wave] + inc - v;
  *total = wsum[nwaves];
  __syncthreads();
  return r;
}

// LDS carve-up of the dense kernel.
struct DenseLds {
  uint8_t* src;
  uint8_t* dst;
  uint64_t* wsum;
  uint64_t* offs;   // staged offsets: 16 bytes holding entry 0, then raw entries i0 .. i0 + cnt
};

__host__ __device__ __forceinline__ uint32_t round16(uint32_t x) { return (x + 15u) & ~15u; }

// Byte unit of object size that SoA image vector v belongs to
// (v / (tile / 16), by multiplier).
template <class DD>
__device__ __forceinline__ uint32_t unit_of(const DD& d, uint32_t v) {
  return d.tile == 16 ? v : __umulhi(v, d.vt_magic);
}

// Load one side's tile into its LDS image.  `idx0` is the index of the
// tile's first object on that side.
template <class DD>
__device__ __forceinline__ void load_side(const DD& d, uint8_t* img, uint64_t idx0, uint32_t cnt,
                          bool full) {
  const auto& s = d.src;
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  if (s.kind == KIND_AOS) {
    g2l(img, s.base + idx0 * s.stride, cnt * s.stride, tid, nt);
  } else if (s.kind == KIND_AOSOA) {
    g2l(img, s.base + idx0 * s.obj_bytes, image_used(s, cnt), tid, nt);
  } else if (full && d.units_src) {
    // SoA, full tile: the image is the columns' runs back to back (column c
    // at tile * prefix(c)); walk it in 16-byte vectors, finding the column
    // of each vector from the byte-unit table.
    const uint32_t vt = d.tile >> 4;           // vectors per byte of object size
    const uint32_t nv = vt * s.obj_bytes;
    v4u* lv = reinterpret_cast<v4u*>(img);
    for (uint32_t v = tid; v < nv; v += nt) {
      const uint32_t c = d.unit_src[unit_of(d, v)];
      const auto& L = d.leaf[c];
      const uint32_t first_v = L.src_off >> 4;   // tile * prefix / 16
      const RL_G v4u* col = gp(reinterpret_cast<const v4u*>(L.src_col + idx0 * L.src_size));
      lv[v] = col[v - first_v];
    }
  } else {
    for (uint32_t c = 0; c < d.n_leaves; ++c) {
      const auto& L = d.leaf[c];
      if (L.op == OP_PTR || L.op == OP_LEN) continue;  // not in SoA images
      g2l(img + L.src_off, L.src_col + idx0 * L.src_size, cnt * L.src_size, tid, nt);
    }
  }
}

template <class DD>
__device__ __forceinline__ void store_side(const DD& d, const uint8_t* img, uint64_t idx0, uint32_t cnt,
                           bool full) {
  const auto& s = d.dst;
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  if (s.kind == KIND_AOS) {
    l2g(s.base + idx0 * s.stride, img, cnt * s.stride, tid, nt);
  } else if (s.kind == KIND_AOSOA) {
    l2g(s.base + idx0 * s.obj_bytes, img, image_used(s, cnt), tid, nt);
  } else if (full && d.units_dst) {
    const uint32_t vt = d.tile >> 4;
    const uint32_t nv = vt * s.obj_bytes;
    const v4u* lv = reinterpret_cast<const v4u*>(img);
    for (uint32_t v = tid; v < nv; v += nt) {
      const uint32_t c = d.unit_dst[unit_of(d, v)];
      const auto& L = d.leaf[c];
      const uint32_t first_v = L.dst_off >> 4;
      RL_G v4u* col = gp(reinterpret_cast<v4u*>(L.dst_col + idx0 * L.dst_size));
      st_nt(col + (v - first_v), lv[v]);
    }
  } else {
    for (uint32_t c = 0; c < d.n_leaves; ++c) {
      const auto& L = d.leaf[c];
      if (L.op == OP_PTR || L.op == OP_LEN) continue;  // not in SoA images
      l2g(L.dst_col + idx0 * L.dst_size, img + L.dst_off, cnt * L.dst_size, tid, nt);
    }
  }
}

template <class DD>
__device__ __forceinline__ DenseLds carve(uint8_t* smem, const DD& d) {
  DenseLds m;
  m.src = smem;
  m.dst = smem + round16(d.src.image_bytes);
  m.wsum = reinterpret_cast<uint64_t*>(m.dst + (d.dst_direct ? 0u : round16(d.dst.image_bytes)));
  m.offs = m.wsum + 18;
  return m;
}

// Count and source base of a conversion: host-given, or read on the device
// from an offsets column (member columns of a jagged group).
template <class DD>
__device__ __forceinline__ void dense_count(const DD& d, uint64_t* count, uint64_t* base) {
  if (d.count_offsets) {
    const uint64_t b = load_off(d.count_offsets, d.count_off_type, 0);
    const uint64_t e = load_off(d.count_offsets, d.count_off_type, d.count_index);
    uint64_t c = e >= b ? e - b : 0;
    if (c > d.n) c = d.n;   // never beyond the destination capacity
    if (b > d.src_capacity) c = 0;
    else if (c > d.src_capacity - b) c = d.src_capacity - b;  // nor the source's
    *count = c;
    *base = b;
  } else {
    *count = d.n;
    *base = 0;
  }
}

// ------------------------------------------------------------------ tile pipeline
//
// A work-group converts a sequence of tiles.  Source images travel from
// global memory straight into LDS (global_load_lds, 16 bytes per lane, no
// registers in between): every vector of a tile is in flight at once, and
// the next tile's vectors are issued as soon as the current source image
// has been consumed, so they overlap the current tile's stores.

struct TileJob {
  uint32_t valid;       // 0: no more work
  uint32_t item;        // descriptor index (batches)
  uint64_t tile, count, base;
};

typedef __attribute__((address_space(3))) uint8_t* lds_ptr;

// One 16-byte DMA per lane from global memory into LDS: lane l of the wave
// lands at LDS byte lds_base + 16 l (lds_base wave-uniform).  Issued as
// inline assembly: the compiler, which cannot tell which LDS bytes the DMA
// writes, would otherwise wait for every outstanding vector-memory
// operation (stores included) before each later LDS read.  Kernels wait
// for the DMA themselves (dma_wait, then a barrier) before reading.
__device__ __forceinline__ void dma16(const uint8_t* g, uint32_t lds_base) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
               :: "v"(g), "s"(lds_base) : "memory", "m0");
}
// The same with the non-temporal cache policy, for source bytes read once.
__device__ __forceinline__ void dma16_nt(const uint8_t* g, uint32_t lds_base) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off nt"
               :: "v"(g), "s"(lds_base) : "memory", "m0");
}

// Copy a 16-byte aligned global run of `bytes` into LDS (16-byte aligned)
// by DMA; the last bytes % 16 go through registers.  Wave w takes the
// 64-vector chunks w, w + waves, ...
template <bool NT = false>
__device__ __forceinline__ void dma_run(uint8_t* lds, const uint8_t* g, uint32_t bytes, uint32_t nthreads = blockDim.x) {
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = nthreads >> 6;
  const uint32_t nv = bytes >> 4;
  for (uint32_t vb = wave * 64; vb < nv; vb += nw * 64) {
    const uint32_t v = vb + lane;
    const uint32_t base = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_ptr)(lds + (size_t)vb * 16));
    if (v < nv) {
      if (NT) dma16_nt(g + (size_t)v * 16, base);
      else dma16(g + (size_t)v * 16, base);
    }
  }
  for (uint32_t b = (nv << 4) + threadIdx.x; b < bytes; b += nthreads) lds[b] = gp(g)[b];
}

// Wait for this wave's DMA into LDS (and every earlier vector-memory
// operation: the counter retires in order).  A barrier must follow before
// other waves read what this wave loaded.
__device__ __forceinline__ void dma_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); /* vmcnt(0) */ }

// Wait until at most `n` of this wave's vector-memory operations are
// outstanding (n wave-uniform).  The counter retires in order, so every
// operation issued before the last n has completed.  Rounded down to a
// few counts (waiting for more is always correct); vmcnt's 6 bits are
// split over simm16 bits 3:0 and 15:14, expcnt and lgkmcnt left at their
// maxima.
template <uint32_t N>
__device__ __forceinline__ void vm_wait_le() {
  __builtin_amdgcn_s_waitcnt(0x0F70 | (N & 15) | ((N >> 4) << 14));
}
__device__ __forceinline__ void vm_wait_at_most(uint32_t n) {
  if (n >= 56) vm_wait_le<56>();
  else if (n >= 48) vm_wait_le<48>();
  else if (n >= 40) vm_wait_le<40>();
  else if (n >= 32) vm_wait_le<32>();
  else if (n >= 24) vm_wait_le<24>();
  else if (n >= 16) vm_wait_le<16>();
  else if (n >= 8) vm_wait_le<8>();
  else if (n >= 4) vm_wait_le<4>();
  else vm_wait_le<0>();
}

// A wave's copy of the fast-path fields of a descriptor's leaves: lane c
// holds leaf c (a schema has at most one wavefront of leaves).  Loaded with
// vector loads when a tile of another descriptor is issued, so the tile's
// DMA wait covers them; the transform reads them with v_readlane and makes
// no memory access per leaf.
struct LeafLanes {
  uint32_t src_off, dst_off;   // OP_PTR: src_off holds the member record stride
  uint32_t code;               // LeafCode | source size << 8 | op << 16 | byte_wise << 24
                               // | offsets rl_type << 25 (OP_PTR / OP_LEN)
  uint32_t col_lo, col_hi;     // SoA destination column
  uint32_t scol_lo, scol_hi;   // SoA source column
  uint32_t item;               // descriptor the lanes hold
};

// The leaf's fields are read as whole words, all at once (no load waits
// on another: a byte field read first to choose the next field would put
// a second memory round trip before the lanes are ready).
template <class LD>
__device__ __forceinline__ uint32_t leaf_word(const LD& L, uint32_t k);

template <class DD>
__device__ __forceinline__ void load_lanes(const DD& d, uint32_t item, LeafLanes& t) {
  const uint32_t lane = threadIdx.x & 63;
  if (lane < d.n_leaves) {
    const auto& L = d.leaf[lane];
    const uint32_t w2 = leaf_word(L, 2), w3 = leaf_word(L, 3);
    const uint32_t src_off = L.src_off, dst_off = L.dst_off;
    const uint64_t col = reinterpret_cast<uint64_t>(L.dst_col);
    const uint64_t scol = reinterpret_cast<uint64_t>(L.src_col);
    const uint32_t op = (w2 >> 16) & 255;
    t.src_off = op == OP_PTR ? (w3 & 0xffff) : src_off;
    t.dst_off = dst_off;
    t.code = (w3 >> 24) | ((w2 & 255) << 8) | (op << 16) | ((w2 >> 24) << 24) | (((w3 >> 16) & 255) << 25);
    t.col_lo = (uint32_t)col;
    t.col_hi = (uint32_t)(col >> 32);
    t.scol_lo = (uint32_t)scol;
    t.scol_hi = (uint32_t)(scol >> 32);
  }
  t.item = item;
}

// load_lanes through scalar loads (leaf c read at a uniform index, then
// placed in lane c): no vector-memory operation, so nothing that waits on
// the in-order vector counter (the double-buffered pipeline fills the lanes
// of its next tile while the current tile's stores are still in flight).
// The byte fields of a leaf descriptor in constant memory, read as whole
// words: there are no sub-word scalar loads, so a u8 or u16 field would be
// read with a per-lane vector load that waits behind every store in
// flight.  Word 2: src_size | dst_size << 8 | op << 16 | byte_wise << 24;
// word 3: mstride | off_type << 16 | code << 24.
template <class LD>
__device__ __forceinline__ uint32_t leaf_word(const LD& L, uint32_t k) {
  return reinterpret_cast<const RL_C uint32_t*>(&L)[k];
}

// vec with lane c set to v (v and c wave-uniform).  The empty asm keeps v
// a per-iteration scalar: without it the compiler turns the caller's loop
// over leaves into one vector load per lane, whose wait would also wait
// for every store in flight.
__device__ __forceinline__ uint32_t put_lane(uint32_t vec, uint32_t v, uint32_t c) {
  return (threadIdx.x & 63) == c ? v : vec;
}

template <class DD>
__device__ __forceinline__ void load_lanes_scalar(const DD& d, uint32_t item, LeafLanes& t) {
  const uint32_t nl = d.n_leaves;
  for (uint32_t c = 0; c < nl; ++c) {
    const auto& L = d.leaf[c];
    const uint32_t w2 = leaf_word(L, 2), w3 = leaf_word(L, 3);
    const uint32_t op = (w2 >> 16) & 255;
    const uint32_t src_off = op == OP_PTR ? (w3 & 0xffff) : L.src_off;
    const uint32_t code = (w3 >> 24) | ((w2 & 255) << 8) | (op << 16) | ((w2 >> 24) << 24) |
                          (((w3 >> 16) & 255) << 25);
    const uint64_t col = reinterpret_cast<uint64_t>(L.dst_col);
    const uint64_t scol = reinterpret_cast<uint64_t>(L.src_col);
    t.src_off = put_lane(t.src_off, src_off, c);
    t.dst_off = put_lane(t.dst_off, L.dst_off, c);
    t.code = put_lane(t.code, code, c);
    t.col_lo = put_lane(t.col_lo, (uint32_t)col, c);
    t.col_hi = put_lane(t.col_hi, (uint32_t)(col >> 32), c);
    t.scol_lo = put_lane(t.scol_lo, (uint32_t)scol, c);
    t.scol_hi = put_lane(t.scol_hi, (uint32_t)(scol >> 32), c);
  }
  t.item = item;
}

__device__ __forceinline__ uint32_t lane_of(uint32_t v, uint32_t c) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)c);
}

// Start bringing a tile's source image into LDS: by DMA when every run is
// 16-byte aligned, else through registers (complete on return).
template <class DD>
__device__ __forceinline__ void issue_image(const DD& d, uint8_t* img, const TileJob& j, const LeafLanes& lt,
                                            bool lanes_ready, uint32_t nthreads = blockDim.x) {
  const uint64_t i0 = j.tile * d.tile;
  const uint32_t cnt = (uint32_t)min<uint64_t>(d.tile, j.count - i0);
  const uint64_t idx0 = i0 + j.base;
  const auto& s = d.src;
  if (d.dma) {
    if (s.kind == KIND_AOS || s.kind == KIND_AOSOA) {
      const uint8_t* run = s.base + idx0 * (s.kind == KIND_AOS ? s.stride : s.obj_bytes);
      if (((uintptr_t)run & 15) == 0) {
        // records are read once: non-temporal (AoS -> SoA at 2^24 objects
        // 5.38 -> 5.48 TB/s, the step 8.45 -> 8.12 us, a single
        // conversion 7.2 -> 6.4 us); AoSoA blocks keep the default policy
        // (AoSoA -> AoS lost 8% with it)
        if (s.kind == KIND_AOS) dma_run<true>(img, run, cnt * s.stride, nthreads);
        else dma_run(img, run, image_used(s, cnt), nthreads);
        return;
      }
    } else if ((idx0 & 15) == 0) {
      // SoA (16-byte aligned columns): every column run starts 16-byte
      // aligned when the first index is a multiple of 16.  Column fields
      // come from the wave's leaf lanes (no dependent memory access per
      // column) unless those were just loaded: reading them then would wait
      // for every earlier store of this wave (in-order counter).
      const uint32_t nl = d.n_leaves;
      if (lanes_ready) {
        for (uint32_t c = 0; c < nl; ++c) {
          const uint32_t w = lane_of(lt.code, c);
          const uint32_t op = (w >> 16) & 255, sz = (w >> 8) & 255;
          if (op == OP_PTR || op == OP_LEN) continue;
          const uint8_t* col =
              reinterpret_cast<const uint8_t*>(((uint64_t)lane_of(lt.scol_hi, c) << 32) | lane_of(lt.scol_lo, c));
          dma_run(img + lane_of(lt.src_off, c), col + idx0 * sz, cnt * sz, nthreads);
        }
      } else {
        for (uint32_t c = 0; c < nl; ++c) {
          const auto& L = d.leaf[c];
          const uint32_t w2 = leaf_word(L, 2);
          const uint32_t op = (w2 >> 16) & 255, sz = w2 & 255;
          if (op == OP_PTR || op == OP_LEN) continue;
          dma_run(img + L.src_off, L.src_col + idx0 * sz, cnt * sz, nthreads);
        }
      }
      return;
    }
  }
  load_side(d, img, idx0, cnt, cnt == d.tile && j.base == 0);
}

__device__ __forceinline__ uint32_t off_bytes(uint32_t type) { return type == RL_U64 ? 8u : 4u; }

// Entry k of a raw offsets run staged in LDS.
__device__ __forceinline__ uint64_t staged_off(const uint8_t* run, uint32_t type, uint32_t k) {
  if (type == RL_U64) return reinterpret_cast<const uint64_t*>(run)[k];
  if (type == RL_I32) return (uint64_t)(int64_t)reinterpret_cast<const int32_t*>(run)[k];
  return reinterpret_cast<const uint32_t*>(run)[k];
}

// A tile's source image plus, for destination records of a jagged group,
// the raw offsets entries i0 .. i0 + cnt and the column's first 16 bytes
// (entry 0), which travel with the image: by DMA when the column is
// 16-byte aligned, whole vectors while they stay inside the column's
// n + 1 entries.  LDS holds entry 0's vector, then the run.
template <class DD>
__device__ __forceinline__ void issue_source(const DD& d, uint8_t* smem, const TileJob& j, const LeafLanes& lt,
                                             bool lanes_ready, uint32_t nthreads = blockDim.x) {
  issue_image(d, smem, j, lt, lanes_ready, nthreads);
  if (!d.stage_offsets) return;
  const uint64_t i0 = j.tile * d.tile;
  const uint32_t cnt = (uint32_t)min<uint64_t>(d.tile, j.count - i0);
  const uint32_t es = off_bytes(d.stage_type);
  const uint8_t* g = d.stage_offsets + i0 * es;
  uint8_t* head = reinterpret_cast<uint8_t*>(carve(smem, d).offs);
  const uint32_t need = (cnt + 1) * es;
  const uint64_t column = (d.n + 1) * es;
  if (d.dma && ((uintptr_t)g & 15) == 0) {
    const uint32_t up = round16(need);
    dma_run(head, d.stage_offsets, column >= 16 ? 16u : es, nthreads);
    dma_run(head + 16, g, (uint64_t)up <= column - i0 * es ? up : need, nthreads);
  } else {
    g2l(head, d.stage_offsets, es, threadIdx.x, blockDim.x);
    g2l(head + 16, g, need, threadIdx.x, blockDim.x);
  }
}

// Fused local scan of jagged counts held in the source records: writes the
// tile's exclusive offsets (entry i0 holds the tile total until the totals
// pass replaces it with the tile's prefix).
template <class DD>
__device__ __forceinline__ void scan_tile(const DD& d, const DenseLds& m, uint64_t i0, uint32_t cnt,
                                          uint32_t* status) {
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const uint32_t per = (d.tile + nt - 1) / nt;
  const uint32_t o0 = tid * per;
  uint64_t sum = 0;
  for (uint32_t k = 0; k < per; ++k) {
    const uint32_t o = o0 + k;
    if (o < cnt) sum += *reinterpret_cast<const uint32_t*>(m.src + o * d.src.stride + d.scan_len_off);
  }
  uint64_t total;
  uint64_t run = block_exclusive_scan(sum, m.wsum, &total);
  for (uint32_t k = 0; k < per; ++k) {
    const uint32_t o = o0 + k;
    if (o < cnt) {
      store_off(d.scan_offsets, d.scan_off_type, i0 + o, o == 0 ? total : run);
      run += *reinterpret_cast<const uint32_t*>(m.src + o * d.src.stride + d.scan_len_off);
    }
  }
  if (tid == 0 && total > off_limit(d.scan_off_type)) flag(status, ST_FLAG_OVERFLOW);
}

// ------------------------------------------------------------------ transform
//
// Every leaf value of the tile moves from the source image to the
// destination image.  The transform is specialised on the two layout
// kinds, and each thread takes kObjPerThread objects per pass: the
// object-dependent part of every image address is computed once per
// object, and the per-leaf work (descriptor load, one switch) is shared by
// all of a thread's objects.  Full passes carry no per-object guards.

constexpr uint32_t kObjPerThread = 2;


// Object-dependent address terms of one side: addr = a + off + b * size.
template <uint32_t K, class SD>
__device__ __forceinline__ void obj_terms(const SD& s, uint32_t o, uint32_t& a, uint32_t& b) {
  if (K == KIND_AOS) {
    a = o * s.stride;
    b = 0;
  } else if (K == KIND_SOA) {
    a = 0;
    b = o;
  } else {
    const uint32_t blk = s.width == 1 ? o : __umulhi(o, s.width_magic);
    a = blk * s.width * s.obj_bytes;
    b = o - blk * s.width;
  }
}

template <uint32_t K, uint32_t SIZE>
__device__ __forceinline__ uint32_t at(uint32_t a, uint32_t off, uint32_t b) {
  return K == KIND_AOS ? a + off : a + off + b * SIZE;
}

// Store a value into an LDS image, or (GLOBAL) into global memory,
// non-temporally with NT.
template <bool GLOBAL, class T, bool NT = false>
__device__ __forceinline__ void put(uint8_t* p, T v) {
  if (GLOBAL && NT) st_nt(gp(reinterpret_cast<T*>(p)), v);
  else if (GLOBAL) *gp(reinterpret_cast<T*>(p)) = v;
  else *reinterpret_cast<T*>(p) = v;
}

// Threads tx of ntx (normally the whole work-group) take part.
template <uint32_t SK, uint32_t DK, bool FULL, bool DIRECT, bool NT = false, class DD>
__device__ __forceinline__ void transform_pass(const DD& d, const DenseLds& m, const LeafLanes& lt, uint64_t i0,
                                               uint32_t o0, uint32_t cnt, uint32_t tx, uint32_t ntx) {
  constexpr uint32_t P = kObjPerThread;
  const uint32_t nt = ntx;
  uint32_t sa[P], sb[P], da[P], db[P];
  bool ok[P];
#pragma unroll
  for (uint32_t k = 0; k < P; ++k) {
    const uint32_t o = o0 + tx + k * nt;
    ok[k] = FULL || o < cnt;
    obj_terms<SK>(d.src, o, sa[k], sb[k]);
    obj_terms<DK>(d.dst, o, da[k], db[k]);
  }
  const uint8_t* S = m.src;
  // Destination: the LDS image, or (DIRECT) the tile's place in global
  // memory -- AoSoA: the tile's first block, whose runs sit at the image
  // offsets; SoA: each column at the tile's first object.
  uint8_t* const Dtile = DIRECT ? d.dst.base + i0 * (DK == KIND_AOS ? d.dst.stride : d.dst.obj_bytes) : m.dst;
#define RL_MOVE(ST, DT, SS, DS, EXPR)                                                  \
  _Pragma("unroll") for (uint32_t k = 0; k < P; ++k) {                                 \
    if (FULL || ok[k]) {                                                               \
      const ST x = *reinterpret_cast<const ST*>(S + at<SK, SS>(sa[k], so, sb[k]));     \
      put<DIRECT, DT, NT>((col ? colp + i0 * DS : Dtile) + at<DK, DS>(da[k], dof, db[k]), (EXPR)); \
    }                                                                                  \
  }
  const uint32_t nl = d.n_leaves;
  for (uint32_t c = 0; c < nl; ++c) {
    const uint32_t so = lane_of(lt.src_off, c);
    const bool col = DIRECT && DK == KIND_SOA;
    uint8_t* const colp = col ? reinterpret_cast<uint8_t*>(((uint64_t)lane_of(lt.col_hi, c) << 32) | lane_of(lt.col_lo, c))
                              : nullptr;
    const uint32_t dof = col ? 0u : lane_of(lt.dst_off, c);
    switch (lane_of(lt.code, c) & 255) {
      case CODE_COPY1: RL_MOVE(uint8_t, uint8_t, 1, 1, x); break;
      case CODE_COPY2: RL_MOVE(uint16_t, uint16_t, 2, 2, x); break;
      case CODE_COPY4: RL_MOVE(uint32_t, uint32_t, 4, 4, x); break;
      case CODE_COPY8: RL_MOVE(uint64_t, uint64_t, 8, 8, x); break;
      case CODE_NARROW: RL_MOVE(double, float, 8, 4, narrow_value(x)); break;
      case CODE_WIDEN: RL_MOVE(float, double, 4, 8, widen_value(x)); break;
      default: break;   // slow leaves: transform_slow
    }
  }
#undef RL_MOVE
}

// Leaves at misaligned image addresses and destination record (pointer,
// count) pairs: one object per thread, generic address arithmetic.  Which
// leaves take this path, and the (pointer, count) fields, come from the
// wave's leaf lanes.  `run` holds the staged offsets entries i0 .. i0 + cnt
// of d.stage_offsets, whose entry 0 is `first`.
template <class DD>
__device__ __forceinline__ void transform_slow(const DD& d, const LeafLanes& lt, uint8_t* src_img, uint8_t* dst_img,
                                               const uint8_t* run, uint64_t first, uint64_t i0, uint32_t cnt) {
  const uint32_t nl = d.n_leaves;
  for (uint32_t c = 0; c < nl; ++c) {
    const uint32_t w = lane_of(lt.code, c);
    const uint32_t code = w & 255;
    if (code < CODE_BYTES) continue;
    if (code == CODE_BYTES) {
      const auto& L = d.leaf[c];
      for (uint32_t o = threadIdx.x; o < cnt; o += blockDim.x) {
        uint32_t sa, sb, da, db;
        if (d.src.kind == KIND_AOS) obj_terms<KIND_AOS>(d.src, o, sa, sb);
        else if (d.src.kind == KIND_SOA) obj_terms<KIND_SOA>(d.src, o, sa, sb);
        else obj_terms<KIND_AOSOA>(d.src, o, sa, sb);
        if (d.dst.kind == KIND_AOS) obj_terms<KIND_AOS>(d.dst, o, da, db);
        else if (d.dst.kind == KIND_SOA) obj_terms<KIND_SOA>(d.dst, o, da, db);
        else obj_terms<KIND_AOSOA>(d.dst, o, da, db);
        move_value(dst_img + da + L.dst_off + db * L.dst_size, src_img + sa + L.src_off + sb * L.src_size, L);
      }
      continue;
    }
    // destination record (pointer, count) from the source offsets: the
    // destination is a record image
    const uint32_t dof = lane_of(lt.dst_off, c), stride = d.dst.stride;
    const bool byte_wise = (w >> 24) & 1;
    const uint32_t ot = (w >> 25) & 15;
    const uint8_t* col =
        reinterpret_cast<const uint8_t*>(((uint64_t)lane_of(lt.scol_hi, c) << 32) | lane_of(lt.scol_lo, c));
    const bool staged = col == d.stage_offsets;
    const uint64_t f = staged ? first : load_off(col, ot, 0);
    const uint64_t ms = lane_of(lt.src_off, c);
    for (uint32_t o = threadIdx.x; o < cnt; o += blockDim.x) {
      uint8_t* dp = dst_img + o * stride + dof;
      const uint64_t a = staged ? staged_off(run, ot, o) : load_off(col, ot, i0 + o);
      if (code == CODE_PTR) {
        const uint64_t v = (a - f) * ms;
        if (byte_wise) copy_bytes(dp, reinterpret_cast<const uint8_t*>(&v), 8);
        else *reinterpret_cast<uint64_t*>(dp) = v;
      } else {
        const uint32_t v = (uint32_t)((staged ? staged_off(run, ot, o + 1) : load_off(col, ot, i0 + o + 1)) - a);
        if (byte_wise) copy_bytes(dp, reinterpret_cast<const uint8_t*>(&v), 4);
        else *reinterpret_cast<uint32_t*>(dp) = v;
      }
    }
  }
}

// Checks of the staged offsets of a tile: non-decreasing and inside the
// source member capacity for every object, and (last tile) the total
// inside the destination member capacity.  Status flags as the offsets
// pass sets them.
template <class DD>
__device__ __forceinline__ void check_staged(const DD& d, const uint8_t* run, uint64_t first, uint64_t i0,
                                             uint32_t cnt, uint32_t* status) {
  const uint32_t ot = d.stage_type;
  const uint64_t cap = d.stage_src_capacity;
  bool overflow = false, bounds = false;
  for (uint32_t o = threadIdx.x; o < cnt; o += blockDim.x) {
    const uint64_t a = staged_off(run, ot, o), b = staged_off(run, ot, o + 1);
    if (b < a) overflow = true;
    else if (a > cap || b - a > cap - a) bounds = true;
  }
  if (overflow) flag(status, ST_FLAG_OVERFLOW);
  if (bounds) flag(status, ST_FLAG_BOUNDS);
  if (i0 + cnt == d.n && threadIdx.x == 0) {
    const uint64_t a = staged_off(run, ot, cnt);
    if (a >= first && a - first > d.stage_dst_capacity) flag(status, ST_FLAG_CAPACITY);
  }
}

// Unused slots of the last AoSoA block of a partial tile, written as zeros
// in global memory (the image path zero-fills its LDS image instead).
template <class DD>
__device__ __forceinline__ void zero_tail_direct(const DD& d, uint64_t i0, uint32_t cnt, uint32_t tx, uint32_t ntx) {
  const auto& s = d.dst;
  const uint32_t end = s.width == 1 ? cnt : __umulhi(cnt + s.width - 1, s.width_magic) * s.width;
  if (end == cnt) return;
  uint8_t* const Dtile = s.base + i0 * s.obj_bytes;
  for (uint32_t c = 0; c < d.n_leaves; ++c) {
    const auto& L = d.leaf[c];
    const uint32_t dsz = (leaf_word(L, 2) >> 8) & 255;
    for (uint32_t o = cnt + tx; o < end; o += ntx) {
      uint32_t a, b;
      obj_terms<KIND_AOSOA>(s, o, a, b);
      uint8_t* p = Dtile + a + L.dst_off + b * dsz;
      switch (dsz) {
        case 1: put<true, uint8_t>(p, 0); break;
        case 2: put<true, uint16_t>(p, 0); break;
        case 4: put<true, uint32_t>(p, 0); break;
        default: put<true, uint64_t>(p, 0); break;
      }
    }
  }
}

template <uint32_t SK, uint32_t DK, bool DIRECT, bool NT = false, class DD>
__device__ __forceinline__ void transform_kinds(const DD& d, const DenseLds& m, const LeafLanes& lt, uint64_t i0,
                                                uint32_t cnt, uint32_t tx = threadIdx.x, uint32_t ntx = blockDim.x) {
  const uint32_t per_pass = kObjPerThread * ntx;
  for (uint32_t o0 = 0; o0 < cnt; o0 += per_pass) {
    if (o0 + per_pass <= cnt) transform_pass<SK, DK, true, DIRECT, NT>(d, m, lt, i0, o0, cnt, tx, ntx);
    else transform_pass<SK, DK, false, DIRECT, NT>(d, m, lt, i0, o0, cnt, tx, ntx);
  }
  if (DIRECT && DK == KIND_AOSOA) zero_tail_direct(d, i0, cnt, tx, ntx);
}

// Direct destinations (SoA columns, AoSoA blocks): each leaf of a wave's
// consecutive objects is one contiguous run in global memory, so the
// stores coalesce without a destination image.
template <bool NT, class DD>
__device__ __forceinline__ void transform_direct_kinds(const DD& d, const DenseLds& m, const LeafLanes& lt,
                                                       uint64_t i0, uint32_t cnt, uint32_t nt, uint32_t tx) {
  switch (d.src.kind * 3 + d.dst.kind) {
    case KIND_AOS * 3 + KIND_SOA: transform_kinds<KIND_AOS, KIND_SOA, true, NT>(d, m, lt, i0, cnt, tx, nt); break;
    case KIND_AOS * 3 + KIND_AOSOA: transform_kinds<KIND_AOS, KIND_AOSOA, true, NT>(d, m, lt, i0, cnt, tx, nt); break;
    case KIND_SOA * 3 + KIND_SOA: transform_kinds<KIND_SOA, KIND_SOA, true, NT>(d, m, lt, i0, cnt, tx, nt); break;
    case KIND_SOA * 3 + KIND_AOSOA: transform_kinds<KIND_SOA, KIND_AOSOA, true, NT>(d, m, lt, i0, cnt, tx, nt); break;
    case KIND_AOSOA * 3 + KIND_SOA: transform_kinds<KIND_AOSOA, KIND_SOA, true, NT>(d, m, lt, i0, cnt, tx, nt); break;
    case KIND_SOA * 3 + KIND_AOS: transform_kinds<KIND_SOA, KIND_AOS, true, NT>(d, m, lt, i0, cnt, tx, nt); break;
    case KIND_AOSOA * 3 + KIND_AOS: transform_kinds<KIND_AOSOA, KIND_AOS, true, NT>(d, m, lt, i0, cnt, tx, nt); break;
    default: transform_kinds<KIND_AOSOA, KIND_AOSOA, true, NT>(d, m, lt, i0, cnt, tx, nt); break;
  }
}

template <class DD>
__device__ __forceinline__ void transform_direct(const DD& d, const DenseLds& m, const LeafLanes& lt, uint64_t i0,
                                                 uint32_t cnt, uint32_t nt, uint32_t tx = threadIdx.x) {
  if (d.stream_stores) transform_direct_kinds<true>(d, m, lt, i0, cnt, nt, tx);
  else transform_direct_kinds<false>(d, m, lt, i0, cnt, nt, tx);
}

template <class DD>
__device__ __forceinline__ void transform_tile(const DD& d, const DenseLds& m, const LeafLanes& lt, uint64_t i0,
                                               uint32_t cnt, uint32_t* status, uint32_t nt = blockDim.x) {
  if (d.dst_direct) {
    transform_direct(d, m, lt, i0, cnt, nt);
    return;
  }
  if (d.slow_leaves) {
    const uint8_t* run = reinterpret_cast<const uint8_t*>(m.offs) + 16;
    const uint64_t first = d.stage_offsets ? staged_off(run - 16, d.stage_type, 0) : 0;
    if (d.stage_offsets) check_staged(d, run, first, i0, cnt, status);
    transform_slow(d, lt, m.src, m.dst, run, first, i0, cnt);
  }
  switch (d.src.kind * 3 + d.dst.kind) {
    case KIND_AOS * 3 + KIND_AOS: transform_kinds<KIND_AOS, KIND_AOS, false>(d, m, lt, i0, cnt); break;
    case KIND_AOS * 3 + KIND_SOA: transform_kinds<KIND_AOS, KIND_SOA, false>(d, m, lt, i0, cnt); break;
    case KIND_AOS * 3 + KIND_AOSOA: transform_kinds<KIND_AOS, KIND_AOSOA, false>(d, m, lt, i0, cnt); break;
    case KIND_SOA * 3 + KIND_AOS: transform_kinds<KIND_SOA, KIND_AOS, false>(d, m, lt, i0, cnt); break;
    case KIND_SOA * 3 + KIND_SOA: transform_kinds<KIND_SOA, KIND_SOA, false>(d, m, lt, i0, cnt); break;
    case KIND_SOA * 3 + KIND_AOSOA: transform_kinds<KIND_SOA, KIND_AOSOA, false>(d, m, lt, i0, cnt); break;
    case KIND_AOSOA * 3 + KIND_AOS: transform_kinds<KIND_AOSOA, KIND_AOS, false>(d, m, lt, i0, cnt); break;
    case KIND_AOSOA * 3 + KIND_SOA: transform_kinds<KIND_AOSOA, KIND_SOA, false>(d, m, lt, i0, cnt); break;
    default: transform_kinds<KIND_AOSOA, KIND_AOSOA, false>(d, m, lt, i0, cnt); break;
  }
}

// Convert the tiles handed out by `next` (a functor returning TileJob);
// `desc(item)` gives a job's descriptor.  (Jobs carry an index, not a
// pointer: the address of a kernel-argument descriptor must not escape
// into a loop-carried value, or the compiler copies it to scratch.)
template <class Next, class Desc>
__device__ __forceinline__ void dense_pipeline(uint8_t* smem, Next next, Desc desc, uint32_t* status) {
  LeafLanes lt;
  TileJob cur = next();
  if (cur.valid) {
    load_lanes(desc(cur.item), cur.item, lt);
    issue_source(desc(cur.item), smem, cur, lt, true);   // no stores outstanding yet
  }
  while (cur.valid) {
    const auto& d = desc(cur.item);
    const DenseLds m = carve(smem, d);
    const uint64_t i0 = cur.tile * d.tile;
    const uint32_t cnt = (uint32_t)min<uint64_t>(d.tile, cur.count - i0);
    const bool full = cnt == d.tile;
    // 1. source image in LDS
    dma_wait();
    __syncthreads();
    // 2. zero-filled destination image where padding or unused block slots exist
    if (!d.dst_direct && (d.zero_dst || (!full && d.dst.kind == KIND_AOSOA))) {
      v4u* z = reinterpret_cast<v4u*>(m.dst);
      const uint32_t nv = d.dst.image_bytes >> 4;
      for (uint32_t v = threadIdx.x; v < nv; v += blockDim.x) z[v] = v4u{0u, 0u, 0u, 0u};
      __syncthreads();
    }
    // 3. counts scan and value moves (into the destination image, or
    //    straight to global memory)
    if (d.scan_offsets) scan_tile(d, m, i0, cnt, status);
    transform_tile(d, m, lt, i0, cnt, status);
    __syncthreads();
    // 4. this tile's destination image out, then the next tile's source
    //    image in (its DMA is issued after the image reads, and overlaps
    //    the stores).  A next tile of another descriptor carves LDS
    //    differently: its source image may cover this destination image.
    const TileJob nxt = next();
    if (!d.dst_direct) {
      store_side(d, m.dst, i0, cnt, full);
      if (nxt.valid && nxt.item != cur.item) __syncthreads();
    }
    if (nxt.valid) {
      const bool reuse = nxt.item == lt.item;
      if (!reuse) load_lanes(desc(nxt.item), nxt.item, lt);
      issue_source(desc(nxt.item), smem, nxt, lt, reuse);
    }
    cur = nxt;
  }
}

// A lower bound of the vector-memory instructions each wave issues while
// transforming a tile: direct destinations store every fast leaf of each
// of a thread's kObjPerThread objects with one instruction per full pass
// (full passes have no per-object branches).  Other paths count nothing,
// which is always a lower bound.
template <class DD>
__device__ __forceinline__ uint32_t stores_at_least(const DD& d, uint32_t cnt, uint32_t nt) {
  if (!d.dst_direct || d.slow_leaves || d.scan_offsets) return 0;
  const uint32_t per_pass = kObjPerThread * nt;
  return (cnt / per_pass) * kObjPerThread * d.fast_leaves;
}

// One tile of the double-buffered pipeline: `cur` (its image in `cur_smem`,
// its leaf lanes in lc) is converted while the next tile's DMA, issued
// first into `nxt_smem` with its lanes in ln, is in flight.  `after` holds
// a lower bound of this wave's vector-memory instructions issued after the
// current tile's DMA; the wait lets that many stay outstanding, so the
// previous tile's stores keep draining while this tile starts.  Returns
// false when no tile follows.
template <class Next, class Desc>
__device__ __forceinline__ bool db_tile(uint8_t* cur_smem, uint8_t* nxt_smem, LeafLanes& lc, LeafLanes& ln,
                                        TileJob& cur, uint32_t& after, Next& next, Desc& desc, uint32_t* status,
                                        uint32_t nt) {
  vm_wait_at_most(after);
  __syncthreads();
  // every wave is past the previous tile, whose slot the next DMA reuses
  const TileJob nxt = next();
  if (nxt.valid) {
    const bool same = nxt.item == lc.item;
    if (same) ln = lc;
    else load_lanes_scalar(desc(nxt.item), nxt.item, ln);
    issue_source(desc(nxt.item), nxt_smem, nxt, lc, same, nt);
  }
  const auto& d = desc(cur.item);
  const DenseLds m = carve(cur_smem, d);
  const uint64_t i0 = cur.tile * d.tile;
  const uint32_t cnt = (uint32_t)min<uint64_t>(d.tile, cur.count - i0);
  const bool full = cnt == d.tile;
  if (!d.dst_direct && (d.zero_dst || (!full && d.dst.kind == KIND_AOSOA))) {
    v4u* z = reinterpret_cast<v4u*>(m.dst);
    const uint32_t nv = d.dst.image_bytes >> 4;
    for (uint32_t v = threadIdx.x; v < nv; v += nt) z[v] = v4u{0u, 0u, 0u, 0u};
    __syncthreads();
  }
  if (d.scan_offsets) scan_tile(d, m, i0, cnt, status);
  transform_tile(d, m, lc, i0, cnt, status, nt);
  if (!d.dst_direct) {
    __syncthreads();
    store_side(d, m.dst, i0, cnt, full);
  }
  after = stores_at_least(d, cnt, nt);
  cur = nxt;
  return nxt.valid != 0;
}

// The tiles handed out by `next`, two at a time: each work-group owns two
// LDS slots of `slot` bytes, and a tile's source DMA is issued before the
// previous tile's transform, so loads and stores of consecutive tiles
// overlap instead of the next DMA waiting behind the stores (the
// vector-memory counter retires in order).
template <class Next, class Desc>
__device__ __forceinline__ void dense_pipeline_db(uint8_t* smem, uint32_t slot, Next next, Desc desc,
                                                  uint32_t* status) {
  // the thread count is read once: blockDim.x is a 16-bit implicit
  // argument, read with a vector load wherever it is evaluated
  const uint32_t nt = blockDim.x;
  LeafLanes l0, l1;
  TileJob cur = next();
  if (!cur.valid) return;
  load_lanes_scalar(desc(cur.item), cur.item, l0);
  issue_source(desc(cur.item), smem, cur, l0, false, nt);
  uint32_t after = 0;
  while (db_tile(smem, smem + slot, l0, l1, cur, after, next, desc, status, nt) &&
         db_tile(smem + slot, smem, l1, l0, cur, after, next, desc, status, nt)) {
  }
}

// Tiles blockIdx.x, blockIdx.x + gridDim.x, ... of one conversion.
struct StridedTiles {
  uint64_t t, ntiles, count, base;
  uint32_t g;   // gridDim.x, read once (a 16-bit implicit argument is read with a vector load)
  __device__ __forceinline__ TileJob operator()() {
    TileJob j{0, 0, 0, count, base};
    if (t < ntiles) {
      j.valid = 1;
      j.tile = t;
      t += g;
    }
    return j;
  }
};

__global__ void __launch_bounds__(256, 7) dense_kernel(const DenseDesc) {
  extern __shared__ uint4 smem_raw[];
  const RL_C DenseDesc& d = kernel_arg<DenseDesc>();
  uint64_t count, base;
  dense_count(d, &count, &base);
  dense_pipeline(reinterpret_cast<uint8_t*>(smem_raw),
                 StridedTiles{blockIdx.x, (count + d.tile - 1) / d.tile, count, base, gridDim.x},
                 [&](uint32_t) -> const RL_C DenseDesc& { return kernel_arg<DenseDesc>(); }, d.status);
}

// The same conversion double-buffered (two tile slots of d.pipe_slot bytes
// per work-group).  The slots already limit residency, so registers may
// hold both tiles' leaf lanes: at least 4 waves per SIMD.
__global__ void __launch_bounds__(256, 4) dense_db_kernel(const DenseDesc) {
  extern __shared__ uint4 smem_raw[];
  const RL_C DenseDesc& d = kernel_arg<DenseDesc>();
  uint64_t count, base;
  dense_count(d, &count, &base);
  dense_pipeline_db(reinterpret_cast<uint8_t*>(smem_raw), d.pipe_slot,
                    StridedTiles{blockIdx.x, (count + d.tile - 1) / d.tile, count, base, gridDim.x},
                    [&](uint32_t) -> const RL_C DenseDesc& { return kernel_arg<DenseDesc>(); }, d.status);
}

// ------------------------------------------------------------------ offsets

// Exclusive scan of the per-tile totals left by the dense kernel's fused
// scan (stored at entry tile * T), writing each tile's prefix there and the
// grand total at entry n.  One work-group.
template <class TD>
__device__ void scan_totals_body(const TD& d, uint64_t* wsum, uint32_t* status) {
  const uint64_t ntiles = (d.n + d.tile - 1) / d.tile;
  uint64_t carry = 0;
  for (uint64_t c0 = 0; c0 < ntiles; c0 += blockDim.x) {
    const uint64_t k = c0 + threadIdx.x;
    const uint64_t v = k < ntiles ? load_off(d.offsets, d.off_type, k * d.tile) : 0;
    uint64_t total;
    const uint64_t ex = block_exclusive_scan(v, wsum, &total);
    if (k < ntiles) store_off(d.offsets, d.off_type, k * d.tile, carry + ex);
    carry += total;
  }
  if (threadIdx.x == 0) {
    store_off(d.offsets, d.off_type, d.n, carry);
    if (carry > off_limit(d.off_type)) flag(status, ST_FLAG_OVERFLOW);
    else if (carry > d.capacity) flag(status, ST_FLAG_CAPACITY);
  }
}

__global__ void __launch_bounds__(1024) scan_totals_kernel(const ScanTotalsDesc d) {
  __shared__ uint64_t wsum[17];
  scan_totals_body(d, wsum, d.status);
}

// Add tile prefixes, then copy the members of the tile's objects from the
// pool into the member columns.  One work-group per tile (grid-stride).
// Members [m_lo, m_hi) of a tile, four consecutive members per thread
// (groups aligned to 4 member indices): one binary search per group for the
// owner of its first member, then the owner advances member by member.
// NW > 0: every member leaf is a 4-byte word at offset 4k of a packed
// record of NW words, and every member column is 16-byte aligned; each
// column then receives one 16-byte store per full group.  NW == 0: any
// member record, value by value.  Every read stays inside the member block
// the object's record validated against the pool (vlen).
template <uint32_t NW, class GD>
__device__ __forceinline__ void gather_members(const GD& d, const uint64_t* offs, const uint64_t* ptrs,
                                               const uint32_t* vlen, uint32_t cnt, uint64_t m_lo, uint64_t m_hi) {
  const uint64_t start = m_lo & ~3ull;
  const uint64_t ngroups = (m_hi - start + 3) >> 2;
  for (uint64_t g = threadIdx.x; g < ngroups; g += blockDim.x) {
    const uint64_t base = start + 4 * g;
    const uint64_t first = base < m_lo ? m_lo : base;
    uint32_t lo = 0, hi = cnt;   // owner of `first`: last object with offs <= first
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (offs[mid] <= first) lo = mid; else hi = mid;
    }
    const uint8_t* src[4];
    bool ok[4];
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
      const uint64_t m = base + k;
      ok[k] = false;
      src[k] = nullptr;
      if (m < m_lo || m >= m_hi) continue;
      while (lo + 1 < cnt && offs[lo + 1] <= m) ++lo;
      const uint64_t j = m - offs[lo];
      if (m < offs[lo] || j >= vlen[lo]) continue;
      ok[k] = true;
      src[k] = d.pool + ptrs[lo] + j * d.mstride;
    }
    if (NW > 0) {
      uint32_t w[4][NW > 0 ? NW : 1];
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k)
#pragma unroll
        for (uint32_t q = 0; q < NW; ++q) w[k][q] = ok[k] ? gp(reinterpret_cast<const uint32_t*>(src[k]))[q] : 0u;
      const bool full = ok[0] && ok[1] && ok[2] && ok[3];
#pragma unroll
      for (uint32_t q = 0; q < NW; ++q) {
        RL_G uint32_t* col = gp(reinterpret_cast<uint32_t*>(d.mcol[q]));
        if (full) {
          *reinterpret_cast<RL_G v4u*>(col + base) = v4u{w[0][q], w[1][q], w[2][q], w[3][q]};
        } else {
#pragma unroll
          for (uint32_t k = 0; k < 4; ++k)
            if (ok[k]) col[base + k] = w[k][q];
        }
      }
    } else {
      for (uint32_t q = 0; q < d.n_members; ++q) {
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) {
          if (!ok[k]) continue;
          const uint8_t* s = src[k] + d.moff[q];
          uint8_t* dst = d.mcol[q] + (base + k) * d.msize[q];
          switch (d.msize[q]) {
            case 1: put<true, uint8_t>(dst, *gp(s)); break;
            case 2: put<true, uint16_t>(dst, *gp(reinterpret_cast<const uint16_t*>(s))); break;
            case 4: put<true, uint32_t>(dst, *gp(reinterpret_cast<const uint32_t*>(s))); break;
            default: put<true, uint64_t>(dst, *gp(reinterpret_cast<const uint64_t*>(s))); break;
          }
        }
      }
    }
  }
}

// One 4-byte DMA per lane from global memory into LDS: lane l lands at
// lds_base + 4 l (lds_base wave-uniform).  See dma16.
__device__ __forceinline__ void dma4(const uint8_t* g, uint32_t lds_base) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dword %0, off"
               :: "v"(g), "s"(lds_base) : "memory", "m0");
}

// Members [m_lo, m_hi) whose records are NW packed 4-byte words: each lane
// finds its member's owner (binary search over the staged offsets) and
// DMAs the member's words into one LDS column per word; after one wait the
// columns go out as 16-byte vectors.  No member's load waits behind another
// member's store.  A member's LDS slot has the same address mod 16 as its
// place in the destination column.  Members outside their record's
// validated block are not loaded (their column entries are then
// unspecified; the status word says so).
template <uint32_t NW, class GD>
__device__ __forceinline__ void gather_words(const GD& d, const uint64_t* offs, const uint64_t* ptrs,
                                             const uint32_t* vlen, uint32_t cnt, uint64_t m_lo, uint64_t m_hi,
                                             uint32_t* stage) {
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const uint32_t lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  for (uint64_t p0 = m_lo; p0 < m_hi; p0 += kGatherStage) {
    const uint32_t pm = (uint32_t)min<uint64_t>(kGatherStage, m_hi - p0);
    const uint32_t sh = (uint32_t)(p0 & 3);   // slot of member p0
    for (uint32_t vb = wave * 64; vb < pm; vb += nw * 64) {
      const uint32_t k = vb + lane;
      const uint64_t m = p0 + k;
      bool ok = k < pm;
      const uint8_t* src = d.pool;
      if (ok) {
        uint32_t lo = 0, hi = cnt;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (offs[mid] <= m) lo = mid; else hi = mid;
        }
        const uint64_t j = m - offs[lo];
        ok = m >= offs[lo] && j < vlen[lo];
        src = d.pool + ptrs[lo] + j * d.mstride;
      }
#pragma unroll
      for (uint32_t q = 0; q < NW; ++q) {
        uint8_t* col = reinterpret_cast<uint8_t*>(stage + q * (kGatherStage + 4) + sh + vb);
        const uint32_t base = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_ptr)col);
        if (ok) dma4(src + 4 * q, base);
      }
    }
    dma_wait();
    __syncthreads();
    // columns out: head words up to 16-byte alignment, vectors, tail words
    const uint64_t a0 = min<uint64_t>((p0 + 3) & ~3ull, p0 + pm), a1 = max<uint64_t>(a0, (p0 + pm) & ~3ull);
#pragma unroll
    for (uint32_t q = 0; q < NW; ++q) {
      const uint32_t* sq = stage + q * (kGatherStage + 4) + sh;   // member p0 + i at sq[i]
      RL_G uint32_t* col = gp(reinterpret_cast<uint32_t*>(d.mcol[q])) + p0;
      const uint32_t head = (uint32_t)(a0 - p0), body = (uint32_t)(a1 - a0) >> 2;
      for (uint32_t i = tid; i < head; i += nt) col[i] = sq[i];
      const v4u* sv = reinterpret_cast<const v4u*>(sq + head);
      RL_G v4u* cv = reinterpret_cast<RL_G v4u*>(col + head);
      for (uint32_t v = tid; v < body; v += nt) cv[v] = sv[v];
      for (uint32_t i = head + 4 * body + tid; i < pm; i += nt) col[i] = sq[i];
    }
    __syncthreads();
  }
}

// Sub-tile u of d.sub objects (a part of a scan tile of d.tile objects):
// its offsets made final and its objects' members copied from the pool into
// the member columns.  The fused scan left tile-local offsets; the totals
// pass put the tile's prefix at the tile's first entry.  Each work-group
// reads and rewrites only its own entries plus that prefix (which keeps its
// value); the end of its last object is final(last) + count(last), as the
// scan computed it.  Objects (final offset, validated record pointer and
// count) are staged in LDS; every pool read stays inside the member block
// the record validated (vlen).
template <class GD>
__device__ __forceinline__ void gather_sub(const GD& d, uint64_t u, uint8_t* smem, uint32_t* status) {
  const uint32_t S = d.sub;
  uint64_t* offs = reinterpret_cast<uint64_t*>(smem);   // S + 1
  uint64_t* ptrs = offs + (S + 1);                      // S
  uint32_t* vlen = reinterpret_cast<uint32_t*>(ptrs + S);
  uint32_t* stage = reinterpret_cast<uint32_t*>(smem + gather_stage_offset(S));
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const uint64_t i0 = u * S;
  if (i0 >= d.n) return;   // uniform
  const uint32_t cnt = (uint32_t)min<uint64_t>(S, d.n - i0);
  const uint64_t t0 = i0 / d.tile * d.tile;
  const uint64_t prefix = load_off(d.offsets, d.off_type, t0);
  const uint64_t limit = off_limit(d.off_type);
  const uint64_t pool_end = d.pool_bytes;
  for (uint32_t k = tid; k < cnt; k += nt) {
    const uint64_t i = i0 + k;
    uint64_t v = prefix;
    if (i != t0) {
      v += load_off(d.offsets, d.off_type, i);
      store_off(d.offsets, d.off_type, i, v);
    }
    offs[k] = v & limit;
    if (d.n_members == 0 && k + 1 < cnt) continue;
    const uint8_t* rec = d.records + i * d.rec_stride;
    const uint64_t len = *gp(reinterpret_cast<const uint32_t*>(rec + d.len_off));
    if (k + 1 == cnt) offs[cnt] = (v + len) & limit;
    if (d.n_members == 0) continue;
    const uint64_t p = *gp(reinterpret_cast<const uint64_t*>(rec + d.ptr_off));
    const bool good = (p & (uint64_t)(d.malign - 1)) == 0 && p <= pool_end && len <= (pool_end - p) / d.mstride;
    ptrs[k] = p;
    vlen[k] = good ? (uint32_t)len : 0u;   // members readable for this object
    if (!good) flag(status, ST_FLAG_BOUNDS);
  }
  if (d.n_members == 0) return;   // uniform: offsets only
  __syncthreads();
  const uint64_t lo = offs[0];
  uint64_t hi = offs[cnt];
  if (hi > d.capacity) hi = d.capacity;
  if (hi > lo) {
    switch (d.packed_words) {
      case 1: gather_words<1>(d, offs, ptrs, vlen, cnt, lo, hi, stage); break;
      case 2: gather_words<2>(d, offs, ptrs, vlen, cnt, lo, hi, stage); break;
      case 3: gather_words<3>(d, offs, ptrs, vlen, cnt, lo, hi, stage); break;
      case 4: gather_words<4>(d, offs, ptrs, vlen, cnt, lo, hi, stage); break;
      default: gather_members<0>(d, offs, ptrs, vlen, cnt, lo, hi); break;
    }
  }
  __syncthreads();
}

__global__ void __launch_bounds__(256) gather_kernel(const GatherDesc) {
  extern __shared__ uint4 smem_raw[];
  const RL_C GatherDesc& d = kernel_arg<GatherDesc>();
  const uint64_t nsub = (d.n + d.sub - 1) / d.sub;
  for (uint64_t u = blockIdx.x; u < nsub; u += gridDim.x)
    gather_sub(kernel_arg<GatherDesc>(), u, reinterpret_cast<uint8_t*>(smem_raw), d.status);
}

// Offsets column -> offsets column, rebased to start at 0, with the checks
// of a well-formed source (non-decreasing, inside the source capacity) and
// of the destination capacity.
template <class RD>
__device__ void rebase_range(const RD& d, uint64_t begin, uint64_t step, uint64_t last, uint32_t* status) {
  const uint64_t first = load_off(d.src, d.off_type, 0);
  if (last > d.n) last = d.n;
  for (uint64_t i = begin; i <= last; i += step) {
    const uint64_t a = load_off(d.src, d.off_type, i);
    if (d.dst) store_off(d.dst, d.off_type, i, a - first);
    if (i < d.n) {
      const uint64_t b = load_off(d.src, d.off_type, i + 1);
      if (b < a) flag(status, ST_FLAG_OVERFLOW);
      else if (a > d.src_capacity || b - a > d.src_capacity - a) flag(status, ST_FLAG_BOUNDS);
    } else if (a >= first && a - first > d.dst_capacity) {
      flag(status, ST_FLAG_CAPACITY);
    }
  }
}

__global__ void rebase_kernel(const RebaseDesc d) {
  rebase_range(d, blockIdx.x * (uint64_t)blockDim.x + threadIdx.x, (uint64_t)gridDim.x * blockDim.x, d.n, d.status);
}

// ------------------------------------------------------------------ single-pass jagged forward
//
// AoS records holding (pointer, count) pairs of one jagged group, member
// records of NW packed 4-byte words, into an offsets column and member
// columns, in one kernel (Sec. VI: the prefix sum of the member counts).
// Work-group b converts tile b.  Per tile:
//  1. the records arrive in LDS by DMA;
//  2. their counts are scanned (tile-local exclusive offsets, aggregate A)
//     and A is published at once in the tile's look-back word;
//  3. the per-object leaves go straight to their destination;
//  4. the first staging pass of the tile's members is DMA'd from the pool
//     into LDS columns by tile-local member index;
//  5. meanwhile the tile's prefix P (the members of all earlier tiles) is
//     assembled by a block-wide look-back: in rounds of up to four words
//     per thread, every earlier tile's word is read at once, back to the
//     nearest tile that has published its inclusive prefix; a tile whose
//     word is not there yet is summed from its records in global memory
//     instead of being waited for.  P + A is published;
//  6. the offsets (P + local) and the members (at P + local index) are
//     stored at their final places.
// No work-group ever waits for another, so no dispatch order or residency
// is assumed, and no atomic read-modify-write is used (same-address
// atomics serialise at about 11 ns each on this chip).
//
// Look-back words: bits 63..62 state (1: aggregate, 2: inclusive prefix),
// bits 61..40 the launch epoch (low 22 bits; the host numbers the launches
// on each look-back buffer), bits 39..0 the value, saturated at 2^40 - 1
// (any member total that large exceeds every capacity; the plan only uses
// this kernel for capacities below 2^39).  A word of another launch counts
// as missing (a buffer would have to see 2^22 launches, all with fewer
// tiles, for an old word to carry the current epoch).

constexpr uint32_t kLbEpochMask = (1u << 22) - 1;

__device__ __forceinline__ uint64_t sat40(uint64_t v) { return v < kLookbackValueLimit ? v : kLookbackValueLimit; }

__device__ __forceinline__ uint64_t lb_word(uint32_t state, uint32_t epoch, uint64_t v) {
  return ((uint64_t)state << 62) | ((uint64_t)(epoch & kLbEpochMask) << 40) | sat40(v);
}

__device__ __forceinline__ uint64_t lb_load(const uint64_t* p) {
  return __hip_atomic_load(gp(const_cast<uint64_t*>(p)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void lb_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, d, 64));
  return v;
}
// Inclusive prefix sum over the 64 lanes of a wave by DPP moves (no LDS):
// shifts by 1, 2, 4, 8 inside each row of 16 lanes, then each row adds the
// last lane of the rows before it (lanes outside a move's source read 0).
__device__ __forceinline__ uint32_t wave_inclusive_scan_u32(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);   // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);   // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);   // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);   // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);   // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);   // row_bcast:31
  return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// LDS carve-up of the single-pass jagged kernel.
struct JagLds {
  uint8_t* img;        // records of the tile
  uint64_t* loff;      // tile-local exclusive offsets, T + 1 entries (entry cnt = aggregate)
  uint64_t* ptrs;      // pool byte offsets of the tile's objects
  uint32_t* vlen;      // members readable per object (0 for a record outside its pool)
  uint64_t* wsum;      // block scan: one u64 per wave + 1
  uint64_t* rsum;      // look-back sums, one per wave
  uint32_t* rmin;      // look-back minimum, one per wave
  uint16_t* own;       // tile-local object of each member of a staging pass
  uint32_t* stage;     // NW columns of (stage + 4) words
};

// LDS bytes before the staging columns: records, offsets, pointers,
// counts, scan and look-back sums.
template <class JD>
__host__ __device__ __forceinline__ uint32_t jag_head_bytes(const JD& j) {
  const uint32_t T = j.dense.tile;
  return round16(j.dense.src.image_bytes) + round16((T + 1) * 8) + round16(T * 8) + round16(T * 4) +
         round16(18 * 8) + round16(4 * 8) + round16(4 * 4) + round16(j.stage * 2);
}

template <class JD>
__host__ __device__ __forceinline__ uint32_t jag_lds_layout(const JD& j) {
  return jag_head_bytes(j) + j.words * (j.stage + 4) * 4;
}

template <class JD>
__device__ __forceinline__ JagLds jag_carve(uint8_t* smem, const JD& j) {
  const uint32_t T = j.dense.tile;
  JagLds m;
  uint8_t* p = smem;
  m.img = p; p += round16(j.dense.src.image_bytes);
  m.loff = reinterpret_cast<uint64_t*>(p); p += round16((T + 1) * 8);
  m.ptrs = reinterpret_cast<uint64_t*>(p); p += round16(T * 8);
  m.vlen = reinterpret_cast<uint32_t*>(p); p += round16(T * 4);
  m.wsum = reinterpret_cast<uint64_t*>(p); p += round16(18 * 8);
  m.rsum = reinterpret_cast<uint64_t*>(p); p += round16(4 * 8);
  m.rmin = reinterpret_cast<uint32_t*>(p); p += round16(4 * 4);
  m.own = reinterpret_cast<uint16_t*>(p); p += round16(j.stage * 2);
  m.stage = reinterpret_cast<uint32_t*>(p);
  return m;
}

// Member total of tile `tile` summed from its records in global memory by
// the whole wave (for a tile whose look-back word did not arrive in time).
template <class JD>
__device__ __forceinline__ uint64_t jag_tile_total(const JD& j, uint64_t tile) {
  const uint32_t T = j.dense.tile, stride = j.dense.src.stride;
  const uint64_t i0 = tile * T;
  const uint32_t cnt = (uint32_t)min<uint64_t>(T, j.dense.n - i0);
  const uint8_t* rec = j.dense.src.base + i0 * stride + j.len_off;
  uint64_t s = 0;
  for (uint32_t k = threadIdx.x & 63; k < cnt; k += 64) s += *gp(reinterpret_cast<const uint32_t*>(rec + (uint64_t)k * stride));
  return wave_sum_u64(s);
}

// Prefix of tile t (t >= 1): the saturated member total of tiles 0 .. t-1,
// assembled by one wave (its loads must not queue behind member DMAs of
// the same wave: a wave's memory counter retires in order).  In rounds of
// 64 x kLookbackPerLane words, every earlier tile's word is read at once,
// back to the nearest tile with an inclusive prefix of this launch.  Words
// that have not arrived are polled again for a bounded time (their tiles
// are running and publish within microseconds); after that, a missing
// tile's total is summed from its records, so no tile ever depends on
// another work-group making progress.
constexpr uint32_t kLookbackPerLane = 8;
constexpr uint32_t kLookbackPolls = 256;   // a few hundred microseconds of polling before summing records

template <class JD>
__device__ uint64_t jag_look_back(const JD& j, const uint64_t* flags, uint64_t t, uint32_t epoch) {
  constexpr uint32_t K = kLookbackPerLane;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t ep = epoch & kLbEpochMask;
  auto valid = [&](uint64_t w) { return (w >> 62) != 0 && (uint32_t)((w >> 40) & kLbEpochMask) == ep; };
  uint64_t prefix = 0;
  uint64_t hi = t;   // this round: tiles hi - 1 - d for distances d = lane + 64 k
  while (hi > 0) {
    uint64_t w[K];
#pragma unroll
    for (uint32_t k = 0; k < K; ++k) {
      const uint64_t d = lane + 64ull * k;
      w[k] = d < hi ? lb_load(flags + (hi - 1 - d)) : 0;
    }
    uint32_t near, missing;
    for (uint32_t poll = 0;; ++poll) {
      near = 0xFFFFFFFFu;   // nearest inclusive prefix of this launch
#pragma unroll
      for (uint32_t k = 0; k < K; ++k) {
        const uint64_t d = lane + 64ull * k;
        if (d < hi && (w[k] >> 62) == 2 && valid(w[k])) near = min(near, (uint32_t)d);
      }
      near = wave_min_u32(near);
      missing = 0;   // words needed (up to the nearest prefix) and not there
#pragma unroll
      for (uint32_t k = 0; k < K; ++k) {
        const uint64_t d = lane + 64ull * k;
        if (d < hi && d <= near && !valid(w[k])) missing |= 1u << k;
      }
      if (!__any(missing != 0) || poll == kLookbackPolls) break;
      __builtin_amdgcn_s_sleep(8);
#pragma unroll
      for (uint32_t k = 0; k < K; ++k)
        if (missing & (1u << k)) w[k] = lb_load(flags + (hi - 1 - (lane + 64ull * k)));
    }
    uint64_t sum = 0;
#pragma unroll
    for (uint32_t k = 0; k < K; ++k) {
      const uint64_t d = lane + 64ull * k;
      if (d < hi && d <= near && valid(w[k])) sum += w[k] & kLookbackValueLimit;
    }
    // still missing after the polls: the whole wave sums those tiles'
    // records, one tile at a time
    for (;;) {
      const uint64_t b = __ballot(missing != 0);
      if (!b) break;
      const uint32_t src = (uint32_t)__builtin_ctzll(b);
      const uint32_t mk = __shfl(missing, src, 64);
      const uint32_t k = __builtin_ctz(mk);
      const uint64_t total = jag_tile_total(j, hi - 1 - (src + 64ull * k));
      if (lane == src) {
        sum += total;
        missing &= missing - 1;
      }
    }
    prefix = sat40(prefix + wave_sum_u64(sat40(sum)));
    if (near != 0xFFFFFFFFu) break;
    hi = hi > 64ull * K ? hi - 64ull * K : 0;
  }
  return prefix;
}

// Owners (tile-local object index) of tile-local members [p0, p0 + pm)
// into m.own[0 .. pm): each thread fills a contiguous run, finding the
// owner of its first member by binary search over the tile-local offsets
// and then stepping over object boundaries, so the work is spread by
// members whatever the counts are.  All threads of the work-group take
// part; a barrier must follow before m.own is read.
__device__ __forceinline__ void jag_owners(const JagLds& m, uint32_t cnt, uint64_t p0, uint32_t pm) {
  const uint32_t nt = blockDim.x;
  const uint32_t R = (pm + nt - 1) / nt;
  const uint32_t r0 = threadIdx.x * R, r1 = min(pm, r0 + R);
  if (r0 >= r1) return;
  const uint64_t k0 = p0 + r0;
  uint32_t lo = 0, hi = cnt;   // last object whose first member is <= k0
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (m.loff[mid] <= k0) lo = mid; else hi = mid;
  }
  uint64_t next = m.loff[lo + 1];   // member k < total = loff[cnt], so lo + 1 <= cnt
  for (uint32_t r = r0; r < r1; ++r) {
    const uint64_t k = p0 + r;
    while (k >= next) next = m.loff[++lo + 1];
    m.own[r] = (uint16_t)lo;
  }
}

// DMA the words of tile-local members [p0, p0 + pm) from the pool into the
// LDS columns (slot k of a column holds member p0 + k); owners from m.own.
// Members outside their record's validated block are not loaded (their
// destination entries are then unspecified and the status says so).
// Waves w0 .. w0 + nw - 1 of the work-group take part (the calling wave
// must be one of them).
template <uint32_t NW, class JD>
__device__ __forceinline__ void jag_issue(const JD& j, const JagLds& m, uint64_t p0, uint32_t pm,
                                          uint32_t w0, uint32_t nw) {
  const uint32_t lane = threadIdx.x & 63, wave = (threadIdx.x >> 6) - w0;
  for (uint32_t vb = wave * 64; vb < pm; vb += nw * 64) {
    const uint32_t k = vb + lane;
    bool ok = k < pm;
    const uint8_t* src = j.pool;
    if (ok) {
      const uint32_t o = m.own[k];
      const uint64_t jj = p0 + k - m.loff[o];
      ok = jj < m.vlen[o];
      src = j.pool + m.ptrs[o] + jj * j.mstride;
    }
#pragma unroll
    for (uint32_t q = 0; q < NW; ++q) {
      uint32_t* col = m.stage + q * (j.stage + 4) + vb;
      const uint32_t base = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_ptr)(uint8_t*)col);
      if (ok) dma4(src + 4 * q, base);
    }
  }
}

// Store staged members [p0, p0 + pm) at destination index P + p0 + k, up
// to the capacity: 16-byte vectors where the destination is aligned, words
// at the ends.
template <uint32_t NW, class JD>
__device__ __forceinline__ void jag_store(const JD& j, const JagLds& m, uint64_t P, uint64_t p0, uint32_t pm) {
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const uint64_t lo = P + p0;
  const uint64_t hi = min<uint64_t>(lo + pm, j.capacity);
  if (hi <= lo) return;
  const uint64_t a0 = min<uint64_t>((lo + 3) & ~3ull, hi), a1 = max<uint64_t>(a0, hi & ~3ull);
#pragma unroll
  for (uint32_t q = 0; q < NW; ++q) {
    const uint32_t* sq = m.stage + q * (j.stage + 4);   // destination index x at sq[x - lo]
    RL_G uint32_t* col = gp(reinterpret_cast<uint32_t*>(j.mcol[q]));
    for (uint32_t i = tid; lo + i < a0; i += nt) col[lo + i] = sq[i];
    const uint32_t nv = (uint32_t)((a1 - a0) >> 2);
    const uint32_t* s0 = sq + (a0 - lo);
    RL_G v4u* cv = reinterpret_cast<RL_G v4u*>(col + a0);
    for (uint32_t v = tid; v < nv; v += nt) {
      const uint32_t* x = s0 + 4 * v;
      if (j.stream_members) st_nt(cv + v, v4u{x[0], x[1], x[2], x[3]});
      else cv[v] = v4u{x[0], x[1], x[2], x[3]};
    }
    for (uint64_t i = a1 + tid; i < hi; i += nt) col[i] = sq[i - lo];
  }
}

template <uint32_t NW>
__global__ void __launch_bounds__(256) jagged_kernel(const JaggedDesc) {
  extern __shared__ uint4 smem_raw[];
  uint8_t* smem = reinterpret_cast<uint8_t*>(smem_raw);
  const RL_C JaggedDesc& j = kernel_arg<JaggedDesc>();
  const RL_C DenseDesc& d = j.dense;
  const JagLds m = jag_carve(smem, j);
  uint64_t* const flags = j.lookback;
  uint32_t* const status = d.status;
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const uint64_t n = d.n;
  const uint32_t T = d.tile;
  const uint64_t t = blockIdx.x;
  const uint64_t i0 = t * T;
  if (i0 >= n) return;   // uniform
  const uint32_t cnt = (uint32_t)min<uint64_t>(T, n - i0);
  const uint32_t epoch = j.epoch;
  // 1. records (the leaf lanes are loaded first: issued after the DMA,
  // their wait would also wait for it, which cost 10% at 2^21 objects)
  LeafLanes lt;
  load_lanes(d, 0, lt);
  issue_source(d, smem, TileJob{1, 0, t, n, 0}, lt, true);
  // the descriptor fields of the scan and the member requests, read while
  // the records are in flight (the empty asm makes them arrive here: left
  // to the compiler, each would be read where it is first used, one
  // scalar-cache miss after another on the path to the first request)
  const uint32_t stride = d.src.stride, len_off = j.len_off, ptr_off = j.ptr_off;
  const uint64_t pool_end = j.pool_bytes;
  const uint32_t mstride = j.mstride, malign = j.malign;
  const uint32_t S = j.stage;
  const uint8_t* const pool = j.pool;
  asm volatile("" ::"s"(stride), "s"(len_off), "s"(ptr_off), "s"(pool_end), "s"(mstride), "s"(malign), "s"(S),
               "s"(pool), "s"(flags), "s"(epoch));
  dma_wait();
  __syncthreads();
  // 2. counts: every wave scans the tile's counts by itself, one object
  // per lane, 64 at a time (a DPP prefix sum: no LDS scan and no barrier
  // inside it); the last wave keeps the tile-local offsets, pointers and
  // validated counts in LDS, wave 1 publishes the tile's aggregate (wave
  // 0's look-back loads would otherwise wait for the store)
  const uint32_t lane = tid & 63, wave = tid >> 6, nwaves = nt >> 6;
  uint64_t A = 0;
  bool bad = false;
  for (uint32_t c0 = 0; c0 < cnt; c0 += 64) {
    const uint32_t o = c0 + lane;
    uint64_t len = 0, p = 0;
    if (o < cnt) {
      const uint8_t* rec = m.img + o * stride;
      len = *reinterpret_cast<const uint32_t*>(rec + len_off);
      p = *reinterpret_cast<const uint64_t*>(rec + ptr_off);
    }
    const bool good = o >= cnt || ((p & (uint64_t)(malign - 1)) == 0 && p <= pool_end && len * mstride <= pool_end - p);
    bad |= !good;
    // counts below 2^26 sum to less than 2^32 over 64 lanes: a 32-bit scan
    uint64_t inc;
    if (__all(len < (1u << 26))) {
      inc = wave_inclusive_scan_u32((uint32_t)len);
    } else {
      inc = len;
#pragma unroll
      for (int dd = 1; dd < 64; dd <<= 1) {
        const uint64_t x = __shfl_up(inc, dd, 64);
        if (lane >= (uint32_t)dd) inc += x;
      }
    }
    if (wave == nwaves - 1 && o < cnt) {
      m.loff[o] = A + inc - len;
      m.ptrs[o] = p;
      m.vlen[o] = good ? (uint32_t)len : 0u;
    }
    A += ((uint64_t)__builtin_amdgcn_readlane((int)(uint32_t)(inc >> 32), 63) << 32) |
         (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)inc, 63);
  }
  if (bad && wave == 0) flag(status, ST_FLAG_BOUNDS);
  if (tid == (nt > 64 ? 64u : 0u)) lb_store(flags + t, lb_word(t == 0 ? 2u : 1u, epoch, A));
  if (wave == nwaves - 1 && lane == 0) m.loff[cnt] = A;
  __syncthreads();   // tile-local offsets, pointers and counts in LDS
  const uint32_t pm0 = (uint32_t)min<uint64_t>(A, S);
  jag_owners(m, cnt, 0, pm0);
  __syncthreads();
  // 3.-5. wave 0 assembles the prefix while the other waves request the
  // first members and store the per-object leaves (a one-wave work-group
  // does the three in turn, the look-back first)
  DenseLds dm;
  dm.src = smem;
  dm.dst = smem;
  dm.wsum = m.wsum;
  dm.offs = m.wsum;
  uint64_t P = 0;
  if (wave == 0 && t > 0) P = jag_look_back(j, flags, t, epoch);
  if (nwaves == 1 || wave > 0) {
    const uint32_t w0 = nwaves == 1 ? 0 : 1;
    jag_issue<NW>(j, m, 0, pm0, w0, nwaves - w0);
    const uint32_t tx = tid - 64 * w0, ntx = nt - 64 * w0;
    // the two destination kinds of this kernel only (the whole switch of
    // transform_direct would raise the kernel's registers)
    if (d.stream_stores) {
      if (d.dst.kind == KIND_SOA) transform_kinds<KIND_AOS, KIND_SOA, true, true>(d, dm, lt, i0, cnt, tx, ntx);
      else transform_kinds<KIND_AOS, KIND_AOSOA, true, true>(d, dm, lt, i0, cnt, tx, ntx);
    } else {
      if (d.dst.kind == KIND_SOA) transform_kinds<KIND_AOS, KIND_SOA, true>(d, dm, lt, i0, cnt, tx, ntx);
      else transform_kinds<KIND_AOS, KIND_AOSOA, true>(d, dm, lt, i0, cnt, tx, ntx);
    }
  }
  if (tid == 0) m.rsum[0] = P;
  __syncthreads();
  P = m.rsum[0];
  if (tid == 0 && t > 0) lb_store(flags + t, lb_word(2u, epoch, P + A));
  // 6. offsets, then members that land inside the destination capacity
  //    (the loop is bounded by a real buffer whatever the counts say)
  for (uint32_t o = tid; o < cnt; o += nt) store_off(j.offsets, j.off_type, i0 + o, P + m.loff[o]);
  if (i0 + cnt == n && tid == 0) {
    const uint64_t all = sat40(P + A);
    store_off(j.offsets, j.off_type, n, all);
    if (all > off_limit(j.off_type)) flag(status, ST_FLAG_OVERFLOW);
    else if (all > j.capacity) flag(status, ST_FLAG_CAPACITY);
  }
  const uint64_t stored = min<uint64_t>(A, P < j.capacity ? j.capacity - P : 0);
  for (uint64_t p0 = 0; p0 < stored; p0 += S) {
    const uint32_t pm = (uint32_t)min<uint64_t>(S, stored - p0);
    if (p0 > 0) {
      jag_owners(m, cnt, p0, pm);
      __syncthreads();
      jag_issue<NW>(j, m, p0, pm, 0, nwaves);
    }
    dma_wait();
    __syncthreads();
    jag_store<NW>(j, m, P, p0, pm);
    __syncthreads();
  }
  // no DMA into LDS may be left in flight when the work-group ends (members
  // requested before the prefix showed them beyond the capacity)
  dma_wait();
}

// ------------------------------------------------------------------ plain copies

// Copy `bytes` from src to dst (device memory, or pinned host memory
// through its device address; ranges disjoint).  Where both ends share
// their address mod 16, the body moves as 16-byte vectors, one per thread
// per round of a grid-stride loop, with non-temporal loads and stores (a
// streaming copy leaves nothing worth caching); the head up to the
// alignment and the tail move as bytes; otherwise every byte moves on its
// own.  Measured over 1 GiB buffers (cold): one vector per thread per
// round at 4-5 work-groups per compute unit beats unrolled rounds and
// larger grids (5.9 against 4.1-4.9 TB/s read + write).
__global__ void __launch_bounds__(256) copy_kernel(uint8_t* dst, const uint8_t* src, uint64_t bytes) {
  const uint64_t tid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t nt = (uint64_t)gridDim.x * blockDim.x;
  uint64_t head = 0, nv = 0;
  if ((((uintptr_t)dst ^ (uintptr_t)src) & 15) == 0) {
    head = min<uint64_t>((16 - ((uintptr_t)dst & 15)) & 15, bytes);
    nv = (bytes - head) >> 4;
  } else {
    head = bytes;
  }
  for (uint64_t b = tid; b < head; b += nt) gp(dst)[b] = gp(src)[b];
  const RL_G v4u* sv = reinterpret_cast<const RL_G v4u*>(gp(src + head));
  RL_G v4u* dv = reinterpret_cast<RL_G v4u*>(gp(dst + head));
  for (uint64_t v = tid; v < nv; v += nt) __builtin_nontemporal_store(__builtin_nontemporal_load(sv + v), dv + v);
  for (uint64_t b = head + (nv << 4) + tid; b < bytes; b += nt) gp(dst)[b] = gp(src)[b];
}

// ------------------------------------------------------------------ insertion, deletion, compaction
//
// Insertion and deletion on a collection's arrays and the compaction of a
// filtered collection (Sec. VII-B) are gathers: destination object k takes
// every value of a chosen source object.  The mover below handles any pair
// of layout kinds at any object index, one thread per object (simple and
// general: these are not the bandwidth-critical path); members of jagged
// groups move with a wave per object.  The same mover converts layouts
// whose arrays are a user's index-to-address map (strided leaves, reached
// directly or through an index table; Sec. VII-B).

// Where object i sits in a side: its element for a strided side with an
// index table (false if past the elements), else i itself.
template <class GS>
__device__ __forceinline__ bool gen_element(const GS& s, uint64_t i, uint64_t* e) {
  if (s.kind != KIND_STRIDED || !s.index) {
    *e = i;
    return true;
  }
  *e = gp(s.index)[i];
  return *e < s.elements;
}

// Address of leaf c at position i (the object index, or a strided side's
// element from gen_element).
template <class GS>
__device__ __forceinline__ uint8_t* gen_addr(const GS& s, uint32_t c, uint32_t size, uint64_t i) {
  if (s.kind == KIND_STRIDED) return s.col[c] + i * s.off[c];
  if (s.kind == KIND_AOS) return s.base + i * s.stride + s.off[c];
  if (s.kind == KIND_SOA) return s.col[c] + i * size;
  const uint64_t blk = i / s.width;
  return s.base + blk * s.width * s.obj_bytes + (uint64_t)s.width * s.off[c] + (i - blk * s.width) * size;
}

// A value of 1, 2, 4 or 8 bytes at any address (little-endian).
__device__ __forceinline__ uint64_t gload(const uint8_t* p, uint32_t size) {
  if (((uintptr_t)p & (size - 1)) == 0) {
    switch (size) {
      case 1: return *gp(p);
      case 2: return *gp(reinterpret_cast<const uint16_t*>(p));
      case 4: return *gp(reinterpret_cast<const uint32_t*>(p));
      default: return *gp(reinterpret_cast<const uint64_t*>(p));
    }
  }
  uint64_t v = 0;
  for (uint32_t k = 0; k < size; ++k) v |= (uint64_t)gp(p)[k] << (8 * k);
  return v;
}

__device__ __forceinline__ void gstore(uint8_t* p, uint32_t size, uint64_t v) {
  if (((uintptr_t)p & (size - 1)) == 0) {
    switch (size) {
      case 1: *gp(p) = (uint8_t)v; return;
      case 2: *gp(reinterpret_cast<uint16_t*>(p)) = (uint16_t)v; return;
      case 4: *gp(reinterpret_cast<uint32_t*>(p)) = (uint32_t)v; return;
      default: *gp(reinterpret_cast<uint64_t*>(p)) = v; return;
    }
  }
  for (uint32_t k = 0; k < size; ++k) gp(p)[k] = (uint8_t)(v >> (8 * k));
}

__device__ __forceinline__ uint64_t gop(uint64_t v, uint32_t op) {
  if (op == OP_NARROW) return __float_as_uint(narrow_value(__longlong_as_double((long long)v)));
  if (op == OP_WIDEN) return (uint64_t)__double_as_longlong(widen_value(__uint_as_float((uint32_t)v)));
  return v;
}

__global__ void __launch_bounds__(256) move_kernel(const MoveDesc) {
  const RL_C MoveDesc& d = kernel_arg<MoveDesc>();
  const uint64_t count = d.count_dev ? *gp(d.count_dev) : d.count;
  const uint64_t nt = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < count; k += nt) {
    uint64_t i = 0, o;
    const bool in_src = d.zero_only || gen_element(d.src, d.map ? gp(d.map)[k] : d.src0 + k, &i);
    const bool in_dst = gen_element(d.dst, d.dst0 + k, &o);
    if (!in_src || !in_dst) {
      flag(d.status, ST_FLAG_BOUNDS);
      continue;
    }
    for (uint32_t c = 0; c < d.n_leaves; ++c) {
      uint8_t* dp = gen_addr(d.dst, c, d.dst_size[c], o);
      if (d.zero_only) {
        gstore(dp, d.dst_size[c], 0);
        continue;
      }
      gstore(dp, d.dst_size[c], gop(gload(gen_addr(d.src, c, d.src_size[c], i), d.src_size[c]), d.op[c]));
    }
  }
}

// Member count and first member index of object i of a group (form 0:
// validated against the pool; form 1: against the member storage).  *ok
// false for a block outside its storage.
template <class GG>
__device__ __forceinline__ void gen_block(const GG& g, uint64_t i, uint64_t* len, uint64_t* first, bool* ok) {
  if (g.form == 0) {
    const uint8_t* rec = g.records + i * g.rec_stride;
    const uint64_t l = gload(rec + g.len_off, 4);
    const uint64_t p = gload(rec + g.ptr_off, 8);
    const uint64_t pool_end = g.capacity * g.mstride;
    *ok = (p & (uint64_t)(g.malign - 1)) == 0 && p <= pool_end && l <= (pool_end - p) / g.mstride;
    *len = l;
    *first = p / g.mstride;
  } else {
    const uint64_t a = load_off(g.offsets, g.off_type, i), b = load_off(g.offsets, g.off_type, i + 1);
    *ok = b >= a && a <= g.capacity && b - a <= g.capacity - a;
    *len = b >= a ? b - a : 0;
    *first = a;
  }
}

template <class GG>
__device__ __forceinline__ uint8_t* gen_member(const GG& g, uint64_t first, uint64_t j, uint32_t q) {
  if (g.form == 0) return g.pool + (first + j) * g.mstride + g.moff[q];
  return g.mcol[q] + (first + j) * g.msize[q];
}

// Block-wide sum of one u64 per thread (result valid in every thread).
__device__ __forceinline__ uint64_t block_sum(uint64_t v, uint64_t* wsum) {
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wave_sum_u64(v);
  if (lane == 0) wsum[wave] = v;
  __syncthreads();
  uint64_t s = 0;
  for (uint32_t w = 0; w < nw; ++w) s += wsum[w];
  __syncthreads();
  return s;
}

// Compaction, pass 1: kept flags per tile.
__global__ void __launch_bounds__(256) select_count_kernel(const SelectDesc d) {
  __shared__ uint64_t wsum[8];
  const uint64_t i0 = (uint64_t)blockIdx.x * kSelectTile;
  const uint32_t cnt = (uint32_t)min<uint64_t>(kSelectTile, d.n - i0);
  uint64_t c = 0;
  for (uint32_t k = threadIdx.x; k < cnt; k += blockDim.x) c += gp(d.keep)[i0 + k] != 0;
  c = block_sum(c, wsum);
  if (threadIdx.x == 0) gp(d.tile_tot)[blockIdx.x] = c;
}

// Exclusive scan of `ntiles` per-tile totals in place (one work-group);
// the grand total goes to *total (and *total2 when set).
__device__ void scan_tiles_body(uint64_t* tot, uint64_t ntiles, uint64_t* total, uint64_t* total2, uint64_t* wsum) {
  uint64_t carry = 0;
  for (uint64_t c0 = 0; c0 < ntiles; c0 += blockDim.x) {
    const uint64_t k = c0 + threadIdx.x;
    const uint64_t v = k < ntiles ? gp(tot)[k] : 0;
    uint64_t all;
    const uint64_t ex = block_exclusive_scan(v, wsum, &all);
    if (k < ntiles) gp(tot)[k] = carry + ex;
    carry += all;
  }
  if (threadIdx.x == 0) {
    *gp(total) = carry;
    if (total2) *gp(total2) = carry;
  }
}

__global__ void __launch_bounds__(1024) select_scan_kernel(const SelectDesc d) {
  __shared__ uint64_t wsum[17];
  scan_tiles_body(d.tile_tot, (d.n + kSelectTile - 1) / kSelectTile, d.count, d.count_out, wsum);
}

// Compaction, pass 3: kept object indices at their places (each thread
// takes four consecutive flags of its tile).
__global__ void __launch_bounds__(256) select_map_kernel(const SelectDesc d) {
  __shared__ uint64_t wsum[17];
  const uint64_t i0 = (uint64_t)blockIdx.x * kSelectTile;
  const uint32_t cnt = (uint32_t)min<uint64_t>(kSelectTile, d.n - i0);
  const uint32_t per = kSelectTile / blockDim.x;
  const uint32_t o0 = threadIdx.x * per;
  uint64_t c = 0;
  for (uint32_t k = 0; k < per; ++k)
    if (o0 + k < cnt) c += gp(d.keep)[i0 + o0 + k] != 0;
  uint64_t all;
  uint64_t pos = gp(d.tile_tot)[blockIdx.x] + block_exclusive_scan(c, wsum, &all);
  for (uint32_t k = 0; k < per; ++k)
    if (o0 + k < cnt && gp(d.keep)[i0 + o0 + k] != 0) gp(d.map)[pos++] = i0 + o0 + k;
}

// Members of the kept objects, pass 1: each kept object's member count
// (lens[k]) and the per-tile sums (over kept-object tiles).
__global__ void __launch_bounds__(256) select_lens_kernel(const SelectDesc d) {
  __shared__ uint64_t wsum[8];
  const uint64_t count = *gp(d.count);
  const uint64_t k0 = (uint64_t)blockIdx.x * kSelectTile;
  uint64_t c = 0;
  for (uint32_t k = threadIdx.x; k < kSelectTile; k += blockDim.x) {
    const uint64_t kk = k0 + k;
    if (kk >= count) break;
    uint64_t len, first;
    bool ok;
    gen_block(d.src, gp(d.map)[kk], &len, &first, &ok);
    gp(d.lens)[kk] = len;
    c += len;
  }
  c = block_sum(c, wsum);
  if (threadIdx.x == 0) gp(d.tile_tot)[blockIdx.x] = c;
}

__global__ void __launch_bounds__(1024) select_lens_scan_kernel(const SelectDesc d) {
  __shared__ uint64_t wsum[17];
  // the total lands at lens[count]: the entry after the last kept object
  scan_tiles_body(d.tile_tot, (d.n + kSelectTile - 1) / kSelectTile, d.lens + *gp(d.count), nullptr, wsum);
}

// Pass 3: lens[k] becomes the first member index of kept object k.
__global__ void __launch_bounds__(256) select_offsets_kernel(const SelectDesc d) {
  __shared__ uint64_t wsum[17];
  const uint64_t count = *gp(d.count);
  const uint64_t k0 = (uint64_t)blockIdx.x * kSelectTile;
  const uint32_t per = kSelectTile / blockDim.x;
  const uint64_t o0 = k0 + threadIdx.x * per;
  uint64_t c = 0;
  for (uint32_t k = 0; k < per; ++k)
    if (o0 + k < count) c += gp(d.lens)[o0 + k];
  uint64_t all;
  uint64_t run = gp(d.tile_tot)[blockIdx.x] + block_exclusive_scan(c, wsum, &all);
  for (uint32_t k = 0; k < per; ++k)
    if (o0 + k < count) {
      const uint64_t l = gp(d.lens)[o0 + k];
      gp(d.lens)[o0 + k] = run;
      run += l;
    }
}

// Members of gathered objects: a wave per destination object.  Writes the
// destination's offsets entries (form 1) or records' (pointer, count)
// (form 0), checks the total against the offset type and the capacity,
// and copies the members that fit.
__global__ void __launch_bounds__(256) member_move_kernel(const MemberMoveDesc) {
  const RL_C MemberMoveDesc& d = kernel_arg<MemberMoveDesc>();
  const uint64_t count = *gp(d.count_dev);
  const uint64_t total = gp(d.out_off)[count];
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const uint64_t limit = d.dst.form == 1 ? off_limit(d.dst.off_type) : ~0ull;
  if (wave == 0 && lane == 0) {
    if (total > limit) flag(d.status, ST_FLAG_OVERFLOW);
    else if (total > d.dst.capacity) flag(d.status, ST_FLAG_CAPACITY);
    if (d.dst.form == 1) store_off(d.dst.offsets, d.dst.off_type, count, total);
  }
  for (uint64_t k = wave; k < count; k += nwaves) {
    const uint64_t i = gp(d.map)[k];
    uint64_t len, first;
    bool ok;
    gen_block(d.src, i, &len, &first, &ok);
    const uint64_t at = gp(d.out_off)[k];
    if (lane == 0) {
      if (!ok) flag(d.status, ST_FLAG_BOUNDS);
      if (d.dst.form == 1) {
        store_off(d.dst.offsets, d.dst.off_type, k, at);
      } else {
        uint8_t* rec = d.dst.records + k * d.dst.rec_stride;
        gstore(rec + d.dst.ptr_off, 8, at * d.dst.mstride);
        gstore(rec + d.dst.len_off, 4, len);
      }
    }
    if (!ok || at > d.dst.capacity || len > d.dst.capacity - at) continue;   // wave-uniform
    for (uint64_t j = lane; j < len; j += 64)
      for (uint32_t q = 0; q < d.src.n_members; ++q)
        gstore(gen_member(d.dst, at, j, q), d.dst.msize[q], gload(gen_member(d.src, first, j, q), d.src.msize[q]));
  }
}

// Append to a resident jagged group (both sides offsets + member columns):
// the destination's member count so far is its offsets entry `at`.
__global__ void __launch_bounds__(256) append_kernel(const AppendDesc d) {
  const uint64_t base = load_off(d.dst.offsets, d.dst.off_type, d.at);
  const uint64_t s0 = load_off(d.src.offsets, d.src.off_type, 0);
  const uint64_t s1 = load_off(d.src.offsets, d.src.off_type, d.count);
  const uint64_t tid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t nt = (uint64_t)gridDim.x * blockDim.x;
  // checks every thread makes alike (uniform early exit)
  uint32_t bad = 0;
  if (s1 < s0) bad = ST_FLAG_OVERFLOW;
  else if (s1 > d.src.capacity) bad = ST_FLAG_BOUNDS;
  else if (base + (s1 - s0) < base || base + (s1 - s0) > off_limit(d.dst.off_type)) bad = ST_FLAG_OVERFLOW;
  else if (base + (s1 - s0) > d.dst.capacity) bad = ST_FLAG_CAPACITY;
  if (bad) {
    if (tid == 0) flag(d.status, bad);
    return;
  }
  bool decreasing = false;
  for (uint64_t k = 1 + tid; k <= d.count; k += nt) {
    const uint64_t v = load_off(d.src.offsets, d.src.off_type, k);
    if (v < load_off(d.src.offsets, d.src.off_type, k - 1)) decreasing = true;
    store_off(d.dst.offsets, d.dst.off_type, d.at + k, base + (v - s0));
  }
  if (decreasing) flag(d.status, ST_FLAG_OVERFLOW);
  const uint64_t len = s1 - s0;
  for (uint32_t q = 0; q < d.src.n_members; ++q)
    for (uint64_t m = tid; m < len; m += nt)
      gstore(d.dst.mcol[q] + (base + m) * d.dst.msize[q], d.dst.msize[q],
             gload(d.src.mcol[q] + (s0 + m) * d.src.msize[q], d.src.msize[q]));
}

__global__ void zero_bytes_kernel(uint8_t* p, uint64_t bytes) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < bytes; i += (uint64_t)gridDim.x * blockDim.x)
    gp(p)[i] = 0;
}

__global__ void zero_kernel(uint32_t* p, uint64_t words) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < words; i += (uint64_t)gridDim.x * blockDim.x)
    gp(p)[i] = 0u;
}

// Status words of streams: one per stream that has run a conversion (the
// host assigns slots), so that reading and clearing one stream's word never
// races with another stream's kernels.
__device__ __align__(256) uint32_t g_status_words[kStatusSlots];

// Hand a stream's status flags to `out` (device memory, or the device
// address of pinned host memory) and clear them, in stream order.
__global__ void take_status_kernel(uint32_t* status, uint32_t* out) {
  RL_G uint32_t* w = gp(status);
  const uint32_t f = *w;
  *w = 0;
  *gp(out) = f;
}

// ------------------------------------------------------------------ batches

// Per dense step: the object count and source base (device-side counts of
// member steps are read here once, before the dense pass).
__global__ void batch_count_kernel(const BatchTables b) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < b.n_dense; k += gridDim.x * blockDim.x) {
    uint64_t count, base;
    dense_count(cdesc(b.dense, k), &count, &base);
    gp(b.dense_counts)[2 * k] = count;
    gp(b.dense_counts)[2 * k + 1] = base;
  }
}

// Every dense step of every item: the tiles of all items form one space;
// work-group w takes tiles w, w + grid, ... (no shared counters: same-address
// atomics from thousands of work-groups serialise in L2).  A tile's map
// entry is loaded two tiles ahead and its step's counts one tile ahead, so
// handing out a tile never waits on a dependent load.
// A vector-memory load: uniform addresses would otherwise become scalar
// loads, whose completion the next LDS wait (same counter) would also wait
// for; vector loads are waited for only where their values are used.
__device__ __forceinline__ uint64_t vload(const uint64_t* p) {
  return *reinterpret_cast<const volatile RL_G uint64_t*>(gp(p));
}

struct BatchTiles {
  const BatchTables* b;
  uint64_t t;              // tile handed out by the next call
  uint64_t e1, e2;         // map entries of tiles t and t + grid
  uint64_t c1, base1;      // counts of tile t's step
  __device__ __forceinline__ BatchTiles(const BatchTables* tb, uint64_t first) : b(tb), t(first), e1(0), e2(0), c1(0), base1(0) {
    const uint64_t g = gridDim.x;
    if (t < b->dense_tiles) {
      e1 = vload(b->dense_map + t);
      const uint32_t item = (uint32_t)(e1 >> 32);
      c1 = vload(b->dense_counts + 2 * item);
      base1 = vload(b->dense_counts + 2 * item + 1);
    }
    if (t + g < b->dense_tiles) e2 = vload(b->dense_map + t + g);
  }
  __device__ __forceinline__ TileJob operator()() {
    const uint64_t g = gridDim.x;
    while (t < b->dense_tiles) {
      const uint32_t item = __builtin_amdgcn_readfirstlane((uint32_t)(e1 >> 32));
      const uint32_t local = __builtin_amdgcn_readfirstlane((uint32_t)e1);
      const uint64_t count = c1, base = base1;
      // advance the two-stage prefetch
      t += g;
      if (t < b->dense_tiles) {
        const uint32_t it2 = (uint32_t)(e2 >> 32);
        c1 = vload(b->dense_counts + 2 * it2);
        base1 = vload(b->dense_counts + 2 * it2 + 1);
        e1 = e2;
        if (t + g < b->dense_tiles) e2 = vload(b->dense_map + t + g);
      }
      const uint32_t tile = cdesc(b->dense, item).tile;
      if ((uint64_t)local * tile < count) {
        TileJob j{1, item, local, 0, 0};
        j.count = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(count >> 32)) << 32) |
                  __builtin_amdgcn_readfirstlane((uint32_t)count);
        j.base = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(base >> 32)) << 32) |
                 __builtin_amdgcn_readfirstlane((uint32_t)base);
        return j;
      }
    }
    return TileJob{0, 0, 0, 0, 0};
  }
};

__global__ void __launch_bounds__(256, 6) batch_dense_kernel(const BatchTables b) {
  extern __shared__ uint4 smem_raw[];
  dense_pipeline(reinterpret_cast<uint8_t*>(smem_raw), BatchTiles(&b, blockIdx.x),
                 [&](uint32_t item) -> const RL_C DenseDesc& { return cdesc(b.dense, item); }, b.status);
}

// The same tiles for the double-buffered pipeline: each wave holds the
// work-group's next 64 map entries, one per lane (with their steps' counts
// and bases), loaded together and refilled every 64 tiles, so handing out
// a tile makes no memory access: a load there would be waited for with
// every store still in flight (the counter retires in order).
struct ChunkTiles {
  const BatchTables* b;
  uint64_t t;         // first tile of the held chunk
  uint32_t k, n;      // next entry to hand out, entries held
  uint64_t e, c, base;
  uint32_t g;         // gridDim.x, read once
  __device__ __forceinline__ explicit ChunkTiles(const BatchTables* tb)
      : b(tb), t(blockIdx.x), k(0), n(0), e(0), c(0), base(0), g(gridDim.x) {}
  __device__ __forceinline__ void refill() {
    const uint64_t tiles = b->dense_tiles;
    const uint64_t tl = t + (uint64_t)(threadIdx.x & 63) * g;
    n = t < tiles ? (uint32_t)min<uint64_t>(64, (tiles - t + g - 1) / g) : 0;
    k = 0;
    if (tl < tiles) {
      e = gp(b->dense_map)[tl];
      const uint32_t item = (uint32_t)(e >> 32);
      c = gp(b->dense_counts)[2 * item];
      base = gp(b->dense_counts)[2 * item + 1];
    }
  }
  __device__ __forceinline__ static uint64_t lane64(uint64_t v, uint32_t l) {
    return ((uint64_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), (int)l) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, (int)l);
  }
  __device__ __forceinline__ TileJob operator()() {
    while (true) {
      if (k == n) {
        if (t >= b->dense_tiles) return TileJob{0, 0, 0, 0, 0};
        refill();
        if (n == 0) return TileJob{0, 0, 0, 0, 0};
      }
      const uint32_t idx = k++;
      if (k == n) t += 64ull * g;
      const uint64_t ee = lane64(e, idx), cc = lane64(c, idx), bb = lane64(base, idx);
      const uint32_t item = (uint32_t)(ee >> 32), local = (uint32_t)ee;
      if ((uint64_t)local * cdesc(b->dense, item).tile < cc) return TileJob{1, item, local, cc, bb};
    }
  }
};

// Batches with double-buffered dense steps (two slots of b.pipe_slot bytes).
__global__ void __launch_bounds__(256, 4) batch_dense_db_kernel(const BatchTables b) {
  extern __shared__ uint4 smem_raw[];
  dense_pipeline_db(reinterpret_cast<uint8_t*>(smem_raw), b.pipe_slot, ChunkTiles(&b),
                    [&](uint32_t item) -> const RL_C DenseDesc& { return cdesc(b.dense, item); }, b.status);
}

// Fan-out groups (steps converting the same source tiles, their counts
// known on the host, direct destinations): a work-group brings a source
// tile into LDS once, and its thread groups of b.fan_per threads convert
// it, group k into step k's destination.  Each wave holds its own step's
// leaf lanes; the source fields of a group's steps are identical, so any
// wave's lanes serve the shared DMA.
__global__ void __launch_bounds__(512) batch_fanout_kernel(const BatchTables b) {
  extern __shared__ uint4 smem_raw[];
  uint8_t* const smem = reinterpret_cast<uint8_t*>(smem_raw);
  // 16-bit implicit arguments, read once
  const uint32_t nt = blockDim.x, g = gridDim.x;
  const uint32_t per = b.fan_per;
  const uint32_t sub = __builtin_amdgcn_readfirstlane(threadIdx.x / per);
  const uint32_t tx = threadIdx.x - sub * per;
  LeafLanes lt;
  lt.item = ~0u;
  // a tile's group is found by walking the group ranges with scalar loads
  // (a vector load of a tile map would wait behind this wave's stores)
  uint32_t grp = 0;
  for (uint32_t u = blockIdx.x; u < b.fan_tiles; u += g) {
    while (u >= cdesc(b.fan, grp).end) ++grp;
    const RL_C FanGroup& fg = cdesc(b.fan, grp);
    const uint64_t tile = u - fg.first;
    const uint32_t nd = fg.n_dst, s0 = fg.step[0];
    const uint32_t mine = sub < nd ? fg.step[sub] : s0;
    const bool fresh = mine != lt.item;
    if (fresh) load_lanes(cdesc(b.dense, mine), mine, lt);
    const RL_C DenseDesc& d0 = cdesc(b.dense, s0);
    issue_source(d0, smem, TileJob{1, s0, tile, d0.n, 0}, lt, !fresh, nt);
    dma_wait();
    __syncthreads();
    if (sub < nd) {
      const RL_C DenseDesc& d = cdesc(b.dense, mine);
      const uint64_t i0 = tile * d.tile;
      transform_direct(d, carve(smem, d), lt, i0, (uint32_t)min<uint64_t>(d.tile, d.n - i0), per, tx);
    }
    // the next tile's DMA overwrites the image
    __syncthreads();
  }
}

// A fan-out tile: its group, the tile within the group's source, and the
// step this thread group converts (the group's first step for thread
// groups beyond its steps, which only help with the DMA).
struct FanJob {
  uint32_t valid, step, s0, nd;
  uint64_t tile;
};

// Job of fan-out tile u; grp walks forward over the group ranges (u only
// grows within a work-group).
__device__ __forceinline__ FanJob fan_job(const BatchTables& b, uint32_t u, uint32_t& grp, uint32_t sub) {
  FanJob j{0, 0, 0, 0, 0};
  if (u >= b.fan_tiles) return j;
  while (u >= cdesc(b.fan, grp).end) ++grp;
  const RL_C FanGroup& fg = cdesc(b.fan, grp);
  j.valid = 1;
  j.nd = fg.n_dst;
  j.s0 = fg.step[0];
  j.step = sub < j.nd ? fg.step[sub] : j.s0;
  j.tile = u - fg.first;
  return j;
}

// The fan-out tiles double-buffered: two LDS slots of b.fan_slot bytes;
// the next tile's source DMA is issued before the current tile's
// transform, and the wait at the top of the next tile lets this wave's
// stores of the current tile stay in flight (the counter retires in
// order: with at most `after` operations outstanding, `after` a lower
// bound of the stores issued after that DMA, the DMA is done).
__global__ void __launch_bounds__(512) batch_fanout_db_kernel(const BatchTables b) {
  extern __shared__ uint4 smem_raw[];
  uint8_t* cs = reinterpret_cast<uint8_t*>(smem_raw);
  uint8_t* ns = cs + b.fan_slot;
  const uint32_t nt = blockDim.x, g = gridDim.x;
  const uint32_t per = b.fan_per;
  const uint32_t sub = __builtin_amdgcn_readfirstlane(threadIdx.x / per);
  const uint32_t tx = threadIdx.x - sub * per;
  uint32_t grp = 0, u = blockIdx.x;
  FanJob cur = fan_job(b, u, grp, sub);
  if (!cur.valid) return;
  LeafLanes lc, ln;
  load_lanes_scalar(cdesc(b.dense, cur.step), cur.step, lc);
  {
    const RL_C DenseDesc& d0 = cdesc(b.dense, cur.s0);
    issue_source(d0, cs, TileJob{1, cur.s0, cur.tile, d0.n, 0}, lc, false, nt);
  }
  uint32_t after = 0;
  while (true) {
    vm_wait_at_most(after);
    __syncthreads();
    // every wave is past the previous tile, whose slot the next DMA reuses
    u += g;
    const FanJob nxt = fan_job(b, u, grp, sub);
    if (nxt.valid) {
      if (nxt.step == lc.item) ln = lc;
      else load_lanes_scalar(cdesc(b.dense, nxt.step), nxt.step, ln);
      const RL_C DenseDesc& d0 = cdesc(b.dense, nxt.s0);
      issue_source(d0, ns, TileJob{1, nxt.s0, nxt.tile, d0.n, 0}, lc, false, nt);
    }
    after = 0;
    if (sub < cur.nd) {
      const RL_C DenseDesc& d = cdesc(b.dense, cur.step);
      const uint64_t i0 = cur.tile * d.tile;
      const uint32_t cnt = (uint32_t)min<uint64_t>(d.tile, d.n - i0);
      transform_direct(d, carve(cs, d), lc, i0, cnt, per, tx);
      after = stores_at_least(d, cnt, per);
    }
    if (!nxt.valid) break;
    cur = nxt;
    lc = ln;
    uint8_t* const t = cs;
    cs = ns;
    ns = t;
  }
}

// Tile-total scans (one work-group each) and offsets rebases.
__global__ void __launch_bounds__(1024) batch_misc_kernel(const BatchTables b) {
  __shared__ uint64_t wsum[17];
  const uint32_t j = blockIdx.x;
  if (j < b.n_totals) {
    scan_totals_body(cdesc(b.totals, j), wsum, b.status);
  } else if (j - b.n_totals < b.rebase_tiles) {
    // rebases in tiles of kRebaseTile entries, spread over work-groups
    const uint32_t t = j - b.n_totals;
    const uint32_t item = b.rebase_item[t];
    const uint64_t begin = (t - b.rebase_prefix[item]) * (uint64_t)kRebaseTile;
    rebase_range(cdesc(b.rebase, item), begin + threadIdx.x, blockDim.x, begin + kRebaseTile - 1, b.status);
  }
}

// Sub-tiles of every jagged item, strided like the dense kernel.
__global__ void __launch_bounds__(256) batch_gather_kernel(const BatchTables b) {
  extern __shared__ uint4 smem_raw[];
  for (uint64_t u = blockIdx.x; u < b.gather_tiles; u += gridDim.x) {
    const uint32_t item = __builtin_amdgcn_readfirstlane(b.gather_item[u]);
    gather_sub(cdesc(b.gather, item), u - b.gather_prefix[item], reinterpret_cast<uint8_t*>(smem_raw), b.status);
  }
}

// ------------------------------------------------------------------ launchers

uint32_t dense_lds_bytes(const DenseDesc& d) {
  return round16(d.src.image_bytes) + (d.dst_direct ? 0u : round16(d.dst.image_bytes)) +
         round16(17 * sizeof(uint64_t)) + (d.stage_offsets ? (d.tile + 4) * 8 : 0u);
}

uint64_t dense_tiles(const DenseDesc& d) { return (d.n + d.tile - 1) / d.tile; }

// LDS is handed to work-groups in granules of 1,280 bytes on gfx950
// (measured: residency against dynamic LDS size from 16 to 64 KiB in 512 B
// steps matches floor(160 KiB / round_up(bytes, 1280)) exactly); the
// occupancy query assumes finer granules and overcounts just below each
// granule boundary.
constexpr uint32_t kLdsGranule = 1280;

// Work-groups of a kernel that fit on the device at once (occupancy x
// compute units), per (device, kernel, threads, LDS bytes); 0 if unknown.
static uint32_t resident_blocks(const void* kernel, uint32_t threads, uint32_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, uint32_t, uint32_t>, uint32_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  const auto key = std::make_tuple(dev, kernel, threads, lds);
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0, lds_cu = 0;
  uint32_t r = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, (int)threads, lds) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && per_cu > 0) {
    if (lds && hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess &&
        lds_cu > 0) {
      const uint32_t granules = (lds + kLdsGranule - 1) / kLdsGranule;
      per_cu = std::min<int>(per_cu, (int)((uint32_t)lds_cu / (granules * kLdsGranule)));
    }
    if (per_cu > 0) r = (uint32_t)(per_cu * cus);
  }
  cache[key] = r;
  return r;
}

uint32_t batch_resident_blocks(uint32_t threads, uint32_t lds, bool pipelined) {
  return resident_blocks(pipelined ? reinterpret_cast<const void*>(batch_dense_db_kernel)
                                   : reinterpret_cast<const void*>(batch_dense_kernel), threads, lds);
}

uint32_t fanout_resident_blocks(uint32_t threads, uint32_t lds, bool pipelined) {
  return resident_blocks(pipelined ? reinterpret_cast<const void*>(batch_fanout_db_kernel)
                                   : reinterpret_cast<const void*>(batch_fanout_kernel), threads, lds);
}

hipError_t launch_dense(const DenseDesc& d, uint32_t threads, uint32_t grid, hipStream_t s) {
  if (threads == 0 || threads > kDenseMaxThreads || threads % 64) return hipErrorInvalidValue;
  if (d.pipe_slot && d.pipe_slot < dense_lds_bytes(d)) return hipErrorInvalidValue;
  const uint32_t lds = d.pipe_slot ? 2 * d.pipe_slot : dense_lds_bytes(d);
  // persistent work-groups: no more than fit at once (a second round of
  // work-groups would start late and leave the tail on few units)
  const void* k = d.pipe_slot ? reinterpret_cast<const void*>(dense_db_kernel) : reinterpret_cast<const void*>(dense_kernel);
  const uint32_t res = resident_blocks(k, threads, lds);
  if (res && grid > res) grid = res;
  if (d.pipe_slot) hipLaunchKernelGGL(dense_db_kernel, dim3(grid), dim3(threads), lds, s, d);
  else hipLaunchKernelGGL(dense_kernel, dim3(grid), dim3(threads), lds, s, d);
  return hipGetLastError();
}

hipError_t launch_scan_totals(const ScanTotalsDesc& d, hipStream_t s) {
  hipLaunchKernelGGL(scan_totals_kernel, dim3(1), dim3(1024), 0, s, d);
  return hipGetLastError();
}

uint32_t gather_lds_bytes(uint32_t sub, uint32_t words) {
  return gather_stage_offset(sub) + words * (kGatherStage + 4) * 4;
}

hipError_t launch_gather(const GatherDesc& d, uint32_t threads, hipStream_t s) {
  if (threads == 0 || threads > 256 || threads % 64 || d.sub == 0) return hipErrorInvalidValue;
  const uint64_t nsub = (d.n + d.sub - 1) / d.sub;
  const uint32_t lds = gather_lds_bytes(d.sub, d.packed_words);
  uint64_t grid = std::min<uint64_t>(nsub ? nsub : 1, 65535ull * 8);
  const uint32_t res = resident_blocks(reinterpret_cast<const void*>(gather_kernel), threads, lds);
  if (res && grid > res) grid = res;
  hipLaunchKernelGGL(gather_kernel, dim3((uint32_t)grid), dim3(threads), lds, s, d);
  return hipGetLastError();
}

hipError_t launch_rebase(const RebaseDesc& d, hipStream_t s) {
  const uint64_t work = d.n + 1;
  const uint32_t grid = (uint32_t)((work + 255) / 256 < 4096 ? (work + 255) / 256 : 4096);
  hipLaunchKernelGGL(rebase_kernel, dim3(grid), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_batch(const BatchTables& b, uint32_t dense_threads, uint32_t gather_threads,
                        uint32_t grid, uint32_t dense_lds, uint32_t gather_lds, hipStream_t s,
                        uint32_t fan_threads, uint32_t fan_lds) {
  if (dense_threads == 0 || dense_threads > kDenseMaxThreads || dense_threads % 64) return hipErrorInvalidValue;
  if (gather_threads == 0 || gather_threads > 256 || gather_threads % 64) return hipErrorInvalidValue;
  if (b.fan_tiles && (b.fan_per == 0 || b.fan_per % 64 || fan_threads % b.fan_per || fan_threads == 0 ||
                      fan_threads > kFanMaxThreads || (b.fan_slot && (b.fan_slot % 16 || fan_lds < 2 * b.fan_slot))))
    return hipErrorInvalidValue;
  const uint32_t grid_req = grid;
  const uint32_t dense_grid = std::min<uint32_t>(
      grid ? grid : std::max<uint32_t>(1, batch_resident_blocks(dense_threads, dense_lds, b.pipe_slot != 0)),
      std::max(1u, b.dense_tiles));
  if (!grid) grid = 2048;   // finalisation and gather kernels
  if (b.dense_tiles) {
    if (b.device_counts) {
      hipLaunchKernelGGL(batch_count_kernel, dim3((b.n_dense + 255) / 256), dim3(256), 0, s, b);
      hipError_t e0 = hipGetLastError();
      if (e0 != hipSuccess) return e0;
    }
    if (b.pipe_slot) hipLaunchKernelGGL(batch_dense_db_kernel, dim3(dense_grid), dim3(dense_threads), dense_lds, s, b);
    else hipLaunchKernelGGL(batch_dense_kernel, dim3(dense_grid), dim3(dense_threads), dense_lds, s, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (b.fan_tiles) {
    const uint32_t fres = fanout_resident_blocks(fan_threads, fan_lds, b.fan_slot != 0);
    const uint32_t fgrid = std::min<uint32_t>(b.fan_tiles, grid_req ? grid_req : (fres ? fres : 2048));
    if (b.fan_slot) hipLaunchKernelGGL(batch_fanout_db_kernel, dim3(fgrid), dim3(fan_threads), fan_lds, s, b);
    else hipLaunchKernelGGL(batch_fanout_kernel, dim3(fgrid), dim3(fan_threads), fan_lds, s, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (b.n_totals + b.rebase_tiles) {
    hipLaunchKernelGGL(batch_misc_kernel, dim3(b.n_totals + b.rebase_tiles), dim3(1024), 0, s, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (b.gather_tiles) {
    const uint32_t gres = resident_blocks(reinterpret_cast<const void*>(batch_gather_kernel), gather_threads, gather_lds);
    const uint32_t ggrid = std::min<uint32_t>(b.gather_tiles, gres ? gres : grid);
    hipLaunchKernelGGL(batch_gather_kernel, dim3(ggrid), dim3(gather_threads), gather_lds, s, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

uint32_t jagged_lds_bytes(const JaggedDesc& j) { return jag_lds_layout(j); }

hipError_t launch_jagged(const JaggedDesc& j, uint32_t threads, hipStream_t s) {
  if (threads == 0 || threads > 256 || threads % 64 || !j.lookback || j.words < 1 || j.words > 4 ||
      j.dense.tile == 0 || j.stage == 0)
    return hipErrorInvalidValue;
  const uint32_t lds = jagged_lds_bytes(j);
  const uint64_t tiles = (j.dense.n + j.dense.tile - 1) / j.dense.tile;
  if (tiles > 0x7fffffffull) return hipErrorInvalidValue;
  const uint64_t grid = tiles ? tiles : 1;
  switch (j.words) {
    case 1: hipLaunchKernelGGL(jagged_kernel<1>, dim3((uint32_t)grid), dim3(threads), lds, s, j); break;
    case 2: hipLaunchKernelGGL(jagged_kernel<2>, dim3((uint32_t)grid), dim3(threads), lds, s, j); break;
    case 3: hipLaunchKernelGGL(jagged_kernel<3>, dim3((uint32_t)grid), dim3(threads), lds, s, j); break;
    default: hipLaunchKernelGGL(jagged_kernel<4>, dim3((uint32_t)grid), dim3(threads), lds, s, j); break;
  }
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, uint64_t bytes, hipStream_t s) {
  if (!bytes) return hipSuccess;
  // four work-groups per compute unit, no more than one vector per thread
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
      hipSuccess || cus <= 0)
    cus = 256;
  const uint64_t want = (bytes + 256 * 16 - 1) / (256 * 16);
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, 4ull * (uint32_t)cus));
  hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, s, reinterpret_cast<uint8_t*>(dst),
                     reinterpret_cast<const uint8_t*>(src), bytes);
  return hipGetLastError();
}

hipError_t launch_move(const MoveDesc& d, uint64_t grid_objects, hipStream_t s) {
  if (!grid_objects) return hipSuccess;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((grid_objects + 255) / 256, 4096);
  hipLaunchKernelGGL(move_kernel, dim3(grid), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_select(const SelectDesc& d, hipStream_t s) {
  const uint64_t tiles = (d.n + kSelectTile - 1) / kSelectTile;
  if (tiles > 0x7fffffffull) return hipErrorInvalidValue;
  if (tiles) hipLaunchKernelGGL(select_count_kernel, dim3((uint32_t)tiles), dim3(256), 0, s, d);
  hipLaunchKernelGGL(select_scan_kernel, dim3(1), dim3(1024), 0, s, d);
  if (tiles) hipLaunchKernelGGL(select_map_kernel, dim3((uint32_t)tiles), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_select_members(const SelectDesc& d, hipStream_t s) {
  const uint64_t tiles = std::max<uint64_t>(1, (d.n + kSelectTile - 1) / kSelectTile);
  hipLaunchKernelGGL(select_lens_kernel, dim3((uint32_t)tiles), dim3(256), 0, s, d);
  hipLaunchKernelGGL(select_lens_scan_kernel, dim3(1), dim3(1024), 0, s, d);
  hipLaunchKernelGGL(select_offsets_kernel, dim3((uint32_t)tiles), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_member_move(const MemberMoveDesc& d, hipStream_t s) {
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((d.n_max + 3) / 4, 4096));
  hipLaunchKernelGGL(member_move_kernel, dim3(grid), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_append(const AppendDesc& d, hipStream_t s) {
  hipLaunchKernelGGL(append_kernel, dim3(1024), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_zero_bytes(void* p, uint64_t bytes, hipStream_t s) {
  if (!bytes) return hipSuccess;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((bytes + 255) / 256, 2048);
  hipLaunchKernelGGL(zero_bytes_kernel, dim3(grid), dim3(256), 0, s, reinterpret_cast<uint8_t*>(p), bytes);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, uint64_t bytes, hipStream_t s) {
  if (((uintptr_t)p & 3) || (bytes & 3)) return hipErrorInvalidValue;
  const uint64_t words = bytes / 4;
  if (!words) return hipSuccess;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((words + 255) / 256, 1024);
  hipLaunchKernelGGL(zero_kernel, dim3(grid), dim3(256), 0, s, reinterpret_cast<uint32_t*>(p), words);
  return hipGetLastError();
}

hipError_t launch_take_status(uint32_t* status, uint32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(take_status_kernel, dim3(1), dim3(1), 0, s, status, out);
  return hipGetLastError();
}

hipError_t status_words(uint32_t** out) {
  return hipGetSymbolAddress(reinterpret_cast<void**>(out), HIP_SYMBOL(g_status_words));
}

}  // namespace rl
