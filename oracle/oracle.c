/*
 * CPU oracle for schema-driven layout conversion.  TEST INFRASTRUCTURE ONLY:
 * it is used by the tests, by the smoke check and by the benchmark's CPU
 * baseline, never by the library.
 *
 * It is the plain definition of the operation, written for a reader to check
 * by eye: the default transfer between two layouts copies every property of
 * every object, one value at a time (Sec. VII-B, the default transfers).
 * Sub-groups and array properties are flattened to separate leaf values
 * (Sec. VI); a jagged vector property is a per-object list whose sizes are
 * kept as a prefix sum in a collection-wide property (Sec. VI).
 *
 * Values are moved as bytes (memcpy), never through a floating-point
 * register, so every bit pattern (signalling NaNs, negative zero) survives a
 * copy.  The only arithmetic is the change of precision of a floating-point
 * leaf: double -> float by the C cast (IEEE round to nearest, ties to even,
 * under the default rounding mode, which is asserted) and float -> double
 * (exact).
 *
 * Build: gcc -O2 -std=c11 -shared -fPIC (no -ffast-math, no intrinsics).
 */
#include <fenv.h>
#include <stdint.h>
#include <string.h>

enum { T_U8, T_I8, T_U16, T_I16, T_U32, T_I32, T_U64, T_I64, T_F32, T_F64 };
enum { ST_OK = 0, ST_ALIGN = 2, ST_CAPACITY = 4, ST_OVERFLOW = 5,
       ST_UNSUPPORTED = 8, ST_BOUNDS = 11 };
enum { K_AOS = 0, K_SOA = 1, K_AOSOA = 2, K_STRIDED = 3 };

static uint64_t type_size(int32_t t) {
  switch (t) {
    case T_U8: case T_I8: return 1;
    case T_U16: case T_I16: return 2;
    case T_U32: case T_I32: case T_F32: return 4;
    default: return 8;
  }
}

/* ---- per-object leaves ------------------------------------------------ */

typedef struct {
  int32_t kind;                 /* K_AOS, K_SOA, K_AOSOA or K_STRIDED */
  uint64_t stride;              /* AoS: bytes per record */
  uint64_t width;               /* AoSoA: objects per block (W) */
  uint64_t obj_bytes;           /* AoSoA: sum of the leaf sizes (B) */
  const uint64_t* offset;       /* AoS: offset of leaf c in a record;
                                   AoSoA: sum of the sizes of leaves < c;
                                   strided: bytes from one element of leaf c
                                   to the next */
  const int32_t* type;          /* storage type of each leaf */
  unsigned char* const* base;   /* AoS/AoSoA: base[0]; SoA, strided: base[c] */
  const uint64_t* index;        /* strided: NULL (object i is element i) or
                                   the element of each object */
  uint64_t elements;            /* strided with an index: elements each leaf
                                   holds (an index must be below it) */
} or_objects;

/* Element that object i of a strided layout maps to (Sec. VII-B: a layout's
   arrays need only map an index to a value, not be contiguous). */
static uint64_t element_of(const or_objects* L, uint64_t i) {
  return L->index ? L->index[i] : i;
}

/* Whether object i has an address: always, except in an indexed strided
   layout whose index points past its elements. */
static int object_in_range(const or_objects* L, uint64_t i) {
  return L->kind != K_STRIDED || !L->index || L->index[i] < L->elements;
}

/* Address of leaf c of object i. */
static unsigned char* leaf_addr(const or_objects* L, uint32_t c, uint64_t i) {
  uint64_t size = type_size(L->type[c]);
  if (L->kind == K_STRIDED)
    return L->base[c] + element_of(L, i) * L->offset[c];
  if (L->kind == K_AOS)
    return L->base[0] + i * L->stride + L->offset[c];
  if (L->kind == K_SOA)
    return L->base[c] + i * size;
  /* AoSoA: block i/W holds W objects; inside it every leaf is a run of W
     values, the runs following each other in leaf order. */
  {
    uint64_t block = i / L->width, lane = i % L->width;
    return L->base[0] + block * L->width * L->obj_bytes
           + L->width * L->offset[c] + lane * size;
  }
}

/* A NaN keeps its sign and the leading bits of its payload through a change
   of precision and comes out quiet (the quiet bit is the payload's leading
   bit in both formats).  Built from the bit fields, so the result does not
   depend on how the host's conversion instructions treat NaNs. */
static uint32_t nan_to_f32(uint64_t b) {
  return (uint32_t)((b >> 63) << 31) | 0x7FC00000u
         | (uint32_t)((b & 0x000FFFFFFFFFFFFFull) >> 29);
}

static uint64_t nan_to_f64(uint32_t b) {
  return ((uint64_t)(b >> 31) << 63) | 0x7FF8000000000000ull
         | ((uint64_t)(b & 0x007FFFFFu) << 29);
}

/* One value: copy, narrow (f64 -> f32) or widen (f32 -> f64). */
static int move_value(int32_t st, const unsigned char* s, int32_t dt, unsigned char* d) {
  if (st == dt) {
    memcpy(d, s, type_size(st));
    return ST_OK;
  }
  if (st == T_F64 && dt == T_F32) {
    double x; float y;
    memcpy(&x, s, 8);
    if (x != x) {
      uint64_t b; uint32_t r;
      memcpy(&b, s, 8);
      r = nan_to_f32(b);
      memcpy(d, &r, 4);
      return ST_OK;
    }
    y = (float)x;
    memcpy(d, &y, 4);
    return ST_OK;
  }
  if (st == T_F32 && dt == T_F64) {
    float x; double y;
    memcpy(&x, s, 4);
    if (x != x) {
      uint32_t b; uint64_t r;
      memcpy(&b, s, 4);
      r = nan_to_f64(b);
      memcpy(d, &r, 8);
      return ST_OK;
    }
    y = (double)x;
    memcpy(d, &y, 8);
    return ST_OK;
  }
  return ST_UNSUPPORTED;
}

int or_rounding_is_nearest(void) { return fegetround() == FE_TONEAREST; }

/* For every object in order, for every leaf in schema order, move the value.
   The destination is expected zero-filled by the caller, so padding bytes
   and the unused slots of a last partial AoSoA block stay zero.
   or_convert_objects_range does objects i0 .. i1-1 only; contiguous ranges
   on several threads (for timing on all host cores) give the same bytes,
   since every object's values land at addresses of that object alone. */
int or_convert_objects_range(const or_objects* src, const or_objects* dst,
                             uint32_t n_leaves, uint64_t i0, uint64_t i1) {
  if (!or_rounding_is_nearest()) return ST_UNSUPPORTED;
  for (uint64_t i = i0; i < i1; ++i) {
    if (!object_in_range(src, i) || !object_in_range(dst, i)) return ST_BOUNDS;
    for (uint32_t c = 0; c < n_leaves; ++c) {
      int st = move_value(src->type[c], leaf_addr(src, c, i),
                          dst->type[c], leaf_addr(dst, c, i));
      if (st != ST_OK) return st;
    }
  }
  return ST_OK;
}

int or_convert_objects(const or_objects* src, const or_objects* dst,
                       uint32_t n_leaves, uint64_t n) {
  return or_convert_objects_range(src, dst, n_leaves, 0, n);
}

/* ---- jagged groups ---------------------------------------------------- */

typedef struct {
  int32_t form;                 /* 0: records carry (ptr, len) + a member pool;
                                   1: offsets column + one column per member leaf */
  uint32_t n_members;           /* member leaves of the group */
  const int32_t* type;          /* storage type of each member leaf */
  uint64_t capacity;            /* members the member storage can hold */
  /* form 0 */
  unsigned char* records;       /* the object records (AoS) */
  uint64_t rec_stride;          /* bytes per object record */
  uint64_t ptr_off, len_off;    /* u64 byte offset into pool, u32 count */
  unsigned char* pool;          /* member records */
  uint64_t mstride;             /* bytes per member record */
  uint64_t malign;              /* alignment a member record needs */
  const uint64_t* moff;         /* offset of each member leaf in a member record */
  /* form 1 */
  unsigned char* offsets;       /* n + 1 entries of off_type */
  int32_t off_type;             /* T_U32, T_I32 or T_U64 */
  unsigned char* const* mcol;   /* one column per member leaf */
} or_group;

static uint64_t load_uint(const unsigned char* p, int32_t t) {
  if (t == T_U64) { uint64_t v; memcpy(&v, p, 8); return v; }
  if (t == T_I32) { int32_t v; memcpy(&v, p, 4); return (uint64_t)(int64_t)v; }
  { uint32_t v; memcpy(&v, p, 4); return v; }
}

static void store_uint(unsigned char* p, int32_t t, uint64_t v) {
  if (t == T_U64) { memcpy(p, &v, 8); return; }
  if (t == T_I32) { int32_t w = (int32_t)v; memcpy(p, &w, 4); return; }
  { uint32_t w = (uint32_t)v; memcpy(p, &w, 4); }
}

static uint64_t offset_type_max(int32_t t) {
  if (t == T_U64) return UINT64_MAX;
  if (t == T_I32) return (uint64_t)INT32_MAX;
  return (uint64_t)UINT32_MAX;
}

/* Number of members of object i in the source group. */
static uint64_t src_length(const or_group* g, uint64_t i) {
  if (g->form == 0) {
    uint32_t len;
    memcpy(&len, g->records + i * g->rec_stride + g->len_off, 4);
    return len;
  }
  return load_uint(g->offsets + (i + 1) * type_size(g->off_type), g->off_type)
       - load_uint(g->offsets + i * type_size(g->off_type), g->off_type);
}

/* Index (into member storage) of the first member of object i. */
static uint64_t src_first(const or_group* g, uint64_t i) {
  return load_uint(g->offsets + i * type_size(g->off_type), g->off_type);
}

static unsigned char* member_addr_ptr(const or_group* g, uint64_t byte_ptr,
                                      uint64_t j, uint32_t m) {
  return g->pool + byte_ptr + j * g->mstride + g->moff[m];
}

/*
 * Convert the members of one jagged group for objects 0..n-1.
 * 1. the lengths are read from the source and their exclusive prefix sum is
 *    written to the destination (offsets column, or (ptr, len) records with
 *    ptr = first member index times the member stride: members packed in
 *    object order with no gaps);
 * 2. every member j of every object i is moved leaf by leaf.
 * The status reports, in this order of precedence: a total beyond the
 * destination offset type, a total beyond the destination capacity, a
 * source member block outside the source pool (or misaligned).
 */
int or_convert_group(const or_group* src, const or_group* dst, uint64_t n,
                     uint64_t* total_out) {
  uint64_t run = 0;
  int overflow = 0, bounds = 0;
  uint64_t limit = dst->form == 1 ? offset_type_max(dst->off_type) : UINT64_MAX;
  if (!or_rounding_is_nearest()) return ST_UNSUPPORTED;
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t len = src_length(src, i);
    if (dst->form == 1) store_uint(dst->offsets + i * type_size(dst->off_type),
                                   dst->off_type, run);
    if (run + len < run || run + len > limit) overflow = 1;
    run += len;
  }
  if (dst->form == 1) store_uint(dst->offsets + n * type_size(dst->off_type),
                                 dst->off_type, run);
  if (total_out) *total_out = run;
  if (overflow) return ST_OVERFLOW;
  if (run > dst->capacity) return ST_CAPACITY;

  /* source bounds: every member block must lie inside the pool / columns */
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t len = src_length(src, i);
    if (src->form == 0) {
      uint64_t ptr;
      memcpy(&ptr, src->records + i * src->rec_stride + src->ptr_off, 8);
      if (ptr % src->malign != 0) { bounds = 1; continue; }
      if (ptr > src->capacity * src->mstride ||
          len > (src->capacity * src->mstride - ptr) / src->mstride) bounds = 1;
    } else {
      uint64_t first = src_first(src, i);
      if (first > src->capacity || len > src->capacity - first) bounds = 1;
    }
  }
  if (bounds) return ST_BOUNDS;

  run = 0;
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t len = src_length(src, i);
    uint64_t sptr = 0, sfirst = 0;
    if (src->form == 0) memcpy(&sptr, src->records + i * src->rec_stride + src->ptr_off, 8);
    else sfirst = src_first(src, i);
    if (dst->form == 0) {
      uint64_t dptr = run * dst->mstride;
      uint32_t dlen = (uint32_t)len;
      memcpy(dst->records + i * dst->rec_stride + dst->ptr_off, &dptr, 8);
      memcpy(dst->records + i * dst->rec_stride + dst->len_off, &dlen, 4);
    }
    for (uint64_t j = 0; j < len; ++j)
      for (uint32_t m = 0; m < src->n_members; ++m) {
        const unsigned char* s = src->form == 0
            ? member_addr_ptr(src, sptr, j, m)
            : src->mcol[m] + (sfirst + j) * type_size(src->type[m]);
        unsigned char* d = dst->form == 0
            ? dst->pool + (run + j) * dst->mstride + dst->moff[m]
            : dst->mcol[m] + (run + j) * type_size(dst->type[m]);
        int st = move_value(src->type[m], s, dst->type[m], d);
        if (st != ST_OK) return st;
      }
    run += len;
  }
  return ST_OK;
}

/* Exclusive prefix sum of n lengths into n + 1 offsets (a standalone form of
   step 1 above, on a plain lengths array).  Returns ST_OVERFLOW when the
   total does not fit the offset type. */
int or_exclusive_scan(const uint32_t* lengths, uint64_t n, unsigned char* offsets,
                      int32_t off_type, uint64_t* total_out) {
  uint64_t run = 0, limit = offset_type_max(off_type);
  int overflow = 0;
  for (uint64_t i = 0; i < n; ++i) {
    store_uint(offsets + i * type_size(off_type), off_type, run);
    if (run + lengths[i] > limit) overflow = 1;
    run += lengths[i];
  }
  store_uint(offsets + n * type_size(off_type), off_type, run);
  if (total_out) *total_out = run;
  return overflow ? ST_OVERFLOW : ST_OK;
}

/* ---- gathers: insertion, deletion and compaction ------------------------- */

/*
 * Insertion and deletion on the arrays of a collection (Sec. VII-B) and the
 * compaction of a filtered collection all give a collection whose objects
 * are existing objects in a chosen order.  The plain definition: a gather.
 * Destination object k0 + k takes every per-object value of source object
 * idx[k], for k = 0 .. m-1 (moved as in or_convert_objects).
 */
int or_gather_objects(const or_objects* src, const or_objects* dst, uint32_t n_leaves,
                      const uint64_t* idx, uint64_t m, uint64_t k0) {
  if (!or_rounding_is_nearest()) return ST_UNSUPPORTED;
  for (uint64_t k = 0; k < m; ++k) {
    if (!object_in_range(src, idx[k]) || !object_in_range(dst, k0 + k)) return ST_BOUNDS;
    for (uint32_t c = 0; c < n_leaves; ++c) {
      int st = move_value(src->type[c], leaf_addr(src, c, idx[k]),
                          dst->type[c], leaf_addr(dst, c, k0 + k));
      if (st != ST_OK) return st;
    }
  }
  return ST_OK;
}

/*
 * The members of one jagged group in a gather: destination object k0 + k
 * receives the members of source object idx[k], placed one object after
 * the other from destination member `base` on.  The destination's offsets
 * entries k0 .. k0 + m are written (entry k0 = base), or its records'
 * (ptr, len) pairs with ptr = member index times the member stride.  The
 * status reports, in this order of precedence: an end beyond the offset
 * type, an end beyond the destination capacity, a gathered source member
 * block outside its storage (or misaligned).  *end_out receives the member
 * index after the last one placed.
 */
int or_gather_group(const or_group* src, const or_group* dst, const uint64_t* idx,
                    uint64_t m, uint64_t k0, uint64_t base, uint64_t* end_out) {
  uint64_t run = base;
  int overflow = 0, bounds = 0;
  uint64_t limit = dst->form == 1 ? offset_type_max(dst->off_type) : UINT64_MAX;
  if (!or_rounding_is_nearest()) return ST_UNSUPPORTED;
  for (uint64_t k = 0; k < m; ++k) {
    uint64_t len = src_length(src, idx[k]);
    if (dst->form == 1) store_uint(dst->offsets + (k0 + k) * type_size(dst->off_type),
                                   dst->off_type, run);
    if (run + len < run || run + len > limit) overflow = 1;
    run += len;
  }
  if (dst->form == 1) store_uint(dst->offsets + (k0 + m) * type_size(dst->off_type),
                                 dst->off_type, run);
  if (end_out) *end_out = run;
  if (overflow || run > limit) return ST_OVERFLOW;
  if (run > dst->capacity) return ST_CAPACITY;

  for (uint64_t k = 0; k < m; ++k) {
    uint64_t i = idx[k], len = src_length(src, i);
    if (src->form == 0) {
      uint64_t ptr;
      memcpy(&ptr, src->records + i * src->rec_stride + src->ptr_off, 8);
      if (ptr % src->malign != 0) { bounds = 1; continue; }
      if (ptr > src->capacity * src->mstride ||
          len > (src->capacity * src->mstride - ptr) / src->mstride) bounds = 1;
    } else {
      uint64_t first = src_first(src, i);
      if (first > src->capacity || len > src->capacity - first) bounds = 1;
    }
  }
  if (bounds) return ST_BOUNDS;

  run = base;
  for (uint64_t k = 0; k < m; ++k) {
    uint64_t i = idx[k], len = src_length(src, i);
    uint64_t sptr = 0, sfirst = 0;
    if (src->form == 0) memcpy(&sptr, src->records + i * src->rec_stride + src->ptr_off, 8);
    else sfirst = src_first(src, i);
    if (dst->form == 0) {
      uint64_t dptr = run * dst->mstride;
      uint32_t dlen = (uint32_t)len;
      memcpy(dst->records + (k0 + k) * dst->rec_stride + dst->ptr_off, &dptr, 8);
      memcpy(dst->records + (k0 + k) * dst->rec_stride + dst->len_off, &dlen, 4);
    }
    for (uint64_t j = 0; j < len; ++j)
      for (uint32_t mm = 0; mm < src->n_members; ++mm) {
        const unsigned char* s = src->form == 0
            ? member_addr_ptr(src, sptr, j, mm)
            : src->mcol[mm] + (sfirst + j) * type_size(src->type[mm]);
        unsigned char* d = dst->form == 0
            ? dst->pool + (run + j) * dst->mstride + dst->moff[mm]
            : dst->mcol[mm] + (run + j) * type_size(dst->type[mm]);
        int st = move_value(src->type[mm], s, dst->type[mm], d);
        if (st != ST_OK) return st;
      }
    run += len;
  }
  return ST_OK;
}
