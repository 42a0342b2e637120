/*
 * relayout: schema-driven conversion of object collections between memory
 * layouts on AMD Instinct MI355X (gfx950), and the host <-> device transfers
 * that carry those conversions.
 *
 * The operation is the data movement behind the layout abstraction of the
 * Marionette paper (arXiv 2511.04853): a collection is described once as a
 * list of properties (Sec. VI), its storage is chosen separately as a layout
 * (Sec. V and VII-B), and transfers between layouts copy every property of
 * every object (Sec. VII-B, the default transfers), possibly across memory
 * contexts (Sec. VII-A).
 *
 * Conventions for every entry point:
 *  - No call throws; each returns an rl_status.  On a status other than
 *    RL_OK, rl_last_error() gives a message (thread-local, valid until the
 *    next call on that thread).
 *  - Validation failures found on the host return at once and enqueue no
 *    work.  Failures that only the device can see (a member total beyond a
 *    capacity, an offset-type overflow, a member block outside its pool)
 *    are recorded in a status word of the stream the work was enqueued on
 *    and returned by rl_sync() on that stream.
 *  - The caller owns every data buffer; the library never frees them.
 *    Handles (schemas, layouts, batches, servers) are owned by the library
 *    until their destroy call; schemas and layouts are immutable and may be
 *    shared between threads.
 *  - Streams are borrowed hipStream_t values passed as void*; NULL is the
 *    null stream.  Work is asynchronous on that stream: buffers must stay
 *    alive and unmodified until the stream has been synchronised.
 *  - Device pointers must point to memory of the current HIP device.
 */
#ifndef RELAYOUT_H
#define RELAYOUT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rl_status {
  RL_OK = 0,
  RL_EINVAL = 1,        /* malformed argument */
  RL_EALIGN = 2,        /* a buffer not aligned as the layout needs */
  RL_EOVERLAP = 3,      /* source and destination buffers overlap */
  RL_ECAPACITY = 4,     /* members do not fit the destination capacity */
  RL_EOVERFLOW = 5,     /* a member total does not fit the offset type */
  RL_ENOMEM = 6,        /* an allocation of the library failed */
  RL_EBUDGET = 7,       /* a request larger than the serving budget */
  RL_EUNSUPPORTED = 8,  /* a valid request this library does not perform */
  RL_EHIP = 9,          /* a HIP runtime call failed (message has its text) */
  RL_EBUSY = 10,        /* the object is in use (e.g. ticket not complete) */
  RL_EBOUNDS = 11,      /* a source member block outside its pool/columns, or misaligned */
  RL_ELIMIT = 12,       /* a request beyond a fixed size limit of the library */
  RL_ECANCELED = 13     /* the event was cancelled before it was admitted */
} rl_status;

/* Scalar types of a property (Sec. VI: per-item properties hold one native
   type).  The numeric values are part of the ABI. */
typedef enum rl_type {
  RL_U8 = 0, RL_I8 = 1, RL_U16 = 2, RL_I16 = 3, RL_U32 = 4, RL_I32 = 5,
  RL_U64 = 6, RL_I64 = 7, RL_F32 = 8, RL_F64 = 9
} rl_type;

/* ------------------------------------------------------------------ schema */

/* One property of a schema (Sec. VI).
 *  - extent == 1: per-item property, one leaf value per object;
 *    extent  > 1: array property, E leaf values kept as E separate leaves.
 *  - group == -1: the value belongs to the object;
 *    group == g >= 0: the field is a member property of jagged vector group
 *    g (each object holds a variable number of members).
 *  - subgroup == -1: top level; subgroup == s >= 0: the field belongs to
 *    sub-group s, whose fields must be consecutive.  Sub-group members are
 *    separate leaves (kept in separate columns in SoA layouts) and form a
 *    nested struct in natural record layouts.
 *  - name: informational, may be NULL; copied. */
typedef struct rl_field {
  const char* name;
  rl_type type;
  uint32_t extent;
  int32_t group;
  int32_t subgroup;
} rl_field;

/* A jagged vector group (Sec. VI): the type of the prefix sum of member
   counts, which may be narrower than the object index type.  One of RL_U32,
   RL_I32, RL_U64. */
typedef struct rl_jagged {
  rl_type offset_type;
} rl_jagged;

typedef struct rl_schema rl_schema;

/* Register a schema.  Fields are flattened in declaration order into
 * per-object leaves (extent E gives E consecutive leaves) and, per jagged
 * group, member leaves.  Limits: at most 64 per-object leaves, 8 member
 * leaves per group, 4 groups, extent <= 64.
 * Errors: RL_EINVAL (bad type/extent/group index, non-consecutive sub-group,
 * a member field inside a sub-group, a group with no member field, an
 * offset type other than U32/I32/U64, a limit exceeded). */
rl_status rl_schema_create(const rl_field* fields, uint32_t n_fields,
                           const rl_jagged* groups, uint32_t n_groups,
                           rl_schema** out);
void rl_schema_destroy(rl_schema* schema);

/* A node of a property tree (Sec. VI: the kinds of property), for schemas
 * whose properties nest: arrays holding several properties, sub-groups or
 * jagged vectors inside arrays, arrays and sub-groups inside jagged vectors.
 *  - RL_PROP_ITEM: a per-item property holding one value of `type`
 *    (n_children 0).
 *  - RL_PROP_ARRAY: an array property of `extent` elements (1..64), each
 *    element holding the n_children child properties.
 *  - RL_PROP_SUBGROUP: the n_children child properties as a sub-object.
 *  - RL_PROP_JAGGED: a jagged vector property: each object holds a
 *    variable number of members, each member holding the n_children child
 *    properties; `type` is the type of the prefix sum of member counts
 *    (RL_U32, RL_I32 or RL_U64).  A jagged vector inside another is not
 *    supported.
 * Nodes are listed in pre-order: a node is followed by its children's
 * subtrees; the top-level properties follow each other.  name: may be
 * NULL; copied. */
typedef enum rl_prop_kind {
  RL_PROP_ITEM = 0,
  RL_PROP_ARRAY = 1,
  RL_PROP_SUBGROUP = 2,
  RL_PROP_JAGGED = 3
} rl_prop_kind;

typedef struct rl_prop {
  rl_prop_kind kind;
  const char* name;
  rl_type type;
  uint32_t extent;
  uint32_t n_children;
} rl_prop;

/* Register a schema from a property tree.  Flattening walks the tree in
 * pre-order, each array element in turn (element-major): every item
 * outside a jagged vector is a per-object leaf and a record slot; every
 * jagged vector reached (each element of an array holding one is its own)
 * is the next jagged group, with a (ptr, len) slot pair where it is
 * reached and its items as the group's member leaves.  The natural record
 * (RL_AOS without explicit offsets) follows C rules: a sub-group is a
 * nested struct; an array element is a struct of the element's properties
 * (each element aligned to its largest member, its size rounded up to
 * it); a jagged vector's pair is two members (u64 ptr, u32 len) of the
 * enclosing struct; member records are the struct of a member's
 * properties.  rl_schema_create's flat fields are the special case of
 * extents over one item, one level of sub-groups, and jagged groups of
 * items.  Limits as rl_schema_create.
 * Errors: RL_EINVAL (bad kind, type, extent or child count, children past
 * the end, an empty array, sub-group or jagged vector, a limit exceeded);
 * RL_EUNSUPPORTED (a jagged vector inside another). */
rl_status rl_schema_create_tree(const rl_prop* props, uint32_t n_props, rl_schema** out);

/* Leaf counts of a schema.  Any out pointer may be NULL. */
rl_status rl_schema_info(const rl_schema* schema, uint32_t* n_leaves,
                         uint32_t* n_groups, uint32_t* n_slots);

/* ------------------------------------------------------------------ layouts */

typedef enum rl_kind {
  RL_AOS = 0,    /* records: object i at i * stride, leaf at a byte offset;
                    each jagged group as a (u64 byte offset into a member
                    pool, u32 member count) pair in the record, the pool
                    holding member records */
  RL_SOA = 1,    /* one column per leaf; each jagged group as an offsets
                    column (n + 1 entries, exclusive prefix sum) and one
                    column per member leaf */
  RL_AOSOA = 2,  /* blocks of W objects; inside a block each leaf is a run
                    of W values, runs in leaf order; the block stride is
                    W * (sum of leaf sizes); the unused slots of a last
                    partial block are zero.  Jagged groups as in RL_SOA. */
  RL_STRIDED = 3 /* a user's map from object index to address (Sec. VII-B:
                    a layout's arrays need not be contiguous, only map an
                    index to a value): leaf c of object i is element e of
                    buffer c, at byte e * leaf_strides[c], with e = i, or
                    e = index[i] read from a u64 index table (the buffer
                    after the leaves) when the layout is indexed.  Several
                    leaves may share memory (the fields of an existing
                    record array: buffer c at the field's offset, every
                    stride the record size); the caller keeps the elements
                    of different leaves, and the index table, apart.  Bytes
                    no object addresses are never written.  Per-object
                    leaves only (no jagged groups). */
} rl_kind;

typedef enum rl_space {
  RL_SPACE_DEVICE = 0,       /* device memory of the current device */
  RL_SPACE_HOST = 1,         /* pageable host memory */
  RL_SPACE_HOST_PINNED = 2   /* page-locked host memory (hipHostMalloc) */
} rl_space;

/* Description of a layout (Sec. VII-B: the layout decides where each
 * property's values live; Sec. VII-A: its memory context).
 *  - block_width: RL_AOSOA only, W >= 1.
 *  - record_stride / slot_offsets: RL_AOS only.  A record has n_slots
 *    slots: every per-object leaf in order and, where a jagged group's
 *    first field is declared, its (ptr u64, len u32) pair.  NULL / 0 select
 *    C natural alignment (scalars at multiples of their size, sub-groups as
 *    nested structs aligned to their largest member, stride rounded up to
 *    the largest alignment).  Explicit offsets describe a pre-existing
 *    struct; slots may not overlap and must fit the stride.
 *  - storage_type: per per-object leaf, the type stored in this layout;
 *    NULL = the schema's type.  RL_F32 for an RL_F64 leaf stores it
 *    narrowed (round to nearest even; overflow to infinity; subnormals
 *    kept); RL_F64 for an RL_F32 leaf widens it (exact).  No other change.
 *  - member pools (RL_AOS with jagged groups) use natural alignment of the
 *    group's member leaves.
 *  - leaf_strides / indexed: RL_STRIDED only.  leaf_strides: per per-object
 *    leaf, the bytes from one element to the next, a non-zero multiple of
 *    the leaf's storage size below 2^31; NULL = the storage size (packed
 *    columns).  indexed != 0: objects reach their elements through the
 *    index table; a view of capacity C then has C elements per leaf and C
 *    index entries, and an index >= C is a device error (RL_EBOUNDS, the
 *    object is skipped).  Without an index table object i is element i. */
typedef struct rl_layout_desc {
  rl_kind kind;
  rl_space space;
  uint32_t block_width;
  uint64_t record_stride;
  const uint64_t* slot_offsets;
  const rl_type* storage_type;
  const uint64_t* leaf_strides;
  uint32_t indexed;
} rl_layout_desc;

typedef struct rl_layout rl_layout;

/* Errors: RL_EINVAL (bad kind/space, W == 0 for AoSoA, overlapping or
 * out-of-stride slots, an unsupported storage change, a stride over 2^31,
 * a leaf stride that is zero or not a multiple of the leaf's size);
 * RL_EUNSUPPORTED (RL_STRIDED for a schema with jagged groups). */
rl_status rl_layout_create(const rl_schema* schema, const rl_layout_desc* desc,
                           rl_layout** out);
void rl_layout_destroy(rl_layout* layout);

/* Buffers of a layout holding n_objects objects and n_members[g] members of
 * each jagged group (n_members may be NULL without groups), in order:
 *   RL_AOS:   records, then one member pool per group;
 *   RL_SOA:   one column per per-object leaf, then per group the offsets
 *             column and one column per member leaf;
 *   RL_AOSOA: the blocks, then per group as RL_SOA;
 *   RL_STRIDED: one buffer per leaf, reaching the end of its last element
 *             ((n_objects - 1) * stride + size bytes), then, when indexed,
 *             the index table (8 * n_objects bytes).
 * *n_buffers receives the count; bytes (may be NULL) receives each buffer's
 * byte size and must have room for rl_layout_info's max_buffers entries. */
rl_status rl_layout_buffers(const rl_layout* layout, uint64_t n_objects,
                            const uint64_t* n_members, uint32_t* n_buffers,
                            uint64_t* bytes);

/* The resolved record layout of an RL_AOS layout: slot offsets (room for
 * n_slots entries, may be NULL) and stride; and the buffer count. */
rl_status rl_layout_info(const rl_layout* layout, uint64_t* slot_offsets,
                         uint64_t* record_stride, uint32_t* max_buffers);

/* ------------------------------------------------------------------ views */

/* A collection stored in a layout: the buffers (see rl_layout_buffers) able
 * to hold `capacity` objects and member_capacity[g] members per group
 * (NULL without groups; for an RL_AOS pool, in member records). */
typedef struct rl_view {
  const rl_layout* layout;
  uint64_t capacity;
  const uint64_t* member_capacity;
  void* const* buffers;
} rl_view;

/* ------------------------------------------------------------------ conversion */

/* Convert objects 0..n-1 of src into dst (Sec. VII-B transfers between
 * layouts): every leaf value is copied (or narrowed/widened as the two
 * storage types say); jagged members are moved with their objects, the
 * destination's member storage packed in object order from index 0
 * (offsets rebased to start at 0; record pointers = first member index *
 * member record size).  Padding bytes and unused block slots of dst are
 * zero.  Both views must use device memory; the schemas must be the same
 * object.  Asynchronous on `stream`.
 * Host errors: RL_EINVAL (n over a capacity, mismatched schemas, NULL
 * buffers), RL_EALIGN (a buffer not aligned to its element size, or a
 * record buffer to its largest slot), RL_EOVERLAP (a destination buffer
 * overlapping any source buffer), RL_EUNSUPPORTED (host spaces; AoS -> AoS
 * with jagged groups; unsupported storage change).
 * Device errors (rl_sync): RL_EOVERFLOW, RL_ECAPACITY, RL_EBOUNDS; dst is
 * then unspecified but no memory outside the views is touched.
 * n == 0: RL_OK, nothing enqueued.
 * A strided side (RL_STRIDED) is converted by a general kernel, one thread
 * per object, reading and writing each leaf at its element; the other
 * side may be of any kind.
 * Records with one jagged group of packed 4-byte member words convert in
 * one kernel whose work-groups pass running member totals to each other
 * through a small per-stream device buffer of the library (8 bytes per
 * tile; allocated on the stream's first such call, grown when needed,
 * held until the process ends); callers that cannot allocate use
 * rl_transfer_noalloc.  Under stream capture the multi-kernel path, which
 * needs no such buffer, is taken. */
rl_status rl_convert(const rl_view* src, const rl_view* dst, uint64_t n,
                     void* stream);

/* The offsets step alone (Sec. VI: the prefix sum of the member counts of
 * jagged group `group`): reads the counts of objects 0..n-1 from src
 * (RL_AOS records, or an offsets column) and writes the n + 1 exclusive
 * offsets into dst's offsets column (dst must be RL_SOA or RL_AOSOA).
 * If total_host is not NULL the call synchronises the stream and stores
 * the total there.  Device errors as rl_convert (RL_EOVERFLOW). */
rl_status rl_offsets(const rl_view* src, const rl_view* dst, uint32_t group,
                     uint64_t n, uint64_t* total_host, void* stream);

/* ------------------------------------------------------------------ collections with a memory context */

typedef struct rl_collection rl_collection;

/* A collection owning its buffers in its layout's memory context (Sec.
 * VII-A: every collection has a memory context that says how memory is
 * allocated, deallocated and set): buffers for `capacity` objects and
 * member_capacity[g] members per group (NULL without groups), allocated in
 * the layout's space (device: hipMalloc; pinned host: hipHostMalloc;
 * pageable host: malloc) and zero-filled (device memory by a kernel on
 * `stream`).  The layout must outlive the collection.
 * Errors: RL_EINVAL, RL_ENOMEM (nothing is kept), RL_EUNSUPPORTED (an
 * RL_STRIDED layout: its memory belongs to someone else). */
rl_status rl_collection_create(const rl_layout* layout, uint64_t capacity,
                               const uint64_t* member_capacity, void* stream,
                               rl_collection** out);
/* The collection's view; its pointers stay valid until the next
 * rl_collection_rehome or rl_collection_destroy. */
rl_status rl_collection_view(const rl_collection* c, rl_view* out);
/* Move the collection to another memory context and, optionally, another
 * layout (Sec. VII-A: updating a collection's memory context information
 * allocates with the new information, copies from the old memory and frees
 * it): new buffers for the same capacities in `layout` (same schema, any
 * space and kind), objects 0..n-1 and their members converted into them
 * (rl_convert between device layouts, rl_transfer across host and device,
 * through a temporary device copy between host layouts), then the old
 * buffers freed; the call synchronises `stream`.  On an error the
 * collection keeps its old memory.  Errors: as rl_convert / rl_transfer,
 * RL_EINVAL (another schema, n over the capacity), RL_ENOMEM.  Device
 * errors found by the conversion are returned by rl_sync on `stream`. */
rl_status rl_collection_rehome(rl_collection* c, const rl_layout* layout, uint64_t n,
                               void* stream);
/* Free the collection's buffers (waits for the device first). */
void rl_collection_destroy(rl_collection* c);

/* ------------------------------------------------------------------ user transfers */

/* A user implementation of a transfer between two layouts (Sec. VII-B:
 * transfers may be given more optimal implementations, or read
 * pre-existing structures defined outside the library, through
 * specialisations with a priority that falls back to more general
 * implementations).  Called by rl_convert and rl_transfer, after their
 * argument validation, with the caller's arguments.  Returns RL_OK once it
 * has enqueued the whole transfer on `stream`; RL_EUNSUPPORTED to decline
 * (the next matching specialisation is tried, then the library's own
 * implementation); any other status fails the call with that status.
 * rl_convert and rl_transfer called from inside a user transfer (on the
 * same thread) go straight to the library's own implementation, so a
 * specialisation can wrap the default transfer without recursing. */
typedef rl_status (*rl_transfer_fn)(const rl_view* src, const rl_view* dst,
                                    uint64_t n, void* stream, void* user);

/* Register fn for transfers from layout src to layout dst; either may be
 * NULL (any layout of the other's schema), not both.  Higher priorities
 * are tried first, equal ones in registration order.  *id (may be NULL)
 * receives the handle for rl_unregister_transfer.  The layouts must
 * outlive the registration; registration is thread-safe, and a call in
 * progress keeps using the list it started with.
 * Errors: RL_EINVAL (NULL fn, both layouts NULL, different schemas). */
rl_status rl_register_transfer(const rl_layout* src, const rl_layout* dst,
                               int32_t priority, rl_transfer_fn fn, void* user,
                               uint64_t* id);
/* Errors: RL_EINVAL (unknown id). */
rl_status rl_unregister_transfer(uint64_t id);

/* ------------------------------------------------------------------ insertion, deletion, compaction */

/* Compaction after a filter (Sec. VII-B: operations on every property's
 * array of a collection): dst receives, in order, the objects i < n of src
 * whose keep[i] != 0; every value moves as rl_convert moves it, and each
 * jagged group's members follow their objects, packed from member 0 in
 * dst (offsets rebuilt, or record pointers = first member index * member
 * record size).  keep: n bytes of device memory.  n_kept: NULL, or device
 * memory receiving the kept count (u64).  dst must hold n objects (the
 * count is only known on the device); dst's slots past the kept objects
 * are left zero in AoSoA blocks and record padding.  Any layout kinds on
 * either side (an RL_STRIDED object whose index is past its elements is
 * skipped and reported as RL_EBOUNDS); the schemas must be the same object.
 * Host errors: as rl_convert (RL_EINVAL also for keep == NULL with n > 0).
 * Device errors (rl_sync): RL_EOVERFLOW (member total beyond dst's offset
 * type), RL_ECAPACITY (beyond dst's member capacity: members that do not
 * fit are not written), RL_EBOUNDS (a kept object's member block outside
 * src's storage: its members are not copied).  Uses a per-stream scratch
 * buffer of the library (about 16 bytes per object; allocated on first
 * use, grown when needed, held until the process ends). */
rl_status rl_select(const rl_view* src, const rl_view* dst, uint64_t n,
                    const uint8_t* keep, uint64_t* n_kept, void* stream);

/* Erase objects [at, at + count) of a view holding n objects, in place
 * (Sec. VII-B: the layout holder's erase on every array): objects
 * [at + count, n) move to [at, n - count), as if through a separate buffer;
 * the view then holds n - count objects and the unused slots of its last
 * AoSoA block are zero.  Collections with jagged groups: only the last
 * objects (at + count == n; nothing moves), else RL_EUNSUPPORTED.
 * Errors: RL_EINVAL (range outside n objects), RL_EUNSUPPORTED (an
 * RL_STRIDED view), as rl_convert for the view.
 * AoSoA views move through a per-stream scratch buffer of the library
 * (at most 64 MiB, allocated on first use). */
rl_status rl_erase(const rl_view* view, uint64_t n, uint64_t at, uint64_t count,
                   void* stream);

/* Insert objects 0 .. count-1 of src before object `at` of a view holding
 * n objects, in place (Sec. VII-B: the layout holder's insert; at == n
 * appends): objects [at, n) move to [at + count, n + count) as if through a
 * separate buffer, then src's objects are converted into [at, at + count)
 * (copy / narrowing / widening as the storage types say).  The view's
 * capacity must hold n + count objects; src must not overlap it.  Jagged
 * groups: appends only (at == n), between offsets layouts (SoA / AoSoA on
 * both sides): src's members follow the view's, offsets entries
 * n .. n + count continue from the view's total.
 * Host errors: RL_EINVAL (position or capacity), RL_EUNSUPPORTED (jagged
 * other than an append between offsets layouts; an RL_STRIDED view; src
 * may be strided), as rl_convert otherwise.
 * Device errors (rl_sync, appends): RL_ECAPACITY (members beyond the view's
 * member capacity: nothing appended to that group), RL_EOVERFLOW (total
 * beyond the offset type, or decreasing src offsets), RL_EBOUNDS (src
 * offsets beyond src's member capacity). */
rl_status rl_insert(const rl_view* view, uint64_t n, uint64_t at,
                    const rl_view* src, uint64_t count, void* stream);

/* Options of rl_transfer. */
typedef enum rl_xfer_mode {
  RL_XFER_AUTO = 0,      /* zero-copy for pinned collections, staged for
                            pageable ones */
  RL_XFER_STAGED = 1,    /* DMA copies of the host buffers into a device
                            staging buffer of the library (one per stream,
                            grown on demand, kept until the process ends),
                            conversion from (or into) it, on the caller's
                            stream */
  RL_XFER_ZERO_COPY = 2  /* the conversion kernels read/write the pinned
                            host buffers directly (one pass, no staging) */
} rl_xfer_mode;

typedef struct rl_xfer_opts {
  rl_xfer_mode mode;
} rl_xfer_opts;

/* Convert objects 0..n-1 between a host view and a device view (Sec. VII-A:
 * copies between memory contexts, with extra arguments controlling the
 * copy; Sec. VII-B: copy with conversion).  Exactly one side must be on
 * the host (RL_SPACE_HOST or RL_SPACE_HOST_PINNED).  Results are the same
 * bytes rl_convert would give.  The call returns once the work is
 * enqueued; `stream` is ordered with it: work enqueued earlier on `stream`
 * happens before the transfer, later work after it.  Host buffers must
 * stay alive until then.  opts may be NULL (RL_XFER_AUTO).
 * Zero-copy needs pinned host memory.  Errors as rl_convert;
 * RL_EUNSUPPORTED for an RL_STRIDED side unless a user transfer
 * (rl_register_transfer) takes the pair. */
rl_status rl_transfer(const rl_view* src, const rl_view* dst, uint64_t n,
                      void* stream, const rl_xfer_opts* opts);

/* Copy `bytes` from src, in memory context src_space, to dst, in dst_space
 * (Sec. VII-A: copies between memory contexts, with the variants for
 * partially overlapping arrays that insertion and deletion use).
 *  - device -> device: a copy kernel; the ranges may overlap (the result
 *    is as if the source went through a separate buffer first).  Moves of
 *    overlapping ranges by less than 64 MiB go through a 64 MiB per-stream
 *    scratch buffer of the library (allocated on first use, held until the
 *    process ends), band by band.
 *  - host <-> device: a DMA-engine copy; host memory that is pageable is
 *    copied synchronously by the runtime.
 *  - host -> host: memmove, once the stream has finished its earlier work
 *    (synchronous).
 * Asynchronous on `stream` otherwise.  Errors: RL_EINVAL (bad context,
 * NULL pointer with bytes > 0), RL_ENOMEM (scratch), RL_EHIP.
 * bytes == 0: RL_OK, nothing enqueued. */
rl_status rl_memcopy(void* dst, rl_space dst_space, const void* src,
                     rl_space src_space, uint64_t bytes, void* stream);

/* rl_transfer for callers that cannot allocate memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, results and errors as rl_transfer, but the call makes
 * no device or pinned-memory allocation (no hipMalloc / hipFree): staged
 * transfers stage the host side in a fixed device array of the library
 * (RL_TRANSFER_NOALLOC_LIMIT bytes = 32 MiB; one copy per device, held
 * from library load until the process ends) instead of the library's
 * per-stream staging buffers.  A staged transfer whose host side needs
 * more than the limit (every host buffer rounded up to 256 bytes) returns
 * RL_ELIMIT and enqueues nothing; zero-copy transfers need no staging and
 * have no limit.  Every call on one device shares that device's array:
 * calls whose work overlaps in time (on different streams, or from
 * different threads) race and give unspecified results; calls on one
 * stream are ordered by it.  The array
 * also holds the look-back state of jagged conversions (1 MiB after the
 * staging bytes).  The array keeps the last call's bytes; no
 * result depends on its earlier contents. */
#define RL_TRANSFER_NOALLOC_LIMIT (32ull << 20)
rl_status rl_transfer_noalloc(const rl_view* src, const rl_view* dst, uint64_t n,
                              void* stream, const rl_xfer_opts* opts);

/* Wait for `stream`, then return (and clear) the device status word of
 * that stream: RL_EOVERFLOW, RL_ECAPACITY or RL_EBOUNDS (in that order of
 * precedence) if any conversion, transfer, offsets step or batch enqueued
 * on `stream` since the last rl_sync on it found one, else RL_OK; RL_EHIP
 * if the wait failed.  Each stream has its own word (up to 4,095 streams
 * per device and process; streams beyond those share one word), so work
 * on other streams neither sets nor clears it. */
rl_status rl_sync(void* stream);

/* Message of the last failed call on this thread ("" if none). */
const char* rl_last_error(void);

/* ------------------------------------------------------------------ batches */

typedef struct rl_batch rl_batch;

typedef struct rl_batch_opts {
  int autotune;          /* 1: time candidate tile shapes (and block widths
                            of destinations whose width is 0) and keep the
                            fastest; 0: use the tuning cache or defaults */
  const char* tune_cache;/* JSON file of tuned choices; NULL: $RL_TUNE_CACHE
                            or no cache */
} rl_batch_opts;

/* A batch converts many collections with one launch of a captured HIP graph
 * whose kernels walk a device-resident table of all items.  Items are added
 * with the same arguments as rl_convert and must be device views.  An
 * AoSoA destination layout whose block width is 0 lets the batch choose the
 * width ("auto"); the chosen width is readable with rl_batch_item_width.
 * The items of one launch run concurrently: rl_batch_finalize returns
 * RL_EOVERLAP if a destination of one item overlaps a buffer (source or
 * destination) of another; sources may be shared.  Device-detected errors
 * go to the status word of the stream the batch is launched on.
 * rl_batch_add returns RL_EUNSUPPORTED for an RL_STRIDED side (batches
 * walk their items with the tiled kernels; convert such items with
 * rl_convert). */
rl_status rl_batch_create(const rl_batch_opts* opts, rl_batch** out);
rl_status rl_batch_add(rl_batch* batch, const rl_view* src, const rl_view* dst,
                       uint64_t n);
/* Plan every item, tune if asked, upload the table, capture the graph on
   `stream`.  Items cannot be added afterwards. */
rl_status rl_batch_finalize(rl_batch* batch, void* stream);
rl_status rl_batch_launch(rl_batch* batch, void* stream);
/* Run the same items one rl_convert call at a time (the launch loop the
   batch replaces), for comparison. */
rl_status rl_batch_launch_loop(rl_batch* batch, void* stream);
rl_status rl_batch_item_width(const rl_batch* batch, uint32_t item,
                              uint32_t* block_width);
/* Shape chosen for the batch: objects per tile, threads per block,
   persistent blocks, and whether rl_batch_launch replays the captured graph
   (1) or launches the same kernels directly (0; the autotuner keeps
   whichever it measured faster).  When every dense step sits in a fan-out
   group (rl_batch_info), threads and blocks are those of the fan-out
   launch.  Any out pointer may be NULL. */
rl_status rl_batch_shape(const rl_batch* batch, uint32_t* tile_objects,
                         uint32_t* block_threads, uint32_t* grid_blocks,
                         uint32_t* graph_replay);
/* How the batch's dense steps run, as the autotuner (or the RL_BATCH_*
   environment overrides) left them.  Steps that convert the same source
   view into direct destinations (SoA, AoSoA) may form fan-out groups of up
   to four: one work-group per source tile reads the tile into LDS once and
   a thread group per step stores that step's destination. */
typedef struct rl_batch_info {
  uint32_t double_buffered;   /* 1: dense steps (fan-out groups included) run with two
                                 tile slots per work-group */
  uint32_t fanout_threads;    /* threads per destination in fan-out groups; 0: no fan-out */
  uint32_t fanout_groups;     /* fan-out groups formed */
  uint32_t fanout_steps;      /* dense steps inside them */
  uint32_t dense_steps;       /* dense steps in all */
  uint32_t stream_stores;     /* 1: values written straight to SoA / AoSoA destinations
                                 use non-temporal stores (the tuner's choice) */
  uint32_t reserved[2];
} rl_batch_info;
/* RL_EINVAL for a NULL argument or a batch not finalized. */
rl_status rl_batch_get_info(const rl_batch* batch, rl_batch_info* info);
void rl_batch_destroy(rl_batch* batch);

/* ------------------------------------------------------------------ serving */

typedef struct rl_server rl_server;

typedef struct rl_server_opts {
  uint64_t budget_bytes;   /* device memory for resident results */
  uint32_t max_in_flight;  /* events converting at once (slots) */
  uint32_t n_streams;      /* streams the events are spread over */
} rl_server_opts;

/* One collection of an event: a pinned host source and the device layout
   its result is to have. */
typedef struct rl_event_item {
  rl_view src;
  const rl_layout* dst_layout;
  uint64_t n;
} rl_event_item;

typedef struct rl_event {
  const rl_event_item* items;
  uint32_t n_items;
} rl_event;

typedef struct rl_event_result {
  uint32_t n_items;
  uint64_t latency_ns;                /* submit -> last conversion done */
  uint64_t bytes;                     /* device bytes held */
  void* const* const* buffers;        /* per item: the device buffers */
  const uint64_t* member_capacity;    /* per item and group, flattened */
  rl_status status;                   /* RL_OK, a host error of its enqueue, or
                                         the device status of this event's
                                         conversions alone (RL_EOVERFLOW,
                                         RL_ECAPACITY, RL_EBOUNDS) */
} rl_event_result;

typedef struct rl_server_stats {
  uint64_t completed;
  uint64_t submitted;
  double p50_ms, p99_ms, max_ms;
  double events_per_s;                /* completed / (last done - first submit) */
  uint64_t peak_bytes;                /* largest resident + in-flight bytes */
  uint64_t h2d_bytes;
} rl_server_stats;

/* A serving loop: events are admitted in arrival order while their result
 * bytes (plus, while converting, the device staging of collections that
 * are copied before conversion: pageable ones) fit the budget
 * and a slot is free; admitted events convert concurrently on the server's
 * streams; results stay resident until released.  All of it is carved
 * from one device allocation of budget_bytes made at creation.  The caller
 * keeps each event's host sources alive until its wait returns.
 * max_in_flight: 1..65536; n_streams: 1..64. */
rl_status rl_server_create(const rl_server_opts* opts, rl_server** out);
/* Errors: RL_EBUDGET (the event alone exceeds the budget), RL_EINVAL. */
rl_status rl_server_submit(rl_server* server, const rl_event* event,
                           uint64_t* ticket);
/* Block until the event is done (timeout_ms < 0: forever) and return its
   status (result, may be NULL, receives its buffers).  RL_EBUSY on
   timeout; RL_ECANCELED if the event is cancelled (or the server destroyed)
   while waiting; RL_EINVAL for an unknown ticket (released or cancelled
   before the call).  The result's pointers stay valid until the event is
   released. */
rl_status rl_server_wait(rl_server* server, uint64_t ticket, int64_t timeout_ms,
                         rl_event_result* result);
/* Free a finished event's resident results (RL_EBUSY if it is not done). */
rl_status rl_server_release(rl_server* server, uint64_t ticket);
/* Withdraw an event that is still queued (not yet admitted): it is never
   converted and its ticket is forgotten.  RL_EBUSY once it has been
   admitted (it then runs to completion and is released as usual);
   RL_EINVAL for an unknown ticket.  The head of the queue admits in
   arrival order and waits for budget; cancelling it lets the next one
   through. */
rl_status rl_server_cancel(rl_server* server, uint64_t ticket);
rl_status rl_server_stats_get(rl_server* server, rl_server_stats* stats);
void rl_server_destroy(rl_server* server);

#ifdef __cplusplus
}
#endif

#endif /* RELAYOUT_H */
