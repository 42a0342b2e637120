// Internal declarations shared by the host sources and the HIP kernels of
// librelayout.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/relayout.h"

namespace rl {

constexpr int kMaxLeaves = 64;        // per-object leaves of a schema
constexpr int kMaxMembers = 8;        // member leaves of one jagged group
constexpr int kMaxGroups = 4;
constexpr int kMaxObjBytes = 512;     // sum of leaf sizes on one side
constexpr int kMaxUnits = 256;        // SoA images up to this many bytes per object use the unit table
constexpr int kMaxExtent = 64;
constexpr uint32_t kAutoWidthMax = 128; // "auto" AoSoA widths are 32, 64 or 128
constexpr uint32_t kDenseMaxThreads = 256;  // launch bound of the dense kernels
constexpr uint32_t kStatusSlots = 4096;     // device status words (one per stream)

// Kinds of one side of a dense conversion (match rl_kind).
enum SideKind : uint32_t { KIND_AOS = 0, KIND_SOA = 1, KIND_AOSOA = 2, KIND_STRIDED = 3 };

// Value operations of one leaf.
enum LeafOp : uint8_t {
  OP_COPY = 0,    // same type: size bytes
  OP_NARROW = 1,  // f64 -> f32, round to nearest even
  OP_WIDEN = 2,   // f32 -> f64
  OP_PTR = 3,     // destination record pointer: (off[i] - off[0]) * mstride (u64)
  OP_LEN = 4      // destination record count: off[i+1] - off[i] (u32)
};

// A leaf move as one value (host-computed from op, sizes and alignment).
enum LeafCode : uint8_t {
  CODE_COPY1 = 0, CODE_COPY2 = 1, CODE_COPY4 = 2, CODE_COPY8 = 3,
  CODE_NARROW = 4, CODE_WIDEN = 5,
  CODE_BYTES = 6,   // any copy/narrow/widen at a misaligned image address
  CODE_PTR = 7, CODE_LEN = 8
};

// Device status flags (ORed by kernels, read by rl_sync).
enum StatusFlag : uint32_t {
  ST_FLAG_OVERFLOW = 1u,
  ST_FLAG_CAPACITY = 2u,
  ST_FLAG_BOUNDS = 4u
};

// One leaf of a dense (per-object) conversion.  "Image offset" is the term
// of the leaf's byte address inside the LDS image of a tile that does not
// depend on the object: AoS: offset in the record; SoA: tile * prefix;
// AoSoA: width * prefix.
struct LeafDesc {
  uint32_t src_off;
  uint32_t dst_off;
  uint8_t src_size;
  uint8_t dst_size;
  uint8_t op;
  uint8_t byte_wise;       // 1: an access in an image is not naturally aligned
  uint16_t mstride;        // OP_PTR: member record stride
  uint8_t off_type;        // OP_PTR/OP_LEN: rl_type of the source offsets
  uint8_t code;            // LeafCode: the move as one switch value
  const uint8_t* src_col;  // SoA source column, or the offsets for OP_PTR/OP_LEN
  uint8_t* dst_col;        // SoA destination column
};
static_assert(sizeof(LeafDesc) == 32, "LeafDesc layout");

struct SideDesc {
  uint8_t* base;           // AoS records / AoSoA blocks
  uint32_t kind;
  uint32_t stride;         // AoS record stride
  uint32_t width;          // AoSoA block width W
  uint32_t obj_bytes;      // sum of the leaf sizes on this side
  uint32_t width_magic;    // ceil(2^32 / W): q = umulhi(i, magic) for i < 2^16
  uint32_t image_bytes;    // bytes of this side's LDS image of one full tile
};

// Dense conversion of `n` objects (or of a count read on the device).
struct DenseDesc {
  SideDesc src, dst;
  uint64_t n;              // objects; with count_offsets: the capacity bound
  // Optional device-side count and index base (member columns of a group):
  // count = off[count_index] - off[0], base = off[0], both read on the device.
  const uint8_t* count_offsets;
  uint64_t count_index;
  uint32_t count_off_type; // rl_type of count_offsets
  uint32_t tile;           // objects per tile (multiple of 16 and of W)
  uint32_t n_leaves;
  uint32_t zero_dst;       // zero the destination image before filling it
  // Optional fused local scan of jagged counts (AoS record source):
  uint8_t* scan_offsets;   // destination offsets column (null: no scan)
  uint32_t scan_len_off;   // byte offset of the u32 count in a record
  uint32_t scan_off_type;  // rl_type of scan_offsets
  uint32_t* status;        // device status word
  uint32_t units_src;      // 1: SoA source, full tiles walk the image by unit_src
  uint32_t units_dst;      // 1: SoA destination, full tiles walk the image by unit_dst
  uint32_t dma;            // 1: source runs may be DMA'd into LDS (AoS / AoSoA: when a
                           //    tile's run is 16-byte aligned; SoA: 16-byte aligned columns)
  uint32_t slow_leaves;    // 1: some leaf needs the generic (byte-wise / offsets) path
  uint32_t dst_direct;     // 1: values go straight from the source image to global memory
                           //    (SoA / AoSoA destination, no destination image in LDS)
  uint32_t vt_magic;       // ceil(2^32 / (tile / 16)): SoA image vector -> byte unit
  uint32_t fast_leaves;    // leaves on the fast transform path (code below CODE_BYTES)
  uint32_t pipe_slot;      // single conversions: LDS bytes of each of two tile slots
                           // (double-buffered pipeline); 0: one slot
  uint64_t src_capacity;   // with count_offsets: source member capacity (count <= it - base)
  // Offsets column staged in LDS per tile for the record (pointer, count)
  // leaves of an AoS destination (null: read from global memory per object).
  // The kernel that stages them also checks them (non-decreasing, inside
  // the source member capacity, total inside the destination's).
  const uint8_t* stage_offsets;
  uint32_t stage_type;     // rl_type of stage_offsets
  uint32_t stream_stores;  // 1: values stored straight from the transform are non-temporal
  uint64_t stage_src_capacity;
  uint64_t stage_dst_capacity;
  LeafDesc leaf[kMaxLeaves];
  uint8_t unit_src[kMaxUnits];   // SoA image: byte unit of object size -> leaf
  uint8_t unit_dst[kMaxUnits];
};

// Second pass of the offsets scan: exclusive scan of per-tile totals.
struct ScanTotalsDesc {
  uint8_t* offsets;        // n + 1 entries
  uint64_t n;
  uint32_t tile;
  uint32_t off_type;
  uint64_t capacity;       // destination member capacity
  uint32_t* status;
};

// Third pass: add tile prefixes to the local offsets and gather the members
// of each tile's objects from a pool of member records.
struct GatherDesc {
  uint8_t* offsets;        // final offsets after this pass
  uint64_t n;
  uint32_t tile;
  uint32_t off_type;
  uint64_t capacity;       // destination member capacity
  const uint8_t* records;  // source records
  uint32_t rec_stride;
  uint32_t ptr_off;        // u64 byte offset into the pool
  uint32_t len_off;        // u32 member count
  uint32_t mstride;        // member record bytes
  uint32_t malign;         // member record alignment
  uint32_t n_members;      // member leaves (0: offsets only)
  uint32_t packed_words;   // 1..4: member leaves are the words of a packed record (fast path); 0: generic
  uint32_t sub;            // objects per gather work-group (divides tile)
  uint32_t pad0;
  const uint8_t* pool;
  uint64_t pool_bytes;
  uint32_t* status;
  uint32_t moff[kMaxMembers];
  uint32_t msize[kMaxMembers];
  uint8_t* mcol[kMaxMembers];
};

// Offsets column to offsets column: rebased copy with checks.
struct RebaseDesc {
  const uint8_t* src;
  uint8_t* dst;
  uint64_t n;
  uint32_t off_type;
  uint64_t src_capacity;
  uint64_t dst_capacity;
  uint32_t* status;
};

// Single-pass conversion of AoS records holding one jagged group's
// (pointer, count) pairs into an offsets column and member columns, for
// member records of 1..4 packed 4-byte words: one work-group per tile does
// the per-object leaves (as a dense step), the scan of the counts, a
// look-back over the tiles before it for the tile's prefix, the offsets
// and the members.
struct JaggedDesc {
  DenseDesc dense;         // per-object leaves of the records: source records, tile, direct stores
  uint8_t* offsets;        // destination offsets column (n + 1 entries)
  uint64_t capacity;       // destination member capacity
  const uint8_t* pool;     // source member pool
  uint64_t pool_bytes;
  uint64_t* lookback;      // one 64-bit word per tile
  uint8_t* mcol[4];        // destination member columns (16-byte aligned)
  uint32_t ptr_off;        // u64 byte offset into the pool, in a record
  uint32_t len_off;        // u32 member count, in a record
  uint32_t mstride;        // member record bytes (4 * words)
  uint32_t malign;         // member record alignment
  uint32_t words;          // 1..4
  uint32_t off_type;       // rl_type of the offsets
  uint32_t stage;          // members per LDS staging pass
  uint32_t epoch;          // launch number on this look-back buffer (set at enqueue)
  uint32_t stream_members; // 1: member columns stored non-temporally
};
// Look-back memory: one word per tile, zero before its first use; launches
// on one buffer must be ordered (one stream) and numbered by the host.
inline uint64_t lookback_bytes(uint64_t tiles) { return tiles * 8; }
// Counts and prefixes in look-back words are kept below 2^40 (saturating).
constexpr uint64_t kLookbackValueLimit = (1ull << 40) - 1;

// One side of the generic object mover: any layout kind, any object index.
// Address of leaf c of object i: AoS base + i * stride + off[c]; SoA
// col[c] + i * size; AoSoA base + (i / W) * W * obj_bytes + W * off[c] +
// (i % W) * size (off[c] = prefix of the leaf sizes).
struct GenSide {
  uint8_t* base;
  uint32_t kind, stride, width, obj_bytes;
  uint32_t off[kMaxLeaves];      // AoS/AoSoA: leaf offsets; strided: leaf strides
  uint8_t* col[kMaxLeaves];      // SoA, strided: one buffer per leaf
  const uint64_t* index;         // strided: element of each object, or NULL
  uint64_t elements;             // strided with an index: elements per leaf
};

// Objects moved one thread per object: destination object dst0 + k takes
// source object map[k] (or src0 + k) for k < count (host count, or *count_dev
// when set); zero_only: the destination objects' slots are zeroed instead.
struct MoveDesc {
  GenSide src, dst;
  uint8_t src_size[kMaxLeaves];
  uint8_t dst_size[kMaxLeaves];
  uint8_t op[kMaxLeaves];   // LeafOp: copy, narrow, widen
  uint32_t n_leaves;
  uint32_t zero_only;
  uint64_t count;
  const uint64_t* count_dev;
  const uint64_t* map;
  uint64_t src0, dst0;
  uint32_t* status;              // bounds flag for indexes past the elements
};

// Member storage of one jagged group for the member mover: records with
// (pointer, count) pairs and a pool (form 0), or an offsets column and
// member columns (form 1).
struct GenGroup {
  uint32_t form;
  uint32_t n_members;
  uint64_t capacity;        // members the storage holds
  uint8_t* records;         // form 0
  uint32_t rec_stride, ptr_off, len_off, mstride, malign;
  uint8_t* pool;
  uint8_t* offsets;         // form 1: n + 1 entries
  uint32_t off_type;
  uint32_t moff[kMaxMembers];     // form 0: member leaf offsets in a member record
  uint8_t* mcol[kMaxMembers];     // form 1: member columns
  uint8_t msize[kMaxMembers];
};

// Members of gathered objects: destination object k (k < *count_dev) takes
// the members of source object map[k], placed from member index out_off[k]
// (exclusive scan of the gathered counts, out_off[*count_dev] = total).
struct MemberMoveDesc {
  GenGroup src, dst;
  const uint64_t* map;
  const uint64_t* count_dev;
  const uint64_t* out_off;
  uint64_t n_max;           // host bound of *count_dev
  uint32_t* status;
};

// Scans over a device-side count of entries (compaction).  Tiles of
// kSelectTile entries.
constexpr uint32_t kSelectTile = 1024;
struct SelectDesc {
  const uint8_t* keep;      // n flags (0 = drop)
  uint64_t n;
  uint64_t* tile_tot;       // per tile: count, then exclusive prefix
  uint64_t* map;            // kept object indices, in order
  uint64_t* count;          // kept objects (device)
  uint64_t* count_out;      // optional second copy for the caller (device)
  // counts of gathered objects, for their member offsets
  GenGroup src;             // source group (counts read from it)
  uint64_t* lens;           // per kept object: its member count, then exclusive offsets (n + 1)
  uint32_t* status;
};

// Device-side (index, count) copy of jagged member columns for appends:
// members [src_off[0], src_off[count]) of the source go to member index
// dst_off[at] on of the destination; the offsets entries at+1 .. at+count
// become dst_off[at] + (src_off[k] - src_off[0]).
struct AppendDesc {
  GenGroup src, dst;        // both form 1
  uint64_t at, count;
  uint32_t* status;
};

// Device-resident tables of a batch: every step of every item, grouped by
// the kernel that runs it.  Prefix arrays have one entry per item plus one.
// A fan-out group of a batch: dense steps that read the same source tiles
// (one source converted into several layouts).  One work-group converts a
// tile of the source for all of them: the tile is read into LDS once and
// thread group k (fan_per threads) stores destination k.
constexpr uint32_t kFanMax = 4;
constexpr uint32_t kFanMaxThreads = 512;
struct FanGroup {
  uint32_t n_dst;              // steps in the group (2 .. kFanMax)
  uint32_t step[kFanMax];      // their dense step indices
  uint32_t first, end;         // the group's tiles in the fan-out tile space
};

struct BatchTables {
  const DenseDesc* dense;
  const uint64_t* dense_prefix;     // first tile of each dense step
  const uint64_t* dense_map;        // tile -> (dense step << 32 | tile within the step)
  uint64_t* dense_counts;           // per dense step: (count, source base)
  uint32_t device_counts;           // 1: some dense step's count is read on the device (count pass needed)
  uint32_t n_dense;
  uint32_t dense_tiles;
  const GatherDesc* gather;
  const uint64_t* gather_prefix;    // first sub-tile of each gather step
  const uint32_t* gather_item;      // sub-tile -> gather step
  uint32_t n_gather;
  uint32_t gather_tiles;            // sub-tiles of all gather steps
  const ScanTotalsDesc* totals;
  uint32_t n_totals;
  uint32_t n_rebase;
  const RebaseDesc* rebase;
  const uint64_t* rebase_prefix;    // first rebase tile of each rebase step
  const uint32_t* rebase_item;      // rebase tile -> rebase step
  uint32_t rebase_tiles;
  uint32_t pipe_slot;               // dense steps: LDS bytes of each of two tile slots; 0: one slot
  const FanGroup* fan;              // fan-out groups (their steps are not in dense_map)
  uint32_t fan_tiles;               // tiles of all fan-out groups
  uint32_t fan_per;                 // threads per destination of a fan-out group (a multiple of 64)
  uint32_t fan_slot;                // fan-out tiles: LDS bytes of each of two tile slots; 0: one slot
  uint32_t* status;                 // status word of the launching stream
};
constexpr uint32_t kRebaseTile = 8192;   // offsets entries per rebase work-group

// ---- kernel launchers (kernels.hip) ----
hipError_t launch_dense(const DenseDesc& d, uint32_t threads, uint32_t grid,
                        hipStream_t s);
hipError_t launch_scan_totals(const ScanTotalsDesc& d, hipStream_t s);
hipError_t launch_gather(const GatherDesc& d, uint32_t threads, hipStream_t s);
hipError_t launch_rebase(const RebaseDesc& d, hipStream_t s);
hipError_t launch_take_status(uint32_t* status, uint32_t* out, hipStream_t s);
// One work-group per tile.
hipError_t launch_jagged(const JaggedDesc& j, uint32_t threads, hipStream_t s);
uint32_t jagged_lds_bytes(const JaggedDesc& j);
// Members per staging pass of the single-pass jagged kernel (32 KB of words).
constexpr uint32_t jagged_stage_members(uint32_t words) { return (8192 / words) / 64 * 64; }
// Zero `bytes` of device memory with a kernel (usable where a memset node is not).
hipError_t launch_zero(void* p, uint64_t bytes, hipStream_t s);
// Plain copy between disjoint ranges reachable from the device.
hipError_t launch_copy(void* dst, const void* src, uint64_t bytes, hipStream_t s);
// Generic object and member movers, compaction scans, appends.
hipError_t launch_move(const MoveDesc& d, uint64_t grid_objects, hipStream_t s);
hipError_t launch_select(const SelectDesc& d, hipStream_t s);
hipError_t launch_select_members(const SelectDesc& d, hipStream_t s);
hipError_t launch_member_move(const MemberMoveDesc& d, hipStream_t s);
hipError_t launch_append(const AppendDesc& d, hipStream_t s);
hipError_t launch_zero_bytes(void* p, uint64_t bytes, hipStream_t s);
// Device address of the status words of the current device.
hipError_t status_words(uint32_t** out);
hipError_t launch_batch(const BatchTables& b, uint32_t dense_threads, uint32_t gather_threads,
                        uint32_t grid, uint32_t dense_lds, uint32_t gather_lds, hipStream_t s,
                        uint32_t fan_threads = 0, uint32_t fan_lds = 0);
// Members per pass of the packed-word gather (LDS staging per word).
constexpr uint32_t kGatherStage = 1024;
// LDS of a gather work-group: staged objects, then the word columns.
__host__ __device__ inline uint32_t gather_stage_offset(uint32_t sub) {
  return ((2 * sub + 1) * 8 + sub * 4 + 15) & ~15u;
}
uint32_t gather_lds_bytes(uint32_t sub, uint32_t words);
// Threads of a gather work-group.
constexpr uint32_t kGatherThreads = 128;
uint32_t dense_lds_bytes(const DenseDesc& d);
// Work-groups of the batch dense kernel that fit on the current device at
// once for this block size and LDS size (0 if unknown).
uint32_t batch_resident_blocks(uint32_t threads, uint32_t lds, bool pipelined);
// Fan-out work-groups of a batch that fit on the device at once; 0 if unknown.
uint32_t fanout_resident_blocks(uint32_t threads, uint32_t lds, bool pipelined);
uint64_t dense_tiles(const DenseDesc& d);

// ---- errors ----
void set_error(const char* fmt, ...);
rl_status fail(rl_status st, const char* fmt, ...);
rl_status hip_fail(hipError_t e, const char* what);

// ---- device state ----
// Status word of a stream on the current device (nullptr on a HIP error).
uint32_t* stream_status(hipStream_t s);
// The status (and message) of a set of device status flags.
rl_status status_of_flags(uint32_t flags);

}  // namespace rl

// ---- opaque handle types ----
struct rl_schema {
  struct Leaf {
    rl_type type;
    uint32_t size;
    int32_t field;
    uint32_t element;
    int32_t subgroup;
  };
  // Record slots in order: per-object leaves and, per jagged group, the
  // (ptr, len) pair.  kind 0: leaf index; 1: ptr of group; 2: len of group.
  struct Slot {
    int kind;
    int index;
    int32_t subgroup;
  };
  // A property of the schema's tree; flat field lists are turned into one.
  struct Prop {
    rl_prop_kind kind;
    rl_type type;                  // item: value type; jagged: offset type
    uint32_t extent;               // array
    int32_t group;                 // jagged from a flat list: its group; -1: numbered in walk order
    std::string name;
    std::vector<Prop> children;
  };
  std::vector<Prop> tree;
  std::vector<const Prop*> group_prop;      // per group: its jagged property
  std::vector<rl_field> fields;
  std::vector<std::string> names;
  std::vector<Leaf> leaves;
  std::vector<std::vector<Leaf>> members;   // per group
  std::vector<rl_type> offset_types;        // per group
  std::vector<Slot> slots;
};

struct rl_layout {
  const rl_schema* schema;
  rl_kind kind;
  rl_space space;
  uint32_t width;
  uint64_t stride;
  std::vector<uint64_t> slot_offsets;       // AoS
  std::vector<rl_type> storage;             // per per-object leaf
  std::vector<uint32_t> leaf_offset;        // AoS: offset of each leaf in the record
  std::vector<uint32_t> prefix;             // prefix sums of storage sizes
  uint32_t obj_bytes;                       // sum of storage sizes
  uint32_t record_align;                    // AoS: largest slot alignment
  std::vector<uint32_t> ptr_off, len_off;   // AoS: per group
  std::vector<uint32_t> mstride, malign;    // AoS: per group member record
  std::vector<std::vector<uint32_t>> moff;  // AoS: per group member offsets
  bool has_gaps;                            // AoS: bytes not covered by a written slot
  std::vector<uint64_t> leaf_stride;        // strided: bytes between elements, per leaf
  bool indexed;                             // strided: elements reached through an index table
};
