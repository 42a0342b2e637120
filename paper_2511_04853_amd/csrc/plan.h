// Conversion plans: the kernel steps that convert one collection.
#pragma once

#include <vector>

#include "rl_internal.h"

namespace rl {

struct PlanShape {
  uint32_t tile = 0;      // objects per tile (0: default)
  uint32_t threads = 0;   // threads per work-group (0: a quarter of the tile)
  uint32_t grid = 0;      // work-groups of dense steps (0: one per tile, capped)
  int direct = -1;        // destination values stored straight to global memory:
                          // -1 where the destination allows it, 0 never
  int dma = -1;           // source runs DMA'd into LDS: -1 where aligned, 0 never
  int fused = -1;         // single-pass jagged kernel: -1 where it applies, 0 never,
                          // 2 required (a jagged records source fails where it does not apply)
  int pipe = -1;          // dense steps double-buffered (two tile slots in LDS):
                          // 1 wherever two slots fit; otherwise (-1, 0) never
  int stream = 1;         // 1: values stored straight from the transform are non-temporal
  // Look-back memory of single-pass jagged steps given by the caller
  // (zeroed before its first use, used by one stream at a time); null:
  // the library's per-stream buffer.  A step needing more tiles than it
  // holds takes the multi-kernel path.
  uint64_t* lookback = nullptr;
  uint64_t lookback_bytes = 0;
};

struct Step {
  enum Kind { DENSE, SCAN_TOTALS, GATHER, REBASE, JAGGED } kind;
  uint32_t threads = 256;
  uint32_t grid = 0;
  DenseDesc dense;
  ScanTotalsDesc totals;
  GatherDesc gather;
  RebaseDesc rebase;
  JaggedDesc jagged;
};

struct Plan {
  std::vector<Step> steps;
};

// One side of a dense conversion, independent of where its leaves come
// from (the per-object leaves of a layout, or a jagged group's members).
struct SideSpec {
  uint32_t kind = KIND_SOA;
  uint8_t* base = nullptr;           // AoS records / AoSoA blocks
  uint32_t stride = 0;               // AoS
  uint32_t width = 0;                // AoSoA
  std::vector<uint32_t> off;         // AoS: per leaf offset in the record
  std::vector<uint8_t*> cols;        // SoA: per leaf column
  std::vector<rl_type> types;        // storage type per leaf
};

struct Range {
  uintptr_t lo, hi;
};
rl_status validate_view(const rl_view* v, uint64_t n, const char* which, std::vector<Range>* ranges,
                        bool want_device);
// dst_shared: the destination's buffers may overlap each other (the leaves
// of a strided layout sharing a record array); they are still checked
// against the source.
rl_status check_overlap(const std::vector<Range>& src, const std::vector<Range>& dst, bool dst_shared = false);
// Conversion through the general one-thread-per-object mover (any kinds on
// either side; used for strided layouts).
rl_status convert_general(const rl_view& src, const rl_view& dst, uint64_t n, hipStream_t s);

uint32_t type_size(rl_type t);
// Natural (C) record of a schema's per-object slots in the given leaf
// storage types, and of group g's member record.
void natural_record(const rl_schema* s, const std::vector<rl_type>& storage, std::vector<uint64_t>& offs,
                    uint64_t& stride);
void natural_member_record(const rl_schema* s, uint32_t g, std::vector<uint32_t>& offs, uint32_t& stride,
                           uint32_t& align);
uint32_t layout_n_buffers(const rl_layout* L);
void layout_buffer_bytes(const rl_layout* L, uint64_t n, const uint64_t* members, uint64_t* bytes);
uint32_t group_buffer(const rl_layout* L, uint32_t g);

SideSpec object_side(const rl_layout* L, void* const* bufs, uint64_t index0);
SideSpec member_side(const rl_layout* L, void* const* bufs, uint32_t g);

// Tile size for two sides given a target (multiple of 16 and of the block
// widths, images within the LDS budget); 0 if none fits.
uint32_t choose_tile(const SideSpec& s, const SideSpec& d, uint32_t target, uint64_t n);
rl_status build_dense(const SideSpec& s, const SideSpec& d, uint64_t n, uint32_t tile,
                      DenseDesc* out);

// Full conversion of objects 0..n-1 (views already validated).
rl_status make_plan(const rl_view& src, const rl_view& dst, uint64_t n, const PlanShape& shape,
                    Plan* plan);
rl_status make_offsets_plan(const rl_view& src, const rl_view& dst, uint32_t group, uint64_t n,
                            const PlanShape& shape, Plan* plan);
rl_status enqueue_plan(const Plan& plan, hipStream_t stream);
PlanShape shape_from_env();
// Whether `s` is being captured into a graph (single-pass jagged steps
// number their launches on the host, so they are not captured).
bool stream_capturing(hipStream_t s);
bool auto_width(const rl_view* v);

// Host <-> device transfer (rl_transfer) with an optional staging block
// owned by the caller (device memory of at least staging_bytes(host view)
// bytes; nullptr: the library's per-stream staging buffer).
rl_status transfer_impl(const rl_view* src, const rl_view* dst, uint64_t n, hipStream_t stream,
                        const rl_xfer_opts* opts, uint8_t* stage, uint64_t stage_bytes,
                        uint64_t* lookback = nullptr, uint64_t lookback_bytes = 0);
uint64_t staging_bytes(const rl_view& host_view, uint64_t n);
bool transfer_is_staged(const rl_view& host_view, const rl_xfer_opts* opts);
bool is_host(rl_space s);
// User transfer specialisations matching (src, dst), in priority order;
// *handled when one took the call.
rl_status run_specialisations(const rl_view* src, const rl_view* dst, uint64_t n, void* stream, bool* handled);
// Device-to-device copy with memmove semantics (overlap allowed).
rl_status device_move(uint8_t* dst, const uint8_t* src, uint64_t bytes, hipStream_t s);

}  // namespace rl
