// Batched conversion: many collections through one launch of a captured
// HIP graph.  Every item is planned as for rl_convert; the steps of all
// items are gathered into device-resident tables by kernel kind, and three
// persistent kernels (dense tiles, tile-total scans and rebases, member
// gathers) stride over the tiles of all items.  The graph holds the three
// launches; a per-collection loop over rl_convert plans is kept for
// comparison.  An autotuner times candidate tile shapes (and block widths
// of "auto" AoSoA destinations) on the batch itself and keeps the fastest,
// remembering the choice in a JSON cache.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>

#include "plan.h"
#include "rl_internal.h"

using namespace rl;

namespace {

constexpr uint32_t kAutoWidths[] = {32, 64, 128};

struct Item {
  const rl_layout* src_layout;
  const rl_layout* dst_layout;        // as given (width 0 = auto)
  std::unique_ptr<rl_layout> resolved;  // auto width resolved
  uint64_t src_cap, dst_cap, n;
  std::vector<void*> src_bufs, dst_bufs;
  std::vector<uint64_t> src_mcap, dst_mcap;
  rl_view src_view() const {
    return rl_view{src_layout, src_cap, src_mcap.empty() ? nullptr : src_mcap.data(),
                   const_cast<void* const*>(src_bufs.data())};
  }
  rl_view dst_view() const {
    return rl_view{resolved ? resolved.get() : dst_layout, dst_cap,
                   dst_mcap.empty() ? nullptr : dst_mcap.data(), const_cast<void* const*>(dst_bufs.data())};
  }
  bool auto_width() const { return dst_layout->kind == RL_AOSOA && dst_layout->width == 0; }
};

constexpr uint32_t kOnePerTile = 1u << 30;   // grid larger than any tile count

struct Config {
  uint32_t tile = 256, threads = 128, width = 64;   // threads: dense work-groups
  uint32_t grid = 0;     // dense work-groups; 0: as many as fit on the device at once
  uint32_t direct = 0;   // 1: launch the batch kernels directly instead of replaying the graph
  uint32_t gather_threads = kGatherThreads;   // member-gather work-groups
  uint32_t pipe = 0;     // 1: dense steps double-buffered (two tile slots per work-group)
  uint32_t stream = 1;   // 1: values stored straight from the transform are non-temporal
  uint32_t fanout = 0;   // >0: steps reading the same source tiles share one work-group per tile,
                         // this many threads per destination (64 or 128)
};

struct DeviceTables {
  uint8_t* mem = nullptr;
  BatchTables t{};
  uint32_t dense_lds = 0, gather_lds = 0;
  uint32_t fan_threads = 0, fan_lds = 0;
  uint32_t fan_groups = 0, fan_steps = 0, dense_steps = 0;
  void release() {
    if (mem) (void)hipFree(mem);
    mem = nullptr;
  }
};

}  // namespace

struct rl_batch {
  int autotune = 0;
  std::string cache;
  std::vector<Item> items;
  bool finalized = false;
  Config cfg;
  std::vector<Plan> plans;   // per item (for the launch loop)
  DeviceTables dev;
  hipStream_t cap = nullptr;
  // captured graphs, one per status word of the streams launched on (the
  // kernels report device-detected errors to the launching stream's word)
  std::map<uint32_t*, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
  double tuned_us = 0;
  ~rl_batch() {
    for (auto& g : graphs) {
      if (g.second.second) (void)hipGraphExecDestroy(g.second.second);
      if (g.second.first) (void)hipGraphDestroy(g.second.first);
    }
    if (cap) (void)hipStreamDestroy(cap);
    dev.release();
  }
};

namespace {

rl_status resolve_widths(rl_batch* b, uint32_t width) {
  for (auto& it : b->items) {
    if (!it.auto_width()) continue;
    it.resolved.reset(new rl_layout(*it.dst_layout));
    it.resolved->width = width;
  }
  return RL_OK;
}

rl_status plan_all(rl_batch* b, const Config& c) {
  b->plans.clear();
  PlanShape shape;
  shape.tile = c.tile;
  shape.threads = c.threads;
  shape.direct = shape_from_env().direct;
  shape.fused = 0;   // batches run their jagged items through the table kernels
  shape.stream = c.stream ? 1 : 0;
  for (auto& it : b->items) {
    Plan p;
    if (it.n) {
      rl_view s = it.src_view(), d = it.dst_view();
      rl_status st = make_plan(s, d, it.n, shape, &p);
      if (st) return st;
    }
    b->plans.push_back(std::move(p));
  }
  return RL_OK;
}

// Where the source bytes of a dense step's tiles live: the records, blocks
// or first column of its source (0 when the step's count is known only on
// the device, which gives each such step keys of its own).
static uint64_t source_key(const DenseDesc& d) {
  if (d.count_offsets) return 0;
  if (d.src.kind != KIND_SOA) return (uint64_t)(uintptr_t)d.src.base;
  return d.n_leaves ? (uint64_t)(uintptr_t)d.leaf[0].src_col : 0;
}

// Tile map of the dense kernel: entry g = (step << 32) | tile of the step.
// Work-group w runs on XCD w mod 8 and takes map entries w, w + grid, ...
// (grids are multiples of 8), so entry g runs on XCD g mod 8, and entries
// x, x + 8, x + 16, ... of one XCD run in that order.  Tiles that read the
// same source objects (one source converted into several layouts) form a
// run that goes to one XCD's consecutive entries: the later reads of the
// run hit that XCD's L2.  Runs go to the XCD with the most entries left,
// so single-tile runs interleave over the XCDs as in plain order.
// `steps` lists the dense steps the map covers (those not in a fan-out
// group); prefix[k] is the first tile of steps[k].
static void fill_dense_map(const std::vector<DenseDesc>& dense, const std::vector<uint32_t>& steps,
                           const std::vector<uint64_t>& prefix, uint64_t* map) {
  struct T {
    uint64_t key, first, entry;
  };
  std::vector<T> tiles;
  tiles.reserve(prefix.back());
  for (size_t i = 0; i + 1 < prefix.size(); ++i) {
    const uint32_t k = steps[i];
    const uint64_t key = source_key(dense[k]);
    for (uint64_t t = 0; t < prefix[i + 1] - prefix[i]; ++t)
      tiles.push_back({key ? key : (uint64_t)k + 1, t * dense[k].tile, ((uint64_t)k << 32) | t});
  }
  std::stable_sort(tiles.begin(), tiles.end(),
                   [](const T& a, const T& b) { return a.key != b.key ? a.key < b.key : a.first < b.first; });
  const uint64_t L = tiles.size();
  uint64_t next[8], left[8];
  for (uint64_t x = 0; x < 8; ++x) {
    next[x] = x;
    left[x] = x < L ? (L - x + 7) / 8 : 0;
  }
  uint32_t rr = 0;
  for (uint64_t i = 0; i < L;) {
    uint64_t j = i + 1;
    while (j < L && tiles[j].key == tiles[i].key && tiles[j].first == tiles[i].first) ++j;
    for (uint64_t k = i; k < j;) {
      uint32_t x = rr;
      for (uint32_t y = 0; y < 8; ++y) {
        const uint32_t c = (rr + y) & 7;
        if (left[c] > left[x]) x = c;
      }
      rr = (x + 1) & 7;
      for (; k < j && left[x]; ++k, --left[x], next[x] += 8) map[next[x]] = tiles[k].entry;
    }
    i = j;
  }
}

rl_status build_tables(rl_batch* b, const Config& c, DeviceTables* out) {
  std::vector<DenseDesc> dense;
  std::vector<GatherDesc> gather;
  std::vector<ScanTotalsDesc> totals;
  std::vector<RebaseDesc> rebase;
  std::vector<uint64_t> dprefix{0}, gprefix{0}, rprefix{0};
  uint32_t dense_lds = 0, gather_lds = 0;
  for (const Plan& p : b->plans)
    for (const Step& s : p.steps) {
      switch (s.kind) {
        case Step::DENSE:
          dense.push_back(s.dense);
          break;
        case Step::GATHER:
          gather.push_back(s.gather);
          gprefix.push_back(gprefix.back() + (s.gather.n + s.gather.sub - 1) / s.gather.sub);
          gather_lds = std::max(gather_lds, gather_lds_bytes(s.gather.sub, s.gather.packed_words));
          break;
        case Step::SCAN_TOTALS: totals.push_back(s.totals); break;
        case Step::REBASE:
          rebase.push_back(s.rebase);
          rprefix.push_back(rprefix.back() + (s.rebase.n + 1 + kRebaseTile - 1) / kRebaseTile);
          break;
      }
    }
  // fan-out groups: steps that read the same source tiles, their counts
  // known on the host, with direct destinations and no scan, staged
  // offsets or slow leaves; up to kFanMax steps per group
  std::vector<FanGroup> fans;
  std::vector<uint8_t> grouped(dense.size(), 0);
  if (c.fanout) {
    std::map<std::string, std::vector<uint32_t>> by_source;
    for (uint32_t k = 0; k < dense.size(); ++k) {
      const DenseDesc& d = dense[k];
      if (d.count_offsets || d.scan_offsets || d.stage_offsets || !d.dst_direct || d.slow_leaves || !d.n) continue;
      std::string key(reinterpret_cast<const char*>(&d.src), sizeof d.src);
      auto add = [&](const void* p, size_t n) { key.append(reinterpret_cast<const char*>(p), n); };
      add(&d.n, sizeof d.n);
      add(&d.tile, sizeof d.tile);
      add(&d.n_leaves, sizeof d.n_leaves);
      add(&d.dma, sizeof d.dma);
      for (uint32_t c2 = 0; c2 < d.n_leaves; ++c2) {
        add(&d.leaf[c2].src_off, sizeof d.leaf[c2].src_off);
        add(&d.leaf[c2].src_size, sizeof d.leaf[c2].src_size);
        add(&d.leaf[c2].src_col, sizeof d.leaf[c2].src_col);
      }
      by_source[key].push_back(k);
    }
    for (auto& kv : by_source) {
      const auto& v = kv.second;
      if (v.size() < 2) continue;
      for (size_t i = 0; i < v.size(); i += kFanMax) {
        FanGroup g{};
        g.n_dst = (uint32_t)std::min<size_t>(kFanMax, v.size() - i);
        if (g.n_dst < 2) break;   // a lone remainder stays a plain step
        for (uint32_t w = 0; w < g.n_dst; ++w) {
          g.step[w] = v[i + w];
          grouped[v[i + w]] = 1;
        }
        fans.push_back(g);
      }
    }
  }
  std::vector<uint32_t> singles;
  for (uint32_t k = 0; k < dense.size(); ++k)
    if (!grouped[k]) {
      singles.push_back(k);
      dprefix.push_back(dprefix.back() + dense_tiles(dense[k]));
      dense_lds = std::max(dense_lds, dense_lds_bytes(dense[k]));
    }
  uint64_t fan_tiles = 0;
  uint32_t fan_lds = 0, fan_threads = 0;
  for (uint32_t g = 0; g < fans.size(); ++g) {
    fans[g].first = (uint32_t)std::min<uint64_t>(fan_tiles, UINT32_MAX);
    fan_tiles += dense_tiles(dense[fans[g].step[0]]);
    fans[g].end = (uint32_t)std::min<uint64_t>(fan_tiles, UINT32_MAX);
    for (uint32_t w = 0; w < fans[g].n_dst; ++w) fan_lds = std::max(fan_lds, dense_lds_bytes(dense[fans[g].step[w]]));
    fan_threads = std::max(fan_threads, c.fanout * fans[g].n_dst);
  }
  if (dprefix.back() >= (1ull << 32) || gprefix.back() >= (1ull << 32) || fan_tiles >= (1ull << 32))
    return fail(RL_EUNSUPPORTED, "batch has more than 2^32 tiles");
  // one allocation: tables, prefix arrays and tile -> item maps
  size_t sz = 0;
  auto reserve = [&](size_t bytes) { size_t at = sz; sz += (bytes + 255) & ~size_t(255); return at; };
  const size_t o_dense = reserve(dense.size() * sizeof(DenseDesc));
  const size_t o_dp = reserve(dprefix.size() * 8);
  const size_t o_gather = reserve(gather.size() * sizeof(GatherDesc));
  const size_t o_gp = reserve(gprefix.size() * 8);
  const size_t o_tot = reserve(totals.size() * sizeof(ScanTotalsDesc));
  const size_t o_reb = reserve(rebase.size() * sizeof(RebaseDesc));
  const size_t o_dmap = reserve(dprefix.back() * 8);
  const size_t o_dcnt = reserve(dense.size() * 16);
  const size_t o_gitem = reserve(gprefix.back() * 4);
  const size_t o_rp = reserve(rprefix.size() * 8);
  const size_t o_ritem = reserve(rprefix.back() * 4);
  const size_t o_fan = reserve(fans.size() * sizeof(FanGroup));
  std::vector<uint8_t> host(sz, 0);
  memcpy(host.data() + o_dense, dense.data(), dense.size() * sizeof(DenseDesc));
  memcpy(host.data() + o_dp, dprefix.data(), dprefix.size() * 8);
  memcpy(host.data() + o_gather, gather.data(), gather.size() * sizeof(GatherDesc));
  memcpy(host.data() + o_gp, gprefix.data(), gprefix.size() * 8);
  memcpy(host.data() + o_tot, totals.data(), totals.size() * sizeof(ScanTotalsDesc));
  memcpy(host.data() + o_reb, rebase.data(), rebase.size() * sizeof(RebaseDesc));
  {
    // host-known counts are written here; device-side ones by the count pass
    uint64_t* dc = (uint64_t*)(host.data() + o_dcnt);
    for (size_t k = 0; k < dense.size(); ++k) {
      dc[2 * k] = dense[k].n;
      dc[2 * k + 1] = 0;
    }
    fill_dense_map(dense, singles, dprefix, (uint64_t*)(host.data() + o_dmap));
    memcpy(host.data() + o_fan, fans.data(), fans.size() * sizeof(FanGroup));
    uint32_t* gi = (uint32_t*)(host.data() + o_gitem);
    for (size_t k = 0; k + 1 < gprefix.size(); ++k)
      for (uint64_t t = gprefix[k]; t < gprefix[k + 1]; ++t) gi[t] = (uint32_t)k;
    memcpy(host.data() + o_rp, rprefix.data(), rprefix.size() * 8);
    uint32_t* ri = (uint32_t*)(host.data() + o_ritem);
    for (size_t k = 0; k + 1 < rprefix.size(); ++k)
      for (uint64_t t = rprefix[k]; t < rprefix[k + 1]; ++t) ri[t] = (uint32_t)k;
  }
  out->release();
  hipError_t e = hipMalloc(&out->mem, sz);
  if (e != hipSuccess) return fail(RL_ENOMEM, "batch tables (%zu bytes): %s", sz, hipGetErrorString(e));
  if ((e = hipMemcpy(out->mem, host.data(), sz, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "hipMemcpy(batch tables)");
  BatchTables& t = out->t;
  t.dense = (const DenseDesc*)(out->mem + o_dense);
  t.dense_prefix = (const uint64_t*)(out->mem + o_dp);
  t.dense_map = (const uint64_t*)(out->mem + o_dmap);
  t.dense_counts = (uint64_t*)(out->mem + o_dcnt);
  t.device_counts = std::any_of(dense.begin(), dense.end(), [](const DenseDesc& d) { return d.count_offsets != nullptr; });
  t.gather_item = (const uint32_t*)(out->mem + o_gitem);
  t.n_dense = (uint32_t)dense.size();
  t.dense_tiles = (uint32_t)dprefix.back();
  t.gather = (const GatherDesc*)(out->mem + o_gather);
  t.gather_prefix = (const uint64_t*)(out->mem + o_gp);
  t.n_gather = (uint32_t)gather.size();
  t.gather_tiles = (uint32_t)gprefix.back();
  t.totals = (const ScanTotalsDesc*)(out->mem + o_tot);
  t.n_totals = (uint32_t)totals.size();
  t.rebase = (const RebaseDesc*)(out->mem + o_reb);
  t.n_rebase = (uint32_t)rebase.size();
  t.rebase_prefix = (const uint64_t*)(out->mem + o_rp);
  t.rebase_item = (const uint32_t*)(out->mem + o_ritem);
  t.rebase_tiles = (uint32_t)rprefix.back();
  t.fan = (const FanGroup*)(out->mem + o_fan);
  t.fan_tiles = (uint32_t)fan_tiles;
  t.fan_per = c.fanout;
  out->fan_threads = fan_threads;
  out->fan_lds = fan_lds;
  t.fan_slot = 0;
  if (c.pipe && fan_tiles) {
    const uint32_t fslot = (fan_lds + 15u) & ~15u;
    if (2 * fslot <= 64 * 1024) {
      t.fan_slot = fslot;
      out->fan_lds = 2 * fslot;
    }
  }
  out->fan_groups = (uint32_t)fans.size();
  out->fan_steps = (uint32_t)(dense.size() - singles.size());
  out->dense_steps = (uint32_t)dense.size();
  out->dense_lds = dense_lds;
  out->gather_lds = gather_lds;
  t.pipe_slot = 0;
  const uint32_t slot = (dense_lds + 15u) & ~15u;
  if (c.pipe && 2 * slot <= 64 * 1024) {
    t.pipe_slot = slot;
    out->dense_lds = 2 * slot;
  }
  return RL_OK;
}

// Launch the batch kernels on `s`, reporting device-detected errors to
// `status` (the status word of the stream the batch is launched for).
rl_status launch_tables(const DeviceTables& d, const Config& c, hipStream_t s, uint32_t* status) {
  const uint32_t dt = std::min<uint32_t>(c.threads, kDenseMaxThreads);
  BatchTables t = d.t;
  t.status = status;
  hipError_t e = launch_batch(t, dt, c.gather_threads, c.grid, d.dense_lds, d.gather_lds, s, d.fan_threads, d.fan_lds);
  return e == hipSuccess ? RL_OK : hip_fail(e, "batch launch");
}

rl_status launch_tables(const DeviceTables& d, const Config& c, hipStream_t s) {
  uint32_t* status = stream_status(s);
  if (!status) return fail(RL_EHIP, "status words of the current device");
  return launch_tables(d, c, s, status);
}

// Signature of a batch for the tuning cache: item shapes with object counts
// bucketed by powers of two, and the device.
std::string signature(const rl_batch* b) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) { h = (h ^ v) * 1099511628211ull; };
  for (const auto& it : b->items) {
    for (const rl_layout* L : {it.src_layout, it.dst_layout}) {
      mix((uint64_t)L->kind);
      mix(L->width);
      mix(L->stride);
      for (auto t : L->storage) mix((uint64_t)t);
      mix(L->schema->members.size());
    }
    uint64_t bucket = 0;
    while ((1ull << bucket) < it.n) ++bucket;
    mix(bucket);
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    for (const char* p = prop.gcnArchName; *p; ++p) mix((uint64_t)*p);
    mix((uint64_t)prop.multiProcessorCount);
  }
  char buf[32];
  snprintf(buf, sizeof buf, "%016llx", (unsigned long long)h);
  return buf;
}

// The cache is a JSON object {"<signature>": {"tile": .., "threads": ..,
// "grid": .., "width": .., "us": ..}, ...}, one entry per line.
bool cache_lookup(const std::string& path, const std::string& sig, Config* c) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  const std::string key = "\"" + sig + "\"";
  while (std::getline(f, line)) {
    if (line.find(key) == std::string::npos) continue;
    auto num = [&](const char* name, uint32_t* v) {
      const std::string k = std::string("\"") + name + "\":";
      size_t p = line.find(k);
      if (p == std::string::npos) return false;
      *v = (uint32_t)strtoul(line.c_str() + p + k.size(), nullptr, 10);
      return true;
    };
    Config t;
    if (num("tile", &t.tile) && num("threads", &t.threads) && num("grid", &t.grid) && num("width", &t.width)) {
      num("direct", &t.direct);
      num("gather_threads", &t.gather_threads);
      num("pipe", &t.pipe);
      num("fanout", &t.fanout);
      num("stream", &t.stream);
      if (t.fanout) t.fanout = t.fanout >= 128 ? 128 : 64;
      *c = t;
      return true;
    }
  }
  return false;
}

void cache_store(const std::string& path, const std::string& sig, const Config& c, double us) {
  std::vector<std::string> keep;
  {
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
      if (line.size() < 4 || line[0] == '{' || line[0] == '}') continue;
      if (line.find("\"" + sig + "\"") != std::string::npos) continue;
      if (!line.empty() && line.back() == ',') line.pop_back();
      keep.push_back(line);
    }
  }
  char buf[256];
  snprintf(buf, sizeof buf,
           "  \"%s\": {\"tile\":%u, \"threads\":%u, \"grid\":%u, \"width\":%u, \"direct\":%u, "
           "\"gather_threads\":%u, \"pipe\":%u, \"fanout\":%u, \"stream\":%u, \"us\":%.2f}",
           sig.c_str(), c.tile, c.threads, c.grid, c.width, c.direct, c.gather_threads, c.pipe, c.fanout, c.stream, us);
  keep.push_back(buf);
  std::ofstream o(path + ".tmp");
  o << "{\n";
  for (size_t k = 0; k < keep.size(); ++k) o << keep[k] << (k + 1 < keep.size() ? ",\n" : "\n");
  o << "}\n";
  o.close();
  rename((path + ".tmp").c_str(), path.c_str());
}

// Device memory the tuner copies through between timed launches.
struct FlushBuffer {
  void* mem = nullptr;
  uint64_t bytes = 0;
};
constexpr uint64_t kFlushBytes = 512ull << 20;   // twice the 256 MB Infinity Cache

// Time one configuration (direct launches of the batch kernels).  A batch
// whose launch takes under 100 us is timed cold, as it runs over data it
// has not just touched: before each of 16 timed launches a copy through
// the flush buffer evicts L2 and the Infinity Cache, and each launch is
// timed alone.  Longer batches are timed back to back (their own
// footprint evicts the caches).
rl_status time_config(rl_batch* b, const Config& c, hipStream_t s, const FlushBuffer& flush, double* us) {
  rl_status st = resolve_widths(b, c.width);
  if (!st) st = plan_all(b, c);
  DeviceTables d;
  if (!st) st = build_tables(b, c, &d);
  if (st) { d.release(); return st; }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  for (int k = 0; k < 2 && !st; ++k) st = launch_tables(d, c, s);
  int reps = 5;
  float ms = 0;
  (void)hipEventRecord(e0, s);
  for (int k = 0; k < reps && !st; ++k) st = launch_tables(d, c, s);
  (void)hipEventRecord(e1, s);
  hipError_t e = hipEventSynchronize(e1);
  if (!st && e != hipSuccess) st = hip_fail(e, "tuning run");
  if (!st) (void)hipEventElapsedTime(&ms, e0, e1);
  if (!st && flush.mem && ms < 0.1f * reps) {
    constexpr int kCold = 16;
    hipEvent_t ev[2 * kCold];
    for (hipEvent_t& x : ev) (void)hipEventCreate(&x);
    const uint64_t half = flush.bytes / 2;
    for (int k = 0; k < kCold && !st; ++k) {
      hipError_t fe = launch_copy(static_cast<uint8_t*>(flush.mem) + half, flush.mem, half, s);
      if (fe != hipSuccess) st = hip_fail(fe, "tuning flush");
      (void)hipEventRecord(ev[2 * k], s);
      if (!st) st = launch_tables(d, c, s);
      (void)hipEventRecord(ev[2 * k + 1], s);
    }
    e = hipEventSynchronize(ev[2 * kCold - 1]);
    if (!st && e != hipSuccess) st = hip_fail(e, "tuning run");
    ms = 0;
    for (int k = 0; k < kCold && !st; ++k) {
      float one = 0;
      (void)hipEventElapsedTime(&one, ev[2 * k], ev[2 * k + 1]);
      ms += one;
    }
    reps = kCold;
    for (hipEvent_t& x : ev) (void)hipEventDestroy(x);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  d.release();
  *us = ms * 1000.0 / reps;
  return st;
}

// Whether two items convert the same source view (candidates for a
// fan-out group; build_tables decides which steps qualify).
static bool has_fanout(const rl_batch* b) {
  for (size_t i = 0; i < b->items.size(); ++i)
    for (size_t k = i + 1; k < b->items.size(); ++k) {
      const Item& x = b->items[i];
      const Item& y = b->items[k];
      if (x.src_layout == y.src_layout && x.n == y.n && x.src_bufs == y.src_bufs) return true;
    }
  return false;
}

rl_status autotune(rl_batch* b, hipStream_t s, Config* best) {
  FlushBuffer flush;
  if (hipMalloc(&flush.mem, kFlushBytes) == hipSuccess) {
    flush.bytes = kFlushBytes;
  } else {
    flush.mem = nullptr;   // timed warm: still a valid comparison
    (void)hipGetLastError();
  }
  struct Free {
    FlushBuffer& f;
    hipStream_t s;
    ~Free() {
      if (f.mem) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(f.mem);
      }
    }
  } free_flush{flush, s};
  const bool any_auto = std::any_of(b->items.begin(), b->items.end(), [](const Item& i) { return i.auto_width(); });
  double best_us = 1e30;
  Config bc;
  std::vector<std::pair<double, Config>> seen;   // every shape candidate timed
  for (uint32_t tile : {64u, 128u, 256u, 512u, 1024u})
    for (uint32_t threads : {64u, 128u, 256u})
      // 0: as many work-groups as fit at once (persistent); kOnePerTile: one
      // work-group per tile (the dispatcher balances uneven tiles)
      for (uint32_t grid : {0u, 1024u, 2048u, 4096u, 8192u, kOnePerTile})
        // double-buffered work-groups need more than one tile each
        for (uint32_t pipe : {0u, 1u}) {
          if (threads > 2 * tile) continue;   // at least half the threads hold an object
          if (pipe && grid == kOnePerTile) continue;
          Config c;
          c.tile = tile;
          c.threads = threads;
          c.grid = grid;
          c.width = 64;
          c.pipe = pipe;
          double us;
          rl_status st = time_config(b, c, s, flush, &us);
          if (st) return st;
          seen.emplace_back(us, c);
          if (us < best_us) { best_us = us; bc = c; }
        }
  // member gathers: one-wave work-groups keep more sub-tiles in flight,
  // larger ones fewer instructions per member
  if (std::any_of(b->items.begin(), b->items.end(), [](const Item& i) { return !i.src_layout->schema->members.empty(); }))
    for (uint32_t gt : {64u, 256u}) {
      Config c = bc;
      c.gather_threads = gt;
      double us;
      rl_status st = time_config(b, c, s, flush, &us);
      if (st) return st;
      if (us < best_us * 0.98) { best_us = us; bc = c; }
    }
  // steps sharing a source: one work-group per source tile for all of them
  if (has_fanout(b)) {
    const Config base = bc;
    for (uint32_t tile : {64u, 128u, 256u, 512u}) {
      // threads per destination: a tile in one pass of two objects per
      // thread, 64 to 128 (on the step, 64 and 128 at 256 objects per tile
      // time within the tuner's noise of each other, while 128 is 4% faster
      // in back-to-back launches over cold data)
      const uint32_t per = std::min(128u, std::max(64u, tile / 2));
      // double-buffered: work-groups that convert two or more tiles each
      for (uint32_t pipe : {0u, 1u})
        for (uint32_t grid : {0u, 256u, 512u}) {
          if (!pipe && grid) continue;
          Config c = base;
          c.tile = tile;
          c.fanout = per;
          c.pipe = pipe;
          c.grid = grid;
          double us;
          rl_status st = time_config(b, c, s, flush, &us);
          if (st) return st;
          seen.emplace_back(us, c);
          if (us < best_us * 0.98) { best_us = us; bc = c; }
        }
    }
  }
  // ordinary stores for the values of direct destinations (non-temporal
  // ones help a few conversions of one source and cost the 512-collection
  // batch 5%)
  {
    Config c = bc;
    c.stream = 0;
    double us;
    rl_status st = time_config(b, c, s, flush, &us);
    if (st) return st;
    seen.emplace_back(us, c);
    if (us < best_us * 0.98) { best_us = us; bc = c; }
  }
  // the three fastest shapes timed twice more, interleaved: single timings
  // of shapes within a few percent of each other order them at random
  {
    std::sort(seen.begin(), seen.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
    const size_t top = std::min<size_t>(3, seen.size());
    if (top > 1) {
      std::vector<double> sum(top);
      for (size_t i = 0; i < top; ++i) {
        seen[i].second.gather_threads = bc.gather_threads;
        sum[i] = seen[i].first;
      }
      for (int round = 0; round < 2; ++round)
        for (size_t i = 0; i < top; ++i) {
          double us;
          rl_status st = time_config(b, seen[i].second, s, flush, &us);
          if (st) return st;
          sum[i] += us;
        }
      const size_t k = std::min_element(sum.begin(), sum.end()) - sum.begin();
      bc = seen[k].second;
      best_us = sum[k] / 3;
    }
  }
  if (any_auto)
    for (uint32_t w : kAutoWidths) {
      Config c = bc;
      c.width = w;
      double us;
      rl_status st = time_config(b, c, s, flush, &us);
      if (st) return st;
      if (us < best_us * 0.98) { best_us = us; bc = c; }
    }
  *best = bc;
  b->tuned_us = best_us;
  return RL_OK;
}

// The captured graph of the batch kernels for launches on stream `s`
// (captured on first use for the status word of `s`).
rl_status graph_for(rl_batch* b, hipStream_t s, hipGraphExec_t* out) {
  uint32_t* status = stream_status(s);
  if (!status) return fail(RL_EHIP, "status words of the current device");
  auto it = b->graphs.find(status);
  if (it != b->graphs.end()) {
    *out = it->second.second;
    return RL_OK;
  }
  hipError_t e;
  if (!b->cap && (e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess)
    return hip_fail(e, "stream");
  if ((e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return hip_fail(e, "hipStreamBeginCapture");
  rl_status st = launch_tables(b->dev, b->cfg, b->cap, status);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->cap, &g);
  if (st) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  hipGraphExec_t x = nullptr;
  if ((e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0)) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(e, "hipGraphInstantiate");
  }
  b->graphs[status] = {g, x};
  *out = x;
  return RL_OK;
}

// Reject batches in which an item writes memory that another item reads or
// writes: the items of one launch run at the same time, in no order.
// Sources shared between items (read-only) are allowed.
rl_status check_items_disjoint(const rl_batch* b) {
  struct R {
    uintptr_t lo, hi;
    size_t item;
    bool dst;
  };
  std::vector<R> rs;
  for (size_t k = 0; k < b->items.size(); ++k) {
    const Item& it = b->items[k];
    if (!it.n) continue;
    std::vector<Range> s, d;
    rl_view sv = it.src_view(), dv = it.dst_view();
    if (validate_view(&sv, it.n, "src", &s, true) || validate_view(&dv, it.n, "dst", &d, true))
      return RL_EINVAL;
    for (const auto& r : s) rs.push_back({r.lo, r.hi, k, false});
    for (const auto& r : d) rs.push_back({r.lo, r.hi, k, true});
  }
  std::sort(rs.begin(), rs.end(), [](const R& a, const R& b) { return a.lo < b.lo; });
  // sweep: every range against the earlier ones still open at its start
  std::vector<const R*> open;
  for (const R& r : rs) {
    size_t w = 0;
    for (size_t j = 0; j < open.size(); ++j)
      if (open[j]->hi > r.lo) open[w++] = open[j];
    open.resize(w);
    for (const R* o : open)
      if (o->item != r.item && (o->dst || r.dst))
        return fail(RL_EOVERLAP, "batch items %zu and %zu: a destination overlaps the other item's buffers",
                    std::min(o->item, r.item), std::max(o->item, r.item));
    open.push_back(&r);
  }
  return RL_OK;
}

// Time graph replay against direct launches of the chosen configuration.
rl_status choose_launch(rl_batch* b, hipStream_t s) {
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  float ms[2] = {0, 0};
  const int reps = 10;
  for (int mode = 0; mode < 2; ++mode) {
    for (int k = 0; k < reps + 2; ++k) {
      if (k == 2) (void)hipEventRecord(e0, s);
      rl_status st = RL_OK;
      if (mode == 0) {
        hipGraphExec_t x = nullptr;
        if ((st = graph_for(b, s, &x))) return st;
        const hipError_t e = hipGraphLaunch(x, s);
        if (e != hipSuccess) return hip_fail(e, "tuning launch");
      } else if ((st = launch_tables(b->dev, b->cfg, s))) {
        return st;
      }
    }
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    (void)hipEventElapsedTime(&ms[mode], e0, e1);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->cfg.direct = ms[1] < ms[0] * 0.97 ? 1 : 0;
  return RL_OK;
}

}  // namespace

extern "C" rl_status rl_batch_create(const rl_batch_opts* opts, rl_batch** out) {
  if (!out) return fail(RL_EINVAL, "rl_batch_create: out is NULL");
  auto* b = new rl_batch();
  if (opts) {
    b->autotune = opts->autotune;
    if (opts->tune_cache) b->cache = opts->tune_cache;
  }
  if (b->cache.empty())
    if (const char* p = getenv("RL_TUNE_CACHE")) b->cache = p;
  *out = b;
  return RL_OK;
}

extern "C" rl_status rl_batch_add(rl_batch* b, const rl_view* src, const rl_view* dst, uint64_t n) {
  if (!b) return fail(RL_EINVAL, "batch is NULL");
  if (b->finalized) return fail(RL_EBUSY, "batch already finalized");
  std::vector<Range> rs, rd;
  rl_status st = validate_view(src, n, "src", &rs, true);
  if (st) return st;
  if ((st = validate_view(dst, n, "dst", &rd, true))) return st;
  if (src->layout->schema != dst->layout->schema) return fail(RL_EINVAL, "src and dst use different schemas");
  if (src->layout->kind == RL_STRIDED || dst->layout->kind == RL_STRIDED)
    return fail(RL_EUNSUPPORTED, "batches do not take strided layouts (use rl_convert)");
  if ((st = check_overlap(rs, rd))) return st;
  if (src->layout->kind == RL_AOSOA && src->layout->width == 0)
    return fail(RL_EINVAL, "a source block width cannot be auto");
  if (!src->layout->schema->members.empty() && src->layout->kind == RL_AOS && dst->layout->kind == RL_AOS)
    return fail(RL_EUNSUPPORTED, "AoS -> AoS conversion of a schema with jagged groups");
  Item it;
  it.src_layout = src->layout;
  it.dst_layout = dst->layout;
  it.src_cap = src->capacity;
  it.dst_cap = dst->capacity;
  it.n = n;
  it.src_bufs.assign(src->buffers, src->buffers + layout_n_buffers(src->layout));
  it.dst_bufs.assign(dst->buffers, dst->buffers + layout_n_buffers(dst->layout));
  const size_t ng = src->layout->schema->members.size();
  if (ng) {
    it.src_mcap.assign(src->member_capacity, src->member_capacity + ng);
    it.dst_mcap.assign(dst->member_capacity, dst->member_capacity + ng);
  }
  b->items.push_back(std::move(it));
  return RL_OK;
}

extern "C" rl_status rl_batch_finalize(rl_batch* b, void* stream) {
  if (!b) return fail(RL_EINVAL, "batch is NULL");
  if (b->finalized) return fail(RL_EBUSY, "batch already finalized");
  hipStream_t s = (hipStream_t)stream;
  if (rl_status st0 = check_items_disjoint(b)) return st0;
  Config c;
  const std::string sig = signature(b);
  bool have = false;
  if (b->autotune) {
    rl_status st = autotune(b, s, &c);
    if (st) return st;
    have = true;
  } else if (!b->cache.empty()) {
    have = cache_lookup(b->cache, sig, &c);
  }
  (void)have;
  if (const char* v = getenv("RL_BATCH_TILE")) c.tile = (uint32_t)strtoul(v, nullptr, 10);
  if (const char* v = getenv("RL_BATCH_GRID")) c.grid = (uint32_t)strtoul(v, nullptr, 10);
  if (const char* v = getenv("RL_BATCH_THREADS")) c.threads = (uint32_t)strtoul(v, nullptr, 10);
  if (const char* v = getenv("RL_BATCH_GATHER_THREADS")) c.gather_threads = (uint32_t)strtoul(v, nullptr, 10);
  if (const char* v = getenv("RL_BATCH_PIPE")) c.pipe = (uint32_t)strtoul(v, nullptr, 10) ? 1 : 0;
  if (const char* v = getenv("RL_BATCH_STREAM")) c.stream = (uint32_t)strtoul(v, nullptr, 10) ? 1 : 0;
  if (const char* v = getenv("RL_BATCH_FANOUT")) {
    const uint32_t f = (uint32_t)strtoul(v, nullptr, 10);
    c.fanout = f == 0 ? 0 : f >= 128 ? 128 : 64;
  }
  if (c.threads < 64 || c.threads > kDenseMaxThreads || c.threads % 64) c.threads = 128;
  if (c.gather_threads < 64 || c.gather_threads > 256 || c.gather_threads % 64) c.gather_threads = kGatherThreads;

  b->cfg = c;
  rl_status st = resolve_widths(b, c.width);
  if (!st) st = plan_all(b, c);
  if (!st) st = build_tables(b, c, &b->dev);
  if (st) return st;
  hipGraphExec_t x = nullptr;
  if ((st = graph_for(b, s, &x))) return st;
  if (b->autotune) {
    if ((st = choose_launch(b, s))) return st;
    if (!b->cache.empty()) cache_store(b->cache, sig, b->cfg, b->tuned_us);
  }
  b->finalized = true;
  return RL_OK;
}

extern "C" rl_status rl_batch_launch(rl_batch* b, void* stream) {
  if (!b || !b->finalized) return fail(RL_EINVAL, "batch not finalized");
  if (!b->dev.t.dense_tiles && !b->dev.t.fan_tiles && !b->dev.t.gather_tiles && !b->dev.t.n_totals &&
      !b->dev.t.rebase_tiles)
    return RL_OK;
  if (b->cfg.direct) return launch_tables(b->dev, b->cfg, (hipStream_t)stream);
  hipGraphExec_t x = nullptr;
  if (rl_status st = graph_for(b, (hipStream_t)stream, &x)) return st;
  hipError_t e = hipGraphLaunch(x, (hipStream_t)stream);
  return e == hipSuccess ? RL_OK : hip_fail(e, "hipGraphLaunch");
}

extern "C" rl_status rl_batch_launch_loop(rl_batch* b, void* stream) {
  if (!b || !b->finalized) return fail(RL_EINVAL, "batch not finalized");
  for (const Plan& p : b->plans) {
    rl_status st = enqueue_plan(p, (hipStream_t)stream);
    if (st) return st;
  }
  return RL_OK;
}

extern "C" rl_status rl_batch_item_width(const rl_batch* b, uint32_t item, uint32_t* w) {
  if (!b || !w) return fail(RL_EINVAL, "NULL argument");
  if (!b->finalized) return fail(RL_EINVAL, "batch not finalized");
  if (item >= b->items.size()) return fail(RL_EINVAL, "no item %u", item);
  const rl_layout* L = b->items[item].resolved ? b->items[item].resolved.get() : b->items[item].dst_layout;
  *w = L->kind == RL_AOSOA ? L->width : 0;
  return RL_OK;
}

extern "C" rl_status rl_batch_shape(const rl_batch* b, uint32_t* tile, uint32_t* threads, uint32_t* grid,
                                    uint32_t* graph_replay) {
  if (!b) return fail(RL_EINVAL, "batch is NULL");
  if (tile) *tile = b->cfg.tile;
  if (!b->dev.t.dense_tiles && b->dev.t.fan_tiles) {
    // every dense step is in a fan-out group: the fan-out kernel's launch
    if (threads) *threads = b->dev.fan_threads;
    if (grid) {
      const uint32_t r = fanout_resident_blocks(b->dev.fan_threads, b->dev.fan_lds, b->dev.t.fan_slot != 0);
      *grid = std::min<uint32_t>(b->cfg.grid ? b->cfg.grid : (r ? r : 2048), b->dev.t.fan_tiles);
    }
    if (graph_replay) *graph_replay = b->cfg.direct ? 0 : 1;
    return RL_OK;
  }
  if (threads) *threads = b->cfg.threads;
  if (grid) {
    // dense work-groups as launched: the configured count or as many as fit
    // at once, at most one per tile
    const uint32_t g = b->cfg.grid ? b->cfg.grid
                                   : batch_resident_blocks(std::min<uint32_t>(b->cfg.threads, kDenseMaxThreads),
                                                           b->dev.dense_lds, b->dev.t.pipe_slot != 0);
    *grid = std::min<uint32_t>(g, std::max(1u, b->dev.t.dense_tiles));
  }
  if (graph_replay) *graph_replay = b->cfg.direct ? 0 : 1;
  return RL_OK;
}

extern "C" rl_status rl_batch_get_info(const rl_batch* b, rl_batch_info* info) {
  if (!b || !info) return fail(RL_EINVAL, "NULL argument");
  if (!b->finalized) return fail(RL_EINVAL, "batch not finalized");
  *info = rl_batch_info{};
  info->double_buffered = b->dev.t.pipe_slot != 0 || b->dev.t.fan_slot != 0;
  info->fanout_threads = b->dev.t.fan_tiles ? b->dev.t.fan_per : 0;
  info->fanout_groups = b->dev.fan_groups;
  info->fanout_steps = b->dev.fan_steps;
  info->dense_steps = b->dev.dense_steps;
  info->stream_stores = b->cfg.stream;
  return RL_OK;
}

extern "C" void rl_batch_destroy(rl_batch* b) {
  if (!b) return;
  if (b->finalized) (void)hipDeviceSynchronize();
  delete b;
}
