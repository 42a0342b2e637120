// User transfer specialisations (Sec. VII-B: transfers between layouts can
// be given more optimal implementations by the user, or read pre-existing
// structures defined outside the library, with a priority that lets a
// specialisation fall back to more general ones): a registry of callbacks
// per (source layout, destination layout) consulted by rl_convert and
// rl_transfer before the library's own implementation.
#include <algorithm>
#include <atomic>
#include <mutex>
#include <vector>

#include "plan.h"
#include "rl_internal.h"

namespace rl {

namespace {

struct Spec {
  uint64_t id;
  const rl_layout* src;   // null: any
  const rl_layout* dst;   // null: any
  const rl_schema* schema;
  int32_t priority;
  rl_transfer_fn fn;
  void* user;
};

std::mutex g_spec_mu;
std::vector<Spec> g_specs;   // sorted by priority (high first), then registration
std::atomic<size_t> g_n_specs{0};
uint64_t g_next_id = 1;
// set while this thread runs a user transfer: the transfers it calls go to
// the library's own implementation (no recursion into the registry)
thread_local bool t_in_spec = false;

}  // namespace

// Run the matching specialisations in priority order; *handled is set when
// one of them took the call (its status is returned).
rl_status run_specialisations(const rl_view* src, const rl_view* dst, uint64_t n, void* stream, bool* handled) {
  *handled = false;
  if (t_in_spec || g_n_specs.load(std::memory_order_acquire) == 0) return RL_OK;
  std::vector<Spec> match;
  {
    std::lock_guard<std::mutex> lk(g_spec_mu);
    for (const Spec& s : g_specs)
      if ((!s.src || s.src == src->layout) && (!s.dst || s.dst == dst->layout) &&
          s.schema == src->layout->schema)
        match.push_back(s);
  }
  for (const Spec& s : match) {
    t_in_spec = true;
    const rl_status st = s.fn(src, dst, n, stream, s.user);
    t_in_spec = false;
    if (st == RL_EUNSUPPORTED) continue;   // declined: the next one, then the library's own
    *handled = true;
    if (st != RL_OK) return fail(st, "user transfer %llu failed with status %d", (unsigned long long)s.id, (int)st);
    return RL_OK;
  }
  return RL_OK;
}

}  // namespace rl

using namespace rl;

extern "C" rl_status rl_register_transfer(const rl_layout* src, const rl_layout* dst, int32_t priority,
                                          rl_transfer_fn fn, void* user, uint64_t* id) {
  if (!fn) return fail(RL_EINVAL, "rl_register_transfer: fn is NULL");
  if (!src && !dst) return fail(RL_EINVAL, "rl_register_transfer: a source or a destination layout is needed");
  if (src && dst && src->schema != dst->schema) return fail(RL_EINVAL, "layouts of different schemas");
  std::lock_guard<std::mutex> lk(g_spec_mu);
  Spec s{g_next_id++, src, dst, src ? src->schema : dst->schema, priority, fn, user};
  auto at = std::find_if(g_specs.begin(), g_specs.end(), [&](const Spec& o) { return o.priority < priority; });
  g_specs.insert(at, s);
  g_n_specs.store(g_specs.size(), std::memory_order_release);
  if (id) *id = s.id;
  return RL_OK;
}

extern "C" rl_status rl_unregister_transfer(uint64_t id) {
  std::lock_guard<std::mutex> lk(g_spec_mu);
  auto it = std::find_if(g_specs.begin(), g_specs.end(), [&](const Spec& o) { return o.id == id; });
  if (it == g_specs.end()) return fail(RL_EINVAL, "no user transfer %llu", (unsigned long long)id);
  g_specs.erase(it);
  g_n_specs.store(g_specs.size(), std::memory_order_release);
  return RL_OK;
}
