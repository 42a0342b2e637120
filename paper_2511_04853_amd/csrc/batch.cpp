// Batched conversion (placeholder entry points until the batch engine lands).
#include "plan.h"
#include "rl_internal.h"

using namespace rl;

struct rl_batch {
  int unused;
};

extern "C" rl_status rl_batch_create(const rl_batch_opts*, rl_batch** out) {
  if (out) *out = nullptr;
  return fail(RL_EUNSUPPORTED, "batches are not available yet");
}
extern "C" rl_status rl_batch_add(rl_batch*, const rl_view*, const rl_view*, uint64_t) { return fail(RL_EUNSUPPORTED, "batches"); }
extern "C" rl_status rl_batch_finalize(rl_batch*, void*) { return fail(RL_EUNSUPPORTED, "batches"); }
extern "C" rl_status rl_batch_launch(rl_batch*, void*) { return fail(RL_EUNSUPPORTED, "batches"); }
extern "C" rl_status rl_batch_launch_loop(rl_batch*, void*) { return fail(RL_EUNSUPPORTED, "batches"); }
extern "C" rl_status rl_batch_item_width(const rl_batch*, uint32_t, uint32_t*) { return fail(RL_EUNSUPPORTED, "batches"); }
extern "C" rl_status rl_batch_shape(const rl_batch*, uint32_t*, uint32_t*, uint32_t*) { return fail(RL_EUNSUPPORTED, "batches"); }
extern "C" void rl_batch_destroy(rl_batch*) {}
