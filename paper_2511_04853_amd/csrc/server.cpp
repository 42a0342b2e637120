// Serving loop (placeholder entry points until the server lands).
#include "plan.h"
#include "rl_internal.h"

using namespace rl;

struct rl_server {
  int unused;
};

extern "C" rl_status rl_server_create(const rl_server_opts*, rl_server** out) {
  if (out) *out = nullptr;
  return fail(RL_EUNSUPPORTED, "serving is not available yet");
}
extern "C" rl_status rl_server_submit(rl_server*, const rl_event*, uint64_t*) { return fail(RL_EUNSUPPORTED, "serving"); }
extern "C" rl_status rl_server_wait(rl_server*, uint64_t, int64_t, rl_event_result*) { return fail(RL_EUNSUPPORTED, "serving"); }
extern "C" rl_status rl_server_release(rl_server*, uint64_t) { return fail(RL_EUNSUPPORTED, "serving"); }
extern "C" rl_status rl_server_stats_get(rl_server*, rl_server_stats*) { return fail(RL_EUNSUPPORTED, "serving"); }
extern "C" void rl_server_destroy(rl_server*) {}
