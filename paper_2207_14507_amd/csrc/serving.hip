// Serving engine (submit / poll): continuous batching of videos.
#include "runtime.hpp"

namespace prnu {

struct ServingEngine {};
void ServingDeleter::operator()(ServingEngine* e) const { delete e; }

void Context::shutdown_serving() { serving.reset(); }
bool Context::fp_in_use(prnu_fp) { return false; }

}  // namespace prnu

using namespace prnu;

extern "C" {

prnu_status prnu_submit_video(prnu_ctx* ctx, prnu_fp, const prnu_frames*, const prnu_search_opts*, prnu_ticket* out) {
  if (!ctx || !out) return fail(PRNU_E_ARG, "null argument");
  return fail(PRNU_E_ARG, "serving engine not available");
}

prnu_status prnu_poll(prnu_ctx* ctx, prnu_ticket, int32_t, prnu_frame_result*, prnu_video_summary*) {
  if (!ctx) return fail(PRNU_E_ARG, "null argument");
  return fail(PRNU_E_HANDLE, "unknown ticket");
}

prnu_status prnu_cancel(prnu_ctx* ctx, prnu_ticket) {
  if (!ctx) return fail(PRNU_E_ARG, "null argument");
  return fail(PRNU_E_HANDLE, "unknown ticket");
}

}  // extern "C"
