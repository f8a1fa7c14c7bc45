// LEVELS and HYBRID executors instantiated for float32 log-domain messages.
#include "exec.h"

namespace fastlbp {

void levels_run_f32(fastlbp_graph *g, int32_t max_iters, double tol, double damping, bool fuse, bool plain) {
    levels_run<PolLog32>(g, max_iters, tol, damping, fuse, plain);
}

void levels_step_f32(fastlbp_graph *g, double damping, int32_t iters) { step_levels_p<PolLog32>(g, damping, iters); }

void init_beliefs_f32(fastlbp_graph *g) { launch_init_beliefs<PolLog32>(g, g->view<PolLog32>(0.0)); }

}  // namespace fastlbp
