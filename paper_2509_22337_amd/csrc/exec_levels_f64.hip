// LEVELS and HYBRID executors instantiated for float64 messages.
#include "exec.h"

namespace fastlbp {

void levels_run_f64(fastlbp_graph *g, int32_t max_iters, double tol, double damping, bool fuse, bool plain) {
    levels_run<PolLin64>(g, max_iters, tol, damping, fuse, plain);
}

void levels_step_f64(fastlbp_graph *g, double damping, int32_t iters) { step_levels_p<PolLin64>(g, damping, iters); }

void init_beliefs_f64(fastlbp_graph *g) { launch_init_beliefs<PolLin64>(g, g->view<PolLin64>(0.0)); }

}  // namespace fastlbp
