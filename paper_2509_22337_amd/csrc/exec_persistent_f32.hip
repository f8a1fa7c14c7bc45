// Persistent executor instantiated for float32 log-domain messages.
#include "exec.h"

namespace fastlbp {

void persistent_launch_f32(Launcher &lc, int n, fastlbp_graph *const *gs, const double *damping, int32_t step,
                           const FixedArea *fixed, const int32_t *steps) {
    launch_persistent<PolLog32>(lc, n, gs, damping, step, fixed, steps);
}

}  // namespace fastlbp
