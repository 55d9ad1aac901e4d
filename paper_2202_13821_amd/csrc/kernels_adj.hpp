// kernels_adj.hpp -- reverse-mode (adjoint) kernels of the S2O4 step.
#pragma once

#include "kernels_fwd.hpp"

namespace dgk {

// Number of per-block partial sums of dJ/dmu kept in the workspace.
inline size_t adj_mu_slots(size_t ncell) { return 3 * ncell + 64; }

}  // namespace dgk
