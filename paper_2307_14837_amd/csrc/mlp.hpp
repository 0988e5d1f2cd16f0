// Shared constants of the patch-network kernels.
#pragma once

#include "dnnmg.h"

namespace dnnmg {

constexpr int N_IN = 165;   // 81 velocities + 81 residuals + 3 cell sizes
constexpr int N_OUT = 81;   // 27 nodes x 3 velocity components
constexpr int IN_PAD = 192; // N_IN rounded up to the MFMA K granule
constexpr int OUT_PAD = 96; // N_OUT rounded up to 16-row output tiles

int check_net(const dnnmg_mlp *net);

} // namespace dnnmg
