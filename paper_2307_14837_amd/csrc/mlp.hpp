// Shared constants of the patch-network kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "dnnmg.h"

namespace dnnmg {

constexpr int N_IN = 165;   // 81 velocities + 81 residuals + 3 cell sizes
constexpr int N_OUT = 81;   // 27 nodes x 3 velocity components
constexpr int IN_PAD = 192; // N_IN rounded up to the MFMA K granule
constexpr int OUT_PAD = 96; // N_OUT rounded up to 16-row output tiles

int check_net(const dnnmg_mlp *net);

struct BoxDesc;
// Forward pass of the patch network over tiles of 16 pt patches (one
// workgroup per tile, persistent when 0 < grid < ntiles).  gather = false:
// inputs are the rows of X [n_rows][ldx]; gather = true: inputs are gathered
// from the node fields xt, r of the boxes D (or of `one` when D is null).
int fwd_launch(const dnnmg_mlp *net, int pt, bool gather, int64_t ntiles, int grid, int64_t n_rows,
               const void *X, int64_t ldx, const BoxDesc *D, int nbox, const BoxDesc &one, const float *xt,
               const float *r, const float *shift, const float *inv, float *Y, void *saved, hipStream_t s);
bool fwd_has_pt(const dnnmg_mlp *net, int pt);
int fwd_default_pt(const dnnmg_mlp *net, int64_t n, int ncu);
int device_cus();

} // namespace dnnmg
