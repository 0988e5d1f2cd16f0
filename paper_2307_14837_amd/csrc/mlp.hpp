// Shared constants of the patch-network kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "dnnmg.h"

namespace dnnmg {

constexpr int N_IN = 165;   // 81 velocities + 81 residuals + 3 cell sizes
constexpr int N_OUT = 81;   // 27 nodes x 3 velocity components
constexpr int IN_PAD = 192; // N_IN rounded up to the MFMA K granule
constexpr int OUT_PAD = 96; // N_OUT rounded up to 16-row output tiles

// Input and output widths of the patch network for a prediction J levels
// above the coarse mesh (Sec. 4.2): a patch of 2^J x 2^J x 2^J fine cells has
// (2^J + 1)^3 nodes; inputs are 3 velocities and 3 momentum residuals per
// node plus 3 cell sizes, outputs 3 velocities per node.
template <int J> struct NetIo;
template <> struct NetIo<1> {
    static constexpr int NIN = N_IN, NOUT = N_OUT, INP = IN_PAD, OUTP = OUT_PAD;
};
template <> struct NetIo<2> {
    static constexpr int NIN = 753, NOUT = 375, INP = 768, OUTP = 384;
};
// J of a network description by its widths (0: not a supported shape)
inline int net_levels(int n_in, int n_out) {
    if (n_in == NetIo<1>::NIN && n_out == NetIo<1>::NOUT) return 1;
    if (n_in == NetIo<2>::NIN && n_out == NetIo<2>::NOUT) return 2;
    return 0;
}
inline int io_in_pad(int J) { return J == 2 ? NetIo<2>::INP : NetIo<1>::INP; }
inline int io_out_pad(int J) { return J == 2 ? NetIo<2>::OUTP : NetIo<1>::OUTP; }

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
