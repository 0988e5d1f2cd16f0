// Internal helpers shared by the HIP translation units of libdnnmg.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "dnnmg.h"

namespace dnnmg {

// ------------------------------------------------------------ error state --
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_check(hipError_t e, const char *what);

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// ------------------------------------------------------------------- mesh --
// Unsigned 32-bit division by a runtime constant: q = floor(n / d) for
// n < 2^31, via a 32x32 high multiply (round-up reciprocal method).
struct FastDiv {
    uint32_t d, m, s;
};
FastDiv make_fastdiv(uint32_t d);

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f) {
    uint32_t hi = __umulhi(n, f.m);
    return (uint32_t)(((uint64_t)hi + n) >> f.s);
}

// Two-level structured mesh in the form the kernels use.  Fine node
// (i,j,k) -> i + nf[0] (j + nf[1] k); coarse likewise with nc.
struct Mesh {
    int32_t n[3];   // coarse cells per axis
    int32_t nf[3];  // fine nodes per axis
    int32_t nc[3];  // coarse nodes per axis
    int32_t per[3]; // periodic axis flags
    uint32_t dmask; // Dirichlet face bits (2a low, 2a+1 high)
    int64_t n_fine, n_coarse, n_patches;
    float h[3];     // fine cell sizes
    float H[3];     // coarse cell sizes
    double hd[3];
    FastDiv fx, fy, cx, cy, px, py; // fine/coarse/patch lattice divisors
};

// Validates the box (positive sizes, even n >= 2 on periodic axes, node
// counts below 2^31) and fills the kernel description.
int make_mesh(const dnnmg_box *box, Mesh *m);

__device__ __forceinline__ int wrap(int i, int N, int per) {
    if (per) {
        if (i < 0) i += N;
        else if (i >= N) i -= N;
    }
    return i;
}

__device__ __forceinline__ bool on_dirichlet(const Mesh &m, int i, int j, int k) {
    int c[3] = {i, j, k};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (m.per[a]) continue;
        if (c[a] == 0 && ((m.dmask >> (2 * a)) & 1u)) return true;
        if (c[a] == m.nf[a] - 1 && ((m.dmask >> (2 * a + 1)) & 1u)) return true;
    }
    return false;
}

// Workgroups go to the chip's 8 XCDs (each with its own L2) round-robin by
// workgroup index.  A launch of xcd_blocks(n) workgroups where workgroup b
// takes item xcd_item(b, gridDim) gives each XCD one contiguous range of
// items, so neighbouring tiles (which read each other's halos) share an L2.
constexpr int NXCD = 8;
inline unsigned xcd_blocks(int64_t n) { return (unsigned)(NXCD * ((n + NXCD - 1) / NXCD)); }
__device__ __forceinline__ int64_t xcd_item(int64_t b, int64_t nblocks) {
    return (b % NXCD) * (nblocks / NXCD) + b / NXCD;
}

inline unsigned blocks_for(int64_t n, int threads) {
    return (unsigned)((n + threads - 1) / threads);
}

// Crank-Nicolson / stabilisation constants of one box, in kernel form.
struct ResParams {
    float inv_dt, half_nu, alpha0, delta0, nu;
    float ih[3];
    float hT, wq; // cell diameter, quadrature weight |T| / 8
};

// One box of a batch of independent simulations.  Field arrays of a batch
// are the concatenation of the boxes' SoA blocks: box b's fine field with c
// components starts at c * off_fine, its coarse field at c * off_coarse, its
// patch rows at off_patch.  blk_* are the first block index of the box in
// each batched launch (prefix sums over the boxes).
struct BoxDesc {
    Mesh m;
    ResParams rp;
    int64_t off_fine, off_coarse, off_patch;
    int64_t blk_fine, blk_coarse, blk_ptile;
    int64_t blk_stile;          // extension (scatter) tiles: prefix sum over the boxes
    int64_t blk_full, blk_part; // residual tiles: prefix sums of full / partial tiles
    int32_t rtiles[3];          // residual tile grid of the box
    int32_t rfull[3];           // its box of full tiles (no node beyond the mesh)
    const float *geom;          // geometry inputs per patch [n_patches][3], or null: the box's cell sizes
};

// Box holding block `blk` of a batched launch: the last b with first[b] <= blk.
template <typename F>
__device__ __forceinline__ int find_box(int nbox, int64_t blk, F first) {
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (first(mid) <= blk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

} // namespace dnnmg
