// Extension operator L of DNN-MG (arXiv 2307.14837, eq. (defL)): the value
// at a fine node is the average of the network outputs of the patches that
// hold the node (multiplicity 1, 2, 4 or 8); velocity rows on Dirichlet faces
// are 0.
#pragma once

#include "common.hpp"

namespace dnnmg {

// Patches holding fine index i along one axis (n patches, periodic or not):
// up to two, in ascending patch order, with the node's local index 0..2.
struct Hold1 {
    int P[2];
    int loc[2];
    float w[2];
    int cnt;
};

__device__ __forceinline__ Hold1 holders(int i, int n, int per) {
    Hold1 h;
    if (i & 1) {
        h.P[0] = h.P[1] = (i - 1) >> 1;
        h.loc[0] = h.loc[1] = 1;
        h.w[0] = 1.f;
        h.w[1] = 0.f;
        h.cnt = 1;
        return h;
    }
    int hi = i >> 1;   // patch starting here (local 0)
    int lo = hi - 1;   // patch ending here (local 2)
    if (per) {
        if (lo < 0) lo += n;
        bool lo_first = lo < hi; // ascending patch order
        h.P[0] = lo_first ? lo : hi;
        h.loc[0] = lo_first ? 2 : 0;
        h.P[1] = lo_first ? hi : lo;
        h.loc[1] = lo_first ? 0 : 2;
        h.w[0] = h.w[1] = 1.f;
        h.cnt = 2;
        return h;
    }
    bool has_lo = lo >= 0, has_hi = hi < n;
    h.P[0] = has_lo ? lo : hi;
    h.loc[0] = has_lo ? 2 : 0;
    h.P[1] = has_hi ? hi : h.P[0];
    h.loc[1] = has_hi ? 0 : h.loc[0];
    h.w[0] = 1.f;
    h.w[1] = (has_lo && has_hi) ? 1.f : 0.f;
    h.cnt = (int)has_lo + (int)has_hi;
    return h;
}


// d = L(Y) at fine node (i, j, k): Y FP32 [n_patches][81] (27 nodes x u, v, w).
__device__ __forceinline__ void extension_at(const Mesh &m, int i, int j, int k, const float *__restrict__ Y,
                                             float out[3]) {
    float acc[3] = {0.0f, 0.0f, 0.0f};
    const bool dir = on_dirichlet(m, i, j, k);
    Hold1 hx = holders(i, m.n[0], m.per[0]);
    Hold1 hy = holders(j, m.n[1], m.per[1]);
    Hold1 hz = holders(k, m.n[2], m.per[2]);
    float y[8][3], wgt[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        int a = q & 1, b = (q >> 1) & 1, c = q >> 2;
        int64_t M = hx.P[a] + (int64_t)m.n[0] * (hy.P[b] + (int64_t)m.n[1] * hz.P[c]);
        int iota = hx.loc[a] + 3 * hy.loc[b] + 9 * hz.loc[c];
        const float *src = Y + M * 81 + iota;
        y[q][0] = src[0];
        y[q][1] = src[27];
        y[q][2] = src[54];
        wgt[q] = hx.w[a] * hy.w[b] * hz.w[c];
    }
    // sum in ascending patch order (z, then y, then x of the candidates)
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) acc[cc] = fmaf(wgt[q], y[q][cc], acc[cc]);
    const float inv = 1.0f / (float)(hx.cnt * hy.cnt * hz.cnt); // power of two: exact
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c] = dir ? 0.0f : acc[c] * inv;
}

} // namespace dnnmg
