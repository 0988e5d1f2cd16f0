// Prediction two levels above the coarse mesh (J = 2; arXiv 2307.14837,
// Sec. 4.2: the network predicts the correction on level L + J, and its
// patches are the coarse cells, each of 2^J x 2^J x 2^J fine cells).  With
// J = 2 a patch has 4 x 4 x 4 fine cells and 5^3 = 125 nodes (375 velocity
// unknowns).  Grid transfer spans two levels: prolongation L -> L + 2 and its
// transpose.  The residual, the right-hand side, the indicator and the
// fallback live on the fine mesh and use the one-level kernels on the box
// whose own fine mesh is level L + 2 (n doubled); their local projection is
// onto level L + 1, which does not depend on J.
//
// Lattices: `m` is the mesh of the coarse box (n cells, its coarse nodes are
// level L), `m2` the mesh of the doubled box (its coarse nodes are level
// L + 1, its fine nodes level L + 2).  Patch M = coarse cell (I, J, K), local
// node iota = a + 5 b + 25 c, fine node (4I + a, 4J + b, 4K + c).
#include <math.h>

#include "common.hpp"
#include "lowp.hpp"

namespace dnnmg {

constexpr int L2_SIDE = 5, L2_NODES = 125, L2_NIN = 753, L2_NOUT = 375;

// ------------------------------------------------- two-level prolongation --
// The value of the 2x-prolongation at offset (oa, ob, oc) in {0, 1}^3 of the
// 2x2x2 block v (v[a + 2b + 4c]): axis by axis, x then y then z, each
// midpoint 0.5 (a + b) in FP32.  These are the operations of the one-level
// prolongation kernel, so level L + 2 equals its own patch interpolant of
// level L + 1 bit for bit (the local projection terms vanish exactly).
__device__ __forceinline__ float interp2(const float v[8], int oa, int ob, int oc) {
    float X[4];
#pragma unroll
    for (int bc = 0; bc < 4; ++bc) X[bc] = oa ? 0.5f * (v[2 * bc] + v[2 * bc + 1]) : v[2 * bc];
    float Y[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) Y[c] = ob ? 0.5f * (X[2 * c] + X[2 * c + 1]) : X[2 * c];
    return oc ? 0.5f * (Y[0] + Y[1]) : Y[0];
}

// lower node of the 2x2x2 block and the offset (0: coincident, 1: midpoint)
// of lattice index i on the next-coarser lattice with Nc nodes; the upper
// node wraps on a periodic axis and is clamped where it is absent
__device__ __forceinline__ void coarse_pair(int i, int Nc, int per, int &lo, int &hi, int &off) {
    lo = i >> 1;
    off = i & 1;
    hi = lo + 1;
    if (per && hi == Nc) hi = 0;
    if (!off) hi = lo;
    if (hi >= Nc) hi = lo;
}

__global__ void __launch_bounds__(256) k_prolong2(Mesh m, Mesh m2, int ncomp, const double *__restrict__ xc,
                                                  float *__restrict__ xf) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)ncomp * m2.n_fine) return;
    const int comp = (int)(t / m2.n_fine);
    const int64_t node = t - (int64_t)comp * m2.n_fine;
    const uint32_t jk = fdiv((uint32_t)node, m2.fx), i = (uint32_t)node - jk * m2.nf[0];
    const uint32_t k = fdiv(jk, m2.fy), j = jk - k * m2.nf[1];
    const int f[3] = {(int)i, (int)j, (int)k};
    // level L + 1 nodes under this level L + 2 node, then the level L nodes
    // under each of those
    int lo1[3], hi1[3], off1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) coarse_pair(f[a], m2.nc[a], m2.per[a], lo1[a], hi1[a], off1[a]);
    const double *x = xc + (int64_t)comp * m.n_coarse;
    float v1[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int c1[3] = {(q & 1) ? hi1[0] : lo1[0], (q & 2) ? hi1[1] : lo1[1], (q & 4) ? hi1[2] : lo1[2]};
        int lo0[3], hi0[3], off0[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) coarse_pair(c1[a], m.nc[a], m.per[a], lo0[a], hi0[a], off0[a]);
        float v0[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int ii = (r & 1) ? hi0[0] : lo0[0], jj = (r & 2) ? hi0[1] : lo0[1], kk = (r & 4) ? hi0[2] : lo0[2];
            v0[r] = (float)x[ii + (int64_t)m.nc[0] * (jj + (int64_t)m.nc[1] * kk)];
        }
        v1[q] = interp2(v0, off0[0], off0[1], off0[2]);
    }
    xf[t] = interp2(v1, off1[0], off1[1], off1[2]);
}

// Row form of k_prolong2 (the same values, bit for bit): one workgroup per
// level L + 2 lattice row (j, k) and component.  The level L + 1 values of
// the (up to) 2 x 2 level L + 1 rows above it are formed once per x node
// (interp2 of their 8 level L corners, as k_prolong2 forms them per node)
// into LDS; each fine node of the row then interpolates its 8 level L + 1
// values from there.  LDS: 4 x (level L + 1 nodes along x) floats.
__global__ void __launch_bounds__(256) k_prolong2_rows(Mesh m, Mesh m2, const double *__restrict__ xc,
                                                       float *__restrict__ xf) {
    extern __shared__ float sV[]; // [y, z slot][level L + 1 x node]
    const int comp = blockIdx.y;
    const int64_t row = blockIdx.x;
    const int j = (int)(row % m2.nf[1]), k = (int)(row / m2.nf[1]);
    int lo1y, hi1y, offy, lo1z, hi1z, offz;
    coarse_pair(j, m2.nc[1], m2.per[1], lo1y, hi1y, offy);
    coarse_pair(k, m2.nc[2], m2.per[2], lo1z, hi1z, offz);
    const int nc1x = m2.nc[0];
    const double *x = xc + (int64_t)comp * m.n_coarse;
    for (int t = threadIdx.x; t < 4 * nc1x; t += blockDim.x) {
        const int yz = t / nc1x, x1 = t - yz * nc1x;
        const int c1[3] = {x1, (yz & 1) ? hi1y : lo1y, (yz & 2) ? hi1z : lo1z};
        int lo0[3], hi0[3], off0[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) coarse_pair(c1[a], m.nc[a], m.per[a], lo0[a], hi0[a], off0[a]);
        float v0[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int ii = (r & 1) ? hi0[0] : lo0[0], jj = (r & 2) ? hi0[1] : lo0[1], kk = (r & 4) ? hi0[2] : lo0[2];
            v0[r] = (float)x[ii + (int64_t)m.nc[0] * (jj + (int64_t)m.nc[1] * kk)];
        }
        sV[t] = interp2(v0, off0[0], off0[1], off0[2]);
    }
    __syncthreads();
    float *out = xf + (int64_t)comp * m2.n_fine + (int64_t)m2.nf[0] * (j + (int64_t)m2.nf[1] * k);
    for (int i = threadIdx.x; i < m2.nf[0]; i += blockDim.x) {
        int lo1x, hi1x, offx;
        coarse_pair(i, m2.nc[0], m2.per[0], lo1x, hi1x, offx);
        float v1[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v1[q] = sV[(q >> 1) * nc1x + ((q & 1) ? hi1x : lo1x)];
        out[i] = interp2(v1, offx, offy, offz);
    }
}

// --------------------------------------------------- two-level restriction --
// bc(I) = sum over fine indices i = 4I + d, |d| <= 3, of prod_a (1 - |d_a|/4)
// bf(i) (the transpose of the two-level Q1 prolongation), FP64 accumulation;
// absent fine nodes (beyond a non-periodic edge) carry weight 0.
__global__ void __launch_bounds__(256) k_restrict2(Mesh m, Mesh m2, int ncomp, const float *__restrict__ bf,
                                                   double *__restrict__ bc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)ncomp * m.n_coarse) return;
    const int comp = (int)(t / m.n_coarse);
    const int64_t node = t - (int64_t)comp * m.n_coarse;
    const uint32_t JK = fdiv((uint32_t)node, m.cx), I = (uint32_t)node - JK * m.nc[0];
    const uint32_t K = fdiv(JK, m.cy), J = JK - K * m.nc[1];
    const int C[3] = {(int)I, (int)J, (int)K};
    int fi[3][7];
    double w[3][7];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int d = 0; d < 7; ++d) {
            int q = 4 * C[a] + d - 3;
            bool ok = true;
            if (m2.per[a]) q = wrap(q, m2.nf[a], 1);
            else if (q < 0 || q >= m2.nf[a]) { ok = false; q = 4 * C[a]; }
            fi[a][d] = q;
            w[a][d] = ok ? 1.0 - 0.25 * (double)(d > 3 ? d - 3 : 3 - d) : 0.0;
        }
    const float *b = bf + (int64_t)comp * m2.n_fine;
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 7; ++c)
        for (int bb = 0; bb < 7; ++bb) {
            const int64_t rowb = (int64_t)m2.nf[0] * (fi[1][bb] + (int64_t)m2.nf[1] * fi[2][c]);
            float v[7];
#pragma unroll
            for (int a = 0; a < 7; ++a) v[a] = b[fi[0][a] + rowb];
            double row = 0.0;
#pragma unroll
            for (int a = 0; a < 7; ++a) row += w[0][a] * (double)v[a];
            acc += w[1][bb] * w[2][c] * row;
        }
    bc[t] = acc;
}

// Row form of k_restrict2: one workgroup per level L lattice row (J, K) and
// component.  Every level L + 2 node along x is first summed over the row's
// 7 x 7 (y, z) stencil (weights and wrapping as in k_restrict2, absent nodes
// read at a present one with weight 0; the 49 loads requested together)
// into LDS in FP64, then each coarse node of the row takes its 7 x terms
// from there.  The same weights as k_restrict2, summed (y, z) first.  LDS:
// the level L + 2 nodes along x, in doubles.
__global__ void __launch_bounds__(256) k_restrict2_rows(Mesh m, Mesh m2, const float *__restrict__ bf,
                                                        double *__restrict__ bc) {
    extern __shared__ double sT[];
    const int comp = blockIdx.y;
    const int64_t row = blockIdx.x;
    const int J = (int)(row % m.nc[1]), K = (int)(row / m.nc[1]);
    const int C[2] = {J, K};
    int fi[2][7];
    double w[2][7];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int d = 0; d < 7; ++d) {
            int q = 4 * C[a] + d - 3;
            bool ok = true;
            if (m2.per[a + 1]) q = wrap(q, m2.nf[a + 1], 1);
            else if (q < 0 || q >= m2.nf[a + 1]) { ok = false; q = 4 * C[a]; }
            fi[a][d] = q;
            w[a][d] = ok ? 1.0 - 0.25 * (double)(d > 3 ? d - 3 : 3 - d) : 0.0;
        }
    const float *b = bf + (int64_t)comp * m2.n_fine;
    const int nf0 = m2.nf[0];
    for (int i = threadIdx.x; i < nf0; i += blockDim.x) {
        float v[7][7];
#pragma unroll
        for (int c = 0; c < 7; ++c)
#pragma unroll
            for (int bb = 0; bb < 7; ++bb) v[c][bb] = b[i + (int64_t)nf0 * (fi[0][bb] + (int64_t)m2.nf[1] * fi[1][c])];
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < 7; ++c) {
            double col = 0.0;
#pragma unroll
            for (int bb = 0; bb < 7; ++bb) col += w[0][bb] * (double)v[c][bb];
            acc += w[1][c] * col;
        }
        sT[i] = acc;
    }
    __syncthreads();
    double *out = bc + (int64_t)comp * m.n_coarse + (int64_t)m.nc[0] * (J + (int64_t)m.nc[1] * K);
    for (int I = threadIdx.x; I < m.nc[0]; I += blockDim.x) {
        double acc = 0.0;
#pragma unroll
        for (int d = 0; d < 7; ++d) {
            int q = 4 * I + d - 3;
            bool ok = true;
            if (m2.per[0]) q = wrap(q, nf0, 1);
            else if (q < 0 || q >= nf0) { ok = false; q = 4 * I; }
            const double wx = ok ? 1.0 - 0.25 * (double)(d > 3 ? d - 3 : 3 - d) : 0.0;
            acc += wx * sT[q];
        }
        out[I] = acc;
    }
}

// ------------------------------------------------------- dof map, valence --
__global__ void k_dofmap2(Mesh m, Mesh m2, int32_t *__restrict__ map) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m.n_patches * L2_NODES) return;
    const uint32_t M = (uint32_t)(t / L2_NODES), iota = (uint32_t)(t - (int64_t)M * L2_NODES);
    const uint32_t JK = fdiv(M, m.px), I = M - JK * m.n[0];
    const uint32_t K = fdiv(JK, m.py), J = JK - K * m.n[1];
    const int a = iota % 5, b = (iota / 5) % 5, c = iota / 25;
    const int i = wrap(4 * I + a, m2.nf[0], m2.per[0]);
    const int j = wrap(4 * J + b, m2.nf[1], m2.per[1]);
    const int k = wrap(4 * K + c, m2.nf[2], m2.per[2]);
    map[t] = i + m2.nf[0] * (j + m2.nf[1] * k);
}

// valence: 2 per axis at indices divisible by 4 that are interior (or on a
// periodic axis), else 1
__global__ void k_mult2(Mesh m2, uint8_t *__restrict__ mult) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m2.n_fine) return;
    const uint32_t jk = fdiv((uint32_t)t, m2.fx), i = (uint32_t)t - jk * m2.nf[0];
    const uint32_t k = fdiv(jk, m2.fy), j = jk - k * m2.nf[1];
    const int c[3] = {(int)i, (int)j, (int)k};
    int v = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (!(c[a] & 3) && (m2.per[a] || (c[a] > 0 && c[a] < m2.nf[a] - 1))) v *= 2;
    mult[t] = (uint8_t)v;
}

// ----------------------------------------------------------- gather Q -----
// Row M = [u(125 nodes), v, w, r_u, r_v, r_w, H0, H1, H2, 0 ...]: one thread
// per four consecutive columns; standardisation (X - shift) * inv_scale as
// the one-level gather applies it.
template <int DT>
__global__ void __launch_bounds__(256)
    k_gather2(Mesh m, Mesh m2, const float *__restrict__ x, const float *__restrict__ r,
              const float *__restrict__ shift, const float *__restrict__ inv_scale, void *__restrict__ Xout,
              int64_t ldx) {
    const int quads = (int)(ldx / 4);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t M = t / quads;
    if (M >= m.n_patches) return;
    const int col0 = (int)(t - M * quads) * 4;
    const uint32_t JK = fdiv((uint32_t)M, m.px), I = (uint32_t)M - JK * m.n[0];
    const uint32_t K = fdiv(JK, m.py), J = JK - K * m.n[1];
    float sh[4], sc[4], v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int col = col0 + q;
        const int cc = col < L2_NIN ? col : L2_NIN - 1;
        sh[q] = shift ? shift[cc] : 0.0f;
        sc[q] = inv_scale ? inv_scale[cc] : 1.0f;
        // node columns read a clamped (always valid) address
        const int cn = col < 6 * L2_NODES ? col : 0;
        const int f = cn / L2_NODES, iota = cn - L2_NODES * f;
        const int a = iota % 5, b = (iota / 5) % 5, c = iota / 25;
        const int i = wrap(4 * (int)I + a, m2.nf[0], m2.per[0]);
        const int j = wrap(4 * (int)J + b, m2.nf[1], m2.per[1]);
        const int k = wrap(4 * (int)K + c, m2.nf[2], m2.per[2]);
        const int64_t node = i + (int64_t)m2.nf[0] * (j + (int64_t)m2.nf[1] * k);
        v[q] = f < 3 ? x[f * m2.n_fine + node] : r[(f - 3) * m2.n_fine + node];
    }
    float z[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int col = col0 + q;
        float val = col < 6 * L2_NODES ? v[q] : (col < L2_NIN ? m.H[col - 6 * L2_NODES] : 0.0f);
        if (col < L2_NIN) {
            if (shift) val -= sh[q];
            if (inv_scale) val *= sc[q];
        }
        z[q] = val;
    }
    if (DT == DNNMG_F32) {
        *(float4 *)((float *)Xout + M * ldx + col0) = make_float4(z[0], z[1], z[2], z[3]);
    } else {
        uint2 o;
        o.x = pack_bf16x2_hw(z[0], z[1]);
        o.y = pack_bf16x2_hw(z[2], z[3]);
        *(uint2 *)((uint16_t *)Xout + M * ldx + col0) = o;
    }
}

// ----------------------------------------------------- extension L --------
// Patches holding lattice index i along one axis (n patches of 4 cells):
// one (local index i mod 4) or, at indices divisible by 4, two (local 4 and
// 0), in ascending patch order (the wrapped lower patch of a periodic axis
// last at i = 0); an absent second holder repeats the first with weight 0.
struct Hold2 {
    int P[2], loc[2];
    float w[2];
    int cnt;
};

__device__ __forceinline__ Hold2 holders2(int i, int n, int per) {
    Hold2 h;
    if (i & 3) {
        h.P[0] = h.P[1] = i >> 2;
        h.loc[0] = h.loc[1] = i & 3;
        h.w[0] = 1.f;
        h.w[1] = 0.f;
        h.cnt = 1;
        return h;
    }
    int hi = i >> 2, lo = hi - 1;
    if (per) {
        if (lo < 0) lo += n;
        const bool lo_first = lo < hi;
        h.P[0] = lo_first ? lo : hi;
        h.loc[0] = lo_first ? 4 : 0;
        h.P[1] = lo_first ? hi : lo;
        h.loc[1] = lo_first ? 0 : 4;
        h.w[0] = h.w[1] = 1.f;
        h.cnt = 2;
        return h;
    }
    const bool has_lo = lo >= 0, has_hi = hi < n;
    h.P[0] = has_lo ? lo : hi;
    h.loc[0] = has_lo ? 4 : 0;
    h.P[1] = has_hi ? hi : h.P[0];
    h.loc[1] = has_hi ? 0 : h.loc[0];
    h.w[0] = 1.f;
    h.w[1] = (has_lo && has_hi) ? 1.f : 0.f;
    h.cnt = (int)has_lo + (int)has_hi;
    return h;
}

// d = mu (.) sum over the holding patches of Y[M][125 c + iota], summed in
// ascending patch order; Dirichlet velocity nodes get 0; with vbase the
// output is the corrected iterate (vbase + d, pressure of vbase).
__global__ void __launch_bounds__(256) k_scatter2(Mesh m, Mesh m2, const float *__restrict__ Y,
                                                  const float *__restrict__ vbase, float *__restrict__ d) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m2.n_fine) return;
    const uint32_t jk = fdiv((uint32_t)t, m2.fx), i = (uint32_t)t - jk * m2.nf[0];
    const uint32_t k = fdiv(jk, m2.fy), j = jk - k * m2.nf[1];
    float b[4] = {0.f, 0.f, 0.f, 0.f};
    if (vbase)
#pragma unroll
        for (int c = 0; c < 4; ++c) b[c] = vbase[c * m2.n_fine + t];
    const Hold2 hx = holders2((int)i, m.n[0], m.per[0]);
    const Hold2 hy = holders2((int)j, m.n[1], m.per[1]);
    const Hold2 hz = holders2((int)k, m.n[2], m.per[2]);
    float y[8][3], wgt[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int a = q & 1, bb = (q >> 1) & 1, c = q >> 2;
        const int64_t M = hx.P[a] + (int64_t)m.n[0] * (hy.P[bb] + (int64_t)m.n[1] * hz.P[c]);
        const int iota = hx.loc[a] + L2_SIDE * hy.loc[bb] + L2_SIDE * L2_SIDE * hz.loc[c];
        const float *src = Y + M * L2_NOUT + iota;
        y[q][0] = src[0];
        y[q][1] = src[L2_NODES];
        y[q][2] = src[2 * L2_NODES];
        wgt[q] = hx.w[a] * hy.w[bb] * hz.w[c];
    }
    float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = fmaf(wgt[q], y[q][c], acc[c]);
    const float inv = 1.0f / (float)(hx.cnt * hy.cnt * hz.cnt); // a power of two: exact
    const bool dir = on_dirichlet(m2, (int)i, (int)j, (int)k);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float v = dir ? 0.0f : acc[c] * inv;
        d[c * m2.n_fine + t] = vbase ? v + b[c] : v;
    }
    if (vbase) d[3 * m2.n_fine + t] = b[3];
}

// ----------------------------------------- inputs of the paper's network --
// Row M = [x~ (4 fields) at the S^3 patch nodes, r (4 fields) there, 24
// geometry features (row M of geo_rows, or the box's brick features when
// geo_rows is null)]: one thread per four consecutive columns.  The fine
// lattice is mf (m itself for one-level patches), S = 2^J + 1.
struct Geo24 {
    float f[24];
};

template <int DT, int J>
__global__ void __launch_bounds__(256)
    k_gather_paper(Mesh m, Mesh mf, const float *__restrict__ x, const float *__restrict__ r,
                   const float *__restrict__ shift, const float *__restrict__ inv_scale, Geo24 geo,
                   const float *__restrict__ geo_rows, void *__restrict__ Xout, int64_t ldx) {
    constexpr int P = 1 << J, S = P + 1, NL = S * S * S, NIN = 8 * NL + 24;
    const int quads = (int)(ldx / 4);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t M = t / quads;
    if (M >= m.n_patches) return;
    const int col0 = (int)(t - M * quads) * 4;
    const uint32_t JK = fdiv((uint32_t)M, m.px), I = (uint32_t)M - JK * m.n[0];
    const uint32_t K = fdiv(JK, m.py), Jj = JK - K * m.n[1];
    float sh[4], sc[4], v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int col = col0 + q;
        const int cc = col < NIN ? col : NIN - 1;
        sh[q] = shift ? shift[cc] : 0.0f;
        sc[q] = inv_scale ? inv_scale[cc] : 1.0f;
        const int cn = col < 8 * NL ? col : 0; // node columns read a valid address
        const int f = cn / NL, iota = cn - NL * f;
        const int a = iota % S, b = (iota / S) % S, c = iota / (S * S);
        const int i = wrap(P * (int)I + a, mf.nf[0], mf.per[0]);
        const int j = wrap(P * (int)Jj + b, mf.nf[1], mf.per[1]);
        const int k = wrap(P * (int)K + c, mf.nf[2], mf.per[2]);
        const int64_t node = i + (int64_t)mf.nf[0] * (j + (int64_t)mf.nf[1] * k);
        v[q] = f < 4 ? x[f * mf.n_fine + node] : r[(f - 4) * mf.n_fine + node];
    }
    float z[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int col = col0 + q;
        float val = col < 8 * NL ? v[q]
                    : (col < NIN ? (geo_rows ? geo_rows[24 * M + (col - 8 * NL)] : geo.f[col - 8 * NL]) : 0.0f);
        if (col < NIN) {
            if (shift) val -= sh[q];
            if (inv_scale) val *= sc[q];
        }
        z[q] = val;
    }
    if (DT == DNNMG_F32) {
        *(float4 *)((float *)Xout + M * ldx + col0) = make_float4(z[0], z[1], z[2], z[3]);
    } else {
        uint2 o;
        o.x = pack_bf16x2_hw(z[0], z[1]);
        o.y = pack_bf16x2_hw(z[2], z[3]);
        *(uint2 *)((uint16_t *)Xout + M * ldx + col0) = o;
    }
}

// The 24 geometry features of a coarse cell of the box (all cells are the
// same axis-parallel brick): edges H0 x4, H1 x4, H2 x4; the 4 diagonals
// |H|; the mean dihedral angle at each vertex, pi/2.
static Geo24 brick_features(const dnnmg_box *box) {
    Geo24 g;
    double H[3], d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        H[a] = box->len[a] / box->n[a];
        d2 += H[a] * H[a];
    }
    for (int a = 0; a < 3; ++a)
        for (int e = 0; e < 4; ++e) g.f[4 * a + e] = (float)H[a];
    for (int e = 0; e < 4; ++e) g.f[12 + e] = (float)sqrt(d2);
    for (int e = 0; e < 8; ++e) g.f[16 + e] = (float)(0.5 * 3.14159265358979323846);
    return g;
}

// the doubled box (its fine mesh is level L + 2)
static int level2_meshes(const dnnmg_box *box, Mesh *m, Mesh *m2) {
    int rc = make_mesh(box, m);
    if (rc) return rc;
    dnnmg_box b2 = *box;
    for (int a = 0; a < 3; ++a) b2.n[a] = 2 * box->n[a];
    return make_mesh(&b2, m2);
}

void prolong_wide_launch(const Mesh &m, int ncomp, const double *xc, double *xf, hipStream_t s);

} // namespace dnnmg

using namespace dnnmg;

#define STREAM ((hipStream_t)stream)

static int check_levels(int levels, const char *who) {
    if (levels != 1 && levels != 2) return fail(DNNMG_ERR_UNSUPPORTED, "%s: levels %d (1 or 2)", who, levels);
    return DNNMG_OK;
}

extern "C" int dnnmg_level_sizes(const dnnmg_box *box, int levels, int64_t *n_fine, int64_t *n_coarse,
                                 int64_t *n_patches) {
    int rc = check_levels(levels, "dnnmg_level_sizes");
    if (rc) return rc;
    Mesh m, m2;
    if (levels == 1) return dnnmg_box_sizes(box, n_fine, n_coarse, n_patches);
    if ((rc = level2_meshes(box, &m, &m2))) return rc;
    if (n_fine) *n_fine = m2.n_fine;
    if (n_coarse) *n_coarse = m.n_coarse;
    if (n_patches) *n_patches = m.n_patches;
    return DNNMG_OK;
}

extern "C" int dnnmg_patch_dofmap_levels(const dnnmg_box *box, int levels, int32_t *map, uint8_t *mult,
                                         void *stream) {
    int rc = check_levels(levels, "dnnmg_patch_dofmap_levels");
    if (rc) return rc;
    if (levels == 1) return dnnmg_patch_dofmap(box, map, mult, stream);
    Mesh m, m2;
    if ((rc = level2_meshes(box, &m, &m2))) return rc;
    if (!map && !mult) return fail(DNNMG_ERR_ARG, "dnnmg_patch_dofmap_levels: map and mult are both NULL");
    if (map) k_dofmap2<<<blocks_for(m.n_patches * L2_NODES, 256), 256, 0, STREAM>>>(m, m2, map);
    if (mult) k_mult2<<<blocks_for(m2.n_fine, 256), 256, 0, STREAM>>>(m2, mult);
    return hip_check(hipGetLastError(), "dnnmg_patch_dofmap_levels launch");
}

extern "C" int dnnmg_prolong_levels(const dnnmg_box *box, int levels, int ncomp, const double *xc, float *xf,
                                    void *stream) {
    int rc = check_levels(levels, "dnnmg_prolong_levels");
    if (rc) return rc;
    if (levels == 1) return dnnmg_prolong(box, ncomp, xc, xf, stream);
    Mesh m, m2;
    if ((rc = level2_meshes(box, &m, &m2))) return rc;
    if (ncomp < 1 || ncomp > 4) return fail(DNNMG_ERR_ARG, "dnnmg_prolong_levels: ncomp %d not in 1..4", ncomp);
    if (!xc || !xf) return fail(DNNMG_ERR_ARG, "dnnmg_prolong_levels: NULL pointer");
    // the row form where its LDS row fits 64 KB, else the per-node form
    const size_t lds = sizeof(float) * 4 * (size_t)m2.nc[0];
    if (lds <= 65536)
        k_prolong2_rows<<<dim3((unsigned)((int64_t)m2.nf[1] * m2.nf[2]), (unsigned)ncomp), 256, lds, STREAM>>>(m, m2, xc,
                                                                                                          xf);
    else
        k_prolong2<<<blocks_for((int64_t)ncomp * m2.n_fine, 256), 256, 0, STREAM>>>(m, m2, ncomp, xc, xf);
    return hip_check(hipGetLastError(), "dnnmg_prolong_levels launch");
}

extern "C" size_t dnnmg_prolong_residual_b_levels_workspace(const dnnmg_box *box, int levels) {
    if (check_levels(levels, "dnnmg_prolong_residual_b_levels_workspace")) return 0;
    Mesh m;
    if (make_mesh(box, &m)) return 0;
    return levels == 1 ? 0 : (sizeof(double) * 4 * (size_t)m.n_fine + 255) / 256 * 256;
}

// J = 2: level L + 1 = P x^L in FP32 operations (widened to FP64 in the
// workspace), then the one-level fused pass on the doubled box prolongs it
// to level L + 2 with the same operations -- x~ is the two-level
// prolongation bit for bit -- and evaluates only the new iterate's terms:
// x~ is the patch interpolant of level L + 1 exactly, so the local
// projection terms (onto level L + 1) vanish and are not evaluated.
extern "C" int dnnmg_prolong_residual_b_levels(const dnnmg_box *box, int levels, const dnnmg_ns *ns,
                                               const double *xc, const float *b, float *xt, float *r, void *ws,
                                               size_t ws_bytes, void *stream) {
    int rc = check_levels(levels, "dnnmg_prolong_residual_b_levels");
    if (rc) return rc;
    if (levels == 1) return dnnmg_prolong_residual_b(box, ns, xc, b, xt, r, stream);
    Mesh m, m2;
    if ((rc = level2_meshes(box, &m, &m2))) return rc;
    if (!xc || !b || !xt || !r || !ws) return fail(DNNMG_ERR_ARG, "dnnmg_prolong_residual_b_levels: NULL pointer");
    const size_t need = dnnmg_prolong_residual_b_levels_workspace(box, levels);
    if (ws_bytes < need)
        return fail(DNNMG_ERR_SHAPE, "dnnmg_prolong_residual_b_levels: workspace %zu < %zu bytes", ws_bytes, need);
    if ((uintptr_t)ws % 16) return fail(DNNMG_ERR_ARG, "dnnmg_prolong_residual_b_levels: ws not 16-byte aligned");
    double *x1 = (double *)ws;
    prolong_wide_launch(m, 4, xc, x1, STREAM);
    if ((rc = hip_check(hipGetLastError(), "dnnmg_prolong_residual_b_levels launch"))) return rc;
    dnnmg_box b2 = *box;
    for (int a = 0; a < 3; ++a) b2.n[a] = 2 * box->n[a];
    return dnnmg_prolong_residual_b(&b2, ns, x1, b, xt, r, stream);
}

extern "C" int dnnmg_restrict_levels(const dnnmg_box *box, int levels, int ncomp, const float *bf, double *bc,
                                     void *stream) {
    int rc = check_levels(levels, "dnnmg_restrict_levels");
    if (rc) return rc;
    if (levels == 1) return dnnmg_restrict(box, ncomp, bf, bc, stream);
    Mesh m, m2;
    if ((rc = level2_meshes(box, &m, &m2))) return rc;
    if (ncomp < 1 || ncomp > 4) return fail(DNNMG_ERR_ARG, "dnnmg_restrict_levels: ncomp %d not in 1..4", ncomp);
    if (!bf || !bc) return fail(DNNMG_ERR_ARG, "dnnmg_restrict_levels: NULL pointer");
    // the row form where its LDS row fits 64 KB, else the per-node form
    const size_t lds = sizeof(double) * (size_t)m2.nf[0];
    if (lds <= 65536)
        k_restrict2_rows<<<dim3((unsigned)((int64_t)m.nc[1] * m.nc[2]), (unsigned)ncomp), 256, lds, STREAM>>>(m, m2, bf,
                                                                                                         bc);
    else
        k_restrict2<<<blocks_for((int64_t)ncomp * m.n_coarse, 256), 256, 0, STREAM>>>(m, m2, ncomp, bf, bc);
    return hip_check(hipGetLastError(), "dnnmg_restrict_levels launch");
}

extern "C" int dnnmg_patch_gather_levels(const dnnmg_box *box, int levels, const float *x, const float *r,
                                         const dnnmg_feat *feat, int dtype, void *X, int64_t ldx, void *stream) {
    int rc = check_levels(levels, "dnnmg_patch_gather_levels");
    if (rc) return rc;
    if (levels == 1) return dnnmg_patch_gather(box, x, r, feat, dtype, 1.0f, X, ldx, stream);
    Mesh m, m2;
    if ((rc = level2_meshes(box, &m, &m2))) return rc;
    if (!x || !r || !X) return fail(DNNMG_ERR_ARG, "dnnmg_patch_gather_levels: NULL pointer");
    if (!aligned16(X)) return fail(DNNMG_ERR_ARG, "dnnmg_patch_gather_levels: X not 16-byte aligned");
    const int align = dtype == DNNMG_F32 ? 4 : 8;
    if (ldx < L2_NIN || ldx % align)
        return fail(DNNMG_ERR_SHAPE, "dnnmg_patch_gather_levels: ldx %lld must be >= %d and a multiple of %d",
                    (long long)ldx, L2_NIN, align);
    const float *sh = feat ? feat->shift : nullptr;
    const float *sc = feat ? feat->inv_scale : nullptr;
    const unsigned g = blocks_for(m.n_patches * (ldx / 4), 256);
    if (dtype == DNNMG_F32)
        k_gather2<DNNMG_F32><<<g, 256, 0, STREAM>>>(m, m2, x, r, sh, sc, X, ldx);
    else if (dtype == DNNMG_BF16)
        k_gather2<DNNMG_BF16><<<g, 256, 0, STREAM>>>(m, m2, x, r, sh, sc, X, ldx);
    else
        return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_patch_gather_levels: dtype %d (FP32 or BF16 inputs)", dtype);
    return hip_check(hipGetLastError(), "dnnmg_patch_gather_levels launch");
}

extern "C" int dnnmg_scatter_avg_levels(const dnnmg_box *box, int levels, const float *Y, const float *vbase,
                                        float *d, void *stream) {
    int rc = check_levels(levels, "dnnmg_scatter_avg_levels");
    if (rc) return rc;
    if (levels == 1) return dnnmg_scatter_avg(box, Y, vbase, d, stream);
    Mesh m, m2;
    if ((rc = level2_meshes(box, &m, &m2))) return rc;
    if (!Y || !d) return fail(DNNMG_ERR_ARG, "dnnmg_scatter_avg_levels: NULL pointer");
    k_scatter2<<<blocks_for(m2.n_fine, 256), 256, 0, STREAM>>>(m, m2, Y, vbase, d);
    return hip_check(hipGetLastError(), "dnnmg_scatter_avg_levels launch");
}

static int gather_paper(const dnnmg_box *box, int levels, const float *geo_rows, const float *x, const float *r,
                        const dnnmg_feat *feat, int dtype, void *X, int64_t ldx, void *stream) {
    int rc = check_levels(levels, "dnnmg_patch_gather_paper");
    if (rc) return rc;
    Mesh m, m2;
    if (levels == 1) {
        if ((rc = make_mesh(box, &m))) return rc;
        m2 = m;
    } else if ((rc = level2_meshes(box, &m, &m2))) {
        return rc;
    }
    if (!x || !r || !X) return fail(DNNMG_ERR_ARG, "dnnmg_patch_gather_paper: NULL pointer");
    if (!aligned16(X)) return fail(DNNMG_ERR_ARG, "dnnmg_patch_gather_paper: X not 16-byte aligned");
    const int nin = levels == 1 ? 240 : 1024;
    const int align = dtype == DNNMG_F32 ? 4 : 8;
    if (ldx < nin || ldx % align)
        return fail(DNNMG_ERR_SHAPE, "dnnmg_patch_gather_paper: ldx %lld must be >= %d and a multiple of %d",
                    (long long)ldx, nin, align);
    const float *sh = feat ? feat->shift : nullptr;
    const float *sc = feat ? feat->inv_scale : nullptr;
    const Geo24 geo = brick_features(box);
    const unsigned g = blocks_for(m.n_patches * (ldx / 4), 256);
#define GP(DT, JJ) k_gather_paper<DT, JJ><<<g, 256, 0, STREAM>>>(m, m2, x, r, sh, sc, geo, geo_rows, X, ldx)
    if (dtype == DNNMG_F32 && levels == 1) GP(DNNMG_F32, 1);
    else if (dtype == DNNMG_F32) GP(DNNMG_F32, 2);
    else if (dtype == DNNMG_BF16 && levels == 1) GP(DNNMG_BF16, 1);
    else if (dtype == DNNMG_BF16) GP(DNNMG_BF16, 2);
    else return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_patch_gather_paper: dtype %d (FP32 or BF16)", dtype);
#undef GP
    return hip_check(hipGetLastError(), "dnnmg_patch_gather_paper launch");
}

extern "C" int dnnmg_patch_gather_paper(const dnnmg_box *box, int levels, const float *x, const float *r,
                                        const dnnmg_feat *feat, int dtype, void *X, int64_t ldx, void *stream) {
    return gather_paper(box, levels, nullptr, x, r, feat, dtype, X, ldx, stream);
}

extern "C" int dnnmg_patch_gather_paper_geom(const dnnmg_box *box, const float *geo24, const float *x,
                                             const float *r, const dnnmg_feat *feat, int dtype, void *X,
                                             int64_t ldx, void *stream) {
    if (!geo24) return fail(DNNMG_ERR_ARG, "dnnmg_patch_gather_paper_geom: geo24 is NULL");
    return gather_paper(box, 1, geo24, x, r, feat, dtype, X, ldx, stream);
}
