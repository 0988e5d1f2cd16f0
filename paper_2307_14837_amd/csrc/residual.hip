// Matrix-free fine residual r = F - A(x) and right-hand side b = Rhs(v) of the
// Crank-Nicolson system (arXiv 2307.14837, Sec. 2.3, eq. (4cranknicholson3),
// stabilisation parameters eq. (stabparams), local projection terms of
// eq. (disc:ns)) on the uniform fine hexahedral mesh, with Q1 elements and
// 2x2x2 Gauss quadrature on every fine cell.  The LPS projection pi is the
// interpolation onto the Q1 space of the patch (coarse cell) holding the
// fine cell.
//
// Work decomposition.  A workgroup owns a block of TX x TY x TZ fine nodes
// whose origin is even in every axis (so it is aligned to patches).  It
// stages the fields of the node block plus a halo into LDS and evaluates
// every fine cell touching an owned node (one extra cell layer on the low
// side), one thread per cell.  Per equation the cells' vertex integrals go
// to LDS and each owned node sums its 8 cells in a fixed order, so no
// atomics are used and the result does not depend on scheduling.  Owned
// nodes are written once.  The local projection terms vanish exactly on
// cells where the iterate equals its patch interpolant (always the case for
// a prolongated coarse solution); they are evaluated in a second pass only
// for the other cells.  Their test functions pi(phi_i) live on the corners
// of a patch: those contributions are summed per owned patch and written to
// a workspace (with a per-tile flag), and a second small kernel adds them to
// the coarse-vertex nodes.  Tiles are laid out so that each XCD takes one
// contiguous range of them (halo reads then hit the XCD's own L2).
//
// Per cell the quadrature uses sum factorisation: values and gradients at
// the 8 Gauss points from the 8 vertex values, and the transpose to vertex
// integrals, each by three 1-D passes.
#include <mutex>

#include "common.hpp"
#include "mlp.hpp"

// Floating-point contraction only within a source expression: every kernel
// instance (single box, batched, with or without forcing) then rounds the
// same terms alike, and batched results equal single-box results bit for bit.
#pragma clang fp contract(on)

namespace dnnmg {

// Gauss points on [0,1]: 1/2 -+ 1/(2 sqrt 3)
constexpr float GLO = 0.21132486540518713f;

// --------------------------------------------------- 1-D building blocks --
// value at the two Gauss points of a linear function with end values u0, u1
__device__ __forceinline__ void lin2(float u0, float u1, float &q0, float &q1) {
    float d = u1 - u0;
    q0 = fmaf(GLO, d, u0);
    q1 = fmaf(-GLO, d, u1);
}

// Values at the 8 Gauss points (q = qa + 2 qb + 4 qc) of the trilinear
// function with vertex values u (j = a + 2 b + 4 c).
__device__ __forceinline__ void eval_val(const float u[8], float v[8]) {
    float X[8], Y[8];
#pragma unroll
    for (int bc = 0; bc < 4; ++bc) lin2(u[2 * bc], u[2 * bc + 1], X[2 * bc], X[2 * bc + 1]);
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int qa = 0; qa < 2; ++qa) lin2(X[qa + 4 * c], X[qa + 2 + 4 * c], Y[qa + 4 * c], Y[qa + 2 + 4 * c]);
#pragma unroll
    for (int ab = 0; ab < 4; ++ab) lin2(Y[ab], Y[ab + 4], v[ab], v[ab + 4]);
}

// Values and physical gradients at the Gauss points.
__device__ __forceinline__ void eval_vg(const float u[8], float ih0, float ih1, float ih2, float v[8],
                                        float g0[8], float g1[8], float g2[8]) {
    float X[8], DX[4];
#pragma unroll
    for (int bc = 0; bc < 4; ++bc) {
        lin2(u[2 * bc], u[2 * bc + 1], X[2 * bc], X[2 * bc + 1]);
        DX[bc] = u[2 * bc + 1] - u[2 * bc];
    }
    float Y[8], DY[4], DXY[4]; // DY[qa + 2c], DXY[qb + 2c]
#pragma unroll
    for (int c = 0; c < 2; ++c) {
#pragma unroll
        for (int qa = 0; qa < 2; ++qa) {
            lin2(X[qa + 4 * c], X[qa + 2 + 4 * c], Y[qa + 4 * c], Y[qa + 2 + 4 * c]);
            DY[qa + 2 * c] = X[qa + 2 + 4 * c] - X[qa + 4 * c];
        }
        lin2(DX[2 * c], DX[2 * c + 1], DXY[2 * c], DXY[2 * c + 1]);
    }
    float GX[4], GY[4]; // GX[qb + 2qc], GY[qa + 2qc]
#pragma unroll
    for (int ab = 0; ab < 4; ++ab) lin2(Y[ab], Y[ab + 4], v[ab], v[ab + 4]);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        lin2(DXY[t], DXY[t + 2], GX[t], GX[t + 2]);
        lin2(DY[t], DY[t + 2], GY[t], GY[t + 2]);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        int qa = q & 1, qb = (q >> 1) & 1, qc = q >> 2;
        g0[q] = GX[qb + 2 * qc] * ih0;
        g1[q] = GY[qa + 2 * qc] * ih1;
        g2[q] = (Y[qa + 2 * qb + 4] - Y[qa + 2 * qb]) * ih2;
    }
}

// 1-D transpose: vertex integrals of f (tested with the shape function) and
// g (tested with its derivative, 1/h folded into ih) from two Gauss points.
__device__ __forceinline__ void tr2(float f0, float f1, float gsum_ih, float &o0, float &o1) {
    float e = f0 - f1;
    o0 = fmaf(-GLO, e, f0) - gsum_ih;
    o1 = fmaf(GLO, e, f1) + gsum_ih;
}
__device__ __forceinline__ void tv2(float f0, float f1, float &o0, float &o1) {
    float e = f0 - f1;
    o0 = fmaf(-GLO, e, f0);
    o1 = fmaf(GLO, e, f1);
}

// out[j] = sum_q ( F[q] phi_j(q) + sum_d G_d[q] d_d phi_j(q) )  (unit weights;
// the caller scales by the quadrature weight).  Any of G may be null.
template <bool HX, bool HY, bool HZ>
__device__ __forceinline__ void integrate(const float F[8], const float *Gx, const float *Gy,
                                          const float *Gz, float ih0, float ih1, float ih2,
                                          float out[8]) {
    // x pass: per (qb, qc)
    float A[8], BY[8], BZ[8]; // index a + 2 qb + 4 qc
#pragma unroll
    for (int bc = 0; bc < 4; ++bc) {
        int q0 = 2 * bc, q1 = 2 * bc + 1;
        float gs = HX ? (Gx[q0] + Gx[q1]) * ih0 : 0.0f;
        tr2(F[q0], F[q1], gs, A[q0], A[q1]);
        if (HY) tv2(Gy[q0], Gy[q1], BY[q0], BY[q1]);
        if (HZ) tv2(Gz[q0], Gz[q1], BZ[q0], BZ[q1]);
    }
    // y pass: per (a, qc)
    float A2[8], BZ2[8]; // index a + 2 b + 4 qc
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            int q0 = a + 4 * c, q1 = a + 2 + 4 * c;
            float gs = HY ? (BY[q0] + BY[q1]) * ih1 : 0.0f;
            tr2(A[q0], A[q1], gs, A2[q0], A2[q1]);
            if (HZ) tv2(BZ[q0], BZ[q1], BZ2[q0], BZ2[q1]);
        }
    // z pass: per (a, b)
#pragma unroll
    for (int ab = 0; ab < 4; ++ab) {
        float gs = HZ ? (BZ2[ab] + BZ2[ab + 4]) * ih2 : 0.0f;
        tr2(A2[ab], A2[ab + 4], gs, out[ab], out[ab + 4]);
    }
}

// Patch-local Q1 interpolation (pi): values at the 8 vertices of the fine
// cell with offset (ox, oy, oz) in its patch, from the patch's 8 corners.
__device__ __forceinline__ float half_or(int t, float c0, float c1) {
    return t == 0 ? c0 : (t == 2 ? c1 : 0.5f * (c0 + c1));
}
__device__ __forceinline__ void pi_vertices(const float cor[8], int ox, int oy, int oz, float out[8]) {
    float X[8]; // index a + 2B + 4C (a = vertex x, B, C = corner y, z)
#pragma unroll
    for (int BC = 0; BC < 4; ++BC)
#pragma unroll
        for (int a = 0; a < 2; ++a) X[a + 2 * BC] = half_or(ox + a, cor[2 * BC], cor[2 * BC + 1]);
    float Yv[8]; // a + 2b + 4C
#pragma unroll
    for (int C = 0; C < 2; ++C)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                Yv[a + 2 * b + 4 * C] = half_or(oy + b, X[a + 4 * C], X[a + 2 + 4 * C]);
#pragma unroll
    for (int ab = 0; ab < 4; ++ab)
#pragma unroll
        for (int c = 0; c < 2; ++c) out[ab + 4 * c] = half_or(oz + c, Yv[ab], Yv[ab + 4]);
}

// Transpose of pi_vertices: corner sums of vertex values weighted by the
// interpolation weights (the patch-local restriction).
__device__ __forceinline__ void w_pair(int t, float &w0, float &w1) {
    w0 = t == 0 ? 1.0f : (t == 2 ? 0.0f : 0.5f);
    w1 = t == 2 ? 1.0f : (t == 0 ? 0.0f : 0.5f);
}
__device__ __forceinline__ void pi_transpose(const float vals[8], int ox, int oy, int oz, float cor[8]) {
    float wx[2][2], wy[2][2], wz[2][2]; // w[vertex a][corner A]
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        w_pair(ox + a, wx[a][0], wx[a][1]);
        w_pair(oy + a, wy[a][0], wy[a][1]);
        w_pair(oz + a, wz[a][0], wz[a][1]);
    }
    float X[8]; // A + 2b + 4c
#pragma unroll
    for (int bc = 0; bc < 4; ++bc)
#pragma unroll
        for (int A = 0; A < 2; ++A) X[A + 2 * bc] = wx[0][A] * vals[2 * bc] + wx[1][A] * vals[2 * bc + 1];
    float Yv[8]; // A + 2B + 4c
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int A = 0; A < 2; ++A)
#pragma unroll
            for (int B = 0; B < 2; ++B)
                Yv[A + 2 * B + 4 * c] = wy[0][B] * X[A + 4 * c] + wy[1][B] * X[A + 2 + 4 * c];
#pragma unroll
    for (int AB = 0; AB < 4; ++AB)
#pragma unroll
        for (int C = 0; C < 2; ++C) cor[AB + 4 * C] = wz[0][C] * Yv[AB] + wz[1][C] * Yv[AB + 4];
}

// The patch interpolant evaluated directly at the Gauss points of one of its
// cells.  Along an axis the cell with offset o covers the coarse coordinates
// [o/2, (o+1)/2] of its patch, so its Gauss points sit at s = (o + xi) / 2.
__device__ __forceinline__ void patch_coords(int o, float s[2]) {
    s[0] = 0.5f * ((float)o + GLO);
    s[1] = 0.5f * ((float)o + (1.0f - GLO));
}
// a patch-linear function with end values c0, c1 at the two coordinates s
__device__ __forceinline__ void plin2(float c0, float c1, const float s[2], float &q0, float &q1) {
    float d = c1 - c0;
    q0 = fmaf(s[0], d, c0);
    q1 = fmaf(s[1], d, c0);
}
// Values of the interpolant with corner values c at the cell's Gauss points
// (what eval_val gives from pi_vertices, up to rounding).
__device__ __forceinline__ void patch_val(const float c[8], const float sx[2], const float sy[2],
                                          const float sz[2], float v[8]) {
    float X[8]; // qa + 2B + 4C
#pragma unroll
    for (int BC = 0; BC < 4; ++BC) plin2(c[2 * BC], c[2 * BC + 1], sx, X[2 * BC], X[2 * BC + 1]);
    float Y[8]; // qa + 2qb + 4C
#pragma unroll
    for (int C = 0; C < 2; ++C)
#pragma unroll
        for (int qa = 0; qa < 2; ++qa) plin2(X[qa + 4 * C], X[qa + 2 + 4 * C], sy, Y[qa + 4 * C], Y[qa + 2 + 4 * C]);
#pragma unroll
    for (int ab = 0; ab < 4; ++ab) plin2(Y[ab], Y[ab + 4], sz, v[ab], v[ab + 4]);
}
// Its physical gradient at the Gauss points (the patch is two cells wide, so
// a corner difference is divided by 2h).  Each component is constant along
// its own axis: GX[qb + 2qc], GY[qa + 2qc], GZ[qa + 2qb].
__device__ __forceinline__ void patch_grad(const float c[8], const float sx[2], const float sy[2],
                                           const float sz[2], float ih0, float ih1, float ih2, float GX[4],
                                           float GY[4], float GZ[4]) {
    float D[4], t[4];
    // x: differences per (B, C), interpolated in y, then z
#pragma unroll
    for (int BC = 0; BC < 4; ++BC) D[BC] = c[2 * BC + 1] - c[2 * BC];
#pragma unroll
    for (int C = 0; C < 2; ++C) plin2(D[2 * C], D[2 * C + 1], sy, t[2 * C], t[2 * C + 1]); // qb + 2C
#pragma unroll
    for (int qb = 0; qb < 2; ++qb) plin2(t[qb], t[qb + 2], sz, GX[qb], GX[qb + 2]);
    // y: differences per (A, C), interpolated in x, then z
#pragma unroll
    for (int C = 0; C < 2; ++C)
#pragma unroll
        for (int A = 0; A < 2; ++A) D[A + 2 * C] = c[A + 2 + 4 * C] - c[A + 4 * C];
#pragma unroll
    for (int C = 0; C < 2; ++C) plin2(D[2 * C], D[2 * C + 1], sx, t[2 * C], t[2 * C + 1]); // qa + 2C
#pragma unroll
    for (int qa = 0; qa < 2; ++qa) plin2(t[qa], t[qa + 2], sz, GY[qa], GY[qa + 2]);
    // z: differences per (A, B), interpolated in x, then y
#pragma unroll
    for (int AB = 0; AB < 4; ++AB) D[AB] = c[AB + 4] - c[AB];
#pragma unroll
    for (int B = 0; B < 2; ++B) plin2(D[2 * B], D[2 * B + 1], sx, t[2 * B], t[2 * B + 1]); // qa + 2B
#pragma unroll
    for (int qa = 0; qa < 2; ++qa) plin2(t[qa], t[qa + 2], sy, GZ[qa], GZ[qa + 2]);
    const float hx = 0.5f * ih0, hy = 0.5f * ih1, hz = 0.5f * ih2;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        GX[k] *= hx;
        GY[k] *= hy;
        GZ[k] *= hz;
    }
}
// out[A + 2B + 4C] = sum over the cell's Gauss points of G . grad psi, psi
// the patch's Q1 function of corner (A, B, C) (unit weights): what
// pi_transpose gives from integrate with gradient terms only, up to rounding.
// Along an axis psi is l_0(s) = 1 - s or l_1(s) = s, with derivative -+1/(2h).
__device__ __forceinline__ void patch_integrate_grad(const float G0[8], const float G1[8], const float G2[8],
                                                     const float sx[2], const float sy[2], const float sz[2],
                                                     float ih0, float ih1, float ih2, float out[8]) {
    const float hx = 0.5f * ih0, hy = 0.5f * ih1, hz = 0.5f * ih2;
    // x pass per p = qb + 2qc: the x-derivative part summed over qa, the y
    // and z parts weighted with l_A(sx[qa])
    float SX[4], BY[8], BZ[8]; // BY, BZ: A + 2p
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int q0 = 2 * p, q1 = 2 * p + 1;
        SX[p] = (G0[q0] + G0[q1]) * hx;
        const float y1 = fmaf(sx[1], G1[q1], sx[0] * G1[q0]);
        BY[1 + 2 * p] = y1;
        BY[2 * p] = (G1[q0] + G1[q1]) - y1;
        const float z1 = fmaf(sx[1], G2[q1], sx[0] * G2[q0]);
        BZ[1 + 2 * p] = z1;
        BZ[2 * p] = (G2[q0] + G2[q1]) - z1;
    }
    // y pass per qc: value parts weighted with l_B(sy[qb]), y part summed over qb
    float Y[8], Z[8]; // A + 2B + 4qc
#pragma unroll
    for (int qc = 0; qc < 2; ++qc) {
        const int p0 = 2 * qc, p1 = 1 + 2 * qc;
        const float t1 = fmaf(sy[1], SX[p1], sy[0] * SX[p0]);
        const float t0 = (SX[p0] + SX[p1]) - t1;
#pragma unroll
        for (int A = 0; A < 2; ++A) {
            const float gy = (BY[A + 2 * p0] + BY[A + 2 * p1]) * hy;
            Y[A + 4 * qc] = (A ? t0 : -t0) - gy;
            Y[A + 2 + 4 * qc] = (A ? t1 : -t1) + gy;
            const float z1 = fmaf(sy[1], BZ[A + 2 * p1], sy[0] * BZ[A + 2 * p0]);
            Z[A + 2 + 4 * qc] = z1;
            Z[A + 4 * qc] = (BZ[A + 2 * p0] + BZ[A + 2 * p1]) - z1;
        }
    }
    // z pass per (A, B): value part weighted with l_C(sz[qc]), z part summed over qc
#pragma unroll
    for (int AB = 0; AB < 4; ++AB) {
        const float v1 = fmaf(sz[1], Y[AB + 4], sz[0] * Y[AB]);
        const float v0 = (Y[AB] + Y[AB + 4]) - v1;
        const float gz = (Z[AB] + Z[AB + 4]) * hz;
        out[AB] = v0 - gz;
        out[AB + 4] = v1 + gz;
    }
}

// ------------------------------------------------------------ kernel ------
constexpr int MODE_RES = 0;
constexpr int MODE_RHS = 1;
// residual of the prolongation of a coarse iterate, which the tile computes
// itself (and writes out): the iterate is patchwise Q1, so every local
// projection term vanishes identically and none is evaluated
constexpr int MODE_PRES = 2;
// the same against a given right-hand side b (the Rhs of the previous step's
// corrected velocity): r = b - A(x~); the tile evaluates only the terms of
// the new iterate and adds b at its owned nodes
constexpr int MODE_PRESB = 3;
// the general residual (any iterate, LPS terms where they do not vanish)
// against a given right-hand side: r = b - A(x)
constexpr int MODE_RESB = 4;
__host__ __device__ constexpr bool mode_prolongs(int mode) { return mode == MODE_PRES || mode == MODE_PRESB; }
__host__ __device__ constexpr bool mode_general(int mode) { return mode == MODE_RES || mode == MODE_RESB; }
__host__ __device__ constexpr bool mode_against_b(int mode) { return mode == MODE_PRESB || mode == MODE_RESB; }
__host__ __device__ constexpr bool mode_has_vp(int mode) { return mode == MODE_RES || mode == MODE_PRES; }

template <int MODE>
struct ResTile {
    static constexpr int TX = 16, TY = 8, TZ = 4;  // owned nodes
    static constexpr int NOWN = TX * TY * TZ;
    static constexpr int EX = TX + 1, EY = TY + 1, EZ = TZ + 1; // cells
    static constexpr int NCELL = EX * EY * EZ;
    // staged node range: [o-2, o+T] for x, p (patch corners), [o-1, o+T] for vp
    static constexpr int SX = TX + 3, SY = TY + 3, SZ = TZ + 3, SN = SX * SY * SZ;
    static constexpr int VX = TX + 2, VY = TY + 2, VZ = TZ + 2, VN = VX * VY * VZ;
    static constexpr int NPX = TX / 2, NPY = TY / 2, NPZ = TZ / 2, NP = NPX * NPY * NPZ;
    static constexpr int NT = 768; // one thread per cell (765 cells)
    // the right-hand side and the residual against a given one fit in 85
    // registers: two workgroups (six waves per SIMD) share a compute unit
    static constexpr int WAVES_PER_SIMD = MODE == MODE_RHS || MODE == MODE_PRESB ? 6 : 3;

    static constexpr int NF_STAGE = MODE != MODE_RHS ? 4 : 0; // x, p on the wide range
    static constexpr int NF_V = mode_against_b(MODE) ? 0 : 3; // vp (res) or v (rhs)
    static constexpr int NACC = MODE != MODE_RHS ? 4 : 3;
    // coarse nodes under the staged range (prolongating tiles)
    static constexpr int CX = TX / 2 + 2, CY = TY / 2 + 2, CZ = TZ / 2 + 2, CN = CX * CY * CZ;
    static_assert(NT >= NCELL && NT >= NOWN && NT >= 8 * NP, "one pass per role");
};

// One tile (bx, by, bz) of owned nodes of one box.  Thread e evaluates cell
// e; per equation the cells' 8 vertex integrals go to an LDS cell array, and
// after a barrier thread s < TX TY TZ sums the 8 cells around owned node s
// in a fixed order (and, for the LPS corner terms, thread 8 P + j the 8
// cells of owned patch P at corner j), so the sums need no atomics and the
// result does not depend on scheduling.
//
// RHS_OUT (general residual against b only): the tile also evaluates the
// next step's right-hand side Rhs(v) at the same iterate (no forcing) and
// replaces b by it at the owned nodes: b is then read from and written to
// b_io (vp unused), each owned node's b is loaded by its owner before any
// store, and b_save (optional) receives the b read.
template <int MODE, bool DELTA_MERGED = false, bool RHS_OUT = false>
__device__ __forceinline__ void residual_tile(const Mesh &m, const ResParams &P, int bx, int by, int bz,
                                              const float *__restrict__ x, const float *__restrict__ vp,
                                              const float *__restrict__ fmid, float *__restrict__ out,
                                              float *__restrict__ aux, int *__restrict__ tflag,
                                              const double *__restrict__ xc = nullptr,
                                              float *__restrict__ xt_out = nullptr, float *b_io = nullptr,
                                              float *__restrict__ b_save = nullptr) {
    static_assert(!RHS_OUT || MODE == MODE_RESB, "the right-hand side output is built for r = b - A(x)");
    using T = ResTile<MODE>;
    __shared__ float sX[T::NF_STAGE > 0 ? T::NF_STAGE * T::SN : 1];
    __shared__ float sV[T::NF_V > 0 ? T::NF_V * T::VN : 1];
    __shared__ float sF[mode_against_b(MODE) ? 1 : 3 * T::VN]; // forcing, when given
    __shared__ float sCell[8 * T::NCELL]; // [vertex j][cell]
    __shared__ float sCor[mode_general(MODE) ? 8 * T::NCELL : 1];
    __shared__ float sRhs[RHS_OUT ? 8 * T::NCELL : 1]; // [vertex j][cell], Rhs integrals
    __shared__ float sC[mode_prolongs(MODE) ? 4 * T::CN : 1]; // coarse iterate, rounded to FP32

    const int x0 = bx * T::TX, y0 = by * T::TY, z0 = bz * T::TZ;
    const int tid = threadIdx.x;
    const int64_t nfn = m.n_fine;

    // ---- stage fields into LDS (zero outside a non-periodic domain) ----
    auto gnode = [&](int gi, int gj, int gk, bool &ok) -> int64_t {
        gi = wrap(gi, m.nf[0], m.per[0]);
        gj = wrap(gj, m.nf[1], m.per[1]);
        gk = wrap(gk, m.nf[2], m.per[2]);
        ok = gi >= 0 && gi < m.nf[0] && gj >= 0 && gj < m.nf[1] && gk >= 0 && gk < m.nf[2];
        return gi + (int64_t)m.nf[0] * (gj + (int64_t)m.nf[1] * gk);
    };
    // b at the owned node is loaded first: its latency overlaps the staging
    float bown[mode_against_b(MODE) ? 4 : 1] = {};
    if constexpr (mode_against_b(MODE)) {
        const int gi = x0 + tid % T::TX, gj = y0 + (tid / T::TX) % T::TY, gk = z0 + tid / (T::TX * T::TY);
        if (tid < T::NOWN && gi < m.nf[0] && gj < m.nf[1] && gk < m.nf[2]) {
            const int64_t g = gi + (int64_t)m.nf[0] * (gj + (int64_t)m.nf[1] * gk);
#pragma unroll
            for (int f = 0; f < 4; ++f) bown[f] = RHS_OUT ? b_io[f * nfn + g] : vp[f * nfn + g];
        }
    }
    // all loads of a thread are issued before its LDS stores, so the staging
    // costs one memory round trip
    if constexpr (mode_prolongs(MODE)) {
        // coarse nodes x0/2 - 1 .. of the staged range, then Q1 interpolation
        // axis by axis (x, y, z) in FP32: the operations of the prolongation
        // kernel, so x~ is the same to the bit
        const int64_t ncn = m.n_coarse;
        for (int s = tid; s < T::CN; s += T::NT) {
            int ci = x0 / 2 - 1 + s % T::CX, cj = y0 / 2 - 1 + (s / T::CX) % T::CY, ck = z0 / 2 - 1 + s / (T::CX * T::CY);
            ci = wrap(ci, m.nc[0], m.per[0]);
            cj = wrap(cj, m.nc[1], m.per[1]);
            ck = wrap(ck, m.nc[2], m.per[2]);
            const bool ok = ci >= 0 && ci < m.nc[0] && cj >= 0 && cj < m.nc[1] && ck >= 0 && ck < m.nc[2];
            // absent nodes read node 0 and discard it: the loads carry no
            // branch and go out together
            const int64_t g = ok ? ci + (int64_t)m.nc[0] * (cj + (int64_t)m.nc[1] * ck) : 0;
            double d[4];
#pragma unroll
            for (int f = 0; f < 4; ++f) d[f] = xc[f * ncn + g];
            float v[4];
#pragma unroll
            for (int f = 0; f < 4; ++f) v[f] = ok ? (float)d[f] : 0.0f;
#pragma unroll
            for (int f = 0; f < 4; ++f) sC[f * T::CN + s] = v[f];
        }
        __syncthreads();
        for (int s = tid; s < T::SN; s += T::NT) {
            const int lx = s % T::SX, ly = (s / T::SX) % T::SY, lz = s / (T::SX * T::SY);
            bool ok;
            (void)gnode(x0 - 2 + lx, y0 - 2 + ly, z0 - 2 + lz, ok);
            // the staged origin x0 - 2 is even: parities and coarse cells follow lx
            const int ox = lx & 1, oy = ly & 1, oz = lz & 1;
            const int cb = (lx >> 1) + T::CX * ((ly >> 1) + T::CY * (lz >> 1));
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const float *c = sC + f * T::CN + cb;
                float X[2][2] = {{0.f, 0.f}, {0.f, 0.f}}; // [y][z] after the x pass
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int cc = 0; cc < 2; ++cc) {
                        if ((b && !oy) || (cc && !oz)) continue;
                        const int o = T::CX * (b + T::CY * cc);
                        X[b][cc] = ox ? 0.5f * (c[o] + c[o + 1]) : c[o];
                    }
                float Yv[2];
#pragma unroll
                for (int cc = 0; cc < 2; ++cc) Yv[cc] = oy ? 0.5f * (X[0][cc] + X[1][cc]) : X[0][cc];
                const float v = oz ? 0.5f * (Yv[0] + Yv[1]) : Yv[0];
                sX[f * T::SN + s] = ok ? v : 0.0f;
            }
        }
    }
    if constexpr (mode_general(MODE)) {
        constexpr int IT = (T::SN + T::NT - 1) / T::NT;
        float tmp[IT][4];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            int s = tid + it * T::NT;
            int lx = s % T::SX, ly = (s / T::SX) % T::SY, lz = s / (T::SX * T::SY);
            bool ok;
            int64_t g = gnode(x0 - 2 + lx, y0 - 2 + ly, z0 - 2 + lz, ok);
            ok &= s < T::SN;
            g = ok ? g : 0; // absent nodes read node 0 and discard it
#pragma unroll
            for (int f = 0; f < 4; ++f) tmp[it][f] = x[f * nfn + g];
#pragma unroll
            for (int f = 0; f < 4; ++f) tmp[it][f] = ok ? tmp[it][f] : 0.0f;
        }
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            int s = tid + it * T::NT;
            if (s < T::SN)
#pragma unroll
                for (int f = 0; f < 4; ++f) sX[f * T::SN + s] = tmp[it][f];
        }
    }
    auto stage_v = [&](const float *__restrict__ src, float *dst) {
        constexpr int IT = (T::VN + T::NT - 1) / T::NT;
        float tmp[IT][3];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            int s = tid + it * T::NT;
            int lx = s % T::VX, ly = (s / T::VX) % T::VY, lz = s / (T::VX * T::VY);
            bool ok;
            int64_t g = gnode(x0 - 1 + lx, y0 - 1 + ly, z0 - 1 + lz, ok);
            ok &= s < T::VN;
            g = ok ? g : 0; // absent nodes read node 0 and discard it
#pragma unroll
            for (int f = 0; f < 3; ++f) tmp[it][f] = src[f * nfn + g];
#pragma unroll
            for (int f = 0; f < 3; ++f) tmp[it][f] = ok ? tmp[it][f] : 0.0f;
        }
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            int s = tid + it * T::NT;
            if (s < T::VN)
#pragma unroll
                for (int f = 0; f < 3; ++f) dst[f * T::VN + s] = tmp[it][f];
        }
    };
    if constexpr (!mode_against_b(MODE)) {
        stage_v(MODE != MODE_RHS ? vp : x, sV);
        if (fmid) stage_v(fmid, sF);
    }
    for (int s = tid; s < 8 * T::NCELL; s += T::NT) {
        sCell[s] = 0.0f;
        if constexpr (mode_general(MODE)) sCor[s] = 0.0f;
        if constexpr (RHS_OUT) sRhs[s] = 0.0f;
    }
    __syncthreads();

    const int ncx = 2 * m.n[0], ncy = 2 * m.n[1], ncz = 2 * m.n[2]; // fine cells per axis
    const float ih0 = P.ih[0], ih1 = P.ih[1], ih2 = P.ih[2];

    // ---- this thread's cell: lower corner at origin - 1 + (ex, ey, ez) ----
    // The cells of the tile inside the domain form a box; thread e takes its
    // e-th cell, so the waves past the live count skip the cell work (a tile
    // on a non-periodic upper face owns one node layer and few live cells).
    // Cell integrals go to the cell's slot ce = ex + EX (ey + EY ez); the slots
    // of cells outside the domain stay zero.
    int elo[3], ecnt[3];
    {
        const int o3[3] = {x0, y0, z0}, n3[3] = {ncx, ncy, ncz}, E3[3] = {T::EX, T::EY, T::EZ};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int lo = 0, hi = E3[a] - 1;
            if (!m.per[a]) {
                lo = max(0, 1 - o3[a]);              // x0 - 1 + ex >= 0
                hi = min(E3[a] - 1, n3[a] - o3[a]);  // x0 - 1 + ex < cells
            }
            elo[a] = lo;
            ecnt[a] = max(1, hi - lo + 1);
        }
    }
    const int e = tid;
    const bool live = e < ecnt[0] * ecnt[1] * ecnt[2];
    const int ec = live ? e : 0;
    const int ex = elo[0] + ec % ecnt[0], ey = elo[1] + (ec / ecnt[0]) % ecnt[1], ez = elo[2] + ec / (ecnt[0] * ecnt[1]);
    const int ce = ex + T::EX * (ey + T::EY * ez);
    // offset of the cell inside its patch (the tile origin is even)
    const int ox = (ex + 1) & 1, oy = (ey + 1) & 1, oz = (ez + 1) & 1;
    // node slots of vertex j = a + 2b + 4c as base + offset, so the LDS
    // accesses take immediate offsets
    auto voff = [](int j) { return (j & 1) + T::VX * (((j >> 1) & 1) + T::VY * (j >> 2)); };
    auto xoff = [](int j) { return (j & 1) + T::SX * (((j >> 1) & 1) + T::SY * (j >> 2)); };
    auto coff = [](int j) { return 2 * ((j & 1) + T::SX * (((j >> 1) & 1) + T::SY * (j >> 2))); };
    const int vb = ex + T::VX * (ey + T::VY * ez);
    const int xb = (ex + 1) + T::SX * ((ey + 1) + T::SY * (ez + 1));
    const int cb = (ex + 1 - ox) + T::SX * ((ey + 1 - oy) + T::SY * (ez + 1 - oz));

    // ---- this thread's owned node: the 8 cells around it, in vertex order ----
    const bool owner = tid < T::NOWN;
    const int lx = tid % T::TX, ly = (tid / T::TX) % T::TY, lz = tid / (T::TX * T::TY);
    // cell (lx + 1 - a, ly + 1 - b, lz + 1 - c) has this node as vertex a + 2b + 4c
    const int nb = (lx + 1) + T::EX * ((ly + 1) + T::EY * (lz + 1));
    auto ncell = [](int j) { return -((j & 1) + T::EX * (((j >> 1) & 1) + T::EY * (j >> 2))); };
    float res[T::NACC];
    // RHS_OUT: the owned node's Rhs of the three momentum equations; a
    // Rhs integral staged in sRhs is summed in the barrier phase of the
    // next reduction that is given its destination rs
    float rhsv[3] = {0.0f, 0.0f, 0.0f};
    auto take_rhs = [&](float *rs) {
        if constexpr (RHS_OUT) {
            if (rs && owner) {
                float t = 0.0f;
#pragma unroll
                for (int j = 0; j < 8; ++j) t += sRhs[j * T::NCELL + nb + ncell(j)];
                *rs = t;
            }
        }
    };

    // Cell integrals of equation a -> LDS; the owners sum them.
    auto reduce = [&](const float c[8], float wq, float *rs = nullptr) -> float {
        if (live)
#pragma unroll
            for (int j = 0; j < 8; ++j) sCell[j * T::NCELL + ce] = c[j] * wq;
        __syncthreads();
        float s = 0.0f;
        if (owner)
#pragma unroll
            for (int j = 0; j < 8; ++j) s += sCell[j * T::NCELL + nb + ncell(j)];
        take_rhs(rs);
        __syncthreads();
        return s;
    };

    bool need = false, need_p = false;
    float xv[3][8]; // x~ at the Gauss points (both passes of the general residual)
    // tile-wide LPS decisions, the cell's LPS denominator (stabparams) and
    // pi v at its Gauss points (general residual)
    bool any_v = false, any_p = false;
    float den = 1.0f, piv[3][8], sx[2], sy[2], sz[2];
    // LPS corner sums of the owned patches: owned patch P = tid / 8, corner
    // j = tid % 8; cell of offset o = ox + 2 oy + 4 oz in patch (ppx, ppy,
    // ppz) is ex = 2 ppx + 1 + ox
    float corner[mode_general(MODE) ? 4 : 1] = {};
    const bool pown = mode_general(MODE) && tid < 8 * T::NP;
    const int pslot = tid >> 3, pj = tid & 7;
    const int ppx = pslot % T::NPX, ppy = (pslot / T::NPX) % T::NPY, ppz = pslot / (T::NPX * T::NPY);
    const int pcb = (2 * ppx + 1) + T::EX * ((2 * ppy + 1) + T::EY * (2 * ppz + 1));
    // halo cells (ex == 0 etc.) belong to a neighbour's patch
    const bool own_patch = ex >= 1 && ey >= 1 && ez >= 1;
    // equation a's cell integrals (own vertices c, patch corners cr) -> LDS;
    // the owners sum their 8 cells, the patch-corner threads the 8 cells of
    // their patch, after one barrier
    auto reduce_c = [&](const float c[8], const float cr[8], float wq, float &corner_out,
                        float *rs = nullptr) -> float {
        if (live)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                sCell[j * T::NCELL + ce] = c[j] * wq;
                sCor[j * T::NCELL + ce] = own_patch ? cr[j] * wq : 0.0f;
            }
        __syncthreads();
        float s = 0.0f;
        if (owner)
#pragma unroll
            for (int j = 0; j < 8; ++j) s += sCell[j * T::NCELL + nb + ncell(j)];
        if (pown) {
            float t = 0.0f;
#pragma unroll
            for (int o = 0; o < 8; ++o)
                t += sCor[pj * T::NCELL + pcb + (o & 1) + T::EX * (((o >> 1) & 1) + T::EY * (o >> 2))];
            corner_out = t;
        }
        take_rhs(rs);
        __syncthreads();
        return s;
    };
    // the cell's LPS denominator (stabparams: |v|_inf over its vertices), its
    // offsets in the patch and pi v at its Gauss points
    auto lps_setup = [&]() {
        patch_coords(ox, sx);
        patch_coords(oy, sy);
        patch_coords(oz, sz);
        if (live && (need || need_p)) {
            float vmax2 = 0.0f;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                float u0 = sX[0 * T::SN + xb + xoff(j)], u1 = sX[1 * T::SN + xb + xoff(j)],
                      u2 = sX[2 * T::SN + xb + xoff(j)];
                vmax2 = fmaxf(vmax2, u0 * u0 + u1 * u1 + u2 * u2);
            }
            den = P.nu * (1.0f / (P.hT * P.hT)) + sqrtf(vmax2) / P.hT + P.inv_dt;
        }
        if (live && need) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                float w[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) w[j] = sX[d * T::SN + cb + coff(j)];
                patch_val(w, sx, sy, sz, piv[d]);
            }
        }
    };
    if constexpr (MODE == MODE_RHS) {
        float w[3][8], wv[3][8];
        if (live) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
#pragma unroll
                for (int j = 0; j < 8; ++j) w[d][j] = sV[d * T::VN + vb + voff(j)];
                eval_val(w[d], wv[d]);
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // (1/k) v_a - 1/2 v . grad v_a (+ (f^{n-1} + f^n)/2) and -nu/2 grad v_a
            float acc[8];
            if (live) {
            float F[8], va[8], g0[8], g1[8], g2[8];
            eval_vg(w[a], ih0, ih1, ih2, va, g0, g1, g2);
            if (fmid) {
                float fv[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) fv[j] = sF[a * T::VN + vb + voff(j)];
                eval_val(fv, F);
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) F[q] = 0.0f;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                float conv = wv[0][q] * g0[q] + wv[1][q] * g1[q] + wv[2][q] * g2[q];
                F[q] += P.inv_dt * va[q] - 0.5f * conv;
                g0[q] *= -P.half_nu;
                g1[q] *= -P.half_nu;
                g2[q] *= -P.half_nu;
            }
            integrate<true, true, true>(F, g0, g1, g2, ih0, ih1, ih2, acc);
            }
            res[a] = reduce(acc, P.wq);
        }
    } else {
        // The LPS terms vanish identically where x~ on the patch equals its
        // patch interpolant.  When the vertex values and the interpolant
        // computed here agree bit for bit every LPS contribution of the cell
        // is exactly zero; the other cells get them in a second pass.
        // The delta terms depend on the velocity only and the alpha term on
        // the pressure only, so the two are decided separately: `need` for
        // the velocity (field by field until one differs; a wave whose cells
        // all differ in the first field skips the other two), `need_p` for
        // the pressure (the network corrects only the velocity, so on the
        // indicator's and the fallback's iterates the alpha term vanishes).
        if (mode_general(MODE) && live) {
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                if (d < 3 && need) continue;
                float cv[8], pw[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) cv[j] = sX[d * T::SN + cb + coff(j)];
                pi_vertices(cv, ox, oy, oz, pw);
                bool differs = false;
#pragma unroll
                for (int j = 0; j < 8; ++j) differs |= pw[j] != sX[d * T::SN + xb + xoff(j)];
                if (d < 3) need |= differs;
                else need_p = differs;
            }
        }
        // x~, vp and p~ at the Gauss points; divergence of x~
        float pv[3][8], pq[8], div[8];
        if (live) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                float w[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) w[j] = sX[d * T::SN + xb + xoff(j)];
                eval_val(w, xv[d]);
                if constexpr (mode_has_vp(MODE)) {
#pragma unroll
                    for (int j = 0; j < 8; ++j) w[j] = sV[d * T::VN + vb + voff(j)];
                    eval_val(w, pv[d]);
                }
            }
            float w[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) w[j] = sX[3 * T::SN + xb + xoff(j)];
            eval_val(w, pq);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) div[q] = 0.0f;
        // Against a given right-hand side on one box (the indicator's and the
        // fallback's form) the velocity LPS terms (delta) of a momentum
        // equation are evaluated with its Galerkin terms: the own-vertex part
        // is a flux -delta_T R v added to the viscous flux before the one
        // transpose to vertex integrals, the patch-corner part is reduced in
        // the same barrier phase.  The other forms, whose Galerkin pass holds
        // more values, evaluate them in a pass of their own below (merged,
        // they would spill registers).
        if constexpr (mode_general(MODE)) {
            any_v = __syncthreads_or(need);
            any_p = __syncthreads_or(need_p);
            if constexpr (DELTA_MERGED) lps_setup();
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float acc[8], cor[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) cor[j] = 0.0f;
            if (live) {
                float w[8], tmp[8], g0[8], g1[8], g2[8], G0[8], G1[8], G2[8], F[8];
                if constexpr (mode_has_vp(MODE)) {
                    // (1/k)(vp_a - v_a) (+ (f^{n-1} + f^n)/2) at the Gauss points
                    if (fmid) {
#pragma unroll
                        for (int j = 0; j < 8; ++j) w[j] = sF[a * T::VN + vb + voff(j)];
                        eval_val(w, F);
                    } else {
#pragma unroll
                        for (int q = 0; q < 8; ++q) F[q] = 0.0f;
                    }
#pragma unroll
                    for (int q = 0; q < 8; ++q) F[q] += P.inv_dt * (pv[a][q] - xv[a][q]);
                    // -1/2 vp . grad vp_a; the gradient also enters -nu/2 grad(vp_a + v_a)
#pragma unroll
                    for (int j = 0; j < 8; ++j) w[j] = sV[a * T::VN + vb + voff(j)];
                    eval_vg(w, ih0, ih1, ih2, tmp, G0, G1, G2);
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        F[q] -= 0.5f * (pv[0][q] * G0[q] + pv[1][q] * G1[q] + pv[2][q] * G2[q]);
                } else {
                    // the previous step's terms are in b: -(1/k) v_a only
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        F[q] = -P.inv_dt * xv[a][q];
                        G0[q] = G1[q] = G2[q] = 0.0f;
                    }
                }
                // -1/2 v . grad v_a, divergence
#pragma unroll
                for (int j = 0; j < 8; ++j) w[j] = sX[a * T::SN + xb + xoff(j)];
                eval_vg(w, ih0, ih1, ih2, tmp, g0, g1, g2);
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    F[q] -= 0.5f * (xv[0][q] * g0[q] + xv[1][q] * g1[q] + xv[2][q] * g2[q]);
                    if constexpr (mode_has_vp(MODE)) {
                        G0[q] = -P.half_nu * (G0[q] + g0[q]);
                        G1[q] = -P.half_nu * (G1[q] + g1[q]);
                        G2[q] = -P.half_nu * (G2[q] + g2[q]);
                    } else {
                        G0[q] = -P.half_nu * g0[q];
                        G1[q] = -P.half_nu * g1[q];
                        G2[q] = -P.half_nu * g2[q];
                    }
                }
                if constexpr (RHS_OUT) {
                    // Rhs(v) of this equation at the same velocity:
                    // (1/k) v_a - 1/2 v . grad v_a tested with phi and
                    // -nu/2 grad v_a (G here) with grad phi
                    float Fr[8], accr[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        Fr[q] = P.inv_dt * xv[a][q] - 0.5f * (xv[0][q] * g0[q] + xv[1][q] * g1[q] + xv[2][q] * g2[q]);
                    integrate<true, true, true>(Fr, G0, G1, G2, ih0, ih1, ih2, accr);
#pragma unroll
                    for (int j = 0; j < 8; ++j) sRhs[j * T::NCELL + ce] = accr[j] * P.wq;
                }
                const float *ga = a == 0 ? g0 : (a == 1 ? g1 : g2);
                float *Ga = a == 0 ? G0 : (a == 1 ? G1 : G2);
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    div[q] += ga[q];
                    Ga[q] += pq[q]; // + (p, d_a phi)
                }
                if constexpr (DELTA_MERGED) {
                    if (need) {
                        // -delta_T (R_a, v.grad phi - pi v.grad pi phi) with
                        // R_a = v.grad v_a - pi v.grad pi v_a
                        const float deltaT = P.delta0 / den;
                        float ca[8], HX[4], HY[4], HZ[4], C0[8], C1[8], C2[8];
#pragma unroll
                        for (int j = 0; j < 8; ++j) ca[j] = sX[a * T::SN + cb + coff(j)];
                        patch_grad(ca, sx, sy, sz, ih0, ih1, ih2, HX, HY, HZ);
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const int qa = q & 1, qb = (q >> 1) & 1, qc = q >> 2;
                            const float R = (xv[0][q] * g0[q] + xv[1][q] * g1[q] + xv[2][q] * g2[q]) -
                                            (piv[0][q] * HX[qb + 2 * qc] + piv[1][q] * HY[qa + 2 * qc] +
                                             piv[2][q] * HZ[qa + 2 * qb]);
                            const float dR = deltaT * R;
                            G0[q] -= dR * xv[0][q];
                            G1[q] -= dR * xv[1][q];
                            G2[q] -= dR * xv[2][q];
                            C0[q] = dR * piv[0][q];
                            C1[q] = dR * piv[1][q];
                            C2[q] = dR * piv[2][q];
                        }
                        patch_integrate_grad(C0, C1, C2, sx, sy, sz, ih0, ih1, ih2, cor);
                    }
                }
                integrate<true, true, true>(F, G0, G1, G2, ih0, ih1, ih2, acc);
            }
            float *rs = RHS_OUT ? &rhsv[a] : nullptr;
            if (DELTA_MERGED && any_v) res[a] = reduce_c(acc, cor, P.wq, corner[a], rs);
            else res[a] = reduce(acc, P.wq, rs);
        }
        // continuity: -(div v, xi)
        {
#pragma unroll
            for (int q = 0; q < 8; ++q) div[q] = -div[q];
            float acc[8];
            if (live) integrate<false, false, false>(div, nullptr, nullptr, nullptr, ih0, ih1, ih2, acc);
            res[3] = reduce(acc, P.wq);
        }
    }

    // ---- LPS terms not taken with the Galerkin pass ----
    bool any_lps = false;
    if constexpr (mode_general(MODE)) {
        any_lps = any_v || any_p;
        if constexpr (!DELTA_MERGED)
            if (any_lps) lps_setup();
        if (!DELTA_MERGED && any_v) {
            for (int a = 0; a < 3; ++a) {
                // R_a = v.grad v_a - pi v . grad pi v_a, tested with
                // v.grad phi (own vertices) and pi v . grad pi phi (patch
                // corners)
                float acc[8], cor[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) acc[j] = cor[j] = 0.0f;
                if (live && need) {
                    const float deltaT = P.delta0 / den;
                    float ca[8], va[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        ca[j] = sX[a * T::SN + cb + coff(j)];
                        va[j] = sX[a * T::SN + xb + xoff(j)];
                    }
                    float tmp[8], g0[8], g1[8], g2[8], HX[4], HY[4], HZ[4];
                    eval_vg(va, ih0, ih1, ih2, tmp, g0, g1, g2);
                    patch_grad(ca, sx, sy, sz, ih0, ih1, ih2, HX, HY, HZ);
                    float C0[8], C1[8], C2[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const int qa = q & 1, qb = (q >> 1) & 1, qc = q >> 2;
                        float R = (xv[0][q] * g0[q] + xv[1][q] * g1[q] + xv[2][q] * g2[q]) -
                                  (piv[0][q] * HX[qb + 2 * qc] + piv[1][q] * HY[qa + 2 * qc] +
                                   piv[2][q] * HZ[qa + 2 * qb]);
                        float dR = deltaT * R;
                        g0[q] = -dR * xv[0][q];
                        g1[q] = -dR * xv[1][q];
                        g2[q] = -dR * xv[2][q];
                        C0[q] = dR * piv[0][q];
                        C1[q] = dR * piv[1][q];
                        C2[q] = dR * piv[2][q];
                        tmp[q] = 0.0f;
                    }
                    integrate<true, true, true>(tmp, g0, g1, g2, ih0, ih1, ih2, acc);
                    patch_integrate_grad(C0, C1, C2, sx, sy, sz, ih0, ih1, ih2, cor);
                }
                res[a] += reduce_c(acc, cor, P.wq, corner[a]);
            }
        }
        if (any_p) {
            // -alpha_T (grad(p - pi p), grad(xi - pi xi)): own-vertex and
            // patch-corner parts
            float acc[8], cor[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] = cor[j] = 0.0f;
            if (live && need_p) {
                const float alphaT = P.alpha0 / den;
                float w[8], pw[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) w[j] = sX[3 * T::SN + cb + coff(j)];
                pi_vertices(w, ox, oy, oz, pw);
#pragma unroll
                for (int j = 0; j < 8; ++j) w[j] = sX[3 * T::SN + xb + xoff(j)] - pw[j];
                float tmp[8], g0[8], g1[8], g2[8];
                eval_vg(w, ih0, ih1, ih2, tmp, g0, g1, g2);
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    g0[q] *= -alphaT;
                    g1[q] *= -alphaT;
                    g2[q] *= -alphaT;
                    tmp[q] = 0.0f;
                }
                integrate<true, true, true>(tmp, g0, g1, g2, ih0, ih1, ih2, acc);
                float dv[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) dv[j] = -acc[j];
                pi_transpose(dv, ox, oy, oz, cor);
            }
            res[3] += reduce_c(acc, cor, P.wq, corner[3]);
        }
    }

    // ---- write owned nodes and patch corner sums ----
    if (owner) {
        int gi = x0 + lx, gj = y0 + ly, gk = z0 + lz;
        if (gi < m.nf[0] && gj < m.nf[1] && gk < m.nf[2]) {
            int64_t g = gi + (int64_t)m.nf[0] * (gj + (int64_t)m.nf[1] * gk);
            bool dir = on_dirichlet(m, gi, gj, gk);
            if constexpr (mode_against_b(MODE)) {
                // r = b - A(x): vp carries b [4][n_fine]
#pragma unroll
                for (int f = 0; f < 3; ++f) out[f * nfn + g] = dir ? 0.0f : bown[f] + res[f];
                out[3 * nfn + g] = bown[3] + res[3];
                if constexpr (RHS_OUT) {
                    if (b_save)
#pragma unroll
                        for (int f = 0; f < 4; ++f) b_save[f * nfn + g] = bown[f];
#pragma unroll
                    for (int f = 0; f < 3; ++f) b_io[f * nfn + g] = dir ? 0.0f : rhsv[f];
                    b_io[3 * nfn + g] = 0.0f;
                }
            } else {
#pragma unroll
                for (int f = 0; f < 3; ++f) out[f * nfn + g] = dir ? 0.0f : res[f];
                if constexpr (MODE != MODE_RHS) out[3 * nfn + g] = res[3];
                else out[3 * nfn + g] = 0.0f;
            }
            if constexpr (mode_prolongs(MODE)) {
                const int slot = (lx + 2) + T::SX * ((ly + 2) + T::SY * (lz + 2));
#pragma unroll
                for (int f = 0; f < 4; ++f) xt_out[f * nfn + g] = sX[f * T::SN + slot];
            }
        }
    }
    if constexpr (mode_general(MODE)) {
        // the tile's flag says whether its patches' corner sums were written
        if (tid == 0) *tflag = any_lps ? 1 : 0;
        if (pown && any_lps) {
            int PI = x0 / 2 + ppx, PJ = y0 / 2 + ppy, PK = z0 / 2 + ppz;
            if (PI < m.n[0] && PJ < m.n[1] && PK < m.n[2]) {
                int64_t M = PI + (int64_t)m.n[0] * (PJ + (int64_t)m.n[1] * PK);
                *(float4 *)(aux + M * 32 + 4 * pj) = make_float4(corner[0], corner[1], corner[2], corner[3]);
            }
        }
    }
}

// Tile order of a launch: the tiles that hold a full block of owned nodes
// come first (each XCD takes a contiguous range of them), then the partial
// tiles on the upper faces of non-periodic axes, which hold one node layer.
// With one full tile per compute unit in the first wave, the cheap partial
// tiles fill in after instead of doubling the critical path.  t in [0, F):
// full tile; t in [F, G): partial tiles, as the slabs bz >= Fz, then
// by >= Fy (bz < Fz), then bx >= Fx (by < Fy, bz < Fz).
__device__ __forceinline__ void tile_of(int64_t t64, const int G[3], const int F[3], int c[3]) {
    // tile counts fit 32 bits (a tile holds hundreds of the < 2^31 nodes), and
    // 32-bit divisions are a fraction of the 64-bit sequences
    const uint32_t t = (uint32_t)t64;
    const uint32_t g0 = G[0], g1 = G[1], f0 = F[0], f1 = F[1];
    const uint32_t nf = f0 * f1 * (uint32_t)F[2];
    if (t < nf) {
        const uint32_t q = t / f0;
        c[0] = (int)(t - q * f0);
        c[1] = (int)(q % f1);
        c[2] = (int)(q / f1);
        return;
    }
    uint32_t p = t - nf;
    const uint32_t r1 = (uint32_t)(G[2] - F[2]) * g0 * g1;
    if (p < r1) {
        const uint32_t q = p / g0;
        c[0] = (int)(p - q * g0);
        c[1] = (int)(q % g1);
        c[2] = F[2] + (int)(q / g1);
        return;
    }
    p -= r1;
    const uint32_t gy = g1 - f1;
    const uint32_t r2 = gy * g0 * (uint32_t)F[2];
    if (p < r2) {
        const uint32_t q = p / g0;
        c[0] = (int)(p - q * g0);
        c[1] = F[1] + (int)(q % gy);
        c[2] = (int)(q / gy);
        return;
    }
    p -= r2;
    const uint32_t gx = g0 - f0;
    const uint32_t q = p / gx;
    c[0] = F[0] + (int)(p - q * gx);
    c[1] = (int)(q % f1);
    c[2] = (int)(q / f1);
}

// The tiles of a block, in the order of tile_of: fn(c, tl) with c the tile
// coordinates and tl its index in the tile grid.  STRIDED = false: one tile
// per block (the grid covers the tiles); STRIDED = true: blocks walk the
// tiles with stride gridDim.x, for launches that a device flag may skip on a
// small grid.
template <int MODE, bool STRIDED, class Fn>
__device__ __forceinline__ void walk_tiles(const Mesh &m, Fn fn) {
    using T = ResTile<MODE>;
    const int G[3] = {(m.nf[0] + T::TX - 1) / T::TX, (m.nf[1] + T::TY - 1) / T::TY, (m.nf[2] + T::TZ - 1) / T::TZ};
    const int F[3] = {m.nf[0] / T::TX, m.nf[1] / T::TY, m.nf[2] / T::TZ};
    const int64_t nfull = (int64_t)F[0] * F[1] * F[2];
    const int64_t xf = NXCD * ((nfull + NXCD - 1) / NXCD);
    const int64_t nblk = xf + ((int64_t)G[0] * G[1] * G[2] - nfull);
    for (int64_t vb = blockIdx.x; vb < nblk; vb += STRIDED ? gridDim.x : nblk) {
        int64_t t;
        if (vb < xf) {
            t = xcd_item(vb, xf);
            if (t >= nfull) continue;
        } else {
            t = nfull + (vb - xf);
        }
        int c[3];
        tile_of(t, G, F, c);
        fn(c, c[0] + G[0] * (c[1] + G[1] * c[2]));
        if constexpr (STRIDED) __syncthreads(); // the tile's LDS reads are done before the next stages
    }
}

// The strided (predicated, fallback) forms run at three waves per SIMD: the
// right-hand side's would spill at six, and its skipped launches would then
// set up scratch memory for nothing.
template <int MODE, bool STRIDED = false>
__global__ void __launch_bounds__(ResTile<MODE>::NT, STRIDED ? 3 : ResTile<MODE>::WAVES_PER_SIMD)
    k_residual(Mesh m, ResParams P, const float *__restrict__ x, const float *__restrict__ vp,
               const float *__restrict__ fmid, float *__restrict__ out, float *__restrict__ aux,
               int *__restrict__ tflag, const int *__restrict__ flag, const double *__restrict__ xc,
               float *__restrict__ xt_out) {
    if (flag && *flag == 0) return; // predicated launch (fallback path not taken)
    walk_tiles<MODE, STRIDED>(m, [&](const int c[3], int tl) {
        residual_tile<MODE, MODE == MODE_RESB && !STRIDED>(m, P, c[0], c[1], c[2], x, vp, fmid, out, aux,
                                                            mode_general(MODE) ? tflag + tl : nullptr, xc, xt_out);
    });
}

// r = b - A(x) and, in place of b, the next right-hand side Rhs(v) at the
// same iterate (b_save, if not null, receives b as it was read).
__global__ void __launch_bounds__(ResTile<MODE_RESB>::NT, ResTile<MODE_RESB>::WAVES_PER_SIMD)
    k_residual_rhs_b(Mesh m, ResParams P, const float *__restrict__ x, float *__restrict__ out,
                     float *__restrict__ aux, int *__restrict__ tflag, float *b_io, float *__restrict__ b_save) {
    walk_tiles<MODE_RESB, false>(m, [&](const int c[3], int tl) {
        residual_tile<MODE_RESB, true, true>(m, P, c[0], c[1], c[2], x, nullptr, nullptr, out, aux, tflag + tl,
                                             nullptr, nullptr, b_io, b_save);
    });
}

// Launch size of a tile grid in the order of tile_of.
template <int MODE>
static unsigned tile_blocks(const Mesh &m) {
    using T = ResTile<MODE>;
    const int64_t g = (int64_t)((m.nf[0] + T::TX - 1) / T::TX) * ((m.nf[1] + T::TY - 1) / T::TY) *
                      ((m.nf[2] + T::TZ - 1) / T::TZ);
    const int64_t f = (int64_t)(m.nf[0] / T::TX) * (m.nf[1] / T::TY) * (m.nf[2] / T::TZ);
    return (unsigned)(xcd_blocks(f) + (g - f));
}

// Batched: one flat grid over the tiles of all boxes.  x is a 4-component
// iterate in the batch layout (the right-hand side reads its velocity
// part), vp has 3 components, out 4; aux holds 32 floats per patch.
template <int MODE>
__global__ void __launch_bounds__(ResTile<MODE>::NT, ResTile<MODE>::WAVES_PER_SIMD)
    k_residual_batch(const BoxDesc *__restrict__ D, int nbox, int64_t nfull, int64_t npart,
                     const float *__restrict__ x, const float *__restrict__ vp, float *__restrict__ out,
                     float *__restrict__ aux, int *__restrict__ tflag, const double *__restrict__ xc,
                     float *__restrict__ xt_out) {
    // full tiles of all boxes first (XCD-contiguous), then the partial ones
    const int64_t xf = NXCD * ((nfull + NXCD - 1) / NXCD);
    int b;
    int64_t t;
    if (blockIdx.x < xf) {
        const int64_t f = xcd_item(blockIdx.x, xf);
        if (f >= nfull) return;
        b = find_box(nbox, f, [&](int i) { return D[i].blk_full; });
        t = f - D[b].blk_full;
    } else {
        const int64_t q = blockIdx.x - xf;
        if (q >= npart) return;
        b = find_box(nbox, q, [&](int i) { return D[i].blk_part; });
        t = (int64_t)D[b].rfull[0] * D[b].rfull[1] * D[b].rfull[2] + (q - D[b].blk_part);
    }
    const BoxDesc &d = D[b];
    const Mesh m = d.m;
    const ResParams P = d.rp;
    int c[3];
    tile_of(t, d.rtiles, d.rfull, c);
    const int tl = c[0] + d.rtiles[0] * (c[1] + d.rtiles[1] * c[2]);
    (void)tl;
    const int bx = c[0], by = c[1], bz = c[2];
    residual_tile<MODE>(m, P, bx, by, bz, !mode_prolongs(MODE) ? x + 4 * d.off_fine : nullptr,
                        MODE == MODE_RHS ? nullptr : vp + (MODE == MODE_PRESB ? 4 : 3) * d.off_fine, nullptr,
                        out + 4 * d.off_fine, nullptr, nullptr,
                        mode_prolongs(MODE) ? xc + 4 * d.off_coarse : nullptr,
                        mode_prolongs(MODE) ? xt_out + 4 * d.off_fine : nullptr);
}

// Adds the corner (pi phi) parts of the LPS terms: a coarse vertex collects
// the per-patch sums of the patches it is a corner of, in ascending patch
// order.  aux[M][4 j + f]: corner j = A + 2B + 4C of patch M, field f.
__device__ __forceinline__ void lps_corner_node(const Mesh &m, int64_t t, const float *__restrict__ aux,
                                                const int *__restrict__ tflag, const int rt[3],
                                                float *__restrict__ r) {
    if (t >= m.n_coarse) return;
    uint32_t JK = fdiv((uint32_t)t, m.cx), I = (uint32_t)t - JK * m.nc[0];
    uint32_t K = fdiv(JK, m.cy), J = JK - K * m.nc[1];
    // patches with this vertex as a corner, per axis, ascending
    int P[3][2] = {}, L[3][2] = {}, cnt[3];
    const int C[3] = {(int)I, (int)J, (int)K};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int lo = C[a] - 1, hi = C[a];
        cnt[a] = 0;
        if (m.per[a]) {
            if (lo < 0) lo += m.n[a];
            if (lo < hi) { P[a][0] = lo; L[a][0] = 1; P[a][1] = hi; L[a][1] = 0; }
            else { P[a][0] = hi; L[a][0] = 0; P[a][1] = lo; L[a][1] = 1; }
            cnt[a] = 2;
        } else {
            if (lo >= 0) { P[a][cnt[a]] = lo; L[a][cnt[a]] = 1; ++cnt[a]; }
            if (hi < m.n[a]) { P[a][cnt[a]] = hi; L[a][cnt[a]] = 0; ++cnt[a]; }
        }
    }
    // a patch's corner sums exist when its residual tile had LPS work
    constexpr int PX = ResTile<MODE_RES>::NPX, PY = ResTile<MODE_RES>::NPY, PZ = ResTile<MODE_RES>::NPZ;
    // all 2 x 2 x 2 candidates (a fastest), their tile flags, corner sums
    // and the node's residual are requested at once; absent candidates read
    // patch 0 and are skipped in the sums, which run in the same order
    int fl[8];
    float4 v[8];
    bool valid[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int a = q & 1, b = (q >> 1) & 1, c = q >> 2;
        valid[q] = a < cnt[0] && b < cnt[1] && c < cnt[2];
        const int pa = valid[q] ? P[0][a] : 0, pb = valid[q] ? P[1][b] : 0, pc = valid[q] ? P[2][c] : 0;
        const int tl = pa / PX + rt[0] * (pb / PY + rt[1] * (pc / PZ));
        fl[q] = tflag[tl];
        const int64_t M = pa + (int64_t)m.n[0] * (pb + (int64_t)m.n[1] * pc);
        const int j = L[0][a] + 2 * L[1][b] + 4 * L[2][c];
        v[q] = *(const float4 *)(aux + M * 32 + 4 * j);
    }
    int gi = 2 * I, gj = 2 * J, gk = 2 * K;
    int64_t g = gi + (int64_t)m.nf[0] * (gj + (int64_t)m.nf[1] * gk);
    float rv[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) rv[f] = r[f * m.n_fine + g];
    float s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    bool any = false;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        if (!valid[q] || !fl[q]) continue;
        any = true;
        s[0] += v[q].x;
        s[1] += v[q].y;
        s[2] += v[q].z;
        s[3] += v[q].w;
    }
    if (!any) return;
    bool dir = on_dirichlet(m, gi, gj, gk);
#pragma unroll
    for (int f = 0; f < 3; ++f)
        if (!dir) r[f * m.n_fine + g] = rv[f] + s[f];
    r[3 * m.n_fine + g] = rv[3] + s[3];
}

__global__ void __launch_bounds__(256) k_lps_corners(Mesh m, const float *__restrict__ aux,
                                                     const int *__restrict__ tflag, int rt0, int rt1, int rt2,
                                                     float *__restrict__ r, const int *__restrict__ flag) {
    if (flag && *flag == 0) return;
    const int rt[3] = {rt0, rt1, rt2};
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m.n_coarse;
         t += (int64_t)gridDim.x * blockDim.x)
        lps_corner_node(m, t, aux, tflag, rt, r);
}

// Grid of a launch that a device flag may skip: a few workgroups per compute
// unit walk the work, so a launch that is not taken costs little.
static unsigned predicated_grid(unsigned full, const int *flag, unsigned per_cu) {
    if (!flag) return full;
    const unsigned cap = per_cu * (unsigned)device_cus();
    return full < cap ? full : cap;
}


ResParams make_params(const Mesh &m, const dnnmg_ns *ns) {
    ResParams P;
    P.inv_dt = (float)(1.0 / ns->dt);
    P.half_nu = (float)(0.5 * ns->nu);
    P.nu = (float)ns->nu;
    P.alpha0 = (float)ns->alpha0;
    P.delta0 = (float)ns->delta0;
    for (int a = 0; a < 3; ++a) P.ih[a] = (float)(1.0 / m.hd[a]);
    P.hT = (float)sqrt(m.hd[0] * m.hd[0] + m.hd[1] * m.hd[1] + m.hd[2] * m.hd[2]);
    P.wq = (float)(0.125 * m.hd[0] * m.hd[1] * m.hd[2]);
    return P;
}

static int check_ns(const dnnmg_ns *ns) {
    if (!ns) return fail(DNNMG_ERR_ARG, "ns is NULL");
    if (!(ns->dt > 0.0) || !(ns->nu >= 0.0) || !(ns->alpha0 >= 0.0) || !(ns->delta0 >= 0.0))
        return fail(DNNMG_ERR_ARG, "ns: need dt > 0, nu >= 0, alpha0 >= 0, delta0 >= 0");
    return DNNMG_OK;
}

template <int MODE>
dim3 res_grid(const Mesh &m) {
    using T = ResTile<MODE>;
    return dim3((m.nf[0] + T::TX - 1) / T::TX, (m.nf[1] + T::TY - 1) / T::TY,
                (m.nf[2] + T::TZ - 1) / T::TZ);
}

// LPS workspace of one box: corner sums (32 floats per patch), then one
// flag per residual tile.
static size_t up256(size_t b) { return (b + 255) / 256 * 256; }
size_t lps_ws_bytes(const Mesh &m) {
    dim3 g = res_grid<MODE_RES>(m);
    return up256(sizeof(float) * 32 * m.n_patches) + up256(sizeof(int) * (size_t)g.x * g.y * g.z);
}

int residual_launch(const Mesh &m, const dnnmg_ns *ns, const float *x, const float *vprev,
                    const float *fmid, float *r, float *aux, const int *flag, hipStream_t s) {
    ResParams P = make_params(m, ns);
    dim3 g = res_grid<MODE_RES>(m);
    int *tflag = (int *)((char *)aux + up256(sizeof(float) * 32 * m.n_patches));
    if (flag)
        k_residual<MODE_RES, true><<<predicated_grid(tile_blocks<MODE_RES>(m), flag, 2), ResTile<MODE_RES>::NT, 0,
                                     s>>>(m, P, x, vprev, fmid, r, aux, tflag, flag, nullptr, nullptr);
    else
        k_residual<MODE_RES><<<tile_blocks<MODE_RES>(m), ResTile<MODE_RES>::NT, 0, s>>>(m, P, x, vprev, fmid, r, aux,
                                                                                     tflag, nullptr, nullptr, nullptr);
    k_lps_corners<<<predicated_grid(blocks_for(m.n_coarse, 256), flag, 4), 256, 0, s>>>(m, aux, tflag, g.x, g.y, g.z,
                                                                                        r, flag);
    return hip_check(hipGetLastError(), "dnnmg_residual launch");
}

int residual_launch_b(const Mesh &m, const dnnmg_ns *ns, const float *x, const float *b, float *r, float *aux,
                      const int *flag, hipStream_t s) {
    ResParams P = make_params(m, ns);
    dim3 g = res_grid<MODE_RES>(m);
    int *tflag = (int *)((char *)aux + up256(sizeof(float) * 32 * m.n_patches));
    if (flag)
        k_residual<MODE_RESB, true><<<predicated_grid(tile_blocks<MODE_RESB>(m), flag, 2), ResTile<MODE_RESB>::NT, 0,
                                      s>>>(m, P, x, b, nullptr, r, aux, tflag, flag, nullptr, nullptr);
    else
        k_residual<MODE_RESB><<<tile_blocks<MODE_RESB>(m), ResTile<MODE_RESB>::NT, 0, s>>>(m, P, x, b, nullptr, r, aux,
                                                                                        tflag, nullptr, nullptr,
                                                                                        nullptr);
    k_lps_corners<<<predicated_grid(blocks_for(m.n_coarse, 256), flag, 4), 256, 0, s>>>(m, aux, tflag, g.x, g.y, g.z,
                                                                                        r, flag);
    return hip_check(hipGetLastError(), "dnnmg_residual_b launch");
}

// Tile grid of a box (rt) and its box of full tiles (rf).
void residual_tiles(const Mesh &m, int rt[3], int rf[3]) {
    using T = ResTile<MODE_RES>;
    dim3 g = res_grid<MODE_RES>(m);
    rt[0] = g.x;
    rt[1] = g.y;
    rt[2] = g.z;
    rf[0] = m.nf[0] / T::TX;
    rf[1] = m.nf[1] / T::TY;
    rf[2] = m.nf[2] / T::TZ;
}

void rhs_batch_launch(const BoxDesc *D, int nbox, int64_t nfull, int64_t npart, const float *v, float *b,
                      hipStream_t s) {
    k_residual_batch<MODE_RHS><<<(unsigned)(xcd_blocks(nfull) + npart), ResTile<MODE_RHS>::NT, 0, s>>>(
        D, nbox, nfull, npart, v, nullptr, b, nullptr, nullptr, nullptr, nullptr);
}

void prolong_residual_batch_launch(const BoxDesc *D, int nbox, int64_t nfull, int64_t npart, const double *xc,
                                   const float *vp, float *xt, float *r, hipStream_t s) {
    k_residual_batch<MODE_PRES><<<(unsigned)(xcd_blocks(nfull) + npart), ResTile<MODE_PRES>::NT, 0, s>>>(
        D, nbox, nfull, npart, nullptr, vp, r, nullptr, nullptr, xc, xt);
}

void prolong_residual_b_batch_launch(const BoxDesc *D, int nbox, int64_t nfull, int64_t npart, const double *xc,
                                     const float *b, float *xt, float *r, hipStream_t s) {
    k_residual_batch<MODE_PRESB><<<(unsigned)(xcd_blocks(nfull) + npart), ResTile<MODE_PRESB>::NT, 0, s>>>(
        D, nbox, nfull, npart, nullptr, b, r, nullptr, nullptr, xc, xt);
}

} // namespace dnnmg

using namespace dnnmg;

extern "C" size_t dnnmg_residual_workspace(const dnnmg_box *box) {
    Mesh m;
    if (make_mesh(box, &m)) return 0;
    return lps_ws_bytes(m);
}

extern "C" int dnnmg_residual(const dnnmg_box *box, const dnnmg_ns *ns, const float *x,
                              const float *vprev, const float *fmid, float *r, void *ws,
                              size_t ws_bytes, void *stream) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    if ((rc = check_ns(ns))) return rc;
    if (!x || !vprev || !r || !ws) return fail(DNNMG_ERR_ARG, "dnnmg_residual: NULL pointer");
    if (!aligned16(ws)) return fail(DNNMG_ERR_ARG, "dnnmg_residual: workspace not 16-byte aligned");
    if (ws_bytes < lps_ws_bytes(m))
        return fail(DNNMG_ERR_SHAPE, "dnnmg_residual: workspace %zu < %zu bytes", ws_bytes, lps_ws_bytes(m));
    return residual_launch(m, ns, x, vprev, fmid, r, (float *)ws, nullptr, (hipStream_t)stream);
}

extern "C" int dnnmg_residual_b(const dnnmg_box *box, const dnnmg_ns *ns, const float *x, const float *b, float *r,
                                void *ws, size_t ws_bytes, void *stream) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    if ((rc = check_ns(ns))) return rc;
    if (!x || !b || !r || !ws) return fail(DNNMG_ERR_ARG, "dnnmg_residual_b: NULL pointer");
    if (b == r) return fail(DNNMG_ERR_ARG, "dnnmg_residual_b: b and r must not alias");
    if (!aligned16(ws)) return fail(DNNMG_ERR_ARG, "dnnmg_residual_b: workspace not 16-byte aligned");
    if (ws_bytes < lps_ws_bytes(m))
        return fail(DNNMG_ERR_SHAPE, "dnnmg_residual_b: workspace %zu < %zu bytes", ws_bytes, lps_ws_bytes(m));
    return residual_launch_b(m, ns, x, b, r, (float *)ws, nullptr, (hipStream_t)stream);
}

extern "C" int dnnmg_residual_rhs_b(const dnnmg_box *box, const dnnmg_ns *ns, const float *x, float *b, float *r,
                                    float *b_save, void *ws, size_t ws_bytes, void *stream) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    if ((rc = check_ns(ns))) return rc;
    if (!x || !b || !r || !ws) return fail(DNNMG_ERR_ARG, "dnnmg_residual_rhs_b: NULL pointer");
    if (b == r || (const float *)b == x || (const float *)r == x)
        return fail(DNNMG_ERR_ARG, "dnnmg_residual_rhs_b: x, b and r must not alias");
    if (b_save && (b_save == b || b_save == r || (const float *)b_save == x))
        return fail(DNNMG_ERR_ARG, "dnnmg_residual_rhs_b: b_save must not alias x, b or r");
    if (!aligned16(ws)) return fail(DNNMG_ERR_ARG, "dnnmg_residual_rhs_b: workspace not 16-byte aligned");
    if (ws_bytes < lps_ws_bytes(m))
        return fail(DNNMG_ERR_SHAPE, "dnnmg_residual_rhs_b: workspace %zu < %zu bytes", ws_bytes, lps_ws_bytes(m));
    hipStream_t s = (hipStream_t)stream;
    ResParams P = make_params(m, ns);
    dim3 g = res_grid<MODE_RES>(m);
    float *aux = (float *)ws;
    int *tflag = (int *)((char *)aux + up256(sizeof(float) * 32 * m.n_patches));
    k_residual_rhs_b<<<tile_blocks<MODE_RESB>(m), ResTile<MODE_RESB>::NT, 0, s>>>(m, P, x, r, aux, tflag, b, b_save);
    k_lps_corners<<<blocks_for(m.n_coarse, 256), 256, 0, s>>>(m, aux, tflag, g.x, g.y, g.z, r, nullptr);
    return hip_check(hipGetLastError(), "dnnmg_residual_rhs_b launch");
}

// ------------------------------------------- allocation-free residual_b --
// Scratch of dnnmg_residual_b_noalloc: the LPS corner sums and tile flags of
// one box, in a device array of fixed size that every GPU the library runs
// on holds until the process ends.  Host code never passes the array's name
// to a kernel (on the host it is a stand-in, not a device address): the
// device address is looked up once per device and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[DNNMG_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of this device's scratch array (looked up on the first call
// on the device, with the device current).
int scratch_address(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_check(e, "dnnmg_residual_b_noalloc: hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES)
        return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_residual_b_noalloc: device index %d >= %d", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_check(e, "dnnmg_residual_b_noalloc: hipGetSymbolAddress(scratch)");
        if (!p) return fail(DNNMG_ERR_HIP, "dnnmg_residual_b_noalloc: scratch has no device address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DNNMG_OK;
}
} // namespace

extern "C" int dnnmg_residual_b_noalloc(const dnnmg_box *box, const dnnmg_ns *ns, const float *x, const float *b,
                                        float *r, void *stream) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    if ((rc = check_ns(ns))) return rc;
    if (!x || !b || !r) return fail(DNNMG_ERR_ARG, "dnnmg_residual_b_noalloc: NULL pointer");
    if (b == r) return fail(DNNMG_ERR_ARG, "dnnmg_residual_b_noalloc: b and r must not alias");
    const size_t need = lps_ws_bytes(m);
    if (need > (size_t)DNNMG_NOALLOC_SCRATCH_BYTES)
        return fail(DNNMG_ERR_SHAPE,
                    "dnnmg_residual_b_noalloc: the box needs %zu bytes of scratch, more than the %zu built in "
                    "(%lld patches; use dnnmg_residual_b with a workspace)",
                    need, (size_t)DNNMG_NOALLOC_SCRATCH_BYTES, (long long)m.n_patches);
    void *ws = nullptr;
    if ((rc = scratch_address(&ws))) return rc;
    // every tile of this box writes its flag before the corner kernel reads
    // it, and corner sums are read only under a set flag, so nothing left by
    // an earlier call is read: no clearing is needed
    return residual_launch_b(m, ns, x, b, r, (float *)ws, nullptr, (hipStream_t)stream);
}

extern "C" int dnnmg_rhs(const dnnmg_box *box, const dnnmg_ns *ns, const float *v, const float *fmid,
                         float *b, void *stream) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    if ((rc = check_ns(ns))) return rc;
    if (!v || !b) return fail(DNNMG_ERR_ARG, "dnnmg_rhs: NULL pointer");
    ResParams P = make_params(m, ns);
    k_residual<MODE_RHS><<<tile_blocks<MODE_RHS>(m), ResTile<MODE_RHS>::NT, 0, (hipStream_t)stream>>>(
        m, P, v, nullptr, fmid, b, nullptr, nullptr, nullptr, nullptr, nullptr);
    return hip_check(hipGetLastError(), "dnnmg_rhs launch");
}

extern "C" int dnnmg_rhs_if(const dnnmg_box *box, const dnnmg_ns *ns, const float *v, const float *fmid, float *b,
                            const int *flag, void *stream) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    if ((rc = check_ns(ns))) return rc;
    if (!v || !b || !flag) return fail(DNNMG_ERR_ARG, "dnnmg_rhs_if: NULL pointer");
    ResParams P = make_params(m, ns);
    k_residual<MODE_RHS, true><<<predicated_grid(tile_blocks<MODE_RHS>(m), flag, 2), ResTile<MODE_RHS>::NT, 0,
                                 (hipStream_t)stream>>>(m, P, v, nullptr, fmid, b, nullptr, nullptr, flag, nullptr,
                                                        nullptr);
    return hip_check(hipGetLastError(), "dnnmg_rhs_if launch");
}

extern "C" int dnnmg_prolong_residual_b(const dnnmg_box *box, const dnnmg_ns *ns, const double *xc,
                                        const float *b, float *xt, float *r, void *stream) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    if ((rc = check_ns(ns))) return rc;
    if (!xc || !b || !xt || !r) return fail(DNNMG_ERR_ARG, "dnnmg_prolong_residual_b: NULL pointer");
    if (b == r) return fail(DNNMG_ERR_ARG, "dnnmg_prolong_residual_b: b and r must not alias");
    ResParams P = make_params(m, ns);
    k_residual<MODE_PRESB><<<tile_blocks<MODE_PRESB>(m), ResTile<MODE_PRESB>::NT, 0, (hipStream_t)stream>>>(
        m, P, nullptr, b, nullptr, r, nullptr, nullptr, nullptr, xc, xt);
    return hip_check(hipGetLastError(), "dnnmg_prolong_residual_b launch");
}

extern "C" int dnnmg_prolong_residual(const dnnmg_box *box, const dnnmg_ns *ns, const double *xc,
                                      const float *vprev, const float *fmid, float *xt, float *r, void *stream) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    if ((rc = check_ns(ns))) return rc;
    if (!xc || !vprev || !xt || !r) return fail(DNNMG_ERR_ARG, "dnnmg_prolong_residual: NULL pointer");
    ResParams P = make_params(m, ns);
    k_residual<MODE_PRES><<<tile_blocks<MODE_PRES>(m), ResTile<MODE_PRES>::NT, 0, (hipStream_t)stream>>>(
        m, P, nullptr, vprev, fmid, r, nullptr, nullptr, nullptr, xc, xt);
    return hip_check(hipGetLastError(), "dnnmg_prolong_residual launch");
}

