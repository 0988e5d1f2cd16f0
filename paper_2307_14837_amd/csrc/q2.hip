// DNN-MG fine level with the paper's discretisation: equal-order Q2 elements
// for velocity and pressure on isoparametric hexahedra, local projection
// stabilisation with pi_h the interpolation Q2 -> Q1 (arXiv 2307.14837,
// Sec. 2.2, eq. (disc:ns)), the Crank-Nicolson system of Sec. 2.3, eq.
// (4cranknicholson3) with the parameters of eq. (stabparams), the transfer of
// Algorithm 1 between the Q2 spaces of levels L and L + 1, and the patch
// inputs of Sec. 4.2 on the fine Q2 elements.
//
// Mesh: the box topology of the Q1 kernels (n elements = patches per axis,
// 2n + 1 nodes per axis, no periodic axes); element (I, J, K) holds the 27
// nodes (2I + a, 2J + b, 2K + c) and maps the reference cube by the Q2
// interpolation of their positions (FP64 [3][n_nodes], read as offsets from
// the element's first vertex so the Jacobian keeps FP32 accuracy).
//
// Element integrals (3 x 3 x 3 Gauss points) run inside one workgroup of 9
// elements x 27 threads, with the tensor-product structure of the element
// used in both directions (sum factorisation):
//   1. the node values of the coordinates and fields are taken to values and
//      reference gradients at the 27 points by three 1-D passes (z, y, x),
//      each a thread per (node or point) index triple and 3 terms;
//   2. one thread per quadrature point evaluates the Jacobian, its inverse,
//      the physical gradients and the Q1 interpolants and reduces every term
//      of the weak form to 7 coefficients per equation: the factor of the
//      test function, of its reference gradient and of the reference
//      gradient of its Q1 interpolant (nonzero for vertex nodes only);
//   3. three 1-D passes (x, y, z) sum those coefficients against the shape
//      functions (and, for the vertices, against the linear functions of the
//      Q1 space) into the 27 test nodes.
// Element vectors go to a workspace (108 floats per element, stored by local
// node, from one launch over all elements); a second launch sums each
// node's at most 8 entries in a fixed order, without atomics, so results
// are reproducible bit for bit.
#include "common.hpp"
#include "lowp.hpp"

#include <math.h>

namespace dnnmg {

#define STREAM ((hipStream_t)stream)

struct Q2Params {
    float inv_dt, half_nu, nu, alpha0, delta0;
};

// 1-D quadratic Lagrange functions on [0,1] (nodes 0, 1/2, 1), their
// derivatives and the linear functions of the Q1 space, at the three
// Gauss-Legendre points 1/2 - sqrt(15)/10, 1/2, 1/2 + sqrt(15)/10.
__device__ __forceinline__ float gauss_pt(int g) {
    const float s = 0.38729833462074170f; // sqrt(3/5) / 2
    return g == 0 ? 0.5f - s : (g == 1 ? 0.5f : 0.5f + s);
}
__device__ __forceinline__ float gauss_wt(int g) { return g == 1 ? (8.0f / 18.0f) : (5.0f / 18.0f); }
__device__ __forceinline__ float quad_fn(int a, float t) {
    return a == 0 ? 2.0f * (t - 0.5f) * (t - 1.0f) : (a == 1 ? 4.0f * t * (1.0f - t) : 2.0f * t * (t - 0.5f));
}
__device__ __forceinline__ float quad_dfn(int a, float t) {
    return a == 0 ? 4.0f * t - 3.0f : (a == 1 ? 4.0f - 8.0f * t : 4.0f * t - 1.0f);
}

constexpr int Q2_EPB = 8;    // elements per workgroup: one per 32-lane half of each of its 4 waves
constexpr int Q2_NT = 256;   // threads per workgroup (27 active per half wave)
constexpr int Q2_NSTR = 8;   // per node: 3 offsets, pad, 4 fields
constexpr int Q2_CSTR = 28;  // per point: 4 equations x 7 coefficients

// APPLY: A(x); RHS: Rhs(v, fmid); BOTH: A(x) and Rhs(v) (no forcing) at the
// same iterate, sharing the staging, the interpolation and the point terms.
enum { Q2_APPLY = 0, Q2_RHS = 1, Q2_BOTH = 2 };

// An element's 27 threads lie in one 32-lane half of a wave and exchange
// data only among themselves through LDS, so the phases of the element
// kernel are ordered within the wave: LDS instructions of a wave execute in
// order, and the fences keep the compiler from moving LDS accesses across
// the point (no workgroup barrier; the waves of a workgroup run freely).
__device__ __forceinline__ void q2_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-element LDS arena (floats): the interpolation passes keep 2 and then 3
// arrays of 27 per quantity (945 for 7 quantities); the test contraction
// keeps the 28 coefficients of each point (0..755), the x-pass sums
// (756..1079) and the vertex x-pass sums (1080..1403), then the y-pass sums
// over the coefficients' region.
constexpr int Q2_ARENA = 1404;
constexpr int Q2_P = 756, Q2_A = 1080;
// element vectors of one workgroup in the workspace: [27 e + node][slot]
constexpr int Q2_GROUP = 108 * Q2_EPB;
constexpr int Q2_GROUP_BOTH = 189 * Q2_EPB; // 4 + 3 equations

// MODE Q2_APPLY: the element vector of A(x) (x = u, v, w, p); MODE Q2_RHS:
// that of Rhs(x = velocity, fmid).  The element vectors of workgroup g
// (elements 9g .. 9g + 8) are stored as one block of 972 floats,
// E[972 g + 9 (27 e + node) + slot], so the stores are contiguous and the
// per-node sum reads neighbouring elements at neighbouring addresses.  Thread
// l = (l0, l1, l2) (l0 + 3 l1 + 9 l2) of an element plays node (a, b, c) or
// quadrature point (q0, q1, q2) or a mix of both in the 1-D passes below.
template <int MODE>
__global__ void __launch_bounds__(Q2_NT, 3) k_q2_element(Mesh m, Q2Params P, const double *__restrict__ X,
                                                      const float *__restrict__ x, const float *__restrict__ fmid,
                                                      float *__restrict__ E) {
    // quantities interpolated to the points: 3 coordinates (gradients only),
    // u, v, w (values and gradients), then p (APPLY) or the 3 forcing
    // components (RHS, values only)
    constexpr bool HAS_A = MODE != Q2_RHS; // the iterate's terms (and p, the LPS terms)
    constexpr int NQ = HAS_A ? 7 : 9;
    constexpr int NE = HAS_A ? 4 : 3; // equations of the first test contraction
    __shared__ __align__(16) float sQ[Q2_EPB][NQ][27];
    constexpr int ARENA = HAS_A ? Q2_ARENA : 5 * NQ * 27; // RHS: interpolation of 9 quantities
    __shared__ __align__(16) float sW[Q2_EPB][ARENA];
    __shared__ float sV[Q2_EPB][27]; // |v|^2 per node
    __shared__ float sH[Q2_EPB][8];  // largest squared vertex distance per vertex

    const int tid = threadIdx.x;
    const int s = tid >> 5, l = tid & 31;
    const bool active_t = l < 27;
    const int64_t el = (int64_t)blockIdx.x * Q2_EPB + s;
    const bool valid = active_t && el < m.n_patches;
    int I = 0, J = 0, K = 0;
    if (valid) {
        I = (int)(el % m.n[0]);
        J = (int)((el / m.n[0]) % m.n[1]);
        K = (int)(el / ((int64_t)m.n[0] * m.n[1]));
    }
    const int64_t nf = m.n_fine;
    const int l0 = l % 3, l1 = (l / 3) % 3, l2 = l / 9;
    const int gi = 2 * I + l0, gj = 2 * J + l1, gk = 2 * K + l2;
    const int64_t g = gi + (int64_t)m.nf[0] * (gj + (int64_t)m.nf[1] * gk);
    float *W = sW[s];

    // ---- stage the element's node positions (relative to its first vertex) and fields
    if (valid) {
        const int64_t g0 = 2 * I + (int64_t)m.nf[0] * (2 * J + (int64_t)m.nf[1] * (2 * K));
#pragma unroll
        for (int d = 0; d < 3; ++d) sQ[s][d][l] = (float)(X[d * nf + g] - X[d * nf + g0]);
        float v2 = 0.0f;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const float val = x[f * nf + g];
            sQ[s][3 + f][l] = val;
            v2 += val * val;
        }
        if (HAS_A) {
            sQ[s][6][l] = x[3 * nf + g];
        } else {
#pragma unroll
            for (int f = 0; f < 3; ++f) sQ[s][6 + f][l] = fmid ? fmid[f * nf + g] : 0.0f;
        }
        sV[s][l] = v2;
    }
    q2_wave_sync();

    float alphaT = 0.0f, deltaT = 0.0f;
    if (HAS_A) {
        // h_T = the largest vertex distance; |v|_inf = the largest |v| over the 27 nodes
        if (valid && l < 8) {
            const int vi = 2 * (l & 1) + 6 * ((l >> 1) & 1) + 18 * ((l >> 2) & 1);
            float best = 0.0f;
            for (int w = l + 1; w < 8; ++w) {
                const int wi = 2 * (w & 1) + 6 * ((w >> 1) & 1) + 18 * ((w >> 2) & 1);
                float d2 = 0.0f;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const float e = sQ[s][d][wi] - sQ[s][d][vi];
                    d2 += e * e;
                }
                best = fmaxf(best, d2);
            }
            sH[s][l] = best;
        }
    }

    // ---- interpolation, pass z: thread (a, b, q2): values and z-derivatives
    if (valid) {
        const float t = gauss_pt(l2);
        const float Q0 = quad_fn(0, t), Q1 = quad_fn(1, t), Q2 = quad_fn(2, t);
        const float D0 = quad_dfn(0, t), D1 = quad_dfn(1, t), D2 = quad_dfn(2, t);
        const int n0 = l0 + 3 * l1;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const float u0 = sQ[s][q][n0], u1 = sQ[s][q][n0 + 9], u2 = sQ[s][q][n0 + 18];
            W[(2 * q) * 27 + l] = u0 * Q0 + u1 * Q1 + u2 * Q2;
            if (HAS_A || q < 6) W[(2 * q + 1) * 27 + l] = u0 * D0 + u1 * D1 + u2 * D2;
        }
    }
    q2_wave_sync();
    if (HAS_A && valid) {
        float h2 = 0.0f, v2 = 0.0f;
#pragma unroll
        for (int v = 0; v < 8; ++v) h2 = fmaxf(h2, sH[s][v]);
#pragma unroll
        for (int n = 0; n < 27; ++n) v2 = fmaxf(v2, sV[s][n]);
        const float hT = sqrtf(h2);
        const float den = P.nu / h2 + sqrtf(v2) / hT + P.inv_dt;
        alphaT = P.alpha0 / den;
        deltaT = P.delta0 / den;
    }
    // ---- pass y: thread (a, q1, q2): value, y-derivative, and the z-derivative carried
    constexpr int YOFF = 2 * NQ * 27;
    if (valid) {
        const float t = gauss_pt(l1);
        const float Q0 = quad_fn(0, t), Q1 = quad_fn(1, t), Q2 = quad_fn(2, t);
        const float D0 = quad_dfn(0, t), D1 = quad_dfn(1, t), D2 = quad_dfn(2, t);
        const int n0 = l0 + 9 * l2;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const float *z = W + (2 * q) * 27 + n0;
            const float z0 = z[0], z1 = z[3], z2 = z[6];
            W[YOFF + (3 * q) * 27 + l] = z0 * Q0 + z1 * Q1 + z2 * Q2;
            if (HAS_A || q < 6) {
                const float *w = W + (2 * q + 1) * 27 + n0;
                W[YOFF + (3 * q + 1) * 27 + l] = z0 * D0 + z1 * D1 + z2 * D2;
                W[YOFF + (3 * q + 2) * 27 + l] = w[0] * Q0 + w[3] * Q1 + w[6] * Q2;
            }
        }
    }
    q2_wave_sync();

    // ---- pass x: thread (q0, q1, q2) = its quadrature point
    float co[4][7];
    float coR[3][4]; // BOTH: the Rhs's factors of phi and of its reference gradient
    if (valid) {
        const float t0 = gauss_pt(l0), t1 = gauss_pt(l1), t2 = gauss_pt(l2);
        const float Q0 = quad_fn(0, t0), Q1 = quad_fn(1, t0), Q2 = quad_fn(2, t0);
        const float D0 = quad_dfn(0, t0), D1 = quad_dfn(1, t0), D2 = quad_dfn(2, t0);
        const int n0 = 3 * l1 + 9 * l2;
        float val[NQ], grd[NQ][3];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const float *y0 = W + YOFF + (3 * q) * 27 + n0;
            val[q] = y0[0] * Q0 + y0[1] * Q1 + y0[2] * Q2;
            if (HAS_A || q < 6) {
                const float *y1 = W + YOFF + (3 * q + 1) * 27 + n0;
                const float *y2 = W + YOFF + (3 * q + 2) * 27 + n0;
                grd[q][0] = y0[0] * D0 + y0[1] * D1 + y0[2] * D2;
                grd[q][1] = y1[0] * Q0 + y1[1] * Q1 + y1[2] * Q2;
                grd[q][2] = y2[0] * Q0 + y2[1] * Q1 + y2[2] * Q2;
            }
        }
        float Jm[3][3], v[3], gv[3][3];
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                Jm[d][e] = grd[d][e];
                gv[d][e] = grd[3 + d][e];
            }
#pragma unroll
        for (int d = 0; d < 3; ++d) v[d] = val[3 + d];
        const float det = Jm[0][0] * (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1]) -
                          Jm[0][1] * (Jm[1][0] * Jm[2][2] - Jm[1][2] * Jm[2][0]) +
                          Jm[0][2] * (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]);
        const float id = 1.0f / det;
        float Ji[3][3]; // Ji[e][d] = d xi_e / d x_d
        Ji[0][0] = (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1]) * id;
        Ji[0][1] = (Jm[0][2] * Jm[2][1] - Jm[0][1] * Jm[2][2]) * id;
        Ji[0][2] = (Jm[0][1] * Jm[1][2] - Jm[0][2] * Jm[1][1]) * id;
        Ji[1][0] = (Jm[1][2] * Jm[2][0] - Jm[1][0] * Jm[2][2]) * id;
        Ji[1][1] = (Jm[0][0] * Jm[2][2] - Jm[0][2] * Jm[2][0]) * id;
        Ji[1][2] = (Jm[0][2] * Jm[1][0] - Jm[0][0] * Jm[1][2]) * id;
        Ji[2][0] = (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]) * id;
        Ji[2][1] = (Jm[0][1] * Jm[2][0] - Jm[0][0] * Jm[2][1]) * id;
        Ji[2][2] = (Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0]) * id;
        const float w = gauss_wt(l0) * gauss_wt(l1) * gauss_wt(l2) * det;

        // physical gradients: grad f = Ji^T (reference gradient)
        float G[3][3];
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int d = 0; d < 3; ++d) G[q][d] = gv[q][0] * Ji[0][d] + gv[q][1] * Ji[1][d] + gv[q][2] * Ji[2][d];
        float conv[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) conv[q] = v[0] * G[q][0] + v[1] * G[q][1] + v[2] * G[q][2];

        if (HAS_A) {
            if (MODE == Q2_BOTH) {
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    coR[q][0] = w * (P.inv_dt * v[q] - 0.5f * conv[q]);
#pragma unroll
                    for (int e = 0; e < 3; ++e)
                        coR[q][1 + e] = -w * P.half_nu * (Ji[e][0] * G[q][0] + Ji[e][1] * G[q][1] + Ji[e][2] * G[q][2]);
                }
            }
            const float p = val[6];
            // Q1 interpolants from the 8 vertices (local nodes 2va + 6vb + 18vc)
            const float Lx[2] = {1.0f - t0, t0}, Ly[2] = {1.0f - t1, t1}, Lz[2] = {1.0f - t2, t2};
            float pv[3] = {}, gpv[3][3] = {}, gpp[3] = {};
#pragma unroll
            for (int vtx = 0; vtx < 8; ++vtx) {
                const int va = vtx & 1, vb = (vtx >> 1) & 1, vc = (vtx >> 2) & 1;
                const int vn = 2 * va + 6 * vb + 18 * vc;
                const float sx = va ? 1.0f : -1.0f, sy = vb ? 1.0f : -1.0f, sz = vc ? 1.0f : -1.0f;
                const float L = Lx[va] * Ly[vb] * Lz[vc];
                const float dL[3] = {sx * Ly[vb] * Lz[vc], Lx[va] * sy * Lz[vc], Lx[va] * Ly[vb] * sz};
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const float fq = sQ[s][3 + q][vn];
                    pv[q] += fq * L;
#pragma unroll
                    for (int e = 0; e < 3; ++e) gpv[q][e] += fq * dL[e];
                }
                const float fp = sQ[s][6][vn];
#pragma unroll
                for (int e = 0; e < 3; ++e) gpp[e] += fp * dL[e];
            }
            float gpi[3][3], gpp_phys[3], gp_phys[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    gpi[q][d] = gpv[q][0] * Ji[0][d] + gpv[q][1] * Ji[1][d] + gpv[q][2] * Ji[2][d];
                gpp_phys[d] = gpp[0] * Ji[0][d] + gpp[1] * Ji[1][d] + gpp[2] * Ji[2][d];
                gp_phys[d] = grd[6][0] * Ji[0][d] + grd[6][1] * Ji[1][d] + grd[6][2] * Ji[2][d];
            }
            // momentum rows: factor of phi, of grad phi and of grad pi phi (reference)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const float R = conv[q] - (pv[0] * gpi[q][0] + pv[1] * gpi[q][1] + pv[2] * gpi[q][2]);
                const float dr = deltaT * R;
                float gph[3], gpy[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    gph[d] = w * (P.half_nu * G[q][d] + dr * v[d] - (d == q ? p : 0.0f));
                    gpy[d] = -w * dr * pv[d];
                }
                co[q][0] = w * (P.inv_dt * v[q] + 0.5f * conv[q]);
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    co[q][1 + e] = Ji[e][0] * gph[0] + Ji[e][1] * gph[1] + Ji[e][2] * gph[2];
                    co[q][4 + e] = Ji[e][0] * gpy[0] + Ji[e][1] * gpy[1] + Ji[e][2] * gpy[2];
                }
            }
            // continuity row: (div v, xi) + alpha_T (grad(p - pi p), grad(xi - pi xi))
            float ga[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) ga[d] = w * alphaT * (gp_phys[d] - gpp_phys[d]);
            co[3][0] = w * (G[0][0] + G[1][1] + G[2][2]);
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                co[3][1 + e] = Ji[e][0] * ga[0] + Ji[e][1] * ga[1] + Ji[e][2] * ga[2];
                co[3][4 + e] = -co[3][1 + e];
            }
        } else {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                co[q][0] = w * (P.inv_dt * v[q] - 0.5f * conv[q] + val[6 + q]);
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    co[q][1 + e] = -w * P.half_nu * (Ji[e][0] * G[q][0] + Ji[e][1] * G[q][1] + Ji[e][2] * G[q][2]);
                    co[q][4 + e] = 0.0f;
                }
            }
#pragma unroll
            for (int k = 0; k < 7; ++k) co[3][k] = 0.0f;
        }
    }
    q2_wave_sync(); // every pass-x read of the arena is done
    if (valid) {
        // the 28 coefficients of the point, equation-major (7 per equation)
        float4 *c4 = reinterpret_cast<float4 *>(W + 28 * l);
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            float t4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) t4[u] = co[(4 * k + u) / 7][(4 * k + u) % 7];
            c4[k] = make_float4(t4[0], t4[1], t4[2], t4[3]);
        }
    }
    q2_wave_sync();

    // ---- test contraction, pass x: thread (a, q1, q2) sums over q0
    float P0[NE] = {}, P1[NE] = {}, P2[NE] = {}, A0[NE] = {}, A1[NE] = {}, A2[NE] = {};
    if (valid) {
        const int a = l0;
#pragma unroll
        for (int q0 = 0; q0 < 3; ++q0) {
            const float t = gauss_pt(q0);
            const float Qa = quad_fn(a, t), Da = quad_dfn(a, t), la = a ? t : 1.0f - t;
            const float4 *c4 = reinterpret_cast<const float4 *>(W + 28 * (q0 + 3 * l1 + 9 * l2));
            float cf[28];
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                const float4 t4 = c4[k];
                cf[4 * k] = t4.x;
                cf[4 * k + 1] = t4.y;
                cf[4 * k + 2] = t4.z;
                cf[4 * k + 3] = t4.w;
            }
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const float *c = cf + 7 * e;
                P0[e] += c[0] * Qa + c[1] * Da;
                P1[e] += c[2] * Qa;
                P2[e] += c[3] * Qa;
                if (HAS_A) {
                    A0[e] += c[4];
                    A1[e] += c[5] * la;
                    A2[e] += c[6] * la;
                }
            }
        }
    }
    if (valid) {
        const float dla = l0 ? 1.0f : -1.0f;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            W[Q2_P + (3 * e) * 27 + l] = P0[e];
            W[Q2_P + (3 * e + 1) * 27 + l] = P1[e];
            W[Q2_P + (3 * e + 2) * 27 + l] = P2[e];
            if (HAS_A && l0 < 2) {
                W[Q2_A + (3 * e) * 27 + l] = dla * A0[e];
                W[Q2_A + (3 * e + 1) * 27 + l] = A1[e];
                W[Q2_A + (3 * e + 2) * 27 + l] = A2[e];
            }
        }
    }
    q2_wave_sync();
    // ---- pass y: thread (a, b, q2) sums over q1
    const bool vtx = HAS_A && l0 < 2 && l1 < 2;
    float S0[NE] = {}, S2[NE] = {}, B01[NE] = {}, B2[NE] = {};
    if (valid) {
        const int a = l0, b = l1;
        const float dlb = b ? 1.0f : -1.0f;
#pragma unroll
        for (int q1 = 0; q1 < 3; ++q1) {
            const float t = gauss_pt(q1);
            const float Qb = quad_fn(b, t), Db = quad_dfn(b, t), lb = b ? t : 1.0f - t;
            const int idx = a + 3 * q1 + 9 * l2;
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                S0[e] += W[Q2_P + (3 * e) * 27 + idx] * Qb + W[Q2_P + (3 * e + 1) * 27 + idx] * Db;
                S2[e] += W[Q2_P + (3 * e + 2) * 27 + idx] * Qb;
                if (vtx) {
                    B01[e] += W[Q2_A + (3 * e) * 27 + idx] * lb + W[Q2_A + (3 * e + 1) * 27 + idx] * dlb;
                    B2[e] += W[Q2_A + (3 * e + 2) * 27 + idx] * lb;
                }
            }
        }
    }
    if (valid) {
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            W[(2 * e) * 27 + l] = S0[e];
            W[(2 * e + 1) * 27 + l] = S2[e];
            if (vtx) {
                W[216 + (2 * e) * 27 + l] = B01[e];
                W[216 + (2 * e + 1) * 27 + l] = B2[e];
            }
        }
    }
    q2_wave_sync();
    // ---- pass z: thread (a, b, c) = its test node
    const bool vert = HAS_A && !(l0 & 1) && !(l1 & 1) && !(l2 & 1);
    const int vidx = (l0 >> 1) + 3 * (l1 >> 1);
    const float dlc = (l2 >> 1) ? 1.0f : -1.0f;
    float acc[4] = {};
    if (valid) {
#pragma unroll
        for (int q2 = 0; q2 < 3; ++q2) {
            const float t = gauss_pt(q2);
            const float Qc = quad_fn(l2, t), Dc = quad_dfn(l2, t), lc = (l2 >> 1) ? t : 1.0f - t;
            const int idx = l0 + 3 * l1 + 9 * q2;
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                acc[e] += W[(2 * e) * 27 + idx] * Qc + W[(2 * e + 1) * 27 + idx] * Dc;
                if (vert)
                    acc[e] += W[216 + (2 * e) * 27 + vidx + 9 * q2] * lc + W[216 + (2 * e + 1) * 27 + vidx + 9 * q2] * dlc;
            }
        }
    }
    // BOTH: a second test contraction for the Rhs's 3 equations (factors of
    // phi and of its reference gradient only), through the same arena: the
    // coefficients at 0..323, the x-pass sums at 324..566, the y-pass sums at
    // 567..728
    float accR[3] = {};
    if constexpr (MODE == Q2_BOTH) {
        q2_wave_sync(); // the first contraction's reads are done
        if (valid) {
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int k = 0; k < 4; ++k) W[(4 * q + k) * 27 + l] = coR[q][k];
        }
        q2_wave_sync();
        if (valid) {
            float R0[3] = {}, R1[3] = {}, R2[3] = {};
#pragma unroll
            for (int q0 = 0; q0 < 3; ++q0) {
                const float t = gauss_pt(q0);
                const float Qa = quad_fn(l0, t), Da = quad_dfn(l0, t);
                const int idx = q0 + 3 * l1 + 9 * l2;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    R0[q] += W[(4 * q) * 27 + idx] * Qa + W[(4 * q + 1) * 27 + idx] * Da;
                    R1[q] += W[(4 * q + 2) * 27 + idx] * Qa;
                    R2[q] += W[(4 * q + 3) * 27 + idx] * Qa;
                }
            }
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                W[324 + (3 * q) * 27 + l] = R0[q];
                W[324 + (3 * q + 1) * 27 + l] = R1[q];
                W[324 + (3 * q + 2) * 27 + l] = R2[q];
            }
        }
        q2_wave_sync();
        if (valid) {
            float T0[3] = {}, T2[3] = {};
#pragma unroll
            for (int q1 = 0; q1 < 3; ++q1) {
                const float t = gauss_pt(q1);
                const float Qb = quad_fn(l1, t), Db = quad_dfn(l1, t);
                const int idx = l0 + 3 * q1 + 9 * l2;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    T0[q] += W[324 + (3 * q) * 27 + idx] * Qb + W[324 + (3 * q + 1) * 27 + idx] * Db;
                    T2[q] += W[324 + (3 * q + 2) * 27 + idx] * Qb;
                }
            }
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                W[567 + (2 * q) * 27 + l] = T0[q];
                W[567 + (2 * q + 1) * 27 + l] = T2[q];
            }
        }
        q2_wave_sync();
        if (valid) {
#pragma unroll
            for (int q2 = 0; q2 < 3; ++q2) {
                const float t = gauss_pt(q2);
                const float Qc = quad_fn(l2, t), Dc = quad_dfn(l2, t);
                const int idx = l0 + 3 * l1 + 9 * q2;
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    accR[q] += W[567 + (2 * q) * 27 + idx] * Qc + W[567 + (2 * q + 1) * 27 + idx] * Dc;
            }
        }
    }
    // the workgroup's 8 element vectors as one block [27 e + node][slot]
    if (valid) {
        constexpr int GROUPW = MODE == Q2_BOTH ? Q2_GROUP_BOTH : Q2_GROUP;
        float *dst = E + (int64_t)blockIdx.x * GROUPW + (int64_t)l * Q2_EPB + s;
#pragma unroll
        for (int e = 0; e < NE; ++e) dst[27 * Q2_EPB * e] = acc[e];
        if constexpr (MODE == Q2_BOTH) {
#pragma unroll
            for (int q = 0; q < 3; ++q) dst[27 * Q2_EPB * (4 + q)] = accR[q];
        }
    }
}

// Elements holding node i on an axis with n elements (nodes 0..2n), in
// ascending order, with the node's local index in each: an odd i lies in
// element (i - 1) / 2 only (local 1); an even i is the last node of element
// i/2 - 1 (local 2) and the first of element i/2 (local 0) where they exist.
__device__ __forceinline__ int q2_owners(int i, int n, int el[2], int loc[2]) {
    if (i & 1) {
        el[0] = (i - 1) >> 1;
        loc[0] = 1;
        el[1] = el[0];
        loc[1] = 1;
        return 1;
    }
    int c = 0;
    el[0] = el[1] = i >> 1;
    loc[0] = loc[1] = 0;
    if (i >= 2) {
        el[c] = (i >> 1) - 1;
        loc[c++] = 2;
    }
    if ((i >> 1) < n) {
        el[c] = i >> 1;
        loc[c++] = 0;
    }
    return c;
}

// Per-node sum of the element vectors in a fixed order (elements ascending
// in z, then y, then x): APPLY out = b - sum with Dirichlet velocity rows 0;
// RHS out = sum for the momentum rows (pressure and Dirichlet velocity rows
// 0).  Threads run over consecutive x nodes.
template <int MODE>
__global__ void __launch_bounds__(256) k_q2_sum_nodes(Mesh m, const float *__restrict__ E, const float *b, float *out,
                                                      float *bnext) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m.n_fine) return;
    const int64_t jk = t / m.nf[0];
    const int i = (int)(t - jk * m.nf[0]), j = (int)(jk % m.nf[1]), k = (int)(jk / m.nf[1]);
    int ex[2], ey[2], ez[2], lx[2], ly[2], lz[2];
    const int cx = q2_owners(i, m.n[0], ex, lx), cy = q2_owners(j, m.n[1], ey, ly), cz = q2_owners(k, m.n[2], ez, lz);
    constexpr int NF = MODE == Q2_BOTH ? 7 : 4;
    constexpr int GROUPW = MODE == Q2_BOTH ? Q2_GROUP_BOTH : Q2_GROUP;
    float sum[NF] = {};
#pragma unroll
    for (int uz = 0; uz < 2; ++uz) {
        if (uz >= cz) break;
#pragma unroll
        for (int uy = 0; uy < 2; ++uy) {
            if (uy >= cy) break;
#pragma unroll
            for (int ux = 0; ux < 2; ++ux) {
                if (ux >= cx) break;
                const int64_t M = ex[ux] + (int64_t)m.n[0] * (ey[uy] + (int64_t)m.n[1] * ez[uz]);
                const int64_t grp = M / Q2_EPB;
                const float *e = E + grp * GROUPW + (lx[ux] + 3 * ly[uy] + 9 * lz[uz]) * Q2_EPB + (M - grp * Q2_EPB);
#pragma unroll
                for (int f = 0; f < NF; ++f)
                    if (MODE != Q2_RHS || f < 3) sum[f] += e[27 * Q2_EPB * f];
            }
        }
    }
    const bool dir = on_dirichlet(m, i, j, k);
    // b is read before bnext (which may be b itself) is written
    float r[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        if (MODE != Q2_RHS)
            r[f] = (f < 3 && dir) ? 0.0f : b[f * m.n_fine + t] - sum[f];
        else
            r[f] = (f == 3 || dir) ? 0.0f : sum[f];
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) out[f * m.n_fine + t] = r[f];
    if constexpr (MODE == Q2_BOTH) {
#pragma unroll
        for (int f = 0; f < 4; ++f) bnext[f * m.n_fine + t] = (f == 3 || dir) ? 0.0f : sum[4 + f];
    }
}

// 1-D Q2 prolongation weights from the coarse nodes of level L (n / 2
// elements, nodes 0..n) to the fine nodes of level L + 1 (0..2n): fine node
// i lies in coarse element e = min(i / 4, n/2 - 1) at t = (i - 4e) / 4 and
// takes the element's quadratic interpolant there.
__device__ __forceinline__ void q2_pw(int i, int n, int idx[3], double w[3]) {
    int e = i >> 2;
    if (e > n / 2 - 1) e = n / 2 - 1;
    const double t = 0.25 * (i - 4 * e);
    idx[0] = 2 * e;
    idx[1] = 2 * e + 1;
    idx[2] = 2 * e + 2;
    w[0] = 2.0 * (t - 0.5) * (t - 1.0);
    w[1] = 4.0 * t * (1.0 - t);
    w[2] = 2.0 * t * (t - 0.5);
}

// Nonzero entries of column I of the 1-D prolongation (coarse node I on an
// axis with n fine elements), padded to 5 with zero weights: a coarse vertex
// (I even) reaches the fine nodes 2I + {-3, -1, 0, 1, 3} with weights
// {-1/8, 3/8, 1, 3/8, -1/8}, a coarse mid node (I odd) the fine nodes
// 2I + {-1, 0, 1} with {3/4, 1, 3/4} (the quadratic functions at the quarter
// points); the offsets +-2 fall on coarse nodes, where the other functions
// vanish.  Padding and out-of-range entries point at fine node 2I.
__device__ __forceinline__ void q2_rcol(int I, int n, int fi[5], double w[5]) {
    const int c = 2 * I;
    const bool mid = I & 1;
    const int off[5] = {-3, -1, 0, 1, 3};
    const double wv[5] = {-0.125, 0.375, 1.0, 0.375, -0.125};
    const double wm[5] = {0.0, 0.75, 1.0, 0.75, 0.0};
#pragma unroll
    for (int s = 0; s < 5; ++s) {
        const int f = c + off[s];
        const bool ok = f >= 0 && f <= 2 * n;
        fi[s] = ok ? f : c;
        w[s] = ok ? (mid ? wm[s] : wv[s]) : 0.0;
    }
}

// Prolongation, one workgroup per fine lattice row (j, k): the (y, z)
// weights are the same for the whole row, so each coarse x node is first
// combined over its (y, z) stencil (into LDS), then every fine node of the
// row takes its three x terms from there.  Coarse reads are coalesced along
// x and each is made once per row.
__global__ void __launch_bounds__(256) k_q2_prolong_rows(Mesh m, int ncomp, const double *__restrict__ xc,
                                                         float *__restrict__ xf) {
    extern __shared__ double sU[]; // [ncomp][nc0]
    const int64_t row = blockIdx.x;
    const int j = (int)(row % m.nf[1]), k = (int)(row / m.nf[1]);
    int iy[3], iz[3];
    double wy[3], wz[3];
    q2_pw(j, m.n[1], iy, wy);
    q2_pw(k, m.n[2], iz, wz);
    const int nc0 = m.nc[0];
    for (int t = threadIdx.x; t < ncomp * nc0; t += blockDim.x) {
        const int c = t / nc0, I = t - c * nc0;
        const double *src = xc + c * m.n_coarse + I;
        // every stencil entry is a node of the mesh, so all nine are
        // requested at once (zero weights add exact zeros)
        double v[3][3];
#pragma unroll
        for (int z = 0; z < 3; ++z)
#pragma unroll
            for (int y = 0; y < 3; ++y) v[z][y] = src[(int64_t)m.nc[0] * (iy[y] + (int64_t)m.nc[1] * iz[z])];
        double s = 0.0;
#pragma unroll
        for (int z = 0; z < 3; ++z)
#pragma unroll
            for (int y = 0; y < 3; ++y) s += (wz[z] * wy[y]) * v[z][y];
        sU[t] = s;
    }
    __syncthreads();
    const int64_t base = (int64_t)m.nf[0] * (j + (int64_t)m.nf[1] * k);
    for (int i = threadIdx.x; i < m.nf[0]; i += blockDim.x) {
        int ix[3];
        double wx[3];
        q2_pw(i, m.n[0], ix, wx);
        for (int c = 0; c < ncomp; ++c) {
            const double *u = sU + c * nc0;
            xf[c * m.n_fine + base + i] = (float)(wx[0] * u[ix[0]] + wx[1] * u[ix[1]] + wx[2] * u[ix[2]]);
        }
    }
}

// Restriction (the transpose), one workgroup per coarse lattice row (J, K):
// every fine x node is first summed over the row's (y, z) stencil (at most
// 5 x 5 fine values, read coalesced along x, into LDS in FP64), then each
// coarse node of the row takes its at most 5 x terms from there.
__global__ void __launch_bounds__(256) k_q2_restrict_rows(Mesh m, int ncomp, const float *__restrict__ bf,
                                                          double *__restrict__ bc) {
    extern __shared__ double sT[]; // [ncomp][nf0]
    const int64_t row = blockIdx.x;
    const int J = (int)(row % m.nc[1]), K = (int)(row / m.nc[1]);
    int fy[5], fz[5];
    double wy[5], wz[5];
    q2_rcol(J, m.n[1], fy, wy);
    q2_rcol(K, m.n[2], fz, wz);
    const int nf0 = m.nf[0];
    for (int t = threadIdx.x; t < ncomp * nf0; t += blockDim.x) {
        const int c = t / nf0, i = t - c * nf0;
        const float *src = bf + c * m.n_fine + i;
        // padded entries point at a node of the mesh with weight 0, so all 25
        // are requested at once (zero weights add exact zeros)
        float v[5][5];
#pragma unroll
        for (int z = 0; z < 5; ++z)
#pragma unroll
            for (int y = 0; y < 5; ++y) v[z][y] = src[(int64_t)m.nf[0] * (fy[y] + (int64_t)m.nf[1] * fz[z])];
        double s = 0.0;
#pragma unroll
        for (int z = 0; z < 5; ++z) {
            double sy = 0.0;
#pragma unroll
            for (int y = 0; y < 5; ++y) sy += wy[y] * (double)v[z][y];
            s += wz[z] * sy;
        }
        sT[t] = s;
    }
    __syncthreads();
    const int64_t base = (int64_t)m.nc[0] * (J + (int64_t)m.nc[1] * K);
    for (int I = threadIdx.x; I < m.nc[0]; I += blockDim.x) {
        int fx[5];
        double wx[5];
        q2_rcol(I, m.n[0], fx, wx);
        for (int c = 0; c < ncomp; ++c) {
            const double *t = sT + c * nf0;
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < 5; ++q) s += wx[q] * t[fx[q]];
            bc[c * m.n_coarse + base + I] = s;
        }
    }
}

// Geometry inputs of Sec. 4.2 for curved cells, once per mesh: g_a of
// element M = the mean length of its 4 vertex-to-vertex edges along axis a
// (the cell sizes on axis-parallel cells), from the FP64 node positions.
__global__ void k_q2_features(Mesh m, const double *__restrict__ X, float *__restrict__ geom) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * m.n_patches) return;
    const int64_t M = t / 3;
    const int a = (int)(t - 3 * M);
    const int I = (int)(M % m.n[0]), J = (int)((M / m.n[0]) % m.n[1]), K = (int)(M / ((int64_t)m.n[0] * m.n[1]));
    const int64_t nf = m.n_fine;
    double sum = 0.0;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        if ((v >> a) & 1) continue;
        const int w = v | (1 << a);
        const int64_t p0 = (2 * I + 2 * (v & 1)) +
                           (int64_t)m.nf[0] * ((2 * J + 2 * ((v >> 1) & 1)) + (int64_t)m.nf[1] * (2 * K + 2 * ((v >> 2) & 1)));
        const int64_t p1 = (2 * I + 2 * (w & 1)) +
                           (int64_t)m.nf[0] * ((2 * J + 2 * ((w >> 1) & 1)) + (int64_t)m.nf[1] * (2 * K + 2 * ((w >> 2) & 1)));
        double d2 = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double e = X[d * nf + p1] - X[d * nf + p0];
            d2 += e * e;
        }
        sum += sqrt(d2);
    }
    geom[t] = (float)(0.25 * sum);
}

// The 24 geometry features of Sec. 4.2 of element M, from the positions of
// its 8 vertices P_j (j = a + 2b + 4c at node (2I + 2a, 2J + 2b, 2K + 2c)):
// the 12 edge lengths (edges along x, then y, then z, each group ordered by
// the two other corner bits, lower axis first), the 4 diagonals |P_{7-j} -
// P_j| (j = 0..3), and at each vertex the mean of the three dihedral angles
// of the faces meeting there (along edge e_a the angle between the
// components of the other two edges normal to e_a).  FP64, once per mesh.
__global__ void k_q2_features24(Mesh m, const double *__restrict__ X, float *__restrict__ geo) {
    const int64_t M = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (M >= m.n_patches) return;
    const int I = (int)(M % m.n[0]), J = (int)((M / m.n[0]) % m.n[1]), K = (int)(M / ((int64_t)m.n[0] * m.n[1]));
    const int64_t nf = m.n_fine;
    double P[8][3];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int64_t n = (2 * I + 2 * (j & 1)) +
                          (int64_t)m.nf[0] * ((2 * J + 2 * ((j >> 1) & 1)) + (int64_t)m.nf[1] * (2 * K + 2 * (j >> 2)));
#pragma unroll
        for (int d = 0; d < 3; ++d) P[j][d] = X[d * nf + n];
    }
    auto dist = [&](int i, int j) {
        double s = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) s += (P[j][d] - P[i][d]) * (P[j][d] - P[i][d]);
        return sqrt(s);
    };
    float *out = geo + 24 * M;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int o0 = ax == 0 ? 1 : 0, o1 = ax == 2 ? 1 : 2;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int j0 = ((t & 1) << o0) | ((t >> 1) << o1);
            out[4 * ax + t] = (float)dist(j0, j0 + (1 << ax));
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) out[12 + j] = (float)dist(j, 7 - j);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        double e[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int d = 0; d < 3; ++d) e[a][d] = P[j ^ (1 << a)][d] - P[j][d];
        double sum = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
            const double na = sqrt(e[a][0] * e[a][0] + e[a][1] * e[a][1] + e[a][2] * e[a][2]);
            double u[3], pb[3], pc[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) u[d] = e[a][d] / na;
            const double db = e[b][0] * u[0] + e[b][1] * u[1] + e[b][2] * u[2];
            const double dc = e[c][0] * u[0] + e[c][1] * u[1] + e[c][2] * u[2];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                pb[d] = e[b][d] - db * u[d];
                pc[d] = e[c][d] - dc * u[d];
            }
            const double nb = sqrt(pb[0] * pb[0] + pb[1] * pb[1] + pb[2] * pb[2]);
            const double nc = sqrt(pc[0] * pc[0] + pc[1] * pc[1] + pc[2] * pc[2]);
            double cv = (pb[0] * pc[0] + pb[1] * pc[1] + pb[2] * pc[2]) / (nb * nc);
            cv = cv > 1.0 ? 1.0 : (cv < -1.0 ? -1.0 : cv);
            sum += acos(cv);
        }
        out[16 + j] = (float)(sum / 3.0);
    }
}

static int q2_mesh(const char *who, const dnnmg_box *box, Mesh *m, bool even) {
    int rc = make_mesh(box, m);
    if (rc) return rc;
    if (box->periodic_mask) return fail(DNNMG_ERR_SHAPE, "%s: the Q2 mesh has no periodic axes", who);
    if (even && ((box->n[0] | box->n[1] | box->n[2]) & 1))
        return fail(DNNMG_ERR_SHAPE, "%s: the coarse Q2 mesh needs even element counts (%d, %d, %d)", who,
                    box->n[0], box->n[1], box->n[2]);
    return DNNMG_OK;
}

static int q2_params(const char *who, const dnnmg_ns *ns, Q2Params *P) {
    if (!ns) return fail(DNNMG_ERR_ARG, "%s: ns is NULL", who);
    if (!(ns->nu >= 0.0) || !(ns->dt > 0.0) || !(ns->alpha0 >= 0.0) || !(ns->delta0 >= 0.0))
        return fail(DNNMG_ERR_ARG, "%s: need nu >= 0, dt > 0, alpha0 >= 0, delta0 >= 0", who);
    P->inv_dt = (float)(1.0 / ns->dt);
    P->half_nu = (float)(0.5 * ns->nu);
    P->nu = (float)ns->nu;
    P->alpha0 = (float)ns->alpha0;
    P->delta0 = (float)ns->delta0;
    return DNNMG_OK;
}

static size_t q2_ws_bytes(const Mesh &m) {
    const int64_t groups = (m.n_patches + Q2_EPB - 1) / Q2_EPB;
    return (size_t)((groups * Q2_GROUP_BOTH * 4 + 255) / 256 * 256);
}

template <int MODE>
static int q2_assemble(const Mesh &m, const Q2Params &P, const double *X, const float *x, const float *fmid,
                       const float *b, float *out, void *ws, size_t ws_bytes, void *stream, float *bnext = nullptr) {
    if (!ws || !aligned16(ws) || ws_bytes < q2_ws_bytes(m))
        return fail(DNNMG_ERR_ARG, "Q2 assembly: workspace of %zu bytes (16-byte aligned) needed, %zu given",
                    q2_ws_bytes(m), ws_bytes);
    float *E = static_cast<float *>(ws);
    k_q2_element<MODE><<<blocks_for(m.n_patches, Q2_EPB), Q2_NT, 0, STREAM>>>(m, P, X, x, fmid, E);
    k_q2_sum_nodes<MODE><<<blocks_for(m.n_fine, 256), 256, 0, STREAM>>>(m, E, b, out, bnext);
    return hip_check(hipGetLastError(), "Q2 element launch");
}

} // namespace dnnmg

using namespace dnnmg;

extern "C" size_t dnnmg_q2_workspace(const dnnmg_box *box) {
    Mesh m;
    if (q2_mesh("dnnmg_q2_workspace", box, &m, false)) return 0;
    return q2_ws_bytes(m);
}

extern "C" int dnnmg_q2_residual_b(const dnnmg_box *box, const dnnmg_ns *ns, const double *coords, const float *x,
                                   const float *b, float *r, void *ws, size_t ws_bytes, void *stream) {
    Mesh m;
    Q2Params P;
    int rc = q2_mesh("dnnmg_q2_residual_b", box, &m, false);
    if (rc) return rc;
    if ((rc = q2_params("dnnmg_q2_residual_b", ns, &P))) return rc;
    if (!coords || !x || !b || !r) return fail(DNNMG_ERR_ARG, "dnnmg_q2_residual_b: NULL pointer");
    if (r == b || r == x) return fail(DNNMG_ERR_ARG, "dnnmg_q2_residual_b: r must not alias x or b");
    return q2_assemble<Q2_APPLY>(m, P, coords, x, nullptr, b, r, ws, ws_bytes, stream);
}

extern "C" int dnnmg_q2_residual_rhs(const dnnmg_box *box, const dnnmg_ns *ns, const double *coords, const float *x,
                                     const float *b, float *r, float *bnext, void *ws, size_t ws_bytes, void *stream) {
    Mesh m;
    Q2Params P;
    int rc = q2_mesh("dnnmg_q2_residual_rhs", box, &m, false);
    if (rc) return rc;
    if ((rc = q2_params("dnnmg_q2_residual_rhs", ns, &P))) return rc;
    if (!coords || !x || !b || !r || !bnext) return fail(DNNMG_ERR_ARG, "dnnmg_q2_residual_rhs: NULL pointer");
    if (r == b || r == x || r == bnext || bnext == x)
        return fail(DNNMG_ERR_ARG, "dnnmg_q2_residual_rhs: r and bnext must not alias x, and r not b or bnext");
    return q2_assemble<Q2_BOTH>(m, P, coords, x, nullptr, b, r, ws, ws_bytes, stream, bnext);
}

extern "C" int dnnmg_q2_rhs(const dnnmg_box *box, const dnnmg_ns *ns, const double *coords, const float *v,
                            const float *fmid, float *b, void *ws, size_t ws_bytes, void *stream) {
    Mesh m;
    Q2Params P;
    int rc = q2_mesh("dnnmg_q2_rhs", box, &m, false);
    if (rc) return rc;
    if ((rc = q2_params("dnnmg_q2_rhs", ns, &P))) return rc;
    if (!coords || !v || !b) return fail(DNNMG_ERR_ARG, "dnnmg_q2_rhs: NULL pointer");
    if (b == v || (fmid && b == fmid)) return fail(DNNMG_ERR_ARG, "dnnmg_q2_rhs: b must not alias v or fmid");
    return q2_assemble<Q2_RHS>(m, P, coords, v, fmid, nullptr, b, ws, ws_bytes, stream);
}

extern "C" int dnnmg_q2_prolong(const dnnmg_box *box, int ncomp, const double *xc, float *xf, void *stream) {
    Mesh m;
    int rc = q2_mesh("dnnmg_q2_prolong", box, &m, true);
    if (rc) return rc;
    if (ncomp < 1 || ncomp > 4) return fail(DNNMG_ERR_ARG, "dnnmg_q2_prolong: ncomp %d not in 1..4", ncomp);
    if (!xc || !xf) return fail(DNNMG_ERR_ARG, "dnnmg_q2_prolong: NULL pointer");
    if ((size_t)ncomp * m.nc[0] * sizeof(double) > 64 * 1024)
        return fail(DNNMG_ERR_SHAPE, "dnnmg_q2_prolong: %d nodes per x row exceed the row buffer", m.nc[0]);
    k_q2_prolong_rows<<<(unsigned)((int64_t)m.nf[1] * m.nf[2]), 256, (size_t)ncomp * m.nc[0] * sizeof(double),
                        STREAM>>>(m, ncomp, xc, xf);
    return hip_check(hipGetLastError(), "dnnmg_q2_prolong launch");
}

extern "C" int dnnmg_q2_restrict(const dnnmg_box *box, int ncomp, const float *bf, double *bc, void *stream) {
    Mesh m;
    int rc = q2_mesh("dnnmg_q2_restrict", box, &m, true);
    if (rc) return rc;
    if (ncomp < 1 || ncomp > 4) return fail(DNNMG_ERR_ARG, "dnnmg_q2_restrict: ncomp %d not in 1..4", ncomp);
    if (!bf || !bc) return fail(DNNMG_ERR_ARG, "dnnmg_q2_restrict: NULL pointer");
    if ((size_t)ncomp * m.nf[0] * sizeof(double) > 64 * 1024)
        return fail(DNNMG_ERR_SHAPE, "dnnmg_q2_restrict: %d nodes per x row exceed the row buffer", m.nf[0]);
    k_q2_restrict_rows<<<(unsigned)((int64_t)m.nc[1] * m.nc[2]), 256, (size_t)ncomp * m.nf[0] * sizeof(double),
                         STREAM>>>(m, ncomp, bf, bc);
    return hip_check(hipGetLastError(), "dnnmg_q2_restrict launch");
}

extern "C" int dnnmg_q2_patch_features24(const dnnmg_box *box, const double *coords, float *geo24, void *stream) {
    Mesh m;
    int rc = q2_mesh("dnnmg_q2_patch_features24", box, &m, false);
    if (rc) return rc;
    if (!coords || !geo24) return fail(DNNMG_ERR_ARG, "dnnmg_q2_patch_features24: NULL pointer");
    k_q2_features24<<<blocks_for(m.n_patches, 128), 128, 0, STREAM>>>(m, coords, geo24);
    return hip_check(hipGetLastError(), "dnnmg_q2_patch_features24 launch");
}

extern "C" int dnnmg_q2_patch_features(const dnnmg_box *box, const double *coords, float *geom, void *stream) {
    Mesh m;
    int rc = q2_mesh("dnnmg_q2_patch_features", box, &m, false);
    if (rc) return rc;
    if (!coords || !geom) return fail(DNNMG_ERR_ARG, "dnnmg_q2_patch_features: NULL pointer");
    k_q2_features<<<blocks_for(3 * m.n_patches, 256), 256, 0, STREAM>>>(m, coords, geom);
    return hip_check(hipGetLastError(), "dnnmg_q2_patch_features launch");
}
