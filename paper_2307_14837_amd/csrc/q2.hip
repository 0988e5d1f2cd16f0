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
// Element integrals (3 x 3 x 3 Gauss points) run in two phases per element
// inside one workgroup of 9 elements x 27 threads:
//   1. one thread per quadrature point evaluates the Jacobian, the fields,
//      their gradients and the Q1 interpolants there and reduces every term
//      of the weak form to 7 coefficients per equation: the factor of the
//      test function, of its reference gradient and of the reference
//      gradient of its Q1 interpolant (nonzero for vertex nodes only);
//   2. one thread per test node sums those coefficients against its shape
//      functions over the 27 points.
// Element vectors are added into the global vector colour by colour: the 8
// classes of elements with equal index parities share no node, so each of
// the 8 launches updates its nodes without atomics and the sum order is
// fixed (results are reproducible bit for bit).
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

constexpr int Q2_EPB = 9;    // elements per workgroup
constexpr int Q2_NT = 256;   // threads per workgroup (243 active)
constexpr int Q2_NSTR = 8;   // per node: 3 offsets, pad, 4 fields
constexpr int Q2_CSTR = 28;  // per point: 4 equations x 7 coefficients

enum { Q2_APPLY = 0, Q2_RHS = 1 };

// Element (I, J, K) of colour `col` from its index within the colour.
__device__ __forceinline__ bool colour_element(const Mesh &m, int col, int64_t e, int &I, int &J, int &K) {
    const int cx = col & 1, cy = (col >> 1) & 1, cz = (col >> 2) & 1;
    const int mx = (m.n[0] - cx + 1) >> 1, my = (m.n[1] - cy + 1) >> 1, mz = (m.n[2] - cz + 1) >> 1;
    if (e >= (int64_t)mx * my * mz) return false;
    const int ex = (int)(e % mx);
    const int64_t r = e / mx;
    const int ey = (int)(r % my), ez = (int)(r / my);
    I = 2 * ex + cx;
    J = 2 * ey + cy;
    K = 2 * ez + cz;
    return true;
}

// MODE Q2_APPLY: out -= A(x) (x = u, v, w, p); MODE Q2_RHS: out += Rhs(x =
// velocity, fmid).  Dirichlet velocity rows are left untouched.
template <int MODE>
__global__ void __launch_bounds__(Q2_NT, 4) k_q2_element(Mesh m, Q2Params P, int col, const double *__restrict__ X,
                                                      const float *__restrict__ x,
                                                      const float *__restrict__ fmid, float *__restrict__ out) {
    __shared__ __align__(16) float sN[Q2_EPB][27][Q2_NSTR];
    __shared__ float sF[Q2_EPB][27][4]; // fmid (RHS mode)
    __shared__ __align__(16) float sC[Q2_EPB][27][Q2_CSTR];
    __shared__ float sV[Q2_EPB][27];    // |v|^2 per node
    __shared__ float sH[Q2_EPB][8];     // largest squared vertex distance per vertex

    const int tid = threadIdx.x;
    const int s = tid / 27, l = tid - 27 * (tid / 27);
    const bool active_t = tid < 27 * Q2_EPB;
    int I = 0, J = 0, K = 0;
    const bool valid =
        active_t && colour_element(m, col, (int64_t)blockIdx.x * Q2_EPB + s, I, J, K);
    const int64_t nf = m.n_fine;
    const int la = l % 3, lb = (l / 3) % 3, lc = l / 9;
    const int gi = 2 * I + la, gj = 2 * J + lb, gk = 2 * K + lc;
    const int64_t g = gi + (int64_t)m.nf[0] * (gj + (int64_t)m.nf[1] * gk);

    // ---- stage the element's node positions (relative to its first vertex) and fields
    if (valid) {
        const int64_t g0 = 2 * I + (int64_t)m.nf[0] * (2 * J + (int64_t)m.nf[1] * (2 * K));
        float v2 = 0.0f;
#pragma unroll
        for (int d = 0; d < 3; ++d) sN[s][l][d] = (float)(X[d * nf + g] - X[d * nf + g0]);
        sN[s][l][3] = 0.0f;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            float val = (MODE == Q2_RHS && f == 3) ? 0.0f : x[f * nf + g];
            sN[s][l][4 + f] = val;
            if (f < 3) v2 += val * val;
        }
        sV[s][l] = v2;
        if (MODE == Q2_RHS) {
#pragma unroll
            for (int f = 0; f < 3; ++f) sF[s][l][f] = fmid ? fmid[f * nf + g] : 0.0f;
        }
    }
    __syncthreads();

    float alphaT = 0.0f, deltaT = 0.0f;
    if (MODE == Q2_APPLY) {
        // h_T = the largest vertex distance; |v|_inf = the largest |v| over the 27 nodes
        if (valid && l < 8) {
            const int vi = 2 * (l & 1) + 6 * ((l >> 1) & 1) + 18 * ((l >> 2) & 1);
            float best = 0.0f;
            for (int w = l + 1; w < 8; ++w) {
                const int wi = 2 * (w & 1) + 6 * ((w >> 1) & 1) + 18 * ((w >> 2) & 1);
                float d2 = 0.0f;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    float e = sN[s][wi][d] - sN[s][vi][d];
                    d2 += e * e;
                }
                best = fmaxf(best, d2);
            }
            sH[s][l] = best;
        }
        __syncthreads();
        if (valid) {
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
    }

    // ---- phase 1: thread l is quadrature point (q0, q1, q2) = (la, lb, lc)
    if (valid) {
        float Qx[3], Dx[3], Qy[3], Dy[3];
        const float t0 = gauss_pt(la), t1 = gauss_pt(lb), t2 = gauss_pt(lc);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            Qx[a] = quad_fn(a, t0);
            Dx[a] = quad_dfn(a, t0);
            Qy[a] = quad_fn(a, t1);
            Dy[a] = quad_dfn(a, t1);
        }
        float Jm[3][3] = {}, v[3] = {}, gv[3][3] = {}, p = 0.0f, gp[3] = {}, f[3] = {};
#pragma unroll 1
        for (int c = 0; c < 3; ++c) {
            const float qz = quad_fn(c, t2), dqz = quad_dfn(c, t2);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const float yz = Qy[b] * qz, dy = Dy[b] * qz, dz = Qy[b] * dqz;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int n = a + 3 * b + 9 * c;
                    const float N = Qx[a] * yz;
                    const float dN[3] = {Dx[a] * yz, Qx[a] * dy, Qx[a] * dz};
                    const float4 pos = *reinterpret_cast<const float4 *>(&sN[s][n][0]);
                    const float4 fld = *reinterpret_cast<const float4 *>(&sN[s][n][4]);
                    const float pv[3] = {pos.x, pos.y, pos.z};
                    const float fv[4] = {fld.x, fld.y, fld.z, fld.w};
#pragma unroll
                    for (int e = 0; e < 3; ++e) {
#pragma unroll
                        for (int d = 0; d < 3; ++d) Jm[d][e] += pv[d] * dN[e];
#pragma unroll
                        for (int q = 0; q < 3; ++q) gv[q][e] += fv[q] * dN[e];
                        if (MODE == Q2_APPLY) gp[e] += fv[3] * dN[e];
                    }
#pragma unroll
                    for (int q = 0; q < 3; ++q) v[q] += fv[q] * N;
                    if (MODE == Q2_APPLY) p += fv[3] * N;
                    if (MODE == Q2_RHS) {
#pragma unroll
                        for (int q = 0; q < 3; ++q) f[q] += sF[s][n][q] * N;
                    }
                }
            }
        }
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
        const float w = gauss_wt(la) * gauss_wt(lb) * gauss_wt(lc) * det;

        // physical gradients: grad f = Ji^T (reference gradient)
        float G[3][3];
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int d = 0; d < 3; ++d) G[q][d] = gv[q][0] * Ji[0][d] + gv[q][1] * Ji[1][d] + gv[q][2] * Ji[2][d];
        float conv[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) conv[q] = v[0] * G[q][0] + v[1] * G[q][1] + v[2] * G[q][2];

        float co[4][7];
        if (MODE == Q2_APPLY) {
            // Q1 interpolants from the 8 vertices (local nodes 2va + 6vb + 18vc)
            const float Lx[2] = {1.0f - t0, t0}, Ly[2] = {1.0f - t1, t1}, Lz[2] = {1.0f - t2, t2};
            float pv[3] = {}, gpv[3][3] = {}, gpp[3] = {};
#pragma unroll
            for (int vtx = 0; vtx < 8; ++vtx) {
                const int va = vtx & 1, vb = (vtx >> 1) & 1, vc = (vtx >> 2) & 1;
                const float sx = va ? 1.0f : -1.0f, sy = vb ? 1.0f : -1.0f, sz = vc ? 1.0f : -1.0f;
                const float L = Lx[va] * Ly[vb] * Lz[vc];
                const float dL[3] = {sx * Ly[vb] * Lz[vc], Lx[va] * sy * Lz[vc], Lx[va] * Ly[vb] * sz};
                const float4 fld = *reinterpret_cast<const float4 *>(&sN[s][2 * va + 6 * vb + 18 * vc][4]);
                const float fv[4] = {fld.x, fld.y, fld.z, fld.w};
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    pv[q] += fv[q] * L;
#pragma unroll
                    for (int e = 0; e < 3; ++e) gpv[q][e] += fv[q] * dL[e];
                }
#pragma unroll
                for (int e = 0; e < 3; ++e) gpp[e] += fv[3] * dL[e];
            }
            float gpi[3][3], gpp_phys[3], gp_phys[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    gpi[q][d] = gpv[q][0] * Ji[0][d] + gpv[q][1] * Ji[1][d] + gpv[q][2] * Ji[2][d];
                gpp_phys[d] = gpp[0] * Ji[0][d] + gpp[1] * Ji[1][d] + gpp[2] * Ji[2][d];
                gp_phys[d] = gp[0] * Ji[0][d] + gp[1] * Ji[1][d] + gp[2] * Ji[2][d];
            }
            // momentum rows: factor of phi, of grad phi and of grad pi phi (physical)
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
                co[q][0] = w * (P.inv_dt * v[q] - 0.5f * conv[q] + f[q]);
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    co[q][1 + e] = -w * P.half_nu * (Ji[e][0] * G[q][0] + Ji[e][1] * G[q][1] + Ji[e][2] * G[q][2]);
                    co[q][4 + e] = 0.0f;
                }
            }
#pragma unroll
            for (int k = 0; k < 7; ++k) co[3][k] = 0.0f;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int k = 0; k < 7; ++k) sC[s][l][7 * e + k] = co[e][k];
    }
    __syncthreads();

    // ---- phase 2: thread l is test node (a, b, c) = (la, lb, lc)
    if (!valid) return;
    float Qa[3], Da[3], La[3];
    const bool vert = !(la & 1) && !(lb & 1) && !(lc & 1);
    const float vm = vert ? 1.0f : 0.0f;
    const float sa = la ? 1.0f : -1.0f, sb = lb ? 1.0f : -1.0f, sc = lc ? 1.0f : -1.0f;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const float t = gauss_pt(q);
        Qa[q] = quad_fn(la, t);
        Da[q] = quad_dfn(la, t);
        La[q] = la ? t : 1.0f - t; // the vertex's linear function (used when vert)
    }
    float acc[4] = {};
#pragma unroll 1
    for (int q12 = 0; q12 < 9; ++q12) {
        const int q1 = q12 % 3, q2 = q12 / 3;
        const float t1 = gauss_pt(q1), t2 = gauss_pt(q2);
        const float qb1 = quad_fn(lb, t1), db1 = quad_dfn(lb, t1), qc2 = quad_fn(lc, t2), dc2 = quad_dfn(lc, t2);
        const float lb1 = lb ? t1 : 1.0f - t1, lc2 = lc ? t2 : 1.0f - t2;
        {
            const float yz = qb1 * qc2, dy = db1 * qc2, dz = qb1 * dc2;
            const float lyz = vm * lb1 * lc2, ly = vm * sb * lc2, lz = vm * lb1 * sc;
#pragma unroll
            for (int q0 = 0; q0 < 3; ++q0) {
                const int qi = q0 + 3 * q1 + 9 * q2;
                const float N = Qa[q0] * yz;
                const float dN0 = Da[q0] * yz, dN1 = Qa[q0] * dy, dN2 = Qa[q0] * dz;
                const float dL0 = sa * lyz, dL1 = La[q0] * ly, dL2 = La[q0] * lz;
                const float4 *cq = reinterpret_cast<const float4 *>(&sC[s][qi][0]);
                float cf[28];
#pragma unroll
                for (int k = 0; k < 7; ++k) {
                    const float4 t4 = cq[k];
                    cf[4 * k] = t4.x;
                    cf[4 * k + 1] = t4.y;
                    cf[4 * k + 2] = t4.z;
                    cf[4 * k + 3] = t4.w;
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (MODE == Q2_RHS && e == 3) continue;
                    const float *c = cf + 7 * e;
                    float a = c[0] * N + c[1] * dN0 + c[2] * dN1 + c[3] * dN2;
                    if (MODE == Q2_APPLY) a += c[4] * dL0 + c[5] * dL1 + c[6] * dL2;
                    acc[e] += a;
                }
            }
        }
    }
    const bool dir = on_dirichlet(m, gi, gj, gk);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        if (e < 3 && dir) continue;
        if (MODE == Q2_RHS && e == 3) continue;
        float *o = out + e * nf + g;
        *o = MODE == Q2_APPLY ? *o - acc[e] : *o + acc[e];
    }
}

// r = b with Dirichlet velocity rows 0 (APPLY), or out = 0 (RHS).
__global__ void k_q2_init(Mesh m, const float *__restrict__ b, float *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * m.n_fine) return;
    const int64_t n = t % m.n_fine;
    const int f = (int)(t / m.n_fine);
    float val = b ? b[t] : 0.0f;
    if (f < 3 && b) {
        const int64_t jk = n / m.nf[0];
        const int i = (int)(n - jk * m.nf[0]), j = (int)(jk % m.nf[1]), k = (int)(jk / m.nf[1]);
        if (on_dirichlet(m, i, j, k)) val = 0.0f;
    }
    out[t] = val;
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
        double s = 0.0;
#pragma unroll
        for (int z = 0; z < 3; ++z)
#pragma unroll
            for (int y = 0; y < 3; ++y) {
                const double w = wz[z] * wy[y];
                if (w != 0.0) s += w * src[(int64_t)m.nc[0] * (iy[y] + (int64_t)m.nc[1] * iz[z])];
            }
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
        double s = 0.0;
#pragma unroll
        for (int z = 0; z < 5; ++z) {
            if (wz[z] == 0.0) continue;
            double sy = 0.0;
#pragma unroll
            for (int y = 0; y < 5; ++y)
                if (wy[y] != 0.0) sy += wy[y] * (double)src[(int64_t)m.nf[0] * (fy[y] + (int64_t)m.nf[1] * fz[z])];
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

static int64_t colour_count(const Mesh &m, int col) {
    int64_t c = 1;
    for (int a = 0; a < 3; ++a) c *= (m.n[a] - ((col >> a) & 1) + 1) >> 1;
    return c;
}

template <int MODE>
static int q2_assemble(const Mesh &m, const Q2Params &P, const double *X, const float *x, const float *fmid,
                       const float *b, float *out, void *stream) {
    k_q2_init<<<blocks_for(4 * m.n_fine, 256), 256, 0, STREAM>>>(m, MODE == Q2_APPLY ? b : nullptr, out);
    for (int col = 0; col < 8; ++col) {
        const int64_t ne = colour_count(m, col);
        if (ne == 0) continue;
        k_q2_element<MODE><<<blocks_for(ne, Q2_EPB), Q2_NT, 0, STREAM>>>(m, P, col, X, x, fmid, out);
    }
    return hip_check(hipGetLastError(), "Q2 element launch");
}

} // namespace dnnmg

using namespace dnnmg;

extern "C" int dnnmg_q2_residual_b(const dnnmg_box *box, const dnnmg_ns *ns, const double *coords, const float *x,
                                   const float *b, float *r, void *stream) {
    Mesh m;
    Q2Params P;
    int rc = q2_mesh("dnnmg_q2_residual_b", box, &m, false);
    if (rc) return rc;
    if ((rc = q2_params("dnnmg_q2_residual_b", ns, &P))) return rc;
    if (!coords || !x || !b || !r) return fail(DNNMG_ERR_ARG, "dnnmg_q2_residual_b: NULL pointer");
    if (r == b || r == x) return fail(DNNMG_ERR_ARG, "dnnmg_q2_residual_b: r must not alias x or b");
    return q2_assemble<Q2_APPLY>(m, P, coords, x, nullptr, b, r, stream);
}

extern "C" int dnnmg_q2_rhs(const dnnmg_box *box, const dnnmg_ns *ns, const double *coords, const float *v,
                            const float *fmid, float *b, void *stream) {
    Mesh m;
    Q2Params P;
    int rc = q2_mesh("dnnmg_q2_rhs", box, &m, false);
    if (rc) return rc;
    if ((rc = q2_params("dnnmg_q2_rhs", ns, &P))) return rc;
    if (!coords || !v || !b) return fail(DNNMG_ERR_ARG, "dnnmg_q2_rhs: NULL pointer");
    if (b == v || (fmid && b == fmid)) return fail(DNNMG_ERR_ARG, "dnnmg_q2_rhs: b must not alias v or fmid");
    return q2_assemble<Q2_RHS>(m, P, coords, v, fmid, nullptr, b, stream);
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

extern "C" int dnnmg_q2_patch_features(const dnnmg_box *box, const double *coords, float *geom, void *stream) {
    Mesh m;
    int rc = q2_mesh("dnnmg_q2_patch_features", box, &m, false);
    if (rc) return rc;
    if (!coords || !geom) return fail(DNNMG_ERR_ARG, "dnnmg_q2_patch_features: NULL pointer");
    k_q2_features<<<blocks_for(3 * m.n_patches, 256), 256, 0, STREAM>>>(m, coords, geom);
    return hip_check(hipGetLastError(), "dnnmg_q2_patch_features launch");
}
