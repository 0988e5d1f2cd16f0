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
// stages the fields of the node block plus a halo into LDS, evaluates every
// fine cell touching an owned node (one extra cell layer on the low side),
// and accumulates the cells' vertex integrals into an LDS node array in 8
// colour phases (cells of one parity class share no vertex), so the sum
// order is fixed and no atomics are used.  Owned nodes are then written
// once.  The LPS test functions pi(phi_i) live on the corners of a patch;
// those contributions are summed per owned patch in LDS and written to a
// workspace, and a second small kernel adds them to the coarse-vertex nodes.
//
// Per cell the quadrature uses sum factorisation: values and gradients at
// the 8 Gauss points from the 8 vertex values, and the transpose to vertex
// integrals, each by three 1-D passes.
#include "common.hpp"

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

// ------------------------------------------------------------ kernel ------
constexpr int MODE_RES = 0;
constexpr int MODE_RHS = 1;

template <int MODE>
struct ResTile {
    static constexpr int TX = 16, TY = 8, TZ = 4;  // owned nodes
    static constexpr int EX = TX + 1, EY = TY + 1, EZ = TZ + 1; // cells
    static constexpr int NCELL = EX * EY * EZ;
    // staged node range: [o-2, o+T] for x, p (patch corners), [o-1, o+T] for vp
    static constexpr int SX = TX + 3, SY = TY + 3, SZ = TZ + 3, SN = SX * SY * SZ;
    static constexpr int VX = TX + 2, VY = TY + 2, VZ = TZ + 2, VN = VX * VY * VZ;
    static constexpr int NPX = TX / 2, NPY = TY / 2, NPZ = TZ / 2, NP = NPX * NPY * NPZ;
    static constexpr int NT = 384;
    static constexpr int ROUNDS = (NCELL + NT - 1) / NT;
    static constexpr int NF_STAGE = MODE == MODE_RES ? 4 : 0; // x, p on the wide range
    static constexpr int NF_V = 3;                            // vp (res) or v (rhs)
    static constexpr int NACC = MODE == MODE_RES ? 4 : 3;
};

struct ResParams {
    float inv_dt, half_nu, alpha0, delta0, nu;
    float ih[3];
    float hT, wq; // cell diameter, quadrature weight |T| / 8
};

template <int MODE>
__global__ void __launch_bounds__(ResTile<MODE>::NT)
    k_residual(Mesh m, ResParams P, const float *__restrict__ x, const float *__restrict__ vp,
               const float *__restrict__ fmid, float *__restrict__ out, float *__restrict__ aux,
               const int *__restrict__ flag) {
    using T = ResTile<MODE>;
    if (flag && *flag == 0) return; // predicated launch (fallback path not taken)
    __shared__ float sX[T::NF_STAGE > 0 ? T::NF_STAGE * T::SN : 1];
    __shared__ float sV[T::NF_V * T::VN];
    __shared__ float sAcc[T::NACC * T::VN];
    __shared__ float sAux[MODE == MODE_RES ? T::NP * 32 : 1];

    const int x0 = blockIdx.x * T::TX, y0 = blockIdx.y * T::TY, z0 = blockIdx.z * T::TZ;
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
    // all loads of a thread are issued before its LDS stores, so the staging
    // costs one memory round trip
    if constexpr (MODE == MODE_RES) {
        constexpr int IT = (T::SN + T::NT - 1) / T::NT;
        float tmp[IT][4];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            int s = tid + it * T::NT;
            int lx = s % T::SX, ly = (s / T::SX) % T::SY, lz = s / (T::SX * T::SY);
            bool ok;
            int64_t g = gnode(x0 - 2 + lx, y0 - 2 + ly, z0 - 2 + lz, ok);
            ok &= s < T::SN;
#pragma unroll
            for (int f = 0; f < 4; ++f) tmp[it][f] = ok ? x[f * nfn + g] : 0.0f;
        }
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            int s = tid + it * T::NT;
            if (s < T::SN)
#pragma unroll
                for (int f = 0; f < 4; ++f) sX[f * T::SN + s] = tmp[it][f];
        }
    }
    {
        constexpr int IT = (T::VN + T::NT - 1) / T::NT;
        float tmp[IT][3];
        const float *src = MODE == MODE_RES ? vp : x;
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            int s = tid + it * T::NT;
            int lx = s % T::VX, ly = (s / T::VX) % T::VY, lz = s / (T::VX * T::VY);
            bool ok;
            int64_t g = gnode(x0 - 1 + lx, y0 - 1 + ly, z0 - 1 + lz, ok);
            ok &= s < T::VN;
#pragma unroll
            for (int f = 0; f < 3; ++f) tmp[it][f] = ok ? src[f * nfn + g] : 0.0f;
        }
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            int s = tid + it * T::NT;
            if (s < T::VN) {
#pragma unroll
                for (int f = 0; f < 3; ++f) sV[f * T::VN + s] = tmp[it][f];
#pragma unroll
                for (int f = 0; f < T::NACC; ++f) sAcc[f * T::VN + s] = 0.0f;
            }
        }
    }
    if (MODE == MODE_RES)
        for (int s = tid; s < T::NP * 32; s += T::NT) sAux[s] = 0.0f;
    __syncthreads();

    const int ncx = 2 * m.n[0], ncy = 2 * m.n[1], ncz = 2 * m.n[2]; // fine cells per axis

    for (int round = 0; round < T::ROUNDS; ++round) {
        int e = tid + round * T::NT;
        bool live = e < T::NCELL;
        int ex = 0, ey = 0, ez = 0;
        if (live) {
            ex = e % T::EX;
            ey = (e / T::EX) % T::EY;
            ez = e / (T::EX * T::EY);
        }
        // global cell (lower corner node) and its existence
        int gx = x0 - 1 + ex, gy = y0 - 1 + ey, gz = z0 - 1 + ez;
        if (live) {
            if (m.per[0]) gx = wrap(gx, ncx, 1); else live &= gx >= 0 && gx < ncx;
            if (m.per[1]) gy = wrap(gy, ncy, 1); else live &= gy >= 0 && gy < ncy;
            if (m.per[2]) gz = wrap(gz, ncz, 1); else live &= gz >= 0 && gz < ncz;
        }
        const int colour = ((ex + 1) & 1) | (((ey + 1) & 1) << 1) | (((ez + 1) & 1) << 2);
        // offset of the cell inside its patch (the tile origin is even)
        const int ox = (ex + 1) & 1, oy = (ey + 1) & 1, oz = (ez + 1) & 1;

        float acc[T::NACC][8];
        float cor[4][8];
#pragma unroll
        for (int f = 0; f < T::NACC; ++f)
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[f][j] = 0.0f;
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int j = 0; j < 8; ++j) cor[f][j] = 0.0f;

        if (live) {
            // vertex slots in the staged arrays
            int vs[8], xs[8], cs[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                int a = j & 1, b = (j >> 1) & 1, c = j >> 2;
                vs[j] = (ex + a) + T::VX * ((ey + b) + T::VY * (ez + c));
                xs[j] = (ex + 1 + a) + T::SX * ((ey + 1 + b) + T::SY * (ez + 1 + c));
                // patch corner j: staged coordinate of the patch origin + 2 (a,b,c)
                int px = ex + 1 - ox, py = ey + 1 - oy, pz = ez + 1 - oz;
                cs[j] = (px + 2 * a) + T::SX * ((py + 2 * b) + T::SY * (pz + 2 * c));
            }
            const float ih0 = P.ih[0], ih1 = P.ih[1], ih2 = P.ih[2];

            if (MODE == MODE_RHS) {
                float w[3][8];
#pragma unroll
                for (int d = 0; d < 3; ++d)
#pragma unroll
                    for (int j = 0; j < 8; ++j) w[d][j] = sV[d * T::VN + vs[j]];
                float wv[3][8];
#pragma unroll
                for (int d = 0; d < 3; ++d) eval_val(w[d], wv[d]);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    float va[8], g0[8], g1[8], g2[8];
                    eval_vg(w[a], ih0, ih1, ih2, va, g0, g1, g2);
                    float F[8];
                    if (fmid) {
                        float fj[8], fq[8];
                        const int64_t gbase = 0;
                        (void)gbase;
#pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            int ii = gx + (j & 1), jj = gy + ((j >> 1) & 1), kk = gz + (j >> 2);
                            ii = wrap(ii, m.nf[0], m.per[0]);
                            jj = wrap(jj, m.nf[1], m.per[1]);
                            kk = wrap(kk, m.nf[2], m.per[2]);
                            fj[j] = fmid[a * nfn + ii + (int64_t)m.nf[0] * (jj + (int64_t)m.nf[1] * kk)];
                        }
                        eval_val(fj, fq);
#pragma unroll
                        for (int q = 0; q < 8; ++q) F[q] = fq[q];
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
                    integrate<true, true, true>(F, g0, g1, g2, ih0, ih1, ih2, acc[a]);
                }
            } else {
                // current iterate (x~, p~) at the cell vertices and patch corners
                float vv[3][8], pp[8], cv[3][8], cp[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        vv[d][j] = sX[d * T::SN + xs[j]];
                        cv[d][j] = sX[d * T::SN + cs[j]];
                    }
                    pp[j] = sX[3 * T::SN + xs[j]];
                    cp[j] = sX[3 * T::SN + cs[j]];
                }
                // stabilisation parameters (stabparams): |v|_inf over the vertices
                float vmax2 = 0.0f;
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    vmax2 = fmaxf(vmax2, vv[0][j] * vv[0][j] + vv[1][j] * vv[1][j] + vv[2][j] * vv[2][j]);
                float den = P.nu * (1.0f / (P.hT * P.hT)) + sqrtf(vmax2) / P.hT + P.inv_dt;
                float alphaT = P.alpha0 / den, deltaT = P.delta0 / den;

                // values at Gauss points of x~, vp and pi x~
                float xv[3][8], pv[3][8], piv[3][8], pq[8], div[8];
                float pvert[3][8]; // pi x~ at the cell vertices
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    eval_val(vv[d], xv[d]);
                    float w[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) w[j] = sV[d * T::VN + vs[j]];
                    eval_val(w, pv[d]);
                    pi_vertices(cv[d], ox, oy, oz, pvert[d]);
                    eval_val(pvert[d], piv[d]);
                }
                eval_val(pp, pq);
#pragma unroll
                for (int q = 0; q < 8; ++q) div[q] = 0.0f;

#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    float wa[8], dif[8], sum[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        wa[j] = sV[a * T::VN + vs[j]];
                        dif[j] = wa[j] - vv[a][j];
                        sum[j] = wa[j] + vv[a][j];
                    }
                    float F[8], Gx[8], Gy[8], Gz[8], tmp[8];
                    // (1/k)(vp_a - v_a) and -nu/2 grad(vp_a + v_a), + p d_a phi
                    eval_vg(sum, ih0, ih1, ih2, tmp, Gx, Gy, Gz);
                    eval_val(dif, F);
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        F[q] *= P.inv_dt;
                        Gx[q] *= -P.half_nu;
                        Gy[q] *= -P.half_nu;
                        Gz[q] *= -P.half_nu;
                    }
                    float *Ga = a == 0 ? Gx : (a == 1 ? Gy : Gz);
#pragma unroll
                    for (int q = 0; q < 8; ++q) Ga[q] += pq[q];
                    if (fmid) {
                        float fj[8], fq[8];
#pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            int ii = gx + (j & 1), jj = gy + ((j >> 1) & 1), kk = gz + (j >> 2);
                            ii = wrap(ii, m.nf[0], m.per[0]);
                            jj = wrap(jj, m.nf[1], m.per[1]);
                            kk = wrap(kk, m.nf[2], m.per[2]);
                            fj[j] = fmid[a * nfn + ii + (int64_t)m.nf[0] * (jj + (int64_t)m.nf[1] * kk)];
                        }
                        eval_val(fj, fq);
#pragma unroll
                        for (int q = 0; q < 8; ++q) F[q] += fq[q];
                    }
                    // -1/2 (vp . grad vp_a)
                    float g0[8], g1[8], g2[8];
                    eval_vg(wa, ih0, ih1, ih2, tmp, g0, g1, g2);
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        F[q] -= 0.5f * (pv[0][q] * g0[q] + pv[1][q] * g1[q] + pv[2][q] * g2[q]);
                    // -1/2 (v . grad v_a); keep v . grad v_a for the LPS term
                    float conv[8];
                    eval_vg(vv[a], ih0, ih1, ih2, tmp, g0, g1, g2);
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        conv[q] = xv[0][q] * g0[q] + xv[1][q] * g1[q] + xv[2][q] * g2[q];
                        F[q] -= 0.5f * conv[q];
                    }
                    if (a == 0)
#pragma unroll
                        for (int q = 0; q < 8; ++q) div[q] += g0[q];
                    if (a == 1)
#pragma unroll
                        for (int q = 0; q < 8; ++q) div[q] += g1[q];
                    if (a == 2)
#pragma unroll
                        for (int q = 0; q < 8; ++q) div[q] += g2[q];
                    // LPS: R_a = v.grad v_a - pi v . grad pi v_a, tested with
                    // v.grad phi (own vertices) and pi v . grad pi phi (corners)
                    eval_vg(pvert[a], ih0, ih1, ih2, tmp, g0, g1, g2);
                    float C0[8], C1[8], C2[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        float R = conv[q] - (piv[0][q] * g0[q] + piv[1][q] * g1[q] + piv[2][q] * g2[q]);
                        float dR = deltaT * R;
                        Gx[q] -= dR * xv[0][q];
                        Gy[q] -= dR * xv[1][q];
                        Gz[q] -= dR * xv[2][q];
                        C0[q] = dR * piv[0][q];
                        C1[q] = dR * piv[1][q];
                        C2[q] = dR * piv[2][q];
                    }
                    integrate<true, true, true>(F, Gx, Gy, Gz, ih0, ih1, ih2, acc[a]);
                    float zero[8], cvals[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) zero[q] = 0.0f;
                    integrate<true, true, true>(zero, C0, C1, C2, ih0, ih1, ih2, cvals);
                    pi_transpose(cvals, ox, oy, oz, cor[a]);
                }
                // continuity: -(div v, xi) - alpha_T (grad(p - pi p), grad(xi - pi xi))
                {
                    float tmp[8], g0[8], g1[8], g2[8], h0[8], h1[8], h2[8], pvv[8];
                    eval_vg(pp, ih0, ih1, ih2, tmp, g0, g1, g2);
                    pi_vertices(cp, ox, oy, oz, pvv);
                    eval_vg(pvv, ih0, ih1, ih2, tmp, h0, h1, h2);
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        g0[q] = -alphaT * (g0[q] - h0[q]);
                        g1[q] = -alphaT * (g1[q] - h1[q]);
                        g2[q] = -alphaT * (g2[q] - h2[q]);
                        div[q] = -div[q];
                    }
                    float lps[8], dv[8];
                    integrate<true, true, true>(div, g0, g1, g2, ih0, ih1, ih2, acc[3]);
                    float zero[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) zero[q] = 0.0f;
                    integrate<true, true, true>(zero, g0, g1, g2, ih0, ih1, ih2, lps);
#pragma unroll
                    for (int j = 0; j < 8; ++j) dv[j] = -lps[j];
                    pi_transpose(dv, ox, oy, oz, cor[3]);
                }
            }
#pragma unroll
            for (int f = 0; f < T::NACC; ++f)
#pragma unroll
                for (int j = 0; j < 8; ++j) acc[f][j] *= P.wq;
#pragma unroll
            for (int f = 0; f < 4; ++f)
#pragma unroll
                for (int j = 0; j < 8; ++j) cor[f][j] *= P.wq;
        }

        // ---- colour-ordered accumulation into LDS ----
        // patch slot of an owned patch (halo cells ex == 0 etc. belong to a
        // neighbour's patch and do not contribute corner terms)
        const bool own_patch = ex >= 1 && ey >= 1 && ez >= 1;
        const int pslot = own_patch ? ((ex - 1) / 2 + T::NPX * ((ey - 1) / 2 + T::NPY * ((ez - 1) / 2))) : 0;
        for (int c = 0; c < 8; ++c) {
            if (live && colour == c) {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    int s = (ex + (j & 1)) + T::VX * ((ey + ((j >> 1) & 1)) + T::VY * (ez + (j >> 2)));
#pragma unroll
                    for (int f = 0; f < T::NACC; ++f) sAcc[f * T::VN + s] += acc[f][j];
                }
                if (MODE == MODE_RES && own_patch) {
#pragma unroll
                    for (int j = 0; j < 8; ++j)
#pragma unroll
                        for (int f = 0; f < 4; ++f) sAux[pslot * 32 + 4 * j + f] += cor[f][j];
                }
            }
            __syncthreads();
        }
    }

    // ---- write owned nodes ----
    for (int s = tid; s < T::TX * T::TY * T::TZ; s += T::NT) {
        int lx = s % T::TX, ly = (s / T::TX) % T::TY, lz = s / (T::TX * T::TY);
        int gi = x0 + lx, gj = y0 + ly, gk = z0 + lz;
        if (gi >= m.nf[0] || gj >= m.nf[1] || gk >= m.nf[2]) continue;
        int64_t g = gi + (int64_t)m.nf[0] * (gj + (int64_t)m.nf[1] * gk);
        int slot = (lx + 1) + T::VX * ((ly + 1) + T::VY * (lz + 1));
        bool dir = on_dirichlet(m, gi, gj, gk);
#pragma unroll
        for (int f = 0; f < 3; ++f) out[f * nfn + g] = dir ? 0.0f : sAcc[f * T::VN + slot];
        if (MODE == MODE_RES) out[3 * nfn + g] = sAcc[3 * T::VN + slot];
        else out[3 * nfn + g] = 0.0f;
    }
    if (MODE == MODE_RES) {
        for (int s = tid; s < T::NP * 32; s += T::NT) {
            int ps = s / 32, w = s % 32;
            int px = ps % T::NPX, py = (ps / T::NPX) % T::NPY, pz = ps / (T::NPX * T::NPY);
            int PI = x0 / 2 + px, PJ = y0 / 2 + py, PK = z0 / 2 + pz;
            if (PI >= m.n[0] || PJ >= m.n[1] || PK >= m.n[2]) continue;
            int64_t M = PI + (int64_t)m.n[0] * (PJ + (int64_t)m.n[1] * PK);
            aux[M * 32 + w] = sAux[s];
        }
    }
}

// Adds the corner (pi phi) parts of the LPS terms: a coarse vertex collects
// the per-patch sums of the patches it is a corner of, in ascending patch
// order.  aux[M][4 j + f]: corner j = A + 2B + 4C of patch M, field f.
__global__ void __launch_bounds__(256) k_lps_corners(Mesh m, const float *__restrict__ aux,
                                                     float *__restrict__ r, const int *__restrict__ flag) {
    if (flag && *flag == 0) return;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m.n_coarse) return;
    uint32_t JK = fdiv((uint32_t)t, m.cx), I = (uint32_t)t - JK * m.nc[0];
    uint32_t K = fdiv(JK, m.cy), J = JK - K * m.nc[1];
    // patches with this vertex as a corner, per axis, ascending
    int P[3][2], L[3][2], cnt[3];
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
    float s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int c = 0; c < cnt[2]; ++c)
        for (int b = 0; b < cnt[1]; ++b)
            for (int a = 0; a < cnt[0]; ++a) {
                int64_t M = P[0][a] + (int64_t)m.n[0] * (P[1][b] + (int64_t)m.n[1] * P[2][c]);
                int j = L[0][a] + 2 * L[1][b] + 4 * L[2][c];
                const float *src = aux + M * 32 + 4 * j;
#pragma unroll
                for (int f = 0; f < 4; ++f) s[f] += src[f];
            }
    int gi = 2 * I, gj = 2 * J, gk = 2 * K;
    int64_t g = gi + (int64_t)m.nf[0] * (gj + (int64_t)m.nf[1] * gk);
    bool dir = on_dirichlet(m, gi, gj, gk);
#pragma unroll
    for (int f = 0; f < 3; ++f)
        if (!dir) r[f * m.n_fine + g] += s[f];
    r[3 * m.n_fine + g] += s[3];
}

static ResParams make_params(const Mesh &m, const dnnmg_ns *ns) {
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
static dim3 res_grid(const Mesh &m) {
    using T = ResTile<MODE>;
    return dim3((m.nf[0] + T::TX - 1) / T::TX, (m.nf[1] + T::TY - 1) / T::TY,
                (m.nf[2] + T::TZ - 1) / T::TZ);
}

int residual_launch(const Mesh &m, const dnnmg_ns *ns, const float *x, const float *vprev,
                    const float *fmid, float *r, float *aux, const int *flag, hipStream_t s) {
    ResParams P = make_params(m, ns);
    k_residual<MODE_RES><<<res_grid<MODE_RES>(m), ResTile<MODE_RES>::NT, 0, s>>>(m, P, x, vprev, fmid, r,
                                                                                 aux, flag);
    k_lps_corners<<<blocks_for(m.n_coarse, 256), 256, 0, s>>>(m, aux, r, flag);
    return hip_check(hipGetLastError(), "dnnmg_residual launch");
}

} // namespace dnnmg

using namespace dnnmg;

extern "C" size_t dnnmg_residual_workspace(const dnnmg_box *box) {
    Mesh m;
    if (make_mesh(box, &m)) return 0;
    return (size_t)m.n_patches * 32 * sizeof(float);
}

extern "C" int dnnmg_residual(const dnnmg_box *box, const dnnmg_ns *ns, const float *x,
                              const float *vprev, const float *fmid, float *r, void *ws,
                              size_t ws_bytes, void *stream) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    if ((rc = check_ns(ns))) return rc;
    if (!x || !vprev || !r || !ws) return fail(DNNMG_ERR_ARG, "dnnmg_residual: NULL pointer");
    if (ws_bytes < (size_t)m.n_patches * 32 * sizeof(float))
        return fail(DNNMG_ERR_SHAPE, "dnnmg_residual: workspace %zu < %zu bytes", ws_bytes,
                    (size_t)m.n_patches * 32 * sizeof(float));
    return residual_launch(m, ns, x, vprev, fmid, r, (float *)ws, nullptr, (hipStream_t)stream);
}

extern "C" int dnnmg_rhs(const dnnmg_box *box, const dnnmg_ns *ns, const float *v, const float *fmid,
                         float *b, void *stream) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    if ((rc = check_ns(ns))) return rc;
    if (!v || !b) return fail(DNNMG_ERR_ARG, "dnnmg_rhs: NULL pointer");
    ResParams P = make_params(m, ns);
    k_residual<MODE_RHS><<<res_grid<MODE_RHS>(m), ResTile<MODE_RHS>::NT, 0, (hipStream_t)stream>>>(
        m, P, v, nullptr, fmid, b, nullptr, nullptr);
    return hip_check(hipGetLastError(), "dnnmg_rhs launch");
}
