// Plain fine-level correction: additive patch-Vanka sweeps on the fine
// Crank-Nicolson system (the local-problem smoother of arXiv 2307.14837,
// Sec. 2.4, applied on the patches of Sec. 4.2), used as the fallback of the
// residual indicator.  One sweep:
//   r = F - A(x);  on every patch P solve A_P delta_P = r_P;
//   x <- x + omega * mu (.) sum_P L(delta_P)     (the averaging of eq. (defL))
// A_P is the Crank-Nicolson operator linearised at the current velocity with
// frozen convection, restricted to the patch's 108 unknowns: Galerkin terms
// from the 64 fine cells touching the patch, the pressure stabilisation
// alpha_T over the patch's own 8 cells; Dirichlet velocities are fixed.
//
// Kernel layout: one wave per patch.  The 27 x 27 blocks (velocity K shared
// by the three components, divergence blocks B_a, pressure block C) are
// assembled in LDS from per-cell element tables; the local system is solved
// through the velocity block's LU and the pressure Schur complement
//   S = C + sum_a B_a K^-1 B_a^T,  S dp = r_p - sum_a B_a K^-1 r_a,
//   du_a = K^-1 (r_a + B_a^T dp).
#include "common.hpp"
#include "mlp.hpp"

namespace dnnmg {

constexpr float VGLO = 0.21132486540518713f; // Gauss points 1/2 -+ 1/(2 sqrt 3)

// Element tables of one fine cell (uniform mesh), computed on the host in FP64.
struct VankaTables {
    float M[64];      // (phi_j, phi_i)              [i*8 + j]
    float K[64];      // (grad phi_j, grad phi_i)
    float D[3][64];   // (d_a phi_j, phi_i)
    float phi[8][8];  // phi_v at Gauss point q       [q][v]
    float dphi[8][8][3]; // grad phi_v at q            [q][v][d]
    float wq;         // quadrature weight |T| / 8
};

struct VankaParams {
    float inv_dt, half_nu, nu, alpha0, hT;
    float ih[3], iH[3];
};

__device__ __forceinline__ float l1f(int a, float t) { return a ? t : 1.0f - t; }
__device__ __forceinline__ float dl1f(int a) { return a ? 1.0f : -1.0f; }

// Patch-local node (a,b,c) in {0,1,2}^3 -> iota
__device__ __forceinline__ int iota_of(int a, int b, int c) { return a + 3 * b + 9 * c; }

// COUPLED: full velocity-pressure local systems; otherwise the momentum
// equations with the pressure held (K delta_a = r_a per component, dp = 0).
// STRIDED = false: one patch per block (the grid covers the patches);
// STRIDED = true: blocks walk the patches with stride gridDim.x, for launches
// that a device flag may skip on a smaller grid.
// INVERSE (coupled only): r is not read; D receives the local inverse
// A_P^-1 of every patch instead, column-major (D[M][j][row], 108 x 108),
// each column the local solve of a unit right-hand side.
template <bool COUPLED, bool STRIDED = false, bool INVERSE = false>
__global__ void __launch_bounds__(64)
    k_vanka_local(Mesh m, VankaTables T, VankaParams P, const float *__restrict__ x,
                  const float *__restrict__ r, float *__restrict__ D, const int *__restrict__ flag) {
    static_assert(!INVERSE || (COUPLED && !STRIDED), "local inverses are built for the coupled systems");
    constexpr int NB = COUPLED ? 3 : 1;   // divergence blocks kept
    constexpr int NO = COUPLED ? 8 : 1;   // own cells with LPS tables
    constexpr int NZ = COUPLED ? 84 : 3;  // right-hand sides of K
    if (flag && *flag == 0) return;
    const int lane = threadIdx.x;
    int64_t M = blockIdx.x;
    do { // one patch; STRIDED: the next one gridDim.x on
    if constexpr (STRIDED) __syncthreads(); // the previous patch's LDS reads are complete
    uint32_t J_K = fdiv((uint32_t)M, m.px), I = (uint32_t)M - J_K * m.n[0];
    uint32_t K = fdiv(J_K, m.py), J = J_K - K * m.n[1];
    const int64_t nfn = m.n_fine;

    __shared__ float sW[3][125];       // velocity at patch-local nodes {-1..3}^3
    __shared__ float sWq[64][8][3];    // velocity at the Gauss points of the 64 cells
    __shared__ float sAlpha[8];        // alpha_T of the own cells
    __shared__ float sK[27][28];       // velocity block (LU in place)
    __shared__ float sB[NB][27][28];   // divergence blocks B_a[i][j] = (d_a phi_j, phi_i)
    __shared__ float sC[27][28];       // pressure block, then the Schur complement
    __shared__ float sZ[NZ][28];       // K^-1 B_a^T columns (81) and K^-1 r_a (last 3)
    __shared__ float sR[108];
    __shared__ float sKap[NO][8][27][3]; // grad(phi_i - pi phi_i) on own cell o at Gauss point q
    __shared__ int sDir[27];
    __shared__ int sExist[64];

    // ---- velocity around the patch, residual on the patch ----
    for (int s = lane; s < 125; s += 64) {
        int a = s % 5 - 1, b = (s / 5) % 5 - 1, c = s / 25 - 1;
        int gi = wrap(2 * (int)I + a, m.nf[0], m.per[0]);
        int gj = wrap(2 * (int)J + b, m.nf[1], m.per[1]);
        int gk = wrap(2 * (int)K + c, m.nf[2], m.per[2]);
        bool ok = gi >= 0 && gi < m.nf[0] && gj >= 0 && gj < m.nf[1] && gk >= 0 && gk < m.nf[2];
        int64_t g = gi + (int64_t)m.nf[0] * (gj + (int64_t)m.nf[1] * gk);
#pragma unroll
        for (int d = 0; d < 3; ++d) sW[d][s] = ok ? x[d * nfn + g] : 0.0f;
    }
    for (int s = lane; s < 108; s += 64) {
        int f = s / 27, t = s % 27;
        int a = t % 3, b = (t / 3) % 3, c = t / 9;
        int gi = wrap(2 * (int)I + a, m.nf[0], m.per[0]);
        int gj = wrap(2 * (int)J + b, m.nf[1], m.per[1]);
        int gk = wrap(2 * (int)K + c, m.nf[2], m.per[2]);
        sR[s] = INVERSE ? 0.0f : r[f * nfn + gi + (int64_t)m.nf[0] * (gj + (int64_t)m.nf[1] * gk)];
        if (f == 0) sDir[t] = on_dirichlet(m, gi, gj, gk) ? 1 : 0;
    }
    for (int s = lane; s < 27 * 28; s += 64) {
        (&sK[0][0])[s] = 0.0f;
        if constexpr (COUPLED) {
            (&sC[0][0])[s] = 0.0f;
#pragma unroll
            for (int a = 0; a < NB; ++a) (&sB[a][0][0])[s] = 0.0f;
        }
    }
    __syncthreads();

    // ---- per cell (lane = cell): existence and velocity at Gauss points ----
    {
        int cx = lane % 4 - 1, cy = (lane / 4) % 4 - 1, cz = lane / 16 - 1;
        int g0[3] = {2 * (int)I + cx, 2 * (int)J + cy, 2 * (int)K + cz};
        bool ex = true;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (!m.per[a] && (g0[a] < 0 || g0[a] >= 2 * m.n[a])) ex = false;
        sExist[lane] = ex ? 1 : 0;
        float wv[3][8];
        float vmax2 = 0.0f;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            int s = (cx + 1 + (v & 1)) + 5 * ((cy + 1 + ((v >> 1) & 1)) + 5 * (cz + 1 + (v >> 2)));
            float n2 = 0.0f;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                wv[d][v] = sW[d][s];
                n2 += wv[d][v] * wv[d][v];
            }
            vmax2 = fmaxf(vmax2, n2);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                float acc = 0.0f;
#pragma unroll
                for (int v = 0; v < 8; ++v) acc = fmaf(T.phi[q][v], wv[d][v], acc);
                sWq[lane][q][d] = acc;
            }
        bool own = cx >= 0 && cx <= 1 && cy >= 0 && cy <= 1 && cz >= 0 && cz <= 1;
        if (own) {
            float den = P.nu / (P.hT * P.hT) + sqrtf(vmax2) / P.hT + P.inv_dt;
            sAlpha[cx + 2 * cy + 4 * cz] = P.alpha0 / den;
        }
    }
    // ---- fluctuation gradients grad(phi_i - pi phi_i) on the own cells ----
    if constexpr (COUPLED)
    for (int s = lane; s < 8 * 8 * 27; s += 64) {
        int o = s / 216, q = (s / 27) % 8, t = s % 27;
        int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
        int a = t % 3, b = (t / 3) % 3, c = t / 9;
        float xi[3] = {(q & 1) ? 1.0f - VGLO : VGLO, ((q >> 1) & 1) ? 1.0f - VGLO : VGLO,
                       (q >> 2) ? 1.0f - VGLO : VGLO};
        float g[3] = {0.f, 0.f, 0.f};
        int la = a - ox, lb = b - oy, lc = c - oz;
        if (la >= 0 && la <= 1 && lb >= 0 && lb <= 1 && lc >= 0 && lc <= 1) {
            g[0] = dl1f(la) * P.ih[0] * l1f(lb, xi[1]) * l1f(lc, xi[2]);
            g[1] = l1f(la, xi[0]) * dl1f(lb) * P.ih[1] * l1f(lc, xi[2]);
            g[2] = l1f(la, xi[0]) * l1f(lb, xi[1]) * dl1f(lc) * P.ih[2];
        }
        if (!(a & 1) && !(b & 1) && !(c & 1)) { // patch corner: subtract the coarse function
            int A = a >> 1, B = b >> 1, C = c >> 1;
            float xc[3] = {(ox + xi[0]) * 0.5f, (oy + xi[1]) * 0.5f, (oz + xi[2]) * 0.5f};
            g[0] -= dl1f(A) * P.iH[0] * l1f(B, xc[1]) * l1f(C, xc[2]);
            g[1] -= l1f(A, xc[0]) * dl1f(B) * P.iH[1] * l1f(C, xc[2]);
            g[2] -= l1f(A, xc[0]) * l1f(B, xc[1]) * dl1f(C) * P.iH[2];
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) sKap[o][q][t][d] = g[d];
    }
    __syncthreads();

    // ---- Galerkin assembly: lane = (i, j) of the cell's 8 x 8 element block ----
    {
        const int i = lane >> 3, j = lane & 7;
        const float Mij = T.M[i * 8 + j], Kij = T.K[i * 8 + j];
        const float D0 = T.D[0][i * 8 + j], D1 = T.D[1][i * 8 + j], D2 = T.D[2][i * 8 + j];
        for (int cell = 0; cell < 64; ++cell) {
            __syncthreads();             // previous cell's LDS sums are complete
            if (!sExist[cell]) continue; // uniform across the wave
            int cx = cell % 4 - 1, cy = (cell / 4) % 4 - 1, cz = cell / 16 - 1;
            int ai = cx + (i & 1), bi = cy + ((i >> 1) & 1), ci = cz + (i >> 2);
            int aj = cx + (j & 1), bj = cy + ((j >> 1) & 1), cj = cz + (j >> 2);
            bool in = ai >= 0 && ai <= 2 && bi >= 0 && bi <= 2 && ci >= 0 && ci <= 2 && aj >= 0 &&
                      aj <= 2 && bj >= 0 && bj <= 2 && cj >= 0 && cj <= 2;
            float conv = 0.0f;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                float wg = sWq[cell][q][0] * T.dphi[q][j][0] + sWq[cell][q][1] * T.dphi[q][j][1] +
                           sWq[cell][q][2] * T.dphi[q][j][2];
                conv = fmaf(wg, T.phi[q][i], conv);
            }
            if (in) {
                int ti = iota_of(ai, bi, ci), tj = iota_of(aj, bj, cj);
                sK[ti][tj] += P.inv_dt * Mij + 0.5f * T.wq * conv + P.half_nu * Kij;
                if constexpr (COUPLED) {
                    sB[0][ti][tj] += D0;
                    sB[NB - 2][ti][tj] += D1;
                    sB[NB - 1][ti][tj] += D2;
                }
            }
        }
    }
    // ---- pressure stabilisation over the own cells: lane over (i, j) ----
    if constexpr (COUPLED)
    for (int e = lane; e < 729; e += 64) {
        int i = e / 27, j = e % 27;
        float acc = 0.0f;
        for (int o = 0; o < 8; ++o) {
            float s = 0.0f;
#pragma unroll
            for (int q = 0; q < 8; ++q)
                s += sKap[o][q][i][0] * sKap[o][q][j][0] + sKap[o][q][i][1] * sKap[o][q][j][1] +
                     sKap[o][q][i][2] * sKap[o][q][j][2];
            acc = fmaf(sAlpha[o], s, acc);
        }
        sC[i][j] = acc * T.wq;
    }
    __syncthreads();

    // ---- Dirichlet velocities: identity rows/columns of K, zero B columns ----
    for (int e = lane; e < 729; e += 64) {
        int i = e / 27, j = e % 27;
        if (sDir[i] || sDir[j]) sK[i][j] = (i == j) ? 1.0f : 0.0f;
        if constexpr (COUPLED)
            if (sDir[j]) {
#pragma unroll
                for (int a = 0; a < NB; ++a) sB[a][i][j] = 0.0f;
            }
    }
    __syncthreads();

    // ---- LU of K (no pivoting: mass-dominated, diagonally dominant) ----
    for (int k = 0; k < 27; ++k) {
        float piv = sK[k][k];
        for (int e = lane; e < (26 - k) * (27 - k); e += 64) {
            int i = k + 1 + e / (27 - k), j = k + e % (27 - k);
            float lik = sK[i][k] / piv;
            if (j > k) sK[i][j] -= lik * sK[k][j];
        }
        __syncthreads();
        for (int i = k + 1 + lane; i < 27; i += 64) sK[i][k] /= piv;
        __syncthreads();
    }
    // ---- K^-1 applied to the right-hand sides: B_a^T columns and r_a ----
    for (int col = lane; col < NZ; col += 64) {
        float v[27];
        if (COUPLED && col < NZ - 3) {
            int a = col / 27, jj = col % 27; // column jj of B_a^T = row jj of B_a
#pragma unroll
            for (int i = 0; i < 27; ++i) v[i] = sB[a % NB][jj][i];
        } else {
            int a = col - (NZ - 3);
#pragma unroll
            for (int i = 0; i < 27; ++i) v[i] = sDir[i] ? 0.0f : sR[27 * a + i];
        }
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            float s = v[i];
            for (int k = 0; k < i; ++k) s -= sK[i][k] * v[k];
            v[i] = s;
        }
#pragma unroll
        for (int i = 26; i >= 0; --i) {
            float s = v[i];
            for (int k = i + 1; k < 27; ++k) s -= sK[i][k] * v[k];
            v[i] = s / sK[i][i];
        }
#pragma unroll
        for (int i = 0; i < 27; ++i) sZ[col][i] = v[i];
    }
    __syncthreads();
    float *out = D + M * 108;
    if constexpr (!COUPLED) {
        for (int s2 = lane; s2 < 108; s2 += 64) {
            int f = s2 / 27, i = s2 % 27;
            out[s2] = (f < 3 && !sDir[i]) ? sZ[f][i] : 0.0f;
        }
        continue;
    } else {
    // ---- Schur complement S = C + sum_a B_a K^-1 B_a^T, s = r_p - sum_a B_a K^-1 r_a ----
    for (int e = lane; e < 729; e += 64) {
        int i = e / 27, j = e % 27;
        float acc = sC[i][j];
#pragma unroll
        for (int a = 0; a < 3; ++a)
            for (int k = 0; k < 27; ++k) acc = fmaf(sB[a][i][k], sZ[27 * a + j][k], acc);
        sC[i][j] = acc;
    }
    __shared__ float sS[27];
    if (lane < 27) {
        float acc = sR[81 + lane];
#pragma unroll
        for (int a = 0; a < 3; ++a)
            for (int k = 0; k < 27; ++k) acc -= sB[a][lane][k] * sZ[81 + a][k];
        sS[lane] = acc;
    }
    __syncthreads();
    // ---- LU of S (positive definite symmetric part; no pivoting) ----
    for (int k = 0; k < 27; ++k) {
        float piv = sC[k][k];
        for (int e = lane; e < (26 - k) * (27 - k); e += 64) {
            int i = k + 1 + e / (27 - k), j = k + e % (27 - k);
            float lik = sC[i][k] / piv;
            if (j > k) sC[i][j] -= lik * sC[k][j];
        }
        __syncthreads();
        for (int i = k + 1 + lane; i < 27; i += 64) sC[i][k] /= piv;
        __syncthreads();
    }
    if constexpr (INVERSE) {
        // column j of A_P^-1: the local solve of e_j.  A velocity unit
        // vector (f, jj): y = K^-1 e_jj, dp = S^-1 (-B_f y), du_a = [a = f] y
        // + K^-1 B_a^T dp; a pressure one (jj): dp = S^-1 e_jj, du_a =
        // K^-1 B_a^T dp.  Dirichlet velocities: zero rows and columns.
        float *Ai = D + M * (108 * 108);
        for (int j = lane; j < 108; j += 64) {
            const int f = j / 27, jj = j % 27;
            const bool vel = f < 3;
            float y[27], v[27];
#pragma unroll
            for (int i = 0; i < 27; ++i) y[i] = (vel && i == jj && !sDir[jj]) ? 1.0f : 0.0f;
            if (vel) {
#pragma unroll
                for (int i = 0; i < 27; ++i) {
                    float t = y[i];
#pragma unroll
                    for (int k = 0; k < i; ++k) t -= sK[i][k] * y[k];
                    y[i] = t;
                }
#pragma unroll
                for (int i = 26; i >= 0; --i) {
                    float t = y[i];
#pragma unroll
                    for (int k = i + 1; k < 27; ++k) t -= sK[i][k] * y[k];
                    y[i] = t / sK[i][i];
                }
#pragma unroll
                for (int i = 0; i < 27; ++i) {
                    float t = 0.0f;
#pragma unroll
                    for (int k = 0; k < 27; ++k) t = fmaf(sB[f][i][k], y[k], t);
                    v[i] = -t;
                }
            } else {
#pragma unroll
                for (int i = 0; i < 27; ++i) v[i] = i == jj ? 1.0f : 0.0f;
            }
#pragma unroll
            for (int i = 0; i < 27; ++i) {
                float t = v[i];
#pragma unroll
                for (int k = 0; k < i; ++k) t -= sC[i][k] * v[k];
                v[i] = t;
            }
#pragma unroll
            for (int i = 26; i >= 0; --i) {
                float t = v[i];
#pragma unroll
                for (int k = i + 1; k < 27; ++k) t -= sC[i][k] * v[k];
                v[i] = t / sC[i][i];
            }
            float *col = Ai + j * 108;
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int i = 0; i < 27; ++i) {
                    float t = a == f ? y[i] : 0.0f;
#pragma unroll
                    for (int k = 0; k < 27; ++k) t = fmaf(sZ[27 * a + k][i], v[k], t);
                    col[27 * a + i] = sDir[i] ? 0.0f : t;
                }
#pragma unroll
            for (int i = 0; i < 27; ++i) col[81 + i] = v[i];
        }
        continue;
    }
    __shared__ float sDp[27];
    if (lane == 0) {
        float v[27];
        for (int i = 0; i < 27; ++i) {
            float s = sS[i];
            for (int k = 0; k < i; ++k) s -= sC[i][k] * v[k];
            v[i] = s;
        }
        for (int i = 26; i >= 0; --i) {
            float s = v[i];
            for (int k = i + 1; k < 27; ++k) s -= sC[i][k] * v[k];
            v[i] = s / sC[i][i];
        }
        for (int i = 0; i < 27; ++i) sDp[i] = v[i];
    }
    __syncthreads();
    // ---- velocity corrections du_a = K^-1 r_a + K^-1 B_a^T dp; write delta_P ----
    for (int s = lane; s < 108; s += 64) {
        int f = s / 27, i = s % 27;
        float v;
        if (f < 3) {
            v = sZ[81 + f][i];
            for (int jj = 0; jj < 27; ++jj) v = fmaf(sZ[27 * f + jj][i], sDp[jj], v);
            if (sDir[i]) v = 0.0f;
        } else {
            v = sDp[i];
        }
        out[s] = v;
    }

    }
    } while (STRIDED && (M += gridDim.x) < m.n_patches);
}

// x_out = x + omega * mu (.) sum over patches holding the node of delta_P;
// Dirichlet velocities unchanged.  Safe in place (x_out == x).
__global__ void __launch_bounds__(256) k_vanka_apply(Mesh m, const float *__restrict__ D, float omega,
                                                     const float *x, float *xout,
                                                     const int *__restrict__ flag) {
    if (flag && *flag == 0) return;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m.n_fine;
         t += (int64_t)gridDim.x * blockDim.x) {
    uint32_t jk = fdiv((uint32_t)t, m.fx), i = (uint32_t)t - jk * m.nf[0];
    uint32_t k = fdiv(jk, m.fy), j = jk - k * m.nf[1];
    int P[3][2], Lc[3][2], cnt[3];
    const int c3[3] = {(int)i, (int)j, (int)k};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int ci = c3[a];
        cnt[a] = 0;
        if (ci & 1) {
            P[a][0] = (ci - 1) >> 1;
            Lc[a][0] = 1;
            cnt[a] = 1;
            continue;
        }
        int hi = ci >> 1, lo = hi - 1;
        if (m.per[a]) {
            if (lo < 0) lo += m.n[a];
            P[a][0] = lo < hi ? lo : hi;
            Lc[a][0] = lo < hi ? 2 : 0;
            P[a][1] = lo < hi ? hi : lo;
            Lc[a][1] = lo < hi ? 0 : 2;
            cnt[a] = 2;
        } else {
            if (lo >= 0) { P[a][cnt[a]] = lo; Lc[a][cnt[a]] = 2; ++cnt[a]; }
            if (hi < m.n[a]) { P[a][cnt[a]] = hi; Lc[a][cnt[a]] = 0; ++cnt[a]; }
        }
    }
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int c = 0; c < cnt[2]; ++c)
        for (int b = 0; b < cnt[1]; ++b)
            for (int a = 0; a < cnt[0]; ++a) {
                int64_t Mp = P[0][a] + (int64_t)m.n[0] * (P[1][b] + (int64_t)m.n[1] * P[2][c]);
                int io = Lc[0][a] + 3 * Lc[1][b] + 9 * Lc[2][c];
#pragma unroll
                for (int f = 0; f < 4; ++f) acc[f] += D[Mp * 108 + 27 * f + io];
            }
    const float inv = 1.0f / (float)(cnt[0] * cnt[1] * cnt[2]);
    const bool dir = on_dirichlet(m, i, j, k);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        float dv = (f < 3 && dir) ? 0.0f : acc[f] * inv;
        xout[f * m.n_fine + t] = x[f * m.n_fine + t] + omega * dv;
    }
    }
}

static void make_tables(const Mesh &m, const dnnmg_ns *ns, VankaTables &T, VankaParams &P) {
    const double g[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
    const double *h = m.hd;
    const double vol = h[0] * h[1] * h[2], wq = 0.125 * vol;
    auto l1 = [](int a, double t) { return a ? t : 1.0 - t; };
    auto dl1 = [](int a) { return a ? 1.0 : -1.0; };
    double phi[8][8], dphi[8][8][3];
    for (int q = 0; q < 8; ++q) {
        double xi[3] = {g[q & 1], g[(q >> 1) & 1], g[q >> 2]};
        for (int v = 0; v < 8; ++v) {
            int a = v & 1, b = (v >> 1) & 1, c = v >> 2;
            phi[q][v] = l1(a, xi[0]) * l1(b, xi[1]) * l1(c, xi[2]);
            dphi[q][v][0] = dl1(a) / h[0] * l1(b, xi[1]) * l1(c, xi[2]);
            dphi[q][v][1] = l1(a, xi[0]) * dl1(b) / h[1] * l1(c, xi[2]);
            dphi[q][v][2] = l1(a, xi[0]) * l1(b, xi[1]) * dl1(c) / h[2];
            T.phi[q][v] = (float)phi[q][v];
            for (int d = 0; d < 3; ++d) T.dphi[q][v][d] = (float)dphi[q][v][d];
        }
    }
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) {
            double Mm = 0, Kk = 0, Dd[3] = {0, 0, 0};
            for (int q = 0; q < 8; ++q) {
                Mm += wq * phi[q][j] * phi[q][i];
                Kk += wq * (dphi[q][j][0] * dphi[q][i][0] + dphi[q][j][1] * dphi[q][i][1] +
                            dphi[q][j][2] * dphi[q][i][2]);
                for (int a = 0; a < 3; ++a) Dd[a] += wq * dphi[q][j][a] * phi[q][i];
            }
            T.M[i * 8 + j] = (float)Mm;
            T.K[i * 8 + j] = (float)Kk;
            for (int a = 0; a < 3; ++a) T.D[a][i * 8 + j] = (float)Dd[a];
        }
    T.wq = (float)wq;
    P.inv_dt = (float)(1.0 / ns->dt);
    P.half_nu = (float)(0.5 * ns->nu);
    P.nu = (float)ns->nu;
    P.alpha0 = (float)ns->alpha0;
    P.hT = (float)sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
    for (int a = 0; a < 3; ++a) {
        P.ih[a] = (float)(1.0 / h[a]);
        P.iH[a] = (float)(0.5 / h[a]);
    }
}

// Entry used by the public calls: `sweeps` sweeps on x (in place), each
// preceded by a residual of the current iterate (from vprev and fmid, or,
// when b is given, against that right-hand side).  ws layout: r (4 n_fine
// floats), residual workspace, D (n_patches * 108 floats).
int vanka_sweeps(const dnnmg_box *box, const dnnmg_ns *ns, float *x, const float *vprev,
                 const float *fmid, int sweeps, float omega, int coupled, char *ws, const int *flag,
                 hipStream_t s, const float *b = nullptr);

} // namespace dnnmg

using namespace dnnmg;

// residual launch with an optional device flag (defined in residual.hip)
namespace dnnmg {
int residual_launch(const Mesh &m, const dnnmg_ns *ns, const float *x, const float *vprev,
                    const float *fmid, float *r, float *aux, const int *flag, hipStream_t s);
int residual_launch_b(const Mesh &m, const dnnmg_ns *ns, const float *x, const float *b, float *r, float *aux,
                      const int *flag, hipStream_t s);
size_t lps_ws_bytes(const Mesh &m);
size_t vanka_ws_bytes(const Mesh &m) {
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    return up(sizeof(float) * 4 * m.n_fine) + lps_ws_bytes(m) + up(sizeof(float) * 108 * m.n_patches);
}

int vanka_sweeps(const dnnmg_box *box, const dnnmg_ns *ns, float *x, const float *vprev,
                 const float *fmid, int sweeps, float omega, int coupled, char *ws, const int *flag,
                 hipStream_t s, const float *b) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    VankaTables T;
    VankaParams P;
    make_tables(m, ns, T, P);
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    float *r = (float *)ws;
    float *aux = (float *)(ws + up(sizeof(float) * 4 * m.n_fine));
    float *D = (float *)(ws + up(sizeof(float) * 4 * m.n_fine) + lps_ws_bytes(m));
    // predicated sweeps (fallback): grid-stride grids of a few workgroups per
    // compute unit, so sweeps that are not taken cost little
    const int ncu = device_cus();
    const unsigned strided_grid = (unsigned)(m.n_patches < 16 * (int64_t)ncu ? m.n_patches : 16 * (int64_t)ncu);
    const unsigned apply_grid =
        flag && blocks_for(m.n_fine, 256) > 4u * ncu ? 4u * ncu : blocks_for(m.n_fine, 256);
    for (int it = 0; it < sweeps; ++it) {
        if ((rc = b ? residual_launch_b(m, ns, x, b, r, aux, flag, s)
                    : residual_launch(m, ns, x, vprev, fmid, r, aux, flag, s)))
            return rc;
        if (flag && coupled)
            k_vanka_local<true, true><<<strided_grid, 64, 0, s>>>(m, T, P, x, r, D, flag);
        else if (flag)
            k_vanka_local<false, true><<<strided_grid, 64, 0, s>>>(m, T, P, x, r, D, flag);
        else if (coupled)
            k_vanka_local<true><<<(unsigned)m.n_patches, 64, 0, s>>>(m, T, P, x, r, D, nullptr);
        else
            k_vanka_local<false><<<(unsigned)m.n_patches, 64, 0, s>>>(m, T, P, x, r, D, nullptr);
        k_vanka_apply<<<apply_grid, 256, 0, s>>>(m, D, omega, x, x, flag);
    }
    return hip_check(hipGetLastError(), "dnnmg_vanka launch");
}
} // namespace dnnmg

namespace dnnmg {
// D_P = A_P^-1 d_P on every patch from the column-major local inverses of
// k_vanka_local<true, false, true>: two patches per block, lane = row.
__global__ void __launch_bounds__(128) k_vanka_apply_inverse(Mesh m, const float *__restrict__ Ainv,
                                                             const float *__restrict__ d, float *__restrict__ D) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t M = 2 * (int64_t)blockIdx.x + w;
    __shared__ float sd[2][108];
    if (M < m.n_patches) {
        const uint32_t JK = fdiv((uint32_t)M, m.px), I = (uint32_t)M - JK * m.n[0];
        const uint32_t K = fdiv(JK, m.py), J = JK - K * m.n[1];
        for (int s = lane; s < 108; s += 64) {
            const int f = s / 27, t = s % 27, a = t % 3, b = (t / 3) % 3, c = t / 9;
            const int gi = wrap(2 * (int)I + a, m.nf[0], m.per[0]);
            const int gj = wrap(2 * (int)J + b, m.nf[1], m.per[1]);
            const int gk = wrap(2 * (int)K + c, m.nf[2], m.per[2]);
            sd[w][s] = d[f * m.n_fine + gi + (int64_t)m.nf[0] * (gj + (int64_t)m.nf[1] * gk)];
        }
    }
    __syncthreads();
    if (M >= m.n_patches) return;
    const float *A = Ainv + M * (108 * 108);
    const bool two = lane + 64 < 108;
    float a0 = 0.0f, a1 = 0.0f;
    for (int j = 0; j < 108; ++j) {
        const float dj = sd[w][j];
        a0 = fmaf(A[j * 108 + lane], dj, a0);
        if (two) a1 = fmaf(A[j * 108 + 64 + lane], dj, a1);
    }
    D[M * 108 + lane] = a0;
    if (two) D[M * 108 + 64 + lane] = a1;
}

size_t vanka_local_bytes(const Mesh &m) { return sizeof(float) * 108 * (size_t)m.n_patches; }
size_t vanka_inverse_bytes(const Mesh &m) { return sizeof(float) * 108 * 108 * (size_t)m.n_patches; }

// The local inverses of the coupled patch-Vanka systems (the multigrid
// smoother of the coarse solve, Sec. 2.4): A_P, the local Crank-Nicolson
// operator linearised at x (frozen convection), inverted on every patch.
// They depend on x only, so one factorisation serves every application at
// that linearisation.  Ainv: vanka_inverse_bytes(m).
int vanka_factor(const Mesh &m, const dnnmg_ns *ns, const float *x, float *Ainv, hipStream_t s) {
    VankaTables T;
    VankaParams P;
    make_tables(m, ns, T, P);
    k_vanka_local<true, false, true><<<(unsigned)m.n_patches, 64, 0, s>>>(m, T, P, x, nullptr, Ainv, nullptr);
    return hip_check(hipGetLastError(), "vanka factor launch");
}

// One linear coupled patch-Vanka step with factored local systems:
// D_P = A_P^-1 d_P, then z <- z + omega * mu (.) sum_P L(D_P) with Dirichlet
// velocities unchanged.  D: vanka_local_bytes(m).
int vanka_apply_factored(const Mesh &m, const float *Ainv, const float *d, float *D, float omega, float *z,
                         hipStream_t s) {
    k_vanka_apply_inverse<<<(unsigned)((m.n_patches + 1) / 2), 128, 0, s>>>(m, Ainv, d, D);
    k_vanka_apply<<<blocks_for(m.n_fine, 256), 256, 0, s>>>(m, D, omega, z, z, nullptr);
    return hip_check(hipGetLastError(), "vanka apply launch");
}
} // namespace dnnmg

// Indicator decision on the device: fall back unless ||r(x_corr)||^2 <=
// theta^2 ||r(x~)||^2 (a NaN in the corrected residual also falls back).
__global__ void k_indicator_flag(const double *__restrict__ norms, double theta2, int *flag,
                                 int *flag_out) {
    if (threadIdx.x != 0) return;
    // eta^2 = norms[1] / norms[0] against theta^2.  An infinite threshold
    // never falls back (the indicator is only evaluated); a zero reference
    // residual falls back only if the corrected one is not zero too (0/0 is
    // read as eta = 0); a NaN corrected residual falls back.
    const double n0 = norms[0], n1 = norms[1];
    int f;
    if (isinf(theta2))
        f = 0;
    else if (n0 > 0.0)
        f = (n1 <= theta2 * n0) ? 0 : 1;
    else
        f = (n1 <= 0.0) ? 0 : 1;
    *flag = f;
    if (flag_out) *flag_out = f;
}

__global__ void __launch_bounds__(256) k_copy_pred(int64_t n, const float *__restrict__ src,
                                                   float *__restrict__ dst, const int *__restrict__ flag) {
    if (*flag == 0) return;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        dst[t] = src[t];
}

// grid of the predicated copy: a few workgroups per compute unit
static unsigned copy_grid(const Mesh &m) {
    const unsigned full = blocks_for(4 * m.n_fine, 256), cap = 4u * (unsigned)device_cus();
    return full < cap ? full : cap;
}

extern "C" size_t dnnmg_fallback_workspace(const dnnmg_box *box) {
    Mesh m;
    if (make_mesh(box, &m)) return 0;
    return vanka_ws_bytes(m) + 256;
}

extern "C" int dnnmg_fallback(const dnnmg_box *box, const dnnmg_ns *ns, const float *xt, const float *vprev,
                              const float *fmid, const double *norms, double theta, int sweeps, float omega,
                              float *xcorr, int *flag_out, void *ws, size_t ws_bytes, void *stream) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    if (!ns || !(ns->dt > 0.0)) return fail(DNNMG_ERR_ARG, "dnnmg_fallback: bad ns");
    if (!xt || !vprev || !norms || !xcorr || !ws) return fail(DNNMG_ERR_ARG, "dnnmg_fallback: NULL pointer");
    if (sweeps < 0 || !(omega > 0.0f) || !(theta >= 0.0))
        return fail(DNNMG_ERR_ARG, "dnnmg_fallback: need sweeps >= 0, omega > 0, theta >= 0");
    if (ws_bytes < dnnmg_fallback_workspace(box))
        return fail(DNNMG_ERR_SHAPE, "dnnmg_fallback: workspace %zu < %zu bytes", ws_bytes,
                    dnnmg_fallback_workspace(box));
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    int *flag = (int *)(w + vanka_ws_bytes(m));
    k_indicator_flag<<<1, 64, 0, s>>>(norms, theta * theta, flag, flag_out);
    k_copy_pred<<<copy_grid(m), 256, 0, s>>>(4 * m.n_fine, xt, xcorr, flag);
    if ((rc = hip_check(hipGetLastError(), "dnnmg_fallback launch"))) return rc;
    return vanka_sweeps(box, ns, xcorr, vprev, fmid, sweeps, omega, 0, w, flag, s);
}

extern "C" int dnnmg_fallback_b(const dnnmg_box *box, const dnnmg_ns *ns, const float *xt, const float *b,
                                const double *norms, double theta, int sweeps, float omega, float *xcorr,
                                int *flag_out, void *ws, size_t ws_bytes, void *stream) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    if (!ns || !(ns->dt > 0.0)) return fail(DNNMG_ERR_ARG, "dnnmg_fallback_b: bad ns");
    if (!xt || !b || !norms || !xcorr || !ws) return fail(DNNMG_ERR_ARG, "dnnmg_fallback_b: NULL pointer");
    if (b == xcorr) return fail(DNNMG_ERR_ARG, "dnnmg_fallback_b: b and xcorr must not alias");
    if (sweeps < 0 || !(omega > 0.0f) || !(theta >= 0.0))
        return fail(DNNMG_ERR_ARG, "dnnmg_fallback_b: need sweeps >= 0, omega > 0, theta >= 0");
    if (ws_bytes < dnnmg_fallback_workspace(box))
        return fail(DNNMG_ERR_SHAPE, "dnnmg_fallback_b: workspace %zu < %zu bytes", ws_bytes,
                    dnnmg_fallback_workspace(box));
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    int *flag = (int *)(w + vanka_ws_bytes(m));
    k_indicator_flag<<<1, 64, 0, s>>>(norms, theta * theta, flag, flag_out);
    k_copy_pred<<<copy_grid(m), 256, 0, s>>>(4 * m.n_fine, xt, xcorr, flag);
    if ((rc = hip_check(hipGetLastError(), "dnnmg_fallback_b launch"))) return rc;
    return vanka_sweeps(box, ns, xcorr, nullptr, nullptr, sweeps, omega, 0, w, flag, s, b);
}

extern "C" size_t dnnmg_vanka_workspace(const dnnmg_box *box) {
    Mesh m;
    if (make_mesh(box, &m)) return 0;
    return vanka_ws_bytes(m);
}

extern "C" int dnnmg_vanka_sweeps(const dnnmg_box *box, const dnnmg_ns *ns, float *x, const float *vprev,
                                  const float *fmid, int sweeps, float omega, int coupled, void *ws,
                                  size_t ws_bytes, void *stream) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    if (!ns || !(ns->dt > 0.0)) return fail(DNNMG_ERR_ARG, "dnnmg_vanka_sweeps: bad ns");
    if (!x || !vprev || !ws) return fail(DNNMG_ERR_ARG, "dnnmg_vanka_sweeps: NULL pointer");
    if (sweeps < 0 || !(omega > 0.0f)) return fail(DNNMG_ERR_ARG, "dnnmg_vanka_sweeps: sweeps >= 0, omega > 0");
    if (ws_bytes < vanka_ws_bytes(m))
        return fail(DNNMG_ERR_SHAPE, "dnnmg_vanka_sweeps: workspace %zu < %zu bytes", ws_bytes, vanka_ws_bytes(m));
    return vanka_sweeps(box, ns, x, vprev, fmid, sweeps, omega, coupled, (char *)ws, nullptr,
                        (hipStream_t)stream);
}
