/*
 * DNN-MG fine-level correction: plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU path is checked against.  Only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product
 * path never calls it and shares no code, header or table with it.
 *
 * Everything is written from the method's definitions (arXiv 2307.14837):
 *   - Crank-Nicolson step of the stabilised Navier-Stokes system: Sec. 2.3,
 *     eq. (4cranknicholson3); stabilisation parameters eq. (stabparams);
 *     local projection stabilisation: Sec. 2.2, eq. (disc:ns).
 *   - DNN-MG time step: Sec. 4.1, Algorithm 1 (prolongation, fine residual,
 *     prediction, right-hand side, restriction).
 *   - Patches, dof map, local restriction Q, batch operator, extension L with
 *     the valence vector mu: Sec. 4.2, eqs. (Eq:DefR), (eq:defQ), (eq:defL).
 *   - Feed-forward network and AdamW: Sec. 3.
 * Readings where the paper is silent (Q1 elements, one patch per coarse cell,
 * two-level LPS projection onto the patch's coarse Q1 space, 2x2x2 Gauss
 * quadrature, tanh MLP with biases) are the project's documented readings.
 *
 * Conventions (shared by meaning, not by code, with the GPU library):
 *   box: n[3] coarse cells per axis; fine mesh = 2n cells per axis; len[3]
 *   physical lengths; periodic_mask bit a = axis a periodic; dirichlet_mask
 *   bit 2a = low face of axis a, bit 2a+1 = high face, carries Dirichlet
 *   velocity.  Nodes per axis: 2n (periodic) or 2n+1; index
 *   node = i + Nx*(j + Ny*k).  Fields are SoA [component][node].
 *
 * Nothing here is blocked, fused or reordered beyond the definitions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n[3];
    double len[3];
    uint32_t periodic_mask;
    uint32_t dirichlet_mask;
} or_box;

typedef struct {
    double nu, dt, alpha0, delta0;
} or_ns;

/* ---------------------------------------------------------------- mesh -- */

static int periodic(const or_box *b, int a) { return (b->periodic_mask >> a) & 1u; }

/* fine nodes along axis a */
static int64_t nf_axis(const or_box *b, int a) {
    return periodic(b, a) ? 2 * (int64_t)b->n[a] : 2 * (int64_t)b->n[a] + 1;
}
/* coarse nodes along axis a */
static int64_t nc_axis(const or_box *b, int a) {
    return periodic(b, a) ? (int64_t)b->n[a] : (int64_t)b->n[a] + 1;
}

int64_t or_fine_nodes(const or_box *b) { return nf_axis(b, 0) * nf_axis(b, 1) * nf_axis(b, 2); }
int64_t or_coarse_nodes(const or_box *b) { return nc_axis(b, 0) * nc_axis(b, 1) * nc_axis(b, 2); }
int64_t or_patches(const or_box *b) { return (int64_t)b->n[0] * b->n[1] * b->n[2]; }

/* global fine node of fine lattice coordinates (wrapping periodic axes) */
static int64_t fine_node(const or_box *b, int64_t i, int64_t j, int64_t k) {
    int64_t c[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) {
        int64_t N = nf_axis(b, a);
        if (periodic(b, a)) c[a] = ((c[a] % N) + N) % N;
    }
    return c[0] + nf_axis(b, 0) * (c[1] + nf_axis(b, 1) * c[2]);
}

static int64_t coarse_node(const or_box *b, int64_t I, int64_t J, int64_t K) {
    int64_t c[3] = {I, J, K};
    for (int a = 0; a < 3; ++a) {
        int64_t N = nc_axis(b, a);
        if (periodic(b, a)) c[a] = ((c[a] % N) + N) % N;
    }
    return c[0] + nc_axis(b, 0) * (c[1] + nc_axis(b, 1) * c[2]);
}

/* Is fine node (i,j,k) on a face that carries Dirichlet velocity data? */
static int is_dirichlet(const or_box *b, int64_t i, int64_t j, int64_t k) {
    int64_t c[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) {
        if (periodic(b, a)) continue;
        if (c[a] == 0 && ((b->dirichlet_mask >> (2 * a)) & 1u)) return 1;
        if (c[a] == nf_axis(b, a) - 1 && ((b->dirichlet_mask >> (2 * a + 1)) & 1u)) return 1;
    }
    return 0;
}

/* Dirichlet flag per fine node (1 = velocity prescribed). */
void or_dirichlet_flags(const or_box *b, uint8_t *flag) {
    for (int64_t k = 0; k < nf_axis(b, 2); ++k)
        for (int64_t j = 0; j < nf_axis(b, 1); ++j)
            for (int64_t i = 0; i < nf_axis(b, 0); ++i)
                flag[fine_node(b, i, j, k)] = (uint8_t)is_dirichlet(b, i, j, k);
}

/* --------------------------------------------------- patches (Sec. 4.2) -- */

/* dof(P_M, iota): patch M = coarse cell (I,J,K), M = I + nx(J + ny K);
 * local node iota = a + 3b + 9c, a,b,c in {0,1,2};  the global node is the
 * fine node (2I+a, 2J+b, 2K+c).  Valence = number of patches holding a node,
 * counted here by brute force over all patches. */
void or_dofmap(const or_box *b, int32_t *map, uint8_t *mult) {
    int64_t nf = or_fine_nodes(b);
    for (int64_t n = 0; n < nf; ++n) mult[n] = 0;
    for (int64_t K = 0; K < b->n[2]; ++K)
        for (int64_t J = 0; J < b->n[1]; ++J)
            for (int64_t I = 0; I < b->n[0]; ++I) {
                int64_t M = I + b->n[0] * (J + b->n[1] * K);
                for (int c = 0; c < 3; ++c)
                    for (int bb = 0; bb < 3; ++bb)
                        for (int a = 0; a < 3; ++a) {
                            int64_t g = fine_node(b, 2 * I + a, 2 * J + bb, 2 * K + c);
                            map[M * 27 + a + 3 * bb + 9 * c] = (int32_t)g;
                            mult[g] += 1;
                        }
            }
}

/* ------------------------------------ prolongation / restriction (Alg.1) -- */

/* 1-D Q1 prolongation weight from coarse node I to fine node i along axis a:
 * coincident nodes take weight 1, a fine midpoint takes 1/2 from each of the
 * two coarse ends (wrapping on periodic axes). */
static double w1d(const or_box *b, int a, int64_t i, int64_t I) {
    int64_t Nc = nc_axis(b, a);
    if (i % 2 == 0) return (i / 2) % Nc == I ? 1.0 : 0.0;
    int64_t lo = (i - 1) / 2, hi = (i + 1) / 2;
    if (periodic(b, a)) { lo %= Nc; hi %= Nc; }
    double w = 0.0;
    if (lo == I) w += 0.5;
    if (hi == I) w += 0.5;
    return w;
}

/* the (at most two) coarse nodes with nonzero weight for fine index i */
static int coarse_support(const or_box *b, int a, int64_t i, int64_t out[2]) {
    int64_t Nc = nc_axis(b, a);
    if (i % 2 == 0) { out[0] = (i / 2) % Nc; return 1; }
    out[0] = ((i - 1) / 2) % Nc;
    out[1] = ((i + 1) / 2) % Nc;
    return 2;
}

/* xf = P xc per component: the coarse Q1 function evaluated at fine nodes. */
void or_prolong(const or_box *b, int ncomp, const double *xc, double *xf) {
    int64_t ncn = or_coarse_nodes(b), nfn = or_fine_nodes(b);
    for (int comp = 0; comp < ncomp; ++comp)
        for (int64_t k = 0; k < nf_axis(b, 2); ++k)
            for (int64_t j = 0; j < nf_axis(b, 1); ++j)
                for (int64_t i = 0; i < nf_axis(b, 0); ++i) {
                    int64_t sI[2], sJ[2], sK[2];
                    int nI = coarse_support(b, 0, i, sI);
                    int nJ = coarse_support(b, 1, j, sJ);
                    int nK = coarse_support(b, 2, k, sK);
                    double s = 0.0;
                    for (int c = 0; c < nK; ++c)
                        for (int bb = 0; bb < nJ; ++bb)
                            for (int a = 0; a < nI; ++a) {
                                double w = w1d(b, 0, i, sI[a]) * w1d(b, 1, j, sJ[bb]) *
                                           w1d(b, 2, k, sK[c]);
                                s += w * xc[comp * ncn + coarse_node(b, sI[a], sJ[bb], sK[c])];
                            }
                    xf[comp * nfn + fine_node(b, i, j, k)] = s;
                }
}

/* bc = P^T bf per component (restriction of a dual vector). */
void or_restrict(const or_box *b, int ncomp, const double *bf, double *bc) {
    int64_t ncn = or_coarse_nodes(b), nfn = or_fine_nodes(b);
    for (int64_t t = 0; t < ncomp * ncn; ++t) bc[t] = 0.0;
    for (int comp = 0; comp < ncomp; ++comp)
        for (int64_t k = 0; k < nf_axis(b, 2); ++k)
            for (int64_t j = 0; j < nf_axis(b, 1); ++j)
                for (int64_t i = 0; i < nf_axis(b, 0); ++i) {
                    int64_t sI[2], sJ[2], sK[2];
                    int nI = coarse_support(b, 0, i, sI);
                    int nJ = coarse_support(b, 1, j, sJ);
                    int nK = coarse_support(b, 2, k, sK);
                    double v = bf[comp * nfn + fine_node(b, i, j, k)];
                    for (int c = 0; c < nK; ++c)
                        for (int bb = 0; bb < nJ; ++bb)
                            for (int a = 0; a < nI; ++a) {
                                double w = w1d(b, 0, i, sI[a]) * w1d(b, 1, j, sJ[bb]) *
                                           w1d(b, 2, k, sK[c]);
                                bc[comp * ncn + coarse_node(b, sI[a], sJ[bb], sK[c])] += w * v;
                            }
                }
}

/* ------------------------- Crank-Nicolson residual and RHS (Sec. 2.3) -- */

/* 1-D linear shape functions on [0,1] and their derivatives */
static double l1(int a, double t) { return a ? t : 1.0 - t; }
static double dl1(int a) { return a ? 1.0 : -1.0; }

/* Weak form contributions of one fine cell T of patch M.
 *
 * Momentum test function phi_i e_a, continuity test function xi_i:
 *   rhs part   (1/k)(vp_a, phi) - 1/2 (vp.grad vp_a, phi) - nu/2 (grad vp_a, grad phi)
 *              + (fmid_a, phi)
 *   minus LHS  (1/k)(v_a, phi) + 1/2 (v.grad v_a, phi) + nu/2 (grad v_a, grad phi)
 *              - (p, d_a phi) + delta_T (v.grad v_a - pi v.grad pi v_a,
 *                                         v.grad phi - pi v.grad pi phi)
 *   continuity -(div v, xi) - alpha_T (grad(p - pi p), grad(xi - pi xi))
 * where pi is interpolation onto the Q1 space of the coarse cell (patch).
 * Quadrature: 2x2x2 Gauss-Legendre on every fine cell.
 * mode 0: residual (uses vp and the LHS at (v, p)); mode 1: RHS of v only.
 */
static void cell_terms(const or_box *b, const or_ns *ns, int mode, int64_t ci, int64_t cj,
                       int64_t ck, const double *x, const double *vp, const double *fmid,
                       double *out) {
    const int64_t nfn = or_fine_nodes(b);
    double h[3], H[3];
    for (int a = 0; a < 3; ++a) {
        h[a] = b->len[a] / (2.0 * b->n[a]);
        H[a] = 2.0 * h[a];
    }
    const double vol = h[0] * h[1] * h[2];
    const double gp = 0.5 / sqrt(3.0);
    const double gq[2] = {0.5 - gp, 0.5 + gp};

    /* vertices of T: local j = a + 2b + 4c */
    int64_t vnode[8];
    for (int j = 0; j < 8; ++j)
        vnode[j] = fine_node(b, ci + (j & 1), cj + ((j >> 1) & 1), ck + ((j >> 2) & 1));
    /* corners of the patch (coarse cell) holding T: local c = A + 2B + 4C */
    int64_t PI = ci / 2, PJ = cj / 2, PK = ck / 2;
    int64_t cnode[8];
    for (int c = 0; c < 8; ++c)
        cnode[c] = fine_node(b, 2 * (PI + (c & 1)), 2 * (PJ + ((c >> 1) & 1)),
                             2 * (PK + ((c >> 2) & 1)));
    /* offset of T inside its patch, in fine cells */
    int off[3] = {(int)(ci - 2 * PI), (int)(cj - 2 * PJ), (int)(ck - 2 * PK)};

    /* stabilisation parameters eq. (stabparams): |v|_inf over the vertices */
    double alphaT = 0.0, deltaT = 0.0;
    if (mode == 0) {
        double vmax = 0.0;
        for (int j = 0; j < 8; ++j) {
            double s = 0.0;
            for (int a = 0; a < 3; ++a) s += x[a * nfn + vnode[j]] * x[a * nfn + vnode[j]];
            if (sqrt(s) > vmax) vmax = sqrt(s);
        }
        double hT = sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
        double den = ns->nu / (hT * hT) + vmax / hT + 1.0 / ns->dt;
        alphaT = ns->alpha0 / den;
        deltaT = ns->delta0 / den;
    }

    /* test slots: 0..7 = the vertices of T (phi part), 8..15 = the patch
     * corners (pi-phi part; nonzero only through the LPS terms) */
    for (int q = 0; q < 8; ++q) {
        double xi[3] = {gq[q & 1], gq[(q >> 1) & 1], gq[(q >> 2) & 1]};
        /* coarse local coordinate of the same point */
        double xc[3];
        for (int a = 0; a < 3; ++a) xc[a] = (off[a] + xi[a]) * 0.5;
        double wq = 0.125 * vol;

        double phi[8], dphi[8][3], Phi[8], dPhi[8][3];
        for (int j = 0; j < 8; ++j) {
            int aa[3] = {j & 1, (j >> 1) & 1, (j >> 2) & 1};
            phi[j] = l1(aa[0], xi[0]) * l1(aa[1], xi[1]) * l1(aa[2], xi[2]);
            dphi[j][0] = dl1(aa[0]) / h[0] * l1(aa[1], xi[1]) * l1(aa[2], xi[2]);
            dphi[j][1] = l1(aa[0], xi[0]) * dl1(aa[1]) / h[1] * l1(aa[2], xi[2]);
            dphi[j][2] = l1(aa[0], xi[0]) * l1(aa[1], xi[1]) * dl1(aa[2]) / h[2];
            Phi[j] = l1(aa[0], xc[0]) * l1(aa[1], xc[1]) * l1(aa[2], xc[2]);
            dPhi[j][0] = dl1(aa[0]) / H[0] * l1(aa[1], xc[1]) * l1(aa[2], xc[2]);
            dPhi[j][1] = l1(aa[0], xc[0]) * dl1(aa[1]) / H[1] * l1(aa[2], xc[2]);
            dPhi[j][2] = l1(aa[0], xc[0]) * l1(aa[1], xc[1]) * dl1(aa[2]) / H[2];
        }

        /* field values and gradients at the point */
        double v[3] = {0, 0, 0}, gv[3][3] = {{0}}, pv = 0, gpv[3] = {0, 0, 0};
        double w[3] = {0, 0, 0}, gw[3][3] = {{0}}; /* vp (residual) or v (rhs) */
        double f[3] = {0, 0, 0};
        double gpiv[3][3] = {{0}}, pip = 0, gpip[3] = {0, 0, 0};
        for (int j = 0; j < 8; ++j) {
            int64_t g = vnode[j];
            for (int a = 0; a < 3; ++a) {
                double va = x[a * nfn + g];
                double wa = (mode == 0) ? vp[a * nfn + g] : x[a * nfn + g];
                v[a] += va * phi[j];
                w[a] += wa * phi[j];
                if (fmid) f[a] += fmid[a * nfn + g] * phi[j];
                for (int d = 0; d < 3; ++d) {
                    gv[a][d] += va * dphi[j][d];
                    gw[a][d] += wa * dphi[j][d];
                }
            }
            if (mode == 0) {
                double pj = x[3 * nfn + g];
                pv += pj * phi[j];
                for (int d = 0; d < 3; ++d) gpv[d] += pj * dphi[j][d];
            }
        }
        double piv[3] = {0, 0, 0};
        if (mode == 0) {
            for (int c = 0; c < 8; ++c) {
                int64_t g = cnode[c];
                for (int a = 0; a < 3; ++a) {
                    double va = x[a * nfn + g];
                    piv[a] += va * Phi[c];
                    for (int d = 0; d < 3; ++d) gpiv[a][d] += va * dPhi[c][d];
                }
                double pc = x[3 * nfn + g];
                pip += pc * Phi[c];
                for (int d = 0; d < 3; ++d) gpip[d] += pc * dPhi[c][d];
            }
        }
        (void)pip;

        double convw[3], convv[3], R[3];
        for (int a = 0; a < 3; ++a) {
            convw[a] = 0.0;
            convv[a] = 0.0;
            double cpi = 0.0;
            for (int d = 0; d < 3; ++d) {
                convw[a] += w[d] * gw[a][d];
                convv[a] += v[d] * gv[a][d];
                cpi += piv[d] * gpiv[a][d];
            }
            R[a] = convv[a] - cpi;
        }
        double divv = gv[0][0] + gv[1][1] + gv[2][2];

        for (int t = 0; t < 16; ++t) {
            double phi_i = 0.0, dphi_i[3] = {0, 0, 0}, dPhi_i[3] = {0, 0, 0};
            if (t < 8) {
                phi_i = phi[t];
                for (int d = 0; d < 3; ++d) dphi_i[d] = dphi[t][d];
            } else {
                if (mode != 0) continue; /* corners only enter through LPS */
                for (int d = 0; d < 3; ++d) dPhi_i[d] = dPhi[t - 8][d];
            }
            /* a test node that is both a vertex of T and a patch corner gets
             * its phi part from slot t<8 and its pi-phi part from slot t>=8 */
            double *o = out + 4 * t;
            if (mode == 0) {
                double sv = 0.0, spi = 0.0;
                for (int d = 0; d < 3; ++d) {
                    sv += v[d] * dphi_i[d];
                    spi += piv[d] * dPhi_i[d];
                }
                double stream_test = sv - spi;
                for (int a = 0; a < 3; ++a) {
                    double vis = 0.0;
                    for (int d = 0; d < 3; ++d) vis += (gw[a][d] + gv[a][d]) * dphi_i[d];
                    double val = (1.0 / ns->dt) * (w[a] - v[a]) * phi_i -
                                 0.5 * (convw[a] + convv[a]) * phi_i - 0.5 * ns->nu * vis +
                                 pv * dphi_i[a] + f[a] * phi_i - deltaT * R[a] * stream_test;
                    o[a] += wq * val;
                }
                double lps = 0.0;
                for (int d = 0; d < 3; ++d) lps += (gpv[d] - gpip[d]) * (dphi_i[d] - dPhi_i[d]);
                o[3] += wq * (-divv * phi_i - alphaT * lps);
            } else {
                for (int a = 0; a < 3; ++a) {
                    double vis = 0.0;
                    for (int d = 0; d < 3; ++d) vis += gw[a][d] * dphi_i[d];
                    double val = (1.0 / ns->dt) * w[a] * phi_i - 0.5 * convw[a] * phi_i -
                                 0.5 * ns->nu * vis + f[a] * phi_i;
                    o[a] += wq * val;
                }
            }
        }
    }
}

static void assemble(const or_box *b, const or_ns *ns, int mode, const double *x,
                     const double *vp, const double *fmid, double *r) {
    const int64_t nfn = or_fine_nodes(b);
    for (int64_t t = 0; t < 4 * nfn; ++t) r[t] = 0.0;
    for (int64_t ck = 0; ck < 2 * (int64_t)b->n[2]; ++ck)
        for (int64_t cj = 0; cj < 2 * (int64_t)b->n[1]; ++cj)
            for (int64_t ci = 0; ci < 2 * (int64_t)b->n[0]; ++ci) {
                double out[64];
                memset(out, 0, sizeof out);
                cell_terms(b, ns, mode, ci, cj, ck, x, vp, fmid, out);
                for (int t = 0; t < 16; ++t) {
                    int64_t g;
                    if (t < 8)
                        g = fine_node(b, ci + (t & 1), cj + ((t >> 1) & 1), ck + ((t >> 2) & 1));
                    else {
                        int c = t - 8;
                        g = fine_node(b, 2 * (ci / 2 + (c & 1)), 2 * (cj / 2 + ((c >> 1) & 1)),
                                      2 * (ck / 2 + ((c >> 2) & 1)));
                    }
                    for (int a = 0; a < 4; ++a) r[a * nfn + g] += out[4 * t + a];
                }
            }
    /* Dirichlet velocity rows carry no equation */
    for (int64_t k = 0; k < nf_axis(b, 2); ++k)
        for (int64_t j = 0; j < nf_axis(b, 1); ++j)
            for (int64_t i = 0; i < nf_axis(b, 0); ++i)
                if (is_dirichlet(b, i, j, k)) {
                    int64_t g = fine_node(b, i, j, k);
                    for (int a = 0; a < 3; ++a) r[a * nfn + g] = 0.0;
                }
}

/* r = F - A(x): fine residual of Alg. 1 (line "Residual on level L+J") for the
 * Crank-Nicolson system (4cranknicholson3) with F built from the previous
 * velocity vp and fmid = (f_{n-1} + f_n)/2 (NULL = no forcing).
 * x = (u, v, w, p) [4][N_f]; vp [3][N_f]; r [4][N_f]. */
void or_residual(const or_box *b, const or_ns *ns, const double *x, const double *vp,
                 const double *fmid, double *r) {
    assemble(b, ns, 0, x, vp, fmid, r);
}

/* b = Rhs(v): right-hand side of (4cranknicholson3) for the next step, built
 * from velocity v [3][N_f] and fmid = (f_n + f_{n+1})/2; pressure rows 0. */
void or_rhs(const or_box *b, const or_ns *ns, const double *v, const double *fmid,
            double *out) {
    const int64_t nfn = or_fine_nodes(b);
    double *x = (double *)malloc(sizeof(double) * 4 * nfn);
    for (int64_t t = 0; t < 3 * nfn; ++t) x[t] = v[t];
    for (int64_t t = 0; t < nfn; ++t) x[3 * nfn + t] = 0.0;
    assemble(b, ns, 1, x, NULL, fmid, out);
    for (int64_t t = 0; t < nfn; ++t) out[3 * nfn + t] = 0.0;
    free(x);
}

/* ------------------------------------------ gather / scatter (Sec. 4.2) -- */

/* Q applied to (v~, r) plus the coarse cell sizes, then the per-feature
 * affine standardisation z = (X - shift) * inv_scale (NULL = identity).
 * Row M: [u(dof(M,0..26)), v(..), w(..), r_u(..), r_v(..), r_w(..), Hx, Hy, Hz]. */
void or_gather(const or_box *b, const double *x, const double *r, const double *shift,
               const double *inv_scale, double *X) {
    const int64_t nfn = or_fine_nodes(b), np = or_patches(b);
    int32_t *map = (int32_t *)malloc(sizeof(int32_t) * 27 * np);
    uint8_t *mult = (uint8_t *)malloc(nfn);
    or_dofmap(b, map, mult);
    for (int64_t M = 0; M < np; ++M) {
        double *row = X + M * 165;
        for (int c = 0; c < 3; ++c)
            for (int i = 0; i < 27; ++i) {
                row[27 * c + i] = x[c * nfn + map[M * 27 + i]];
                row[81 + 27 * c + i] = r[c * nfn + map[M * 27 + i]];
            }
        for (int a = 0; a < 3; ++a) row[162 + a] = b->len[a] / b->n[a];
        for (int f = 0; f < 165; ++f) {
            double s = shift ? shift[f] : 0.0, g = inv_scale ? inv_scale[f] : 1.0;
            row[f] = (row[f] - s) * g;
        }
    }
    free(map);
    free(mult);
}

/* L of eq. (defL): d = mu (.) sum_M L(Y[M], P_M), mu = 1 / valence; the
 * network's 81 outputs per patch are the velocity components c*27 + iota.
 * Dirichlet velocity nodes receive no correction. d [3][N_f]. */
void or_scatter(const or_box *b, const double *Y, double *d) {
    const int64_t nfn = or_fine_nodes(b), np = or_patches(b);
    int32_t *map = (int32_t *)malloc(sizeof(int32_t) * 27 * np);
    uint8_t *mult = (uint8_t *)malloc(nfn);
    uint8_t *dir = (uint8_t *)malloc(nfn);
    or_dofmap(b, map, mult);
    or_dirichlet_flags(b, dir);
    for (int64_t t = 0; t < 3 * nfn; ++t) d[t] = 0.0;
    for (int64_t M = 0; M < np; ++M)
        for (int c = 0; c < 3; ++c)
            for (int i = 0; i < 27; ++i) d[c * nfn + map[M * 27 + i]] += Y[M * 81 + 27 * c + i];
    for (int64_t n = 0; n < nfn; ++n)
        for (int c = 0; c < 3; ++c) d[c * nfn + n] = dir[n] ? 0.0 : d[c * nfn + n] / mult[n];
    free(map);
    free(mult);
    free(dir);
}

/* ---------------------- patches of the two-level prediction (Sec. 4.2) -- */

/* Prediction J levels above the coarse mesh of b (J = 1 or 2): the fine
 * lattice is that of the box bJ with n * 2^(J-1) cells per axis (its own
 * fine mesh has n * 2^J cells); patch M = cell (I,J,K) of b covers P^3 fine
 * cells, P = 2^J, and its (P+1)^3 local nodes iota = a + (P+1) b + (P+1)^2 c,
 * a,b,c in 0..P, are the fine nodes (P I + a, P J + b, P K + c) of bJ.
 * J = 1 is the single-level patch of or_dofmap. */
static or_box level_box(const or_box *b, int J) {
    or_box c = *b;
    for (int a = 0; a < 3; ++a) c.n[a] = b->n[a] << (J - 1);
    return c;
}

/* dof map [np][(P+1)^3] and valence (counted over all patches). */
void or_dofmap_levels(const or_box *b, int J, int32_t *map, uint8_t *mult) {
    const int P = 1 << J, S = P + 1, NL = S * S * S;
    const or_box f = level_box(b, J);
    const int64_t nf = or_fine_nodes(&f);
    for (int64_t n = 0; n < nf; ++n) mult[n] = 0;
    for (int64_t K = 0; K < b->n[2]; ++K)
        for (int64_t Jj = 0; Jj < b->n[1]; ++Jj)
            for (int64_t I = 0; I < b->n[0]; ++I) {
                int64_t M = I + b->n[0] * (Jj + b->n[1] * K);
                for (int c = 0; c < S; ++c)
                    for (int bb = 0; bb < S; ++bb)
                        for (int a = 0; a < S; ++a) {
                            int64_t g = fine_node(&f, P * I + a, P * Jj + bb, P * K + c);
                            map[M * NL + a + S * bb + S * S * c] = (int32_t)g;
                            mult[g] += 1;
                        }
            }
}

/* Q of eq. (defQ) on the patches of the J-level prediction: row M =
 * [u(nodes), v(..), w(..), r_u(..), r_v(..), r_w(..), H0, H1, H2] with the
 * coarse cell sizes H of b, then z = (X - shift) * inv_scale.
 * x, r on the fine lattice of level_box(b, J); X [np][6 (P+1)^3 + 3]. */
void or_gather_levels(const or_box *b, int J, const double *x, const double *r, const double *shift,
                      const double *inv_scale, double *X) {
    const int P = 1 << J, S = P + 1, NL = S * S * S, NC = 6 * NL + 3;
    const or_box f = level_box(b, J);
    const int64_t nfn = or_fine_nodes(&f), np = or_patches(b);
    int32_t *map = (int32_t *)malloc(sizeof(int32_t) * NL * np);
    uint8_t *mult = (uint8_t *)malloc(nfn);
    or_dofmap_levels(b, J, map, mult);
    for (int64_t M = 0; M < np; ++M) {
        double *row = X + M * NC;
        for (int c = 0; c < 3; ++c)
            for (int i = 0; i < NL; ++i) {
                row[NL * c + i] = x[c * nfn + map[M * NL + i]];
                row[3 * NL + NL * c + i] = r[c * nfn + map[M * NL + i]];
            }
        for (int a = 0; a < 3; ++a) row[6 * NL + a] = b->len[a] / b->n[a];
        for (int q = 0; q < NC; ++q) {
            double sh = shift ? shift[q] : 0.0, g = inv_scale ? inv_scale[q] : 1.0;
            row[q] = (row[q] - sh) * g;
        }
    }
    free(map);
    free(mult);
}

/* L of eq. (defL) on the patches of the J-level prediction: Y [np][3 (P+1)^3]
 * (component-major per patch) averaged by valence into d [3][N_f] on the
 * fine lattice of level_box(b, J); Dirichlet velocity nodes get 0. */
void or_scatter_levels(const or_box *b, int J, const double *Y, double *d) {
    const int P = 1 << J, S = P + 1, NL = S * S * S;
    const or_box f = level_box(b, J);
    const int64_t nfn = or_fine_nodes(&f), np = or_patches(b);
    int32_t *map = (int32_t *)malloc(sizeof(int32_t) * NL * np);
    uint8_t *mult = (uint8_t *)malloc(nfn);
    uint8_t *dir = (uint8_t *)malloc(nfn);
    or_dofmap_levels(b, J, map, mult);
    or_dirichlet_flags(&f, dir);
    for (int64_t t = 0; t < 3 * nfn; ++t) d[t] = 0.0;
    for (int64_t M = 0; M < np; ++M)
        for (int c = 0; c < 3; ++c)
            for (int i = 0; i < NL; ++i) d[c * nfn + map[M * NL + i]] += Y[M * 3 * NL + NL * c + i];
    for (int64_t n = 0; n < nfn; ++n)
        for (int c = 0; c < 3; ++c) d[c * nfn + n] = dir[n] ? 0.0 : d[c * nfn + n] / mult[n];
    free(map);
    free(mult);
    free(dir);
}

/* ------------------------------------------------ network (Sec. 3) ------ */

/* Y = W3^T tanh(W2^T tanh(W1^T x + b1) + b2) + b3 for every row x of X.
 * W_l is [fan_in][fan_out] row-major; A1, A2 (optional) receive the hidden
 * activations [n][H]. */
void or_mlp_forward(int64_t n, int nin, int H, int nout, const double *X, const double *W1,
                    const double *b1, const double *W2, const double *b2, const double *W3,
                    const double *b3, double *Y, double *A1, double *A2) {
    double *a1 = (double *)malloc(sizeof(double) * H), *a2 = (double *)malloc(sizeof(double) * H);
    for (int64_t m = 0; m < n; ++m) {
        for (int j = 0; j < H; ++j) {
            double s = b1 ? b1[j] : 0.0;
            for (int k = 0; k < nin; ++k) s += X[m * nin + k] * W1[(int64_t)k * H + j];
            a1[j] = tanh(s);
        }
        for (int j = 0; j < H; ++j) {
            double s = b2 ? b2[j] : 0.0;
            for (int k = 0; k < H; ++k) s += a1[k] * W2[(int64_t)k * H + j];
            a2[j] = tanh(s);
        }
        for (int j = 0; j < nout; ++j) {
            double s = b3 ? b3[j] : 0.0;
            for (int k = 0; k < H; ++k) s += a2[k] * W3[(int64_t)k * nout + j];
            Y[m * nout + j] = s;
        }
        if (A1) memcpy(A1 + m * H, a1, sizeof(double) * H);
        if (A2) memcpy(A2 + m * H, a2, sizeof(double) * H);
    }
    free(a1);
    free(a2);
}

/* Gradients of sum over rows of <dY, Y> with respect to W_l, b_l, by the
 * chain rule through the two tanh layers (d tanh = 1 - tanh^2).  Input
 * gradient is not formed.  Gradients are overwritten. */
void or_mlp_backward(int64_t n, int nin, int H, int nout, const double *X, const double *W2,
                     const double *W3, const double *A1, const double *A2, const double *dY,
                     double *dW1, double *db1, double *dW2, double *db2, double *dW3,
                     double *db3) {
    memset(dW1, 0, sizeof(double) * nin * H);
    memset(dW2, 0, sizeof(double) * H * H);
    memset(dW3, 0, sizeof(double) * H * nout);
    memset(db1, 0, sizeof(double) * H);
    memset(db2, 0, sizeof(double) * H);
    memset(db3, 0, sizeof(double) * nout);
    double *dz2 = (double *)malloc(sizeof(double) * H), *dz1 = (double *)malloc(sizeof(double) * H);
    for (int64_t m = 0; m < n; ++m) {
        const double *x = X + m * nin, *a1 = A1 + m * H, *a2 = A2 + m * H, *dy = dY + m * nout;
        for (int k = 0; k < H; ++k)
            for (int j = 0; j < nout; ++j) dW3[(int64_t)k * nout + j] += a2[k] * dy[j];
        for (int j = 0; j < nout; ++j) db3[j] += dy[j];
        for (int k = 0; k < H; ++k) {
            double s = 0.0;
            for (int j = 0; j < nout; ++j) s += dy[j] * W3[(int64_t)k * nout + j];
            dz2[k] = s * (1.0 - a2[k] * a2[k]);
        }
        for (int k = 0; k < H; ++k)
            for (int j = 0; j < H; ++j) dW2[(int64_t)k * H + j] += a1[k] * dz2[j];
        for (int j = 0; j < H; ++j) db2[j] += dz2[j];
        for (int k = 0; k < H; ++k) {
            double s = 0.0;
            for (int j = 0; j < H; ++j) s += dz2[j] * W2[(int64_t)k * H + j];
            dz1[k] = s * (1.0 - a1[k] * a1[k]);
        }
        for (int k = 0; k < nin; ++k)
            for (int j = 0; j < H; ++j) dW1[(int64_t)k * H + j] += x[k] * dz1[j];
        for (int j = 0; j < H; ++j) db1[j] += dz1[j];
    }
    free(dz2);
    free(dz1);
}

/* Patch loss of the training objective: (1/n) sum_M ||Y_M - T_M||^2, and its
 * gradient dY = 2 (Y - T) / n. Returns the loss. */
double or_mse(int64_t n, int nout, const double *Y, const double *T, double *dY) {
    double s = 0.0;
    for (int64_t t = 0; t < n * nout; ++t) {
        double e = Y[t] - T[t];
        s += e * e;
        if (dY) dY[t] = 2.0 * e / (double)n;
    }
    return s / (double)n;
}

/* AdamW (decoupled weight decay), step t >= 1:
 *   m <- b1 m + (1-b1) g ; v <- b2 v + (1-b2) g^2
 *   theta <- theta - lr wd theta - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps) */
void or_adamw(int64_t n, double *theta, double *m, double *v, const double *g, double lr,
              double b1, double b2, double eps, double wd, int64_t t) {
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        theta[i] = theta[i] - lr * wd * theta[i] - lr * mh / (sqrt(vh) + eps);
    }
}

/* Euclidean norm squared of a (or of a - b when b is given). */
double or_norm2(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double e = b ? a[i] - b[i] : a[i];
        s += e * e;
    }
    return s;
}

/* -------------------------------------- low-precision number formats ---- */

/* Round to the nearest bfloat16 value (8 exponent bits, 7 stored mantissa
 * bits), ties to even; overflow goes to infinity as in IEEE rounding. */
double or_round_bf16(double x) {
    if (x != x || x == 0.0 || isinf(x)) return x;
    int e;
    frexp(x, &e);                  /* |x| = m 2^e, 0.5 <= m < 1 */
    int lead = e - 1;              /* exponent of the leading bit */
    if (lead < -126) lead = -126;  /* subnormals share the spacing of 2^-126 */
    double q = ldexp(1.0, lead - 7); /* 8 significant bits */
    double r = nearbyint(x / q) * q; /* default rounding mode: ties to even */
    if (fabs(r) >= ldexp(1.0, 128)) return x > 0 ? INFINITY : -INFINITY;
    return r;
}

/* Round to the nearest OCP FP8 E4M3FN value (4 exponent bits, bias 7, 3
 * mantissa bits, max finite 448, no infinities), ties to even, saturating
 * at +-448. */
double or_round_e4m3(double x) {
    if (x != x) return x;
    if (x == 0.0) return x;
    double ax = fabs(x);
    int e;
    frexp(ax, &e);       /* ax = m 2^e, 0.5 <= m < 1: leading bit 2^(e-1) */
    int lead = e - 1;    /* exponent of the leading bit */
    if (lead < -6) lead = -6; /* subnormals share the spacing of 2^-6 */
    double q = ldexp(1.0, lead - 3);
    double r = nearbyint(ax / q) * q;
    if (r > 448.0) r = 448.0;
    return x < 0 ? -r : r;
}

/* ------------------------------- plain fine-level correction (patch Vanka) */

/* Shape functions of patch-local node (a,b,c) in {0,1,2}^3 on the fine cell
 * with offset (ox,oy,oz) in the patch, at the cell-local point xi: value and
 * gradient (zero if the node is not a vertex of the cell). */
static void fine_shape(const double h[3], int a, int b, int c, int ox, int oy, int oz,
                       const double xi[3], double *phi, double dphi[3]) {
    int la = a - ox, lb = b - oy, lc = c - oz;
    if (la < 0 || la > 1 || lb < 0 || lb > 1 || lc < 0 || lc > 1) {
        *phi = 0.0;
        dphi[0] = dphi[1] = dphi[2] = 0.0;
        return;
    }
    *phi = l1(la, xi[0]) * l1(lb, xi[1]) * l1(lc, xi[2]);
    dphi[0] = dl1(la) / h[0] * l1(lb, xi[1]) * l1(lc, xi[2]);
    dphi[1] = l1(la, xi[0]) * dl1(lb) / h[1] * l1(lc, xi[2]);
    dphi[2] = l1(la, xi[0]) * l1(lb, xi[1]) * dl1(lc) / h[2];
}

/* Coarse (patch) shape function of a corner node, zero for other nodes. */
static void coarse_shape(const double H[3], int a, int b, int c, const double xc[3],
                         double *Phi, double dPhi[3]) {
    if ((a & 1) || (b & 1) || (c & 1)) {
        *Phi = 0.0;
        dPhi[0] = dPhi[1] = dPhi[2] = 0.0;
        return;
    }
    int A = a / 2, B = b / 2, C = c / 2;
    *Phi = l1(A, xc[0]) * l1(B, xc[1]) * l1(C, xc[2]);
    dPhi[0] = dl1(A) / H[0] * l1(B, xc[1]) * l1(C, xc[2]);
    dPhi[1] = l1(A, xc[0]) * dl1(B) / H[1] * l1(C, xc[2]);
    dPhi[2] = l1(A, xc[0]) * l1(B, xc[1]) * dl1(C) / H[2];
}

/* Local matrix of the plain fine-level correction on patch M (the Vanka
 * local problem of Sec. 2.4 on the patch's 27 nodes): the rows and columns of
 * the patch's 108 unknowns [u(27) v(27) w(27) p(27)] (local node iota =
 * a + 3b + 9c) taken from the Crank-Nicolson operator linearised at the
 * velocity w with frozen convection (Picard).  Galerkin terms come from every
 * fine cell that has a patch node as a vertex (the 4x4x4 cell block around
 * the patch), so each row is the full operator row restricted to the patch:
 *   velocity-velocity (per component): (1/k)(phi_j, phi_i)
 *        + 1/2 (w.grad phi_j, phi_i) + nu/2 (grad phi_j, grad phi_i)
 *   velocity row (a,i), pressure column j: -(phi_j, d_a phi_i)
 *   pressure row i, velocity column (a,j): (d_a phi_j, phi_i)
 * The pressure stabilisation alpha_T (grad(phi_j - pi phi_j), grad(phi_i -
 * pi phi_i)) is taken over the patch's own cells (pi = interpolation onto
 * the patch's Q1 space), the convection stabilisation is left out.  Velocity
 * dofs on Dirichlet faces get identity rows and columns.  A is row-major
 * 108 x 108, row = test function, column = trial function. */
void or_vanka_matrix(const or_box *bx, const or_ns *ns, const double *w, int64_t M, double *A) {
    const int64_t nfn = or_fine_nodes(bx);
    double h[3], H[3];
    for (int a = 0; a < 3; ++a) {
        h[a] = bx->len[a] / (2.0 * bx->n[a]);
        H[a] = 2.0 * h[a];
    }
    const double vol = h[0] * h[1] * h[2];
    const double gp = 0.5 / sqrt(3.0);
    const double gq[2] = {0.5 - gp, 0.5 + gp};
    const double hT = sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
    int64_t I = M % bx->n[0], J = (M / bx->n[0]) % bx->n[1], K = M / ((int64_t)bx->n[0] * bx->n[1]);
    int dir[27];
    for (int t = 0; t < 27; ++t)
        dir[t] = is_dirichlet(bx, 2 * I + t % 3, 2 * J + (t / 3) % 3, 2 * K + t / 9);
    for (int t = 0; t < 108 * 108; ++t) A[t] = 0.0;
    /* cells with patch-local origin o in {-1,0,1,2}^3 */
    for (int cz = -1; cz <= 2; ++cz)
        for (int cy = -1; cy <= 2; ++cy)
            for (int cx = -1; cx <= 2; ++cx) {
                int64_t g0[3] = {2 * I + cx, 2 * J + cy, 2 * K + cz};
                int exists = 1;
                for (int a = 0; a < 3; ++a)
                    if (!periodic(bx, a) && (g0[a] < 0 || g0[a] >= 2 * (int64_t)bx->n[a])) exists = 0;
                if (!exists) continue;
                const int own = cx >= 0 && cx <= 1 && cy >= 0 && cy <= 1 && cz >= 0 && cz <= 1;
                /* velocity at the cell's vertices and its stabilisation parameter */
                double wv8[3][8], vmax = 0.0;
                for (int v = 0; v < 8; ++v) {
                    int64_t g = fine_node(bx, g0[0] + (v & 1), g0[1] + ((v >> 1) & 1), g0[2] + (v >> 2));
                    double s2 = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        wv8[d][v] = w[d * nfn + g];
                        s2 += wv8[d][v] * wv8[d][v];
                    }
                    if (sqrt(s2) > vmax) vmax = sqrt(s2);
                }
                double alphaT = ns->alpha0 / (ns->nu / (hT * hT) + vmax / hT + 1.0 / ns->dt);
                for (int q = 0; q < 8; ++q) {
                    double xi[3] = {gq[q & 1], gq[(q >> 1) & 1], gq[(q >> 2) & 1]};
                    double xc[3] = {(cx + xi[0]) * 0.5, (cy + xi[1]) * 0.5, (cz + xi[2]) * 0.5};
                    double wq = 0.125 * vol;
                    double phi[27], dphi[27][3], Phi[27], dPhi[27][3];
                    for (int t = 0; t < 27; ++t) {
                        int a = t % 3, b = (t / 3) % 3, c = t / 9;
                        fine_shape(h, a, b, c, cx, cy, cz, xi, &phi[t], dphi[t]);
                        if (own) coarse_shape(H, a, b, c, xc, &Phi[t], dPhi[t]);
                    }
                    double wv[3] = {0, 0, 0};
                    for (int v = 0; v < 8; ++v) {
                        double pv = l1(v & 1, xi[0]) * l1((v >> 1) & 1, xi[1]) * l1(v >> 2, xi[2]);
                        for (int d = 0; d < 3; ++d) wv[d] += wv8[d][v] * pv;
                    }
                    for (int i = 0; i < 27; ++i)
                        for (int j = 0; j < 27; ++j) {
                            double conv = wv[0] * dphi[j][0] + wv[1] * dphi[j][1] + wv[2] * dphi[j][2];
                            double kin = (1.0 / ns->dt) * phi[j] * phi[i] + 0.5 * conv * phi[i] +
                                         0.5 * ns->nu *
                                             (dphi[j][0] * dphi[i][0] + dphi[j][1] * dphi[i][1] +
                                              dphi[j][2] * dphi[i][2]);
                            for (int a = 0; a < 3; ++a) {
                                A[(27 * a + i) * 108 + 27 * a + j] += wq * kin;
                                A[(27 * a + i) * 108 + 81 + j] += wq * (-phi[j] * dphi[i][a]);
                                A[(81 + i) * 108 + 27 * a + j] += wq * (dphi[j][a] * phi[i]);
                            }
                            if (own) {
                                double lps = 0.0;
                                for (int d = 0; d < 3; ++d)
                                    lps += (dphi[j][d] - dPhi[j][d]) * (dphi[i][d] - dPhi[i][d]);
                                A[(81 + i) * 108 + 81 + j] += wq * alphaT * lps;
                            }
                        }
                }
            }
    for (int t = 0; t < 27; ++t) {
        if (!dir[t]) continue;
        for (int a = 0; a < 3; ++a) {
            int r = 27 * a + t;
            for (int c = 0; c < 108; ++c) {
                A[r * 108 + c] = 0.0;
                A[c * 108 + r] = 0.0;
            }
            A[r * 108 + r] = 1.0;
        }
    }
}

/* Solve A x = b (n x n, row-major, overwritten) by Gaussian elimination with
 * partial pivoting; b is overwritten by x.  Returns 0, or -1 if singular. */
int or_dense_solve(int n, double *A, double *b) {
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > fabs(A[p * n + k])) p = i;
        if (A[p * n + k] == 0.0) return -1;
        if (p != k) {
            for (int c = 0; c < n; ++c) {
                double t = A[k * n + c];
                A[k * n + c] = A[p * n + c];
                A[p * n + c] = t;
            }
            double t = b[k];
            b[k] = b[p];
            b[p] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            double f = A[i * n + k] / A[k * n + k];
            if (f == 0.0) continue;
            for (int c = k; c < n; ++c) A[i * n + c] -= f * A[k * n + c];
            b[i] -= f * b[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double s = b[k];
        for (int c = k + 1; c < n; ++c) s -= A[k * n + c] * b[c];
        b[k] = s / A[k * n + k];
    }
    return 0;
}

/* One sweep of the plain fine-level correction, additive over patches with
 * the averaging of the extension operator L, eq. (defL): r = residual(x);
 * on every patch solve a local problem with the local matrix at the current
 * velocity; x_out = x + omega * mu (.) sum_P L(delta_P), Dirichlet
 * velocities unchanged.
 *   coupled = 1: the full 108 x 108 velocity-pressure system A_P delta_P = r_P
 *                (all four fields corrected);
 *   coupled = 0: the momentum equations with the pressure held at its
 *                current value: K_P delta_a = r_a for each velocity component
 *                (K_P = velocity block of A_P); the pressure is not changed,
 *                as the network's correction leaves it to the coarse level.
 * Returns 0 or -1. */
int or_vanka_sweep(const or_box *bx, const or_ns *ns, const double *x, const double *vp,
                   const double *fmid, double omega, int coupled, double *xout) {
    const int64_t nfn = or_fine_nodes(bx), np = or_patches(bx);
    double *r = (double *)malloc(sizeof(double) * 4 * nfn);
    double *d = (double *)calloc(4 * nfn, sizeof(double));
    double *A = (double *)malloc(sizeof(double) * 108 * 108);
    int32_t *map = (int32_t *)malloc(sizeof(int32_t) * 27 * np);
    uint8_t *mult = (uint8_t *)malloc(nfn);
    uint8_t *dir = (uint8_t *)malloc(nfn);
    int rc = 0;
    or_residual(bx, ns, x, vp, fmid, r);
    or_dofmap(bx, map, mult);
    or_dirichlet_flags(bx, dir);
    for (int64_t M = 0; M < np && rc == 0; ++M) {
        double rhs[108];
        or_vanka_matrix(bx, ns, x, M, A);
        for (int f = 0; f < 4; ++f)
            for (int t = 0; t < 27; ++t) rhs[27 * f + t] = r[f * nfn + map[M * 27 + t]];
        if (coupled) {
            if (or_dense_solve(108, A, rhs)) rc = -1;
        } else {
            double Kb[27 * 27], tmp[27];
            for (int a = 0; a < 3; ++a) {
                for (int i = 0; i < 27; ++i)
                    for (int j = 0; j < 27; ++j) Kb[i * 27 + j] = A[i * 108 + j];
                for (int i = 0; i < 27; ++i) tmp[i] = rhs[27 * a + i];
                if (or_dense_solve(27, Kb, tmp)) rc = -1;
                for (int i = 0; i < 27; ++i) rhs[27 * a + i] = tmp[i];
            }
            for (int i = 0; i < 27; ++i) rhs[81 + i] = 0.0;
        }
        for (int f = 0; f < 4; ++f)
            for (int t = 0; t < 27; ++t) d[f * nfn + map[M * 27 + t]] += rhs[27 * f + t];
    }
    for (int64_t n = 0; n < nfn; ++n)
        for (int f = 0; f < 4; ++f) {
            double v = d[f * nfn + n] / mult[n];
            if (f < 3 && dir[n]) v = 0.0;
            xout[f * nfn + n] = x[f * nfn + n] + omega * v;
        }
    free(r);
    free(d);
    free(A);
    free(map);
    free(mult);
    free(dir);
    return rc;
}
