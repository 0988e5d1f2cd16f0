/*
 * DNN-MG fine level with the paper's Q2/Q2 elements on isoparametric
 * hexahedra: plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU path is checked against.  Only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product
 * path never calls it and shares no code, header or table with it.
 *
 * Written from the method's definitions (arXiv 2307.14837):
 *   - equal-order continuous Q2 elements for velocity and pressure on
 *     hexahedral meshes, local projection stabilisation with pi_h the
 *     interpolation Q2 -> Q1: Sec. 2.2, eq. (disc:ns);
 *   - the Crank-Nicolson system, Sec. 2.3, eq. (4cranknicholson3), with the
 *     parameters of eq. (stabparams);
 *   - prolongation and restriction of Algorithm 1 between the Q2 spaces of
 *     levels L and L + 1;
 *   - one patch per cell of level L (Sec. 4.2): here one fine Q2 element.
 * Readings where the paper is silent:
 *   - mesh: a logically structured box of n[a] fine Q2 elements per axis;
 *     element (I, J, K) holds the 27 nodes (2I + a, 2J + b, 2K + c),
 *     a, b, c in {0, 1, 2}, local index a + 3b + 9c; node positions are given
 *     (FP64 [3][n_nodes]) and the element map is the Q2 interpolation of its
 *     27 positions (isoparametric);
 *   - the coarse Q2 mesh has the elements of 2 x 2 x 2 fine elements (n even);
 *     its nodes are the fine nodes with even indices;
 *   - pi_h on an element: Q1 interpolation of its 8 vertex values in
 *     reference coordinates;
 *   - h_T: the largest distance between two vertices of T; |v|_inf,T: the
 *     largest Euclidean |v| over the 27 nodes of T;
 *   - quadrature: 3 x 3 x 3 Gauss-Legendre points on every element;
 *   - Dirichlet velocity rows are zero; no periodic axes.
 *
 * Nothing here is blocked, fused or reordered beyond the definitions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n[3];
    double len[3]; /* unused: the node positions define the geometry */
    uint32_t periodic_mask;
    uint32_t dirichlet_mask;
} q2_box;

typedef struct {
    double nu, dt, alpha0, delta0;
} q2_ns;

/* ---------------------------------------------------------------- mesh -- */

static int64_t naxis(const q2_box *b, int a) { return 2 * (int64_t)b->n[a] + 1; }
int64_t q2_fine_nodes(const q2_box *b) { return naxis(b, 0) * naxis(b, 1) * naxis(b, 2); }
int64_t q2_coarse_nodes(const q2_box *b) {
    return ((int64_t)b->n[0] + 1) * ((int64_t)b->n[1] + 1) * ((int64_t)b->n[2] + 1);
}
int64_t q2_elements(const q2_box *b) { return (int64_t)b->n[0] * b->n[1] * b->n[2]; }

static int64_t fnode(const q2_box *b, int64_t i, int64_t j, int64_t k) {
    return i + naxis(b, 0) * (j + naxis(b, 1) * k);
}
static int64_t cnode(const q2_box *b, int64_t I, int64_t J, int64_t K) {
    return I + ((int64_t)b->n[0] + 1) * (J + ((int64_t)b->n[1] + 1) * K);
}

static int on_dirichlet(const q2_box *b, int64_t i, int64_t j, int64_t k) {
    int64_t idx[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) {
        if (idx[a] == 0 && ((b->dirichlet_mask >> (2 * a)) & 1u)) return 1;
        if (idx[a] == naxis(b, a) - 1 && ((b->dirichlet_mask >> (2 * a + 1)) & 1u)) return 1;
    }
    return 0;
}

/* ------------------------------------------------ 1-D shape functions -- */

/* quadratic Lagrange basis on [0,1] with nodes 0, 1/2, 1 */
static double qb(int a, double t) {
    if (a == 0) return 2.0 * (t - 0.5) * (t - 1.0);
    if (a == 1) return 4.0 * t * (1.0 - t);
    return 2.0 * t * (t - 0.5);
}
static double dqb(int a, double t) {
    if (a == 0) return 4.0 * t - 3.0;
    if (a == 1) return 4.0 - 8.0 * t;
    return 4.0 * t - 1.0;
}
/* linear basis on [0,1] (the Q1 space pi_h maps into) */
static double lb(int a, double t) { return a ? t : 1.0 - t; }
static double dlb(int a) { return a ? 1.0 : -1.0; }

/* ------------------------- Crank-Nicolson operator and RHS (Sec. 2.3) -- */

/* Weak-form contributions of element (EI, EJ, EK) for the 27 test nodes.
 *
 * mode 0, the terms of eq. (4cranknicholson3) that depend on the iterate
 * x = (v, p), test functions phi_i e_a and xi_i:
 *   (1/k)(v_a, phi) + 1/2 (v.grad v_a, phi) + nu/2 (grad v_a, grad phi)
 *     - (p, d_a phi) + delta_T (v.grad v_a - pi v.grad pi v_a,
 *                               v.grad phi - pi v.grad pi phi)
 *   (div v, xi) + alpha_T (grad(p - pi p), grad(xi - pi xi))
 * mode 1, the right-hand side built from the velocity v = x[0..2]:
 *   (1/k)(v_a, phi) - 1/2 (v.grad v_a, phi) - nu/2 (grad v_a, grad phi)
 *     + (fmid_a, phi)                      (continuity rows: nothing)
 * pi is Q1 interpolation from the element's vertices, so pi phi_i is the
 * trilinear function of vertex i when i is a vertex and 0 otherwise. */
static void element_terms(const q2_box *b, const q2_ns *ns, int mode, const double *X,
                          const double *x, const double *fmid, int64_t EI, int64_t EJ,
                          int64_t EK, double out[27][4]) {
    const int64_t nn = q2_fine_nodes(b);
    const double s = 0.5 * sqrt(0.6);
    const double gpt[3] = {0.5 - s, 0.5, 0.5 + s};
    const double gwt[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};

    int64_t g[27];
    for (int c = 0; c < 3; ++c)
        for (int bb = 0; bb < 3; ++bb)
            for (int a = 0; a < 3; ++a) g[a + 3 * bb + 9 * c] = fnode(b, 2 * EI + a, 2 * EJ + bb, 2 * EK + c);
    /* vertex v = (v & 1, v >> 1 & 1, v >> 2 & 1) is local node 2 va + 6 vb + 18 vc */
    int vloc[8], vof[27];
    for (int i = 0; i < 27; ++i) vof[i] = -1;
    for (int v = 0; v < 8; ++v) {
        vloc[v] = 2 * (v & 1) + 6 * ((v >> 1) & 1) + 18 * ((v >> 2) & 1);
        vof[vloc[v]] = v;
    }

    double alphaT = 0.0, deltaT = 0.0;
    if (mode == 0) {
        double hT = 0.0;
        for (int v = 0; v < 8; ++v)
            for (int w = v + 1; w < 8; ++w) {
                double d2 = 0.0;
                for (int d = 0; d < 3; ++d) {
                    double e = X[d * nn + g[vloc[v]]] - X[d * nn + g[vloc[w]]];
                    d2 += e * e;
                }
                if (sqrt(d2) > hT) hT = sqrt(d2);
            }
        double vmax = 0.0;
        for (int i = 0; i < 27; ++i) {
            double s2 = 0.0;
            for (int a = 0; a < 3; ++a) s2 += x[a * nn + g[i]] * x[a * nn + g[i]];
            if (sqrt(s2) > vmax) vmax = sqrt(s2);
        }
        double den = ns->nu / (hT * hT) + vmax / hT + 1.0 / ns->dt;
        alphaT = ns->alpha0 / den;
        deltaT = ns->delta0 / den;
    }

    for (int q = 0; q < 27; ++q) {
        double xi[3] = {gpt[q % 3], gpt[(q / 3) % 3], gpt[q / 9]};
        double wq = gwt[q % 3] * gwt[(q / 3) % 3] * gwt[q / 9];

        double N[27], dN[27][3];
        for (int i = 0; i < 27; ++i) {
            int a = i % 3, bb = (i / 3) % 3, c = i / 9;
            N[i] = qb(a, xi[0]) * qb(bb, xi[1]) * qb(c, xi[2]);
            dN[i][0] = dqb(a, xi[0]) * qb(bb, xi[1]) * qb(c, xi[2]);
            dN[i][1] = qb(a, xi[0]) * dqb(bb, xi[1]) * qb(c, xi[2]);
            dN[i][2] = qb(a, xi[0]) * qb(bb, xi[1]) * dqb(c, xi[2]);
        }
        /* J[d][e] = d x_d / d xi_e */
        double J[3][3] = {{0}};
        for (int i = 0; i < 27; ++i)
            for (int d = 0; d < 3; ++d)
                for (int e = 0; e < 3; ++e) J[d][e] += X[d * nn + g[i]] * dN[i][e];
        double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        /* Ji[e][d] = d xi_e / d x_d (inverse by cofactors) */
        double Ji[3][3];
        Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
        const double w = wq * det;

        /* physical gradients of the Q2 functions and of the vertex Q1 functions */
        double G[27][3], L[8], GL[8][3];
        for (int i = 0; i < 27; ++i)
            for (int d = 0; d < 3; ++d) {
                G[i][d] = 0.0;
                for (int e = 0; e < 3; ++e) G[i][d] += dN[i][e] * Ji[e][d];
            }
        for (int v = 0; v < 8; ++v) {
            int va = v & 1, vb = (v >> 1) & 1, vc = (v >> 2) & 1;
            double dL[3] = {dlb(va) * lb(vb, xi[1]) * lb(vc, xi[2]),
                            lb(va, xi[0]) * dlb(vb) * lb(vc, xi[2]),
                            lb(va, xi[0]) * lb(vb, xi[1]) * dlb(vc)};
            L[v] = lb(va, xi[0]) * lb(vb, xi[1]) * lb(vc, xi[2]);
            for (int d = 0; d < 3; ++d) {
                GL[v][d] = 0.0;
                for (int e = 0; e < 3; ++e) GL[v][d] += dL[e] * Ji[e][d];
            }
        }

        /* fields at the point: v, grad v (gv[a][d] = d v_a / d x_d), p, grad p,
         * the forcing, and the interpolants pi v, grad pi v, grad pi p */
        double v[3] = {0, 0, 0}, gv[3][3] = {{0}}, p = 0.0, gp[3] = {0, 0, 0}, f[3] = {0, 0, 0};
        for (int i = 0; i < 27; ++i) {
            for (int a = 0; a < 3; ++a) {
                double va = x[a * nn + g[i]];
                v[a] += va * N[i];
                for (int d = 0; d < 3; ++d) gv[a][d] += va * G[i][d];
                if (fmid) f[a] += fmid[a * nn + g[i]] * N[i];
            }
            if (mode == 0) {
                double pi_ = x[3 * nn + g[i]];
                p += pi_ * N[i];
                for (int d = 0; d < 3; ++d) gp[d] += pi_ * G[i][d];
            }
        }
        double piv[3] = {0, 0, 0}, gpiv[3][3] = {{0}}, gpip[3] = {0, 0, 0};
        if (mode == 0)
            for (int vv = 0; vv < 8; ++vv) {
                int64_t gn = g[vloc[vv]];
                for (int a = 0; a < 3; ++a) {
                    double va = x[a * nn + gn];
                    piv[a] += va * L[vv];
                    for (int d = 0; d < 3; ++d) gpiv[a][d] += va * GL[vv][d];
                }
                for (int d = 0; d < 3; ++d) gpip[d] += x[3 * nn + gn] * GL[vv][d];
            }

        double conv[3], R[3];
        for (int a = 0; a < 3; ++a) {
            double cpi = 0.0;
            conv[a] = 0.0;
            for (int d = 0; d < 3; ++d) {
                conv[a] += v[d] * gv[a][d];
                cpi += piv[d] * gpiv[a][d];
            }
            R[a] = conv[a] - cpi;
        }
        double divv = gv[0][0] + gv[1][1] + gv[2][2];

        for (int i = 0; i < 27; ++i) {
            double Gpi[3] = {0, 0, 0}; /* grad pi phi_i */
            if (vof[i] >= 0)
                for (int d = 0; d < 3; ++d) Gpi[d] = GL[vof[i]][d];
            if (mode == 0) {
                double st = 0.0;
                for (int d = 0; d < 3; ++d) st += v[d] * G[i][d] - piv[d] * Gpi[d];
                for (int a = 0; a < 3; ++a) {
                    double vis = 0.0;
                    for (int d = 0; d < 3; ++d) vis += gv[a][d] * G[i][d];
                    double val = (1.0 / ns->dt) * v[a] * N[i] + 0.5 * conv[a] * N[i] +
                                 0.5 * ns->nu * vis - p * G[i][a] + deltaT * R[a] * st;
                    out[i][a] += w * val;
                }
                double lps = 0.0;
                for (int d = 0; d < 3; ++d) lps += (gp[d] - gpip[d]) * (G[i][d] - Gpi[d]);
                out[i][3] += w * (divv * N[i] + alphaT * lps);
            } else {
                for (int a = 0; a < 3; ++a) {
                    double vis = 0.0;
                    for (int d = 0; d < 3; ++d) vis += gv[a][d] * G[i][d];
                    double val = (1.0 / ns->dt) * v[a] * N[i] - 0.5 * conv[a] * N[i] -
                                 0.5 * ns->nu * vis + f[a] * N[i];
                    out[i][a] += w * val;
                }
            }
        }
    }
}

static void assemble(const q2_box *b, const q2_ns *ns, int mode, const double *X, const double *x,
                     const double *fmid, double *out) {
    const int64_t nn = q2_fine_nodes(b);
    for (int64_t t = 0; t < 4 * nn; ++t) out[t] = 0.0;
    for (int64_t K = 0; K < b->n[2]; ++K)
        for (int64_t J = 0; J < b->n[1]; ++J)
            for (int64_t I = 0; I < b->n[0]; ++I) {
                double e[27][4];
                memset(e, 0, sizeof e);
                element_terms(b, ns, mode, X, x, fmid, I, J, K, e);
                for (int c = 0; c < 3; ++c)
                    for (int bb = 0; bb < 3; ++bb)
                        for (int a = 0; a < 3; ++a) {
                            int64_t gn = fnode(b, 2 * I + a, 2 * J + bb, 2 * K + c);
                            for (int f = 0; f < 4; ++f) out[f * nn + gn] += e[a + 3 * bb + 9 * c][f];
                        }
            }
    for (int64_t k = 0; k < naxis(b, 2); ++k)
        for (int64_t j = 0; j < naxis(b, 1); ++j)
            for (int64_t i = 0; i < naxis(b, 0); ++i)
                if (on_dirichlet(b, i, j, k))
                    for (int a = 0; a < 3; ++a) out[a * nn + fnode(b, i, j, k)] = 0.0;
}

/* A(x): the terms of eq. (4cranknicholson3) and the LPS terms of eq.
 * (disc:ns) that depend on the iterate x = (u, v, w, p) [4][n_nodes];
 * X: node positions [3][n_nodes]; Dirichlet velocity rows 0. */
void q2_apply(const q2_box *b, const q2_ns *ns, const double *X, const double *x, double *out) {
    assemble(b, ns, 0, X, x, NULL, out);
}

/* r = bvec - A(x) (Algorithm 1, residual on the fine level against the
 * right-hand side of the previous step); Dirichlet velocity rows 0. */
void q2_residual_b(const q2_box *b, const q2_ns *ns, const double *X, const double *x,
                   const double *bvec, double *r) {
    const int64_t nn = q2_fine_nodes(b);
    assemble(b, ns, 0, X, x, NULL, r);
    for (int64_t t = 0; t < 4 * nn; ++t) r[t] = bvec[t] - r[t];
    for (int64_t k = 0; k < naxis(b, 2); ++k)
        for (int64_t j = 0; j < naxis(b, 1); ++j)
            for (int64_t i = 0; i < naxis(b, 0); ++i)
                if (on_dirichlet(b, i, j, k))
                    for (int a = 0; a < 3; ++a) r[a * nn + fnode(b, i, j, k)] = 0.0;
}

/* b = Rhs(v, fmid) of eq. (4cranknicholson3) (Algorithm 1, "Rhs"): velocity
 * v [3][n_nodes], fmid [3][n_nodes] or NULL; pressure and Dirichlet velocity
 * rows 0. */
void q2_rhs(const q2_box *b, const q2_ns *ns, const double *X, const double *v, const double *fmid,
            double *out) {
    const int64_t nn = q2_fine_nodes(b);
    double *x = (double *)calloc((size_t)(4 * nn), sizeof(double));
    memcpy(x, v, sizeof(double) * 3 * nn);
    assemble(b, ns, 1, X, x, fmid, out);
    for (int64_t t = 0; t < nn; ++t) out[3 * nn + t] = 0.0;
    free(x);
}

/* Smallest det J over the Gauss points of all elements (mesh validity). */
double q2_min_det(const q2_box *b, const double *X) {
    const int64_t nn = q2_fine_nodes(b);
    const double s = 0.5 * sqrt(0.6);
    const double gpt[3] = {0.5 - s, 0.5, 0.5 + s};
    double mn = INFINITY;
    for (int64_t K = 0; K < b->n[2]; ++K)
        for (int64_t J = 0; J < b->n[1]; ++J)
            for (int64_t I = 0; I < b->n[0]; ++I)
                for (int q = 0; q < 27; ++q) {
                    double xi[3] = {gpt[q % 3], gpt[(q / 3) % 3], gpt[q / 9]};
                    double Jm[3][3] = {{0}};
                    for (int i = 0; i < 27; ++i) {
                        int a = i % 3, bb = (i / 3) % 3, c = i / 9;
                        double dN[3] = {dqb(a, xi[0]) * qb(bb, xi[1]) * qb(c, xi[2]),
                                        qb(a, xi[0]) * dqb(bb, xi[1]) * qb(c, xi[2]),
                                        qb(a, xi[0]) * qb(bb, xi[1]) * dqb(c, xi[2])};
                        int64_t gn = fnode(b, 2 * I + a, 2 * J + bb, 2 * K + c);
                        for (int d = 0; d < 3; ++d)
                            for (int e = 0; e < 3; ++e) Jm[d][e] += X[d * nn + gn] * dN[e];
                    }
                    double det = Jm[0][0] * (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1]) -
                                 Jm[0][1] * (Jm[1][0] * Jm[2][2] - Jm[1][2] * Jm[2][0]) +
                                 Jm[0][2] * (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]);
                    if (det < mn) mn = det;
                }
    return mn;
}

/* --------------------------- transfer between levels L and L+1 (Alg. 1) -- */

/* Fine node i on axis a lies in coarse element e = min(i / 4, n/2 - 1) at
 * reference coordinate t = (i - 4e) / 4; its value is the coarse element's
 * Q2 interpolant there (coarse nodes 2e, 2e + 1, 2e + 2). */
static void pweights(const q2_box *b, int a, int64_t i, int64_t idx[3], double w[3]) {
    int64_t m = b->n[a] / 2;
    int64_t e = i / 4;
    if (e > m - 1) e = m - 1;
    double t = (double)(i - 4 * e) / 4.0;
    for (int s = 0; s < 3; ++s) {
        idx[s] = 2 * e + s;
        w[s] = qb(s, t);
    }
}

/* xf = P xc: xc [ncomp][n_coarse], xf [ncomp][n_nodes]. */
void q2_prolong(const q2_box *b, int ncomp, const double *xc, double *xf) {
    const int64_t nn = q2_fine_nodes(b), nc = q2_coarse_nodes(b);
    for (int64_t k = 0; k < naxis(b, 2); ++k)
        for (int64_t j = 0; j < naxis(b, 1); ++j)
            for (int64_t i = 0; i < naxis(b, 0); ++i) {
                int64_t I[3], Jx[3], Kx[3];
                double wi[3], wj[3], wk[3];
                pweights(b, 0, i, I, wi);
                pweights(b, 1, j, Jx, wj);
                pweights(b, 2, k, Kx, wk);
                for (int c = 0; c < ncomp; ++c) {
                    double s = 0.0;
                    for (int z = 0; z < 3; ++z)
                        for (int y = 0; y < 3; ++y)
                            for (int xx = 0; xx < 3; ++xx)
                                s += wi[xx] * wj[y] * wk[z] * xc[c * nc + cnode(b, I[xx], Jx[y], Kx[z])];
                    xf[c * nn + fnode(b, i, j, k)] = s;
                }
            }
}

/* bc = P^T bf: bf [ncomp][n_nodes], bc [ncomp][n_coarse]. */
void q2_restrict(const q2_box *b, int ncomp, const double *bf, double *bc) {
    const int64_t nn = q2_fine_nodes(b), nc = q2_coarse_nodes(b);
    for (int64_t t = 0; t < ncomp * nc; ++t) bc[t] = 0.0;
    for (int64_t k = 0; k < naxis(b, 2); ++k)
        for (int64_t j = 0; j < naxis(b, 1); ++j)
            for (int64_t i = 0; i < naxis(b, 0); ++i) {
                int64_t I[3], Jx[3], Kx[3];
                double wi[3], wj[3], wk[3];
                pweights(b, 0, i, I, wi);
                pweights(b, 1, j, Jx, wj);
                pweights(b, 2, k, Kx, wk);
                for (int c = 0; c < ncomp; ++c) {
                    double v = bf[c * nn + fnode(b, i, j, k)];
                    for (int z = 0; z < 3; ++z)
                        for (int y = 0; y < 3; ++y)
                            for (int xx = 0; xx < 3; ++xx)
                                bc[c * nc + cnode(b, I[xx], Jx[y], Kx[z])] += wi[xx] * wj[y] * wk[z] * v;
                }
            }
}

/* ----------------------------------------- network inputs (Sec. 4.2) -- */

/* Geometry inputs of element M: g_a = mean length of its 4 vertex-to-vertex
 * edges along logical axis a.  feat [n_elements][3]. */
void q2_features(const q2_box *b, const double *X, double *feat) {
    const int64_t nn = q2_fine_nodes(b);
    for (int64_t K = 0; K < b->n[2]; ++K)
        for (int64_t J = 0; J < b->n[1]; ++J)
            for (int64_t I = 0; I < b->n[0]; ++I) {
                int64_t M = I + b->n[0] * (J + (int64_t)b->n[1] * K);
                for (int a = 0; a < 3; ++a) {
                    double sum = 0.0;
                    for (int v = 0; v < 8; ++v) {
                        if ((v >> a) & 1) continue; /* edge from vertex v to v + 2^a */
                        int w = v | (1 << a);
                        int64_t p0 = fnode(b, 2 * I + 2 * (v & 1), 2 * J + 2 * ((v >> 1) & 1), 2 * K + 2 * ((v >> 2) & 1));
                        int64_t p1 = fnode(b, 2 * I + 2 * (w & 1), 2 * J + 2 * ((w >> 1) & 1), 2 * K + 2 * ((w >> 2) & 1));
                        double d2 = 0.0;
                        for (int d = 0; d < 3; ++d) {
                            double e = X[d * nn + p1] - X[d * nn + p0];
                            d2 += e * e;
                        }
                        sum += sqrt(d2);
                    }
                    feat[3 * M + a] = 0.25 * sum;
                }
            }
}

/* Q of eq. (defQ) on the fine Q2 elements plus the geometry inputs: row M =
 * [u(27), v(27), w(27), r_u(27), r_v(27), r_w(27), g0, g1, g2] (local node
 * a + 3b + 9c), then z = (row - shift) * inv_scale (NULL = identity).
 * x, r [>=3][n_nodes]; out [n_elements][165]. */
void q2_gather(const q2_box *b, const double *X, const double *x, const double *r,
               const double *shift, const double *inv_scale, double *out) {
    const int64_t nn = q2_fine_nodes(b), ne = q2_elements(b);
    double *feat = (double *)malloc(sizeof(double) * 3 * ne);
    q2_features(b, X, feat);
    for (int64_t K = 0; K < b->n[2]; ++K)
        for (int64_t J = 0; J < b->n[1]; ++J)
            for (int64_t I = 0; I < b->n[0]; ++I) {
                int64_t M = I + b->n[0] * (J + (int64_t)b->n[1] * K);
                double *row = out + 165 * M;
                for (int i = 0; i < 27; ++i) {
                    int64_t gn = fnode(b, 2 * I + i % 3, 2 * J + (i / 3) % 3, 2 * K + i / 9);
                    for (int a = 0; a < 3; ++a) {
                        row[27 * a + i] = x[a * nn + gn];
                        row[81 + 27 * a + i] = r[a * nn + gn];
                    }
                }
                for (int a = 0; a < 3; ++a) row[162 + a] = feat[3 * M + a];
                for (int c = 0; c < 165; ++c) {
                    double z = row[c];
                    if (shift) z -= shift[c];
                    if (inv_scale) z *= inv_scale[c];
                    row[c] = z;
                }
            }
    free(feat);
}
