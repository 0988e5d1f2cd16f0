// GPU-resident coarse step (Alg. 1: the coarse problem of a time step;
// Sec. 2.4: Newton's method, GMRES preconditioned by geometric multigrid,
// local Vanka smoothing).  Solves A(x) = b on the coarse mesh of a box.
//
// Levels: mesh l has n / 2^l cells per axis (l = 0 is the coarse mesh of
// the box).  It is the fine mesh of the kernel description M[l] (a box of
// n / 2^(l+1) cells), so the residual, Vanka and transfer kernels of the
// hot path apply to it unchanged: M[l]'s coarse nodes are mesh l+1.
//
// Newton step k:  r = b - A(x);  FGMRES(m) on J dx = r with right
// preconditioner V (one V-cycle);  x += dx.
// J z = (A(x + eps z) - A(x)) / eps is evaluated with the FP32 residual
// kernel (matrix-free; eps scaled by rms(x) / rms(z)).  The V-cycle smooths
// J_l z = s_l with linear coupled patch-Vanka steps linearised at x_l (the
// Newton iterate injected to mesh l), restricts defects with the transpose
// of the Q1 prolongation and prolongates corrections with it.  The local
// Vanka systems depend on x_l only: they are inverted once per Newton step
// (108 x 108 per patch) and each smoothing step is a local mat-vec.
// Inner products and norms accumulate in FP64; the Hessenberg system is
// FP64 and solved with Givens rotations on the device, so nothing returns
// to the host and the whole solve can be recorded into a graph.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace dnnmg {

int residual_launch_b(const Mesh &m, const dnnmg_ns *ns, const float *x, const float *b, float *r, float *aux,
                      const int *flag, hipStream_t s);
size_t lps_ws_bytes(const Mesh &m);
size_t vanka_local_bytes(const Mesh &m);
size_t vanka_inverse_bytes(const Mesh &m);
int vanka_factor(const Mesh &m, const dnnmg_ns *ns, const float *x, float *Ainv, hipStream_t s);
int vanka_apply_factored(const Mesh &m, const float *Ainv, const float *d, float *D, float omega, float *z,
                         hipStream_t s);
int device_cus();

namespace {

constexpr int NPART = 256;  // partial sums of a reduction
constexpr int MAXDOT = DNNMG_COARSE_MAX_KRYLOV + 1;

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

unsigned vec_grid(int64_t n) {
    const unsigned cap = 8u * (unsigned)device_cus();
    const unsigned g = blocks_for(n, 256);
    return g < cap ? g : cap;
}

// ------------------------------------------------------------ kernels ----

__global__ void __launch_bounds__(256) k_f64_to_f32(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        b[t] = (float)a[t];
}

__global__ void __launch_bounds__(256) k_zero(int64_t n, float *__restrict__ a) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        a[t] = 0.0f;
}

// x <- x + dx (FP64 iterate, FP32 correction)
__global__ void __launch_bounds__(256) k_add_f32(int64_t n, double *__restrict__ x, const float *__restrict__ dx) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        x[t] += (double)dx[t];
}

// Coarse node (I, J, K) of M takes the value of fine node (2I, 2J, 2K).
__global__ void __launch_bounds__(256) k_inject(Mesh m, const float *__restrict__ xf, float *__restrict__ xc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * m.n_coarse) return;
    const int comp = (int)(t / m.n_coarse);
    const int64_t c = t - (int64_t)comp * m.n_coarse;
    const uint32_t JK = fdiv((uint32_t)c, m.cx), I = (uint32_t)c - JK * m.nc[0];
    const uint32_t K = fdiv(JK, m.cy), J = JK - K * m.nc[1];
    xc[t] = xf[(int64_t)comp * m.n_fine + 2 * (int64_t)I + (int64_t)m.nf[0] * (2 * (int64_t)J + (int64_t)m.nf[1] * 2 * K)];
}

// Is coarse node C of M on a Dirichlet face?
__device__ __forceinline__ bool coarse_dirichlet(const Mesh &m, const int C[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (m.per[a]) continue;
        if (C[a] == 0 && ((m.dmask >> (2 * a)) & 1u)) return true;
        if (C[a] == m.nc[a] - 1 && ((m.dmask >> (2 * a + 1)) & 1u)) return true;
    }
    return false;
}

// Defect restriction s_c = P^T d_f (P the Q1 prolongation: weight 1 at the
// coincident fine node, 1/2 at its two neighbours per axis), FP64 sums;
// Dirichlet velocity rows of the coarse mesh zero.
__global__ void __launch_bounds__(256) k_mg_restrict(Mesh m, const float *__restrict__ df, float *__restrict__ sc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * m.n_coarse) return;
    const int comp = (int)(t / m.n_coarse);
    const int64_t c = t - (int64_t)comp * m.n_coarse;
    const uint32_t JK = fdiv((uint32_t)c, m.cx), I = (uint32_t)c - JK * m.nc[0];
    const uint32_t K = fdiv(JK, m.cy), J = JK - K * m.nc[1];
    const int C[3] = {(int)I, (int)J, (int)K};
    if (comp < 3 && coarse_dirichlet(m, C)) {
        sc[t] = 0.0f;
        return;
    }
    int f[3][3];
    double w[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int fi = 2 * C[a] + d - 1;
            bool ok = true;
            if (m.per[a]) fi = wrap(fi, m.nf[a], 1);
            else if (fi < 0 || fi >= m.nf[a]) {
                ok = false;
                fi = 2 * C[a];
            }
            f[a][d] = fi;
            w[a][d] = ok ? (d == 1 ? 1.0 : 0.5) : 0.0;
        }
    const float *src = df + (int64_t)comp * m.n_fine;
    double acc = 0.0;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) {
            const int64_t row = (int64_t)m.nf[0] * (f[1][bb] + (int64_t)m.nf[1] * f[2][cc]);
            const double s = w[0][0] * src[f[0][0] + row] + w[0][1] * src[f[0][1] + row] + w[0][2] * src[f[0][2] + row];
            acc += w[1][bb] * w[2][cc] * s;
        }
    sc[t] = (float)acc;
}

// Correction prolongation z_f += P z_c: the thread of coarse node C adds to
// the fine nodes 2C + {0, 1}^3 that exist (each fine node has one such C).
__global__ void __launch_bounds__(256) k_mg_prolong_add(Mesh m, const float *__restrict__ zc, float *__restrict__ zf) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * m.n_coarse) return;
    const int comp = (int)(t / m.n_coarse);
    const int64_t c = t - (int64_t)comp * m.n_coarse;
    const uint32_t JK = fdiv((uint32_t)c, m.cx), I = (uint32_t)c - JK * m.nc[0];
    const uint32_t K = fdiv(JK, m.cy), J = JK - K * m.nc[1];
    const int C[3] = {(int)I, (int)J, (int)K};
    int hi[3];
    bool odd[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int upn = C[a] + 1;
        if (m.per[a]) upn = upn == m.nc[a] ? 0 : upn;
        odd[a] = m.per[a] || C[a] + 1 < m.nc[a];
        hi[a] = odd[a] ? upn : C[a];
    }
    const float *z = zc + (int64_t)comp * m.n_coarse;
    float v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int ii = (q & 1) ? hi[0] : C[0], jj = (q & 2) ? hi[1] : C[1], kk = (q & 4) ? hi[2] : C[2];
        v[q] = z[ii + (int64_t)m.nc[0] * (jj + (int64_t)m.nc[1] * kk)];
    }
    float *out = zf + (int64_t)comp * m.n_fine + 2 * (int64_t)I +
                 (int64_t)m.nf[0] * (2 * (int64_t)J + (int64_t)m.nf[1] * 2 * K);
#pragma unroll
    for (int cz = 0; cz < 2; ++cz) {
        if (cz && !odd[2]) break;
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
            if (cy && !odd[1]) break;
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                if (cx && !odd[0]) break;
                // trilinear weights at the offsets (cx, cy, cz) in {0, 1/2}
                float s = 0.0f;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int qa = q & 1, qb = (q >> 1) & 1, qc = q >> 2;
                    const float wx = cx ? 0.5f : (qa ? 0.0f : 1.0f);
                    const float wy = cy ? 0.5f : (qb ? 0.0f : 1.0f);
                    const float wz = cz ? 0.5f : (qc ? 0.0f : 1.0f);
                    s += wx * wy * wz * v[q];
                }
                out[cx + (int64_t)m.nf[0] * (cy + (int64_t)m.nf[1] * cz)] += s;
            }
        }
    }
}

// Partial inner products part[c][block] = sum_t w[t] * V[c][t] (c < nvec;
// V[c] = V + c * ldv; V == nullptr: the squares of w), FP64.
__global__ void __launch_bounds__(256) k_dots_partial(int64_t n, const float *__restrict__ w,
                                                      const float *__restrict__ V, int64_t ldv, int nvec,
                                                      double *__restrict__ part) {
    double acc[MAXDOT];
#pragma unroll
    for (int c = 0; c < MAXDOT; ++c) acc[c] = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const double wt = w[t];
        if (!V) {
            acc[0] += wt * wt;
            continue;
        }
#pragma unroll
        for (int c = 0; c < MAXDOT; ++c)
            if (c < nvec) acc[c] += wt * (double)V[c * ldv + t];
    }
    __shared__ double red[256];
    for (int c = 0; c < nvec; ++c) {
        red[threadIdx.x] = acc[0];
#pragma unroll
        for (int q = 1; q < MAXDOT; ++q)
            if (q == c) red[threadIdx.x] = acc[q];
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(int64_t)c * NPART + blockIdx.x] = red[0];
        __syncthreads();
    }
}

// out[c] = sum of part[c][0 .. nparts) (one block per c); sqrt_out: the
// square root (a norm).
__global__ void __launch_bounds__(256) k_dots_final(int nparts, const double *__restrict__ part,
                                                    double *__restrict__ out, int sqrt_out) {
    __shared__ double red[256];
    const double *p = part + (int64_t)blockIdx.x * NPART;
    double s = 0.0;
    for (int t = threadIdx.x; t < nparts; t += 256) s += p[t];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sqrt_out ? sqrt(red[0]) : red[0];
}

// Finite-difference step from ||x|| and ||z|| (2-norms over n entries):
// eps = eta (rms x + eta) / rms z, 0 when z = 0.
__global__ void k_fd_eps(const double *__restrict__ xnorm, const double *__restrict__ znorm, double rn, double eta,
                         double *__restrict__ eps) {
    const double zr = *znorm * rn;
    *eps = zr > 0.0 ? eta * (*xnorm * rn + eta) / zr : 0.0;
}

// y = x + eps z
__global__ void __launch_bounds__(256) k_perturb(int64_t n, const float *__restrict__ x, const float *__restrict__ z,
                                                 const double *__restrict__ eps, float *__restrict__ y) {
    const float e = (float)*eps;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        y[t] = x[t] + e * z[t];
}

// out = s - (a0 - a1) / eps  (s == nullptr: out = (a0 - a1) / eps), the
// defect s - J z with a0 = b0 - A(x), a1 = b0 - A(x + eps z); J z = 0 when
// eps = 0 (z = 0).
__global__ void __launch_bounds__(256) k_fd_defect(int64_t n, const float *__restrict__ s, const float *__restrict__ a0,
                                                   const float *__restrict__ a1, const double *__restrict__ eps,
                                                   float *__restrict__ out) {
    const double e = *eps;
    const float ie = e > 0.0 ? (float)(1.0 / e) : 0.0f;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const float jz = (a0[t] - a1[t]) * ie;
        out[t] = s ? s[t] - jz : jz;
    }
}

// out = in / nrm (0 where nrm = 0)
__global__ void __launch_bounds__(256) k_scale_inv(int64_t n, const float *__restrict__ in,
                                                   const double *__restrict__ nrm, float *__restrict__ out) {
    const double v = *nrm;
    const float s = v > 0.0 ? (float)(1.0 / v) : 0.0f;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        out[t] = in[t] * s;
}

// w -= sum_{c < nvec} h[c] V[c]  (or out = sum h[c] V[c] when sub = 0)
__global__ void __launch_bounds__(256) k_combine(int64_t n, const float *__restrict__ V, int64_t ldv, int nvec,
                                                 const double *__restrict__ h, float *__restrict__ w, int sub) {
    float hc[MAXDOT];
#pragma unroll
    for (int c = 0; c < MAXDOT; ++c) hc[c] = c < nvec ? (float)h[c] : 0.0f;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
#pragma unroll
        for (int c = 0; c < MAXDOT; ++c)
            if (c < nvec) s += hc[c] * V[c * ldv + t];
        w[t] = sub ? w[t] - s : s;
    }
}

// Arnoldi column j of the FGMRES Hessenberg matrix H ((m+1) x m, column
// major, ld m+1): H[0..j][j] = h1 + h2 (the two Gram-Schmidt passes),
// H[j+1][j] = hn; then the rotations of columns 0..j-1 are applied to it,
// a new rotation zeroes H[j+1][j], and g (the rotated right-hand side,
// g[0] = beta at the start) is updated.  One thread.
__global__ void k_arnoldi_givens(int j, int m, const double *__restrict__ h1, const double *__restrict__ h2,
                                 const double *__restrict__ hn, double *__restrict__ H, double *__restrict__ cs,
                                 double *__restrict__ sn, double *__restrict__ g) {
    double *col = H + (int64_t)j * (m + 1);
    for (int i = 0; i <= j; ++i) col[i] = h1[i] + h2[i];
    col[j + 1] = *hn;
    for (int i = 0; i < j; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = cs[i] * a + sn[i] * b;
        col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double a = col[j], b = col[j + 1];
    const double r = hypot(a, b);
    const double c = r > 0.0 ? a / r : 1.0, s = r > 0.0 ? b / r : 0.0;
    cs[j] = c;
    sn[j] = s;
    col[j] = r;
    col[j + 1] = 0.0;
    const double gj = g[j];
    g[j] = c * gj;
    g[j + 1] = -s * gj;
}

// g = (beta, 0, ..., 0)
__global__ void k_gmres_start(int m, const double *__restrict__ beta, double *__restrict__ g) {
    for (int i = 0; i <= m; ++i) g[i] = i ? 0.0 : *beta;
}

// y = R^-1 g[0..m) (R the rotated upper triangle of H); a zero pivot (a
// breakdown before column m) gives y = 0 from there on.  One thread.
__global__ void k_backsolve(int m, const double *__restrict__ H, const double *__restrict__ g, double *__restrict__ y) {
    for (int i = m - 1; i >= 0; --i) {
        double s = g[i];
        for (int k = i + 1; k < m; ++k) s -= H[(int64_t)k * (m + 1) + i] * y[k];
        const double d = H[(int64_t)i * (m + 1) + i];
        y[i] = d != 0.0 ? s / d : 0.0;
    }
}

// ------------------------------------------------------------- layout ----

struct Level {
    dnnmg_box box; // n / 2^(l+1) cells: its fine mesh is mesh l
    Mesh m;
    int64_t n4;    // 4 * nodes of mesh l
    float *x, *a0, *s, *z, *d, *y, *ra, *D, *Ainv;
    char *aux;
    double *xnorm, *eps, *znorm;
};

struct Layout {
    std::vector<Level> L;
    int krylov = 0, newton = 0;
    // level-0 Newton / Krylov vectors
    float *b32 = nullptr, *r = nullptr, *w = nullptr, *V = nullptr, *Z = nullptr, *dx = nullptr, *zeros = nullptr;
    double *part = nullptr, *h1 = nullptr, *h2 = nullptr, *hn = nullptr, *beta = nullptr, *H = nullptr,
           *cs = nullptr, *sn = nullptr, *g = nullptr, *yk = nullptr;
    size_t bytes = 0;
};

int check_opts(const dnnmg_coarse_opts *o) {
    if (!o) return fail(DNNMG_ERR_ARG, "coarse options are NULL");
    if (o->newton_its < 1) return fail(DNNMG_ERR_ARG, "newton_its must be >= 1 (got %d)", o->newton_its);
    if (o->krylov_dim < 1 || o->krylov_dim > DNNMG_COARSE_MAX_KRYLOV)
        return fail(DNNMG_ERR_ARG, "krylov_dim must be in 1..%d (got %d)", DNNMG_COARSE_MAX_KRYLOV, o->krylov_dim);
    if (o->levels < 0) return fail(DNNMG_ERR_ARG, "levels must be >= 0 (got %d)", o->levels);
    if (o->pre_sweeps < 1 || o->post_sweeps < 0 || o->coarsest_sweeps < 1)
        return fail(DNNMG_ERR_ARG, "sweeps: pre >= 1, post >= 0, coarsest >= 1");
    if (!(o->omega > 0.0 && o->omega < 2.0)) return fail(DNNMG_ERR_ARG, "omega must lie in (0, 2)");
    if (!(o->fd_eta > 0.0)) return fail(DNNMG_ERR_ARG, "fd_eta must be > 0");
    return DNNMG_OK;
}

// Meshes of the hierarchy: mesh l has n / 2^l cells; mesh l needs an even
// count of at least 4 cells on every axis (it is the fine mesh of a box of
// half as many cells, and those boxes keep at least 2 cells per axis, the
// smallest the residual and Vanka kernels are built and tested for), and a
// periodic axis an even count of box cells.
int count_levels(const dnnmg_box *box, const dnnmg_coarse_opts *o) {
    if (!box) return fail(DNNMG_ERR_ARG, "box is NULL");
    int rc = check_opts(o);
    if (rc) return rc;
    int lev = 0;
    int n[3] = {box->n[0], box->n[1], box->n[2]};
    for (;;) {
        bool ok = true;
        for (int a = 0; a < 3; ++a) {
            const bool per = (box->periodic_mask >> a) & 1u;
            if (n[a] < 4 || (n[a] & 1) || (per && ((n[a] / 2) & 1))) ok = false;
        }
        if (!ok) break;
        ++lev;
        for (int a = 0; a < 3; ++a) n[a] /= 2;
        if (o->levels > 0 && lev == o->levels) break;
    }
    if (lev == 0)
        return fail(DNNMG_ERR_SHAPE, "the coarse mesh needs even cell counts of at least 4 (%d, %d, %d)",
                    box->n[0], box->n[1], box->n[2]);
    return lev;
}

// Offsets of every buffer in the workspace (base == nullptr: sizes only).
int make_layout(const dnnmg_box *box, const dnnmg_coarse_opts *o, char *base, Layout &Y) {
    const int nl = count_levels(box, o);
    if (nl < 0) return nl;
    Y.L.assign(nl, Level{});
    Y.krylov = o->krylov_dim;
    Y.newton = o->newton_its;
    size_t off = 0;
    auto take = [&](size_t b) -> char * {
        char *p = base ? base + off : nullptr;
        off += up256(b);
        return p;
    };
    for (int l = 0; l < nl; ++l) {
        Level &v = Y.L[l];
        v.box = *box;
        for (int a = 0; a < 3; ++a) v.box.n[a] = box->n[a] >> (l + 1);
        int rc = make_mesh(&v.box, &v.m);
        if (rc) return rc;
        v.n4 = 4 * v.m.n_fine;
        const size_t vb = sizeof(float) * (size_t)v.n4;
        v.x = (float *)take(vb);
        v.a0 = (float *)take(vb);
        v.s = (float *)take(vb);
        v.z = (float *)take(vb);
        v.d = (float *)take(vb);
        v.y = (float *)take(vb);
        v.ra = (float *)take(vb);
        v.D = (float *)take(vanka_local_bytes(v.m));
        v.Ainv = (float *)take(vanka_inverse_bytes(v.m));
        v.aux = take(lps_ws_bytes(v.m));
        v.xnorm = (double *)take(sizeof(double));
        v.eps = (double *)take(sizeof(double));
        v.znorm = (double *)take(sizeof(double));
    }
    const int64_t n4 = Y.L[0].n4;
    const size_t vb = sizeof(float) * (size_t)n4;
    const int m = o->krylov_dim;
    Y.b32 = (float *)take(vb);
    Y.r = (float *)take(vb);
    Y.w = (float *)take(vb);
    Y.dx = (float *)take(vb);
    Y.zeros = (float *)take(vb);
    Y.V = (float *)take(vb * (m + 1));
    Y.Z = (float *)take(vb * m);
    Y.part = (double *)take(sizeof(double) * NPART * MAXDOT);
    Y.h1 = (double *)take(sizeof(double) * MAXDOT);
    Y.h2 = (double *)take(sizeof(double) * MAXDOT);
    Y.hn = (double *)take(sizeof(double));
    Y.beta = (double *)take(sizeof(double));
    Y.H = (double *)take(sizeof(double) * (m + 1) * m);
    Y.cs = (double *)take(sizeof(double) * m);
    Y.sn = (double *)take(sizeof(double) * m);
    Y.g = (double *)take(sizeof(double) * (m + 1));
    Y.yk = (double *)take(sizeof(double) * m);
    Y.bytes = off;
    return DNNMG_OK;
}

// ------------------------------------------------------------ drivers ----

struct Ctx {
    const dnnmg_ns *ns;
    const dnnmg_coarse_opts *o;
    Layout *Y;
    hipStream_t s;
};

#define TRY(call)                    \
    do {                             \
        int rc_ = (call);            \
        if (rc_) return rc_;         \
    } while (0)

// out[c] = <w, V[c]> for c < nvec, or the 2-norm of w (V == nullptr)
int dots(const Ctx &c, int64_t n, const float *w, const float *V, int64_t ldv, int nvec, double *out) {
    const unsigned g = blocks_for(n, 256) < (unsigned)NPART ? blocks_for(n, 256) : (unsigned)NPART;
    k_dots_partial<<<g, 256, 0, c.s>>>(n, w, V, ldv, V ? nvec : 1, c.Y->part);
    k_dots_final<<<V ? nvec : 1, 256, 0, c.s>>>((int)g, c.Y->part, out, V ? 0 : 1);
    return hip_check(hipGetLastError(), "coarse dots");
}

int zero(const Ctx &c, int64_t n, float *p) {
    k_zero<<<vec_grid(n), 256, 0, c.s>>>(n, p);
    return hip_check(hipGetLastError(), "coarse zero");
}

// out = s - J_l z (s == nullptr: out = J_l z), J_l at the level's x.
int defect(const Ctx &c, Level &v, const float *s, const float *z, float *out) {
    const int64_t n = v.n4;
    TRY(dots(c, n, z, nullptr, 0, 1, v.znorm));
    k_fd_eps<<<1, 1, 0, c.s>>>(v.xnorm, v.znorm, 1.0 / sqrt((double)n), c.o->fd_eta, v.eps);
    k_perturb<<<vec_grid(n), 256, 0, c.s>>>(n, v.x, z, v.eps, v.y);
    TRY(residual_launch_b(v.m, c.ns, v.y, c.Y->zeros, v.ra, (float *)v.aux, nullptr, c.s));
    k_fd_defect<<<vec_grid(n), 256, 0, c.s>>>(n, s, v.a0, v.ra, v.eps, out);
    return hip_check(hipGetLastError(), "coarse defect");
}

// Linearisation of every level at x_0 (already in L[0].x): x_{l+1} the
// injection of x_l, a0_l = -A_l(x_l), ||x_l||.
int linearise(const Ctx &c) {
    std::vector<Level> &L = c.Y->L;
    for (size_t l = 0; l < L.size(); ++l) {
        Level &v = L[l];
        if (l > 0) {
            const Mesh &mp = L[l - 1].m;
            k_inject<<<blocks_for(4 * mp.n_coarse, 256), 256, 0, c.s>>>(mp, L[l - 1].x, v.x);
        }
        TRY(residual_launch_b(v.m, c.ns, v.x, c.Y->zeros, v.a0, (float *)v.aux, nullptr, c.s));
        TRY(dots(c, v.n4, v.x, nullptr, 0, 1, v.xnorm));
        TRY(vanka_factor(v.m, c.ns, v.x, v.Ainv, c.s));
    }
    return hip_check(hipGetLastError(), "coarse linearisation");
}

int smooth(const Ctx &c, Level &v, const float *s, float *z) {
    TRY(defect(c, v, s, z, v.d));
    return vanka_apply_factored(v.m, v.Ainv, v.d, v.D, (float)c.o->omega, z, c.s);
}

// z0 = V s0: one V-cycle over the levels.  Level 0 reads s0 and writes z0;
// the others use their own s and z.
int vcycle(const Ctx &c, const float *s0, float *z0) {
    std::vector<Level> &L = c.Y->L;
    const int nl = (int)L.size();
    auto S = [&](int l) { return l ? (const float *)L[l].s : s0; };
    auto Zp = [&](int l) { return l ? L[l].z : z0; };
    for (int l = 0; l < nl; ++l) {
        Level &v = L[l];
        float *z = Zp(l);
        TRY(zero(c, v.n4, z));
        // the first sweep's defect is s itself (z = 0)
        TRY(vanka_apply_factored(v.m, v.Ainv, S(l), v.D, (float)c.o->omega, z, c.s));
        const int sweeps = l == nl - 1 ? c.o->coarsest_sweeps : c.o->pre_sweeps;
        for (int it = 1; it < sweeps; ++it) TRY(smooth(c, v, S(l), z));
        if (l == nl - 1) break;
        TRY(defect(c, v, S(l), z, v.d));
        k_mg_restrict<<<blocks_for(4 * v.m.n_coarse, 256), 256, 0, c.s>>>(v.m, v.d, L[l + 1].s);
    }
    for (int l = nl - 2; l >= 0; --l) {
        Level &v = L[l];
        float *z = Zp(l);
        k_mg_prolong_add<<<blocks_for(4 * v.m.n_coarse, 256), 256, 0, c.s>>>(v.m, L[l + 1].z, z);
        for (int it = 0; it < c.o->post_sweeps; ++it) TRY(smooth(c, v, S(l), z));
    }
    return hip_check(hipGetLastError(), "coarse v-cycle");
}

// One FGMRES(m) cycle on J dx = r (r in Y.r), right-preconditioned by the
// V-cycle: dx = sum_j y_j V^-1 v_j.
int fgmres(const Ctx &c) {
    Layout &Y = *c.Y;
    Level &v0 = Y.L[0];
    const int64_t n = v0.n4;
    const int m = Y.krylov;
    TRY(dots(c, n, Y.r, nullptr, 0, 1, Y.beta));
    k_scale_inv<<<vec_grid(n), 256, 0, c.s>>>(n, Y.r, Y.beta, Y.V);
    k_gmres_start<<<1, 1, 0, c.s>>>(m, Y.beta, Y.g);
    for (int j = 0; j < m; ++j) {
        float *vj = Y.V + (int64_t)j * n, *zj = Y.Z + (int64_t)j * n, *vn = Y.V + (int64_t)(j + 1) * n;
        TRY(vcycle(c, vj, zj));
        TRY(defect(c, v0, nullptr, zj, Y.w)); // w = J z_j
        // classical Gram-Schmidt, twice
        TRY(dots(c, n, Y.w, Y.V, n, j + 1, Y.h1));
        k_combine<<<vec_grid(n), 256, 0, c.s>>>(n, Y.V, n, j + 1, Y.h1, Y.w, 1);
        TRY(dots(c, n, Y.w, Y.V, n, j + 1, Y.h2));
        k_combine<<<vec_grid(n), 256, 0, c.s>>>(n, Y.V, n, j + 1, Y.h2, Y.w, 1);
        TRY(dots(c, n, Y.w, nullptr, 0, 1, Y.hn));
        k_scale_inv<<<vec_grid(n), 256, 0, c.s>>>(n, Y.w, Y.hn, vn);
        k_arnoldi_givens<<<1, 1, 0, c.s>>>(j, m, Y.h1, Y.h2, Y.hn, Y.H, Y.cs, Y.sn, Y.g);
    }
    k_backsolve<<<1, 1, 0, c.s>>>(m, Y.H, Y.g, Y.yk);
    k_combine<<<vec_grid(n), 256, 0, c.s>>>(n, Y.Z, n, m, Y.yk, Y.dx, 0);
    return hip_check(hipGetLastError(), "coarse fgmres");
}

int setup(const dnnmg_box *box, const dnnmg_ns *ns, const dnnmg_coarse_opts *o, void *ws, size_t ws_bytes,
          Layout &Y) {
    if (!ns) return fail(DNNMG_ERR_ARG, "ns is NULL");
    if (!ws) return fail(DNNMG_ERR_ARG, "workspace is NULL");
    TRY(make_layout(box, o, nullptr, Y));
    if (ws_bytes < Y.bytes)
        return fail(DNNMG_ERR_ARG, "coarse workspace of %zu bytes, %zu needed", ws_bytes, Y.bytes);
    return make_layout(box, o, (char *)ws, Y);
}

} // namespace
} // namespace dnnmg

using namespace dnnmg;

extern "C" int dnnmg_coarse_levels(const dnnmg_box *box, const dnnmg_coarse_opts *opts) {
    return count_levels(box, opts);
}

extern "C" size_t dnnmg_coarse_workspace(const dnnmg_box *box, const dnnmg_coarse_opts *opts) {
    Layout Y;
    return make_layout(box, opts, nullptr, Y) ? 0 : Y.bytes;
}

extern "C" int dnnmg_coarse_solve(const dnnmg_box *box, const dnnmg_ns *ns, const double *b, double *x,
                                  const dnnmg_coarse_opts *opts, double *res_norms, void *ws, size_t ws_bytes,
                                  void *stream) {
    Layout Y;
    TRY(setup(box, ns, opts, ws, ws_bytes, Y));
    if (!b || !x) return fail(DNNMG_ERR_ARG, "b or x is NULL");
    if ((const void *)b == (const void *)x) return fail(DNNMG_ERR_ARG, "b and x must not alias");
    const hipStream_t s = (hipStream_t)stream;
    const Ctx c{ns, opts, &Y, s};
    Level &v0 = Y.L[0];
    const int64_t n = v0.n4;
    TRY(zero(c, n, Y.zeros));
    k_f64_to_f32<<<vec_grid(n), 256, 0, s>>>(n, b, Y.b32);
    for (int k = 0; k <= Y.newton; ++k) {
        k_f64_to_f32<<<vec_grid(n), 256, 0, s>>>(n, x, v0.x);
        TRY(residual_launch_b(v0.m, ns, v0.x, Y.b32, Y.r, (float *)v0.aux, nullptr, s));
        if (res_norms) TRY(dots(c, n, Y.r, nullptr, 0, 1, res_norms + k));
        if (k == Y.newton) break;
        TRY(linearise(c));
        TRY(fgmres(c));
        k_add_f32<<<vec_grid(n), 256, 0, s>>>(n, x, Y.dx);
    }
    return hip_check(hipGetLastError(), "dnnmg_coarse_solve");
}

extern "C" int dnnmg_coarse_jv(const dnnmg_box *box, const dnnmg_ns *ns, const float *x, const float *z, float *w,
                               const dnnmg_coarse_opts *opts, void *ws, size_t ws_bytes, void *stream) {
    Layout Y;
    TRY(setup(box, ns, opts, ws, ws_bytes, Y));
    if (!x || !z || !w) return fail(DNNMG_ERR_ARG, "x, z or w is NULL");
    if (w == x || w == z) return fail(DNNMG_ERR_ARG, "w must not alias x or z");
    const hipStream_t s = (hipStream_t)stream;
    const Ctx c{ns, opts, &Y, s};
    Level &v0 = Y.L[0];
    TRY(zero(c, v0.n4, Y.zeros));
    TRY(hip_check(hipMemcpyAsync(v0.x, x, sizeof(float) * v0.n4, hipMemcpyDeviceToDevice, s), "coarse jv copy"));
    TRY(residual_launch_b(v0.m, ns, v0.x, Y.zeros, v0.a0, (float *)v0.aux, nullptr, s));
    TRY(dots(c, v0.n4, v0.x, nullptr, 0, 1, v0.xnorm));
    return defect(c, v0, nullptr, z, w);
}

extern "C" int dnnmg_coarse_vcycle(const dnnmg_box *box, const dnnmg_ns *ns, const float *x, const float *sv,
                                   float *z, const dnnmg_coarse_opts *opts, void *ws, size_t ws_bytes, void *stream) {
    Layout Y;
    TRY(setup(box, ns, opts, ws, ws_bytes, Y));
    if (!x || !sv || !z) return fail(DNNMG_ERR_ARG, "x, s or z is NULL");
    if (z == x || z == sv) return fail(DNNMG_ERR_ARG, "z must not alias x or s");
    const hipStream_t s = (hipStream_t)stream;
    const Ctx c{ns, opts, &Y, s};
    Level &v0 = Y.L[0];
    TRY(zero(c, v0.n4, Y.zeros));
    TRY(hip_check(hipMemcpyAsync(v0.x, x, sizeof(float) * v0.n4, hipMemcpyDeviceToDevice, s), "coarse v-cycle copy"));
    TRY(linearise(c));
    return vcycle(c, sv, z);
}
