// Grid-transfer and patch kernels of the DNN-MG correction (Algorithm 1 and
// Sec. 4.2 of arXiv 2307.14837): dof map and valence, Q1 prolongation, its
// transpose (restriction of the right-hand side), the patch gather Q with
// feature standardisation and quantisation, the multiplicity-averaged
// extension L, and FP64 norms.  All of these move little arithmetic per byte
// and are bound by HBM bandwidth; threads map to consecutive x nodes so that
// the fine-field streams are coalesced.
#include "common.hpp"
#include "extension.hpp"
#include "lowp.hpp"
#include "mlp.hpp"

namespace dnnmg {

// ----------------------------------------------------------- dof map ------

__global__ void k_dofmap(Mesh m, int32_t *__restrict__ map) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m.n_patches * 27) return;
    uint32_t M = (uint32_t)(t / 27), iota = (uint32_t)(t - (int64_t)M * 27);
    uint32_t J_K = fdiv(M, m.px), I = M - J_K * m.n[0];
    uint32_t K = fdiv(J_K, m.py), J = J_K - K * m.n[1];
    int a = iota % 3, b = (iota / 3) % 3, c = iota / 9;
    int i = wrap(2 * I + a, m.nf[0], m.per[0]);
    int j = wrap(2 * J + b, m.nf[1], m.per[1]);
    int k = wrap(2 * K + c, m.nf[2], m.per[2]);
    map[t] = i + m.nf[0] * (j + m.nf[1] * k);
}

// valence of a fine node = product over axes of the patches sharing it:
// 2 at even lattice indices that are interior (or on a periodic axis), else 1
__device__ __forceinline__ int valence(const Mesh &m, int i, int j, int k) {
    int c[3] = {i, j, k}, v = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (!(c[a] & 1) && (m.per[a] || (c[a] > 0 && c[a] < 2 * m.n[a]))) v *= 2;
    return v;
}

__global__ void k_mult(Mesh m, uint8_t *__restrict__ mult) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m.n_fine) return;
    uint32_t jk = fdiv((uint32_t)t, m.fx), i = (uint32_t)t - jk * m.nf[0];
    uint32_t k = fdiv(jk, m.fy), j = jk - k * m.nf[1];
    mult[t] = (uint8_t)valence(m, i, j, k);
}

// ------------------------------------------------------- prolongation -----
// 1-D Q1 interpolation: even fine index = coarse node, odd = mean of the two
// coarse neighbours (wrapping on periodic axes).  One thread per (component,
// coarse node) C = (I, J, K) writes the fine nodes 2C + (a, b, c), a, b, c in
// {0, 1}, that exist, from the 2x2x2 coarse block C .. C+1: all loads are
// issued at once (one memory round trip per thread); consecutive threads
// take consecutive nodes of one component.  The FP64 coarse values are
// rounded to FP32 and averaged axis by axis (x, then y, then z) in FP32, the
// same operations the residual kernel uses for the patch interpolant, so a
// prolongated field equals its own patch interpolant bit for bit.
template <typename TO>
__device__ __forceinline__ void prolong_node(const Mesh &m, int64_t t, int ncomp, const double *__restrict__ xc,
                                             TO *__restrict__ xf) {
    if (t >= (int64_t)ncomp * m.n_coarse) return;
    const int comp = (int)(t / m.n_coarse);
    t -= (int64_t)comp * m.n_coarse;
    uint32_t JK = fdiv((uint32_t)t, m.cx), I = (uint32_t)t - JK * m.nc[0];
    uint32_t K = fdiv(JK, m.cy), J = JK - K * m.nc[1];
    const int C[3] = {(int)I, (int)J, (int)K};
    int hi[3];   // index of the upper coarse neighbour (clamped where absent)
    bool odd[3]; // does the odd fine node 2C + 1 exist on this axis?
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int up = C[a] + 1;
        if (m.per[a]) up = up == m.nc[a] ? 0 : up;
        odd[a] = m.per[a] || C[a] + 1 < m.nc[a];
        hi[a] = odd[a] ? up : C[a];
    }
    const double *x = xc + (int64_t)comp * m.n_coarse;
    float v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        int ii = (q & 1) ? hi[0] : C[0], jj = (q & 2) ? hi[1] : C[1], kk = (q & 4) ? hi[2] : C[2];
        v[q] = (float)x[ii + (int64_t)m.nc[0] * (jj + (int64_t)m.nc[1] * kk)];
    }
    // x pass, y pass, z pass: value at offset 0 = corner, at 1 = mean
    float px[8];
#pragma unroll
    for (int q = 0; q < 8; q += 2) { px[q] = v[q]; px[q + 1] = 0.5f * (v[q] + v[q + 1]); }
    float py[8];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            py[a + 4 * c] = px[a + 4 * c];
            py[a + 2 + 4 * c] = 0.5f * (px[a + 4 * c] + px[a + 2 + 4 * c]);
        }
    float pz[8];
#pragma unroll
    for (int ab = 0; ab < 4; ++ab) { pz[ab] = py[ab]; pz[ab + 4] = 0.5f * (py[ab] + py[ab + 4]); }
    const int64_t f0 = 2 * (int64_t)I + (int64_t)m.nf[0] * (2 * (int64_t)J + (int64_t)m.nf[1] * 2 * K);
    TO *out = xf + (int64_t)comp * m.n_fine + f0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        if (c && !odd[2]) break;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            if (b && !odd[1]) break;
            TO *row = out + (int64_t)m.nf[0] * (b + (int64_t)m.nf[1] * c);
            row[0] = pz[2 * b + 4 * c];
            if (odd[0]) row[1] = pz[1 + 2 * b + 4 * c];
        }
    }
}

__global__ void __launch_bounds__(256) k_prolong(Mesh m, int ncomp, const double *__restrict__ xc,
                                                 float *__restrict__ xf) {
    prolong_node(m, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, ncomp, xc, xf);
}

// The same FP32 values widened to FP64 (exact): the level L + 1 iterate of a
// two-level prolongation, which the level L + 2 residual pass prolongs again.
__global__ void __launch_bounds__(256) k_prolong_wide(Mesh m, int ncomp, const double *__restrict__ xc,
                                                      double *__restrict__ xf) {
    prolong_node(m, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, ncomp, xc, xf);
}
void prolong_wide_launch(const Mesh &m, int ncomp, const double *xc, double *xf, hipStream_t s) {
    k_prolong_wide<<<blocks_for((int64_t)ncomp * m.n_coarse, 256), 256, 0, s>>>(m, ncomp, xc, xf);
}


// --------------------------------------------------------- restriction ----
// bc(I) = sum over fine nodes i in {2I-1, 2I, 2I+1} (per axis) of
// w(i, I) bf(i), w = 1 at the coincident node and 1/2 at the two neighbours;
// absent neighbours (domain edge) get weight 0.  27 loads per component are
// issued together; FP64 accumulation.
__device__ __forceinline__ void restrict_node(const Mesh &m, int64_t t, int ncomp, const float *__restrict__ bf,
                                              double *__restrict__ bc) {
    // one thread per (component, coarse node): consecutive threads take
    // consecutive nodes of one component
    if (t >= (int64_t)ncomp * m.n_coarse) return;
    const int comp = (int)(t / m.n_coarse);
    t -= (int64_t)comp * m.n_coarse;
    uint32_t JK = fdiv((uint32_t)t, m.cx), I = (uint32_t)t - JK * m.nc[0];
    uint32_t K = fdiv(JK, m.cy), J = JK - K * m.nc[1];
    const int C[3] = {(int)I, (int)J, (int)K};
    int f[3][3];
    double w[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int fi = 2 * C[a] + d - 1;
            bool ok = true;
            if (m.per[a]) fi = wrap(fi, m.nf[a], 1);
            else if (fi < 0 || fi >= m.nf[a]) { ok = false; fi = 2 * C[a]; }
            f[a][d] = fi;
            w[a][d] = ok ? (d == 1 ? 1.0 : 0.5) : 0.0;
        }
    const float *b = bf + (int64_t)comp * m.n_fine;
    float v[27];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int bb = 0; bb < 3; ++bb)
#pragma unroll
            for (int a = 0; a < 3; ++a)
                v[a + 3 * bb + 9 * c] = b[f[0][a] + (int64_t)m.nf[0] * (f[1][bb] + (int64_t)m.nf[1] * f[2][c])];
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) {
            double row = w[0][0] * v[9 * c + 3 * bb] + w[0][1] * v[1 + 9 * c + 3 * bb] + w[0][2] * v[2 + 9 * c + 3 * bb];
            acc += w[1][bb] * w[2][c] * row;
        }
    bc[(int64_t)comp * m.n_coarse + t] = acc;
}

__global__ void __launch_bounds__(256) k_restrict(Mesh m, int ncomp, const float *__restrict__ bf,
                                                  double *__restrict__ bc) {
    restrict_node(m, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, ncomp, bf, bc);
}

__global__ void __launch_bounds__(256) k_restrict_batch(const BoxDesc *__restrict__ D, int nbox,
                                                        const float *__restrict__ bf, double *__restrict__ bc) {
    const int64_t blk = blockIdx.x;
    const int b = find_box(nbox, blk, [&](int i) { return D[i].blk_coarse; });
    const BoxDesc &d = D[b];
    const Mesh m = d.m;
    restrict_node(m, (blk - d.blk_coarse) * blockDim.x + threadIdx.x, 4, bf + 4 * d.off_fine,
                  bc + 4 * d.off_coarse);
}

// ----------------------------------------------------------- gather Q -----
// One thread writes 4 consecutive columns of a patch row.  Columns
// 27 c + iota (c < 6) read field c of [u, v, w, r_u, r_v, r_w] at
// dof(M, iota); 162..164 are the geometry inputs (row M of geom, or the
// coarse cell sizes when geom is null); the rest is zero padding.
template <int DT>
__global__ void __launch_bounds__(256)
    k_gather(Mesh m, const float *__restrict__ x, const float *__restrict__ r,
             const float *__restrict__ shift, const float *__restrict__ inv_scale, float qinv,
             void *__restrict__ Xout, int64_t ldx, const float *__restrict__ geom) {
    // block = GP patches x (ldx / 4) column quads
    const int quads = (int)(ldx / 4);
    const int local = threadIdx.x / quads;
    const int64_t M = (int64_t)blockIdx.x * (blockDim.x / quads) + local;
    if (local >= (int)(blockDim.x / quads) || M >= m.n_patches) return;
    const int col0 = (int)(threadIdx.x - local * quads) * 4;
    uint32_t J_K = fdiv((uint32_t)M, m.px), I = (uint32_t)M - J_K * m.n[0];
    uint32_t K = fdiv(J_K, m.py), J = J_K - K * m.n[1];
    // standardisation constants (clamped to the last input column) are
    // requested with the node values
    float sh[4], sc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int cc = col0 + q < 165 ? col0 + q : 164;
        sh[q] = shift ? shift[cc] : 0.0f;
        sc[q] = inv_scale ? inv_scale[cc] : 1.0f;
    }
    float z[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int col = col0 + q;
        float v = 0.0f;
        if (col < 162) {
            int c = col / 27, iota = col - 27 * c;
            int a = iota % 3, b = (iota / 3) % 3, cc = iota / 9;
            int i = wrap(2 * I + a, m.nf[0], m.per[0]);
            int j = wrap(2 * J + b, m.nf[1], m.per[1]);
            int k = wrap(2 * K + cc, m.nf[2], m.per[2]);
            int64_t node = i + (int64_t)m.nf[0] * (j + (int64_t)m.nf[1] * k);
            v = c < 3 ? x[c * m.n_fine + node] : r[(c - 3) * m.n_fine + node];
        } else if (col < 165) {
            v = geom ? geom[3 * M + (col - 162)] : m.H[col - 162];
        }
        if (col < 165) {
            if (shift) v -= sh[q];
            if (inv_scale) v *= sc[q];
        }
        z[q] = v;
    }
    if (DT == DNNMG_F32) {
        float4 o = make_float4(z[0], z[1], z[2], z[3]);
        *(float4 *)((float *)Xout + M * ldx + col0) = o;
    } else if (DT == DNNMG_BF16) {
        uint2 o;
        o.x = pack_bf16x2_hw(z[0], z[1]);
        o.y = pack_bf16x2_hw(z[2], z[3]);
        *(uint2 *)((uint16_t *)Xout + M * ldx + col0) = o;
    } else {
        uint32_t o = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) o |= (uint32_t)f32_to_e4m3(z[q] * qinv) << (8 * q);
        *(uint32_t *)((uint8_t *)Xout + M * ldx + col0) = o;
    }
}

// ----------------------------------------------------- extension L --------
// Per fine node: the patches holding it along each axis (ascending patch
// index, at most two) and the node's local coordinate in each; the mean of
// the network outputs over these patches.  The 2x2x2 candidate set is fixed
// (absent candidates carry weight 0) so all loads are issued at once.
__device__ __forceinline__ void scatter_node(const Mesh &m, int64_t t, const float *__restrict__ Y,
                                             const float *__restrict__ vbase, float *__restrict__ d) {
    if (t >= m.n_fine) return;
    uint32_t jk = fdiv((uint32_t)t, m.fx), i = (uint32_t)t - jk * m.nf[0];
    uint32_t k = fdiv(jk, m.fy), j = jk - k * m.nf[1];
    // the base field is requested with the network outputs (one round trip)
    float b[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (vbase)
#pragma unroll
        for (int c = 0; c < 4; ++c) b[c] = vbase[c * m.n_fine + t];
    float v[3];
    extension_at(m, (int)i, (int)j, (int)k, Y, v);
#pragma unroll
    for (int c = 0; c < 3; ++c) d[c * m.n_fine + t] = vbase ? v[c] + b[c] : v[c];
    // the network predicts no pressure correction: the corrected iterate
    // keeps the prolongated pressure
    if (vbase) d[3 * m.n_fine + t] = b[3];
}

__global__ void __launch_bounds__(256) k_scatter(Mesh m, const float *__restrict__ Y,
                                                 const float *__restrict__ vbase, float *__restrict__ d) {
    scatter_node(m, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, Y, vbase, d);
}

__global__ void __launch_bounds__(256) k_scatter_batch(const BoxDesc *__restrict__ D, int nbox,
                                                       const float *__restrict__ Y, const float *__restrict__ vbase,
                                                       float *__restrict__ xc) {
    const int64_t blk = blockIdx.x;
    const int b = find_box(nbox, blk, [&](int i) { return D[i].blk_fine; });
    const BoxDesc &dd = D[b];
    const Mesh m = dd.m;
    scatter_node(m, (blk - dd.blk_fine) * blockDim.x + threadIdx.x, Y + 81 * dd.off_patch,
                 vbase + 4 * dd.off_fine, xc + 4 * dd.off_fine);
}

// Tiled form of the same sums.  Patch outputs are stored patch by patch
// (81 floats each), so node-order reads of them touch one cache line per
// lane; a workgroup instead copies the patch rows its nodes need into LDS
// with contiguous reads (rows of consecutive x patches are adjacent in
// memory) and sums from there.  Tile = ST_X x ST_Y x ST_Z owned fine nodes;
// on a non-periodic axis the last tile also owns the final node 2n, so no
// tile is a one-node sliver.  Patch slot s along an axis holds patch
// b + s, b = first owned node / 2 - 1 (wrapped on a periodic axis).
constexpr int ST_X = 16, ST_Y = 8;
constexpr int SCATTER_TZ = 2, SCATTER_NT = 256; // the built tile depth and workgroup size
constexpr int SS_X = ST_X / 2 + 1, SS_Y = ST_Y / 2 + 1;
constexpr int SS_RUN = 81 * SS_X;                       // floats per run of x slots

// tiles along an axis with nf nodes: ceil(nf / T), less one where that
// would leave a single node to the last tile
__host__ __device__ inline int stiles_axis(int nf, int T) {
    int t = (nf + T - 1) / T;
    if (t > 1 && nf % T == 1) --t;
    return t;
}

// Holders of the node at local index l (global i) along one axis as
// (slot, local node, weight) in the ascending patch order of holders(); an
// absent second holder repeats the first with weight 0.
struct SHold {
    int s[2], loc[2];
    float w[2];
    int cnt;
};

__device__ __forceinline__ SHold stile_holders(int l, int i, int n, int per) {
    SHold h;
    const int lo_s = l >> 1, hi_s = lo_s + 1;
    if (i & 1) {
        h.s[0] = h.s[1] = hi_s;
        h.loc[0] = h.loc[1] = 1;
        h.w[0] = 1.f;
        h.w[1] = 0.f;
        h.cnt = 1;
        return h;
    }
    // periodic: the wrapped lower patch n - 1 comes last at i = 0
    const bool has_lo = per || i > 0, has_hi = per || i < 2 * n;
    const bool lo_first = has_lo && !(per && i == 0);
    h.s[0] = lo_first ? lo_s : hi_s;
    h.loc[0] = lo_first ? 2 : 0;
    h.s[1] = has_lo && has_hi ? (lo_first ? hi_s : lo_s) : h.s[0];
    h.loc[1] = has_lo && has_hi ? (lo_first ? 0 : 2) : h.loc[0];
    h.w[0] = 1.f;
    h.w[1] = has_lo && has_hi ? 1.f : 0.f;
    h.cnt = (int)has_lo + (int)has_hi;
    return h;
}

template <int ST_Z, int ST_NT>
__device__ __forceinline__ void scatter_tile(const Mesh &m, int tx, int ty, int tz, int gx, int gy, int gz,
                                             const float *__restrict__ Y, const float *__restrict__ vbase,
                                             float *__restrict__ d) {
    constexpr int SS_Z = ST_Z / 2 + 1;
    constexpr int SS_ITER = (SS_RUN + ST_NT - 1) / ST_NT;   // loads per thread per run
    __shared__ float sY[SS_Z * SS_Y * SS_RUN];
    const int tid = threadIdx.x;
    const int x0 = tx * ST_X, y0 = ty * ST_Y, z0 = tz * ST_Z;
    const int nx = (tx == gx - 1 ? m.nf[0] : x0 + ST_X) - x0;   // owned nodes per axis
    const int ny = (ty == gy - 1 ? m.nf[1] : y0 + ST_Y) - y0;
    const int nz = (tz == gz - 1 ? m.nf[2] : z0 + ST_Z) - z0;
    const int nn = nx * ny * nz;
    const bool full = nx == ST_X && ny == ST_Y && nz == ST_Z;
    const int bI = x0 / 2 - 1, bJ = y0 / 2 - 1, bK = z0 / 2 - 1;
    // node coordinates of this thread's passes, and their base field,
    // requested with the patch rows so the tile waits for memory once
    constexpr int NPASS = ((ST_X + 1) * (ST_Y + 1) * (ST_Z + 1) + ST_NT - 1) / ST_NT;
    int lx[NPASS], ly[NPASS], lz[NPASS];
    int64_t node[NPASS];
    float vb[NPASS][4];
#pragma unroll
    for (int p = 0; p < NPASS; ++p) {
        const int q = tid + p * ST_NT;
        if (full) {
            lx[p] = q % ST_X;
            ly[p] = (q / ST_X) % ST_Y;
            lz[p] = q / (ST_X * ST_Y);
        } else {
            lx[p] = q % nx;
            ly[p] = (q / nx) % ny;
            lz[p] = q / (nx * ny);
        }
        node[p] = x0 + lx[p] + (int64_t)m.nf[0] * (y0 + ly[p] + (int64_t)m.nf[1] * (z0 + lz[p]));
#pragma unroll
        for (int c = 0; c < 4; ++c) vb[p][c] = (vbase && q < nn) ? vbase[c * m.n_fine + node[p]] : 0.0f;
    }
    // stage: one run of SS_X consecutive x patches per (y, z) slot; patches
    // outside the mesh are zero (read only with weight 0).  Along x a run is
    // at most two contiguous stretches of patch rows: elements [e_lo, sp)
    // at row offset offA + e and, where a periodic run wraps, [sp, e_hi) at
    // offB + e.  Only a periodic axis of fewer than SS_X patches wraps more
    // than once; it takes the per-element form.  The two forms are separate
    // loops so each issues all its loads at once.
    float t[SS_Z * SS_Y][SS_ITER];
    auto run_ok = [&](int r, int64_t &row) {
        const int J = wrap(bJ + r % SS_Y, m.n[1], m.per[1]);
        const int K = wrap(bK + r / SS_Y, m.n[2], m.per[2]);
        row = (int64_t)m.n[0] * (J + (int64_t)m.n[1] * K);
        return J >= 0 && J < m.n[1] && K >= 0 && K < m.n[2];
    };
    const int n0 = m.n[0];
    int e_lo = 0, e_hi = SS_RUN, sp = SS_RUN;
    int64_t offA = (int64_t)bI * 81, offB = 0;
    const bool stretches = !m.per[0] || n0 >= SS_X;
    if (m.per[0]) {
        if (bI < 0) {                      // slot 0 is patch n0 - 1
            sp = 81;
            offA = (int64_t)(n0 - 1) * 81;
            offB = -81;
        } else if (bI + SS_X > n0) {       // slots from n0 - bI on are patches 0, 1, ..
            sp = (n0 - bI) * 81;
            offB = -(int64_t)sp;
        }
    } else {
        e_lo = (bI < 0 ? -bI : 0) * 81;
        e_hi = (n0 - bI < SS_X ? n0 - bI : SS_X) * 81;
    }
    if (stretches) {
#pragma unroll
        for (int r = 0; r < SS_Z * SS_Y; ++r) {
            int64_t row;
            const bool rok = run_ok(r, row);
            const float *rb = Y + row * 81;
#pragma unroll
            for (int u = 0; u < SS_ITER; ++u) {
                const int e = tid + u * ST_NT;
                t[r][u] = rok && e >= e_lo && e < e_hi ? rb[(e < sp ? offA : offB) + e] : 0.0f;
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < SS_Z * SS_Y; ++r) {
            int64_t row;
            const bool rok = run_ok(r, row);
#pragma unroll
            for (int u = 0; u < SS_ITER; ++u) {
                const int e = tid + u * ST_NT;
                const int sx = e / 81;
                const int I = wrap(bI + sx, m.n[0], m.per[0]);
                t[r][u] = 0.0f;
                if (rok && e < SS_RUN && I >= 0 && I < m.n[0]) t[r][u] = Y[(row + I) * 81 + (e - 81 * sx)];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < SS_Z * SS_Y; ++r)
#pragma unroll
        for (int u = 0; u < SS_ITER; ++u) {
            const int e = tid + u * ST_NT;
            if (e < SS_RUN) sY[r * SS_RUN + e] = t[r][u];
        }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < NPASS; ++p) {
        if (tid + p * ST_NT >= nn) break;
        const int i = x0 + lx[p], j = y0 + ly[p], k = z0 + lz[p];
        const SHold hx = stile_holders(lx[p], i, m.n[0], m.per[0]);
        const SHold hy = stile_holders(ly[p], j, m.n[1], m.per[1]);
        const SHold hz = stile_holders(lz[p], k, m.n[2], m.per[2]);
        // all 2 x 2 x 2 candidates, z, then y, then x, as extension_at
        float acc[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int rb = (hz.s[c] * SS_Y + hy.s[b]) * SS_RUN + 3 * hy.loc[b] + 9 * hz.loc[c];
                const float wbc = hy.w[b] * hz.w[c];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const float *src = sY + rb + 81 * hx.s[a] + hx.loc[a];
                    const float w = hx.w[a] * wbc;
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) acc[cc] = fmaf(w, src[27 * cc], acc[cc]);
                }
            }
        const float inv = 1.0f / (float)(hx.cnt * hy.cnt * hz.cnt); // power of two: exact
        const bool dir = on_dirichlet(m, i, j, k);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float v = dir ? 0.0f : acc[c] * inv;
            if (vbase) v += vb[p][c];
            d[c * m.n_fine + node[p]] = v;
        }
        if (vbase) d[3 * m.n_fine + node[p]] = vb[p][3];
    }
}

template <int ST_Z, int ST_NT>
__global__ void __launch_bounds__(ST_NT) k_scatter_tiled(Mesh m, int gx, int gy, int gz, const float *__restrict__ Y,
                                                         const float *__restrict__ vbase, float *__restrict__ d) {
    const int64_t t = xcd_item(blockIdx.x, gridDim.x);
    if (t >= (int64_t)gx * gy * gz) return;
    scatter_tile<ST_Z, ST_NT>(m, (int)(t % gx), (int)((t / gx) % gy), (int)(t / ((int64_t)gx * gy)), gx, gy, gz, Y,
                              vbase, d);
}

constexpr int NORM_BLOCKS = 1024;

// Batched tiled extension: one flat grid over the scatter tiles of all boxes
// (prefix sums blk_stile), in the XCD-contiguous order of the single box.
template <int ST_Z, int ST_NT>
__global__ void __launch_bounds__(ST_NT) k_scatter_tiled_batch(const BoxDesc *__restrict__ D, int nbox,
                                                               int64_t ntiles, const float *__restrict__ Y,
                                                               const float *__restrict__ vbase,
                                                               float *__restrict__ xc) {
    const int64_t t = xcd_item(blockIdx.x, gridDim.x);
    if (t >= ntiles) return;
    const int b = find_box(nbox, t, [&](int i) { return D[i].blk_stile; });
    const BoxDesc &dd = D[b];
    const Mesh m = dd.m;
    const int gx = stiles_axis(m.nf[0], ST_X), gy = stiles_axis(m.nf[1], ST_Y), gz = stiles_axis(m.nf[2], ST_Z);
    const int64_t l = t - dd.blk_stile;
    scatter_tile<ST_Z, ST_NT>(m, (int)(l % gx), (int)((l / gx) % gy), (int)(l / ((int64_t)gx * gy)), gx, gy, gz,
                              Y + 81 * dd.off_patch, vbase + 4 * dd.off_fine, xc + 4 * dd.off_fine);
}

// -------------------------------------------------------------- norms -----
// Block (x, y) sums vector y (a, or a1 for y = 1) over the grid-stride
// range of x; part[y][x].  Every vector is reduced over the same partition
// in the same order, whichever launch it is in.
__global__ void __launch_bounds__(256) k_norm_partial(int64_t n, const float *__restrict__ a,
                                                      const float *__restrict__ b,
                                                      const float *__restrict__ a1,
                                                      double *__restrict__ part) {
    if (blockIdx.y == 1) {
        a = a1;
        b = nullptr;
    }
    double s = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        double e = (double)a[t] - (b ? (double)b[t] : 0.0);
        s += e * e;
    }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// Block y sums part[y][0 .. nparts) into out[y].
__global__ void __launch_bounds__(256) k_norm_final(int nparts, const double *__restrict__ part,
                                                    double *__restrict__ out) {
    __shared__ double red[256];
    part += (int64_t)blockIdx.x * nparts;
    out += blockIdx.x;
    double s = 0.0;
    for (int t = threadIdx.x; t < nparts; t += 256) s += part[t];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// The tiled form wins once every compute unit has several tiles; on smaller
// meshes the per-node form (no staging round trip) is faster.
static bool scatter_prefers_tiles(int64_t n_fine) {
    return n_fine >= (int64_t)4 * device_cus() * ST_X * ST_Y * SCATTER_TZ;
}

void restrict_batch_launch(const BoxDesc *D, int nbox, int64_t nblk, const float *bf, double *bc, hipStream_t s) {
    k_restrict_batch<<<(unsigned)nblk, 256, 0, s>>>(D, nbox, bf, bc);
}
void scatter_batch_launch(const BoxDesc *D, int nbox, int64_t nblk, const float *Y, const float *vbase, float *xc,
                          hipStream_t s) {
    k_scatter_batch<<<(unsigned)nblk, 256, 0, s>>>(D, nbox, Y, vbase, xc);
}
// Extension tiles of one box (the tiled form's grid).
int64_t scatter_tiles(const Mesh &m) {
    return (int64_t)stiles_axis(m.nf[0], ST_X) * stiles_axis(m.nf[1], ST_Y) * stiles_axis(m.nf[2], SCATTER_TZ);
}
void scatter_tiled_batch_launch(const BoxDesc *D, int nbox, int64_t ntiles, const float *Y, const float *vbase,
                                float *xc, hipStream_t s) {
    k_scatter_tiled_batch<SCATTER_TZ, SCATTER_NT>
        <<<xcd_blocks(ntiles), SCATTER_NT, 0, s>>>(D, nbox, ntiles, Y, vbase, xc);
}


} // namespace dnnmg

using namespace dnnmg;

#define STREAM ((hipStream_t)stream)

extern "C" int dnnmg_patch_dofmap(const dnnmg_box *box, int32_t *map, uint8_t *mult, void *stream) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    if (!map && !mult) return fail(DNNMG_ERR_ARG, "dnnmg_patch_dofmap: map and mult are both NULL");
    if (map) k_dofmap<<<blocks_for(m.n_patches * 27, 256), 256, 0, STREAM>>>(m, map);
    if (mult) k_mult<<<blocks_for(m.n_fine, 256), 256, 0, STREAM>>>(m, mult);
    return hip_check(hipGetLastError(), "dnnmg_patch_dofmap launch");
}

extern "C" int dnnmg_prolong(const dnnmg_box *box, int ncomp, const double *xc, float *xf,
                             void *stream) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    if (ncomp < 1 || ncomp > 4) return fail(DNNMG_ERR_ARG, "dnnmg_prolong: ncomp %d not in 1..4", ncomp);
    if (!xc || !xf) return fail(DNNMG_ERR_ARG, "dnnmg_prolong: NULL pointer");
    k_prolong<<<blocks_for((int64_t)ncomp * m.n_coarse, 256), 256, 0, STREAM>>>(m, ncomp, xc, xf);
    return hip_check(hipGetLastError(), "dnnmg_prolong launch");
}

extern "C" int dnnmg_restrict(const dnnmg_box *box, int ncomp, const float *bf, double *bc,
                              void *stream) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    if (ncomp < 1 || ncomp > 4) return fail(DNNMG_ERR_ARG, "dnnmg_restrict: ncomp %d not in 1..4", ncomp);
    if (!bf || !bc) return fail(DNNMG_ERR_ARG, "dnnmg_restrict: NULL pointer");
    k_restrict<<<blocks_for((int64_t)ncomp * m.n_coarse, 256), 256, 0, STREAM>>>(m, ncomp, bf, bc);
    return hip_check(hipGetLastError(), "dnnmg_restrict launch");
}

static int gather_launch(const dnnmg_box *box, const float *geom, const float *x, const float *r,
                         const dnnmg_feat *feat, int dtype, float x_scale, void *X, int64_t ldx, void *stream) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    if (!x || !r || !X) return fail(DNNMG_ERR_ARG, "dnnmg_patch_gather: NULL pointer");
    if (!aligned16(X)) return fail(DNNMG_ERR_ARG, "dnnmg_patch_gather: X not 16-byte aligned");
    int align = dtype == DNNMG_F32 ? 4 : dtype == DNNMG_BF16 ? 8 : 16;
    if (ldx < 165 || ldx % align)
        return fail(DNNMG_ERR_SHAPE, "dnnmg_patch_gather: ldx %lld must be >= 165 and a multiple of %d",
                    (long long)ldx, align);
    const float *sh = feat ? feat->shift : nullptr;
    const float *sc = feat ? feat->inv_scale : nullptr;
    if (ldx / 4 > 256) return fail(DNNMG_ERR_SHAPE, "dnnmg_patch_gather: ldx %lld > 1024", (long long)ldx);
    int per_block = (int)(256 / (ldx / 4));
    unsigned g = blocks_for(m.n_patches, per_block);
    if (dtype == DNNMG_F32)
        k_gather<DNNMG_F32><<<g, 256, 0, STREAM>>>(m, x, r, sh, sc, 1.0f, X, ldx, geom);
    else if (dtype == DNNMG_BF16)
        k_gather<DNNMG_BF16><<<g, 256, 0, STREAM>>>(m, x, r, sh, sc, 1.0f, X, ldx, geom);
    else if (dtype == DNNMG_FP8_E4M3) {
        if (!(x_scale > 0.0f)) return fail(DNNMG_ERR_ARG, "dnnmg_patch_gather: x_scale must be > 0 for FP8");
        k_gather<DNNMG_FP8_E4M3><<<g, 256, 0, STREAM>>>(m, x, r, sh, sc, 1.0f / x_scale, X, ldx, geom);
    } else
        return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_patch_gather: dtype %d", dtype);
    return hip_check(hipGetLastError(), "dnnmg_patch_gather launch");
}

extern "C" int dnnmg_patch_gather(const dnnmg_box *box, const float *x, const float *r,
                                  const dnnmg_feat *feat, int dtype, float x_scale, void *X,
                                  int64_t ldx, void *stream) {
    return gather_launch(box, nullptr, x, r, feat, dtype, x_scale, X, ldx, stream);
}

extern "C" int dnnmg_patch_gather_geom(const dnnmg_box *box, const float *geom, const float *x, const float *r,
                                       const dnnmg_feat *feat, int dtype, float x_scale, void *X, int64_t ldx,
                                       void *stream) {
    if (!geom) return fail(DNNMG_ERR_ARG, "dnnmg_patch_gather_geom: geom is NULL");
    return gather_launch(box, geom, x, r, feat, dtype, x_scale, X, ldx, stream);
}

// The tiled form wins once every compute unit has several tiles; on smaller
// meshes the per-node form (no staging round trip) is faster.

static bool scatter_prefers_tiles(const Mesh &m) { return scatter_prefers_tiles(m.n_fine); }

extern "C" int dnnmg_scatter_avg_form(const dnnmg_box *box, const float *Y, const float *vbase, float *d, int form,
                                      void *stream) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    if (!Y || !d) return fail(DNNMG_ERR_ARG, "dnnmg_scatter_avg: NULL pointer");
    if (form < DNNMG_SCATTER_AUTO || form > DNNMG_SCATTER_TILED)
        return fail(DNNMG_ERR_ARG, "dnnmg_scatter_avg_form: unknown form %d", form);
    if (form == DNNMG_SCATTER_AUTO) form = scatter_prefers_tiles(m) ? DNNMG_SCATTER_TILED : DNNMG_SCATTER_NODES;
    if (form == DNNMG_SCATTER_TILED) {
        const int gx = stiles_axis(m.nf[0], ST_X), gy = stiles_axis(m.nf[1], ST_Y);
        const int gz = stiles_axis(m.nf[2], SCATTER_TZ);
        k_scatter_tiled<SCATTER_TZ, SCATTER_NT>
            <<<xcd_blocks((int64_t)gx * gy * gz), SCATTER_NT, 0, STREAM>>>(m, gx, gy, gz, Y, vbase, d);
    } else {
        k_scatter<<<blocks_for(m.n_fine, 256), 256, 0, STREAM>>>(m, Y, vbase, d);
    }
    return hip_check(hipGetLastError(), "dnnmg_scatter_avg launch");
}

extern "C" int dnnmg_scatter_avg(const dnnmg_box *box, const float *Y, const float *vbase, float *d,
                                 void *stream) {
    return dnnmg_scatter_avg_form(box, Y, vbase, d, DNNMG_SCATTER_AUTO, stream);
}

extern "C" size_t dnnmg_norm2_workspace(void) { return NORM_BLOCKS * sizeof(double); }

extern "C" int dnnmg_norm2_f64(int64_t n, const float *a, const float *b, double *out, void *ws,
                               size_t ws_bytes, void *stream) {
    if (n < 0) return fail(DNNMG_ERR_SHAPE, "dnnmg_norm2_f64: n < 0");
    if (!a || !out || !ws) return fail(DNNMG_ERR_ARG, "dnnmg_norm2_f64: NULL pointer");
    if (ws_bytes < dnnmg_norm2_workspace())
        return fail(DNNMG_ERR_SHAPE, "dnnmg_norm2_f64: workspace %zu < %zu bytes", ws_bytes,
                    dnnmg_norm2_workspace());
    k_norm_partial<<<NORM_BLOCKS, 256, 0, STREAM>>>(n, a, b, nullptr, (double *)ws);
    k_norm_final<<<1, 256, 0, STREAM>>>(NORM_BLOCKS, (const double *)ws, out);
    return hip_check(hipGetLastError(), "dnnmg_norm2_f64 launch");
}

extern "C" int dnnmg_norm2_pair_f64(int64_t n, const float *a0, const float *a1, double *out, void *ws,
                                    size_t ws_bytes, void *stream) {
    if (n < 0) return fail(DNNMG_ERR_SHAPE, "dnnmg_norm2_pair_f64: n < 0");
    if (!a0 || !a1 || !out || !ws) return fail(DNNMG_ERR_ARG, "dnnmg_norm2_pair_f64: NULL pointer");
    if (ws_bytes < 2 * dnnmg_norm2_workspace())
        return fail(DNNMG_ERR_SHAPE, "dnnmg_norm2_pair_f64: workspace %zu < %zu bytes", ws_bytes,
                    2 * dnnmg_norm2_workspace());
    k_norm_partial<<<dim3(NORM_BLOCKS, 2), 256, 0, STREAM>>>(n, a0, nullptr, a1, (double *)ws);
    k_norm_final<<<2, 256, 0, STREAM>>>(NORM_BLOCKS, (const double *)ws, out);
    return hip_check(hipGetLastError(), "dnnmg_norm2_pair_f64 launch");
}
