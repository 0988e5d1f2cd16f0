// Error state, mesh validation and small host utilities of libdnnmg.
#include <stdarg.h>
#include <stdio.h>

#include "common.hpp"

namespace dnnmg {

static thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return DNNMG_OK;
    return fail(DNNMG_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

FastDiv make_fastdiv(uint32_t d) {
    FastDiv f;
    f.d = d;
    uint32_t s = 0;
    while ((1ull << s) < d) ++s;
    f.s = s;
    f.m = (uint32_t)(((1ull << 32) * ((1ull << s) - d)) / d + 1);
    return f;
}

int make_mesh(const dnnmg_box *box, Mesh *m) {
    if (!box) return fail(DNNMG_ERR_ARG, "box is NULL");
    int64_t nf = 1, nc = 1, np = 1;
    for (int a = 0; a < 3; ++a) {
        int per = (box->periodic_mask >> a) & 1u;
        if (box->n[a] < 1) return fail(DNNMG_ERR_SHAPE, "n[%d] = %d < 1", a, box->n[a]);
        if (per && (box->n[a] < 2 || (box->n[a] & 1)))
            return fail(DNNMG_ERR_SHAPE, "periodic axis %d needs an even n >= 2 (got %d)", a,
                        box->n[a]);
        if (!(box->len[a] > 0.0)) return fail(DNNMG_ERR_SHAPE, "len[%d] must be > 0", a);
        m->n[a] = box->n[a];
        m->per[a] = per;
        m->nf[a] = per ? 2 * box->n[a] : 2 * box->n[a] + 1;
        m->nc[a] = per ? box->n[a] : box->n[a] + 1;
        m->hd[a] = box->len[a] / (2.0 * box->n[a]);
        m->h[a] = (float)m->hd[a];
        m->H[a] = (float)(box->len[a] / box->n[a]);
        nf *= m->nf[a];
        nc *= m->nc[a];
        np *= box->n[a];
    }
    if (nf >= (1ll << 31) || np * 27 >= (1ll << 31))
        return fail(DNNMG_ERR_SHAPE, "mesh too large for 32-bit node indices");
    m->dmask = box->dirichlet_mask;
    m->n_fine = nf;
    m->n_coarse = nc;
    m->n_patches = np;
    m->fx = make_fastdiv(m->nf[0]);
    m->fy = make_fastdiv(m->nf[1]);
    m->cx = make_fastdiv(m->nc[0]);
    m->cy = make_fastdiv(m->nc[1]);
    m->px = make_fastdiv(m->n[0]);
    m->py = make_fastdiv(m->n[1]);
    return DNNMG_OK;
}

} // namespace dnnmg

using namespace dnnmg;

extern "C" int dnnmg_version(void) { return 1; }

extern "C" const char *dnnmg_last_error(void) { return g_last_error.c_str(); }

extern "C" int dnnmg_box_sizes(const dnnmg_box *box, int64_t *n_fine, int64_t *n_coarse,
                               int64_t *n_patches) {
    Mesh m;
    int rc = make_mesh(box, &m);
    if (rc) return rc;
    if (n_fine) *n_fine = m.n_fine;
    if (n_coarse) *n_coarse = m.n_coarse;
    if (n_patches) *n_patches = m.n_patches;
    return DNNMG_OK;
}
