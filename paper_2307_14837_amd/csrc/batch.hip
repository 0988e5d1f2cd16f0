// Batched correction step over many independent boxes of uneven size, with a
// launch plan and an autotuner.  The per-box field blocks are concatenated
// (BoxDesc); one step is five kernel launches whatever the number of boxes:
//   prolongation fused with the residual, fused gather + network
//   (persistent: blocks walk the patch tiles of all boxes), extension
//   (v~ + d, per node or in LDS-staged tiles), right-hand side, restriction.
// The plan keeps the layout, the launch geometry and the tuned choices of
// the network stage (patches per workgroup tile, persistent grid size) and
// of the extension (per node or tiled).
#include <vector>

#include "common.hpp"
#include "mlp.hpp"

namespace dnnmg {

ResParams make_params(const Mesh &m, const dnnmg_ns *ns);
void residual_tiles(const Mesh &m, int rt[3], int rf[3]);
void prolong_residual_batch_launch(const BoxDesc *D, int nbox, int64_t nfull, int64_t npart, const double *xc,
                                   const float *vp, float *xt, float *r, hipStream_t s);
void restrict_batch_launch(const BoxDesc *D, int nbox, int64_t nblk, const float *bf, double *bc, hipStream_t s);
void rhs_batch_launch(const BoxDesc *D, int nbox, int64_t nfull, int64_t npart, const float *v, float *b,
                      hipStream_t s);
void prolong_residual_b_batch_launch(const BoxDesc *D, int nbox, int64_t nfull, int64_t npart, const double *xc,
                                     const float *b, float *xt, float *r, hipStream_t s);
void scatter_batch_launch(const BoxDesc *D, int nbox, int64_t nblk, const float *Y, const float *vbase, float *xc,
                          hipStream_t s);
int64_t scatter_tiles(const Mesh &m);
void scatter_tiled_batch_launch(const BoxDesc *D, int nbox, int64_t ntiles, const float *Y, const float *vbase,
                                float *xc, hipStream_t s);

} // namespace dnnmg

using namespace dnnmg;

struct dnnmg_plan {
    int nbox;
    dnnmg_ns ns;
    std::vector<BoxDesc> desc;
    BoxDesc *d_desc;   // in the caller's workspace
    int64_t n_fine, n_coarse, n_patches;
    int64_t blk_fine, blk_coarse, tiles_full, tiles_part, ptiles, stiles;
    int pt;            // tuned: patches per network tile / 16
    int grid;          // tuned: persistent grid of the network stage (0 = one block per tile)
    int scatter_form;  // tuned: extension per node or in LDS-staged tiles (DNNMG_SCATTER_*)
};

static size_t up256(size_t b) { return (b + 255) / 256 * 256; }

static int layout(dnnmg_plan *p, const dnnmg_box *boxes, int nbox) {
    p->desc.resize(nbox);
    int64_t of = 0, oc = 0, op = 0, bf = 0, bc = 0, bt = 0, bpart = 0, bp = 0, bs = 0;
    for (int i = 0; i < nbox; ++i) {
        BoxDesc &d = p->desc[i];
        int rc = make_mesh(&boxes[i], &d.m);
        if (rc) return rc;
        d.rp = make_params(d.m, &p->ns);
        int rt[3], rf[3];
        residual_tiles(d.m, rt, rf);
        for (int a = 0; a < 3; ++a) {
            d.rtiles[a] = rt[a];
            d.rfull[a] = rf[a];
        }
        d.off_fine = of;
        d.off_coarse = oc;
        d.off_patch = op;
        d.blk_fine = bf;
        d.blk_coarse = bc;
        d.blk_full = bt;
        d.blk_part = bpart;
        d.blk_ptile = bp;
        d.blk_stile = bs;
        of += d.m.n_fine;
        oc += d.m.n_coarse;
        op += d.m.n_patches;
        bf += (d.m.n_fine + 255) / 256;
        bc += (4 * d.m.n_coarse + 255) / 256; // restriction: one thread per component and node
        const int64_t nfull = (int64_t)rf[0] * rf[1] * rf[2];
        bt += nfull;
        bpart += (int64_t)rt[0] * rt[1] * rt[2] - nfull;
        bp += (d.m.n_patches + 16 * p->pt - 1) / (16 * p->pt);
        bs += scatter_tiles(d.m);
    }
    p->n_fine = of;
    p->n_coarse = oc;
    p->n_patches = op;
    p->blk_fine = bf;
    p->blk_coarse = bc;
    p->tiles_full = bt;
    p->tiles_part = bpart;
    p->ptiles = bp;
    p->stiles = bs;
    return DNNMG_OK;
}

static int upload(dnnmg_plan *p, hipStream_t s) {
    return hip_check(hipMemcpyAsync(p->d_desc, p->desc.data(), sizeof(BoxDesc) * p->nbox, hipMemcpyHostToDevice, s),
                     "plan upload");
}

extern "C" size_t dnnmg_plan_workspace(const dnnmg_box *boxes, int nbox) {
    if (!boxes || nbox < 1) return 0;
    for (int i = 0; i < nbox; ++i) {
        Mesh m;
        if (make_mesh(&boxes[i], &m)) return 0;
    }
    return up256(sizeof(BoxDesc) * nbox);
}

extern "C" int dnnmg_plan_create(const dnnmg_box *boxes, int nbox, const dnnmg_ns *ns, void *ws, size_t ws_bytes,
                                 dnnmg_plan **out, void *stream) {
    if (!boxes || nbox < 1 || !ns || !ws || !out) return fail(DNNMG_ERR_ARG, "dnnmg_plan_create: bad argument");
    if (!(ns->dt > 0.0)) return fail(DNNMG_ERR_ARG, "dnnmg_plan_create: dt must be > 0");
    size_t need = dnnmg_plan_workspace(boxes, nbox);
    if (need == 0) return fail(DNNMG_ERR_SHAPE, "dnnmg_plan_create: invalid box");
    if (ws_bytes < need) return fail(DNNMG_ERR_SHAPE, "dnnmg_plan_create: workspace %zu < %zu bytes", ws_bytes, need);
    dnnmg_plan *p = new dnnmg_plan();
    p->nbox = nbox;
    p->ns = *ns;
    p->pt = 2; // instantiated for every network; the autotuner may change it
    p->grid = 0;
    p->scatter_form = DNNMG_SCATTER_TILED;
    int rc = layout(p, boxes, nbox);
    if (rc) {
        delete p;
        return rc;
    }
    p->d_desc = (BoxDesc *)ws;
    if ((rc = upload(p, (hipStream_t)stream))) {
        delete p;
        return rc;
    }
    *out = p;
    return DNNMG_OK;
}

extern "C" int dnnmg_plan_destroy(dnnmg_plan *p) {
    delete p;
    return DNNMG_OK;
}

extern "C" int dnnmg_plan_sizes(const dnnmg_plan *p, int64_t *n_fine, int64_t *n_coarse, int64_t *n_patches) {
    if (!p) return fail(DNNMG_ERR_ARG, "dnnmg_plan_sizes: plan is NULL");
    if (n_fine) *n_fine = p->n_fine;
    if (n_coarse) *n_coarse = p->n_coarse;
    if (n_patches) *n_patches = p->n_patches;
    return DNNMG_OK;
}

extern "C" int dnnmg_plan_choice(const dnnmg_plan *p, int *patches_per_tile, int *grid) {
    if (!p) return fail(DNNMG_ERR_ARG, "dnnmg_plan_choice: plan is NULL");
    if (patches_per_tile) *patches_per_tile = 16 * p->pt;
    if (grid) *grid = p->grid;
    return DNNMG_OK;
}

extern "C" int dnnmg_plan_scatter_form(const dnnmg_plan *p, int *form) {
    if (!p || !form) return fail(DNNMG_ERR_ARG, "dnnmg_plan_scatter_form: NULL argument");
    *form = p->scatter_form;
    return DNNMG_OK;
}

extern "C" int dnnmg_plan_set_scatter_form(dnnmg_plan *p, int form) {
    if (!p) return fail(DNNMG_ERR_ARG, "dnnmg_plan_set_scatter_form: plan is NULL");
    if (form != DNNMG_SCATTER_NODES && form != DNNMG_SCATTER_TILED)
        return fail(DNNMG_ERR_ARG, "dnnmg_plan_set_scatter_form: form %d is neither nodes nor tiled", form);
    p->scatter_form = form;
    return DNNMG_OK;
}

static void scatter_stage(const dnnmg_plan *p, int form, const float *Y, const float *xt, float *xcorr,
                          hipStream_t s) {
    if (form == DNNMG_SCATTER_TILED) scatter_tiled_batch_launch(p->d_desc, p->nbox, p->stiles, Y, xt, xcorr, s);
    else scatter_batch_launch(p->d_desc, p->nbox, p->blk_fine, Y, xt, xcorr, s);
}

// vprev == NULL: b holds the previous step's right-hand side on entry and
// the residual is r = b - A(x~); b is then overwritten with the new one.
static int step_impl(const dnnmg_plan *p, const dnnmg_mlp *net, const float *shift, const float *inv,
                     const double *xc, const float *vprev, float *xt, float *r, float *Y, float *xcorr, float *b,
                     double *bc, hipStream_t s) {
    const BoxDesc *D = p->d_desc;
    if (vprev) prolong_residual_batch_launch(D, p->nbox, p->tiles_full, p->tiles_part, xc, vprev, xt, r, s);
    else prolong_residual_b_batch_launch(D, p->nbox, p->tiles_full, p->tiles_part, xc, b, xt, r, s);
    BoxDesc none{};
    int rc = fwd_launch(net, p->pt, true, p->ptiles, p->grid, 0, nullptr, 0, D, p->nbox, none, xt, r, shift, inv,
                        Y, nullptr, s);
    if (rc) return rc;
    scatter_stage(p, p->scatter_form, Y, xt, xcorr, s);
    rhs_batch_launch(D, p->nbox, p->tiles_full, p->tiles_part, xcorr, b, s);
    restrict_batch_launch(D, p->nbox, p->blk_coarse, b, bc, s);
    return hip_check(hipGetLastError(), "dnnmg_batch_step launch");
}

static int check_step(const dnnmg_plan *p, const dnnmg_mlp *net, const double *xc, const float *vprev, float *xt,
                      float *r, float *Y, float *xcorr, float *b, double *bc) {
    if (!p) return fail(DNNMG_ERR_ARG, "batch step: plan is NULL");
    int rc = check_net(net);
    if (rc) return rc;
    if (!xc || !vprev || !xt || !r || !Y || !xcorr || !b || !bc)
        return fail(DNNMG_ERR_ARG, "batch step: NULL buffer");
    return DNNMG_OK;
}

extern "C" int dnnmg_batch_step(const dnnmg_plan *p, const dnnmg_mlp *net, const float *shift,
                                const float *inv_scale, const double *xc, const float *vprev, float *xt, float *r,
                                float *Y, float *xcorr, float *b, double *bc, void *stream) {
    int rc = check_step(p, net, xc, vprev, xt, r, Y, xcorr, b, bc);
    if (rc) return rc;
    return step_impl(p, net, shift, inv_scale, xc, vprev, xt, r, Y, xcorr, b, bc, (hipStream_t)stream);
}

extern "C" int dnnmg_batch_step_b(const dnnmg_plan *p, const dnnmg_mlp *net, const float *shift,
                                  const float *inv_scale, const double *xc, float *b, float *xt, float *r, float *Y,
                                  float *xcorr, double *bc, void *stream) {
    if (!b) return fail(DNNMG_ERR_ARG, "batch step: NULL buffer");
    int rc = check_step(p, net, xc, b, xt, r, Y, xcorr, b, bc);
    if (rc) return rc;
    if (b == r || b == xt || b == xcorr) return fail(DNNMG_ERR_ARG, "dnnmg_batch_step_b: b overlaps an output");
    return step_impl(p, net, shift, inv_scale, xc, nullptr, xt, r, Y, xcorr, b, bc, (hipStream_t)stream);
}

extern "C" int dnnmg_batch_rhs(const dnnmg_plan *p, const float *v, float *b, void *stream) {
    if (!p || !v || !b) return fail(DNNMG_ERR_ARG, "dnnmg_batch_rhs: NULL argument");
    rhs_batch_launch(p->d_desc, p->nbox, p->tiles_full, p->tiles_part, v, b, (hipStream_t)stream);
    return hip_check(hipGetLastError(), "dnnmg_batch_rhs launch");
}

extern "C" int dnnmg_plan_autotune(dnnmg_plan *p, const dnnmg_mlp *net, const float *shift, const float *inv_scale,
                                   const double *xc, const float *vprev, float *xt, float *r, float *Y, float *xcorr,
                                   float *b, double *bc, int reps, void *stream) {
    int rc = check_step(p, net, xc, vprev, xt, r, Y, xcorr, b, bc);
    if (rc) return rc;
    if (reps < 1) reps = 1;
    hipStream_t s = (hipStream_t)stream;
    // inputs of the network stage
    prolong_residual_batch_launch(p->d_desc, p->nbox, p->tiles_full, p->tiles_part, xc, vprev, xt, r, s);
    int dev = 0, ncu = 256;
    if ((rc = hip_check(hipGetDevice(&dev), "autotune device"))) return rc;
    if ((rc = hip_check(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev), "autotune CU count")))
        return rc;
    hipEvent_t e0, e1;
    if ((rc = hip_check(hipEventCreate(&e0), "autotune event"))) return rc;
    if ((rc = hip_check(hipEventCreate(&e1), "autotune event"))) {
        (void)hipEventDestroy(e0);
        return rc;
    }
    float best = 1e30f;
    int best_pt = p->pt, best_grid = p->grid;
    auto set_pt = [&](int pt) {
        p->pt = pt;
        int64_t bp = 0;
        for (auto &d : p->desc) {
            d.blk_ptile = bp;
            bp += (d.m.n_patches + 16 * pt - 1) / (16 * pt);
        }
        p->ptiles = bp;
        // the host table is rewritten for the next candidate: finish the copy
        int e = upload(p, s);
        return e ? e : hip_check(hipStreamSynchronize(s), "autotune upload");
    };
    const int pts[3] = {1, 2, 4};
    for (int pi = 0; pi < 3 && !rc; ++pi) {
        const int pt = pts[pi];
        if (!fwd_has_pt(net, pt)) continue;
        if ((rc = set_pt(pt))) break;
        const int grids[4] = {0, ncu, 2 * ncu, 4 * ncu};
        for (int gi = 0; gi < 4 && !rc; ++gi) {
            int grid = grids[gi];
            if (grid >= p->ptiles) continue;
            BoxDesc none{};
            auto launch = [&]() {
                return fwd_launch(net, pt, true, p->ptiles, grid, 0, nullptr, 0, p->d_desc, p->nbox, none, xt, r,
                                  shift, inv_scale, Y, nullptr, s);
            };
            if ((rc = launch())) break;
            if ((rc = hip_check(hipEventRecord(e0, s), "autotune event record"))) break;
            for (int k = 0; k < reps && !rc; ++k) rc = launch();
            if (rc) break;
            if ((rc = hip_check(hipEventRecord(e1, s), "autotune event record"))) break;
            if ((rc = hip_check(hipEventSynchronize(e1), "autotune launch"))) break;
            float ms = 0.f;
            if ((rc = hip_check(hipEventElapsedTime(&ms, e0, e1), "autotune timing"))) break;
            if (ms < best) {
                best = ms;
                best_pt = pt;
                best_grid = grid;
            }
        }
    }
    p->grid = best_grid;
    if (!rc) rc = set_pt(best_pt);
    // the extension stage: per node or in tiles, on the network's outputs
    float best_s = 1e30f;
    int best_form = p->scatter_form;
    const int forms[2] = {DNNMG_SCATTER_NODES, DNNMG_SCATTER_TILED};
    for (int fi = 0; fi < 2 && !rc; ++fi) {
        scatter_stage(p, forms[fi], Y, xt, xcorr, s);
        if ((rc = hip_check(hipEventRecord(e0, s), "autotune event record"))) break;
        for (int k = 0; k < reps; ++k) scatter_stage(p, forms[fi], Y, xt, xcorr, s);
        if ((rc = hip_check(hipEventRecord(e1, s), "autotune event record"))) break;
        if ((rc = hip_check(hipEventSynchronize(e1), "autotune launch"))) break;
        float ms = 0.f;
        if ((rc = hip_check(hipEventElapsedTime(&ms, e0, e1), "autotune timing"))) break;
        if (ms < best_s) {
            best_s = ms;
            best_form = forms[fi];
        }
    }
    p->scatter_form = best_form;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!rc) rc = hip_check(hipStreamSynchronize(s), "autotune sync");
    return rc;
}
