/*
 * dnnmg.h - C ABI of the MI355X (gfx950) DNN-MG fine-level correction library.
 *
 * The library evaluates the per-time-step correction of DNN-MG (arXiv
 * 2307.14837, Algorithm 1, the steps after the coarse Newton solve):
 *   prolongate the coarse solution one level      dnnmg_prolong
 *   fine Crank-Nicolson residual                  dnnmg_residual
 *   gather patch inputs (operator Q)              dnnmg_patch_gather
 *   patch network forward / backward              dnnmg_patch_forward / _backward
 *   multiplicity-averaged extension (operator L)  dnnmg_scatter_avg
 *   right-hand side for the next step             dnnmg_rhs
 *   restriction of that rhs to the coarse level   dnnmg_restrict
 * plus the index maps, FP64 norms for the residual indicator, the AdamW
 * update and weight packing for the network.
 *
 * Conventions for every entry point
 *   - Return value: DNNMG_OK (0) or a negative DNNMG_ERR_* code;
 *     dnnmg_last_error() returns a message for the calling thread.
 *   - All arguments are validated on the host before anything is enqueued,
 *     so an error leaves no partial work on the stream.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = legacy default
 *     stream).  No call synchronises, allocates device memory or keeps a
 *     pointer after it returns.  The caller owns every buffer.
 *   - Device pointers must be 16-byte aligned unless stated otherwise.
 *   - Mesh: a box [0,len0]x[0,len1]x[0,len2] with n[a] coarse cells per axis;
 *     the fine mesh has 2 n[a] cells per axis.  Nodes per axis: 2n (fine) /
 *     n (coarse) on periodic axes, 2n+1 / n+1 otherwise.  Node index
 *     i + Nx (j + Ny k).  Fields are SoA [component][node] (u, v, w, p).
 *   - Patch M = coarse cell (I,J,K), M = I + n0 (J + n1 K); its 27 local
 *     nodes are iota = a + 3b + 9c, fine node (2I+a, 2J+b, 2K+c) (Sec. 4.2).
 *   - Periodic axes need an even n >= 2.
 */
#ifndef DNNMG_H
#define DNNMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DNNMG_OK 0
#define DNNMG_ERR_ARG (-1)         /* null or misaligned pointer, bad scalar */
#define DNNMG_ERR_SHAPE (-2)       /* mesh, width, leading dimension or size */
#define DNNMG_ERR_UNSUPPORTED (-3) /* dtype or width not built */
#define DNNMG_ERR_HIP (-4)         /* a HIP runtime call or launch failed */

/* Mesh.  dirichlet_mask bit 2a = low face of axis a carries Dirichlet velocity
 * data, bit 2a+1 = high face; faces without the bit are do-nothing (natural)
 * boundaries.  Bits on periodic axes are ignored. */
typedef struct dnnmg_box {
    int32_t n[3];
    double len[3];
    uint32_t periodic_mask;
    uint32_t dirichlet_mask;
} dnnmg_box;

/* Crank-Nicolson step and stabilisation parameters, eq. (stabparams):
 * alpha_T = alpha0 / (nu/h_T^2 + |v|_inf,T / h_T + 1/dt), delta_T likewise. */
typedef struct dnnmg_ns {
    double nu, dt, alpha0, delta0;
} dnnmg_ns;

/* Network element types */
#define DNNMG_F32 0
#define DNNMG_BF16 1
#define DNNMG_FP8_E4M3 2 /* OCP E4M3FN, max 448, saturating */

/* Patch network 165 -> H -> H -> 81 with tanh (Sec. 3; width H in
 * {64,128,256,512}; 753 -> H -> H -> 375 for the two-level prediction, see
 * dnnmg_mlp_prepare_io).  W[l] are packed by dnnmg_mlp_pack; b[l] are FP32
 * biases (length H, H, 81).  Products accumulate in FP32 and bias and tanh are
 * applied in FP32.  Element types per layer (1, 2, 3):
 *   DNNMG_F32       FP32, FP32, FP32   (inputs X FP32)
 *   DNNMG_BF16      BF16, BF16, BF16   (inputs X BF16)
 *   DNNMG_FP8_E4M3  BF16, FP8,  BF16   (inputs X BF16; H >= 128): the H x H
 *                   product runs in OCP E4M3 with per-tensor scales, W2 =
 *                   W2q * w_scale[1] and layer-2 inputs a = aq * a_scale[1];
 *                   the other scales are ignored. */
typedef struct dnnmg_mlp {
    int32_t n_in;  /* 165 (or 753, two-level prediction) */
    int32_t hidden;
    int32_t n_out; /* 81 (or 375) */
    int32_t dtype; /* DNNMG_F32 | DNNMG_BF16 | DNNMG_FP8_E4M3 */
    const void *W[3];
    const float *b[3];
    float w_scale[3];
    float a_scale[3];
} dnnmg_mlp;

/* Per-feature standardisation of the 165 network inputs, z = (X - shift) *
 * inv_scale, applied by the gather (device arrays of 165 floats; NULL =
 * identity). */
typedef struct dnnmg_feat {
    const float *shift;
    const float *inv_scale;
} dnnmg_feat;

int dnnmg_version(void);
const char *dnnmg_last_error(void);

/* Host-only size queries.  Any output pointer may be NULL. */
int dnnmg_box_sizes(const dnnmg_box *box, int64_t *n_fine, int64_t *n_coarse,
                    int64_t *n_patches);

/* dof(P_M, iota) and valence (Sec. 4.2, the dof map and the vector mu of the
 * extension operator).  map: int32 [n_patches][27] fine node indices;
 * mult: uint8 [n_fine], number of patches holding each node (1, 2, 4 or 8). */
int dnnmg_patch_dofmap(const dnnmg_box *box, int32_t *map, uint8_t *mult, void *stream);

/* Prolongation of Algorithm 1: Q1 interpolation of the coarse solution onto
 * the fine mesh.  xc: FP64 [ncomp][n_coarse]; xf: FP32 [ncomp][n_fine];
 * 1 <= ncomp <= 4.  The coarse values are rounded to FP32 and averaged axis
 * by axis in FP32 (the patch interpolant of the residual kernel, so the LPS
 * terms of a prolongated field vanish exactly).  xc and xf must not overlap. */
int dnnmg_prolong(const dnnmg_box *box, int ncomp, const double *xc, float *xf, void *stream);

/* Fine residual of Algorithm 1, r = F - A(x), for the Crank-Nicolson system
 * (4cranknicholson3) with the two-level local projection stabilisation of
 * eq. (disc:ns) (projection onto the Q1 space of each patch).
 *   x     FP32 [4][n_fine]  current iterate (u, v, w, p)
 *   vprev FP32 [3][n_fine]  velocity of the previous step (builds F)
 *   fmid  FP32 [3][n_fine]  (f_{n-1} + f_n) / 2, or NULL for no forcing
 *   r     FP32 [4][n_fine]  output; velocity rows on Dirichlet faces are 0
 *   ws    device workspace of at least dnnmg_residual_workspace(box) bytes,
 *         16-byte aligned (per-patch LPS corner sums and per-tile flags)
 * Element integrals use 2x2x2 Gauss points on every fine cell. */
size_t dnnmg_residual_workspace(const dnnmg_box *box);
int dnnmg_residual(const dnnmg_box *box, const dnnmg_ns *ns, const float *x, const float *vprev,
                   const float *fmid, float *r, void *ws, size_t ws_bytes, void *stream);

/* The same residual against a given right-hand side (Algorithm 1: the fine
 * Rhs of the previous step): r = b - A(x), A holding the terms of eq.
 * (4cranknicholson3) and the LPS terms of eq. (disc:ns) that depend on the
 * iterate x (see dnnmg_prolong_residual_b).  With b = dnnmg_rhs(vprev, fmid)
 * it equals dnnmg_residual up to FP32 rounding.
 *   x FP32 [4][n_fine]; b FP32 [4][n_fine]; r FP32 [4][n_fine] output (r == b
 *   is DNNMG_ERR_ARG); ws as for dnnmg_residual. */
int dnnmg_residual_b(const dnnmg_box *box, const dnnmg_ns *ns, const float *x, const float *b, float *r, void *ws,
                     size_t ws_bytes, void *stream);

/* The indicator's residual and the next right-hand side in one pass
 * (Algorithm 1: the residual of the corrected iterate, then Rhs of its
 * velocity, both at x): r = b - A(x) as dnnmg_residual_b computes it, and b
 * is replaced by dnnmg_rhs(x's velocity, NULL) (up to FP32 rounding order)
 * in place.  Each node's b is read before it is overwritten.  b_save, if
 * not NULL, receives b as it was on entry (the right-hand side a fallback
 * of this step still needs).
 *   x FP32 [4][n_fine]; b FP32 [4][n_fine] in/out; r FP32 [4][n_fine]
 *   output; b_save FP32 [4][n_fine] output or NULL; x, b, r and b_save must
 *   not alias (DNNMG_ERR_ARG); ws as for dnnmg_residual. */
int dnnmg_residual_rhs_b(const dnnmg_box *box, const dnnmg_ns *ns, const float *x, float *b, float *r, float *b_save,
                         void *ws, size_t ws_bytes, void *stream);

/* dnnmg_residual_b for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and the same results, bit for bit, with the LPS workspace taken
 * from a device array of DNNMG_NOALLOC_SCRATCH_BYTES built into the library
 * (one per GPU, held until the process ends) instead of a caller workspace.
 * Makes no allocation of any kind.  A box needing more than the built-in
 * size (dnnmg_residual_workspace(box) > DNNMG_NOALLOC_SCRATCH_BYTES, about
 * 270,000 patches) is DNNMG_ERR_SHAPE.  All calls on one GPU share its
 * array: calls that may overlap on one GPU (other streams, other threads)
 * race and must be ordered by the caller.  The first call on a device looks
 * up the array's address (a host-side query, no allocation); call it once
 * outside capture before capturing it in a graph. */
#define DNNMG_NOALLOC_SCRATCH_BYTES (33u << 20)
int dnnmg_residual_b_noalloc(const dnnmg_box *box, const dnnmg_ns *ns, const float *x, const float *b, float *r,
                             void *stream);

/* Prolongation and fine residual fused (Algorithm 1): xt = P xc exactly as
 * dnnmg_prolong computes it (ncomp 4), and r = F - A(xt) as dnnmg_residual
 * computes it, bit for bit, in one pass.  Since xt is patchwise Q1 (the Q1
 * interpolant of the coarse solution on every patch), the local projection
 * terms of eq. (disc:ns) vanish identically and are not evaluated, so no
 * workspace is needed.
 *   xc FP64 [4][n_coarse]; vprev FP32 [3][n_fine]; fmid FP32 [3][n_fine] or
 *   NULL; xt FP32 [4][n_fine] and r FP32 [4][n_fine] outputs (must not
 *   overlap the inputs). */
int dnnmg_prolong_residual(const dnnmg_box *box, const dnnmg_ns *ns, const double *xc, const float *vprev,
                           const float *fmid, float *xt, float *r, void *stream);

/* The same fused pass against a given right-hand side (Algorithm 1: the fine
 * Rhs of the previous step feeds the next step's residual):
 *   xt = P xc (as dnnmg_prolong) and r = b - A(xt),
 * where A(x) holds the terms of eq. (4cranknicholson3) that depend on the
 * new iterate: (1/k) M v + 1/2 N(v) + nu/2 K v - (p, div phi) for the
 * momentum rows and (div v, xi) for the continuity row.  With b =
 * dnnmg_rhs(vprev, fmid) this is the residual dnnmg_prolong_residual
 * computes (same terms, summed as b plus the new-iterate part, so equal up
 * to FP32 rounding); in a time loop b is the previous step's Rhs output, so
 * the terms of the previous velocity are not evaluated twice.
 *   xc FP64 [4][n_coarse]; b FP32 [4][n_fine] (pressure row added as given,
 *   0 from dnnmg_rhs); xt and r FP32 [4][n_fine] outputs, not overlapping
 *   the inputs (r == b is DNNMG_ERR_ARG).  Velocity rows of r on Dirichlet
 *   faces are 0. */
int dnnmg_prolong_residual_b(const dnnmg_box *box, const dnnmg_ns *ns, const double *xc, const float *b, float *xt,
                             float *r, void *stream);

/* Right-hand side of (4cranknicholson3) for the next step (Algorithm 1,
 * "Rhs"): b_a = (1/k)(v_a, phi) - 1/2 (v.grad v_a, phi) - nu/2 (grad v_a,
 * grad phi) + (fmid_a, phi); pressure rows 0; Dirichlet velocity rows 0.
 *   v FP32 [3][n_fine]; fmid FP32 [3][n_fine] = (f_n + f_{n+1})/2 or NULL;
 *   b FP32 [4][n_fine]. */
int dnnmg_rhs(const dnnmg_box *box, const dnnmg_ns *ns, const float *v, const float *fmid,
              float *b, void *stream);

/* dnnmg_rhs predicated on a device flag (Algorithm 1: the right-hand side of
 * the velocity the fallback produced): computes b = Rhs(v, fmid) when *flag
 * != 0 at run time and leaves b untouched otherwise, so a graph holds it
 * unconditionally.  flag: device int (e.g. dnnmg_fallback's flag_out),
 * required; other arguments as for dnnmg_rhs. */
int dnnmg_rhs_if(const dnnmg_box *box, const dnnmg_ns *ns, const float *v, const float *fmid, float *b,
                 const int *flag, void *stream);


/* Restriction of Algorithm 1: bc = P^T bf, the transpose of dnnmg_prolong,
 * accumulated and stored in FP64.  bf: FP32 [ncomp][n_fine];
 * bc: FP64 [ncomp][n_coarse]. */
int dnnmg_restrict(const dnnmg_box *box, int ncomp, const float *bf, double *bc, void *stream);

/* Operator Q of eq. (defQ) applied to the prolongated solution and to the
 * residual, plus the coarse cell sizes (the geometry inputs of Sec. 4.2):
 * row M = [u(dof(M,0..26)), v(..), w(..), r_u(..), r_v(..), r_w(..), H0, H1,
 * H2], standardised by `feat` and stored as `dtype` in X [n_patches][ldx]
 * (ldx >= 165; columns 165..ldx-1 are written as zero).  For FP8 the stored
 * value is round_e4m3(z / x_scale) (x_scale = the network's a_scale[0]);
 * otherwise x_scale is ignored.  x: FP32 [>=3][n_fine]; r: FP32 [>=3][n_fine]. */
int dnnmg_patch_gather(const dnnmg_box *box, const float *x, const float *r, const dnnmg_feat *feat,
                       int dtype, float x_scale, void *X, int64_t ldx, void *stream);

/* Packed weight layout used by the network kernels.  dnnmg_mlp_packed_bytes
 * gives the size for layer `layer` (0, 1, 2) of a width-`hidden` network of
 * element type dtype; dnnmg_mlp_pack converts an FP32 row-major
 * [fan_in][fan_out] matrix W (device) into it (FP8: Wq = round(W / w_scale)). */
size_t dnnmg_mlp_packed_bytes(int dtype, int hidden, int layer);
int dnnmg_mlp_pack(int dtype, int hidden, int layer, const float *W, float w_scale, void *Wp,
                   void *stream);

/* Setup of a network for the kernels (Sec. 3 network; the per-tensor
 * scaling of the FP8 precision scheme): packs the three FP32 layers W[l]
 * (device, row-major [fan_in][fan_out]: 165 x H, H x H, H x 81) into Wp[l]
 * (device, dnnmg_mlp_packed_bytes(dtype, hidden, l) bytes each, 16-byte
 * aligned), chooses the scales and fills *net (n_in, hidden, n_out, dtype,
 * W = Wp, b = b, w_scale, a_scale).  Scales: FP8 networks get w_scale[1] =
 * max |W2| / 448 (the amax taken on the device, so W2 / w_scale spans the
 * E4M3 range) and a_scale[1] = 1 / 448 for the tanh outputs entering the
 * E4M3 product (|tanh| < 1); every other scale is 1.  b[l]: FP32 biases
 * (device, H, H, 81).  ws: device workspace of at least 256 bytes.  A setup
 * call: it synchronises `stream` (the FP8 scale is read back into *net).
 * A non-finite or zero max |W2| of an FP8 network is DNNMG_ERR_ARG. */
int dnnmg_mlp_prepare(int dtype, int hidden, const float *const W[3], const float *const b[3], void *const Wp[3],
                      void *ws, size_t ws_bytes, dnnmg_mlp *net, void *stream);

/* Patch network N applied to every row of X (Sec. 4.2, patch-wise
 * prediction): Y = W3^T tanh(W2^T tanh(W1^T x + b1) + b2) + b3, FP32
 * accumulation, FP32 outputs Y [n][81].  X has the network's dtype and
 * leading dimension ldx >= 165 (padding columns must be zero).  If `saved` is
 * not NULL the hidden activations are stored for dnnmg_patch_backward:
 * bf16 [2][n][hidden] for BF16, fp32 [2][n][hidden] for F32 (FP8 does not
 * save).  n may be 0. */
int dnnmg_patch_forward(const dnnmg_mlp *net, int64_t n, const void *X, int64_t ldx, float *Y,
                        void *saved, void *stream);
/* dnnmg_patch_forward with an explicit launch geometry, for tuning: each
 * workgroup takes tiles of tile_patches rows (16, 32 or 64 as built for the
 * network's type and width; 0 = the library's choice) and the grid has
 * `grid` workgroups walking the tiles (0 = one workgroup per tile).
 * DNNMG_ERR_UNSUPPORTED for a tile size not built. */
int dnnmg_patch_forward_tiles(const dnnmg_mlp *net, int64_t n, const void *X, int64_t ldx, float *Y,
                              void *saved, int tile_patches, int grid, void *stream);
size_t dnnmg_patch_saved_bytes(const dnnmg_mlp *net, int64_t n);

/* Training objective of Sec. 4.2 restricted to patches: loss = (1/n) sum_M
 * ||Y_M - T_M||^2.  Writes its gradient dY = 2 (Y - T) / n (FP32 [n][81]);
 * the loss itself is dnnmg_norm2_f64(Y, T) / n. */
int dnnmg_mse_grad(int64_t n, const float *Y, const float *T, float *dY, void *stream);

/* dnnmg_mse_grad with the loss in the same pass (Sec. 4.2 training
 * objective): dY as dnnmg_mse_grad, and *loss_sum (FP64, device) = sum of
 * (Y - T)^2 over the n x 81 outputs, the value dnnmg_norm2_f64(Y, T) gives
 * (same partition and summation order).  ws: device workspace of at least
 * dnnmg_norm2_workspace() bytes.  n = 0 gives loss_sum = 0. */
int dnnmg_mse_grad_loss(int64_t n, const float *Y, const float *T, float *dY, double *loss_sum, void *ws,
                        size_t ws_bytes, void *stream);

/* Gradients of sum_M <dY_M, Y_M> with respect to the network parameters
 * (chain rule through both tanh layers; the input gradient is not formed),
 * for F32 or BF16 networks.  net gives dtype and width; W2 and W3 are the FP32
 * master weights of layers 2 and 3 (row-major [fan_in][fan_out]); X and ldx
 * are the forward's inputs and `saved` its activations.  dW[l] (FP32
 * row-major [fan_in][fan_out]) and db[l] are overwritten.  Products run on
 * the network's own element type (BF16 MFMA with operands rounded to BF16
 * for a BF16 network, FP32 MFMA for an F32 network), always with FP32
 * accumulation; sums over patches are split into fixed ranges and added in a
 * fixed order (deterministic).  ws: device workspace of
 * dnnmg_patch_backward_workspace(net, n) bytes. */
size_t dnnmg_patch_backward_workspace(const dnnmg_mlp *net, int64_t n);
int dnnmg_patch_backward(const dnnmg_mlp *net, const float *W2, const float *W3, int64_t n,
                         const void *X, int64_t ldx, const void *saved, const float *dY,
                         float *dW[3], float *db[3], void *ws, size_t ws_bytes, void *stream);

/* AdamW step (Sec. 3), t >= 1, in place on FP32 master weights theta and
 * moments m, v (n elements, gradient g):
 *   m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 *   theta -= lr wd theta + lr (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps). */
int dnnmg_adamw_step(int64_t n, float *theta, float *m, float *v, const float *g, float lr,
                     float b1, float b2, float eps, float wd, int64_t t, void *stream);

/* Extension L of eq. (defL): d = mu (.) sum_M L(Y[M], P_M), mu = 1/valence,
 * computed per fine node as a gather over the patches holding it, in
 * ascending patch order (deterministic, no atomics).  Y FP32 [n_patches][81]
 * (component-major per patch); Dirichlet velocity nodes get no correction.
 * vbase == NULL: d FP32 [3][n_fine] receives the correction.
 * vbase != NULL: vbase FP32 [4][n_fine] is the prolongated iterate (v~, p~)
 * and d FP32 [4][n_fine] receives the corrected iterate (v~ + L(Y), p~); the
 * network gives no pressure correction (Sec. 4.2). */
int dnnmg_scatter_avg(const dnnmg_box *box, const float *Y, const float *vbase, float *d,
                      void *stream);

/* dnnmg_scatter_avg with the kernel form chosen by the caller (the results
 * are bit for bit the same):
 *   DNNMG_SCATTER_NODES  one thread per fine node reading the patch rows
 *                        directly (fastest while the mesh gives each compute
 *                        unit little work);
 *   DNNMG_SCATTER_TILED  workgroups over 16 x 8 x 2 node tiles that first
 *                        copy the patch rows they need into LDS with
 *                        contiguous reads (fastest on large meshes);
 *   DNNMG_SCATTER_AUTO   the choice dnnmg_scatter_avg makes: tiled once the
 *                        fine mesh has at least 4 x (compute units) x 256
 *                        nodes.
 * Any other form is DNNMG_ERR_ARG. */
enum { DNNMG_SCATTER_AUTO = 0, DNNMG_SCATTER_NODES = 1, DNNMG_SCATTER_TILED = 2 };
int dnnmg_scatter_avg_form(const dnnmg_box *box, const float *Y, const float *vbase, float *d, int form,
                           void *stream);

/* Squared Euclidean norm in FP64 of a (or of a - b if b != NULL) over n
 * FP32 elements, written to *out (device).  Used for the residual indicator
 * eta = ||r(v~ + d)|| / ||r(v~)||.  Fixed-order two-level reduction
 * (deterministic); ws: device workspace of dnnmg_norm2_workspace() bytes. */
size_t dnnmg_norm2_workspace(void);
int dnnmg_norm2_f64(int64_t n, const float *a, const float *b, double *out, void *ws,
                    size_t ws_bytes, void *stream);

/* Both squared norms of the residual indicator in one pass: out[0] =
 * ||a0||^2, out[1] = ||a1||^2 (FP64, device), each bit for bit what
 * dnnmg_norm2_f64 gives for that vector alone (same partition, same order).
 * ws: device workspace of 2 * dnnmg_norm2_workspace() bytes. */
int dnnmg_norm2_pair_f64(int64_t n, const float *a0, const float *a1, double *out, void *ws, size_t ws_bytes,
                         void *stream);

/* Plain fine-level correction used by the residual-indicator fallback:
 * `sweeps` additive patch sweeps with the local problems of the Vanka
 * smoother (Sec. 2.4) on the patches of Sec. 4.2, in place on x FP32
 * [4][n_fine]:  r = F - A(x) (as dnnmg_residual, with vprev and fmid); on
 * every patch solve its local problem; x += omega * mu (.) sum_P L(delta_P)
 * (the averaging of eq. (defL)).  The local matrix A_P is the operator
 * linearised at the current velocity with frozen convection, restricted to
 * the patch's 108 unknowns (Galerkin terms of the 64 cells touching the
 * patch, pressure stabilisation of its own 8 cells); Dirichlet velocities
 * stay fixed.
 *   coupled = 0: momentum equations with the pressure held,
 *                K_P delta_a = r_a per velocity component (the fallback);
 *   coupled = 1: the full 108 x 108 velocity-pressure local systems.
 * ws: device workspace of dnnmg_vanka_workspace(box) bytes. */
size_t dnnmg_vanka_workspace(const dnnmg_box *box);
int dnnmg_vanka_sweeps(const dnnmg_box *box, const dnnmg_ns *ns, float *x, const float *vprev,
                       const float *fmid, int sweeps, float omega, int coupled, void *ws,
                       size_t ws_bytes, void *stream);

/* Residual-indicator fallback (taken on the device, no host synchronisation):
 * norms = {||r(x~)||^2, ||r(x_corr)||^2} (device FP64, from dnnmg_norm2_f64).
 * If eta = ||r(x_corr)|| / ||r(x~)|| exceeds theta (or is NaN), x_corr FP32
 * [4][n_fine] is replaced by `sweeps` pressure-held sweeps of
 * dnnmg_vanka_sweeps started from x~; otherwise x_corr is left as it is and
 * the launched kernels exit at once.  theta = +inf never falls back (only the
 * indicator is evaluated); with ||r(x~)|| = 0 the fallback is taken only if
 * ||r(x_corr)|| is not 0 as well (0/0 counts as eta = 0).  flag_out (device int, optional)
 * receives 1 when the fallback was taken.  ws: dnnmg_fallback_workspace(box)
 * bytes. */
size_t dnnmg_fallback_workspace(const dnnmg_box *box);
int dnnmg_fallback(const dnnmg_box *box, const dnnmg_ns *ns, const float *xt, const float *vprev,
                   const float *fmid, const double *norms, double theta, int sweeps, float omega,
                   float *xcorr, int *flag_out, void *ws, size_t ws_bytes, void *stream);

/* The fallback against a given right-hand side: as dnnmg_fallback with every
 * residual of the sweeps computed as dnnmg_residual_b(x, b) (b: FP32
 * [4][n_fine], the Rhs of the previous step; must not alias x_corr). */
int dnnmg_fallback_b(const dnnmg_box *box, const dnnmg_ns *ns, const float *xt, const float *b, const double *norms,
                     double theta, int sweeps, float omega, float *xcorr, int *flag_out, void *ws, size_t ws_bytes,
                     void *stream);

/* Operators Q and N fused (eqs. defQ and NN): the network's first-layer
 * inputs are built in on-chip memory from x~ (FP32 [4][n_fine]) and r (FP32
 * [4][n_fine]) with the standardisation `feat`, so the gathered batch is
 * never stored; Y FP32 [n_patches][81].  Same arithmetic as
 * dnnmg_patch_gather followed by dnnmg_patch_forward (every network
 * dnnmg_patch_forward takes). */
int dnnmg_patch_gather_forward(const dnnmg_box *box, const dnnmg_mlp *net, const float *xt, const float *r,
                               const dnnmg_feat *feat, float *Y, void *stream);

/* Batch of independent boxes (same dnnmg_ns and network, uneven sizes).
 * Field arrays of a batch concatenate the boxes' SoA blocks in box order:
 * box b's fine field with c components starts at c * (sum of n_fine of the
 * boxes before b), coarse fields likewise, patch rows at the patch prefix.
 * The plan holds the layout and launch geometry (host memory); its device
 * descriptor table lives in the caller's workspace (dnnmg_plan_workspace
 * bytes, kept alive with the plan) and is uploaded on `stream`. */
typedef struct dnnmg_plan dnnmg_plan;
size_t dnnmg_plan_workspace(const dnnmg_box *boxes, int nbox);
int dnnmg_plan_create(const dnnmg_box *boxes, int nbox, const dnnmg_ns *ns, void *ws, size_t ws_bytes,
                      dnnmg_plan **plan, void *stream);
int dnnmg_plan_destroy(dnnmg_plan *plan);
int dnnmg_plan_sizes(const dnnmg_plan *plan, int64_t *n_fine, int64_t *n_coarse, int64_t *n_patches);
/* Choice of the network stage: patches per workgroup tile (16, 32 or 64;
 * 32 until tuned) and the persistent grid size (0 = one workgroup per tile). */
int dnnmg_plan_choice(const dnnmg_plan *plan, int *patches_per_tile, int *grid);

/* Form of the plan's extension stage (eq. defL; the same sums in either
 * form, bit for bit): DNNMG_SCATTER_NODES (one thread per fine node) or
 * DNNMG_SCATTER_TILED (workgroups over the extension tiles of all boxes,
 * patch rows staged in LDS; the default until tuned).  *form receives it;
 * the setter fixes it (any other value: DNNMG_ERR_ARG). */
int dnnmg_plan_scatter_form(const dnnmg_plan *plan, int *form);
int dnnmg_plan_set_scatter_form(dnnmg_plan *plan, int form);

/* One correction step (Algorithm 1 after the coarse solve) for every box of
 * the plan in five kernel launches, independent of the number of boxes (not
 * one fused launch): prolongation fused with the residual (as
 * dnnmg_prolong_residual), gather + network in one persistent launch over
 * the patch tiles of all boxes, extension giving the corrected iterate
 * (v~ + d, p~; per node or tiled, dnnmg_plan_scatter_form), right-hand
 * side, restriction (FP64).
 * Buffers (batch layout): xc FP64 [4 comps], vprev FP32 [3], xt, r, xcorr,
 * b FP32 [4], Y FP32 [patches][81], bc FP64 [4].  No forcing.  The step can
 * be captured in a HIP graph. */
int dnnmg_batch_step(const dnnmg_plan *plan, const dnnmg_mlp *net, const float *shift, const float *inv_scale,
                     const double *xc, const float *vprev, float *xt, float *r, float *Y, float *xcorr,
                     float *b, double *bc, void *stream);

/* The batched step against the previous step's right-hand side (as
 * dnnmg_prolong_residual_b): on entry b FP32 [4] (batch layout) holds the
 * Rhs the previous step left; the step computes r = b - A(x~), ..., then
 * overwrites b with the new Rhs and restricts it to bc.  b must not overlap
 * xt, r, Y, xcorr or bc.  Same launches as dnnmg_batch_step. */
int dnnmg_batch_step_b(const dnnmg_plan *plan, const dnnmg_mlp *net, const float *shift, const float *inv_scale,
                       const double *xc, float *b, float *xt, float *r, float *Y, float *xcorr, double *bc,
                       void *stream);

/* Right-hand side (as dnnmg_rhs, no forcing) of every box of the plan, in one
 * launch: v FP32 [3 or 4] and b FP32 [4] in the batch layout.  Starts a time
 * loop run with dnnmg_batch_step_b from a given previous velocity. */
int dnnmg_batch_rhs(const dnnmg_plan *plan, const float *v, float *b, void *stream);
/* Autotuner (setup call, synchronises the stream): times the network stage
 * on the batch's own inputs for every candidate (16, 32 or 64 patches per
 * workgroup tile, as built for the network's type and width; one workgroup
 * per tile or a persistent grid of 1, 2 or 4 workgroups per compute unit)
 * with `reps` launches each, and keeps the fastest; then times the
 * extension stage in both forms (per node, tiled) on the network's outputs
 * and keeps the faster.  Overwrites xt, r, Y and xcorr. */
int dnnmg_plan_autotune(dnnmg_plan *plan, const dnnmg_mlp *net, const float *shift, const float *inv_scale,
                        const double *xc, const float *vprev, float *xt, float *r, float *Y, float *xcorr,
                        float *b, double *bc, int reps, void *stream);

/* Prediction J levels above the coarse mesh (Sec. 4.2; J = `levels`, 1 or 2):
 * the network corrects the solution on level L + J, whose mesh has 2^J n
 * cells per axis; a patch is one coarse cell with 2^J x 2^J x 2^J fine cells
 * and (2^J + 1)^3 nodes, local node iota = a + (2^J+1) b + (2^J+1)^2 c, fine
 * node (2^J I + a, 2^J J + b, 2^J K + c).  `box` is always the coarse box (n
 * cells); the fine fields live on the level-(L + J) lattice (node counts
 * from dnnmg_level_sizes).  The residual, Rhs, norms and fallback of level
 * L + J are the one-level calls on the box with 2^(J-1) n cells (their local
 * projection is onto the next-coarser level, independent of J).  levels = 1
 * is the same as the one-level calls.  J = 2: 125 nodes, network inputs 753
 * = 375 velocities + 375 momentum residuals + 3 cell sizes (ldx >= 753), 375
 * outputs. */
int dnnmg_level_sizes(const dnnmg_box *box, int levels, int64_t *n_fine, int64_t *n_coarse, int64_t *n_patches);
/* map int32 [n_patches][(2^J+1)^3]; mult uint8 [n_fine(L+J)] (1, 2, 4 or 8). */
int dnnmg_patch_dofmap_levels(const dnnmg_box *box, int levels, int32_t *map, uint8_t *mult, void *stream);
/* Prolongation L -> L + J (Algorithm 1), J times the one-level prolongation:
 * xc FP64 [ncomp][n_coarse] -> xf FP32 [ncomp][n_fine(L+J)].  The values are
 * those of dnnmg_prolong applied level by level in FP32, bit for bit, so the
 * result equals its own patch interpolant on level L + J - 1 exactly. */
int dnnmg_prolong_levels(const dnnmg_box *box, int levels, int ncomp, const double *xc, float *xf, void *stream);
/* Its transpose (restriction of the rhs, Algorithm 1), FP64 accumulation:
 * bf FP32 [ncomp][n_fine(L+J)] -> bc FP64 [ncomp][n_coarse]. */
int dnnmg_restrict_levels(const dnnmg_box *box, int levels, int ncomp, const float *bf, double *bc, void *stream);

/* Prolongation J levels up fused with the residual of level L + J against a
 * given right-hand side (Algorithm 1, the fine residual at x~ = P^J x^L;
 * Sec. 4.2 for J): xt = dnnmg_prolong_levels(xc) bit for bit and
 * r = b - A(xt) with A the new-iterate terms of eq. (4cranknicholson3), as
 * dnnmg_prolong_residual_b on the box of level L + J.  The local projection
 * terms of eq. (disc:ns) project onto level L + J - 1, of which xt is the
 * patchwise Q1 interpolant, so they vanish and are not evaluated.  J = 1 is
 * dnnmg_prolong_residual_b (ws unused, may be NULL).  J = 2 first writes
 * level L + 1 (FP32 values, widened to FP64) to ws, then runs the one-level
 * pass on the doubled box.
 *   xc FP64 [4][n_coarse]; b, xt, r FP32 [4][n_fine of level L + J];
 *   ws device, 16-byte aligned, dnnmg_prolong_residual_b_levels_workspace()
 *   bytes (0 for J = 1; 0 also for an invalid box or J); b == r is
 *   DNNMG_ERR_ARG, a short workspace DNNMG_ERR_SHAPE. */
size_t dnnmg_prolong_residual_b_levels_workspace(const dnnmg_box *box, int levels);
int dnnmg_prolong_residual_b_levels(const dnnmg_box *box, int levels, const dnnmg_ns *ns, const double *xc,
                                    const float *b, float *xt, float *r, void *ws, size_t ws_bytes, void *stream);
/* Operator Q of eq. (defQ) on the J-level patches: row M = [u(nodes), v, w,
 * r_u, r_v, r_w, H0, H1, H2] standardised by `feat` (device arrays of
 * 6 (2^J+1)^3 + 3 floats or NULL), FP32 or BF16, X [n_patches][ldx]
 * (padding columns zero). */
int dnnmg_patch_gather_levels(const dnnmg_box *box, int levels, const float *x, const float *r,
                              const dnnmg_feat *feat, int dtype, void *X, int64_t ldx, void *stream);
/* Extension L of eq. (defL) on the J-level patches: Y FP32 [n_patches][3
 * (2^J+1)^3]; vbase / d as for dnnmg_scatter_avg, on the level-(L + J)
 * lattice. */
int dnnmg_scatter_avg_levels(const dnnmg_box *box, int levels, const float *Y, const float *vbase, float *d,
                             void *stream);
/* Packing and setup of networks of either width pair (n_in, n_out) = (165,
 * 81) or (753, 375) (J = 1 or 2); dnnmg_mlp_packed_bytes / _pack / _prepare
 * are these with (165, 81).  dnnmg_patch_forward takes either network (the
 * J = 2 one as FP32, BF16 or FP8 rows, widths 256 and 512 as built);
 * dnnmg_patch_gather_forward and the backward are built for J = 1. */
size_t dnnmg_mlp_packed_bytes_io(int dtype, int n_in, int hidden, int n_out, int layer);
int dnnmg_mlp_pack_io(int dtype, int n_in, int hidden, int n_out, int layer, const float *W, float w_scale,
                      void *Wp, void *stream);
int dnnmg_mlp_prepare_io(int dtype, int n_in, int hidden, int n_out, const float *const W[3],
                         const float *const b[3], void *const Wp[3], void *ws, size_t ws_bytes, dnnmg_mlp *net,
                         void *stream);

/* The paper's network form (Sec. 3; widths and depth of Sec. 5.3): D hidden
 * layers of width H (512 or 750) without biases, batch normalisation
 * N_i(z) = (z - mu_i) / s_i * gamma_i + beta_i before each tanh, and skip
 * connections where the widths match:
 *   f_1(x) = tanh(N_1(W_1 x)),  f_i(x) = tanh(N_i(W_i x)) + x (i = 2..D),
 *   Y = W_{D+1} f_D(...),
 * on the inputs of Sec. 4.2 (dnnmg_patch_gather_paper): 240 -> 81 for
 * one-level patches, 1024 -> 375 for the two-level ones.  Inference only:
 * mu_i and s_i are the statistics of a trained network, and the setup folds
 * each normalisation into its layer (weights times gamma / s per output
 * unit, bias beta - gamma mu / s), the widths padded for the matrix cores
 * (dnnmg_deepnet_widths: inputs 256 / 1024, hidden 512 / 768, outputs 96 /
 * 384; padding units have zero weights and biases, so their activations are
 * exactly 0).  FP32 or BF16 (BF16 operands and activations, FP32
 * accumulation, bias, tanh and skip additions). */
#define DNNMG_DEEP_MAX_DEPTH 16
typedef struct dnnmg_deepnet {
    int32_t n_in, hidden, n_out, depth, dtype;
    const void *W[DNNMG_DEEP_MAX_DEPTH + 1];  /* packed layers 0..depth (device) */
    const float *b[DNNMG_DEEP_MAX_DEPTH + 1]; /* folded biases (device; the last is zero) */
} dnnmg_deepnet;
/* Padded widths of a (n_in, hidden, n_out) network; any output may be NULL. */
int dnnmg_deepnet_widths(int n_in, int hidden, int n_out, int *in_pad, int *hidden_pad, int *out_pad);
/* Bytes of packed layer `layer` (0..depth). */
size_t dnnmg_deepnet_packed_bytes(int dtype, int n_in, int hidden, int n_out, int depth, int layer);
/* Setup (enqueued on `stream`, no synchronisation): W[l] FP32 row-major
 * [fan_in][fan_out] for l = 0..depth; gamma[l], beta[l], mean[l], sd[l] FP32
 * [hidden] for l = 0..depth-1 (sd > 0); Wp[l] (dnnmg_deepnet_packed_bytes)
 * and bias[l] (hidden_pad floats, out_pad for l = depth) receive the folded
 * layers; ws: device workspace of hidden_pad floats; *net is filled. */
int dnnmg_deepnet_prepare(int dtype, int n_in, int hidden, int n_out, int depth, const float *const W[],
                          const float *const gamma[], const float *const beta[], const float *const mean[],
                          const float *const sd[], void *const Wp[], float *const bias[], void *ws, size_t ws_bytes,
                          dnnmg_deepnet *net, void *stream);
/* Y FP32 [n][n_out] = the network on the rows of X [n][ldx] (FP32 for FP32
 * networks, BF16 otherwise; ldx >= in_pad, padding columns zero). */
int dnnmg_deepnet_forward(const dnnmg_deepnet *net, int64_t n, const void *X, int64_t ldx, float *Y, void *stream);
/* The inputs of the paper's form (Sec. 4.2) on the J-level patches: row M =
 * [u, v, w, p at the (2^J+1)^3 patch nodes, r_u, r_v, r_w, r_p there, the 12
 * edge lengths of the coarse cell (x-directed, then y, then z), its 4
 * diagonals, and at its 8 vertices the mean of the 3 angles between the
 * faces meeting there (pi/2 on these axis-parallel cells)], standardised by
 * `feat` (8 (2^J+1)^3 + 24 floats or NULL), FP32 or BF16, X [n_patches][ldx]
 * (ldx >= 240 / 1024; padding columns zero).  x, r: FP32 [4][n_fine(L+J)]. */
int dnnmg_patch_gather_paper(const dnnmg_box *box, int levels, const float *x, const float *r,
                             const dnnmg_feat *feat, int dtype, void *X, int64_t ldx, void *stream);

/* HIP-graph capture of library calls (Algorithm 1 as one replayable time
 * step).  dnnmg_graph_capture_begin starts capturing `stream` (a non-default
 * stream that is not already capturing; thread-local capture mode); every
 * library call enqueued on it until dnnmg_graph_capture_end is recorded
 * instead of run.  dnnmg_graph_capture_end stops the capture and
 * instantiates the executable graph into *graph (owned by the caller, freed
 * by dnnmg_graph_destroy); it must be called even when a call in between
 * failed, and then returns that failure and no graph.  dnnmg_graph_replay
 * launches the graph on `stream`: the recorded kernels run again on the
 * buffers they were recorded with, whose current contents they read.  No
 * recorded call allocates or sets memory with a runtime memset, so replays
 * are repeatable.  Begin, end and destroy are setup calls (end allocates the
 * graph's host-side description); replay does not synchronise. */
typedef struct dnnmg_graph dnnmg_graph;
int dnnmg_graph_capture_begin(void *stream);
int dnnmg_graph_capture_end(void *stream, dnnmg_graph **graph);
int dnnmg_graph_replay(const dnnmg_graph *graph, void *stream);
int dnnmg_graph_destroy(dnnmg_graph *graph);

/* GPU-resident coarse step (Alg. 1, the coarse problem of a time step;
 * Sec. 2.4): A(x^L) = b^L on the coarse mesh of `box` (box->n cells per
 * axis, all even and >= 4), the Crank-Nicolson operator of eq. (disc:ns) with its
 * LPS terms, solved by `newton_its` inexact Newton steps.  Each Newton
 * correction is one cycle of FGMRES(krylov_dim) on J dx = b - A(x),
 * right-preconditioned by one geometric multigrid V-cycle over `levels`
 * meshes (the coarse mesh and its halvings while every axis keeps an even
 * count of at least 4 cells; 0: all of them) whose smoother is the coupled patch-Vanka step (the 108 x 108
 * velocity-pressure systems of the 2 x 2 x 2-cell patches, linearised at
 * the Newton iterate, damped by omega, pre_sweeps before and post_sweeps
 * after the coarse-grid correction, coarsest_sweeps on the last mesh).
 * J is applied matrix-free: J z = (A(x + eps z) - A(x)) / eps with
 * eps = fd_eta (rms(x) + fd_eta) / rms(z) on each mesh.  The residual and
 * the smoother run in FP32, the iterate, norms and FGMRES's Hessenberg
 * system in FP64.  Every count is fixed, so a solve can be recorded into a
 * graph. */
typedef struct dnnmg_coarse_opts {
    int32_t newton_its;      /* >= 1 */
    int32_t krylov_dim;      /* 1 .. DNNMG_COARSE_MAX_KRYLOV */
    int32_t levels;          /* 0 or >= 1 */
    int32_t pre_sweeps;      /* >= 1 */
    int32_t post_sweeps;     /* >= 0 */
    int32_t coarsest_sweeps; /* >= 1 */
    double omega;            /* Vanka damping, (0, 2) */
    double fd_eta;           /* > 0 */
} dnnmg_coarse_opts;
#define DNNMG_COARSE_MAX_KRYLOV 16

/* Multigrid levels a solve on `box` with `opts` uses (>= 1), or a negative
 * error code (an odd or too small cell count, invalid options). */
int dnnmg_coarse_levels(const dnnmg_box *box, const dnnmg_coarse_opts *opts);
/* Bytes of device workspace of dnnmg_coarse_solve, _jv and _vcycle. */
size_t dnnmg_coarse_workspace(const dnnmg_box *box, const dnnmg_coarse_opts *opts);
/* x (FP64 [4][n_coarse], in/out: start and result; its Dirichlet velocity
 * entries are kept), b (FP64 [4][n_coarse], the right-hand side, e.g.
 * dnnmg_restrict of the fine Rhs with its Dirichlet velocity rows zero).
 * res_norms (device FP64 [newton_its + 1], or NULL) receives ||b - A(x_k)||_2
 * before each Newton step and after the last.  b and x must not alias. */
int dnnmg_coarse_solve(const dnnmg_box *box, const dnnmg_ns *ns, const double *b, double *x,
                       const dnnmg_coarse_opts *opts, double *res_norms, void *ws, size_t ws_bytes, void *stream);
/* The solve's Jacobian-vector product on the coarse mesh: w = J(x) z
 * (FP32 [4][n_coarse] each; w must not alias x or z), with the solve's
 * finite-difference step (opts->fd_eta). */
int dnnmg_coarse_jv(const dnnmg_box *box, const dnnmg_ns *ns, const float *x, const float *z, float *w,
                    const dnnmg_coarse_opts *opts, void *ws, size_t ws_bytes, void *stream);
/* The solve's preconditioner: z = one V-cycle applied to s (FP32
 * [4][n_coarse] each, not aliased), linearised at x. */
int dnnmg_coarse_vcycle(const dnnmg_box *box, const dnnmg_ns *ns, const float *x, const float *s, float *z,
                        const dnnmg_coarse_opts *opts, void *ws, size_t ws_bytes, void *stream);


/* The paper's discretisation (Sec. 2.2): equal-order Q2 elements for
 * velocity and pressure on hexahedral meshes with curved (isoparametric)
 * cells, local projection stabilisation of eq. (disc:ns) with pi_h the
 * interpolation Q2 -> Q1 on each element, the Crank-Nicolson system of eq.
 * (4cranknicholson3) with the parameters of eq. (stabparams).
 *   Mesh: the topology of `box` (no periodic axes; box->len is not used):
 *   n[a] fine Q2 elements per axis, 2 n[a] + 1 nodes per axis, node index as
 *   above; element (I, J, K) holds the 27 nodes (2I + a, 2J + b, 2K + c)
 *   and maps the reference cube by the Q2 interpolation of their positions
 *   coords (device FP64 [3][n_fine], every element with a positive Jacobian
 *   determinant).  The elements are the patches of Sec. 4.2 (one per cell
 *   of level L), so the dof map, dnnmg_scatter_avg and the patch network
 *   apply unchanged.  The coarse Q2 mesh (level L) has the elements of
 *   2 x 2 x 2 fine elements (n[a] even) and the nodes with even indices.
 *   pi_h: Q1 interpolation of the element's 8 vertex values; h_T: the
 *   largest distance between two vertices of T; |v|_inf,T: the largest |v|
 *   over T's 27 nodes; 3 x 3 x 3 Gauss points per element; FP32 arithmetic.
 *   Element vectors go to the workspace ws (at least dnnmg_q2_workspace(box)
 *   bytes, 16-byte aligned: 189 floats per element) and are summed per node
 *   in a fixed order, so results are reproducible bit for bit.
 * dnnmg_q2_residual_b: r = b - A(x), A holding the iterate's terms of eq.
 *   (4cranknicholson3) and the LPS terms; x FP32 [4][n_fine], b FP32
 *   [4][n_fine], r FP32 [4][n_fine] output (not aliasing x or b), velocity
 *   rows on Dirichlet faces 0.
 * dnnmg_q2_rhs: b = (1/k)(v_a, phi) - 1/2 (v.grad v_a, phi) - nu/2 (grad v_a,
 *   grad phi) + (fmid_a, phi) (Algorithm 1, "Rhs"); v FP32 [3][n_fine],
 *   fmid FP32 [3][n_fine] or NULL, b FP32 [4][n_fine] (pressure and Dirichlet
 *   velocity rows 0). */
size_t dnnmg_q2_workspace(const dnnmg_box *box);
int dnnmg_q2_residual_b(const dnnmg_box *box, const dnnmg_ns *ns, const double *coords, const float *x,
                        const float *b, float *r, void *ws, size_t ws_bytes, void *stream);
int dnnmg_q2_rhs(const dnnmg_box *box, const dnnmg_ns *ns, const double *coords, const float *v,
                 const float *fmid, float *b, void *ws, size_t ws_bytes, void *stream);
/* Both at one iterate (Algorithm 1 after the correction: the indicator's
 * residual and the next step's right-hand side at x_corr): r = b - A(x) as
 * dnnmg_q2_residual_b and bnext = Rhs(velocity of x) as dnnmg_q2_rhs without
 * forcing, in one pass that shares the element work.  bnext may be b itself
 * (each node's b is read before it is replaced); r must not alias x, b or
 * bnext.  ws as for dnnmg_q2_residual_b. */
int dnnmg_q2_residual_rhs(const dnnmg_box *box, const dnnmg_ns *ns, const double *coords, const float *x,
                          const float *b, float *r, float *bnext, void *ws, size_t ws_bytes, void *stream);
/* Prolongation of Algorithm 1 between the Q2 spaces: each fine node takes the
 * Q2 interpolant of its coarse element (reference coordinates) in FP64,
 * rounded to FP32.  xc FP64 [ncomp][n_coarse] -> xf FP32 [ncomp][n_fine],
 * 1 <= ncomp <= 4, n[a] even.  dnnmg_q2_restrict is its transpose applied to
 * a fine dual vector, accumulated in FP64: bf FP32 [ncomp][n_fine] -> bc FP64
 * [ncomp][n_coarse]. */
int dnnmg_q2_prolong(const dnnmg_box *box, int ncomp, const double *xc, float *xf, void *stream);
int dnnmg_q2_restrict(const dnnmg_box *box, int ncomp, const float *bf, double *bc, void *stream);
/* Geometry inputs of Sec. 4.2 for curved cells, a setup call (the mesh is
 * fixed): geom FP32 [n_patches][3], g_a of element M = the mean length of its
 * 4 vertex-to-vertex edges along axis a (the cell sizes on axis-parallel
 * cells), from coords as for dnnmg_q2_residual_b.  The rows feed
 * dnnmg_patch_gather_geom / dnnmg_patch_gather_forward_geom. */
int dnnmg_q2_patch_features(const dnnmg_box *box, const double *coords, float *geom, void *stream);
/* dnnmg_patch_gather and dnnmg_patch_gather_forward with geometry inputs per
 * patch: columns 162..164 of row M are geom[3M .. 3M+2] (device FP32
 * [n_patches][3], not NULL; standardised by `feat` like every column)
 * instead of the box's cell sizes; everything else as there. */
int dnnmg_patch_gather_geom(const dnnmg_box *box, const float *geom, const float *x, const float *r,
                            const dnnmg_feat *feat, int dtype, float x_scale, void *X, int64_t ldx, void *stream);
int dnnmg_patch_gather_forward_geom(const dnnmg_box *box, const dnnmg_mlp *net, const float *geom, const float *xt,
                                    const float *r, const dnnmg_feat *feat, float *Y, void *stream);
/* The 24 geometry features of the paper's network inputs (Sec. 4.2) for
 * curved cells, a setup call: geo24 FP32 [n_patches][24], for element M from
 * the positions of its 8 vertices: the 12 vertex-to-vertex edge lengths
 * (x-directed edges first, then y, then z, each ordered by the other two
 * corner bits), the 4 diagonals between vertices sharing no face (vertex j
 * to 7 - j, j = 0..3, vertex j = a + 2b + 4c), and per vertex the mean of the
 * 3 dihedral angles between the faces meeting there. */
int dnnmg_q2_patch_features24(const dnnmg_box *box, const double *coords, float *geo24, void *stream);
/* dnnmg_patch_gather_paper (one-level patches) with the 24 geometry columns
 * of row M taken from geo24[24 M ..] (device FP32 [n_patches][24], not NULL)
 * instead of the box's brick features. */
int dnnmg_patch_gather_paper_geom(const dnnmg_box *box, const float *geo24, const float *x, const float *r,
                                  const dnnmg_feat *feat, int dtype, void *X, int64_t ldx, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* DNNMG_H */
