// Patch network of DNN-MG (arXiv 2307.14837, Sec. 3 and Sec. 4.2: a
// feed-forward network applied to every patch row of the gathered batch):
//   Y = W3^T tanh(W2^T tanh(W1^T x + b1) + b2) + b3,  165 -> H -> H -> 81.
//
// Layout.  The kernels compute the transposed products Z^T = W^T X^T on
// MFMA tiles of 16 hidden units x 16 patches, so a wave holds, after each
// layer, the hidden activations of its patches in the accumulator layout
// (lane = 16 g + p holds units 4 g .. 4 g + 3 of patch p).  That layout is
// used directly as the B operand of the next layer: the K (input) index of
// the next layer is permuted to match, and the weights are packed once in
// that permuted order, so no LDS transpose is needed between layers.
//
// Element types: FP32 (v_mfma_f32_16x16x4f32), BF16 (v_mfma_f32_16x16x32_bf16)
// and OCP FP8 E4M3 (v_mfma_f32_16x16x32_fp8_fp8) with per-tensor scales; all
// accumulate in FP32 and apply bias and tanh in FP32.
#include "common.hpp"
#include "lowp.hpp"
#include "mlp.hpp"

namespace dnnmg {

// ------------------------------------------------------- layer kinds ----
// Each layer runs on one MFMA kind:
//   KF32  v_mfma_f32_16x16x4f32            E = 1 element  per lane, K = 4
//   KBF16 v_mfma_f32_16x16x32_bf16         E = 8 elements per lane, K = 32
//   KFP8  v_mfma_scale_f32_16x16x128_f8f6f4 (E4M3, unit scales)
//                                          E = 32 elements per lane, K = 128
// Network dtype -> kinds of (layer 1, layer 2, layer 3):
//   F32: all KF32; BF16: all KBF16; FP8: KBF16, KFP8, KBF16 (the H x H
//   product in FP8, the 165-wide input and the 81-wide output in BF16).
enum Kind { KF32 = 0, KBF16 = 1, KFP8 = 2 };

__host__ __device__ constexpr int layer_kind(int dt, int layer) {
    return dt == DNNMG_F32 ? KF32 : (dt == DNNMG_BF16 ? KBF16 : (layer == 1 ? KFP8 : KBF16));
}
__host__ __device__ constexpr int kind_E(int k) { return k == KF32 ? 1 : (k == KBF16 ? 8 : 32); }
__host__ __device__ constexpr int kind_bytes(int k) { return k == KF32 ? 4 : (k == KBF16 ? 2 : 1); }

// ------------------------------------------------------------- packing ----
// Fragment (ot, kc) of a layer: 64 lanes x E elements; lane 16 g + i holds
// the weights of output unit 16 ot + i for the K slots (kc, g, e).  Layer-1
// slots are the input columns in order.  Hidden inputs arrive in the
// accumulator layout of the previous layer (lane 16 g + p holds units
// 16 t + 4 g + 0..3 of tile t), so slot (kc, g, e) is unit
// 16 (kc E/4 + e/4) + 4 g + e%4  (E >= 4), or 16 (kc/4) + 4 g + kc%4 (E = 1).
__host__ __device__ inline int kslot_to_input(int kind, int layer, int kc, int g, int e) {
    const int E = kind_E(kind);
    if (layer == 0) return kc * 4 * E + g * E + e;
    if (E == 1) return 16 * (kc >> 2) + 4 * g + (kc & 3);
    return 16 * (kc * (E / 4) + (e >> 2)) + 4 * g + (e & 3);
}

template <typename OUT>
__global__ void k_pack(int kind, int layer, int fan_in, int fan_out, int ntiles, int nchunks,
                       const float *__restrict__ W, float inv_wscale, OUT *__restrict__ Wp) {
    const int E = kind_E(kind);
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)ntiles * nchunks * 64 * E;
    if (t >= total) return;
    int e = (int)(t % E);
    int lane = (int)((t / E) % 64);
    int kc = (int)((t / (E * 64)) % nchunks);
    int ot = (int)(t / ((int64_t)E * 64 * nchunks));
    int g = lane >> 4, i = lane & 15;
    int o = 16 * ot + i;
    int k = kslot_to_input(kind, layer, kc, g, e);
    float w = (o < fan_out && k < fan_in) ? W[(int64_t)k * fan_out + o] : 0.0f;
    if constexpr (sizeof(OUT) == 4) Wp[t] = w;
    else if constexpr (sizeof(OUT) == 2) Wp[t] = f32_to_bf16(w);
    else Wp[t] = f32_to_e4m3(w * inv_wscale);
}

// ------------------------------------------------------------- forward ----
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

template <int K> struct Frag;
template <> struct Frag<KF32> { using T = float; };
template <> struct Frag<KBF16> { using T = u32x4; };  // 8 bf16
template <> struct Frag<KFP8> { using T = i32x8; };   // 32 fp8

template <int K>
__device__ __forceinline__ f32x4 mfma(typename Frag<K>::T a, typename Frag<K>::T b, f32x4 c) {
    if constexpr (K == KF32) return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    else if constexpr (K == KBF16)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    else // format 0 = E4M3 for both operands; E8M0 scales 127 = 1.0
        return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
}

__device__ __forceinline__ float tanh_fast(float z) {
    // tanh z = 1 - 2 / (exp(2z) + 1); saturates cleanly for large |z|
    float t = __expf(2.0f * z);
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(t + 1.0f);
}

template <int K>
__device__ __forceinline__ float act(float z) {
    if constexpr (K == KF32) return tanhf(z);
    else return tanh_fast(z);
}

// Activations of 4 units (one accumulator of output tile ot) into the B
// fragments of a layer of kind K (see kslot_to_input).
template <int K>
__device__ __forceinline__ void put_act(typename Frag<K>::T *B, int ot, const float v[4], float qinv) {
    if constexpr (K == KF32) {
#pragma unroll
        for (int e = 0; e < 4; ++e) B[4 * ot + e] = v[e];
    } else if constexpr (K == KBF16) {
        int kc = ot >> 1, half = ot & 1;
        B[kc][2 * half] = pack_bf16x2(v[0], v[1]);
        B[kc][2 * half + 1] = pack_bf16x2(v[2], v[3]);
    } else {
        int kc = ot >> 3, q = ot & 7;
        uint32_t w = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) w |= (uint32_t)f32_to_e4m3(v[e] * qinv) << (8 * e);
        B[kc][q] = (int)w;
    }
}

// One dense layer on the wave's NP patch tiles: acc = W^T B, then bias and
// (unless LAST) tanh into the next layer's fragments.
template <int K, int KNEXT, int NTILES, int NCH, int NP, bool LAST, int H>
__device__ __forceinline__ void layer(const typename Frag<K>::T *__restrict__ Wl, const float *__restrict__ bias,
                                      const typename Frag<K>::T (&B)[NP][NCH],
                                      typename Frag<KNEXT>::T (&Bn)[NP][H / (4 * kind_E(KNEXT))],
                                      float scale, float qinv, int lane, int g, int p, int64_t base,
                                      int64_t n, float *__restrict__ Y, void *__restrict__ saved,
                                      int64_t save_off, int save_bytes) {
#pragma unroll
    for (int ot = 0; ot < NTILES; ++ot) {
        f32x4 acc[NP];
#pragma unroll
        for (int t = 0; t < NP; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < NCH; ++kc) {
            typename Frag<K>::T a = Wl[((int64_t)ot * NCH + kc) * 64 + lane];
#pragma unroll
            for (int t = 0; t < NP; ++t) acc[t] = mfma<K>(a, B[t][kc], acc[t]);
        }
        if constexpr (LAST) {
#pragma unroll
            for (int t = 0; t < NP; ++t) {
                int64_t row = base + 16 * t + p;
                if (row >= n) continue;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    int o = 16 * ot + 4 * g + e;
                    if (o < N_OUT) Y[row * N_OUT + o] = acc[t][e] * scale + bias[o];
                }
            }
        } else {
            const float4 bb = *(const float4 *)(bias + 16 * ot + 4 * g);
            const float bv[4] = {bb.x, bb.y, bb.z, bb.w};
#pragma unroll
            for (int t = 0; t < NP; ++t) {
                float v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = act<K>(acc[t][e] * scale + bv[e]);
                put_act<KNEXT>(Bn[t], ot, v, qinv);
                if (saved) {
                    int64_t row = base + 16 * t + p;
                    if (row < n) {
                        int64_t idx = save_off + row * H + 16 * ot + 4 * g;
                        if (save_bytes == 4)
                            *(float4 *)((float *)saved + idx) = make_float4(v[0], v[1], v[2], v[3]);
                        else
                            *(uint2 *)((uint16_t *)saved + idx) =
                                make_uint2(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]));
                    }
                }
            }
        }
    }
}

template <int DT, int H, int NP>
__global__ void __launch_bounds__(256)
    k_mlp_fwd(int64_t n, const void *__restrict__ Xv, int64_t ldx, const void *__restrict__ W0,
              const void *__restrict__ W1, const void *__restrict__ W2, const float *__restrict__ b0,
              const float *__restrict__ b1, const float *__restrict__ b2, float *__restrict__ Y,
              void *__restrict__ saved, float s0, float s1, float s2, float q1inv, float q2inv) {
    constexpr int K1 = layer_kind(DT, 0), K2 = layer_kind(DT, 1), K3 = layer_kind(DT, 2);
    constexpr int NCH0 = IN_PAD / (4 * kind_E(K1));
    constexpr int NCH1 = H / (4 * kind_E(K2));
    constexpr int NCH2 = H / (4 * kind_E(K3));
    using F1 = typename Frag<K1>::T;
    using F2 = typename Frag<K2>::T;
    using F3 = typename Frag<K3>::T;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4, p = lane & 15;
    const int64_t base = ((int64_t)blockIdx.x * 4 + wave) * 16 * NP;
    if (base >= n) return;
    const int sbytes = DT == DNNMG_F32 ? 4 : 2;

    // layer-1 input fragments straight from the gathered rows (row-major,
    // E consecutive columns per lane)
    F1 Bx[NP][NCH0];
#pragma unroll
    for (int t = 0; t < NP; ++t) {
        int64_t row = base + 16 * t + p;
#pragma unroll
        for (int kc = 0; kc < NCH0; ++kc) {
            if (row < n) {
                if constexpr (K1 == KF32)
                    Bx[t][kc] = ((const float *)Xv)[row * ldx + kc * 4 + g];
                else
                    Bx[t][kc] = *(const F1 *)((const uint16_t *)Xv + row * ldx + kc * 32 + g * 8);
            } else {
                Bx[t][kc] = F1{};
            }
        }
    }
    F2 Ba[NP][NCH1];
    layer<K1, K2, H / 16, NCH0, NP, false, H>((const F1 *)W0, b0, Bx, Ba, s0, q1inv, lane, g, p, base, n,
                                              Y, saved, 0, sbytes);
    F3 Bb[NP][NCH2];
    layer<K2, K3, H / 16, NCH1, NP, false, H>((const F2 *)W1, b1, Ba, Bb, s1, q2inv, lane, g, p, base, n,
                                              Y, saved, n * H, sbytes);
    F3 dummy[NP][H / (4 * kind_E(K3))];
    layer<K3, K3, OUT_PAD / 16, NCH2, NP, true, H>((const F3 *)W2, b2, Bb, dummy, s2, 1.f, lane, g, p,
                                                   base, n, Y, nullptr, 0, sbytes);
}

// ---------------------------------------------- fused gather + network ----
// Layer-1 fragments built directly from the node fields (operator Q of
// eq. (defQ) with the standardisation), so the gathered batch never goes
// through HBM.  Column col of the input row of patch (I,J,K): field
// col / 27 of [u, v, w, r_u, r_v, r_w] at local node col % 27; 162..164 the
// coarse cell sizes; zero padding to 192.
__device__ __forceinline__ float input_col(const Mesh &m, int I, int J, int K, int col,
                                           const float *__restrict__ xt, const float *__restrict__ r,
                                           const float *__restrict__ shift, const float *__restrict__ inv) {
    if (col >= N_IN) return 0.0f;
    float v;
    if (col < 162) {
        int c = col / 27, iota = col - 27 * c;
        int a = iota % 3, b = (iota / 3) % 3, cc = iota / 9;
        int i = wrap(2 * I + a, m.nf[0], m.per[0]);
        int j = wrap(2 * J + b, m.nf[1], m.per[1]);
        int k = wrap(2 * K + cc, m.nf[2], m.per[2]);
        int64_t node = i + (int64_t)m.nf[0] * (j + (int64_t)m.nf[1] * k);
        v = c < 3 ? xt[c * m.n_fine + node] : r[(c - 3) * m.n_fine + node];
    } else {
        v = m.H[col - 162];
    }
    if (shift) v -= shift[col];
    if (inv) v *= inv[col];
    return v;
}

// Persistent: blocks walk the 64-patch tiles of all boxes (tile -> box by
// the prefix sums blk_ptile); D == nullptr means the single box `one`.
template <int DT, int H, int NP>
__global__ void __launch_bounds__(256)
    k_mlp_gather_fwd(const BoxDesc *__restrict__ D, int nbox, BoxDesc one, int64_t ntiles,
                     const float *__restrict__ xt_all, const float *__restrict__ r_all,
                     const float *__restrict__ shift, const float *__restrict__ inv,
                     const void *__restrict__ W0, const void *__restrict__ W1, const void *__restrict__ W2,
                     const float *__restrict__ b0, const float *__restrict__ b1, const float *__restrict__ b2,
                     float *__restrict__ Y_all, float s1, float q1inv) {
    constexpr int K1 = layer_kind(DT, 0), K2 = layer_kind(DT, 1), K3 = layer_kind(DT, 2);
    constexpr int E1 = kind_E(K1);
    constexpr int NCH0 = IN_PAD / (4 * E1);
    constexpr int NCH1 = H / (4 * kind_E(K2));
    constexpr int NCH2 = H / (4 * kind_E(K3));
    using F1 = typename Frag<K1>::T;
    using F2 = typename Frag<K2>::T;
    using F3 = typename Frag<K3>::T;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, p = lane & 15;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int b = D ? find_box(nbox, tile, [&](int i) { return D[i].blk_ptile; }) : 0;
        const BoxDesc &d = D ? D[b] : one;
        const Mesh m = d.m;
        const float *xt = xt_all + 4 * d.off_fine;
        const float *r = r_all + 4 * d.off_fine;
        float *Y = Y_all + 81 * d.off_patch;
        const int64_t n = m.n_patches;
        const int64_t base = (tile - d.blk_ptile) * 64 * NP + 16 * NP * wave;
        if (base >= n) continue; // wave-uniform; no block-wide barrier below
        F1 Bx[NP][NCH0];
#pragma unroll
        for (int t = 0; t < NP; ++t) {
            const int64_t row = base + 16 * t + p;
            int I = 0, J = 0, K = 0;
            if (row < n) {
                uint32_t JK = fdiv((uint32_t)row, m.px);
                I = (int)((uint32_t)row - JK * m.n[0]);
                K = (int)fdiv(JK, m.py);
                J = (int)(JK - (uint32_t)K * m.n[1]);
            }
#pragma unroll
            for (int kc = 0; kc < NCH0; ++kc) {
                if constexpr (K1 == KF32) {
                    Bx[t][kc] = row < n ? input_col(m, I, J, K, kc * 4 + g, xt, r, shift, inv) : 0.0f;
                } else {
                    float v[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        v[e] = row < n ? input_col(m, I, J, K, kc * 32 + g * 8 + e, xt, r, shift, inv) : 0.0f;
                    F1 f;
#pragma unroll
                    for (int q = 0; q < 4; ++q) f[q] = pack_bf16x2(v[2 * q], v[2 * q + 1]);
                    Bx[t][kc] = f;
                }
            }
        }
        F2 Ba[NP][NCH1];
        layer<K1, K2, H / 16, NCH0, NP, false, H>((const F1 *)W0, b0, Bx, Ba, 1.0f, q1inv, lane, g, p, base, n,
                                                  Y, nullptr, 0, 2);
        F3 Bb[NP][NCH2];
        layer<K2, K3, H / 16, NCH1, NP, false, H>((const F2 *)W1, b1, Ba, Bb, s1, 1.0f, lane, g, p, base, n, Y,
                                                  nullptr, 0, 2);
        F3 dummy[NP][H / (4 * kind_E(K3))];
        layer<K3, K3, OUT_PAD / 16, NCH2, NP, true, H>((const F3 *)W2, b2, Bb, dummy, 1.0f, 1.0f, lane, g, p,
                                                       base, n, Y, nullptr, 0, 2);
    }
}

int gather_fwd_launch(const dnnmg_mlp *net, int np, const BoxDesc *D, int nbox, const BoxDesc &one,
                      int64_t ntiles, int grid, const float *xt, const float *r, const float *shift,
                      const float *inv, float *Y, hipStream_t s) {
    float s1 = 1.f, q1 = 1.f;
    if (net->dtype == DNNMG_FP8_E4M3) {
        s1 = net->w_scale[1] * net->a_scale[1];
        q1 = 1.0f / net->a_scale[1];
    }
    if (grid <= 0 || grid > ntiles) grid = (int)ntiles;
#define GF(DT, HH, NPV)                                                                                  \
    if (net->dtype == DT && net->hidden == HH && np == NPV) {                                           \
        k_mlp_gather_fwd<DT, HH, NPV><<<grid, 256, 0, s>>>(D, nbox, one, ntiles, xt, r, shift, inv,      \
                                                           net->W[0], net->W[1], net->W[2], net->b[0],  \
                                                           net->b[1], net->b[2], Y, s1, q1);             \
        return hip_check(hipGetLastError(), "fused gather+forward launch");                             \
    }
    GF(DNNMG_F32, 128, 1) GF(DNNMG_F32, 256, 1)
    GF(DNNMG_BF16, 128, 1) GF(DNNMG_BF16, 256, 1) GF(DNNMG_BF16, 512, 1)
    GF(DNNMG_BF16, 128, 2) GF(DNNMG_BF16, 256, 2)
    GF(DNNMG_FP8_E4M3, 256, 1) GF(DNNMG_FP8_E4M3, 512, 1) GF(DNNMG_FP8_E4M3, 256, 2) GF(DNNMG_FP8_E4M3, 512, 2)
#undef GF
    return fail(DNNMG_ERR_UNSUPPORTED, "fused gather+forward: dtype %d width %d", net->dtype, net->hidden);
}

template <int DT, int H, int NP>
static int launch_fwd(const dnnmg_mlp *net, int64_t n, const void *X, int64_t ldx, float *Y,
                      void *saved, hipStream_t s) {
    float s0 = 1.f, s1 = 1.f, s2 = 1.f, q1 = 1.f, q2 = 1.f;
    if (DT == DNNMG_FP8_E4M3) {
        // only the hidden product is FP8: its weights (w_scale[1]) and its
        // input activations (a_scale[1]) carry scales
        s1 = net->w_scale[1] * net->a_scale[1];
        q1 = 1.0f / net->a_scale[1];
    }
    int64_t per_block = 4 * 16 * NP;
    unsigned grid = (unsigned)((n + per_block - 1) / per_block);
    k_mlp_fwd<DT, H, NP><<<grid, 256, 0, s>>>(n, X, ldx, net->W[0], net->W[1], net->W[2], net->b[0],
                                              net->b[1], net->b[2], Y, DT == DNNMG_FP8_E4M3 ? nullptr : saved,
                                              s0, s1, s2, q1, q2);
    return hip_check(hipGetLastError(), "dnnmg_patch_forward launch");
}

int check_net(const dnnmg_mlp *net) {
    if (!net) return fail(DNNMG_ERR_ARG, "net is NULL");
    if (net->n_in != N_IN || net->n_out != N_OUT)
        return fail(DNNMG_ERR_SHAPE, "network must be %d -> H -> H -> %d (got %d, %d)", N_IN, N_OUT,
                    net->n_in, net->n_out);
    if (net->hidden != 64 && net->hidden != 128 && net->hidden != 256 && net->hidden != 512)
        return fail(DNNMG_ERR_UNSUPPORTED, "hidden width %d not in {64,128,256,512}", net->hidden);
    if (net->dtype != DNNMG_F32 && net->dtype != DNNMG_BF16 && net->dtype != DNNMG_FP8_E4M3)
        return fail(DNNMG_ERR_UNSUPPORTED, "network dtype %d", net->dtype);
    for (int l = 0; l < 3; ++l) {
        if (!net->W[l] || !net->b[l]) return fail(DNNMG_ERR_ARG, "network W[%d]/b[%d] is NULL", l, l);
        if (!aligned16(net->W[l]) || !aligned16(net->b[l]))
            return fail(DNNMG_ERR_ARG, "network W[%d]/b[%d] not 16-byte aligned", l, l);
        if (net->dtype == DNNMG_FP8_E4M3 && l == 1 && (!(net->w_scale[1] > 0.f) || !(net->a_scale[1] > 0.f)))
            return fail(DNNMG_ERR_ARG, "FP8 network needs positive w_scale[1] and a_scale[1]");
    }
    return DNNMG_OK;
}

} // namespace dnnmg

using namespace dnnmg;

extern "C" size_t dnnmg_mlp_packed_bytes(int dtype, int hidden, int layer) {
    if (layer < 0 || layer > 2) return 0;
    if (dtype != DNNMG_F32 && dtype != DNNMG_BF16 && dtype != DNNMG_FP8_E4M3) return 0;
    int kp = layer == 0 ? IN_PAD : hidden;
    int np = layer == 2 ? OUT_PAD : hidden;
    return (size_t)kp * np * kind_bytes(layer_kind(dtype, layer));
}

extern "C" int dnnmg_mlp_pack(int dtype, int hidden, int layer, const float *W, float w_scale,
                              void *Wp, void *stream) {
    if (hidden != 64 && hidden != 128 && hidden != 256 && hidden != 512)
        return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_mlp_pack: hidden %d", hidden);
    if (layer < 0 || layer > 2) return fail(DNNMG_ERR_ARG, "dnnmg_mlp_pack: layer %d", layer);
    if (dtype != DNNMG_F32 && dtype != DNNMG_BF16 && dtype != DNNMG_FP8_E4M3)
        return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_mlp_pack: dtype %d", dtype);
    if (!W || !Wp || !aligned16(Wp)) return fail(DNNMG_ERR_ARG, "dnnmg_mlp_pack: bad pointer");
    const int kind = layer_kind(dtype, layer);
    if (kind == KFP8 && !(w_scale > 0.f)) return fail(DNNMG_ERR_ARG, "dnnmg_mlp_pack: w_scale must be > 0");
    if (kind == KFP8 && hidden < 128)
        return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_mlp_pack: FP8 needs hidden >= 128");
    int fan_in = layer == 0 ? N_IN : hidden;
    int fan_out = layer == 2 ? N_OUT : hidden;
    int kp = layer == 0 ? IN_PAD : hidden;
    int np = layer == 2 ? OUT_PAD : hidden;
    int E = kind_E(kind);
    int ntiles = np / 16, nchunks = kp / (4 * E);
    int64_t total = (int64_t)ntiles * nchunks * 64 * E;
    hipStream_t s = (hipStream_t)stream;
    unsigned grid = blocks_for(total, 256);
    if (kind == KF32)
        k_pack<float><<<grid, 256, 0, s>>>(kind, layer, fan_in, fan_out, ntiles, nchunks, W, 1.f, (float *)Wp);
    else if (kind == KBF16)
        k_pack<uint16_t><<<grid, 256, 0, s>>>(kind, layer, fan_in, fan_out, ntiles, nchunks, W, 1.f,
                                              (uint16_t *)Wp);
    else
        k_pack<uint8_t><<<grid, 256, 0, s>>>(kind, layer, fan_in, fan_out, ntiles, nchunks, W,
                                             1.f / w_scale, (uint8_t *)Wp);
    return hip_check(hipGetLastError(), "dnnmg_mlp_pack launch");
}

extern "C" size_t dnnmg_patch_saved_bytes(const dnnmg_mlp *net, int64_t n) {
    if (!net) return 0;
    size_t es = net->dtype == DNNMG_F32 ? 4 : net->dtype == DNNMG_BF16 ? 2 : 0;
    return (size_t)2 * n * net->hidden * es;
}

extern "C" int dnnmg_patch_forward(const dnnmg_mlp *net, int64_t n, const void *X, int64_t ldx,
                                   float *Y, void *saved, void *stream) {
    int rc = check_net(net);
    if (rc) return rc;
    if (n < 0) return fail(DNNMG_ERR_SHAPE, "dnnmg_patch_forward: n < 0");
    if (n == 0) return DNNMG_OK;
    if (!X || !Y) return fail(DNNMG_ERR_ARG, "dnnmg_patch_forward: NULL pointer");
    if (!aligned16(X)) return fail(DNNMG_ERR_ARG, "dnnmg_patch_forward: X not 16-byte aligned");
    int align = net->dtype == DNNMG_F32 ? 4 : 8;
    if (ldx < IN_PAD || ldx % align)
        return fail(DNNMG_ERR_SHAPE, "dnnmg_patch_forward: ldx %lld must be >= %d and a multiple of %d",
                    (long long)ldx, IN_PAD, align);
    if (saved && net->dtype == DNNMG_FP8_E4M3)
        return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_patch_forward: FP8 networks do not save activations");
    if (saved && !aligned16(saved)) return fail(DNNMG_ERR_ARG, "dnnmg_patch_forward: saved not aligned");
    hipStream_t s = (hipStream_t)stream;
    const int H = net->hidden;
#define FWD(DT, HH, NP)                                                   \
    if (net->dtype == DT && H == HH) return launch_fwd<DT, HH, NP>(net, n, X, ldx, Y, saved, s);
    FWD(DNNMG_F32, 64, 1) FWD(DNNMG_F32, 128, 1) FWD(DNNMG_F32, 256, 1)
    FWD(DNNMG_BF16, 64, 2) FWD(DNNMG_BF16, 128, 2) FWD(DNNMG_BF16, 256, 2) FWD(DNNMG_BF16, 512, 1)
    FWD(DNNMG_FP8_E4M3, 128, 2) FWD(DNNMG_FP8_E4M3, 256, 2) FWD(DNNMG_FP8_E4M3, 512, 2)
#undef FWD
    return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_patch_forward: dtype %d width %d", net->dtype, H);
}

extern "C" int dnnmg_patch_gather_forward(const dnnmg_box *box, const dnnmg_mlp *net, const float *xt,
                                          const float *r, const dnnmg_feat *feat, float *Y, void *stream) {
    int rc = check_net(net);
    if (rc) return rc;
    BoxDesc one{};
    if ((rc = make_mesh(box, &one.m))) return rc;
    if (!xt || !r || !Y) return fail(DNNMG_ERR_ARG, "dnnmg_patch_gather_forward: NULL pointer");
    const float *sh = feat ? feat->shift : nullptr;
    const float *sc = feat ? feat->inv_scale : nullptr;
    int64_t ntiles = (one.m.n_patches + 63) / 64;
    return gather_fwd_launch(net, 1, nullptr, 1, one, ntiles, 0, xt, r, sh, sc, Y, (hipStream_t)stream);
}
