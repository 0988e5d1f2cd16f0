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
// and OCP FP8 E4M3 (v_mfma_scale_f32_16x16x128_f8f6f4) with per-tensor
// scales; all accumulate in FP32 and apply bias and tanh in FP32.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

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
// the weights of output unit 16 ot + i for the K slots (kc, g, e).  The
// fragments are stored K-chunk major (kc, ot): the fragments all waves read
// at one step of the K loop are contiguous, which spreads the concurrent
// reads of many workgroups over the memory channels.  Layer-1
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

// colscale (optional): every weight of output column o is multiplied by
// colscale[o] first (a batch normalisation folded into the layer).
template <typename OUT>
__global__ void k_pack(int kind, int layer, int fan_in, int fan_out, int ntiles, int nchunks,
                       const float *__restrict__ W, float inv_wscale, OUT *__restrict__ Wp,
                       const float *__restrict__ colscale) {
    const int E = kind_E(kind);
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)ntiles * nchunks * 64 * E;
    if (t >= total) return;
    int e = (int)(t % E);
    int lane = (int)((t / E) % 64);
    int ot = (int)((t / (E * 64)) % ntiles);
    int kc = (int)(t / ((int64_t)E * 64 * ntiles));
    int g = lane >> 4, i = lane & 15;
    int o = 16 * ot + i;
    int k = kslot_to_input(kind, layer, kc, g, e);
    float w = (o < fan_out && k < fan_in) ? W[(int64_t)k * fan_out + o] : 0.0f;
    if (colscale && o < fan_out) w *= colscale[o];
    if constexpr (sizeof(OUT) == 4) Wp[t] = w;
    else if constexpr (sizeof(OUT) == 2) Wp[t] = f32_to_bf16(w);
    else Wp[t] = f32_to_e4m3(w * inv_wscale);
}

// ------------------------------------------------------------- forward ----
// A workgroup of NW waves takes tiles of 16 PT patches.  Each layer's input
// lives in LDS in the B-fragment layout of its MFMA kind: fragment (t, kc)
// of patch tile t and K chunk kc is 64 lanes x FB bytes at
// ((t NCH + kc) 64 + lane) FB.  Output tile ot (16 units) of a layer is
// computed by wave ot % NW for all PT patch tiles, so every weight fragment
// (A operand, read from global memory where it stays cache resident) feeds
// PT products and every activation fragment read from LDS feeds the
// wave's output tiles.  Bias, tanh and the conversion to the next layer's
// element type are applied on the accumulators, which are written straight
// into the next layer's LDS fragments.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

template <int K> struct Frag;
template <> struct Frag<KF32> { using T = float; };
template <> struct Frag<KBF16> { using T = u32x4; };  // 8 bf16
template <> struct Frag<KFP8> { using T = i32x8; };   // 32 fp8

// largest divisor of n that is at most cap
__host__ __device__ constexpr int unroll_divisor(int n, int cap) {
    int d = cap;
    while (d > 1 && n % d != 0) --d;
    return d;
}
__host__ __device__ constexpr int frag_bytes(int k) { return k == KF32 ? 4 : (k == KBF16 ? 16 : 32); }

template <int K>
__device__ __forceinline__ f32x4 mfma(typename Frag<K>::T a, typename Frag<K>::T b, f32x4 c) {
    if constexpr (K == KF32) return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    else if constexpr (K == KBF16)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    else // format 0 = E4M3 for both operands; E8M0 scales 127 = 1.0
        return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
}

// A weight fragment through a buffer resource: byte offset voff (the lane's
// term, one VGPR) plus soff (wave-uniform, an SGPR), so the addresses of a
// layer's fragments take no vector registers of their own.  Reads past the
// resource's size return zero.
template <int K>
__device__ __forceinline__ typename Frag<K>::T load_frag(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    if constexpr (K == KF32) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    } else if constexpr (K == KBF16) {
        return __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    } else {
        const u32x4 lo = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
        const u32x4 hi = __builtin_amdgcn_raw_buffer_load_b128(r, voff + 16, soff, 0);
        return i32x8{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
    }
}

// Activations v[0..3] of units 16 ot + 4 g + e of patch p (lane 16 g + p) of
// patch tile t into the next layer's LDS fragments (kind KN: FP32 or BF16,
// NCHN chunks); see kslot_to_input for the slot order.
template <int KN, int NCHN>
__device__ __forceinline__ void put_act(unsigned char *out, int t, int ot, int lane, const float v[4]) {
    static_assert(KN == KF32 || KN == KBF16, "FP8 activations go through put_fp8");
    if constexpr (KN == KF32) {
#pragma unroll
        for (int e = 0; e < 4; ++e) ((float *)out)[(t * NCHN + 4 * ot + e) * 64 + lane] = v[e];
    } else {
        uint2 w = make_uint2(pack_bf16x2_hw(v[0], v[1]), pack_bf16x2_hw(v[2], v[3]));
        *(uint2 *)(out + ((t * NCHN + (ot >> 1)) * 64 + lane) * 16 + 8 * (ot & 1)) = w;
    }
}

// FP8 codes of qinv tanh z = qinv (1 - 2 r) for units 16 ot + 4 g + e of
// patch p (lane 16 g + p) of patch tile t, from r = 1 / (exp(2 z) + 1), into
// the next layer's LDS fragments (NCHN chunks), with the hardware E4M3
// conversion (round to nearest even).  Since 0 <= r <= 1 the codes lie in
// [-qinv, qinv]; SAT (qinv above 448, the largest E4M3 value) clamps them to
// +-448 first, as the software encoder saturates.  NaN passes either way.
template <int NCHN, bool SAT>
__device__ __forceinline__ void put_fp8(unsigned char *out, int t, int ot, int lane, const float r[4], float qinv) {
    float q[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float x = fmaf(-2.0f * qinv, r[e], qinv);
        q[e] = SAT ? (x != x ? x : fminf(fmaxf(x, -448.0f), 448.0f)) : x;
    }
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(q[0], q[1], 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(q[2], q[3], w, true);
    *(int *)(out + ((t * NCHN + (ot >> 3)) * 64 + lane) * 32 + 4 * (ot & 7)) = w;
}

// Barrier for the LDS hand-offs between the layers of a tile: it waits for
// this wave's LDS operations only, so weight loads and output stores stay in
// flight across it (a full __syncthreads also drains the vector memory
// counter).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// One dense layer for the tile: acc = W^T B over the wave's output tiles,
// then bias and (unless LAST) tanh into the next layer's fragments, or (LAST)
// the output rows.  INPLACE: `out` is `in`; every wave's products (all its
// reads of `in`) end at a workgroup barrier before the first output is
// written, and a skip connection reads the input only at the positions the
// same lane then overwrites.
template <int K, int KN, int NTILES, int NCH, int PT, bool LAST, int H, int NW, int NO = N_OUT, bool SKIP = false,
          bool INPLACE = false>
__device__ __forceinline__ void layer(const typename Frag<K>::T *__restrict__ Wl, const float *__restrict__ bias,
                                      const unsigned char *in, unsigned char *out, float scale, float qinv,
                                      int wave, int lane, int64_t base, int64_t n, float *__restrict__ Y,
                                      void *__restrict__ saved, int64_t save_off, int save_bytes) {
    using FA = typename Frag<K>::T;
    constexpr int OTW = (NTILES + NW - 1) / NW;
    constexpr int NCHN = LAST ? 1 : H / (4 * kind_E(KN));
    const int g = lane >> 4, p = lane & 15;
    f32x4 acc[OTW][PT];
    // UNROLL K chunks per step: the weight and activation fragments of a
    // step are requested together.  A step holds OTW + PT fragments per K
    // chunk; UNROLL is the largest divisor of NCH (at most 8) whose fragments
    // fit in what the accumulators leave of a 192-register budget, and at
    // least 2 where NCH is even.
    constexpr int FRAG_REGS = frag_bytes(K) / 4;
    constexpr int STEP_REGS = (OTW + PT) * FRAG_REGS;
    constexpr int FIT = (192 - 4 * OTW * PT) / STEP_REGS;
    constexpr int U0 = unroll_divisor(NCH, FIT < 1 ? 1 : (FIT > 8 ? 8 : FIT));
    constexpr int UNROLL = (U0 < 2 && NCH % 2 == 0) ? 2 : U0;
    constexpr int FB = frag_bytes(K);
    const __amdgpu_buffer_rsrc_t wr =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<FA *>(Wl), (short)0, NCH * NTILES * 64 * FB, 0x00020000);
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);
    // products over the wave's first NT output tiles; the tile test sits
    // outside the K loop, so a step's weight loads carry no branch and are
    // requested together
    auto products = [&](auto nt) {
        constexpr int NT = decltype(nt)::value;
        auto chunk = [&](int kc, auto first) {
            FA b[PT];
#pragma unroll
            for (int t = 0; t < PT; ++t) b[t] = ((const FA *)in)[(t * NCH + kc) * 64 + lane];
#pragma unroll
            for (int i = 0; i < NT; ++i) {
                FA a = load_frag<K>(wr, lane * FB, (kc * NTILES + wave_u + NW * i) * 64 * FB);
#pragma unroll
                for (int t = 0; t < PT; ++t)
                    acc[i][t] = mfma<K>(a, b[t], decltype(first)::value ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[i][t]);
            }
        };
        // the accumulators start from zero
#pragma unroll
        for (int i = 0; i < OTW; ++i)
#pragma unroll
            for (int t = 0; t < PT; ++t) acc[i][t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll UNROLL
        for (int kc = 0; kc < NCH; ++kc) chunk(kc, std::false_type{});
    };
    if (NTILES % NW == 0 || wave + NW * (OTW - 1) < NTILES) products(std::integral_constant<int, OTW>{});
    else if constexpr (OTW > 1) products(std::integral_constant<int, OTW - 1>{});
    if constexpr (INPLACE) lds_barrier();
#pragma unroll
    for (int i = 0; i < OTW; ++i) {
        const int ot = wave + NW * i;
        if (!(NTILES % NW == 0 || ot < NTILES)) continue;
        if constexpr (LAST) {
            // outputs of the tile to LDS rows [16 t + p][81]; written out
            // contiguously afterwards (the lane's four biases are loaded
            // once, clamped to the last output, without a branch)
            float *ys = (float *)out;
            float bl[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int o = 16 * ot + 4 * g + e;
                bl[e] = bias[o < NO ? o : NO - 1];
            }
#pragma unroll
            for (int t = 0; t < PT; ++t) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    int o = 16 * ot + 4 * g + e;
                    if (o < NO) ys[(16 * t + p) * NO + o] = acc[i][t][e] * scale + bl[e];
                }
            }
        } else {
            const float4 bb = *(const float4 *)(bias + 16 * ot + 4 * g);
            // low precision: tanh z = 1 - 2 / (2^(2 z log2 e) + 1) with the
            // factor 2 log2 e folded into the scale and the bias
            constexpr float K2 = 2.8853900817779268f; // 2 log2(e)
            const float sc = K == KF32 ? scale : scale * K2;
            const float bv[4] = {K == KF32 ? bb.x : bb.x * K2, K == KF32 ? bb.y : bb.y * K2,
                                 K == KF32 ? bb.z : bb.z * K2, K == KF32 ? bb.w : bb.w * K2};
            auto tail = [&](auto satc) {
                // SAT: the FP8 codes are clamped (activation scale above 448)
#pragma unroll
                for (int t = 0; t < PT; ++t) {
                    float v[4];
                    if constexpr (KN == KFP8) {
                        // FP8 next layer: its codes straight from r (one FMA)
                        float r[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            r[e] = __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(acc[i][t][e] * sc + bv[e]) + 1.0f);
                        put_fp8<NCHN, decltype(satc)::value>(out, t, ot, lane, r, qinv);
                        if (saved)
#pragma unroll
                            for (int e = 0; e < 4; ++e) v[e] = 1.0f - 2.0f * r[e];
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const float z = acc[i][t][e] * sc + bv[e];
                            if constexpr (K == KF32) v[e] = tanhf(z);
                            else v[e] = 1.0f - 2.0f * __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(z) + 1.0f);
                        }
                        if constexpr (SKIP) {
                            // skip connection: + the layer's own input at these units
                            // (an H-wide input of the same kind has the output's layout)
                            static_assert(K == KN && (K == KF32 || K == KBF16), "skip needs equal FP32/BF16 layouts");
                            if constexpr (KN == KF32) {
#pragma unroll
                                for (int e = 0; e < 4; ++e) v[e] += ((const float *)in)[(t * NCHN + 4 * ot + e) * 64 + lane];
                            } else {
                                const uint2 w = *(const uint2 *)(in + ((t * NCHN + (ot >> 1)) * 64 + lane) * 16 + 8 * (ot & 1));
                                v[0] += bf16_to_f32((uint16_t)(w.x & 0xffffu));
                                v[1] += bf16_to_f32((uint16_t)(w.x >> 16));
                                v[2] += bf16_to_f32((uint16_t)(w.y & 0xffffu));
                                v[3] += bf16_to_f32((uint16_t)(w.y >> 16));
                            }
                        }
                        put_act<KN, NCHN>(out, t, ot, lane, v);
                    }
                    if (saved) {
                        int64_t row = base + 16 * t + p;
                        if (row < n) {
                            int64_t idx = save_off + row * H + 16 * ot + 4 * g;
                            if (save_bytes == 4)
                                *(float4 *)((float *)saved + idx) = make_float4(v[0], v[1], v[2], v[3]);
                            else
                                *(uint2 *)((uint16_t *)saved + idx) =
                                    make_uint2(pack_bf16x2_hw(v[0], v[1]), pack_bf16x2_hw(v[2], v[3]));
                        }
                    }
                }
            };
            if constexpr (KN == KFP8) {
                if (qinv > 448.0f) tail(std::true_type{});
                else tail(std::false_type{});
            } else {
                tail(std::false_type{});
            }
        }
    }
}

// LDS sizes of the forward kernels: buffer 0 holds the network input, then
// the layer-3 input; buffer 1 the layer-2 input.
template <int DT, int H, int PT, int J = 1>
struct FwdShape {
    using IO = NetIo<J>;
    static constexpr int K1 = layer_kind(DT, 0), K2 = layer_kind(DT, 1), K3 = layer_kind(DT, 2);
    static constexpr int NCH0 = IO::INP / (4 * kind_E(K1));
    static constexpr int NCH1 = H / (4 * kind_E(K2));
    static constexpr int NCH2 = H / (4 * kind_E(K3));
    static constexpr int IN0 = PT * NCH0 * 64 * frag_bytes(K1);
    static constexpr int IN1 = PT * NCH1 * 64 * frag_bytes(K2);
    static constexpr int IN2 = PT * NCH2 * 64 * frag_bytes(K3);
    static constexpr int YB = 16 * PT * IO::NOUT * 4; // output rows of the tile
    static constexpr int BUF0 = IN0 > IN2 ? IN0 : IN2;
    static constexpr int BUF1 = IN1 > YB ? IN1 : YB;
    // waves per workgroup: 64-patch tiles take 8 waves (two output tiles of
    // a hidden layer each), smaller tiles 4
    static constexpr int NW = PT == 4 ? 8 : 4;
    static constexpr int NTHR = 64 * NW;
};

// Network input rows X [n][ldx] (FP32 or BF16) of patches base .. base + 16 PT
// into the layer-1 fragments: one thread per 16-byte piece of a row, so the
// rows are read contiguously.
template <int K1, int NCH0, int PT, int NTHR, int INP = IN_PAD>
__device__ __forceinline__ void stage_rows(const void *__restrict__ Xv, int64_t ldx, int64_t base, int64_t n,
                                           unsigned char *buf, int tid) {
    constexpr int PIECES = INP * kind_bytes(K1) / 16; // 16-byte pieces per row
    for (int it = tid; it < 16 * PT * PIECES; it += NTHR) {
        const int pl = it / PIECES, pc = it - pl * PIECES;
        const int64_t row = base + pl;
        const int t = pl >> 4, p = pl & 15;
        u32x4 v = u32x4{0u, 0u, 0u, 0u};
        if (row < n) v = *(const u32x4 *)((const unsigned char *)Xv + (row * ldx) * kind_bytes(K1) + 16 * pc);
        if constexpr (K1 == KF32) {
            // columns 4 pc .. 4 pc + 3: chunk pc, lane 16 g + p for g = 0..3
#pragma unroll
            for (int g = 0; g < 4; ++g) ((uint32_t *)buf)[(t * NCH0 + pc) * 64 + 16 * g + p] = v[g];
        } else {
            // columns 8 pc .. 8 pc + 7: chunk pc / 4, lane 16 (pc % 4) + p
            *(u32x4 *)(buf + ((t * NCH0 + (pc >> 2)) * 64 + 16 * (pc & 3) + p) * 16) = v;
        }
    }
}

// One input value of patch slot pl, column col, into the layer-1 fragments.
template <int K1, int NCH0>
__device__ __forceinline__ void put_input(unsigned char *buf, int pl, int col, float v) {
    const int t = pl >> 4, p = pl & 15;
    if constexpr (K1 == KF32) {
        ((float *)buf)[(t * NCH0 + (col >> 2)) * 64 + 16 * (col & 3) + p] = v;
    } else {
        const int w = col & 31;
        *(uint16_t *)(buf + ((t * NCH0 + (col >> 5)) * 64 + 16 * (w >> 3) + p) * 16 + 2 * (w & 7)) = f32_to_bf16_hw(v);
    }
}

// Operator Q of eq. (defQ) with the standardisation, straight into the
// layer-1 fragments: input column 27 c + iota of patch (I,J,K) is field c of
// [u, v, w, r_u, r_v, r_w] at local node iota = a + 3 b + 9 c'; columns
// 162..164 are the geometry inputs (the patch's row of geom, or the coarse
// cell sizes of the box when geom is null), 165..191 zero.  Lanes run over the
// patches of the tile and waves over the local nodes: consecutive patches
// of a row of the coarse mesh read fine nodes two apart, so a wave's load of
// one field touches a few cache lines, and the standardisation constants of
// a wave's node are the same for all its lanes.
template <int K1, int NCH0, int PT, int NTHR>
__device__ __forceinline__ void stage_gather(const Mesh &m, const float *__restrict__ xt, const float *__restrict__ r,
                                             const float *__restrict__ shift, const float *__restrict__ inv,
                                             const float *__restrict__ geom, int64_t base, int64_t n,
                                             unsigned char *buf, int tid) {
    constexpr int NPL = 16 * PT, STEP = NTHR / NPL;
    static_assert(NTHR % NPL == 0, "a thread keeps one patch of the tile");
    const int pl = tid % NPL;
    const int64_t row = base + pl;
    const bool ok = row < n;
    int I = 0, J = 0, K = 0;
    if (ok) {
        const uint32_t JK = fdiv((uint32_t)row, m.px);
        I = (int)((uint32_t)row - JK * m.n[0]);
        K = (int)fdiv(JK, m.py);
        J = (int)(JK - (uint32_t)K * m.n[1]);
    }
    // two of a thread's nodes are requested together (all of them would
    // spill registers in the widest kernels)
#pragma unroll 2
    for (int q = 0; q < (27 + STEP - 1) / STEP; ++q) {
        const int iota = tid / NPL + STEP * q;
        if (iota >= 27) break;
        float v[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (ok) {
            const int a = iota % 3, b = (iota / 3) % 3, c = iota / 9;
            const int i = wrap(2 * I + a, m.nf[0], m.per[0]);
            const int j = wrap(2 * J + b, m.nf[1], m.per[1]);
            const int k = wrap(2 * K + c, m.nf[2], m.per[2]);
            const int64_t node = i + (int64_t)m.nf[0] * (j + (int64_t)m.nf[1] * k);
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                v[f] = xt[f * m.n_fine + node];
                v[3 + f] = r[f * m.n_fine + node];
            }
            // the standardisation constants are requested with the node
            // values (a branch per field would wait for each load in turn)
            float sh[6], sc[6];
            if (shift)
#pragma unroll
                for (int f = 0; f < 6; ++f) sh[f] = shift[27 * f + iota];
            if (inv)
#pragma unroll
                for (int f = 0; f < 6; ++f) sc[f] = inv[27 * f + iota];
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                if (shift) v[f] -= sh[f];
                if (inv) v[f] *= sc[f];
            }
        }
#pragma unroll
        for (int f = 0; f < 6; ++f) put_input<K1, NCH0>(buf, pl, 27 * f + iota, v[f]);
    }
    for (int it = tid; it < 16 * PT * (IN_PAD - 162); it += NTHR) {
        const int pl = it / (IN_PAD - 162), col = 162 + (it - pl * (IN_PAD - 162));
        const int cc = col < N_IN ? col : N_IN - 1;
        const float sh = shift ? shift[cc] : 0.0f, sc = inv ? inv[cc] : 1.0f;
        float v = 0.0f;
        if (col < N_IN && base + pl < n) {
            v = geom ? geom[3 * (base + pl) + (col - 162)] : m.H[col - 162];
            if (shift) v -= sh;
            if (inv) v *= sc;
        }
        put_input<K1, NCH0>(buf, pl, col, v);
    }
}

// Forward pass over tiles of 16 PT patches.  GATHER = false: the inputs are
// the rows of X and tile t covers rows 16 PT t ..; GATHER = true: the inputs
// are gathered from the node fields of the boxes (D, or the single box `one`
// when D is null), and tile -> box by the prefix sums blk_ptile.  Workgroups
// walk the tiles with stride gridDim.x; every thread of a workgroup takes the
// same tiles, so the barriers inside the loop are uniform.
template <int DT, int H, int PT, bool GATHER, int J = 1>
__global__ void __launch_bounds__((FwdShape<DT, H, PT, J>::NTHR))
    k_mlp_fwd(int64_t ntiles, int64_t n_rows, const void *__restrict__ Xv, int64_t ldx,
              const BoxDesc *__restrict__ D, int nbox, BoxDesc one, const float *__restrict__ xt_all,
              const float *__restrict__ r_all, const float *__restrict__ shift, const float *__restrict__ inv,
              const void *__restrict__ W0, const void *__restrict__ W1, const void *__restrict__ W2,
              const float *__restrict__ b0, const float *__restrict__ b1, const float *__restrict__ b2,
              float *__restrict__ Y_all, void *__restrict__ saved, float s1, float q1inv) {
    static_assert(!GATHER || J == 1, "the fused gather is built for one-level patches");
    using S = FwdShape<DT, H, PT, J>;
    constexpr int NO = S::IO::NOUT;
    using F1 = typename Frag<S::K1>::T;
    using F2 = typename Frag<S::K2>::T;
    using F3 = typename Frag<S::K3>::T;
    __shared__ __attribute__((aligned(16))) unsigned char smem[S::BUF0 + S::BUF1];
    unsigned char *buf0 = smem, *buf1 = smem + S::BUF0;
    const int sbytes = DT == DNNMG_F32 ? 4 : 2;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        // the thread index is read anew for each tile (the empty asm hides
        // that it does not change), so the per-lane addresses of the layers
        // are formed where they are used rather than held in registers
        // across the whole loop
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int lane = tid & 63, wave = tid >> 6;
        int64_t base, n;
        float *Y = Y_all;
        if constexpr (GATHER) {
            const int b = D ? find_box(nbox, tile, [&](int i) { return D[i].blk_ptile; }) : 0;
            const BoxDesc &d = D ? D[b] : one;
            n = d.m.n_patches;
            base = (tile - d.blk_ptile) * 16 * PT;
            Y = Y_all + NO * d.off_patch;
            stage_gather<S::K1, S::NCH0, PT, S::NTHR>(d.m, xt_all + 4 * d.off_fine, r_all + 4 * d.off_fine, shift, inv,
                                                      d.geom, base, n, buf0, tid);
        } else {
            n = n_rows;
            base = tile * 16 * PT;
            stage_rows<S::K1, S::NCH0, PT, S::NTHR, S::IO::INP>(Xv, ldx, base, n, buf0, tid);
        }
        lds_barrier();
        layer<S::K1, S::K2, H / 16, S::NCH0, PT, false, H, S::NW>((const F1 *)W0, b0, buf0, buf1, 1.0f, q1inv, wave,
                                                          lane, base, n, Y, saved, 0, sbytes);
        lds_barrier();
        layer<S::K2, S::K3, H / 16, S::NCH1, PT, false, H, S::NW>((const F2 *)W1, b1, buf1, buf0, s1, 1.0f, wave, lane,
                                                          base, n, Y, saved, n * H, sbytes);
        lds_barrier();
        layer<S::K3, S::K3, S::IO::OUTP / 16, S::NCH2, PT, true, H, S::NW, NO>((const F3 *)W2, b2, buf0, buf1, 1.0f,
                                                                                1.0f, wave, lane, base, n, Y, nullptr,
                                                                                0, sbytes);
        lds_barrier();
        {
            // the tile's rows are contiguous in Y
            const int cnt = (int)((n - base < 16 * PT ? n - base : 16 * PT) * NO);
            const float *ys = (const float *)buf1;
            float *yd = Y + base * NO;
            int q0 = 0;
            if ((((uintptr_t)yd) & 15) == 0) {
                for (int q = tid; q < cnt / 4; q += S::NTHR) ((float4 *)yd)[q] = ((const float4 *)ys)[q];
                q0 = cnt / 4 * 4;
            }
            for (int q = q0 + tid; q < cnt; q += S::NTHR) yd[q] = ys[q];
        }
        lds_barrier();
    }
}

// ------------------------------------------------- the paper's network ----
// Sec. 3: f_1 = tanh(N_1(W_1 x)), f_i = tanh(N_i(W_i x)) + x (i = 2 .. D),
// f_L = W_L x, with the batch normalisations N_i folded into the packed
// weights (column scale gamma / s) and a bias (beta - gamma mu / s).  Widths:
// inputs INP (240 -> 256 or 1024), hidden HP (512, or 750 -> 768: the padded
// units have zero weights and bias, so their activations stay exactly 0),
// outputs NO (81 or 375).  Activations ping-pong between two LDS buffers.
struct DeepArgs {
    const void *W[DNNMG_DEEP_MAX_DEPTH + 1];
    const float *b[DNNMG_DEEP_MAX_DEPTH + 1];
};

template <int DT, int HP, int PT, int J>
struct DeepShape {
    static constexpr int INP = J == 1 ? 256 : 1024;
    static constexpr int NO = J == 1 ? 81 : 375, OUTP = J == 1 ? 96 : 384;
    static constexpr int K = DT == DNNMG_F32 ? KF32 : KBF16;
    static constexpr int NCH0 = INP / (4 * kind_E(K)), NCHH = HP / (4 * kind_E(K));
    static constexpr int IN0 = PT * NCH0 * 64 * frag_bytes(K), INH = PT * NCHH * 64 * frag_bytes(K);
    static constexpr int YB = 16 * PT * NO * 4;
    static constexpr int BUF = IN0 > INH ? (IN0 > YB ? IN0 : YB) : (INH > YB ? INH : YB);
    static constexpr int NW = (PT == 4 || HP > 512) ? 8 : 4;
    static constexpr int NTHR = 64 * NW;
    // where two activation buffers would not fit LDS, one buffer and every
    // layer in place
    static constexpr bool ONEBUF = 2 * BUF > 160 * 1024;
    static constexpr int SMEM = ONEBUF ? BUF : 2 * BUF;
};

template <int DT, int HP, int PT, int J>
__global__ void __launch_bounds__((DeepShape<DT, HP, PT, J>::NTHR))
    k_deep_fwd(int64_t ntiles, int64_t n, const void *__restrict__ Xv, int64_t ldx, DeepArgs a, int depth,
               float *__restrict__ Y) {
    using S = DeepShape<DT, HP, PT, J>;
    using F = typename Frag<S::K>::T;
    __shared__ __attribute__((aligned(16))) unsigned char smem[S::SMEM];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr bool IP = S::ONEBUF;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t base = tile * 16 * PT;
        unsigned char *cur = smem, *nxt = IP ? smem : smem + S::BUF;
        stage_rows<S::K, S::NCH0, PT, S::NTHR, S::INP>(Xv, ldx, base, n, cur, tid);
        lds_barrier();
        layer<S::K, S::K, HP / 16, S::NCH0, PT, false, HP, S::NW, N_OUT, false, IP>(
            (const F *)a.W[0], a.b[0], cur, nxt, 1.0f, 1.0f, wave, lane, base, n, Y, nullptr, 0, 0);
        lds_barrier();
        for (int l = 1; l < depth; ++l) {
            unsigned char *t = cur;
            cur = nxt;
            nxt = t;
            layer<S::K, S::K, HP / 16, S::NCHH, PT, false, HP, S::NW, S::NO, true, IP>(
                (const F *)a.W[l], a.b[l], cur, nxt, 1.0f, 1.0f, wave, lane, base, n, Y, nullptr, 0, 0);
            lds_barrier();
        }
        layer<S::K, S::K, S::OUTP / 16, S::NCHH, PT, true, HP, S::NW, S::NO, false, IP>(
            (const F *)a.W[depth], a.b[depth], nxt, cur, 1.0f, 1.0f, wave, lane, base, n, Y, nullptr, 0, 0);
        lds_barrier();
        {
            const int cnt = (int)((n - base < 16 * PT ? n - base : 16 * PT) * S::NO);
            const float *ys = (const float *)cur;
            float *yd = Y + base * S::NO;
            int q0 = 0;
            if ((((uintptr_t)yd) & 15) == 0) {
                for (int q = tid; q < cnt / 4; q += S::NTHR) ((float4 *)yd)[q] = ((const float4 *)ys)[q];
                q0 = cnt / 4 * 4;
            }
            for (int q = q0 + tid; q < cnt; q += S::NTHR) yd[q] = ys[q];
        }
        lds_barrier();
    }
}

// batch normalisation folded into a layer: colscale = gamma / s, bias =
// beta - gamma mu / s for the H real units, 0 for the padding up to HP
__global__ void __launch_bounds__(256) k_bn_fold(int H, int HP, const float *__restrict__ gamma,
                                                 const float *__restrict__ beta, const float *__restrict__ mean,
                                                 const float *__restrict__ sd, float *__restrict__ colscale,
                                                 float *__restrict__ bias) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= HP) return;
    if (u >= H) {
        bias[u] = 0.0f;
        return;
    }
    const float c = gamma[u] / sd[u];
    colscale[u] = c;
    bias[u] = beta[u] - c * mean[u];
}

__global__ void __launch_bounds__(256) k_zero_f32(int n, float *__restrict__ p) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n) p[u] = 0.0f;
}

// Instantiated (dtype, padded width, PT, J) variants of the paper's network.
#define DNNMG_DEEP_VARIANTS(X)                                                                          \
    X(DNNMG_F32, 512, 1, 1) X(DNNMG_F32, 768, 1, 1) X(DNNMG_BF16, 512, 2, 1) X(DNNMG_BF16, 512, 4, 1)     \
    X(DNNMG_BF16, 768, 1, 1) X(DNNMG_BF16, 768, 2, 1) X(DNNMG_BF16, 768, 4, 1)                            \
    X(DNNMG_F32, 512, 1, 2) X(DNNMG_F32, 768, 1, 2) X(DNNMG_BF16, 512, 1, 2) X(DNNMG_BF16, 512, 2, 2)     \
    X(DNNMG_BF16, 768, 1, 2) X(DNNMG_BF16, 768, 2, 2)

static int deep_levels(int n_in, int n_out) {
    if (n_in == 240 && n_out == 81) return 1;
    if (n_in == 1024 && n_out == 375) return 2;
    return 0;
}
static int deep_hpad(int hidden) { return (hidden + 255) / 256 * 256; }

static void fp8_scales(const dnnmg_mlp *net, float &s1, float &q1) {
    s1 = 1.f;
    q1 = 1.f;
    if (net->dtype == DNNMG_FP8_E4M3) {
        // only the hidden product is FP8: its weights (w_scale[1]) and its
        // input activations (a_scale[1]) carry scales
        s1 = net->w_scale[1] * net->a_scale[1];
        q1 = 1.0f / net->a_scale[1];
    }
}

// Instantiated (dtype, width, PT) forward variants.
#define DNNMG_FWD_VARIANTS(X)                                                                           \
    X(DNNMG_F32, 64, 1) X(DNNMG_F32, 64, 2) X(DNNMG_F32, 128, 1) X(DNNMG_F32, 128, 2)                   \
    X(DNNMG_F32, 256, 1) X(DNNMG_F32, 256, 2) X(DNNMG_F32, 512, 1) X(DNNMG_F32, 512, 2)                  \
    X(DNNMG_BF16, 64, 1) X(DNNMG_BF16, 64, 2) X(DNNMG_BF16, 64, 4)                                       \
    X(DNNMG_BF16, 128, 1) X(DNNMG_BF16, 128, 2) X(DNNMG_BF16, 128, 4)                                    \
    X(DNNMG_BF16, 256, 1) X(DNNMG_BF16, 256, 2) X(DNNMG_BF16, 256, 4)                                    \
    X(DNNMG_BF16, 512, 1) X(DNNMG_BF16, 512, 2) X(DNNMG_BF16, 512, 4)                                    \
    X(DNNMG_FP8_E4M3, 128, 1) X(DNNMG_FP8_E4M3, 128, 2) X(DNNMG_FP8_E4M3, 128, 4)                        \
    X(DNNMG_FP8_E4M3, 256, 1) X(DNNMG_FP8_E4M3, 256, 2) X(DNNMG_FP8_E4M3, 256, 4)                        \
    X(DNNMG_FP8_E4M3, 512, 1) X(DNNMG_FP8_E4M3, 512, 2) X(DNNMG_FP8_E4M3, 512, 4)

// Variants of the two-level prediction (753 inputs, 375 outputs): tiles of
// 16 or 32 patches (the 768-wide input rows of 64 patches would not fit LDS).
#define DNNMG_FWD_VARIANTS2(X)                                                                          \
    X(DNNMG_F32, 256, 1) X(DNNMG_BF16, 256, 1) X(DNNMG_BF16, 256, 2) X(DNNMG_BF16, 512, 1)              \
    X(DNNMG_BF16, 512, 2) X(DNNMG_FP8_E4M3, 512, 1) X(DNNMG_FP8_E4M3, 512, 2)

bool fwd_has_pt(const dnnmg_mlp *net, int pt) {
    const int J = net_levels(net->n_in, net->n_out);
#define HAS(DT, HH, P)                                                                                  \
    if (net->dtype == DT && net->hidden == HH && pt == P) return true;
    if (J == 1) {
        DNNMG_FWD_VARIANTS(HAS)
    } else if (J == 2) {
        DNNMG_FWD_VARIANTS2(HAS)
    }
#undef HAS
    return false;
}

// Patches per tile of 16 PT: the largest instantiated PT that still gives
// every compute unit a tile, else 1.
int fwd_default_pt(const dnnmg_mlp *net, int64_t n, int ncu) {
    for (int pt = 4; pt > 1; pt /= 2)
        if (fwd_has_pt(net, pt) && n >= (int64_t)ncu * 16 * pt) return pt;
    return 1;
}

int fwd_launch(const dnnmg_mlp *net, int pt, bool gather, int64_t ntiles, int grid, int64_t n_rows,
               const void *X, int64_t ldx, const BoxDesc *D, int nbox, const BoxDesc &one, const float *xt,
               const float *r, const float *shift, const float *inv, float *Y, void *saved, hipStream_t s) {
    float s1, q1;
    fp8_scales(net, s1, q1);
    if (ntiles <= 0) return DNNMG_OK;
    if (grid <= 0 || grid > ntiles) grid = (int)ntiles;
#define LAUNCH(DT, HH, P)                                                                               \
    if (net->dtype == DT && net->hidden == HH && pt == P) {                                             \
        if (gather)                                                                                     \
            k_mlp_fwd<DT, HH, P, true><<<grid, FwdShape<DT, HH, P>::NTHR, 0, s>>>(ntiles, 0, nullptr, 0, D, nbox, one, xt, r,  \
                                                            shift, inv, net->W[0], net->W[1], net->W[2], \
                                                            net->b[0], net->b[1], net->b[2], Y, nullptr, \
                                                            s1, q1);                                     \
        else                                                                                            \
            k_mlp_fwd<DT, HH, P, false><<<grid, FwdShape<DT, HH, P>::NTHR, 0, s>>>(ntiles, n_rows, X, ldx, nullptr, 0, one,    \
                                                             nullptr, nullptr, nullptr, nullptr,        \
                                                             net->W[0], net->W[1], net->W[2], net->b[0], \
                                                             net->b[1], net->b[2], Y, saved, s1, q1);    \
        return hip_check(hipGetLastError(), "patch network forward launch");                            \
    }
    if (net_levels(net->n_in, net->n_out) == 1) {
        DNNMG_FWD_VARIANTS(LAUNCH)
    }
#undef LAUNCH
#define LAUNCH2(DT, HH, P)                                                                              \
    if (net->dtype == DT && net->hidden == HH && pt == P) {                                             \
        if (gather) return fail(DNNMG_ERR_UNSUPPORTED, "patch network forward: no fused gather for J = 2"); \
        k_mlp_fwd<DT, HH, P, false, 2><<<grid, FwdShape<DT, HH, P, 2>::NTHR, 0, s>>>(                    \
            ntiles, n_rows, X, ldx, nullptr, 0, one, nullptr, nullptr, nullptr, nullptr, net->W[0], net->W[1], \
            net->W[2], net->b[0], net->b[1], net->b[2], Y, saved, s1, q1);                               \
        return hip_check(hipGetLastError(), "patch network forward launch");                            \
    }
    if (net_levels(net->n_in, net->n_out) == 2) {
        DNNMG_FWD_VARIANTS2(LAUNCH2)
    }
#undef LAUNCH2
    return fail(DNNMG_ERR_UNSUPPORTED, "patch network forward: dtype %d width %d tile %d", net->dtype,
                net->hidden, pt);
}

int device_cus() {
    static int ncu = 0;
    if (!ncu) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            ncu = v;
        else
            ncu = 256;
    }
    return ncu;
}

int check_net(const dnnmg_mlp *net) {
    if (!net) return fail(DNNMG_ERR_ARG, "net is NULL");
    if (!net_levels(net->n_in, net->n_out))
        return fail(DNNMG_ERR_SHAPE, "network must be %d -> H -> H -> %d or %d -> H -> H -> %d (got %d, %d)",
                    NetIo<1>::NIN, NetIo<1>::NOUT, NetIo<2>::NIN, NetIo<2>::NOUT, net->n_in, net->n_out);
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

extern "C" size_t dnnmg_mlp_packed_bytes_io(int dtype, int n_in, int hidden, int n_out, int layer) {
    const int J = net_levels(n_in, n_out);
    if (!J || layer < 0 || layer > 2) return 0;
    if (dtype != DNNMG_F32 && dtype != DNNMG_BF16 && dtype != DNNMG_FP8_E4M3) return 0;
    int kp = layer == 0 ? io_in_pad(J) : hidden;
    int np = layer == 2 ? io_out_pad(J) : hidden;
    return (size_t)kp * np * kind_bytes(layer_kind(dtype, layer));
}

extern "C" size_t dnnmg_mlp_packed_bytes(int dtype, int hidden, int layer) {
    return dnnmg_mlp_packed_bytes_io(dtype, N_IN, hidden, N_OUT, layer);
}

extern "C" int dnnmg_mlp_pack_io(int dtype, int n_in, int hidden, int n_out, int layer, const float *W,
                                 float w_scale, void *Wp, void *stream) {
    const int J = net_levels(n_in, n_out);
    if (!J) return fail(DNNMG_ERR_SHAPE, "dnnmg_mlp_pack: widths %d -> %d not supported", n_in, n_out);
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
    int fan_in = layer == 0 ? n_in : hidden;
    int fan_out = layer == 2 ? n_out : hidden;
    int kp = layer == 0 ? io_in_pad(J) : hidden;
    int np = layer == 2 ? io_out_pad(J) : hidden;
    int E = kind_E(kind);
    int ntiles = np / 16, nchunks = kp / (4 * E);
    int64_t total = (int64_t)ntiles * nchunks * 64 * E;
    hipStream_t s = (hipStream_t)stream;
    unsigned grid = blocks_for(total, 256);
    if (kind == KF32)
        k_pack<float><<<grid, 256, 0, s>>>(kind, layer, fan_in, fan_out, ntiles, nchunks, W, 1.f, (float *)Wp,
                                           nullptr);
    else if (kind == KBF16)
        k_pack<uint16_t><<<grid, 256, 0, s>>>(kind, layer, fan_in, fan_out, ntiles, nchunks, W, 1.f,
                                              (uint16_t *)Wp, nullptr);
    else
        k_pack<uint8_t><<<grid, 256, 0, s>>>(kind, layer, fan_in, fan_out, ntiles, nchunks, W,
                                             1.f / w_scale, (uint8_t *)Wp, nullptr);
    return hip_check(hipGetLastError(), "dnnmg_mlp_pack launch");
}

extern "C" int dnnmg_mlp_pack(int dtype, int hidden, int layer, const float *W, float w_scale,
                              void *Wp, void *stream) {
    return dnnmg_mlp_pack_io(dtype, N_IN, hidden, N_OUT, layer, W, w_scale, Wp, stream);
}

// max |w| over n weights as the bit pattern of a non-negative float (the
// integer order of such patterns is their numeric order, and a NaN compares
// above +inf), combined across workgroups with an atomic maximum, so the
// result does not depend on the order of the workgroups.
__global__ void __launch_bounds__(256) k_amax_init(unsigned *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = 0u;
}

__global__ void __launch_bounds__(256) k_amax(int64_t n, const float *__restrict__ W, unsigned *__restrict__ out) {
    unsigned m = 0u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, __float_as_uint(W[i]) & 0x7fffffffu);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, o));
    if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

extern "C" int dnnmg_mlp_prepare_io(int dtype, int n_in, int hidden, int n_out, const float *const W[3],
                                    const float *const b[3], void *const Wp[3], void *ws, size_t ws_bytes,
                                    dnnmg_mlp *net, void *stream) {
    if (!W || !b || !Wp || !net) return fail(DNNMG_ERR_ARG, "dnnmg_mlp_prepare: NULL pointer");
    if (!net_levels(n_in, n_out))
        return fail(DNNMG_ERR_SHAPE, "dnnmg_mlp_prepare: widths %d -> %d not supported", n_in, n_out);
    if (hidden != 64 && hidden != 128 && hidden != 256 && hidden != 512)
        return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_mlp_prepare: hidden %d", hidden);
    if (dtype != DNNMG_F32 && dtype != DNNMG_BF16 && dtype != DNNMG_FP8_E4M3)
        return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_mlp_prepare: dtype %d", dtype);
    if (dtype == DNNMG_FP8_E4M3 && hidden < 128)
        return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_mlp_prepare: FP8 needs hidden >= 128");
    for (int l = 0; l < 3; ++l) {
        if (!W[l] || !b[l] || !Wp[l]) return fail(DNNMG_ERR_ARG, "dnnmg_mlp_prepare: W/b/Wp[%d] is NULL", l);
        if (!aligned16(Wp[l]) || !aligned16(b[l]))
            return fail(DNNMG_ERR_ARG, "dnnmg_mlp_prepare: Wp/b[%d] not 16-byte aligned", l);
    }
    if (!ws || !aligned16(ws) || ws_bytes < 256)
        return fail(DNNMG_ERR_ARG, "dnnmg_mlp_prepare: workspace must be >= 256 bytes, 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    float w_scale[3] = {1.f, 1.f, 1.f}, a_scale[3] = {1.f, 1.f, 1.f};
    if (dtype == DNNMG_FP8_E4M3) {
        const int64_t n = (int64_t)hidden * hidden;
        unsigned *d = (unsigned *)ws;
        k_amax_init<<<1, 64, 0, s>>>(d);
        k_amax<<<(unsigned)std::min<int64_t>(blocks_for(n, 256), 1024), 256, 0, s>>>(n, W[1], d);
        int rc = hip_check(hipGetLastError(), "dnnmg_mlp_prepare: amax launch");
        if (rc) return rc;
        unsigned bits = 0;
        if ((rc = hip_check(hipMemcpyAsync(&bits, d, sizeof bits, hipMemcpyDeviceToHost, s),
                            "dnnmg_mlp_prepare: amax read-back")))
            return rc;
        if ((rc = hip_check(hipStreamSynchronize(s), "dnnmg_mlp_prepare: synchronise"))) return rc;
        float amax;
        memcpy(&amax, &bits, sizeof amax);
        if (!(amax > 0.f) || !std::isfinite(amax))
            return fail(DNNMG_ERR_ARG, "dnnmg_mlp_prepare: max |W2| = %g (needs a finite value > 0)", (double)amax);
        w_scale[1] = amax / 448.f;
        a_scale[1] = 1.f / 448.f;
    }
    for (int l = 0; l < 3; ++l) {
        int rc = dnnmg_mlp_pack_io(dtype, n_in, hidden, n_out, l, W[l], w_scale[l], Wp[l], stream);
        if (rc) return rc;
    }
    net->n_in = n_in;
    net->hidden = hidden;
    net->n_out = n_out;
    net->dtype = dtype;
    for (int l = 0; l < 3; ++l) {
        net->W[l] = Wp[l];
        net->b[l] = b[l];
        net->w_scale[l] = w_scale[l];
        net->a_scale[l] = a_scale[l];
    }
    return DNNMG_OK;
}

extern "C" int dnnmg_mlp_prepare(int dtype, int hidden, const float *const W[3], const float *const b[3],
                                 void *const Wp[3], void *ws, size_t ws_bytes, dnnmg_mlp *net, void *stream) {
    return dnnmg_mlp_prepare_io(dtype, N_IN, hidden, N_OUT, W, b, Wp, ws, ws_bytes, net, stream);
}

extern "C" size_t dnnmg_patch_saved_bytes(const dnnmg_mlp *net, int64_t n) {
    if (!net) return 0;
    size_t es = net->dtype == DNNMG_F32 ? 4 : net->dtype == DNNMG_BF16 ? 2 : 0;
    return (size_t)2 * n * net->hidden * es;
}

extern "C" int dnnmg_patch_forward_tiles(const dnnmg_mlp *net, int64_t n, const void *X, int64_t ldx, float *Y,
                                         void *saved, int tile_patches, int grid, void *stream);

extern "C" int dnnmg_patch_forward(const dnnmg_mlp *net, int64_t n, const void *X, int64_t ldx,
                                   float *Y, void *saved, void *stream) {
    return dnnmg_patch_forward_tiles(net, n, X, ldx, Y, saved, 0, 0, stream);
}

extern "C" int dnnmg_patch_forward_tiles(const dnnmg_mlp *net, int64_t n, const void *X, int64_t ldx, float *Y,
                                         void *saved, int tile_patches, int grid, void *stream) {
    int rc = check_net(net);
    if (rc) return rc;
    if (n < 0) return fail(DNNMG_ERR_SHAPE, "dnnmg_patch_forward: n < 0");
    if (n == 0) return DNNMG_OK;
    if (!X || !Y) return fail(DNNMG_ERR_ARG, "dnnmg_patch_forward: NULL pointer");
    if (!aligned16(X)) return fail(DNNMG_ERR_ARG, "dnnmg_patch_forward: X not 16-byte aligned");
    int align = net->dtype == DNNMG_F32 ? 4 : 8;
    const int inp = io_in_pad(net_levels(net->n_in, net->n_out));
    if (ldx < inp || ldx % align)
        return fail(DNNMG_ERR_SHAPE, "dnnmg_patch_forward: ldx %lld must be >= %d and a multiple of %d",
                    (long long)ldx, inp, align);
    if (saved && net->dtype == DNNMG_FP8_E4M3)
        return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_patch_forward: FP8 networks do not save activations");
    if (saved && !aligned16(saved)) return fail(DNNMG_ERR_ARG, "dnnmg_patch_forward: saved not aligned");
    if (grid < 0) return fail(DNNMG_ERR_ARG, "dnnmg_patch_forward: grid < 0");
    int pt = fwd_default_pt(net, n, device_cus());
    if (tile_patches) {
        pt = tile_patches / 16;
        if (tile_patches % 16 || !fwd_has_pt(net, pt))
            return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_patch_forward: %d patches per tile not built for this network",
                        tile_patches);
    }
    const int64_t ntiles = (n + 16 * pt - 1) / (16 * pt);
    BoxDesc none{};
    return fwd_launch(net, pt, false, ntiles, grid, n, X, ldx, nullptr, 0, none, nullptr, nullptr, nullptr, nullptr,
                      Y, saved, (hipStream_t)stream);
}

static int gather_forward(const dnnmg_box *box, const dnnmg_mlp *net, const float *geom, const float *xt,
                          const float *r, const dnnmg_feat *feat, float *Y, void *stream) {
    int rc = check_net(net);
    if (rc) return rc;
    if (net->n_in != N_IN)
        return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_patch_gather_forward: one-level patches only (%d inputs)", N_IN);
    BoxDesc one{};
    if ((rc = make_mesh(box, &one.m))) return rc;
    if (!xt || !r || !Y) return fail(DNNMG_ERR_ARG, "dnnmg_patch_gather_forward: NULL pointer");
    one.geom = geom;
    const float *sh = feat ? feat->shift : nullptr;
    const float *sc = feat ? feat->inv_scale : nullptr;
    const int pt = fwd_default_pt(net, one.m.n_patches, device_cus());
    const int64_t ntiles = (one.m.n_patches + 16 * pt - 1) / (16 * pt);
    return fwd_launch(net, pt, true, ntiles, 0, 0, nullptr, 0, nullptr, 1, one, xt, r, sh, sc, Y, nullptr,
                      (hipStream_t)stream);
}

extern "C" int dnnmg_patch_gather_forward(const dnnmg_box *box, const dnnmg_mlp *net, const float *xt,
                                          const float *r, const dnnmg_feat *feat, float *Y, void *stream) {
    return gather_forward(box, net, nullptr, xt, r, feat, Y, stream);
}

extern "C" int dnnmg_patch_gather_forward_geom(const dnnmg_box *box, const dnnmg_mlp *net, const float *geom,
                                               const float *xt, const float *r, const dnnmg_feat *feat, float *Y,
                                               void *stream) {
    if (!geom) return fail(DNNMG_ERR_ARG, "dnnmg_patch_gather_forward_geom: geom is NULL");
    return gather_forward(box, net, geom, xt, r, feat, Y, stream);
}

// ------------------------------------------------- the paper's network ----
extern "C" int dnnmg_deepnet_widths(int n_in, int hidden, int n_out, int *in_pad, int *hidden_pad, int *out_pad) {
    const int J = deep_levels(n_in, n_out);
    if (!J) return fail(DNNMG_ERR_SHAPE, "paper network widths %d -> %d (240 -> 81 or 1024 -> 375)", n_in, n_out);
    if (hidden != 512 && hidden != 750)
        return fail(DNNMG_ERR_UNSUPPORTED, "paper network hidden width %d (512 or 750)", hidden);
    if (in_pad) *in_pad = J == 1 ? 256 : 1024;
    if (hidden_pad) *hidden_pad = deep_hpad(hidden);
    if (out_pad) *out_pad = J == 1 ? 96 : 384;
    return DNNMG_OK;
}

extern "C" size_t dnnmg_deepnet_packed_bytes(int dtype, int n_in, int hidden, int n_out, int depth, int layer) {
    int ip, hp, op;
    if (dnnmg_deepnet_widths(n_in, hidden, n_out, &ip, &hp, &op)) return 0;
    if (dtype != DNNMG_F32 && dtype != DNNMG_BF16) return 0;
    if (depth < 2 || depth > DNNMG_DEEP_MAX_DEPTH || layer < 0 || layer > depth) return 0;
    const int kp = layer == 0 ? ip : hp, np = layer == depth ? op : hp;
    return (size_t)kp * np * (dtype == DNNMG_F32 ? 4 : 2);
}

extern "C" int dnnmg_deepnet_prepare(int dtype, int n_in, int hidden, int n_out, int depth, const float *const W[],
                                     const float *const gamma[], const float *const beta[],
                                     const float *const mean[], const float *const sd[], void *const Wp[],
                                     float *const bias[], void *ws, size_t ws_bytes, dnnmg_deepnet *net,
                                     void *stream) {
    int ip, hp, op, rc;
    if ((rc = dnnmg_deepnet_widths(n_in, hidden, n_out, &ip, &hp, &op))) return rc;
    if (dtype != DNNMG_F32 && dtype != DNNMG_BF16)
        return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_deepnet_prepare: dtype %d (FP32 or BF16)", dtype);
    if (depth < 2 || depth > DNNMG_DEEP_MAX_DEPTH)
        return fail(DNNMG_ERR_ARG, "dnnmg_deepnet_prepare: depth %d not in 2..%d", depth, DNNMG_DEEP_MAX_DEPTH);
    if (!W || !gamma || !beta || !mean || !sd || !Wp || !bias || !net || !ws)
        return fail(DNNMG_ERR_ARG, "dnnmg_deepnet_prepare: NULL pointer");
    if (ws_bytes < sizeof(float) * (size_t)hp || !aligned16(ws))
        return fail(DNNMG_ERR_ARG, "dnnmg_deepnet_prepare: workspace needs %zu bytes, 16-byte aligned",
                    sizeof(float) * (size_t)hp);
    for (int l = 0; l <= depth; ++l) {
        if (!W[l] || !Wp[l] || !bias[l] || !aligned16(Wp[l]) || !aligned16(bias[l]))
            return fail(DNNMG_ERR_ARG, "dnnmg_deepnet_prepare: layer %d pointers NULL or misaligned", l);
        if (l < depth && (!gamma[l] || !beta[l] || !mean[l] || !sd[l]))
            return fail(DNNMG_ERR_ARG, "dnnmg_deepnet_prepare: normalisation %d NULL", l);
    }
    hipStream_t s = (hipStream_t)stream;
    float *colscale = (float *)ws;
    const int kind = dtype == DNNMG_F32 ? KF32 : KBF16, E = kind_E(kind);
    for (int l = 0; l <= depth; ++l) {
        const bool last = l == depth;
        const int fan_in = l == 0 ? n_in : hidden, fan_out = last ? n_out : hidden;
        const int kp = l == 0 ? ip : hp, np = last ? op : hp;
        // packing slot order: direct input columns for the first layer, the
        // accumulator layout of the previous layer for the others
        const int lk = l == 0 ? 0 : 1;
        if (!last)
            k_bn_fold<<<blocks_for(hp, 256), 256, 0, s>>>(hidden, hp, gamma[l], beta[l], mean[l], sd[l], colscale,
                                                        bias[l]);
        else
            k_zero_f32<<<blocks_for(op, 256), 256, 0, s>>>(op, bias[l]);
        const int ntiles = np / 16, nchunks = kp / (4 * E);
        const int64_t total = (int64_t)ntiles * nchunks * 64 * E;
        if (kind == KF32)
            k_pack<float><<<blocks_for(total, 256), 256, 0, s>>>(kind, lk, fan_in, fan_out, ntiles, nchunks, W[l],
                                                                 1.f, (float *)Wp[l], last ? nullptr : colscale);
        else
            k_pack<uint16_t><<<blocks_for(total, 256), 256, 0, s>>>(kind, lk, fan_in, fan_out, ntiles, nchunks, W[l],
                                                                    1.f, (uint16_t *)Wp[l],
                                                                    last ? nullptr : colscale);
    }
    if ((rc = hip_check(hipGetLastError(), "dnnmg_deepnet_prepare launch"))) return rc;
    net->n_in = n_in;
    net->hidden = hidden;
    net->n_out = n_out;
    net->depth = depth;
    net->dtype = dtype;
    for (int l = 0; l <= DNNMG_DEEP_MAX_DEPTH; ++l) {
        net->W[l] = l <= depth ? Wp[l] : nullptr;
        net->b[l] = l <= depth ? bias[l] : nullptr;
    }
    return DNNMG_OK;
}

extern "C" int dnnmg_deepnet_forward(const dnnmg_deepnet *net, int64_t n, const void *X, int64_t ldx, float *Y,
                                     void *stream) {
    if (!net) return fail(DNNMG_ERR_ARG, "dnnmg_deepnet_forward: net is NULL");
    int ip, hp, op, rc;
    if ((rc = dnnmg_deepnet_widths(net->n_in, net->hidden, net->n_out, &ip, &hp, &op))) return rc;
    if (net->depth < 2 || net->depth > DNNMG_DEEP_MAX_DEPTH)
        return fail(DNNMG_ERR_ARG, "dnnmg_deepnet_forward: depth %d", net->depth);
    if (n < 0) return fail(DNNMG_ERR_SHAPE, "dnnmg_deepnet_forward: n < 0");
    if (n == 0) return DNNMG_OK;
    if (!X || !Y || !aligned16(X)) return fail(DNNMG_ERR_ARG, "dnnmg_deepnet_forward: X/Y NULL or X misaligned");
    const int align = net->dtype == DNNMG_F32 ? 4 : 8;
    if (ldx < ip || ldx % align)
        return fail(DNNMG_ERR_SHAPE, "dnnmg_deepnet_forward: ldx %lld must be >= %d and a multiple of %d",
                    (long long)ldx, ip, align);
    DeepArgs a{};
    for (int l = 0; l <= net->depth; ++l) {
        if (!net->W[l] || !net->b[l]) return fail(DNNMG_ERR_ARG, "dnnmg_deepnet_forward: layer %d NULL", l);
        a.W[l] = net->W[l];
        a.b[l] = net->b[l];
    }
    const int J = deep_levels(net->n_in, net->n_out);
    const int ncu = device_cus();
    // the largest built tile that still gives every compute unit work
    int pt = 0;
#define PICK(DT, H, P, JJ)                                                                              \
    if (net->dtype == DT && hp == H && J == JJ && (pt == 0 || (P > pt && n >= (int64_t)ncu * 16 * P))) pt = P;
    DNNMG_DEEP_VARIANTS(PICK)
#undef PICK
    if (!pt) return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_deepnet_forward: dtype %d width %d not built", net->dtype, hp);
    const int64_t ntiles = (n + 16 * pt - 1) / (16 * pt);
    hipStream_t s = (hipStream_t)stream;
#define LAUNCH(DT, H, P, JJ)                                                                            \
    if (net->dtype == DT && hp == H && J == JJ && pt == P) {                                            \
        k_deep_fwd<DT, H, P, JJ><<<(unsigned)ntiles, DeepShape<DT, H, P, JJ>::NTHR, 0, s>>>(ntiles, n, X, ldx, a, \
                                                                                          net->depth, Y); \
        return hip_check(hipGetLastError(), "dnnmg_deepnet_forward launch");                            \
    }
    DNNMG_DEEP_VARIANTS(LAUNCH)
#undef LAUNCH
    return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_deepnet_forward: no variant");
}
