// Training kernels for the patch network (arXiv 2307.14837, Sec. 4.2 training
// objective; Sec. 3 AdamW): gradient of the patch loss, backward pass through
// the two tanh layers, and the AdamW update on FP32 master weights.
//
// The backward pass is five products of the forward's shapes:
//   dZ2 = (dY W3^T) (.) (1 - A2^2),   dZ1 = (dZ2 W2^T) (.) (1 - A1^2)
//   dW3 = A2^T dY,  dW2 = A1^T dZ2,  dW1 = X^T dZ1,  db = column sums
// (of dY, dZ2, dZ1, summed from the tiles the weight-gradient products stage).
// For an FP32 network they run on one tiled GEMM kernel (64x64 output tiles,
// LDS-staged operands, v_mfma_f32_16x16x4f32); for a BF16 network on BF16
// MFMA kernels with the operands rounded to BF16 as in the forward pass (the
// dZ products of widths 128 and 256 weight-stationary, W^T in registers,
// writing dZ in BF16 as its consumers stage it and summing its columns for
// the bias gradients).
// All accumulate in FP32.  The weight gradients reduce over patches; they are
// split over K (patch ranges) and the partial tiles are summed in a fixed
// order, so results are run-to-run identical.
#include "common.hpp"
#include "lowp.hpp"
#include "mlp.hpp"

namespace dnnmg {

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T> __device__ __forceinline__ float ld(const T *p, int64_t i);
template <> __device__ __forceinline__ float ld<float>(const float *p, int64_t i) { return p[i]; }
template <> __device__ __forceinline__ float ld<uint16_t>(const uint16_t *p, int64_t i) {
    return bf16_to_f32(p[i]);
}

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int STAGE = BM * BK / 256; // elements of each operand a thread stages per K step

// C[M x N] (+= split) = op(A) op(B); op(A)[m][k] = TA ? A[k*lda + m] : A[m*lda + k],
// op(B)[k][n] = TB ? B[n*ldb + k] : B[k*ldb + n].  EPI: C *= (1 - S[m][n]^2).
// blockIdx.z = split index over K; C + z*M*N receives that split's partial.
// The next K step's operands are loaded into registers while the current
// step's products run (one memory round trip per step, overlapped).
// colsum != NULL: the blocks of the first M tile also sum op(B) over their
// K range from the staged tiles (colsum + z*N: the column sums of B over
// split z, in K order), which gives the bias gradients without another pass.
template <bool TA, bool TB, typename TAe, typename TBe, typename TSe, bool EPI>
__global__ void __launch_bounds__(256)
    k_gemm(int64_t M, int64_t N, int64_t K, int64_t kchunk, const TAe *__restrict__ A, int64_t lda,
           const TBe *__restrict__ B, int64_t ldb, float *__restrict__ C, int64_t ldc,
           const TSe *__restrict__ S, int64_t lds_, float *__restrict__ colsum) {
    __shared__ float As[BK][BM + 4];
    __shared__ float Bs[BK][BN + 4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t m0 = (int64_t)blockIdx.x * BM, n0 = (int64_t)blockIdx.y * BN;
    const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
    const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    const int g = lane >> 4, i16 = lane & 15;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    float ra[STAGE], rb[STAGE];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int r = 0; r < STAGE; ++r) {
            const int e = tid + 256 * r;
            int mm, kk;
            if (TA) { mm = e % BM; kk = e / BM; } else { kk = e % BK; mm = e / BK; }
            // out-of-range elements read the last row / column (k0 < kend,
            // M, N >= 1): the loads carry no branch and go out together;
            // store() zeroes them
            int64_t gm = m0 + mm, gk = k0 + kk;
            gm = gm < M ? gm : M - 1;
            gk = gk < kend ? gk : kend - 1;
            ra[r] = TA ? ld(A, gk * lda + gm) : ld(A, gm * lda + gk);
            int nn;
            if (TB) { kk = e % BK; nn = e / BK; } else { nn = e % BN; kk = e / BN; }
            int64_t gn = n0 + nn;
            gn = gn < N ? gn : N - 1;
            gk = k0 + kk;
            gk = gk < kend ? gk : kend - 1;
            rb[r] = TB ? ld(B, gn * ldb + gk) : ld(B, gk * ldb + gn);
        }
    };
    auto store = [&](int64_t k0) {
#pragma unroll
        for (int r = 0; r < STAGE; ++r) {
            const int e = tid + 256 * r;
            int mm, kk, nn, kb;
            if (TA) { mm = e % BM; kk = e / BM; } else { kk = e % BK; mm = e / BK; }
            if (TB) { kb = e % BK; nn = e / BK; } else { nn = e % BN; kb = e / BN; }
            const float va = (m0 + mm < M && k0 + kk < kend) ? ra[r] : 0.f;
            const float vb = (n0 + nn < N && k0 + kb < kend) ? rb[r] : 0.f;
            if (TA) As[e / BM][e % BM] = va;
            else As[e % BK][e / BK] = va;
            if (TB) Bs[e % BK][e / BK] = vb;
            else Bs[e / BN][e % BN] = vb;
        }
    };
    const bool csum = colsum && blockIdx.x == 0 && tid < BN;
    float cs = 0.f;
    if (kbeg < kend) load(kbeg);
    for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
        store(k0);
        __syncthreads();
        if (k0 + BK < kend) load(k0 + BK);
        if (csum)
#pragma unroll
            for (int kk = 0; kk < BK; ++kk) cs += Bs[kk][tid];
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            float af[2], bfv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) af[a] = As[ks + g][wm + 16 * a + i16];
#pragma unroll
            for (int b = 0; b < 2; ++b) bfv[b] = Bs[ks + g][wn + 16 * b + i16];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[a], bfv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    if (csum && n0 + tid < N) colsum[(int64_t)blockIdx.z * N + n0 + tid] = cs;
    float *Cz = C + (int64_t)blockIdx.z * M * N;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int64_t gm = m0 + wm + 16 * a + 4 * g + e;
                int64_t gn = n0 + wn + 16 * b + i16;
                if (gm < M && gn < N) {
                    float v = acc[a][b][e];
                    if (EPI) {
                        float s = ld(S, gm * lds_ + gn);
                        v *= 1.0f - s * s;
                    }
                    if (gridDim.z == 1) C[gm * ldc + gn] = v;
                    else Cz[gm * N + gn] = v;
                }
            }
}

// Weight gradient of a BF16 network on BF16 MFMA: C = sum_k A[k][m] B[k][n]
// over split z's K range (C + z*M*N receives the partial; M, N <= any),
// A [K][lda] BF16 (activations or network inputs), B [K][N] FP32 (dZ, rounded
// to BF16 as it is staged), FP32 accumulation; the same BF16 operand
// rounding as the forward pass.  Tiles of 128 x 128 outputs, 32 K per step
// (one v_mfma_f32_16x16x32_bf16 deep), four waves of 64 x 64; operands are
// staged K-minor in LDS so a fragment (8 consecutive K of one row) is one
// 16-byte read; the next step's operands are loaded during the current
// step's products.  colsum != NULL: the blocks of the first M tile also sum
// B (in FP32, before rounding) over their K range, in a fixed order.  TB =
// uint16_t: B is already BF16 (rounded by its producer as the staging would
// round it), and no column sums are formed.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
constexpr int WB = 128, WK = 32, WKP = WK + 8; // tile, K step, padded LDS row (bf16)

template <typename TB>
__global__ void __launch_bounds__(256)
    k_wgrad_bf16(int64_t M, int64_t N, int64_t K, int64_t kchunk, const uint16_t *__restrict__ A, int64_t lda,
                 const TB *__restrict__ B, float *__restrict__ C, float *__restrict__ colsum) {
    constexpr bool BF = sizeof(TB) == 2;
    __shared__ __attribute__((aligned(16))) uint16_t As[WB * WKP];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[WB * WKP];
    __shared__ float cred[2][WB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t m0 = (int64_t)blockIdx.x * WB, n0 = (int64_t)blockIdx.y * WB;
    const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
    const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;
    const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
    const int g = lane >> 4, i16 = lane & 15;
    // staging: thread covers column c = tid % 128 of both operand tiles and
    // K rows kk = 2 (tid / 128) + 4 r + {0, 1}, r < 8
    const int c = tid & 127, kh = (tid >> 7) * 2;
    f32x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    uint16_t ra[8][2];
    TB rb[8][2];
    const int64_t mc = m0 + c < M ? m0 + c : M - 1, nc = n0 + c < N ? n0 + c : N - 1;
    auto load = [&](int64_t k0) {
        if (k0 + WK <= kend) {
            // a whole step inside the range: fixed offsets from the step's rows
            const uint16_t *pa = A + (k0 + kh) * lda + mc;
            const TB *pb = B + (k0 + kh) * N + nc;
#pragma unroll
            for (int r = 0; r < 8; ++r)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    ra[r][h] = pa[(4 * r + h) * lda];
                    rb[r][h] = pb[(4 * r + h) * N];
                }
            return;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                // clamped reads with no branch (k0 < kend, M, N >= 1); the
                // staging below zeroes the out-of-range ones
                int64_t gk = k0 + kh + 4 * r + h;
                gk = gk < kend ? gk : kend - 1;
                ra[r][h] = A[gk * lda + mc];
                rb[r][h] = B[gk * N + nc];
            }
    };
    const bool csum = !BF && colsum && blockIdx.x == 0;
    float cs = 0.f;
    if (kbeg < kend) load(kbeg);
    const bool mok = m0 + c < M, nok = n0 + c < N;
    for (int64_t k0 = kbeg; k0 < kend; k0 += WK) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int kk = kh + 4 * r;
            const bool k0ok = k0 + kk < kend, k1ok = k0 + kk + 1 < kend;
            const uint16_t a0 = (k0ok && mok) ? ra[r][0] : (uint16_t)0, a1 = (k1ok && mok) ? ra[r][1] : (uint16_t)0;
            *(uint32_t *)&As[c * WKP + kk] = (uint32_t)a0 | ((uint32_t)a1 << 16);
            if constexpr (BF) {
                const uint32_t b0 = (k0ok && nok) ? rb[r][0] : 0u, b1 = (k1ok && nok) ? rb[r][1] : 0u;
                *(uint32_t *)&Bs[c * WKP + kk] = b0 | (b1 << 16);
            } else {
                const float b0 = (k0ok && nok) ? rb[r][0] : 0.0f, b1 = (k1ok && nok) ? rb[r][1] : 0.0f;
                *(uint32_t *)&Bs[c * WKP + kk] = pack_bf16x2_hw(b0, b1);
                if (csum) cs += b0 + b1;
            }
        }
        __syncthreads();
        if (k0 + WK < kend) load(k0 + WK);
        u32x4_t af[4], bf[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) af[a] = *(const u32x4_t *)&As[(wm + 16 * a + i16) * WKP + 8 * g];
#pragma unroll
        for (int b = 0; b < 4; ++b) bf[b] = *(const u32x4_t *)&Bs[(wn + 16 * b + i16) * WKP + 8 * g];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, af[a]),
                                                                    __builtin_bit_cast(bf16x8_t, bf[b]), acc[a][b],
                                                                    0, 0, 0);
        __syncthreads();
    }
    if (csum) {
        cred[tid >> 7][c] = cs;
        __syncthreads();
        if (tid < 128 && n0 + c < N) colsum[(int64_t)blockIdx.z * N + n0 + c] = cred[0][c] + cred[1][c];
    }
    float *Cz = C + (int64_t)blockIdx.z * M * N;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t gm = m0 + wm + 16 * a + 4 * g + e, gn = n0 + wn + 16 * b + i16;
                if (gm < M && gn < N) Cz[gm * N + gn] = acc[a][b][e];
            }
}

// dZ of a BF16 network on BF16 MFMA: C[m][n] = (sum_k A[m][k] W[n][k])
// (1 - S[m][n]^2), A FP32 [M][lda] (dY or dZ2), W FP32 [N][ldw] (the next
// layer's master weights, so the product is by W^T), S BF16 [M][lds] (the
// saved activations); A and W rounded to BF16 as they are staged, FP32
// accumulation.  128 x 128 tiles, 32 K per step; both operands are K-minor
// in memory already, so a thread stages 16 consecutive K of one row.
__global__ void __launch_bounds__(256)
    k_dz_bf16(int64_t M, int64_t N, int64_t K, const float *__restrict__ A, int64_t lda,
              const float *__restrict__ W, int64_t ldw, const uint16_t *__restrict__ S, int64_t lds_,
              float *__restrict__ C, int64_t ldc) {
    __shared__ __attribute__((aligned(16))) uint16_t As[WB * WKP];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[WB * WKP];
    constexpr int SP = WB + 8; // row pitch of the S tile in LDS
    __shared__ __attribute__((aligned(16))) uint16_t Ss[WB * SP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t m0 = (int64_t)blockIdx.x * WB, n0 = (int64_t)blockIdx.y * WB;
    const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
    const int g = lane >> 4, i16 = lane & 15;
    const int row = tid >> 1, kq = (tid & 1) * 16; // staged row and its 16 K
    // the tile's saved activations (row `row`, 64 columns per thread) are
    // requested now and held through the K loop, then staged in LDS for the
    // epilogue: one round trip, hidden behind the products (clamped reads;
    // the epilogue writes only the elements inside the matrix)
    u32x4_t sreg[8];
    {
        const int64_t sr = m0 + row < M ? m0 + row : M - 1;
        const int64_t c0 = n0 + 64 * (tid & 1);
        if (n0 + WB <= N && lds_ % 8 == 0 && ((uintptr_t)S & 15) == 0) {
#pragma unroll
            for (int j = 0; j < 8; ++j) sreg[j] = *(const u32x4_t *)(S + sr * lds_ + c0 + 8 * j);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                uint32_t w[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t ca = c0 + 8 * j + 2 * q, cb = ca + 1;
                    const uint32_t lo = S[sr * lds_ + (ca < N ? ca : N - 1)];
                    const uint32_t hi = S[sr * lds_ + (cb < N ? cb : N - 1)];
                    w[q] = lo | (hi << 16);
                }
                sreg[j] = u32x4_t{w[0], w[1], w[2], w[3]};
            }
        }
    }
    f32x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    float ra[16], rw[16];
    // 16-byte loads when the rows allow them (K a multiple of the step and
    // 16-byte aligned rows), else clamped element reads
    const bool vec = K % WK == 0 && lda % 4 == 0 && ldw % 4 == 0 && ((uintptr_t)A & 15) == 0 &&
                     ((uintptr_t)W & 15) == 0;
    auto load = [&](int64_t k0) {
        const int64_t mr = m0 + row < M ? m0 + row : M - 1, nr = n0 + row < N ? n0 + row : N - 1;
        if (vec) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 va = *(const float4 *)(A + mr * lda + k0 + kq + 4 * q);
                const float4 vw = *(const float4 *)(W + nr * ldw + k0 + kq + 4 * q);
                ra[4 * q] = va.x, ra[4 * q + 1] = va.y, ra[4 * q + 2] = va.z, ra[4 * q + 3] = va.w;
                rw[4 * q] = vw.x, rw[4 * q + 1] = vw.y, rw[4 * q + 2] = vw.z, rw[4 * q + 3] = vw.w;
            }
            return;
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            // clamped reads with no branch (K, M, N >= 1); the staging
            // below zeroes the out-of-range ones
            const int64_t k = k0 + kq + e < K ? k0 + kq + e : K - 1;
            ra[e] = A[mr * lda + k];
            rw[e] = W[nr * ldw + k];
        }
    };
    const bool mok = m0 + row < M, nok = n0 + row < N;
    load(0);
    for (int64_t k0 = 0; k0 < K; k0 += WK) {
        u32x4_t pa[2], pw[2];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e0 = 8 * h + 2 * q;
                const bool k0ok = k0 + kq + e0 < K, k1ok = k0 + kq + e0 + 1 < K;
                pa[h][q] = pack_bf16x2_hw((mok && k0ok) ? ra[e0] : 0.0f, (mok && k1ok) ? ra[e0 + 1] : 0.0f);
                pw[h][q] = pack_bf16x2_hw((nok && k0ok) ? rw[e0] : 0.0f, (nok && k1ok) ? rw[e0 + 1] : 0.0f);
            }
        *(u32x4_t *)&As[row * WKP + kq] = pa[0];
        *(u32x4_t *)&As[row * WKP + kq + 8] = pa[1];
        *(u32x4_t *)&Bs[row * WKP + kq] = pw[0];
        *(u32x4_t *)&Bs[row * WKP + kq + 8] = pw[1];
        __syncthreads();
        if (k0 + WK < K) load(k0 + WK);
        u32x4_t af[4], bf[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) af[a] = *(const u32x4_t *)&As[(wm + 16 * a + i16) * WKP + 8 * g];
#pragma unroll
        for (int b = 0; b < 4; ++b) bf[b] = *(const u32x4_t *)&Bs[(wn + 16 * b + i16) * WKP + 8 * g];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, af[a]),
                                                                    __builtin_bit_cast(bf16x8_t, bf[b]), acc[a][b],
                                                                    0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) *(u32x4_t *)&Ss[row * SP + 64 * (tid & 1) + 8 * j] = sreg[j];
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int lm = wm + 16 * a + 4 * g + e, ln = wn + 16 * b + i16;
                const int64_t gm = m0 + lm, gn = n0 + ln;
                if (gm < M && gn < N) {
                    const float sv = bf16_to_f32(Ss[lm * SP + ln]);
                    C[gm * ldc + gn] = acc[a][b][e] * (1.0f - sv * sv);
                }
            }
}

// out[i] = sum_z part[z][i] in a fixed order: a block takes 64 elements and
// four split lanes (lane q sums z = q, q + 4, ..; the four are combined as
// (s0 + s1) + (s2 + s3)), loads issued eight at a time.
__global__ void __launch_bounds__(256) k_sum_splits(int64_t len, int nz, const float *__restrict__ part,
                                                    float *__restrict__ out) {
    __shared__ float red[4][64];
    const int el = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 64 + el;
    float s = 0.f;
    if (i < len) {
#pragma unroll 8
        for (int z = q; z < nz; z += 4) s += part[(int64_t)z * len + i];
    }
    red[q][el] = s;
    __syncthreads();
    if (q == 0 && i < len) out[i] = (red[0][el] + red[1][el]) + (red[2][el] + red[3][el]);
}

__global__ void k_mse_grad(int64_t len, float scale, const float *__restrict__ Y,
                           const float *__restrict__ T, float *__restrict__ dY) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) dY[i] = scale * (Y[i] - T[i]);
}

// The loss gradient and the loss in one pass: dY as k_mse_grad, and per
// workgroup the FP64 sum of (Y - T)^2 over a grid-stride range of LOSS_BLOCKS
// x 256 threads, reduced by a fixed tree (the partition and order of
// dnnmg_norm2_f64, so the sum is that norm's to the bit); k_loss_final adds
// the partials in a fixed order.
constexpr int LOSS_BLOCKS = 1024;
__global__ void __launch_bounds__(256) k_mse_grad_loss(int64_t len, float scale, const float *__restrict__ Y,
                                                       const float *__restrict__ T, float *__restrict__ dY,
                                                       double *__restrict__ part) {
    double s = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < len; t += (int64_t)gridDim.x * blockDim.x) {
        const float y = Y[t], tt = T[t];
        dY[t] = scale * (y - tt);
        const double e = (double)y - (double)tt;
        s += e * e;
    }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_loss_final(int nparts, const double *__restrict__ part,
                                                    double *__restrict__ out) {
    __shared__ double red[256];
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

__global__ void k_adamw(int64_t n, float *__restrict__ th, float *__restrict__ m, float *__restrict__ v,
                        const float *__restrict__ g, float lr, float b1, float b2, float eps, float wd,
                        float inv_c1, float inv_sqrt_c2) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.0f - b1) * gi;
    float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float t = th[i];
    float upd = (mi * inv_c1) / (sqrtf(vi) * inv_sqrt_c2 + eps);
    th[i] = t - lr * wd * t - lr * upd;
}

constexpr int DZ_MAX_GRID = 1024; // workgroups of a weight-stationary dZ launch (column-sum partials)

struct BwdPlan {
    int64_t n, H, splits, kchunk, rsplits;
    int64_t wsplits, wkchunk; // the BF16 weight-gradient products: more, shorter splits
    size_t off_dz2, off_dz1, off_part, off_cpart, off_dzc, total;
};

static BwdPlan plan_bwd(int H, int64_t n) {
    BwdPlan p;
    p.n = n;
    p.H = H;
    p.splits = (n + 2047) / 2048;
    if (p.splits > 64) p.splits = 64;
    if (p.splits < 1) p.splits = 1;
    p.kchunk = ((n + p.splits - 1) / p.splits + BK - 1) / BK * BK;
    p.rsplits = p.splits; // bias gradients: one column-sum partial per split
    p.wsplits = (n + 511) / 512;
    if (p.wsplits > 256) p.wsplits = 256;
    if (p.wsplits < 1) p.wsplits = 1;
    p.wkchunk = ((n + p.wsplits - 1) / p.wsplits + WK - 1) / WK * WK;
    const int64_t ps = p.splits > p.wsplits ? p.splits : p.wsplits;
    size_t a = 256;
    auto up = [&](size_t b) { return (b + a - 1) / a * a; };
    p.off_dz2 = 0;
    p.off_dz1 = up(p.off_dz2 + sizeof(float) * n * H);
    p.off_part = up(p.off_dz1 + sizeof(float) * n * H);
    size_t part = sizeof(float) * ps * (size_t)((size_t)N_IN * H + (size_t)H * H + (size_t)H * N_OUT);
    p.off_cpart = up(p.off_part + part);
    // column-sum partials of the weight-stationary dZ products (dZ2, dZ1)
    p.off_dzc = up(p.off_cpart + sizeof(float) * ps * (size_t)(2 * H + N_OUT));
    p.total = up(p.off_dzc + sizeof(float) * 2 * (size_t)DZ_MAX_GRID * H);
    return p;
}

template <bool TA, bool TB, typename TAe, typename TBe, typename TSe, bool EPI>
static void gemm(int64_t M, int64_t N, int64_t K, int64_t splits, int64_t kchunk, const TAe *A,
                 int64_t lda, const TBe *B, int64_t ldb, float *C, int64_t ldc, float *part,
                 const TSe *S, int64_t lds_, hipStream_t s, float *cpart = nullptr, float *colsum = nullptr) {
    dim3 grid((unsigned)((M + BM - 1) / BM), (unsigned)((N + BN - 1) / BN), (unsigned)splits);
    k_gemm<TA, TB, TAe, TBe, TSe, EPI><<<grid, 256, 0, s>>>(M, N, K, kchunk, A, lda, B, ldb,
                                                            splits == 1 ? C : part, ldc, S, lds_,
                                                            colsum ? cpart : nullptr);
    if (splits > 1) k_sum_splits<<<blocks_for(M * N, 64), 256, 0, s>>>(M * N, (int)splits, part, C);
    if (colsum) k_sum_splits<<<blocks_for(N, 64), 256, 0, s>>>(N, (int)splits, cpart, colsum);
}

template <typename TB>
static void wgrad_bf16(int64_t M, int64_t N, int64_t K, int64_t splits, int64_t kchunk, const uint16_t *A,
                       int64_t lda, const TB *B, float *C, float *part, float *cpart, float *colsum,
                       hipStream_t s) {
    dim3 grid((unsigned)((M + WB - 1) / WB), (unsigned)((N + WB - 1) / WB), (unsigned)splits);
    k_wgrad_bf16<TB><<<grid, 256, 0, s>>>(M, N, K, kchunk, A, lda, B, part, colsum ? cpart : nullptr);
    k_sum_splits<<<blocks_for(M * N, 64), 256, 0, s>>>(M * N, (int)splits, part, C);
    if (colsum) k_sum_splits<<<blocks_for(N, 64), 256, 0, s>>>(N, (int)splits, cpart, colsum);
}

// dZ of a BF16 network of width N = 128 or 256, weight-stationary: the same
// product and epilogue as k_dz_bf16, C[m][n] = (sum_k A[m][k] W[n][k]) (1 -
// S[m][n]^2), with W^T held in registers.  Eight waves each keep the BF16
// fragments of their NT x 16 output units over all NK K chunks (W rows are
// the MFMA's A operand, so a lane holds 8 consecutive K of one unit) for
// the whole launch; a persistent grid walks blocks of MB patch rows.  A
// block's rows of A are staged once in LDS as BF16 (a lane's B fragment is 8
// consecutive K of one patch row), double buffered: the next block's rows
// are requested before the current block's products and written to the
// other buffer after them, so one barrier per block orders the buffers.  A
// lane's accumulator holds 4 consecutive units of one patch row, which the
// epilogue scales by (1 - s^2) and writes as one 16-byte store.  The K
// chunks are summed in ascending order as in k_dz_bf16.
constexpr int DZ_NW = 8, DZ_NT = 64 * DZ_NW;
// TA: element type of A (float, or uint16_t for a BF16 dZ from the previous
// product, staged as it is).  BOUT: C is written in BF16 (rounded as a
// consumer's staging would round it) to Cb, and each workgroup also sums
// its rows of C (FP32, before rounding) per unit into cpart[blockIdx.x][N]:
// lanes accumulate over their rows in block order, the 16 lanes of a unit
// group are then added by a fixed butterfly, so the partials (and their sum
// in workgroup order) are run-to-run identical.
template <int NT, int NK, int MB, typename TA, bool BOUT>
__global__ void __launch_bounds__(DZ_NT)
    k_dz_ws(int64_t M, int K, const TA *__restrict__ A, int64_t lda, const float *__restrict__ W, int64_t ldw,
            const uint16_t *__restrict__ S, int64_t lds_, float *__restrict__ C, uint16_t *__restrict__ Cb,
            int64_t ldc, float *__restrict__ cpart) {
    constexpr int N = 16 * NT * DZ_NW, KP = 32 * NK, PITCH = KP + 8; // LDS row pitch (bf16)
    constexpr int TPR = DZ_NT / MB, NJ = MB / 16;                    // staging threads per row; m tiles
    constexpr int EPT = KP / TPR;                                    // K elements a thread stages
    constexpr bool ABF = sizeof(TA) == 2;
    static_assert(KP % TPR == 0 && EPT % 8 == 0, "staging splits a row into 16-byte pieces");
    __shared__ __attribute__((aligned(16))) uint16_t sA[2][MB * PITCH];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, i16 = lane & 15;
    const int nb = 16 * NT * wave; // the wave's first unit
    // W^T fragments: unit nb + 16 t + i16, K 32 c + 8 g .. + 8 (zero past K)
    u32x4_t wf[NT][NK];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            const float *wr = W + (int64_t)(nb + 16 * t + i16) * ldw;
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 32 * c + 8 * g + e;
                v[e] = wr[k < K ? k : K - 1];
                v[e] = k < K ? v[e] : 0.0f;
            }
            wf[t][c] = u32x4_t{pack_bf16x2_hw(v[0], v[1]), pack_bf16x2_hw(v[2], v[3]), pack_bf16x2_hw(v[4], v[5]),
                               pack_bf16x2_hw(v[6], v[7])};
        }
    // staging: thread tid takes row tid / TPR of the block, K (tid % TPR) EPT ..
    const int srow = tid / TPR, sk = (tid % TPR) * EPT;
    const bool vec = K == KP && lda % (ABF ? 8 : 4) == 0 && ((uintptr_t)A & 15) == 0;
    TA ra[EPT];
    auto load = [&](int64_t mb) {
        const int64_t m = mb * MB + srow;
        const int64_t mr = m < M ? m : M - 1;
        const TA *ar = A + mr * lda;
        if (vec) {
            if constexpr (ABF) {
#pragma unroll
                for (int q = 0; q < EPT / 8; ++q) {
                    const u32x4_t x = *(const u32x4_t *)(ar + sk + 8 * q);
#pragma unroll
                    for (int h = 0; h < 4; ++h) {
                        ra[8 * q + 2 * h] = (uint16_t)(x[h] & 0xffffu);
                        ra[8 * q + 2 * h + 1] = (uint16_t)(x[h] >> 16);
                    }
                }
            } else {
#pragma unroll
                for (int q = 0; q < EPT / 4; ++q) {
                    const float4 x = *(const float4 *)(ar + sk + 4 * q);
                    ra[4 * q] = x.x, ra[4 * q + 1] = x.y, ra[4 * q + 2] = x.z, ra[4 * q + 3] = x.w;
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int k = sk + e;
                ra[e] = ar[k < K ? k : K - 1];
            }
        }
    };
    auto store = [&](int buf, int64_t mb) {
        const bool mok = mb * MB + srow < M;
#pragma unroll
        for (int q = 0; q < EPT / 8; ++q) {
            u32x4_t pk;
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int e = 8 * q + 2 * h;
                const bool k0 = mok && sk + e < K, k1 = mok && sk + e + 1 < K;
                if constexpr (ABF)
                    pk[h] = (k0 ? (uint32_t)ra[e] : 0u) | ((k1 ? (uint32_t)ra[e + 1] : 0u) << 16);
                else
                    pk[h] = pack_bf16x2_hw(k0 ? ra[e] : 0.0f, k1 ? ra[e + 1] : 0.0f);
            }
            *(u32x4_t *)&sA[buf][srow * PITCH + sk + 8 * q] = pk;
        }
    };
    float cs[NT][4] = {};
    const int64_t nmb = (M + MB - 1) / MB;
    int64_t mb = blockIdx.x;
    int buf = 0;
    if (mb < nmb) {
        load(mb);
        store(0, mb);
    }
    for (; mb < nmb; mb += gridDim.x, buf ^= 1) {
        __syncthreads();
        // the epilogue's saved activations of this block, then the next
        // block's rows (so waiting for the former does not wait for the latter)
        uint2 sv[NT][NJ];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const int64_t m = mb * MB + 16 * j + i16;
                const int64_t mr = m < M ? m : M - 1;
                sv[t][j] = *(const uint2 *)(S + mr * lds_ + nb + 16 * t + 4 * g);
            }
        const int64_t next = mb + gridDim.x;
        if (next < nmb) load(next);
        f32x4 acc[NT][NJ];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int j = 0; j < NJ; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            u32x4_t bf[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j) bf[j] = *(const u32x4_t *)&sA[buf][(16 * j + i16) * PITCH + 32 * c + 8 * g];
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int j = 0; j < NJ; ++j)
                    acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, wf[t][c]),
                                                                        __builtin_bit_cast(bf16x8_t, bf[j]),
                                                                        acc[t][j], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const int64_t m = mb * MB + 16 * j + i16;
                if (m >= M) continue;
                float v[4];
                v[0] = bf16_to_f32((uint16_t)(sv[t][j].x & 0xffffu));
                v[1] = bf16_to_f32((uint16_t)(sv[t][j].x >> 16));
                v[2] = bf16_to_f32((uint16_t)(sv[t][j].y & 0xffffu));
                v[3] = bf16_to_f32((uint16_t)(sv[t][j].y >> 16));
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = acc[t][j][e] * (1.0f - v[e] * v[e]);
                if constexpr (BOUT) {
                    *(uint2 *)(Cb + m * ldc + nb + 16 * t + 4 * g) =
                        make_uint2(pack_bf16x2_hw(v[0], v[1]), pack_bf16x2_hw(v[2], v[3]));
#pragma unroll
                    for (int e = 0; e < 4; ++e) cs[t][e] += v[e];
                } else {
                    *(float4 *)(C + m * ldc + nb + 16 * t + 4 * g) = make_float4(v[0], v[1], v[2], v[3]);
                }
            }
        if (next < nmb) store(buf ^ 1, next);
    }
    if constexpr (BOUT) {
        // the 16 rows a unit's lanes hold, by a fixed butterfly
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float x = cs[t][e];
                x += __shfl_xor(x, 8, 16);
                x += __shfl_xor(x, 4, 16);
                x += __shfl_xor(x, 2, 16);
                x += __shfl_xor(x, 1, 16);
                if (i16 == 0) cpart[(int64_t)blockIdx.x * N + nb + 16 * t + 4 * g + e] = x;
            }
    }
}

// One weight-stationary dZ product on a persistent grid of at most one
// workgroup per compute unit; returns the grid size (BOUT: the number of
// column-sum partials written to cpart, one row of N per workgroup).
template <int NT, int NK, int MB, typename TA, bool BOUT>
static int dz_ws_launch(int64_t M, int K, const TA *A, int64_t lda, const float *W, int64_t ldw, const uint16_t *S,
                        int64_t lds_, float *C, uint16_t *Cb, int64_t ldc, float *cpart, hipStream_t s) {
    const int64_t nmb = (M + MB - 1) / MB;
    int64_t cap = (int64_t)device_cus();
    if (cap > DZ_MAX_GRID) cap = DZ_MAX_GRID;
    const unsigned grid = (unsigned)(nmb < cap ? nmb : cap);
    k_dz_ws<NT, NK, MB, TA, BOUT><<<grid, DZ_NT, 0, s>>>(M, K, A, lda, W, ldw, S, lds_, C, Cb, ldc, cpart);
    return (int)grid;
}

// The shapes the weight-stationary dZ products are built for: width 128 or
// 256 (K = 81, then the width), 8-byte aligned rows of S and of the BF16 dZ.
static bool dz_ws_shape(int64_t M, int64_t N, const void *S, int64_t lds_, int64_t ldc) {
    return M > 0 && (N == 128 || N == 256) && lds_ % 4 == 0 && ldc % 8 == 0 && ((uintptr_t)S & 7) == 0;
}

template <typename TX, typename TS>
static void backward_impl(const BwdPlan &p, const TX *X, int64_t ldx, const TS *saved, const float *W2,
                          const float *W3, const float *dY, float *dW[3], float *db[3], char *ws,
                          hipStream_t s) {
    const int64_t n = p.n, H = p.H;
    float *dz2 = (float *)(ws + p.off_dz2);
    float *dz1 = (float *)(ws + p.off_dz1);
    float *part = (float *)(ws + p.off_part);
    float *cpart = (float *)(ws + p.off_cpart);
    const TS *A1 = saved, *A2 = saved + n * H;
    if constexpr (sizeof(TS) == 2 && sizeof(TX) == 2) {
        if (dz_ws_shape(n, H, A2, H, H)) {
            // BF16 network of width 128 or 256: the weight-stationary dZ
            // products keep dZ2 and dZ1 in BF16 (as every consumer stages
            // them) and sum their columns for the bias gradients on the way
            uint16_t *dz2b = (uint16_t *)(ws + p.off_dz2), *dz1b = (uint16_t *)(ws + p.off_dz1);
            float *cs2 = (float *)(ws + p.off_dzc), *cs1 = cs2 + (size_t)DZ_MAX_GRID * H;
            const uint16_t *S2 = (const uint16_t *)A2, *S1 = (const uint16_t *)A1;
            int g2, g1;
            if (H == 256) {
                g2 = dz_ws_launch<2, 4, 64, float, true>(n, N_OUT, dY, N_OUT, W3, N_OUT, S2, H, nullptr, dz2b, H, cs2,
                                                         s);
                g1 = dz_ws_launch<2, 8, 32, uint16_t, true>(n, (int)H, dz2b, H, W2, H, S1, H, nullptr, dz1b, H, cs1,
                                                            s);
            } else {
                g2 = dz_ws_launch<1, 4, 64, float, true>(n, N_OUT, dY, N_OUT, W3, N_OUT, S2, H, nullptr, dz2b, H, cs2,
                                                         s);
                g1 = dz_ws_launch<1, 4, 64, uint16_t, true>(n, (int)H, dz2b, H, W2, H, S1, H, nullptr, dz1b, H, cs1,
                                                            s);
            }
            k_sum_splits<<<blocks_for(H, 64), 256, 0, s>>>(H, g2, cs2, db[1]);
            k_sum_splits<<<blocks_for(H, 64), 256, 0, s>>>(H, g1, cs1, db[0]);
            wgrad_bf16<float>(H, N_OUT, n, p.wsplits, p.wkchunk, A2, H, dY, dW[2], part, cpart, db[2], s);
            wgrad_bf16<uint16_t>(H, H, n, p.wsplits, p.wkchunk, A1, H, dz2b, dW[1], part, cpart, nullptr, s);
            wgrad_bf16<uint16_t>(N_IN, H, n, p.wsplits, p.wkchunk, X, ldx, dz1b, dW[0], part, cpart, nullptr, s);
            return;
        }
    }
    if constexpr (sizeof(TS) == 2) {
        // BF16 network: dZ products on BF16 MFMA (W3 is [H][81], W2 [H][H])
        dim3 grid((unsigned)((n + WB - 1) / WB), (unsigned)((H + WB - 1) / WB));
        k_dz_bf16<<<grid, 256, 0, s>>>(n, H, N_OUT, dY, N_OUT, W3, N_OUT, (const uint16_t *)A2, H, dz2, H);
        k_dz_bf16<<<grid, 256, 0, s>>>(n, H, H, dz2, H, W2, H, (const uint16_t *)A1, H, dz1, H);
    } else {
        // dZ2 = (dY W3^T) (.) (1 - A2^2): W3 is [H][81] -> op(B)[k=o][n=h] = W3[h][o]
        gemm<false, true, float, float, TS, true>(n, H, N_OUT, 1, N_OUT + BK, dY, N_OUT, W3, N_OUT, dz2, H,
                                                  nullptr, A2, H, s);
        // dZ1 = (dZ2 W2^T) (.) (1 - A1^2): W2 is [H_in][H_out] -> op(B)[k=j][n=h] = W2[h][j]
        gemm<false, true, float, float, TS, true>(n, H, H, 1, H + BK, dz2, H, W2, H, dz1, H, nullptr, A1, H,
                                                  s);
    }
    // weight gradients, split over patches; the bias gradients (column sums
    // of dY, dZ2, dZ1) come from the same staged tiles
    if constexpr (sizeof(TS) == 2 && sizeof(TX) == 2) {
        // BF16 network: BF16 products with FP32 accumulation
        wgrad_bf16<float>(H, N_OUT, n, p.wsplits, p.wkchunk, A2, H, dY, dW[2], part, cpart, db[2], s);
        wgrad_bf16<float>(H, H, n, p.wsplits, p.wkchunk, A1, H, dz2, dW[1], part, cpart, db[1], s);
        wgrad_bf16<float>(N_IN, H, n, p.wsplits, p.wkchunk, X, ldx, dz1, dW[0], part, cpart, db[0], s);
    } else {
        gemm<true, false, TS, float, float, false>(H, N_OUT, n, p.splits, p.kchunk, A2, H, dY, N_OUT, dW[2],
                                                   N_OUT, part, nullptr, 0, s, cpart, db[2]);
        gemm<true, false, TS, float, float, false>(H, H, n, p.splits, p.kchunk, A1, H, dz2, H, dW[1], H,
                                                   part, nullptr, 0, s, cpart, db[1]);
        gemm<true, false, TX, float, float, false>(N_IN, H, n, p.splits, p.kchunk, X, ldx, dz1, H, dW[0], H,
                                                   part, nullptr, 0, s, cpart, db[0]);
    }
}

} // namespace dnnmg

using namespace dnnmg;

extern "C" int dnnmg_mse_grad(int64_t n, const float *Y, const float *T, float *dY, void *stream) {
    if (n < 0) return fail(DNNMG_ERR_SHAPE, "dnnmg_mse_grad: n < 0");
    if (n == 0) return DNNMG_OK;
    if (!Y || !T || !dY) return fail(DNNMG_ERR_ARG, "dnnmg_mse_grad: NULL pointer");
    int64_t len = n * N_OUT;
    k_mse_grad<<<blocks_for(len, 256), 256, 0, (hipStream_t)stream>>>(len, 2.0f / (float)n, Y, T, dY);
    return hip_check(hipGetLastError(), "dnnmg_mse_grad launch");
}

extern "C" int dnnmg_mse_grad_loss(int64_t n, const float *Y, const float *T, float *dY, double *loss_sum,
                                   void *ws, size_t ws_bytes, void *stream) {
    if (n < 0) return fail(DNNMG_ERR_SHAPE, "dnnmg_mse_grad_loss: n < 0");
    if (!Y || !T || !dY || !loss_sum || !ws) return fail(DNNMG_ERR_ARG, "dnnmg_mse_grad_loss: NULL pointer");
    if (ws_bytes < LOSS_BLOCKS * sizeof(double))
        return fail(DNNMG_ERR_SHAPE, "dnnmg_mse_grad_loss: workspace %zu < %zu bytes", ws_bytes,
                    LOSS_BLOCKS * sizeof(double));
    const int64_t len = n * N_OUT;
    hipStream_t s = (hipStream_t)stream;
    k_mse_grad_loss<<<LOSS_BLOCKS, 256, 0, s>>>(len, n > 0 ? 2.0f / (float)n : 0.0f, Y, T, dY, (double *)ws);
    k_loss_final<<<1, 256, 0, s>>>(LOSS_BLOCKS, (const double *)ws, loss_sum);
    return hip_check(hipGetLastError(), "dnnmg_mse_grad_loss launch");
}

extern "C" int dnnmg_adamw_step(int64_t n, float *theta, float *m, float *v, const float *g, float lr,
                                float b1, float b2, float eps, float wd, int64_t t, void *stream) {
    if (n < 0 || t < 1) return fail(DNNMG_ERR_ARG, "dnnmg_adamw_step: need n >= 0 and t >= 1");
    if (n == 0) return DNNMG_OK;
    if (!theta || !m || !v || !g) return fail(DNNMG_ERR_ARG, "dnnmg_adamw_step: NULL pointer");
    if (!(b1 >= 0.f && b1 < 1.f && b2 >= 0.f && b2 < 1.f && eps > 0.f))
        return fail(DNNMG_ERR_ARG, "dnnmg_adamw_step: bad betas or eps");
    double c1 = 1.0 - pow((double)b1, (double)t), c2 = 1.0 - pow((double)b2, (double)t);
    k_adamw<<<blocks_for(n, 256), 256, 0, (hipStream_t)stream>>>(
        n, theta, m, v, g, lr, b1, b2, eps, wd, (float)(1.0 / c1), (float)(1.0 / sqrt(c2)));
    return hip_check(hipGetLastError(), "dnnmg_adamw_step launch");
}

extern "C" size_t dnnmg_patch_backward_workspace(const dnnmg_mlp *net, int64_t n) {
    if (!net || n < 0) return 0;
    return plan_bwd(net->hidden, n).total;
}

extern "C" int dnnmg_patch_backward(const dnnmg_mlp *net, const float *W2, const float *W3, int64_t n,
                                    const void *X, int64_t ldx, const void *saved, const float *dY,
                                    float *dW[3], float *db[3], void *ws, size_t ws_bytes,
                                    void *stream) {
    if (!net) return fail(DNNMG_ERR_ARG, "dnnmg_patch_backward: net is NULL");
    if (net->n_in != N_IN || net->n_out != N_OUT)
        return fail(DNNMG_ERR_SHAPE, "dnnmg_patch_backward: network must be 165 -> H -> H -> 81");
    if (net->dtype != DNNMG_F32 && net->dtype != DNNMG_BF16)
        return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_patch_backward: dtype %d (F32 or BF16 only)", net->dtype);
    const int H = net->hidden;
    if (H != 64 && H != 128 && H != 256 && H != 512)
        return fail(DNNMG_ERR_UNSUPPORTED, "dnnmg_patch_backward: hidden %d", H);
    if (n < 1) return fail(DNNMG_ERR_SHAPE, "dnnmg_patch_backward: n must be >= 1");
    if (ldx < N_IN) return fail(DNNMG_ERR_SHAPE, "dnnmg_patch_backward: ldx < 165");
    if (!W2 || !W3 || !X || !saved || !dY || !dW || !db || !ws)
        return fail(DNNMG_ERR_ARG, "dnnmg_patch_backward: NULL pointer");
    for (int l = 0; l < 3; ++l)
        if (!dW[l] || !db[l]) return fail(DNNMG_ERR_ARG, "dnnmg_patch_backward: dW/db[%d] NULL", l);
    BwdPlan p = plan_bwd(H, n);
    if (ws_bytes < p.total)
        return fail(DNNMG_ERR_SHAPE, "dnnmg_patch_backward: workspace %zu < %zu bytes", ws_bytes, p.total);
    hipStream_t s = (hipStream_t)stream;
    if (net->dtype == DNNMG_F32)
        backward_impl<float, float>(p, (const float *)X, ldx, (const float *)saved, W2, W3, dY, dW, db,
                                    (char *)ws, s);
    else
        backward_impl<uint16_t, uint16_t>(p, (const uint16_t *)X, ldx, (const uint16_t *)saved, W2, W3, dY,
                                          dW, db, (char *)ws, s);
    return hip_check(hipGetLastError(), "dnnmg_patch_backward launch");
}
