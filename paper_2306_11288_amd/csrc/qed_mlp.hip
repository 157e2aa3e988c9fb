// Learned samplers: a 4-128-128-128-3 perceptron (SiLU) per process.  The NCS network maps
// an emission's (log chi, S.b, S.n, energy draw) to the photon-fraction variable
// t = (2u/(3 chi))^(1/3) and the spin-summed mean photon Stokes xi3, xi2 (eqs. F0-F3 of
// Sec. III.C.1 summed over the final spins); the NBW network maps a pair creation's
// (log chi_gamma, xi3, 0, energy draw) to the positron's energy fraction delta and the mean
// positron and electron spin along b (eqs. G0-G3 of Sec. III.D summed over the partner's
// spin).  Each replaces the table inverse-CDF search of an event; the table sampler stays
// as the fallback outside the trained range and as the reference for its error.
//
//   * inference: k_mlp_forward, BF16 MFMA (v_mfma_f32_32x32x16_bf16) with FP32
//     accumulation for the two 128 x 128 layers, weights and activations in LDS;
//   * training data: k_mlp_samples draws inputs with Philox and computes the targets with
//     the FP64 tables and the F formulas of the library itself;
//   * training: three FP32 launches per step, the dense layers on FP32 matrix cores
//     (v_mfma_f32_32x32x2_f32), the weight gradients split over the batch and summed in a
//     fixed order, Adam fused with the sum.
#include "qed_dev.hpp"

namespace qed {

namespace {

constexpr int HS = 136;           // padded row stride (bf16) of activations / transposed weights in LDS
constexpr int MB = 512;           // threads of a forward block: 8 wavefronts of 32 samples each

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

__device__ __forceinline__ float silu(float z) {
    return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}
__device__ __forceinline__ float silu_prime(float z) {
    const float sg = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
    return sg * (1.0f + z * (1.0f - sg));
}

// ------------------------------------------------------------------------- training data
struct SampleArgs {
    const double *tab64;
    int64_t n;
    uint64_t seed;
    float *X, *Y;        // [n][4], [n][3]
};

// The table sampler on normalised inputs x (the function the network learns): t from the
// spin-dependent inverse CDF, mean xi3, xi2 = F3/F0, F2/F0 at S_f = 0.  T: table precision.
template <class T>
__device__ __forceinline__ void table_sampler(const T *tab, const float x[4], float y[3]) {
    const double chi = exp10(MLP_L10_HALF * (double)x[0] + MLP_L10_MID);
    const T s = (T)x[1], c = (T)x[2], rr = (T)(0.5 * ((double)x[3] + 1.0));
    const Tabs<T> tb = {tab};
    T Ia, Ib;
    uint32_t st = 0;
    ncs_rate<T>(tb.ncs_rate(), chi, Ia, Ib, st);
    const T tt = ncs_sample_t<T>(tb, chi, Ib / Ia, s, rr);
    const T x3 = tt * tt * tt, u = (T)1.5 * (T)chi * x3;
    T I, K1, K2;
    bessel_scaled<T>(tb, x3, I, K1, K2);
    const V3<T> ax = {1, 0, 0}, bx = {0, 1, 0}, nx = {0, 0, 1}, Si = {0, s, c}, Sf = {0, 0, 0};
    T F[4];
    ncs_F<T>(u, I, K1, K2, Si, Sf, ax, bx, nx, F);
    y[0] = (float)(tt / (T)T_MAX);
    y[1] = (float)(F[3] / F[0]);
    y[2] = (float)(F[2] / F[0]);
}

__global__ __launch_bounds__(BLOCK) void k_mlp_samples(SampleArgs a) {
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= a.n) return;
    double r[4];
    uniform4((uint64_t)k, 0, STREAM_MLP, a.seed, r);
    // inputs: log10 chi uniform on [-3, log10 50]; an isotropic unit spin (S.b uniform,
    // S.n its transverse part times a uniform azimuth cosine); the energy draw.  The
    // targets are computed from the rounded inputs, so every pair is exact.
    const double l10 = -3.0 + r[0] * (MLP_L10_HI + 3.0);
    const double s0 = 2.0 * r[1] - 1.0;
    const double c0 = sqrt(1.0 - s0 * s0) * cospi(2.0 * r[2]);
    const float x[4] = {(float)((l10 - MLP_L10_MID) / MLP_L10_HALF), (float)s0, (float)c0,
                        (float)(2.0 * r[3] - 1.0)};
    float y[3];
    table_sampler<double>(a.tab64, x, y);
    for (int j = 0; j < 4; ++j) a.X[4 * k + j] = x[j];
    for (int j = 0; j < 3; ++j) a.Y[3 * k + j] = y[j];
}

// The NBW table sampler on normalised inputs (the function the NBW network learns): delta
// from the tabulated pair spectrum at xi3; with xi1 = xi2 = 0, the sum of eqs. G0-G3 over the
// partner's spin leaves A + S.B at the member's spin S, A = I + (rs - xi3) K2,
// B_+ . b = K1 (xi3 / e_- - 1 / e_+), B_- . b = K1 (1 / e_- - xi3 / e_+) (e_+ = delta,
// e_- = 1 - delta, rs = (e_+^2 + e_-^2) / (e_+ e_-)); the mean spins along b are B.b / A.
template <class T>
__device__ __forceinline__ void nbw_table_sampler(const T *tab, const float x[4], float y[3]) {
    const double chi = exp10(MLP_NBW_L10_HALF * (double)x[0] + MLP_NBW_L10_MID);
    const T xi3 = (T)x[1], rr = (T)(0.5 * ((double)x[3] + 1.0));
    const Tabs<T> tb = {tab};
    T Ja, Jb, kappa;
    uint32_t st = 0;
    nbw_rate<T>(tb, chi, Ja, Jb, kappa, st);
    const T d = nbw_sample_delta<T>(tb, chi, kappa, xi3, rr);
    T I, K1, K2;
    bessel_scaled<T>(tb, (T)(2.0 / (3.0 * chi * (double)d * (1.0 - (double)d))), I, K1, K2);
    const T ep = d, em = (T)1 - d, rs = (ep * ep + em * em) / (ep * em), A = I + (rs - xi3) * K2;
    y[0] = (float)d;
    y[1] = (float)(K1 * (xi3 / em - (T)1 / ep) / A);
    y[2] = (float)(K1 * ((T)1 / em - xi3 / ep) / A);
}

// NBW training pairs: log10 chi_gamma uniform on the trained range, xi3 uniform on [-1, 1],
// x2 = 0, the energy draw; targets from the rounded inputs
__global__ __launch_bounds__(BLOCK) void k_nbw_samples(SampleArgs a) {
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= a.n) return;
    double r[4];
    uniform4((uint64_t)k, 0, STREAM_MLP + 1, a.seed, r);
    const double l10 = MLP_NBW_L10_LO + r[0] * (MLP_NBW_L10_HI - MLP_NBW_L10_LO);
    const float x[4] = {(float)((l10 - MLP_NBW_L10_MID) / MLP_NBW_L10_HALF), (float)(2.0 * r[1] - 1.0), 0.0f,
                        (float)(2.0 * r[3] - 1.0)};
    float y[3];
    nbw_table_sampler<double>(a.tab64, x, y);
    for (int j = 0; j < 4; ++j) a.X[4 * k + j] = x[j];
    for (int j = 0; j < 3; ++j) a.Y[3 * k + j] = y[j];
}

template <class T, int NET>
__global__ __launch_bounds__(BLOCK) void k_table_sampler(const T *tab, const float *X, float *Y, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= n) return;
    const float4 v = ((const float4 *)X)[k];
    const float x[4] = {v.x, v.y, v.z, v.w};
    float y[3];
    if constexpr (NET == QED_NET_NBW) nbw_table_sampler<T>(tab, x, y);
    else table_sampler<T>(tab, x, y);
    for (int j = 0; j < 3; ++j) Y[3 * k + j] = y[j];
}

// ------------------------------------------------------------------------- inference
// One block = 8 wavefronts; a wavefront takes 32 samples at a time (one 32-column MFMA
// tile).  The matrix-core layers compute the transposed product D[out][sample] =
// W^T[out][in] H^T[in][sample]: the weights are the A operand (rows of the transposed
// weights in LDS), the activations the B operand (rows of the wavefront's activation tile
// in LDS), so a lane's 16 results per 32 outputs are four runs of four consecutive
// outputs of one sample and go back to LDS as four 8-byte stores.  Layer 3's outputs stay
// in registers and feed layer 4 (FP32 weights) directly.
// LDS: the two 128 x 128 weight matrices transposed ([out][in], bf16, rows padded to HS)
// and one activation tile per wavefront (32 x 128 bf16, padded).
struct FwdArgs {
    const float *P;        // FP32 master parameters (flat layout)
    const __bf16 *WT;      // [2][128][HS] transposed bf16 copies of W2, W3
    const float *X;        // [n][4]
    float *Y;              // [n][3]
    int64_t n;
    const int64_t *n_dev;  // optional device count (used when non-null)
};

typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;

__global__ __launch_bounds__(MB) void k_mlp_forward(FwdArgs a) {
    __shared__ __attribute__((aligned(16))) __bf16 sW[2 * 128 * HS];
    __shared__ __attribute__((aligned(16))) __bf16 sH[(MB / 64) * 32 * HS];
    __shared__ __attribute__((aligned(16))) float sW1[4 * 128];
    __shared__ __attribute__((aligned(16))) float sB[3 * 128];
    __shared__ __attribute__((aligned(16))) float sW4[128 * 4];   // [in][4]: W4 row, then 0
    __shared__ float sB4[4];
    const int64_t n = a.n_dev ? *a.n_dev : a.n;
    const int64_t ntile = (n + 31) / 32;
    if ((int64_t)blockIdx.x * (MB / 64) >= ntile) return;
    for (int k = threadIdx.x; k < 2 * 128 * HS / 8; k += MB) ((bf16x8 *)sW)[k] = ((const bf16x8 *)a.WT)[k];
    for (int k = threadIdx.x; k < 4 * 128; k += MB) sW1[k] = a.P[MLP_OW1 + k];
    for (int k = threadIdx.x; k < 128; k += MB) {
        sB[k] = a.P[MLP_OB1 + k];
        sB[128 + k] = a.P[MLP_OB2 + k];
        sB[256 + k] = a.P[MLP_OB3 + k];
    }
    for (int k = threadIdx.x; k < 128 * 4; k += MB) sW4[k] = (k & 3) < 3 ? a.P[MLP_OW4 + (k >> 2) * 3 + (k & 3)] : 0.0f;
    if (threadIdx.x < 3) sB4[threadIdx.x] = a.P[MLP_OB4 + threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int row = lane & 31, half = lane >> 5;
    __bf16 *H = sH + w * 32 * HS;
    for (int64_t tile = (int64_t)blockIdx.x * (MB / 64) + w; tile < ntile; tile += (int64_t)gridDim.x * (MB / 64)) {
        const int64_t smp = tile * 32 + row;
        float x[4] = {0, 0, 0, 0};
        if (smp < n) {
            const float4 v = ((const float4 *)a.X)[smp];
            x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
        }
        // layer 1 (4 -> 128, FP32 on the VALU): this lane's sample, columns half 64 .. +64,
        // eight at a time (vector LDS reads of the weights, one 16-byte store)
        for (int j0 = 0; j0 < 64; j0 += 8) {
            const int c0 = half * 64 + j0;
            float z[8];
            const float4 b0 = *(const float4 *)(sB + c0), b1 = *(const float4 *)(sB + c0 + 4);
            z[0] = b0.x; z[1] = b0.y; z[2] = b0.z; z[3] = b0.w;
            z[4] = b1.x; z[5] = b1.y; z[6] = b1.z; z[7] = b1.w;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float4 w0 = *(const float4 *)(sW1 + i * 128 + c0), w1 = *(const float4 *)(sW1 + i * 128 + c0 + 4);
                z[0] += x[i] * w0.x; z[1] += x[i] * w0.y; z[2] += x[i] * w0.z; z[3] += x[i] * w0.w;
                z[4] += x[i] * w1.x; z[5] += x[i] * w1.y; z[6] += x[i] * w1.z; z[7] += x[i] * w1.w;
            }
            bf16x8 hv;
#pragma unroll
            for (int j = 0; j < 8; ++j) hv[j] = (__bf16)silu(z[j]);
            *(bf16x8 *)(H + row * HS + c0) = hv;
        }
        // layers 2, 3 (128 -> 128) on the matrix cores; D element v of this lane is output
        // ct 32 + 8 (v / 4) + 4 half + v % 4 of sample `row`
        float y[3] = {0.0f, 0.0f, 0.0f};
        for (int L = 0; L < 2; ++L) {
            const __bf16 *WL = sW + L * 128 * HS;
            const float *bL = sB + (L + 1) * 128;
            f32x16 acc[4];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const float4 bv = *(const float4 *)(bL + ct * 32 + 8 * g + 4 * half);
                    acc[ct][4 * g + 0] = bv.x; acc[ct][4 * g + 1] = bv.y;
                    acc[ct][4 * g + 2] = bv.z; acc[ct][4 * g + 3] = bv.w;
                }
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                const bf16x8 hv = *(const bf16x8 *)(H + row * HS + kk * 16 + half * 8);
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    const bf16x8 wv = *(const bf16x8 *)(WL + (ct * 32 + row) * HS + kk * 16 + half * 8);
                    acc[ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wv, hv, acc[ct], 0, 0, 0);
                }
            }
            if (L == 0) {
                // layer-2 activations back over the tile (every read of it above is done)
#pragma unroll
                for (int ct = 0; ct < 4; ++ct)
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        bf16x4 q;
#pragma unroll
                        for (int r = 0; r < 4; ++r) q[r] = (__bf16)silu(acc[ct][4 * g + r]);
                        *(bf16x4 *)(H + row * HS + ct * 32 + 8 * g + 4 * half) = q;
                    }
            } else {
                // layer 4 (128 -> 3): this lane's 64 layer-3 outputs (rounded to bf16 like a
                // stored activation) times the FP32 weights; the other half holds the rest
#pragma unroll
                for (int ct = 0; ct < 4; ++ct)
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int o = ct * 32 + 8 * g + 4 * half + r;
                            const float h = (float)(__bf16)silu(acc[ct][4 * g + r]);
                            const float4 w4 = *(const float4 *)(sW4 + 4 * o);
                            y[0] += h * w4.x;
                            y[1] += h * w4.y;
                            y[2] += h * w4.z;
                        }
                        // keep the weight reads of later groups from being hoisted here
                        // (all 64 at once would not fit in registers)
                        __builtin_amdgcn_sched_barrier(0);
                    }
            }
        }
        // the two halves of the wavefront hold the two halves of the layer-4 sums
#pragma unroll
        for (int o = 0; o < 3; ++o) y[o] = sB4[o] + (y[o] + __shfl_xor(y[o], 32));
        if (smp < n && half == 0) {
            a.Y[3 * smp + 0] = y[0];
            a.Y[3 * smp + 1] = y[1];
            a.Y[3 * smp + 2] = y[2];
        }
    }
}

// bf16 transposed copies of W2, W3 for the forward kernel
__global__ void k_mlp_pack(const float *P, __bf16 *WT) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;   // over 2 * 128 * HS
    if (k >= 2 * 128 * HS) return;
    const int L = k / (128 * HS), rem = k % (128 * HS), out = rem / HS, in = rem % HS;
    const float *W = P + (L == 0 ? MLP_OW2 : MLP_OW3);
    WT[k] = in < 128 ? (__bf16)W[in * 128 + out] : (__bf16)0.0f;
}

// ------------------------------------------------------------------------- training (FP32)
// Three launches per step, the dense layers on FP32 matrix cores (v_mfma_f32_32x32x2_f32:
// FP32 operands, FP32 accumulation), everything else on the vector unit in FP32:
//  k_train_fb     one block per tile of 32 samples, each wavefront owning 32 of the 128
//                 outputs of a layer: forward (layers 1 and 4 on the VALU, 2 and 3 on the
//                 matrix cores), the loss and its gradient dY, and the backward pass through
//                 the activations (dZ3 = dY W4^T * SiLU'(Z3); dZ2 = dZ3 W3^T * SiLU'(Z2) and
//                 dZ1 = dZ2 W2^T * SiLU'(Z1) on the matrix cores).  A layer's input tile sits
//                 in LDS; H1, H2, H3, dZ1, dZ2, dZ3 and dY go to global memory feature-major
//                 ([feature][sample]) for the weight gradients, with the tile's loss.
//  k_train_dw     the weight and bias gradients as sums over TR_NS slices of consecutive
//                 samples: dW2 = H1^T dZ2 and dW3 = H2^T dZ3 on the matrix cores (TR_CH-sample
//                 chunks of both operands staged in LDS, 32 input rows per block), dW1 = X^T
//                 dZ1, dW4 = H3^T dY and the bias gradients on the VALU; each slice writes its
//                 partial sums.
//  k_train_reduce per parameter the sum of the slice partials in slice order, and the loss as
//                 a fixed-order sum of the tile losses, so results do not depend on
//                 scheduling; when training, the Adam update and the copies of the weights
//                 the kernels read (W2, W3 transposed in FP32 for the backward pass, and in
//                 bf16 for inference).
// Matrix-core operand layout: lane l supplies A[l % 32][k + l / 32] and B[k + l / 32][l % 32]
// and holds D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32] in accumulator v.
constexpr int TR_NS = 64;         // batch slices of the weight gradients
constexpr int TR_CH = 64;         // samples per staged chunk of the weight gradients
constexpr int TR_TP = 129;        // LDS row of a tile (floats): a column read hits distinct banks
constexpr int TR_CP = TR_CH + 1;  // LDS row of a staged chunk

struct TrainArgs {
    const float *P;                   // parameters (flat)
    const float *W2T, *W3T;           // W2, W3 transposed ([out][in]) in FP32
    const float *X, *T;               // [n][4], [n][3]
    int64_t n, Bp;                    // samples; the padded batch (a multiple of TR_NS TR_CH)
    float w0, w1, w2;                 // loss weights
    float *H1T, *H2T, *H3T, *dZ1T, *dZ2T, *dZ3T;   // [128][Bp]
    float *dYT;                       // [3][Bp]
    float *lossp;                     // per 32-sample tile
    float *part;                      // [TR_NS][MLP_NPARAM]
};

// row of accumulator v (within a 32 x 32 block) for this lane's half h
__device__ __forceinline__ int acc_row(int v, int h) { return 8 * (v >> 2) + 4 * h + (v & 3); }

// acc[v] += sum over in of W[in][o0 + row] Bt[j][in]: outputs o0 .. o0+31 of a 128 x 128
// layer for the 32 samples of the tile Bt (LDS, [sample][in]); W row-major [in][out] from
// global memory (L2 resident) through buffer loads (one lane offset register, the row in
// a scalar offset), 16 weights in flight while the previous 16 products run
__device__ __forceinline__ void wload(float *w, __amdgpu_buffer_rsrc_t rs, int vo, int k0) {
#pragma unroll
    for (int i = 0; i < 16; ++i)
        w[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, (k0 + 2 * i) * 512, 0));
}
__device__ __forceinline__ f32x16 wmul(const float *w, const float *br, int k0, f32x16 acc) {
#pragma unroll
    for (int i = 0; i < 16; ++i) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(w[i], br[k0 + 2 * i], acc, 0, 0, 0);
    return acc;
}
__device__ __forceinline__ f32x16 tile_layer(const float *__restrict__ W, const float *Bt, int o0, int j, int h,
                                             f32x16 acc) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)W, 0, 128 * 128 * 4, 0x00020000);
    const int vo = (h * 128 + o0 + j) * 4;
    const float *br = Bt + j * TR_TP + h;
    float wa[16], wb[16];
    wload(wa, rs, vo, 0);
    wload(wb, rs, vo, 32);
    acc = wmul(wa, br, 0, acc);
    __builtin_amdgcn_sched_barrier(0);
    wload(wa, rs, vo, 64);
    acc = wmul(wb, br, 32, acc);
    __builtin_amdgcn_sched_barrier(0);
    wload(wb, rs, vo, 96);
    acc = wmul(wa, br, 64, acc);
    __builtin_amdgcn_sched_barrier(0);
    return wmul(wb, br, 96, acc);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_train_fb(TrainArgs a) {
    __shared__ float sA[32 * TR_TP], sC[32 * TR_TP];
    __shared__ float sW1[4 * 128], sB[3 * 128], sW4[128 * 3], sB4[4], sY[4][32][3];
    const int tid = threadIdx.x;
    for (int k = tid; k < 4 * 128; k += 256) sW1[k] = a.P[MLP_OW1 + k];
    for (int k = tid; k < 128; k += 256) {
        sB[k] = a.P[MLP_OB1 + k];
        sB[128 + k] = a.P[MLP_OB2 + k];
        sB[256 + k] = a.P[MLP_OB3 + k];
    }
    for (int k = tid; k < 128 * 3; k += 256) sW4[k] = a.P[MLP_OW4 + k];
    if (tid < 3) sB4[tid] = a.P[MLP_OB4 + tid];
    __syncthreads();
    const float inv_n = 1.0f / (float)a.n, wl[3] = {a.w0, a.w1, a.w2};
    const int64_t ntile = a.Bp / 32;
    for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        // the thread index and the row stride taken afresh in every tile: otherwise the
        // row indices and store addresses (the same in every tile) are computed once before
        // the loop and held in ~200 registers for its whole length
        int tid = threadIdx.x;
        int64_t Bp = a.Bp;
        asm volatile("" : "+v"(tid), "+s"(Bp));
        const int lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6), j = lane & 31, h = lane >> 5,
                  o0 = wv * 32;
        const int64_t base = tile * 32;
        {   // layer 1 (VALU): thread -> sample tid % 32, outputs 16 (tid / 32) .. +16
            const int s = tid & 31, q0 = (tid >> 5) * 16;
            const int64_t smp = base + s;
            float x[4] = {0, 0, 0, 0};
            if (smp < a.n) {
                const float4 v = ((const float4 *)a.X)[smp];
                x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
            }
            for (int q = q0; q < q0 + 16; ++q) {
                float z = sB[q];
#pragma unroll
                for (int i = 0; i < 4; ++i) z += x[i] * sW1[i * 128 + q];
                const float hv = silu(z);
                sA[s * TR_TP + q] = hv;
                a.H1T[(int64_t)q * Bp + smp] = hv;
            }
        }
        __syncthreads();
        const int64_t smp = base + j;    // this lane's sample from here on
        const bool live = smp < a.n;
        // layer 2: H1 (sA) -> H2 (sC); Z2 stays in registers for SiLU'(Z2)
        f32x16 z2, z3, g;
#pragma unroll
        for (int v = 0; v < 16; ++v) z2[v] = sB[128 + o0 + acc_row(v, h)];
        z2 = tile_layer(a.P + MLP_OW2, sA, o0, j, h, z2);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int o = o0 + acc_row(v, h);
            const float hv = silu(z2[v]);
            a.H2T[(int64_t)o * Bp + smp] = hv;
            sC[j * TR_TP + o] = hv;
        }
        __syncthreads();
        // layer 3: H2 (sC) -> H3; layer 4 partial sums over this wave's 32 outputs
#pragma unroll
        for (int v = 0; v < 16; ++v) z3[v] = sB[256 + o0 + acc_row(v, h)];
        z3 = tile_layer(a.P + MLP_OW3, sC, o0, j, h, z3);
        float y[3] = {0, 0, 0};
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int o = o0 + acc_row(v, h);
            const float hv = silu(z3[v]);
            a.H3T[(int64_t)o * Bp + smp] = hv;
#pragma unroll
            for (int c = 0; c < 3; ++c) y[c] += hv * sW4[o * 3 + c];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) y[c] += __shfl_xor(y[c], 32);
        if (h == 0)
#pragma unroll
            for (int c = 0; c < 3; ++c) sY[wv][j][c] = y[c];
        __syncthreads();
        // outputs, loss and dY (the four waves' partial sums added in a fixed order)
        float dy[3], l = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float yc = sB4[c] + ((sY[0][j][c] + sY[1][j][c]) + (sY[2][j][c] + sY[3][j][c]));
            const float d = live ? yc - a.T[3 * smp + c] : 0.0f;
            dy[c] = 2.0f * wl[c] * d * inv_n;
            l += wl[c] * d * d;
        }
        if (wv == 0) {
            if (h == 0)
#pragma unroll
                for (int c = 0; c < 3; ++c) a.dYT[(int64_t)c * Bp + smp] = dy[c];
            l = h == 0 ? l : 0.0f;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) l += __shfl_xor(l, d);
            if (lane == 0) a.lossp[tile] = l;
        }
        // dZ3 = (dY W4^T) * SiLU'(Z3) -> sA
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int o = o0 + acc_row(v, h);
            const float dh = dy[0] * sW4[o * 3] + dy[1] * sW4[o * 3 + 1] + dy[2] * sW4[o * 3 + 2];
            const float dz = dh * silu_prime(z3[v]);
            a.dZ3T[(int64_t)o * Bp + smp] = dz;
            sA[j * TR_TP + o] = dz;
        }
        __syncthreads();
        // dZ2 = (dZ3 W3^T) * SiLU'(Z2) -> sC
#pragma unroll
        for (int v = 0; v < 16; ++v) g[v] = 0.0f;
        g = tile_layer(a.W3T, sA, o0, j, h, g);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int o = o0 + acc_row(v, h);
            const float dz = g[v] * silu_prime(z2[v]);
            a.dZ2T[(int64_t)o * Bp + smp] = dz;
            sC[j * TR_TP + o] = dz;
        }
        __syncthreads();
        // dZ1 = (dZ2 W2^T) * SiLU'(Z1), Z1 recomputed at this lane's outputs
#pragma unroll
        for (int v = 0; v < 16; ++v) g[v] = 0.0f;
        g = tile_layer(a.W2T, sC, o0, j, h, g);
        float x[4] = {0, 0, 0, 0};
        if (live) {
            const float4 xv = ((const float4 *)a.X)[smp];
            x[0] = xv.x; x[1] = xv.y; x[2] = xv.z; x[3] = xv.w;
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int o = o0 + acc_row(v, h);
            float z = sB[o];
#pragma unroll
            for (int i = 0; i < 4; ++i) z += x[i] * sW1[i * 128 + o];
            a.dZ1T[(int64_t)o * Bp + smp] = g[v] * silu_prime(z);
        }
        // the next tile's first writes (sA) follow this tile's last read of sA (before the
        // barrier above); its next write of sC follows its own first barrier
    }
}

// Weight and bias gradients of one batch slice (blockIdx.x).  blockIdx.y < 8: matrix
// y / 4 (dW2 from H1, dZ2; dW3 from H2, dZ3), input rows 32 (y % 4) .. +32 on the matrix
// cores, each wavefront 32 of the outputs, the next chunk loaded into registers while the
// current one is multiplied; blockIdx.y = 8 + q: the small gradients of features
// 32 q .. 32 q + 31 (VALU).
constexpr int TR_DW_Y = 8 + 4;
__global__ __launch_bounds__(256) void k_train_dw(TrainArgs a) {
    __shared__ float sH[32 * TR_CP], sD[128 * TR_CP];
    const int sl = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, j = lane & 31, h = lane >> 5;
    const int64_t Bp = a.Bp, len = Bp / TR_NS, s0 = (int64_t)sl * len;
    float *part = a.part + (int64_t)sl * MLP_NPARAM;
    if (blockIdx.y < 8) {
        const int m = blockIdx.y >> 2, rb = (blockIdx.y & 3) * 32;
        const float *HT = m == 0 ? a.H1T : a.H2T, *DT = m == 0 ? a.dZ2T : a.dZ3T;
        f32x16 acc;
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
        constexpr int Q = TR_CH / 4;                 // float4 per row of a chunk
        constexpr int NH = 32 * Q / 256, ND = 128 * Q / 256;
        float4 rh[NH], rd[ND];
        auto fetch = [&](int64_t c0) {
#pragma unroll
            for (int i = 0; i < NH; ++i) {
                const int e = tid + 256 * i, r = e / Q, c = (e % Q) * 4;
                rh[i] = *(const float4 *)(HT + (int64_t)(rb + r) * Bp + c0 + c);
            }
#pragma unroll
            for (int i = 0; i < ND; ++i) {
                const int e = tid + 256 * i, r = e / Q, c = (e % Q) * 4;
                rd[i] = *(const float4 *)(DT + (int64_t)r * Bp + c0 + c);
            }
        };
        fetch(s0);
        for (int64_t c0 = s0; c0 < s0 + len; c0 += TR_CH) {
#pragma unroll
            for (int i = 0; i < NH; ++i) {
                const int e = tid + 256 * i;
                float *d = sH + (e / Q) * TR_CP + (e % Q) * 4;
                d[0] = rh[i].x; d[1] = rh[i].y; d[2] = rh[i].z; d[3] = rh[i].w;
            }
#pragma unroll
            for (int i = 0; i < ND; ++i) {
                const int e = tid + 256 * i;
                float *d = sD + (e / Q) * TR_CP + (e % Q) * 4;
                d[0] = rd[i].x; d[1] = rd[i].y; d[2] = rd[i].z; d[3] = rd[i].w;
            }
            __syncthreads();
            if (c0 + TR_CH < s0 + len) fetch(c0 + TR_CH);
            // D[in][out] += sum over the chunk's samples of H[in][s] dZ[out][s]
#pragma unroll 8
            for (int k = 0; k < TR_CH; k += 2)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(sH[j * TR_CP + k + h], sD[(wv * 32 + j) * TR_CP + k + h], acc,
                                                          0, 0, 0);
            __syncthreads();
        }
        const int ow = m == 0 ? MLP_OW2 : MLP_OW3;
#pragma unroll
        for (int v = 0; v < 16; ++v) part[ow + (rb + acc_row(v, h)) * 128 + wv * 32 + j] = acc[v];
        return;
    }
    // small gradients: wavefront wv takes 8 features, its lanes stride over the slice's
    // samples (all 8 features' loads of a sample in flight together) and the lanes' sums
    // are added across the wavefront in a fixed pattern
    constexpr int NR = 8;
    const int f0 = (blockIdx.y - 8) * 32 + wv * NR;
    float r[NR][10];          // dW1[0..3][o], db1, db2, db3, dW4[o][0..2]
    float r4[3] = {0, 0, 0};  // db4 (kept by the first wavefront of feature block 0)
#pragma unroll
    for (int f = 0; f < NR; ++f)
#pragma unroll
        for (int q = 0; q < 10; ++q) r[f][q] = 0.0f;
    for (int64_t k = s0 + lane; k < s0 + len; k += 64) {
        float4 xv = {0, 0, 0, 0};
        if (k < a.n) xv = ((const float4 *)a.X)[k];
        const float dy0 = a.dYT[k], dy1 = a.dYT[Bp + k], dy2 = a.dYT[2 * Bp + k];
        r4[0] += dy0; r4[1] += dy1; r4[2] += dy2;
#pragma unroll
        for (int f = 0; f < NR; ++f) {
            const int64_t ro = (int64_t)(f0 + f) * Bp + k;
            const float d1 = a.dZ1T[ro], hv = a.H3T[ro];
            r[f][0] += xv.x * d1; r[f][1] += xv.y * d1; r[f][2] += xv.z * d1; r[f][3] += xv.w * d1;
            r[f][4] += d1;
            r[f][5] += a.dZ2T[ro];
            r[f][6] += a.dZ3T[ro];
            r[f][7] += hv * dy0; r[f][8] += hv * dy1; r[f][9] += hv * dy2;
        }
    }
#pragma unroll
    for (int f = 0; f < NR; ++f) {
#pragma unroll
        for (int q = 0; q < 10; ++q)
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) r[f][q] += __shfl_xor(r[f][q], d);
        if (lane == 0) {
            const int o = f0 + f;
#pragma unroll
            for (int i = 0; i < 4; ++i) part[MLP_OW1 + i * 128 + o] = r[f][i];
            part[MLP_OB1 + o] = r[f][4];
            part[MLP_OB2 + o] = r[f][5];
            part[MLP_OB3 + o] = r[f][6];
#pragma unroll
            for (int c = 0; c < 3; ++c) part[MLP_OW4 + o * 3 + c] = r[f][7 + c];
        }
    }
    if (f0 == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) r4[c] += __shfl_xor(r4[c], d);
            if (lane == 0) part[MLP_OB4 + c] = r4[c];
        }
    }
}

struct ReduceArgs {
    const float *part, *lossp;
    int64_t ntile;
    float inv_n;
    float *G, *loss;
    int train, t;                 // Adam (train = 1): step count t >= 1
    float lr, b1, b2, eps;
    float *P, *m, *v, *W2T, *W3T;
    __bf16 *WT;                   // [2][128][HS] inference copies
};
// per parameter: gradient = sum over the slices in slice order; block 0 also the loss (a
// fixed-order sum of the tile losses); with train, Adam and the weight copies
__global__ __launch_bounds__(256) void k_train_reduce(ReduceArgs a) {
    if (blockIdx.x == 0) {
        __shared__ float s[256];
        float l = 0.0f;
        const int64_t per = (a.ntile + 255) / 256, t0 = threadIdx.x * per;
        for (int64_t t = t0; t < t0 + per && t < a.ntile; ++t) l += a.lossp[t];
        s[threadIdx.x] = l;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0 && a.loss) *a.loss = s[0] * a.inv_n;
    }
    const int k = (int)(blockIdx.x * 256 + threadIdx.x);
    if (k >= MLP_NPARAM) return;
    float g = 0.0f;
    for (int z = 0; z < TR_NS; ++z) g += a.part[(int64_t)z * MLP_NPARAM + k];
    a.G[k] = g;
    if (!a.train) return;
    const float mk = a.b1 * a.m[k] + (1.0f - a.b1) * g, vk = a.b2 * a.v[k] + (1.0f - a.b2) * g * g;
    a.m[k] = mk;
    a.v[k] = vk;
    const float mh = mk / (1.0f - powf(a.b1, (float)a.t)), vh = vk / (1.0f - powf(a.b2, (float)a.t));
    const float p = a.P[k] - a.lr * mh / (sqrtf(vh) + a.eps);
    a.P[k] = p;
    if (k >= MLP_OW2 && k < MLP_OW2 + 128 * 128) {
        const int in = (k - MLP_OW2) >> 7, out = (k - MLP_OW2) & 127;
        a.W2T[out * 128 + in] = p;
        a.WT[out * HS + in] = (__bf16)p;
    } else if (k >= MLP_OW3 && k < MLP_OW3 + 128 * 128) {
        const int in = (k - MLP_OW3) >> 7, out = (k - MLP_OW3) & 127;
        a.W3T[out * 128 + in] = p;
        a.WT[128 * HS + out * HS + in] = (__bf16)p;
    }
}

// transposed FP32 copies of W2, W3 (the A operands of the backward pass)
__global__ void k_mlp_pack32(const float *P, float *W2T, float *W3T) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;   // over 2 * 128 * 128
    if (k >= 2 * 128 * 128) return;
    const int L = k >> 14, rem = k & 16383, out = rem >> 7, in = rem & 127;
    (L == 0 ? W2T : W3T)[out * 128 + in] = P[(L == 0 ? MLP_OW2 : MLP_OW3) + in * 128 + out];
}

// initial weights: uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) from Philox, biases 0
__global__ void k_mlp_init(float *P, uint64_t seed) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= MLP_NPARAM) return;
    struct Blk { int off, len, fan; };
    const Blk W[4] = {{MLP_OW1, 4 * 128, 4}, {MLP_OW2, 128 * 128, 128}, {MLP_OW3, 128 * 128, 128},
                      {MLP_OW4, 128 * 3, 128}};
    float val = 0.0f;
    for (int b = 0; b < 4; ++b)
        if (k >= W[b].off && k < W[b].off + W[b].len) {
            double r[4];
            uniform4((uint64_t)k, 1, STREAM_MLP, seed, r);
            val = (float)((2.0 * r[0] - 1.0) / sqrt((double)W[b].fan));
        }
    P[k] = val;
}

}  // namespace

// ------------------------------------------------------------------------- host side
hipError_t mlp_alloc(MlpNet &N) {
    if (N.P) return hipSuccess;
    hipError_t e = hipMalloc(&N.P, MLP_NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&N.m, MLP_NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&N.v, MLP_NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&N.G, MLP_NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&N.WT, 2 * 128 * HS * sizeof(__bf16));
    if (e == hipSuccess) e = hipMalloc(&N.W32, 2 * 128 * 128 * sizeof(float));
    return e;
}

void mlp_free(MlpNet &N) {
    (void)hipFree(N.P);
    (void)hipFree(N.m);
    (void)hipFree(N.v);
    (void)hipFree(N.G);
    (void)hipFree(N.WT);
    (void)hipFree(N.W32);
    N = MlpNet{};
}

hipError_t mlp_pack(MlpNet &N, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_pack, dim3((2 * 128 * HS + 255) / 256), dim3(256), 0, s, N.P, (__bf16 *)N.WT);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_pack32, dim3(2 * 128 * 128 / 256), dim3(256), 0, s, N.P, N.W32, N.W32 + 128 * 128);
    return hipGetLastError();
}

hipError_t mlp_init(qed_ctx *ctx, uint64_t seed, hipStream_t s) {
    MlpNet &N = ctx->nets[ctx->mlp_sel];
    hipError_t e = mlp_alloc(N);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_init, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, N.P, seed);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemsetAsync(N.m, 0, MLP_NPARAM * sizeof(float), s)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(N.v, 0, MLP_NPARAM * sizeof(float), s)) != hipSuccess) return e;
    N.t = 0;
    return mlp_pack(N, s);
}

hipError_t mlp_samples(qed_ctx *ctx, int64_t n, uint64_t seed, float *X, float *Y, hipStream_t s) {
    SampleArgs a{ctx->tab64, n, seed, X, Y};
    const dim3 g((unsigned)((n + BLOCK - 1) / BLOCK));
    if (ctx->mlp_sel == QED_NET_NBW) hipLaunchKernelGGL(k_nbw_samples, g, dim3(BLOCK), 0, s, a);
    else hipLaunchKernelGGL(k_mlp_samples, g, dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

template <int NET>
static void table_sampler_launch(qed_ctx *ctx, const float *X, float *Y, int64_t n, hipStream_t s) {
    const dim3 g((unsigned)((n + BLOCK - 1) / BLOCK));
    if (ctx->cfg.precision == QED_MIXED)
        hipLaunchKernelGGL((k_table_sampler<float, NET>), g, dim3(BLOCK), 0, s, ctx->tab32, X, Y, n);
    else hipLaunchKernelGGL((k_table_sampler<double, NET>), g, dim3(BLOCK), 0, s, ctx->tab64, X, Y, n);
}
hipError_t table_sampler_run(qed_ctx *ctx, const float *X, float *Y, int64_t n, hipStream_t s) {
    if (ctx->mlp_sel == QED_NET_NBW) table_sampler_launch<QED_NET_NBW>(ctx, X, Y, n, s);
    else table_sampler_launch<QED_NET_NCS>(ctx, X, Y, n, s);
    return hipGetLastError();
}

hipError_t mlp_forward(qed_ctx *ctx, const MlpNet &N, const float *X, float *Y, int64_t n, const int64_t *n_dev,
                       int64_t n_max, hipStream_t s) {
    FwdArgs a{N.P, (const __bf16 *)N.WT, X, Y, n, n_dev};
    const int64_t tiles = (n_max + 31) / 32, per = MB / 64;
    int64_t blocks = (tiles + per - 1) / per;
    const int64_t cap = 4 * (int64_t)ctx->num_cu;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)blocks), dim3(MB), 0, s, a);
    return hipGetLastError();
}

// One forward + backward pass over a batch (FP32 matrix cores): the gradient (flat
// layout) into the selected network's G and the mean loss into *loss; with train, also the Adam step on
// the parameters.  Work buffers come from ctx->mlp_work (grown on demand).
static hipError_t mlp_pass(qed_ctx *ctx, const float *X, const float *T, int64_t n, const float w[3], float *loss,
                           int train, float lr, hipStream_t s) {
    const int64_t unit = (int64_t)TR_CH * TR_NS;
    const int64_t Bp = (n + unit - 1) / unit * unit, ntile = Bp / 32;
    const int64_t need = 6 * 128 * Bp + 3 * Bp + ntile + (int64_t)TR_NS * MLP_NPARAM;
    if (need > ctx->mlp_work_len) {
        (void)hipFree(ctx->mlp_work);
        ctx->mlp_work = nullptr;
        ctx->mlp_work_len = 0;
        hipError_t e = hipMalloc(&ctx->mlp_work, need * sizeof(float));
        if (e != hipSuccess) return e;
        ctx->mlp_work_len = need;
    }
    float *q = ctx->mlp_work;
    MlpNet &N = ctx->nets[ctx->mlp_sel];
    TrainArgs a{};
    a.P = N.P;
    a.W2T = N.W32;
    a.W3T = N.W32 + 128 * 128;
    a.X = X;
    a.T = T;
    a.n = n;
    a.Bp = Bp;
    a.w0 = w[0]; a.w1 = w[1]; a.w2 = w[2];
    float **arr[6] = {&a.H1T, &a.H2T, &a.H3T, &a.dZ1T, &a.dZ2T, &a.dZ3T};
    for (int k = 0; k < 6; ++k) {
        *arr[k] = q;
        q += 128 * Bp;
    }
    a.dYT = q;
    q += 3 * Bp;
    a.lossp = q;
    q += ntile;
    a.part = q;
    int64_t blocks = ntile;
    const int64_t cap = 4 * (int64_t)ctx->num_cu;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(k_train_fb, dim3((unsigned)blocks), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_train_dw, dim3(TR_NS, TR_DW_Y), dim3(256), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    ReduceArgs r{};
    r.part = a.part;
    r.lossp = a.lossp;
    r.ntile = ntile;
    r.inv_n = 1.0f / (float)n;
    r.G = N.G;
    r.loss = loss;
    r.train = train;
    if (train) {
        N.t += 1;
        r.t = N.t;
        r.lr = lr;
        r.b1 = 0.9f;
        r.b2 = 0.999f;
        r.eps = 1e-8f;
        r.P = N.P;
        r.m = N.m;
        r.v = N.v;
        r.W2T = N.W32;
        r.W3T = N.W32 + 128 * 128;
        r.WT = (__bf16 *)N.WT;
    }
    hipLaunchKernelGGL(k_train_reduce, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, r);
    return hipGetLastError();
}

hipError_t mlp_grad(qed_ctx *ctx, const float *X, const float *T, int64_t n, const float w[3], float *loss,
                    hipStream_t s) {
    return mlp_pass(ctx, X, T, n, w, loss, 0, 0.0f, s);
}

hipError_t mlp_train(qed_ctx *ctx, const float *X, const float *T, int64_t n, const float w[3], float lr,
                     float *loss, hipStream_t s) {
    return mlp_pass(ctx, X, T, n, w, loss, 1, lr, s);
}

}  // namespace qed
