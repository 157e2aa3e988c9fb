// Learned NCS sampler: a 4-128-128-128-3 perceptron (SiLU) that maps an emission's
// (log chi, S.b, S.n, energy draw) to the photon-fraction variable t = (2u/(3 chi))^(1/3)
// and the spin-summed mean photon Stokes xi3, xi2 (eqs. F0-F3 of Sec. III.C.1 summed over
// the final spins).  It replaces the table inverse-CDF search of an emission; the table
// sampler stays as the fallback outside the trained range and as the reference for its error.
//
//   * inference: k_mlp_forward, BF16 MFMA (v_mfma_f32_32x32x16_bf16) with FP32
//     accumulation for the two 128 x 128 layers, weights and activations in LDS;
//   * training data: k_mlp_samples draws inputs with Philox and computes the targets with
//     the FP64 tables and the F formulas of the library itself;
//   * training: FP32 kernels (tiled GEMM with a deterministic split-K for the weight
//     gradients, SiLU and its derivative, loss, column sums, Adam).
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

template <class T>
__global__ __launch_bounds__(BLOCK) void k_table_sampler(const T *tab, const float *X, float *Y, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= n) return;
    const float4 v = ((const float4 *)X)[k];
    const float x[4] = {v.x, v.y, v.z, v.w};
    float y[3];
    table_sampler<T>(tab, x, y);
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
// C[m][n] (+)= sum_k A(m, k) B(k, n) over k in [k0, k1), A(m, k) = A[m sam + k sak],
// B(k, n) = B[k sbk + n sbn]; 64 x 64 tile per block (256 threads, 4 x 4 outputs each),
// K in chunks of 16 through LDS.  Epilogue: + bias[n] if bias; Z stored to C; if H, also
// H = SiLU(C).  Split-K: blockIdx.z selects a K slice, C += ldc_slice * z.
struct GemmArgs {
    const float *A, *B, *bias;
    float *C, *H;
    int M, N, K;
    int64_t sam, sak, sbk, sbn;
    int ldc;
    int kslice;            // K per slice (split-K), K if no split
    int64_t slice_stride;  // floats between the C slices
};

__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    __shared__ float sA[16][65], sBt[16][65];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int kb = blockIdx.z * g.kslice, ke = kb + g.kslice < g.K ? kb + g.kslice : g.K;
    const bool a_k_fast = g.sak == 1 && g.sam != 1, b_k_fast = g.sbk == 1 && g.sbn != 1;
    float acc[4][4] = {};
    for (int k0 = kb; k0 < ke; k0 += 16) {
        // consecutive threads walk the operand's contiguous dimension (coalesced loads)
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int kk = a_k_fast ? e % 16 : e / 64, mm = a_k_fast ? e / 16 : e % 64;
            const int m = m0 + mm, k = k0 + kk;
            sA[kk][mm] = (m < g.M && k < ke) ? g.A[(int64_t)m * g.sam + (int64_t)k * g.sak] : 0.0f;
            const int kb2 = b_k_fast ? e % 16 : e / 64, nn = b_k_fast ? e / 16 : e % 64;
            const int n = n0 + nn, k2 = k0 + kb2;
            sBt[kb2][nn] = (n < g.N && k2 < ke) ? g.B[(int64_t)k2 * g.sbk + (int64_t)n * g.sbn] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            float av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = sA[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = sBt[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
        }
        __syncthreads();
    }
    float *C = g.C + (int64_t)blockIdx.z * g.slice_stride;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = m0 + ty * 4 + i, n = n0 + tx * 4 + j;
            if (m >= g.M || n >= g.N) continue;
            const float z = acc[i][j] + (g.bias ? g.bias[n] : 0.0f);
            C[(int64_t)m * g.ldc + n] = z;
            if (g.H) g.H[(int64_t)m * g.ldc + n] = silu(z);
        }
}

// dY = 2 w (Y - T) / B; loss partial sums per block
__global__ __launch_bounds__(256) void k_loss(const float *Y, const float *T, int64_t n, float w0, float w1, float w2,
                                              float *dY, float *part) {
    __shared__ float s[256];
    const float w[3] = {w0, w1, w2};
    float acc = 0;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n * 3; k += (int64_t)gridDim.x * 256) {
        const float d = Y[k] - T[k], wk = w[k % 3];
        acc += wk * d * d;
        dY[k] = 2.0f * wk * d / (float)n;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}
__global__ void k_loss_total(const float *part, int nb, int64_t n, float *loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float s = 0;
    for (int k = 0; k < nb; ++k) s += part[k];
    *loss = s / (float)n;
}

// dZ = dH * SiLU'(Z), elementwise
__global__ void k_silu_back(const float *dH, const float *Z, float *dZ, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dZ[k] = dH[k] * silu_prime(Z[k]);
}

// column sums of D [rows][ncol] in slices of rows: part[slice][col].  A block covers 64
// columns of one slice; its four row lanes take every fourth row and are added in a fixed
// order, so the sums do not depend on scheduling.
__global__ __launch_bounds__(256) void k_colsum(const float *D, int64_t rows, int ncol, int rows_per_slice,
                                                float *part) {
    __shared__ float s_part[4][64];
    const int cl = threadIdx.x & 63, rl = threadIdx.x >> 6;
    const int col = blockIdx.x * 64 + cl;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per_slice;
    const int64_t r1 = r0 + rows_per_slice < rows ? r0 + rows_per_slice : rows;
    float s = 0;
    if (col < ncol)
        for (int64_t r = r0 + rl; r < r1; r += 4) s += D[r * ncol + col];
    s_part[rl][cl] = s;
    __syncthreads();
    if (rl == 0 && col < ncol)
        part[(int64_t)blockIdx.y * ncol + col] = ((s_part[0][cl] + s_part[1][cl]) + s_part[2][cl]) + s_part[3][cl];
}
// out[k] = sum over slices of part[slice][k], slices in order (deterministic)
__global__ void k_sum_slices(const float *part, int nslice, int64_t len, float *out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= len) return;
    float s = 0;
    for (int z = 0; z < nslice; ++z) s += part[(int64_t)z * len + k];
    out[k] = s;
}

// Adam (bias-corrected moments); step t >= 1
__global__ void k_adam(float *P, const float *G, float *m, float *v, int64_t n, float lr, float b1, float b2,
                       float eps, int t) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float g = G[k];
    const float mk = b1 * m[k] + (1.0f - b1) * g, vk = b2 * v[k] + (1.0f - b2) * g * g;
    m[k] = mk;
    v[k] = vk;
    const float mh = mk / (1.0f - powf(b1, (float)t)), vh = vk / (1.0f - powf(b2, (float)t));
    P[k] -= lr * mh / (sqrtf(vh) + eps);
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
hipError_t mlp_alloc(qed_ctx *ctx) {
    if (ctx->mlp_P) return hipSuccess;
    hipError_t e = hipMalloc(&ctx->mlp_P, MLP_NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&ctx->mlp_m, MLP_NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&ctx->mlp_v, MLP_NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&ctx->mlp_G, MLP_NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&ctx->mlp_WT, 2 * 128 * HS * sizeof(__bf16));
    return e;
}

hipError_t mlp_pack(qed_ctx *ctx, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_pack, dim3((2 * 128 * HS + 255) / 256), dim3(256), 0, s, ctx->mlp_P, (__bf16 *)ctx->mlp_WT);
    return hipGetLastError();
}

hipError_t mlp_init(qed_ctx *ctx, uint64_t seed, hipStream_t s) {
    hipError_t e = mlp_alloc(ctx);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_init, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, ctx->mlp_P, seed);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemsetAsync(ctx->mlp_m, 0, MLP_NPARAM * sizeof(float), s)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(ctx->mlp_v, 0, MLP_NPARAM * sizeof(float), s)) != hipSuccess) return e;
    ctx->mlp_t = 0;
    return mlp_pack(ctx, s);
}

hipError_t mlp_samples(qed_ctx *ctx, int64_t n, uint64_t seed, float *X, float *Y, hipStream_t s) {
    SampleArgs a{ctx->tab64, n, seed, X, Y};
    hipLaunchKernelGGL(k_mlp_samples, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t table_sampler_run(qed_ctx *ctx, const float *X, float *Y, int64_t n, hipStream_t s) {
    const dim3 g((unsigned)((n + BLOCK - 1) / BLOCK));
    if (ctx->cfg.precision == QED_MIXED) hipLaunchKernelGGL(k_table_sampler<float>, g, dim3(BLOCK), 0, s, ctx->tab32, X, Y, n);
    else hipLaunchKernelGGL(k_table_sampler<double>, g, dim3(BLOCK), 0, s, ctx->tab64, X, Y, n);
    return hipGetLastError();
}

hipError_t mlp_forward(qed_ctx *ctx, const float *X, float *Y, int64_t n, const int64_t *n_dev, int64_t n_max,
                       hipStream_t s) {
    FwdArgs a{ctx->mlp_P, (const __bf16 *)ctx->mlp_WT, X, Y, n, n_dev};
    const int64_t tiles = (n_max + 31) / 32, per = MB / 64;
    int64_t blocks = (tiles + per - 1) / per;
    const int64_t cap = 4 * (int64_t)ctx->num_cu;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)blocks), dim3(MB), 0, s, a);
    return hipGetLastError();
}

namespace {
hipError_t gemm(const float *A, int64_t sam, int64_t sak, const float *B, int64_t sbk, int64_t sbn, float *C, int ldc,
                int M, int N, int K, const float *bias, float *H, int nslice, int64_t slice_stride, hipStream_t s) {
    GemmArgs g{A, B, bias, C, H, M, N, K, sam, sak, sbk, sbn, ldc, (K + nslice - 1) / nslice, slice_stride};
    hipLaunchKernelGGL(k_gemm, dim3((N + 63) / 64, (M + 63) / 64, nslice), dim3(256), 0, s, g);
    return hipGetLastError();
}
}  // namespace

// One forward + backward pass over a batch in FP32: gradient (flat layout) into ctx->mlp_G
// and the mean loss into *loss.  Work buffers come from ctx->mlp_work (grown on demand).
hipError_t mlp_grad(qed_ctx *ctx, const float *X, const float *T, int64_t n, const float w[3], float *loss,
                    hipStream_t s) {
    const int64_t B = n;
    constexpr int NS = 64;    // K slices of the weight gradients (64 x 64 tiles x slices fill the chip)
    constexpr int NSB = 128;  // row slices of the bias gradients
    static_assert(NSB * 128 <= NS * 128 * 128, "bias partial sums fit the slice buffer");
    const int64_t need = (int64_t)(3 * 2 * B * 128 + 2 * B * 3 + NS * 128 * 128 + 1024 + 64);
    if (need > ctx->mlp_work_len) {
        (void)hipFree(ctx->mlp_work);
        ctx->mlp_work = nullptr;
        ctx->mlp_work_len = 0;
        hipError_t e = hipMalloc(&ctx->mlp_work, need * sizeof(float));
        if (e != hipSuccess) return e;
        ctx->mlp_work_len = need;
    }
    float *Z1 = ctx->mlp_work, *H1 = Z1 + B * 128, *Z2 = H1 + B * 128, *H2 = Z2 + B * 128, *Z3 = H2 + B * 128,
          *H3 = Z3 + B * 128, *Yo = H3 + B * 128, *dY = Yo + B * 3, *part = dY + B * 3, *lpart = part + NS * 128 * 128;
    const float *P = ctx->mlp_P;
    float *G = ctx->mlp_G;
    hipError_t e;
#define QED_TRY(x) \
    if ((e = (x)) != hipSuccess) return e
    // forward: Z = H W + b, H = SiLU(Z)
    QED_TRY(gemm(X, 4, 1, P + MLP_OW1, 128, 1, Z1, 128, (int)B, 128, 4, P + MLP_OB1, H1, 1, 0, s));
    QED_TRY(gemm(H1, 128, 1, P + MLP_OW2, 128, 1, Z2, 128, (int)B, 128, 128, P + MLP_OB2, H2, 1, 0, s));
    QED_TRY(gemm(H2, 128, 1, P + MLP_OW3, 128, 1, Z3, 128, (int)B, 128, 128, P + MLP_OB3, H3, 1, 0, s));
    QED_TRY(gemm(H3, 128, 1, P + MLP_OW4, 3, 1, Yo, 3, (int)B, 3, 128, P + MLP_OB4, nullptr, 1, 0, s));
    const int lb = 64;
    hipLaunchKernelGGL(k_loss, dim3(lb), dim3(256), 0, s, Yo, T, B, w[0], w[1], w[2], dY, lpart);
    QED_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(64), 0, s, lpart, lb, B, loss);
    QED_TRY(hipGetLastError());
    // backward, last layer first: dW = H^T dZ (split over the batch), db = column sums,
    // dH = dZ W^T, dZ_prev = dH * SiLU'(Z_prev)
    struct Lay { const float *Hin; int in; const float *W; int out; int ow, ob; float *Zin; };
    const Lay lay[4] = {{X, 4, P + MLP_OW1, 128, MLP_OW1, MLP_OB1, nullptr},
                        {H1, 128, P + MLP_OW2, 128, MLP_OW2, MLP_OB2, Z1},
                        {H2, 128, P + MLP_OW3, 128, MLP_OW3, MLP_OB3, Z2},
                        {H3, 128, P + MLP_OW4, 3, MLP_OW4, MLP_OB4, Z3}};
    float *dZ = dY;   // dL/dZ of the current layer [B][out]
    for (int L = 3; L >= 0; --L) {
        const Lay &l = lay[L];
        // dW [in][out] = sum_b Hin[b][in] dZ[b][out]
        QED_TRY(gemm(l.Hin, 1, l.in, dZ, l.out, 1, part, l.out, l.in, l.out, (int)B, nullptr, nullptr, NS,
                     (int64_t)l.in * l.out, s));
        hipLaunchKernelGGL(k_sum_slices, dim3((l.in * l.out + 255) / 256), dim3(256), 0, s, part, NS,
                           (int64_t)l.in * l.out, G + l.ow);
        QED_TRY(hipGetLastError());
        const int rps = (int)((B + NSB - 1) / NSB);
        hipLaunchKernelGGL(k_colsum, dim3((l.out + 63) / 64, NSB), dim3(256), 0, s, dZ, B, l.out, rps, part);
        QED_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_sum_slices, dim3((l.out + 255) / 256), dim3(256), 0, s, part, NSB, (int64_t)l.out,
                           G + l.ob);
        QED_TRY(hipGetLastError());
        if (L == 0) break;
        // dH [B][in] = dZ [B][out] W^T, written over this layer's input activations (their
        // weight gradient is done), then dZ_prev = dH * SiLU'(Z_prev) in place
        float *dH = L == 3 ? H3 : (L == 2 ? H2 : H1);
        QED_TRY(gemm(dZ, l.out, 1, l.W, 1, l.out, dH, l.in, (int)B, l.in, l.out, nullptr, nullptr, 1, 0, s));
        const int64_t cnt = B * l.in;
        hipLaunchKernelGGL(k_silu_back, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, dH, l.Zin, dH, cnt);
        QED_TRY(hipGetLastError());
        dZ = dH;
    }
#undef QED_TRY
    return hipSuccess;
}

hipError_t mlp_adam(qed_ctx *ctx, float lr, hipStream_t s) {
    ctx->mlp_t += 1;
    hipLaunchKernelGGL(k_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, ctx->mlp_P, ctx->mlp_G, ctx->mlp_m,
                       ctx->mlp_v, (int64_t)MLP_NPARAM, lr, 0.9f, 0.999f, 1e-8f, ctx->mlp_t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return mlp_pack(ctx, s);
}

}  // namespace qed
