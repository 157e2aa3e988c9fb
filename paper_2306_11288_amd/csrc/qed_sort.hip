// Reordering of a particle list by the grid bin of its particles (a data-layout step, not
// part of the physics): neighbouring particles then sit at neighbouring grid nodes, so the
// TSC gather of a wavefront reads shared cache lines instead of one line per lane, and the
// list stays ordered for the particles it gives birth to (born at their parent's place, in
// parent order).  The order is fixed by the data alone: a stable sort on the bin key
// (particles of one bin keep their list order), dead photons dropped.
//
// Method: a least-significant-digit radix sort of (key, index) pairs with two passes over
// 8-bit digits (keys < 2^16).  Each pass is a stable counting sort: every block of a fixed
// grid takes a contiguous range of the pairs, counts its digits in LDS, a scan over
// (digit, block) gives each block's first slot per digit, and the block writes its pairs in
// rounds of 256 (a round in list order): a pair's slot is its block's running offset for
// its digit + the pairs of that digit in earlier wavefronts of the round + those in earlier
// lanes of its wavefront (wave ballots).  No atomics decide a position; LDS atomics only
// count.  A last kernel gathers every array of the list through the final indices.
#include "qed_internal.hpp"

namespace qed {
namespace {

constexpr uint32_t KEY_NONE = 0xffffffffu;   // a dead photon: not sorted, not kept
constexpr int SORT_BLOCKS = 1024;            // blocks of the counting passes
constexpr int DIGITS = 256;

struct SortArgs {
    const double *x, *y;
    const uint8_t *alive;      // photons only (null for leptons)
    const int64_t *count;
    int64_t capacity;
    SortGrid g;
    uint32_t *key[2], *idx[2];
    int *hist;                 // [DIGITS][SORT_BLOCKS]
    const int64_t *off;        // exclusive prefix of hist, digit-major
    int64_t *nlive;            // particles kept (written by the scan of the first pass)
};

__device__ __forceinline__ int bin_of(double v, double v0, double inv, int nb) {
    const double f = floor((v - v0) * inv);
    if (!(f >= 0.0)) return 0;               // also NaN
    return f >= (double)(nb - 1) ? nb - 1 : (int)f;
}

// key of every particle [0, count): bin index by * nbx + bx, KEY_NONE for dead photons;
// index = position in the list
__global__ __launch_bounds__(BLOCK) void k_sort_keys(SortArgs a) {
    const int n = (int)(*a.count < 0 ? 0 : (*a.count > a.capacity ? a.capacity : *a.count));
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
        uint32_t k = KEY_NONE;
        if (!a.alive || a.alive[i]) {
            const int bx = bin_of(a.x[i], a.g.gx0, a.g.inv_bx, a.g.nbx);
            const int by = bin_of(a.y[i], a.g.gy0, a.g.inv_by, a.g.nby);
            k = (uint32_t)by * (uint32_t)a.g.nbx + (uint32_t)bx;
        }
        a.key[0][i] = k;
        a.idx[0][i] = (uint32_t)i;
    }
}

// pairs the pass works on: all of the list in the first pass, the kept ones in the second
__device__ __forceinline__ int pass_count(const SortArgs &a, int pass) {
    if (pass == 0) return (int)(*a.count < 0 ? 0 : (*a.count > a.capacity ? a.capacity : *a.count));
    return (int)*a.nlive;
}
// contiguous range [lo, hi) of block b (the same partition in the count and write kernels)
__device__ __forceinline__ void block_range(int n, int b, int &lo, int &hi) {
    int chunk = (n + SORT_BLOCKS - 1) / SORT_BLOCKS;
    chunk = (chunk + BLOCK - 1) / BLOCK * BLOCK;
    lo = b * chunk;
    hi = lo + chunk < n ? lo + chunk : n;
    if (lo > n) lo = n;
}

__global__ __launch_bounds__(BLOCK) void k_sort_count(SortArgs a, int pass) {
    __shared__ int h[DIGITS];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int n = pass_count(a, pass), shift = 8 * pass;
    int lo, hi;
    block_range(n, blockIdx.x, lo, hi);
    const uint32_t *key = a.key[pass];
    for (int i = lo + (int)threadIdx.x; i < hi; i += BLOCK) {
        const uint32_t k = key[i];
        if (k != KEY_NONE) atomicAdd(&h[(k >> shift) & 255u], 1);
    }
    __syncthreads();
    a.hist[threadIdx.x * SORT_BLOCKS + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(BLOCK) void k_sort_write(SortArgs a, int pass) {
    __shared__ int run[DIGITS];                 // next slot of each digit for this block
    __shared__ uint32_t wc[BLOCK / 64][DIGITS]; // per round: (round << 16) | pairs of the digit in the wave
    const int tid = (int)threadIdx.x, lane = tid & 63, wid = tid >> 6;
    run[tid] = (int)a.off[tid * SORT_BLOCKS + blockIdx.x];
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) wc[w][tid] = KEY_NONE;
    __syncthreads();
    const int n = pass_count(a, pass), shift = 8 * pass;
    int lo, hi;
    block_range(n, blockIdx.x, lo, hi);
    const uint32_t *kin = a.key[pass], *iin = a.idx[pass];
    uint32_t *kout = a.key[pass ^ 1], *iout = a.idx[pass ^ 1];
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int r0 = lo, round = 0; r0 < hi; r0 += BLOCK, ++round) {
        const int i = r0 + tid;
        const uint32_t k = i < hi ? kin[i] : KEY_NONE;
        const bool valid = k != KEY_NONE;
        const uint32_t d = valid ? (k >> shift) & 255u : 0u;
        // lanes of this wave holding a pair of the same digit
        unsigned long long same = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const unsigned long long m = __ballot((d >> bit) & 1u);
            same &= ((d >> bit) & 1u) ? m : ~m;
        }
        const int in_wave = __popcll(same & below);
        const bool first = valid && in_wave == 0;
        if (first) wc[wid][d] = ((uint32_t)round << 16) | (uint32_t)__popcll(same);
        __syncthreads();
        int slot = 0;
        if (valid) {
            int pre = 0;
            for (int w = 0; w < wid; ++w) {
                const uint32_t v = wc[w][d];
                pre += (v >> 16) == (uint32_t)round ? (int)(v & 0xffffu) : 0;
            }
            slot = run[d] + pre + in_wave;
        }
        __syncthreads();
        {   // advance the running slot of digit tid by this round's pairs of that digit
            int add = 0;
#pragma unroll
            for (int w = 0; w < BLOCK / 64; ++w) {
                const uint32_t v = wc[w][tid];
                add += (v >> 16) == (uint32_t)round ? (int)(v & 0xffffu) : 0;
            }
            run[tid] += add;
        }
        if (valid) {
            kout[slot] = k;
            iout[slot] = iin[i];
        }
        __syncthreads();
    }
}

struct GatherPhotons {
    qed_photons in, out;
    const uint32_t *idx;
    const int64_t *nlive;
    uint32_t *status;
    int mixed;
};
template <class T>
__global__ __launch_bounds__(BLOCK) void k_sort_gather_photons(GatherPhotons a) {
    const int64_t n = *a.nlive;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *a.out.count = n < a.out.capacity ? n : a.out.capacity;
        if (n > a.out.capacity) atomicOr(a.status, QED_ST_OVERFLOW);
    }
    for (int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x; p < n && p < a.out.capacity;
         p += (int64_t)gridDim.x * BLOCK) {
        const int64_t j = a.idx[p];
        a.out.x[p] = a.in.x[j]; a.out.y[p] = a.in.y[j]; a.out.z[p] = a.in.z[j];
        a.out.kx[p] = a.in.kx[j]; a.out.ky[p] = a.in.ky[j]; a.out.kz[p] = a.in.kz[j];
        a.out.w[p] = a.in.w[j];
        ((T *)a.out.xi1)[p] = ((const T *)a.in.xi1)[j];
        ((T *)a.out.xi2)[p] = ((const T *)a.in.xi2)[j];
        ((T *)a.out.xi3)[p] = ((const T *)a.in.xi3)[j];
        ((T *)a.out.e1x)[p] = ((const T *)a.in.e1x)[j];
        ((T *)a.out.e1y)[p] = ((const T *)a.in.e1y)[j];
        ((T *)a.out.e1z)[p] = ((const T *)a.in.e1z)[j];
        a.out.id[p] = a.in.id[j];
        a.out.alive[p] = 1;
    }
}
struct GatherLeptons {
    qed_leptons in, out;
    const uint32_t *idx;
    const int64_t *nlive;
    uint32_t *status;
};
template <class T>
__global__ __launch_bounds__(BLOCK) void k_sort_gather_leptons(GatherLeptons a) {
    const int64_t n = *a.nlive;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *a.out.count = n < a.out.capacity ? n : a.out.capacity;
        if (n > a.out.capacity) atomicOr(a.status, QED_ST_OVERFLOW);
    }
    for (int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x; p < n && p < a.out.capacity;
         p += (int64_t)gridDim.x * BLOCK) {
        const int64_t j = a.idx[p];
        a.out.x[p] = a.in.x[j]; a.out.y[p] = a.in.y[j]; a.out.z[p] = a.in.z[j];
        a.out.px[p] = a.in.px[j]; a.out.py[p] = a.in.py[j]; a.out.pz[p] = a.in.pz[j];
        a.out.w[p] = a.in.w[j];
        ((T *)a.out.sx)[p] = ((const T *)a.in.sx)[j];
        ((T *)a.out.sy)[p] = ((const T *)a.in.sy)[j];
        ((T *)a.out.sz)[p] = ((const T *)a.in.sz)[j];
        a.out.id[p] = a.in.id[j];
    }
}

// work memory: keys and indices twice, digit counts, their prefix, the kept count
hipError_t ensure_sort_work(qed_ctx *ctx, int64_t capacity, SortArgs &a) {
    auto al = [](int64_t b) { return (b + 255) / 256 * 256; };
    const int64_t nh = (int64_t)DIGITS * SORT_BLOCKS;
    const int64_t need = 4 * al(capacity * 4) + al(nh * 4) + al((nh + 1) * 8) + al(8);
    if (capacity > ctx->sort_cap || !ctx->sort_work) {
        hipFree(ctx->sort_work);
        ctx->sort_work = nullptr;
        ctx->sort_cap = 0;
        const hipError_t e = hipMalloc(&ctx->sort_work, (size_t)need);
        if (e != hipSuccess) return e;
        ctx->sort_cap = capacity;
    }
    char *q = (char *)ctx->sort_work;
    const int64_t cap4 = al(ctx->sort_cap * 4);
    a.key[0] = (uint32_t *)q; q += cap4;
    a.key[1] = (uint32_t *)q; q += cap4;
    a.idx[0] = (uint32_t *)q; q += cap4;
    a.idx[1] = (uint32_t *)q; q += cap4;
    a.hist = (int *)q; q += al(nh * 4);
    a.off = (const int64_t *)q; q += al((nh + 1) * 8);
    a.nlive = (int64_t *)q;
    return hipSuccess;
}

hipError_t sort_pairs(qed_ctx *ctx, SortArgs &a, hipStream_t s) {
    const int64_t kb = (a.capacity + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL(k_sort_keys, dim3((unsigned)(kb < 1 ? 1 : (kb < 8192 ? kb : 8192))), dim3(BLOCK), 0, s, a);
    hipError_t e = hipGetLastError();
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
        hipLaunchKernelGGL(k_sort_count, dim3(SORT_BLOCKS), dim3(BLOCK), 0, s, a, pass);
        if ((e = hipGetLastError()) != hipSuccess) break;
        e = launch_scan_ints(ctx, a.hist, (int64_t)DIGITS * SORT_BLOCKS, const_cast<int64_t *>(a.off), a.nlive,
                             ctx->launch, s);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_sort_write, dim3(SORT_BLOCKS), dim3(BLOCK), 0, s, a, pass);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace

hipError_t launch_sort_photons(qed_ctx *ctx, const qed_photons &in, const qed_photons &out, const SortGrid &g,
                               hipStream_t s) {
    SortArgs a{};
    a.x = in.x;
    a.y = in.y;
    a.alive = in.alive;
    a.count = in.count;
    a.capacity = in.capacity;
    a.g = g;
    hipError_t e = ensure_sort_work(ctx, in.capacity, a);
    if (e == hipSuccess) e = sort_pairs(ctx, a, s);
    if (e != hipSuccess) return e;
    GatherPhotons ga{in, out, a.idx[0], a.nlive, ctx->status, ctx->cfg.precision == QED_MIXED};
    const int64_t gb = (in.capacity + BLOCK - 1) / BLOCK;
    const dim3 gd((unsigned)(gb < 1 ? 1 : (gb < 4096 ? gb : 4096)));
    if (ga.mixed) hipLaunchKernelGGL(k_sort_gather_photons<float>, gd, dim3(BLOCK), 0, s, ga);
    else hipLaunchKernelGGL(k_sort_gather_photons<double>, gd, dim3(BLOCK), 0, s, ga);
    return hipGetLastError();
}

hipError_t launch_sort_leptons(qed_ctx *ctx, const qed_leptons &in, const qed_leptons &out, const SortGrid &g,
                               hipStream_t s) {
    SortArgs a{};
    a.x = in.x;
    a.y = in.y;
    a.alive = nullptr;
    a.count = in.count;
    a.capacity = in.capacity;
    a.g = g;
    hipError_t e = ensure_sort_work(ctx, in.capacity, a);
    if (e == hipSuccess) e = sort_pairs(ctx, a, s);
    if (e != hipSuccess) return e;
    GatherLeptons ga{in, out, a.idx[0], a.nlive, ctx->status};
    const int64_t gb = (in.capacity + BLOCK - 1) / BLOCK;
    const dim3 gd((unsigned)(gb < 1 ? 1 : (gb < 4096 ? gb : 4096)));
    if (ctx->cfg.precision == QED_MIXED) hipLaunchKernelGGL(k_sort_gather_leptons<float>, gd, dim3(BLOCK), 0, s, ga);
    else hipLaunchKernelGGL(k_sort_gather_leptons<double>, gd, dim3(BLOCK), 0, s, ga);
    return hipGetLastError();
}

}  // namespace qed
