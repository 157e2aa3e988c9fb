// Detector diagnostics: the post-processing step of the VB algorithm (Sec. III.F) on the
// device.  Particles heading to +x are binned on two axes; per bin the kernel adds w,
// w eps and w times the photon Stokes vector in the detector's polarisation basis (or the
// lepton spin) to a caller-owned FP64 histogram.
//
// Bin decisions use only correctly rounded operations (division, square root, multiply,
// floor, comparison with host-computed edges) evaluated in the order of the definition
// with contraction off, so they agree with any implementation of the same definition.
#include "qed_dev.hpp"

namespace qed {
namespace {

__device__ __forceinline__ int64_t clamp_count64(const int64_t *count, int64_t capacity) {
    const int64_t n = *count;
    return n < 0 ? 0 : (n > capacity ? capacity : n);
}

__device__ __forceinline__ int hist_bin(const HistArgs &a, const double *edges, int k, double v) {
    if (k == a.eaxis) {
        const int n = a.n[k];
        if (!(v >= edges[0]) || !(v < edges[n])) return -1;
        int lo = 0, hi = n;   // largest i < n with edges[i] <= v
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (edges[mid] <= v) lo = mid;
            else hi = mid;
        }
        return lo;
    }
    const double x = floor((v - a.lo[k]) * a.inv_w[k]);
    return (x >= 0.0 && x < (double)a.n[k]) ? (int)x : -1;
}

__device__ __forceinline__ int hist_cell(const HistArgs &a, const double *edges, const V3<double> &p, double energy) {
#pragma clang fp contract(off)
    if (!(p.x > 0.0)) return -1;
    double v[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        switch (a.axis[k]) {
        case QED_AX_SLOPE_Y: v[k] = p.y / p.x; break;
        case QED_AX_SLOPE_Z: v[k] = p.z / p.x; break;
        case QED_AX_SLOPE_R: v[k] = sqrt(p.y * p.y + p.z * p.z) / p.x; break;
        default: v[k] = energy; break;
        }
    }
    const int c0 = hist_bin(a, edges, 0, v[0]), c1 = hist_bin(a, edges, 1, v[1]);
    return (c0 < 0 || c1 < 0) ? -1 : c1 * a.n[0] + c0;
}

__device__ __forceinline__ double norm_exact(const V3<double> &v) {
#pragma clang fp contract(off)
    return sqrt(v.x * v.x + v.y * v.y + v.z * v.z);
}
__device__ __forceinline__ double gamma_exact(const V3<double> &p) {
#pragma clang fp contract(off)
    return sqrt(1.0 + (p.x * p.x + p.y * p.y + p.z * p.z));
}

// the block's histogram: one of a.rep replicas (blocks spread their atomics over the
// replicas, which a final pass adds up in a fixed order), or the output itself
__device__ __forceinline__ double *block_hist(const HistArgs &a) {
    return a.rep > 1 ? a.acc + (int64_t)(blockIdx.x % a.rep) * a.rep_stride : a.out;
}
__device__ __forceinline__ void add5(double *out, int cell, double a0, double a1, double a2, double a3, double a4) {
    double *o = out + 5 * (int64_t)cell;
    unsafeAtomicAdd(o + 0, a0);
    unsafeAtomicAdd(o + 1, a1);
    unsafeAtomicAdd(o + 2, a2);
    unsafeAtomicAdd(o + 3, a3);
    unsafeAtomicAdd(o + 4, a4);
}

template <class T>
__global__ __launch_bounds__(BLOCK) void k_hist_photons(HistArgs a) {
    __shared__ double s_edges[HIST_EMAX + 1];
    if (a.eaxis >= 0) {
        for (int k = threadIdx.x; k <= a.n[a.eaxis]; k += BLOCK) s_edges[k] = a.edges[k];
        __syncthreads();
    }
    const int64_t n = clamp_count64(a.G.count, a.G.capacity);
    const T *xi1 = (const T *)a.G.xi1, *xi2 = (const T *)a.G.xi2, *xi3 = (const T *)a.G.xi3;
    const T *e1x = (const T *)a.G.e1x, *e1y = (const T *)a.G.e1y, *e1z = (const T *)a.G.e1z;
    const V3<double> ref = {a.pol_ref[0], a.pol_ref[1], a.pol_ref[2]};
    double *hist = block_hist(a);
    for (int64_t j = a.begin + (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < n; j += (int64_t)gridDim.x * BLOCK) {
        if (!a.G.alive[j]) continue;
        const V3<double> k = {a.G.kx[j], a.G.ky[j], a.G.kz[j]};
        const double eps = norm_exact(k);
        const int cell = hist_cell(a, s_edges, k, eps);
        if (cell < 0) continue;
        // rotation from (e1, n x e1) to (d, n x d), d the part of pol_ref transverse to n
        // (eq. rotation, through cos 2psi and sin 2psi)
        const V3<double> nn = (1.0 / eps) * k;
        V3<double> d = ref - dot(nn, ref) * nn;
        d = rsqrt(dot(d, d)) * d;
        const V3<double> e1 = {(double)e1x[j], (double)e1y[j], (double)e1z[j]};
        const V3<double> e2 = cross(nn, e1);
        const double c = dot(e1, d), s = dot(e2, d), c2 = c * c - s * s, s2 = 2.0 * c * s;
        const double x1 = (double)xi1[j], x2 = (double)xi2[j], x3 = (double)xi3[j], w = a.G.w[j];
        add5(hist, cell, w, w * eps, w * (c2 * x1 - s2 * x3), w * x2, w * (s2 * x1 + c2 * x3));
    }
}

template <class T>
__global__ __launch_bounds__(BLOCK) void k_hist_leptons(HistArgs a) {
    __shared__ double s_edges[HIST_EMAX + 1];
    if (a.eaxis >= 0) {
        for (int k = threadIdx.x; k <= a.n[a.eaxis]; k += BLOCK) s_edges[k] = a.edges[k];
        __syncthreads();
    }
    const int64_t n = clamp_count64(a.L.count, a.L.capacity);
    const T *sx = (const T *)a.L.sx, *sy = (const T *)a.L.sy, *sz = (const T *)a.L.sz;
    double *hist = block_hist(a);
    for (int64_t i = a.begin + (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        const V3<double> p = {a.L.px[i], a.L.py[i], a.L.pz[i]};
        const double g = gamma_exact(p);
        const int cell = hist_cell(a, s_edges, p, g);
        if (cell < 0) continue;
        const double w = a.L.w[i];
        add5(hist, cell, w, w * g, w * (double)sx[i], w * (double)sy[i], w * (double)sz[i]);
    }
}

__global__ void k_zero(double *p, int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = 0.0;
}
// out[k] += rep[0][k] + rep[1][k] + ... (in replica order)
__global__ void k_hist_reduce(const double *rep, int R, int64_t len, double *out) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < len; k += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int r = 0; r < R; ++r) v += rep[(int64_t)r * len + k];
        out[k] += v;
    }
}

}  // namespace

// Replicas: when the list can hold several times as many particles as there are bins, the
// atomics of the bins a beam concentrates on contend; HIST_REP copies (context-owned,
// grown on demand, at most HIST_REP_MAX doubles) spread them.
constexpr int HIST_REP = 16;
constexpr int64_t HIST_REP_MAX = (int64_t)1 << 25;

hipError_t launch_hist(qed_ctx *ctx, const HistArgs &a0, bool photons, int64_t capacity, hipStream_t s) {
    HistArgs a = a0;
    const int64_t len = 5LL * a.n[0] * a.n[1];
    int64_t b = (capacity - a.begin + BLOCK - 1) / BLOCK;
    b = b < 1 ? 1 : (b > 65536 ? 65536 : b);
    a.rep = 1;
    if (capacity - a.begin >= 4 * (int64_t)a.n[0] * a.n[1] && HIST_REP * len <= HIST_REP_MAX && b >= HIST_REP) {
        if (ctx->hist_rep_len < HIST_REP * len) {
            (void)hipFree(ctx->hist_rep);
            ctx->hist_rep = nullptr;
            ctx->hist_rep_len = 0;
            const hipError_t e = hipMalloc(&ctx->hist_rep, HIST_REP * len * sizeof(double));
            if (e != hipSuccess) return e;
            ctx->hist_rep_len = HIST_REP * len;
        }
        a.rep = HIST_REP;
        a.acc = ctx->hist_rep;
        a.rep_stride = len;
        hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, s, a.acc, HIST_REP * len);
    }
    const dim3 gd((unsigned)b), bd(BLOCK);
    const bool mixed = ctx->cfg.precision == QED_MIXED;
    if (photons) {
        if (mixed) hipLaunchKernelGGL(k_hist_photons<float>, gd, bd, 0, s, a);
        else hipLaunchKernelGGL(k_hist_photons<double>, gd, bd, 0, s, a);
    } else {
        if (mixed) hipLaunchKernelGGL(k_hist_leptons<float>, gd, bd, 0, s, a);
        else hipLaunchKernelGGL(k_hist_leptons<double>, gd, bd, 0, s, a);
    }
    if (a.rep > 1) hipLaunchKernelGGL(k_hist_reduce, dim3(1024), dim3(256), 0, s, (const double *)a.acc, a.rep, len, a.out);
    return hipGetLastError();
}

}  // namespace qed
