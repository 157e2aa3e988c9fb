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
        add5(a.out, cell, w, w * eps, w * (c2 * x1 - s2 * x3), w * x2, w * (s2 * x1 + c2 * x3));
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
    for (int64_t i = a.begin + (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        const V3<double> p = {a.L.px[i], a.L.py[i], a.L.pz[i]};
        const double g = gamma_exact(p);
        const int cell = hist_cell(a, s_edges, p, g);
        if (cell < 0) continue;
        const double w = a.L.w[i];
        add5(a.out, cell, w, w * g, w * (double)sx[i], w * (double)sy[i], w * (double)sz[i]);
    }
}

}  // namespace

hipError_t launch_hist(qed_ctx *ctx, const HistArgs &a, bool photons, int64_t capacity, hipStream_t s) {
    int64_t b = (capacity - a.begin + BLOCK - 1) / BLOCK;
    b = b < 1 ? 1 : (b > 65536 ? 65536 : b);
    const dim3 gd((unsigned)b), bd(BLOCK);
    const bool mixed = ctx->cfg.precision == QED_MIXED;
    if (photons) {
        if (mixed) hipLaunchKernelGGL(k_hist_photons<float>, gd, bd, 0, s, a);
        else hipLaunchKernelGGL(k_hist_photons<double>, gd, bd, 0, s, a);
    } else {
        if (mixed) hipLaunchKernelGGL(k_hist_leptons<float>, gd, bd, 0, s, a);
        else hipLaunchKernelGGL(k_hist_leptons<double>, gd, bd, 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace qed
