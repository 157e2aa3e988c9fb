// GPU construction of the rate, spectrum, Bessel and birefringence tables in FP64.
//
// Special functions come from integral representations evaluated by quadrature on the
// device:  K_nu(x) = int_0^inf exp(-x cosh s) cosh(nu s) ds and int_x^inf K_nu = the same
// with an extra 1/cosh s (trapezoid rule, geometric convergence for this analytic even
// integrand); Scorer's Gi'(X) from its integral turned onto the ray arg t = pi/6, where it
// neither oscillates nor grows.  Integrals over the emitted-photon variable use
// t = (2u/(3chi))^(1/3) (u = omega/(eps - omega)), in which the integrands are analytic.
#include "qed_internal.hpp"

namespace qed {
namespace {

constexpr double PI_ = 3.14159265358979323846;
constexpr int GQ = 8;   // Gauss-Legendre points per panel
struct GaussRule {
    double x[GQ], w[GQ];
};

// Gauss-Legendre abscissae/weights on [-1, 1]: Newton iteration on P_8 from the
// asymptotic initial guess.
GaussRule make_rule() {
    GaussRule g{};
    for (int i = 0; i < GQ; ++i) {
        double z = std::cos(PI_ * (i + 0.75) / (GQ + 0.5)), dp = 0;
        for (int it = 0; it < 60; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= GQ; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = GQ * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        g.x[i] = z;
        g.w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    return g;
}

__device__ void bessel3(double x, double &k13, double &k23, double &ik13) {
    x = x > 1e-300 ? x : 1e-300;              // callers pass x > 0; keep the node count finite
    const double h = x > 16.0 ? 0.32 / sqrt(x) : 0.08;
    const double smax = acosh(1.0 + 70.0 / x) + 0.5;
    const int n = (int)fmin(smax / h, 20000.0) + 1;
    const double e0 = 0.5 * exp(-x);
    double a = e0, b = e0, c = e0;
    for (int i = 1; i <= n; ++i) {
        const double s = i * h, ch = cosh(s), e = exp(-x * ch);
        const double c1 = cosh(s * (1.0 / 3.0));
        a += e * c1;
        b += e * cosh(s * (2.0 / 3.0));
        c += e * c1 / ch;
    }
    k13 = h * a;
    k23 = h * b;
    ik13 = h * c;
}

// the trio times exp(x), integrating exp(-x (cosh s - 1)) so that large x cannot overflow
__device__ void bessel3_scaled(double x, double &k13, double &k23, double &ik13) {
    x = x > 1e-300 ? x : 1e-300;
    const double h = x > 16.0 ? 0.32 / sqrt(x) : 0.08;
    const double smax = acosh(1.0 + 70.0 / x) + 0.5;
    const int n = (int)fmin(smax / h, 20000.0) + 1;
    double a = 0.5, b = 0.5, c = 0.5;
    for (int i = 1; i <= n; ++i) {
        const double s = i * h, ch = cosh(s), sh = sinh(0.5 * s), e = exp(-2.0 * x * sh * sh);
        const double c1 = cosh(s * (1.0 / 3.0));
        a += e * c1;
        b += e * cosh(s * (2.0 / 3.0));
        c += e * c1 / ch;
    }
    k13 = h * a;
    k23 = h * b;
    ik13 = h * c;
}

__device__ double scorer_gip(double X, const GaussRule &g) {
    double S = 6.0;
    if (X > 0.0 && 80.0 / X < S) S = 80.0 / X;
    const int np = 40;
    const double hp = S / np;
    double sum = 0.0;
    for (int p = 0; p < np; ++p)
        for (int i = 0; i < GQ; ++i) {
            const double s = hp * (p + 0.5 * (g.x[i] + 1.0));
            sum += g.w[i] * s * exp(-s * s * s / 3.0 - 0.5 * X * s) * sin(0.8660254037844386 * X * s + 2.6179938779914944);
        }
    return 0.5 * hp * sum / PI_;
}

// NCS integrands in t: Ia-type (photon-summed, spin-independent) and Ib-type (spin part)
__device__ __forceinline__ void ncs_integrand(double chi, double t, double &fa, double &fb) {
    double K1, K2, I;
    bessel3(t * t * t, K1, K2, I);
    const double u = 1.5 * chi * t * t * t, jac = 4.5 * chi * t * t, o = 1.0 + u, o3 = o * o * o;
    fa = jac * (-(o)*I + (2.0 + 2.0 * u + u * u) * K2) / o3;
    fb = jac * u * K1 / o3;
}
__device__ __forceinline__ void nbw_integrand(double chi, double d, double &fa, double &fb) {
    const double dd = d * (1.0 - d), rho = 2.0 / (3.0 * chi * dd);
    if (!(dd > 0.0) || rho > 700.0) {
        fa = 0.0;
        fb = 0.0;
        return;
    }
    double K1, K2, I;
    bessel3(rho, K1, K2, I);
    fa = I + (d * d + (1.0 - d) * (1.0 - d)) / dd * K2;
    fb = K2;
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    return s;
}

__global__ void k_bessel(double *tab) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NB) return;
    const double x = exp(B_LO + i * ((B_HI - B_LO) / (NB - 1)));
    double K1, K2, I;
    bessel3_scaled(x, K1, K2, I);
    const double x13 = cbrt(x);
    double *o = tab + OFF_BES + 4 * i;
    o[0] = x13 * K1;
    o[1] = x13 * x13 * K2;
    o[2] = I;
    o[3] = 0.0;
}

// NCS total-rate integrals: one block per chi node
__global__ void k_ncs_rate(double *tab, GaussRule g) {
    __shared__ double sh[8];
    const int r = blockIdx.x;
    const double chi = exp(R_LO + r * ((R_HI - R_LO) / (NR - 1)));
    const double tcut = 3.9148676411688634, hp = 0.04;   // 60^(1/3): exp(-60) tail dropped
    const int np = (int)ceil(tcut / hp);
    const double hq = tcut / np;
    double sa = 0.0, sb = 0.0;
    for (int q = threadIdx.x; q < np * GQ; q += blockDim.x) {
        const int p = q / GQ, i = q % GQ;
        const double t = hq * (p + 0.5 * (g.x[i] + 1.0));
        double fa, fb;
        ncs_integrand(chi, t, fa, fb);
        sa += 0.5 * hq * g.w[i] * fa;
        sb += 0.5 * hq * g.w[i] * fb;
    }
    const double Ia = block_sum(sa, sh);
    const double Ib = block_sum(sb, sh);
    if (threadIdx.x == 0) {
        tab[OFF_NCS_RATE + 2 * r] = Ia / chi;
        tab[OFF_NCS_RATE + 2 * r + 1] = Ib / Ia;
    }
}

// Radiation-reaction coefficients on the NCS rate grid: the emitted power over the Larmor
// power (2/3) alpha chi^2 / xi_L, g = 3/(2 sqrt3 pi chi^2) int u w/(1+u)^4 du, and the
// radiative T-BMT integrals psi1 = int u''K23(u'), psi2 = int u''IntK13(u') - psi1,
// psi3 = int u''K13(u') with u'' = u^2/(1+u)^3, u' = 2u/(3chi) = t^3.  Stored as
// g (1+chi)^(4/3) and psi (1+chi)^(7/3)/chi^3, functions that are flat at both ends.
__global__ void k_rad_rate(double *tab, GaussRule g) {
    __shared__ double sh[8];
    const int r = blockIdx.x;
    const double chi = exp(R_LO + r * ((R_HI - R_LO) / (NR - 1)));
    const double tcut = 3.9148676411688634, hp = 0.04;   // as the NCS rates
    const int np = (int)ceil(tcut / hp);
    const double hq = tcut / np;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = threadIdx.x; q < np * GQ; q += blockDim.x) {
        const int p = q / GQ, i = q % GQ;
        const double t = hq * (p + 0.5 * (g.x[i] + 1.0));
        double K1, K2, I;
        bessel3(t * t * t, K1, K2, I);
        const double u = 1.5 * chi * t * t * t, jac = 4.5 * chi * t * t, o = 1.0 + u, o3 = o * o * o;
        const double wq = 0.5 * hq * g.w[i] * jac;
        s[0] += wq * u * (-o * I + (2.0 + 2.0 * u + u * u) * K2) / (o3 * o);
        s[1] += wq * u * u * K2 / o3;
        s[2] += wq * u * u * I / o3;
        s[3] += wq * u * u * K1 / o3;
    }
    double v[4];
    for (int k = 0; k < 4; ++k) v[k] = block_sum(s[k], sh);
    if (threadIdx.x == 0) {
        const double oc = cbrt(1.0 + chi), o43 = (1.0 + chi) * oc, o73 = (1.0 + chi) * (1.0 + chi) * oc;
        const double c3 = chi * chi * chi;
        double *o = tab + OFF_RAD + 4 * r;
        o[0] = 3.0 / (2.0 * 1.7320508075688772 * PI_ * chi * chi) * v[0] * o43;
        o[1] = v[1] * o73 / c3;
        o[2] = (v[2] - v[1]) * o73 / c3;
        o[3] = v[3] * o73 / c3;
    }
}

// per-interval integrals of the NCS spectrum pieces: scratch[2 * (row * NCT + j + 1)]
__global__ void k_ncs_panels(double *scratch, GaussRule g) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)NCR * (NCT - 1)) return;
    const int row = (int)(id / (NCT - 1)), j = (int)(id % (NCT - 1));
    const double chi = exp(C_LO + row * ((C_HI - C_LO) / (NCR - 1)));
    const double ht = T_MAX / (NCT - 1), t0 = j * ht;
    double sa = 0.0, sb = 0.0;
    for (int i = 0; i < GQ; ++i) {
        double fa, fb;
        ncs_integrand(chi, t0 + 0.5 * ht * (g.x[i] + 1.0), fa, fb);
        sa += g.w[i] * fa;
        sb += g.w[i] * fb;
    }
    scratch[2 * ((int64_t)row * NCT + j + 1)] = 0.5 * ht * sa;
    scratch[2 * ((int64_t)row * NCT + j + 1) + 1] = 0.5 * ht * sb;
}

// Gauss-Legendre over [lo, hi] of both NBW integrands
__device__ __forceinline__ void nbw_panel(double chi, double lo, double hi, const GaussRule &g, double &sa,
                                          double &sb) {
    const double h = hi - lo;
    double a = 0.0, b = 0.0;
    for (int i = 0; i < GQ; ++i) {
        double fa, fb;
        nbw_integrand(chi, lo + 0.5 * h * (g.x[i] + 1.0), fa, fb);
        a += g.w[i] * fa;
        b += g.w[i] * fb;
    }
    sa += 0.5 * h * a;
    sb += 0.5 * h * b;
}

// per-cell integrals; the first cell (from delta = 0) is split into halving panels because
// at large chi the spectrum switches on within delta ~ 1/chi
__global__ void k_nbw_panels(double *scratch, GaussRule g) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)NDR * (NDD - 1)) return;
    const int row = (int)(id / (NDD - 1)), j = (int)(id % (NDD - 1));
    const double chi = exp(P_LO + row * ((P_HI - P_LO) / (NDR - 1)));
    const double hd = 0.5 / (NDD - 1);
    double sa = 0.0, sb = 0.0;
    if (j == 0) {
        for (int k = 0; k < 52; ++k) nbw_panel(chi, ldexp(hd, -(k + 1)), ldexp(hd, -k), g, sa, sb);
    } else {
        nbw_panel(chi, j * hd, (j + 1) * hd, g, sa, sb);
    }
    scratch[2 * ((int64_t)row * NDD + j + 1)] = sa;
    scratch[2 * ((int64_t)row * NDD + j + 1) + 1] = sb;
}

// running sums along each row, normalised so the last column equals `last`
__global__ void k_cdf_rows(const double *scratch, double *out, int nrow, int ncol, double last) {
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= nrow) return;
    const double *s = scratch + 2 * (int64_t)row * ncol;
    double *o = out + 2 * (int64_t)row * ncol;
    double a = 0.0, b = 0.0;
    o[0] = 0.0;
    o[1] = 0.0;
    for (int j = 1; j < ncol; ++j) {
        a += s[2 * j];
        b += s[2 * j + 1];
        o[2 * j] = a;
        o[2 * j + 1] = b;
    }
    const double na = last / a, nb = last / b;
    for (int j = 1; j < ncol - 1; ++j) {
        o[2 * j] *= na;
        o[2 * j + 1] *= nb;
    }
    o[2 * (ncol - 1)] = last;
    o[2 * (ncol - 1) + 1] = last;
}

// NBW total-rate integrals: one block per chi node (the spectrum is symmetric in delta)
__global__ void k_nbw_rate(double *tab, GaussRule g) {
    __shared__ double sh[8];
    const int r = blockIdx.x;
    const double chi = exp(P_LO + r * ((P_HI - P_LO) / (NP - 1)));
    // [0, 1/64] in halving panels (onset at delta ~ 1/chi), then 124 panels up to 1/2
    const int ng = 50, nu = 124;
    const double g0 = 1.0 / 64.0, hq = (0.5 - g0) / nu;
    double sa = 0.0, sb = 0.0;
    for (int q = threadIdx.x; q < (ng + nu) * GQ; q += blockDim.x) {
        const int p = q / GQ, i = q % GQ;
        const double lo = p < ng ? ldexp(g0, -(p + 1)) : g0 + (p - ng) * hq;
        const double hi = p < ng ? ldexp(g0, -p) : g0 + (p - ng + 1) * hq;
        double fa, fb;
        nbw_integrand(chi, lo + 0.5 * (hi - lo) * (g.x[i] + 1.0), fa, fb);
        sa += 0.5 * (hi - lo) * g.w[i] * fa;
        sb += 0.5 * (hi - lo) * g.w[i] * fb;
    }
    const double Ja = 2.0 * block_sum(sa, sh);
    const double Jb = 2.0 * block_sum(sb, sh);
    if (threadIdx.x == 0) {
        tab[OFF_NBW_RATE + 2 * r] = Ja * exp(8.0 / (3.0 * chi)) / chi;
        tab[OFF_NBW_RATE + 2 * r + 1] = Jb / Ja;
    }
}

// VB coefficients M+, M-: one block per chi node, panels graded towards v = 1
__global__ void k_vb(double *tab, GaussRule g) {
    __shared__ double sh[8];
    const int r = blockIdx.x;
    const double chi = exp(V_LO + r * ((V_HI - V_LO) / (NV - 1)));
    const int np = 44;      // the last panel [1 - 2^-43, 1] adds O(2^-86)
    double sp = 0.0, sm = 0.0;
    for (int q = threadIdx.x; q < np * GQ; q += blockDim.x) {
        const int p = q / GQ, i = q % GQ;
        const double lo = 1.0 - ldexp(1.0, -p), hi = (p == np - 1) ? 1.0 : 1.0 - ldexp(1.0, -(p + 1));
        const double v = lo + 0.5 * (hi - lo) * (g.x[i] + 1.0), om = (1.0 - v) * (1.0 + v);
        if (!(om > 0.0)) continue;
        const double x = 4.0 / (om * chi), X = cbrt(x * x);
        const double core = PI_ * X * X * scorer_gip(X, g);
        const double wq = 0.5 * (hi - lo) * g.w[i] * om * core;
        sp += wq * 0.5 * (1.0 + v * v / 3.0);
        sm += wq * (1.0 - v * v / 3.0);
    }
    const double Mp = block_sum(sp, sh);
    const double Mm = block_sum(sm, sh);
    if (threadIdx.x == 0) {
        tab[OFF_VB + 2 * r] = -11.25 * Mp;
        tab[OFF_VB + 2 * r + 1] = -11.25 * Mm;
    }
}

__global__ void k_to_f32(const double *a, float *b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

// the paired-row copy of an FP32 spectrum CDF: out[r][c] = {A_r, B_r, A_r+1, B_r+1}[c]
__global__ void k_pair_rows(const float *src, float4 *out, int nrow, int ncol) {
    const int64_t n = (int64_t)(nrow - 1) * ncol;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / ncol, c = i - r * ncol;
        const float *a = src + 2 * (r * ncol + c), *b = src + 2 * ((r + 1) * ncol + c);
        out[i] = make_float4(a[0], a[1], b[0], b[1]);
    }
}

// ------------------------------------------------------------------ bremsstrahlung
// The braces of the cross-section of Sec. III.E with Tsai's screening functions (his fitted
// forms for Z >= 5), y dsigma/dy = alpha r0^2 max(braces, 0): near the tip of heavy atoms
// the Coulomb correction drives the braces below zero, where there is no cross-section.
__device__ double br_braces(double y, double E, const BremsDev &m) {
    const double q = 100.0 * y / ((1.0 - y) * E);
    const double g = q / m.z13, e = q / m.z23;
    const double p1 = 20.863 - 2.0 * log(1.0 + (0.55846 * g) * (0.55846 * g)) -
                      4.0 * (1.0 - 0.6 * exp(-0.9 * g) - 0.4 * exp(-1.5 * g));
    const double p2 = p1 - (2.0 / 3.0) / (1.0 + 6.5 * g + 6.0 * g * g);
    const double s1 = 28.340 - 2.0 * log(1.0 + (3.621 * e) * (3.621 * e)) -
                      4.0 * (1.0 - 0.7 * exp(-8.0 * e) - 0.3 * exp(-29.2 * e));
    const double s2 = s1 - (2.0 / 3.0) / (1.0 + 40.0 * e + 400.0 * e * e);
    const double Z = m.Z;
    const double a = (4.0 / 3.0 - 4.0 / 3.0 * y + y * y) *
                     (Z * Z * (p1 - 4.0 / 3.0 * m.lnZ - 4.0 * m.f) + Z * (s1 - 8.0 / 3.0 * m.lnZ));
    const double b = (2.0 / 3.0) * (1.0 - y) * (Z * Z * (p1 - p2) + Z * (s1 - s2));
    return fmax(a + b, 0.0);
}

// one block per energy node: the u intervals' integrals (one 8-point Gauss-Legendre rule in
// the logit t each, integrand y (1 - y) dsigma/dy), then their running sum in u order
__global__ void k_brems_rows(double *tab, BremsDev m, GaussRule g) {
    __shared__ double s_int[BR_NU];
    const int j = blockIdx.x;
    const double lnE = m.lnE0 + (m.lnE_hi - m.lnE0) * j / (BR_NE - 1);
    const double E = exp(lnE);
    const double ymin = m.k_cut / E;
    const double t0 = log(ymin / (1.0 - ymin)), t1 = log(E - 1.0);
    for (int i = threadIdx.x; i < BR_NU; i += blockDim.x) {
        double v = 0.0;
        if (i > 0) {
            const double a = t0 + (t1 - t0) * ((double)(i - 1) / (BR_NU - 1));
            const double b = t0 + (t1 - t0) * ((double)i / (BR_NU - 1));
            double sum = 0.0;
            for (int k = 0; k < GQ; ++k) {
                const double t = 0.5 * (a + b) + 0.5 * (b - a) * g.x[k];
                const double y = 1.0 / (1.0 + exp(-t));
                sum += g.w[k] * (m.ar02 * br_braces(y, E, m) * (1.0 - y));
            }
            v = 0.5 * (b - a) * sum;
        }
        s_int[i] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double *row = tab + BR_NE + (int64_t)j * BR_NU;
        double acc = 0.0;
        row[0] = 0.0;
        for (int i = 1; i < BR_NU; ++i) {
            acc += s_int[i];
            row[i] = acc;
        }
        tab[j] = acc;
    }
}

}  // namespace

hipError_t build_brems_tables(qed_ctx *ctx, hipStream_t s) {
    const GaussRule g = make_rule();
    hipLaunchKernelGGL(k_brems_rows, dim3(BR_NE), dim3(BR_NU), 0, s, ctx->br_tab64, ctx->br, g);
    hipLaunchKernelGGL(k_to_f32, dim3(64), dim3(256), 0, s, (const double *)ctx->br_tab64, ctx->br_tab32, BR_TAB_LEN);
    return hipGetLastError();
}

hipError_t build_tables(qed_ctx *ctx, hipStream_t s) {
    const GaussRule g = make_rule();
    double *scratch = nullptr;
    const int64_t ns = 2LL * NCR * NCT;   // larger of the two spectrum tables
    hipError_t e = hipMalloc(&scratch, ns * sizeof(double));
    if (e != hipSuccess) return e;
    double *tab = ctx->tab64;
    hipLaunchKernelGGL(k_bessel, dim3((NB + 255) / 256), dim3(256), 0, s, tab);
    hipLaunchKernelGGL(k_ncs_rate, dim3(NR), dim3(256), 0, s, tab, g);
    {
        const int64_t n = (int64_t)NCR * (NCT - 1);
        hipLaunchKernelGGL(k_ncs_panels, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, scratch, g);
        hipLaunchKernelGGL(k_cdf_rows, dim3((NCR + 63) / 64), dim3(64), 0, s, (const double *)scratch,
                           tab + OFF_NCS_CDF, NCR, NCT, 1.0);
    }
    hipLaunchKernelGGL(k_nbw_rate, dim3(NP), dim3(256), 0, s, tab, g);
    {
        const int64_t n = (int64_t)NDR * (NDD - 1);
        hipLaunchKernelGGL(k_nbw_panels, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, scratch, g);
        hipLaunchKernelGGL(k_cdf_rows, dim3((NDR + 63) / 64), dim3(64), 0, s, (const double *)scratch,
                           tab + OFF_NBW_CDF, NDR, NDD, 0.5);
    }
    hipLaunchKernelGGL(k_vb, dim3(NV), dim3(256), 0, s, tab, g);
    hipLaunchKernelGGL(k_rad_rate, dim3(NR), dim3(256), 0, s, tab, g);
    hipLaunchKernelGGL(k_to_f32, dim3(1024), dim3(256), 0, s, (const double *)tab, ctx->tab32, TAB_TOTAL);
    hipLaunchKernelGGL(k_pair_rows, dim3(1024), dim3(256), 0, s, (const float *)(ctx->tab32 + OFF_NCS_CDF),
                       (float4 *)(ctx->tab32 + OFF_NCS_CDF_PAIR), NCR, NCT);
    hipLaunchKernelGGL(k_pair_rows, dim3(1024), dim3(256), 0, s, (const float *)(ctx->tab32 + OFF_NBW_CDF),
                       (float4 *)(ctx->tab32 + OFF_NBW_CDF_PAIR), NDR, NDD);
    e = hipGetLastError();
    const hipError_t e2 = hipStreamSynchronize(s);
    hipFree(scratch);
    return e != hipSuccess ? e : e2;
}

}  // namespace qed
