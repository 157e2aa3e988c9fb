// Device-side physics of the QED particle step.  Everything here is per particle;
// templates take the "rate" real type T (double for FP64 contexts, float for mixed).
// Momenta, positions, event probabilities and their comparison are always double.
#pragma once
#include "qed_internal.hpp"

namespace qed {

constexpr double PI = 3.14159265358979323846;
constexpr double SQRT3 = 1.7320508075688772935;
constexpr double TWO_PI = 6.28318530717958647692;
constexpr uint32_t STREAM_NCS = 1, STREAM_NBW = 2, STREAM_MLP = 7;   // STREAM_MLP: learned-sampler data

// ------------------------------------------------------------------------- small vectors
template <class T>
struct V3 {
    T x, y, z;
};
template <class T>
__device__ __forceinline__ T dot(const V3<T> &a, const V3<T> &b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T>
__device__ __forceinline__ V3<T> cross(const V3<T> &a, const V3<T> &b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T>
__device__ __forceinline__ V3<T> operator+(const V3<T> &a, const V3<T> &b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T>
__device__ __forceinline__ V3<T> operator-(const V3<T> &a, const V3<T> &b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T>
__device__ __forceinline__ V3<T> operator*(T s, const V3<T> &a) { return {s * a.x, s * a.y, s * a.z}; }
template <class T, class U>
__device__ __forceinline__ V3<T> cvt(const V3<U> &a) { return {(T)a.x, (T)a.y, (T)a.z}; }

// ------------------------------------------------------------------------- Philox4x32-10
// Ten rounds of the Philox S-box (two 32x32 -> 64-bit products) with the Weyl key
// schedule between rounds (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // one 32 x 32 -> 64-bit product gives both halves (a single v_mad_u64_u32)
        const uint64_t m0 = (uint64_t)0xD2511F53u * c[0], m1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t lo0 = (uint32_t)m0, hi0 = (uint32_t)(m0 >> 32);
        const uint32_t lo1 = (uint32_t)m1, hi1 = (uint32_t)(m1 >> 32);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}
// four uniforms in (0,1) for (id, step, stream, seed)
__device__ __forceinline__ void uniform4(uint64_t id, int64_t step, uint32_t stream, uint64_t seed, double r[4]) {
    const uint64_t s = (uint64_t)step;
    uint32_t c[4] = {(uint32_t)s, (uint32_t)((s >> 32) & 0xFFFFu) | (stream << 16), (uint32_t)seed,
                     (uint32_t)(seed >> 32)};
    philox4x32_10(c, (uint32_t)id, (uint32_t)(id >> 32));
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = ((double)c[k] + 0.5) * 2.3283064365386963e-10;
}

// ------------------------------------------------------------------------- fields
// FT: real type of the transcendental work (double, or float after an FP64 reduction of
// the carrier phase).  Output fields are double.
// Reciprocal and natural log: FP32 uses the hardware approximations (v_rcp_f32, v_log_f32,
// about 1 ulp).  FP64: the hardware reciprocal estimate (v_rcp_f64) refined by two Newton
// steps, e = 1 - v r, r += r e, each squaring the relative error, so within an ulp or two
// of 1/v for the finite non-zero v it is used on (five instructions instead of the
// correctly rounded division's ten); the library log.
__device__ __forceinline__ float rcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double rcp(double v) {
    double r = __builtin_amdgcn_rcp(v);
    double e = fma(-v, r, 1.0);
    r = fma(r, e, r);
    e = fma(-v, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float lnx(float v) { return __builtin_amdgcn_logf(v) * 0.69314718055994531f; }
__device__ __forceinline__ double lnx(double v) { return log(v); }
// a - round(a) for a phase given in revolutions, i.e. the phase reduced to [-1/2, 1/2]
__device__ __forceinline__ double frac_rev(double a) { return a - rint(a); }
__device__ __forceinline__ float rsq(float v) { return rsqrtf(v); }
__device__ __forceinline__ double rsq(double v) { return rsqrt(v); }

// TSC weights of a node-centred (half = 0) or half-staggered (half = 1) component at grid
// position xg: the node and the offset from it in FP64 (positions), the weights in FT
template <class FT>
__device__ __forceinline__ void tsc_w(double xg, int half, int &j0, FT w[3]) {
    const int j = half ? (int)floor(xg) : (int)floor(xg + 0.5);
    const FT d = (FT)(xg - ((double)j + (half ? 0.5 : 0.0)));
    w[0] = (FT)0.5 * ((FT)0.5 - d) * ((FT)0.5 - d);
    w[1] = (FT)0.75 - d * d;
    w[2] = (FT)0.5 * ((FT)0.5 + d) * ((FT)0.5 + d);
    j0 = j - 1;
}

// TSC gather of one staggered component at (x, y); row(j, on_grid, s) gives the three
// consecutive nodes s, s+1, s+2 of grid row j (any finite values where on_grid is false:
// they get weight zero)
template <class FT, class RowFn>
__device__ __forceinline__ double tsc_gather(const GridDev &f, int hx, int hy, double x, double y, RowFn row) {
    int i0, j0;
    FT wx[3], wy[3];
    tsc_w<FT>((x - f.gx0) * f.inv_dx, hx, i0, wx);
    tsc_w<FT>((y - f.gy0) * f.inv_dy, hy, j0, wy);
    // A row's three taps are read by one load of three consecutive nodes s, s+1, s+2, with
    // s = i0 clamped into [0, nx - 3] (nx >= 3).  Node s + k is tap k - (i0 - s); every tap
    // on the grid falls in this window and every tap off it falls outside, so slot k takes
    // that tap's weight, or zero when there is no such tap.  Rows off the grid are read
    // with weight zero.  Zero-weighted terms add exactly zero.
    const int s = min(max(i0, 0), f.nx - 3), d = i0 - s;
    FT ws[3], wr[3];
    int jj[3];
    bool on[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int a = k - d, j = j0 + k;
        // selects, not branches: a is the same for every lane away from the grid's edges
        const FT s01 = a == 0 ? wx[0] : wx[1], s2 = a == 2 ? wx[2] : (FT)0;
        ws[k] = (a == 0 || a == 1) ? s01 : s2;
        on[k] = j >= 0 && j < f.ny;
        jj[k] = j;
        wr[k] = on[k] ? wy[k] : (FT)0;
    }
    FT sum = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const float *r = row(jj[b], on[b], s);
        const float v0 = r[0], v1 = r[1], v2 = r[2];
        sum += wr[b] * (ws[0] * (FT)v0 + ws[1] * (FT)v1 + ws[2] * (FT)v2);
    }
    return (double)sum;
}

// from the grid in global memory (rows off the grid read at row 0)
template <class FT>
__device__ __forceinline__ double grid_gather(const GridDev &f, const float *__restrict__ g, int hx, int hy,
                                              double x, double y) {
    // 32-bit byte offsets from the array base (grids hold fewer than 2^29 nodes)
    const char *gb = (const char *)g;
    return tsc_gather<FT>(f, hx, hy, x, y, [&](int j, bool on, int s) {
        return (const float *)(gb + 4u * ((uint32_t)(on ? j : 0) * (uint32_t)f.nx + (uint32_t)s));
    });
}

// The grid gather of a wavefront whose particles lie close together (a list sorted by grid
// bin): the w x h nodes that the live lanes' stencils touch (any stagger), for all six
// components, are staged in the wavefront's own LDS box (at most WB_NODES nodes per
// component) with one or two coalesced loads per component, one float per lane each, and
// the taps are read from there.  Six to twelve vector memory instructions per wavefront
// instead of eighteen three-float loads per lane, which the texture-address unit otherwise
// works through lane by lane.  No block barrier: the box is the wavefront's, whose LDS
// writes are ordered before its reads by a wavefront-scope fence.  Returns false (nothing
// done) when the stencils do not fit one box inside the grid; the caller then gathers from
// global memory.  Every lane of the wavefront must call it.
constexpr int WB_NODES = 128;                   // nodes per component, two loads per lane
constexpr int WB_FLOATS = 6 * WB_NODES;         // per wavefront
// minimum over the wavefront (all 64 lanes active): running minima over 2, 4, 8, 16 lanes
// of each row by row shifts, then across rows by the row broadcasts; lane 63 holds the
// result.  Lanes without a source keep the identity.
__device__ __forceinline__ int wave_min_i(int v) {
    constexpr int ID = 0x7fffffff;
    v = min(v, __builtin_amdgcn_update_dpp(ID, v, 0x111, 0xf, 0xf, false));   // row_shr:1
    v = min(v, __builtin_amdgcn_update_dpp(ID, v, 0x112, 0xf, 0xf, false));   // row_shr:2
    v = min(v, __builtin_amdgcn_update_dpp(ID, v, 0x114, 0xf, 0xf, false));   // row_shr:4
    v = min(v, __builtin_amdgcn_update_dpp(ID, v, 0x118, 0xf, 0xf, false));   // row_shr:8
    v = min(v, __builtin_amdgcn_update_dpp(ID, v, 0x142, 0xa, 0xf, false));   // row_bcast:15
    v = min(v, __builtin_amdgcn_update_dpp(ID, v, 0x143, 0xc, 0xf, false));   // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}
// sum over the wavefront (all 64 lanes active); every lane gets the total
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
    long long x = (long long)v;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
    return (int64_t)x;
}
template <class FT>
__device__ __forceinline__ bool grid_fields_wavebox(const GridDev &f, float *box, bool live, double x, double y,
                                                    V3<double> &E, V3<double> &B) {
    // stencil nodes of any staggering: columns floor(X) - 1 .. floor(X + 1/2) + 1, rows alike
    const double X = (x - f.gx0) * f.inv_dx, Y = (y - f.gy0) * f.inv_dy;
    constexpr int BIG = 0x3fffffff;
    int v[4] = {BIG, BIG, BIG, BIG};
    if (live) {
        if (fabs(X) < 1e9 && fabs(Y) < 1e9) {
            v[0] = (int)floor(X) - 1;
            v[1] = (int)floor(Y) - 1;
            v[2] = -((int)floor(X + 0.5) + 1);
            v[3] = -((int)floor(Y + 0.5) + 1);
        } else {
            v[0] = -BIG;                        // far off the grid or not finite: no box
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = wave_min_i(v[k]);
    const int i0 = v[0], j0 = v[1], i1 = -v[2], j1 = -v[3];
    // no live lane (i0 = BIG), a lane off the grid, or a box too large
    if (i0 < 0 || j0 < 0 || i0 == BIG || i1 >= f.nx || j1 >= f.ny)
        return false;
    const int w = i1 - i0 + 1, h = j1 - j0 + 1;
    if (w > WB_NODES || h > WB_NODES || w * h > WB_NODES)
        return false;
    // fill: element c WB_NODES + e of the box, e = r w + q < w h, is node (i0 + q, j0 + r)
    // of component c; lane l loads e = l and, where w h > 64, e = l + 64 (elements past
    // w h repeat the last node: in bounds, never read)
    static_assert(WB_NODES > 64 && WB_NODES <= 128, "at most two loads per lane and component");
    const int wh = w * h, l0 = threadIdx.x & 63, l1 = l0 + 64;
    const int e0 = min(l0, wh - 1), e1 = min(l1, wh - 1);
    // e / w as floor((e + 1/2) / w) in FP32: exact, the quotient being at least 1/(2w)
    // away from an integer (e < 128, w <= 128) and the FP32 error far below that
    const float iw = __builtin_amdgcn_rcpf((float)w);
    const int r0 = (int)(((float)e0 + 0.5f) * iw), r1 = (int)(((float)e1 + 0.5f) * iw);
    // 32-bit byte offsets from the arrays' bases (grids hold fewer than 2^29 nodes)
    const uint32_t o0 = 4u * (uint32_t)((j0 + r0) * f.nx + i0 + e0 - r0 * w);
    const uint32_t o1 = 4u * (uint32_t)((j0 + r1) * f.nx + i0 + e1 - r1 * w);
    float u[12];
#pragma unroll
    for (int c = 0; c < 6; ++c) u[2 * c] = *(const float *)((const char *)f.g[c] + o0);
    if (wh > 64) {
#pragma unroll
        for (int c = 0; c < 6; ++c) u[2 * c + 1] = *(const float *)((const char *)f.g[c] + o1);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) box[c * WB_NODES + l0] = u[2 * c];
    if (wh > 64) {
#pragma unroll
        for (int c = 0; c < 6; ++c) box[c * WB_NODES + l1] = u[2 * c + 1];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (live) {
        // the TSC taps of each stagger (every tap inside the box: no edge handling), summed
        // in the order of tsc_gather
        int ix[2], jy[2];
        FT wx[2][3], wy[2][3];
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            tsc_w<FT>(X, hf, ix[hf], wx[hf]);
            tsc_w<FT>(Y, hf, jy[hf], wy[hf]);
        }
        auto from = [&](int c, int hx, int hy) {
            const float *r = box + c * WB_NODES + (jy[hy] - j0) * w + (ix[hx] - i0);
            FT sum = 0;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const float *rb = r + b * w;
                sum += wy[hy][b] * (wx[hx][0] * (FT)rb[0] + wx[hx][1] * (FT)rb[1] + wx[hx][2] * (FT)rb[2]);
            }
            return (double)sum;
        };
        E = {from(0, 1, 0), from(1, 0, 1), from(2, 0, 0)};
        __builtin_amdgcn_sched_barrier(0);
        B = {from(3, 0, 1), from(4, 1, 0), from(5, 1, 1)};
    }
    // the box is read before the next tile's fill overwrites it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return true;
}

// Laser pulses (plane wave E = -dA/dphi with a sin^2 envelope; paraxial Gaussian beam at
// zeroth order), KIND = QED_FIELD_PW or QED_FIELD_GAUSS.  In single precision every phase
// is reduced in FP64 and handed to the hardware sine / cosine in revolutions (v_sin_f32
// and v_cos_f32 return sin(2 pi x), cos(2 pi x)); the Gaussian amplitude uses v_exp_f32,
// v_rsq_f32 and v_rcp_f32.
template <class FT, int KIND>
__device__ __forceinline__ void field_pulse(const FieldDev &f, double t, double x, double y, double z,
                                            V3<double> &E, V3<double> &B) {
    const PulseDev &P = f.p;
    E = {0, 0, 0};
    B = {0, 0, 0};
    const double phi = t + x - P.phi_start;
    if (phi < 0.0 || phi > P.L) return;
    FT c1, c2;
    if constexpr (sizeof(FT) == 4) {
        constexpr double INV_2PI = 0.15915494309189535;
        const float se = __builtin_amdgcn_sinf((float)(phi * P.inv_2L));   // sin(pi phi / L)
        const float env = se * se;
        const double rev = frac_rev((phi + P.phase0) * INV_2PI);
        if constexpr (KIND == QED_FIELD_PW) {
            // d env / d phi = (pi/L) sin(2 pi phi / L)
            const float denv = P.f_pi_over_L * __builtin_amdgcn_sinf((float)frac_rev(phi * P.inv_L));
            const float ss = __builtin_amdgcn_sinf((float)rev), cs = __builtin_amdgcn_cosf((float)rev);
            const float a0 = P.f_a0;
            c1 = -a0 * (denv * ss + env * cs);
            c2 = f.circular ? -a0 * (denv * cs - env * ss) : 0.0f;
        } else {
            const float zr = P.f_zr;
            const float xi = (float)(P.x_focus - x);
            const float rho2 = (float)(y * y + z * z);
            const float q = xi * P.f_inv_zr, opq = 1.0f + q * q, iopq = rcp(opq);
            constexpr float LOG2E = 1.4426950408889634f;
            const float amp = P.f_a0 * __builtin_amdgcn_rsqf(opq) *
                              __builtin_amdgcn_exp2f(-LOG2E * rho2 * P.f_inv_w0sq * iopq);
            const float small = atanf(q) - 0.5f * rho2 * xi * rcp(xi * xi + zr * zr);
            const float ph = (float)rev + small * (float)INV_2PI;
            const float ss = __builtin_amdgcn_sinf(ph), cs = __builtin_amdgcn_cosf(ph);
            c1 = amp * env * cs;
            c2 = f.circular ? amp * env * ss : 0.0f;
        }
    } else {
        // phases in half-turns, reduced to [-1, 1] before sinpi / cospi, which then need
        // no large-argument reduction
        constexpr double INV_PI = 0.3183098861837907;
        double env = sinpi(phi * P.inv_L);      // sin(pi phi / L), phi / L in [0, 1]
        env *= env;
        if constexpr (KIND == QED_FIELD_PW) {
            const double denv = P.pi_over_L * sinpi(2.0 * frac_rev(phi * P.inv_L));
            double ss, cs;
            sincospi(2.0 * frac_rev((phi + P.phase0) * (0.5 * INV_PI)), &ss, &cs);
            c1 = -P.a0 * (denv * ss + env * cs);
            c2 = f.circular ? -P.a0 * (denv * cs - env * ss) : 0.0;
        } else {
            const double xi = P.x_focus - x;
            const double rho2 = y * y + z * z;
            // xi / (xi^2 + zr^2) = (q / zr) / (1 + q^2): one reciprocal serves the width, the
            // Gaussian and the curvature term
            const double q = xi * P.inv_zr, opq = 1.0 + q * q, iopq = rcp(opq);
            const double amp = P.a0 * rsqrt(opq) * exp(-rho2 * P.inv_w0sq * iopq);
            const double small = atan(q) - 0.5 * rho2 * q * P.inv_zr * iopq;
            double ss, cs;
            sincospi(2.0 * frac_rev((phi + P.phase0) * (0.5 * INV_PI)) + small * INV_PI, &ss, &cs);
            c1 = amp * env * cs;
            c2 = f.circular ? amp * env * ss : 0.0;
        }
    }
    FT cp, sp;
    if constexpr (sizeof(FT) == 4) {
        cp = P.f_cp;
        sp = P.f_sp;
    } else {
        cp = P.cp;
        sp = P.sp;
    }
    E.y = (double)(c1 * cp - c2 * sp);
    E.z = (double)(c1 * sp + c2 * cp);
    B.y = E.z;
    B.z = -E.y;
}

// 2D Yee grid (TSC gather of the six staggered components), uniform field, nothing
template <class FT, int KIND>
__device__ __forceinline__ void field_kind(const FieldDev &f, double t, double x, double y, double z,
                                           V3<double> &E, V3<double> &B) {
    if constexpr (KIND == QED_FIELD_PW || KIND == QED_FIELD_GAUSS) {
        field_pulse<FT, KIND>(f, t, x, y, z, E, B);
    } else if constexpr (KIND == QED_FIELD_GRID2D) {
        E.x = grid_gather<FT>(f.g, f.g.g[0], 1, 0, x, y);
        E.y = grid_gather<FT>(f.g, f.g.g[1], 0, 1, x, y);
        E.z = grid_gather<FT>(f.g, f.g.g[2], 0, 0, x, y);
        // E's nine loads, then B's: all eighteen in flight at once would hold 54 registers
        __builtin_amdgcn_sched_barrier(0);
        B.x = grid_gather<FT>(f.g, f.g.g[3], 0, 1, x, y);
        B.y = grid_gather<FT>(f.g, f.g.g[4], 1, 0, x, y);
        B.z = grid_gather<FT>(f.g, f.g.g[5], 1, 1, x, y);
    } else if constexpr (KIND == QED_FIELD_CONST) {
        E = {f.c.e0[0], f.c.e0[1], f.c.e0[2]};
        B = {f.c.b0[0], f.c.b0[1], f.c.b0[2]};
    } else {
        E = {0, 0, 0};
        B = {0, 0, 0};
    }
}
// field kind chosen at run time
template <class FT>
__device__ void field_at(const FieldDev &f, double t, double x, double y, double z, V3<double> &E, V3<double> &B) {
    switch (f.kind) {
    case QED_FIELD_CONST: field_kind<FT, QED_FIELD_CONST>(f, t, x, y, z, E, B); return;
    case QED_FIELD_PW: field_kind<FT, QED_FIELD_PW>(f, t, x, y, z, E, B); return;
    case QED_FIELD_GAUSS: field_kind<FT, QED_FIELD_GAUSS>(f, t, x, y, z, E, B); return;
    case QED_FIELD_GRID2D: field_kind<FT, QED_FIELD_GRID2D>(f, t, x, y, z, E, B); return;
    default: field_kind<FT, QED_FIELD_NONE>(f, t, x, y, z, E, B); return;
    }
}

// ------------------------------------------------------------------------- push + spin
// Boris rotation (eqs. boris1-boris6): p in/out p^{n-1/2} -> p^{n+1/2}; returns p-, p+
// and 1/gamma^n = 1/sqrt(1 + |p-|^2).
__device__ __forceinline__ double boris(double q, double dt, const V3<double> &E, const V3<double> &B, V3<double> &p,
                                        V3<double> &pm, V3<double> &pp) {
    const double h = 0.5 * q * dt;
    pm = p + h * E;
    const double ig = rsqrt(1.0 + dot(pm, pm));
    const V3<double> tau = (h * ig) * B;
    const V3<double> sig = (2.0 * rcp(1.0 + dot(tau, tau))) * tau;
    const V3<double> pr = pm + cross(pm, tau);
    pp = pm + cross(pr, sig);
    p = pp + h * E;
    return ig;
}
// T-BMT (eq. bmteqn) by the Boris rotation of eqs. bmt-boris1-4: dS/dt = q S x Omega,
// gamma^n = sqrt(1+|p-|^2) (passed as ig = 1/gamma^n), beta^n = (p- + p+)/(2 gamma^n),
// g/2 - 1 = a_e.
template <class T>
__device__ __forceinline__ void bmt(const Consts &c, double q, const V3<double> &E, const V3<double> &B,
                                    const V3<double> &pm, const V3<double> &pp, double ig, V3<T> &S) {
    const double gd = (1.0 + dot(pm, pm)) * ig;
    const V3<T> beta = cvt<T>((0.5 * ig) * (pm + pp));
    const V3<T> Et = cvt<T>(E), Bt = cvt<T>(B);
    // q = +-1, so (T)(q dt/2) = q (T)(dt/2) exactly
    T ae, hqdt;
    if constexpr (sizeof(T) == 4) {
        ae = c.f_a_e;
        hqdt = (float)q * c.f_half_dt;
    } else {
        ae = c.a_e;
        hqdt = 0.5 * q * c.dt;
    }
    const T g = (T)gd, igp = rcp(g + (T)1);
    const T c1 = -ae * g * igp * dot(beta, Bt), c2 = ae + (T)ig, c3 = ae + igp;
    const V3<T> om = c1 * beta + c2 * Bt - c3 * cross(beta, Et);
    const V3<T> tv = hqdt * om;
    const V3<T> o = ((T)2 * rcp((T)1 + dot(tv, tv))) * tv;
    const V3<T> Sp = S + cross(S, tv);
    S = S + cross(Sp, o);
}
// chi_e = xi_L sqrt((gamma E + p x B)^2 - (p.E)^2)
// (the square root in the precision T of the rates it feeds)
// from v = gamma E + p x B and p.E
template <class T>
__device__ __forceinline__ double chi_of(double xi_L, const V3<double> &v, double pe) {
    const double s = dot(v, v) - pe * pe;
    if constexpr (sizeof(T) == 4) return xi_L * (double)__builtin_amdgcn_sqrtf(s > 0.0 ? (float)s : 0.0f);
    return xi_L * sqrt(s > 0.0 ? s : 0.0);
}

// ------------------------------------------------------------------------- table lookups
template <class T>
__device__ __forceinline__ int lag4(T pos, int n, T w[4]) {
    pos = pos < (T)0 ? (T)0 : pos;
    pos = pos > (T)(n - 1) ? (T)(n - 1) : pos;
    int i = (int)floor(pos);
    i = i < 1 ? 1 : (i > n - 3 ? n - 3 : i);
    const T f = pos - (T)i, fm1 = f - (T)1, fm2 = f - (T)2, fp1 = f + (T)1;
    w[0] = -f * fm1 * fm2 * (T)(1.0 / 6.0);
    w[1] = fp1 * fm1 * fm2 * (T)0.5;
    w[2] = -fp1 * f * fm2 * (T)0.5;
    w[3] = fp1 * f * fm1 * (T)(1.0 / 6.0);
    return i;
}
template <class T>
__device__ __forceinline__ T gridpos(T l, double lo, double hi, int n) {
    return (l - (T)lo) * (T)((n - 1) / (hi - lo));
}

// Bessel trio at x, all three multiplied by x^(2/3) e^x (only ratios are used)
template <class T>
__device__ __forceinline__ void bessel_scaled(const Tabs<T> &tb, T x, T &I, T &K1, T &K2) {
    T w[4];
    const int i = lag4(gridpos<T>(log(x), B_LO, B_HI, NB), NB, w);
    const T *b = tb.bes() + 4 * (i - 1);
    T b1 = 0, b2 = 0, b3 = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        b1 += w[k] * b[4 * k];
        b2 += w[k] * b[4 * k + 1];
        b3 += w[k] * b[4 * k + 2];
    }
    const T x13 = cbrt(x);
    I = b3 * x13 * x13;
    K1 = b1 * x13;
    K2 = b2;
}

// r: the NCS rate table (global memory, or a copy staged in LDS)
template <class T>
__device__ __forceinline__ void ncs_rate(const T *r, double chi, T &Ia, T &Ib, uint32_t &st) {
    if (!(chi > 0.0)) {
        Ia = 0;
        Ib = 0;
        return;
    }
    const T c = (T)chi, l = lnx(c);
    if (l < (T)R_LO) {
        Ia = r[0] * c;
        Ib = r[1] * (c / (T)1e-6) * Ia;
        return;
    }
    if (l > (T)R_HI) st |= QED_ST_CLAMP;
    T w[4];
    const int i = lag4(gridpos<T>(l, R_LO, R_HI, NR), NR, w);
    T fa = 0, fk = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        fa += w[k] * r[2 * (i - 1 + k)];
        fk += w[k] * r[2 * (i - 1 + k) + 1];
    }
    Ia = fa * c;
    Ib = fk * Ia;
}

// Inverse of the piecewise-linear CDF D_j = a_j - m b_j, rows r0 and r0+1 mixed with
// weight f, at `target`; returns the fractional column.  Bisection keeps D(lo) <= target <
// D(hi) (D is non-decreasing), so the bracket [lo, lo + 1] is the last column with
// D <= target and its successor, and the values of D at its ends come from the probes.
// Bisection (10 probes for 1024 columns) measured faster here than wider searches with
// fewer dependent rounds (an 8-way search: 22 probes in 4 rounds): the event pass is
// limited by the number of scattered probes more than by their latency.
// The two rows are read through an accessor: CdfRows (rows r0 and r0+1 of a [row][col][2]
// table: two 8-byte loads per probe) or CdfPairs (the FP32 paired copy: one 16-byte load).
// Both hand the same four values to the same arithmetic.
template <class T>
struct CdfRows {
    const T *__restrict__ R0, *__restrict__ R1;
    __device__ __forceinline__ void at(int j, T &a0, T &b0, T &a1, T &b1) const {
        a0 = R0[2 * j];
        b0 = R0[2 * j + 1];
        a1 = R1[2 * j];
        b1 = R1[2 * j + 1];
    }
};
struct CdfPairs {
    const float4 *__restrict__ P;
    __device__ __forceinline__ void at(int j, float &a0, float &b0, float &a1, float &b1) const {
        const float4 v = P[j];
        a0 = v.x;
        b0 = v.y;
        a1 = v.z;
        b1 = v.w;
    }
};
template <class T, class Rows>
__device__ __forceinline__ T cdf_at(const Rows &R, int j, T g, T f, T m) {
    T a0, b0, a1, b1;
    R.at(j, a0, b0, a1, b1);
    const T a = g * a0 + f * a1;
    const T b = g * b0 + f * b1;
    return a - m * b;
}
template <class T, class Rows>
__device__ __forceinline__ T cdf_invert(const Rows &R, int ncol, T f, T m, T target) {
    int lo = 0, hi = ncol - 1;
    const T g = (T)1 - f;
    T dlo = cdf_at<T>(R, lo, g, f, m), dhi = cdf_at<T>(R, hi, g, f, m);
    while (hi - lo > 1) {
        const int mid = lo + (hi - lo) / 2;
        const T d = cdf_at<T>(R, mid, g, f, m);
        if (d <= target) {
            lo = mid;
            dlo = d;
        } else {
            hi = mid;
            dhi = d;
        }
    }
    T tau = dhi > dlo ? (target - dlo) / (dhi - dlo) : (T)0;
    tau = tau < (T)0 ? (T)0 : (tau > (T)1 ? (T)1 : tau);
    return (T)lo + tau;
}
// The same inversion by a K-ary search: each round reads K - 1 columns inside (lo, hi) at
// once and keeps the interval before the first of them above the target, so a row of 512
// columns takes three rounds of memory latency instead of nine.  On a non-decreasing row it
// brackets the same pair of columns as the bisection (the last column at or below the
// target, capped at ncol - 2); for the rare events, where the latency of one lane's
// dependent reads is the kernel's time.
template <class T, int K, class Rows>
__device__ __forceinline__ T cdf_invert_wide(const Rows &R, int ncol, T f, T m, T target) {
    int lo = 0, hi = ncol - 1;
    const T g = (T)1 - f;
    T dlo, dhi;
    // one round of K - 1 columns inside (lo, hi): the interval before the first one above
    // the target
    auto round = [&](T lo_v, T hi_v, bool first) {
        int p[K - 1];
        T d[K - 1];
#pragma unroll
        for (int q = 0; q < K - 1; ++q) {
            p[q] = lo + 1 + ((hi - lo - 1) * (q + 1)) / K;   // in [lo + 1, hi - 1]
            d[q] = cdf_at<T>(R, p[q], g, f, m);
        }
        if (first) {   // the ends, read together with the first round's columns
            lo_v = cdf_at<T>(R, lo, g, f, m);
            hi_v = cdf_at<T>(R, hi, g, f, m);
        }
        int nlo = lo, nhi = hi;
        T vlo = lo_v, vhi = hi_v;
        bool above = false;
#pragma unroll
        for (int q = 0; q < K - 1; ++q) {
            if (!above && d[q] > target) {
                above = true;
                nhi = p[q];
                vhi = d[q];
            } else if (!above) {
                nlo = p[q];
                vlo = d[q];
            }
        }
        lo = nlo;
        hi = nhi;
        dlo = vlo;
        dhi = vhi;
    };
    if (hi - lo > 1) {
        round((T)0, (T)0, true);
    } else {
        dlo = cdf_at<T>(R, lo, g, f, m);
        dhi = cdf_at<T>(R, hi, g, f, m);
    }
    while (hi - lo > 1) round(dlo, dhi, false);
    T tau = dhi > dlo ? (target - dlo) / (dhi - dlo) : (T)0;
    tau = tau < (T)0 ? (T)0 : (tau > (T)1 ? (T)1 : tau);
    return (T)lo + tau;
}
template <class T>
__device__ __forceinline__ void row_pos(T l, double lo, double hi, int n, int &r0, T &f) {
    T q = gridpos<T>(l, lo, hi, n);
    q = q < (T)0 ? (T)0 : (q > (T)(n - 1) ? (T)(n - 1) : q);
    int r = (int)floor(q);
    r = r > n - 2 ? n - 2 : (r < 0 ? 0 : r);
    r0 = r;
    f = q - (T)r;
}
// photon-fraction variable t = (2u/(3chi))^(1/3) sampled from the spin-dependent spectrum
template <class T>
__device__ __forceinline__ T ncs_sample_t(const Tabs<T> &tb, double chi, T kappa, T s, T r) {
    const T m = s * kappa;
    int r0;
    T f;
    row_pos<T>(log((T)chi), C_LO, C_HI, NCR, r0, f);
    T col;
    if constexpr (sizeof(T) == 4) {
        col = cdf_invert<T>(CdfPairs{tb.ncs_cdf_pair() + (int64_t)r0 * NCT}, NCT, f, m, r * ((T)1 - m));
    } else {
        const T *R0 = tb.ncs_cdf() + (int64_t)r0 * NCT * 2;
        col = cdf_invert<T>(CdfRows<T>{R0, R0 + 2 * NCT}, NCT, f, m, r * ((T)1 - m));
    }
    return col * (T)(T_MAX / (NCT - 1));
}

// tb: any table source with nbw_rate() (the global tables, or a copy of that table in LDS)
template <class T, class TB>
__device__ __forceinline__ void nbw_rate(const TB &tb, double chi, T &Ja, T &Jb, T &kappa, uint32_t &st) {
    const T c = (T)chi, l = chi > 0.0 ? log(c) : (T)-1e30;
    if (l < (T)P_LO) {
        Ja = 0;
        Jb = 0;
        kappa = 0;
        return;
    }
    if (l > (T)P_HI) st |= QED_ST_CLAMP;
    T w[4];
    const int i = lag4(gridpos<T>(l, P_LO, P_HI, NP), NP, w);
    const T *r = tb.nbw_rate();
    T ga = 0, gk = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        ga += w[k] * r[2 * (i - 1 + k)];
        gk += w[k] * r[2 * (i - 1 + k) + 1];
    }
    Ja = ga * c * exp((T)(-8.0 / 3.0) / c);
    Jb = gk * Ja;
    kappa = gk;
}
template <class T>
__device__ __forceinline__ T nbw_sample_delta(const Tabs<T> &tb, double chi, T kappa, T xi3, T r) {
    const T m = xi3 * kappa;
    int r0;
    T f;
    row_pos<T>(log((T)chi), P_LO, P_HI, NDR, r0, f);
    const T hd = (T)(0.5 / (NDD - 1));
    const bool lower = r <= (T)0.5;
    const T target = (lower ? r : (T)1 - r) * ((T)1 - m);
    T col;
    if constexpr (sizeof(T) == 4) {
        col = cdf_invert_wide<T, 8>(CdfPairs{tb.nbw_cdf_pair() + (int64_t)r0 * NDD}, NDD, f, m, target);
    } else {
        const T *R0 = tb.nbw_cdf() + (int64_t)r0 * NDD * 2;
        col = cdf_invert_wide<T, 8>(CdfRows<T>{R0, R0 + 2 * NDD}, NDD, f, m, target);
    }
    return lower ? col * hd : (T)1 - col * hd;
}
// tb: any table source with vb()
template <class T, class TB>
__device__ __forceinline__ void vb_M(const TB &tb, double chi, T &Mp, T &Mm, uint32_t &st) {
    const T c = (T)chi, l = chi > 0.0 ? log(c) : (T)-1e30;
    if (l < (T)V_LO) {
        Mp = 4;
        Mm = 7;
        return;
    }
    if (l > (T)V_HI) st |= QED_ST_CLAMP;
    T w[4];
    const int i = lag4(gridpos<T>(l, V_LO, V_HI, NV), NV, w);
    const T *v = tb.vb();
    Mp = 0;
    Mm = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        Mp += w[k] * v[2 * (i - 1 + k)];
        Mm += w[k] * v[2 * (i - 1 + k) + 1];
    }
}

// Radiation-reaction coefficients {g, psi1, psi2, psi3} at chi from the RAD table (stored
// as g (1+chi)^(4/3) and psi (1+chi)^(7/3)/chi^3; below the grid g = 1 - (55 sqrt3/16) chi
// and the psi scale from the first node; above: clamp + flag).
template <class T>
struct RadCoef {
    T g, p1, p2, p3;
};
template <class T>
__device__ __forceinline__ RadCoef<T> rad_coeffs(const Tabs<T> &tb, double chi, uint32_t &st) {
    if (!(chi > 0.0)) return {(T)1, (T)0, (T)0, (T)0};
    const T c = (T)chi, l = lnx(c), o = (T)1 + c, oc = cbrt(o), sp = c * c * c / (o * o * oc);
    const T *r = tb.rad();
    if (l < (T)R_LO) return {(T)1 - (T)(55.0 * 1.7320508075688772 / 16.0) * c, r[1] * sp, r[2] * sp, r[3] * sp};
    if (l > (T)R_HI) st |= QED_ST_CLAMP;
    T w[4];
    const int i = lag4(gridpos<T>(l, R_LO, R_HI, NR), NR, w);
    T h0 = 0, h1 = 0, h2 = 0, h3 = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const T *q = r + 4 * (i - 1 + j);
        h0 += w[j] * q[0];
        h1 += w[j] * q[1];
        h2 += w[j] * q[2];
        h3 += w[j] * q[3];
    }
    return {h0 / (o * oc), h1 * sp, h2 * sp, h3 * sp};
}

// ------------------------------------------------------------------------- NCS
// Emitted photon of one event (Sec. III.C.1): momentum k, Stokes xi, basis vector e1.
template <class T>
struct NcsPhoton {
    V3<double> k;
    V3<T> xi, e1;
};

// The F functions of eqs. (F0)-(F3) (Bessel values share a common positive factor).
template <class T>
__device__ __forceinline__ void ncs_F(T u, T I, T K1, T K2, const V3<T> &Si, const V3<T> &Sf, const V3<T> &a,
                                      const V3<T> &b, const V3<T> &n, T F[4]) {
    const T Sif = dot(Si, Sf), sia = dot(Si, a), sfa = dot(Sf, a), sib = dot(Si, b), sfb = dot(Sf, b);
    const T sin_ = dot(Si, n), sfn = dot(Sf, n);
    const V3<T> fxs = cross(Sf, Si);
    const T nfx = dot(n, fxs), afx = dot(a, fxs), u2 = u * u;
    F[0] = -(2 + u) * (2 + u) * (I - 2 * K2) * (1 + Sif) + u2 * (1 - Sif) * (I + 2 * K2) + 2 * u2 * Sif * I -
           (4 * u + 2 * u2) * (sfb + sib) * K1 - 2 * u2 * (sfb - sib) * K1 - 4 * u2 * (I - K2) * sin_ * sfn;
    F[1] = -2 * u2 * I * (sia * sfb + sfa * sib) + 4 * u * (sia * (1 + u) + sfa) * K1 + 2 * u * (2 + u) * nfx * K2;
    F[2] = -(2 * u2 * (sin_ * sfb + sfn * sib) + 2 * u * (2 + u) * afx) * K1 - 4 * u * (sin_ + sfn * (1 + u)) * I +
           4 * u * (2 + u) * (sin_ + sfn) * K2;
    F[3] = 4 * (1 + u + (1 + u + (T)0.5 * u2) * Sif - (T)0.5 * u2 * sin_ * sfn) * K2 +
           2 * u2 * (sib * sfb - sia * sfa) * I - 4 * u * ((1 + u) * sib + sfb) * K1;
}

// Local frame and rates of one lepton with p = p^{n+1/2}, S = S^{n+1/2} and the fields of
// x^n (Sec. III.C.1): n = p/|p|, a = unit transverse part of q(E + beta x B - beta(beta.E)),
// b = n x a, s = S.b, W = C Ia, W_tot = C (Ia - s Ib), C = alpha/(sqrt3 pi xi_L gamma).
// Returns false where chi = 0 or the acceleration vanishes (nothing happens then).
// Both chi and a come from v = gamma E + p x B: chi = xi_L sqrt(|v|^2 - (p.E)^2), and as
// beta is parallel to n, the part of E + beta x B - beta(beta.E) transverse to n is the
// transverse part of v divided by gamma.
template <class T>
struct NcsFrame {
    double chi, C, W, Wt, P;
    V3<T> n, a, b;
    T s, Ia, Ib;
};
// ig = 1/gamma = 1/sqrt(1 + |p|^2), computed by the caller; rate = the NCS rate table.
template <class T>
__device__ __forceinline__ bool ncs_frame(const Consts &c, const T *rate, double q, const V3<double> &p,
                                          double ig, const V3<T> &S, const V3<double> &E, const V3<double> &B,
                                          uint32_t &st, NcsFrame<T> &f) {
    const double pp2 = dot(p, p), g = (1.0 + pp2) * ig;
    const V3<double> v = g * E + cross(p, B);
    f.chi = chi_of<T>(c.xi_L, v, dot(p, E));
    if (!(f.chi > 0.0) || !(pp2 > 0.0)) return false;
    const V3<double> nd = rsqrt(pp2) * p;
    const V3<double> ad = v - dot(nd, v) * nd;
    const double a2 = dot(ad, ad);
    if (!(a2 > 0.0)) return false;
    f.n = cvt<T>(nd);
    f.a = cvt<T>((q * rsqrt(a2)) * ad);
    f.b = cross(f.n, f.a);
    f.s = dot(S, f.b);
    ncs_rate<T>(rate, f.chi, f.Ia, f.Ib, st);
    f.C = c.c_ncs * ig;
    f.W = f.C * (double)f.Ia;
    f.Wt = f.C * ((double)f.Ia - (double)f.s * (double)f.Ib);
    f.P = f.Wt * c.dt;
    if (f.P > c.p_max) st |= QED_ST_PMAX;
    return true;
}
// no emission: S -> [S(1 - W dt) - f dt]/(1 - W_tot dt), renormalised (f = -C Ib b)
template <class T>
__device__ __forceinline__ void ncs_no_event(const Consts &c, const NcsFrame<T> &f, V3<T> &S) {
    // called only when no emission happened, so 1 - W~ dt > 0 and the common factor
    // 1/(1 - W~ dt) drops out of the normalised spin
    const T wdt = (T)(f.W * c.dt), fb = (T)(f.C * (double)f.Ib * c.dt);
    const V3<T> Sb = ((T)1 - wdt) * S + fb * f.b;
    S = rsq(dot(Sb, Sb)) * Sb;
}
// emission (given the draws r): photon fraction y by the inverse of the spin-dependent
// spectrum (r1), k = y p, p -> (1-y) p; final spin +-g/|g| with P(+) = (1 + |g|/(w+f.S))/2
// (r3); photon pure state +-F/|F| with P(+) = (F0 + |F|)/(2 F0) at the chosen S_f (r4).
// ncs_event_t: the same with the photon-fraction variable tt already drawn (by the table
// inverse CDF with r1, or by the learned sampler).
template <class T>
__device__ __forceinline__ void ncs_event_t(const Consts &c, const Tabs<T> &tb, const NcsFrame<T> &f, T tt,
                                            const double r[4], V3<double> &p, V3<T> &S, NcsPhoton<T> &ph) {
    const T t3 = tt * tt * tt;
    const T u = (T)1.5 * (T)f.chi * t3, y = u / ((T)1 + u);
    ph.k = (double)y * p;
    p = (1.0 - (double)y) * p;
    T I, K1, K2;
    bessel_scaled<T>(tb, t3, I, K1, K2);
    const T w = -(1 + u) * I + (2 + 2 * u + u * u) * K2;
    const T fS = -u * K1 * f.s;
    const T sn = dot(S, f.n);
    const V3<T> gv = (-(1 + u) * (I - 2 * K2)) * S + (-u * (1 + u) * K1) * f.b + (-u * u * (I - K2) * sn) * f.n;
    const T gn = sqrt(dot(gv, gv));
    const V3<T> zeta = gn > (T)0 ? ((T)1 / gn) * gv : S;
    const T pplus = (T)0.5 * ((T)1 + gn / (w + fS));
    const V3<T> Sf = (r[2] < (double)pplus ? (T)1 : (T)-1) * zeta;
    V3<T> xi = {0, 0, 0};
    if (c.procs & QED_PROC_NCS_STOKES) {
        T F[4];
        ncs_F<T>(u, I, K1, K2, S, Sf, f.a, f.b, f.n, F);
        const T fn = sqrt(F[1] * F[1] + F[2] * F[2] + F[3] * F[3]);
        if (fn > (T)0) {
            const T sx = r[3] < (double)((F[0] + fn) / ((T)2 * F[0])) ? (T)1 : (T)-1;
            xi = {sx * F[1] / fn, sx * F[2] / fn, sx * F[3] / fn};
        } else {
            xi.z = r[3] < 0.5 ? (T)1 : (T)-1;
        }
    }
    S = Sf;
    ph.xi = xi;
    ph.e1 = f.a;
}
template <class T>
__device__ __forceinline__ void ncs_event(const Consts &c, const Tabs<T> &tb, const NcsFrame<T> &f, const double r[4],
                                          V3<double> &p, V3<T> &S, NcsPhoton<T> &ph) {
    ncs_event_t<T>(c, tb, f, ncs_sample_t<T>(tb, f.chi, f.Ib / f.Ia, f.s, (T)r[0]), r, p, S, ph);
}

// ------------------------------------------------------------------------- photons
// The G functions of eqs. (G0)-(G3) without W0/2 (a, b, v = a_+, b_+, v_+).
template <class T>
__device__ __forceinline__ T nbw_weight(T d, T I, T K1, T K2, const V3<T> &Sp, const V3<T> &Sm, const V3<T> &a,
                                        const V3<T> &b, const V3<T> &v, const V3<T> &xi) {
    const T ep = d, em = (T)1 - d;
    const T rs = (em * em + ep * ep) / (em * ep), ds = (ep * ep - em * em) / (em * ep),
            sq = (ep - em) * (ep - em) / (em * ep);
    const T gp = (T)1 / ep, gm = (T)1 / em, g2 = (T)1 / ((T)2 * em * ep);
    const T spm = dot(Sm, Sp), spa = dot(Sp, a), sma = dot(Sm, a), spb = dot(Sp, b), smb = dot(Sm, b);
    const T spv = dot(Sp, v), smv = dot(Sm, v);
    const V3<T> mxp = cross(Sm, Sp);
    const T mv = dot(mxp, v), ma = dot(mxp, a);
    const T G0 = I + rs * K2 + (I - 2 * K2) * spm + K1 * (-gp * spb + gm * smb) + (rs * I - sq * K2) * spv * smv;
    const T G1 = K1 * (-gm * spa + gp * sma) + (T)0.5 * ds * K2 * mv - g2 * I * (spa * smb + sma * spb);
    const T G2 = g2 * K1 * ma + (T)0.5 * ds * K1 * (smv * spb + spv * smb) + (gm * I - ds * K2) * smv +
                 (gp * I + ds * K2) * spv;
    const T G3 = -K2 + (T)0.5 * rs * K2 * spm - K1 * (gp * smb - gm * spb) + g2 * I * (spb * smb - spa * sma) -
                 (T)0.5 * sq * K2 * spv * smv;
    const T wv = G0 + xi.x * G1 + xi.y * G2 + xi.z * G3;
    return wv > (T)0 ? wv : (T)0;
}

template <class T>
struct PairOut {
    V3<double> pm, pp;   // electron, positron momenta
    V3<T> Sm, Sp;        // spins
};

// A photon's direction, reduced transverse field and chi_gamma: n = k/|k|, E_red =
// E - n(n.E) + n x B, chi = xi_L eps |E_red| (eps = |k|).  The reciprocal lengths come
// from one reciprocal square root each (no square root, no division).
struct PhotonFrame {
    double eps, inv_eps, an, inv_an, chi;
    V3<double> n, er;
};
__device__ __forceinline__ void photon_frame(double xi_L, const V3<double> &k, const V3<double> &E,
                                             const V3<double> &B, PhotonFrame &f) {
    const double kk = dot(k, k);
    f.inv_eps = rsqrt(kk);
    f.eps = kk * f.inv_eps;
    f.n = f.inv_eps * k;
    f.er = E - dot(f.n, E) * f.n + cross(f.n, B);
    const double a2 = dot(f.er, f.er);
    f.inv_an = a2 > 0.0 ? rsqrt(a2) : 0.0;
    f.an = a2 * f.inv_an;
    f.chi = xi_L * f.eps * f.an;
}
// sin and cos of a small angle |d| < 0.02 by their Taylor series (the first omitted term
// is below 1e-19 of the result there), of a larger one by the library
template <class T>
__device__ __forceinline__ void sincos_small(T d, T &sd, T &cd) {
    if (fabs(d) < (T)0.02) {
        const T d2 = d * d;
        sd = d * ((T)1 - d2 * ((T)(1.0 / 6.0) - d2 * ((T)(1.0 / 120.0) - d2 * (T)(1.0 / 5040.0))));
        cd = (T)1 - d2 * ((T)0.5 - d2 * ((T)(1.0 / 24.0) - d2 * ((T)(1.0 / 720.0) - d2 * (T)(1.0 / 40320.0))));
    } else if constexpr (sizeof(T) == 8) {
        sincos(d, &sd, &cd);
    } else {
        sincosf(d, &sd, &cd);
    }
}

// Photon transport at x^n (Algorithm 1): basis rotation of the Stokes vector to the frame
// of E_red (eq. rotation) and, if do_vb, the birefringent phase (eq. rotation2), whose
// chi^2 / (eps xi_L) is written chi |E_red|.  Returns chi_gamma (0 where E_red vanishes:
// nothing changes then).
template <class T, class TB>
__device__ __forceinline__ double photon_transport(const Consts &c, const TB &tb, const PhotonFrame &f, V3<T> &xi,
                                                   V3<T> &e1, bool do_vb, uint32_t &st) {
    if (!(f.an > 0.0)) return 0.0;
    const double chi = f.chi;
    const V3<T> nt = cvt<T>(f.n);
    const V3<T> e1n = cvt<T>(f.inv_an * f.er);
    const V3<T> e2 = cross(nt, e1);
    const T cp = dot(e1, e1n), sp = dot(e2, e1n), inn = rcp(cp * cp + sp * sp);
    const T c2 = (cp * cp - sp * sp) * inn, s2 = (T)2 * cp * sp * inn;
    {
        const T x1 = c2 * xi.x - s2 * xi.z, x3 = s2 * xi.x + c2 * xi.z;
        xi.x = x1;
        xi.z = x3;
    }
    e1 = e1n;
    if (do_vb) {
        T Mp, Mm;
        vb_M<T>(tb, chi, Mp, Mm, st);
        constexpr double VB = 1.0 / (90.0 * PI);
        const T dphi = (T)((double)(Mp - Mm) * (c.alpha * VB) * chi * f.an * c.dt);
        T sd, cd;
        sincos_small<T>(dphi, sd, cd);
        const T y1 = cd * xi.x - sd * xi.y, y2 = sd * xi.x + cd * xi.y;
        xi.x = y1;
        xi.y = y2;
    }
    return chi;
}
// NBW event probability W_pair dt (eq. BWprob with the rate normalisation of the readings)
template <class T, class TB>
__device__ __forceinline__ double nbw_prob(const Consts &c, const TB &tb, double eps, double chi, T xi3, T &Ja,
                                           T &kappa, uint32_t &st) {
    T Jb;
    nbw_rate<T>(tb, chi, Ja, Jb, kappa, st);
    const double P = c.alpha / (SQRT3 * PI * c.xi_L * eps) * ((double)Ja - (double)xi3 * (double)Jb) * c.dt;
    if (P > c.p_max) st |= QED_ST_PMAX;
    return P;
}
// pair creation (given the draws r, the rotated xi and basis e1): delta by the inverse
// spectrum (r1), SQAs D/|D|, D'/|D'| (eqs. BWposAxis, BWeleAxis), spin pair picked by r3
// from the weights of eqs. G0-G3 in the order (+,+),(+,-),(-,+),(-,-).
// nbw_pair_d: the same with delta already drawn (by the table inverse CDF with r1, or by
// the learned sampler).
template <class T>
__device__ __forceinline__ void nbw_pair_d(const Tabs<T> &tb, const V3<double> &k, double chi, T d, const V3<T> &xi,
                                           const V3<T> &e1, const double r[4], uint32_t &st, PairOut<T> &po) {
    const double eps = sqrt(dot(k, k));
    const V3<double> n = (1.0 / eps) * k;
    const V3<T> nt = cvt<T>(n);
    const double epl = (double)d * eps, emi = eps - epl;
    T I, K1, K2;
    bessel_scaled<T>(tb, (T)(2.0 / (3.0 * chi * (double)d * (1.0 - (double)d))), I, K1, K2);
    const V3<T> a = e1, bb = cross(nt, a);
    const T ip = (T)(eps / epl), im = (T)(eps / emi), ds = (T)((epl * epl - emi * emi) / (emi * epl));
    const V3<T> D = (-(ip - xi.z * im) * K1) * bb + (-xi.x * im * K1) * a + (xi.y * (ds * K2 + ip * I)) * nt;
    const V3<T> Dm = ((im - xi.z * ip) * K1) * bb + (xi.x * ip * K1) * a + (-xi.y * (ds * K2 - im * I)) * nt;
    const T dn = sqrt(dot(D, D)), dmn = sqrt(dot(Dm, Dm));
    const V3<T> zp = dn > (T)0 ? ((T)1 / dn) * D : bb;
    const V3<T> zm = dmn > (T)0 ? ((T)1 / dmn) * Dm : bb;
    T Pk[4], tot = 0;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const T sgp = kk < 2 ? (T)1 : (T)-1, sgm = (kk & 1) == 0 ? (T)1 : (T)-1;
        Pk[kk] = nbw_weight<T>(d, I, K1, K2, sgp * zp, sgm * zm, a, bb, nt, xi);
        tot += Pk[kk];
    }
    int sel = 3;
    T acc = 0;
    const T thr = (T)r[2] * tot;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        acc += Pk[kk];
        if (sel == 3 && kk < 3 && thr < acc) sel = kk;
    }
    if (epl < 1.0 || emi < 1.0) st |= QED_ST_EPS_LT1;
    double qp = epl * epl - 1.0, qm = emi * emi - 1.0;
    qp = qp > 0.0 ? sqrt(qp) : 0.0;
    qm = qm > 0.0 ? sqrt(qm) : 0.0;
    po.pp = qp * n;
    po.pm = qm * n;
    po.Sp = (sel < 2 ? (T)1 : (T)-1) * zp;
    po.Sm = ((sel & 1) == 0 ? (T)1 : (T)-1) * zm;
}
template <class T>
__device__ __forceinline__ void nbw_pair(const Tabs<T> &tb, const V3<double> &k, double chi, T kappa, const V3<T> &xi,
                                         const V3<T> &e1, const double r[4], uint32_t &st, PairOut<T> &po) {
    nbw_pair_d<T>(tb, k, chi, nbw_sample_delta<T>(tb, chi, kappa, xi.z, (T)r[0]), xi, e1, r, st, po);
}

// ------------------------------------------------------------------------- list access, ranks
// step number of a launch: the argument plus the optional device counter
template <class A>
__device__ __forceinline__ int64_t step_of(const A &a) {
    return a.step + (a.step_dev ? *a.step_dev : 0);
}

// element of an array at a 32-bit byte offset
template <class T>
__device__ __forceinline__ T &at(T *base, uint32_t off) {
    return *(T *)((char *)base + off);
}
// streaming access to the particle arrays (read once, written once per step): the
// non-temporal hint on both the loads and the stores keeps the stream from displacing the
// tables and the staging records in the caches; together (not either alone) they make the
// decide kernel about 20 % faster at 1e7 leptons
template <class T>
__device__ __forceinline__ T ld_nt(T *base, uint32_t off) {
    return __builtin_nontemporal_load(&at(base, off));
}
template <class T>
__device__ __forceinline__ void st_nt(T *base, uint32_t off, T v) {
    __builtin_nontemporal_store(v, &at(base, off));
}

// device list counts are trusted only up to the list capacity
__device__ __forceinline__ int64_t clamp_count(const int64_t *count, int64_t capacity) {
    const int64_t n = *count;
    return n < 0 ? 0 : (n > capacity ? capacity : n);
}

// Block-wide exclusive rank of a 0/1 flag: wave ballot + popcount, waves combined in LDS.
__device__ __forceinline__ int block_rank(bool flag, int &total, int *s_wave) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const unsigned long long m = __ballot(flag);
    const int below = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) s_wave[wid] = __popcll(m);
    __syncthreads();
    int pre = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) {
        const int v = s_wave[w];
        pre += w < wid ? v : 0;
        total += v;
    }
    return pre + below;
}

__device__ __forceinline__ void stage(EventRec *stg, int64_t slot, int64_t idx, const V3<double> &E,
                                      const V3<double> &B) {
    EventRec &r = stg[slot];
    r.idx = idx;
    r.f[0] = E.x; r.f[1] = E.y; r.f[2] = E.z;
    r.f[3] = B.x; r.f[4] = B.y; r.f[5] = B.z;
}

// photon events: the photon index of the event of rank r (bytes [0, 8) of staging slot r)
// and the record of photon j's event (bytes [8, ...) of slot j)
__device__ __forceinline__ int64_t *event_index(void *stg, int64_t r) {
    return (int64_t *)((char *)stg + r * (int64_t)STAGING_SLOT);
}
template <class T>
__device__ __forceinline__ PhotonEvent<T> *photon_event(void *stg, int64_t j) {
    return (PhotonEvent<T> *)((char *)stg + j * (int64_t)STAGING_SLOT + 8);
}

// tile whose event range [off[t], off[t+1]) holds global event e (last t with off[t] <= e)
__device__ __forceinline__ int64_t tile_of(const int64_t *off, int64_t ntiles, int64_t e) {
    int64_t lo = 0, hi = ntiles - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}


// The events of one group of G consecutive tiles, handled by one wavefront (call it with all
// 64 lanes active and a wavefront-uniform first tile t0 < ntiles): the lanes' running sum of
// the G tile counts gives each event its tile (no per-event search); f(e, slot) is called
// for every event, e its global rank (e0, the rank of the group's first event, + rank in
// the group), slot its staging slot tile * BLOCK + rank in the tile.  Suits sparse events
// (a few per tile).
template <int G, class F>
__device__ __forceinline__ void group_events(const int *counts, int64_t e0, int64_t ntiles, int64_t t0, F &&f) {
    static_assert(G <= 64, "one count per lane");
    const int lane = threadIdx.x & 63;
    const int cnt = lane < G && t0 + lane < ntiles ? counts[t0 + lane] : 0;
    int incl = cnt;
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
        const int v = __shfl_up(incl, d);
        if (lane >= d) incl += v;
    }
    const int excl = incl - cnt;
    int exs[G];   // every tile's first rank, in scalar registers (read while all lanes are active)
#pragma unroll
    for (int k = 0; k < G; ++k) exs[k] = __builtin_amdgcn_readlane(excl, k);
    const int total = __builtin_amdgcn_readlane(incl, G - 1);
    for (int le = lane; le < total; le += 64) {
        // the last tile whose first rank is at or before the event (a tile without events
        // shares its first rank with the next, so this is never an empty tile)
        int kk = 0, ek = 0;
#pragma unroll
        for (int k = 0; k < G; ++k)
            if (exs[k] <= le) {
                kk = k;
                ek = exs[k];
            }
        f(e0 + le, (t0 + kk) * BLOCK + (le - ek));
    }
}

}  // namespace qed
