/*
 * qed_oracle.c -- plain, slow, FP64 CPU oracle for the spin/polarisation-resolved
 * strong-field QED particle step of Wan et al. (arXiv:2306.11288).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark load this library.  It shares no code with the HIP library.
 *
 * Organisation (each part cites the passage of the paper it follows):
 *   1. Philox4x32-10                    -- published method (Salmon et al., SC'11)
 *   2. K_nu, IntK_nu, Scorer Gi'        -- integral representations, plain quadrature
 *   3. direct quadrature of the rates   -- Sec. III.C (NCS), III.D (NBW), III.F (VB),
 *                                          III.B.2 (radiative T-BMT psi integrals)
 *   4. the table specification          -- grids and interpolation written out in full
 *   5. fields                           -- plane wave / focused pulse / 2D Yee grid + TSC
 *                                          (Sec. II.D-E, the pulse of Fig. "pusher")
 *   6. Boris + T-BMT                    -- eqs. (boris1)-(boris6), (bmteqn), (bmt-boris1-4)
 *   7. NCS Monte-Carlo step             -- Sec. III.C.1 with the readings listed in DESIGN
 *   8. photon step: frame rotation, VB, NBW -- Sec. III.C.2 eq. (rotation), III.F eq.
 *                                          (rotation2) and Algorithm 1, III.D
 * Parity pinned: every part above has CPU tests against closed forms, limits, library
 * routines (scipy / mpmath / rocRAND's Philox) or brute force.
 */
#include "qed_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846
#define SQRT3 1.7320508075688772935

/* ===================================================================== 0. vectors */
static double dot3(const double a[3], const double b[3]) { return a[0]*b[0] + a[1]*b[1] + a[2]*b[2]; }
static void cross3(const double a[3], const double b[3], double c[3]) {
    double t0 = a[1]*b[2] - a[2]*b[1], t1 = a[2]*b[0] - a[0]*b[2], t2 = a[0]*b[1] - a[1]*b[0];
    c[0] = t0; c[1] = t1; c[2] = t2;
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

/* ===================================================================== 1. Philox */
/* Philox4x32-10: ten rounds of the S-box (two 32x32->64 multiplies) with a Weyl key
 * schedule between rounds, as published by Salmon, Moraes, Dror and Shaw (SC'11).   */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0], n1 = lo1, n2 = hi0 ^ c[3] ^ k[1], n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k[0] += 0x9E3779B9u; k[1] += 0xBB67AE85u; }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof c);
}
/* Counter = (step low word, step bits 32..47 | stream << 16, seed low, seed high);
 * key = particle id.  Uniform = (u + 1/2) 2^-32, strictly inside (0,1).            */
void orc_uniform4(uint64_t id, int64_t step, uint32_t stream, uint64_t seed, double r[4]) {
    uint64_t s = (uint64_t)step;
    uint32_t ctr[4] = {(uint32_t)s, (uint32_t)((s >> 32) & 0xFFFFu) | (stream << 16),
                       (uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t key[2] = {(uint32_t)id, (uint32_t)(id >> 32)};
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    for (int i = 0; i < 4; ++i) r[i] = ((double)o[i] + 0.5) * (1.0 / 4294967296.0);
}

/* ============================================== 2. special functions by quadrature */
/* K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt; the integral of K_nu from x to
 * infinity is the same integral with an extra 1/cosh t.  The integrand is even and
 * analytic, so the trapezoid rule on [0, T] converges geometrically.                */
static void kquad(double x, double nu, double *k, double *ik) {
    double h = 0.1;
    if (x > 25.0) h = 0.5 / sqrt(x);
    double T = acosh(1.0 + 60.0 / x) + 1.0;
    int n = (int)(T / h) + 1;
    double sk = 0.5 * exp(-x), sik = 0.5 * exp(-x);
    for (int i = 1; i <= n; ++i) {
        double t = i * h, ch = cosh(t);
        double e = exp(-x * ch) * cosh(nu * t);
        sk += e;
        sik += e / ch;
    }
    *k = h * sk;
    *ik = h * sik;
}
double orc_bessel_k(double nu, double x) { double k, ik; kquad(x, nu, &k, &ik); return k; }
double orc_int_bessel_k(double nu, double x) { double k, ik; kquad(x, nu, &k, &ik); return ik; }
/* K_{1/3}(x), K_{2/3}(x), IntK_{1/3}(x) sharing the exponentials */
static void bessel_trio(double x, double *k13, double *k23, double *ik13) {
    double h = 0.1;
    if (x > 25.0) h = 0.5 / sqrt(x);
    double T = acosh(1.0 + 60.0 / x) + 1.0;
    int n = (int)(T / h) + 1;
    double e0 = 0.5 * exp(-x);
    double a = e0, b = e0, c = e0;
    for (int i = 1; i <= n; ++i) {
        double t = i * h, ch = cosh(t);
        double e = exp(-x * ch);
        double c13 = cosh(t / 3.0);
        a += e * c13;
        b += e * cosh(2.0 * t / 3.0);
        c += e * c13 / ch;
    }
    *k13 = h * a; *k23 = h * b; *ik13 = h * c;
}

/* the same trio multiplied by exp(x): the integrand exp(-x (cosh t - 1)) stays finite
 * where exp(x) itself would overflow                                                    */
static void bessel_trio_scaled(double x, double *k13, double *k23, double *ik13) {
    double h = 0.1;
    if (x > 25.0) h = 0.5 / sqrt(x);
    double T = acosh(1.0 + 60.0 / x) + 1.0;
    int n = (int)(T / h) + 1;
    double a = 0.5, b = 0.5, c = 0.5;
    for (int i = 1; i <= n; ++i) {
        double t = i * h, ch = cosh(t), sh = sinh(0.5 * t);
        double e = exp(-2.0 * x * sh * sh);          /* cosh t - 1 = 2 sinh^2(t/2) */
        double c13 = cosh(t / 3.0);
        a += e * c13;
        b += e * cosh(2.0 * t / 3.0);
        c += e * c13 / ch;
    }
    *k13 = h * a; *k23 = h * b; *ik13 = h * c;
}

/* Gauss-Legendre nodes on [-1,1] by Newton iteration on P_n */
#define GLN 10
static double gl_x[GLN], gl_w[GLN];
static int gl_ready = 0;
static void gl_init(void) {
    if (gl_ready) return;
    for (int i = 0; i < GLN; ++i) {
        double z = cos(PI * (i + 0.75) / (GLN + 0.5)), pp = 0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1, p2 = 0;
            for (int j = 1; j <= GLN; ++j) { double p3 = p2; p2 = p1; p1 = ((2.0*j - 1) * z * p2 - (j - 1.0) * p3) / j; }
            pp = GLN * (z * p1 - p2) / (z * z - 1);
            double dz = p1 / pp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        gl_x[i] = z;
        gl_w[i] = 2.0 / ((1 - z * z) * pp * pp);
    }
    gl_ready = 1;
}

/* Scorer's Gi'(x) for x >= 0.  Gi(x) = (1/pi) int_0^inf sin(t^3/3 + x t) dt; turning
 * the contour to t = s exp(i pi/6) gives a non-oscillating, decaying integrand:
 * Gi'(x) = (1/pi) int_0^inf s exp(-s^3/3 - x s/2) sin(sqrt3 x s/2 + 5 pi/6) ds.     */
double orc_scorer_gi_prime(double x) {
    gl_init();
    double S = 6.0;
    if (x > 0 && 80.0 / x < S) S = 80.0 / x;
    int np = 40;
    double hp = S / np, sum = 0;
    for (int p = 0; p < np; ++p) {
        for (int i = 0; i < GLN; ++i) {
            double s = hp * (p + 0.5 * (gl_x[i] + 1));
            sum += gl_w[i] * 0.5 * hp * s * exp(-s * s * s / 3.0 - 0.5 * x * s) *
                   sin(0.5 * SQRT3 * x * s + 5.0 * PI / 6.0);
        }
    }
    return sum / PI;
}

/* ================================================ 3. direct quadrature of the rates */
/* NCS (eq. Wspin2 with the rate per unit normalised time, i.e. W_R carrying 1/gamma):
 *   d2W/du dt = alpha/(sqrt3 pi xi_L gamma) (1+u)^-3 [ w(u) - u K13(u') S.b ],
 *   w(u) = -(1+u) IntK13(u') + (2+2u+u^2) K23(u'),  u' = 2u/(3 chi).
 * The integration variable is t = u'^(1/3), u = (3 chi/2) t^3, du = (9 chi/2) t^2 dt,
 * in which every integrand below is analytic on [0, inf).                           */
#define T_CUT 3.9148676411688634   /* 60^(1/3): exp(-60) tail neglected               */
#define T_PANEL 0.05
static int tq_n = 0;
static double *tq_t, *tq_w, *tq_i, *tq_k1, *tq_k2;
static void tq_init(void) {
    if (tq_n) return;
    gl_init();
    int np = (int)ceil(T_CUT / T_PANEL);
    int n = np * GLN;
    tq_t = malloc(n * sizeof(double)); tq_w = malloc(n * sizeof(double));
    tq_i = malloc(n * sizeof(double)); tq_k1 = malloc(n * sizeof(double)); tq_k2 = malloc(n * sizeof(double));
    for (int p = 0; p < np; ++p)
        for (int i = 0; i < GLN; ++i) {
            int j = p * GLN + i;
            double t = T_PANEL * (p + 0.5 * (gl_x[i] + 1));
            tq_t[j] = t; tq_w[j] = 0.5 * T_PANEL * gl_w[i];
            bessel_trio(t * t * t, &tq_k1[j], &tq_k2[j], &tq_i[j]);
        }
    tq_n = n;
}
/* integrand selector: 0 -> w/(1+u)^3, 1 -> u K13/(1+u)^3, 2 -> u w/(1+u)^4,
 * 3,4,5 -> u^2/(1+u)^3 {K23, IntK13, K13}                                           */
static double ncs_integrand(int which, double chi, double t, double I, double K1, double K2) {
    double u = 1.5 * chi * t * t * t;
    double jac = 4.5 * chi * t * t;
    double opu = 1 + u, opu3 = opu * opu * opu;
    double w = -(1 + u) * I + (2 + 2*u + u*u) * K2;
    switch (which) {
    case 0: return jac * w / opu3;
    case 1: return jac * u * K1 / opu3;
    case 2: return jac * u * w / (opu3 * opu);
    case 3: return jac * u * u * K2 / opu3;
    case 4: return jac * u * u * I / opu3;
    default: return jac * u * u * K1 / opu3;
    }
}
static double ncs_full(int which, double chi) {
    if (chi <= 0) return 0;
    tq_init();
    double s = 0;
    for (int j = 0; j < tq_n; ++j)
        s += tq_w[j] * ncs_integrand(which, chi, tq_t[j], tq_i[j], tq_k1[j], tq_k2[j]);
    return s;
}
/* partial integral over t in [0, tend] */
static double ncs_partial(int which, double chi, double tend) {
    gl_init();
    if (tend <= 0) return 0;
    int np = (int)ceil(tend / T_PANEL);
    double hp = tend / np, s = 0;
    for (int p = 0; p < np; ++p)
        for (int i = 0; i < GLN; ++i) {
            double t = hp * (p + 0.5 * (gl_x[i] + 1)), I, K1, K2;
            bessel_trio(t * t * t, &K1, &K2, &I);
            s += 0.5 * hp * gl_w[i] * ncs_integrand(which, chi, t, I, K1, K2);
        }
    return s;
}
double orc_ncs_Ia(double chi) { return ncs_full(0, chi); }
double orc_ncs_Ib(double chi) { return ncs_full(1, chi); }
static double t_of_y(double chi, double y) {
    if (y >= 1) return T_CUT;
    double u = y / (1 - y);
    double t = cbrt(u / (1.5 * chi));
    return t > T_CUT ? T_CUT : t;
}
double orc_ncs_A(double chi, double y) { return ncs_partial(0, chi, t_of_y(chi, y)); }
double orc_ncs_B(double chi, double y) { return ncs_partial(1, chi, t_of_y(chi, y)); }
/* emitted power / Larmor power (2/3) alpha chi^2 / xi_L (the paper's classical limit
 * of the radiation-reaction force, Sec. III.A.1), i.e. the Gaunt factor q(chi).      */
double orc_ncs_power_ratio(double chi) {
    return 3.0 / (2.0 * SQRT3 * PI * chi * chi) * ncs_full(2, chi);
}
/* psi1 = int u''K23(u'), psi2 = int u''IntK13(u') - psi1, psi3 = int u''K13(u'),
 * u'' = u^2/(1+u)^3 (Sec. III.B.2)                                                   */
void orc_rbmt_psi(double chi, double psi[3]) {
    psi[0] = ncs_full(3, chi);
    psi[1] = ncs_full(4, chi) - psi[0];
    psi[2] = ncs_full(5, chi);
}

/* NBW (eq. BWprob, normalised as the total rate per unit normalised time):
 *   dW/d delta dt = alpha/(sqrt3 pi xi_L eps) [IntK13(rho) + r(delta) K23(rho) - xi3 K23(rho)],
 *   rho = 2/(3 chi delta (1-delta)),  r = (delta^2 + (1-delta)^2)/(delta (1-delta)).  */
static double nbw_integrand(int which, double chi, double d) {
    double dd = d * (1 - d);
    if (dd <= 0) return 0;
    double rho = 2.0 / (3.0 * chi * dd);
    if (rho > 700) return 0;          /* exp(-700) relative to the peak: nothing */
    double K1, K2, I;
    bessel_trio(rho, &K1, &K2, &I);
    if (which == 0) return I + (d * d + (1 - d) * (1 - d)) / dd * K2;
    return K2;
}
/* Gauss-Legendre on [lo, hi] */
static double nbw_gl(int which, double chi, double lo, double hi) {
    double s = 0, h = hi - lo;
    for (int i = 0; i < GLN; ++i) s += gl_w[i] * nbw_integrand(which, chi, lo + 0.5 * h * (gl_x[i] + 1));
    return 0.5 * h * s;
}
/* integral over [0, dend]: panels halving towards delta = 0 below min(dend, 0.01), where
 * at large chi the spectrum switches on within delta ~ 1/chi, then panels <= 0.005      */
static double nbw_partial(int which, double chi, double dend) {
    gl_init();
    if (dend <= 0) return 0;
    if (dend > 0.5) return 2 * nbw_partial(which, chi, 0.5) - nbw_partial(which, chi, 1 - dend);
    double g = dend < 0.01 ? dend : 0.01, s = 0;
    for (int k = 0; k < 48; ++k) s += nbw_gl(which, chi, ldexp(g, -(k + 1)), ldexp(g, -k));
    if (dend > g) {
        int np = (int)ceil((dend - g) / 0.005);
        double hp = (dend - g) / np;
        for (int p = 0; p < np; ++p) s += nbw_gl(which, chi, g + p * hp, g + (p + 1) * hp);
    }
    return s;
}
double orc_nbw_Ja(double chi) { return chi > 0 ? 2 * nbw_partial(0, chi, 0.5) : 0; }
double orc_nbw_Jb(double chi) { return chi > 0 ? 2 * nbw_partial(1, chi, 0.5) : 0; }
double orc_nbw_Ka(double chi, double d) { return nbw_partial(0, chi, d); }
double orc_nbw_Kb(double chi, double d) { return nbw_partial(1, chi, d); }

/* VB (Sec. III.F): M(chi) = -(45/4) int_0^1 dv (1-v^2) {c+(v), c-(v)} pi x^(4/3) Gi'(x^(2/3)),
 * x = 4/((1-v^2) chi), c+ = (1 + v^2/3)/2 (mode along E_red), c- = 1 - v^2/3.         */
void orc_vb_M(double chi, double M[2]) {
    gl_init();
    /* panels [1 - 2^-k, 1 - 2^-(k+1)], graded towards v = 1 where the integrand varies
     * on the scale 1 - v ~ 2/chi                                                     */
    double sp = 0, sm = 0;
    for (int p = 0; p < 48; ++p) {
        double lo = 1 - ldexp(1.0, -p), hi = p == 47 ? 1.0 : 1 - ldexp(1.0, -(p + 1)), hp = hi - lo;
        for (int i = 0; i < GLN; ++i) {
            double v = lo + 0.5 * hp * (gl_x[i] + 1), om = 1 - v * v;
            double x = 4.0 / (om * chi), X = cbrt(x * x);
            double core = PI * X * X * orc_scorer_gi_prime(X);
            double wq = 0.5 * hp * gl_w[i];
            sp += wq * om * 0.5 * (1 + v * v / 3.0) * core;
            sm += wq * om * (1 - v * v / 3.0) * core;
        }
    }
    M[0] = -11.25 * sp;
    M[1] = -11.25 * sm;
}

/* The F functions of eqs. (F0)-(F3).  The caller passes the three Bessel values at
 * u' multiplied by any common positive factor (only ratios are used downstream).    */
static void ncs_F_bessel(double u, double I, double K1, double K2, const double Si[3],
                         const double Sf[3], const double a[3], const double b[3],
                         const double n[3], double F[4]) {
    double Sif = dot3(Si, Sf);
    double sia = dot3(Si, a), sfa = dot3(Sf, a), sib = dot3(Si, b), sfb = dot3(Sf, b);
    double sin_ = dot3(Si, n), sfn = dot3(Sf, n);
    double fxs[3];
    cross3(Sf, Si, fxs);
    double n_fxs = dot3(n, fxs), a_fxs = dot3(a, fxs);
    double u2 = u * u;
    F[0] = -(2 + u) * (2 + u) * (I - 2 * K2) * (1 + Sif) + u2 * (1 - Sif) * (I + 2 * K2)
           + 2 * u2 * Sif * I - (4 * u + 2 * u2) * (sfb + sib) * K1 - 2 * u2 * (sfb - sib) * K1
           - 4 * u2 * (I - K2) * sin_ * sfn;
    F[1] = -2 * u2 * I * (sia * sfb + sfa * sib) + 4 * u * (sia * (1 + u) + sfa) * K1
           + 2 * u * (2 + u) * n_fxs * K2;
    F[2] = -(2 * u2 * (sin_ * sfb + sfn * sib) + 2 * u * (2 + u) * a_fxs) * K1
           - 4 * u * (sin_ + sfn * (1 + u)) * I + 4 * u * (2 + u) * (sin_ + sfn) * K2;
    F[3] = 4 * (1 + u + (1 + u + 0.5 * u2) * Sif - 0.5 * u2 * sin_ * sfn) * K2
           + 2 * u2 * (sib * sfb - sia * sfa) * I - 4 * u * ((1 + u) * sib + sfb) * K1;
}
void orc_ncs_F(double u, double chi, const double Si[3], const double Sf[3], const double a[3],
               const double b[3], const double n[3], double F[4]) {
    double K1, K2, I;
    bessel_trio(2 * u / (3 * chi), &K1, &K2, &I);
    ncs_F_bessel(u, I, K1, K2, Si, Sf, a, b, n, F);
}
/* The G functions of eqs. (G0)-(G3) without the common factor W0/2; a, b, v are
 * a_+, b_+ = v_+ x a_+, v_+ (the reading of the unlabelled a, b in G1 is a_+, b_+).  */
static void nbw_G_bessel(double d, double I, double K1, double K2, const double Sp[3],
                         const double Sm[3], const double a[3], const double b[3],
                         const double v[3], double G[4]) {
    double ep = d, em = 1 - d;                     /* energies in units of eps_gamma */
    double rs = (em * em + ep * ep) / (em * ep);
    double ds = (ep * ep - em * em) / (em * ep);
    double sq = (ep - em) * (ep - em) / (em * ep);
    double gp = 1 / ep, gm = 1 / em, g2 = 1 / (2 * em * ep);
    double spm = dot3(Sm, Sp);
    double spa = dot3(Sp, a), sma = dot3(Sm, a), spb = dot3(Sp, b), smb = dot3(Sm, b);
    double spv = dot3(Sp, v), smv = dot3(Sm, v);
    double mxp[3];
    cross3(Sm, Sp, mxp);
    double mxp_v = dot3(mxp, v), mxp_a = dot3(mxp, a);
    G[0] = I + rs * K2 + (I - 2 * K2) * spm + K1 * (-gp * spb + gm * smb)
           + (rs * I - sq * K2) * spv * smv;
    G[1] = K1 * (-gm * spa + gp * sma) + 0.5 * ds * K2 * mxp_v
           - g2 * I * (spa * smb + sma * spb);
    G[2] = g2 * K1 * mxp_a + 0.5 * ds * K1 * (smv * spb + spv * smb)
           + (gm * I - ds * K2) * smv + (gp * I + ds * K2) * spv;
    G[3] = -K2 + 0.5 * rs * K2 * spm - K1 * (gp * smb - gm * spb)
           + g2 * I * (spb * smb - spa * sma) - 0.5 * sq * K2 * spv * smv;
}
void orc_nbw_G(double d, double chi, const double Sp[3], const double Sm[3], const double a[3],
               const double b[3], const double v[3], double G[4]) {
    double K1, K2, I;
    bessel_trio(2 / (3 * chi * d * (1 - d)), &K1, &K2, &I);
    nbw_G_bessel(d, I, K1, K2, Sp, Sm, a, b, v, G);
}

/* ======================================================== 4. table specification */
/* Grids (all uniform in the stated variable; "ln" grids are uniform in the natural log):
 *  BESSEL   NB=2048  ln x in [ln 1e-15, ln 1e3]; b1 = x^(1/3) e^x K13, b2 = x^(2/3) e^x K23,
 *                    b3 = e^x IntK13; 4-point Lagrange in ln x; x outside -> clamped node.
 *  NCS_RATE NR=512   ln chi in [ln 1e-6, ln 1e3]; fa = Ia/chi, fk = Ib/Ia; 4-point Lagrange.
 *                    chi < 1e-6: Ia = fa0 chi, fk = fk0 chi/1e-6.  chi > 1e3: clamp + flag.
 *  NCS_CDF  512 rows ln chi in [ln 1e-5, ln 1e3] x 1024 columns t in [0, 40^(1/3)];
 *                    normalised cumulative integrals A/A(tmax), B/B(tmax); linear in
 *                    ln chi between rows (clamped), piecewise linear in t.
 *  NBW_RATE NP=256   ln chi in [ln 0.05, ln 1e3]; ga = Ja e^(8/(3chi))/chi, gk = Jb/Ja;
 *                    4-point Lagrange; chi < 0.05: no pairs.
 *  NBW_CDF  256 rows ln chi in [ln 0.05, ln 1e3] x 512 columns delta in [0, 1/2];
 *                    Ka/Ja, Kb/Jb (value 1/2 at delta = 1/2); as NCS_CDF, mirrored.
 *  VB       NV=1024  ln chi in [ln 1e-4, ln 1e3]; M+, M-; 4-point Lagrange; below: 4, 7.
 *  RAD      NR=512   grid of NCS_RATE; h0 = g (1+chi)^(4/3) with g = emitted / Larmor power,
 *                    h_k = psi_k (1+chi)^(7/3) / chi^3 (k = 1, 2, 3): flat at both ends
 *                    (g ~ chi^(-4/3), psi ~ chi^(2/3) or less at large chi); 4-point
 *                    Lagrange, (1+chi)^(1/3) by cbrt.  chi < 1e-6: g = 1 - (55 sqrt3/16) chi,
 *                    psi_k = h_k(first node) chi^3 / (1+chi)^(7/3).  chi > 1e3: clamp + flag. */
#define NB 2048
#define B_LO (-34.538776394910684)   /* ln 1e-15 */
#define B_HI (6.907755278982137)     /* ln 1e3   */
#define NR 512
#define R_LO (-13.815510557964274)   /* ln 1e-6  */
#define R_HI (6.907755278982137)
#define NCR 512
#define NCT 1024
#define C_LO (-11.512925464970229)   /* ln 1e-5  */
#define C_HI (6.907755278982137)
#define T_MAX 3.4199518933533937     /* 40^(1/3) */
#define NP 256
#define P_LO (-2.995732273553991)    /* ln 0.05  */
#define P_HI (6.907755278982137)
#define NDR 256
#define NDD 512
#define NV 1024
#define V_LO (-9.210340371976182)    /* ln 1e-4  */
#define V_HI (6.907755278982137)

struct orc_tables {
    double bes[3][NB];
    double ncs_fa[NR], ncs_fk[NR];
    double *ncs_A, *ncs_B;     /* NCR x NCT each */
    double nbw_ga[NP], nbw_gk[NP];
    double *nbw_A, *nbw_B;     /* NDR x NDD each */
    double vb[2][NV];
    double rad[4][NR];         /* g, psi1/chi^3, psi2/chi^3, psi3/chi^3 */
};

static double grid_h(double lo, double hi, int n) { return (hi - lo) / (n - 1); }

orc_tables *orc_tables_build(void) {
    gl_init();
    orc_tables *T = calloc(1, sizeof(orc_tables));
    T->ncs_A = malloc(sizeof(double) * NCR * NCT);
    T->ncs_B = malloc(sizeof(double) * NCR * NCT);
    T->nbw_A = malloc(sizeof(double) * NDR * NDD);
    T->nbw_B = malloc(sizeof(double) * NDR * NDD);
    /* Bessel */
    double hb = grid_h(B_LO, B_HI, NB);
    for (int i = 0; i < NB; ++i) {
        double x = exp(B_LO + i * hb), K1, K2, I;
        bessel_trio_scaled(x, &K1, &K2, &I);
        T->bes[0][i] = cbrt(x) * K1;
        T->bes[1][i] = cbrt(x * x) * K2;
        T->bes[2][i] = I;
    }
    /* NCS rates */
    double hr = grid_h(R_LO, R_HI, NR);
    for (int i = 0; i < NR; ++i) {
        double chi = exp(R_LO + i * hr);
        double Ia = orc_ncs_Ia(chi), Ib = orc_ncs_Ib(chi);
        T->ncs_fa[i] = Ia / chi;
        T->ncs_fk[i] = Ib / Ia;
    }
    /* NCS CDF: Bessel values at the Gauss nodes of every t-panel do not depend on chi */
    {
        double ht = T_MAX / (NCT - 1);
        int nn = (NCT - 1) * GLN;
        double *bt = malloc(sizeof(double) * nn * 4);
        for (int j = 0; j < NCT - 1; ++j)
            for (int i = 0; i < GLN; ++i) {
                double t = ht * (j + 0.5 * (gl_x[i] + 1));
                double *q = bt + 4 * (j * GLN + i);
                q[0] = t;
                bessel_trio(t * t * t, &q[2], &q[3], &q[1]);   /* q1 = I, q2 = K1, q3 = K2 */
            }
        double hc = grid_h(C_LO, C_HI, NCR);
        for (int r = 0; r < NCR; ++r) {
            double chi = exp(C_LO + r * hc);
            double *A = T->ncs_A + (size_t)r * NCT, *B = T->ncs_B + (size_t)r * NCT;
            A[0] = 0; B[0] = 0;
            for (int j = 0; j < NCT - 1; ++j) {
                double sa = 0, sb = 0;
                for (int i = 0; i < GLN; ++i) {
                    double *q = bt + 4 * (j * GLN + i);
                    double wq = 0.5 * ht * gl_w[i];
                    sa += wq * ncs_integrand(0, chi, q[0], q[1], q[2], q[3]);
                    sb += wq * ncs_integrand(1, chi, q[0], q[1], q[2], q[3]);
                }
                A[j + 1] = A[j] + sa;
                B[j + 1] = B[j] + sb;
            }
            double na = A[NCT - 1], nb = B[NCT - 1];
            for (int j = 0; j < NCT; ++j) { A[j] /= na; B[j] /= nb; }
            A[NCT - 1] = 1; B[NCT - 1] = 1;
        }
        free(bt);
    }
    /* NBW rates */
    double hp = grid_h(P_LO, P_HI, NP);
    for (int i = 0; i < NP; ++i) {
        double chi = exp(P_LO + i * hp);
        double Ja = orc_nbw_Ja(chi), Jb = orc_nbw_Jb(chi);
        T->nbw_ga[i] = Ja * exp(8.0 / (3.0 * chi)) / chi;
        T->nbw_gk[i] = Jb / Ja;
    }
    /* NBW CDF */
    {
        double hd = 0.5 / (NDD - 1);
        double hq = grid_h(P_LO, P_HI, NDR);
        for (int r = 0; r < NDR; ++r) {
            double chi = exp(P_LO + r * hq);
            double *A = T->nbw_A + (size_t)r * NDD, *B = T->nbw_B + (size_t)r * NDD;
            A[0] = 0; B[0] = 0;
            for (int j = 0; j < NDD - 1; ++j) {
                double sa, sb;
                if (j == 0) {            /* first cell: panels halving towards delta = 0 */
                    sa = sb = 0;
                    for (int k = 0; k < 48; ++k) {
                        sa += nbw_gl(0, chi, ldexp(hd, -(k + 1)), ldexp(hd, -k));
                        sb += nbw_gl(1, chi, ldexp(hd, -(k + 1)), ldexp(hd, -k));
                    }
                } else {
                    sa = nbw_gl(0, chi, j * hd, (j + 1) * hd);
                    sb = nbw_gl(1, chi, j * hd, (j + 1) * hd);
                }
                A[j + 1] = A[j] + sa;
                B[j + 1] = B[j] + sb;
            }
            double na = 2 * A[NDD - 1], nb = 2 * B[NDD - 1];
            for (int j = 0; j < NDD; ++j) { A[j] /= na; B[j] /= nb; }
            A[NDD - 1] = 0.5; B[NDD - 1] = 0.5;
        }
    }
    /* VB */
    double hv = grid_h(V_LO, V_HI, NV);
    for (int i = 0; i < NV; ++i) {
        double M[2];
        orc_vb_M(exp(V_LO + i * hv), M);
        T->vb[0][i] = M[0];
        T->vb[1][i] = M[1];
    }
    /* radiative-correction coefficients on the NCS rate grid */
    for (int i = 0; i < NR; ++i) {
        double chi = exp(R_LO + i * hr), psi[3], o = 1 + chi, oc = cbrt(o);
        T->rad[0][i] = orc_ncs_power_ratio(chi) * o * oc;
        orc_rbmt_psi(chi, psi);
        for (int k = 0; k < 3; ++k) T->rad[k + 1][i] = psi[k] * (o * o * oc) / (chi * chi * chi);
    }
    return T;
}
void orc_tables_free(orc_tables *T) {
    if (!T) return;
    free(T->ncs_A); free(T->ncs_B); free(T->nbw_A); free(T->nbw_B);
    free(T);
}
int64_t orc_tables_size(int which) {
    switch (which) {
    case ORC_TAB_BESSEL: return 3 * NB;
    case ORC_TAB_NCS_RATE: return 2 * NR;
    case ORC_TAB_NCS_CDF: return 2 * (int64_t)NCR * NCT;
    case ORC_TAB_NBW_RATE: return 2 * NP;
    case ORC_TAB_NBW_CDF: return 2 * (int64_t)NDR * NDD;
    case ORC_TAB_VB: return 2 * NV;
    case ORC_TAB_RAD: return 4 * NR;
    }
    return 0;
}
void orc_tables_export(const orc_tables *T, int which, double *o) {
    switch (which) {
    case ORC_TAB_BESSEL: memcpy(o, T->bes, sizeof T->bes); break;
    case ORC_TAB_NCS_RATE: memcpy(o, T->ncs_fa, sizeof T->ncs_fa); memcpy(o + NR, T->ncs_fk, sizeof T->ncs_fk); break;
    case ORC_TAB_NCS_CDF:
        memcpy(o, T->ncs_A, sizeof(double) * NCR * NCT);
        memcpy(o + (size_t)NCR * NCT, T->ncs_B, sizeof(double) * NCR * NCT); break;
    case ORC_TAB_NBW_RATE: memcpy(o, T->nbw_ga, sizeof T->nbw_ga); memcpy(o + NP, T->nbw_gk, sizeof T->nbw_gk); break;
    case ORC_TAB_NBW_CDF:
        memcpy(o, T->nbw_A, sizeof(double) * NDR * NDD);
        memcpy(o + (size_t)NDR * NDD, T->nbw_B, sizeof(double) * NDR * NDD); break;
    case ORC_TAB_VB: memcpy(o, T->vb, sizeof T->vb); break;
    case ORC_TAB_RAD: memcpy(o, T->rad, sizeof T->rad); break;
    }
}

/* 4-point Lagrange interpolation on a uniform grid: stencil i-1..i+2, i = floor(pos)
 * clamped to [1, n-3], pos clamped to [0, n-1].  Returns the weights and i.          */
static int lagrange4(double pos, int n, double w[4]) {
    if (pos < 0) pos = 0;
    if (pos > n - 1) pos = n - 1;
    int i = (int)floor(pos);
    if (i < 1) i = 1;
    if (i > n - 3) i = n - 3;
    double f = pos - i;
    w[0] = -f * (f - 1) * (f - 2) / 6.0;
    w[1] = (f + 1) * (f - 1) * (f - 2) / 2.0;
    w[2] = -(f + 1) * f * (f - 2) / 2.0;
    w[3] = (f + 1) * f * (f - 1) / 6.0;
    return i;
}
static double lag_eval(const double *v, int i, const double w[4]) {
    return w[0] * v[i - 1] + w[1] * v[i] + w[2] * v[i + 1] + w[3] * v[i + 2];
}
/* scaled Bessel trio at x: returns I, K1, K2 multiplied by x^(2/3) e^x */
static void tab_bessel_scaled(const orc_tables *T, double x, double *I, double *K1, double *K2) {
    double w[4];
    int i = lagrange4((log(x) - B_LO) / grid_h(B_LO, B_HI, NB), NB, w);
    double b1 = lag_eval(T->bes[0], i, w), b2 = lag_eval(T->bes[1], i, w), b3 = lag_eval(T->bes[2], i, w);
    double x13 = cbrt(x);
    *I = b3 * x13 * x13;
    *K1 = b1 * x13;
    *K2 = b2;
}
void orc_tab_bessel(const orc_tables *T, double x, double out[3]) {
    double I, K1, K2;
    tab_bessel_scaled(T, x, &I, &K1, &K2);
    double s = exp(-x) / cbrt(x * x);
    out[0] = K1 * s; out[1] = K2 * s; out[2] = I * s;
}
static uint32_t g_status_scratch;
static void ncs_rate_lookup(const orc_tables *T, double chi, double *Ia, double *Ib, uint32_t *st) {
    if (chi <= 0) { *Ia = 0; *Ib = 0; return; }
    double l = log(chi);
    if (l < R_LO) {
        *Ia = T->ncs_fa[0] * chi;
        *Ib = T->ncs_fk[0] * (chi / 1e-6) * (*Ia);
        return;
    }
    if (l > R_HI) *st |= ORC_ST_CLAMP;
    double w[4];
    int i = lagrange4((l - R_LO) / grid_h(R_LO, R_HI, NR), NR, w);
    *Ia = lag_eval(T->ncs_fa, i, w) * chi;
    *Ib = lag_eval(T->ncs_fk, i, w) * (*Ia);
}
void orc_tab_ncs_rate(const orc_tables *T, double chi, double *Ia, double *Ib) {
    ncs_rate_lookup(T, chi, Ia, Ib, &g_status_scratch);
}
/* inverse of a piecewise-linear CDF D_j = a_j - m b_j (rows r0, r0+1 mixed with weight
 * f) at the target value; returns the fractional column position.                     */
static double cdf_invert(const double *A0, const double *A1, const double *B0, const double *B1,
                         int ncol, double f, double m, double target) {
    int lo = 0, hi = ncol - 1;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        double a = (1 - f) * A0[mid] + f * A1[mid];
        double b = (1 - f) * B0[mid] + f * B1[mid];
        if (a - m * b <= target) lo = mid; else hi = mid;
    }
    double dlo = ((1 - f) * A0[lo] + f * A1[lo]) - m * ((1 - f) * B0[lo] + f * B1[lo]);
    double dhi = ((1 - f) * A0[hi] + f * A1[hi]) - m * ((1 - f) * B0[hi] + f * B1[hi]);
    double tau = dhi > dlo ? (target - dlo) / (dhi - dlo) : 0.0;
    if (tau < 0) tau = 0;
    if (tau > 1) tau = 1;
    return lo + tau;
}
static void row_pos(double l, double lo, double hi, int n, int *r0, double *f) {
    double q = (l - lo) / grid_h(lo, hi, n);
    if (q < 0) q = 0;
    if (q > n - 1) q = n - 1;
    int r = (int)floor(q);
    if (r > n - 2) r = n - 2;
    *r0 = r;
    *f = q - r;
}
double orc_tab_ncs_sample_t(const orc_tables *T, double chi, double s, double r) {
    double Ia, Ib;
    uint32_t st = 0;
    ncs_rate_lookup(T, chi, &Ia, &Ib, &st);
    double kappa = Ib / Ia, m = s * kappa;
    int r0; double f;
    row_pos(log(chi), C_LO, C_HI, NCR, &r0, &f);
    const double *A0 = T->ncs_A + (size_t)r0 * NCT, *A1 = A0 + NCT;
    const double *B0 = T->ncs_B + (size_t)r0 * NCT, *B1 = B0 + NCT;
    double col = cdf_invert(A0, A1, B0, B1, NCT, f, m, r * (1 - m));
    return col * (T_MAX / (NCT - 1));
}

/* Targets of the learned NCS sampler (a function the library's network is trained to
 * reproduce; not a step of the paper's algorithm).  For an emission at chi with initial
 * spin components s = S.b and c = S.n in the local frame (Sec. III.C.1) and energy draw r:
 * out[0] = t = (2u/(3 chi))^(1/3) from the tabulated spin-dependent spectrum (the table
 * sampler), out[1], out[2] = F3/F0, F2/F0 of eqs. (F0)-(F3) at that u, summed over the two
 * final spins (terms linear in S_f cancel, so the sum is the S_f = 0 value): the mean
 * photon Stokes parameters xi3, xi2 at that energy.  S.a enters only F1 and is not needed. */
void orc_sampler_targets(const orc_tables *T, double chi, double s, double c, double r, double out[3]) {
    const double tt = orc_tab_ncs_sample_t(T, chi, s, r);
    const double x = tt * tt * tt, u = 1.5 * chi * x;
    double I, K1, K2;
    tab_bessel_scaled(T, x, &I, &K1, &K2);
    const double a[3] = {1, 0, 0}, b[3] = {0, 1, 0}, n[3] = {0, 0, 1};
    const double Si[3] = {0, s, c}, Sf[3] = {0, 0, 0};
    double F[4];
    ncs_F_bessel(u, I, K1, K2, Si, Sf, a, b, n, F);
    out[0] = tt;
    out[1] = F[3] / F[0];
    out[2] = F[2] / F[0];
}
void orc_sampler_targets_n(const orc_tables *T, int64_t n, const double *chi, const double *s, const double *c,
                           const double *r, double *out) {
    for (int64_t k = 0; k < n; ++k) orc_sampler_targets(T, chi[k], s[k], c[k], r[k], out + 3 * k);
}
static void nbw_rate_lookup(const orc_tables *T, double chi, double *Ja, double *Jb, uint32_t *st) {
    double l = chi > 0 ? log(chi) : -1e300;
    if (l < P_LO) { *Ja = 0; *Jb = 0; return; }
    if (l > P_HI) *st |= ORC_ST_CLAMP;
    double w[4];
    int i = lagrange4((l - P_LO) / grid_h(P_LO, P_HI, NP), NP, w);
    *Ja = lag_eval(T->nbw_ga, i, w) * chi * exp(-8.0 / (3.0 * chi));
    *Jb = lag_eval(T->nbw_gk, i, w) * (*Ja);
}
void orc_tab_nbw_rate(const orc_tables *T, double chi, double *Ja, double *Jb) {
    nbw_rate_lookup(T, chi, Ja, Jb, &g_status_scratch);
}
double orc_tab_nbw_sample_delta(const orc_tables *T, double chi, double xi3, double r) {
    double l = log(chi), w[4];
    int i = lagrange4((l - P_LO) / grid_h(P_LO, P_HI, NP), NP, w);
    double m = xi3 * lag_eval(T->nbw_gk, i, w);
    int r0; double f;
    row_pos(l, P_LO, P_HI, NDR, &r0, &f);
    const double *A0 = T->nbw_A + (size_t)r0 * NDD, *A1 = A0 + NDD;
    const double *B0 = T->nbw_B + (size_t)r0 * NDD, *B1 = B0 + NDD;
    double hd = 0.5 / (NDD - 1);
    if (r <= 0.5) return cdf_invert(A0, A1, B0, B1, NDD, f, m, r * (1 - m)) * hd;
    return 1.0 - cdf_invert(A0, A1, B0, B1, NDD, f, m, (1 - r) * (1 - m)) * hd;
}
/* Targets of the learned NBW sampler (a function the library's second network is trained
 * to reproduce; not a step of the paper's algorithm).  For a pair creation at chi_gamma by
 * a photon with Stokes parameter xi3 (in its basis e1 = a_+, Sec. III.D) and energy draw r:
 * out[0] = delta, the positron's energy fraction, from the tabulated spectrum (the table
 * sampler); out[1], out[2] = the mean spin of the positron and of the electron along
 * b = v x a at that delta with xi1 = xi2 = 0, summed over the partner's spin.  Summing
 * eqs. (G0)-(G3) over S_- = +-zeta drops every term linear in S_-; what is left at S_+ is
 * 2 [A + S_+ . B_+] with A = I + (rs - xi3) K2 and B_+ . b = K1 (xi3 / e_- - 1 / e_+), so
 * <S_+ . b> = B_+ . b / A; for the electron B_- . b = K1 (1 / e_- - xi3 / e_+) by the same
 * sum over S_+.  (e_+ = delta, e_- = 1 - delta, rs = (e_+^2 + e_-^2) / (e_+ e_-).)          */
void orc_nbw_sampler_targets(const orc_tables *T, double chi, double xi3, double r, double out[3]) {
    const double d = orc_tab_nbw_sample_delta(T, chi, xi3, r);
    const double ep = d, em = 1 - d;
    double I, K1, K2;
    tab_bessel_scaled(T, 2 / (3 * chi * ep * em), &I, &K1, &K2);
    const double rs = (ep * ep + em * em) / (ep * em);
    const double A = I + (rs - xi3) * K2;
    out[0] = d;
    out[1] = K1 * (xi3 / em - 1 / ep) / A;
    out[2] = K1 * (1 / em - xi3 / ep) / A;
}
void orc_nbw_sampler_targets_n(const orc_tables *T, int64_t n, const double *chi, const double *xi3, const double *r,
                               double *out) {
    for (int64_t k = 0; k < n; ++k) orc_nbw_sampler_targets(T, chi[k], xi3[k], r[k], out + 3 * k);
}
static void vb_lookup(const orc_tables *T, double chi, double M[2], uint32_t *st) {
    double l = chi > 0 ? log(chi) : -1e300;
    if (l < V_LO) { M[0] = 4.0; M[1] = 7.0; return; }
    if (l > V_HI) *st |= ORC_ST_CLAMP;
    double w[4];
    int i = lagrange4((l - V_LO) / grid_h(V_LO, V_HI, NV), NV, w);
    M[0] = lag_eval(T->vb[0], i, w);
    M[1] = lag_eval(T->vb[1], i, w);
}
void orc_tab_vb_M(const orc_tables *T, double chi, double M[2]) { vb_lookup(T, chi, M, &g_status_scratch); }
/* g(chi) and psi_1..3(chi) from the RAD table (specification in section 4) */
static void rad_lookup(const orc_tables *T, double chi, double out[4], uint32_t *st) {
    if (!(chi > 0)) { out[0] = 1; out[1] = out[2] = out[3] = 0; return; }
    double l = log(chi), o = 1 + chi, oc = cbrt(o), sp = chi * chi * chi / (o * o * oc);
    if (l < R_LO) {
        out[0] = 1 - 55 * SQRT3 / 16 * chi;
        for (int k = 1; k < 4; ++k) out[k] = T->rad[k][0] * sp;
        return;
    }
    if (l > R_HI) *st |= ORC_ST_CLAMP;
    double w[4];
    int i = lagrange4((l - R_LO) / grid_h(R_LO, R_HI, NR), NR, w);
    out[0] = lag_eval(T->rad[0], i, w) / (o * oc);
    for (int k = 1; k < 4; ++k) out[k] = lag_eval(T->rad[k], i, w) * sp;
}
void orc_tab_rad(const orc_tables *T, double chi, double out[4]) { rad_lookup(T, chi, out, &g_status_scratch); }

/* =========================================================================== 5. fields */
/* Plane wave travelling along -x (phase t + x, as in the pulse of Fig. "pusher"):
 * A(phi) = a0 sin^2(pi phi/L) [sin(phi + phase0) e1 + cos(phi + phase0) e2 (circular)],
 * phi = t + x - phi_start in [0, L], L = 2 pi ncycles; E = -dA/dphi, B = -x_hat cross E.
 * Focused pulse: zeroth-order paraxial Gaussian about x_focus with waist w0
 * (Rayleigh length w0^2/2 in units of 1/k), Gouy phase and wave-front curvature, the
 * same sin^2 envelope in t + x, E given directly, B = -x_hat cross E.
 * Grid: 2D Yee cell in the x-y plane (Ex (i+1/2,j), Ey (i,j+1/2), Ez (i,j),
 * Bx (i,j+1/2), By (i+1/2,j), Bz (i+1/2,j+1/2)), gathered with the TSC weights of
 * Sec. II.E on the nearest integer / half-integer node of Sec. II.D.                   */
static void pol_axes(const orc_field *f, double e1[3], double e2[3]) {
    double c = cos(f->pol_angle), s = sin(f->pol_angle);
    e1[0] = 0; e1[1] = c; e1[2] = s;
    e2[0] = 0; e2[1] = -s; e2[2] = c;
}
static void tsc_weights(double xg, int half, int *j0, double w[3]) {
    /* xg: position in cell units; node j sits at j (integer) or j + 1/2 (half) */
    int j = half ? (int)floor(xg) : (int)floor(xg + 0.5);
    double d = xg - (j + (half ? 0.5 : 0.0));
    w[0] = 0.5 * (0.5 - d) * (0.5 - d);
    w[1] = 0.75 - d * d;
    w[2] = 0.5 * (0.5 + d) * (0.5 + d);
    *j0 = j - 1;
}
static double grid_gather(const orc_field *f, const float *g, int hx, int hy, double x, double y) {
    int i0, j0;
    double wx[3], wy[3];
    tsc_weights((x - f->gx0) / f->dx, hx, &i0, wx);
    tsc_weights((y - f->gy0) / f->dy, hy, &j0, wy);
    double s = 0;
    for (int b = 0; b < 3; ++b) {
        int j = j0 + b;
        if (j < 0 || j >= f->ny) continue;
        for (int a = 0; a < 3; ++a) {
            int i = i0 + a;
            if (i < 0 || i >= f->nx) continue;
            s += wx[a] * wy[b] * (double)g[(size_t)j * f->nx + i];
        }
    }
    return s;
}
void orc_field_eval(const orc_field *f, double t, const double r[3], double E[3], double B[3]) {
    E[0] = E[1] = E[2] = B[0] = B[1] = B[2] = 0;
    if (!f) return;
    if (f->kind == ORC_FIELD_CONST) {
        memcpy(E, f->e0, 3 * sizeof(double));
        memcpy(B, f->b0, 3 * sizeof(double));
        return;
    }
    if (f->kind == ORC_FIELD_GRID2D) {
        static const int hx[6] = {1, 0, 0, 0, 1, 1}, hy[6] = {0, 1, 0, 1, 0, 1};
        double v[6];
        for (int c = 0; c < 6; ++c) v[c] = grid_gather(f, f->grid[c], hx[c], hy[c], r[0], r[1]);
        E[0] = v[0]; E[1] = v[1]; E[2] = v[2]; B[0] = v[3]; B[1] = v[4]; B[2] = v[5];
        return;
    }
    if (f->kind != ORC_FIELD_PW && f->kind != ORC_FIELD_GAUSS) return;
    double L = 2 * PI * f->ncycles;
    double phi = t + r[0] - f->phi_start;
    if (phi < 0 || phi > L) return;
    double e1[3], e2[3];
    pol_axes(f, e1, e2);
    double env = sin(PI * phi / L);
    env *= env;
    double c1, c2;     /* components of E along e1, e2 */
    if (f->kind == ORC_FIELD_PW) {
        double denv = (PI / L) * sin(2 * PI * phi / L);
        double ps = phi + f->phase0;
        c1 = -f->a0 * (denv * sin(ps) + env * cos(ps));
        c2 = f->circular ? -f->a0 * (denv * cos(ps) - env * sin(ps)) : 0.0;
    } else {
        double zr = 0.5 * f->w0 * f->w0;
        double xi = -(r[0] - f->x_focus);
        double rho2 = r[1] * r[1] + r[2] * r[2];
        double q = xi / zr, opq = 1 + q * q;
        double amp = f->a0 / sqrt(opq) * exp(-rho2 / (f->w0 * f->w0 * opq));
        double th = phi + f->phase0 - rho2 * xi / (2 * (xi * xi + zr * zr)) + atan(q);
        c1 = amp * env * cos(th);
        c2 = f->circular ? amp * env * sin(th) : 0.0;
    }
    for (int k = 0; k < 3; ++k) E[k] = c1 * e1[k] + c2 * e2[k];
    B[0] = 0; B[1] = E[2]; B[2] = -E[1];
}

/* ==================================================================== 6. push + spin */
/* Boris rotation, eqs. (boris1)-(boris6); p in/out is p^{n-1/2} -> p^{n+1/2}.          */
void orc_boris(double q, double dt, const double E[3], const double B[3], double p[3],
               double pm_out[3], double pp_out[3]) {
    double h = 0.5 * q * dt, pm[3], pp[3], pr[3], tau[3], sig[3], c[3];
    for (int k = 0; k < 3; ++k) pm[k] = p[k] + h * E[k];
    double g = sqrt(1 + dot3(pm, pm));
    for (int k = 0; k < 3; ++k) tau[k] = h * B[k] / g;
    double t2 = dot3(tau, tau);
    for (int k = 0; k < 3; ++k) sig[k] = 2 * tau[k] / (1 + t2);
    cross3(pm, tau, c);
    for (int k = 0; k < 3; ++k) pr[k] = pm[k] + c[k];
    cross3(pr, sig, c);
    for (int k = 0; k < 3; ++k) pp[k] = pm[k] + c[k];
    for (int k = 0; k < 3; ++k) p[k] = pp[k] + h * E[k];
    if (pm_out) memcpy(pm_out, pm, sizeof pm);
    if (pp_out) memcpy(pp_out, pp, sizeof pp);
}
/* T-BMT, eq. (bmteqn), advanced by the Boris rotation of eqs. (bmt-boris1)-(bmt-boris4):
 * dS/dt = q S x Omega, gamma^n = sqrt(1+|p-|^2), beta^n = (p- + p+)/(2 gamma^n),
 * g/2 - 1 = a_e.                                                                         */
void orc_bmt(double q, double a_e, double dt, const double E[3], const double B[3],
             const double pm[3], const double pp[3], double S[3]) {
    double g = sqrt(1 + dot3(pm, pm)), beta[3], bxe[3], om[3], tv[3], o[3], c[3], Sp[3];
    for (int k = 0; k < 3; ++k) beta[k] = (pm[k] + pp[k]) / (2 * g);
    double bB = dot3(beta, B);
    cross3(beta, E, bxe);
    double c1 = -a_e * g / (g + 1) * bB, c2 = a_e + 1 / g, c3 = a_e + 1 / (g + 1);
    for (int k = 0; k < 3; ++k) om[k] = c1 * beta[k] + c2 * B[k] - c3 * bxe[k];
    for (int k = 0; k < 3; ++k) tv[k] = 0.5 * q * dt * om[k];
    double t2 = dot3(tv, tv);
    for (int k = 0; k < 3; ++k) o[k] = 2 * tv[k] / (1 + t2);
    cross3(S, tv, c);
    for (int k = 0; k < 3; ++k) Sp[k] = S[k] + c[k];
    cross3(Sp, o, c);
    for (int k = 0; k < 3; ++k) S[k] += c[k];
}
/* chi_e = xi_L sqrt((gamma E + p x B)^2 - (p.E)^2) (Sec. III.A.1, read with p = gamma beta) */
double orc_chi_e(double xi_L, const double p[3], const double E[3], const double B[3]) {
    double g = sqrt(1 + dot3(p, p)), pxb[3], v[3];
    cross3(p, B, pxb);
    for (int k = 0; k < 3; ++k) v[k] = g * E[k] + pxb[k];
    double pe = dot3(p, E), s = dot3(v, v) - pe * pe;
    return xi_L * sqrt(s > 0 ? s : 0);
}
/* chi_gamma = xi_L eps |E - n (n.E) + n x B| (the reduced transverse field of Sec. III.C.2) */
static void ered(const double n[3], const double E[3], const double B[3], double er[3]) {
    double nE = dot3(n, E), nxb[3];
    cross3(n, B, nxb);
    for (int k = 0; k < 3; ++k) er[k] = E[k] - n[k] * nE + nxb[k];
}
double orc_chi_gamma(double xi_L, const double k[3], const double E[3], const double B[3]) {
    double e = norm3(k), n[3], er[3];
    if (e <= 0) return 0;
    for (int i = 0; i < 3; ++i) n[i] = k[i] / e;
    ered(n, E, B, er);
    return xi_L * e * norm3(er);
}
static int finite3(const double v[3]) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }

void orc_push_spin(orc_config *c, const orc_field *f, orc_leptons *L, int64_t step, double *E6) {
    double dt = c->dt, t = step * dt, q = (double)L->charge;
    for (int64_t i = 0; i < L->count; ++i) {
        double r[3] = {L->x[i], L->y[i], L->z[i]}, E[3], B[3];
        orc_field_eval(f, t, r, E, B);
        if (E6) { memcpy(E6 + 6 * i, E, sizeof E); memcpy(E6 + 6 * i + 3, B, sizeof B); }
        double p[3] = {L->px[i], L->py[i], L->pz[i]}, pm[3], pp[3];
        double S[3] = {L->sx[i], L->sy[i], L->sz[i]};
        orc_boris(q, dt, E, B, p, pm, pp);
        orc_bmt(q, c->a_e, dt, E, B, pm, pp, S);
        double g = sqrt(1 + dot3(p, p));
        for (int k = 0; k < 3; ++k) r[k] += dt * p[k] / g;
        if (!finite3(p) || !finite3(r) || !finite3(S)) c->status |= ORC_ST_NAN;
        L->x[i] = r[0]; L->y[i] = r[1]; L->z[i] = r[2];
        L->px[i] = p[0]; L->py[i] = p[1]; L->pz[i] = p[2];
        L->sx[i] = S[0]; L->sy[i] = S[1]; L->sz[i] = S[2];
    }
}

/* ============================================ 6b. radiation reaction (Sec. III.A, III.B) */
/* Classical Landau-Lifshitz force of eq. (eq1-1), its two leading terms (the paper names
 * them dominant; the field-derivative term is not included), with the 1/gamma of the
 * Gaussian-unit form (eq1) on E(p.E):
 *   F = (2/3) alpha xi_L { E x B + [B x (B x p) + E (p.E)] / gamma
 *                          - gamma p [(E + beta x B)^2 - (beta.E)^2] },  beta = p/gamma. */
void orc_ll_force(double alpha, double xi_L, double g, const double p[3], const double E[3],
                  const double B[3], double F[3]) {
    double beta[3], exb[3], bxp[3], bbp[3], bxb[3], v[3];
    for (int k = 0; k < 3; ++k) beta[k] = p[k] / g;
    cross3(E, B, exb);
    cross3(B, p, bxp);
    cross3(B, bxp, bbp);
    cross3(beta, B, bxb);
    for (int k = 0; k < 3; ++k) v[k] = E[k] + bxb[k];
    double pe = dot3(p, E), be = pe / g, s = dot3(v, v) - be * be;
    double c = 2.0 / 3.0 * alpha * xi_L;
    for (int k = 0; k < 3; ++k) F[k] = c * (exb[k] + (bbp[k] + E[k] * pe) / g - g * p[k] * s);
}

/* S += dt/2 R(S), R(S) = -P [psi1 S + psi2 (S.beta) beta + psi3 b]  (rc = {g, psi1..3}) */
static void rbmt_half_kick(double P, const double rc[4], const double beta[3], const double b[3], double dt,
                           double S[3]) {
    double sb = dot3(S, beta), R[3];
    for (int k = 0; k < 3; ++k) R[k] = -P * (rc[1] * S[k] + rc[2] * sb * beta[k] + rc[3] * b[k]);
    for (int k = 0; k < 3; ++k) S[k] += 0.5 * dt * R[k];
}
/* Radiative push (Sec. III.A.3) and radiative T-BMT (Sec. III.B.3) for every lepton:
 *   Boris with E^n, B^n: p^{n-1/2} -> p_L^{n+1/2};
 *   time-centred gamma^n = sqrt(1 + |p-|^2), beta^n = (p- + p+)/(2 gamma^n), p^n = gamma^n beta^n,
 *   chi^n = xi_L gamma^n sqrt((E + beta^n x B)^2 - (beta^n.E)^2);
 *   LL:  p^{n+1/2} = p_L^{n+1/2} + F(p^n) dt;  MLL: the same with g(chi^n) F;
 *   RBMT: S += dt/2 R(S), T-BMT rotation, S += dt/2 R(S), with
 *         R(S) = -P [psi1 S + psi2 (S.beta^n) beta^n + psi3 b],  P = alpha/(sqrt3 pi xi_L gamma^n),
 *         b = n x a of the local frame at time n (n = beta^n/|beta^n|, a = unit transverse part
 *         of q(E + beta^n x B)); S is not renormalised (it is the mean polarisation);
 *   x^{n+1} = x^n + dt p^{n+1/2}/gamma^{n+1/2}.                                          */
void orc_push_radiative(orc_config *c, const orc_tables *T, const orc_field *f, orc_leptons *L, int64_t step,
                        uint32_t mode) {
    double dt = c->dt, t = step * dt, q = (double)L->charge;
    const int force = mode & (ORC_RR_LL | ORC_RR_MLL), rbmt = (mode & ORC_RR_RBMT) != 0;
    for (int64_t i = 0; i < L->count; ++i) {
        double r[3] = {L->x[i], L->y[i], L->z[i]}, E[3], B[3];
        orc_field_eval(f, t, r, E, B);
        double p[3] = {L->px[i], L->py[i], L->pz[i]}, pm[3], pp[3];
        double S[3] = {L->sx[i], L->sy[i], L->sz[i]};
        orc_boris(q, dt, E, B, p, pm, pp);
        double g = sqrt(1 + dot3(pm, pm)), beta[3], pn[3], bxb[3], v[3];
        for (int k = 0; k < 3; ++k) { beta[k] = (pm[k] + pp[k]) / (2 * g); pn[k] = g * beta[k]; }
        cross3(beta, B, bxb);
        for (int k = 0; k < 3; ++k) v[k] = E[k] + bxb[k];
        double be = dot3(beta, E), s2 = dot3(v, v) - be * be;
        double chi = c->xi_L * g * sqrt(s2 > 0 ? s2 : 0), rc[4] = {1, 0, 0, 0};
        if ((force & ORC_RR_MLL) || rbmt) rad_lookup(T, chi, rc, &c->status);
        if (force) {
            double F[3];
            orc_ll_force(c->alpha, c->xi_L, g, pn, E, B, F);
            double scale = (force & ORC_RR_MLL) ? rc[0] : 1.0;
            for (int k = 0; k < 3; ++k) p[k] += scale * F[k] * dt;
        }
        if (rbmt) {
            double bn = norm3(beta), b[3] = {0, 0, 0};
            if (bn > 0) {
                double n[3], ad[3];
                for (int k = 0; k < 3; ++k) n[k] = beta[k] / bn;
                double nv = dot3(n, v);
                for (int k = 0; k < 3; ++k) ad[k] = q * (v[k] - nv * n[k]);
                double an = norm3(ad);
                if (an > 0) {
                    for (int k = 0; k < 3; ++k) ad[k] /= an;
                    cross3(n, ad, b);
                }
            }
            double P = c->alpha / (SQRT3 * PI * c->xi_L * g);
            rbmt_half_kick(P, rc, beta, b, dt, S);
            orc_bmt(q, c->a_e, dt, E, B, pm, pp, S);
            rbmt_half_kick(P, rc, beta, b, dt, S);
        } else {
            orc_bmt(q, c->a_e, dt, E, B, pm, pp, S);
        }
        double gp = sqrt(1 + dot3(p, p));
        for (int k = 0; k < 3; ++k) r[k] += dt * p[k] / gp;
        if (!finite3(p) || !finite3(r) || !finite3(S)) c->status |= ORC_ST_NAN;
        L->x[i] = r[0]; L->y[i] = r[1]; L->z[i] = r[2];
        L->px[i] = p[0]; L->py[i] = p[1]; L->pz[i] = p[2];
        L->sx[i] = S[0]; L->sy[i] = S[1]; L->sz[i] = S[2];
    }
}

/* ========================================================================= 7. NCS step */
/* Per lepton and step (Sec. III.C.1, with the readings of the rate normalisation, the
 * w/f/g decomposition, the no-emission update and the acceptance listed in DESIGN):
 *   frames: n = p/|p|, a = unit transverse part of q(E + beta x B - beta(beta.E)),
 *           b = n x a;  s = S.b
 *   W = C Ia(chi), f = -C Ib(chi) b, W_tot = W + f.S, C = alpha/(sqrt3 pi xi_L gamma)
 *   r2 < W_tot dt: emission.  r1 -> photon fraction y by the inverse of the
 *   spin-dependent spectrum; k = y p, p -> (1-y) p.  Final spin along g/|g| with
 *   probability (1 + |g|/(w + f.S))/2 (r3), otherwise antiparallel.  Photon Stokes
 *   (r4): pure state +-F/|F| with probability (F0 +- |F|)/(2 F0), F at the chosen S_f.
 *   no emission: S -> [S(1 - W dt) - f dt]/(1 - W_tot dt), renormalised.               */
static void emit_one(orc_config *c, const orc_tables *T, orc_leptons *L, int64_t i,
                     const double *E6, orc_photons *G, int64_t step) {
    const double *E = E6 + 6 * i, *B = E6 + 6 * i + 3;
    double p[3] = {L->px[i], L->py[i], L->pz[i]}, S[3] = {L->sx[i], L->sy[i], L->sz[i]};
    double q = (double)L->charge;
    double pp2 = dot3(p, p), g = sqrt(1 + pp2), pm = sqrt(pp2);
    double chi = orc_chi_e(c->xi_L, p, E, B);
    if (!(chi > 0) || pm <= 0) return;
    double n[3], beta[3], bxb[3], acc[3], a[3], b[3];
    for (int k = 0; k < 3; ++k) { n[k] = p[k] / pm; beta[k] = p[k] / g; }
    cross3(beta, B, bxb);
    double be = dot3(beta, E);
    for (int k = 0; k < 3; ++k) acc[k] = q * (E[k] + bxb[k] - beta[k] * be);
    double an = dot3(n, acc);
    for (int k = 0; k < 3; ++k) a[k] = acc[k] - n[k] * an;
    double anorm = norm3(a);
    if (!(anorm > 0)) return;
    for (int k = 0; k < 3; ++k) a[k] /= anorm;
    cross3(n, a, b);
    double s = dot3(S, b);
    double Ia, Ib;
    ncs_rate_lookup(T, chi, &Ia, &Ib, &c->status);
    double C = c->alpha / (SQRT3 * PI * c->xi_L * g);
    double W = C * Ia, Wt = C * (Ia - s * Ib), P = Wt * c->dt;
    if (P > c->p_max) c->status |= ORC_ST_PMAX;
    double r[4];
    orc_uniform4(L->id[i], step, ORC_STREAM_NCS, c->seed, r);
    if (r[1] < P) {
        double tt = orc_tab_ncs_sample_t(T, chi, s, r[0]);
        double u = 1.5 * chi * tt * tt * tt, y = u / (1 + u);
        double k[3], pf[3];
        for (int j = 0; j < 3; ++j) { k[j] = y * p[j]; pf[j] = (1 - y) * p[j]; }
        double I, K1, K2;
        tab_bessel_scaled(T, tt * tt * tt, &I, &K1, &K2);
        double w = -(1 + u) * I + (2 + 2 * u + u * u) * K2;
        double fS = -u * K1 * s;
        double sn = dot3(S, n), gv[3];
        for (int j = 0; j < 3; ++j)
            gv[j] = -(1 + u) * (I - 2 * K2) * S[j] - u * (1 + u) * K1 * b[j] - u * u * (I - K2) * sn * n[j];
        double gn = norm3(gv), zeta[3];
        if (gn > 0) for (int j = 0; j < 3; ++j) zeta[j] = gv[j] / gn;
        else memcpy(zeta, S, sizeof zeta);
        double pplus = 0.5 * (1 + gn / (w + fS));
        double Sf[3], sg = r[2] < pplus ? 1.0 : -1.0;
        for (int j = 0; j < 3; ++j) Sf[j] = sg * zeta[j];
        double xi[3] = {0, 0, 0};
        if (c->procs & ORC_PROC_NCS_STOKES) {
            double F[4];
            ncs_F_bessel(u, I, K1, K2, S, Sf, a, b, n, F);
            double fn = sqrt(F[1] * F[1] + F[2] * F[2] + F[3] * F[3]);
            if (fn > 0) {
                double sx = r[3] < (F[0] + fn) / (2 * F[0]) ? 1.0 : -1.0;
                for (int j = 0; j < 3; ++j) xi[j] = sx * F[j + 1] / fn;
            } else {
                xi[2] = r[3] < 0.5 ? 1.0 : -1.0;
            }
        }
        L->px[i] = pf[0]; L->py[i] = pf[1]; L->pz[i] = pf[2];
        L->sx[i] = Sf[0]; L->sy[i] = Sf[1]; L->sz[i] = Sf[2];
        uint64_t nid = c->next_id++;
        if (G) {
            if (G->count < G->capacity) {
                int64_t o = G->count++;
                G->x[o] = L->x[i]; G->y[o] = L->y[i]; G->z[o] = L->z[i];
                G->kx[o] = k[0]; G->ky[o] = k[1]; G->kz[o] = k[2];
                G->w[o] = L->w[i];
                G->xi1[o] = xi[0]; G->xi2[o] = xi[1]; G->xi3[o] = xi[2];
                G->e1x[o] = a[0]; G->e1y[o] = a[1]; G->e1z[o] = a[2];
                G->id[o] = nid;
                G->alive[o] = 1;
            } else {
                c->status |= ORC_ST_OVERFLOW;
            }
        }
    } else {
        double den = 1 - Wt * c->dt, Sb[3];
        for (int j = 0; j < 3; ++j) Sb[j] = (S[j] * (1 - W * c->dt) + C * Ib * c->dt * b[j]) / den;
        double sn = norm3(Sb);
        L->sx[i] = Sb[0] / sn; L->sy[i] = Sb[1] / sn; L->sz[i] = Sb[2] / sn;
    }
}
void orc_emit(orc_config *c, const orc_tables *T, orc_leptons *L, const double *E6, orc_photons *G,
              int64_t step) {
    if (!(c->procs & ORC_PROC_NCS)) return;
    int64_t n = L->count;
    for (int64_t i = 0; i < n; ++i) emit_one(c, T, L, i, E6, G, step);
}

/* ================================================================ 8. photon step */
/* Per live photon (Algorithm 1 and Sec. III.D):
 *   E_red = E - n(n.E) + n x B, chi_gamma = xi_L eps |E_red|.
 *   Frame: e1' = E_red/|E_red|; cos psi = e1.e1', sin psi = (n x e1).e1'; xi -> ROT(psi) xi
 *   (eq. rotation); e1 -> e1'.
 *   VB: delta phi = (M+ - M-)(alpha/(90 pi)) chi^2 dt/(eps xi_L); xi -> QED(delta phi) xi
 *   (eq. rotation2, phase over the step length of a photon of wavenumber eps/xi_L).
 *   NBW (eps >= 2): W = alpha/(sqrt3 pi xi_L eps)(Ja - xi3 Jb); r2 < W dt: pair.
 *   r1 -> delta by the inverse spectrum; SQAs D/|D|, D'/|D'| (eqs. BWposAxis, BWeleAxis);
 *   r3 picks (S+,S-) in the order (+,+),(+,-),(-,+),(-,-) with weights max(0, G0 + xi.G).
 *   Pair placed at the photon position, p = sqrt(eps^2-1) n; photon removed.
 *   Surviving photons move x += n dt.                                                    */
static void append_lepton(orc_config *c, orc_leptons *L, const double x[3], const double p[3],
                          const double S[3], double w, uint64_t id) {
    if (!L) return;
    if (L->count >= L->capacity) { c->status |= ORC_ST_OVERFLOW; return; }
    int64_t o = L->count++;
    L->x[o] = x[0]; L->y[o] = x[1]; L->z[o] = x[2];
    L->px[o] = p[0]; L->py[o] = p[1]; L->pz[o] = p[2];
    L->sx[o] = S[0]; L->sy[o] = S[1]; L->sz[o] = S[2];
    L->w[o] = w;
    L->id[o] = id;
}
void orc_photon_step(orc_config *c, const orc_tables *T, const orc_field *f, orc_photons *Gp,
                     orc_leptons *em, orc_leptons *ep, int64_t step) {
    double dt = c->dt, t = step * dt;
    int64_t n0 = Gp->count;
    for (int64_t j = 0; j < n0; ++j) {
        if (!Gp->alive[j]) continue;
        double x[3] = {Gp->x[j], Gp->y[j], Gp->z[j]}, k[3] = {Gp->kx[j], Gp->ky[j], Gp->kz[j]};
        double eps = norm3(k), n[3], E[3], B[3], er[3];
        for (int i = 0; i < 3; ++i) n[i] = k[i] / eps;
        orc_field_eval(f, t, x, E, B);
        ered(n, E, B, er);
        double an = norm3(er), chi = c->xi_L * eps * an;
        double xi[3] = {Gp->xi1[j], Gp->xi2[j], Gp->xi3[j]};
        double e1[3] = {Gp->e1x[j], Gp->e1y[j], Gp->e1z[j]};
        int killed = 0;
        if (an > 0 && (c->procs & (ORC_PROC_VB | ORC_PROC_NBW))) {
            double e1n[3], e2[3];
            for (int i = 0; i < 3; ++i) e1n[i] = er[i] / an;
            cross3(n, e1, e2);
            double cp = dot3(e1, e1n), sp = dot3(e2, e1n), nn = cp * cp + sp * sp;
            double c2 = (cp * cp - sp * sp) / nn, s2 = 2 * cp * sp / nn;
            double x1 = c2 * xi[0] - s2 * xi[2], x3 = s2 * xi[0] + c2 * xi[2];
            xi[0] = x1; xi[2] = x3;
            memcpy(e1, e1n, sizeof e1);
            if (c->procs & ORC_PROC_VB) {
                double M[2];
                vb_lookup(T, chi, M, &c->status);
                double dphi = (M[0] - M[1]) * (c->alpha / (90 * PI)) * chi * chi * dt / (eps * c->xi_L);
                double cd = cos(dphi), sd = sin(dphi);
                double y1 = cd * xi[0] - sd * xi[1], y2 = sd * xi[0] + cd * xi[1];
                xi[0] = y1; xi[1] = y2;
            }
            if ((c->procs & ORC_PROC_NBW) && eps >= 2) {
                double Ja, Jb;
                nbw_rate_lookup(T, chi, &Ja, &Jb, &c->status);
                double P = c->alpha / (SQRT3 * PI * c->xi_L * eps) * (Ja - xi[2] * Jb) * dt;
                if (P > c->p_max) c->status |= ORC_ST_PMAX;
                double r[4];
                orc_uniform4(Gp->id[j], step, ORC_STREAM_NBW, c->seed, r);
                if (Ja > 0 && r[1] < P) {
                    double d = orc_tab_nbw_sample_delta(T, chi, xi[2], r[0]);
                    double epl = d * eps, emi = eps - epl;
                    double I, K1, K2;
                    tab_bessel_scaled(T, 2.0 / (3.0 * chi * d * (1 - d)), &I, &K1, &K2);
                    double *a = e1, bb[3], D[3], Dm[3];
                    cross3(n, a, bb);
                    double ip = eps / epl, im = eps / emi, ds = (epl * epl - emi * emi) / (emi * epl);
                    for (int i = 0; i < 3; ++i) {
                        D[i] = -(ip - xi[2] * im) * K1 * bb[i] - xi[0] * im * K1 * a[i]
                               + xi[1] * (ds * K2 + ip * I) * n[i];
                        Dm[i] = (im - xi[2] * ip) * K1 * bb[i] + xi[0] * ip * K1 * a[i]
                                - xi[1] * (ds * K2 - im * I) * n[i];
                    }
                    double dn = norm3(D), dmn = norm3(Dm), zp[3], zm[3];
                    for (int i = 0; i < 3; ++i) {
                        zp[i] = dn > 0 ? D[i] / dn : bb[i];
                        zm[i] = dmn > 0 ? Dm[i] / dmn : bb[i];
                    }
                    double Pk[4], tot = 0;
                    for (int kk = 0; kk < 4; ++kk) {
                        double sp_ = kk < 2 ? 1.0 : -1.0, sm_ = (kk % 2 == 0) ? 1.0 : -1.0;
                        double Sp[3], Sm[3], Gv[4];
                        for (int i = 0; i < 3; ++i) { Sp[i] = sp_ * zp[i]; Sm[i] = sm_ * zm[i]; }
                        nbw_G_bessel(d, I, K1, K2, Sp, Sm, a, bb, n, Gv);
                        double v = Gv[0] + xi[0] * Gv[1] + xi[1] * Gv[2] + xi[2] * Gv[3];
                        Pk[kk] = v > 0 ? v : 0;
                        tot += Pk[kk];
                    }
                    int sel = 3;
                    double acc = 0, thr = r[2] * tot;
                    for (int kk = 0; kk < 4; ++kk) { acc += Pk[kk]; if (thr < acc) { sel = kk; break; } }
                    double sgp = sel < 2 ? 1.0 : -1.0, sgm = (sel % 2 == 0) ? 1.0 : -1.0;
                    double Sp[3], Sm[3], ppl[3], pmi[3];
                    if (epl < 1 || emi < 1) c->status |= ORC_ST_EPS_LT1;
                    double qp = epl * epl - 1, qm = emi * emi - 1;
                    qp = qp > 0 ? sqrt(qp) : 0;
                    qm = qm > 0 ? sqrt(qm) : 0;
                    for (int i = 0; i < 3; ++i) {
                        Sp[i] = sgp * zp[i]; Sm[i] = sgm * zm[i];
                        ppl[i] = qp * n[i]; pmi[i] = qm * n[i];
                    }
                    uint64_t id0 = c->next_id;
                    c->next_id += 2;
                    append_lepton(c, em, x, pmi, Sm, Gp->w[j], id0);
                    append_lepton(c, ep, x, ppl, Sp, Gp->w[j], id0 + 1);
                    Gp->alive[j] = 0;
                    killed = 1;
                }
            }
        }
        Gp->xi1[j] = xi[0]; Gp->xi2[j] = xi[1]; Gp->xi3[j] = xi[2];
        Gp->e1x[j] = e1[0]; Gp->e1y[j] = e1[1]; Gp->e1z[j] = e1[2];
        if (!killed) {
            Gp->x[j] = x[0] + n[0] * dt; Gp->y[j] = x[1] + n[1] * dt; Gp->z[j] = x[2] + n[2] * dt;
        }
    }
}
int64_t orc_compact_photons(orc_photons *G) {
    int64_t o = 0;
    for (int64_t j = 0; j < G->count; ++j) {
        if (!G->alive[j]) continue;
        if (o != j) {
            G->x[o] = G->x[j]; G->y[o] = G->y[j]; G->z[o] = G->z[j];
            G->kx[o] = G->kx[j]; G->ky[o] = G->ky[j]; G->kz[o] = G->kz[j];
            G->w[o] = G->w[j];
            G->xi1[o] = G->xi1[j]; G->xi2[o] = G->xi2[j]; G->xi3[o] = G->xi3[j];
            G->e1x[o] = G->e1x[j]; G->e1y[o] = G->e1y[j]; G->e1z[o] = G->e1z[j];
            G->id[o] = G->id[j];
            G->alive[o] = 1;
        }
        ++o;
    }
    G->count = o;
    return o;
}

/* ============================================================ 10. detector diagnostics */
/* bin of value v on axis k of h (energy axes: by comparison with the log10-spaced edges);
 * -1 outside                                                                            */
static int hist_bin(const orc_hist_spec *h, int k, double v) {
    if (h->axis[k] == ORC_AX_ENERGY) {
        int n = h->n[k];
        double w = (h->hi[k] - h->lo[k]) / n;
        if (!(v >= pow(10.0, h->lo[k])) || !(v < pow(10.0, h->lo[k] + n * w))) return -1;
        int i = 0;
        while (i + 1 < n && pow(10.0, h->lo[k] + (i + 1) * w) <= v) ++i;
        return i;
    }
    double x = floor((v - h->lo[k]) * (h->n[k] / (h->hi[k] - h->lo[k])));
    return (x >= 0 && x < h->n[k]) ? (int)x : -1;
}
static double axis_value(int axis, const double p[3], double energy) {
    switch (axis) {
    case ORC_AX_SLOPE_Y: return p[1] / p[0];
    case ORC_AX_SLOPE_Z: return p[2] / p[0];
    case ORC_AX_SLOPE_R: return sqrt(p[1] * p[1] + p[2] * p[2]) / p[0];
    default: return energy;
    }
}
static int hist_cell(const orc_hist_spec *h, const double p[3], double energy) {
    if (!(p[0] > 0)) return -1;
    int a = hist_bin(h, 0, axis_value(h->axis[0], p, energy));
    int b = hist_bin(h, 1, axis_value(h->axis[1], p, energy));
    return (a < 0 || b < 0) ? -1 : b * h->n[0] + a;
}
void orc_hist_photons(const orc_photons *G, int64_t begin, const orc_hist_spec *h, double *out) {
    for (int64_t j = begin; j < G->count; ++j) {
        if (!G->alive[j]) continue;
        double k[3] = {G->kx[j], G->ky[j], G->kz[j]}, eps = norm3(k);
        int cell = hist_cell(h, k, eps);
        if (cell < 0) continue;
        double n[3], e1[3] = {G->e1x[j], G->e1y[j], G->e1z[j]}, e2[3], d[3];
        for (int q = 0; q < 3; ++q) n[q] = k[q] / eps;
        double nd = dot3(n, h->pol_ref);
        for (int q = 0; q < 3; ++q) d[q] = h->pol_ref[q] - nd * n[q];
        double dn = norm3(d);
        for (int q = 0; q < 3; ++q) d[q] /= dn;
        cross3(n, e1, e2);
        /* rotation from (e1, n x e1) to (d, n x d): eq. (rotation) with cos psi = e1.d,
         * sin psi = e2.d, applied through cos 2psi, sin 2psi                              */
        double c = dot3(e1, d), s = dot3(e2, d), c2 = c * c - s * s, s2 = 2 * c * s;
        double x1 = G->xi1[j], x2 = G->xi2[j], x3 = G->xi3[j], w = G->w[j];
        double *o = out + 5 * (int64_t)cell;
        o[0] += w;
        o[1] += w * eps;
        o[2] += w * (c2 * x1 - s2 * x3);
        o[3] += w * x2;
        o[4] += w * (s2 * x1 + c2 * x3);
    }
}
void orc_hist_leptons(const orc_leptons *L, int64_t begin, const orc_hist_spec *h, double *out) {
    for (int64_t i = begin; i < L->count; ++i) {
        double p[3] = {L->px[i], L->py[i], L->pz[i]}, g = sqrt(1 + dot3(p, p));
        int cell = hist_cell(h, p, g);
        if (cell < 0) continue;
        double w = L->w[i], *o = out + 5 * (int64_t)cell;
        o[0] += w;
        o[1] += w * g;
        o[2] += w * L->sx[i];
        o[3] += w * L->sy[i];
        o[4] += w * L->sz[i];
    }
}

