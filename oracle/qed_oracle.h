/*
 * qed_oracle.h -- plain, slow, FP64 CPU oracle for the spin/polarisation-resolved
 * strong-field QED particle step of Wan et al., "Simulations of spin/polarization-
 * resolved laser-plasma interactions in the nonlinear QED regime" (arXiv:2306.11288).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls this
 * code; only the tests, the smoke check and the CPU-baseline leg of the benchmark do.
 * It shares no source with the HIP library: every formula here is written out again
 * from the paper, in the paper's order and notation.
 *
 * Units (paper Sec. I, last paragraph): t in 1/omega, x in 1/k, p in m c, energy in
 * m c^2, E and B in m c omega / e.  xi_L = hbar omega / m c^2.
 *
 * Every function is single-threaded and allocation-free unless stated.
 */
#ifndef QED_ORACLE_H
#define QED_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------- counter-based RNG (Salmon et al., SC'11, Philox4x32-10) -------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* four uniforms in (0,1) for particle `id` at `step`, process stream `stream` */
void orc_uniform4(uint64_t id, int64_t step, uint32_t stream, uint64_t seed, double r[4]);

/* ---------------- special functions ---------------------------------------------- */
double orc_bessel_k(double nu, double x);      /* K_nu(x), x > 0                      */
double orc_int_bessel_k(double nu, double x);  /* int_x^inf K_nu(z) dz                */
double orc_scorer_gi_prime(double x);          /* Gi'(x), x >= 0                      */

/* ---------------- direct quadrature ("truth") of the paper's integrals ------------ */
/* NCS: total rate W = alpha/(sqrt3 pi xi_L gamma) * (Ia - s Ib), s = S.(n x a)      */
double orc_ncs_Ia(double chi);
double orc_ncs_Ib(double chi);
/* partial integrals up to photon energy fraction y (the unnormalised CDF pieces)   */
double orc_ncs_A(double chi, double y);
double orc_ncs_B(double chi, double y);
/* quantum/classical emitted power ratio (the Gaunt factor q(chi) of Sec. III.A.2)  */
double orc_ncs_power_ratio(double chi);
/* radiative T-BMT integrals psi1..psi3 (Sec. III.B.2)                               */
void orc_rbmt_psi(double chi, double psi[3]);
/* NBW: W_pair = alpha/(sqrt3 pi xi_L eps_gamma) * (Ja - xi3 Jb)                      */
double orc_nbw_Ja(double chi);
double orc_nbw_Jb(double chi);
double orc_nbw_Ka(double chi, double delta);   /* partial integral over [0, delta]   */
double orc_nbw_Kb(double chi, double delta);
/* VB: Re n = 1 + M(chi) D; M[0] = M_plus (mode along E_red), M[1] = M_minus         */
void orc_vb_M(double chi, double M[2]);
/* the F0..F3 functions of the NCS rate (eqs. F0-F3) for given u, chi and spins,
 * triad (a, b = n x a, n).  Returns F[0..3].                                        */
void orc_ncs_F(double u, double chi, const double Si[3], const double Sf[3],
               const double a[3], const double b[3], const double n[3], double F[4]);
/* the NBW G0..G3 (eqs. G0-G3) without the common W0/2 factor                       */
void orc_nbw_G(double delta, double chi, const double Sp[3], const double Sm[3],
               const double a[3], const double b[3], const double v[3], double G[4]);

/* ---------------- the table specification (shared *spec*, not shared code) ------- */
typedef struct orc_tables orc_tables;
orc_tables *orc_tables_build(void);
void orc_tables_free(orc_tables *t);
/* table ids for export */
enum { ORC_TAB_BESSEL = 0, ORC_TAB_NCS_RATE = 1, ORC_TAB_NCS_CDF = 2, ORC_TAB_NBW_RATE = 3,
       ORC_TAB_NBW_CDF = 4, ORC_TAB_VB = 5, ORC_TAB_RAD = 6 };
int64_t orc_tables_size(int which);                    /* number of doubles           */
void orc_tables_export(const orc_tables *t, int which, double *out);
/* lookups that follow the specification exactly                                    */
void orc_tab_bessel(const orc_tables *t, double x, double out[3]);  /* K13, K23, IntK13 */
void orc_tab_ncs_rate(const orc_tables *t, double chi, double *Ia, double *Ib);
double orc_tab_ncs_sample_t(const orc_tables *t, double chi, double s, double r);
/* learned-sampler targets: t, mean xi3, mean xi2 (see the definition) */
void orc_sampler_targets(const orc_tables *t, double chi, double s, double c, double r, double out[3]);
void orc_sampler_targets_n(const orc_tables *t, int64_t n, const double *chi, const double *s, const double *c,
                           const double *r, double *out);
void orc_tab_nbw_rate(const orc_tables *t, double chi, double *Ja, double *Jb);
double orc_tab_nbw_sample_delta(const orc_tables *t, double chi, double xi3, double r);
/* learned NBW sampler targets: delta from the table sampler, mean positron / electron spin along b */
void orc_nbw_sampler_targets(const orc_tables *t, double chi, double xi3, double r, double out[3]);
void orc_nbw_sampler_targets_n(const orc_tables *t, int64_t n, const double *chi, const double *xi3, const double *r,
                               double *out);
void orc_tab_vb_M(const orc_tables *t, double chi, double M[2]);
/* radiative coefficients: out = {g(chi), psi1, psi2, psi3}                          */
void orc_tab_rad(const orc_tables *t, double chi, double out[4]);

/* ---------------- fields, particles, segments ------------------------------------ */
enum { ORC_FIELD_NONE = 0, ORC_FIELD_CONST = 1, ORC_FIELD_PW = 2, ORC_FIELD_GAUSS = 3,
       ORC_FIELD_GRID2D = 4 };
typedef struct {
    int32_t kind;
    int32_t circular;                 /* 0 linear, 1 circular                         */
    double a0, ncycles, phase0, pol_angle, w0, x_focus, phi_start;
    double e0[3], b0[3];              /* ORC_FIELD_CONST                              */
    const float *grid[6];             /* ORC_FIELD_GRID2D: Ex,Ey,Ez,Bx,By,Bz           */
    int32_t nx, ny;
    double dx, dy, gx0, gy0;
} orc_field;
void orc_field_eval(const orc_field *f, double t, const double r[3], double E[3], double B[3]);

typedef struct {
    double *x, *y, *z, *px, *py, *pz, *w, *sx, *sy, *sz;
    uint64_t *id;
    int64_t count, capacity;
    int32_t charge;
} orc_leptons;
typedef struct {
    double *x, *y, *z, *kx, *ky, *kz, *w, *xi1, *xi2, *xi3, *e1x, *e1y, *e1z;
    uint64_t *id;
    uint8_t *alive;
    int64_t count, capacity;
} orc_photons;

enum { ORC_PROC_NCS = 1, ORC_PROC_NCS_STOKES = 2, ORC_PROC_NBW = 4, ORC_PROC_VB = 8 };
enum { ORC_ST_OVERFLOW = 1, ORC_ST_NAN = 2, ORC_ST_PMAX = 4, ORC_ST_EPS_LT1 = 8,
       ORC_ST_CLAMP = 16 };
enum { ORC_STREAM_NCS = 1, ORC_STREAM_NBW = 2 };

typedef struct {
    double xi_L, alpha, a_e, dt, p_max;
    uint64_t seed;
    uint64_t next_id;                 /* in/out: id given to the next new particle    */
    uint32_t procs;
    uint32_t status;                  /* in/out: sticky status bits                   */
} orc_config;

/* Lorentz + T-BMT for every lepton (fields at x^n, t^n = step*dt).  If E6 is not
 * NULL the fields used are written there (6 doubles per particle).                 */
void orc_push_spin(orc_config *c, const orc_field *f, orc_leptons *L, int64_t step, double *E6);
/* radiation reaction (Sec. III.A-B): Landau-Lifshitz force (LL), the same scaled by the
 * emitted/Larmor power ratio g(chi) (MLL), radiative T-BMT (RBMT); see the definition.   */
enum { ORC_RR_LL = 1, ORC_RR_MLL = 2, ORC_RR_RBMT = 4 };
void orc_ll_force(double alpha, double xi_L, double g, const double p[3], const double E[3],
                  const double B[3], double F[3]);
void orc_push_radiative(orc_config *c, const orc_tables *tab, const orc_field *f, orc_leptons *L, int64_t step,
                        uint32_t mode);
/* NCS for every lepton that existed at the start of the step; E6 holds E^n,B^n.
 * Photons are appended in parent order.                                            */
void orc_emit(orc_config *c, const orc_tables *tab, orc_leptons *L, const double *E6,
              orc_photons *G, int64_t step);
/* photon step: VB (and the frame rotation), then NBW with pair append in parent
 * order (electrons to em, positrons to ep), then straight-line move.               */
void orc_photon_step(orc_config *c, const orc_tables *tab, const orc_field *f, orc_photons *G,
                     orc_leptons *em, orc_leptons *ep, int64_t step);
/* stable removal of dead photons; returns the new count                             */
int64_t orc_compact_photons(orc_photons *G);

/* detector diagnostics (the post-processing step of the VB algorithm, Sec. III.F):
 * particles heading to +x are binned on two axes and, per bin, w, w eps, and w times the
 * photon Stokes vector in the detector basis (or the lepton spin) are summed.  Axes:
 * slopes p_y/p_x, p_z/p_x, sqrt(p_y^2+p_z^2)/p_x (linear bins: i = floor((v - lo) n/(hi-lo)))
 * or the energy (|k| or gamma) on bins uniform in log10 between 10^lo and 10^hi (edges
 * 10^(lo + k (hi-lo)/n), found by comparison).  Photon detector basis: e1 = unit part of
 * pol_ref transverse to k, e2 = n x e1; xi rotated from (e1, n x e1) of the photon.       */
enum { ORC_AX_SLOPE_Y = 0, ORC_AX_SLOPE_Z = 1, ORC_AX_SLOPE_R = 2, ORC_AX_ENERGY = 3 };
typedef struct {
    int32_t axis[2], n[2];
    double lo[2], hi[2];
    double pol_ref[3];
} orc_hist_spec;
/* out[((b n[0]) + a) 5 + q] += (w, w eps, w xi1', w xi2', w xi3') for photons [begin, count) */
void orc_hist_photons(const orc_photons *G, int64_t begin, const orc_hist_spec *h, double *out);
/* the same for leptons: (w, w gamma, w Sx, w Sy, w Sz)                                 */
void orc_hist_leptons(const orc_leptons *L, int64_t begin, const orc_hist_spec *h, double *out);

/* single-particle pieces used by the pins */
void orc_boris(double q, double dt, const double E[3], const double B[3], double p[3],
               double pminus_out[3], double pplus_out[3]);
void orc_bmt(double q, double a_e, double dt, const double E[3], const double B[3],
             const double pminus[3], const double pplus[3], double S[3]);
double orc_chi_e(double xi_L, const double p[3], const double E[3], const double B[3]);
double orc_chi_gamma(double xi_L, const double k[3], const double E[3], const double B[3]);

#ifdef __cplusplus
}
#endif
#endif
