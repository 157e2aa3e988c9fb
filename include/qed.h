/*
 * qed.h -- C ABI of libqed: the per-particle hot path of spin/polarisation-resolved
 * strong-field QED in a particle-in-cell step (Wan et al., arXiv:2306.11288), on AMD
 * Instinct MI355X (gfx950).
 *
 * The path, per time step n (t^n = n dt):
 *   photons : field gather -> basis rotation to the pair-production frame (Sec. III.C.2,
 *             eq. rotation) -> vacuum birefringence (Sec. III.F, eq. rotation2,
 *             Algorithm 1) -> nonlinear Breit-Wheeler pair creation (Sec. III.D) ->
 *             straight-line move
 *   leptons : field gather (Sec. II.D-E) -> Boris push (Sec. II.A, eqs. boris1-boris6)
 *             -> T-BMT spin rotation (Sec. III.B, eqs. bmteqn, bmt-boris1-4) ->
 *             spin/polarisation-resolved nonlinear Compton emission (Sec. III.C.1)
 * qed_step runs one whole step with the result of the paper's Spin-QED chain (Sec. IV:
 * Lorentz push and T-BMT -> vacuum birefringence -> NBW -> NCS; bremsstrahlung is not
 * included): particles created in step n are first stepped in step n + 1.
 * Around it: the radiative-correction push (Sec. III.A-B, qed_push_radiative), the PIC
 * loop's charge-conserving current deposition and 2D Yee field solver (Sec. II.B-C, F;
 * qed_save_start, qed_deposit_current, qed_field_advance) and detector histograms
 * (Sec. III.F; qed_hist_photons, qed_hist_leptons).
 *
 * Conventions
 *  - Units: t in 1/omega, x in 1/k, momenta in m c, energies in m c^2, fields in
 *    m c omega / e (paper Sec. I).
 *  - Particle buffers are structure-of-arrays in device memory, owned by the caller.
 *    The library never allocates or frees them.  `count` is a device-resident int64;
 *    kernels read it and (for output lists) update it, so calls need no host sync.
 *  - Every call is asynchronous on the given stream and returns synchronously only
 *    argument errors (nothing is enqueued then; see qed_last_error).  Conditions found
 *    on the device set sticky bits in a device status word (qed_read_status).
 *  - Appended particles are stored in parent-index order (photons: order of the
 *    emitting lepton; pairs: order of the decaying photon) with ids taken from a
 *    device counter owned by the context (photon: id_base + rank; pair: electron
 *    id_base + 2 rank, positron id_base + 2 rank + 1).  Appends past `capacity` are
 *    dropped, still consume ids, and set QED_ST_OVERFLOW.
 *  - Random numbers: Philox4x32-10 with key = particle id and counter = (step low word,
 *    step bits 32..47 | stream << 16, seed low, seed high), stream 1 = NCS, 2 = NBW;
 *    uniforms (u + 1/2) 2^-32 in the order r1 (energy), r2 (event), r3 (spin),
 *    r4 (photon polarisation).
 *  - A context is used by one host thread and one stream at a time (the append calls
 *    share its scan state).
 */
#ifndef QED_H
#define QED_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *hipStream_t;
/* opaque context: device tables, constants, id counter, status word, scan state */
typedef struct qed_ctx qed_ctx_t;

/* Launch shape of the lepton step (decide / scan / event kernels).  Every choice gives
 * bitwise the same results; only the speed differs.  Default {0, 0, 8}.               */
typedef struct {
    int32_t blocks_per_cu;   /* 0: one block per 256-lepton tile; k > 0: a persistent grid
                                of k blocks per compute unit sweeping the tiles            */
    int32_t rate_lds;        /* 1: each decide block stages the NCS rate table in LDS     */
    int32_t ev_group;        /* tiles per wavefront of the event kernel: 4, 8 or 16       */
} qed_tuning;

typedef enum { QED_OK = 0, QED_EARG = 1, QED_ENOMEM = 2, QED_EHIP = 3, QED_ESTATE = 4 } qed_status;
typedef enum { QED_FP64 = 0, QED_MIXED = 1 } qed_precision;

/* process mask (qed_config.procs) */
enum { QED_PROC_NCS = 1, QED_PROC_NCS_STOKES = 2, QED_PROC_NBW = 4, QED_PROC_VB = 8 };
/* sticky device status bits */
enum {
    QED_ST_OVERFLOW = 1,   /* an append went past capacity (dropped)                   */
    QED_ST_NAN = 2,        /* non-finite momentum, position or spin after a push        */
    QED_ST_PMAX = 4,       /* a per-step event probability exceeded cfg.p_max          */
    QED_ST_EPS_LT1 = 8,    /* a pair member was born with energy below m c^2            */
    QED_ST_CLAMP = 16,     /* chi above the tabulated range (value clamped)             */
    QED_ST_SCAN = 32,      /* reserved; not set by this version */
    QED_ST_DEPOSIT = 64    /* current deposition skipped a particle that moved a cell or more
                              in one step, or whose position or weight is not finite     */
};
/* field kinds */
enum { QED_FIELD_NONE = 0, QED_FIELD_CONST = 1, QED_FIELD_PW = 2, QED_FIELD_GAUSS = 3,
       QED_FIELD_GRID2D = 4 };
/* table ids for qed_table_export */
enum { QED_TAB_BESSEL = 0, QED_TAB_NCS_RATE = 1, QED_TAB_NCS_CDF = 2, QED_TAB_NBW_RATE = 3,
       QED_TAB_NBW_CDF = 4, QED_TAB_VB = 5, QED_TAB_RAD = 6 };

typedef struct {
    double xi_L;        /* hbar omega / m c^2 of the reference wavelength (Sec. III.A.1)   */
    double alpha;       /* fine-structure constant                                        */
    double a_e;         /* anomalous magnetic moment, g = 2 (1 + a_e) (eq. bmteqn)        */
    double dt;          /* time step                                                      */
    double p_max;       /* event probability per step above which QED_ST_PMAX is set      */
    uint64_t seed;      /* Philox seed (counter words 2-3)                                */
    uint64_t id_start;  /* id of the first particle the library creates                   */
    int32_t precision;  /* qed_precision: storage/compute type of S, Stokes, basis, rates  */
    uint32_t procs;     /* QED_PROC_* mask                                                */
} qed_config;

/* electrons (charge -1) or positrons (+1).  sx, sy, sz are double for QED_FP64 and float
 * for QED_MIXED contexts.  Momenta live at half steps, positions at integer steps.      */
typedef struct {
    double *x, *y, *z, *px, *py, *pz, *w;
    void *sx, *sy, *sz;
    uint64_t *id;
    int64_t *count;     /* device scalar                                                  */
    int64_t capacity;
    int32_t charge;
} qed_leptons;

/* photons: momentum k (|k| = energy), Stokes parameters xi in the basis (e1, n x e1, n),
 * n = k/|k|; xi and e1 are double (QED_FP64) or float (QED_MIXED).  alive = 0 marks a
 * photon removed by pair creation (compact with qed_compact_photons).                   */
typedef struct {
    double *x, *y, *z, *kx, *ky, *kz, *w;
    void *xi1, *xi2, *xi3, *e1x, *e1y, *e1z;
    uint64_t *id;
    uint8_t *alive;
    int64_t *count;
    int64_t capacity;
} qed_photons;

/* External fields.
 *  CONST : uniform static E = e0, B = b0.
 *  PW    : plane wave along -x, A(phi) = a0 sin^2(pi phi/L)[sin(phi+phase0) e1 +
 *          cos(phi+phase0) e2 (circular only)], phi = t + x - phi_start in [0, L],
 *          L = 2 pi ncycles, e1 = (0, cos pol_angle, sin pol_angle), e2 = x_hat cross e1;
 *          E = -dA/dphi, B = -x_hat cross E.
 *  GAUSS : zeroth-order paraxial Gaussian pulse along -x focused at x_focus, waist w0,
 *          same envelope; E = a0 (w0/w) exp(-r^2/w^2) env [cos(Theta) e1 + sin(Theta) e2],
 *          Theta = phi + phase0 + Gouy - curvature phase; B = -x_hat cross E.
 *  GRID2D: six fp32 arrays [ny][nx] on a 2D Yee cell in the x-y plane, node (i,j) at
 *          (gx0 + i dx, gy0 + j dy); Ex (i+1/2,j), Ey (i,j+1/2), Ez (i,j), Bx (i,j+1/2),
 *          By (i+1/2,j), Bz (i+1/2,j+1/2); gathered with TSC weights (Sec. II.D-E), nodes
 *          outside the grid contribute zero.  nx >= 3, ny >= 1, at most 2^29 nodes.   */
typedef struct {
    int32_t kind, circular;
    double a0, ncycles, phase0, pol_angle, w0, x_focus, phi_start;
    double e0[3], b0[3];
    const float *grid[6];
    int32_t nx, ny;
    double dx, dy, gx0, gy0;
} qed_field;

/* a contiguous index range of one particle list under one field (one collision) */
typedef struct {
    int64_t begin, end;
    qed_field field;
} qed_segment;

/* Create a context and build the rate / spectrum / Bessel / birefringence tables on the
 * current device (FP64 quadrature, FP32 copies for QED_MIXED): the NCS rate and photon
 * spectrum integrals of eqs. (Wspin2) and (F0) (Sec. III.C.1), the NBW rate and pair
 * spectrum of eqs. (BW), (BWprob) (Sec. III.D), the birefringence coefficients of eq.
 * (eqnn) (Sec. III.F) and the radiative-correction factors of Sec. III.A.2 and III.B.2.
 * Synchronises `stream`.  The context owns every table (freed by qed_destroy).
 * Errors: QED_EARG (null pointers, non-positive dt or xi_L, unknown precision),
 * QED_ENOMEM, QED_EHIP; *ctx_out is NULL then.                                            */
qed_status qed_init_tables(qed_ctx_t **ctx_out, const qed_config *cfg, hipStream_t stream);
qed_status qed_destroy(qed_ctx_t *ctx);

/* Field gather (Sec. II.D-E: force at the particle from the grid with the TSC weights of
 * Sec. II.E; or the analytic pulse of qed_field): E6[6 i + (0..5)] = Ex, Ey, Ez, Bx, By, Bz
 * at x_i, t^n for leptons [0, *count) (doubles, caller-owned device buffer of 6 * capacity,
 * row per lepton).  Fields of lepton i come from the segment containing i (segments sorted
 * by begin; indices outside every segment see no field).  Errors: QED_EARG for a NULL
 * array or E6, bad segments or a capacity outside [0, 2^28].                             */
qed_status qed_gather(qed_ctx_t *ctx, const qed_segment *segs, int nseg, const qed_leptons *p,
                      double *E6, int64_t step, hipStream_t stream);
/* Boris push (Sec. II.A, eqs. boris1-boris6, leapfrog of Sec. II.F) and T-BMT rotation
 * (Sec. III.B, eqs. bmteqn, bmt-boris1-4) of leptons [0, *count), in place:
 * p^{n-1/2} -> p^{n+1/2}, S^{n-1/2} -> S^{n+1/2}, x^n -> x^{n+1}.  Fields from E6 (as
 * written by qed_gather) or, if E6 is NULL, gathered in the same kernel.  Momenta and
 * positions are FP64 in both precisions.  A non-finite result sets QED_ST_NAN.           */
qed_status qed_push_spin(qed_ctx_t *ctx, const qed_segment *segs, int nseg, qed_leptons *p,
                         const double *E6, int64_t step, hipStream_t stream);
/* qed_step_leptons for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same kernels and results,
 * with the event staging and scan work memory in a fixed device array of the library
 * (about 76 MB on every GPU the library runs on, held until the process ends) instead of
 * context-owned buffers.  Nothing is allocated or freed.  Limits: exactly one segment,
 * p->capacity <= QED_NOALLOC_MAX_LEPTONS (QED_EARG otherwise), the table sampler for NCS
 * (QED_ESTATE with the QED_SAMPLER_MLP bit set), the context's device current.  All calls on one
 * GPU share that array: calls that overlap on one GPU (other streams, other contexts,
 * other host threads) race and must not be made.                                       */
#define QED_NOALLOC_MAX_LEPTONS 524288
qed_status qed_step_leptons_noalloc(qed_ctx_t *ctx, const qed_segment *segs, int nseg, qed_leptons *p,
                                    qed_photons *out, int64_t step, hipStream_t stream);
/* Radiative push (Sec. III.A.3) and radiative T-BMT (Sec. III.B.3): the push of
 * qed_push_spin (fields gathered in the kernel) with, at the time-centred gamma^n =
 * sqrt(1+|p-|^2), beta^n = (p- + p+)/(2 gamma^n) and chi^n,
 *   QED_RR_LL  : p^{n+1/2} += F dt, F the Landau-Lifshitz force of eq. (eq1-1) (its two
 *                leading terms; the E(p.E) term with the 1/gamma of eq. (eq1));
 *   QED_RR_MLL : the same with g(chi^n) F, g the emitted / Larmor power ratio (Sec. III.A.2);
 *   QED_RR_RBMT: the spin gets dt/2 R(S) before and after the T-BMT rotation,
 *                R = -P [psi1 S + psi2 (S.beta) beta + psi3 b], P = alpha/(sqrt3 pi xi_L gamma),
 *                b = n x a of the NCS local frame; S then is a mean polarisation (|S| <= 1).
 * mode = 0 is qed_push_spin.  LL and MLL exclude each other (QED_EARG).  Deterministic: no
 * random numbers, no events.  chi beyond 1e3 sets QED_ST_CLAMP.                          */
enum { QED_RR_LL = 1, QED_RR_MLL = 2, QED_RR_RBMT = 4 };
qed_status qed_push_radiative(qed_ctx_t *ctx, const qed_segment *segs, int nseg, qed_leptons *p, uint32_t mode,
                              int64_t step, hipStream_t stream);
/* Nonlinear Compton step (Sec. III.C.1: event probability from eq. (Wspin2), photon energy
 * by inverse CDF of that spectrum, final spin along the SQA of the (w, f, g) form, photon
 * Stokes from eqs. (F0)-(F3); without an event the no-emission spin update) for leptons
 * [0, *count) already pushed in this step, using the fields E6 of x^n (required).  Photons
 * are appended to `out` (may be NULL: recoil and spin only) at x^{n+1}, in lepton order.
 * Uses the context's staging area (grown with hipMalloc to the list's capacity on first
 * use).                                                                                  */
qed_status qed_emit(qed_ctx_t *ctx, const qed_segment *segs, int nseg, qed_leptons *p,
                    const double *E6, qed_photons *out, int64_t step, hipStream_t stream);
/* Fused gather + push + T-BMT + NCS of leptons [0, *count) (Sec. II.A, II.D-E, III.B,
 * III.C.1, as qed_gather + qed_push_spin + qed_emit): a decide kernel over all leptons, a
 * scan of the event counts and an event kernel over the emitting leptons.               */
qed_status qed_step_leptons(qed_ctx_t *ctx, const qed_segment *segs, int nseg, qed_leptons *p,
                            qed_photons *out, int64_t step, hipStream_t stream);
/* Photon polarisation transport of the live photons [0, *count): rotation of the Stokes
 * vector to the frame of E_red (Sec. III.C.2, eq. rotation) and, if QED_PROC_VB, the
 * birefringent phase retardation (Sec. III.F, eqs. eqnn, rotation2; Algorithm 1).  Does
 * not move photons.                                                                      */
qed_status qed_birefringence(qed_ctx_t *ctx, const qed_segment *segs, int nseg, qed_photons *g,
                             int64_t step, hipStream_t stream);
/* Basis rotation (eq. rotation), NBW pair creation (Sec. III.D: event probability from eq.
 * (BWprob), pair energy by inverse CDF of eq. (BW), spins along the axes of eqs.
 * (BWposAxis), (BWeleAxis); if QED_PROC_NBW: pairs appended to em / ep in photon order at
 * the photon's position, the photon marked dead) and the straight-line move x += n dt of
 * surviving photons, for the live photons [0, *count).                                  */
qed_status qed_pair(qed_ctx_t *ctx, const qed_segment *segs, int nseg, qed_photons *g,
                    qed_leptons *em, qed_leptons *ep, int64_t step, hipStream_t stream);
/* Whole photon step in one kernel (= qed_birefringence then qed_pair, one rotation). */
qed_status qed_step_photons(qed_ctx_t *ctx, const qed_segment *segs, int nseg, qed_photons *g,
                            qed_leptons *em, qed_leptons *ep, int64_t step, hipStream_t stream);
/* One whole step of the electrons em, the positrons ep and the photons g (each may be
 * NULL) with the result of the paper's Spin-QED chain (Sec. IV): Lorentz push and T-BMT of
 * the leptons alive at the start of the step, VB and NBW of the photons alive at the start
 * of the step, NCS of the pushed leptons.  Pairs created in the step are placed at their
 * photon and first pushed, and tested for NCS, in step n + 1; photons emitted in the step
 * see VB and NBW from step n + 1 on; pair ids precede the step's photon ids.  On the
 * device the photon stage runs first (it records the lepton counts before its appends)
 * and the lepton stage covers only the leptons counted then; the two stages touch
 * disjoint particles, so the outcome is the chain's.  The photon stage needs nseg = 1.
 * Asynchronous; capturable like the calls it is made of.  Errors as those calls.        */
qed_status qed_step(qed_ctx_t *ctx, const qed_segment *segs, int nseg, qed_leptons *em, qed_leptons *ep,
                    qed_photons *g, int64_t step, hipStream_t stream);
/* Stable compaction of the live photons of `in` into `out` (distinct buffers): `out`
 * receives them in their order, count = number of live photons (its previous contents and
 * count are replaced).  Live photons beyond out's capacity are dropped and set
 * QED_ST_OVERFLOW.                                                                      */
qed_status qed_compact_photons(qed_ctx_t *ctx, const qed_photons *in, qed_photons *out,
                               hipStream_t stream);

/* ---------------------------------------------------------------- bremsstrahlung
 * High-energy bremsstrahlung of electrons in a target (Sec. III.E): the cross-section of
 * that section with the screening functions of Tsai's Thomas-Fermi fits (the paper's
 * choice for Z >= 5; lighter targets need tabulated scaled cross-sections and are
 * refused), a Coulomb correction, and the direct Monte Carlo of the free path.  The
 * material is one slab x_lo <= x < x_hi (all y, z) of n_atoms atoms of charge Z per
 * (c / omega_L)^3; photons below k_cut (m c^2; the paper's minimum-energy threshold) are not
 * produced.  Positrons (whose cross-section the paper scales by a factor from another
 * code) and Bethe-Heitler pair creation (not written out in the paper) are not covered. */
typedef struct qed_material {
    int32_t Z;            /* atomic number, 5..100                                          */
    int32_t reserved;
    double n_atoms;       /* atoms per (c / omega_L)^3                                      */
    double x_lo, x_hi;    /* the slab                                                       */
    double k_cut;         /* lowest photon energy produced (m c^2), 0 < k_cut < 1e6 - 1     */
} qed_material;
/* Tables of the material (FP64 on the device, with an FP32 copy): sigma(E) on 256 nodes of
 * ln E from ln((k_cut + 1)(1 + 1e-6)) to ln 4e6, and per node the cumulative cross-section
 * at 128 nodes of u in [0, 1], u mapping linearly to the logit ln(y / (1 - y)) of the photon
 * fraction y between y = k_cut / E and y = 1 - 1/E (8-point Gauss-Legendre per interval).
 * Allocates on first use (not capturable); replaces an earlier material.  EARG: Z outside
 * [5, 100], a non-positive density, an empty slab or k_cut out of range.                */
qed_status qed_brems_init(qed_ctx_t *ctx, const qed_material *m, hipStream_t stream);
/* Copies of the FP64 tables into device memory: sigma [256] (per atom, (c / omega_L)^2)
 * and the cumulative rows [256][128].  ESTATE without a material.                        */
qed_status qed_brems_tables(qed_ctx_t *ctx, double *sigma, double *cdf, hipStream_t stream);
/* One bremsstrahlung step over the electrons of em (charge -1).  An electron inside the
 * slab with total energy E emits with probability P = 1 - exp(-n sigma(E) |v| dt) (the
 * paper's free-path probability; sigma linear in ln E between nodes, 0 below the table,
 * the top node and QED_ST_CLAMP above 4e6 m c^2; QED_ST_PMAX when P > cfg.p_max), decided
 * by r[0] < P with r = the Philox draws of (id, step, stream 3).  The photon energy
 * k = y E: r[1] inverts the CDF of the two nodes around E mixed at E's weight (the last
 * node at or below r, u linear between nodes), y from u at E.  The photon, appended to g
 * in electron order with the next ids (past capacity: dropped, id consumed,
 * QED_ST_OVERFLOW), starts at the electron's position along its velocity with weight w,
 * unpolarised (xi = 0), e1 = unit(y_hat - (y_hat.n) n) (of z_hat when n is along y); the
 * electron keeps its direction with energy E - k.  Asynchronous; capturable once the
 * staging area covers em's capacity.  ESTATE without a material; EARG for bad lists.    */
qed_status qed_step_brems(qed_ctx_t *ctx, qed_leptons *em, qed_photons *g, int64_t step, hipStream_t stream);

/* Reordering of a list by grid bin (a data-layout step, no physics): the live particles
 * of `in` are written to `out` (distinct buffers, out->capacity >= in->capacity; out's
 * previous contents and count are replaced) sorted by the bin of their (x, y) on the grid
 * of `grid` (kind QED_FIELD_GRID2D; only nx, ny, dx, dy, gx0, gy0 are used): bins of
 * bin_cells x bin_cells cells, bx = floor((x - gx0) / (bin_cells dx)) clamped to
 * [0, nbx - 1] (NaN to 0), by likewise, key = by nbx + bx, at most 65536 bins.  The sort
 * is stable (particles of one bin keep their order) and the same on every run; dead
 * photons (alive = 0) are dropped, so the photon call also compacts.  Neighbouring
 * particles then share the cache lines of the TSC gather (Sec. II.D-E), which otherwise
 * bounds the step on grid fields.  It changes the order in which later appends (photons,
 * pairs in parent order) and their ids come out.  Context-owned work memory of 16 bytes
 * per particle of in's capacity plus 3 MB (hipMalloc on first use or growth).       */
qed_status qed_sort_photons(qed_ctx_t *ctx, const qed_photons *in, qed_photons *out, const qed_field *grid,
                            int32_t bin_cells, hipStream_t stream);
qed_status qed_sort_leptons(qed_ctx_t *ctx, const qed_leptons *in, qed_leptons *out, const qed_field *grid,
                            int32_t bin_cells, hipStream_t stream);

/* Boundaries of qed_field_advance.  open_x = 0: periodic in x.  open_x = 1: the first and
 * last node columns carry the first-order absorbing condition of Mur on Ey, Ez (one-way
 * wave equation of the outgoing field, discretised over the step between the boundary
 * node and its neighbour), and the pulse `incoming` (QED_FIELD_NONE, PW or GAUSS, a wave
 * along -x as in qed_field) enters through x_max: the condition there applies to E minus
 * the pulse, evaluated in FP64 at each node's staggered position.  (gx0, gy0): position of
 * node (0, 0); t0: time of the grid on entry.  y stays periodic.  The paper names boundary
 * and laser settings without an algorithm; this is the standard absorbing condition.    */
typedef struct {
    int32_t open_x, pad;
    qed_field incoming;
    double gx0, gy0, t0;
} qed_field_bc;

/* 2D field solver (Sec. II.B curl equations with z squeezed; leapfrog of Sec. II.F):
 * advances the six FP32 arrays of a GRID2D field ([ny][nx], the staggering of qed_field) in
 * place by `steps` steps of dt, each  B -= dt/2 curl E;  E += dt (curl B - J);
 * B -= dt/2 curl E  (E and B both at integer times for the gather), with periodic wrap in
 * y and, for bc NULL or bc->open_x = 0, in x.  `current` is NULL (vacuum) or three FP32
 * arrays Jx, Jy, Jz [ny][nx] at the staggering of Ex, Ey, Ez (as qed_deposit_current
 * writes them), held fixed over the steps.  dt must satisfy the Courant limit
 * dt < 1/sqrt(1/dx^2 + 1/dy^2) (QED_EARG otherwise); nx, ny >= 2 (nx >= 4 with open x).
 * Asynchronous on `stream`; 3 launches per step (5 with open x; the first open call
 * allocates 8 ny floats of context-owned memory).                                       */
qed_status qed_field_advance(qed_ctx_t *ctx, float *const grid[6], const float *const current[3],
                             const qed_field_bc *bc, int32_t nx, int32_t ny, double dx, double dy, double dt,
                             int64_t steps, hipStream_t stream);

/* Charge-conserving current deposition (Sec. II.C, Esirkepov's decomposition with the TSC
 * shapes of Sec. II.E).  Each source is a lepton list with the positions of its first *n0
 * particles at the start of the step (x0[0..2]: device FP64 arrays, caller-saved, e.g. by
 * qed_save_start; *n0: device scalar, the list's count then: particles appended during the
 * step start with the next one).  Those particles, moved to their current positions over
 * one step dt, ADD their current to `current` (three caller-owned device FP32 arrays
 * [ny][nx], not cleared: Jx at (i+1/2, j), Jy at (i, j+1/2), Jz at (i, j), node (i, j) at
 * (gx0 + i dx, gy0 + j dy), periodic in x and y).  A particle of weight w carries charge
 * Q = charge w qscale (qscale: the charge of a unit weight in the units of the field
 * equations); its current satisfies (rho1 - rho0)/dt + div J = 0 at every node with
 * rho = Q Sx Sy/(dx dy), so the solver keeps Gauss's law.  1 <= nsrc <= 4 (electrons and
 * positrons in one call cost one pass).  A move of a cell or more per axis, or a
 * non-finite position or weight, skips the particle and sets QED_ST_DEPOSIT.  nx, ny >= 2,
 * at most 2^29 nodes.
 * Grids of at most 8192 tiles of 32 x 32 nodes take a binned path: particles sorted by
 * tile, each tile summed in LDS in 64-bit fixed point (quantum 2^-32 of the largest
 * possible contribution of the call), the sums converted to FP32 and added to `current`
 * once per node, so the result is the same on every run.  It uses context-owned work
 * memory (tile counters; 56 bytes per lepton of the sources' capacities; a 64-bit copy of
 * the grid, 24 bytes per node), allocated with hipMalloc on first use or growth.  Larger
 * grids add each contribution with FP32 atomics (sums in an order that may change from
 * run to run).  Calls on one context must not overlap.                                   */
#define QED_DEPOSIT_MAX_SRC 4
#define QED_DEPOSIT_BINNED 0
#define QED_DEPOSIT_LOCAL 1
/* The tiled grids' path of later qed_deposit_current calls on this context.
 * QED_DEPOSIT_BINNED (default): the binned path above, for particles in any order.
 * QED_DEPOSIT_LOCAL: for lists kept in cell order (qed_sort_leptons every few steps): no
 * binning; each block of 256 consecutive particles of a source adds its contributions to
 * an LDS window over the box of its particles' start nodes (with the two-node halo) and
 * then the window's sums to the 64-bit grid; a block whose box exceeds 1024 nodes adds its
 * contributions to the 64-bit grid directly (slower, still exact).  The same fixed-point
 * contributions as the binned path, so the same J bit for bit; it needs no per-particle
 * work memory.  QED_EARG for another value; a host-side setting, no device work.          */
qed_status qed_set_deposit_path(qed_ctx_t *ctx, int path);
typedef struct {
    const qed_leptons *leptons;
    const double *x0[3];
    const int64_t *n0;
} qed_deposit_src;
qed_status qed_deposit_current(qed_ctx_t *ctx, const qed_deposit_src *src, int32_t nsrc, float *const current[3],
                               int32_t nx, int32_t ny, double dx, double dy, double gx0, double gy0, double dt,
                               double qscale, hipStream_t stream);
/* The start state qed_deposit_current needs: copies positions [0, count) of `l` into the
 * device FP64 arrays x0[0..2] (capacity entries each, caller-owned) and the count into the
 * device scalar *n0.  Asynchronous on `stream`; call it before the step that moves them.  */
qed_status qed_save_start(qed_ctx_t *ctx, const qed_leptons *l, double *const x0[3], int64_t *n0,
                          hipStream_t stream);

/* Detector diagnostics: the post-processing step of the VB algorithm (Sec. III.F) on the
 * device.  Particles [begin, count) heading to +x (p_x > 0; photons also alive) are
 * binned on two axes and, per bin, added to out[((b * n[0]) + a) * 5 + q] (caller-owned
 * device FP64 array of n[0] n[1] 5, not cleared):
 *   photons: w, w eps, w xi1', w xi2', w xi3' with xi' the Stokes vector rotated from the
 *            photon's basis (e1, n x e1) to the detector basis (d, n x d), d = unit part of
 *            pol_ref transverse to k (eq. rotation);
 *   leptons: w, w gamma, w Sx, w Sy, w Sz.
 * Axes: QED_AX_SLOPE_Y = p_y/p_x, QED_AX_SLOPE_Z = p_z/p_x, QED_AX_SLOPE_R =
 * sqrt(p_y^2+p_z^2)/p_x, each with bins floor((v - lo) n/(hi - lo)); QED_AX_ENERGY = |k| or
 * gamma on n <= 256 bins uniform in log10 between 10^lo and 10^hi (edges computed on the host
 * and compared against).  At most one energy axis; n[0] n[1] <= 2^24; lo < hi.  Sums use
 * floating-point atomics: counts of unit weights are exact, the other sums are correct to
 * rounding in an order that may change from run to run.  When the list holds at least four
 * particles per bin the blocks spread their atomics over 16 copies of the histogram
 * (context-owned device memory of 16 n[0] n[1] 5 doubles, at most 2^25, kept for later
 * calls; hipMalloc on first use or growth), added to `out` in copy order by a last launch.
 * Calls on one context must not overlap.                                                  */
enum { QED_AX_SLOPE_Y = 0, QED_AX_SLOPE_Z = 1, QED_AX_SLOPE_R = 2, QED_AX_ENERGY = 3 };
typedef struct {
    int32_t axis[2], n[2];
    double lo[2], hi[2];
    double pol_ref[3];
} qed_hist_spec;
qed_status qed_hist_photons(qed_ctx_t *ctx, const qed_photons *g, int64_t begin, const qed_hist_spec *h, double *out,
                            hipStream_t stream);
qed_status qed_hist_leptons(qed_ctx_t *ctx, const qed_leptons *l, int64_t begin, const qed_hist_spec *h, double *out,
                            hipStream_t stream);

/* Synchronises `stream`, returns the sticky status bits; qed_clear_status zeroes them. */
qed_status qed_read_status(qed_ctx_t *ctx, uint32_t *flags_out, hipStream_t stream);
qed_status qed_clear_status(qed_ctx_t *ctx, hipStream_t stream);
/* id counter (synchronises on read) */
qed_status qed_get_next_id(qed_ctx_t *ctx, uint64_t *next_id, hipStream_t stream);
qed_status qed_set_next_id(qed_ctx_t *ctx, uint64_t next_id, hipStream_t stream);
/* Copies a table (FP64 master) to host memory in the layout of the table specification:
 * BESSEL b1[NB] b2[NB] b3[NB]; NCS_RATE fa[NR] fk[NR]; NCS_CDF A[rows][cols] B[rows][cols];
 * NBW_RATE ga[NP] gk[NP]; NBW_CDF A B; VB Mplus[NV] Mminus[NV]; RAD g (1+chi)^(4/3) [NR],
 * psi1..3 (1+chi)^(7/3) / chi^3 [NR] each (NCS rate grid).  n must equal the size
 * returned by qed_table_size.                                                           */
int64_t qed_table_size(int which);
qed_status qed_table_export(qed_ctx_t *ctx, int which, double *host_out, int64_t n);
/* Optional timing of the NCS launches: with ev non-NULL, every later qed_step_leptons /
 * qed_emit call that runs NCS records ev[0] before its decide kernel, ev[1] after it,
 * ev[2] after the scan and ev[3] after the event kernel, on the call's stream.  The four
 * events belong to the caller (created with hipEventCreate, alive while set); the array
 * is copied.  NULL switches the recording off.                                         */
qed_status qed_set_step_events(qed_ctx_t *ctx, const hipEvent_t *ev);
/* Optional timing of the photon stage: with ev non-NULL, every later call that runs the
 * photon kernels (qed_step, qed_step_photons, qed_pair, qed_birefringence) records ev[0]
 * before its first photon kernel and ev[1] after its last, on the call's stream.  Events
 * and lifetime as for qed_set_step_events; NULL switches the recording off.             */
qed_status qed_set_photon_events(qed_ctx_t *ctx, const hipEvent_t *ev);
/* Batching and graph capture (many collisions as segments of one list, step loops
 * captured in a hipGraph).  With a device step counter registered, every later call uses
 * step + *dev_step as its step number, so one captured sequence of calls can be replayed
 * for consecutive steps; qed_advance_step adds `by` to the counter on the stream (a kernel,
 * capturable).  dev_step is caller-owned device memory (one int64); NULL unregisters.
 * Calls stay capturable as long as they do not grow the staging area or upload a new
 * segment list: make one call with the same list sizes and segments before capturing.
 * Captured graphs read the context's staging area and uploaded segment list in place, so
 * while a counter is registered a call that would replace the segment list or grow the
 * staging area is refused with QED_ESTATE (unregister first; graphs captured before such
 * a change must not be replayed after it).                                              */
qed_status qed_set_step_counter(qed_ctx_t *ctx, int64_t *dev_step);
qed_status qed_advance_step(qed_ctx_t *ctx, int64_t by, hipStream_t stream);
/* Current launch shape / set one (rejects unknown values). */
qed_status qed_get_tuning(qed_ctx_t *ctx, qed_tuning *out);
qed_status qed_set_tuning(qed_ctx_t *ctx, const qed_tuning *t);
/* Autotuner: times every launch shape on a copy of `p` (its first *count leptons, step
 * `step`, photons to a scratch list): one warm-up round, then `reps` rounds over all
 * shapes in turn, fastest time per shape; the context switches to the fastest shape if it
 * beats its current one by at least 3 %, and returns the result in `chosen` (may be NULL).  Leaves p, the id counter and the
 * status word as they were.  Synchronises, allocates and frees scratch memory: call it
 * outside graph capture, typically once per workload.                                  */
qed_status qed_autotune(qed_ctx_t *ctx, const qed_segment *segs, int nseg, const qed_leptons *p,
                        int64_t step, int reps, qed_tuning *chosen, hipStream_t stream);
/* ---- learned samplers (NCS and NBW) -------------------------------------------------
 * A 4-128-128-128-3 perceptron (SiLU after each hidden layer) per process and context.
 * NCS network (QED_NET_NCS), inputs of an emission: x0 = (log10 chi + 0.65)/2.35 (chi in
 * [1e-3, 50]), x1 = S.b, x2 = S.n (spin in the local frame of Sec. III.C.1), x3 = 2 r - 1
 * (the energy draw); outputs: y0 = t/40^(1/3) with t = (2u/(3 chi))^(1/3) the
 * photon-fraction variable of the spectrum tables, y1, y2 = the mean photon Stokes xi3, xi2
 * at that energy summed over the final spins (eqs. F0-F3).
 * NBW network (QED_NET_NBW), inputs of a pair creation (Sec. III.D): x0 = (log10 chi_gamma
 * - m) / h with m, h the centre and half width of log10 chi_gamma over [0.1, 50], x1 = xi3
 * (the photon's Stokes parameter in its basis e1), x2 = 0, x3 = 2 r - 1; outputs: y0 =
 * delta, the positron's energy fraction, y1, y2 = the mean positron and electron spin
 * along b = v x e1 at that delta with xi1 = xi2 = 0, summed over the partner's spin
 * (eqs. G0-G3).
 * Parameters: one flat FP32 vector of QED_MLP_NPARAM = 34051 numbers, W1 (4 x 128, row =
 * input), b1, W2 (128 x 128), b2, W3, b3, W4 (128 x 3), b4.  Inference runs on BF16
 * matrix cores with FP32 accumulation; training (gradient, Adam) in FP32.  The qed_mlp_*
 * calls and qed_sampler_table act on the network chosen by qed_mlp_select (QED_NET_NCS
 * by default).  All pointers below are device pointers unless stated; X is [n][4], Y / T
 * are [n][3] floats.                                                                   */
#define QED_MLP_NPARAM 34051
#define QED_NET_NCS 0
#define QED_NET_NBW 1
#define QED_SAMPLER_TABLE 0
#define QED_SAMPLER_MLP 1
#define QED_SAMPLER_MLP_NBW 2
/* the network the following qed_mlp_* / qed_sampler_table calls act on (QED_EARG for
 * another value); a host-side setting, no device work                                   */
qed_status qed_mlp_select(qed_ctx_t *ctx, int net);
/* fresh weights (uniform +-1/sqrt(fan-in) from Philox(seed)), zero biases and Adam state */
qed_status qed_mlp_init(qed_ctx_t *ctx, uint64_t seed, hipStream_t stream);
/* copy parameters in / out (QED_MLP_NPARAM floats each) */
qed_status qed_mlp_set_params(qed_ctx_t *ctx, const float *params, hipStream_t stream);
qed_status qed_mlp_get_params(qed_ctx_t *ctx, float *params_out, hipStream_t stream);
/* n training pairs from the library's FP64 tables: inputs drawn with Philox(seed) (NCS: chi
 * log-uniform on [1e-3, 50], isotropic spin, uniform draw; NBW: chi_gamma log-uniform on
 * [0.1, 50], xi3 uniform on [-1, 1], uniform draw), targets = the table sampler's t (delta)
 * and the exact spin-summed means at that energy, computed from the rounded X            */
qed_status qed_mlp_samples(qed_ctx_t *ctx, int64_t n, uint64_t seed, float *X, float *Y, hipStream_t stream);
/* inference: Y = net(X) */
qed_status qed_mlp_forward(qed_ctx_t *ctx, const float *X, float *Y, int64_t n, hipStream_t stream);
/* loss (1/n) sum_i sum_o w_o (net(X)_io - T_io)^2 into *loss_out (device float) and its
 * gradient into grad_out (QED_MLP_NPARAM floats, may be NULL); w is a host array of 3   */
qed_status qed_mlp_gradient(qed_ctx_t *ctx, const float *X, const float *T, int64_t n, const float *w,
                            float *grad_out, float *loss_out, hipStream_t stream);
/* one Adam step (beta 0.9, 0.999, eps 1e-8) on that gradient with learning rate lr */
qed_status qed_mlp_train_step(qed_ctx_t *ctx, const float *X, const float *T, int64_t n, const float *w, float lr,
                              float *loss_out, hipStream_t stream);
/* the table sampler on the same normalised inputs and outputs (tables of the context's
 * precision): the reference for the network's error and its fallback                */
qed_status qed_sampler_table(qed_ctx_t *ctx, const float *X, float *Y, int64_t n, hipStream_t stream);
/* which samplers later events use: QED_SAMPLER_TABLE (default), or the bits
 * QED_SAMPLER_MLP (NCS emissions: the network's t inside its trained chi range where
 * 0.5 <= t < t_max, the table elsewhere: below t = 0.5 the network's absolute error is a
 * large relative error in the photon energy u ~ t^3) and QED_SAMPLER_MLP_NBW (pair
 * creations: the network's delta inside its trained chi_gamma range where
 * 0.05 <= delta <= 0.95, the table elsewhere).  The final spins and the photon's Stokes
 * state are always drawn from the exact F / G at the sampled energy.  QED_ESTATE if the
 * network a bit asks for has no parameters.                                              */
qed_status qed_set_sampler(qed_ctx_t *ctx, int sampler);
/* Last argument / HIP error of this context as text (empty if none). */
const char *qed_last_error(const qed_ctx_t *ctx);

#ifdef __cplusplus
}
#endif
#endif
