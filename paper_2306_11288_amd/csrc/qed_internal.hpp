// Internal declarations shared by the host ABI layer and the HIP kernels of libqed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "qed.h"

namespace qed {

// ------------------------------------------------------------------ table specification
// Grids are uniform in the stated variable ("ln" = natural log).  The CPU oracle builds
// the same specification with its own code; both must agree to rounding.
constexpr int NB = 2048;                 // Bessel: ln x in [ln 1e-15, ln 1e3]
constexpr double B_LO = -34.538776394910684, B_HI = 6.907755278982137;
constexpr int NR = 512;                  // NCS rates: ln chi in [ln 1e-6, ln 1e3]
constexpr double R_LO = -13.815510557964274, R_HI = 6.907755278982137;
constexpr int NCR = 512, NCT = 1024;     // NCS spectrum: rows ln chi in [ln 1e-5, ln 1e3], t in [0, 40^(1/3)]
constexpr double C_LO = -11.512925464970229, C_HI = 6.907755278982137;
constexpr double T_MAX = 3.4199518933533937;
constexpr int NP = 256;                  // NBW rates: ln chi in [ln 0.05, ln 1e3]
constexpr double P_LO = -2.995732273553991, P_HI = 6.907755278982137;
constexpr int NDR = 256, NDD = 512;      // NBW spectrum: rows as NBW rates, delta in [0, 1/2]
constexpr int NV = 1024;                 // VB: ln chi in [ln 1e-4, ln 1e3]
constexpr double V_LO = -9.210340371976182, V_HI = 6.907755278982137;

// element offsets inside one table allocation (same layout for the double and float copy)
constexpr int64_t OFF_BES = 0;                                   // [NB][4]  b1 b2 b3 0
constexpr int64_t OFF_NCS_RATE = OFF_BES + 4 * NB;                // [NR][2]  fa fk
constexpr int64_t OFF_NCS_CDF = OFF_NCS_RATE + 2 * NR;            // [NCR][NCT][2] A B
constexpr int64_t OFF_NBW_RATE = OFF_NCS_CDF + 2LL * NCR * NCT;   // [NP][2]  ga gk
constexpr int64_t OFF_NBW_CDF = OFF_NBW_RATE + 2 * NP;            // [NDR][NDD][2] A B
constexpr int64_t OFF_VB = OFF_NBW_CDF + 2LL * NDR * NDD;         // [NV][2]  M+ M-
constexpr int64_t OFF_RAD = OFF_VB + 2 * NV;                      // [NR][4]  g (1+chi)^(4/3),
                                                                  //          psi1..3 (1+chi)^(7/3) / chi^3
constexpr int64_t TAB_TOTAL = OFF_RAD + 4 * NR;
// FP32 copy only, after the shared layout: the two spectrum CDFs again with each pair of
// adjacent rows interleaved, entry [r][col] = {A_r, B_r, A_r+1, B_r+1} (the same rounded
// values), so an inverse-CDF probe, which mixes rows r and r+1, is one 16-byte load
constexpr int64_t OFF_NCS_CDF_PAIR = TAB_TOTAL;                                  // [NCR-1][NCT][4]
constexpr int64_t OFF_NBW_CDF_PAIR = OFF_NCS_CDF_PAIR + 4LL * (NCR - 1) * NCT;  // [NDR-1][NDD][4]
constexpr int64_t TAB32_TOTAL = OFF_NBW_CDF_PAIR + 4LL * (NDR - 1) * NDD;
static_assert(TAB_TOTAL % 4 == 0, "paired rows must start 16-byte aligned");

template <class T>
struct Tabs {
    const T *base;
    __device__ __forceinline__ const T *bes() const { return base + OFF_BES; }
    __device__ __forceinline__ const T *ncs_rate() const { return base + OFF_NCS_RATE; }
    __device__ __forceinline__ const T *ncs_cdf() const { return base + OFF_NCS_CDF; }
    __device__ __forceinline__ const T *nbw_rate() const { return base + OFF_NBW_RATE; }
    __device__ __forceinline__ const T *nbw_cdf() const { return base + OFF_NBW_CDF; }
    __device__ __forceinline__ const T *vb() const { return base + OFF_VB; }
    __device__ __forceinline__ const T *rad() const { return base + OFF_RAD; }
    // FP32 tables only (T = float)
    __device__ __forceinline__ const float4 *ncs_cdf_pair() const { return (const float4 *)(base + OFF_NCS_CDF_PAIR); }
    __device__ __forceinline__ const float4 *nbw_cdf_pair() const { return (const float4 *)(base + OFF_NBW_CDF_PAIR); }
};

// ------------------------------------------------------------------ bremsstrahlung
// Tables of one material: sigma(E) on BR_NE nodes of ln E in [ln E_lo, ln BR_E_HI]
// (E_lo = (k_cut + 1)(1 + 1e-6)), then the cumulative integrals C_j(u_i) of each node on
// BR_NU nodes of u in [0, 1] (row-major).  u maps to the logit t = ln(y / (1 - y)) of the
// photon fraction y linearly between logit(k_cut / E) and ln(E - 1).
constexpr int BR_NE = 256, BR_NU = 128;
constexpr double BR_E_HI = 4.0e6;
constexpr int64_t BR_TAB_LEN = BR_NE + (int64_t)BR_NE * BR_NU;
struct BremsDev {
    double Z, lnZ, z13, z23, f;        // Z, ln Z, Z^(1/3), Z^(2/3), Coulomb correction
    double n_atoms, x_lo, x_hi, k_cut; // atoms per (c / omega_L)^3, target slab in x, photon cut
    double ar02;                       // alpha r0^2, r0 = alpha xi_L (c / omega_L units)
    double lnE0, lnE_hi, inv_dlnE;     // table energy range
};

// ------------------------------------------------------------------ constants per context
struct Consts {
    double xi_L, alpha, a_e, dt, p_max;
    double c_ncs;      // alpha / (sqrt3 pi xi_L): NCS rate prefactor times gamma
    uint64_t seed;
    uint32_t procs;
    float f_a_e, f_half_dt;   // a_e and dt/2 rounded to single precision
};

// A field as the kernels use it: the quantities that are uniform over a segment
// (polarisation axes, pi/L, Rayleigh length, inverse grid spacings) are computed once on
// the host, so the per-particle code has no uniform transcendental or division.  Kernels of
// the hot path are specialised on the field kind, so only one kind's members are read.
struct PulseDev {                // QED_FIELD_PW, QED_FIELD_GAUSS
    double a0, phase0, phi_start, L, pi_over_L;
    double inv_L, inv_2L;        // 1/L, 1/(2L): the envelope phases in revolutions
    double cp, sp;               // e1 = (0, cp, sp), e2 = (0, -sp, cp)
    double x_focus, zr, inv_zr, w0sq, inv_w0sq;
    // single-precision copies for the FP32 pulse (rounded once here: uniform conversions
    // in a kernel would run on the vector unit of every wave)
    float f_a0, f_pi_over_L, f_cp, f_sp, f_zr, f_inv_zr, f_inv_w0sq;
};
struct GridDev {                 // QED_FIELD_GRID2D
    const float *g[6];
    int32_t nx, ny;
    double inv_dx, inv_dy, gx0, gy0;
};
struct ConstDev {                // QED_FIELD_CONST
    double e0[3], b0[3];
};
struct FieldDev {
    int32_t kind, circular;
    PulseDev p;
    GridDev g;
    ConstDev c;
};
constexpr int FK_MULTI = -1;     // kernel template argument: field kind read per segment
constexpr int FK_MULTI_BASE = 16;  // FK_MULTI_BASE + kind: several segments, all of that kind
struct DevSegment {
    int64_t begin, end;
    FieldDev f;
};

// staging record of one event of the compaction or bremsstrahlung kernels (decide kernel ->
// event kernel): particle index and up to six values the event needs
struct EventRec {
    long long idx;
    double f[6];
};
// staging record of one lepton event: the state the decide kernel reached for it (index,
// id, weight, x^{n+1}, p^{n+1/2}, fields of x^n, S^{n+1/2} after the T-BMT rotation)
template <class T>
struct LepEvent {
    int64_t i;
    unsigned long long id;
    double w;
    double r[3], p[3], E[3], B[3];
    T S[3];
};

// Field selection for a launch.  One segment: its field travels in the kernel arguments
// and is read at constant offsets.  Several segments: they live in a device buffer owned
// by the context and each particle finds its own by binary search on `begin` (indexing
// an argument array at run time would copy it to private memory in every thread).
constexpr int MAX_SEG = 1 << 16;
struct SegArgs {
    int nseg;
    int multi_kind;            // nseg > 1: the kind every segment has, or -1 if they differ
    int64_t begin0, end0;
    FieldDev f0;
    const DevSegment *segs;    // device copy when nseg > 1
    const int64_t *seg_begin;  // the segments' starts, compact (same allocation)
    const int32_t *tile_seg;   // per 256-particle tile: segment of its first index (or the last
                               // before it) in the low bits, SEG_NONE / SEG_MIXED flags above
    int64_t ntile_seg;
};
// tile table entries: the segment index, and whether the tile's indices all lie in no
// segment (SEG_NONE) or not all in that one segment (SEG_MIXED: across a boundary or a gap)
constexpr int32_t SEG_INDEX = 0xffff, SEG_NONE = 1 << 29, SEG_MIXED = 1 << 30;
FieldDev field_dev(const qed_field &f);   // host: derived constants of a field

// learned sampler: 4-128-128-128-3 perceptron, flat FP32 parameters W1 b1 W2 b2 W3 b3 W4 b4
constexpr int MLP_OW1 = 0, MLP_OB1 = 512, MLP_OW2 = 640, MLP_OB2 = 17024, MLP_OW3 = 17152, MLP_OB3 = 33536,
              MLP_OW4 = 33664, MLP_OB4 = 34048, MLP_NPARAM = 34051;
// input normalisation: x0 = (log10 chi - MID) / HALF over the trained range chi in [1e-3, 50]
constexpr double MLP_L10_MID = -0.65, MLP_L10_HALF = 2.35, MLP_L10_HI = 1.6989700043360187;
// below this t (in units of T_MAX) the network's absolute error is a large relative error
// in the photon energy u ~ t^3, and the step takes t from the table
constexpr float MLP_Y_LO = 0.5f / 3.4199518933533937f;
constexpr double MLP_CHI_LO = 1e-3, MLP_CHI_HI = 50.0;
// the NBW network: chi_gamma in [0.1, 50] (pair creation below 0.1 is suppressed by
// exp(-8 / (3 chi)) < 3e-12), x0 = (log10 chi - MID) / HALF; its delta is used inside
// [MLP_D_LO, 1 - MLP_D_LO], where an absolute error is a small relative one in both
// members' energies, the table's elsewhere
constexpr double MLP_NBW_L10_LO = -1.0, MLP_NBW_L10_HI = 1.6989700043360187;
constexpr double MLP_NBW_L10_MID = 0.5 * (MLP_NBW_L10_LO + MLP_NBW_L10_HI),
                 MLP_NBW_L10_HALF = 0.5 * (MLP_NBW_L10_HI - MLP_NBW_L10_LO);
constexpr double MLP_NBW_CHI_LO = 0.1, MLP_NBW_CHI_HI = 50.0;
constexpr float MLP_D_LO = 0.05f;
// one network per process: QED_NET_NCS (0), QED_NET_NBW (1)
constexpr int MLP_NETS = 2;
struct MlpNet {
    float *P, *m, *v, *G;              // parameters, Adam moments, gradient [MLP_NPARAM]
    void *WT;                          // bf16 transposed W2, W3 for the forward kernel
    float *W32;                        // FP32 transposed W2, W3 for the backward pass
    int t;                             // Adam step count
};

// detector histogram launch (one energy axis at most, HIST_EMAX bins on it)
constexpr int HIST_EMAX = 256;
struct HistArgs {
    qed_photons G;
    qed_leptons L;
    int64_t begin;
    int32_t axis[2], n[2];
    double lo[2], inv_w[2];       // linear axes: bin = floor((v - lo) inv_w), inv_w = n / (hi - lo)
    double pol_ref[3];
    int32_t eaxis;                // index of the energy axis, or -1
    double *out;
    double *acc;                  // replicas [rep][bins][5] when rep > 1 (then added to out)
    int32_t rep;
    int64_t rep_stride;
    double edges[HIST_EMAX + 1];  // energy axis: 10^(lo + k (hi - lo)/n), k = 0..n
};

constexpr int BLOCK = 256;             // threads per block = particles per tile
constexpr int EV_GROUP_MAX = 16;       // lepton step: largest tiles-per-group of the event kernel

// photon (pair) event record: what the decide kernel reached for a converting photon (its
// momentum and place, chi, kappa, the two draws the pair needs, Stokes vector and basis
// after this step's rotation)
template <class T>
struct PhotonEvent {
    double k[3], x[3];
    double chi, r0, r2;
    T xi[3], e1[3], kappa;
};

// photon stage: pair events are counted per group of PH_GROUP tiles and per 64 groups
// (lists of at most 2^28 photons)
constexpr int PH_GROUP = 32;
constexpr int64_t PH_GROUPS_MAX = ((int64_t)1 << 20) / PH_GROUP + 1;
constexpr int64_t PH_SUPER_MAX = PH_GROUPS_MAX / 64 + 1;
constexpr int64_t PH_TOT_LEN = 2 * PH_GROUPS_MAX + 2 * PH_SUPER_MAX + 3;

// bytes of one staging slot: the largest record any kernel parks there
constexpr size_t STAGING_SLOT = sizeof(LepEvent<double>) > sizeof(EventRec) ? sizeof(LepEvent<double>)
                                                                             : sizeof(EventRec);
// a photon event sits in bytes [8, ...) of the converting photon's own slot, the photon
// index of the event of rank r in bytes [0, 8) of slot r: the two never overlap
static_assert(8 + sizeof(PhotonEvent<double>) <= STAGING_SLOT, "a photon event fits a staging slot");

}  // namespace qed

struct qed_ctx {
    qed_config cfg;
    int device;
    double *br_tab64;                  // bremsstrahlung tables of the material (null: none)
    float *br_tab32;
    qed::BremsDev br;
    double *tab64;                     // FP64 master tables
    float *tab32;                      // FP32 copies (mixed precision)
    uint32_t *status;                  // sticky status word
    unsigned long long *next_id;       // id counter
    int *tile_counts;                  // events per 256-particle tile   [max_tiles]
    int *ph_tot;                       // photon stage: pair events per group of PH_GROUP tiles
                                       // [2][PH_GROUPS_MAX], then per 64 groups [2][PH_SUPER_MAX]
                                       // (two parities), the parity and the groups each used [3]
    int *group_tot;                    // events per group of ev_group tiles [max_tiles / 4 + 1];
                                       // zero between launches (the scan clears what it reads)
    int64_t *tile_off;                 // exclusive prefix of tile_counts [max_tiles + 1]
    int64_t *launch;                   // bases of the last append launch [8]: out0, out1, id, events;
                                       // [4] the photon stage's parity
    int64_t *scan_sums;                // block totals of the prefix scan [SCAN_MAX_BLOCKS]
    int64_t *lep_start;                // lepton counts before the pair appends of qed_step [2]
    void *na_scratch;                  // device address of this device's allocation-free scratch array
    void *staging;                     // one STAGING_SLOT per particle of the largest list seen,
    int64_t staging_cap;               // rounded up to whole tiles
    qed::DevSegment *dsegs;            // device copy of the last multi-segment list
    qed::DevSegment *hsegs;            // pinned host staging of that copy
    int nseg_dev;                      // segments in the uploaded list
    size_t seg_bytes, seg_cap_bytes;   // bytes of the uploaded list (with its tile table), capacity
    hipEvent_t seg_copied;             // completion of the last upload
    int64_t max_tiles;
    hipEvent_t step_ev[4];             // optional timing events of the NCS launches
    int step_ev_on;
    hipEvent_t ph_ev[2];               // optional timing events around each photon stage
    int ph_ev_on;
    int64_t *step_dev;                 // optional device step counter (caller-owned)
    int num_cu;                        // compute units of the device
    qed_tuning tune;                   // launch shape of the lepton step (qed_autotune)
    // learned samplers
    qed::MlpNet nets[qed::MLP_NETS];   // the NCS and the NBW network
    int mlp_sel;                       // the network the qed_mlp_* calls act on
    float *mlp_work;                   // training work buffers
    int64_t mlp_work_len;
    int sampler;                       // QED_SAMPLER_TABLE, or bits QED_SAMPLER_MLP (NCS), QED_SAMPLER_MLP_NBW
    float *ev_in, *ev_out;             // learned sampler: per-event network inputs [ev_cap][4], outputs [ev_cap][3]
    double *hist_rep;                  // detector histogram replicas
    int64_t hist_rep_len;
    int dep_path;                      // QED_DEPOSIT_BINNED or QED_DEPOSIT_LOCAL (qed_set_deposit_path)
    int *dep_cnt;                      // current deposition: tile counts, offsets, cursors (zero between calls)
    void *dep_work;                    // chunk work list
    void *dep_rec;                     // particle records sorted by tile
    int64_t dep_cap;                   // particles the records can hold
    void *dep_acc;                     // 64-bit fixed-point current grid (zero between calls)
    int64_t dep_acc_len;
    void *sort_work;                   // particle sort: keys, indices, digit counts and offsets
    int64_t sort_cap;                  // particles the sort work memory holds
    float *yee_save;                   // open-boundary columns of the field solver
    int64_t yee_save_len;
    int64_t ev_cap;
    char err[256];
};

namespace qed {
// the work memory of one ordered-append launch sequence (decide -> scan -> events)
struct ScanState {
    void *staging;         // one STAGING_SLOT per particle
    int *tile_counts;      // events per tile
    int *group_tot;        // events per event group (zero between launches)
    int64_t *tile_off;     // exclusive prefix of the counts
    int64_t *launch;       // bases of the launch [4]
    int64_t *sums;         // block totals of the scan [SCAN_MAX_BLOCKS]
};
constexpr int SCAN_MAX_BLOCKS = 64;   // blocks of the prefix scan
// table construction (qed_tables.hip); returns hipSuccess or the first HIP error
hipError_t build_tables(qed_ctx *ctx, hipStream_t s);
Consts consts_of(const qed_ctx *ctx);     // the per-launch constants of the context's configuration
// bremsstrahlung (Sec. III.E): tables of the context's material (ctx->br), then the step
hipError_t build_brems_tables(qed_ctx *ctx, hipStream_t s);
hipError_t launch_brems(qed_ctx *ctx, const qed_leptons &L, const qed_photons &G, int64_t step, hipStream_t s);
// ordered append of per-tile event counts of a list to one output list (ids per event)
hipError_t launch_scan_events(qed_ctx *ctx, const int64_t *in_count, int64_t in_cap, const int *counts, int64_t *c0,
                              int64_t cap0, int ids, hipStream_t s);
// launches (qed_kernels.hip)
enum LeptonMode { LM_GATHER = 0, LM_PUSH = 1, LM_EMIT = 2, LM_FUSED = 3 };
// n_in (device scalar, optional): the launch covers leptons [0, *n_in) instead of [0, *L.count)
// ss (optional): work memory to use instead of the context's
hipError_t launch_leptons(qed_ctx *ctx, LeptonMode mode, const SegArgs &sa, const qed_leptons &L,
                          double *E6, const qed_photons *out, int64_t step, hipStream_t s,
                          const int64_t *n_in = nullptr, const ScanState *ss = nullptr);
// allocation-free lepton step (qed_noalloc.hip): the file-scope scratch array of the current
// device (its address taken once per device), its size limit, and the clearing of the part
// that must start at zero
constexpr int64_t NOALLOC_MAX = QED_NOALLOC_MAX_LEPTONS;   // leptons per call
static_assert(NOALLOC_MAX % BLOCK == 0, "whole tiles");
hipError_t noalloc_scratch(void **ptr);
ScanState noalloc_state(void *scratch);
hipError_t noalloc_clear(const ScanState &ss, hipStream_t s);
enum PhotonMode { PM_BIREF = 0, PM_PAIR = 1, PM_FULL = 2 };
// lep_start (device [2], optional): receives the counts of em / ep before the pair appends
hipError_t launch_photons(qed_ctx *ctx, PhotonMode mode, const SegArgs &sa, const qed_photons &G,
                          const qed_leptons *em, const qed_leptons *ep, int64_t step, hipStream_t s,
                          int64_t *lep_start = nullptr);
hipError_t launch_compact(qed_ctx *ctx, const qed_photons &in, const qed_photons &out, hipStream_t s);
// exclusive prefix of n ints (counts) into off[0..n], the total also into *total and
// launch[3] (launch: 4 int64 of scratch)
hipError_t launch_scan_ints(qed_ctx *ctx, const int *counts, int64_t n, int64_t *off, int64_t *total,
                            int64_t *launch, hipStream_t s);
// particle sort by grid bin (qed_sort.hip): the key of every particle, then two stable
// counting-sort passes over 8-bit digits, then the gather into the output list
struct SortGrid {
    double gx0, gy0, inv_bx, inv_by;   // bin of (x, y): floor((x - gx0) inv_bx), clamped
    int32_t nbx, nby;
};
hipError_t launch_sort_photons(qed_ctx *ctx, const qed_photons &in, const qed_photons &out, const SortGrid &g,
                               hipStream_t s);
hipError_t launch_sort_leptons(qed_ctx *ctx, const qed_leptons &in, const qed_leptons &out, const SortGrid &g,
                               hipStream_t s);
hipError_t launch_advance_step(int64_t *step, int64_t by, hipStream_t s);
hipError_t launch_radiative(qed_ctx *ctx, const SegArgs &sa, const qed_leptons &L, uint32_t mode, int64_t step,
                            hipStream_t s);
// 2D Yee solver (qed_fdtd.hip): steps of dt, optional current J (NULL: vacuum), periodic
// or (bc) open in x with an incoming pulse
struct YeeBoundary {
    FieldDev inc;          // kind QED_FIELD_NONE: no injection
    double gx0, gy0, t0;
};
hipError_t launch_yee(qed_ctx *ctx, float *const g[6], const float *const J[3], const YeeBoundary *bc, int nx, int ny,
                      double dx, double dy, double dt, int64_t steps, hipStream_t s);
// positions and count of a lepton list at the start of a step (qed_deposit.hip)
hipError_t launch_save_start(qed_ctx *ctx, const qed_leptons &L, double *const x0[3], int64_t *n0, hipStream_t s);
// current deposition (qed_deposit.hip): for each source, leptons [0, *n0) from x0 to their
// current position
constexpr int DEP_MAX_SRC = QED_DEPOSIT_MAX_SRC;
hipError_t launch_deposit(qed_ctx *ctx, const qed_deposit_src *src, int nsrc, float *const J[3], int nx, int ny,
                          double dx, double dy, double gx0, double gy0, double dt, double qscale, hipStream_t s);
// detector histograms (qed_detector.hip)
hipError_t launch_hist(qed_ctx *ctx, const HistArgs &a, bool photons, int64_t capacity, hipStream_t s);
// learned sampler (qed_mlp.hip)
// (the network is ctx->nets[ctx->mlp_sel] except where one is passed; samples and the
// table sampler follow the selected network's process)
hipError_t mlp_alloc(MlpNet &N);
void mlp_free(MlpNet &N);
hipError_t mlp_init(qed_ctx *ctx, uint64_t seed, hipStream_t s);
hipError_t mlp_pack(MlpNet &N, hipStream_t s);
hipError_t mlp_samples(qed_ctx *ctx, int64_t n, uint64_t seed, float *X, float *Y, hipStream_t s);
hipError_t mlp_forward(qed_ctx *ctx, const MlpNet &N, const float *X, float *Y, int64_t n, const int64_t *n_dev,
                       int64_t n_max, hipStream_t s);
hipError_t mlp_grad(qed_ctx *ctx, const float *X, const float *T, int64_t n, const float w[3], float *loss,
                    hipStream_t s);
hipError_t mlp_train(qed_ctx *ctx, const float *X, const float *T, int64_t n, const float w[3], float lr,
                     float *loss, hipStream_t s);
hipError_t table_sampler_run(qed_ctx *ctx, const float *X, float *Y, int64_t n, hipStream_t s);
}  // namespace qed
