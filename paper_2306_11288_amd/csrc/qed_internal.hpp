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
constexpr int64_t TAB_TOTAL = OFF_VB + 2 * NV;

template <class T>
struct Tabs {
    const T *base;
    __device__ __forceinline__ const T *bes() const { return base + OFF_BES; }
    __device__ __forceinline__ const T *ncs_rate() const { return base + OFF_NCS_RATE; }
    __device__ __forceinline__ const T *ncs_cdf() const { return base + OFF_NCS_CDF; }
    __device__ __forceinline__ const T *nbw_rate() const { return base + OFF_NBW_RATE; }
    __device__ __forceinline__ const T *nbw_cdf() const { return base + OFF_NBW_CDF; }
    __device__ __forceinline__ const T *vb() const { return base + OFF_VB; }
};

// ------------------------------------------------------------------ constants per context
struct Consts {
    double xi_L, alpha, a_e, dt, p_max;
    uint64_t seed;
    uint32_t procs;
};

// staging record of one event (decide kernel -> event kernel): particle index and the
// fields of x^n at which the event was decided
struct EventRec {
    long long idx;
    double f[6];
};

constexpr int MAX_SEG = 8;             // segments passed by value in kernel arguments
struct SegArgs {
    int nseg;
    qed_segment seg[MAX_SEG];
};

constexpr int BLOCK = 256;             // threads per block = particles per tile

}  // namespace qed

struct qed_ctx {
    qed_config cfg;
    int device;
    double *tab64;                     // FP64 master tables
    float *tab32;                      // FP32 copies (mixed precision)
    uint32_t *status;                  // sticky status word
    unsigned long long *next_id;       // id counter
    int *tile_counts;                  // events per 256-particle tile   [max_tiles]
    int64_t *tile_off;                 // exclusive prefix of tile_counts [max_tiles + 1]
    int64_t *launch;                   // bases of the last append launch [4]
    qed::EventRec *staging;            // one slot per particle of the largest list seen
    int64_t staging_cap;
    int64_t max_tiles;
    char err[256];
};

namespace qed {
// table construction (qed_tables.hip); returns hipSuccess or the first HIP error
hipError_t build_tables(qed_ctx *ctx, hipStream_t s);
// launches (qed_kernels.hip)
enum LeptonMode { LM_GATHER = 0, LM_PUSH = 1, LM_EMIT = 2, LM_FUSED = 3 };
hipError_t launch_leptons(qed_ctx *ctx, LeptonMode mode, const SegArgs &sa, const qed_leptons &L,
                          double *E6, const qed_photons *out, int64_t step, hipStream_t s);
enum PhotonMode { PM_BIREF = 0, PM_PAIR = 1, PM_FULL = 2 };
hipError_t launch_photons(qed_ctx *ctx, PhotonMode mode, const SegArgs &sa, const qed_photons &G,
                          const qed_leptons *em, const qed_leptons *ep, int64_t step, hipStream_t s);
hipError_t launch_compact(qed_ctx *ctx, const qed_photons &in, const qed_photons &out, hipStream_t s);
}  // namespace qed
