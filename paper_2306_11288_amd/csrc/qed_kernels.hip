// HIP kernels of the QED particle step for gfx950 and their host launchers.
//
// Every step that can create particles runs as three launches on the caller's stream:
//   1. decide  (one thread per particle, 256-particle tiles = blocks): gather, push, spin,
//      event test; particles without an event are finished here.  Event particles are
//      ranked inside their tile with a wavefront ballot + popcount (waves combined in
//      LDS) and leave a 56-byte record (index, E, B) in a staging slot tile*256 + rank;
//      the tile's event count goes to tile_counts[tile].
//   2. scan    (one block): exclusive prefix sum of the tile counts, launch bases (output
//      list counts, id counter) and the new counts / id counter.
//   3. events  (one thread per event, dense): finish each event from its record and write
//      the new particle(s) at base + global rank.
// The output order is the parent index order and the result is independent of thread
// scheduling; there are no atomics on the data path and no inter-block waits, and the
// event work (inverse-CDF search, spin and Stokes algebra) runs without divergence.
#include "qed_dev.hpp"

namespace qed {

// ------------------------------------------------------------------------- segments
// Lanes of a wavefront over several segments: a waterfall from segment lo (the segment of
// the wavefront's first tile index, or the last one before it): the lanes inside the
// current segment evaluate its field (the descriptor comes through scalar loads and its
// kind is uniform); if lanes remain, the first of them picks the next segment by a search on
// wavefront-uniform values.  KIND < 0: the kind is read from each segment.
template <class FT, int KIND>
__device__ __forceinline__ void fields_waterfall(const SegArgs &sa, int64_t i, double t, const V3<double> &r,
                                                 int lo, V3<double> &E, V3<double> &B) {
    bool done = false;
    for (;;) {
        const DevSegment &sg = sa.segs[lo];
        if (!done && i >= sg.begin && i < sg.end) {
            if constexpr (KIND < 0) field_at<FT>(sg.f, t, r.x, r.y, r.z, E, B);
            else field_kind<FT, KIND>(sg.f, t, r.x, r.y, r.z, E, B);
            done = true;
        }
        const unsigned long long pending = __ballot(!done);
        if (pending == 0) break;
        const int leader = __ffsll((long long)pending) - 1;
        const int il = __builtin_amdgcn_readlane((int)i, leader);
        int a = 0, b = sa.nseg - 1;   // last segment with begin <= il
        while (a < b) {
            const int mid = (a + b + 1) >> 1;
            if (sa.seg_begin[mid] <= il) a = mid;
            else b = mid - 1;
        }
        if (a == lo) {                // the leader lies outside every segment: no field
            if ((int)i == il) done = true;
            if (__ballot(!done) == 0) break;
            continue;
        }
        lo = a;
    }
}

// FK: the kind of the single segment (fields read at constant offsets of the kernel
// arguments), FK_MULTI (several segments, kind read from each) or FK_MULTI_BASE + kind
// (several segments of that one kind).  Segments are index ranges and a wavefront holds
// consecutive indices, so it almost always lies in one segment: with several segments the
// tile's table entry (read after the particle loads are on their way) tells; for
// FK_MULTI_BASE + kind a tile inside one segment or one gap takes straight-line code with no
// per-lane test, only a SEG_MIXED tile (across a boundary or a gap edge) the waterfall.
template <class FT, int FK>
__device__ __forceinline__ void fields_for(const SegArgs &sa, int64_t i, double t, const V3<double> &r,
                                           V3<double> &E, V3<double> &B) {
    E = {0, 0, 0};
    B = {0, 0, 0};
    if constexpr (FK != FK_MULTI && FK < FK_MULTI_BASE) {
        if (i >= sa.begin0 && i < sa.end0) field_kind<FT, FK>(sa.f0, t, r.x, r.y, r.z, E, B);
    } else {
        const int t0 = __builtin_amdgcn_readfirstlane((int)i) / BLOCK;
        const int32_t seg = t0 < sa.ntile_seg ? sa.tile_seg[t0] : (sa.nseg - 1) | SEG_MIXED;
        if constexpr (FK == FK_MULTI) {
            fields_waterfall<FT, -1>(sa, i, t, r, seg & SEG_INDEX, E, B);
        } else if (seg & SEG_MIXED) {
            fields_waterfall<FT, FK - FK_MULTI_BASE>(sa, i, t, r, seg & SEG_INDEX, E, B);
        } else if (!(seg & SEG_NONE)) {
            field_kind<FT, FK - FK_MULTI_BASE>(sa.segs[seg & SEG_INDEX].f, t, r.x, r.y, r.z, E, B);
        }
    }
}

// ------------------------------------------------------------------------- scan kernel
struct ScanArgs {
    const int *counts;        // events per unit (a 256-particle tile)
    int64_t *off;             // [nunits + 1]: exclusive prefix
    const int64_t *in_count;  // list whose units were counted (null: in_capacity particles)
    int64_t in_capacity;
    int unit;                 // particles per unit
    int64_t chunk;            // units per block (a multiple of SCAN_THREADS)
    int64_t *out_count[2];    // output lists (may be null)
    int64_t out_cap[2];
    unsigned long long *next_id;
    int ids_per_event;        // 0 (compaction), 1 (photon), 2 (pair)
    int zero_base;            // output lists are replaced, not appended to (compaction)
    int64_t *base_out;        // optional [2]: receives the output counts before the append
    int64_t *launch;          // [0] out0 base, [1] out1 base, [2] id base, [3] events
    int64_t *sums;            // [SCAN_MAX_BLOCKS]: total of each block
    int clear;                // set the counts to zero once read (accumulated by atomics)
    uint32_t *status;
};
constexpr int SCAN_THREADS = 256, SCAN_MIN_CHUNK = 2048, SCAN_ONE_THREADS = 1024;
// units a single block scans: up to eight per thread, all held in registers; a longer run
// per thread strides through memory (39k tile counts took 65 us in one block, 11 us in the
// two-launch form)
constexpr int64_t SCAN_ONE_BLOCK = 8 * SCAN_ONE_THREADS;
static_assert(SCAN_MAX_BLOCKS <= SCAN_THREADS, "one block total per thread");

// sum over the block of NT threads (every thread gets it)
template <int NT>
__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t *s_w) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    __syncthreads();
    if (lane == 0) s_w[wid] = v;
    __syncthreads();
    int64_t t = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) t += s_w[w];
    return t;
}

// The unit counts a thread owns: `per` consecutive units from t0 (fewer at the end),
// loaded eight at a time so that the loads of a batch are in flight together.
__device__ __forceinline__ int64_t run_sum(const int *c, int64_t t0, int64_t per, int64_t nunits) {
    int64_t sum = 0;
    for (int64_t b = 0; b < per; b += 8) {
        int v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t u = t0 + b + k;
            v[k] = (b + k < per && u < nunits) ? c[u] : 0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) sum += v[k];
    }
    return sum;
}
__device__ __forceinline__ int64_t scan_units(const ScanArgs &a, int64_t &nunits) {
    const int64_t n = a.in_count ? clamp_count(a.in_count, a.in_capacity) : a.in_capacity;
    nunits = (n + a.unit - 1) / a.unit;
    return nunits > 0 ? (nunits - 1) / a.chunk : 0;   // the block holding the last unit
}

// Exclusive prefix sums of the unit counts and the launch bases.  A list of at most
// SCAN_ONE_BLOCK (8192) units is scanned by one block of 1024 threads in one launch.  A longer one
// takes two launches over blocks of 256 threads and `chunk` units: k_scan_sums writes each
// block's total, k_scan then gives block b the total of blocks [0, b) (at most
// SCAN_MAX_BLOCKS values).  In k_scan each thread owns a run of chunk / threads units
// (wave shuffles, then the waves through LDS) and writes their offsets; the block holding
// the last unit also writes the total, the launch bases, the new output counts and the id
// counter.  With `clear`, k_scan zeroes the units it read (only its own block's: no other
// block of k_scan reads them), so counts accumulated by atomics start at zero next time.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_sums(ScanArgs a) {
    __shared__ int64_t s_w[SCAN_THREADS / 64];
    int64_t nunits;
    const int64_t lastb = scan_units(a, nunits);
    if ((int64_t)blockIdx.x > lastb) return;
    const int64_t per = a.chunk / SCAN_THREADS;
    const int64_t t0 = (int64_t)blockIdx.x * a.chunk + threadIdx.x * per;
    const int64_t tot = block_sum<SCAN_THREADS>(run_sum(a.counts, t0, per, nunits), s_w);
    if (threadIdx.x == 0) a.sums[blockIdx.x] = tot;
}
template <int NT>
__global__ __launch_bounds__(NT) void k_scan(ScanArgs a) {
    __shared__ int64_t s_w[NT / 64];
    const int tid = (int)threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int64_t nunits;
    const int64_t lastb = scan_units(a, nunits);
    if ((int64_t)blockIdx.x > lastb) return;
    const bool finisher = (int64_t)blockIdx.x == lastb && tid == NT - 1;
    int64_t base[2] = {0, 0};
    unsigned long long id0 = 0;
    if (finisher) {   // read early: the latency overlaps the scan
        for (int k = 0; k < 2; ++k) base[k] = (a.out_count[k] && !a.zero_base) ? *a.out_count[k] : 0;
        id0 = *a.next_id;
    }
    // the total of the blocks before this one
    const int64_t before = gridDim.x > 1 ? block_sum<NT>(tid < (int)blockIdx.x ? a.sums[tid] : 0, s_w) : 0;
    const int64_t per = a.chunk / NT;
    const int64_t t0 = (int64_t)blockIdx.x * a.chunk + tid * per;
    // the first eight counts of the run stay in registers for the second pass
    int v0[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v0[k] = (k < per && t0 + k < nunits) ? a.counts[t0 + k] : 0;
    int64_t sum = per > 8 ? run_sum(a.counts, t0 + 8, per - 8, nunits) : 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) sum += v0[k];
    int64_t incl = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t v = __shfl_up(incl, d);
        if (lane >= d) incl += v;
    }
    __syncthreads();
    if (lane == 63) s_w[wid] = incl;
    __syncthreads();
    int64_t wbefore = 0, btot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        const int64_t x = s_w[w];
        wbefore += w < wid ? x : 0;
        btot += x;
    }
    int64_t run = before + wbefore + incl - sum;
    for (int64_t b = 0; b < per; b += 8) {   // the offsets, a batch of eight counts at a time
        int v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t u = t0 + b + k;
            v[k] = b == 0 ? v0[k] : ((b + k < per && u < nunits) ? a.counts[u] : 0);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t u = t0 + b + k;
            if (b + k < per && u < nunits) {
                a.off[u] = run;
                if (a.clear) const_cast<int *>(a.counts)[u] = 0;
            }
            run += v[k];
        }
    }
    if (finisher) {
        const int64_t tot = before + btot;
        a.off[nunits] = tot;
        uint32_t st = 0;
        for (int k = 0; k < 2; ++k) {
            a.launch[k] = base[k];
            if (a.out_count[k]) {
                const int64_t c = base[k] + tot;
                if (c > a.out_cap[k]) st |= QED_ST_OVERFLOW;
                *a.out_count[k] = c < a.out_cap[k] ? c : a.out_cap[k];
            }
        }
        if (a.base_out)
            for (int k = 0; k < 2; ++k) a.base_out[k] = base[k];
        a.launch[2] = (int64_t)id0;
        a.launch[3] = tot;
        *a.next_id = id0 + (unsigned long long)(a.ids_per_event * tot);
        if (st) atomicOr(a.status, st);
    }
}

// ------------------------------------------------------------------------- leptons
struct LeptonArgs {
    Consts c;
    const void *tab;
    SegArgs sa;
    qed_leptons L;
    const int64_t *n_in;       // optional: process leptons [0, *n_in) (those alive when a step began)
    qed_photons out;
    int has_out;
    double *E6;
    int64_t step;
    const int64_t *step_dev;   // optional device step counter, added to step
    uint32_t *status;
    void *stg;
    int *tile_counts;
    int *group_tot;            // events per group of ev_group tiles (zero between launches)
    int64_t *scan_sums;        // block totals of the scan
    int ev_group, ev_shift;    // tiles per wavefront of the event kernel and its log2
    float *ev_in;              // learned sampler: per-event network inputs [events][4]
    const float *ev_out;       // and outputs [events][3]
    const int64_t *tile_off;
    const int64_t *launch;
};

// leptons a launch covers: [0, *n_in) when given (the list's count at the start of a
// whole step, before pairs were appended to it), else the whole list
__device__ __forceinline__ int64_t lepton_count(const LeptonArgs &a) {
    return clamp_count(a.n_in ? a.n_in : a.L.count, a.L.capacity);
}

// push + T-BMT + drift; returns 1/gamma^{n+1/2}
template <class T>
__device__ __forceinline__ double push_one(const LeptonArgs &a, double q, double dt, const V3<double> &E,
                                           const V3<double> &B, V3<double> &r, V3<double> &p, V3<T> &S,
                                           uint32_t &st) {
    V3<double> pm, pp;
    const double ign = boris(q, dt, E, B, p, pm, pp);
    bmt<T>(a.c, q, E, B, pm, pp, ign, S);
    const double ig = rsqrt(1.0 + dot(p, p));
    r = r + (dt * ig) * p;
    if (!isfinite(p.x + p.y + p.z + r.x + r.y + r.z) || !isfinite((double)(S.x + S.y + S.z))) st |= QED_ST_NAN;
    return ig;
}

// gather and/or push, no NCS: grid-stride loop
template <class T, bool WRITE_E6, bool PUSH, bool E6_IN, bool MULTI>
__global__ __launch_bounds__(BLOCK) void k_leptons_simple(LeptonArgs a) {
    const int64_t n = lepton_count(a);
    const double dt = a.c.dt, t = (double)step_of(a) * dt, q = (double)a.L.charge;
    T *sx = (T *)a.L.sx, *sy = (T *)a.L.sy, *sz = (T *)a.L.sz;
    uint32_t st = 0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        V3<double> r = {a.L.x[i], a.L.y[i], a.L.z[i]}, E, B;
        if constexpr (E6_IN) {
            const double *e = a.E6 + 6 * i;
            E = {e[0], e[1], e[2]};
            B = {e[3], e[4], e[5]};
        } else {
            if constexpr (MULTI) fields_for<T, FK_MULTI>(a.sa, i, t, r, E, B);
            else if (i >= a.sa.begin0 && i < a.sa.end0) field_at<T>(a.sa.f0, t, r.x, r.y, r.z, E, B);
            else E = B = {0, 0, 0};
        }
        if constexpr (WRITE_E6) {
            double *e = a.E6 + 6 * i;
            e[0] = E.x; e[1] = E.y; e[2] = E.z;
            e[3] = B.x; e[4] = B.y; e[5] = B.z;
        }
        if constexpr (PUSH) {
            V3<double> p = {a.L.px[i], a.L.py[i], a.L.pz[i]};
            V3<T> S = {sx[i], sy[i], sz[i]};
            push_one<T>(a, q, dt, E, B, r, p, S, st);
            a.L.x[i] = r.x; a.L.y[i] = r.y; a.L.z[i] = r.z;
            a.L.px[i] = p.x; a.L.py[i] = p.y; a.L.pz[i] = p.z;
            sx[i] = S.x; sy[i] = S.y; sz[i] = S.z;
        }
    }
    if (st) atomicOr(a.status, st);
}

// State of lepton i after the push (PUSH: gather at x^n, Boris, T-BMT, drift) or with the
// fields of x^n taken from E6 (emission only).  Returns 1/gamma of the resulting momentum.  Lepton arrays are addressed with 32-bit byte
// offsets from the array base (lists hold at most 2^28 particles), which lets every load
// and store use the scalar-base + vector-offset form.
// PRE: r, E and B given (the grid fields gathered by the wavefront beforehand)
template <class T, bool PUSH, int FK, bool PRE = false>
__device__ __forceinline__ double lepton_state(const LeptonArgs &a, int64_t i, double t, double q, V3<double> &r,
                                               V3<double> &p, V3<T> &S, V3<double> &E, V3<double> &B,
                                               uint32_t &st) {
    const uint32_t o = (uint32_t)i * 8u, os = (uint32_t)i * (uint32_t)sizeof(T);
    if constexpr (!PRE) r = {ld_nt(a.L.x, o), ld_nt(a.L.y, o), ld_nt(a.L.z, o)};
    p = {ld_nt(a.L.px, o), ld_nt(a.L.py, o), ld_nt(a.L.pz, o)};
    S = {ld_nt((T *)a.L.sx, os), ld_nt((T *)a.L.sy, os), ld_nt((T *)a.L.sz, os)};
    if constexpr (PUSH) {
        if constexpr (!PRE) fields_for<T, FK>(a.sa, i, t, r, E, B);
        return push_one<T>(a, q, a.c.dt, E, B, r, p, S, st);
    } else {
        const double *e = a.E6 + 6 * i;
        E = {e[0], e[1], e[2]};
        B = {e[3], e[4], e[5]};
        return rsqrt(1.0 + dot(p, p));
    }
}
template <class T>
__device__ __forceinline__ void store_xp(const LeptonArgs &a, uint32_t o, const V3<double> &r, const V3<double> &p) {
    st_nt(a.L.x, o, r.x); st_nt(a.L.y, o, r.y); st_nt(a.L.z, o, r.z);
    st_nt(a.L.px, o, p.x); st_nt(a.L.py, o, p.y); st_nt(a.L.pz, o, p.z);
}
template <class T>
__device__ __forceinline__ void store_s(const LeptonArgs &a, uint32_t os, const V3<T> &S) {
    st_nt((T *)a.L.sx, os, S.x); st_nt((T *)a.L.sy, os, S.y); st_nt((T *)a.L.sz, os, S.z);
}

// Radiative push (Sec. III.A.3) and radiative T-BMT (Sec. III.B.3), grid-stride over the
// leptons: Boris with E^n, B^n gives p_L^{n+1/2}; at the time-centred gamma^n, beta^n =
// (p- + p+)/(2 gamma^n) and chi^n, the Landau-Lifshitz force (its two leading terms,
// eq. eq1-1, with the 1/gamma of eq. eq1 on E(p.E)) adds F dt, scaled by the emitted /
// Larmor power ratio g(chi^n) for MLL; the spin takes half kicks dt/2 R(S),
// R = -P [psi1 S + psi2 (S.beta) beta + psi3 b], P = alpha/(sqrt3 pi xi_L gamma^n), around
// the T-BMT rotation (b = n x a of the local frame at time n).  S is not renormalised.
template <class T>
__device__ __forceinline__ void rbmt_half_kick(T P, const RadCoef<T> &rc, const V3<T> &beta, const V3<T> &b, T hdt,
                                               V3<T> &S) {
    const T sb = dot(S, beta);
    S = S - (hdt * P) * (rc.p1 * S + (rc.p2 * sb) * beta + rc.p3 * b);
}
template <class T, int FK>
__global__ __launch_bounds__(BLOCK) void k_leptons_radiative(LeptonArgs a, uint32_t mode) {
    const int64_t n = lepton_count(a);
    const double dt = a.c.dt, t = (double)step_of(a) * dt, q = (double)a.L.charge;
    const Tabs<T> tb = {(const T *)a.tab};
    const uint32_t force = mode & (QED_RR_LL | QED_RR_MLL);
    const bool rbmt = (mode & QED_RR_RBMT) != 0;
    uint32_t st = 0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        const uint32_t o = (uint32_t)i * 8u, os = (uint32_t)i * (uint32_t)sizeof(T);
        V3<double> r = {ld_nt(a.L.x, o), ld_nt(a.L.y, o), ld_nt(a.L.z, o)};
        V3<double> p = {ld_nt(a.L.px, o), ld_nt(a.L.py, o), ld_nt(a.L.pz, o)};
        V3<T> S = {ld_nt((T *)a.L.sx, os), ld_nt((T *)a.L.sy, os), ld_nt((T *)a.L.sz, os)};
        V3<double> E, B, pm, pp;
        fields_for<T, FK>(a.sa, i, t, r, E, B);
        const double ign = boris(q, dt, E, B, p, pm, pp);
        const double g = 1.0 / ign;
        const V3<double> beta = (0.5 * ign) * (pm + pp);
        const V3<double> v = E + cross(beta, B);
        const double be = dot(beta, E), s2 = dot(v, v) - be * be;
        const double chi = a.c.xi_L * g * sqrt(s2 > 0.0 ? s2 : 0.0);
        RadCoef<T> rc = {(T)1, (T)0, (T)0, (T)0};
        if ((force & QED_RR_MLL) || rbmt) rc = rad_coeffs<T>(tb, chi, st);
        if (force) {
            const V3<double> pn = g * beta;
            const V3<double> F = (2.0 / 3.0 * a.c.alpha * a.c.xi_L) *
                                 (cross(E, B) + ign * (cross(B, cross(B, pn)) + dot(pn, E) * E) - (g * s2) * pn);
            const double scale = (force & QED_RR_MLL) ? (double)rc.g : 1.0;
            p = p + (scale * dt) * F;
        }
        if (rbmt) {
            V3<double> bd = {0, 0, 0};
            const double bn2 = dot(beta, beta);
            if (bn2 > 0.0) {
                const V3<double> nd = rsqrt(bn2) * beta;
                const V3<double> ad = v - dot(nd, v) * nd;
                const double a2 = dot(ad, ad);
                if (a2 > 0.0) bd = cross(nd, (q * rsqrt(a2)) * ad);
            }
            const V3<T> bt = cvt<T>(beta), b = cvt<T>(bd);
            const T P = (T)(a.c.c_ncs * ign), hdt = (T)(0.5 * dt);
            rbmt_half_kick<T>(P, rc, bt, b, hdt, S);
            bmt<T>(a.c, q, E, B, pm, pp, ign, S);
            rbmt_half_kick<T>(P, rc, bt, b, hdt, S);
        } else {
            bmt<T>(a.c, q, E, B, pm, pp, ign, S);
        }
        const double igp = rsqrt(1.0 + dot(p, p));
        r = r + (dt * igp) * p;
        if (!isfinite(p.x + p.y + p.z + r.x + r.y + r.z) || !isfinite((double)(S.x + S.y + S.z))) st |= QED_ST_NAN;
        store_xp<T>(a, o, r, p);
        store_s<T>(a, os, S);
    }
    if (st) atomicOr(a.status, st);
}

// Decide (lepton step with NCS), one thread per particle, BLOCK-particle tiles; a block
// takes tiles blockIdx.x, blockIdx.x + gridDim.x, ... (one tile per block when the grid
// covers the list, a persistent sweep when the grid is a few blocks per CU): gather, push,
// T-BMT, local frame, rates, event test.  Every particle writes back x^{n+1}, p^{n+1/2}
// and its spin (after the no-emission update when nothing happened).  Event particles
// also park their state in a LepEvent record at their tile's staging slot tile*BLOCK +
// rank (rank in index order: wave ballot + popcount, waves combined in LDS); the tile's
// event count goes to tile_counts and is added to its group's total (integer atomics: the
// sum does not depend on their order; the scan clears the totals it reads).  RATE_LDS: the
// NCS rate table is staged in LDS once per block instead of being read through the caches.
// The FP64 instances are held to at least five wavefronts per SIMD (83-94 VGPRs, no
// spills): forcing six (79 VGPRs with spills) measured 4 % slower, seven 25 % slower.  So
// is the FP32 grid instance with its LDS box (96 VGPRs, no spills; 100 unconstrained).
template <class T, bool PUSH, int FK, bool RATE_LDS>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu((sizeof(T) == 8 || (PUSH && FK == QED_FIELD_GRID2D)) ? 5 : 1))) void k_leptons_decide(LeptonArgs a) {
    __shared__ int s_wave[2][BLOCK / 64];
    __shared__ T s_rate[RATE_LDS ? 2 * NR : 1];
    // a grid field of one segment: each wavefront's LDS box of stencil nodes
    // (grid_fields_wavebox), the global gather where the box does not serve
    constexpr bool WBOX = PUSH && FK == QED_FIELD_GRID2D;
    __shared__ float s_box[WBOX ? BLOCK / 64 : 1][WBOX ? WB_FLOATS : 1];
    // 32-bit indices: lists hold at most 2^28 particles
    const int n = (int)lepton_count(a);
    const int ntiles = (n + BLOCK - 1) / BLOCK;
    if ((int)blockIdx.x >= ntiles) return;
    const Tabs<T> tb = {(const T *)a.tab};
    const T *rate = tb.ncs_rate();
    if constexpr (RATE_LDS) {
        for (int k = threadIdx.x; k < 2 * NR; k += BLOCK) s_rate[k] = rate[k];
        __syncthreads();
        rate = s_rate;
    }
    const int64_t step = step_of(a);
    const double t = (double)step * a.c.dt, q = (double)a.L.charge;
    uint32_t st = 0;
    int par = 0;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x, par ^= 1) {
        const int base = tile * BLOCK, i = base + (int)threadIdx.x;
        bool ev = false;
        V3<double> r, p, E, B;
        V3<T> S;
        if constexpr (WBOX) {
            r = {0, 0, 0};
            E = {0, 0, 0};
            B = {0, 0, 0};
            bool in = false;
            if (i < n) {
                const uint32_t o = (uint32_t)i * 8u;
                r = {ld_nt(a.L.x, o), ld_nt(a.L.y, o), ld_nt(a.L.z, o)};
                in = i >= a.sa.begin0 && i < a.sa.end0;
            }
            const bool have = grid_fields_wavebox<T>(a.sa.f0.g, s_box[threadIdx.x >> 6], in, r.x, r.y, E, B);
            if (in && !have) field_kind<T, FK>(a.sa.f0, t, r.x, r.y, r.z, E, B);
        }
        if (i < n) {
            const double ig = lepton_state<T, PUSH, FK, WBOX>(a, i, t, q, r, p, S, E, B, st);
            if constexpr (PUSH) store_xp<T>(a, (uint32_t)i * 8u, r, p);
            NcsFrame<T> f;
            if (ncs_frame<T>(a.c, rate, q, p, ig, S, E, B, st, f)) {
                double rr[4];
                uniform4(at(a.L.id, (uint32_t)i * 8u), step, STREAM_NCS, a.c.seed, rr);
                ev = rr[1] < f.P;
                if (!ev) ncs_no_event<T>(a.c, f, S);
            }
            if (!ev) store_s<T>(a, (uint32_t)i * (uint32_t)sizeof(T), S);
        }
        int total;
        const int rank = block_rank(ev, total, s_wave[par]);
        if (ev) {
            LepEvent<T> &o = ((LepEvent<T> *)a.stg)[(int64_t)(base + rank)];
            o.i = i;
            o.id = at(a.L.id, (uint32_t)i * 8u);
            o.w = at(a.L.w, (uint32_t)i * 8u);
            o.r[0] = r.x; o.r[1] = r.y; o.r[2] = r.z;
            o.p[0] = p.x; o.p[1] = p.y; o.p[2] = p.z;
            o.E[0] = E.x; o.E[1] = E.y; o.E[2] = E.z;
            o.B[0] = B.x; o.B[1] = B.y; o.B[2] = B.z;
            o.S[0] = S.x; o.S[1] = S.y; o.S[2] = S.z;
        }
        if (threadIdx.x == 0) {
            a.tile_counts[tile] = total;
            if (total) atomicAdd(a.group_tot + (tile >> a.ev_shift), total);
        }
    }
    if (st) atomicOr(a.status, st);
}

// Events of the last decide, after the scan.  One wavefront per group of G tiles: the
// tile counts of the group are scanned across lanes, lane k takes the group's events k,
// k + 64, ..., finds its tile and record, rebuilds the local frame from the parked state,
// emits, and writes the photon straight to its ordered place: global rank = group offset
// + rank in the group, id = id base + global rank.
// MODE: EV_FULL (table sampler), EV_PREP (learned sampler, first pass: write the network
// inputs of every event at its global rank), EV_FINISH (second pass: the photon-fraction
// variable from the network's output inside its chi range, from the table outside it).
enum { EV_FULL = 0, EV_PREP = 1, EV_FINISH = 2 };
template <class T, int G, int MODE>
__global__ __launch_bounds__(BLOCK) void k_leptons_events(LeptonArgs a) {
    static_assert(G <= 64, "one group = at most one wave of tiles");
    const int64_t n = lepton_count(a);
    const int64_t ntiles = (n + BLOCK - 1) / BLOCK;
    const int64_t ngroups = (ntiles + G - 1) / G;
    const int64_t obase = a.launch[0], id0 = a.launch[2];
    const Tabs<T> tb = {(const T *)a.tab};
    const int64_t step = step_of(a);
    const double q = (double)a.L.charge;
    const int lane = threadIdx.x & 63;
    uint32_t st = 0;
    const int64_t g = (int64_t)blockIdx.x * (BLOCK / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (g < ngroups) {
        const int64_t c0 = g * G;
        const int cnt = (lane < G && c0 + lane < ntiles) ? a.tile_counts[c0 + lane] : 0;
        int incl = cnt;   // inclusive scan of the tile counts over the lanes
#pragma unroll
        for (int d = 1; d < G; d <<= 1) {
            const int v = __shfl_up(incl, d);
            incl += lane >= d ? v : 0;
        }
        int pre[G];   // wave-uniform inclusive prefix per tile
#pragma unroll
        for (int k = 0; k < G; ++k) pre[k] = __builtin_amdgcn_readlane(incl, k);
        const int gtot = pre[G - 1];
        const int64_t goff = a.tile_off[g];
        for (int e = lane; e < gtot; e += 64) {
            int j = 0, below = 0;   // tile of event e and the events before that tile
#pragma unroll
            for (int k = 0; k < G - 1; ++k) {
                const bool past = pre[k] <= e;
                j += past ? 1 : 0;
                below = past ? pre[k] : below;
            }
            const LepEvent<T> &o = ((const LepEvent<T> *)a.stg)[(c0 + j) * BLOCK + (e - below)];
            const int64_t i = o.i;
            V3<double> p = {o.p[0], o.p[1], o.p[2]};
            const V3<double> E = {o.E[0], o.E[1], o.E[2]}, B = {o.B[0], o.B[1], o.B[2]};
            V3<T> S = {o.S[0], o.S[1], o.S[2]};
            // the photon's birth place and weight, read with the rest of the record: read after
            // the lepton's write-back (which may alias the record, for all the compiler
            // knows), each would wait for the store before it, four round trips in a row
            const double bx = o.r[0], by = o.r[1], bz = o.r[2], bw = o.w;
            NcsFrame<T> f;
            ncs_frame<T>(a.c, tb.ncs_rate(), q, p, rsqrt(1.0 + dot(p, p)), S, E, B, st, f);
            double rr[4];
            uniform4(o.id, step, STREAM_NCS, a.c.seed, rr);
            const int64_t ge = goff + e;
            const bool in_range = f.chi >= MLP_CHI_LO && f.chi <= MLP_CHI_HI;
            if constexpr (MODE == EV_PREP) {
                float4 x = {0.0f, 0.0f, 0.0f, 0.0f};
                if (in_range)
                    x = {(float)((log10(f.chi) - MLP_L10_MID) / MLP_L10_HALF), (float)f.s, (float)dot(S, f.n),
                         (float)(2.0 * rr[0] - 1.0)};
                ((float4 *)a.ev_in)[ge] = x;
                continue;
            }
            // the network's t is used where it is a valid sample (t_lo <= t < t_max, t_lo =
            // 0.5: below it the network's absolute error is a large relative error in the
            // energy) inside its trained chi range; the table decides everywhere else
            const float yn = MODE == EV_FINISH ? a.ev_out[3 * ge] : -1.0f;
            const T tt = (MODE == EV_FINISH && in_range && yn >= MLP_Y_LO && yn < 1.0f)
                             ? (T)(yn * (float)T_MAX)
                             : ncs_sample_t<T>(tb, f.chi, f.Ib / f.Ia, f.s, (T)rr[0]);
            NcsPhoton<T> ph;
            ncs_event_t<T>(a.c, tb, f, tt, rr, p, S, ph);
            const uint32_t o8 = (uint32_t)i * 8u;
            at(a.L.px, o8) = p.x; at(a.L.py, o8) = p.y; at(a.L.pz, o8) = p.z;
            store_s<T>(a, (uint32_t)i * (uint32_t)sizeof(T), S);
            const int64_t pos = obase + ge;
            if (a.has_out && pos < a.out.capacity) {
                a.out.x[pos] = bx; a.out.y[pos] = by; a.out.z[pos] = bz;
                a.out.kx[pos] = ph.k.x; a.out.ky[pos] = ph.k.y; a.out.kz[pos] = ph.k.z;
                a.out.w[pos] = bw;
                ((T *)a.out.xi1)[pos] = ph.xi.x; ((T *)a.out.xi2)[pos] = ph.xi.y; ((T *)a.out.xi3)[pos] = ph.xi.z;
                ((T *)a.out.e1x)[pos] = ph.e1.x; ((T *)a.out.e1y)[pos] = ph.e1.y; ((T *)a.out.e1z)[pos] = ph.e1.z;
                a.out.id[pos] = (unsigned long long)(id0 + ge);
                a.out.alive[pos] = 1;
            }
        }
    }
    if (st) atomicOr(a.status, st);
}

// advance the device step counter
__global__ void k_advance_step(int64_t *step, int64_t by) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *step += by;
}

// ------------------------------------------------------------------------- photons
struct PhotonArgs {
    Consts c;
    const void *tab;
    FieldDev field;
    qed_photons G;
    qed_leptons em, ep;
    int has_em, has_ep;
    int do_vb, do_nbw, do_move;
    int64_t step;
    const int64_t *step_dev;   // optional device step counter, added to step
    uint32_t *status;
    EventRec *stg;
    int *tile_counts;
    int *ph_tot;               // pair events per group and per 64 groups, two parities (ctx)
    int64_t *launch;           // [0] em base, [1] ep base, [2] id base, [3] pairs, [4] parity
    int64_t *base_out;         // optional [2]: the lepton counts before the append
    unsigned long long *next_id;
    float *ev_in;              // learned NBW sampler: per-pair network inputs [pairs][4]
    const float *ev_out;       // and outputs [pairs][3]
    int ev_net;                // pair events: the network's delta used where valid
    int ev_update;             // pair events: this pass sets the counts, the id counter, the parity
};

// transport (+ NBW test), specialised on the field kind: a persistent grid sweeps the
// 256-photon tiles of the live list (blocks beyond the list's tiles exit at once, so a
// list far below its capacity costs no empty waves); with NBW each tile ranks its events
// in photon order (wave ballot + popcount, waves combined in LDS) and parks their records
// at the tile's staging slots
// the photon step's two rate tables (NBW rates, VB indices) copied to LDS by each block:
// their lookups come after the gather on every photon's dependent chain
template <class T>
struct PhotonTabsLds {
    const T *nbw, *vbt;
    __device__ __forceinline__ const T *nbw_rate() const { return nbw; }
    __device__ __forceinline__ const T *vb() const { return vbt; }
};

// FP64: held to four wavefronts per SIMD (at most 128 VGPRs)
// Pair events are rare (well under one per tile).  The decide kernel adds each tile's count
// to its group of PH_GROUP tiles and to its run of 64 groups (integer atomics: the sums do
// not depend on their order), in the buffers of the current parity; the event kernel, one
// wavefront per group, takes the group's first rank from those sums itself (no scan
// launch).  The buffers of the other parity, read by the previous stage's event kernel,
// are cleared by this stage's decide kernel, and the event kernel flips the parity.  Block
// 0 of the decide kernel also records the lepton counts and the id counter before the
// append, which the event kernel's wavefronts read while its wavefront 0 advances them.
__device__ __forceinline__ int *ph_groups(int *t, int p) { return t + p * PH_GROUPS_MAX; }
__device__ __forceinline__ int *ph_super(int *t, int p) { return t + 2 * PH_GROUPS_MAX + p * PH_SUPER_MAX; }
__device__ __forceinline__ int *ph_state(int *t) { return t + 2 * PH_GROUPS_MAX + 2 * PH_SUPER_MAX; }
template <class T, bool NBW, int FK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 4 : 1))) void k_photons_decide(PhotonArgs a) {
    __shared__ int s_wave[2][BLOCK / 64];
    __shared__ T s_tab[2 * NP + 2 * NV];
    // grid fields: each wavefront's LDS box of stencil nodes (grid_fields_wavebox)
    __shared__ float s_box[FK == QED_FIELD_GRID2D ? BLOCK / 64 : 1][FK == QED_FIELD_GRID2D ? WB_FLOATS : 1];
    // 32-bit indices: lists hold at most 2^28 particles
    const int n = (int)clamp_count(a.G.count, a.G.capacity);
    const int ntiles = (n + BLOCK - 1) / BLOCK;
    int ph_par = 0;
    if constexpr (NBW) {   // the pair-event bookkeeping (before any block leaves)
        int *state = ph_state(a.ph_tot);
        ph_par = state[0];
        const int q = 1 - ph_par;
        // groups [0, used) and their runs of 64 (used <= 2^15: inside the buffers)
        const int64_t used = state[1 + q], uses = (used + 63) / 64;
        int *og = ph_groups(a.ph_tot, q), *os = ph_super(a.ph_tot, q);
        for (int64_t u = (int64_t)blockIdx.x * BLOCK + threadIdx.x; u < used; u += (int64_t)gridDim.x * BLOCK)
            og[u] = 0;
        for (int64_t u = (int64_t)blockIdx.x * BLOCK + threadIdx.x; u < uses; u += (int64_t)gridDim.x * BLOCK)
            os[u] = 0;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            const int64_t b0 = a.has_em ? *a.em.count : 0, b1 = a.has_ep ? *a.ep.count : 0;
            a.launch[0] = b0;
            a.launch[1] = b1;
            a.launch[2] = (int64_t)*a.next_id;
            a.launch[4] = ph_par;
            if (a.base_out) {
                a.base_out[0] = b0;
                a.base_out[1] = b1;
            }
        }
    }
    if ((int)blockIdx.x >= ntiles) return;
    {
        const Tabs<T> tg = {(const T *)a.tab};
        for (int k = threadIdx.x; k < 2 * NP; k += BLOCK) s_tab[k] = tg.nbw_rate()[k];
        for (int k = threadIdx.x; k < 2 * NV; k += BLOCK) s_tab[2 * NP + k] = tg.vb()[k];
        __syncthreads();
    }
    const PhotonTabsLds<T> tb = {s_tab, s_tab + 2 * NP};
    const int64_t step = step_of(a);
    const double t = (double)step * a.c.dt;
    T *xi1 = (T *)a.G.xi1, *xi2 = (T *)a.G.xi2, *xi3 = (T *)a.G.xi3;
    T *e1x = (T *)a.G.e1x, *e1y = (T *)a.G.e1y, *e1z = (T *)a.G.e1z;
    uint32_t st = 0;
    int par = 0;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x, par ^= 1) {
        const int j = tile * BLOCK + (int)threadIdx.x;
        bool ev = false;
        V3<double> E = {0, 0, 0}, B = {0, 0, 0};
        // the photon's record is read together with its alive flag (not after it), so the
        // gather waits for one memory round trip, not two
        const bool inr = j < n;
        const uint32_t o = (uint32_t)j * 8u, os = (uint32_t)j * (uint32_t)sizeof(T);
        V3<double> x = {0, 0, 0}, k = {0, 0, 0};
        V3<T> xi = {0, 0, 0}, e1 = {0, 0, 0};
        bool live = false;
        if (inr) {
            live = a.G.alive[j] != 0;
            x = {ld_nt(a.G.x, o), ld_nt(a.G.y, o), ld_nt(a.G.z, o)};
            k = {ld_nt(a.G.kx, o), ld_nt(a.G.ky, o), ld_nt(a.G.kz, o)};
            xi = {ld_nt(xi1, os), ld_nt(xi2, os), ld_nt(xi3, os)};
            e1 = {ld_nt(e1x, os), ld_nt(e1y, os), ld_nt(e1z, os)};
        }
        bool have = false;
        if constexpr (FK == QED_FIELD_GRID2D)
            have = grid_fields_wavebox<T>(a.field.g, s_box[threadIdx.x >> 6], live, x.x, x.y, E, B);
        if (live) {
            if (!have) field_kind<T, FK>(a.field, t, x.x, x.y, x.z, E, B);
            PhotonFrame f;
            photon_frame(a.c.xi_L, k, E, B, f);
            const double chi = photon_transport<T>(a.c, tb, f, xi, e1, a.do_vb, st);
            const double eps = f.eps;
            if (NBW && chi > 0.0 && eps >= 2.0) {
                T Ja, kappa;
                const double P = nbw_prob<T>(a.c, tb, eps, chi, xi.z, Ja, kappa, st);
                // a draw is at least 2^-33 (the generator's smallest uniform), so below that
                // probability there is no event whatever the draw: the generator is skipped
                if (Ja > (T)0 && P > 0x1p-33) {
                    double rr[4];
                    uniform4(at(a.G.id, o), step, STREAM_NBW, a.c.seed, rr);
                    ev = rr[1] < P;
                    if (ev) {   // the event's record, in this photon's own staging slot
                        PhotonEvent<T> &r = *photon_event<T>(a.stg, j);
                        r.k[0] = k.x; r.k[1] = k.y; r.k[2] = k.z;
                        r.x[0] = x.x; r.x[1] = x.y; r.x[2] = x.z;
                        r.chi = chi; r.r0 = rr[0]; r.r2 = rr[2];
                        r.xi[0] = xi.x; r.xi[1] = xi.y; r.xi[2] = xi.z;
                        r.e1[0] = e1.x; r.e1[1] = e1.y; r.e1[2] = e1.z;
                        r.kappa = kappa;
                    }
                }
            }
            st_nt(xi1, os, xi.x); st_nt(xi2, os, xi.y); st_nt(xi3, os, xi.z);
            st_nt(e1x, os, e1.x); st_nt(e1y, os, e1.y); st_nt(e1z, os, e1.z);
            if (ev) {
                a.G.alive[j] = 0;
            } else if (a.do_move) {
                const double ie = a.c.dt * f.inv_eps;
                st_nt(a.G.x, o, x.x + ie * k.x);
                st_nt(a.G.y, o, x.y + ie * k.y);
                st_nt(a.G.z, o, x.z + ie * k.z);
            }
        }
        if constexpr (NBW) {
            int total;
            const int rank = block_rank(ev, total, s_wave[par]);
            if (ev) *event_index(a.stg, (int64_t)tile * BLOCK + rank) = j;
            if (threadIdx.x == 0) {
                a.tile_counts[tile] = total;
                if (total) {
                    atomicAdd(ph_groups(a.ph_tot, ph_par) + tile / PH_GROUP, total);
                    atomicAdd(ph_super(a.ph_tot, ph_par) + tile / (PH_GROUP * 64), total);
                }
            }
        }
    }
    if (st) atomicOr(a.status, st);
}

// pair events: electron to em, positron to ep, in photon order; one wavefront per group
// of PH_GROUP tiles.  MODE EV_PREP writes the NBW
// network's inputs of every pair at its rank, nothing else; EV_FINISH writes the pairs,
// with the network's delta where valid when ev_net is set.  The table sampler runs the
// same EV_FINISH code with ev_net clear, so that its pairs are bitwise those of the
// learned sampler wherever the network's delta is not used.
template <class T, int MODE>
__global__ __launch_bounds__(BLOCK) void k_photons_events(PhotonArgs a) {
    const int64_t n = clamp_count(a.G.count, a.G.capacity);
    const int64_t ntiles = (n + BLOCK - 1) / BLOCK, ngroups = (ntiles + PH_GROUP - 1) / PH_GROUP;
    const int64_t wv = (int64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6), t0 = wv * PH_GROUP;
    const int lane = threadIdx.x & 63;
    const int p = (int)a.launch[4];
    const int *gt = ph_groups(a.ph_tot, p), *su = ph_super(a.ph_tot, p);
    if (wv == 0 && a.ev_update) {   // the append: new counts, id counter, pair total, parity
        int64_t tot = 0;
        for (int64_t u = lane; u < (ngroups + 63) / 64; u += 64) tot += su[u];
        tot = wave_sum_i64(tot);
        if (lane == 0) {
            uint32_t so = 0;
            const qed_leptons *Ls[2] = {&a.em, &a.ep};
            const int has[2] = {a.has_em, a.has_ep};
            for (int k = 0; k < 2; ++k) {
                if (!has[k]) continue;
                const int64_t c = a.launch[k] + tot;
                if (c > Ls[k]->capacity) so |= QED_ST_OVERFLOW;
                *Ls[k]->count = c < Ls[k]->capacity ? c : Ls[k]->capacity;
            }
            *a.next_id = (unsigned long long)a.launch[2] + 2ull * (unsigned long long)tot;
            a.launch[3] = tot;
            int *state = ph_state(a.ph_tot);
            state[0] = 1 - p;
            state[1 + p] = (int)ngroups;
            if (so) atomicOr(a.status, so);
        }
    }
    if (t0 >= ntiles) return;
    // the group's first rank: its runs of 64 groups before it, then its own run's groups
    // before it
    const int64_t sg = wv / 64;
    int64_t pre = 0;
    for (int64_t u = lane; u < sg; u += 64) pre += su[u];
    if (sg * 64 + lane < wv) pre += gt[sg * 64 + lane];
    pre = wave_sum_i64(pre);
    const int64_t id0 = a.launch[2];
    const Tabs<T> tb = {(const T *)a.tab};
    uint32_t st = 0;
    group_events<PH_GROUP>(a.tile_counts, pre, ntiles, t0, [&](int64_t e, int64_t slot) {
        // the decide kernel's record of the event (no frame, rate or generator recomputed:
        // one lane's chain of dependent reads and arithmetic is this kernel's time)
        const int64_t j = *event_index(a.stg, slot);
        const PhotonEvent<T> &r = *photon_event<T>(a.stg, j);
        const V3<double> k = {r.k[0], r.k[1], r.k[2]};
        const V3<T> xi = {r.xi[0], r.xi[1], r.xi[2]}, e1 = {r.e1[0], r.e1[1], r.e1[2]};
        const double bx = r.x[0], by = r.x[1], bz = r.x[2], bw = a.G.w[j];
        const double chi = r.chi;
        const T kappa = r.kappa;
        const double rr[4] = {r.r0, 0.0, r.r2, 0.0};   // the delta and spin draws
        const bool in_range = chi >= MLP_NBW_CHI_LO && chi <= MLP_NBW_CHI_HI;
        if constexpr (MODE == EV_PREP) {
            float4 x = {0.0f, 0.0f, 0.0f, 0.0f};
            if (in_range) x = {(float)((log10(chi) - MLP_NBW_L10_MID) / MLP_NBW_L10_HALF), (float)xi.z, 0.0f,
                               (float)(2.0 * rr[0] - 1.0)};
            ((float4 *)a.ev_in)[e] = x;
            return;
        }
        // the network's delta inside its trained chi range where it lies in [MLP_D_LO,
        // 1 - MLP_D_LO] (away from the ends, where an absolute error is a large relative
        // one in the softer member's energy); the table everywhere else
        const float dn = a.ev_net ? a.ev_out[3 * e] : -1.0f;
        const T d = (a.ev_net && in_range && dn >= MLP_D_LO && dn <= 1.0f - MLP_D_LO)
                        ? (T)dn
                        : nbw_sample_delta<T>(tb, chi, kappa, xi.z, (T)rr[0]);
        PairOut<T> po;
        nbw_pair_d<T>(tb, k, chi, d, xi, e1, rr, st, po);
        const qed_leptons *Ls[2] = {&a.em, &a.ep};
        const int has[2] = {a.has_em, a.has_ep};
        for (int s = 0; s < 2; ++s) {
            if (!has[s]) continue;
            const qed_leptons &L = *Ls[s];
            const int64_t pos = a.launch[s] + e;
            if (pos >= L.capacity) continue;
            const V3<double> &p = s == 0 ? po.pm : po.pp;
            const V3<T> &S = s == 0 ? po.Sm : po.Sp;
            L.x[pos] = bx; L.y[pos] = by; L.z[pos] = bz;
            L.px[pos] = p.x; L.py[pos] = p.y; L.pz[pos] = p.z;
            ((T *)L.sx)[pos] = S.x; ((T *)L.sy)[pos] = S.y; ((T *)L.sz)[pos] = S.z;
            L.w[pos] = bw;
            L.id[pos] = (unsigned long long)(id0 + 2 * e + s);
        }
    });
    if (st) atomicOr(a.status, st);
}

// ------------------------------------------------------------------------- compaction
struct CompactArgs {
    qed_photons in, out;
    EventRec *stg;
    int *tile_counts;
    const int64_t *tile_off;
    const int64_t *launch;
};
__global__ __launch_bounds__(BLOCK) void k_compact_mark(CompactArgs a) {
    __shared__ int s_wave[BLOCK / 64];
    const int64_t n = clamp_count(a.in.count, a.in.capacity);
    const int64_t tile = blockIdx.x;
    if (tile * BLOCK >= n) return;
    const int64_t j = tile * BLOCK + threadIdx.x;
    const bool live = j < n && a.in.alive[j];
    int total;
    const int rank = block_rank(live, total, s_wave);
    if (live) a.stg[tile * BLOCK + rank].idx = j;
    if (threadIdx.x == 0) a.tile_counts[tile] = total;
}
template <class T>
__global__ __launch_bounds__(BLOCK) void k_compact_copy(CompactArgs a) {
    const int64_t n = clamp_count(a.in.count, a.in.capacity);
    const int64_t ntiles = (n + BLOCK - 1) / BLOCK;
    const int64_t nlive = a.launch[3];
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < nlive; e += (int64_t)gridDim.x * BLOCK) {
        if (e >= a.out.capacity) break;
        const int64_t tile = tile_of(a.tile_off, ntiles, e);
        const int64_t j = a.stg[tile * BLOCK + (e - a.tile_off[tile])].idx;
        a.out.x[e] = a.in.x[j]; a.out.y[e] = a.in.y[j]; a.out.z[e] = a.in.z[j];
        a.out.kx[e] = a.in.kx[j]; a.out.ky[e] = a.in.ky[j]; a.out.kz[e] = a.in.kz[j];
        a.out.w[e] = a.in.w[j];
        ((T *)a.out.xi1)[e] = ((const T *)a.in.xi1)[j];
        ((T *)a.out.xi2)[e] = ((const T *)a.in.xi2)[j];
        ((T *)a.out.xi3)[e] = ((const T *)a.in.xi3)[j];
        ((T *)a.out.e1x)[e] = ((const T *)a.in.e1x)[j];
        ((T *)a.out.e1y)[e] = ((const T *)a.in.e1y)[j];
        ((T *)a.out.e1z)[e] = ((const T *)a.in.e1z)[j];
        a.out.id[e] = a.in.id[j];
        a.out.alive[e] = 1;
    }
}

// ------------------------------------------------------------------------- launchers
Consts consts_of(const qed_ctx *ctx) {
    const qed_config &g = ctx->cfg;
    return {g.xi_L, g.alpha, g.a_e, g.dt, g.p_max, g.alpha / (SQRT3 * PI * g.xi_L), g.seed, g.procs,
            (float)g.a_e, (float)(0.5 * g.dt)};
}
static int tiles_grid(int64_t cap, int64_t tile = BLOCK) {
    const int64_t b = (cap + tile - 1) / tile;
    return b < 1 ? 1 : (int)b;
}
static int stride_grid(int64_t cap, int64_t limit) {
    int64_t b = (cap + BLOCK - 1) / BLOCK;
    if (b > limit) b = limit;
    return b < 1 ? 1 : (int)b;
}
// scan of per-tile counts (256 particles per unit) of a list of capacity in_cap
static hipError_t launch_scan(qed_ctx *ctx, const int64_t *in_count, int64_t in_cap, const int *counts,
                              int64_t *c0, int64_t cap0, int64_t *c1, int64_t cap1, int ids,
                              hipStream_t s, int zero_base = 0, int64_t *base_out = nullptr,
                              int64_t *off = nullptr, int64_t *launch = nullptr, int unit = BLOCK,
                              int64_t *sums = nullptr, int clear = 0) {
    ScanArgs sa{};
    sa.clear = clear;
    sa.zero_base = zero_base;
    sa.base_out = base_out;
    sa.counts = counts;
    sa.off = off ? off : ctx->tile_off;
    sa.unit = unit;
    sa.sums = sums ? sums : ctx->scan_sums;
    sa.in_count = in_count;
    sa.in_capacity = in_cap;
    sa.out_count[0] = c0;
    sa.out_cap[0] = cap0;
    sa.out_count[1] = c1;
    sa.out_cap[1] = cap1;
    sa.next_id = ctx->next_id;
    sa.ids_per_event = ids;
    sa.launch = launch ? launch : ctx->launch;
    sa.status = ctx->status;
    // every pointer the kernel dereferences unconditionally must be set before a launch
    if (!sa.counts || !sa.off || !sa.sums || !sa.next_id || !sa.launch || !sa.status || unit < 1)
        return hipErrorInvalidValue;
    const int64_t units = (in_cap + unit - 1) / unit;
    if (units <= SCAN_ONE_BLOCK) {   // one block, one launch
        sa.chunk = (units + SCAN_ONE_THREADS - 1) / SCAN_ONE_THREADS * SCAN_ONE_THREADS;
        if (sa.chunk < SCAN_ONE_THREADS) sa.chunk = SCAN_ONE_THREADS;
        hipLaunchKernelGGL(k_scan<SCAN_ONE_THREADS>, dim3(1), dim3(SCAN_ONE_THREADS), 0, s, sa);
        return hipGetLastError();
    }
    // blocks of at least SCAN_MIN_CHUNK units, at most SCAN_MAX_BLOCKS of them
    int64_t nb = (units + SCAN_MIN_CHUNK - 1) / SCAN_MIN_CHUNK;
    nb = nb > SCAN_MAX_BLOCKS ? SCAN_MAX_BLOCKS : nb;
    int64_t chunk = (units + nb - 1) / nb;
    chunk = (chunk + SCAN_THREADS - 1) / SCAN_THREADS * SCAN_THREADS;
    sa.chunk = chunk;
    hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, sa);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan<SCAN_THREADS>, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, sa);
    return hipGetLastError();
}

hipError_t launch_scan_events(qed_ctx *ctx, const int64_t *in_count, int64_t in_cap, const int *counts, int64_t *c0,
                              int64_t cap0, int ids, hipStream_t s) {
    return launch_scan(ctx, in_count, in_cap, counts, c0, cap0, nullptr, 0, ids, s);
}

hipError_t launch_scan_ints(qed_ctx *ctx, const int *counts, int64_t n, int64_t *off, int64_t *total,
                            int64_t *launch, hipStream_t s) {
    return launch_scan(ctx, nullptr, n, counts, total, (int64_t)1 << 62, nullptr, 0, 0, s, 1, nullptr, off, launch, 1);
}

// decide + scan + events of a step with NCS; FK as in fields_for (PUSH = false: fields
// from E6, no field evaluation)
template <class T, int G>
static hipError_t launch_events(qed_ctx *ctx, const LeptonArgs &a, hipStream_t s) {
    const int64_t groups = ((a.L.capacity + BLOCK - 1) / BLOCK + G - 1) / G;
    const int64_t nb = (groups + BLOCK / 64 - 1) / (BLOCK / 64);
    const dim3 gd(nb < 1 ? 1 : (unsigned)nb);
    if (!(ctx->sampler & QED_SAMPLER_MLP)) {
        hipLaunchKernelGGL((k_leptons_events<T, G, EV_FULL>), gd, dim3(BLOCK), 0, s, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_leptons_events<T, G, EV_PREP>), gd, dim3(BLOCK), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the network over all events of the launch (count from the scan, on the device)
    if ((e = mlp_forward(ctx, ctx->nets[QED_NET_NCS], a.ev_in, ctx->ev_out, 0, a.launch + 3, a.L.capacity, s)) !=
        hipSuccess)
        return e;
    hipLaunchKernelGGL((k_leptons_events<T, G, EV_FINISH>), gd, dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

// decide + scan + events of a step with NCS; FK as in fields_for (PUSH = false: fields
// from E6, no field evaluation).  The launch shape and the rate-table placement follow
// the context's tuning (qed_autotune); every choice gives bitwise the same results.
template <class T, bool PUSH, int FK>
static hipError_t launch_ncs(qed_ctx *ctx, const LeptonArgs &a0, hipStream_t s) {
    LeptonArgs a = a0;
    a.ev_group = ctx->tune.ev_group;
    a.ev_shift = a.ev_group == 4 ? 2 : (a.ev_group == 16 ? 4 : 3);
    auto mark = [&](int k) { return ctx->step_ev_on ? hipEventRecord(ctx->step_ev[k], s) : hipSuccess; };
    hipError_t e = mark(0);
    if (e != hipSuccess) return e;
    const int64_t ntiles = (a.L.capacity + BLOCK - 1) / BLOCK;
    int64_t grid = ntiles;
    if (ctx->tune.blocks_per_cu > 0) {
        const int64_t pg = (int64_t)ctx->tune.blocks_per_cu * ctx->num_cu;
        grid = pg < ntiles ? pg : ntiles;
    }
    const dim3 gd((unsigned)(grid < 1 ? 1 : grid));
    if (ctx->tune.rate_lds) hipLaunchKernelGGL((k_leptons_decide<T, PUSH, FK, true>), gd, dim3(BLOCK), 0, s, a);
    else hipLaunchKernelGGL((k_leptons_decide<T, PUSH, FK, false>), gd, dim3(BLOCK), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess || (e = mark(1)) != hipSuccess) return e;
    e = launch_scan(ctx, a.n_in ? a.n_in : a.L.count, a.L.capacity, a.group_tot,
                    a.has_out ? a.out.count : nullptr, a.has_out ? a.out.capacity : 0, nullptr, 0, 1, s, 0, nullptr,
                    const_cast<int64_t *>(a.tile_off), const_cast<int64_t *>(a.launch), BLOCK * a.ev_group,
                    a.scan_sums, 1);
    if (e != hipSuccess || (e = mark(2)) != hipSuccess) return e;
    switch (a.ev_group) {
    case 4: e = launch_events<T, 4>(ctx, a, s); break;
    case 16: e = launch_events<T, 16>(ctx, a, s); break;
    default: e = launch_events<T, 8>(ctx, a, s); break;
    }
    if (e != hipSuccess) return e;
    return mark(3);
}

template <class T, bool M>
static hipError_t launch_leptons_t(qed_ctx *ctx, LeptonMode mode, const LeptonArgs &a, hipStream_t s) {
    const int gs = stride_grid(a.L.capacity, 65536);
    switch (mode) {
    case LM_GATHER:
        hipLaunchKernelGGL((k_leptons_simple<T, true, false, false, M>), dim3(gs), dim3(BLOCK), 0, s, a);
        return hipGetLastError();
    case LM_PUSH:
        if (a.E6) hipLaunchKernelGGL((k_leptons_simple<T, false, true, true, false>), dim3(gs), dim3(BLOCK), 0, s, a);
        else hipLaunchKernelGGL((k_leptons_simple<T, false, true, false, M>), dim3(gs), dim3(BLOCK), 0, s, a);
        return hipGetLastError();
    case LM_EMIT:
    case LM_FUSED:
        break;
    }
    if (!(a.c.procs & QED_PROC_NCS)) {   // a fused step without NCS is a push
        hipLaunchKernelGGL((k_leptons_simple<T, false, true, false, M>), dim3(gs), dim3(BLOCK), 0, s, a);
        return hipGetLastError();
    }
    if (mode == LM_EMIT) return launch_ncs<T, false, QED_FIELD_NONE>(ctx, a, s);
    if (M) {   // several segments: specialised on their kind when they share one
        switch (a.sa.multi_kind) {
        case QED_FIELD_PW: return launch_ncs<T, true, FK_MULTI_BASE + QED_FIELD_PW>(ctx, a, s);
        case QED_FIELD_GAUSS: return launch_ncs<T, true, FK_MULTI_BASE + QED_FIELD_GAUSS>(ctx, a, s);
        default: return launch_ncs<T, true, FK_MULTI>(ctx, a, s);
        }
    }
    switch (a.sa.f0.kind) {
    case QED_FIELD_CONST: return launch_ncs<T, true, QED_FIELD_CONST>(ctx, a, s);
    case QED_FIELD_PW: return launch_ncs<T, true, QED_FIELD_PW>(ctx, a, s);
    case QED_FIELD_GAUSS: return launch_ncs<T, true, QED_FIELD_GAUSS>(ctx, a, s);
    case QED_FIELD_GRID2D: return launch_ncs<T, true, QED_FIELD_GRID2D>(ctx, a, s);
    default: return launch_ncs<T, true, QED_FIELD_NONE>(ctx, a, s);
    }
}

hipError_t launch_leptons(qed_ctx *ctx, LeptonMode mode, const SegArgs &sa, const qed_leptons &L, double *E6,
                          const qed_photons *out, int64_t step, hipStream_t s, const int64_t *n_in,
                          const ScanState *ss) {
    LeptonArgs a{};
    a.c = consts_of(ctx);
    a.sa = sa;
    a.L = L;
    a.n_in = n_in;
    a.has_out = out != nullptr;
    if (out) a.out = *out;
    a.E6 = E6;
    a.step = step;
    a.step_dev = ctx->step_dev;
    a.status = ctx->status;
    a.stg = (EventRec *)(ss ? ss->staging : ctx->staging);
    a.tile_counts = ss ? ss->tile_counts : ctx->tile_counts;
    a.group_tot = ss ? ss->group_tot : ctx->group_tot;
    a.tile_off = ss ? ss->tile_off : ctx->tile_off;
    a.launch = ss ? ss->launch : ctx->launch;
    a.scan_sums = ss ? ss->sums : ctx->scan_sums;
    a.ev_in = ctx->ev_in;
    a.ev_out = ctx->ev_out;
    const bool multi = sa.nseg > 1;
    if (ctx->cfg.precision == QED_MIXED) {
        a.tab = ctx->tab32;
        return multi ? launch_leptons_t<float, true>(ctx, mode, a, s) : launch_leptons_t<float, false>(ctx, mode, a, s);
    }
    a.tab = ctx->tab64;
    return multi ? launch_leptons_t<double, true>(ctx, mode, a, s) : launch_leptons_t<double, false>(ctx, mode, a, s);
}

// persistent photon grid: PHOTON_BLOCKS_PER_CU blocks per compute unit, at most one per tile
constexpr int PHOTON_BLOCKS_PER_CU = 8;
template <class T, int FK>
static void launch_photons_decide(const qed_ctx *ctx, const PhotonArgs &a, hipStream_t s) {
    const int64_t ntiles = (a.G.capacity + BLOCK - 1) / BLOCK, pg = (int64_t)PHOTON_BLOCKS_PER_CU * ctx->num_cu;
    const dim3 gd((unsigned)(ntiles < 1 ? 1 : (ntiles < pg ? ntiles : pg)));
    if (!a.do_nbw) hipLaunchKernelGGL((k_photons_decide<T, false, FK>), gd, dim3(BLOCK), 0, s, a);
    else hipLaunchKernelGGL((k_photons_decide<T, true, FK>), gd, dim3(BLOCK), 0, s, a);
}
template <class T>
static hipError_t launch_photons_stage(qed_ctx *ctx, const PhotonArgs &a, hipStream_t s) {
    switch (a.field.kind) {
    case QED_FIELD_CONST: launch_photons_decide<T, QED_FIELD_CONST>(ctx, a, s); break;
    case QED_FIELD_PW: launch_photons_decide<T, QED_FIELD_PW>(ctx, a, s); break;
    case QED_FIELD_GAUSS: launch_photons_decide<T, QED_FIELD_GAUSS>(ctx, a, s); break;
    case QED_FIELD_GRID2D: launch_photons_decide<T, QED_FIELD_GRID2D>(ctx, a, s); break;
    default: launch_photons_decide<T, QED_FIELD_NONE>(ctx, a, s); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !a.do_nbw) return e;
    // no scan launch: the event kernel ranks the groups itself (k_photons_decide)
    const int64_t groups = (a.G.capacity + (int64_t)BLOCK * PH_GROUP - 1) / ((int64_t)BLOCK * PH_GROUP);
    const int64_t nb = (groups + BLOCK / 64 - 1) / (BLOCK / 64);
    const dim3 gd((unsigned)(nb < 1 ? 1 : nb));
    PhotonArgs b = a;
    b.ev_net = (ctx->sampler & QED_SAMPLER_MLP_NBW) != 0;
    b.ev_update = 1;
    if (b.ev_net) {
        // learned delta: the network's inputs of every pair at its rank (this pass also
        // makes the append), the network over the device pair count, then the events
        hipLaunchKernelGGL((k_photons_events<T, EV_PREP>), gd, dim3(BLOCK), 0, s, b);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = mlp_forward(ctx, ctx->nets[QED_NET_NBW], b.ev_in, ctx->ev_out, 0, b.launch + 3, b.G.capacity, s)) !=
            hipSuccess)
            return e;
        b.ev_update = 0;
    }
    hipLaunchKernelGGL((k_photons_events<T, EV_FINISH>), gd, dim3(BLOCK), 0, s, b);
    return hipGetLastError();
}

template <class T>
static hipError_t launch_photons_t(qed_ctx *ctx, const PhotonArgs &a, hipStream_t s) {
    if (ctx->ph_ev_on) {
        const hipError_t e = hipEventRecord(ctx->ph_ev[0], s);
        if (e != hipSuccess) return e;
    }
    hipError_t e = launch_photons_stage<T>(ctx, a, s);
    if (e == hipSuccess && ctx->ph_ev_on) e = hipEventRecord(ctx->ph_ev[1], s);
    return e;
}

hipError_t launch_photons(qed_ctx *ctx, PhotonMode mode, const SegArgs &sa, const qed_photons &G,
                          const qed_leptons *em, const qed_leptons *ep, int64_t step, hipStream_t s,
                          int64_t *lep_start) {
    PhotonArgs a{};
    a.c = consts_of(ctx);
    a.field = sa.f0;
    a.G = G;
    a.has_em = em != nullptr;
    a.has_ep = ep != nullptr;
    if (em) a.em = *em;
    if (ep) a.ep = *ep;
    a.do_vb = (mode != PM_PAIR) && (ctx->cfg.procs & QED_PROC_VB);
    a.do_nbw = (mode != PM_BIREF) && (ctx->cfg.procs & QED_PROC_NBW);
    a.do_move = mode != PM_BIREF;
    a.step = step;
    a.step_dev = ctx->step_dev;
    a.status = ctx->status;
    a.stg = (EventRec *)ctx->staging;
    a.tile_counts = ctx->tile_counts;
    a.ph_tot = ctx->ph_tot;
    a.launch = ctx->launch;
    a.base_out = lep_start;
    a.next_id = ctx->next_id;
    a.ev_in = ctx->ev_in;
    a.ev_out = ctx->ev_out;
    if (ctx->cfg.precision == QED_MIXED) {
        a.tab = ctx->tab32;
        return launch_photons_t<float>(ctx, a, s);
    }
    a.tab = ctx->tab64;
    return launch_photons_t<double>(ctx, a, s);
}

template <class T>
static hipError_t launch_radiative_t(const LeptonArgs &a, uint32_t mode, hipStream_t s) {
    const dim3 gd(stride_grid(a.L.capacity, 65536)), bd(BLOCK);
    if (a.sa.nseg > 1) {
        hipLaunchKernelGGL((k_leptons_radiative<T, FK_MULTI>), gd, bd, 0, s, a, mode);
        return hipGetLastError();
    }
    switch (a.sa.f0.kind) {
    case QED_FIELD_CONST: hipLaunchKernelGGL((k_leptons_radiative<T, QED_FIELD_CONST>), gd, bd, 0, s, a, mode); break;
    case QED_FIELD_PW: hipLaunchKernelGGL((k_leptons_radiative<T, QED_FIELD_PW>), gd, bd, 0, s, a, mode); break;
    case QED_FIELD_GAUSS: hipLaunchKernelGGL((k_leptons_radiative<T, QED_FIELD_GAUSS>), gd, bd, 0, s, a, mode); break;
    case QED_FIELD_GRID2D:
        hipLaunchKernelGGL((k_leptons_radiative<T, QED_FIELD_GRID2D>), gd, bd, 0, s, a, mode);
        break;
    default: hipLaunchKernelGGL((k_leptons_radiative<T, QED_FIELD_NONE>), gd, bd, 0, s, a, mode); break;
    }
    return hipGetLastError();
}

hipError_t launch_radiative(qed_ctx *ctx, const SegArgs &sa, const qed_leptons &L, uint32_t mode, int64_t step,
                            hipStream_t s) {
    LeptonArgs a{};
    a.c = consts_of(ctx);
    a.sa = sa;
    a.L = L;
    a.step = step;
    a.step_dev = ctx->step_dev;
    a.status = ctx->status;
    if (ctx->cfg.precision == QED_MIXED) {
        a.tab = ctx->tab32;
        return launch_radiative_t<float>(a, mode, s);
    }
    a.tab = ctx->tab64;
    return launch_radiative_t<double>(a, mode, s);
}

hipError_t launch_advance_step(int64_t *step, int64_t by, hipStream_t s) {
    hipLaunchKernelGGL(k_advance_step, dim3(1), dim3(64), 0, s, step, by);
    return hipGetLastError();
}

hipError_t launch_compact(qed_ctx *ctx, const qed_photons &in, const qed_photons &out, hipStream_t s) {
    CompactArgs a{in, out, (EventRec *)ctx->staging, ctx->tile_counts, ctx->tile_off, ctx->launch};
    hipLaunchKernelGGL(k_compact_mark, dim3(tiles_grid(in.capacity)), dim3(BLOCK), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the live photons replace the contents of `out` (its count on entry is not a base)
    e = launch_scan(ctx, in.count, in.capacity, ctx->tile_counts, out.count, out.capacity, nullptr, 0, 0, s, 1);
    if (e != hipSuccess) return e;
    if (ctx->cfg.precision == QED_MIXED)
        hipLaunchKernelGGL(k_compact_copy<float>, dim3(stride_grid(in.capacity, 2048)), dim3(BLOCK), 0, s, a);
    else
        hipLaunchKernelGGL(k_compact_copy<double>, dim3(stride_grid(in.capacity, 2048)), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace qed
