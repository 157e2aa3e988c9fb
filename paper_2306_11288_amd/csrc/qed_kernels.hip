// HIP kernels of the QED particle step for gfx950 and their host launchers.
//
// Layout: one thread per particle, 256-thread blocks (4 wave64s).  Kernels that append
// particles run a persistent grid that takes 256-particle tiles from a ticket counter in
// index order; each tile ranks its events with a wavefront ballot + popcount, combines
// the four waves in LDS, and obtains the number of events before it by a decoupled
// look-back over the earlier tiles.  Output order is therefore the parent index order for
// any grid size and any scheduling.  The last block to finish publishes the new list
// counts and the id counter and clears the scan state for the next launch.
#include "qed_dev.hpp"

namespace qed {

// ------------------------------------------------------------------------- scan helpers
constexpr unsigned long long FLAG_AGG = 1ull << 62, FLAG_INC = 2ull << 62, VAL_MASK = (1ull << 62) - 1;
constexpr int SPIN_LIMIT = 1 << 24;

__device__ __forceinline__ void st_publish(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long st_read(unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Number of events in all tiles before `tile` (called by one thread of the block).
__device__ long long tile_lookback(const ScanState &sc, long long tile, long long agg, uint32_t *status) {
    if (tile == 0) {
        st_publish(sc.tile_status, FLAG_INC | (unsigned long long)agg);
        return 0;
    }
    st_publish(sc.tile_status + tile, FLAG_AGG | (unsigned long long)agg);
    long long excl = 0, j = tile - 1;
    int spins = 0;
    while (j >= 0) {
        const unsigned long long s = st_read(sc.tile_status + j);
        const unsigned long long flag = s & ~VAL_MASK;
        if (flag == 0) {
            if (++spins > SPIN_LIMIT) {     // cannot happen while earlier tiles progress
                atomicOr(status, (uint32_t)QED_ST_SCAN);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += (long long)(s & VAL_MASK);
        if (flag == FLAG_INC) break;
        --j;
    }
    st_publish(sc.tile_status + tile, FLAG_INC | (unsigned long long)(excl + agg));
    return excl;
}

struct AppendShared {
    int wave[BLOCK / 64];
    long long tile;
    long long excl;
    long long base[3];   // launch bases (output counts, id counter) as seen by tile 0
    int last;
};

// Block-wide exclusive rank of a 0/1 flag: wave ballot + popcount, waves combined in LDS.
__device__ __forceinline__ int block_rank(bool flag, int &total, AppendShared &sh) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const unsigned long long m = __ballot(flag);
    const int below = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) sh.wave[wid] = __popcll(m);
    __syncthreads();
    int pre = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) {
        const int v = sh.wave[w];
        pre += w < wid ? v : 0;
        total += v;
    }
    return pre + below;
}

// Next tile from the ticket counter (one atomic per block), broadcast through LDS.
__device__ __forceinline__ long long next_tile(const ScanState &sc, AppendShared &sh) {
    __syncthreads();
    if (threadIdx.x == 0) sh.tile = (long long)atomicAdd(sc.ticket, 1u);
    __syncthreads();
    return sh.tile;
}

// Tile rank -> global rank; tile 0 also records the launch bases (read before any
// output of this launch is published) for every other block to read after its look-back.
__device__ __forceinline__ void tile_offsets(const ScanState &sc, long long tile, int total, AppendShared &sh,
                                             uint32_t *status, long long b0, long long b1, long long b2) {
    if (threadIdx.x == 0) {
        if (tile == 0) {
            sc.info[0] = b0;
            sc.info[1] = b1;
            sc.info[2] = b2;
        }
        sh.excl = tile_lookback(sc, tile, total, status);
        // ordered after the look-back's acquire (tile 0 wrote info before its release)
        sh.base[0] = tile == 0 ? b0 : sc.info[0];
        sh.base[1] = tile == 0 ? b1 : sc.info[1];
        sh.base[2] = tile == 0 ? b2 : sc.info[2];
    }
    __syncthreads();
}

// Last block out: total events = inclusive value of the last tile.  Returns it in sh.excl
// (or -1 for blocks that are not last); the caller publishes counts, then calls
// scan_reset.
__device__ __forceinline__ bool scan_last_block(const ScanState &sc, long long ntiles, AppendShared &sh) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int e = __hip_atomic_fetch_add(sc.exits, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        sh.last = (e == gridDim.x - 1);
        if (sh.last) {
            __threadfence();
            sh.excl = ntiles > 0 ? (long long)(st_read(sc.tile_status + ntiles - 1) & VAL_MASK) : 0;
            sh.base[0] = sc.info[0];
            sh.base[1] = sc.info[1];
            sh.base[2] = sc.info[2];
        }
    }
    __syncthreads();
    return sh.last != 0;
}
__device__ __forceinline__ void scan_reset(const ScanState &sc, long long ntiles) {
    for (long long j = threadIdx.x; j < ntiles; j += BLOCK) sc.tile_status[j] = 0;
    if (threadIdx.x == 0) {
        *sc.ticket = 0;
        *sc.exits = 0;
    }
}

// ------------------------------------------------------------------------- segments
__device__ __forceinline__ const qed_field *seg_field(const SegArgs &sa, int64_t i) {
    for (int s = 0; s < sa.nseg; ++s)
        if (i >= sa.seg[s].begin && i < sa.seg[s].end) return &sa.seg[s].field;
    return nullptr;
}
template <class FT>
__device__ __forceinline__ void fields_for(const SegArgs &sa, int64_t i, double t, const V3<double> &r,
                                           V3<double> &E, V3<double> &B) {
    const qed_field *f = seg_field(sa, i);
    if (f) {
        field_at<FT>(*f, t, r.x, r.y, r.z, E, B);
    } else {
        E = {0, 0, 0};
        B = {0, 0, 0};
    }
}

// ------------------------------------------------------------------------- leptons
struct LeptonArgs {
    Consts c;
    const void *tab;
    SegArgs sa;
    qed_leptons L;
    qed_photons out;
    int has_out;
    double *E6;
    int64_t step;
    uint32_t *status;
    unsigned long long *next_id;
    ScanState sc;
};

template <class T>
__device__ __forceinline__ void push_one(const LeptonArgs &a, double q, double dt, const V3<double> &E,
                                         const V3<double> &B, V3<double> &r, V3<double> &p, V3<T> &S, uint32_t &st) {
    V3<double> pm, pp;
    boris(q, dt, E, B, p, pm, pp);
    bmt<T>(q, a.c.a_e, dt, E, B, pm, pp, S);
    const double ig = dt / sqrt(1.0 + dot(p, p));
    r = r + ig * p;
    if (!isfinite(p.x + p.y + p.z + r.x + r.y + r.z) || !isfinite((double)(S.x + S.y + S.z))) st |= QED_ST_NAN;
}

// device list counts are trusted only up to the list capacity
__device__ __forceinline__ int64_t clamp_count(const int64_t *count, int64_t capacity) {
    const int64_t n = *count;
    return n < 0 ? 0 : (n > capacity ? capacity : n);
}

// gather and/or push without appends: grid-stride loop
template <class T, bool WRITE_E6, bool PUSH, bool E6_IN>
__global__ __launch_bounds__(BLOCK) void k_leptons_simple(LeptonArgs a) {
    const int64_t n = clamp_count(a.L.count, a.L.capacity);
    const double dt = a.c.dt, t = (double)a.step * dt, q = (double)a.L.charge;
    T *sx = (T *)a.L.sx, *sy = (T *)a.L.sy, *sz = (T *)a.L.sz;
    uint32_t st = 0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        V3<double> r = {a.L.x[i], a.L.y[i], a.L.z[i]}, E, B;
        if constexpr (E6_IN) {
            const double *e = a.E6 + 6 * i;
            E = {e[0], e[1], e[2]};
            B = {e[3], e[4], e[5]};
        } else {
            fields_for<T>(a.sa, i, t, r, E, B);
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

// NCS (optionally fused with gather + push); photons appended in lepton order
template <class T, bool PUSH>
__global__ __launch_bounds__(BLOCK) void k_leptons_emit(LeptonArgs a) {
    __shared__ AppendShared sh;
    const Tabs<T> tb = {(const T *)a.tab};
    const int64_t n = clamp_count(a.L.count, a.L.capacity);
    const long long ntiles = (n + BLOCK - 1) / BLOCK;
    const double dt = a.c.dt, t = (double)a.step * dt, q = (double)a.L.charge;
    T *sx = (T *)a.L.sx, *sy = (T *)a.L.sy, *sz = (T *)a.L.sz;
    uint32_t st = 0;
    for (;;) {
        const long long tile = next_tile(a.sc, sh);
        if (tile >= ntiles) break;
        const int64_t i = tile * BLOCK + threadIdx.x;
        bool ev = false;
        NcsPhoton<T> ph;
        V3<double> r = {0, 0, 0};
        double w = 0;
        if (i < n) {
            r = {a.L.x[i], a.L.y[i], a.L.z[i]};
            V3<double> E, B, p = {a.L.px[i], a.L.py[i], a.L.pz[i]};
            V3<T> S = {sx[i], sy[i], sz[i]};
            if constexpr (PUSH) {
                fields_for<T>(a.sa, i, t, r, E, B);
                push_one<T>(a, q, dt, E, B, r, p, S, st);
                a.L.x[i] = r.x; a.L.y[i] = r.y; a.L.z[i] = r.z;
            } else {
                const double *e = a.E6 + 6 * i;
                E = {e[0], e[1], e[2]};
                B = {e[3], e[4], e[5]};
            }
            ev = ncs_step<T>(a.c, tb, q, p, S, E, B, a.L.id[i], a.step, st, ph);
            a.L.px[i] = p.x; a.L.py[i] = p.y; a.L.pz[i] = p.z;
            sx[i] = S.x; sy[i] = S.y; sz[i] = S.z;
            if (ev) w = a.L.w[i];
        }
        int total;
        const int rank = block_rank(ev, total, sh);
        long long b0 = 0, b2 = 0;
        if (tile == 0 && threadIdx.x == 0) {
            b0 = a.has_out ? (long long)*a.out.count : 0;
            b2 = (long long)*a.next_id;
        }
        tile_offsets(a.sc, tile, total, sh, a.status, b0, 0, b2);
        if (ev && a.has_out) {
            const long long k = sh.excl + rank, pos = sh.base[0] + k;
            if (pos < a.out.capacity) {
                a.out.x[pos] = r.x; a.out.y[pos] = r.y; a.out.z[pos] = r.z;
                a.out.kx[pos] = ph.k.x; a.out.ky[pos] = ph.k.y; a.out.kz[pos] = ph.k.z;
                a.out.w[pos] = w;
                ((T *)a.out.xi1)[pos] = ph.xi.x; ((T *)a.out.xi2)[pos] = ph.xi.y; ((T *)a.out.xi3)[pos] = ph.xi.z;
                ((T *)a.out.e1x)[pos] = ph.e1.x; ((T *)a.out.e1y)[pos] = ph.e1.y; ((T *)a.out.e1z)[pos] = ph.e1.z;
                a.out.id[pos] = (unsigned long long)(sh.base[2] + k);
                a.out.alive[pos] = 1;
            } else {
                st |= QED_ST_OVERFLOW;
            }
        }
    }
    if (st) atomicOr(a.status, st);
    if (!scan_last_block(a.sc, ntiles, sh)) return;
    if (threadIdx.x == 0 && ntiles > 0) {
        const long long tot = sh.excl;
        *a.next_id = (unsigned long long)(sh.base[2] + tot);
        if (a.has_out) {
            const long long c = sh.base[0] + tot;
            *a.out.count = c < a.out.capacity ? c : a.out.capacity;
        }
    }
    scan_reset(a.sc, ntiles);
}

// ------------------------------------------------------------------------- photons
struct PhotonArgs {
    Consts c;
    const void *tab;
    qed_field field;
    qed_photons G;
    qed_leptons em, ep;
    int has_em, has_ep;
    int do_vb, do_nbw, do_move;
    int64_t step;
    uint32_t *status;
    unsigned long long *next_id;
    ScanState sc;
};

template <class T>
__device__ __forceinline__ bool photon_one(const PhotonArgs &a, const Tabs<T> &tb, int64_t j, double t, V3<double> &x,
                                           uint32_t &st, PairOut<T> &po) {
    const V3<double> k = {a.G.kx[j], a.G.ky[j], a.G.kz[j]};
    T *xi1 = (T *)a.G.xi1, *xi2 = (T *)a.G.xi2, *xi3 = (T *)a.G.xi3;
    T *e1x = (T *)a.G.e1x, *e1y = (T *)a.G.e1y, *e1z = (T *)a.G.e1z;
    V3<T> xi = {xi1[j], xi2[j], xi3[j]}, e1 = {e1x[j], e1y[j], e1z[j]};
    V3<double> E, B;
    field_at<T>(a.field, t, x.x, x.y, x.z, E, B);
    const bool ev = photon_step<T>(a.c, tb, k, xi, e1, E, B, a.G.id[j], a.step, a.do_vb, a.do_nbw, st, po);
    xi1[j] = xi.x; xi2[j] = xi.y; xi3[j] = xi.z;
    e1x[j] = e1.x; e1y[j] = e1.y; e1z[j] = e1.z;
    if (ev) {
        a.G.alive[j] = 0;
    } else if (a.do_move) {
        const double ie = a.c.dt / sqrt(dot(k, k));
        const V3<double> xn = x + ie * k;
        a.G.x[j] = xn.x; a.G.y[j] = xn.y; a.G.z[j] = xn.z;
    }
    return ev;
}

// rotation / VB / move without pair creation: grid-stride loop
template <class T>
__global__ __launch_bounds__(BLOCK) void k_photons_simple(PhotonArgs a) {
    const Tabs<T> tb = {(const T *)a.tab};
    const int64_t n = clamp_count(a.G.count, a.G.capacity);
    const double t = (double)a.step * a.c.dt;
    uint32_t st = 0;
    for (int64_t j = (int64_t)blockIdx.x * BLOCK + threadIdx.x; j < n; j += (int64_t)gridDim.x * BLOCK) {
        if (!a.G.alive[j]) continue;
        V3<double> x = {a.G.x[j], a.G.y[j], a.G.z[j]};
        PairOut<T> po;
        photon_one<T>(a, tb, j, t, x, st, po);
    }
    if (st) atomicOr(a.status, st);
}

// with NBW: pairs appended in photon order
template <class T>
__global__ __launch_bounds__(BLOCK) void k_photons_pair(PhotonArgs a) {
    __shared__ AppendShared sh;
    const Tabs<T> tb = {(const T *)a.tab};
    const int64_t n = clamp_count(a.G.count, a.G.capacity);
    const long long ntiles = (n + BLOCK - 1) / BLOCK;
    const double t = (double)a.step * a.c.dt;
    uint32_t st = 0;
    for (;;) {
        const long long tile = next_tile(a.sc, sh);
        if (tile >= ntiles) break;
        const int64_t j = tile * BLOCK + threadIdx.x;
        bool ev = false;
        PairOut<T> po;
        V3<double> x = {0, 0, 0};
        double w = 0;
        if (j < n && a.G.alive[j]) {
            x = {a.G.x[j], a.G.y[j], a.G.z[j]};
            ev = photon_one<T>(a, tb, j, t, x, st, po);
            if (ev) w = a.G.w[j];
        }
        int total;
        const int rank = block_rank(ev, total, sh);
        long long b0 = 0, b1 = 0, b2 = 0;
        if (tile == 0 && threadIdx.x == 0) {
            b0 = a.has_em ? (long long)*a.em.count : 0;
            b1 = a.has_ep ? (long long)*a.ep.count : 0;
            b2 = (long long)*a.next_id;
        }
        tile_offsets(a.sc, tile, total, sh, a.status, b0, b1, b2);
        if (ev) {
            const long long k = sh.excl + rank;
            const unsigned long long id0 = (unsigned long long)(sh.base[2] + 2 * k);
            const qed_leptons *Ls[2] = {&a.em, &a.ep};
            const int has[2] = {a.has_em, a.has_ep};
            for (int s = 0; s < 2; ++s) {
                if (!has[s]) continue;
                const qed_leptons &L = *Ls[s];
                const long long pos = sh.base[s] + k;
                if (pos >= L.capacity) {
                    st |= QED_ST_OVERFLOW;
                    continue;
                }
                const V3<double> &p = s == 0 ? po.pm : po.pp;
                const V3<T> &S = s == 0 ? po.Sm : po.Sp;
                L.x[pos] = x.x; L.y[pos] = x.y; L.z[pos] = x.z;
                L.px[pos] = p.x; L.py[pos] = p.y; L.pz[pos] = p.z;
                ((T *)L.sx)[pos] = S.x; ((T *)L.sy)[pos] = S.y; ((T *)L.sz)[pos] = S.z;
                L.w[pos] = w;
                L.id[pos] = id0 + (unsigned long long)s;
            }
        }
    }
    if (st) atomicOr(a.status, st);
    if (!scan_last_block(a.sc, ntiles, sh)) return;
    if (threadIdx.x == 0 && ntiles > 0) {
        const long long tot = sh.excl;
        *a.next_id = (unsigned long long)(sh.base[2] + 2 * tot);
        if (a.has_em) {
            const long long c = sh.base[0] + tot;
            *a.em.count = c < a.em.capacity ? c : a.em.capacity;
        }
        if (a.has_ep) {
            const long long c = sh.base[1] + tot;
            *a.ep.count = c < a.ep.capacity ? c : a.ep.capacity;
        }
    }
    scan_reset(a.sc, ntiles);
}

// ------------------------------------------------------------------------- compaction
struct CompactArgs {
    qed_photons in, out;
    uint32_t *status;
    ScanState sc;
};
template <class T>
__global__ __launch_bounds__(BLOCK) void k_compact(CompactArgs a) {
    __shared__ AppendShared sh;
    const int64_t n = clamp_count(a.in.count, a.in.capacity);
    const long long ntiles = (n + BLOCK - 1) / BLOCK;
    uint32_t st = 0;
    for (;;) {
        const long long tile = next_tile(a.sc, sh);
        if (tile >= ntiles) break;
        const int64_t j = tile * BLOCK + threadIdx.x;
        const bool live = j < n && a.in.alive[j];
        int total;
        const int rank = block_rank(live, total, sh);
        tile_offsets(a.sc, tile, total, sh, a.status, 0, 0, 0);
        if (live) {
            const long long pos = sh.excl + rank;
            if (pos < a.out.capacity) {
                a.out.x[pos] = a.in.x[j]; a.out.y[pos] = a.in.y[j]; a.out.z[pos] = a.in.z[j];
                a.out.kx[pos] = a.in.kx[j]; a.out.ky[pos] = a.in.ky[j]; a.out.kz[pos] = a.in.kz[j];
                a.out.w[pos] = a.in.w[j];
                ((T *)a.out.xi1)[pos] = ((const T *)a.in.xi1)[j];
                ((T *)a.out.xi2)[pos] = ((const T *)a.in.xi2)[j];
                ((T *)a.out.xi3)[pos] = ((const T *)a.in.xi3)[j];
                ((T *)a.out.e1x)[pos] = ((const T *)a.in.e1x)[j];
                ((T *)a.out.e1y)[pos] = ((const T *)a.in.e1y)[j];
                ((T *)a.out.e1z)[pos] = ((const T *)a.in.e1z)[j];
                a.out.id[pos] = a.in.id[j];
                a.out.alive[pos] = 1;
            } else {
                st |= QED_ST_OVERFLOW;
            }
        }
    }
    if (st) atomicOr(a.status, st);
    if (!scan_last_block(a.sc, ntiles, sh)) return;
    if (threadIdx.x == 0) {
        const long long c = sh.excl;
        *a.out.count = c < a.out.capacity ? c : a.out.capacity;
    }
    scan_reset(a.sc, ntiles);
}

// ------------------------------------------------------------------------- launchers
static Consts consts_of(const qed_ctx *ctx) {
    return {ctx->cfg.xi_L, ctx->cfg.alpha, ctx->cfg.a_e, ctx->cfg.dt, ctx->cfg.p_max, ctx->cfg.seed, ctx->cfg.procs};
}
static int simple_grid(int64_t cap) {
    int64_t b = (cap + BLOCK - 1) / BLOCK;
    if (b > 65536) b = 65536;
    return b < 1 ? 1 : (int)b;
}
static int append_grid(const qed_ctx *ctx, int64_t cap) {
    int64_t b = (cap + BLOCK - 1) / BLOCK;
    if (b > ctx->grid_blocks) b = ctx->grid_blocks;
    return b < 1 ? 1 : (int)b;
}

template <class T>
static hipError_t launch_leptons_t(qed_ctx *ctx, LeptonMode mode, const LeptonArgs &a, hipStream_t s) {
    const int gs = simple_grid(a.L.capacity), ga = append_grid(ctx, a.L.capacity);
    switch (mode) {
    case LM_GATHER:
        hipLaunchKernelGGL((k_leptons_simple<T, true, false, false>), dim3(gs), dim3(BLOCK), 0, s, a);
        break;
    case LM_PUSH:
        if (a.E6) hipLaunchKernelGGL((k_leptons_simple<T, false, true, true>), dim3(gs), dim3(BLOCK), 0, s, a);
        else hipLaunchKernelGGL((k_leptons_simple<T, false, true, false>), dim3(gs), dim3(BLOCK), 0, s, a);
        break;
    case LM_EMIT:
        hipLaunchKernelGGL((k_leptons_emit<T, false>), dim3(ga), dim3(BLOCK), 0, s, a);
        break;
    case LM_FUSED:
        if (a.c.procs & QED_PROC_NCS) hipLaunchKernelGGL((k_leptons_emit<T, true>), dim3(ga), dim3(BLOCK), 0, s, a);
        else hipLaunchKernelGGL((k_leptons_simple<T, false, true, false>), dim3(gs), dim3(BLOCK), 0, s, a);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_leptons(qed_ctx *ctx, LeptonMode mode, const SegArgs &sa, const qed_leptons &L, double *E6,
                          const qed_photons *out, int64_t step, hipStream_t s) {
    LeptonArgs a{};
    a.c = consts_of(ctx);
    a.sa = sa;
    a.L = L;
    a.has_out = out != nullptr;
    if (out) a.out = *out;
    a.E6 = E6;
    a.step = step;
    a.status = ctx->status;
    a.next_id = ctx->next_id;
    a.sc = ctx->scan;
    if (ctx->cfg.precision == QED_MIXED) {
        a.tab = ctx->tab32;
        return launch_leptons_t<float>(ctx, mode, a, s);
    }
    a.tab = ctx->tab64;
    return launch_leptons_t<double>(ctx, mode, a, s);
}

hipError_t launch_photons(qed_ctx *ctx, PhotonMode mode, const SegArgs &sa, const qed_photons &G,
                          const qed_leptons *em, const qed_leptons *ep, int64_t step, hipStream_t s) {
    PhotonArgs a{};
    a.c = consts_of(ctx);
    a.field = sa.seg[0].field;
    a.G = G;
    a.has_em = em != nullptr;
    a.has_ep = ep != nullptr;
    if (em) a.em = *em;
    if (ep) a.ep = *ep;
    a.do_vb = (mode != PM_PAIR) && (ctx->cfg.procs & QED_PROC_VB);
    a.do_nbw = (mode != PM_BIREF) && (ctx->cfg.procs & QED_PROC_NBW);
    a.do_move = mode != PM_BIREF;
    a.step = step;
    a.status = ctx->status;
    a.next_id = ctx->next_id;
    a.sc = ctx->scan;
    const bool mixed = ctx->cfg.precision == QED_MIXED;
    a.tab = mixed ? (const void *)ctx->tab32 : (const void *)ctx->tab64;
    const int gs = simple_grid(G.capacity), ga = append_grid(ctx, G.capacity);
    if (a.do_nbw) {
        if (mixed) hipLaunchKernelGGL(k_photons_pair<float>, dim3(ga), dim3(BLOCK), 0, s, a);
        else hipLaunchKernelGGL(k_photons_pair<double>, dim3(ga), dim3(BLOCK), 0, s, a);
    } else {
        if (mixed) hipLaunchKernelGGL(k_photons_simple<float>, dim3(gs), dim3(BLOCK), 0, s, a);
        else hipLaunchKernelGGL(k_photons_simple<double>, dim3(gs), dim3(BLOCK), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_compact(qed_ctx *ctx, const qed_photons &in, const qed_photons &out, hipStream_t s) {
    CompactArgs a{in, out, ctx->status, ctx->scan};
    const int ga = append_grid(ctx, in.capacity);
    if (ctx->cfg.precision == QED_MIXED) hipLaunchKernelGGL(k_compact<float>, dim3(ga), dim3(BLOCK), 0, s, a);
    else hipLaunchKernelGGL(k_compact<double>, dim3(ga), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace qed
