// High-energy bremsstrahlung of electrons in a target slab (Sec. III.E): the direct
// Monte Carlo of the free path.  An electron inside x_lo <= x < x_hi with total energy E
// emits with probability P = 1 - exp(-n sigma(E) |v| dt) (the paper prints the exponent
// without its minus sign; this is the free-path probability it describes); the photon
// energy y E follows the cross-section above the cut k_cut, the photon moves along the
// electron's velocity, unpolarised, and the electron keeps its direction with energy
// E (1 - y).  sigma(E) and the energy draw come from the tables of qed_tables.hip.
//
// Three launches, as the other event steps: decide (one thread per electron: slab test,
// probability, draw, rank of the events in electron order, a staging record per event),
// the ordered scan of the per-tile counts (photon slots and ids), events (energy draw,
// photon written at its slot, electron momentum lowered).
#include "qed_dev.hpp"

namespace qed {
namespace {

constexpr uint32_t STREAM_BREMS = 3;

struct BremsArgs {
    Consts c;
    BremsDev m;
    const void *tab;           // the material's tables in T
    qed_leptons L;
    qed_photons G;
    int64_t step;
    const int64_t *step_dev;
    uint32_t *status;
    EventRec *stg;
    int *tile_counts;
    const int64_t *tile_off;
    const int64_t *launch;
};

// node j below E and the weight w of node j + 1 (false below the table; clamped above)
__device__ __forceinline__ bool br_locate(const BremsDev &m, double E, int &j, double &w, uint32_t &st) {
    const double pos = (log(E) - m.lnE0) * m.inv_dlnE;
    if (!(pos >= 0.0)) return false;
    if (pos >= (double)(BR_NE - 1)) {
        if (pos > (double)(BR_NE - 1)) st |= QED_ST_CLAMP;
        j = BR_NE - 2;
        w = 1.0;
        return true;
    }
    j = (int)pos;
    w = pos - j;
    return true;
}

template <class T>
__global__ __launch_bounds__(BLOCK) void k_brems_decide(BremsArgs a) {
    __shared__ int s_wave[BLOCK / 64];
    const int64_t n = clamp_count(a.L.count, a.L.capacity);
    const int64_t tile = blockIdx.x, i = tile * BLOCK + threadIdx.x;
    if (tile * BLOCK >= n) return;
    const T *tab = (const T *)a.tab;
    uint32_t st = 0;
    bool ev = false;
    double r1 = 0.0;
    if (i < n) {
        // the electron's record is read in one round trip (x, p and id together, streaming:
        // read once per step) even though electrons outside the slab need only x
        const uint32_t o = (uint32_t)i * 8u;
        const double x = ld_nt(a.L.x, o), px = ld_nt(a.L.px, o), py = ld_nt(a.L.py, o), pz = ld_nt(a.L.pz, o);
        const unsigned long long id = ld_nt(a.L.id, o);
        if (a.m.x_lo <= x && x < a.m.x_hi) {
            const double pp = sqrt(px * px + py * py + pz * pz), E = sqrt(1.0 + pp * pp);
            int j;
            double w;
            if (br_locate(a.m, E, j, w, st)) {
                const double sig = (1.0 - w) * (double)tab[j] + w * (double)tab[j + 1];
                if (sig > 0.0) {
                    const double P = -expm1(-(a.m.n_atoms * sig * (pp / E) * a.c.dt));
                    if (P > a.c.p_max) st |= QED_ST_PMAX;
                    double r[4];
                    uniform4(id, step_of(a), STREAM_BREMS, a.c.seed, r);
                    ev = r[0] < P;
                    r1 = r[1];
                }
            }
        }
    }
    int total;
    const int rank = block_rank(ev, total, s_wave);
    if (ev) {
        EventRec &rec = a.stg[tile * BLOCK + rank];
        rec.idx = i;
        rec.f[0] = r1;
    }
    if (threadIdx.x == 0) a.tile_counts[tile] = total;
    if (st) atomicOr(a.status, st);
}

// the photon variable u of draw r at energy E: the row pair's CDF at E's weight, the last
// node with F <= r, linear between nodes
template <class T>
__device__ double br_sample_u(const T *tab, int j, double w, double r) {
    const T *c0 = tab + BR_NE + (int64_t)j * BR_NU, *c1 = c0 + BR_NU;
    const double norm = (1.0 - w) * (double)tab[j] + w * (double)tab[j + 1];
    auto F = [&](int i) { return ((1.0 - w) * (double)c0[i] + w * (double)c1[i]) / norm; };
    int lo = 0, hi = BR_NU - 2;            // F(0) = 0 <= r; F(BR_NU - 1) = 1 > r
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (F(mid) <= r) lo = mid;
        else hi = mid - 1;
    }
    const double f0 = F(lo), d = F(lo + 1) - f0;
    double f = d > 0.0 ? (r - f0) / d : 0.0;
    f = fmin(fmax(f, 0.0), 1.0);
    return (lo + f) / (BR_NU - 1);
}

// one wavefront per group of BR_GROUP tiles (events are sparse, a few per tile, so a
// group's events fill about one wavefront)
constexpr int BR_GROUP = 16;

template <class T>
__global__ __launch_bounds__(BLOCK) void k_brems_events(BremsArgs a) {
    const int64_t n = clamp_count(a.L.count, a.L.capacity);
    const int64_t ntiles = (n + BLOCK - 1) / BLOCK;
    const int64_t t0 = ((int64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6)) * BR_GROUP;
    if (t0 >= ntiles) return;
    const int64_t base = a.launch[0], id0 = a.launch[2];
    const T *tab = (const T *)a.tab;
    uint32_t st = 0;
    group_events<BR_GROUP>(a.tile_counts, a.tile_off[t0], ntiles, t0, [&](int64_t e, int64_t slot) {
        const EventRec &rec = a.stg[slot];
        const int64_t i = rec.idx;
        const double px = a.L.px[i], py = a.L.py[i], pz = a.L.pz[i];
        // the photon's birth place and weight read here, with p: read after the stores below
        // (which may alias them, for all the compiler knows) each would wait for the store
        // before it, four round trips in a row
        const double bx = a.L.x[i], by = a.L.y[i], bz = a.L.z[i], bw = a.L.w[i];
        const double pp = sqrt(px * px + py * py + pz * pz), E = sqrt(1.0 + pp * pp);
        int j;
        double w;
        br_locate(a.m, E, j, w, st);      // as in the decide kernel (an event implies a node)
        const double u = br_sample_u<T>(tab, j, w, rec.f[0]);
        const double ymin = a.m.k_cut / E;
        const double ta = log(ymin / (1.0 - ymin)), tb = log(E - 1.0);   // logit range at E
        const double y = 1.0 / (1.0 + exp(-(ta + u * (tb - ta))));
        const double k = y * E, Ep = E - k;
        const double nx = px / pp, ny = py / pp, nz = pz / pp;
        const double s = sqrt(Ep * Ep - 1.0) / pp;
        a.L.px[i] = px * s;
        a.L.py[i] = py * s;
        a.L.pz[i] = pz * s;
        const int64_t pos = base + e;
        if (pos >= a.G.capacity) return;
        a.G.x[pos] = bx;
        a.G.y[pos] = by;
        a.G.z[pos] = bz;
        a.G.kx[pos] = k * nx;
        a.G.ky[pos] = k * ny;
        a.G.kz[pos] = k * nz;
        a.G.w[pos] = bw;
        // unpolarised; basis e1 = unit(y_hat - (y_hat . n) n), else from z_hat
        double ex = -ny * nx, ey = 1.0 - ny * ny, ez = -ny * nz;
        double nn = ex * ex + ey * ey + ez * ez;
        if (!(nn > 1e-12)) {
            ex = -nz * nx;
            ey = -nz * ny;
            ez = 1.0 - nz * nz;
            nn = ex * ex + ey * ey + ez * ez;
        }
        const double inv = 1.0 / sqrt(nn);
        ((T *)a.G.xi1)[pos] = (T)0;
        ((T *)a.G.xi2)[pos] = (T)0;
        ((T *)a.G.xi3)[pos] = (T)0;
        ((T *)a.G.e1x)[pos] = (T)(ex * inv);
        ((T *)a.G.e1y)[pos] = (T)(ey * inv);
        ((T *)a.G.e1z)[pos] = (T)(ez * inv);
        a.G.id[pos] = (unsigned long long)(id0 + e);
        a.G.alive[pos] = 1;
    });
    if (st) atomicOr(a.status, st);
}

template <class T>
hipError_t launch_brems_t(qed_ctx *ctx, BremsArgs &a, hipStream_t s) {
    const int64_t ntiles = (a.L.capacity + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL(k_brems_decide<T>, dim3((unsigned)(ntiles < 1 ? 1 : ntiles)), dim3(BLOCK), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_scan_events(ctx, a.L.count, a.L.capacity, ctx->tile_counts, a.G.count, a.G.capacity, 1, s);
    if (e != hipSuccess) return e;
    const int64_t groups = (ntiles + BR_GROUP - 1) / BR_GROUP, per = BLOCK / 64;
    const int64_t nb = (groups + per - 1) / per;
    hipLaunchKernelGGL(k_brems_events<T>, dim3((unsigned)(nb < 1 ? 1 : nb)), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_brems(qed_ctx *ctx, const qed_leptons &L, const qed_photons &G, int64_t step, hipStream_t s) {
    BremsArgs a{};
    a.c = consts_of(ctx);
    a.m = ctx->br;
    a.L = L;
    a.G = G;
    a.step = step;
    a.step_dev = ctx->step_dev;
    a.status = ctx->status;
    a.stg = (EventRec *)ctx->staging;
    a.tile_counts = ctx->tile_counts;
    a.tile_off = ctx->tile_off;
    a.launch = ctx->launch;
    if (ctx->cfg.precision == QED_MIXED) {
        a.tab = ctx->br_tab32;
        return launch_brems_t<float>(ctx, a, s);
    }
    a.tab = ctx->br_tab64;
    return launch_brems_t<double>(ctx, a, s);
}

}  // namespace qed
