// C ABI of libqed: argument validation, context lifetime and kernel dispatch.
// Argument errors are returned synchronously with a message in qed_last_error and
// nothing is enqueued; device-side conditions go to the sticky status word.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cmath>
#include <new>
#include <vector>
#include "qed_internal.hpp"

using namespace qed;

namespace {

constexpr int64_t MAX_TILES = 1 << 20;   // ordered-append tiles: lists up to 2^28 particles
constexpr int64_t GROUP_TOT_LEN = MAX_TILES / EV_GROUP + 1;

qed_status fail(qed_ctx *ctx, qed_status code, const char *fmt, ...) {
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->err, sizeof ctx->err, fmt, ap);
        va_end(ap);
    }
    return code;
}
qed_status hip_fail(qed_ctx *ctx, hipError_t e, const char *where) {
    return fail(ctx, QED_EHIP, "%s: %s", where, hipGetErrorString(e));
}

qed_status check_field(qed_ctx *ctx, const qed_field &f) {
    switch (f.kind) {
    case QED_FIELD_NONE:
    case QED_FIELD_CONST:
        return QED_OK;
    case QED_FIELD_PW:
    case QED_FIELD_GAUSS:
        if (!(f.ncycles > 0)) return fail(ctx, QED_EARG, "field: ncycles must be positive");
        if (f.kind == QED_FIELD_GAUSS && !(f.w0 > 0)) return fail(ctx, QED_EARG, "field: w0 must be positive");
        return QED_OK;
    case QED_FIELD_GRID2D:
        for (int c = 0; c < 6; ++c)
            if (!f.grid[c]) return fail(ctx, QED_EARG, "field: grid component %d is NULL", c);
        if (f.nx <= 0 || f.ny <= 0) return fail(ctx, QED_EARG, "field: grid size must be positive");
        if (!(f.dx > 0) || !(f.dy > 0)) return fail(ctx, QED_EARG, "field: grid spacing must be positive");
        return QED_OK;
    }
    return fail(ctx, QED_EARG, "field: unknown kind %d", f.kind);
}

}  // namespace

FieldDev qed::field_dev(const qed_field &f) {
    constexpr double PI = 3.141592653589793;
    FieldDev d;
    std::memset(&d, 0, sizeof d);
    d.kind = f.kind;
    d.circular = f.circular;
    if (f.kind == QED_FIELD_CONST) {
        for (int c = 0; c < 3; ++c) {
            d.c.e0[c] = f.e0[c];
            d.c.b0[c] = f.b0[c];
        }
    } else if (f.kind == QED_FIELD_GRID2D) {
        for (int c = 0; c < 6; ++c) d.g.g[c] = f.grid[c];
        d.g.nx = f.nx;
        d.g.ny = f.ny;
        d.g.inv_dx = 1.0 / f.dx;
        d.g.inv_dy = 1.0 / f.dy;
        d.g.gx0 = f.gx0;
        d.g.gy0 = f.gy0;
    } else if (f.kind == QED_FIELD_PW || f.kind == QED_FIELD_GAUSS) {
        PulseDev &p = d.p;
        p.a0 = f.a0;
        p.phase0 = f.phase0;
        p.phi_start = f.phi_start;
        p.L = 2.0 * PI * f.ncycles;
        p.pi_over_L = PI / p.L;
        p.inv_L = 1.0 / p.L;
        p.inv_2L = 0.5 * p.inv_L;
        p.cp = std::cos(f.pol_angle);
        p.sp = std::sin(f.pol_angle);
        p.x_focus = f.x_focus;
        p.w0sq = f.w0 * f.w0;
        p.zr = 0.5 * p.w0sq;
        p.inv_zr = p.zr > 0 ? 1.0 / p.zr : 0.0;
        p.inv_w0sq = p.w0sq > 0 ? 1.0 / p.w0sq : 0.0;
    }
    return d;
}

namespace {

qed_status seg_args(qed_ctx *ctx, const qed_segment *segs, int nseg, SegArgs &sa, hipStream_t stream) {
    if (!segs) return fail(ctx, QED_EARG, "segments: NULL");
    if (nseg < 1 || nseg > MAX_SEG) return fail(ctx, QED_EARG, "segments: nseg must be in [1, %d]", MAX_SEG);
    for (int s = 0; s < nseg; ++s) {
        if (segs[s].begin < 0 || segs[s].end < segs[s].begin)
            return fail(ctx, QED_EARG, "segment %d: bad range [%lld, %lld)", s, (long long)segs[s].begin,
                        (long long)segs[s].end);
        if (s > 0 && segs[s].begin < segs[s - 1].end)
            return fail(ctx, QED_EARG, "segment %d: ranges must be sorted and disjoint", s);
        const qed_status st = check_field(ctx, segs[s].field);
        if (st != QED_OK) return st;
    }
    sa.nseg = nseg;
    sa.begin0 = segs[0].begin;
    sa.end0 = segs[0].end;
    sa.f0 = field_dev(segs[0].field);
    sa.segs = nullptr;
    if (nseg == 1) return QED_OK;
    // several segments: upload unless identical to the list already on the device
    const size_t bytes = sizeof(DevSegment) * (size_t)nseg;
    std::vector<DevSegment> dev((size_t)nseg);
    for (int k = 0; k < nseg; ++k) {
        std::memset(&dev[k], 0, sizeof(DevSegment));   // padding too, for the comparison below
        dev[k].begin = segs[k].begin;
        dev[k].end = segs[k].end;
        dev[k].f = field_dev(segs[k].field);
    }
    if (nseg != ctx->nseg_dev || std::memcmp(ctx->hsegs, dev.data(), bytes) != 0) {
        hipError_t e = hipSuccess;
        if (ctx->nseg_dev > 0) e = hipEventSynchronize(ctx->seg_copied);   // host staging reusable
        if (e == hipSuccess && nseg > ctx->nseg_cap) {
            hipFree(ctx->dsegs);
            hipHostFree(ctx->hsegs);
            ctx->dsegs = nullptr;
            ctx->hsegs = nullptr;
            ctx->nseg_cap = 0;
            e = hipMalloc(&ctx->dsegs, bytes);
            if (e == hipSuccess) e = hipHostMalloc((void **)&ctx->hsegs, bytes, hipHostMallocDefault);
            if (e == hipSuccess) ctx->nseg_cap = nseg;
        }
        if (e == hipSuccess) {
            std::memcpy(ctx->hsegs, dev.data(), bytes);
            e = hipMemcpyAsync(ctx->dsegs, ctx->hsegs, bytes, hipMemcpyHostToDevice, stream);
        }
        if (e == hipSuccess) e = hipEventRecord(ctx->seg_copied, stream);
        if (e != hipSuccess) {
            ctx->nseg_dev = 0;
            return hip_fail(ctx, e, "segment upload");
        }
        ctx->nseg_dev = nseg;
    }
    sa.segs = ctx->dsegs;
    return QED_OK;
}

qed_status check_leptons(qed_ctx *ctx, const qed_leptons *L, const char *what) {
    if (!L) return fail(ctx, QED_EARG, "%s: NULL", what);
    if (!L->x || !L->y || !L->z || !L->px || !L->py || !L->pz || !L->w || !L->sx || !L->sy || !L->sz || !L->id ||
        !L->count)
        return fail(ctx, QED_EARG, "%s: NULL array", what);
    if (L->capacity < 0 || L->capacity > MAX_TILES * BLOCK)
        return fail(ctx, QED_EARG, "%s: capacity %lld outside [0, %lld]", what, (long long)L->capacity,
                    (long long)(MAX_TILES * BLOCK));
    if (L->charge != -1 && L->charge != 1) return fail(ctx, QED_EARG, "%s: charge must be -1 or +1", what);
    return QED_OK;
}
qed_status check_photons(qed_ctx *ctx, const qed_photons *G, const char *what) {
    if (!G) return fail(ctx, QED_EARG, "%s: NULL", what);
    if (!G->x || !G->y || !G->z || !G->kx || !G->ky || !G->kz || !G->w || !G->xi1 || !G->xi2 || !G->xi3 ||
        !G->e1x || !G->e1y || !G->e1z || !G->id || !G->alive || !G->count)
        return fail(ctx, QED_EARG, "%s: NULL array", what);
    if (G->capacity < 0 || G->capacity > MAX_TILES * BLOCK)
        return fail(ctx, QED_EARG, "%s: capacity %lld outside [0, %lld]", what, (long long)G->capacity,
                    (long long)(MAX_TILES * BLOCK));
    return QED_OK;
}
qed_status ready(qed_ctx *ctx) {
    if (!ctx) return QED_EARG;
    ctx->err[0] = 0;
    if (!ctx->tab64) return fail(ctx, QED_ESTATE, "context has no tables");
    return QED_OK;
}
qed_status launched(qed_ctx *ctx, hipError_t e, const char *where) {
    return e == hipSuccess ? QED_OK : hip_fail(ctx, e, where);
}

void free_ctx(qed_ctx *c) {
    if (!c) return;
    hipFree(c->tab64);
    hipFree(c->tab32);
    hipFree(c->status);
    hipFree(c->next_id);
    hipFree(c->tile_counts);
    hipFree(c->group_tot);
    hipFree(c->tile_off);
    hipFree(c->launch);
    hipFree(c->staging);
    hipFree(c->dsegs);
    if (c->hsegs) hipHostFree(c->hsegs);
    if (c->seg_copied) hipEventDestroy(c->seg_copied);
    delete c;
}

// The event staging area holds one record per particle of the largest list passed so far.
// Growing it synchronises the device (hipFree); lists of a fixed size allocate once.
qed_status ensure_staging(qed_ctx *ctx, int64_t capacity) {
    const int64_t need = ((capacity + BLOCK - 1) / BLOCK) * BLOCK;
    if (need <= ctx->staging_cap) return QED_OK;
    hipError_t e = hipSuccess;
    if (ctx->staging) e = hipFree(ctx->staging);
    ctx->staging = nullptr;
    ctx->staging_cap = 0;
    if (e == hipSuccess) e = hipMalloc(&ctx->staging, (size_t)need * STAGING_SLOT);
    if (e != hipSuccess) return fail(ctx, QED_ENOMEM, "staging buffer of %lld records: %s", (long long)need,
                                     hipGetErrorString(e));
    ctx->staging_cap = need;
    return QED_OK;
}

}  // namespace

extern "C" {

qed_status qed_init_tables(qed_ctx_t **out, const qed_config *cfg, hipStream_t s) {
    if (!out || !cfg) return QED_EARG;
    *out = nullptr;
    if (!(cfg->dt > 0) || !(cfg->xi_L > 0) || !(cfg->alpha > 0) ||
        (cfg->precision != QED_FP64 && cfg->precision != QED_MIXED))
        return QED_EARG;
    qed_ctx *c = new (std::nothrow) qed_ctx{};
    if (!c) return QED_ENOMEM;
    c->cfg = *cfg;
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
        free_ctx(c);
        return QED_EHIP;
    }
    c->max_tiles = MAX_TILES;
    const bool ok = hipMalloc(&c->tab64, TAB_TOTAL * sizeof(double)) == hipSuccess &&
                    hipMalloc(&c->tab32, TAB_TOTAL * sizeof(float)) == hipSuccess &&
                    hipMalloc(&c->status, sizeof(uint32_t)) == hipSuccess &&
                    hipMalloc(&c->next_id, sizeof(unsigned long long)) == hipSuccess &&
                    hipMalloc(&c->tile_counts, MAX_TILES * sizeof(int)) == hipSuccess &&
                    hipMalloc(&c->group_tot, GROUP_TOT_LEN * sizeof(int)) == hipSuccess &&
                    hipMalloc(&c->tile_off, (MAX_TILES + 1) * sizeof(int64_t)) == hipSuccess &&
                    hipMalloc(&c->launch, 4 * sizeof(int64_t)) == hipSuccess &&
                    hipEventCreateWithFlags(&c->seg_copied, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        free_ctx(c);
        return QED_ENOMEM;
    }
    e = hipMemsetAsync(c->status, 0, sizeof(uint32_t), s);
    if (e == hipSuccess) e = hipMemsetAsync(c->launch, 0, 4 * sizeof(int64_t), s);
    if (e == hipSuccess) e = hipMemsetAsync(c->group_tot, 0, GROUP_TOT_LEN * sizeof(int), s);
    if (e == hipSuccess) {
        const unsigned long long v = cfg->id_start;
        e = hipMemcpyAsync(c->next_id, &v, sizeof v, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e == hipSuccess) e = build_tables(c, s);
    if (e != hipSuccess) {
        free_ctx(c);
        return QED_EHIP;
    }
    *out = c;
    return QED_OK;
}

qed_status qed_destroy(qed_ctx_t *ctx) {
    if (!ctx) return QED_EARG;
    hipDeviceSynchronize();
    free_ctx(ctx);
    return QED_OK;
}

qed_status qed_gather(qed_ctx_t *ctx, const qed_segment *segs, int nseg, const qed_leptons *p, double *E6,
                      int64_t step, hipStream_t s) {
    qed_status st = ready(ctx);
    if (st != QED_OK) return st;
    SegArgs sa{};
    if ((st = seg_args(ctx, segs, nseg, sa, s)) != QED_OK) return st;
    if ((st = check_leptons(ctx, p, "leptons")) != QED_OK) return st;
    if (!E6) return fail(ctx, QED_EARG, "qed_gather: E6 is NULL");
    return launched(ctx, launch_leptons(ctx, LM_GATHER, sa, *p, E6, nullptr, step, s), "qed_gather");
}

qed_status qed_push_spin(qed_ctx_t *ctx, const qed_segment *segs, int nseg, qed_leptons *p, const double *E6,
                         int64_t step, hipStream_t s) {
    qed_status st = ready(ctx);
    if (st != QED_OK) return st;
    SegArgs sa{};
    if ((st = seg_args(ctx, segs, nseg, sa, s)) != QED_OK) return st;
    if ((st = check_leptons(ctx, p, "leptons")) != QED_OK) return st;
    return launched(ctx, launch_leptons(ctx, LM_PUSH, sa, *p, const_cast<double *>(E6), nullptr, step, s),
                    "qed_push_spin");
}

qed_status qed_emit(qed_ctx_t *ctx, const qed_segment *segs, int nseg, qed_leptons *p, const double *E6,
                    qed_photons *out, int64_t step, hipStream_t s) {
    qed_status st = ready(ctx);
    if (st != QED_OK) return st;
    SegArgs sa{};
    if ((st = seg_args(ctx, segs, nseg, sa, s)) != QED_OK) return st;
    if ((st = check_leptons(ctx, p, "leptons")) != QED_OK) return st;
    if (out && (st = check_photons(ctx, out, "photons")) != QED_OK) return st;
    if (!E6) return fail(ctx, QED_EARG, "qed_emit: E6 (fields of x^n) is required");
    if (!(ctx->cfg.procs & QED_PROC_NCS)) return QED_OK;
    if ((st = ensure_staging(ctx, p->capacity)) != QED_OK) return st;
    return launched(ctx, launch_leptons(ctx, LM_EMIT, sa, *p, const_cast<double *>(E6), out, step, s), "qed_emit");
}

qed_status qed_step_leptons(qed_ctx_t *ctx, const qed_segment *segs, int nseg, qed_leptons *p, qed_photons *out,
                            int64_t step, hipStream_t s) {
    qed_status st = ready(ctx);
    if (st != QED_OK) return st;
    SegArgs sa{};
    if ((st = seg_args(ctx, segs, nseg, sa, s)) != QED_OK) return st;
    if ((st = check_leptons(ctx, p, "leptons")) != QED_OK) return st;
    if (out && (st = check_photons(ctx, out, "photons")) != QED_OK) return st;
    if ((st = ensure_staging(ctx, p->capacity)) != QED_OK) return st;
    return launched(ctx, launch_leptons(ctx, LM_FUSED, sa, *p, nullptr, out, step, s), "qed_step_leptons");
}

static qed_status photon_call(qed_ctx *ctx, PhotonMode mode, const qed_segment *segs, int nseg, qed_photons *g,
                              qed_leptons *em, qed_leptons *ep, int64_t step, hipStream_t s, const char *name) {
    qed_status st = ready(ctx);
    if (st != QED_OK) return st;
    SegArgs sa{};
    if ((st = seg_args(ctx, segs, nseg, sa, s)) != QED_OK) return st;
    if (nseg != 1) return fail(ctx, QED_EARG, "%s: photon calls take exactly one segment", name);
    if ((st = check_photons(ctx, g, "photons")) != QED_OK) return st;
    if (em && (st = check_leptons(ctx, em, "electrons")) != QED_OK) return st;
    if (ep && (st = check_leptons(ctx, ep, "positrons")) != QED_OK) return st;
    if (em && em->charge != -1) return fail(ctx, QED_EARG, "%s: em must have charge -1", name);
    if (ep && ep->charge != 1) return fail(ctx, QED_EARG, "%s: ep must have charge +1", name);
    if ((st = ensure_staging(ctx, g->capacity)) != QED_OK) return st;
    return launched(ctx, launch_photons(ctx, mode, sa, *g, em, ep, step, s), name);
}

qed_status qed_birefringence(qed_ctx_t *ctx, const qed_segment *segs, int nseg, qed_photons *g, int64_t step,
                             hipStream_t s) {
    return photon_call(ctx, PM_BIREF, segs, nseg, g, nullptr, nullptr, step, s, "qed_birefringence");
}
qed_status qed_pair(qed_ctx_t *ctx, const qed_segment *segs, int nseg, qed_photons *g, qed_leptons *em,
                    qed_leptons *ep, int64_t step, hipStream_t s) {
    return photon_call(ctx, PM_PAIR, segs, nseg, g, em, ep, step, s, "qed_pair");
}
qed_status qed_step_photons(qed_ctx_t *ctx, const qed_segment *segs, int nseg, qed_photons *g, qed_leptons *em,
                            qed_leptons *ep, int64_t step, hipStream_t s) {
    return photon_call(ctx, PM_FULL, segs, nseg, g, em, ep, step, s, "qed_step_photons");
}

qed_status qed_compact_photons(qed_ctx_t *ctx, const qed_photons *in, qed_photons *out, hipStream_t s) {
    qed_status st = ready(ctx);
    if (st != QED_OK) return st;
    if ((st = check_photons(ctx, in, "in")) != QED_OK) return st;
    if ((st = check_photons(ctx, out, "out")) != QED_OK) return st;
    if (in->x == out->x || in->count == out->count)
        return fail(ctx, QED_EARG, "qed_compact_photons: in and out must be distinct buffers");
    if ((st = ensure_staging(ctx, in->capacity)) != QED_OK) return st;
    return launched(ctx, launch_compact(ctx, *in, *out, s), "qed_compact_photons");
}

qed_status qed_read_status(qed_ctx_t *ctx, uint32_t *flags, hipStream_t s) {
    if (!ctx || !flags) return QED_EARG;
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpy(flags, ctx->status, sizeof(uint32_t), hipMemcpyDeviceToHost);
    return e == hipSuccess ? QED_OK : hip_fail(ctx, e, "qed_read_status");
}
qed_status qed_clear_status(qed_ctx_t *ctx, hipStream_t s) {
    if (!ctx) return QED_EARG;
    const hipError_t e = hipMemsetAsync(ctx->status, 0, sizeof(uint32_t), s);
    return e == hipSuccess ? QED_OK : hip_fail(ctx, e, "qed_clear_status");
}
qed_status qed_get_next_id(qed_ctx_t *ctx, uint64_t *v, hipStream_t s) {
    if (!ctx || !v) return QED_EARG;
    unsigned long long h = 0;
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpy(&h, ctx->next_id, sizeof h, hipMemcpyDeviceToHost);
    *v = h;
    return e == hipSuccess ? QED_OK : hip_fail(ctx, e, "qed_get_next_id");
}
qed_status qed_set_next_id(qed_ctx_t *ctx, uint64_t v, hipStream_t s) {
    if (!ctx) return QED_EARG;
    const unsigned long long h = v;
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpy(ctx->next_id, &h, sizeof h, hipMemcpyHostToDevice);
    return e == hipSuccess ? QED_OK : hip_fail(ctx, e, "qed_set_next_id");
}

int64_t qed_table_size(int which) {
    switch (which) {
    case QED_TAB_BESSEL: return 3 * NB;
    case QED_TAB_NCS_RATE: return 2 * NR;
    case QED_TAB_NCS_CDF: return 2LL * NCR * NCT;
    case QED_TAB_NBW_RATE: return 2 * NP;
    case QED_TAB_NBW_CDF: return 2LL * NDR * NDD;
    case QED_TAB_VB: return 2 * NV;
    }
    return -1;
}

qed_status qed_table_export(qed_ctx_t *ctx, int which, double *host, int64_t n) {
    qed_status st = ready(ctx);
    if (st != QED_OK) return st;
    const int64_t need = qed_table_size(which);
    if (need < 0) return fail(ctx, QED_EARG, "qed_table_export: unknown table %d", which);
    if (!host || n != need) return fail(ctx, QED_EARG, "qed_table_export: need a host buffer of %lld", (long long)need);
    int64_t off = 0, stride = 2, len = need / 2;
    switch (which) {
    case QED_TAB_BESSEL: off = OFF_BES; stride = 4; len = NB; break;
    case QED_TAB_NCS_RATE: off = OFF_NCS_RATE; break;
    case QED_TAB_NCS_CDF: off = OFF_NCS_CDF; break;
    case QED_TAB_NBW_RATE: off = OFF_NBW_RATE; break;
    case QED_TAB_NBW_CDF: off = OFF_NBW_CDF; break;
    case QED_TAB_VB: off = OFF_VB; break;
    }
    const int nc = which == QED_TAB_BESSEL ? 3 : 2;
    double *tmp = new (std::nothrow) double[stride * len];
    if (!tmp) return QED_ENOMEM;
    const hipError_t e = hipMemcpy(tmp, ctx->tab64 + off, stride * len * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        for (int c = 0; c < nc; ++c)
            for (int64_t i = 0; i < len; ++i) host[c * len + i] = tmp[stride * i + c];
    delete[] tmp;
    return e == hipSuccess ? QED_OK : hip_fail(ctx, e, "qed_table_export");
}

qed_status qed_set_step_events(qed_ctx_t *ctx, const hipEvent_t *ev) {
    if (!ctx) return QED_EARG;
    if (!ev) {
        ctx->step_ev_on = 0;
        return QED_OK;
    }
    for (int k = 0; k < 4; ++k) {
        if (!ev[k]) return fail(ctx, QED_EARG, "qed_set_step_events: event %d is NULL", k);
        ctx->step_ev[k] = ev[k];
    }
    ctx->step_ev_on = 1;
    return QED_OK;
}

const char *qed_last_error(const qed_ctx_t *ctx) { return ctx ? ctx->err : "null context"; }

}  // extern "C"
