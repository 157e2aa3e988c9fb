// Charge-conserving current deposition (Sec. II.C) onto the 2D Yee grid of the GRID2D
// field: Jx at (i+1/2, j), Jy at (i, j+1/2), Jz at (i, j), array index [j][i], periodic.
//
// A particle moving from xa to xb within one step (less than a cell per axis) has TSC
// shapes (Sec. II.E, node-centred) S0 at the start and S1 at the end, both taken on the
// 5 x 5 node window centred on the start node; with DS = S1 - S0 (Esirkepov's
// decomposition of the change of its charge):
//   Wx = DSx (S0y + DSy/2),  Wy = DSy (S0x + DSx/2),
//   Wz = S0x S0y + DSx S0y/2 + S0x DSy/2 + DSx DSy/3,
//   Jx(i+1/2, j) = Jx(i-1/2, j) - Q Wx / (dy dt),  Jy(i, j+1/2) = Jy(i, j-1/2) - Q Wy / (dx dt),
//   Jz = Q vz Wz / (dx dy),  vz = (zb - za)/dt,  Q = q w qscale,
// which makes (rho1 - rho0)/dt + div J vanish node by node.  Weights in FP64 (the DS are
// small differences of O(1) values), contributions rounded to FP32 (the grid's precision)
// and summed in FP32 in an order that is not fixed; exact zeros are skipped (a particle
// moving along x at a tenth of a cell per step adds about 25 values).
//
// Beams put hundreds of particles on each node, so adding every contribution to HBM with
// a device-wide atomic serialises on the hot nodes.  The tiled path bins the particles by
// the tile of T x T nodes that holds their start node and accumulates each tile in LDS:
//   1. count   : particles per tile (LDS histogram per block over its share of the list,
//                one global add per tile), largest |w| and |w dz| (bound_terms);
//   2. scan    : tile offsets, a work list of chunks of at most DEP_CH particles, and the
//                fixed-point scale of each component (a power of two that maps the largest
//                possible contribution to 2^32);
//   3. scatter : a 56-byte record per particle (offsets from the nodes, weight, shifts,
//                node in the tile) at its tile's place: each block counts its share per
//                tile, reserves that many slots per tile with one global add, then hands
//                them out through an LDS cursor;
//   4. tiles   : one block per chunk adds its records, in 64-bit fixed point, to the
//                (T+4)^2 LDS window of the tile (two-node halo: LDS integer atomics run at
//                several times the rate of LDS float atomics here), then adds the non-zero
//                window sums to a context-owned 64-bit grid with global integer atomics;
//   5. convert : the 64-bit grid, scaled back, is added to J (FP32) and cleared.
// Integer sums do not depend on the order of the additions, so the tiled path gives the
// same J on every run; its only roundings are the fixed-point quantum (2^-32 of the largest
// contribution) and one FP32 rounding per node.  T is 16 or 32, the smaller one with at
// most DEP_MAX_TILES tiles; larger grids take the direct path (one thread per particle,
// FP32 global atomics, order of the sums not fixed).  Lists kept in cell order can take
// the local path instead (QED_DEPOSIT_LOCAL, below): no binning, a window per block of
// consecutive particles, the same integer sums.
#include "qed_internal.hpp"

namespace qed {
namespace {

constexpr int DBLOCK = 256;
constexpr int DEP_BPC = 2;                 // blocks per compute unit of the persistent kernels
constexpr int DEP_MAX_TILES = 8192;        // tiles of the tiled path (LDS histograms of this many ints)
constexpr int DEP_CH = 4096;               // records per block of the tile kernel

// a particle's deposit, relative to its start node: offsets of the start and end positions
// from their nearest nodes (cell units), weight, weight times the z move; code = node in the
// tile (x | y << 8) | (end node - start node + 1) in x << 16 and in y << 18
struct DepRec {
    double ax, ay, bx, by, w, wdz;
    int32_t code, pad;
};

// one lepton list of the call
struct DepSource {
    const double *x, *y, *z, *w;      // positions at the end of the step, weights
    const double *x0, *y0, *z0;       // positions at the start of the step
    const int64_t *n0;                // particles [0, *n0) are deposited
    int64_t capacity;
    double charge;                    // -1 or +1 (folded into each record's weight)
};

struct DepositArgs {
    DepSource src[DEP_MAX_SRC];
    int32_t nsrc;
    float *jx, *jy, *jz;
    int32_t nx, ny;
    double gx0, gy0, inv_dx, inv_dy;
    double cx, cy, cz;                // -qscale/(dy dt), -qscale/(dx dt), qscale/(dx dy dt)
    uint32_t *status;
    // tiled path
    int32_t T, ntx, nt;
    int *cnt, *off, *cur, *nwork;      // per tile: count, offset, cursor; chunks in the work list
    int4 *work;
    DepRec *rec;
    unsigned long long *amax;          // bit patterns of the largest |w| and |w dz| (zero between calls)
    double *scale;                     // fixed-point scale and its inverse per component [6]
    unsigned long long *acc;           // 64-bit fixed-point J [3][ny][nx] (zero between calls)
};

__device__ __forceinline__ int64_t dep_count(const DepSource &d) {
    const int64_t n = *d.n0;
    return n < 0 ? 0 : (n > d.capacity ? d.capacity : n);
}

// start node (wrapped into the grid) and record of particle i of source d (weight times
// charge); false for a particle that is not deposited (non-finite, absurdly far, or a move
// of a cell or more)
__device__ __forceinline__ bool classify(const DepositArgs &a, const DepSource &d, int64_t i, DepRec &r, int &ic,
                                         int &lc, int *raw = nullptr) {
    const double Xa = (d.x0[i] - a.gx0) * a.inv_dx, Ya = (d.y0[i] - a.gy0) * a.inv_dy;
    const double Xb = (d.x[i] - a.gx0) * a.inv_dx, Yb = (d.y[i] - a.gy0) * a.inv_dy;
    const double dz = d.z[i] - d.z0[i], w = d.charge * d.w[i];
    const double lim = 1073741824.0;
    if (!(fabs(Xa) < lim && fabs(Ya) < lim && fabs(Xb - Xa) < 1.0 && fabs(Yb - Ya) < 1.0 && isfinite(dz) &&
          isfinite(w)))
        return false;
    const double ja = floor(Xa + 0.5), ka = floor(Ya + 0.5);
    const double jb = floor(Xb + 0.5), kb = floor(Yb + 0.5);
    r.ax = Xa - ja;
    r.ay = Ya - ka;
    r.bx = Xb - jb;
    r.by = Yb - kb;
    r.w = w;
    r.wdz = w * dz;
    r.code = ((int)(jb - ja) + 1) << 16 | ((int)(kb - ka) + 1) << 18;
    if (raw) {                        // the start node before wrapping (|ja|, |ka| < 2^30)
        raw[0] = (int)ja;
        raw[1] = (int)ka;
    }
    const int ia = (int)(ja - a.nx * floor(ja / a.nx)), la = (int)(ka - a.ny * floor(ka / a.ny));
    ic = ia >= a.nx ? ia - a.nx : (ia < 0 ? ia + a.nx : ia);
    lc = la >= a.ny ? la - a.ny : (la < 0 ? la + a.ny : la);
    return true;
}

// the largest |w| and |w dz| that set the fixed-point scales, over every particle of the
// call with a finite weight and z move (deposited or not: the maxima then need only w and
// z, and both paths find the same ones); the same products as the records' w and wdz
__device__ __forceinline__ void bound_terms(const DepSource &d, int64_t i, double &mw, double &mz) {
    const double w = d.charge * d.w[i], wdz = w * (d.z[i] - d.z0[i]);
    if (isfinite(w) && isfinite(wdz)) {
        mw = fmax(mw, fabs(w));
        mz = fmax(mz, fabs(wdz));
    }
}

// the block's maxima of mw, mz (non-negative) into s_max[2] (zeroed before the block's
// barrier that precedes this call; a barrier must follow): a wavefront reduction, then one
// LDS atomic per wavefront (non-negative doubles order like their bit patterns)
__device__ __forceinline__ void block_max2(double mw, double mz, unsigned long long *s_max) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        mw = fmax(mw, __shfl_xor(mw, d));
        mz = fmax(mz, __shfl_xor(mz, d));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&s_max[0], (unsigned long long)__double_as_longlong(mw));
        atomicMax(&s_max[1], (unsigned long long)__double_as_longlong(mz));
    }
}

// TSC weights of nodes j-1, j, j+1 for offset d = X - j in [-1/2, 1/2], on a 4-slot window
// whose slot k is slot k + o of the 5-slot window, where slot 2 + s holds node j
__device__ __forceinline__ void window4(double d, int s, int o, double out[4]) {
    const double a = 0.5 - d, b = 0.5 + d;
    const double m = 0.5 * a * a, c = 0.75 - d * d, p = 0.5 * b * b;
    const int k0 = s + 1 - o;
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = k == k0 ? m : (k == k0 + 1 ? c : (k == k0 + 2 ? p : 0.0));
}

// adds the record's current through sink.add(component, row slot l, column slot m, value)
// (slots of the 5 x 5 window centred on the start node).  The start and end shapes of a
// move of less than a cell cover at most 4 consecutive slots per axis, from o = 1 + min(s, 0).
template <class Sink>
__device__ __forceinline__ void deposit_record(const DepositArgs &a, const DepRec &r, Sink &sink) {
    const int sx = ((r.code >> 16) & 3) - 1, sy = ((r.code >> 18) & 3) - 1;
    const int ox = 1 + (sx < 0 ? sx : 0), oy = 1 + (sy < 0 ? sy : 0);
    double S0x[4], S1x[4], S0y[4], S1y[4];
    window4(r.ax, 0, ox, S0x);
    window4(r.bx, sx, ox, S1x);
    window4(r.ay, 0, oy, S0y);
    window4(r.by, sy, oy, S1y);
    const double qx = a.cx * r.w, qy = a.cy * r.w, qz = a.cz * r.wdz;
    // Jx: running sum along x in each row (the sum over the window is zero, so the last
    // slot carries nothing)
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        const double wy = S0y[l] + 0.5 * (S1y[l] - S0y[l]);
        if (wy == 0.0) continue;
        double run = 0.0;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            run += qx * (S1x[m] - S0x[m]) * wy;
            sink.add(0, l + oy, m + ox, run);
        }
    }
    // Jy: running sum along y in each column
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const double wx = S0x[m] + 0.5 * (S1x[m] - S0x[m]);
        if (wx == 0.0) continue;
        double run = 0.0;
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            run += qy * (S1y[l] - S0y[l]) * wx;
            sink.add(1, l + oy, m + ox, run);
        }
    }
    // Jz: step average of the product of the linearly interpolated shapes
    if (qz != 0.0) {
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const double s0y = S0y[l], dsy = S1y[l] - S0y[l];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const double s0x = S0x[m], dsx = S1x[m] - S0x[m];
                const double wz = s0x * s0y + 0.5 * dsx * s0y + 0.5 * s0x * dsy + dsx * dsy * (1.0 / 3.0);
                sink.add(2, l + oy, m + ox, qz * wz);
            }
        }
    }
}

// node index of j + m - 2 wrapped into [0, n), m = 0..4 (n >= 2)
__device__ __forceinline__ int wrap(int j, int m, int n) {
    int k = j + m - 2;
    k = k < 0 ? k + n : k;
    return k >= n ? k - n : k;
}

struct GlobalSink {
    float *j[3];
    int col[5], row[5];
    __device__ __forceinline__ void add(int c, int l, int m, double v) {
        if (v != 0.0) unsafeAtomicAdd(j[c] + row[l] + col[m], (float)v);
    }
};

// v scaled to a 64-bit fixed-point integer (|v| scale <= 2^33), rounded to nearest even.
// The scale is a power of two, so v scale is exact and one fused add of 1.5 2^52 rounds it
// to an integer held in the low mantissa bits (the sum has exponent 52 for |v scale| < 2^51);
// subtracting the constant's bit pattern leaves it as a two's-complement 64-bit integer.
__device__ __forceinline__ unsigned long long fixed64(double v, double scale) {
    constexpr double MAGIC = 6755399441055744.0;                     // 1.5 * 2^52
    return (unsigned long long)__double_as_longlong(fma(v, scale, MAGIC)) -
           (unsigned long long)__double_as_longlong(MAGIC);
}

struct LdsSink {
    unsigned long long *acc;   // [3][plane]: a window of rows of `stride` nodes
    int stride, plane, base;   // base: LDS index of window slot (0, 0)
    double sc[3];              // fixed-point scale per component
    __device__ __forceinline__ void add(int c, int l, int m, double v) {
        if (v != 0.0) atomicAdd(acc + c * plane + base + l * stride + m, fixed64(v, sc[c]));
    }
};
// fixed-point contributions straight to the 64-bit grid (global integer atomics)
struct FixedSink {
    unsigned long long *acc;   // [3][nodes]
    int64_t nodes;
    int col[5], row[5];
    double sc[3];
    __device__ __forceinline__ void add(int c, int l, int m, double v) {
        if (v != 0.0) atomicAdd(acc + c * nodes + row[l] + col[m], fixed64(v, sc[c]));
    }
};

// direct path: one thread per particle, global atomics
__global__ __launch_bounds__(DBLOCK) void k_deposit(DepositArgs a, int sidx) {
    const DepSource &d = a.src[sidx];
    const int64_t i = (int64_t)blockIdx.x * DBLOCK + threadIdx.x;
    if (i >= dep_count(d)) return;
    DepRec r;
    int ic, lc;
    if (!classify(a, d, i, r, ic, lc)) {
        atomicOr(a.status, (uint32_t)QED_ST_DEPOSIT);
        return;
    }
    GlobalSink s{{a.jx, a.jy, a.jz}, {}, {}};
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        s.col[m] = wrap(ic, m, a.nx);
        s.row[m] = wrap(lc, m, a.ny) * a.nx;
    }
    deposit_record(a, r, s);
}

__device__ __forceinline__ int tile_of(const DepositArgs &a, int ic, int lc) {
    return (lc / a.T) * a.ntx + ic / a.T;
}

// 1. particles per tile; largest |w| and |w dz| (non-negative doubles order like their
// bit patterns).  Persistent: block b takes particles b*DBLOCK + tid + k*gridDim.x*DBLOCK.
__global__ __launch_bounds__(DBLOCK) void k_dep_count(DepositArgs a) {
    __shared__ int h[DEP_MAX_TILES];
    __shared__ unsigned long long s_max[2];
    const int64_t stride = (int64_t)gridDim.x * DBLOCK;
    for (int k = threadIdx.x; k < a.nt; k += DBLOCK) h[k] = 0;
    if (threadIdx.x < 2) s_max[threadIdx.x] = 0;
    __syncthreads();
    double mw = 0.0, mz = 0.0;
    for (int q = 0; q < a.nsrc; ++q) {
        const DepSource &d = a.src[q];
        const int64_t n = dep_count(d);
        for (int64_t i = (int64_t)blockIdx.x * DBLOCK + threadIdx.x; i < n; i += stride) {
            DepRec r;
            int ic, lc;
            bound_terms(d, i, mw, mz);
            if (classify(a, d, i, r, ic, lc)) atomicAdd(&h[tile_of(a, ic, lc)], 1);
            else atomicOr(a.status, (uint32_t)QED_ST_DEPOSIT);
        }
    }
    block_max2(mw, mz, s_max);
    __syncthreads();
    for (int k = threadIdx.x; k < a.nt; k += DBLOCK)
        if (h[k]) atomicAdd(&a.cnt[k], h[k]);
    if (threadIdx.x < 2 && s_max[threadIdx.x]) atomicMax(&a.amax[threadIdx.x], s_max[threadIdx.x]);
}

// power-of-two scale that maps |v| <= bound to at most 2^32
__device__ __forceinline__ double fixed_scale(double bound) {
    if (!(bound > 0.0)) return 1.0;
    int e;
    frexp(bound, &e);          // bound < 2^e
    return ldexp(1.0, 32 - e);
}
// the fixed-point scales of the three components from the largest |w| and |w dz|: running
// sums of Jx, Jy are at most 2 |c w|, Jz at most |c w dz|
__device__ __forceinline__ void fixed_scales(const DepositArgs &a, double sc[3]) {
    const double mw = __longlong_as_double((long long)a.amax[0]), mz = __longlong_as_double((long long)a.amax[1]);
    sc[0] = fixed_scale(2.0 * fabs(a.cx) * mw);
    sc[1] = fixed_scale(2.0 * fabs(a.cy) * mw);
    sc[2] = fixed_scale(fabs(a.cz) * mz);
}

// 2. tile offsets, chunk work list; clears the counts and the cursors for the next call
constexpr int SCAN_T = 1024;
constexpr int SCAN_PER = DEP_MAX_TILES / SCAN_T;
__global__ __launch_bounds__(SCAN_T) void k_dep_scan(DepositArgs a) {
    __shared__ int s_cnt[SCAN_T], s_chk[SCAN_T];
    const int t0 = threadIdx.x * SCAN_PER;
    int c[SCAN_PER], sc = 0, sk = 0;
#pragma unroll
    for (int q = 0; q < SCAN_PER; ++q) {
        c[q] = t0 + q < a.nt ? a.cnt[t0 + q] : 0;
        sc += c[q];
        sk += (c[q] + DEP_CH - 1) / DEP_CH;
    }
    s_cnt[threadIdx.x] = sc;
    s_chk[threadIdx.x] = sk;
    __syncthreads();
    for (int d = 1; d < SCAN_T; d <<= 1) {   // inclusive scan (Hillis-Steele)
        const int vc = threadIdx.x >= d ? s_cnt[threadIdx.x - d] : 0;
        const int vk = threadIdx.x >= d ? s_chk[threadIdx.x - d] : 0;
        __syncthreads();
        s_cnt[threadIdx.x] += vc;
        s_chk[threadIdx.x] += vk;
        __syncthreads();
    }
    int off = s_cnt[threadIdx.x] - sc, chunk = s_chk[threadIdx.x] - sk;
#pragma unroll
    for (int q = 0; q < SCAN_PER; ++q) {
        const int t = t0 + q;
        if (t >= a.nt) break;
        a.off[t] = off;
        for (int b = 0; b < c[q]; b += DEP_CH) a.work[chunk++] = make_int4(t, off + b, off + min(c[q], b + DEP_CH), 0);
        off += c[q];
        a.cnt[t] = 0;
        a.cur[t] = 0;
    }
    if (threadIdx.x == SCAN_T - 1) *a.nwork = s_chk[SCAN_T - 1];
    if (threadIdx.x == 0) {
        double sc[3];
        fixed_scales(a, sc);
        for (int c = 0; c < 3; ++c) {
            a.scale[c] = sc[c];
            a.scale[3 + c] = 1.0 / sc[c];
        }
        a.amax[0] = 0;
        a.amax[1] = 0;
    }
}

// 3. records sorted by tile.  Same particles per block as the count kernel: count them
// per tile, reserve the block's slots of each tile (one global add), then place each
// record at the next slot of its tile (LDS cursor).
__global__ __launch_bounds__(DBLOCK) void k_dep_scatter(DepositArgs a) {
    __shared__ int h[DEP_MAX_TILES];
    const int64_t stride = (int64_t)gridDim.x * DBLOCK;
    for (int k = threadIdx.x; k < a.nt; k += DBLOCK) h[k] = 0;
    __syncthreads();
    for (int q = 0; q < a.nsrc; ++q) {
        const DepSource &d = a.src[q];
        const int64_t n = dep_count(d);
        for (int64_t i = (int64_t)blockIdx.x * DBLOCK + threadIdx.x; i < n; i += stride) {
            DepRec r;
            int ic, lc;
            if (classify(a, d, i, r, ic, lc)) atomicAdd(&h[tile_of(a, ic, lc)], 1);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < a.nt; k += DBLOCK)
        if (h[k]) h[k] = a.off[k] + atomicAdd(&a.cur[k], h[k]);
    __syncthreads();
    for (int q = 0; q < a.nsrc; ++q) {
        const DepSource &d = a.src[q];
        const int64_t n = dep_count(d);
        for (int64_t i = (int64_t)blockIdx.x * DBLOCK + threadIdx.x; i < n; i += stride) {
            DepRec r;
            int ic, lc;
            if (!classify(a, d, i, r, ic, lc)) continue;
            r.code |= (ic % a.T) | (lc % a.T) << 8;
            a.rec[atomicAdd(&h[tile_of(a, ic, lc)], 1)] = r;
        }
    }
}

// 4. one block per chunk of a tile (persistent over the work list): LDS window of the tile,
// added to the 64-bit grid with global atomics (16 wavefronts per block: a chunk's records
// are spread over a whole compute unit)
constexpr int TBLOCK = 1024;
__global__ __launch_bounds__(TBLOCK) void k_dep_tiles(DepositArgs a) {
    extern __shared__ unsigned long long acc[];
    const int nw = *a.nwork;
    const int W = a.T + 4, WW = W * W;
    const double s0 = a.scale[0], s1 = a.scale[1], s2 = a.scale[2];
    const int64_t nodes = (int64_t)a.nx * a.ny;
    for (int w = blockIdx.x; w < nw; w += gridDim.x) {   // persistent over the work list
        const int4 wk = a.work[w];
        for (int k = threadIdx.x; k < 3 * WW; k += TBLOCK) acc[k] = 0;
        __syncthreads();
        for (int k = wk.y + threadIdx.x; k < wk.z; k += TBLOCK) {
            const DepRec r = a.rec[k];
            LdsSink s{acc, W, WW, ((r.code >> 8) & 255) * W + (r.code & 255), {s0, s1, s2}};
            deposit_record(a, r, s);
        }
        __syncthreads();
        const int tx0 = (wk.x % a.ntx) * a.T - 2, ty0 = (wk.x / a.ntx) * a.T - 2;
        for (int k = threadIdx.x; k < 3 * WW; k += TBLOCK) {
            const unsigned long long v = acc[k];
            if (v == 0) continue;
            const int c = k / WW, rem = k - c * WW, l = rem / W, m = rem - l * W;
            int gx = (tx0 + m) % a.nx, gy = (ty0 + l) % a.ny;
            gx = gx < 0 ? gx + a.nx : gx;
            gy = gy < 0 ? gy + a.ny : gy;
            atomicAdd(a.acc + c * nodes + (int64_t)gy * a.nx + gx, v);
        }
        __syncthreads();   // the window is cleared for the next work item
    }
}

// Local path (lists kept in cell order, e.g. by qed_sort_leptons): the same fixed-point
// contributions without binning.
//   L1. amax  : the largest |w| and |w dz| (bound_terms, as the count kernel: w and z only);
//   L2. local : a chunk of 256 consecutive particles of a source per block and turn; the
//               chunk's start nodes span a box; if the box and its two-node halo fit LWIN
//               nodes the block adds its records to that LDS window and then the window's
//               non-zero sums to the 64-bit grid, otherwise each contribution goes to the
//               64-bit grid;
//   then the convert kernel.  Integer sums: the same J as the binned path, bit for bit.
constexpr int LWIN = 1024;   // nodes of a block's LDS window (3 x 8 bytes each: 24 KB)
constexpr int DEP_LOCAL_BPC = 6;   // blocks per compute unit of the local path (LDS: six fit)

// Chunks of 256 particles of the sources' live counts, sources in order: live_chunks is
// their number, chunk_at maps chunk g to its source and the chunk within that source.  The
// kernels below sweep them persistently (a grid sized by the capacities would be mostly
// empty blocks, and launching those costs more than the work).
__device__ __forceinline__ int64_t live_chunks(const DepositArgs &a) {
    int64_t t = 0;
    for (int q = 0; q < a.nsrc; ++q) t += (dep_count(a.src[q]) + DBLOCK - 1) / DBLOCK;
    return t;
}
__device__ __forceinline__ int chunk_at(const DepositArgs &a, int64_t g, int64_t &c) {
    int q = 0;
    for (; q < a.nsrc - 1; ++q) {
        const int64_t nc = (dep_count(a.src[q]) + DBLOCK - 1) / DBLOCK;
        if (g < nc) break;
        g -= nc;
    }
    c = g;
    return q;
}

__global__ __launch_bounds__(DBLOCK) void k_dep_amax(DepositArgs a) {
    __shared__ unsigned long long s_max[2];
    const int64_t nch = live_chunks(a);
    if (threadIdx.x < 2) s_max[threadIdx.x] = 0;
    __syncthreads();
    double mw = 0.0, mz = 0.0;
    for (int64_t g = blockIdx.x; g < nch; g += gridDim.x) {
        int64_t c;
        const DepSource &d = a.src[chunk_at(a, g, c)];
        const int64_t i = c * DBLOCK + threadIdx.x;
        if (i < dep_count(d)) bound_terms(d, i, mw, mz);
    }
    block_max2(mw, mz, s_max);
    __syncthreads();
    // only blocks above the running maximum add an atomic on its one address (the value
    // read can only be below the final one, so none is missed)
    if (threadIdx.x < 2) {
        const unsigned long long v = s_max[threadIdx.x];
        if (v > *(volatile unsigned long long *)&a.amax[threadIdx.x]) atomicMax(&a.amax[threadIdx.x], v);
    }
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = min(v, __shfl_xor(v, d));
    return v;
}

// one chunk of the local path (s_box: this chunk's LDS slots for the box reduction; the
// caller alternates two sets, so no barrier is needed before they are written again)
__device__ __forceinline__ void local_chunk(const DepositArgs &a, const DepSource &d, int64_t c, const double sc[3],
                                            unsigned long long *win, int (*s_box)[DBLOCK / 64]) {
    const int64_t n = dep_count(d);
    const int64_t i = c * DBLOCK + threadIdx.x;
    DepRec r;
    int ic = 0, lc = 0, raw[2] = {0, 0};
    const bool ok = i < n && classify(a, d, i, r, ic, lc, raw);
    if (i < n && !ok) atomicOr(a.status, (uint32_t)QED_ST_DEPOSIT);
    // box of the block's start nodes (min of j, k, -j, -k; INT_MAX where no particle)
    constexpr int BIG = 0x7fffffff;
    const int v[4] = {ok ? raw[0] : BIG, ok ? raw[1] : BIG, ok ? -raw[0] : BIG, ok ? -raw[1] : BIG};
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int m = wave_min(v[k]);
        if ((threadIdx.x & 63) == 0) s_box[k][wv] = m;
    }
    __syncthreads();
    int b[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        b[k] = s_box[k][0];
        for (int w = 1; w < DBLOCK / 64; ++w) b[k] = min(b[k], s_box[k][w]);
    }
    if (b[0] == BIG) return;                        // no particle of this chunk is deposited
    const int j0 = b[0], k0 = b[1];
    const int64_t bw = (int64_t)(-b[2]) - j0 + 5, bh = (int64_t)(-b[3]) - k0 + 5;
    const int64_t nodes = (int64_t)a.nx * a.ny;
    if (bw * bh > LWIN) {                           // spread out: straight to the 64-bit grid
        if (!ok) return;
        FixedSink s{a.acc, nodes, {}, {}, {sc[0], sc[1], sc[2]}};
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            s.col[m] = wrap(ic, m, a.nx);
            s.row[m] = wrap(lc, m, a.ny) * a.nx;
        }
        deposit_record(a, r, s);
        return;
    }
    const int W = (int)bw, plane = (int)(bw * bh);
    for (int k = threadIdx.x; k < 3 * plane; k += DBLOCK) win[k] = 0;
    __syncthreads();
    if (ok) {
        LdsSink s{win, W, plane, (raw[1] - k0) * W + (raw[0] - j0), {sc[0], sc[1], sc[2]}};
        deposit_record(a, r, s);
    }
    __syncthreads();
    // window slot (l, m) is node (j0 - 2 + m, k0 - 2 + l), wrapped into the grid; the slot
    // of entry k is stepped along without divisions (k grows by DBLOCK = dl rows + dm)
    int ox = (j0 - 2) % a.nx, oy = (k0 - 2) % a.ny;
    ox = ox < 0 ? ox + a.nx : ox;
    oy = oy < 0 ? oy + a.ny : oy;
    const int dl = DBLOCK / W, dm = DBLOCK - dl * W;
    int l = (int)threadIdx.x / W, m = (int)threadIdx.x - l * W;
    for (int k = threadIdx.x; k < plane; k += DBLOCK) {
        int gx = ox + m, gy = oy + l;
        while (gx >= a.nx) gx -= a.nx;     // a window wider than the grid wraps more than once
        while (gy >= a.ny) gy -= a.ny;
        const int64_t g = (int64_t)gy * a.nx + gx;
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            const unsigned long long val = win[cc * plane + k];
            if (val != 0) atomicAdd(a.acc + cc * nodes + g, val);
        }
        m += dm;
        l += dl;
        if (m >= W) {
            m -= W;
            ++l;
        }
    }
}

__global__ __launch_bounds__(DBLOCK) void k_dep_local(DepositArgs a) {
    __shared__ unsigned long long win[3 * LWIN];
    __shared__ int s_box[2][4][DBLOCK / 64];
    double sc[3];
    fixed_scales(a, sc);
    if (blockIdx.x == 0 && threadIdx.x < 3) {       // the scales the convert kernel divides by
        a.scale[threadIdx.x] = sc[threadIdx.x];
        a.scale[3 + threadIdx.x] = 1.0 / sc[threadIdx.x];
    }
    const int64_t nch = live_chunks(a);
    int par = 0;
    for (int64_t g = blockIdx.x; g < nch; g += gridDim.x, par ^= 1) {
        int64_t c;
        const DepSource &d = a.src[chunk_at(a, g, c)];
        local_chunk(a, d, c, sc, win, s_box[par]);
    }
}

// 5. J += fixed-point grid / scale, which is cleared
__global__ __launch_bounds__(DBLOCK) void k_dep_convert(DepositArgs a) {
    const int64_t nodes = (int64_t)a.nx * a.ny, stride = (int64_t)gridDim.x * DBLOCK;
    const double inv[3] = {a.scale[3], a.scale[4], a.scale[5]};
    if (blockIdx.x == 0 && threadIdx.x < 2) a.amax[threadIdx.x] = 0;   // zero for the next call
    for (int64_t k = (int64_t)blockIdx.x * DBLOCK + threadIdx.x; k < 3 * nodes; k += stride) {
        const unsigned long long v = a.acc[k];
        if (v == 0) continue;
        const int c = (int)(k / nodes);
        const int64_t o = k - c * nodes;
        float *J = c == 0 ? a.jx : (c == 1 ? a.jy : a.jz);
        J[o] += (float)((double)(long long)v * inv[c]);
        a.acc[k] = 0;
    }
}

// positions [0, count) and the count, for the deposit after the next step
__global__ __launch_bounds__(DBLOCK) void k_save_start(const double *x, const double *y, const double *z,
                                                       const int64_t *count, int64_t capacity, double *x0, double *y0,
                                                       double *z0, int64_t *n0) {
    int64_t n = *count;
    n = n < 0 ? 0 : (n > capacity ? capacity : n);
    const int64_t stride = (int64_t)gridDim.x * DBLOCK;
    for (int64_t i = (int64_t)blockIdx.x * DBLOCK + threadIdx.x; i < n; i += stride) {
        x0[i] = x[i];
        y0[i] = y[i];
        z0[i] = z[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *n0 = n;
}

// tile counters, offsets, cursors [3][DEP_MAX_TILES + 1] ints, then 2 maxima (uint64) and
// 6 scale factors (double)
constexpr size_t DEP_CNT_BYTES = 3 * (DEP_MAX_TILES + 1) * sizeof(int) + 8 * sizeof(double) + 8;

hipError_t ensure_deposit(qed_ctx *ctx, int64_t capacity, int64_t nodes, bool binned) {
    hipError_t e = hipSuccess;
    if (!ctx->dep_cnt) {
        e = hipMalloc(&ctx->dep_cnt, DEP_CNT_BYTES);
        if (e != hipSuccess) return e;
        e = hipMemset(ctx->dep_cnt, 0, DEP_CNT_BYTES);
        if (e != hipSuccess) return e;
    }
    if (3 * nodes > ctx->dep_acc_len) {
        (void)hipFree(ctx->dep_acc);
        ctx->dep_acc = nullptr;
        ctx->dep_acc_len = 0;
        if ((e = hipMalloc(&ctx->dep_acc, 3 * nodes * sizeof(unsigned long long))) != hipSuccess) return e;
        if ((e = hipMemset(ctx->dep_acc, 0, 3 * nodes * sizeof(unsigned long long))) != hipSuccess) return e;
        ctx->dep_acc_len = 3 * nodes;
    }
    if (binned && capacity > ctx->dep_cap) {   // records and work list: the binned path only
        (void)hipFree(ctx->dep_rec);
        (void)hipFree(ctx->dep_work);
        ctx->dep_rec = nullptr;
        ctx->dep_work = nullptr;
        ctx->dep_cap = 0;
        const int64_t nwork = capacity / DEP_CH + DEP_MAX_TILES + 1;
        if ((e = hipMalloc(&ctx->dep_rec, capacity * sizeof(DepRec))) != hipSuccess) return e;
        if ((e = hipMalloc(&ctx->dep_work, nwork * sizeof(int4))) != hipSuccess) return e;
        ctx->dep_cap = capacity;
    }
    return e;
}

}  // namespace

hipError_t launch_save_start(qed_ctx *ctx, const qed_leptons &L, double *const x0[3], int64_t *n0, hipStream_t s) {
    int64_t b = (L.capacity + DBLOCK - 1) / DBLOCK;
    const int64_t cap = 8LL * ctx->num_cu;   // grid-stride: a few blocks per compute unit
    b = b < 1 ? 1 : (b > cap ? cap : b);
    hipLaunchKernelGGL(k_save_start, dim3((unsigned)b), dim3(DBLOCK), 0, s, L.x, L.y, L.z, L.count, L.capacity,
                       x0[0], x0[1], x0[2], n0);
    return hipGetLastError();
}

hipError_t launch_deposit(qed_ctx *ctx, const qed_deposit_src *src, int nsrc, float *const J[3], int nx, int ny,
                          double dx, double dy, double gx0, double gy0, double dt, double qscale, hipStream_t s) {
    DepositArgs a{};
    int64_t total = 0;
    for (int q = 0; q < nsrc; ++q) {
        const qed_leptons &L = *src[q].leptons;
        DepSource &d = a.src[q];
        d.x = L.x;
        d.y = L.y;
        d.z = L.z;
        d.w = L.w;
        d.x0 = src[q].x0[0];
        d.y0 = src[q].x0[1];
        d.z0 = src[q].x0[2];
        d.n0 = src[q].n0;
        d.capacity = L.capacity;
        d.charge = (double)L.charge;
        total += L.capacity;
    }
    a.nsrc = nsrc;
    a.jx = J[0];
    a.jy = J[1];
    a.jz = J[2];
    a.nx = nx;
    a.ny = ny;
    a.gx0 = gx0;
    a.gy0 = gy0;
    a.inv_dx = 1.0 / dx;
    a.inv_dy = 1.0 / dy;
    a.cx = -qscale / (dy * dt);
    a.cy = -qscale / (dx * dt);
    a.cz = qscale / (dx * dy * dt);
    a.status = ctx->status;
    if (total == 0) return hipGetLastError();
    for (int T = 16; T <= 32; T *= 2) {
        const int64_t ntx = (nx + T - 1) / T, nty = (ny + T - 1) / T;
        if (ntx * nty <= DEP_MAX_TILES) {
            a.T = T;
            a.ntx = (int)ntx;
            a.nt = (int)(ntx * nty);
            break;
        }
    }
    if (a.T == 0) {
        for (int q = 0; q < nsrc; ++q) {
            if (a.src[q].capacity == 0) continue;
            const dim3 gd((unsigned)((a.src[q].capacity + DBLOCK - 1) / DBLOCK)), bd(DBLOCK);
            hipLaunchKernelGGL(k_deposit, gd, bd, 0, s, a, q);
        }
        return hipGetLastError();
    }
    const int64_t nodes = (int64_t)nx * ny;
    const bool local = ctx->dep_path == QED_DEPOSIT_LOCAL;
    const hipError_t e = ensure_deposit(ctx, total, nodes, !local);
    if (e != hipSuccess) return e;
    a.cnt = ctx->dep_cnt;
    a.off = ctx->dep_cnt + (DEP_MAX_TILES + 1);
    a.cur = ctx->dep_cnt + 2 * (DEP_MAX_TILES + 1);
    a.nwork = a.off + DEP_MAX_TILES;
    char *tail = (char *)(ctx->dep_cnt + 3 * (DEP_MAX_TILES + 1));
    tail += (8 - (uintptr_t)tail % 8) % 8;
    a.amax = (unsigned long long *)tail;
    a.scale = (double *)(tail + 2 * sizeof(unsigned long long));
    a.acc = (unsigned long long *)ctx->dep_acc;
    a.work = (int4 *)ctx->dep_work;
    a.rec = (DepRec *)ctx->dep_rec;
    const int64_t persist = (int64_t)DEP_BPC * ctx->num_cu;
    const int64_t pb = (total + DBLOCK - 1) / DBLOCK, wb = total / DEP_CH + a.nt + 1;
    const unsigned pblocks = (unsigned)(pb < persist ? pb : persist);
    const unsigned wblocks = (unsigned)(wb < persist ? wb : persist);
    const size_t lds = 3 * (size_t)(a.T + 4) * (a.T + 4) * sizeof(unsigned long long);
    if (local) {
        int64_t chunks = 0;
        for (int q = 0; q < nsrc; ++q) chunks += (a.src[q].capacity + DBLOCK - 1) / DBLOCK;
        // persistent over the live chunks (their number is on the device)
        const int64_t cap = (int64_t)DEP_LOCAL_BPC * ctx->num_cu;
        const unsigned lb = (unsigned)(chunks < cap ? (chunks < 1 ? 1 : chunks) : cap);
        hipLaunchKernelGGL(k_dep_amax, dim3(lb), dim3(DBLOCK), 0, s, a);
        hipLaunchKernelGGL(k_dep_local, dim3(lb), dim3(DBLOCK), 0, s, a);
    } else {
        hipLaunchKernelGGL(k_dep_count, dim3(pblocks), dim3(DBLOCK), 0, s, a);
        hipLaunchKernelGGL(k_dep_scan, dim3(1), dim3(SCAN_T), 0, s, a);
        hipLaunchKernelGGL(k_dep_scatter, dim3(pblocks), dim3(DBLOCK), 0, s, a);
        hipLaunchKernelGGL(k_dep_tiles, dim3(wblocks), dim3(TBLOCK), lds, s, a);
    }
    int64_t cb = (3 * nodes + DBLOCK - 1) / DBLOCK;
    cb = cb > 8LL * ctx->num_cu ? 8LL * ctx->num_cu : cb;
    hipLaunchKernelGGL(k_dep_convert, dim3((unsigned)cb), dim3(DBLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace qed
