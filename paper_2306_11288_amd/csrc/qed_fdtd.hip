// 2D field solver on the Yee grid of the GRID2D field (Sec. II.B, z squeezed), periodic in
// x and y.  Array index [j][i] holds Ex (i+1/2, j), Ey (i, j+1/2), Ez (i, j), Bx (i, j+1/2),
// By (i+1/2, j), Bz (i+1/2, j+1/2); an optional current J has the staggering of E.  One
// step of dt (leapfrog of Sec. II.F with B split in two half steps, so that E and B are both
// known at integer times for the gather):
//   B -= dt/2 curl E;   E += dt (curl B - J);   B -= dt/2 curl E.
// One thread per node, FP32 like the grid; the stencil neighbours of a row come through
// the caches (every array is read by the neighbouring rows' threads too).
//
// Open x boundaries (first-order absorbing condition of Mur; y stays periodic): before the
// E update the tangential Ey, Ez of the first two and last two node columns are saved;
// after it, the first and last columns are replaced by the one-way wave condition of the
// outgoing field, discretised between the boundary node and its neighbour over the step,
//   E_0^{n+1} = E_1^n + k (E_1^{n+1} - E_0^n),   k = (dt - dx)/(dt + dx),
// at x_max applied to E - E_inc with E_inc an analytic pulse (plane wave or Gaussian beam,
// evaluated in FP64 at each node's staggered position) that enters through x_max.  The
// values the periodic wrap leaves beyond the boundary columns never reach the interior;
// the components half a cell beyond x_max (Ex, By, Bz of the last column) lie outside the
// box and are kept at zero.
#include "qed_dev.hpp"

namespace qed {
namespace {

struct YeeArgs {
    float *g[6];
    const float *j[3];     // current (E kernel with CUR only)
    int32_t nx, ny, nxb;   // nxb: blocks per row
    int32_t open;          // open x: the last column's Ex, By, Bz (beyond x_max) stay zero
    float cx, cy;          // h/dx, h/dy with h the (half) step of this kernel
    float h;               // the step of this kernel
};

// B -= h curl E:  Bx -= h dEz/dy,  By += h dEz/dx,  Bz -= h (dEy/dx - dEx/dy)   (forward differences)
__global__ __launch_bounds__(256) void k_yee_b(YeeArgs a) {
    const int j = blockIdx.x / a.nxb, i = (blockIdx.x % a.nxb) * 256 + threadIdx.x;
    if (i >= a.nx) return;
    const int ip = i + 1 == a.nx ? 0 : i + 1, jp = j + 1 == a.ny ? 0 : j + 1;
    const int64_t o = (int64_t)j * a.nx + i, oi = (int64_t)j * a.nx + ip, oj = (int64_t)jp * a.nx + i;
    const float *Ex = a.g[0], *Ey = a.g[1], *Ez = a.g[2];
    float *Bx = a.g[3], *By = a.g[4], *Bz = a.g[5];
    const float ez = Ez[o];
    Bx[o] -= a.cy * (Ez[oj] - ez);
    if (a.open && i == a.nx - 1) {
        By[o] = 0.0f;
        Bz[o] = 0.0f;
        return;
    }
    By[o] += a.cx * (Ez[oi] - ez);
    Bz[o] -= a.cx * (Ey[oi] - Ey[o]) - a.cy * (Ex[oj] - Ex[o]);
}

// E += h (curl B - J):  Ex += h (dBz/dy - Jx),  Ey -= h (dBz/dx + Jy),
//                       Ez += h (dBy/dx - dBx/dy - Jz)   (backward differences)
template <bool CUR>
__global__ __launch_bounds__(256) void k_yee_e(YeeArgs a) {
    const int j = blockIdx.x / a.nxb, i = (blockIdx.x % a.nxb) * 256 + threadIdx.x;
    if (i >= a.nx) return;
    const int im = i == 0 ? a.nx - 1 : i - 1, jm = j == 0 ? a.ny - 1 : j - 1;
    const int64_t o = (int64_t)j * a.nx + i, oi = (int64_t)j * a.nx + im, oj = (int64_t)jm * a.nx + i;
    float *Ex = a.g[0], *Ey = a.g[1], *Ez = a.g[2];
    const float *Bx = a.g[3], *By = a.g[4], *Bz = a.g[5];
    const float bz = Bz[o];
    float ex = Ex[o] + a.cy * (bz - Bz[oj]);
    float ey = Ey[o] - a.cx * (bz - Bz[oi]);
    float ez = Ez[o] + (a.cx * (By[o] - By[oi]) - a.cy * (Bx[o] - Bx[oj]));
    if (CUR) {
        ex -= a.h * a.j[0][o];
        ey -= a.h * a.j[1][o];
        ez -= a.h * a.j[2][o];
    }
    Ex[o] = (a.open && i == a.nx - 1) ? 0.0f : ex;
    Ey[o] = ey;
    Ez[o] = ez;
}

// saved columns: [component Ey, Ez][column 0, 1, nx-2, nx-1][ny]
__global__ __launch_bounds__(256) void k_mur_save(YeeArgs a, float *save) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= 8 * a.ny) return;
    const int c = k / (4 * a.ny), q = (k / a.ny) % 4, j = k % a.ny;
    const int col = q == 0 ? 0 : (q == 1 ? 1 : (q == 2 ? a.nx - 2 : a.nx - 1));
    save[k] = a.g[1 + c][(int64_t)j * a.nx + col];
}

struct MurArgs {
    float *g[6];
    const float *save;
    FieldDev inc;            // incoming pulse (kind NONE: no injection)
    int32_t nx, ny;
    double k;                // (dt - dx)/(dt + dx)
    double xN, xM, gy0, dy;  // x of the last two columns, grid origin in y, spacing
    double t0, t1;           // times of the step's start and end
};

__device__ __forceinline__ double incoming(const MurArgs &a, int comp, double x, double y, double t) {
    V3<double> E, B;
    field_at<double>(a.inc, t, x, y, 0.0, E, B);
    return comp == 0 ? E.y : E.z;
}

// one thread per (component, side, row)
__global__ __launch_bounds__(256) void k_mur(MurArgs a) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= 4 * a.ny) return;
    const int c = k / (2 * a.ny), side = (k / a.ny) % 2, j = k % a.ny;
    float *E = a.g[1 + c];
    const float *sv = a.save + (int64_t)c * 4 * a.ny;
    const int64_t row = (int64_t)j * a.nx;
    if (side == 0) {
        const double L0 = sv[j], L1 = sv[a.ny + j];
        E[row] = (float)(L1 + a.k * ((double)E[row + 1] - L0));
        return;
    }
    const double R1 = sv[2 * a.ny + j], R0 = sv[3 * a.ny + j];
    double v = R1 + a.k * ((double)E[row + a.nx - 2] - R0);
    if (a.inc.kind != QED_FIELD_NONE) {
        const double y = a.gy0 + (j + (c == 0 ? 0.5 : 0.0)) * a.dy;   // Ey at (i, j+1/2), Ez at (i, j)
        const double iN0 = incoming(a, c, a.xN, y, a.t0), iN1 = incoming(a, c, a.xN, y, a.t1);
        const double iM0 = incoming(a, c, a.xM, y, a.t0), iM1 = incoming(a, c, a.xM, y, a.t1);
        v = iN1 + (R1 - iM0) + a.k * (((double)E[row + a.nx - 2] - iM1) - (R0 - iN0));
    }
    E[row + a.nx - 1] = (float)v;
}

}  // namespace

hipError_t launch_yee(qed_ctx *ctx, float *const g[6], const float *const J[3], const YeeBoundary *bc, int nx, int ny,
                      double dx, double dy, double dt, int64_t steps, hipStream_t s) {
    YeeArgs hb{}, fe{};
    for (int c = 0; c < 6; ++c) hb.g[c] = fe.g[c] = g[c];
    if (J)
        for (int c = 0; c < 3; ++c) fe.j[c] = J[c];
    fe.h = (float)dt;
    hb.nx = fe.nx = nx;
    hb.ny = fe.ny = ny;
    hb.nxb = fe.nxb = (nx + 255) / 256;
    hb.cx = (float)(0.5 * dt / dx);
    hb.cy = (float)(0.5 * dt / dy);
    fe.cx = (float)(dt / dx);
    fe.cy = (float)(dt / dy);
    const dim3 gd((unsigned)(((nx + 255) / 256) * (int64_t)ny)), bd(256);   // one block per 256 nodes of a row
    MurArgs m{};
    hb.open = fe.open = bc ? 1 : 0;
    if (bc) {
        if (ctx->yee_save_len < 8LL * ny) {
            (void)hipFree(ctx->yee_save);
            ctx->yee_save = nullptr;
            ctx->yee_save_len = 0;
            const hipError_t e = hipMalloc(&ctx->yee_save, 8LL * ny * sizeof(float));
            if (e != hipSuccess) return e;
            ctx->yee_save_len = 8LL * ny;
        }
        for (int c = 0; c < 6; ++c) m.g[c] = g[c];
        m.save = ctx->yee_save;
        m.inc = bc->inc;
        m.nx = nx;
        m.ny = ny;
        m.k = (dt - dx) / (dt + dx);
        m.xN = bc->gx0 + (nx - 1) * dx;
        m.xM = bc->gx0 + (nx - 2) * dx;
        m.gy0 = bc->gy0;
        m.dy = dy;
    }
    const unsigned sb = (unsigned)((8LL * ny + 255) / 256), mb = (unsigned)((4LL * ny + 255) / 256);
    for (int64_t n = 0; n < steps; ++n) {
        hipLaunchKernelGGL(k_yee_b, gd, bd, 0, s, hb);
        if (bc) hipLaunchKernelGGL(k_mur_save, dim3(sb), bd, 0, s, fe, ctx->yee_save);
        if (J) hipLaunchKernelGGL(k_yee_e<true>, gd, bd, 0, s, fe);
        else hipLaunchKernelGGL(k_yee_e<false>, gd, bd, 0, s, fe);
        if (bc) {
            m.t0 = bc->t0 + n * dt;
            m.t1 = bc->t0 + (n + 1) * dt;
            hipLaunchKernelGGL(k_mur, dim3(mb), bd, 0, s, m);
        }
        hipLaunchKernelGGL(k_yee_b, gd, bd, 0, s, hb);
    }
    return hipGetLastError();
}

}  // namespace qed
