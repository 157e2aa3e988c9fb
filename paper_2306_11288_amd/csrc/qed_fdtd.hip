// 2D field solver on the Yee grid of the GRID2D field (Sec. II.B, z squeezed), periodic in
// x and y.  Array index [j][i] holds Ex (i+1/2, j), Ey (i, j+1/2), Ez (i, j), Bx (i, j+1/2),
// By (i+1/2, j), Bz (i+1/2, j+1/2); an optional current J has the staggering of E.  One
// step of dt (leapfrog of Sec. II.F with B split in two half steps, so that E and B are both
// known at integer times for the gather):
//   B -= dt/2 curl E;   E += dt (curl B - J);   B -= dt/2 curl E.
// One thread per node, FP32 like the grid; the stencil neighbours of a row come through
// the caches (every array is read by the neighbouring rows' threads too).
#include "qed_internal.hpp"

namespace qed {
namespace {

struct YeeArgs {
    float *g[6];
    const float *j[3];     // current (E kernel with CUR only)
    int32_t nx, ny, nxb;   // nxb: blocks per row
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
    Ex[o] += a.cy * (bz - Bz[oj]);
    Ey[o] -= a.cx * (bz - Bz[oi]);
    Ez[o] += a.cx * (By[o] - By[oi]) - a.cy * (Bx[o] - Bx[oj]);
    if (CUR) {
        Ex[o] -= a.h * a.j[0][o];
        Ey[o] -= a.h * a.j[1][o];
        Ez[o] -= a.h * a.j[2][o];
    }
}

}  // namespace

hipError_t launch_yee(float *const g[6], const float *const J[3], int nx, int ny, double dx, double dy, double dt,
                      int64_t steps, hipStream_t s) {
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
    for (int64_t n = 0; n < steps; ++n) {
        hipLaunchKernelGGL(k_yee_b, gd, bd, 0, s, hb);
        if (J) hipLaunchKernelGGL(k_yee_e<true>, gd, bd, 0, s, fe);
        else hipLaunchKernelGGL(k_yee_e<false>, gd, bd, 0, s, fe);
        hipLaunchKernelGGL(k_yee_b, gd, bd, 0, s, hb);
    }
    return hipGetLastError();
}

}  // namespace qed
