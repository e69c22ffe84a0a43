// dmrt_device.hpp -- device code of libdmrt for gfx950: the double-MRT
// collision (Li, Yang & Zhang, arXiv:1601.04633, Sections 3.1-3.2) held in
// registers, and the fused pull-stream + collide kernel.
//
// Storage: structure of arrays, one plane per population,
//   buf[q * plane + y * pitch + x],  plane = rows * pitch,
// two ping-pong copies.  The stored state at step t is the post-collision
// population f*(t), g*(t).  One step of the kernel for node r:
//   1. gather f_i(r, t+1) = f*_i(r - e_i, t)  (halfway bounce-back or
//      anti-bounce-back where r - e_i lies outside the walls);
//   2. collide at t+1 in registers;
//   3. store f*(r, t+1) into the other copy.
// The stored f is the deviation from w_i rho0, so that sum f = drho
// (Eq. 33); this is the paper's own incompressible formulation and keeps
// FP32 storage accurate.
#pragma once

#include <hip/hip_runtime.h>

namespace dmrt {

enum Bc { BC_CAVITY = 0, BC_PERIODIC = 1, BC_CHANNEL_X = 2, BC_ADIABATIC_BOX = 3 };

// Per-cavity scalars in the compute precision.
template <typename real>
struct Coef {
    real s_nu, s_q;      // Eq. 32; s_e = s_eps = s_nu
    real sk, se, sn;     // Eq. 38: sigma_k, sigma_e, sigma_nu
    real a;              // Eq. 42: n_eq[4] = a theta
    real cabb;           // Eq. 45 constant (4 + a)/10
    real gbeta, gy0;     // Eq. 27: G_y = gbeta theta + gy0, gy0 = -gbeta theta_ref
    real gx;             // constant horizontal force (test boxes)
    real cold;           // cabb * theta_cold
};

// Pre-collision populations in, post-collision populations out (Eq. 25 and
// Eq. 36 right-hand sides).  Moments of Eq. 30 and Eq. 37 are expanded into
// the +-1/+-2/+-4 adds the matrices encode; the inverse transforms use
// M^-1 = M^T diag(1/9, 1/6, 1/6, 1/36, 1/4, 1/4, 1/12, 1/12, 1/36) and
// N^-1 = N^T diag(1/5, 1/2, 1/2, 1/20, 1/4) (both matrices have orthogonal
// rows).  Only the moment changes are transformed back.
template <typename real>
__device__ __forceinline__ void collide(real (&f)[9], real (&g)[5], const Coef<real>& c,
                                        real& theta_out, real& ux_out, real& uy_out)
{
    const real one = real(1), two = real(2), three = real(3);
    // Eq. 33, Eq. 41
    const real s1234 = (f[1] + f[3]) + (f[2] + f[4]);
    const real s5678 = (f[5] + f[7]) + (f[6] + f[8]);
    const real drho = f[0] + s1234 + s5678;
    const real u = (f[1] - f[3]) + (f[5] - f[7]) + (f[8] - f[6]);
    const real v = (f[2] - f[4]) + (f[5] - f[7]) + (f[6] - f[8]);
    const real theta = g[0] + (g[1] + g[3]) + (g[2] + g[4]);

    // non-conserved moments, rows 4-9 of Eq. 30
    const real m3 = two * s5678 - s1234 - real(4) * f[0];
    const real m4 = (f[1] + f[3]) - (f[2] + f[4]);
    const real m5 = (f[5] + f[7]) - (f[6] + f[8]);
    const real m6 = two * (f[3] - f[1]) + (f[5] - f[7]) + (f[8] - f[6]);
    const real m7 = two * (f[4] - f[2]) + (f[5] - f[7]) + (f[6] - f[8]);
    const real m8 = real(4) * f[0] - two * s1234 + s5678;

    // equilibria, Eq. 34 (energy moment with the factor 3)
    const real uu = u * u, vv = v * v, q2 = uu + vv;
    const real e3 = three * q2 - two * drho;
    const real e4 = uu - vv;
    const real e5 = u * v;
    const real e8 = drho - three * q2;

    // moment image of the force of Eq. 26 with G = (gx, gbeta theta + gy0):
    // the moments of 3 G.(e_i - u) w_i (1 + 3 e.u + 9/2 (e.u)^2 - 3/2 u^2)
    const real Gx = c.gx;
    const real Gy = c.gbeta * theta + c.gy0;
    const real F3 = three * (Gx * u + Gy * v) * (two - three * q2);
    const real F4 = Gx * u * (two - three * uu + three * vv) - Gy * v * (two + three * uu - three * vv);
    const real F5 = Gx * v * (one - three * uu) + Gy * u * (one - three * vv);
    const real F6 = real(6) * Gy * u * v - Gx * (one - three * vv);
    const real F7 = real(6) * Gx * u * v - Gy * (one - three * uu);

    // moment changes: -S (m - m_eq) + F   (Eq. 28, Eq. 31)
    const real a1 = Gx * real(1.0 / 6.0);
    const real a2 = Gy * real(1.0 / 6.0);
    const real a3 = (F3 - c.s_nu * (m3 - e3)) * real(1.0 / 36.0);
    const real a4 = (F4 - c.s_nu * (m4 - e4)) * real(0.25);
    const real a5 = (F5 - c.s_nu * (m5 - e5)) * real(0.25);
    const real a6 = (F6 - c.s_q * (m6 + u)) * real(1.0 / 12.0);
    const real a7 = (F7 - c.s_q * (m7 + v)) * real(1.0 / 12.0);
    const real a8 = (-F3 - c.s_nu * (m8 - e8)) * real(1.0 / 36.0);

    // f += M^T a
    const real d2 = two * a3 + a8;              // shared by the four diagonals
    f[0] += real(4) * (a8 - a3);
    f[1] += a1 - a3 + a4 - two * a6 - two * a8;
    f[2] += a2 - a3 - a4 - two * a7 - two * a8;
    f[3] += -a1 - a3 + a4 + two * a6 - two * a8;
    f[4] += -a2 - a3 - a4 + two * a7 - two * a8;
    f[5] += d2 + (a1 + a2) + (a5 + a6 + a7);
    f[6] += d2 + (a2 - a1) + (a7 - a5 - a6);
    f[7] += d2 - (a1 + a2) + (a5 - a6 - a7);
    f[8] += d2 + (a1 - a2) + (a6 - a5 - a7);

    // D2Q5, Eqs. 36-42 (last row of N read as e_x^2 - e_y^2)
    const real n1 = g[1] - g[3];
    const real n2 = g[2] - g[4];
    const real n3 = (g[1] + g[3]) + (g[2] + g[4]) - real(4) * g[0];
    const real n4 = (g[1] + g[3]) - (g[2] + g[4]);
    const real b1 = -c.sk * (n1 - u * theta) * real(0.5);
    const real b2 = -c.sk * (n2 - v * theta) * real(0.5);
    const real b3 = -c.se * (n3 - c.a * theta) * real(0.05);
    const real b4 = -c.sn * n4 * real(0.25);
    g[0] += real(-4) * b3;
    g[1] += b1 + b3 + b4;
    g[2] += b2 + b3 - b4;
    g[3] += b3 + b4 - b1;
    g[4] += b3 - b4 - b2;

    theta_out = theta;
    ux_out = u;
    uy_out = v;
}

// ---------------------------------------------------------------------------
// Fused step kernel
// ---------------------------------------------------------------------------
template <typename real>
struct StepArgs {
    const real* __restrict__ fin;
    const real* __restrict__ gin;
    real* __restrict__ fout;
    real* __restrict__ gout;
    const real* __restrict__ thw;   // hot-wall theta per row
    int n, pitch;
    int plane;                      // n * pitch
    int tiles_x, tiles;             // tile grid of the launch
    int xcd_remap;
    Coef<real> c;
};

// Maps the hardware workgroup id to a tile so that each of the 8 dies gets
// a contiguous range of tiles (the dispatcher deals workgroups round-robin
// over the dies).  The grid is padded to a multiple of 8; padded ids map
// past the last tile and exit.
__device__ __forceinline__ int tile_of_block(int bid, int nblocks, int remap)
{
    if (!remap) return bid;
    const int per = nblocks >> 3;
    return (bid & 7) * per + (bid >> 3);
}

// One node update (rows a1-a5): gather from the current copy with the wall
// rules, collide in registers, store into the other copy.
template <typename real, int BC>
__device__ __forceinline__ void node_update(const real* __restrict__ fi, const real* __restrict__ gi,
                                            real* __restrict__ fo, real* __restrict__ go,
                                            const real* __restrict__ thw, int n, int pitch, int P,
                                            int x, int y, const Coef<real>& c)
{
    constexpr bool PX = (BC == BC_PERIODIC || BC == BC_CHANNEL_X);
    constexpr bool PY = (BC == BC_PERIODIC);
    constexpr bool ABB = (BC == BC_CAVITY);

    const int k = y * pitch + x;
    // neighbour offsets (wrapped in periodic directions)
    const bool hxm = PX || x > 0, hxp = PX || x < n - 1;
    const bool hym = PY || y > 0, hyp = PY || y < n - 1;
    const int dxm = (PX && x == 0) ? (n - 1) : -1;
    const int dxp = (PX && x == n - 1) ? -(n - 1) : 1;
    const int dym = (PY && y == 0) ? (n - 1) * pitch : -pitch;
    const int dyp = (PY && y == n - 1) ? -(n - 1) * pitch : pitch;

    real f[9], g[5];
    // pull: f_i(r) = f*_i(r - e_i), else bounce-back f*_opp(i)(r)
    f[0] = fi[k];
    f[1] = hxm ? fi[1 * P + k + dxm] : fi[3 * P + k];
    f[2] = hym ? fi[2 * P + k + dym] : fi[4 * P + k];
    f[3] = hxp ? fi[3 * P + k + dxp] : fi[1 * P + k];
    f[4] = hyp ? fi[4 * P + k + dyp] : fi[2 * P + k];
    f[5] = (hxm && hym) ? fi[5 * P + k + dxm + dym] : fi[7 * P + k];
    f[6] = (hxp && hym) ? fi[6 * P + k + dxp + dym] : fi[8 * P + k];
    f[7] = (hxp && hyp) ? fi[7 * P + k + dxp + dyp] : fi[5 * P + k];
    f[8] = (hxm && hyp) ? fi[8 * P + k + dxm + dyp] : fi[6 * P + k];

    g[0] = gi[k];
    g[2] = hym ? gi[2 * P + k + dym] : gi[4 * P + k];       // Eq. 44
    g[4] = hyp ? gi[4 * P + k + dyp] : gi[2 * P + k];
    if (ABB) {                                              // Eq. 45
        g[1] = hxm ? gi[1 * P + k + dxm] : c.cabb * thw[y] - gi[3 * P + k];
        g[3] = hxp ? gi[3 * P + k + dxp] : c.cold - gi[1 * P + k];
    } else {
        g[1] = hxm ? gi[1 * P + k + dxm] : gi[3 * P + k];
        g[3] = hxp ? gi[3 * P + k + dxp] : gi[1 * P + k];
    }

    real th, ux, uy;
    collide<real>(f, g, c, th, ux, uy);

#pragma unroll
    for (int i = 0; i < 9; ++i) fo[i * P + k] = f[i];
#pragma unroll
    for (int i = 0; i < 5; ++i) go[i * P + k] = g[i];
}

template <typename real, int BC>
__global__ void __launch_bounds__(1024) step_kernel(StepArgs<real> A)
{
    const int tile = tile_of_block(blockIdx.x, gridDim.x, A.xcd_remap);
    if (tile >= A.tiles) return;
    const int ty = tile / A.tiles_x;
    const int tx = tile - ty * A.tiles_x;
    const int x = tx * blockDim.x + threadIdx.x;
    const int y = ty * blockDim.y + threadIdx.y;
    if (x >= A.n || y >= A.n) return;
    node_update<real, BC>(A.fin, A.gin, A.fout, A.gout, A.thw, A.n, A.pitch, A.plane, x, y, A.c);
}

// ---------------------------------------------------------------------------
// Batched sweep: many independent cavities advanced by one launch
// ---------------------------------------------------------------------------
// Per-cavity parameter block, resident in device memory.
template <typename real>
struct CavityDev {
    real* f[2];            // ping-pong copies of the 9 D2Q9 planes
    real* g[2];            // ping-pong copies of the 5 D2Q5 planes
    const real* thw;       // hot-wall theta per row
    const double* thw_d;   // the same in FP64 (Nusselt number)
    double H, inv_dT, theta_cold;
    int n, pitch, plane;
    int dead;              // 1: skipped (non-finite state was detected)
    Coef<real> c;
};

// One entry per workgroup-sized tile: cavity and tile origin.
struct TileRef {
    int cav, x0, y0, pad;
};

// Grid-stride over the tiles [t_begin, t_end): with gridDim.x equal to the
// tile count every workgroup takes one tile; with fewer workgroups the
// launch is persistent.  All cavities step from copy `cur` to `cur ^ 1`.
template <typename real>
__global__ void __launch_bounds__(1024) batch_step_kernel(const CavityDev<real>* __restrict__ cavs,
                                                          const TileRef* __restrict__ tiles,
                                                          int t_begin, int t_end, int cur)
{
    for (int t = t_begin + blockIdx.x; t < t_end; t += gridDim.x) {
        const TileRef tr = tiles[t];
        const CavityDev<real>& cv = cavs[tr.cav];
        if (cv.dead) continue;
        const int x = tr.x0 + threadIdx.x;
        const int y = tr.y0 + threadIdx.y;
        if (x >= cv.n || y >= cv.n) continue;
        node_update<real, BC_CAVITY>(cv.f[cur], cv.g[cur], cv.f[cur ^ 1], cv.g[cur ^ 1], cv.thw,
                                     cv.n, cv.pitch, cv.plane, x, y, cv.c);
    }
}

// ---------------------------------------------------------------------------
// Initialisation at equilibrium, then one collision (stores f*(0), g*(0))
// ---------------------------------------------------------------------------
template <typename real>
__global__ void init_kernel(real* __restrict__ fout, real* __restrict__ gout,
                            const double* __restrict__ drho, const double* __restrict__ U,
                            const double* __restrict__ V, const double* __restrict__ T,
                            int n, int pitch, int plane, Coef<real> c, real w0, real wm)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= n || y >= n) return;
    const int src = y * n + x;
    const real r = drho ? real(drho[src]) : real(0);
    const real u = U ? real(U[src]) : real(0);
    const real v = V ? real(V[src]) : real(0);
    const real th = T ? real(T[src]) : real(0);
    // D2Q9 incompressible equilibrium (deviation form) = M^-1 m_eq of Eq. 34
    const real w[3] = {real(4.0 / 9.0), real(1.0 / 9.0), real(1.0 / 36.0)};
    const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const real q2 = u * u + v * v;
    real f[9], g[5];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const real eu = real(ex[i]) * u + real(ey[i]) * v;
        const real wi = i == 0 ? w[0] : (i < 5 ? w[1] : w[2]);
        f[i] = wi * (r + real(3) * eu + real(4.5) * eu * eu - real(1.5) * q2);
    }
    // D2Q5 equilibrium = N^-1 n_eq of Eq. 42
    g[0] = w0 * th;
#pragma unroll
    for (int i = 1; i < 5; ++i)
        g[i] = wm * th + real(0.5) * th * (real(ex[i]) * u + real(ey[i]) * v);
    real a, b, d;
    collide<real>(f, g, c, a, b, d);
    const int k = y * pitch + x;
#pragma unroll
    for (int i = 0; i < 9; ++i) fout[i * plane + k] = f[i];
#pragma unroll
    for (int i = 0; i < 5; ++i) gout[i * plane + k] = g[i];
}

// ---------------------------------------------------------------------------
// Fields from the stored post-collision state (Eq. 9, 33, 41)
// ---------------------------------------------------------------------------
template <typename real>
__global__ void fields_kernel(const real* __restrict__ fs, const real* __restrict__ gs,
                              int n, int pitch, int plane, double gbeta, double gy0, double gx,
                              double* __restrict__ U, double* __restrict__ V,
                              double* __restrict__ T, double* __restrict__ P)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= n || y >= n) return;
    const int k = y * pitch + x;
    double f[9], th = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = double(fs[i * plane + k]);
#pragma unroll
    for (int i = 0; i < 5; ++i) th += double(gs[i * plane + k]);
    const double drho = f[0] + (f[1] + f[3]) + (f[2] + f[4]) + (f[5] + f[7]) + (f[6] + f[8]);
    const double jx = (f[1] - f[3]) + (f[5] - f[7]) + (f[8] - f[6]);
    const double jy = (f[2] - f[4]) + (f[5] - f[7]) + (f[6] - f[8]);
    // the collision added rho0 G to the momentum; remove it to get Eq. 33's u
    const int o = y * n + x;
    U[o] = jx - gx;
    V[o] = jy - (gbeta * th + gy0);
    T[o] = th;
    P[o] = drho / 3.0;
}

// ---------------------------------------------------------------------------
// Wall Nusselt number, Eqs. 18-19: one workgroup, FP64 accumulation.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the rows of the local Nusselt numbers of one wall, by one
// workgroup of 256 threads; returns the average to thread 0.
template <typename real>
__device__ __forceinline__ double nusselt_block(const real* __restrict__ gs, int n, int pitch,
                                                int plane, int wall, const double* __restrict__ thw,
                                                double theta_cold, double H, double inv_dT,
                                                double* __restrict__ nu_local)
{
    __shared__ double part[4];
    double acc = 0.0;
    const int x0 = wall == 0 ? 0 : n - 1;
    const int x1 = wall == 0 ? 1 : n - 2;
    for (int y = threadIdx.x; y < n; y += blockDim.x) {
        const int k0 = y * pitch + x0, k1 = y * pitch + x1;
        double t0 = 0.0, t1 = 0.0;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            t0 += double(gs[i * plane + k0]);
            t1 += double(gs[i * plane + k1]);
        }
        const double tw = wall == 0 ? thw[y] : theta_cold;
        // slope into the fluid from the quadratic through (0, tw), (1/2, t0), (3/2, t1)
        const double slope_in = (9.0 * t0 - t1 - 8.0 * tw) * (1.0 / 3.0);
        const double nu = (wall == 0 ? -slope_in : slope_in) * H * inv_dT;
        if (nu_local) nu_local[y] = nu;
        acc += nu;
    }
    acc = wave_sum(acc);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) part[wid] = acc;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += part[w];
    return s / n;
}

template <typename real>
__global__ void __launch_bounds__(256) nusselt_kernel(
    const real* __restrict__ gs, int n, int pitch, int plane, int wall,
    const double* __restrict__ thw, double theta_cold, double H, double inv_dT,
    double* __restrict__ nu_local, double* __restrict__ nu_avg,
    double* __restrict__ ring, unsigned long long* __restrict__ ring_count, long ring_cap)
{
    const double avg = nusselt_block<real>(gs, n, pitch, plane, wall, thw, theta_cold, H, inv_dT,
                                           nu_local);
    if (threadIdx.x == 0) {
        if (nu_avg) *nu_avg = avg;
        if (ring) {
            const unsigned long long c = *ring_count;
            ring[c % (unsigned long long)ring_cap] = avg;
            *ring_count = c + 1;
        }
    }
}

// Hot-wall Nusselt number of every cavity of a batch: one workgroup each.
template <typename real>
__global__ void __launch_bounds__(256) batch_nusselt_kernel(const CavityDev<real>* __restrict__ cavs,
                                                            int cur, double* __restrict__ out)
{
    const CavityDev<real>& cv = cavs[blockIdx.x];
    const double avg = nusselt_block<real>(cv.g[cur], cv.n, cv.pitch, cv.plane, 0, cv.thw_d,
                                           cv.theta_cold, cv.H, cv.inv_dT, nullptr);
    if (threadIdx.x == 0) out[blockIdx.x] = cv.dead ? __builtin_nan("") : avg;
}

// Non-finite check of every cavity's state: grid (blocks per cavity, count).
template <typename real>
__global__ void __launch_bounds__(256) batch_check_kernel(const CavityDev<real>* __restrict__ cavs,
                                                          int cur, int* __restrict__ flags)
{
    const CavityDev<real>& cv = cavs[blockIdx.y];
    const long nn = (long)cv.n * cv.n;
    int bad = 0;
    for (long o = (long)blockIdx.x * blockDim.x + threadIdx.x; o < nn;
         o += (long)gridDim.x * blockDim.x) {
        const int y = (int)(o / cv.n), x = (int)(o - (long)y * cv.n);
        const int k = y * cv.pitch + x;
        real s = real(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) s += fabs(cv.f[cur][i * cv.plane + k]);
#pragma unroll
        for (int i = 0; i < 5; ++i) s += fabs(cv.g[cur][i * cv.plane + k]);
        bad |= !isfinite(s);
    }
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0 && bad) atomicOr(&flags[blockIdx.y], 1);
}

// ---------------------------------------------------------------------------
// Residual / watchdog: per-block partial sums (FP64), then a final pass.
// part[b*5 + {0..4}] = sum dtheta^2, sum theta^2, sum du^2, sum u^2, nonfinite
// ---------------------------------------------------------------------------
template <typename real>
__global__ void __launch_bounds__(256) residual_kernel(
    const real* __restrict__ fs, const real* __restrict__ gs, int n, int pitch, int plane,
    double gbeta, double gy0, double gx, double* __restrict__ ref, double* __restrict__ part)
{
    __shared__ double sh[4][5];
    double acc[5] = {0, 0, 0, 0, 0};
    const long nn = (long)n * n;
    for (long o = (long)blockIdx.x * blockDim.x + threadIdx.x; o < nn;
         o += (long)gridDim.x * blockDim.x) {
        const int y = (int)(o / n), x = (int)(o - (long)y * n);
        const int k = y * pitch + x;
        double f[9], th = 0.0, mag = 0.0;
#pragma unroll
        for (int i = 0; i < 9; ++i) { f[i] = double(fs[i * plane + k]); mag += fabs(f[i]); }
#pragma unroll
        for (int i = 0; i < 5; ++i) { const double gv = double(gs[i * plane + k]); th += gv; mag += fabs(gv); }
        const double jx = (f[1] - f[3]) + (f[5] - f[7]) + (f[8] - f[6]) - gx;
        const double jy = (f[2] - f[4]) + (f[5] - f[7]) + (f[6] - f[8]) - (gbeta * th + gy0);
        if (!isfinite(mag)) { acc[4] += 1.0; continue; }
        const double dt = th - ref[o], du = jx - ref[nn + o], dv = jy - ref[2 * nn + o];
        acc[0] += dt * dt; acc[1] += th * th;
        acc[2] += du * du + dv * dv; acc[3] += jx * jx + jy * jy;
        ref[o] = th; ref[nn + o] = jx; ref[2 * nn + o] = jy;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const double s = wave_sum(acc[j]);
        if (lane == 0) sh[wid][j] = s;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w][threadIdx.x];
        part[blockIdx.x * 5 + threadIdx.x] = s;
    }
}

static __global__ void __launch_bounds__(64) residual_final_kernel(const double* __restrict__ part,
                                                            int nparts, double* __restrict__ out)
{
    if (threadIdx.x < 5) {
        double s = 0.0;
        for (int b = 0; b < nparts; ++b) s += part[b * 5 + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

}  // namespace dmrt
