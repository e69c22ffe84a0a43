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

// Every multiply-add below is written out (fmr); nothing is contracted by
// the compiler, so the arithmetic of a node update is the same in every
// kernel it is inlined into and results do not depend on the launch shape
// or on the number of steps per launch.
#pragma clang fp contract(off)

namespace dmrt {

// a * b + c with one rounding.
__host__ __device__ __forceinline__ float fmr(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__host__ __device__ __forceinline__ double fmr(double a, double b, double c) { return __builtin_fma(a, b, c); }

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
    // relaxation rates divided by the squared norms of their rows of M
    // (Eq. 30) and N (Eq. 37), negated: the moment changes come out
    // already scaled for the inverse transform
    real nsn36, nsn4, nsq12;   // -s_nu/36, -s_nu/4, -s_q/12
    real nsn12;                // -s_nu/12: the epsilon change from a third of m8 - m8_eq
    real nsk2, nse20, nsg4;    // -sigma_k/2, -sigma_e/20, -sigma_nu/4
    real gbh, gy0h, gxh;       // gbeta/2, gy0/2, gx/2 (exact halves): the force image uses G/2
};

// Sum over a 64-wide wavefront (FP64).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Pre-collision populations in, post-collision populations out (Eq. 25 and
// Eq. 36 right-hand sides).  The moments of Eq. 30 and Eq. 37 are expanded
// into the +-1/+-2/+-4 sums the matrices encode; the inverse transforms use
// M^-1 = M^T diag(1/9, 1/6, 1/6, 1/36, 1/4, 1/4, 1/12, 1/12, 1/36) and
// N^-1 = N^T diag(1/5, 1/2, 1/2, 1/20, 1/4) (both matrices have orthogonal
// rows), and only the moment changes are transformed back.  Moment order:
// 1 j_x, 2 j_y, 3 e, 4 p_xx, 5 p_xy, 6 q_x, 7 q_y, 8 epsilon.  The
// distances of the non-conserved moments from the equilibria of Eq. 34 are
// formed directly from the population sums: the density deviation cancels
// from both energy moments, and q_x + u, q_y + v reduce to one term each.
// With GX false the horizontal force is zero (the cavity, G = (0, G_y) of
// Eq. 27) and its terms are left out.
template <typename real, bool GX = false>
__host__ __device__ __forceinline__ void collide(real (&f)[9], real (&g)[5], const Coef<real>& c,
                                        real& theta_out, real& ux_out, real& uy_out)
{
    const real two = real(2), four = real(4);
    // Eq. 33, Eq. 41
    const real p13 = f[1] + f[3], p24 = f[2] + f[4], p57 = f[5] + f[7], p68 = f[6] + f[8];
    const real d13 = f[1] - f[3], d24 = f[2] - f[4], d57 = f[5] - f[7], d86 = f[8] - f[6];
    const real s1234 = p13 + p24, s5678 = p57 + p68;
    const real w = d57 + d86, z = d57 - d86;
    const real u = d13 + w, v = d24 + z;
    const real g13 = g[1] + g[3], g24 = g[2] + g[4];
    const real gs = g13 + g24;
    const real theta = g[0] + gs;

    // m_k - m_k^eq for rows 3-8 of Eq. 30 against Eq. 34 (energy moment
    // with the factor 3):
    //   r3 = e + 2 drho - 3|u|^2 = -2 f0 + s1234 + 4 s5678 - 3|u|^2
    //   r8 = (epsilon - drho + 3|u|^2) / 3 = f0 - s1234 + |u|^2
    //   r4 = p_xx - (u^2 - v^2), r5 = p_xy - uv
    //   r6 = q_x + u = 2 w - d13, r7 = q_y + v = 2 z - d24
    const real uu = u * u, vv = v * v, uv = u * v;
    const real q2 = uu + vv, e4 = uu - vv;
    const real r3 = fmr(real(-3), q2, fmr(four, s5678, fmr(-two, f[0], s1234)));
    const real r8 = (f[0] - s1234) + q2;
    const real r4 = (p13 - p24) - e4, r5 = (p57 - p68) - uv;
    const real r6 = fmr(two, w, -d13), r7 = fmr(two, z, -d24);

    // moment image of the force of Eq. 26, 3 G.(e_i - u) f_i^eq(rho0, u),
    // divided by the squared row norms, in terms of H = G / 2:
    //   F3 = (H.u)(2/3 - |u|^2) / 2 = (H.u)(1/3 - |u|^2 / 2)      F8 = -F3
    //   F4 = Hx u (1 - 3(u^2 - v^2)/2) - Hy v (1 + 3(u^2 - v^2)/2)
    //   F5 = Hx v (1/2 - 3u^2/2) + Hy u (1/2 - 3v^2/2)
    //   F6 = Hy uv + Hx (v^2/2 - 1/6)          F7 = Hx uv + Hy (u^2/2 - 1/6)
    const real Hy = fmr(c.gbh, theta, c.gy0h);
    const real Hv = Hy * v, Hu = Hy * u;
    const real h3 = fmr(real(-0.5), q2, real(1.0 / 3.0));
    real F3, F4, F5, F6, F7, a1;
    if constexpr (GX) {
        const real Hx = c.gxh;
        F3 = fmr(Hx, u, Hv) * h3;
        F4 = fmr(Hx * u, fmr(real(-1.5), e4, real(1)), Hv * fmr(real(-1.5), e4, real(-1)));
        F5 = fmr(Hx * v, fmr(real(-1.5), uu, real(0.5)), Hu * fmr(real(-1.5), vv, real(0.5)));
        F6 = fmr(Hx, fmr(real(0.5), vv, real(-1.0 / 6.0)), Hy * uv);
        F7 = fmr(Hx, uv, Hy * fmr(real(0.5), uu, real(-1.0 / 6.0)));
        a1 = Hx * real(1.0 / 3.0);
    } else {
        F3 = Hv * h3;
        F4 = Hv * fmr(real(-1.5), e4, real(-1));
        F5 = Hu * fmr(real(-1.5), vv, real(0.5));
        F6 = Hy * uv;
        F7 = Hy * fmr(real(0.5), uu, real(-1.0 / 6.0));
        a1 = real(0);
    }

    // scaled moment changes -S (m - m_eq) + F   (Eq. 28, Eq. 31)
    const real a2 = Hy * real(1.0 / 3.0);
    const real a3 = fmr(c.nsn36, r3, F3);
    const real a8 = fmr(c.nsn12, r8, -F3);
    const real a4 = fmr(c.nsn4, r4, F4);
    const real a5 = fmr(c.nsn4, r5, F5);
    const real a6 = fmr(c.nsq12, r6, F6);
    const real a7 = fmr(c.nsq12, r7, F7);

    // f += M^T a
    const real A = fmr(-two, a8, -a3);          // f1..f4: -a3 - 2 a8
    const real D = fmr(two, a3, a8);            // f5..f8: 2 a3 + a8
    const real P = A + a4, Q = A - a4;
    const real V1 = fmr(-two, a7, a2);
    const real X = GX ? a1 + a6 : a6;
    const real Y = a2 + a7;
    const real S = X + Y, T = Y - X, Rp = D + a5, Rm = D - a5;
    f[0] = fmr(four, a8 - a3, f[0]);
    if constexpr (GX) {
        const real U1 = fmr(-two, a6, a1);
        f[1] += P + U1;
        f[3] += P - U1;
    } else {
        f[1] = fmr(-two, a6, f[1] + P);
        f[3] = fmr(two, a6, f[3] + P);
    }
    f[2] += Q + V1;
    f[4] += Q - V1;
    f[5] += Rp + S;
    f[7] += Rp - S;
    f[6] += Rm + T;
    f[8] += Rm - T;

    // D2Q5, Eqs. 36-42 (last row of N read as e_x^2 - e_y^2): with the
    // changes b1 = -sk/2 (n1 - u theta), b2 = -sk/2 (n2 - v theta),
    // b3 = -se/20 (n3 - a theta), b4 = -snu/4 n4,
    // g0 -= 4 b3, g1,3 += b3 + b4 +- b1, g2,4 += b3 - b4 +- b2
    const real b3 = c.nse20 * fmr(-c.a, theta, fmr(-four, g[0], gs));
    const real d4 = g13 - g24;
    const real t34 = fmr(c.nsg4, d4, b3), t34m = fmr(-c.nsg4, d4, b3);
    const real dx = fmr(-u, theta, g[1] - g[3]), dy = fmr(-v, theta, g[2] - g[4]);
    g[0] = fmr(-four, b3, g[0]);
    g[1] = fmr(c.nsk2, dx, g[1] + t34);
    g[3] = fmr(-c.nsk2, dx, g[3] + t34);
    g[2] = fmr(c.nsk2, dy, g[2] + t34m);
    g[4] = fmr(-c.nsk2, dy, g[4] + t34m);

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
    // Nusselt samples taken by a K-step launch: for every step t + j
    // (1 <= j <= K) whose bit is set in samp_mask, the temperature sums of
    // the post-collision g at x = 0 and x = 1 of every row go to slot
    // (number of set bits below j) of samp, samp[slot * 2 n + 2 y + x]
    // (FP64, summed as the Nusselt kernels sum)
    double* __restrict__ samp = nullptr;
    int samp_mask = 0;
    // adjoint recompute: the linearisation point (u, v, theta planes) of
    // every step, step t + j at lp + (j - 1) lslot
    real* __restrict__ lp = nullptr;
    long lslot = 0;
    // non-finite watchdog folded into the launch: the last wblocks
    // workgroups of the grid check the wall columns of (fin, gin) and set
    // *wflag when one holds a non-finite value (wall_check_blocks)
    int* __restrict__ wflag = nullptr;
    int wblocks = 0;
};

// Non-finite test of wall node t (0 <= t < 2n: row t / 2, column 0 for even
// t, n - 1 for odd t) of the state (fs, gs): the sum of the magnitudes of
// its 14 populations is not finite.  A non-finite value anywhere in the
// cavity reaches one of the two wall columns within n steps (information
// moves one node per step).
template <typename real>
__device__ __forceinline__ bool wall_node_bad(const real* __restrict__ fs, const real* __restrict__ gs, int n,
                                              int pitch, int plane, int t)
{
    const int y = t >> 1, x = (t & 1) ? n - 1 : 0;
    const int k = y * pitch + x;
    real s = real(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) s += fabs(fs[i * plane + k]);
#pragma unroll
    for (int i = 0; i < 5; ++i) s += fabs(gs[i * plane + k]);
    return !isfinite(s);
}

// The workgroups past the stepping grid (the last A.wblocks of it, each
// thread one wall node of the launch's input) run the watchdog and return
// true; the others return false at once (a uniform test per workgroup).
template <typename real>
__device__ __forceinline__ bool wall_check_blocks(const StepArgs<real>& A)
{
    const int first = int(gridDim.x) - A.wblocks;
    if (int(blockIdx.x) < first) return false;
    const int nt = blockDim.x * blockDim.y;
    const int t = (int(blockIdx.x) - first) * nt + threadIdx.y * blockDim.x + threadIdx.x;
    int bad = t < 2 * A.n ? wall_node_bad(A.fin, A.gin, A.n, A.pitch, A.plane, t) : 0;
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0 && threadIdx.y == 0 && bad) *A.wflag = 1;
    return true;
}

// Temperature sum of a node's post-collision g in FP64, in the order the
// Nusselt kernels use, into the sample slot of step t + j when x is 0 or 1
// (lanes left of the wall, x < 0, write nothing).
template <typename real>
__device__ __forceinline__ void samp_put(const StepArgs<real>& A, int j, int x, int y, const real (&g)[5])
{
    if (x == 0 || x == 1) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < 5; ++i) t += double(g[i]);
        const int slot = __builtin_popcount(unsigned(A.samp_mask) & ((1u << j) - 1u));
        A.samp[(size_t)slot * 2 * A.n + 2 * y + x] = t;
    }
}

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

// Element at byte offset `b` from `base`: a uniform base pointer and a
// 32-bit per-lane offset, so a load needs no 64-bit address arithmetic.
template <typename real>
__device__ __forceinline__ real ldb(const real* __restrict__ base, unsigned b)
{
    return *reinterpret_cast<const real*>(reinterpret_cast<const char*>(base) + b);
}
template <typename real>
__device__ __forceinline__ void stb(real* __restrict__ base, unsigned b, real v)
{
    *reinterpret_cast<real*>(reinterpret_cast<char*>(base) + b) = v;
}

// Raw buffer access: element at byte offset voff + soff of the array at p,
// with voff per lane (a VGPR) and soff uniform (an SGPR), so that a fixed
// per-lane offset and a uniform row offset meet in the instruction itself.
// Offsets stay below 4 GiB (the state's planes do, see the size limit).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, int(0xffffffffu), 0x00020000);
}
template <typename real>
__device__ __forceinline__ real bld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    if constexpr (sizeof(real) == 4)
        return __builtin_bit_cast(real, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    else
        return __builtin_bit_cast(real, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <typename real>
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, real v)
{
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    if constexpr (sizeof(real) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}

// Wall temperature of row y, uniform per wave: a scalar load through the
// constant address space, which does not wait for vector memory operations
// in flight.
template <typename real>
__device__ __forceinline__ real thw_row(const real* thw, int y)
{
    typedef const __attribute__((address_space(4))) real creal;
    return ((creal*)thw)[y];
}

// Pull-streaming with the wall rules (Eq. 25, Eqs. 44-45): f_i(r) = f*_i(r - e_i) when
// r - e_i is inside, else the halfway bounce-back f*_opp(i)(r); for g the
// same, with Eq. 44 on adiabatic walls and Eq. 45 on the isothermal walls.
template <typename real, int BC>
__device__ __forceinline__ void gather(const real* __restrict__ fi, const real* __restrict__ gi,
                                       const real* __restrict__ thw, int n, int pitch, int P,
                                       int x, int y, const Coef<real>& c, real (&f)[9], real (&g)[5])
{
    if constexpr (BC == BC_CAVITY) {
        // every offset below is >= 0 (plane index >= 1 for the neighbour reads)
        constexpr unsigned E = sizeof(real);
        const unsigned kb = unsigned(y * pitch + x) * E, Pb = unsigned(P) * E, rb = unsigned(pitch) * E;
        const bool hxm = x > 0, hxp = x < n - 1, hym = y > 0, hyp = y < n - 1;
        f[0] = ldb(fi, kb);
        f[1] = ldb(fi, hxm ? kb + Pb - E : kb + 3 * Pb);
        f[2] = ldb(fi, hym ? kb + 2 * Pb - rb : kb + 4 * Pb);
        f[3] = ldb(fi, hxp ? kb + 3 * Pb + E : kb + Pb);
        f[4] = ldb(fi, hyp ? kb + 4 * Pb + rb : kb + 2 * Pb);
        f[5] = ldb(fi, (hxm && hym) ? kb + 5 * Pb - rb - E : kb + 7 * Pb);
        f[6] = ldb(fi, (hxp && hym) ? kb + 6 * Pb - rb + E : kb + 8 * Pb);
        f[7] = ldb(fi, (hxp && hyp) ? kb + 7 * Pb + rb + E : kb + 5 * Pb);
        f[8] = ldb(fi, (hxm && hyp) ? kb + 8 * Pb + rb - E : kb + 6 * Pb);
        g[0] = ldb(gi, kb);
        g[2] = ldb(gi, hym ? kb + 2 * Pb - rb : kb + 4 * Pb);        // Eq. 44
        g[4] = ldb(gi, hyp ? kb + 4 * Pb + rb : kb + 2 * Pb);
        // one read per link, the address selected, so no read sits in a
        // branch; Eq. 45 is applied to the value afterwards.  Every launch
        // shape has rows of a multiple of 64 threads, so y is uniform per
        // wavefront and the wall temperature is one scalar read.
        const real g1 = ldb(gi, hxm ? kb + Pb - E : kb + 3 * Pb);
        const real g3 = ldb(gi, hxp ? kb + 3 * Pb + E : kb + Pb);
        const real tw = thw_row<real>(thw, __builtin_amdgcn_readfirstlane(y));
        g[1] = hxm ? g1 : fmr(c.cabb, tw, -g1);                      // Eq. 45
        g[3] = hxp ? g3 : c.cold - g3;
        return;
    }
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
        g[1] = hxm ? gi[1 * P + k + dxm] : fmr(c.cabb, thw[y], -gi[3 * P + k]);
        g[3] = hxp ? gi[3 * P + k + dxp] : c.cold - gi[1 * P + k];
    } else {
        g[1] = hxm ? gi[1 * P + k + dxm] : gi[3 * P + k];
        g[3] = hxp ? gi[3 * P + k + dxp] : gi[1 * P + k];
    }
}

// The cavity gather split in two for prefetching: the loads alone, with
// selected addresses but no branches (every address in bounds for x, y in
// [0, n)), and the isothermal-wall formula of Eq. 45 applied to them where
// the values are used; together they give exactly gather<real, BC_CAVITY>.
template <typename real>
__device__ __forceinline__ void gather_cavity_loads(const real* __restrict__ fi, const real* __restrict__ gi,
                                                    int n, int pitch, int P, int x, int y, real (&f)[9],
                                                    real (&g)[5])
{
    constexpr unsigned E = sizeof(real);
    const unsigned kb = unsigned(y * pitch + x) * E, Pb = unsigned(P) * E, rb = unsigned(pitch) * E;
    const bool hxm = x > 0, hxp = x < n - 1, hym = y > 0, hyp = y < n - 1;
    f[0] = ldb(fi, kb);
    f[1] = ldb(fi, hxm ? kb + Pb - E : kb + 3 * Pb);
    f[2] = ldb(fi, hym ? kb + 2 * Pb - rb : kb + 4 * Pb);
    f[3] = ldb(fi, hxp ? kb + 3 * Pb + E : kb + Pb);
    f[4] = ldb(fi, hyp ? kb + 4 * Pb + rb : kb + 2 * Pb);
    f[5] = ldb(fi, (hxm && hym) ? kb + 5 * Pb - rb - E : kb + 7 * Pb);
    f[6] = ldb(fi, (hxp && hym) ? kb + 6 * Pb - rb + E : kb + 8 * Pb);
    f[7] = ldb(fi, (hxp && hyp) ? kb + 7 * Pb + rb + E : kb + 5 * Pb);
    f[8] = ldb(fi, (hxm && hyp) ? kb + 8 * Pb + rb - E : kb + 6 * Pb);
    g[0] = ldb(gi, kb);
    g[1] = ldb(gi, hxm ? kb + Pb - E : kb + 3 * Pb);
    g[2] = ldb(gi, hym ? kb + 2 * Pb - rb : kb + 4 * Pb);        // Eq. 44
    g[3] = ldb(gi, hxp ? kb + 3 * Pb + E : kb + Pb);
    g[4] = ldb(gi, hyp ? kb + 4 * Pb + rb : kb + 2 * Pb);
}

template <typename real>
__device__ __forceinline__ void gather_cavity_walls(real thw_y, int n, int x, const Coef<real>& c, real (&g)[5])
{
    if (x == 0) g[1] = fmr(c.cabb, thw_y, -g[1]);                // Eq. 45
    if (x == n - 1) g[3] = c.cold - g[3];
}

// One node update (Eqs. 25-45): gather from the current copy with the wall
// rules, collide in registers, store into the other copy.  Returns the
// node's temperature sum of the stored g* in FP64 (used only by the
// Nusselt-accumulating variant; dead code elsewhere).
template <typename real, int BC>
__device__ __forceinline__ double node_update(const real* __restrict__ fi, const real* __restrict__ gi,
                                              real* __restrict__ fo, real* __restrict__ go,
                                              const real* __restrict__ thw, int n, int pitch, int P,
                                              int x, int y, const Coef<real>& c)
{
    real f[9], g[5];
    gather<real, BC>(fi, gi, thw, n, pitch, P, x, y, c, f, g);
    real th, ux, uy;
    collide<real, BC != BC_CAVITY>(f, g, c, th, ux, uy);
    const unsigned kb = unsigned(y * pitch + x) * sizeof(real), Pb = unsigned(P) * sizeof(real);
#pragma unroll
    for (int i = 0; i < 9; ++i) stb(fo, kb + i * Pb, f[i]);
#pragma unroll
    for (int i = 0; i < 5; ++i) stb(go, kb + i * Pb, g[i]);
    double ts = 0.0;
#pragma unroll
    for (int i = 0; i < 5; ++i) ts += double(g[i]);
    return ts;
}

template <typename real, int BC>
__global__ void __launch_bounds__(1024) step_kernel(StepArgs<real> A)
{
    if (wall_check_blocks(A)) return;
    const int tile = tile_of_block(blockIdx.x, gridDim.x - A.wblocks, A.xcd_remap);
    if (tile >= A.tiles) return;
    const int ty = tile / A.tiles_x;
    const int tx = tile - ty * A.tiles_x;
    const int x = tx * blockDim.x + threadIdx.x;
    const int y = ty * blockDim.y + threadIdx.y;
    if (x >= A.n || y >= A.n) return;
    node_update<real, BC>(A.fin, A.gin, A.fout, A.gout, A.thw, A.n, A.pitch, A.plane, x, y, A.c);
}

// Cavity step that also accumulates, per row, the hot-wall Nusselt sum
// 8 theta_w - 9 theta(0, y) + theta(1, y) of the new step (Eqs. 18-19) into
// acc[y] in FP64 (one writer per row; launches are ordered).  Tiles start
// at multiples of blockDim.x >= 64, so x = 0 and x = 1 share a wavefront.
template <typename real>
__global__ void __launch_bounds__(1024) step_nu_kernel(StepArgs<real> A, const double* __restrict__ thw_d,
                                                       double* __restrict__ acc)
{
    const int tile = tile_of_block(blockIdx.x, gridDim.x, A.xcd_remap);
    if (tile >= A.tiles) return;
    const int ty = tile / A.tiles_x;
    const int tx = tile - ty * A.tiles_x;
    const int x = tx * blockDim.x + threadIdx.x;
    const int y = ty * blockDim.y + threadIdx.y;
    const bool valid = x < A.n && y < A.n;
    double ts = 0.0;
    if (valid)
        ts = node_update<real, BC_CAVITY>(A.fin, A.gin, A.fout, A.gout, A.thw, A.n, A.pitch, A.plane,
                                          x, y, A.c);
    const double ts1 = __shfl_down(ts, 1, 64);
    if (valid && x == 0) acc[y] += 8.0 * thw_d[y] - 9.0 * ts + ts1;
}

// ---------------------------------------------------------------------------
// Adjoint (reverse mode) of the step
// ---------------------------------------------------------------------------
// Vector-Jacobian product of collide() at the pre-collision state (f, g)
// for the cavity (G_x = 0): on entry lf, lg hold the adjoints of the
// post-collision populations, on exit the adjoints of the pre-collision
// ones.  Derived by hand from the moment form of collide(): since
// f* = f + M^T a, the adjoints of the scaled moment changes are La = M lf
// (the forward moment transform applied to lf); they flow back through the
// relaxation, the equilibria of Eq. 34 and Eq. 42 and the force image of
// Eq. 26 into drho, u, v, theta and the non-conserved moments, and return
// to the populations as lf += M^T (Ldrho, Lu, Lv, Lm3, ..., Lm8) (the
// forward reconstruction, here with density and momentum terms), likewise
// lg += N^T (...) + Ltheta for D2Q5.
//
// The Jacobian depends on the pre-collision state only through its velocity
// (u, v) and temperature theta (the relaxation and the moment transforms
// are linear, the equilibria of Eq. 34 and Eq. 42 and the force image of
// Eq. 26 are functions of u, v, theta), so collide_vjp_at takes just those
// three values: the forward step's own u, v, theta, bitwise.
template <typename real>
__host__ __device__ __forceinline__ void collide_vjp_at(real u, real v, real theta, const Coef<real>& c,
                                                        real (&lf)[9], real (&lg)[5])
{
    const real two = real(2), four = real(4);
    const real uu = u * u, vv = v * v, uv = u * v;
    const real q2 = uu + vv, e4 = uu - vv;
    const real Gy = fmr(c.gbeta, theta, c.gy0);
    const real Gv = Gy * v, Gu = Gy * u;
    const real h3 = fmr(real(-0.25), q2, real(1.0 / 6.0));

    // La = M lf
    const real lp13 = lf[1] + lf[3], lp24 = lf[2] + lf[4], lp57 = lf[5] + lf[7], lp68 = lf[6] + lf[8];
    const real ld13 = lf[1] - lf[3], ld24 = lf[2] - lf[4], ld57 = lf[5] - lf[7], ld86 = lf[8] - lf[6];
    const real ls1234 = lp13 + lp24, ls5678 = lp57 + lp68;
    const real lw = ld57 + ld86, lz = ld57 - ld86;
    const real La2 = ld24 + lz;
    const real La3 = fmr(-four, lf[0], fmr(two, ls5678, -ls1234));
    const real La4 = lp13 - lp24;
    const real La5 = lp57 - lp68;
    const real La6 = fmr(-two, ld13, lw);
    const real La7 = fmr(-two, ld24, lz);
    const real La8 = fmr(four, lf[0], fmr(-two, ls1234, ls5678));

    // relaxation: a_k = -s_k/|row k|^2 r_k + F_k, r_k = m_k - m_k^eq
    const real Lr3 = c.nsn36 * La3, Lr8 = c.nsn36 * La8;
    const real Lr4 = c.nsn4 * La4, Lr5 = c.nsn4 * La5;
    const real Lr6 = c.nsq12 * La6, Lr7 = c.nsq12 * La7;
    // force image (F3 = Gv h3 enters a3 and -a8; F4 = Gv (-1/2 - 3/4 e4);
    // F5 = Gu (1/4 - 3/4 v^2); F6 = Gy uv/2; F7 = Gy (u^2/4 - 1/12))
    const real LF3 = La3 - La8;
    const real LGv = fmr(LF3, h3, La4 * fmr(real(-0.75), e4, real(-0.5)));
    const real LGu = La5 * fmr(real(-0.75), vv, real(0.25));
    // the quadratic terms of the equilibria and of the force image
    const real Lq2 = fmr(real(-0.25) * Gv, LF3, real(3) * (Lr8 - Lr3));
    const real E = fmr(real(-0.75) * Gv, La4, -Lr4);                   // d/d(u^2 - v^2)
    const real Luu = fmr(real(0.25) * Gy, La7, Lq2 + E);
    const real Lvv = fmr(real(-0.75) * Gu, La5, Lq2 - E);
    const real Luv = fmr(real(0.5) * Gy, La6, -Lr5);
    const real LGy = fmr(LGu, u, fmr(LGv, v, fmr(La7, fmr(real(0.25), uu, real(-1.0 / 12.0)),
                                                 fmr(La6, real(0.5) * uv, La2 * real(1.0 / 6.0)))));

    // D2Q5: b1 = -sk/2 (n1 - u theta), b2 = -sk/2 (n2 - v theta),
    // b3 = -se/20 (n3 - a theta), b4 = -snu/4 n4
    const real lg13 = lg[1] + lg[3], lg24 = lg[2] + lg[4];
    const real Ln1 = c.nsk2 * (lg[1] - lg[3]);
    const real Ln2 = c.nsk2 * (lg[2] - lg[4]);
    const real Ln3 = c.nse20 * fmr(-four, lg[0], lg13 + lg24);
    const real Ln4 = c.nsg4 * (lg13 - lg24);

    const real Lu = fmr(-theta, Ln1, fmr(two * u, Luu, fmr(v, Luv, fmr(LGu, Gy, Lr6))));
    const real Lv = fmr(-theta, Ln2, fmr(two * v, Lvv, fmr(u, Luv, fmr(LGv, Gy, Lr7))));
    const real Ldrho = fmr(two, Lr3, -Lr8);
    const real Lth = fmr(-c.a, Ln3, fmr(-v, Ln2, fmr(-u, Ln1, c.gbeta * LGy)));

    // lf += M^T (Ldrho, Lu, Lv, Lr3, Lr4, Lr5, Lr6, Lr7, Lr8)
    const real A = fmr(-two, Lr8, -Lr3) + Ldrho;
    const real D = fmr(two, Lr3, Lr8) + Ldrho;
    const real P = A + Lr4, Q = A - Lr4;
    const real U1 = fmr(-two, Lr6, Lu), V1 = fmr(-two, Lr7, Lv);
    const real X = Lu + Lr6, Y = Lv + Lr7;
    const real S = X + Y, T = Y - X, Rp = D + Lr5, Rm = D - Lr5;
    lf[0] = fmr(four, Lr8 - Lr3, lf[0] + Ldrho);
    lf[1] += P + U1;
    lf[3] += P - U1;
    lf[2] += Q + V1;
    lf[4] += Q - V1;
    lf[5] += Rp + S;
    lf[7] += Rp - S;
    lf[6] += Rm + T;
    lf[8] += Rm - T;
    // lg += N^T (., Ln1, Ln2, Ln3, Ln4) + Ltheta
    const real t34 = (Ln3 + Ln4) + Lth, t34m = (Ln3 - Ln4) + Lth;
    lg[0] = fmr(-four, Ln3, lg[0] + Lth);
    lg[1] += Ln1 + t34;
    lg[3] += t34 - Ln1;
    lg[2] += Ln2 + t34m;
    lg[4] += t34m - Ln2;
}

// The same at the pre-collision state (f, g), with u, v, theta formed as
// collide() forms them.
template <typename real>
__host__ __device__ __forceinline__ void collide_vjp(const real (&f)[9], const real (&g)[5], const Coef<real>& c,
                                            real (&lf)[9], real (&lg)[5])
{
    const real d13 = f[1] - f[3], d24 = f[2] - f[4], d57 = f[5] - f[7], d86 = f[8] - f[6];
    const real u = d13 + (d57 + d86), v = d24 + (d57 - d86);
    const real theta = g[0] + ((g[1] + g[3]) + (g[2] + g[4]));
    collide_vjp_at<real>(u, v, theta, c, lf, lg);
}

template <typename real>
struct AdjArgs {
    // linearisation point of step m (segment slot j - 1): the u, v and
    // theta planes of the pre-collision state p(m), as the forward step
    // computed them
    const real* __restrict__ lp;
    const real* __restrict__ lin;    // mu(m+1): 14 planes (f then g)
    real* __restrict__ lout;         // mu(m), or mu(m-K+1) for K steps per launch
    const real* __restrict__ thw;
    double* __restrict__ gthw;       // accumulates dJ/dtheta_w (anti-bounce-back links)
    const int* __restrict__ n0p;     // step index of the segment's first state
    int j;                           // m = *n0p + j is the newest step of this launch
    int win_start;                   // first step of the objective window
    real seed0, seed1;               // dJ/dg*_i(m) at x = 0 and x = 1 for m in the window
    double cabb;                     // Eq. 45 constant in FP64
    long lslot;                      // elements between consecutive segment slots (3 planes)
    int n, pitch, plane, tiles_x, tiles;
    int xcd_remap;
    Coef<real> c;
};

// dJ/dg*_i(m) at column x: the Nusselt objective (Eqs. 18-19) reads the
// temperatures of the two columns next to the hot wall on window steps.
template <typename real>
__device__ __forceinline__ real adj_seed_at(int x, bool win, real s0, real s1)
{
    return win ? (x == 0 ? s0 : (x == 1 ? s1 : real(0))) : real(0);
}

// lambda(m) = S^T mu(m+1) + dJ/ds(m) at node (x, y), with mu(m+1) in global
// memory.  The streaming/wall map S of step m + 1 sends population i of
// s(m) at r to r + e_i, or, across a wall, back into population opp(i) at
// r (sign -1 on the anti-bounce-back links of Eq. 45), so its transpose is
// a pull in the direction opposite to the forward gather.
template <typename real>
__device__ __forceinline__ void adj_pull(const real* __restrict__ mu, int n, int pitch, int P, int x,
                                         int y, real sd, real (&lf)[9], real (&lg)[5])
{
    // every offset below is >= 0 (plane index >= 1 for the neighbour reads)
    constexpr unsigned E = sizeof(real);
    const unsigned kb = unsigned(y * pitch + x) * E, Pb = unsigned(P) * E, rb = unsigned(pitch) * E;
    const bool hxm = x > 0, hxp = x < n - 1, hym = y > 0, hyp = y < n - 1;
    lf[0] = ldb(mu, kb);
    lf[1] = ldb(mu, hxp ? kb + Pb + E : kb + 3 * Pb);
    lf[2] = ldb(mu, hyp ? kb + 2 * Pb + rb : kb + 4 * Pb);
    lf[3] = ldb(mu, hxm ? kb + 3 * Pb - E : kb + Pb);
    lf[4] = ldb(mu, hym ? kb + 4 * Pb - rb : kb + 2 * Pb);
    lf[5] = ldb(mu, (hxp && hyp) ? kb + 5 * Pb + rb + E : kb + 7 * Pb);
    lf[6] = ldb(mu, (hxm && hyp) ? kb + 6 * Pb + rb - E : kb + 8 * Pb);
    lf[7] = ldb(mu, (hxm && hym) ? kb + 7 * Pb - rb - E : kb + 5 * Pb);
    lf[8] = ldb(mu, (hxp && hym) ? kb + 8 * Pb - rb + E : kb + 6 * Pb);
    const real* __restrict__ mg = mu + 9 * P;
    // one load per link (the address selected), so no load sits in a branch
    const real m1 = ldb(mg, hxp ? kb + Pb + E : kb + 3 * Pb);
    const real m3 = ldb(mg, hxm ? kb + 3 * Pb - E : kb + Pb);
    lg[0] = ldb(mg, kb) + sd;
    lg[1] = hxp ? m1 + sd : sd - m1;                                               // Eq. 45, right wall
    lg[2] = ldb(mg, hyp ? kb + 2 * Pb + rb : kb + 4 * Pb) + sd;                    // Eq. 44
    lg[3] = hxm ? m3 + sd : sd - m3;                                               // Eq. 45, left wall
    lg[4] = ldb(mg, hym ? kb + 4 * Pb - rb : kb + 2 * Pb) + sd;
}

// Adjoint of step m for the cavity: lambda(m) = S^T mu(m+1) + dJ/ds(m),
// mu(m) = C'(p(m))^T lambda(m), the Jacobian taken at the linearisation
// point of step m (segment slot j - 1).  Storing mu rather than lambda
// makes the transposed streaming a pull, so every thread writes only its
// own node.  The derivative of the anti-bounce-back constant feeds
// dJ/dtheta_w at the hot wall.
template <typename real>
__device__ __forceinline__ void adj_tile(const AdjArgs<real>& A, int tile)
{
    const int ty = tile / A.tiles_x;
    const int tx = tile - ty * A.tiles_x;
    const int x = tx * blockDim.x + threadIdx.x;
    const int y = ty * blockDim.y + threadIdx.y;
    const int n = A.n;
    if (x >= n || y >= n) return;
    const int P = A.plane, k = y * A.pitch + x;
    const int m = *A.n0p + A.j;
    real lf[9], lg[5];
    adj_pull<real>(A.lin, n, A.pitch, P, x, y, adj_seed_at<real>(x, m >= A.win_start, A.seed0, A.seed1),
                   lf, lg);
    collide_vjp_at<real>(A.lp[k], A.lp[P + k], A.lp[2 * P + k], A.c, lf, lg);
    const unsigned kb = unsigned(k) * sizeof(real), Pb = unsigned(P) * sizeof(real);
#pragma unroll
    for (int i = 0; i < 9; ++i) stb(A.lout, kb + i * Pb, lf[i]);
#pragma unroll
    for (int i = 0; i < 5; ++i) stb(A.lout, kb + (9 + i) * Pb, lg[i]);
    if (x == 0) A.gthw[y] = __builtin_fma(A.cabb, double(lg[1]), A.gthw[y]);
}

// Linearisation point of a node: the u, v, theta of its pre-collision
// state (collide's outputs) into the three planes at lp.
template <typename real>
__device__ __forceinline__ void store_lp(real* __restrict__ lp, int P, int k, real u, real v, real theta)
{
    lp[k] = u;
    lp[P + k] = v;
    lp[2 * P + k] = theta;
}

template <typename real>
__global__ void __launch_bounds__(1024) adj_step_kernel(AdjArgs<real> A)
{
    if ((int)blockIdx.x >= A.tiles) return;
    adj_tile<real>(A, blockIdx.x);
}

// One forward step of the recompute: gather, collide, store the state and
// the node's linearisation point (R.lp).
template <typename real>
__device__ __forceinline__ void rec_node(const StepArgs<real>& R, int x, int y)
{
    real f[9], g[5];
    gather<real, BC_CAVITY>(R.fin, R.gin, R.thw, R.n, R.pitch, R.plane, x, y, R.c, f, g);
    real th, ux, uy;
    collide<real>(f, g, R.c, th, ux, uy);
    const int k = y * R.pitch + x, P = R.plane;
#pragma unroll
    for (int i = 0; i < 9; ++i) R.fout[i * P + k] = f[i];
#pragma unroll
    for (int i = 0; i < 5; ++i) R.gout[i * P + k] = g[i];
    store_lp<real>(R.lp, P, k, ux, uy, th);
}

template <typename real>
__global__ void __launch_bounds__(1024) rec_step_kernel(StepArgs<real> R)
{
    const int tile = tile_of_block(blockIdx.x, gridDim.x, R.xcd_remap);
    if (tile >= R.tiles) return;
    const int ty = tile / R.tiles_x;
    const int tx = tile - ty * R.tiles_x;
    const int x = tx * blockDim.x + threadIdx.x;
    const int y = ty * blockDim.y + threadIdx.y;
    if (x >= R.n || y >= R.n) return;
    rec_node<real>(R, x, y);
}

// One adjoint step of the current segment and, in the same launch, one
// forward step recomputing the next (older) segment: the two touch disjoint
// buffers.  Workgroups [0, A.tiles) take adjoint tiles, the rest take
// recompute tiles of R.
template <typename real>
__global__ void __launch_bounds__(1024) adj_fused_kernel(AdjArgs<real> A, StepArgs<real> R)
{
    const int b = blockIdx.x;
    if (b < A.tiles) {
        adj_tile<real>(A, b);
        return;
    }
    const int tile = b - A.tiles;
    if (tile >= R.tiles) return;
    const int ty = tile / R.tiles_x;
    const int tx = tile - ty * R.tiles_x;
    const int x = tx * blockDim.x + threadIdx.x;
    const int y = ty * blockDim.y + threadIdx.y;
    if (x >= R.n || y >= R.n) return;
    rec_node<real>(R, x, y);
}

// mu(N+1) = 0: the first adjoint step then forms lambda(N) = dJ/ds(N).
template <typename real>
__global__ void adj_zero_kernel(real* __restrict__ mu, int n, int pitch, int plane)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= n || y >= n) return;
    const int k = y * pitch + x;
#pragma unroll
    for (int i = 0; i < 14; ++i) mu[i * plane + k] = real(0);
}

// dJ/dtheta0 from mu(1): lambda(0) = S^T mu(1) + dJ/ds(0); the initial
// pre-collision state is f = 0, g_i = w_i theta0, so
// dJ/dtheta0 = sum_i w_i (C'(p(0))^T lambda(0))_g,i.
template <typename real>
__global__ void adj_init_grad_kernel(const real* __restrict__ mu, const double* __restrict__ theta0,
                                     int n, int pitch, int plane, Coef<real> c, real w0, real wm,
                                     bool win0, real seed0, real seed1, double* __restrict__ grad)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= n || y >= n) return;
    const real th = real(theta0[y * n + x]);
    real f[9], g[5], lf[9], lg[5];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = real(0);
    g[0] = w0 * th;
#pragma unroll
    for (int i = 1; i < 5; ++i) g[i] = wm * th;
    adj_pull<real>(mu, n, pitch, plane, x, y, adj_seed_at<real>(x, win0, seed0, seed1), lf, lg);
    collide_vjp<real>(f, g, c, lf, lg);
    grad[y * n + x] = double(w0) * double(lg[0]) +
                      double(wm) * (double(lg[1]) + double(lg[2]) + double(lg[3]) + double(lg[4]));
}

// Sum of n doubles by one workgroup (FP64).
static __global__ void __launch_bounds__(256) sum_kernel(const double* __restrict__ a, int n,
                                                   double* __restrict__ out)
{
    __shared__ double part[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += a[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += part[w];
        *out = t;
    }
}

// ---------------------------------------------------------------------------
// Several time steps per launch through LDS (temporal blocking), cavity walls.
// ---------------------------------------------------------------------------
// Workgroup of 64 x R threads; its footprint is 64 x R nodes starting K - 1
// nodes left of and below its output tile.  Phase 1: every thread computes
// s(t+1) at its footprint node from s(t) in global memory (the ordinary
// gather + collide) into LDS.  Later phases compute the next step on a
// footprint shrunk by one node per side, gathering from LDS with the same
// wall rules; the last one stores to global memory.  Each node's neighbours
// lie in the previous phase's region, so the K steps equal K single-step
// launches exactly.  Global traffic per node update: about 28 / K words
// instead of 28 (the footprint ring's re-reads hit L2).
constexpr int kFootW = 64;         // footprint width (one wavefront)

// First phase of the K-step update: s(t+1) at footprint node (x, y) into LDS.
// Every lane reads (at its node clamped into the cavity, y uniform per
// wave), so no global read sits in a branch; lanes outside the cavity
// store nothing.
template <typename real, int R>
__device__ __forceinline__ void lds_first_phase(real* lds, const real* __restrict__ fi,
                                          const real* __restrict__ gi, const real* __restrict__ thw,
                                          int n, int pitch, int P, int x, int y, int lx, int ly,
                                          bool inside, const Coef<real>& c)
{
    real f[9], g[5];
    const int xc = min(max(x, 0), n - 1), yc = min(max(y, 0), n - 1);
    gather_cavity_loads<real>(fi, gi, n, pitch, P, xc, yc, f, g);
    if (!inside) return;
    gather_cavity_walls<real>(thw_row<real>(thw, yc), n, x, c, g);
    real th, ux, uy;
    collide<real>(f, g, c, th, ux, uy);
#pragma unroll
    for (int i = 0; i < 9; ++i) lds[(i * R + ly) * kFootW + lx] = f[i];
#pragma unroll
    for (int i = 0; i < 5; ++i) lds[((9 + i) * R + ly) * kFootW + lx] = g[i];
}

// Gather of s(t+j-1) for node (x, y) from LDS with the cavity's wall rules.
// Every lane first reads the interior neighbours (one base address and
// constant offsets, all inside the footprint for an active lane); lanes on
// a wall then replace the links that cross it by the bounce-back values of
// their own node.
template <typename real, int R>
__device__ __forceinline__ void gather_lds(const real* lds, const real* __restrict__ thw, int n,
                                              int x, int y, int lx, int ly, const Coef<real>& c,
                                              real (&f)[9], real (&g)[5])
{
    constexpr int W = kFootW, PL = R * kFootW;
    const real* b = lds + (ly * W + lx);
    f[0] = b[0];
    f[1] = b[1 * PL - 1];
    f[2] = b[2 * PL - W];
    f[3] = b[3 * PL + 1];
    f[4] = b[4 * PL + W];
    f[5] = b[5 * PL - W - 1];
    f[6] = b[6 * PL - W + 1];
    f[7] = b[7 * PL + W + 1];
    f[8] = b[8 * PL + W - 1];
    g[0] = b[9 * PL];
    g[1] = b[10 * PL - 1];
    g[2] = b[11 * PL - W];
    g[3] = b[12 * PL + 1];
    g[4] = b[13 * PL + W];
    const bool hxm = x > 0, hxp = x < n - 1, hym = y > 0, hyp = y < n - 1;
    if (!(hxm && hxp && hym && hyp)) {
        // a lane on a wall (0 <= x, y < n for every caller): all own-node
        // values its wall links may take, read together, then selected; a
        // read per branch would make the wave wait for each in turn
        const real r1 = b[3 * PL], s1 = b[12 * PL], r3 = b[1 * PL], s3 = b[10 * PL];
        const real r2 = b[4 * PL], s2 = b[13 * PL], r4 = b[2 * PL], s4 = b[11 * PL];
        const real r5 = b[7 * PL], r6 = b[8 * PL], r7 = b[5 * PL], r8 = b[6 * PL];
        const real tw = thw[y];
        f[1] = hxm ? f[1] : r1;
        g[1] = hxm ? g[1] : fmr(c.cabb, tw, -s1);                  // Eq. 45
        f[3] = hxp ? f[3] : r3;
        g[3] = hxp ? g[3] : c.cold - s3;
        f[2] = hym ? f[2] : r2;
        g[2] = hym ? g[2] : s2;                                    // Eq. 44
        f[4] = hyp ? f[4] : r4;
        g[4] = hyp ? g[4] : s4;
        f[5] = hxm && hym ? f[5] : r5;
        f[6] = hxp && hym ? f[6] : r6;
        f[7] = hxp && hyp ? f[7] : r7;
        f[8] = hxm && hyp ? f[8] : r8;
    }
}

// Last phase: the final step at output node (x, y) from LDS, stored to global.
template <typename real, int R>
__device__ __forceinline__ void lds_last_phase(const real* lds, real* __restrict__ fo, real* __restrict__ go,
                                          const real* __restrict__ thw, int n, int pitch, int P, int x,
                                          int y, int lx, int ly, const Coef<real>& c)
{
    real f[9], g[5];
    gather_lds<real, R>(lds, thw, n, x, y, lx, ly, c, f, g);
    real th, ux, uy;
    collide<real>(f, g, c, th, ux, uy);
    const unsigned kb = unsigned(y * pitch + x) * sizeof(real), Pb = unsigned(P) * sizeof(real);
#pragma unroll
    for (int i = 0; i < 9; ++i) stb(fo, kb + i * Pb, f[i]);
#pragma unroll
    for (int i = 0; i < 5; ++i) stb(go, kb + i * Pb, g[i]);
}

// K steps per launch.  Footprint 64 x R nodes, output (64 - 2(K-1)) x
// (R - 2(K-1)) nodes; phase j computes step t + j on the footprint shrunk by
// j - 1 nodes on each side (phase 1 from HBM, the others from LDS; the
// intermediate phases hold their result in registers across a barrier and
// then overwrite the LDS copy), and the last phase stores to HBM.  With REC
// (the adjoint's recompute), every phase also stores the linearisation
// point (u, v, theta) of its step on the output tile (a partition of the
// domain), step t + j at A.lp + (j - 1) A.lslot.
// With NU, every step of the launch also adds its hot-wall Nusselt sum
// 8 theta_w - 9 theta(0, y) + theta(1, y) (Eqs. 18-19) to acc[y], in FP64
// and in the same order and arithmetic as step_nu_kernel; the x = 0 and
// x = 1 nodes are neighbouring lanes of one wavefront.  The owning lane
// keeps acc[y] in a register for the whole launch (read at the start,
// written at the end), so no phase waits on a global read.
template <typename real>
__device__ __forceinline__ void nu_row_add(const real (&g)[5], bool have, bool wall_lane, double tw, double& acc)
{
    double ts = 0.0;
    if (have) {
#pragma unroll
        for (int i = 0; i < 5; ++i) ts += double(g[i]);
    }
    const double ts1 = __shfl_down(ts, 1, 64);
    if (wall_lane) acc += 8.0 * tw - 9.0 * ts + ts1;
}

template <typename real, int R, int K, bool REC, bool NU = false>
__device__ __forceinline__ void stepk_tile(const StepArgs<real>& A, real* lds, int tile,
                                           const double* __restrict__ thw_d = nullptr,
                                           double* __restrict__ acc = nullptr)
{
    constexpr int W = kFootW - 2 * (K - 1), HO = R - 2 * (K - 1);
    static_assert(W > 0 && HO > 0, "tile too small for K steps");
    const int tyt = tile / A.tiles_x;
    const int txt = tile - tyt * A.tiles_x;
    const int lx = threadIdx.x;
    const int ly = __builtin_amdgcn_readfirstlane(threadIdx.y);   // blockDim.x = 64: one row per wave
    const int x = txt * W - (K - 1) + lx;
    const int y = tyt * HO - (K - 1) + ly;
    const int n = A.n, P = A.plane, k = y * A.pitch + x;
    const bool inside = x >= 0 && x < n && y >= 0 && y < n;
    const bool own = inside && lx >= K - 1 && lx <= kFootW - K && ly >= K - 1 && ly <= R - K;
    const bool nown = NU && own && x == 0;
    double nacc = 0.0, ntw = 0.0;
    if (nown) {
        nacc = acc[y];
        ntw = thw_d[y];
    }
    real f[9], g[5];
    // phase 1 reads at the node clamped into the cavity on every lane (no
    // global read in a branch); lanes outside compute nothing
    {
        const int xc = min(max(x, 0), n - 1), yc = min(max(y, 0), n - 1);
        gather_cavity_loads<real>(A.fin, A.gin, n, A.pitch, P, xc, yc, f, g);
        if (inside) gather_cavity_walls<real>(thw_row<real>(A.thw, yc), n, x, A.c, g);
    }
    if (inside) {
        real th, ux, uy;
        collide<real>(f, g, A.c, th, ux, uy);
#pragma unroll
        for (int i = 0; i < 9; ++i) lds[(i * R + ly) * kFootW + lx] = f[i];
#pragma unroll
        for (int i = 0; i < 5; ++i) lds[((9 + i) * R + ly) * kFootW + lx] = g[i];
        if (REC && own) store_lp<real>(A.lp, P, k, ux, uy, th);
        if (!REC && !NU && (A.samp_mask & 2) && own) samp_put<real>(A, 1, x, y, g);
    }
    if constexpr (NU) nu_row_add<real>(g, inside, nown, ntw, nacc);
    __syncthreads();
#pragma unroll
    for (int j = 2; j < K; ++j) {
        const bool act = inside && lx >= j - 1 && lx <= kFootW - j && ly >= j - 1 && ly <= R - j;
        real lth = real(0), lux = real(0), luy = real(0);
        if (act) {
            gather_lds<real, R>(lds, A.thw, n, x, y, lx, ly, A.c, f, g);
            collide<real>(f, g, A.c, lth, lux, luy);
        }
        if constexpr (NU) nu_row_add<real>(g, act, nown, ntw, nacc);
        __syncthreads();
        if (act) {
#pragma unroll
            for (int i = 0; i < 9; ++i) lds[(i * R + ly) * kFootW + lx] = f[i];
#pragma unroll
            for (int i = 0; i < 5; ++i) lds[((9 + i) * R + ly) * kFootW + lx] = g[i];
            if (REC && own) store_lp<real>(A.lp + (j - 1) * A.lslot, P, k, lux, luy, lth);
            if (!REC && !NU && (A.samp_mask & (1 << j)) && own) samp_put<real>(A, j, x, y, g);
        }
        __syncthreads();
    }
    if constexpr (NU) {
        // last phase with every lane present for the wavefront shuffle
        if (own) {
            gather_lds<real, R>(lds, A.thw, n, x, y, lx, ly, A.c, f, g);
            real th, ux, uy;
            collide<real>(f, g, A.c, th, ux, uy);
            const unsigned kb = unsigned(k) * sizeof(real), Pb = unsigned(P) * sizeof(real);
#pragma unroll
            for (int i = 0; i < 9; ++i) stb(A.fout, kb + i * Pb, f[i]);
#pragma unroll
            for (int i = 0; i < 5; ++i) stb(A.gout, kb + i * Pb, g[i]);
        }
        nu_row_add<real>(g, own, nown, ntw, nacc);
        if (nown) acc[y] = nacc;
        return;
    }
    if (!own) return;
    if (!REC && (A.samp_mask & (1 << K))) {
        // the last step is a Nusselt sample too
        gather_lds<real, R>(lds, A.thw, n, x, y, lx, ly, A.c, f, g);
        real th, ux, uy;
        collide<real>(f, g, A.c, th, ux, uy);
        const unsigned kb = unsigned(k) * sizeof(real), Pb = unsigned(P) * sizeof(real);
#pragma unroll
        for (int i = 0; i < 9; ++i) stb(A.fout, kb + i * Pb, f[i]);
#pragma unroll
        for (int i = 0; i < 5; ++i) stb(A.gout, kb + i * Pb, g[i]);
        samp_put<real>(A, K, x, y, g);
        return;
    }
    if constexpr (REC) {
        gather_lds<real, R>(lds, A.thw, n, x, y, lx, ly, A.c, f, g);
        real th, ux, uy;
        collide<real>(f, g, A.c, th, ux, uy);
        const unsigned kb = unsigned(k) * sizeof(real), Pb = unsigned(P) * sizeof(real);
#pragma unroll
        for (int i = 0; i < 9; ++i) stb(A.fout, kb + i * Pb, f[i]);
#pragma unroll
        for (int i = 0; i < 5; ++i) stb(A.gout, kb + i * Pb, g[i]);
        store_lp<real>(A.lp + (K - 1) * A.lslot, P, k, ux, uy, th);
        return;
    }
    lds_last_phase<real, R>(lds, A.fout, A.gout, A.thw, n, A.pitch, P, x, y, lx, ly, A.c);
}

template <typename real, int R, int K>
__global__ void __launch_bounds__(kFootW * R) stepk_kernel(StepArgs<real> A)
{
    __shared__ real lds[14 * R * kFootW];
    if (wall_check_blocks(A)) return;
    const int tile = tile_of_block(blockIdx.x, gridDim.x - A.wblocks, A.xcd_remap);
    if (tile >= A.tiles) return;                      // uniform per workgroup
    stepk_tile<real, R, K, false>(A, lds, tile);
}

// K steps per launch that also accumulate the hot-wall Nusselt sums
// (the objective window of the adjoint's forward run).
template <typename real, int R, int K>
__global__ void __launch_bounds__(kFootW * R) stepk_nu_kernel(StepArgs<real> A, const double* __restrict__ thw_d,
                                                              double* __restrict__ acc)
{
    __shared__ real lds[14 * R * kFootW];
    const int tile = tile_of_block(blockIdx.x, gridDim.x, A.xcd_remap);
    if (tile >= A.tiles) return;
    stepk_tile<real, R, K, false, true>(A, lds, tile, thw_d, acc);
}

// K forward steps storing every state (the adjoint's recompute on its own).
template <typename real, int R, int K>
__global__ void __launch_bounds__(kFootW * R) stepk_rec_kernel(StepArgs<real> A)
{
    __shared__ real lds[14 * R * kFootW];
    const int tile = tile_of_block(blockIdx.x, gridDim.x, A.xcd_remap);
    if (tile >= A.tiles) return;
    stepk_tile<real, R, K, true>(A, lds, tile);
}

// ---------------------------------------------------------------------------
// K steps per launch, marching up the rows
// ---------------------------------------------------------------------------
// The workgroup is K groups of B wavefronts; the waves of group j compute
// step t + j.  It owns an x tile of 64 - 2(K - 1) columns (64-wide footprint
// as above) and a chunk of rows [y0, y1) and sweeps it upwards: at
// iteration i, wave r of group j computes row a_j + B i + r, with
// a_1 = y0 - (K - 1) and each group B + 1 rows behind the one before, so
// that the three rows a node gathers from were produced by the previous
// group in an earlier iteration.  Group j < K keeps its newest B + 2 rows in
// an LDS ring that group j + 1 reads; group 1 gathers from global memory and
// group K stores to it.  Odd chunks run the same schedule downwards.  Each
// iteration has a compute stage and a ring-write stage separated by
// barriers.  The rows computed twice are the K - 1 halo rows at each chunk
// end instead of at each 16-row tile, and the result equals K single-step
// launches exactly (same gathers, same arithmetic).

// Gather of node (x, y) from the previous group's ring (14 planes of B + 2
// rows of 64; `ring` points at this lane's column) with the cavity's wall
// rules, rows y - 1, y and y + 1 starting om, o0 and op elements into each
// plane: every interior link from constant offsets, then, when `wall` (a
// uniform flag: the wave has a lane on a side wall or the row is a bottom
// or top row), the wall links of lanes on a wall (as gather_lds).  Every
// read stays inside the ring for any lane, so lanes outside the band's
// output columns may run it too.
template <typename real, int B>
__device__ __forceinline__ void gather_ring(const real* ring, const real* thw, int wallx, int n, int x, int y,
                                            int om, int o0, int op, int o8, const Coef<real>& c, real (&f)[9],
                                            real (&g)[5])
{
    constexpr int PL = (B + 2) * kFootW;
    const real* bm = ring + om;   // row y - 1
    const real* b0 = ring + o0;   // row y
    const real* bp = ring + op;   // row y + 1
    f[0] = b0[0];
    f[1] = b0[1 * PL - 1];
    f[2] = bm[2 * PL];
    f[3] = b0[3 * PL + 1];
    f[4] = bp[4 * PL];
    f[5] = bm[5 * PL - 1];
    f[6] = bm[6 * PL + 1];
    f[7] = bp[7 * PL + 1];
    f[8] = bp[o8];                // o8 = 8 PL - 1, opaque to the compiler (see MarchWave)
    g[0] = b0[9 * PL];
    g[1] = b0[10 * PL - 1];
    g[2] = bm[11 * PL];
    g[3] = b0[12 * PL + 1];
    g[4] = bp[13 * PL];
    // Links that cross a wall take the node's own value of the opposite
    // link (halfway bounce-back; Eq. 45 adds the wall temperature on the
    // left, Eq. 44's adiabatic walls bounce g back).  wallx (bit 0: the
    // band holds the left wall, bit 1: the right one) and the row are
    // uniform per wave, so each wall is a uniform branch; within a side-wall
    // band every lane reads the own-node values together and then selects
    // (one read per lane-dependent branch would wait for each in turn).
    const bool bot = y == 0, top = y == n - 1;
    if (!wallx && !bot && !top) return;
    if (wallx & 1) {                                              // x = 0
        const bool in = x > 0;
        const real r1 = b0[3 * PL], s1 = b0[12 * PL], r5 = b0[7 * PL], r8 = b0[6 * PL];
        const real tw = thw_row<real>(thw, y);
        f[1] = in ? f[1] : r1;
        g[1] = in ? g[1] : fmr(c.cabb, tw, -s1);                  // Eq. 45
        f[5] = in ? f[5] : r5;
        f[8] = in ? f[8] : r8;
    }
    if (wallx & 2) {                                              // x = n - 1
        const bool in = x < n - 1;
        const real r3 = b0[1 * PL], s3 = b0[10 * PL], r6 = b0[8 * PL], r7 = b0[5 * PL];
        f[3] = in ? f[3] : r3;
        g[3] = in ? g[3] : c.cold - s3;                           // Eq. 45
        f[6] = in ? f[6] : r6;
        f[7] = in ? f[7] : r7;
    }
    if (bot) {                                                    // Eq. 44, y = 0
        f[2] = b0[4 * PL];
        g[2] = b0[13 * PL];
        f[5] = b0[7 * PL];
        f[6] = b0[8 * PL];
    }
    if (top) {                                                    // Eq. 44, y = n - 1
        f[4] = b0[2 * PL];
        g[4] = b0[11 * PL];
        f[7] = b0[5 * PL];
        f[8] = b0[6 * PL];
    }
}

// Per-wave constants of the row-marching kernel.  off[] holds per-lane byte
// offsets that stay fixed while the wave marches: for group 1 those of the
// nine links it gathers (march_lane_offsets), for group K those of the nine
// planes it stores (x E + q P E); rows enter as uniform base pointers.
template <typename real>
struct MarchWave {
    int j, x, y0, y1;
    int ydir;            // marching row v stands for cavity row ybase + ydir v
    int vlo, vhi;        // marching rows this group computes: its rows of the chunk, inside the cavity
    int wallx;           // the band holds the left wall (bit 0) or the right one (bit 1)
    int samp;            // a Nusselt sample is due at this group's step
    bool xact;           // the lane's column is one of this group's, inside the cavity
    const real* rin;     // previous group's ring at this lane
    real* rout;          // own ring at this lane
    unsigned off[9];
    // ring offset of link 8 in its source row, 8 (B + 2) 64 - 1, held in a
    // register the compiler cannot see through: with a constant it would
    // pair that read with link 7's (one 64-bit LDS read into adjacent
    // registers) and then copy both values out of the pair every row
    int o8;
    // the force's constant term in a vector register for the whole sweep
    // (its multiply-add also takes gbh from a scalar register, and one
    // instruction reads at most one)
    real gy0h;
};

// Uniform position of a wave in its sweep: marching row v, the cavity row
// y it stands for, and the ring offsets (elements into each plane) of the
// rows y - 1, y and y + 1, advanced by B rows per iteration.
struct MarchPos {
    int v, y, olo, o0, ohi;
};

// Byte offsets of the links a lane at column x (0 <= x < n) gathers in the
// pull-stream of Eq. 25, relative to the start of the source row in plane
// 0: row y for links 0, 1, 3, row y - 1 for 2, 5, 6 and row y + 1 for 4, 7,
// 8.  The left and right walls are folded in: a link that would come from
// outside reads the lane's own node in the opposite plane (halfway
// bounce-back; the Eq. 45 temperature term is added at use), which for
// the diagonals of the wall lanes lies one row up (links 5, 6) or down
// (7, 8) from the source row.  The same offsets serve g (planes 0-4).
template <typename real>
__device__ __forceinline__ void march_lane_offsets(int x, int n, int pitch, int P, unsigned (&o)[9])
{
    constexpr unsigned E = sizeof(real);
    const unsigned xe = unsigned(x) * E, Pb = unsigned(P) * E, rb = unsigned(pitch) * E;
    const bool hxm = x > 0, hxp = x < n - 1;
    o[0] = xe;
    o[1] = hxm ? xe - E + Pb : xe + 3 * Pb;
    o[2] = xe + 2 * Pb;
    o[3] = hxp ? xe + E + 3 * Pb : xe + Pb;
    o[4] = xe + 4 * Pb;
    o[5] = hxm ? xe - E + 5 * Pb : xe + 7 * Pb + rb;
    o[6] = hxp ? xe + E + 6 * Pb : xe + 8 * Pb + rb;
    o[7] = hxp ? xe + E + 7 * Pb : xe + 5 * Pb - rb;
    o[8] = hxm ? xe - E + 8 * Pb : xe + 6 * Pb - rb;
}

// Group 1's gather of row y (0 <= y < n) from global memory with the lane
// offsets above: the row bases are uniform, so the loads need no per-lane
// address arithmetic.  On the bottom and top rows (Eq. 44 walls) the links
// that cross the wall are loaded again from the lane's own node; every
// address stays inside the two planes' rows 0 ... n - 1.
template <typename real>
__device__ __forceinline__ void march_loads(const StepArgs<real>& A, const unsigned (&o)[9], int y,
                                            real (&f)[9], real (&g)[5])
{
    constexpr unsigned E = sizeof(real);
    const int n = A.n;
    const unsigned rb = unsigned(A.pitch) * E;
    const unsigned r0 = unsigned(y) * rb, rm = unsigned(max(y - 1, 0)) * rb, rp = unsigned(min(y + 1, n - 1)) * rb;
    const __amdgpu_buffer_rsrc_t fr = buf_rsrc(A.fin), gr = buf_rsrc(A.gin);
    f[0] = bld<real>(fr, o[0], r0);
    f[1] = bld<real>(fr, o[1], r0);
    f[2] = bld<real>(fr, o[2], rm);
    f[3] = bld<real>(fr, o[3], r0);
    f[4] = bld<real>(fr, o[4], rp);
    f[5] = bld<real>(fr, o[5], rm);
    f[6] = bld<real>(fr, o[6], rm);
    f[7] = bld<real>(fr, o[7], rp);
    f[8] = bld<real>(fr, o[8], rp);
    g[0] = bld<real>(gr, o[0], r0);
    g[1] = bld<real>(gr, o[1], r0);
    g[2] = bld<real>(gr, o[2], rm);
    g[3] = bld<real>(gr, o[3], r0);
    g[4] = bld<real>(gr, o[4], rp);
    if (y == 0 || y == n - 1) {
        // own-node planes: o[0] + q P E
        const unsigned Pb = unsigned(A.plane) * E;
        if (y == 0) {                                  // Eq. 44, bottom
            f[2] = bld<real>(fr, o[4], r0);
            f[5] = bld<real>(fr, o[0], r0 + 7 * Pb);
            f[6] = bld<real>(fr, o[0], r0 + 8 * Pb);
            g[2] = bld<real>(gr, o[4], r0);
        }
        if (y == n - 1) {                              // Eq. 44, top
            f[4] = bld<real>(fr, o[2], r0);
            f[7] = bld<real>(fr, o[0], r0 + 5 * Pb);
            f[8] = bld<real>(fr, o[0], r0 + 6 * Pb);
            g[4] = bld<real>(gr, o[2], r0);
        }
    }
}

// One iteration of the row-marching kernel for the calling wave: group 1
// computes the row gathered into (cf, cg) one iteration earlier and gathers
// the row of its next iteration into (nf, ng) first, so that those global
// loads stay in flight across this iteration's barriers.  The other groups
// gather from the previous group's ring.  Whether the wave computes is
// decided per wave (its row); all its lanes compute, and only the global
// stores and the Nusselt sums are limited to the group's columns.
template <typename real, int K, int B, bool FIRST, bool SAMP, bool PAIRED = false>
__device__ __forceinline__ void march_iter(const StepArgs<real>& A, const MarchWave<real>& w, MarchPos& p,
                                           real (&cf)[9], real (&cg)[5], real (&nf)[9], real (&ng)[5])
{
    constexpr int RS = B + 2, PL = RS * kFootW, RING = 14 * PL;
    const int n = A.n, v = p.v, y = p.y;
    const bool row = v >= w.vlo && v < w.vhi;        // uniform
    if constexpr (FIRST) {
        // unconditional loads of a clamped row: the wait for them is then
        // placed exactly, one iteration later
        march_loads<real>(A, w.off, min(max(y + w.ydir * B, 0), n - 1), nf, ng);
        if (row && w.wallx) gather_cavity_walls<real>(thw_row<real>(A.thw, y), n, w.x, A.c, cg);
    } else if (row) {
        gather_ring<real, B>(w.rin, A.thw, w.wallx, n, w.x, y, p.olo, p.o0, p.ohi, w.o8, A.c, cf, cg);
    }
    if (row) {
        real th, ux, uy;
        Coef<real> c = A.c;
        c.gy0h = w.gy0h;
        collide<real>(cf, cg, c, th, ux, uy);
        // a Nusselt sample due at this group's step: rows of this chunk only
        if (SAMP && w.samp && y >= w.y0 && y < w.y1 && w.xact) samp_put<real>(A, w.j, w.x, y, cg);
    }
    __syncthreads();
    // the same test once more (written differently, so that the compiler
    // does not carry the first one across the barrier as a lane mask)
    if (unsigned(v - w.vlo) < unsigned(w.vhi - w.vlo)) {
        if (FIRST || w.j < K) {
            // the own ring follows the previous group's: the write address
            // is the gather's row-y address plus constants
            real* o = FIRST ? w.rout + p.o0 : const_cast<real*>(w.rin) + p.o0 + RING;
#pragma unroll
            for (int q = 0; q < 9; ++q) o[q * PL] = cf[q];
#pragma unroll
            for (int q = 0; q < 5; ++q) o[(9 + q) * PL] = cg[q];
        } else if (w.xact) {
            const unsigned rs = unsigned(y) * unsigned(A.pitch) * unsigned(sizeof(real));
            const __amdgpu_buffer_rsrc_t fr = buf_rsrc(A.fout), gr = buf_rsrc(A.gout);
#pragma unroll
            for (int q = 0; q < 9; ++q) bst<real>(fr, w.off[q], rs, cf[q]);
#pragma unroll
            for (int q = 0; q < 5; ++q) bst<real>(gr, w.off[q], rs, cg[q]);
        }
    }
    __syncthreads();
    if constexpr (PAIRED) {
        // the caller alternates two positions whose ring slots repeat
        // every two iterations (2B a multiple of B + 2): only the row moves
        p.v = v + 2 * B;
        p.y = y + 2 * w.ydir * B;
    } else {
        // next row: B further, each ring slot B further round the ring
        constexpr int STEP = B * kFootW, WRAP = RS * kFootW;
        p.v = v + B;
        p.y = y + w.ydir * B;
        p.olo = p.olo + STEP >= WRAP ? p.olo + STEP - WRAP : p.olo + STEP;
        p.o0 = p.o0 + STEP >= WRAP ? p.o0 + STEP - WRAP : p.o0 + STEP;
        p.ohi = p.ohi + STEP >= WRAP ? p.ohi + STEP - WRAP : p.ohi + STEP;
    }
}

// One workgroup's sweep: the column band whose footprint starts at column
// x_band (64 lanes, output columns x_band + K - 1 ... x_band + 64 - K) over
// the chunk of rows [y0, y1), marching down the rows when `down`; lds holds
// the K - 1 rings of 14 planes x (B + 2) rows x 64.
template <typename real, int K, int B, bool SAMP = false>
__device__ __forceinline__ void stepm_sweep(const StepArgs<real>& A, real* lds, int x_band, int y0, int y1,
                                            bool down)
{
    constexpr int RS = B + 2, RING = 14 * RS * kFootW;
    MarchWave<real> w;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.y);   // blockDim.x = 64: one wave per y index
    w.j = wv / B + 1;
    const int r = wv - (w.j - 1) * B;
    const int lx = threadIdx.x;
    w.x = x_band + lx;
    const int n = A.n;
    const int a1 = y0 - (K - 1);
    const int aj = a1 - (w.j - 1) * (B + 1);
    const int aK = a1 - (K - 1) * (B + 1);
    const int T = (y1 - 1 - aK) / B + 1;              // iterations until group K has passed y1 - 1
    const int ybase = down ? y0 + y1 - 1 : 0;
    w.ydir = down ? -1 : 1;
    // group j computes the marching rows [y0 - (K - j), y1 + (K - j)) whose
    // cavity rows lie in [0, n)
    w.vlo = max(y0 - (K - w.j), down ? ybase - n + 1 : 0);
    w.vhi = min(y1 + (K - w.j), down ? ybase + 1 : n);
    w.wallx = (x_band <= 0 && x_band + kFootW > 0 ? 1 : 0) | (x_band <= n - 1 && x_band + kFootW > n - 1 ? 2 : 0);
    w.samp = (A.samp_mask >> w.j) & 1;
    w.y0 = y0;
    w.y1 = y1;
    w.xact = w.x >= 0 && w.x < n && lx >= w.j - 1 && lx <= kFootW - w.j;
    w.o8 = 8 * RS * kFootW - 1;
    asm("" : "+v"(w.o8));
    w.gy0h = A.c.gy0h;
    asm("" : "+v"(w.gy0h));
    w.rin = lds + (w.j >= 2 ? (w.j - 2) * RING : 0) + lx;
    w.rout = lds + (w.j < K ? (w.j - 1) * RING : 0) + lx;
    const int xn = min(max(w.x, 0), n - 1);           // lanes outside the cavity gather a clamped column
    if (w.j == 1) {
        march_lane_offsets<real>(xn, n, A.pitch, A.plane, w.off);
    } else {
#pragma unroll
        for (int q = 0; q < 9; ++q) w.off[q] = (unsigned(xn) + unsigned(q) * unsigned(A.plane)) * sizeof(real);
    }
    // first row, and the ring slots of its rows y - 1, y, y + 1 (marching
    // rows v - ydir, v, v + ydir; row v sits in slot (v - aK) mod (B + 2))
    MarchPos p;
    p.v = aj + r;
    p.y = ybase + w.ydir * p.v;
    const int s0 = (p.v - aK) % RS;
    p.o0 = s0 * kFootW;
    p.olo = ((s0 + RS - w.ydir) % RS) * kFootW;
    p.ohi = ((s0 + RS + w.ydir) % RS) * kFootW;
    real af[9], ag[5], bf[9], bg[5];
    if (w.j == 1) march_loads<real>(A, w.off, min(max(p.y, 0), n - 1), af, ag);
    // group 1 and the others run separate loops (the same number of
    // barriers each); two iterations per trip with the roles of the two
    // register sets swapped, so the prefetched values need no copies
    if (w.j == 1) {
        for (int i = 0; i < T; i += 2) {
            march_iter<real, K, B, true, SAMP>(A, w, p, af, ag, bf, bg);
            if (i + 1 < T) march_iter<real, K, B, true, SAMP>(A, w, p, bf, bg, af, ag);
        }
    } else if constexpr ((2 * B) % RS == 0) {
        // two rows per group: the ring slots of a wave repeat every two
        // iterations, so two positions with fixed slots alternate and the
        // ring addresses stay the same from one trip to the next
        MarchPos q = p;
        q.v = p.v + B;
        q.y = p.y + w.ydir * B;
        q.olo = (p.olo + B * kFootW) % (RS * kFootW);
        q.o0 = (p.o0 + B * kFootW) % (RS * kFootW);
        q.ohi = (p.ohi + B * kFootW) % (RS * kFootW);
        for (int i = 0; i < T; i += 2) {
            march_iter<real, K, B, false, SAMP, true>(A, w, p, af, ag, bf, bg);
            if (i + 1 < T) march_iter<real, K, B, false, SAMP, true>(A, w, q, af, ag, bf, bg);
        }
    } else {
        for (int i = 0; i < T; ++i) march_iter<real, K, B, false, SAMP>(A, w, p, af, ag, bf, bg);
    }
}

// Tiles of a marching launch: first the bands without a side wall (1 ...
// tiles_x - 2), chunk rows each, chunk row by chunk row; then the two bands
// that hold the side walls, chunk_w rows each, the left and right band of a
// chunk row in turn (a single band holds both walls).
template <typename real, int K, int B, bool SAMP>
__device__ __forceinline__ void stepm_body(const StepArgs<real>& A, int chunk, int chunk_w)
{
    constexpr int RS = B + 2, W = kFootW - 2 * (K - 1), RING = 14 * RS * kFootW;
    static_assert(K >= 2 && W > 0, "K out of range");
    __shared__ real lds[(K - 1) * RING];
    if (wall_check_blocks(A)) return;
    const int tile = tile_of_block(blockIdx.x, gridDim.x - A.wblocks, A.xcd_remap);
    if (tile >= A.tiles) return;                      // uniform per workgroup
    const int nb = A.tiles_x;
    const int ni = nb > 2 ? (nb - 2) * ((A.n + chunk - 1) / chunk) : 0;
    int txt, tyt, ch;
    if (tile < ni) {
        tyt = tile / (nb - 2);
        txt = 1 + (tile - tyt * (nb - 2));
        ch = chunk;
    } else {
        const int t = tile - ni;
        tyt = nb == 1 ? t : t >> 1;
        txt = nb == 1 ? 0 : ((t & 1) ? nb - 1 : 0);
        ch = chunk_w;
    }
    const int y0 = tyt * ch;
    // odd chunks march down (row y0 + y1 - 1 - v for marching row v), so
    // that two neighbouring chunks read the rows they share at the same
    // time, at the end of both sweeps or at the start of both
    stepm_sweep<real, K, B, SAMP>(A, lds, txt * W - (K - 1), y0, min(y0 + ch, A.n), (tyt & 1) != 0);
}

template <typename real, int K, int B>
__global__ void __launch_bounds__(kFootW * K * B) stepm_kernel(StepArgs<real> A, int chunk, int chunk_w)
{
    stepm_body<real, K, B, false>(A, chunk, chunk_w);
}

// The same with Nusselt samples taken in the launch (samp_mask non-zero).
template <typename real, int K, int B>
__global__ void __launch_bounds__(kFootW * K * B) stepm_samp_kernel(StepArgs<real> A, int chunk, int chunk_w)
{
    stepm_body<real, K, B, true>(A, chunk, chunk_w);
}

// lambda at footprint node (lx, ly) from mu of the previous phase in LDS:
// interior links first (one base address, constant offsets), then the wall
// links of lanes on a wall.
template <typename real, int R>
__device__ __forceinline__ void adj_pull_lds(const real* lds, int n, int x, int y, int lx, int ly,
                                             real sd, real (&lf)[9], real (&lg)[5])
{
    constexpr int W = kFootW, PL = R * kFootW;
    const real* b = lds + (ly * W + lx);
    lf[0] = b[0];
    lf[1] = b[1 * PL + 1];
    lf[2] = b[2 * PL + W];
    lf[3] = b[3 * PL - 1];
    lf[4] = b[4 * PL - W];
    lf[5] = b[5 * PL + W + 1];
    lf[6] = b[6 * PL + W - 1];
    lf[7] = b[7 * PL - W - 1];
    lf[8] = b[8 * PL - W + 1];
    lg[0] = b[9 * PL] + sd;
    lg[1] = b[10 * PL + 1] + sd;
    lg[2] = b[11 * PL + W] + sd;
    lg[3] = b[12 * PL - 1] + sd;
    lg[4] = b[13 * PL - W] + sd;
    const bool hxm = x > 0, hxp = x < n - 1, hym = y > 0, hyp = y < n - 1;
    if (!(hxm && hxp && hym && hyp)) {
        // a lane on a wall: the own-node values read together, then selected
        // (a read per branch would make the wave wait for each in turn)
        const real r1 = b[3 * PL], s1 = b[12 * PL], r3 = b[1 * PL], s3 = b[10 * PL];
        const real r2 = b[4 * PL], s2 = b[13 * PL], r4 = b[2 * PL], s4 = b[11 * PL];
        const real r5 = b[7 * PL], r6 = b[8 * PL], r7 = b[5 * PL], r8 = b[6 * PL];
        lf[1] = hxp ? lf[1] : r1;
        lg[1] = hxp ? lg[1] : sd - s1;                                 // Eq. 45, right wall
        lf[3] = hxm ? lf[3] : r3;
        lg[3] = hxm ? lg[3] : sd - s3;                                 // Eq. 45, left wall
        lf[2] = hyp ? lf[2] : r2;
        lg[2] = hyp ? lg[2] : s2 + sd;                                 // Eq. 44
        lf[4] = hym ? lf[4] : r4;
        lg[4] = hym ? lg[4] : s4 + sd;
        lf[5] = hxp && hyp ? lf[5] : r5;
        lf[6] = hxm && hyp ? lf[6] : r6;
        lf[7] = hxm && hym ? lf[7] : r7;
        lf[8] = hxp && hym ? lf[8] : r8;
    }
}

// K adjoint steps per launch (m = *n0p + j down to m - K + 1): the mirror
// image of stepk_tile.  Phase 1 pulls mu(m+1) from HBM on the footprint and
// forms mu(m) into LDS; phase i pulls mu(m-i+2) from LDS on the footprint
// shrunk by i - 1 nodes per side and forms mu(m-i+1), linearised at the
// point stored in segment slot j - i (HBM); the last phase stores mu(m-K+1)
// on the output tile.  Only output-tile nodes add to dJ/dtheta_w, in the same
// order as single steps, so the result equals K single-step launches.
template <typename real, int R, int K>
__device__ __forceinline__ void adjk_tile(const AdjArgs<real>& A, real* lds, int tile)
{
    constexpr int W = kFootW - 2 * (K - 1), HO = R - 2 * (K - 1);
    static_assert(W > 0 && HO > 0, "tile too small for K steps");
    const int tyt = tile / A.tiles_x;
    const int txt = tile - tyt * A.tiles_x;
    const int lx = threadIdx.x;
    const int ly = __builtin_amdgcn_readfirstlane(threadIdx.y);   // blockDim.x = 64: one row per wave
    const int x = txt * W - (K - 1) + lx;
    const int y = tyt * HO - (K - 1) + ly;
    const int n = A.n, P = A.plane;
    const bool inside = x >= 0 && x < n && y >= 0 && y < n;
    const bool own = inside && lx >= K - 1 && lx <= kFootW - K && ly >= K - 1 && ly <= R - K;
    // dJ/dtheta_w of row y: the owning lane at x = 0 keeps it in a register
    // for the whole launch (same fma sequence as single steps)
    const bool gown = own && x == 0;
    double gacc = 0.0;
    if (gown) gacc = A.gthw[y];
    // the segment's first step index through the constant address space (a
    // scalar load that does not wait for the vector loads in flight)
    const int m = ((const __attribute__((address_space(4))) int*)A.n0p)[0] + A.j;
    // every global read below is unconditional, at the node clamped into
    // the cavity (values of lanes outside are never used), so no read sits
    // in a branch and the reads of the next phase stay in flight while the
    // current one computes
    const int xc = min(max(x, 0), n - 1), yc = min(max(y, 0), n - 1);
    const int kc = yc * A.pitch + xc;
    real lf[9], lg[5];
    // linearisation points: this phase's (cu, cv, ct) and the next one's
    // (su, sv, st), one read of each plane at the node itself
    real cu = A.lp[kc], cv = A.lp[P + kc], ct = A.lp[2 * P + kc];
    real su = real(0), sv = real(0), st = real(0);
    adj_pull<real>(A.lin, n, A.pitch, P, xc, yc, adj_seed_at<real>(x, m >= A.win_start, A.seed0, A.seed1),
                   lf, lg);
    if (K >= 2) {
        const real* q = A.lp - A.lslot;
        su = q[kc]; sv = q[P + kc]; st = q[2 * P + kc];
    }
    if (inside) {
        collide_vjp_at<real>(cu, cv, ct, A.c, lf, lg);
        if (gown) gacc = __builtin_fma(A.cabb, double(lg[1]), gacc);
#pragma unroll
        for (int i = 0; i < 9; ++i) lds[(i * R + ly) * kFootW + lx] = lf[i];
#pragma unroll
        for (int i = 0; i < 5; ++i) lds[((9 + i) * R + ly) * kFootW + lx] = lg[i];
    }
    __syncthreads();
#pragma unroll
    for (int j = 2; j <= K; ++j) {
        const bool act = inside && lx >= j - 1 && lx <= kFootW - j && ly >= j - 1 && ly <= R - j;
        cu = su; cv = sv; ct = st;
        if (j < K) {
            const real* q = A.lp - j * A.lslot;
            su = q[kc]; sv = q[P + kc]; st = q[2 * P + kc];
        }
        if (act) {
            const int mj = m - j + 1;
            adj_pull_lds<real, R>(lds, n, x, y, lx, ly,
                                  adj_seed_at<real>(x, mj >= A.win_start, A.seed0, A.seed1), lf, lg);
            collide_vjp_at<real>(cu, cv, ct, A.c, lf, lg);
            if (gown) gacc = __builtin_fma(A.cabb, double(lg[1]), gacc);
        }
        if (j == K) break;
        __syncthreads();
        if (act) {
#pragma unroll
            for (int i = 0; i < 9; ++i) lds[(i * R + ly) * kFootW + lx] = lf[i];
#pragma unroll
            for (int i = 0; i < 5; ++i) lds[((9 + i) * R + ly) * kFootW + lx] = lg[i];
        }
        __syncthreads();
    }
    if (!own) return;
    if (gown) A.gthw[y] = gacc;
    const unsigned kb = unsigned(y * A.pitch + x) * sizeof(real), Pb = unsigned(P) * sizeof(real);
#pragma unroll
    for (int i = 0; i < 9; ++i) stb(A.lout, kb + i * Pb, lf[i]);
#pragma unroll
    for (int i = 0; i < 5; ++i) stb(A.lout, kb + (9 + i) * Pb, lg[i]);
}

template <typename real, int R, int K>
__global__ void __launch_bounds__(kFootW * R) adjk_kernel(AdjArgs<real> A)
{
    __shared__ real lds[14 * R * kFootW];
    const int tile = tile_of_block(blockIdx.x, gridDim.x, A.xcd_remap);
    if (tile >= A.tiles) return;
    adjk_tile<real, R, K>(A, lds, tile);
}

// K adjoint steps of the current segment and K recompute steps of the
// next-older one (every state stored) in one launch: workgroups
// [0, A.tiles) take adjoint tiles, the rest forward tiles.
template <typename real, int R, int K>
__global__ void __launch_bounds__(kFootW * R) adjk_fused_kernel(AdjArgs<real> A, StepArgs<real> F)
{
    __shared__ real lds[14 * R * kFootW];
    const int b = blockIdx.x;
    if (b < A.tiles) {
        adjk_tile<real, R, K>(A, lds, b);
        return;
    }
    if (b - A.tiles >= F.tiles) return;
    stepk_tile<real, R, K, true>(F, lds, b - A.tiles);
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
    collide<real, true>(f, g, c, a, b, d);
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

// Hot-wall Nusselt samples from the temperature sums that K-step launches
// wrote into nslots consecutive slots, appended to the ring in slot order:
// per slot the arithmetic and reduction of nusselt_block, so each sample
// equals what nusselt_kernel gives after single steps.
static __global__ void __launch_bounds__(256) nusselt_slots_kernel(
    const double* __restrict__ t, int nslots, int n, const double* __restrict__ thw, double H,
    double inv_dT, double* __restrict__ ring, unsigned long long* __restrict__ ring_count, long ring_cap)
{
    __shared__ double part[4];
    unsigned long long c = 0;
    if (threadIdx.x == 0) c = *ring_count;
    for (int sl = 0; sl < nslots; ++sl) {
        const double* ts = t + (size_t)sl * 2 * n;
        double acc = 0.0;
        for (int y = threadIdx.x; y < n; y += blockDim.x) {
            const double t0 = ts[2 * y], t1 = ts[2 * y + 1];
            const double slope_in = (9.0 * t0 - t1 - 8.0 * thw[y]) * (1.0 / 3.0);
            acc += -slope_in * H * inv_dT;
        }
        acc = wave_sum(acc);
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        if (lane == 0) part[wid] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double sum = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += part[w];
            ring[c % (unsigned long long)ring_cap] = sum / n;
            ++c;
        }
        __syncthreads();                              // part is reused by the next slot
    }
    if (threadIdx.x == 0) *ring_count = c;
}

// K steps per launch for the batch: tiles are footprints (origin K - 1 nodes
// left of and below the output tile) of one member each; phases as in
// stepk_kernel, with two barriers per tile around the LDS reuse.
template <typename real, int R, int K>
__global__ void __launch_bounds__(kFootW * R) batch_stepk_kernel(
    const CavityDev<real>* __restrict__ cavs, const TileRef* __restrict__ tiles, int t_begin,
    int t_end, int cur)
{
    __shared__ real lds[14 * R * kFootW];
    const int lx = threadIdx.x;
    const int ly = __builtin_amdgcn_readfirstlane(threadIdx.y);   // blockDim.x = 64: one row per wave
    for (int t = t_begin + blockIdx.x; t < t_end; t += gridDim.x) {
        const TileRef tr = tiles[t];
        const CavityDev<real>& cv = cavs[tr.cav];
        if (cv.dead) continue;                        // uniform per workgroup
        const int x = tr.x0 + lx, y = tr.y0 + ly, n = cv.n;
        const bool inside = x >= 0 && x < n && y >= 0 && y < n;
        lds_first_phase<real, R>(lds, cv.f[cur], cv.g[cur], cv.thw, n, cv.pitch, cv.plane, x, y, lx, ly, inside,
                                 cv.c);
        __syncthreads();
        real f[9], g[5];
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = real(0);
#pragma unroll
        for (int i = 0; i < 5; ++i) g[i] = real(0);
#pragma unroll
        for (int j = 2; j < K; ++j) {
            const bool act = inside && lx >= j - 1 && lx <= kFootW - j && ly >= j - 1 && ly <= R - j;
            if (act) {
                gather_lds<real, R>(lds, cv.thw, n, x, y, lx, ly, cv.c, f, g);
                real th, ux, uy;
                collide<real>(f, g, cv.c, th, ux, uy);
            }
            __syncthreads();
            if (act) {
#pragma unroll
                for (int i = 0; i < 9; ++i) lds[(i * R + ly) * kFootW + lx] = f[i];
#pragma unroll
                for (int i = 0; i < 5; ++i) lds[((9 + i) * R + ly) * kFootW + lx] = g[i];
            }
            __syncthreads();
        }
        if (inside && lx >= K - 1 && lx <= kFootW - K && ly >= K - 1 && ly <= R - K)
            lds_last_phase<real, R>(lds, cv.f[cur ^ 1], cv.g[cur ^ 1], cv.thw, n, cv.pitch, cv.plane, x, y,
                               lx, ly, cv.c);
        __syncthreads();                              // the next tile reuses the LDS
    }
}

// One entry per workgroup of the batched row-marching kernel: cavity, first
// footprint column of the band, and the chunk's rows [y0, y1) with the
// marching direction in bit 30 of y1d (cav < 0: an unused slot of the
// die-aware table).
struct MarchRef {
    int cav, x0, y0, y1d;
};

// K steps of many cavities in one launch with the row-marching sweep: each
// workgroup takes one (cavity, band, chunk) entry and runs the same sweep
// as stepm_kernel on that cavity, so every member evolves bitwise as it
// would alone.  All cavities step from copy `cur` to `cur ^ 1`.
template <typename real, int K, int B>
__global__ void __launch_bounds__(kFootW * K * B) batch_stepm_kernel(const CavityDev<real>* __restrict__ cavs,
                                                                     const MarchRef* __restrict__ tiles,
                                                                     int t_begin, int t_end, int cur)
{
    constexpr int RS = B + 2, W = kFootW - 2 * (K - 1), RING = 14 * RS * kFootW;
    static_assert(K >= 2 && W > 0, "K out of range");
    __shared__ real lds[(K - 1) * RING];
    const int t = t_begin + (int)blockIdx.x;
    if (t >= t_end) return;
    const MarchRef tr = tiles[t];
    if (tr.cav < 0) return;                           // uniform per workgroup
    const CavityDev<real>& cv = cavs[tr.cav];
    if (cv.dead) return;
    StepArgs<real> A;
    A.fin = cv.f[cur];
    A.gin = cv.g[cur];
    A.fout = cv.f[cur ^ 1];
    A.gout = cv.g[cur ^ 1];
    A.thw = cv.thw;
    A.n = cv.n;
    A.pitch = cv.pitch;
    A.plane = cv.plane;
    A.c = cv.c;
    stepm_sweep<real, K, B>(A, lds, tr.x0, tr.y0, tr.y1d & 0x3fffffff, ((tr.y1d >> 30) & 1) != 0);
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

// The watchdog of wall_check_blocks as a launch of its own (for a state no
// stepping launch reads next): one thread per wall node, a grid of
// ceil(2n / 256) workgroups; sets *flag (pinned host memory) when a wall
// node holds a non-finite value.
template <typename real>
__global__ void __launch_bounds__(256) wall_check_kernel(const real* __restrict__ fs,
                                                         const real* __restrict__ gs, int n, int pitch,
                                                         int plane, int* __restrict__ flag)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    int bad = t < 2 * n ? wall_node_bad(fs, gs, n, pitch, plane, t) : 0;
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0 && bad) *flag = 1;
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
