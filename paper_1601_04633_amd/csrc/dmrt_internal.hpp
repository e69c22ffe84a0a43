// dmrt_internal.hpp -- host helpers shared by the translation units of libdmrt.
#pragma once

#include <hip/hip_runtime.h>

#include "dmrt.h"
#include "dmrt_device.hpp"

namespace dmrt {

// Records the HIP error text for dmrt_last_error() and maps it to a code.
int record_hip(hipError_t e, const char* what);

// Parameter map of dmrt_derive (Eq. 9, Eqs. 11-13, 32, 38-43).
int derive(const dmrt_params* p, dmrt_derived* d);

// Row pitch in elements: n rounded up to a multiple of 64.
int pitch_of(int n);

inline size_t elem_size(int precision) { return precision == DMRT_FP64 ? sizeof(double) : sizeof(float); }

// Kernel coefficients in the compute precision.
template <typename real>
Coef<real> make_coef(const dmrt_params& p, const dmrt_derived& d)
{
    Coef<real> c;
    c.s_nu = real(d.s_nu); c.s_q = real(d.s_q);
    c.sk = real(d.sigma_k); c.se = real(d.sigma_e); c.sn = real(d.sigma_nu);
    c.a = real(d.a);
    c.cabb = real((4.0 + d.a) / 10.0);
    c.gbeta = real(d.gbeta);
    c.gy0 = real(-d.gbeta * p.theta_ref);
    c.gx = real(p.force_x);
    c.cold = real((4.0 + d.a) / 10.0 * p.theta_cold);
    c.nsn36 = real(-d.s_nu / 36.0); c.nsn4 = real(-d.s_nu / 4.0); c.nsq12 = real(-d.s_q / 12.0);
    c.nsn12 = real(-d.s_nu / 12.0);
    c.nsk2 = real(-d.sigma_k / 2.0); c.nse20 = real(-d.sigma_e / 20.0); c.nsg4 = real(-d.sigma_nu / 4.0);
    c.gbh = real(d.gbeta) * real(0.5); c.gy0h = c.gy0 * real(0.5); c.gxh = c.gx * real(0.5);
    return c;
}

// Thread-local text of the last HIP error.
void set_last_error(const char* msg);

struct AdjointState;          // dmrt_adjoint.hip
void free_adjoint(AdjointState* a);
// Marks the stored forward run as no longer matching the handle (its hot
// wall, initial field or state changed): the next backward is refused.
void invalidate_adjoint(AdjointState* a);

}  // namespace dmrt

#include <algorithm>
#include <vector>

struct dmrt_cavity {
    dmrt_params p;
    dmrt_derived d;
    int dev = 0;
    int n = 0, pitch = 0, plane = 0;
    size_t esz = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap_stream = nullptr;
    void* fbuf = nullptr;     // [2][9][plane]
    void* gbuf = nullptr;     // [2][5][plane]
    bool own_bufs = false;
    int cur = 0;              // copy holding the current state
    long step = 0;
    // hot wall
    void* thw_real = nullptr;         // n reals
    double* thw_dbl = nullptr;        // n doubles
    std::vector<double> thw_host;
    // diagnostics scratch
    double* scratch = nullptr;        // fields upload / download, 4 n^2 doubles
    double* nu_buf = nullptr;         // n + 1 doubles
    double* res_ref = nullptr;        // 3 n^2 doubles
    double* res_part = nullptr;       // residual partials
    int res_blocks = 0;
    double* ring = nullptr;
    double* samp = nullptr;           // Nusselt sample sums of K-step launches, kSampSlots x 2 n doubles
    unsigned long long* ring_count = nullptr;
    long ring_cap = 0;
    int series_stride = 0;
    // launch
    int block_x = 256, block_y = 1, xcd_remap = 1, graph_steps = 60;   // 60: a multiple of every K
    int temporal = 1, t_rows = 10;    // steps per launch (1, or 2..4 through LDS) and its tile rows
    int march = 0, march_chunk = 0;   // K-step launches marching up the rows: wave rows per step
                                      // group (0: off) and rows per workgroup
    // marching launches of fewer steps that end a count which is not a
    // multiple of K: wave rows per group (0: none) and chunk rows, by steps
    int march_rem_B[8] = {}, march_rem_chunk[8] = {};   // indexed by steps, up to kMaxK
    // chunk rows of the two bands that hold the side walls (shorter where
    // the chunk is chosen automatically: their rows cost more)
    int march_chunk_w = 0, march_rem_chunk_w[8] = {};
    int adj_temporal = 1, adj_rows = 10;   // the same for the adjoint's backward launches
    int graph_flips[2] = {0, 0};      // copy changes made by one replay of graph[p]
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    hipGraph_t graph_def[2] = {nullptr, nullptr};
    // initial temperature of the last dmrt_set_theta (gradient problem)
    double* theta0 = nullptr;         // n^2 doubles
    bool theta0_valid = false;
    // set by the watchdog after it found a non-finite value in a wall
    // column (pinned host memory, written by the device)
    volatile int* nonfinite = nullptr;
    // the next stepping launch runs the watchdog on its input (extra
    // workgroups; set for the first launch of a dmrt_step call)
    bool wcheck = false;
    // steps enqueued since the last watchdog pass (dmrt_sync runs one)
    bool unchecked = false;
    dmrt::AdjointState* adj = nullptr;
    long adj_gen = 0;                 // successful dmrt_adjoint_forward calls
};


#define DMRT_HIPCHK(expr)                                          \
    do {                                                           \
        hipError_t e_ = (expr);                                    \
        if (e_ != hipSuccess) return ::dmrt::record_hip(e_, #expr); \
    } while (0)

namespace dmrt {

// Valid (steps per launch, footprint rows) pairs of stepk_kernel.
// The (steps per launch K, footprint rows R) pairs the K-step kernels are
// built for; every launcher instantiates its kernels over this one list.
#define DMRT_FOR_EACH_KR(X)                                                     \
    X(2, 4) X(2, 6) X(2, 10) X(2, 16)                                          \
    X(3, 6) X(3, 10) X(3, 12) X(3, 14) X(3, 16)                                \
    X(4, 10) X(4, 12) X(4, 14) X(4, 16)

inline bool valid_temporal(int k, int rows)
{
    if (k == 1) return rows == 4 || rows == 6 || rows == 10 || rows == 16;
#define DMRT_KR_OK(KK, RR) if (k == KK && rows == RR) return true;
    DMRT_FOR_EACH_KR(DMRT_KR_OK)
#undef DMRT_KR_OK
    return false;
}

// The (steps per launch K, wave rows per step group B) pairs of the
// row-marching K-step kernel (K B wavefronts per workgroup); a pair exists
// for a precision when its LDS rings fit a workgroup's 160 KB.
#define DMRT_FOR_EACH_KB(X) X(2, 8) X(3, 2) X(3, 4) X(4, 1) X(4, 2) X(4, 3) X(4, 4) X(6, 2)

constexpr long kLdsBytes = 160 * 1024;
constexpr int kMaxK = 6;           // most steps per launch of any K-step form
static_assert(kMaxK < 8, "dmrt_cavity::march_rem_B holds steps up to 7");
constexpr int kSampSlots = 32;     // Nusselt sample slots reduced by one kernel (>= kMaxK)

constexpr long march_lds_bytes(int k, int b, int esz)
{
    return long(k - 1) * 14 * (b + 2) * kFootW * esz;
}

inline bool valid_march(int k, int b, int esz)
{
#define DMRT_KB_OK(KK, BB) if (k == KK && b == BB) return march_lds_bytes(k, b, esz) <= kLdsBytes;
    DMRT_FOR_EACH_KB(DMRT_KB_OK)
#undef DMRT_KB_OK
    return false;
}

// A row of a band that holds a side wall costs this much more than an
// interior row (the wall links' own-node reads and selects, the wall
// temperature; measured at 1024^2 with six steps per launch).
constexpr double kWallRowCost = 1.08;

// Rows per workgroup of the row-marching kernel that leave every workgroup
// of one launch resident at once (at least 1 row), and in *chunk_w those of
// the two side-wall bands: shorter, so that their workgroups take about as
// long as the others (a sweep of c rows takes c plus 2(K - 1) halo and
// (K - 1)(B + 1) pipeline rows), as far as the resident slots allow.
template <typename real>
int march_chunk_auto(int n, int K, int B, int dev, int* chunk_w = nullptr)
{
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return -1;
#define DMRT_KB_OCC(KK, BB)                                                                      \
    if constexpr (march_lds_bytes(KK, BB, sizeof(real)) <= kLdsBytes)                             \
        if (K == KK && B == BB &&                                                                \
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stepm_kernel<real, KK, BB>,     \
                                                         kFootW * KK * BB, 0) != hipSuccess)      \
            return -1;
    DMRT_FOR_EACH_KB(DMRT_KB_OCC)
#undef DMRT_KB_OCC
    if (per_cu <= 0) return -1;
    const int W = kFootW - 2 * (K - 1);
    const int tiles_x = (n + W - 1) / W;
    const int slots = per_cu * cus;
    const int chunks = std::max(1, slots / tiles_x);
    const int chunk = std::max(1, (n + chunks - 1) / chunks);
    if (chunk_w) {
        int cw = chunk;
        if (tiles_x >= 3) {
            const int L = 2 * (K - 1) + (K - 1) * (B + 1);
            cw = std::max(1, std::min(chunk, int((chunk + L) / kWallRowCost - L + 0.5)));
            const long ni = long(tiles_x - 2) * ((n + chunk - 1) / chunk);
            while (cw < chunk && ni + 2L * ((n + cw - 1) / cw) > slots) ++cw;
        }
        *chunk_w = cw;
    }
    return chunk;
}

// Workgroups to append to a stepping launch of `threads` threads per
// workgroup so that it also runs the watchdog on its input (h->wcheck set;
// the launch's kernel calls wall_check_blocks), else 0.
template <typename real>
int add_wall_check(const dmrt_cavity* h, StepArgs<real>& A, int threads)
{
    if (!h->wcheck) return 0;
    A.wflag = const_cast<int*>(h->nonfinite);
    A.wblocks = (2 * h->n + threads - 1) / threads;
    return A.wblocks;
}

// Launches K = h->temporal steps of the cavity with the row-marching kernel
// (h->march wave rows per step group, h->march_chunk rows per workgroup),
// or k < K steps in the shape of h->march_rem_B[k] and h->march_rem_chunk[k].
template <typename real>
int launch_stepm(const dmrt_cavity* h, hipStream_t s, const real* fin, const real* gin, real* fout,
                 real* gout, double* samp = nullptr, int samp_mask = 0, int k = 0)
{
    const bool rem = k > 0 && k != h->temporal;
    const int K = rem ? k : h->temporal, B = rem ? h->march_rem_B[k] : h->march;
    const int chunk = rem ? h->march_rem_chunk[k] : h->march_chunk;
    const int chunk_w = rem ? h->march_rem_chunk_w[k] : h->march_chunk_w;
    StepArgs<real> A;
    A.fin = fin; A.gin = gin; A.fout = fout; A.gout = gout;
    A.samp = samp; A.samp_mask = samp_mask;
    A.thw = static_cast<const real*>(h->thw_real);
    A.n = h->n; A.pitch = h->pitch; A.plane = h->plane;
    const int W = kFootW - 2 * (K - 1);
    A.tiles_x = (h->n + W - 1) / W;
    // the bands without a side wall, then the one or two that hold them
    // (stepm_body's order)
    const int nb = A.tiles_x, nw = std::min(nb, 2);
    A.tiles = (nb - nw) * ((h->n + chunk - 1) / chunk) + nw * ((h->n + chunk_w - 1) / chunk_w);
    A.xcd_remap = h->xcd_remap;
    A.c = make_coef<real>(h->p, h->d);
    int nblocks = A.tiles;
    if (h->xcd_remap) nblocks = (nblocks + 7) / 8 * 8;
    nblocks += add_wall_check(h, A, kFootW * K * B);
    const dim3 grid(nblocks), block(kFootW, K * B);
#define DMRT_KB(KK, BB)                                                                  \
    if constexpr (march_lds_bytes(KK, BB, sizeof(real)) <= kLdsBytes)                     \
        if (K == KK && B == BB) {                                                         \
            if (samp_mask)                                                                \
                hipLaunchKernelGGL((stepm_samp_kernel<real, KK, BB>), grid, block, 0, s, A, chunk, \
                                   chunk_w);                                              \
            else                                                                          \
                hipLaunchKernelGGL((stepm_kernel<real, KK, BB>), grid, block, 0, s, A, chunk,  \
                                   chunk_w);                                              \
            return record_hip(hipGetLastError(), "stepm_kernel");                        \
        }
    DMRT_FOR_EACH_KB(DMRT_KB)
#undef DMRT_KB
    return DMRT_EINVAL;
}

// Launches K = h->temporal steps of the cavity from (fin, gin) to (fout, gout)
// through LDS with footprint rows h->t_rows (K >= 2).  With acc non-null the
// launch also adds each step's hot-wall Nusselt row sums to acc (FP64, n
// entries; thw_d the FP64 wall temperatures).  samp_mask bit j (1 <= j <= K):
// the launch writes the wall-column temperature sums of step t + j to the
// slot (set bits below j) of samp, 2 n doubles each (see StepArgs).
template <typename real>
int launch_stepk(const dmrt_cavity* h, hipStream_t s, const real* fin, const real* gin, real* fout,
                 real* gout, const double* thw_d = nullptr, double* acc = nullptr,
                 double* samp = nullptr, int samp_mask = 0)
{
    if (h->march && !acc) return launch_stepm<real>(h, s, fin, gin, fout, gout, samp, samp_mask);
    const int K = h->temporal, R = h->t_rows;
    StepArgs<real> A;
    A.fin = fin; A.gin = gin; A.fout = fout; A.gout = gout;
    A.samp = samp; A.samp_mask = samp_mask;
    A.thw = static_cast<const real*>(h->thw_real);
    A.n = h->n; A.pitch = h->pitch; A.plane = h->plane;
    const int W = kFootW - 2 * (K - 1), HO = R - 2 * (K - 1);
    A.tiles_x = (h->n + W - 1) / W;
    A.tiles = A.tiles_x * ((h->n + HO - 1) / HO);
    A.xcd_remap = h->xcd_remap;
    A.c = make_coef<real>(h->p, h->d);
    int nblocks = A.tiles;
    if (h->xcd_remap) nblocks = (nblocks + 7) / 8 * 8;
    if (!acc) nblocks += add_wall_check(h, A, kFootW * R);   // stepk_kernel only
    const dim3 grid(nblocks), block(kFootW, R);
#define DMRT_KR(KK, RR)                                                                   \
    if (K == KK && R == RR) {                                                              \
        if (acc) {                                                                         \
            hipLaunchKernelGGL((stepk_nu_kernel<real, RR, KK>), grid, block, 0, s, A, thw_d, acc); \
            return record_hip(hipGetLastError(), "stepk_nu_kernel");                      \
        }                                                                                  \
        hipLaunchKernelGGL((stepk_kernel<real, RR, KK>), grid, block, 0, s, A);            \
        return record_hip(hipGetLastError(), "stepk_kernel");                             \
    }
    DMRT_FOR_EACH_KR(DMRT_KR)
#undef DMRT_KR
    return DMRT_EINVAL;
}

}  // namespace dmrt
