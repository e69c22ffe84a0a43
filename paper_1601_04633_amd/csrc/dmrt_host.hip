// dmrt_host.hip -- host side of libdmrt: the C ABI declared in include/dmrt.h.
//
// Owns parameters, device buffers, the stream, the captured step graphs and
// the diagnostics scratch of one cavity.  Every entry point returns an error
// code; HIP failures are recorded per thread for dmrt_last_error().
#include "dmrt.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dmrt_device.hpp"
#include "dmrt_internal.hpp"

namespace {

thread_local std::string g_last_error;

}  // namespace

namespace dmrt {

void set_last_error(const char* msg) { g_last_error = msg; }

int record_hip(hipError_t e, const char* what)
{
    if (e == hipSuccess) return DMRT_OK;
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
    g_last_error = buf;
    if (e == hipErrorOutOfMemory) return DMRT_ENOMEM;
    if (e == hipErrorNoDevice || e == hipErrorInvalidDevice) return DMRT_ENODEV;
    return DMRT_EHIP;
}

// Parameter map (Eq. 9 with Eqs. 11-13; Eq. 32; Eqs. 38-43).
int derive(const dmrt_params* p, dmrt_derived* d)
{
    if (!p || !d) return DMRT_EINVAL;
    if (p->n < 4 || p->n > 32768) return DMRT_EINVAL;
    const double vals[] = {p->Ra, p->Pr, p->Ma, p->theta_hot, p->theta_cold, p->force_x,
                           p->theta_ref};
    for (double v : vals)
        if (!std::isfinite(v)) return DMRT_EINVAL;
    if (p->precision != DMRT_FP32 && p->precision != DMRT_FP64) return DMRT_EINVAL;
    // kernels address a 14-plane state with 32-bit byte offsets
    const double esz = p->precision == DMRT_FP64 ? 8.0 : 4.0;
    if (14.0 * esz * (double)((p->n + 63) / 64 * 64) * p->n >= 4294967296.0) return DMRT_EINVAL;
    if (p->bc_mode < DMRT_BC_CAVITY || p->bc_mode > DMRT_BC_ADIABATIC_BOX) return DMRT_EINVAL;
    if (p->bc_mode == DMRT_BC_CAVITY && p->force_x != 0.0) return DMRT_EINVAL;   // G = (0, G_y)
    if (p->collision != DMRT_COLL_MRT && p->collision != DMRT_COLL_LBGK) return DMRT_EINVAL;
    if (!(p->Ra > 0.0) || !(p->Pr > 0.0) || !(p->Ma > 0.0)) return DMRT_EUNSTABLE;
    const double H = p->n;
    const double dT = p->theta_hot - p->theta_cold;
    double gbeta;
    if (std::isnan(p->gbeta_override)) {
        if (!(dT > 0.0)) return DMRT_EINVAL;
        // u_c^2 = g beta dT H = Ma^2 c_s^2
        gbeta = p->Ma * p->Ma / (3.0 * H * dT);
    } else {
        if (!std::isfinite(p->gbeta_override)) return DMRT_EINVAL;
        gbeta = p->gbeta_override;
    }
    const double nu = p->Ma * H * std::sqrt(p->Pr / (3.0 * p->Ra));
    const double alpha = nu / p->Pr;
    const double s_nu = 2.0 / (6.0 * nu + 1.0);
    double s_q = 8.0 * (2.0 - s_nu) / (8.0 - s_nu);
    double a, sk, se;
    if (p->q5_mode == DMRT_Q5_PAPER) {
        const double lk = std::sqrt(3.0) / 6.0;       // Eq. 40
        sk = 1.0 / (0.5 + lk);
        se = 1.0 / (0.5 + std::sqrt(3.0) / 3.0);
        a = 10.0 * alpha / lk - 4.0;                   // Eq. 43 solved for a
    } else if (p->q5_mode == DMRT_Q5_FIXED_A) {
        if (!std::isfinite(p->a)) return DMRT_EINVAL;
        a = p->a;
        if (!(a > -4.0)) return DMRT_EUNSTABLE;
        const double lk = 10.0 * alpha / (4.0 + a);   // Eq. 43 solved for sigma_k
        sk = 1.0 / (0.5 + lk);
        se = 1.0 / (0.5 + 1.0 / (6.0 * lk));           // Eq. 39
    } else {
        return DMRT_EINVAL;
    }
    if (p->collision == DMRT_COLL_LBGK) {
        // one rate per distribution: BGK written in moment space
        s_q = s_nu;
        se = sk;
    }
    if (!(a > -4.0 && a < 1.0)) return DMRT_EUNSTABLE;
    const double rates[] = {s_nu, s_q, sk, se};
    for (double r : rates)
        if (!(r > 0.0 && r < 2.0)) return DMRT_EUNSTABLE;
    d->nu = nu; d->alpha = alpha; d->gbeta = gbeta;
    d->s_nu = s_nu; d->s_q = s_q;
    d->sigma_k = sk; d->sigma_e = se; d->sigma_nu = se;
    d->a = a; d->w0 = (1.0 - a) / 5.0; d->wm = (4.0 + a) / 20.0; d->H = H;
    return DMRT_OK;
}

int pitch_of(int n) { return (n + 63) / 64 * 64; }

}  // namespace dmrt

using namespace dmrt;

#define HIPCHK(expr) DMRT_HIPCHK(expr)

namespace {

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

namespace {

void drop_graphs(dmrt_cavity* h)
{
    for (int i = 0; i < 2; ++i) {
        if (h->graph[i]) (void)hipGraphExecDestroy(h->graph[i]);
        if (h->graph_def[i]) (void)hipGraphDestroy(h->graph_def[i]);
        h->graph[i] = nullptr;
        h->graph_def[i] = nullptr;
    }
}

template <typename real>
real* fptr(dmrt_cavity* h, int copy) { return static_cast<real*>(h->fbuf) + (size_t)copy * 9 * h->plane; }
template <typename real>
real* gptr(dmrt_cavity* h, int copy) { return static_cast<real*>(h->gbuf) + (size_t)copy * 5 * h->plane; }

template <typename real>
int launch_step_t(dmrt_cavity* h, hipStream_t s, int from)
{
    StepArgs<real> A;
    A.fin = fptr<real>(h, from);
    A.gin = gptr<real>(h, from);
    A.fout = fptr<real>(h, from ^ 1);
    A.gout = gptr<real>(h, from ^ 1);
    A.thw = static_cast<const real*>(h->thw_real);
    A.n = h->n; A.pitch = h->pitch; A.plane = h->plane;
    A.tiles_x = (h->n + h->block_x - 1) / h->block_x;
    const int tiles_y = (h->n + h->block_y - 1) / h->block_y;
    A.tiles = A.tiles_x * tiles_y;
    A.xcd_remap = h->xcd_remap;
    A.c = make_coef<real>(h->p, h->d);
    int nblocks = A.tiles;
    if (h->xcd_remap) nblocks = (nblocks + 7) / 8 * 8;
    nblocks += add_wall_check(h, A, h->block_x * h->block_y);
    dim3 grid(nblocks), block(h->block_x, h->block_y);
    switch (h->p.bc_mode) {
    case DMRT_BC_CAVITY: hipLaunchKernelGGL((step_kernel<real, BC_CAVITY>), grid, block, 0, s, A); break;
    case DMRT_BC_PERIODIC: hipLaunchKernelGGL((step_kernel<real, BC_PERIODIC>), grid, block, 0, s, A); break;
    case DMRT_BC_CHANNEL_X: hipLaunchKernelGGL((step_kernel<real, BC_CHANNEL_X>), grid, block, 0, s, A); break;
    default: hipLaunchKernelGGL((step_kernel<real, BC_ADIABATIC_BOX>), grid, block, 0, s, A); break;
    }
    HIPCHK(hipGetLastError());
    return DMRT_OK;
}

int launch_step(dmrt_cavity* h, hipStream_t s, int from)
{
    return h->esz == sizeof(double) ? launch_step_t<double>(h, s, from)
                                    : launch_step_t<float>(h, s, from);
}

template <typename real>
int launch_nusselt_t(dmrt_cavity* h, hipStream_t s, int copy, int wall, double* local,
                     double* avg, bool to_ring)
{
    const double dT = h->p.theta_hot - h->p.theta_cold;
    const double inv_dT = dT != 0.0 ? 1.0 / dT : 1.0;
    hipLaunchKernelGGL((nusselt_kernel<real>), dim3(1), dim3(256), 0, s, gptr<real>(h, copy),
                       h->n, h->pitch, h->plane, wall, h->thw_dbl, h->p.theta_cold, h->d.H, inv_dT,
                       local, avg, to_ring ? h->ring : nullptr, h->ring_count, h->ring_cap);
    HIPCHK(hipGetLastError());
    return DMRT_OK;
}

int launch_nusselt(dmrt_cavity* h, hipStream_t s, int copy, int wall, double* local, double* avg,
                   bool to_ring)
{
    return h->esz == sizeof(double) ? launch_nusselt_t<double>(h, s, copy, wall, local, avg, to_ring)
                                    : launch_nusselt_t<float>(h, s, copy, wall, local, avg, to_ring);
}

// Hot-wall Nusselt samples that K-step launches left in the first nslots
// slots of h->samp, appended to the ring in order by one kernel.
int launch_nusselt_slots(dmrt_cavity* h, hipStream_t s, int nslots)
{
    const double dT = h->p.theta_hot - h->p.theta_cold;
    const double inv_dT = dT != 0.0 ? 1.0 / dT : 1.0;
    hipLaunchKernelGGL(nusselt_slots_kernel, dim3(1), dim3(256), 0, s, h->samp, nslots, h->n, h->thw_dbl,
                       h->d.H, inv_dT, h->ring, h->ring_count, h->ring_cap);
    HIPCHK(hipGetLastError());
    return DMRT_OK;
}

// Enqueue `count` steps starting at copy `from` with Nu samples where due;
// `base` is the step counter before the first of them.  Groups of K =
// h->temporal steps run as one launch through LDS when enabled; a sample
// due at any step of a group is taken by that launch (the wall-column sums
// of the step, into the next free slot of h->samp), and the slots are
// reduced into the ring by one kernel when they run out and at the end, in
// step order.  A sample after a single step is taken directly, after the
// pending slots.  *flips receives the number of launches (each moves the
// state to the other copy).
//
// With the marching form, a count that is not a multiple of K ends in
// marching launches of fewer steps where the kernel has such shapes (the
// last K + r or r steps split into the fewest of them), and only what is
// left in single steps; every form computes the same arithmetic, so the
// state is bitwise the same.
namespace {
// Launch sizes, from the set `sz` (at most kMaxK each), that add up to
// `total` <= 2 kMaxK: the fewest launches, and of those the one whose
// smallest launch is largest (short launches are the least efficient per
// step); empty if there is none.
void split_rec(int left, int maxk, const std::vector<int>& sz, std::vector<int>& cur, std::vector<int>& best)
{
    if (left == 0) {
        const bool better = best.empty() || cur.size() < best.size() ||
                            (cur.size() == best.size() && cur.back() > best.back());
        if (better) best = cur;
        return;
    }
    if (!best.empty() && cur.size() >= best.size()) return;
    for (int k : sz)
        if (k <= left && k <= maxk) {   // non-increasing sizes: each multiset once
            cur.push_back(k);
            split_rec(left - k, k, sz, cur, best);
            cur.pop_back();
        }
}
std::vector<int> split_steps(int total, std::vector<int> sz)
{
    std::sort(sz.rbegin(), sz.rend());
    std::vector<int> cur, best;
    split_rec(total, total, sz, cur, best);
    return best;
}
}  // namespace

int enqueue_steps(dmrt_cavity* h, hipStream_t s, int from, long base, long count, int* flips)
{
    int c = from, nflip = 0, pend = 0;
    const int K = h->p.bc_mode == DMRT_BC_CAVITY ? h->temporal : 1;
    // launch sizes of the whole count: full K-step launches, the tail's
    // multi-step launches, then single steps
    long full = K >= 2 ? count / K : 0, singles = count - full * K;
    std::vector<int> tail;
    if (K >= 2 && singles > 0 && h->march) {
        std::vector<int> sz{K};
        for (int k = 2; k < K; ++k)
            if (h->march_rem_B[k]) sz.push_back(k);
        // the tail of r steps alone, or with the last full launch (the
        // fewer launches in all, then the larger smallest launch)
        const int r = int(singles);
        tail = split_steps(r, sz);
        if (full > 0) {
            std::vector<int> t2 = split_steps(K + r, sz);
            const bool better = !t2.empty() &&
                                (tail.empty() || t2.size() < tail.size() + 1 ||
                                 (t2.size() == tail.size() + 1 && t2.back() > tail.back()));
            if (better) {
                tail = t2;
                --full;
            }
        }
        if (!tail.empty()) singles = 0;
    }
    long launch = 0;
    const long nlaunch = full + long(tail.size()) + singles;
    auto flush = [&]() -> int {
        if (pend == 0) return DMRT_OK;
        const int rc = launch_nusselt_slots(h, s, pend);
        pend = 0;
        return rc;
    };
    long i = 0;
    for (; launch < nlaunch; ++launch) {
        int rc;
        const long t = launch - full;
        const int m = t < 0 ? K : (t < long(tail.size()) ? tail[size_t(t)] : 1);
        if (m >= 2) {
            int mask = 0;
            if (h->series_stride > 0)
                for (int j = 1; j <= m; ++j)
                    if ((base + i + j) % h->series_stride == 0) mask |= 1 << j;
            const int ns = __builtin_popcount(unsigned(mask));
            if (pend + ns > kSampSlots && (rc = flush())) return rc;
            double* slots = h->samp ? h->samp + (size_t)pend * 2 * h->n : nullptr;
            if (m == K)
                rc = h->esz == sizeof(double)
                         ? launch_stepk<double>(h, s, fptr<double>(h, c), gptr<double>(h, c),
                                                fptr<double>(h, c ^ 1), gptr<double>(h, c ^ 1), nullptr,
                                                nullptr, slots, mask)
                         : launch_stepk<float>(h, s, fptr<float>(h, c), gptr<float>(h, c),
                                               fptr<float>(h, c ^ 1), gptr<float>(h, c ^ 1), nullptr,
                                               nullptr, slots, mask);
            else
                rc = h->esz == sizeof(double)
                         ? launch_stepm<double>(h, s, fptr<double>(h, c), gptr<double>(h, c),
                                                fptr<double>(h, c ^ 1), gptr<double>(h, c ^ 1), slots, mask, m)
                         : launch_stepm<float>(h, s, fptr<float>(h, c), gptr<float>(h, c),
                                               fptr<float>(h, c ^ 1), gptr<float>(h, c ^ 1), slots, mask, m);
            pend += ns;
            i += m;
            h->wcheck = false;                       // the first launch took the watchdog
            if (rc) return rc;
            c ^= 1;
            ++nflip;
        } else {
            rc = launch_step(h, s, c);
            i += 1;
            h->wcheck = false;
            if (rc) return rc;
            c ^= 1;
            ++nflip;
            if (h->series_stride > 0 && (base + i) % h->series_stride == 0) {
                if ((rc = flush())) return rc;
                rc = launch_nusselt(h, s, c, 0, nullptr, nullptr, true);
                if (rc) return rc;
            }
        }
    }
    const int rc = flush();
    if (rc) return rc;
    if (flips) *flips = nflip;
    return DMRT_OK;
}

int graph_unit(const dmrt_cavity* h)
{
    // steps per graph: even (returns to the same copy) and a multiple of the
    // Nu sampling stride, so that replays stay aligned with the samples
    long k = h->graph_steps;
    if (k <= 0) return 0;
    if (k % 2) ++k;
    if (h->series_stride > 0) {
        long s = h->series_stride;
        long l = (s % 2) ? 2 * s : s;
        k = (k + l - 1) / l * l;
    }
    return (int)k;
}

int build_graph(dmrt_cavity* h, int parity, int unit)
{
    HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_steps(h, h->cap_stream, parity, 0, unit, &h->graph_flips[parity]);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) return record_hip(e, "hipStreamEndCapture");
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { (void)hipGraphDestroy(g); return record_hip(e, "hipGraphInstantiate"); }
    h->graph_def[parity] = g;
    h->graph[parity] = ge;
    return DMRT_OK;
}

int upload_hot_wall(dmrt_cavity* h)
{
    const int n = h->n;
    HIPCHK(hipMemcpyAsync(h->thw_dbl, h->thw_host.data(), n * sizeof(double),
                          hipMemcpyHostToDevice, h->stream));
    if (h->esz == sizeof(double)) {
        HIPCHK(hipMemcpyAsync(h->thw_real, h->thw_host.data(), n * sizeof(double),
                              hipMemcpyHostToDevice, h->stream));
    } else {
        std::vector<float> tmp(n);
        for (int i = 0; i < n; ++i) tmp[i] = (float)h->thw_host[i];
        HIPCHK(hipMemcpyAsync(h->thw_real, tmp.data(), n * sizeof(float), hipMemcpyHostToDevice,
                              h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    return DMRT_OK;
}

template <typename real>
int launch_init_t(dmrt_cavity* h, const double* dr, const double* U, const double* V,
                  const double* T)
{
    const dim3 block(64, 4), grid((h->n + 63) / 64, (h->n + 3) / 4);
    hipLaunchKernelGGL((init_kernel<real>), grid, block, 0, h->stream, fptr<real>(h, 0),
                       gptr<real>(h, 0), dr, U, V, T, h->n, h->pitch, h->plane,
                       make_coef<real>(h->p, h->d), real(h->d.w0), real(h->d.wm));
    HIPCHK(hipGetLastError());
    return DMRT_OK;
}

int ensure_scratch(dmrt_cavity* h)
{
    if (!h->scratch) {
        const size_t nn = (size_t)h->n * h->n;
        HIPCHK(hipMalloc(&h->scratch, 4 * nn * sizeof(double)));
    }
    return DMRT_OK;
}

int check_host_array(const double* a, size_t count)
{
    if (!a) return DMRT_OK;
    for (size_t i = 0; i < count; ++i)
        if (!std::isfinite(a[i])) return DMRT_EINVAL;
    return DMRT_OK;
}

int reset_series(dmrt_cavity* h)
{
    if (h->ring_count) HIPCHK(hipMemsetAsync(h->ring_count, 0, sizeof(unsigned long long), h->stream));
    return DMRT_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int dmrt_params_default(dmrt_params* p)
{
    if (!p) return DMRT_EINVAL;
    p->n = 64;
    p->Ra = 1e3; p->Pr = 0.01; p->Ma = 0.1;
    p->theta_hot = 0.5; p->theta_cold = -0.5;
    p->precision = DMRT_FP64;
    p->q5_mode = DMRT_Q5_FIXED_A;
    p->a = -2.0 / 3.0;
    p->bc_mode = DMRT_BC_CAVITY;
    p->gbeta_override = NAN;
    p->force_x = 0.0;
    p->theta_ref = 0.0;
    p->collision = DMRT_COLL_MRT;
    return DMRT_OK;
}

int dmrt_derive(const dmrt_params* p, dmrt_derived* out) { return derive(p, out); }

int dmrt_buffer_bytes(const dmrt_params* p, size_t* f_bytes, size_t* g_bytes)
{
    dmrt_derived d;
    int rc = derive(p, &d);
    if (rc) return rc;
    const size_t plane = (size_t)p->n * pitch_of(p->n);
    const size_t e = elem_size(p->precision);
    if (f_bytes) *f_bytes = 2 * 9 * plane * e;
    if (g_bytes) *g_bytes = 2 * 5 * plane * e;
    return DMRT_OK;
}

int dmrt_destroy(dmrt_cavity* h);

int dmrt_create(const dmrt_params* p, void* ext_f, void* ext_g, void* hip_stream,
                dmrt_cavity** out)
{
    if (!out) return DMRT_EINVAL;
    *out = nullptr;
    dmrt_derived d;
    int rc = derive(p, &d);
    if (rc) return rc;
    if ((ext_f == nullptr) != (ext_g == nullptr)) return DMRT_EINVAL;
    if ((ext_f && ((uintptr_t)ext_f % 256)) || (ext_g && ((uintptr_t)ext_g % 256))) return DMRT_EINVAL;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_last_error = std::string("device is ") + prop.gcnArchName + ", not gfx950";
        return DMRT_ENODEV;
    }
    dmrt_cavity* h = new (std::nothrow) dmrt_cavity();
    if (!h) return DMRT_ENOMEM;
    h->p = *p;
    h->d = d;
    h->dev = dev;
    h->n = p->n;
    h->pitch = pitch_of(p->n);
    h->plane = h->n * h->pitch;
    h->esz = elem_size(p->precision);
    h->thw_host.assign(h->n, p->theta_hot);
    auto fail = [&](int code) { dmrt_destroy(h); return code; };
    hipError_t e;
    if (hip_stream) {
        h->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return fail(record_hip(e, "hipStreamCreate"));
        h->own_stream = true;
    }
    e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(record_hip(e, "hipStreamCreate(capture)"));
    const size_t fbytes = 2 * 9 * (size_t)h->plane * h->esz;
    const size_t gbytes = 2 * 5 * (size_t)h->plane * h->esz;
    if (ext_f) {
        h->fbuf = ext_f;
        h->gbuf = ext_g;
    } else {
        if ((e = hipMalloc(&h->fbuf, fbytes)) != hipSuccess) return fail(record_hip(e, "hipMalloc(f)"));
        if ((e = hipMalloc(&h->gbuf, gbytes)) != hipSuccess) return fail(record_hip(e, "hipMalloc(g)"));
        h->own_bufs = true;
    }
    // padding columns are never read or written by the kernels; clear them
    // once so that checkpoints and counters see defined memory
    if ((e = hipMemsetAsync(h->fbuf, 0, fbytes, h->stream)) != hipSuccess) return fail(record_hip(e, "memset f"));
    if ((e = hipMemsetAsync(h->gbuf, 0, gbytes, h->stream)) != hipSuccess) return fail(record_hip(e, "memset g"));
    if ((e = hipMalloc(&h->thw_real, h->n * h->esz)) != hipSuccess) return fail(record_hip(e, "hipMalloc(thw)"));
    if ((e = hipMalloc(&h->thw_dbl, h->n * sizeof(double))) != hipSuccess) return fail(record_hip(e, "hipMalloc(thw)"));
    if ((e = hipMalloc(&h->nu_buf, (h->n + 1) * sizeof(double))) != hipSuccess) return fail(record_hip(e, "hipMalloc(nu)"));
    {
        void* nf = nullptr;
        if ((e = hipHostMalloc(&nf, sizeof(int), hipHostMallocDefault)) != hipSuccess)
            return fail(record_hip(e, "hipHostMalloc(watchdog flag)"));
        h->nonfinite = static_cast<volatile int*>(nf);
        *h->nonfinite = 0;
    }
    if ((rc = upload_hot_wall(h))) return fail(rc);
    *out = h;
    rc = dmrt_set_theta(h, nullptr);
    if (rc) { *out = nullptr; return fail(rc); }
    return DMRT_OK;
}

int dmrt_set_equilibrium(dmrt_cavity* h, const double* drho, const double* U, const double* V,
                         const double* theta)
{
    if (!h) return DMRT_EINVAL;
    const size_t nn = (size_t)h->n * h->n;
    const double* src[4] = {drho, U, V, theta};
    for (auto a : src)
        if (check_host_array(a, nn)) return DMRT_EINVAL;
    DeviceGuard g(h->dev);
    if (!g.ok) return record_hip(hipErrorInvalidDevice, "hipSetDevice");
    invalidate_adjoint(h->adj);   // the gradient problem's initial field changes
    int rc = ensure_scratch(h);
    if (rc) return rc;
    const double* dptr[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int i = 0; i < 4; ++i) {
        if (!src[i]) continue;
        double* dst = h->scratch + i * nn;
        HIPCHK(hipMemcpyAsync(dst, src[i], nn * sizeof(double), hipMemcpyHostToDevice, h->stream));
        dptr[i] = dst;
    }
    rc = h->esz == sizeof(double) ? launch_init_t<double>(h, dptr[0], dptr[1], dptr[2], dptr[3])
                                  : launch_init_t<float>(h, dptr[0], dptr[1], dptr[2], dptr[3]);
    if (rc) return rc;
    // a rest state with a temperature field is the initial condition of the
    // gradient problem: keep theta0 on the device
    h->theta0_valid = false;
    if (!drho && !U && !V) {
        if (!h->theta0) HIPCHK(hipMalloc(&h->theta0, nn * sizeof(double)));
        if (theta)
            HIPCHK(hipMemcpyAsync(h->theta0, dptr[3], nn * sizeof(double), hipMemcpyDeviceToDevice,
                                  h->stream));
        else
            HIPCHK(hipMemsetAsync(h->theta0, 0, nn * sizeof(double), h->stream));
        h->theta0_valid = true;
    }
    h->cur = 0;
    h->step = 0;
    if ((rc = reset_series(h))) return rc;
    HIPCHK(hipStreamSynchronize(h->stream));
    *h->nonfinite = 0;
    return DMRT_OK;
}

int dmrt_set_theta(dmrt_cavity* h, const double* theta0)
{
    return dmrt_set_equilibrium(h, nullptr, nullptr, nullptr, theta0);
}

int dmrt_set_hot_wall(dmrt_cavity* h, const double* theta_w)
{
    if (!h || !theta_w) return DMRT_EINVAL;
    if (check_host_array(theta_w, h->n)) return DMRT_EINVAL;
    DeviceGuard g(h->dev);
    invalidate_adjoint(h->adj);   // the backward differentiates about the forward's wall
    h->thw_host.assign(theta_w, theta_w + h->n);
    return upload_hot_wall(h);
}

static int launch_wall_check(dmrt_cavity* h)
{
    const dim3 grid((2 * h->n + 255) / 256);
    if (h->esz == sizeof(double))
        hipLaunchKernelGGL((wall_check_kernel<double>), grid, dim3(256), 0, h->stream,
                           static_cast<const double*>(h->fbuf) + (size_t)h->cur * 9 * h->plane,
                           static_cast<const double*>(h->gbuf) + (size_t)h->cur * 5 * h->plane, h->n,
                           h->pitch, h->plane, const_cast<int*>(h->nonfinite));
    else
        hipLaunchKernelGGL((wall_check_kernel<float>), grid, dim3(256), 0, h->stream,
                           static_cast<const float*>(h->fbuf) + (size_t)h->cur * 9 * h->plane,
                           static_cast<const float*>(h->gbuf) + (size_t)h->cur * 5 * h->plane, h->n,
                           h->pitch, h->plane, const_cast<int*>(h->nonfinite));
    HIPCHK(hipGetLastError());
    return DMRT_OK;
}

int dmrt_step(dmrt_cavity* h, long nsteps)
{
    if (!h || nsteps < 0) return DMRT_EINVAL;
    DeviceGuard g(h->dev);
    if (!g.ok) return record_hip(hipErrorInvalidDevice, "hipSetDevice");
    // a watchdog pass of an earlier call (finished by now or not) found a
    // non-finite state: report it and enqueue nothing
    if (*h->nonfinite) return DMRT_ENONFINITE;
    if (nsteps == 0) return DMRT_OK;
    const int unit = graph_unit(h);
    // the watchdog runs on the state this call starts from: in the workgroups
    // its first launch appends, or on its own before a graph replay
    const bool graph_first = unit > 0 && (h->step % unit) == 0 && nsteps >= unit;
    if (graph_first) {
        const int rc = launch_wall_check(h);
        if (rc) return rc;
    }
    h->wcheck = !graph_first;
    h->unchecked = true;
    long left = nsteps;
    while (left > 0) {
        const bool aligned = unit > 0 && (h->step % unit) == 0;
        if (aligned && left >= unit) {
            if (!h->graph[h->cur]) {
                int rc = build_graph(h, h->cur, unit);
                if (rc) return rc;
            }
            // replay one unit at a time: a unit may move the state to the
            // other copy (odd number of launches), whose graph then follows
            const long reps = left / unit;
            for (long r = 0; r < reps; ++r) {
                if (!h->graph[h->cur]) {
                    int rc = build_graph(h, h->cur, unit);
                    if (rc) return rc;
                }
                HIPCHK(hipGraphLaunch(h->graph[h->cur], h->stream));
                h->cur ^= (h->graph_flips[h->cur] & 1);
            }
            h->step += reps * unit;
            left -= reps * unit;
        } else {
            long chunk = left;
            if (unit > 0) {
                const long to_align = unit - (h->step % unit);
                if (to_align < chunk) chunk = to_align;
            }
            int flips = 0;
            int rc = enqueue_steps(h, h->stream, h->cur, h->step, chunk, &flips);
            h->wcheck = false;
            if (rc) return rc;
            h->step += chunk;
            if (flips & 1) h->cur ^= 1;
            left -= chunk;
        }
    }
    return DMRT_OK;
}

int dmrt_sync(dmrt_cavity* h)
{
    if (!h) return DMRT_EINVAL;
    DeviceGuard g(h->dev);
    if (h->unchecked) {               // the state the last call left
        const int rc = launch_wall_check(h);
        if (rc) return rc;
        h->unchecked = false;
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    return *h->nonfinite ? DMRT_ENONFINITE : DMRT_OK;
}

int dmrt_get_step(dmrt_cavity* h, long* step)
{
    if (!h || !step) return DMRT_EINVAL;
    *step = h->step;
    return DMRT_OK;
}

int dmrt_get_fields(dmrt_cavity* h, double* U, double* V, double* theta, double* P)
{
    if (!h) return DMRT_EINVAL;
    DeviceGuard g(h->dev);
    int rc = ensure_scratch(h);
    if (rc) return rc;
    const size_t nn = (size_t)h->n * h->n;
    double* s = h->scratch;
    const dim3 block(64, 4), grid((h->n + 63) / 64, (h->n + 3) / 4);
    const double gy0 = -h->d.gbeta * h->p.theta_ref;
    if (h->esz == sizeof(double)) {
        hipLaunchKernelGGL((fields_kernel<double>), grid, block, 0, h->stream, fptr<double>(h, h->cur),
                           gptr<double>(h, h->cur), h->n, h->pitch, h->plane, h->d.gbeta, gy0,
                           h->p.force_x, s, s + nn, s + 2 * nn, s + 3 * nn);
    } else {
        // FP32 storage: coefficients rounded as the step kernel rounds them
        hipLaunchKernelGGL((fields_kernel<float>), grid, block, 0, h->stream, fptr<float>(h, h->cur),
                           gptr<float>(h, h->cur), h->n, h->pitch, h->plane,
                           (double)(float)h->d.gbeta, (double)(float)gy0, (double)(float)h->p.force_x,
                           s, s + nn, s + 2 * nn, s + 3 * nn);
    }
    HIPCHK(hipGetLastError());
    double* outs[4] = {U, V, theta, P};
    for (int i = 0; i < 4; ++i)
        if (outs[i])
            HIPCHK(hipMemcpyAsync(outs[i], s + i * nn, nn * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return DMRT_OK;
}

int dmrt_nusselt(dmrt_cavity* h, int wall, double* nu_avg, double* nu_local)
{
    if (!h || (wall != 0 && wall != 1)) return DMRT_EINVAL;
    DeviceGuard g(h->dev);
    int rc = launch_nusselt(h, h->stream, h->cur, wall, h->nu_buf + 1, h->nu_buf, false);
    if (rc) return rc;
    if (nu_avg) HIPCHK(hipMemcpyAsync(nu_avg, h->nu_buf, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    if (nu_local)
        HIPCHK(hipMemcpyAsync(nu_local, h->nu_buf + 1, h->n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return DMRT_OK;
}

int dmrt_nu_series(dmrt_cavity* h, int stride, long cap)
{
    if (!h || stride < 0 || (stride > 0 && cap <= 0)) return DMRT_EINVAL;
    DeviceGuard g(h->dev);
    HIPCHK(hipStreamSynchronize(h->stream));
    drop_graphs(h);
    if (h->ring) { (void)hipFree(h->ring); h->ring = nullptr; }
    h->ring_cap = 0;
    h->series_stride = stride;
    if (stride == 0) return DMRT_OK;
    if (!h->ring_count) HIPCHK(hipMalloc(&h->ring_count, sizeof(unsigned long long)));
    if (!h->samp) HIPCHK(hipMalloc(&h->samp, (size_t)kSampSlots * 2 * h->n * sizeof(double)));
    HIPCHK(hipMalloc(&h->ring, cap * sizeof(double)));
    h->ring_cap = cap;
    int rc = reset_series(h);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(h->stream));
    return DMRT_OK;
}

int dmrt_nu_series_read(dmrt_cavity* h, double* out, long* count)
{
    if (!h || !count) return DMRT_EINVAL;
    *count = 0;
    if (!h->ring) return DMRT_OK;
    DeviceGuard g(h->dev);
    unsigned long long c = 0;
    HIPCHK(hipMemcpyAsync(&c, h->ring_count, sizeof c, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    const unsigned long long cap = (unsigned long long)h->ring_cap;
    const unsigned long long have = c < cap ? c : cap;
    if (have && !out) return DMRT_EINVAL;
    std::vector<double> tmp(h->ring_cap);
    HIPCHK(hipMemcpyAsync(tmp.data(), h->ring, cap * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    const unsigned long long first = c - have;
    for (unsigned long long i = 0; i < have; ++i) out[i] = tmp[(first + i) % cap];
    *count = (long)have;
    return DMRT_OK;
}

int dmrt_residual(dmrt_cavity* h, double* res_theta, double* res_u)
{
    if (!h) return DMRT_EINVAL;
    DeviceGuard g(h->dev);
    const size_t nn = (size_t)h->n * h->n;
    if (!h->res_ref) {
        HIPCHK(hipMalloc(&h->res_ref, 3 * nn * sizeof(double)));
        HIPCHK(hipMemsetAsync(h->res_ref, 0, 3 * nn * sizeof(double), h->stream));
        h->res_blocks = (int)std::min<size_t>(1024, (nn + 255) / 256);
        HIPCHK(hipMalloc(&h->res_part, (h->res_blocks * 5 + 5) * sizeof(double)));
    }
    const double gy0 = -h->d.gbeta * h->p.theta_ref;
    double* fin = h->res_part + h->res_blocks * 5;
    if (h->esz == sizeof(double)) {
        hipLaunchKernelGGL((residual_kernel<double>), dim3(h->res_blocks), dim3(256), 0, h->stream,
                           fptr<double>(h, h->cur), gptr<double>(h, h->cur), h->n, h->pitch, h->plane,
                           h->d.gbeta, gy0, h->p.force_x, h->res_ref, h->res_part);
    } else {
        hipLaunchKernelGGL((residual_kernel<float>), dim3(h->res_blocks), dim3(256), 0, h->stream,
                           fptr<float>(h, h->cur), gptr<float>(h, h->cur), h->n, h->pitch, h->plane,
                           (double)(float)h->d.gbeta, (double)(float)gy0, (double)(float)h->p.force_x,
                           h->res_ref, h->res_part);
    }
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(residual_final_kernel, dim3(1), dim3(64), 0, h->stream, h->res_part,
                       h->res_blocks, fin);
    HIPCHK(hipGetLastError());
    double r[5];
    HIPCHK(hipMemcpyAsync(r, fin, sizeof r, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (res_theta) *res_theta = r[1] > 0 ? std::sqrt(r[0] / r[1]) : std::sqrt(r[0]);
    if (res_u) *res_u = r[3] > 0 ? std::sqrt(r[2] / r[3]) : std::sqrt(r[2]);
    if (r[4] > 0) return DMRT_ENONFINITE;
    return DMRT_OK;
}

// checkpoint layout: header (8 x int64), hot wall (n doubles), f (9 n^2), g (5 n^2)
int dmrt_state_bytes(dmrt_cavity* h, size_t* bytes)
{
    if (!h || !bytes) return DMRT_EINVAL;
    const size_t nn = (size_t)h->n * h->n;
    *bytes = 8 * sizeof(int64_t) + h->n * sizeof(double) + 14 * nn * h->esz;
    return DMRT_OK;
}

static const int64_t kStateMagic = 0x444d5254'53544154LL;   // "DMRTSTAT"

int dmrt_save_state(dmrt_cavity* h, void* host, size_t bytes)
{
    size_t need = 0;
    if (!h || !host) return DMRT_EINVAL;
    dmrt_state_bytes(h, &need);
    if (bytes < need) return DMRT_EINVAL;
    DeviceGuard g(h->dev);
    char* out = static_cast<char*>(host);
    int64_t hdr[8] = {kStateMagic, h->n, h->p.precision, h->step, h->p.bc_mode, 0, 0, 0};
    std::memcpy(out, hdr, sizeof hdr);
    std::memcpy(out + sizeof hdr, h->thw_host.data(), h->n * sizeof(double));
    char* data = out + sizeof hdr + h->n * sizeof(double);
    const size_t row = (size_t)h->n * h->esz;
    char* fb = static_cast<char*>(h->fbuf) + (size_t)h->cur * 9 * h->plane * h->esz;
    char* gb = static_cast<char*>(h->gbuf) + (size_t)h->cur * 5 * h->plane * h->esz;
    HIPCHK(hipMemcpy2DAsync(data, row, fb, h->pitch * h->esz, row, (size_t)9 * h->n,
                            hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpy2DAsync(data + 9 * (size_t)h->n * row, row, gb, h->pitch * h->esz, row,
                            (size_t)5 * h->n, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return DMRT_OK;
}

int dmrt_load_state(dmrt_cavity* h, const void* host, size_t bytes)
{
    size_t need = 0;
    if (!h || !host) return DMRT_EINVAL;
    dmrt_state_bytes(h, &need);
    if (bytes < need) return DMRT_EINVAL;
    const char* in = static_cast<const char*>(host);
    int64_t hdr[8];
    std::memcpy(hdr, in, sizeof hdr);
    if (hdr[0] != kStateMagic || hdr[1] != h->n || hdr[2] != h->p.precision || hdr[3] < 0)
        return DMRT_EINVAL;
    DeviceGuard g(h->dev);
    std::vector<double> thw(h->n);
    std::memcpy(thw.data(), in + sizeof hdr, h->n * sizeof(double));
    if (check_host_array(thw.data(), h->n)) return DMRT_EINVAL;
    HIPCHK(hipStreamSynchronize(h->stream));
    invalidate_adjoint(h->adj);
    h->thw_host = thw;
    int rc = upload_hot_wall(h);
    if (rc) return rc;
    const char* data = in + sizeof hdr + h->n * sizeof(double);
    const size_t row = (size_t)h->n * h->esz;
    h->cur = 0;
    char* fb = static_cast<char*>(h->fbuf);
    char* gb = static_cast<char*>(h->gbuf);
    HIPCHK(hipMemcpy2DAsync(fb, h->pitch * h->esz, data, row, row, (size_t)9 * h->n,
                            hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpy2DAsync(gb, h->pitch * h->esz, data + 9 * (size_t)h->n * row, row, row,
                            (size_t)5 * h->n, hipMemcpyHostToDevice, h->stream));
    h->step = hdr[3];
    if ((rc = reset_series(h))) return rc;
    HIPCHK(hipStreamSynchronize(h->stream));
    *h->nonfinite = 0;
    return DMRT_OK;
}

int dmrt_set_launch(dmrt_cavity* h, int block_x, int block_y, int xcd_remap, int graph_steps)
{
    if (!h) return DMRT_EINVAL;
    if (block_x != 64 && block_x != 128 && block_x != 256 && block_x != 512) return DMRT_EINVAL;
    if (block_y < 1 || block_x * block_y > 1024) return DMRT_EINVAL;
    if (xcd_remap != 0 && xcd_remap != 1) return DMRT_EINVAL;
    if (graph_steps < 0) return DMRT_EINVAL;
    DeviceGuard g(h->dev);
    HIPCHK(hipStreamSynchronize(h->stream));
    drop_graphs(h);
    if (h->adj) { free_adjoint(h->adj); h->adj = nullptr; }   // its graphs bake the shape
    h->block_x = block_x;
    h->block_y = block_y;
    h->xcd_remap = xcd_remap;
    h->graph_steps = graph_steps;
    return DMRT_OK;
}

int dmrt_set_temporal(dmrt_cavity* h, int steps_per_launch, int tile_rows)
{
    if (!h) return DMRT_EINVAL;
    if (!valid_temporal(steps_per_launch, tile_rows)) return DMRT_EINVAL;
    if (steps_per_launch >= 2 && h->p.bc_mode != DMRT_BC_CAVITY) return DMRT_EINVAL;
    DeviceGuard g(h->dev);
    HIPCHK(hipStreamSynchronize(h->stream));
    drop_graphs(h);
    if (h->adj) { free_adjoint(h->adj); h->adj = nullptr; }   // its graphs bake the mode
    h->temporal = steps_per_launch;
    h->t_rows = tile_rows;
    h->march = 0;
    return DMRT_OK;
}

int dmrt_set_temporal_march(dmrt_cavity* h, int steps_per_launch, int group_rows, int chunk_rows)
{
    if (!h) return DMRT_EINVAL;
    if (!valid_march(steps_per_launch, group_rows, int(h->esz)) || chunk_rows < 0) return DMRT_EINVAL;
    if (h->p.bc_mode != DMRT_BC_CAVITY) return DMRT_EINVAL;
    DeviceGuard g(h->dev);
    int chunk = chunk_rows, chunk_w = chunk_rows;   // a given chunk serves every band
    if (chunk == 0)
        chunk = h->esz == sizeof(double)
                    ? march_chunk_auto<double>(h->n, steps_per_launch, group_rows, h->dev, &chunk_w)
                    : march_chunk_auto<float>(h->n, steps_per_launch, group_rows, h->dev, &chunk_w);
    if (chunk <= 0) return record_hip(hipErrorInvalidValue, "occupancy query for the marching kernel");
    HIPCHK(hipStreamSynchronize(h->stream));
    drop_graphs(h);
    if (h->adj) { free_adjoint(h->adj); h->adj = nullptr; }
    h->temporal = steps_per_launch;
    // the adjoint's Nusselt-window launches use the tile form: keep its rows
    // valid for this K where the tile form has K (else those run single steps)
    if (steps_per_launch <= 4 && !valid_temporal(steps_per_launch, h->t_rows)) h->t_rows = 10;
    h->march = group_rows;
    h->march_chunk = std::min(chunk, h->n);
    h->march_chunk_w = std::min(std::max(chunk_w, 1), h->n);
    // shapes for the launches of fewer steps that end a count (the same
    // wave rows per group where the kernel has them, else the most)
    for (int k = 0; k < 8; ++k) h->march_rem_B[k] = h->march_rem_chunk[k] = h->march_rem_chunk_w[k] = 0;
    for (int k = 2; k < steps_per_launch; ++k) {
        int bk = valid_march(k, group_rows, int(h->esz)) ? group_rows : 0;
        for (int b = 8; b >= 1 && !bk; --b)
            if (valid_march(k, b, int(h->esz))) bk = b;
        if (!bk) continue;
        int ck = chunk_rows, ckw = chunk_rows;
        if (ck == 0)
            ck = h->esz == sizeof(double) ? march_chunk_auto<double>(h->n, k, bk, h->dev, &ckw)
                                          : march_chunk_auto<float>(h->n, k, bk, h->dev, &ckw);
        if (ck <= 0) continue;
        h->march_rem_B[k] = bk;
        h->march_rem_chunk[k] = std::min(ck, h->n);
        h->march_rem_chunk_w[k] = std::min(std::max(ckw, 1), h->n);
    }
    return DMRT_OK;
}

int dmrt_get_temporal_march(const dmrt_cavity* h, int* group_rows, int* chunk_rows)
{
    if (!h) return DMRT_EINVAL;
    if (group_rows) *group_rows = h->march;
    if (chunk_rows) *chunk_rows = h->march ? h->march_chunk : 0;
    return DMRT_OK;
}

int dmrt_buffers(dmrt_cavity* h, void** f, void** g, int* current)
{
    if (!h) return DMRT_EINVAL;
    if (f) *f = h->fbuf;
    if (g) *g = h->gbuf;
    if (current) *current = h->cur;
    return DMRT_OK;
}

int dmrt_destroy(dmrt_cavity* h)
{
    if (!h) return DMRT_OK;
    DeviceGuard g(h->dev);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    drop_graphs(h);
    if (h->own_bufs) { (void)hipFree(h->fbuf); (void)hipFree(h->gbuf); }
    if (h->adj) free_adjoint(h->adj);
    void* ptrs[] = {h->thw_real, h->thw_dbl, h->scratch, h->nu_buf, h->res_ref, h->res_part,
                    h->ring, h->samp, h->ring_count, h->theta0};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    if (h->nonfinite) (void)hipHostFree(const_cast<int*>(h->nonfinite));
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return DMRT_OK;
}

const char* dmrt_strerror(int code)
{
    switch (code) {
    case DMRT_OK: return "ok";
    case DMRT_EINVAL: return "invalid argument";
    case DMRT_EUNSTABLE: return "parameters outside the stable range of the scheme";
    case DMRT_ENOMEM: return "out of memory";
    case DMRT_EHIP: return "HIP runtime error";
    case DMRT_ENONFINITE: return "non-finite values in the state";
    case DMRT_ENODEV: return "no usable gfx950 device";
    default: return "unknown error";
    }
}

const char* dmrt_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
