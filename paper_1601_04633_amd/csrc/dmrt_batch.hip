// dmrt_batch.hip -- batched Ra x Pr sweep: many independent cavities of
// uneven size advanced together by one launch per step (C ABI in dmrt.h).
//
// All members live in one device arena (each with its own ping-pong planes,
// rows padded to 64 elements).  A device table of per-cavity parameter
// blocks and a table of workgroup tiles (cavity, x0, y0) drive one
// grid-stride kernel that applies the same per-node update as the
// single-cavity kernel, so every member evolves bitwise as it would alone.
//
// Schedule (chosen by the caller or the autotuner; results do not depend on
// it): tile shape, tile order (cavity-major / largest first / interleaved),
// workgroups per launch (one per tile, or a persistent grid), and cavity
// groups: members are packed in order into groups of at most `group_bytes`
// of state, and each group runs `group_steps` steps before the next group
// starts, so a group small enough for the last-level cache stays there.
// Steps per launch: one, K through LDS on overlapping footprints (the tile
// form), or K with the row-marching sweep, each workgroup taking one
// (member, column band, chunk of rows) of its group.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "dmrt.h"
#include "dmrt_device.hpp"
#include "dmrt_internal.hpp"

using namespace dmrt;

#define HIPCHK(expr) DMRT_HIPCHK(expr)

struct dmrt_batch {
    int count = 0;
    int precision = DMRT_FP32;
    size_t esz = 4;
    int dev = 0;
    std::vector<dmrt_params> p;
    std::vector<dmrt_derived> d;
    std::vector<size_t> off;        // byte offset of each member's f block in the arena
    std::vector<std::vector<double>> thw_host;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    void* thw_real = nullptr;       // concatenated hot-wall rows (compute precision)
    double* thw_d = nullptr;        // concatenated hot-wall rows (FP64)
    std::vector<size_t> thw_off;    // element offset of each member's hot-wall row
    void* cavs = nullptr;           // CavityDev<real>[count]
    size_t cav_size = 0;
    TileRef* tiles = nullptr;
    std::vector<int> group_tile_begin;   // tile range of each group, plus end
    int ntiles = 0;
    TileRef* foot_tiles = nullptr;           // footprints of the K-step kernel
    std::vector<int> group_foot_begin;
    int temporal = 1, t_rows = 10;       // steps per launch and footprint rows
    // row-marching form (march_B > 0: wave rows per step group; chunk rows,
    // 0 = chosen per group so that its workgroups are resident at once)
    int march_B = 0, march_chunk = 0;
    MarchRef* march_tiles = nullptr;
    std::vector<int> group_march_begin;
    int graph_flips[2] = {0, 0};
    double* nu = nullptr;
    int* flags = nullptr;
    double* scratch = nullptr;      // fields of one member
    size_t scratch_elems = 0;
    std::vector<int> dead;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap_stream = nullptr;
    int cur = 0;
    long step = 0;
    // schedule
    int block_x = 64, block_y = 4, order = 1, grid_blocks = 0;
    size_t group_bytes = 0;
    int group_steps = 64;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    hipGraph_t graph_def[2] = {nullptr, nullptr};
};

namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t member_bytes(const dmrt_batch* b, int i)
{
    const size_t plane = (size_t)b->p[i].n * pitch_of(b->p[i].n);
    return 2 * 14 * plane * b->esz;
}

void drop_graphs(dmrt_batch* b)
{
    for (int i = 0; i < 2; ++i) {
        if (b->graph[i]) (void)hipGraphExecDestroy(b->graph[i]);
        if (b->graph_def[i]) (void)hipGraphDestroy(b->graph_def[i]);
        b->graph[i] = nullptr;
        b->graph_def[i] = nullptr;
    }
}

template <typename real>
CavityDev<real> make_cav(const dmrt_batch* b, int i)
{
    CavityDev<real> c;
    const int n = b->p[i].n, pitch = pitch_of(n);
    const size_t plane = (size_t)n * pitch;
    real* base = reinterpret_cast<real*>(static_cast<char*>(b->arena) + b->off[i]);
    c.f[0] = base;
    c.f[1] = base + 9 * plane;
    c.g[0] = base + 18 * plane;
    c.g[1] = base + 23 * plane;
    c.thw = static_cast<const real*>(b->thw_real) + b->thw_off[i];
    c.thw_d = b->thw_d + b->thw_off[i];
    c.H = b->d[i].H;
    const double dT = b->p[i].theta_hot - b->p[i].theta_cold;
    c.inv_dT = dT != 0.0 ? 1.0 / dT : 1.0;
    c.theta_cold = b->p[i].theta_cold;
    c.n = n;
    c.pitch = pitch;
    c.plane = (int)plane;
    c.dead = b->dead[i];
    c.c = make_coef<real>(b->p[i], b->d[i]);
    return c;
}

template <typename real>
int upload_cavs_t(dmrt_batch* b)
{
    std::vector<CavityDev<real>> h(b->count);
    for (int i = 0; i < b->count; ++i) h[i] = make_cav<real>(b, i);
    HIPCHK(hipMemcpyAsync(b->cavs, h.data(), h.size() * sizeof(CavityDev<real>),
                          hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return DMRT_OK;
}

int upload_cavs(dmrt_batch* b)
{
    return b->esz == 8 ? upload_cavs_t<double>(b) : upload_cavs_t<float>(b);
}

int upload_hot_walls(dmrt_batch* b)
{
    size_t total = b->thw_off.back();
    std::vector<double> all(total);
    for (int i = 0; i < b->count; ++i)
        std::copy(b->thw_host[i].begin(), b->thw_host[i].end(), all.begin() + b->thw_off[i]);
    HIPCHK(hipMemcpyAsync(b->thw_d, all.data(), total * sizeof(double), hipMemcpyHostToDevice, b->stream));
    if (b->esz == 8) {
        HIPCHK(hipMemcpyAsync(b->thw_real, all.data(), total * sizeof(double), hipMemcpyHostToDevice,
                              b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
    } else {
        std::vector<float> f(all.begin(), all.end());
        HIPCHK(hipMemcpyAsync(b->thw_real, f.data(), total * sizeof(float), hipMemcpyHostToDevice,
                              b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
    }
    return DMRT_OK;
}

// Resident workgroups per CU of the batched marching kernel (K, B) in the
// batch's precision, or -1.
template <typename real>
int march_per_cu(int K, int B)
{
    int per_cu = 0;
#define DMRT_KB_OCC(KK, BB)                                                                           \
    if constexpr (march_lds_bytes(KK, BB, sizeof(real)) <= kLdsBytes)                                  \
        if (K == KK && B == BB &&                                                                     \
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_stepm_kernel<real, KK, BB>,    \
                                                         kFootW * KK * BB, 0) != hipSuccess)           \
            return -1;
    DMRT_FOR_EACH_KB(DMRT_KB_OCC)
#undef DMRT_KB_OCC
    return per_cu > 0 ? per_cu : -1;
}

// The row-marching table: for every group, its members' (column band,
// chunk) pairs, member by member, chunk rows row-major, odd chunks marching
// down; then dealt so that each of the 8 dies gets a contiguous range (the
// dispatcher deals workgroups round-robin over the dies; unused slots have
// cav = -1).  The chunk length of a group is march_chunk, or else the
// shortest that leaves all of the group's workgroups resident at once.
int build_march_tiles(dmrt_batch* b, const std::vector<std::vector<int>>& groups)
{
    b->group_march_begin.clear();
    if (b->march_tiles) { (void)hipFree(b->march_tiles); b->march_tiles = nullptr; }
    if (b->march_B <= 0) return DMRT_OK;
    const int K = b->temporal, B = b->march_B;
    const int W = kFootW - 2 * (K - 1);
    int slots = 0;
    if (b->march_chunk <= 0) {
        int cus = 0;
        HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->dev));
        const int per_cu = b->esz == 8 ? march_per_cu<double>(K, B) : march_per_cu<float>(K, B);
        if (per_cu <= 0 || cus <= 0) {
            set_last_error("batch marching schedule: occupancy query failed");
            return DMRT_EHIP;
        }
        slots = per_cu * cus;
    }
    std::vector<MarchRef> all;
    for (const auto& g : groups) {
        b->group_march_begin.push_back((int)all.size());
        int chunk = b->march_chunk;
        if (chunk <= 0) {
            int nmax = 1;
            for (int i : g) nmax = std::max(nmax, b->p[i].n);
            chunk = nmax;
            for (int c = 1; c <= nmax; ++c) {
                long wgs = 0;
                for (int i : g) {
                    const int n = b->p[i].n;
                    wgs += (long)((n + W - 1) / W) * ((n + c - 1) / c);
                }
                if (wgs <= slots) { chunk = c; break; }
            }
        }
        std::vector<MarchRef> list;
        for (int i : g) {
            const int n = b->p[i].n, tiles_x = (n + W - 1) / W;
            for (int ty = 0, y0 = 0; y0 < n; ++ty, y0 += chunk)
                for (int tx = 0; tx < tiles_x; ++tx)
                    list.push_back({i, tx * W - (K - 1), y0, std::min(y0 + chunk, n) | ((ty & 1) << 30)});
        }
        const int per = ((int)list.size() + 7) / 8;
        std::vector<MarchRef> dealt((size_t)per * 8, MarchRef{-1, 0, 0, 0});
        for (int blk = 0; blk < per * 8; ++blk) {
            const int t = (blk & 7) * per + (blk >> 3);
            if (t < (int)list.size()) dealt[blk] = list[t];
        }
        all.insert(all.end(), dealt.begin(), dealt.end());
    }
    b->group_march_begin.push_back((int)all.size());
    HIPCHK(hipMalloc(&b->march_tiles, all.size() * sizeof(MarchRef)));
    HIPCHK(hipMemcpyAsync(b->march_tiles, all.data(), all.size() * sizeof(MarchRef), hipMemcpyHostToDevice,
                          b->stream));
    return DMRT_OK;
}

// Builds the tile table and the group ranges for the current schedule.
int build_tiles(dmrt_batch* b)
{
    std::vector<int> ord(b->count);
    std::iota(ord.begin(), ord.end(), 0);
    if (b->order == 1)   // largest first, stable
        std::stable_sort(ord.begin(), ord.end(),
                         [&](int a, int c) { return b->p[a].n > b->p[c].n; });
    // groups of members, in order, of at most group_bytes state each
    std::vector<std::vector<int>> groups;
    size_t acc = 0;
    for (int i : ord) {
        const size_t mb = member_bytes(b, i);
        if (groups.empty() || (b->group_bytes > 0 && acc + mb > b->group_bytes && acc > 0)) {
            groups.emplace_back();
            acc = 0;
        }
        groups.back().push_back(i);
        acc += mb;
    }
    std::vector<TileRef> tiles;
    b->group_tile_begin.clear();
    for (const auto& g : groups) {
        b->group_tile_begin.push_back((int)tiles.size());
        // per-member tile lists
        std::vector<std::vector<TileRef>> per(g.size());
        for (size_t j = 0; j < g.size(); ++j) {
            const int i = g[j], n = b->p[i].n;
            for (int y0 = 0; y0 < n; y0 += b->block_y)
                for (int x0 = 0; x0 < n; x0 += b->block_x) per[j].push_back({i, x0, y0, 0});
        }
        if (b->order == 2) {   // interleave the members' tiles round-robin
            size_t k = 0;
            bool any = true;
            while (any) {
                any = false;
                for (auto& v : per)
                    if (k < v.size()) { tiles.push_back(v[k]); any = true; }
                ++k;
            }
        } else {
            for (auto& v : per) tiles.insert(tiles.end(), v.begin(), v.end());
        }
    }
    b->group_tile_begin.push_back((int)tiles.size());
    b->ntiles = (int)tiles.size();
    if (b->tiles) { (void)hipFree(b->tiles); b->tiles = nullptr; }
    HIPCHK(hipMalloc(&b->tiles, tiles.size() * sizeof(TileRef)));
    HIPCHK(hipMemcpyAsync(b->tiles, tiles.data(), tiles.size() * sizeof(TileRef),
                          hipMemcpyHostToDevice, b->stream));
    // footprints of the K-step tile kernel, same groups and member order
    // (none in the row-marching form)
    std::vector<TileRef> fp;
    b->group_foot_begin.clear();
    const bool tile_form = b->march_B <= 0 && b->temporal <= 4;
    const int K = std::max(2, b->temporal), R = b->t_rows;
    const int W = kFootW - 2 * (K - 1), HO = R - 2 * (K - 1);
    for (const auto& g : groups) {
        b->group_foot_begin.push_back((int)fp.size());
        if (!tile_form || HO <= 0) continue;
        for (int i : g) {
            const int n = b->p[i].n;
            for (int y0 = 0; y0 < n; y0 += HO)
                for (int x0 = 0; x0 < n; x0 += W) fp.push_back({i, x0 - (K - 1), y0 - (K - 1), 0});
        }
    }
    b->group_foot_begin.push_back((int)fp.size());
    if (b->foot_tiles) { (void)hipFree(b->foot_tiles); b->foot_tiles = nullptr; }
    HIPCHK(hipMalloc(&b->foot_tiles, std::max<size_t>(1, fp.size()) * sizeof(TileRef)));
    HIPCHK(hipMemcpyAsync(b->foot_tiles, fp.data(), fp.size() * sizeof(TileRef), hipMemcpyHostToDevice,
                          b->stream));
    int rc = build_march_tiles(b, groups);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(b->stream));
    return DMRT_OK;
}

template <typename real>
int launch_range_t(dmrt_batch* b, hipStream_t s, int t0, int t1, int from)
{
    const int span = t1 - t0;
    if (span <= 0) return DMRT_OK;
    const int grid = b->grid_blocks > 0 ? std::min(span, b->grid_blocks) : span;
    hipLaunchKernelGGL((batch_step_kernel<real>), dim3(grid), dim3(b->block_x, b->block_y), 0, s,
                       static_cast<const CavityDev<real>*>(b->cavs), b->tiles, t0, t1, from);
    HIPCHK(hipGetLastError());
    return DMRT_OK;
}

int launch_range(dmrt_batch* b, hipStream_t s, int t0, int t1, int from)
{
    return b->esz == 8 ? launch_range_t<double>(b, s, t0, t1, from)
                       : launch_range_t<float>(b, s, t0, t1, from);
}

template <typename real>
int launch_rangek_t(dmrt_batch* b, hipStream_t s, int t0, int t1, int from)
{
    const int span = t1 - t0;
    if (span <= 0) return DMRT_OK;
    const int grid = b->grid_blocks > 0 ? std::min(span, b->grid_blocks) : span;
    const CavityDev<real>* cv = static_cast<const CavityDev<real>*>(b->cavs);
    const dim3 block(kFootW, b->t_rows);
    const int K = b->temporal, R = b->t_rows;
#define DMRT_BKR(KK, RR)                                                                             \
    if (K == KK && R == RR) {                                                                         \
        hipLaunchKernelGGL((batch_stepk_kernel<real, RR, KK>), dim3(grid), block, 0, s, cv, b->foot_tiles, \
                           t0, t1, from);                                                             \
        HIPCHK(hipGetLastError());                                                                    \
        return DMRT_OK;                                                                               \
    }
    DMRT_FOR_EACH_KR(DMRT_BKR)
#undef DMRT_BKR
    return DMRT_EINVAL;
}

template <typename real>
int launch_rangem_t(dmrt_batch* b, hipStream_t s, int t0, int t1, int from)
{
    const int span = t1 - t0;
    if (span <= 0) return DMRT_OK;
    const CavityDev<real>* cv = static_cast<const CavityDev<real>*>(b->cavs);
    const int K = b->temporal, B = b->march_B;
#define DMRT_BKB(KK, BB)                                                                               \
    if constexpr (march_lds_bytes(KK, BB, sizeof(real)) <= kLdsBytes)                                    \
        if (K == KK && B == BB) {                                                                       \
            hipLaunchKernelGGL((batch_stepm_kernel<real, KK, BB>), dim3(span), dim3(kFootW, KK * BB), 0, s, \
                               cv, b->march_tiles, t0, t1, from);                                       \
            HIPCHK(hipGetLastError());                                                                  \
            return DMRT_OK;                                                                             \
        }
    DMRT_FOR_EACH_KB(DMRT_BKB)
#undef DMRT_BKB
    return DMRT_EINVAL;
}

// One round: each group in turn advances `steps` steps (K steps per launch
// when the K-step kernel is selected).  *flips receives the
// number of launches per group (each moves the state to the other copy).
int enqueue_round(dmrt_batch* b, hipStream_t s, int from, int steps, int* flips)
{
    const int ng = (int)b->group_tile_begin.size() - 1;
    int nf = 0;
    for (int g = 0; g < ng; ++g) {
        int c = from, k = steps;
        nf = 0;
        while (k > 0) {
            int rc;
            if (b->temporal >= 2 && k >= b->temporal && b->march_B > 0) {
                const int m0 = b->group_march_begin[g], m1 = b->group_march_begin[g + 1];
                rc = b->esz == 8 ? launch_rangem_t<double>(b, s, m0, m1, c) : launch_rangem_t<float>(b, s, m0, m1, c);
                k -= b->temporal;
            } else if (b->temporal >= 2 && k >= b->temporal) {
                rc = b->esz == 8 ? launch_rangek_t<double>(b, s, b->group_foot_begin[g], b->group_foot_begin[g + 1], c)
                                 : launch_rangek_t<float>(b, s, b->group_foot_begin[g], b->group_foot_begin[g + 1], c);
                k -= b->temporal;
            } else {
                rc = launch_range(b, s, b->group_tile_begin[g], b->group_tile_begin[g + 1], c);
                k -= 1;
            }
            if (rc) return rc;
            c ^= 1;
            ++nf;
        }
    }
    if (flips) *flips = nf;
    return DMRT_OK;
}

int build_graph(dmrt_batch* b, int parity)
{
    HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_round(b, b->cap_stream, parity, b->group_steps, &b->graph_flips[parity]);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) return record_hip(e, "hipStreamEndCapture");
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { (void)hipGraphDestroy(g); return record_hip(e, "hipGraphInstantiate"); }
    b->graph_def[parity] = g;
    b->graph[parity] = ge;
    return DMRT_OK;
}

template <typename real>
int init_member_t(dmrt_batch* b, int i, const double* theta_dev)
{
    const CavityDev<real> c = make_cav<real>(b, i);
    const dim3 block(64, 4), grid((c.n + 63) / 64, (c.n + 3) / 4);
    hipLaunchKernelGGL((init_kernel<real>), grid, block, 0, b->stream, c.f[b->cur], c.g[b->cur],
                       nullptr, nullptr, nullptr, theta_dev, c.n, c.pitch, c.plane, c.c,
                       real(b->d[i].w0), real(b->d[i].wm));
    HIPCHK(hipGetLastError());
    return DMRT_OK;
}

int check_finite(const double* a, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return DMRT_EINVAL;
    return DMRT_OK;
}

}  // namespace

extern "C" {

int dmrt_batch_destroy(dmrt_batch* b);

int dmrt_batch_create(const dmrt_params* p, int count, void* hip_stream, dmrt_batch** out)
{
    if (!out || !p || count <= 0 || count > 65535) return DMRT_EINVAL;
    *out = nullptr;
    std::vector<dmrt_derived> d(count);
    for (int i = 0; i < count; ++i) {
        int rc = derive(&p[i], &d[i]);
        if (rc) return rc;
        if (p[i].precision != p[0].precision || p[i].bc_mode != DMRT_BC_CAVITY) return DMRT_EINVAL;
    }
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return DMRT_ENODEV;
    dmrt_batch* b = new (std::nothrow) dmrt_batch();
    if (!b) return DMRT_ENOMEM;
    auto fail = [&](int code) { dmrt_batch_destroy(b); return code; };
    b->count = count;
    b->precision = p[0].precision;
    b->esz = elem_size(b->precision);
    b->dev = dev;
    b->p.assign(p, p + count);
    b->d = d;
    b->dead.assign(count, 0);
    b->thw_host.resize(count);
    b->off.resize(count);
    b->thw_off.resize(count + 1);
    size_t bytes = 0, thw = 0, max_nn = 0;
    for (int i = 0; i < count; ++i) {
        b->off[i] = bytes;
        bytes = align_up(bytes + member_bytes(b, i), 256);
        b->thw_off[i] = thw;
        thw += align_up((size_t)p[i].n, 64);
        b->thw_host[i].assign(p[i].n, p[i].theta_hot);
        max_nn = std::max(max_nn, (size_t)p[i].n * p[i].n);
    }
    b->thw_off[count] = thw;
    b->arena_bytes = bytes;
    b->scratch_elems = 4 * max_nn;
    hipError_t e;
    if (hip_stream) {
        b->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if ((e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking)) != hipSuccess)
            return fail(record_hip(e, "hipStreamCreate"));
        b->own_stream = true;
    }
    if ((e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess)
        return fail(record_hip(e, "hipStreamCreate"));
    b->cav_size = b->esz == 8 ? sizeof(CavityDev<double>) : sizeof(CavityDev<float>);
    if ((e = hipMalloc(&b->arena, bytes)) != hipSuccess) return fail(record_hip(e, "hipMalloc(arena)"));
    if ((e = hipMemsetAsync(b->arena, 0, bytes, b->stream)) != hipSuccess) return fail(record_hip(e, "memset"));
    if ((e = hipMalloc(&b->thw_real, thw * b->esz)) != hipSuccess) return fail(record_hip(e, "hipMalloc"));
    if ((e = hipMalloc(&b->thw_d, thw * sizeof(double))) != hipSuccess) return fail(record_hip(e, "hipMalloc"));
    if ((e = hipMalloc(&b->cavs, count * b->cav_size)) != hipSuccess) return fail(record_hip(e, "hipMalloc"));
    if ((e = hipMalloc(&b->nu, count * sizeof(double))) != hipSuccess) return fail(record_hip(e, "hipMalloc"));
    if ((e = hipMalloc(&b->flags, count * sizeof(int))) != hipSuccess) return fail(record_hip(e, "hipMalloc"));
    if ((e = hipMalloc(&b->scratch, b->scratch_elems * sizeof(double))) != hipSuccess)
        return fail(record_hip(e, "hipMalloc"));
    int rc;
    if ((rc = upload_hot_walls(b))) return fail(rc);
    if ((rc = upload_cavs(b))) return fail(rc);
    if ((rc = build_tiles(b))) return fail(rc);
    for (int i = 0; i < count; ++i) {
        rc = b->esz == 8 ? init_member_t<double>(b, i, nullptr) : init_member_t<float>(b, i, nullptr);
        if (rc) return fail(rc);
    }
    if ((e = hipStreamSynchronize(b->stream)) != hipSuccess) return fail(record_hip(e, "sync"));
    *out = b;
    return DMRT_OK;
}

int dmrt_batch_set_theta(dmrt_batch* b, int index, const double* theta0)
{
    if (!b || index < 0 || index >= b->count || !theta0) return DMRT_EINVAL;
    const size_t nn = (size_t)b->p[index].n * b->p[index].n;
    if (check_finite(theta0, nn)) return DMRT_EINVAL;
    HIPCHK(hipMemcpyAsync(b->scratch, theta0, nn * sizeof(double), hipMemcpyHostToDevice, b->stream));
    int rc = b->esz == 8 ? init_member_t<double>(b, index, b->scratch)
                         : init_member_t<float>(b, index, b->scratch);
    if (rc) return rc;
    if (b->dead[index]) {
        b->dead[index] = 0;
        if ((rc = upload_cavs(b))) return rc;
    }
    HIPCHK(hipStreamSynchronize(b->stream));
    return DMRT_OK;
}

int dmrt_batch_set_hot_wall(dmrt_batch* b, int index, const double* theta_w)
{
    if (!b || index < 0 || index >= b->count || !theta_w) return DMRT_EINVAL;
    if (check_finite(theta_w, b->p[index].n)) return DMRT_EINVAL;
    HIPCHK(hipStreamSynchronize(b->stream));
    b->thw_host[index].assign(theta_w, theta_w + b->p[index].n);
    return upload_hot_walls(b);
}

int dmrt_batch_set_schedule(dmrt_batch* b, int block_x, int block_y, int order, int grid_blocks,
                            size_t group_bytes, int group_steps)
{
    if (!b) return DMRT_EINVAL;
    if (block_x != 64 && block_x != 128 && block_x != 256 && block_x != 512) return DMRT_EINVAL;
    if (block_y < 1 || block_x * block_y > 1024) return DMRT_EINVAL;
    if (order < 0 || order > 2 || grid_blocks < 0 || group_steps < 1) return DMRT_EINVAL;
    HIPCHK(hipStreamSynchronize(b->stream));
    drop_graphs(b);
    b->block_x = block_x;
    b->block_y = block_y;
    b->order = order;
    b->grid_blocks = grid_blocks;
    b->group_bytes = group_bytes;
    b->group_steps = group_steps;
    return build_tiles(b);
}

int dmrt_batch_set_temporal(dmrt_batch* b, int steps_per_launch, int tile_rows)
{
    if (!b) return DMRT_EINVAL;
    if (!valid_temporal(steps_per_launch, tile_rows)) return DMRT_EINVAL;
    HIPCHK(hipStreamSynchronize(b->stream));
    drop_graphs(b);
    b->temporal = steps_per_launch;
    b->t_rows = tile_rows;
    b->march_B = 0;
    return build_tiles(b);
}

int dmrt_batch_set_temporal_march(dmrt_batch* b, int steps_per_launch, int group_rows, int chunk_rows)
{
    if (!b || chunk_rows < 0) return DMRT_EINVAL;
    if (!valid_march(steps_per_launch, group_rows, (int)b->esz)) return DMRT_EINVAL;
    HIPCHK(hipStreamSynchronize(b->stream));
    drop_graphs(b);
    b->temporal = steps_per_launch;
    b->march_B = group_rows;
    b->march_chunk = chunk_rows;
    return build_tiles(b);
}

int dmrt_batch_step(dmrt_batch* b, long nsteps)
{
    if (!b || nsteps < 0) return DMRT_EINVAL;
    const int G = b->group_steps;
    long left = nsteps;
    if (G >= 2) {
        // whole rounds by graph replay (one graph per starting copy)
        while (left >= G) {
            const int p = b->cur;
            if (!b->graph[p]) {
                int rc = build_graph(b, p);
                if (rc) return rc;
            }
            HIPCHK(hipGraphLaunch(b->graph[p], b->stream));
            b->cur ^= (b->graph_flips[p] & 1);
            b->step += G;
            left -= G;
        }
    }
    while (left > 0) {
        const int k = (int)std::min<long>(left, G);
        int flips = 0;
        int rc = enqueue_round(b, b->stream, b->cur, k, &flips);
        if (rc) return rc;
        if (flips & 1) b->cur ^= 1;
        b->step += k;
        left -= k;
    }
    return DMRT_OK;
}

int dmrt_batch_sync(dmrt_batch* b)
{
    if (!b) return DMRT_EINVAL;
    HIPCHK(hipStreamSynchronize(b->stream));
    return DMRT_OK;
}

int dmrt_batch_nusselt(dmrt_batch* b, double* nu_avg)
{
    if (!b || !nu_avg) return DMRT_EINVAL;
    if (b->esz == 8)
        hipLaunchKernelGGL((batch_nusselt_kernel<double>), dim3(b->count), dim3(256), 0, b->stream,
                           static_cast<const CavityDev<double>*>(b->cavs), b->cur, b->nu);
    else
        hipLaunchKernelGGL((batch_nusselt_kernel<float>), dim3(b->count), dim3(256), 0, b->stream,
                           static_cast<const CavityDev<float>*>(b->cavs), b->cur, b->nu);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(nu_avg, b->nu, b->count * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return DMRT_OK;
}

int dmrt_batch_status(dmrt_batch* b, int* status)
{
    if (!b || !status) return DMRT_EINVAL;
    HIPCHK(hipMemsetAsync(b->flags, 0, b->count * sizeof(int), b->stream));
    const dim3 grid(64, b->count);
    if (b->esz == 8)
        hipLaunchKernelGGL((batch_check_kernel<double>), grid, dim3(256), 0, b->stream,
                           static_cast<const CavityDev<double>*>(b->cavs), b->cur, b->flags);
    else
        hipLaunchKernelGGL((batch_check_kernel<float>), grid, dim3(256), 0, b->stream,
                           static_cast<const CavityDev<float>*>(b->cavs), b->cur, b->flags);
    HIPCHK(hipGetLastError());
    std::vector<int> f(b->count);
    HIPCHK(hipMemcpyAsync(f.data(), b->flags, b->count * sizeof(int), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    bool changed = false;
    for (int i = 0; i < b->count; ++i) {
        if (f[i] && !b->dead[i]) { b->dead[i] = 1; changed = true; }
        status[i] = b->dead[i] ? DMRT_ENONFINITE : DMRT_OK;
    }
    if (changed) return upload_cavs(b);   // dead members are skipped from now on
    return DMRT_OK;
}

int dmrt_batch_get_fields(dmrt_batch* b, int index, double* U, double* V, double* theta, double* P)
{
    if (!b || index < 0 || index >= b->count) return DMRT_EINVAL;
    const int n = b->p[index].n;
    const size_t nn = (size_t)n * n;
    double* s = b->scratch;
    const dim3 block(64, 4), grid((n + 63) / 64, (n + 3) / 4);
    const double gy0 = -b->d[index].gbeta * b->p[index].theta_ref;
    if (b->esz == 8) {
        const CavityDev<double> c = make_cav<double>(b, index);
        hipLaunchKernelGGL((fields_kernel<double>), grid, block, 0, b->stream, c.f[b->cur], c.g[b->cur],
                           n, c.pitch, c.plane, b->d[index].gbeta, gy0, b->p[index].force_x,
                           s, s + nn, s + 2 * nn, s + 3 * nn);
    } else {
        const CavityDev<float> c = make_cav<float>(b, index);
        hipLaunchKernelGGL((fields_kernel<float>), grid, block, 0, b->stream, c.f[b->cur], c.g[b->cur],
                           n, c.pitch, c.plane, (double)(float)b->d[index].gbeta, (double)(float)gy0,
                           (double)(float)b->p[index].force_x, s, s + nn, s + 2 * nn, s + 3 * nn);
    }
    HIPCHK(hipGetLastError());
    double* outs[4] = {U, V, theta, P};
    for (int i = 0; i < 4; ++i)
        if (outs[i])
            HIPCHK(hipMemcpyAsync(outs[i], s + i * nn, nn * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return DMRT_OK;
}

int dmrt_batch_member_state(dmrt_batch* b, int index, void* host_f, void* host_g)
{
    if (!b || index < 0 || index >= b->count) return DMRT_EINVAL;
    const int n = b->p[index].n, pitch = pitch_of(n);
    const size_t plane = (size_t)n * pitch, row = (size_t)n * b->esz;
    char* base = static_cast<char*>(b->arena) + b->off[index];
    char* fb = base + (size_t)b->cur * 9 * plane * b->esz;
    char* gb = base + (18 + (size_t)b->cur * 5) * plane * b->esz;
    if (host_f)
        HIPCHK(hipMemcpy2DAsync(host_f, row, fb, pitch * b->esz, row, (size_t)9 * n,
                                hipMemcpyDeviceToHost, b->stream));
    if (host_g)
        HIPCHK(hipMemcpy2DAsync(host_g, row, gb, pitch * b->esz, row, (size_t)5 * n,
                                hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return DMRT_OK;
}

int dmrt_batch_load_member_state(dmrt_batch* b, int index, const void* host_f, const void* host_g)
{
    if (!b || index < 0 || index >= b->count || !host_f || !host_g) return DMRT_EINVAL;
    const int n = b->p[index].n, pitch = pitch_of(n);
    const size_t plane = (size_t)n * pitch, row = (size_t)n * b->esz;
    char* base = static_cast<char*>(b->arena) + b->off[index];
    char* fb = base + (size_t)b->cur * 9 * plane * b->esz;
    char* gb = base + (18 + (size_t)b->cur * 5) * plane * b->esz;
    HIPCHK(hipMemcpy2DAsync(fb, pitch * b->esz, host_f, row, row, (size_t)9 * n,
                            hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipMemcpy2DAsync(gb, pitch * b->esz, host_g, row, row, (size_t)5 * n,
                            hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    if (b->dead[index]) {
        b->dead[index] = 0;
        return upload_cavs(b);
    }
    return DMRT_OK;
}

int dmrt_batch_get_step(dmrt_batch* b, long* step)
{
    if (!b || !step) return DMRT_EINVAL;
    *step = b->step;
    return DMRT_OK;
}

int dmrt_batch_destroy(dmrt_batch* b)
{
    if (!b) return DMRT_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    void* ptrs[] = {b->arena, b->thw_real, b->thw_d, b->cavs, b->tiles, b->foot_tiles, b->march_tiles,
                    b->nu, b->flags, b->scratch};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return DMRT_OK;
}

}  // extern "C"
