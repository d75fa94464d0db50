// Random walks on the graphs (Sec. 2, spectral dimension; App. A): the
// histogram of the times at which a walker is back at its starting site
// estimates P(tau) ~ tau^(-dbar/2).  All graphs in one launch.  A step loads
// the site's 16-byte record and a second, dependent neighbour index only when
// the chosen neighbour is not in the record (one scattered line per step
// instead of two for most steps): degree and the offset of the rest packed in
// one word with the first three neighbours when every graph has fewer than
// 2^24 - 3 neighbour entries, else degree, first two neighbours and offset.
// One Philox4x32-10 call serves four steps.
// The per-block histogram lives in LDS (walks up to 8191 steps; longer ones
// count in global memory) and is added to the caller's histogram with 64-bit
// integer atomics, so the result does not depend on the order in which
// walkers finish.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "xy_internal.hpp"

namespace xy {
namespace {

struct WalkDesc {
    int64_t od;        // int4 pool per site: the record (see k_walk)
    int64_t nbr;       // int32 pool: neighbours, ascending lattice index per site
    int64_t elig;      // int32 pool: sites of degree > 2, ascending
    int32_t n, n_elig, centre, pad_;
    uint32_t seed_lo, seed_hi;
};

constexpr int kWalkBlock = 256;
constexpr int kWalkers = 1;             // walkers per thread
constexpr int kWalkLdsBins = 8192;      // steps + 1 up to this: LDS histogram (dynamic, 4 B a bin)

// Each XCD takes one contiguous run of the (graph, block) units (the
// hardware deals workgroup w to XCD w mod 8), so an XCD's L2 holds the few
// graphs its walkers visit.  A bijection on [0, n).
__device__ __forceinline__ int xcd_run(int lin, int n)
{
    const int x = lin & 7, k = lin >> 3, per = n >> 3, rem = n & 7;
    return x * per + min(x, rem) + k;
}

// One thread runs kW walkers in lock step (their loads overlap).  Record of a
// site: kPacked: (degree | offset of neighbour 3 << 8, n0, n1, n2); else
// (degree, n0, n1, offset of neighbour 2).
template <bool kLds, int kW, bool kPacked>
__global__ __launch_bounds__(kWalkBlock) void k_walk(const WalkDesc *desc, const int4 *od_pool, const int32_t *i32,
                                                    int n_walkers, int n_steps, int start_mode, int blocks_per_graph,
                                                    unsigned long long *hist)
{
    extern __shared__ uint32_t lds[];   // n_steps + 1 bins when kLds
    const int unit = xcd_run(blockIdx.x, gridDim.x);
    const int gi = unit / blocks_per_graph, bx = unit % blocks_per_graph;
    const WalkDesc d = desc[gi];
    unsigned long long *h = hist + (int64_t)gi * (n_steps + 1);
    if constexpr (kLds) {
        for (int t = threadIdx.x; t <= n_steps; t += kWalkBlock) lds[t] = 0u;
        __syncthreads();
    }
    const int4 *od = od_pool + d.od;
    const int32_t *nbr = i32 + d.nbr;
    int w[kW], s0[kW], cur[kW];
    bool live[kW];
#pragma unroll
    for (int a = 0; a < kW; ++a) {
        w[a] = (bx * kW + a) * kWalkBlock + threadIdx.x;
        live[a] = w[a] < n_walkers;
        s0[a] = d.centre;
        if (live[a] && start_mode == 1) {
            const U4 x = philox4x32_10({(uint32_t)w[a], 0u, 0u, (uint32_t)kWalkStart << 24}, d.seed_lo, d.seed_hi);
            s0[a] = i32[d.elig + (int)(((uint64_t)x.x * (uint32_t)d.n_elig) >> 32)];
        }
        cur[a] = s0[a];
    }
    U4 x[kW];
    for (int t = 0; t < n_steps; ++t) {
#pragma unroll
        for (int a = 0; a < kW; ++a) {
            if ((t & 3) == 0)
                x[a] = philox4x32_10({(uint32_t)w[a], (uint32_t)(t >> 2), 0u, (uint32_t)kWalk << 24}, d.seed_lo,
                                     d.seed_hi);
        }
        int4 e[kW];
#pragma unroll
        for (int a = 0; a < kW; ++a) e[a] = od[cur[a]];
#pragma unroll
        for (int a = 0; a < kW; ++a) {
            const uint32_t r = (t & 3) == 0 ? x[a].x : (t & 3) == 1 ? x[a].y : (t & 3) == 2 ? x[a].z : x[a].w;
            const uint32_t dg = kPacked ? ((uint32_t)e[a].x & 255u) : (uint32_t)e[a].x;
            const int j = (int)(((uint64_t)r * dg) >> 32);               // neighbour number, < degree
            if (dg > 0) {
                if constexpr (kPacked)
                    cur[a] = j == 0 ? e[a].y : j == 1 ? e[a].z : j == 2 ? e[a].w
                                                                         : nbr[((uint32_t)e[a].x >> 8) + j - 3];
                else
                    cur[a] = j == 0 ? e[a].y : j == 1 ? e[a].z : nbr[e[a].w + j - 2];
            }
        }
        // walkers at their start: counted per wave (one atomic per wave and
        // step instead of one per walker, which all hit the same bin)
        uint32_t n_at = 0;
#pragma unroll
        for (int a = 0; a < kW; ++a) n_at += (uint32_t)__popcll(__ballot(live[a] && cur[a] == s0[a]));
        if (n_at && __lane_id() == 0) {
            if constexpr (kLds) atomicAdd(&lds[t + 1], n_at); else atomicAdd(&h[t + 1], (unsigned long long)n_at);
        }
    }
    if constexpr (kLds) {
        __syncthreads();
        for (int t = threadIdx.x + 1; t <= n_steps; t += kWalkBlock)
            if (lds[t]) atomicAdd(&h[t], (unsigned long long)lds[t]);
    }
}

// The histograms before the walks: every walker is at its start at t = 0.
__global__ void k_walk_hist_init(unsigned long long *p, int64_t n, int bins, int n_walkers)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (i % bins) == 0 ? (unsigned long long)n_walkers : 0ull;
}

struct WalkPlan {
    std::vector<WalkDesc> desc;
    size_t n_od = 0, n_i32 = 0;
    size_t off_desc = 0, off_od = 0, off_i32 = 0, total = 0;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

xy_status plan_walk(const xy_graph *const *g, int G, WalkPlan &p)
{
    if (!g || G < 1 || G > 65535) return set_error(XY_EINVAL, "walk: need 1 to 65535 graphs");
    p.desc.assign(G, WalkDesc{});
    for (int k = 0; k < G; ++k) {
        if (!g[k]) return set_error(XY_EINVAL, "walk: NULL graph");
        const xy_graph &gr = *g[k];
        WalkDesc &d = p.desc[k];
        d.n = gr.n;
        d.od = (int64_t)p.n_od;     p.n_od += gr.n;
        d.nbr = (int64_t)p.n_i32;   p.n_i32 += 2 * (size_t)gr.m;
        d.elig = (int64_t)p.n_i32;  p.n_i32 += gr.n;
    }
    p.off_desc = 0;
    p.off_od = align256(sizeof(WalkDesc) * G);
    p.off_i32 = align256(p.off_od + 16 * p.n_od);
    p.total = align256(p.off_i32 + 4 * p.n_i32);
    return XY_OK;
}

}  // namespace
}  // namespace xy

using namespace xy;

extern "C" xy_status xy_walk_bytes(const xy_graph *const *g, int n_graphs, size_t *graph_bytes)
{
    if (!graph_bytes) return set_error(XY_EINVAL, "xy_walk_bytes: graph_bytes is NULL");
    WalkPlan p;
    const xy_status st = plan_walk(g, n_graphs, p);
    if (st != XY_OK) return st;
    *graph_bytes = p.total;
    return XY_OK;
}

// Workspace of xy_random_walk_noalloc: the walk records of its graphs.  Each
// device holds its own copy from the library's load to the end of the
// process; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (kept per device).
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// The walk: stages the graphs' walk records from a host image into d_graph
// (at least p.total bytes, 256-byte aligned), then runs the walks.
xy_status walk_run(const xy_graph *const *g, int n_graphs, int n_walkers, int n_steps, const uint64_t *seeds,
                   int start_mode, const WalkPlan &plan, void *d_graph, uint64_t *d_hist, void *stream,
                   float *kernel_ms)
{
    try {
        WalkPlan p = plan;
        std::vector<unsigned char> img(p.total, 0);
        int4 *od = reinterpret_cast<int4 *>(img.data() + p.off_od);
        int32_t *i32 = reinterpret_cast<int32_t *>(img.data() + p.off_i32);
        std::vector<int32_t> deg, fill;
        // packed records when every graph's neighbour list (offset of neighbour 3 included) fits 24 bits;
        // degrees are below 256 for every graph the library builds
        // (XY_WALK_PACKED=0 forces the other form; tests compare both)
        bool packed = true;
        if (const char *env = std::getenv("XY_WALK_PACKED")) packed = std::atoi(env) != 0;
        for (int k = 0; k < n_graphs; ++k) packed = packed && 2 * (int64_t)g[k]->m + 3 < (int64_t)1 << 24;
        for (int k = 0; k < n_graphs; ++k) {
            const xy_graph &gr = *g[k];
            WalkDesc &d = p.desc[k];
            const int n = gr.n;
            deg.assign(n, 0);
            for (int e = 0; e < gr.m; ++e) { ++deg[gr.edges[2 * e]]; ++deg[gr.edges[2 * e + 1]]; }
            std::vector<int32_t> first(n);
            int32_t acc = 0;
            for (int i = 0; i < n; ++i) { first[i] = acc; acc += deg[i]; }
            int32_t *nb = i32 + d.nbr;
            fill.assign(n, 0);
            for (int e = 0; e < gr.m; ++e) {
                const int a = gr.edges[2 * e], b = gr.edges[2 * e + 1];
                nb[first[a] + fill[a]++] = b;
                nb[first[b] + fill[b]++] = a;
            }
            // neighbours in ascending lattice index; the record holds the first
            // ones and the offset in nb of the rest
            for (int i = 0; i < n; ++i) {
                std::sort(nb + first[i], nb + first[i] + deg[i]);
                const int32_t *f = nb + first[i];
                if (packed)
                    od[d.od + i] = make_int4((int32_t)((uint32_t)deg[i] | ((uint32_t)(first[i] + 3) << 8)),
                                             deg[i] > 0 ? f[0] : 0, deg[i] > 1 ? f[1] : 0, deg[i] > 2 ? f[2] : 0);
                else
                    od[d.od + i] = make_int4(deg[i], deg[i] > 0 ? f[0] : 0, deg[i] > 1 ? f[1] : 0, first[i] + 2);
            }
            int n_elig = 0;
            for (int i = 0; i < n; ++i)
                if (deg[i] > 2) i32[d.elig + n_elig++] = i;
            d.n_elig = n_elig;
            if (start_mode == 1 && n_elig == 0)
                return set_error(XY_EUNSUP, "xy_random_walk: a graph has no site of degree > 2");
            if (start_mode == 0) {
                if (gr.L < 2 || gr.L * gr.L != n) return set_error(XY_EINVAL, "xy_random_walk: centre start needs an L x L graph");
                d.centre = (gr.L / 2) * gr.L + gr.L / 2;
            }
            d.seed_lo = (uint32_t)seeds[k];
            d.seed_hi = (uint32_t)(seeds[k] >> 32);
        }
        std::memcpy(img.data() + p.off_desc, p.desc.data(), sizeof(WalkDesc) * n_graphs);
        hipStream_t s = static_cast<hipStream_t>(stream);
        hipError_t e = hipMemcpyAsync(d_graph, img.data(), p.total, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        const int64_t n_hist = (int64_t)n_graphs * (n_steps + 1);
        auto *h = reinterpret_cast<unsigned long long *>(d_hist);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_walk_hist_init, dim3((unsigned)((n_hist + 255) / 256)), dim3(256), 0, s, h, n_hist,
                               n_steps + 1, n_walkers);
            e = hipGetLastError();
        }
        hipEvent_t ev[2] = {nullptr, nullptr};
        if (e == hipSuccess && kernel_ms) {
            *kernel_ms = 0.f;
            e = hipEventCreateWithFlags(&ev[0], hipEventDisableSystemFence);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ev[1], hipEventDisableSystemFence);
            if (e == hipSuccess) e = hipEventRecord(ev[0], s);
        }
        if (e == hipSuccess && n_walkers > 0) {
            unsigned char *base = static_cast<unsigned char *>(d_graph);
            const auto *dd = reinterpret_cast<const WalkDesc *>(base + p.off_desc);
            const auto *dod = reinterpret_cast<const int4 *>(base + p.off_od);
            const auto *di = reinterpret_cast<const int32_t *>(base + p.off_i32);
            // kWalkers walkers per thread; one flat grid of (graph, block) units
            const int64_t per = (n_walkers + kWalkBlock * kWalkers - 1) / (kWalkBlock * kWalkers);
            const int64_t units = per * n_graphs;
            if (units > 0x7fffffff) return set_error(XY_EINVAL, "xy_random_walk: too many walkers");
            const bool lds = n_steps + 1 <= kWalkLdsBins;
            const size_t lds_bytes = lds ? 4 * (size_t)(n_steps + 1) : 0;
            auto kern = lds ? (packed ? k_walk<true, kWalkers, true> : k_walk<true, kWalkers, false>)
                            : (packed ? k_walk<false, kWalkers, true> : k_walk<false, kWalkers, false>);
            hipLaunchKernelGGL(kern, dim3((unsigned)units), dim3(kWalkBlock), lds_bytes, s, dd, dod, di, n_walkers,
                               n_steps, start_mode, (int)per, h);
            e = hipGetLastError();
        }
        if (e == hipSuccess && kernel_ms) {
            e = hipEventRecord(ev[1], s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e == hipSuccess) e = hipEventElapsedTime(kernel_ms, ev[0], ev[1]);
        }
        for (hipEvent_t x : ev)
            if (x) (void)hipEventDestroy(x);
        if (e != hipSuccess) return set_error(XY_EHIP, std::string("xy_random_walk: ") + hipGetErrorString(e));
        return XY_OK;
    } catch (const std::bad_alloc &) {
        return set_error(XY_ENOMEM, "xy_random_walk: host allocation failed");
    }
}

xy_status walk_args(int n_walkers, int n_steps, const uint64_t *seeds, int start_mode, const uint64_t *d_hist)
{
    if (n_walkers < 0 || n_steps < 0 || n_steps >= (1 << 24) || !seeds || !d_hist ||
        (start_mode != 0 && start_mode != 1))
        return set_error(XY_EINVAL, "xy_random_walk: bad arguments");
    return XY_OK;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on the current device (looked up on the first call
// on that device, with it current).
hipError_t scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255) != 0) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" xy_status xy_random_walk(const xy_graph *const *g, int n_graphs, int n_walkers, int n_steps,
                                    const uint64_t *seeds, int start_mode, void *d_graph, size_t graph_bytes,
                                    uint64_t *d_hist, void *stream, float *kernel_ms)
{
    xy_status st = walk_args(n_walkers, n_steps, seeds, start_mode, d_hist);
    if (st != XY_OK) return st;
    if (!d_graph) return set_error(XY_EINVAL, "xy_random_walk: bad arguments");
    if ((reinterpret_cast<uintptr_t>(d_graph) & 255) != 0)
        return set_error(XY_EINVAL, "xy_random_walk: d_graph must be 256-byte aligned");
    WalkPlan p;
    st = plan_walk(g, n_graphs, p);
    if (st != XY_OK) return st;
    if (graph_bytes < p.total) return set_error(XY_EINVAL, "xy_random_walk: d_graph smaller than xy_walk_bytes");
    return walk_run(g, n_graphs, n_walkers, n_steps, seeds, start_mode, p, d_graph, d_hist, stream, kernel_ms);
}

extern "C" xy_status xy_random_walk_noalloc(const xy_graph *const *g, int n_graphs, int n_walkers, int n_steps,
                                            const uint64_t *seeds, int start_mode, uint64_t *d_hist, void *stream,
                                            float *kernel_ms)
{
    xy_status st = walk_args(n_walkers, n_steps, seeds, start_mode, d_hist);
    if (st != XY_OK) return st;
    WalkPlan p;
    st = plan_walk(g, n_graphs, p);
    if (st != XY_OK) return st;
    if (p.total > kScratchBytes)
        return set_error(XY_EINVAL, "xy_random_walk_noalloc: the walk graphs need " + std::to_string(p.total) +
                                        " bytes, more than the " + std::to_string(kScratchBytes) +
                                        "-byte static workspace (use xy_random_walk)");
    void *ws = nullptr;
    const hipError_t e = scratch_address(&ws);
    if (e != hipSuccess)
        return set_error(XY_EHIP, std::string("xy_random_walk_noalloc: workspace address: ") + hipGetErrorString(e));
    return walk_run(g, n_graphs, n_walkers, n_steps, seeds, start_mode, p, ws, d_hist, stream, kernel_ms);
}
