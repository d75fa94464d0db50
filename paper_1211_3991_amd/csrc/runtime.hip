// Batch runtime: device layout, uploads, the sweep schedule and the C ABI
// entry points of include/xy_levy.h that touch the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "kernels.hpp"

using namespace xy;

struct xy_batch {
    int G = 0, R = 0, precision = 0, max_records = 0, max_n = 0, Qmax = 0;
    std::vector<int> max_class;               // per colour, over samples
    std::vector<std::vector<int32_t>> perm;   // per sample: colour-major -> lattice
    std::vector<int> n;                       // per sample
    std::vector<int64_t> state_off;           // per sample, elements
    size_t state_bytes = 0;
    void *d_state = nullptr, *d_graph = nullptr, *d_work = nullptr, *d_obs = nullptr;
    DevBatch dev{};
    WorkLayout wl{};
    // fix16 launch groups: (storage mode, block size) with their work items
    struct Group { int mode, block, n_items; size_t lds; Item *items; };
    std::vector<Group> groups;
    std::vector<SampleDesc> desc_host;        // fix16: for regrouping
    // fix16 phase form (site-major samples, one launch per colour phase)
    int n_phase = 0;
    int32_t *d_phase = nullptr;
    std::vector<int> phase_units;             // per colour: work units of its launch
    std::vector<size_t> phase_unit_off;       // per colour: first int4 of its units in d_units
    int4 *d_units = nullptr;                  // two int4 per unit (see k_fix16_phase)
    int phase_stride = 0;                     // largest block count (energy partial stride)
    bool serpentine = true;                   // alternate the unit order of consecutive colour phases
    // the phase launches of a sweep split by sample over the caller's stream
    // and `aux`, so that the ramp and tail of one launch overlap the other
    // stream's work; fork and join through events on the caller's stream
    std::vector<hipStream_t> aux;             // groups 1.. (group 0 runs on the caller's stream)
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;          // per auxiliary stream
    std::vector<int> phase_bounds;            // [colour][group + 1]: first unit of each group
    std::vector<int> group_first;             // [group + 1]: first phase sample of each group
    // independent groups only: n_slices groups per stream, run one after the
    // other (group g on stream g % n_streams, in slice g / n_streams), so that
    // only one slice's samples are swept at a time
    int n_slices = 1;
    std::vector<int32_t> unit_k;              // phase index of each work unit, in d_units order
    // every sample in the phase form: each group also runs its own energies,
    // tempering and records with its own control block b.ctl[g], so the
    // groups fork once per xy_sweep call and join at its end
    bool indep = false;
    std::vector<int> event_sweeps;            // sweeps covered by each timing event pair
    size_t item_cap = 0;
    Item *d_items = nullptr;
    int lds_limit = 0;
    uint32_t host_sweep = 0;
    // HIP graph replay of `chunk` sweeps of one shape
    int chunk = 0;
    hipGraphExec_t gexec = nullptr;
    hipStream_t gstream = nullptr;
    int g_n_or = -1, g_pt = -1, g_meas = -1;
    uint64_t g_phase = 0;   // host_sweep modulo the pattern period at capture time
    uint64_t g_period = 0;  // period of the tempering / record pattern of the captured chunk
    // temperature ladder by temperature index: host copy of the last upload
    double *d_beta = nullptr;
    std::vector<double> beta_host;
    hipEvent_t ev_beta = nullptr;   // the last ladder upload (the host copy may be reused after it)
    // kernel timing (event pairs around the dominant kernel of each sweep)
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    size_t events_used = 0;
    hipStream_t timed_stream = nullptr;
};

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

constexpr int kGroups = 4;   // fix16 launch groups
// (storage mode, block size): unit vectors in LDS with 256 threads (graphs of
// at most 4096 sites) or 1024, angles in LDS, angles in global memory with 512
// threads (several workgroups per CU hide the latency of the gathers)
constexpr int kGroupMode[kGroups] = {2, 2, 0, 1};
constexpr int kGroupBlock[kGroups] = {256, 1024, 1024, 512};

xy_status hip_err(hipError_t e, const char *where)
{
    return set_error(XY_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Splits the phase samples into n_streams x n_slices contiguous groups of
// about equal work units, group g on stream g % n_streams (stream 0 the
// caller's, the others auxiliary streams created here; the previous ones are
// released); no work may be in flight on them.  Slices apply to independent
// groups only (every sample in the phase form); otherwise n_slices is 1.
hipError_t setup_phase_groups(xy_batch *b, int n_streams, int n_slices)
{
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    for (hipEvent_t ev : b->ev_join) (void)hipEventDestroy(ev);
    for (hipStream_t st : b->aux) (void)hipStreamDestroy(st);
    b->ev_fork = nullptr;
    b->ev_join.clear();
    b->aux.clear();
    const int n_ph = b->n_phase, Q = (int)b->phase_units.size();
    n_streams = std::max(1, std::min({n_streams, kMaxPhaseStreams, std::max(n_ph, 1)}));
    n_slices = (n_ph == b->G) ? std::max(1, std::min(n_slices, std::min(kMaxPhaseGroups, n_ph) / n_streams)) : 1;
    const int n_groups = n_streams * n_slices;
    std::vector<int> first(n_groups + 1, n_ph);    // group g: phase samples [first[g], first[g+1])
    first[0] = 0;
    std::vector<size_t> per(std::max(n_ph, 1), 0);
    for (int32_t k : b->unit_k) ++per[k];
    size_t total = 0, acc = 0;
    for (size_t v : per) total += v;
    int g = 1;
    for (int k = 0; k < n_ph && g < n_groups; ++k) {
        acc += per[k];
        // close group g-1 after sample k once it holds its share, leaving a
        // sample for each later group
        if (acc * n_groups >= total * g && n_ph - (k + 1) >= n_groups - g) first[g++] = k + 1;
    }
    for (; g < n_groups; ++g) first[g] = std::min(n_ph, first[g - 1] + 1);
    b->phase_bounds.assign((size_t)Q * (n_groups + 1), 0);
    for (int c = 0; c < Q; ++c) {
        int *bd = b->phase_bounds.data() + (size_t)c * (n_groups + 1);
        const int32_t *uk = b->unit_k.data() + b->phase_unit_off[c] / 2;
        for (int h = 0; h <= n_groups; ++h) {
            int n = 0;   // units of colour c whose sample precedes group h
            for (int a = 0; a < b->phase_units[c]; ++a) n += uk[a] < first[h];
            bd[h] = n;
        }
    }
    b->group_first = first;
    b->n_slices = n_slices;
    b->indep = n_groups > 1 && n_ph == b->G;
    hipError_t e = hipSuccess;
    if (n_streams > 1) {
        e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
        for (int h = 1; h < n_streams && e == hipSuccess; ++h) {
            hipStream_t st = nullptr;
            hipEvent_t ev = nullptr;
            e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
            if (e == hipSuccess) b->aux.push_back(st);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) b->ev_join.push_back(ev);
        }
    }
    return e;
}

struct Plan {
    GraphLayout gl{};
    WorkLayout wl{};
    size_t state_bytes = 0, obs_bytes = 0;
    std::vector<SampleDesc> desc;
    int max_n = 0, Qmax = 0;
    std::vector<int64_t> state_off;
    size_t item_cap = 0;
    std::vector<Sell> sell;      // fix16 only
    bool idx16 = false;
    int phase_blocks = 0;        // largest phase-form block count of any colour
    size_t phase_units = 0;      // phase-form blocks over all colours and samples
};

xy_status plan_batch(const xy_graph *const *g, int G, int R, int precision, int max_records, Plan &p)
{
    if (!g || G < 1) return set_error(XY_EINVAL, "batch: need at least one graph");
    if (R < 1 || R > kMaxT) return set_error(XY_EINVAL, "batch: n_T must be in [1, 256]");
    if (precision != XY_FP64 && precision != XY_FIX16) return set_error(XY_EINVAL, "batch: unknown precision");
    if (max_records < 0) return set_error(XY_EINVAL, "batch: max_records < 0");
    p.desc.assign(G, SampleDesc{});
    p.state_off.assign(G, 0);
    size_t n_i32 = 0, n_u32 = 0, n_f64 = 0, n_u16 = 0, n_u8 = 0, state_elems = 0;
    const bool fix16 = precision == XY_FIX16;
    int max_n = 0;
    for (int s = 0; s < G; ++s) {
        if (!g[s]) return set_error(XY_EINVAL, "batch: NULL graph");
        max_n = std::max(max_n, g[s]->n);
    }
    p.idx16 = fix16 && max_n <= 65536;
    if (fix16) p.sell.resize(G);
    // fix16 storage of a sample: the site-major phase form (one launch per
    // colour phase for all such samples, four slots per thread) for graphs of
    // at least XY_FIX16_PHASE_MIN sites (default 16384) when n_T is a multiple
    // of 4; below that a workgroup per replica with the replica in LDS wins.
    // XY_FIX16_PHASE=1 / 0 puts every sample in / out of it.
    int phase_mode = -1;
    if (const char *env = std::getenv("XY_FIX16_PHASE"))
        if (*env) phase_mode = std::atoi(env) != 0 ? 1 : 0;
    int phase_min = 16384;
    if (const char *env = std::getenv("XY_FIX16_PHASE_MIN"))
        if (*env) phase_min = std::atoi(env);
    int n_phase = 0, phase_blocks = 0;
    for (int s = 0; s < G; ++s) {
        const xy_graph &gr = *g[s];
        SampleDesc &d = p.desc[s];
        d.n = gr.n; d.Q = gr.Q; d.L = gr.L; d.max_deg = gr.max_deg;
        const bool phase = fix16 && R % 4 == 0 && (phase_mode == 1 || (phase_mode < 0 && gr.n >= phase_min));
        if (!fix16) {
            d.row_ptr = (int64_t)n_i32; n_i32 += gr.n + 1;
            d.col = (int64_t)n_i32;     n_i32 += 2 * (size_t)gr.m;
        } else {
            // phase-form samples take their own degree-sort window
            // (XY_SELL_WINDOW overrides it): their gathers come from global memory
            int window = phase ? kPhaseSellWindow : sell_window(gr.n);
            if (phase)
                if (const char *env = std::getenv("XY_SELL_WINDOW"))
                    if (*env && std::atoi(env) > 0) window = std::atoi(env);
            p.sell[s] = build_sell(gr, window);
            const Sell &S = p.sell[s];
            d.sell_ptr = (int64_t)n_i32; n_i32 += S.chunk_ptr.size();
            d.sell_w = (int64_t)n_i32;   n_i32 += S.chunk_w.size();
            if (p.idx16) { d.sell_col = (int64_t)n_u16; n_u16 += align_up(S.col.size(), 8); }
            else         { d.sell_col = (int64_t)n_i32; n_i32 += S.col.size(); }
            d.deg = (int64_t)n_u8;      n_u8 += align_up(gr.n, 16);
            for (int c = 0; c <= kMaxColours; ++c) d.chunk_off[c] = S.chunk_off[std::min(c, gr.Q)];
        }
        d.perm = (int64_t)n_i32;    n_i32 += gr.n;
        n_i32 = align_up(n_i32, 4);
        d.coord = (int64_t)n_u32;   n_u32 += align_up(gr.n, 4);
        d.trig = (int64_t)n_f64;    n_f64 += gr.L;
        for (int c = 0; c <= kMaxColours; ++c) d.colour_off[c] = gr.colour_off[std::min(c, gr.Q)];
        d.layout = phase ? 1 : 0;
        n_phase += d.layout;
        if (d.layout) {
            const int spb = fix16_phase_sites_per_block(R);
            for (int c = 0; c < gr.Q; ++c) {
                const int nb = (gr.colour_off[c + 1] - gr.colour_off[c] + spb - 1) / spb;
                phase_blocks = std::max(phase_blocks, nb);
                p.phase_units += nb;
            }
        }
        d.state = (int64_t)state_elems;
        p.state_off[s] = d.state;
        state_elems += fix16 ? (size_t)((gr.n + 7) & ~7) * R : (size_t)gr.n * R;
        p.max_n = std::max(p.max_n, gr.n);
        p.Qmax = std::max(p.Qmax, gr.Q);
    }
    p.item_cap = 8 * (size_t)G * R + 8;   // XCD interleave pads short queues (per launch group)
    GraphLayout &gl = p.gl;
    size_t off = 0;
    gl.desc = off;      off = align_up(off + sizeof(SampleDesc) * G, 256);
    gl.i32_pool = off;  off = align_up(off + 4 * n_i32, 256);
    gl.u32_pool = off;  off = align_up(off + 4 * n_u32, 256);
    gl.f64_pool = off;  off = align_up(off + 16 * n_f64, 256);
    gl.u16_pool = off;  off = align_up(off + 2 * n_u16, 256);
    gl.u8_pool = off;   off = align_up(off + n_u8, 256);
    gl.items = off;     off = align_up(off + kGroups * sizeof(Item) * p.item_cap, 256);
    // phase-form sample list, then per colour the (sample, block) work units
    gl.phase = off;     off = align_up(off + align_up(4 * (size_t)G, 16) + 32 * p.phase_units, 256);
    gl.tab32 = off;     off = align_up(off + 512 * 8, 256);
    gl.tab2k = off;     off = align_up(off + 2048 * 8, 256);
    gl.tab64 = off;     off = align_up(off + 512 * 16, 256);
    gl.total = off;
    gl.n_i32 = n_i32; gl.n_u32 = n_u32; gl.n_f64 = n_f64; gl.n_u16 = n_u16; gl.n_u8 = n_u8;
    WorkLayout &wl = p.wl;
    const size_t GR = (size_t)G * R;
    off = 0;
    wl.ctl = off;       off = align_up(off + sizeof(Ctl) * kMaxPhaseGroups, 256);
    wl.beta = off;      off = align_up(off + 8 * GR, 256);
    wl.slot_of_T = off; off = align_up(off + 4 * GR, 256);
    wl.T_of_slot = off; off = align_up(off + 4 * GR, 256);
    wl.fac_slot = off;  off = align_up(off + 4 * GR, 256);
    wl.E_slot = off;    off = align_up(off + 8 * GR, 256);
    wl.obs_slot = off;  off = align_up(off + 8 * XY_NOBS * GR, 256);
    wl.pt_acc = off;    off = align_up(off + 8 * GR, 256);
    wl.pt_try = off;    off = align_up(off + 8 * GR, 256);
    wl.partial = off;   off = align_up(off + ((fix16 && n_phase == 0) ? 0 : 8 * 64 * 11 * GR), 256);
    // FP64: the energy partials of the last sub-sweep, [G][Qmax][blocks][R]
    int fp64_blocks = 0;
    if (!fix16)
        for (int s = 0; s < G; ++s)
            for (int c = 0; c < g[s]->Q; ++c)
                fp64_blocks = std::max(fp64_blocks, fp64_phase_blocks(g[s]->colour_off[c + 1] - g[s]->colour_off[c], R));
    wl.epart = off;
    off = align_up(off + (fix16 ? 8 * (size_t)n_phase * kMaxColours * phase_blocks * R
                                : 8 * (size_t)G * p.Qmax * fp64_blocks * R), 256);
    p.phase_blocks = fix16 ? phase_blocks : fp64_blocks;
    wl.total = off;
    p.state_bytes = align_up(state_elems * (precision == XY_FP64 ? 16 : 2), 256);
    p.obs_bytes = align_up((size_t)max_records * GR * XY_NOBS * 8, 256);
    return XY_OK;
}

// Items of the fix16 sweep, ordered so that blockIdx b runs on XCD b % 8 and
// all slots of one sample run on one XCD (they share its CSR in that L2).
// Samples go to the least-loaded XCD in order of decreasing work.
std::vector<Item> xcd_order(const std::vector<int> &samples, const std::vector<SampleDesc> &desc, int R)
{
    constexpr int kXcd = 8;
    std::vector<int> order(samples);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return desc[a].n > desc[b].n; });
    if (order.size() < (size_t)kXcd) {   // too few samples to spread: plain order
        std::vector<Item> out;
        for (int s : order)
            for (int r = 0; r < R; ++r) out.push_back({s, r});
        return out;
    }
    std::vector<std::vector<Item>> q(kXcd);
    std::vector<double> load(kXcd, 0.0);
    for (int s : order) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        for (int r = 0; r < R; ++r) q[x].push_back({s, r});
        load[x] += (double)desc[s].n * R;
    }
    size_t longest = 0;
    for (auto &v : q) longest = std::max(longest, v.size());
    std::vector<Item> out;
    for (size_t r = 0; r < longest; ++r)
        for (int x = 0; x < kXcd; ++x) out.push_back(r < q[x].size() ? q[x][r] : Item{-1, -1});
    while (!out.empty() && out.back().sample < 0) out.pop_back();
    return out;
}

// Splits the samples of a fix16 batch into launch groups by the storage form
// that fits: unit vectors in LDS (block 256 up to 4096 sites, else 1024),
// angles in LDS, angles in global memory; writes each group's XCD-ordered
// items at items + k * item_cap.  Returns false if a list overflows.
bool build_groups(xy_batch *b, int trig, bool allow_unit, bool force_global, Item *items)
{
    const int G = b->G, R = b->R;
    const size_t limit = force_global ? 0 : (size_t)b->lds_limit;
    std::vector<std::vector<int>> members(kGroups);
    std::vector<size_t> lds_need(kGroups, 0);
    for (int s_ = 0; s_ < G; ++s_) {
        if (b->desc_host[s_].layout) continue;          // phase form
        const int n_pad = (b->desc_host[s_].n + 7) & ~7;
        int grp;
        if (allow_unit && fix16_lds_bytes(n_pad, trig, 2) <= limit)
            grp = b->desc_host[s_].n <= 4096 ? 0 : 1;
        else if (fix16_lds_bytes(n_pad, trig, 0) <= limit)
            grp = 2;
        else
            grp = 3;
        members[grp].push_back(s_);
        lds_need[grp] = std::max(lds_need[grp], fix16_lds_bytes(grp == 3 ? 0 : n_pad, trig, kGroupMode[grp]));
    }
    b->groups.clear();
    for (int k = 0; k < kGroups; ++k) {
        const std::vector<Item> list = xcd_order(members[k], b->desc_host, R);
        if (list.size() > b->item_cap) return false;
        std::copy(list.begin(), list.end(), items + k * b->item_cap);
        if (!list.empty())
            b->groups.push_back({kGroupMode[k], kGroupBlock[k], (int)list.size(), lds_need[k],
                                 b->d_items + k * b->item_cap});
    }
    b->dev.trig = trig;
    return true;
}

}  // namespace

extern "C" xy_status xy_batch_sizes(const xy_graph *const *g, int n_graphs, int n_T, int precision,
                                    int max_records, xy_sizes *out)
{
    if (!out) return set_error(XY_EINVAL, "xy_batch_sizes: out is NULL");
    Plan p;
    const xy_status st = plan_batch(g, n_graphs, n_T, precision, max_records, p);
    if (st != XY_OK) return st;
    out->state_bytes = p.state_bytes;
    out->graph_bytes = p.gl.total;
    out->work_bytes = p.wl.total;
    out->obs_bytes = p.obs_bytes;
    return XY_OK;
}

extern "C" xy_status xy_batch_init(xy_batch **out, const xy_graph *const *g, int n_graphs, int n_T,
                                   const double *T, int precision, const uint64_t *seeds, int max_records,
                                   void *d_state, void *d_graph, void *d_work, void *d_obs, void *stream)
{
    if (!out) return set_error(XY_EINVAL, "xy_batch_init: out is NULL");
    *out = nullptr;
    Plan p;
    xy_status st = plan_batch(g, n_graphs, n_T, precision, max_records, p);
    if (st != XY_OK) return st;
    if (!T || !seeds) return set_error(XY_EINVAL, "xy_batch_init: T and seeds are required");
    for (int k = 0; k < n_graphs * n_T; ++k)
        if (!(T[k] > 0.0) || !std::isfinite(T[k])) return set_error(XY_EINVAL, "xy_batch_init: temperatures must be finite and > 0");
    if (!d_state || !d_graph || !d_work || (max_records > 0 && !d_obs))
        return set_error(XY_EINVAL, "xy_batch_init: NULL device buffer");
    for (void *ptr : {d_state, d_graph, d_work})
        if (reinterpret_cast<uintptr_t>(ptr) % 256 != 0) return set_error(XY_EINVAL, "xy_batch_init: buffers must be 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);

    xy_batch *b = new (std::nothrow) xy_batch;
    if (!b) return set_error(XY_ENOMEM, "xy_batch_init: out of memory");
    try {
        const int G = n_graphs, R = n_T;
        b->G = G; b->R = R; b->precision = precision; b->max_records = max_records;
        b->max_n = p.max_n; b->Qmax = p.Qmax;
        b->d_state = d_state; b->d_graph = d_graph; b->d_work = d_work; b->d_obs = d_obs;
        b->wl = p.wl;
        b->state_bytes = p.state_bytes;
        b->state_off = p.state_off;
        b->phase_stride = p.phase_blocks;
        b->max_class.assign(p.Qmax, 0);
        b->perm.resize(G);
        b->n.resize(G);
        for (int s_ = 0; s_ < G; ++s_) {
            const xy_graph &gr = *g[s_];
            for (int c = 0; c < gr.Q; ++c)
                b->max_class[c] = std::max(b->max_class[c], gr.colour_off[c + 1] - gr.colour_off[c]);
            if (precision == XY_FIX16) {
                const Sell &S = p.sell[s_];
                b->perm[s_].resize(gr.n);
                for (int k = 0; k < gr.n; ++k) b->perm[s_][k] = gr.perm[S.order[k]];
            } else {
                b->perm[s_] = gr.perm;
            }
            b->n[s_] = gr.n;
            p.desc[s_].seed_lo = (uint32_t)seeds[s_];
            p.desc[s_].seed_hi = (uint32_t)(seeds[s_] >> 32);
        }

        // ---- graph region image
        const GraphLayout &gl = p.gl;
        std::vector<unsigned char> gimg(gl.total, 0);
        std::memcpy(gimg.data() + gl.desc, p.desc.data(), sizeof(SampleDesc) * G);
        int32_t *i32 = reinterpret_cast<int32_t *>(gimg.data() + gl.i32_pool);
        uint32_t *u32 = reinterpret_cast<uint32_t *>(gimg.data() + gl.u32_pool);
        double *f64 = reinterpret_cast<double *>(gimg.data() + gl.f64_pool);
        uint16_t *u16 = reinterpret_cast<uint16_t *>(gimg.data() + gl.u16_pool);
        uint8_t *u8 = reinterpret_cast<uint8_t *>(gimg.data() + gl.u8_pool);
        const double two_pi = 6.283185307179586476925286766559;
        for (int s_ = 0; s_ < G; ++s_) {
            const xy_graph &gr = *g[s_];
            const SampleDesc &d = p.desc[s_];
            if (precision == XY_FP64) {
                std::copy(gr.row_ptr.begin(), gr.row_ptr.end(), i32 + d.row_ptr);
                std::copy(gr.col.begin(), gr.col.end(), i32 + d.col);
            } else {
                const Sell &S = p.sell[s_];
                std::copy(S.chunk_ptr.begin(), S.chunk_ptr.end(), i32 + d.sell_ptr);
                std::copy(S.chunk_w.begin(), S.chunk_w.end(), i32 + d.sell_w);
                if (p.idx16)
                    for (size_t k = 0; k < S.col.size(); ++k) u16[d.sell_col + k] = (uint16_t)S.col[k];
                else
                    std::copy(S.col.begin(), S.col.end(), i32 + d.sell_col);
                std::copy(S.deg.begin(), S.deg.end(), u8 + d.deg);
            }
            const std::vector<int32_t> &pm = b->perm[s_];   // device index -> lattice index
            std::copy(pm.begin(), pm.end(), i32 + d.perm);
            for (int k = 0; k < gr.n; ++k) {
                const int v = pm[k];
                u32[d.coord + k] = (uint32_t)gr.cx[v] | ((uint32_t)gr.cy[v] << 16);
            }
            for (int x = 0; x < gr.L; ++x) {
                f64[2 * (d.trig + x)] = std::cos(two_pi * x / gr.L);
                f64[2 * (d.trig + x) + 1] = std::sin(two_pi * x / gr.L);
            }
        }
        const size_t off_tab32 = gl.tab32, off_tab64 = gl.tab64;
        float *t32 = reinterpret_cast<float *>(gimg.data() + off_tab32);
        float *t2k = reinterpret_cast<float *>(gimg.data() + gl.tab2k);
        double *t64 = reinterpret_cast<double *>(gimg.data() + off_tab64);
        for (int k = 0; k < 2048; ++k) {
            const double a = two_pi * (32.0 * k) / 65536.0;
            t2k[2 * k] = (float)std::cos(a);
            t2k[2 * k + 1] = (float)std::sin(a);
        }
        for (int k = 0; k < 256; ++k) {
            const double ahi = two_pi * (256.0 * k) / 65536.0, alo = two_pi * k / 65536.0;
            t64[2 * k] = std::cos(ahi);          t64[2 * k + 1] = std::sin(ahi);
            t64[512 + 2 * k] = std::cos(alo);    t64[512 + 2 * k + 1] = std::sin(alo);
            t32[2 * k] = (float)t64[2 * k];      t32[2 * k + 1] = (float)t64[2 * k + 1];
            t32[512 + 2 * k] = (float)t64[512 + 2 * k];
            t32[512 + 2 * k + 1] = (float)t64[512 + 2 * k + 1];
        }
        // fix16 items: LDS-resident where the replica fits, else global state
        // (cos, sin) form of the fixed-point sweep: the hardware sine/cosine by
        // default (fastest on gfx950); XY_FIX16_TRIG=0/1 selects a table form
        int trig = 2;
        if (const char *env = std::getenv("XY_FIX16_TRIG")) trig = std::atoi(env);
        if (trig < 0 || trig > 2) trig = 2;
        if (precision == XY_FIX16) {
            int dev = 0, lds_limit = 0;
            (void)hipGetDevice(&dev);
            if (hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
                lds_limit = 65536;
            // XY_FIX16_GLOBAL=1 keeps every replica in global memory (the form
            // for graphs too large for LDS when n_T is not a multiple of 4);
            // tests use it at small sizes
            bool force_global = false;
            if (const char *env = std::getenv("XY_FIX16_GLOBAL"))
                if (std::atoi(env) != 0) force_global = true;
            // XY_FIX16_NOUNIT=1 disables the unit-vector form (tests compare the forms)
            bool allow_unit = true;
            if (const char *env = std::getenv("XY_FIX16_NOUNIT"))
                if (std::atoi(env) != 0) allow_unit = false;
            b->desc_host = p.desc;
            b->item_cap = p.item_cap;
            b->lds_limit = lds_limit;
            b->d_items = reinterpret_cast<Item *>(static_cast<unsigned char *>(d_graph) + gl.items);
            // phase form: the samples, and for each colour the launch's work
            // units in sample order (each a block of sites of that sample's
            // colour class), so every workgroup of a launch has work
            std::vector<int32_t> phase;
            for (int s_ = 0; s_ < G; ++s_)
                if (p.desc[s_].layout) phase.push_back(s_);
            std::vector<int4> units;
            b->phase_units.assign(p.Qmax, 0);
            b->phase_unit_off.assign(p.Qmax, 0);
            const int spb = R % 4 == 0 ? fix16_phase_sites_per_block(R) : 1;
            bool fits = true;
            auto u32 = [&fits](int64_t v) {
                if (v < 0 || v > (int64_t)UINT32_MAX) fits = false;
                return (int)(uint32_t)v;
            };
            for (int c = 0; c < p.Qmax; ++c) {
                b->phase_unit_off[c] = units.size();
                for (int k = 0; k < (int)phase.size(); ++k) {
                    const SampleDesc &d = p.desc[phase[k]];
                    if (c >= d.Q) continue;
                    const Sell &Sl = p.sell[phase[k]];
                    const int c0 = d.colour_off[c], c1 = d.colour_off[c + 1];
                    const int nb = (c1 - c0 + spb - 1) / spb;
                    for (int bx = 0; bx < nb; ++bx) {
                        // unit of kernel_phase: two int4, see k_fix16_phase
                        const int r0 = bx * spb, n_act = std::min(spb, c1 - c0 - r0);
                        const int chA = Sl.chunk_off[c] + (r0 >> 6);
                        int kmin = 255, kmax = 0;
                        for (int ch = r0 >> 6; ch <= (r0 + n_act - 1) >> 6; ++ch) {
                            const int w = Sl.chunk_w[Sl.chunk_off[c] + ch];
                            kmin = std::min(kmin, w & 255);
                            kmax = std::max(kmax, w >> 8);
                        }
                        const int64_t colA = d.sell_col + Sl.chunk_ptr[chA];
                        const int64_t colB = chA + 1 < Sl.chunk_off[c + 1] ? d.sell_col + Sl.chunk_ptr[chA + 1] : colA;
                        units.push_back(make_int4(u32(colA), u32(colB), u32(d.state / 8), c0 + r0));
                        units.push_back(make_int4(phase[k], k, bx, kmin | kmax << 8 | (n_act - 1) << 16 | (r0 & 63) << 24));
                    }
                }
                b->phase_units[c] = (int)((units.size() - b->phase_unit_off[c]) / 2);
            }
            if (!fits) {
                delete b;
                return set_error(XY_EUNSUP, "xy_batch_init: phase-form offsets exceed 32 bits (batch too large)");
            }
            if (units.size() != 2 * p.phase_units) {
                delete b;
                return set_error(XY_EUNSUP, "xy_batch_init: phase-form work units do not match the plan");
            }
            // phase index of every work unit, for regrouping
            b->unit_k.resize(units.size() / 2);
            for (size_t a = 0; a < b->unit_k.size(); ++a) b->unit_k[a] = units[2 * a + 1].y;
            b->n_phase = (int)phase.size();
            if (const char *env = std::getenv("XY_PHASE_SERPENTINE")) b->serpentine = std::atoi(env) != 0;
            int n_streams = 2, n_slices = 1;   // XY_PHASE_STREAMS=1..4 and XY_PHASE_SLICES override
            if (const char *env = std::getenv("XY_PHASE_STREAMS")) n_streams = std::atoi(env);
            if (const char *env = std::getenv("XY_PHASE_SLICES")) n_slices = std::atoi(env);
            const hipError_t e = setup_phase_groups(b, n_streams, n_slices);
            if (e != hipSuccess) {
                xy_batch_free(b);
                return hip_err(e, "xy_batch_init: phase streams");
            }
            unsigned char *ph = gimg.data() + gl.phase;
            std::copy(phase.begin(), phase.end(), reinterpret_cast<int32_t *>(ph));
            std::copy(units.begin(), units.end(), reinterpret_cast<int4 *>(ph + align_up(4 * (size_t)G, 16)));
            b->phase_stride = p.phase_blocks;
            b->d_phase = reinterpret_cast<int32_t *>(static_cast<unsigned char *>(d_graph) + gl.phase);
            b->d_units = reinterpret_cast<int4 *>(static_cast<unsigned char *>(d_graph) + gl.phase +
                                                  align_up(4 * (size_t)G, 16));
            Item *items = reinterpret_cast<Item *>(gimg.data() + gl.items);
            if (!build_groups(b, trig, allow_unit, force_global, items)) {
                xy_batch_free(b);
                return set_error(XY_EUNSUP, "xy_batch_init: work-item list exceeds its capacity");
            }
        }

        // ---- work region image
        const WorkLayout &wl = p.wl;
        std::vector<unsigned char> wimg(wl.total, 0);
        double *beta = reinterpret_cast<double *>(wimg.data() + wl.beta);
        int32_t *sot = reinterpret_cast<int32_t *>(wimg.data() + wl.slot_of_T);
        int32_t *tos = reinterpret_cast<int32_t *>(wimg.data() + wl.T_of_slot);
        for (int k = 0; k < G * R; ++k) {
            beta[k] = 1.0 / T[k];
            sot[k] = k % R;
            tos[k] = k % R;
        }
        b->beta_host.assign(beta, beta + (size_t)G * R);
        b->d_beta = reinterpret_cast<double *>(static_cast<unsigned char *>(d_work) + wl.beta);

        hipError_t e;
        if ((e = hipMemcpyAsync(d_graph, gimg.data(), gimg.size(), hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(d_work, wimg.data(), wimg.size(), hipMemcpyHostToDevice, s)) != hipSuccess) {
            xy_batch_free(b);
            return hip_err(e, "xy_batch_init upload");
        }

        unsigned char *gbase = static_cast<unsigned char *>(d_graph);
        unsigned char *wbase = static_cast<unsigned char *>(d_work);
        DevBatch &dv = b->dev;
        dv.desc = reinterpret_cast<const SampleDesc *>(gbase + gl.desc);
        dv.i32 = reinterpret_cast<const int32_t *>(gbase + gl.i32_pool);
        dv.u32 = reinterpret_cast<const uint32_t *>(gbase + gl.u32_pool);
        dv.f64 = reinterpret_cast<const double2 *>(gbase + gl.f64_pool);
        dv.u16 = reinterpret_cast<const uint16_t *>(gbase + gl.u16_pool);
        dv.u8 = reinterpret_cast<const uint8_t *>(gbase + gl.u8_pool);
        dv.tab32 = reinterpret_cast<const float2 *>(gbase + off_tab32);
        dv.tab2k = reinterpret_cast<const float2 *>(gbase + gl.tab2k);
        dv.tab64 = reinterpret_cast<const double2 *>(gbase + off_tab64);
        dv.state = d_state;
        dv.ctl = reinterpret_cast<Ctl *>(wbase + wl.ctl);
        dv.beta = reinterpret_cast<const double *>(wbase + wl.beta);
        dv.slot_of_T = reinterpret_cast<int32_t *>(wbase + wl.slot_of_T);
        dv.T_of_slot = reinterpret_cast<int32_t *>(wbase + wl.T_of_slot);
        dv.fac_slot = reinterpret_cast<float *>(wbase + wl.fac_slot);
        dv.E_slot = reinterpret_cast<double *>(wbase + wl.E_slot);
        dv.obs_slot = reinterpret_cast<double *>(wbase + wl.obs_slot);
        dv.pt_acc = reinterpret_cast<unsigned long long *>(wbase + wl.pt_acc);
        dv.pt_try = reinterpret_cast<unsigned long long *>(wbase + wl.pt_try);
        dv.partial = reinterpret_cast<double *>(wbase + wl.partial);
        dv.epart = reinterpret_cast<double *>(wbase + wl.epart);
        dv.records = static_cast<double *>(d_obs);
        dv.G = G; dv.R = R; dv.max_records = max_records; dv.max_n = p.max_n;
        dv.log = nullptr; dv.log_sweeps = 0;
        dv.idx16 = p.idx16 ? 1 : 0;
        dv.trig = trig;

        e = launch_slot_factors(dv, s);
        if (e == hipSuccess)
            e = (precision == XY_FP64) ? launch_fp64_init(dv, p.max_n, s) : launch_fix16_init(dv, p.max_n, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);   // host images must outlive the copies
        if (e != hipSuccess) { xy_batch_free(b); return hip_err(e, "xy_batch_init"); }
    } catch (const std::bad_alloc &) {
        xy_batch_free(b);
        return set_error(XY_ENOMEM, "xy_batch_init: out of memory");
    }
    *out = b;
    return XY_OK;
}

namespace {

// Event pair for the next timed sweep (created on first use, then reused).
hipError_t next_events(xy_batch *b, hipEvent_t *start, hipEvent_t *stop)
{
    if (b->events_used == b->events.size()) {
        // timing only: no system-scope fence on record (that fence writes
        // back and invalidates the caches, which costs the following kernels);
        // xy_kernel_time synchronises the stream before reading them
        hipEvent_t a = nullptr, c = nullptr;
        hipError_t e = hipEventCreateWithFlags(&a, hipEventDisableSystemFence);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c, hipEventDisableSystemFence);
        if (e != hipSuccess) return e;
        b->events.emplace_back(a, c);
    }
    *start = b->events[b->events_used].first;
    *stop = b->events[b->events_used].second;
    b->events_used++;
    return hipSuccess;
}

// Forks the auxiliary streams of the phase form from s, and joins them back.
hipError_t fork_groups(xy_batch *b, hipStream_t s)
{
    if (b->aux.empty()) return hipSuccess;   // one stream (groups in slices only): nothing to fork
    hipError_t e = hipEventRecord(b->ev_fork, s);
    for (size_t g = 0; g < b->aux.size() && e == hipSuccess; ++g) e = hipStreamWaitEvent(b->aux[g], b->ev_fork, 0);
    return e;
}

hipError_t join_groups(xy_batch *b, hipStream_t s)
{
    hipError_t e = hipSuccess;
    for (size_t g = 0; g < b->aux.size() && e == hipSuccess; ++g) {
        e = hipEventRecord(b->ev_join[g], b->aux[g]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, b->ev_join[g], 0);
    }
    return e;
}

// Enqueues one sweep with the given flags.  With independent groups: one
// sweep of the groups of slice `slice`; the caller has forked the streams
// (fork_groups) and joins them after its last sweep.
hipError_t enqueue_sweep(xy_batch *b, int n_or, int do_pt, int do_rec, hipStream_t s, int slice = 0)
{
    hipError_t e = hipSuccess;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (b->timing && !b->indep) {
        e = next_events(b, &ev0, &ev1);
        if (e == hipSuccess) e = hipEventRecord(ev0, s);
        if (e != hipSuccess) return e;
        b->event_sweeps.push_back(1);
        b->timed_stream = s;
    }
    const int n_st = 1 + (int)b->aux.size();
    const int n_gr = n_st * (b->indep ? b->n_slices : 1);   // groups: the stride of phase_bounds
    if (b->precision == XY_FP64) {
        // the energies for tempering are summed in the last sub-sweep, except
        // on a measurement sweep, whose observation pass sums them anyway
        const int fuse = do_pt && !do_rec;
        for (int sub = 0; sub <= n_or && e == hipSuccess; ++sub)
            for (int c = 0; c < b->Qmax && e == hipSuccess; ++c)
                e = launch_fp64_phase(b->dev, c, sub == 0, fuse && sub == n_or, b->max_class[c], b->Qmax,
                                      b->phase_stride, s);
        if (e == hipSuccess && ev1) e = hipEventRecord(ev1, s);
        if (e == hipSuccess && do_rec) e = launch_fp64_observe(b->dev, 1, nullptr, s);
        if (e == hipSuccess && fuse)
            e = launch_fp64_energy_final(b->dev, b->max_class.data(), b->Qmax, b->phase_stride, s);
    } else if (b->indep) {
        // each group of the slice: its colour phases, then its energies,
        // tempering, records and sweep counter, all on its own stream
        const int g0 = slice * n_st;
        for (int sub = 0; sub <= n_or && e == hipSuccess; ++sub)
            for (int c = 0; c < (int)b->phase_units.size() && e == hipSuccess; ++c) {
                const int *bd = b->phase_bounds.data() + (size_t)c * (n_gr + 1);
                const int4 *u = b->d_units + b->phase_unit_off[c];
                const int rev = b->serpentine ? (sub * (int)b->phase_units.size() + c) & 1 : 0;
                for (int h = 0; h < n_st && e == hipSuccess; ++h) {
                    const int g = g0 + h;
                    e = launch_fix16_phase(b->dev, u + 2 * (size_t)bd[g], c, sub, sub == n_or, bd[g + 1] - bd[g],
                                           b->phase_stride, g, rev, h == 0 ? s : b->aux[h - 1]);
                }
            }
        for (int h = 0; h < n_st && e == hipSuccess; ++h) {
            hipStream_t st = h == 0 ? s : b->aux[h - 1];
            const int g = g0 + h;
            const int k0 = b->group_first[g], nk = b->group_first[g + 1] - k0;
            if (do_rec) e = launch_fix16_observe_sm(b->dev, b->d_phase, k0, nk, 1, st);
            if (e == hipSuccess && do_pt) e = launch_fix16_phase_energy(b->dev, b->d_phase, k0, nk, b->phase_stride, st);
            if (e == hipSuccess) e = launch_end_sweep(b->dev, b->d_phase + k0, nk, g, do_pt, do_rec, 1, st);
        }
        return e;
    } else {
        // the workgroup-form samples on the caller's stream, after the fork,
        // so that the other groups' colour phases overlap them
        const bool fork = b->n_phase > 0 && n_st > 1;
        if (e == hipSuccess && fork) e = fork_groups(b, s);
        for (const auto &grp : b->groups) {
            if (e != hipSuccess) break;
            e = launch_fix16_sweep(b->dev, grp.items, grp.n_items, grp.mode, grp.block, n_or, do_rec, grp.lds, s);
        }
        for (int sub = 0; sub <= n_or && e == hipSuccess && b->n_phase > 0; ++sub)
            for (int c = 0; c < (int)b->phase_units.size() && e == hipSuccess; ++c) {
                const int *bd = b->phase_bounds.data() + (size_t)c * (n_gr + 1);
                const int4 *u = b->d_units + b->phase_unit_off[c];
                const int rev = b->serpentine ? (sub * (int)b->phase_units.size() + c) & 1 : 0;
                for (int g = 0; g < n_st && e == hipSuccess; ++g)
                    e = launch_fix16_phase(b->dev, u + 2 * (size_t)bd[g], c, sub, sub == n_or, bd[g + 1] - bd[g],
                                           b->phase_stride, 0, rev, g == 0 ? s : b->aux[g - 1]);
            }
        if (e == hipSuccess && fork) e = join_groups(b, s);
        // the timed part: the sweep kernels (with their fused energies) and the
        // colour-phase kernels of the phase form
        if (e == hipSuccess && ev1) e = hipEventRecord(ev1, s);
        if (e == hipSuccess && b->n_phase > 0) {
            if (do_rec) e = launch_fix16_observe_sm(b->dev, b->d_phase, 0, b->n_phase, 1, s);
            // E_slot for tempering: the FP32-form energies fused in the last sub-sweep
            if (e == hipSuccess && do_pt)
                e = launch_fix16_phase_energy(b->dev, b->d_phase, 0, b->n_phase, b->phase_stride, s);
        }
    }
    if (e == hipSuccess) e = launch_end_sweep(b->dev, nullptr, 0, 0, do_pt, do_rec, 1, s);
    return e;
}

bool flag_at(uint32_t sweep, int every) { return every > 0 && (sweep + 1) % (uint32_t)every == 0; }

uint64_t gcd_u64(uint64_t a, uint64_t c)
{
    while (c) { const uint64_t t = a % c; a = c; c = t; }
    return a;
}

// Period of the per-sweep pattern a captured chunk bakes in: tempering after
// sweeps with (sweep + 1) % pt_every == 0 and records after sweeps with
// (sweep + 1) % meas_every == 0 repeat with lcm(pt_every, meas_every).  (The
// pair parity of a tempering step is read from the device's sweep counter,
// so it is not baked in.)
uint64_t pattern_period(int pt_every, int meas_every)
{
    const uint64_t a = pt_every > 0 ? (uint64_t)pt_every : 1u, c = meas_every > 0 ? (uint64_t)meas_every : 1u;
    return a / gcd_u64(a, c) * c;
}

// n sweeps by direct launches.  With independent stream groups: one fork and
// one join around them, and with timing one event pair around the whole.
hipError_t run_direct(xy_batch *b, int n, int n_or, int pt_every, int meas_every, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipError_t e = hipSuccess;
    if (b->indep) {
        if (b->timing) {
            e = next_events(b, &ev0, &ev1);
            if (e == hipSuccess) e = hipEventRecord(ev0, s);
            if (e != hipSuccess) return e;
            b->event_sweeps.push_back(n);
            b->timed_stream = s;
        }
        e = fork_groups(b, s);
        if (e != hipSuccess) return e;
    }
    // independent groups: the slices one after the other, each for all n sweeps
    const uint32_t sw0 = b->host_sweep;
    const int n_sl = b->indep ? b->n_slices : 1;
    for (int sl = 0; sl < n_sl && e == hipSuccess; ++sl) {
        b->host_sweep = sw0;
        for (int k = 0; k < n && e == hipSuccess; ++k) {
            const uint32_t sw = b->host_sweep;
            e = enqueue_sweep(b, n_or, flag_at(sw, pt_every), flag_at(sw, meas_every), s, sl);
            if (e == hipSuccess) b->host_sweep++;
        }
    }
    if (b->indep) {
        const hipError_t e2 = join_groups(b, s);   // also after a failed launch: leave no stream forked
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess && ev1) e = hipEventRecord(ev1, s);
    }
    return e;
}

// Captures b->chunk sweeps starting at the current sweep into b->gexec.  The
// graph holds no timing events: a replay is timed as a whole.
hipError_t capture_chunk(xy_batch *b, int n_or, int pt_every, int meas_every, uint64_t period, hipStream_t s)
{
    if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
    const bool timing = b->timing;
    b->timing = false;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        if (b->indep) e = fork_groups(b, s);
        const int n_sl = b->indep ? b->n_slices : 1;
        for (int sl = 0; sl < n_sl && e == hipSuccess; ++sl) {
            uint32_t sw = b->host_sweep;
            for (int k = 0; k < b->chunk && e == hipSuccess; ++k, ++sw)
                e = enqueue_sweep(b, n_or, flag_at(sw, pt_every), flag_at(sw, meas_every), s, sl);
        }
        if (b->indep && e == hipSuccess) e = join_groups(b, s);
        const hipError_t e2 = hipStreamEndCapture(s, &graph);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
    }
    b->timing = timing;
    if (e != hipSuccess) { b->gexec = nullptr; return e; }
    b->g_n_or = n_or; b->g_pt = pt_every; b->g_meas = meas_every; b->gstream = s;
    b->g_period = period;
    b->g_phase = b->host_sweep % period;
    return hipSuccess;
}

// New temperature ladder by temperature index (the slot labels are kept):
// beta is uploaded on s from a host copy that the batch keeps until the
// upload has been read (an event waits for the previous one first).
xy_status set_ladder(xy_batch *b, const double *T, hipStream_t s)
{
    const size_t GR = (size_t)b->G * b->R;
    for (size_t k = 0; k < GR; ++k)
        if (!(T[k] > 0.0) || !std::isfinite(T[k])) return set_error(XY_EINVAL, "xy_sweep: temperatures must be finite and > 0");
    hipError_t e = hipSuccess;
    if (!b->ev_beta) e = hipEventCreateWithFlags(&b->ev_beta, hipEventDisableTiming);
    else e = hipEventSynchronize(b->ev_beta);
    if (e != hipSuccess) return hip_err(e, "xy_sweep ladder");
    for (size_t k = 0; k < GR; ++k) b->beta_host[k] = 1.0 / T[k];
    e = hipMemcpyAsync(b->d_beta, b->beta_host.data(), 8 * GR, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(b->ev_beta, s);
    if (e == hipSuccess) e = launch_slot_factors(b->dev, s);
    return e == hipSuccess ? XY_OK : hip_err(e, "xy_sweep ladder");
}

}  // namespace

extern "C" xy_status xy_sweep(xy_batch *b, const double *T, int n_sweeps, int n_or, int pt_every, int meas_every,
                              void *stream)
{
    if (!b) return set_error(XY_EINVAL, "xy_sweep: batch is NULL");
    if (n_sweeps < 0 || n_or < 0 || n_or > 255 || pt_every < 0 || meas_every < 0)
        return set_error(XY_EINVAL, "xy_sweep: bad arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (b->chunk > 0 && !s) return set_error(XY_EINVAL, "xy_sweep: HIP graph capture needs a non-null stream");
    if (T) {
        const xy_status st = set_ladder(b, T, s);
        if (st != XY_OK) return st;
    }
    int done = 0;
    hipError_t e = hipSuccess;
    // HIP graph replay: a captured chunk is valid where the sweep index is
    // congruent to the one it was captured at, modulo the period of its
    // tempering / record pattern; in between, direct launches realign it.
    if (b->chunk > 0) {
        const uint64_t period = pattern_period(pt_every, meas_every);
        while (e == hipSuccess && n_sweeps - done >= b->chunk) {
            const bool same = b->gexec && b->g_n_or == n_or && b->g_pt == pt_every && b->g_meas == meas_every &&
                              b->gstream == s && b->g_period == period;
            if (same) {
                const uint64_t ph = b->host_sweep % period;
                if (ph != b->g_phase) {
                    const uint64_t k = (b->g_phase + period - ph) % period;   // sweeps to the captured phase
                    if (k > (uint64_t)(n_sweeps - done - b->chunk)) break;
                    e = run_direct(b, (int)k, n_or, pt_every, meas_every, s);
                    done += (int)k;
                    continue;
                }
            } else {
                e = capture_chunk(b, n_or, pt_every, meas_every, period, s);
                if (e != hipSuccess) return hip_err(e, "xy_sweep graph capture");
            }
            hipEvent_t ev0 = nullptr, ev1 = nullptr;
            if (b->timing) {
                e = next_events(b, &ev0, &ev1);
                if (e == hipSuccess) e = hipEventRecord(ev0, s);
                if (e != hipSuccess) break;
                b->event_sweeps.push_back(b->chunk);
                b->timed_stream = s;
            }
            e = hipGraphLaunch(b->gexec, s);
            if (e == hipSuccess && ev1) e = hipEventRecord(ev1, s);
            if (e != hipSuccess) break;
            b->host_sweep += (uint32_t)b->chunk;
            done += b->chunk;
        }
    }
    if (e == hipSuccess) e = run_direct(b, n_sweeps - done, n_or, pt_every, meas_every, s);
    return e == hipSuccess ? XY_OK : hip_err(e, "xy_sweep");
}

extern "C" xy_status xy_batch_use_graph(xy_batch *b, int chunk)
{
    if (!b || chunk < 0) return set_error(XY_EINVAL, "xy_batch_use_graph: bad arguments");
    if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
    b->chunk = chunk;
    return XY_OK;
}

extern "C" xy_status xy_pt_energies(xy_batch *b, double *d_out, void *stream)
{
    if (!b || !d_out) return set_error(XY_EINVAL, "xy_pt_energies: NULL argument");
    const hipError_t e = hipMemcpyAsync(d_out, b->dev.E_slot, sizeof(double) * (size_t)b->G * b->R,
                                        hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? XY_OK : hip_err(e, "xy_pt_energies");
}

extern "C" xy_status xy_measure(xy_batch *b, double *d_out, void *stream)
{
    if (!b || !d_out) return set_error(XY_EINVAL, "xy_measure: bad arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const hipError_t e = (b->precision == XY_FP64) ? launch_fp64_observe(b->dev, 1, d_out, s)
                                                   : launch_fix16_observe(b->dev, d_out, s);
    return e == hipSuccess ? XY_OK : hip_err(e, "xy_measure");
}

extern "C" xy_status xy_pt_swap(xy_batch *b, void *stream)
{
    if (!b) return set_error(XY_EINVAL, "xy_pt_swap: batch is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = (b->precision == XY_FP64) ? launch_fp64_observe(b->dev, 0, nullptr, s)
                                             : launch_fix16_observe(b->dev, nullptr, s);
    if (e == hipSuccess) e = launch_end_sweep(b->dev, nullptr, 0, 0, 1, 0, 0, s);
    return e == hipSuccess ? XY_OK : hip_err(e, "xy_pt_swap");
}

extern "C" xy_status xy_get_state(xy_batch *b, void *h_state, int32_t *h_slot_of_T, uint32_t *sweep, void *stream)
{
    if (!b) return set_error(XY_EINVAL, "xy_get_state: batch is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int G = b->G, R = b->R;
    try {
        std::vector<unsigned char> raw(h_state ? b->state_bytes : 0);
        std::vector<int32_t> sot(h_slot_of_T ? (size_t)G * R : 0);
        Ctl ctl{};
        hipError_t e = hipSuccess;
        if (h_state) e = hipMemcpyAsync(raw.data(), b->d_state, raw.size(), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && h_slot_of_T)
            e = hipMemcpyAsync(sot.data(), b->dev.slot_of_T, sot.size() * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&ctl, b->dev.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_err(e, "xy_get_state");
        if (h_state) {
            size_t out_off = 0;
            for (int g = 0; g < G; ++g) {
                const int n = b->n[g];
                const std::vector<int32_t> &pm = b->perm[g];
                if (b->precision == XY_FP64) {
                    const double *src = reinterpret_cast<const double *>(raw.data()) + 2 * b->state_off[g];
                    double *dst = static_cast<double *>(h_state) + out_off;
                    for (int r = 0; r < R; ++r)
                        for (int k = 0; k < n; ++k) {
                            dst[2 * ((size_t)r * n + pm[k])] = src[2 * ((size_t)k * R + r)];
                            dst[2 * ((size_t)r * n + pm[k]) + 1] = src[2 * ((size_t)k * R + r) + 1];
                        }
                    out_off += 2 * (size_t)R * n;
                } else {
                    const int n_pad = (n + 7) & ~7;
                    const bool site_major = b->desc_host[g].layout != 0;
                    const uint16_t *src = reinterpret_cast<const uint16_t *>(raw.data()) + b->state_off[g];
                    uint16_t *dst = static_cast<uint16_t *>(h_state) + out_off;
                    for (int r = 0; r < R; ++r)
                        for (int k = 0; k < n; ++k)
                            dst[(size_t)r * n + pm[k]] = site_major ? src[(size_t)k * R + r] : src[(size_t)r * n_pad + k];
                    out_off += (size_t)R * n;
                }
            }
        }
        if (h_slot_of_T) std::copy(sot.begin(), sot.end(), h_slot_of_T);
        if (sweep) *sweep = ctl.sweep;
    } catch (const std::bad_alloc &) {
        return set_error(XY_ENOMEM, "xy_get_state: out of memory");
    }
    return XY_OK;
}

extern "C" xy_status xy_set_state(xy_batch *b, const void *h_state, const int32_t *h_slot_of_T, uint32_t sweep,
                                  void *stream)
{
    if (!b) return set_error(XY_EINVAL, "xy_set_state: batch is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int G = b->G, R = b->R;
    try {
        std::vector<int32_t> sot, tos;
        if (h_slot_of_T) {
            sot.assign(h_slot_of_T, h_slot_of_T + (size_t)G * R);
            tos.assign((size_t)G * R, -1);
            for (int g = 0; g < G; ++g)
                for (int k = 0; k < R; ++k) {
                    const int r = sot[(size_t)g * R + k];
                    if (r < 0 || r >= R || tos[(size_t)g * R + r] >= 0)
                        return set_error(XY_EINVAL, "xy_set_state: slot_of_T is not a permutation");
                    tos[(size_t)g * R + r] = k;
                }
        }
        std::vector<unsigned char> raw(h_state ? b->state_bytes : 0, 0);
        if (h_state) {
            size_t in_off = 0;
            for (int g = 0; g < G; ++g) {
                const int n = b->n[g];
                const std::vector<int32_t> &pm = b->perm[g];
                if (b->precision == XY_FP64) {
                    double *dst = reinterpret_cast<double *>(raw.data()) + 2 * b->state_off[g];
                    const double *src = static_cast<const double *>(h_state) + in_off;
                    for (int r = 0; r < R; ++r)
                        for (int k = 0; k < n; ++k) {
                            dst[2 * ((size_t)k * R + r)] = src[2 * ((size_t)r * n + pm[k])];
                            dst[2 * ((size_t)k * R + r) + 1] = src[2 * ((size_t)r * n + pm[k]) + 1];
                        }
                    in_off += 2 * (size_t)R * n;
                } else {
                    const int n_pad = (n + 7) & ~7;
                    const bool site_major = b->desc_host[g].layout != 0;
                    uint16_t *dst = reinterpret_cast<uint16_t *>(raw.data()) + b->state_off[g];
                    const uint16_t *src = static_cast<const uint16_t *>(h_state) + in_off;
                    for (int r = 0; r < R; ++r)
                        for (int k = 0; k < n; ++k)
                            (site_major ? dst[(size_t)k * R + r] : dst[(size_t)r * n_pad + k]) = src[(size_t)r * n + pm[k]];
                    in_off += (size_t)R * n;
                }
            }
        }
        hipError_t e = hipSuccess;
        if (h_state) e = hipMemcpyAsync(b->d_state, raw.data(), raw.size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess && h_slot_of_T) {
            e = hipMemcpyAsync(b->dev.slot_of_T, sot.data(), sot.size() * 4, hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipMemcpyAsync(b->dev.T_of_slot, tos.data(), tos.size() * 4, hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = launch_slot_factors(b->dev, s);
        }
        for (int g = 0; g < kMaxPhaseGroups && e == hipSuccess; ++g)
            e = hipMemcpyAsync(&b->dev.ctl[g].sweep, &sweep, 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_err(e, "xy_set_state");
        b->host_sweep = sweep;
        if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
    } catch (const std::bad_alloc &) {
        return set_error(XY_ENOMEM, "xy_set_state: out of memory");
    }
    return XY_OK;
}

extern "C" xy_status xy_get_counters(xy_batch *b, int *n_records, uint64_t *pt_accepted, uint64_t *pt_attempted,
                                     void *stream)
{
    if (!b) return set_error(XY_EINVAL, "xy_get_counters: batch is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t GR = (size_t)b->G * b->R;
    Ctl ctl{};
    hipError_t e = hipMemcpyAsync(&ctl, b->dev.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && pt_accepted) e = hipMemcpyAsync(pt_accepted, b->dev.pt_acc, 8 * GR, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && pt_attempted) e = hipMemcpyAsync(pt_attempted, b->dev.pt_try, 8 * GR, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(e, "xy_get_counters");
    if (n_records) *n_records = (int)std::min<uint32_t>(ctl.n_records, (uint32_t)b->max_records);
    return XY_OK;
}

extern "C" xy_status xy_decision_log(xy_batch *b, uint8_t *d_log, int max_sweeps)
{
    if (!b) return set_error(XY_EINVAL, "xy_decision_log: batch is NULL");
    if (b->precision != XY_FP64) return set_error(XY_EUNSUP, "xy_decision_log: FP64 batches only");
    if (d_log && max_sweeps < 0) return set_error(XY_EINVAL, "xy_decision_log: max_sweeps < 0");
    // the log base is the sweep counter now; it is written synchronously
    const uint32_t base = b->host_sweep;
    const hipError_t e = hipMemcpy(&b->dev.ctl->log_base, &base, 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_err(e, "xy_decision_log");
    b->dev.log = d_log;
    b->dev.log_sweeps = d_log ? max_sweeps : 0;
    if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
    return XY_OK;
}

extern "C" xy_status xy_kernel_timing(xy_batch *b, int enable)
{
    if (!b) return set_error(XY_EINVAL, "xy_kernel_timing: batch is NULL");
    if (b->timed_stream || b->events_used) {
        const hipError_t e = hipStreamSynchronize(b->timed_stream);
        if (e != hipSuccess) return hip_err(e, "xy_kernel_timing");
    }
    b->timing = enable != 0;
    b->events_used = 0;
    b->event_sweeps.clear();
    return XY_OK;
}

extern "C" xy_status xy_kernel_time(xy_batch *b, double *ms_total, int *n_timed)
{
    if (!b) return set_error(XY_EINVAL, "xy_kernel_time: batch is NULL");
    double total = 0.0;
    if (b->events_used) {
        hipError_t e = hipStreamSynchronize(b->timed_stream);
        for (size_t k = 0; k < b->events_used && e == hipSuccess; ++k) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, b->events[k].first, b->events[k].second);
            total += ms;
        }
        if (e != hipSuccess) return hip_err(e, "xy_kernel_time");
    }
    int n = 0;
    for (size_t k = 0; k < b->events_used && k < b->event_sweeps.size(); ++k) n += b->event_sweeps[k];
    if (ms_total) *ms_total = total;
    if (n_timed) *n_timed = n;
    return XY_OK;
}

extern "C" xy_status xy_batch_set_phase_groups(xy_batch *b, int n_streams, int n_slices, void *stream)
{
    if (!b || n_streams < 1 || n_streams > kMaxPhaseStreams || n_slices < 1 || n_streams * n_slices > kMaxPhaseGroups)
        return set_error(XY_EINVAL, "xy_batch_set_phase_groups: need 1 <= n_streams <= 4, n_slices >= 1 and "
                                    "n_streams * n_slices <= 8");
    if (b->precision != XY_FIX16 || b->n_phase == 0) return XY_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamSynchronize(s);
    for (size_t g = 0; g < b->aux.size() && e == hipSuccess; ++g) e = hipStreamSynchronize(b->aux[g]);
    if (e == hipSuccess) e = setup_phase_groups(b, n_streams, n_slices);
    // every group's control block continues from group 0's (equal after a sweep call)
    for (int g = 1; g < kMaxPhaseGroups && e == hipSuccess; ++g)
        e = hipMemcpyAsync(b->dev.ctl + g, b->dev.ctl, sizeof(Ctl), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
    return e == hipSuccess ? XY_OK : hip_err(e, "xy_batch_set_phase_groups");
}

extern "C" xy_status xy_batch_set_phase_streams(xy_batch *b, int n_streams, void *stream)
{
    if (!b || n_streams < 1 || n_streams > kMaxPhaseStreams)
        return set_error(XY_EINVAL, "xy_batch_set_phase_streams: n_streams must be in [1, 4]");
    return xy_batch_set_phase_groups(b, n_streams, 1, stream);
}

extern "C" xy_status xy_batch_phase_groups(const xy_batch *b, int *n_streams, int *n_slices)
{
    if (!b || !n_streams || !n_slices) return set_error(XY_EINVAL, "xy_batch_phase_groups: NULL argument");
    *n_streams = 1 + (int)b->aux.size();
    *n_slices = b->indep ? b->n_slices : 1;
    return XY_OK;
}

extern "C" xy_status xy_batch_phase_streams(const xy_batch *b, int *n_streams)
{
    if (!b || !n_streams) return set_error(XY_EINVAL, "xy_batch_phase_streams: NULL argument");
    *n_streams = 1 + (int)b->aux.size();
    return XY_OK;
}

extern "C" xy_status xy_batch_forms(const xy_batch *b, int32_t *out)
{
    if (!b || !out) return set_error(XY_EINVAL, "xy_batch_forms: bad arguments");
    for (int s = 0; s < b->G; ++s)
        out[s] = (b->precision == XY_FIX16 && s < (int)b->desc_host.size()) ? b->desc_host[s].layout : 0;
    return XY_OK;
}

extern "C" xy_status xy_batch_set_fix16_form(xy_batch *b, int trig, int allow_unit, int force_global, void *stream)
{
    if (!b) return set_error(XY_EINVAL, "xy_batch_set_fix16_form: batch is NULL");
    if (b->precision != XY_FIX16) return set_error(XY_EUNSUP, "xy_batch_set_fix16_form: fix16 batches only");
    if (trig < 0 || trig > 2) return set_error(XY_EINVAL, "xy_batch_set_fix16_form: trig must be 0, 1 or 2");
    hipStream_t s = static_cast<hipStream_t>(stream);
    try {
        std::vector<Item> items(kGroups * b->item_cap, Item{-1, -1});
        if (!build_groups(b, trig, allow_unit != 0, force_global != 0, items.data())) return set_error(XY_EUNSUP, "xy_batch_set_fix16_form: work-item list exceeds its capacity");
        hipError_t e = hipStreamSynchronize(s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->d_items, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_err(e, "xy_batch_set_fix16_form");
    } catch (const std::bad_alloc &) {
        return set_error(XY_ENOMEM, "xy_batch_set_fix16_form: out of memory");
    }
    if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
    return XY_OK;
}

extern "C" void xy_batch_free(xy_batch *b)
{
    if (!b) return;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    for (auto &pr : b->events) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    for (hipEvent_t ev : b->ev_join) (void)hipEventDestroy(ev);
    for (hipStream_t st : b->aux) (void)hipStreamDestroy(st);
    if (b->ev_beta) {
        (void)hipEventSynchronize(b->ev_beta);   // the host copy of the ladder is read until then
        (void)hipEventDestroy(b->ev_beta);
    }
    delete b;
}
