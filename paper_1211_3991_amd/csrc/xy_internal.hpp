// Internal definitions shared by the library's host and device sources.
// Nothing here is part of the public ABI (include/xy_levy.h).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/xy_levy.h"

#if defined(__HIPCC__)
#define XY_HD __host__ __device__ __forceinline__
#else
#define XY_HD inline
#endif

namespace xy {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11).  The counter-based
// generator replaces the paper's per-thread lagged-Fibonacci streams (App. B,
// "Memory management"): a draw is a pure function of (key, counter), so no
// generator state is stored and any draw can be recomputed anywhere.
// ---------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

XY_HD U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
    const uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    const uint32_t kBumpA = 0x9E3779B9u, kBumpB = 0xBB67AE85u;
#if defined(__HIPCC__)
#pragma unroll
#endif
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = (uint64_t)kMulA * c.x;
        const uint64_t pb = (uint64_t)kMulB * c.z;
        U4 n;
        n.x = (uint32_t)(pb >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)pb;
        n.z = (uint32_t)(pa >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)pa;
        c = n;
        k0 += kBumpA;
        k1 += kBumpB;
    }
    return c;
}

// Draw purposes: top byte of counter word w.  Word z carries the slot,
// word y the sweep, word x the site (or the draw index).
enum Purpose : uint32_t { kGraph = 1, kInit = 2, kMet = 3, kMetAcc = 4, kOR = 5, kPT = 6, kWalk = 7, kWalkStart = 8 };

XY_HD uint32_t tag(Purpose p, uint32_t sub = 0, uint32_t attempt = 0)
{
    return ((uint32_t)p << 24) | (sub << 16) | attempt;
}

// 53-bit uniform in [0,1): 32 bits of `hi` above the top 21 bits of `lo`.
XY_HD double unit53(uint32_t hi, uint32_t lo)
{
    const uint64_t bits = ((uint64_t)hi << 21) | (uint64_t)(lo >> 11);
    return (double)bits * 0x1.0p-53;
}

// ---------------------------------------------------------------------------
// Host graph object.
// ---------------------------------------------------------------------------
}  // namespace xy

struct xy_graph {
    int n = 0, m = 0, L = 0, Q = 0, max_deg = 0;
    int64_t attempts = 0;
    std::vector<int32_t> edges;       // 2m, acceptance order (i, j)
    std::vector<int32_t> colour;      // by lattice index
    std::vector<int32_t> perm;        // colour-major index -> lattice index
    std::vector<int32_t> inv;         // lattice index -> colour-major index
    std::vector<int32_t> colour_off;  // Q + 1
    std::vector<int32_t> row_ptr;     // n + 1, colour-major
    std::vector<int32_t> col;         // 2m, colour-major neighbours, ascending per row
    std::vector<int32_t> cx, cy;      // lattice coordinates by lattice index
};

namespace xy {

constexpr int kMaxColours = 31;
constexpr int kMaxPhaseStreams = 4;   // streams of the phase form's sample groups (the caller's and three more)
constexpr int kMaxPhaseGroups = 8;    // sample groups of the phase form, each with its own control block
constexpr int kMaxT = 256;

xy_status set_error(xy_status code, const std::string &msg);

// Builds colouring + colour-sorted CSR of a graph whose n, m, L, edges, cx,
// cy are filled.  Returns XY_OK or an error status.
xy_status finish_graph(xy_graph &g);

// ---------------------------------------------------------------------------
// Device-side descriptors (plain data, copied into the graph region).
// ---------------------------------------------------------------------------
struct SampleDesc {
    int32_t n, Q, L, max_deg;
    int64_t row_ptr;      // element offsets into the graph region's int32 pool
    int64_t col;
    int64_t perm;
    int64_t coord;        // uint32 pool: x | y << 16, by colour-major index
    int64_t trig;         // double2 pool: (cos, sin)(2 pi x / L), x < L
    int64_t state;        // element offset into the state region (double2 or uint16)
    int64_t sell_ptr;     // fix16: int32 pool, first column entry of each 64-site chunk (+1 end)
    int64_t sell_w;       // fix16: int32 pool, per chunk: smallest degree | largest degree << 8
    int64_t sell_col;     // fix16: u16 or int32 pool, columns chunk by chunk, [k][lane] inside a chunk
    int64_t deg;          // fix16: u8 pool, degree by site
    uint32_t seed_lo, seed_hi;
    int32_t layout;       // fix16 state: 0 slot-major [slot][site_pad], 1 site-major [site][slot]
    int32_t pad_;
    int32_t colour_off[kMaxColours + 1];
    int32_t chunk_off[kMaxColours + 1];   // fix16: first chunk of each colour class
};

struct Ctl {
    uint32_t sweep;        // sweeps completed
    uint32_t n_records;    // records written (may exceed max_records: then dropped)
    uint32_t log_base;     // sweep at which the decision log was enabled
    uint32_t pad;
};

// Work region layout (byte offsets computed by layout_work()).
struct WorkLayout {
    size_t ctl, beta, slot_of_T, T_of_slot, fac_slot, E_slot, obs_slot, pt_acc, pt_try, partial, epart, total;
};

struct GraphLayout {
    size_t desc, i32_pool, u32_pool, f64_pool, u16_pool, u8_pool, items, phase, tab32, tab2k, tab64, total;
    size_t n_i32, n_u32, n_f64, n_u16, n_u8;
};

// Sliced-ELL form of a graph used by the fixed-point sweep.  Sites are
// renumbered inside each colour class by decreasing degree within windows of
// consecutive sites (ties: colour-major order), so the 64 sites of a chunk
// have nearly equal degree; chunk columns
// are stored k-major ([k][lane]) so that the k-th neighbour loads of a wave are
// contiguous.  A chunk has at least kSellRows rows; a site's rows past its
// degree hold the site itself (lanes past the class end hold 0).
constexpr int kSellRows = 8;
struct Sell {
    std::vector<int32_t> order;      // fix16 index -> colour-major index
    std::vector<int32_t> chunk_ptr;  // n_chunks + 1
    std::vector<int32_t> chunk_w;    // n_chunks: smallest degree | largest degree << 8
    std::vector<int32_t> col;        // fix16 indices
    std::vector<uint8_t> deg;
    std::vector<int32_t> chunk_off;  // Q + 1
};
// window: sites per degree-sorted window (the whole class when >= n).
Sell build_sell(const xy_graph &g, int window);

// Window for a graph of n sites in a workgroup-per-replica form: whole
// classes when a replica fits in LDS (n <= 65536 on gfx950; neighbour
// locality is irrelevant there and uniform chunks matter), 4096-site windows
// otherwise (gathers from global memory).
inline int sell_window(int n) { return n <= 65536 ? n : 4096; }
// Window of the phase form, whose gathers always come from global memory: a
// window of a class covers a compact band of the lattice, so the blocks that
// run together gather from a small part of the state (measured on 64 x L=256:
// whole classes 317, 4096 sites 323.5, 8192 323, 16384 318.5 updates/ns; on
// 32 x L=512: 2048 297, 4096 299, 8192 299, 16384 287).
constexpr int kPhaseSellWindow = 4096;

// One fix16 work item: a (sample, slot) pair run by one workgroup.
struct Item { int32_t sample, slot; };

}  // namespace xy
