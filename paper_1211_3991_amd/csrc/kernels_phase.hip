// Fixed-point path, phase form (graphs from 16384 sites when the temperature
// count is a multiple of 4): the state of a sample is site-major, [site][slot],
// and one launch updates one colour class of the phase-form samples of one
// stream group (App. B's colour phases as launches over many samples).
#include <hip/hip_runtime.h>

#include "fix16_common.hpp"
#include "kernels.hpp"

namespace xy {
namespace {

// A thread (site, q) of a work unit updates slots 4q..4q+3 of one site: the
// neighbour index is read once for the four slots and their four angles are
// one 8-byte load, so graph and gather traffic are shared by four replicas.
// Random words: one Philox call per (site, sweep, slot 4q), word r for slot
// 4q + r.  (cos, sin) of an angle: the form kTrig of Trig (an LDS table
// loaded by the workgroup, or the hardware sine and cosine).
//
// A work unit is two int4: the pool offsets of the columns of the block's
// first two chunks, the sample's state base / 8, the block's first site; then
// sample, phase-sample index, block index in the colour class, and
// kmin | kmax << 8 | (sites - 1) << 16 | (first site's chunk lane) << 24.
// The index loads depend on nothing but the unit.

// The hardware deals the workgroups of a launch to the 8 XCDs in turn
// (workgroup w to XCD w mod 8).  Work unit of workgroup `lin` out of `n`:
// each XCD takes one contiguous run of units, so the neighbouring blocks of a
// sample, whose gathers overlap, meet in the same L2.  A bijection on [0, n).
// With `reverse`, each XCD takes its run from the end: consecutive colour
// phases alternate the direction, so that an XCD starts a launch on the
// samples it finished the previous one with, whose state is still in its L2.
__device__ __forceinline__ int xcd_contiguous(int lin, int n, int reverse)
{
    const int x = lin & 7, k = lin >> 3, per = n >> 3, rem = n & 7;
    const int count = per + (x < rem ? 1 : 0);
    return x * per + min(x, rem) + (reverse ? count - 1 - k : k);
}

// Lane layout of a workgroup: Lq = R/4 threads per site, S sites.
struct PhaseLanes {
    int R, Lq, S, sl, q;
};

__device__ __forceinline__ PhaseLanes phase_lanes(const DevBatch &b)
{
    PhaseLanes pl;
    pl.R = b.R;
    pl.Lq = pl.R >> 2;
    pl.S = kPhaseBlock / pl.Lq;
    // t / Lq through the FP32 reciprocal: exact for t < 256, Lq <= 64, even
    // with a reciprocal 1 ulp off (checked exhaustively)
    pl.sl = (int)(((float)threadIdx.x + 0.5f) * __builtin_amdgcn_rcpf((float)pl.Lq));
    pl.q = (int)threadIdx.x - pl.sl * pl.Lq;
    return pl;
}

// Where one thread's work of a unit lives: its site, whether it stores (lanes
// past the unit's last site mirror that site and store nothing), its chunk
// column (row k at colb + k * 64 * sizeof(Idx)) and the sample's state.
struct UnitPtrs {
    int i;
    bool active;
    const char *colb;
    char *Ab;
};

template <typename Idx>
__device__ __forceinline__ UnitPtrs unit_ptrs(const DevBatch &b, const PhaseLanes &pl, const int4 &ua, const int4 &ub,
                                              int colour)
{
    UnitPtrs p;
    const int n_act = ((ub.w >> 16) & 255) + 1, lnA = (int)((uint32_t)ub.w >> 24);
    p.active = pl.sl < n_act;
    const int sc = min(pl.sl, n_act - 1);
    p.i = ua.w + sc;                                              // colour-major site index in the sample
    const int pos = lnA + sc, ln = pos & 63;
    uint32_t cbase = pos < 64 ? (uint32_t)ua.x : (uint32_t)ua.y;  // pool element offset of the site's chunk
    if (pos >= 128) {                                             // blocks of more than 64 sites (R < 16)
        const SampleDesc &d = b.desc[ub.x];
        const int c0 = d.colour_off[colour];
        cbase = (uint32_t)(d.sell_col + b.i32[d.sell_ptr + d.chunk_off[colour] + ((p.i - c0) >> 6)]);
    }
    p.colb = reinterpret_cast<const char *>(sizeof(Idx) == 2 ? (const void *)b.u16 : (const void *)b.i32) +
             ((uint64_t)cbase + (uint32_t)ln) * sizeof(Idx);
    p.Ab = reinterpret_cast<char *>(b.state) + (uint64_t)(uint32_t)ua.z * 16u;
    return p;
}

// [site][Lq] words of 4 angles; 32-bit byte offsets from the sample's base
__device__ __forceinline__ uint2 &angle_word(char *Ab, const PhaseLanes &pl, int j)
{
    return *reinterpret_cast<uint2 *>(Ab + (__umul24((uint32_t)j, 8u * (uint32_t)pl.Lq) + 8u * (uint32_t)pl.q));
}

// 8 rows of neighbour indices (every chunk has at least 8; a site's rows past
// its degree hold the site itself, which is never its own neighbour)
template <typename Idx>
__device__ __forceinline__ void load_rows(const char *colb, int *jj)
{
    static_assert(kSellRows >= 8, "the phase kernel reads 8 rows of every chunk");
#pragma unroll
    for (int k = 0; k < 8; ++k) jj[k] = (int)*reinterpret_cast<const Idx *>(colb + k * 64 * sizeof(Idx));
}

// the 4-slot angle words of those 8 (unconditional loads keep the wait
// counts exact; a padding row reads the site's own word)
__device__ __forceinline__ void load_words(char *Ab, const PhaseLanes &pl, const int *jj, uint2 *vv)
{
#pragma unroll
    for (int k = 0; k < 8; ++k) vv[k] = angle_word(Ab, pl, jj[k]);
}

// The update of one unit's sites by this thread, from its loaded rows jj and
// neighbour words vv.  kLast: the last sub-sweep of the sweep, which also sums
// the links to lower colours into the energy partials (uses esum and a
// workgroup barrier; every thread of the workgroup calls it).  kMetro: the
// Metropolis sub-sweep (sub == 0; a uniform new angle), else an
// over-relaxation one (the reflection about the local field).
template <typename Idx, bool kLast, int kTrig, bool kMetro>
__device__ __forceinline__ void update_unit(const DevBatch &b, const PhaseLanes &pl, const float2 *tab, float *esum,
                                            int colour, int sub, int max_blocks, uint32_t sweep, const int4 &ua,
                                            const int4 &ub, const UnitPtrs &p, const int *jj, const uint2 *vv,
                                            const uint2 me)
{
    const int R = pl.R, Lq = pl.Lq, S = pl.S, q = pl.q, i = p.i;
    // the unit is the workgroup's: its fields are uniform, and reading them
    // through the scalar unit keeps the sample's descriptor, key schedule and
    // loop bounds scalar (a divergent branch before this point can otherwise
    // leave them in vector registers)
    const int s = __builtin_amdgcn_readfirstlane(ub.x), k_ph = __builtin_amdgcn_readfirstlane(ub.y);
    const int bx = __builtin_amdgcn_readfirstlane(ub.z), uw = __builtin_amdgcn_readfirstlane(ub.w);
    const int kmin = uw & 255, kmax = (uw >> 8) & 255;
    const SampleDesc &d = b.desc[s];
    const uint32_t seed_lo = d.seed_lo, seed_hi = d.seed_hi;   // the Philox key (scalar loads, with the unit's)
    // accept_factor of the inverse temperatures at the thread's four slots
    const float4 fq = *reinterpret_cast<const float4 *>(b.fac_slot + s * R + 4 * q);
    const float factor[4] = {fq.x, fq.y, fq.z, fq.w};
    const int c0 = __builtin_amdgcn_readfirstlane(ua.w) - bx * S; // first site of the colour class
    float hx[4] = {0.f, 0.f, 0.f, 0.f}, hy[4] = {0.f, 0.f, 0.f, 0.f};
    float lx[4] = {0.f, 0.f, 0.f, 0.f}, ly[4] = {0.f, 0.f, 0.f, 0.f};   // last sub-sweep: links to lower colours
    // a row's neighbours are sorted by colour-major index, so the links to
    // lower colours are a prefix: their field is the running sum taken after
    // the last of them
    auto add = [&](uint2 v, int j, bool first) {                // first: the sum starts here
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t w = r < 2 ? v.x : v.y;
            const float2 e = (r & 1) ? Trig<kTrig>::unit_hi(w, tab) : Trig<kTrig>::unit_lo(w, tab);
            hx[r] = first ? e.x : hx[r] + e.x;
            hy[r] = first ? e.y : hy[r] + e.y;
        }
        if (kLast && j < c0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) { lx[r] = hx[r]; ly[r] = hy[r]; }
        }
    };
    // the site's degree, in flight while the first eight rows are added
    // (needed only for blocks with rows past the eighth; uniform branch)
    const int dg = kmax > 8 ? (int)b.u8[d.deg + i] : 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (k < kmin) add(vv[k], jj[k], k == 0);                 // uniform, unmasked
        else if (k < kmax && jj[k] != i) add(vv[k], jj[k], false);
    }
    // rows past the eighth, eight at a time: the indices of a batch, then its
    // neighbour words, all in flight before the first use (the batch count
    // kmax is uniform).  Every load is unconditional, so that the wait counts
    // stay exact: a row at or past the lane's degree reads row dg instead,
    // which lies in the lane's chunk, the chunk after it or the pool's
    // trailing padding rows, and its gather reads the site's own word; only
    // the additions are masked.
    for (int k0 = 8; k0 < kmax; k0 += 8) {
        int j2[8];
        uint2 v2[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int jr = (int)*reinterpret_cast<const Idx *>(p.colb + min(k0 + k, dg) * 64 * (int)sizeof(Idx));
            j2[k] = k0 + k < dg ? jr : i;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) v2[k] = angle_word(p.Ab, pl, j2[k]);
        // (empty volatile asm on the words: the compiler may not sink a load
        // into the masked addition that alone uses it, where it would wait at once)
#pragma unroll
        for (int k = 0; k < 8; ++k) asm volatile("" : "+v"(v2[k].x), "+v"(v2[k].y));
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k0 + k < dg) add(v2[k], j2[k], false);
    }
    // the key is the sample's seed, the same in every lane (s is uniform)
    const U4 w = philox4x32_10_uniform_key(
        {(uint32_t)i, sweep, (uint32_t)(4 * q), tag(kMetro ? kMet : kOR, (uint32_t)sub)}, seed_lo, seed_hi);
    const uint32_t words[4] = {w.x, w.y, w.z, w.w};
    // the angles in the low 16 bits (higher bits are not part of them: the
    // (cos, sin) forms and the packing below ignore them)
    const uint32_t cur_th[4] = {me.x, me.x >> 16, me.y, me.y >> 16};
    uint32_t out[4];
    float e_q[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int slot = 4 * q + r;
        const uint32_t th = cur_th[r];
        const uint32_t th_new = kMetro ? words[r] : field_axis2(hx[r], hy[r]) - th;
        const uint32_t w = r < 2 ? me.x : me.y;
        // an over-relaxation move that is surely accepted skips the energy
        // change (its result is the same); the branch is per lane, and a wave
        // whose lanes all skip jumps over the evaluation
        const bool full = kMetro || !or_accepts_surely(hx[r], hy[r], factor[r], words[r]);
        float2 nu = kLast ? Trig<kTrig>::unit_lo(th_new, tab) : make_float2(0.f, 0.f);   // the energy needs it
        float2 cur = nu;
        bool acc = true;
        if (full) {
            cur = (r & 1) ? Trig<kTrig>::unit_hi(w, tab) : Trig<kTrig>::unit_lo(w, tab);
            if (!kLast) nu = Trig<kTrig>::unit_lo(th_new, tab);
            const float dE = hx[r] * (cur.x - nu.x) + hy[r] * (cur.y - nu.y);
            acc = accept_move(dE, factor[r], words[r], (uint32_t)i, sweep, (uint32_t)slot, (uint32_t)sub, d);
        }
        out[r] = acc ? th_new : th;
        const float2 f = acc ? nu : cur;
        e_q[r] = p.active ? -(f.x * lx[r] + f.y * ly[r]) : 0.f;
    }
    // low halves of out[2k + 1] over those of out[2k], one byte permute each
    if (p.active)
        angle_word(p.Ab, pl, i) =
            make_uint2(__builtin_amdgcn_perm(out[1], out[0], 0x05040100u), __builtin_amdgcn_perm(out[3], out[2], 0x05040100u));
    if constexpr (kLast) {
        // per-slot energy of this unit, summed in a fixed order, to
        // epart[k_ph][colour][block][slot]; a final pass adds the blocks in order
        const int t = threadIdx.x;
#pragma unroll
        for (int r = 0; r < 4; ++r) esum[t * 4 + r] = e_q[r];
        __syncthreads();
        if (t < R) {
            const int qq = t >> 2, r = t & 3;
            double acc = 0.0;
            for (int k = 0; k < S; ++k) acc += (double)esum[(k * Lq + qq) * 4 + r];
            b.epart[(((int64_t)k_ph * kMaxColours + colour) * max_blocks + bx) * R + t] = acc;
        }
    }
}

// One work unit per workgroup (gridDim.x == n_units).
template <typename Idx, bool kLast, int kTrig, bool kMetro>
__global__ __launch_bounds__(kPhaseBlock) void k_fix16_phase(DevBatch b, const int4 *units, int n_units, int colour,
                                                            int sub, int max_blocks, int grp, int reverse)
{
    __shared__ float esum[kLast ? kPhaseBlock * 4 : 1];
    __shared__ float2 tab[Trig<kTrig>::kBytes ? Trig<kTrig>::kBytes / sizeof(float2) : 1];
    const PhaseLanes pl = phase_lanes(b);
    const int u = xcd_contiguous(blockIdx.x, n_units, reverse);
    const int4 ua = units[2 * u], ub = units[2 * u + 1];
    const UnitPtrs p = unit_ptrs<Idx>(b, pl, ua, ub, colour);
    // rows and neighbour words in flight before the first use
    int jj[8];
    uint2 vv[8];
    load_rows<Idx>(p.colb, jj);
    // the site's own word (no other thread writes it during the phase), in
    // flight with the rows
    const uint2 me = angle_word(p.Ab, pl, p.i);
    load_words(p.Ab, pl, jj, vv);
    // the (cos, sin) table of a table form, while the gathers are in flight
    if constexpr (Trig<kTrig>::kBytes > 0) {
        Trig<kTrig>::load(tab, b, threadIdx.x, kPhaseBlock);
        __syncthreads();
    }
    update_unit<Idx, kLast, kTrig, kMetro>(b, pl, tab, esum, colour, sub, max_blocks, b.ctl[grp].sweep, ua, ub, p, jj,
                                           vv, me);
}

}  // namespace

int fix16_phase_sites_per_block(int R) { return kPhaseBlock / (R / 4); }

using PhaseKernel = void (*)(DevBatch, const int4 *, int, int, int, int, int, int);

template <int kTrig, bool kMetro>
PhaseKernel phase_kernel(int idx16, int last)
{
    return idx16 ? (last ? k_fix16_phase<uint16_t, true, kTrig, kMetro> : k_fix16_phase<uint16_t, false, kTrig, kMetro>)
                 : (last ? k_fix16_phase<int32_t, true, kTrig, kMetro> : k_fix16_phase<int32_t, false, kTrig, kMetro>);
}

template <bool kMetro>
PhaseKernel phase_kernel(int trig, int idx16, int last)
{
    return trig == 0 ? phase_kernel<0, kMetro>(idx16, last)
                     : trig == 1 ? phase_kernel<1, kMetro>(idx16, last) : phase_kernel<2, kMetro>(idx16, last);
}

hipError_t launch_fix16_phase(const DevBatch &b, const int4 *units, int colour, int sub,
                              int last, int n_units, int max_blocks, int grp, int reverse, hipStream_t s)
{
    if (n_units == 0) return hipSuccess;
    const PhaseKernel k = sub == 0 ? phase_kernel<true>(b.trig, b.idx16, last) : phase_kernel<false>(b.trig, b.idx16, last);
    hipLaunchKernelGGL(k, dim3((unsigned)n_units), dim3(kPhaseBlock), 0, s, b, units, n_units, colour, sub, max_blocks,
                       grp, reverse);
    return hipGetLastError();
}

}  // namespace xy
