// Fixed-point path: each spin is an angle theta = k * 2pi / 2^16 stored as
// uint16 (an exact representation of the 2^16-state clock model), local
// fields are accumulated in FP32, and energies / observables in FP64.
//
// This file: the workgroup-per-replica forms, used for graphs below the
// phase-form threshold (or any n_T not a multiple of 4), and the measurement
// and tempering kernels of every form; the phase form's colour-phase kernel
// is in kernels_phase.hip.  One workgroup runs one whole sweep of one (sample,
// temperature slot): the replica's angles are staged in LDS (when they fit)
// and the colour phases of App. B become workgroup barriers, so a sweep needs
// no grid-wide synchronisation and no host round trip.  The graph is read in sliced-ELL
// form (64-site chunks, columns stored [k][lane], sites degree-sorted inside
// each colour class): a wave's k-th neighbour indices are one contiguous
// load, and all indices of a site are in flight before the first is used.
// Each lane updates four sites of one colour at a time (four chunks), which
// overlaps their latencies and lets one Philox4x32-10 call supply the random
// words of all four updates.  The workgroups of one sample are placed on one
// XCD by the item order the host builds, so they share its graph in that L2.
//
// Over-relaxation on the clock model: theta' = (q - theta) mod 2^16 with
// q = round(2 phi_h * 2^16 / 2pi), phi_h the angle of the local field.  The
// map is an involution that depends only on the neighbours, so accepting it
// with probability min(1, exp(-beta dE)) keeps detailed balance exactly; dE
// is tiny (the axis is quantised to 2pi/2^17) and almost every move is taken.
#include <hip/hip_runtime.h>

#include "fix16_common.hpp"
#include "kernels.hpp"

namespace xy {
namespace {

constexpr int kUnroll = 8;     // neighbour indices loaded up front per site
constexpr int kObsBlock = 256;
constexpr int kNRed = 11;      // E, m_x, m_y, 4 Fourier sums along x, 4 along y


template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *scratch)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q)
        for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_down(v[q], off, 64);
    __syncthreads();   // scratch may still be read by a previous reduction
    if (lane == 0)
        for (int q = 0; q < NV; ++q) scratch[wave * NV + q] = v[q];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
            for (int q = 0; q < NV; ++q) v[q] += scratch[w * NV + q];
}

// Observables of Sec. 3 from the angles `ang` of one (sample, slot), FP64:
// E = -sum_links cos(theta_i - theta_j) (each link once, at its higher
// endpoint), m = (1/N) sum S_j, F_a = |sum_j S_j e^{i 2pi a_j/L}|^2/N.
template <typename Idx>
__device__ __forceinline__ void observe(const DevBatch &b, const SampleDesc &d, const uint16_t *ang, int stride,
                                        double *scratch, double *dst)
{
    const int32_t *cptr = b.i32 + d.sell_ptr;
    const Idx *col = reinterpret_cast<const Idx *>(sizeof(Idx) == 2 ? (const void *)b.u16 : (const void *)b.i32) + d.sell_col;
    const uint8_t *deg = b.u8 + d.deg;
    const uint32_t *xy = b.u32 + d.coord;
    const double2 *trig = b.f64 + d.trig;
    const double2 *t64 = b.tab64;
    double v[kNRed] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int c = 0; c < d.Q; ++c) {
        const int c0 = d.colour_off[c], c1 = d.colour_off[c + 1], ch0 = d.chunk_off[c];
        for (int ch = wave; ch < d.chunk_off[c + 1] - ch0; ch += nw) {
            const int i = c0 + ch * 64 + lane;
            if (i >= c1) continue;
            const double2 si = unit64(ang[(int64_t)i * stride], t64);
            const int base = cptr[ch0 + ch], dg = deg[i];
            double e = 0.0;
            for (int k = 0; k < dg; ++k) {
                const int j = (int)col[base + k * 64 + lane];
                if (j < i) {
                    const double2 sj = unit64(ang[(int64_t)j * stride], t64);
                    e += si.x * sj.x + si.y * sj.y;
                }
            }
            v[0] -= e;
            const uint32_t p = xy[i];
            const double2 ex = trig[p & 0xFFFFu], ey = trig[p >> 16];
            v[1] += si.x; v[2] += si.y;
            v[3] += si.x * ex.x; v[4] += si.x * ex.y; v[5] += si.y * ex.x; v[6] += si.y * ex.y;
            v[7] += si.x * ey.x; v[8] += si.x * ey.y; v[9] += si.y * ey.x; v[10] += si.y * ey.y;
        }
    }
    block_sum<kNRed>(v, scratch);
    if (threadIdx.x != 0) return;
    const double N = (double)d.n;
    const double mx = v[1] / N, my = v[2] / N, m2 = mx * mx + my * my;
    dst[0] = v[0];
    dst[1] = m2;
    dst[2] = m2 * m2;
    dst[3] = (v[3] * v[3] + v[4] * v[4] + v[5] * v[5] + v[6] * v[6]) / N;
    dst[4] = (v[7] * v[7] + v[8] * v[8] + v[9] * v[9] + v[10] * v[10]) / N;
    dst[5] = mx; dst[6] = my; dst[7] = 0.0;
}


// Where a replica's spins live during a sweep, and how a site's FP32 unit
// vector is obtained.  Angles (uint16, in LDS or global memory) evaluate
// (cos, sin) at every use; kUnitLds keeps the unit vector of every site in LDS
// (8 bytes per site, graphs of up to ~20k sites) next to the angles in global
// memory, so a neighbour costs one LDS read.  The unit vectors are exactly
// Trig<kTrig>::unit of the angles, so all three give identical trajectories.
enum Mode { kAngLds = 0, kAngGlobal = 1, kUnitLds = 2 };

template <int kMode, int kTrig> struct Spins {
    static constexpr bool kStoresUnit = false;   // set() keeps the angle only
    uint16_t *ang;
    const float2 *tab;
    __device__ __forceinline__ float2 nbr(int j) const { return Trig<kTrig>::unit(ang[j], tab); }
    __device__ __forceinline__ uint32_t angle(int i) const { return ang[i]; }
    __device__ __forceinline__ float2 own(int, uint32_t th) const { return Trig<kTrig>::unit(th, tab); }
    __device__ __forceinline__ float2 unit(uint32_t th) const { return Trig<kTrig>::unit(th, tab); }
    __device__ __forceinline__ void set(int i, uint32_t th, float2) const { ang[i] = (uint16_t)th; }
};

template <int kTrig> struct Spins<kUnitLds, kTrig> {
    static constexpr bool kStoresUnit = true;    // set() also stores the unit vector
    uint16_t *ang;          // global memory
    float2 *uv;             // LDS
    const float2 *tab;
    __device__ __forceinline__ float2 nbr(int j) const { return uv[j]; }
    __device__ __forceinline__ uint32_t angle(int i) const { return ang[i]; }
    __device__ __forceinline__ float2 own(int i, uint32_t) const { return uv[i]; }
    __device__ __forceinline__ float2 unit(uint32_t th) const { return Trig<kTrig>::unit(th, tab); }
    __device__ __forceinline__ void set(int i, uint32_t th, float2 u) const { ang[i] = (uint16_t)th; uv[i] = u; }
};

// One colour phase of one sub-sweep for this workgroup's replica: every site
// of colour class [c0, c1) is updated once (Metropolis when sub == 0, else
// over-relaxation).  Returns, when kLast, the energy of the links from the
// updated sites to lower colours (their final values in the last sub-sweep).
template <bool kLast, int kWaves, int kGroup, typename Idx, typename Sp>
__device__ __forceinline__ double colour_phase(const SampleDesc &d, const Sp &sp,
                                               const int32_t *cptr, const int32_t *cw, const Idx *col,
                                               const uint8_t *deg, int c0, int c1, int ch0, int nch, int wave,
                                               int lane, uint32_t sweep, int slot, int sub, float factor)
{
    static_assert(kGroup == 1 || kGroup == 2 || kGroup == 4, "groups must tile the 4-chunk key groups");
    double e_acc = 0.0;
    for (int g0 = wave * kGroup; g0 < nch; g0 += kWaves * kGroup) {
        // chunk records are the same for the whole wave: scalar loads
        int site[kGroup], dg[kGroup], base[kGroup], wmin[kGroup];
        Idx jj[kGroup][kUnroll];
#pragma unroll
        for (int r = 0; r < kGroup; ++r) {
            const int ch = g0 + r;
            site[r] = c0 + ch * 64 + lane;
            const bool have = ch < nch;
            base[r] = have ? __builtin_amdgcn_readfirstlane(cptr[ch0 + ch]) : 0;
            wmin[r] = have ? __builtin_amdgcn_readfirstlane(cw[ch0 + ch]) & 255 : 0;
            dg[r] = (have && site[r] < c1) ? (int)deg[site[r]] : 0;
        }
#pragma unroll
        for (int r = 0; r < kGroup; ++r)
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) jj[r][k] = col[base[r] + k * 64 + lane];

        // local fields: the first wmin neighbours of every lane of a chunk are
        // real (uniform loop, no masking); lanes of higher degree finish alone
        float hx[kGroup], hy[kGroup], lx[kGroup], ly[kGroup];
#pragma unroll
        for (int r = 0; r < kGroup; ++r) {
            hx[r] = hy[r] = lx[r] = ly[r] = 0.f;
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                if (k < wmin[r]) {
                    const int j = (int)jj[r][k];
                    const float2 u = sp.nbr(j);
                    hx[r] += u.x; hy[r] += u.y;
                    if (kLast && j < c0) { lx[r] += u.x; ly[r] += u.y; }
                }
            }
            for (int k = kUnroll; k < wmin[r]; ++k) {                // wide chunks (uniform)
                const int j = (int)col[base[r] + k * 64 + lane];
                const float2 u = sp.nbr(j);
                hx[r] += u.x; hy[r] += u.y;
                if (kLast && j < c0) { lx[r] += u.x; ly[r] += u.y; }
            }
            for (int k = wmin[r]; k < dg[r]; ++k) {                   // lanes above the chunk minimum
                const int j = (int)col[base[r] + k * 64 + lane];
                const float2 u = sp.nbr(j);
                hx[r] += u.x; hy[r] += u.y;
                if (kLast && j < c0) { lx[r] += u.x; ly[r] += u.y; }
            }
        }

        // Random words: one Philox call per 4-chunk key group (chunks 4m..4m+3
        // of the colour class), keyed by the first chunk's site of this lane;
        // word (chunk mod 4) drives that chunk's site.  The keying depends on
        // the site only, never on the launch shape, so every storage form and
        // block size gives the same trajectory.  Metropolis: 16 proposal bits
        // | 16 uniform bits; over-relaxation: the top 16 bits as the uniform.
        uint32_t words[kGroup];
        {
            const int kg0 = g0 & ~3;
            const U4 w = philox4x32_10({(uint32_t)(c0 + kg0 * 64 + lane), sweep, (uint32_t)slot,
                                        tag(sub == 0 ? kMet : kOR, (uint32_t)sub)}, d.seed_lo, d.seed_hi);
            const uint32_t all[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int r = 0; r < kGroup; ++r) words[r] = all[(g0 - kg0 + r) & 3];
        }
        float e_grp = 0.f;
#pragma unroll
        for (int r = 0; r < kGroup; ++r) {
            if (site[r] >= c1 || g0 + r >= nch) continue;
            const uint32_t th = sp.angle(site[r]);
            uint32_t th_new;
            if (sub == 0) {
                th_new = words[r] & 0xFFFFu;                          // uniform proposal
            } else {
                th_new = (field_axis2(hx[r], hy[r]) - th) & 0xFFFFu;   // reflection
            }
            // a surely accepted reflection skips its energy change (the same
            // decision, see or_accepts_surely); the proposal's unit vector is
            // still needed where it is stored or enters the energy
            constexpr bool kNeedNu = Sp::kStoresUnit || kLast;
            const bool full = sub == 0 || !or_accepts_surely(hx[r], hy[r], factor, words[r]);
            float2 nu = kNeedNu ? sp.unit(th_new) : make_float2(0.f, 0.f);
            float2 cur = nu;
            bool accept = true;
            if (full) {
                cur = sp.own(site[r], th);
                if (!kNeedNu) nu = sp.unit(th_new);
                const float dE = hx[r] * (cur.x - nu.x) + hy[r] * (cur.y - nu.y);
                accept = accept_move(dE, factor, words[r], (uint32_t)site[r], sweep, (uint32_t)slot, (uint32_t)sub, d);
            }
            if (accept) sp.set(site[r], th_new, nu);
            if (kLast) {
                const float2 f = accept ? nu : cur;
                e_grp -= f.x * lx[r] + f.y * ly[r];
            }
        }
        if (kLast) e_acc += (double)e_grp;
    }
    return e_acc;
}

// LDS map: [double scratch 16*kNRed][trig table][replica: uint16 angles
// (kAngLds) or float2 unit vectors (kUnitLds), n_pad entries]
constexpr size_t kOffTab = 1536;

template <int kMode, int kTrig, int kBlock, typename Idx>
__global__ __launch_bounds__(kBlock) void k_fix16_sweep(DevBatch b, const Item *items, int n_or, int measure)
{
    constexpr int kW = kBlock / 64;
    // sites per lane at a time: 4 where the replica is in LDS; 2 from global
    // memory (fewer registers, so two workgroups share a CU to hide latency)
    constexpr int kG = kMode == kAngGlobal ? 2 : 4;
    extern __shared__ __align__(16) unsigned char smem[];
    const Item it = items[blockIdx.x];
    if (it.sample < 0) return;
    const int s = it.sample, slot = it.slot, R = b.R;
    const SampleDesc &d = b.desc[s];
    const int n = d.n, n_pad = (n + 7) & ~7, tid = threadIdx.x;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    double *scratch = reinterpret_cast<double *>(smem);
    float2 *tab = reinterpret_cast<float2 *>(smem + kOffTab);
    unsigned char *rep = smem + kOffTab + Trig<kTrig>::kBytes;
    uint16_t *g_ang = static_cast<uint16_t *>(b.state) + d.state + (int64_t)slot * n_pad;

    Spins<kMode, kTrig> sp;
    sp.tab = tab;
    sp.ang = kMode == kAngLds ? reinterpret_cast<uint16_t *>(rep) : g_ang;
    Trig<kTrig>::load(tab, b, tid, kBlock);
    if constexpr (kMode == kAngLds) {
        const uint4 *src = reinterpret_cast<const uint4 *>(g_ang);
        uint4 *dst = reinterpret_cast<uint4 *>(rep);
        for (int k = tid; k < n_pad / 8; k += kBlock) dst[k] = src[k];
    }
    if constexpr (kMode == kUnitLds) {
        sp.uv = reinterpret_cast<float2 *>(rep);
        __syncthreads();                                      // the table must be in place
        for (int k = tid; k < n; k += kBlock) sp.uv[k] = Trig<kTrig>::unit(g_ang[k], tab);
    }
    __syncthreads();

    const float factor = b.fac_slot[s * R + slot];
    const uint32_t sweep = b.ctl->sweep;
    const int32_t *cptr = b.i32 + d.sell_ptr;
    const int32_t *cw = b.i32 + d.sell_w;
    const Idx *col = reinterpret_cast<const Idx *>(sizeof(Idx) == 2 ? (const void *)b.u16 : (const void *)b.i32) + d.sell_col;
    const uint8_t *deg = b.u8 + d.deg;
    double e_acc = 0.0;

    for (int sub = 0; sub <= n_or; ++sub) {
        const bool last = (sub == n_or);
        for (int c = 0; c < d.Q; ++c) {
            const int c0 = d.colour_off[c], c1 = d.colour_off[c + 1];
            const int ch0 = d.chunk_off[c], nch = d.chunk_off[c + 1] - ch0;
            if (last)
                e_acc += colour_phase<true, kW, kG, Idx>(d, sp, cptr, cw, col, deg, c0, c1, ch0, nch, wave, lane, sweep,
                                                     slot, sub, factor);
            else
                colour_phase<false, kW, kG, Idx>(d, sp, cptr, cw, col, deg, c0, c1, ch0, nch, wave, lane, sweep, slot,
                                             sub, factor);
            __syncthreads();
        }
    }

    {
        double v[1] = {e_acc};
        block_sum<1>(v, scratch);
        if (tid == 0) b.E_slot[s * R + slot] = v[0];
    }
    if (measure) observe<Idx>(b, d, sp.ang, 1, scratch, b.obs_slot + ((int64_t)s * R + slot) * XY_NOBS);
    if constexpr (kMode == kAngLds) {
        __syncthreads();
        const uint4 *src = reinterpret_cast<const uint4 *>(rep);
        uint4 *dst = reinterpret_cast<uint4 *>(g_ang);
        for (int k = tid; k < n_pad / 8; k += kBlock) dst[k] = src[k];
    }
}

// Random initial angles: 16 uniform bits per (sample, slot, site).
__global__ __launch_bounds__(256) void k_fix16_init(DevBatch b)
{
    const int s = blockIdx.y;
    const SampleDesc &d = b.desc[s];
    const int n_pad = (d.n + 7) & ~7;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)n_pad * b.R) return;
    // element t of the sample's block: slot-major [slot][site_pad] or
    // site-major [site][slot]; the value depends on (site, slot) only
    const int slot = d.layout ? (int)(t % b.R) : (int)(t / n_pad);
    const int site = d.layout ? (int)(t / b.R) : (int)(t % n_pad);
    uint16_t *S = static_cast<uint16_t *>(b.state) + d.state;
    uint16_t v = 0;
    if (site < d.n) {
        const U4 w = philox4x32_10({(uint32_t)site, 0u, (uint32_t)slot, tag(kInit)}, d.seed_lo, d.seed_hi);
        v = (uint16_t)(w.x & 0xFFFFu);
    }
    S[t] = v;
}

// Stand-alone measurement from the state in global memory.
template <typename Idx>
__global__ __launch_bounds__(kObsBlock) void k_fix16_observe(DevBatch b, double *out_by_T)
{
    __shared__ double scratch[(kObsBlock / 64) * kNRed];
    const int slot = blockIdx.x, s = blockIdx.y, R = b.R;
    const SampleDesc &d = b.desc[s];
    const int n_pad = (d.n + 7) & ~7;
    const uint16_t *ang = static_cast<const uint16_t *>(b.state) + d.state +
                          (d.layout ? (int64_t)slot : (int64_t)slot * n_pad);
    double o[XY_NOBS];
    observe<Idx>(b, d, ang, d.layout ? R : 1, scratch, o);
    if (threadIdx.x != 0) return;
    double *dst = out_by_T ? out_by_T + ((int64_t)s * R + b.T_of_slot[s * R + slot]) * XY_NOBS
                           : b.obs_slot + ((int64_t)s * R + slot) * XY_NOBS;
    for (int q = 0; q < XY_NOBS; ++q) dst[q] = o[q];
    b.E_slot[s * R + slot] = o[0];
}



// Energies of the phase-form samples from the per-block sums of the last
// sub-sweep.  One block per sample; thread (part, slot) adds every P-th block
// partial of each colour in order, then part 0 adds the P sums in order.
constexpr int kPhaseEnergyBlock = 1024;

__global__ __launch_bounds__(kPhaseEnergyBlock) void k_fix16_phase_energy(DevBatch b, const int32_t *phase_samples,
                                                                          int k_first, int max_blocks)
{
    __shared__ double red[kPhaseEnergyBlock];
    const int R = b.R, S = kPhaseBlock / (R >> 2), P = kPhaseEnergyBlock / R;   // R <= 256, so P >= 4
    const int k = k_first + (int)blockIdx.x, s = phase_samples[k];
    const SampleDesc &d = b.desc[s];
    const int t = threadIdx.x, part = t / R, slot = t % R;
    double e = 0.0;
    if (part < P) {
        for (int c = 0; c < d.Q; ++c) {
            const int nb = (d.colour_off[c + 1] - d.colour_off[c] + S - 1) / S;
            const double *src = b.epart + ((int64_t)k * kMaxColours + c) * max_blocks * R + slot;
            // eight loads in flight, added in block order
            int blk = part;
            for (; blk + 7 * P < nb; blk += 8 * P) {
                double a[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) a[u] = src[(int64_t)(blk + u * P) * R];
#pragma unroll
                for (int u = 0; u < 8; ++u) e += a[u];
            }
            for (; blk < nb; blk += P) e += src[(int64_t)blk * R];
        }
    }
    red[t] = e;
    __syncthreads();
    if (t < R) {
        double acc = 0.0;
        for (int q = 0; q < P; ++q) acc += red[q * R + t];
        b.E_slot[s * R + t] = acc;
    }
}

// Energies (and observables when full) of the phase-form samples, stage 1:
// block b of a sample covers a contiguous site range for all slots, S sites
// at a time; FP64 unit vectors of the 16-bit angles.  Each link is counted
// once, at its higher endpoint.  Stage 2 adds the kObsBlocks partials in
// block order.
constexpr int kObsBlocks = 64;

template <typename Idx>
__global__ __launch_bounds__(kObsBlock) void k_fix16_observe_sm_partial(DevBatch b, const int32_t *phase_samples,
                                                                       int k_first, int full)
{
    __shared__ double red[kObsBlock * 4];
    __shared__ double2 t64[512];          // the FP64 two-level (cos, sin) table
    const int kk = k_first + (int)blockIdx.y, s = phase_samples[kk], R = b.R, Lq = R >> 2;
    const SampleDesc &d = b.desc[s];
    for (int k = threadIdx.x; k < 512; k += kObsBlock) t64[k] = b.tab64[k];
    __syncthreads();
    // thread (site, q) handles slots 4q..4q+3 of one site at a time, the
    // block's S sites in parallel: one 8-byte gather per neighbour for four
    // slots, eight in flight
    const int S = kObsBlock / Lq, t = threadIdx.x, q = t % Lq, sl = t / Lq;
    const int per = (d.n + kObsBlocks - 1) / kObsBlocks;
    const int i0 = blockIdx.x * per, i1 = min(d.n, i0 + per);
    double v[kNRed][4];
#pragma unroll
    for (int qq = 0; qq < kNRed; ++qq)
#pragma unroll
        for (int r = 0; r < 4; ++r) v[qq][r] = 0.0;
    if (sl < S) {
        const uint2 *A = reinterpret_cast<const uint2 *>(static_cast<const uint16_t *>(b.state) + d.state);
        const int32_t *cptr = b.i32 + d.sell_ptr;
        const Idx *col = reinterpret_cast<const Idx *>(sizeof(Idx) == 2 ? (const void *)b.u16 : (const void *)b.i32) + d.sell_col;
        const uint8_t *deg = b.u8 + d.deg;
        const uint32_t *xy = b.u32 + d.coord;
        const double2 *trig = b.f64 + d.trig;
        int c = 0;
        for (int i = i0 + sl; i < i1; i += S) {
            while (i >= d.colour_off[c + 1]) ++c;
            const int rel = i - d.colour_off[c];
            const int base = cptr[d.chunk_off[c] + (rel >> 6)], ln = rel & 63;
            const int dg = deg[i];
            const uint2 me = A[(uint32_t)i * (uint32_t)Lq + (uint32_t)q];
            const uint32_t th[4] = {me.x & 0xFFFFu, me.x >> 16, me.y & 0xFFFFu, me.y >> 16};
            double2 si[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) si[r] = unit64(th[r], t64);
            // rows past a chunk's width hold valid sites (next chunk or padding)
            int jj[8];
            uint2 vv[8];
            const Idx *cl = col + (uint32_t)(base + ln);
#pragma unroll
            for (int k = 0; k < 8; ++k) jj[k] = k < dg ? (int)cl[k * 64] : i;
#pragma unroll
            for (int k = 0; k < 8; ++k) vv[k] = A[(uint32_t)jj[k] * (uint32_t)Lq + (uint32_t)q];
            double e[4] = {0.0, 0.0, 0.0, 0.0};
            // each link once, at its higher endpoint (j < i), in row order;
            // S_i . S_j = cos(theta_i - theta_j), the difference taken exactly
            // on the 2^16 circle: cos(a + b) from the two-level table
            auto link = [&](uint2 w) {
                const uint32_t tj[4] = {w.x & 0xFFFFu, w.x >> 16, w.y & 0xFFFFu, w.y >> 16};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const uint32_t dl = (th[r] - tj[r]) & 0xFFFFu;
                    const double2 a = t64[dl >> 8], cc = t64[256 + (dl & 255u)];
                    e[r] += a.x * cc.x - a.y * cc.y;
                }
            };
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (k < dg && jj[k] < i) link(vv[k]);
            for (int k = 8; k < dg; ++k) {
                const int j = (int)cl[k * 64];
                if (j < i) link(A[(uint32_t)j * (uint32_t)Lq + (uint32_t)q]);
            }
            const uint32_t p = xy[i];
            const double2 ex = trig[p & 0xFFFFu], ey = trig[p >> 16];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                v[0][r] -= e[r];
                if (full) {
                    v[1][r] += si[r].x; v[2][r] += si[r].y;
                    v[3][r] += si[r].x * ex.x; v[4][r] += si[r].x * ex.y;
                    v[5][r] += si[r].y * ex.x; v[6][r] += si[r].y * ex.y;
                    v[7][r] += si[r].x * ey.x; v[8][r] += si[r].x * ey.y;
                    v[9][r] += si[r].y * ey.x; v[10][r] += si[r].y * ey.y;
                }
            }
        }
    }
    // per quantity: the block's sites added in a fixed order, per slot
    for (int qq = 0; qq < kNRed; ++qq) {
#pragma unroll
        for (int r = 0; r < 4; ++r) red[t * 4 + r] = v[qq][r];
        __syncthreads();
        if (t < R) {
            const int qd = t >> 2, r = t & 3;
            double acc = 0.0;
            for (int k = 0; k < S; ++k) acc += red[(k * Lq + qd) * 4 + r];
            b.partial[(((int64_t)kk * kObsBlocks + blockIdx.x) * R + t) * kNRed + qq] = acc;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kObsBlock) void k_fix16_observe_sm_final(DevBatch b, const int32_t *phase_samples,
                                                                     int k_first, int n_phase, int full)
{
    const int R = b.R;
    const int64_t t = (int64_t)blockIdx.x * kObsBlock + threadIdx.x;
    if (t >= (int64_t)n_phase * R) return;
    const int k = k_first + (int)(t / R), slot = (int)(t % R), s = phase_samples[k];
    const SampleDesc &d = b.desc[s];
    double v[kNRed];
    for (int qq = 0; qq < kNRed; ++qq) v[qq] = 0.0;
    for (int blk = 0; blk < kObsBlocks; ++blk)
        for (int qq = 0; qq < kNRed; ++qq) v[qq] += b.partial[(((int64_t)k * kObsBlocks + blk) * R + slot) * kNRed + qq];
    b.E_slot[s * R + slot] = v[0];
    if (!full) return;
    const double N = (double)d.n;
    const double mx = v[1] / N, my = v[2] / N, m2 = mx * mx + my * my;
    double *dst = b.obs_slot + ((int64_t)s * R + slot) * XY_NOBS;
    dst[0] = v[0];
    dst[1] = m2;
    dst[2] = m2 * m2;
    dst[3] = (v[3] * v[3] + v[4] * v[4] + v[5] * v[5] + v[6] * v[6]) / N;
    dst[4] = (v[7] * v[7] + v[8] * v[8] + v[9] * v[9] + v[10] * v[10]) / N;
    dst[5] = mx; dst[6] = my; dst[7] = 0.0;
}

template <int kMode, int kTrig, int kBlock, typename Idx>
hipError_t launch_sweep_t(const DevBatch &b, const Item *items, int n_items, int n_or, int measure, size_t lds,
                          hipStream_t s)
{
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fix16_sweep<kMode, kTrig, kBlock, Idx>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr_set = true;
    }
    hipLaunchKernelGGL((k_fix16_sweep<kMode, kTrig, kBlock, Idx>), dim3(n_items), dim3(kBlock), lds, s, b, items,
                       n_or, measure);
    return hipGetLastError();
}

template <int kMode, int kBlock, typename Idx>
hipError_t launch_sweep_i(const DevBatch &b, const Item *items, int n_items, int n_or, int measure, size_t lds,
                          hipStream_t s)
{
    switch (b.trig) {
    case 0: return launch_sweep_t<kMode, 0, kBlock, Idx>(b, items, n_items, n_or, measure, lds, s);
    case 1: return launch_sweep_t<kMode, 1, kBlock, Idx>(b, items, n_items, n_or, measure, lds, s);
    default: return launch_sweep_t<kMode, 2, kBlock, Idx>(b, items, n_items, n_or, measure, lds, s);
    }
}

template <int kMode, int kBlock>
hipError_t launch_sweep_m(const DevBatch &b, const Item *items, int n_items, int n_or, int measure, size_t lds,
                          hipStream_t s)
{
    return b.idx16 ? launch_sweep_i<kMode, kBlock, uint16_t>(b, items, n_items, n_or, measure, lds, s)
                   : launch_sweep_i<kMode, kBlock, int32_t>(b, items, n_items, n_or, measure, lds, s);
}

}  // namespace

size_t fix16_lds_bytes(int n_pad, int trig, int mode)
{
    const size_t tab = trig == 0 ? Trig<0>::kBytes : trig == 1 ? Trig<1>::kBytes : Trig<2>::kBytes;
    const size_t per_site = mode == kAngLds ? 2 : mode == kUnitLds ? 8 : 0;
    return kOffTab + tab + per_site * (size_t)n_pad;
}

hipError_t launch_fix16_init(const DevBatch &b, int max_n, hipStream_t s)
{
    const int64_t threads = (int64_t)((max_n + 7) & ~7) * b.R;
    dim3 grid((unsigned)((threads + 255) / 256), (unsigned)b.G);
    hipLaunchKernelGGL(k_fix16_init, grid, dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_fix16_sweep(const DevBatch &b, const Item *items, int n_items, int mode, int block, int n_or,
                              int measure, size_t lds_bytes, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    if (mode == kUnitLds && block == 256)
        return launch_sweep_m<kUnitLds, 256>(b, items, n_items, n_or, measure, lds_bytes, s);
    if (mode == kUnitLds) return launch_sweep_m<kUnitLds, 1024>(b, items, n_items, n_or, measure, lds_bytes, s);
    if (mode == kAngLds) return launch_sweep_m<kAngLds, 1024>(b, items, n_items, n_or, measure, lds_bytes, s);
    return launch_sweep_m<kAngGlobal, 512>(b, items, n_items, n_or, measure, lds_bytes, s);
}


hipError_t launch_fix16_phase_energy(const DevBatch &b, const int32_t *phase_samples, int k_first, int n_phase,
                                     int max_blocks, hipStream_t s)
{
    if (n_phase == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fix16_phase_energy, dim3((unsigned)n_phase), dim3(kPhaseEnergyBlock), 0, s, b, phase_samples,
                       k_first, max_blocks);
    return hipGetLastError();
}

hipError_t launch_fix16_observe_sm(const DevBatch &b, const int32_t *phase_samples, int k_first, int n_phase,
                                   int full, hipStream_t s)
{
    if (n_phase == 0) return hipSuccess;
    dim3 grid(kObsBlocks, (unsigned)n_phase);
    if (b.idx16)
        hipLaunchKernelGGL(k_fix16_observe_sm_partial<uint16_t>, grid, dim3(kObsBlock), 0, s, b, phase_samples, k_first,
                           full);
    else
        hipLaunchKernelGGL(k_fix16_observe_sm_partial<int32_t>, grid, dim3(kObsBlock), 0, s, b, phase_samples, k_first,
                           full);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)n_phase * b.R;
    hipLaunchKernelGGL(k_fix16_observe_sm_final, dim3((unsigned)((n + kObsBlock - 1) / kObsBlock)), dim3(kObsBlock),
                       0, s, b, phase_samples, k_first, n_phase, full);
    return hipGetLastError();
}

hipError_t launch_fix16_observe(const DevBatch &b, double *out_by_T, hipStream_t s)
{
    if (b.idx16)
        hipLaunchKernelGGL(k_fix16_observe<uint16_t>, dim3((unsigned)b.R, (unsigned)b.G), dim3(kObsBlock), 0, s, b,
                           out_by_T);
    else
        hipLaunchKernelGGL(k_fix16_observe<int32_t>, dim3((unsigned)b.R, (unsigned)b.G), dim3(kObsBlock), 0, s, b,
                           out_by_T);
    return hipGetLastError();
}

}  // namespace xy
