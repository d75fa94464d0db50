// FP64 plain path: spins are FP64 unit vectors, one thread per (site, slot)
// of one colour class, one launch per colour phase (App. B: sites of one
// colour are updated synchronously, colours one after another).  Built with
// -ffp-contract=off: every state operation is a correctly rounded + - * / or
// sqrt evaluated in the order written, so the trajectory is bit-identical to
// a sequential FP64 evaluation of the same sweep.
//
// Also holds the end-of-sweep kernel (parallel tempering, records, sweep
// counter) that both precisions share.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace xy {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ U4 draw(const SampleDesc &d, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3)
{
    return philox4x32_10({c0, c1, c2, c3}, d.seed_lo, d.seed_hi);
}

// Uniform direction on the circle: points of the square [-1,1)^2 drawn until
// one falls in the unit disk (0 < r^2 <= 1), then normalised.  Only correctly
// rounded operations touch the result.
__device__ __forceinline__ double2 uniform_direction(const SampleDesc &d, uint32_t site, uint32_t sweep,
                                                     uint32_t slot, Purpose p)
{
    for (uint32_t attempt = 0; attempt < 64; ++attempt) {
        const U4 w = draw(d, site, sweep, slot, tag(p, 0, attempt));
        const double x = 2.0 * unit53(w.x, w.y) - 1.0;
        const double y = 2.0 * unit53(w.z, w.w) - 1.0;
        const double r2 = x * x + y * y;
        if (r2 > 1.0 || r2 == 0.0) continue;
        const double r = sqrt(r2);
        return make_double2(x / r, y / r);
    }
    return make_double2(1.0, 0.0);
}

__global__ __launch_bounds__(kBlock) void k_fp64_init(DevBatch b)
{
    const SampleDesc d = b.desc[blockIdx.y];
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int site = (int)(t / b.R), slot = (int)(t % b.R);
    if (site >= d.n) return;
    double2 *S = static_cast<double2 *>(b.state) + d.state;
    const uint32_t lattice = (uint32_t)b.i32[d.perm + site];
    S[(int64_t)site * b.R + slot] = uniform_direction(d, lattice, 0u, (uint32_t)slot, kInit);
}

// One colour phase of one sub-sweep.  Thread t of sample blockIdx.y handles
// site colour_off[c] + t / R in slot t % R; neighbouring threads read
// neighbouring slots of the same site, so every gather is a contiguous run of
// R * 16 bytes.
// energy: the last sub-sweep of a sweep that tempers: the replica energies
// are summed here.  A row's neighbours are sorted by colour-major index, so
// its links to lower colours (whose sites are final in this sub-sweep) are a
// prefix, and their field is the running sum taken after the last of them;
// E = -sum_i S_i . (that field) counts every link once, at its upper colour.
// Per block and slot the site terms are added in site order into
// epart[s][colour][block][slot] (colour stride n_col, block stride
// max_blocks); k_fp64_energy_final adds the blocks in order.
__global__ __launch_bounds__(kBlock) void k_fp64_phase(DevBatch b, int colour, int met, int energy, int n_col,
                                                      int max_blocks)
{
    __shared__ double esum[kBlock];
    const int s = blockIdx.y;
    const SampleDesc &d = b.desc[s];
    if (colour >= d.Q) return;
    const int c0 = d.colour_off[colour], c1 = d.colour_off[colour + 1];
    const int R = b.R;
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int site = c0 + (int)(t / R), slot = (int)(t % R);
    double e = 0.0;
    if (site < c1) {
        double2 *S = static_cast<double2 *>(b.state) + d.state;
        const int32_t *row = b.i32 + d.row_ptr;
        const int32_t *col = b.i32 + d.col;
        double hx = 0.0, hy = 0.0, lx = 0.0, ly = 0.0;
        for (int a = row[site]; a < row[site + 1]; ++a) {
            const int j = col[a];
            const double2 v = S[(int64_t)j * R + slot];
            hx = hx + v.x;
            hy = hy + v.y;
            if (j < c0) { lx = hx; ly = hy; }
        }
        const int64_t me = (int64_t)site * R + slot;
        const double2 cur = S[me];
        double2 fin = cur;
        if (met) {
            const uint32_t sweep = b.ctl->sweep;
            const uint32_t lattice = (uint32_t)b.i32[d.perm + site];
            const double beta = b.beta[s * R + b.T_of_slot[s * R + slot]];
            const double2 nw = uniform_direction(d, lattice, sweep, (uint32_t)slot, kMet);
            const double e_old = hx * cur.x + hy * cur.y;
            const double e_new = hx * nw.x + hy * nw.y;
            const double dE = e_old - e_new;                 // H = -h.S
            const U4 w = draw(d, lattice, sweep, (uint32_t)slot, tag(kMetAcc));
            const bool accept = dE <= 0.0 || unit53(w.x, w.y) < exp(-(beta * dE));
            if (accept) { S[me] = nw; fin = nw; }
            if (b.log) {
                const uint32_t rel = sweep - b.ctl->log_base;
                if (rel < (uint32_t)b.log_sweeps)
                    b.log[(((int64_t)rel * b.G + s) * R + slot) * b.max_n + lattice] = accept ? 1 : 0;
            }
        } else {
            // over-relaxation: reflection of S about h (h = 0: unchanged)
            const double hh = hx * hx + hy * hy;
            if (hh != 0.0) {
                const double a = (hx * cur.x + hy * cur.y) / hh;
                const double two_a = 2.0 * a;
                fin = make_double2(two_a * hx - cur.x, two_a * hy - cur.y);
                S[me] = fin;
            }
        }
        e = -(fin.x * lx + fin.y * ly);
    }
    if (!energy) return;                                 // uniform: the whole launch
    esum[threadIdx.x] = e;
    __syncthreads();
    if ((int)threadIdx.x < R) {
        // slot r's threads of this block: (lin0 + k) % R == r, in site order
        const int r = threadIdx.x;
        const int first = (int)(((int64_t)r - (int64_t)blockIdx.x * kBlock % R + R) % R);
        double acc = 0.0;
        for (int k = first; k < kBlock; k += R) acc += esum[k];
        b.epart[(((int64_t)s * n_col + colour) * max_blocks + blockIdx.x) * R + r] = acc;
    }
}

// E_slot of every (sample, slot) from the energy partials of the last
// sub-sweep: colours in order, blocks in order.  nblk[c]: blocks of colour
// c's launch.
struct BlockCounts { int n[kMaxColours]; };

__global__ __launch_bounds__(kBlock) void k_fp64_energy_final(DevBatch b, BlockCounts nblk, int n_col, int max_blocks)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)b.G * b.R) return;
    const int R = b.R, s = (int)(t / R), slot = (int)(t % R);
    const int Q = b.desc[s].Q;
    double acc = 0.0;
    for (int c = 0; c < Q; ++c)
        for (int k = 0; k < nblk.n[c]; ++k) acc += b.epart[(((int64_t)s * n_col + c) * max_blocks + k) * R + slot];
    b.E_slot[s * R + slot] = acc;
}

// Energy (and, when full, the observables) of every (sample, slot), in two
// deterministic stages.  Stage 1: block b of sample s covers a contiguous
// range of sites for all slots; thread t handles slot t % R of sites
// t / R, t / R + nsl, ... so that a warp reads whole [site][slot] rows, and
// accumulates E = -sum over links S_i.S_j (each link once, at its higher
// colour-major endpoint), m and the Fourier sums of Sec. 3; the per-slot sums
// of the block go to partial[s][b][slot][11].  Stage 2 adds the kObsBlocks
// partials of each (sample, slot) in block order.
constexpr int kObsBlocks = 64;
constexpr int kNRed = 11;

__global__ __launch_bounds__(kBlock) void k_fp64_observe_partial(DevBatch b, int full)
{
    __shared__ double red[kBlock * kNRed];
    const int s = blockIdx.y, R = b.R;
    const SampleDesc &d = b.desc[s];
    const int nsl = kBlock / R;                         // site lanes per block (R <= 256)
    const int t = threadIdx.x, slot = t % R, sl = t / R;
    const int per = (d.n + kObsBlocks - 1) / kObsBlocks;
    const int i0 = blockIdx.x * per, i1 = min(d.n, i0 + per);
    double v[kNRed] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (sl < nsl) {
        const double2 *S = static_cast<const double2 *>(b.state) + d.state;
        const int32_t *row = b.i32 + d.row_ptr;
        const int32_t *col = b.i32 + d.col;
        const uint32_t *xy = b.u32 + d.coord;
        const double2 *trig = b.f64 + d.trig;
        for (int i = i0 + sl; i < i1; i += nsl) {
            const double2 si = S[(int64_t)i * R + slot];
            double e = 0.0;
            for (int a = row[i]; a < row[i + 1]; ++a) {
                const int j = col[a];
                if (j >= i) break;                      // ascending rows: lower indices first
                const double2 sj = S[(int64_t)j * R + slot];
                e += si.x * sj.x + si.y * sj.y;
            }
            v[0] -= e;
            if (full) {
                const uint32_t p = xy[i];
                const double2 ex = trig[p & 0xFFFFu], ey = trig[p >> 16];
                v[1] += si.x; v[2] += si.y;
                v[3] += si.x * ex.x; v[4] += si.x * ex.y; v[5] += si.y * ex.x; v[6] += si.y * ex.y;
                v[7] += si.x * ey.x; v[8] += si.x * ey.y; v[9] += si.y * ey.x; v[10] += si.y * ey.y;
            }
        }
    }
    for (int q = 0; q < kNRed; ++q) red[t * kNRed + q] = v[q];
    __syncthreads();
    if (t < R) {
        for (int q = 0; q < kNRed; ++q) {
            double acc = 0.0;
            for (int k = 0; k < nsl; ++k) acc += red[(k * R + t) * kNRed + q];
            b.partial[(((int64_t)s * kObsBlocks + blockIdx.x) * R + t) * kNRed + q] = acc;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_fp64_observe_final(DevBatch b, int full, double *out_by_T)
{
    const int R = b.R;
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)b.G * R) return;
    const int s = (int)(t / R), slot = (int)(t % R);
    const SampleDesc &d = b.desc[s];
    double v[kNRed];
    for (int q = 0; q < kNRed; ++q) v[q] = 0.0;
    for (int blk = 0; blk < kObsBlocks; ++blk)
        for (int q = 0; q < kNRed; ++q) v[q] += b.partial[(((int64_t)s * kObsBlocks + blk) * R + slot) * kNRed + q];
    b.E_slot[s * R + slot] = v[0];
    if (!full) return;
    const double N = (double)d.n;
    const double mx = v[1] / N, my = v[2] / N, m2 = mx * mx + my * my;
    double o[XY_NOBS];
    o[0] = v[0];
    o[1] = m2;
    o[2] = m2 * m2;
    o[3] = (v[3] * v[3] + v[4] * v[4] + v[5] * v[5] + v[6] * v[6]) / N;
    o[4] = (v[7] * v[7] + v[8] * v[8] + v[9] * v[9] + v[10] * v[10]) / N;
    o[5] = mx; o[6] = my; o[7] = 0.0;
    double *dst = out_by_T ? out_by_T + ((int64_t)s * R + b.T_of_slot[s * R + slot]) * XY_NOBS
                           : b.obs_slot + ((int64_t)s * R + slot) * XY_NOBS;
    for (int q = 0; q < XY_NOBS; ++q) dst[q] = o[q];
}

// End of a sweep for a list of samples (all when NULL), one block, so that
// the sweep counter of control block grp is advanced only after every one of
// them has read it:
//  - parallel tempering (App. B; Hukushima-Nemoto): pairs (k, k+1) with
//    k = sweep mod 2, +2, ...; the temperature labels of the two slots are
//    swapped with probability min(1, exp((beta_k - beta_{k+1})(E_k - E_{k+1})));
//    the pairs of one sweep are disjoint, so a thread takes one (sample, k)
//  - a record of the per-slot observables, reordered by temperature, one
//    thread per (sample, temperature) after the swaps;
//  - sweep counter (and record counter) advance.
constexpr int kEndBlock = 1024;

__global__ __launch_bounds__(kEndBlock) void k_end_sweep(DevBatch b, const int32_t *samples, int n_samples, int grp,
                                                        int do_pt, int do_record, int advance)
{
    Ctl *ctl = b.ctl + grp;
    const uint32_t sweep = ctl->sweep;
    const uint32_t rec = ctl->n_records;
    const int R = b.R, n = samples ? n_samples : b.G;
    if (do_pt) {
        for (int t = threadIdx.x; t < n * R; t += kEndBlock) {
            const int j = t / R, k = t - j * R, s = samples ? samples[j] : j;
            if (((k ^ (int)sweep) & 1) || k + 1 >= R) continue;
            int32_t *sot = b.slot_of_T + s * R;
            int32_t *tos = b.T_of_slot + s * R;
            const double *beta = b.beta + s * R;
            const double *E = b.E_slot + s * R;
            const int lo = sot[k], hi = sot[k + 1];
            const double delta = (beta[k] - beta[k + 1]) * (E[lo] - E[hi]);
            const U4 w = draw(b.desc[s], (uint32_t)k, sweep, 0u, tag(kPT));
            const bool accept = delta >= 0.0 || unit53(w.x, w.y) < exp(delta);
            b.pt_try[s * R + k] += 1;
            if (accept) {
                sot[k] = hi; sot[k + 1] = lo;
                tos[hi] = k; tos[lo] = k + 1;
                b.fac_slot[s * R + hi] = accept_factor(beta[k]);
                b.fac_slot[s * R + lo] = accept_factor(beta[k + 1]);
                b.pt_acc[s * R + k] += 1;
            }
        }
    }
    __syncthreads();                                   // the swapped labels, before the record
    if (do_record && rec < (uint32_t)b.max_records) {
        for (int t = threadIdx.x; t < n * R; t += kEndBlock) {
            const int j = t / R, k = t - j * R, s = samples ? samples[j] : j;
            const double *src = b.obs_slot + ((int64_t)s * R + b.slot_of_T[s * R + k]) * XY_NOBS;
            double *dst = b.records + (((int64_t)rec * b.G + s) * R + k) * XY_NOBS;
            for (int q = 0; q < XY_NOBS; ++q) dst[q] = src[q];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (advance) ctl->sweep = sweep + 1;
        if (do_record) ctl->n_records = rec + 1;
    }
}

__global__ __launch_bounds__(kBlock) void k_slot_factors(DevBatch b)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= b.G * b.R) return;
    const int s = t / b.R;
    b.fac_slot[t] = accept_factor(b.beta[s * b.R + b.T_of_slot[t]]);
}

}  // namespace

hipError_t launch_slot_factors(const DevBatch &b, hipStream_t s)
{
    const int n = b.G * b.R;
    hipLaunchKernelGGL(k_slot_factors, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_fp64_init(const DevBatch &b, int max_n, hipStream_t s)
{
    const int64_t threads = (int64_t)max_n * b.R;
    dim3 grid((unsigned)((threads + kBlock - 1) / kBlock), (unsigned)b.G);
    hipLaunchKernelGGL(k_fp64_init, grid, dim3(kBlock), 0, s, b);
    return hipGetLastError();
}

int fp64_phase_blocks(int max_class, int R) { return (int)(((int64_t)max_class * R + kBlock - 1) / kBlock); }

hipError_t launch_fp64_phase(const DevBatch &b, int colour, int met, int energy, int max_class, int n_col,
                             int max_blocks, hipStream_t s)
{
    const int nb = fp64_phase_blocks(max_class, b.R);
    if (nb == 0) return hipSuccess;
    dim3 grid((unsigned)nb, (unsigned)b.G);
    hipLaunchKernelGGL(k_fp64_phase, grid, dim3(kBlock), 0, s, b, colour, met, energy, n_col, max_blocks);
    return hipGetLastError();
}

hipError_t launch_fp64_energy_final(const DevBatch &b, const int *max_class, int n_colours, int max_blocks,
                                    hipStream_t s)
{
    BlockCounts nblk{};
    for (int c = 0; c < n_colours && c < kMaxColours; ++c) nblk.n[c] = fp64_phase_blocks(max_class[c], b.R);
    const int64_t n = (int64_t)b.G * b.R;
    hipLaunchKernelGGL(k_fp64_energy_final, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, b,
                       nblk, n_colours, max_blocks);
    return hipGetLastError();
}

hipError_t launch_fp64_observe(const DevBatch &b, int full, double *out_by_T, hipStream_t s)
{
    hipLaunchKernelGGL(k_fp64_observe_partial, dim3(kObsBlocks, (unsigned)b.G), dim3(kBlock), 0, s, b, full);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)b.G * b.R;
    hipLaunchKernelGGL(k_fp64_observe_final, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, b,
                       full, out_by_T);
    return hipGetLastError();
}

hipError_t launch_end_sweep(const DevBatch &b, const int32_t *samples, int n_samples, int grp, int do_pt,
                            int do_record, int advance, hipStream_t s)
{
    hipLaunchKernelGGL(k_end_sweep, dim3(1), dim3(kEndBlock), 0, s, b, samples, n_samples, grp, do_pt, do_record,
                       advance);
    return hipGetLastError();
}

}  // namespace xy
