// Fixed-point path: each spin is an angle theta = k * 2pi / 2^16 stored as
// uint16 (an exact representation of the 2^16-state clock model), local
// fields are accumulated in FP32 from (cos, sin) tables held in LDS, and
// energies / observables are accumulated in FP64.
//
// One workgroup runs one whole sweep of one (sample, temperature slot): the
// replica's angles are staged in LDS (when they fit) and the colour phases of
// App. B become workgroup barriers, so a sweep needs no grid-wide
// synchronisation and no host round trip.  The CSR is streamed from L2; the
// workgroups of one sample are placed on one XCD by the item order the host
// builds, so they share its CSR in that XCD's L2.
//
// Over-relaxation on the clock model: theta' = (q - theta) mod 2^16 with
// q = round(2 phi_h * 2^16 / 2pi), phi_h the angle of the local field.  The
// map is an involution that depends only on the neighbours, so accepting it
// with probability min(1, exp(-beta dE)) keeps detailed balance exactly; dE
// is tiny (the axis is quantised to 2pi/2^17) and almost every move is taken.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace xy {
namespace {

constexpr int kSweepBlock = 1024;
constexpr int kObsBlock = 256;
constexpr int kNRed = 11;   // E, m_x, m_y, 4 Fourier sums along x, 4 along y
constexpr float kTwoPhiScale = 20860.756700940907f;   // 2^16 / pi: 2*phi in angle units

__device__ __forceinline__ float2 unit32(uint32_t th, const float2 *hi, const float2 *lo)
{
    const float2 a = hi[th >> 8], c = lo[th & 255u];
    return make_float2(a.x * c.x - a.y * c.y, a.y * c.x + a.x * c.y);
}

__device__ __forceinline__ double2 unit64(uint32_t th, const double2 *hi, const double2 *lo)
{
    const double2 a = hi[th >> 8], c = lo[th & 255u];
    return make_double2(a.x * c.x - a.y * c.y, a.y * c.x + a.x * c.y);
}

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
// colour-major endpoint), m = (1/N) sum S_j, F_a = |sum_j S_j e^{i 2pi a_j/L}|^2/N.
__device__ __forceinline__ void observe(const DevBatch &b, const SampleDesc &d, const uint16_t *ang,
                                        const double2 *dhi, const double2 *dlo, const double2 *trig,
                                        double *scratch, double *dst)
{
    const int32_t *row = b.i32 + d.row_ptr;
    const int32_t *col = b.i32 + d.col;
    const uint32_t *xy = b.u32 + d.coord;
    double v[kNRed] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < d.n; i += blockDim.x) {
        const double2 si = unit64(ang[i], dhi, dlo);
        double e = 0.0;
        for (int a = row[i]; a < row[i + 1]; ++a) {
            const int j = col[a];
            if (j >= i) break;
            const double2 sj = unit64(ang[j], dhi, dlo);
            e += si.x * sj.x + si.y * sj.y;
        }
        v[0] -= e;
        const uint32_t p = xy[i];
        const double2 ex = trig[p & 0xFFFFu], ey = trig[p >> 16];
        v[1] += si.x; v[2] += si.y;
        v[3] += si.x * ex.x; v[4] += si.x * ex.y; v[5] += si.y * ex.x; v[6] += si.y * ex.y;
        v[7] += si.x * ey.x; v[8] += si.x * ey.y; v[9] += si.y * ey.x; v[10] += si.y * ey.y;
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

// LDS map: [float2 hi 256][float2 lo 256][double2 hi 256][double2 lo 256]
//          [double scratch 16*kNRed][double2 trig L][uint16 angles n_pad (LDS variant)]
constexpr size_t kOffT32 = 0, kOffT64 = 4096, kOffRed = 12288;
constexpr size_t kOffTrig = kOffRed + 16 * kNRed * 8;   // 13696, multiple of 16

template <bool kLds>
__global__ __launch_bounds__(kSweepBlock) void k_fix16_sweep(DevBatch b, const Item *items, int n_or, int measure)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Item it = items[blockIdx.x];
    if (it.sample < 0) return;
    const int s = it.sample, slot = it.slot, R = b.R;
    const SampleDesc &d = b.desc[s];
    const int n = d.n, n_pad = (n + 7) & ~7, tid = threadIdx.x;

    float2 *t32 = reinterpret_cast<float2 *>(smem + kOffT32);
    double2 *t64 = reinterpret_cast<double2 *>(smem + kOffT64);
    double *scratch = reinterpret_cast<double *>(smem + kOffRed);
    double2 *trig = reinterpret_cast<double2 *>(smem + kOffTrig);
    uint16_t *g_ang = static_cast<uint16_t *>(b.state) + d.state + (int64_t)slot * n_pad;
    uint16_t *ang = kLds ? reinterpret_cast<uint16_t *>(smem + kOffTrig + 16 * (size_t)d.L) : g_ang;
    const float2 *hi32 = t32, *lo32 = t32 + 256;
    const double2 *hi64 = t64, *lo64 = t64 + 256;

    for (int k = tid; k < 512; k += kSweepBlock) { t32[k] = b.tab32[k]; t64[k] = b.tab64[k]; }
    for (int x = tid; x < d.L; x += kSweepBlock) trig[x] = b.f64[d.trig + x];
    if (kLds) {
        const uint4 *src = reinterpret_cast<const uint4 *>(g_ang);
        uint4 *dst = reinterpret_cast<uint4 *>(ang);
        for (int k = tid; k < n_pad / 8; k += kSweepBlock) dst[k] = src[k];
    }
    __syncthreads();

    const float beta = (float)b.beta[s * R + b.T_of_slot[s * R + slot]];
    const uint32_t sweep = b.ctl->sweep;
    const int32_t *row = b.i32 + d.row_ptr;
    const int32_t *col = b.i32 + d.col;
    double e_acc = 0.0;

    for (int sub = 0; sub <= n_or; ++sub) {
        const bool last = (sub == n_or);
        for (int c = 0; c < d.Q; ++c) {
            const int c0 = d.colour_off[c], c1 = d.colour_off[c + 1];
            for (int i = c0 + tid; i < c1; i += kSweepBlock) {
                // local field; the lower-colour part is final in the last sub-sweep
                float hx = 0.f, hy = 0.f, lx = 0.f, ly = 0.f;
                const int a1 = row[i + 1];
                for (int a = row[i]; a < a1; ++a) {
                    const int j = col[a];
                    const float2 u = unit32(ang[j], hi32, lo32);
                    hx += u.x; hy += u.y;
                    if (j < c0) { lx += u.x; ly += u.y; }
                }
                const uint32_t th = ang[i];
                uint32_t th_new, ubits;
                if (sub == 0) {
                    // Metropolis: uniform proposal
                    const U4 w = philox4x32_10({(uint32_t)i, sweep, (uint32_t)slot, tag(kMet)}, d.seed_lo, d.seed_hi);
                    th_new = w.x & 0xFFFFu;
                    ubits = w.y;
                } else {
                    // over-relaxation: reflection about the quantised field axis
                    const int q = __float2int_rn(atan2f(hy, hx) * kTwoPhiScale);
                    th_new = (uint32_t)(q - (int)th) & 0xFFFFu;
                    const U4 w = philox4x32_10({(uint32_t)i, sweep, (uint32_t)slot, tag(kOR, (uint32_t)sub)},
                                               d.seed_lo, d.seed_hi);
                    ubits = w.x;
                }
                const float2 cur = unit32(th, hi32, lo32);
                const float2 nu = unit32(th_new, hi32, lo32);
                const float dE = hx * (cur.x - nu.x) + hy * (cur.y - nu.y);
                const bool accept = dE <= 0.f || (float)(ubits >> 8) * 0x1.0p-24f < __expf(-beta * dE);
                if (accept) ang[i] = (uint16_t)th_new;
                if (last) {
                    const float2 f = accept ? nu : cur;
                    e_acc -= (double)(f.x * lx + f.y * ly);
                }
            }
            __syncthreads();
        }
    }

    {
        double v[1] = {e_acc};
        block_sum<1>(v, scratch);
        if (tid == 0) b.E_slot[s * R + slot] = v[0];
    }
    if (measure) observe(b, d, ang, hi64, lo64, trig, scratch, b.obs_slot + ((int64_t)s * R + slot) * XY_NOBS);
    if (kLds) {
        __syncthreads();
        const uint4 *src = reinterpret_cast<const uint4 *>(ang);
        uint4 *dst = reinterpret_cast<uint4 *>(g_ang);
        for (int k = tid; k < n_pad / 8; k += kSweepBlock) dst[k] = src[k];
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
    const int slot = (int)(t / n_pad), site = (int)(t % n_pad);
    uint16_t *S = static_cast<uint16_t *>(b.state) + d.state;
    uint16_t v = 0;
    if (site < d.n) {
        const U4 w = philox4x32_10({(uint32_t)site, 0u, (uint32_t)slot, tag(kInit)}, d.seed_lo, d.seed_hi);
        v = (uint16_t)(w.x & 0xFFFFu);
    }
    S[t] = v;
}

// Stand-alone measurement from the state in global memory.
__global__ __launch_bounds__(kObsBlock) void k_fix16_observe(DevBatch b, double *out_by_T)
{
    __shared__ double2 t64[512];
    __shared__ double scratch[(kObsBlock / 64) * kNRed];
    const int slot = blockIdx.x, s = blockIdx.y, R = b.R;
    const SampleDesc &d = b.desc[s];
    for (int k = threadIdx.x; k < 512; k += kObsBlock) t64[k] = b.tab64[k];
    __syncthreads();
    const int n_pad = (d.n + 7) & ~7;
    const uint16_t *ang = static_cast<const uint16_t *>(b.state) + d.state + (int64_t)slot * n_pad;
    double o[XY_NOBS];
    observe(b, d, ang, t64, t64 + 256, b.f64 + d.trig, scratch, o);
    if (threadIdx.x != 0) return;
    double *dst = out_by_T ? out_by_T + ((int64_t)s * R + b.T_of_slot[s * R + slot]) * XY_NOBS
                           : b.obs_slot + ((int64_t)s * R + slot) * XY_NOBS;
    for (int q = 0; q < XY_NOBS; ++q) dst[q] = o[q];
    b.E_slot[s * R + slot] = o[0];
}

}  // namespace

size_t fix16_lds_bytes(int n_pad, int L)
{
    return kOffTrig + 16 * (size_t)L + 2 * (size_t)n_pad;
}

hipError_t launch_fix16_init(const DevBatch &b, int max_n, hipStream_t s)
{
    const int64_t threads = (int64_t)((max_n + 7) & ~7) * b.R;
    dim3 grid((unsigned)((threads + 255) / 256), (unsigned)b.G);
    hipLaunchKernelGGL(k_fix16_init, grid, dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_fix16_sweep(const DevBatch &b, const Item *items, int n_items, bool lds, int n_or,
                              int measure, size_t lds_bytes, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    if (lds) {
        static bool attr_set = false;
        if (!attr_set) {
            (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fix16_sweep<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            attr_set = true;
        }
        hipLaunchKernelGGL(k_fix16_sweep<true>, dim3(n_items), dim3(kSweepBlock), lds_bytes, s, b, items, n_or,
                           measure);
    } else {
        hipLaunchKernelGGL(k_fix16_sweep<false>, dim3(n_items), dim3(kSweepBlock), lds_bytes, s, b, items, n_or,
                           measure);
    }
    return hipGetLastError();
}

hipError_t launch_fix16_observe(const DevBatch &b, double *out_by_T, hipStream_t s)
{
    hipLaunchKernelGGL(k_fix16_observe, dim3((unsigned)b.R, (unsigned)b.G), dim3(kObsBlock), 0, s, b, out_by_T);
    return hipGetLastError();
}

}  // namespace xy
