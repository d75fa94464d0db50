// Kernel argument blocks and host-side launchers (one TU per precision).
#pragma once

#include <hip/hip_runtime.h>

#include "xy_internal.hpp"

namespace xy {

// Everything a kernel needs to find a sample's data on the device.
struct DevBatch {
    const SampleDesc *desc;   // [G]
    const int32_t *i32;       // row_ptr / col / perm pool
    const uint32_t *u32;      // packed coordinates pool
    const double2 *f64;       // (cos, sin)(2 pi x / L) pool
    const uint16_t *u16;      // fix16 sliced-ELL columns (graphs with at most 65536 sites)
    const uint8_t *u8;        // fix16 degrees
    const float2 *tab32;      // [512]: (cos, sin)(2 pi * 256a / 2^16) then (cos, sin)(2 pi * b / 2^16)
    const float2 *tab2k;      // [2048]: (cos, sin)(2 pi * 32a / 2^16)
    const double2 *tab64;     // [512]: same angles as tab32 in FP64
    void *state;              // fp64: double2 [site][slot]; fix16: uint16 [slot][site_pad]
    Ctl *ctl;
    const double *beta;       // [G][R] by temperature index
    int32_t *slot_of_T;       // [G][R]
    int32_t *T_of_slot;       // [G][R]
    float *fac_slot;          // [G][R]: accept_factor of the inverse temperature each slot holds (fix16)
    double *E_slot;           // [G][R]
    double *obs_slot;         // [G][R][XY_NOBS]
    double *partial;          // [G][64][R][11] block partial sums of the observables (fp64, fix16 phase form)
    double *epart;            // energy partials: fix16 phase form [n_phase][31][max_blocks][R], fp64 [G][Q][max_blocks][R]
    unsigned long long *pt_acc, *pt_try;  // [G][R]
    double *records;          // [max_records][G][R][XY_NOBS]
    int G, R, max_records, max_n;
    int idx16;                // fix16 columns are uint16 (else int32)
    int trig;                 // fix16 (cos, sin) evaluation: 0 two-level table, 1 2048-table + rotation, 2 hardware
    uint8_t *log;             // Metropolis decision log (fp64) or NULL
    int log_sweeps;
};

// -beta log2(e) in FP32: the factor of dE in the exponent of the fixed-point
// acceptance probability 2^(dE * factor) = exp(-beta dE).  The table
// fac_slot holds it by slot; whatever moves a temperature to another slot
// (tempering, a new ladder, a restored state) rewrites it.
__device__ __forceinline__ float accept_factor(double beta) { return -(float)beta * 1.4426950408889634f; }

// fac_slot of every (sample, slot) from beta and T_of_slot
hipError_t launch_slot_factors(const DevBatch &b, hipStream_t s);

// FP64 path (kernels_fp64.hip, built with -ffp-contract=off).
hipError_t launch_fp64_init(const DevBatch &b, int max_n, hipStream_t s);
// energy: also sum the replica energies into b.epart (the last sub-sweep of a
// tempering sweep), [G][n_col][max_blocks][R] with n_col the batch's largest
// colour count and max_blocks at least fp64_phase_blocks of every colour.
int fp64_phase_blocks(int max_class, int R);
hipError_t launch_fp64_phase(const DevBatch &b, int colour, int met, int energy, int max_class, int n_col,
                             int max_blocks, hipStream_t s);
// E_slot from those partials (max_class: the launch sizes of the n_colours colours)
hipError_t launch_fp64_energy_final(const DevBatch &b, const int *max_class, int n_colours, int max_blocks,
                                    hipStream_t s);
hipError_t launch_fp64_observe(const DevBatch &b, int full, double *out_by_T, hipStream_t s);
// samples: the samples to temper and record (NULL: all); ctl: b.ctl[grp]
hipError_t launch_end_sweep(const DevBatch &b, const int32_t *samples, int n_samples, int grp, int do_pt,
                            int do_record, int advance, hipStream_t s);

// fix16 path (kernels_fix16.hip).
hipError_t launch_fix16_init(const DevBatch &b, int max_n, hipStream_t s);
// mode: 0 angles in LDS, 1 angles in global memory, 2 unit vectors in LDS
// (angles in global memory); block: mode 2 takes 256 or 1024, mode 0 1024, mode 1 512
hipError_t launch_fix16_sweep(const DevBatch &b, const Item *items, int n_items, int mode, int block,
                              int n_or, int measure, size_t lds_bytes, hipStream_t s);
hipError_t launch_fix16_observe(const DevBatch &b, double *out_by_T, hipStream_t s);
size_t fix16_lds_bytes(int n_pad, int trig, int mode);

// fix16 phase form (site-major state, one launch per colour phase) for the
// samples listed in phase_samples; sites_per_block(R) sites per block.
int fix16_phase_sites_per_block(int R);
// units: the n_units work units (two int4 each, see k_fix16_phase) of this
// colour, one workgroup each; max_blocks: stride of the energy partials (the
// largest block count of any colour); last: fuse the energy; grp: the
// control block b.ctl[grp] whose sweep counter keys the random words;
// reverse: each XCD takes its run of units from the end (alternated between
// consecutive colour phases).
hipError_t launch_fix16_phase(const DevBatch &b, const int4 *units, int colour, int sub,
                              int last, int n_units, int max_blocks, int grp, int reverse, hipStream_t s);
// phase samples [k_first, k_first + n_phase) of the list
hipError_t launch_fix16_phase_energy(const DevBatch &b, const int32_t *phase_samples, int k_first, int n_phase,
                                     int max_blocks, hipStream_t s);
// Energies (and, when full, observables) of phase samples [k_first,
// k_first + n_phase): two deterministic stages through b.partial.
hipError_t launch_fix16_observe_sm(const DevBatch &b, const int32_t *phase_samples, int k_first, int n_phase,
                                   int full, hipStream_t s);

}  // namespace xy
