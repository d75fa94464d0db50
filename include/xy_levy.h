/*
 * xy_levy.h -- C ABI of the MI355X (gfx950) library for equilibrium Monte
 * Carlo of O(2)/XY spins on dilute Levy graphs.
 *
 * Paper: M. Ibanez Berganza and L. Leuzzi, "Critical behavior of the XY model
 * in complex topologies", arXiv:1211.3991.
 *
 * The library covers the data-parallel hot path of the paper's method:
 *   graph build (Sec. 2, Eq. Levyi) -> smallest-last colouring (App. B,
 *   "Graph coloring") -> colour-sorted CSR -> sweeps of Metropolis plus
 *   over-relaxation with parallel tempering (App. B, "Improved equilibrium
 *   dynamics") -> measurement of E, |m|^2, |m|^4 and chi(k_min) (Sec. 3).
 *
 * Conventions for every entry point:
 *   - Return value: XY_OK (0) or a negative xy_status.  On error the call has
 *     no effect on device memory unless stated, and xy_last_error() returns a
 *     message (thread-local, valid until the next call on the same thread).
 *   - Device memory is CALLER-OWNED: the caller allocates the buffers whose
 *     sizes xy_batch_sizes() reports and passes raw device pointers; the
 *     library never allocates, frees or keeps device memory beyond a batch.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is enqueued asynchronously on it; a HIP launch error is
 *     reported as XY_EHIP by the call that observes it.
 *   - Host objects (xy_graph, xy_batch) are library-owned and freed with the
 *     matching *_free call.  Calls on one handle are not thread-safe; calls on
 *     different handles are.
 *   - Site numbering: "lattice index" i = y*L + x of the L x L torus; the
 *     device works in "colour-major index" (sites sorted by (colour, lattice
 *     index)).  Host-visible state is always in lattice order.
 */
#ifndef XY_LEVY_H
#define XY_LEVY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int xy_status;
#define XY_OK         0
#define XY_EINVAL    -1   /* bad argument */
#define XY_ENOMEM    -2   /* host allocation failed */
#define XY_EHIP      -3   /* HIP runtime error */
#define XY_ESTATE    -4   /* call not valid in the handle's current state */
#define XY_EUNSUP    -5   /* valid request the library does not support */
#define XY_ECONVERGE -6   /* graph sampler hit its attempt cap */

/* Spin representation. */
#define XY_FP64  0   /* unit vector (x, y) in FP64; decisions bit-identical to the oracle */
#define XY_FIX16 1   /* angle k * 2pi/65536 as uint16, FP32 local fields, FP64 accumulators */

#define XY_NOBS 8    /* per (sample, temperature) record: E, |m|^2, |m|^4, F_x, F_y, m_x, m_y, 0 */

typedef struct xy_graph xy_graph;
typedef struct xy_batch xy_batch;

/* ----------------------------------------------------------------------- */
/* Graphs (host)                                                           */
/* ----------------------------------------------------------------------- */

/* Dilute Levy graph on the periodic L x L lattice (Sec. 2, Eq. Levyi):
 * N = L*L sites and exactly N*z/2 links.  Each raw draw t (t = 0, 1, ...)
 * takes Philox4x32-10 of counter (t lo, t hi, 0, 1<<24) under key `seed`:
 * site i = floor(w0 * N / 2^32); a displacement d = (dx, dy) with
 * dx, dy in {-L/2+1..L/2}, d != 0, listed dy-outer/dx-inner, drawn with
 * weight (dx^2+dy^2)^(-rho/2) by inverting the sequential prefix sums with the
 * 53-bit uniform ((w1 << 21) | (w2 >> 11)) * 2^-53; j = i + d on the torus.
 * A draw that repeats an existing link is rejected.  Then the graph is
 * coloured by smallest-last ordering (App. B; ties to the smallest lattice
 * index, greedy smallest colour in reverse removal order) and laid out as a
 * colour-sorted CSR.
 *   L    : even, >= 2.         z : >= 1, N*z even, z < N-1.     rho : >= 0.
 *   out  : receives a new graph (free with xy_graph_free).
 * Errors: XY_EINVAL for bad arguments, XY_ECONVERGE if 1000*M + 10^6 draws do
 * not give M links, XY_ENOMEM. */
xy_status xy_graph_levy(int L, int z, double rho, uint64_t seed, xy_graph **out);

/* The same graph with free boundaries (Sec. 2: distances within the L x L
 * square, r_max = L sqrt 2; the paper's degree distributions and one FSS check
 * use it).  Raw draw t takes counter (t lo, t hi, 1, 1<<24); the displacement
 * set is dx, dy in {-(L-1)..L-1}, d != 0, in the same raster order and by the
 * same inversion; a draw whose j = i + d leaves the square is rejected like a
 * repeated link, so every pair is drawn with probability proportional to
 * r^-rho.  2 <= L <= 4096 (any parity); errors as xy_graph_levy (at large rho
 * and z = 4 the open square has too few short pairs: XY_ECONVERGE). */
xy_status xy_graph_levy_free(int L, int z, double rho, uint64_t seed, xy_graph **out);

/* Graph from an explicit edge list (tiny exact-physics graphs, tests).
 *   edges  : int32[2*m], pairs (i, j), 0 <= i, j < n, no self or repeated links.
 *   coords : int32[2*n] lattice coordinates (x, y) of each site, 0 <= x, y < L,
 *            or NULL for (i % L, i / L).  L (1..65535) is the period used by
 *            the Fourier observables.
 * Errors: XY_EINVAL (bad index, self or duplicate link), XY_ENOMEM. */
xy_status xy_graph_from_edges(int n, int m, const int32_t *edges, const int32_t *coords,
                              int L, xy_graph **out);

/* Sizes: any pointer may be NULL.  attempts = raw draws used (0 for edge lists). */
xy_status xy_graph_info(const xy_graph *g, int *n, int *m, int *n_colours, int *max_degree,
                        int64_t *attempts);

/* Copies out the graph (each pointer may be NULL; host buffers, caller-owned):
 *   edges      int32[2m]   links in acceptance order, as drawn (i, j)
 *   colour     int32[n]    colour of each lattice site
 *   perm       int32[n]    lattice index of each colour-major index
 *   colour_off int32[Q+1]  first colour-major index of each colour
 *   row_ptr    int32[n+1]  CSR over colour-major indices
 *   col        int32[2m]   neighbours (colour-major indices), ascending per row */
xy_status xy_graph_export(const xy_graph *g, int32_t *edges, int32_t *colour, int32_t *perm,
                          int32_t *colour_off, int32_t *row_ptr, int32_t *col);

void xy_graph_free(xy_graph *g);

/* ----------------------------------------------------------------------- */
/* Batches (device): n_graphs samples x n_T temperatures, one replica slot  */
/* per temperature.                                                         */
/* ----------------------------------------------------------------------- */

typedef struct {
    size_t state_bytes;   /* spins */
    size_t graph_bytes;   /* CSR, coordinates, tables (read-only after init) */
    size_t work_bytes;    /* temperatures, permutations, energies, counters */
    size_t obs_bytes;     /* measurement records [max_records][n_graphs][n_T][XY_NOBS] double */
} xy_sizes;

/* Device bytes needed for a batch.  n_T in [1, 256]; precision XY_FP64 or
 * XY_FIX16; max_records >= 0. */
xy_status xy_batch_sizes(const xy_graph *const *g, int n_graphs, int n_T, int precision,
                         int max_records, xy_sizes *out);

/* Creates a batch on caller-owned device buffers (sizes from xy_batch_sizes,
 * 256-byte aligned) and enqueues the upload of the graphs and the random
 * initial state (an independent uniform direction per (sample, slot, site),
 * Philox purpose 2) on `stream`.
 *   T     : double[n_graphs * n_T] temperature ladders (T > 0), slot k starts at T[k]
 *   seeds : uint64[n_graphs] Philox keys of the samples' dynamics
 * The graphs may be freed after this call returns.
 * fix16 storage per sample: graphs of at least 16384 sites, when n_T is a
 * multiple of 4, are stored site-major and swept one colour phase of many such
 * samples per launch (the phase form; the samples form stream groups, see
 * xy_batch_set_phase_streams); smaller graphs, or any n_T, get one
 * workgroup per replica with the replica in LDS when it fits (else in global
 * memory).  The environment variables XY_FIX16_PHASE_MIN (the site threshold)
 * and XY_FIX16_PHASE (1: every sample, 0: none) override the rule; they are
 * read here and by xy_batch_sizes, which must see the same values.  The
 * phase form sorts each colour class by degree inside windows of 4096 sites
 * (XY_SELL_WINDOW overrides the window); the other forms inside whole classes
 * for graphs of up to 65536 sites and inside windows of 4096 sites above. */
xy_status xy_batch_init(xy_batch **out, const xy_graph *const *g, int n_graphs, int n_T,
                        const double *T, int precision, const uint64_t *seeds, int max_records,
                        void *d_state, void *d_graph, void *d_work, void *d_obs, void *stream);

/* Runs n_sweeps sweeps (App. B).  A sweep is one Metropolis sub-sweep
 * (uniform proposal) and n_or over-relaxation sub-sweeps; each sub-sweep
 * visits the colours in increasing order.  After the sweep, when
 * pt_every > 0 and (sweep+1) % pt_every == 0, parallel-tempering swaps of the
 * temperature labels are attempted between T_k and T_{k+1} for k = sweep mod
 * 2, sweep mod 2 + 2, ...; then, when meas_every > 0 and
 * (sweep+1) % meas_every == 0, a record [n_graphs][n_T][XY_NOBS] is appended
 * to the observation buffer (ignored once max_records are stored).
 *   T : NULL keeps the ladder; else double[n_graphs * n_T], the new
 *       temperature of every (sample, temperature index) from this call on
 *       (finite, > 0).  The labels stay: the replica that holds index k
 *       continues at the new T_k.  The host array may be reused when the call
 *       returns (the batch uploads a copy of 1/T on `stream`).
 * n_sweeps >= 0, 0 <= n_or <= 255.  Errors: XY_EINVAL (bad argument; no
 * effect), XY_EHIP. */
xy_status xy_sweep(xy_batch *b, const double *T, int n_sweeps, int n_or, int pt_every, int meas_every,
                   void *stream);

/* Observables of the current state, by temperature, into caller-owned device
 * memory d_out: double[n_graphs][n_T][XY_NOBS] (E, |m|^2, |m|^4, F_x, F_y,
 * m_x, m_y, 0), with m = (1/N) sum_j S_j and
 * F_a = |sum_j S_j exp(2 pi i a_j / L)|^2 / N (Sec. 3). */
xy_status xy_measure(xy_batch *b, double *d_out, void *stream);

/* Enqueues one parallel-tempering step now (App. B, parallel tempering:
 * exchanges of the temperatures of neighbouring replicas with the
 * Hukushima-Nemoto probability), with the replica energies recomputed from
 * the current state and the pair parity from the sweep counter. */
xy_status xy_pt_swap(xy_batch *b, void *stream);

/* The replica energies E = -sum over links cos(theta_i - theta_j) (Sec. 2,
 * Eq. HXY) that the last tempering step (App. B) used, by replica slot:
 * copies double[n_graphs][n_T slots] into caller-owned device memory d_out,
 * asynchronously on `stream`.  Defined after a sweep with tempering or an
 * xy_pt_swap; the fixed-point path sums them from FP32 link energies in FP64. */
xy_status xy_pt_energies(xy_batch *b, double *d_out, void *stream);

/* Synchronous copies of the state (checkpoint, tests).  Host layout:
 *   fp64 : double[n_graphs][n_T slots][n_i][2], lattice order
 *   fix16: uint16[n_graphs][n_T slots][n_i], lattice order
 * plus int32 slot_of_T[n_graphs][n_T] and the sweep counter.  Either array
 * pointer may be NULL.  set_state does not touch records or PT counters. */
xy_status xy_get_state(xy_batch *b, void *h_state, int32_t *h_slot_of_T, uint32_t *sweep,
                       void *stream);
xy_status xy_set_state(xy_batch *b, const void *h_state, const int32_t *h_slot_of_T,
                       uint32_t sweep, void *stream);

/* Synchronous read of counters: records stored so far; PT accepted/attempted
 * per (sample, k) as uint64[n_graphs][n_T] (k = lower temperature of the
 * pair); either pointer may be NULL. */
xy_status xy_get_counters(xy_batch *b, int *n_records, uint64_t *pt_accepted,
                          uint64_t *pt_attempted, void *stream);

/* Parity harness (FP64 batches): while enabled, each Metropolis decision of
 * sweep w < max_sweeps is written as one byte (1 accepted, 0 rejected) to
 * d_log[w][sample][slot][lattice site] (caller-owned device memory of
 * max_sweeps * n_graphs * n_T * max_n bytes, max_n = largest graph).
 * Sweeps are counted from the enabling call.  d_log = NULL disables. */
xy_status xy_decision_log(xy_batch *b, uint8_t *d_log, int max_sweeps);

/* HIP-graph replay: xy_sweep captures `chunk` sweeps of its shape (n_or,
 * pt_every, meas_every, stream) into a HIP graph on first use and replays it
 * for every whole chunk of later calls of the same shape (chunk = 0 turns it
 * off; with chunk > 0, xy_sweep needs a non-null stream).  The graph holds
 * the launches of chunk sweeps of every sample group: (n_or + 1) per colour
 * and a few more per group and sweep.  The captured tempering and
 * record flags repeat with P = lcm(pt_every, meas_every) (0 counting as 1):
 * a replay starts only at a sweep index congruent modulo P to the one it was
 * captured at, and direct launches reach that index first (chunk a multiple
 * of P keeps every later chunk aligned).  Replays and direct launches give
 * identical trajectories.  A ladder change (xy_sweep's T) needs no new
 * capture: the kernels read 1/T from device memory. */
xy_status xy_batch_use_graph(xy_batch *b, int chunk);

/* Kernel timing for roofline reports: while enabled, every xy_sweep records a
 * HIP event pair on its stream around the dominant kernels of each sweep (the
 * fix16 sweep kernels and the fix16 phase-form colour-phase kernels, or the
 * colour-phase kernels of an FP64 sweep).  When every sample is in the phase
 * form and its samples run as two or more stream groups, the groups fork from
 * the caller's stream once per run of direct launches and each runs its own
 * energies, tempering and records; the event pair then brackets that whole
 * run, whose sweeps it counts.  A HIP-graph replay is bracketed as a whole
 * (all kernels of its chunk of sweeps).  xy_kernel_time synchronises the
 * stream of the last sweep, returns the summed elapsed milliseconds and the
 * number of timed sweeps since timing was enabled, and keeps timing on. */
xy_status xy_kernel_timing(xy_batch *b, int enable);
xy_status xy_kernel_time(xy_batch *b, double *ms_total, int *n_timed);

/* Stream groups of the phase form (fix16 batches; used by the autotuner):
 * the phase-form samples are split into n_streams (1..4) contiguous groups of
 * about equal work, group 0 launched on the caller's stream and the others on
 * streams the library owns.  Every group updates its samples exactly as one
 * group would, so the trajectory does not depend on the choice; only the
 * overlap of the launches does (App. B's colour phases, here per group).
 * Initial value 2 (the environment variable XY_PHASE_STREAMS overrides it at
 * xy_batch_init).  Synchronises `stream` and the library's streams; no effect
 * on batches without phase-form samples.  XY_EINVAL outside [1, 4]. */
xy_status xy_batch_set_phase_streams(xy_batch *b, int n_streams, void *stream);
xy_status xy_batch_phase_streams(const xy_batch *b, int *n_streams);

/* Stream groups in slices (fix16 batches whose samples are all in the phase
 * form; used by the autotuner): n_streams * n_slices groups of about equal
 * work, group g on stream g % n_streams; within an xy_sweep call the slices
 * run one after the other, each for all the call's sweeps (its groups
 * concurrently on the n_streams streams), so that only one slice's samples
 * are swept at a time: a smaller working set for the memory-side caches.
 * Samples are independent (each group has its own tempering, records and
 * sweep counter), so the trajectory does not depend on the choice.
 * xy_batch_set_phase_streams(b, n, s) is n streams in one slice.  Batches
 * with workgroup-form samples keep one slice.  Synchronises like
 * xy_batch_set_phase_streams.  XY_EINVAL unless 1 <= n_streams <= 4,
 * n_slices >= 1 and n_streams * n_slices <= 8; the slice count is lowered
 * where the phase samples are fewer than the groups.  Initial value one
 * slice (XY_PHASE_SLICES overrides it at xy_batch_init).
 * xy_batch_phase_groups returns the configuration in effect. */
xy_status xy_batch_set_phase_groups(xy_batch *b, int n_streams, int n_slices, void *stream);
xy_status xy_batch_phase_groups(const xy_batch *b, int *n_streams, int *n_slices);

/* Fixed-point sweep configuration (fix16 batches; used by the autotuner).
 *   trig        : (cos, sin) of a 16-bit angle, for every sample: 0 two-level
 *                 LDS table, 1 2048-entry LDS table with a small-angle
 *                 rotation, 2 hardware sine/cosine
 *   allow_unit  : keep FP32 unit vectors in LDS for graphs that fit (else angles)
 *   force_global: keep every replica in global memory
 * Each choice samples the clock model with its own FP32 (cos, sin); all are
 * exact Metropolis samplers.  allow_unit and force_global concern the
 * workgroup-per-replica samples only (the phase-form samples keep their
 * site-major storage, chosen at xy_batch_init).  Synchronises `stream`, then
 * uploads the new work-item lists.  Initial values: trig 2, allow_unit 1,
 * force_global 0 (the environment variables XY_FIX16_TRIG, XY_FIX16_NOUNIT
 * and XY_FIX16_GLOBAL override them at xy_batch_init). */
xy_status xy_batch_set_fix16_form(xy_batch *b, int trig, int allow_unit, int force_global, void *stream);

/* Storage form of each sample, as chosen at xy_batch_init: out[s] = 1 for
 * the site-major phase form, 0 for a workgroup per replica (FP64 batches: 0
 * for every sample).  out: host int32[n_graphs], caller-owned. */
xy_status xy_batch_forms(const xy_batch *b, int32_t *out);

/* ----------------------------------------------------------------------- */
/* Random walks for the spectral dimension (Sec. 2, spectral dimension;    */
/* App. A): P(tau), the probability that a walker is back at its starting  */
/* site after tau steps, behaves as tau^(-dbar/2).                          */
/* ----------------------------------------------------------------------- */

/* Device bytes for the walk graphs of xy_random_walk (n_graphs >= 1). */
xy_status xy_walk_bytes(const xy_graph *const *g, int n_graphs, size_t *graph_bytes);

/* Self-return histograms of n_walkers walkers on each graph, into
 * caller-owned device memory d_hist: uint64[n_graphs][n_steps + 1], entry
 * (g, t) = walkers of graph g at their start after t steps (t = 0 counts
 * them all).  Walker w of graph g, under the Philox key seeds[g], starts at
 *   start_mode 0: the lattice centre, site (L/2) L + L/2 (needs N = L*L);
 *   start_mode 1: the k-th site, in lattice order, of degree larger than
 *     two, k = floor(x * count / 2^32), x word 0 of counter (w, 0, 0, 8<<24);
 * step t moves to the site's neighbour number floor(x * deg / 2^32),
 * neighbours in ascending lattice index, x word t mod 4 of counter
 * (w, floor(t/4), 0, 7<<24); a walker on a site of degree 0 stays.
 * d_graph: graph_bytes (xy_walk_bytes) of device memory, 256-byte aligned,
 * filled by this call.  0 <= n_walkers, 0 <= n_steps < 2^24.  The call
 * uploads the graphs on `stream` and synchronises it before returning (the
 * host staging buffer is released); the walks run asynchronously after,
 * unless kernel_ms is not NULL: then the call waits for them and stores the
 * duration of the walk kernel in milliseconds (HIP events on `stream`).
 * Errors: XY_EINVAL for bad arguments or start_mode 0 on a graph that is not
 * L x L, XY_EUNSUP for start_mode 1 on a graph with no site of degree > 2. */
xy_status xy_random_walk(const xy_graph *const *g, int n_graphs, int n_walkers, int n_steps,
                         const uint64_t *seeds, int start_mode, void *d_graph, size_t graph_bytes,
                         uint64_t *d_hist, void *stream, float *kernel_ms);

/* xy_random_walk for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid allocation): the same walks,
 * histograms and errors, but the walk graphs are staged in the library's
 * static device workspace instead of a caller-provided d_graph.  Like
 * xy_random_walk it synchronises `stream` after the upload, so it is not a
 * call to record into a HIP graph.  The workspace is 32 MiB (33554432 bytes) per
 * device, held from the library's load to the end of the process; a set of
 * graphs whose xy_walk_bytes exceeds it is rejected with XY_EINVAL before any
 * device work.  The call allocates no device memory (it still builds the
 * records in host memory, uploads them on `stream` and synchronises it, as
 * xy_random_walk does).  Every call on a device shares that device's
 * workspace: calls that overlap on one device (other threads or streams)
 * race and must be serialised by the caller; a call overwrites what the
 * previous one staged.  d_hist: caller-owned uint64[n_graphs][n_steps + 1]. */
xy_status xy_random_walk_noalloc(const xy_graph *const *g, int n_graphs, int n_walkers, int n_steps,
                                 const uint64_t *seeds, int start_mode, uint64_t *d_hist, void *stream,
                                 float *kernel_ms);

const char *xy_last_error(void);
void xy_batch_free(xy_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* XY_LEVY_H */
