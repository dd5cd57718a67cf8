/*
 * ssa_rp.h - C ABI of the MI355X ensemble direct-method library (libssa_rp.so).
 *
 * The library runs ensembles of Gillespie direct-method trajectories
 * (Kimpson, Flegg & Flegg, "Reduced-Precision Stochastic Simulation for
 * Mathematical Biology", Sec. 2: propensities, their sum a0, waiting time
 * tau = -ln(u1)/a0, selection of the smallest mu whose partial sum exceeds
 * u2*a0, integer state update) on one gfx950 GPU, one trajectory per lane,
 * in the precision configurations of Sec. 3-4:
 *   - FP64 and FP32: every operation in that type;
 *   - mixed (Sec. 3.2): propensities in fp16 or bf16, propensity sum,
 *     waiting time and clock in binary32, species counts as exact int32;
 *   - uniform (Sec. 3.2, last paragraph): every operation in fp16 or bf16;
 *   - rounding after each 16-bit operation by round-to-nearest-even or
 *     stochastic rounding (Sec. 3.3, SR equation), optionally with
 *     propensities divided by their running maximum (uniform mode only;
 *     "propensity normalisation" of the abstract).
 *
 * Conventions
 *   - Every call returns SSA_OK (0) or an SSA_E_* code; no exception crosses
 *     the ABI. ssa_last_error() gives a message for the calling thread's last
 *     failure (valid until that thread's next call).
 *   - Handles are opaque. The library is thread-compatible: concurrent calls
 *     on distinct handles are fine; one handle must not be used by two threads
 *     at once.
 *   - "Host" pointers point to CPU memory, "device" pointers to memory of the
 *     current HIP device. Input arrays are copied before the call returns.
 */
#ifndef SSA_RP_H
#define SSA_RP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define SSA_OK 0
#define SSA_E_INVALID 1      /* an argument is out of range or inconsistent */
#define SSA_E_NOMEM 2        /* host or device allocation failed */
#define SSA_E_DEVICE 3       /* a HIP call failed (message in ssa_last_error) */
#define SSA_E_UNSUPPORTED 4  /* valid request this build does not implement */
#define SSA_E_COMPILE 5      /* run-time kernel compilation failed */

/* ---- propensity laws (Sec. 2; Hill form of Sec. 4.5) -------------------- */
#define SSA_LAW_MASS_ACTION 0   /* a = k * prod_s C(x_s, o_s)                    */
#define SSA_LAW_HILL_REPRESS 1  /* a = basal + k / (1 + (x_r / K)^h)             */
#define SSA_LAW_HILL_ACTIVATE 2 /* a = basal + k (x_r / K)^h / (1 + (x_r / K)^h) */

/* ---- precision configuration (Sec. 4 opening: six configurations x mixed/uniform) */
#define SSA_FMT_FP64 0
#define SSA_FMT_FP32 1
#define SSA_FMT_FP16 2
#define SSA_FMT_BF16 3
#define SSA_ACC_MIXED 0    /* 16-bit propensities, binary32 sums and clock */
#define SSA_ACC_UNIFORM 1  /* every operation in the 16-bit format          */
#define SSA_RND_RTN 0      /* round to nearest, ties to even                */
#define SSA_RND_SR 1       /* stochastic rounding with Philox halfwords     */
#define SSA_RND_SR_ACC 2   /* SR only at the partial sums and the clock,
                              round to nearest elsewhere (uniform mode; the
                              selective SR of Sec. 3.3, last paragraph)     */
#define SSA_NORM_NONE 0
#define SSA_NORM_RUNNING_MAX 1 /* uniform 16-bit only */

/* ---- per-trajectory status ---------------------------------------------- */
#define SSA_STATUS_DONE 0     /* next event would pass t_end                 */
#define SSA_STATUS_ABSORBED 1 /* all propensities zero                       */
#define SSA_STATUS_OVERFLOW 2 /* a propensity or their sum is not finite     */
#define SSA_STATUS_CAPPED 3   /* max_events events fired                     */

typedef struct ssa_model ssa_model;
typedef struct ssa_run ssa_run;

/* One reaction's propensity law.
 *   kind == SSA_LAW_MASS_ACTION: k >= 0 is the rate constant; the reactant
 *     orders come from ssa_model_create's reactant_order row (total order
 *     0..4); the propensity is (k / prod_s o_s!) prod_s x_s (x_s-1)...(x_s-o_s+1).
 *   kind == SSA_LAW_HILL_*: k = vmax >= 0, basal >= 0, K > 0, 1 <= h <= 8,
 *     0 <= regulator < n_species. */
typedef struct ssa_law {
    int32_t kind;
    int32_t regulator;
    int32_t h;
    int32_t reserved;
    double k;
    double basal;
    double K;
} ssa_law;

/* Build a reaction network (host only; no GPU needed).
 *   n_species N in [1, 32], n_reactions M in [1, 64].
 *   reactant_order: host [M][N] int32, row-major by reaction; entries >= 0
 *     (read for mass-action reactions only).
 *   stoich: host [M][N] int32 net change of each species, |entry| <= 1024.
 *   laws: host [M].
 *   out: receives the model; release with ssa_model_destroy.
 * Errors: SSA_E_INVALID (sizes, orders, non-finite or negative constants,
 *   h, K or regulator out of range, NULL pointers); SSA_E_NOMEM. */
int ssa_model_create(int32_t n_species, int32_t n_reactions, const int32_t *reactant_order,
                     const int32_t *stoich, const ssa_law *laws, ssa_model **out);

/* Release a model (NULL is ignored). Runs that used it keep their own copy. */
void ssa_model_destroy(ssa_model *model);

/* One network's share of an ensemble run.
 *   x0: host [N] initial counts, each >= 0.
 *   n_traj: trajectories of this item, < 2^31.
 *   set_rates: optional host [n_sets][M] table replacing the model's k
 *     (mass action: k; Hill: vmax), finite and >= 0; trajectory i uses row
 *     i / traj_per_set (n_traj <= n_sets * traj_per_set). NULL: the model's k.
 *   d_snap, d_n_events, d_t_last, d_status: optional device outputs owned by
 *     the caller, laid out as [n_snap][N][n_traj] int32, [n_traj] uint64,
 *     [n_traj] double and [n_traj] uint8. NULL: the run allocates them.
 *   record_mask, record_cap: event record (the switching times behind the
 *     dwell-time distributions of Sec. 4.3). Every firing of a reaction j with
 *     bit j of record_mask set is logged with the clock after it (the run's
 *     clock type, widened to double) and j, up to record_cap entries per
 *     trajectory; the count of such firings goes on past record_cap. 0 / 0:
 *     no record. record_cap in [0, 2^20], record_cap * n_traj <= 2^31.
 *   d_rec_t, d_rec_j, d_rec_n: optional caller-owned device outputs of the
 *     record, [n_traj][record_cap] double, [n_traj][record_cap] uint8 and
 *     [n_traj] uint32 (entries past a trajectory's count are undefined). NULL:
 *     the run allocates them. */
typedef struct ssa_item {
    const ssa_model *model;
    const int32_t *x0;
    int64_t n_traj;
    const double *set_rates;
    int64_t n_sets;
    int64_t traj_per_set;
    int32_t *d_snap;
    uint64_t *d_n_events;
    double *d_t_last;
    uint8_t *d_status;
    uint64_t record_mask;
    int32_t record_cap;
    int32_t reserved;
    double *d_rec_t;
    uint8_t *d_rec_j;
    uint32_t *d_rec_n;
} ssa_item;

/* An ensemble run over one or more items in one persistent launch.
 *   t_end > 0, finite. snap_t: host [n_snap] ascending times in [0, t_end];
 *     snapshot k holds the state at snap_t[k] (an event at exactly snap_t[k]
 *     is included). n_snap in [0, 65536].
 *   seed: Philox key. Trajectory i of item m draws with trajectory id
 *     traj_id_base + (sum of n_traj of items before m) + i (< 2^32), so runs
 *     that split an ensemble differently give identical trajectories.
 *   format/accum/rounding/norm: SSA_FMT_*, SSA_ACC_*, SSA_RND_*, SSA_NORM_*.
 *     FP64 and FP32 take accum = MIXED, rounding = RTN, norm = NONE.
 *     norm = RUNNING_MAX and rounding = SR_ACC need a 16-bit format and
 *     accum = UNIFORM.
 *   max_events: per-trajectory event cap; a trajectory that fires it stops
 *     with SSA_STATUS_CAPPED. 0 = none, allowed for FP64 only: a binary32 or
 *     16-bit clock stops advancing once the waiting time falls below half its
 *     spacing (the stagnation of uniform round-to-nearest runs, Sec. 4), and
 *     such a trajectory would never end (SSA_E_INVALID).
 *   hip_stream: hipStream_t to run on (NULL = the null stream).
 *   n_chunks: 1 runs the horizon in one launch; c > 1 splits the snapshot
 *     rows into c windows, one launch each (with the small kernels that
 *     reorder claims between them). Up to 16 windows are launched directly on
 *     hip_stream; a longer sequence is captured once per run into a hipGraph,
 *     which is launched on hip_stream. Results are bit-identical to one
 *     launch. 0 = the autotuned choice for this kernel and workload shape if
 *     ssa_autotune stored one, else 1.
 *   block_size, grid_size: launch shape; 0 = the autotuned choice if stored,
 *     else 256 threads and enough workgroups for one trajectory per lane (up
 *     to what stays resident). block_size a multiple of 64 up to 256, or 512:
 *     then waves 0-3 of each workgroup run trajectories and wave w + 4, on
 *     the same SIMD as wave w, forms wave w's random draws ahead of use and
 *     passes them through LDS (results are bit-identical: the draws are the
 *     same function of seed, trajectory and event index).
 *   reorder: chunked runs only. 0 or 1: before each chunk after the first,
 *     trajectories are claimed in order of the events they fired in the
 *     previous chunk, heaviest first (results are unchanged: draws are keyed
 *     by trajectory id); -1: claim in id order.
 *   first_window: chunked runs only. 0: the n_chunks windows split the
 *     snapshot rows evenly. w > 0: the first window holds rows [0, w) and the
 *     other n_chunks - 1 split the rest evenly; a short first window measures
 *     each trajectory's event rate, so that with reorder the longest
 *     trajectories start first in the next window. Must leave at least one row
 *     for every later window (else SSA_E_INVALID). With n_chunks = 0 the
 *     autotuned value is used.
 *   placement: SSA_PLACE_AUTO, or SSA_PLACE_EXPLICIT | SSA_PLACE_* flags
 *     (else SSA_E_INVALID). Results do not depend on it: draws are keyed by
 *     trajectory id, not by lane. */
/* Placement of work in a launch (ssa_run_desc.placement). */
#define SSA_PLACE_AUTO 0               /* the autotuned choice if stored, else none of the flags */
#define SSA_PLACE_EXPLICIT 1           /* the flags below are the caller's choice            */
#define SSA_PLACE_NEIGHBOUR_PRODUCER 2 /* 512-thread workgroups: event-loop wave c takes its
                                          draws from the producer on the next SIMD (mod 4),
                                          so a wave left running alone has its SIMD to itself */
#define SSA_PLACE_WAVE_MAJOR 4         /* single-item runs: each launch's first claims are
                                          static, wave-major (the first 64 claims of the
                                          claim order go to wave 0 of workgroup 0, the next
                                          to wave 0 of workgroup 1, ...), so after a
                                          reordering window the heaviest trajectories share
                                          one wave per workgroup                            */
#define SSA_PLACE_SOLO_WAVE0 8         /* 512-thread workgroups, one-item launches (SSA_E_INVALID
                                          otherwise): event-loop wave 0 runs with its
                                          SIMD to itself (producers feed the next SIMD's wave,
                                          event-loop wave 3 forms its own draws, wave 4 does
                                          not run); with SSA_PLACE_WAVE_MAJOR the heaviest
                                          trajectories get those SIMDs                      */
#define SSA_PLACE_FEED_WAVE0 16        /* 512-thread workgroups: the producer wave that feeds
                                          event-loop wave 0 issues ahead of event-loop waves
                                          1-3 (wave priorities), so wave 0 keeps its draws
                                          while the chip is busy                            */
#define SSA_PLACE_PRODUCER_FIRST 32    /* 512-thread workgroups: producer waves issue ahead of
                                          event-loop waves (a producer stops at a full ring) */
#define SSA_PLACE_DEDICATED_FEED0 64   /* 512-thread workgroups: three event-loop waves; wave 0
                                          alone on its SIMD and its producer alone on the
                                          next, the other two fed from their own SIMDs (with
                                          SSA_PLACE_WAVE_MAJOR: the heaviest trajectories on
                                          wave 0, never short of draws)                    */
#define SSA_PLACE_TWO_FEED0 128        /* with SSA_PLACE_DEDICATED_FEED0, one-item launches
                                          (SSA_E_INVALID otherwise): two producer waves share
                                          wave 0's draws, one the even and one the odd event
                                          indices (a lone event loop on the conversion path
                                          uses draws faster than one producer makes them);
                                          no effect where the draw ring holds fewer than 4
                                          slots (the largest networks)                     */

typedef struct ssa_run_desc {
    const ssa_item *items;
    int32_t n_items;
    int32_t n_snap;
    double t_end;
    const double *snap_t;
    uint64_t seed;
    uint32_t traj_id_base;
    int32_t format;
    int32_t accum;
    int32_t rounding;
    int32_t norm;
    int32_t n_chunks;
    uint64_t max_events;
    void *hip_stream;
    int32_t block_size;
    int32_t grid_size;
    int32_t reorder;
    int32_t first_window;
    int32_t placement;
} ssa_run_desc;

/* Start an ensemble run; returns once the work is queued on hip_stream
 * (asynchronous). The first run of a (networks, precision) combination
 * compiles its kernel for gfx950 (ROCm's offline clang at
 * $ROCM_PATH/llvm/bin/clang++, run as a child process, or the one named by
 * SSA_RP_CLANG; hipRTC when there is none or SSA_RP_CLANG is empty), cached
 * in memory and on disk (SSA_RP_CACHE_DIR, else _kcache beside the library).
 *   out: receives the run; release with ssa_run_destroy.
 * Errors: SSA_E_INVALID (see ssa_run_desc), SSA_E_UNSUPPORTED (precision
 *   combination), SSA_E_COMPILE, SSA_E_NOMEM, SSA_E_DEVICE. */
int ssa_ensemble_run(const ssa_run_desc *desc, ssa_run **out);

/* The allocation-free variant of ssa_ensemble_run, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation). Same descriptor, same kernels, same
 * results; differences:
 *   - every item must bring its device outputs (d_snap unless it has no
 *     cells, d_n_events, d_t_last, d_status; a recording item also d_rec_t,
 *     d_rec_j, d_rec_n), else SSA_E_INVALID;
 *   - the kernel for the run's networks and precision must already be loaded
 *     on the current device by an earlier ssa_ensemble_run or ssa_autotune
 *     (compiling and loading allocate), else SSA_E_INVALID;
 *   - the run's tables, work counters, carry state and claim order live in a
 *     fixed 64 MiB device array of the library (one per device, held until
 *     the process ends); a run that needs more (chunked runs of very large
 *     ensembles) gets SSA_E_INVALID. The first call on a device looks the
 *     array's address up once;
 *   - snapshot windows are always launched directly (no graph), and no run
 *     handle, events or timings are made: the work is queued on
 *     desc->hip_stream (tables copied asynchronously on it) and the results
 *     are in the caller's buffers once that stream has passed it.
 * Every call on one device shares that device's array: calls whose work may
 * overlap on a device (other streams, other threads) race and must be
 * serialised by the caller. Allocates no device memory and calls no device
 * allocator. Errors: as ssa_ensemble_run's validation, SSA_E_DEVICE. */
int ssa_ensemble_run_noalloc(const ssa_run_desc *desc);

/* Block until the run's work on its stream is complete. SSA_E_DEVICE on a
 * HIP error. */
int ssa_run_wait(ssa_run *run);

/* Copy item `item`'s snapshots, [n_snap][N][n_traj] int32, to dst (host or
 * device per dst_is_device); waits for the run. SSA_E_INVALID if
 * dst_elems != n_snap * N * n_traj or item is out of range. */
int ssa_snapshots_get(const ssa_run *run, int32_t item, int32_t *dst, size_t dst_elems,
                      int dst_is_device);

/* Copy item `item`'s per-trajectory results: events fired (uint64), time of
 * the last fired event (double) and SSA_STATUS_* (uint8), each [n_traj];
 * any pointer may be NULL. Waits for the run. */
int ssa_run_stats_get(const ssa_run *run, int32_t item, uint64_t *n_events, double *t_last,
                      uint8_t *status, int dst_is_device);

/* Copy item `item`'s event record to host or device memory (waits for the
 * run): t and j [n_traj][record_cap] (entries past a trajectory's count are
 * undefined), n [n_traj]; any pointer may be NULL. SSA_E_INVALID if the item
 * has no record or is out of range. */
int ssa_records_get(const ssa_run *run, int32_t item, double *t, uint8_t *j, uint32_t *n, int dst_is_device);

/* Timing and launch facts of a finished run. */
typedef struct ssa_run_info {
    double elapsed_ms;        /* device time from first to last launch (HIP events) */
    double kernel_ms;         /* sum of the simulation kernels' own durations */
    int32_t n_launches;       /* simulation kernel launches (chunks) */
    int32_t block_size;
    int32_t grid_size;
    int32_t vgprs;            /* not known: -1 */
    uint64_t total_events;    /* sum of events over all trajectories */
    int32_t first_window;     /* snapshot rows of the first launch (0: even windows) */
    int32_t graph;            /* 1 if the launches ran as one captured hipGraph */
    int32_t placement;        /* SSA_PLACE_EXPLICIT | SSA_PLACE_* flags the launches used */
} ssa_run_info;

/* Fill info for a run (waits for it). */
int ssa_run_info_get(const ssa_run *run, ssa_run_info *info);

/* Result of ssa_autotune. */
typedef struct ssa_tune_result {
    int32_t block_size;   /* threads per workgroup */
    int32_t grid_size;    /* workgroups: sets waves per CU and trajectories per lane */
    int32_t n_chunks;     /* snapshot windows (one launch each) */
    int32_t first_window; /* snapshot rows of the first window (0: even windows) */
    int32_t placement;    /* SSA_PLACE_EXPLICIT | chosen SSA_PLACE_* flags */
    int32_t n_candidates; /* launch shapes timed */
    double best_ms;       /* device time of the chosen shape */
} ssa_tune_result;

/* Launch-shape autotuner. Runs desc's workload (into scratch outputs owned by
 * the library; desc's output pointers are ignored) once per candidate shape:
 * block size 64 or 256; grid holding 1, 2 or 4 waves per SIMD with lane
 * refill, or one lane per trajectory, and 512 (producer waves) with one
 * workgroup per CU; one launch, 4 even snapshot windows, a first window of a
 * tenth of the rows followed by 1 or 2 windows, or of 15% or 20% of the rows
 * followed by 1. Times
 * each with HIP events, keeps the fastest in memory and in
 * <cache dir>/tune.txt, keyed by the generated kernel and the workload shape
 * (ensemble sizes, snapshot count, t_end, max_events). Later runs of the same
 * key that pass block_size = 0, grid_size = 0 or n_chunks = 0 use it.
 * res may be NULL. Errors: as ssa_ensemble_run. */
int ssa_autotune(const ssa_run_desc *desc, ssa_tune_result *res);

/* Release a run and the device memory it owns (NULL is ignored). */
void ssa_run_destroy(ssa_run *run);

/* Message of the calling thread's last failure ("" if none). */
const char *ssa_last_error(void);

/* Library version string. */
const char *ssa_version(void);

/* Compile, and store in the on-disk kernel cache, the kernel that
 * ssa_ensemble_run would use for desc (validated as there; output pointers
 * and hip_stream are ignored). Needs no GPU. The cache directory is
 * $SSA_RP_CACHE_DIR, else "_kcache" beside the library.
 * Errors: as ssa_ensemble_run's validation; SSA_E_COMPILE. */
int ssa_prepare(const ssa_run_desc *desc);

/* Compile if needed and write to path (a buffer of len bytes) the file name
 * of the cached code object ssa_ensemble_run would load for desc, for
 * instruction-level analysis. Needs no GPU. Errors: validation codes;
 * SSA_E_INVALID if the buffer is too small; SSA_E_COMPILE. */
int ssa_kernel_file(const ssa_run_desc *desc, char *path, size_t len);

/* Write the generated kernel source for desc to the file `path` (for
 * inspection). Errors: validation codes; SSA_E_INVALID if path cannot be
 * opened. */
int ssa_dump_source(const ssa_run_desc *desc, const char *path);

#ifdef __cplusplus
}
#endif

#endif /* SSA_RP_H */
