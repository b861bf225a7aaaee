/*
 * sic.h - C ABI of libsic: the simplex-in-cell (SIC) 1D1V Vlasov-Poisson
 * step on MI355X (gfx950).
 *
 * Method (Kates-Harbeck, Totorica, Zrake & Abel, arXiv:1506.07207):
 *   - section 2.1, eqs. 1-3: Vlasov-Poisson with C = 1 and the mean density
 *     removed on a periodic box; the acceleration E = -dPhi/dx obeys
 *     dE/dx = rho = n - nbar (units: plasma frequency 1, mean density 1);
 *   - section 2.2-2.3: the plasma is a set of sheets of ordered tracers; each
 *     pair of adjacent tracers bounds a segment (a "particle") carrying a fixed
 *     charge spread uniformly between them (the box function); a closed sheet
 *     also joins its last tracer to its first;
 *   - section 2.3, eqs. "overlap" and "rho_sum": the charge of every segment is
 *     deposited onto the periodic mesh by its exact overlap with each cell;
 *   - section 2.6: optional refinement, a centre tracer inserted into every
 *     segment that has grown longer than a set length;
 *   - the paragraph after eq. "j_sum": solve for the field, gather it to the
 *     tracers with linear (first-order) weighting (section 2.4) and move the
 *     tracers as PIC particles - here with a leapfrog.
 *
 * Mesh: n_cells cells [j dx, (j+1) dx), dx = L / n_cells; charge, density and
 * field values sit at the cell centres (j + 1/2) dx.  The field solve is the
 * 3-point periodic Poisson equation with a centred-difference field.
 *
 * Conventions shared by every call:
 *   - Tracer arrays (x, v) hold the tracers of sheet 0, then sheet 1, ... as
 *     contiguous float64 values (sheet-major).
 *   - mem_kind says where a caller pointer lives: SIC_MEM_HOST (ordinary or
 *     pinned host memory) or SIC_MEM_DEVICE (device memory on the current HIP
 *     device, e.g. a torch CUDA tensor's data pointer).
 *   - The library copies what it is given and never keeps a caller pointer;
 *     caller buffers only need to stay valid for the duration of the call.
 *   - All device work is ordered on the hipStream_t given at creation (NULL =
 *     the default stream).  Calls marked "async" return before the GPU has
 *     finished; calls that return data synchronise that stream first.
 *   - Errors are returned as sic_status; nothing is thrown across the ABI.
 *     sic_last_error() gives a message for the last failing call on a handle.
 *   - A handle must not be used from two host threads at once.
 */
#ifndef SIC_H
#define SIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIC_ABI_VERSION 2
#define SIC_MAX_CELLS 4096

typedef enum sic_status {
    SIC_OK = 0,
    SIC_EINVAL = 1,   /* invalid argument (sizes, pointers, non-finite inputs) */
    SIC_ENOMEM = 2,   /* device or host allocation failed */
    SIC_EDEVICE = 3,  /* a HIP runtime call failed */
    SIC_ESTATE = 4,   /* call out of order (e.g. push before solve) */
    SIC_EBUSY = 5,    /* batch: no free slot or over the tracer budget */
    SIC_ENOTSUP = 6   /* valid but unsupported request (e.g. deposit_order != 0) */
} sic_status;

/* Position storage.
 *   SIC_FP64:      x in float64; mesh charge accumulated with float64 atomics.
 *   SIC_SPLIT_F32: x as an integer cell index + float32 offset: the 32-bit
 *                  index counts sub-cells of 2^-20 cell (cell = index >> 20)
 *                  and the float32 offset in [0, 1) places the tracer within
 *                  its sub-cell, about 2^-44 cell resolution;
 *   SIC_SPLIT_U32: x as int32 cell index + uint32 fraction of a cell (2^-32
 *                  cell resolution).
 * Both split forms keep v in float64, deposit into int64 fixed point (bitwise
 * reproducible, order independent) and solve in float64.  A non-finite move
 * leaves a split position where it was (the velocity stays non-finite and the
 * diagnostics flag it). */
typedef enum sic_precision { SIC_FP64 = 0, SIC_SPLIT_F32 = 1, SIC_SPLIT_U32 = 2 } sic_precision;

enum { SIC_MEM_HOST = 0, SIC_MEM_DEVICE = 1 };

/* sic_diag.flags bits (sticky per simulation). */
enum {
    SIC_DIAG_NONFINITE = 1,    /* a non-finite field value or segment length, or a move
                                  with a non-finite kinetic energy or momentum */
    SIC_DIAG_LONG_SEGMENT = 2  /* some segment longer than 0.45 L (segments join
                                  tracers the shorter way round the box, so a
                                  segment cannot be longer than L/2) */
};

typedef struct sic_config {
    int32_t abi_version;   /* SIC_ABI_VERSION */
    int32_t n_cells;       /* 1 .. SIC_MAX_CELLS */
    double L;              /* box length, > 0 */
    double dt;             /* time step, > 0 */
    int32_t precision;     /* sic_precision */
    int32_t deposit_order; /* 0: piecewise-constant segments (section 2.3); 1: piecewise-linear
                              segments with the fold-corner check (section 2.5); 2: first-order
                              (W_1) weighting of constant segments to the grid points (section
                              2.4); others SIC_ENOTSUP */
    int64_t history_rows;  /* capacity of the per-simulation diagnostics ring; 0: 65536 */
    double l_max;          /* refinement length (section 2.6): after every move, each segment
                              longer than l_max gets a new tracer at its centre with the mean
                              velocity of its two tracers, and each half carries half of its
                              charge; 0: no refinement.  In a batch it needs
                              SIC_BATCH_SEGMENT_CHARGES (else SIC_ENOTSUP). */
    int64_t max_tracers;   /* tracer capacity for refinement growth; 0: the initial count.  The
                              simulation reserves room for this many tracers (in a batch the
                              reservation counts against the budget).  A refinement that would
                              exceed it fails with SIC_ENOMEM and leaves the state unchanged. */
} sic_config;

typedef struct sic_sheet {
    int32_t n_tracers; /* >= 2 */
    int32_t closed;    /* 1: segment from the last tracer back to the first; 0: open chain */
    double q_seg;      /* charge carried by every segment of the sheet, unless per-segment
                          charges are given */
} sic_sheet;

/* Per-segment charges (section 2.3: the segments are the particles and carry
 * the charge).  Where a call takes seg_charges, NULL means every segment of
 * sheet s carries sheets[s].q_seg; otherwise it holds sum(n_tracers) doubles,
 * sheet-major, and entry t of a sheet is the charge of the segment from tracer
 * t to tracer t + 1 (for the last tracer of a closed sheet, the closing
 * segment back to tracer 0; the entry of the last tracer of an open sheet is
 * ignored and reads back as 0).  Tracer t carries mass (c_{t-1} + c_t) / 2,
 * half of each segment it bounds (a missing segment counts 0), so the total
 * mass is the total charge (equal charge-to-mass ratio). */

/* One row of diagnostics, at step n (positions x^n, time t = n dt):
 *   W_E          = 1/2 dx sum_j E_j^2 (field energy, section 3 "E_pot");
 *   KE           = 1/2 sum m v^{n-1/2} v^{n+1/2}, momentum = sum m (v^{n-1/2}+v^{n+1/2})/2
 *                  with the tracer masses m defined with the segment charges;
 *                  both need the push from step n, so the newest row has them
 *                  as NaN;
 *   total_charge = sum_j Q_j (charge conservation check);
 *   max_segment  = longest segment at x^n. */
typedef struct sic_diag {
    int64_t step;
    double t;
    double W_E;
    double KE;
    double momentum;
    double total_charge;
    double max_segment;
    int64_t flags;
} sic_diag;

typedef struct sic_sim sic_sim;

/* Creates a simulation and ingests its initial state: x0 is reduced into
 * [0, L), the charge Q^0 is deposited, the field E^0 solved, and the
 * velocities are moved back half a step, v^{-1/2} = v0 - dt/2 E^0(x0)
 * (leapfrog start).  On return the simulation is at step 0 with its field
 * current.  x0 and v0 hold sum(n_tracers) values; seg_charges is NULL or the
 * per-segment charges (see above), in the same memory as x0.  hip_stream:
 * hipStream_t or NULL.  Synchronous (returns after the ingest has run). */
sic_status sic_init(const sic_config *cfg, const sic_sheet *sheets, int32_t n_sheets, const double *x0,
                    const double *v0, const double *seg_charges, int32_t mem_kind, void *hip_stream,
                    sic_sim **out);

/* Deposit (section 2.3): Q <- charge of every segment at the current
 * positions x^n, by exact box-cell overlap.  Allowed in any state.  Async. */
sic_status sic_deposit(sic_sim *sim);

/* Solve: E^n and W_E^n from Q.  Requires a deposit of the current positions
 * since the last push (else SIC_ESTATE).  Async. */
sic_status sic_solve_field(sic_sim *sim);

/* Gather + move: v^{n+1/2} = v^{n-1/2} + dt E^n(x^n), x^{n+1} = x^n + dt v^{n+1/2}
 * wrapped into [0, L); the step becomes n + 1.  Requires the field of the
 * current step (else SIC_ESTATE).  Async. */
sic_status sic_push(sic_sim *sim);

/* n_steps full steps.  Each step moves the tracers with the current field,
 * deposits the new positions and solves the new field, so on return the field
 * is current for the new step.  If the field is stale it is brought up to date
 * first.  Steps run as captured HIP graphs of a tracer launch and a solve
 * launch each (SIC_PATH_FUSED).  With constant segments and at most 512
 * workgroups per launch (two per compute unit) a simulation's tracer
 * launches solve the previous step's charge themselves, in every workgroup,
 * and one solve launch closes each graph of up to 32 steps
 * (SIC_PATH_SOLVE_FIRST); a small simulation (at most 32 chunks of 64 tracer
 * slots) runs its steps in one launch of a single workgroup
 * (SIC_PATH_RESIDENT).  All give the bits of the fused path in the split
 * forms.  Timing mode (sic_set_timing) always takes the fused path.  Async;
 * with refinement on (l_max > 0) each step is followed by a refinement pass
 * on the device (SIC_PATH_REFINING: graphs of steps and passes; the host
 * reads the layout back when it needs it). */
sic_status sic_step(sic_sim *sim, int64_t n_steps);

enum {
    SIC_PATH_NONE = -1,
    SIC_PATH_FUSED = 0,
    SIC_PATH_RESIDENT = 1,
    SIC_PATH_REFINING = 2,
    SIC_PATH_SOLVE_FIRST = 3
};
/* The launch path of the last sic_step call on sim (SIC_PATH_NONE before
 * any). */
sic_status sic_last_step_path(const sic_sim *sim, int32_t *path);

/* One refinement pass (section 2.6) over the current positions: every segment
 * longer than l_max (minimum-image length) gets a tracer at its centre, with
 * the mean velocity of its two tracers, and both halves carry half its
 * charge; a segment longer than 2 l_max is halved once per pass.  When a
 * tracer was inserted, the new state is deposited and solved and the newest
 * diagnostics row is rewritten with it.  *inserted (may be NULL) receives the
 * number of tracers added.  Needs a simulation created with per-segment
 * charges or l_max > 0 (else SIC_ENOTSUP); SIC_ENOMEM beyond max_tracers
 * (state unchanged).  Synchronous. */
sic_status sic_refine(sic_sim *sim, double l_max, int64_t *inserted);

/* Tracers per sheet now (n_tracers_out: NULL or n_sheets entries) and their
 * total; refinement changes them. */
sic_status sic_get_layout(const sic_sim *sim, int32_t *n_tracers_out, int64_t *total);

/* Per-segment charges now (sum of the current n_tracers doubles, in mem_kind
 * memory; fixed-point charges of the split forms converted to float64).
 * Synchronous. */
sic_status sic_get_charges(sic_sim *sim, double *seg_charges, int32_t mem_kind);

/* Replaces the tracer state with n_tracers[s] tracers per sheet (the sheets
 * and their closure stay those given at creation): positions x^n, velocities
 * v^{n-1/2}, per-segment charges (NULL: each sheet's q_seg from creation; a
 * simulation created without per-segment charges and without refinement
 * accepts only NULL) and step n.  The field becomes stale.  SIC_ENOMEM beyond
 * the tracer capacity.  Synchronous. */
sic_status sic_load_state(sic_sim *sim, int64_t step, const int32_t *n_tracers, const double *x,
                          const double *v_half, const double *seg_charges, int32_t mem_kind);

/* Synchronises the stream and reads diagnostics.  out (may be NULL) receives
 * the newest row.  rho_out / E_out (NULL or n_cells doubles, host memory)
 * receive the charge density n_j - nbar and the field of the newest solve.
 * history_out (NULL or *history_len rows) receives the oldest-first rows still
 * in the ring, from the step the simulation started at or its state was last
 * set or loaded at; *history_len is set to the number of rows written (or,
 * when history_out is NULL, to the number available). */
sic_status sic_diagnostics(sic_sim *sim, sic_diag *out, double *rho_out, double *E_out, sic_diag *history_out,
                           int64_t *history_len);

/* Checkpoint: x^n and v^{n-1/2} (sum(n_tracers) doubles each, in mem_kind
 * memory) and the step n.  Synchronous. */
sic_status sic_get_state(sic_sim *sim, double *x, double *v_half, int64_t *step, int32_t mem_kind);

/* Resume: replaces positions and velocities with x^n (wrapped into [0, L)) and
 * v^{n-1/2}, sets the step to n and marks the field stale (the next sic_step
 * deposits and solves first).  Synchronous. */
sic_status sic_set_state(sic_sim *sim, int64_t step, const double *x, const double *v_half, int32_t mem_kind);

/* Largest simulation (tracers) whose host inputs sic_set_state_noalloc stages. */
#define SIC_NOALLOC_MAX_TRACERS (1 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): sic_set_state
 * without any allocation.  Host inputs (SIC_MEM_HOST) are staged through a
 * fixed device array of 16 * SIC_NOALLOC_MAX_TRACERS bytes (16 MiB) that the
 * library holds on each GPU it runs on until the process ends, instead of a
 * buffer allocated for the call; device inputs are read in place.  With host
 * inputs a simulation of more than SIC_NOALLOC_MAX_TRACERS tracers gets
 * SIC_EINVAL and nothing changes.  The array is shared by every call on that
 * GPU and keeps the last call's contents: calls that overlap on one GPU (from
 * several host threads) race on it and must be serialised by the caller.
 * Otherwise exactly sic_set_state (synchronous). */
sic_status sic_set_state_noalloc(sic_sim *sim, int64_t step, const double *x, const double *v_half,
                                 int32_t mem_kind);

void sic_destroy(sic_sim *sim);
const char *sic_status_str(sic_status s);
/* Message of the last failing call on sim; with sim == NULL, of the last
 * failing call on this host thread (e.g. a sic_init that returned no handle). */
const char *sic_last_error(const sic_sim *sim);
int32_t sic_abi_version(void);

/* Launch shape of the tracer kernels (see sic_tune in the batch section).
 *   tile_chunks:   64-tracer chunks per workgroup work item (one LDS mesh
 *                  accumulation and flush per item); 0 = automatic;
 *   block_threads: 64, 128, 256, 512 or 1024; 0 = automatic;
 *   grid_blocks:   workgroups of the tracer kernels, which loop over the
 *                  work items (any count is valid); 0 = automatic: one work
 *                  item per workgroup (batches: the item count rounded up to
 *                  a power of two, at least 4096);
 *   fused_only:    single simulations: nonzero keeps sic_step on the fused
 *                  launch pairs where it would take the resident or
 *                  solve-first path; 0 = automatic (batches ignore it).
 * sic_get_tuning reports the shape in effect (fused_only as set). */
typedef struct sic_tuning {
    int32_t tile_chunks;
    int32_t block_threads;
    int32_t grid_blocks;
    int32_t fused_only;
} sic_tuning;

sic_status sic_set_tuning(sic_sim *sim, const sic_tuning *t);
sic_status sic_get_tuning(const sic_sim *sim, sic_tuning *t);

/* ------------------------------------------------------------------------
 * Batch: many independent simulations resident on one GPU, advanced together
 * (continuous batching).  Every slot follows exactly the single-simulation
 * semantics above; the batch only shares launches.  All instances of a batch
 * use the batch's precision.
 * ---------------------------------------------------------------------- */
typedef struct sic_batch sic_batch;

/* Batch flags. */
#define SIC_BATCH_SEGMENT_CHARGES 1 /* store a charge per segment: admissions may pass
                                       seg_charges (8 more bytes per tracer of budget, read
                                       every step) */

/* budget_tracers: maximum resident tracers over all slots (the tracer arena
 * holds every sheet in whole 64-tracer chunks, with about 1/8 spare for the
 * padding of partly filled last chunks: many sheets of fewer than 64 tracers
 * can fill it before the budget, and admission then returns SIC_EBUSY);
 * max_slots: maximum resident simulations; max_cells: largest n_cells
 * admitted (<= SIC_MAX_CELLS);
 * precision and deposit_order: shared by every admitted simulation (as in
 * sic_config); flags: SIC_BATCH_* bits; history_rows: diagnostics rows kept
 * per slot (ring; 0: 4096).  Synchronous. */
sic_status sic_batch_create(int64_t budget_tracers, int32_t max_slots, int32_t max_cells, int32_t precision,
                            int32_t deposit_order, int32_t flags, int64_t history_rows, void *hip_stream,
                            sic_batch **out);

/* Admits one simulation that will run n_steps steps (n_steps < 0: until
 * released).  Ingests it as sic_init does.  seg_charges: NULL, or per-segment
 * charges for a batch created with SIC_BATCH_SEGMENT_CHARGES (else
 * SIC_ENOTSUP).  Returns SIC_EBUSY when no slot is free or its tracers do not
 * fit the budget.  *slot receives the slot index.  Ordered on the batch
 * stream; returns after the inputs have been copied. */
sic_status sic_batch_admit(sic_batch *b, const sic_config *cfg, const sic_sheet *sheets, int32_t n_sheets,
                           const double *x0, const double *v0, const double *seg_charges, int32_t mem_kind,
                           int64_t n_steps, int32_t *slot);

/* Advances every unfinished resident simulation by up to n_steps steps in
 * shared launches (captured HIP graphs); a simulation stops when its own step
 * count is reached.  Async.  While a resident simulation refines (l_max > 0),
 * steps run one at a time and each is followed by a refinement pass of every
 * refining simulation that took it, as sic_step does (synchronous). */
sic_status sic_batch_step(sic_batch *b, int64_t n_steps);

/* Tracers per sheet of one slot now, and their total, as sic_get_layout. */
sic_status sic_batch_get_layout(const sic_batch *b, int32_t slot, int32_t *n_tracers_out, int64_t *total);

/* Synchronises the stream and lists slots whose simulation has finished and
 * has not been reported before (at most cap entries). */
sic_status sic_batch_poll(sic_batch *b, int32_t *done_slots, int32_t cap, int32_t *n_done);

/* Synchronises and copies a slot's diagnostics as sic_diagnostics does. */
sic_status sic_batch_result(sic_batch *b, int32_t slot, sic_diag *out, double *rho_out, double *E_out,
                            sic_diag *history_out, int64_t *history_len);

/* Checkpoint of one slot, as sic_get_state. */
sic_status sic_batch_get_state(sic_batch *b, int32_t slot, double *x, double *v_half, int64_t *step,
                               int32_t mem_kind);

/* Per-segment charges of one slot, as sic_get_charges. */
sic_status sic_batch_get_charges(sic_batch *b, int32_t slot, double *seg_charges, int32_t mem_kind);

/* Frees a slot (finished or not) and its tracer budget.  Ordered on the stream. */
sic_status sic_batch_release(sic_batch *b, int32_t slot);

/* Resident tracers and simulations. */
sic_status sic_batch_usage(const sic_batch *b, int64_t *tracers, int32_t *slots);

sic_status sic_batch_set_tuning(sic_batch *b, const sic_tuning *t);
sic_status sic_batch_get_tuning(const sic_batch *b, sic_tuning *t);
void sic_batch_destroy(sic_batch *b);
const char *sic_batch_last_error(const sic_batch *b);

/* Average device time (milliseconds, from HIP events on the batch stream) of
 * the last sic_batch_step call, per step, split into the tracer kernel and the
 * field-solve kernel; 0 when not measured.  Enable with timing = 1 (adds
 * events between launches, so graphs are not used while it is on). */
sic_status sic_batch_set_timing(sic_batch *b, int32_t timing);
sic_status sic_batch_last_timing(const sic_batch *b, double *tracer_ms, double *solve_ms);

/* Autotuner.  Times every candidate launch shape (chunks per work item,
 * threads per workgroup, grid size) for steps_per_trial steps on
 * the handle's own resident simulations, with HIP events around each kernel,
 * then restores the simulations to their state before the call (the trial
 * steps leave no trace; the device briefly holds a second copy of the state)
 * and applies the fastest shape; the shape in effect is timed first and kept
 * unless another is more than 2 % faster.  best / best_ms (may be NULL)
 * receive the shape applied and its time per step.  Synchronous; SIC_ENOMEM
 * if the state copy does not fit. */
sic_status sic_autotune(sic_sim *sim, int32_t steps_per_trial, sic_tuning *best, double *best_ms);
sic_status sic_batch_autotune(sic_batch *b, int32_t steps_per_trial, sic_tuning *best, double *best_ms);

/* Single-simulation timing, as sic_batch_set_timing / sic_batch_last_timing. */
sic_status sic_set_timing(sic_sim *sim, int32_t timing);
sic_status sic_last_timing(const sic_sim *sim, double *tracer_ms, double *solve_ms);

/* Device copy bandwidth in GB/s (bytes read + bytes written per second) of a
 * streaming copy of n_bytes (non-temporal 16-byte loads and stores, four
 * loads in flight per lane), best of iters runs at each of four grid sizes,
 * on the given stream.  A calibration for the HBM roofline.  Synchronous. */
sic_status sic_copy_bandwidth(int64_t n_bytes, int32_t iters, void *hip_stream, double *gbps);

#ifdef __cplusplus
}
#endif

#endif /* SIC_H */
