// sic_internal.h - device-side layout shared by the kernels and the host
// side of libsic (not part of the public ABI).
//
// Tracer storage.  Tracers live in 64-slot chunks, one wavefront per chunk;
// every sheet starts on a chunk boundary (its last chunk may be partly
// empty), so a wavefront never straddles two sheets.  State is two arrays of
// 8-byte words per tracer slot:
//   word 0: x (float64)                      - SIC_FP64
//           index (low 32 bits) | offset (high) - split forms: U32 the cell
//           and a uint32 fraction of it; F32 an index of 2^-20-cell
//           sub-cells (cell = index >> 20) and a float32 offset in [0, 1)
//           of the sub-cell
//   word 1: v (float64)
// Every chunk also keeps a copy of its first tracer's state in a "halo"
// array.  A step that moves tracers and deposits their new positions in the
// same kernel needs, for the last tracer of each chunk, the new position of
// the first tracer of the next chunk, which another workgroup may already
// have overwritten; it recomputes that move from the halo copy written by the
// previous step.  The halo is double-buffered (read one, write the other).
//
// Charges.  By default every segment of a sheet carries the sheet's charge,
// kept in the chunk descriptor.  Pools created for per-segment charges (and
// refinement, which halves segments) keep a third 8-byte word per tracer
// slot: the charge of the segment that starts at that tracer (float64, or
// int64 fixed point in the split forms), plus per chunk the charge of the
// segment that ends at its first tracer and of the segment that starts at
// its partner tracer ("charge edges").
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sic {

constexpr int kChunk = 64;          // tracer slots per chunk = wavefront width
constexpr int kMaxCells = 4096;     // mirrors SIC_MAX_CELLS
// Copies of a single simulation's charge accumulators (P, D, R): its work
// items merge into copy (item mod copies), so each address takes that
// fraction of the atomics, and the solve sums the copies in order.  Four for
// meshes of up to kSolveThreads cells; two for larger ones, whose every
// solve-first workgroup reads all copies of the whole mesh (the reads then
// cost more than the contention saves).  Batches, with few items per
// simulation, keep one copy.
constexpr int single_rep(int max_cells) { return max_cells <= 256 ? 4 : 2; }
constexpr int kSolveThreads = 256;  // field-solve workgroup

enum Prec : int { kFP64 = 0, kSplitF32 = 1, kSplitU32 = 2 };

// Tracer-kernel modes (bit set).
enum Mode : int {
  kDeposit = 1,      // deposit the (possibly new) positions into the mesh
  kPush = 2,         // kick with E and drift
  kKickHalf = 4,     // start-up: v <- v - dt/2 E(x), positions unchanged
};

// Solve-kernel flags.
enum SolveFlags : int {
  kHavePush = 1,     // a push ran since the last solve: step += 1, KE/momentum rows
  kHaveDeposit = 2,  // partials hold the max segment of the deposited positions
  kBatchStep = 4,    // count the step against steps_left; finish at zero
};

struct alignas(16) InstDesc {
  double L, half_L, dx, inv_dx;
  double dt, q_unit;      // q_unit: charge of one fixed-point unit (split forms)
  int64_t mesh_off;       // first cell of this slot in the mesh arrays
  int64_t hist_off;       // first row of this slot in the history array
  int64_t hist_cap;       // rows in the ring
  int64_t step;           // positions are x^step
  int64_t steps_left;     // batch: steps still to run (< 0: unlimited)
  int32_t n_cells;
  int32_t active;         // 1: advanced by batch steps
  int32_t flags;          // sticky sic_diag flags
  int32_t live;           // slot holds a simulation
};

struct alignas(16) ChunkDesc {
  double q;               // segment charge
  int64_t q_fix;          // segment charge in fixed-point units
  int32_t partner;        // chunk whose first tracer follows this chunk's last
                          // valid tracer in the sheet; -1: open sheet end
  int32_t n_valid;        // valid tracer slots (1..64)
  int32_t inst;           // slot
  int32_t flags;          // kChunkOpenStart
};

enum ChunkFlags : int {
  kChunkOpenStart = 1,    // lane 0 is the first tracer of an open sheet (no segment before it)
};

struct alignas(16) Item {
  int32_t inst;
  int32_t chunk_begin;
  int32_t chunk_end;
  int32_t pad;
};

struct alignas(32) Partial {
  double ke, mom, maxseg, pad;
};

// Row layout of the history ring (matches sic_diag).
struct alignas(64) DiagRow {
  int64_t step;
  double t, W_E, KE, momentum, total_charge, max_segment;
  int64_t flags;
};

// Links from a chunk to single tracers of other chunks (piecewise-linear
// segments need two tracers past a chunk's end and one before its start):
// (chunk << 2) | which, which = 0 first, 1 second, 2 last tracer of that
// chunk; -1 when there is no such tracer (ends of an open sheet, or a closed
// sheet too short to have a gradient).
enum HaloWhich : int { kHaloFirst = 0, kHaloSecond = 1, kHaloLast = 2 };

struct SolveArgs {
  InstDesc *inst;
  const int2 *slot_items;    // per slot: (first item, item count) in the item list
  const int32_t *slot_list;  // NULL: slot = blockIdx.x
  const Partial *partials;
  void *meshP;
  void *meshD;
  void *meshR;               // order 1 only
  double *meshE;
  double *meshRho;           // n_j - nbar of the newest solve
  DiagRow *hist;
  int32_t *done;             // per slot: set to 1 when a batch run finishes
  int32_t flags;
  int32_t respect_active;
  int32_t order;             // deposit order of the pool (0, 1 or 2); R exists only for 1
  const int32_t *gate = nullptr;  // non-NULL: the launch does nothing unless *gate > 0
  // P, D and R are held in rep copies rep_stride words apart; the solve
  // sums them in copy order and clears each
  int32_t rep = 1;
  int64_t rep_stride = 0;
};

struct TracerArgs {
  const Item *items;
  const int32_t *n_items;  // device-side item count
  const InstDesc *inst;
  const ChunkDesc *chunks;
  const int2 *links;       // per chunk (prev link, next-but-one link); order 1
  const double2 *halo3_in; // per chunk: first, second, last tracer; order 1
  double2 *halo3_out;
  void *meshR;             // second-difference array for linear ramps; order 1
  uint64_t *xs;            // word 0 per slot
  double *vs;              // word 1 per slot
  const double2 *halo_in;  // (x word as bits, v) per chunk
  double2 *halo_out;
  void *meshP;             // direct cell charge (double or int64)
  void *meshD;             // difference array for covered cell runs
  const double *meshE;
  Partial *partials;       // per item
  const uint64_t *segq;    // per slot: charge of the segment starting there (per-segment pools)
  const uint64_t *cedge;   // per chunk: charge ending at lane 0, charge starting at the partner
  int32_t mesh_cells;      // LDS capacity in cells (max n_cells of the pool)
  int32_t tile_cap;        // LDS capacity in chunks per work item
  int32_t respect_active;  // skip slots with active == 0
  const int32_t *gate = nullptr;  // non-NULL: the launch does nothing unless *gate > 0
  // copies of P, D and R, rep_stride words apart: work item i merges into
  // copy i mod rep (fewer atomics on one address when many items share a
  // mesh)
  int32_t rep = 1;
  int64_t rep_stride = 0;
  // Solve-first launches of a single simulation (launch_tracers_sf): every
  // workgroup solves the previous step's charge for the field it pushes
  // with, instead of reading meshE; the first also writes what a solve
  // launch would (the diagnostics row, the step, the field and density).
  const void *sf_P = nullptr, *sf_D = nullptr;  // the previous step's accumulators
  void *sf_zP = nullptr, *sf_zD = nullptr;      // accumulators to clear, a slice per workgroup
  const Partial *sf_partials = nullptr;         // the previous launch's work-item partials
  SolveArgs sf{};                               // what the first workgroup's solve writes to
};

struct IngestArgs {
  const double *x_in;
  const uint64_t *w_in;       // raw state words instead of x_in (re-layout), or NULL
  const double *v_in;
  const double *c_in;         // per-segment charges (float64), or NULL
  const uint64_t *cw_in;      // raw per-segment charge words (re-layout), or NULL
  uint64_t *segq;             // NULL: the pool keeps no per-segment charges
  double q_scale;             // fixed-point units per unit charge (split forms)
  const int64_t *chunk_in_off;  // per chunk of the range: first input index
  int32_t chunk_begin;
  int32_t n_chunks;
  const ChunkDesc *chunks;
  const InstDesc *inst;
  uint64_t *xs;
  double *vs;
  double2 *halo;
  double2 *halo3;  // order 1 (NULL otherwise)
  const int32_t *state = nullptr;  // device refinement: skip unless state[kRefInserted] > 0, chunk
                                   // count state[kRefChunks] (the launch covers the capacity)
};

struct ExtractArgs {
  const int64_t *chunk_in_off;
  int32_t chunk_begin;
  int32_t n_chunks;
  const ChunkDesc *chunks;
  const InstDesc *inst;
  const uint64_t *xs;
  const double *vs;
  const uint64_t *segq;  // with c_out: per-segment charges
  double *x_out;
  double *v_out;
  double *c_out;         // NULL: positions and velocities only
};

// Refinement (section 2.6) of one slot's chunk range: a marking pass counts
// per chunk the segments longer than l_max (and keeps their lane mask); the
// scatter pass writes every tracer, plus a centre tracer after each marked
// one, to flat sheet-major output arrays (chunk cl starts at out_off[cl]).
struct RefineArgs {
  const ChunkDesc *chunks;
  const InstDesc *inst;
  const uint64_t *xs;
  const double *vs;
  const uint64_t *segq;
  int32_t chunk_begin;
  int32_t n_chunks;
  double l_max;
  int32_t *cnt;            // per chunk of the range
  uint64_t *mask;          // per chunk of the range
  const int64_t *out_off;  // per chunk of the range (scatter)
  uint64_t *w_out;
  double *v_out;
  uint64_t *c_out;
  const int32_t *state = nullptr;  // device refinement: chunk count state[kRefChunks]; the marking pass
                                   // skips after a halt, the scatter unless state[kRefInserted] > 0
};

// Refinement done entirely on the device (one simulation, steps in a row):
// int32 words of its state.  kRefChunks: chunks of the slot now;
// kRefInserted: tracers the last pass inserted (0: nothing to re-lay out);
// kRefHalt: set when a pass would exceed the capacity (sticky; the slot is
// made inactive, so the following steps do nothing); kRefNextChunks: chunks
// after the pending re-layout.
enum RefineState : int { kRefChunks = 0, kRefInserted = 1, kRefHalt = 2, kRefNextChunks = 3, kRefWords = 8 };

// The re-layout of one simulation after a refinement pass, planned and
// written on the device (the counterpart of the host's layout building).
struct RefinePlanArgs {
  ChunkDesc *chunks;       // pool descriptors; the slot's range is rewritten
  int2 *links;             // order 1 (NULL otherwise)
  int64_t *edge_prev;      // per chunk: slot of the tracer before its first one
  int64_t *in_off;         // per chunk of the range: first index in the flat staging
  Item *items;             // the slot's item range (room for the capacity)
  int2 *slot_items;        // per slot: (first item, item count)
  int32_t *n_items;        // item count the tracer kernel walks
  InstDesc *inst;
  const int32_t *cnt;      // per chunk of the range: segments to split
  int64_t *out_off;        // per chunk of the range: first index in the flat staging
  int32_t *nt;             // per sheet: tracers now
  const int32_t *closed;   // per sheet
  const double *q;         // per sheet: charge kept in the descriptors
  int64_t *work;           // 3 n_sheets + 3 entries (per sheet: new count, new first chunk, flat start)
  int32_t *state;          // RefineState words
  int64_t max_tracers;
  double q_scale;
  int32_t n_sheets;
  int32_t chunk_begin;
  int32_t chunk_cap;       // chunks reserved for the slot
  int32_t tile;            // chunks per work item
  int32_t slot;
  int32_t item_begin;
  int32_t order;
  int32_t fixed;           // split forms: descriptors carry fixed-point charges
};

// Launchers (sic_kernels.hip).  All return hipError_t as int.
int launch_tracers(int prec, int mode, int order, bool seg, const TracerArgs &a, int grid, int block,
                   size_t lds_bytes, void *stream);
// A fused step (push + deposit, constant segments) of a single simulation in
// solve-first form (TracerArgs sf_*); max_cells sizes the solve.
int launch_tracers_sf(int prec, bool seg, const TracerArgs &a, int grid, int block, size_t lds_bytes,
                      int max_cells, void *stream);
int set_tracer_lds_limit(int prec, int order, bool seg, size_t lds_bytes);
size_t tracer_lds_size(int prec, int order, bool seg, int mesh_cells, int tile_cap);
// max_cells: the largest mesh of the slots the launch may solve.
int launch_solve(int prec, const SolveArgs &a, int n_blocks, int max_cells, void *stream);
int launch_ingest(int prec, const IngestArgs &a, void *stream);
int launch_extract(int prec, const ExtractArgs &a, void *stream);
// Clears the meshes of the listed slots in all rep copies (rep_stride words apart).
int launch_zero_mesh(int prec, void *meshP, void *meshD, void *meshR, const InstDesc *inst,
                     const int32_t *slot_list, int n_blocks, int rep, int64_t rep_stride, void *stream);
// grid: workgroups of 256 threads
int launch_copy_bench(const double *src, double *dst, int64_t n, int grid, void *stream);
// Charge edges of chunks [chunk_begin, chunk_begin + n_chunks): prev_slot[c]
// is the slot of the tracer before chunk c's first one (-1: none).
int launch_charge_edges(const ChunkDesc *chunks, const int64_t *prev_slot, const uint64_t *segq, uint64_t *cedge,
                        int32_t chunk_begin, int32_t n_chunks, void *stream, const int32_t *state = nullptr);
// A small simulation's n_steps fused steps (push, deposit, solve) in one
// launch of one workgroup; chunks [chunk_begin, chunk_begin + n_chunks) of
// slot 0, constant segments.  a.halo_out receives the first-tracer halos of
// the final state.
int resident_max_chunks();
int launch_resident(int prec, bool seg, const TracerArgs &a, const SolveArgs &sa, int chunk_begin, int n_chunks,
                    int n_cells, int64_t n_steps, void *stream);
// With a.state the launches cover a.n_chunks chunks (the capacity) and read
// the count from the device.
int launch_refine_mark(int prec, const RefineArgs &a, void *stream);
int launch_refine_scatter(int prec, const RefineArgs &a, void *stream);
// Device re-layout: the plan (one workgroup) and the descriptor/item writer
// (covers chunk_cap chunks).
int launch_refine_plan(const RefinePlanArgs &a, void *stream);
int launch_refine_layout(const RefinePlanArgs &a, void *stream);

}  // namespace sic
