// sic_api.hip - host side of libsic: the C ABI declared in include/sic.h.
//
// One internal object, Pool, backs both handles.  A pool owns device memory
// for a fixed number of simulation slots, a chunk-granular tracer arena, the
// per-slot meshes and diagnostics rings, and the work-item list that the
// tracer kernel walks.  A sic_sim is a pool with one slot; a sic_batch is a
// pool with many slots whose simulations advance in shared launches.
//
// Per step the device runs two kernels: the tracer kernel (gather, leapfrog
// move, deposit of the new positions into the mesh) and the field solve (one
// workgroup per slot).  Runs of steps are captured once into HIP graphs on a
// private stream and replayed on the caller's stream; the graphs read the
// item list and slot table from device memory, so admitting or retiring a
// simulation never needs a new capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/sic.h"
#include "sic_internal.h"

using namespace sic;

namespace {

constexpr int kGraphSteps = 32;         // steps per captured graph
constexpr int kSfMaxGrid = 512;         // solve-first steps up to this many workgroups (two per CU)
constexpr int kDefaultGrid = 2048;       // grid of a pool before its first items are placed
constexpr int kMinBatchGrid = 4096;      // smallest default batch grid (16 workgroups per CU)
constexpr int kMaxGrid = 1 << 20;        // largest default grid (the kernels loop over any excess items)
constexpr int kDefaultBlock = 256;       // single simulations
constexpr int kDefaultBatchBlock = 512;  // batches
constexpr int kDefaultBatchTile = 256;   // chunks per batch work item (16k tracers per LDS mesh merge)
constexpr int kLinearBatchTile = 192;    // piecewise-linear segments: three workgroups per CU in LDS
// (batch defaults: the autotuner's choice on the 4096-instance mixed batch)
constexpr int kMinTile = 4;             // chunks per work item, lower bound
constexpr int kMaxTile = 256;

enum SimState { kStale = 0, kDeposited = 1, kField = 2 };

struct Range {
  int64_t begin, end;
};

// First-fit allocator of contiguous chunk ranges.
class ChunkAllocator {
 public:
  void init(int64_t n) {
    free_.clear();
    if (n > 0) free_.push_back({0, n});
  }
  int64_t alloc(int64_t n) {
    for (size_t i = 0; i < free_.size(); ++i) {
      if (free_[i].end - free_[i].begin >= n) {
        const int64_t b = free_[i].begin;
        free_[i].begin += n;
        if (free_[i].begin == free_[i].end) free_.erase(free_.begin() + (long)i);
        return b;
      }
    }
    return -1;
  }
  // One past the last allocated element (0 when nothing is allocated).
  int64_t used_end(int64_t cap) const {
    if (!free_.empty() && free_.back().end == cap) return free_.back().begin;
    return cap;
  }
  void release(int64_t b, int64_t n) {
    if (n <= 0) return;
    Range r{b, b + n};
    auto it = std::lower_bound(free_.begin(), free_.end(), r,
                               [](const Range &a, const Range &c) { return a.begin < c.begin; });
    it = free_.insert(it, r);
    // merge with neighbours
    if (it + 1 != free_.end() && it->end == (it + 1)->begin) {
      it->end = (it + 1)->end;
      free_.erase(it + 1);
    }
    if (it != free_.begin() && (it - 1)->end == it->begin) {
      (it - 1)->end = it->end;
      free_.erase(it);
    }
  }

 private:
  std::vector<Range> free_;
};

struct SlotHost {
  bool live = false;
  int32_t n_cells = 0;
  double L = 0.0, dt = 0.0;
  int64_t n_tracers = 0;
  // sheets as they are now (refinement grows n_tracers_s)
  std::vector<int32_t> n_tracers_s, closed_s;
  std::vector<double> q_s;
  double q_scale = 1.0;   // fixed-point units per unit charge (split forms)
  double l_max = 0.0;     // refinement length; 0: off
  int64_t max_tracers = 0;
  int32_t chunk_begin = 0, n_chunks = 0;
  int32_t n_chunks_res = 0;  // chunks reserved from chunk_begin (room to grow by refinement)
  int32_t item_begin = 0, n_items = 0;
  std::vector<int64_t> chunk_in_off;
  int64_t *d_in_off = nullptr;
  int state = kStale;
  // the step the diagnostics history starts at: 0, or the step a state was
  // set or loaded at (rows before it were never written by this simulation)
  int64_t hist_from = 0;
  bool pending_push = false, pending_dep = false;
  bool reported = false;
};

}  // namespace

struct Pool {
  int prec = 0;
  int order = 0;  // deposit order: 0 piecewise-constant, 1 piecewise-linear, 2 first-order weighting
  int device = 0;    // HIP device current at creation
  bool seg = false;  // per-segment charges
  bool batch = false;
  hipStream_t stream = nullptr;  // caller's stream
  hipStream_t cap = nullptr;     // private capture stream
  int32_t slot_cap = 0, max_cells = 0;
  int64_t chunk_cap = 0, item_cap = 0, hist_rows = 0, budget = 0;
  int64_t used_tracers = 0;
  int32_t used_slots = 0;
  size_t lds_bytes = 0;

  uint64_t *xs = nullptr;
  double *vs = nullptr;
  double2 *halo[2] = {nullptr, nullptr};
  double2 *halo3[2] = {nullptr, nullptr};  // order 1
  int2 *links = nullptr;
  ChunkDesc *chunks = nullptr;
  Item *items = nullptr;
  int32_t *n_items = nullptr;
  InstDesc *inst = nullptr;
  int2 *slot_items = nullptr;
  Partial *partials = nullptr;
  // P, D (and R) in rep copies of slot_cap * max_cells words each
  void *meshP = nullptr;
  void *meshD = nullptr;
  void *meshR = nullptr;  // order 1
  int rep = 1;
  double *meshE = nullptr;
  double *meshRho = nullptr;
  DiagRow *hist = nullptr;
  int32_t *done = nullptr;
  int32_t *slot_ids = nullptr;
  uint64_t *segq = nullptr;      // per slot (seg)
  uint64_t *cedge = nullptr;     // 2 per chunk (seg)
  int64_t *edge_prev = nullptr;  // per chunk (seg)
  // refinement scratch (allocated on first use)
  int32_t *ref_cnt = nullptr;
  uint64_t *ref_mask = nullptr;
  int64_t *ref_off = nullptr;
  uint64_t *ref_w = nullptr;
  double *ref_v = nullptr;
  uint64_t *ref_c = nullptr;
  int64_t ref_stage_cap = 0;
  // device-side refinement of a single simulation (allocated on first use)
  bool dev_refine = false;       // steps are refining on the device (host layout mirror stale)
  bool dr_items = false;         // slot 0's work items are laid out for its whole reservation
  int32_t *dr_nt = nullptr;      // per sheet: tracers now
  int32_t *dr_closed = nullptr;  // per sheet
  double *dr_q = nullptr;        // per sheet
  int64_t *dr_work = nullptr;    // plan scratch, 3 n_sheets + 3
  int32_t *dr_state = nullptr;   // RefineState words
  int64_t *dr_in_off = nullptr;  // per chunk of the reservation: first staging index
  int32_t dr_sheets = 0, dr_chunks = 0;
  // solve-first steps of a single simulation (allocated on first use): two
  // more accumulator pairs (the pool's own is the third) and a second set of
  // work-item partials
  void *sf_mesh = nullptr;     // P1, D1, P2, D2: rep copies of mesh_words each
  Partial *sf_part = nullptr;  // item_cap

  std::vector<SlotHost> slots;
  ChunkAllocator alloc;       // tracer chunks
  ChunkAllocator item_alloc;  // work items
  std::vector<int2> slot_items_h;
  int32_t n_items_h = 0;      // item high-water mark (items the kernel walks)
  int parity = 0;
  sic_tuning tune{};  // requested (0 = automatic)
  int block = kDefaultBlock, grid = kDefaultGrid, tile = kMinTile;
  int solve_grid = 1;  // solve workgroups of a whole-pool step: live slot indices, rounded up
  // (steps, parity, grid, solve grid, device refinement: the launches then skip an inactive slot)
  std::map<std::tuple<int64_t, int, int, int, int>, hipGraphExec_t> graphs;
  std::vector<hipGraph_t> graph_objs;
  bool timing = false;
  double t_tracer = 0.0, t_solve = 0.0;
  int last_path = SIC_PATH_NONE;  // launch path of the last single-simulation step call
  std::string err;
};

struct sic_sim {
  Pool *pool;
};
struct sic_batch {
  Pool *pool;
};

namespace {

// Message of the last failure on this host thread (reported through
// sic_last_error(NULL) when no handle exists, e.g. after a failed sic_init).
thread_local std::string g_last_error;

sic_status fail(Pool *p, sic_status s, const std::string &msg) {
  if (p) p->err = msg;
  g_last_error = msg;
  return s;
}

// Staging memory of the entry points that allocate nothing: one fixed array
// per GPU (each device holds its own copy of this module-scope array), 16
// bytes per tracer for SIC_NOALLOC_MAX_TRACERS tracers.  In host code the
// name stands for a host-side shadow, not a device address: kernels and
// copies get the address hipGetSymbolAddress returns for the device, looked
// up once per device when a pool is created there.
static __device__ __align__(256) double scratch[2 * (size_t)SIC_NOALLOC_MAX_TRACERS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device.
hipError_t scratch_address(int device, double **out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[device] = static_cast<double *>(ptr);
  }
  *out = g_scratch_dev[device];
  return hipSuccess;
}

#define HIPCHK(p, expr)                                                                          \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) {                                                                      \
      return fail((p), SIC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));          \
    }                                                                                            \
  } while (0)

#define LAUNCHCHK(p, expr)                                                                       \
  do {                                                                                           \
    int e_ = (expr);                                                                             \
    if (e_ != 0) {                                                                               \
      return fail((p), SIC_EDEVICE,                                                              \
                  std::string(#expr) + ": " + hipGetErrorString((hipError_t)e_));                \
    }                                                                                            \
  } while (0)

template <class T>
hipError_t dalloc(T **p, size_t n) {
  if (n == 0) n = 1;
  return hipMalloc((void **)p, n * sizeof(T));
}

void destroy_graphs(Pool *p) {
  for (auto &kv : p->graphs) hipGraphExecDestroy(kv.second);
  p->graphs.clear();
  for (auto g : p->graph_objs) hipGraphDestroy(g);
  p->graph_objs.clear();
}

void pool_free(Pool *p) {
  if (!p) return;
  hipStreamSynchronize(p->stream);  // teardown: nothing to report an error to
  destroy_graphs(p);
  for (auto &s : p->slots)
    if (s.d_in_off) hipFree(s.d_in_off);
  void *bufs[] = {p->xs,        p->vs,       p->halo[0],  p->halo[1],  p->halo3[0],  p->halo3[1],
                  p->links,     p->chunks,   p->items,    p->n_items,  p->inst,      p->slot_items,
                  p->partials,  p->meshP,    p->meshD,    p->meshR,    p->meshE,     p->meshRho,
                  p->hist,      p->done,     p->slot_ids, p->segq,     p->cedge,     p->edge_prev,
                  p->ref_cnt,   p->ref_mask, p->ref_off,  p->ref_w,    p->ref_v,     p->ref_c,
                  p->dr_nt,     p->dr_closed, p->dr_q,    p->dr_work,  p->dr_state,  p->dr_in_off,
                  p->sf_mesh,   p->sf_part};
  for (void *b : bufs)
    if (b) hipFree(b);
  if (p->cap) hipStreamDestroy(p->cap);
  delete p;
}

sic_status pool_create(int prec, int order, bool seg, bool batch, int32_t slot_cap, int32_t max_cells,
                       int64_t chunk_cap, int64_t hist_rows, int64_t budget, void *stream, Pool **out,
                       std::string *err) {
  if (chunk_cap >= ((int64_t)1 << 29)) {  // chunk links pack a chunk index into 29 bits
    if (err) *err = "tracer arena too large";
    g_last_error = "tracer arena too large";
    return SIC_ENOMEM;
  }
  Pool *p = new Pool();
  p->prec = prec;
  p->order = order;
  p->seg = seg;
  p->batch = batch;
  if (hipGetDevice(&p->device) != hipSuccess) p->device = 0;
  p->stream = (hipStream_t)stream;
  p->slot_cap = slot_cap;
  p->max_cells = max_cells;
  p->chunk_cap = chunk_cap;
  p->item_cap = chunk_cap / kMinTile + slot_cap + 1;
  p->hist_rows = hist_rows;
  p->budget = budget;
  p->lds_bytes = tracer_lds_size(prec, order, seg, max_cells, kMaxTile);
  p->slots.resize(slot_cap);
  p->slot_items_h.assign(slot_cap, make_int2(0, 0));
  p->alloc.init(chunk_cap);
  p->item_alloc.init(p->item_cap);

  auto bail = [&](const std::string &m, sic_status s) {
    if (err) *err = m;
    g_last_error = m;
    pool_free(p);
    return s;
  };
  hipError_t e = hipSuccess;
#define ALLOC(ptr, n)                                                                  \
  e = dalloc(&(ptr), (n));                                                             \
  if (e != hipSuccess) return bail(std::string("hipMalloc ") + #ptr + ": " + hipGetErrorString(e), SIC_ENOMEM);
  const size_t slotsz = (size_t)chunk_cap * kChunk;
  ALLOC(p->xs, slotsz);
  ALLOC(p->vs, slotsz);
  ALLOC(p->halo[0], (size_t)chunk_cap);
  ALLOC(p->halo[1], (size_t)chunk_cap);
  ALLOC(p->links, (size_t)chunk_cap);
  if (order == 1) {
    ALLOC(p->halo3[0], 3 * (size_t)chunk_cap);
    ALLOC(p->halo3[1], 3 * (size_t)chunk_cap);
  }
  ALLOC(p->chunks, (size_t)chunk_cap);
  if (seg) {
    ALLOC(p->segq, slotsz);
    ALLOC(p->cedge, 2 * (size_t)chunk_cap);
    ALLOC(p->edge_prev, (size_t)chunk_cap);
  }
  ALLOC(p->items, (size_t)p->item_cap);
  ALLOC(p->n_items, 1);
  ALLOC(p->inst, (size_t)slot_cap);
  ALLOC(p->slot_items, (size_t)slot_cap);
  ALLOC(p->partials, (size_t)p->item_cap);
  {
    // the no-allocation entry points' staging array on this device, looked
    // up here once per device (a failure is reported by those entry points,
    // which look it up again)
    double *sp = nullptr;
    (void)scratch_address(p->device, &sp);
  }
  p->rep = batch ? 1 : single_rep(max_cells);
  {
    const size_t mc = (size_t)slot_cap * max_cells;
    long long *mp = nullptr, *md = nullptr;
    ALLOC(mp, mc * p->rep);
    p->meshP = mp;
    ALLOC(md, mc * p->rep);
    p->meshD = md;
    if (order == 1) {
      long long *mr = nullptr;
      ALLOC(mr, mc * p->rep);
      p->meshR = mr;
    }
    ALLOC(p->meshE, mc);
    ALLOC(p->meshRho, mc);
  }
  ALLOC(p->hist, (size_t)slot_cap * hist_rows);
  ALLOC(p->done, (size_t)slot_cap);
  ALLOC(p->slot_ids, (size_t)slot_cap);
#undef ALLOC
  e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
  if (e != hipSuccess) return bail(std::string("hipStreamCreate: ") + hipGetErrorString(e), SIC_EDEVICE);
  // zero-initialise everything the kernels accumulate into or read as tables
  const size_t mc = (size_t)slot_cap * max_cells;
  e = hipMemsetAsync(p->meshP, 0, mc * 8 * p->rep, p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(p->meshD, 0, mc * 8 * p->rep, p->stream);
  if (e == hipSuccess && p->meshR) e = hipMemsetAsync(p->meshR, 0, mc * 8 * p->rep, p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(p->meshE, 0, mc * 8, p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(p->meshRho, 0, mc * 8, p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(p->inst, 0, sizeof(InstDesc) * (size_t)slot_cap, p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(p->slot_items, 0, sizeof(int2) * (size_t)slot_cap, p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(p->done, 0, sizeof(int32_t) * (size_t)slot_cap, p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(p->n_items, 0, sizeof(int32_t), p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(p->partials, 0, sizeof(Partial) * (size_t)p->item_cap, p->stream);
  if (e != hipSuccess) return bail(std::string("hipMemsetAsync: ") + hipGetErrorString(e), SIC_EDEVICE);
  std::vector<int32_t> ids(slot_cap);
  for (int32_t i = 0; i < slot_cap; ++i) ids[i] = i;
  e = hipMemcpyAsync(p->slot_ids, ids.data(), sizeof(int32_t) * (size_t)slot_cap, hipMemcpyHostToDevice,
                     p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return bail(std::string("init copy: ") + hipGetErrorString(e), SIC_EDEVICE);
  if (p->lds_bytes > 65536) {
    int le = set_tracer_lds_limit(prec, order, seg, p->lds_bytes);
    if (le != 0) return bail(std::string("LDS limit: ") + hipGetErrorString((hipError_t)le), SIC_ENOTSUP);
  }
  *out = p;
  return SIC_OK;
}

// Work-item size in chunks for a slot of n_chunks chunks.  A batch uses one
// size for every slot; a single simulation sizes its items to give the
// machine about 2048 of them, up to the largest item (fewer, larger items
// spend less on zeroing and merging the item's LDS mesh).  An item clears
// and scans its whole LDS mesh, and once a sheet has folded over the box it
// merges nearly every cell into the global mesh (one atomic each), so items
// hold at least 4 tracers per mesh cell where that still leaves one item per
// compute unit.  Atomics on one address serialise (about 22 ns each), so a
// small mesh also caps the items that merge into one accumulator copy: at
// most max(256, cells x copies / 2) items (a million tracers on 100 cells:
// 256 items of 64 chunks, not 2048 of 8); not for the layout of a refining
// simulation's whole reservation (cap_items false), whose items are mostly
// empty while it grows.
int slot_tile(const Pool *p, int64_t n_chunks, bool cap_items = true) {
  if (p->tune.tile_chunks > 0) return std::max(kMinTile, std::min(kMaxTile, (int)p->tune.tile_chunks));
  const int wave_min = p->block / kChunk;
  if (p->batch) return std::max(p->order == 1 ? kLinearBatchTile : kDefaultBatchTile, wave_min);
  const int64_t per = (n_chunks + 2047) / 2048;
  const int64_t mesh_min = (4 * (int64_t)p->max_cells + kChunk - 1) / kChunk;
  const int64_t max_items = std::max<int64_t>(256, (int64_t)p->max_cells * p->rep / 2);
  const int64_t contention = cap_items ? (n_chunks + max_items - 1) / max_items : 1;
  const int64_t want = std::max(std::max(per, contention), std::min(mesh_min, n_chunks / 256));
  int t = (int)std::max<int64_t>(kMinTile, std::min<int64_t>(kMaxTile, want));
  t = (t + 3) / 4 * 4;
  return std::max(t, wave_min);
}

constexpr size_t kLdsPerCU = 160 * 1024;

void apply_launch_shape(Pool *p) {
  if (p->tune.block_threads > 0) {
    p->block = p->tune.block_threads;
  } else {
    // Large meshes leave room for one or two workgroups per CU in LDS; give
    // those workgroups more waves so the CU still has enough loads in flight.
    const size_t lds = tracer_lds_size(p->prec, p->order, p->seg, p->max_cells, p->tile);
    const size_t per_cu = lds > 0 ? kLdsPerCU / lds : 8;
    // items of 8 chunks or more have work for 8 wavefronts each
    p->block = (p->batch || p->tile >= 8) ? kDefaultBatchBlock : kDefaultBlock;
    if (per_cu <= 1) p->block = 1024;
    else if (per_cu == 2) p->block = std::max(p->block, 512);
  }
  if (p->tune.grid_blocks > 0) {
    p->grid = p->tune.grid_blocks;
  } else if (p->batch) {
    // One work item per workgroup: the dispatcher starts a new workgroup as
    // soon as one retires, so one workgroup's mesh clear and merge overlap
    // the streaming of the others, which a persistent grid serialises.  The
    // count is rounded up to a power of two so that a batch whose item
    // arena grows slot by slot captures new graphs only now and then (the
    // surplus workgroups read the item count and exit).
    int g = kMinBatchGrid;
    while (g < p->n_items_h && g < kMaxGrid) g *= 2;
    p->grid = g;
  } else {
    p->grid = std::max(1, std::min<int>(p->n_items_h, kMaxGrid));
  }
}

// The whole-pool solve launches one workgroup per slot index up to the
// highest live one (slots are taken lowest first), rounded up to a power of
// two so that graphs are captured again only when that crosses one; the
// workgroups of slots that are not live return at once.
void update_solve_grid(Pool *p) {
  int32_t hw = 0;
  for (int32_t i = p->slot_cap - 1; i >= 0; --i)
    if (p->slots[i].live) {
      hw = i + 1;
      break;
    }
  int g = 1;
  while (g < hw) g *= 2;
  p->solve_grid = std::min(g, (int)p->slot_cap);
}

// Uploads the device-side item count (the high-water mark of the item arena).
sic_status upload_item_count(Pool *p) {
  p->n_items_h = (int32_t)p->item_alloc.used_end(p->item_cap);
  HIPCHK(p, hipMemcpyAsync(p->n_items, &p->n_items_h, sizeof(int32_t), hipMemcpyHostToDevice, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  apply_launch_shape(p);
  return SIC_OK;
}

// Lays out the work items of one slot in the item arena and uploads them.
sic_status place_slot_items(Pool *p, int32_t slot) {
  SlotHost &s = p->slots[slot];
  p->dr_items = false;
  const int tile = slot_tile(p, s.n_chunks);
  p->tile = tile;
  const int32_t n = (s.n_chunks + tile - 1) / tile;
  const int64_t ib = p->item_alloc.alloc(n);
  if (ib < 0) return fail(p, SIC_EBUSY, "work-item arena full");
  std::vector<Item> its((size_t)n);
  for (int32_t k = 0; k < n; ++k) {
    its[k].inst = slot;
    its[k].chunk_begin = s.chunk_begin + k * tile;
    its[k].chunk_end = s.chunk_begin + std::min(s.n_chunks, (k + 1) * tile);
    its[k].pad = 0;
  }
  s.item_begin = (int32_t)ib;
  s.n_items = n;
  p->slot_items_h[slot] = make_int2((int32_t)ib, n);
  HIPCHK(p, hipMemcpyAsync(p->items + ib, its.data(), sizeof(Item) * (size_t)n, hipMemcpyHostToDevice, p->stream));
  HIPCHK(p, hipMemcpyAsync(p->slot_items + slot, &p->slot_items_h[slot], sizeof(int2), hipMemcpyHostToDevice,
                           p->stream));
  return upload_item_count(p);
}

// Marks a slot's items dead (the kernels skip them) and frees their range.
sic_status clear_slot_items(Pool *p, int32_t slot) {
  SlotHost &s = p->slots[slot];
  if (s.n_items > 0) {
    std::vector<Item> dead((size_t)s.n_items);
    for (auto &it : dead) {
      it.inst = -1;
      it.chunk_begin = it.chunk_end = it.pad = 0;
    }
    HIPCHK(p, hipMemcpyAsync(p->items + s.item_begin, dead.data(), sizeof(Item) * dead.size(), hipMemcpyHostToDevice,
                             p->stream));
    HIPCHK(p, hipStreamSynchronize(p->stream));
    p->item_alloc.release(s.item_begin, s.n_items);
  }
  s.item_begin = 0;
  s.n_items = 0;
  p->slot_items_h[slot] = make_int2(0, 0);
  HIPCHK(p, hipMemcpyAsync(p->slot_items + slot, &p->slot_items_h[slot], sizeof(int2), hipMemcpyHostToDevice,
                           p->stream));
  return upload_item_count(p);
}

sic_status run_fused(Pool *p, int64_t n);

// Re-lays out every live slot's items (after a tuning change) in one upload.
sic_status relayout_items(Pool *p) {
  HIPCHK(p, hipStreamSynchronize(p->stream));
  p->item_alloc.init(p->item_cap);
  std::vector<Item> its;
  int tile = p->tile;
  for (int32_t i = 0; i < p->slot_cap; ++i) {
    SlotHost &s = p->slots[i];
    if (!s.live) {
      p->slot_items_h[i] = make_int2(0, 0);
      continue;
    }
    tile = slot_tile(p, s.n_chunks);
    const int32_t n = (s.n_chunks + tile - 1) / tile;
    const int64_t ib = p->item_alloc.alloc(n);
    if (ib < 0 || ib != (int64_t)its.size()) return fail(p, SIC_ENOMEM, "work-item arena full");
    for (int32_t k = 0; k < n; ++k) {
      Item it;
      it.inst = i;
      it.chunk_begin = s.chunk_begin + k * tile;
      it.chunk_end = s.chunk_begin + std::min(s.n_chunks, (k + 1) * tile);
      it.pad = 0;
      its.push_back(it);
    }
    s.item_begin = (int32_t)ib;
    s.n_items = n;
    p->slot_items_h[i] = make_int2((int32_t)ib, n);
  }
  p->tile = tile;
  if (!its.empty())
    HIPCHK(p, hipMemcpyAsync(p->items, its.data(), sizeof(Item) * its.size(), hipMemcpyHostToDevice, p->stream));
  HIPCHK(p, hipMemcpyAsync(p->slot_items, p->slot_items_h.data(), sizeof(int2) * p->slot_items_h.size(),
                           hipMemcpyHostToDevice, p->stream));
  return upload_item_count(p);
}

// Device copy of everything a step modifies, so trial steps (autotuning) can
// be undone.
struct Snapshot {
  std::vector<std::pair<void *, size_t>> bufs;  // (copy, bytes) per source buffer
  std::vector<void *> srcs;
  int parity = 0;
};

void snapshot_free(Snapshot &s) {
  for (auto &b : s.bufs)
    if (b.first) hipFree(b.first);
  s.bufs.clear();
  s.srcs.clear();
}

sic_status snapshot_take(Pool *p, Snapshot &s) {
  const size_t mc = (size_t)p->slot_cap * p->max_cells * 8;
  const size_t slots = (size_t)p->chunk_cap * kChunk * 8;
  std::pair<void *, size_t> src[] = {
      {p->xs, slots},
      {p->vs, slots},
      {p->halo[0], (size_t)p->chunk_cap * sizeof(double2)},
      {p->halo[1], (size_t)p->chunk_cap * sizeof(double2)},
      {p->halo3[0], p->halo3[0] ? 3 * (size_t)p->chunk_cap * sizeof(double2) : 0},
      {p->halo3[1], p->halo3[1] ? 3 * (size_t)p->chunk_cap * sizeof(double2) : 0},
      {p->meshR, p->meshR ? mc * p->rep : 0},
      {p->meshP, mc * p->rep},
      {p->meshD, mc * p->rep},
      {p->meshE, mc},
      {p->meshRho, mc},
      {p->inst, sizeof(InstDesc) * (size_t)p->slot_cap},
      {p->hist, sizeof(DiagRow) * (size_t)p->slot_cap * p->hist_rows},
      {p->done, sizeof(int32_t) * (size_t)p->slot_cap},
  };
  HIPCHK(p, hipStreamSynchronize(p->stream));
  for (auto &b : src) {
    if (!b.first || b.second == 0) continue;
    void *d = nullptr;
    if (hipMalloc(&d, b.second) != hipSuccess) {
      snapshot_free(s);
      return fail(p, SIC_ENOMEM, "no device memory for the tuning snapshot");
    }
    s.bufs.push_back({d, b.second});
    s.srcs.push_back(b.first);
    HIPCHK(p, hipMemcpyAsync(d, b.first, b.second, hipMemcpyDeviceToDevice, p->stream));
  }
  s.parity = p->parity;
  HIPCHK(p, hipStreamSynchronize(p->stream));
  return SIC_OK;
}

sic_status snapshot_restore(Pool *p, Snapshot &s) {
  for (size_t i = 0; i < s.bufs.size(); ++i)
    HIPCHK(p, hipMemcpyAsync(s.srcs[i], s.bufs[i].first, s.bufs[i].second, hipMemcpyDeviceToDevice, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  p->parity = s.parity;
  return SIC_OK;
}

// Times every candidate launch shape on the pool's own resident simulations
// (HIP events around each kernel), then restores the state and keeps the
// fastest shape.  Candidates: chunks per work item (LDS mesh merges per
// tracer), threads per workgroup (waves sharing one LDS mesh) and grid size
// (one item per workgroup, or fewer workgroups looping over the items).
sic_status pool_autotune(Pool *p, int32_t steps, sic_tuning *best_out, double *best_ms_out) {
  if (steps < 1) return fail(p, SIC_EINVAL, "steps_per_trial < 1");
  Snapshot snap;
  sic_status st = snapshot_take(p, snap);
  if (st != SIC_OK) return st;
  const sic_tuning saved = p->tune;
  const bool saved_timing = p->timing;
  p->timing = true;
  const int tiles[] = {0, 16, 32, 64, 128, 256};  // 0: the default item size
  const int blocks[] = {256, 512, 1024};
  const int grids[] = {0, 1024, 2048, 4096};  // 0: one work item per workgroup
  // the shape in effect is timed first, and a candidate replaces it only when
  // it is faster by more than the trials' noise
  constexpr double kMargin = 0.98;
  sic_tuning best = saved;
  double best_ms = 1e300, best_key = 1e300;  // measured time; time compared (the margin applied)
  {
    p->tune = saved;
    destroy_graphs(p);
    apply_launch_shape(p);
    st = relayout_items(p);
    if (st == SIC_OK) st = run_fused(p, 1);
    if (st == SIC_OK) st = run_fused(p, steps);
    if (st == SIC_OK) {
      best_ms = p->t_tracer + p->t_solve;
      best_key = kMargin * best_ms;
    }
  }
  for (int t : tiles) {
    if (st != SIC_OK) break;
    for (int b : blocks) {
      if (t > 0 && t * kChunk < b) continue;  // every wave gets at least one chunk
      for (int g : grids) {
        sic_tuning cand{t, b, g, saved.fused_only};
        p->tune = cand;
        destroy_graphs(p);
        apply_launch_shape(p);
        st = relayout_items(p);
        if (st == SIC_OK) st = run_fused(p, 1);
        if (st == SIC_OK) st = run_fused(p, steps);
        if (st != SIC_OK) break;
        const double ms = p->t_tracer + p->t_solve;
        if (ms < best_key) {
          best_ms = best_key = ms;
          best = cand;
        }
      }
      if (st != SIC_OK) break;
    }
    if (st != SIC_OK) break;
  }
  p->timing = saved_timing;
  sic_status rs = snapshot_restore(p, snap);
  snapshot_free(snap);
  p->tune = (st == SIC_OK) ? best : saved;
  destroy_graphs(p);
  apply_launch_shape(p);
  sic_status ls = relayout_items(p);
  if (st != SIC_OK) return st;
  if (rs != SIC_OK) return rs;
  if (ls != SIC_OK) return ls;
  if (best_out) {
    best_out->tile_chunks = p->tile;
    best_out->block_threads = p->block;
    best_out->grid_blocks = p->grid;
    best_out->fused_only = p->tune.fused_only;
  }
  if (best_ms_out) *best_ms_out = best_ms;
  return SIC_OK;
}

// Words of one copy of a charge accumulator (every slot's mesh).
int64_t mesh_words(const Pool *p) { return (int64_t)p->slot_cap * p->max_cells; }

TracerArgs tracer_args(Pool *p, int mode, int slot) {
  TracerArgs a;
  const bool one = slot >= 0;
  const int first = one ? p->slot_items_h[slot].x : 0;
  a.items = p->items + first;
  a.n_items = one ? &(p->slot_items + slot)->y : p->n_items;
  a.inst = p->inst;
  a.chunks = p->chunks;
  a.links = p->links;
  a.xs = p->xs;
  a.vs = p->vs;
  const int out_parity = (mode == (kPush | kDeposit)) ? p->parity ^ 1 : p->parity;
  a.halo_in = p->halo[p->parity];
  a.halo_out = p->halo[out_parity];
  a.halo3_in = p->halo3[p->parity];
  a.halo3_out = p->halo3[out_parity];
  a.meshR = p->meshR;
  a.meshP = p->meshP;
  a.meshD = p->meshD;
  a.meshE = p->meshE;
  a.partials = p->partials + first;
  a.segq = p->segq;
  a.cedge = p->cedge;
  a.mesh_cells = p->max_cells;
  a.tile_cap = p->tile;
  a.rep = p->rep;
  a.rep_stride = mesh_words(p);
  // batches skip finished slots; a single simulation refining on the device
  // is made inactive when a pass would exceed its capacity
  a.respect_active = ((p->batch || p->dev_refine) && !one) ? 1 : 0;
  return a;
}

SolveArgs solve_args(Pool *p, int flags, int slot) {
  SolveArgs a;
  a.inst = p->inst;
  a.slot_items = p->slot_items;
  a.slot_list = slot >= 0 ? p->slot_ids + slot : nullptr;
  a.partials = p->partials;
  a.meshP = p->meshP;
  a.meshD = p->meshD;
  a.meshR = p->meshR;
  a.order = p->order;
  a.meshE = p->meshE;
  a.meshRho = p->meshRho;
  a.hist = p->hist;
  a.done = p->done;
  a.flags = flags;
  a.respect_active = ((p->batch || p->dev_refine) && slot < 0) ? 1 : 0;
  a.rep = p->rep;
  a.rep_stride = mesh_words(p);
  return a;
}

int grid_for(Pool *p, int slot) {
  if (slot >= 0) return std::max(1, std::min(p->grid, p->slot_items_h[slot].y));
  return p->grid;
}

sic_status launch_tracer_mode(Pool *p, int mode, int slot, hipStream_t st) {
  TracerArgs a = tracer_args(p, mode, slot);
  const size_t lds = tracer_lds_size(p->prec, p->order, p->seg, p->max_cells, p->tile);
  LAUNCHCHK(p, launch_tracers(p->prec, mode, p->order, p->seg, a, grid_for(p, slot), p->block, lds, st));
  return SIC_OK;
}

sic_status launch_solve_mode(Pool *p, int flags, int slot, hipStream_t st) {
  SolveArgs a = solve_args(p, flags, slot);
  LAUNCHCHK(p, launch_solve(p->prec, a, slot >= 0 ? 1 : p->solve_grid, p->max_cells, st));
  return SIC_OK;
}

// One fused step for the whole pool (every live slot; batch pools skip
// finished slots): move + deposit, then solve.
sic_status enqueue_fused(Pool *p, hipStream_t st) {
  sic_status s = launch_tracer_mode(p, kPush | kDeposit, -1, st);
  if (s != SIC_OK) return s;
  int flags = kHavePush | kHaveDeposit | (p->batch ? kBatchStep : 0);
  s = launch_solve_mode(p, flags, -1, st);
  if (s != SIC_OK) return s;
  p->parity ^= 1;
  return SIC_OK;
}

sic_status get_graph(Pool *p, int64_t k, hipGraphExec_t *out) {
  auto key = std::make_tuple(k, p->parity, p->grid, p->solve_grid, p->dev_refine ? 1 : 0);
  auto it = p->graphs.find(key);
  if (it != p->graphs.end()) {
    *out = it->second;
    return SIC_OK;
  }
  const int parity0 = p->parity;
  HIPCHK(p, hipStreamBeginCapture(p->cap, hipStreamCaptureModeRelaxed));
  sic_status s = SIC_OK;
  for (int64_t i = 0; i < k && s == SIC_OK; ++i) s = enqueue_fused(p, p->cap);
  p->parity = parity0;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(p->cap, &g);
  if (s != SIC_OK) {
    if (g) hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return fail(p, SIC_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(g);
    return fail(p, SIC_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  p->graph_objs.push_back(g);
  p->graphs[key] = ex;
  *out = ex;
  return SIC_OK;
}

// Solve-first steps: a single simulation with constant segments (not timed,
// not refining on the device) runs k steps as k tracer launches whose
// second and later ones solve the previous step's charge in every workgroup
// (launch_tracers_sf), then one solve launch for the last step.  The charge
// rotates through three accumulator pairs A0 (the pool's own), A1, A2 and
// the partials through two buffers: launch i (1-based) merges into
// A[(i - 1) mod 3] and writes partials (i - 1) mod 2, reads A[(i - 2) mod 3]
// and partials (i - 2) mod 2, and clears A[i mod 3], which launch i - 1 read
// and launch i + 1 merges into after this one has ended.  The closing solve
// clears what it reads and a zero launch the pair launch k read, so every
// pair is clear again, as the other paths expect.  The bits are those of the
// tracer/solve launch pairs: the same solve code, the same sums in the same
// order.
bool sf_ready(Pool *p) {
  if (p->batch || p->order != 0 || p->timing || p->dev_refine || p->tune.fused_only || p->block < kSolveThreads ||
      p->rep != single_rep(p->max_cells))
    return false;
  // every workgroup solves first: worth it while the workgroups run in one
  // round on the machine, not when each CU works through several in turn
  // (a 33.5M-tracer job's 2048 workgroups: 400 against 290 us per step)
  if (grid_for(p, -1) > kSfMaxGrid) return false;
  if (!p->sf_mesh) {
    const size_t bytes = sizeof(double) * 4 * (size_t)p->rep * mesh_words(p);
    if (hipMalloc(&p->sf_mesh, bytes) != hipSuccess) {
      p->sf_mesh = nullptr;
      return false;
    }
    if (hipMemsetAsync(p->sf_mesh, 0, bytes, p->stream) != hipSuccess) return false;
  }
  if (!p->sf_part) {
    if (hipMalloc((void **)&p->sf_part, sizeof(Partial) * (size_t)p->item_cap) != hipSuccess) {
      p->sf_part = nullptr;
      return false;
    }
  }
  return true;
}

sic_status enqueue_sf(Pool *p, int64_t k, hipStream_t st) {
  // each pair's copies lie mesh_words apart, as the pool's own
  double *m = static_cast<double *>(p->sf_mesh);
  const size_t mc = (size_t)p->rep * mesh_words(p);
  void *AP[3] = {p->meshP, m, m + 2 * mc};
  void *AD[3] = {p->meshD, m + mc, m + 3 * mc};
  Partial *PB[2] = {p->partials, p->sf_part};
  const size_t lds = tracer_lds_size(p->prec, p->order, p->seg, p->max_cells, p->tile);
  for (int64_t i = 1; i <= k; ++i) {
    TracerArgs a = tracer_args(p, kPush | kDeposit, -1);
    a.meshP = AP[(i - 1) % 3];
    a.meshD = AD[(i - 1) % 3];
    a.partials = PB[(i - 1) % 2];
    if (i == 1) {
      LAUNCHCHK(p, launch_tracers(p->prec, kPush | kDeposit, p->order, p->seg, a, grid_for(p, -1), p->block, lds, st));
    } else {
      a.sf_P = AP[(i - 2) % 3];
      a.sf_D = AD[(i - 2) % 3];
      a.sf_zP = AP[i % 3];
      a.sf_zD = AD[i % 3];
      a.sf_partials = PB[(i - 2) % 2];
      a.sf = solve_args(p, kHavePush | kHaveDeposit, -1);
      LAUNCHCHK(p, launch_tracers_sf(p->prec, p->seg, a, grid_for(p, -1), p->block, lds, p->max_cells, st));
    }
    p->parity ^= 1;
  }
  SolveArgs sa = solve_args(p, kHavePush | kHaveDeposit, -1);
  sa.meshP = AP[(k - 1) % 3];
  sa.meshD = AD[(k - 1) % 3];
  sa.partials = PB[(k - 1) % 2];
  LAUNCHCHK(p, launch_solve(p->prec, sa, p->solve_grid, p->max_cells, st));
  if (k >= 2)
    LAUNCHCHK(p, launch_zero_mesh(p->prec, AP[(k - 2) % 3], AD[(k - 2) % 3], nullptr, p->inst, p->slot_ids, 1, p->rep,
                                  mesh_words(p), st));
  return SIC_OK;
}

sic_status get_sf_graph(Pool *p, int64_t k, hipGraphExec_t *out) {
  auto key = std::make_tuple(k, p->parity, p->grid, p->solve_grid, 3);
  auto it = p->graphs.find(key);
  if (it != p->graphs.end()) {
    *out = it->second;
    return SIC_OK;
  }
  const int parity0 = p->parity;
  HIPCHK(p, hipStreamBeginCapture(p->cap, hipStreamCaptureModeRelaxed));
  sic_status s = enqueue_sf(p, k, p->cap);
  p->parity = parity0;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(p->cap, &g);
  if (s != SIC_OK) {
    if (g) hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return fail(p, SIC_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(g);
    return fail(p, SIC_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  p->graph_objs.push_back(g);
  p->graphs[key] = ex;
  *out = ex;
  return SIC_OK;
}

sic_status run_fused(Pool *p, int64_t n) {
  if (n <= 0) return SIC_OK;
  if (p->timing) {
    std::vector<hipEvent_t> ev(3 * (size_t)n);
    for (auto &e : ev) HIPCHK(p, hipEventCreate(&e));
    sic_status s = SIC_OK;
    hipError_t e = hipSuccess;
    for (int64_t i = 0; i < n && s == SIC_OK && e == hipSuccess; ++i) {
      e = hipEventRecord(ev[3 * i], p->stream);
      if (e != hipSuccess) break;
      s = launch_tracer_mode(p, kPush | kDeposit, -1, p->stream);
      if (s != SIC_OK) break;
      e = hipEventRecord(ev[3 * i + 1], p->stream);
      if (e != hipSuccess) break;
      s = launch_solve_mode(p, kHavePush | kHaveDeposit | (p->batch ? kBatchStep : 0), -1, p->stream);
      if (s == SIC_OK) e = hipEventRecord(ev[3 * i + 2], p->stream);
      p->parity ^= 1;
    }
    const hipError_t es = hipStreamSynchronize(p->stream);
    if (e == hipSuccess) e = es;
    double tt = 0.0, ts = 0.0;
    for (int64_t i = 0; i < n && e == hipSuccess && s == SIC_OK; ++i) {
      float a = 0.f, b = 0.f;
      e = hipEventElapsedTime(&a, ev[3 * i], ev[3 * i + 1]);
      if (e == hipSuccess) e = hipEventElapsedTime(&b, ev[3 * i + 1], ev[3 * i + 2]);
      tt += a;
      ts += b;
    }
    for (auto &x : ev) hipEventDestroy(x);
    if (s != SIC_OK) return s;
    if (e != hipSuccess) return fail(p, SIC_EDEVICE, std::string("timed step: ") + hipGetErrorString(e));
    p->t_tracer = tt / (double)n;
    p->t_solve = ts / (double)n;
    return SIC_OK;
  }
  const bool sf = sf_ready(p);
  while (n > 0) {
    const int64_t k = std::min<int64_t>(n, kGraphSteps);
    hipGraphExec_t ex;
    sic_status s = sf ? get_sf_graph(p, k, &ex) : get_graph(p, k, &ex);
    if (s != SIC_OK) return s;
    HIPCHK(p, hipGraphLaunch(ex, p->stream));
    if (k & 1) p->parity ^= 1;
    n -= k;
  }
  return SIC_OK;
}

// A small simulation: all its steps in launches of one resident workgroup
// (at most kResidentSteps steps each, to keep launches short).
constexpr int64_t kResidentSteps = 8192;

sic_status run_resident(Pool *p, int64_t n) {
  const SlotHost &sh = p->slots[0];
  while (n > 0) {
    const int64_t k = std::min<int64_t>(n, kResidentSteps);
    TracerArgs a = tracer_args(p, kPush | kDeposit, 0);
    a.halo_out = p->halo[p->parity ^ (int)(k & 1)];
    SolveArgs sa = solve_args(p, kHavePush | kHaveDeposit, 0);
    LAUNCHCHK(p, launch_resident(p->prec, p->seg, a, sa, sh.chunk_begin, sh.n_chunks, sh.n_cells, k, p->stream));
    if (k & 1) p->parity ^= 1;
    n -= k;
  }
  return SIC_OK;
}

bool finite(double x) { return std::isfinite(x); }

sic_status validate(Pool *p, const sic_config *cfg, const sic_sheet *sheets, int32_t n_sheets, const double *x0,
                    const double *v0) {
  if (!cfg || !sheets || !x0 || !v0) return fail(p, SIC_EINVAL, "null argument");
  if (cfg->abi_version != SIC_ABI_VERSION) return fail(p, SIC_EINVAL, "abi_version mismatch");
  if (cfg->n_cells < 1 || cfg->n_cells > SIC_MAX_CELLS) return fail(p, SIC_EINVAL, "n_cells out of range");
  if (!(cfg->L > 0.0) || !finite(cfg->L)) return fail(p, SIC_EINVAL, "L must be positive and finite");
  if (!(cfg->dt > 0.0) || !finite(cfg->dt)) return fail(p, SIC_EINVAL, "dt must be positive and finite");
  if (cfg->precision < 0 || cfg->precision > 2) return fail(p, SIC_EINVAL, "unknown precision");
  if (cfg->deposit_order < 0 || cfg->deposit_order > 2)
    return fail(p, SIC_ENOTSUP, "deposit_order must be 0 (constant), 1 (linear segments) or 2 (first-order weighting)");
  if (cfg->history_rows < 0) return fail(p, SIC_EINVAL, "history_rows < 0");
  if (!(cfg->l_max >= 0.0) || !finite(cfg->l_max)) return fail(p, SIC_EINVAL, "l_max must be >= 0 and finite");
  if (cfg->max_tracers < 0) return fail(p, SIC_EINVAL, "max_tracers < 0");
  if (n_sheets < 1) return fail(p, SIC_EINVAL, "need at least one sheet");
  for (int32_t s = 0; s < n_sheets; ++s) {
    if (sheets[s].n_tracers < 2) return fail(p, SIC_EINVAL, "every sheet needs at least 2 tracers");
    if (sheets[s].closed != 0 && sheets[s].closed != 1) return fail(p, SIC_EINVAL, "closed must be 0 or 1");
    if (!finite(sheets[s].q_seg)) return fail(p, SIC_EINVAL, "non-finite segment charge");
  }
  return SIC_OK;
}

bool all_finite_host(const double *a, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

// Chunk layout of one slot's sheets from chunk cb on: descriptors, input
// offsets, piecewise-linear links and the slot of the tracer before each
// chunk (charge edges).
struct Layout {
  std::vector<ChunkDesc> cd;
  std::vector<int64_t> in_off;
  std::vector<int2> links;
  std::vector<int64_t> prev;
};

int64_t chunks_for(const std::vector<int32_t> &nt) {
  int64_t n = 0;
  for (int32_t t : nt) n += (t + kChunk - 1) / kChunk;
  return n;
}

void build_layout(int32_t slot, int64_t cb, const std::vector<int32_t> &nt, const std::vector<int32_t> &closed,
                  const std::vector<double> &q, double q_scale, bool fixed, Layout *L) {
  const int64_t n_ch = chunks_for(nt);
  L->cd.assign((size_t)n_ch, ChunkDesc{});
  L->in_off.assign((size_t)n_ch, 0);
  L->links.assign((size_t)n_ch, make_int2(-1, -1));
  L->prev.assign((size_t)n_ch, -1);
  int64_t c = 0, in = 0;
  for (size_t s = 0; s < nt.size(); ++s) {
    const int32_t n = nt[s];
    const int32_t nch = (n + kChunk - 1) / kChunk;
    const int64_t first = cb + c;
    const bool cl = closed[s] != 0;
    for (int32_t k = 0; k < nch; ++k) {
      ChunkDesc &d = L->cd[(size_t)(c + k)];
      d.q = q[s];
      d.q_fix = fixed ? (int64_t)std::llrint(q[s] * q_scale) : 0;
      d.n_valid = std::min(kChunk, n - k * kChunk);
      d.inst = slot;
      d.flags = (k == 0 && !cl) ? kChunkOpenStart : 0;
      if (k + 1 < nch) d.partner = (int32_t)(first + k + 1);
      else d.partner = cl ? (int32_t)first : -1;
      L->in_off[(size_t)(c + k)] = in + (int64_t)k * kChunk;
      // the tracer before this chunk's first: the previous chunk's last, or
      // for a closed sheet's first chunk the sheet's last tracer
      if (k > 0) L->prev[(size_t)(c + k)] = (first + k - 1) * kChunk + (kChunk - 1);
      else if (cl) L->prev[(size_t)(c + k)] = (first + nch - 1) * kChunk + (n - (nch - 1) * kChunk - 1);
    }
    // Links to the tracer before each chunk and the one two past its end
    // (piecewise-linear segments); a closed sheet of fewer than 3 tracers has
    // no gradient, so it gets no links.
    const bool grad = !cl || n >= 3;
    for (int32_t k = 0; k < nch && grad; ++k) {
      int2 &lk = L->links[(size_t)(c + k)];
      if (k > 0) lk.x = (int32_t)(((first + k - 1) << 2) | kHaloLast);
      else if (cl) lk.x = (int32_t)(((first + nch - 1) << 2) | kHaloLast);
      const int32_t P = L->cd[(size_t)(c + k)].partner;
      if (P >= 0) {
        const int64_t pk = P - first;
        if (L->cd[(size_t)(c + pk)].n_valid >= 2) lk.y = (P << 2) | kHaloSecond;
        else {
          const int32_t PP = L->cd[(size_t)(c + pk)].partner;
          if (PP >= 0) lk.y = (PP << 2) | kHaloFirst;
        }
      }
    }
    c += nch;
    in += n;
  }
}

// Uploads a layout for chunks [cb, cb + n) of a slot (ordered on the stream).
hipError_t upload_layout(Pool *p, SlotHost &sh, int64_t cb, const Layout &L) {
  const size_t n = L.cd.size();
  hipError_t e = hipSuccess;
  if (sh.d_in_off) hipFree(sh.d_in_off);
  sh.d_in_off = nullptr;
  e = hipMalloc((void **)&sh.d_in_off, sizeof(int64_t) * std::max<size_t>(n, 1));
  if (e != hipSuccess) {
    sh.d_in_off = nullptr;
    return e;
  }
  e = hipMemcpyAsync(p->chunks + cb, L.cd.data(), sizeof(ChunkDesc) * n, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sh.d_in_off, L.in_off.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->links + cb, L.links.data(), sizeof(int2) * n, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess && p->seg)
    e = hipMemcpyAsync(p->edge_prev + cb, L.prev.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, p->stream);
  return e;
}

// Places a slot's tracers from flat sheet-major inputs: float64 positions or
// raw state words, velocities, and per-segment charges (float64, raw words,
// or none: the sheet charges); then the charge edges.  keep_charges leaves
// the charge words as they are (same layout, new positions).
int ingest_slot(Pool *p, int32_t slot, const double *x, const uint64_t *w, const double *v, const double *c,
                const uint64_t *cw, bool keep_charges = false) {
  SlotHost &sh = p->slots[slot];
  IngestArgs ia;
  ia.x_in = x;
  ia.w_in = w;
  ia.v_in = v;
  ia.c_in = c;
  ia.cw_in = cw;
  ia.segq = keep_charges ? nullptr : p->segq;
  ia.q_scale = sh.q_scale;
  ia.chunk_in_off = sh.d_in_off;
  ia.chunk_begin = sh.chunk_begin;
  ia.n_chunks = sh.n_chunks;
  ia.chunks = p->chunks;
  ia.inst = p->inst;
  ia.xs = p->xs;
  ia.vs = p->vs;
  ia.halo = p->halo[p->parity];
  ia.halo3 = p->halo3[p->parity];
  int le = launch_ingest(p->prec, ia, p->stream);
  if (le == 0 && p->seg && !keep_charges)
    le = launch_charge_edges(p->chunks, p->edge_prev, p->segq, p->cedge, sh.chunk_begin, sh.n_chunks, p->stream);
  return le;
}

// Sum of |charge| over the segments (fixed-point scale of the split forms).
double total_abs_charge(const sic_sheet *sheets, int32_t n_sheets, const double *c_host) {
  double total = 0.0;
  int64_t base = 0;
  for (int32_t s = 0; s < n_sheets; ++s) {
    const int32_t nt = sheets[s].n_tracers;
    const int32_t nseg = sheets[s].closed ? nt : nt - 1;
    if (c_host) {
      for (int32_t t = 0; t < nseg; ++t) total += std::fabs(c_host[base + t]);
    } else {
      total += std::fabs(sheets[s].q_seg) * (double)nseg;
    }
    base += nt;
  }
  return total;
}

// Admits one simulation into a free slot and ingests it (see sic_init).
sic_status pool_admit(Pool *p, const sic_config *cfg, const sic_sheet *sheets, int32_t n_sheets, const double *x0,
                      const double *v0, const double *c0, int32_t mem_kind, int64_t n_steps, int32_t *slot_out) {
  sic_status st = validate(p, cfg, sheets, n_sheets, x0, v0);
  if (st != SIC_OK) return st;
  if (cfg->precision != p->prec) return fail(p, SIC_EINVAL, "precision differs from the batch precision");
  if (cfg->deposit_order != p->order) return fail(p, SIC_EINVAL, "deposit_order differs from the batch's");
  if (cfg->n_cells > p->max_cells) return fail(p, SIC_EINVAL, "n_cells above the batch max_cells");
  if (mem_kind != SIC_MEM_HOST && mem_kind != SIC_MEM_DEVICE) return fail(p, SIC_EINVAL, "bad mem_kind");
  if (c0 && !p->seg) return fail(p, SIC_ENOTSUP, "per-segment charges need a batch created for them");
  if (cfg->l_max != 0.0 && !p->seg)
    return fail(p, SIC_ENOTSUP, "refinement in a batch needs SIC_BATCH_SEGMENT_CHARGES");

  int64_t n_tr = 0;
  std::vector<int32_t> nt((size_t)n_sheets), closed((size_t)n_sheets);
  std::vector<double> q((size_t)n_sheets);
  for (int32_t s = 0; s < n_sheets; ++s) {
    nt[(size_t)s] = sheets[s].n_tracers;
    closed[(size_t)s] = sheets[s].closed;
    q[(size_t)s] = sheets[s].q_seg;
    n_tr += sheets[s].n_tracers;
  }
  const int64_t n_ch = chunks_for(nt);
  if (mem_kind == SIC_MEM_HOST && (!all_finite_host(x0, n_tr) || !all_finite_host(v0, n_tr)))
    return fail(p, SIC_EINVAL, "non-finite initial position or velocity");
  // per-segment charges on the host (finiteness, fixed-point scale)
  std::vector<double> c_host;
  if (c0) {
    if (mem_kind == SIC_MEM_HOST) {
      c_host.assign(c0, c0 + n_tr);
    } else {
      c_host.resize((size_t)n_tr);
      HIPCHK(p, hipStreamSynchronize(p->stream));
      HIPCHK(p, hipMemcpy(c_host.data(), c0, sizeof(double) * (size_t)n_tr, hipMemcpyDeviceToHost));
    }
    if (!all_finite_host(c_host.data(), n_tr)) return fail(p, SIC_EINVAL, "non-finite segment charge");
  }
  int32_t slot = -1;
  for (int32_t i = 0; i < p->slot_cap; ++i)
    if (!p->slots[i].live) {
      slot = i;
      break;
    }
  if (slot < 0) return fail(p, SIC_EBUSY, "no free slot");
  // A slot reserves room for max_tracers (refinement grows it in place): the
  // reservation counts against the budget and its chunks are allocated now.
  const int64_t reserve_tr = std::max<int64_t>(cfg->max_tracers, n_tr);
  const int64_t n_res = reserve_tr > n_tr ? std::max<int64_t>(n_ch, (reserve_tr + kChunk - 1) / kChunk + n_sheets)
                                          : n_ch;
  if (p->budget > 0 && p->used_tracers + reserve_tr > p->budget)
    return fail(p, SIC_EBUSY, "over the tracer budget");
  const int64_t cb = p->alloc.alloc(n_res);
  if (cb < 0) return fail(p, SIC_EBUSY, "tracer arena full");

  const double total_abs = total_abs_charge(sheets, n_sheets, c0 ? c_host.data() : nullptr);
  double q_unit = 1.0, q_scale = 1.0;
  if (p->prec != kFP64) {
    // fixed point: total |charge| just under 2^62 units
    int ex = 0;
    std::frexp(total_abs > 0.0 ? total_abs : 1.0, &ex);  // total_abs < 2^ex
    const int S = 62 - ex;
    q_scale = std::ldexp(1.0, S);
    q_unit = std::ldexp(1.0, -S);
  }
  SlotHost &sh = p->slots[slot];
  Layout L;
  build_layout(slot, cb, nt, closed, q, q_scale, p->prec != kFP64, &L);
  sh.chunk_in_off = L.in_off;
  sh.live = true;
  sh.n_cells = cfg->n_cells;
  sh.L = cfg->L;
  sh.dt = cfg->dt;
  sh.n_tracers = n_tr;
  sh.n_tracers_s = nt;
  sh.closed_s = closed;
  sh.q_s = q;
  sh.q_scale = q_scale;
  sh.l_max = cfg->l_max;
  sh.max_tracers = reserve_tr;
  sh.hist_from = 0;
  sh.chunk_begin = (int32_t)cb;
  sh.n_chunks = (int32_t)n_ch;
  sh.n_chunks_res = (int32_t)n_res;
  sh.state = kStale;
  sh.pending_push = sh.pending_dep = false;
  sh.reported = false;

  InstDesc I;
  std::memset(&I, 0, sizeof(I));
  I.L = cfg->L;
  I.half_L = 0.5 * cfg->L;
  I.dx = cfg->L / cfg->n_cells;
  I.inv_dx = (double)cfg->n_cells / cfg->L;
  I.dt = cfg->dt;
  I.q_unit = q_unit;
  I.mesh_off = (int64_t)slot * p->max_cells;
  I.hist_off = (int64_t)slot * p->hist_rows;
  I.hist_cap = p->hist_rows;
  I.step = 0;
  I.steps_left = p->batch ? n_steps : -1;
  I.n_cells = cfg->n_cells;
  I.active = (p->batch && n_steps == 0) ? 0 : 1;
  I.flags = 0;
  I.live = 1;

  auto undo = [&]() {
    if (sh.n_items > 0) clear_slot_items(p, slot);
    p->alloc.release(cb, n_res);
    sh.live = false;
    sh.chunk_in_off.clear();
  };
  st = place_slot_items(p, slot);
  if (st != SIC_OK) {
    undo();
    return st;
  }
  double *stage = nullptr;
  const double *dx0 = x0, *dv0 = v0, *dc0 = c0;
  hipError_t e = hipSuccess;
  if (mem_kind == SIC_MEM_HOST) {
    e = hipMalloc((void **)&stage, sizeof(double) * (c0 ? 3 : 2) * (size_t)std::max<int64_t>(n_tr, 1));
    if (e != hipSuccess) {
      undo();
      return fail(p, SIC_ENOMEM, "hipMalloc staging");
    }
    e = hipMemcpyAsync(stage, x0, sizeof(double) * (size_t)n_tr, hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(stage + n_tr, v0, sizeof(double) * (size_t)n_tr, hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess && c0)
      e = hipMemcpyAsync(stage + 2 * n_tr, c0, sizeof(double) * (size_t)n_tr, hipMemcpyHostToDevice, p->stream);
    dx0 = stage;
    dv0 = stage + n_tr;
    dc0 = c0 ? stage + 2 * n_tr : nullptr;
  }
  const int32_t zero = 0;
  if (e == hipSuccess) e = upload_layout(p, sh, cb, L);
  if (e == hipSuccess) e = hipMemcpyAsync(p->inst + slot, &I, sizeof(I), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(p->done + slot, &zero, sizeof(zero), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) {
    if (stage) hipFree(stage);
    undo();
    return fail(p, SIC_EDEVICE, std::string("admission copies: ") + hipGetErrorString(e));
  }
  p->used_tracers += reserve_tr;
  p->used_slots += 1;
  update_solve_grid(p);
  // ingest: place tracers, deposit, solve, half back-kick
  int le = ingest_slot(p, slot, dx0, nullptr, dv0, dc0, nullptr);
  if (le == 0) le = launch_zero_mesh(p->prec, p->meshP, p->meshD, p->meshR, p->inst, p->slot_ids + slot, 1, p->rep,
                                         mesh_words(p), p->stream);
  if (le != 0) {
    if (stage) hipFree(stage);
    return fail(p, SIC_EDEVICE, std::string("ingest: ") + hipGetErrorString((hipError_t)le));
  }
  st = launch_tracer_mode(p, kDeposit, slot, p->stream);
  if (st == SIC_OK) st = launch_solve_mode(p, kHaveDeposit, slot, p->stream);
  if (st == SIC_OK) st = launch_tracer_mode(p, kKickHalf, slot, p->stream);
  e = hipStreamSynchronize(p->stream);
  if (stage) hipFree(stage);
  if (st != SIC_OK) return st;
  if (e != hipSuccess) return fail(p, SIC_EDEVICE, std::string("ingest: ") + hipGetErrorString(e));
  sh.state = kField;
  *slot_out = slot;
  return SIC_OK;
}

// Replaces a slot's tracers with a new layout inside its reserved chunk range
// (refinement, sic_load_state): nt[s] tracers per sheet from flat device inputs (float64
// positions or raw state words; velocities; float64 charges, raw charge words
// or none).  step >= 0 sets the step.  With redeposit the new state is
// deposited and solved at once (the newest diagnostics row is rewritten);
// otherwise the field becomes stale.  Synchronous.
sic_status pool_relayout(Pool *p, int32_t slot, const std::vector<int32_t> &nt, const double *x, const uint64_t *w,
                         const double *v, const double *c, const uint64_t *cw, int64_t step, bool redeposit) {
  SlotHost &sh = p->slots[slot];
  int64_t n_tr = 0;
  for (int32_t t : nt) n_tr += t;
  const int64_t n_ch = chunks_for(nt);
  if (n_ch > sh.n_chunks_res || n_tr > sh.max_tracers)
    return fail(p, SIC_ENOMEM, "refined or loaded state exceeds the tracer capacity");
  HIPCHK(p, hipStreamSynchronize(p->stream));
  const int tile0 = p->tile, grid0 = p->grid;
  sic_status st = clear_slot_items(p, slot);
  if (st != SIC_OK) return st;
  const int64_t cb = sh.chunk_begin;  // the new layout stays inside the reservation
  Layout L;
  build_layout(slot, cb, nt, sh.closed_s, sh.q_s, sh.q_scale, p->prec != kFP64, &L);
  sh.n_tracers = n_tr;
  sh.n_tracers_s = nt;
  sh.chunk_in_off = L.in_off;
  sh.n_chunks = (int32_t)n_ch;
  st = place_slot_items(p, slot);
  if (st != SIC_OK) return st;
  // captured graphs carry the tile (LDS size) and grid of their capture
  if (p->tile != tile0 || p->grid != grid0) destroy_graphs(p);
  hipError_t e = upload_layout(p, sh, cb, L);
  if (e == hipSuccess && step >= 0) {
    InstDesc I;
    e = hipMemcpyAsync(&I, p->inst + slot, sizeof(I), hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    I.step = step;
    if (e == hipSuccess) e = hipMemcpyAsync(p->inst + slot, &I, sizeof(I), hipMemcpyHostToDevice, p->stream);
  }
  if (e != hipSuccess) return fail(p, SIC_EDEVICE, std::string("re-layout copies: ") + hipGetErrorString(e));
  int le = ingest_slot(p, slot, x, w, v, c, cw);
  if (le == 0) le = launch_zero_mesh(p->prec, p->meshP, p->meshD, p->meshR, p->inst, p->slot_ids + slot, 1, p->rep,
                                         mesh_words(p), p->stream);
  if (le != 0) return fail(p, SIC_EDEVICE, std::string("re-layout ingest: ") + hipGetErrorString((hipError_t)le));
  sh.pending_push = sh.pending_dep = false;
  if (redeposit) {
    st = launch_tracer_mode(p, kDeposit, slot, p->stream);
    if (st == SIC_OK) st = launch_solve_mode(p, kHaveDeposit, slot, p->stream);
    if (st != SIC_OK) return st;
    sh.state = kField;
  } else {
    sh.state = kStale;
  }
  HIPCHK(p, hipStreamSynchronize(p->stream));
  return SIC_OK;
}

sic_status ensure_refine_scratch(Pool *p, int64_t stage_tracers) {
  if (!p->ref_cnt) {
    HIPCHK(p, dalloc(&p->ref_cnt, (size_t)p->chunk_cap));
    HIPCHK(p, dalloc(&p->ref_mask, (size_t)p->chunk_cap));
    HIPCHK(p, dalloc(&p->ref_off, (size_t)p->chunk_cap));
  }
  if (stage_tracers > p->ref_stage_cap) {
    if (p->ref_w) hipFree(p->ref_w);
    if (p->ref_v) hipFree(p->ref_v);
    if (p->ref_c) hipFree(p->ref_c);
    p->ref_w = nullptr;
    p->ref_v = nullptr;
    p->ref_c = nullptr;
    p->ref_stage_cap = 0;
    HIPCHK(p, dalloc(&p->ref_w, (size_t)stage_tracers));
    HIPCHK(p, dalloc(&p->ref_v, (size_t)stage_tracers));
    HIPCHK(p, dalloc(&p->ref_c, (size_t)stage_tracers));
    p->ref_stage_cap = stage_tracers;
  }
  return SIC_OK;
}

// One refinement pass over a single simulation (section 2.6).
sic_status pool_refine(Pool *p, int32_t slot, double l_max, int64_t *inserted) {
  if (inserted) *inserted = 0;
  if (!p->seg) return fail(p, SIC_ENOTSUP, "refinement needs per-segment charges (or l_max at creation)");
  if (!(l_max > 0.0) || !std::isfinite(l_max)) return fail(p, SIC_EINVAL, "l_max must be positive and finite");
  SlotHost &sh = p->slots[slot];
  if (sh.state != kField) return fail(p, SIC_ESTATE, "refinement needs the field of the current step");
  sic_status st = ensure_refine_scratch(p, 0);
  if (st != SIC_OK) return st;
  RefineArgs ra;
  ra.chunks = p->chunks;
  ra.inst = p->inst;
  ra.xs = p->xs;
  ra.vs = p->vs;
  ra.segq = p->segq;
  ra.chunk_begin = sh.chunk_begin;
  ra.n_chunks = sh.n_chunks;
  ra.l_max = l_max;
  ra.cnt = p->ref_cnt;
  ra.mask = p->ref_mask;
  ra.out_off = p->ref_off;
  ra.w_out = nullptr;
  ra.v_out = nullptr;
  ra.c_out = nullptr;
  LAUNCHCHK(p, launch_refine_mark(p->prec, ra, p->stream));
  std::vector<int32_t> cnt((size_t)sh.n_chunks);
  HIPCHK(p, hipStreamSynchronize(p->stream));
  HIPCHK(p, hipMemcpy(cnt.data(), p->ref_cnt, sizeof(int32_t) * cnt.size(), hipMemcpyDeviceToHost));
  // new sheet sizes and the output offset of every chunk
  std::vector<int32_t> nt = sh.n_tracers_s;
  std::vector<int64_t> off((size_t)sh.n_chunks);
  int64_t add = 0, out = 0;
  {
    int64_t c = 0;
    for (size_t s = 0; s < nt.size(); ++s) {
      const int32_t nch = (sh.n_tracers_s[s] + kChunk - 1) / kChunk;
      int64_t sheet_add = 0;
      for (int32_t k = 0; k < nch; ++k) {
        off[(size_t)(c + k)] = out;
        const int32_t nv = std::min(kChunk, sh.n_tracers_s[s] - k * kChunk);
        out += nv + cnt[(size_t)(c + k)];
        sheet_add += cnt[(size_t)(c + k)];
      }
      if ((int64_t)nt[s] + sheet_add > (int64_t)INT32_MAX) return fail(p, SIC_ENOMEM, "sheet too long");
      nt[s] += (int32_t)sheet_add;
      add += sheet_add;
      c += nch;
    }
  }
  if (add == 0) return SIC_OK;
  const int64_t n_new = sh.n_tracers + add;
  if (n_new > sh.max_tracers || chunks_for(nt) > sh.n_chunks_res)
    return fail(p, SIC_ENOMEM, "refinement exceeds the tracer capacity");
  st = ensure_refine_scratch(p, n_new);
  if (st != SIC_OK) return st;
  HIPCHK(p, hipMemcpyAsync(p->ref_off, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice, p->stream));
  ra.w_out = p->ref_w;
  ra.v_out = p->ref_v;
  ra.c_out = p->ref_c;
  LAUNCHCHK(p, launch_refine_scatter(p->prec, ra, p->stream));
  st = pool_relayout(p, slot, nt, nullptr, p->ref_w, p->ref_v, nullptr, p->ref_c, -1, true);
  if (st != SIC_OK) return st;
  if (inserted) *inserted = add;
  return SIC_OK;
}

sic_status pool_release(Pool *p, int32_t slot) {
  if (slot < 0 || slot >= p->slot_cap || !p->slots[slot].live) return fail(p, SIC_EINVAL, "slot not live");
  SlotHost &sh = p->slots[slot];
  InstDesc I;
  std::memset(&I, 0, sizeof(I));
  HIPCHK(p, hipMemcpyAsync(p->inst + slot, &I, sizeof(I), hipMemcpyHostToDevice, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  sic_status st = clear_slot_items(p, slot);
  if (st != SIC_OK) return st;
  p->alloc.release(sh.chunk_begin, sh.n_chunks_res);
  p->used_tracers -= sh.max_tracers;
  p->used_slots -= 1;
  sh.live = false;
  update_solve_grid(p);
  sh.chunk_in_off.clear();
  if (sh.d_in_off) {
    hipFree(sh.d_in_off);
    sh.d_in_off = nullptr;
  }
  return SIC_OK;
}

sic_status read_inst(Pool *p, int32_t slot, InstDesc *I) {
  HIPCHK(p, hipStreamSynchronize(p->stream));
  HIPCHK(p, hipMemcpy(I, p->inst + slot, sizeof(InstDesc), hipMemcpyDeviceToHost));
  return SIC_OK;
}

sic_status pool_diagnostics(Pool *p, int32_t slot, sic_diag *out, double *rho_out, double *E_out,
                            sic_diag *history_out, int64_t *history_len) {
  if (slot < 0 || slot >= p->slot_cap || !p->slots[slot].live) return fail(p, SIC_EINVAL, "slot not live");
  InstDesc I;
  sic_status st = read_inst(p, slot, &I);
  if (st != SIC_OK) return st;
  const int64_t step = I.step;
  const int64_t cap = I.hist_cap;
  const int64_t avail = std::min<int64_t>(step + 1 - std::min(step, p->slots[slot].hist_from), cap);
  const DiagRow *H = p->hist + I.hist_off;
  if (out) {
    DiagRow r;
    HIPCHK(p, hipMemcpy(&r, H + step % cap, sizeof(r), hipMemcpyDeviceToHost));
    static_assert(sizeof(DiagRow) == sizeof(sic_diag), "row layout");
    std::memcpy(out, &r, sizeof(r));
  }
  const int nc = p->slots[slot].n_cells;
  if (rho_out) HIPCHK(p, hipMemcpy(rho_out, p->meshRho + I.mesh_off, sizeof(double) * nc, hipMemcpyDeviceToHost));
  if (E_out) HIPCHK(p, hipMemcpy(E_out, p->meshE + I.mesh_off, sizeof(double) * nc, hipMemcpyDeviceToHost));
  if (history_len) {
    if (history_out) {
      const int64_t want = std::min<int64_t>(*history_len, avail);
      // the newest `want` rows, oldest first
      std::vector<DiagRow> all((size_t)avail);
      const int64_t first = step + 1 - avail;
      const int64_t r0 = first % cap;
      const int64_t n1 = std::min<int64_t>(avail, cap - r0);
      HIPCHK(p, hipMemcpy(all.data(), H + r0, sizeof(DiagRow) * (size_t)n1, hipMemcpyDeviceToHost));
      if (n1 < avail)
        HIPCHK(p, hipMemcpy(all.data() + n1, H, sizeof(DiagRow) * (size_t)(avail - n1), hipMemcpyDeviceToHost));
      std::memcpy(history_out, all.data() + (avail - want), sizeof(DiagRow) * (size_t)want);
      *history_len = want;
    } else {
      *history_len = avail;
    }
  }
  return SIC_OK;
}

sic_status pool_get_state(Pool *p, int32_t slot, double *x, double *v, int64_t *step, int32_t mem_kind) {
  if (slot < 0 || slot >= p->slot_cap || !p->slots[slot].live) return fail(p, SIC_EINVAL, "slot not live");
  SlotHost &sh = p->slots[slot];
  double *dx = x, *dv = v, *stage = nullptr;
  if (mem_kind == SIC_MEM_HOST) {
    HIPCHK(p, hipMalloc((void **)&stage, sizeof(double) * 2 * (size_t)std::max<int64_t>(sh.n_tracers, 1)));
    dx = stage;
    dv = stage + sh.n_tracers;
  }
  ExtractArgs ea;
  ea.chunk_in_off = sh.d_in_off;
  ea.chunk_begin = sh.chunk_begin;
  ea.n_chunks = sh.n_chunks;
  ea.chunks = p->chunks;
  ea.inst = p->inst;
  ea.xs = p->xs;
  ea.vs = p->vs;
  ea.segq = p->segq;
  ea.x_out = dx;
  ea.v_out = dv;
  ea.c_out = nullptr;
  int le = launch_extract(p->prec, ea, p->stream);
  hipError_t e = hipStreamSynchronize(p->stream);
  if (le == 0 && e == hipSuccess && stage && x)
    e = hipMemcpy(x, dx, sizeof(double) * (size_t)sh.n_tracers, hipMemcpyDeviceToHost);
  if (le == 0 && e == hipSuccess && stage && v)
    e = hipMemcpy(v, dv, sizeof(double) * (size_t)sh.n_tracers, hipMemcpyDeviceToHost);
  if (stage) hipFree(stage);
  if (le != 0) return fail(p, SIC_EDEVICE, std::string("extract: ") + hipGetErrorString((hipError_t)le));
  if (e != hipSuccess) return fail(p, SIC_EDEVICE, std::string("get_state: ") + hipGetErrorString(e));
  if (step) {
    InstDesc I;
    sic_status st = read_inst(p, slot, &I);
    if (st != SIC_OK) return st;
    *step = I.step;
  }
  return SIC_OK;
}

sic_status pool_get_charges(Pool *p, int32_t slot, double *c, int32_t mem_kind) {
  if (slot < 0 || slot >= p->slot_cap || !p->slots[slot].live) return fail(p, SIC_EINVAL, "slot not live");
  if (!c || (mem_kind != SIC_MEM_HOST && mem_kind != SIC_MEM_DEVICE)) return fail(p, SIC_EINVAL, "bad arguments");
  SlotHost &sh = p->slots[slot];
  const size_t n = (size_t)sh.n_tracers;
  if (!p->seg) {
    // every segment carries its sheet's charge
    std::vector<double> h(n);
    size_t b = 0;
    for (size_t s = 0; s < sh.n_tracers_s.size(); ++s) {
      const size_t nt = (size_t)sh.n_tracers_s[s];
      for (size_t t = 0; t < nt; ++t) h[b + t] = sh.q_s[s];
      if (!sh.closed_s[s]) h[b + nt - 1] = 0.0;
      b += nt;
    }
    if (mem_kind == SIC_MEM_HOST) std::memcpy(c, h.data(), sizeof(double) * n);
    else HIPCHK(p, hipMemcpy(c, h.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    return SIC_OK;
  }
  double *stage = nullptr;
  HIPCHK(p, hipMalloc((void **)&stage, sizeof(double) * 3 * std::max<size_t>(n, 1)));
  ExtractArgs ea;
  ea.chunk_in_off = sh.d_in_off;
  ea.chunk_begin = sh.chunk_begin;
  ea.n_chunks = sh.n_chunks;
  ea.chunks = p->chunks;
  ea.inst = p->inst;
  ea.xs = p->xs;
  ea.vs = p->vs;
  ea.segq = p->segq;
  ea.x_out = stage;
  ea.v_out = stage + n;
  ea.c_out = stage + 2 * n;
  int le = launch_extract(p->prec, ea, p->stream);
  hipError_t e = hipStreamSynchronize(p->stream);
  if (le == 0 && e == hipSuccess)
    e = hipMemcpy(c, stage + 2 * n, sizeof(double) * n,
                  mem_kind == SIC_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice);
  hipFree(stage);
  if (le != 0) return fail(p, SIC_EDEVICE, std::string("extract: ") + hipGetErrorString((hipError_t)le));
  if (e != hipSuccess) return fail(p, SIC_EDEVICE, std::string("get_charges: ") + hipGetErrorString(e));
  return SIC_OK;
}

// sic_load_state: a new layout for a single simulation.
sic_status pool_load_state(Pool *p, int64_t step, const int32_t *n_tracers, const double *x, const double *v,
                           const double *c, int32_t mem_kind) {
  SlotHost &sh = p->slots[0];
  if (!n_tracers || !x || !v || step < 0) return fail(p, SIC_EINVAL, "bad state arguments");
  if (mem_kind != SIC_MEM_HOST && mem_kind != SIC_MEM_DEVICE) return fail(p, SIC_EINVAL, "bad mem_kind");
  if (c && !p->seg)
    return fail(p, SIC_ENOTSUP, "per-segment charges need a simulation created with them (or with refinement)");
  std::vector<int32_t> nt(sh.n_tracers_s.size());
  int64_t n = 0;
  for (size_t s = 0; s < nt.size(); ++s) {
    nt[s] = n_tracers[s];
    if (nt[s] < 2) return fail(p, SIC_EINVAL, "every sheet needs at least 2 tracers");
    n += nt[s];
  }
  if (n > sh.max_tracers || chunks_for(nt) > sh.n_chunks_res)
    return fail(p, SIC_ENOMEM, "state exceeds the tracer capacity");
  if (mem_kind == SIC_MEM_HOST &&
      (!all_finite_host(x, n) || !all_finite_host(v, n) || (c && !all_finite_host(c, n))))
    return fail(p, SIC_EINVAL, "non-finite state");
  double *stage = nullptr;
  const double *dx = x, *dv = v, *dc = c;
  if (mem_kind == SIC_MEM_HOST) {
    HIPCHK(p, hipMalloc((void **)&stage, sizeof(double) * 3 * (size_t)std::max<int64_t>(n, 1)));
    hipError_t e = hipMemcpy(stage, x, sizeof(double) * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(stage + n, v, sizeof(double) * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess && c) e = hipMemcpy(stage + 2 * n, c, sizeof(double) * (size_t)n, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      hipFree(stage);
      return fail(p, SIC_EDEVICE, std::string("load_state copies: ") + hipGetErrorString(e));
    }
    dx = stage;
    dv = stage + n;
    dc = c ? stage + 2 * n : nullptr;
  }
  sic_status st = pool_relayout(p, 0, nt, dx, nullptr, dv, dc, nullptr, step, false);
  if (stage) hipFree(stage);
  if (st == SIC_OK) sh.hist_from = step;
  return st;
}

// fixed_stage: device memory of at least 2 n_tracers doubles for staging host
// inputs (the no-allocation entry point's array); nullptr: allocated here.
sic_status pool_set_state(Pool *p, int32_t slot, int64_t step, const double *x, const double *v,
                          int32_t mem_kind, double *fixed_stage = nullptr) {
  if (slot < 0 || slot >= p->slot_cap || !p->slots[slot].live) return fail(p, SIC_EINVAL, "slot not live");
  if (!x || !v || step < 0) return fail(p, SIC_EINVAL, "bad state arguments");
  SlotHost &sh = p->slots[slot];
  if (mem_kind == SIC_MEM_HOST && (!all_finite_host(x, sh.n_tracers) || !all_finite_host(v, sh.n_tracers)))
    return fail(p, SIC_EINVAL, "non-finite state");
  InstDesc I;
  sic_status st = read_inst(p, slot, &I);
  if (st != SIC_OK) return st;
  I.step = step;
  double *stage = nullptr;  // allocated here (freed below)
  const double *dx = x, *dv = v;
  if (mem_kind == SIC_MEM_HOST) {
    double *buf = fixed_stage;
    if (!buf) {
      HIPCHK(p, hipMalloc((void **)&stage, sizeof(double) * 2 * (size_t)std::max<int64_t>(sh.n_tracers, 1)));
      buf = stage;
    }
    hipMemcpyAsync(buf, x, sizeof(double) * (size_t)sh.n_tracers, hipMemcpyHostToDevice, p->stream);
    hipMemcpyAsync(buf + sh.n_tracers, v, sizeof(double) * (size_t)sh.n_tracers, hipMemcpyHostToDevice, p->stream);
    dx = buf;
    dv = buf + sh.n_tracers;
  }
  hipError_t e = hipMemcpyAsync(p->inst + slot, &I, sizeof(I), hipMemcpyHostToDevice, p->stream);
  // positions and velocities only: the layout and the charges stay
  int le = (e == hipSuccess) ? ingest_slot(p, slot, dx, nullptr, dv, nullptr, nullptr, true) : 0;
  if (le == 0 && e == hipSuccess)
    le = launch_zero_mesh(p->prec, p->meshP, p->meshD, p->meshR, p->inst, p->slot_ids + slot, 1, p->rep,
                                         mesh_words(p), p->stream);
  hipError_t e2 = hipStreamSynchronize(p->stream);
  if (stage) hipFree(stage);
  if (e != hipSuccess || e2 != hipSuccess || le != 0) return fail(p, SIC_EDEVICE, "set_state failed");
  sh.state = kStale;
  sh.pending_push = sh.pending_dep = false;
  sh.hist_from = step;
  return SIC_OK;
}

// ---- single-simulation state machine ----
sic_status sim_deposit(Pool *p) {
  SlotHost &sh = p->slots[0];
  if (sh.state == kDeposited) {
    LAUNCHCHK(p, launch_zero_mesh(p->prec, p->meshP, p->meshD, p->meshR, p->inst, p->slot_ids, 1, p->rep,
                                  mesh_words(p), p->stream));
  }
  sic_status st = launch_tracer_mode(p, kDeposit, -1, p->stream);
  if (st != SIC_OK) return st;
  sh.state = kDeposited;
  sh.pending_dep = true;
  return SIC_OK;
}

sic_status sim_solve(Pool *p) {
  SlotHost &sh = p->slots[0];
  if (sh.state != kDeposited) return fail(p, SIC_ESTATE, "solve needs a deposit of the current positions");
  const int flags = (sh.pending_push ? kHavePush : 0) | (sh.pending_dep ? kHaveDeposit : 0);
  sic_status st = launch_solve_mode(p, flags, -1, p->stream);
  if (st != SIC_OK) return st;
  sh.state = kField;
  sh.pending_push = sh.pending_dep = false;
  return SIC_OK;
}

sic_status sim_push(Pool *p) {
  SlotHost &sh = p->slots[0];
  if (sh.state != kField) return fail(p, SIC_ESTATE, "push needs the field of the current step");
  sic_status st = launch_tracer_mode(p, kPush, -1, p->stream);
  if (st != SIC_OK) return st;
  sh.state = kStale;
  sh.pending_push = true;
  return SIC_OK;
}

// ---- refinement on the device (single simulation) ----
//
// Every step: the fused step and its solve, then a marking pass, the plan
// (flat staging offsets, new sheet sizes, capacity), the scatter into the
// flat staging, the new layout (descriptors, links, charge edges, work
// items), the re-ingest, and a deposit and solve of the refined state - each
// launch reading the counts the previous ones left on the device, the
// launches sized for the simulation's reservation, and the ones after the
// plan doing nothing when no segment was split.  No host round trip per
// step: the host layout is brought up to date once at the end.

// Work items for the whole reservation (tile fixed for it), the first
// ceil(n_chunks / tile) of them live; the rest are written by the device as
// the simulation grows.
sic_status place_slot_items_reserved(Pool *p, int32_t slot) {
  SlotHost &s = p->slots[slot];
  sic_status st = clear_slot_items(p, slot);
  if (st != SIC_OK) return st;
  const int tile = slot_tile(p, s.n_chunks_res, false);
  p->tile = tile;
  const int32_t cap = (s.n_chunks_res + tile - 1) / tile;
  const int32_t now = (s.n_chunks + tile - 1) / tile;
  const int64_t ib = p->item_alloc.alloc(cap);
  if (ib < 0) return fail(p, SIC_EBUSY, "work-item arena full");
  std::vector<Item> its((size_t)cap);
  for (int32_t k = 0; k < cap; ++k) {
    its[k].inst = k < now ? slot : -1;
    its[k].chunk_begin = s.chunk_begin + k * tile;
    its[k].chunk_end = s.chunk_begin + std::min(s.n_chunks, (k + 1) * tile);
    its[k].pad = 0;
  }
  s.item_begin = (int32_t)ib;
  s.n_items = cap;  // the range held (released as a whole)
  p->slot_items_h[slot] = make_int2((int32_t)ib, cap);  // grids cover the reservation
  const int2 live = make_int2((int32_t)ib, now);
  HIPCHK(p, hipMemcpyAsync(p->items + ib, its.data(), sizeof(Item) * (size_t)cap, hipMemcpyHostToDevice, p->stream));
  HIPCHK(p, hipMemcpyAsync(p->slot_items + slot, &live, sizeof(int2), hipMemcpyHostToDevice, p->stream));
  st = upload_item_count(p);  // the host high-water mark (grid) covers the reservation
  if (st != SIC_OK) return st;
  const int32_t walk = (int32_t)ib + now;  // the kernels walk the live items only
  HIPCHK(p, hipMemcpyAsync(p->n_items, &walk, sizeof(int32_t), hipMemcpyHostToDevice, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  p->dr_items = true;
  return SIC_OK;
}

sic_status dev_refine_begin(Pool *p) {
  SlotHost &sh = p->slots[0];
  sic_status st = ensure_refine_scratch(p, sh.max_tracers);
  if (st != SIC_OK) return st;
  const int32_t S = (int32_t)sh.n_tracers_s.size();
  if (p->dr_sheets < S || p->dr_chunks < sh.n_chunks_res) {
    for (void *b : {(void *)p->dr_nt, (void *)p->dr_closed, (void *)p->dr_q, (void *)p->dr_work, (void *)p->dr_state,
                    (void *)p->dr_in_off})
      if (b) hipFree(b);
    p->dr_nt = p->dr_closed = p->dr_state = nullptr;
    p->dr_q = nullptr;
    p->dr_work = p->dr_in_off = nullptr;
    p->dr_sheets = p->dr_chunks = 0;
    HIPCHK(p, dalloc(&p->dr_nt, (size_t)S));
    HIPCHK(p, dalloc(&p->dr_closed, (size_t)S));
    HIPCHK(p, dalloc(&p->dr_q, (size_t)S));
    HIPCHK(p, dalloc(&p->dr_work, 3 * (size_t)S + 3));
    HIPCHK(p, dalloc(&p->dr_state, (size_t)kRefWords));
    HIPCHK(p, dalloc(&p->dr_in_off, (size_t)sh.n_chunks_res));
    p->dr_sheets = S;
    p->dr_chunks = sh.n_chunks_res;
  }
  int32_t stw[kRefWords] = {};
  stw[kRefChunks] = sh.n_chunks;
  HIPCHK(p, hipMemcpyAsync(p->dr_nt, sh.n_tracers_s.data(), sizeof(int32_t) * (size_t)S, hipMemcpyHostToDevice,
                           p->stream));
  HIPCHK(p, hipMemcpyAsync(p->dr_closed, sh.closed_s.data(), sizeof(int32_t) * (size_t)S, hipMemcpyHostToDevice,
                           p->stream));
  HIPCHK(p, hipMemcpyAsync(p->dr_q, sh.q_s.data(), sizeof(double) * (size_t)S, hipMemcpyHostToDevice, p->stream));
  HIPCHK(p, hipMemcpyAsync(p->dr_state, stw, sizeof(stw), hipMemcpyHostToDevice, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  if (!p->dr_items) {  // kept from an earlier call unless the host laid the slot out since
    const int tile0 = p->tile, grid0 = p->grid;
    st = place_slot_items_reserved(p, 0);
    if (st != SIC_OK) return st;
    if (p->tile != tile0 || p->grid != grid0) destroy_graphs(p);
  }
  p->dev_refine = true;
  return SIC_OK;
}

// The host mirror of the layout after device refinement: the sheets' sizes
// come back and the layout is rebuilt as the host builds it (the same
// content; uploaded again, which also sizes the host's chunk offsets); the
// work items stay laid out for the reservation, so the next refining call
// reuses them and its captured step.  Returns SIC_ENOMEM when a pass was
// refused for capacity.
sic_status dev_refine_end(Pool *p) {
  SlotHost &sh = p->slots[0];
  p->dev_refine = false;
  std::vector<int32_t> nt(sh.n_tracers_s.size());
  int32_t stw[kRefWords];
  HIPCHK(p, hipMemcpyAsync(nt.data(), p->dr_nt, sizeof(int32_t) * nt.size(), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipMemcpyAsync(stw, p->dr_state, sizeof(stw), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  int64_t n_tr = 0;
  for (int32_t t : nt) n_tr += t;
  Layout L;
  build_layout(0, sh.chunk_begin, nt, sh.closed_s, sh.q_s, sh.q_scale, p->prec != kFP64, &L);
  sh.n_tracers = n_tr;
  sh.n_tracers_s = nt;
  sh.chunk_in_off = L.in_off;
  sh.n_chunks = (int32_t)L.cd.size();
  hipError_t e = upload_layout(p, sh, sh.chunk_begin, L);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return fail(p, SIC_EDEVICE, std::string("layout upload: ") + hipGetErrorString(e));
  sic_status st = SIC_OK;
  if (stw[kRefHalt] != 0) {
    // the pass that did not fit inserted nothing; the simulation stays at
    // that step, active again for the caller
    InstDesc I;
    st = read_inst(p, 0, &I);
    if (st != SIC_OK) return st;
    I.active = 1;
    HIPCHK(p, hipMemcpyAsync(p->inst, &I, sizeof(I), hipMemcpyHostToDevice, p->stream));
    HIPCHK(p, hipStreamSynchronize(p->stream));
    return fail(p, SIC_ENOMEM, "refinement exceeds the tracer capacity");
  }
  return SIC_OK;
}

// One refinement pass of slot 0 on the device, after its fused step, on
// stream st.
sic_status dev_refine_pass(Pool *p, double l_max, hipStream_t st) {
  SlotHost &sh = p->slots[0];
  RefineArgs ra;
  ra.chunks = p->chunks;
  ra.inst = p->inst;
  ra.xs = p->xs;
  ra.vs = p->vs;
  ra.segq = p->segq;
  ra.chunk_begin = sh.chunk_begin;
  ra.n_chunks = sh.n_chunks_res;
  ra.l_max = l_max;
  ra.cnt = p->ref_cnt;
  ra.mask = p->ref_mask;
  ra.out_off = p->ref_off;
  ra.w_out = p->ref_w;
  ra.v_out = p->ref_v;
  ra.c_out = p->ref_c;
  ra.state = p->dr_state;
  RefinePlanArgs pa;
  pa.chunks = p->chunks;
  pa.links = p->order == 1 ? p->links : nullptr;
  pa.edge_prev = p->edge_prev;
  pa.in_off = p->dr_in_off;
  pa.items = p->items;
  pa.slot_items = p->slot_items;
  pa.n_items = p->n_items;
  pa.inst = p->inst;
  pa.cnt = p->ref_cnt;
  pa.out_off = p->ref_off;
  pa.nt = p->dr_nt;
  pa.closed = p->dr_closed;
  pa.q = p->dr_q;
  pa.work = p->dr_work;
  pa.state = p->dr_state;
  pa.max_tracers = sh.max_tracers;
  pa.q_scale = sh.q_scale;
  pa.n_sheets = (int32_t)sh.n_tracers_s.size();
  pa.chunk_begin = sh.chunk_begin;
  pa.chunk_cap = sh.n_chunks_res;
  pa.tile = p->tile;
  pa.slot = 0;
  pa.item_begin = sh.item_begin;
  pa.order = p->order;
  pa.fixed = p->prec != kFP64 ? 1 : 0;
  LAUNCHCHK(p, launch_refine_mark(p->prec, ra, st));
  LAUNCHCHK(p, launch_refine_plan(pa, st));
  LAUNCHCHK(p, launch_refine_scatter(p->prec, ra, st));
  LAUNCHCHK(p, launch_refine_layout(pa, st));
  IngestArgs ia;
  ia.x_in = nullptr;
  ia.w_in = p->ref_w;
  ia.v_in = p->ref_v;
  ia.c_in = nullptr;
  ia.cw_in = p->ref_c;
  ia.segq = p->segq;
  ia.q_scale = sh.q_scale;
  ia.chunk_in_off = p->dr_in_off;
  ia.chunk_begin = sh.chunk_begin;
  ia.n_chunks = sh.n_chunks_res;
  ia.chunks = p->chunks;
  ia.inst = p->inst;
  ia.xs = p->xs;
  ia.vs = p->vs;
  ia.halo = p->halo[p->parity];
  ia.halo3 = p->halo3[p->parity];
  ia.state = p->dr_state;
  LAUNCHCHK(p, launch_ingest(p->prec, ia, st));
  LAUNCHCHK(p, launch_charge_edges(p->chunks, p->edge_prev, p->segq, p->cedge, sh.chunk_begin, sh.n_chunks_res,
                                   st, p->dr_state));
  // the refined state's charge and field (only when a segment was split)
  TracerArgs ta = tracer_args(p, kDeposit, 0);
  ta.gate = p->dr_state + kRefInserted;
  const size_t lds = tracer_lds_size(p->prec, p->order, p->seg, p->max_cells, p->tile);
  LAUNCHCHK(p, launch_tracers(p->prec, kDeposit, p->order, p->seg, ta, grid_for(p, 0), p->block, lds, st));
  SolveArgs sa = solve_args(p, kHaveDeposit, 0);
  sa.gate = p->dr_state + kRefInserted;
  LAUNCHCHK(p, launch_solve(p->prec, sa, 1, p->max_cells, st));
  return SIC_OK;
}

// Graphs of k refining steps (fused step, solve, refinement pass), keyed
// apart from the plain step graphs.
sic_status get_refine_graph(Pool *p, int64_t k, double l_max, hipGraphExec_t *out) {
  auto key = std::make_tuple(k, p->parity, p->grid, p->solve_grid, 2);
  auto it = p->graphs.find(key);
  if (it != p->graphs.end()) {
    *out = it->second;
    return SIC_OK;
  }
  const int parity0 = p->parity;
  HIPCHK(p, hipStreamBeginCapture(p->cap, hipStreamCaptureModeRelaxed));
  sic_status s = SIC_OK;
  for (int64_t i = 0; i < k && s == SIC_OK; ++i) {
    s = enqueue_fused(p, p->cap);
    if (s == SIC_OK) s = dev_refine_pass(p, l_max, p->cap);
  }
  p->parity = parity0;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(p->cap, &g);
  if (s != SIC_OK) {
    if (g) hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return fail(p, SIC_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(g);
    return fail(p, SIC_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  p->graph_objs.push_back(g);
  p->graphs[key] = ex;
  *out = ex;
  return SIC_OK;
}

sic_status sim_step_refining(Pool *p, int64_t n) {
  SlotHost &sh = p->slots[0];
  InstDesc I0;
  sic_status st = read_inst(p, 0, &I0);
  if (st == SIC_OK) st = dev_refine_begin(p);
  const int parity0 = p->parity;
  while (n > 0 && st == SIC_OK) {
    const int64_t k = std::min<int64_t>(n, kGraphSteps);
    hipGraphExec_t ex;
    st = get_refine_graph(p, k, sh.l_max, &ex);
    if (st != SIC_OK) break;
    const hipError_t e = hipGraphLaunch(ex, p->stream);
    if (e != hipSuccess) st = fail(p, SIC_EDEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    if (k & 1) p->parity ^= 1;
    n -= k;
  }
  if (!p->dev_refine) return st;
  sic_status st2 = dev_refine_end(p);
  // after a refused pass the remaining steps did nothing (the slot was
  // inactive): the halo buffers alternate only for the steps that ran
  InstDesc I1;
  const sic_status st3 = read_inst(p, 0, &I1);
  if (st3 == SIC_OK) p->parity = parity0 ^ (int)((I1.step - I0.step) & 1);
  if (st != SIC_OK) return st;
  return st2 != SIC_OK ? st2 : st3;
}

sic_status sim_step(Pool *p, int64_t n) {
  if (n < 0) return fail(p, SIC_EINVAL, "n_steps < 0");
  SlotHost &sh = p->slots[0];
  sic_status st = SIC_OK;
  if (sh.state == kStale) st = sim_deposit(p);
  if (st == SIC_OK && sh.state == kDeposited) st = sim_solve(p);
  if (st != SIC_OK) return st;
  if (sh.l_max > 0.0) {
    // refinement after every move: the fused step deposits the moved
    // tracers; when a segment is split the refined state is deposited and
    // solved again, so the step's field and row are those of the refined
    // sheets (all on the device; the timing mode keeps the host passes)
    p->last_path = SIC_PATH_REFINING;
    if (p->timing) {
      for (int64_t i = 0; i < n && st == SIC_OK; ++i) {
        st = run_fused(p, 1);
        if (st == SIC_OK) st = pool_refine(p, 0, sh.l_max, nullptr);
      }
      return st;
    }
    return sim_step_refining(p, n);
  }
  if (p->order == 0 && !p->timing && !p->tune.fused_only && sh.n_chunks <= resident_max_chunks()) {
    p->last_path = SIC_PATH_RESIDENT;
    return run_resident(p, n);
  }
  p->last_path = sf_ready(p) ? SIC_PATH_SOLVE_FIRST : SIC_PATH_FUSED;
  return run_fused(p, n);
}

const char *status_str(sic_status s) {
  switch (s) {
    case SIC_OK: return "ok";
    case SIC_EINVAL: return "invalid argument";
    case SIC_ENOMEM: return "out of memory";
    case SIC_EDEVICE: return "HIP runtime error";
    case SIC_ESTATE: return "call out of order";
    case SIC_EBUSY: return "no free slot or budget";
    case SIC_ENOTSUP: return "not supported";
  }
  return "unknown status";
}

// Batch steps.  Without refining slots: captured graphs of up to 32 steps.
// With refining slots (l_max > 0): one step at a time, each followed by a
// refinement pass of every refining slot that took the step.
sic_status batch_step(Pool *p, int64_t n) {
  std::vector<int32_t> refining;
  for (int32_t i = 0; i < p->slot_cap; ++i)
    if (p->slots[i].live && p->slots[i].l_max > 0.0) refining.push_back(i);
  if (refining.empty()) return run_fused(p, n);
  for (int64_t k = 0; k < n; ++k) {
    std::vector<int32_t> stepping;
    for (int32_t slot : refining) {
      InstDesc I;
      sic_status st = read_inst(p, slot, &I);
      if (st != SIC_OK) return st;
      if (I.active) stepping.push_back(slot);
    }
    if (stepping.empty()) return run_fused(p, n - k);  // no refining slot left to advance
    sic_status st = run_fused(p, 1);
    if (st != SIC_OK) return st;
    for (int32_t slot : stepping) {
      st = pool_refine(p, slot, p->slots[slot].l_max, nullptr);
      if (st != SIC_OK) return st;
    }
  }
  return SIC_OK;
}

sic_status apply_tuning(Pool *p, const sic_tuning *t) {
  if (!t) return fail(p, SIC_EINVAL, "null tuning");
  const int b = t->block_threads;
  if (b != 0 && b != 64 && b != 128 && b != 256 && b != 512 && b != 1024)
    return fail(p, SIC_EINVAL, "block_threads must be 64..1024, a power of two");
  if (t->tile_chunks < 0 || t->grid_blocks < 0) return fail(p, SIC_EINVAL, "negative tuning value");
  HIPCHK(p, hipStreamSynchronize(p->stream));
  p->tune = *t;
  destroy_graphs(p);
  apply_launch_shape(p);
  return relayout_items(p);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int32_t sic_abi_version(void) { return SIC_ABI_VERSION; }

const char *sic_status_str(sic_status s) { return status_str(s); }

sic_status sic_init(const sic_config *cfg, const sic_sheet *sheets, int32_t n_sheets, const double *x0,
                    const double *v0, const double *seg_charges, int32_t mem_kind, void *hip_stream,
                    sic_sim **out) {
  if (!out) return SIC_EINVAL;
  *out = nullptr;
  sic_status st = validate(nullptr, cfg, sheets, n_sheets, x0, v0);
  if (st != SIC_OK) return st;
  int64_t n_ch = 0, n_tr = 0;
  for (int32_t s = 0; s < n_sheets; ++s) {
    n_ch += (sheets[s].n_tracers + kChunk - 1) / kChunk;
    n_tr += sheets[s].n_tracers;
  }
  // room to grow: every sheet may end in a partly filled chunk
  if (cfg->max_tracers > n_tr) n_ch = std::max<int64_t>(n_ch, (cfg->max_tracers + kChunk - 1) / kChunk + n_sheets);
  const int64_t rows = cfg->history_rows > 0 ? std::max<int64_t>(2, cfg->history_rows) : 65536;
  const bool seg = seg_charges != nullptr || cfg->l_max > 0.0;
  Pool *p = nullptr;
  std::string err;
  st = pool_create(cfg->precision, cfg->deposit_order, seg, false, 1, cfg->n_cells, n_ch, rows, 0, hip_stream, &p,
                   &err);
  if (st != SIC_OK) return st;
  int32_t slot = -1;
  st = pool_admit(p, cfg, sheets, n_sheets, x0, v0, seg_charges, mem_kind, -1, &slot);
  if (st != SIC_OK) {
    pool_free(p);
    return st;
  }
  sic_sim *s = new sic_sim();
  s->pool = p;
  *out = s;
  return SIC_OK;
}

sic_status sic_deposit(sic_sim *sim) {
  if (!sim) return SIC_EINVAL;
  return sim_deposit(sim->pool);
}

sic_status sic_solve_field(sic_sim *sim) {
  if (!sim) return SIC_EINVAL;
  return sim_solve(sim->pool);
}

sic_status sic_push(sic_sim *sim) {
  if (!sim) return SIC_EINVAL;
  return sim_push(sim->pool);
}

sic_status sic_step(sic_sim *sim, int64_t n_steps) {
  if (!sim) return SIC_EINVAL;
  return sim_step(sim->pool, n_steps);
}

sic_status sic_diagnostics(sic_sim *sim, sic_diag *out, double *rho_out, double *E_out, sic_diag *history_out,
                           int64_t *history_len) {
  if (!sim) return SIC_EINVAL;
  return pool_diagnostics(sim->pool, 0, out, rho_out, E_out, history_out, history_len);
}

sic_status sic_get_state(sic_sim *sim, double *x, double *v_half, int64_t *step, int32_t mem_kind) {
  if (!sim) return SIC_EINVAL;
  return pool_get_state(sim->pool, 0, x, v_half, step, mem_kind);
}

sic_status sic_set_state(sic_sim *sim, int64_t step, const double *x, const double *v_half, int32_t mem_kind) {
  if (!sim) return SIC_EINVAL;
  return pool_set_state(sim->pool, 0, step, x, v_half, mem_kind);
}

sic_status sic_set_state_noalloc(sic_sim *sim, int64_t step, const double *x, const double *v_half,
                                 int32_t mem_kind) {
  if (!sim) return SIC_EINVAL;
  Pool *p = sim->pool;
  double *stage = nullptr;
  if (mem_kind == SIC_MEM_HOST) {
    if (p->slots[0].n_tracers > (int64_t)SIC_NOALLOC_MAX_TRACERS)
      return fail(p, SIC_EINVAL,
                  "sic_set_state_noalloc: host inputs of more than SIC_NOALLOC_MAX_TRACERS tracers (use sic_set_state "
                  "or device inputs)");
    int cur = 0;
    HIPCHK(p, hipGetDevice(&cur));
    if (cur != p->device) HIPCHK(p, hipSetDevice(p->device));
    const hipError_t e = scratch_address(p->device, &stage);
    if (cur != p->device) (void)hipSetDevice(cur);
    if (e != hipSuccess)
      return fail(p, SIC_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  return pool_set_state(p, 0, step, x, v_half, mem_kind, stage);
}

sic_status sic_refine(sic_sim *sim, double l_max, int64_t *inserted) {
  if (!sim) return SIC_EINVAL;
  return pool_refine(sim->pool, 0, l_max, inserted);
}

sic_status sic_get_layout(const sic_sim *sim, int32_t *n_tracers_out, int64_t *total) {
  if (!sim) return SIC_EINVAL;
  const SlotHost &sh = sim->pool->slots[0];
  if (n_tracers_out) std::memcpy(n_tracers_out, sh.n_tracers_s.data(), sizeof(int32_t) * sh.n_tracers_s.size());
  if (total) *total = sh.n_tracers;
  return SIC_OK;
}

sic_status sic_get_charges(sic_sim *sim, double *seg_charges, int32_t mem_kind) {
  if (!sim) return SIC_EINVAL;
  return pool_get_charges(sim->pool, 0, seg_charges, mem_kind);
}

sic_status sic_load_state(sic_sim *sim, int64_t step, const int32_t *n_tracers, const double *x,
                          const double *v_half, const double *seg_charges, int32_t mem_kind) {
  if (!sim) return SIC_EINVAL;
  return pool_load_state(sim->pool, step, n_tracers, x, v_half, seg_charges, mem_kind);
}

void sic_destroy(sic_sim *sim) {
  if (!sim) return;
  pool_free(sim->pool);
  delete sim;
}

const char *sic_last_error(const sic_sim *sim) { return sim ? sim->pool->err.c_str() : g_last_error.c_str(); }

sic_status sic_set_tuning(sic_sim *sim, const sic_tuning *t) {
  if (!sim) return SIC_EINVAL;
  return apply_tuning(sim->pool, t);
}

sic_status sic_get_tuning(const sic_sim *sim, sic_tuning *t) {
  if (!sim || !t) return SIC_EINVAL;
  t->tile_chunks = sim->pool->tile;
  t->block_threads = sim->pool->block;
  t->grid_blocks = sim->pool->grid;
  t->fused_only = sim->pool->tune.fused_only;
  return SIC_OK;
}

sic_status sic_set_timing(sic_sim *sim, int32_t timing) {
  if (!sim) return SIC_EINVAL;
  sim->pool->timing = timing != 0;
  return SIC_OK;
}

sic_status sic_last_step_path(const sic_sim *sim, int32_t *path) {
  if (!sim || !path) return SIC_EINVAL;
  *path = sim->pool->last_path;
  return SIC_OK;
}

sic_status sic_last_timing(const sic_sim *sim, double *tracer_ms, double *solve_ms) {
  if (!sim) return SIC_EINVAL;
  if (tracer_ms) *tracer_ms = sim->pool->t_tracer;
  if (solve_ms) *solve_ms = sim->pool->t_solve;
  return SIC_OK;
}

// ---- batch ----
sic_status sic_batch_create(int64_t budget_tracers, int32_t max_slots, int32_t max_cells, int32_t precision,
                            int32_t deposit_order, int32_t flags, int64_t history_rows, void *hip_stream,
                            sic_batch **out) {
  if (!out) return SIC_EINVAL;
  *out = nullptr;
  if (budget_tracers < 2 || max_slots < 1 || max_cells < 1 || max_cells > SIC_MAX_CELLS) return SIC_EINVAL;
  if (flags & ~SIC_BATCH_SEGMENT_CHARGES) return SIC_EINVAL;
  if (precision < 0 || precision > 2 || history_rows < 0) return SIC_EINVAL;
  if (deposit_order < 0 || deposit_order > 2) return SIC_ENOTSUP;
  const int64_t rows = history_rows > 0 ? std::max<int64_t>(2, history_rows) : 4096;
  // arena: the budget plus the padding of partly filled last chunks
  const int64_t chunks = (budget_tracers + kChunk - 1) / kChunk + budget_tracers / 512 + 8 * (int64_t)max_slots;
  Pool *p = nullptr;
  std::string err;
  sic_status st = pool_create(precision, deposit_order, (flags & SIC_BATCH_SEGMENT_CHARGES) != 0, true, max_slots,
                              max_cells, chunks, rows, budget_tracers, hip_stream, &p, &err);
  if (st != SIC_OK) return st;
  st = upload_item_count(p);
  if (st != SIC_OK) {
    pool_free(p);
    return st;
  }
  sic_batch *b = new sic_batch();
  b->pool = p;
  *out = b;
  return SIC_OK;
}

sic_status sic_batch_admit(sic_batch *b, const sic_config *cfg, const sic_sheet *sheets, int32_t n_sheets,
                           const double *x0, const double *v0, const double *seg_charges, int32_t mem_kind,
                           int64_t n_steps, int32_t *slot) {
  if (!b || !slot) return SIC_EINVAL;
  return pool_admit(b->pool, cfg, sheets, n_sheets, x0, v0, seg_charges, mem_kind, n_steps, slot);
}

sic_status sic_batch_get_charges(sic_batch *b, int32_t slot, double *seg_charges, int32_t mem_kind) {
  if (!b) return SIC_EINVAL;
  return pool_get_charges(b->pool, slot, seg_charges, mem_kind);
}

sic_status sic_batch_step(sic_batch *b, int64_t n_steps) {
  if (!b) return SIC_EINVAL;
  if (n_steps < 0) return fail(b->pool, SIC_EINVAL, "n_steps < 0");
  return batch_step(b->pool, n_steps);
}

sic_status sic_batch_get_layout(const sic_batch *b, int32_t slot, int32_t *n_tracers_out, int64_t *total) {
  if (!b) return SIC_EINVAL;
  const Pool *p = b->pool;
  if (slot < 0 || slot >= p->slot_cap || !p->slots[slot].live) return SIC_EINVAL;
  const SlotHost &sh = p->slots[slot];
  if (n_tracers_out) std::memcpy(n_tracers_out, sh.n_tracers_s.data(), sizeof(int32_t) * sh.n_tracers_s.size());
  if (total) *total = sh.n_tracers;
  return SIC_OK;
}

sic_status sic_batch_poll(sic_batch *b, int32_t *done_slots, int32_t cap, int32_t *n_done) {
  if (!b || !n_done) return SIC_EINVAL;
  Pool *p = b->pool;
  std::vector<int32_t> d((size_t)p->slot_cap);
  HIPCHK(p, hipStreamSynchronize(p->stream));
  HIPCHK(p, hipMemcpy(d.data(), p->done, sizeof(int32_t) * d.size(), hipMemcpyDeviceToHost));
  int32_t n = 0;
  for (int32_t i = 0; i < p->slot_cap; ++i) {
    if (p->slots[i].live && d[i] && !p->slots[i].reported) {
      if (n >= cap) break;
      if (done_slots) done_slots[n] = i;
      p->slots[i].reported = true;
      ++n;
    }
  }
  *n_done = n;
  return SIC_OK;
}

sic_status sic_batch_result(sic_batch *b, int32_t slot, sic_diag *out, double *rho_out, double *E_out,
                            sic_diag *history_out, int64_t *history_len) {
  if (!b) return SIC_EINVAL;
  return pool_diagnostics(b->pool, slot, out, rho_out, E_out, history_out, history_len);
}

sic_status sic_batch_get_state(sic_batch *b, int32_t slot, double *x, double *v_half, int64_t *step,
                               int32_t mem_kind) {
  if (!b) return SIC_EINVAL;
  return pool_get_state(b->pool, slot, x, v_half, step, mem_kind);
}

sic_status sic_batch_release(sic_batch *b, int32_t slot) {
  if (!b) return SIC_EINVAL;
  return pool_release(b->pool, slot);
}

sic_status sic_batch_usage(const sic_batch *b, int64_t *tracers, int32_t *slots) {
  if (!b) return SIC_EINVAL;
  if (tracers) *tracers = b->pool->used_tracers;
  if (slots) *slots = b->pool->used_slots;
  return SIC_OK;
}

sic_status sic_batch_set_tuning(sic_batch *b, const sic_tuning *t) {
  if (!b) return SIC_EINVAL;
  return apply_tuning(b->pool, t);
}

sic_status sic_batch_get_tuning(const sic_batch *b, sic_tuning *t) {
  if (!b || !t) return SIC_EINVAL;
  t->tile_chunks = b->pool->tile;
  t->block_threads = b->pool->block;
  t->grid_blocks = b->pool->grid;
  t->fused_only = 0;
  return SIC_OK;
}

void sic_batch_destroy(sic_batch *b) {
  if (!b) return;
  pool_free(b->pool);
  delete b;
}

const char *sic_batch_last_error(const sic_batch *b) { return b ? b->pool->err.c_str() : g_last_error.c_str(); }

sic_status sic_autotune(sic_sim *sim, int32_t steps_per_trial, sic_tuning *best, double *best_ms) {
  if (!sim) return SIC_EINVAL;
  return pool_autotune(sim->pool, steps_per_trial, best, best_ms);
}

sic_status sic_batch_autotune(sic_batch *b, int32_t steps_per_trial, sic_tuning *best, double *best_ms) {
  if (!b) return SIC_EINVAL;
  return pool_autotune(b->pool, steps_per_trial, best, best_ms);
}

sic_status sic_batch_set_timing(sic_batch *b, int32_t timing) {
  if (!b) return SIC_EINVAL;
  b->pool->timing = timing != 0;
  return SIC_OK;
}

sic_status sic_batch_last_timing(const sic_batch *b, double *tracer_ms, double *solve_ms) {
  if (!b) return SIC_EINVAL;
  if (tracer_ms) *tracer_ms = b->pool->t_tracer;
  if (solve_ms) *solve_ms = b->pool->t_solve;
  return SIC_OK;
}

sic_status sic_copy_bandwidth(int64_t n_bytes, int32_t iters, void *hip_stream, double *gbps) {
  if (n_bytes < 1024 || iters < 1 || !gbps) return SIC_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t n = n_bytes / 16 * 2;  // doubles, even
  double *a = nullptr, *b = nullptr;
  if (hipMalloc((void **)&a, sizeof(double) * (size_t)n) != hipSuccess) return SIC_ENOMEM;
  if (hipMalloc((void **)&b, sizeof(double) * (size_t)n) != hipSuccess) {
    hipFree(a);
    return SIC_ENOMEM;
  }
  hipMemsetAsync(a, 0, sizeof(double) * (size_t)n, st);
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  double best = 0.0;
  sic_status rc = SIC_OK;
  // grids of 4 to 32 workgroups of 256 threads per CU (256 CUs)
  for (int grid : {1024, 2048, 4096, 8192}) {
    launch_copy_bench(a, b, n, grid, st);  // warm-up
    for (int i = 0; i < iters && rc == SIC_OK; ++i) {
      hipEventRecord(e0, st);
      if (launch_copy_bench(a, b, n, grid, st) != 0) {
        rc = SIC_EDEVICE;
        break;
      }
      hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) {
        rc = SIC_EDEVICE;
        break;
      }
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      const double g = 2.0 * 8.0 * (double)n / (ms * 1e-3) / 1e9;
      best = std::max(best, g);
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(a);
  hipFree(b);
  *gbps = best;
  return rc;
}

}  // extern "C"
