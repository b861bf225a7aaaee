// sic_kernels.hip - gfx950 kernels of the simplex-in-cell (SIC) 1D1V step.
//
//   k_tracers  one pass over the tracers: gather + leapfrog move (section 2.3,
//              "gather" with first-order weighting of section 2.4, "move"),
//              and/or the exact segment deposit (section 2.3, eqs. "overlap"
//              and "rho_sum") of the resulting positions.  Workgroups walk
//              a list of work items (by default one item each); one item is
//              a run of 64-tracer chunks of one simulation.  Each workgroup
//              accumulates the item's charge in a private LDS copy of that
//              simulation's mesh and merges it into the global mesh with one
//              atomic per touched cell.
//   k_deposit_faces  the deposit alone (constant segments): per tracer only
//              its cell and segment length; the segments that cross a cell
//              face are queued per wavefront and their face geometry runs 64
//              at a time.
//   k_resident a small simulation (up to 32 chunks) stepped many times in one
//              launch of one workgroup: state in registers, mesh in LDS.
//   k_solve    one workgroup per simulation: finishes the deposit (prefix sum
//              of the covered-run difference array), removes the mean density,
//              integrates Gauss's law for the face fields, averages them to
//              cell centres (identical to the 3-point Poisson equation with a
//              centred-difference field), and writes the field energy and
//              the diagnostics row.
//
// Deposit of one segment.  In mesh units (u = x / dx) a segment [u0, u1]
// covers cells c0 = floor(u0) .. c1 = ceil(u1) - 1.  Its charge q is spread
// with density q / (u1 - u0): the two end cells get their partial overlaps,
// and each fully covered cell in between gets the same amount q / (u1 - u0).
// The covered run is added through a difference array D (+w at its first
// cell, -w after its last) that the solve kernel prefix-sums, so a segment
// costs O(1) however many cells it spans.
//
// Split forms keep positions as (cell, fraction) and deposit int64
// fixed-point charge: the first end cell gets round(q * f0), every covered
// cell round(q / len) and the last end cell the remainder, so each segment
// deposits exactly its fixed-point charge and the mesh is independent of the
// order of the atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "sic_internal.h"

namespace sic {

namespace {

// Cell index modulo nc for c in [-nc, 2nc); anything else (only reachable
// from non-finite data) is clamped to cell 0 so that no access leaves the mesh.
__device__ __forceinline__ int wrap_cell(int c, int nc) {
  c = c < 0 ? c + nc : (c >= nc ? c - nc : c);
  return ((unsigned)c < (unsigned)nc) ? c : 0;
}

// Periodic reduction of a position into [0, L).  The common case moves at
// most one period, where x - L is exact; a sum that rounds up to L is 0.
__device__ __forceinline__ double wrap_into_box(double x, double L) {
  if (x >= L) {
    x = x - L;
    if (x >= L) x = x - L * floor(x / L);
  } else if (x < 0.0) {
    x = (x >= -L) ? x + L : x - L * floor(x / L);
    if (x < 0.0) x += L;
  }
  return (x >= L) ? 0.0 : x;
}

// ---- split position words ----
//
// U32: the low 32 bits hold the cell, the high 32 bits the fraction of the
// cell as an unsigned integer in units of 2^-32 cell.
// F32: the low 32 bits hold an index on a lattice of 2^kSubBits sub-cells
// per cell (cell = index >> kSubBits), the high 32 bits a float32 offset in
// [0, 1) of a sub-cell.  With 4096 cells at most the index fits 32 bits; the
// float's 24-bit significand then resolves about 2^-44 of a cell, the
// resolution of a float64 position near the top of such a mesh, where a
// float32 offset spanning a whole cell would only resolve 2^-24 of it.
constexpr int kSubBits = 20;
constexpr uint32_t kSubMask = (1u << kSubBits) - 1u;

template <int PREC>
__device__ __forceinline__ int split_cell(uint64_t w) {
  if constexpr (PREC == kSplitF32) return (int)((uint32_t)w >> kSubBits);
  else return (int)(uint32_t)w;
}

// Position within the cell, in [0, 1) cell.
template <int PREC>
__device__ __forceinline__ double split_frac(uint64_t w) {
  if constexpr (PREC == kSplitF32) {
    return ((double)((uint32_t)w & kSubMask) + (double)__uint_as_float((uint32_t)(w >> 32))) * 0x1p-20;
  } else {
    return (double)(uint32_t)(w >> 32) * 0x1p-32;
  }
}

// Word of the point cell + r (r in [0, 1] cell, cell any integer the caller
// has reduced to -nc .. 2nc - 1): the rounding of r to the offset type may
// carry into the next cell.
template <int PREC>
__device__ __forceinline__ uint64_t split_word(int cell, double r, int nc) {
  if constexpr (PREC == kSplitF32) {
    const double ts = r * 0x1p20;  // sub-cells, exact
    double sub = floor(ts);
    float o = (float)(ts - sub);
    if (o >= 1.0f) {
      o = 0.0f;
      sub += 1.0;
    }
    int c = cell;
    if (sub >= 0x1p20) {
      sub -= 0x1p20;
      c += 1;
    }
    c = wrap_cell(c, nc);
    const uint32_t idx = ((uint32_t)c << kSubBits) | ((uint32_t)sub & kSubMask);
    return (uint64_t)idx | ((uint64_t)__float_as_uint(o) << 32);
  } else {
    double sc = rint(r * 4294967296.0);
    int c = cell;
    if (sc >= 4294967296.0) {
      sc = 0.0;
      c += 1;
    }
    return (uint64_t)(uint32_t)wrap_cell(c, nc) | ((uint64_t)(uint32_t)sc << 32);
  }
}

// Position in mesh units of a state word.
template <int PREC>
__device__ __forceinline__ double mesh_pos(uint64_t w, double inv_dx) {
  if constexpr (PREC == kFP64) {
    return __longlong_as_double((long long)w) * inv_dx;
  } else {
    return (double)split_cell<PREC>(w) + split_frac<PREC>(w);
  }
}

// Field at a tracer: linear interpolation between the two cell centres
// around it (first-order weighting).  u is the position in mesh units.
__device__ __forceinline__ double gather_field(const double *E, double u, int nc) {
  const double g = u - 0.5;
  const double f = floor(g);
  const double s = g - f;
  const int j0 = wrap_cell((int)f, nc);
  const int j1 = (j0 + 1 == nc) ? 0 : j0 + 1;
  return (1.0 - s) * E[j0] + s * E[j1];
}

// The same interpolation from a field array with one ghost cell on each side
// (E[-1] = E[nc-1], E[nc] = E[0]): no periodic wrap of the two indices; the
// clamp keeps non-finite positions inside the array.
__device__ __forceinline__ double gather_field_ghost(const double *E, double u, int nc) {
  const double g = u - 0.5;
  const double f = floor(g);
  const double s = g - f;
  const int j = min(max((int)f, -1), nc - 1);
  return (1.0 - s) * E[j] + s * E[j + 1];
}

// Split-form word moved by du cells: the position advances by whole cells
// (or, in the F32 form, whole sub-cells) plus a rest that is re-quantised;
// the index wraps periodically.  A non-finite move (a non-finite velocity,
// which the diagnostics flag) leaves the word as it is: a split position has
// no non-finite value.
template <int PREC>
__device__ __forceinline__ uint64_t advance_split(uint64_t w, double du, int nc) {
  // F32 counts in sub-cells, U32 in cells
  constexpr double kUnit = PREC == kSplitF32 ? 0x1p20 : 1.0;
  const double t = (PREC == kSplitF32 ? (double)__uint_as_float((uint32_t)(w >> 32)) : split_frac<PREC>(w)) +
                   du * kUnit;
  if (!(t - t == 0.0)) return w;
  const double k = floor(t);
  const double r = t - k;
  // a step of under 2^31 units converts through a 32-bit integer; longer
  // ones (and their 64-bit conversion) take the rare branch below
  const bool near = fabs(k) < 0x1p31;
  long long carry = 0;
  uint32_t bits;
  if constexpr (PREC == kSplitF32) {
    float o = (float)r;
    if (o >= 1.0f) {
      o = 0.0f;
      carry = 1;
    }
    bits = __float_as_uint(o);
  } else {
    double sc = rint(r * 4294967296.0);
    if (sc >= 4294967296.0) {
      sc = 0.0;
      carry = 1;
    }
    bits = (uint32_t)sc;
  }
  const long long period = (long long)nc << (PREC == kSplitF32 ? kSubBits : 0);
  // a move of less than a period needs one conditional wrap; the (slow,
  // 64-bit) remainder only for longer ones
  bool far = !near;
  long long idx = 0;
  if constexpr (PREC == kSplitU32) {
    // the cell index is below 4096: a near move stays in 32-bit integers
    int c = (int)(uint32_t)w + (int)(near ? k : 0.0) + (int)carry;
    if (c >= nc) c -= nc;
    else if (c < 0) c += nc;
    far = far || (unsigned)c >= (unsigned)nc;
    idx = c;
  } else {
    idx = (long long)(uint32_t)w + (long long)(int)(near ? k : 0.0) + carry;
    if (idx >= period) idx -= period;
    else if (idx < 0) idx += period;
    far = far || (unsigned long long)idx >= (unsigned long long)period;
  }
  if (far) {
    idx = ((long long)(uint32_t)w + (long long)k + carry) % period;
    if (idx < 0) idx += period;
  }
  return (uint64_t)(uint32_t)idx | ((uint64_t)bits << 32);
}

// Drift of a state word by dt * v.
template <int PREC>
__device__ __forceinline__ uint64_t drift(uint64_t w, double v, double dt, double L, double inv_dx, int nc) {
  if constexpr (PREC == kFP64) {
    const double x = __longlong_as_double((long long)w);
    return (uint64_t)__double_as_longlong(wrap_into_box(x + dt * v, L));
  } else {
    return advance_split<PREC>(w, (dt * v) * inv_dx, nc);
  }
}

template <class T>
__device__ __forceinline__ void lds_add(T *p, T v) {
  if constexpr (std::is_same<T, double>::value) {
    unsafeAtomicAdd(p, v);
  } else {
    atomicAdd(p, v);
  }
}

// Adds w to cells lo..hi (unwrapped indices, 0 <= hi - lo < nc) of the
// difference array: +w at the first cell, -w after the last.
template <class T>
__device__ __forceinline__ void add_run(T *sD, int lo, int hi, T w, int nc) {
  const int l = wrap_cell(lo, nc);
  const int h = l + min(hi - lo, nc - 1);
  lds_add(sD + l, w);
  if (h + 1 < nc) {
    lds_add(sD + h + 1, (T)(0 - w));
  } else if (h >= nc) {
    lds_add(sD, w);
    lds_add(sD + (h - nc + 1), (T)(0 - w));
  }
}

// 1 / x (x finite, non-zero, normal) by the hardware reciprocal and two
// Newton steps: within an ulp or so of the correctly rounded quotient, at
// about half the instructions of a division.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

struct Geo {
  double L, half_L, dx, inv_dx, dt;
  int nc;
};

// ---- deposit of constant segments (section 2.3): per segment ----
//
// Used where the tracers are also moved (the fused step): each lane adds its
// segment's end-cell overlaps and covered run directly; the LDS atomics hide
// behind the state the step streams.

// FP64 segment from position a to position b (both in [0, L)).
__device__ __forceinline__ double deposit_fp64(double a, double b, double q, const Geo &g, double *sP,
                                               double *sD) {
  double d = b - a;
  if (d >= g.half_L) d -= g.L;
  else if (d < -g.half_L) d += g.L;
  const double ad = fabs(d);
  if (!(ad <= g.half_L)) return ad;  // non-finite positions: nothing deposited
  if (d == 0.0) {
    // zero-length segment: all of q into the cell owning the point, a point
    // on a face belonging to the lower cell
    const int c = wrap_cell((int)ceil(a / g.dx) - 1, g.nc);
    lds_add(sP + c, q);
    return 0.0;
  }
  const double ua = a * g.inv_dx;
  const double ue = ua + d * g.inv_dx;
  const double u0 = d > 0.0 ? ua : ue;
  const double u1 = d > 0.0 ? ue : ua;
  const double len = u1 - u0;
  const double f0 = floor(u0);
  const int c0 = (int)f0;
  const int c1 = (int)ceil(u1) - 1;
  if (!(len > 0.0) || c1 <= c0) {
    lds_add(sP + wrap_cell(c0, g.nc), q);
    return ad;
  }
  const double w = q / len;
  lds_add(sP + wrap_cell(c0, g.nc), w * ((f0 + 1.0) - u0));
  lds_add(sP + wrap_cell(c1, g.nc), w * (u1 - (double)c1));
  if (c1 - c0 >= 2) add_run(sD, c0 + 1, c1 - 1, w, g.nc);
  return ad;
}

// Split-form segment; positions in mesh units ua = cell + fraction.
template <int PREC>
__device__ __forceinline__ double deposit_split(uint64_t wa, uint64_t wb, long long qf, const Geo &g,
                                                unsigned long long *sP, unsigned long long *sD) {
  const int ca = split_cell<PREC>(wa);
  const double fa = split_frac<PREC>(wa);
  const double ua = (double)ca + fa;
  const double ub = mesh_pos<PREC>(wb, g.inv_dx);
  const double half_nc = 0.5 * (double)g.nc;
  double du = ub - ua;
  if (du >= half_nc) du -= (double)g.nc;
  else if (du < -half_nc) du += (double)g.nc;
  const double ad = fabs(du) * g.dx;
  if (!(fabs(du) <= half_nc)) return ad;
  if (du == 0.0) {
    const int c = wrap_cell(fa == 0.0 ? ca - 1 : ca, g.nc);
    lds_add(sP + c, (unsigned long long)qf);
    return 0.0;
  }
  const double ue = ua + du;
  const double u0 = du > 0.0 ? ua : ue;
  const double u1 = du > 0.0 ? ue : ua;
  const double len = u1 - u0;
  const double f0 = floor(u0);
  const int c0 = (int)f0;
  const int c1 = (int)ceil(u1) - 1;
  if (!(len > 0.0) || c1 <= c0) {
    lds_add(sP + wrap_cell(c0, g.nc), (unsigned long long)qf);
    return ad;
  }
  // a correctly rounded quotient is not needed: the shares are rounded to
  // fixed point and the last takes the rest, so the charge is conserved
  // exactly
  const double inv = recip(len);
  const double qd = (double)qf;
  const long long p0 = llrint(qd * (((f0 + 1.0) - u0) * inv));
  long long p1 = qf - p0;
  if (c1 - c0 >= 2) {
    const long long wfix = llrint(qd * inv);
    add_run(sD, c0 + 1, c1 - 1, (unsigned long long)wfix, g.nc);
    p1 -= (long long)(c1 - c0 - 1) * wfix;
  }
  lds_add(sP + wrap_cell(c0, g.nc), (unsigned long long)p0);
  lds_add(sP + wrap_cell(c1, g.nc), (unsigned long long)p1);
  return ad;
}

// ---- deposit of constant segments (section 2.3): face-crossing form ----
//
// Within one 64-tracer chunk let S_t be the charge of the segments before
// segment t.  Walking along the sheet, the charge passed so far at a point of
// segment t is S_t plus the share of q_t before that point (the box function
// is uniform).  The charge of a cell is that cumulative charge where the
// sheet leaves the cell minus where it entered, summed over its visits, so
// every face a segment crosses adds the cumulative charge C at that face to
// the cell being left and subtracts it from the cell being entered.  The two
// terms at a tracer (the end of one segment, the start of the next) fall in
// the same cell and cancel, so a segment inside one cell adds nothing; the
// chunk adds its total charge to the cell where its last segment ends (its
// start contributes -S_0 = 0).  Faces strictly between a segment's first and
// last crossing enclose fully covered cells, which all get q/length (one
// run in the difference array).  The result equals the exact overlap
// deposit; on a dense sheet a wavefront issues LDS atomics only where it
// crosses faces, instead of one or two per tracer.  In fixed point every term
// is an integer and the terms telescope, so each chunk deposits exactly its
// charge.  Used for deposits that do not also move the tracers (the
// deposit-only kernel below), where the per-tracer arithmetic, not the state
// traffic, sets the pace; inside the fused step the per-segment form is
// faster (measured: 8 %).
//
// Cells here are raw: -1 .. nc - 1 before the periodic wrap, a point on a
// face belonging to the lower cell (the W_0 tie rule, which decides where a
// zero-length segment puts its charge): ceil(x / dx) - 1 with the rounded
// quotient.

template <class T>
struct Crossings {
  int lo, hi;  // faces crossed, unwrapped (hi < lo: none)
  T cf, cl;    // cumulative charge at the first and at the last face crossed
  T w;         // charge of each fully covered cell
};

// Faces crossed by the segment from tracer a (cell pa) to tracer b (cell pb),
// the shorter way round, with charge q and chunk charge S before it.
template <int PREC, class T>
__device__ __forceinline__ Crossings<T> face_crossings(uint64_t wa, uint64_t wb, int pa, int pb, T q, T S,
                                                       const Geo &g, double *len_out) {
  Crossings<T> c;
  c.lo = 1;
  c.hi = 0;
  c.cf = c.cl = c.w = (T)0;
  double ua, dm;
  int m = 0;  // periodic image of b relative to a
  if constexpr (PREC == kFP64) {
    const double xa = __longlong_as_double((long long)wa);
    double d = __longlong_as_double((long long)wb) - xa;
    if (d >= g.half_L) {
      d -= g.L;
      m = -1;
    } else if (d < -g.half_L) {
      d += g.L;
      m = 1;
    }
    *len_out = fabs(d);
    if (!(fabs(d) <= g.half_L)) return c;  // non-finite positions
    ua = xa * g.inv_dx;
    dm = d * g.inv_dx;
  } else {
    ua = mesh_pos<PREC>(wa, g.inv_dx);
    const double half_nc = 0.5 * (double)g.nc;
    double du = mesh_pos<PREC>(wb, g.inv_dx) - ua;
    if (du >= half_nc) {
      du -= (double)g.nc;
      m = -1;
    } else if (du < -half_nc) {
      du += (double)g.nc;
      m = 1;
    }
    *len_out = fabs(du) * g.dx;
    if (!(fabs(du) <= half_nc)) return c;
    dm = du;
  }
  const int pbu = pb + m * g.nc;
  if (dm > 0.0) {
    c.lo = pa + 1;  // upward: faces pa+1 .. pb
    c.hi = pbu;
  } else if (dm < 0.0) {
    c.lo = pbu + 1;  // downward: faces pa .. pb+1
    c.hi = pa;
  }
  if (c.hi < c.lo) return c;
  const double len = fabs(dm);
  // length of the segment before its first face, and the charge on it
  const double before = fmin(fmax(dm > 0.0 ? (double)c.lo - ua : ua - (double)c.hi, 0.0), len);
  if constexpr (PREC == kFP64) {
    c.w = q / len;
    c.cf = S + c.w * before;
    c.cl = c.cf + (double)(c.hi - c.lo) * c.w;
  } else {
    const double r = (double)(long long)q / len;
    const long long wfix = llrint(r);
    c.w = (T)wfix;
    c.cf = S + (T)llrint(r * before);
    c.cl = c.cf + (T)((long long)(c.hi - c.lo) * wfix);
  }
  return c;
}

template <class T, class Op>
__device__ __forceinline__ T wave_incl_scan(T v, Op op);
template <class T>
__device__ __forceinline__ T lane_up1(T v);

// Exclusive prefix sum over the wavefront (called by all 64 lanes): the
// inclusive scan moved up one lane.
template <class T>
__device__ __forceinline__ T wave_exclusive_sum(T v) {
  const int lane = threadIdx.x & 63;
  const T prev = lane_up1(wave_incl_scan(v, [](T x, T y) { return x + y; }));
  return lane == 0 ? (T)0 : prev;
}

// ---- piecewise-linear segments (section 2.5) ----
//
// Segment i (tracer i to tracer i+1) carries rho(u) = rho0 + (u - c) g in mesh
// units, rho0 = q / length, c its centroid, g the central difference of the
// neighbouring segments' rho0 over their centroid separation, or 0 at a fold
// corner (centroids not monotone), at an open sheet's end, or when any of the
// three segments has zero length.  Each end cell gets the integral over its
// overlap; the fully covered cells l..h get rho0 + g (j + 1/2 - c), a linear
// ramp A + B (j - l) added through the difference arrays D (constant part)
// and R (second difference of the ramp), so a segment still costs O(1).

// Ramp A + B (j - l) on cells l..h of one period (0 <= l <= h < nc).
template <class T>
__device__ __forceinline__ void add_ramp_nowrap(T *sD, T *sR, int l, int h, T A, T B, int nc) {
  lds_add(sD + l, A);
  if (h + 1 < nc) lds_add(sD + h + 1, (T)(0 - (A + B * (T)(h - l))));
  if (l + 1 <= h) {  // the slope needs a run of two cells or more
    lds_add(sR + l + 1, B);
    if (h + 1 < nc) lds_add(sR + h + 1, (T)(0 - B));
  }
}

// Ramp on unwrapped cells lo..hi (0 <= hi - lo < nc).
template <class T>
__device__ __forceinline__ void add_ramp(T *sD, T *sR, int lo, int hi, T A, T B, int nc) {
  const int l = wrap_cell(lo, nc);
  const int h = l + min(hi - lo, nc - 1);
  if (h < nc) {
    add_ramp_nowrap(sD, sR, l, h, A, B, nc);
  } else {
    add_ramp_nowrap(sD, sR, l, nc - 1, A, B, nc);
    add_ramp_nowrap(sD, sR, 0, h - nc, (T)(A + B * (T)(nc - l)), B, nc);
  }
}

__device__ __forceinline__ double min_image_cells(double d, double half_nc, double nc) {
  if (d >= half_nc) d -= nc;
  else if (d < -half_nc) d += nc;
  return d;
}

// Geometry of a segment in mesh units: start, signed length along the
// shorter way round the box and centroid.
struct SegGeo {
  double u, d, c;
};

// Geometry of the segment from state word wa to wb.  Float64 positions take
// the physical minimum image, as the constant scheme does; split positions
// take it in mesh units.
template <int PREC>
__device__ __forceinline__ SegGeo lin_geo(uint64_t wa, uint64_t wb, const Geo &g) {
  SegGeo s;
  if constexpr (PREC == kFP64) {
    const double xa = __longlong_as_double((long long)wa);
    double d = __longlong_as_double((long long)wb) - xa;
    if (d >= g.half_L) d -= g.L;
    else if (d < -g.half_L) d += g.L;
    s.u = xa * g.inv_dx;
    s.d = d * g.inv_dx;
  } else {
    s.u = mesh_pos<PREC>(wa, g.inv_dx);
    s.d = min_image_cells(mesh_pos<PREC>(wb, g.inv_dx) - s.u, 0.5 * (double)g.nc, (double)g.nc);
  }
  s.c = s.u + 0.5 * s.d;
  return s;
}

// Mean density q / length of a segment (q in the accumulator's units), the
// length taken over the extent the deposit integrates so that its pieces add
// up to q; 0 for a zero-length segment.  The quotient by the reciprocal
// (recip): every density, a lane's own and the staged neighbours', comes
// from this one function, so neighbours see the same bits.
__device__ __forceinline__ double lin_density(const SegGeo &s, double q) {
  const double u0 = s.d > 0.0 ? s.u : s.u + s.d;
  const double u1 = s.d > 0.0 ? s.u + s.d : s.u;
  const double len = u1 - u0;
  return len > 0.0 ? q * recip(len) : 0.0;
}

// The density a neighbour's gradient takes from a segment: NaN marks a
// missing segment or one of zero signed length, which drop the gradient.
__device__ __forceinline__ double lin_nb_density(double d, double r) {
  return d != 0.0 ? r : __longlong_as_double(0x7ff8000000000000ll);
}

// Gradient of a segment of signed length d from its neighbours' signed
// lengths and densities (m: the segment before, p: the one after;
// lin_nb_density): the central difference of the densities over the centroid
// separation, 0 at a fold corner (centroids not monotone) or when a neighbour
// is missing or has zero length (density NaN).  Consecutive segments share an
// end, so the centroid before lies (dm_len + d) / 2 behind this one and the
// one after (d + dp_len) / 2 ahead, along the shorter way round the box
// (each length is at most half the box).
__device__ __forceinline__ double lin_gradient(double d, double dm_len, double rm, double dp_len, double rp) {
  // without branches: a wavefront's lanes mostly take the quotient, and the
  // others select 0 (their divisor replaced by 1)
  const double dm = -0.5 * (dm_len + d);
  const double dp = 0.5 * (d + dp_len);
  const bool ok = rm == rm && rp == rp && ((dm < 0.0 && dp > 0.0) || (dm > 0.0 && dp < 0.0));
  const double q = (rp - rm) * recip(ok ? dp - dm : 1.0);
  return ok ? q : 0.0;
}

// A neighbouring segment as the gradient needs it: signed length and density
// (lin_nb_density).
struct LinNb {
  double d, r;
};

// FP64: deposit segment i given its geometry, gradient and density
// r0 = q / length (lin_density; mesh units).
__device__ __forceinline__ void deposit_linear_fp64(double a_phys, const SegGeo &sg, double g, double q, double r0,
                                                    const Geo &geo, double *sP, double *sD, double *sR) {
  if (sg.d == 0.0) {
    const int c = wrap_cell((int)ceil(a_phys / geo.dx) - 1, geo.nc);
    lds_add(sP + c, q);
    return;
  }
  const double u0 = sg.d > 0.0 ? sg.u : sg.u + sg.d;
  const double u1 = sg.d > 0.0 ? sg.u + sg.d : sg.u;
  const double len = u1 - u0;
  const double f0 = floor(u0);
  const int c0 = (int)f0;
  const int c1 = (int)ceil(u1) - 1;
  // a segment inside one cell puts q there; a longer one its first piece
  // (one atomic for both kinds, so a wavefront that holds both issues one)
  const bool multi = (len > 0.0) && c1 > c0;
  const double e0 = f0 + 1.0;
  const double w0 = e0 - u0;
  lds_add(sP + wrap_cell(c0, geo.nc), multi ? w0 * (r0 + g * (0.5 * (u0 + e0) - sg.c)) : q);
  if (multi) {
    const double w1 = u1 - (double)c1;
    lds_add(sP + wrap_cell(c1, geo.nc), w1 * (r0 + g * (0.5 * ((double)c1 + u1) - sg.c)));
    if (c1 - c0 >= 2) {
      const double A = r0 + g * ((double)(c0 + 1) + 0.5 - sg.c);
      add_ramp(sD, sR, c0 + 1, c1 - 1, A, g, geo.nc);
    }
  }
}

// Split form: fixed-point pieces, the last end cell takes the remainder so
// the segment deposits exactly q_fix.
__device__ __forceinline__ void deposit_linear_split(int cell_a, double frac_a, const SegGeo &sg, double g,
                                                     long long qf, double r0, const Geo &geo, unsigned long long *sP,
                                                     unsigned long long *sD, unsigned long long *sR) {
  if (sg.d == 0.0) {
    const int c = wrap_cell(frac_a == 0.0 ? cell_a - 1 : cell_a, geo.nc);
    lds_add(sP + c, (unsigned long long)qf);
    return;
  }
  const double u0 = sg.d > 0.0 ? sg.u : sg.u + sg.d;
  const double u1 = sg.d > 0.0 ? sg.u + sg.d : sg.u;
  const double len = u1 - u0;
  const double f0 = floor(u0);
  const int c0 = (int)f0;
  const int c1 = (int)ceil(u1) - 1;
  // a segment inside one cell puts qf there; a longer one its first piece
  // (one atomic for both kinds)
  const bool multi = (len > 0.0) && c1 > c0;
  const double e0 = f0 + 1.0;
  const long long p0 = multi ? llrint((e0 - u0) * (r0 + g * (0.5 * (u0 + e0) - sg.c))) : qf;
  lds_add(sP + wrap_cell(c0, geo.nc), (unsigned long long)p0);
  if (multi) {
    long long p1 = qf - p0;
    if (c1 - c0 >= 2) {
      const long long n = c1 - c0 - 1;
      const long long A = llrint(r0 + g * ((double)(c0 + 1) + 0.5 - sg.c));
      const long long B = llrint(g);
      add_ramp(sD, sR, c0 + 1, c1 - 1, (unsigned long long)A, (unsigned long long)B, geo.nc);
      p1 -= n * A + B * (n * (n - 1) / 2);
    }
    lds_add(sP + wrap_cell(c1, geo.nc), (unsigned long long)p1);
  }
}

// ---- first-order weighting of segments (section 2.4) ----
//
// Every slice of the box is assigned to the grid points (cell centres) with
// the hat W_1.  With s = u - 1/2 (grid point j at s = j) and r the charge per
// mesh unit, grid point j receives r [H(s1 - j) - H(s0 - j)], H the
// antiderivative of the unit hat.  For a point s = f + t (f = floor(s)), the
// vector H(s - j) over j is 1 up to j = f, less (1 - t)^2 / 2 at f, plus
// t^2 / 2 at f + 1.  With n = f1 - f0 the segment therefore adds
//   f0: a0                 f0 + 1: r - b0 (n >= 1)
//   f0 + 2 .. f1 - 1: r    f1: r - a1 (n >= 2)        f1 + 1: b1 (n >= 1)
// where a = r (1 - t)^2 / 2 and b = r t^2 / 2 at either end; the terms that
// land on one grid point are summed first, so a segment costs as many LDS
// additions as it has distinct grid points, up to four, plus the difference
// array pair for a run of fully covered ones.  Summed terms are written in
// factored form, which keeps a short segment's pieces accurate to rounding of
// its own charge (the plain differences would lose q/length times the
// rounding of O(1) numbers): n = 0 gives f0 q (1 - tm) and f0 + 1 q tm with
// tm = (t0 + t1) / 2 (the hat at the segment's midpoint); n = 1 gives f0 + 1
// r [(1 - t0)(1 + t0) + t1 (2 - t1)] / 2.

__device__ __forceinline__ void deposit_cic_fp64(double u_a, double d_mesh, double q, const Geo &g, double *sP,
                                                 double *sD) {
  const double s0 = (d_mesh > 0.0 ? u_a : u_a + d_mesh) - 0.5;
  const double s1 = (d_mesh > 0.0 ? u_a + d_mesh : u_a) - 0.5;
  const double fl0 = floor(s0);
  const double t0 = s0 - fl0;
  const int f0 = (int)fl0;
  const double fl1 = floor(s1);
  const double t1 = s1 - fl1;
  const int n = (int)fl1 - f0;  // 0 for a point (s1 = s0: t1 = t0, so tm = t0)
  // grid points f0 and f0 + 1 take one addition each in every case; the
  // density (a division) is computed when some lane of the wavefront needs it
  const bool longseg = n >= 1;
  double r = 0.0;
  if (__builtin_amdgcn_ballot_w64(longseg) != 0) r = q / (longseg ? s1 - s0 : 1.0);
  const double hr = 0.5 * r;
  const double tm = 0.5 * (t0 + t1);
  const double a0 = hr * ((1.0 - t0) * (1.0 - t0)), b0 = hr * (t0 * t0);
  lds_add(sP + wrap_cell(f0, g.nc), longseg ? a0 : q * (1.0 - tm));
  lds_add(sP + wrap_cell(f0 + 1, g.nc),
          longseg ? (n == 1 ? hr * ((1.0 - t0) * (1.0 + t0) + t1 * (2.0 - t1)) : r - b0) : q * tm);
  if (longseg) {
    const double a1 = hr * ((1.0 - t1) * (1.0 - t1)), b1 = hr * (t1 * t1);
    lds_add(sP + wrap_cell(f0 + n + 1, g.nc), b1);
    if (n >= 2) {
      lds_add(sP + wrap_cell(f0 + n, g.nc), r - a1);
      if (n >= 3) add_run(sD, f0 + 2, f0 + n - 1, r, g.nc);
    }
  }
}

// Split form: the same terms in fixed-point units; the term at f1 + 1 (at
// f0 + 1 when n = 0) takes the remainder so the segment deposits exactly qf.
__device__ __forceinline__ void deposit_cic_split(double u_a, double d_mesh, long long qf, const Geo &g,
                                                  unsigned long long *sP, unsigned long long *sD) {
  const double qd = (double)qf;
  const double s0 = (d_mesh > 0.0 ? u_a : u_a + d_mesh) - 0.5;
  const double s1 = (d_mesh > 0.0 ? u_a + d_mesh : u_a) - 0.5;
  const double fl0 = floor(s0);
  const double t0 = s0 - fl0;
  const int f0 = (int)fl0;
  if (!(s1 > s0)) {
    const long long p1 = llrint(qd * t0);
    lds_add(sP + wrap_cell(f0, g.nc), (unsigned long long)(qf - p1));
    lds_add(sP + wrap_cell(f0 + 1, g.nc), (unsigned long long)p1);
    return;
  }
  const double fl1 = floor(s1);
  const double t1 = s1 - fl1;
  const int n = (int)fl1 - f0;
  if (n == 0) {
    const long long p0 = llrint(qd * (1.0 - 0.5 * (t0 + t1)));
    lds_add(sP + wrap_cell(f0, g.nc), (unsigned long long)p0);
    lds_add(sP + wrap_cell(f0 + 1, g.nc), (unsigned long long)(qf - p0));
    return;
  }
  const double r = qd / (s1 - s0);
  const double hr = 0.5 * r;
  const double a0 = hr * ((1.0 - t0) * (1.0 - t0)), b0 = hr * (t0 * t0);
  const double a1 = hr * ((1.0 - t1) * (1.0 - t1));
  const long long p0 = llrint(a0);
  const long long p1 = llrint(n == 1 ? hr * ((1.0 - t0) * (1.0 + t0) + t1 * (2.0 - t1)) : r - b0);
  long long rest = qf - p0 - p1;
  lds_add(sP + wrap_cell(f0, g.nc), (unsigned long long)p0);
  lds_add(sP + wrap_cell(f0 + 1, g.nc), (unsigned long long)p1);
  if (n >= 2) {
    const long long pn = llrint(r - a1);
    lds_add(sP + wrap_cell(f0 + n, g.nc), (unsigned long long)pn);
    rest -= pn;
    if (n >= 3) {
      const long long G = llrint(r);
      add_run(sD, f0 + 2, f0 + n - 1, (unsigned long long)G, g.nc);
      rest -= (long long)(n - 2) * G;
    }
  }
  lds_add(sP + wrap_cell(f0 + n + 1, g.nc), (unsigned long long)rest);
}

// A 64-bit value of one lane, broadcast to the wave.
__device__ __forceinline__ uint64_t read_lane64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

__device__ __forceinline__ double nan_max(double a, double b) {
  // max that propagates NaN (a non-finite segment must reach the flags)
  return (b > a || b != b) ? b : a;
}

// A 4- or 8-byte value moved across lanes by a DPP control (CTRL), written
// in the rows of ROWS; lanes left without a source, and rows not written,
// get 0.  Register moves: no LDS round trip.
template <int CTRL, int ROWS, class T>
__device__ __forceinline__ T dpp_move(T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte values");
  T r;
  if constexpr (sizeof(T) == 4) {
    int i;
    __builtin_memcpy(&i, &v, 4);
    i = __builtin_amdgcn_update_dpp(0, i, CTRL, ROWS, 0xf, true);
    __builtin_memcpy(&r, &i, 4);
  } else {
    uint64_t u;
    __builtin_memcpy(&u, &v, 8);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWS, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWS, 0xf, true);
    u = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
    __builtin_memcpy(&r, &u, 8);
  }
  return r;
}

// Inclusive scan over the wavefront (lane i: v_0 op ... op v_i; all 64
// lanes active): within each 16-lane row by shifts of 1, 2, 4 and 8 lanes,
// then across rows by broadcasting lane 15 into rows 1 and 3 and lane 31
// into rows 2 and 3.  Empty sources contribute 0 (an identity for the sums
// and for the maximum of non-negative values here).
template <class T, class Op>
__device__ __forceinline__ T wave_incl_scan(T v, Op op) {
  v = op(v, dpp_move<0x111, 0xf>(v));  // row_shr:1
  v = op(v, dpp_move<0x112, 0xf>(v));  // row_shr:2
  v = op(v, dpp_move<0x114, 0xf>(v));  // row_shr:4
  v = op(v, dpp_move<0x118, 0xf>(v));  // row_shr:8
  v = op(v, dpp_move<0x142, 0xa>(v));  // row_bcast:15
  v = op(v, dpp_move<0x143, 0xc>(v));  // row_bcast:31
  return v;
}

// Lane 63's value in every lane.
template <class T>
__device__ __forceinline__ T from_lane63(T v) {
  T r;
  if constexpr (sizeof(T) == 4) {
    int i;
    __builtin_memcpy(&i, &v, 4);
    i = __builtin_amdgcn_readlane(i, 63);
    __builtin_memcpy(&r, &i, 4);
  } else {
    uint64_t u;
    __builtin_memcpy(&u, &v, 8);
    u = read_lane64(u, 63);
    __builtin_memcpy(&r, &u, 8);
  }
  return r;
}

// Sum and NaN-propagating maximum over the wavefront, the same bits in every
// lane (all 64 lanes active).
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
  return from_lane63(wave_incl_scan(v, [](T x, T y) { return x + y; }));
}
__device__ __forceinline__ double wave_max(double v) {
  return from_lane63(wave_incl_scan(v, [](double x, double y) { return nan_max(x, y); }));
}

// The value of the next lane (lane_down1) or of the previous one (lane_up1),
// a lane at the wavefront's edge keeping its own: __shfl_down / __shfl_up
// by one lane, as a DPP register move (all 64 lanes active).
template <int CTRL, class T>
__device__ __forceinline__ T dpp_wave_shift(T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte values");
  T r;
  if constexpr (sizeof(T) == 4) {
    int i;
    __builtin_memcpy(&i, &v, 4);
    i = __builtin_amdgcn_update_dpp(i, i, CTRL, 0xf, 0xf, false);
    __builtin_memcpy(&r, &i, 4);
  } else {
    uint64_t u;
    __builtin_memcpy(&u, &v, 8);
    const int lo0 = (int)(uint32_t)u, hi0 = (int)(uint32_t)(u >> 32);
    const int lo = __builtin_amdgcn_update_dpp(lo0, lo0, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(hi0, hi0, CTRL, 0xf, 0xf, false);
    u = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
    __builtin_memcpy(&r, &u, 8);
  }
  return r;
}
template <class T>
__device__ __forceinline__ T lane_down1(T v) {
  return dpp_wave_shift<0x130>(v);  // wave_shl:1
}
template <class T>
__device__ __forceinline__ T lane_up1(T v) {
  return dpp_wave_shift<0x138>(v);  // wave_shr:1
}

}  // namespace

// ---------------------------------------------------------------------------
// Field solve
// ---------------------------------------------------------------------------
namespace {

// Inclusive scan over the 256-thread block of one value per thread, in a
// fixed order.  sWave holds 4 entries.
template <class T>
__device__ __forceinline__ T block_incl_scan(T v, T *sWave) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  v = wave_incl_scan(v, [](T x, T y) { return x + y; });
  if (lane == 63) sWave[wave] = v;
  __syncthreads();
  T base = (T)0;
  for (int w = 0; w < wave; ++w) base += sWave[w];
  __syncthreads();
  return v + base;
}

template <class T>
__device__ __forceinline__ T block_sum(T v, T *sWave) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sWave[wave] = v;
  __syncthreads();
  const T r = sWave[0] + sWave[1] + sWave[2] + sWave[3];
  __syncthreads();
  return r;
}

// The solve's scan and sum over its kSolveThreads threads (four wavefronts;
// wider workgroups' other wavefronts hold zeros and take no part), with the
// sums in the order of block_incl_scan and block_sum.  Each call site passes
// four LDS words of its own, so one barrier per call suffices (nothing
// writes them again before the next solve).
template <class T>
__device__ __forceinline__ T solve_incl_scan(T v, T *slot4) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  v = wave_incl_scan(v, [](T x, T y) { return x + y; });
  if (lane == 63 && wave < 4) slot4[wave] = v;
  __syncthreads();
  // wavefronts 0..wave-1 in order; the zeros added after them change no bits
  T base = (T)0;
#pragma unroll
  for (int w = 0; w < 3; ++w) base += (w < wave) ? slot4[w] : (T)0;
  return v + base;
}
template <class T>
__device__ __forceinline__ T solve_sum(T v, T *slot4) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0 && wave < 4) slot4[wave] = v;
  __syncthreads();
  return slot4[0] + slot4[1] + slot4[2] + slot4[3];
}


}  // namespace

// The solve of one slot by one workgroup of kSolveThreads threads: charge
// per cell from the P/D (and R) accumulators, which it clears; mean removal,
// Gauss's law, cell-centre field, field energy; the diagnostics row and the
// step count.  ke, mom, ms are the slot's kinetic-energy, momentum and
// max-segment sums of the step.  The accumulators may be the slot's global
// mesh (k_solve) or a workgroup's LDS copy (k_resident); with sE the field is
// also left in LDS.
// The slot's constants the solve needs, read once by its caller.
struct SlotConst {
  int nc;
  double L, dx, dt, q_unit;
  int64_t mesh_off, hist_off, hist_cap;
};

__device__ __forceinline__ SlotConst slot_const(const InstDesc &I) {
  SlotConst k;
  k.nc = I.n_cells;
  k.L = I.L;
  k.dx = I.dx;
  k.dt = I.dt;
  k.q_unit = I.q_unit;
  k.mesh_off = I.mesh_off;
  k.hist_off = I.hist_off;
  k.hist_cap = I.hist_cap;
  return k;
}

// The slot's point (P) and difference (D) accumulators of this thread's
// cells, summed over their REP copies (rep_stride words apart) in copy
// order and cleared: the first half of the solve, apart so that a caller can
// have these loads in flight with others.  The loads are unconditional (a
// thread past the mesh reads cell 0 and adds zero), so all of them are in
// flight together; the clearing stores follow.
template <int PREC, int CELLS, int REP, class Acc, class T>
__device__ __forceinline__ void solve_take(const SlotConst &kc, Acc *gP, Acc *gD, int64_t rep_stride,
                                           T (&pv)[CELLS], T (&dv)[CELLS]) {
  const int nc = kc.nc;
  const int per = (nc + kSolveThreads - 1) / kSolveThreads;
  const int j0 = threadIdx.x * per;
#pragma unroll
  for (int k = 0; k < CELLS; ++k) {
    pv[k] = (T)0;
    dv[k] = (T)0;
  }
#pragma unroll
  for (int r = 0; r < REP; ++r) {
#pragma unroll
    for (int k = 0; k < CELLS; ++k) {
      const int j = j0 + k;
      const bool own = k < per && j < nc;
      const int64_t at = r * rep_stride + (own ? j : 0);
      const T p = (T)gP[at];
      const T d = (T)gD[at];
      pv[k] += own ? p : (T)0;
      dv[k] += own ? d : (T)0;
    }
  }
#pragma unroll
  for (int r = 0; r < REP; ++r) {
#pragma unroll
    for (int k = 0; k < CELLS; ++k) {
      const int j = j0 + k;
      if (k < per && j < nc) {
        gP[r * rep_stride + j] = (Acc)0;
        gD[r * rep_stride + j] = (Acc)0;
      }
    }
  }
}

// step0 and flags0 are the slot's step and sticky flags before this solve;
// pv, dv this thread's accumulators from solve_take; returns the flags after
// it (the same value in every thread).  With write_field false the field and
// density are left in sE only (the resident kernel writes them to global
// memory on its last step); with writer false nothing at all is written to
// global memory (the workgroups of a launch that each solve the same charge
// for their own use, all but one).  The field in sE is complete only after a
// barrier following the return (without writer the solve passes none after
// its field loop).
template <int PREC, int CELLS, int REP = 1, class Acc, class T>
__device__ __forceinline__ int solve_slot(const SolveArgs &a, int slot, const SlotConst &kc, int64_t step0,
                                          int flags0, const T (&pv)[CELLS], const T (&dv)[CELLS], Acc *gRamp,
                                          double ke, double mom, double ms, double *sE, bool write_field,
                                          bool writer = true) {
  using acc_t = typename std::conditional<PREC == kFP64, double, long long>::type;
  static_assert(std::is_same<acc_t, T>::value, "accumulator type");
  // The cells are partitioned over kSolveThreads threads; a wider workgroup
  // (the resident kernel's) runs the same code, its other threads holding no
  // cells and adding zeros, so the result has the same bits.
  // LDS words of the scans and sums, four per call site
  __shared__ acc_t sA[4][4];
  __shared__ double sF[3][4];
  __shared__ int sBad[4];
  __shared__ double sLastF[kSolveThreads];
  InstDesc *Ip = a.inst + slot;
  const int tid = threadIdx.x;
  const int nc = kc.nc;
  const double L = kc.L, dx = kc.dx, dt = kc.dt;
  const double q_unit = kc.q_unit;

  // 2. charge per cell: Q_j = P_j + sum_{m <= j} D_m
  const int per = (nc + kSolveThreads - 1) / kSolveThreads;
  const int j0 = tid * per;
  double *gE = a.meshE + kc.mesh_off;
  double *gR = a.meshRho + kc.mesh_off;
  acc_t dsum = (acc_t)0;
#pragma unroll
  for (int k = 0; k < CELLS; ++k) dsum += dv[k];
  const acc_t dbase = solve_incl_scan(dsum, sA[0]) - dsum;
  // Linear ramps of piecewise-linear segments: the charge adds the second
  // prefix sum of R (zero for piecewise-constant segments).
  acc_t r2[CELLS];
#pragma unroll
  for (int k = 0; k < CELLS; ++k) r2[k] = (acc_t)0;
  if (gRamp != nullptr) {  // only piecewise-linear segments have ramps; REP copies as P and D
#pragma unroll
    for (int r = 0; r < REP; ++r) {
#pragma unroll
      for (int k = 0; k < CELLS; ++k) {
        const int j = j0 + k;
        const bool own = k < per && j < nc;
        const acc_t v = (acc_t)gRamp[r * a.rep_stride + (own ? j : 0)];
        r2[k] += own ? v : (acc_t)0;
      }
    }
#pragma unroll
    for (int r = 0; r < REP; ++r) {
#pragma unroll
      for (int k = 0; k < CELLS; ++k) {
        const int j = j0 + k;
        if (k < per && j < nc) gRamp[r * a.rep_stride + j] = (Acc)0;
      }
    }
    acc_t rsum = (acc_t)0;
#pragma unroll
    for (int k = 0; k < CELLS; ++k) rsum += r2[k];
    const acc_t base1 = solve_incl_scan(rsum, sA[1]) - rsum;
    acc_t run1 = base1, s1sum = (acc_t)0;
#pragma unroll
    for (int k = 0; k < CELLS; ++k) {
      run1 += r2[k];
      r2[k] = run1;
      if ((k < per) && (j0 + k < nc)) s1sum += run1;
    }
    const acc_t base2 = solve_incl_scan(s1sum, sA[2]) - s1sum;
    acc_t run2 = base2;
#pragma unroll
    for (int k = 0; k < CELLS; ++k) {
      if ((k < per) && (j0 + k < nc)) run2 += r2[k];
      r2[k] = run2;
    }
  }
  double Q[CELLS];
  acc_t qsum_acc = (acc_t)0;
  {
    acc_t run = dbase;
#pragma unroll
    for (int k = 0; k < CELLS; ++k) {
      run += dv[k];
      const acc_t qa = pv[k] + run + r2[k];
      const bool in = (k < per) && (j0 + k < nc);
      if constexpr (PREC == kFP64) Q[k] = in ? qa : 0.0;
      else Q[k] = in ? (double)qa * q_unit : 0.0;
      if (in) qsum_acc += qa;
    }
  }
  double Qtot;
  if constexpr (PREC == kFP64) Qtot = solve_sum(qsum_acc, sA[3]);
  else Qtot = (double)solve_sum(qsum_acc, sA[3]) * q_unit;

  // 3. Gauss's law on faces: F_{j+1/2} = F_{j-1/2} + (Q_j - Qtot/nc),
  //    F shifted to zero mean; E_j = (F_{j-1/2} + F_{j+1/2}) / 2.
  const double qmean = Qtot / (double)nc;
  double F[CELLS];
  double rsum = 0.0;
#pragma unroll
  for (int k = 0; k < CELLS; ++k) {
    const bool in = (k < per) && (j0 + k < nc);
    const double r = in ? (Q[k] - qmean) : 0.0;
    rsum += r;
    F[k] = r;
  }
  const double fbase = solve_incl_scan(rsum, sF[0]) - rsum;
  double fsum = 0.0;
  {
    double run = fbase;
#pragma unroll
    for (int k = 0; k < CELLS; ++k) {
      const bool in = (k < per) && (j0 + k < nc);
      run += F[k];
      F[k] = in ? run : 0.0;
      if (in) fsum += F[k];
    }
  }
  // F's mean and each thread's last face value behind one barrier; the
  // neighbour's value is shifted by the mean after the exchange (the same
  // subtraction, the same bits)
  double lastF = 0.0;
#pragma unroll
  for (int k = 0; k < CELLS; ++k)
    if ((k < per) && (j0 + k < nc)) lastF = F[k];
  {
    const double fw = wave_sum(fsum);
    const int wave = tid >> 6;
    if ((tid & 63) == 0 && wave < 4) sF[1][wave] = fw;
    if (tid < kSolveThreads) sLastF[tid] = lastF;
  }
  __syncthreads();
  const double fmean = (sF[1][0] + sF[1][1] + sF[1][2] + sF[1][3]) / (double)nc;
#pragma unroll
  for (int k = 0; k < CELLS; ++k)
    if ((k < per) && (j0 + k < nc)) F[k] -= fmean;
  double prevF =
      (tid == 0) ? sLastF[(nc - 1) / per] - fmean : (tid < kSolveThreads ? sLastF[tid - 1] - fmean : 0.0);
  double w2 = 0.0;
  bool finite = true;
#pragma unroll
  for (int k = 0; k < CELLS; ++k) {
    const int j = j0 + k;
    if ((k < per) && (j < nc)) {
      const double e = 0.5 * (prevF + F[k]);
      prevF = F[k];
      if (sE) sE[j] = e;
      if (write_field) {
        gE[j] = e;
        gR[j] = (Q[k] - qmean) / dx;
      }
      w2 += e * e;
      finite = finite && (e - e == 0.0);
    }
  }
  // the field energy and the count of non-finite values, in one pass (only
  // a workgroup that writes the diagnostics needs them)
  double W = 0.0;
  int bad = 0;
  if (writer) {
    w2 = wave_sum(w2);
    const int nbad = wave_sum(finite ? 0 : 1);
    const int wave = tid >> 6;
    if ((tid & 63) == 0 && wave < 4) {
      sF[2][wave] = w2;
      sBad[wave] = nbad;
    }
    __syncthreads();
    W = 0.5 * dx * (sF[2][0] + sF[2][1] + sF[2][2] + sF[2][3]);
    bad = sBad[0] + sBad[1] + sBad[2] + sBad[3];
  }

  // 4. diagnostics and step bookkeeping
  const bool pushed = (a.flags & kHavePush) != 0;
  const int64_t step = pushed ? step0 + 1 : step0;
  int f = 0;
  if (bad || !(W - W == 0.0)) f |= 1;
  // a move with a non-finite velocity (its kinetic energy or momentum)
  if (pushed && !((ke - ke == 0.0) && (mom - mom == 0.0))) f |= 1;
  if (a.flags & kHaveDeposit) {
    if (ms != ms) f |= 1;
    else if (ms > 0.45 * L) f |= 2;
  }
  const int flags = flags0 | f;
  if (tid == 0 && writer) {
    Ip->flags = flags;
    const int64_t cap = kc.hist_cap;
    DiagRow *H = a.hist + kc.hist_off;
    DiagRow r;
    r.step = step;
    r.t = (double)step * dt;
    r.W_E = W;
    r.KE = __longlong_as_double(0x7ff8000000000000ll);
    r.momentum = r.KE;
    r.total_charge = Qtot;
    r.max_segment = (a.flags & kHaveDeposit) ? ms : r.KE;
    r.flags = flags;
    H[step % cap] = r;
    if (pushed && step >= 1) {
      DiagRow *prev = H + (step - 1) % cap;
      prev->KE = ke;
      prev->momentum = mom;
    }
    Ip->step = step;
    if ((a.flags & kBatchStep) && pushed && Ip->steps_left > 0) {
      const int64_t left = Ip->steps_left - 1;
      Ip->steps_left = left;
      if (left == 0) {
        Ip->active = 0;
        a.done[slot] = 1;
      }
    }
  }
  return flags;
}

// ---------------------------------------------------------------------------
// Tracer kernel
// ---------------------------------------------------------------------------
// Per-item LDS layout (bytes): P, D (and for linear segments R) accumulators
// and the field E for mesh_cells cells; for tile_cap chunks the item's chunk
// descriptors, the halo copy of the tracer after each chunk (constant
// segments: its state; linear segments: its position word, plus the
// geometry and density of the segment before the chunk and of the one after
// its last segment) and, with per-segment charges, the two charge edges; 48
// doubles for the block reduction.
// ORDER: 0 piecewise-constant segments, 1 piecewise-linear segments (ramp
// array R and three halo copies per chunk), 2 first-order weighting of
// constant segments.  SEG: per-segment charges (a charge word per tracer).
template <class Acc, int ORDER, bool SEG>
__host__ __device__ constexpr size_t tracer_lds_bytes(int mesh_cells, int tile_cap) {
  return (size_t)(2 + (ORDER == 1)) * mesh_cells * sizeof(Acc) + (size_t)(mesh_cells + 2) * sizeof(double) +
         (size_t)tile_cap *
             (sizeof(ChunkDesc) + (ORDER == 1 ? sizeof(uint64_t) + 2 * sizeof(LinNb) : sizeof(double2)) +
              (SEG ? 2 * sizeof(uint64_t) : 0)) +
         48 * sizeof(double);
}

// Charge word -> charge as float64 (split forms: fixed-point units times q_unit).
template <int PREC>
__device__ __forceinline__ double charge_value(uint64_t w, double q_unit) {
  if constexpr (PREC == kFP64) return __longlong_as_double((long long)w);
  else return (double)(long long)w * q_unit;
}

// Mass of a tracer bounded by segments of charge words `left` and `right`:
// half of each.
template <int PREC>
__device__ __forceinline__ double tracer_mass(uint64_t left, uint64_t right, double q_unit) {
  if constexpr (PREC == kFP64) {
    return 0.5 * (__longlong_as_double((long long)left) + __longlong_as_double((long long)right));
  } else {
    return 0.5 * ((double)((long long)left + (long long)right) * q_unit);
  }
}

// SF > 0: a solve-first launch of a single simulation (push + deposit,
// constant segments): before its work items the workgroup solves the
// previous step's charge (SF cells per solve thread) for the field, as a
// solve launch would, instead of reading it.
template <int PREC, int MODE, int ORDER, bool SEG, int SF = 0>
__global__ void __launch_bounds__(1024) k_tracers(TracerArgs a) {
  using acc_t = typename std::conditional<PREC == kFP64, double, unsigned long long>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  acc_t *sP = reinterpret_cast<acc_t *>(smem);
  acc_t *sD = sP + a.mesh_cells;
  constexpr bool kLin = ORDER == 1;
  acc_t *sR = sD + a.mesh_cells;  // linear segments only
  double *sE = reinterpret_cast<double *>(sR + (kLin ? a.mesh_cells : 0)) + 1;  // ghost cells at -1 and nc
  ChunkDesc *sDesc = reinterpret_cast<ChunkDesc *>(sE + a.mesh_cells + 1);
  double2 *sHalo = reinterpret_cast<double2 *>(sDesc + a.tile_cap);     // orders 0, 2: the next tracer
  uint64_t *sNextW = reinterpret_cast<uint64_t *>(sDesc + a.tile_cap);  // order 1: the next tracer's word
  LinNb *sPrevNb = reinterpret_cast<LinNb *>(sNextW + a.tile_cap);      // order 1: segment before the chunk
  LinNb *sNextNb = sPrevNb + a.tile_cap;                                // order 1: segment after its last one
  uint64_t *sEdge = kLin ? reinterpret_cast<uint64_t *>(sNextNb + a.tile_cap)
                         : reinterpret_cast<uint64_t *>(sHalo + a.tile_cap);  // per-segment charges
  double *sRed = reinterpret_cast<double *>(sEdge + (SEG ? 2 * a.tile_cap : 0));  // 3 x 16 waves

  if (a.gate != nullptr && *a.gate <= 0) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nwaves = blockDim.x >> 6;
  const int n_items = *a.n_items;
  constexpr bool kDep = (MODE & kDeposit) != 0;
  constexpr bool kMove = (MODE & kPush) != 0;
  constexpr bool kKick = (MODE & kKickHalf) != 0;
  constexpr bool kField = kMove || kKick;
  constexpr bool kNeedQ = SEG && (kDep || kMove);  // per-segment charges are read
  // chunks whose state is in flight per wavefront (a deposit alone reads 8
  // bytes per tracer and keeps more of them in flight)
  constexpr int kPrefetch = kField ? 3 : 6;
  static_assert(SF == 0 || (MODE == (kPush | kDeposit) && ORDER == 0), "solve-first: the fused step, constant segments");

  if constexpr (SF > 0) {
    // Every workgroup solves the same charge with the same arithmetic, so
    // all hold the field the previous solve launch would have written; the
    // first one writes it and the diagnostics row (with the previous
    // launch's partials, summed in the order the solve launch sums them)
    // and advances the step.  The accumulators of two steps back are
    // cleared here, a slice per workgroup (no launch merges into them
    // before the next one).
    using sacc_t = typename std::conditional<PREC == kFP64, double, long long>::type;
    // the accumulator copies of a mesh of up to SF * kSolveThreads cells
    constexpr int kRep = single_rep(SF * kSolveThreads);
    const int slot = a.items[0].inst;
    const InstDesc &I0 = a.inst[slot];
    const SlotConst kc = slot_const(I0);
    const bool writer = blockIdx.x == 0;
    sacc_t pv[SF], dv[SF];
    {
      // the copies summed in copy order, as the solve launch sums them
      const int per = (kc.nc + kSolveThreads - 1) / kSolveThreads;
      const int j0 = tid * per;
#pragma unroll
      for (int k = 0; k < SF; ++k) {
        pv[k] = (sacc_t)0;
        dv[k] = (sacc_t)0;
      }
      // the loads are unconditional (a thread past the mesh reads cell 0 and
      // adds zero), all copies' in flight together where the registers allow
      auto take = [&](const void *base, int r, sacc_t(&acc)[SF]) {
        const sacc_t *g = reinterpret_cast<const sacc_t *>(base) + kc.mesh_off + r * a.rep_stride;
#pragma unroll
        for (int k = 0; k < SF; ++k) {
          const int j = j0 + k;
          const bool own = k < per && j < kc.nc;
          const sacc_t v = g[own ? j : 0];
          acc[k] += own ? v : (sacc_t)0;
        }
      };
      if constexpr (SF * kRep <= 16) {
#pragma unroll
        for (int r = 0; r < kRep; ++r) {
          take(a.sf_P, r, pv);
          take(a.sf_D, r, dv);
        }
      } else {
#pragma unroll 1
        for (int r = 0; r < kRep; ++r) take(a.sf_P, r, pv);
#pragma unroll 1
        for (int r = 0; r < kRep; ++r) take(a.sf_D, r, dv);
      }
    }
    {
      // this workgroup's slice of every copy
      const int z0 = (int)((int64_t)kc.nc * blockIdx.x / gridDim.x);
      const int z1 = (int)((int64_t)kc.nc * (blockIdx.x + 1) / gridDim.x);
      for (int r = 0; r < kRep; ++r) {
        acc_t *zP = reinterpret_cast<acc_t *>(a.sf_zP) + kc.mesh_off + r * a.rep_stride;
        acc_t *zD = reinterpret_cast<acc_t *>(a.sf_zD) + kc.mesh_off + r * a.rep_stride;
        for (int i = z0 + tid; i < z1; i += blockDim.x) {
          zP[i] = (acc_t)0;
          zD[i] = (acc_t)0;
        }
      }
    }
    double ke = 0.0, mom = 0.0, ms = 0.0;
    if (writer) {
      // as the solve launch: threads tid < 256 sum the slot's items tid,
      // tid + 256, ... (four at a time), then the wavefront sums and waves
      // 0..3 in order
      constexpr int kU = 4;
      const int2 si = a.sf.slot_items[slot];
      const Partial *pp = a.sf_partials + si.x;
      if (tid < kSolveThreads) {
        for (int i0 = tid; i0 < si.y; i0 += kU * kSolveThreads) {
          Partial pr[kU];
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const int i = i0 + u * kSolveThreads;
            if (i < si.y) pr[u] = pp[i];
          }
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            if (i0 + u * kSolveThreads < si.y) {
              ke += pr[u].ke;
              mom += pr[u].mom;
              ms = nan_max(ms, pr[u].maxseg);
            }
          }
        }
      }
      ke = wave_sum(ke);
      mom = wave_sum(mom);
      ms = wave_max(ms);
      if (lane == 0) {
        sRed[wave] = ke;
        sRed[16 + wave] = mom;
        sRed[32 + wave] = ms;
      }
      __syncthreads();
      ke = sRed[0] + sRed[1] + sRed[2] + sRed[3];
      mom = sRed[16] + sRed[17] + sRed[18] + sRed[19];
      ms = nan_max(nan_max(sRed[32], sRed[33]), nan_max(sRed[34], sRed[35]));
      __syncthreads();
    }
    solve_slot<PREC, SF>(a.sf, slot, kc, writer ? I0.step : 0, writer ? I0.flags : 0, pv, dv, (acc_t *)nullptr, ke,
                         mom, ms, sE, writer, writer);
    // the ghost cells copy cells other threads wrote: a barrier first (a
    // workgroup that writes nothing passes none in the solve after its field
    // loop)
    __syncthreads();
    if (tid == 0) {
      sE[-1] = sE[kc.nc - 1];
      sE[kc.nc] = sE[0];
    }
    __syncthreads();
  }

  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const Item item = a.items[it];
    if (item.inst < 0) continue;  // freed slot
    const InstDesc &I = a.inst[item.inst];
    if (a.respect_active && !I.active) continue;
    Geo g;
    g.L = I.L;
    g.half_L = I.half_L;
    g.dx = I.dx;
    g.inv_dx = I.inv_dx;
    g.dt = I.dt;
    g.nc = I.n_cells;
    const int cb = item.chunk_begin;
    const int nch = item.chunk_end - item.chunk_begin;

    // Loads and stores are unconditional (a chunk always has 64 slots; the
    // padding slots of a sheet's last chunk are read and written back
    // unchanged), so the only branches around memory operations are uniform.
    // The state is streamed once per step: non-temporal loads and stores
    // keep it from displacing the meshes and tables in the caches.
    auto load_state = [&](int kk, uint64_t &xw, double &v, uint64_t &cw) {
      // past the item's last chunk every lane reads the item's first slot: the
      // loads are still issued, so the count of loads in flight is the same at
      // every stage and the wait before a stage leaves the later ones in flight
      const size_t s = kk < nch ? (size_t)(cb + kk) * kChunk + lane : (size_t)cb * kChunk;
      xw = __builtin_nontemporal_load(a.xs + s);
      if constexpr (kField) v = __builtin_nontemporal_load(a.vs + s);  // a deposit alone needs no velocity
      if constexpr (kNeedQ) cw = a.segq[s];
    };
    // kPrefetch chunks in flight per wavefront, in fixed registers (the
    // loop is fully unrolled over them).  The first ones are issued before
    // the item's tables are staged: they need only the item's chunk range,
    // so their latency overlaps the staging's.
    uint64_t xr[kPrefetch], cr_[kPrefetch];
    double vr[kPrefetch];
#pragma unroll
    for (int j = 0; j < kPrefetch; ++j) {
      xr[j] = cr_[j] = 0;
      vr[j] = 0.0;
      load_state(wave + j * nwaves, xr[j], vr[j], cr_[j]);
      // issue in stage order, as the loop does: the wait before a stage's
      // first use then leaves the later stages' loads in flight
      __builtin_amdgcn_sched_barrier(0);
    }
    // Stage the item's tables in LDS: one pass of global reads per item
    // instead of dependent reads per chunk.
    for (int i = tid; i < g.nc; i += blockDim.x) {
      if constexpr (kDep) {
        sP[i] = (acc_t)0;
        sD[i] = (acc_t)0;
        if constexpr (kLin) sR[i] = (acc_t)0;
      }
      if constexpr (kField && SF == 0) sE[i] = a.meshE[I.mesh_off + i];
    }
    if constexpr (kField && SF == 0) {
      if (tid == 0) {
        sE[-1] = a.meshE[I.mesh_off + g.nc - 1];
        sE[g.nc] = a.meshE[I.mesh_off];
      }
    }
    for (int i = tid; i < nch; i += blockDim.x) {
      sDesc[i] = a.chunks[cb + i];
      // the next chunk's halo, read with the descriptor: it is the partner
      // of every chunk but a sheet's last (checked below)
      if constexpr (kDep && !kLin) {
        if (i + 1 < nch) sHalo[i] = a.halo_in[cb + i + 1];
      }
      if constexpr (kNeedQ) {
        sEdge[2 * i] = a.cedge[2 * (size_t)(cb + i)];
        sEdge[2 * i + 1] = a.cedge[2 * (size_t)(cb + i) + 1];
      }
    }
    __syncthreads();
    if constexpr (kDep) {
      for (int i = tid; i < nch; i += blockDim.x) {
        const int pc = sDesc[i].partner;
        if constexpr (kLin) {
          // The tracers around the chunk, moved here (once per chunk, one
          // thread) when this step moves, as for the constant scheme below:
          // the next tracer (the partner's first), whose word the last lane's
          // segment ends at, and the segments just outside the chunk, whose
          // geometry and density the gradients of the first and last lanes'
          // segments need (the same functions as the lanes', so the same bits).
          auto moved = [&](double2 h) -> uint64_t {
            uint64_t w = (uint64_t)__double_as_longlong(h.x);
            if constexpr (kMove) {
              const double e = gather_field_ghost(sE, mesh_pos<PREC>(w, g.inv_dx), g.nc);
              w = drift<PREC>(w, h.y + g.dt * e, g.dt, g.L, g.inv_dx, g.nc);
            }
            return w;
          };
          auto neighbour = [&](uint64_t wa, uint64_t wb, uint64_t cword) {
            const SegGeo sgn = lin_geo<PREC>(wa, wb, g);
            double q;
            if constexpr (SEG) q = PREC == kFP64 ? __longlong_as_double((long long)cword) : (double)(long long)cword;
            else q = PREC == kFP64 ? sDesc[i].q : (double)sDesc[i].q_fix;
            LinNb nb;
            nb.d = sgn.d;
            nb.r = lin_nb_density(sgn.d, lin_density(sgn, q));
            return nb;
          };
          const int2 lk = a.links[cb + i];
          LinNb none;
          none.d = 0.0;
          none.r = lin_nb_density(0.0, 0.0);
          LinNb prev = none, next = none;
          uint64_t wn1 = 0;
          if (pc >= 0) wn1 = moved(a.halo3_in[3 * pc + kHaloFirst]);
          if (lk.x >= 0) {
            const uint64_t wpv = moved(a.halo3_in[3 * (lk.x >> 2) + (lk.x & 3)]);
            const uint64_t w0 = moved(a.halo3_in[3 * (size_t)(cb + i) + kHaloFirst]);
            prev = neighbour(wpv, w0, SEG ? sEdge[2 * i] : 0ull);
          }
          if (pc >= 0 && lk.y >= 0) {
            const uint64_t wn2 = moved(a.halo3_in[3 * (lk.y >> 2) + (lk.y & 3)]);
            next = neighbour(wn1, wn2, SEG ? sEdge[2 * i + 1] : 0ull);
          }
          sNextW[i] = wn1;
          sPrevNb[i] = prev;
          sNextNb[i] = next;
        } else if (pc >= 0) {
          double2 h = (pc == cb + i + 1 && i + 1 < nch) ? sHalo[i] : a.halo_in[pc];
          if constexpr (kMove) {
            // the partner's move, from its state before this step: done here
            // once per chunk by one thread rather than by a whole wavefront
            // for its last lane
            uint64_t pw = (uint64_t)__double_as_longlong(h.x);
            const double e = gather_field_ghost(sE, mesh_pos<PREC>(pw, g.inv_dx), g.nc);
            pw = drift<PREC>(pw, h.y + g.dt * e, g.dt, g.L, g.inv_dx, g.nc);
            h.x = __longlong_as_double((long long)pw);
          }
          sHalo[i] = h;
        }
      }
      __syncthreads();
    }

    // Chunk loop: wave w takes local chunks w, w + nwaves, ...  The loop is
    // unrolled three times with fixed registers per stage, so the state of
    // the next two chunks is in flight while the current one is processed
    // (moving a register whose load is pending would force a wait).
    double ke = 0.0, mom = 0.0, ms = 0.0;
    auto process = [&](int kk, uint64_t xw, double v, uint64_t cw) {
      const ChunkDesc ch = sDesc[kk];
      const int n_valid = __builtin_amdgcn_readfirstlane(ch.n_valid);
      const bool valid = lane < n_valid;
      const size_t s = (size_t)(cb + kk) * kChunk + lane;
      // Per-segment charges: this lane's segment (cw), the one ending at this
      // tracer (cl) and, for linear segments, the next one (cn).
      uint64_t cl = 0, cn = 0;
      if constexpr (kNeedQ) {
        const uint64_t up = lane_up1(cw);
        const uint64_t dn = lane_down1(cw);
        cl = lane == 0 ? sEdge[2 * kk] : up;
        cn = lane == n_valid - 1 ? sEdge[2 * kk + 1] : dn;
      }
      if constexpr (kField) {
        const double e = gather_field_ghost(sE, mesh_pos<PREC>(xw, g.inv_dx), g.nc);
        if constexpr (kKick) {
          const double vk = v - (0.5 * g.dt) * e;
          v = valid ? vk : v;
          a.vs[s] = v;
        } else {
          const double vn = v + g.dt * e;
          double m;
          if constexpr (SEG) {
            m = tracer_mass<PREC>(cl, cw, I.q_unit);
          } else {
            // half of each segment the tracer bounds: the ends of an open
            // sheet bound one
            const bool end = (lane == 0 && (ch.flags & kChunkOpenStart)) || (lane == n_valid - 1 && ch.partner < 0);
            m = end ? 0.5 * ch.q : ch.q;
          }
          const double qv = valid ? m : 0.0;
          // twice the kinetic energy and momentum: the factor 1/2 is applied
          // to the item's sums (a power of two, so the same bits)
          ke += qv * v * vn;
          mom += qv * (v + vn);
          const uint64_t xn = drift<PREC>(xw, vn, g.dt, g.L, g.inv_dx, g.nc);
          xw = valid ? xn : xw;
          v = valid ? vn : v;
          __builtin_nontemporal_store(xw, a.xs + s);
          __builtin_nontemporal_store(v, a.vs + s);
        }
        const double2 hv2 = make_double2(__longlong_as_double((long long)xw), v);
        if constexpr (kLin) {
          const size_t hb = 3 * (size_t)(cb + kk);
          if (lane == 0) a.halo3_out[hb + kHaloFirst] = hv2;
          if (lane == 1) a.halo3_out[hb + kHaloSecond] = hv2;
          if (lane == n_valid - 1) a.halo3_out[hb + kHaloLast] = hv2;
        } else {
          if (lane == 0) a.halo_out[cb + kk] = hv2;
        }
      }
      if constexpr (kDep && kLin) {
        // Every lane computes its own segment's geometry and density; the
        // gradient takes the neighbouring segments' from the lanes next to
        // it (DPP moves), and the first and last lanes take the segments
        // outside the chunk from the staged neighbours.
        const bool last = lane == n_valid - 1;
        const uint64_t dn1 = lane_down1(xw);  // all lanes active: a DPP move reads its neighbour's register
        const uint64_t xp1 = last ? sNextW[kk] : dn1;
        const bool has_seg = valid && (!last || ch.partner >= 0);
        SegGeo sg = lin_geo<PREC>(xw, xp1, g);
        if (!has_seg) sg.d = 0.0;  // a neighbour without a segment drops the gradient
        double q0 = ch.q;
        long long q0_fix = ch.q_fix;
        if constexpr (SEG) {
          if constexpr (PREC == kFP64) q0 = __longlong_as_double((long long)cw);
          else q0_fix = (long long)cw;
        }
        const double r0 = lin_density(sg, PREC == kFP64 ? q0 : (double)q0_fix);
        const double rv = lin_nb_density(sg.d, r0);
        double dm = lane_up1(sg.d), rm = lane_up1(rv);
        double dp = lane_down1(sg.d), rp = lane_down1(rv);
        if (lane == 0) {
          const LinNb nb = sPrevNb[kk];
          dm = nb.d;
          rm = nb.r;
        }
        if (last) {
          const LinNb nb = sNextNb[kk];
          dp = nb.d;
          rp = nb.r;
        }
        if (has_seg) {
          const double grad = lin_gradient(sg.d, dm, rm, dp, rp);
          const double len = fabs(sg.d) * g.dx;
          if (len <= g.half_L) {
            if constexpr (PREC == kFP64) {
              deposit_linear_fp64(__longlong_as_double((long long)xw), sg, grad, q0, r0, g, sP, sD, sR);
            } else {
              deposit_linear_split(split_cell<PREC>(xw), split_frac<PREC>(xw), sg, grad, q0_fix, r0, g, sP, sD,
                                   sR);
            }
          }
          ms = nan_max(ms, len);
        }
      }
      if constexpr (kDep && !kLin) {
        uint64_t pw = lane_down1(xw);
        const bool tail = (lane == n_valid - 1);
        bool has_seg = valid;
        if (tail) {
          if (ch.partner < 0) {
            has_seg = false;  // open sheet: the last tracer ends the chain
          } else {
            pw = (uint64_t)__double_as_longlong(sHalo[kk].x);  // moved at staging when this step moves
          }
        }
        if (has_seg) {
          double len;
          double q0 = ch.q;
          long long q0_fix = ch.q_fix;
          if constexpr (SEG) {
            if constexpr (PREC == kFP64) q0 = __longlong_as_double((long long)cw);
            else q0_fix = (long long)cw;
          }
          if constexpr (ORDER == 2) {
            // first-order weighting: geometry in mesh units, minimum image as
            // for the constant scheme
            double ua, dm;
            if constexpr (PREC == kFP64) {
              const double xa = __longlong_as_double((long long)xw);
              double d = __longlong_as_double((long long)pw) - xa;
              if (d >= g.half_L) d -= g.L;
              else if (d < -g.half_L) d += g.L;
              ua = xa * g.inv_dx;
              dm = d * g.inv_dx;
            } else {
              ua = mesh_pos<PREC>(xw, g.inv_dx);
              dm = min_image_cells(mesh_pos<PREC>(pw, g.inv_dx) - ua, 0.5 * (double)g.nc, (double)g.nc);
            }
            len = fabs(dm) * g.dx;
            if (len <= g.half_L) {
              if constexpr (PREC == kFP64) deposit_cic_fp64(ua, dm, q0, g, sP, sD);
              else deposit_cic_split(ua, dm, q0_fix, g, sP, sD);
            }
          } else {
            if constexpr (PREC == kFP64) {
              len = deposit_fp64(__longlong_as_double((long long)xw), __longlong_as_double((long long)pw), q0, g,
                                 sP, sD);
            } else {
              len = deposit_split<PREC>(xw, pw, q0_fix, g, sP, sD);
            }
          }
          ms = nan_max(ms, len);
        }
      }
    };
    for (int k = wave; k < nch; k += kPrefetch * nwaves) {
#pragma unroll
      for (int j = 0; j < kPrefetch; ++j) {
        if (k + j * nwaves < nch) process(k + j * nwaves, xr[j], vr[j], cr_[j]);
        load_state(k + (j + kPrefetch) * nwaves, xr[j], vr[j], cr_[j]);
      }
    }

    // Work-item partial sums in a fixed order (deterministic for a fixed
    // item decomposition).
    if constexpr (kMove) {
      ke = wave_sum(ke);
      mom = wave_sum(mom);
    }
    if constexpr (kDep) ms = wave_max(ms);
    if (lane == 0) {
      sRed[wave] = ke;
      sRed[16 + wave] = mom;
      sRed[32 + wave] = ms;
    }
    __syncthreads();
    if (tid == 0) {
      double kk = 0.0, m = 0.0, x = 0.0;
      for (int w = 0; w < nwaves; ++w) {
        kk += sRed[w];
        m += sRed[16 + w];
        x = nan_max(x, sRed[32 + w]);
      }
      if constexpr (kMove) {
        a.partials[it].ke = 0.5 * kk;
        a.partials[it].mom = 0.5 * m;
      }
      if constexpr (kDep) a.partials[it].maxseg = x;
    }
    if constexpr (kDep) {
      const int64_t roff = I.mesh_off + (int64_t)(it % a.rep) * a.rep_stride;
      acc_t *gP = reinterpret_cast<acc_t *>(a.meshP) + roff;
      acc_t *gD = reinterpret_cast<acc_t *>(a.meshD) + roff;
      for (int i = tid; i < g.nc; i += blockDim.x) {
        const acc_t p = sP[i];
        const acc_t d = sD[i];
        if (p != (acc_t)0) {
          if constexpr (PREC == kFP64) unsafeAtomicAdd(gP + i, p);
          else atomicAdd(gP + i, p);
        }
        if (d != (acc_t)0) {
          if constexpr (PREC == kFP64) unsafeAtomicAdd(gD + i, d);
          else atomicAdd(gD + i, d);
        }
        if constexpr (kLin) {
          acc_t *gR = reinterpret_cast<acc_t *>(a.meshR) + roff;
          const acc_t r = sR[i];
          if (r != (acc_t)0) {
            if constexpr (PREC == kFP64) unsafeAtomicAdd(gR + i, r);
            else atomicAdd(gR + i, r);
          }
        }
      }
    }
    __syncthreads();
  }
}

size_t tracer_lds_size(int prec, int order, bool seg, int mesh_cells, int tile_cap) {
  // the accumulators are 8 bytes in every precision
  if (order == 1)
    return seg ? tracer_lds_bytes<double, 1, true>(mesh_cells, tile_cap)
               : tracer_lds_bytes<double, 1, false>(mesh_cells, tile_cap);
  return seg ? tracer_lds_bytes<double, 0, true>(mesh_cells, tile_cap)
             : tracer_lds_bytes<double, 0, false>(mesh_cells, tile_cap);
}

// ---------------------------------------------------------------------------
// Deposit-only kernel (constant segments, face-crossing form)
// ---------------------------------------------------------------------------
// A deposit that does not also move the tracers reads 8 bytes per tracer, so
// its pace is set by the arithmetic per tracer, not by HBM.  On a sheet with
// several tracers per cell most segments cross no cell face: all they need is
// their length (the max-segment diagnostic) and their charge, which the
// chunk's running sum carries to the next crossing.  So the wavefront does
// only that per tracer, and appends every segment whose two ends lie in
// different cells to a per-wavefront ring in LDS; the face geometry of the
// queued segments (a division each) runs 64 at a time, with every lane busy.
// The sum over crossings and chunk ends is the same as in the per-chunk form
// above, term by term.

constexpr int kDepQueue = 64;      // ring entries per wavefront (drained before it would overflow)
constexpr int kDepPrefetch = 6;    // chunks in flight per wavefront

// The word and cell (plus one) of the tracer after a chunk.
struct alignas(16) DepHalo {
  uint64_t w;
  int32_t c;
  int32_t pad;
};

__host__ __device__ constexpr size_t dep_lds_offset_queue(int mesh_cells, int tile_cap) {
  // P, D; descriptors; halos
  return (size_t)2 * mesh_cells * 8 + (size_t)tile_cap * (sizeof(ChunkDesc) + sizeof(DepHalo));
}

// The ring of one wavefront is three arrays (kept apart so that the lanes of
// one queue write or read touch consecutive LDS words): the segment's two
// state words; the cells of its ends (plus one, 16 bits each) and its local
// chunk and lane; with per-segment charges, the chunk's charge before it and
// its own.  24 (40) bytes per entry: a 512-thread workgroup of a 1024-cell
// mesh and 256 chunks per item takes 40 KB, four workgroups per CU.  At the
// end of an item each wavefront's ring holds its segment-length maximum.
template <bool SEG>
__host__ __device__ constexpr size_t dep_lds_bytes(int mesh_cells, int tile_cap, int nwaves) {
  return dep_lds_offset_queue(mesh_cells, tile_cap) + (size_t)nwaves * kDepQueue * (16 + 8 + (SEG ? 16 : 0));
}

// Length of the segment between two state words (minimum image), in the same
// rounding as the per-segment deposit.
template <int PREC>
__device__ __forceinline__ double seg_length(uint64_t wa, uint64_t wb, const Geo &g) {
  // min(|d|, period - |d|) is |d| up to half a period and the other image
  // beyond, and propagates NaN
  if constexpr (PREC == kFP64) {
    const double ad = fabs(__longlong_as_double((long long)wb) - __longlong_as_double((long long)wa));
    return fmin(ad, g.L - ad);
  } else {
    const double nc = (double)g.nc;
    const double ad = fabs(mesh_pos<PREC>(wb, g.inv_dx) - mesh_pos<PREC>(wa, g.inv_dx));
    return fmin(ad, nc - ad) * g.dx;
  }
}

// ceil(x / dx), the raw cell of a tracer plus one (0 .. nc).  x * inv_dx
// is within 2^-50 relative of the rounded quotient, and |u| <= nc, so when
// u's distance to a whole number exceeds tol = (nc + 1) 2^-49 both have the
// same ceiling; otherwise the division decides.
template <int PREC>
__device__ __forceinline__ int point_cell_up(uint64_t w, const Geo &g, double tol, double tol_hi) {
  if constexpr (PREC == kFP64) {
    const double x = __longlong_as_double((long long)w);
    const double u = x * g.inv_dx;
    const double c = ceil(u);
    const double r = c - u;
    if (r > tol && r < tol_hi) return (int)c;
    return (int)ceil(x / g.dx);
  } else {
    return split_frac<PREC>(w) == 0.0 ? split_cell<PREC>(w) : split_cell<PREC>(w) + 1;
  }
}

// Without per-segment charges the kernel is held to 64 VGPRs, so that the
// eight wavefronts of each of four workgroups per CU all fit.
template <int PREC, bool SEG>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(SEG ? 4 : 8)))
k_deposit_faces(TracerArgs a) {
  using acc_t = typename std::conditional<PREC == kFP64, double, unsigned long long>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  if (a.gate != nullptr && *a.gate <= 0) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nwaves = blockDim.x >> 6;
  acc_t *sP = reinterpret_cast<acc_t *>(smem);
  acc_t *sD = sP + a.mesh_cells;
  ChunkDesc *sDesc = reinterpret_cast<ChunkDesc *>(sD + a.mesh_cells);
  DepHalo *sHalo = reinterpret_cast<DepHalo *>(sDesc + a.tile_cap);
  ulonglong2 *const qBase = reinterpret_cast<ulonglong2 *>(smem + dep_lds_offset_queue(a.mesh_cells, a.tile_cap));
  ulonglong2 *qW = qBase;
  int2 *qC = reinterpret_cast<int2 *>(qW + nwaves * kDepQueue) + wave * kDepQueue;
  ulonglong2 *qS = reinterpret_cast<ulonglong2 *>(qC + (nwaves - wave) * kDepQueue) + wave * kDepQueue;  // SEG
  qW += wave * kDepQueue;
  const int n_items = *a.n_items;

  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const Item item = a.items[it];
    if (item.inst < 0) continue;  // freed slot
    const InstDesc &I = a.inst[item.inst];
    if (a.respect_active && !I.active) continue;
    Geo g;
    g.L = I.L;
    g.half_L = I.half_L;
    g.dx = I.dx;
    g.inv_dx = I.inv_dx;
    g.dt = I.dt;
    g.nc = I.n_cells;
    const int cb = item.chunk_begin;
    const int nch = item.chunk_end - item.chunk_begin;

    for (int i = tid; i < g.nc; i += blockDim.x) {
      sP[i] = (acc_t)0;
      sD[i] = (acc_t)0;
    }
    // descriptors, and the word and cell of the tracer after each chunk
    for (int i = tid; i < nch; i += blockDim.x) {
      sDesc[i] = a.chunks[cb + i];
      const int pc = a.chunks[cb + i].partner;
      if (pc >= 0) {
        const uint64_t w = (uint64_t)__double_as_longlong(a.halo_in[pc].x);
        sHalo[i].w = w;
        sHalo[i].c = point_cell_up<PREC>(w, g, (double)(g.nc + 1) * 0x1p-49, 1.0 - (double)(g.nc + 1) * 0x1p-49);
      }
    }
    __syncthreads();

    double ms = 0.0;
    bool bad = false;             // a non-finite segment length (reported as NaN)
    int q_head = 0, q_count = 0;  // the wavefront's ring (uniform)

    // The n <= 64 oldest queued segments, one per lane: the faces each
    // crosses, and for the last segment of a chunk the chunk's charge where
    // it ends.
    auto drain = [&](int n) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (lane < n) {
        const int e = (q_head + lane) & (kDepQueue - 1);
        const ulonglong2 w = qW[e];
        const int2 c = qC[e];
        const int pa = (c.x & 0xffff) - 1;
        const int pb = ((c.x >> 16) & 0xffff) - 1;
        const ChunkDesc &d = sDesc[(c.y >> 6) & 0x3fff];
        const int ln = c.y & 63;
        // the chunk's last segment: its last lane, or the one before for an
        // open sheet's end
        const bool end = ln == (d.partner < 0 ? d.n_valid - 2 : d.n_valid - 1);
        acc_t S, ql;
        if constexpr (SEG) {
          const ulonglong2 sq = qS[e];
          if constexpr (PREC == kFP64) {
            S = __longlong_as_double((long long)sq.x);
            ql = __longlong_as_double((long long)sq.y);
          } else {
            S = sq.x;
            ql = sq.y;
          }
        } else {
          ql = PREC == kFP64 ? (acc_t)d.q : (acc_t)d.q_fix;
          S = ql * (acc_t)ln;
        }
        acc_t eb = (acc_t)0;  // added to the cell where the segment ends
        bool add_b = end;
        if (pa != pb) {
          double len;
          const Crossings<acc_t> cr = face_crossings<PREC, acc_t>(w.x, w.y, pa, pb, ql, S, g, &len);
          if (cr.hi >= cr.lo) {
            lds_add(sP + wrap_cell(pa, g.nc), cr.cf);
            if (cr.hi > cr.lo) add_run(sD, cr.lo, cr.hi - 1, cr.w, g.nc);
            eb = (acc_t)(0 - cr.cl);
            add_b = true;
          }
        }
        if (end) eb += S + ql;
        if (add_b) lds_add(sP + wrap_cell(pb, g.nc), eb);
      }
      q_head = (q_head + n) & (kDepQueue - 1);
      q_count -= n;
      // the entries just read are written again by the next appends
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };

    auto load_state = [&](int kk, uint64_t &xw, uint64_t &cw) {
      const size_t s = kk < nch ? (size_t)(cb + kk) * kChunk + lane : (size_t)cb * kChunk;  // as in k_tracers
      xw = __builtin_nontemporal_load(a.xs + s);
      if constexpr (SEG) cw = a.segq[s];
    };
    const double tol = (double)(g.nc + 1) * 0x1p-49, tol_hi = 1.0 - tol;
    auto process = [&](int kk, uint64_t xw, uint64_t cw) {
      const int n_valid = __builtin_amdgcn_readfirstlane(sDesc[kk].n_valid);
      const bool open_end = __builtin_amdgcn_readfirstlane(sDesc[kk].partner) < 0;
      const int last = open_end ? n_valid - 2 : n_valid - 1;  // lane of the chunk's last segment
      const bool has_seg = lane <= last;
      // the segment's far end: the next lane, or past the chunk the partner's
      // first tracer
      uint64_t xb = lane_down1(xw);
      const int ca = point_cell_up<PREC>(xw, g, tol, tol_hi);
      int cb1 = lane_down1(ca);
      if (!open_end) {
        const bool tail = lane == n_valid - 1;
        const DepHalo h = sHalo[kk];
        xb = tail ? h.w : xb;
        cb1 = tail ? h.c : cb1;
      }
      if (has_seg) {
        const double len = seg_length<PREC>(xw, xb, g);
        ms = fmax(ms, len);
        bad = bad || len != len;
      }
      // queue the segments whose ends lie in different cells, and the
      // chunk's last segment
      const bool rec = has_seg && (ca != cb1 || lane == last);
      acc_t S = (acc_t)0, ql = (acc_t)0;
      if constexpr (SEG) {
        if (has_seg) ql = PREC == kFP64 ? (acc_t)__longlong_as_double((long long)cw) : (acc_t)cw;
        S = wave_exclusive_sum(ql);
      }
      const uint64_t mask = __builtin_amdgcn_ballot_w64(rec);
      if (mask) {
        const int n_new = __builtin_popcountll(mask);
        if (q_count + n_new > kDepQueue) drain(q_count);
        if (rec) {
          const int rank =
              __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
          const int e = (q_head + q_count + rank) & (kDepQueue - 1);
          qW[e] = make_ulonglong2(xw, xb);
          qC[e] = make_int2(ca | (cb1 << 16), (kk << 6) | lane);
          if constexpr (SEG) {
            if constexpr (PREC == kFP64) {
              qS[e] = make_ulonglong2((uint64_t)__double_as_longlong(S), (uint64_t)__double_as_longlong(ql));
            } else {
              qS[e] = make_ulonglong2((uint64_t)S, (uint64_t)ql);
            }
          }
        }
        q_count += n_new;
      }
    };

    uint64_t xr[kDepPrefetch], cr_[kDepPrefetch];
#pragma unroll
    for (int j = 0; j < kDepPrefetch; ++j) {
      xr[j] = cr_[j] = 0;
      load_state(wave + j * nwaves, xr[j], cr_[j]);
      __builtin_amdgcn_sched_barrier(0);  // stage order, as in the loop
    }
    for (int k = wave; k < nch; k += kDepPrefetch * nwaves) {
#pragma unroll
      for (int j = 0; j < kDepPrefetch; ++j) {
        if (k + j * nwaves < nch) process(k + j * nwaves, xr[j], cr_[j]);
        load_state(k + (j + kDepPrefetch) * nwaves, xr[j], cr_[j]);
      }
    }
    if (q_count > 0) drain(q_count);

    if (bad) ms = __longlong_as_double(0x7ff8000000000000ll);
    ms = wave_max(ms);
    if (lane == 0) reinterpret_cast<double *>(qW)[0] = ms;  // the ring is empty now
    __syncthreads();
    if (tid == 0) {
      double x = 0.0;
      for (int w = 0; w < nwaves; ++w) x = nan_max(x, reinterpret_cast<const double *>(qBase + w * kDepQueue)[0]);
      a.partials[it].maxseg = x;
    }
    const int64_t roff = I.mesh_off + (int64_t)(it % a.rep) * a.rep_stride;
    acc_t *gP = reinterpret_cast<acc_t *>(a.meshP) + roff;
    acc_t *gD = reinterpret_cast<acc_t *>(a.meshD) + roff;
    for (int i = tid; i < g.nc; i += blockDim.x) {
      const acc_t p = sP[i];
      const acc_t d = sD[i];
      if (p != (acc_t)0) {
        if constexpr (PREC == kFP64) unsafeAtomicAdd(gP + i, p);
        else atomicAdd(gP + i, p);
      }
      if (d != (acc_t)0) {
        if constexpr (PREC == kFP64) unsafeAtomicAdd(gD + i, d);
        else atomicAdd(gD + i, d);
      }
    }
    __syncthreads();
  }
}

// CELLS: cells per thread the solve is unrolled for (at least the pool's
// largest mesh over kSolveThreads; the unused ones add exact zeros, so every
// instance gives the same bits).
template <int PREC, int CELLS, int REP>
__global__ void __launch_bounds__(kSolveThreads) k_solve(SolveArgs a) {
  using acc_t = typename std::conditional<PREC == kFP64, double, long long>::type;
  __shared__ double sWd[4];
  if (a.gate != nullptr && *a.gate <= 0) return;
  const int slot = a.slot_list ? a.slot_list[blockIdx.x] : (int)blockIdx.x;
  InstDesc *Ip = a.inst + slot;
  if (!Ip->live) return;
  if (a.respect_active && !Ip->active) return;
  const int tid = threadIdx.x;
  const int2 si = a.slot_items[slot];
  const int item_begin = si.x, item_count = si.y;
  const SlotConst kc = slot_const(*Ip);
  acc_t *gP = reinterpret_cast<acc_t *>(a.meshP) + kc.mesh_off;
  acc_t *gD = reinterpret_cast<acc_t *>(a.meshD) + kc.mesh_off;
  acc_t pv[CELLS], dv[CELLS];
  solve_take<PREC, CELLS, REP>(kc, gP, gD, a.rep_stride, pv, dv);  // in flight with the partial loads below

  // 1. work-item partials, in item order: each thread sums items tid,
  // tid + 256, ... (loads issued four at a time), then the wavefront and
  // workgroup sums, all three in one pass
  __shared__ double sMom[4], sMs[4];
  constexpr int kU = 4;
  double ke = 0.0, mom = 0.0, ms = 0.0;
  for (int i0 = tid; i0 < item_count; i0 += kU * kSolveThreads) {
    Partial pr[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u * kSolveThreads;
      if (i < item_count) pr[u] = a.partials[item_begin + i];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (i0 + u * kSolveThreads < item_count) {
        ke += pr[u].ke;
        mom += pr[u].mom;
        ms = nan_max(ms, pr[u].maxseg);
      }
    }
  }
  ke = wave_sum(ke);
  mom = wave_sum(mom);
  ms = wave_max(ms);
  const int wave = tid >> 6;
  if ((tid & 63) == 0) {
    sWd[wave] = ke;
    sMom[wave] = mom;
    sMs[wave] = ms;
  }
  __syncthreads();
  ke = sWd[0] + sWd[1] + sWd[2] + sWd[3];
  mom = sMom[0] + sMom[1] + sMom[2] + sMom[3];
  ms = nan_max(nan_max(sMs[0], sMs[1]), nan_max(sMs[2], sMs[3]));
  acc_t *gRamp = (a.order == 1 && a.meshR) ? reinterpret_cast<acc_t *>(a.meshR) + kc.mesh_off : nullptr;
  solve_slot<PREC, CELLS, REP>(a, slot, kc, Ip->step, Ip->flags, pv, dv, gRamp, ke, mom, ms,
                          (double *)nullptr, true);
}

// ---------------------------------------------------------------------------
// Resident small simulation
// ---------------------------------------------------------------------------
// A simulation of at most kResidentChunks chunks runs many steps in one
// launch of one workgroup: its tracers stay in registers (each of the W
// wavefronts owns chunks w, w + W, ...), the mesh accumulators and the field in LDS, and
// each step is push, deposit and solve separated by workgroup barriers.  The
// arithmetic is that of the fused step (same move, same segment deposit,
// same solve code), so only the order of the floating-point sums of the
// deposit and of the kinetic-energy and momentum diagnostics can differ; the
// split forms give the same bits.  Small simulations are latency-bound: this
// replaces two kernel launches per step with one launch per call.

constexpr int kResidentChunks = 32;  // chunks (2048 tracer slots) a resident launch holds

// P, D, E; then (16-byte aligned) descriptors, new first-tracer words and
// charge edges
__host__ __device__ constexpr size_t resident_desc_offset(int n_cells) {
  return ((size_t)n_cells * 24 + 15) & ~(size_t)15;
}
__host__ __device__ constexpr size_t resident_lds_bytes(int n_cells, bool seg) {
  return resident_desc_offset(n_cells) + (size_t)kResidentChunks * (sizeof(ChunkDesc) + 8 + (seg ? 16 : 0));
}

// A workgroup barrier that orders LDS only: global stores in flight (the
// diagnostics rows) are not waited for.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int PREC, bool SEG, int CELLS, int NT>
__global__ void __launch_bounds__(NT) k_resident(TracerArgs a, SolveArgs sa, int chunk_begin, int n_chunks,
                                                 int64_t n_steps) {
  using acc_t = typename std::conditional<PREC == kFP64, double, unsigned long long>::type;
  // NT / 64 wavefronts share the chunks (wave w takes w, w + waves, ...)
  constexpr int kResidentWaves = NT / kChunk;
  constexpr int kResidentPerWave = kResidentChunks / kResidentWaves;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double sRed[3 * kResidentWaves];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int slot = 0;
  const InstDesc *Ip = a.inst + slot;
  const int nc = Ip->n_cells;
  acc_t *sP = reinterpret_cast<acc_t *>(smem);
  acc_t *sD = sP + nc;
  double *sE = reinterpret_cast<double *>(sD + nc);
  ChunkDesc *sDesc = reinterpret_cast<ChunkDesc *>(smem + resident_desc_offset(nc));
  uint64_t *sHx = reinterpret_cast<uint64_t *>(sDesc + kResidentChunks);
  uint64_t *sEdge = sHx + kResidentChunks;  // per-segment charges
  Geo g;
  g.L = Ip->L;
  g.half_L = Ip->half_L;
  g.dx = Ip->dx;
  g.inv_dx = Ip->inv_dx;
  g.dt = Ip->dt;
  g.nc = nc;
  const double q_unit = Ip->q_unit;
  const SlotConst kc = slot_const(*Ip);
  int64_t step_now = Ip->step;
  int flags = Ip->flags;

  for (int i = tid; i < nc; i += NT) {
    sP[i] = (acc_t)0;
    sD[i] = (acc_t)0;
    sE[i] = a.meshE[Ip->mesh_off + i];
  }
  for (int i = tid; i < n_chunks; i += NT) {
    sDesc[i] = a.chunks[chunk_begin + i];
    if constexpr (SEG) {
      sEdge[2 * i] = a.cedge[2 * (size_t)(chunk_begin + i)];
      sEdge[2 * i + 1] = a.cedge[2 * (size_t)(chunk_begin + i) + 1];
    }
  }
  // the wavefront's chunks, in registers for the whole launch
  uint64_t xr[kResidentPerWave], cwr[kResidentPerWave];
  double vr[kResidentPerWave];
#pragma unroll
  for (int j = 0; j < kResidentPerWave; ++j) {
    const int c = wave + j * kResidentWaves;
    xr[j] = cwr[j] = 0;
    vr[j] = 0.0;
    if (c < n_chunks) {
      const size_t sidx = (size_t)(chunk_begin + c) * kChunk + lane;
      xr[j] = a.xs[sidx];
      vr[j] = a.vs[sidx];
      if constexpr (SEG) cwr[j] = a.segq[sidx];
    }
  }
  __syncthreads();

  for (int64_t step = 0; step < n_steps; ++step) {
    // push: gather, kick, drift; the first tracer of each chunk is
    // published for the segment that ends at it
    double ke = 0.0, mom = 0.0, ms = 0.0;
#pragma unroll
    for (int j = 0; j < kResidentPerWave; ++j) {
      const int c = wave + j * kResidentWaves;
      if (c < n_chunks) {
        const ChunkDesc &ch = sDesc[c];
        const int n_valid = __builtin_amdgcn_readfirstlane(ch.n_valid);
        const bool valid = lane < n_valid;
        uint64_t xw = xr[j];
        double v = vr[j];
        const double e = gather_field(sE, mesh_pos<PREC>(xw, g.inv_dx), g.nc);
        const double vn = v + g.dt * e;
        double m;
        if constexpr (SEG) {
          const uint64_t up = lane_up1(cwr[j]);
          m = tracer_mass<PREC>(lane == 0 ? sEdge[2 * c] : up, cwr[j], q_unit);
        } else {
          const bool end =
              (lane == 0 && (ch.flags & kChunkOpenStart)) || (lane == n_valid - 1 && ch.partner < 0);
          m = end ? 0.5 * ch.q : ch.q;
        }
        const double qv = valid ? m : 0.0;
        ke += qv * v * vn;  // twice the kinetic energy and momentum, halved below
        mom += qv * (v + vn);
        const uint64_t xn = drift<PREC>(xw, vn, g.dt, g.L, g.inv_dx, g.nc);
        xr[j] = valid ? xn : xw;
        vr[j] = valid ? vn : v;
        if (lane == 0) sHx[c] = xr[j];
      }
    }
    lds_barrier();
    // deposit of the moved segments into the LDS mesh
#pragma unroll
    for (int j = 0; j < kResidentPerWave; ++j) {
      const int c = wave + j * kResidentWaves;
      if (c < n_chunks) {
        const ChunkDesc &ch = sDesc[c];
        const int n_valid = __builtin_amdgcn_readfirstlane(ch.n_valid);
        const uint64_t xw = xr[j];
        uint64_t pw = lane_down1(xw);
        bool has_seg = lane < n_valid;
        if (lane == n_valid - 1) {
          if (ch.partner < 0) has_seg = false;  // open sheet: the last tracer ends the chain
          else pw = sHx[ch.partner - chunk_begin];
        }
        if (has_seg) {
          double len;
          if constexpr (PREC == kFP64) {
            const double q0 = SEG ? __longlong_as_double((long long)cwr[j]) : ch.q;
            len = deposit_fp64(__longlong_as_double((long long)xw), __longlong_as_double((long long)pw), q0, g,
                               sP, sD);
          } else {
            const long long q0 = SEG ? (long long)cwr[j] : ch.q_fix;
            len = deposit_split<PREC>(xw, pw, q0, g, sP, sD);
          }
          ms = nan_max(ms, len);
        }
      }
    }
    ke = wave_sum(ke);
    mom = wave_sum(mom);
    ms = wave_max(ms);
    if (lane == 0) {
      sRed[wave] = ke;
      sRed[kResidentWaves + wave] = mom;
      sRed[2 * kResidentWaves + wave] = ms;
    }
    lds_barrier();
    ke = mom = ms = 0.0;
    for (int w = 0; w < kResidentWaves; ++w) {
      ke += sRed[w];
      mom += sRed[kResidentWaves + w];
      ms = nan_max(ms, sRed[2 * kResidentWaves + w]);
    }
    ke *= 0.5;
    mom *= 0.5;
    // solve (clears the accumulators, leaves the field in sE; in global
    // memory too after the last step)
    using sacc_t = typename std::conditional<PREC == kFP64, double, long long>::type;
    sacc_t pv[CELLS], dv[CELLS];
    solve_take<PREC, CELLS, 1>(kc, sP, sD, 0, pv, dv);
    flags = solve_slot<PREC, CELLS>(sa, slot, kc, step_now, flags, pv, dv, (acc_t *)nullptr, ke, mom, ms, sE,
                                    step == n_steps - 1);
    step_now += 1;
    lds_barrier();
  }

  // state and first-tracer halos back to global memory
#pragma unroll
  for (int j = 0; j < kResidentPerWave; ++j) {
    const int c = wave + j * kResidentWaves;
    if (c < n_chunks) {
      const size_t sidx = (size_t)(chunk_begin + c) * kChunk + lane;
      a.xs[sidx] = xr[j];
      a.vs[sidx] = vr[j];
      if (lane == 0) a.halo_out[chunk_begin + c] = make_double2(__longlong_as_double((long long)xr[j]), vr[j]);
    }
  }
}

// ---------------------------------------------------------------------------
// Ingest / extract / utilities
// ---------------------------------------------------------------------------
template <int PREC>
__global__ void __launch_bounds__(256) k_ingest(IngestArgs a) {
  const int cl = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (a.state != nullptr && (a.state[kRefInserted] <= 0 || cl >= a.state[kRefChunks])) return;
  if (cl >= a.n_chunks) return;
  const int lane = threadIdx.x & 63;
  const int c = a.chunk_begin + cl;
  const ChunkDesc ch = a.chunks[c];
  const InstDesc &I = a.inst[ch.inst];
  const size_t s = (size_t)c * kChunk + lane;
  uint64_t w = 0, cw = 0;
  double v = 0.0;
  if (lane < ch.n_valid) {
    const int64_t src = a.chunk_in_off[cl] + lane;
    v = a.v_in[src];
    if (a.w_in) {
      w = a.w_in[src];  // a state word of this pool (re-layout)
    } else {
      const double x = wrap_into_box(a.x_in[src], I.L);
      if constexpr (PREC == kFP64) {
        w = (uint64_t)__double_as_longlong(x);
      } else {
        const double u = x * I.inv_dx;
        const double f = floor(u);
        w = split_word<PREC>((int)f, u - f, I.n_cells);
      }
    }
    if (a.segq) {
      if (a.cw_in) {
        cw = a.cw_in[src];
      } else if (a.c_in) {
        if constexpr (PREC == kFP64) cw = (uint64_t)__double_as_longlong(a.c_in[src]);
        else cw = (uint64_t)llrint(a.c_in[src] * a.q_scale);
      } else {
        if constexpr (PREC == kFP64) cw = (uint64_t)__double_as_longlong(ch.q);
        else cw = (uint64_t)ch.q_fix;
      }
      if (lane == ch.n_valid - 1 && ch.partner < 0) cw = 0;  // an open sheet's last tracer starts no segment
    }
  }
  a.xs[s] = w;
  a.vs[s] = v;
  if (a.segq) a.segq[s] = cw;
  const double2 hv = make_double2(__longlong_as_double((long long)w), v);
  if (lane == 0) a.halo[c] = hv;
  if (a.halo3) {
    if (lane == 0) a.halo3[3 * (size_t)c + kHaloFirst] = hv;
    if (lane == 1) a.halo3[3 * (size_t)c + kHaloSecond] = hv;
    if (lane == ch.n_valid - 1) a.halo3[3 * (size_t)c + kHaloLast] = hv;
  }
}

template <int PREC>
__global__ void __launch_bounds__(256) k_extract(ExtractArgs a) {
  const int cl = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (cl >= a.n_chunks) return;
  const int lane = threadIdx.x & 63;
  const int c = a.chunk_begin + cl;
  const ChunkDesc ch = a.chunks[c];
  if (lane >= ch.n_valid) return;
  const InstDesc &I = a.inst[ch.inst];
  const size_t s = (size_t)c * kChunk + lane;
  const int64_t dst = a.chunk_in_off[cl] + lane;
  const uint64_t w = a.xs[s];
  double x;
  if constexpr (PREC == kFP64) {
    x = __longlong_as_double((long long)w);
  } else {
    x = mesh_pos<PREC>(w, I.inv_dx) * I.dx;
  }
  a.x_out[dst] = x;
  a.v_out[dst] = a.vs[s];
  if (a.c_out) a.c_out[dst] = charge_value<PREC>(a.segq[s], I.q_unit);
}

// Charge edges of a chunk range (one thread per chunk): the charge of the
// segment ending at the chunk's first tracer and of the segment starting at
// its partner tracer.
__global__ void __launch_bounds__(256) k_charge_edges(const ChunkDesc *chunks, const int64_t *prev_slot,
                                                      const uint64_t *segq, uint64_t *cedge, int32_t chunk_begin,
                                                      int32_t n_chunks, const int32_t *state) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (state != nullptr && (state[kRefInserted] <= 0 || i >= state[kRefChunks])) return;
  if (i >= n_chunks) return;
  const int c = chunk_begin + i;
  const int64_t pv = prev_slot[c];
  const int32_t pc = chunks[c].partner;
  cedge[2 * (size_t)c] = pv >= 0 ? segq[pv] : 0ull;
  cedge[2 * (size_t)c + 1] = pc >= 0 ? segq[(size_t)pc * kChunk] : 0ull;
}

// Refinement, one wavefront per chunk.  Each valid lane looks at its segment
// (to the next tracer, or for the last lane to the partner tracer; none at
// an open sheet's end) and marks it when its minimum-image length exceeds
// l_max.
template <int PREC>
__device__ __forceinline__ bool refine_segment(const RefineArgs &a, const ChunkDesc &ch, const InstDesc &I,
                                               int lane, uint64_t w, uint64_t &wn, double &vn, double &du) {
  bool has = lane < ch.n_valid;
  if (lane == ch.n_valid - 1) {
    if (ch.partner >= 0) {
      wn = a.xs[(size_t)ch.partner * kChunk];
      vn = a.vs[(size_t)ch.partner * kChunk];
    } else {
      has = false;
    }
  }
  if (!has) return false;
  double len;
  if constexpr (PREC == kFP64) {
    const double xa = __longlong_as_double((long long)w);
    double d = __longlong_as_double((long long)wn) - xa;
    if (d >= I.half_L) d -= I.L;
    else if (d < -I.half_L) d += I.L;
    du = d;
    len = fabs(d);
  } else {
    const double ua = mesh_pos<PREC>(w, I.inv_dx);
    const double dm = min_image_cells(mesh_pos<PREC>(wn, I.inv_dx) - ua, 0.5 * (double)I.n_cells, (double)I.n_cells);
    du = dm;
    len = fabs(dm) * I.dx;
  }
  return len > a.l_max;
}

template <int PREC>
__global__ void __launch_bounds__(256) k_refine_mark(RefineArgs a) {
  const int cl = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (a.state != nullptr && (a.state[kRefHalt] != 0 || cl >= a.state[kRefChunks])) return;
  if (cl >= a.n_chunks) return;  // uniform per wavefront
  const int lane = threadIdx.x & 63;
  const int c = a.chunk_begin + cl;
  const ChunkDesc ch = a.chunks[c];
  const InstDesc &I = a.inst[ch.inst];
  const size_t s = (size_t)c * kChunk + lane;
  const uint64_t w = a.xs[s];
  uint64_t wn = lane_down1(w);
  double vn = 0.0, du = 0.0;
  const bool flag = refine_segment<PREC>(a, ch, I, lane, w, wn, vn, du);
  const uint64_t mask = __ballot(flag);
  if (lane == 0) {
    a.cnt[cl] = __popcll(mask);
    a.mask[cl] = mask;
  }
}

// Writes the chunk's tracers to the flat output, each marked one followed by
// the centre of its segment: mean velocity, and the charge split in halves
// (fixed point: the halves differ by at most one unit and sum exactly).
template <int PREC>
__global__ void __launch_bounds__(256) k_refine_scatter(RefineArgs a) {
  const int cl = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (a.state != nullptr && (a.state[kRefInserted] <= 0 || cl >= a.state[kRefChunks])) return;
  if (cl >= a.n_chunks) return;  // uniform per wavefront
  const int lane = threadIdx.x & 63;
  const int c = a.chunk_begin + cl;
  const ChunkDesc ch = a.chunks[c];
  const InstDesc &I = a.inst[ch.inst];
  const size_t s = (size_t)c * kChunk + lane;
  const uint64_t w = a.xs[s];
  const double v = a.vs[s];
  const uint64_t cq = a.segq[s];
  uint64_t wn = lane_down1(w);
  double vn = lane_down1(v);
  double du = 0.0;
  refine_segment<PREC>(a, ch, I, lane, w, wn, vn, du);
  // the marking pass decided (the host sized the output from its counts)
  const uint64_t mask = a.mask[cl];
  const bool flag = ((mask >> lane) & 1ull) != 0;
  if (lane >= ch.n_valid) return;
  const int64_t out = a.out_off[cl] + lane + __popcll(mask & ((1ull << lane) - 1ull));
  uint64_t c0 = cq;
  if (flag) {
    uint64_t c1, wm;
    if constexpr (PREC == kFP64) {
      const double h = 0.5 * __longlong_as_double((long long)cq);
      c0 = c1 = (uint64_t)__double_as_longlong(h);
      const double xa = __longlong_as_double((long long)w);
      wm = (uint64_t)__double_as_longlong(wrap_into_box(xa + 0.5 * du, I.L));
    } else {
      const long long q = (long long)cq;
      const long long q1 = q >> 1;
      c0 = (uint64_t)(q - q1);
      c1 = (uint64_t)q1;
      wm = advance_split<PREC>(w, 0.5 * du, I.n_cells);
    }
    a.w_out[out + 1] = wm;
    a.v_out[out + 1] = 0.5 * (v + vn);
    a.c_out[out + 1] = c1;
  }
  a.w_out[out] = w;
  a.v_out[out] = v;
  a.c_out[out] = c0;
}

// Device re-layout after a marking pass (one simulation; the host's layout
// building done on the device, so that refining steps need no round trip).
// The plan, one workgroup: the flat staging offset of every chunk (the old
// tracers plus the inserted ones, sheet-major), each sheet's new tracer
// count, its first chunk in the new layout and its first staging index, and
// the capacity check.  A pass that would exceed the capacity inserts nothing
// and halts the simulation (inactive; the host reports it).
__global__ void __launch_bounds__(1024) k_refine_plan(RefinePlanArgs a) {
  __shared__ long long sW[16];
  __shared__ long long sTk[16];
  __shared__ long long sTot[2];
  __shared__ int sOver;
  const int tid = threadIdx.x;
  const int nth = blockDim.x;
  int32_t *st = a.state;
  if (st[kRefHalt] != 0) {
    if (tid == 0) st[kRefInserted] = 0;
    return;
  }
  if (tid == 0) sOver = 0;
  const int n = st[kRefChunks];
  // Each wavefront takes a contiguous range of chunks and walks it 64 chunks
  // (one per lane, coalesced) at a time, kB groups of loads in flight
  // together: a wavefront scan gives each chunk its offset within the range
  // (written to out_off), the ranges' totals are scanned across the
  // wavefronts, and a second coalesced pass adds each range's base.
  const int lane = tid & 63, wave = tid >> 6, nw = nth >> 6;
  const int per_w = (n + nw - 1) / nw;
  const int w0 = min(n, wave * per_w), w1 = min(n, w0 + per_w);
  constexpr int kB = 4;
  long long run_v = 0, run_k = 0;  // the range so far (every lane)
  for (int gb = w0; gb < w1; gb += kB * 64) {
    long long kv[kB], vv[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int c = gb + u * 64 + lane;
      const int cc = min(c, w1 - 1);
      const long long k = a.cnt[cc];
      const long long v = (long long)a.chunks[a.chunk_begin + cc].n_valid + k;
      kv[u] = c < w1 ? k : 0;
      vv[u] = c < w1 ? v : 0;
    }
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int c = gb + u * 64 + lane;
      const long long iv = wave_incl_scan(vv[u], [](long long x, long long y) { return x + y; });
      const long long ik = wave_incl_scan(kv[u], [](long long x, long long y) { return x + y; });
      if (c < w1) a.out_off[c] = run_v + iv - vv[u];
      run_v += from_lane63(iv);
      run_k += from_lane63(ik);
    }
  }
  if (lane == 0) {
    sW[wave] = run_v;
    sTk[wave] = run_k;
  }
  __syncthreads();
  long long base_v = 0, tot_v = 0, tot_k = 0;
  for (int w = 0; w < nw; ++w) {
    if (w < wave) base_v += sW[w];
    tot_v += sW[w];
    tot_k += sTk[w];
  }
#pragma unroll 4
  for (int c = w0 + lane; c < w1; c += 64) a.out_off[c] += base_v;
  if (tid == 0) {
    sTot[0] = tot_v;
    sTot[1] = tot_k;
  }
  __syncthreads();
  const long long carry = sTot[0], inserted = sTot[1];
  const long long total_new = carry;
  const int S = a.n_sheets;
  int64_t *newnt = a.work;
  int64_t *first2 = a.work + S;  // S + 1 entries
  int64_t *flat0 = a.work + 2 * S + 1;
  long long old_first = 0, new_first = 0;
  for (int base = 0; base < S; base += nth) {
    const int s = base + tid;
    long long och = 0, nch = 0, nn = 0, o0 = 0;
    if (s < S) och = ((long long)a.nt[s] + kChunk - 1) / kChunk;
    const long long io = block_incl_scan(och, sW);
    if (s < S) {
      const long long f0 = old_first + io - och, f1 = old_first + io;  // old chunks of sheet s
      o0 = a.out_off[f0];
      const long long o1 = f1 < n ? a.out_off[f1] : total_new;
      nn = o1 - o0;
      nch = (nn + kChunk - 1) / kChunk;
      if (nn > 0x7fffffffll) sOver = 1;
    }
    const long long in2 = block_incl_scan(nch, sW);
    if (s < S) {
      newnt[s] = nn;
      first2[s] = new_first + in2 - nch;
      flat0[s] = o0;
    }
    if (tid == nth - 1) {
      sTot[0] = io;
      sTot[1] = in2;
    }
    __syncthreads();
    old_first += sTot[0];
    new_first += sTot[1];
    __syncthreads();
  }
  if (tid == 0) {
    first2[S] = new_first;
    const bool over = sOver != 0 || total_new > a.max_tracers || new_first > a.chunk_cap;
    if (over) {
      st[kRefHalt] = 1;
      st[kRefInserted] = 0;
      a.inst[a.slot].active = 0;
    } else {
      st[kRefInserted] = (int32_t)(inserted < 0x7fffffffll ? inserted : 0x7fffffffll);
      st[kRefNextChunks] = (int32_t)new_first;
    }
  }
}

// Writes the planned layout: per new chunk its descriptor (sheet charge,
// fixed-point charge, valid count, partner chunk, open-sheet start), its
// first staging index, the slot of the tracer before it (charge edges) and,
// for piecewise-linear segments, its links; the slot's work items (runs of
// tile chunks); the new counts.  Mirrors the host's layout building.
__global__ void __launch_bounds__(256) k_refine_layout(RefinePlanArgs a) {
  int32_t *st = a.state;
  if (st[kRefInserted] <= 0) return;
  const int S = a.n_sheets;
  const int64_t *newnt = a.work;
  const int64_t *first2 = a.work + S;
  const int64_t *flat0 = a.work + 2 * S + 1;
  const int n2 = st[kRefNextChunks];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  auto n_valid_of = [](long long n, long long k) { return (int32_t)min((long long)kChunk, n - k * kChunk); };
  if (c < n2) {
    int lo = 0, hi = S - 1;  // the sheet holding new chunk c: last s with first2[s] <= c
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (first2[mid] <= c) lo = mid;
      else hi = mid - 1;
    }
    const int s = lo;
    const long long k = c - first2[s];
    const long long n = newnt[s];
    const long long nch = (n + kChunk - 1) / kChunk;
    const int32_t first = a.chunk_begin + (int32_t)first2[s];
    const bool cl = a.closed[s] != 0;
    ChunkDesc d;
    d.q = a.q[s];
    d.q_fix = a.fixed ? (int64_t)llrint(a.q[s] * a.q_scale) : 0;
    d.n_valid = n_valid_of(n, k);
    d.inst = a.slot;
    d.flags = (k == 0 && !cl) ? kChunkOpenStart : 0;
    d.partner = (k + 1 < nch) ? (int32_t)(first + k + 1) : (cl ? first : -1);
    a.chunks[first + k] = d;
    a.in_off[c] = flat0[s] + k * kChunk;
    if (a.edge_prev) {
      int64_t pv = -1;
      if (k > 0) pv = (int64_t)(first + k - 1) * kChunk + (kChunk - 1);
      else if (cl) pv = (int64_t)(first + nch - 1) * kChunk + (n - (nch - 1) * kChunk - 1);
      a.edge_prev[first + k] = pv;
    }
    if (a.links) {
      int2 lk = make_int2(-1, -1);
      if (!cl || n >= 3) {
        if (k > 0) lk.x = (int32_t)(((first + k - 1) << 2) | kHaloLast);
        else if (cl) lk.x = (int32_t)(((first + nch - 1) << 2) | kHaloLast);
        if (d.partner >= 0) {
          const long long pk = d.partner - first;
          if (n_valid_of(n, pk) >= 2) {
            lk.y = (d.partner << 2) | kHaloSecond;
          } else {
            const int32_t pp = (pk + 1 < nch) ? (int32_t)(first + pk + 1) : (cl ? first : -1);
            if (pp >= 0) lk.y = (pp << 2) | kHaloFirst;
          }
        }
      }
      a.links[first + k] = lk;
    }
  }
  const int n_items = (n2 + a.tile - 1) / a.tile;
  if (c < n_items) {
    Item it;
    it.inst = a.slot;
    it.chunk_begin = a.chunk_begin + c * a.tile;
    it.chunk_end = a.chunk_begin + min(n2, (c + 1) * a.tile);
    it.pad = 0;
    a.items[a.item_begin + c] = it;
  }
  for (int s = c; s < S; s += gridDim.x * blockDim.x) a.nt[s] = (int32_t)newnt[s];
  if (c == 0) {
    st[kRefChunks] = n2;
    a.slot_items[a.slot].y = n_items;
    *a.n_items = a.item_begin + n_items;
  }
}

template <int PREC>
__global__ void __launch_bounds__(256) k_zero_mesh(void *meshP, void *meshD, void *meshR, const InstDesc *inst,
                                                   const int32_t *slot_list, int rep, int64_t rep_stride) {
  using acc_t = typename std::conditional<PREC == kFP64, double, long long>::type;
  const int slot = slot_list ? slot_list[blockIdx.x] : (int)blockIdx.x;
  const InstDesc &I = inst[slot];
  for (int r = 0; r < rep; ++r) {
    const int64_t off = I.mesh_off + r * rep_stride;
    acc_t *P = reinterpret_cast<acc_t *>(meshP) + off;
    acc_t *D = reinterpret_cast<acc_t *>(meshD) + off;
    acc_t *R = meshR ? reinterpret_cast<acc_t *>(meshR) + off : nullptr;
    for (int j = threadIdx.x; j < I.n_cells; j += blockDim.x) {
      P[j] = (acc_t)0;
      D[j] = (acc_t)0;
      if (R) R[j] = (acc_t)0;
    }
  }
}

// Streaming copy for the bandwidth calibration: per iteration each lane has
// kCopyUnroll 16-byte loads in flight before it stores them; loads and stores
// are non-temporal (the array streams through once), and the workgroups
// stride over the array together.
typedef double f64x2 __attribute__((ext_vector_type(2)));
constexpr int kCopyUnroll = 4;

__global__ void __launch_bounds__(256) k_copy(const f64x2 *__restrict__ src, f64x2 *__restrict__ dst, int64_t n2) {
  const int64_t bd = blockDim.x;
  const int64_t per_iter = (int64_t)gridDim.x * bd * kCopyUnroll;
  int64_t i = (int64_t)blockIdx.x * bd * kCopyUnroll + threadIdx.x;
  for (; i + (kCopyUnroll - 1) * bd < n2; i += per_iter) {
    f64x2 r[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) r[u] = __builtin_nontemporal_load(src + i + u * bd);
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) __builtin_nontemporal_store(r[u], dst + i + u * bd);
  }
  for (int u = 0; u < kCopyUnroll; ++u) {
    if (i + u * bd < n2) dst[i + u * bd] = src[i + u * bd];
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
constexpr size_t kLdsMax = 160 * 1024;  // per workgroup on gfx950

// The deposit-only launch of constant segments: its own LDS layout (no field,
// a ring per wavefront), with the workgroup narrowed until it fits.
template <int PREC, bool SEG>
static hipError_t deposit_faces(const TracerArgs &a, int grid, int block, hipStream_t st) {
  static bool limit_set = false;
  if (!limit_set) {
    const hipError_t e = hipFuncSetAttribute((const void *)k_deposit_faces<PREC, SEG>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
    if (e != hipSuccess) return e;
    limit_set = true;
  }
  size_t lds = dep_lds_bytes<SEG>(a.mesh_cells, a.tile_cap, block / kChunk);
  while (lds > kLdsMax && block > kChunk) {
    block /= 2;
    lds = dep_lds_bytes<SEG>(a.mesh_cells, a.tile_cap, block / kChunk);
  }
  if (lds > kLdsMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_deposit_faces<PREC, SEG>), dim3(grid), dim3(block), lds, st, a);
  return hipGetLastError();
}

template <int PREC, int ORDER, bool SEG>
static hipError_t tracers_prec(int mode, const TracerArgs &a, int grid, int block, size_t lds, hipStream_t st) {
  switch (mode) {
    case kDeposit:
      if constexpr (ORDER == 0) {
        return deposit_faces<PREC, SEG>(a, grid, block, st);
      } else {
        hipLaunchKernelGGL((k_tracers<PREC, kDeposit, ORDER, SEG>), dim3(grid), dim3(block), lds, st, a);
      }
      break;
    case kPush:
      hipLaunchKernelGGL((k_tracers<PREC, kPush, ORDER, SEG>), dim3(grid), dim3(block), lds, st, a);
      break;
    case kPush | kDeposit:
      hipLaunchKernelGGL((k_tracers<PREC, kPush | kDeposit, ORDER, SEG>), dim3(grid), dim3(block), lds, st, a);
      break;
    case kKickHalf:
      hipLaunchKernelGGL((k_tracers<PREC, kKickHalf, ORDER, SEG>), dim3(grid), dim3(block), lds, st, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int PREC, int ORDER, bool SEG>
static hipError_t set_lds_limit(size_t bytes) {
  const int b = (int)bytes;
  const void *fns[] = {(const void *)k_tracers<PREC, kPush, ORDER, SEG>,
                       (const void *)k_tracers<PREC, kPush | kDeposit, ORDER, SEG>,
                       (const void *)k_tracers<PREC, kKickHalf, ORDER, SEG>};
  for (const void *f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e != hipSuccess) return e;
  }
  if constexpr (ORDER != 0) {
    return hipFuncSetAttribute((const void *)k_tracers<PREC, kDeposit, ORDER, SEG>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, b);
  }
  return hipSuccess;
}

// Dispatch of a runtime (precision, order, per-segment charges) triple to a
// template instance.
template <template <int, int, bool> class F, class... Args>
static hipError_t dispatch(int prec, int order, bool seg, Args &&...args) {
#define SIC_CASE(P, O)                                                                    \
  if (prec == P && order == O)                                                            \
    return seg ? F<P, O, true>::run(args...) : F<P, O, false>::run(args...);
  SIC_CASE(kFP64, 0) SIC_CASE(kFP64, 1) SIC_CASE(kFP64, 2)
  SIC_CASE(kSplitF32, 0) SIC_CASE(kSplitF32, 1) SIC_CASE(kSplitF32, 2)
  SIC_CASE(kSplitU32, 0) SIC_CASE(kSplitU32, 1) SIC_CASE(kSplitU32, 2)
#undef SIC_CASE
  return hipErrorInvalidValue;
}

template <int PREC, int ORDER, bool SEG>
struct LaunchTracers {
  static hipError_t run(int mode, const TracerArgs &a, int grid, int block, size_t lds, hipStream_t st) {
    return tracers_prec<PREC, ORDER, SEG>(mode, a, grid, block, lds, st);
  }
};

template <int PREC, int ORDER, bool SEG>
struct SetLdsLimit {
  static hipError_t run(size_t bytes) { return set_lds_limit<PREC, ORDER, SEG>(bytes); }
};

// The limit is a property of the kernel function, shared by every pool in
// the process, so it only ever grows.
int set_tracer_lds_limit(int prec, int order, bool seg, size_t lds) {
  static size_t granted[3][3][2] = {};
  if (prec < 0 || prec > 2 || order < 0 || order > 2) return (int)hipErrorInvalidValue;
  size_t &g = granted[prec][order][seg ? 1 : 0];
  if (lds <= std::max<size_t>(g, 65536)) return 0;
  const hipError_t e = dispatch<SetLdsLimit>(prec, order, seg, lds);
  if (e == hipSuccess) g = lds;
  return (int)e;
}

// Solve-first launches (single simulations, constant segments).
template <int PREC, bool SEG, int SF>
static hipError_t tracers_sf_launch(const TracerArgs &a, int grid, int block, size_t lds, hipStream_t st) {
  // the dynamic LDS limit is raised to what a launch asks for, not to the
  // whole 160 KB: the solve's static LDS takes part of it
  static size_t granted = 65536;
  if (lds > granted) {
    const hipError_t e = hipFuncSetAttribute((const void *)k_tracers<PREC, kPush | kDeposit, 0, SEG, SF>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) {
      (void)hipGetLastError();  // not left for the next launch to report
      return e;
    }
    granted = lds;
  }
  hipLaunchKernelGGL((k_tracers<PREC, kPush | kDeposit, 0, SEG, SF>), dim3(grid), dim3(block), lds, st, a);
  return hipGetLastError();
}

template <int PREC, bool SEG>
static hipError_t tracers_sf_cells(const TracerArgs &a, int grid, int block, size_t lds, int max_cells,
                                   hipStream_t st) {
  const int per = (max_cells + kSolveThreads - 1) / kSolveThreads;
  if (per <= 1) return tracers_sf_launch<PREC, SEG, 1>(a, grid, block, lds, st);
  if (per <= 4) return tracers_sf_launch<PREC, SEG, 4>(a, grid, block, lds, st);
  return tracers_sf_launch<PREC, SEG, 16>(a, grid, block, lds, st);
}

int launch_tracers_sf(int prec, bool seg, const TracerArgs &a, int grid, int block, size_t lds, int max_cells,
                      void *stream) {
  if (grid <= 0) return 0;
  if (max_cells < 1 || max_cells > kMaxCells || block < kSolveThreads || a.rep != single_rep(max_cells))
    return (int)hipErrorInvalidValue;
  hipStream_t st = (hipStream_t)stream;
  switch (prec) {
    case kFP64:
      return (int)(seg ? tracers_sf_cells<kFP64, true>(a, grid, block, lds, max_cells, st)
                       : tracers_sf_cells<kFP64, false>(a, grid, block, lds, max_cells, st));
    case kSplitF32:
      return (int)(seg ? tracers_sf_cells<kSplitF32, true>(a, grid, block, lds, max_cells, st)
                       : tracers_sf_cells<kSplitF32, false>(a, grid, block, lds, max_cells, st));
    case kSplitU32:
      return (int)(seg ? tracers_sf_cells<kSplitU32, true>(a, grid, block, lds, max_cells, st)
                       : tracers_sf_cells<kSplitU32, false>(a, grid, block, lds, max_cells, st));
    default: return (int)hipErrorInvalidValue;
  }
}

int launch_tracers(int prec, int mode, int order, bool seg, const TracerArgs &a, int grid, int block, size_t lds,
                   void *stream) {
  if (grid <= 0) return 0;
  return (int)dispatch<LaunchTracers>(prec, order, seg, mode, a, grid, block, lds, (hipStream_t)stream);
}

// Meshes of up to 1024 cells run the resident kernel with 8 wavefronts (four
// chunks each: twice the latency hiding of four; 16 wavefronts would leave
// 128 VGPRs and spill); larger ones, whose solve holds 16 cells per thread
// in registers, with four.
template <int PREC, bool SEG, int CELLS>
static hipError_t resident_launch(const TracerArgs &a, const SolveArgs &sa, int chunk_begin, int n_chunks,
                                  int64_t n_steps, size_t lds, hipStream_t st) {
  constexpr int NT = CELLS <= 4 ? 512 : kSolveThreads;
  static bool limit_set = false;
  if (!limit_set) {
    const hipError_t e = hipFuncSetAttribute((const void *)k_resident<PREC, SEG, CELLS, NT>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)resident_lds_bytes(kMaxCells, true));
    if (e != hipSuccess) return e;
    limit_set = true;
  }
  hipLaunchKernelGGL((k_resident<PREC, SEG, CELLS, NT>), dim3(1), dim3(NT), lds, st, a, sa, chunk_begin,
                     n_chunks, n_steps);
  return hipGetLastError();
}

// Cells per solve thread the kernels are built for: 1, 4 or 16.
static int solve_cells(int max_cells) {
  const int per = (max_cells + kSolveThreads - 1) / kSolveThreads;
  return per <= 1 ? 1 : (per <= 4 ? 4 : 16);
}

template <int PREC, bool SEG>
static hipError_t resident_prec(const TracerArgs &a, const SolveArgs &sa, int chunk_begin, int n_chunks,
                                int n_cells, int64_t n_steps, size_t lds, hipStream_t st) {
  switch (solve_cells(n_cells)) {
    case 1: return resident_launch<PREC, SEG, 1>(a, sa, chunk_begin, n_chunks, n_steps, lds, st);
    case 4: return resident_launch<PREC, SEG, 4>(a, sa, chunk_begin, n_chunks, n_steps, lds, st);
    default: return resident_launch<PREC, SEG, 16>(a, sa, chunk_begin, n_chunks, n_steps, lds, st);
  }
}

int resident_max_chunks() { return kResidentChunks; }

int launch_resident(int prec, bool seg, const TracerArgs &a, const SolveArgs &sa, int chunk_begin, int n_chunks,
                    int n_cells, int64_t n_steps, void *stream) {
  if (n_steps <= 0) return 0;
  if (n_chunks < 1 || n_chunks > kResidentChunks || n_cells < 1 || n_cells > kMaxCells)
    return (int)hipErrorInvalidValue;
  const size_t lds = resident_lds_bytes(n_cells, seg);
  hipStream_t st = (hipStream_t)stream;
  switch (prec) {
    case kFP64:
      return (int)(seg ? resident_prec<kFP64, true>(a, sa, chunk_begin, n_chunks, n_cells, n_steps, lds, st)
                       : resident_prec<kFP64, false>(a, sa, chunk_begin, n_chunks, n_cells, n_steps, lds, st));
    case kSplitF32:
      return (int)(seg ? resident_prec<kSplitF32, true>(a, sa, chunk_begin, n_chunks, n_cells, n_steps, lds, st)
                       : resident_prec<kSplitF32, false>(a, sa, chunk_begin, n_chunks, n_cells, n_steps, lds, st));
    case kSplitU32:
      return (int)(seg ? resident_prec<kSplitU32, true>(a, sa, chunk_begin, n_chunks, n_cells, n_steps, lds, st)
                       : resident_prec<kSplitU32, false>(a, sa, chunk_begin, n_chunks, n_cells, n_steps, lds, st));
    default:
      return (int)hipErrorInvalidValue;
  }
}

template <int CELLS, int REP>
static hipError_t solve_cells_launch(int prec, const SolveArgs &a, int n_blocks, hipStream_t st) {
  switch (prec) {
    case kFP64:
      hipLaunchKernelGGL((k_solve<kFP64, CELLS, REP>), dim3(n_blocks), dim3(kSolveThreads), 0, st, a);
      break;
    case kSplitF32:
      hipLaunchKernelGGL((k_solve<kSplitF32, CELLS, REP>), dim3(n_blocks), dim3(kSolveThreads), 0, st, a);
      break;
    case kSplitU32:
      hipLaunchKernelGGL((k_solve<kSplitU32, CELLS, REP>), dim3(n_blocks), dim3(kSolveThreads), 0, st, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int REP>
static hipError_t solve_rep_launch(int prec, const SolveArgs &a, int n_blocks, int max_cells, hipStream_t st) {
  switch (solve_cells(max_cells)) {
    case 1: return solve_cells_launch<1, REP>(prec, a, n_blocks, st);
    case 4: return solve_cells_launch<4, REP>(prec, a, n_blocks, st);
    default: return solve_cells_launch<16, REP>(prec, a, n_blocks, st);
  }
}

int launch_solve(int prec, const SolveArgs &a, int n_blocks, int max_cells, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (n_blocks <= 0) return 0;
  if (max_cells < 1 || max_cells > kMaxCells) return (int)hipErrorInvalidValue;
  if (a.rep == 1) return (int)solve_rep_launch<1>(prec, a, n_blocks, max_cells, st);
  if (a.rep == 2) return (int)solve_rep_launch<2>(prec, a, n_blocks, max_cells, st);
  if (a.rep == 4) return (int)solve_rep_launch<4>(prec, a, n_blocks, max_cells, st);
  return (int)hipErrorInvalidValue;
}

int launch_ingest(int prec, const IngestArgs &a, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const int grid = (a.n_chunks + 3) / 4;
  if (grid <= 0) return 0;
  switch (prec) {
    case kFP64: hipLaunchKernelGGL(k_ingest<kFP64>, dim3(grid), dim3(256), 0, st, a); break;
    case kSplitF32: hipLaunchKernelGGL(k_ingest<kSplitF32>, dim3(grid), dim3(256), 0, st, a); break;
    case kSplitU32: hipLaunchKernelGGL(k_ingest<kSplitU32>, dim3(grid), dim3(256), 0, st, a); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

int launch_extract(int prec, const ExtractArgs &a, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const int grid = (a.n_chunks + 3) / 4;
  if (grid <= 0) return 0;
  switch (prec) {
    case kFP64: hipLaunchKernelGGL(k_extract<kFP64>, dim3(grid), dim3(256), 0, st, a); break;
    case kSplitF32: hipLaunchKernelGGL(k_extract<kSplitF32>, dim3(grid), dim3(256), 0, st, a); break;
    case kSplitU32: hipLaunchKernelGGL(k_extract<kSplitU32>, dim3(grid), dim3(256), 0, st, a); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

int launch_zero_mesh(int prec, void *meshP, void *meshD, void *meshR, const InstDesc *inst,
                     const int32_t *slot_list, int n_blocks, int rep, int64_t rep_stride, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (n_blocks <= 0) return 0;
  if (rep < 1) return (int)hipErrorInvalidValue;
  if (prec == kFP64)
    hipLaunchKernelGGL(k_zero_mesh<kFP64>, dim3(n_blocks), dim3(256), 0, st, meshP, meshD, meshR, inst, slot_list,
                       rep, rep_stride);
  else
    hipLaunchKernelGGL(k_zero_mesh<kSplitF32>, dim3(n_blocks), dim3(256), 0, st, meshP, meshD, meshR, inst,
                       slot_list, rep, rep_stride);
  return (int)hipGetLastError();
}

int launch_charge_edges(const ChunkDesc *chunks, const int64_t *prev_slot, const uint64_t *segq, uint64_t *cedge,
                        int32_t chunk_begin, int32_t n_chunks, void *stream, const int32_t *state) {
  if (n_chunks <= 0) return 0;
  hipLaunchKernelGGL(k_charge_edges, dim3((n_chunks + 255) / 256), dim3(256), 0, (hipStream_t)stream, chunks,
                     prev_slot, segq, cedge, chunk_begin, n_chunks, state);
  return (int)hipGetLastError();
}

int launch_refine_mark(int prec, const RefineArgs &a, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const int grid = (a.n_chunks + 3) / 4;
  if (grid <= 0) return 0;
  switch (prec) {
    case kFP64: hipLaunchKernelGGL(k_refine_mark<kFP64>, dim3(grid), dim3(256), 0, st, a); break;
    case kSplitF32: hipLaunchKernelGGL(k_refine_mark<kSplitF32>, dim3(grid), dim3(256), 0, st, a); break;
    case kSplitU32: hipLaunchKernelGGL(k_refine_mark<kSplitU32>, dim3(grid), dim3(256), 0, st, a); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

int launch_refine_scatter(int prec, const RefineArgs &a, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const int grid = (a.n_chunks + 3) / 4;
  if (grid <= 0) return 0;
  switch (prec) {
    case kFP64: hipLaunchKernelGGL(k_refine_scatter<kFP64>, dim3(grid), dim3(256), 0, st, a); break;
    case kSplitF32: hipLaunchKernelGGL(k_refine_scatter<kSplitF32>, dim3(grid), dim3(256), 0, st, a); break;
    case kSplitU32: hipLaunchKernelGGL(k_refine_scatter<kSplitU32>, dim3(grid), dim3(256), 0, st, a); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

int launch_refine_plan(const RefinePlanArgs &a, void *stream) {
  hipLaunchKernelGGL(k_refine_plan, dim3(1), dim3(1024), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int launch_refine_layout(const RefinePlanArgs &a, void *stream) {
  const int grid = std::max(1, (a.chunk_cap + 255) / 256);
  hipLaunchKernelGGL(k_refine_layout, dim3(grid), dim3(256), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int launch_copy_bench(const double *src, double *dst, int64_t n, int grid, void *stream) {
  const int64_t n2 = n / 2;
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const f64x2 *)src, (f64x2 *)dst, n2);
  return (int)hipGetLastError();
}

}  // namespace sic
