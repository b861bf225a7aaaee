/*
 * sic_oracle.c - plain, slow, FP64 CPU reference of one simplex-in-cell (SIC)
 * 1D1V Vlasov-Poisson step (Kates-Harbeck, Totorica, Zrake & Abel,
 * arXiv:1506.07207).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity oracle for the GPU
 * library: it shares no code, header, table or helper with it, and only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It is written for a reader checking it against the paper, not for
 * speed: no blocking, no fusion, no vectorisation.  Build with IEEE semantics
 * (-O2 -ffp-contract=off, no fast-math).
 *
 * Units and conventions (paper section 2.1, eqs. 1-3 with C = 1):
 *   - the Vlasov equation accelerates a tracer by -dPhi/dx, written E here, so
 *     the Poisson equation d2Phi/dx2 = -rho becomes dE/dx = rho;
 *   - rho = n - nbar: the mean density is removed (periodic box);
 *   - the mesh has nc cells [j dx, (j+1) dx), dx = L / nc, with mesh values at
 *     the cell centres X_j = (j + 1/2) dx (the grid points of section 2.4).
 *
 * Step (section 2.3 and the "solve, gather, move" paragraph after it):
 *   deposit: rho_j = (1/dx) sum_i o_ji q_i, with o_ji the overlap of the box
 *            function of segment i (height 1/|length|) with cell j
 *            (eqs. "overlap" and "rho_sum");
 *   solve:   3-point finite-difference Poisson equation on the periodic mesh,
 *            E_j = -(Phi_{j+1} - Phi_{j-1}) / (2 dx); solved here exactly in
 *            the discrete Fourier basis that diagonalises it;
 *   gather:  linear (first-order, W_1) weighting from the grid points
 *            (section 2.4 and the gather remark of section 2.3);
 *   move:    leapfrog, v^{n+1/2} = v^{n-1/2} + dt E^n(x^n),
 *            x^{n+1} = x^n + dt v^{n+1/2}, wrapped into [0, L).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - a point exactly on a face belongs to the lower cell (the tie rule of
 *     the zero-order weight W_0, section 2.4); this decides where a
 *     zero-length segment puts its charge;
 *   - a zero-length segment deposits all of its charge into that one cell
 *     (footnote on equal tracer positions, section 2.3: any handling that
 *     keeps the total charge is acceptable);
 *   - a segment joins its tracers along the shorter way round the periodic
 *     box (minimum image); a separation of exactly L/2 is taken downwards;
 *   - the segments are the particles of section 2.3 and carry the charge:
 *     segment t of a sheet joins tracer t to tracer t+1 and carries c_t (in
 *     the common case the same q_s for every segment of sheet s); each tracer
 *     carries half the mass of each segment it bounds, m_t = (c_{t-1} + c_t)/2
 *     (a missing segment at an open sheet's end counts 0), so the total mass
 *     equals the total charge (equal charge-to-mass ratio);
 *   - KE^n = 1/2 sum q v^{n-1/2} v^{n+1/2} (the leapfrog-centred product),
 *     W_E^n = 1/2 dx sum_j E_j^2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ROW 8 /* step, t, W_E, KE, momentum, total_charge, max_segment, flags */
#define ORC_FLAG_NONFINITE 1.0
#define ORC_FLAG_LONG_SEGMENT 2.0

/* Reduce a position into [0, L).  One period either way is handled by a
 * single add or subtract (x - L is exact for x in [L, 2L)); a sum that rounds
 * up to L is the point 0 of the periodic box. */
double orc_wrap(double x, double L)
{
    if (x >= 0.0 && x < L) return x;
    if (x >= L && x < 2.0 * L) return x - L;
    if (x < 0.0 && x >= -L) {
        double y = x + L;
        return (y >= L) ? 0.0 : y;
    }
    {
        double y = x - L * floor(x / L);
        if (y < 0.0) y += L;
        if (y >= L) y = 0.0;
        return y;
    }
}

/* Signed separation from a to b along the shorter way round the box. */
double orc_min_image(double a, double b, double L)
{
    double d = b - a;
    if (d >= 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

static int mod_cell(long j, int nc)
{
    long r = j % nc;
    return (int)(r < 0 ? r + nc : r);
}

/* Cell that owns a point, with a point on a face assigned to the lower cell
 * (the W_0 tie rule). */
int orc_point_cell(double x, double L, int nc)
{
    double dx = L / nc;
    long j = (long)ceil(x / dx) - 1;
    return mod_cell(j, nc);
}

static double face(int j, int nc, double dx, double L)
{
    return (j >= nc) ? L : (double)j * dx;
}

/* Add w * |[lo, hi] ∩ cell_j| for every cell, 0 <= lo <= hi <= L. */
static void add_interval(double lo, double hi, double w, double L, int nc, double *Q)
{
    double dx = L / nc;
    /* one extra cell either side guards against lo/dx or hi/dx rounding
     * across a face; cells that do not meet [lo, hi] add nothing */
    int j0 = (int)floor(lo / dx) - 1;
    int j1 = (int)floor(hi / dx) + 1;
    if (j0 < 0) j0 = 0;
    if (j1 > nc - 1) j1 = nc - 1;
    for (int j = j0; j <= j1; ++j) {
        double a = face(j, nc, dx, L);
        double b = face(j + 1, nc, dx, L);
        double left = lo > a ? lo : a;
        double right = hi < b ? hi : b;
        if (right > left) Q[j] += w * (right - left);
    }
}

/* Running maximum of segment lengths; a NaN length (a segment with a
 * non-finite end) makes the result NaN for good, so it reaches the flags. */
static double longest(double m, double len)
{
    if (isnan(m) || isnan(len)) return NAN;
    return len > m ? len : m;
}

/* Deposit one segment from tracer position a to tracer position b (both in
 * [0, L)) carrying charge q: the box function of height 1/length is
 * integrated over every cell it overlaps (eqs. "overlap" and "rho_sum",
 * multiplied by the cell volume).  Returns the segment length (NaN, with
 * nothing deposited, when an end is not a finite position). */
double orc_deposit_segment(double a, double b, double q, double L, int nc, double *Q)
{
    double d = orc_min_image(a, b, L);
    if (!isfinite(d)) return NAN; /* a non-finite end: nothing deposited, length NaN */
    if (d == 0.0) {
        Q[orc_point_cell(a, L, nc)] += q;
        return 0.0;
    }
    /* The segment as a set of at most two non-wrapping intervals. */
    double lo1, hi1, lo2 = 0.0, hi2 = 0.0;
    int two = 0;
    if (d > 0.0) {
        if (b > a) { lo1 = a; hi1 = b; }
        else { lo1 = a; hi1 = L; lo2 = 0.0; hi2 = b; two = 1; }
    } else {
        if (b < a) { lo1 = b; hi1 = a; }
        else { lo1 = b; hi1 = L; lo2 = 0.0; hi2 = a; two = 1; }
    }
    double len = (hi1 - lo1) + (two ? (hi2 - lo2) : 0.0);
    if (!(len > 0.0)) { /* a sub-rounding separation: treat as a point */
        Q[orc_point_cell(a, L, nc)] += q;
        return fabs(d);
    }
    double w = q / len;
    add_interval(lo1, hi1, w, L, nc, Q);
    if (two) add_interval(lo2, hi2, w, L, nc, Q);
    return fabs(d);
}

/* Charge per cell Q_j = dx * rho_j (before the mean is removed) for all
 * sheets.  Sheets are stored one after another; a closed sheet also joins its
 * last tracer to its first (section 2.3, periodic closure).  Q is zeroed. */
void orc_deposit_c(double L, int nc, int n_sheets, const int32_t *n_tracers, const int32_t *closed,
                   const double *c, const double *x, double *Q, double *max_segment)
{
    double maxseg = 0.0;
    memset(Q, 0, sizeof(double) * (size_t)nc);
    int64_t base = 0;
    for (int s = 0; s < n_sheets; ++s) {
        int nt = n_tracers[s];
        int nseg = closed[s] ? nt : nt - 1;
        for (int t = 0; t < nseg; ++t) {
            int u = (t + 1 == nt) ? 0 : t + 1;
            double len = orc_deposit_segment(x[base + t], x[base + u], c[base + t], L, nc, Q);
            maxseg = longest(maxseg, len);
        }
        base += nt;
    }
    if (max_segment) *max_segment = maxseg;
}

/* Per-segment charges of sheets whose segments all carry the sheet's q_s
 * (entry t is the segment that starts at tracer t; the last tracer of an
 * open sheet starts none and gets 0).  Returns a malloc'ed array. */
static double *uniform_charges(int n_sheets, const int32_t *n_tracers, const double *q, const int32_t *closed)
{
    int64_t n = 0;
    for (int s = 0; s < n_sheets; ++s) n += n_tracers[s];
    double *c = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!c) return NULL;
    int64_t base = 0;
    for (int s = 0; s < n_sheets; ++s) {
        for (int t = 0; t < n_tracers[s]; ++t) c[base + t] = q[s];
        if (!closed[s] && n_tracers[s] > 0) c[base + n_tracers[s] - 1] = 0.0;
        base += n_tracers[s];
    }
    return c;
}

void orc_deposit(double L, int nc, int n_sheets, const int32_t *n_tracers, const double *q,
                 const int32_t *closed, const double *x, double *Q, double *max_segment)
{
    double *c = uniform_charges(n_sheets, n_tracers, q, closed);
    orc_deposit_c(L, nc, n_sheets, n_tracers, closed, c, x, Q, max_segment);
    free(c);
}

/* Piecewise-linear segments (section 2.5, eqs. "piecewise_linear" and
 * "gradient_rho_estimate").  Segment i of a sheet carries the density
 *     rho_i(x) = rho0_i + (x - c_i) g_i   on its extent,
 * with rho0_i = q / |segment i| and c_i its centroid.  The gradient is the
 * central difference of the neighbouring segments' rho0 over their centroid
 * separation, g_i = (rho0_{i+1} - rho0_{i-1}) / (c_{i+1} - c_{i-1}), and is
 * left out (g_i = 0) where the centroids c_{i-1}, c_i, c_{i+1} are not in
 * monotone order (the corner of a fold), where a neighbouring segment is
 * missing (ends of an open sheet) or where a segment of the three has zero
 * length.  Centroid separations take the shorter way round the box.  Every
 * cell receives the exact integral of rho_i over its overlap with the
 * segment; the linear term integrates to zero over the segment, so each
 * segment still deposits exactly q.  Segments are laid out in unwrapped
 * coordinates [lo, hi] around their first tracer; a cell index outside
 * 0..nc-1 is taken modulo nc. */
void orc_deposit_linear_c(double L, int nc, int n_sheets, const int32_t *n_tracers, const int32_t *closed,
                          const double *cq, const double *x, double *Q, double *max_segment)
{
    double dx = L / nc;
    double maxseg = 0.0;
    memset(Q, 0, sizeof(double) * (size_t)nc);
    int64_t base = 0;
    for (int s = 0; s < n_sheets; ++s) {
        int nt = n_tracers[s];
        int nseg = closed[s] ? nt : nt - 1;
        double *a = (double *)malloc(sizeof(double) * (size_t)nseg);
        double *d = (double *)malloc(sizeof(double) * (size_t)nseg);
        double *c = (double *)malloc(sizeof(double) * (size_t)nseg);
        double *r0 = (double *)malloc(sizeof(double) * (size_t)nseg);
        for (int t = 0; t < nseg; ++t) {
            int u = (t + 1 == nt) ? 0 : t + 1;
            a[t] = x[base + t];
            d[t] = orc_min_image(a[t], x[base + u], L);
            c[t] = a[t] + 0.5 * d[t];
            r0[t] = d[t] != 0.0 ? cq[base + t] / fabs(d[t]) : 0.0;
            maxseg = longest(maxseg, fabs(d[t]));
        }
        for (int t = 0; t < nseg; ++t) {
            if (!isfinite(d[t])) continue; /* a non-finite end: nothing deposited */
            if (d[t] == 0.0) {
                Q[orc_point_cell(a[t], L, nc)] += cq[base + t];
                continue;
            }
            double g = 0.0;
            int has_prev = closed[s] ? (nseg >= 3) : (t > 0);
            int has_next = closed[s] ? (nseg >= 3) : (t + 1 < nseg);
            if (has_prev && has_next) {
                int tp = (t == 0) ? nseg - 1 : t - 1;
                int tn = (t + 1 == nseg) ? 0 : t + 1;
                if (d[tp] != 0.0 && d[tn] != 0.0) {
                    double dm = orc_min_image(c[t], c[tp], L); /* c_{i-1} - c_i */
                    double dp = orc_min_image(c[t], c[tn], L); /* c_{i+1} - c_i */
                    if ((dm < 0.0 && dp > 0.0) || (dm > 0.0 && dp < 0.0))
                        g = (r0[tn] - r0[tp]) / (dp - dm);
                }
            }
            double lo = d[t] > 0.0 ? a[t] : a[t] + d[t];
            double hi = d[t] > 0.0 ? a[t] + d[t] : a[t];
            long j0 = (long)floor(lo / dx) - 1, j1 = (long)floor(hi / dx) + 1;
            for (long j = j0; j <= j1; ++j) {
                double fa = (double)j * dx, fb = (double)(j + 1) * dx;
                double al = lo > fa ? lo : fa;
                double be = hi < fb ? hi : fb;
                if (be > al) {
                    /* exact integral of r0 + (x - c) g over [al, be] */
                    double w = be - al;
                    Q[mod_cell(j, nc)] += r0[t] * w + g * w * (0.5 * (al + be) - c[t]);
                }
            }
        }
        free(a); free(d); free(c); free(r0);
        base += nt;
    }
    if (max_segment) *max_segment = maxseg;
}

void orc_deposit_linear(double L, int nc, int n_sheets, const int32_t *n_tracers, const double *q,
                        const int32_t *closed, const double *x, double *Q, double *max_segment)
{
    double *c = uniform_charges(n_sheets, n_tracers, q, closed);
    orc_deposit_linear_c(L, nc, n_sheets, n_tracers, closed, c, x, Q, max_segment);
    free(c);
}

/* First-order weighting of segments (section 2.4): every slice of a
 * segment's box function is assigned to the grid points X_j = (j + 1/2) dx
 * with the first-order weight W_1(x - X_j) = max(0, 1 - |x - X_j| / dx), so
 * grid point j receives h * integral over the segment of W_1(x - X_j) dx,
 * h = q / length.  Every hat is linear between consecutive grid points, so
 * the grid points inside the segment cut it into pieces on each of which
 * only the two grid points X_m, X_{m+1} around it have weight, linear in x;
 * the integral of a linear function over a piece is its length times its
 * value at the midpoint.  A piece [p0, p1] therefore gives its charge
 * h (p1 - p0) to X_m and X_{m+1} in the proportions 1 - t and t, t the
 * midpoint's distance from X_m in cells.  Consecutive pieces share their
 * end points, so the pieces of a segment add up to its charge to rounding
 * however short it is.  A zero-length segment is a point charge: W_1
 * weights of the point.  The result is the charge per grid point
 * (dx * density), as for the other deposits. */
static double hat(double x, double X, double dx)
{
    double w = 1.0 - fabs(x - X) / dx;
    return w > 0.0 ? w : 0.0;
}

void orc_deposit_cic_c(double L, int nc, int n_sheets, const int32_t *n_tracers, const int32_t *closed,
                       const double *c, const double *x, double *Q, double *max_segment)
{
    double dx = L / nc;
    double maxseg = 0.0;
    memset(Q, 0, sizeof(double) * (size_t)nc);
    int64_t base = 0;
    for (int s = 0; s < n_sheets; ++s) {
        int nt = n_tracers[s];
        int nseg = closed[s] ? nt : nt - 1;
        for (int t = 0; t < nseg; ++t) {
            int u = (t + 1 == nt) ? 0 : t + 1;
            double a = x[base + t];
            double d = orc_min_image(a, x[base + u], L);
            maxseg = longest(maxseg, fabs(d));
            if (!isfinite(d)) continue; /* a non-finite end: nothing deposited */
            if (d == 0.0) {
                long j0 = (long)floor(a / dx - 0.5);
                for (long j = j0; j <= j0 + 1; ++j)
                    Q[mod_cell(j, nc)] += c[base + t] * hat(a, ((double)j + 0.5) * dx, dx);
                continue;
            }
            double lo = d > 0.0 ? a : a + d, hi = d > 0.0 ? a + d : a;
            double h = c[base + t] / (hi - lo);
            /* grid interval m is [X_m, X_{m+1}]; start from the one holding lo
             * (a rounding of lo / dx that lands one interval off only gives an
             * empty first piece or a first piece reaching a rounding past X_m) */
            long m = (long)floor(lo / dx - 0.5);
            double p0 = lo;
            for (;;) {
                double Xr = ((double)(m + 1) + 0.5) * dx;
                double p1 = Xr < hi ? Xr : hi;
                if (p1 > p0) {
                    double piece = h * (p1 - p0);
                    double tm = (0.5 * (p0 + p1) - ((double)m + 0.5) * dx) / dx;
                    Q[mod_cell(m, nc)] += piece * (1.0 - tm);
                    Q[mod_cell(m + 1, nc)] += piece * tm;
                    p0 = p1;
                }
                if (p1 >= hi) break;
                ++m;
            }
        }
        base += nt;
    }
    if (max_segment) *max_segment = maxseg;
}

void orc_deposit_cic(double L, int nc, int n_sheets, const int32_t *n_tracers, const double *q,
                     const int32_t *closed, const double *x, double *Q, double *max_segment)
{
    double *c = uniform_charges(n_sheets, n_tracers, q, closed);
    orc_deposit_cic_c(L, nc, n_sheets, n_tracers, closed, c, x, Q, max_segment);
    free(c);
}

/* Solve the periodic 3-point Poisson equation
 *     (Phi_{j+1} - 2 Phi_j + Phi_{j-1}) / dx^2 = -rho_j,  rho_j = Q_j/dx - nbar,
 * and return the centred-difference field E_j = -(Phi_{j+1} - Phi_{j-1})/(2 dx)
 * and W_E = 1/2 dx sum E_j^2.  The discrete Fourier modes exp(2 pi i j m / nc)
 * diagonalise both operators: Phi_m = dx^2 rho_m / (4 sin^2(pi m / nc)) and
 * E_m = -i sin(2 pi m / nc) Phi_m / dx; mode 0 (the mean) is zero.  Plain
 * O(nc^2) transforms. */
void orc_solve(double L, int nc, const double *Q, double *E, double *W_E, double *total_charge)
{
    double dx = L / nc;
    double qtot = 0.0;
    for (int j = 0; j < nc; ++j) qtot += Q[j];
    double nbar = qtot / L;
    double *rho = (double *)malloc(sizeof(double) * (size_t)nc);
    double *cs = (double *)malloc(sizeof(double) * (size_t)nc);
    double *sn = (double *)malloc(sizeof(double) * (size_t)nc);
    double *er = (double *)malloc(sizeof(double) * (size_t)nc);
    double *ei = (double *)malloc(sizeof(double) * (size_t)nc);
    const double two_pi = 6.283185307179586476925286766559;
    for (int j = 0; j < nc; ++j) {
        rho[j] = Q[j] / dx - nbar;
        cs[j] = cos(two_pi * (double)j / (double)nc);
        sn[j] = sin(two_pi * (double)j / (double)nc);
    }
    if (nc % 2 == 0) { sn[nc / 2] = 0.0; cs[nc / 2] = -1.0; }
    if (nc % 4 == 0) { cs[nc / 4] = 0.0; sn[nc / 4] = 1.0; cs[3 * nc / 4] = 0.0; sn[3 * nc / 4] = -1.0; }
    sn[0] = 0.0; cs[0] = 1.0;
    er[0] = 0.0; ei[0] = 0.0;
    for (int m = 1; m < nc; ++m) {
        double re = 0.0, im = 0.0;
        int idx = 0;
        for (int j = 0; j < nc; ++j) {
            re += rho[j] * cs[idx];
            im -= rho[j] * sn[idx];
            idx += m;
            if (idx >= nc) idx -= nc;
        }
        double s = sin(0.5 * two_pi * (double)m / (double)nc);
        double lap = 4.0 * s * s / (dx * dx);
        double pr = re / lap, pi = im / lap;
        double g = sn[m] / dx;
        er[m] = g * pi;   /* (-i g)(pr + i pi) = g pi - i g pr */
        ei[m] = -g * pr;
    }
    double w = 0.0;
    for (int j = 0; j < nc; ++j) {
        double acc = 0.0;
        int idx = 0;
        for (int m = 0; m < nc; ++m) {
            acc += er[m] * cs[idx] - ei[m] * sn[idx];
            idx += j;
            if (idx >= nc) idx -= nc;
        }
        E[j] = acc / (double)nc;
        w += E[j] * E[j];
    }
    if (W_E) *W_E = 0.5 * dx * w;
    if (total_charge) *total_charge = qtot;
    free(rho); free(cs); free(sn); free(er); free(ei);
}

/* Field at a tracer: first-order weighting W_1(x - X_j) = 1 - |x - X_j|/dx
 * from the two grid points X_j = (j + 1/2) dx around x (periodic). */
double orc_gather(double L, int nc, const double *E, double x)
{
    if (!isfinite(x)) return NAN; /* no mesh point to read */
    double dx = L / nc;
    long j0 = (long)floor(x / dx - 0.5);
    double X0 = ((double)j0 + 0.5) * dx;
    double X1 = ((double)j0 + 1.5) * dx;
    double w0 = 1.0 - fabs(x - X0) / dx;
    double w1 = 1.0 - fabs(x - X1) / dx;
    return w0 * E[mod_cell(j0, nc)] + w1 * E[mod_cell(j0 + 1, nc)];
}

void orc_gather_many(double L, int nc, const double *E, int64_t n, const double *x, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_gather(L, nc, E, x[i]);
}

/* Per-tracer mass: half of each segment the tracer bounds,
 * m_t = (c_{t-1} + c_t) / 2, with the closing segment of a closed sheet
 * joining its last tracer to its first and nothing beyond an open sheet's
 * ends. */
static void tracer_masses(int n_sheets, const int32_t *n_tracers, const int32_t *closed, const double *c,
                          double *mass)
{
    int64_t base = 0;
    for (int s = 0; s < n_sheets; ++s) {
        int nt = n_tracers[s];
        for (int t = 0; t < nt; ++t) {
            double right = (closed[s] || t + 1 < nt) ? c[base + t] : 0.0;
            double left = 0.0;
            if (t > 0) left = c[base + t - 1];
            else if (closed[s]) left = c[base + nt - 1];
            mass[base + t] = 0.5 * (left + right);
        }
        base += nt;
    }
}

/* One leapfrog move with the field E^n: kick then drift.  Returns KE^n and
 * momentum^n through the pointers (centred on x^n). */
void orc_push_c(double L, int nc, double dt, int n_sheets, const int32_t *n_tracers, const int32_t *closed,
                const double *c, const double *E, double *x, double *v, double *ke, double *mom)
{
    int64_t n = 0;
    for (int s = 0; s < n_sheets; ++s) n += n_tracers[s];
    double *mass = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    tracer_masses(n_sheets, n_tracers, closed, c, mass);
    double k = 0.0, p = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double e = orc_gather(L, nc, E, x[i]);
        double vn = v[i] + dt * e;
        k += 0.5 * mass[i] * v[i] * vn;
        p += mass[i] * 0.5 * (v[i] + vn);
        x[i] = orc_wrap(x[i] + dt * vn, L);
        v[i] = vn;
    }
    free(mass);
    if (ke) *ke = k;
    if (mom) *mom = p;
}

void orc_push(double L, int nc, double dt, int n_sheets, const int32_t *n_tracers, const double *q,
              const int32_t *closed, const double *E, double *x, double *v, double *ke, double *mom)
{
    double *c = uniform_charges(n_sheets, n_tracers, q, closed);
    orc_push_c(L, nc, dt, n_sheets, n_tracers, closed, c, E, x, v, ke, mom);
    free(c);
}

/* Refinement (section 2.6): every segment longer than l_max gets a new
 * tracer at its centre (along the shorter way round the box), with the mean
 * of its end tracers' velocities; the two halves each carry half of the
 * segment's charge.  One pass over the segments as they are when called (a
 * segment longer than 2 l_max is halved once; the check runs again after the
 * next move).  n_tracers, x, v and c (capacity cap entries each) are updated
 * in place; returns the number of tracers inserted, or -1 (nothing changed)
 * if the result would not fit in cap. */
int64_t orc_refine(double L, double l_max, int n_sheets, int32_t *n_tracers, const int32_t *closed, double *x,
                   double *v, double *c, int64_t cap)
{
    int64_t n = 0, add = 0;
    for (int s = 0; s < n_sheets; ++s) {
        int nt = n_tracers[s];
        int nseg = closed[s] ? nt : nt - 1;
        for (int t = 0; t < nseg; ++t) {
            int u = (t + 1 == nt) ? 0 : t + 1;
            if (fabs(orc_min_image(x[n + t], x[n + u], L)) > l_max) ++add;
        }
        n += nt;
    }
    if (add == 0) return 0;
    if (n + add > cap) return -1;
    double *nx = (double *)malloc(sizeof(double) * (size_t)(n + add));
    double *nv = (double *)malloc(sizeof(double) * (size_t)(n + add));
    double *ncq = (double *)malloc(sizeof(double) * (size_t)(n + add));
    if (!nx || !nv || !ncq) { free(nx); free(nv); free(ncq); return -1; }
    int64_t base = 0, out = 0;
    for (int s = 0; s < n_sheets; ++s) {
        int nt = n_tracers[s];
        int nseg = closed[s] ? nt : nt - 1;
        int64_t first = out;
        for (int t = 0; t < nt; ++t) {
            nx[out] = x[base + t];
            nv[out] = v[base + t];
            ncq[out] = c[base + t];
            ++out;
            if (t < nseg) {
                int u = (t + 1 == nt) ? 0 : t + 1;
                double d = orc_min_image(x[base + t], x[base + u], L);
                if (fabs(d) > l_max) {
                    double half = 0.5 * c[base + t];
                    ncq[out - 1] = half;
                    nx[out] = orc_wrap(x[base + t] + 0.5 * d, L);
                    nv[out] = 0.5 * (v[base + t] + v[base + u]);
                    ncq[out] = half;
                    ++out;
                }
            }
        }
        n_tracers[s] = (int32_t)(out - first);
        base += nt;
    }
    memcpy(x, nx, sizeof(double) * (size_t)out);
    memcpy(v, nv, sizeof(double) * (size_t)out);
    memcpy(c, ncq, sizeof(double) * (size_t)out);
    free(nx); free(nv); free(ncq);
    return add;
}

/* Status flags of one diagnostics row, two independent bits: NONFINITE when
 * a field value, the longest segment, or the kinetic energy or momentum of
 * the move into this step is not finite (moved_finite = 0); LONG_SEGMENT
 * when the longest segment is finite and longer than 0.45 L (segments join
 * tracers the shorter way round, so none can exceed L/2). */
static double row_flags(double L, int nc, const double *E, double maxseg, int moved_finite)
{
    int nonfinite = !moved_finite || !isfinite(maxseg);
    for (int j = 0; j < nc; ++j)
        if (!isfinite(E[j])) nonfinite = 1;
    double f = nonfinite ? ORC_FLAG_NONFINITE : 0.0;
    if (isfinite(maxseg) && maxseg > 0.45 * L) f += ORC_FLAG_LONG_SEGMENT;
    return f;
}

/* Full run.  With init_kick = 1, (x0, v0) are the initial positions and
 * velocities: x0 is wrapped into [0, L), the field E^0 is computed and the
 * velocities are moved back half a step, v^{-1/2} = v^0 - dt/2 E^0(x^0).
 * With init_kick = 0, v0 is already v^{-1/2} at step step0 (a resumed state).
 * Each step is: push with E^n (KE^n and momentum^n), refinement of the moved
 * sheets when l_max > 0, deposit of x^{n+1}, solve.  hist holds (n_steps + 1)
 * rows of ORC_ROW doubles; the KE and momentum of the last row need the next
 * push and are NaN.  n_tracers and c (per-segment charges) are updated in
 * place when refinement inserts tracers; x_out and v_out then need room for
 * cap entries.  count_out (optional, n_steps + 1 entries) receives the total
 * tracer count after each step.  Returns 0, 1 when out of memory, 2 when
 * refinement would exceed cap tracers (the run stops there). */
static void deposit_by_order(int order, double L, int nc, int n_sheets, const int32_t *n_tracers,
                             const int32_t *closed, const double *c, const double *x, double *Q, double *max_segment)
{
    if (order == 1) orc_deposit_linear_c(L, nc, n_sheets, n_tracers, closed, c, x, Q, max_segment);
    else if (order == 2) orc_deposit_cic_c(L, nc, n_sheets, n_tracers, closed, c, x, Q, max_segment);
    else orc_deposit_c(L, nc, n_sheets, n_tracers, closed, c, x, Q, max_segment);
}

int orc_run_seg(int order, double L, int nc, double dt, int n_sheets, int32_t *n_tracers, const int32_t *closed,
                double *c, const double *x0, const double *v0, int64_t step0, int init_kick, int64_t n_steps,
                double l_max, int64_t cap, double *hist, int64_t *count_out, double *x_out, double *v_out,
                double *Q_out, double *E_out)
{
    int64_t n = 0;
    for (int s = 0; s < n_sheets; ++s) n += n_tracers[s];
    if (cap < n) cap = n;
    double *x = (double *)calloc((size_t)(cap > 0 ? cap : 1), sizeof(double));
    double *v = (double *)calloc((size_t)(cap > 0 ? cap : 1), sizeof(double));
    double *Q = (double *)malloc(sizeof(double) * (size_t)nc);
    double *E = (double *)malloc(sizeof(double) * (size_t)nc);
    if (!x || !v || !Q || !E) { free(x); free(v); free(Q); free(E); return 1; }
    for (int64_t i = 0; i < n; ++i) { x[i] = orc_wrap(x0[i], L); v[i] = v0[i]; }

    int rc = 0;
    double W, qt, ms;
    deposit_by_order(order, L, nc, n_sheets, n_tracers, closed, c, x, Q, &ms);
    orc_solve(L, nc, Q, E, &W, &qt);
    if (init_kick) {
        for (int64_t i = 0; i < n; ++i) v[i] = v[i] - 0.5 * dt * orc_gather(L, nc, E, x[i]);
    }
    double *row = hist;
    row[0] = (double)step0; row[1] = (double)step0 * dt; row[2] = W; row[3] = NAN; row[4] = NAN;
    row[5] = qt; row[6] = ms; row[7] = row_flags(L, nc, E, ms, 1);
    if (count_out) count_out[0] = n;
    for (int64_t it = 0; it < n_steps; ++it) {
        double ke, mom;
        orc_push_c(L, nc, dt, n_sheets, n_tracers, closed, c, E, x, v, &ke, &mom);
        hist[it * ORC_ROW + 3] = ke;
        hist[it * ORC_ROW + 4] = mom;
        if (l_max > 0.0) {
            int64_t added = orc_refine(L, l_max, n_sheets, n_tracers, closed, x, v, c, cap);
            if (added < 0) { rc = 2; break; }
            n += added;
        }
        deposit_by_order(order, L, nc, n_sheets, n_tracers, closed, c, x, Q, &ms);
        orc_solve(L, nc, Q, E, &W, &qt);
        row = hist + (it + 1) * ORC_ROW;
        row[0] = (double)(step0 + it + 1); row[1] = (double)(step0 + it + 1) * dt; row[2] = W;
        row[3] = NAN; row[4] = NAN; row[5] = qt; row[6] = ms;
        row[7] = row_flags(L, nc, E, ms, isfinite(ke) && isfinite(mom));
        if (count_out) count_out[it + 1] = n;
    }
    if (x_out) memcpy(x_out, x, sizeof(double) * (size_t)n);
    if (v_out) memcpy(v_out, v, sizeof(double) * (size_t)n);
    if (Q_out) memcpy(Q_out, Q, sizeof(double) * (size_t)nc);
    if (E_out) memcpy(E_out, E, sizeof(double) * (size_t)nc);
    free(x); free(v); free(Q); free(E);
    return rc;
}

/* The run with every segment of sheet s carrying q_s and no refinement. */
int orc_run_order(int order, double L, int nc, double dt, int n_sheets, const int32_t *n_tracers, const double *q,
                  const int32_t *closed, const double *x0, const double *v0, int64_t step0, int init_kick,
                  int64_t n_steps, double *hist, double *x_out, double *v_out, double *Q_out, double *E_out)
{
    double *c = uniform_charges(n_sheets, n_tracers, q, closed);
    int32_t *nt = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_sheets > 0 ? n_sheets : 1));
    if (!c || !nt) { free(c); free(nt); return 1; }
    memcpy(nt, n_tracers, sizeof(int32_t) * (size_t)n_sheets);
    int rc = orc_run_seg(order, L, nc, dt, n_sheets, nt, closed, c, x0, v0, step0, init_kick, n_steps, 0.0, 0, hist,
                         NULL, x_out, v_out, Q_out, E_out);
    free(c); free(nt);
    return rc;
}

int orc_run(double L, int nc, double dt, int n_sheets, const int32_t *n_tracers, const double *q,
            const int32_t *closed, const double *x0, const double *v0, int64_t step0, int init_kick,
            int64_t n_steps, double *hist, double *x_out, double *v_out, double *Q_out, double *E_out)
{
    return orc_run_order(0, L, nc, dt, n_sheets, n_tracers, q, closed, x0, v0, step0, init_kick, n_steps, hist,
                         x_out, v_out, Q_out, E_out);
}
