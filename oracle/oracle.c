/*
 * oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE LIBRARY.
 *
 * A plain, slow, double-precision CPU implementation of what the stencil
 * library and the ADI Cahn-Hilliard step of "cuSten -- CUDA Finite Difference
 * and Stencil Library" (Gloster, O Naraigh, Pham; arXiv 1902.09931) compute.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no code, header or table with the GPU path.
 *
 * Every function computes the plain definition of its result, in the written
 * order, one output at a time.  It is built with
 *     gcc -O2 -fno-fast-math -ffp-contract=off
 * so that products and sums are rounded separately, in source order.
 *
 * Conventions (readings of the paper where it leaves the choice open):
 *   - grids are row-major, x contiguous: element (j, i) sits at in[j*ld + i]
 *     (x is the contiguous direction and tiles split y, Sec. 2);
 *   - a window with extents left/right (x) and top/bottom (y) has weight
 *     index (b+top)*(left+right+1) + (a+left) for tap (a, b), counted from
 *     the top left, left to right in i, row by row in j (Sec. 5.3); "top" is
 *     the smaller j;
 *   - non-periodic stencils leave the boundary cells of the output untouched
 *     (Sec. 3).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef long long i64;

static i64 wrap_index(i64 k, i64 n)
{
    i64 r = k % n;
    return r < 0 ? r + n : r;
}

/* The point function of the "Fun" variants (Sec. 4.2, Sec. 5.3), in its
 * point-wise polynomial reading: f(c) = sum_m coe[m] c^m, the identity when
 * ncoe == 0.  The cubic of the Cahn-Hilliard term is coe = {0, -1, 0, 1}. */
static double point_fun(double c, const double *coe, int ncoe)
{
    if (ncoe <= 0)
        return c;
    double s = 0.0, p = 1.0;
    for (int m = 0; m < ncoe; ++m) {
        s += coe[m] * p;
        p *= c;
    }
    return s;
}

/* One output of a 2D stencil (Sec. 3): the weighted sum over the window of
 * f(input), with periodic wrap of both indices when periodic != 0. */
static double stencil_point(const double *in, i64 nx, i64 ny, i64 ld,
                            int left, int right, int top, int bottom,
                            const double *w, int periodic,
                            const double *coe, int ncoe, i64 j, i64 i)
{
    const int width = left + right + 1;
    double acc = 0.0;
    for (int b = -top; b <= bottom; ++b) {
        i64 J = periodic ? wrap_index(j + b, ny) : j + b;
        for (int a = -left; a <= right; ++a) {
            i64 I = periodic ? wrap_index(i + a, nx) : i + a;
            double wt = w[(b + top) * width + (a + left)];
            acc += wt * point_fun(in[J * ld + I], coe, ncoe);
        }
    }
    return acc;
}

/* Whether output (j, i) is written: always for periodic stencils; only in the
 * interior for non-periodic ones, whose boundary cells stay untouched
 * (Sec. 3, Sec. 4.1). */
static int is_written(i64 nx, i64 ny, int left, int right, int top,
                      int bottom, int periodic, i64 j, i64 i)
{
    if (periodic)
        return 1;
    return i >= left && i <= nx - 1 - right && j >= top && j <= ny - 1 - bottom;
}

static int check_extents(i64 nx, i64 ny, i64 ld, int left, int right,
                         int top, int bottom)
{
    if (nx <= 0 || ny <= 0 || ld < nx)
        return -1;
    if (left < 0 || right < 0 || top < 0 || bottom < 0)
        return -1;
    if (left + right >= nx || top + bottom >= ny)
        return -1;
    return 0;
}

/* 2D stencil over a whole grid: directions X (top = bottom = 0), Y
 * (left = right = 0) and XY, periodic or non-periodic, weights or point
 * function (Sec. 3, Sec. 4.1, Sec. 4.2). */
int orc_stencil2d(const double *in, double *out, i64 nx, i64 ny, i64 ld,
                  int left, int right, int top, int bottom,
                  const double *weights, int periodic,
                  const double *coe, int ncoe)
{
    if (check_extents(nx, ny, ld, left, right, top, bottom))
        return -1;
    for (i64 j = 0; j < ny; ++j)
        for (i64 i = 0; i < nx; ++i)
            if (is_written(nx, ny, left, right, top, bottom, periodic, j, i))
                out[j * ld + i] = stencil_point(in, nx, ny, ld, left, right,
                                                top, bottom, weights, periodic,
                                                coe, ncoe, j, i);
    return 0;
}

/* The same definition evaluated at npts chosen points (j[k], i[k]); written[k]
 * says whether the library writes that output at all. */
int orc_stencil2d_at(const double *in, i64 nx, i64 ny, i64 ld,
                     int left, int right, int top, int bottom,
                     const double *weights, int periodic,
                     const double *coe, int ncoe,
                     i64 npts, const i64 *js, const i64 *is,
                     double *vals, int *written)
{
    if (check_extents(nx, ny, ld, left, right, top, bottom))
        return -1;
    for (i64 k = 0; k < npts; ++k) {
        written[k] = is_written(nx, ny, left, right, top, bottom, periodic,
                                js[k], is[k]);
        vals[k] = written[k]
            ? stencil_point(in, nx, ny, ld, left, right, top, bottom,
                            weights, periodic, coe, ncoe, js[k], is[k])
            : 0.0;
    }
    return 0;
}

/* Batched 1D stencils over uneven signals stored back to back: signal b
 * occupies [offsets[b], offsets[b+1]) and wraps onto itself when periodic
 * (the batched 1D form named in the abstract).  Each signal is the 2D X
 * stencil on a grid of one row. */
int orc_stencil1d_batch(const double *in, double *out, const i64 *offsets,
                        i64 nbatch, int left, int right,
                        const double *weights, int periodic,
                        const double *coe, int ncoe)
{
    for (i64 b = 0; b < nbatch; ++b) {
        i64 base = offsets[b];
        i64 n = offsets[b + 1] - offsets[b];
        if (check_extents(n, 1, n, left, right, 0, 0))
            return -1;
        for (i64 i = 0; i < n; ++i)
            if (is_written(n, 1, left, right, 0, 0, periodic, 0, i))
                out[base + i] = stencil_point(in + base, n, 1, n, left, right,
                                              0, 0, weights, periodic, coe,
                                              ncoe, 0, i);
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Cyclic banded solve.
 *
 * A is the n x n circulant whose row i holds a[d + bw] in column (i + d) mod
 * n for d = -bw..bw; it is the matrix of the periodic stencil with weights a,
 * and the matrix of the periodic line inversions of the ADI step (Sec. 5.1).
 * The solve splits A = T + E: T is the banded, non-wrapping part and E holds
 * the 2*bw wrapped corner rows.  T is factored by banded LU without pivoting
 * (Doolittle), and E is folded back with the Sherman-Morrison-Woodbury
 * formula
 *     A^-1 r = y - Z (I + W Z)^-1 W y,   y = T^-1 r,  Z = T^-1 U,
 * where E = U W, U holds the unit columns of the corner rows and W those
 * rows of E.  The small 2bw x 2bw system is solved by Gaussian elimination
 * with partial pivoting.  Requires n >= 2*bw + 1.
 * ------------------------------------------------------------------------- */

typedef struct {
    int n, bw;
    double *band; /* band[i*(2bw+1) + (j - i + bw)] = T[i][j], |j - i| <= bw */
} banded_t;

static double *band_at(banded_t *t, i64 i, i64 j)
{
    return &t->band[i * (2 * t->bw + 1) + (j - i + t->bw)];
}

/* LU factorisation in place, without pivoting: L unit lower (stored below
 * the diagonal), U upper. */
static int banded_lu(banded_t *t)
{
    const int n = t->n, bw = t->bw;
    for (i64 k = 0; k < n; ++k) {
        double piv = *band_at(t, k, k);
        if (piv == 0.0)
            return -1;
        i64 iend = k + bw < n - 1 ? k + bw : n - 1;
        for (i64 i = k + 1; i <= iend; ++i) {
            double l = *band_at(t, i, k) / piv;
            *band_at(t, i, k) = l;
            for (i64 j = k + 1; j <= iend; ++j)
                *band_at(t, i, j) -= l * *band_at(t, k, j);
        }
    }
    return 0;
}

/* Solve L U y = r in place (r becomes y). */
static void banded_lu_solve(banded_t *t, double *y)
{
    const int n = t->n, bw = t->bw;
    for (i64 i = 0; i < n; ++i) {
        i64 j0 = i - bw > 0 ? i - bw : 0;
        double s = y[i];
        for (i64 j = j0; j < i; ++j)
            s -= *band_at(t, i, j) * y[j];
        y[i] = s;
    }
    for (i64 i = n - 1; i >= 0; --i) {
        i64 j1 = i + bw < n - 1 ? i + bw : n - 1;
        double s = y[i];
        for (i64 j = i + 1; j <= j1; ++j)
            s -= *band_at(t, i, j) * y[j];
        y[i] = s / *band_at(t, i, i);
    }
}

/* Dense m x m solve by Gaussian elimination with partial pivoting; H and g
 * are overwritten, the solution is returned in g. */
static int dense_solve(int m, double *H, double *g)
{
    for (int k = 0; k < m; ++k) {
        int p = k;
        for (int i = k + 1; i < m; ++i)
            if (fabs(H[i * m + k]) > fabs(H[p * m + k]))
                p = i;
        if (H[p * m + k] == 0.0)
            return -1;
        if (p != k) {
            for (int j = 0; j < m; ++j) {
                double tmp = H[k * m + j];
                H[k * m + j] = H[p * m + j];
                H[p * m + j] = tmp;
            }
            double tmp = g[k];
            g[k] = g[p];
            g[p] = tmp;
        }
        for (int i = k + 1; i < m; ++i) {
            double l = H[i * m + k] / H[k * m + k];
            for (int j = k; j < m; ++j)
                H[i * m + j] -= l * H[k * m + j];
            g[i] -= l * g[k];
        }
    }
    for (int i = m - 1; i >= 0; --i) {
        double s = g[i];
        for (int j = i + 1; j < m; ++j)
            s -= H[i * m + j] * g[j];
        g[i] = s / H[i * m + i];
    }
    return 0;
}

/* Solve the cyclic banded system A x = r for one line of length n, reading r
 * and writing x with element stride `stride`. */
static int cyclic_solve_line(int bw, const double *a, int n, const double *r,
                             i64 rstride, double *x, i64 xstride)
{
    if (bw < 1 || n < 2 * bw + 1)
        return -1;
    const int q = 2 * bw; /* number of corner rows */
    banded_t t;
    t.n = n;
    t.bw = bw;
    t.band = (double *)calloc((size_t)n * (2 * bw + 1), sizeof(double));
    double *y = (double *)malloc(sizeof(double) * n);
    double *Z = (double *)calloc((size_t)n * q, sizeof(double));
    double *H = (double *)malloc(sizeof(double) * q * q);
    double *g = (double *)malloc(sizeof(double) * q);
    int rows[8];
    int st = -1;
    if (!t.band || !y || !Z || !H || !g || q > 8)
        goto done;

    /* T: the band of A without the wrapped entries. */
    for (i64 i = 0; i < n; ++i)
        for (int d = -bw; d <= bw; ++d)
            if (i + d >= 0 && i + d < n)
                *band_at(&t, i, i + d) = a[d + bw];
    if (banded_lu(&t))
        goto done;

    /* Corner rows: the first bw rows wrap to the right end, the last bw rows
     * wrap to the left end. */
    for (int k = 0; k < bw; ++k) {
        rows[k] = k;
        rows[bw + k] = n - bw + k;
    }

    /* y = T^-1 r */
    for (i64 i = 0; i < n; ++i)
        y[i] = r[i * rstride];
    banded_lu_solve(&t, y);

    /* Z = T^-1 U, one column per corner row */
    for (int k = 0; k < q; ++k) {
        double *z = Z + (i64)k * n;
        z[rows[k]] = 1.0;
        banded_lu_solve(&t, z);
    }

    /* H = I + W Z and g = W y, where row k of W is the wrapped part of row
     * rows[k] of A. */
    for (int k = 0; k < q; ++k) {
        i64 i = rows[k];
        for (int c = 0; c < q; ++c)
            H[k * q + c] = (k == c) ? 1.0 : 0.0;
        g[k] = 0.0;
        for (int d = -bw; d <= bw; ++d) {
            i64 col = i + d;
            if (col >= 0 && col < n)
                continue; /* in T, not in E */
            col = wrap_index(col, n);
            double e = a[d + bw];
            for (int c = 0; c < q; ++c)
                H[k * q + c] += e * Z[(i64)c * n + col];
            g[k] += e * y[col];
        }
    }
    if (dense_solve(q, H, g))
        goto done;

    /* x = y - Z h */
    for (i64 i = 0; i < n; ++i) {
        double s = y[i];
        for (int c = 0; c < q; ++c)
            s -= Z[(i64)c * n + i] * g[c];
        x[i * xstride] = s;
    }
    st = 0;
done:
    free(t.band);
    free(y);
    free(Z);
    free(H);
    free(g);
    return st;
}

/* Batched cyclic solves over uneven lines stored back to back (line b is
 * [offsets[b], offsets[b+1])). a holds the 2*bw+1 band values a[-bw..bw]. */
int orc_cyclic_solve_batch(int bw, const double *a, const i64 *offsets,
                           i64 nbatch, const double *r, double *x)
{
    for (i64 b = 0; b < nbatch; ++b) {
        i64 base = offsets[b];
        int n = (int)(offsets[b + 1] - offsets[b]);
        if (cyclic_solve_line(bw, a, n, r + base, 1, x + base, 1))
            return -1;
    }
    return 0;
}

/* Cyclic solves along every row (axis = 0) or every column (axis = 1) of an
 * nx x ny grid with row pitch ld. */
int orc_cyclic_solve_grid(int bw, const double *a, int axis, i64 nx, i64 ny,
                          i64 ld, const double *r, double *x)
{
    if (axis == 0) {
        for (i64 j = 0; j < ny; ++j)
            if (cyclic_solve_line(bw, a, (int)nx, r + j * ld, 1, x + j * ld, 1))
                return -1;
    } else {
        for (i64 i = 0; i < nx; ++i)
            if (cyclic_solve_line(bw, a, (int)ny, r + i, ld, x + i, ld))
                return -1;
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * One step of the ADI scheme for the Cahn-Hilliard equation (Sec. 5, the
 * equation dC/dt = D lap(C^3 - C - gamma lap C) and its ADI discretisation),
 * on an nx x ny periodic grid with spacings dx, dy:
 *
 *   Cbar = 2 C^n - C^{n-1}                                    (reading)
 *   R    = -2/3 (C^n - C^{n-1}) - 2/3 D gamma dt lap_h^2 Cbar
 *          + 2/3 D dt lap_h (C^3 - C)^n                       (reading: D gamma)
 *   L_x w = R on every row,  L_y v = w on every column,
 *   L_x = I + 2/3 D gamma dt d_xxxx  (periodic pentadiagonal),
 *   C^{n+1} = Cbar + v.
 *
 * lap_h is the 5-point second-order Laplacian and lap_h^2 the 13-point
 * biharmonic d_xxxx + 2 d_xxyy + d_yyyy, both written as 5x5 windows from
 * the second-order central differences of Sec. 5.1 and the cross stencil of
 * Fig. 1.  nonlinear = 0 drops the cubic term, leaving the scheme for linear
 * hyperdiffusion on which the paper's method is built (Sec. 5.1).
 * ------------------------------------------------------------------------- */

/* 5x5 biharmonic window: d_xxxx on the centre row, d_yyyy on the centre
 * column, twice the Fig. 1 cross stencil on the centre 3x3 block. */
static void biharmonic_5x5(double dx, double dy, double *w)
{
    static const double d4[5] = {1.0, -4.0, 6.0, -4.0, 1.0};
    static const double fig1[3][3] = {{1.0, -2.0, 1.0},
                                      {-2.0, 4.0, -2.0},
                                      {1.0, -2.0, 1.0}};
    const double dx4 = dx * dx * dx * dx, dy4 = dy * dy * dy * dy;
    const double dxdy2 = dx * dx * dy * dy;
    memset(w, 0, sizeof(double) * 25);
    for (int k = 0; k < 5; ++k) {
        w[2 * 5 + k] += d4[k] / dx4;
        w[k * 5 + 2] += d4[k] / dy4;
    }
    for (int b = 0; b < 3; ++b)
        for (int c = 0; c < 3; ++c)
            w[(b + 1) * 5 + (c + 1)] += 2.0 * fig1[b][c] / dxdy2;
}

/* 5x5 window holding the 5-point Laplacian (Sec. 5.1 second derivatives in
 * x and in y). */
static void laplacian_5x5(double dx, double dy, double *w)
{
    static const double d2[3] = {1.0, -2.0, 1.0};
    memset(w, 0, sizeof(double) * 25);
    for (int k = 0; k < 3; ++k) {
        w[2 * 5 + (k + 1)] += d2[k] / (dx * dx);
        w[(k + 1) * 5 + 2] += d2[k] / (dy * dy);
    }
}

/* Rounding of a double to the nearest float (ties to even), and to the
 * nearest bfloat16 (8 significant bits, the exponent range of float; ties to
 * even), each in one step from the double value.  Used by the stored-
 * precision form of the step below. */
static double round_f32(double v)
{
    return (double)(float)v;
}

static double round_bf16(double v)
{
    if (v == 0.0 || !isfinite(v))
        return v;
    int e;
    double m = frexp(v, &e); /* v = m 2^e, 0.5 <= |m| < 1 */
    if (e - 1 < -126)        /* below the smallest normal: fixed spacing 2^-133 */
        return ldexp(nearbyint(ldexp(v, 133)), -133);
    return ldexp(nearbyint(ldexp(m, 8)), e - 8);
}

static double round_storage(double v, int storage)
{
    return storage == 1 ? round_f32(v) : storage == 2 ? round_bf16(v) : v;
}

static int ch_step_impl(i64 nx, i64 ny, double dx, double dy, double dt,
                        double D, double gamma, int nonlinear, int storage,
                        unsigned long long nudge, const double *c_prev,
                        const double *c_cur, double *c_next);

/* Every nonzero coefficient w moved by one unit in the last place, up or
 * down by the bits of a splitmix64 sequence started at seed (nudge = 0:
 * unchanged).  A double evaluation of the scheme must round its window
 * weights and band values; this gives another equally valid rounding, for
 * measuring how far two such evaluations drift apart. */
static unsigned long long splitmix64(unsigned long long *x)
{
    unsigned long long z = (*x += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static void nudge_ulp(double *w, int n, unsigned long long *state)
{
    for (int k = 0; k < n; ++k)
        if (w[k] != 0.0)
            w[k] = nextafter(w[k], (splitmix64(state) & 1) ? INFINITY : -INFINITY);
}

int orc_ch_step(i64 nx, i64 ny, double dx, double dy, double dt, double D,
                double gamma, int nonlinear, const double *c_prev,
                const double *c_cur, double *c_next)
{
    return ch_step_impl(nx, ny, dx, dy, dt, D, gamma, nonlinear, 0, 0, c_prev,
                        c_cur, c_next);
}

/* The same step with the stored quantities rounded as a reduced-precision
 * implementation stores them (the mixed-precision reading: state fields in
 * the storage dtype, intermediate right-hand side and x-sweep result in
 * float, all arithmetic in double): storage = 1 (float state) or 2
 * (bfloat16 state); R and w are rounded to float, C^{n+1} to the storage
 * dtype.  storage = 0 is orc_ch_step. */
int orc_ch_step_stored(i64 nx, i64 ny, double dx, double dy, double dt,
                       double D, double gamma, int nonlinear, int storage,
                       const double *c_prev, const double *c_cur,
                       double *c_next)
{
    if (storage < 0 || storage > 2)
        return -1;
    return ch_step_impl(nx, ny, dx, dy, dt, D, gamma, nonlinear, storage, 0,
                        c_prev, c_cur, c_next);
}

static int ch_step_impl(i64 nx, i64 ny, double dx, double dy, double dt,
                        double D, double gamma, int nonlinear, int storage,
                        unsigned long long nudge, const double *c_prev,
                        const double *c_cur, double *c_next)
{
    const i64 npts = nx * ny;
    if (nx < 5 || ny < 5)
        return -1;
    double *cbar = (double *)malloc(sizeof(double) * npts);
    double *bih = (double *)malloc(sizeof(double) * npts);
    double *lap = (double *)malloc(sizeof(double) * npts);
    double *rhs = (double *)malloc(sizeof(double) * npts);
    double *w = (double *)malloc(sizeof(double) * npts);
    double *v = (double *)malloc(sizeof(double) * npts);
    double wb[25], wl[25];
    static const double cubic[4] = {0.0, -1.0, 0.0, 1.0};
    int st = -1;
    if (!cbar || !bih || !lap || !rhs || !w || !v)
        goto done;

    for (i64 k = 0; k < npts; ++k)
        cbar[k] = 2.0 * c_cur[k] - c_prev[k];

    biharmonic_5x5(dx, dy, wb);
    laplacian_5x5(dx, dy, wl);
    unsigned long long nstate = nudge;
    if (nudge) {
        nudge_ulp(wb, 25, &nstate);
        nudge_ulp(wl, 25, &nstate);
    }
    if (orc_stencil2d(cbar, bih, nx, ny, nx, 2, 2, 2, 2, wb, 1, NULL, 0))
        goto done;
    if (nonlinear) {
        if (orc_stencil2d(c_cur, lap, nx, ny, nx, 2, 2, 2, 2, wl, 1, cubic, 4))
            goto done;
    } else {
        for (i64 k = 0; k < npts; ++k)
            lap[k] = 0.0;
    }

    const double a = 2.0 / 3.0 * D * gamma * dt;
    for (i64 k = 0; k < npts; ++k)
        rhs[k] = -2.0 / 3.0 * (c_cur[k] - c_prev[k]) - a * bih[k]
                 + 2.0 / 3.0 * D * dt * lap[k];
    if (storage)
        for (i64 k = 0; k < npts; ++k)
            rhs[k] = round_f32(rhs[k]);

    {
        const double bx = a / (dx * dx * dx * dx);
        const double by = a / (dy * dy * dy * dy);
        double lx[5] = {bx, -4.0 * bx, 1.0 + 6.0 * bx, -4.0 * bx, bx};
        double ly[5] = {by, -4.0 * by, 1.0 + 6.0 * by, -4.0 * by, by};
        if (nudge) {
            /* symmetric bands stay symmetric */
            double hx[3] = {lx[2], lx[1], lx[0]}, hy[3] = {ly[2], ly[1], ly[0]};
            nudge_ulp(hx, 3, &nstate);
            nudge_ulp(hy, 3, &nstate);
            lx[2] = hx[0]; lx[1] = lx[3] = hx[1]; lx[0] = lx[4] = hx[2];
            ly[2] = hy[0]; ly[1] = ly[3] = hy[1]; ly[0] = ly[4] = hy[2];
        }
        if (orc_cyclic_solve_grid(2, lx, 0, nx, ny, nx, rhs, w))
            goto done;
        if (storage)
            for (i64 k = 0; k < npts; ++k)
                w[k] = round_f32(w[k]);
        if (orc_cyclic_solve_grid(2, ly, 1, nx, ny, nx, w, v))
            goto done;
    }

    for (i64 k = 0; k < npts; ++k)
        c_next[k] = round_storage(cbar[k] + v[k], storage);
    st = 0;
done:
    free(cbar);
    free(bih);
    free(lap);
    free(rhs);
    free(w);
    free(v);
    return st;
}

/* nsteps steps of orc_ch_step_stored, rotating the two time levels; on
 * return c_prev/c_cur hold C^{n-1}, C^n of the last step. */
int orc_ch_run_stored(i64 nx, i64 ny, double dx, double dy, double dt,
                      double D, double gamma, int nonlinear, int storage,
                      i64 nsteps, double *c_prev, double *c_cur)
{
    const i64 npts = nx * ny;
    double *nxt = (double *)malloc(sizeof(double) * npts);
    if (!nxt)
        return -1;
    for (i64 s = 0; s < nsteps; ++s) {
        if (orc_ch_step_stored(nx, ny, dx, dy, dt, D, gamma, nonlinear,
                               storage, c_prev, c_cur, nxt)) {
            free(nxt);
            return -1;
        }
        memcpy(c_prev, c_cur, sizeof(double) * npts);
        memcpy(c_cur, nxt, sizeof(double) * npts);
    }
    free(nxt);
    return 0;
}

/* nsteps steps of the double step with every window weight and band value
 * moved by one ulp (nudge_ulp, seed != 0), the same coefficients at every
 * step: another equally valid double rounding of the scheme's
 * coefficients. */
int orc_ch_run_nudged(i64 nx, i64 ny, double dx, double dy, double dt,
                      double D, double gamma, int nonlinear, i64 nsteps,
                      unsigned long long seed, double *c_prev, double *c_cur)
{
    const i64 npts = nx * ny;
    if (!seed)
        return -1;
    double *nxt = (double *)malloc(sizeof(double) * npts);
    if (!nxt)
        return -1;
    for (i64 s = 0; s < nsteps; ++s) {
        if (ch_step_impl(nx, ny, dx, dy, dt, D, gamma, nonlinear, 0, seed,
                         c_prev, c_cur, nxt)) {
            free(nxt);
            return -1;
        }
        memcpy(c_prev, c_cur, sizeof(double) * npts);
        memcpy(c_cur, nxt, sizeof(double) * npts);
    }
    free(nxt);
    return 0;
}

/* nsteps steps of orc_ch_step (double precision throughout). */
int orc_ch_run(i64 nx, i64 ny, double dx, double dy, double dt, double D,
               double gamma, int nonlinear, i64 nsteps, double *c_prev,
               double *c_cur)
{
    return orc_ch_run_stored(nx, ny, dx, dy, dt, D, gamma, nonlinear, 0,
                             nsteps, c_prev, c_cur);
}

/* The rounding of n values to a storage dtype as the stored-precision step
 * applies it (storage = 1 float, 2 bfloat16); exported for its pins. */
int orc_round_storage(const double *x, double *y, i64 n, int storage)
{
    if (storage < 1 || storage > 2)
        return -1;
    for (i64 k = 0; k < n; ++k)
        y[k] = round_storage(x[k], storage);
    return 0;
}

/* Sum of n values with Neumaier's compensated summation: the grid mass
 * M = sum_ij C_ij that the periodic scheme conserves (Sec. 5, mass
 * conservation of the model). */
double orc_sum(const double *x, i64 n)
{
    double s = 0.0, c = 0.0;
    for (i64 k = 0; k < n; ++k) {
        double t = s + x[k];
        if (fabs(s) >= fabs(x[k]))
            c += (s - t) + x[k];
        else
            c += (x[k] - t) + s;
        s = t;
    }
    return s + c;
}

/* ------------------------------------------------------------------------
 * WENO advection (the 2D periodic xy advection variant of Sec. 4.3).
 *
 * The variant replaces the weighted sum of the periodic XY stencil with a
 * WENO evaluation of the advection term and takes the velocities u, v as
 * extra inputs.  Reading: out = u phi_x + v phi_y at every grid point of a
 * periodic grid, each derivative the fifth-order Hamilton-Jacobi WENO
 * approximation of the level-set text the section cites (Osher and Fedkiw,
 * "Level Set Methods and Dynamic Implicit Surfaces", Sec. 3.4, after Jiang
 * and Peng), upwinded by the sign of the velocity: phi_x^- (built from the
 * backward differences D^- at i-2 .. i+2) where u > 0, phi_x^+ (forward
 * differences D^+ at i+2 .. i-2) where u < 0, and likewise in y with v.
 * Where the velocity is zero its term is zero whichever side is taken.
 * ---------------------------------------------------------------------- */

/* The WENO combination of five consecutive one-sided differences v1..v5
 * (ordered away from the upwind side, v3 the difference at the point). */
static double weno5(double v1, double v2, double v3, double v4, double v5)
{
    /* the three third-order ENO candidates */
    double p1 = v1 / 3.0 - 7.0 * v2 / 6.0 + 11.0 * v3 / 6.0;
    double p2 = -v2 / 6.0 + 5.0 * v3 / 6.0 + v4 / 3.0;
    double p3 = v3 / 3.0 + 5.0 * v4 / 6.0 - v5 / 6.0;
    /* their smoothness indicators */
    double a = v1 - 2.0 * v2 + v3, b = v1 - 4.0 * v2 + 3.0 * v3;
    double s1 = 13.0 / 12.0 * (a * a) + 0.25 * (b * b);
    a = v2 - 2.0 * v3 + v4;
    b = v2 - v4;
    double s2 = 13.0 / 12.0 * (a * a) + 0.25 * (b * b);
    a = v3 - 2.0 * v4 + v5;
    b = 3.0 * v3 - 4.0 * v4 + v5;
    double s3 = 13.0 / 12.0 * (a * a) + 0.25 * (b * b);
    /* epsilon scaled by the largest squared difference, plus a floor */
    double m = v1 * v1;
    if (v2 * v2 > m) m = v2 * v2;
    if (v3 * v3 > m) m = v3 * v3;
    if (v4 * v4 > m) m = v4 * v4;
    if (v5 * v5 > m) m = v5 * v5;
    double eps = 1e-6 * m + 1e-99;
    double d1 = s1 + eps, d2 = s2 + eps, d3 = s3 + eps;
    double a1 = 0.1 / (d1 * d1), a2 = 0.6 / (d2 * d2), a3 = 0.3 / (d3 * d3);
    double sum = a1 + a2 + a3;
    double w1 = a1 / sum, w2 = a2 / sum, w3 = a3 / sum;
    return w1 * p1 + w2 * p2 + w3 * p3;
}

/* The upwind WENO derivative of a periodic line f[0 .. n-1] with spacing h at
 * index k, in the stride s of the grid: the backward-biased value when
 * upwind_left != 0, else the forward-biased one. */
static double weno_derivative(const double *f, i64 n, i64 s, double h, i64 k,
                              int upwind_left)
{
    double d[5];
    for (int q = 0; q < 5; ++q) {
        if (upwind_left) {
            /* D^- phi at k-2+q: (phi_{k-2+q} - phi_{k-3+q}) / h */
            i64 hi = wrap_index(k - 2 + q, n), lo = wrap_index(k - 3 + q, n);
            d[q] = (f[hi * s] - f[lo * s]) / h;
        } else {
            /* D^+ phi at k+2-q: (phi_{k+3-q} - phi_{k+2-q}) / h */
            i64 hi = wrap_index(k + 3 - q, n), lo = wrap_index(k + 2 - q, n);
            d[q] = (f[hi * s] - f[lo * s]) / h;
        }
    }
    return weno5(d[0], d[1], d[2], d[3], d[4]);
}

int orc_weno_adv(const double *phi, const double *u, const double *v,
                 double *out, i64 nx, i64 ny, i64 ld, double dx, double dy)
{
    if (nx < 6 || ny < 6 || ld < nx || !(dx > 0) || !(dy > 0))
        return -1;
    for (i64 j = 0; j < ny; ++j)
        for (i64 i = 0; i < nx; ++i) {
            double uu = u[j * ld + i], vv = v[j * ld + i];
            double px = weno_derivative(phi + j * ld, nx, 1, dx, i, uu > 0.0);
            double py = weno_derivative(phi + i, ny, ld, dy, j, vv > 0.0);
            out[j * ld + i] = uu * px + vv * py;
        }
    return 0;
}

/* The upwind WENO derivatives themselves at every point (test access):
 * dx_out = phi_x on the side the sign of u selects, dy_out likewise. */
int orc_weno_derivatives(const double *phi, const double *u, const double *v,
                         double *dx_out, double *dy_out, i64 nx, i64 ny,
                         i64 ld, double dx, double dy)
{
    if (nx < 6 || ny < 6 || ld < nx || !(dx > 0) || !(dy > 0))
        return -1;
    for (i64 j = 0; j < ny; ++j)
        for (i64 i = 0; i < nx; ++i) {
            dx_out[j * ld + i] = weno_derivative(phi + j * ld, nx, 1, dx, i, u[j * ld + i] > 0.0);
            dy_out[j * ld + i] = weno_derivative(phi + i, ny, ld, dy, j, v[j * ld + i] > 0.0);
        }
    return 0;
}
