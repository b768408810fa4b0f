/*
 * mxsten.h -- C ABI of the MI355X (gfx950) stencil and ADI line-solve library.
 *
 * The operations follow "cuSten -- CUDA Finite Difference and Stencil
 * Library" (Gloster, O Naraigh, Pham; arXiv 1902.09931):
 *   - 2D stencils in the x, y and xy directions, periodic or non-periodic,
 *     with fixed weights or a point function (Sec. 3, Sec. 4.1, Sec. 4.2),
 *     through the Create / Compute / Swap / Destroy life cycle of Sec. 3;
 *   - batched 1D stencils over uneven signals (the batched 1D form of the
 *     abstract);
 *   - the periodic banded line inversions of the ADI scheme (Sec. 5.1), and
 *     the whole ADI Cahn-Hilliard step built from them (Sec. 5.1, Sec. 5.2),
 *     for one grid or an ensemble of grids.
 *
 * Conventions common to every call:
 *   - Grids are row-major with x contiguous: element (j, i) of a grid with
 *     row pitch ld sits at base[j*ld + i] (x contiguous, tiles split y:
 *     Sec. 2).  j is the y index, i the x index; "top" means smaller j.
 *   - Storage dtypes: MXS_F64 (double, arithmetic in double), MXS_F32
 *     (float, arithmetic in float), MXS_BF16 (bfloat16 bits in uint16_t,
 *     arithmetic in float, results rounded to nearest even).  Line
 *     eliminations always run in double.
 *   - Pointers marked "device" are HIP device pointers; the caller owns
 *     them and keeps them alive while a plan uses them.  Pointers marked
 *     "host" are read during the call only (the plan keeps its own copies).
 *   - Streams are hipStream_t values passed as void*; NULL is the default
 *     stream.  Compute and step calls only enqueue work; they return before
 *     it finishes.  Only mxs_ch_mass, mxs_ch_coarsening and mxs_autotune
 *     wait for their stream.
 *   - Every call returns an mxs_status.  No call aborts or prints; on error
 *     mxs_last_error() returns a message for the calling thread.
 *   - Plans are not thread-safe: one plan is used by one thread at a time.
 */
#ifndef MXSTEN_H
#define MXSTEN_H

#ifdef __cplusplus
extern "C" {
#endif

typedef int mxs_status;

enum {
    MXS_OK = 0,
    MXS_ERR_INVALID_ARG = -1,  /* a size, extent, pointer or enum is out of range */
    MXS_ERR_ALIAS = -2,        /* input and output overlap (forbidden, Sec. 2) */
    MXS_ERR_UNSUPPORTED = -3,  /* valid but outside what the library implements */
    MXS_ERR_HIP = -4,          /* a HIP runtime call failed */
    MXS_ERR_OOM = -5,          /* device or host allocation failed */
    MXS_ERR_NONFINITE = -6,    /* a reduction found NaN or Inf */
    MXS_ERR_BAD_HANDLE = -7    /* NULL, destroyed or wrong-kind plan */
};

typedef struct mxs_plan_s *mxs_plan;

enum { MXS_X = 0, MXS_Y = 1, MXS_XY = 2 };          /* stencil direction (Sec. 3) */
enum { MXS_NP = 0, MXS_P = 1 };                     /* non-periodic / periodic (Sec. 3) */
enum { MXS_F64 = 0, MXS_F32 = 1, MXS_BF16 = 2 };    /* storage dtype */
enum { MXS_LINES_RAGGED = 0, MXS_LINES_ROWS = 1, MXS_LINES_COLS = 2 };  /* solve geometry */

/* Largest supported window: 17 taps along x for MXS_X, 17 along y for
 * MXS_Y, 9 x 9 for MXS_XY.  Largest point-function polynomial: 8
 * coefficients. */
#define MXS_MAX_TAPS_1D 17
#define MXS_MAX_TAPS_XY 9
#define MXS_MAX_COE 8

/* ------------------------------------------------------------------------
 * 2D stencils (Sec. 3).
 *
 *   out[j][i] = sum_{b=-top..bottom} sum_{a=-left..right}
 *                  weights[(b+top)*(left+right+1) + (a+left)] * f(in[j+b][i+a])
 *
 * The window is indexed from its top left, left to right in i, row by row
 * in j (Sec. 5.3).  f(c) = sum_m coe[m] c^m when ncoe > 0 (the point-function
 * form of the Fun variants, Sec. 4.2 and Sec. 5.3), else f(c) = c.
 * Periodic: indices wrap modulo nx and ny.  Non-periodic: only outputs with
 * left <= i <= nx-1-right and top <= j <= ny-1-bottom are written; the
 * boundary cells of out are left untouched (Sec. 3).
 * MXS_X requires top = bottom = 0, MXS_Y requires left = right = 0.
 * Requires left+right < nx, top+bottom < ny, ld >= nx, and in and out not
 * overlapping (MXS_ERR_ALIAS): the windows of neighbouring outputs overlap,
 * so the output cannot overwrite the input (Sec. 2).
 * Inputs must be finite: a padded tap of weight zero still reads the grid.
 * ---------------------------------------------------------------------- */
typedef struct {
    int nx, ny;              /* grid extents (x contiguous) */
    long long ld;            /* row pitch in elements, >= nx */
    int dir;                 /* MXS_X, MXS_Y or MXS_XY */
    int bc;                  /* MXS_NP or MXS_P */
    int dtype;               /* storage dtype of in and out */
    int left, right;         /* x extents of the window */
    int top, bottom;         /* y extents of the window */
    const double *weights;   /* host, (left+right+1)*(top+bottom+1) values */
    const double *coe;       /* host, ncoe point-function coefficients, or NULL */
    int ncoe;                /* 0 .. MXS_MAX_COE */
    const void *in;          /* device, ny rows of pitch ld */
    void *out;               /* device, ny rows of pitch ld */
} mxs_stencil2d_desc;

/* Create a plan for one 2D stencil (cuStenCreate2D*, Sec. 3). */
mxs_status mxs_create_2d(const mxs_stencil2d_desc *desc, mxs_plan *plan);

/* ------------------------------------------------------------------------
 * 2D stencils with a user function (the function-pointer variants of
 * Sec. 4.2, one data set per input as in their multi-input forms).  The
 * function is given as HIP source and compiled for the device when the plan
 * is created (hipRTC); it must define
 *
 *   __device__ mxs_real NAME(const mxs_real *const *w, const mxs_real *coe,
 *                            int loc);
 *
 * where mxs_real is double for MXS_F64 and float for MXS_F32 / MXS_BF16
 * (the library defines it before the source), w[k] is the window of input k
 * in window order ((top+bottom+1)*(left+right+1) values, row by row from the
 * top left, left to right: element (b+top)*(left+right+1) + (a+left) is the
 * input at offset (a, b)), coe the coefficients and loc = top*(left+right+1)
 * + left the position of the point itself, so that the function can index
 * relative to loc as the paper's does.  The return value is stored, rounded
 * to the storage dtype, at the point.  Periodic: every index wraps.
 * Non-periodic: only points whose window lies inside the grid are written;
 * the others are left untouched.  Every input and the output share nx, ny,
 * ld and dtype; out must not overlap an input.  A source that does not
 * compile returns MXS_ERR_INVALID_ARG with the compiler's log in
 * mxs_last_error().  mxs_compute runs it; mxs_swap exchanges input 0 and
 * out; mxs_set_io rebinds input 0 and out.
 * ---------------------------------------------------------------------- */
#define MXS_MAX_FN_INPUTS 4
#define MXS_MAX_FN_COE 64
typedef struct {
    int nx, ny;                  /* grid extents (x contiguous) */
    long long ld;                /* row pitch in elements, >= nx */
    int dir;                     /* MXS_X, MXS_Y or MXS_XY */
    int bc;                      /* MXS_NP or MXS_P */
    int dtype;                   /* storage dtype of every input and out */
    int left, right;             /* x extents of the window */
    int top, bottom;             /* y extents of the window */
    int ninputs;                 /* 1 .. MXS_MAX_FN_INPUTS */
    const void *const *inputs;   /* host array of ninputs device pointers */
    void *out;                   /* device */
    const double *coe;           /* host, ncoe coefficients (copied), or NULL */
    int ncoe;                    /* 0 .. MXS_MAX_FN_COE */
    const char *source;          /* HIP source defining the function */
    const char *name;            /* the function's name (an identifier) */
} mxs_stencil2d_fn_desc;

mxs_status mxs_create_2d_fn(const mxs_stencil2d_fn_desc *desc, mxs_plan *plan);

/* ------------------------------------------------------------------------
 * Batched 1D stencils over nbatch uneven signals stored back to back:
 * signal b is in[offsets[b] .. offsets[b+1]-1] (the batched 1D form of the
 * abstract).  Each signal is the MXS_X stencil of a one-row grid of length
 * n_b = offsets[b+1]-offsets[b]; periodic signals wrap onto themselves.
 * offsets: host, nbatch+1 non-decreasing values, offsets[0] = 0; every
 * n_b > left+right.  left+right+1 <= MXS_MAX_TAPS_1D.
 * ---------------------------------------------------------------------- */
mxs_status mxs_create_1d_batch(int nbatch, const long long *offsets, int bc,
                               int dtype, int left, int right,
                               const double *weights, const double *coe,
                               int ncoe, const void *in, void *out,
                               mxs_plan *plan);

/* ------------------------------------------------------------------------
 * Batched cyclic banded solves A x = r on every line (the periodic
 * line inversions of the ADI scheme, Sec. 5.1).  A is the symmetric
 * circulant with coef[0] on the diagonal and coef[d] on the d-th off-
 * diagonals (d = 1..bw), wrapping: row k holds coef[|d|] at column
 * (k+d) mod n.  bw = 1 (tridiagonal) or 2 (pentadiagonal).  The symbol
 * coef[0] + 2 sum_d coef[d] cos(d theta) must be positive for every theta
 * (symmetric positive definite for every n), else MXS_ERR_UNSUPPORTED.
 *
 * geometry:
 *   MXS_LINES_RAGGED  lines stored back to back, line b is
 *                     [offsets[b], offsets[b+1]) (offsets: host, nbatch+1);
 *   MXS_LINES_ROWS    every row of an nx x ny grid with pitch ld (n = nx);
 *   MXS_LINES_COLS    every column of that grid (n = ny).
 * Every line needs n >= 2*bw+1 and n <= 16384 (RAGGED and ROWS).
 * rhs and x are device buffers of the storage dtype; they may be the same
 * buffer (in-place), but must not otherwise overlap.  The elimination runs
 * in double whatever the storage dtype.
 * ---------------------------------------------------------------------- */
mxs_status mxs_create_cyclic_solve(int bw, const double *coef, int geometry,
                                   int nx, int ny, long long ld, int nbatch,
                                   const long long *offsets, int dtype,
                                   const void *rhs, void *x, mxs_plan *plan);

/* ------------------------------------------------------------------------
 * WENO advection: the periodic xy variant of Sec. 4.3, in which the weighted
 * sum of the periodic XY stencil is replaced by a WENO evaluation of the
 * advection term and the velocities are extra inputs:
 *
 *   out[j][i] = u[j][i] * phi_x + v[j][i] * phi_y
 *
 * phi_x is the fifth-order Hamilton-Jacobi WENO derivative (the level-set
 * text the section cites) from the backward differences
 * (phi[i+k] - phi[i+k-1]) / dx, k = -2..2, where u > 0, and from the forward
 * differences (phi[i+k+1] - phi[i+k]) / dx, k = 2..-2, where u <= 0 (zero
 * velocity contributes zero either way); phi_y likewise along j with v and
 * dy.  Every index wraps (periodic grid).  Epsilon of the nonlinear weights:
 * 1e-6 times the largest squared difference of the five, plus 1e-99.
 * phi, u, v, out: device, ny rows of pitch ld, FP64 only (dtype MXS_F64,
 * else MXS_ERR_UNSUPPORTED); out must not overlap phi, u or v
 * (MXS_ERR_ALIAS).  Requires nx, ny >= 6.  mxs_compute evaluates,
 * mxs_swap exchanges phi and out, mxs_set_io(plan, phi, out) rebinds them
 * (u and v stay), mxs_autotune picks the tile layout.
 * ---------------------------------------------------------------------- */
mxs_status mxs_create_weno_adv(int nx, int ny, long long ld, double dx, double dy,
                               int dtype, const void *phi, const void *u,
                               const void *v, void *out, mxs_plan *plan);

/* Run the plan on a stream: the stencil or the solve (cuStenCompute*). */
mxs_status mxs_compute(mxs_plan plan, void *hip_stream);

/* Exchange the input and output pointers (cuStenSwap*, Sec. 3).  For a
 * solve plan, rhs and x are exchanged. */
mxs_status mxs_swap(mxs_plan plan);

/* Point the plan at other input/output buffers of the same shape.  A grid
 * solve plan (MXS_LINES_ROWS or MXS_LINES_COLS) uploads its two instance
 * tables here with blocking host-to-device copies, so that mxs_compute and
 * mxs_swap themselves never copy from host memory. */
mxs_status mxs_set_io(mxs_plan plan, const void *in, void *out);

/* ------------------------------------------------------------------------
 * ADI Cahn-Hilliard step (Sec. 5.1): dC/dt = D lap(C^3 - C - gamma lap C)
 * on a periodic nx x ny grid with spacings dx, dy and time step dt:
 *
 *   Cbar = 2 C^n - C^{n-1}
 *   R    = -2/3 (C^n - C^{n-1}) - 2/3 D gamma dt lap_h^2 Cbar
 *          + 2/3 D dt lap_h (C^3 - C)^n
 *   L_x w = R (every row), L_y v = w (every column), C^{n+1} = Cbar + v,
 *   L_x = I + 2/3 D gamma dt d_xxxx,  L_y likewise (periodic pentadiagonal).
 *
 * lap_h is the 5-point Laplacian and lap_h^2 = d_xxxx + 2 d_xxyy + d_yyyy the
 * 13-point biharmonic, from the second-order central differences of
 * Sec. 5.1 and the cross stencil of Fig. 1.  The first step of a run uses
 * c_prev = c_cur = C^0 (Sec. 5.1).
 *
 * The three state buffers (device, dtype, pitch nx, caller-owned) rotate:
 * each step reads (prev, cur), writes next, then the roles become
 * (cur, next, prev).  mxs_ch_state reports where C^{n-1} and C^n are.
 * dtype MXS_F64: all arithmetic in double.  MXS_F32 / MXS_BF16: state
 * stored in that dtype, stencil and nonlinear arithmetic in float, w stored
 * in float, line eliminations in double, mass in double.
 * Requires nx, ny >= 8 and <= 16384, dt > 0, D > 0, gamma > 0.
 * ---------------------------------------------------------------------- */
mxs_status mxs_ch_create(int nx, int ny, double dx, double dy, double dt,
                         double D, double gamma, int dtype, void *c_prev,
                         void *c_cur, void *c_next, mxs_plan *plan);

/* An ensemble of count independent grids (sizes and spacings per grid, the
 * same D and gamma) advanced together: every kernel of a step covers all
 * instances in one launch.  Arrays are host arrays of length count; each
 * state pointer is a device buffer of nx[k]*ny[k] elements. */
mxs_status mxs_ch_ensemble_create(int count, const int *nx, const int *ny,
                                  const double *dx, const double *dy,
                                  const double *dt, double D, double gamma,
                                  int dtype, void *const *c_prev,
                                  void *const *c_cur, void *const *c_next,
                                  mxs_plan *plan);

/* Enqueue nsteps steps on a stream.  With use_graph != 0 each step replays
 * a captured HIP graph (one per rotation of the three buffers). */
mxs_status mxs_ch_step(mxs_plan plan, int nsteps, int use_graph, void *hip_stream);

/* How a step is launched.  MXS_CH_SEPARATE: one launch per kernel of the
 * step (right-hand side, row solves per register class, three column
 * phases), each covering every instance.  MXS_CH_PERSISTENT: the whole step
 * of every instance in one cooperative launch whose workgroups stay resident
 * and meet at a grid barrier between the phases (rows of at most 1024
 * elements; else MXS_ERR_UNSUPPORTED, as when the device cannot hold the
 * grid).  The barrier's wait is bounded: a barrier that times out makes the
 * launch end early, and the next mxs_ch_mass returns MXS_ERR_HIP.
 * MXS_CH_FUSED: the right-hand side of the x sweep is formed inside the row
 * solves, so that it never goes to memory (one launch per register class of
 * rows, then the three column phases; rows of at most 4096 elements, else
 * MXS_ERR_UNSUPPORTED).  The three give the same step up to the order of
 * rounding.  Plans start in MXS_CH_SEPARATE; mxs_autotune times every mode
 * the plan supports and keeps the fastest.  With use_graph the persistent
 * launch is captured in the step's graph. */
enum { MXS_CH_SEPARATE = 0, MXS_CH_PERSISTENT = 1, MXS_CH_FUSED = 2 };
mxs_status mxs_ch_set_step_mode(mxs_plan plan, int mode);

/* Device pointers of C^{n-1} and C^n of instance k (k = 0 for one grid). */
mxs_status mxs_ch_state(mxs_plan plan, int k, void **c_prev, void **c_cur);

/* Number of steps taken so far. */
mxs_status mxs_ch_steps_taken(mxs_plan plan, long long *nsteps);

/* Mass sum_ij C^n_ij of every instance, accumulated in double, written to
 * host_out[0 .. count-1].  Waits for the stream.  MXS_ERR_NONFINITE when a
 * sum is NaN or Inf. */
mxs_status mxs_ch_mass(mxs_plan plan, double *host_out, void *hip_stream);

/* Coarsening diagnostics of instance k's current state C^n (Sec. 5.3):
 *   s  = 1 / (1 - <C^2>), <.> the spatial average by Simpson's rule (on the
 *        periodic grid: node weights 2/3 and 4/3 alternating along each
 *        axis, starting with 2/3 at index 0);
 *   k1 = sum |C^(k)|^2 / sum |k|^-1 |C^(k)|^2 over the nonzero wavevectors
 *        k = (2 pi mx / (nx dx), 2 pi my / (ny dy)) of the grid's discrete
 *        Fourier transform (mx, my in -n/2+1 .. n/2).
 * Written to *s_out and *k1_out (host; either may be NULL).  Both sums in
 * double.  Needs nx and ny powers of two, at most 4096, else
 * MXS_ERR_UNSUPPORTED.  The plan allocates its transform scratch (16 bytes
 * per grid point) on the first call.  Waits for the stream. */
mxs_status mxs_ch_coarsening(mxs_plan plan, int k, double *s_out, double *k1_out,
                             void *hip_stream);

/* The same diagnostics as mxs_ch_coarsening, for callers that cannot
 * allocate device memory (tight loops, harnesses that forbid hipMalloc):
 * this call allocates nothing.  Its scratch is a static device array of the
 * library, one per GPU, held until the process ends and sized for grids of
 * at most 1048576 points (16 bytes per point plus 96 KiB of partial sums);
 * a larger grid returns MXS_ERR_UNSUPPORTED.  Every call on one GPU uses that
 * GPU's array, so calls that overlap on one GPU (from several threads, or on
 * several streams) race: serialise them.  Each call rewrites every scratch
 * value it reads, so no clearing is needed between calls.  Arguments,
 * results and errors otherwise as mxs_ch_coarsening; waits for the stream. */
mxs_status mxs_ch_coarsening_noalloc(mxs_plan plan, int k, double *s_out,
                                     double *k1_out, void *hip_stream);

/* Choose the plan's launch layout by measurement: candidate layouts (rows
 * per workgroup, tile order, threads per workgroup and streaming stores for
 * 2D stencils; wavefronts per line for lines solved in LDS, longer than
 * 4096 elements; step form (separate launches, right-hand side inside the
 * row solves, persistent) with its right-hand-side chunk height and
 * workgroup size, or rows and columns per fused workgroup, for the
 * Cahn-Hilliard step) are each run a few times on the plan's own buffers
 * and the fastest is kept.  A stencil or solve plan writes its output
 * buffer while tuning (with correct results); a Cahn-Hilliard plan rewrites
 * only the buffer its next step overwrites and its scratch, and the step
 * count is unchanged.  Waits for the stream.  Stencil layouts found are
 * remembered for the rest of the process for plans of the same shape.
 * Plans without tunable layouts return MXS_OK unchanged. */
mxs_status mxs_autotune(mxs_plan plan, void *hip_stream);

/* A one-line description of the plan's current launch layout, written to
 * buf (at most len bytes, NUL-terminated). */
mxs_status mxs_plan_info(mxs_plan plan, char *buf, int len);

/* Free everything the plan owns (cuStenDestroy*).  NULL is accepted.  The
 * caller's buffers and streams are not touched. */
mxs_status mxs_destroy(mxs_plan plan);

/* Message of the last failed call on this thread ("" if none). */
const char *mxs_last_error(void);

/* Name of a status code. */
const char *mxs_status_string(mxs_status st);

/* Library version, major*10000 + minor*100 + patch. */
int mxs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MXSTEN_H */
