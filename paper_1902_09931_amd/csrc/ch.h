// ADI Cahn-Hilliard step: structures shared by the kernels and the plan.
#pragma once

#include "mxs_internal.h"

namespace mxs {

// Right-hand side of the x sweep (Sec. 5.1), per instance:
//   R = cdiff (C^n - C^{n-1}) + sum wb * Cbar + sum wl * (C^n^3 - C^n),
//   Cbar = 2 C^n - C^{n-1}; wb is the 5x5 biharmonic window scaled by
//   -2/3 D gamma dt, wl the 3x3 Laplacian window scaled by 2/3 D dt, and
//   cdiff = -2/3.
struct RhsInst {
    const void *cur;     // C^n, state dtype
    const void *prev;    // C^{n-1}, state dtype
    void *R;             // right-hand side, w dtype
    int nx, ny;          // pitch == nx
    int nstrips, nchunks, rows;
    int blk0;            // first block of this instance
    double wb[25];
    double wl[9];
    double cdiff;
    float wbf[25];
    float wlf[9];
    float cdifff;
};

// Threads per workgroup of the right-hand side: at most kRhsThreads, at
// least kRhsThreadsMin (a multiple of 64); a strip is threads * V columns,
// V = 16 bytes of state per thread (2 doubles, 4 floats, 8 bfloat16s).
constexpr int kRhsThreads = 256;
constexpr int kRhsThreadsMin = 64;

// One launch over every instance of the table with `threads` threads per
// workgroup; map[b] is the instance of workgroup b (nullptr: every
// workgroup belongs to instance 0).
hipError_t launch_ch_rhs(int state_dtype, const RhsInst *inst, const int *map, int blocks,
                         int threads, hipStream_t s);

// The right-hand side formed inside the row solves (chrows.hip): one
// workgroup of wr wavefronts per group of wr consecutive rows of one
// instance, work[b] naming the instance and first row of group b, cpt
// columns per thread and sub-block; shapes (wr, cpt) = (4, 1), (8, 1) or
// (4, 2).  One launch per register class nb of the rows (wave_nb of nx); R is
// never stored and each wavefront writes w of its row through rows[inst].out.
// ch_rhs_rows_lds_bytes returns 0 for a shape that does not exist.
struct RowsInst;
struct RowGroup {
    int inst, j0;
};
size_t ch_rhs_rows_lds_bytes(int state_dtype, int wr, int cpt, int nb);
hipError_t launch_ch_rhs_rows(int state_dtype, int wr, int cpt, int nb, const RhsInst *rhs, const RowsInst *rows,
                              const RowGroup *work, int count, hipStream_t s);

// Mass: per-instance double sums of a state buffer.
struct MassInst {
    const void *c;
    long long n;
    int blk0, nblk;
};
constexpr int kMassThreads = 256;
hipError_t launch_ch_mass(int state_dtype, const MassInst *inst, const int *map, int ninst,
                          int blocks, double *partial, double *out, hipStream_t s);

}  // namespace mxs
