// WENO advection variant of the periodic xy stencil (Sec. 4.3): launch
// arguments shared by the kernel (weno.hip) and its plan (api.cpp).
#pragma once

#include "mxs_internal.h"

namespace mxs {

struct WenoArgs {
    const void *phi, *u, *v;   // device, FP64, ny rows of pitch ld
    void *out;                 // device, FP64
    long long ld;
    int nx, ny;
    double rdx, rdy;           // 1 / dx, 1 / dy
    int rows;                  // output rows per workgroup (4 or 8)
    int nchunks, nstrips;
    int order;                 // tile order, as for the 2D stencils
    int nt_store;              // non-temporal output stores
    int vec_ok;                // 16-byte aligned rows of every array
};

size_t weno_lds_bytes(int rows, int threads);
bool weno_rows_ok(int rows);
hipError_t launch_weno_adv(const WenoArgs &a, int threads, hipStream_t s);

}  // namespace mxs
