// Coarsening diagnostics of a Cahn-Hilliard state (Sec. 5.3): shared by the
// kernels (diag.hip) and the plan (ch_plan.cpp).
#pragma once

#include "mxs_internal.h"

namespace mxs {

constexpr int kDiagThreads = 256;
constexpr int kDiagMaxSide = 4096;   // a transformed row or column fits the LDS of one workgroup
// Largest grid (points) of the allocation-free diagnostics entry point: its
// transform scratch is a static device array of 16 bytes per point.
constexpr long long kNoAllocDiagPoints = 1LL << 20;
constexpr int kMaxDevices = 64;

struct DiagArgs {
    const void *c;        // the state, storage dtype, nx * ny, pitch nx
    int nx, ny;           // powers of two, at most kDiagMaxSide
    double kx0, ky0;      // wavenumber steps 2 pi / (nx dx), 2 pi / (ny dy)
    double2 *spec;        // scratch, nx * ny complex values
    double *partial;      // scratch, ny + 2 nx doubles
    double *out;          // device, 3 doubles: sum a_i a_j C^2, sum |C^|^2, sum |C^|^2 / |k|
};

bool diag_shape_ok(int nx, int ny);
// Point d->spec, d->partial and d->out into the static scratch of the current
// device (nx * ny <= kNoAllocDiagPoints, checked by the caller); the device
// address is looked up once per device.  Allocates nothing.
hipError_t noalloc_diag_scratch(int nx, int ny, DiagArgs *d);
hipError_t launch_coarsening(int dtype, const DiagArgs &d, hipStream_t s);

}  // namespace mxs
