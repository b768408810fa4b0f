// Kernels of the ADI Cahn-Hilliard step (Sec. 5.1) other than the line
// solves: the fused right-hand side of the x sweep, and the mass reduction.
//
// The right-hand side streams the rows of C^n and C^{n-1} once: every input
// row is turned into Cbar = 2 C^n - C^{n-1} and f = C^n^3 - C^n (staged in LDS
// with a two-column periodic halo), then multiplied into the five pending
// output rows it meets (5x5 biharmonic window on Cbar, 3x3 Laplacian window
// on f), and the centre row adds -2/3 (C^n - C^{n-1}).  One read of each
// state element and one write of R per point, as for the stencils.
#include "ch_dev.h"

namespace mxs {

namespace {

template <typename T, typename TW>
__global__ void __launch_bounds__(kRhsThreads) ch_rhs_kernel(const RhsInst *__restrict__ inst,
                                                             const int *__restrict__ map) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int g = map ? map[blockIdx.x] : 0;
    const RhsInst &I = inst[g];
    rhs_tile<T, TW>(I, blockIdx.x - I.blk0, smem_raw);
}

// ---- mass ------------------------------------------------------------------------

template <typename T> __device__ __forceinline__ double elem_f64(gptr<const T> p, long long i);
template <> __device__ __forceinline__ double elem_f64<double>(gptr<const double> p, long long i) { return p[i]; }
template <> __device__ __forceinline__ double elem_f64<float>(gptr<const float> p, long long i) { return p[i]; }
template <> __device__ __forceinline__ double elem_f64<bf16>(gptr<const bf16> p, long long i) {
    return bf16_to_float(p[i].bits);
}

__device__ double block_sum(double v, double *red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int h = kMassThreads / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

template <typename T>
__global__ void __launch_bounds__(kMassThreads) mass_partial_kernel(const MassInst *__restrict__ inst,
                                                                   const int *__restrict__ map,
                                                                   double *partial) {
    __shared__ double red[kMassThreads];
    const int g = map ? map[blockIdx.x] : 0;
    const MassInst &I = inst[g];
    const long long local = blockIdx.x - I.blk0;
    const long long chunk = (I.n + I.nblk - 1) / I.nblk;
    const long long a = local * chunk;
    const long long b = min(I.n, a + chunk);
    const gptr<const T> c = as_global(static_cast<const T *>(I.c));
    double s = 0.0;
    for (long long i = a + threadIdx.x; i < b; i += kMassThreads) s += elem_f64<T>(c, i);
    const double tot = block_sum(s, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kMassThreads) mass_final_kernel(const MassInst *__restrict__ inst,
                                                                 const double *partial, double *out) {
    __shared__ double red[kMassThreads];
    const MassInst &I = inst[blockIdx.x];
    double s = 0.0;
    for (int i = threadIdx.x; i < I.nblk; i += kMassThreads) s += partial[I.blk0 + i];
    const double tot = block_sum(s, red);
    if (threadIdx.x == 0) out[blockIdx.x] = tot;
}

template <typename T, typename TW>
hipError_t rhs_one(const RhsInst *inst, const int *map, int blocks, int threads, hipStream_t s) {
    if (threads < kRhsThreadsMin || threads > kRhsThreads || threads % 64) return hipErrorInvalidValue;
    const size_t lds = rhs_lds_bytes<T>(threads);
    hipLaunchKernelGGL((ch_rhs_kernel<T, TW>), dim3(blocks), dim3(threads), lds, s, inst, map);
    return hipGetLastError();
}

template <typename T>
hipError_t mass_one(const MassInst *inst, const int *map, int ninst, int blocks, double *partial,
                    double *out, hipStream_t s) {
    hipLaunchKernelGGL((mass_partial_kernel<T>), dim3(blocks), dim3(kMassThreads), 0, s, inst, map,
                       partial);
    hipLaunchKernelGGL(mass_final_kernel, dim3(ninst), dim3(kMassThreads), 0, s, inst, partial, out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ch_rhs(int state_dtype, const RhsInst *inst, const int *map, int blocks,
                         int threads, hipStream_t s) {
    switch (state_dtype) {
    case F64: return rhs_one<double, double>(inst, map, blocks, threads, s);
    case F32: return rhs_one<float, float>(inst, map, blocks, threads, s);
    case BF16: return rhs_one<bf16, float>(inst, map, blocks, threads, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ch_mass(int state_dtype, const MassInst *inst, const int *map, int ninst,
                          int blocks, double *partial, double *out, hipStream_t s) {
    switch (state_dtype) {
    case F64: return mass_one<double>(inst, map, ninst, blocks, partial, out, s);
    case F32: return mass_one<float>(inst, map, ninst, blocks, partial, out, s);
    case BF16: return mass_one<bf16>(inst, map, ninst, blocks, partial, out, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mxs
