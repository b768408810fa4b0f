// Coarsening diagnostics of a Cahn-Hilliard state (Sec. 5.3):
//
//   s(t)  = 1 / (1 - <C^2>), <.> the spatial average by Simpson's rule;
//   k1(t) = sum_k |C^(k)|^2 / sum_k |k|^-1 |C^(k)|^2, over the nonzero
//           wavevectors of the grid's discrete Fourier transform.
//
// Simpson's rule on a periodic grid of N (even) nodes x_i = i h: the
// composite rule over [0, N h] with the end node identified with node 0
// gives node i the weight (2 h / 3) for even i and (4 h / 3) for odd i, so
// the average is (1 / (nx ny)) sum_ij a_i a_j C_ij^2 with a = 2/3, 4/3.
// Both sums are accumulated in double by fixed-order two-level reductions
// (deterministic).
//
// The transform: every row is transformed by one workgroup in LDS
// (radix-2, decimation in time from bit-reversed order, complex double),
// written to a scratch grid, then every column likewise; the column
// workgroups weight |C^|^2 by 1 and by 1/|k| and reduce both sums.  Grid
// sides must be powers of two, at most kDiagMaxSide.
#include "diag.h"

#include <mutex>

namespace mxs {

// Scratch of the allocation-free diagnostics entry point: the transform grid
// (kNoAllocDiagPoints complex values), then the partial sums (ny + 2 nx
// doubles), then the 3 results.  Every GPU the library runs on holds its own
// copy for the life of the process.  Host code never passes this name to a
// kernel: its device address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) double scratch[2 * kNoAllocDiagPoints + 3 * kDiagMaxSide + 8];

namespace {

template <typename T> __device__ __forceinline__ double load_f64(gptr<const T> p, long long i);
template <> __device__ __forceinline__ double load_f64<double>(gptr<const double> p, long long i) { return p[i]; }
template <> __device__ __forceinline__ double load_f64<float>(gptr<const float> p, long long i) { return p[i]; }
template <> __device__ __forceinline__ double load_f64<bf16>(gptr<const bf16> p, long long i) {
    return bf16_to_float(reinterpret_cast<gptr<const uint16_t>>(p)[i]);
}

// Sum of v over the workgroup, in a fixed order (tree over kDiagThreads).
__device__ double wg_sum(double v, double *red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int h = kDiagThreads / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Row j of the Simpson-weighted sum of C^2: a_j sum_i a_i C_ij^2.
template <typename T>
__global__ void __launch_bounds__(kDiagThreads) simpson_rows_kernel(const T *c, int nx, double *partial) {
    __shared__ double red[kDiagThreads];
    const int j = blockIdx.x;
    const gptr<const T> row = as_global(c) + static_cast<long long>(j) * nx;
    double s = 0.0;
    for (int i = threadIdx.x; i < nx; i += kDiagThreads) {
        const double v = load_f64<T>(row, i);
        s += ((i & 1) ? 4.0 / 3.0 : 2.0 / 3.0) * (v * v);
    }
    const double tot = wg_sum(s, red);
    if (threadIdx.x == 0) partial[j] = ((j & 1) ? 4.0 / 3.0 : 2.0 / 3.0) * tot;
}

// In-place radix-2 transform of n = 2^logn complex values in LDS, already in
// bit-reversed order: X_k = sum_m x_m exp(-2 pi i k m / n).
__device__ void fft_lds(double2 *a, int n, int logn) {
    for (int s = 1; s <= logn; ++s) {
        const int half = 1 << (s - 1);
        for (int t = threadIdx.x; t < n / 2; t += kDiagThreads) {
            const int pos = t & (half - 1);
            const int i0 = ((t >> (s - 1)) << s) + pos;
            const int i1 = i0 + half;
            double sn, cs;
            sincospi(-static_cast<double>(pos) / half, &sn, &cs);
            const double2 x = a[i0], y = a[i1];
            const double br = y.x * cs - y.y * sn, bi = y.x * sn + y.y * cs;
            a[i0] = make_double2(x.x + br, x.y + bi);
            a[i1] = make_double2(x.x - br, x.y - bi);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int bitrev(int i, int logn) {
    return static_cast<int>(__brev(static_cast<unsigned>(i)) >> (32 - logn));
}

template <typename T>
__global__ void __launch_bounds__(kDiagThreads) fft_rows_kernel(const T *c, int nx, int lognx, double2 *out) {
    extern __shared__ double2 lds[];
    const int j = blockIdx.x;
    const gptr<const T> row = as_global(c) + static_cast<long long>(j) * nx;
    for (int i = threadIdx.x; i < nx; i += kDiagThreads)
        lds[bitrev(i, lognx)] = make_double2(load_f64<T>(row, i), 0.0);
    __syncthreads();
    fft_lds(lds, nx, lognx);
    const gptr<double> o = as_global(reinterpret_cast<double *>(out)) + 2 * static_cast<long long>(j) * nx;
    for (int i = threadIdx.x; i < nx; i += kDiagThreads) {
        o[2 * i] = lds[i].x;
        o[2 * i + 1] = lds[i].y;
    }
}

// Column i of the transformed rows: transform, then this column's share of
// sum |X|^2 and sum |X|^2 / |k| (k = 0 left out).
__global__ void __launch_bounds__(kDiagThreads) fft_cols_kernel(const double2 *rows, int nx, int ny, int logny,
                                                                double kx0, double ky0, double *partial) {
    extern __shared__ double2 lds[];
    __shared__ double red[kDiagThreads];
    const int i = blockIdx.x;
    const gptr<const double> col = as_global(reinterpret_cast<const double *>(rows)) + 2 * i;
    for (int j = threadIdx.x; j < ny; j += kDiagThreads) {
        const long long o = 2 * static_cast<long long>(j) * nx;
        lds[bitrev(j, logny)] = make_double2(col[o], col[o + 1]);
    }
    __syncthreads();
    fft_lds(lds, ny, logny);
    const int mx = i <= nx / 2 ? i : i - nx;
    const double kx = kx0 * mx;
    double p = 0.0, q = 0.0;
    for (int j = threadIdx.x; j < ny; j += kDiagThreads) {
        const int my = j <= ny / 2 ? j : j - ny;
        if (mx == 0 && my == 0) continue;
        const double ky = ky0 * my;
        const double2 x = lds[j];
        const double e = x.x * x.x + x.y * x.y;
        p += e;
        q += e / sqrt(kx * kx + ky * ky);
    }
    const double ps = wg_sum(p, red);
    const double qs = wg_sum(q, red);
    if (threadIdx.x == 0) {
        partial[2 * i] = ps;
        partial[2 * i + 1] = qs;
    }
}

// out[k] = sum_{m < n} partial[stride m + k], k < stride, in a fixed order.
__global__ void __launch_bounds__(kDiagThreads) diag_final_kernel(const double *partial, int n, int stride,
                                                                  double *out) {
    __shared__ double red[kDiagThreads];
    const int k = blockIdx.x;
    double s = 0.0;
    for (int m = threadIdx.x; m < n; m += kDiagThreads) s += partial[static_cast<long long>(m) * stride + k];
    const double tot = wg_sum(s, red);
    if (threadIdx.x == 0) out[k] = tot;
}

int log2_exact(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return (1 << l) == n ? l : -1;
}

template <typename T>
hipError_t diag_one(const DiagArgs &d, hipStream_t s) {
    const int lx = log2_exact(d.nx), ly = log2_exact(d.ny);
    hipLaunchKernelGGL((simpson_rows_kernel<T>), dim3(d.ny), dim3(kDiagThreads), 0, s,
                       static_cast<const T *>(d.c), d.nx, d.partial);
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(kDiagThreads), 0, s, d.partial, d.ny, 1, d.out);
    hipLaunchKernelGGL((fft_rows_kernel<T>), dim3(d.ny), dim3(kDiagThreads), sizeof(double2) * d.nx, s,
                       static_cast<const T *>(d.c), d.nx, lx, d.spec);
    hipLaunchKernelGGL(fft_cols_kernel, dim3(d.nx), dim3(kDiagThreads), sizeof(double2) * d.ny, s, d.spec,
                       d.nx, d.ny, ly, d.kx0, d.ky0, d.partial + d.ny);
    hipLaunchKernelGGL(diag_final_kernel, dim3(2), dim3(kDiagThreads), 0, s, d.partial + d.ny, d.nx, 2,
                       d.out + 1);
    return hipGetLastError();
}

}  // namespace

bool diag_shape_ok(int nx, int ny) {
    return nx >= 2 && ny >= 2 && nx <= kDiagMaxSide && ny <= kDiagMaxSide && log2_exact(nx) >= 0 &&
           log2_exact(ny) >= 0;
}

hipError_t noalloc_diag_scratch(int nx, int ny, DiagArgs *d) {
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    double *base;
    {
        std::lock_guard<std::mutex> lock(mu);
        if (!addr[dev]) {
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            addr[dev] = static_cast<double *>(p);
        }
        base = addr[dev];
    }
    d->spec = reinterpret_cast<double2 *>(base);
    d->partial = base + 2 * static_cast<size_t>(nx) * ny;
    d->out = d->partial + ny + 2 * static_cast<size_t>(nx);
    return hipSuccess;
}

hipError_t launch_coarsening(int dtype, const DiagArgs &d, hipStream_t s) {
    if (!diag_shape_ok(d.nx, d.ny)) return hipErrorInvalidValue;
    switch (dtype) {
    case F64: return diag_one<double>(d, s);
    case F32: return diag_one<float>(d, s);
    case BF16: return diag_one<bf16>(d, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mxs
