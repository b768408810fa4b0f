// Batched 1D stencils over uneven signals stored back to back (the batched
// 1D form of the abstract).
//
// The concatenated array is cut into equal tiles of W = threads * V * U
// elements (U = kS1dVecs vectors per thread),
// regardless of where signals begin and end, so every workgroup moves the
// same number of bytes whatever the length mix.  One workgroup per tile (the
// launch is a single sweep over the array, like a copy): it stages the
// values (plus an x halo of PAD elements each side) and the slice of signal
// offsets that meets the tile in LDS, requesting all three at once.  Each
// vector of outputs finds its signal by binary search in that slice.
// Outputs whose window stays inside their signal read LDS directly (a
// vector whose elements all do takes a straight-line path); the few near a
// signal end wrap within the signal (periodic) and read the wrapped value
// from LDS when it is staged, else from global memory.
#include "mxs_internal.h"

namespace mxs {

namespace {

template <typename A> __device__ __forceinline__ const A *coe_of(const Stencil1DArgs &a);
template <> __device__ __forceinline__ const double *coe_of<double>(const Stencil1DArgs &a) { return a.coe_d; }
template <> __device__ __forceinline__ const float *coe_of<float>(const Stencil1DArgs &a) { return a.coe_f; }

// Output vector stores: non-temporal for 8- and 2-byte elements, plain for
// FP32, whichever measured faster over the 65,536-signal batch (FP64 419
// against 433 us; FP32 250 against 254 us).
template <typename T> __device__ __forceinline__ void put_vec(T *p, const typename St<T>::acc *x) {
    if constexpr (sizeof(T) == 4) store_vec<T>(p, x);
    else store_vec_nt<T>(p, x);
}

template <int NWX, int V> constexpr int halo_pad() {
    return NWX > 1 ? ((NWX - 1 + V - 1) / V) * V : 0;
}

template <typename T, int NWX>
__global__ void __launch_bounds__(256) stencil1d_kernel(const Stencil1DArgs a) {
    using A = typename St<T>::acc;
    constexpr int V = St<T>::V;
    constexpr int U = kS1dVecs;
    constexpr int PAD = halo_pad<NWX, V>();

    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int nt = blockDim.x;
    const int t = threadIdx.x;
    const int W = nt * V * U;
    A *lds = reinterpret_cast<A *>(smem_raw);
    long long *soff = reinterpret_cast<long long *>(smem_raw + ((static_cast<size_t>(2 * PAD + W) * sizeof(A) + 15) & ~static_cast<size_t>(15)));

    const T *__restrict__ in = static_cast<const T *>(a.in);
    T *__restrict__ out = static_cast<T *>(a.out);
    const A *__restrict__ w = static_cast<const A *>(a.wts);
    const A *coe = coe_of<A>(a);
    const bool periodic = a.periodic != 0;
    const int taps = a.L + a.R + 1;

    // one tile per workgroup: the values (U vectors per thread, each vector
    // of the workgroup adjacent to the next thread's), their halo and the
    // offsets of the signals meeting the tile are all requested before any
    // is used
    const int tile = blockIdx.x;
    const long long e0 = static_cast<long long>(tile) * W;
    const int b0 = a.tile_first[tile];
    const int cnt = a.tile_first[tile + 1] - b0 + 2;   // offsets b0 .. b_last+1
    A xv[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const long long eb = e0 + static_cast<long long>(u * nt + t) * V;
        if (a.vec_ok && eb + V <= a.total) {
            load_vec<T>(in + eb, xv[u]);
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) xv[u][v] = eb + v < a.total ? to_acc<T>(in[eb + v]) : A(0);
        }
    }
    A hv = A(0);
    if (t < 2 * PAD) {
        const long long c = t < PAD ? e0 - PAD + t : e0 + W + (t - PAD);
        if (c >= 0 && c < a.total) hv = to_acc<T>(in[c]);
    }
    for (int k = t; k < cnt; k += nt) soff[k] = a.offsets[b0 + k];
    if (a.ncoe) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int v = 0; v < V; ++v) xv[u][v] = point_fun<A>(xv[u][v], coe, a.ncoe);
        hv = point_fun<A>(hv, coe, a.ncoe);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int v = 0; v < V; ++v) lds[PAD + (u * nt + t) * V + v] = xv[u][v];
    if (t < 2 * PAD) lds[t < PAD ? t : W + t] = hv;
    __syncthreads();

#pragma unroll
    for (int u = 0; u < U; ++u) {
        const long long eb = e0 + static_cast<long long>(u * nt + t) * V;
        A res[V];
        bool wr[V];
        // the signal holding the vector's first element (binary search in
        // the tile's offsets); later elements of the vector step to the next
        // signal when they cross its start
        int lo = 0;
        {
            int hi = cnt - 2;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (soff[mid] <= eb) lo = mid; else hi = mid - 1;
            }
        }
        long long sb = soff[lo], se = soff[lo + 1];
        // the common case: the whole vector lies in one signal with every
        // window inside it (no wrap, every output written): straight-line
        // FMAs over the staged values
        if (a.vec_ok && eb >= sb + a.L && eb + V - 1 + a.R <= se - 1) {
            const A *lp = lds + PAD + (eb - e0) - a.L;
            A x[V + NWX - 1];
#pragma unroll
            for (int k = 0; k < V + NWX - 1; ++k) x[k] = lp[k];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                A acc = A(0);
#pragma unroll
                for (int p = 0; p < NWX; ++p) acc = fma(w[p], x[v + p], acc);
                res[v] = acc;
            }
            put_vec<T>(out + eb, res);
            continue;
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const long long e = eb + v;
            res[v] = A(0);
            wr[v] = false;
            if (e >= a.total) continue;
            while (e >= se) {
                ++lo;
                sb = se;
                se = soff[lo + 1];
            }
            const long long n = se - sb;
            const long long i = e - sb;
            if (!periodic && (i < a.L || i > n - 1 - a.R)) continue;
            wr[v] = true;
            A acc = A(0);
            if (i >= a.L && i - a.L + (NWX - 1) <= n - 1) {
                const A *lp = lds + PAD + (e - e0) - a.L;
#pragma unroll
                for (int p = 0; p < NWX; ++p) acc = fma(w[p], lp[p], acc);
            } else {
                for (int p = 0; p < taps; ++p) {
                    long long ii = i + p - a.L;
                    if (ii < 0) ii += n;
                    else if (ii >= n) ii -= n;
                    const long long idx = sb + ii;
                    A val;
                    if (idx >= e0 - PAD && idx < e0 + W + PAD) {
                        val = lds[PAD + (idx - e0)];
                    } else {
                        val = to_acc<T>(in[idx]);
                        if (a.ncoe) val = point_fun<A>(val, coe, a.ncoe);
                    }
                    acc = fma(w[p], val, acc);
                }
            }
            res[v] = acc;
        }
        bool all = a.vec_ok && eb + V <= a.total;
#pragma unroll
        for (int v = 0; v < V; ++v) all = all && wr[v];
        if (all) {
            put_vec<T>(out + eb, res);
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v)
                if (wr[v]) out[eb + v] = from_acc<T>(res[v]);
        }
    }
}

template <typename T, int NWX>
hipError_t launch_one(const Stencil1DArgs &a, int threads, int grid, hipStream_t s) {
    const size_t lds = stencil1d_lds_bytes(std::is_same<T, double>::value ? F64
                                           : std::is_same<T, float>::value ? F32 : BF16,
                                           NWX, threads, a.max_sig_per_tile);
    hipLaunchKernelGGL((stencil1d_kernel<T, NWX>), dim3(grid), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t dispatch(int nwx, const Stencil1DArgs &a, int threads, int grid, hipStream_t s) {
    switch (nwx) {
    case 1: return launch_one<T, 1>(a, threads, grid, s);
    case 3: return launch_one<T, 3>(a, threads, grid, s);
    case 5: return launch_one<T, 5>(a, threads, grid, s);
    case 9: return launch_one<T, 9>(a, threads, grid, s);
    case 17: return launch_one<T, 17>(a, threads, grid, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

size_t stencil1d_lds_bytes(int dtype, int nwx, int threads, int max_sig) {
    const int V = dtype == F64 ? St<double>::V : dtype == F32 ? St<float>::V : St<bf16>::V;
    const int acc = dtype == F64 ? 8 : 4;
    const int pad = nwx > 1 ? ((nwx - 1 + V - 1) / V) * V : 0;
    const size_t vals = (static_cast<size_t>(2 * pad + threads * V * kS1dVecs) * acc + 15) & ~static_cast<size_t>(15);
    return vals + static_cast<size_t>(max_sig) * sizeof(long long);
}

hipError_t launch_stencil1d(int dtype, int nwx, const Stencil1DArgs &a, int threads, int grid,
                            hipStream_t s) {
    switch (dtype) {
    case F64: return dispatch<double>(nwx, a, threads, grid, s);
    case F32: return dispatch<float>(nwx, a, threads, grid, s);
    case BF16: return dispatch<bf16>(nwx, a, threads, grid, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mxs
