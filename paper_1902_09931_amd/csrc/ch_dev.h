// Device code of the right-hand side of the x sweep of the ADI
// Cahn-Hilliard step (described in ch.hip), shared by its kernel (ch.hip)
// and the persistent step (persist.hip).
#pragma once

#include "ch.h"

#include <type_traits>

namespace mxs {
namespace {

// Elements per thread and strip column group of the right-hand side: one
// 16-byte vector of the state per thread (2 doubles, 4 floats, 8 bfloat16s).
template <typename T> struct RhsVec { static constexpr int V = 16 / static_cast<int>(sizeof(T)); };

// V consecutive state values from a 16-byte aligned address, as floats or
// doubles.
template <typename T, int V>
__device__ __forceinline__ void rhs_load(gptr<const T> p, typename St<T>::acc *x) {
    if constexpr (std::is_same<T, bf16>::value) {
        const v4u_t v = *reinterpret_cast<gptr<const v4u_t>>(p);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            x[2 * k] = __uint_as_float(w[k] << 16);
            x[2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
        }
    } else {
        load_vec<T>(p, x);
    }
}

// V values of R (float or double) with streaming stores, 16 bytes at a time.
template <typename TW, int V>
__device__ __forceinline__ void rhs_store(gptr<TW> p, const TW *x) {
    constexpr int W = St<TW>::V;
#pragma unroll
    for (int k = 0; k < V; k += W) store_vec_nt<TW>(p + k, x + k);
}

// Input rows per stage: 4, or 2 for bfloat16, whose 8 values per thread and
// row would otherwise hold too many registers for the double-buffered loads.
template <typename T> constexpr int kRhsStage = sizeof(T) == 2 ? 2 : 4;

template <typename A> __device__ __forceinline__ A wb_of(const RhsInst &I, int k);
template <> __device__ __forceinline__ double wb_of<double>(const RhsInst &I, int k) { return I.wb[k]; }
template <> __device__ __forceinline__ float wb_of<float>(const RhsInst &I, int k) { return I.wbf[k]; }
template <typename A> __device__ __forceinline__ A wl_of(const RhsInst &I, int k);
template <> __device__ __forceinline__ double wl_of<double>(const RhsInst &I, int k) { return I.wl[k]; }
template <> __device__ __forceinline__ float wl_of<float>(const RhsInst &I, int k) { return I.wlf[k]; }
template <typename A> __device__ __forceinline__ A cd_of(const RhsInst &I);
template <> __device__ __forceinline__ double cd_of<double>(const RhsInst &I) { return I.cdiff; }
template <> __device__ __forceinline__ float cd_of<float>(const RhsInst &I) { return I.cdifff; }

// Taps of the 13-point biharmonic (5x5) and 5-point Laplacian (3x3) windows;
// the others are zero and are skipped at compile time.
constexpr bool bih_tap(int q, int p) {
    return q == 2 || p == 2 || ((q == 1 || q == 3) && (p == 1 || p == 3));
}
constexpr bool lap_tap(int q, int p) { return q == 1 || p == 1; }

// The right-hand side over tile `local` of instance I (a strip of
// blockDim.x * V columns and a chunk of I.rows rows), with the workgroup's
// LDS at smem (2 * 4 rows of blockDim.x * V + 2 PAD values).
template <typename T, typename TW>
__device__ __forceinline__ void rhs_tile(const RhsInst &I, const int local, unsigned char *smem) {
    using A = typename St<T>::acc;
    constexpr int V = RhsVec<T>::V;
    constexpr int PAD = V >= 2 ? V : 2;   // two halo columns, rounded up to a vector
    constexpr int G = kRhsStage<T>;       // input rows per stage
    constexpr int XB = V + 4;             // biharmonic window per thread
    constexpr int XL = V + 2;             // Laplacian window per thread

    const int nt = blockDim.x;
    const int t = threadIdx.x;
    const int W = nt * V;
    const int rowlen = PAD + W + PAD;
    A *lcb = reinterpret_cast<A *>(smem);
    A *lfc = lcb + G * rowlen;

    const int tile = xcd_tile(local, I.nstrips * I.nchunks);
    const int strip = tile / I.nchunks;
    const int chunk = tile - strip * I.nchunks;
    const int i0 = strip * W;
    const int j0 = chunk * I.rows;
    const int H = min(I.rows, I.ny - j0);
    const int niter = H + 4;
    const int ib = i0 + t * V;
    const int nx = I.nx, ny = I.ny;
    const bool full_vec = ((nx % V) == 0) && (ib + V <= nx);
    const gptr<const T> cur = as_global(static_cast<const T *>(I.cur));
    const gptr<const T> prev = as_global(static_cast<const T *>(I.prev));
    const gptr<TW> R = as_global(static_cast<TW *>(I.R));
    const A cdiff = cd_of<A>(I);
    A wb[25], wl[9];
#pragma unroll
    for (int k = 0; k < 25; ++k) wb[k] = bih_tap(k / 5, k % 5) ? wb_of<A>(I, k) : A(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) wl[k] = lap_tap(k / 3, k % 3) ? wl_of<A>(I, k) : A(0);
    // Odd chunks walk their rows upward (the windows are symmetric in y), so
    // the halo rows two neighbouring chunks share are read by both at about
    // the same time and the second read hits in L2.
    const bool up = (chunk & 1) != 0;
    const int rfirst = up ? j0 + H - 1 + 2 : j0 - 2;
    const int rstep = up ? -1 : 1;

    A acc[5][V];
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int v = 0; v < V; ++v) acc[k][v] = A(0);

    // halo columns per stage: G rows x 2*PAD, at most HPT per thread
    constexpr int HPT = (G * 2 * PAD + kRhsThreadsMin - 1) / kRhsThreadsMin;
    const int hcount = G * 2 * PAD;

    // issue the loads of C^n and C^{n-1} for the G input rows of stage s0
    auto load_stage = [&](int s0, A (&c)[G][V], A (&p)[G][V], A (&hc)[HPT], A (&hp)[HPT]) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int r = static_cast<int>(wrap_fast(rfirst + rstep * (s0 + u), ny));
            const gptr<const T> cr = cur + static_cast<long long>(r) * nx;
            const gptr<const T> pr = prev + static_cast<long long>(r) * nx;
            if (full_vec) {
                rhs_load<T, V>(cr + ib, c[u]);
                rhs_load<T, V>(pr + ib, p[u]);
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int col = static_cast<int>(wrap_ll(ib + v, nx));
                    c[u][v] = to_acc<T>(gld<T>(cr, col));
                    p[u][v] = to_acc<T>(gld<T>(pr, col));
                }
            }
        }
#pragma unroll
        for (int q = 0; q < HPT; ++q) {
            const int h = t + q * nt;
            A vc = A(0), vp = A(0);
            if (h < hcount) {
                const int u = h / (2 * PAD);
                const int hh = h - u * 2 * PAD;
                const int r = static_cast<int>(wrap_fast(rfirst + rstep * (s0 + u), ny));
                const long long col = hh < PAD ? static_cast<long long>(i0) - PAD + hh
                                               : static_cast<long long>(i0) + W + (hh - PAD);
                const long long o = static_cast<long long>(r) * nx + wrap_fast(col, nx);
                vc = to_acc<T>(gld<T>(cur, o));
                vp = to_acc<T>(gld<T>(prev, o));
            }
            hc[q] = vc;
            hp[q] = vp;
        }
    };

    A c0[G][V], p0[G][V], c1[G][V], p1[G][V], hc0[HPT], hp0[HPT], hc1[HPT], hp1[HPT];
    load_stage(0, c0, p0, hc0, hp0);

    for (int s0 = 0; s0 < niter; s0 += G) {
        __syncthreads();   // the previous stage's LDS reads are done
#pragma unroll
        for (int u = 0; u < G; ++u)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const A c = c0[u][v], p = p0[u][v];
                lcb[u * rowlen + PAD + t * V + v] = A(2) * c - p;
                lfc[u * rowlen + PAD + t * V + v] = c * c * c - c;
            }
#pragma unroll
        for (int q = 0; q < HPT; ++q) {
            const int h = t + q * nt;
            if (h < hcount) {
                const int u = h / (2 * PAD);
                const int hh = h - u * 2 * PAD;
                const int pos = u * rowlen + (hh < PAD ? hh : W + hh);
                const A c = hc0[q], p = hp0[q];
                lcb[pos] = A(2) * c - p;
                lfc[pos] = c * c * c - c;
            }
        }
        // the next stage's loads overlap this stage's arithmetic
        if (s0 + G < niter) load_stage(s0 + G, c1, p1, hc1, hp1);
        __syncthreads();

#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int s = s0 + u;
            if (s < niter) {
                A x[XB], y[XL];
                const A *bp = lcb + u * rowlen + PAD + t * V - 2;
                const A *fp = lfc + u * rowlen + PAD + t * V - 1;
#pragma unroll
                for (int q = 0; q < XB; ++q) x[q] = bp[q];
#pragma unroll
                for (int q = 0; q < XL; ++q) y[q] = fp[q];
                // acc[k] is output row s - 4 + k, met by window row 4 - k
#pragma unroll
                for (int k = 0; k < 5; ++k) {
#pragma unroll
                    for (int p = 0; p < 5; ++p) {
                        if (bih_tap(4 - k, p)) {
                            const A w = wb[(4 - k) * 5 + p];
#pragma unroll
                            for (int v = 0; v < V; ++v) acc[k][v] = fma(w, x[v + p], acc[k][v]);
                        }
                    }
                }
#pragma unroll
                for (int k = 1; k <= 3; ++k) {
#pragma unroll
                    for (int p = 0; p < 3; ++p) {
                        if (lap_tap(3 - k, p)) {
                            const A w = wl[(3 - k) * 3 + p];
#pragma unroll
                            for (int v = 0; v < V; ++v) acc[k][v] = fma(w, y[v + p], acc[k][v]);
                        }
                    }
                }
#pragma unroll
                for (int v = 0; v < V; ++v) acc[2][v] = fma(cdiff, c0[u][v] - p0[u][v], acc[2][v]);

                const int jj = s - 4;
                if (jj >= 0 && jj < H) {
                    const gptr<TW> rowp = R + static_cast<long long>(up ? j0 + H - 1 - jj : j0 + jj) * nx;
                    if (full_vec) {
                        rhs_store<TW, V>(rowp + ib, acc[0]);
                    } else {
#pragma unroll
                        for (int v = 0; v < V; ++v)
                            if (ib + v < nx) gst<TW>(rowp, ib + v, from_acc<TW>(acc[0][v]));
                    }
                }
#pragma unroll
                for (int k = 0; k < 4; ++k)
#pragma unroll
                    for (int v = 0; v < V; ++v) acc[k][v] = acc[k + 1][v];
#pragma unroll
                for (int v = 0; v < V; ++v) acc[4][v] = A(0);
            }
        }
#pragma unroll
        for (int u = 0; u < G; ++u)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                c0[u][v] = c1[u][v];
                p0[u][v] = p1[u][v];
            }
#pragma unroll
        for (int q = 0; q < HPT; ++q) {
            hc0[q] = hc1[q];
            hp0[q] = hp1[q];
        }
    }
}

// Bytes of LDS the right-hand side of a workgroup of `threads` threads uses.
template <typename T> constexpr size_t rhs_lds_bytes(int threads) {
    return 2 * kRhsStage<T> * static_cast<size_t>((RhsVec<T>::V >= 2 ? RhsVec<T>::V : 2) * 2 + threads * RhsVec<T>::V) *
           sizeof(typename St<T>::acc);
}

}  // namespace
}  // namespace mxs
