// 2D stencils in the x, y and xy directions, periodic or non-periodic, with
// fixed weights or a point function (Sec. 3, Sec. 4.1, Sec. 4.2).
//
// One kernel template covers every direction.  A workgroup owns a strip of
// W = threads * V columns and a chunk of `rows` output rows.  It streams the
// input rows of its chunk top to bottom; each thread keeps, per pending
// output row, an accumulator vector of V outputs in registers (NWY rows,
// shifted by one row as each output row completes).  When an input row arrives, its window along x (V + NWX - 1 values,
// read from an LDS copy of the row with its x halo, or straight from
// registers when NWX == 1) is multiplied into every pending output row it
// touches; the output row whose window is complete is written out.  Each
// input element is therefore read from HBM once per chunk (plus the NWY - 1
// halo rows shared with the chunk above), and each output element written
// once, with 8- or 16-byte vector accesses.
//
// The window is padded to the compiled widths NWX x NWY in {1,3,5,9,17};
// padded taps carry weight zero.  Weights live in device memory in the
// accumulation type and are read with uniform (scalar) loads.
#include "mxs_internal.h"

#include <type_traits>

namespace mxs {

namespace {

// Strip and chunk of this workgroup.  order 0: the workgroups of one XCD
// take one contiguous range of tiles numbered strip by strip (a band of
// strips, chunks top to bottom); order 2: the same ranges numbered chunk by
// chunk (a band of chunks, strips left to right), so that horizontal
// neighbours, which share x halo columns, and vertical ones, which share
// rows, run on the same XCD at about the same time; order 1: workgroups in
// launch order, chunk by chunk.
__device__ __forceinline__ void tile_of(const Stencil2DArgs &a, int &strip, int &chunk) {
    if (a.order == 1) {
        chunk = blockIdx.x / a.nstrips;
        strip = blockIdx.x - chunk * a.nstrips;
        return;
    }
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (a.order == 0) {
        strip = tile / a.nchunks;
        chunk = tile - strip * a.nchunks;
    } else {
        chunk = tile / a.nstrips;
        strip = tile - chunk * a.nstrips;
    }
}

template <int NWX, int V> constexpr int halo_pad() {
    return NWX > 1 ? ((NWX - 1 + V - 1) / V) * V : 0;
}

// Input rows loaded per round (into LDS when NWX > 1).
template <int NWY> constexpr int stage_rows() {
    return 4;
}

template <typename A> __device__ __forceinline__ const A *coe_of(const Stencil2DArgs &a);
template <> __device__ __forceinline__ const double *coe_of<double>(const Stencil2DArgs &a) { return a.coe_d; }
template <> __device__ __forceinline__ const float *coe_of<float>(const Stencil2DArgs &a) { return a.coe_f; }

// Load element c of an input row, wrapping (periodic) or as zero when outside
// [0, nx) (non-periodic: such values never reach a written output).
template <typename T>
__device__ __forceinline__ typename St<T>::acc load_elem(const T *rowp, long long c, int nx,
                                                         bool periodic) {
    using A = typename St<T>::acc;
    if (c < 0 || c >= nx) {
        if (!periodic) return A(0);
        c = wrap_ll(c, nx);
    }
    return to_acc<T>(rowp[c]);
}

template <typename T, int NWX, int NWY>
__global__ void __launch_bounds__(256) stencil2d_kernel(const Stencil2DArgs a) {
    using A = typename St<T>::acc;
    constexpr int V = St<T>::V;
    constexpr int PAD = halo_pad<NWX, V>();
    constexpr int G = stage_rows<NWY>();
    constexpr int XW = V + NWX - 1;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    A *lds = reinterpret_cast<A *>(smem_raw);

    const T *__restrict__ in = static_cast<const T *>(a.in);
    T *__restrict__ out = static_cast<T *>(a.out);
    const A *__restrict__ w = static_cast<const A *>(a.wts);
    const A *coe = coe_of<A>(a);

    const int nt = blockDim.x;
    const int t = threadIdx.x;
    const int W = nt * V;
    const int rowlen = PAD + W + PAD;
    int strip, chunk;
    tile_of(a, strip, chunk);
    const long long i0 = static_cast<long long>(strip) * W;
    const int j0 = chunk * a.rows;
    const int H = min(a.rows, a.ny - j0);
    const int niter = H + NWY - 1;
    const long long ib = i0 + static_cast<long long>(t) * V;
    const bool periodic = a.periodic != 0;
    // Odd chunks walk their rows bottom to top (the window flipped
    // vertically), so the halo rows two neighbouring chunks share are read
    // by both at about the same time and the second read hits in L2.
    const bool up = (chunk & 1) != 0;
    // first input row, and the step between input rows
    const long long rfirst = up ? static_cast<long long>(j0) + H - 1 + a.B : static_cast<long long>(j0) - a.T;
    const int rstep = up ? -1 : 1;
    // upward chunks use the vertically flipped weights (uploaded by the plan)
    const A *__restrict__ wv = up ? static_cast<const A *>(a.wts_up) : w;
    const bool full_vec = a.vec_ok && (ib + V <= a.nx);
    const bool store_vec_ok = full_vec && (periodic || (ib >= a.L && ib + V - 1 <= a.nx - 1 - a.R));

    A acc[NWY][V];
#pragma unroll
    for (int q = 0; q < NWY; ++q)
#pragma unroll
        for (int v = 0; v < V; ++v) acc[q][v] = A(0);

    // Halo values per stage: G rows x 2*PAD columns, at most HPT per thread.
    constexpr int HPT = (G * 2 * PAD + 63) / 64;
    const int hcount = G * 2 * PAD;

    // A stage is "clean" when all its G rows exist (periodic, or inside the
    // grid) and the strip lies inside the grid with aligned vectors: its
    // loads are then issued as straight-line code with no alternative path
    // writing the same registers, so none of them waits for the others (or
    // for earlier stores); halo values outside a non-periodic grid are loaded
    // from a clamped address and zeroed when staged.
    const bool strip_clean = a.vec_ok && i0 + W <= a.nx;
    auto clean_stage = [&](int s0) __attribute__((always_inline)) {
        if (!strip_clean || s0 + G > niter) return false;
        if (periodic) return true;
        const long long ra = rfirst + static_cast<long long>(rstep) * s0;
        const long long rb = rfirst + static_cast<long long>(rstep) * (s0 + G - 1);
        return (ra < rb ? ra : rb) >= 0 && (ra > rb ? ra : rb) < a.ny;
    };
    // halo slot h of a stage: its row within the stage and its column
    auto halo_slot = [&](int h, int &u, long long &c) __attribute__((always_inline)) {
        u = h / (2 * PAD);
        const int hh = h - u * 2 * PAD;
        c = hh < PAD ? i0 - PAD + hh : i0 + W + (hh - PAD);
    };

    // Loads of a clean stage s0 (main vectors and halo values) into registers.
    auto load_clean = [&](int s0, A (&xin)[G][V], A (&hv)[HPT > 0 ? HPT : 1]) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
            long long r = rfirst + static_cast<long long>(rstep) * (s0 + u);
            if (periodic) r = wrap_fast(r, a.ny);
            load_vec<T>(in + r * a.ld + ib, xin[u]);
        }
        if constexpr (NWX > 1) {
#pragma unroll
            for (int q = 0; q < HPT; ++q) {
                const int h = min(t + q * nt, hcount - 1);
                int u;
                long long c;
                halo_slot(h, u, c);
                c = periodic ? wrap_fast(c, a.nx) : (c < 0 ? 0 : (c >= a.nx ? a.nx - 1 : c));
                long long r = rfirst + static_cast<long long>(rstep) * (s0 + u);
                if (periodic) r = wrap_fast(r, a.ny);
                hv[q] = to_acc<T>(in[r * a.ld + c]);
            }
        }
    };
    // Loads of any stage s0.
    auto load_stage = [&](int s0, A (&xin)[G][V], A (&hv)[HPT > 0 ? HPT : 1]) __attribute__((always_inline)) {
        if (clean_stage(s0)) {
            load_clean(s0, xin, hv);
            return;
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int s = s0 + u;
            long long r = rfirst + static_cast<long long>(rstep) * s;
            bool rv = s < niter;
            if (periodic) r = wrap_fast(r, a.ny);
            else rv = rv && r >= 0 && r < a.ny;
            if (rv) {
                const T *rowp = in + r * a.ld;
                if (full_vec) {
                    load_vec<T>(rowp + ib, xin[u]);
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v) xin[u][v] = load_elem<T>(rowp, ib + v, a.nx, periodic);
                }
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v) xin[u][v] = A(0);
            }
        }
        if constexpr (NWX > 1) {
#pragma unroll
            for (int q = 0; q < HPT; ++q) {
                const int h = t + q * nt;
                A val = A(0);
                if (h < hcount) {
                    const int u = h / (2 * PAD);
                    const int hh = h - u * 2 * PAD;
                    const long long c = hh < PAD ? i0 - PAD + hh : i0 + W + (hh - PAD);
                    const int s = s0 + u;
                    long long r = rfirst + static_cast<long long>(rstep) * s;
                    bool rv = s < niter;
                    if (periodic) r = wrap_fast(r, a.ny);
                    else rv = rv && r >= 0 && r < a.ny;
                    if (rv) val = load_elem<T>(in + r * a.ld, c, a.nx, periodic);
                }
                hv[q] = val;
            }
        }
    };

    // acc[k] holds output row s - (NWY-1) + k; input row s meets it with
    // window row NWY-1-k.  After the row, acc[0] is complete: it is written
    // and the window shifts by one row.
    // clean: the output row exists and the whole strip is stored with vectors
    auto consume = [&](const A *x, int s, bool clean) __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < NWY; ++k) {
#pragma unroll
            for (int p = 0; p < NWX; ++p) {
                const A wt = wv[(NWY - 1 - k) * NWX + p];
#pragma unroll
                for (int v = 0; v < V; ++v) acc[k][v] = fma(wt, x[v + p], acc[k][v]);
            }
        }
        const int jj = s - (NWY - 1);
        if (clean) {
            T *rowp = out + static_cast<long long>(up ? j0 + H - 1 - jj : j0 + jj) * a.ld;
            if (a.nt_store) store_vec_nt<T>(rowp + ib, acc[0]);
            else store_vec<T>(rowp + ib, acc[0]);
        } else if (jj >= 0 && jj < H) {
            const int j = up ? j0 + H - 1 - jj : j0 + jj;
            if (periodic || (j >= a.T && j <= a.ny - 1 - a.B)) {
                T *rowp = out + static_cast<long long>(j) * a.ld;
                if (store_vec_ok) {
                    if (a.nt_store) store_vec_nt<T>(rowp + ib, acc[0]);
                    else store_vec<T>(rowp + ib, acc[0]);
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const long long c = ib + v;
                        if (c < a.nx && (periodic || (c >= a.L && c <= a.nx - 1 - a.R)))
                            rowp[c] = from_acc<T>(acc[0][v]);
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k + 1 < NWY; ++k)
#pragma unroll
            for (int v = 0; v < V; ++v) acc[k][v] = acc[k + 1][v];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[NWY - 1][v] = A(0);
    };

    // A stage is consumed "clean" when its G rows all produce output rows that
    // exist, the strip is stored with whole vectors, and the next stage's
    // loads are clean too: its loads and stores are then straight-line code
    // with fixed counts, so waiting for the next stage's loads never waits
    // for this stage's stores.
    const bool strip_store_clean =
        strip_clean && (periodic || (i0 >= a.L && i0 + W - 1 <= static_cast<long long>(a.nx) - 1 - a.R));
    auto clean_iter = [&](int s0) __attribute__((always_inline)) {
        if (!strip_store_clean || s0 < NWY - 1 || s0 + G - NWY >= H || !clean_stage(s0 + G)) return false;
        if (periodic) return true;
        const int ja = up ? j0 + H - 1 - (s0 - (NWY - 1)) : j0 + (s0 - (NWY - 1));
        const int jb = up ? j0 + H - 1 - (s0 + G - NWY) : j0 + (s0 + G - NWY);
        return (ja < jb ? ja : jb) >= a.T && (ja > jb ? ja : jb) <= a.ny - 1 - a.B;
    };

    A cur[G][V], nxt[G][V];
    A hcur[HPT > 0 ? HPT : 1], hnxt[HPT > 0 ? HPT : 1];
    load_stage(0, cur, hcur);

    auto iteration = [&](int s0, bool clean) __attribute__((always_inline)) {
        // the point function is applied once per loaded element: Horner's
        // rule with the coefficient loop outside and the stage's elements
        // inside (the same operations, in the same order, per element)
        if (a.ncoe) {
            constexpr int HQ = NWX > 1 ? HPT : 0;
            A f[G][V], hf[HQ > 0 ? HQ : 1];
            const A top = coe[a.ncoe - 1];
#pragma unroll
            for (int u = 0; u < G; ++u)
#pragma unroll
                for (int v = 0; v < V; ++v) f[u][v] = top;
#pragma unroll
            for (int q = 0; q < HQ; ++q) hf[q] = top;
            for (int m = a.ncoe - 2; m >= 0; --m) {
                const A cm = coe[m];
#pragma unroll
                for (int u = 0; u < G; ++u)
#pragma unroll
                    for (int v = 0; v < V; ++v) f[u][v] = f[u][v] * cur[u][v] + cm;
#pragma unroll
                for (int q = 0; q < HQ; ++q) hf[q] = hf[q] * hcur[q] + cm;
            }
#pragma unroll
            for (int u = 0; u < G; ++u)
#pragma unroll
                for (int v = 0; v < V; ++v) cur[u][v] = f[u][v];
#pragma unroll
            for (int q = 0; q < HQ; ++q) hcur[q] = hf[q];
        }
        if constexpr (NWX > 1) {
            __syncthreads();   // the previous stage's LDS reads are done
#pragma unroll
            for (int u = 0; u < G; ++u) {
                A *dst = lds + u * rowlen + PAD + t * V;
#pragma unroll
                for (int v = 0; v < V; ++v) dst[v] = cur[u][v];
            }
            const bool cl = clean_stage(s0);
#pragma unroll
            for (int q = 0; q < HPT; ++q) {
                const int h = t + q * nt;
                if (h < hcount) {
                    const int u = h / (2 * PAD);
                    const int hh = h - u * 2 * PAD;
                    long long c;
                    int uu;
                    halo_slot(h, uu, c);
                    const bool zero = cl && !periodic && (c < 0 || c >= a.nx);
                    lds[u * rowlen + (hh < PAD ? hh : W + hh)] = zero ? A(0) : hcur[q];
                }
            }
        }
        // next stage's loads overlap this stage's arithmetic
        if (clean) load_clean(s0 + G, nxt, hnxt);
        else if (s0 + G < niter) load_stage(s0 + G, nxt, hnxt);
        if constexpr (NWX > 1) {
            __syncthreads();
            const int nu = clean ? G : min(G, niter - s0);
#pragma unroll 1
            for (int u = 0; u < nu; ++u) {
                A x[XW];
                const A *lp = lds + u * rowlen + PAD + t * V - a.L;
#pragma unroll
                for (int k = 0; k < XW; ++k) x[k] = lp[k];
                consume(x, s0 + u, clean);
            }
        } else {
#pragma unroll
            for (int u = 0; u < G; ++u)
                if (clean || s0 + u < niter) consume(cur[u], s0 + u, clean);
        }
#pragma unroll
        for (int u = 0; u < G; ++u)
#pragma unroll
            for (int v = 0; v < V; ++v) cur[u][v] = nxt[u][v];
#pragma unroll
        for (int q = 0; q < (HPT > 0 ? HPT : 1); ++q) hcur[q] = hnxt[q];
    };

    int s0 = 0;
    while (s0 < niter && !clean_iter(s0)) {
        iteration(s0, false);
        s0 += G;
    }
    while (s0 < niter && clean_iter(s0)) {
        iteration(s0, true);
        s0 += G;
    }
    while (s0 < niter) {
        iteration(s0, false);
        s0 += G;
    }
}

// Value of the neighbouring lane across the whole wavefront: SHR gives lane
// i the value of lane i - 1, SHL the value of lane i + 1 (DPP wave shifts;
// the lane at the end of the wavefront receives 0).
template <int CTRL> __device__ __forceinline__ double wave_shift(double v) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, 0xf, 0xf, false));
    const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xf, 0xf, false));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}
template <int CTRL> __device__ __forceinline__ float wave_shift(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppWaveShr1 = 0x138;

// Block form (windows of 3 or 5 rows): a workgroup requests all GIN input
// rows of its chunk at once, GIN - NWY + 1 output rows, stages them in LDS
// with their x halo (NWX > 1) and computes every output row of the chunk;
// there is no streaming loop, so every load of the workgroup is in flight
// together, as in a plain copy.  Neighbouring chunks both read the NWY - 1
// rows they share; with chunks of one strip dispatched close together the
// second read is served by L2.  Rows and columns outside a non-periodic grid
// are read from clamped addresses: they only meet outputs that are not
// written (or padded taps of weight zero).
//
// XS (x exchange by lanes, centred windows only: left = right = NWX / 2 <=
// V): the x neighbours of a thread's V values come from the neighbouring
// lanes by DPP wave shifts instead of an LDS row; the two lanes at the ends
// of a wavefront load their outside neighbours themselves.  No LDS, no
// barrier.
template <typename T, int NWX, int NWY, int GIN, bool CLEAN, bool XS>
__device__ __forceinline__ void block_body(const Stencil2DArgs &a, int strip, int chunk, unsigned char *smem) {
    using A = typename St<T>::acc;
    constexpr int V = St<T>::V;
    constexpr int PAD = halo_pad<NWX, V>();
    constexpr int XW = V + NWX - 1;
    constexpr int ROWS = GIN - NWY + 1;
    constexpr int HPT = (GIN * 2 * PAD + 63) / 64;
    A *lds = reinterpret_cast<A *>(smem);
    const gptr<const T> in = as_global(static_cast<const T *>(a.in));
    const gptr<T> out = as_global(static_cast<T *>(a.out));
    const A *__restrict__ w = static_cast<const A *>(a.wts);
    const A *coe = coe_of<A>(a);
    const int nt = blockDim.x;
    const int t = threadIdx.x;
    const int W = nt * V;
    const int rowlen = PAD + W + PAD;
    const long long i0 = static_cast<long long>(strip) * W;
    const int j0 = chunk * ROWS;
    const int H = min(ROWS, a.ny - j0);
    const long long ib = i0 + static_cast<long long>(t) * V;
    const bool periodic = a.periodic != 0;

    // grid row of input row u
    auto in_row = [&](int u) __attribute__((always_inline)) {
        long long r = static_cast<long long>(j0) - a.T + u;
        if (periodic) return wrap_fast(r, a.ny);
        return r < 0 ? 0LL : (r >= a.ny ? static_cast<long long>(a.ny) - 1 : r);
    };
    A xin[GIN][V];
#pragma unroll
    for (int u = 0; u < GIN; ++u) {
        const gptr<const T> rowp = in + in_row(u) * a.ld;
        if (CLEAN) {
            load_vec<T>(rowp + ib, xin[u]);
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                long long c = ib + v;
                c = periodic ? wrap_fast(c, a.nx) : (c >= a.nx ? a.nx - 1 : c);
                xin[u][v] = to_acc<T>(gld<T>(rowp, c));
            }
        }
    }
    constexpr int HX = NWX / 2;   // lane exchange: neighbours on each side
    const int lane = t & 63;
    // lane exchange: lane 0 loads the HX values left of its vector, lane 63
    // the HX values right of it
    A ev[GIN][HX > 0 ? HX : 1];
    if constexpr (XS && HX > 0) {
        if (lane == 0 || lane == 63) {
#pragma unroll
            for (int u = 0; u < GIN; ++u) {
                const gptr<const T> rowp = in + in_row(u) * a.ld;
#pragma unroll
                for (int h = 0; h < HX; ++h) {
                    long long c = lane == 0 ? ib - HX + h : ib + V + h;
                    c = periodic ? wrap_fast(c, a.nx) : (c < 0 ? 0 : (c >= a.nx ? a.nx - 1 : c));
                    ev[u][h] = to_acc<T>(gld<T>(rowp, c));
                }
            }
        }
    }
    A hv[HPT > 0 ? HPT : 1];
    const int hcount = GIN * 2 * PAD;
#pragma unroll
    for (int q = 0; q < (XS ? 0 : HPT); ++q) {
        const int h = min(t + q * nt, hcount - 1);
        const int u = h / (2 * PAD);
        const int hh = h - u * 2 * PAD;
        long long c = hh < PAD ? i0 - PAD + hh : i0 + W + (hh - PAD);
        c = periodic ? wrap_fast(c, a.nx) : (c < 0 ? 0 : (c >= a.nx ? a.nx - 1 : c));
        hv[q] = to_acc<T>(gld<T>(in + in_row(u) * a.ld, c));
    }
    if (a.ncoe) {
        // Horner's rule, coefficient loop outside (one uniform load per
        // coefficient), the same operations per element as point_fun
        const A top = coe[a.ncoe - 1];
        A f[GIN][V], hf[HPT > 0 ? HPT : 1];
#pragma unroll
        for (int u = 0; u < GIN; ++u)
#pragma unroll
            for (int v = 0; v < V; ++v) f[u][v] = top;
        constexpr int HQ = XS ? 0 : HPT;
        constexpr int EQ = XS ? HX : 0;
        A ef[GIN][EQ > 0 ? EQ : 1];
#pragma unroll
        for (int q = 0; q < HQ; ++q) hf[q] = top;
#pragma unroll
        for (int u = 0; u < GIN; ++u)
#pragma unroll
            for (int h = 0; h < EQ; ++h) ef[u][h] = top;
        for (int m = a.ncoe - 2; m >= 0; --m) {
            const A cm = coe[m];
#pragma unroll
            for (int u = 0; u < GIN; ++u)
#pragma unroll
                for (int v = 0; v < V; ++v) f[u][v] = f[u][v] * xin[u][v] + cm;
#pragma unroll
            for (int q = 0; q < HQ; ++q) hf[q] = hf[q] * hv[q] + cm;
#pragma unroll
            for (int u = 0; u < GIN; ++u)
#pragma unroll
                for (int h = 0; h < EQ; ++h) ef[u][h] = ef[u][h] * ev[u][h] + cm;
        }
#pragma unroll
        for (int u = 0; u < GIN; ++u)
#pragma unroll
            for (int v = 0; v < V; ++v) xin[u][v] = f[u][v];
#pragma unroll
        for (int q = 0; q < HQ; ++q) hv[q] = hf[q];
#pragma unroll
        for (int u = 0; u < GIN; ++u)
#pragma unroll
            for (int h = 0; h < EQ; ++h) ev[u][h] = ef[u][h];
    }
    // lane exchange: the window of every input row, columns ib - HX ..
    // ib + V - 1 + HX
    A xw[XS ? GIN : 1][XS ? V + 2 * HX : 1];
    if constexpr (XS) {
#pragma unroll
        for (int u = 0; u < GIN; ++u) {
#pragma unroll
            for (int h = 0; h < HX; ++h) {
                const A l = wave_shift<kDppWaveShr1>(xin[u][V - HX + h]);
                const A r = wave_shift<kDppWaveShl1>(xin[u][h]);
                xw[u][h] = lane == 0 ? ev[u][h] : l;
                xw[u][HX + V + h] = lane == 63 ? ev[u][h] : r;
            }
#pragma unroll
            for (int v = 0; v < V; ++v) xw[u][HX + v] = xin[u][v];
        }
    }
    if constexpr (NWX > 1 && !XS) {
#pragma unroll
        for (int u = 0; u < GIN; ++u) {
            A *dst = lds + u * rowlen + PAD + t * V;
#pragma unroll
            for (int v = 0; v < V; ++v) dst[v] = xin[u][v];
        }
#pragma unroll
        for (int q = 0; q < HPT; ++q) {
            const int h = t + q * nt;
            if (h < hcount) {
                const int u = h / (2 * PAD);
                const int hh = h - u * 2 * PAD;
                lds[u * rowlen + (hh < PAD ? hh : W + hh)] = hv[q];
            }
        }
        __syncthreads();
    }
    const bool store_vec_ok = a.vec_ok && ib + V <= a.nx &&
                              (periodic || (ib >= a.L && ib + V - 1 <= a.nx - 1 - a.R));
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        A acc[V];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] = A(0);
#pragma unroll
        for (int q = 0; q < NWY; ++q) {
            if constexpr (XS) {
#pragma unroll
                for (int p = 0; p < NWX; ++p) {
                    const A wt = w[q * NWX + p];
#pragma unroll
                    for (int v = 0; v < V; ++v) acc[v] = fma(wt, xw[k + q][v + p], acc[v]);
                }
            } else if constexpr (NWX > 1) {
                A x[XW];
                const A *lp = lds + (k + q) * rowlen + PAD + t * V - a.L;
#pragma unroll
                for (int m = 0; m < XW; ++m) x[m] = lp[m];
#pragma unroll
                for (int p = 0; p < NWX; ++p) {
                    const A wt = w[q * NWX + p];
#pragma unroll
                    for (int v = 0; v < V; ++v) acc[v] = fma(wt, x[v + p], acc[v]);
                }
            } else {
                const A wt = w[q];
#pragma unroll
                for (int v = 0; v < V; ++v) acc[v] = fma(wt, xin[k + q][v], acc[v]);
            }
        }
        const int j = j0 + k;
        if (k >= H || (!periodic && (j < a.T || j > a.ny - 1 - a.B))) continue;
        const gptr<T> rowp = out + static_cast<long long>(j) * a.ld;
        if (CLEAN && store_vec_ok) {
            if (a.nt_store) store_vec_nt<T>(rowp + ib, acc);
            else store_vec<T>(rowp + ib, acc);
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const long long c = ib + v;
                if (c < a.nx && (periodic || (c >= a.L && c <= a.nx - 1 - a.R)))
                    gst<T>(rowp, c, from_acc<T>(acc[v]));
            }
        }
    }
}

template <typename T, int NWX, int NWY, int GIN, bool XS>
__global__ void __launch_bounds__(256) stencil2d_block_kernel(const Stencil2DArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int strip, chunk;
    tile_of(a, strip, chunk);
    const long long W = static_cast<long long>(blockDim.x) * St<T>::V;
    // a strip whose vectors all lie inside the grid, aligned: vector loads only
    if (a.vec_ok && (strip + 1) * W <= a.nx)
        block_body<T, NWX, NWY, GIN, true, XS>(a, strip, chunk, smem_raw);
    else
        block_body<T, NWX, NWY, GIN, false, XS>(a, strip, chunk, smem_raw);
}

template <typename T, int NWX, int NWY, int GIN>
hipError_t launch_block(const Stencil2DArgs &a, int threads, hipStream_t s) {
    using A = typename St<T>::acc;
    constexpr int V = St<T>::V;
    const int grid = a.nstrips * a.nchunks;
    if constexpr (NWX > 1 && NWX / 2 <= V) {
        if (a.xshuffle) {
            if (a.L != NWX / 2 || a.R != NWX / 2) return hipErrorInvalidValue;
            hipLaunchKernelGGL((stencil2d_block_kernel<T, NWX, NWY, GIN, true>), dim3(grid), dim3(threads), 0, s, a);
            return hipGetLastError();
        }
    }
    if (a.xshuffle) return hipErrorInvalidValue;
    const size_t lds = NWX > 1 ? static_cast<size_t>(GIN) * (2 * halo_pad<NWX, V>() + threads * V) * sizeof(A) : 0;
    hipLaunchKernelGGL((stencil2d_block_kernel<T, NWX, NWY, GIN, false>), dim3(grid), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <typename T, int NWX, int NWY>
hipError_t launch_one(const Stencil2DArgs &a, int threads, hipStream_t s) {
    using A = typename St<T>::acc;
    constexpr int V = St<T>::V;
    const size_t lds = NWX > 1
        ? static_cast<size_t>(stage_rows<NWY>()) * (2 * halo_pad<NWX, V>() + threads * V) * sizeof(A)
        : 0;
    const int grid = a.nstrips * a.nchunks;
    hipLaunchKernelGGL((stencil2d_kernel<T, NWX, NWY>), dim3(grid), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t dispatch_block(int nwx, int nwy, const Stencil2DArgs &a, int threads, hipStream_t s) {
#define MXS_BCASE(X, Y, G) \
    if (nwx == X && nwy == Y && a.block_rows == G) return launch_block<T, X, Y, G>(a, threads, s);
    MXS_BCASE(1, 3, 8) MXS_BCASE(1, 3, 12) MXS_BCASE(1, 3, 16)
    MXS_BCASE(1, 5, 8) MXS_BCASE(1, 5, 12) MXS_BCASE(1, 5, 16)
    MXS_BCASE(3, 3, 8) MXS_BCASE(3, 3, 12) MXS_BCASE(3, 3, 16)
    MXS_BCASE(3, 5, 8) MXS_BCASE(3, 5, 12) MXS_BCASE(3, 5, 16)
    MXS_BCASE(5, 3, 8) MXS_BCASE(5, 3, 12) MXS_BCASE(5, 3, 16)
    MXS_BCASE(5, 5, 8) MXS_BCASE(5, 5, 12) MXS_BCASE(5, 5, 16)
#undef MXS_BCASE
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t dispatch(int nwx, int nwy, const Stencil2DArgs &a, int threads, hipStream_t s) {
    if (a.block_rows) return dispatch_block<T>(nwx, nwy, a, threads, s);
#define MXS_CASE(X, Y) \
    if (nwx == X && nwy == Y) return launch_one<T, X, Y>(a, threads, s);
    MXS_CASE(1, 1) MXS_CASE(3, 1) MXS_CASE(5, 1) MXS_CASE(9, 1) MXS_CASE(17, 1)
    MXS_CASE(1, 3) MXS_CASE(1, 5) MXS_CASE(1, 9) MXS_CASE(1, 17)
    MXS_CASE(3, 3) MXS_CASE(3, 5) MXS_CASE(3, 9)
    MXS_CASE(5, 3) MXS_CASE(5, 5) MXS_CASE(5, 9)
    MXS_CASE(9, 3) MXS_CASE(9, 5) MXS_CASE(9, 9)
#undef MXS_CASE
    return hipErrorInvalidValue;
}

// Reads a buffer once (grid-stride, 16-byte loads) and writes nothing back
// unless its words XOR to a fixed value (then one word of the same buffer,
// which only serves this kernel): the loads replace the contents of the
// memory-side cache with clean lines.
__global__ void __launch_bounds__(256) cache_flush_kernel(void *buf, size_t n16) {
    const gptr<const v4u_t> p = as_global(static_cast<const v4u_t *>(buf));
    uint32_t x = 0;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n16;
         i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const v4u_t v = p[i];
        x ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (x == 0x9e3779b9u) as_global(reinterpret_cast<uint32_t *>(buf))[0] = x;
}

}  // namespace

hipError_t launch_cache_flush(void *buf, size_t bytes, hipStream_t s) {
    hipLaunchKernelGGL(cache_flush_kernel, dim3(2048), dim3(256), 0, s, buf, bytes / 16);
    return hipGetLastError();
}

int bucket_width(int taps) {
    if (taps <= 1) return 1;
    if (taps <= 3) return 3;
    if (taps <= 5) return 5;
    if (taps <= 9) return 9;
    if (taps <= 17) return 17;
    return 0;
}

bool stencil2d_block_ok(int nwx, int nwy, int block_rows) {
    return (nwx == 1 || nwx == 3 || nwx == 5) && (nwy == 3 || nwy == 5) &&
           (block_rows == 8 || block_rows == 12 || block_rows == 16);
}

bool stencil2d_xshuffle_ok(int dtype, int nwx, int nwy, int left, int right, int block_rows) {
    const int V = dtype == F64 ? St<double>::V : dtype == F32 ? St<float>::V : St<bf16>::V;
    return stencil2d_block_ok(nwx, nwy, block_rows) && nwx > 1 && nwx / 2 <= V && left == nwx / 2 &&
           right == nwx / 2;
}

size_t stencil2d_lds_bytes(int dtype, int nwx, int nwy, int threads, int block_rows, int xshuffle) {
    if (nwx <= 1 || xshuffle) return 0;
    const int V = dtype == F64 ? St<double>::V : dtype == F32 ? St<float>::V : St<bf16>::V;
    const int acc = dtype == F64 ? 8 : 4;
    const int pad = ((nwx - 1 + V - 1) / V) * V;
    const int g = block_rows ? block_rows : 4;
    (void)nwy;
    return static_cast<size_t>(g) * (2 * pad + threads * V) * acc;
}

hipError_t launch_stencil2d(int dtype, int nwx, int nwy, const Stencil2DArgs &a, int threads,
                            hipStream_t s) {
    switch (dtype) {
    case F64: return dispatch<double>(nwx, nwy, a, threads, s);
    case F32: return dispatch<float>(nwx, nwy, a, threads, s);
    case BF16: return dispatch<bf16>(nwx, nwy, a, threads, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mxs
