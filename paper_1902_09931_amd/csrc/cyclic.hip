// Cyclic banded line solves (the periodic line inversions of the ADI scheme,
// Sec. 5.1) on the GPU, from the factorisation A = K P(S) P(S^-1) described
// in solve.h.  All elimination arithmetic is double.
//
// Contiguous lines (rows of a grid, or uneven lines stored back to back) go
// one line per workgroup of one or four wavefronts.  The line is copied into
// LDS with coalesced loads (16 in flight per thread); thread t owns the k
// consecutive elements of chunk t.  Each cyclic recurrence is then
//   1. a local pass: every thread runs the recurrence over its chunk from a
//      zero state, giving the affine map state_out = M^len state_in + e;
//   2. an inclusive scan of these affine maps: across the 64 lanes of a
//      wavefront with cross-lane shuffles, then across the wavefronts
//      through LDS; the total gives the wrap-around closure
//      state_-1 = (I - M^n)^-1 e_total;
//   3. a final pass from each thread's true incoming state.
// The backward recurrence is the same with the index order reversed.
//
// Columns of a grid go in three phases over segments of kSeg rows, one lane
// per column (coalesced row accesses):
//   A. per segment: the forward recurrence from zero (end state e) and the
//      backward recurrence from zero over that output (top state g);
//   B. per column: scans over the segments give every segment's true
//      forward incoming state c_s and backward incoming state d_s;
//   C. per segment: both recurrences again from (c_s, d_s), then the output
//      (optionally fused with the Cahn-Hilliard update C^{n+1} = Cbar + v).
#include "cols_dev.h"

namespace mxs {

namespace {

// One step of the recurrence y = b + p1 s0 + p2 s1; the p2 term does not
// depend on the previous step, so the dependent chain is one FMA long.
template <int BW> __device__ __forceinline__ double rec_step(double b, double s0, double s1,
                                                            double p1, double p2) {
    return BW == 2 ? fma(p1, s0, fma(p2, s1, b)) : fma(p1, s0, b);
}

// Chunk length (even, so that chunk strides k + 1 are odd) of a line of n
// elements spread over NT threads; chunk t is stored in LDS at t * (k + 1).
template <int NT> __device__ __forceinline__ int chunk_len(int n) {
    const int k = (n + 2 * NT - 1) / (2 * NT) * 2;
    return k < 2 ? 2 : k;
}

__device__ __forceinline__ int lds_pos(int i, int k, float kinv) {
    int c = static_cast<int>(static_cast<float>(i) * kinv);
    if (c * k > i) --c;
    else if ((c + 1) * k <= i) ++c;
    return c * (k + 1) + (i - c * k);
}

// One cyclic recurrence over a line held in LDS, in place, by the NT = 64 NW
// threads of the workgroup (REV: the index order reversed, i.e. the backward
// recurrence).  xchg holds NW affine maps in LDS.
template <int BW, int NW, bool REV>
__device__ __forceinline__ void block_cyclic_pass(double *line, int n, int k, double p1, double p2, Aff *xchg) {
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int start = min(t * k, n);
    const int len = min(start + k, n) - start;
    double *base = line + t * (k + 1);

    double s0 = 0.0, s1 = 0.0;
    for (int q = 0; q < len; ++q) {
        const int j = REV ? len - 1 - q : q;
        const double y = rec_step<BW>(base[j], s0, s1, p1, p2);
        s1 = s0;
        s0 = y;
    }
    Aff m;
    companion_pow(p1, BW == 2 ? p2 : 0.0, len, m);
    m.e0 = s0;
    m.e1 = s1;

    // inclusive scan within the wavefront, in processing order
    Aff inc = m;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const Aff o = shfl_aff<!REV>(inc, d);
        if (REV ? lane + d < 64 : lane >= d) inc = compose(inc, o);
    }
    // maps of the earlier wavefronts (processing order) and of the whole line
    Aff pre_wave = aff_identity(), tot;
    if constexpr (NW > 1) {
        if (REV ? lane == 0 : lane == 63) xchg[wave] = inc;
        __syncthreads();
        tot = aff_identity();
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const int w = REV ? NW - 1 - q : q;
            const Aff x = xchg[w];
            if ((REV && w > wave) || (!REV && w < wave)) pre_wave = compose(x, pre_wave);
            tot = compose(x, tot);
        }
        __syncthreads();
    } else {
        tot = bcast_aff(inc, REV ? 0 : 63);
    }
    // wrap-around closure: state before the first element = (I - T)^-1 e
    const double ia = 1.0 - tot.a, ib = -tot.b, ic = -tot.c, id = 1.0 - tot.d;
    const double det = ia * id - ib * ic;
    const double x0 = (id * tot.e0 - ib * tot.e1) / det;
    const double x1 = (ia * tot.e1 - ic * tot.e0) / det;
    const Aff prev = shfl_aff<!REV>(inc, 1);
    const Aff pre = (REV ? lane == 63 : lane == 0) ? pre_wave : compose(prev, pre_wave);
    s0 = pre.a * x0 + pre.b * x1 + pre.e0;
    s1 = pre.c * x0 + pre.d * x1 + pre.e1;

    for (int q = 0; q < len; ++q) {
        const int j = REV ? len - 1 - q : q;
        const double y = rec_step<BW>(base[j], s0, s1, p1, p2);
        base[j] = y;
        s1 = s0;
        s0 = y;
    }
}

// Contiguous lines solved by a persistent workgroup, one line at a time.
// The first U * NT elements of the next line are loaded into registers while
// the current line is being solved, so the copy into LDS rarely waits for
// memory; longer lines load their remaining elements in further batches.
// Src::get(li) describes line li: input, output, length and coefficients.
template <typename TI, typename TO, int BW, int NW, class Src>
__device__ __forceinline__ void solve_lines(const Src &src, int nlines, double *smem) {
    constexpr int NT = 64 * NW;
    constexpr int U = 32;
    const int t = threadIdx.x;
    // raw storage values: every load is unconditional (index clamped into
    // the line) so all U are in flight at once; conversion waits for the
    // copy into LDS
    TI r[U];
    auto fetch = [&](const LineRef &L, int b0) {
        const gptr<const TI> in = as_global(static_cast<const TI *>(L.in));
#pragma unroll
        for (int u = 0; u < U; ++u) r[u] = gld<TI>(in, min(b0 + u * NT + t, L.n - 1));
    };
    int li = blockIdx.x;
    LineRef L{};
    if (li < nlines) {
        L = src.get(li);
        fetch(L, 0);
    }
    while (li < nlines) {
        const int n = L.n;
        const int k = chunk_len<NT>(n);
        const float kinv = 1.0f / static_cast<float>(k);
        double *line = smem;
        Aff *xchg = reinterpret_cast<Aff *>(smem + NT * (k + 1));
        __syncthreads();   // the previous line's LDS reads are done
        for (int b0 = 0; b0 < n; b0 += U * NT) {
            if (b0 > 0) fetch(L, b0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = b0 + u * NT + t;
                if (i < n) line[lds_pos(i, k, kinv)] = to_f64<TI>(r[u]);
            }
        }
        __syncthreads();
        const int next = li + gridDim.x;
        LineRef Ln{};
        if (next < nlines) {
            Ln = src.get(next);
            fetch(Ln, 0);   // in flight while this line is solved
        }
        block_cyclic_pass<BW, NW, false>(line, n, k, L.p1, L.p2, xchg);
        block_cyclic_pass<BW, NW, true>(line, n, k, L.p1, L.p2, xchg);
        __syncthreads();
        const gptr<TO> out = as_global(static_cast<TO *>(L.out));
        for (int i = t; i < n; i += NT) gst<TO>(out, i, from_f64<TO>(line[lds_pos(i, k, kinv)] * L.invK));
        li = next;
        L = Ln;
    }
}

template <typename T, int BW, int NW>
__global__ void __launch_bounds__(64 * NW) ragged_lines_kernel(const RaggedLines a) {
    extern __shared__ double smem[];
    solve_lines<T, T, BW, NW>(RaggedSrc<T>{a}, a.nlines, smem);
}

template <typename T, int BW, int NW>
__global__ void __launch_bounds__(64 * NW) rows_kernel(const RowsInst *__restrict__ inst,
                                                       const int *__restrict__ map, int nlines) {
    extern __shared__ double smem[];
    solve_lines<T, T, BW, NW>(RowsSrc<T>{inst, map}, nlines, smem);
}

// ---- column kernels ---------------------------------------------------------------

template <typename TR, int BW>
__global__ void __launch_bounds__(kColsThreads) cols_phase_a(const ColsInst *__restrict__ inst,
                                                            const int *__restrict__ map) {
    cols_a_block<TR, BW>(inst, map, blockIdx.x);
}

template <int BW, int G>
__global__ void __launch_bounds__(kColsThreads) cols_phase_b(const ColsInst *__restrict__ inst,
                                                            const int *__restrict__ map) {
    __shared__ Aff xa[kColsThreads];
    cols_b_block<BW, G>(inst, map, blockIdx.x, xa);
}

template <typename TR, typename TX, int BW, int EPI>
__global__ void __launch_bounds__(kColsThreads) cols_phase_c(const ColsInst *__restrict__ inst,
                                                            const int *__restrict__ map) {
    cols_c_block<TR, TX, BW, EPI>(inst, map, blockIdx.x);
}


template <typename T, int BW>
hipError_t ragged_one(const RaggedLines &a, int nw, int grid, size_t lds, hipStream_t s) {
    if (nw == 4)
        hipLaunchKernelGGL((ragged_lines_kernel<T, BW, 4>), dim3(grid), dim3(256), lds, s, a);
    else if (nw == 2)
        hipLaunchKernelGGL((ragged_lines_kernel<T, BW, 2>), dim3(grid), dim3(128), lds, s, a);
    else
        hipLaunchKernelGGL((ragged_lines_kernel<T, BW, 1>), dim3(grid), dim3(64), lds, s, a);
    return hipGetLastError();
}

template <typename T, int BW>
hipError_t rows_one(const RowsInst *inst, const int *map, int nlines, int nw, int grid, size_t lds,
                    hipStream_t s) {
    if (nw == 4)
        hipLaunchKernelGGL((rows_kernel<T, BW, 4>), dim3(grid), dim3(256), lds, s, inst, map, nlines);
    else if (nw == 2)
        hipLaunchKernelGGL((rows_kernel<T, BW, 2>), dim3(grid), dim3(128), lds, s, inst, map, nlines);
    else
        hipLaunchKernelGGL((rows_kernel<T, BW, 1>), dim3(grid), dim3(64), lds, s, inst, map, nlines);
    return hipGetLastError();
}

template <typename TR, typename TX, int BW, int EPI>
hipError_t cols_one(const ColsInst *inst, const int *mapAC, const int *mapB, int blocksAC,
                    int blocksB, int bgroups, hipStream_t s) {
    hipLaunchKernelGGL((cols_phase_a<TR, BW>), dim3(blocksAC), dim3(kColsThreads), 0, s, inst, mapAC);
    if (bgroups == 16)
        hipLaunchKernelGGL((cols_phase_b<BW, 16>), dim3(blocksB), dim3(kColsThreads), 0, s, inst, mapB);
    else if (bgroups == 4)
        hipLaunchKernelGGL((cols_phase_b<BW, 4>), dim3(blocksB), dim3(kColsThreads), 0, s, inst, mapB);
    else
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((cols_phase_c<TR, TX, BW, EPI>), dim3(blocksAC), dim3(kColsThreads), 0, s,
                       inst, mapAC);
    return hipGetLastError();
}

template <typename TR, typename TX, int EPI>
hipError_t cols_bw(int bw, const ColsInst *inst, const int *mapAC, const int *mapB, int blocksAC,
                   int blocksB, int bgroups, hipStream_t s) {
    return bw == 1 ? cols_one<TR, TX, 1, EPI>(inst, mapAC, mapB, blocksAC, blocksB, bgroups, s)
                   : cols_one<TR, TX, 2, EPI>(inst, mapAC, mapB, blocksAC, blocksB, bgroups, s);
}

}  // namespace

hipError_t launch_ragged_lines(int dtype, int bw, const RaggedLines &a, int nw, int grid,
                               size_t lds, hipStream_t s) {
    switch (dtype * 2 + (bw - 1)) {
    case F64 * 2 + 0: return ragged_one<double, 1>(a, nw, grid, lds, s);
    case F64 * 2 + 1: return ragged_one<double, 2>(a, nw, grid, lds, s);
    case F32 * 2 + 0: return ragged_one<float, 1>(a, nw, grid, lds, s);
    case F32 * 2 + 1: return ragged_one<float, 2>(a, nw, grid, lds, s);
    case BF16 * 2 + 0: return ragged_one<bf16, 1>(a, nw, grid, lds, s);
    case BF16 * 2 + 1: return ragged_one<bf16, 2>(a, nw, grid, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_rows(int dtype, int bw, const RowsInst *inst, const int *map, int nlines, int nw,
                       int grid, size_t lds, hipStream_t s) {
    switch (dtype * 2 + (bw - 1)) {
    case F64 * 2 + 0: return rows_one<double, 1>(inst, map, nlines, nw, grid, lds, s);
    case F64 * 2 + 1: return rows_one<double, 2>(inst, map, nlines, nw, grid, lds, s);
    case F32 * 2 + 0: return rows_one<float, 1>(inst, map, nlines, nw, grid, lds, s);
    case F32 * 2 + 1: return rows_one<float, 2>(inst, map, nlines, nw, grid, lds, s);
    case BF16 * 2 + 0: return rows_one<bf16, 1>(inst, map, nlines, nw, grid, lds, s);
    case BF16 * 2 + 1: return rows_one<bf16, 2>(inst, map, nlines, nw, grid, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_cols(int rhs_dtype, int x_dtype, int bw, int epilogue, const ColsInst *inst,
                       const int *mapAC, const int *mapB, int blocksAC, int blocksB, int bgroups,
                       hipStream_t s) {
    if (bw != 1 && bw != 2) return hipErrorInvalidValue;
    if (epilogue == 0) {
        if (rhs_dtype == F64 && x_dtype == F64) return cols_bw<double, double, 0>(bw, inst, mapAC, mapB, blocksAC, blocksB, bgroups, s);
        if (rhs_dtype == F32 && x_dtype == F32) return cols_bw<float, float, 0>(bw, inst, mapAC, mapB, blocksAC, blocksB, bgroups, s);
        if (rhs_dtype == BF16 && x_dtype == BF16) return cols_bw<bf16, bf16, 0>(bw, inst, mapAC, mapB, blocksAC, blocksB, bgroups, s);
    } else if (bw == 2) {
        if (rhs_dtype == F64 && x_dtype == F64) return cols_one<double, double, 2, 1>(inst, mapAC, mapB, blocksAC, blocksB, bgroups, s);
        if (rhs_dtype == F32 && x_dtype == F32) return cols_one<float, float, 2, 1>(inst, mapAC, mapB, blocksAC, blocksB, bgroups, s);
        if (rhs_dtype == F32 && x_dtype == BF16) return cols_one<float, bf16, 2, 1>(inst, mapAC, mapB, blocksAC, blocksB, bgroups, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace mxs
