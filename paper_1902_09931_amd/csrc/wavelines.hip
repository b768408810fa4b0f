// Cyclic banded line solves with the whole line in the registers of one
// wavefront (lines of at most kWaveLineMax elements).  Same factorisation as
// the other line kernels: the forward recurrence y_i = r_i + p1 y_{i-1} +
// p2 y_{i-2} and the backward one u_i = y_i + p1 u_{i+1} + p2 u_{i+2}, both
// cyclic, then x = u / K (the periodic line inversions of the ADI scheme,
// Sec. 5.1).
//
// Layout: the line is cut into blocks of 64 E elements; in every block lane l
// holds the E consecutive elements 64 E c + E l + j, j = 0..E-1 (E = 4, 8 or
// 16 by line length).  Loads and stores stay coalesced: a block is read with
// one element per lane per instruction and transposed through a small LDS
// buffer of the wavefront.  With the state s_i = (y_i, y_{i-1}) the
// recurrence is s_i = M s_{i-1} + (r_i, 0), M = [[p1, p2], [1, 0]].
//
// Each direction takes two passes over the registers:
//   A. from a zero state at the line start: every lane runs the recurrence
//      over its E elements; a scan of the lane totals within each row of 16
//      lanes (DPP row shifts, multipliers M^E .. M^8E) and a chain over the
//      four row totals (readlane, multiplier M^16E) from the state entering
//      the block give every lane the state entering it, and the state after
//      the line's last element, F;
//   B. the cyclic closure x0 = (I - M^n)^{-1} F is the true state entering
//      the line; a lane's true incoming state is its zero-start state plus
//      M^(index of its first element) x0, and the lane reruns its recurrence
//      from it, which gives the true values directly.
// The backward recurrence is the same with the order of blocks, rows, lanes
// and elements reversed (closure z0 from the state after element 0), and its
// values leave scaled by 1/K.  Elements past the line's end are zero inputs;
// from a zero state they keep the state zero, so the top of a partial block
// needs no special case in the backward zero-start pass.  All powers of M
// come from a table computed on the host: M^k (k <= 256) and M^(256 c).
#include "wave_dev.h"

namespace mxs {

namespace {

// One work unit of ragged lines: `count` consecutive lines (at most K =
// kWaveNBMax / NB) of length class NB, solved one after the other by the
// calling wavefront, every element of line q + 1 requested while line q is
// solved.  Requests past the unit's last line repeat that line (its elements
// come from the cache) so that the request sequence, and with it the waits
// for each line's elements, is the same in every unit.  Double-precision
// pentadiagonal lines of class 8 are not prefetched: the second line's
// registers would not fit beside the first one's solve without spilling.
template <typename T, int BW, int NB>
__device__ __forceinline__ void wave_unit(const RaggedLines &a, int first, int count, T *buf) {
    constexpr int K = kWaveNBMax / NB;
    constexpr bool PREFETCH = !(NB == 8 && BW == 2 && sizeof(T) == 8);
    constexpr int E = WaveShape<NB>::E, NBB = WaveShape<NB>::NBB;
    const gptr<const T> in = as_global(static_cast<const T *>(a.in));
    const gptr<const int> order = as_global(a.order);
    const gptr<const long long> offs = as_global(a.offsets);
    auto line_of = [&](int q, long long &base, int &len) __attribute__((always_inline)) {
        const int b = order[first + min(q, count - 1)];
        base = offs[b];
        len = static_cast<int>(offs[b + 1] - base);
    };
    auto solve = [&](long long base, int len, T (&raw)[NBB][E]) __attribute__((always_inline)) {
        LineRef L;
        L.in = static_cast<const T *>(a.in) + base;
        L.out = static_cast<T *>(a.out) + base;
        L.n = len;
        L.p1 = a.p1;
        L.p2 = a.p2;
        L.invK = a.invK;
        L.pow = a.pow;
        wave_solve<T, BW, NB>(L, raw, buf);
    };
    T ra[NBB][E], rb[NBB][E];
    long long b0, b1;
    int n0, n1;
    line_of(0, b0, n0);
    wave_fetch<T, NB>(in + b0, n0, ra);
    if constexpr (!PREFETCH) {
        solve(b0, n0, ra);
#pragma unroll
        for (int q = 1; q < K; ++q) {
            if (q < count) {
                line_of(q, b0, n0);
                wave_fetch<T, NB>(in + b0, n0, ra);
                solve(b0, n0, ra);
            }
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < K; q += 2) {
        if (q + 1 < K) {
            line_of(q + 1, b1, n1);
            wave_fetch<T, NB>(in + b1, n1, rb);
        }
        if (q < count) solve(b0, n0, ra);
        if (q + 1 < K) {
            if (q + 2 < K) {
                line_of(q + 2, b0, n0);
                wave_fetch<T, NB>(in + b0, n0, ra);
            }
            if (q + 1 < count) solve(b1, n1, rb);
        }
    }
}

// Every ragged line of at most kWaveLineMax elements in one launch: one
// wavefront per workgroup and one work unit per wavefront, the unit's length
// class read from the unit table (a workgroup's registers are released when
// its own unit is done, whatever the lengths of the lines beside it).
template <typename T, int BW>
__global__ void __launch_bounds__(64) wave_units_kernel(const RaggedLines a,
                                                        const WaveUnit *__restrict__ units, int nunits) {
    __shared__ __align__(16) T stage[Stage<T, WaveShape<kWaveNBMax>::E>::SIZE];
    const int u = blockIdx.x;
    if (u >= nunits) return;
    const WaveUnit w = units[u];
    switch (w.nb) {
    case 1: wave_unit<T, BW, 1>(a, w.first, w.count, stage); break;
    case 2: wave_unit<T, BW, 2>(a, w.first, w.count, stage); break;
    case 4: wave_unit<T, BW, 4>(a, w.first, w.count, stage); break;
    case 8: wave_unit<T, BW, 8>(a, w.first, w.count, stage); break;
    default: wave_unit<T, BW, 16>(a, w.first, w.count, stage); break;
    }
}

// One ragged line of class NB per wavefront (positions first .. first +
// count - 1 of the sorted order): one launch per class, each with the
// registers of its own class.
template <typename T, int BW, int NB>
__global__ void __launch_bounds__(64) wave_ragged_kernel(const RaggedLines a, int first, int count) {
    __shared__ __align__(16) T stage[Stage<T, WaveShape<NB>::E>::SIZE];
    const int k = blockIdx.x;
    if (k >= count) return;
    wave_line<T, BW, NB>(RaggedSrc<T>{a}, first + k, stage);
}

template <typename T, int BW, int NB>
__global__ void __launch_bounds__(64) wave_rows_kernel(const RowsInst *__restrict__ inst,
                                                       const int *__restrict__ map, int first,
                                                       int count) {
    __shared__ __align__(16) T stage[Stage<T, WaveShape<NB>::E>::SIZE];
    const int k = blockIdx.x;
    if (k >= count) return;
    wave_line<T, BW, NB>(RowsSrc<T>{inst, map}, first + k, stage);
}

template <typename T>
hipError_t units_bw(int bw, const RaggedLines &a, const WaveUnit *units, int nunits, hipStream_t s) {
    const dim3 grid(nunits), block(64);
    if (bw == 2)
        hipLaunchKernelGGL((wave_units_kernel<T, 2>), grid, block, 0, s, a, units, nunits);
    else
        hipLaunchKernelGGL((wave_units_kernel<T, 1>), grid, block, 0, s, a, units, nunits);
    return hipGetLastError();
}

template <typename T, int BW>
hipError_t ragged_nb(int nb, const RaggedLines &a, int first, int count, hipStream_t s) {
    const dim3 grid(count), block(64);
    switch (nb) {
    case 1: hipLaunchKernelGGL((wave_ragged_kernel<T, BW, 1>), grid, block, 0, s, a, first, count); break;
    case 2: hipLaunchKernelGGL((wave_ragged_kernel<T, BW, 2>), grid, block, 0, s, a, first, count); break;
    case 4: hipLaunchKernelGGL((wave_ragged_kernel<T, BW, 4>), grid, block, 0, s, a, first, count); break;
    case 8: hipLaunchKernelGGL((wave_ragged_kernel<T, BW, 8>), grid, block, 0, s, a, first, count); break;
    case 16: hipLaunchKernelGGL((wave_ragged_kernel<T, BW, 16>), grid, block, 0, s, a, first, count); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int BW>
hipError_t rows_nb(int nb, const RowsInst *inst, const int *map, int first, int count, hipStream_t s) {
    const dim3 grid(count), block(64);
    switch (nb) {
    case 1: hipLaunchKernelGGL((wave_rows_kernel<T, BW, 1>), grid, block, 0, s, inst, map, first, count); break;
    case 2: hipLaunchKernelGGL((wave_rows_kernel<T, BW, 2>), grid, block, 0, s, inst, map, first, count); break;
    case 4: hipLaunchKernelGGL((wave_rows_kernel<T, BW, 4>), grid, block, 0, s, inst, map, first, count); break;
    case 8: hipLaunchKernelGGL((wave_rows_kernel<T, BW, 8>), grid, block, 0, s, inst, map, first, count); break;
    case 16: hipLaunchKernelGGL((wave_rows_kernel<T, BW, 16>), grid, block, 0, s, inst, map, first, count); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t rows_bw(int bw, int nb, const RowsInst *inst, const int *map, int first, int count,
                   hipStream_t s) {
    return bw == 2 ? rows_nb<T, 2>(nb, inst, map, first, count, s)
                   : rows_nb<T, 1>(nb, inst, map, first, count, s);
}

}  // namespace

hipError_t launch_wave_units(int dtype, int bw, const RaggedLines &a, const WaveUnit *units, int nunits,
                             hipStream_t s) {
    if (nunits <= 0) return hipSuccess;
    if (bw != 1 && bw != 2) return hipErrorInvalidValue;
    switch (dtype) {
    case F64: return units_bw<double>(bw, a, units, nunits, s);
    case F32: return units_bw<float>(bw, a, units, nunits, s);
    case BF16: return units_bw<bf16>(bw, a, units, nunits, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_wave_ragged(int dtype, int bw, int nb, const RaggedLines &a, int first, int count,
                              hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (bw != 1 && bw != 2) return hipErrorInvalidValue;
    switch (dtype) {
    case F64: return bw == 2 ? ragged_nb<double, 2>(nb, a, first, count, s) : ragged_nb<double, 1>(nb, a, first, count, s);
    case F32: return bw == 2 ? ragged_nb<float, 2>(nb, a, first, count, s) : ragged_nb<float, 1>(nb, a, first, count, s);
    case BF16: return bw == 2 ? ragged_nb<bf16, 2>(nb, a, first, count, s) : ragged_nb<bf16, 1>(nb, a, first, count, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_wave_rows(int dtype, int bw, int nb, const RowsInst *inst, const int *map, int first,
                            int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    switch (dtype) {
    case F64: return rows_bw<double>(bw, nb, inst, map, first, count, s);
    case F32: return rows_bw<float>(bw, nb, inst, map, first, count, s);
    case BF16: return rows_bw<bf16>(bw, nb, inst, map, first, count, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mxs
