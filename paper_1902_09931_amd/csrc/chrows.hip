// The x sweep of the ADI Cahn-Hilliard step (Sec. 5.1) with its right-hand
// side formed inside the row solves, so that R never goes to memory:
//
//   L_x w = R,  R = cdiff (C^n - C^{n-1}) + sum wb * Cbar + sum wl * (C^n^3 - C^n),
//
// Cbar = 2 C^n - C^{n-1} (the terms as in ch.h).  A workgroup of WR
// wavefronts (WR = 4 or 8) takes WR consecutive rows of one instance.  The
// rows are walked in sub-blocks of 64 WR CPT columns (CPT = 1 or 2 columns
// per thread): for each, every thread requests its columns of the WR + 4
// input rows of C^n and C^{n-1} the rows' windows reach (periodic in both
// directions; two halo columns on each side from 4 (WR + 4) threads), the
// workgroup stages Cbar, C^n^3 - C^n and C^n - C^{n-1} in LDS, and each
// wavefront forms R of its own row at the sub-block's columns, directly in
// the register layout the line solver starts from (element BLK c + 64 k +
// lane of the line in raw[c][k] of lane `lane`).  With four rows and one
// column per thread the next sub-block's values are requested before the
// current one is staged.  Then every wavefront solves its row in registers
// (the register line solver of wave_dev.h) and stores w.
//
// Memory: C^n and C^{n-1} are read once per workgroup, WR + 4 rows for WR
// rows of output; the 4 rows a workgroup shares with its neighbours come from
// L2 when the neighbours run at the same time (row groups in one contiguous
// band per XCD).  Only w is written: 2 words read and 1 written per point,
// against 3 + 2 for the right-hand side and row solve as two kernels.
#include "ch_dev.h"
#include "wave_dev.h"

namespace mxs {

namespace {

// Geometry of a workgroup of WR rows: 64 WR threads, sub-blocks of
// 64 WR CPT columns (CPT columns per thread, 64 WR apart), WR + 4 input rows
// per sub-block, LDS rows with two halo columns on each side.
template <int WR, int CPT> struct FusedShape {
    static constexpr int NT = 64 * WR;
    static constexpr int SUB = NT * CPT;
    static constexpr int GIN = WR + 4;
    static constexpr int LW = SUB + 4;
    // LDS values: Cbar on every input row, C^3 - C on the inner GIN - 2,
    // C^n - C^{n-1} on the WR output rows, and 256 values of R per wavefront
    static constexpr int VALS = GIN * LW + (GIN - 2) * LW + WR * SUB + WR * 256;
};

// N consecutive values from LDS at a 16-byte aligned address, by 16-byte reads.
template <typename A, int N> __device__ __forceinline__ void lds_read(const A *p, A *x) {
    constexpr int PER = 16 / static_cast<int>(sizeof(A));
    static_assert(N % PER == 0, "whole 16-byte vectors");
#pragma unroll
    for (int k = 0; k < N; k += PER) {
        if constexpr (PER == 2) {
            const v2d_t v = *reinterpret_cast<const v2d_t *>(p + k);
            x[k] = v.x;
            x[k + 1] = v.y;
        } else {
            const v4f_t v = *reinterpret_cast<const v4f_t *>(p + k);
            x[k] = v.x;
            x[k + 1] = v.y;
            x[k + 2] = v.z;
            x[k + 3] = v.w;
        }
    }
}

// The slots [s0, s0 + n) a lane reads from an LDS row for taps lo..hi of its
// four outputs (output i, tap p at slot i + p + shift), widened to whole
// 16-byte vectors.
struct SlotRange {
    int s0, n;
};
template <typename A> constexpr SlotRange slot_range(int lo, int hi, int shift) {
    const int per = 16 / static_cast<int>(sizeof(A));
    const int first = lo + shift, last = 3 + hi + shift;
    const int s0 = first / per * per;
    return SlotRange{s0, (last + 1 - s0 + per - 1) / per * per};
}

template <typename T, typename TW, int NB, int WR, int CPT>
__global__ void __launch_bounds__(64 * WR) ch_rhs_rows_kernel(const RhsInst *__restrict__ rhs,
                                                              const RowsInst *__restrict__ rows,
                                                              const RowGroup *__restrict__ work, int count) {
    using A = typename St<T>::acc;
    using FS = FusedShape<WR, CPT>;
    constexpr int NT = FS::NT, SUB = FS::SUB, GIN = FS::GIN, LW = FS::LW;
    constexpr int E = WaveShape<NB>::E, NBB = WaveShape<NB>::NBB;
    constexpr int BLK = 64 * E;
    constexpr int NST = (NBB * BLK + SUB - 1) / SUB;   // sub-blocks of the longest line of the class
    // With one column per thread and four rows the next sub-block is
    // requested before the current one is staged; wider sub-blocks (or
    // eight rows) hold as many values per thread in flight at once instead,
    // and the registers of a second set would not fit beside the line.
    constexpr bool PREFETCH = WR <= 4 && CPT == 1;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    A *lb = reinterpret_cast<A *>(smem_raw);   // Cbar           [GIN][LW]
    A *lf = lb + GIN * LW;                     // C^3 - C        [GIN - 2][LW], input rows 1 .. GIN - 2
    A *ld = lf + (GIN - 2) * LW;               // C^n - C^{n-1}  [WR][SUB]

    const RowGroup g = work[xcd_tile(blockIdx.x, count)];
    const RhsInst &I = rhs[g.inst];
    const RowsInst &RI = rows[g.inst];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const int nx = I.nx, ny = I.ny, j0 = g.j0;
    const int nsub = ((nx - 1) / BLK + 1) * BLK;   // columns of the line's blocks
    const gptr<const T> cur = as_global(static_cast<const T *>(I.cur));
    const gptr<const T> prev = as_global(static_cast<const T *>(I.prev));

    A wb[25], wl[9];
#pragma unroll
    for (int k = 0; k < 25; ++k) wb[k] = bih_tap(k / 5, k % 5) ? wb_of<A>(I, k) : A(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) wl[k] = lap_tap(k / 3, k % 3) ? wl_of<A>(I, k) : A(0);
    const A cdiff = cd_of<A>(I);

    long long roff[GIN];   // offsets of the input rows j0 - 2 .. j0 + WR + 1
#pragma unroll
    for (int u = 0; u < GIN; ++u) roff[u] = wrap_fast(static_cast<long long>(j0) - 2 + u, ny) * nx;
    // halo: thread t < 4 GIN loads halo slot h = t % 4 of input row t / 4
    const int hu = min(t >> 2, GIN - 1), hh = t & 3;

    // request the values of sub-block st (columns SUB st ..): column
    // SUB st + t + NT j of every input row into c[u][j], p[u][j]
    auto load = [&](int st, A (&c)[GIN][CPT], A (&p)[GIN][CPT], A &hc, A &hp) __attribute__((always_inline)) {
        const long long cb = static_cast<long long>(st) * SUB;
        long long col[CPT];
#pragma unroll
        for (int j = 0; j < CPT; ++j) col[j] = wrap_fast(cb + t + NT * j, nx);
#pragma unroll
        for (int u = 0; u < GIN; ++u)
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                c[u][j] = to_acc<T>(gld<T>(cur, roff[u] + col[j]));
                p[u][j] = to_acc<T>(gld<T>(prev, roff[u] + col[j]));
            }
        hc = A(0);
        hp = A(0);
        if (t < 4 * GIN) {
            const long long hcol = wrap_fast(hh < 2 ? cb - 2 + hh : cb + SUB + (hh - 2), nx);
            hc = to_acc<T>(gld<T>(cur, roff[hu] + hcol));
            hp = to_acc<T>(gld<T>(prev, roff[hu] + hcol));
        }
    };

    TW raw[NBB][E];
#pragma unroll
    for (int c = 0; c < NBB; ++c)
#pragma unroll
        for (int k = 0; k < E; ++k) raw[c][k] = TW(0);

    A c0[GIN][CPT], p0[GIN][CPT], c1[PREFETCH ? GIN : 1][CPT], p1[PREFETCH ? GIN : 1][CPT];
    A hc0, hp0, hc1, hp1;
    load(0, c0, p0, hc0, hp0);
#pragma unroll
    for (int st = 0; st < NST; ++st) {
        if (st * SUB >= nsub) continue;   // uniform: past the line's last block
        if (!PREFETCH && st > 0) load(st, c0, p0, hc0, hp0);
        __syncthreads();                  // the previous sub-block's LDS reads are done
#pragma unroll
        for (int u = 0; u < GIN; ++u)
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const A cv = c0[u][j], pv = p0[u][j];
                const int x = 2 + t + NT * j;
                lb[u * LW + x] = A(2) * cv - pv;
                if (u >= 1 && u <= GIN - 2) lf[(u - 1) * LW + x] = cv * cv * cv - cv;
                if (u >= 2 && u < 2 + WR) ld[(u - 2) * SUB + t + NT * j] = cv - pv;
            }
        if (t < 4 * GIN) {
            const int slot = hh < 2 ? hh : SUB + hh;
            lb[hu * LW + slot] = A(2) * hc0 - hp0;
            if (hu >= 1 && hu <= GIN - 2) lf[(hu - 1) * LW + slot] = hc0 * hc0 * hc0 - hc0;
        }
        // the next sub-block's requests overlap this one's arithmetic
        if constexpr (PREFETCH) {
            if (st + 1 < NST && (st + 1) * SUB < nsub) load(st + 1, c1, p1, hc1, hp1);
        }
        __syncthreads();

        // each lane forms R at 4 consecutive columns of every 256 (ob .. ob
        // + 3), reading every window row once with 16-byte reads, and the
        // wavefront moves the values to the line solver's layout (column
        // 64 m + lane) through 256 LDS words of its own
        A *ws = ld + WR * SUB + w * 256;
#pragma unroll
        for (int gq = 0; gq < SUB / 256; ++gq) {
            const int ob = 256 * gq + 4 * lane;
            A acc[4] = {A(0), A(0), A(0), A(0)};
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const int plo = (q == 0 || q == 4) ? 2 : (q == 1 || q == 3) ? 1 : 0;
                constexpr SlotRange r0 = slot_range<A>(2, 2, 0), r1 = slot_range<A>(1, 3, 0),
                                    r2 = slot_range<A>(0, 4, 0);
                const SlotRange r = plo == 2 ? r0 : plo == 1 ? r1 : r2;
                A x[8];
                if (r.n == 4) lds_read<A, 4>(lb + (w + q) * LW + ob + r.s0, x);
                else lds_read<A, 8>(lb + (w + q) * LW + ob + r.s0, x);
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int pp = 0; pp < 5; ++pp)
                        if (bih_tap(q, pp)) acc[i] = fma(wb[q * 5 + pp], x[i + pp - r.s0], acc[i]);
            }
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int plo = q == 1 ? 0 : 1;
                constexpr SlotRange r0 = slot_range<A>(1, 1, 1), r1 = slot_range<A>(0, 2, 1);
                const SlotRange r = plo == 1 ? r0 : r1;
                A x[8];
                if (r.n == 4) lds_read<A, 4>(lf + (w + q) * LW + ob + r.s0, x);
                else lds_read<A, 8>(lf + (w + q) * LW + ob + r.s0, x);
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int pp = 0; pp < 3; ++pp)
                        if (lap_tap(q, pp)) acc[i] = fma(wl[q * 3 + pp], x[i + pp + 1 - r.s0], acc[i]);
            }
            A dv[4];
            lds_read<A, 4>(ld + w * SUB + ob, dv);
#pragma unroll
            for (int i = 0; i < 4; ++i) ws[4 * lane + i] = fma(cdiff, dv[i], acc[i]);
            wave_sync();
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                // column SUB st + 256 gq + 64 m + lane of the line: element
                // BLK c + 64 k + lane
                const int x0 = st * SUB + 256 * gq + 64 * m;   // compile time after unrolling
                const int c = x0 / BLK, k = (x0 % BLK) / 64;
                if (c < NBB) raw[c][k] = static_cast<TW>(ws[64 * m + lane]);
            }
            wave_sync();   // the reads are done before the next group's writes
        }
        if constexpr (PREFETCH) {
#pragma unroll
            for (int u = 0; u < GIN; ++u)
#pragma unroll
                for (int j = 0; j < CPT; ++j) {
                    c0[u][j] = c1[u][j];
                    p0[u][j] = p1[u][j];
                }
            hc0 = hc1;
            hp0 = hp1;
        }
    }
    __syncthreads();   // the LDS becomes the wavefronts' solver stages

    if (j0 + w >= ny) return;
    LineRef L;
    L.in = nullptr;
    L.out = static_cast<TW *>(RI.out) + static_cast<long long>(j0 + w) * RI.ld;
    L.n = nx;
    L.p1 = RI.p1;
    L.p2 = RI.p2;
    L.invK = RI.invK;
    L.pow = RI.pow;
    TW *stage = reinterpret_cast<TW *>(smem_raw) + static_cast<size_t>(w) * Stage<TW, E>::SIZE;
    wave_solve<TW, 2, NB>(L, raw, stage);
}

template <typename T, typename TW, int WR, int CPT>
size_t lds_bytes_of(int nb) {
    using A = typename St<T>::acc;
    const int E = nb <= 1 ? WaveShape<1>::E : nb <= 2 ? WaveShape<2>::E : WaveShape<4>::E;
    const size_t rhs = static_cast<size_t>(FusedShape<WR, CPT>::VALS) * sizeof(A);
    const size_t stage = static_cast<size_t>(WR) * 64 * (E + 16 / sizeof(TW)) * sizeof(TW);
    return rhs > stage ? rhs : stage;
}

template <typename T, typename TW, int NB, int WR, int CPT>
hipError_t launch_nb(const RhsInst *rhs, const RowsInst *rows, const RowGroup *work, int count, hipStream_t s) {
    const size_t lds = lds_bytes_of<T, TW, WR, CPT>(NB);
    hipLaunchKernelGGL((ch_rhs_rows_kernel<T, TW, NB, WR, CPT>), dim3(count), dim3(64 * WR), lds, s, rhs, rows,
                       work, count);
    return hipGetLastError();
}

template <typename T, typename TW, int WR, int CPT>
hipError_t launch_t(int nb, const RhsInst *rhs, const RowsInst *rows, const RowGroup *work, int count,
                    hipStream_t s) {
    switch (nb) {
    case 1: return launch_nb<T, TW, 1, WR, CPT>(rhs, rows, work, count, s);
    case 2: return launch_nb<T, TW, 2, WR, CPT>(rhs, rows, work, count, s);
    case 4: return launch_nb<T, TW, 4, WR, CPT>(rhs, rows, work, count, s);
    case 8: return launch_nb<T, TW, 8, WR, CPT>(rhs, rows, work, count, s);
    case 16: return launch_nb<T, TW, 16, WR, CPT>(rhs, rows, work, count, s);
    default: return hipErrorInvalidValue;
    }
}

// Shapes: (rows per workgroup, columns per thread) = (4, 1), (8, 1), (4, 2).
template <typename T, typename TW>
hipError_t launch_shape(int wr, int cpt, int nb, const RhsInst *rhs, const RowsInst *rows, const RowGroup *work,
                        int count, hipStream_t s) {
    if (wr == 4 && cpt == 1) return launch_t<T, TW, 4, 1>(nb, rhs, rows, work, count, s);
    if (wr == 8 && cpt == 1) return launch_t<T, TW, 8, 1>(nb, rhs, rows, work, count, s);
    if (wr == 4 && cpt == 2) return launch_t<T, TW, 4, 2>(nb, rhs, rows, work, count, s);
    return hipErrorInvalidValue;
}

template <typename T, typename TW>
size_t lds_shape(int wr, int cpt, int nb) {
    if (wr == 4 && cpt == 1) return lds_bytes_of<T, TW, 4, 1>(nb);
    if (wr == 8 && cpt == 1) return lds_bytes_of<T, TW, 8, 1>(nb);
    if (wr == 4 && cpt == 2) return lds_bytes_of<T, TW, 4, 2>(nb);
    return 0;
}

}  // namespace

size_t ch_rhs_rows_lds_bytes(int state_dtype, int wr, int cpt, int nb) {
    switch (state_dtype) {
    case F64: return lds_shape<double, double>(wr, cpt, nb);
    case F32: return lds_shape<float, float>(wr, cpt, nb);
    default: return lds_shape<bf16, float>(wr, cpt, nb);
    }
}

hipError_t launch_ch_rhs_rows(int state_dtype, int wr, int cpt, int nb, const RhsInst *rhs, const RowsInst *rows,
                              const RowGroup *work, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    switch (state_dtype) {
    case F64: return launch_shape<double, double>(wr, cpt, nb, rhs, rows, work, count, s);
    case F32: return launch_shape<float, float>(wr, cpt, nb, rhs, rows, work, count, s);
    case BF16: return launch_shape<bf16, float>(wr, cpt, nb, rhs, rows, work, count, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mxs
