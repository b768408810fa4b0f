// Cyclic banded line solves with the whole line in the registers of one
// wavefront (lines of at most kWaveLineMax elements).  Same factorisation as
// the other line kernels: the forward recurrence y_i = r_i + p1 y_{i-1} +
// p2 y_{i-2} and the backward one u_i = y_i + p1 u_{i+1} + p2 u_{i+2}, both
// cyclic, then x = u / K (the periodic line inversions of the ADI scheme,
// Sec. 5.1).
//
// Layout: block c of the line holds elements 256 c .. 256 c + 255; lane l
// holds the four consecutive elements 256 c + 4 l + j, j = 0..3, of every
// block, so no shared memory is needed.  With the state s_i = (y_i, y_{i-1})
// the recurrence is s_i = M s_{i-1} + (r_i, 0), M = [[p1, p2], [1, 0]], and
// a value is its local value from a zero state plus row 0 of M^{k+1} times
// the state k + 1 steps before it.
//
// Forward recurrence:
//   1. block by block, from zero at the line start: each lane runs the
//      recurrence over its four elements from zero; an inclusive scan within
//      each row of 16 lanes (DPP row shifts, multipliers M^4, M^8, M^16,
//      M^32) and a chain over the four row totals (read with readlane,
//      multiplier M^64) starting from the state entering the block give
//      every lane its incoming state, hence every value, and the state after
//      the block;
//   2. the cyclic closure: with F the state after the last element, the true
//      state entering the line is x0 = (I - M^n)^{-1} F, and value i gains
//      row 0 of M^{i+1} x0 (M^{i+1} = M^{j+1} M^{4p} M^{64 row} M^{256 c}).
// The backward recurrence is the same with the order of blocks, rows, lanes
// and elements reversed, its closure term row 0 of M^{n-i} z0.  All powers of
// M come from a table computed on the host.
#include "lines_dev.h"

namespace mxs {

namespace {

struct S2 {
    double x, y;   // (newest value, previous value)
};

struct Mat {
    double a, b, c, d;   // row-major
};

__device__ __forceinline__ Mat load_mat(gptr<const double> m) { return Mat{m[0], m[1], m[2], m[3]}; }

// s' = M s + (r, 0); the p2 term does not depend on the newest value, so the
// dependent chain is one FMA long.
template <int BW> __device__ __forceinline__ S2 rec(S2 s, double r, double p1, double p2) {
    if constexpr (BW == 2) return S2{fma(p1, s.x, fma(p2, s.y, r)), s.x};
    else return S2{fma(p1, s.x, r), 0.0};
}

// m u + v and m u (BW 1: the scalar state, m.a only)
template <int BW> __device__ __forceinline__ S2 mv_add(const Mat &m, S2 u, S2 v) {
    if constexpr (BW == 2) return S2{fma(m.a, u.x, fma(m.b, u.y, v.x)), fma(m.c, u.x, fma(m.d, u.y, v.y))};
    else return S2{fma(m.a, u.x, v.x), 0.0};
}
template <int BW> __device__ __forceinline__ S2 mv(const Mat &m, S2 u) {
    if constexpr (BW == 2) return S2{fma(m.a, u.x, m.b * u.y), fma(m.c, u.x, m.d * u.y)};
    else return S2{m.a * u.x, 0.0};
}
// row 0 of m times u
template <int BW> __device__ __forceinline__ double row0(const Mat &m, S2 u) {
    if constexpr (BW == 2) return fma(m.a, u.x, m.b * u.y);
    else return m.a * u.x;
}

__device__ __forceinline__ Mat mat_mul(const Mat &x, const Mat &y) {
    return Mat{fma(x.a, y.a, x.b * y.c), fma(x.a, y.b, x.b * y.d), fma(x.c, y.a, x.d * y.c),
               fma(x.c, y.b, x.d * y.d)};
}

// (I - m)^{-1} f
template <int BW> __device__ __forceinline__ S2 closure(const Mat &m, S2 f) {
    if constexpr (BW == 2) {
        const double a = 1.0 - m.a, b = -m.b, c = -m.c, d = 1.0 - m.d;
        const double det = a * d - b * c;
        return S2{(d * f.x - b * f.y) / det, (a * f.y - c * f.x) / det};
    } else {
        return S2{f.x / (1.0 - m.a), 0.0};
    }
}

// Cross-lane moves of a double.  CTRL is a DPP control: 0x100 + d = row_shl:d
// (lane p of a row of 16 reads lane p + d), 0x110 + d = row_shr:d (reads
// p - d); a source outside the row reads zero.  Every lane of the wavefront
// is active where these are used.
template <int CTRL> __device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
                                                       static_cast<unsigned>(lo)));
}
template <int CTRL, int BW> __device__ __forceinline__ S2 dpp_s(S2 v) {
    return S2{dpp_d<CTRL>(v.x), BW == 2 ? dpp_d<CTRL>(v.y) : 0.0};
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b), lane));
    const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b >> 32), lane));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}
template <int BW> __device__ __forceinline__ S2 readlane_s(S2 v, int lane) {
    return S2{readlane_d(v.x, lane), BW == 2 ? readlane_d(v.y, lane) : 0.0};
}

template <int BW> __device__ __forceinline__ S2 pick_row(int r, S2 a0, S2 a1, S2 a2, S2 a3) {
    const S2 lo = r == 0 ? a0 : a1, hi = r == 2 ? a2 : a3;
    return r < 2 ? lo : hi;
}

// Uniform powers of M used by every block.
struct Powers {
    Mat m4[4];          // M^4, M^8, M^16, M^32 (row scan steps)
    Mat m64;            // row carries
    Mat e[5];           // M^1 .. M^4 (element factors; e[0] unused)
};

// Forward recurrence over one block, given fin, the state entering the block
// (from zero at the line start): r[j] inputs (zero where invalid); v[j]
// receive the values and the state after the block is returned (for a full
// block).  Within a row of 16 lanes the lane states are scanned with DPP row
// shifts; the four row totals are chained from fin.
template <int BW>
__device__ __forceinline__ S2 block_forward(const double (&r)[4], double (&v)[4], const Powers &P,
                                            const Mat &Mp, int row, S2 fin, double p1, double p2) {
    S2 s{0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        s = rec<BW>(s, r[j], p1, p2);
        v[j] = s.x;
    }
    s = mv_add<BW>(P.m4[0], dpp_s<0x111, BW>(s), s);
    s = mv_add<BW>(P.m4[1], dpp_s<0x112, BW>(s), s);
    s = mv_add<BW>(P.m4[2], dpp_s<0x114, BW>(s), s);
    s = mv_add<BW>(P.m4[3], dpp_s<0x118, BW>(s), s);
    const S2 ex = dpp_s<0x111, BW>(s);
    const S2 c0 = fin;
    const S2 c1 = mv_add<BW>(P.m64, c0, readlane_s<BW>(s, 15));
    const S2 c2 = mv_add<BW>(P.m64, c1, readlane_s<BW>(s, 31));
    const S2 c3 = mv_add<BW>(P.m64, c2, readlane_s<BW>(s, 47));
    const S2 in = mv_add<BW>(Mp, pick_row<BW>(row, c0, c1, c2, c3), ex);
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] += row0<BW>(P.e[j + 1], in);
    return mv_add<BW>(P.m64, c3, readlane_s<BW>(s, 63));
}

// The same for the backward recurrence (elements, lanes and rows in
// decreasing order); gin is the state entering the block's top element and
// the state after its first element is returned.
template <int BW>
__device__ __forceinline__ S2 block_backward(const double (&r)[4], double (&v)[4], const Powers &P,
                                             const Mat &Mq, int row, S2 gin, double p1, double p2) {
    S2 s{0.0, 0.0};
#pragma unroll
    for (int j = 3; j >= 0; --j) {
        s = rec<BW>(s, r[j], p1, p2);
        v[j] = s.x;
    }
    s = mv_add<BW>(P.m4[0], dpp_s<0x101, BW>(s), s);
    s = mv_add<BW>(P.m4[1], dpp_s<0x102, BW>(s), s);
    s = mv_add<BW>(P.m4[2], dpp_s<0x104, BW>(s), s);
    s = mv_add<BW>(P.m4[3], dpp_s<0x108, BW>(s), s);
    const S2 ex = dpp_s<0x101, BW>(s);
    const S2 c3 = gin;
    const S2 c2 = mv_add<BW>(P.m64, c3, readlane_s<BW>(s, 48));
    const S2 c1 = mv_add<BW>(P.m64, c2, readlane_s<BW>(s, 32));
    const S2 c0 = mv_add<BW>(P.m64, c1, readlane_s<BW>(s, 16));
    const S2 in = mv_add<BW>(Mq, pick_row<BW>(row, c0, c1, c2, c3), ex);
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] += row0<BW>(P.e[4 - j], in);
    return mv_add<BW>(P.m64, c0, readlane_s<BW>(s, 0));
}

// M^(64 r) u for the row r of the calling lane (m[k] = M^(64 k)).
template <int BW> __device__ __forceinline__ S2 by_row(int row, const Mat (&m)[4], S2 u) {
    return pick_row<BW>(row, u, mv<BW>(m[1], u), mv<BW>(m[2], u), mv<BW>(m[3], u));
}

// Solve line li with the wavefront of the calling lanes (all 64 active).
template <typename TI, typename TO, int BW, int NB, class Src>
__device__ __forceinline__ void wave_line(const Src &src, int li) {
    constexpr int B = kWaveBlock;
    const int lane = threadIdx.x & 63;
    const int row = lane >> 4, p = lane & 15;
    const LineRef L = src.get(li);
    const int n = L.n;
    const gptr<const double> pw = as_global(L.pow);   // M^k at pw + 4 k, k <= B
    const gptr<const double> pb = pw + 4 * (B + 1);   // M^(B c) at pb + 4 c
    const double p1 = L.p1, p2 = L.p2;
    const int nblk = (n + B - 1) / B;
    const int last = nblk - 1;
    const int len_last = n - B * last;

    // every element of the line requested before any is used
    const gptr<const TI> in = as_global(static_cast<const TI *>(L.in));
    TI raw[4 * NB];
    // (per-lane 32-bit offsets from the uniform line base; only the last
    // block is clamped into the line)
    const unsigned lo = 4u * lane;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        if (c < last) {
#pragma unroll
            for (int j = 0; j < 4; ++j) raw[4 * c + j] = gld<TI>(in, lo + static_cast<unsigned>(B * c + j));
        } else if (c == last) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                raw[4 * c + j] = gld<TI>(in, min(static_cast<int>(lo) + B * c + j, n - 1));
        }
    }
    Powers P;
    P.m4[0] = load_mat(pw + 16);
    P.m4[1] = load_mat(pw + 32);
    P.m4[2] = load_mat(pw + 64);
    P.m4[3] = load_mat(pw + 128);
    P.m64 = load_mat(pw + 4 * 64);
#pragma unroll
    for (int k = 1; k <= 4; ++k) P.e[k] = load_mat(pw + 4 * k);
    const Mat m64r[4] = {Mat{1.0, 0.0, 0.0, 1.0}, P.m64, load_mat(pw + 4 * 128), load_mat(pw + 4 * 192)};
    const Mat Mp = load_mat(pw + 16 * p);          // M^(4 p)
    const Mat Mq = load_mat(pw + 16 * (15 - p));   // M^(4 (15 - p))
    const Mat Mlen = load_mat(pw + 4 * len_last);
    const Mat Mn = mat_mul(Mlen, load_mat(pb + 4 * last));   // M^n

    // forward recurrence from zero at the line start
    double y[4 * NB];
    S2 F{0.0, 0.0};
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        if (c < last) {
            double r[4], v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) r[j] = to_f64<TI>(raw[4 * c + j]);
            F = block_forward<BW>(r, v, P, Mp, row, F, p1, p2);
#pragma unroll
            for (int j = 0; j < 4; ++j) y[4 * c + j] = v[j];
        } else if (c == last) {
            const int i0 = B * c + 4 * lane;
            double r[4], v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) r[j] = i0 + j < n ? to_f64<TI>(raw[4 * c + j]) : 0.0;
            (void)block_forward<BW>(r, v, P, Mp, row, F, p1, p2);
#pragma unroll
            for (int j = 0; j < 4; ++j) y[4 * c + j] = v[j];
        }
    }
    // state after element n - 1, read from the values of the last block
    // (element n - 2 may be the last one of the block before)
    S2 Fl{0.0, 0.0};
    {
        const int jl = len_last - 1, jm = len_last - 2;
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            if (c == last) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if ((jl & 3) == j) Fl.x = readlane_d(y[4 * c + j], jl >> 2);
                    if (BW == 2 && jm >= 0 && (jm & 3) == j) Fl.y = readlane_d(y[4 * c + j], jm >> 2);
                }
                if (BW == 2 && jm < 0 && c > 0) Fl.y = readlane_d(y[4 * c - 1], 63);
            }
        }
    }
    const S2 x0 = closure<BW>(Mn, Fl);

    // true forward values (+ row 0 of M^(i+1) x0), then the backward
    // recurrence from zero at the top, top block first
    S2 G{0.0, 0.0};
#pragma unroll
    for (int c = NB - 1; c >= 0; --c) {
        if (c <= last) {
            const S2 w = mv<BW>(Mp, by_row<BW>(row, m64r, mv<BW>(load_mat(pb + 4 * c), x0)));
            double r[4], v[4];
            if (c == last) {
                const int i0 = B * c + 4 * lane;
#pragma unroll
                for (int j = 0; j < 4; ++j) r[j] = i0 + j < n ? y[4 * c + j] + row0<BW>(P.e[j + 1], w) : 0.0;
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) r[j] = y[4 * c + j] + row0<BW>(P.e[j + 1], w);
            }
            G = block_backward<BW>(r, v, P, Mq, row, G, p1, p2);
#pragma unroll
            for (int j = 0; j < 4; ++j) y[4 * c + j] = v[j];
        }
    }
    const S2 z0 = closure<BW>(Mn, G);

    // true backward values (+ row 0 of M^(n-i) z0), scaled output
    const gptr<TO> out = as_global(static_cast<TO *>(L.out));
    const double invK = L.invK;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        if (c < last) {
            // n - i = len_last + B (last - 1 - c) + 64 (3 - row) + 4 (15 - p) + (4 - j)
            const S2 u = mv<BW>(Mlen, mv<BW>(load_mat(pb + 4 * (last - 1 - c)), z0));
            const S2 w = mv<BW>(Mq, by_row<BW>(3 - row, m64r, u));
#pragma unroll
            for (int j = 0; j < 4; ++j)
                gst<TO>(out, lo + static_cast<unsigned>(B * c + j),
                        from_f64<TO>((y[4 * c + j] + row0<BW>(P.e[4 - j], w)) * invK));
        } else if (c == last) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = len_last - 4 * lane - j;   // n - i, in 1..len_last when valid
                if (k >= 1)
                    gst<TO>(out, B * c + 4 * lane + j, from_f64<TO>((y[4 * c + j] + row0<BW>(load_mat(pw + 4 * k), z0)) * invK));
            }
        }
    }
}

template <typename T, int BW, int NB>
__global__ void __launch_bounds__(256) wave_ragged_kernel(const RaggedLines a, int first, int count) {
    const int k = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (k >= count) return;
    wave_line<T, T, BW, NB>(RaggedSrc<T>{a}, first + k);
}

template <typename T, int BW, int NB>
__global__ void __launch_bounds__(256) wave_rows_kernel(const RowsInst *__restrict__ inst,
                                                        const int *__restrict__ map, int first,
                                                        int count) {
    const int k = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (k >= count) return;
    wave_line<T, T, BW, NB>(RowsSrc<T>{inst, map}, first + k);
}

template <typename T, int BW>
hipError_t ragged_nb(int nb, const RaggedLines &a, int first, int count, hipStream_t s) {
    const dim3 grid((count + 3) / 4), block(256);
    switch (nb) {
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
    const dim3 grid((count + 3) / 4), block(256);
    switch (nb) {
    case 2: hipLaunchKernelGGL((wave_rows_kernel<T, BW, 2>), grid, block, 0, s, inst, map, first, count); break;
    case 4: hipLaunchKernelGGL((wave_rows_kernel<T, BW, 4>), grid, block, 0, s, inst, map, first, count); break;
    case 8: hipLaunchKernelGGL((wave_rows_kernel<T, BW, 8>), grid, block, 0, s, inst, map, first, count); break;
    case 16: hipLaunchKernelGGL((wave_rows_kernel<T, BW, 16>), grid, block, 0, s, inst, map, first, count); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t ragged_bw(int bw, int nb, const RaggedLines &a, int first, int count, hipStream_t s) {
    return bw == 2 ? ragged_nb<T, 2>(nb, a, first, count, s) : ragged_nb<T, 1>(nb, a, first, count, s);
}
template <typename T>
hipError_t rows_bw(int bw, int nb, const RowsInst *inst, const int *map, int first, int count,
                   hipStream_t s) {
    return bw == 2 ? rows_nb<T, 2>(nb, inst, map, first, count, s)
                   : rows_nb<T, 1>(nb, inst, map, first, count, s);
}

}  // namespace

hipError_t launch_wave_ragged(int dtype, int bw, int nb, const RaggedLines &a, int first, int count,
                              hipStream_t s) {
    if (count <= 0) return hipSuccess;
    switch (dtype) {
    case F64: return ragged_bw<double>(bw, nb, a, first, count, s);
    case F32: return ragged_bw<float>(bw, nb, a, first, count, s);
    case BF16: return ragged_bw<bf16>(bw, nb, a, first, count, s);
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
