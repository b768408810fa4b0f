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

__device__ __forceinline__ Mat mat_mul(const Mat &x, const Mat &y) {
    return Mat{fma(x.a, y.a, x.b * y.c), fma(x.a, y.b, x.b * y.d), fma(x.c, y.a, x.d * y.c),
               fma(x.c, y.b, x.d * y.d)};
}

// M^k for 0 <= k <= 16 * 256, from the table (pw: M^k, k <= 256; pb: M^(256 c))
__device__ __forceinline__ Mat pow_mat(gptr<const double> pw, gptr<const double> pb, int k) {
    return mat_mul(load_mat(pw + 4 * (k & (kWaveBlock - 1))), load_mat(pb + 4 * (k / kWaveBlock)));
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

// value of lane `lane` (uniform) of a double
__device__ __forceinline__ double readlane_d(double v, int lane) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b), lane));
    const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b >> 32), lane));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}
template <int BW> __device__ __forceinline__ S2 readlane_s(S2 v, int lane) {
    return S2{readlane_d(v.x, lane), BW == 2 ? readlane_d(v.y, lane) : 0.0};
}

// cond ? a : b, per component (a select of the whole struct goes through
// the stack)
template <int BW> __device__ __forceinline__ S2 keep_if(bool cond, S2 a, S2 b) {
    return S2{cond ? a.x : b.x, BW == 2 ? (cond ? a.y : b.y) : 0.0};
}

template <int BW> __device__ __forceinline__ S2 pick_row(int r, S2 a0, S2 a1, S2 a2, S2 a3) {
    return keep_if<BW>(r < 2, keep_if<BW>(r == 0, a0, a1), keep_if<BW>(r == 2, a2, a3));
}

// Orders the LDS accesses of one wavefront around a lane exchange: the
// hardware executes a wavefront's LDS instructions in order, the fences keep
// the compiler from moving them.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Register layout of a length class (nb = blocks of 256 the line may span):
// E elements per lane, NBB blocks of 64 E elements.
template <int NB> struct WaveShape;
template <> struct WaveShape<1> { static constexpr int E = 4, NBB = 1; };
template <> struct WaveShape<2> { static constexpr int E = 8, NBB = 1; };
template <> struct WaveShape<4> { static constexpr int E = 16, NBB = 1; };
template <> struct WaveShape<8> { static constexpr int E = 16, NBB = 2; };
template <> struct WaveShape<16> { static constexpr int E = 16, NBB = 4; };

// LDS of one wavefront: one block, each lane's E elements followed by 16
// bytes of padding, so that the chunk reads of consecutive lanes fall in
// different banks.
template <typename T, int E> struct Stage {
    static constexpr int CH = E + 16 / static_cast<int>(sizeof(T));
    static constexpr int SIZE = 64 * CH;
};

// Request every element of a line of n elements (n <= 256 NB) into the
// registers of the calling wavefront, none used yet: element BLK c + 64 k +
// lane goes to raw[c][k] of lane `lane` (coalesced), clamped into the line
// in the last block.
template <typename T, int NB>
__device__ __forceinline__ void wave_fetch(gptr<const T> in, int n,
                                           T (&raw)[WaveShape<NB>::NBB][WaveShape<NB>::E]) {
    constexpr int E = WaveShape<NB>::E, NBB = WaveShape<NB>::NBB;
    constexpr int BLK = 64 * E;
    const int lane = threadIdx.x & 63;
    const int last = (n - 1) / BLK;
#pragma unroll
    for (int c = 0; c < NBB; ++c) {
        if (c < last) {
#pragma unroll
            for (int k = 0; k < E; ++k) raw[c][k] = gld<T>(in, static_cast<unsigned>(BLK * c + 64 * k + lane));
        } else if (c == last) {
#pragma unroll
            for (int k = 0; k < E; ++k) raw[c][k] = gld<T>(in, min(BLK * c + 64 * k + lane, n - 1));
        }
    }
}

// Solve line L, whose elements wave_fetch has requested into raw, with the
// wavefront of the calling lanes (all 64 active), and store it; buf is the
// wavefront's LDS stage.
template <typename T, int BW, int NB>
__device__ __forceinline__ void wave_solve(const LineRef &L,
                                           T (&raw)[WaveShape<NB>::NBB][WaveShape<NB>::E], T *buf) {
    constexpr int E = WaveShape<NB>::E, NBB = WaveShape<NB>::NBB;
    constexpr int BLK = 64 * E;
    constexpr int CH = Stage<T, E>::CH;
    constexpr int LPC = 64 / E;   // lane chunks per 64 consecutive elements
    const int lane = threadIdx.x & 63;
    const int row = lane >> 4, p = lane & 15;
    const int n = L.n;
    const gptr<const double> pw = as_global(L.pow);
    const gptr<const double> pb = pw + 4 * (kWaveBlock + 1);
    const double p1 = L.p1, p2 = L.p2;
    const int last = (n - 1) / BLK;

    // element 64 k + lane of a block sits in chunk LPC k + lane / E, slot lane % E
    const int wslot = (lane / E) * CH + lane % E;

    Mat K[4];   // M^E, M^2E, M^4E, M^8E: the row scan steps
#pragma unroll
    for (int i = 0; i < 4; ++i) K[i] = load_mat(pw + 4 * (E << i));
    const Mat Mrow = load_mat(pw + 4 * (16 * E));   // M^16E: one row of lanes
    const Mat Mn = pow_mat(pw, pb, n);

    double v[NBB][E];
    // valid elements of the calling lane in the last block
    const int cnt = min(max(n - BLK * last - E * lane, 0), E);

    // forward pass A: zero-start state entering every lane, and F
    S2 in0[NBB];
    S2 F{0.0, 0.0};
    {
        const Mat Mp = load_mat(pw + 4 * (E * p));   // M^(E p)
        S2 C{0.0, 0.0};                              // zero-start state entering block c
#pragma unroll
        for (int c = 0; c < NBB; ++c) {
            if (c <= last) {
                // the block into the lanes' registers (through the LDS
                // stage), while the later blocks' loads are still in flight
#pragma unroll
                for (int k = 0; k < E; ++k) buf[LPC * k * CH + wslot] = raw[c][k];
                wave_sync();
#pragma unroll
                for (int j = 0; j < E; ++j) v[c][j] = to_f64<T>(buf[lane * CH + j]);
                wave_sync();
                S2 s{0.0, 0.0};
                if (c < last) {
#pragma unroll
                    for (int j = 0; j < E; ++j) s = rec<BW>(s, v[c][j], p1, p2);
                } else {
#pragma unroll
                    for (int j = 0; j < E; ++j) {
                        if (j >= cnt) v[c][j] = 0.0;
                        const S2 t = rec<BW>(s, v[c][j], p1, p2);
                        s = keep_if<BW>(j < cnt, t, s);
                    }
                }
                const S2 tot = s;
                s = mv_add<BW>(K[0], dpp_s<0x111, BW>(s), s);
                s = mv_add<BW>(K[1], dpp_s<0x112, BW>(s), s);
                s = mv_add<BW>(K[2], dpp_s<0x114, BW>(s), s);
                s = mv_add<BW>(K[3], dpp_s<0x118, BW>(s), s);
                const S2 c0 = C;
                const S2 c1 = mv_add<BW>(Mrow, c0, readlane_s<BW>(s, 15));
                const S2 c2 = mv_add<BW>(Mrow, c1, readlane_s<BW>(s, 31));
                const S2 c3 = mv_add<BW>(Mrow, c2, readlane_s<BW>(s, 47));
                in0[c] = mv_add<BW>(Mp, pick_row<BW>(row, c0, c1, c2, c3), dpp_s<0x111, BW>(s));
                if (c < last) {
                    C = mv_add<BW>(Mrow, c3, readlane_s<BW>(s, 63));
                } else {
                    // state after element n - 1: its lane's incoming state
                    // carried over the lane's valid elements
                    const int ll = (n - 1 - BLK * c) / E;
                    const int cl = n - BLK * c - E * ll;
                    F = mv_add<BW>(load_mat(pw + 4 * cl), readlane_s<BW>(in0[c], ll), readlane_s<BW>(tot, ll));
                }
            }
        }
    }
    const S2 x0 = closure<BW>(Mn, F);

    // forward pass B: true values from the true incoming states
    {
        const Mat W = pow_mat(pw, pb, E * lane);   // M^(E lane)
#pragma unroll
        for (int c = 0; c < NBB; ++c) {
            if (c <= last) {
                const S2 xc = mv<BW>(load_mat(pb + 4 * ((BLK / kWaveBlock) * c)), x0);   // M^(BLK c) x0
                S2 s = mv_add<BW>(W, xc, in0[c]);
                if (c < last) {
#pragma unroll
                    for (int j = 0; j < E; ++j) {
                        s = rec<BW>(s, v[c][j], p1, p2);
                        v[c][j] = s.x;
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < E; ++j) {
                        s = rec<BW>(s, v[c][j], p1, p2);
                        v[c][j] = j < cnt ? s.x : 0.0;
                    }
                }
            }
        }
    }

    // backward pass A: zero-start state entering every lane from above, and
    // the state after element 0 (the elements past the line's end are zero
    // and keep the zero start state zero)
    S2 in1[NBB];
    S2 G{0.0, 0.0};
    {
        const Mat Mq = load_mat(pw + 4 * (E * (15 - p)));   // M^(E (15 - p))
#pragma unroll
        for (int c = NBB - 1; c >= 0; --c) {
            if (c <= last) {
                S2 s{0.0, 0.0};
#pragma unroll
                for (int j = E - 1; j >= 0; --j) s = rec<BW>(s, v[c][j], p1, p2);
                s = mv_add<BW>(K[0], dpp_s<0x101, BW>(s), s);
                s = mv_add<BW>(K[1], dpp_s<0x102, BW>(s), s);
                s = mv_add<BW>(K[2], dpp_s<0x104, BW>(s), s);
                s = mv_add<BW>(K[3], dpp_s<0x108, BW>(s), s);
                const S2 c3 = G;
                const S2 c2 = mv_add<BW>(Mrow, c3, readlane_s<BW>(s, 48));
                const S2 c1 = mv_add<BW>(Mrow, c2, readlane_s<BW>(s, 32));
                const S2 c0 = mv_add<BW>(Mrow, c1, readlane_s<BW>(s, 16));
                in1[c] = mv_add<BW>(Mq, pick_row<BW>(row, c0, c1, c2, c3), dpp_s<0x101, BW>(s));
                G = mv_add<BW>(Mrow, c0, readlane_s<BW>(s, 0));
            }
        }
    }
    const S2 z0 = closure<BW>(Mn, G);

    // backward pass B, scaled by 1/K, and the stores
    const gptr<T> out = as_global(static_cast<T *>(L.out));
    const double invK = L.invK;
    {
        const Mat Wq = pow_mat(pw, pb, E * (63 - lane));   // M^(E (63 - lane))
#pragma unroll
        for (int c = NBB - 1; c >= 0; --c) {
            if (c <= last) {
                S2 s;
                if (c < last) {
                    // z0 carried from the line's top to the block's top
                    const Mat Md = pow_mat(pw, pb, n - BLK * (c + 1));
                    s = mv_add<BW>(Wq, mv<BW>(Md, z0), in1[c]);
#pragma unroll
                    for (int j = E - 1; j >= 0; --j) {
                        s = rec<BW>(s, v[c][j], p1, p2);
                        v[c][j] = s.x * invK;
                    }
                } else {
                    // lanes of the last block: z0 carried over the valid
                    // elements above the lane (d < BLK), as M^(d mod 256)
                    // times M^(256 q) z0
                    const int d = max(n - BLK * c - E * (lane + 1), 0);
                    const int q = d / kWaveBlock;
                    S2 zq = z0;
#pragma unroll
                    for (int qq = 1; qq < (BLK + kWaveBlock - 1) / kWaveBlock; ++qq) {
                        const S2 t = mv<BW>(load_mat(pb + 4 * qq), z0);
                        zq = keep_if<BW>(q == qq, t, zq);
                    }
                    s = mv_add<BW>(load_mat(pw + 4 * (d & (kWaveBlock - 1))), zq, in1[c]);
#pragma unroll
                    for (int j = E - 1; j >= 0; --j) {
                        const S2 t = rec<BW>(s, v[c][j], p1, p2);
                        s = keep_if<BW>(j < cnt, t, s);
                        v[c][j] = s.x * invK;
                    }
                }
#pragma unroll
                for (int j = 0; j < E; ++j) buf[lane * CH + j] = from_f64<T>(v[c][j]);
                wave_sync();
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    const int idx = BLK * c + 64 * k + lane;
                    const T val = buf[LPC * k * CH + wslot];
                    if (c < last || idx < n) gst<T>(out, static_cast<unsigned>(idx), val);
                }
                wave_sync();
            }
        }
    }
}

// Solve line li of a source (rows of a grid table) with the calling
// wavefront.
template <typename T, int BW, int NB, class Src>
__device__ __forceinline__ void wave_line(const Src &src, int li, T *buf) {
    const LineRef L = src.get(li);
    T raw[WaveShape<NB>::NBB][WaveShape<NB>::E];
    wave_fetch<T, NB>(as_global(static_cast<const T *>(L.in)), L.n, raw);
    wave_solve<T, BW, NB>(L, raw, buf);
}

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
