// Device code of the register line solver (one wavefront per line of at
// most kWaveLineMax elements; the method is described in wavelines.hip),
// shared by its kernels (wavelines.hip) and the persistent Cahn-Hilliard step
// (persist.hip).
#pragma once

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
                // every value of the block out of LDS first, then the stores:
                // one wait for the LDS reads instead of one per store
                T ov[E];
#pragma unroll
                for (int k = 0; k < E; ++k) ov[k] = buf[LPC * k * CH + wslot];
                wave_sync();
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    const int idx = BLK * c + 64 * k + lane;
                    if (c < last || idx < n) gst<T>(out, static_cast<unsigned>(idx), ov[k]);
                }
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

}  // namespace
}  // namespace mxs
