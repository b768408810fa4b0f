// Device code of the column solves over segments of kSeg rows (phases A, B
// and C of the cyclic line solve along columns, with the optional fused
// Cahn-Hilliard update), shared by their kernels (cyclic.hip) and the
// persistent Cahn-Hilliard step (persist.hip).  Each phase is a function of
// the workgroup index it plays, so that one kernel can run it for any block.
#pragma once

#include "lines_dev.h"

namespace mxs {
namespace {

// ---- affine maps on the 2-vector state (y_i, y_{i-1}) ----------------------
struct Aff {
    double a, b, c, d;   // matrix, row-major
    double e0, e1;       // offset
};

__device__ __forceinline__ Aff compose(const Aff &hi, const Aff &lo) {
    // (hi o lo)(s) = hi.T (lo.T s + lo.e) + hi.e
    Aff r;
    r.a = hi.a * lo.a + hi.b * lo.c;
    r.b = hi.a * lo.b + hi.b * lo.d;
    r.c = hi.c * lo.a + hi.d * lo.c;
    r.d = hi.c * lo.b + hi.d * lo.d;
    r.e0 = hi.a * lo.e0 + hi.b * lo.e1 + hi.e0;
    r.e1 = hi.c * lo.e0 + hi.d * lo.e1 + hi.e1;
    return r;
}

// compose with each sum of products rounded as written (explicit fma), so
// that the result does not depend on how the compiler contracts the code
// around it: code paths that must agree bit for bit use this form
__device__ __forceinline__ Aff compose_x(const Aff &hi, const Aff &lo) {
    Aff r;
    r.a = fma(hi.a, lo.a, hi.b * lo.c);
    r.b = fma(hi.a, lo.b, hi.b * lo.d);
    r.c = fma(hi.c, lo.a, hi.d * lo.c);
    r.d = fma(hi.c, lo.b, hi.d * lo.d);
    r.e0 = fma(hi.a, lo.e0, fma(hi.b, lo.e1, hi.e0));
    r.e1 = fma(hi.c, lo.e0, fma(hi.d, lo.e1, hi.e1));
    return r;
}

template <bool UP> __device__ __forceinline__ double shfl_step(double v, int d) {
    return UP ? __shfl_up(v, d, 64) : __shfl_down(v, d, 64);
}

template <bool UP> __device__ __forceinline__ Aff shfl_aff(const Aff &x, int d) {
    Aff r;
    r.a = shfl_step<UP>(x.a, d);
    r.b = shfl_step<UP>(x.b, d);
    r.c = shfl_step<UP>(x.c, d);
    r.d = shfl_step<UP>(x.d, d);
    r.e0 = shfl_step<UP>(x.e0, d);
    r.e1 = shfl_step<UP>(x.e1, d);
    return r;
}

__device__ __forceinline__ Aff bcast_aff(const Aff &x, int lane) {
    Aff r;
    r.a = __shfl(x.a, lane, 64);
    r.b = __shfl(x.b, lane, 64);
    r.c = __shfl(x.c, lane, 64);
    r.d = __shfl(x.d, lane, 64);
    r.e0 = __shfl(x.e0, lane, 64);
    r.e1 = __shfl(x.e1, lane, 64);
    return r;
}

// M^len for the companion matrix M = [[p1, p2], [1, 0]].
__device__ __forceinline__ void companion_pow(double p1, double p2, int len, Aff &m) {
    double ra = 1, rb = 0, rc = 0, rd = 1;
    double ba = p1, bb = p2, bc = 1, bd = 0;
    while (len) {
        if (len & 1) {
            const double na = ra * ba + rb * bc, nb = ra * bb + rb * bd;
            const double nc = rc * ba + rd * bc, nd = rc * bb + rd * bd;
            ra = na; rb = nb; rc = nc; rd = nd;
        }
        const double na = ba * ba + bb * bc, nb = ba * bb + bb * bd;
        const double nc = bc * ba + bd * bc, nd = bc * bb + bd * bd;
        ba = na; bb = nb; bc = nc; bd = nd;
        len >>= 1;
    }
    m.a = ra; m.b = rb; m.c = rc; m.d = rd;
}

__device__ __forceinline__ Aff aff_identity() {
    Aff r;
    r.a = 1.0; r.b = 0.0; r.c = 0.0; r.d = 1.0; r.e0 = 0.0; r.e1 = 0.0;
    return r;
}

// ---- columns -------------------------------------------------------------------

__device__ __forceinline__ int find_inst(const int *map, int blk) { return map ? map[blk] : 0; }

// Forward recurrence from zero over one segment, then the backward one from
// zero over its output; returns both end states.  FULL: the segment has
// kSeg rows, so the body has no branch and every load can be in flight at
// once.
template <typename TR, int BW, bool FULL>
__device__ __forceinline__ void seg_a(gptr<const TR> rhs, long long ld, int len, double p1, double p2,
                                      double &s0, double &s1, double &t0, double &t1) {
    const int n = FULL ? kSeg : len;
    TR raw[kSeg];
#pragma unroll
    for (int j = 0; j < kSeg; ++j)
        if (j < n) raw[j] = gld<TR>(rhs, static_cast<long long>(j) * ld);
    double y[kSeg];
    s0 = s1 = 0.0;
#pragma unroll
    for (int j = 0; j < kSeg; ++j) {
        if (j < n) {
            const double b = to_f64<TR>(raw[j]);
            const double v = BW == 2 ? fma(p2, s1, fma(p1, s0, b)) : fma(p1, s0, b);
            y[j] = v;
            s1 = s0;
            s0 = v;
        }
    }
    t0 = t1 = 0.0;
#pragma unroll
    for (int j = kSeg - 1; j >= 0; --j) {
        if (j < n) {
            const double v = BW == 2 ? fma(p2, t1, fma(p1, t0, y[j])) : fma(p1, t0, y[j]);
            t1 = t0;
            t0 = v;
        }
    }
}

template <typename TR, int BW>
__device__ __forceinline__ void cols_a_block(const ColsInst *__restrict__ inst, const int *__restrict__ map,
                                             const int blk) {
    const int g = find_inst(map, blk);
    const ColsInst &I = inst[g];
    const int local = blk - I.blk0;
    const int seg = local / I.nstrips;
    const int strip = local - seg * I.nstrips;
    const int i = strip * kColsThreads + threadIdx.x;
    if (i >= I.nx) return;
    const int r0 = seg * kSeg;
    const int len = min(kSeg, I.ny - r0);
    const gptr<const TR> rhs = as_global(static_cast<const TR *>(I.rhs)) + static_cast<long long>(r0) * I.ld + i;
    double s0, s1, t0, t1;
    if (len == kSeg)
        seg_a<TR, BW, true>(rhs, I.ld, len, I.p1, I.p2, s0, s1, t0, t1);
    else
        seg_a<TR, BW, false>(rhs, I.ld, len, I.p1, I.p2, s0, s1, t0, t1);
    const gptr<double> cy = as_global(I.carry) + static_cast<long long>(seg) * 4 * I.nx + i;
    cy[0] = s0;
    cy[I.nx] = s1;
    cy[2 * I.nx] = t0;
    cy[3 * I.nx] = t1;
}

// Phase B: the segments of a column are split into G groups, one thread
// each (a workgroup covers kColsThreads / G columns).  Each thread composes the
// affine maps of its segments, the groups of a column combine their maps
// through LDS (wrap-around closure included), and each thread then writes
// the true incoming states of its own segments.  Summaries are loaded PB
// segments at a time so that their loads are in flight together; when a
// thread has at most PB segments, all four words of each are loaded once and
// kept in registers through both recurrences (one round of loads instead of
// four, the same arithmetic in the same order).  REG = false keeps the
// batched loads only (for kernels that have no registers to spare).
constexpr int PB = 8;

__device__ __forceinline__ void mat2_load(const double *m, Aff &x) {
    x.a = m[0]; x.b = m[1]; x.c = m[2]; x.d = m[3];
}

template <int BW, int G, bool REG = true>
__device__ __forceinline__ void cols_b_block(const ColsInst *__restrict__ inst, const int *__restrict__ map,
                                             const int blk, Aff *xa) {
    constexpr int kBCols = kColsThreads / G;
    const int g = find_inst(map, blk);
    const ColsInst &I = inst[g];
    const int cl = threadIdx.x % kBCols, q = threadIdx.x / kBCols;
    const int col = (blk - I.blkB0) * kBCols + cl;
    const bool valid = col < I.nx;
    const long long nx = I.nx;
    const gptr<double> cy = as_global(I.carry) + (valid ? col : 0);
    const int ns = I.nseg;
    const int sp = (ns + G - 1) / G;
    const int sb = min(q * sp, ns), se = min(sb + sp, ns);
    Aff Tf, Tl, Qf, Ql;
    mat2_load(I.Tf, Tf);
    mat2_load(I.Tl, Tl);
    mat2_load(I.Qf, Qf);
    mat2_load(I.Ql, Ql);

    if (REG && sp <= PB) {   // uniform
        const int n = se - sb;
        double e0[PB], e1[PB], g0[PB], g1[PB], cs0[PB], cs1[PB];
        if (valid) {
#pragma unroll
            for (int u = 0; u < PB; ++u)
                if (u < n) {
                    const long long o = static_cast<long long>(sb + u) * 4 * nx;
                    e0[u] = cy[o];
                    e1[u] = cy[o + nx];
                    g0[u] = cy[o + 2 * nx];
                    g1[u] = cy[o + 3 * nx];
                }
        }
        // forward: c_{s+1} = T_s c_s + e_s
        Aff m = aff_identity();
        if (valid) {
#pragma unroll
            for (int u = 0; u < PB; ++u)
                if (u < n) {
                    Aff x = sb + u == ns - 1 ? Tl : Tf;
                    x.e0 = e0[u];
                    x.e1 = e1[u];
                    m = compose_x(x, m);
                }
        }
        xa[q * kBCols + cl] = m;
        __syncthreads();
        Aff pre = aff_identity(), tot = aff_identity();
#pragma unroll
        for (int r = 0; r < G; ++r) {
            const Aff x = xa[r * kBCols + cl];
            if (r < q) pre = compose_x(x, pre);
            tot = compose_x(x, tot);
        }
        __syncthreads();
        double x0 = fma(I.Cinv[0], tot.e0, I.Cinv[1] * tot.e1);
        double x1 = fma(I.Cinv[2], tot.e0, I.Cinv[3] * tot.e1);
        double c0 = fma(pre.a, x0, fma(pre.b, x1, pre.e0));
        double c1 = fma(pre.c, x0, fma(pre.d, x1, pre.e1));
        if (valid) {
#pragma unroll
            for (int u = 0; u < PB; ++u)
                if (u < n) {
                    const long long o = static_cast<long long>(sb + u) * 4 * nx;
                    const Aff &T = sb + u == ns - 1 ? Tl : Tf;
                    cy[o] = c0;
                    cy[o + nx] = c1;
                    cs0[u] = c0;
                    cs1[u] = c1;
                    const double n0 = fma(T.a, c0, fma(T.b, c1, e0[u]));
                    const double n1 = fma(T.c, c0, fma(T.d, c1, e1[u]));
                    c0 = n0;
                    c1 = n1;
                }
        }
        // backward: d_{s-1} = T_s d_s + g_s + Q_s c_s
        m = aff_identity();
        if (valid) {
#pragma unroll
            for (int u = PB - 1; u >= 0; --u)
                if (u < n) {
                    const int s = sb + u;
                    const Aff &Q = s == ns - 1 ? Ql : Qf;
                    Aff x = s == ns - 1 ? Tl : Tf;
                    x.e0 = fma(Q.a, cs0[u], fma(Q.b, cs1[u], g0[u]));
                    x.e1 = fma(Q.c, cs0[u], fma(Q.d, cs1[u], g1[u]));
                    m = compose_x(x, m);
                }
        }
        xa[q * kBCols + cl] = m;
        __syncthreads();
        pre = aff_identity();
        tot = aff_identity();
#pragma unroll
        for (int r = G - 1; r >= 0; --r) {
            const Aff x = xa[r * kBCols + cl];
            if (r > q) pre = compose_x(x, pre);
            tot = compose_x(x, tot);
        }
        x0 = fma(I.Cinv[0], tot.e0, I.Cinv[1] * tot.e1);
        x1 = fma(I.Cinv[2], tot.e0, I.Cinv[3] * tot.e1);
        double d0 = fma(pre.a, x0, fma(pre.b, x1, pre.e0));
        double d1 = fma(pre.c, x0, fma(pre.d, x1, pre.e1));
        if (valid) {
#pragma unroll
            for (int u = PB - 1; u >= 0; --u)
                if (u < n) {
                    const int s = sb + u;
                    const long long o = static_cast<long long>(s) * 4 * nx;
                    const Aff &Q = s == ns - 1 ? Ql : Qf;
                    const Aff &T = s == ns - 1 ? Tl : Tf;
                    cy[o + 2 * nx] = d0;
                    cy[o + 3 * nx] = d1;
                    const double n0 = fma(T.a, d0, fma(T.b, d1, fma(Q.a, cs0[u], fma(Q.b, cs1[u], g0[u]))));
                    const double n1 = fma(T.c, d0, fma(T.d, d1, fma(Q.c, cs0[u], fma(Q.d, cs1[u], g1[u]))));
                    d0 = n0;
                    d1 = n1;
                }
        }
        return;
    }

    // ---- forward: c_{s+1} = T_s c_s + e_s --------------------------------------
    Aff m = aff_identity();
    if (valid) {
        for (int s0 = sb; s0 < se; s0 += PB) {
            double e0[PB], e1[PB];
#pragma unroll
            for (int u = 0; u < PB; ++u)
                if (s0 + u < se) {
                    e0[u] = cy[(s0 + u) * 4 * nx];
                    e1[u] = cy[(s0 + u) * 4 * nx + nx];
                }
#pragma unroll
            for (int u = 0; u < PB; ++u)
                if (s0 + u < se) {
                    Aff x = s0 + u == ns - 1 ? Tl : Tf;
                    x.e0 = e0[u];
                    x.e1 = e1[u];
                    m = compose_x(x, m);
                }
        }
    }
    xa[q * kBCols + cl] = m;
    __syncthreads();
    Aff pre = aff_identity(), tot = aff_identity();
#pragma unroll 4   // bounded: this path serves the persistent kernel, whose registers are full
    for (int r = 0; r < G; ++r) {
        const Aff x = xa[r * kBCols + cl];
        if (r < q) pre = compose_x(x, pre);
        tot = compose_x(x, tot);
    }
    __syncthreads();
    double x0 = fma(I.Cinv[0], tot.e0, I.Cinv[1] * tot.e1);
    double x1 = fma(I.Cinv[2], tot.e0, I.Cinv[3] * tot.e1);
    double c0 = fma(pre.a, x0, fma(pre.b, x1, pre.e0));
    double c1 = fma(pre.c, x0, fma(pre.d, x1, pre.e1));
    if (valid) {
        for (int s0 = sb; s0 < se; s0 += PB) {
            double e0[PB], e1[PB];
#pragma unroll
            for (int u = 0; u < PB; ++u)
                if (s0 + u < se) {
                    e0[u] = cy[(s0 + u) * 4 * nx];
                    e1[u] = cy[(s0 + u) * 4 * nx + nx];
                }
#pragma unroll
            for (int u = 0; u < PB; ++u)
                if (s0 + u < se) {
                    const Aff &T = s0 + u == ns - 1 ? Tl : Tf;
                    cy[(s0 + u) * 4 * nx] = c0;
                    cy[(s0 + u) * 4 * nx + nx] = c1;
                    const double n0 = fma(T.a, c0, fma(T.b, c1, e0[u]));
                    const double n1 = fma(T.c, c0, fma(T.d, c1, e1[u]));
                    c0 = n0;
                    c1 = n1;
                }
        }
    }

    // ---- backward: d_{s-1} = T_s d_s + g_s + Q_s c_s ---------------------------
    // (every thread reads back only the c_s it wrote itself)
    m = aff_identity();
    if (valid) {
        for (int s1 = se - 1; s1 >= sb; s1 -= PB) {
            double cs0[PB], cs1[PB], g0[PB], g1[PB];
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                const int s = s1 - u;
                if (s >= sb) {
                    cs0[u] = cy[s * 4 * nx];
                    cs1[u] = cy[s * 4 * nx + nx];
                    g0[u] = cy[s * 4 * nx + 2 * nx];
                    g1[u] = cy[s * 4 * nx + 3 * nx];
                }
            }
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                const int s = s1 - u;
                if (s >= sb) {
                    const Aff &Q = s == ns - 1 ? Ql : Qf;
                    Aff x = s == ns - 1 ? Tl : Tf;
                    x.e0 = fma(Q.a, cs0[u], fma(Q.b, cs1[u], g0[u]));
                    x.e1 = fma(Q.c, cs0[u], fma(Q.d, cs1[u], g1[u]));
                    m = compose_x(x, m);
                }
            }
        }
    }
    xa[q * kBCols + cl] = m;
    __syncthreads();
    pre = aff_identity();
    tot = aff_identity();
#pragma unroll 4   // bounded: this path serves the persistent kernel, whose registers are full
    for (int r = G - 1; r >= 0; --r) {
        const Aff x = xa[r * kBCols + cl];
        if (r > q) pre = compose_x(x, pre);
        tot = compose_x(x, tot);
    }
    x0 = fma(I.Cinv[0], tot.e0, I.Cinv[1] * tot.e1);
    x1 = fma(I.Cinv[2], tot.e0, I.Cinv[3] * tot.e1);
    double d0 = fma(pre.a, x0, fma(pre.b, x1, pre.e0));
    double d1 = fma(pre.c, x0, fma(pre.d, x1, pre.e1));
    if (valid) {
        for (int s1 = se - 1; s1 >= sb; s1 -= PB) {
            double cs0[PB], cs1[PB], g0[PB], g1[PB];
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                const int s = s1 - u;
                if (s >= sb) {
                    cs0[u] = cy[s * 4 * nx];
                    cs1[u] = cy[s * 4 * nx + nx];
                    g0[u] = cy[s * 4 * nx + 2 * nx];
                    g1[u] = cy[s * 4 * nx + 3 * nx];
                }
            }
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                const int s = s1 - u;
                if (s >= sb) {
                    const Aff &Q = s == ns - 1 ? Ql : Qf;
                    const Aff &T = s == ns - 1 ? Tl : Tf;
                    cy[s * 4 * nx + 2 * nx] = d0;
                    cy[s * 4 * nx + 3 * nx] = d1;
                    const double n0 = fma(T.a, d0, fma(T.b, d1, fma(Q.a, cs0[u], fma(Q.b, cs1[u], g0[u]))));
                    const double n1 = fma(T.c, d0, fma(T.d, d1, fma(Q.c, cs0[u], fma(Q.d, cs1[u], g1[u]))));
                    d0 = n0;
                    d1 = n1;
                }
            }
        }
    }
}

// Both recurrences over one segment from its true incoming states, then the
// output (EPI 1: the Cahn-Hilliard update x = 2 cur - prev + v / K).  FULL as
// in seg_a.
template <typename TR, typename TX, int BW, int EPI, bool FULL>
__device__ __forceinline__ void seg_c(gptr<const TR> rhs, gptr<TX> x, gptr<const TX> cur, gptr<const TX> prev,
                                      long long ld, int len, double p1, double p2, double invK,
                                      double s0, double s1, double t0, double t1) {
    const int n = FULL ? kSeg : len;
    TR raw[kSeg];
#pragma unroll
    for (int j = 0; j < kSeg; ++j)
        if (j < n) raw[j] = gld<TR>(rhs, static_cast<long long>(j) * ld);
    double y[kSeg];
#pragma unroll
    for (int j = 0; j < kSeg; ++j) {
        if (j < n) {
            const double b = to_f64<TR>(raw[j]);
            const double v = BW == 2 ? fma(p2, s1, fma(p1, s0, b)) : fma(p1, s0, b);
            y[j] = v;
            s1 = s0;
            s0 = v;
        }
    }
    // backward pass in groups of G rows; the group's cur/prev values are
    // requested together before any of its outputs is stored
    constexpr int G = 8;
    static_assert(kSeg % G == 0, "segment must be a whole number of groups");
#pragma unroll
    for (int jg = kSeg - G; jg >= 0; jg -= G) {
        double cb[G];
        if (EPI == 1) {
#pragma unroll
            for (int q = 0; q < G; ++q) {
                const long long o = static_cast<long long>(jg + q) * ld;
                if (jg + q < n) cb[q] = 2.0 * to_f64<TX>(gld<TX>(cur, o)) - to_f64<TX>(gld<TX>(prev, o));
            }
        }
#pragma unroll
        for (int q = G - 1; q >= 0; --q) {
            const int j = jg + q;
            if (j < n) {
                const double v = BW == 2 ? fma(p2, t1, fma(p1, t0, y[j])) : fma(p1, t0, y[j]);
                t1 = t0;
                t0 = v;
                const long long o = static_cast<long long>(j) * ld;
                gst<TX>(x, o, from_f64<TX>(EPI == 1 ? cb[q] + v * invK : v * invK));
            }
        }
    }
}

template <typename TR, typename TX, int BW, int EPI>
__device__ __forceinline__ void cols_c_block(const ColsInst *__restrict__ inst, const int *__restrict__ map,
                                             const int blk) {
    const int g = find_inst(map, blk);
    const ColsInst &I = inst[g];
    const int local = blk - I.blk0;
    const int seg = local / I.nstrips;
    const int strip = local - seg * I.nstrips;
    const int i = strip * kColsThreads + threadIdx.x;
    if (i >= I.nx) return;
    const int r0 = seg * kSeg;
    const int len = min(kSeg, I.ny - r0);
    const long long off = static_cast<long long>(r0) * I.ld + i;
    const gptr<const TR> rhs = as_global(static_cast<const TR *>(I.rhs)) + off;
    const gptr<const double> cy = as_global(static_cast<const double *>(I.carry)) + static_cast<long long>(seg) * 4 * I.nx + i;
    const double s0 = cy[0], s1 = cy[I.nx];
    const double t0 = cy[2 * I.nx], t1 = cy[3 * I.nx];
    const gptr<TX> x = as_global(static_cast<TX *>(I.x)) + off;
    const gptr<const TX> cur = as_global(static_cast<const TX *>(I.cur)) + off;
    const gptr<const TX> prev = as_global(static_cast<const TX *>(I.prev)) + off;
    if (len == kSeg)
        seg_c<TR, TX, BW, EPI, true>(rhs, x, cur, prev, I.ld, len, I.p1, I.p2, I.invK, s0, s1, t0, t1);
    else
        seg_c<TR, TX, BW, EPI, false>(rhs, x, cur, prev, I.ld, len, I.p1, I.p2, I.invK, s0, s1, t0, t1);
}

}  // namespace
}  // namespace mxs
