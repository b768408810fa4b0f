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
__global__ void __launch_bounds__(kColsThreads) cols_phase_a(const ColsInst *__restrict__ inst,
                                                            const int *__restrict__ map) {
    const int g = find_inst(map, blockIdx.x);
    const ColsInst &I = inst[g];
    const int local = blockIdx.x - I.blk0;
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

// Phase B: the segments of a column are split into kBGroups groups, one
// thread each (a workgroup covers kBCols columns).  Each thread composes the
// affine maps of its segments, the groups of a column combine their maps
// through LDS (wrap-around closure included), and each thread then writes
// the true incoming states of its own segments.  Summaries are loaded PB
// segments at a time so that their loads are in flight together.
constexpr int PB = 8;

__device__ __forceinline__ void mat2_load(const double *m, Aff &x) {
    x.a = m[0]; x.b = m[1]; x.c = m[2]; x.d = m[3];
}

template <int BW>
__global__ void __launch_bounds__(kColsThreads) cols_phase_b(const ColsInst *__restrict__ inst,
                                                            const int *__restrict__ map) {
    __shared__ Aff xa[kBGroups][kBCols];
    const int g = find_inst(map, blockIdx.x);
    const ColsInst &I = inst[g];
    const int cl = threadIdx.x % kBCols, q = threadIdx.x / kBCols;
    const int col = (blockIdx.x - I.blkB0) * kBCols + cl;
    const bool valid = col < I.nx;
    const long long nx = I.nx;
    const gptr<double> cy = as_global(I.carry) + (valid ? col : 0);
    const int ns = I.nseg;
    const int sp = (ns + kBGroups - 1) / kBGroups;
    const int sb = min(q * sp, ns), se = min(sb + sp, ns);
    Aff Tf, Tl, Qf, Ql;
    mat2_load(I.Tf, Tf);
    mat2_load(I.Tl, Tl);
    mat2_load(I.Qf, Qf);
    mat2_load(I.Ql, Ql);

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
                    m = compose(x, m);
                }
        }
    }
    xa[q][cl] = m;
    __syncthreads();
    Aff pre = aff_identity(), tot = aff_identity();
#pragma unroll
    for (int r = 0; r < kBGroups; ++r) {
        const Aff x = xa[r][cl];
        if (r < q) pre = compose(x, pre);
        tot = compose(x, tot);
    }
    __syncthreads();
    double x0 = I.Cinv[0] * tot.e0 + I.Cinv[1] * tot.e1;
    double x1 = I.Cinv[2] * tot.e0 + I.Cinv[3] * tot.e1;
    double c0 = pre.a * x0 + pre.b * x1 + pre.e0;
    double c1 = pre.c * x0 + pre.d * x1 + pre.e1;
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
                    const double n0 = T.a * c0 + T.b * c1 + e0[u];
                    const double n1 = T.c * c0 + T.d * c1 + e1[u];
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
                    x.e0 = g0[u] + Q.a * cs0[u] + Q.b * cs1[u];
                    x.e1 = g1[u] + Q.c * cs0[u] + Q.d * cs1[u];
                    m = compose(x, m);
                }
            }
        }
    }
    xa[q][cl] = m;
    __syncthreads();
    pre = aff_identity();
    tot = aff_identity();
#pragma unroll
    for (int r = kBGroups - 1; r >= 0; --r) {
        const Aff x = xa[r][cl];
        if (r > q) pre = compose(x, pre);
        tot = compose(x, tot);
    }
    x0 = I.Cinv[0] * tot.e0 + I.Cinv[1] * tot.e1;
    x1 = I.Cinv[2] * tot.e0 + I.Cinv[3] * tot.e1;
    double d0 = pre.a * x0 + pre.b * x1 + pre.e0;
    double d1 = pre.c * x0 + pre.d * x1 + pre.e1;
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
                    const double n0 = g0[u] + Q.a * cs0[u] + Q.b * cs1[u] + T.a * d0 + T.b * d1;
                    const double n1 = g1[u] + Q.c * cs0[u] + Q.d * cs1[u] + T.c * d0 + T.d * d1;
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
__global__ void __launch_bounds__(kColsThreads) cols_phase_c(const ColsInst *__restrict__ inst,
                                                            const int *__restrict__ map) {
    const int g = find_inst(map, blockIdx.x);
    const ColsInst &I = inst[g];
    const int local = blockIdx.x - I.blk0;
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
                    int blocksB, hipStream_t s) {
    hipLaunchKernelGGL((cols_phase_a<TR, BW>), dim3(blocksAC), dim3(kColsThreads), 0, s, inst, mapAC);
    hipLaunchKernelGGL((cols_phase_b<BW>), dim3(blocksB), dim3(kColsThreads), 0, s, inst, mapB);
    hipLaunchKernelGGL((cols_phase_c<TR, TX, BW, EPI>), dim3(blocksAC), dim3(kColsThreads), 0, s,
                       inst, mapAC);
    return hipGetLastError();
}

template <typename TR, typename TX, int EPI>
hipError_t cols_bw(int bw, const ColsInst *inst, const int *mapAC, const int *mapB, int blocksAC,
                   int blocksB, hipStream_t s) {
    return bw == 1 ? cols_one<TR, TX, 1, EPI>(inst, mapAC, mapB, blocksAC, blocksB, s)
                   : cols_one<TR, TX, 2, EPI>(inst, mapAC, mapB, blocksAC, blocksB, s);
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
                       const int *mapAC, const int *mapB, int blocksAC, int blocksB, hipStream_t s) {
    if (bw != 1 && bw != 2) return hipErrorInvalidValue;
    if (epilogue == 0) {
        if (rhs_dtype == F64 && x_dtype == F64) return cols_bw<double, double, 0>(bw, inst, mapAC, mapB, blocksAC, blocksB, s);
        if (rhs_dtype == F32 && x_dtype == F32) return cols_bw<float, float, 0>(bw, inst, mapAC, mapB, blocksAC, blocksB, s);
        if (rhs_dtype == BF16 && x_dtype == BF16) return cols_bw<bf16, bf16, 0>(bw, inst, mapAC, mapB, blocksAC, blocksB, s);
    } else if (bw == 2) {
        if (rhs_dtype == F64 && x_dtype == F64) return cols_one<double, double, 2, 1>(inst, mapAC, mapB, blocksAC, blocksB, s);
        if (rhs_dtype == F32 && x_dtype == F32) return cols_one<float, float, 2, 1>(inst, mapAC, mapB, blocksAC, blocksB, s);
        if (rhs_dtype == F32 && x_dtype == BF16) return cols_one<float, bf16, 2, 1>(inst, mapAC, mapB, blocksAC, blocksB, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace mxs
