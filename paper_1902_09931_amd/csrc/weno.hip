// WENO advection, the periodic xy variant of Sec. 4.3: the weighted sum of
// the periodic XY stencil is replaced by a WENO evaluation of the advection
// term, with the velocities u and v as extra inputs:
//
//   out = u phi_x + v phi_y,
//
// each derivative the fifth-order Hamilton-Jacobi WENO approximation
// (Jiang and Peng; the level-set text the section cites, Sec. 3.4 there),
// upwinded by the sign of its velocity: from the backward differences at
// i-2 .. i+2 where the velocity is positive, from the forward differences at
// i+2 .. i-2 otherwise.
//
// Layout as the block form of the 2D stencils: a workgroup owns a strip of
// W = threads * 2 columns and a chunk of ROWS output rows; it requests the
// ROWS + 6 rows of phi its chunk needs (three above, three below, periodic)
// and the ROWS rows of u and v at once.  The y derivative reads the thread's
// own column from registers; the x derivative reads the output rows, staged
// in LDS with three halo columns on each side.  Algorithmic traffic: read
// phi, u, v and write out, 4 words per point.
#include "weno.h"

namespace mxs {

namespace {

constexpr int kWenoPad = 4;   // halo columns staged on each side (3 used), a whole vector

// The WENO combination of five consecutive one-sided differences v1..v5,
// ordered away from the upwind side (v3 the difference at the point): the
// three third-order ENO candidates, their smoothness indicators s_k, and the
// nonlinear weights w_k = a_k / sum a, a_k = g_k / (s_k + eps)^2 with the
// optimal weights g = 1/10, 6/10, 3/10 and eps = 1e-6 times the largest
// squared difference plus 1e-99.
//
// Arithmetic: the candidates by multiplications with rounded constants
// instead of divisions, and the weights with one quotient instead of four:
// w_k = g_k prod_{m != k} d_m^2 / sum_l g_l prod_{m != l} d_m^2, d = s + eps,
// the same ratio.  The d_m are first scaled by the same power of two
// (exactly), so that the largest lies in [1/2, 1): since s_m <= 34 max v^2
// and eps >= 1e-6 max v^2 (or all d_m = eps when every v is zero), every
// scaled d_m is at least 1.4e-8 and no product underflows.
__device__ __forceinline__ double weno5(double v1, double v2, double v3, double v4, double v5) {
    constexpr double third = 1.0 / 3.0, sixth = 1.0 / 6.0;
    const double p1 = fma(v1, third, fma(v2, -7.0 * sixth, v3 * (11.0 * sixth)));
    const double p2 = fma(v2, -sixth, fma(v3, 5.0 * sixth, v4 * third));
    const double p3 = fma(v3, third, fma(v4, 5.0 * sixth, v5 * -sixth));
    double a = v1 - 2.0 * v2 + v3, b = v1 - 4.0 * v2 + 3.0 * v3;
    const double s1 = fma(13.0 / 12.0, a * a, 0.25 * (b * b));
    a = v2 - 2.0 * v3 + v4;
    b = v2 - v4;
    const double s2 = fma(13.0 / 12.0, a * a, 0.25 * (b * b));
    a = v3 - 2.0 * v4 + v5;
    b = 3.0 * v3 - 4.0 * v4 + v5;
    const double s3 = fma(13.0 / 12.0, a * a, 0.25 * (b * b));
    // the largest square is the square of the largest magnitude (rounding
    // of a square is monotone in |v|), one multiplication instead of five
    const double va = fmax(fmax(fmax(fabs(v1), fabs(v2)), fmax(fabs(v3), fabs(v4))), fabs(v5));
    const double eps = fma(1e-6, va * va, 1e-99);
    double d1 = s1 + eps, d2 = s2 + eps, d3 = s3 + eps;
    const int ex = __builtin_amdgcn_frexp_exp(fmax(fmax(d1, d2), d3));
    d1 = __builtin_amdgcn_ldexp(d1, -ex);
    d2 = __builtin_amdgcn_ldexp(d2, -ex);
    d3 = __builtin_amdgcn_ldexp(d3, -ex);
    const double q1 = d1 * d1, q2 = d2 * d2, q3 = d3 * d3;
    const double n1 = 0.1 * (q2 * q3), n2 = 0.6 * (q1 * q3), n3 = 0.3 * (q1 * q2);
    // num / den with the hardware reciprocal refined by two Newton steps and
    // a final residual correction (den is a normal number in [4e-33, 1]
    // after the scaling, so none of the special cases of a general division
    // arise); within one rounding of the quotient
    const double num = fma(n1, p1, fma(n2, p2, n3 * p3)), den = n1 + n2 + n3;
    double r = __builtin_amdgcn_rcp(den);
    r = fma(fma(-den, r, 1.0), r, r);
    r = fma(fma(-den, r, 1.0), r, r);
    const double q = num * r;
    return fma(fma(-den, q, num), r, q);
}

// The upwind WENO derivative from seven consecutive values f[0..6] centred on
// the point (f[3]), spacing 1/rh.
__device__ __forceinline__ double weno_deriv(const double (&f)[7], bool left, double rh) {
    double d[5];
#pragma unroll
    for (int q = 0; q < 5; ++q)
        d[q] = left ? (f[1 + q] - f[q]) * rh : (f[6 - q] - f[5 - q]) * rh;
    return weno5(d[0], d[1], d[2], d[3], d[4]);
}

template <int ROWS>
__global__ void __launch_bounds__(256) weno_adv_kernel(const WenoArgs a) {
    constexpr int V = 2;
    constexpr int GIN = ROWS + 6;
    constexpr int PAD = kWenoPad;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *lds = reinterpret_cast<double *>(smem_raw);
    const gptr<const double> phi = as_global(static_cast<const double *>(a.phi));
    const gptr<const double> uu = as_global(static_cast<const double *>(a.u));
    const gptr<const double> vv = as_global(static_cast<const double *>(a.v));
    const gptr<double> out = as_global(static_cast<double *>(a.out));
    const int nt = blockDim.x, t = threadIdx.x;
    const int W = nt * V;
    const int rowlen = PAD + W + PAD;
    int strip, chunk;
    if (a.order == 0) {
        const int tile = xcd_tile(blockIdx.x, gridDim.x);
        strip = tile / a.nchunks;
        chunk = tile - strip * a.nchunks;
    } else {
        chunk = blockIdx.x / a.nstrips;
        strip = blockIdx.x - chunk * a.nstrips;
    }
    const long long i0 = static_cast<long long>(strip) * W;
    const int j0 = chunk * ROWS;
    const int H = min(ROWS, a.ny - j0);
    const long long ib = i0 + static_cast<long long>(t) * V;
    const bool clean = a.vec_ok && i0 + W <= a.nx;   // uniform per workgroup

    // every request of the workgroup before any value is used
    auto col = [&](long long c) __attribute__((always_inline)) { return wrap_fast(c, a.nx); };
    double f[GIN][V], u[ROWS][V], v[ROWS][V];
#pragma unroll
    for (int r = 0; r < GIN; ++r) {
        const long long row = wrap_fast(static_cast<long long>(j0) - 3 + r, a.ny);
        const gptr<const double> p = phi + row * a.ld;
        if (clean) {
            load_vec<double>(p + ib, f[r]);
        } else {
#pragma unroll
            for (int q = 0; q < V; ++q) f[r][q] = p[col(ib + q)];
        }
    }
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        const long long row = min(j0 + k, a.ny - 1);
        if (clean) {
            load_vec<double>(uu + row * a.ld + ib, u[k]);
            load_vec<double>(vv + row * a.ld + ib, v[k]);
        } else {
#pragma unroll
            for (int q = 0; q < V; ++q) {
                u[k][q] = uu[row * a.ld + col(ib + q)];
                v[k][q] = vv[row * a.ld + col(ib + q)];
            }
        }
    }
    // x halo of the output rows: ROWS x 2 x 3 values
    constexpr int HN = ROWS * 6;
    constexpr int HPT = (HN + 63) / 64;
    double hv[HPT];
#pragma unroll
    for (int q = 0; q < HPT; ++q) {
        const int h = min(t + q * nt, HN - 1);
        const int k = h / 6, s = h - k * 6;
        const long long c = s < 3 ? i0 - 3 + s : i0 + W + (s - 3);
        const long long row = min(j0 + k, a.ny - 1);
        hv[q] = phi[row * a.ld + col(c)];
    }

    // stage the output rows with their halo
#pragma unroll
    for (int k = 0; k < ROWS; ++k)
#pragma unroll
        for (int q = 0; q < V; ++q) lds[k * rowlen + PAD + t * V + q] = f[k + 3][q];
#pragma unroll
    for (int q = 0; q < HPT; ++q) {
        const int h = t + q * nt;
        if (h < HN) {
            const int k = h / 6, s = h - k * 6;
            lds[k * rowlen + (s < 3 ? PAD - 3 + s : PAD + W + (s - 3))] = hv[q];
        }
    }
    __syncthreads();

    const double rdx = a.rdx, rdy = a.rdy;
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        if (k >= H) continue;
        double x[V + 6];
        const double *lp = lds + k * rowlen + PAD + t * V - 3;
#pragma unroll
        for (int m = 0; m < V + 6; ++m) x[m] = lp[m];
        double res[V];
#pragma unroll
        for (int q = 0; q < V; ++q) {
            double fx[7], fy[7];
#pragma unroll
            for (int m = 0; m < 7; ++m) {
                fx[m] = x[q + m];
                fy[m] = f[k + m][q];
            }
            const double px = weno_deriv(fx, u[k][q] > 0.0, rdx);
            const double py = weno_deriv(fy, v[k][q] > 0.0, rdy);
            res[q] = u[k][q] * px + v[k][q] * py;
        }
        const gptr<double> rowp = out + static_cast<long long>(j0 + k) * a.ld;
        if (clean) {
            if (a.nt_store) store_vec_nt<double>(rowp + ib, res);
            else store_vec<double>(rowp + ib, res);
        } else {
#pragma unroll
            for (int q = 0; q < V; ++q)
                if (ib + q < a.nx) rowp[ib + q] = res[q];
        }
    }
}

}  // namespace

size_t weno_lds_bytes(int rows, int threads) {
    return static_cast<size_t>(rows) * (2 * kWenoPad + 2 * threads) * sizeof(double);
}

bool weno_rows_ok(int rows) { return rows == 4 || rows == 8; }

hipError_t launch_weno_adv(const WenoArgs &a, int threads, hipStream_t s) {
    const int grid = a.nstrips * a.nchunks;
    const size_t lds = weno_lds_bytes(a.rows, threads);
    if (a.rows == 4)
        hipLaunchKernelGGL(weno_adv_kernel<4>, dim3(grid), dim3(threads), lds, s, a);
    else if (a.rows == 8)
        hipLaunchKernelGGL(weno_adv_kernel<8>, dim3(grid), dim3(threads), lds, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace mxs
