// Host-side factorisation of symmetric circulants and the per-segment
// matrices of the column solve.
#include "solve.h"

#include <cmath>
#include <complex>

namespace mxs {

namespace {

using ld = long double;
using cld = std::complex<long double>;

// Root of z^2 - q z + 1 = 0 inside the unit circle.
cld inner_root(cld q) {
    cld s = std::sqrt(q * q - cld(4));
    cld z1 = (q + s) / cld(2), z2 = (q - s) / cld(2);
    // z1 z2 = 1: take the smaller one, computed without cancellation
    return std::abs(z1) < std::abs(z2) ? cld(1) / z2 : cld(1) / z1;
}

// Residuals of K P(z) P(1/z) = c0 + c1 (z + 1/z) + c2 (z^2 + 1/z^2) with
// P(z) = 1 - p1 z - p2 z^2:
//   c0 = K (1 + p1^2 + p2^2),  c1 = K p1 (p2 - 1),  c2 = -K p2.
void newton_refine(int bw, const double *c, ld &K, ld &p1, ld &p2) {
    for (int it = 0; it < 8; ++it) {
        if (bw == 1) {
            const ld F0 = K * (1 + p1 * p1) - c[0];
            const ld F1 = -K * p1 - c[1];
            const ld J00 = 1 + p1 * p1, J01 = 2 * K * p1;
            const ld J10 = -p1, J11 = -K;
            const ld det = J00 * J11 - J01 * J10;
            if (det == 0) return;
            K -= (F0 * J11 - F1 * J01) / det;
            p1 -= (-F0 * J10 + F1 * J00) / det;
        } else {
            const ld F[3] = {K * (1 + p1 * p1 + p2 * p2) - c[0], K * p1 * (p2 - 1) - c[1],
                             -K * p2 - c[2]};
            ld J[3][3] = {{1 + p1 * p1 + p2 * p2, 2 * K * p1, 2 * K * p2},
                          {p1 * (p2 - 1), K * (p2 - 1), K * p1},
                          {-p2, 0, -K}};
            // solve J d = F by Cramer's rule
            auto det3 = [](ld m[3][3]) {
                return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
                       m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
                       m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
            };
            const ld D = det3(J);
            if (D == 0) return;
            ld d[3];
            for (int col = 0; col < 3; ++col) {
                ld Mx[3][3];
                for (int r = 0; r < 3; ++r)
                    for (int q = 0; q < 3; ++q) Mx[r][q] = q == col ? F[r] : J[r][q];
                d[col] = det3(Mx) / D;
            }
            K -= d[0];
            p1 -= d[1];
            p2 -= d[2];
        }
    }
}

}  // namespace

int factor_symmetric_circulant(int bw, const double *c, CyclicFactor *f) {
    if (!c || !f || (bw != 1 && bw != 2)) return -1;
    for (int d = 0; d <= bw; ++d)
        if (!std::isfinite(c[d])) return -1;
    const ld c0 = c[0], c1 = c[1], c2 = bw == 2 ? c[2] : 0;
    // positivity of the symbol g(t) = c0 + 2 c1 cos t + 2 c2 cos 2t; with
    // u = cos t: g = (c0 - 2 c2) + 2 c1 u + 4 c2 u^2 on [-1, 1].
    ld gmin = std::min(c0 + 2 * c1 + 2 * c2, c0 - 2 * c1 + 2 * c2);
    if (c2 > 0) {
        const ld u = -c1 / (4 * c2);
        if (u > -1 && u < 1) gmin = std::min(gmin, c0 - 2 * c2 - c1 * c1 / (4 * c2));
    }
    const ld scale = std::fabs(c0) + 2 * std::fabs(c1) + 2 * std::fabs(c2);
    if (!(gmin > 1e-13L * scale)) return -2;

    ld K, p1 = 0, p2 = 0;
    if (c2 == 0 && c1 == 0) {
        K = c0;
    } else if (c2 == 0) {
        // c1 z^2 + c0 z + c1 = 0, inner root r; P(z) = 1 - r z, K = -c1 / r
        const ld r = -2 * c1 / (c0 + std::sqrt(c0 * c0 - 4 * c1 * c1));
        p1 = r;
        K = -c1 / r;
        newton_refine(1, c, K, p1, p2);
    } else {
        // q = z + 1/z solves c2 q^2 + c1 q + (c0 - 2 c2) = 0
        const cld disc = std::sqrt(cld(c1 * c1 - 4 * c2 * (c0 - 2 * c2)));
        const cld q1 = (cld(-c1) + disc) / cld(2 * c2);
        const cld q2 = (cld(-c1) - disc) / cld(2 * c2);
        const cld r1 = inner_root(q1), r2 = inner_root(q2);
        p1 = std::real(r1 + r2);
        p2 = -std::real(r1 * r2);
        K = c2 / std::real(r1 * r2);
        newton_refine(2, c, K, p1, p2);
    }
    f->p1 = static_cast<double>(p1);
    f->p2 = static_cast<double>(p2);
    f->K = static_cast<double>(K);
    f->invK = static_cast<double>(1 / K);
    return 0;
}

namespace {

// 2x2 row-major helpers in long double
struct M2 {
    ld a, b, c, d;
};
M2 mul(const M2 &x, const M2 &y) {
    return {x.a * y.a + x.b * y.c, x.a * y.b + x.b * y.d, x.c * y.a + x.d * y.c,
            x.c * y.b + x.d * y.d};
}
M2 mpow(const M2 &m, long long e) {
    M2 r{1, 0, 0, 1}, base = m;
    while (e) {
        if (e & 1) r = mul(r, base);
        base = mul(base, base);
        e >>= 1;
    }
    return r;
}
void store(const M2 &m, double *o) {
    o[0] = static_cast<double>(m.a);
    o[1] = static_cast<double>(m.b);
    o[2] = static_cast<double>(m.c);
    o[3] = static_cast<double>(m.d);
}

// Column q of Q: forward homogeneous recurrence from state e_q over len
// steps, then the backward recurrence from zero over those values; the
// resulting top state (u_0, u_1) is the column.
M2 q_matrix(ld p1, ld p2, int len) {
    M2 Q{};
    ld y[64];
    for (int q = 0; q < 2; ++q) {
        ld s0 = q == 0 ? 1 : 0, s1 = q == 1 ? 1 : 0;
        for (int j = 0; j < len; ++j) {
            const ld v = p1 * s0 + p2 * s1;
            y[j] = v;
            s1 = s0;
            s0 = v;
        }
        ld t0 = 0, t1 = 0;
        for (int j = len - 1; j >= 0; --j) {
            const ld v = y[j] + p1 * t0 + p2 * t1;
            t1 = t0;
            t0 = v;
        }
        if (q == 0) {
            Q.a = t0;
            Q.c = t1;
        } else {
            Q.b = t0;
            Q.d = t1;
        }
    }
    return Q;
}

}  // namespace

void fill_cols_coef(const CyclicFactor &f, int bw, int ny, ColsInst *ci) {
    const ld p1 = f.p1, p2 = bw == 2 ? f.p2 : 0;
    const M2 M{p1, p2, 1, 0};
    const int nseg = (ny + kSeg - 1) / kSeg;
    const int last = ny - (nseg - 1) * kSeg;
    ci->nseg = nseg;
    ci->p1 = f.p1;
    ci->p2 = bw == 2 ? f.p2 : 0.0;
    ci->invK = f.invK;
    store(mpow(M, kSeg), ci->Tf);
    store(mpow(M, last), ci->Tl);
    store(q_matrix(p1, p2, kSeg), ci->Qf);
    store(q_matrix(p1, p2, last), ci->Ql);
    const M2 Mn = mpow(M, ny);
    const ld a = 1 - Mn.a, b = -Mn.b, c = -Mn.c, d = 1 - Mn.d;
    const ld det = a * d - b * c;
    store(M2{d / det, -b / det, -c / det, a / det}, ci->Cinv);
}

}  // namespace mxs

namespace mxs {

void fill_pow_table(const CyclicFactor &f, int bw, double *out) {
    const ld p1 = f.p1, p2 = bw == 2 ? f.p2 : 0;
    const M2 M{p1, p2, 1, 0};
    M2 r{1, 0, 0, 1};
    for (int k = 0; k <= kWaveBlock; ++k) {
        store(r, out + 4 * k);
        r = mul(r, M);
    }
    const M2 Mb = mpow(M, kWaveBlock);
    r = M2{1, 0, 0, 1};
    for (int c = 0; c <= kWaveNBMax; ++c) {
        store(r, out + 4 * (kWaveBlock + 1 + c));
        r = mul(r, Mb);
    }
}

}  // namespace mxs
