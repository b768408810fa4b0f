// Device-side pieces shared by the line-solve kernels: storage conversions
// and the description of one line (input, output, length, coefficients).
#pragma once

#include "solve.h"

namespace mxs {
namespace {

template <typename T> __device__ __forceinline__ double to_f64(T v);
template <> __device__ __forceinline__ double to_f64<double>(double v) { return v; }
template <> __device__ __forceinline__ double to_f64<float>(float v) { return static_cast<double>(v); }
template <> __device__ __forceinline__ double to_f64<bf16>(bf16 v) {
    return static_cast<double>(bf16_to_float(v.bits));
}
template <typename T> __device__ __forceinline__ T from_f64(double v);
template <> __device__ __forceinline__ double from_f64<double>(double v) { return v; }
template <> __device__ __forceinline__ float from_f64<float>(double v) { return static_cast<float>(v); }
// double -> bf16 rounds once, to nearest even, via the exact float split:
// the float nearest to v can round the wrong way only at a bf16 tie; the
// remainder v - float(v) decides that case.
template <> __device__ __forceinline__ bf16 from_f64<bf16>(double v) {
    const float f = static_cast<float>(v);
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return bf16{float_to_bf16(f)};
    const double rem = v - static_cast<double>(f);
    if ((u & 0xffffu) == 0x8000u && rem != 0.0) {
        // exactly halfway in float but not in double: round by the remainder
        const bool up = (rem > 0) == ((u & 0x80000000u) == 0);
        return bf16{static_cast<uint16_t>((u >> 16) + (up ? 1u : 0u))};
    }
    return bf16{float_to_bf16(f)};
}

struct LineRef {
    const void *in;
    void *out;
    int n;
    double p1, p2, invK;
    const double *pow;   // power table of the register kernel
};

template <typename T>
struct RaggedSrc {
    RaggedLines a;
    __device__ LineRef get(int li) const {
        const int b = a.order[li];
        const long long base = a.offsets[b];
        LineRef L;
        L.in = static_cast<const T *>(a.in) + base;
        L.out = static_cast<T *>(a.out) + base;
        L.n = static_cast<int>(a.offsets[b + 1] - base);
        L.p1 = a.p1;
        L.p2 = a.p2;
        L.invK = a.invK;
        L.pow = a.pow;
        return L;
    }
};

template <typename T>
struct RowsSrc {
    const RowsInst *inst;
    const int *map;
    __device__ LineRef get(int li) const {
        const RowsInst &I = inst[map ? map[li] : 0];
        const long long j = li - I.line0;
        LineRef L;
        L.in = static_cast<const T *>(I.in) + j * I.ld;
        L.out = static_cast<T *>(I.out) + j * I.ld;
        L.n = I.nx;
        L.p1 = I.p1;
        L.p2 = I.p2;
        L.invK = I.invK;
        L.pow = I.pow;
        return L;
    }
};

}  // namespace
}  // namespace mxs
