// Internal declarations shared by the HIP kernels and the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace mxs {

// Pointers to global memory.  A pointer read from an instance table in
// device memory is generic (its accesses would be flat instructions, which
// also occupy the LDS counter); converted with as_global, its accesses are
// global loads and stores, or scalar loads where uniform.
template <typename T> using gptr = T __attribute__((address_space(1))) *;
template <typename T> __device__ __forceinline__ gptr<T> as_global(T *p) { return (gptr<T>)p; }

// ---------------------------------------------------------------------------
// Storage types.  bfloat16 is carried as its 16 raw bits.
// ---------------------------------------------------------------------------
struct bf16 {
    uint16_t bits;
};

enum Dtype { F64 = 0, F32 = 1, BF16 = 2 };

inline int dtype_size(int dt) { return dt == F64 ? 8 : dt == F32 ? 4 : 2; }

// Storage traits: accumulation type and elements per 8- or 16-byte vector.
template <typename T> struct St;
template <> struct St<double> { using acc = double; static constexpr int V = 2; };
template <> struct St<float>  { using acc = float;  static constexpr int V = 4; };
template <> struct St<bf16>   { using acc = float;  static constexpr int V = 8; };

__device__ __forceinline__ float bf16_to_float(uint16_t b) {
    return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

// float -> bfloat16, round to nearest, ties to even; NaN stays NaN.
__device__ __forceinline__ uint16_t float_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
        return static_cast<uint16_t>((u >> 16) | 0x0040u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

template <typename T> __device__ __forceinline__ typename St<T>::acc to_acc(T v);
template <> __device__ __forceinline__ double to_acc<double>(double v) { return v; }
template <> __device__ __forceinline__ float to_acc<float>(float v) { return v; }
template <> __device__ __forceinline__ float to_acc<bf16>(bf16 v) { return bf16_to_float(v.bits); }

template <typename T> __device__ __forceinline__ T from_acc(typename St<T>::acc v);
template <> __device__ __forceinline__ double from_acc<double>(double v) { return v; }
template <> __device__ __forceinline__ float from_acc<float>(float v) { return v; }
template <> __device__ __forceinline__ bf16 from_acc<bf16>(float v) { return bf16{float_to_bf16(v)}; }

// Vector load/store of St<T>::V consecutive elements (16 bytes: 2 doubles, 4
// floats or 8 bfloat16s).  The address must be aligned to 16 bytes.
template <typename T>
__device__ __forceinline__ void load_vec(const T *p, typename St<T>::acc *x);
template <>
__device__ __forceinline__ void load_vec<double>(const double *p, double *x) {
    double2 v = *reinterpret_cast<const double2 *>(p);
    x[0] = v.x; x[1] = v.y;
}
template <>
__device__ __forceinline__ void load_vec<float>(const float *p, float *x) {
    float4 v = *reinterpret_cast<const float4 *>(p);
    x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
}
// 8 bfloat16s from / to 4 packed words
__device__ __forceinline__ void unpack_bf16x8(const uint32_t (&w)[4], float *x) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        x[2 * k] = __uint_as_float(w[k] << 16);
        x[2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
    }
}
__device__ __forceinline__ void pack_bf16x8(const float *x, uint32_t (&w)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
        w[k] = static_cast<uint32_t>(float_to_bf16(x[2 * k])) | (static_cast<uint32_t>(float_to_bf16(x[2 * k + 1])) << 16);
}
template <>
__device__ __forceinline__ void load_vec<bf16>(const bf16 *p, float *x) {
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    unpack_bf16x8(w, x);
}

template <typename T>
__device__ __forceinline__ void store_vec(T *p, const typename St<T>::acc *x);
template <>
__device__ __forceinline__ void store_vec<double>(double *p, const double *x) {
    *reinterpret_cast<double2 *>(p) = make_double2(x[0], x[1]);
}
template <>
__device__ __forceinline__ void store_vec<float>(float *p, const float *x) {
    *reinterpret_cast<float4 *>(p) = make_float4(x[0], x[1], x[2], x[3]);
}
template <>
__device__ __forceinline__ void store_vec<bf16>(bf16 *p, const float *x) {
    uint32_t w[4];
    pack_bf16x8(x, w);
    *reinterpret_cast<uint4 *>(p) = make_uint4(w[0], w[1], w[2], w[3]);
}

// Streaming (non-temporal) vector stores: the line is written without being
// kept in the caches, leaving L2 to the inputs that are read again.
typedef double v2d_t __attribute__((ext_vector_type(2)));
typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef unsigned int v2u_t __attribute__((ext_vector_type(2)));
typedef unsigned int v4u_t __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ void store_vec_nt(T *p, const typename St<T>::acc *x);
template <>
__device__ __forceinline__ void store_vec_nt<double>(double *p, const double *x) {
    v2d_t v = {x[0], x[1]};
    __builtin_nontemporal_store(v, reinterpret_cast<v2d_t *>(p));
}
template <>
__device__ __forceinline__ void store_vec_nt<float>(float *p, const float *x) {
    v4f_t v = {x[0], x[1], x[2], x[3]};
    __builtin_nontemporal_store(v, reinterpret_cast<v4f_t *>(p));
}
template <>
__device__ __forceinline__ void store_vec_nt<bf16>(bf16 *p, const float *x) {
    uint32_t w[4];
    pack_bf16x8(x, w);
    v4u_t v = {w[0], w[1], w[2], w[3]};
    __builtin_nontemporal_store(v, reinterpret_cast<v4u_t *>(p));
}

// Element access through global-memory pointers (bf16 by its bits).
template <typename T, typename I> __device__ __forceinline__ T gld(gptr<const T> p, I i) {
    if constexpr (std::is_same<T, bf16>::value) return bf16{reinterpret_cast<gptr<const uint16_t>>(p)[i]};
    else return p[i];
}
template <typename T, typename I> __device__ __forceinline__ void gst(gptr<T> p, I i, T v) {
    if constexpr (std::is_same<T, bf16>::value) reinterpret_cast<gptr<uint16_t>>(p)[i] = v.bits;
    else p[i] = v;
}

// The same vector accesses through global-memory pointers.
template <typename T>
__device__ __forceinline__ void load_vec(gptr<const T> p, typename St<T>::acc *x);
template <>
__device__ __forceinline__ void load_vec<double>(gptr<const double> p, double *x) {
    const v2d_t v = *reinterpret_cast<gptr<const v2d_t>>(p);
    x[0] = v.x; x[1] = v.y;
}
template <>
__device__ __forceinline__ void load_vec<float>(gptr<const float> p, float *x) {
    const v4f_t v = *reinterpret_cast<gptr<const v4f_t>>(p);
    x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
}
template <>
__device__ __forceinline__ void load_vec<bf16>(gptr<const bf16> p, float *x) {
    const v4u_t v = *reinterpret_cast<gptr<const v4u_t>>(p);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    unpack_bf16x8(w, x);
}
template <typename T>
__device__ __forceinline__ void store_vec(gptr<T> p, const typename St<T>::acc *x);
template <>
__device__ __forceinline__ void store_vec<double>(gptr<double> p, const double *x) {
    const v2d_t v = {x[0], x[1]};
    *reinterpret_cast<gptr<v2d_t>>(p) = v;
}
template <>
__device__ __forceinline__ void store_vec<float>(gptr<float> p, const float *x) {
    const v4f_t v = {x[0], x[1], x[2], x[3]};
    *reinterpret_cast<gptr<v4f_t>>(p) = v;
}
template <>
__device__ __forceinline__ void store_vec<bf16>(gptr<bf16> p, const float *x) {
    uint32_t w[4];
    pack_bf16x8(x, w);
    const v4u_t v = {w[0], w[1], w[2], w[3]};
    *reinterpret_cast<gptr<v4u_t>>(p) = v;
}
template <typename T>
__device__ __forceinline__ void store_vec_nt(gptr<T> p, const typename St<T>::acc *x);
template <>
__device__ __forceinline__ void store_vec_nt<double>(gptr<double> p, const double *x) {
    v2d_t v = {x[0], x[1]};
    __builtin_nontemporal_store(v, reinterpret_cast<gptr<v2d_t>>(p));
}
template <>
__device__ __forceinline__ void store_vec_nt<float>(gptr<float> p, const float *x) {
    v4f_t v = {x[0], x[1], x[2], x[3]};
    __builtin_nontemporal_store(v, reinterpret_cast<gptr<v4f_t>>(p));
}
template <>
__device__ __forceinline__ void store_vec_nt<bf16>(gptr<bf16> p, const float *x) {
    uint32_t w[4];
    pack_bf16x8(x, w);
    v4u_t v = {w[0], w[1], w[2], w[3]};
    __builtin_nontemporal_store(v, reinterpret_cast<gptr<v4u_t>>(p));
}

__device__ __forceinline__ long long wrap_ll(long long k, long long n) {
    long long r = k % n;
    return r < 0 ? r + n : r;
}
// k mod n with one conditional add or subtract for -n <= k < 2n (halo
// indices); the division only for indices farther out.
__device__ __forceinline__ long long wrap_fast(long long k, long long n) {
    if (k < 0) k += n;
    else if (k >= n) k -= n;
    if (k < 0 || k >= n) k = wrap_ll(k, n);
    return k;
}

// Point function f(c) = sum_m coe[m] c^m by Horner's rule; identity when
// ncoe == 0.
template <typename A>
__device__ __forceinline__ A point_fun(A c, const A *coe, int ncoe) {
    if (ncoe == 0) return c;
    A f = coe[ncoe - 1];
    for (int m = ncoe - 2; m >= 0; --m) f = f * c + coe[m];
    return f;
}

// Map a workgroup index to a tile index so that the workgroups the hardware
// sends to one XCD (round robin: block b goes to XCD b % 8) cover one
// contiguous range of tiles.  A bijection on [0, n).
__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int q = n >> 3, r = n & 7;
    const int x = b & 7, k = b >> 3;
    const int base = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    return base + k;
}

constexpr int kMaxCoe = 8;

// ---------------------------------------------------------------------------
// 2D stencil launch arguments.
// ---------------------------------------------------------------------------
struct Stencil2DArgs {
    const void *in;
    void *out;
    long long ld;
    int nx, ny;
    int L, R, T, B;         // actual extents
    int periodic;
    int ncoe;
    const void *wts;        // device, NWY x NWX padded weights in the accumulation type
    const void *wts_up;     // the same window flipped vertically (rows walked upward)
    double coe_d[kMaxCoe];
    float coe_f[kMaxCoe];
    int rows;               // output rows per workgroup
    int nchunks;            // row chunks per strip
    int nstrips;            // column strips
    int vec_ok;             // 16-byte aligned rows
    int order;              // tile order: 0 = each XCD a contiguous run of row chunks
                            // of one strip; 1 = row-major sweep (strips fastest);
                            // 2 = each XCD a contiguous band of chunks, row-major
    int nt_store;           // 1: non-temporal output stores
    int block_rows;         // 0: streaming form; 8 or 16: block form reading
                            // that many input rows per workgroup at once
                            // (rows = block_rows - NWY + 1 output rows)
    int xshuffle;           // block form, centred windows: x neighbours by
                            // lane shifts instead of an LDS row
};

// Vectors per thread in one tile of the batched 1D stencil (a tile is
// threads * V * kS1dVecs elements, so one workgroup has that many bytes in
// flight at once).
constexpr int kS1dVecs = 4;

struct Stencil1DArgs {
    const void *in;
    void *out;
    const long long *offsets;   // device, nbatch + 1
    const int *tile_first;      // device, ntiles + 1: first signal of each tile
    long long total;
    int nbatch;
    int ntiles;
    int L, R;
    int periodic;
    int ncoe;
    const void *wts;            // device, NWX padded weights
    double coe_d[kMaxCoe];
    float coe_f[kMaxCoe];
    int max_sig_per_tile;       // LDS slots reserved for offsets
    int vec_ok;
};

// Window buckets: padded widths the kernels are compiled for.
int bucket_width(int taps);   // 1, 3, 5, 9 or 17; 0 if too wide

hipError_t launch_stencil2d(int dtype, int nwx, int nwy, const Stencil2DArgs &a,
                            int threads, hipStream_t s);
hipError_t launch_stencil1d(int dtype, int nwx, const Stencil1DArgs &a, int threads,
                            int grid, hipStream_t s);
size_t stencil2d_lds_bytes(int dtype, int nwx, int nwy, int threads, int block_rows, int xshuffle);
// Read `bytes` (a multiple of 16) of a device buffer once, so that the
// memory-side cache holds none of the data timed next.
hipError_t launch_cache_flush(void *buf, size_t bytes, hipStream_t s);
// Whether the block form is compiled for this padded window and row count.
bool stencil2d_block_ok(int nwx, int nwy, int block_rows);
// Whether the block form can take x neighbours from neighbouring lanes
// (centred windows of padded width nwx, at most one vector on each side).
bool stencil2d_xshuffle_ok(int dtype, int nwx, int nwy, int left, int right, int block_rows);
size_t stencil1d_lds_bytes(int dtype, int nwx, int threads, int max_sig);

}  // namespace mxs
