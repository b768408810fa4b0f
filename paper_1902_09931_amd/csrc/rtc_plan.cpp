// Stencils with a user function compiled at run time (the function-pointer
// variants of Sec. 4.2, with several input data sets per function).
//
// The paper hands the library a device function that receives the input
// data, the coefficients and the position of the point, and returns the
// output value.  A C ABI cannot carry a device function pointer, so the
// caller passes the function's HIP source instead; the plan generates a
// kernel around it, compiles it for the device with hipRTC and loads it.
// The generated kernel stages, for a workgroup's strip of columns and chunk
// of rows, a tile of every input (with the window's halo, periodic wrap or
// clamped at a non-periodic border) in LDS; each thread then fills, per
// input, the window of its point in window order (row by row from the top
// left, left to right) and calls the function with those windows, the
// coefficients and loc, the position of the point in the window.  Window
// extents, input count and storage type are compile-time constants of the
// generated code, so the windows live in registers.
#include "plans.h"

#include <hip/hiprtc.h>

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace mxs {

namespace {

// Launch arguments, laid out identically in the generated source.
struct FnArgs {
    const void *in[MXS_MAX_FN_INPUTS];
    void *out;
    const void *coe;   // device, ncoe values of the arithmetic type
    long long ld;
    int nx, ny;
    int nstrips, nchunks;
};

const char *kPrelude = R"(
typedef unsigned short mxs_bf16_bits;
struct FnArgs {
    const void *in[%d];
    void *out;
    const void *coe;
    long long ld;
    int nx, ny;
    int nstrips, nchunks;
};
__device__ __forceinline__ float mxs_bf16_to_float(mxs_bf16_bits b) { return __uint_as_float((unsigned)b << 16); }
__device__ __forceinline__ mxs_bf16_bits mxs_float_to_bf16(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (mxs_bf16_bits)((u >> 16) | 0x0040u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (mxs_bf16_bits)(u >> 16);
}
)";

// The kernel around the user function; %s/%d fields filled by the plan.
const char *kKernel = R"(
#define MXS_NIN %d
#define MXS_L %d
#define MXS_R %d
#define MXS_T %d
#define MXS_B %d
#define MXS_PERIODIC %d
#define MXS_ROWS %d
#define MXS_NT %d
#define MXS_STORAGE %d
constexpr int kWX = MXS_L + MXS_R + 1, kWY = MXS_T + MXS_B + 1, kNWIN = kWX * kWY;
constexpr int kLoc = MXS_T * kWX + MXS_L;
constexpr int kTW = MXS_NT + MXS_L + MXS_R, kTH = MXS_ROWS + MXS_T + MXS_B;

__device__ __forceinline__ long long mxs_fix(long long k, long long n) {
    if (MXS_PERIODIC) { k %%= n; return k < 0 ? k + n : k; }
    return k < 0 ? 0 : (k >= n ? n - 1 : k);
}
#define MXS_GLOBAL __attribute__((address_space(1)))
__device__ __forceinline__ mxs_real mxs_load(const void *p, long long i) {
#if MXS_STORAGE == 0
    return ((const MXS_GLOBAL double *)p)[i];
#elif MXS_STORAGE == 1
    return ((const MXS_GLOBAL float *)p)[i];
#else
    return mxs_bf16_to_float(((const MXS_GLOBAL mxs_bf16_bits *)p)[i]);
#endif
}
__device__ __forceinline__ void mxs_store(void *p, long long i, mxs_real v) {
#if MXS_STORAGE == 0
    ((MXS_GLOBAL double *)p)[i] = v;
#elif MXS_STORAGE == 1
    ((MXS_GLOBAL float *)p)[i] = v;
#else
    ((MXS_GLOBAL mxs_bf16_bits *)p)[i] = mxs_float_to_bf16(v);
#endif
}

extern "C" __global__ void __launch_bounds__(MXS_NT) mxs_user_stencil(const FnArgs a) {
    extern __shared__ mxs_real mxs_tile[];
    const int strip = blockIdx.x %% a.nstrips, chunk = blockIdx.x / a.nstrips;
    const long long i0 = static_cast<long long>(strip) * MXS_NT;
    const long long j0 = static_cast<long long>(chunk) * MXS_ROWS;
#pragma unroll
    for (int k = 0; k < MXS_NIN; ++k)
        for (int e = threadIdx.x; e < kTH * kTW; e += MXS_NT) {
            const int r = e / kTW, c = e - r * kTW;
            const long long J = mxs_fix(j0 - MXS_T + r, a.ny), I = mxs_fix(i0 - MXS_L + c, a.nx);
            mxs_tile[(k * kTH + r) * kTW + c] = mxs_load(a.in[k], J * a.ld + I);
        }
    __syncthreads();
    const long long i = i0 + threadIdx.x;
    if (i >= a.nx) return;
    const mxs_real *coe = static_cast<const mxs_real *>(a.coe);
#pragma unroll 1
    for (int q = 0; q < MXS_ROWS; ++q) {
        const long long j = j0 + q;
        if (j >= a.ny) break;
        if (!MXS_PERIODIC && (i < MXS_L || i > a.nx - 1 - MXS_R || j < MXS_T || j > a.ny - 1 - MXS_B)) continue;
        mxs_real w[MXS_NIN][kNWIN];
#pragma unroll
        for (int k = 0; k < MXS_NIN; ++k)
#pragma unroll
            for (int b = 0; b < kWY; ++b)
#pragma unroll
                for (int c = 0; c < kWX; ++c)
                    w[k][b * kWX + c] = mxs_tile[(k * kTH + q + b) * kTW + threadIdx.x + c];
        const mxs_real *wp[MXS_NIN];
#pragma unroll
        for (int k = 0; k < MXS_NIN; ++k) wp[k] = w[k];
        mxs_store(a.out, j * a.ld + i, %s(wp, coe, kLoc));
    }
}
)";

std::string format(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    va_list ap2;
    va_copy(ap2, ap);
    const int n = vsnprintf(nullptr, 0, fmt, ap);
    va_end(ap);
    std::string s(static_cast<size_t>(n) + 1, '\0');
    vsnprintf(&s[0], s.size(), fmt, ap2);
    va_end(ap2);
    s.resize(static_cast<size_t>(n));
    return s;
}

// Compiled code objects by generated source, for the life of the process.
std::mutex g_rtc_mu;
std::map<std::string, std::vector<char>> g_rtc_code;

mxs_status compile(const std::string &src, std::vector<char> *code) {
    {
        std::lock_guard<std::mutex> g(g_rtc_mu);
        auto it = g_rtc_code.find(src);
        if (it != g_rtc_code.end()) {
            *code = it->second;
            return MXS_OK;
        }
    }
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "mxs_user_stencil.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
        return fail(MXS_ERR_HIP, "hipRTC could not create the program");
    int dev = 0;
    hipDeviceProp_t prop{};
    std::string arch = "--offload-arch=gfx950";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.gcnArchName[0])
        arch = std::string("--offload-arch=") + prop.gcnArchName;
    const char *opts[] = {arch.c_str(), "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                          "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(prog, 7, opts);
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        std::string log;
        if (hiprtcGetProgramLogSize(prog, &n) == HIPRTC_SUCCESS && n > 1) {
            log.resize(n);
            (void)hiprtcGetProgramLog(prog, &log[0]);
        }
        (void)hiprtcDestroyProgram(&prog);
        if (log.size() > 600) log = log.substr(0, 600) + "...";
        return fail(MXS_ERR_INVALID_ARG, "the user function did not compile: %s", log.c_str());
    }
    size_t n = 0;
    if (hiprtcGetCodeSize(prog, &n) != HIPRTC_SUCCESS || n == 0) {
        (void)hiprtcDestroyProgram(&prog);
        return fail(MXS_ERR_HIP, "hipRTC returned no code");
    }
    code->assign(n, 0);
    const bool ok = hiprtcGetCode(prog, code->data()) == HIPRTC_SUCCESS;
    (void)hiprtcDestroyProgram(&prog);
    if (!ok) return fail(MXS_ERR_HIP, "hipRTC returned no code");
    std::lock_guard<std::mutex> g(g_rtc_mu);
    g_rtc_code[src] = *code;
    return MXS_OK;
}

struct FnPlan final : mxs_plan_s {
    FnArgs a{};
    int dtype = F64, nin = 1, threads = 256, rows = 8;
    size_t lds = 0;
    DevBuf coe;
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    FnPlan() : mxs_plan_s(KIND_FN) {}
    ~FnPlan() override {
        if (mod) (void)hipModuleUnload(mod);
    }
    mxs_status compute(hipStream_t s) override {
        void *params[] = {&a};
        const hipError_t e = hipModuleLaunchKernel(fn, static_cast<unsigned>(a.nstrips * a.nchunks), 1, 1,
                                                   static_cast<unsigned>(threads), 1, 1, static_cast<unsigned>(lds),
                                                   s, params, nullptr);
        return e == hipSuccess ? MXS_OK : hip_fail(e, "user-function stencil launch");
    }
    mxs_status swap() override {
        const void *t = a.in[0];
        a.in[0] = a.out;
        a.out = const_cast<void *>(t);
        return MXS_OK;
    }
    mxs_status rebind(const void *in, void *out) override {
        if (!in || !out) return fail(MXS_ERR_INVALID_ARG, "in/out must be device pointers");
        const size_t bytes = grid_bytes(a.nx, a.ny, a.ld, dtype);
        for (int k = 0; k < nin; ++k)
            if (ranges_overlap(k == 0 ? in : a.in[k], bytes, out, bytes))
                return fail(MXS_ERR_ALIAS, "out overlaps an input");
        a.in[0] = in;
        a.out = out;
        return MXS_OK;
    }
    void info(char *buf, int len) const override {
        snprintf(buf, len, "stencil2d_fn dtype=%d inputs=%d rows=%d threads=%d lds=%zu grid=%d", dtype, nin, rows,
                 threads, lds, a.nstrips * a.nchunks);
    }
};

bool ident_ok(const char *s) {
    if (!s || !*s || !(isalpha(static_cast<unsigned char>(*s)) || *s == '_')) return false;
    for (; *s; ++s)
        if (!(isalnum(static_cast<unsigned char>(*s)) || *s == '_')) return false;
    return true;
}

}  // namespace
}  // namespace mxs

using namespace mxs;

extern "C" {

mxs_status mxs_create_2d_fn(const mxs_stencil2d_fn_desc *d, mxs_plan *plan) {
    if (!plan) return fail(MXS_ERR_INVALID_ARG, "plan output pointer is NULL");
    *plan = nullptr;
    if (!d) return fail(MXS_ERR_INVALID_ARG, "descriptor is NULL");
    if (d->nx <= 0 || d->ny <= 0 || d->ld < d->nx)
        return fail(MXS_ERR_INVALID_ARG, "need nx > 0, ny > 0, ld >= nx");
    if (d->dir != MXS_X && d->dir != MXS_Y && d->dir != MXS_XY)
        return fail(MXS_ERR_INVALID_ARG, "dir must be MXS_X, MXS_Y or MXS_XY");
    if (d->bc != MXS_NP && d->bc != MXS_P) return fail(MXS_ERR_INVALID_ARG, "bc must be MXS_NP or MXS_P");
    if (!valid_dtype(d->dtype)) return fail(MXS_ERR_INVALID_ARG, "unknown dtype %d", d->dtype);
    if (d->left < 0 || d->right < 0 || d->top < 0 || d->bottom < 0)
        return fail(MXS_ERR_INVALID_ARG, "negative stencil extent");
    if ((d->dir == MXS_X && (d->top || d->bottom)) || (d->dir == MXS_Y && (d->left || d->right)))
        return fail(MXS_ERR_INVALID_ARG, "extents do not match the direction");
    if (d->left + d->right >= d->nx || d->top + d->bottom >= d->ny)
        return fail(MXS_ERR_INVALID_ARG, "the window is wider than the grid");
    if (d->left + d->right + 1 > MXS_MAX_TAPS_1D || d->top + d->bottom + 1 > MXS_MAX_TAPS_1D)
        return fail(MXS_ERR_UNSUPPORTED, "window exceeds %d taps along an axis", MXS_MAX_TAPS_1D);
    if (d->ninputs < 1 || d->ninputs > MXS_MAX_FN_INPUTS || !d->inputs)
        return fail(MXS_ERR_INVALID_ARG, "need 1 to %d inputs", MXS_MAX_FN_INPUTS);
    if (d->ncoe < 0 || d->ncoe > MXS_MAX_FN_COE || (d->ncoe > 0 && !d->coe))
        return fail(MXS_ERR_INVALID_ARG, "need 0 to %d coefficients", MXS_MAX_FN_COE);
    if (!d->source || !ident_ok(d->name))
        return fail(MXS_ERR_INVALID_ARG, "need the function's source and a valid identifier for its name");
    if (!d->out) return fail(MXS_ERR_INVALID_ARG, "out is NULL");
    const size_t bytes = grid_bytes(d->nx, d->ny, d->ld, d->dtype);
    for (int k = 0; k < d->ninputs; ++k) {
        if (!d->inputs[k]) return fail(MXS_ERR_INVALID_ARG, "input %d is NULL", k);
        if (ranges_overlap(d->inputs[k], bytes, d->out, bytes)) return fail(MXS_ERR_ALIAS, "out overlaps input %d", k);
    }
    FnPlan *p = new (std::nothrow) FnPlan();
    if (!p) return fail(MXS_ERR_OOM, "host allocation failed");
    p->dtype = d->dtype;
    p->nin = d->ninputs;
    const size_t asz = d->dtype == F64 ? 8 : 4;
    // the largest chunk (then the narrowest strip) whose tiles fit 64 KiB
    auto tile_bytes = [&](int t, int r) {
        return static_cast<size_t>(p->nin) * (r + d->top + d->bottom) * (t + d->left + d->right) * asz;
    };
    p->threads = 256;
    p->rows = 8;
    while (tile_bytes(p->threads, p->rows) > 65536 && p->rows > 1) p->rows /= 2;
    while (tile_bytes(p->threads, p->rows) > 65536 && p->threads > 64) p->threads /= 2;
    if (tile_bytes(p->threads, p->rows) > 65536) {
        delete p;
        return fail(MXS_ERR_UNSUPPORTED, "the input tiles do not fit the LDS of a workgroup");
    }
    p->lds = tile_bytes(p->threads, p->rows);
    const char *real = d->dtype == F64 ? "double" : "float";
    std::string src = "typedef " + std::string(real) + " mxs_real;\n" + format(kPrelude, MXS_MAX_FN_INPUTS) +
                      "\n// ---- user function ----\n" + d->source + "\n// ----\n" +
                      format(kKernel, p->nin, d->left, d->right, d->top, d->bottom, d->bc == MXS_P ? 1 : 0, p->rows,
                             p->threads, d->dtype, d->name);
    std::vector<char> code;
    mxs_status st = compile(src, &code);
    if (st) {
        delete p;
        return st;
    }
    hipError_t e = hipModuleLoadData(&p->mod, code.data());
    if (e == hipSuccess) e = hipModuleGetFunction(&p->fn, p->mod, "mxs_user_stencil");
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "loading the compiled user function");
    }
    if (d->ncoe > 0) {
        if (d->dtype == F64) {
            e = p->coe.upload(d->coe, sizeof(double) * d->ncoe);
        } else {
            std::vector<float> cf(d->coe, d->coe + d->ncoe);
            e = p->coe.upload(cf.data(), sizeof(float) * d->ncoe);
        }
        if (e != hipSuccess) {
            delete p;
            return hip_fail(e, "coefficient upload");
        }
    }
    for (int k = 0; k < p->nin; ++k) p->a.in[k] = d->inputs[k];
    p->a.out = d->out;
    p->a.coe = p->coe.ptr;
    p->a.ld = d->ld;
    p->a.nx = d->nx;
    p->a.ny = d->ny;
    p->a.nstrips = (d->nx + p->threads - 1) / p->threads;
    p->a.nchunks = (d->ny + p->rows - 1) / p->rows;
    register_plan(p);
    *plan = p;
    return MXS_OK;
}

}  // extern "C"
