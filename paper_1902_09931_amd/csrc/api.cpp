// C ABI of the library: argument validation, plan objects and kernel launch.
//
// A plan owns only what it allocates (device copies of weights, tables,
// scratch, captured graphs).  The caller owns every data buffer and stream.
#include "mxsten.h"
#include "plans.h"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

void mxs_plan_s::info(char *buf, int len) const { snprintf(buf, len, "plan kind %d", kind); }

namespace mxs {

namespace {
thread_local std::string g_err;
std::mutex g_live_mu;
std::unordered_set<const mxs_plan_s *> g_live;
}  // namespace

mxs_status fail(mxs_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

mxs_status hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? MXS_ERR_OOM : MXS_ERR_HIP, "%s: %s", what,
                hipGetErrorString(e));
}

void register_plan(const mxs_plan_s *p) {
    std::lock_guard<std::mutex> g(g_live_mu);
    g_live.insert(p);
}

bool unregister_plan(const mxs_plan_s *p) {
    std::lock_guard<std::mutex> g(g_live_mu);
    return g_live.erase(p) == 1;
}

bool is_live(const mxs_plan_s *p) {
    std::lock_guard<std::mutex> g(g_live_mu);
    return g_live.count(p) == 1;
}

// ---------------------------------------------------------------------------
DevBuf::~DevBuf() { reset(); }
void DevBuf::reset() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}
hipError_t DevBuf::alloc(size_t n) {
    reset();
    if (n == 0) return hipSuccess;
    hipError_t e = hipMalloc(&ptr, n);
    if (e != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        return e;
    }
    bytes = n;
    return hipSuccess;
}
hipError_t DevBuf::upload(const void *src, size_t n) {
    hipError_t e = alloc(n);
    if (e != hipSuccess || n == 0) return e;
    return hipMemcpy(ptr, src, n, hipMemcpyHostToDevice);
}

bool ranges_overlap(const void *a, size_t abytes, const void *b, size_t bbytes) {
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
    return a0 < b0 + bbytes && b0 < a0 + abytes;
}

size_t grid_bytes(int nx, int ny, long long ld, int dtype) {
    return (static_cast<size_t>(ny - 1) * static_cast<size_t>(ld) + static_cast<size_t>(nx)) *
           dtype_size(dtype);
}

int device_lds_limit() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        v <= 0)
        return 65536;
    return v;
}

int device_cu_count() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        v <= 0)
        return 256;
    return v;
}

// ---------------------------------------------------------------------------
// 2D stencil plan
// ---------------------------------------------------------------------------
namespace {

int vec_elems(int dtype) { return dtype == F64 ? St<double>::V : dtype == F32 ? St<float>::V : St<bf16>::V; }

bool vec_aligned(const void *p, int dtype) {
    const uintptr_t bytes = static_cast<uintptr_t>(vec_elems(dtype)) * dtype_size(dtype);
    return reinterpret_cast<uintptr_t>(p) % bytes == 0;
}

// Padded weights NWY x NWX in the accumulation type, followed by the same
// window flipped vertically (row q holds window row T + B - q): the kernel
// reads the second copy for row chunks it walks upward.
template <typename A>
std::vector<A> pad_weights(const double *w, int L, int R, int T, int B, int nwx, int nwy) {
    const size_t n = static_cast<size_t>(nwx) * nwy;
    std::vector<A> out(2 * n, A(0));
    const int width = L + R + 1;
    for (int q = 0; q <= T + B; ++q)
        for (int p = 0; p <= L + R; ++p) {
            out[q * nwx + p] = static_cast<A>(w[q * width + p]);
            out[n + (T + B - q) * nwx + p] = static_cast<A>(w[q * width + p]);
        }
    return out;
}

hipError_t upload_weights(DevBuf &buf, const double *w, int L, int R, int T, int B, int nwx,
                          int nwy, int dtype) {
    if (dtype == F64) {
        auto v = pad_weights<double>(w, L, R, T, B, nwx, nwy);
        return buf.upload(v.data(), v.size() * sizeof(double));
    }
    auto v = pad_weights<float>(w, L, R, T, B, nwx, nwy);
    return buf.upload(v.data(), v.size() * sizeof(float));
}

}  // namespace

struct Stencil2DPlan final : mxs_plan_s {
    Stencil2DArgs a{};
    int dtype = F64, nwx = 1, nwy = 1, threads = 256;
    DevBuf wts;
    Stencil2DPlan() : mxs_plan_s(KIND_STENCIL2D) {}

    // rows: output rows per workgroup (streaming form), or ignored in the
    // block form, which reads block rows per workgroup (block_rows - nwy + 1
    // output rows).
    void set_layout(int rows, int order, int nthreads, int nt, int block = 0, int xs = 0) {
        threads = nthreads;
        a.block_rows = block;
        a.xshuffle = block ? xs : 0;
        if (block) rows = block - nwy + 1;
        a.rows = rows;
        a.order = order;
        a.nt_store = nt;
        const int W = threads * vec_elems(dtype);
        a.nstrips = (a.nx + W - 1) / W;
        a.nchunks = (a.ny + rows - 1) / rows;
    }

    // Layout before tuning: streaming stores; row chunks sized per direction
    // (short for x, tall for y, medium for xy), shrunk until the grid keeps
    // several workgroups per CU.
    void default_layout() {
        int rows = nwy == 1 ? 4 : (nwx == 1 ? 64 : 16);
        const int W = 256 * vec_elems(dtype);
        const long long strips = (a.nx + W - 1) / W;
        const long long want = 8LL * device_cu_count();
        while (rows > std::max(4, nwy) && strips * ((a.ny + rows - 1) / rows) < want) rows /= 2;
        set_layout(rows, 1, 256, 1);
        // explicit override "rows,order,threads,nt[,block]" for experiments
        if (const char *env = getenv("MXS_STENCIL_TILE")) {
            int r = 0, o = 0, t = 0, nt = 1, blk = 0, xs = 0;
            const int k = sscanf(env, "%d,%d,%d,%d,%d,%d", &r, &o, &t, &nt, &blk, &xs);
            if (k >= 3 && r > 0 && (o == 0 || o == 1 || o == 2) && (t == 64 || t == 128 || t == 256) &&
                (blk == 0 || stencil2d_block_ok(nwx, nwy, blk)) &&
                (xs == 0 || stencil2d_xshuffle_ok(dtype, nwx, nwy, a.L, a.R, blk)) &&
                stencil2d_lds_bytes(dtype, nwx, nwy, t, blk, xs) <= static_cast<size_t>(device_lds_limit()))
                set_layout(r, o, t, nt != 0, blk, xs);
        }
    }

    std::string key() const {
        char buf[160];
        snprintf(buf, sizeof buf, "s2d:%d:%d:%d:%d:%d:%lld:%d:%d", dtype, nwx, nwy, a.nx, a.ny, a.ld,
                 a.periodic, a.ncoe > 0);
        return buf;
    }

    mxs_status autotune(hipStream_t s) override;
    void info(char *buf, int len) const override {
        snprintf(buf, len, "stencil2d dtype=%d window=%dx%d rows=%d order=%d threads=%d nt_store=%d block=%d xshuffle=%d grid=%d",
                 dtype, nwx, nwy, a.rows, a.order, threads, a.nt_store, a.block_rows, a.xshuffle,
                 a.nstrips * a.nchunks);
    }

    mxs_status set_io(const void *in, void *out) {
        if (!in || !out) return fail(MXS_ERR_INVALID_ARG, "in/out must be device pointers");
        const size_t bytes = grid_bytes(a.nx, a.ny, a.ld, dtype);
        if (ranges_overlap(in, bytes, out, bytes))
            return fail(MXS_ERR_ALIAS, "in and out overlap; stencils must write out of place");
        a.in = in;
        a.out = out;
        a.vec_ok = (a.ld % vec_elems(dtype) == 0) && vec_aligned(in, dtype) && vec_aligned(out, dtype);
        return MXS_OK;
    }

    mxs_status compute(hipStream_t s) override {
        hipError_t e = launch_stencil2d(dtype, nwx, nwy, a, threads, s);
        return e == hipSuccess ? MXS_OK : hip_fail(e, "stencil2d launch");
    }
    mxs_status swap() override {
        const void *tmp = a.in;
        a.in = a.out;
        a.out = const_cast<void *>(tmp);
        return MXS_OK;
    }
    mxs_status rebind(const void *in, void *out) override { return set_io(in, out); }
};

// ---------------------------------------------------------------------------
// Batched ragged 1D stencil plan
// ---------------------------------------------------------------------------
struct Stencil1DPlan final : mxs_plan_s {
    Stencil1DArgs a{};
    int dtype = F64, nwx = 1, threads = 256, grid = 1;
    DevBuf wts, offsets, tile_first;
    Stencil1DPlan() : mxs_plan_s(KIND_STENCIL1D) {}

    mxs_status set_io(const void *in, void *out) {
        if (!in || !out) return fail(MXS_ERR_INVALID_ARG, "in/out must be device pointers");
        const size_t bytes = static_cast<size_t>(a.total) * dtype_size(dtype);
        if (ranges_overlap(in, bytes, out, bytes))
            return fail(MXS_ERR_ALIAS, "in and out overlap; stencils must write out of place");
        a.in = in;
        a.out = out;
        a.vec_ok = vec_aligned(in, dtype) && vec_aligned(out, dtype);
        return MXS_OK;
    }
    mxs_status compute(hipStream_t s) override {
        hipError_t e = launch_stencil1d(dtype, nwx, a, threads, grid, s);
        return e == hipSuccess ? MXS_OK : hip_fail(e, "stencil1d launch");
    }
    mxs_status swap() override {
        const void *tmp = a.in;
        a.in = a.out;
        a.out = const_cast<void *>(tmp);
        return MXS_OK;
    }
    mxs_status rebind(const void *in, void *out) override { return set_io(in, out); }
};

namespace {
struct TunedLayout {
    int rows, order, threads, nt, block, xs;
};
std::mutex g_tune_mu;
std::map<std::string, TunedLayout> g_tuned;
}  // namespace

mxs_status Stencil2DPlan::autotune(hipStream_t s) {
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tuned.find(key());
        if (it != g_tuned.end()) {
            set_layout(it->second.rows, it->second.order, it->second.threads, it->second.nt, it->second.block,
                       it->second.xs);
            return MXS_OK;
        }
    }
    const TunedLayout start{a.rows, a.order, threads, a.nt_store, a.block_rows, a.xshuffle};
    // every candidate is timed in two passes and keeps its faster time (the
    // best layouts differ by a few percent, about the spread of one timing)
    struct Cand {
        TunedLayout l;
        double t;
    };
    std::vector<Cand> cands;
    const size_t lds_limit = static_cast<size_t>(device_lds_limit());
    for (int rows : {2, 4, 8, 16, 32, 64, 128}) {
        if (rows > 2 * a.ny && rows > 2) continue;
        for (int nthreads : {256, 128}) {
            if (stencil2d_lds_bytes(dtype, nwx, nwy, nthreads, 0, 0) > lds_limit) continue;
            for (int order : {1, 0, 2})
                for (int nt : {1, 0}) cands.push_back({TunedLayout{rows, order, nthreads, nt, 0, 0}, 1e30});
        }
    }
    // block form: all input rows of a chunk requested at once
    for (int block : {8, 12, 16}) {
        if (!stencil2d_block_ok(nwx, nwy, block) || block - nwy + 1 > 2 * a.ny) continue;
        for (int xs : {0, 1}) {
            if (xs && !stencil2d_xshuffle_ok(dtype, nwx, nwy, a.L, a.R, block)) continue;
            for (int nthreads : {256, 128}) {
                if (stencil2d_lds_bytes(dtype, nwx, nwy, nthreads, block, xs) > lds_limit) continue;
                for (int order : {1, 0, 2})
                    for (int nt : {1, 0})
                        cands.push_back({TunedLayout{block - nwy + 1, order, nthreads, nt, block, xs}, 1e30});
            }
        }
    }
    if (cands.empty()) return MXS_OK;
    // Grids whose input and output are between half and four times the
    // memory-side cache are timed with that cache flushed before each
    // launch: back to back, such a grid would find part of its data still
    // cached, which a caller streaming over many grids does not.  Smaller
    // grids stay cached in real use too; larger ones (four times the cache
    // or more) evict their own data before they come back to it.
    const size_t data = 2 * grid_bytes(a.nx, a.ny, a.ld, dtype);
    DevBuf flush;
    if (data > kMallBytes / 2 && data < 4 * kMallBytes && flush.alloc(kFlushBytes) != hipSuccess) {
        (void)hipGetLastError();
        flush.bytes = 0;
    }
    for (int pass = 0; pass < 2; ++pass) {
        for (Cand &c : cands) {
            set_layout(c.l.rows, c.l.order, c.l.threads, c.l.nt, c.l.block, c.l.xs);
            auto launch = [&] { return launch_stencil2d(dtype, nwx, nwy, a, threads, s); };
            const double t = flush.bytes ? time_launches_cold(launch, s, 1, 5, flush.ptr, flush.bytes)
                                         : time_launches(launch, s, 2, 5);
            if (t < 0) {
                set_layout(start.rows, start.order, start.threads, start.nt, start.block, start.xs);
                return hip_fail(hipGetLastError(), "autotune launch");
            }
            c.t = std::min(c.t, t);
        }
    }
    // run-off: the six fastest, timed again in three passes of longer runs
    // (several layouts lie within about one percent of each other)
    std::stable_sort(cands.begin(), cands.end(), [](const Cand &x, const Cand &y) { return x.t < y.t; });
    if (cands.size() > 6) cands.resize(6);
    for (int pass = 0; pass < 3; ++pass) {
        for (Cand &c : cands) {
            set_layout(c.l.rows, c.l.order, c.l.threads, c.l.nt, c.l.block, c.l.xs);
            auto launch = [&] { return launch_stencil2d(dtype, nwx, nwy, a, threads, s); };
            const double t = flush.bytes ? time_launches_cold(launch, s, 1, 10, flush.ptr, flush.bytes)
                                         : time_launches(launch, s, 1, 10);
            if (t < 0) {
                set_layout(start.rows, start.order, start.threads, start.nt, start.block, start.xs);
                return hip_fail(hipGetLastError(), "autotune launch");
            }
            c.t = std::min(c.t, t);
        }
    }
    TunedLayout best = cands.front().l;
    double best_t = cands.front().t;
    for (const Cand &c : cands)
        if (c.t < best_t) {
            best_t = c.t;
            best = c.l;
        }
    set_layout(best.rows, best.order, best.threads, best.nt, best.block, best.xs);
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tuned[key()] = best;
    return MXS_OK;
}

mxs_status check_coe(const double *coe, int ncoe) {
    if (ncoe < 0 || ncoe > kMaxCoe)
        return fail(MXS_ERR_UNSUPPORTED, "ncoe=%d outside 0..%d", ncoe, kMaxCoe);
    if (ncoe > 0 && !coe) return fail(MXS_ERR_INVALID_ARG, "coe is NULL with ncoe=%d", ncoe);
    return MXS_OK;
}

bool valid_dtype(int d) { return d == F64 || d == F32 || d == BF16; }

}  // namespace mxs

using namespace mxs;

extern "C" {

mxs_status mxs_create_2d(const mxs_stencil2d_desc *d, mxs_plan *plan) {
    if (!plan) return fail(MXS_ERR_INVALID_ARG, "plan output pointer is NULL");
    *plan = nullptr;
    if (!d) return fail(MXS_ERR_INVALID_ARG, "descriptor is NULL");
    if (d->nx <= 0 || d->ny <= 0 || d->ld < d->nx)
        return fail(MXS_ERR_INVALID_ARG, "need nx > 0, ny > 0, ld >= nx (got %d, %d, %lld)", d->nx,
                    d->ny, d->ld);
    if (d->dir != MXS_X && d->dir != MXS_Y && d->dir != MXS_XY)
        return fail(MXS_ERR_INVALID_ARG, "dir must be MXS_X, MXS_Y or MXS_XY");
    if (d->bc != MXS_NP && d->bc != MXS_P) return fail(MXS_ERR_INVALID_ARG, "bc must be MXS_NP or MXS_P");
    if (!valid_dtype(d->dtype)) return fail(MXS_ERR_INVALID_ARG, "unknown dtype %d", d->dtype);
    if (d->left < 0 || d->right < 0 || d->top < 0 || d->bottom < 0)
        return fail(MXS_ERR_INVALID_ARG, "negative stencil extent");
    if (d->dir == MXS_X && (d->top || d->bottom))
        return fail(MXS_ERR_INVALID_ARG, "an X stencil needs top = bottom = 0");
    if (d->dir == MXS_Y && (d->left || d->right))
        return fail(MXS_ERR_INVALID_ARG, "a Y stencil needs left = right = 0");
    if (d->left + d->right >= d->nx || d->top + d->bottom >= d->ny)
        return fail(MXS_ERR_INVALID_ARG, "stencil extents must be smaller than the grid");
    if (!d->weights) return fail(MXS_ERR_INVALID_ARG, "weights is NULL");
    mxs_status st = check_coe(d->coe, d->ncoe);
    if (st) return st;
    const int wx = d->left + d->right + 1, wy = d->top + d->bottom + 1;
    const int nwx = bucket_width(wx), nwy = bucket_width(wy);
    if (!nwx || !nwy || (nwx > 1 && nwy > 1 && (nwx > MXS_MAX_TAPS_XY || nwy > MXS_MAX_TAPS_XY)))
        return fail(MXS_ERR_UNSUPPORTED, "window %d x %d exceeds the supported sizes", wx, wy);

    Stencil2DPlan *p = new (std::nothrow) Stencil2DPlan();
    if (!p) return fail(MXS_ERR_OOM, "host allocation failed");
    p->dtype = d->dtype;
    p->nwx = nwx;
    p->nwy = nwy;
    p->a.nx = d->nx;
    p->a.ny = d->ny;
    p->a.ld = d->ld;
    p->a.L = d->left;
    p->a.R = d->right;
    p->a.T = d->top;
    p->a.B = d->bottom;
    p->a.periodic = d->bc == MXS_P;
    p->a.ncoe = d->ncoe;
    for (int m = 0; m < d->ncoe; ++m) {
        p->a.coe_d[m] = d->coe[m];
        p->a.coe_f[m] = static_cast<float>(d->coe[m]);
    }
    if ((st = p->set_io(d->in, d->out))) {
        delete p;
        return st;
    }
    p->default_layout();
    if (stencil2d_lds_bytes(p->dtype, nwx, nwy, p->threads, 0, 0) > static_cast<size_t>(device_lds_limit())) {
        delete p;
        return fail(MXS_ERR_UNSUPPORTED, "window needs more LDS than the device offers");
    }
    hipError_t e = upload_weights(p->wts, d->weights, d->left, d->right, d->top, d->bottom, nwx,
                                  nwy, p->dtype);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "weights upload");
    }
    p->a.wts = p->wts.ptr;
    p->a.wts_up = static_cast<const char *>(p->wts.ptr) +
                  static_cast<size_t>(nwx) * nwy * (p->dtype == F64 ? sizeof(double) : sizeof(float));
    register_plan(p);
    *plan = p;
    return MXS_OK;
}

mxs_status mxs_create_1d_batch(int nbatch, const long long *offsets, int bc, int dtype, int left,
                               int right, const double *weights, const double *coe, int ncoe,
                               const void *in, void *out, mxs_plan *plan) {
    if (!plan) return fail(MXS_ERR_INVALID_ARG, "plan output pointer is NULL");
    *plan = nullptr;
    if (nbatch <= 0 || !offsets) return fail(MXS_ERR_INVALID_ARG, "need nbatch > 0 and host offsets");
    if (bc != MXS_NP && bc != MXS_P) return fail(MXS_ERR_INVALID_ARG, "bc must be MXS_NP or MXS_P");
    if (!valid_dtype(dtype)) return fail(MXS_ERR_INVALID_ARG, "unknown dtype %d", dtype);
    if (left < 0 || right < 0) return fail(MXS_ERR_INVALID_ARG, "negative stencil extent");
    if (!weights) return fail(MXS_ERR_INVALID_ARG, "weights is NULL");
    mxs_status st = check_coe(coe, ncoe);
    if (st) return st;
    const int nwx = bucket_width(left + right + 1);
    if (!nwx) return fail(MXS_ERR_UNSUPPORTED, "window of %d taps is too wide", left + right + 1);
    if (offsets[0] != 0) return fail(MXS_ERR_INVALID_ARG, "offsets[0] must be 0");
    for (int b = 0; b < nbatch; ++b)
        if (offsets[b + 1] - offsets[b] <= left + right)
            return fail(MXS_ERR_INVALID_ARG, "signal %d has length %lld <= left+right", b,
                        offsets[b + 1] - offsets[b]);
    const long long total = offsets[nbatch];
    if (total >= (1LL << 40)) return fail(MXS_ERR_UNSUPPORTED, "batch too large");

    Stencil1DPlan *p = new (std::nothrow) Stencil1DPlan();
    if (!p) return fail(MXS_ERR_OOM, "host allocation failed");
    p->dtype = dtype;
    p->nwx = nwx;
    p->a.total = total;
    p->a.nbatch = nbatch;
    p->a.L = left;
    p->a.R = right;
    p->a.periodic = bc == MXS_P;
    p->a.ncoe = ncoe;
    for (int m = 0; m < ncoe; ++m) {
        p->a.coe_d[m] = coe[m];
        p->a.coe_f[m] = static_cast<float>(coe[m]);
    }
    if ((st = p->set_io(in, out))) {
        delete p;
        return st;
    }
    const int W = p->threads * vec_elems(dtype) * kS1dVecs;
    const long long ntiles = (total + W - 1) / W;
    if (ntiles >= (1LL << 31)) {
        delete p;
        return fail(MXS_ERR_UNSUPPORTED, "batch too large");
    }
    p->a.ntiles = static_cast<int>(ntiles);
    // first signal of every tile: the signal holding element min(t*W, total-1)
    std::vector<int> tf(static_cast<size_t>(ntiles) + 1);
    int b = 0, maxsig = 0;
    for (long long t = 0; t <= ntiles; ++t) {
        const long long e = std::min(t * W, total - 1);
        while (offsets[b + 1] <= e) ++b;
        tf[t] = b;
        if (t > 0) maxsig = std::max(maxsig, tf[t] - tf[t - 1] + 2);
    }
    p->a.max_sig_per_tile = std::max(maxsig, 2);
    if (stencil1d_lds_bytes(dtype, nwx, p->threads, p->a.max_sig_per_tile) >
        static_cast<size_t>(device_lds_limit())) {
        delete p;
        return fail(MXS_ERR_UNSUPPORTED, "signals too short for the LDS budget");
    }
    hipError_t e;
    if ((e = p->offsets.upload(offsets, sizeof(long long) * (nbatch + 1))) != hipSuccess ||
        (e = p->tile_first.upload(tf.data(), sizeof(int) * tf.size())) != hipSuccess ||
        (e = upload_weights(p->wts, weights, left, right, 0, 0, nwx, 1, dtype)) != hipSuccess) {
        delete p;
        return hip_fail(e, "batch tables upload");
    }
    p->a.offsets = static_cast<const long long *>(p->offsets.ptr);
    p->a.tile_first = static_cast<const int *>(p->tile_first.ptr);
    p->a.wts = p->wts.ptr;
    p->grid = static_cast<int>(ntiles);
    register_plan(p);
    *plan = p;
    return MXS_OK;
}

mxs_status mxs_compute(mxs_plan plan, void *hip_stream) {
    if (!plan || !is_live(plan)) return fail(MXS_ERR_BAD_HANDLE, "invalid plan");
    return plan->compute(static_cast<hipStream_t>(hip_stream));
}

mxs_status mxs_swap(mxs_plan plan) {
    if (!plan || !is_live(plan)) return fail(MXS_ERR_BAD_HANDLE, "invalid plan");
    return plan->swap();
}

mxs_status mxs_set_io(mxs_plan plan, const void *in, void *out) {
    if (!plan || !is_live(plan)) return fail(MXS_ERR_BAD_HANDLE, "invalid plan");
    return plan->rebind(in, out);
}

mxs_status mxs_autotune(mxs_plan plan, void *hip_stream) {
    if (!plan || !is_live(plan)) return fail(MXS_ERR_BAD_HANDLE, "invalid plan");
    return plan->autotune(static_cast<hipStream_t>(hip_stream));
}

mxs_status mxs_plan_info(mxs_plan plan, char *buf, int len) {
    if (!plan || !is_live(plan)) return fail(MXS_ERR_BAD_HANDLE, "invalid plan");
    if (!buf || len <= 0) return fail(MXS_ERR_INVALID_ARG, "need a buffer");
    plan->info(buf, len);
    return MXS_OK;
}

mxs_status mxs_destroy(mxs_plan plan) {
    if (!plan) return MXS_OK;
    if (!unregister_plan(plan)) return fail(MXS_ERR_BAD_HANDLE, "plan already destroyed or unknown");
    delete plan;
    return MXS_OK;
}

const char *mxs_last_error(void) { return g_err.c_str(); }

const char *mxs_status_string(mxs_status st) {
    switch (st) {
    case MXS_OK: return "MXS_OK";
    case MXS_ERR_INVALID_ARG: return "MXS_ERR_INVALID_ARG";
    case MXS_ERR_ALIAS: return "MXS_ERR_ALIAS";
    case MXS_ERR_UNSUPPORTED: return "MXS_ERR_UNSUPPORTED";
    case MXS_ERR_HIP: return "MXS_ERR_HIP";
    case MXS_ERR_OOM: return "MXS_ERR_OOM";
    case MXS_ERR_NONFINITE: return "MXS_ERR_NONFINITE";
    case MXS_ERR_BAD_HANDLE: return "MXS_ERR_BAD_HANDLE";
    default: return "MXS_ERR_UNKNOWN";
    }
}

int mxs_version(void) { return 100; }

}  // extern "C"
