// Plan of the WENO advection variant (Sec. 4.3): mxs_create_weno_adv, then
// the common mxs_compute / mxs_swap / mxs_set_io / mxs_autotune /
// mxs_destroy calls.
#include "plans.h"
#include "weno.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

namespace mxs {

namespace {

bool aligned16(const void *p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; }

struct WenoPlan final : mxs_plan_s {
    WenoArgs a{};
    int threads = 256;
    WenoPlan() : mxs_plan_s(KIND_WENO) {}

    void set_layout(int rows, int order, int nthreads, int nt) {
        threads = nthreads;
        a.rows = rows;
        a.order = order;
        a.nt_store = nt;
        const int W = 2 * threads;
        a.nstrips = (a.nx + W - 1) / W;
        a.nchunks = (a.ny + rows - 1) / rows;
    }

    mxs_status set_io(const void *phi, void *out) {
        if (!phi || !out) return fail(MXS_ERR_INVALID_ARG, "phi and out must be device pointers");
        const size_t bytes = grid_bytes(a.nx, a.ny, a.ld, F64);
        if (ranges_overlap(phi, bytes, out, bytes) || ranges_overlap(a.u, bytes, out, bytes) ||
            ranges_overlap(a.v, bytes, out, bytes))
            return fail(MXS_ERR_ALIAS, "out overlaps an input");
        a.phi = phi;
        a.out = out;
        a.vec_ok = a.ld % 2 == 0 && aligned16(phi) && aligned16(out) && aligned16(a.u) && aligned16(a.v);
        return MXS_OK;
    }

    mxs_status compute(hipStream_t s) override {
        hipError_t e = launch_weno_adv(a, threads, s);
        return e == hipSuccess ? MXS_OK : hip_fail(e, "WENO advection launch");
    }
    mxs_status swap() override {
        const void *tmp = a.phi;
        a.phi = a.out;
        a.out = const_cast<void *>(tmp);
        return MXS_OK;
    }
    mxs_status rebind(const void *in, void *out) override { return set_io(in, out); }

    // Output rows per workgroup, threads, tile order and store kind, timed as
    // the 2D stencil layouts are (cold memory-side cache for grids between
    // half and four times its size).
    mxs_status autotune(hipStream_t s) override {
        struct Cand {
            int rows, order, threads, nt;
            double t;
        };
        std::vector<Cand> cands;
        for (int rows : {4, 8})
            for (int nthreads : {256, 128})
                for (int order : {1, 0})
                    for (int nt : {1, 0})
                        if (weno_lds_bytes(rows, nthreads) <= static_cast<size_t>(device_lds_limit()))
                            cands.push_back({rows, order, nthreads, nt, 1e30});
        const Cand start{a.rows, a.order, threads, a.nt_store, 0};
        const size_t data = 4 * grid_bytes(a.nx, a.ny, a.ld, F64);
        DevBuf flush;
        if (data > kMallBytes / 2 && data < 4 * kMallBytes && flush.alloc(kFlushBytes) != hipSuccess) {
            (void)hipGetLastError();
            flush.bytes = 0;
        }
        for (int pass = 0; pass < 2; ++pass)
            for (Cand &c : cands) {
                set_layout(c.rows, c.order, c.threads, c.nt);
                auto launch = [&] { return launch_weno_adv(a, threads, s); };
                const double t = flush.bytes ? time_launches_cold(launch, s, 1, 5, flush.ptr, flush.bytes)
                                             : time_launches(launch, s, 2, 5);
                if (t < 0) {
                    set_layout(start.rows, start.order, start.threads, start.nt);
                    return hip_fail(hipGetLastError(), "autotune launch");
                }
                c.t = std::min(c.t, t);
            }
        const Cand *best = &cands.front();
        for (const Cand &c : cands)
            if (c.t < best->t) best = &c;
        set_layout(best->rows, best->order, best->threads, best->nt);
        return MXS_OK;
    }

    void info(char *buf, int len) const override {
        snprintf(buf, len, "weno_adv rows=%d order=%d threads=%d nt_store=%d grid=%d", a.rows, a.order, threads,
                 a.nt_store, a.nstrips * a.nchunks);
    }
};

}  // namespace
}  // namespace mxs

using namespace mxs;

extern "C" {

mxs_status mxs_create_weno_adv(int nx, int ny, long long ld, double dx, double dy, int dtype,
                               const void *phi, const void *u, const void *v, void *out, mxs_plan *plan) {
    if (!plan) return fail(MXS_ERR_INVALID_ARG, "plan output pointer is NULL");
    *plan = nullptr;
    if (nx < 6 || ny < 6 || ld < nx)
        return fail(MXS_ERR_INVALID_ARG, "need nx, ny >= 6 and ld >= nx (got %d, %d, %lld)", nx, ny, ld);
    if (!(dx > 0) || !(dy > 0) || !std::isfinite(dx) || !std::isfinite(dy))
        return fail(MXS_ERR_INVALID_ARG, "need positive finite dx, dy");
    if (!valid_dtype(dtype)) return fail(MXS_ERR_INVALID_ARG, "unknown dtype %d", dtype);
    if (dtype != F64) return fail(MXS_ERR_UNSUPPORTED, "the WENO advection variant is double precision only");
    if (!u || !v) return fail(MXS_ERR_INVALID_ARG, "u and v must be device pointers");
    WenoPlan *p = new (std::nothrow) WenoPlan();
    if (!p) return fail(MXS_ERR_OOM, "host allocation failed");
    p->a.nx = nx;
    p->a.ny = ny;
    p->a.ld = ld;
    p->a.rdx = 1.0 / dx;
    p->a.rdy = 1.0 / dy;
    p->a.u = u;
    p->a.v = v;
    mxs_status st = p->set_io(phi, out);
    if (st) {
        delete p;
        return st;
    }
    p->set_layout(8, 1, 256, 1);
    // explicit layout "rows,order,threads,nt" for experiments and tests
    if (const char *env = getenv("MXS_WENO_TILE")) {
        int r = 0, o = 0, t = 0, nt = 1;
        if (sscanf(env, "%d,%d,%d,%d", &r, &o, &t, &nt) >= 3 && weno_rows_ok(r) && (o == 0 || o == 1) &&
            (t == 64 || t == 128 || t == 256))
            p->set_layout(r, o, t, nt != 0);
    }
    register_plan(p);
    *plan = p;
    return MXS_OK;
}

}  // extern "C"
