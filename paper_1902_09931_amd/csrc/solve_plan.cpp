// Plan for batched cyclic banded solves (mxs_create_cyclic_solve).
#include "plans.h"
#include "solve.h"

#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <numeric>
#include <vector>

namespace mxs {

int device_lds_per_cu() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
            hipSuccess || v <= 0)
        return 65536;
    return v;
}

// Persistent grid for one-wavefront-per-line kernels: as many blocks as the
// LDS of the device holds at once, at most one per line.
int wave_grid(long long nlines, size_t lds_bytes) {
    const long long per_cu = std::max<long long>(1, std::min<long long>(16, device_lds_per_cu() / std::max<size_t>(lds_bytes, 1)));
    return static_cast<int>(std::max<long long>(1, std::min<long long>(nlines, per_cu * device_cu_count())));
}

namespace {

struct SolvePlan final : mxs_plan_s {
    int geometry = 0, bw = 1, dtype = F64;
    CyclicFactor f;
    // ragged
    RaggedLines rl{};
    DevBuf offsets, order, units;
    // rows / cols: the instance table of the current (rhs, x) pair in
    // tables[cur], of the swapped pair in tables[1 - cur]; both are uploaded
    // when the pointers are set, so that compute() only launches (it can be
    // captured into a graph) and swap() only flips cur
    RowsInst rows{};
    ColsInst cols{};
    DevBuf tables[2], carry, pow;
    int cur = 0;
    // register kernel classes (blocks per line, first line, line count), for
    // plan_info; ragged lines longer than kWaveLineMax (the first nlong in
    // sorted order) go to the LDS kernel, the others to one launch of the
    // work-unit kernel
    struct WaveRange {
        int nb, first, count;
    };
    std::vector<WaveRange> wave;
    int nunits = 0;
    int nlong = 0;
    int nlines = 0, grid = 1, blocksAC = 0, blocksB = 0, nw = 1, bgroups = 16;
    size_t lds = 0, bytes = 0;
    SolvePlan() : mxs_plan_s(KIND_SOLVE) {}

    // Upload the instance tables of (rhs, x) and of the swapped pair
    // (synchronous copies from host memory, before any launch uses them).
    hipError_t upload_tables(const void *rhs, void *x) {
        for (int k = 0; k < 2; ++k) {
            const void *in = k == 0 ? rhs : x;
            void *out = k == 0 ? x : const_cast<void *>(rhs);
            hipError_t e;
            if (geometry == MXS_LINES_ROWS) {
                RowsInst ri = rows;
                ri.in = in;
                ri.out = out;
                e = tables[k].upload(&ri, sizeof ri);
            } else {
                ColsInst ci = cols;
                ci.rhs = in;
                ci.x = out;
                e = tables[k].upload(&ci, sizeof ci);
            }
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }

    mxs_status set_io(const void *rhs, void *x) {
        if (!rhs || !x) return fail(MXS_ERR_INVALID_ARG, "rhs/x must be device pointers");
        if (rhs != x && ranges_overlap(rhs, bytes, x, bytes))
            return fail(MXS_ERR_ALIAS, "rhs and x overlap without being the same buffer");
        if (geometry != MXS_LINES_RAGGED) {
            hipError_t e = upload_tables(rhs, x);
            if (e != hipSuccess) return hip_fail(e, "solve table upload");
        }
        rl.in = rhs;
        rl.out = x;
        rows.in = rhs;
        rows.out = x;
        cols.rhs = rhs;
        cols.x = x;
        cur = 0;
        return MXS_OK;
    }

    mxs_status compute(hipStream_t s) override {
        hipError_t e = hipSuccess;
        if (geometry == MXS_LINES_RAGGED) {
            if (nlong > 0) e = launch_ragged_lines(dtype, bw, rl, nw, grid, lds, s);
            if (per_class) {
                for (size_t q = 0; q < wave.size() && e == hipSuccess; ++q)
                    e = launch_wave_ragged(dtype, bw, wave[q].nb, rl, wave[q].first, wave[q].count, s);
            } else if (e == hipSuccess && nunits > 0) {
                e = launch_wave_units(dtype, bw, rl, static_cast<const WaveUnit *>(units.ptr), nunits, s);
            }
        } else if (geometry == MXS_LINES_ROWS) {
            const RowsInst *ti = static_cast<const RowsInst *>(tables[cur].ptr);
            if (!wave.empty())
                e = launch_wave_rows(dtype, bw, wave[0].nb, ti, nullptr, 0, nlines, s);
            else
                e = launch_rows(dtype, bw, ti, nullptr, nlines, nw, grid, lds, s);
        } else {
            e = launch_cols(dtype, dtype, bw, 0, static_cast<const ColsInst *>(tables[cur].ptr), nullptr,
                            nullptr, blocksAC, blocksB, bgroups, s);
        }
        return e == hipSuccess ? MXS_OK : hip_fail(e, "cyclic solve launch");
    }
    mxs_status swap() override {
        const void *r = rl.in;
        rl.in = rl.out;
        rl.out = const_cast<void *>(r);
        rows.in = rl.in;
        rows.out = rl.out;
        cols.rhs = rl.in;
        cols.x = rl.out;
        cur = 1 - cur;
        return MXS_OK;
    }
    mxs_status rebind(const void *in, void *out) override { return set_io(in, out); }

    long long nmax = 0;   // longest line (ragged, rows)

    void set_waves(int w) {
        nw = w;
        lds = line_lds_bytes(nmax, nw);
        grid = wave_grid(std::max(1, geometry == MXS_LINES_RAGGED ? nlong : nlines), lds);
    }

    // Ragged lines of at most 4096 elements go out either in one launch
    // (work-unit table; the kernel holds the registers of the largest class)
    // or in one launch per length class (each with its own registers).
    bool per_class = false;
    double tuned_units = 0, tuned_classes = 0;

    // The form of the ragged register lines, and wavefronts per line of the
    // LDS kernel: one (long chunks, few barriers) to four (more loads in
    // flight per line); chosen by timing.
    mxs_status autotune(hipStream_t s) override {
        auto timed = [&] {
            return time_launches([&] { return compute(s) == MXS_OK ? hipSuccess : hipErrorLaunchFailure; }, s, 2, 5);
        };
        if (geometry == MXS_LINES_RAGGED && nunits > 0 && wave.size() > 1) {
            double t[2] = {1e30, 1e30};
            for (int pass = 0; pass < 2; ++pass)
                for (int f = 0; f < 2; ++f) {
                    per_class = f == 1;
                    const double v = timed();
                    if (v < 0) {
                        per_class = false;
                        return fail(MXS_ERR_HIP, "autotune launch failed");
                    }
                    t[f] = std::min(t[f], v);
                }
            per_class = t[1] < t[0];
            tuned_units = t[0];
            tuned_classes = t[1];
        }
        // only the LDS kernel has a shape to choose
        if (geometry == MXS_LINES_COLS || (geometry == MXS_LINES_RAGGED ? nlong == 0 : !wave.empty()))
            return MXS_OK;
        const int start = nw;
        int best = nw;
        double best_t = 1e30;
        for (int w : {1, 2, 4}) {
            if (line_lds_bytes(nmax, w) > static_cast<size_t>(device_lds_limit())) continue;
            set_waves(w);
            const double t = time_launches([&] {
                return compute(s) == MXS_OK ? hipSuccess : hipErrorLaunchFailure;
            }, s, 1, 3);
            if (t < 0) {
                set_waves(start);
                return fail(MXS_ERR_HIP, "autotune launch failed");
            }
            if (t < best_t) {
                best_t = t;
                best = w;
            }
        }
        set_waves(best);
        return MXS_OK;
    }
    void info(char *buf, int len) const override {
        int n = snprintf(buf, len, "cyclic_solve geometry=%d bw=%d dtype=%d", geometry, bw, dtype);
        const bool lds_kernel = geometry == MXS_LINES_RAGGED ? nlong > 0 : wave.empty();
        if (geometry != MXS_LINES_COLS && lds_kernel && n < len)
            n += snprintf(buf + n, len - n, " lds_kernel_lines=%d waves_per_line=%d grid=%d lds=%zu",
                          geometry == MXS_LINES_RAGGED ? nlong : nlines, nw, grid, lds);
        if (geometry == MXS_LINES_RAGGED && nunits > 0 && n < len)
            n += snprintf(buf + n, len - n, " form=%s launches=%d units=%d", per_class ? "classes" : "units",
                          (nlong > 0) + (per_class ? static_cast<int>(wave.size()) : 1), nunits);
        if (tuned_units > 0 && n < len)
            n += snprintf(buf + n, len - n, " tuned_us_units=%.1f tuned_us_classes=%.1f", tuned_units * 1e6,
                          tuned_classes * 1e6);
        for (size_t q = 0; q < wave.size() && n < len; ++q)
            n += snprintf(buf + n, len - n, " register_kernel(nb=%d lines=%d)", wave[q].nb, wave[q].count);
    }
};

}  // namespace
}  // namespace mxs

using namespace mxs;

extern "C" mxs_status mxs_create_cyclic_solve(int bw, const double *coef, int geometry, int nx,
                                              int ny, long long ld, int nbatch,
                                              const long long *offsets, int dtype,
                                              const void *rhs, void *x, mxs_plan *plan) {
    if (!plan) return fail(MXS_ERR_INVALID_ARG, "plan output pointer is NULL");
    *plan = nullptr;
    if (bw != 1 && bw != 2) return fail(MXS_ERR_INVALID_ARG, "bw must be 1 or 2");
    if (!coef) return fail(MXS_ERR_INVALID_ARG, "coef is NULL");
    if (!valid_dtype(dtype)) return fail(MXS_ERR_INVALID_ARG, "unknown dtype %d", dtype);
    if (geometry != MXS_LINES_RAGGED && geometry != MXS_LINES_ROWS && geometry != MXS_LINES_COLS)
        return fail(MXS_ERR_INVALID_ARG, "unknown geometry %d", geometry);
    const int minlen = 2 * bw + 1;
    constexpr long long kMaxLine = 16384;

    SolvePlan *p = new (std::nothrow) SolvePlan();
    if (!p) return fail(MXS_ERR_OOM, "host allocation failed");
    p->geometry = geometry;
    p->bw = bw;
    p->dtype = dtype;
    const int fst = factor_symmetric_circulant(bw, coef, &p->f);
    if (fst) {
        delete p;
        return fst == -2 ? fail(MXS_ERR_UNSUPPORTED, "the circulant is not symmetric positive definite")
                         : fail(MXS_ERR_INVALID_ARG, "invalid band coefficients");
    }
    mxs_status st;
    hipError_t e = hipSuccess;
    if (geometry != MXS_LINES_COLS) {
        std::vector<double> pt(4 * kPowEntries);
        fill_pow_table(p->f, bw, pt.data());
        if ((e = p->pow.upload(pt.data(), sizeof(double) * pt.size())) != hipSuccess) {
            delete p;
            return hip_fail(e, "power table upload");
        }
        p->rl.pow = static_cast<const double *>(p->pow.ptr);
        p->rows.pow = p->rl.pow;
    }
    if (geometry == MXS_LINES_RAGGED) {
        if (nbatch <= 0 || !offsets) {
            delete p;
            return fail(MXS_ERR_INVALID_ARG, "ragged lines need nbatch > 0 and host offsets");
        }
        if (offsets[0] != 0) {
            delete p;
            return fail(MXS_ERR_INVALID_ARG, "offsets[0] must be 0");
        }
        long long nmax = 0;
        std::vector<long long> len(nbatch);
        for (int b = 0; b < nbatch; ++b) {
            len[b] = offsets[b + 1] - offsets[b];
            if (len[b] < minlen || len[b] > kMaxLine) {
                delete p;
                return fail(len[b] < minlen ? MXS_ERR_INVALID_ARG : MXS_ERR_UNSUPPORTED,
                            "line %d has length %lld outside [%d, %lld]", b, len[b], minlen, kMaxLine);
            }
            nmax = std::max(nmax, len[b]);
        }
        p->bytes = static_cast<size_t>(offsets[nbatch]) * dtype_size(dtype);
        if ((st = p->set_io(rhs, x))) {
            delete p;
            return st;
        }
        std::vector<int> order(nbatch);
        std::iota(order.begin(), order.end(), 0);
        // lines longer than the register kernel holds first, longest first
        // (load balance of the persistent LDS kernel); then the register
        // classes, largest first, each in memory order (neighbouring
        // wavefronts read neighbouring lines)
        auto lclass = [&](int k) { return len[k] > kWaveLineMax ? 32 : wave_nb(len[k]); };
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            const int ca = lclass(a), cb = lclass(b);
            if (ca != cb) return ca > cb;
            return ca == 32 && len[a] > len[b];
        });
        if ((e = p->offsets.upload(offsets, sizeof(long long) * (nbatch + 1))) != hipSuccess ||
            (e = p->order.upload(order.data(), sizeof(int) * nbatch)) != hipSuccess) {
            delete p;
            return hip_fail(e, "line tables upload");
        }
        // lines longer than kWaveLineMax to the LDS kernel, the rest by
        // register-block class (each class is one range of the order)
        p->nlong = 0;
        if (force_lds_lines()) {
            p->nlong = nbatch;
        } else {
            while (p->nlong < nbatch && len[order[p->nlong]] > kWaveLineMax) ++p->nlong;
            for (int q = p->nlong; q < nbatch;) {
                const int nb = wave_nb(len[order[q]]);
                int r = q;
                while (r < nbatch && wave_nb(len[order[r]]) == nb) ++r;
                p->wave.push_back({nb, q, r - q});
                q = r;
            }
        }
        // work units: consecutive lines of one class, kWaveNBMax / nb of
        // them (the last unit of a class may hold fewer), largest class first
        std::vector<WaveUnit> units;
        for (const auto &w : p->wave) {
            const int per = kWaveNBMax / w.nb;
            for (int q = 0; q < w.count; q += per)
                units.push_back({w.first + q, std::min(per, w.count - q), w.nb, 0});
        }
        p->nunits = static_cast<int>(units.size());
        // MXS_RAGGED_FORM=classes starts the plan with one launch per class
        if (const char *env = getenv("MXS_RAGGED_FORM")) p->per_class = env[0] == 'c';
        if (!units.empty() &&
            (e = p->units.upload(units.data(), sizeof(WaveUnit) * units.size())) != hipSuccess) {
            delete p;
            return hip_fail(e, "line tables upload");
        }
        p->rl.offsets = static_cast<const long long *>(p->offsets.ptr);
        p->rl.order = static_cast<const int *>(p->order.ptr);
        p->rl.nlines = p->nlong;
        p->rl.p1 = p->f.p1;
        p->rl.p2 = bw == 2 ? p->f.p2 : 0.0;
        p->rl.invK = p->f.invK;
        p->nmax = nmax;
        p->set_waves(line_waves(nmax));
    } else {
        if (nx <= 0 || ny <= 0 || ld < nx) {
            delete p;
            return fail(MXS_ERR_INVALID_ARG, "need nx, ny > 0 and ld >= nx");
        }
        const long long n = geometry == MXS_LINES_ROWS ? nx : ny;
        if (n < minlen || (geometry == MXS_LINES_ROWS && n > kMaxLine)) {
            delete p;
            return fail(n < minlen ? MXS_ERR_INVALID_ARG : MXS_ERR_UNSUPPORTED,
                        "line length %lld outside [%d, %lld]", n, minlen, kMaxLine);
        }
        p->bytes = grid_bytes(nx, ny, ld, dtype);
        if (geometry == MXS_LINES_ROWS) {
            p->rows.ld = ld;
            p->rows.nx = nx;
            p->rows.ny = ny;
            p->rows.line0 = 0;
            p->rows.p1 = p->f.p1;
            p->rows.p2 = bw == 2 ? p->f.p2 : 0.0;
            p->rows.invK = p->f.invK;
            p->nlines = ny;
            p->nmax = nx;
            if (nx <= kWaveLineMax && !force_lds_lines()) p->wave.push_back({wave_nb(nx), 0, ny});
            p->set_waves(line_waves(nx));
        } else {
            fill_cols_coef(p->f, bw, ny, &p->cols);
            p->cols.ld = ld;
            p->cols.nx = nx;
            p->cols.ny = ny;
            p->cols.nstrips = (nx + kColsThreads - 1) / kColsThreads;
            p->cols.blk0 = 0;
            p->cols.blkB0 = 0;
            p->blocksAC = p->cols.nstrips * p->cols.nseg;
            p->bgroups = cols_b_groups((ny + kSeg - 1) / kSeg);
            p->blocksB = (nx + cols_b_cols(p->bgroups) - 1) / cols_b_cols(p->bgroups);
            e = p->carry.alloc(sizeof(double) * 4 * static_cast<size_t>(nx) * p->cols.nseg);
            p->cols.carry = static_cast<double *>(p->carry.ptr);
        }
        if (e != hipSuccess) {
            delete p;
            return hip_fail(e, "solve scratch allocation");
        }
        // the instance tables, now that every field but the pointers is set
        if ((st = p->set_io(rhs, x))) {
            delete p;
            return st;
        }
    }
    if (p->lds > static_cast<size_t>(device_lds_limit())) {
        delete p;
        return fail(MXS_ERR_UNSUPPORTED, "line too long for the LDS of one workgroup");
    }
    register_plan(p);
    *plan = p;
    return MXS_OK;
}
