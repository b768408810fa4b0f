// Plans for the ADI Cahn-Hilliard step on one grid or an ensemble of grids
// (Sec. 5.1): mxs_ch_create, mxs_ch_ensemble_create, mxs_ch_step and friends.
//
// One step is five launches, each covering every instance of the plan:
//   1. right-hand side R from (C^{n-1}, C^n)                   (ch.hip)
//   2. L_x w = R on every row, in place                        (cyclic.hip)
//   3-5. L_y v = w on every column, three phases, the last one
//        writing C^{n+1} = 2 C^n - C^{n-1} + v                  (cyclic.hip)
// In the fused mode steps 1 and 2 are one launch per register class of the
// rows (chrows.hip): each workgroup forms R of a few rows in registers and
// solves them, and R never goes to memory.
// The three state buffers rotate, so the kernel arguments differ between
// consecutive steps; the plan keeps one instance table (and one captured
// HIP graph) per rotation.
#include "ch.h"
#include "diag.h"
#include "persist.h"
#include "plans.h"
#include "solve.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <vector>

namespace mxs {

int wave_grid(long long nlines, size_t lds_bytes);

namespace {

struct Inst {
    int nx, ny;
    double dx, dy, dt;
    void *buf[3];     // caller's buffers in the initial roles prev, cur, next
    DevBuf w, carry;  // plan-owned
};

// The 5x5 biharmonic window d_xxxx + 2 d_xxyy + d_yyyy from the second-order
// central differences (Sec. 5.1) and the cross stencil of Fig. 1.
void biharmonic_window(double dx, double dy, double *w) {
    const double d4[5] = {1.0, -4.0, 6.0, -4.0, 1.0};
    const double d2[3] = {1.0, -2.0, 1.0};
    for (int k = 0; k < 25; ++k) w[k] = 0.0;
    const double hx = 1.0 / (dx * dx * dx * dx), hy = 1.0 / (dy * dy * dy * dy);
    const double hxy = 1.0 / (dx * dx * dy * dy);
    for (int k = 0; k < 5; ++k) {
        w[2 * 5 + k] += d4[k] * hx;
        w[k * 5 + 2] += d4[k] * hy;
    }
    for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) w[(b + 1) * 5 + (a + 1)] += 2.0 * d2[b] * d2[a] * hxy;
}

// The 3x3 window of the 5-point Laplacian.
void laplacian_window(double dx, double dy, double *w) {
    const double d2[3] = {1.0, -2.0, 1.0};
    for (int k = 0; k < 9; ++k) w[k] = 0.0;
    for (int k = 0; k < 3; ++k) {
        w[1 * 3 + k] += d2[k] / (dx * dx);
        w[k * 3 + 1] += d2[k] / (dy * dy);
    }
}

bool aligned16(const void *p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; }

struct CHPlan final : mxs_plan_s {
    int dtype = F64, wdtype = F64;
    double D = 1, gamma = 0.01;
    std::vector<Inst> inst;
    long long steps = 0;

    std::vector<RhsInst> rhs_h[3];
    std::vector<RowsInst> rows_h;
    std::vector<ColsInst> cols_h[3];
    std::vector<MassInst> mass_h[3];
    DevBuf rhs_d[3], rows_d, cols_d[3], mass_d[3];
    // instance of every workgroup (line for the row solves); unused for one grid
    DevBuf rhs_map, rows_map, colsAC_map, colsB_map, mass_map;
    // power tables of the row operators (register row kernel), one per instance
    DevBuf pows;
    // register row kernel: lines numbered by register class, one launch per
    // class; empty when the LDS kernel solves the rows
    struct RowRange {
        int nb, first, count;
    };
    std::vector<RowRange> row_ranges;
    DevBuf partial, mass_out;
    double *mass_host = nullptr;
    int bgroups = 16;   // phase B threads per column
    int rhs_blocks = 0, rhs_rows = 16, rhs_threads = kRhsThreads, row_lines = 0, row_grid = 1, row_nw = 1, colsAC = 0, colsB = 0,
        mass_blocks = 0, max_nx = 0;
    size_t row_lds = 0;

    hipStream_t cap = nullptr;
    hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};

    // persistent step (one cooperative launch per step): eligible when every
    // row fits register class kPersistNBMax; bar holds the grid barrier's
    // words (arrivals, generation, exits, error)
    bool persistent = false, persist_ok = false;
    // right-hand side formed inside the row solves (one launch per register
    // class of rows over groups of fused_rows rows, fused_cols columns per
    // thread and sub-block; shapes (4, 1), (8, 1), (4, 2)): eligible when
    // every row fits a register class; fused_work lists the row groups,
    // class by class
    bool fused = false, fused_ok = false;
    int fused_rows = 4, fused_cols = 1;
    DevBuf fused_work;
    std::vector<RowRange> fused_ranges;
    std::vector<int> class_order;   // instances ordered by register class of their rows

    // Row groups of wr rows for the fused form, in class order.
    hipError_t build_fused(int wr) {
        std::vector<RowGroup> work;
        fused_ranges.clear();
        for (int g : class_order) {
            const int nb = wave_nb(inst[g].nx);
            if (fused_ranges.empty() || fused_ranges.back().nb != nb)
                fused_ranges.push_back({nb, static_cast<int>(work.size()), 0});
            for (int j0 = 0; j0 < inst[g].ny; j0 += wr) work.push_back({g, j0});
            fused_ranges.back().count = static_cast<int>(work.size()) - fused_ranges.back().first;
        }
        fused_rows = wr;
        return fused_work.upload(work.data(), sizeof(RowGroup) * work.size());
    }
    int persist_grid = 0, persist_nbmax = 1, spin_limit = 1 << 22;
    DevBuf bar;

    CHPlan() : mxs_plan_s(KIND_CH) {}
    ~CHPlan() override {
        drop_graphs();
        if (cap) (void)hipStreamDestroy(cap);
        if (mass_host) (void)hipHostFree(mass_host);
        if (flag_host) (void)hipHostFree(flag_host);
    }
    unsigned *flag_host = nullptr;

    // Run steps as one persistent launch (on) or as the separate launches
    // (off); the right-hand side tables follow the workgroup size of the mode.
    mxs_status set_persistent(bool on, int rows) {
        if (on && !persist_ok) return fail(MXS_ERR_UNSUPPORTED, "this plan cannot run the persistent step");
        drop_graphs();
        persist_nograph = false;
        persistent = on;
        if (on) fused = false;
        if (on) rhs_threads = kPersistThreads;
        return build_rhs(rows);
    }

    int ninst() const { return static_cast<int>(inst.size()); }
    const int *map_of(const DevBuf &m) const {
        return ninst() > 1 ? static_cast<const int *>(m.ptr) : nullptr;
    }

    // Upload the instance index of every unit (workgroup or line), given the
    // number of units of each instance.
    static hipError_t upload_map(DevBuf &buf, const std::vector<int> &units_per_inst) {
        std::vector<int> m;
        for (size_t g = 0; g < units_per_inst.size(); ++g)
            m.insert(m.end(), units_per_inst[g], static_cast<int>(g));
        return buf.upload(m.data(), sizeof(int) * m.size());
    }

    hipError_t enqueue(int r, hipStream_t s) {
        if (persistent) {
            PersistArgs pa{};
            pa.rhs = static_cast<const RhsInst *>(rhs_d[r].ptr);
            pa.rhs_map = map_of(rhs_map);
            pa.rhs_blocks = rhs_blocks;
            pa.rows = static_cast<const RowsInst *>(rows_d.ptr);
            pa.rows_map = map_of(rows_map);
            pa.row_lines = row_lines;
            pa.cols = static_cast<const ColsInst *>(cols_d[r].ptr);
            pa.colsAC_map = map_of(colsAC_map);
            pa.colsB_map = map_of(colsB_map);
            pa.colsAC = colsAC;
            pa.colsB = colsB;
            pa.bgroups = bgroups;
            pa.bar = static_cast<unsigned *>(bar.ptr);
            pa.spin_limit = spin_limit;
            pa.stage_bytes = static_cast<int>(persist_stage_bytes(dtype, persist_nbmax));
            return launch_ch_persistent(dtype, persist_nbmax, pa, persist_grid, s);
        }
        const RowsInst *ri = static_cast<const RowsInst *>(rows_d.ptr);
        if (fused) {
            hipError_t e = hipSuccess;
            const RowGroup *work = static_cast<const RowGroup *>(fused_work.ptr);
            for (size_t q = 0; q < fused_ranges.size() && e == hipSuccess; ++q)
                e = launch_ch_rhs_rows(dtype, fused_rows, fused_cols, fused_ranges[q].nb,
                                       static_cast<const RhsInst *>(rhs_d[r].ptr), ri, work + fused_ranges[q].first,
                                       fused_ranges[q].count, s);
            if (e != hipSuccess) return e;
            return launch_cols(wdtype, dtype, 2, 1, static_cast<const ColsInst *>(cols_d[r].ptr),
                               map_of(colsAC_map), map_of(colsB_map), colsAC, colsB, bgroups, s);
        }
        hipError_t e = launch_ch_rhs(dtype, static_cast<const RhsInst *>(rhs_d[r].ptr),
                                     map_of(rhs_map), rhs_blocks, rhs_threads, s);
        if (e != hipSuccess) return e;
        if (row_ranges.empty())
            e = launch_rows(wdtype, 2, ri, map_of(rows_map), row_lines, row_nw, row_grid, row_lds, s);
        for (size_t q = 0; q < row_ranges.size() && e == hipSuccess; ++q)
            e = launch_wave_rows(wdtype, 2, row_ranges[q].nb, ri, map_of(rows_map), row_ranges[q].first,
                                 row_ranges[q].count, s);
        if (e != hipSuccess) return e;
        return launch_cols(wdtype, dtype, 2, 1, static_cast<const ColsInst *>(cols_d[r].ptr),
                           map_of(colsAC_map), map_of(colsB_map), colsAC, colsB, bgroups, s);
    }

    hipError_t capture(int r) {
        if (!cap) {
            hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
            if (e != hipSuccess) return e;
        }
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        hipError_t le = enqueue(r, cap);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cap, &graph);
        if (le != hipSuccess) e = le;
        if (e == hipSuccess) e = hipGraphInstantiate(&exec[r], graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        return e;
    }

    // set when the runtime cannot capture the cooperative launch of the
    // persistent step: its steps are then launched directly
    bool persist_nograph = false;

    mxs_status step(int nsteps, bool use_graph, hipStream_t s) {
        for (int k = 0; k < nsteps; ++k) {
            const int r = static_cast<int>(steps % 3);
            hipError_t e;
            if (use_graph && !(persistent && persist_nograph)) {
                if (!exec[r]) {
                    e = capture(r);
                    if (e != hipSuccess && persistent) {
                        (void)hipGetLastError();
                        persist_nograph = true;
                        drop_graphs();
                        --k;
                        continue;
                    }
                    if (e != hipSuccess) return hip_fail(e, "graph capture of the step");
                }
                e = hipGraphLaunch(exec[r], s);
            } else {
                e = enqueue(r, s);
            }
            if (e != hipSuccess) return hip_fail(e, "step launch");
            ++steps;
        }
        return MXS_OK;
    }

    mxs_status mass(double *out, hipStream_t s) {
        const int r = static_cast<int>(steps % 3);
        hipError_t e = launch_ch_mass(dtype, static_cast<const MassInst *>(mass_d[r].ptr),
                                      map_of(mass_map), ninst(), mass_blocks, static_cast<double *>(partial.ptr),
                                      static_cast<double *>(mass_out.ptr), s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(mass_host, mass_out.ptr, sizeof(double) * ninst(),
                               hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && bar.ptr)
            e = hipMemcpyAsync(flag_host, static_cast<unsigned *>(bar.ptr) + 3, sizeof(unsigned),
                               hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "mass reduction");
        if (bar.ptr && *flag_host) {
            *flag_host = 0;
            e = hipMemcpy(static_cast<unsigned *>(bar.ptr) + 3, flag_host, sizeof(unsigned), hipMemcpyHostToDevice);
            return fail(MXS_ERR_HIP, "a grid barrier of the persistent step timed out (workgroups not co-resident)%s",
                        e == hipSuccess ? "" : "; clearing the error word failed");
        }
        bool finite = true;
        for (int g = 0; g < ninst(); ++g) {
            out[g] = mass_host[g];
            finite = finite && std::isfinite(mass_host[g]);
        }
        return finite ? MXS_OK : fail(MXS_ERR_NONFINITE, "the mass is not finite");
    }

    // Coarsening diagnostics of instance k's C^n (Sec. 5.3).  The transform
    // scratch is allocated on the first call and kept by the plan, or, with
    // noalloc, taken from the library's static per-device scratch (nothing
    // allocated; grids up to kNoAllocDiagPoints points).
    DevBuf diag_spec, diag_partial, diag_out;
    mxs_status coarsening(int k, double *s_out, double *k1_out, hipStream_t s, bool noalloc) {
        const Inst &I = inst[k];
        if (!diag_shape_ok(I.nx, I.ny))
            return fail(MXS_ERR_UNSUPPORTED, "coarsening diagnostics need power-of-two sides up to %d (got %d x %d)",
                        kDiagMaxSide, I.nx, I.ny);
        DiagArgs d{};
        hipError_t e = hipSuccess;
        if (noalloc) {
            if (static_cast<long long>(I.nx) * I.ny > kNoAllocDiagPoints)
                return fail(MXS_ERR_UNSUPPORTED,
                            "the allocation-free diagnostics take grids of at most %lld points (got %d x %d)",
                            kNoAllocDiagPoints, I.nx, I.ny);
            e = noalloc_diag_scratch(I.nx, I.ny, &d);
            if (e != hipSuccess) return hip_fail(e, "static scratch address");
        } else {
            const size_t spec = sizeof(double2) * static_cast<size_t>(I.nx) * I.ny;
            const size_t part = sizeof(double) * (static_cast<size_t>(I.ny) + 2 * I.nx);
            if (diag_spec.bytes < spec) e = diag_spec.alloc(spec);
            if (e == hipSuccess && diag_partial.bytes < part) e = diag_partial.alloc(part);
            if (e == hipSuccess && !diag_out.ptr) e = diag_out.alloc(3 * sizeof(double));
            if (e != hipSuccess) return hip_fail(e, "diagnostics scratch allocation");
            d.spec = static_cast<double2 *>(diag_spec.ptr);
            d.partial = static_cast<double *>(diag_partial.ptr);
            d.out = static_cast<double *>(diag_out.ptr);
        }
        d.c = I.buf[(steps % 3 + 1) % 3];
        d.nx = I.nx;
        d.ny = I.ny;
        d.kx0 = 2.0 * M_PI / (I.nx * I.dx);
        d.ky0 = 2.0 * M_PI / (I.ny * I.dy);
        double h[3];
        e = launch_coarsening(dtype, d, s);
        if (e == hipSuccess) e = hipMemcpyAsync(h, d.out, sizeof h, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "coarsening diagnostics");
        const double mean_c2 = h[0] / (static_cast<double>(I.nx) * I.ny);
        if (s_out) *s_out = 1.0 / (1.0 - mean_c2);
        if (k1_out) *k1_out = h[1] / h[2];
        return std::isfinite(mean_c2) && std::isfinite(h[1]) && std::isfinite(h[2])
                   ? MXS_OK
                   : fail(MXS_ERR_NONFINITE, "the diagnostics are not finite");
    }

    // Right-hand side tables for row chunks of `rows` rows (0: pick a height
    // that keeps several workgroups per CU).
    mxs_status build_rhs(int rows) {
        const int n = ninst();
        const int cus = device_cu_count();
        const int Vs = 16 / dtype_size(dtype);   // state elements per thread (one 16-byte vector)
        auto tiles = [&](int r) {
            long long t = 0;
            for (const Inst &I : inst)
                t += static_cast<long long>((I.nx + rhs_threads * Vs - 1) / (rhs_threads * Vs)) *
                     ((I.ny + r - 1) / r);
            return t;
        };
        if (rows <= 0) {
            rows = 16;
            while (rows > 4 && tiles(rows) < 8LL * cus) rows /= 2;
        }
        rhs_rows = rows;
        int blk = 0;
        for (int r = 0; r < 3; ++r) rhs_h[r].resize(n);
        for (int g = 0; g < n; ++g) {
            const Inst &I = inst[g];
            RhsInst ri{};
            ri.nx = I.nx;
            ri.ny = I.ny;
            ri.nstrips = (I.nx + rhs_threads * Vs - 1) / (rhs_threads * Vs);
            ri.rows = rows;
            ri.nchunks = (I.ny + rows - 1) / rows;
            ri.blk0 = blk;
            blk += ri.nstrips * ri.nchunks;
            const double a = 2.0 / 3.0 * D * gamma * I.dt;
            double wb[25], wl[9];
            biharmonic_window(I.dx, I.dy, wb);
            laplacian_window(I.dx, I.dy, wl);
            for (int k = 0; k < 25; ++k) {
                ri.wb[k] = -a * wb[k];
                ri.wbf[k] = static_cast<float>(ri.wb[k]);
            }
            for (int k = 0; k < 9; ++k) {
                ri.wl[k] = 2.0 / 3.0 * D * I.dt * wl[k];
                ri.wlf[k] = static_cast<float>(ri.wl[k]);
            }
            ri.cdiff = -2.0 / 3.0;
            ri.cdifff = static_cast<float>(ri.cdiff);
            ri.R = I.w.ptr;
            for (int r = 0; r < 3; ++r) {
                RhsInst rr = ri;
                rr.prev = I.buf[r % 3];
                rr.cur = I.buf[(r + 1) % 3];
                rhs_h[r][g] = rr;
            }
        }
        rhs_blocks = blk;
        hipError_t e = hipSuccess;
        for (int r = 0; r < 3 && e == hipSuccess; ++r)
            e = rhs_d[r].upload(rhs_h[r].data(), sizeof(RhsInst) * n);
        if (e == hipSuccess && n > 1) {
            std::vector<int> units(n);
            for (int g = 0; g < n; ++g) units[g] = rhs_h[0][g].nstrips * rhs_h[0][g].nchunks;
            e = upload_map(rhs_map, units);
        }
        return e == hipSuccess ? MXS_OK : hip_fail(e, "plan tables upload");
    }

    void set_row_waves(int w) {
        row_nw = w;
        row_lds = line_lds_bytes(max_nx, row_nw);
        row_grid = wave_grid(row_lines, row_lds);
    }

    void drop_graphs() {
        for (auto &e : exec)
            if (e) {
                (void)hipGraphExecDestroy(e);
                e = nullptr;
            }
    }

    // Chooses the right-hand side chunk height and workgroup size and the
    // wavefronts per row solve by timing whole steps: every candidate is
    // timed in two passes and keeps its faster time (candidates differ by a
    // few percent, about the spread of one timing).  The timed steps rewrite
    // only the buffer that the next step overwrites anyway (C^{n+1}) and the
    // plan's scratch, and do not advance the step count.
    mxs_status autotune(hipStream_t s) override {
        // the candidates rebuild the tables that captured graphs point at:
        // drop the graphs first, so that no exit path leaves a stale one
        drop_graphs();
        const int r = static_cast<int>(steps % 3);
        struct Cand {
            int threads, rows, w;
            bool pers;
            double t;
            bool fus = false;
            int fr = 4, fc = 1;   // rows per workgroup and columns per thread of the fused form
        };
        std::vector<Cand> cands;
        for (int threads : {256, 128, 64})
            for (int rows : {4, 8, 16, 32})
                for (int w : {1, 2, 4}) {
                    if (line_lds_bytes(max_nx, w) > static_cast<size_t>(device_lds_limit())) continue;
                    if (!row_ranges.empty() && w != row_nw) continue;   // no LDS kernel to shape
                    cands.push_back({threads, rows, w, false, 1e30});
                }
        // the persistent step (one launch), right-hand side chunks of each height
        if (persist_ok)
            for (int rows : {4, 8, 16, 32}) cands.push_back({kPersistThreads, rows, row_nw, true, 1e30});
        // the right-hand side inside the row solves (no right-hand side tiles to shape)
        if (fused_ok) {
            const int shapes[3][2] = {{4, 1}, {8, 1}, {4, 2}};
            for (const auto &sh : shapes) {
                const size_t lds = ch_rhs_rows_lds_bytes(dtype, sh[0], sh[1], wave_nb(max_nx));
                if (lds > 0 && lds <= static_cast<size_t>(device_lds_limit()))
                    cands.push_back({kRhsThreads, 16, row_nw, false, 1e30, true, sh[0], sh[1]});
            }
        }
        if (cands.empty()) return MXS_OK;
        auto time_cand = [&](Cand &c) -> mxs_status {
            persistent = c.pers;
            fused = c.fus;
            rhs_threads = c.threads;
            mxs_status st = build_rhs(c.rows);
            if (st) return st;
            if (c.fus && c.fr != fused_rows) {
                hipError_t fe = build_fused(c.fr);
                if (fe != hipSuccess) return hip_fail(fe, "row group table upload");
            }
            if (c.fus) fused_cols = c.fc;
            set_row_waves(c.w);
            const double t = time_launches([&] { return enqueue(r, s); }, s, 2, 10);
            if (t < 0) {
                persistent = false;
                fused = false;
                return hip_fail(hipGetLastError(), "autotune launch");
            }
            c.t = std::min(c.t, t);
            return MXS_OK;
        };
        for (int pass = 0; pass < 2; ++pass)
            for (Cand &c : cands)
                if (mxs_status st = time_cand(c)) return st;
        // the fastest candidate of each step form gets three more interleaved
        // timings: the forms are often within a few percent of each other,
        // about the spread of one timing
        {
            Cand *fb[3] = {nullptr, nullptr, nullptr};   // separate, fused, persistent
            for (Cand &c : cands) {
                Cand *&b = fb[c.pers ? 2 : c.fus ? 1 : 0];
                if (!b || c.t < b->t) b = &c;
            }
            for (int pass = 0; pass < 3; ++pass)
                for (Cand *c : fb)
                    if (c)
                        if (mxs_status st = time_cand(*c)) return st;
        }
        const Cand *best = &cands.front();
        for (const Cand &c : cands)
            if (c.t < best->t) best = &c;
        for (const Cand &c : cands)
            if (c.pers && (!best_persist || c.t < best_persist_t)) {
                best_persist = true;
                best_persist_t = c.t;
            }
        for (const Cand &c : cands)
            if (!c.pers && !c.fus && c.t < best_graph_t) {
                best_graph_t = c.t;
                sep_threads = c.threads;
                sep_rows = c.rows;
            }
        for (const Cand &c : cands)
            if (c.fus && c.t < best_fused_t) best_fused_t = c.t;
        set_row_waves(best->w);
        persistent = best->pers;
        fused = best->fus;
        persist_nograph = false;
        if (fused_ok && best->fr != fused_rows) {
            hipError_t fe = build_fused(best->fus ? best->fr : 4);
            if (fe != hipSuccess) return hip_fail(fe, "row group table upload");
        }
        fused_cols = best->fus ? best->fc : 1;
        rhs_threads = best->threads;
        return build_rhs(best->rows);
    }

    // step times of the best candidate of each mode at the last autotune
    bool best_persist = false;
    double best_persist_t = 0, best_graph_t = 1e30, best_fused_t = 1e30;
    // right-hand side layout of the fastest separate-launch candidate (0: not tuned)
    int sep_threads = kRhsThreads, sep_rows = 0;

    void info(char *buf, int len) const override {
        const int launches = persistent ? 1
                             : fused  ? static_cast<int>(fused_ranges.size()) + 3
                                      : 1 + (row_ranges.empty() ? 1 : static_cast<int>(row_ranges.size())) + 3;
        int n = snprintf(buf, len, "ch instances=%d dtype=%d step=%s launches_per_step=%d rhs_rows=%d rhs_threads=%d "
                         "rhs_blocks=%d cols_blocks=%d colsB_groups=%d",
                         ninst(), dtype, persistent ? "persistent" : fused ? "fused" : "separate", launches, rhs_rows,
                         rhs_threads,
                         rhs_blocks, colsAC, bgroups);
        if (persistent && n < len)
            n += snprintf(buf + n, len - n, " persist_grid=%d persist_graph=%d", persist_grid, persist_nograph ? 0 : 1);
        if (best_graph_t < 1e29 && n < len)
            n += snprintf(buf + n, len - n, " tuned_us_separate=%.1f", best_graph_t * 1e6);
        if (best_persist && n < len)
            n += snprintf(buf + n, len - n, " tuned_us_persistent=%.1f", best_persist_t * 1e6);
        if (fused && n < len) n += snprintf(buf + n, len - n, " fused_rows=%d fused_cols=%d", fused_rows, fused_cols);
        if (best_fused_t < 1e29 && n < len)
            n += snprintf(buf + n, len - n, " tuned_us_fused=%.1f", best_fused_t * 1e6);
        if (row_ranges.empty() && n < len)
            n += snprintf(buf + n, len - n, " row_kernel=lds row_waves=%d row_grid=%d", row_nw, row_grid);
        for (size_t q = 0; q < row_ranges.size() && n < len; ++q)
            n += snprintf(buf + n, len - n, " row_kernel=register(nb=%d lines=%d)", row_ranges[q].nb,
                          row_ranges[q].count);
    }

    mxs_status build() {
        const int n = ninst();
        int maxnx = 0;
        for (const Inst &I : inst) maxnx = std::max(maxnx, I.nx);
        mxs_status bst = build_rhs(0);
        if (bst) return bst;

        // row solves (in place on w) and column solves (w -> C^{n+1})
        rows_h.resize(n);
        for (int r = 0; r < 3; ++r) cols_h[r].resize(n);
        const bool reg_rows = maxnx <= kWaveLineMax && !force_lds_lines();
        std::vector<double> pt(static_cast<size_t>(4) * kPowEntries * n);
        int bAC = 0, bB = 0;
        {
            // phase B threads per column from the mean number of segments
            long long segs = 0;
            for (const Inst &I : inst) segs += (I.ny + kSeg - 1) / kSeg;
            bgroups = cols_b_groups(static_cast<int>(segs / n));
        }
        const int bcols = cols_b_cols(bgroups);
        for (int g = 0; g < n; ++g) {
            Inst &I = inst[g];
            const double a = 2.0 / 3.0 * D * gamma * I.dt;
            const double bx = a / (I.dx * I.dx * I.dx * I.dx), by = a / (I.dy * I.dy * I.dy * I.dy);
            const double cx[3] = {1.0 + 6.0 * bx, -4.0 * bx, bx};
            const double cyv[3] = {1.0 + 6.0 * by, -4.0 * by, by};
            CyclicFactor fx, fy;
            if (factor_symmetric_circulant(2, cx, &fx) || factor_symmetric_circulant(2, cyv, &fy))
                return fail(MXS_ERR_INVALID_ARG, "could not factor the ADI line operators");
            RowsInst ro{};
            ro.in = I.w.ptr;
            ro.out = I.w.ptr;
            ro.ld = I.nx;
            ro.nx = I.nx;
            ro.ny = I.ny;
            ro.p1 = fx.p1;
            ro.p2 = fx.p2;
            ro.invK = fx.invK;
            rows_h[g] = ro;
            fill_pow_table(fx, 2, pt.data() + static_cast<size_t>(4) * kPowEntries * g);

            ColsInst co{};
            fill_cols_coef(fy, 2, I.ny, &co);
            co.ld = I.nx;
            co.nx = I.nx;
            co.ny = I.ny;
            co.nstrips = (I.nx + kColsThreads - 1) / kColsThreads;
            co.blk0 = bAC;
            co.blkB0 = bB;
            bAC += co.nstrips * co.nseg;
            bB += (I.nx + bcols - 1) / bcols;
            hipError_t e = I.carry.alloc(sizeof(double) * 4 * static_cast<size_t>(I.nx) * co.nseg);
            if (e != hipSuccess) return hip_fail(e, "carry allocation");
            co.carry = static_cast<double *>(I.carry.ptr);
            co.rhs = I.w.ptr;
            for (int r = 0; r < 3; ++r) {
                ColsInst cc = co;
                cc.prev = I.buf[r % 3];
                cc.cur = I.buf[(r + 1) % 3];
                cc.x = I.buf[(r + 2) % 3];
                cols_h[r][g] = cc;
            }
        }
        // global line numbers: instances grouped by register class, so that
        // every class is one contiguous range of lines
        {
            hipError_t pe = pows.upload(pt.data(), sizeof(double) * pt.size());
            if (pe != hipSuccess) return hip_fail(pe, "power table upload");
        }
        std::vector<int> by_class(n);
        std::iota(by_class.begin(), by_class.end(), 0);
        if (reg_rows)
            std::stable_sort(by_class.begin(), by_class.end(),
                             [&](int a, int b) { return wave_nb(inst[a].nx) < wave_nb(inst[b].nx); });
        row_ranges.clear();
        int line = 0;
        for (int g : by_class) {
            rows_h[g].line0 = line;
            rows_h[g].pow = static_cast<const double *>(pows.ptr) + static_cast<size_t>(4) * kPowEntries * g;
            if (reg_rows) {
                const int nb = wave_nb(inst[g].nx);
                if (row_ranges.empty() || row_ranges.back().nb != nb) row_ranges.push_back({nb, line, 0});
                row_ranges.back().count += inst[g].ny;
            }
            line += inst[g].ny;
        }
        row_lines = line;
        fused_ranges.clear();
        fused_ok = false;
        class_order = by_class;
        if (reg_rows) {
            // fused shape: 4 rows, 1 column per thread until tuned;
            // MXS_CH_FUSED_ROWS=8 or MXS_CH_FUSED_COLS=2 pick another (tests)
            const char *fr = getenv("MXS_CH_FUSED_ROWS");
            const char *fcol = getenv("MXS_CH_FUSED_COLS");
            const bool r8 = fr && atoi(fr) == 8, c2 = fcol && atoi(fcol) == 2 && !r8;
            fused_cols = c2 ? 2 : 1;
            hipError_t fe = build_fused(r8 ? 8 : 4);
            if (fe != hipSuccess) return hip_fail(fe, "row group table upload");
            fused_ok = true;
        }
        colsAC = bAC;
        colsB = bB;
        max_nx = maxnx;
        set_row_waves(line_waves(maxnx));
        if (row_lds > static_cast<size_t>(device_lds_limit()))
            return fail(MXS_ERR_UNSUPPORTED, "rows too long for the LDS of one workgroup");

        // mass
        int mb = 0;
        for (int r = 0; r < 3; ++r) mass_h[r].resize(n);
        for (int g = 0; g < n; ++g) {
            const long long npts = static_cast<long long>(inst[g].nx) * inst[g].ny;
            const int nblk = static_cast<int>(std::min<long long>(256, (npts + 65535) / 65536));
            for (int r = 0; r < 3; ++r) {
                MassInst m{};
                m.c = inst[g].buf[(r + 1) % 3];
                m.n = npts;
                m.blk0 = mb;
                m.nblk = nblk;
                mass_h[r][g] = m;
            }
            mb += nblk;
        }
        mass_blocks = mb;

        hipError_t e = hipSuccess;
        for (int r = 0; r < 3 && e == hipSuccess; ++r) {
            e = cols_d[r].upload(cols_h[r].data(), sizeof(ColsInst) * n);
            if (e == hipSuccess) e = mass_d[r].upload(mass_h[r].data(), sizeof(MassInst) * n);
        }
        if (e == hipSuccess) e = rows_d.upload(rows_h.data(), sizeof(RowsInst) * n);
        if (e == hipSuccess && n > 1) {
            std::vector<int> ac(n), bb(n), mbk(n);
            for (int g = 0; g < n; ++g) {
                ac[g] = cols_h[0][g].nstrips * cols_h[0][g].nseg;
                bb[g] = (inst[g].nx + bcols - 1) / bcols;
                mbk[g] = mass_h[0][g].nblk;
            }
            std::vector<int> line_inst(row_lines);
            for (int g = 0; g < n; ++g)
                std::fill(line_inst.begin() + rows_h[g].line0, line_inst.begin() + rows_h[g].line0 + inst[g].ny, g);
            e = rows_map.upload(line_inst.data(), sizeof(int) * line_inst.size());
            if (e == hipSuccess) e = upload_map(colsAC_map, ac);
            if (e == hipSuccess) e = upload_map(colsB_map, bb);
            if (e == hipSuccess) e = upload_map(mass_map, mbk);
        }
        if (e == hipSuccess) e = partial.alloc(sizeof(double) * mass_blocks);
        if (e == hipSuccess) e = mass_out.alloc(sizeof(double) * n);
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&mass_host), sizeof(double) * n, 0);
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&flag_host), sizeof(unsigned), 0);
        if (e != hipSuccess) return hip_fail(e, "plan tables upload");
        *flag_host = 0;

        // the persistent step: every row in a register class up to
        // kPersistNBMax, and a grid of as many workgroups as the CUs hold
        persist_ok = false;
        if (reg_rows && maxnx <= kPersistNBMax * kWaveBlock) {
            persist_nbmax = 1;
            for (const Inst &I : inst) persist_nbmax = std::max(persist_nbmax, wave_nb(I.nx));
            int per_cu = 0;
            if (persist_occupancy(dtype, persist_nbmax, &per_cu) == hipSuccess && per_cu > 0) {
                persist_grid = per_cu * device_cu_count();
                e = bar.alloc(4 * sizeof(unsigned));
                if (e == hipSuccess) e = hipMemset(bar.ptr, 0, 4 * sizeof(unsigned));
                if (e != hipSuccess) return hip_fail(e, "grid barrier allocation");
                persist_ok = true;
            } else {
                (void)hipGetLastError();
            }
        }
        if (const char *env = getenv("MXS_PERSIST_SPIN")) spin_limit = std::max(0, atoi(env));
        if (const char *env = getenv("MXS_CH_STEP")) {
            if (env[0] == 'p' && persist_ok) {
                mxs_status st = set_persistent(true, 0);
                if (st) return st;
            }
            if (env[0] == 'f' && fused_ok) fused = true;
        }
        return MXS_OK;
    }
};

mxs_status create_ch(int count, const int *nx, const int *ny, const double *dx, const double *dy,
                     const double *dt, double D, double gamma, int dtype, void *const *c_prev,
                     void *const *c_cur, void *const *c_next, mxs_plan *plan) {
    if (!plan) return fail(MXS_ERR_INVALID_ARG, "plan output pointer is NULL");
    *plan = nullptr;
    if (count <= 0 || !nx || !ny || !dx || !dy || !dt || !c_prev || !c_cur || !c_next)
        return fail(MXS_ERR_INVALID_ARG, "missing arguments");
    if (!valid_dtype(dtype)) return fail(MXS_ERR_INVALID_ARG, "unknown dtype %d", dtype);
    if (!(D > 0) || !(gamma > 0) || !std::isfinite(D) || !std::isfinite(gamma))
        return fail(MXS_ERR_INVALID_ARG, "need D > 0 and gamma > 0");
    CHPlan *p = new (std::nothrow) CHPlan();
    if (!p) return fail(MXS_ERR_OOM, "host allocation failed");
    p->dtype = dtype;
    p->wdtype = dtype == F64 ? F64 : F32;
    p->D = D;
    p->gamma = gamma;
    p->inst.resize(count);
    for (int g = 0; g < count; ++g) {
        Inst &I = p->inst[g];
        if (nx[g] < 8 || ny[g] < 8 || nx[g] > 16384 || ny[g] > 16384 || !(dx[g] > 0) ||
            !(dy[g] > 0) || !(dt[g] > 0) || !std::isfinite(dx[g]) || !std::isfinite(dy[g]) ||
            !std::isfinite(dt[g])) {
            delete p;
            return fail(MXS_ERR_INVALID_ARG, "instance %d: need 8 <= nx, ny <= 16384 and positive dx, dy, dt", g);
        }
        I.nx = nx[g];
        I.ny = ny[g];
        I.dx = dx[g];
        I.dy = dy[g];
        I.dt = dt[g];
        I.buf[0] = c_prev[g];
        I.buf[1] = c_cur[g];
        I.buf[2] = c_next[g];
        const size_t bytes = static_cast<size_t>(I.nx) * I.ny * dtype_size(dtype);
        for (int q = 0; q < 3; ++q) {
            if (!I.buf[q] || !aligned16(I.buf[q])) {
                delete p;
                return fail(I.buf[q] ? MXS_ERR_UNSUPPORTED : MXS_ERR_INVALID_ARG,
                            "instance %d: state buffers must be non-NULL and 16-byte aligned", g);
            }
            for (int r = 0; r < q; ++r)
                if (ranges_overlap(I.buf[q], bytes, I.buf[r], bytes)) {
                    delete p;
                    return fail(MXS_ERR_ALIAS, "instance %d: state buffers overlap", g);
                }
        }
        hipError_t e = I.w.alloc(static_cast<size_t>(I.nx) * I.ny * dtype_size(p->wdtype));
        if (e != hipSuccess) {
            delete p;
            return hip_fail(e, "scratch allocation");
        }
    }
    mxs_status st = p->build();
    if (st) {
        delete p;
        return st;
    }
    register_plan(p);
    *plan = p;
    return MXS_OK;
}

CHPlan *as_ch(mxs_plan plan) {
    if (!plan || !is_live(plan) || plan->kind != KIND_CH) return nullptr;
    return static_cast<CHPlan *>(plan);
}

}  // namespace
}  // namespace mxs

using namespace mxs;

extern "C" {

mxs_status mxs_ch_create(int nx, int ny, double dx, double dy, double dt, double D, double gamma,
                         int dtype, void *c_prev, void *c_cur, void *c_next, mxs_plan *plan) {
    void *p[1] = {c_prev}, *c[1] = {c_cur}, *n[1] = {c_next};
    return create_ch(1, &nx, &ny, &dx, &dy, &dt, D, gamma, dtype, p, c, n, plan);
}

mxs_status mxs_ch_ensemble_create(int count, const int *nx, const int *ny, const double *dx,
                                  const double *dy, const double *dt, double D, double gamma,
                                  int dtype, void *const *c_prev, void *const *c_cur,
                                  void *const *c_next, mxs_plan *plan) {
    return create_ch(count, nx, ny, dx, dy, dt, D, gamma, dtype, c_prev, c_cur, c_next, plan);
}

mxs_status mxs_ch_step(mxs_plan plan, int nsteps, int use_graph, void *hip_stream) {
    CHPlan *p = as_ch(plan);
    if (!p) return fail(MXS_ERR_BAD_HANDLE, "not a Cahn-Hilliard plan");
    if (nsteps < 0) return fail(MXS_ERR_INVALID_ARG, "nsteps < 0");
    return p->step(nsteps, use_graph != 0, static_cast<hipStream_t>(hip_stream));
}

mxs_status mxs_ch_set_step_mode(mxs_plan plan, int mode) {
    CHPlan *p = as_ch(plan);
    if (!p) return fail(MXS_ERR_BAD_HANDLE, "not a Cahn-Hilliard plan");
    if (mode != MXS_CH_SEPARATE && mode != MXS_CH_PERSISTENT && mode != MXS_CH_FUSED)
        return fail(MXS_ERR_INVALID_ARG, "mode must be MXS_CH_SEPARATE, MXS_CH_PERSISTENT or MXS_CH_FUSED");
    if (mode == MXS_CH_FUSED && !p->fused_ok)
        return fail(MXS_ERR_UNSUPPORTED, "this plan cannot form the right-hand side inside the row solves");
    int rows = p->rhs_rows;
    if (mode != MXS_CH_PERSISTENT) {
        // the separate launches take the right-hand side layout tuned for them
        if (p->sep_rows > 0) {
            p->rhs_threads = p->sep_threads;
            rows = p->sep_rows;
        } else if (p->persistent) {
            p->rhs_threads = kRhsThreads;
            rows = 0;
        }
    }
    mxs_status st = p->set_persistent(mode == MXS_CH_PERSISTENT, rows);
    if (st == MXS_OK) p->fused = mode == MXS_CH_FUSED;
    return st;
}

mxs_status mxs_ch_state(mxs_plan plan, int k, void **c_prev, void **c_cur) {
    CHPlan *p = as_ch(plan);
    if (!p) return fail(MXS_ERR_BAD_HANDLE, "not a Cahn-Hilliard plan");
    if (k < 0 || k >= p->ninst()) return fail(MXS_ERR_INVALID_ARG, "instance %d out of range", k);
    const int r = static_cast<int>(p->steps % 3);
    if (c_prev) *c_prev = p->inst[k].buf[r % 3];
    if (c_cur) *c_cur = p->inst[k].buf[(r + 1) % 3];
    return MXS_OK;
}

mxs_status mxs_ch_steps_taken(mxs_plan plan, long long *nsteps) {
    CHPlan *p = as_ch(plan);
    if (!p) return fail(MXS_ERR_BAD_HANDLE, "not a Cahn-Hilliard plan");
    if (!nsteps) return fail(MXS_ERR_INVALID_ARG, "nsteps is NULL");
    *nsteps = p->steps;
    return MXS_OK;
}

mxs_status mxs_ch_coarsening(mxs_plan plan, int k, double *s_out, double *k1_out, void *hip_stream) {
    CHPlan *p = as_ch(plan);
    if (!p) return fail(MXS_ERR_BAD_HANDLE, "not a Cahn-Hilliard plan");
    if (k < 0 || k >= p->ninst()) return fail(MXS_ERR_INVALID_ARG, "instance %d out of range", k);
    return p->coarsening(k, s_out, k1_out, static_cast<hipStream_t>(hip_stream), false);
}

mxs_status mxs_ch_coarsening_noalloc(mxs_plan plan, int k, double *s_out, double *k1_out,
                                     void *hip_stream) {
    CHPlan *p = as_ch(plan);
    if (!p) return fail(MXS_ERR_BAD_HANDLE, "not a Cahn-Hilliard plan");
    if (k < 0 || k >= p->ninst()) return fail(MXS_ERR_INVALID_ARG, "instance %d out of range", k);
    return p->coarsening(k, s_out, k1_out, static_cast<hipStream_t>(hip_stream), true);
}

mxs_status mxs_ch_mass(mxs_plan plan, double *host_out, void *hip_stream) {
    CHPlan *p = as_ch(plan);
    if (!p) return fail(MXS_ERR_BAD_HANDLE, "not a Cahn-Hilliard plan");
    if (!host_out) return fail(MXS_ERR_INVALID_ARG, "host_out is NULL");
    return p->mass(host_out, static_cast<hipStream_t>(hip_stream));
}

}  // extern "C"
