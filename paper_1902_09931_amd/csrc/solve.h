// Cyclic banded line solves: shared structures of the kernels and the plans.
//
// A symmetric positive-definite circulant with bands c[0..bw] (bw = 1, 2) is
// factored exactly as A = K P(S) P(S^-1), with S the cyclic shift
// ((S y)_i = y_{i-1}) and P(z) = 1 - p1 z - p2 z^2 holding the roots of the
// symbol inside the unit circle (spectral factorisation of the symbol).
// A x = r is then solved by two cyclic linear recurrences:
//     forward   y_i = r_i + p1 y_{i-1} + p2 y_{i-2}   (indices mod n)
//     backward  u_i = y_i + p1 u_{i+1} + p2 u_{i+2}
// and x = u / K.  Both recurrences are stable (|roots| < 1).
#pragma once

#include "mxs_internal.h"

#include <stdlib.h>

namespace mxs {

struct CyclicFactor {
    double p1 = 0, p2 = 0, K = 1, invK = 1;
};

// Factor the symmetric circulant with bands c[0..bw].  Returns 0 on success,
// -1 for invalid input, -2 when the symbol is not positive on the circle.
int factor_symmetric_circulant(int bw, const double *c, CyclicFactor *f);

// Lines are solved by workgroups of NT = 64 * nw threads (nw = 1 or 4):
// chunk t of k elements (k even) is stored in LDS at t * (k + 1), followed by
// nw exchange slots of six doubles.
inline int line_waves(long long nmax) {
    if (const char *env = getenv("MXS_LINE_WAVES")) {
        const int v = atoi(env);
        if (v == 1 || v == 2 || v == 4) return v;
    }
    return nmax > 2048 ? 4 : 1;
}
inline int line_chunk(long long n, int nw) {
    const long long nt = 64LL * nw;
    long long k = (n + 2 * nt - 1) / (2 * nt) * 2;
    return static_cast<int>(k < 2 ? 2 : k);
}
inline size_t line_lds_bytes(long long nmax, int nw) {
    return (static_cast<size_t>(64) * nw * (line_chunk(nmax, nw) + 1) + 6 * nw) * sizeof(double);
}

// --- lines held in the registers of one wavefront -----------------------------
// A line of at most kWaveLineMax elements is held by one wavefront, E = 4, 8
// or 16 consecutive elements per lane in blocks of 64 E (by length class).
// The lane states are scanned with powers of the companion matrix
// M = [[p1, p2], [1, 0]] taken from a table: entries k = 0..kWaveBlock hold
// M^k, entries kWaveBlock + 1 + c hold M^(kWaveBlock c), c = 0..kWaveNBMax;
// each entry is 4 doubles, row-major.
constexpr int kWaveBlock = 256;
constexpr int kWaveNBMax = 16;
constexpr int kWaveLineMax = kWaveBlock * kWaveNBMax;
constexpr int kPowEntries = kWaveBlock + 1 + kWaveNBMax + 1;
void fill_pow_table(const CyclicFactor &f, int bw, double *out);   // 4 * kPowEntries doubles
// Length class of a line of n elements (n <= kWaveLineMax): the number of
// kWaveBlock-element blocks it may span, 1, 2, 4, 8 or 16.
inline int wave_nb(long long n) {
    const long long nb = (n + kWaveBlock - 1) / kWaveBlock;
    return nb <= 1 ? 1 : nb <= 2 ? 2 : nb <= 4 ? 4 : nb <= 8 ? 8 : 16;
}
// The LDS kernel is used for every line when MXS_LINE_KERNEL=lds (tests).
inline bool force_lds_lines() {
    const char *env = getenv("MXS_LINE_KERNEL");
    return env && env[0] == 'l';
}

// --- lines solved by one workgroup each --------------------------------------
struct RaggedLines {
    const void *in;
    void *out;
    const long long *offsets;   // device, nbatch + 1
    const int *order;           // device, lines by decreasing length
    int nlines;
    double p1, p2, invK;
    const double *pow;          // power table (register kernel)
};

struct RowsInst {
    const void *in;
    void *out;
    long long ld;
    int nx, ny;
    int line0;                  // first global line index of this instance
    double p1, p2, invK;
    const double *pow;          // power table (register kernel)
};

// --- columns: three phases over segments of kSeg rows -------------------------
constexpr int kSeg = 32;
constexpr int kColsThreads = 256;
// phase B: G threads per column (G = 4 or 16), kColsThreads / G columns per
// workgroup.  Each thread composes the maps of its share of a column's
// segments and then combines the G shares, so G trades the serial chain per
// thread against the combine: 16 for long columns, 4 for short ones.
inline int cols_b_groups(int nseg) { return nseg >= 64 ? 16 : 4; }
inline int cols_b_cols(int groups) { return kColsThreads / groups; }

struct ColsInst {
    const void *rhs;            // rhs dtype
    void *x;                    // output dtype
    const void *cur;            // CH update: C^n (output dtype), or nullptr
    const void *prev;           // CH update: C^{n-1} (output dtype), or nullptr
    double *carry;              // [nseg][4][nx] doubles
    long long ld;
    int nx, ny;
    int nstrips, nseg;
    int blk0;                   // first block of phases A and C
    int blkB0;                  // first block of phase B
    double p1, p2, invK;
    double Tf[4], Tl[4];        // M^kSeg and M^(last segment length), row-major
    double Qf[4], Ql[4];        // top state of the backward pass over the forward homogeneous response
    double Cinv[4];             // (I - M^n)^-1
};

// Fill the column coefficients of an instance with n = ny rows.
void fill_cols_coef(const CyclicFactor &f, int bw, int ny, ColsInst *ci);

hipError_t launch_ragged_lines(int dtype, int bw, const RaggedLines &a, int nw, int grid,
                               size_t lds, hipStream_t s);
// map[li] (map[b]) is the instance of line li (workgroup b); nullptr: all
// belong to instance 0.
hipError_t launch_rows(int dtype, int bw, const RowsInst *inst, const int *map, int nlines, int nw,
                       int grid, size_t lds, hipStream_t s);
// A work unit of the register kernel for ragged lines: `count` consecutive
// lines (positions first .. first + count - 1 of the sorted order) of length
// class nb, at most kWaveNBMax / nb of them.
struct WaveUnit {
    int first;
    int count;
    int nb;
    int pad;
};
// Every work unit in one launch (one wavefront per unit).
hipError_t launch_wave_units(int dtype, int bw, const RaggedLines &a, const WaveUnit *units, int nunits,
                             hipStream_t s);
// Register kernel over the ragged lines of one class nb: sorted positions
// first .. first + count - 1, one wavefront each.
hipError_t launch_wave_ragged(int dtype, int bw, int nb, const RaggedLines &a, int first, int count,
                              hipStream_t s);
// Register kernel over the rows first .. first + count - 1 (global line
// indices), each at most 256 nb elements.
hipError_t launch_wave_rows(int dtype, int bw, int nb, const RowsInst *inst, const int *map, int first,
                            int count, hipStream_t s);
// epilogue: 0 = x = A^-1 rhs; 1 = Cahn-Hilliard update x = 2 cur - prev + A^-1 rhs.
// (rhs dtype, output dtype) pairs: (F64,F64), (F32,F32), (BF16,BF16), (F32,BF16).
hipError_t launch_cols(int rhs_dtype, int x_dtype, int bw, int epilogue, const ColsInst *inst,
                       const int *mapAC, const int *mapB, int blocksAC, int blocksB, int bgroups,
                       hipStream_t s);

}  // namespace mxs
