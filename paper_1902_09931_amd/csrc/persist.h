// The persistent form of the ADI Cahn-Hilliard step (one launch per step):
// arguments shared by the kernel (persist.hip) and the plan (ch_plan.cpp).
#pragma once

#include "ch.h"
#include "solve.h"

namespace mxs {

constexpr int kPersistThreads = 256;

struct PersistArgs {
    const RhsInst *rhs;          // right-hand-side tables, tiles of kPersistThreads threads
    const int *rhs_map;          // instance of every tile (nullptr: one instance)
    int rhs_blocks;
    const RowsInst *rows;        // row solves (register kernel, rows <= kWaveLineMax)
    const int *rows_map;         // instance of every line
    int row_lines;
    const ColsInst *cols;        // column phases
    const int *colsAC_map, *colsB_map;
    int colsAC, colsB;
    int bgroups;                 // phase B threads per column (4 or 16)
    unsigned *bar;               // device words: arrivals, generation, exits, error
    int spin_limit;              // polls of a barrier wait before it fails
    int stage_bytes;             // LDS stage of one wavefront in the row phase
};

// Largest register class of the rows the persistent step takes (rows of at
// most 4 * kWaveBlock = 1024 elements); wider grids use the graph of
// separate launches.
constexpr int kPersistNBMax = 4;

// LDS per workgroup and per wavefront stage of the row phase, for the state
// dtype and the largest register class nbmax (1, 2 or 4) of the rows.
size_t persist_lds_bytes(int dtype, int nbmax);
size_t persist_stage_bytes(int dtype, int nbmax);
// Workgroups of the persistent kernel one CU holds at once.
hipError_t persist_occupancy(int dtype, int nbmax, int *blocks_per_cu);
// One cooperative launch of `grid` workgroups (all co-resident, else the
// runtime refuses the launch).
hipError_t launch_ch_persistent(int dtype, int nbmax, const PersistArgs &a, int grid, hipStream_t s);

}  // namespace mxs
