// The whole ADI Cahn-Hilliard step of every instance of a plan in one
// persistent launch (Sec. 5.1): the right-hand side, the row solves and the
// three column phases run one after the other in the same workgroups, which
// stay resident for the whole step and meet at a grid barrier between
// phases.  Each phase hands out the same work items as its own kernel does
// (right-hand-side tiles, rows per wavefront, column segments and column
// groups), strided over the persistent grid.  Two workgroups of four
// wavefronts per CU (256 registers per lane, enough for every phase without
// spilling), rows of at most 1024 elements (register classes up to 4).
//
// The grid barrier is a counter and a generation word in device memory:
// every workgroup adds itself to the counter; the last one resets it and
// advances the generation, for which the others wait.  The wait is bounded:
// past the plan's spin limit a workgroup sets a sticky error word and leaves
// (every later barrier then returns at once and the remaining phases are
// skipped), so a grid that is not co-resident ends instead of hanging, and
// the host reports the error.  The last workgroup to finish resets the
// counters for the next launch.  Agent-scope release and acquire fences
// around the barrier make each phase's stores visible to every XCD.
#include "ch_dev.h"
#include "cols_dev.h"
#include "persist.h"
#include "wave_dev.h"

#include <algorithm>

namespace mxs {

namespace {

// Grid barrier; false when it failed (now or earlier).  ok points to an LDS
// word of the workgroup.
__device__ __forceinline__ bool grid_sync(unsigned *bar, int spin_limit, int *ok) {
    __syncthreads();
    if (threadIdx.x == 0) {
        int good = 1;
        __threadfence();
        const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__hip_atomic_load(&bar[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
            good = 0;
        } else {
            const unsigned arrived =
                __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
            if (arrived == gridDim.x) {
                __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                int spins = 0;
                while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                    if (__hip_atomic_load(&bar[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                        ++spins > spin_limit) {
                        __hip_atomic_store(&bar[3], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        good = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
        }
        __threadfence();
        *ok = good;
    }
    __syncthreads();
    return *ok != 0;
}

// Length class of a row of nx elements (as wave_nb on the host).
__device__ __forceinline__ int row_class(int nx) {
    const int nb = (nx + kWaveBlock - 1) / kWaveBlock;
    return nb <= 1 ? 1 : nb <= 2 ? 2 : nb <= 4 ? 4 : nb <= 8 ? 8 : 16;
}

template <typename TW, int NB>
__device__ __forceinline__ void row_if(const PersistArgs &p, int li, unsigned char *stage) {
    wave_line<TW, 2, NB>(RowsSrc<TW>{p.rows, p.rows_map}, li, reinterpret_cast<TW *>(stage));
}

template <typename T, typename TW, int NBMAX>
__global__ void __launch_bounds__(kPersistThreads, 2) ch_step_persistent(const PersistArgs p) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int *ok = reinterpret_cast<int *>(smem_raw);
    unsigned char *lds = smem_raw + 16;
    const int G = gridDim.x;

    // 1. right-hand side tiles
    for (int b = blockIdx.x; b < p.rhs_blocks; b += G) {
        const RhsInst &I = p.rhs[p.rhs_map ? p.rhs_map[b] : 0];
        rhs_tile<T, TW>(I, b - I.blk0, lds);
    }
    bool good = grid_sync(p.bar, p.spin_limit, ok);

    // 2. row solves, one line per wavefront
    if (good) {
        constexpr int WPB = kPersistThreads / 64;
        const int w = threadIdx.x >> 6;
        unsigned char *stage = lds + static_cast<size_t>(w) * p.stage_bytes;
        for (int li = blockIdx.x * WPB + w; li < p.row_lines; li += G * WPB) {
            const int nb = row_class(p.rows[p.rows_map ? p.rows_map[li] : 0].nx);
            if (nb == 1) row_if<TW, 1>(p, li, stage);
            else if (NBMAX >= 2 && nb == 2) row_if<TW, NBMAX >= 2 ? 2 : 1>(p, li, stage);
            else if (NBMAX >= 4) row_if<TW, NBMAX >= 4 ? 4 : 1>(p, li, stage);
        }
        good = grid_sync(p.bar, p.spin_limit, ok);
    }

    // 3. column phase A: per-segment summaries
    if (good) {
        for (int b = blockIdx.x; b < p.colsAC; b += G) {
            cols_a_block<TW, 2>(p.cols, p.colsAC_map, b);
            __syncthreads();
        }
        good = grid_sync(p.bar, p.spin_limit, ok);
    }

    // 4. column phase B: carries between segments
    if (good) {
        Aff *xa = reinterpret_cast<Aff *>(lds);
        for (int b = blockIdx.x; b < p.colsB; b += G) {
            if (p.bgroups == 16) cols_b_block<2, 16, false>(p.cols, p.colsB_map, b, xa);
            else cols_b_block<2, 4, false>(p.cols, p.colsB_map, b, xa);
            __syncthreads();
        }
        good = grid_sync(p.bar, p.spin_limit, ok);
    }

    // 5. column phase C: both recurrences from the carries, C^{n+1}
    if (good) {
        for (int b = blockIdx.x; b < p.colsAC; b += G) {
            cols_c_block<TW, T, 2, 1>(p.cols, p.colsAC_map, b);
            __syncthreads();
        }
    }

    // the last workgroup out resets the counters for the next launch
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned done = __hip_atomic_fetch_add(&p.bar[2], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        if (done == gridDim.x) {
            __hip_atomic_store(&p.bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&p.bar[2], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
        }
    }
}

template <typename T, typename TW>
const void *kernel_for(int nbmax) {
    switch (nbmax) {
    case 1: return reinterpret_cast<const void *>(&ch_step_persistent<T, TW, 1>);
    case 2: return reinterpret_cast<const void *>(&ch_step_persistent<T, TW, 2>);
    case 4: return reinterpret_cast<const void *>(&ch_step_persistent<T, TW, 4>);
    default: return nullptr;
    }
}

const void *persist_kernel(int dtype, int nbmax) {
    switch (dtype) {
    case F64: return kernel_for<double, double>(nbmax);
    case F32: return kernel_for<float, float>(nbmax);
    case BF16: return kernel_for<bf16, float>(nbmax);
    default: return nullptr;
    }
}

}  // namespace

size_t persist_lds_bytes(int dtype, int nbmax) {
    const size_t rhs = dtype == F64 ? rhs_lds_bytes<double>(kPersistThreads)
                                    : dtype == F32 ? rhs_lds_bytes<float>(kPersistThreads)
                                                   : rhs_lds_bytes<bf16>(kPersistThreads);
    const size_t rows = (kPersistThreads / 64) * persist_stage_bytes(dtype, nbmax);
    const size_t colsb = sizeof(Aff) * kColsThreads;
    return 16 + std::max(rhs, std::max(rows, colsb));
}

size_t persist_stage_bytes(int dtype, int nbmax) {
    // the LDS stage of one wavefront for the largest register class among
    // the rows (Stage<TW, E>: 64 lanes of E values and 16 bytes of padding)
    const int E = nbmax <= 1 ? WaveShape<1>::E : nbmax <= 2 ? WaveShape<2>::E : WaveShape<4>::E;
    const int tsz = dtype == F64 ? 8 : 4;
    return (static_cast<size_t>(64) * (E + 16 / tsz) * tsz + 15) / 16 * 16;
}

hipError_t persist_occupancy(int dtype, int nbmax, int *blocks_per_cu) {
    const void *k = persist_kernel(dtype, nbmax);
    if (!k) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, kPersistThreads,
                                                        persist_lds_bytes(dtype, nbmax));
}

hipError_t launch_ch_persistent(int dtype, int nbmax, const PersistArgs &a, int grid, hipStream_t s) {
    const void *k = persist_kernel(dtype, nbmax);
    if (!k) return hipErrorInvalidValue;
    void *args[] = {const_cast<PersistArgs *>(&a)};
    return hipLaunchCooperativeKernel(k, dim3(grid), dim3(kPersistThreads), args,
                                      static_cast<unsigned>(persist_lds_bytes(dtype, nbmax)), s);
}

}  // namespace mxs
