// Persistent batched sweep kernel for gfx950.
//
// One cooperative launch runs a chunk of sweeps for every film of a batch
// (many replicas of uneven size, each with its own temperature and field
// schedule).  The work of one sublattice phase is the list of all films'
// tiles; every resident block takes tiles from that list, then all blocks
// meet at a grid-wide barrier before the next sublattice (no two neighbours
// share a sublattice, but a sublattice reads what the previous one wrote).
// Per-film bookkeeping (sweep counter, step sums, records, next table) runs
// after the last sublattice of each sweep, one wave per film, followed by one
// more barrier.
//
// Tile -> block mapping is XCD-aware: MI355X dispatches consecutive blocks
// round-robin over its 8 XCDs, each with its own L2, so block b works on the
// (b mod 8)-th contiguous eighth of the tile list; neighbouring tiles, which
// share halo rows, then meet in the same L2.
//
// The barrier is a monotonic arrival counter with a bounded spin: a block that
// waits longer than the bound sets an error flag and every block leaves, so a
// launch always drains (cooperative launch already guarantees residency).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "isf_tiles.h"

namespace isf {

constexpr uint32_t kSpinLimit = 1u << 22;  // ~0.5 s of polling at ~128 cycles per probe

__device__ __forceinline__ bool grid_barrier(uint32_t *bar, uint32_t nblocks, uint32_t &gen) {
    __shared__ uint32_t ok_sh;
    __syncthreads();
    if (threadIdx.x == 0) {
        ++gen;
        const uint32_t target = gen * nblocks;
        __threadfence();
        aadd(&bar[0], 1u);
        uint32_t ok = 1;
        uint32_t spins = 0;
        while (ald(&bar[0]) < target) {
            if (ald(&bar[1]) != 0u || ++spins > kSpinLimit) {
                ast(&bar[1], 1u);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
        ok_sh = ok;
    }
    __syncthreads();
    return ok_sh != 0;
}

// Tile t of the launch's tile list -> (entry, block within entry).
template <int FORMAT, int TX, int TY, int RY>
__global__ __launch_bounds__(TX *TY) void k_persistent(const BatchEntry *__restrict__ ents, uint32_t n_ents,
                                                       uint32_t total_tiles, uint32_t n_sweeps, uint32_t *bar) {
    __shared__ uint32_t tab[kTableWords];
    __shared__ uint32_t t_sh, run_sh;
    const uint32_t G = gridDim.x;
    // XCD-aware split: blocks of XCD x (b mod 8 == x) share the x-th eighth of the tiles
    const uint32_t nx = G >= 8 ? 8u : 1u;
    const uint32_t xcd = blockIdx.x % nx;
    const uint32_t rank = blockIdx.x / nx;
    const uint32_t per_xcd = (G - xcd + nx - 1) / nx;  // blocks on this XCD
    const uint32_t t_lo = (uint32_t)((uint64_t)total_tiles * xcd / nx);
    const uint32_t t_hi = (uint32_t)((uint64_t)total_tiles * (xcd + 1) / nx);
    uint32_t gen = 0;
    for (uint32_t sw = 0; sw < n_sweeps; ++sw) {
        for (uint32_t sigma = 0; sigma < 4; ++sigma) {
            for (uint32_t tile = t_lo + rank; tile < t_hi; tile += per_xcd) {
                const BatchEntry &e = ents[find_entry(ents, n_ents, tile)];
                const LatDev &L = e.lat;
                __syncthreads();  // previous tile's readers of LDS are done
                const uint32_t bl = tile - e.block_begin;
                const uint32_t bx = bl % e.nbx, byz = bl / e.nbx;
                const uint32_t by = byz % e.nby, bz = byz / e.nby;
                int dM = 0, dE = 0, acc = 0;
                if (FORMAT == ISF_FORMAT_INT8) {
                    phase_block_i8<TX, TY, RY, true>(L, sigma, bx, by, bz, dM, dE, acc);
                } else {
                    if (!stage_film<true>(L, tab, &t_sh, &run_sh))
                        continue;
                    phase_tile_bp<TX, TY, RY>(L, sigma, bx, by, bz, tab, t_sh, dM, dE, acc);
                }
                finish_block<TX * TY>(L, dM, dE, acc, bl);
            }
            if (!grid_barrier(bar, G, gen))
                return;
        }
        // sweep end: one wave per running film, then every block sees the new state
        for (uint32_t f = blockIdx.x; f < n_ents; f += G) {
            const LatDev &L = ents[f].lat;
            if (threadIdx.x < 64 && ald(&L.st->step) < ald(&L.st->n_steps))
                sweep_end<true>(L);
        }
        if (!grid_barrier(bar, G, gen))
            return;
    }
}

__global__ void k_zero_words(uint32_t *p, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0u;
}

template <int FORMAT, int TX, int TY, int RY>
static hipError_t launch_one(const BatchEntry *ents, uint32_t n_ents, uint32_t total, uint32_t n_sweeps,
                             uint32_t *bar, hipStream_t s, uint32_t *grid_used) {
    static int max_blocks = -1;
    if (max_blocks < 0) {
        int dev = 0, per_cu = 0, cus = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess)
            return e;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<FORMAT, TX, TY, RY>, TX * TY, 0);
        if (e != hipSuccess)
            return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess)
            return e;
        // Half the occupancy limit: a grid barrier needs every block resident, and a
        // grid at the theoretical maximum leaves no slack for anything else the
        // device keeps on its compute units.  Blocks loop over tiles, so fewer
        // blocks still cover all the work.
        max_blocks = std::max(1, per_cu / 2) * cus;
    }
    uint32_t grid = std::min<uint32_t>((uint32_t)max_blocks, total);
    if (grid == 0)
        grid = 1;
    *grid_used = grid;
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, bar, 2u);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    void *args[] = {(void *)&ents, (void *)&n_ents, (void *)&total, (void *)&n_sweeps, (void *)&bar};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_persistent<FORMAT, TX, TY, RY>), dim3(grid),
                                      dim3(TX * TY), args, 0, s);
}

hipError_t launch_persistent(const BatchEntry *ents_dev, uint32_t n_ents, uint32_t total_blocks, uint32_t format,
                             const Tiling &tl, uint32_t n_sweeps, uint32_t *barrier, hipStream_t s,
                             uint32_t *grid_used) {
#define X(a, b, c)                                                                                                 \
    if (tl.tx == a && tl.ty == b && tl.ry == c)                                                                    \
        return format == ISF_FORMAT_INT8                                                                           \
                   ? launch_one<ISF_FORMAT_INT8, a, b, c>(ents_dev, n_ents, total_blocks, n_sweeps, barrier, s,   \
                                                          grid_used)                                               \
                   : launch_one<ISF_FORMAT_BITPACK, a, b, c>(ents_dev, n_ents, total_blocks, n_sweeps, barrier, s, \
                                                             grid_used);
    X(64, 4, 1) X(64, 4, 2) X(32, 8, 1) X(32, 8, 2) X(16, 16, 1) X(16, 16, 2)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace isf
