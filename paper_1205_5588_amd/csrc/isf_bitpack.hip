// HIP kernels for gfx950: the BITPACK storage format (one spin bit and one
// occupancy bit per site, 32 compact sites per word, the last word of a row
// partly filled where W is not a multiple of 32; layout in isf_internal.h).
// Same draws, same thresholds, same visiting rule as the INT8 kernels, so the
// trajectory is identical.
//
// A thread owns one word (32 consecutive compact sites of one row = 8 Philox
// calls).  For the 12 neighbour rows it forms, bit-sliced over the 32 sites,
// U = number of up neighbours and D = number of vacant neighbour slots
// (vacancies and rows outside the film), so that the biased neighbour sum is
// n + 12 = 2U + D, and the threshold-table index is (2U + D) + 25 s.  Only
// the table lookup and the comparison with the draw are per site.
// Vacant sites keep their spin bit at 0, so U needs no masking.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "isf_books.h"
#include "isf_tiles.h"

namespace isf {

template <int TX, int TY, int RY>
__global__ __launch_bounds__(TX *TY) void k_phase_bp_batch(const BatchEntry *__restrict__ ents, uint32_t n_ents,
                                                           uint32_t sigma) {
    __shared__ uint32_t tab[kTableWords];
    __shared__ uint32_t t_sh, run_sh;
    const uint32_t b = blockIdx.x;
    const BatchEntry &e = ents[find_entry(ents, n_ents, b)];
    const LatDev &L = e.lat;
    if (!stage_film<false>(L, tab, &t_sh, &run_sh))
        return;
    const uint32_t bl = b - e.block_begin;
    const uint32_t bx = bl % e.nbx, byz = bl / e.nbx;
    const uint32_t by = byz % e.nby, bz = byz / e.nby;
    int dM = 0, dE = 0, acc = 0;
    phase_tile_bp<TX, TY, RY>(L, sigma, bx, by, bz, tab, t_sh, dM, dE, acc);
    finish_block<TX * TY>(L, dM, dE, acc, bl);
}

// One sublattice of a sweep of parity q whose books ride in the launches (as
// the whole-sweep kernels keep them): the thresholds, sweep counter and run
// flag come from pos[q], the block sums go to slots_of(q), and in the first
// sublattice wave 0 of block 0 folds the sweep before (parity 1 - q) into the
// film state and its record and writes the next sweep's position.  This saves
// the one-wave sweep-end launch of every sweep.
template <int TX, int TY, int RY>
__global__ __launch_bounds__(TX *TY) void k_phase_bp_pos(LatDev L, uint32_t sigma, uint32_t q) {
    __shared__ uint32_t tab[kTableWords];
    __shared__ uint32_t t_sh, run_sh;
    __shared__ BookLds bk;
    const uint32_t tid = threadIdx.x;
    const uint32_t blin = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    const bool booker = sigma == 0 && blin == 0 && tid < 64;  // uniform per wave
    BookRegs br{};
    if (booker)
        br = book_issue(L, 1 - q, q, tid);
    const SweepPos &P = L.pos[q];
    if (tid < kTableWords)
        tab[tid] = P.table[tid];
    if (tid == 0) {
        t_sh = (uint32_t)P.t;
        run_sh = P.run;
    }
    if (booker)
        book_stage(bk, br, tid);
    __syncthreads();
    if (booker) {
        book_fold(L, 1 - q, bk, tid);
        book_advance(L, q, bk, tab, tid);
    }
    if (!run_sh)  // uniform: the schedule is finished; nothing flips
        return;
    int dM = 0, dE = 0, acc = 0;
    phase_tile_bp<TX, TY, RY>(L, sigma, blockIdx.x, blockIdx.y, blockIdx.z, tab, t_sh, dM, dE, acc);
    finish_block_to<TX * TY>(slots_of(L, q), dM, dE, acc, blin);
}

// Start: spin bit 1 on occupied sites for UP, 0 for DOWN, draw < 2^31 for RANDOM.
__global__ void k_init_bp(LatDev L, int32_t mode) {
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t y = blockIdx.y, z = blockIdx.z;
    const uint32_t nw = L.nd;
    if (w >= nw)
        return;
    uint32_t *row = reinterpret_cast<uint32_t *>(L.spins) + ((size_t)(z + 1) * L.Y + y) * 2 * nw;
    const uint32_t occ = row[nw + w];
    uint32_t v = 0;
    if (mode == ISF_INIT_UP) {
        v = occ;
    } else if (mode == ISF_INIT_RANDOM && occ) {
        const uint32_t sigma = (y & 1u) + 2u * (z & 1u);
        const uint32_t g0 = (z * L.Y + y) * (L.W / 4u) + 8u * w;  // as in the phase kernel
        for (int g = 0; g < 8; ++g) {
            if (!((occ >> (4 * g)) & 0xFu))
                continue;
            uint32_t u[4];
            philox(g0 + g, 0u, L.replica, sigma + 4u, L.key0, L.key1, u);
            for (int j = 0; j < 4; ++j)
                v |= (uint32_t)(u[j] < 0x80000000u) << (4 * g + j);
        }
        v &= occ;
    }
    row[w] = v;
}

// Recount of M, sum s n, occupied sites and occupied-neighbour pairs
// (grid-stride over all words, one set of atomics per block).
__global__ __launch_bounds__(256) void k_recount_bp(LatDev L, int64_t *out) {
    const uint64_t total = (uint64_t)L.Z * L.Y * L.nd;
    int64_t m = 0, sn = 0, no = 0, nb = 0;
    for (uint64_t g = blockIdx.x * 256u + threadIdx.x; g < total; g += (uint64_t)gridDim.x * 256u) {
        const uint32_t w = (uint32_t)(g % L.nd), row = (uint32_t)(g / L.nd);
        const uint32_t y = row % L.Y, z = row / L.Y;
        const bool left = (((y ^ z) & 1u) == 0);
        const NbBits r = gather_bp(reinterpret_cast<const uint32_t *>(L.spins), L.Y, L.nd, L.W, y, z, w, left);
        for (int i = 0; i < 32; ++i) {
            if (!((r.occ >> i) & 1u))
                continue;
            const int s = ((r.spin >> i) & 1u) ? 1 : -1;
            const int U = ((r.up.c0 >> i) & 1) | (((r.up.c1 >> i) & 1) << 1) | (((r.up.c2 >> i) & 1) << 2) |
                          (((r.up.c3 >> i) & 1) << 3);
            const int D = ((r.vac.c0 >> i) & 1) | (((r.vac.c1 >> i) & 1) << 1) | (((r.vac.c2 >> i) & 1) << 2) |
                          (((r.vac.c3 >> i) & 1) << 3);
            const int n = 2 * U + D - 12;
            m += s;
            sn += s * n;
            no += 1;
            nb += 12 - D;
        }
    }
    block_add4(out, m, sn, no, nb);
}

#define ISF_BP_TILINGS(X) \
    X(64, 4, 1) X(64, 4, 2) X(32, 8, 1) X(32, 8, 2) X(16, 16, 1) X(16, 16, 2) X(8, 32, 1) X(8, 32, 2) X(8, 16, 1) X(8, 8, 1)

static void grid_bp(const LatDev &L, const Tiling &tl, dim3 &g) {
    g.x = (L.nd + tl.tx - 1) / tl.tx;
    g.y = (L.Y / 2 + tl.ty * tl.ry - 1) / (tl.ty * tl.ry);
    g.z = (L.Z + 1) / 2;
}

hipError_t launch_phase_bp_pos(const LatDev &L, const Tiling &tl, uint32_t sigma, uint32_t q, hipStream_t s) {
    dim3 g;
    grid_bp(L, tl, g);
#define X(a, b, c)                                                                         \
    if (tl.tx == a && tl.ty == b && tl.ry == c) {                                          \
        hipLaunchKernelGGL((k_phase_bp_pos<a, b, c>), g, dim3(a * b), 0, s, L, sigma, q); \
        return hipGetLastError();                                                          \
    }
    ISF_BP_TILINGS(X)
#undef X
    return hipErrorInvalidValue;
}

void batch_grid_bp(const LatDev &L, const Tiling &tl, uint32_t &nbx, uint32_t &nby, uint32_t &nbz) {
    dim3 g;
    grid_bp(L, tl, g);
    nbx = g.x;
    nby = g.y;
    nbz = g.z;
}

hipError_t launch_phase_bp_batch(const BatchEntry *ents_dev, uint32_t n_ents, uint32_t total_blocks,
                                 const Tiling &tl, uint32_t sigma, hipStream_t s) {
#define X(a, b, c)                                                                                        \
    if (tl.tx == a && tl.ty == b && tl.ry == c) {                                                         \
        hipLaunchKernelGGL((k_phase_bp_batch<a, b, c>), dim3(total_blocks), dim3(a * b), 0, s, ents_dev, \
                           n_ents, sigma);                                                                \
        return hipGetLastError();                                                                         \
    }
    ISF_BP_TILINGS(X)
#undef X
    return hipErrorInvalidValue;
}

bool tiling_supported_bp(const Tiling &tl) {
#define X(a, b, c) \
    if (tl.tx == a && tl.ty == b && tl.ry == c) return true;
    ISF_BP_TILINGS(X)
#undef X
    return false;
}

hipError_t launch_init_bp(const LatDev &L, int32_t mode, hipStream_t s) {
    dim3 g((L.nd + 63) / 64, L.Y, L.Z);
    hipLaunchKernelGGL(k_init_bp, g, dim3(64), 0, s, L, mode);
    return hipGetLastError();
}

hipError_t launch_recount_bp(const LatDev &L, int64_t *out, hipStream_t s) {
    const uint64_t total = (uint64_t)L.Z * L.Y * L.nd;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>(2048, (total + 255) / 256);
    hipLaunchKernelGGL(k_recount_bp, dim3(blocks), dim3(256), 0, s, L, out);
    return hipGetLastError();
}

}  // namespace isf
