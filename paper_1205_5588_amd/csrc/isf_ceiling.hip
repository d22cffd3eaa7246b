// The draw-only ceiling of a sweep: every stored dword of a film draws its
// Philox4x32-10 numbers for n sweeps, exactly as an attempt would (counter
// (site dword, sweep, replica, sublattice), Section 5's uniform random number
// for each site), and nothing else happens.  The four words of every call are
// XORed into one 32-bit checksum, so the draws cannot be skipped and the
// result can be checked against any other implementation of the generator.
//
// A sweep draws once per four compact sites, vacancies included here (the
// sweep kernels skip dwords with no occupied site), so one launch per n
// sweeps bounds what the integer ALU can do when the stencil, the table
// lookups and the observables cost nothing.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "isf_device.h"
#include "isf_internal.h"

namespace isf {

// One block per row (z, y) of the film (grid-stride), one thread per dword.
__global__ __launch_bounds__(256) void k_draw_xor(uint32_t Y, uint32_t Z, uint32_t nd, uint32_t replica, uint32_t key0,
                                                  uint32_t key1, uint32_t t0, uint32_t n_sweeps, uint32_t *out) {
    uint32_t x = 0;
    for (uint32_t i = 0; i < n_sweeps; ++i) {
        const uint32_t t = t0 + i;
        const PhiloxShared psh = philox_shared(t, replica, key0);
        for (uint32_t r = blockIdx.x; r < Y * Z; r += gridDim.x) {
            const uint32_t z = r / Y, y = r - z * Y;
            const uint32_t sigma = (y & 1u) + 2u * (z & 1u);
            for (uint32_t d = threadIdx.x; d < nd; d += 256) {
                uint32_t u[4];
                philox_first_two(u, r * nd + d, sigma, psh, key0, key1);
                philox_rounds<2, 10>(u, key0, key1);
                x ^= (u[0] ^ u[1]) ^ (u[2] ^ u[3]);
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        x ^= __shfl_xor(x, o, 64);
    if ((threadIdx.x & 63u) == 0 && x)
        atomicXor(out, x);
}

__global__ void k_clear_word(uint32_t *p) { *p = 0u; }

hipError_t launch_draw_xor(const LatDev &L, uint32_t t0, uint32_t n_sweeps, uint32_t *out, uint32_t n_cu,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(1), 0, s, out);
    const uint32_t rows = L.Y * L.Z, nd = L.W / 4;
    const uint32_t blocks = rows < 8u * n_cu ? rows : 8u * n_cu;
    hipLaunchKernelGGL(k_draw_xor, dim3(blocks), dim3(256), 0, s, L.Y, L.Z, nd, L.replica, L.key0, L.key1, t0,
                       n_sweeps, out);
    return hipGetLastError();
}

}  // namespace isf
