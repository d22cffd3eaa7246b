// Observables of the film state beyond M and E: the simulated PMOKE image of
// Section 6.  Only surface atoms are shown, white (+1) for spin up and black
// (-1) for spin down; the surface atom of column (x, y) is its occupied site
// with the largest z, and a column without one is background (0).
//
// One thread per pixel, consecutive threads along x; sites of column (x, y)
// exist only at z = x + y (mod 2), so a thread visits every other plane from
// the top down and stops at the first occupied one.  Reads at most Z/2 bytes
// (INT8) or bits (BITPACK) per pixel and writes one byte: HBM-bound and tiny
// next to a sweep.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "isf_internal.h"

namespace isf {

__global__ __launch_bounds__(256) void k_surface_i8(const uint8_t *__restrict__ spins, uint32_t X, uint32_t Y,
                                                    uint32_t Z, int8_t *__restrict__ img) {
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= X)
        return;
    const uint32_t W = X / 2, j = x >> 1;
    const size_t planeb = (size_t)Y * W;
    int8_t v = 0;
    // the top plane whose sites sit in this column: z + x + y even
    for (int z = (int)Z - 1 - (int)((Z - 1 + x + y) & 1u); z >= 0; z -= 2) {
        const uint8_t b = spins[(size_t)(z + 1) * planeb + (size_t)y * W + j];
        if (b != 1) {  // 1 is a vacancy; 0 / 2 are spin -1 / +1
            v = (int8_t)((int)b - 1);
            break;
        }
    }
    img[(size_t)y * X + x] = v;
}

__global__ __launch_bounds__(256) void k_surface_bp(const uint32_t *__restrict__ words, uint32_t X, uint32_t Y,
                                                    uint32_t Z, int8_t *__restrict__ img) {
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= X)
        return;
    const uint32_t nw = (X / 2 + 31) / 32, j = x >> 1, w = j >> 5, bit = j & 31u;
    int8_t v = 0;
    for (int z = (int)Z - 1 - (int)((Z - 1 + x + y) & 1u); z >= 0; z -= 2) {
        const uint32_t *row = words + ((size_t)(z + 1) * Y + y) * 2 * nw;  // spin words, then occupancy words
        if ((row[nw + w] >> bit) & 1u) {
            v = ((row[w] >> bit) & 1u) ? (int8_t)1 : (int8_t)-1;
            break;
        }
    }
    img[(size_t)y * X + x] = v;
}

// Image [Y][X] of the film whose current spins are at `spins` (its layout is L's).
hipError_t launch_surface_image(const LatDev &L, const uint8_t *spins, int8_t *img, hipStream_t s) {
    const dim3 grid((L.X + 255) / 256, L.Y);
    if (L.format == ISF_FORMAT_INT8)
        hipLaunchKernelGGL(k_surface_i8, grid, dim3(256), 0, s, spins, L.X, L.Y, L.Z, img);
    else
        hipLaunchKernelGGL(k_surface_bp, grid, dim3(256), 0, s, reinterpret_cast<const uint32_t *>(spins), L.X, L.Y,
                           L.Z, img);
    return hipGetLastError();
}

}  // namespace isf
