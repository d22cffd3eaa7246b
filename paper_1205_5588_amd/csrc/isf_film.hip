// HIP kernels for gfx950: the whole film in one block's LDS, many sweeps per
// launch (INT8 format).
//
// For films small enough that their planes fit one compute unit's LDS (the
// 64 x 64 x 3 ramp film takes 10 KiB), a sweep is bound by launch and memory
// latency, not by work: one launch per sweep costs about 9 us where the four
// phases' attempts take a fraction of that.  Here one block loads the film
// once and then runs sweep after sweep from LDS: the four phases of a sweep
// with a block barrier between them (the periodic x and y wrap done on the
// indices), the block's sums reduced after the fourth, and the books of the
// sweep (M, E, the step's sums, the record at a step's end, the next step's
// thresholds) kept by every thread alike, exactly as the one-wave sweep-end
// launch of the per-sublattice kernels keeps them.  The film and the state go
// back to memory at the end of the launch.
//
// Two forms.  Where no sublattice has more than one dword per thread (the
// resident form), each thread keeps its dword of each sublattice decoded in
// registers for the whole launch and draws the four phases' random numbers
// together at the top of a sweep (the draws do not depend on the spins), four
// independent Philox chains that fill the issue slots two waves per SIMD leave
// empty.  Otherwise the block lists each sublattice's occupied dwords once
// (occupancy never changes) and the threads stride over the lists.
//
// Draws, thresholds, the acceptance test and the visiting order are those of
// the per-sublattice kernels (a sublattice's dwords have no neighbours in the
// same sublattice, so their order inside a phase does not matter), so the
// trajectory is identical to theirs.  The anisotropy term of Eq. (7) is not
// taken here (the host refuses it for this kernel).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "isf_tiles.h"

namespace isf {

constexpr int kFilmNT = 512;  // threads of the block (8 waves)

// A dword of the film in LDS and its neighbour offsets: rows y - 1 and y + 1
// (dym, dyp) and the dword across the column seam (ddx), each as a difference
// of indices modulo 2^32, so that the periodic wraps cost nothing per attempt.
struct FilmItem {
    uint32_t idx, dym, dyp, ddx, k4;
};

// Dword d of row y of LDS plane p (film plane p - 1), of sublattice s.
__device__ __forceinline__ FilmItem film_item_at(uint32_t p, uint32_t y, uint32_t d, uint32_t s, uint32_t Y,
                                                 uint32_t nd) {
    const uint32_t PLn = Y * nd;
    const bool left = ((s & 1u) ^ (s >> 1)) == 0;
    const uint32_t ym = y == 0 ? Y - 1 : y - 1, yp = y + 1 == Y ? 0 : y + 1;
    const uint32_t dd = left ? (d == 0 ? nd - 1 : d - 1) : (d + 1 == nd ? 0 : d + 1);
    FilmItem it;
    it.idx = p * PLn + y * nd + d;
    it.dym = (ym - y) * nd;
    it.dyp = (yp - y) * nd;
    it.ddx = dd - d;
    it.k4 = ((p - 1u) * Y + y) * nd + d;  // the film dword of the per-sublattice kernels
    return it;
}

// Sublattice s's dword c (c < nz (Y / 2) nd) decoded.
__device__ __forceinline__ FilmItem film_item(uint32_t c, uint32_t s, uint32_t Y, uint32_t nd) {
    const uint32_t half = Y / 2;
    const uint32_t d = c % nd, r = c / nd, yy = r % half, zz = r / half;
    return film_item_at(2u * zz + (s >> 1) + 1u, 2u * yy + (s & 1u), d, s, Y, nd);
}

// The attempt on one dword (four sites) of sublattice s with its draws u.
__device__ __forceinline__ void film_attempt(uint32_t *F, const FilmItem &it, uint32_t PLn, uint32_t s,
                                             const uint32_t (&u)[4], uint32_t tt, const uint32_t *tab,
                                             const LatDev &L, int &dM, int &dE, int &acc) {
    const bool left = ((s & 1u) ^ (s >> 1)) == 0;
    const uint32_t i = it.idx, b = i - PLn, c = i + PLn;
    const uint32_t a1 = F[i + it.dym], a1o = F[i + it.dym + it.ddx];
    const uint32_t a2 = F[i + it.dyp], a2o = F[i + it.dyp + it.ddx];
    const uint32_t b1 = F[b], b1o = F[b + it.ddx];
    const uint32_t b2 = F[c], b2o = F[c + it.ddx];
    const uint32_t e1 = F[b + it.dym], e2 = F[b + it.dyp];
    const uint32_t e3 = F[c + it.dym], e4 = F[c + it.dyp];
    const uint32_t a = F[i];
    const uint32_t sum = (a1 + a2) + (b1 + b2) +
                         ((shifted(left, a1, a1o) + shifted(left, a2, a2o)) +
                          (shifted(left, b1, b1o) + shifted(left, b2, b2o))) +
                         ((e1 + e2) + (e3 + e4));
    const uint32_t up = (a >> 1) & 0x01010101u;
    const uint32_t key = sum + up + (up << 3) + (up << 4);  // n + 12 + 25 [s = +1]
    uint32_t f = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        // downhill thresholds are kSentinel and every other one is below it
        const uint32_t thr = tab[(key >> (8 * j)) & 0xFFu];
        f |= (min(u[j], kSentinel - 1u) < thr) ? (2u << (8 * j)) : 0u;
    }
    f &= (~a & 0x01010101u) << 1;  // vacancies never flip
    if (f)
        f &= gate_mask(tab[kGateWord], it.k4, tt, L.replica, s, L.key0, L.key1);
    if (f) {
        const uint32_t fu = f & a, fdn = f ^ fu;
        const int cu = __popc(fu), cd = __popc(fdn);
        const uint32_t su = __builtin_amdgcn_udot4(sum, fu >> 1, 0u, false);
        const uint32_t sd = __builtin_amdgcn_udot4(sum, fdn >> 1, 0u, false);
        dM += 2 * (cd - cu);
        dE += 2 * ((int)su - (int)sd) - 24 * (cu - cd);
        acc += cu + cd;
        F[i] = a ^ f;
    }
}

// Dwords of sublattice s: nz (Y / 2) nd, nz its planes.
__device__ __forceinline__ uint32_t film_sub_dwords(uint32_t s, uint32_t Y, uint32_t Z, uint32_t nd) {
    return (Z - (s >> 1) + 1) / 2 * (Y / 2) * nd;
}

// n_sweeps sweeps of film L (its state in L.st) by one block.
template <bool kRes>
__global__ __launch_bounds__(kFilmNT) void k_sweep_i8_film(LatDev L, uint32_t n_sweeps) {
    extern __shared__ __align__(16) uint8_t smb[];
    __shared__ uint32_t tab[kTableWords];
    __shared__ int red[2][3][kFilmNT / 64];
    __shared__ uint32_t cnt[4];

    const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid >> 6;
    const uint32_t Y = L.Y, Z = L.Z, nd = L.nd;
    const uint32_t PLn = Y * nd, total = (Z + 2) * PLn;  // the host checks total <= 65536
    uint32_t *F = reinterpret_cast<uint32_t *>(smb);
    uint16_t *lst = reinterpret_cast<uint16_t *>(smb + 4u * total);  // the list form only
    const uint32_t cap = (Z + 1) / 2 * (Y / 2) * nd;                 // most dwords of one sublattice
    const uint32_t *g = reinterpret_cast<const uint32_t *>(L.spins);

    for (uint32_t i = tid; i < total; i += kFilmNT)
        F[i] = g[i];
    if (tid < 4)
        cnt[tid] = 0;
    if (tid < kTableWords)
        tab[tid] = L.st->cur_table[tid];
    // the books: every thread holds the same copy
    const DevState *st = L.st;
    int64_t M = st->M, E = st->E, sM = st->sum_M, sA = st->sum_absM, sE = st->sum_E, sC = st->accepted;
    uint64_t t = st->t;
    uint32_t step = st->step, sis = st->sweep_in_step;
    const uint32_t n_steps = st->n_steps;
    uint32_t ns = 0, ndis = 0;
    if (step < n_steps) {
        ns = L.steps[step].n_sweeps;
        ndis = L.steps[step].n_discard;
    }
    __syncthreads();

    FilmItem it[4];
    bool ok[4];
    if constexpr (kRes) {
        // thread tid takes dword tid of each sublattice (cap <= kFilmNT)
#pragma unroll
        for (uint32_t s = 0; s < 4; ++s) {
            const uint32_t c = tid < film_sub_dwords(s, Y, Z, nd) ? tid : 0u;
            it[s] = film_item(c, s, Y, nd);
            ok[s] = tid < film_sub_dwords(s, Y, Z, nd) && F[it[s].idx] != 0x01010101u;
        }
    } else {
        // occupied dwords of each sublattice, as indices into F
        for (uint32_t s = 0; s < 4; ++s) {
            const uint32_t n = film_sub_dwords(s, Y, Z, nd);
            for (uint32_t c0 = 0; c0 < n; c0 += kFilmNT) {
                const uint32_t c = c0 + tid;
                uint32_t idx = 0;
                bool occ = false;
                if (c < n) {
                    idx = film_item(c, s, Y, nd).idx;
                    occ = F[idx] != 0x01010101u;
                }
                const uint64_t m = __ballot(occ);
                if (m) {
                    const uint32_t below =
                        __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    uint32_t base = 0;
                    if (below == 0 && occ)
                        base = atomicAdd(&cnt[s], (uint32_t)__popcll(m));
                    base = __shfl(base, (int)__builtin_ctzll(m), 64);
                    if (occ)
                        lst[s * cap + base + below] = (uint16_t)idx;
                }
            }
        }
        __syncthreads();
    }

    for (uint32_t k = 0; k < n_sweeps; ++k) {
        int dM = 0, dE = 0, acc = 0;
        const bool run = step < n_steps;  // uniform
        if (run) {
            const uint32_t tt = (uint32_t)t;
            const PhiloxShared psh = philox_shared(tt, L.replica, L.key0);
            if constexpr (kRes) {
                uint32_t u[4][4];
#pragma unroll
                for (uint32_t s = 0; s < 4; ++s) {
                    philox_first_two(u[s], it[s].k4, s, psh, L.key0, L.key1);
                    philox_rounds<2, 10>(u[s], L.key0, L.key1);
                }
#pragma unroll
                for (uint32_t s = 0; s < 4; ++s) {
                    if (ok[s])
                        film_attempt(F, it[s], PLn, s, u[s], tt, tab, L, dM, dE, acc);
                    if (s < 3)
                        __syncthreads();  // the phase's flips, before the next phase reads them
                }
            } else {
                for (uint32_t s = 0; s < 4; ++s) {
                    const uint32_t n = cnt[s];
                    for (uint32_t i = tid; i < n; i += kFilmNT) {
                        const uint32_t idx = lst[s * cap + i];
                        const uint32_t p = idx / PLn, rem = idx - p * PLn, y = rem / nd;
                        const FilmItem fi = film_item_at(p, y, rem - y * nd, s, Y, nd);
                        uint32_t u[4];
                        philox_first_two(u, fi.k4, s, psh, L.key0, L.key1);
                        philox_rounds<2, 10>(u, L.key0, L.key1);
                        film_attempt(F, fi, PLn, s, u, tt, tab, L, dM, dE, acc);
                    }
                    if (s < 3)
                        __syncthreads();
                }
            }
        }
        // the block's sums of the sweep (two buffers: a sweep that does not run
        // has no barrier between its writes and the last reads of the one before)
        dM = wave_sum(dM);
        dE = wave_sum(dE);
        acc = wave_sum(acc);
        const uint32_t rb = k & 1u;
        if (lane == 0) {
            red[rb][0][wid] = dM;
            red[rb][1][wid] = dE;
            red[rb][2][wid] = acc;
        }
        __syncthreads();  // the fourth phase's flips and the sums
        int64_t bM = 0, bE = 0, bA = 0;
#pragma unroll
        for (int w = 0; w < kFilmNT / 64; ++w) {
            bM += red[rb][0][w];
            bE += red[rb][1][w];
            bA += red[rb][2][w];
        }
        // the sweep end of the per-sublattice kernels
        M += bM;
        E += bE;
        ++t;
        if (run) {
            if (sis >= ndis) {
                sM += M;
                sA += M < 0 ? -M : M;
                sE += E;
                sC += bA;
            }
            ++sis;
            if (sis >= ns) {
                if (tid == 0) {
                    isf_record *rec = &L.records[step];
                    rec->M = M;
                    rec->E = E;
                    rec->sum_M = sM;
                    rec->sum_absM = sA;
                    rec->sum_E = sE;
                    rec->accepted = sC;
                }
                sM = sA = sE = sC = 0;
                ++step;
                sis = 0;
                if (step < n_steps) {  // uniform
                    ns = L.steps[step].n_sweeps;
                    ndis = L.steps[step].n_discard;
                    if (tid < kTableWords)  // the next step's thresholds
                        tab[tid] = L.tables[(size_t)step * kTableWords + tid];
                    __syncthreads();
                }
            }
        }
    }
    __syncthreads();

    uint32_t *gw = reinterpret_cast<uint32_t *>(L.spins);
    for (uint32_t i = PLn + tid; i < (Z + 1) * PLn; i += kFilmNT)
        gw[i] = F[i];
    if (tid < kTableWords)
        L.st->cur_table[tid] = tab[tid];
    if (tid == 0) {
        DevState *sw = L.st;
        sw->M = M;
        sw->E = E;
        sw->t = t;
        sw->step = step;
        sw->sweep_in_step = sis;
        sw->sum_M = sM;
        sw->sum_absM = sA;
        sw->sum_E = sE;
        sw->accepted = sC;
    }
}

// The resident form: every sublattice has at most one dword per thread.
static bool film_resident(uint32_t Y, uint32_t Z, uint32_t nd) {
    return (uint64_t)(Z + 1) / 2 * (Y / 2) * nd <= (uint64_t)kFilmNT;
}

// LDS bytes of the film kernel for a film (0: it does not fit one block).
uint32_t film_lds_bytes(uint32_t Y, uint32_t Z, uint32_t nd, uint32_t max_lds) {
    const uint64_t total = (uint64_t)(Z + 2) * Y * nd;
    const uint64_t cap = (uint64_t)(Z + 1) / 2 * (Y / 2) * nd;
    const uint64_t bytes = 4 * total + (film_resident(Y, Z, nd) ? 0 : 2 * 4 * cap);
    const uint32_t fixed = 2048;  // the static LDS of the kernel, with room to spare
    if (total > 65536 || bytes + fixed > max_lds)
        return 0;
    return (uint32_t)bytes;
}

hipError_t launch_sweep_i8_film(const LatDev &L, uint32_t n_sweeps, uint32_t lds, hipStream_t s) {
    if (film_resident(L.Y, L.Z, L.nd))
        hipLaunchKernelGGL(k_sweep_i8_film<true>, dim3(1), dim3(kFilmNT), lds, s, L, n_sweeps);
    else
        hipLaunchKernelGGL(k_sweep_i8_film<false>, dim3(1), dim3(kFilmNT), lds, s, L, n_sweeps);
    return hipGetLastError();
}

}  // namespace isf
