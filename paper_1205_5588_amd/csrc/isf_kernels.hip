// HIP kernels for gfx950: Metropolis sweeps of the FCC-film Ising model.
//
// One launch updates one sublattice sigma = (y & 1) + 2 (z & 1) of a film
// (Section 5, steps 1-3 of the Metropolis algorithm, Eq. 8; Hamiltonian
// Eq. 3).  Sites of one sublattice share no bond, so every thread updates its
// sites independently; four launches make one sweep.  The work is a
// memory-bound integer stencil: no matrix cores.
//
// Layouts and the device state are described in isf_internal.h.
//
// Thread mapping: a thread owns one dword (4 consecutive compact sites of one
// row, which is exactly one Philox4x32-10 call) in each of `RY` active rows.
// A block is TX dwords x (TY * RY) active rows of one active plane; wave64
// lanes run along the row, so all loads and stores are coalesced dwords.
//
// Observables: each accepted flip changes M by -2 s_old and E_bond by
// +2 s_old n.  Blocks reduce these in registers and LDS and add them with
// relaxed agent-scope atomics to one of 64 slots (spread over 128-byte lines).
// After the last sublattice of a sweep a one-wave launch (k_sweep_end) folds
// the slots into M and E, advances the sweep counter, updates the step's sums
// and, at the end of a step, writes its record and stages the next step's
// threshold table.  The host never has to read anything back between sweeps,
// and every launch of a schedule has the same arguments.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "isf_tiles.h"

namespace isf {

template <int TX, int TY, int RY>
__global__ __launch_bounds__(TX *TY) void k_phase_i8(LatDev L, uint32_t sigma) {
    int dM = 0, dE = 0, acc = 0;
    phase_block_i8<TX, TY, RY, false>(L, sigma, blockIdx.x, blockIdx.y, blockIdx.z, dM, dE, acc);
    const uint32_t blin = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    finish_block<TX * TY>(L, dM, dE, acc, blin, L.aniso ? (int)sigma : -1);
}

// Batched: one launch covers the same sublattice of many films.  Block b
// belongs to the film whose block range contains it.
template <int TX, int TY, int RY>
__global__ __launch_bounds__(TX *TY) void k_phase_i8_batch(const BatchEntry *__restrict__ ents, uint32_t n_ents,
                                                           uint32_t sigma) {
    const uint32_t b = blockIdx.x;
    const BatchEntry &e = ents[find_entry(ents, n_ents, b)];
    const LatDev &L = e.lat;
    const uint32_t bl = b - e.block_begin;
    const uint32_t bx = bl % e.nbx, byz = bl / e.nbx;
    const uint32_t by = byz % e.nby, bz = byz / e.nby;
    int dM = 0, dE = 0, acc = 0;
    if (!phase_block_i8<TX, TY, RY, false>(L, sigma, bx, by, bz, dM, dE, acc))
        return;  // finished film: uniform over the block, and no other block of it counts either
    finish_block<TX * TY>(L, dM, dE, acc, bl);
}

// --------------------------------------------------------------------------
// One sublattice phase over the film's list of occupied dwords (INT8).  Each
// thread takes IPT consecutive-by-block list entries; every block holds
// exactly 256 * IPT entries (the last one fewer), so the work per block is the
// same wherever the film is dense or empty.  Entries are in row-major order,
// so a wave's loads stay coalesced along runs of occupied dwords.  kSmall:
// the spin buffer is below 4 GiB and byte offsets fit 32 bits.
template <int IPT, bool kSmall>
__global__ __launch_bounds__(256) void k_phase_i8_list(LatDev L, uint32_t sigma) {
    __shared__ uint32_t tab[kTableWords];
    __shared__ uint32_t t_sh;
    const uint32_t tid = threadIdx.x;
    uint32_t tabv = 0, tv = 0;
    if (tid < kTableWords)
        tabv = L.st->cur_table[tid];
    if (tid == 0)
        tv = (uint32_t)L.st->t;
    const bool aniso = L.aniso && tid < 64;  // uniform over each wave
    AnisoLoads an{};
    if (aniso)
        an = aniso_issue(L, sigma, tid);
    const uint32_t n = L.n_items[sigma];
    const uint32_t *items = L.items + L.items_off[sigma];
    const uint32_t Y = L.Y, nd = L.nd, rowb = nd * 4u;
    const size_t planeb = (size_t)Y * rowb;
    const bool left = (((sigma & 1u) ^ (sigma >> 1)) == 0);
    const uint32_t dbits = L.dbits, ybits = L.ybits;
    const uint32_t dmask = (1u << dbits) - 1u, ymask = (1u << ybits) - 1u;
    char *base = reinterpret_cast<char *>(L.spins);

    uint32_t A[IPT], S[IPT], pos[IPT];
    size_t self_off[IPT];
    bool ok[IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const uint32_t idx = (blockIdx.x * IPT + k) * 256u + tid;
        ok[k] = idx < n;
        const uint32_t it = n ? items[ok[k] ? idx : 0u] : 0u;
        const uint32_t d = it & dmask, y = (it >> dbits) & ymask, z = it >> (dbits + ybits);
        const uint32_t ym = y == 0 ? Y - 1 : y - 1;
        const uint32_t yp = y + 1 == Y ? 0 : y + 1;
        const uint32_t db = d * 4u;
        const uint32_t ddb = (left ? (d == 0 ? nd - 1 : d - 1) : (d + 1 == nd ? 0 : d + 1)) * 4u;
        const uint32_t oy = __umul24(y, rowb), om = __umul24(ym, rowb), op = __umul24(yp, rowb);
        const char *p0, *p2;
        char *p1;
        if (kSmall) {
            const uint32_t pl = (uint32_t)planeb;
            p1 = base + (uint32_t)((z + 1) * pl);
        } else {
            p1 = base + (size_t)(z + 1) * planeb;
        }
        p0 = p1 - planeb;
        p2 = p1 + planeb;
        uint32_t a = 0x01010101u, sum = 0;
        if (n) {
            const uint32_t a1 = ldw(p1, om + db), a1o = ldw(p1, om + ddb);
            const uint32_t a2 = ldw(p1, op + db), a2o = ldw(p1, op + ddb);
            const uint32_t b1 = ldw(p0, oy + db), b1o = ldw(p0, oy + ddb);
            const uint32_t b2 = ldw(p2, oy + db), b2o = ldw(p2, oy + ddb);
            const uint32_t e1 = ldw(p0, om + db), e2 = ldw(p0, op + db);
            const uint32_t e3 = ldw(p2, om + db), e4 = ldw(p2, op + db);
            a = ldw(p1, oy + db);
            sum = (a1 + a2) + (b1 + b2) + ((shifted(left, a1, a1o) + shifted(left, a2, a2o)) +
                                           (shifted(left, b1, b1o) + shifted(left, b2, b2o))) +
                  ((e1 + e2) + (e3 + e4));
        }
        A[k] = a;
        S[k] = sum;
        self_off[k] = (size_t)(p1 - base) + oy + db;
        pos[k] = __umul24(__umul24(z, Y) + y, nd) + d;  // Philox counter word 0 = k div 4
    }
    if (aniso)
        tabv = aniso_select(an, tabv, tid);
    if (tid < kTableWords)
        tab[tid] = tabv;
    if (tid == 0)
        t_sh = tv;
    __syncthreads();
    const uint32_t t = t_sh;
    const PhiloxShared psh = philox_shared(t, L.replica, L.key0);  // the parts of the counter every item shares
    int dM = 0, dE = 0, acc = 0;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const uint32_t a = A[k], sum = S[k];
        const uint32_t occ = ~a & 0x01010101u;
        if (!ok[k] || !occ)
            continue;
        uint32_t u[4];
        philox_first_two(u, pos[k], sigma, psh, L.key0, L.key1);
        philox_rounds<2, 10>(u, L.key0, L.key1);
        const uint32_t up = (a >> 1) & 0x01010101u;
        const uint32_t key = sum + up + (up << 3) + (up << 4);  // n + 12 + 25 [s = +1]
        uint32_t F = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            // downhill thresholds are kSentinel and every other one is below it,
            // so with u clamped to kSentinel - 1 one test is exact
            const uint32_t thr = tab[(key >> (8 * j)) & 0xFFu];
            F |= (min(u[j], kSentinel - 1u) < thr) ? (2u << (8 * j)) : 0u;
        }
        F &= occ << 1;
        if (F)
            F &= gate_mask(tab[kGateWord], pos[k], t, L.replica, sigma, L.key0, L.key1);
        if (F) {
            const uint32_t fu = F & a, fd = F ^ fu;
            const int cu = __popc(fu), cd = __popc(fd);
            const uint32_t su = __builtin_amdgcn_udot4(sum, fu >> 1, 0u, false);  // neighbour sums of the up flips
            const uint32_t sd = __builtin_amdgcn_udot4(sum, fd >> 1, 0u, false);  // and of the down flips
            dM += 2 * (cd - cu);
            dE += 2 * ((int)su - (int)sd) - 24 * (cu - cd);
            acc += cu + cd;
            *reinterpret_cast<uint32_t *>(base + self_off[k]) = a ^ F;
        }
    }
    finish_block<256>(L, dM, dE, acc, blockIdx.x, L.aniso ? (int)sigma : -1);
}

// --------------------------------------------------------------------------
// Sweep end of one film (one wave), or of every running film of a batch (one
// wave per film), launched after the last sublattice of each sweep.
__global__ __launch_bounds__(64) void k_sweep_end(LatDev L) { sweep_end<false>(L); }

__global__ __launch_bounds__(64) void k_sweep_end_batch(const BatchEntry *__restrict__ ents, uint32_t n_ents) {
    const LatDev &L = ents[blockIdx.x].lat;
    if (L.st->step < L.st->n_steps)
        sweep_end<false>(L);
}

// --------------------------------------------------------------------------
// Start: occupied sites get +1, -1, or +1 iff their INIT draw is below 2^31
// (counter word 3 = sigma + 4, sweep word 0).  Vacancies keep the byte 1.
__global__ void k_init_i8(LatDev L, int32_t mode) {
    const uint32_t d = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t y = blockIdx.y, z = blockIdx.z;
    if (d >= L.nd)
        return;
    uint32_t *P = reinterpret_cast<uint32_t *>(L.spins);
    const size_t idx = ((size_t)(z + 1) * L.Y + y) * L.nd + d;
    const uint32_t A = P[idx];
    const uint32_t occ = ~A & 0x01010101u;
    if (!occ)
        return;
    uint32_t v;
    if (mode == ISF_INIT_UP) {
        v = A | (occ << 1);          // 0 -> 2 on occupied bytes
        v &= ~(occ);                 // clear bit 0 (already 0 on occupied)
    } else if (mode == ISF_INIT_DOWN) {
        v = A & ~(occ * 3u);         // occupied bytes -> 0
    } else {
        const uint32_t sigma = (y & 1u) + 2u * (z & 1u);
        uint32_t u[4];
        philox((z * L.Y + y) * L.nd + d, 0u, L.replica, sigma + 4u, L.key0, L.key1, u);
        v = A;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if ((occ >> (8 * i)) & 1u) {
                const uint32_t byte = u[i] < 0x80000000u ? 2u : 0u;
                v = (v & ~(0xFFu << (8 * i))) | (byte << (8 * i));
            }
        }
    }
    P[idx] = v;
}

// Full recount of M, sum_i s_i n_i, occupied sites and occupied-neighbour
// pairs, from the spins alone.  Grid-stride over all dwords; one set of
// atomics per block.  out[4] must be zero on entry.
__global__ __launch_bounds__(256) void k_recount_i8(LatDev L, int64_t *out) {
    const uint64_t total = (uint64_t)L.Z * L.Y * L.nd;
    int64_t m = 0, sn = 0, no = 0, nb = 0;
    for (uint64_t g = blockIdx.x * 256u + threadIdx.x; g < total; g += (uint64_t)gridDim.x * 256u) {
        const uint32_t d = (uint32_t)(g % L.nd), row = (uint32_t)(g / L.nd);
        const uint32_t y = row % L.Y, z = row / L.Y;
        const bool left = (((y ^ z) & 1u) == 0);
        const Nb r = gather_i8<true>(reinterpret_cast<const uint32_t *>(L.spins), L.Y, L.nd, y, z, d, left);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int b = (r.self >> (8 * i)) & 0xFF;
            if (b == 1)
                continue;
            const int s = b - 1;
            const int n = (int)((r.sum >> (8 * i)) & 0xFFu) - 12;
            m += s;
            sn += s * n;
            no += 1;
            nb += (int)((r.occsum >> (8 * i)) & 0xFFu);
        }
    }
    block_add4(out, m, sn, no, nb);
}

// --------------------------------------------------------------------------
// Host-side launchers.

#define ISF_TILINGS(X) X(64, 4, 1) X(64, 4, 2) X(64, 4, 4) X(32, 8, 1) X(32, 8, 2) X(32, 8, 4) X(16, 16, 1) X(16, 16, 2) X(16, 16, 4)

static void grid_i8(const LatDev &L, const Tiling &tl, uint32_t sigma, dim3 &g) {
    const uint32_t half = L.Y / 2;
    const uint32_t nz = (L.Z + 1) / 2;  // active planes of pz = 0; pz = 1 has Z/2, extra blocks exit
    (void)sigma;
    g.x = (L.nd + tl.tx - 1) / tl.tx;
    g.y = (half + tl.ty * tl.ry - 1) / (tl.ty * tl.ry);
    g.z = nz;
}

hipError_t launch_phase_i8(const LatDev &L, const Tiling &tl, uint32_t sigma, hipStream_t s) {
    dim3 g;
    grid_i8(L, tl, sigma, g);
#define X(a, b, c)                                                                  \
    if (tl.tx == a && tl.ty == b && tl.ry == c) {                                   \
        hipLaunchKernelGGL((k_phase_i8<a, b, c>), g, dim3(a * b), 0, s, L, sigma); \
        return hipGetLastError();                                                   \
    }
    ISF_TILINGS(X)
#undef X
    return hipErrorInvalidValue;
}

void batch_grid_i8(const LatDev &L, const Tiling &tl, uint32_t &nbx, uint32_t &nby, uint32_t &nbz) {
    dim3 g;
    grid_i8(L, tl, 0, g);
    nbx = g.x;
    nby = g.y;
    nbz = g.z;
}

hipError_t launch_phase_i8_batch(const BatchEntry *ents_dev, uint32_t n_ents, uint32_t total_blocks,
                                 const Tiling &tl, uint32_t sigma, hipStream_t s) {
#define X(a, b, c)                                                                                        \
    if (tl.tx == a && tl.ty == b && tl.ry == c) {                                                         \
        hipLaunchKernelGGL((k_phase_i8_batch<a, b, c>), dim3(total_blocks), dim3(a * b), 0, s, ents_dev, \
                           n_ents, sigma);                                                                \
        return hipGetLastError();                                                                         \
    }
    ISF_TILINGS(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_sweep_end(const LatDev &L, hipStream_t s) {
    hipLaunchKernelGGL(k_sweep_end, dim3(1), dim3(64), 0, s, L);
    return hipGetLastError();
}

hipError_t launch_sweep_end_batch(const BatchEntry *ents_dev, uint32_t n_ents, hipStream_t s) {
    hipLaunchKernelGGL(k_sweep_end_batch, dim3(n_ents), dim3(64), 0, s, ents_dev, n_ents);
    return hipGetLastError();
}

hipError_t launch_phase_i8_list(const LatDev &L, uint32_t ipt, bool small, uint32_t sigma, hipStream_t s) {
    const uint32_t per_block = 256u * ipt;
    const uint32_t blocks = std::max<uint32_t>(1u, (L.n_items[sigma] + per_block - 1) / per_block);
    if (ipt == 1 && small)
        hipLaunchKernelGGL((k_phase_i8_list<1, true>), dim3(blocks), dim3(256), 0, s, L, sigma);
    else if (ipt == 1)
        hipLaunchKernelGGL((k_phase_i8_list<1, false>), dim3(blocks), dim3(256), 0, s, L, sigma);
    else if (ipt == 2 && small)
        hipLaunchKernelGGL((k_phase_i8_list<2, true>), dim3(blocks), dim3(256), 0, s, L, sigma);
    else if (ipt == 2)
        hipLaunchKernelGGL((k_phase_i8_list<2, false>), dim3(blocks), dim3(256), 0, s, L, sigma);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

bool tiling_supported(const Tiling &tl) {
#define X(a, b, c) \
    if (tl.tx == a && tl.ty == b && tl.ry == c) return true;
    ISF_TILINGS(X)
#undef X
    return false;
}

hipError_t launch_init_i8(const LatDev &L, int32_t mode, hipStream_t s) {
    dim3 g((L.nd + 255) / 256, L.Y, L.Z);
    hipLaunchKernelGGL(k_init_i8, g, dim3(256), 0, s, L, mode);
    return hipGetLastError();
}

hipError_t launch_recount_i8(const LatDev &L, int64_t *out, hipStream_t s) {
    const uint64_t total = (uint64_t)L.Z * L.Y * L.nd;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>(2048, (total + 255) / 256);
    hipLaunchKernelGGL(k_recount_i8, dim3(blocks), dim3(256), 0, s, L, out);
    return hipGetLastError();
}

}  // namespace isf
