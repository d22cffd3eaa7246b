// Device helpers shared by the sweep kernels (INT8, BITPACK, persistent).
//
// Per-sweep bookkeeping: blocks add their flips' changes of M (-2 s_old) and
// E_bond (+2 s_old n) to 64 spread slots with relaxed agent-scope atomics;
// after the last sublattice of a sweep, one wave per film (a separate small
// launch, or a block after a grid barrier in the persistent kernel) folds the
// slots into M and E, advances the sweep counter, adds the sweep to the
// step's sums if it is kept, writes the step record when the step ends and
// stages the next step's threshold table.  Device-state accesses use
// agent-scope atomics so that the same code serves the persistent kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <climits>

#include "isf_internal.h"

namespace isf {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011).  The key and three of
// the four counter words are uniform across a wave, so the compiler keeps the
// key schedule and the first round's uniform product in scalar registers.
// Rounds [R0, R1) of Philox4x32-10 on the counter c (in place); (k0, k1) is
// the key of round 0.  Splitting the ten rounds lets a caller put other work
// between them; the result is the same.
template <int R0, int R1>
__device__ __forceinline__ void philox_rounds(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
    k0 += (uint32_t)R0 * 0x9E3779B9u;
    k1 += (uint32_t)R0 * 0xBB67AE85u;
#pragma unroll
    for (int r = R0; r < R1; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
        // three-input XOR in one gfx950 instruction (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c[1], k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c[3], k1, 0x96);
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Many calls share counter words 1 and 2 (sweep, replica) and differ in word 0
// (the site): the parts of rounds 0 and 1 that do not involve word 0 are the
// same for all of them and are computed once here.
struct PhiloxShared {
    uint32_t r0w0, r0w1;  // words 0 and 1 after round 0
    uint32_t r1hi, r1lo;  // the round-1 product of word 0 (high and low halves)
};

__device__ __forceinline__ PhiloxShared philox_shared(uint32_t c1, uint32_t c2, uint32_t k0) {
    PhiloxShared p;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    p.r0w0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    p.r0w1 = (uint32_t)p1;
    const uint64_t q0 = (uint64_t)0xD2511F53u * (uint64_t)p.r0w0;
    p.r1hi = (uint32_t)(q0 >> 32);
    p.r1lo = (uint32_t)q0;
    return p;
}

// Rounds 0 and 1 of the counter (c0, c1, c2, c3) from its shared part sh
// (made by philox_shared from c1, c2 and k0); rounds 2..9 follow with
// philox_rounds<2, 10>.
__device__ __forceinline__ void philox_first_two(uint32_t (&c)[4], uint32_t c0, uint32_t c3, const PhiloxShared &sh,
                                                 uint32_t k0, uint32_t k1) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;  // round 0
    const uint32_t w2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1, w3 = (uint32_t)p0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)w2;  // round 1
    c[0] = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), sh.r0w1, k0 + 0x9E3779B9u, 0x96);
    c[1] = (uint32_t)p1;
    c[2] = __builtin_amdgcn_bitop3_b32(sh.r1hi, w3, k1 + 0xBB67AE85u, 0x96);
    c[3] = sh.r1lo;
}

__device__ __forceinline__ void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                                       uint32_t out[4]) {
    uint32_t c[4] = {c0, c1, c2, c3};
    philox_rounds<0, 10>(c, k0, k1);
    out[0] = c[0];
    out[1] = c[1];
    out[2] = c[2];
    out[3] = c[3];
}

// Switching-field gate of Eq. (9) (steps 4-5 of the algorithm in Section 5):
// the four sites of dword k4 may flip only where their gate draws (Philox tag
// 2: counter word 3 = sigma + 8) are below the gate threshold gthr, which is
// word kGateWord of the table (kSentinel: no gate).  Returns the flip mask
// (byte j = 2 where site j passes).  Uphill thresholds, gate ones included,
// stay below kSentinel, so u < gthr is the exact test.
__device__ __forceinline__ uint32_t gate_mask(uint32_t gthr, uint32_t k4, uint32_t t, uint32_t replica,
                                              uint32_t sigma, uint32_t key0, uint32_t key1) {
    if (gthr == kSentinel)
        return 0x02020202u;
    uint32_t g[4];
    philox(k4, t, replica, sigma + 8u, key0, key1, g);
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        m |= g[j] < gthr ? (2u << (8 * j)) : 0u;
    return m;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

template <typename T>
__device__ __forceinline__ T ald(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void ast(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T aadd(T *p, T v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Anisotropy of Eq. (7) (Section 5), -h_an |M|, with M frozen at the start of
// each sublattice phase.  The phase's M is the state's M (folded at the end of
// the previous sweep) plus this sweep's slots (every block of the phases
// already done has added to them; a kernel boundary orders them).  A flip of
// spin s changes q by -an (|M - 2s| - |M|) / 2, so each half of the phase's
// table (s = -1: words 0..24, s = +1: words 25..49) is the step's table of
// q + an, of q, or of q - an:
//   M >= 2: s = +1 from q + an, s = -1 from q - an (a field h_an along M);
//   M <= -2: s = +1 from q - an, s = -1 from q + an;
//   M = 0: both from q - an (either flip raises |M|);
//   M = 1: s = +1 from q (|M| falls to 1), s = -1 from q - an;
//   M = -1: s = +1 from q - an, s = -1 from q.
// The loads are issued by one whole wave with the block's other loads, and
// the choice is made when they have landed, so the term adds no memory round
// trip to a phase.
static_assert(kSlots == 64, "one slot per lane of the wave that forms M");
struct AnisoLoads {
    int64_t dM, M;
    uint32_t plus, minus;  // word `lane` (< 50) of the tables of q + an and q - an
};

__device__ __forceinline__ AnisoLoads aniso_issue(const LatDev &L, uint32_t sigma, uint32_t lane) {
    AnisoLoads a;
    // the changes of M in this sweep's earlier phases (all of their blocks have
    // added them: earlier launches); this phase's blocks add to dM_phase[sigma]
    a.dM = 0;
    for (uint32_t j = 0; j < sigma; ++j)
        a.dM += L.slots[lane].dM_phase[j];
    a.M = L.st->M;
    a.plus = lane < 50 ? L.st->cur_atable[lane] : 0u;
    a.minus = lane < 50 ? L.st->cur_atable[50 + lane] : 0u;
    return a;
}

// Word `lane` of the phase's table, from word `base` of the step's plain table.
// Called by all 64 lanes of the wave that issued the loads.
__device__ __forceinline__ uint32_t aniso_select(const AnisoLoads &a, uint32_t base, uint32_t lane) {
    int64_t dM = a.dM;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        dM += __shfl_xor(dM, o, 64);
    const int64_t M = a.M + dM;
    if (lane >= 50)
        return base;  // the gate threshold and padding
    const bool up = lane >= 25;
    uint32_t src;  // 0: q, 1: q + an, 2: q - an
    if (M >= 2)
        src = up ? 1u : 2u;
    else if (M <= -2)
        src = up ? 2u : 1u;
    else if (M == 0)
        src = 2u;
    else if (M == 1)
        src = up ? 0u : 2u;
    else
        src = up ? 2u : 0u;
    return src == 0u ? base : (src == 1u ? a.plus : a.minus);
}

// Stage a film's current table and sweep counter into LDS.  Block-wide;
// ends with a barrier.  Returns false if the film's schedule is finished.
// kAtomic: the state may have been written earlier in the same launch (the
// persistent kernel); otherwise a kernel boundary already orders it.
template <bool kAtomic>
__device__ __forceinline__ bool stage_film(const LatDev &L, uint32_t *tab, uint32_t *t_sh, uint32_t *run_sh) {
    if (kAtomic) {
        if (threadIdx.x < kTableWords)
            tab[threadIdx.x] = ald(&L.st->cur_table[threadIdx.x]);
        if (threadIdx.x == 0) {
            *t_sh = (uint32_t)ald(&L.st->t);
            *run_sh = ald(&L.st->step) < ald(&L.st->n_steps);
        }
    } else {
        const DevState *st = L.st;
        if (threadIdx.x < kTableWords)
            tab[threadIdx.x] = st->cur_table[threadIdx.x];
        if (threadIdx.x == 0) {
            *t_sh = (uint32_t)st->t;
            *run_sh = st->step < st->n_steps;
        }
    }
    __syncthreads();
    return *run_sh != 0;
}

// Sweep end, run by the 64 lanes of one wave.  kAtomic: agent-scope atomics
// for state written earlier in the same launch (persistent kernel); plain
// accesses when a kernel boundary orders everything (separate launch).
template <bool kAtomic, typename T>
__device__ __forceinline__ T sld(const T *p) {
    if (kAtomic)
        return ald(p);
    return *p;
}
template <bool kAtomic, typename T>
__device__ __forceinline__ void sst(T *p, T v) {
    if (kAtomic)
        ast(p, v);
    else
        *p = v;
}

template <bool kAtomic>
__device__ inline void sweep_end(const LatDev &L) {
    const uint32_t lane = threadIdx.x & 63;
    int64_t dM = 0, dE = 0, acc = 0;
    for (uint32_t s = lane; s < kSlots; s += 64) {
        dM += sld<kAtomic>(&L.slots[s].dM);
        dE += sld<kAtomic>(&L.slots[s].dE);
        acc += sld<kAtomic>(&L.slots[s].acc);
        sst<kAtomic>(&L.slots[s].dM, (int64_t)0);
        sst<kAtomic>(&L.slots[s].dE, (int64_t)0);
        sst<kAtomic>(&L.slots[s].acc, (int64_t)0);
        if (L.aniso) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                sst<kAtomic>(&L.slots[s].dM_phase[j], (int64_t)0);
        }
    }
    dM = wave_sum(dM);
    dE = wave_sum(dE);
    acc = wave_sum(acc);
    DevState *st = L.st;
    uint32_t next_step = 0xFFFFFFFFu;
    if (lane == 0) {
        const int64_t M = sld<kAtomic>(&st->M) + dM;
        const int64_t E = sld<kAtomic>(&st->E) + dE;
        sst<kAtomic>(&st->M, M);
        sst<kAtomic>(&st->E, E);
        sst<kAtomic>(&st->t, sld<kAtomic>(&st->t) + 1);
        uint32_t step = sld<kAtomic>(&st->step);
        uint32_t sis = sld<kAtomic>(&st->sweep_in_step);
        const uint32_t n_steps = sld<kAtomic>(&st->n_steps);
        if (step < n_steps) {
            const uint32_t n_sweeps = sld<kAtomic>(&L.steps[step].n_sweeps);
            const uint32_t n_discard = sld<kAtomic>(&L.steps[step].n_discard);
            int64_t sM = sld<kAtomic>(&st->sum_M), sA = sld<kAtomic>(&st->sum_absM);
            int64_t sE = sld<kAtomic>(&st->sum_E), sC = sld<kAtomic>(&st->accepted);
            if (sis >= n_discard) {
                sM += M;
                sA += M < 0 ? -M : M;
                sE += E;
                sC += acc;
            }
            ++sis;
            if (sis >= n_sweeps) {
                isf_record *rec = &L.records[step];
                sst<kAtomic>(&rec->M, M);
                sst<kAtomic>(&rec->E, E);
                sst<kAtomic>(&rec->sum_M, sM);
                sst<kAtomic>(&rec->sum_absM, sA);
                sst<kAtomic>(&rec->sum_E, sE);
                sst<kAtomic>(&rec->accepted, sC);
                sM = sA = sE = sC = 0;
                ++step;
                sis = 0;
                if (step < n_steps)
                    next_step = step;
            }
            sst<kAtomic>(&st->sum_M, sM);
            sst<kAtomic>(&st->sum_absM, sA);
            sst<kAtomic>(&st->sum_E, sE);
            sst<kAtomic>(&st->accepted, sC);
            sst<kAtomic>(&st->step, step);
            sst<kAtomic>(&st->sweep_in_step, sis);
        }
    }
    next_step = __shfl(next_step, 0, 64);
    if (next_step != 0xFFFFFFFFu && lane < kTableWords)
        sst<kAtomic>(&st->cur_table[lane], sld<kAtomic>(&L.tables[(size_t)next_step * kTableWords + lane]));
    if (next_step != 0xFFFFFFFFu && L.aniso)
        for (uint32_t i = lane; i < kAnWords; i += 64)
            sst<kAtomic>(&st->cur_atable[i], sld<kAtomic>(&L.atables[(size_t)next_step * kAnWords + i]));
}

// Block reduction of the per-thread partial sums and the slot atomics.  No
// fence and no returning atomics here: the sweep end runs in a later launch
// (or after a grid barrier).  Measured on MI355X, folding the sweep end into
// the last sublattice launch costs more than the extra launch, whether the
// last block is found behind a device-scope fence per block (an L2 write-back
// each) or through returning atomics (a memory round trip before every block
// can retire).
// phase >= 0: an anisotropic sublattice phase, whose change of M also goes to
// the slot's dM_phase[phase] (read by the sweep's later phases).
template <int NT>
__device__ __forceinline__ void finish_block_to(Slot *slots, int dM, int dE, int acc, uint32_t block_in_lat,
                                                int phase = -1) {
    __shared__ int red[3][NT / 64];
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    dM = wave_sum(dM);
    dE = wave_sum(dE);
    acc = wave_sum(acc);
    if (lane == 0) {
        red[0][wid] = dM;
        red[1][wid] = dE;
        red[2][wid] = acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t sM = 0, sE = 0, sA = 0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) {
            sM += red[0][w];
            sE += red[1][w];
            sA += red[2][w];
        }
        if (sA) {
            Slot *slot = &slots[block_in_lat % kSlots];
            aadd(&slot->dM, sM);
            aadd(&slot->dE, sE);
            aadd(&slot->acc, sA);
            if (phase >= 0)
                aadd(&slot->dM_phase[phase], sM);
        }
    }
    __syncthreads();
}

template <int NT>
__device__ __forceinline__ void finish_block(const LatDev &L, int dM, int dE, int acc, uint32_t block_in_lat,
                                             int phase = -1) {
    finish_block_to<NT>(L.slots, dM, dE, acc, block_in_lat, phase);
}

// Block-wide sum of four 64-bit values into out[0..3] (256-thread blocks).
__device__ __forceinline__ void block_add4(int64_t *out, int64_t a, int64_t b, int64_t c, int64_t e) {
    __shared__ int64_t red[4][4];
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    e = wave_sum(e);
    if (lane == 0) {
        red[0][wid] = a;
        red[1][wid] = b;
        red[2][wid] = c;
        red[3][wid] = e;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int64_t v = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
        if (v)
            aadd(&out[threadIdx.x], v);
    }
}

// Linear block index -> film entry of a batched launch table (binary search).
template <typename Entry>
__device__ __forceinline__ uint32_t find_entry(const Entry *ents, uint32_t n, uint32_t b) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (ents[mid].block_begin <= b)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

}  // namespace isf
