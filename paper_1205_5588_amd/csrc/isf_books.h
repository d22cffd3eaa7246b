// Per-sweep bookkeeping of the launches that carry their own books (the
// whole-sweep kernels, and the per-sublattice bit-packed launches whose first
// sublattice folds the sweep before): a sweep of parity q runs at position
// pos[q] and adds into slots_of(q); wave 0 of block 0 of the sweep after it
// folds those slots into the film state and its step record and writes the
// position of the sweep after that into pos[1 - q].  k_whole_prime opens a run
// of such launches and k_whole_flush closes it.
#pragma once

#include "isf_device.h"

namespace isf {

__device__ __forceinline__ Slot *slots_of(const LatDev &L, uint32_t parity) { return parity ? L.slots2 : L.slots; }

// The per-sweep bookkeeping's inputs, staged in LDS by wave 0 of block 0:
// the previous sweep's position (words 0-7), this sweep's position (8-15),
// the film state's first 18 words (16-33: M, E, t, step, sweep_in_step, the
// step's sums, n_steps) and the previous sweep's 64 slots.  The loads are
// issued before the block's region loads and stored once those have landed,
// so they add neither latency nor live registers to the sweep.
constexpr int kBookWords = 34;
struct BookLds {
    uint32_t w[kBookWords];
    int64_t dM[kSlots], dE[kSlots], acc[kSlots];
};
static_assert(offsetof(SweepPos, pending) == 28 && offsetof(SweepPos, t) == 0, "position words");
static_assert(offsetof(DevState, M) == 0 && offsetof(DevState, sum_M) == 32 && offsetof(DevState, accepted) == 56 &&
                  offsetof(DevState, n_steps) == 68,
              "film state words");

struct BookRegs {
    uint32_t w;
    int64_t dM, dE, acc;
};

__device__ __forceinline__ BookRegs book_issue(const LatDev &L, uint32_t prev, uint32_t cur, uint32_t lane) {
    BookRegs r;
    const uint32_t *src = lane < 8    ? reinterpret_cast<const uint32_t *>(&L.pos[prev]) + lane
                          : lane < 16 ? reinterpret_cast<const uint32_t *>(&L.pos[cur]) + (lane - 8)
                                      : reinterpret_cast<const uint32_t *>(L.st) + (lane - 16);
    r.w = lane < (uint32_t)kBookWords ? *src : 0u;
    const Slot &sl = slots_of(L, prev)[lane];  // kSlots == 64: one slot per lane
    r.dM = sl.dM;
    r.dE = sl.dE;
    r.acc = sl.acc;
    return r;
}

__device__ __forceinline__ void book_stage(BookLds &bk, const BookRegs &r, uint32_t lane) {
    if (lane < (uint32_t)kBookWords)
        bk.w[lane] = r.w;
    bk.dM[lane] = r.dM;
    bk.dE[lane] = r.dE;
    bk.acc[lane] = r.acc;
}

__device__ __forceinline__ int64_t w64(const BookLds &bk, int i) {
    return (int64_t)((uint64_t)bk.w[i] | ((uint64_t)bk.w[i + 1] << 32));
}

// Fold the previous sweep (parity prev) into M, E, the step's sums and, if it
// ended its step, the step's record; clear its slots.  One wave.
__device__ __forceinline__ void book_fold(const LatDev &L, uint32_t prev, const BookLds &bk, uint32_t lane) {
    const int64_t dM = wave_sum(bk.dM[lane]), dE = wave_sum(bk.dE[lane]), acc = wave_sum(bk.acc[lane]);
    Slot *ps = slots_of(L, prev);
    ps[lane].dM = 0;
    ps[lane].dE = 0;
    ps[lane].acc = 0;
    const uint32_t p_step = bk.w[2], p_sis = bk.w[3], p_ns = bk.w[4], p_nd = bk.w[5], p_run = bk.w[6];
    const uint32_t p_pending = bk.w[7];
    if (lane == 0 && p_pending) {
        DevState *st = L.st;
        const int64_t M0 = w64(bk, 16), M = M0 + dM, E = w64(bk, 18) + dE;
        st->M = M;
        st->E = E;
        const int64_t margin = (M0 < 0 ? -M0 : M0) - 2 * acc;
        if (margin < st->spec_margin)
            st->spec_margin = margin;
        if (p_run) {
            int64_t sM = w64(bk, 24), sA = w64(bk, 26), sE = w64(bk, 28), sC = w64(bk, 30);
            if (p_sis >= p_nd) {
                sM += M;
                sA += M < 0 ? -M : M;
                sE += E;
                sC += acc;
            }
            if (p_sis + 1 >= p_ns) {
                isf_record *rec = &L.records[p_step];
                rec->M = M;
                rec->E = E;
                rec->sum_M = sM;
                rec->sum_absM = sA;
                rec->sum_E = sE;
                rec->accepted = sC;
                sM = sA = sE = sC = 0;
            }
            st->sum_M = sM;
            st->sum_absM = sA;
            st->sum_E = sE;
            st->accepted = sC;
        }
        L.pos[prev].pending = 0;
    }
}

// Write the position of the sweep after the current one (parity cur) into
// pos[1 - cur]; tab holds the current sweep's thresholds.  One wave.
__device__ __forceinline__ void book_advance(const LatDev &L, uint32_t cur, const BookLds &bk, const uint32_t *tab,
                                             uint32_t lane) {
    uint32_t next_step = 0xFFFFFFFFu;
    if (lane == 0) {
        uint32_t step = bk.w[10], sis = bk.w[11], ns = bk.w[12], nd = bk.w[13], run = bk.w[14];
        const uint32_t n_steps = bk.w[33];
        if (run) {
            if (++sis >= ns) {
                ++step;
                sis = 0;
                run = step < n_steps;
                if (run) {
                    ns = L.steps[step].n_sweeps;
                    nd = L.steps[step].n_discard;
                    next_step = step;
                }
            }
        }
        // a launch after the film's schedule ended (batches) is no sweep: the
        // position stays and nothing waits to be folded
        const uint32_t ran = bk.w[14];
        SweepPos &np = L.pos[1 - cur];
        np.t = (uint64_t)w64(bk, 8) + ran;
        np.step = step;
        np.sis = sis;
        np.n_sweeps = ns;
        np.n_discard = nd;
        np.run = run;
        np.pending = 0;
        L.pos[cur].pending = ran;  // this sweep's slots wait for the next fold
    }
    next_step = __shfl(next_step, 0, 64);
    if (lane < kTableWords)
        L.pos[1 - cur].table[lane] =
            next_step != 0xFFFFFFFFu ? L.tables[(size_t)next_step * kTableWords + lane] : tab[lane];
}

// book_advance with its loads done in advance: cur_tab / next_tab hold word
// `lane` of the current and of the next step's table, next_ns / next_nd the
// next step's sweeps (valid where that step exists).
__device__ __forceinline__ void book_advance_pre(const LatDev &L, uint32_t cur, const BookLds &bk, uint32_t cur_tab,
                                                 uint32_t next_tab, uint32_t next_ns, uint32_t next_nd,
                                                 uint32_t lane) {
    uint32_t changed = 0;
    if (lane == 0) {
        uint32_t step = bk.w[10], sis = bk.w[11], ns = bk.w[12], nd = bk.w[13], run = bk.w[14];
        const uint32_t n_steps = bk.w[33];
        if (run) {
            if (++sis >= ns) {
                ++step;
                sis = 0;
                run = step < n_steps;
                if (run) {
                    ns = next_ns;
                    nd = next_nd;
                    changed = 1;
                }
            }
        }
        const uint32_t ran = bk.w[14];  // see book_advance: a launch past the schedule is no sweep
        SweepPos &np = L.pos[1 - cur];
        np.t = (uint64_t)w64(bk, 8) + ran;
        np.step = step;
        np.sis = sis;
        np.n_sweeps = ns;
        np.n_discard = nd;
        np.run = run;
        np.pending = 0;
        L.pos[cur].pending = ran;
    }
    changed = __shfl(changed, 0, 64);
    if (lane < kTableWords)
        L.pos[1 - cur].table[lane] = changed ? next_tab : cur_tab;
}

}  // namespace isf
