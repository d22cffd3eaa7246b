// Internal layout shared by the host side of the library and its HIP kernels.
//
// Storage of one film (INT8 format), in the caller's spin buffer:
//   compact rows: site (x, y, z) with x+y+z even lives in row (y, z) at column
//   j = x / 2, so a row holds W = X/2 bytes and X = 2j + ((y+z) & 1);
//   planes z = -1 and z = Z are padding rows of vacancies, so the buffer is
//   [Z+2][Y][W] bytes and the open z boundary needs no test in the kernels;
//   a byte holds s + 1 for an occupied site (0: down, 2: up) and 1 for a
//   vacancy, so the sum of the 12 neighbour bytes of a site is n + 12 in
//   [0, 24] (a vacancy adds 1 = 0 + 1).  Four sites share one dword and
//   twelve dwords add without carries between bytes.
//
// BITPACK format: per row two bit planes of W bits (nw = ceil(W/32) words
//   each): spin bit (1 = up) and occupancy bit; the bits of the last word past
//   column W - 1 and the planes z = -1 and z = Z are zero.  Layout
//   [Z+2][Y][2][nw] uint32 (spin words then occupancy words).
//
// Neighbours of the site at row (y, z), column j (p = (y+z) & 1, delta = -1
// if p == 0 else +1, columns mod W): rows (y+-1, z) and (y, z+-1) at columns
// j and j+delta; rows (y+-1, z+-1) at column j.
#pragma once

#include <stdint.h>

#include "isf.h"

namespace isf {

constexpr uint32_t kSlots = 64;          // spread of the per-sweep atomic accumulators
constexpr uint32_t kTableWords = 52;     // 50 thresholds, the gate threshold, padding
constexpr uint32_t kGateWord = 50;       // switching-field gate threshold (kSentinel: no gate)
// Anisotropy thresholds of one step: words [0, 50) hold the thresholds of
// q + an_num and words [50, 100) those of q - an_num, in the table's order.
constexpr uint32_t kAnWords = 100;
constexpr uint32_t kDefaultMaxSteps = 1024;
constexpr uint32_t kSentinel = 0xFFFFFFFFu;

// Per-film device state, at offset 0 of the aux buffer.
struct alignas(256) DevState {
    int64_t M;              // tracked magnetisation
    int64_t E;              // tracked bond energy
    uint64_t t;             // sweep counter (Philox counter word 1, mod 2^32)
    uint32_t step;          // current step of the loaded schedule
    uint32_t sweep_in_step; // sweeps done in the current step
    int64_t sum_M;          // accumulators of the current step (kept sweeps)
    int64_t sum_absM;
    int64_t sum_E;
    int64_t accepted;
    uint32_t reserved0;
    uint32_t n_steps;       // length of the loaded schedule
    int64_t n_occ;
    int64_t n_bonds;
    int64_t recount[4];     // scratch of the full recount (M, sum s n, sites, occupied pairs)
    uint32_t cur_table[kTableWords];  // thresholds of the current step
    uint32_t cur_atable[kAnWords];    // its anisotropy thresholds (q + an, q - an), if the schedule has the term
    // min over the sweeps the whole-sweep kernels folded since the host last set
    // it of |M at the sweep's start| - 2 (flips in the sweep): while it is >= 2,
    // every sublattice phase of those sweeps started at |M| >= 2 with M's sign
    int64_t spec_margin;
};

// Per-sweep partial sums, one 128-byte line each so that atomics spread.
struct alignas(128) Slot {
    int64_t dM;
    int64_t dE;
    int64_t acc;
    // anisotropic sweeps: the change of M in each sublattice phase, kept apart
    // so that a phase reads the earlier phases' changes and never its own
    int64_t dM_phase[4];
    int64_t pad[9];
};

struct StepDesc {
    uint32_t n_sweeps;
    uint32_t n_discard;
};

// Schedule position of one sweep of the whole-sweep kernel, double-buffered by
// sweep parity: the launch of parity q reads pos[q], and its block 0 writes the
// next sweep's position into pos[1 - q] and folds the previous sweep (whose
// slots are slots[1 - q]) into M, E, the step's sums and records.
struct alignas(256) SweepPos {
    uint64_t t;          // sweep counter of this sweep
    uint32_t step;       // step of this sweep
    uint32_t sis;        // sweeps of the step done before this one
    uint32_t n_sweeps;   // of the step
    uint32_t n_discard;  // of the step
    uint32_t run;        // step < n_steps
    uint32_t pending;    // the slots of this parity hold a sweep not yet folded
    uint32_t table[kTableWords];
};

// Everything a kernel needs to work on one film.
struct LatDev {
    uint8_t *spins;       // INT8: [Z+2][Y][W] bytes; BITPACK: [Z+2][Y][2][ceil(W/32)] words
    DevState *st;
    Slot *slots;          // [kSlots]
    StepDesc *steps;      // [max_steps]
    uint32_t *tables;     // [max_steps][kTableWords]
    uint32_t *atables;    // [max_steps][kAnWords]
    isf_record *records;  // [max_steps]
    uint32_t X, Y, Z;
    uint32_t W;           // compact sites per row = X/2
    uint32_t nd;          // INT8: dwords per row = W/4; BITPACK: words per row = ceil(W/32)
    uint32_t key0, key1;
    uint32_t replica;
    uint32_t format;
    uint32_t aniso;       // the loaded schedule has the anisotropy term of Eq. (7)
    // occupied-dword lists (INT8): item = (((z << ybits) | y) << dbits) | d, per sublattice
    const uint32_t *items;
    uint32_t n_items[4];
    uint32_t items_off[4];
    uint32_t ybits, dbits;
    // whole-sweep kernel: positions of the two sweep parities and the slots of parity 1
    SweepPos *pos;
    Slot *slots2;
};

// Aux buffer layout.
struct AuxLayout {
    uint64_t off_state, off_slots, off_steps, off_tables, off_atables, off_records, off_pos, off_slots2, total;
};

inline AuxLayout aux_layout(uint32_t max_steps) {
    AuxLayout a;
    auto up = [](uint64_t v, uint64_t al) { return (v + al - 1) / al * al; };
    a.off_state = 0;
    // the atomic slots get their own 4 KiB page, apart from the state that every
    // block of every launch reads
    a.off_slots = up(sizeof(DevState), 4096);
    a.off_steps = up(a.off_slots + sizeof(Slot) * kSlots, 4096);
    a.off_tables = up(a.off_steps + sizeof(StepDesc) * max_steps, 256);
    a.off_atables = up(a.off_tables + sizeof(uint32_t) * kTableWords * max_steps, 256);
    a.off_records = up(a.off_atables + sizeof(uint32_t) * kAnWords * max_steps, 256);
    a.off_pos = up(a.off_records + sizeof(isf_record) * max_steps, 4096);
    a.off_slots2 = up(a.off_pos + 2 * sizeof(SweepPos), 4096);
    a.total = up(a.off_slots2 + sizeof(Slot) * kSlots, 256);
    return a;
}

// Launch shape of the phase kernels.
struct Tiling {
    uint32_t tx, ty, ry;  // threads along a row (dwords / words), threads across rows, rows per thread
    uint32_t kernel;      // ISF_KERNEL_TILES, _LIST (ry = list entries per thread), _SWEEP or _PIPE (ry = waves)
};

// One film in a batched launch: its description and where its blocks start.
struct BatchEntry {
    LatDev lat;
    uint32_t block_begin;  // first linear block of this film in the launch
    uint32_t nbx, nby, nbz;  // block grid of this film for the launch's phase
};

// One film in a batched pipelined launch.
struct PipeEntry {
    LatDev lat;
    uint8_t *spare;        // the film's second spin copy
    uint8_t *lists;        // its tile records and tile order, built for its block count
    uint32_t block_begin;  // first linear block of this film
    uint32_t nbx;          // tiles along a row
    uint32_t ntiles;       // tiles of the film
    uint32_t kmax;         // most tiles one of its blocks takes
    uint32_t po;           // sweep parity of the film at the launch with g = 0
    uint32_t pad;
};

// One film in a batched whole-sweep launch.
struct WholeEntry {
    LatDev lat;
    uint8_t *spare;        // the film's second spin copy
    const uint8_t *lists;  // its per-tile lists for the launch's shape
    uint32_t block_begin;  // first linear block (= tile 0) of this film
    uint32_t nbx;          // tiles along a row
    uint32_t po;           // sweep parity of the film at the launch with g = 0
    uint32_t pad;
};

}  // namespace isf
