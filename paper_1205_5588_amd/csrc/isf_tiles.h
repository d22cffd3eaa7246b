// Tile bodies of one sublattice phase, for both storage formats.  Shared by
// the one-launch-per-phase kernels and the persistent batched kernel.
#pragma once

#include "isf_device.h"

namespace isf {

// ---------------------------------------------------------------------------
// INT8 format (one byte per compact site; see isf_internal.h)

// Bytes of a row shifted by one compact column: for delta = -1 the dword of
// columns (4d-1 .. 4d+2), for delta = +1 the dword of columns (4d+1 .. 4d+4).
__device__ __forceinline__ uint32_t shifted(bool left, uint32_t cur, uint32_t other) {
    return left ? __builtin_amdgcn_alignbyte(cur, other, 3) : __builtin_amdgcn_alignbyte(other, cur, 1);
}

// Sum of the 12 neighbour bytes of the 4 sites in dword d of row (y, z)
// (INT8 format), plus the site dword itself.  Returns per byte n + 12.
struct Nb {
    uint32_t self;
    uint32_t sum;     // per byte: sum of the 12 neighbour bytes
    uint32_t occsum;  // per byte: number of occupied neighbours (only if wanted)
};

template <bool kOcc>
__device__ __forceinline__ Nb gather_i8(const uint32_t *P, uint32_t Y, uint32_t nd, uint32_t y, uint32_t z,
                                        uint32_t d, bool left) {
    const uint32_t ym = y == 0 ? Y - 1 : y - 1;
    const uint32_t yp = y + 1 == Y ? 0 : y + 1;
    const uint32_t dd = left ? (d == 0 ? nd - 1 : d - 1) : (d + 1 == nd ? 0 : d + 1);
    const size_t p0 = (size_t)z * Y;  // padded plane index of z-1
    const size_t p1 = p0 + Y;         // plane z
    const size_t p2 = p1 + Y;         // plane z+1
    const size_t r_ym = (p1 + ym) * nd, r_yp = (p1 + yp) * nd;
    const size_t r_zm = (p0 + y) * nd, r_zp = (p2 + y) * nd;
    const uint32_t a1 = P[r_ym + d], a1o = P[r_ym + dd];
    const uint32_t a2 = P[r_yp + d], a2o = P[r_yp + dd];
    const uint32_t b1 = P[r_zm + d], b1o = P[r_zm + dd];
    const uint32_t b2 = P[r_zp + d], b2o = P[r_zp + dd];
    const uint32_t c1 = P[(p0 + ym) * nd + d];
    const uint32_t c2 = P[(p0 + yp) * nd + d];
    const uint32_t c3 = P[(p2 + ym) * nd + d];
    const uint32_t c4 = P[(p2 + yp) * nd + d];
    Nb r;
    r.self = P[(p1 + y) * nd + d];
    const uint32_t s1 = shifted(left, a1, a1o), s2 = shifted(left, a2, a2o);
    const uint32_t s3 = shifted(left, b1, b1o), s4 = shifted(left, b2, b2o);
    r.sum = ((a1 + a2) + (b1 + b2)) + ((s1 + s2) + (s3 + s4)) + ((c1 + c2) + (c3 + c4));
    if (kOcc) {
        const uint32_t m = 0x01010101u;
        r.occsum = ((~a1 & m) + (~a2 & m) + (~b1 & m) + (~b2 & m)) + ((~s1 & m) + (~s2 & m) + (~s3 & m) + (~s4 & m)) +
                   ((~c1 & m) + (~c2 & m) + (~c3 & m) + (~c4 & m));
    } else {
        r.occsum = 0;
    }
    return r;
}

// --------------------------------------------------------------------------
// One tile of one sublattice phase (INT8 format).
//
// Addressing: the block's plane z and its neighbours z-1, z+1 are uniform, so
// their base addresses live in scalar registers and every load is a 32-bit
// byte offset from them.  All rows of a thread are loaded before any is
// computed, so their memory latency overlaps.  Rows past the film end are
// clamped to a valid row and discarded.
__device__ __forceinline__ uint32_t ldw(const char *base, uint32_t off) {
    return *reinterpret_cast<const uint32_t *>(base + off);
}

// One block of one sublattice phase (INT8), with the occupied dwords
// compacted.  About half of all dwords hold only vacancies, but nearly every
// 64-dword wave span holds some occupied site, so skipping has to happen
// inside the block:
//   1. every thread issues the loads of its RY slots (self + 12 neighbour
//      dwords each) and of the film state (table, sweep counter), then forms
//      the biased neighbour sums;
//   2. slots with an occupied site are compacted into LDS in row-major order
//      (wave ballot + mbcnt, block prefix over the (row, wave) counts);
//   3. the Philox draws, acceptance, flips and observables run only on the
//      compacted slots, 256 at a time.
// kAtomic selects agent-scope atomic loads of the film state (needed when the
// state may change inside the same launch, i.e. in the persistent kernel).
// Returns false (uniformly over the block) if the film's schedule is finished.
template <int TX, int TY, int RY, bool kAtomic>
__device__ __forceinline__ bool phase_block_i8(const LatDev &L, uint32_t sigma, uint32_t bx, uint32_t by, uint32_t bz,
                                               int &dM, int &dE, int &acc) {
    constexpr int NT = TX * TY;
    constexpr int NS = NT * RY;
    __shared__ uint32_t tab[kTableWords];
    __shared__ uint32_t t_sh, run_sh;
    __shared__ uint32_t lA[NS], lS[NS];
    __shared__ uint16_t lslot[NS];
    __shared__ uint32_t wcnt[RY * (NT / 64) + 1];

    const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid >> 6;
    // film state: issued first, consumed after the barrier
    uint32_t tabv = 0, tv = 0, runv = 0;
    if (kAtomic) {
        if (tid < kTableWords)
            tabv = ald(&L.st->cur_table[tid]);
        if (tid == 0) {
            tv = (uint32_t)ald(&L.st->t);
            runv = ald(&L.st->step) < ald(&L.st->n_steps);
        }
    } else {
        if (tid < kTableWords)
            tabv = L.st->cur_table[tid];
        if (tid == 0) {
            tv = (uint32_t)L.st->t;
            runv = L.st->step < L.st->n_steps;
        }
    }
    const bool aniso = !kAtomic && L.aniso && wid == 0;  // uniform over each wave
    AnisoLoads an{};
    if (aniso)
        an = aniso_issue(L, sigma, lane);

    const uint32_t py = sigma & 1u, pz = sigma >> 1;
    const uint32_t z = 2 * bz + pz;
    const bool zok = z < L.Z;  // uniform over the block
    const uint32_t tx = tid % TX, ty = tid / TX;
    const uint32_t Y = L.Y, nd = L.nd, half = Y >> 1;
    const uint32_t d_raw = bx * TX + tx;
    const bool dok = d_raw < nd;
    const uint32_t d = dok ? d_raw : nd - 1;
    const uint32_t rowb = nd * 4u;
    const size_t planeb = (size_t)Y * rowb;
    char *c1p = reinterpret_cast<char *>(L.spins) + (size_t)(zok ? z + 1 : 1) * planeb;
    const char *c0p = c1p - planeb;
    const char *c2p = c1p + planeb;
    const bool left = ((py ^ pz) == 0);
    const uint32_t db = d * 4u;
    const uint32_t ddb = (left ? (d == 0 ? nd - 1 : d - 1) : (d + 1 == nd ? 0 : d + 1)) * 4u;

    uint32_t A[RY], S[RY];
    bool need[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const uint32_t yi = (by * RY + r) * TY + ty;
        const bool ok = zok && dok && yi < half;
        const uint32_t y = yi < half ? 2 * yi + py : py;
        const uint32_t ym = y == 0 ? Y - 1 : y - 1;
        const uint32_t yp = y + 1 == Y ? 0 : y + 1;
        // y < 2^16 and rowb < 2^24: 24-bit multiplies are exact
        const uint32_t oy = __umul24(y, rowb), om = __umul24(ym, rowb), op = __umul24(yp, rowb);
        uint32_t a = 0x01010101u, sum = 0;
        if (zok) {
            const uint32_t a1 = ldw(c1p, om + db), a1o = ldw(c1p, om + ddb);
            const uint32_t a2 = ldw(c1p, op + db), a2o = ldw(c1p, op + ddb);
            const uint32_t b1 = ldw(c0p, oy + db), b1o = ldw(c0p, oy + ddb);
            const uint32_t b2 = ldw(c2p, oy + db), b2o = ldw(c2p, oy + ddb);
            const uint32_t e1 = ldw(c0p, om + db), e2 = ldw(c0p, op + db);
            const uint32_t e3 = ldw(c2p, om + db), e4 = ldw(c2p, op + db);
            a = ldw(c1p, oy + db);
            sum = (a1 + a2) + (b1 + b2) + ((shifted(left, a1, a1o) + shifted(left, a2, a2o)) +
                                           (shifted(left, b1, b1o) + shifted(left, b2, b2o))) +
                  ((e1 + e2) + (e3 + e4));
        }
        A[r] = a;
        S[r] = sum;
        need[r] = ok && ((~a & 0x01010101u) != 0u);
    }
    if (aniso)
        tabv = aniso_select(an, tabv, lane);
    if (tid < kTableWords)
        tab[tid] = tabv;
    if (tid == 0) {
        t_sh = tv;
        run_sh = runv;
    }
    // per (row, wave) counts of occupied slots
    uint32_t pos[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const uint64_t m = __ballot(need[r]);
        pos[r] = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (lane == 0)
            wcnt[r * (NT / 64) + wid] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0;
        for (int k = 0; k < RY * (NT / 64); ++k) {
            const uint32_t c = wcnt[k];
            wcnt[k] = run;
            run += c;
        }
        wcnt[RY * (NT / 64)] = run;
    }
    __syncthreads();
    if (!run_sh)
        return false;  // uniform: the film's schedule is finished
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        if (need[r]) {
            const uint32_t i = wcnt[r * (NT / 64) + wid] + pos[r];
            lA[i] = A[r];
            lS[i] = S[r];
            lslot[i] = (uint16_t)(r * NT + tid);
        }
    }
    __syncthreads();
    const uint32_t n_items = wcnt[RY * (NT / 64)];
    const uint32_t t = t_sh;
    const uint32_t cz = z * Y * nd;  // Philox counter word 0 of row (z, 0), dword 0
    // Wave w of this block takes the items of wave slot (w + rot): the partial
    // last 64-item group goes to a different wave in neighbouring blocks, so the
    // extra pass is spread over the SIMDs of a CU instead of piling onto one.
    const uint32_t rot = (bx + by + bz) % (NT / 64);
    const uint32_t i0 = ((wid + rot) % (NT / 64)) * 64u + lane;
    const PhiloxShared psh = philox_shared(t, L.replica, L.key0);  // the parts of the counter every item shares
    for (uint32_t i = i0; i < n_items; i += NT) {
        const uint32_t slot = lslot[i];
        const uint32_t a = lA[i], sum = lS[i];
        const uint32_t r = slot / NT, st = slot % NT;
        const uint32_t y = 2 * ((by * RY + r) * TY + st / TX) + py;
        const uint32_t dd = bx * TX + st % TX;
        const uint32_t k4 = cz + y * nd + dd;
        uint32_t u[4];
        philox_first_two(u, k4, sigma, psh, L.key0, L.key1);
        philox_rounds<2, 10>(u, L.key0, L.key1);
        const uint32_t occ = ~a & 0x01010101u;
        const uint32_t up = (a >> 1) & 0x01010101u;
        const uint32_t key = sum + up + (up << 3) + (up << 4);  // n + 12 + 25 [s = +1], <= 49
        uint32_t F = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            // thresholds of downhill moves are kSentinel and every other one is
            // below it, so with u clamped to kSentinel - 1 one test is exact
            const uint32_t thr = tab[(key >> (8 * j)) & 0xFFu];
            F |= (min(u[j], kSentinel - 1u) < thr) ? (2u << (8 * j)) : 0u;
        }
        F &= occ << 1;  // vacancies never flip
        if (F)
            F &= gate_mask(tab[kGateWord], k4, t, L.replica, sigma, L.key0, L.key1);
        if (F) {
            // up spins flipped: byte 2 in a & F; down spins flipped: the rest of F
            const uint32_t fu = F & a, fd = F ^ fu;
            const int cu = __popc(fu), cd = __popc(fd);
            const uint32_t su = __builtin_amdgcn_udot4(sum, fu >> 1, 0u, false);
            const uint32_t sd = __builtin_amdgcn_udot4(sum, fd >> 1, 0u, false);
            dM += 2 * (cd - cu);
            dE += 2 * ((int)su - (int)sd) - 24 * (cu - cd);
            acc += cu + cd;
            *reinterpret_cast<uint32_t *>(c1p + __umul24(y, rowb) + dd * 4u) = a ^ F;
        }
    }
    return true;
}

// ---------------------------------------------------------------------------
// BITPACK format (spin bit + occupancy bit per site)

// Word w of a row shifted by one column: bit i of the result is column
// 32w + i - 1 (left) or 32w + i + 1 (right), columns mod W.  other is the
// neighbouring word in that direction (w - 1 or w + 1, wrapping), and eb the
// bit where the column from it enters: 31 between whole words; at the row's
// seam (left of word 0, right of the last word) r - 1, r = the number of
// columns in the last word, whose bits past r - 1 are zero.
__device__ __forceinline__ uint32_t shift_bits(bool left, uint32_t cur, uint32_t other, uint32_t eb) {
    return left ? ((cur << 1) | ((other >> eb) & 1u)) : ((cur >> 1) | ((other & 1u) << eb));
}

// 4-bit bit-sliced count per site (counts stay <= 12): plane k holds bit k.
struct Cnt4 {
    uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
};

// Full adder on 32 sites at once: s = a + b + c mod 2, cy = the majority.
__device__ __forceinline__ void full_add(uint32_t a, uint32_t b, uint32_t c, uint32_t &s, uint32_t &cy) {
    s = a ^ b ^ c;
    cy = (a & b) | (c & (a ^ b));
}

// Count of the 12 one-bit inputs x[0..12) per site by a carry-save tree: a
// full adder keeps the weighted sum of its inputs, so the four bits left at
// weights 1, 2, 4 and 8 are the exact count (8 full and 2 half adders,
// against 12 increments of a 4-bit counter).
__device__ __forceinline__ Cnt4 count12(const uint32_t (&x)[12]) {
    uint32_t s0, s1, s2, s3, c0, c1, c2, c3;
    full_add(x[0], x[1], x[2], s0, c0);
    full_add(x[3], x[4], x[5], s1, c1);
    full_add(x[6], x[7], x[8], s2, c2);
    full_add(x[9], x[10], x[11], s3, c3);
    uint32_t t0, d0;  // weight 1: s0..s3
    full_add(s0, s1, s2, t0, d0);
    Cnt4 r;
    r.c0 = t0 ^ s3;
    const uint32_t d1 = t0 & s3;
    uint32_t e0, f0, e1, f1;  // weight 2: c0..c3, d0, d1
    full_add(c0, c1, c2, e0, f0);
    full_add(c3, d0, d1, e1, f1);
    r.c1 = e0 ^ e1;
    const uint32_t f2 = e0 & e1;
    full_add(f0, f1, f2, r.c2, r.c3);  // weight 4: f0, f1, f2
    return r;
}

struct NbBits {
    uint32_t spin, occ;
    Cnt4 up, vac;
};

// Neighbour counts of the 32 sites in word w of row (y, z); W columns per row.
__device__ __forceinline__ NbBits gather_bp(const uint32_t *P, uint32_t Y, uint32_t nw, uint32_t W, uint32_t y,
                                            uint32_t z, uint32_t w, bool left) {
    const uint32_t ym = y == 0 ? Y - 1 : y - 1;
    const uint32_t yp = y + 1 == Y ? 0 : y + 1;
    const uint32_t wo = left ? (w == 0 ? nw - 1 : w - 1) : (w + 1 == nw ? 0 : w + 1);
    const bool seam = left ? w == 0 : w + 1 == nw;
    const uint32_t eb = seam ? W - 32u * (nw - 1u) - 1u : 31u;
    const size_t p0 = (size_t)z * Y, p1 = p0 + Y, p2 = p1 + Y;
    auto row = [&](size_t plane, uint32_t yy) { return P + (plane + yy) * 2 * nw; };
    NbBits r;
    const uint32_t *self = row(p1, y);
    r.spin = self[w];
    r.occ = self[nw + w];
    const uint32_t *sh_rows[4] = {row(p1, ym), row(p1, yp), row(p0, y), row(p2, y)};
    const uint32_t *st_rows[4] = {row(p0, ym), row(p0, yp), row(p2, ym), row(p2, yp)};
    uint32_t up[12], vac[12];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t *q = sh_rows[k];
        const uint32_t s = q[w], so = q[wo], o = q[nw + w], oo = q[nw + wo];
        up[2 * k] = s;
        vac[2 * k] = ~o;
        up[2 * k + 1] = shift_bits(left, s, so, eb);
        vac[2 * k + 1] = ~shift_bits(left, o, oo, eb);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t *q = st_rows[k];
        up[8 + k] = q[w];
        vac[8 + k] = ~q[nw + w];
    }
    r.up = count12(up);
    r.vac = count12(vac);
    return r;
}

// Bit-sliced 6-bit table index idx = 2U + D + 25 s (idx <= 49).
struct Idx6 {
    uint32_t b[6];
};

__device__ __forceinline__ Idx6 table_index(const Cnt4 &U, const Cnt4 &D, uint32_t s) {
    // S = (U << 1) + D, 5 bits
    uint32_t S[5];
    S[0] = D.c0;
    uint32_t c = U.c0 & D.c1;
    S[1] = U.c0 ^ D.c1;
    uint32_t t = U.c1 ^ D.c2;
    S[2] = t ^ c;
    c = (U.c1 & D.c2) | (c & t);
    t = U.c2 ^ D.c3;
    S[3] = t ^ c;
    c = (U.c2 & D.c3) | (c & t);
    S[4] = U.c3 ^ c;  // S <= 24 < 32: no carry out
    // + 25 s: 25 = 0b11001, add s at bits 0, 3 and 4
    Idx6 r;
    uint32_t k = S[0] & s;
    r.b[0] = S[0] ^ s;
    r.b[1] = S[1] ^ k;
    k = S[1] & k;
    r.b[2] = S[2] ^ k;
    k = S[2] & k;
    t = S[3] ^ s;
    r.b[3] = t ^ k;
    k = (S[3] & s) | (k & t);
    t = S[4] ^ s;
    r.b[4] = t ^ k;
    k = (S[4] & s) | (k & t);
    r.b[5] = k;
    return r;
}

// kGate: the step has the switching-field gate (its code is compiled out of
// the ungated path, where it cost 3 % of a sweep).
template <int TX, int TY, int RY, bool kGate>
__device__ __forceinline__ void phase_tile_bp_g(const LatDev &L, uint32_t sigma, uint32_t bx, uint32_t by,
                                                uint32_t bz, const uint32_t *tab, uint32_t t, int &dM, int &dE,
                                                int &acc) {
    const uint32_t py = sigma & 1u, pz = sigma >> 1;
    const uint32_t z = 2 * bz + pz;
    const uint32_t tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const uint32_t w = bx * TX + tx;
    const uint32_t nw = L.nd;
    if (z >= L.Z || w >= nw)
        return;
    const uint32_t Y = L.Y, half = Y >> 1;
    uint32_t *P = reinterpret_cast<uint32_t *>(L.spins);
    const bool left = ((py ^ pz) == 0);
    const uint32_t gthr = kGate ? tab[kGateWord] : kSentinel;
    const PhiloxShared psh = philox_shared(t, L.replica, L.key0);  // the parts of the counter every group shares
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const uint32_t yi = (by * RY + r) * TY + ty;
        if (yi >= half)
            break;
        const uint32_t y = 2 * yi + py;
        const NbBits nb = gather_bp(P, Y, nw, L.W, y, z, w, left);
        if (!nb.occ)
            continue;
        const Idx6 ix = table_index(nb.up, nb.vac, nb.spin);
        // Philox groups: compact index k = (z Y + y) W + 32 w + i, group k >> 2
        // (W is a multiple of 4: the INT8 format's dword index of the same sites)
        const uint32_t g0 = (z * Y + y) * (L.W / 4u) + 8u * w;
        uint32_t F = 0;
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            const uint32_t occ4 = (nb.occ >> (4 * g)) & 0xFu;
            if (!occ4)
                continue;
            uint32_t u[4], fg = 0;
            philox_first_two(u, g0 + g, sigma, psh, L.key0, L.key1);
            philox_rounds<2, 10>(u, L.key0, L.key1);
            // the table indices of the group's 4 sites, one byte each: the
            // group's nibble of each bit plane is spread to bit 0 of 4 bytes
            // (bit j of a nibble n lands on bit 8j of n * 0x204081; the four
            // shifted copies of n do not overlap, so nothing carries)
            uint32_t key = 0;
#pragma unroll
            for (int p = 0; p < 6; ++p)
                key |= ((((ix.b[p] >> (4 * g)) & 0xFu) * 0x00204081u) & 0x01010101u) << p;
            // the four threshold reads are issued together and the vacancies
            // masked afterwards (a read per site behind its occupancy test made
            // four LDS round trips in a row); a vacant site's index is in the
            // table too: 2U + D <= 24 since U + D <= 12, so idx <= 49
            uint32_t thr[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                thr[j] = tab[(key >> (8 * j)) & 0xFFu];
#pragma unroll
            for (int j = 0; j < 4; ++j)  // exact: see phase_block_i8
                fg |= (uint32_t)(min(u[j], kSentinel - 1u) < thr[j]) << j;
            fg &= occ4;
            // the switching-field gate of Eq. (9): the group's own draw (tag 2),
            // needed only where a Metropolis test passed
            if (kGate && fg) {
                philox(g0 + g, t, L.replica, sigma + 8u, L.key0, L.key1, u);
                uint32_t m = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    m |= (uint32_t)(u[j] < gthr) << j;
                fg &= m;
            }
            F |= fg << (4 * g);
        }
        if (F) {
            const uint32_t fu = F & nb.spin, fd = F & ~nb.spin;
            const int cu = __popc(fu), cd = __popc(fd);
            dM += 2 * (cd - cu);
            acc += cu + cd;
            // sum of S = 2U + D over flipped sites, per direction: E changes by 2 s (S - 12)
            const uint32_t U0 = nb.up.c0, U1 = nb.up.c1, U2 = nb.up.c2, U3 = nb.up.c3;
            const uint32_t D0 = nb.vac.c0, D1 = nb.vac.c1, D2 = nb.vac.c2, D3 = nb.vac.c3;
            const int su = 2 * (__popc(U0 & fu) + 2 * __popc(U1 & fu) + 4 * __popc(U2 & fu) + 8 * __popc(U3 & fu)) +
                 (__popc(D0 & fu) + 2 * __popc(D1 & fu) + 4 * __popc(D2 & fu) + 8 * __popc(D3 & fu));
            const int sd = 2 * (__popc(U0 & fd) + 2 * __popc(U1 & fd) + 4 * __popc(U2 & fd) + 8 * __popc(U3 & fd)) +
                 (__popc(D0 & fd) + 2 * __popc(D1 & fd) + 4 * __popc(D2 & fd) + 8 * __popc(D3 & fd));
            dE += 2 * (su - 12 * cu) - 2 * (sd - 12 * cd);
            P[((size_t)(z + 1) * Y + y) * 2 * nw + w] = nb.spin ^ F;
        }
    }
}

template <int TX, int TY, int RY>
__device__ __forceinline__ void phase_tile_bp(const LatDev &L, uint32_t sigma, uint32_t bx, uint32_t by, uint32_t bz,
                                              const uint32_t *tab, uint32_t t, int &dM, int &dE, int &acc) {
    if (tab[kGateWord] == kSentinel)  // uniform: the step has no gate
        phase_tile_bp_g<TX, TY, RY, false>(L, sigma, bx, by, bz, tab, t, dM, dE, acc);
    else
        phase_tile_bp_g<TX, TY, RY, true>(L, sigma, bx, by, bz, tab, t, dM, dE, acc);
}

}  // namespace isf
