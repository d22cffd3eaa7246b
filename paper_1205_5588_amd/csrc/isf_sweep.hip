// One whole Metropolis sweep of an INT8 film per launch (all four sublattice
// phases, Section 5 steps 1-3 with the acceptance rule of Eq. 8).
//
// A block owns a tile of TXD dwords x TYR rows of every plane z.  It loads the
// tile into LDS together with a halo of HX dwords and HY rows on each side
// (x and y are periodic, so halo rows and dwords wrap), runs the four phases
// sigma = 0..3 on the LDS copy, and writes the tile to the other buffer of a
// ping-pong pair: the launch reads one copy of the film and writes the other,
// because blocks that start late must still see the halo values from before
// the sweep.  The halo is updated too, redundantly with the neighbouring
// blocks, so that the tile sees the same neighbour values as the four-launch
// sweep:
//
//   every site's 12 neighbours lie at most one row away in y and at most one
//   byte (compact column) away in x, so a value computed in phase k is right
//   wherever all its neighbours were right before phase k.  Starting from
//   the loaded values (right on the whole region), phase k is evaluated on
//   rows within 3 - k of the tile and, for k < 3, on one halo dword on each
//   side; its results are then right within 3 - k rows and 4 - k bytes of the
//   tile, which covers everything phase k + 1 reads.  Phase 3 runs on the
//   tile alone.
//
// Draws are keyed by (site dword, sweep, replica, sigma) only, so the halo
// copies draw the same numbers as the owning block, and the trajectory is
// identical, bit for bit, to the one-launch-per-sublattice kernels.  Only the
// tile's own flips enter the observables.
//
// The sweep is bound by integer ALU work (Philox and the neighbour sums), so
// the per-site instruction count is what matters:
//   * vacant dwords are skipped: each block's occupied dwords per phase are
//     listed once per film and tiling by k_sweep_lists (occupancy is
//     static) and kept in HBM; a sweep copies its block's lists into LDS next
//     to the region;
//   * a list entry is the dword's region index; the row index follows with
//     one multiply, and a per-row table gives the Philox counter base and
//     whether the row belongs to the tile;
//   * the 13 LDS reads of a dword use one base address and immediate offsets;
//   * two entries per iteration keep two gathers in flight.
// HBM traffic per sweep: each block reads (TXD + 2 HX)(TYR + 2 HY) dwords per
// plane plus its lists and writes its tile's occupied dwords.
//
// Per-sweep bookkeeping needs no launch of its own: the schedule position
// (sweep counter, step, threshold table) is double-buffered by sweep parity.
// The launch of parity q reads pos[q]; wave 0 of its block 0 folds the
// previous sweep's slot sums (parity 1 - q, complete since that launch ended)
// into M, E, the step's sums and its record, and writes the next sweep's
// position into pos[1 - q].  Its loads are issued when the block starts and
// used when its tile is done, so the fold adds no latency in between.  After
// the last sweep of a run, one small launch (k_whole_flush) folds that sweep
// and hands the position back to the film state read by every other path.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "isf_books.h"
#include "isf_device.h"

namespace isf {

namespace {

constexpr int kHX = 2;  // halo dwords on each side along x
constexpr int kHY = 4;  // halo rows on each side along y
constexpr uint32_t kVacant = 0x01010101u;

// Region geometry and the candidate slots of each phase: rows ry = r0, r0+2,
// ... (nry), planes z = pz, pz+2, ... (nz), dwords cx0 .. cx0 + ncx - 1.
template <int TXD, int TYR>
struct Geo {
    static constexpr int RX = TXD + 2 * kHX;
    static constexpr int RYN = TYR + 2 * kHY;
    static constexpr int PL = RX * RYN;
    __host__ __device__ static constexpr int lo(int s) { return kHY - (3 - s); }
    __host__ __device__ static constexpr int hi(int s) { return kHY + TYR + (3 - s); }
    // first row >= lo with parity py (region rows have the parity of their global row: y0 and kHY are even)
    __host__ __device__ static constexpr int r0(int s) { return lo(s) + ((lo(s) ^ (s & 1)) & 1); }
    __host__ __device__ static constexpr int nry(int s) { return (hi(s) - r0(s) + 1) / 2; }
    __host__ __device__ static constexpr int cx0(int s) { return s < 3 ? kHX - 1 : kHX; }
    __host__ __device__ static constexpr int ncx(int s) { return s < 3 ? TXD + 2 : TXD; }
    __host__ __device__ static constexpr uint32_t nz(int s, uint32_t Z) { return (Z - (uint32_t)(s >> 1) + 1) / 2; }
    __host__ __device__ static constexpr uint32_t cand(int s, uint32_t Z) {
        return (uint32_t)(nry(s) * ncx(s)) * nz(s, Z);
    }
    // list capacity of phase s, in entries: a multiple of 4 so that lists stay 8-byte aligned
    __host__ __device__ static constexpr uint32_t cap(int s, uint32_t Z) { return (cand(s, Z) + 3u) & ~3u; }
    __host__ __device__ static constexpr uint32_t list_off(int s, uint32_t Z) {
        uint32_t o = 0;
        for (int k = 0; k < s; ++k)
            o += cap(k, Z);
        return o;
    }
    __host__ __device__ static constexpr uint32_t cap_total(uint32_t Z) { return list_off(4, Z); }
    // HBM record of one tile: 4 uint32 counts, then the four lists of uint16 region indices
    __host__ __device__ static constexpr uint32_t rec_bytes(uint32_t Z) {
        return (16u + 2u * cap_total(Z) + 255u) & ~255u;
    }
    // LDS: region words | row table (uint2 per region row) | ymap | dmap | lists
    __host__ __device__ static constexpr uint32_t off_rowk(uint32_t Z) { return 4u * (Z + 2) * PL; }
    __host__ __device__ static constexpr uint32_t off_ymap(uint32_t Z) { return off_rowk(Z) + 8u * (Z + 2) * RYN; }
    __host__ __device__ static constexpr uint32_t off_dmap(uint32_t Z) { return off_ymap(Z) + 4u * RYN; }
    __host__ __device__ static constexpr uint32_t off_lst(uint32_t Z) { return off_dmap(Z) + 4u * RX; }
    __host__ __device__ static constexpr uint32_t lds_bytes(uint32_t Z) { return off_lst(Z) + 2u * cap_total(Z); }
};

__device__ __forceinline__ int wrap_mod(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

__device__ __forceinline__ uint32_t tile_of_block(uint32_t b, uint32_t per_xcd) {
    // Blocks are dealt to the 8 XCDs round robin; block b takes tile
    // (b % 8) * per_xcd + b / 8, so each XCD works on a contiguous band of
    // tiles and the halo rows shared by neighbouring tiles stay in its L2.
    return (b & 7u) * per_xcd + (b >> 3);
}

}  // namespace

// Start of a run of whole-sweep launches: the position of the first sweep
// (parity q) from the film state; nothing is pending.  One wave.
__global__ __launch_bounds__(64) void k_whole_prime(LatDev L, uint32_t q) {
    const uint32_t lane = threadIdx.x;
    const DevState *st = L.st;
    if (lane == 0) {
        SweepPos &p = L.pos[q];
        const uint32_t step = st->step;
        p.t = st->t;
        p.step = step;
        p.sis = st->sweep_in_step;
        p.run = step < st->n_steps;
        p.n_sweeps = p.run ? L.steps[step].n_sweeps : 0u;
        p.n_discard = p.run ? L.steps[step].n_discard : 0u;
        p.pending = 0;
        L.pos[1 - q].pending = 0;
    }
    if (lane < kTableWords)
        L.pos[q].table[lane] = st->cur_table[lane];
}

// End of a run: fold the last sweep (parity q_last) and make the position
// after it the film state's.  One wave.
__global__ __launch_bounds__(64) void k_whole_flush(LatDev L, uint32_t q_last) {
    __shared__ BookLds bk;
    const uint32_t lane = threadIdx.x;
    book_stage(bk, book_issue(L, q_last, 1 - q_last, lane), lane);
    book_fold(L, q_last, bk, lane);
    const SweepPos &n = L.pos[1 - q_last];
    DevState *st = L.st;
    if (lane == 0) {
        st->t = n.t;
        st->step = n.step;
        st->sweep_in_step = n.sis;
    }
    if (lane < kTableWords)
        st->cur_table[lane] = n.table[lane];
}

// Lists of occupied dwords per phase for every tile (run once per film and
// tiling; occupancy never changes).  One block per tile; the order of entries
// within a list is arbitrary.
template <int TXD, int TYR>
__global__ __launch_bounds__(256) void k_sweep_lists(LatDev L, uint32_t nbx, uint32_t per_xcd, uint8_t *lists) {
    using G = Geo<TXD, TYR>;
    __shared__ uint32_t cnt[4];
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t Y = L.Y, Z = L.Z, nd = L.nd;
    const uint32_t tile = tile_of_block(blockIdx.x, per_xcd);
    const uint32_t nby = (Y + TYR - 1) / TYR;
    if (tile >= nbx * nby)
        return;
    const uint32_t bx = tile % nbx, by = tile / nbx;
    const int d0 = (int)(bx * TXD), y0 = (int)(by * TYR);
    uint8_t *rec = lists + (size_t)tile * G::rec_bytes(Z);
    uint16_t *ent = reinterpret_cast<uint16_t *>(rec + 16);
    if (tid < 4)
        cnt[tid] = 0;
    __syncthreads();
    const char *spins = reinterpret_cast<const char *>(L.spins);
    const size_t rowb = (size_t)nd * 4u, planeb = (size_t)Y * rowb;
    for (int s = 0; s < 4; ++s) {
        const uint32_t n = G::cand(s, Z);
        const uint32_t nr = (n + 255u) / 256u * 256u;
        for (uint32_t c = tid; c < nr; c += 256) {
            uint32_t ri = 0;
            bool occ = false;
            if (c < n) {
                const uint32_t cx = G::cx0(s) + c % G::ncx(s);
                const uint32_t q = c / G::ncx(s);
                const uint32_t ry = G::r0(s) + 2 * (q % G::nry(s));
                const uint32_t z = (uint32_t)(s >> 1) + 2 * (q / G::nry(s));
                ri = ((z + 1) * G::RYN + ry) * G::RX + cx;
                const int y = wrap_mod(y0 - kHY + (int)ry, (int)Y), d = wrap_mod(d0 - kHX + (int)cx, (int)nd);
                const uint32_t v =
                    *reinterpret_cast<const uint32_t *>(spins + (z + 1) * planeb + (size_t)y * rowb + (size_t)d * 4u);
                occ = v != kVacant;
            }
            const uint64_t m = __ballot(occ);
            if (m) {
                const uint32_t pos =
                    __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                uint32_t base_i = 0;
                if (lane == 0)
                    base_i = atomicAdd(&cnt[s], (uint32_t)__popcll(m));
                base_i = __builtin_amdgcn_readfirstlane(base_i);  // lane 0 is active here
                if (occ)
                    ent[G::list_off(s, Z) + base_i + pos] = (uint16_t)ri;
            }
        }
    }
    __syncthreads();
    if (tid < 4)
        reinterpret_cast<uint32_t *>(rec)[tid] = cnt[tid];
}

// One tile of one whole sweep of parity q (the body of the plain and the
// batched kernels).  The block with tile 0 of the film keeps its books.
template <int TXD, int TYR, int NT>
__device__ __forceinline__ void sweep_tile(const LatDev &L, const uint8_t *__restrict__ src,
                                           uint8_t *__restrict__ dst, const uint8_t *__restrict__ lists,
                                           uint32_t nbx, uint32_t tile, uint32_t q) {
    using G = Geo<TXD, TYR>;
    constexpr int RX = G::RX, RYN = G::RYN, PL = G::PL;
    extern __shared__ __align__(16) uint8_t smb[];
    __shared__ uint32_t tab[kTableWords];
    __shared__ uint32_t t_sh, run_sh;

    const uint32_t tid = threadIdx.x;
    const uint32_t Y = L.Y, Z = L.Z, nd = L.nd;
    const uint32_t np = Z + 2;
    uint32_t *R = reinterpret_cast<uint32_t *>(smb);                       // [np][RYN][RX] dwords
    uint2 *rowk = reinterpret_cast<uint2 *>(smb + G::off_rowk(Z));        // per region row: Philox base, ymap
    uint32_t *ymap = reinterpret_cast<uint32_t *>(smb + G::off_ymap(Z));  // global row, bit 31: tile row
    uint32_t *dmap = reinterpret_cast<uint32_t *>(smb + G::off_dmap(Z));  // global dword, bit 31: tile dword
    uint16_t *lst = reinterpret_cast<uint16_t *>(smb + G::off_lst(Z));

    const uint32_t bx = tile % nbx, by = tile / nbx;
    const uint32_t d0 = bx * TXD, y0 = by * TYR;
    const uint8_t *rec = lists + (size_t)tile * G::rec_bytes(Z);
    const uint4 cnt = *reinterpret_cast<const uint4 *>(rec);  // uniform: a scalar load
    const bool booker = tile == 0 && tid < 64;                // wave 0 of tile 0's block keeps the books
    __shared__ BookLds bk;
    BookRegs br;
    if (booker)
        br = book_issue(L, 1 - q, q, tid);

    const SweepPos &P = L.pos[q];
    if (tid < kTableWords)
        tab[tid] = P.table[tid];
    if (tid == 0) {
        t_sh = (uint32_t)P.t;
        run_sh = P.run;
    }
    const uint32_t ynd = Y * nd;
    for (uint32_t i = tid; i < np * RYN + RX; i += NT) {
        if (i < np * RYN) {
            const uint32_t p = i / RYN, ry = i % RYN;
            const uint32_t y = (uint32_t)wrap_mod((int)(y0 + ry) - kHY, (int)Y);
            const bool own = ry >= (uint32_t)kHY && ry < (uint32_t)(kHY + TYR) && y0 + ry - kHY < Y;
            const uint32_t ym = y | (own ? 0x80000000u : 0u);
            rowk[i] = make_uint2((p - 1) * ynd + y * nd, ym);  // p = 0 and np - 1 (padding) are never looked up
            if (p == 0)
                ymap[ry] = ym;
        } else {
            const uint32_t c = i - np * RYN;
            const uint32_t d = (uint32_t)wrap_mod((int)(d0 + c) - kHX, (int)nd);
            const bool own = c >= (uint32_t)kHX && c < (uint32_t)(kHX + TXD) && d0 + c - kHX < nd;
            dmap[c] = d | (own ? 0x80000000u : 0u);
        }
    }

    // The region and this block's lists, HBM -> LDS.  Planes 1..Z come from the
    // film, the padding planes are vacancies; the lists are 8-byte words (4
    // entries) of the four per-phase lists, each 8-byte aligned.  Films at
    // least as large as the region, with an even number of dwords per row, take
    // 8-byte region loads (dword pairs never straddle the periodic seam and stay
    // 8-byte aligned) with the wrap done arithmetically; every load of a batch
    // (KB region pairs and KL list words per thread, one batch for films of up
    // to 8 planes) is issued before the first one is stored, so the load phase
    // costs about one memory round trip.  Other films take 4-byte region loads
    // with the wrap by modulo.
    const uint32_t rowb = nd * 4u;
    const size_t planeb = (size_t)Y * rowb;
    const char *base = reinterpret_cast<const char *>(src);
    const bool wide = (nd & 1u) == 0 && nd >= (uint32_t)RX && Y >= (uint32_t)RYN;  // uniform
    const uint32_t w0 = (cnt.x + 3u) / 4u, w1 = (cnt.y + 3u) / 4u, w2 = (cnt.z + 3u) / 4u, w3 = (cnt.w + 3u) / 4u;
    const uint32_t e1 = w0, e2 = e1 + w1, e3 = e2 + w2, nwl = e3 + w3;  // list word boundaries
    const uint2 *lsrc = reinterpret_cast<const uint2 *>(rec + 16);
    uint2 *ldst = reinterpret_cast<uint2 *>(lst);
    // flat list word i -> word offset of its list's slot (lists start at list_off(s) / 4 words)
    auto list_word = [&](uint32_t i) -> uint32_t {
        if (i < e1)
            return i;
        if (i < e2)
            return G::list_off(1, Z) / 4u + (i - e1);
        if (i < e3)
            return G::list_off(2, Z) / 4u + (i - e2);
        return G::list_off(3, Z) / 4u + (i - e3);
    };
    if (wide && Z * planeb < (1ull << 32)) {  // byte offsets within the film fit 32 bits
        const uint32_t planeb32 = (uint32_t)planeb;
        constexpr uint32_t RX2 = RX / 2, PL2 = PL / 2;
        constexpr int KB = NT >= 1024 ? 6 : 12, KL = NT >= 1024 ? 1 : 2;
        const uint32_t n = Z * PL2;
        for (uint32_t i0 = 0, l0 = 0; i0 < n || l0 < nwl; i0 += KB * NT, l0 += KL * NT) {
            uint2 v[KB], lv[KL];
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                const uint32_t i = i0 + k * NT + tid;
                if (i < n) {
                    const uint32_t p = i / PL2 + 1, r = i % PL2;
                    const uint32_t ry = r / RX2, cx = 2 * (r % RX2);
                    int y = (int)(y0 + ry) - kHY, d = (int)(d0 + cx) - kHX;
                    y += y < 0 ? (int)Y : 0;
                    y -= y >= (int)Y ? (int)Y : 0;
                    d += d < 0 ? (int)nd : 0;
                    d -= d >= (int)nd ? (int)nd : 0;
                    v[k] = *reinterpret_cast<const uint2 *>(base + (p * planeb32 + (uint32_t)y * rowb + (uint32_t)d * 4u));
                }
            }
#pragma unroll
            for (int k = 0; k < KL; ++k) {
                const uint32_t i = l0 + k * NT + tid;
                if (i < nwl)
                    lv[k] = lsrc[list_word(i)];
            }
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                const uint32_t i = i0 + k * NT + tid;
                if (i < n) {
                    const uint32_t p = i / PL2 + 1, r = i % PL2;
                    *reinterpret_cast<uint2 *>(&R[p * PL + 2 * r]) = v[k];
                }
            }
#pragma unroll
            for (int k = 0; k < KL; ++k) {
                const uint32_t i = l0 + k * NT + tid;
                if (i < nwl)
                    ldst[list_word(i)] = lv[k];
            }
        }
    } else {
        for (uint32_t i = tid; i < nwl; i += NT)
            ldst[list_word(i)] = lsrc[list_word(i)];
        const uint32_t n = Z * PL;
#pragma unroll 4
        for (uint32_t i = tid; i < n; i += NT) {
            const uint32_t p = i / PL + 1, r = i % PL;
            const uint32_t ry = r / RX, cx = r % RX;
            const uint32_t y = (uint32_t)wrap_mod((int)(y0 + ry) - kHY, (int)Y);
            const uint32_t d = (uint32_t)wrap_mod((int)(d0 + cx) - kHX, (int)nd);
            R[p * PL + r] = *reinterpret_cast<const uint32_t *>(base + p * planeb + y * rowb + d * 4u);
        }
    }
    for (uint32_t i = tid; i < (uint32_t)PL; i += NT) {
        R[i] = kVacant;
        R[(np - 1) * PL + i] = kVacant;
    }
    if (booker)
        book_stage(bk, br, tid);
    __syncthreads();
    if (!run_sh) {  // uniform: the schedule is finished; the sweep still counts
        if (booker) {
            book_fold(L, 1 - q, bk, tid);
            book_advance(L, q, bk, tab, tid);
        }
        return;
    }

    int dM = 0, dE = 0, acc = 0;
    const uint32_t t = t_sh;
    const PhiloxShared psh = philox_shared(t, L.replica, L.key0);  // the sweep's common draw parts
    const uint32_t c4[4] = {cnt.x, cnt.y, cnt.z, cnt.w};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const uint32_t n = c4[s];
        const uint16_t *ls = lst + G::list_off(s, Z);
        const bool left = ((s & 1) ^ (s >> 1)) == 0;  // (y + z) even: the shifted columns are j - 1
        constexpr int kB = PL + RX;                    // offset of the dword from its gather base
        const int o = left ? -1 : 1;
        auto sh = [left](uint32_t cur, uint32_t other) {
            return left ? __builtin_amdgcn_alignbyte(cur, other, 3) : __builtin_amdgcn_alignbyte(other, cur, 1);
        };
        // two entries per iteration: both gathers are issued before either flip is
        // written, so their LDS latencies overlap (dwords of one phase share no bond)
        for (uint32_t i = tid; i < n; i += 2 * NT) {
            const bool two = i + NT < n;
            uint32_t ri[2];
            ri[0] = ls[i];
            ri[1] = two ? ls[i + NT] : ri[0];
            uint32_t a[2], sum[2], kb[2], ym[2], dm[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const uint32_t q = ri[k];
                const uint32_t row = q / RX, cx = q - row * RX;
                const uint32_t *Rb = R + (q - kB);  // every offset below is >= 0
                a[k] = Rb[kB];
                const uint32_t a1 = Rb[kB - RX], a2 = Rb[kB + RX];
                const uint32_t b1 = Rb[kB - PL], b2 = Rb[kB + PL];
                const uint32_t a1o = Rb[kB - RX + o], a2o = Rb[kB + RX + o];
                const uint32_t b1o = Rb[kB - PL + o], b2o = Rb[kB + PL + o];
                const uint32_t e1 = Rb[0], e2 = Rb[kB - PL + RX];
                const uint32_t e3 = Rb[kB + PL - RX], e4 = Rb[kB + PL + RX];
                sum[k] = (a1 + a2) + (b1 + b2) + ((sh(a1, a1o) + sh(a2, a2o)) + (sh(b1, b1o) + sh(b2, b2o))) +
                         ((e1 + e2) + (e3 + e4));
                const uint2 rk = rowk[row];
                kb[k] = rk.x;
                ym[k] = rk.y;
                dm[k] = dmap[cx];
            }
            uint32_t F[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                uint32_t u[4];
                philox_first_two(u, kb[k] + (dm[k] & 0x7FFFFFFFu), (uint32_t)s, psh, L.key0, L.key1);
                philox_rounds<2, 10>(u, L.key0, L.key1);
                const uint32_t up = (a[k] >> 1) & 0x01010101u;
                const uint32_t key = sum[k] + up + (up << 3) + (up << 4);  // n + 12 + 25 [s = +1], <= 49
                uint32_t f = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    // Downhill and level moves have the sentinel threshold 2^32 - 1, and
                    // every uphill threshold is below 2^32 - 1 (T <= 1e6 and dE >= 0.1),
                    // so with u clamped to 2^32 - 2 the single test u < thr is exact.
                    const uint32_t thr = tab[(key >> (8 * j)) & 0xFFu];
                    f |= (min(u[j], 0xFFFFFFFEu) < thr) ? (2u << (8 * j)) : 0u;
                }
                F[k] = f & ((~a[k] & 0x01010101u) << 1);  // vacancies never flip
                if (F[k])
                    F[k] &= gate_mask(tab[kGateWord], kb[k] + (dm[k] & 0x7FFFFFFFu), t, L.replica, (uint32_t)s,
                                      L.key0, L.key1);
            }
            if (!two)
                F[1] = 0;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (F[k]) {
                    R[ri[k]] = a[k] ^ F[k];
                    if ((ym[k] & dm[k]) >> 31) {  // a dword of this block's tile
                        const uint32_t fu = F[k] & a[k], fd = F[k] ^ fu;
                        const int cu = __popc(fu), cd = __popc(fd);
                        const uint32_t su = __builtin_amdgcn_udot4(sum[k], fu >> 1, 0u, false);
                        const uint32_t sd = __builtin_amdgcn_udot4(sum[k], fd >> 1, 0u, false);
                        dM += 2 * (cd - cu);
                        dE += 2 * ((int)su - (int)sd) - 24 * (cu - cd);
                        acc += cu + cd;
                    }
                }
            }
        }
        __syncthreads();
    }

    // Write the tile's occupied dwords to the other buffer (8-byte stores on
    // the wide path: a pair goes out if either dword holds an occupied site).
    char *out = reinterpret_cast<char *>(dst);
    if (wide) {
        constexpr uint32_t TX2 = TXD / 2;
        const uint32_t n = Z * TYR * TX2;
        for (uint32_t i = tid; i < n; i += NT) {
            const uint32_t cx = 2 * (i % TX2), q = i / TX2;
            const uint32_t ry = q % TYR, p = q / TYR + 1;
            const uint32_t y = y0 + ry, d = d0 + cx;
            const uint2 v = *reinterpret_cast<const uint2 *>(&R[(p * RYN + ry + kHY) * RX + cx + kHX]);
            if (y < Y && d < nd && (v.x != kVacant || v.y != kVacant))
                *reinterpret_cast<uint2 *>(out + p * planeb + y * rowb + d * 4u) = v;
        }
    } else {
        const uint32_t n = Z * TYR * TXD;
        for (uint32_t i = tid; i < n; i += NT) {
            const uint32_t cx = kHX + i % TXD, q = i / TXD;
            const uint32_t ry = kHY + q % TYR, p = q / TYR + 1;
            const uint32_t v = R[(p * RYN + ry) * RX + cx];
            const uint32_t ym = ymap[ry], dm = dmap[cx];
            if (((ym & dm) >> 31) && v != kVacant)
                *reinterpret_cast<uint32_t *>(out + p * planeb + (ym & 0x7FFFFFFFu) * rowb + (dm & 0x7FFFFFFFu) * 4u) = v;
        }
    }
    finish_block_to<NT>(slots_of(L, q), dM, dE, acc, tile);
    if (booker) {
        book_fold(L, 1 - q, bk, tid);
        book_advance(L, q, bk, tab, tid);
    }
}

template <int TXD, int TYR, int NT>
__global__ __launch_bounds__(NT) void k_sweep_i8_halo(LatDev L, const uint8_t *__restrict__ src,
                                                      uint8_t *__restrict__ dst, const uint8_t *__restrict__ lists,
                                                      uint32_t nbx, uint32_t per_xcd, uint32_t q) {
    const uint32_t tile = tile_of_block(blockIdx.x, per_xcd);
    if (tile >= nbx * ((L.Y + TYR - 1) / TYR))
        return;  // uniform: grid padding to a multiple of 8
    sweep_tile<TXD, TYR, NT>(L, src, dst, lists, nbx, tile, q);
}

// Batched: one launch covers one sweep of every film of a batch; block b
// works on the film whose block range [begins[f], begins[f + 1]) holds it,
// found by all threads of the block in one pass over the range starts.  Film
// f's sweep parity is (g ^ po_f) & 1 for the launch's sweep index g.
template <int TXD, int TYR, int NT>
__global__ __launch_bounds__(NT) void k_sweep_i8_halo_batch(const WholeEntry *__restrict__ ents,
                                                            const uint32_t *__restrict__ begins, uint32_t n_ents,
                                                            uint32_t g) {
    __shared__ uint32_t ent_sh;
    const uint32_t b = blockIdx.x;
    for (uint32_t i = threadIdx.x; i < n_ents; i += NT)
        if (begins[i] <= b && b < begins[i + 1])
            ent_sh = i;  // exactly one film's range holds b
    __syncthreads();
    const WholeEntry &e = ents[ent_sh];
    const uint32_t q = (g ^ e.po) & 1u;
    uint8_t *main_copy = e.lat.spins, *spare = e.spare;
    sweep_tile<TXD, TYR, NT>(e.lat, q ? spare : main_copy, q ? main_copy : spare, e.lists, e.nbx, b - e.block_begin,
                             q);
}

// ---------------------------------------------------------------------------
// Pipelined whole sweep: one block per compute unit works through several
// tiles of the same sweep, and while it runs the four phases of one tile the
// region and lists of its next tile stream from HBM straight into the other
// half of a double buffer in LDS (global-to-LDS loads, which hold no
// registers), so the load of every tile but the first hides behind compute.
// The phases, draws and acceptance are those of the single-tile kernel above;
// only the data movement differs:
//   * the halo is 4 dwords wide along x, so that every region row starts on a
//     16-byte boundary and moves as 16-byte pieces that never straddle the
//     periodic seam (rows of the film must hold a multiple of 4 dwords);
//   * the two region buffers share their padding planes: buffer 0 spans
//     planes 0 .. Z+1 and buffer 1 planes Z+1 .. 2Z+2 of one array;
//   * a tile's HBM record packs its four lists (each padded to 8 entries,
//     one 16-byte piece) behind the four counts, so a tile moves exactly its
//     occupied dwords' entries;
//   * a tile's write-back is issued after the next tile's loads are known
//     to have landed, so waiting for one never waits for the other.
constexpr int kPX = 4;               // halo dwords on each side along x (pipelined kernel)
constexpr uint32_t kPipeTiles = 32;  // most tiles per block of the pipelined kernel
// Changed-dword lists of the pipelined kernel (per tile and sweep): entries,
// the marker of a list that overflowed (or of a tile whose other copy must be
// rewritten whole), and the bytes of one HBM record (count + entries).
constexpr uint32_t kChgCap = 128;
constexpr uint32_t kChgAll = 0xFFFFFFFFu;
constexpr uint32_t kChgRecBytes = (4u + 2u * kChgCap + 15u) & ~15u;

template <int TXD, int TYR>
struct GeoP {
    static constexpr int RX = TXD + 2 * kPX;
    static constexpr int RYN = TYR + 2 * kHY;
    static constexpr int PL = RX * RYN;
    static constexpr int CH = RX / 4;  // 16-byte pieces per region row
    static_assert(TXD % 4 == 0, "tile rows must be whole 16-byte pieces");
    __host__ __device__ static constexpr int lo(int s) { return kHY - (3 - s); }
    __host__ __device__ static constexpr int hi(int s) { return kHY + TYR + (3 - s); }
    __host__ __device__ static constexpr int r0(int s) { return lo(s) + ((lo(s) ^ (s & 1)) & 1); }
    __host__ __device__ static constexpr int nry(int s) { return (hi(s) - r0(s) + 1) / 2; }
    __host__ __device__ static constexpr int cx0(int s) { return s < 3 ? kPX - 1 : kPX; }
    __host__ __device__ static constexpr int ncx(int s) { return s < 3 ? TXD + 2 : TXD; }
    __host__ __device__ static constexpr uint32_t nz(int s, uint32_t Z) { return (Z - (uint32_t)(s >> 1) + 1) / 2; }
    __host__ __device__ static constexpr uint32_t cand(int s, uint32_t Z) {
        return (uint32_t)(nry(s) * ncx(s)) * nz(s, Z);
    }
    // most 16-byte pieces of a record: the counts, then each list padded to 8 entries
    __host__ __device__ static constexpr uint32_t cap_pieces(uint32_t Z) {
        return 1u + (cand(0, Z) + 7u) / 8u + (cand(1, Z) + 7u) / 8u + (cand(2, Z) + 7u) / 8u + (cand(3, Z) + 7u) / 8u;
    }
    // then, per sweep parity, the tile's dwords that flipped in the last sweep
    // of that parity (a count, kChgCap region indices; a count above kChgCap:
    // too many to list, the whole tile is written)
    __host__ __device__ static constexpr uint32_t chg_off(uint32_t Z) { return 16u * cap_pieces(Z); }
    __host__ __device__ static constexpr uint32_t rec_bytes(uint32_t Z) {
        return (chg_off(Z) + 2u * kChgRecBytes + 255u) & ~255u;
    }
    // LDS: regions [2Z+3 planes] | lists of buffer 0 | lists of buffer 1 | row table | dword table
    __host__ __device__ static constexpr uint32_t region_words(uint32_t Z) { return (2u * Z + 3u) * PL; }
    __host__ __device__ static constexpr uint32_t list_bytes(uint32_t Z) { return 16u * cap_pieces(Z); }
    __host__ __device__ static constexpr uint32_t off_lists(uint32_t Z) { return 4u * region_words(Z); }
    __host__ __device__ static constexpr uint32_t off_rowk(uint32_t Z) { return off_lists(Z) + 2u * list_bytes(Z); }
    __host__ __device__ static constexpr uint32_t off_dmap(uint32_t Z) { return off_rowk(Z) + 4u * (Z + 2) * RYN; }
    __host__ __device__ static constexpr uint32_t lds_bytes(uint32_t Z) { return off_dmap(Z) + 4u * RX; }
};

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(3))) uint32_t lds_u32_t;
typedef __attribute__((address_space(1))) void glb_void_t;

// 16 bytes per lane from HBM into LDS: lane l's piece lands at lds_wave + 16 l
// (lds_wave is the same for the whole wave).  Completion is counted like any
// vector load; the data may be read after s_waitcnt vmcnt(0) and a barrier.
__device__ __forceinline__ void load_to_lds16(const void *g, void *lds_wave) {
    __builtin_amdgcn_global_load_lds((glb_void_t *)g, (lds_void_t *)lds_wave, 16, 0, 0);
}
// The same with 4 bytes per lane: lane l's dword lands at lds_wave + 4 l.
__device__ __forceinline__ void load_to_lds4(const void *g, void *lds_wave) {
    __builtin_amdgcn_global_load_lds((glb_void_t *)g, (lds_void_t *)lds_wave, 4, 0, 0);
}

// Workgroup barrier for LDS data only.  __syncthreads() also waits for every
// vector memory operation in flight, the loads into the other LDS buffer
// included; between the phases only this block's LDS writes must be done.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt left alone
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// The block's sums of M, E_bond and accepted flips into a slot (as
// finish_block_to), behind a barrier that waits for LDS only and with no
// barrier after the slot atomics: for the end of a kernel, where nothing
// reuses the reduction array.
template <int NT>
__device__ __forceinline__ void finish_block_lds(Slot *slots, int dM, int dE, int acc, uint32_t block_in_lat) {
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
    lds_barrier();
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
        }
    }
}

// Lists of the pipelined kernel: per tile the four counts, then the four lists
// packed (each padded to a multiple of 8 entries).  One block per tile; a
// counting pass fixes the offsets, a second pass writes the entries.
template <int TXD, int TYR>
__global__ __launch_bounds__(256) void k_pipe_lists(LatDev L, uint32_t nbx, uint8_t *lists) {
    using G = GeoP<TXD, TYR>;
    __shared__ uint32_t cnt[4], pos[4];
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t Y = L.Y, Z = L.Z, nd = L.nd;
    const uint32_t tile = blockIdx.x;
    const uint32_t bx = tile % nbx, by = tile / nbx;
    const int d0 = (int)(bx * TXD), y0 = (int)(by * TYR);
    uint8_t *rec = lists + (size_t)tile * G::rec_bytes(Z);
    uint16_t *ent = reinterpret_cast<uint16_t *>(rec);
    if (tid < 4) {
        cnt[tid] = 0;
        pos[tid] = 0;
    }
    __syncthreads();
    const char *spins = reinterpret_cast<const char *>(L.spins);
    const size_t rowb = (size_t)nd * 4u, planeb = (size_t)Y * rowb;
    for (int pass = 0; pass < 2; ++pass) {
        uint32_t base_e = 8;  // list s starts after the counts and the padded lists before it
        for (int s = 0; s < 4; ++s) {
            const uint32_t n = G::cand(s, Z);
            const uint32_t nr = (n + 255u) / 256u * 256u;
            for (uint32_t c = tid; c < nr; c += 256) {
                uint32_t ri = 0;
                bool occ = false;
                if (c < n) {
                    const uint32_t cx = G::cx0(s) + c % G::ncx(s);
                    const uint32_t q = c / G::ncx(s);
                    const uint32_t ry = G::r0(s) + 2 * (q % G::nry(s));
                    const uint32_t z = (uint32_t)(s >> 1) + 2 * (q / G::nry(s));
                    ri = ((z + 1) * G::RYN + ry) * G::RX + cx;
                    const int y = wrap_mod(y0 - kHY + (int)ry, (int)Y), d = wrap_mod(d0 - kPX + (int)cx, (int)nd);
                    const uint32_t v = *reinterpret_cast<const uint32_t *>(spins + (z + 1) * planeb +
                                                                           (size_t)y * rowb + (size_t)d * 4u);
                    occ = v != kVacant;
                }
                const uint64_t m = __ballot(occ);
                if (m) {
                    const uint32_t at =
                        __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    uint32_t b0 = 0;
                    if (lane == 0)
                        b0 = atomicAdd(pass == 0 ? &cnt[s] : &pos[s], (uint32_t)__popcll(m));
                    b0 = __builtin_amdgcn_readfirstlane(b0);  // lane 0 is active here
                    if (pass == 1 && occ)
                        ent[base_e + b0 + at] = (uint16_t)ri;
                }
            }
            if (pass == 1)
                base_e += (cnt[s] + 7u) & ~7u;
        }
        __syncthreads();
    }
    if (tid < 4)
        reinterpret_cast<uint32_t *>(rec)[tid] = cnt[tid];
    // no changed-dword list yet: the first sweeps of either parity write whole tiles
    if (tid < 2)
        *reinterpret_cast<uint32_t *>(rec + G::chg_off(Z) + tid * kChgRecBytes) = kChgAll;
}

// Marks every tile's changed-dword lists "write the whole tile" (at the start
// of a run: the copy a sweep writes may differ from the one it reads anywhere).
template <int TXD, int TYR>
__global__ __launch_bounds__(256) void k_pipe_reset_changes(uint8_t *lists, uint32_t ntiles, uint32_t Z) {
    using G = GeoP<TXD, TYR>;
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < 2u * ntiles)
        *reinterpret_cast<uint32_t *>(lists + (size_t)(i >> 1) * G::rec_bytes(Z) + G::chg_off(Z) +
                                      (i & 1u) * kChgRecBytes) = kChgAll;
}

// The tiles each block of a pipelined sweep takes: order[b * kmax + k] is block
// b's k-th tile (kNoTile past its last one).  Blocks b with b % nb == x (nb =
// min(8, G) bands, one per XCD where blocks are dealt to the 8 XCDs round
// robin) share band x of the tiles, [x * per, (x + 1) * per): neighbouring
// tiles, whose halos overlap, then run on one XCD and share its L2.  Tiles
// differ up to tenfold in occupied dwords (the height map's hills and valleys)
// and a sweep lasts as long as its busiest block, so within a band the tiles
// are sorted by their listed dwords, heaviest first, and dealt back and forth:
// round r goes to the band's blocks in order when r is even and in reverse when
// r is odd (a last, incomplete round in order), pairing the heaviest tiles
// with the lightest.  One block; a counting sort on listed dwords / 64 (ties in
// any order: which block sweeps a tile does not change the result).
constexpr uint32_t kNoTile = 0xFFFFFFFFu;

template <int TXD, int TYR>
__global__ __launch_bounds__(1024) void k_pipe_order(uint8_t *lists, uint32_t ntiles, uint32_t Z, uint32_t G,
                                                     uint32_t kmax) {
    using Geom = GeoP<TXD, TYR>;
    __shared__ uint32_t start[8][256];
    const uint32_t tid = threadIdx.x, recb = Geom::rec_bytes(Z);
    const uint32_t nb = min(8u, G), per = (ntiles + nb - 1) / nb;
    uint32_t *order = reinterpret_cast<uint32_t *>(lists + (size_t)ntiles * recb);
    auto key_of = [&](uint32_t tile) -> uint32_t {
        const uint4 c = *reinterpret_cast<const uint4 *>(lists + (size_t)tile * recb);
        return 255u - min((c.x + c.y + c.z + c.w) / 64u, 255u);  // heaviest first
    };
    for (uint32_t i = tid; i < 8 * 256; i += 1024)
        start[i >> 8][i & 255u] = 0;
    for (uint32_t i = tid; i < G * kmax; i += 1024)
        order[i] = kNoTile;
    __syncthreads();
    for (uint32_t t = tid; t < ntiles; t += 1024)
        atomicAdd(&start[t / per][key_of(t)], 1u);
    __syncthreads();
    if (tid < nb) {  // exclusive prefix sums, one band per thread
        uint32_t acc = 0;
        for (int k = 0; k < 256; ++k) {
            const uint32_t c = start[tid][k];
            start[tid][k] = acc;
            acc += c;
        }
    }
    __syncthreads();
    for (uint32_t t = tid; t < ntiles; t += 1024) {
        const uint32_t x = t / per;
        const uint32_t p = atomicAdd(&start[x][key_of(t)], 1u);  // rank within the band, heaviest first
        const uint32_t gbx = (G - x + nb - 1) / nb;              // the band's blocks: x, x + nb, ...
        const uint32_t nx = min(ntiles, (x + 1) * per) - x * per;
        const uint32_t r = p / gbx, j = p - r * gbx;
        const uint32_t jj = (p < nx / gbx * gbx && (r & 1u)) ? gbx - 1u - j : j;
        order[(jj * nb + x) * kmax + r] = t;
    }
}

// One attempt on the dword at region index qi in phase S of the pipelined
// kernel.  tab64 holds the thresholds at n + 12 + 32 [s = +1], so the key of
// four sites is one shift and OR of their neighbour sums.  (Two dwords per
// thread and iteration, interleaved, measured slower here: the register
// pressure costs more than the overlap gains.)
template <int S, int RX, int PL>
__device__ __forceinline__ void pipe_attempt(uint32_t qi, uint32_t *Rb, const uint32_t *rowk, const uint32_t *dmap,
                                             const uint32_t *tab64, uint32_t gthr, uint32_t t, const PhiloxShared &psh,
                                             const LatDev &L, uint16_t *chg, uint32_t *chg_n, int &dM, int &dE,
                                             int &acc) {
    constexpr bool kLeft = ((S & 1) ^ (S >> 1)) == 0;  // (y + z) even: the shifted columns are j - 1
    constexpr int o = kLeft ? -1 : 1;
    auto sh = [](uint32_t cur, uint32_t other) {
        return kLeft ? __builtin_amdgcn_alignbyte(cur, other, 3) : __builtin_amdgcn_alignbyte(other, cur, 1);
    };
    const uint32_t row = qi / RX, cx = qi - row * RX;
    const uint32_t rk = rowk[row], dm = dmap[cx];
    // the draw needs only the row and dword tables: its counter is formed before
    // the neighbour reads are issued (the empty asm orders them), so the draw
    // runs while those reads are in flight
    const uint32_t site4 = (rk & 0x7FFFFFFFu) + (dm & 0x7FFFFFFFu);
    asm volatile("" ::"v"(site4) : "memory");
    // The 13 reads from three bases, one per plane (z - 1, z, z + 1), each at
    // the row below and one dword further down: within a plane the reads lie at
    // most 2 RX + 2 dwords apart, so pairs of them become single two-address
    // reads with immediate offsets (the empty asm keeps the compiler from
    // folding the bases back; the pointers are LDS ones so that the reads stay
    // LDS reads).
    const lds_u32_t *Pm = (const lds_u32_t *)(Rb + (qi - PL - RX - 1));  // plane z - 1, row y - 1
    const lds_u32_t *P0 = Pm + PL, *Pp = Pm + 2 * PL;
    asm volatile("" : "+v"(Pm), "+v"(P0), "+v"(Pp));
    const uint32_t e1 = Pm[1], b1 = Pm[RX + 1], b1o = Pm[RX + 1 + o], e2 = Pm[2 * RX + 1];
    const uint32_t a1 = P0[1], a1o = P0[1 + o], a = P0[RX + 1], a2 = P0[2 * RX + 1], a2o = P0[2 * RX + 1 + o];
    const uint32_t e3 = Pp[1], b2 = Pp[RX + 1], b2o = Pp[RX + 1 + o], e4 = Pp[2 * RX + 1];
    // six rounds of the draw while the neighbour reads are in flight, the last
    // four while the threshold reads are (the empty asm pins the split)
    uint32_t u[4];
    philox_first_two(u, site4, (uint32_t)S, psh, L.key0, L.key1);
    philox_rounds<2, 6>(u, L.key0, L.key1);
    asm volatile("" : "+v"(u[0]), "+v"(u[1]), "+v"(u[2]), "+v"(u[3]));
    const uint32_t sum = (a1 + a2) + (b1 + b2) + ((sh(a1, a1o) + sh(a2, a2o)) + (sh(b1, b1o) + sh(b2, b2o))) +
                         ((e1 + e2) + (e3 + e4));
    const uint32_t key = sum | (((a >> 1) & 0x01010101u) << 5);  // n + 12 + 32 [s = +1] <= 56
    uint32_t thr[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        thr[j] = tab64[(key >> (8 * j)) & 0xFFu];
    asm volatile("" ::: "memory");
    philox_rounds<6, 10>(u, L.key0, L.key1);
    uint32_t f = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j)  // exact single test: see the acceptance note of the single-tile kernel
        f |= (min(u[j], 0xFFFFFFFEu) < thr[j]) ? (2u << (8 * j)) : 0u;
    f &= (~a & 0x01010101u) << 1;  // vacancies never flip
    if (f)
        f &= gate_mask(gthr, site4, t, L.replica, (uint32_t)S, L.key0, L.key1);
    if (f) {
        Rb[qi] = a ^ f;
        if ((rk & dm) >> 31) {  // a dword of this block's tile
            const uint32_t fu = f & a, fd = f ^ fu;
            const int cu = __popc(fu), cd = __popc(fd);
            const uint32_t su = __builtin_amdgcn_udot4(sum, fu >> 1, 0u, false);  // neighbour sums of the up flips
            const uint32_t sd = __builtin_amdgcn_udot4(sum, fd >> 1, 0u, false);  // and of the down flips
            dM += 2 * (cd - cu);
            dE += 2 * ((int)su - (int)sd) - 24 * (cu - cd);
            acc += cu + cd;
            // a dword belongs to one sublattice: it changes at most once per sweep
            const uint32_t at = atomicAdd(chg_n, 1u);
            if (at < kChgCap)
                chg[at] = (uint16_t)qi;
        }
    }
}

// All dwords of phase S listed in ls[0 .. n), one per thread and iteration;
// q0: the thread's first entry, read when the tile started.  The next entry is
// read before the current attempt, so the few waves that take a second entry
// at the end of the phase do not wait for it.  Every lane reads one (the last
// entry where it has none): a read under a lane mask made the compiler wait
// for it at once, one more LDS round trip per entry.
template <int S, int RX, int PL, int NT>
__device__ __forceinline__ void pipe_phase(const uint16_t *ls, uint32_t n, uint32_t q0, uint32_t *Rb,
                                           const uint32_t *rowk, const uint32_t *dmap, const uint32_t *tab64,
                                           uint32_t gthr, uint32_t t, const PhiloxShared &psh, const LatDev &L,
                                           uint16_t *chg, uint32_t *chg_n, int &dM, int &dE, int &acc) {
    uint32_t i = threadIdx.x, q = q0;
    while (i < n) {
        const uint32_t nxt = ls[min(i + NT, n - 1u)];
        pipe_attempt<S, RX, PL>(q, Rb, rowk, dmap, tab64, gthr, t, psh, L, chg, chg_n, dM, dE, acc);
        q = nxt;
        i += NT;
    }
}

// The books of the pipelined kernel: as book_advance, with everything it reads
// loaded when the block starts (the next step's descriptor and thresholds, the
// current thresholds), so that the block's end waits for no memory.
struct BookNext {
    uint32_t tab;         // lane < kTableWords: word `lane` of the next sweep's table
    uint32_t ns, nd, ok;  // the next step's sweeps and discarded sweeps; ok: that step exists
};

// Issued by the book-keeping wave once bk holds this sweep's position (its step
// in word 10) and the film's step count (word 33).
__device__ __forceinline__ BookNext book_next_issue(const LatDev &L, const BookLds &bk, uint32_t lane) {
    BookNext b;
    const uint32_t step = bk.w[10], n_steps = bk.w[33];
    b.ok = step + 1 < n_steps;
    b.ns = b.ok ? L.steps[step + 1].n_sweeps : 0u;
    b.nd = b.ok ? L.steps[step + 1].n_discard : 0u;
    b.tab = b.ok && lane < kTableWords ? L.tables[(size_t)(step + 1) * kTableWords + lane] : 0u;
    return b;
}

// One pipelined sweep of parity q of film L by block `blk` of the film's blocks
// (the body of the plain and the batched kernels).
template <int TXD, int TYR, int NT>
__device__ __forceinline__ void pipe_sweep(const LatDev &L, const uint8_t *__restrict__ src,
                                           uint8_t *__restrict__ dst, uint8_t *__restrict__ lists, uint32_t nbx,
                                           uint32_t ntiles, uint32_t kmax, uint32_t q, uint32_t blk) {
    using G = GeoP<TXD, TYR>;
    constexpr int RX = G::RX, RYN = G::RYN, PL = G::PL, CH = G::CH;
    extern __shared__ __align__(16) uint8_t smb[];
    __shared__ uint32_t tab64[64];  // thresholds at n + 12 + 32 [s = +1]
    __shared__ uint32_t gthr_sh, t_sh, run_sh;
    __shared__ BookLds bk;
    __shared__ uint16_t chg_sh[2][kChgCap];  // the tile's changed dwords, by tile parity
    __shared__ uint32_t chg_n_sh[2];
    __shared__ uint32_t my_tiles[kPipeTiles];

    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // the wave's index, in a scalar register
    const uint32_t Y = L.Y, Z = L.Z, nd = L.nd;
    const uint32_t np = Z + 2;
    uint32_t *R = reinterpret_cast<uint32_t *>(smb);
    uint8_t *LB = smb + G::off_lists(Z);
    uint32_t *rowk = reinterpret_cast<uint32_t *>(smb + G::off_rowk(Z));  // Philox base | tile-row flag (bit 31)
    uint32_t *dmap = reinterpret_cast<uint32_t *>(smb + G::off_dmap(Z));  // film dword | tile-dword flag (bit 31)
    const uint32_t rowb = nd * 4u;
    const uint32_t planeb = Y * rowb;  // the host checks that (Z + 2) planes fit 32-bit offsets
    const uint32_t recb = G::rec_bytes(Z);

    // This block's tiles, in the order k_pipe_order made (order[b kmax + k],
    // kNoTile past the last).  The first index is a uniform load issued before
    // anything is stored (a scalar load, which no vector load waits behind) and
    // starts the first tile's loads; the others go to LDS for the tile loop.
    const uint32_t *order = reinterpret_cast<const uint32_t *>(lists + (size_t)ntiles * recb) + blk * kmax;
    const uint32_t t0 = order[0];

    // Issue the loads of a tile's planes 1..Z and of its whole list record
    // (at capacity: its length would be one more memory round trip) into
    // buffer buf.
    // A wave's load moves up to kRowsPerLoad whole region rows of one plane (CH
    // pieces each, the other lanes idle): a lane's column piece is fixed, the
    // plane is the same for the whole wave, and only the row varies by lane.
    constexpr uint32_t kRowsPerLoad = 64 / CH;
    constexpr uint32_t kLoadsPerPlane = (RYN + kRowsPerLoad - 1) / kRowsPerLoad;
    const uint32_t lrow = lane / CH, lcol = lane - lrow * CH;
    auto issue = [&](uint32_t tile, uint32_t buf) {
        const uint32_t bx = tile % nbx, by = tile / nbx;
        const int ry0 = (int)(by * TYR) - kHY;
        uint32_t *Rb = R + (buf * (Z + 1) + 1) * PL;  // plane 1 of the buffer
        if ((nd & 3u) == 0) {  // uniform: rows of the film are whole 16-byte pieces
            int d = (int)(bx * TXD) - kPX + 4 * (int)lcol;  // within one period of the row (nd >= RX)
            d += d < 0 ? (int)nd : 0;
            d -= d >= (int)nd ? (int)nd : 0;
            const char *col = reinterpret_cast<const char *>(src) + planeb + (uint32_t)d * 4u;  // plane 1
            for (uint32_t ld = wv; ld < Z * kLoadsPerPlane; ld += NT / 64) {  // uniform
                const uint32_t p = ld / kLoadsPerPlane, r0 = (ld - p * kLoadsPerPlane) * kRowsPerLoad;
                const uint32_t ry = r0 + lrow;
                if (lrow < kRowsPerLoad && ry < (uint32_t)RYN) {
                    int y = ry0 + (int)ry;  // within one period of the film (Y >= RYN)
                    y += y < 0 ? (int)Y : 0;
                    y -= y >= (int)Y ? (int)Y : 0;
                    load_to_lds16(col + (p * planeb + (uint32_t)y * rowb), Rb + (p * RYN + r0) * RX);
                }
            }
        } else {
            // a 16-byte piece would straddle the periodic seam (or a row end):
            // every region dword by itself, 64 consecutive region dwords per load
            const char *base = reinterpret_cast<const char *>(src) + planeb;  // plane 1
            for (uint32_t ld = wv; ld * 64u < Z * (uint32_t)PL; ld += NT / 64) {  // uniform
                const uint32_t j = ld * 64u + lane;
                if (j < Z * (uint32_t)PL) {
                    const uint32_t p = j / PL, rem = j - p * PL, ry = rem / RX, c = rem - ry * RX;
                    int y = ry0 + (int)ry;  // within one period of the film (Y >= RYN)
                    y += y < 0 ? (int)Y : 0;
                    y -= y >= (int)Y ? (int)Y : 0;
                    int d = (int)(bx * TXD) - kPX + (int)c;  // within one period of the row (nd >= RX)
                    d += d < 0 ? (int)nd : 0;
                    d -= d >= (int)nd ? (int)nd : 0;
                    load_to_lds4(base + (p * planeb + (uint32_t)y * rowb + (uint32_t)d * 4u), Rb + ld * 64u);
                }
            }
        }
        const uint8_t *rec = lists + (size_t)tile * recb;
        uint8_t *lb = LB + buf * G::list_bytes(Z);
        const uint32_t pieces = G::cap_pieces(Z);
        for (uint32_t k0 = wv * 64u; k0 < pieces; k0 += NT) {
            const uint32_t k = k0 + lane;
            if (k < pieces)
                load_to_lds16(rec + 16u * k, lb + 16u * k0);
        }
    };

    // padding planes (vacancies): 0, Z + 1 (shared by the buffers) and 2Z + 2
    constexpr uint32_t PL4 = PL / 4;
    for (uint32_t i = tid; i < 3u * PL4; i += NT)
        reinterpret_cast<uint4 *>(R + (i / PL4) * (Z + 1) * PL)[i % PL4] = make_uint4(kVacant, kVacant, kVacant, kVacant);
    // Everything else the block reads before its first tile (thresholds, sweep
    // position, its other tiles' indices, the books) is loaded into registers
    // before the first tile's loads are issued and stored to LDS after they
    // have landed: stored at once, each would wait behind them.
    const bool booker = blk == 0 && tid < 64;  // the film's block 0 keeps the books
    BookRegs br;
    uint32_t cur_tab = 0;
    if (booker) {
        br = book_issue(L, 1 - q, q, tid);
        cur_tab = tid < kTableWords ? L.pos[q].table[tid] : 0u;
    }
    const SweepPos &P = L.pos[q];
    uint32_t pro_tab = 0, pro_tile = 0, pro_gthr = 0, pro_t = 0, pro_run = 0;
    if (tid < 64) {
        const uint32_t up = tid >> 5, m = tid & 31u;
        pro_tab = m < 25u ? P.table[25u * up + m] : 0u;
        pro_tile = tid < kmax ? order[tid] : kNoTile;  // kmax <= kPipeTiles
    }
    if (tid == 0) {
        pro_gthr = P.table[kGateWord];
        pro_t = (uint32_t)P.t;
        pro_run = P.run;
    }
    if (t0 != kNoTile)
        issue(t0, 0);

    int dM = 0, dE = 0, acc = 0;
    uint32_t prev = 0xFFFFFFFFu;
    char *out = reinterpret_cast<char *>(dst);
    // Write tile `tile` (in buffer buf, its changed dwords in list slot) to the
    // other copy.  That copy holds the state before the previous sweep, so the
    // dwords that changed in that sweep or in this one are all that differ; a
    // list that overflowed (or a first sweep) writes every 16-byte piece that
    // holds an occupied site instead.  This sweep's list is kept for the next.
    constexpr uint32_t TX4 = TXD / 4, kPiecesPerPlane = TX4 * TYR, kPlaneStep = NT / kPiecesPerPlane;
    static_assert(NT % kPiecesPerPlane == 0, "a block covers whole planes of a tile");
    const uint32_t wb_cx = 4 * (tid % TX4), wb_ry = (tid / TX4) % TYR, wb_p0 = tid / kPiecesPerPlane + 1;
    // n_prev, e_prev: the tile's change list of the previous sweep (its count, and
    // entry `tid` where tid < the count), loaded into registers when the tile
    // started so that the write-back waits for no memory round trip.
    static_assert(kChgCap <= NT, "one previous change per thread");
    auto write_back = [&](uint32_t tile, uint32_t buf, uint32_t slot, uint32_t n_prev, uint32_t e_prev) {
        const uint32_t bx = tile % nbx, by = tile / nbx;
        const uint32_t *Rt = R + buf * (Z + 1) * PL;
        uint8_t *chg_rec = lists + (size_t)tile * recb + G::chg_off(Z);
        uint32_t *cur = reinterpret_cast<uint32_t *>(chg_rec + q * kChgRecBytes);
        const uint32_t n_cur = chg_n_sh[slot];
        if (n_cur <= kChgCap && n_prev <= kChgCap) {
            auto put = [&](uint32_t qi) {  // listed dwords are the tile's own
                const uint32_t p = qi / PL, rem = qi - p * PL, ry = rem / RX, cx = rem - ry * RX;
                const uint32_t y = by * TYR + ry - kHY, d = bx * TXD + cx - kPX;
                *reinterpret_cast<uint32_t *>(out + (p * planeb + y * rowb + d * 4u)) = Rt[qi];
            };
            for (uint32_t i = tid; i < n_cur; i += NT)
                put(chg_sh[slot][i]);
            if (tid < n_prev)
                put(e_prev);
        } else {
            const uint32_t y = by * TYR + wb_ry, d = bx * TXD + wb_cx;
            if (y < Y && d < nd) {  // else: a ragged tile's part beyond the film
                const uint32_t *from = Rt + (wb_p0 * RYN + wb_ry + kHY) * RX + wb_cx + kPX;
                char *to = out + (wb_p0 * planeb + y * rowb + d * 4u);
                if ((nd & 3u) == 0) {  // uniform: whole 16-byte pieces
                    for (uint32_t p = wb_p0; p <= Z; p += kPlaneStep, from += kPlaneStep * PL, to += kPlaneStep * planeb) {
                        const uint4 v = *reinterpret_cast<const uint4 *>(from);
                        if (v.x != kVacant || v.y != kVacant || v.z != kVacant || v.w != kVacant)
                            *reinterpret_cast<uint4 *>(to) = v;
                    }
                } else {  // rows are not 16-byte aligned: the piece's dwords inside the row, one by one
                    const uint32_t nj = min(4u, nd - d);
                    for (uint32_t p = wb_p0; p <= Z; p += kPlaneStep, from += kPlaneStep * PL, to += kPlaneStep * planeb)
                        for (uint32_t j = 0; j < nj; ++j) {
                            const uint32_t v = from[j];
                            if (v != kVacant)
                                reinterpret_cast<uint32_t *>(to)[j] = v;
                        }
                }
            }
        }
        uint16_t *ce = reinterpret_cast<uint16_t *>(cur + 1);
        for (uint32_t i = tid; i < min(n_cur, kChgCap); i += NT)
            ce[i] = chg_sh[slot][i];
        if (tid == 0)
            cur[0] = n_cur <= kChgCap ? n_cur : kChgAll;
    };

    // A tile's change list of the previous sweep, for its write-back: the count
    // (an atomic load, so that it is a vector load and not a scalar one that every
    // LDS wait of the phases would then wait for) and entry `tid`.
    auto prev_changes = [&](uint32_t tile, uint32_t &n, uint32_t &e) {
        const uint8_t *rec = lists + (size_t)tile * recb + G::chg_off(Z) + (1u - q) * kChgRecBytes;
        n = ald(reinterpret_cast<const uint32_t *>(rec));
        e = tid < kChgCap ? (uint32_t)reinterpret_cast<const uint16_t *>(rec + 4)[tid] : 0u;
    };
    // Philox counter base and tile flags of every region row and dword of a tile.
    auto build_tables = [&](uint32_t tile) {
        const uint32_t bx = tile % nbx, by = tile / nbx;
        const int d0 = (int)(bx * TXD), y0 = (int)(by * TYR);
        const uint32_t ynd = Y * nd;
        for (uint32_t i = tid; i < np * RYN + RX; i += NT) {
            if (i < np * RYN) {
                const uint32_t p = i / RYN, ry = i % RYN;
                int y = y0 + (int)ry - kHY;  // within one period of the film (Y >= RYN)
                y += y < 0 ? (int)Y : 0;
                y -= y >= (int)Y ? (int)Y : 0;
                const bool own = ry >= (uint32_t)kHY && ry < (uint32_t)(kHY + TYR) && y0 + (int)ry - kHY < (int)Y;
                rowk[i] = (p >= 1 ? (p - 1) * ynd + (uint32_t)y * nd : 0u) | (own ? 0x80000000u : 0u);
            } else {
                const uint32_t c = i - np * RYN;
                int d = d0 + (int)c - kPX;  // within one period of the row (nd >= RX)
                d += d < 0 ? (int)nd : 0;
                d -= d >= (int)nd ? (int)nd : 0;
                const bool own = c >= (uint32_t)kPX && c < (uint32_t)(kPX + TXD) && d0 + (int)c - kPX < (int)nd;
                dmap[c] = (uint32_t)d | (own ? 0x80000000u : 0u);
            }
        }
    };

    // the first tile's tables while its loads are in flight
    if (t0 != kNoTile)
        build_tables(t0);
    uint32_t pn_prev = 0, pe_prev = 0;  // change list of the tile whose write-back is pending
    BookNext bn{};
    uint32_t k = 0;
    for (; k < kmax; ++k) {
        const uint32_t tile = k ? my_tiles[k] : t0;  // my_tiles is read after the first tile's barriers
        if (tile == kNoTile)  // uniform
            break;
        const uint32_t buf = k & 1u;
        // this tile's loads (and the write-back of two tiles ago) have landed
        __builtin_amdgcn_s_waitcnt(0);
        if (prev != 0xFFFFFFFFu) {
            write_back(prev, buf ^ 1u, buf ^ 1u, pn_prev, pe_prev);
            build_tables(tile);  // the previous tile's phases, its readers, have ended
        }
        if (tid == 0)
            chg_n_sh[buf] = 0;  // list slot of this tile (its last user, two tiles ago, is written back)
        if (k == 0) {
            if (tid < 64) {
                tab64[tid] = pro_tab;
                if (tid < kPipeTiles)
                    my_tiles[tid] = pro_tile;
            }
            if (tid == 0) {
                gthr_sh = pro_gthr;
                t_sh = pro_t;
                run_sh = pro_run;
            }
            if (booker) {
                book_stage(bk, br, tid);
                bn = book_next_issue(L, bk, tid);  // lands while the tiles are swept
            }
        }
        __syncthreads();
        const uint16_t *lb = reinterpret_cast<const uint16_t *>(LB + buf * G::list_bytes(Z));
        // the counts are read before the next tile's loads are issued: a read
        // of LDS behind those loads would wait for them
        const uint4 cnt = *reinterpret_cast<const uint4 *>(lb);
        // the next tile streams into the other buffer while this one is swept
        const uint32_t nxt = k + 1 < kmax ? my_tiles[k + 1] : kNoTile;
        if (nxt != kNoTile)
            issue(nxt, buf ^ 1u);
        // after the block's last full barrier of the tile, so that the load lands
        // while the tile is swept (a full barrier would wait for it)
        prev_changes(tile, pn_prev, pe_prev);
        prev = tile;
        if (!run_sh) {  // uniform: the schedule is finished; nothing flips
            lds_barrier();
            continue;
        }
        uint32_t *Rb = R + buf * (Z + 1) * PL;
        const uint32_t t = t_sh, gthr = gthr_sh;
        const PhiloxShared psh = philox_shared(t, L.replica, L.key0);  // the sweep's common draw parts
        const uint32_t l1 = 8u + ((cnt.x + 7u) & ~7u), l2 = l1 + ((cnt.y + 7u) & ~7u), l3 = l2 + ((cnt.z + 7u) & ~7u);
        // each thread's first entry of every phase, read together (the lists do
        // not change during the phases)
        const uint32_t f0 = tid < cnt.x ? lb[8 + tid] : 0u, f1 = tid < cnt.y ? lb[l1 + tid] : 0u;
        const uint32_t f2 = tid < cnt.z ? lb[l2 + tid] : 0u, f3 = tid < cnt.w ? lb[l3 + tid] : 0u;
        pipe_phase<0, RX, PL, NT>(lb + 8, cnt.x, f0, Rb, rowk, dmap, tab64, gthr, t, psh, L, chg_sh[buf], &chg_n_sh[buf], dM, dE, acc);
        lds_barrier();
        pipe_phase<1, RX, PL, NT>(lb + l1, cnt.y, f1, Rb, rowk, dmap, tab64, gthr, t, psh, L, chg_sh[buf], &chg_n_sh[buf], dM, dE, acc);
        lds_barrier();
        pipe_phase<2, RX, PL, NT>(lb + l2, cnt.z, f2, Rb, rowk, dmap, tab64, gthr, t, psh, L, chg_sh[buf], &chg_n_sh[buf], dM, dE, acc);
        lds_barrier();
        pipe_phase<3, RX, PL, NT>(lb + l3, cnt.w, f3, Rb, rowk, dmap, tab64, gthr, t, psh, L, chg_sh[buf], &chg_n_sh[buf], dM, dE, acc);
        lds_barrier();
    }
    if (k == 0 && booker) {  // a block without tiles (never block 0)
        book_stage(bk, br, tid);
        bn = book_next_issue(L, bk, tid);
    }
    // the sweep's slot sums and books first, with barriers that wait for LDS
    // only: the slot atomics and the last write-back's stores are then in
    // flight together, and no wave waits for either
    finish_block_lds<NT>(slots_of(L, q), dM, dE, acc, blk);
    if (booker) {
        book_fold(L, 1 - q, bk, tid);
        book_advance_pre(L, q, bk, cur_tab, bn.tab, bn.ns, bn.nd, tid);
    }
    if (prev != 0xFFFFFFFFu)
        write_back(prev, (k - 1u) & 1u, (k - 1u) & 1u, pn_prev, pe_prev);
}

template <int TXD, int TYR, int NT>
__global__ __launch_bounds__(NT) void k_sweep_i8_pipe(LatDev L, const uint8_t *__restrict__ src,
                                                      uint8_t *__restrict__ dst, uint8_t *__restrict__ lists,
                                                      uint32_t nbx, uint32_t ntiles, uint32_t kmax, uint32_t q) {
    pipe_sweep<TXD, TYR, NT>(L, src, dst, lists, nbx, ntiles, kmax, q, blockIdx.x);
}

// Batched: one launch covers one sweep of every film of a batch.  Film f owns
// the blocks [begins[f], begins[f + 1]) and sweeps its tiles with them as the
// plain kernel would with that many blocks (its lists and tile order are built
// for that count); its sweep parity is (g ^ po_f) & 1 for the launch's sweep
// index g.  A film past its schedule's end sits the launch out: its blocks
// copy the state they read, which leaves both copies equal.
template <int TXD, int TYR, int NT>
__global__ __launch_bounds__(NT) void k_sweep_i8_pipe_batch(const PipeEntry *__restrict__ ents,
                                                            const uint32_t *__restrict__ begins, uint32_t n_ents,
                                                            uint32_t g) {
    __shared__ uint32_t ent_sh;
    const uint32_t b = blockIdx.x;
    for (uint32_t i = threadIdx.x; i < n_ents; i += NT)
        if (begins[i] <= b && b < begins[i + 1])
            ent_sh = i;  // exactly one film's range holds b
    __syncthreads();
    const PipeEntry &e = ents[ent_sh];
    const uint32_t q = (g ^ e.po) & 1u;
    uint8_t *main_copy = e.lat.spins, *spare = e.spare;
    pipe_sweep<TXD, TYR, NT>(e.lat, q ? spare : main_copy, q ? main_copy : spare, e.lists, e.nbx, e.ntiles, e.kmax,
                             q, b - e.block_begin);
}

namespace {

template <int TXD, int TYR>
void grid_of(const LatDev &L, uint32_t &nbx, uint32_t &per_xcd, uint32_t &tiles) {
    nbx = (L.nd + TXD - 1) / TXD;
    tiles = nbx * ((L.Y + TYR - 1) / TYR);
    per_xcd = (tiles + 7) / 8;
}

template <int TXD, int TYR>
hipError_t launch_halo_t(const LatDev &L, const uint8_t *src, uint8_t *dst, const uint8_t *lists, uint32_t nt,
                         uint32_t q, hipStream_t s) {
    uint32_t nbx, per_xcd, tiles;
    grid_of<TXD, TYR>(L, nbx, per_xcd, tiles);
    const size_t lds = Geo<TXD, TYR>::lds_bytes(L.Z);
    const dim3 grid(per_xcd * 8);
    if (nt == 1024)
        hipLaunchKernelGGL((k_sweep_i8_halo<TXD, TYR, 1024>), grid, dim3(1024), lds, s, L, src, dst, lists, nbx,
                           per_xcd, q);
    else if (nt == 512)
        hipLaunchKernelGGL((k_sweep_i8_halo<TXD, TYR, 512>), grid, dim3(512), lds, s, L, src, dst, lists, nbx,
                           per_xcd, q);
    else
        hipLaunchKernelGGL((k_sweep_i8_halo<TXD, TYR, 256>), grid, dim3(256), lds, s, L, src, dst, lists, nbx,
                           per_xcd, q);
    return hipGetLastError();
}

template <int TXD, int TYR>
hipError_t launch_halo_batch_t(const WholeEntry *ents, const uint32_t *begins, uint32_t n_ents, uint32_t blocks,
                               uint32_t Zmax, uint32_t nt, uint32_t g, hipStream_t s) {
    const size_t lds = Geo<TXD, TYR>::lds_bytes(Zmax);
    if (nt == 1024)
        hipLaunchKernelGGL((k_sweep_i8_halo_batch<TXD, TYR, 1024>), dim3(blocks), dim3(1024), lds, s, ents, begins,
                           n_ents, g);
    else if (nt == 512)
        hipLaunchKernelGGL((k_sweep_i8_halo_batch<TXD, TYR, 512>), dim3(blocks), dim3(512), lds, s, ents, begins,
                           n_ents, g);
    else
        hipLaunchKernelGGL((k_sweep_i8_halo_batch<TXD, TYR, 256>), dim3(blocks), dim3(256), lds, s, ents, begins,
                           n_ents, g);
    return hipGetLastError();
}

template <int TXD, int TYR>
hipError_t launch_lists_t(const LatDev &L, uint8_t *lists, hipStream_t s) {
    uint32_t nbx, per_xcd, tiles;
    grid_of<TXD, TYR>(L, nbx, per_xcd, tiles);
    hipLaunchKernelGGL((k_sweep_lists<TXD, TYR>), dim3(per_xcd * 8), dim3(256), 0, s, L, nbx, per_xcd, lists);
    return hipGetLastError();
}

template <int TXD, int TYR>
uint64_t lists_bytes_t(uint32_t nd, uint32_t Y, uint32_t Z) {
    const uint64_t tiles = (uint64_t)((nd + TXD - 1) / TXD) * ((Y + TYR - 1) / TYR);
    return tiles * Geo<TXD, TYR>::rec_bytes(Z);
}

// Blocks of a pipelined sweep (one per compute unit, or more where a block
// would get more than kPipeTiles tiles) and kmax, the most tiles a block gets:
// the nb = min(8, blocks) bands hold ceil(tiles / nb) tiles each and at least
// floor(blocks / nb) blocks.
template <int TXD, int TYR>
void pipe_grid_of(const LatDev &L, uint32_t n_cu, uint32_t &nbx, uint32_t &tiles, uint32_t &blocks, uint32_t &kmax) {
    nbx = (L.nd + TXD - 1) / TXD;
    tiles = nbx * ((L.Y + TYR - 1) / TYR);
    blocks = std::max(1u, std::min(n_cu, tiles));
    for (;;) {
        const uint32_t nb = std::min(8u, blocks), per = (tiles + nb - 1) / nb;
        kmax = (per + blocks / nb - 1) / (blocks / nb);
        if (kmax <= kPipeTiles)
            break;
        blocks += nb;
    }
}

template <int TXD, int TYR>
hipError_t launch_pipe_t(const LatDev &L, const uint8_t *src, uint8_t *dst, uint8_t *lists, uint32_t nt,
                         uint32_t q, uint32_t n_cu, hipStream_t s) {
    uint32_t nbx, tiles, blocks, kmax;
    pipe_grid_of<TXD, TYR>(L, n_cu, nbx, tiles, blocks, kmax);
    const size_t lds = GeoP<TXD, TYR>::lds_bytes(L.Z);
    if (nt == 1024)
        hipLaunchKernelGGL((k_sweep_i8_pipe<TXD, TYR, 1024>), dim3(blocks), dim3(1024), lds, s, L, src, dst, lists,
                           nbx, tiles, kmax, q);
    else
        hipLaunchKernelGGL((k_sweep_i8_pipe<TXD, TYR, 512>), dim3(blocks), dim3(512), lds, s, L, src, dst, lists,
                           nbx, tiles, kmax, q);
    return hipGetLastError();
}

template <int TXD, int TYR>
hipError_t launch_pipe_batch_t(const PipeEntry *ents, const uint32_t *begins, uint32_t n_ents, uint32_t blocks,
                               uint32_t Zmax, uint32_t nt, uint32_t g, hipStream_t s) {
    const size_t lds = GeoP<TXD, TYR>::lds_bytes(Zmax);
    if (nt == 1024)
        hipLaunchKernelGGL((k_sweep_i8_pipe_batch<TXD, TYR, 1024>), dim3(blocks), dim3(1024), lds, s, ents, begins,
                           n_ents, g);
    else
        hipLaunchKernelGGL((k_sweep_i8_pipe_batch<TXD, TYR, 512>), dim3(blocks), dim3(512), lds, s, ents, begins,
                           n_ents, g);
    return hipGetLastError();
}

template <int TXD, int TYR>
uint32_t pipe_batch_static_lds_t(uint32_t nt) {
    hipFuncAttributes a{};
    const hipError_t e = nt == 1024
                             ? hipFuncGetAttributes(&a, (const void *)k_sweep_i8_pipe_batch<TXD, TYR, 1024>)
                             : hipFuncGetAttributes(&a, (const void *)k_sweep_i8_pipe_batch<TXD, TYR, 512>);
    return e == hipSuccess ? (uint32_t)a.sharedSizeBytes : 0xFFFFFFFFu;
}

template <int TXD, int TYR>
uint32_t pipe_static_lds_t(uint32_t nt) {
    hipFuncAttributes a{};
    const hipError_t e = nt == 1024 ? hipFuncGetAttributes(&a, (const void *)k_sweep_i8_pipe<TXD, TYR, 1024>)
                                    : hipFuncGetAttributes(&a, (const void *)k_sweep_i8_pipe<TXD, TYR, 512>);
    return e == hipSuccess ? (uint32_t)a.sharedSizeBytes : 0xFFFFFFFFu;
}

template <int TXD, int TYR>
hipError_t launch_pipe_lists_t(const LatDev &L, uint8_t *lists, uint32_t n_cu, hipStream_t s) {
    uint32_t nbx, tiles, blocks, kmax;
    pipe_grid_of<TXD, TYR>(L, n_cu, nbx, tiles, blocks, kmax);
    hipLaunchKernelGGL((k_pipe_lists<TXD, TYR>), dim3(tiles), dim3(256), 0, s, L, nbx, lists);
    hipLaunchKernelGGL((k_pipe_order<TXD, TYR>), dim3(1), dim3(1024), 0, s, lists, tiles, L.Z, blocks, kmax);
    return hipGetLastError();
}

template <int TXD, int TYR>
hipError_t launch_pipe_reset_t(const LatDev &L, uint8_t *lists, hipStream_t s) {
    const uint32_t nbx = (L.nd + TXD - 1) / TXD, tiles = nbx * ((L.Y + TYR - 1) / TYR);
    hipLaunchKernelGGL((k_pipe_reset_changes<TXD, TYR>), dim3((2 * tiles + 255) / 256), dim3(256), 0, s, lists,
                       tiles, L.Z);
    return hipGetLastError();
}

template <int TXD, int TYR>
uint64_t pipe_lists_bytes_t(uint32_t nd, uint32_t Y, uint32_t Z) {
    const uint64_t tiles = (uint64_t)((nd + TXD - 1) / TXD) * ((Y + TYR - 1) / TYR);
    // records, then the tile order: blocks x kmax entries, blocks <= tiles and kmax <= kPipeTiles
    return tiles * GeoP<TXD, TYR>::rec_bytes(Z) + (4ull * kPipeTiles * tiles + 255) / 256 * 256;
}

}  // namespace

#define ISF_HALO_SHAPES(X) X(16, 16) X(32, 8) X(32, 16) X(32, 32) X(64, 8) X(64, 16)

// Dynamic LDS bytes of the whole-sweep kernel for a film of Z planes, or 0 if
// (tile_x, tile_y) is not a compiled shape.
uint32_t halo_lds_bytes(uint32_t tx, uint32_t ty, uint32_t Z) {
#define ISF_CASE(A, B) \
    if (tx == A && ty == B) \
        return Geo<A, B>::lds_bytes(Z);
    ISF_HALO_SHAPES(ISF_CASE)
#undef ISF_CASE
    return 0;
}

// Region dwords of the shape (list entries are 16-bit region indices).
uint32_t halo_region_dwords(uint32_t tx, uint32_t ty, uint32_t Z) {
    return (Z + 2) * (tx + 2 * kHX) * (ty + 2 * kHY);
}

// Bytes of the per-tile lists of a shape, and the most any shape whose region
// indices fit 16 bits needs (the lists' place in the aux buffer is sized for it).
uint64_t halo_lists_bytes(uint32_t tx, uint32_t ty, uint32_t nd, uint32_t Y, uint32_t Z) {
#define ISF_CASE(A, B) \
    if (tx == A && ty == B) \
        return lists_bytes_t<A, B>(nd, Y, Z);
    ISF_HALO_SHAPES(ISF_CASE)
#undef ISF_CASE
    return 0;
}

uint64_t halo_lists_bytes_max(uint32_t nd, uint32_t Y, uint32_t Z) {
    uint64_t m = 0;
#define ISF_CASE(A, B) \
    if (halo_region_dwords(A, B, Z) <= 65536u) \
        m = std::max<uint64_t>(m, lists_bytes_t<A, B>(nd, Y, Z));
    ISF_HALO_SHAPES(ISF_CASE)
#undef ISF_CASE
    return m;
}

// Build the per-tile lists of occupied dwords (reads the film's occupancy from L.spins).
hipError_t launch_sweep_lists(const LatDev &L, const Tiling &tl, uint8_t *lists, hipStream_t s) {
#define ISF_CASE(A, B) \
    if (tl.tx == A && tl.ty == B) \
        return launch_lists_t<A, B>(L, lists, s);
    ISF_HALO_SHAPES(ISF_CASE)
#undef ISF_CASE
    return hipErrorInvalidValue;
}

// One sweep of parity q reading the film from src and writing it to dst (both
// laid out like the spin buffer; dst must already hold the film's vacancies),
// with the lists built for the same tiling; a run of such sweeps starts with
// launch_whole_prime and ends with launch_whole_flush.
hipError_t launch_sweep_i8_halo(const LatDev &L, const Tiling &tl, const uint8_t *src, uint8_t *dst,
                                const uint8_t *lists, uint32_t q, hipStream_t s) {
    const uint32_t nt = 64u * tl.ry;  // 4, 8 or 16 waves
#define ISF_CASE(A, B) \
    if (tl.tx == A && tl.ty == B) \
        return launch_halo_t<A, B>(L, src, dst, lists, nt, q, s);
    ISF_HALO_SHAPES(ISF_CASE)
#undef ISF_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_whole_prime(const LatDev &L, uint32_t q, hipStream_t s) {
    hipLaunchKernelGGL(k_whole_prime, dim3(1), dim3(64), 0, s, L, q);
    return hipGetLastError();
}

hipError_t launch_whole_flush(const LatDev &L, uint32_t q_last, hipStream_t s) {
    hipLaunchKernelGGL(k_whole_flush, dim3(1), dim3(64), 0, s, L, q_last);
    return hipGetLastError();
}

// Tiles of a film for a whole-sweep shape (0 if not a compiled shape).
uint32_t halo_tiles(uint32_t tx, uint32_t ty, uint32_t nd, uint32_t Y, uint32_t &nbx) {
    if (halo_lds_bytes(tx, ty, 1) == 0)
        return 0;
    nbx = (nd + tx - 1) / tx;
    return nbx * ((Y + ty - 1) / ty);
}

// One sweep of every film of a batch (sweep index g; Zmax: the largest film depth).
hipError_t launch_sweep_i8_halo_batch(const WholeEntry *ents, const uint32_t *begins, uint32_t n_ents,
                                      uint32_t blocks, const Tiling &tl, uint32_t Zmax, uint32_t g, hipStream_t s) {
    const uint32_t nt = 64u * tl.ry;
#define ISF_CASE(A, B) \
    if (tl.tx == A && tl.ty == B) \
        return launch_halo_batch_t<A, B>(ents, begins, n_ents, blocks, Zmax, nt, g, s);
    ISF_HALO_SHAPES(ISF_CASE)
#undef ISF_CASE
    return hipErrorInvalidValue;
}

#define ISF_PIPE_SHAPES(X) X(32, 8) X(32, 16) X(32, 32) X(64, 16)

// Pipelined whole-sweep kernel: dynamic LDS bytes for a film of Z planes (0 if
// (tile_x, tile_y) is not a compiled shape), its static LDS, region dwords
// (list entries are 16-bit region indices) and list bytes.
uint32_t pipe_lds_bytes(uint32_t tx, uint32_t ty, uint32_t Z) {
#define ISF_CASE(A, B) \
    if (tx == A && ty == B) \
        return GeoP<A, B>::lds_bytes(Z);
    ISF_PIPE_SHAPES(ISF_CASE)
#undef ISF_CASE
    return 0;
}

uint32_t pipe_static_lds(uint32_t tx, uint32_t ty, uint32_t nt) {
#define ISF_CASE(A, B) \
    if (tx == A && ty == B) \
        return pipe_static_lds_t<A, B>(nt);
    ISF_PIPE_SHAPES(ISF_CASE)
#undef ISF_CASE
    return 0xFFFFFFFFu;
}

uint32_t pipe_batch_static_lds(uint32_t tx, uint32_t ty, uint32_t nt) {
#define ISF_CASE(A, B) \
    if (tx == A && ty == B) \
        return pipe_batch_static_lds_t<A, B>(nt);
    ISF_PIPE_SHAPES(ISF_CASE)
#undef ISF_CASE
    return 0xFFFFFFFFu;
}

// The block grid of a pipelined sweep of film L with at most `cap` blocks (more
// if a block would get over kPipeTiles tiles): tiles along a row, tiles,
// blocks, most tiles per block.  The film's lists must be built with the same cap.
bool pipe_grid(const LatDev &L, uint32_t tx, uint32_t ty, uint32_t cap, uint32_t *nbx, uint32_t *tiles,
               uint32_t *blocks, uint32_t *kmax) {
#define ISF_CASE(A, B)                                                   \
    if (tx == A && ty == B) {                                            \
        pipe_grid_of<A, B>(L, cap, *nbx, *tiles, *blocks, *kmax);        \
        return true;                                                     \
    }
    ISF_PIPE_SHAPES(ISF_CASE)
#undef ISF_CASE
    return false;
}

// One batched pipelined sweep (index g) over every film of the table.
hipError_t launch_sweep_i8_pipe_batch(const PipeEntry *ents, const uint32_t *begins, uint32_t n_ents,
                                      uint32_t blocks, const Tiling &tl, uint32_t Zmax, uint32_t g, hipStream_t s) {
    const uint32_t nt = 64u * tl.ry;
#define ISF_CASE(A, B) \
    if (tl.tx == A && tl.ty == B) \
        return launch_pipe_batch_t<A, B>(ents, begins, n_ents, blocks, Zmax, nt, g, s);
    ISF_PIPE_SHAPES(ISF_CASE)
#undef ISF_CASE
    return hipErrorInvalidValue;
}

uint32_t pipe_region_dwords(uint32_t tx, uint32_t ty, uint32_t Z) {
    return (Z + 2) * (tx + 2 * kPX) * (ty + 2 * kHY);
}

uint64_t pipe_lists_bytes_max(uint32_t nd, uint32_t Y, uint32_t Z) {
    uint64_t m = 0;
#define ISF_CASE(A, B) \
    if (pipe_region_dwords(A, B, Z) <= 65536u) \
        m = std::max<uint64_t>(m, pipe_lists_bytes_t<A, B>(nd, Y, Z));
    ISF_PIPE_SHAPES(ISF_CASE)
#undef ISF_CASE
    return m;
}

hipError_t launch_pipe_lists(const LatDev &L, const Tiling &tl, uint8_t *lists, uint32_t n_cu, hipStream_t s) {
#define ISF_CASE(A, B) \
    if (tl.tx == A && tl.ty == B) \
        return launch_pipe_lists_t<A, B>(L, lists, n_cu, s);
    ISF_PIPE_SHAPES(ISF_CASE)
#undef ISF_CASE
    return hipErrorInvalidValue;
}

// Start of a run of pipelined sweeps: the first sweep of either parity writes
// whole tiles (the lists of changed dwords say nothing about the copies yet).
hipError_t launch_pipe_reset(const LatDev &L, const Tiling &tl, uint8_t *lists, hipStream_t s) {
#define ISF_CASE(A, B) \
    if (tl.tx == A && tl.ty == B) \
        return launch_pipe_reset_t<A, B>(L, lists, s);
    ISF_PIPE_SHAPES(ISF_CASE)
#undef ISF_CASE
    return hipErrorInvalidValue;
}

// One pipelined sweep of parity q from src to dst (as launch_sweep_i8_halo),
// with the lists built by launch_pipe_lists for the same shape (the sweep also
// keeps its changed dwords there); n_cu: compute units of the device (one
// block each at most).
hipError_t launch_sweep_i8_pipe(const LatDev &L, const Tiling &tl, const uint8_t *src, uint8_t *dst,
                                uint8_t *lists, uint32_t q, uint32_t n_cu, hipStream_t s) {
    const uint32_t nt = 64u * tl.ry;  // 8 or 16 waves
#define ISF_CASE(A, B) \
    if (tl.tx == A && tl.ty == B) \
        return launch_pipe_t<A, B>(L, src, dst, lists, nt, q, n_cu, s);
    ISF_PIPE_SHAPES(ISF_CASE)
#undef ISF_CASE
    return hipErrorInvalidValue;
}

}  // namespace isf
