/*
 * Plain CPU oracle for Metropolis dynamics of the ferromagnetic Ising model
 * on a 12-neighbour (FCC) film, as described by Kapitan & Nefedev,
 * "High Performance Calculation of Magnetic Properties and Simulation of
 * Nonequilibrium Phenomena in nanofilms":
 *   - Hamiltonian with exchange J = 1 and external field h, Eq. (3), k = 1
 *     (Section 2);
 *   - Metropolis acceptance, Eq. (8) with steps 1-3 of the algorithm in
 *     Section 5: accept a flip if the energy does not rise, otherwise accept
 *     with probability exp(-dE/T) against a uniform random number;
 *   - film built from a surface height map, rows x columns x layers
 *     (Sections 2-3).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU library
 * is checked against; it is never linked into, called by, or shared with the
 * GPU library.  It works in plain cube coordinates (x, y, z) with the
 * definition of the lattice written out, one site at a time, in the order of
 * the definition.  Speed is not a goal.
 *
 * Conventions where the paper is silent (each is a reading, not the paper's):
 *   - lattice: FCC in cubic-index form: sites are (x, y, z) with x+y+z even,
 *     0 <= x < X, 0 <= y < Y, 0 <= z < Z; neighbours are the 12 permutations
 *     of (+-1, +-1, 0); x and y are periodic, z is open; a site is occupied
 *     iff z < h[y][x];
 *   - each bond counted once: E_bond = -(1/2) sum_i s_i n_i;
 *   - field H = h_num / 20, so dE of flipping s_i is q_i / 10 with the
 *     integer q_i = s_i (20 n_i + h_num);
 *   - dE <= 0 (q <= 0) is always accepted; otherwise the flip is accepted iff
 *     u < floor(2^32 exp(-(q/10)/T)) for a uniform 32-bit draw u;
 *   - the draw for site (x, y, z) in sweep t is word (k mod 4) of
 *     Philox4x32-10 with key (seed mod 2^32, seed div 2^32) and counter
 *     (k div 4, t, replica, sigma + 4 tag), k = (z Y + y)(X/2) + x div 2,
 *     tag 0 for Metropolis, 1 for the random start and 2 for the
 *     switching-field gate;
 *   - switching-field gate (Eq. 9, steps 4-5 of the algorithm in Section 5):
 *     with h_s = hs_num / 20 (the field's units), a site may attempt the
 *     Metropolis move only if its gate draw u_g < floor(2^32 exp(-|h_s|/T));
 *     hs_num = 0 switches the gate off (probability 1).  The gate draw and the
 *     Metropolis draw both exist for every site, so the order of the two tests
 *     does not matter: the flip happens iff both pass, for downhill moves too;
 *   - one sweep visits the four sublattices sigma = (y mod 2) + 2 (z mod 2)
 *     in the order 0, 1, 2, 3; every occupied site of the sublattice gets one
 *     attempt;
 *   - anisotropy field of Eq. (7) (Section 5): the Hamiltonian gains the
 *     term -h_an |M|, h_an = an_num / 20 >= 0, which favours the sign of the
 *     spin excess.  The term couples every site to the global M, and the
 *     sites of one sublattice are updated together, so M is frozen at its
 *     value at the start of each sublattice phase: a flip of spin s then
 *     changes q by the anisotropy energy difference
 *     10 (E_an(M - 2s) - E_an(M)) = -an_num (|M - 2s| - |M|) / 2 with that
 *     M.  With one site per sublattice this is exactly serial Metropolis on
 *     the Hamiltonian of Eq. (7).
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared [-fopenmp] isf_oracle.c -lm
 * (no -ffast-math: the acceptance thresholds come from libm exp in IEEE
 * double precision).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from Salmon, Moraes, Dror and Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3" (SC 2011): ten rounds of a 4x32-bit
 * S-box built from two 32x32->64 multiplications, with a Weyl key schedule. */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Acceptance thresholds of Eq. (8): for an attempted flip with dE = q/10 > 0
 * the probability is p = exp(-dE/T); as a 32-bit threshold it is
 * floor(p * 2^32).  dE <= 0 is accepted without a draw (returned as the
 * sentinel 0xFFFFFFFF, which no q > 0 can produce for T <= 1e6). */
uint32_t orc_threshold(int32_t q, double T)
{
    if (q <= 0)
        return 0xFFFFFFFFu;
    double dE = (double)q / 10.0;
    double p = exp(-dE / T);
    return (uint32_t)floor(ldexp(p, 32));
}

/* Threshold of the switching-field gate, Eq. (9): floor(2^32 exp(-|h_s|/T)),
 * h_s = hs_num / 20; hs_num = 0 gives the sentinel (the gate always passes). */
uint32_t orc_gate_threshold(int32_t hs_num, double T)
{
    if (hs_num == 0)
        return 0xFFFFFFFFu;
    double hs = fabs((double)hs_num) / 20.0;
    double p = exp(-hs / T);
    return (uint32_t)floor(ldexp(p, 32));
}

/* Table over (s, n): entry [s>0][n+12] is the threshold of q = s (20 n + h_num). */
void orc_threshold_table(double T, int32_t h_num, uint32_t out[2][25])
{
    for (int si = 0; si < 2; ++si) {
        int s = si ? 1 : -1;
        for (int n = -12; n <= 12; ++n)
            out[si][n + 12] = orc_threshold(s * (20 * n + h_num), T);
    }
}

/* ------------------------------------------------------------------------ */
typedef struct {
    int X, Y, Z;
    uint64_t seed;
    uint32_t replica;
    uint8_t *occ;   /* [Z][Y][X] 1 iff (x,y,z) is an occupied site */
    int8_t *s;      /* [Z][Y][X] spin +-1 on occupied sites, 0 elsewhere */
    uint64_t t;     /* sweeps done so far (the Philox sweep counter) */
    int64_t M;      /* magnetisation, tracked flip by flip */
    int64_t E;      /* bond energy E_bond, tracked flip by flip */
    int64_t n_occ;
    int64_t n_bonds;
    int order;      /* site order inside a sublattice: 0 canonical, 1 reversed, 2 strided */
} orc_film;

static const int NB[12][3] = {
    { 1,  1,  0}, { 1, -1,  0}, {-1,  1,  0}, {-1, -1,  0},
    { 1,  0,  1}, { 1,  0, -1}, {-1,  0,  1}, {-1,  0, -1},
    { 0,  1,  1}, { 0,  1, -1}, { 0, -1,  1}, { 0, -1, -1},
};

static inline size_t cell(const orc_film *f, int x, int y, int z)
{
    return ((size_t)z * (size_t)f->Y + (size_t)y) * (size_t)f->X + (size_t)x;
}

/* Sum of the spins of the 12 neighbours; vacancies and z outside [0, Z) count 0. */
static int neighbour_sum(const orc_film *f, int x, int y, int z)
{
    int n = 0;
    for (int d = 0; d < 12; ++d) {
        int zz = z + NB[d][2];
        if (zz < 0 || zz >= f->Z)
            continue;
        int xx = (x + NB[d][0] + f->X) % f->X;
        int yy = (y + NB[d][1] + f->Y) % f->Y;
        n += f->s[cell(f, xx, yy, zz)];
    }
    return n;
}

static int occupied_neighbours(const orc_film *f, int x, int y, int z)
{
    int c = 0;
    for (int d = 0; d < 12; ++d) {
        int zz = z + NB[d][2];
        if (zz < 0 || zz >= f->Z)
            continue;
        int xx = (x + NB[d][0] + f->X) % f->X;
        int yy = (y + NB[d][1] + f->Y) % f->Y;
        c += f->occ[cell(f, xx, yy, zz)];
    }
    return c;
}

static uint32_t draw(const orc_film *f, int x, int y, int z, uint32_t t, uint32_t tag)
{
    uint64_t k = ((uint64_t)z * (uint64_t)f->Y + (uint64_t)y) * (uint64_t)(f->X / 2) + (uint64_t)(x / 2);
    uint32_t sigma = (uint32_t)((y & 1) + 2 * (z & 1));
    uint32_t ctr[4] = {(uint32_t)(k >> 2), t, f->replica, sigma + 4u * tag};
    uint32_t key[2] = {(uint32_t)f->seed, (uint32_t)(f->seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[k & 3];
}

/* Full recount of M and E_bond from the spins (no incremental bookkeeping). */
void orc_recount(const orc_film *f, int64_t *M, int64_t *E)
{
    int64_t m = 0, sn = 0;
    for (int z = 0; z < f->Z; ++z)
        for (int y = 0; y < f->Y; ++y)
            for (int x = 0; x < f->X; ++x) {
                int8_t s = f->s[cell(f, x, y, z)];
                if (!s)
                    continue;
                m += s;
                sn += (int64_t)s * neighbour_sum(f, x, y, z);
            }
    *M = m;
    *E = -sn / 2;
}

orc_film *orc_film_new(int X, int Y, int Z, const uint8_t *h, uint64_t seed, uint32_t replica)
{
    if (X < 4 || Y < 4 || (X & 1) || (Y & 1) || Z < 1 || !h)
        return NULL;
    orc_film *f = (orc_film *)calloc(1, sizeof(orc_film));
    if (!f)
        return NULL;
    size_t n = (size_t)X * Y * Z;
    f->X = X; f->Y = Y; f->Z = Z; f->seed = seed; f->replica = replica;
    f->occ = (uint8_t *)calloc(n, 1);
    f->s = (int8_t *)calloc(n, 1);
    if (!f->occ || !f->s) {
        free(f->occ); free(f->s); free(f);
        return NULL;
    }
    for (int z = 0; z < Z; ++z)
        for (int y = 0; y < Y; ++y)
            for (int x = 0; x < X; ++x)
                if (((x + y + z) & 1) == 0 && z < (int)h[(size_t)y * X + x]) {
                    f->occ[cell(f, x, y, z)] = 1;
                    f->n_occ++;
                }
    int64_t half_edges = 0;
    for (int z = 0; z < Z; ++z)
        for (int y = 0; y < Y; ++y)
            for (int x = 0; x < X; ++x)
                if (f->occ[cell(f, x, y, z)])
                    half_edges += occupied_neighbours(f, x, y, z);
    f->n_bonds = half_edges / 2;
    return f;
}

void orc_film_free(orc_film *f)
{
    if (!f)
        return;
    free(f->occ);
    free(f->s);
    free(f);
}

/* mode 0: all +1, 1: all -1, 2: +1 iff the INIT draw (tag 1, t = 0) is < 2^31. */
void orc_init(orc_film *f, int mode)
{
    for (int z = 0; z < f->Z; ++z)
        for (int y = 0; y < f->Y; ++y)
            for (int x = 0; x < f->X; ++x) {
                size_t c = cell(f, x, y, z);
                if (!f->occ[c]) {
                    f->s[c] = 0;
                    continue;
                }
                if (mode == 0)
                    f->s[c] = 1;
                else if (mode == 1)
                    f->s[c] = -1;
                else
                    f->s[c] = draw(f, x, y, z, 0u, 1u) < 0x80000000u ? 1 : -1;
            }
    f->t = 0;
    orc_recount(f, &f->M, &f->E);
}

void orc_set_order(orc_film *f, int order) { f->order = order; }

/* Anisotropy part of q (tenths of the energy) for flipping spin s while the
 * magnetisation is M: 10 (E_an(M - 2s) - E_an(M)) with E_an(M) = -h_an |M|
 * and h_an = an_num / 20 (Eq. 7).  |M - 2s| - |M| is -2, 0 or 2, so the
 * result is an integer. */
static int32_t anisotropy_q(int64_t M, int s, int32_t an_num)
{
    int64_t before = M < 0 ? -M : M;
    int64_t after = (M - 2 * s) < 0 ? -(M - 2 * s) : (M - 2 * s);
    return (int32_t)(-(int64_t)an_num * (after - before) / 2);
}

/* One Metropolis attempt at an occupied site (steps 1-3 of Section 5),
 * behind the switching-field gate (steps 4-5) when gate != sentinel.
 * aq[s > 0] is the anisotropy part of q for the site's spin s, and thr the
 * thresholds of the full q = s (20 n + h_num) + aq[s > 0]. */
static void attempt(orc_film *f, int x, int y, int z, int32_t h_num, const int32_t aq[2],
                    const uint32_t thr[2][25], uint32_t gate, int64_t *dM, int64_t *dE, int64_t *acc)
{
    size_t c = cell(f, x, y, z);
    if (gate != 0xFFFFFFFFu && !(draw(f, x, y, z, (uint32_t)f->t, 2u) < gate))
        return;                              /* the gate keeps the spin's orientation */
    int s = f->s[c];
    int n = neighbour_sum(f, x, y, z);
    int32_t q = s * (20 * n + h_num) + aq[s > 0];  /* 10 * (E2 - E1) */
    int accept;
    if (q <= 0) {
        accept = 1;                          /* E2 <= E1 */
    } else {
        uint32_t u = draw(f, x, y, z, (uint32_t)f->t, 0u);
        accept = u < thr[s > 0][n + 12];     /* p = exp(-dE/T) greater than the draw */
    }
    if (accept) {
        f->s[c] = (int8_t)(-s);
        *dM += -2 * s;
        *dE += 2 * s * n;
        *acc += 1;
    }
}

/* One sweep at (T, h_num): sublattices 0..3 in turn.  Returns accepted flips.
 * thr0 is the table without anisotropy; with an_num != 0 each phase builds
 * its own from the magnetisation at the phase's start. */
static int64_t sweep(orc_film *f, double T, int32_t h_num, int32_t an_num, const uint32_t thr0[2][25],
                     uint32_t gate)
{
    int64_t acc_total = 0;
    for (int sigma = 0; sigma < 4; ++sigma) {
        int py = sigma & 1, pz = sigma >> 1;
        int nrows = f->Z * f->Y;
        int64_t dM = 0, dE = 0, acc = 0;
        int32_t aq[2] = {0, 0};
        uint32_t thr_an[2][25];
        const uint32_t(*thr)[25] = thr0;
        if (an_num != 0) {
            /* M frozen for the phase */
            aq[0] = anisotropy_q(f->M, -1, an_num);
            aq[1] = anisotropy_q(f->M, 1, an_num);
            for (int si = 0; si < 2; ++si) {
                int s = si ? 1 : -1;
                for (int n = -12; n <= 12; ++n)
                    thr_an[si][n + 12] = orc_threshold(s * (20 * n + h_num) + aq[si], T);
            }
            thr = (const uint32_t(*)[25])thr_an;
        }
        /* Sites of one sublattice share no bond, so every order of visiting
         * them gives the same result; rows run in parallel when OpenMP is on. */
#pragma omp parallel for schedule(static) reduction(+ : dM, dE, acc) if ((int64_t)nrows * f->X >= 65536)
        for (int ri = 0; ri < nrows; ++ri) {
            int r = ri;
            if (f->order == 1)
                r = nrows - 1 - ri;
            else if (f->order == 2)
                r = (int)(((int64_t)ri * 7919) % nrows);  /* 7919 is prime; nrows is not a multiple */
            int z = r / f->Y, y = r % f->Y;
            if ((z & 1) != pz || (y & 1) != py)
                continue;
            for (int xi = 0; xi < f->X; ++xi) {
                int x = f->order == 1 ? f->X - 1 - xi : xi;
                if (f->occ[cell(f, x, y, z)])
                    attempt(f, x, y, z, h_num, aq, thr, gate, &dM, &dE, &acc);
            }
        }
        f->M += dM;
        f->E += dE;
        acc_total += acc;
    }
    f->t += 1;
    return acc_total;
}

/* Record of a run of sweeps at fixed (T, h_num); sums over the kept sweeps,
 * each taken after the sweep's last sublattice. */
typedef struct {
    int64_t M;         /* after the last sweep */
    int64_t E;         /* E_bond after the last sweep */
    int64_t sum_M;
    int64_t sum_absM;
    int64_t sum_E;
    int64_t accepted;
} orc_record;

/* n_sweeps sweeps at (T, h_num) behind the switching-field gate of hs_num,
 * with the anisotropy field h_an = an_num / 20 >= 0 of Eq. (7). */
int orc_run_full(orc_film *f, double T, int32_t h_num, int32_t hs_num, int32_t an_num, uint32_t n_sweeps,
                 uint32_t n_discard, orc_record *rec)
{
    if (!(T > 0.0) || n_discard > n_sweeps || an_num < 0)
        return -1;
    if (f->order == 2 && (f->Z * f->Y) % 7919 == 0)
        return -1;
    uint32_t thr[2][25];
    orc_threshold_table(T, h_num, thr);
    const uint32_t gate = orc_gate_threshold(hs_num, T);
    orc_record r;
    memset(&r, 0, sizeof r);
    for (uint32_t i = 0; i < n_sweeps; ++i) {
        int64_t acc = sweep(f, T, h_num, an_num, (const uint32_t(*)[25])thr, gate);
        if (i >= n_discard) {
            r.sum_M += f->M;
            r.sum_absM += f->M < 0 ? -f->M : f->M;
            r.sum_E += f->E;
            r.accepted += acc;
        }
    }
    r.M = f->M;
    r.E = f->E;
    if (rec)
        *rec = r;
    return 0;
}

/* n_sweeps sweeps at (T, h_num) behind the switching-field gate of hs_num. */
int orc_run_gated(orc_film *f, double T, int32_t h_num, int32_t hs_num, uint32_t n_sweeps, uint32_t n_discard,
                  orc_record *rec)
{
    return orc_run_full(f, T, h_num, hs_num, 0, n_sweeps, n_discard, rec);
}

/* n_sweeps sweeps at (T, h_num) without the gate (steps 1-3 only). */
int orc_run(orc_film *f, double T, int32_t h_num, uint32_t n_sweeps, uint32_t n_discard, orc_record *rec)
{
    return orc_run_gated(f, T, h_num, 0, n_sweeps, n_discard, rec);
}

void orc_get_spins(const orc_film *f, int8_t *cube)
{
    memcpy(cube, f->s, (size_t)f->X * f->Y * f->Z);
}

/* Load a spin cube (+-1 on occupied sites; other cells ignored) and the sweep counter. */
int orc_set_spins(orc_film *f, const int8_t *cube, uint64_t t)
{
    size_t n = (size_t)f->X * f->Y * f->Z;
    for (size_t c = 0; c < n; ++c) {
        if (f->occ[c]) {
            if (cube[c] != 1 && cube[c] != -1)
                return -1;
            f->s[c] = cube[c];
        } else {
            f->s[c] = 0;
        }
    }
    f->t = t;
    orc_recount(f, &f->M, &f->E);
    return 0;
}

/* Simulated PMOKE image (Section 6): only the surface atoms count, a white
 * pixel (+1) for spin up and a black one (-1) for spin down.  The surface atom
 * of column (x, y) is its occupied site with the largest z; a column without
 * occupied sites gives the background (0).  img is [Y][X]. */
void orc_surface_image(const orc_film *f, int8_t *img)
{
    for (int y = 0; y < f->Y; ++y)
        for (int x = 0; x < f->X; ++x) {
            int8_t v = 0;
            for (int z = f->Z - 1; z >= 0; --z)
                if (f->occ[cell(f, x, y, z)]) {
                    v = f->s[cell(f, x, y, z)];
                    break;
                }
            img[(size_t)y * f->X + x] = v;
        }
}

void orc_state(const orc_film *f, int64_t out[5])
{
    out[0] = f->M;
    out[1] = f->E;
    out[2] = f->n_occ;
    out[3] = f->n_bonds;
    out[4] = (int64_t)f->t;
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
