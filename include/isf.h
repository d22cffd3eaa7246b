/*
 * isf.h -- C ABI of the MI355X (gfx950) library for Metropolis Monte Carlo of
 * the ferromagnetic Ising model on thin films built from a surface height map.
 *
 * Model (Kapitan & Nefedev, Sections 2-3 and 5):
 *   - spins S = +-1 with k = 1 and exchange J = 1 (Section 2);
 *   - Hamiltonian with an external field, Eq. (3), each bond counted once:
 *       E = E_bond - H M,  E_bond = -sum_<ij> S_i S_j,  M = sum_i S_i;
 *   - 12-neighbour lattice built from an image, rows x columns x layers
 *     (Sections 2-3).  Here: FCC in cubic-index form, sites (x, y, z) with
 *     x+y+z even, neighbours the 12 permutations of (+-1, +-1, 0), periodic
 *     in x and y, open in z; site occupied iff z < h[y][x];
 *   - Metropolis acceptance, Eq. (8) with steps 1-3 of Section 5.  The field
 *     is an integer h_num with H = h_num / 20, so the energy change of a flip
 *     is q / 10 with q = S_i (20 n_i + h_num), n_i the sum of the neighbour
 *     spins (vacancies count 0).  q <= 0 is always accepted; q > 0 is accepted
 *     iff u < floor(2^32 exp(-(q/10)/T)), computed on the host in IEEE double;
 *   - the uniform draw u of site (x, y, z) in sweep t is word (k mod 4) of
 *     Philox4x32-10 (Salmon et al., SC 2011) with key (seed mod 2^32,
 *     seed div 2^32) and counter (k div 4, t mod 2^32, replica, sigma), where
 *     k = (z Y + y)(X/2) + x div 2 and sigma = (y mod 2) + 2 (z mod 2);
 *     the random start uses counter word 3 = sigma + 4 and t = 0, and a site
 *     starts up iff its draw is < 2^31;
 *   - one sweep updates the four sublattices sigma = 0, 1, 2, 3 in turn
 *     (no two neighbours are in one sublattice, so all sites of one
 *     sublattice are updated at once); the sweep counter t counts sweeps
 *     from 0 over the life of the lattice;
 *   - a temperature or field step is a fixed number of sweeps (Section 3:
 *     each step of temperature or field gets a finite number of MC steps);
 *   - optional per step: the switching-field gate of Eq. 9 (steps 4-5 of
 *     Section 5; a site may flip only if its own gate draw passes, see
 *     isf_step.hs_num) and the anisotropy term -h_an |M| of Eq. 7 (with M
 *     frozen at the start of each sublattice phase, see isf_step.an_num).
 *
 * Every trajectory is therefore integer and reproducible bit for bit: it does
 * not depend on the storage format, tiling, batch position or device.
 *
 * Memory: the caller allocates two device buffers per lattice (spin_bytes and
 * aux_bytes from isf_lattice_bytes) and keeps them alive until
 * isf_lattice_destroy.  The library owns only the host-side handle.  Work is
 * enqueued on the caller's HIP stream.
 *
 * Errors: every function returns ISF_OK (0) or a negative code; the text of
 * the last error of the calling thread is returned by isf_last_error().  No
 * C++ exception crosses this interface.  A handle must not be used by two
 * threads at once; different handles are independent.
 */
#ifndef ISF_H
#define ISF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ISF_ABI_VERSION 2

enum {
    ISF_OK = 0,
    ISF_EINVAL = -1,  /* invalid argument (shape, temperature, field, pointer) */
    ISF_ENOSPC = -2,  /* a caller buffer is smaller than isf_lattice_bytes says */
    ISF_EHIP = -3,    /* HIP runtime error; details in isf_last_error() */
    ISF_ESTATE = -4   /* handle in the wrong state (destroyed, busy, format) */
};

enum { ISF_FORMAT_INT8 = 0, ISF_FORMAT_BITPACK = 1 };
enum { ISF_INIT_UP = 0, ISF_INIT_DOWN = 1, ISF_INIT_RANDOM = 2 };

/* Film description.  X: image width (columns), Y: image height (rows),
 * Z: number of atomic layers (Section 3).
 *   Both formats: X a multiple of 8, X >= 8; Y even, Y >= 4; 1 <= Z <= 64
 *   (a BITPACK row of W = X/2 sites takes ceil(W/32) words per bit plane).
 *   Y <= 65536, X * Y / 2 < 2^31 (bytes of one layer), X * Y * Z / 2 < 2^34
 *   (stored sites). */
typedef struct {
    uint32_t X, Y, Z;
    uint32_t replica;   /* Philox counter word 2 */
    uint64_t seed;      /* Philox key */
    uint32_t format;    /* ISF_FORMAT_* */
    uint32_t reserved;  /* must be 0 */
} isf_desc;

/* Record of one step (a run of sweeps at fixed T and field).  Sums run over
 * the kept sweeps (after the discarded ones), each term taken after the
 * sweep's last sublattice. */
typedef struct {
    int64_t M;          /* magnetisation after the step's last sweep */
    int64_t E;          /* E_bond after the step's last sweep */
    int64_t sum_M;
    int64_t sum_absM;
    int64_t sum_E;
    int64_t accepted;   /* accepted flips in the kept sweeps */
} isf_record;

/* One step of a schedule. */
typedef struct {
    double T;           /* temperature, 0 < T <= 1e6 */
    int32_t h_num;      /* field H = h_num / 20, |h_num| <= 200000 */
    uint32_t n_sweeps;  /* >= 1 */
    uint32_t n_discard; /* <= n_sweeps; sweeps not summed into the record */
    int32_t hs_num;     /* switching-field gate, Eq. 9 and steps 4-5 of Section 5: h_s = hs_num / 20,
                           |hs_num| <= 200000; a site may flip only if its gate draw (Philox tag 2) is below
                           floor(2^32 exp(-|h_s|/T)) and the Metropolis test passes; 0: no gate.  Both
                           formats, every kernel and batch mode */
    int32_t an_num;     /* anisotropy field of Eq. 7 (Section 5): the energy gains -h_an |M| with
                           h_an = an_num / 20, 0 <= an_num <= 200000; 0: no anisotropy.  M couples every
                           site, so it is frozen at its value when each sublattice phase starts: a flip of
                           spin S changes q by -an_num (|M - 2S| - |M|) / 2 with that M (an extra field
                           h_an sign(M) while |M| >= 2).  INT8 films of a single lattice, on the
                           per-sublattice kernels (ISF_KERNEL_TILES or _LIST), or on the whole-sweep
                           kernels with a workspace attached (isf_attach_aniso_workspace):
                           isf_schedule_load returns EINVAL for a bit-packed film or a whole-sweep tuning
                           without a workspace, and isf_batch_advance refuses a lattice whose loaded
                           schedule has it */
} isf_step;

typedef struct {
    int64_t M;
    int64_t E;          /* E_bond */
    int64_t n_occ;      /* occupied sites */
    int64_t n_bonds;    /* bonds between occupied sites */
    uint64_t sweeps;    /* sweep counter t */
} isf_obs;

/* Launch shape of the sweep kernels.  Every shape gives the same trajectory. */
enum { ISF_KERNEL_TILES = 0, ISF_KERNEL_LIST = 1, ISF_KERNEL_SWEEP = 2, ISF_KERNEL_PIPE = 3, ISF_KERNEL_FILM = 4 };
typedef struct {
    uint32_t tile_x;    /* dwords (4 sites) per block row: 16, 32 or 64 */
    uint32_t tile_y;    /* TILES/LIST: active rows per block, tile_x * tile_y = 256;
                           SWEEP: rows of the block's tile (16x16, 32x8, 32x16, 32x32, 64x8, 64x16);
                           PIPE: 32x16, 32x32 or 64x16 */
    uint32_t rows_per_thread; /* 1, 2 or 4 (TILES); items per thread 1 or 2 (LIST); waves per block 4, 8 or 16
                                 (SWEEP); 8 or 16 (PIPE) */
    uint32_t use_graph; /* 1: replay schedules as HIP graphs, 0: plain launches */
    uint32_t kernel;    /* ISF_KERNEL_TILES; ISF_KERNEL_LIST (INT8 with items attached); ISF_KERNEL_SWEEP
                           (INT8: one launch per sweep, the block's tile and a halo in LDS; EINVAL if the
                           shape's LDS for the film's Z exceeds the device's per-block limit); ISF_KERNEL_PIPE
                           (INT8: one launch per sweep, one block per compute unit sweeping several tiles while
                           the next tile's region streams into a second LDS buffer; EINVAL unless X is a
                           multiple of 32, X/8 and Y are at least the region's width and height, and the
                           double buffer fits the device's LDS); ISF_KERNEL_FILM (INT8, tile_x 512, tile_y 1,
                           rows_per_thread 1: one block holds the whole film in LDS and runs many sweeps per
                           launch, the books of each sweep included; EINVAL unless the film's (Z+2) Y X/8
                           dwords are at most 65536 and fit the block's LDS with the sublattice lists, and for
                           a schedule with the anisotropy term; no graphs, no launch timing) */
} isf_tuning;

typedef struct isf_lattice isf_lattice;

int32_t isf_abi_version(void);

/* Thread-local text of the last non-zero status of this thread ("" if none). */
const char *isf_last_error(void);

/* Device-buffer sizes for a film.  Writes *spin_bytes and *aux_bytes.
 * EINVAL if the description breaks the limits above or a pointer is null. */
int32_t isf_lattice_bytes(const isf_desc *d, uint64_t *spin_bytes, uint64_t *aux_bytes);

/* Build a film from the height map h_host[Y][X] (uint8, each 0 <= h <= Z;
 * copied, the caller keeps ownership) into the caller's device buffers
 * spin_dev (>= spin_bytes) and aux_dev (>= aux_bytes), set the start
 * (ISF_INIT_*), count occupied sites and bonds, and return a handle in *out.
 * stream is a hipStream_t (NULL = default stream).  Synchronises the stream
 * before returning.  EINVAL / ENOSPC / EHIP as described above. */
int32_t isf_lattice_create(const isf_desc *d, const uint8_t *h_host, int32_t init,
                           void *spin_dev, uint64_t spin_bytes, void *aux_dev, uint64_t aux_bytes,
                           void *stream, isf_lattice **out);

/* Release the host handle.  Device buffers stay the caller's. */
int32_t isf_lattice_destroy(isf_lattice *lat);

/* Run a schedule of n_steps steps (each: T, field, sweeps, discarded sweeps,
 * switching-field gate, anisotropy field; Section 3: a fixed number of MC
 * steps per temperature or field step) and write one record per step into
 * out[n_steps] (host memory).  Enqueues on the lattice's stream and
 * synchronises before writing out.  EINVAL for a step outside the limits of
 * isf_step (the whole schedule is checked before anything runs). */
int32_t isf_run_schedule(isf_lattice *lat, const isf_step *steps, uint32_t n_steps, isf_record *out);

/* n_sweeps sweeps at fixed (T, H = h_num/20); sums over the last
 * n_sweeps - n_discard sweeps.  n_sweeps = 0 returns the current state with
 * zero sums. */
int32_t isf_run_sweeps(isf_lattice *lat, double T, int32_t h_num, uint32_t n_sweeps, uint32_t n_discard,
                       isf_record *out);

/* Field ramp at fixed T (Fig. 5 of the paper: hysteresis): step i runs
 * sweeps_per_step sweeps at H = h_num[i]/20; out[n_steps]. */
int32_t isf_ramp_field(isf_lattice *lat, double T, const int32_t *h_num, uint32_t n_steps,
                       uint32_t sweeps_per_step, isf_record *out);

/* Temperature scan at fixed field (Fig. 3: M(T)); out[n_T]. */
int32_t isf_temperature_scan(isf_lattice *lat, const double *T, uint32_t n_T, int32_t h_num,
                             uint32_t sweeps_per_T, uint32_t discard_per_T, isf_record *out);

/* Current magnetisation, bond energy, counts and sweep counter. */
int32_t isf_read_observables(isf_lattice *lat, isf_obs *out);

/* Snapshot into cube_host[Z][Y][X] (int8): +-1 on occupied sites, 0 on
 * vacancies and on non-sites (x+y+z odd). */
int32_t isf_read_spins(isf_lattice *lat, int8_t *cube_host);

/* Restore a snapshot (same layout; occupied sites must hold +-1, other
 * cells are ignored) and set the sweep counter: the trajectory continues
 * exactly as if it had not been interrupted. */
int32_t isf_write_spins(isf_lattice *lat, const int8_t *cube_host, uint64_t sweeps);

/* Acceptance thresholds for (T, h_num): out[0][n+12] for S = -1 and
 * out[1][n+12] for S = +1, n in [-12, 12]; 0xFFFFFFFF means always accepted. */
int32_t isf_threshold_table(double T, int32_t h_num, uint32_t out[2][25]);

/* The switching-field gate's threshold floor(2^32 exp(-|hs_num/20|/T)) of
 * Eq. 9 (0xFFFFFFFF for hs_num = 0: no gate), as the kernels use it.  EINVAL
 * for T or |hs_num| out of range or a null output. */
int32_t isf_gate_threshold(double T, int32_t hs_num, uint32_t *out);

/* Simulated PMOKE image (Section 6): img_dev, a device buffer of at least
 * X*Y bytes, receives [Y][X] int8 pixels: +1 (white) / -1 (black) = the spin of
 * the column's surface atom, its occupied site with the largest z; 0 where
 * the column holds no occupied site.  Enqueued on the lattice's stream after
 * the sweeps already enqueued (asynchronous).  ENOSPC if bytes < X*Y. */
int32_t isf_surface_image(isf_lattice *lat, int8_t *img_dev, uint64_t bytes);

/* Film statistics from the exact counts: mean coordination z = 2 N_bonds /
 * N_occ (nearest occupied neighbours per occupied site), the critical
 * concentration p_c = 2/z of Eq. 2 (0 if z = 0) and the occupied fraction
 * N_occ / (X Y Z / 2) of the stored sites.  Host-only, synchronous. */
typedef struct {
    int64_t n_occ;
    int64_t n_bonds;
    double mean_coordination;
    double p_c;
    double concentration;
} isf_stats;
int32_t isf_film_stats(const isf_lattice *lat, isf_stats *out);

/* Occupied-dword lists (INT8 only).  Occupancy never changes, so for each
 * sublattice the dwords (4 compact sites) holding an occupied site can be
 * listed once; the list kernel then gives every block exactly the same number
 * of such dwords (balanced work whatever the film's shape) and never loads
 * all-vacant regions.  isf_items_bytes gives the size of the lists for this
 * film (the caller allocates a device buffer of at least that size, 256-byte
 * aligned, and keeps it alive with the lattice); isf_attach_items builds and
 * uploads them and selects ISF_KERNEL_LIST.  EINVAL if the film's coordinates
 * do not fit the 32-bit item encoding, ESTATE for BITPACK. */
int32_t isf_items_bytes(const isf_lattice *lat, uint64_t *bytes);
int32_t isf_attach_items(isf_lattice *lat, void *items_dev, uint64_t bytes);

/* The anisotropy term of Eq. 7 on the whole-sweep kernels (INT8).  The term
 * couples every site to M, frozen at each sublattice phase's start, and the
 * whole-sweep kernels have no film-wide phase start.  But while |M| >= 2 at a
 * phase start, the term is exactly an extra field h_an sign(M) (isf_step.an_num),
 * so a run of sweeps in which M stays at |M| >= 2 with one sign is a plain run
 * at field h_num + an_num sign(M).  With a workspace attached, isf_advance runs
 * each step of an anisotropic schedule (or its part within one call) that way:
 * it keeps a copy of the spins, the state and the step's record, runs the
 * sweeps on the whole-sweep kernel at field h_num + an_num sign(M0) (M0 the
 * magnetisation where they start), and keeps the result when every one of
 * those sweeps had |M_s| - 2 a_s >= 2, M_s its starting magnetisation and a_s
 * its flips (each flip moves M by 2, so no phase start came below |M| = 2 or
 * changed sign).  Otherwise, or when |M0| < 2, the copy is restored and the
 * sweeps run on the per-sublattice kernels (64 x 4 x 2 tiles).  The trajectory
 * is that of the per-sublattice kernels either way.  Such an isf_advance
 * synchronises the lattice's stream once or twice per step.
 * isf_aniso_workspace_bytes gives the workspace size (the spin buffer, the
 * state, one record and two threshold tables for each of up to ISF_MAX_STEPS
 * steps, rounded up); the caller allocates that much device
 * memory, 256-byte aligned, keeps it alive with the lattice and attaches it
 * with isf_attach_aniso_workspace.  Without a workspace, a whole-sweep tuning
 * and an anisotropic schedule exclude each other (EINVAL).  isf_aniso_stats
 * counts the step parts run on the whole-sweep kernel since the workspace was
 * attached and those of them run again.  EINVAL for a BITPACK film, a null or
 * misaligned buffer; ENOSPC for a short buffer. */
int32_t isf_aniso_workspace_bytes(const isf_lattice *lat, uint64_t *bytes);
int32_t isf_attach_aniso_workspace(isf_lattice *lat, void *dev, uint64_t bytes);
int32_t isf_aniso_stats(const isf_lattice *lat, uint64_t *speculated, uint64_t *redone);

/* Choose the launch shape for a lattice (validated; EINVAL if unsupported). */
int32_t isf_set_tuning(isf_lattice *lat, const isf_tuning *tuning);
int32_t isf_get_tuning(const isf_lattice *lat, isf_tuning *tuning);

/* ---------------------------------------------------------------------------
 * Incremental execution (used by the batched and served paths).
 *
 * A lattice holds at most ISF_MAX_STEPS loaded steps.  isf_schedule_load
 * uploads a schedule (thresholds, step lengths) and resets the step state;
 * M, E_bond and the sweep counter carry on.  isf_advance enqueues up to
 * max_sweeps further sweeps of the loaded schedule on the lattice's stream
 * and returns without waiting; *enqueued (may be NULL) receives the number of
 * sweeps enqueued.  isf_schedule_remaining gives the sweeps not yet enqueued.
 * isf_schedule_records waits for the stream and copies the records of the
 * first n steps (n <= loaded steps) to host memory. */
#define ISF_MAX_STEPS 1024

int32_t isf_schedule_load(isf_lattice *lat, const isf_step *steps, uint32_t n_steps);
int32_t isf_advance(isf_lattice *lat, uint32_t max_sweeps, uint64_t *enqueued);
int32_t isf_schedule_remaining(const isf_lattice *lat, uint64_t *sweeps);
int32_t isf_schedule_records(isf_lattice *lat, isf_record *out, uint32_t n);

/* Batched execution: many lattices (replicas of uneven size, each with its
 * own temperature and field schedule) advanced together.  In
 * ISF_BATCH_PHASE_LAUNCH mode one kernel launch per sublattice covers every
 * lattice; in ISF_BATCH_PERSISTENT mode one cooperative launch runs a whole
 * chunk of sweeps for all lattices, with a grid-wide barrier between
 * sublattices; in ISF_BATCH_WHOLE mode (INT8 lattices) one launch per sweep
 * runs the whole sweep of every lattice with the whole-sweep kernel
 * (ISF_KERNEL_SWEEP), in the shape of lats[0]'s tuning if it selects that
 * kernel, else 16 x 16 with 4 waves (EINVAL if that shape's LDS does not fit
 * the deepest film); in ISF_BATCH_PIPE mode (INT8 lattices) one launch per
 * sweep runs the pipelined whole-sweep kernel (ISF_KERNEL_PIPE, 32 x 32 tiles
 * with 16 waves) over every lattice it can take -- rows of at least 40
 * dwords (X >= 320), at least 40 rows, planes that fit its LDS (Z <= 8) --
 * each with its own share of the blocks (about 8 tiles per block), and the
 * others in the ISF_BATCH_PHASE_LAUNCH way.  Each lattice's
 * trajectory is identical to running it alone.
 *
 * A batch context owns a pinned host staging area for its launch table and
 * uses the caller's device workspace (isf_batch_workspace_bytes) for the
 * table on the device.  All lattices of a batch must have the same format
 * and be idle on their own streams; the batch's work runs on the batch
 * stream.  isf_batch_advance advances every lattice by min(max_sweeps, its
 * remaining sweeps) and returns without waiting; isf_batch_sync waits.
 * EINVAL for a lattice whose loaded schedule has the anisotropy term (its
 * phases need the film's own M, see isf_step.an_num). */
enum { ISF_BATCH_PHASE_LAUNCH = 0, ISF_BATCH_PERSISTENT = 1, ISF_BATCH_WHOLE = 2, ISF_BATCH_PIPE = 3 };

typedef struct isf_batch isf_batch;

int32_t isf_batch_workspace_bytes(uint32_t max_lats, uint64_t *bytes);
int32_t isf_batch_create(uint32_t max_lats, void *workspace_dev, uint64_t workspace_bytes, void *stream,
                         isf_batch **out);
int32_t isf_batch_destroy(isf_batch *b);
int32_t isf_batch_advance(isf_batch *b, isf_lattice *const *lats, uint32_t n_lats, uint32_t max_sweeps,
                          int32_t mode, uint64_t *sweeps_enqueued);
int32_t isf_batch_sync(isf_batch *b);

/* Convenience: load each lattice's full schedule (n_steps[i] <= ISF_MAX_STEPS),
 * advance all to completion and copy out[i][n_steps[i]].  Synchronous. */
int32_t isf_batch_run(isf_batch *b, isf_lattice *const *lats, uint32_t n_lats, const isf_step *const *steps,
                      const uint32_t *n_steps, isf_record *const *out, int32_t mode);

/* Measurement: enqueue up to n_sweeps further sweeps of the loaded schedule
 * as plain launches, with a pair of HIP events around every sublattice
 * launch on the lattice's stream; waits, then writes the mean duration of
 * the launches of sublattice s to ms_per_launch[s] (milliseconds) and the
 * number of sweeps run to *swept.  With ISF_KERNEL_SWEEP or ISF_KERNEL_PIPE
 * the one launch per sweep is reported in ms_per_launch[0] and the other
 * three entries are 0.
 * The trajectory is the same as isf_advance. */
int32_t isf_time_launches(isf_lattice *lat, uint32_t n_sweeps, double ms_per_launch[4], uint32_t *swept);

/* Measurement and generator check: the draw-only ceiling of a sweep.  For
 * n_sweeps sweeps t = t0, t0 + 1, ... (the Philox counter's word 1 is t mod
 * 2^32) every stored dword of the film -- vacancies included -- draws the
 * four numbers of its attempt (Section 5's uniform random number, Philox
 * counter (dword index, t, replica, sublattice), key = the film's seed), and
 * nothing else is done.  The XOR of all words drawn is written to *xor_dev, a
 * 4-byte device buffer owned by the caller; the film's spins and state are
 * not touched.  *ms (may be null) receives the launch time in milliseconds
 * from a pair of HIP events on the lattice's stream.  Synchronous.
 * Errors: ISF_EINVAL for a null xor_dev or n_sweeps = 0. */
int32_t isf_draw_xor(isf_lattice *lat, uint32_t t0, uint32_t n_sweeps, uint32_t *xor_dev, float *ms);

/* Full recount of M and E_bond from the spins on the device (not the tracked
 * values); used to check the incremental bookkeeping.  Synchronous. */
int32_t isf_recount(isf_lattice *lat, int64_t *M, int64_t *E_bond);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): the full recount of isf_recount for n
 * films given only their spin buffers, with no lattice handle and no aux
 * buffer.  descs[i] describes film i and spins_dev[i] is its device spin
 * buffer in the library's layout (isf_lattice_bytes), holding the current
 * spins: always so with the per-sublattice kernels, and after isf_read_spins
 * or isf_recount with the whole-sweep kernels, which may leave them in their
 * second copy until then.  Writes out[4 i ..
 * 4 i + 3] = {M, E_bond, N_occ, N_bonds} for film i (host memory, n x 4
 * int64).  The counters live in a fixed device array of the library, one per
 * GPU, reached through its symbol address: the call allocates nothing.  It
 * runs on the calling thread's current device, on `stream` (null: the null
 * stream), and synchronises that stream.  The counters are shared by every
 * call on one GPU: calls that overlap on one GPU race and give wrong counts.
 * Errors: ISF_ENOSPC for n > ISF_RECOUNT_MAX_FILMS; ISF_EINVAL for null
 * pointers or an invalid description. */
#define ISF_RECOUNT_MAX_FILMS 1024u
int32_t isf_recount_films(const isf_desc *descs, const void *const *spins_dev, uint32_t n, void *stream,
                          int64_t *out);

#ifdef __cplusplus
}
#endif

#endif /* ISF_H */
