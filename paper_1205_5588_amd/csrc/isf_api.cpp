// C ABI of the FCC-film Ising library (declared in include/isf.h).
//
// Host side: validation, film construction (compact rows from the height
// map), threshold tables of Eq. (8), schedule bookkeeping, HIP graph replay
// and batched launch tables.  All Monte Carlo work runs in the HIP kernels of
// isf_kernels.hip / isf_bitpack.hip / isf_persistent.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "isf.h"
#include "isf_internal.h"

namespace isf {
hipError_t launch_phase_i8(const LatDev &L, const Tiling &tl, uint32_t sigma, hipStream_t s);
hipError_t launch_phase_i8_batch(const BatchEntry *ents_dev, uint32_t n_ents, uint32_t total_blocks,
                                 const Tiling &tl, uint32_t sigma, hipStream_t s);
void batch_grid_i8(const LatDev &L, const Tiling &tl, uint32_t &nbx, uint32_t &nby, uint32_t &nbz);
bool tiling_supported(const Tiling &tl);
hipError_t launch_init_i8(const LatDev &L, int32_t mode, hipStream_t s);
hipError_t launch_phase_i8_list(const LatDev &L, uint32_t ipt, bool small, uint32_t sigma, hipStream_t s);
hipError_t launch_sweep_end(const LatDev &L, hipStream_t s);
hipError_t launch_sweep_i8_halo(const LatDev &L, const Tiling &tl, const uint8_t *src, uint8_t *dst,
                                const uint8_t *lists, uint32_t q, hipStream_t s);
hipError_t launch_whole_prime(const LatDev &L, uint32_t q, hipStream_t s);
hipError_t launch_surface_image(const LatDev &L, const uint8_t *spins, int8_t *img, hipStream_t s);
hipError_t launch_draw_xor(const LatDev &L, uint32_t t0, uint32_t n_sweeps, uint32_t *out, uint32_t n_cu,
                           hipStream_t s);
hipError_t launch_sweep_i8_halo_batch(const WholeEntry *ents, const uint32_t *begins, uint32_t n_ents,
                                      uint32_t blocks, const Tiling &tl, uint32_t Zmax, uint32_t g, hipStream_t s);
uint32_t halo_tiles(uint32_t tx, uint32_t ty, uint32_t nd, uint32_t Y, uint32_t &nbx);
hipError_t launch_whole_flush(const LatDev &L, uint32_t q_last, hipStream_t s);
hipError_t launch_sweep_lists(const LatDev &L, const Tiling &tl, uint8_t *lists, hipStream_t s);
uint32_t pipe_lds_bytes(uint32_t tx, uint32_t ty, uint32_t Z);
uint32_t pipe_static_lds(uint32_t tx, uint32_t ty, uint32_t nt);
uint32_t pipe_batch_static_lds(uint32_t tx, uint32_t ty, uint32_t nt);
bool pipe_grid(const LatDev &L, uint32_t tx, uint32_t ty, uint32_t cap, uint32_t *nbx, uint32_t *tiles,
               uint32_t *blocks, uint32_t *kmax);
hipError_t launch_sweep_i8_pipe_batch(const PipeEntry *ents, const uint32_t *begins, uint32_t n_ents,
                                      uint32_t blocks, const Tiling &tl, uint32_t Zmax, uint32_t g, hipStream_t s);
uint32_t pipe_region_dwords(uint32_t tx, uint32_t ty, uint32_t Z);
uint64_t pipe_lists_bytes_max(uint32_t nd, uint32_t Y, uint32_t Z);
hipError_t launch_pipe_lists(const LatDev &L, const Tiling &tl, uint8_t *lists, uint32_t n_cu, hipStream_t s);
hipError_t launch_sweep_i8_pipe(const LatDev &L, const Tiling &tl, const uint8_t *src, uint8_t *dst,
                                uint8_t *lists, uint32_t q, uint32_t n_cu, hipStream_t s);
hipError_t launch_pipe_reset(const LatDev &L, const Tiling &tl, uint8_t *lists, hipStream_t s);
uint32_t film_lds_bytes(uint32_t Y, uint32_t Z, uint32_t nd, uint32_t max_lds);
hipError_t launch_sweep_i8_film(const LatDev &L, uint32_t n_sweeps, uint32_t lds, hipStream_t s);
uint32_t halo_lds_bytes(uint32_t tx, uint32_t ty, uint32_t Z);
uint32_t halo_region_dwords(uint32_t tx, uint32_t ty, uint32_t Z);
uint64_t halo_lists_bytes(uint32_t tx, uint32_t ty, uint32_t nd, uint32_t Y, uint32_t Z);
uint64_t halo_lists_bytes_max(uint32_t nd, uint32_t Y, uint32_t Z);
hipError_t launch_sweep_end_batch(const BatchEntry *ents_dev, uint32_t n_ents, hipStream_t s);
hipError_t launch_recount_i8(const LatDev &L, int64_t *out, hipStream_t s);

hipError_t launch_phase_bp_pos(const LatDev &L, const Tiling &tl, uint32_t sigma, uint32_t q, hipStream_t s);
hipError_t launch_phase_bp_batch(const BatchEntry *ents_dev, uint32_t n_ents, uint32_t total_blocks,
                                 const Tiling &tl, uint32_t sigma, hipStream_t s);
void batch_grid_bp(const LatDev &L, const Tiling &tl, uint32_t &nbx, uint32_t &nby, uint32_t &nbz);
bool tiling_supported_bp(const Tiling &tl);
hipError_t launch_init_bp(const LatDev &L, int32_t mode, hipStream_t s);
hipError_t launch_recount_bp(const LatDev &L, int64_t *out, hipStream_t s);

hipError_t launch_persistent(const BatchEntry *ents_dev, uint32_t n_ents, uint32_t total_blocks, uint32_t format,
                             const Tiling &tl, uint32_t n_sweeps, uint32_t *barrier, hipStream_t s,
                             uint32_t *grid_used);
}  // namespace isf

using namespace isf;

// ---------------------------------------------------------------------------
// errors
namespace {
thread_local std::string g_err;

int32_t fail(int32_t code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                             \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(ISF_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                                \
    } while (0)

int32_t validate_desc(const isf_desc *d) {
    if (!d)
        return fail(ISF_EINVAL, "null isf_desc");
    if (d->reserved)
        return fail(ISF_EINVAL, "isf_desc.reserved must be 0");
    if (d->format != ISF_FORMAT_INT8 && d->format != ISF_FORMAT_BITPACK)
        return fail(ISF_EINVAL, "unknown format %u", d->format);
    if (d->X < 8 || d->X % 8)
        return fail(ISF_EINVAL, "X=%u must be a positive multiple of 8", d->X);
    if (d->Y < 4 || (d->Y & 1))
        return fail(ISF_EINVAL, "Y=%u must be even and >= 4", d->Y);
    if (d->Z < 1 || d->Z > 64)
        return fail(ISF_EINVAL, "Z=%u must be in [1, 64]", d->Z);
    if (d->Y > 65536 || (uint64_t)d->X * d->Y / 2 >= (1ull << 31))
        return fail(ISF_EINVAL, "plane too large: Y=%u must be <= 65536 and X*Y/2 < 2^31", d->Y);
    const uint64_t nc = (uint64_t)d->X * d->Y * d->Z / 2;
    if (nc >= (1ull << 34))
        return fail(ISF_EINVAL, "film too large: %llu stored sites >= 2^34", (unsigned long long)nc);
    return ISF_OK;
}

int32_t validate_T(double T) {
    if (!std::isfinite(T) || !(T > 0.0) || T > 1e6)
        return fail(ISF_EINVAL, "temperature %g must be finite with 0 < T <= 1e6", T);
    return ISF_OK;
}

int32_t validate_h(int32_t h) {
    if (h > 200000 || h < -200000)
        return fail(ISF_EINVAL, "|h_num| = %d exceeds 200000", h);
    return ISF_OK;
}

uint64_t spin_bytes_of(const isf_desc *d) {
    const uint64_t W = d->X / 2;
    if (d->format == ISF_FORMAT_INT8)
        return (uint64_t)(d->Z + 2) * d->Y * W;
    return (uint64_t)(d->Z + 2) * d->Y * 2 * ((W + 31) / 32) * 4;
}

// The aux buffer: device state, slots, schedule, tables and records, then (INT8)
// the spare copy of the spins and the per-tile lists used by the whole-sweep
// kernels (sized for the shape that needs the most).
uint64_t spare_offset() { return (aux_layout(ISF_MAX_STEPS).total + 4095) / 4096 * 4096; }

uint64_t lists_offset(const isf_desc *d) { return (spare_offset() + spin_bytes_of(d) + 4095) / 4096 * 4096; }

uint64_t aux_bytes_of(const isf_desc *d) {
    if (d->format != ISF_FORMAT_INT8)
        return aux_layout(ISF_MAX_STEPS).total;
    return lists_offset(d) + std::max(halo_lists_bytes_max(d->X / 8, d->Y, d->Z),
                                      pipe_lists_bytes_max(d->X / 8, d->Y, d->Z));
}

// One launch per sweep (the single-tile or the pipelined whole-sweep kernel).
bool is_whole(uint32_t kernel) { return kernel == ISF_KERNEL_SWEEP || kernel == ISF_KERNEL_PIPE; }

// Threshold of Eq. (8) for an uphill move with dE = q/10: floor(2^32 exp(-dE/T)).
uint32_t threshold_of(int32_t q, double T) {
    if (q <= 0)
        return kSentinel;
    const double p = std::exp(-((double)q / 10.0) / T);
    return (uint32_t)std::floor(std::ldexp(p, 32));
}

// Threshold of the switching-field gate, Eq. (9): floor(2^32 exp(-|h_s|/T)),
// h_s = hs / 20; hs = 0 (no gate) gives the sentinel.
uint32_t gate_threshold_of(int32_t hs, double T) {
    if (hs == 0)
        return kSentinel;
    const double p = std::exp(-(std::fabs((double)hs) / 20.0) / T);
    return (uint32_t)std::floor(std::ldexp(p, 32));
}

// Thresholds of q + an (words [0, 50)) and q - an (words [50, 100)), q = s (20 n + h),
// for the anisotropy of Eq. (7); aniso_select (isf_device.h) picks the halves of a phase.
void aniso_table_of(double T, int32_t h, int32_t an, uint32_t *out /* kAnWords */) {
    for (int si = 0; si < 2; ++si) {
        const int s = si ? 1 : -1;
        for (int n = -12; n <= 12; ++n) {
            out[si * 25 + n + 12] = threshold_of(s * (20 * n + h) + an, T);
            out[50 + si * 25 + n + 12] = threshold_of(s * (20 * n + h) - an, T);
        }
    }
}

void table_of(double T, int32_t h, int32_t hs, uint32_t *out /* kTableWords */) {
    for (int si = 0; si < 2; ++si) {
        const int s = si ? 1 : -1;
        for (int n = -12; n <= 12; ++n)
            out[si * 25 + n + 12] = threshold_of(s * (20 * n + h), T);
    }
    out[kGateWord] = gate_threshold_of(hs, T);
    out[51] = 0;
}

}  // namespace

// ---------------------------------------------------------------------------
struct isf_lattice {
    isf_desc d;
    LatDev L;
    AuxLayout aux;
    uint8_t *aux_dev;
    hipStream_t stream;
    int device;
    uint32_t n_cu;  // compute units of the device
    Tiling tiling;
    bool use_graph;
    int64_t n_occ, n_bonds;
    // loaded schedule, mirrored on the host
    uint32_t sched_steps;
    uint64_t sched_total;      // sweeps in the loaded schedule
    uint64_t sched_enqueued;   // sweeps enqueued so far
    // cached graph of graph_sweeps sweeps, and one of the last shorter count
    // asked for (a request's remainder, e.g. one field step)
    hipGraphExec_t graph;
    uint32_t graph_sweeps;
    Tiling graph_tiling;
    hipGraphExec_t tail_graph;
    uint32_t tail_sweeps;
    Tiling tail_tiling;
    // occupied-dword lists attached (INT8)
    bool items_attached;
    // second copy of the spins for the whole-sweep kernel (INT8), at the end of
    // the aux buffer; cur_spare: the current state is in the spare copy;
    // spare_ready: the spare copy holds the film's vacancies
    uint8_t *spare;
    bool cur_spare;
    bool spare_ready;
    // per-tile lists of occupied dwords of the whole-sweep kernel (after the
    // spare copy in the aux buffer), valid for lists_tiling when lists_ready
    uint8_t *lists;
    bool lists_ready;
    Tiling lists_tiling;
    uint32_t lists_blocks;  // pipelined kernel: the block cap its tile order was built for
    // a run of whole-sweep launches is open: the schedule position lives in the
    // parity-buffered positions until k_whole_flush hands it back
    bool whole_active;
    // parity of the next sweep of a bit-packed film, whose per-sublattice
    // launches carry their books as the whole-sweep kernels do (the INT8
    // whole-sweep kernels take theirs from cur_spare)
    uint32_t bq;
    // the loaded schedule has the anisotropy term (also in L.aniso, which the
    // phase kernels read)
    bool aniso;
    // the anisotropy term on the whole-sweep kernels: the caller's workspace
    // (a copy of the spins, the state and a record, taken before each step),
    // the loaded anisotropic schedule on the host, the host's copy of the
    // schedule position (step, sweeps of it enqueued), and M and the step's
    // accepted count at that position when a synchronisation has read them
    uint8_t *spec_ws;
    uint64_t spec_bytes;
    std::vector<isf_step> spec_steps;
    uint32_t spec_step, spec_sis;
    bool spec_known;
    int64_t spec_M;
    uint64_t spec_runs, spec_redone;
};

struct isf_batch {
    uint32_t max_lats;
    uint8_t *ws_dev;
    uint64_t ws_bytes;
    hipStream_t stream;
    void *staging;         // pinned host: BatchEntry or WholeEntry records
    hipEvent_t staged;     // recorded after the last staging copy
    bool persistent_used;  // a persistent launch ran since the last check
    // cached graphs of the launches of kBatchGraphSweeps sweeps, for the launch
    // sequences graph_key names (mode, table size, blocks, shape, format,
    // depth); two, since the pipelined mode also runs a sublattice sequence
    hipGraphExec_t graph[2];
    uint64_t graph_key[2][4];
    uint32_t graph_next;  // the slot a new sequence replaces
};

namespace {

// Launches that carry their sweep's books (positions and slots by sweep
// parity, opened by k_whole_prime and closed by k_whole_flush): the whole-sweep
// kernels, and the per-sublattice launches of a bit-packed film, whose first
// sublattice folds the sweep before it.
bool books_bp(const isf_lattice *lat) { return lat->d.format == ISF_FORMAT_BITPACK; }
bool books_in_launch(const isf_lattice *lat) { return is_whole(lat->tiling.kernel) || books_bp(lat); }
uint32_t run_parity(const isf_lattice *lat) { return books_bp(lat) ? lat->bq : (lat->cur_spare ? 1u : 0u); }

int32_t set_device_of(const isf_lattice *lat) {
    HIP_TRY(hipSetDevice(lat->device));
    return ISF_OK;
}

int32_t launch_phase(const isf_lattice *lat, uint32_t sigma) {
    hipError_t e;
    if (lat->d.format == ISF_FORMAT_INT8 && lat->tiling.kernel == ISF_KERNEL_LIST)
        e = launch_phase_i8_list(lat->L, lat->tiling.ry, spin_bytes_of(&lat->d) < (1ull << 32), sigma, lat->stream);
    else if (lat->d.format == ISF_FORMAT_INT8)
        e = launch_phase_i8(lat->L, lat->tiling, sigma, lat->stream);
    else
        e = launch_phase_bp_pos(lat->L, lat->tiling, sigma, lat->bq, lat->stream);
    if (e != hipSuccess)
        return fail(ISF_EHIP, "phase launch failed: %s", hipGetErrorString(e));
    return ISF_OK;
}

// After a sweep's four sublattice launches: the one-wave sweep end, or for a
// bit-packed film (whose next sweep's first launch folds this one) the flip of
// the sweep parity.
int32_t launch_end(isf_lattice *lat) {
    if (books_bp(lat)) {
        lat->bq ^= 1u;
        return ISF_OK;
    }
    hipError_t e = launch_sweep_end(lat->L, lat->stream);
    if (e != hipSuccess)
        return fail(ISF_EHIP, "sweep-end launch failed: %s", hipGetErrorString(e));
    return ISF_OK;
}

// The whole-sweep kernel reads one copy of the spins and writes the other.
// The spare copy gets the film's layout (its vacancies) once, before its
// first use; after a whole sweep the state may sit in the spare copy, and
// settle() moves it back before anything else reads or writes the spins.
// cap: for the pipelined kernel, the most blocks a sweep of this film uses (its
// tile order is built for that count): the device's compute units when the
// film runs alone, its share of a batched launch otherwise.
int32_t prepare_spare(isf_lattice *lat, const Tiling &tl, uint32_t cap = 0) {
    if (!lat->spare_ready) {
        HIP_TRY(hipMemcpyAsync(lat->spare, lat->L.spins, spin_bytes_of(&lat->d), hipMemcpyDeviceToDevice,
                               lat->stream));
        lat->spare_ready = true;
    }
    const bool pipe = tl.kernel == ISF_KERNEL_PIPE;
    if (!cap)
        cap = lat->n_cu;
    const Tiling &lt = lat->lists_tiling;
    if (!lat->lists_ready || lt.tx != tl.tx || lt.ty != tl.ty || lt.kernel != tl.kernel ||
        (pipe && lat->lists_blocks != cap)) {
        hipError_t e = pipe ? launch_pipe_lists(lat->L, tl, lat->lists, cap, lat->stream)
                            : launch_sweep_lists(lat->L, tl, lat->lists, lat->stream);
        if (e != hipSuccess)
            return fail(ISF_EHIP, "list launch failed: %s", hipGetErrorString(e));
        lat->lists_ready = true;
        lat->lists_tiling = tl;
        lat->lists_blocks = cap;
    }
    return ISF_OK;
}

// Open a run of whole-sweep launches (before the first one is enqueued or captured).
int32_t prime_whole(isf_lattice *lat) {
    if (!lat->whole_active) {
        hipError_t e = launch_whole_prime(lat->L, run_parity(lat), lat->stream);
        if (e == hipSuccess && lat->lists_ready && lat->lists_tiling.kernel == ISF_KERNEL_PIPE)
            e = launch_pipe_reset(lat->L, lat->lists_tiling, lat->lists, lat->stream);
        if (e != hipSuccess)
            return fail(ISF_EHIP, "prime launch failed: %s", hipGetErrorString(e));
        lat->whole_active = true;
    }
    return ISF_OK;
}

// Whether the pipelined kernel of shape tl can sweep this film when its LDS is
// sized for Zlds planes (Zlds >= the film's Z; a batch sizes it for its deepest
// film): ISF_OK or the reason (ISF_EINVAL, with the message set).
int32_t pipe_fits(const isf_lattice *lat, const Tiling &tl, uint32_t Zlds, bool batched) {
    const uint32_t nd = lat->d.X / 8, Y = lat->d.Y, Z = lat->d.Z;
    const uint32_t lds = pipe_lds_bytes(tl.tx, tl.ty, Zlds);
    if (lds == 0 || (tl.ry != 8 && tl.ry != 16))
        return fail(ISF_EINVAL, "unsupported pipelined shape %ux%u with %u waves", tl.tx, tl.ty, tl.ry);
    // a region (tile and halo) within one period of the film along x and y
    if (nd < tl.tx + 8 || Y < tl.ty + 8)
        return fail(ISF_EINVAL, "pipelined shape %ux%u needs X/8 >= %u and Y >= %u", tl.tx, tl.ty, tl.tx + 8,
                    tl.ty + 8);
    // compact dword indices below 2^31 (bit 31 flags the tile's rows) and plane offsets within 32 bits
    if ((uint64_t)Z * Y * nd >= (1ull << 31) || (uint64_t)(Z + 2) * Y * nd * 4 >= (1ull << 32))
        return fail(ISF_EINVAL, "film too large for the pipelined kernel");
    int max_lds = 0;
    HIP_TRY(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, lat->device));
    const uint32_t st = batched ? pipe_batch_static_lds(tl.tx, tl.ty, 64u * tl.ry)
                                : pipe_static_lds(tl.tx, tl.ty, 64u * tl.ry);
    const uint64_t need = (uint64_t)lds + st;
    if (need > (uint64_t)max_lds || pipe_region_dwords(tl.tx, tl.ty, Zlds) > 65536u)
        return fail(ISF_EINVAL, "pipelined shape %ux%u needs %llu bytes of LDS for Z = %u (limit %d)", tl.tx, tl.ty,
                    (unsigned long long)need, Zlds, max_lds);
    return ISF_OK;
}

// Close the run: fold the last sweep, whose parity is the opposite of the next one's.
int32_t flush_whole(isf_lattice *lat) {
    if (lat->whole_active) {
        hipError_t e = launch_whole_flush(lat->L, 1u - run_parity(lat), lat->stream);
        if (e != hipSuccess)
            return fail(ISF_EHIP, "flush launch failed: %s", hipGetErrorString(e));
        lat->whole_active = false;
    }
    return ISF_OK;
}

int32_t settle(isf_lattice *lat) {
    int32_t rc = flush_whole(lat);  // the parity must be read before the spins move back
    if (rc)
        return rc;
    if (lat->cur_spare) {
        HIP_TRY(hipMemcpyAsync(lat->L.spins, lat->spare, spin_bytes_of(&lat->d), hipMemcpyDeviceToDevice,
                               lat->stream));
        lat->cur_spare = false;
    }
    return ISF_OK;
}

// Sweep parity q = 1 when the current spins are in the spare copy.
int32_t launch_whole_sweep(isf_lattice *lat) {
    uint8_t *a = lat->L.spins, *b = lat->spare;
    const uint8_t *src = lat->cur_spare ? b : a;
    uint8_t *dst = lat->cur_spare ? a : b;
    const uint32_t q = lat->cur_spare ? 1u : 0u;
    hipError_t e = lat->tiling.kernel == ISF_KERNEL_PIPE
                       ? launch_sweep_i8_pipe(lat->L, lat->tiling, src, dst, lat->lists, q, lat->n_cu, lat->stream)
                       : launch_sweep_i8_halo(lat->L, lat->tiling, src, dst, lat->lists, q, lat->stream);
    if (e != hipSuccess)
        return fail(ISF_EHIP, "sweep launch failed: %s", hipGetErrorString(e));
    lat->cur_spare = !lat->cur_spare;
    return ISF_OK;
}

// One sweep = one whole-sweep launch (its bookkeeping rides in the launch), or
// four sublattice launches and the one-wave sweep-end launch.
int32_t enqueue_sweeps_plain(isf_lattice *lat, uint64_t n) {
    const bool whole = is_whole(lat->tiling.kernel);
    for (uint64_t i = 0; i < n; ++i) {
        if (whole) {
            int32_t rc = launch_whole_sweep(lat);
            if (rc)
                return rc;
            continue;
        }
        for (uint32_t s = 0; s < 4; ++s) {
            int32_t rc = launch_phase(lat, s);
            if (rc)
                return rc;
        }
        int32_t rc = launch_end(lat);
        if (rc)
            return rc;
    }
    return ISF_OK;
}

constexpr uint32_t kGraphSweeps = 64;
constexpr uint32_t kTailGraphMin = 16;  // shorter remainders run as plain launches

void drop_graph(isf_lattice *lat) {
    if (lat->graph) {
        (void)hipGraphExecDestroy(lat->graph);
        lat->graph = nullptr;
    }
    if (lat->tail_graph) {
        (void)hipGraphExecDestroy(lat->tail_graph);
        lat->tail_graph = nullptr;
    }
}

bool same_tiling(const Tiling &a, const Tiling &b) {
    return a.tx == b.tx && a.ty == b.ty && a.ry == b.ry && a.kernel == b.kernel;
}

// Capture `sweeps` sweeps of plain launches into an executable graph.  A
// whole-sweep capture must hold an even number of sweeps and start on the main
// spin copy: the launches alternate the two copies, and every replay starts
// where the capture did.
int32_t capture_graph(isf_lattice *lat, uint32_t sweeps, hipGraphExec_t *out) {
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(lat->stream, hipStreamCaptureModeThreadLocal));
    int32_t rc = enqueue_sweeps_plain(lat, sweeps);
    hipError_t e = hipStreamEndCapture(lat->stream, &g);
    if (rc) {
        if (g)
            (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess)
        return fail(ISF_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        *out = nullptr;
        return fail(ISF_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return ISF_OK;
}

int32_t build_graph(isf_lattice *lat) {
    drop_graph(lat);
    int32_t rc = capture_graph(lat, kGraphSweeps, &lat->graph);
    if (rc)
        return rc;
    lat->graph_sweeps = kGraphSweeps;
    lat->graph_tiling = lat->tiling;
    return ISF_OK;
}

int32_t build_tail_graph(isf_lattice *lat, uint32_t sweeps) {
    if (lat->tail_graph) {
        (void)hipGraphExecDestroy(lat->tail_graph);
        lat->tail_graph = nullptr;
    }
    int32_t rc = capture_graph(lat, sweeps, &lat->tail_graph);
    if (rc)
        return rc;
    lat->tail_sweeps = sweeps;
    lat->tail_tiling = lat->tiling;
    return ISF_OK;
}

// The film kernel: one block, many sweeps per launch (at most kFilmChunk each).
constexpr uint64_t kFilmChunk = 4096;

int32_t enqueue_sweeps_film(isf_lattice *lat, uint64_t n) {
    int32_t rc;
    if ((rc = settle(lat)))
        return rc;
    int max_lds = 0;
    HIP_TRY(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, lat->device));
    const uint32_t lds = film_lds_bytes(lat->d.Y, lat->d.Z, lat->L.nd, (uint32_t)max_lds);
    if (!lds)
        return fail(ISF_EINVAL, "the film does not fit one block's LDS");
    while (n > 0) {
        const uint64_t k = std::min(n, kFilmChunk);
        hipError_t e = launch_sweep_i8_film(lat->L, (uint32_t)k, lds, lat->stream);
        if (e != hipSuccess)
            return fail(ISF_EHIP, "film kernel launch failed: %s", hipGetErrorString(e));
        n -= k;
    }
    return ISF_OK;
}

int32_t enqueue_sweeps(isf_lattice *lat, uint64_t n) {
    int32_t rc0;
    if (lat->tiling.kernel == ISF_KERNEL_FILM)
        return enqueue_sweeps_film(lat, n);
    if (books_in_launch(lat)) {
        if ((is_whole(lat->tiling.kernel) && (rc0 = prepare_spare(lat, lat->tiling))) || (rc0 = prime_whole(lat)))
            return rc0;
        // graphs hold an even number of sweeps and start at parity 0 (for the
        // whole-sweep kernels: from the main copy)
        if (run_parity(lat) && n > 0) {
            if ((rc0 = enqueue_sweeps_plain(lat, 1)))
                return rc0;
            --n;
        }
    } else if ((rc0 = settle(lat))) {
        return rc0;
    }
    if (lat->use_graph && lat->stream && n >= kGraphSweeps) {
        if (!lat->graph || !same_tiling(lat->graph_tiling, lat->tiling)) {
            int32_t rc = build_graph(lat);
            if (rc)
                return rc;
        }
        while (n >= lat->graph_sweeps) {
            HIP_TRY(hipGraphLaunch(lat->graph, lat->stream));
            n -= lat->graph_sweeps;
        }
    }
    // the remainder: a graph of exactly that many sweeps, cached for the next
    // request of the same length (whole-sweep graphs need an even count)
    if (lat->use_graph && lat->stream && n >= kTailGraphMin && (n % 2 == 0 || !books_in_launch(lat))) {
        if (!lat->tail_graph || lat->tail_sweeps != n || !same_tiling(lat->tail_tiling, lat->tiling)) {
            int32_t rc = build_tail_graph(lat, (uint32_t)n);
            if (rc)
                return rc;
        }
        HIP_TRY(hipGraphLaunch(lat->tail_graph, lat->stream));
        n = 0;
    }
    return enqueue_sweeps_plain(lat, n);
}

// ---------------------------------------------------------------------------
// The anisotropy term of Eq. (7) on the whole-sweep kernels.  While |M| >= 2 at
// every sublattice phase start, a flip of spin s changes q by an s sign(M), so
// the sweeps are plain sweeps at field h_num + an_num sign(M).  Each step (or its
// part within one advance) is run that way from a copy of the spins, the state
// and the step's record, and kept when every sweep of it had |M0| - 2 a >= 2
// (M0 its starting magnetisation, a its flips: every flip moves M by 2, so no
// phase start within the sweep, and not the next sweep's start, came below 2 or
// changed sign); the books keep the minimum of that margin in the device state.
// Otherwise the copy is restored and the sweeps run on the per-sublattice
// kernels, which apply the term phase by phase.

// Workspace layout: the spin buffer, the state, one record, and per step of
// the schedule the tables of fields h_num + an_num and h_num - an_num.
struct SpecLayout {
    uint64_t state, record, tables, total;
};

SpecLayout spec_layout(const isf_desc &d) {
    auto up = [](uint64_t v) { return (v + 255) / 256 * 256; };
    SpecLayout l;
    l.state = up(spin_bytes_of(&d));
    l.record = l.state + up(sizeof(DevState));
    l.tables = l.record + up(sizeof(isf_record));
    l.total = l.tables + up(sizeof(uint32_t) * 2 * kTableWords * ISF_MAX_STEPS);
    return l;
}

uint32_t *spec_tables(const isf_lattice *lat, uint32_t step, int32_t sgn) {
    return reinterpret_cast<uint32_t *>(lat->spec_ws + spec_layout(lat->d).tables) +
           ((size_t)step * 2 + (sgn > 0 ? 0 : 1)) * kTableWords;
}

// Upload the tables of fields h_num +- an_num of every step of the loaded
// anisotropic schedule (synchronous).
int32_t spec_upload(isf_lattice *lat) {
    const size_t n = lat->spec_steps.size();
    if (!lat->spec_ws || n == 0)
        return ISF_OK;
    std::vector<uint32_t> t(n * 2 * kTableWords);
    for (size_t i = 0; i < n; ++i) {
        const isf_step &st = lat->spec_steps[i];
        table_of(st.T, st.h_num + st.an_num, st.hs_num, &t[(2 * i) * kTableWords]);
        table_of(st.T, st.h_num - st.an_num, st.hs_num, &t[(2 * i + 1) * kTableWords]);
    }
    HIP_TRY(hipMemcpyAsync(spec_tables(lat, 0, 1), t.data(), t.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                           lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    return ISF_OK;
}

const Tiling kSpecFallback{64, 4, 2, ISF_KERNEL_TILES};

// The host's copy of the schedule position after n more sweeps.
void spec_advance_pos(isf_lattice *lat, uint64_t n) {
    while (n > 0 && lat->spec_step < lat->spec_steps.size()) {
        const uint32_t len = lat->spec_steps[lat->spec_step].n_sweeps;
        const uint64_t k = std::min<uint64_t>(n, len - lat->spec_sis);
        lat->spec_sis += (uint32_t)k;
        n -= k;
        if (lat->spec_sis == len) {
            ++lat->spec_step;
            lat->spec_sis = 0;
        }
    }
}

// The device state (into head, synchronously) and its M, the magnetisation at
// the host's copy of the schedule position.
int32_t spec_read(isf_lattice *lat, DevState *head) {
    int32_t rc = flush_whole(lat);
    if (rc)
        return rc;
    HIP_TRY(hipMemcpyAsync(head, lat->L.st, sizeof(DevState), hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    lat->spec_M = head->M;
    lat->spec_known = true;
    return ISF_OK;
}

// The current step's thresholds into the device state, for the next run to
// start from: sgn = +1 / -1 the table of field h_num + / - an_num (workspace),
// 0 the step's own table and its anisotropy halves.
int32_t spec_set_tables(isf_lattice *lat, int32_t sgn) {
    uint8_t *cur = lat->aux_dev + offsetof(DevState, cur_table);
    const uint32_t s = lat->spec_step;
    if (sgn) {
        HIP_TRY(hipMemcpyAsync(cur, spec_tables(lat, s, sgn), sizeof(uint32_t) * kTableWords,
                               hipMemcpyDeviceToDevice, lat->stream));
    } else {
        HIP_TRY(hipMemcpyAsync(cur, lat->L.tables + (size_t)s * kTableWords, sizeof(uint32_t) * kTableWords,
                               hipMemcpyDeviceToDevice, lat->stream));
        HIP_TRY(hipMemcpyAsync(lat->aux_dev + offsetof(DevState, cur_atable), lat->L.atables + (size_t)s * kAnWords,
                               sizeof(uint32_t) * kAnWords, hipMemcpyDeviceToDevice, lat->stream));
    }
    return ISF_OK;
}

// k sweeps on the per-sublattice kernels, the term applied phase by phase.
int32_t spec_fallback(isf_lattice *lat, uint64_t k) {
    int32_t rc;
    if ((rc = settle(lat)) || (rc = spec_set_tables(lat, 0)))
        return rc;
    const Tiling keep = lat->tiling;
    lat->tiling = kSpecFallback;
    rc = enqueue_sweeps_plain(lat, k);
    lat->tiling = keep;
    lat->spec_known = false;
    return rc;
}

// k sweeps of the current step on the whole-sweep kernel, with the table of
// field h_num + sgn an_num (sgn = 0: the step's own).
int32_t spec_whole(isf_lattice *lat, int32_t sgn, uint64_t k) {
    int32_t rc;
    if ((rc = flush_whole(lat)) || (rc = spec_set_tables(lat, sgn)) || (rc = enqueue_sweeps(lat, k)))
        return rc;
    return flush_whole(lat);
}

// k sweeps of the current step with the anisotropy term, from |M0| >= 2.
int32_t spec_try(isf_lattice *lat, uint64_t k) {
    static const int64_t kNoMargin = INT64_MAX;
    const int64_t M0 = lat->spec_M;
    int32_t rc;
    if ((rc = flush_whole(lat)))
        return rc;
    const SpecLayout sl = spec_layout(lat->d);
    const bool was_spare = lat->cur_spare;
    uint8_t *cur = was_spare ? lat->spare : lat->L.spins;
    isf_record *rec = lat->L.records + lat->spec_step;
    HIP_TRY(hipMemcpyAsync(lat->spec_ws, cur, spin_bytes_of(&lat->d), hipMemcpyDeviceToDevice, lat->stream));
    HIP_TRY(hipMemcpyAsync(lat->spec_ws + sl.state, lat->L.st, sizeof(DevState), hipMemcpyDeviceToDevice,
                           lat->stream));
    HIP_TRY(hipMemcpyAsync(lat->spec_ws + sl.record, rec, sizeof(isf_record), hipMemcpyDeviceToDevice, lat->stream));
    HIP_TRY(hipMemcpyAsync(lat->aux_dev + offsetof(DevState, spec_margin), &kNoMargin, sizeof kNoMargin,
                           hipMemcpyHostToDevice, lat->stream));
    if ((rc = spec_whole(lat, M0 > 0 ? 1 : -1, k)))
        return rc;
    DevState head;
    if ((rc = spec_read(lat, &head)))
        return rc;
    ++lat->spec_runs;
    if (head.spec_margin >= 2)
        return ISF_OK;
    // |M| may have come below 2 at some phase start: start again from the copy
    ++lat->spec_redone;
    uint8_t *back = was_spare ? lat->spare : lat->L.spins;
    HIP_TRY(hipMemcpyAsync(back, lat->spec_ws, spin_bytes_of(&lat->d), hipMemcpyDeviceToDevice, lat->stream));
    HIP_TRY(hipMemcpyAsync(lat->L.st, lat->spec_ws + sl.state, sizeof(DevState), hipMemcpyDeviceToDevice,
                           lat->stream));
    HIP_TRY(hipMemcpyAsync(rec, lat->spec_ws + sl.record, sizeof(isf_record), hipMemcpyDeviceToDevice, lat->stream));
    lat->cur_spare = was_spare;
    lat->spec_M = M0;
    return spec_fallback(lat, k);
}

// n sweeps of an anisotropic schedule with a whole-sweep tuning, step by step.
int32_t spec_advance(isf_lattice *lat, uint64_t n) {
    while (n > 0) {
        if (lat->spec_step >= lat->spec_steps.size())
            return fail(ISF_ESTATE, "schedule position beyond the loaded schedule");
        const isf_step &st = lat->spec_steps[lat->spec_step];
        const uint64_t k = std::min<uint64_t>(n, st.n_sweeps - lat->spec_sis);
        int32_t rc;
        if (st.an_num == 0) {
            rc = spec_whole(lat, 0, k);
            lat->spec_known = false;
        } else {
            DevState head;
            if (!lat->spec_known && (rc = spec_read(lat, &head)))
                return rc;
            rc = (lat->spec_M >= -1 && lat->spec_M <= 1) ? spec_fallback(lat, k) : spec_try(lat, k);
        }
        if (rc)
            return rc;
        spec_advance_pos(lat, k);
        n -= k;
    }
    return ISF_OK;
}

// Compact start layout: vacancies 1, occupied sites 0 (INT8) or occupancy bits (BITPACK).
void build_layout(const isf_desc &d, const uint8_t *h, std::vector<uint8_t> &buf) {
    const uint32_t X = d.X, Y = d.Y, Z = d.Z, W = X / 2;
    buf.assign(spin_bytes_of(&d), 0);
    if (d.format == ISF_FORMAT_INT8) {
        std::fill(buf.begin(), buf.end(), (uint8_t)1);
        for (uint32_t z = 0; z < Z; ++z)
            for (uint32_t y = 0; y < Y; ++y) {
                uint8_t *row = &buf[((size_t)(z + 1) * Y + y) * W];
                const uint32_t p = (y + z) & 1u;
                for (uint32_t j = 0; j < W; ++j)
                    if (z < h[(size_t)y * X + 2 * j + p])
                        row[j] = 0;
            }
    } else {
        const uint32_t nw = (W + 31) / 32;
        uint32_t *w = reinterpret_cast<uint32_t *>(buf.data());
        for (uint32_t z = 0; z < Z; ++z)
            for (uint32_t y = 0; y < Y; ++y) {
                uint32_t *occ = w + (((size_t)(z + 1) * Y + y) * 2 + 1) * nw;
                const uint32_t p = (y + z) & 1u;
                for (uint32_t j = 0; j < W; ++j)
                    if (z < h[(size_t)y * X + 2 * j + p])
                        occ[j >> 5] |= 1u << (j & 31);
            }
    }
}

int32_t recount(isf_lattice *lat, int64_t out[4]) {
    int64_t *dev = reinterpret_cast<int64_t *>(lat->aux_dev + offsetof(DevState, recount));
    HIP_TRY(hipMemsetAsync(dev, 0, 4 * sizeof(int64_t), lat->stream));
    hipError_t e = lat->d.format == ISF_FORMAT_INT8 ? launch_recount_i8(lat->L, dev, lat->stream)
                                                    : launch_recount_bp(lat->L, dev, lat->stream);
    if (e != hipSuccess)
        return fail(ISF_EHIP, "recount launch: %s", hipGetErrorString(e));
    HIP_TRY(hipMemcpyAsync(out, dev, 4 * sizeof(int64_t), hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    return ISF_OK;
}

// Write M, E, t and counts into the device state.
int32_t put_state(isf_lattice *lat, int64_t M, int64_t E, uint64_t t) {
    struct {
        int64_t M, E;
        uint64_t t;
    } head = {M, E, t};
    HIP_TRY(hipMemcpyAsync(lat->aux_dev + offsetof(DevState, M), &head, sizeof head, hipMemcpyHostToDevice,
                           lat->stream));
    int64_t counts[2] = {lat->n_occ, lat->n_bonds};
    HIP_TRY(hipMemcpyAsync(lat->aux_dev + offsetof(DevState, n_occ), counts, sizeof counts, hipMemcpyHostToDevice,
                           lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    return ISF_OK;
}

int32_t check_lat(const isf_lattice *lat) {
    if (!lat)
        return fail(ISF_EINVAL, "null lattice handle");
    return ISF_OK;
}

int32_t validate_steps(const isf_step *steps, uint32_t n) {
    if (n && !steps)
        return fail(ISF_EINVAL, "null steps");
    for (uint32_t i = 0; i < n; ++i) {
        int32_t rc = validate_T(steps[i].T);
        if (rc)
            return rc;
        rc = validate_h(steps[i].h_num);
        if (rc)
            return rc;
        if (steps[i].n_sweeps < 1)
            return fail(ISF_EINVAL, "step %u: n_sweeps must be >= 1", i);
        if (steps[i].n_discard > steps[i].n_sweeps)
            return fail(ISF_EINVAL, "step %u: n_discard > n_sweeps", i);
        if (steps[i].hs_num > 200000 || steps[i].hs_num < -200000)
            return fail(ISF_EINVAL, "step %u: |hs_num| = %d exceeds 200000", i, steps[i].hs_num);
        if (steps[i].an_num > 200000 || steps[i].an_num < 0)
            return fail(ISF_EINVAL, "step %u: an_num = %d outside [0, 200000]", i, steps[i].an_num);
    }
    return ISF_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

int32_t isf_abi_version(void) { return ISF_ABI_VERSION; }

const char *isf_last_error(void) { return g_err.c_str(); }

int32_t isf_lattice_bytes(const isf_desc *d, uint64_t *spin_bytes, uint64_t *aux_bytes) {
    int32_t rc = validate_desc(d);
    if (rc)
        return rc;
    if (!spin_bytes || !aux_bytes)
        return fail(ISF_EINVAL, "null output pointer");
    *spin_bytes = spin_bytes_of(d);
    *aux_bytes = aux_bytes_of(d);
    return ISF_OK;
}

int32_t isf_gate_threshold(double T, int32_t hs_num, uint32_t *out) {
    int32_t rc = validate_T(T);
    if (rc)
        return rc;
    if ((rc = validate_h(hs_num)))
        return rc;
    if (!out)
        return fail(ISF_EINVAL, "null output");
    *out = gate_threshold_of(hs_num, T);
    return ISF_OK;
}

int32_t isf_threshold_table(double T, int32_t h_num, uint32_t out[2][25]) {
    int32_t rc = validate_T(T);
    if (rc)
        return rc;
    if ((rc = validate_h(h_num)))
        return rc;
    if (!out)
        return fail(ISF_EINVAL, "null output");
    uint32_t tab[kTableWords];
    table_of(T, h_num, 0, tab);
    std::memcpy(out, tab, 50 * sizeof(uint32_t));
    return ISF_OK;
}

int32_t isf_lattice_create(const isf_desc *d, const uint8_t *h_host, int32_t init, void *spin_dev,
                           uint64_t spin_bytes, void *aux_dev, uint64_t aux_bytes, void *stream, isf_lattice **out) {
    int32_t rc = validate_desc(d);
    if (rc)
        return rc;
    if (!h_host || !spin_dev || !aux_dev || !out)
        return fail(ISF_EINVAL, "null pointer argument");
    if (init != ISF_INIT_UP && init != ISF_INIT_DOWN && init != ISF_INIT_RANDOM)
        return fail(ISF_EINVAL, "unknown init mode %d", init);
    const uint64_t need_spin = spin_bytes_of(d);
    const AuxLayout al = aux_layout(ISF_MAX_STEPS);
    if (spin_bytes < need_spin || aux_bytes < aux_bytes_of(d))
        return fail(ISF_ENOSPC, "buffers too small: need %llu + %llu bytes", (unsigned long long)need_spin,
                    (unsigned long long)aux_bytes_of(d));
    if (((uintptr_t)spin_dev & 255) || ((uintptr_t)aux_dev & 255))
        return fail(ISF_EINVAL, "device buffers must be 256-byte aligned");
    for (uint64_t i = 0, n = (uint64_t)d->X * d->Y; i < n; ++i)
        if (h_host[i] > d->Z)
            return fail(ISF_EINVAL, "height map value %u at %llu exceeds Z=%u", h_host[i], (unsigned long long)i, d->Z);

    isf_lattice *lat = new (std::nothrow) isf_lattice();
    if (!lat)
        return fail(ISF_EINVAL, "out of host memory");
    lat->d = *d;
    lat->aux = al;
    lat->aux_dev = static_cast<uint8_t *>(aux_dev);
    lat->stream = static_cast<hipStream_t>(stream);
    lat->tiling = Tiling{64, 4, 2, ISF_KERNEL_TILES};
    lat->use_graph = true;
    int n_cu = 0;
    if (hipGetDevice(&lat->device) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, lat->device) != hipSuccess) {
        delete lat;
        return fail(ISF_EHIP, "hipGetDevice failed");
    }
    lat->n_cu = (uint32_t)std::max(n_cu, 1);
    LatDev &L = lat->L;
    L.spins = static_cast<uint8_t *>(spin_dev);
    lat->spare = d->format == ISF_FORMAT_INT8 ? lat->aux_dev + spare_offset() : nullptr;
    lat->lists = d->format == ISF_FORMAT_INT8 ? lat->aux_dev + lists_offset(d) : nullptr;
    L.st = reinterpret_cast<DevState *>(lat->aux_dev + al.off_state);
    L.slots = reinterpret_cast<Slot *>(lat->aux_dev + al.off_slots);
    L.steps = reinterpret_cast<StepDesc *>(lat->aux_dev + al.off_steps);
    L.tables = reinterpret_cast<uint32_t *>(lat->aux_dev + al.off_tables);
    L.atables = reinterpret_cast<uint32_t *>(lat->aux_dev + al.off_atables);
    L.records = reinterpret_cast<isf_record *>(lat->aux_dev + al.off_records);
    L.pos = reinterpret_cast<SweepPos *>(lat->aux_dev + al.off_pos);
    L.slots2 = reinterpret_cast<Slot *>(lat->aux_dev + al.off_slots2);
    L.X = d->X;
    L.Y = d->Y;
    L.Z = d->Z;
    L.W = d->X / 2;
    L.nd = d->format == ISF_FORMAT_INT8 ? L.W / 4 : (L.W + 31) / 32;
    L.key0 = (uint32_t)d->seed;
    L.key1 = (uint32_t)(d->seed >> 32);
    L.replica = d->replica;
    L.format = d->format;

    auto bail = [&](int32_t code) {
        delete lat;
        return code;
    };
    std::vector<uint8_t> buf;
    build_layout(*d, h_host, buf);
    if (hipMemsetAsync(aux_dev, 0, al.total, lat->stream) != hipSuccess ||
        hipMemcpyAsync(spin_dev, buf.data(), buf.size(), hipMemcpyHostToDevice, lat->stream) != hipSuccess)
        return bail(fail(ISF_EHIP, "initial upload failed"));
    hipError_t e = d->format == ISF_FORMAT_INT8 ? launch_init_i8(L, init, lat->stream)
                                                : launch_init_bp(L, init, lat->stream);
    if (e != hipSuccess)
        return bail(fail(ISF_EHIP, "init launch: %s", hipGetErrorString(e)));
    int64_t cnt[4];
    if ((rc = recount(lat, cnt)))
        return bail(rc);
    lat->n_occ = cnt[2];
    lat->n_bonds = cnt[3] / 2;
    if ((rc = put_state(lat, cnt[0], -cnt[1] / 2, 0)))
        return bail(rc);
    *out = lat;
    return ISF_OK;
}

int32_t isf_lattice_destroy(isf_lattice *lat) {
    if (!lat)
        return fail(ISF_EINVAL, "null lattice handle");
    drop_graph(lat);
    delete lat;
    return ISF_OK;
}

int32_t isf_aniso_workspace_bytes(const isf_lattice *lat, uint64_t *bytes) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (!bytes)
        return fail(ISF_EINVAL, "null output");
    if (lat->d.format != ISF_FORMAT_INT8)
        return fail(ISF_EINVAL, "the anisotropy term needs an INT8 film");
    *bytes = spec_layout(lat->d).total;
    return ISF_OK;
}

int32_t isf_attach_aniso_workspace(isf_lattice *lat, void *dev, uint64_t bytes) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (lat->d.format != ISF_FORMAT_INT8)
        return fail(ISF_EINVAL, "the anisotropy term needs an INT8 film");
    if (!dev)
        return fail(ISF_EINVAL, "null workspace");
    if ((uintptr_t)dev & 255)
        return fail(ISF_EINVAL, "workspace must be 256-byte aligned");
    const uint64_t need = spec_layout(lat->d).total;
    if (bytes < need)
        return fail(ISF_ENOSPC, "workspace of %llu bytes < %llu", (unsigned long long)bytes,
                    (unsigned long long)need);
    if ((rc = set_device_of(lat)))
        return rc;
    lat->spec_ws = static_cast<uint8_t *>(dev);
    lat->spec_bytes = bytes;
    lat->spec_runs = 0;
    lat->spec_redone = 0;
    return spec_upload(lat);  // the loaded schedule's tables, if it has the term
}

int32_t isf_aniso_stats(const isf_lattice *lat, uint64_t *speculated, uint64_t *redone) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (!speculated || !redone)
        return fail(ISF_EINVAL, "null output");
    *speculated = lat->spec_runs;
    *redone = lat->spec_redone;
    return ISF_OK;
}

int32_t isf_set_tuning(isf_lattice *lat, const isf_tuning *t) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (!t)
        return fail(ISF_EINVAL, "null tuning");
    Tiling tl{t->tile_x, t->tile_y, t->rows_per_thread, t->kernel};
    if (tl.kernel == ISF_KERNEL_LIST) {
        if (lat->d.format != ISF_FORMAT_INT8 || !lat->items_attached)
            return fail(ISF_ESTATE, "the list kernel needs an INT8 film with occupied-dword lists attached");
        if (tl.ry != 1 && tl.ry != 2)
            return fail(ISF_EINVAL, "list kernel: %u entries per thread (1 or 2)", tl.ry);
    } else if (tl.kernel == ISF_KERNEL_SWEEP) {
        if (lat->d.format != ISF_FORMAT_INT8 || !lat->spare)
            return fail(ISF_EINVAL, "the whole-sweep kernel needs an INT8 film");
        const uint32_t lds = halo_lds_bytes(tl.tx, tl.ty, lat->d.Z);
        if (lds == 0 || (tl.ry != 4 && tl.ry != 8 && tl.ry != 16))
            return fail(ISF_EINVAL, "unsupported whole-sweep shape %ux%u with %u waves", tl.tx, tl.ty, tl.ry);
        int max_lds = 0;
        HIP_TRY(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, lat->device));
        if (lds > (uint32_t)max_lds - 1024u || halo_region_dwords(tl.tx, tl.ty, lat->d.Z) > 65536u)
            return fail(ISF_EINVAL, "whole-sweep shape %ux%u needs %u bytes of LDS for Z = %u (limit %d)", tl.tx,
                        tl.ty, lds, lat->d.Z, max_lds);
    } else if (tl.kernel == ISF_KERNEL_PIPE) {
        if (lat->d.format != ISF_FORMAT_INT8 || !lat->spare)
            return fail(ISF_EINVAL, "the pipelined whole-sweep kernel needs an INT8 film");
        int32_t rc = pipe_fits(lat, tl, lat->d.Z, false);
        if (rc)
            return rc;
    } else if (tl.kernel == ISF_KERNEL_FILM) {
        if (lat->d.format != ISF_FORMAT_INT8)
            return fail(ISF_EINVAL, "the film kernel needs an INT8 film");
        if (tl.tx != 512 || tl.ty != 1 || tl.ry != 1)
            return fail(ISF_EINVAL, "film kernel: tile_x 512, tile_y 1, rows_per_thread 1");
        int max_lds = 0;
        HIP_TRY(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, lat->device));
        if (!film_lds_bytes(lat->d.Y, lat->d.Z, lat->L.nd, (uint32_t)max_lds))
            return fail(ISF_EINVAL, "film of %u x %u x %u does not fit one block's LDS", lat->d.X, lat->d.Y,
                        lat->d.Z);
        if (lat->aniso)
            return fail(ISF_EINVAL, "the loaded schedule has the anisotropy term, which the film kernel does not take");
    } else if (tl.kernel != ISF_KERNEL_TILES) {
        return fail(ISF_EINVAL, "unknown kernel %u", tl.kernel);
    } else {
        const bool ok = lat->d.format == ISF_FORMAT_INT8 ? tiling_supported(tl) : tiling_supported_bp(tl);
        if (!ok)
            return fail(ISF_EINVAL, "unsupported tiling %ux%ux%u", tl.tx, tl.ty, tl.ry);
    }
    if (lat->aniso && is_whole(tl.kernel) && !lat->spec_ws)
        return fail(ISF_EINVAL,
                    "the loaded schedule has the anisotropy term, which needs the per-sublattice kernels or a "
                    "workspace for the whole-sweep kernels (isf_attach_aniso_workspace)");
    lat->tiling = tl;
    lat->use_graph = t->use_graph != 0;
    return ISF_OK;
}

int32_t isf_get_tuning(const isf_lattice *lat, isf_tuning *t) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (!t)
        return fail(ISF_EINVAL, "null tuning");
    t->tile_x = lat->tiling.tx;
    t->tile_y = lat->tiling.ty;
    t->rows_per_thread = lat->tiling.ry;
    t->use_graph = lat->use_graph;
    t->kernel = lat->tiling.kernel;
    return ISF_OK;
}

namespace {
uint32_t bits_for(uint32_t v) {  // bits needed to hold values 0..v
    uint32_t b = 0;
    while (b < 32 && (v >> b))
        ++b;
    return b;
}

// Occupied-dword lists of the four sublattices from the device spins.
int32_t build_items(isf_lattice *lat, std::vector<uint32_t> &items, uint32_t n[4], uint32_t &ybits,
                    uint32_t &dbits) {
    const isf_desc &d = lat->d;
    if (d.format != ISF_FORMAT_INT8)
        return fail(ISF_ESTATE, "occupied-dword lists exist for INT8 films only");
    const uint32_t Y = d.Y, Z = d.Z, nd = d.X / 8;
    const uint32_t zbits = bits_for(Z - 1);
    ybits = bits_for(Y - 1);
    dbits = bits_for(nd - 1);
    if (zbits + ybits + dbits > 32)
        return fail(ISF_EINVAL, "film coordinates need %u bits, more than a 32-bit list entry",
                    zbits + ybits + dbits);
    std::vector<uint32_t> buf((size_t)(Z + 2) * Y * nd);
    HIP_TRY(hipMemcpyAsync(buf.data(), lat->L.spins, buf.size() * 4, hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    items.clear();
    for (uint32_t s = 0; s < 4; ++s) {
        const size_t before = items.size();
        for (uint32_t z = s >> 1; z < Z; z += 2)
            for (uint32_t y = s & 1u; y < Y; y += 2) {
                const uint32_t *row = &buf[((size_t)(z + 1) * Y + y) * nd];
                for (uint32_t j = 0; j < nd; ++j)
                    if (row[j] != 0x01010101u)
                        items.push_back((((z << ybits) | y) << dbits) | j);
            }
        n[s] = (uint32_t)(items.size() - before);
    }
    return ISF_OK;
}
}  // namespace

int32_t isf_items_bytes(const isf_lattice *lat, uint64_t *bytes) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (!bytes)
        return fail(ISF_EINVAL, "null output");
    isf_lattice *l = const_cast<isf_lattice *>(lat);
    if ((rc = set_device_of(l)))
        return rc;
    std::vector<uint32_t> items;
    uint32_t n[4], yb, db;
    if ((rc = build_items(l, items, n, yb, db)))
        return rc;
    *bytes = std::max<uint64_t>(256, (uint64_t)items.size() * 4);
    return ISF_OK;
}

int32_t isf_attach_items(isf_lattice *lat, void *dev, uint64_t bytes) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (!dev)
        return fail(ISF_EINVAL, "null items buffer");
    if ((uintptr_t)dev & 255)
        return fail(ISF_EINVAL, "items buffer must be 256-byte aligned");
    if ((rc = set_device_of(lat)))
        return rc;
    std::vector<uint32_t> items;
    uint32_t n[4], yb, db;
    if ((rc = build_items(lat, items, n, yb, db)))
        return rc;
    if (bytes < (uint64_t)items.size() * 4)
        return fail(ISF_ENOSPC, "items buffer of %llu bytes < %llu", (unsigned long long)bytes,
                    (unsigned long long)items.size() * 4);
    if (!items.empty())
        HIP_TRY(hipMemcpyAsync(dev, items.data(), items.size() * 4, hipMemcpyHostToDevice, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    LatDev &L = lat->L;
    L.items = static_cast<const uint32_t *>(dev);
    uint32_t off = 0;
    for (int s = 0; s < 4; ++s) {
        L.n_items[s] = n[s];
        L.items_off[s] = off;
        off += n[s];
    }
    L.ybits = yb;
    L.dbits = db;
    lat->items_attached = true;
    lat->tiling = Tiling{lat->tiling.tx, lat->tiling.ty, 1, ISF_KERNEL_LIST};
    drop_graph(lat);
    return ISF_OK;
}

int32_t isf_schedule_load(isf_lattice *lat, const isf_step *steps, uint32_t n) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (n > ISF_MAX_STEPS)
        return fail(ISF_EINVAL, "schedule of %u steps exceeds %u", n, (unsigned)ISF_MAX_STEPS);
    if ((rc = validate_steps(steps, n)))
        return rc;
    if ((rc = set_device_of(lat)))
        return rc;
    if ((rc = flush_whole(lat)))
        return rc;
    std::vector<StepDesc> sd(n ? n : 1);
    std::vector<uint32_t> tabs((size_t)(n ? n : 1) * kTableWords, 0);
    bool aniso = false;
    uint64_t total = 0;
    for (uint32_t i = 0; i < n; ++i) {
        sd[i] = StepDesc{steps[i].n_sweeps, steps[i].n_discard};
        if (steps[i].an_num != 0) {
            if (lat->d.format != ISF_FORMAT_INT8)
                return fail(ISF_EINVAL, "step %u: the anisotropy term needs an INT8 film", i);
            if ((is_whole(lat->tiling.kernel) && !lat->spec_ws) || lat->tiling.kernel == ISF_KERNEL_FILM)
                return fail(ISF_EINVAL,
                            "step %u: the anisotropy term needs the per-sublattice kernels (tuning kernel TILES "
                            "or LIST), or a workspace for the whole-sweep kernels (isf_attach_aniso_workspace)",
                            i);
            aniso = true;
        }
        table_of(steps[i].T, steps[i].h_num, steps[i].hs_num, &tabs[(size_t)i * kTableWords]);
        total += steps[i].n_sweeps;
    }
    std::vector<uint32_t> atabs;
    if (aniso) {
        atabs.assign((size_t)n * kAnWords, 0);
        for (uint32_t i = 0; i < n; ++i)
            aniso_table_of(steps[i].T, steps[i].h_num, steps[i].an_num, &atabs[(size_t)i * kAnWords]);
    }
    struct {
        uint32_t step, sweep_in_step;
        int64_t sum_M, sum_absM, sum_E, accepted;
        uint32_t reserved0, n_steps;
    } mid = {0, 0, 0, 0, 0, 0, 0, n};
    static_assert(offsetof(DevState, n_steps) + 4 - offsetof(DevState, step) == sizeof(mid), "state layout");
    if (n) {
        HIP_TRY(hipMemcpyAsync(lat->L.steps, sd.data(), sizeof(StepDesc) * n, hipMemcpyHostToDevice, lat->stream));
        HIP_TRY(hipMemcpyAsync(lat->L.tables, tabs.data(), sizeof(uint32_t) * kTableWords * n,
                               hipMemcpyHostToDevice, lat->stream));
        HIP_TRY(hipMemcpyAsync(lat->aux_dev + offsetof(DevState, cur_table), tabs.data(),
                               sizeof(uint32_t) * kTableWords, hipMemcpyHostToDevice, lat->stream));
        if (aniso) {
            HIP_TRY(hipMemcpyAsync(lat->L.atables, atabs.data(), sizeof(uint32_t) * kAnWords * n,
                                   hipMemcpyHostToDevice, lat->stream));
            HIP_TRY(hipMemcpyAsync(lat->aux_dev + offsetof(DevState, cur_atable), atabs.data(),
                                   sizeof(uint32_t) * kAnWords, hipMemcpyHostToDevice, lat->stream));
        }
    }
    HIP_TRY(hipMemcpyAsync(lat->aux_dev + offsetof(DevState, step), &mid, sizeof mid, hipMemcpyHostToDevice,
                           lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    if (aniso != lat->aniso)
        drop_graph(lat);  // a cached graph holds the launches' copy of L.aniso
    lat->aniso = aniso;
    lat->L.aniso = aniso ? 1u : 0u;
    if (aniso)
        lat->spec_steps.assign(steps, steps + n);
    else
        lat->spec_steps.clear();
    lat->spec_step = 0;
    lat->spec_sis = 0;
    lat->spec_known = false;
    if ((rc = spec_upload(lat)))
        return rc;
    lat->sched_steps = n;
    lat->sched_total = total;
    lat->sched_enqueued = 0;
    return ISF_OK;
}

int32_t isf_schedule_remaining(const isf_lattice *lat, uint64_t *sweeps) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (!sweeps)
        return fail(ISF_EINVAL, "null output");
    *sweeps = lat->sched_total - lat->sched_enqueued;
    return ISF_OK;
}

int32_t isf_advance(isf_lattice *lat, uint32_t max_sweeps, uint64_t *enqueued) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if ((rc = set_device_of(lat)))
        return rc;
    const uint64_t n = std::min<uint64_t>(max_sweeps, lat->sched_total - lat->sched_enqueued);
    if (lat->aniso && is_whole(lat->tiling.kernel)) {
        if ((rc = prepare_spare(lat, lat->tiling)) || (rc = spec_advance(lat, n)))
            return rc;
    } else {
        if ((rc = enqueue_sweeps(lat, n)))
            return rc;
        if (lat->aniso) {  // keep the host's copy of the position for a later whole-sweep tuning
            spec_advance_pos(lat, n);
            lat->spec_known = false;
        }
    }
    lat->sched_enqueued += n;
    if (enqueued)
        *enqueued = n;
    return ISF_OK;
}

int32_t isf_schedule_records(isf_lattice *lat, isf_record *out, uint32_t n) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (n > lat->sched_steps)
        return fail(ISF_EINVAL, "asked for %u records of a %u-step schedule", n, lat->sched_steps);
    if (n && !out)
        return fail(ISF_EINVAL, "null output");
    if ((rc = set_device_of(lat)))
        return rc;
    if ((rc = flush_whole(lat)))
        return rc;
    if (n)
        HIP_TRY(hipMemcpyAsync(out, lat->L.records, sizeof(isf_record) * n, hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    return ISF_OK;
}

int32_t isf_run_schedule(isf_lattice *lat, const isf_step *steps, uint32_t n_steps, isf_record *out) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (n_steps && !out)
        return fail(ISF_EINVAL, "null output");
    if ((rc = validate_steps(steps, n_steps)))
        return rc;
    for (uint32_t base = 0; base < n_steps; base += ISF_MAX_STEPS) {
        const uint32_t n = std::min<uint32_t>(ISF_MAX_STEPS, n_steps - base);
        if ((rc = isf_schedule_load(lat, steps + base, n)))
            return rc;
        uint64_t done = 0;
        if ((rc = isf_advance(lat, 0xFFFFFFFFu, &done)))
            return rc;
        if ((rc = isf_schedule_records(lat, out + base, n)))
            return rc;
    }
    return ISF_OK;
}

int32_t isf_read_observables(isf_lattice *lat, isf_obs *out) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (!out)
        return fail(ISF_EINVAL, "null output");
    if ((rc = set_device_of(lat)))
        return rc;
    if ((rc = flush_whole(lat)))
        return rc;
    struct {
        int64_t M, E;
        uint64_t t;
    } head;
    HIP_TRY(hipMemcpyAsync(&head, lat->aux_dev, sizeof head, hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    out->M = head.M;
    out->E = head.E;
    out->n_occ = lat->n_occ;
    out->n_bonds = lat->n_bonds;
    out->sweeps = head.t;
    return ISF_OK;
}

int32_t isf_run_sweeps(isf_lattice *lat, double T, int32_t h_num, uint32_t n_sweeps, uint32_t n_discard,
                       isf_record *out) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (!out)
        return fail(ISF_EINVAL, "null output");
    if ((rc = validate_T(T)) || (rc = validate_h(h_num)))
        return rc;
    if (n_discard > n_sweeps)
        return fail(ISF_EINVAL, "n_discard > n_sweeps");
    if (n_sweeps == 0) {
        isf_obs o;
        if ((rc = isf_read_observables(lat, &o)))
            return rc;
        *out = isf_record{o.M, o.E, 0, 0, 0, 0};
        return ISF_OK;
    }
    isf_step st{T, h_num, n_sweeps, n_discard, 0};
    return isf_run_schedule(lat, &st, 1, out);
}

int32_t isf_ramp_field(isf_lattice *lat, double T, const int32_t *h_num, uint32_t n_steps, uint32_t sweeps_per_step,
                       isf_record *out) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (n_steps && (!h_num || !out))
        return fail(ISF_EINVAL, "null pointer argument");
    if (sweeps_per_step < 1)
        return fail(ISF_EINVAL, "sweeps_per_step must be >= 1");
    std::vector<isf_step> st(n_steps);
    for (uint32_t i = 0; i < n_steps; ++i)
        st[i] = isf_step{T, h_num[i], sweeps_per_step, 0, 0};
    return isf_run_schedule(lat, st.data(), n_steps, out);
}

int32_t isf_temperature_scan(isf_lattice *lat, const double *T, uint32_t n_T, int32_t h_num, uint32_t sweeps_per_T,
                             uint32_t discard_per_T, isf_record *out) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (n_T && (!T || !out))
        return fail(ISF_EINVAL, "null pointer argument");
    std::vector<isf_step> st(n_T);
    for (uint32_t i = 0; i < n_T; ++i)
        st[i] = isf_step{T[i], h_num, sweeps_per_T, discard_per_T, 0};
    return isf_run_schedule(lat, st.data(), n_T, out);
}

int32_t isf_read_spins(isf_lattice *lat, int8_t *cube) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (!cube)
        return fail(ISF_EINVAL, "null output");
    if ((rc = set_device_of(lat)))
        return rc;
    if ((rc = settle(lat)))
        return rc;
    const isf_desc &d = lat->d;
    std::vector<uint8_t> buf(spin_bytes_of(&d));
    HIP_TRY(hipMemcpyAsync(buf.data(), lat->L.spins, buf.size(), hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    const uint32_t X = d.X, Y = d.Y, Z = d.Z, W = X / 2;
    std::memset(cube, 0, (size_t)X * Y * Z);
    for (uint32_t z = 0; z < Z; ++z)
        for (uint32_t y = 0; y < Y; ++y) {
            const uint32_t p = (y + z) & 1u;
            int8_t *out = cube + ((size_t)z * Y + y) * X;
            if (d.format == ISF_FORMAT_INT8) {
                const uint8_t *row = &buf[((size_t)(z + 1) * Y + y) * W];
                for (uint32_t j = 0; j < W; ++j)
                    out[2 * j + p] = row[j] == 1 ? 0 : (int8_t)((int)row[j] - 1);
            } else {
                const uint32_t nw = (W + 31) / 32;
                const uint32_t *w = reinterpret_cast<const uint32_t *>(buf.data()) + ((size_t)(z + 1) * Y + y) * 2 * nw;
                for (uint32_t j = 0; j < W; ++j) {
                    const uint32_t up = (w[j >> 5] >> (j & 31)) & 1u, oc = (w[nw + (j >> 5)] >> (j & 31)) & 1u;
                    out[2 * j + p] = oc ? (up ? 1 : -1) : 0;
                }
            }
        }
    return ISF_OK;
}

int32_t isf_write_spins(isf_lattice *lat, const int8_t *cube, uint64_t sweeps) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (!cube)
        return fail(ISF_EINVAL, "null input");
    if ((rc = set_device_of(lat)))
        return rc;
    if ((rc = settle(lat)))
        return rc;
    const isf_desc &d = lat->d;
    std::vector<uint8_t> buf(spin_bytes_of(&d));
    HIP_TRY(hipMemcpyAsync(buf.data(), lat->L.spins, buf.size(), hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    const uint32_t X = d.X, Y = d.Y, Z = d.Z, W = X / 2;
    for (uint32_t z = 0; z < Z; ++z)
        for (uint32_t y = 0; y < Y; ++y) {
            const uint32_t p = (y + z) & 1u;
            const int8_t *in = cube + ((size_t)z * Y + y) * X;
            if (d.format == ISF_FORMAT_INT8) {
                uint8_t *row = &buf[((size_t)(z + 1) * Y + y) * W];
                for (uint32_t j = 0; j < W; ++j) {
                    if (row[j] == 1)
                        continue;  // vacancy
                    const int8_t s = in[2 * j + p];
                    if (s != 1 && s != -1)
                        return fail(ISF_EINVAL, "occupied site (%u,%u,%u) holds %d, not +-1", 2 * j + p, y, z, s);
                    row[j] = (uint8_t)(s + 1);
                }
            } else {
                const uint32_t nw = (W + 31) / 32;
                uint32_t *w = reinterpret_cast<uint32_t *>(buf.data()) + ((size_t)(z + 1) * Y + y) * 2 * nw;
                for (uint32_t j = 0; j < W; ++j) {
                    if (!((w[nw + (j >> 5)] >> (j & 31)) & 1u))
                        continue;
                    const int8_t s = in[2 * j + p];
                    if (s != 1 && s != -1)
                        return fail(ISF_EINVAL, "occupied site (%u,%u,%u) holds %d, not +-1", 2 * j + p, y, z, s);
                    if (s > 0)
                        w[j >> 5] |= 1u << (j & 31);
                    else
                        w[j >> 5] &= ~(1u << (j & 31));
                }
            }
        }
    HIP_TRY(hipMemcpyAsync(lat->L.spins, buf.data(), buf.size(), hipMemcpyHostToDevice, lat->stream));
    int64_t cnt[4];
    if ((rc = recount(lat, cnt)))
        return rc;
    return put_state(lat, cnt[0], -cnt[1] / 2, sweeps);
}

int32_t isf_time_launches(isf_lattice *lat, uint32_t n_sweeps, double ms[4], uint32_t *swept) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (!ms || !swept)
        return fail(ISF_EINVAL, "null output");
    if ((rc = set_device_of(lat)))
        return rc;
    if (lat->aniso && is_whole(lat->tiling.kernel))
        return fail(ISF_EINVAL, "launch timing of an anisotropic schedule on a whole-sweep kernel is not supported");
    if (lat->tiling.kernel == ISF_KERNEL_FILM)
        return fail(ISF_EINVAL, "the film kernel runs many sweeps per launch: no launch timing");
    const uint32_t n = (uint32_t)std::min<uint64_t>(n_sweeps, lat->sched_total - lat->sched_enqueued);
    // timing-only events: no system-scope fence when they are recorded, so that
    // the pairs measure the launch between them and not a cache write-back
    std::vector<hipEvent_t> ev(8 * (size_t)n);
    for (auto &e : ev)
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    int32_t status = ISF_OK;
    const bool whole = is_whole(lat->tiling.kernel);
    if (books_in_launch(lat) ? ((whole && (rc = prepare_spare(lat, lat->tiling))) || (rc = prime_whole(lat)))
                             : (rc = settle(lat)) != 0) {
        for (auto &e : ev)
            (void)hipEventDestroy(e);
        return rc;
    }
    const uint32_t n_launch = whole ? 1 : 4;  // event pairs per sweep
    for (uint32_t i = 0; i < n && status == ISF_OK; ++i) {
        for (uint32_t s = 0; s < n_launch && status == ISF_OK; ++s) {
            (void)hipEventRecord(ev[8 * i + 2 * s], lat->stream);
            status = whole ? launch_whole_sweep(lat) : launch_phase(lat, s);
            (void)hipEventRecord(ev[8 * i + 2 * s + 1], lat->stream);
        }
        if (status == ISF_OK && !whole)
            status = launch_end(lat);
    }
    double sum[4] = {0, 0, 0, 0};
    if (status == ISF_OK) {
        lat->sched_enqueued += n;
        if (hipStreamSynchronize(lat->stream) != hipSuccess)
            status = fail(ISF_EHIP, "stream synchronisation failed");
        for (uint32_t i = 0; i < n && status == ISF_OK; ++i)
            for (uint32_t s = 0; s < n_launch; ++s) {
                float m = 0.f;
                if (hipEventElapsedTime(&m, ev[8 * i + 2 * s], ev[8 * i + 2 * s + 1]) != hipSuccess) {
                    status = fail(ISF_EHIP, "hipEventElapsedTime failed");
                    break;
                }
                sum[s] += m;
            }
    }
    for (auto &e : ev)
        (void)hipEventDestroy(e);
    if (status)
        return status;
    for (int s = 0; s < 4; ++s)
        ms[s] = n ? sum[s] / n : 0.0;
    *swept = n;
    return ISF_OK;
}

int32_t isf_surface_image(isf_lattice *lat, int8_t *img_dev, uint64_t bytes) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (!img_dev)
        return fail(ISF_EINVAL, "null image buffer");
    if (bytes < (uint64_t)lat->d.X * lat->d.Y)
        return fail(ISF_ENOSPC, "image buffer of %llu bytes < X * Y = %llu", (unsigned long long)bytes,
                    (unsigned long long)lat->d.X * lat->d.Y);
    if ((rc = set_device_of(lat)))
        return rc;
    // the spins of the last enqueued sweep, whichever copy holds them
    const uint8_t *cur = lat->cur_spare ? lat->spare : lat->L.spins;
    hipError_t e = launch_surface_image(lat->L, cur, img_dev, lat->stream);
    if (e != hipSuccess)
        return fail(ISF_EHIP, "surface image launch: %s", hipGetErrorString(e));
    return ISF_OK;
}

int32_t isf_draw_xor(isf_lattice *lat, uint32_t t0, uint32_t n_sweeps, uint32_t *xor_dev, float *ms) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (!xor_dev || n_sweeps == 0)
        return fail(ISF_EINVAL, "null checksum buffer or no sweeps");
    if ((rc = set_device_of(lat)))
        return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
    if (hipEventCreateWithFlags(&e1, hipEventDisableSystemFence) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(ISF_EHIP, "hipEventCreate failed");
    }
    (void)hipEventRecord(e0, lat->stream);
    hipError_t e = launch_draw_xor(lat->L, t0, n_sweeps, xor_dev, lat->n_cu, lat->stream);
    (void)hipEventRecord(e1, lat->stream);
    float m = 0.f;
    if (e == hipSuccess)
        e = hipStreamSynchronize(lat->stream);
    if (e == hipSuccess)
        e = hipEventElapsedTime(&m, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess)
        return fail(ISF_EHIP, "draw ceiling: %s", hipGetErrorString(e));
    if (ms)
        *ms = m;
    return ISF_OK;
}

int32_t isf_film_stats(const isf_lattice *lat, isf_stats *out) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (!out)
        return fail(ISF_EINVAL, "null output");
    out->n_occ = lat->n_occ;
    out->n_bonds = lat->n_bonds;
    out->mean_coordination = lat->n_occ ? 2.0 * (double)lat->n_bonds / (double)lat->n_occ : 0.0;
    out->p_c = out->mean_coordination > 0.0 ? 2.0 / out->mean_coordination : 0.0;
    out->concentration = (double)lat->n_occ / ((double)lat->d.X * lat->d.Y * lat->d.Z / 2.0);
    return ISF_OK;
}

int32_t isf_recount(isf_lattice *lat, int64_t *M, int64_t *E) {
    int32_t rc = check_lat(lat);
    if (rc)
        return rc;
    if (!M || !E)
        return fail(ISF_EINVAL, "null output");
    if ((rc = set_device_of(lat)))
        return rc;
    if ((rc = settle(lat)))
        return rc;
    int64_t cnt[4];
    if ((rc = recount(lat, cnt)))
        return rc;
    *M = cnt[0];
    *E = -cnt[1] / 2;
    return ISF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// recount without allocation

// The counters of isf_recount_films: four int64 per film (M, sum_i s_i n_i,
// occupied sites, occupied neighbours), at most ISF_RECOUNT_MAX_FILMS films.
// Each GPU the library runs on holds its own copy until the process ends.  In
// host code `scratch` names a host-side stand-in: the device address comes
// from hipGetSymbolAddress, per device, and only that address is used.
static __device__ __align__(256) int64_t scratch[4 * ISF_RECOUNT_MAX_FILMS];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
int64_t *g_scratch_dev[kScratchDevices];  // per device; null until its first call

// The device address of `scratch` on device `dev` (the current device).
int32_t scratch_on(int dev, int64_t **out) {
    if (dev < 0 || dev >= kScratchDevices)
        return fail(ISF_EINVAL, "device %d outside the %d devices the recount counters cover", dev,
                    kScratchDevices);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(ISF_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_dev[dev] = static_cast<int64_t *>(p);
    }
    *out = g_scratch_dev[dev];
    return ISF_OK;
}

// A fill kernel rather than hipMemsetAsync, so that the call could be captured.
__global__ void k_zero_counters(int64_t *p, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = 0;
}

}  // namespace

extern "C" {

int32_t isf_recount_films(const isf_desc *descs, const void *const *spins_dev, uint32_t n, void *stream,
                          int64_t *out) {
    if (n > ISF_RECOUNT_MAX_FILMS)
        return fail(ISF_ENOSPC, "%u films exceed the %u the recount counters hold", n,
                    (unsigned)ISF_RECOUNT_MAX_FILMS);
    if (n == 0)
        return ISF_OK;
    if (!descs || !spins_dev || !out)
        return fail(ISF_EINVAL, "null pointer argument");
    for (uint32_t i = 0; i < n; ++i) {
        int32_t rc = validate_desc(&descs[i]);
        if (rc)
            return rc;
        if (!spins_dev[i])
            return fail(ISF_EINVAL, "null spin buffer %u", i);
    }
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    int64_t *cnt = nullptr;
    int32_t rc = scratch_on(dev, &cnt);
    if (rc)
        return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_zero_counters, dim3((4 * n + 255) / 256), dim3(256), 0, s, cnt, 4 * n);
    HIP_TRY(hipGetLastError());
    for (uint32_t i = 0; i < n; ++i) {
        const isf_desc &d = descs[i];
        LatDev L{};
        L.spins = static_cast<uint8_t *>(const_cast<void *>(spins_dev[i]));
        L.X = d.X;
        L.Y = d.Y;
        L.Z = d.Z;
        L.W = d.X / 2;
        L.nd = d.format == ISF_FORMAT_INT8 ? L.W / 4 : (L.W + 31) / 32;
        L.format = d.format;
        const hipError_t e = d.format == ISF_FORMAT_INT8 ? launch_recount_i8(L, cnt + 4 * i, s)
                                                         : launch_recount_bp(L, cnt + 4 * i, s);
        if (e != hipSuccess)
            return fail(ISF_EHIP, "recount launch %u: %s", i, hipGetErrorString(e));
    }
    HIP_TRY(hipMemcpyAsync(out, cnt, sizeof(int64_t) * 4 * n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (uint32_t i = 0; i < n; ++i) {
        int64_t *o = out + 4 * i;
        o[1] = -o[1] / 2;  // E_bond = -(1/2) sum_i s_i n_i
        o[3] /= 2;         // each bond seen from both ends
    }
    return ISF_OK;
}

// ---------------------------------------------------------------------------
// batches

}  // extern "C"

namespace {

// Batch workspace on the device (and the same regions of the pinned host
// staging area): the sublattice launch table, the whole-sweep or pipelined
// launch table, the first block of every film of that table, then the
// persistent kernel's barrier words.
struct WsLayout {
    uint64_t phase, table, begins, barrier, total;
};
WsLayout ws_layout(uint32_t max_lats) {
    auto up = [](uint64_t v) { return (v + 255) / 256 * 256; };
    WsLayout w;
    w.phase = 0;
    w.table = up(sizeof(BatchEntry) * max_lats);
    w.begins = w.table + up(std::max(sizeof(WholeEntry), sizeof(PipeEntry)) * max_lats);
    w.barrier = w.begins + up(sizeof(uint32_t) * ((uint64_t)max_lats + 1));
    w.total = w.barrier + 256;
    return w;
}

}  // namespace

extern "C" {

int32_t isf_batch_workspace_bytes(uint32_t max_lats, uint64_t *bytes) {
    if (!bytes || max_lats == 0)
        return fail(ISF_EINVAL, "bad arguments");
    *bytes = ws_layout(max_lats).total;
    return ISF_OK;
}

int32_t isf_batch_create(uint32_t max_lats, void *ws, uint64_t ws_bytes, void *stream, isf_batch **out) {
    uint64_t need = 0;
    int32_t rc = isf_batch_workspace_bytes(max_lats, &need);
    if (rc)
        return rc;
    if (!ws || !out)
        return fail(ISF_EINVAL, "null pointer argument");
    if (ws_bytes < need)
        return fail(ISF_ENOSPC, "workspace of %llu bytes < %llu", (unsigned long long)ws_bytes,
                    (unsigned long long)need);
    if ((uintptr_t)ws & 255)
        return fail(ISF_EINVAL, "workspace must be 256-byte aligned");
    // the current device, made current explicitly: a batch may be the first
    // object a process creates, before anything else has touched the runtime
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipSetDevice(dev) != hipSuccess)
        return fail(ISF_EHIP, "no usable HIP device");
    isf_batch *b = new (std::nothrow) isf_batch();
    if (!b)
        return fail(ISF_EINVAL, "out of host memory");
    b->max_lats = max_lats;
    b->ws_dev = static_cast<uint8_t *>(ws);
    b->ws_bytes = ws_bytes;
    b->stream = static_cast<hipStream_t>(stream);
    if (hipHostMalloc(&b->staging, ws_layout(max_lats).barrier, hipHostMallocDefault) != hipSuccess) {
        delete b;
        return fail(ISF_EHIP, "hipHostMalloc of the staging area failed");
    }
    if (hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess) {
        (void)hipHostFree(b->staging);
        delete b;
        return fail(ISF_EHIP, "hipEventCreate failed");
    }
    *out = b;
    return ISF_OK;
}

int32_t isf_batch_destroy(isf_batch *b) {
    if (!b)
        return fail(ISF_EINVAL, "null batch");
    for (hipGraphExec_t g : b->graph)
        if (g)
            (void)hipGraphExecDestroy(g);
    (void)hipEventSynchronize(b->staged);
    (void)hipEventDestroy(b->staged);
    (void)hipHostFree(b->staging);
    delete b;
    return ISF_OK;
}

int32_t isf_batch_sync(isf_batch *b) {
    if (!b)
        return fail(ISF_EINVAL, "null batch");
    HIP_TRY(hipStreamSynchronize(b->stream));
    if (b->persistent_used) {
        uint32_t flag = 0;
        HIP_TRY(hipMemcpy(&flag, b->ws_dev + ws_layout(b->max_lats).barrier + sizeof(uint32_t), sizeof flag,
                          hipMemcpyDeviceToHost));
        if (flag)
            return fail(ISF_EHIP, "persistent kernel: grid barrier timed out; results are invalid");
    }
    return ISF_OK;
}

}  // extern "C"

namespace {

constexpr uint32_t kBatchGraphSweeps = 64;  // even: sweep parities alternate within a graph

// Enqueue `sweeps` sweeps of a batch's per-sweep launch sequence `one(g)` (g:
// the sweep's index in this call; launches that alternate with g & 1 need the
// even graph length): replays of a cached graph of kBatchGraphSweeps sweeps
// while that many remain, then plain launches.  The graph is captured again
// when the sequence (key) changes; the launch table it reads is uploaded on
// the stream before it, so a new table needs no new graph.
template <class F>
int32_t batch_enqueue(isf_batch *b, const uint64_t key[4], uint64_t sweeps, F one) {
    uint64_t g = 0;
    if (b->stream && sweeps >= kBatchGraphSweeps) {
        uint32_t slot = 2;
        for (uint32_t i = 0; i < 2; ++i)
            if (b->graph[i] && std::memcmp(b->graph_key[i], key, sizeof b->graph_key[i]) == 0)
                slot = i;
        if (slot == 2) {
            slot = b->graph_next;
            b->graph_next ^= 1u;
            if (b->graph[slot]) {
                (void)hipGraphExecDestroy(b->graph[slot]);
                b->graph[slot] = nullptr;
            }
            hipGraph_t gr = nullptr;
            HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            int32_t rc = ISF_OK;
            for (uint32_t i = 0; i < kBatchGraphSweeps && rc == ISF_OK; ++i)
                rc = one(i);
            const hipError_t e = hipStreamEndCapture(b->stream, &gr);
            if (rc) {
                if (gr)
                    (void)hipGraphDestroy(gr);
                return rc;
            }
            if (e != hipSuccess)
                return fail(ISF_EHIP, "batch graph capture: %s", hipGetErrorString(e));
            const hipError_t ei = hipGraphInstantiate(&b->graph[slot], gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            if (ei != hipSuccess) {
                b->graph[slot] = nullptr;
                return fail(ISF_EHIP, "batch graph instantiate: %s", hipGetErrorString(ei));
            }
            std::memcpy(b->graph_key[slot], key, sizeof b->graph_key[slot]);
        }
        for (; sweeps - g >= kBatchGraphSweeps; g += kBatchGraphSweeps)
            HIP_TRY(hipGraphLaunch(b->graph[slot], b->stream));
    }
    for (; g < sweeps; ++g) {
        int32_t rc = one((uint32_t)g);
        if (rc)
            return rc;
    }
    return ISF_OK;
}

uint64_t tiling_key(const Tiling &t) {
    return (uint64_t)t.tx | ((uint64_t)t.ty << 16) | ((uint64_t)t.ry << 32) | ((uint64_t)t.kernel << 48);
}

// Batched whole-sweep mode: one launch per sweep over the tiles of every film.
// The caller has waited for the staging area and records b->staged after.
int32_t batch_advance_whole(isf_batch *b, isf_lattice *const *lats, uint32_t n, uint32_t max_sweeps,
                            uint64_t *enqueued_out) {
    const Tiling tl = lats[0]->tiling.kernel == ISF_KERNEL_SWEEP ? lats[0]->tiling : Tiling{16, 16, 4, ISF_KERNEL_SWEEP};
    uint32_t Zmax = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (lats[i]->d.format != ISF_FORMAT_INT8 || !lats[i]->spare)
            return fail(ISF_EINVAL, "whole-sweep batches need INT8 lattices");
        Zmax = std::max(Zmax, lats[i]->d.Z);
    }
    const uint32_t lds = halo_lds_bytes(tl.tx, tl.ty, Zmax);
    int max_lds = 0;
    HIP_TRY(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, lats[0]->device));
    if (lds == 0 || lds > (uint32_t)max_lds - 4096u || halo_region_dwords(tl.tx, tl.ty, Zmax) > 65536u ||
        (tl.ry != 4 && tl.ry != 8 && tl.ry != 16))
        return fail(ISF_EINVAL, "whole-sweep shape %ux%u x %u waves does not fit films of %u planes", tl.tx, tl.ty,
                    tl.ry, Zmax);
    // each film: its spare copy and lists for the shape, and an open run of whole sweeps
    for (uint32_t i = 0; i < n; ++i) {
        isf_lattice *lat = lats[i];
        if (lat->sched_total == lat->sched_enqueued)
            continue;
        const bool ready = lat->spare_ready && lat->lists_ready && lat->lists_tiling.tx == tl.tx &&
                           lat->lists_tiling.ty == tl.ty && lat->lists_tiling.kernel == tl.kernel &&
                           lat->whole_active;
        if (ready)
            continue;
        int32_t rc;
        if ((rc = prepare_spare(lat, tl)) || (rc = prime_whole(lat)))
            return rc;
        HIP_TRY(hipStreamSynchronize(lat->stream));
    }
    const WsLayout wl = ws_layout(b->max_lats);
    WholeEntry *stage = reinterpret_cast<WholeEntry *>(static_cast<uint8_t *>(b->staging) + wl.table);
    uint32_t *stage_begins = reinterpret_cast<uint32_t *>(static_cast<uint8_t *>(b->staging) + wl.begins);
    uint64_t sweeps = 0;
    uint32_t m = 0, blocks = 0;
    for (uint32_t i = 0; i < n; ++i) {
        isf_lattice *lat = lats[i];
        const uint64_t rem = lat->sched_total - lat->sched_enqueued;
        if (rem == 0)
            continue;
        WholeEntry &e = stage[m++];
        e.lat = lat->L;
        e.spare = lat->spare;
        e.lists = lat->lists;
        e.block_begin = blocks;
        stage_begins[m - 1] = blocks;
        e.po = lat->cur_spare ? 1u : 0u;
        e.pad = 0;
        blocks += halo_tiles(tl.tx, tl.ty, lat->L.nd, lat->L.Y, e.nbx);
        sweeps = std::max<uint64_t>(sweeps, std::min<uint64_t>(rem, max_sweeps));
    }
    if (m == 0 || sweeps == 0) {
        if (enqueued_out)
            *enqueued_out = 0;
        return ISF_OK;
    }
    stage_begins[m] = blocks;
    WholeEntry *ents = reinterpret_cast<WholeEntry *>(b->ws_dev + wl.table);
    const uint32_t *begins = reinterpret_cast<const uint32_t *>(b->ws_dev + wl.begins);
    HIP_TRY(hipMemcpyAsync(ents, stage, sizeof(WholeEntry) * m, hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->ws_dev + wl.begins, stage_begins, sizeof(uint32_t) * (m + 1), hipMemcpyHostToDevice,
                           b->stream));
    const uint64_t key[4] = {ISF_BATCH_WHOLE, ((uint64_t)m << 32) | blocks, tiling_key(tl), Zmax};
    int32_t rc = batch_enqueue(b, key, sweeps, [&](uint32_t g) -> int32_t {
        hipError_t e = launch_sweep_i8_halo_batch(ents, begins, m, blocks, tl, Zmax, g & 1u, b->stream);
        return e == hipSuccess ? ISF_OK : fail(ISF_EHIP, "batched sweep launch: %s", hipGetErrorString(e));
    });
    if (rc)
        return rc;
    // a film past its schedule's end sits out the remaining launches: its spins
    // moved once per sweep it ran
    for (uint32_t i = 0; i < n; ++i) {
        isf_lattice *lat = lats[i];
        const uint64_t ran = std::min<uint64_t>(lat->sched_total - lat->sched_enqueued, sweeps);
        if (ran & 1u)
            lat->cur_spare = !lat->cur_spare;
        lat->sched_enqueued += ran;
    }
    if (enqueued_out)
        *enqueued_out = sweeps;
    return ISF_OK;
}

// One launch per sublattice (or one persistent launch per chunk) over every
// film.  The caller has waited for the staging area and records b->staged.
int32_t batch_advance_phase(isf_batch *b, isf_lattice *const *lats, uint32_t n, uint32_t max_sweeps, int32_t mode,
                            uint64_t *enqueued_out) {
    const uint32_t format = lats[0]->d.format;
    // batches run the one-launch-per-sublattice tiles; other kernels fall back to the default shape
    const Tiling tl = lats[0]->tiling.kernel == ISF_KERNEL_TILES ? lats[0]->tiling : Tiling{64, 4, 2, ISF_KERNEL_TILES};
    // batch kernels work on the main copy of the spins
    for (uint32_t i = 0; i < n; ++i)
        if (lats[i]->cur_spare || lats[i]->whole_active) {
            int32_t rc = settle(lats[i]);
            if (rc)
                return rc;
            HIP_TRY(hipStreamSynchronize(lats[i]->stream));
        }
    const WsLayout wl = ws_layout(b->max_lats);
    BatchEntry *stage = reinterpret_cast<BatchEntry *>(static_cast<uint8_t *>(b->staging) + wl.phase);
    uint64_t sweeps = 0;
    uint32_t m = 0, blocks = 0;
    for (uint32_t i = 0; i < n; ++i) {
        isf_lattice *lat = lats[i];
        const uint64_t rem = lat->sched_total - lat->sched_enqueued;
        if (rem == 0)
            continue;
        BatchEntry &e = stage[m++];
        e.lat = lat->L;
        e.block_begin = blocks;
        if (format == ISF_FORMAT_INT8)
            batch_grid_i8(lat->L, tl, e.nbx, e.nby, e.nbz);
        else
            batch_grid_bp(lat->L, tl, e.nbx, e.nby, e.nbz);
        blocks += e.nbx * e.nby * e.nbz;
        sweeps = std::max<uint64_t>(sweeps, std::min<uint64_t>(rem, max_sweeps));
    }
    if (m == 0 || sweeps == 0) {
        if (enqueued_out)
            *enqueued_out = 0;
        return ISF_OK;
    }
    BatchEntry *ents = reinterpret_cast<BatchEntry *>(b->ws_dev + wl.phase);
    uint32_t *barrier = reinterpret_cast<uint32_t *>(b->ws_dev + wl.barrier);
    HIP_TRY(hipMemcpyAsync(ents, stage, sizeof(BatchEntry) * m, hipMemcpyHostToDevice, b->stream));
    if (mode == ISF_BATCH_PHASE_LAUNCH) {
        const uint64_t key[4] = {ISF_BATCH_PHASE_LAUNCH, ((uint64_t)m << 32) | blocks, tiling_key(tl), format};
        int32_t rc = batch_enqueue(b, key, sweeps, [&](uint32_t) -> int32_t {
            for (uint32_t s = 0; s < 4; ++s) {
                hipError_t e = format == ISF_FORMAT_INT8
                                   ? launch_phase_i8_batch(ents, m, blocks, tl, s, b->stream)
                                   : launch_phase_bp_batch(ents, m, blocks, tl, s, b->stream);
                if (e != hipSuccess)
                    return fail(ISF_EHIP, "batched phase launch: %s", hipGetErrorString(e));
            }
            hipError_t e = launch_sweep_end_batch(ents, m, b->stream);
            return e == hipSuccess ? ISF_OK : fail(ISF_EHIP, "batched sweep-end launch: %s", hipGetErrorString(e));
        });
        if (rc)
            return rc;
    } else {
        // chunks keep the barrier's arrival counter (sweeps x 5 x grid) far below 2^32
        for (uint64_t done = 0; done < sweeps;) {
            const uint32_t chunk = (uint32_t)std::min<uint64_t>(sweeps - done, 2048);
            uint32_t grid = 0;
            hipError_t e = launch_persistent(ents, m, blocks, format, tl, chunk, barrier, b->stream, &grid);
            if (e != hipSuccess)
                return fail(ISF_EHIP, "persistent launch: %s", hipGetErrorString(e));
            done += chunk;
        }
        b->persistent_used = true;
    }
    for (uint32_t i = 0; i < n; ++i) {
        isf_lattice *lat = lats[i];
        lat->sched_enqueued += std::min<uint64_t>(lat->sched_total - lat->sched_enqueued, sweeps);
    }
    if (enqueued_out)
        *enqueued_out = sweeps;
    return ISF_OK;
}

// Pipelined mode: every film the pipelined kernel can take (INT8, a region
// within one period, LDS for the batch's deepest such film) is swept by one
// launch per sweep over all of them, each film with its own share of the
// blocks (about kPipeBatchTiles tiles per block, its lists and tile order
// built for that count); the others run in the sublattice mode.  The caller
// has waited for the staging area and records b->staged.
constexpr uint32_t kPipeBatchTiles = 8;

int32_t batch_advance_pipe(isf_batch *b, isf_lattice *const *lats, uint32_t n, uint32_t max_sweeps,
                           uint64_t *enqueued_out) {
    std::vector<isf_lattice *> pipe, rest;
    const Tiling tl{32, 32, 16, ISF_KERNEL_PIPE};
    uint32_t Zp = 0;  // the deepest film of the pipelined launch sizes its LDS
    for (uint32_t i = 0; i < n; ++i) {
        isf_lattice *lat = lats[i];
        const bool ok =
            lat->d.format == ISF_FORMAT_INT8 && lat->spare && pipe_fits(lat, tl, lat->d.Z, true) == ISF_OK;
        (ok ? pipe : rest).push_back(lat);
        if (ok)
            Zp = std::max(Zp, lat->d.Z);
    }
    uint64_t enq_rest = 0, sweeps = 0;
    if (!rest.empty()) {
        int32_t rc = batch_advance_phase(b, rest.data(), (uint32_t)rest.size(), max_sweeps, ISF_BATCH_PHASE_LAUNCH,
                                         &enq_rest);
        if (rc)
            return rc;
    }
    const WsLayout wl = ws_layout(b->max_lats);
    PipeEntry *stage = reinterpret_cast<PipeEntry *>(static_cast<uint8_t *>(b->staging) + wl.table);
    uint32_t *stage_begins = reinterpret_cast<uint32_t *>(static_cast<uint8_t *>(b->staging) + wl.begins);
    uint32_t m = 0, blocks = 0;
    for (isf_lattice *lat : pipe) {
        const uint64_t rem = lat->sched_total - lat->sched_enqueued;
        if (rem == 0)
            continue;
        uint32_t nbx = 0, tiles = 0, nb = 0, kmax = 0;
        pipe_grid(lat->L, tl.tx, tl.ty, 1u, &nbx, &tiles, &nb, &kmax);
        const uint32_t cap = std::max(1u, (tiles + kPipeBatchTiles - 1) / kPipeBatchTiles);
        pipe_grid(lat->L, tl.tx, tl.ty, cap, &nbx, &tiles, &nb, &kmax);
        int32_t rc;
        if ((rc = prepare_spare(lat, tl, cap)) || (rc = prime_whole(lat)))
            return rc;
        HIP_TRY(hipStreamSynchronize(lat->stream));
        PipeEntry &e = stage[m++];
        e.lat = lat->L;
        e.spare = lat->spare;
        e.lists = lat->lists;
        e.block_begin = blocks;
        stage_begins[m - 1] = blocks;
        e.nbx = nbx;
        e.ntiles = tiles;
        e.kmax = kmax;
        e.po = lat->cur_spare ? 1u : 0u;
        e.pad = 0;
        blocks += nb;
        sweeps = std::max<uint64_t>(sweeps, std::min<uint64_t>(rem, max_sweeps));
    }
    if (m && sweeps) {
        stage_begins[m] = blocks;
        PipeEntry *ents = reinterpret_cast<PipeEntry *>(b->ws_dev + wl.table);
        const uint32_t *begins = reinterpret_cast<const uint32_t *>(b->ws_dev + wl.begins);
        HIP_TRY(hipMemcpyAsync(ents, stage, sizeof(PipeEntry) * m, hipMemcpyHostToDevice, b->stream));
        HIP_TRY(hipMemcpyAsync(b->ws_dev + wl.begins, stage_begins, sizeof(uint32_t) * (m + 1),
                               hipMemcpyHostToDevice, b->stream));
        const uint64_t key[4] = {ISF_BATCH_PIPE, ((uint64_t)m << 32) | blocks, tiling_key(tl), Zp};
        int32_t rc = batch_enqueue(b, key, sweeps, [&](uint32_t g) -> int32_t {
            hipError_t e = launch_sweep_i8_pipe_batch(ents, begins, m, blocks, tl, Zp, g & 1u, b->stream);
            return e == hipSuccess ? ISF_OK : fail(ISF_EHIP, "batched pipelined launch: %s", hipGetErrorString(e));
        });
        if (rc)
            return rc;
        for (isf_lattice *lat : pipe) {
            const uint64_t ran = std::min<uint64_t>(lat->sched_total - lat->sched_enqueued, sweeps);
            if (ran & 1u)
                lat->cur_spare = !lat->cur_spare;
            lat->sched_enqueued += ran;
        }
    }
    if (enqueued_out)
        *enqueued_out = std::max(sweeps, enq_rest);
    return ISF_OK;
}

}  // namespace

extern "C" {

int32_t isf_batch_advance(isf_batch *b, isf_lattice *const *lats, uint32_t n, uint32_t max_sweeps, int32_t mode,
                          uint64_t *enqueued_out) {
    if (!b || (n && !lats))
        return fail(ISF_EINVAL, "null pointer argument");
    if (n > b->max_lats)
        return fail(ISF_EINVAL, "%u lattices exceed the batch capacity %u", n, b->max_lats);
    if (mode != ISF_BATCH_PHASE_LAUNCH && mode != ISF_BATCH_PERSISTENT && mode != ISF_BATCH_WHOLE &&
        mode != ISF_BATCH_PIPE)
        return fail(ISF_EINVAL, "unknown batch mode %d", mode);
    if (n == 0) {
        if (enqueued_out)
            *enqueued_out = 0;
        return ISF_OK;
    }
    const uint32_t format = lats[0]->d.format;
    for (uint32_t i = 0; i < n; ++i) {
        if (!lats[i])
            return fail(ISF_EINVAL, "null lattice %u", i);
        if (lats[i]->d.format != format)
            return fail(ISF_ESTATE, "lattices of a batch must share one format");
        if (lats[i]->aniso)
            return fail(ISF_EINVAL, "lattice %u: batches do not run the anisotropy term", i);
    }
    // the staging area may still be read by the previous call's copies
    HIP_TRY(hipEventSynchronize(b->staged));
    int32_t rc;
    if (mode == ISF_BATCH_WHOLE)
        rc = batch_advance_whole(b, lats, n, max_sweeps, enqueued_out);
    else if (mode == ISF_BATCH_PIPE)
        rc = batch_advance_pipe(b, lats, n, max_sweeps, enqueued_out);
    else
        rc = batch_advance_phase(b, lats, n, max_sweeps, mode, enqueued_out);
    if (rc)
        return rc;
    HIP_TRY(hipEventRecord(b->staged, b->stream));
    return ISF_OK;
}

int32_t isf_batch_run(isf_batch *b, isf_lattice *const *lats, uint32_t n, const isf_step *const *steps,
                      const uint32_t *n_steps, isf_record *const *out, int32_t mode) {
    if (!b || (n && (!lats || !steps || !n_steps || !out)))
        return fail(ISF_EINVAL, "null pointer argument");
    int32_t rc;
    for (uint32_t i = 0; i < n; ++i)
        if ((rc = isf_schedule_load(lats[i], steps[i], n_steps[i])))
            return rc;
    uint64_t got = 0;
    if ((rc = isf_batch_advance(b, lats, n, 0xFFFFFFFFu, mode, &got)))
        return rc;
    if ((rc = isf_batch_sync(b)))
        return rc;
    for (uint32_t i = 0; i < n; ++i) {
        if (n_steps[i] && !out[i])
            return fail(ISF_EINVAL, "null record buffer %u", i);
        if ((rc = isf_schedule_records(lats[i], out[i], n_steps[i])))
            return rc;
    }
    return ISF_OK;
}

}  // extern "C"
