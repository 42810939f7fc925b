// Internal interface between the C-ABI layer (api.hip) and the kernels (sweep.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lpc {

constexpr int kMaxRegions = 8;

// Device views of one state buffer. Populations are double on every path; the
// magnetisation and moment arrays use the storage type of the precision mode.
struct StateView {
    double *rho;
    void *re, *im;
    void *m1[3], *m2[3];
    void *v[3];        // first-displacement tags per axis (velocity autocorrelation), or null
};

// Track bit of the velocity autocorrelation field (LPC_TRACK_VACF): with it the moment
// template parameter of the sweep is 2 (moments and tags) instead of 1.
constexpr uint32_t kTrackVacf = 4u;

struct Geometry {
    int32_t nx, ny, nz;
    int32_t bc[3];  // 0 periodic, 1 closed
};

// Launch shape of the sweep: a 1-D grid of workgroups, each owning a tx x ty x-y tile
// and a run of zc planes. Blocks are renumbered so that each XCD gets a contiguous
// range of tiles (hardware dispatch is round-robin over the 8 XCDs).
// tx = kTileLinear: a tile is a run of 256 consecutive sites of the x-y plane (x fastest)
// rather than a tx x ty block of columns; ty is then 256.
struct SweepPlan {
    int32_t tx, ty, zc;
    int32_t gx, gy, gz;
    int64_t nblocks;
};

// SweepPlan.tx of a linear tile.
constexpr int32_t kTileLinear = 1;
// SweepPlan.tx of a two-step plan: tiles of 30 x 6 owned columns, each pass two steps
// (plain variant only).
constexpr int32_t kTileTwoStep = 2;
constexpr int32_t kTwoStepTileX = 30, kTwoStepTileY = 6;

// Kernel variant bit carried next to the track bits: the lattice has a mobility field or
// a reservoir axis, and runs the extended sweep variant.
constexpr uint32_t kVariantExtended = 8u;

// Geometry.bc value of an axis with fixed ghost sites beyond its faces.
constexpr int32_t kBcReservoir = 2;

// Stored free energy of an inaccessible site: finite, so that differences with it stay
// finite (and the hop probabilities into and out of it exact zeros), and beyond any
// accepted free energy (|F| <= 1e30); one value per storage precision.
constexpr double kBlockedF64 = 1e300;
constexpr double kBlockedF32 = 3e38;
// A stored free energy at or above this marks an inaccessible site.
constexpr double kBlockedTest = 1e36;

struct StepArgs {
    Geometry g;
    int32_t precision;   // 0 FP64, 1 mixed
    uint32_t track;      // LPC_TRACK_* bits | kVariantExtended
    int32_t R;           // regions
    int32_t K;           // record width
    double p0;
    double fc;             // centre of the accessible free energies (FP64 cell weights)
    const void *F;         // free energies (float path), factors e^{F - fc} (FP64 path)
    const void *theta;
    const uint8_t *region;
    const void *mu;        // per-site mobility (storage type), or null
    const double *ghost;   // 6 faces x (F, rho, Re m, Im m) for reservoir axes
    StateView src, dst;
    double *partials;    // [K][nblocks] for this step
    int32_t tag;         // 1 on the first step after a start: the autocorrelation tags are set
    int32_t pad;
};

// Upper bound on the workgroups of any plan for g (sizes the per-step partial sums).
int64_t max_sweep_blocks(const Geometry &g);
// Plan for g given the resident sweep workgroups per compute unit and the compute units;
// tile_x 64, 32 or 16 fixes the tile width, kTileLinear asks for linear tiles (only when
// g.nx <= linear_nx_max), anything else picks the tiles with the fewest idle lanes.
// linear_nx_max is the widest lattice the kernel variant runs on linear tiles (0: none);
// automatic z-chunks are at least zc_floor planes (or the whole axis).
SweepPlan make_plan(const Geometry &g, int32_t blocks_per_cu, int32_t cus, int32_t tile_x,
                    int32_t linear_nx_max, int32_t zc_floor);
// Widest x extent the sweep variant of this precision and track set runs on linear tiles:
// the LDS window of a linear tile holds 256 + 2 nx cells, within the share of LDS that keeps
// two workgroups resident per compute unit. 0 for the extended variant.
int32_t linear_tile_max_nx(int32_t precision, uint32_t track);
// The plan with its z-chunk forced to zc planes (zc >= 1).
SweepPlan with_z_chunk(SweepPlan p, const Geometry &g, int32_t zc);
// Resident sweep workgroups per compute unit for this precision, track set and regions,
// for the one-step (steps_per_pass 1) or the two-step kernel (2).
int sweep_blocks_per_cu(int32_t precision, uint32_t track, int32_t R, int32_t steps_per_pass = 1);
// Plan of the two-step kernel: 30 x 6 owned columns per tile, z-chunks as make_plan chooses
// them (at least zc_floor planes).
SweepPlan make_plan2(const Geometry &g, int32_t blocks_per_cu, int32_t cus, int32_t zc_floor);

// One entry of a sweep work list: a lattice's step arguments (views of the parity-0 step)
// and its plan.
struct SweepItem {
    StepArgs a;
    SweepPlan plan;
};

// A work list in device memory: items[0, n_items) whose workgroups are numbered by the
// exclusive prefix sums prefix[0, n_items] of their plans' nblocks (total = prefix[n_items]),
// all with tiles tile_x wide; one launch steps them all with the given parity, writing
// partial sums into step slot `slot` of each lattice's partials.
struct StepList {
    const SweepItem *items;
    const int64_t *prefix;
    int32_t n_items;
    int32_t tile_x;
    int64_t total;
    int32_t parity;
    int64_t slot;
};

// Records of a finalisation: partials [steps][K][nblocks] of one lattice into rows
// row_base + first_row + s of its records.
struct FinalizeItem {
    const double *partials;
    double *records;
    int64_t nblocks;
    int64_t row_base;
    int32_t K;
    int32_t pad;
};

hipError_t launch_step_list(const StepList &list, int32_t precision, uint32_t track, int32_t maxr,
                            hipStream_t s);
hipError_t launch_finalize_list(const FinalizeItem *items, const int64_t *kprefix, int32_t n_items,
                                int64_t total_k, int64_t steps, int64_t first_row, hipStream_t s,
                                const int64_t *row_offset = nullptr);
// *counter = value (add == 0) or *counter += add, on the device in stream order.
hipError_t launch_set_counter(int64_t *counter, int64_t value, int64_t add, hipStream_t s);
hipError_t launch_record(const SweepPlan &plan, const StepArgs &a, hipStream_t s);
hipError_t launch_finalize(const double *partials, int64_t nblocks, int32_t K, int64_t steps,
                           double *records_out, hipStream_t s);

// Field set-up: dst[i] = (storage) src[i] or the phase of a shift.
hipError_t launch_store_field(int32_t precision, const double *src, void *dst, int64_t n,
                              double scale, hipStream_t s);
// Initial state: mode 0 uniform, 1 rho from `rho_src` (device, double), with m = rho, moments 0.
hipError_t launch_init_state(int32_t precision, uint32_t track, const StateView &st,
                             const double *rho_src, const void *F, int64_t n, hipStream_t s);
// dst[i] = value for i < n in the storage type.
hipError_t launch_fill_field(int32_t precision, void *dst, int64_t n, double value,
                             hipStream_t s);
// Boltzmann weights w_i = exp(-(F_i - Fmin)) into w, block sums into partials[nb].
hipError_t launch_boltzmann_weights(int32_t precision, const void *F, double Fmin, double *w,
                                    int64_t n, double *partials, int64_t *nb, hipStream_t s);
// E_i = exp(F_i - fc), FP64: the per-site Boltzmann factors the FP64 sweep reads in place of
// the free energies.
hipError_t launch_boltzmann_factors(const double *F, double *E, int64_t n, double fc,
                                    hipStream_t s);
// rho_i = w_i * scale_num / (*Z) in place.
hipError_t launch_boltzmann_scale(double *w, int64_t n, double numer, const double *Z,
                                  hipStream_t s);

// Spectrum of the recorded FID: normalised, zero-filled series in buf_a, Stockham FFT
// ping-ponging between buf_a and buf_b (L complex values each, L a power of two), then
// the ascending-frequency real parts in sorted[0, L) and imaginary parts in
// sorted[L, 2L); sorted == nullptr writes them into whichever buffer is free. Returns
// through *where the buffer holding the sorted output (when sorted is nullptr).
hipError_t launch_fid_spectrum(const double *records, int64_t rows, int32_t K, int32_t R,
                               int32_t region, int64_t L, double2 *buf_a, double2 *buf_b,
                               double *sorted, hipStream_t s);
// Index of the first maximum of v[0, n) into *out (nparts workgroup partials).
hipError_t launch_argmax(const double *v, int64_t n, double *pval, int64_t *pidx, int32_t nparts,
                         int64_t *out, hipStream_t s);
// out[0] = max_i |next_i - prev_i|, out[1] = max_i next_i (nparts workgroup partials of two
// doubles in part).
hipError_t launch_max_change(const double *prev, const double *next, int64_t n, double *part,
                             int32_t nparts, double *out, hipStream_t s);
// Workgroup partials part[k * nparts + b] of the per-region sums k = 7 r + q of rho, M1_a,
// M2_a (q = 0: rho; 1..3: M1 x y z; 4..6: M2 x y z); finalised like record partials.
hipError_t launch_region_sums(int32_t precision, const StateView &st, const uint8_t *region,
                              int64_t n, int32_t R, double *part, int32_t nparts, hipStream_t s);
// Population summed over the planes perpendicular to `axis`.
hipError_t launch_profile(const double *rho, const Geometry &g, int32_t axis, double *profile,
                          hipStream_t s);

// Plain copy of n16 16-byte words (calibration kernel).
hipError_t launch_stream_copy(const void *src, void *dst, int64_t n16, hipStream_t s);

// The FP64 full sweep's column streams without its arithmetic (calibration kernel): 12
// arrays read and 9 written, nx * ny * nz doubles each.
constexpr int kColumnIn = 12, kColumnOut = 9;
struct ColumnArrays {
    const double *in[kColumnIn];
    double *out[kColumnOut];
};
hipError_t launch_stream_columns(const ColumnArrays &c, int32_t nx, int32_t ny, int32_t nz,
                                 int32_t zc, hipStream_t s);

// The mixed full sweep's column streams without its arithmetic (calibration kernel): the
// population in double, 10 float arrays (8 state, free energy, shift) and the region byte
// read; the population and the 8 float state arrays written.
constexpr int kMixedIn = 10, kMixedOut = 8;
struct MixedColumns {
    const double *rho_in;
    const float *in[kMixedIn];
    const uint8_t *region;
    double *rho_out;
    float *out[kMixedOut];
};
hipError_t launch_stream_columns_mixed(const MixedColumns &c, int32_t nx, int32_t ny, int32_t nz,
                                       int32_t zc, hipStream_t s);

}  // namespace lpc
