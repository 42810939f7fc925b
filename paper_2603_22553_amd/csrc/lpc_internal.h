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
};

struct Geometry {
    int32_t nx, ny, nz;
    int32_t bc[3];  // 0 periodic, 1 closed
};

// Launch shape of the sweep: a 1-D grid of workgroups, each owning a TX x TY x-y tile
// and a run of zc planes. Blocks are renumbered so that each XCD gets a contiguous
// range of tiles (hardware dispatch is round-robin over the 8 XCDs).
struct SweepPlan {
    int32_t kernel;      // 0 = direct (cache-read neighbours), 1 = z-march with LDS tiles
    int32_t tx, ty, zc;
    int32_t gx, gy, gz;
    int64_t nblocks;
};

struct StepArgs {
    Geometry g;
    int32_t precision;   // 0 FP64, 1 mixed
    uint32_t track;
    int32_t R;           // regions
    int32_t K;           // record width
    double p0;
    const void *F;
    const void *theta;
    const uint8_t *region;
    StateView src, dst;
    double *partials;    // [K][nblocks] for this step
};

// Upper bound on the workgroups of any plan for g (sizes the per-step partial sums).
int64_t max_sweep_blocks(const Geometry &g);
// Plan for g given the resident sweep workgroups per compute unit and the compute units.
SweepPlan make_plan(const Geometry &g, int32_t blocks_per_cu, int32_t cus);
// Resident sweep workgroups per compute unit for this precision, track set and regions.
int sweep_blocks_per_cu(int32_t precision, uint32_t track, int32_t R);

hipError_t launch_step(const SweepPlan &plan, const StepArgs &a, hipStream_t s);
hipError_t launch_record(const SweepPlan &plan, const StepArgs &a, hipStream_t s);
hipError_t launch_finalize(const double *partials, int64_t nblocks, int32_t K, int64_t steps,
                           double *records_out, hipStream_t s);

// Field set-up: dst[i] = (storage) src[i] or the phase of a shift.
hipError_t launch_store_field(int32_t precision, const double *src, void *dst, int64_t n,
                              double scale, hipStream_t s);
// Initial state: mode 0 uniform, 1 rho from `rho_src` (device, double), with m = rho, moments 0.
hipError_t launch_init_state(int32_t precision, uint32_t track, const StateView &st,
                             const double *rho_src, int64_t n, hipStream_t s);
// Boltzmann weights w_i = exp(-(F_i - Fmin)) into w, block sums into partials[nb].
hipError_t launch_boltzmann_weights(int32_t precision, const void *F, double Fmin, double *w,
                                    int64_t n, double *partials, int64_t *nb, hipStream_t s);
// rho_i = w_i * scale_num / (*Z) in place.
hipError_t launch_boltzmann_scale(double *w, int64_t n, double numer, const double *Z,
                                  hipStream_t s);

// Plain copy of n16 16-byte words (calibration kernel).
hipError_t launch_stream_copy(const void *src, void *dst, int64_t n16, hipStream_t s);

}  // namespace lpc
