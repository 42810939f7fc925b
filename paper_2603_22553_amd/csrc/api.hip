// C-ABI of liblpc: lattice lifetime, arena layout, field set-up, run loop, reads and
// checkpoints. The operation itself is defined in include/lpc.h and the kernels live in
// sweep.hip; this file only validates arguments, places buffers in the caller's arena and
// queues work on the caller's stream.
#include "lpc.h"
#include "lpc_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace {

thread_local std::string g_error;

lpc_status fail(lpc_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return st;
}

lpc_status ok()
{
    return LPC_OK;
}

#define LPC_HIP(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(LPC_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));      \
    } while (0)

constexpr size_t kAlign = 256;
// Arena arrays of at least kStaggerMin bytes start kStagger bytes further apart than their
// sizes require. With a power-of-two site count every per-site array would otherwise begin
// at the same offset modulo the L2 set and HBM channel interleaves, so the same site of all
// of them would compete for one set and one channel. Measured on the 256^3 particle: +2 %
// (mixed) and +4.5 % (FP64); on the 2048 x 256 x 256 film +2 %.
constexpr size_t kStagger = 64 * 1024 + 256;
constexpr size_t kStaggerMin = size_t(1) << 20;
constexpr int64_t kStagingMax = int64_t(1) << 22;   // doubles per host<->device chunk
constexpr int64_t kPartialBudget = int64_t(32) << 20; // bytes of per-step partials per chunk
constexpr int64_t kChunkMax = 256;                    // steps finalised together
constexpr int kScalars = 64;
constexpr int kGhostValues = 24;   // 6 faces x (F, rho, Re m, Im m)
constexpr double kMaxFreeEnergy = 1e30;
constexpr double kMaxFreeEnergySpan = 1400.0;
constexpr int kArgmaxParts = 256;

// Smallest power of two >= 8 * samples: the default zero-filled FFT length.
int64_t fft_length(int64_t samples)
{
    int64_t L = 1;
    while (L < 8 * samples)
        L *= 2;
    return L;
}

size_t align_up(size_t v)
{
    return (v + kAlign - 1) / kAlign * kAlign;
}

struct Layout {
    int64_t n = 0;
    int K = 0;
    size_t storage = 8;
    lpc::SweepPlan plan{};
    int64_t chunk = 1;
    int64_t staging = 0;
    size_t off_F = 0, off_E = 0, off_theta = 0, off_region = 0, off_mu = 0, off_ghost = 0, off_partials = 0,
           off_records = 0, off_staging = 0, off_scalars = 0, off_fft = 0, off_argmax = 0,
           off_profile = 0, off_list = 0, off_regsum = 0;
    int64_t fft_max = 0;
    size_t off_rho[2] = {0, 0}, off_re[2] = {0, 0}, off_im[2] = {0, 0};
    size_t off_m1[2][3] = {}, off_m2[2][3] = {}, off_v[2][3] = {};
    size_t partial_bytes = 0;
    size_t total = 0;
};

// Steps whose partial sums fit the partials buffer together (finalised in one launch).
void set_chunk(Layout &L)
{
    const int64_t per_step = int64_t(L.K) * L.plan.nblocks * 8;
    int64_t c = int64_t(L.partial_bytes) / per_step;
    L.chunk = std::max<int64_t>(1, std::min<int64_t>(kChunkMax, c));
}

// Steps of two-step passes finalised together: an even count whose partials fit the buffer
// (which holds at least two steps of the largest plan).
int64_t two_step_chunk(const Layout &L, const lpc::SweepPlan &p2)
{
    const int64_t per_step = int64_t(L.K) * std::max<int64_t>(1, p2.nblocks) * 8;
    const int64_t c = std::min<int64_t>(kChunkMax, int64_t(L.partial_bytes) / per_step);
    return std::max<int64_t>(2, c - c % 2);
}

bool fid_of(const lpc_config &c)
{
    return (c.track & LPC_TRACK_FID) != 0;
}
bool msd_of(const lpc_config &c)
{
    return (c.track & LPC_TRACK_MSD) != 0;
}
bool vacf_of(const lpc_config &c)
{
    return (c.track & LPC_TRACK_VACF) != 0;
}
// Record width: per region Re/Im G and U, then S1 and S2 per axis, then (with the tags) the
// velocity autocorrelation per axis.
int record_width_of(const lpc_config &c)
{
    return 3 * c.n_regions + 6 + (vacf_of(c) ? 3 : 0);
}
bool mobility_of(const lpc_config &c)
{
    return (c.options & LPC_OPT_MOBILITY) != 0;
}
bool reservoir_of(const lpc_config &c)
{
    return c.bc[0] == LPC_BC_RESERVOIR || c.bc[1] == LPC_BC_RESERVOIR ||
           c.bc[2] == LPC_BC_RESERVOIR;
}
// Track bits plus the kernel variant bits of the configuration.
// Least z-chunk of automatic plans: 4 planes alone, 16 for lattices stepped in batches.
int32_t zc_floor(const lpc_config &c)
{
    return (c.options & LPC_OPT_BATCHED) ? 16 : 4;
}

uint32_t variant_of(const lpc_config &c)
{
    return c.track | (mobility_of(c) || reservoir_of(c) ? lpc::kVariantExtended : 0u);
}

// Two steps per pass are built for the plain variant (no mobility field, no reservoir axis)
// without autocorrelation tags.
bool two_step_available(const lpc_config &c)
{
    return !(variant_of(c) & lpc::kVariantExtended) && !vacf_of(c);
}

lpc_status validate_config(const lpc_config *c)
{
    if (!c)
        return fail(LPC_ERR_ARG, "config is NULL");
    for (int a = 0; a < 3; ++a) {
        if (c->n[a] < 1)
            return fail(LPC_ERR_ARG, "n[%d] = %d must be >= 1", a, c->n[a]);
        if (c->bc[a] != LPC_BC_PERIODIC && c->bc[a] != LPC_BC_CLOSED &&
            c->bc[a] != LPC_BC_RESERVOIR)
            return fail(LPC_ERR_ARG, "bc[%d] = %d is not PERIODIC, CLOSED or RESERVOIR", a,
                        c->bc[a]);
    }
    if (int64_t(c->n[0]) * c->n[1] > (int64_t(1) << 28))
        return fail(LPC_ERR_ARG, "nx * ny must not exceed 2^28 (one z-plane of doubles < 2 GiB)");
    if (c->precision != LPC_PREC_FP64 && c->precision != LPC_PREC_MIXED)
        return fail(LPC_ERR_ARG, "precision %d unknown", c->precision);
    if (c->track & ~uint32_t(LPC_TRACK_FID | LPC_TRACK_MSD | LPC_TRACK_VACF))
        return fail(LPC_ERR_ARG, "track bits 0x%x unknown", c->track);
    if ((c->track & LPC_TRACK_VACF) && !(c->track & LPC_TRACK_MSD))
        return fail(LPC_ERR_ARG, "LPC_TRACK_VACF needs LPC_TRACK_MSD");
    if (c->n_regions < 1 || c->n_regions > LPC_MAX_REGIONS)
        return fail(LPC_ERR_ARG, "n_regions = %d outside 1..%d", c->n_regions, LPC_MAX_REGIONS);
    if (c->options & ~uint32_t(LPC_OPT_MOBILITY | LPC_OPT_BATCHED))
        return fail(LPC_ERR_ARG, "option bits 0x%x unknown", c->options);
    if (!std::isfinite(c->p_hop) || c->p_hop < 0.0 || 6.0 * c->p_hop > 1.0)
        return fail(LPC_ERR_ARG, "p_hop = %g must satisfy 0 <= 6 p_hop <= 1", c->p_hop);
    if (!std::isfinite(c->dt_s) || !std::isfinite(c->larmor_hz) || !std::isfinite(c->spacing_m) ||
        c->dt_s <= 0.0 || c->spacing_m <= 0.0)
        return fail(LPC_ERR_ARG, "dt_s and spacing_m must be positive, larmor_hz finite");
    if (c->max_records < 1)
        return fail(LPC_ERR_ARG, "max_records must be >= 1");
    if (!std::isfinite(c->conservation_tol) || c->conservation_tol < 0.0)
        return fail(LPC_ERR_ARG, "conservation_tol must be >= 0");
    return LPC_OK;
}

// The one-entry work list through which lpc_run steps a lattice alone (the same kernels
// step it inside a batch).
struct SoloTables {
    lpc::SweepItem item;
    int64_t prefix[2];
    lpc::FinalizeItem fin;
    int64_t kprefix[2];
    lpc::SweepItem eq_item;      // the population-only sweep of lpc_equilibrate
    int64_t eq_prefix[2];
    lpc::SweepItem item_tag;     // the first step after a start: sets the autocorrelation tags
    lpc::SweepItem item2;        // the two-step sweep (plans of two steps per pass)
    int64_t prefix2[2];
    lpc::FinalizeItem fin2;
};

// Buffer placement for cfg. The sweep plan depends on the device (resident workgroups per
// compute unit), so the per-step partial sums are sized for the largest plan; `plan` and
// `chunk` are provisional here and fixed by lpc_create.
Layout plan_layout(const lpc_config &c)
{
    Layout L;
    L.n = int64_t(c.n[0]) * c.n[1] * c.n[2];
    L.K = record_width_of(c);
    L.storage = c.precision == LPC_PREC_FP64 ? 8 : 4;
    lpc::Geometry g{c.n[0], c.n[1], c.n[2], {c.bc[0], c.bc[1], c.bc[2]}};
    L.plan = lpc::make_plan(g, 1, 256, 0, lpc::linear_tile_max_nx(c.precision, variant_of(c)),
                            zc_floor(c));
    const int64_t per_step_max = int64_t(L.K) * lpc::max_sweep_blocks(g) * 8;
    L.staging = L.n < kStagingMax ? L.n : kStagingMax;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes) + (bytes >= kStaggerMin ? kStagger : 0);
        return at;
    };
    const size_t ns = size_t(L.n) * L.storage;
    L.off_F = take(ns);
    // FP64 path: the Boltzmann factors e^{F - c} the sweep reads
    L.off_E = take(c.precision == LPC_PREC_FP64 ? ns : 0);
    L.off_theta = take(fid_of(c) ? ns : 0);
    L.off_region = take(size_t(L.n));
    L.off_mu = take(mobility_of(c) ? ns : 0);
    L.off_ghost = take(kGhostValues * 8);
    for (int b = 0; b < 2; ++b) {
        L.off_rho[b] = take(size_t(L.n) * 8);
        L.off_re[b] = take(fid_of(c) ? ns : 0);
        L.off_im[b] = take(fid_of(c) ? ns : 0);
        for (int a = 0; a < 3; ++a) {
            L.off_m1[b][a] = take(msd_of(c) ? ns : 0);
            L.off_m2[b][a] = take(msd_of(c) ? ns : 0);
            L.off_v[b][a] = take(vacf_of(c) ? ns : 0);
        }
    }
    L.partial_bytes = size_t(std::max<int64_t>(kPartialBudget, 2 * per_step_max));
    L.off_partials = take(L.partial_bytes);
    L.off_records = take(size_t(c.max_records) * L.K * 8);
    L.off_staging = take(size_t(L.staging) * 8);
    L.off_scalars = take(kScalars * 8);
    L.fft_max = fid_of(c) ? fft_length(c.max_records) : 0;
    L.off_fft = take(size_t(L.fft_max) * 32);                 // two complex buffers
    L.off_argmax = take(kArgmaxParts * 16 + 64);
    L.off_profile = take(size_t(std::max(c.n[0], std::max(c.n[1], c.n[2]))) * 8);
    L.off_list = take(sizeof(SoloTables));
    L.off_regsum = take(7 * LPC_MAX_REGIONS * 8);
    L.total = o;
    set_chunk(L);
    return L;
}

}  // namespace

struct lpc_lattice {
    lpc_config cfg{};
    Layout L;
    hipStream_t stream = nullptr;
    int device = 0;
    char *arena = nullptr;
    lpc::StateView st[2]{};
    int cur = 0;
    bool initialized = false;
    int64_t steps_done = 0;
    double Fmin = 0.0;
    double Fmid = 0.0;                        // centre of the accessible free energies
    int64_t n_open = 0;                       // accessible sites (F < +inf)
    double ghost[kGhostValues] = {};          // host copy of the reservoir ghost table
    // Plan of the population-only sweeps of lpc_equilibrate: made for that kernel's own
    // occupancy (it keeps more workgroups resident than the full sweep) and tile limits.
    // Their partial sums are discarded, so the plan fixes no result.
    lpc::SweepPlan eq_plan{};
    int occupancy = 1, cus = 1;      // resident sweep workgroups per CU, compute units
    // Temporal blocking: steps per sweep pass (1, or 2 with the two-step plan), the plan of
    // the two-step kernel, its resident workgroups per CU and the steps finalised together.
    int32_t steps_per_pass = 1;
    lpc::SweepPlan plan2{};
    int occupancy2 = 0;
    int64_t chunk2 = 2;

    template <typename T = void>
    T *at(size_t off) const
    {
        return reinterpret_cast<T *>(arena + off);
    }
    double *partials() const { return at<double>(L.off_partials); }
    double *records() const { return at<double>(L.off_records); }
    double *staging() const { return at<double>(L.off_staging); }
    double *scalars() const { return at<double>(L.off_scalars); }

    lpc::SweepItem sweep_item(int src) const
    {
        lpc::SweepItem it{};
        it.a = args(src);
        it.plan = L.plan;
        return it;
    }

    lpc::FinalizeItem finalize_item(int64_t row_base, int64_t nblocks = -1) const
    {
        lpc::FinalizeItem f{};
        f.partials = partials();
        f.records = records();
        f.nblocks = nblocks < 0 ? L.plan.nblocks : nblocks;
        f.row_base = row_base;
        f.K = L.K;
        return f;
    }

    SoloTables *solo() const { return at<SoloTables>(L.off_list); }

    lpc::StepArgs args(int src) const
    {
        lpc::StepArgs a{};
        a.g = {cfg.n[0], cfg.n[1], cfg.n[2], {cfg.bc[0], cfg.bc[1], cfg.bc[2]}};
        a.precision = cfg.precision;
        a.track = variant_of(cfg);
        a.R = cfg.n_regions;
        a.K = L.K;
        a.p0 = cfg.p_hop;
        a.fc = Fmid;
        a.F = at(cfg.precision == LPC_PREC_FP64 ? L.off_E : L.off_F);
        a.theta = at(L.off_theta);
        a.region = at<uint8_t>(L.off_region);
        a.mu = mobility_of(cfg) ? at(L.off_mu) : nullptr;
        a.ghost = at<double>(L.off_ghost);
        a.src = st[src];
        a.dst = st[1 - src];
        a.partials = partials();
        return a;
    }
};

namespace {

lpc_status use_device(const lpc_lattice *lat)
{
    int d = -1;
    LPC_HIP(hipGetDevice(&d));
    if (d != lat->device)
        LPC_HIP(hipSetDevice(lat->device));
    return LPC_OK;
}

// Uploads the one-entry work list of lpc_run (plan and step arguments) after anything it
// holds has changed. The lattice's stream must be idle.
SoloTables solo_tables(const lpc_lattice *lat)
{
    SoloTables tables{};
    tables.item = lat->sweep_item(0);
    tables.prefix[0] = 0;
    tables.prefix[1] = lat->L.plan.nblocks;
    tables.fin = lat->finalize_item(0);
    tables.kprefix[0] = 0;
    tables.kprefix[1] = lat->L.K;
    tables.eq_item = tables.item;
    tables.eq_item.plan = lat->eq_plan;
    tables.eq_prefix[0] = 0;
    tables.eq_prefix[1] = lat->eq_plan.nblocks;
    tables.item_tag = tables.item;
    tables.item_tag.a.tag = 1;
    tables.item2 = tables.item;
    tables.item2.plan = lat->plan2;
    tables.prefix2[0] = 0;
    tables.prefix2[1] = lat->plan2.nblocks;
    tables.fin2 = lat->finalize_item(0, lat->plan2.nblocks);
    return tables;
}

// A copy on the lattice's stream, waited for. A plain hipMemcpy runs on the null stream and
// would also wait for unrelated work queued there, such as a batch stepped on the default
// stream while this lattice is set up or read.
hipError_t copy_sync(const lpc_lattice *lat, void *dst, const void *src, size_t bytes,
                     hipMemcpyKind kind)
{
    const hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, lat->stream);
    return e == hipSuccess ? hipStreamSynchronize(lat->stream) : e;
}

lpc_status upload_solo(lpc_lattice *lat)
{
    const SoloTables tables = solo_tables(lat);
    LPC_HIP(copy_sync(lat, lat->solo(), &tables, sizeof tables, hipMemcpyHostToDevice));
    return LPC_OK;
}

lpc_status check_sites(const lpc_lattice *lat, const void *p, int64_t n)
{
    if (!p)
        return fail(LPC_ERR_ARG, "array is NULL");
    if (n != lat->L.n)
        return fail(LPC_ERR_ARG, "array has %lld values, lattice has %lld sites", (long long)n,
                    (long long)lat->L.n);
    return LPC_OK;
}

// Host doubles -> device field through the staging chunk, converted by a kernel.
lpc_status upload_field(lpc_lattice *lat, const double *src, void *dst, double scale)
{
    const int64_t n = lat->L.n, chunk = lat->L.staging;
    const size_t es = lat->L.storage;
    for (int64_t o = 0; o < n; o += chunk) {
        const int64_t c = n - o < chunk ? n - o : chunk;
        LPC_HIP(hipMemcpyAsync(lat->staging(), src + o, size_t(c) * 8, hipMemcpyHostToDevice,
                               lat->stream));
        LPC_HIP(lpc::launch_store_field(lat->cfg.precision, lat->staging(),
                                        static_cast<char *>(dst) + size_t(o) * es, c, scale,
                                        lat->stream));
    }
    LPC_HIP(hipStreamSynchronize(lat->stream));
    return LPC_OK;
}

lpc_status sync(lpc_lattice *lat)
{
    LPC_HIP(hipStreamSynchronize(lat->stream));
    return LPC_OK;
}

lpc_status fetch_records(lpc_lattice *lat, std::vector<double> &rec)
{
    if (!lat->initialized)
        return fail(LPC_ERR_STATE, "state not initialised");
    if (lpc_status s = sync(lat))
        return s;
    const int64_t rows = lat->steps_done + 1;
    rec.resize(size_t(rows) * lat->L.K);
    LPC_HIP(copy_sync(lat, rec.data(), lat->records(), rec.size() * 8, hipMemcpyDeviceToHost));
    return LPC_OK;
}

lpc_status health(const lpc_lattice *lat, const std::vector<double> &rec)
{
    const int K = lat->L.K, R = lat->cfg.n_regions;
    const int64_t rows = int64_t(rec.size()) / K;
    double m0 = 0.0;
    for (int r = 0; r < R; ++r)
        m0 += rec[2 * R + r];
    for (int64_t t = 0; t < rows; ++t) {
        const double *row = rec.data() + t * K;
        double mass = 0.0;
        for (int r = 0; r < R; ++r) {
            if (!std::isfinite(row[2 * r]) || !std::isfinite(row[2 * r + 1]))
                return fail(LPC_ERR_NONFINITE, "FID is not finite at step %lld", (long long)t);
            mass += row[2 * R + r];
        }
        if (!std::isfinite(mass))
            return fail(LPC_ERR_NONFINITE, "total population is not finite at step %lld",
                        (long long)t);
        // reservoir faces exchange matter with the lattice: no conservation to check
        const double tol = reservoir_of(lat->cfg) ? 0.0 : lat->cfg.conservation_tol;
        if (tol > 0.0 && m0 != 0.0 && std::fabs(mass - m0) > tol * std::fabs(m0))
            return fail(LPC_ERR_CONSERVATION,
                        "total population drifted by %.3e (relative) at step %lld, tolerance %.1e",
                        std::fabs(mass - m0) / std::fabs(m0), (long long)t, tol);
    }
    return LPC_OK;
}

lpc_status write_initial_record(lpc_lattice *lat)
{
    lpc::StepArgs a = lat->args(lat->cur);
    LPC_HIP(lpc::launch_record(lat->L.plan, a, lat->stream));
    LPC_HIP(lpc::launch_finalize(lat->partials(), lat->L.plan.nblocks, lat->L.K, 1, lat->records(),
                                 lat->stream));
    return LPC_OK;
}

struct SaveHeader {
    char magic[8];
    uint32_t version;
    int32_t n[3];
    int32_t precision;
    uint32_t track;
    int32_t n_regions;
    int32_t pad;
    int64_t steps_done;
    int64_t rows;
};

size_t state_bytes(const lpc_lattice *lat)
{
    const int64_t n = lat->L.n;
    size_t b = size_t(n) * 8;
    if (fid_of(lat->cfg))
        b += 2 * size_t(n) * lat->L.storage;
    if (msd_of(lat->cfg))
        b += 6 * size_t(n) * lat->L.storage;
    if (vacf_of(lat->cfg))
        b += 3 * size_t(n) * lat->L.storage;
    return b;
}

}  // namespace

extern "C" {

lpc_status lpc_config_default(lpc_config *cfg, int32_t n)
{
    if (!cfg)
        return fail(LPC_ERR_ARG, "config is NULL");
    std::memset(cfg, 0, sizeof *cfg);
    for (int a = 0; a < 3; ++a) {
        cfg->n[a] = n;
        cfg->bc[a] = LPC_BC_PERIODIC;
    }
    cfg->precision = LPC_PREC_FP64;
    cfg->track = LPC_TRACK_FID | LPC_TRACK_MSD;
    cfg->n_regions = 1;
    cfg->p_hop = 1.0 / 7.0;
    cfg->dt_s = 5e-6;
    cfg->larmor_hz = 400e6;
    cfg->spacing_m = 0.5e-9;
    cfg->max_records = 1;
    cfg->conservation_tol = 1e-12;
    return ok();
}

lpc_status lpc_query_footprint(const lpc_config *cfg, size_t *bytes)
{
    if (lpc_status s = validate_config(cfg))
        return s;
    if (!bytes)
        return fail(LPC_ERR_ARG, "bytes is NULL");
    *bytes = plan_layout(*cfg).total;
    return ok();
}

lpc_status lpc_query_linear_tiles(const lpc_config *cfg, int32_t *max_nx)
{
    if (lpc_status s = validate_config(cfg))
        return s;
    if (!max_nx)
        return fail(LPC_ERR_ARG, "max_nx is NULL");
    *max_nx = lpc::linear_tile_max_nx(cfg->precision, variant_of(*cfg));
    return ok();
}

lpc_status lpc_create(const lpc_config *cfg, void *arena, size_t arena_bytes, void *stream,
                      lpc_lattice **out)
{
    if (lpc_status s = validate_config(cfg))
        return s;
    if (!arena || !out)
        return fail(LPC_ERR_ARG, "arena and out must not be NULL");
    if (reinterpret_cast<uintptr_t>(arena) % kAlign)
        return fail(LPC_ERR_ARG, "arena must be %zu-byte aligned", kAlign);
    Layout L = plan_layout(*cfg);
    if (arena_bytes < L.total)
        return fail(LPC_ERR_OOM, "arena has %zu bytes, lattice needs %zu", arena_bytes, L.total);
    auto *lat = new (std::nothrow) lpc_lattice;
    if (!lat)
        return fail(LPC_ERR_OOM, "host allocation failed");
    lat->cfg = *cfg;
    lat->L = L;
    lat->stream = static_cast<hipStream_t>(stream);
    lat->arena = static_cast<char *>(arena);
    int cus = 0;
    if (hipGetDevice(&lat->device) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, lat->device) !=
            hipSuccess) {
        delete lat;
        return fail(LPC_ERR_DEVICE, "device query failed");
    }
    {
        lpc::Geometry g{cfg->n[0], cfg->n[1], cfg->n[2], {cfg->bc[0], cfg->bc[1], cfg->bc[2]}};
        const int occ = lpc::sweep_blocks_per_cu(cfg->precision, variant_of(*cfg), cfg->n_regions);
        lat->occupancy = occ;
        lat->cus = cus;
        lat->L.plan = lpc::make_plan(g, occ, cus, 0,
                                     lpc::linear_tile_max_nx(cfg->precision, variant_of(*cfg)),
                                     zc_floor(*cfg));
        const uint32_t pop =
            variant_of(*cfg) & ~uint32_t(LPC_TRACK_FID | LPC_TRACK_MSD | LPC_TRACK_VACF);
        lat->eq_plan = lpc::make_plan(g, lpc::sweep_blocks_per_cu(cfg->precision, pop,
                                                                 cfg->n_regions),
                                      cus, 0, lpc::linear_tile_max_nx(cfg->precision, pop),
                                      zc_floor(*cfg));
        set_chunk(lat->L);
        if (two_step_available(*cfg)) {
            lat->occupancy2 = lpc::sweep_blocks_per_cu(cfg->precision, variant_of(*cfg),
                                                       cfg->n_regions, 2);
            lat->plan2 = lpc::make_plan2(g, lat->occupancy2, cus, zc_floor(*cfg));
            lat->chunk2 = two_step_chunk(lat->L, lat->plan2);
        }
    }
    for (int b = 0; b < 2; ++b) {
        lpc::StateView &v = lat->st[b];
        v.rho = lat->at<double>(L.off_rho[b]);
        v.re = fid_of(*cfg) ? lat->at(L.off_re[b]) : nullptr;
        v.im = fid_of(*cfg) ? lat->at(L.off_im[b]) : nullptr;
        for (int a = 0; a < 3; ++a) {
            v.m1[a] = msd_of(*cfg) ? lat->at(L.off_m1[b][a]) : nullptr;
            v.m2[a] = msd_of(*cfg) ? lat->at(L.off_m2[b][a]) : nullptr;
            v.v[a] = vacf_of(*cfg) ? lat->at(L.off_v[b][a]) : nullptr;
        }
    }
    const size_t ns = size_t(L.n) * L.storage;
    const SoloTables tables = solo_tables(lat);
    hipError_t e = copy_sync(lat, lat->solo(), &tables, sizeof tables, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemsetAsync(lat->at(L.off_F), 0, ns, lat->stream);
    if (e == hipSuccess && cfg->precision == LPC_PREC_FP64)   // e^{0 - 0} of the cleared field
        e = lpc::launch_fill_field(cfg->precision, lat->at(L.off_E), L.n, 1.0, lat->stream);
    if (e == hipSuccess && fid_of(*cfg))
        e = hipMemsetAsync(lat->at(L.off_theta), 0, ns, lat->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(lat->at(L.off_region), 0, size_t(L.n), lat->stream);
    if (e == hipSuccess && mobility_of(*cfg))
        e = lpc::launch_fill_field(cfg->precision, lat->at(L.off_mu), L.n, 1.0, lat->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(lat->at(L.off_ghost), lat->ghost, sizeof lat->ghost,
                           hipMemcpyHostToDevice, lat->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(lat->stream);
    lat->n_open = L.n;
    if (e != hipSuccess) {
        delete lat;
        return fail(LPC_ERR_DEVICE, "clearing fields failed: %s", hipGetErrorString(e));
    }
    *out = lat;
    return ok();
}

lpc_status lpc_destroy(lpc_lattice *lat)
{
    if (!lat)
        return fail(LPC_ERR_ARG, "lattice is NULL");
    (void)hipStreamSynchronize(lat->stream);
    delete lat;
    return ok();
}

lpc_status lpc_set_free_energy(lpc_lattice *lat, const double *F_kT, int64_t n)
{
    if (!lat)
        return fail(LPC_ERR_ARG, "lattice is NULL");
    if (lpc_status s = check_sites(lat, F_kT, n))
        return s;
    // +inf marks the solid matrix: stored as a finite sentinel beyond every accepted value
    const double blocked =
        lat->cfg.precision == LPC_PREC_FP64 ? lpc::kBlockedF64 : lpc::kBlockedF32;
    std::vector<double> host;
    double fmin = INFINITY, fmax = -INFINITY;
    int64_t open = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double f = F_kT[i];
        if (std::isinf(f) && f > 0.0) {
            if (host.empty())
                host.assign(F_kT, F_kT + n);
            host[size_t(i)] = blocked;
            continue;
        }
        if (!std::isfinite(f))
            return fail(LPC_ERR_NONFINITE, "F[%lld] is NaN or -Inf", (long long)i);
        if (std::fabs(f) > kMaxFreeEnergy)
            return fail(LPC_ERR_ARG, "|F[%lld]| = %g exceeds %g kT", (long long)i, std::fabs(f),
                        kMaxFreeEnergy);
        fmin = f < fmin ? f : fmin;
        fmax = f > fmax ? f : fmax;
        ++open;
    }
    // the FP64 sweep works with e^{+-(F - centre)}, which must stay finite
    if (open > 0 && fmax - fmin > kMaxFreeEnergySpan)
        return fail(LPC_ERR_ARG, "accessible free energies span %g kT, more than %g", fmax - fmin,
                    kMaxFreeEnergySpan);
    if (lpc_status s = use_device(lat))
        return s;
    if (lpc_status s = upload_field(lat, host.empty() ? F_kT : host.data(),
                                    lat->at(lat->L.off_F), 1.0))
        return s;
    lat->Fmin = open > 0 ? fmin : 0.0;
    lat->Fmid = open > 0 ? 0.5 * (fmin + fmax) : 0.0;
    lat->n_open = open;
    if (lat->cfg.precision == LPC_PREC_FP64) {
        LPC_HIP(lpc::launch_boltzmann_factors(lat->at<double>(lat->L.off_F),
                                              lat->at<double>(lat->L.off_E), lat->L.n, lat->Fmid,
                                              lat->stream));
        if (lpc_status s = sync(lat))
            return s;
    }
    if (lpc_status s = upload_solo(lat))
        return s;
    return ok();
}

lpc_status lpc_set_shift(lpc_lattice *lat, const double *delta_ppm, int64_t n)
{
    if (!lat)
        return fail(LPC_ERR_ARG, "lattice is NULL");
    if (lpc_status s = check_sites(lat, delta_ppm, n))
        return s;
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(delta_ppm[i]))
            return fail(LPC_ERR_NONFINITE, "delta[%lld] is not finite", (long long)i);
    if (!fid_of(lat->cfg))
        return ok();  // no magnetisation tracked: the shift is not used
    if (lpc_status s = use_device(lat))
        return s;
    // phase per step of Eq. (11): theta = 2 pi delta 1e-6 nu0 dt
    const double scale = 2.0 * M_PI * 1e-6 * lat->cfg.larmor_hz * lat->cfg.dt_s;
    return upload_field(lat, delta_ppm, lat->at(lat->L.off_theta), scale);
}

lpc_status lpc_set_regions(lpc_lattice *lat, const uint8_t *region, int64_t n)
{
    if (!lat)
        return fail(LPC_ERR_ARG, "lattice is NULL");
    if (lpc_status s = check_sites(lat, region, n))
        return s;
    for (int64_t i = 0; i < n; ++i)
        if (region[i] >= lat->cfg.n_regions)
            return fail(LPC_ERR_ARG, "region[%lld] = %d is not below n_regions = %d", (long long)i,
                        int(region[i]), lat->cfg.n_regions);
    if (lpc_status s = use_device(lat))
        return s;
    LPC_HIP(hipMemcpyAsync(lat->at(lat->L.off_region), region, size_t(n), hipMemcpyHostToDevice,
                           lat->stream));
    return sync(lat);
}

lpc_status lpc_set_mobility(lpc_lattice *lat, const double *mu, int64_t n)
{
    if (!lat)
        return fail(LPC_ERR_ARG, "lattice is NULL");
    if (!mobility_of(lat->cfg))
        return fail(LPC_ERR_STATE, "the lattice was created without LPC_OPT_MOBILITY");
    if (lpc_status s = check_sites(lat, mu, n))
        return s;
    for (int64_t i = 0; i < n; ++i) {
        if (std::isnan(mu[i]))
            return fail(LPC_ERR_NONFINITE, "mu[%lld] is NaN", (long long)i);
        if (!(mu[i] >= 0.0 && mu[i] <= 1.0))
            return fail(LPC_ERR_ARG, "mu[%lld] = %g is outside [0, 1]", (long long)i, mu[i]);
    }
    if (lpc_status s = use_device(lat))
        return s;
    return upload_field(lat, mu, lat->at(lat->L.off_mu), 1.0);
}

lpc_status lpc_set_reservoir(lpc_lattice *lat, int32_t axis, int32_t side, double F_kT,
                             double rho, double m_re, double m_im)
{
    if (!lat)
        return fail(LPC_ERR_ARG, "lattice is NULL");
    if (axis < 0 || axis > 2 || side < 0 || side > 1)
        return fail(LPC_ERR_ARG, "axis %d / side %d out of range", axis, side);
    if (lat->cfg.bc[axis] != LPC_BC_RESERVOIR)
        return fail(LPC_ERR_STATE, "axis %d is not a reservoir axis", axis);
    if (!std::isfinite(F_kT) || !std::isfinite(rho) || !std::isfinite(m_re) ||
        !std::isfinite(m_im))
        return fail(LPC_ERR_NONFINITE, "reservoir values must be finite");
    if (std::fabs(F_kT) > kMaxFreeEnergy || rho < 0.0)
        return fail(LPC_ERR_ARG, "need |F| <= %g kT and rho >= 0", kMaxFreeEnergy);
    if (lpc_status s = use_device(lat))
        return s;
    double *g = lat->ghost + 4 * (2 * axis + side);
    g[0] = F_kT;
    g[1] = rho;
    g[2] = m_re;
    g[3] = m_im;
    // stream-ordered after the queued steps; the host table outlives the copy (synchronised)
    LPC_HIP(hipMemcpyAsync(lat->at(lat->L.off_ghost), lat->ghost, sizeof lat->ghost,
                           hipMemcpyHostToDevice, lat->stream));
    return sync(lat);
}

lpc_status lpc_init_state(lpc_lattice *lat, int32_t mode, const double *rho, int64_t n)
{
    if (!lat)
        return fail(LPC_ERR_ARG, "lattice is NULL");
    if (mode != LPC_INIT_UNIFORM && mode != LPC_INIT_BOLTZMANN && mode != LPC_INIT_USER)
        return fail(LPC_ERR_ARG, "init mode %d unknown", mode);
    if (mode == LPC_INIT_USER) {
        if (lpc_status s = check_sites(lat, rho, n))
            return s;
        for (int64_t i = 0; i < n; ++i)
            if (!std::isfinite(rho[i]))
                return fail(LPC_ERR_NONFINITE, "rho[%lld] is not finite", (long long)i);
    }
    if (lpc_status s = use_device(lat))
        return s;
    if (lpc_status s = sync(lat))
        return s;
    lat->cur = 0;
    const lpc::StateView &st = lat->st[0];
    const int64_t N = lat->L.n;
    const void *F = lat->at(lat->L.off_F);
    if (mode == LPC_INIT_UNIFORM || (mode == LPC_INIT_BOLTZMANN && lat->n_open == 0)) {
        LPC_HIP(lpc::launch_init_state(lat->cfg.precision, lat->cfg.track, st, nullptr, F, N,
                                       lat->stream));
    } else if (mode == LPC_INIT_BOLTZMANN) {
        // Eq. (2): rho_i = N_open exp(-F_i) / sum_j exp(-F_j); weights relative to min F
        // (inaccessible sites weigh exp(-huge) = 0)
        int64_t nb = 0;
        LPC_HIP(lpc::launch_boltzmann_weights(lat->cfg.precision, F, lat->Fmin, st.rho, N,
                                              lat->partials(), &nb, lat->stream));
        LPC_HIP(lpc::launch_finalize(lat->partials(), nb, 1, 1, lat->scalars(), lat->stream));
        LPC_HIP(lpc::launch_boltzmann_scale(st.rho, N, double(lat->n_open), lat->scalars(),
                                            lat->stream));
        LPC_HIP(lpc::launch_init_state(lat->cfg.precision, lat->cfg.track, st, st.rho, F, N,
                                       lat->stream));
    } else {
        LPC_HIP(hipMemcpyAsync(st.rho, rho, size_t(N) * 8, hipMemcpyHostToDevice, lat->stream));
        LPC_HIP(lpc::launch_init_state(lat->cfg.precision, lat->cfg.track, st, st.rho, F, N,
                                       lat->stream));
    }
    lat->steps_done = 0;
    if (lpc_status s = write_initial_record(lat))
        return s;
    if (lpc_status s = sync(lat))
        return s;
    lat->initialized = true;
    return ok();
}

}  // extern "C"

namespace {

// Queues n_steps steps of a lattice alone on stream s (its own stream, or a batch's), with
// the finalisation of their records. The first step after a start sets the autocorrelation
// tags (lattices that track them).
lpc_status queue_steps(lpc_lattice *lat, int64_t n_steps, hipStream_t stream)
{
    SoloTables *t = lat->solo();
    int64_t left = n_steps;
    if (lat->steps_per_pass == 2) {
        // pairs of steps, one two-step pass each; an odd last step takes a one-step pass
        lpc::StepList list2{&t->item2, t->prefix2, 1, lpc::kTileTwoStep, lat->plan2.nblocks, 0, 0};
        while (left >= 2) {
            const int64_t c = std::min(left - left % 2, lat->chunk2);
            for (int64_t s = 0; s < c; s += 2) {
                list2.parity = lat->cur;
                list2.slot = s;
                LPC_HIP(lpc::launch_step_list(list2, lat->cfg.precision, variant_of(lat->cfg),
                                              lat->cfg.n_regions, stream));
                lat->cur ^= 1;
            }
            LPC_HIP(lpc::launch_finalize_list(&t->fin2, t->kprefix, 1, lat->L.K, c,
                                              lat->steps_done + 1, stream));
            lat->steps_done += c;
            left -= c;
        }
    }
    const bool tags = vacf_of(lat->cfg);
    lpc::StepList list{&t->item, t->prefix, 1, lat->L.plan.tx, lat->L.plan.nblocks, 0, 0};
    while (left > 0) {
        const int64_t c = left < lat->L.chunk ? left : lat->L.chunk;
        for (int64_t s = 0; s < c; ++s) {
            list.items = tags && lat->steps_done + s == 0 ? &t->item_tag : &t->item;
            list.parity = lat->cur;
            list.slot = s;
            LPC_HIP(lpc::launch_step_list(list, lat->cfg.precision, variant_of(lat->cfg),
                                          lat->cfg.n_regions, stream));
            lat->cur ^= 1;
        }
        LPC_HIP(lpc::launch_finalize_list(&t->fin, t->kprefix, 1, lat->L.K, c,
                                          lat->steps_done + 1, stream));
        lat->steps_done += c;
        left -= c;
    }
    return LPC_OK;
}

}  // namespace

extern "C" {

lpc_status lpc_run(lpc_lattice *lat, int64_t n_steps)
{
    if (!lat)
        return fail(LPC_ERR_ARG, "lattice is NULL");
    if (n_steps < 0)
        return fail(LPC_ERR_ARG, "n_steps = %lld is negative", (long long)n_steps);
    if (!lat->initialized)
        return fail(LPC_ERR_STATE, "lpc_init_state or lpc_load_state must come first");
    if (lat->steps_done + n_steps > lat->cfg.max_records - 1)
        return fail(LPC_ERR_STATE, "records hold %lld steps; %lld done, %lld requested",
                    (long long)(lat->cfg.max_records - 1), (long long)lat->steps_done,
                    (long long)n_steps);
    if (lpc_status s = use_device(lat))
        return s;
    return queue_steps(lat, n_steps, lat->stream);
}

lpc_status lpc_equilibrate(lpc_lattice *lat, int64_t max_steps, double tol, int64_t check_every,
                           int64_t *steps_taken, double *residual)
{
    if (!lat)
        return fail(LPC_ERR_ARG, "lattice is NULL");
    if (max_steps < 0 || check_every < 1 || !std::isfinite(tol) || tol < 0.0)
        return fail(LPC_ERR_ARG, "need max_steps >= 0, check_every >= 1, finite tol >= 0");
    if (!lat->initialized)
        return fail(LPC_ERR_STATE, "lpc_init_state or lpc_load_state must come first");
    if (lpc_status s = use_device(lat))
        return s;
    SoloTables *t = lat->solo();
    lpc::StepList list{&t->eq_item, t->eq_prefix, 1, lat->eq_plan.tx, lat->eq_plan.nblocks, 0,
                       0};
    // workgroup maxima in the per-step partial sums (population-only steps discard theirs,
    // and stream order puts each check between the steps): enough workgroups to stream
    // both population buffers at full bandwidth
    constexpr int32_t kChangeParts = 1024;
    static_assert(kChangeParts * 16 <= kPartialBudget, "change partials exceed the buffer");
    double *part = lat->partials();
    double *out = lat->scalars() + 8;
    int64_t done = 0;
    double change[2] = {INFINITY, 1.0};
    while (done < max_steps) {
        const int64_t c = std::min(check_every, max_steps - done);
        for (int64_t s = 0; s < c; ++s) {
            list.parity = lat->cur;
            LPC_HIP(lpc::launch_step_list(list, lat->cfg.precision,
                                          variant_of(lat->cfg) &
                                              ~uint32_t(LPC_TRACK_FID | LPC_TRACK_MSD |
                                                        LPC_TRACK_VACF),
                                          lat->cfg.n_regions, lat->stream));
            lat->cur ^= 1;
        }
        done += c;
        LPC_HIP(lpc::launch_max_change(lat->st[1 - lat->cur].rho, lat->st[lat->cur].rho,
                                       lat->L.n, part, kChangeParts, out, lat->stream));
        if (lpc_status s = sync(lat))
            return s;
        LPC_HIP(copy_sync(lat, change, out, 16, hipMemcpyDeviceToHost));
        if (!std::isfinite(change[0]) || !std::isfinite(change[1]))
            return fail(LPC_ERR_NONFINITE, "populations are not finite after %lld steps",
                        (long long)done);
        if (change[1] > 0.0 ? change[0] <= tol * change[1] : change[0] <= tol)
            break;
    }
    // restart the propagation from the equilibrated populations
    const lpc::StateView &st = lat->st[lat->cur];
    LPC_HIP(lpc::launch_init_state(lat->cfg.precision, lat->cfg.track, st, st.rho,
                                   lat->at(lat->L.off_F), lat->L.n,
                                   lat->stream));
    lat->steps_done = 0;
    if (lpc_status s = write_initial_record(lat))
        return s;
    if (lpc_status s = sync(lat))
        return s;
    if (steps_taken)
        *steps_taken = done;
    if (residual)
        *residual = change[1] > 0.0 ? change[0] / change[1] : change[0];
    return ok();
}

lpc_status lpc_synchronize(lpc_lattice *lat)
{
    if (!lat)
        return fail(LPC_ERR_ARG, "lattice is NULL");
    return sync(lat);
}

lpc_status lpc_steps_done(const lpc_lattice *lat, int64_t *n)
{
    if (!lat || !n)
        return fail(LPC_ERR_ARG, "NULL argument");
    *n = lat->steps_done;
    return ok();
}

lpc_status lpc_record_width(const lpc_lattice *lat, int32_t *K)
{
    if (!lat || !K)
        return fail(LPC_ERR_ARG, "NULL argument");
    *K = lat->L.K;
    return ok();
}

lpc_status lpc_read_records(lpc_lattice *lat, double *records, int64_t cap_rows, int64_t *rows)
{
    if (!lat || !records || !rows)
        return fail(LPC_ERR_ARG, "NULL argument");
    std::vector<double> rec;
    if (lpc_status s = fetch_records(lat, rec))
        return s;
    const int64_t r = lat->steps_done + 1;
    if (cap_rows < r)
        return fail(LPC_ERR_OOM, "records need %lld rows, buffer has %lld", (long long)r,
                    (long long)cap_rows);
    std::memcpy(records, rec.data(), rec.size() * 8);
    *rows = r;
    return ok();
}

lpc_status lpc_read_population(lpc_lattice *lat, double *rho, int64_t n)
{
    if (!lat)
        return fail(LPC_ERR_ARG, "lattice is NULL");
    if (lpc_status s = check_sites(lat, rho, n))
        return s;
    if (!lat->initialized)
        return fail(LPC_ERR_STATE, "state not initialised");
    if (lpc_status s = sync(lat))
        return s;
    LPC_HIP(copy_sync(lat, rho, lat->st[lat->cur].rho, size_t(n) * 8, hipMemcpyDeviceToHost));
    return ok();
}

lpc_status lpc_read_magnetization(lpc_lattice *lat, double *re, double *im, int64_t n)
{
    if (!lat)
        return fail(LPC_ERR_ARG, "lattice is NULL");
    if (lpc_status s = check_sites(lat, re, n))
        return s;
    if (lpc_status s = check_sites(lat, im, n))
        return s;
    if (!fid_of(lat->cfg))
        return fail(LPC_ERR_STATE, "magnetisation is not tracked");
    if (!lat->initialized)
        return fail(LPC_ERR_STATE, "state not initialised");
    if (lpc_status s = sync(lat))
        return s;
    const lpc::StateView &v = lat->st[lat->cur];
    if (lat->L.storage == 8) {
        LPC_HIP(copy_sync(lat, re, v.re, size_t(n) * 8, hipMemcpyDeviceToHost));
        LPC_HIP(copy_sync(lat, im, v.im, size_t(n) * 8, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(static_cast<size_t>(n));
        LPC_HIP(copy_sync(lat, tmp.data(), v.re, size_t(n) * 4, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i)
            re[i] = tmp[size_t(i)];
        LPC_HIP(copy_sync(lat, tmp.data(), v.im, size_t(n) * 4, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i)
            im[i] = tmp[size_t(i)];
    }
    return ok();
}

lpc_status lpc_check(lpc_lattice *lat)
{
    if (!lat)
        return fail(LPC_ERR_ARG, "lattice is NULL");
    std::vector<double> rec;
    if (lpc_status s = fetch_records(lat, rec))
        return s;
    return health(lat, rec);
}

lpc_status lpc_read_fid(lpc_lattice *lat, int32_t region, double *re, double *im, int64_t cap,
                        int64_t *len)
{
    if (!lat || !re || !im || !len)
        return fail(LPC_ERR_ARG, "NULL argument");
    const int R = lat->cfg.n_regions;
    if (region < -1 || region >= R)
        return fail(LPC_ERR_ARG, "region %d outside -1..%d", region, R - 1);
    std::vector<double> rec;
    if (lpc_status s = fetch_records(lat, rec))
        return s;
    if (lpc_status s = health(lat, rec))
        return s;
    const int64_t rows = lat->steps_done + 1;
    if (cap < rows)
        return fail(LPC_ERR_OOM, "FID has %lld samples, buffer holds %lld", (long long)rows,
                    (long long)cap);
    const int K = lat->L.K;
    for (int64_t t = 0; t < rows; ++t) {
        const double *row = rec.data() + t * K;
        double a = 0.0, b = 0.0;
        for (int r = 0; r < R; ++r) {
            if (region >= 0 && r != region)
                continue;
            a += row[2 * r];
            b += row[2 * r + 1];
        }
        re[t] = a;
        im[t] = b;
    }
    *len = rows;
    return ok();
}

lpc_status lpc_read_moments(lpc_lattice *lat, double *mass, double *msd_xyz, double *drift_xyz,
                            int64_t cap, int64_t *len)
{
    if (!lat || !mass || !msd_xyz || !drift_xyz || !len)
        return fail(LPC_ERR_ARG, "NULL argument");
    std::vector<double> rec;
    if (lpc_status s = fetch_records(lat, rec))
        return s;
    if (lpc_status s = health(lat, rec))
        return s;
    const int64_t rows = lat->steps_done + 1;
    if (cap < rows)
        return fail(LPC_ERR_OOM, "moments have %lld rows, buffer holds %lld", (long long)rows,
                    (long long)cap);
    const int K = lat->L.K, R = lat->cfg.n_regions;
    for (int64_t t = 0; t < rows; ++t) {
        const double *row = rec.data() + t * K;
        double m = 0.0;
        for (int r = 0; r < R; ++r)
            m += row[2 * R + r];
        mass[t] = m;
        for (int a = 0; a < 3; ++a) {
            drift_xyz[3 * t + a] = row[3 * R + a] / m;
            msd_xyz[3 * t + a] = row[3 * R + 3 + a] / m;
        }
    }
    *len = rows;
    return ok();
}

lpc_status lpc_read_uptake(lpc_lattice *lat, double *per_step_per_region, int64_t cap,
                           int64_t *len)
{
    if (!lat || !per_step_per_region || !len)
        return fail(LPC_ERR_ARG, "NULL argument");
    std::vector<double> rec;
    if (lpc_status s = fetch_records(lat, rec))
        return s;
    if (lpc_status s = health(lat, rec))
        return s;
    const int64_t rows = lat->steps_done + 1;
    if (cap < rows)
        return fail(LPC_ERR_OOM, "uptake has %lld rows, buffer holds %lld", (long long)rows,
                    (long long)cap);
    const int K = lat->L.K, R = lat->cfg.n_regions;
    for (int64_t t = 0; t < rows; ++t)
        for (int r = 0; r < R; ++r)
            per_step_per_region[t * R + r] = rec[size_t(t * K + 2 * R + r)];
    *len = rows;
    return ok();
}

lpc_status lpc_save_state(lpc_lattice *lat, void *buf, size_t cap, size_t *len)
{
    if (!lat || !len)
        return fail(LPC_ERR_ARG, "NULL argument");
    if (!lat->initialized)
        return fail(LPC_ERR_STATE, "state not initialised");
    const int64_t rows = lat->steps_done + 1;
    const size_t need = sizeof(SaveHeader) + state_bytes(lat) + size_t(rows) * lat->L.K * 8;
    if (!buf) {
        *len = need;
        return ok();
    }
    if (cap < need)
        return fail(LPC_ERR_OOM, "checkpoint needs %zu bytes, buffer has %zu", need, cap);
    if (lpc_status s = sync(lat))
        return s;
    SaveHeader h{};
    std::memcpy(h.magic, "LPCSTATE", 8);
    h.version = 1;
    for (int a = 0; a < 3; ++a)
        h.n[a] = lat->cfg.n[a];
    h.precision = lat->cfg.precision;
    h.track = lat->cfg.track;
    h.n_regions = lat->cfg.n_regions;
    h.steps_done = lat->steps_done;
    h.rows = rows;
    char *p = static_cast<char *>(buf);
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    const lpc::StateView &v = lat->st[lat->cur];
    const size_t n = size_t(lat->L.n), ns = n * lat->L.storage;
    LPC_HIP(copy_sync(lat, p, v.rho, n * 8, hipMemcpyDeviceToHost));
    p += n * 8;
    if (fid_of(lat->cfg)) {
        LPC_HIP(copy_sync(lat, p, v.re, ns, hipMemcpyDeviceToHost));
        p += ns;
        LPC_HIP(copy_sync(lat, p, v.im, ns, hipMemcpyDeviceToHost));
        p += ns;
    }
    if (msd_of(lat->cfg)) {
        for (int a = 0; a < 3; ++a) {
            LPC_HIP(copy_sync(lat, p, v.m1[a], ns, hipMemcpyDeviceToHost));
            p += ns;
        }
        for (int a = 0; a < 3; ++a) {
            LPC_HIP(copy_sync(lat, p, v.m2[a], ns, hipMemcpyDeviceToHost));
            p += ns;
        }
    }
    if (vacf_of(lat->cfg)) {
        for (int a = 0; a < 3; ++a) {
            LPC_HIP(copy_sync(lat, p, v.v[a], ns, hipMemcpyDeviceToHost));
            p += ns;
        }
    }
    LPC_HIP(copy_sync(lat, p, lat->records(), size_t(rows) * lat->L.K * 8, hipMemcpyDeviceToHost));
    *len = need;
    return ok();
}

lpc_status lpc_load_state(lpc_lattice *lat, const void *buf, size_t len)
{
    if (!lat || !buf)
        return fail(LPC_ERR_ARG, "NULL argument");
    if (len < sizeof(SaveHeader))
        return fail(LPC_ERR_ARG, "checkpoint too short");
    SaveHeader h;
    std::memcpy(&h, buf, sizeof h);
    if (std::memcmp(h.magic, "LPCSTATE", 8) != 0 || h.version != 1)
        return fail(LPC_ERR_ARG, "not a version-1 lattice checkpoint");
    for (int a = 0; a < 3; ++a)
        if (h.n[a] != lat->cfg.n[a])
            return fail(LPC_ERR_ARG, "checkpoint shape differs from the lattice");
    if (h.precision != lat->cfg.precision || h.track != lat->cfg.track ||
        h.n_regions != lat->cfg.n_regions)
        return fail(LPC_ERR_ARG, "checkpoint precision, track set or regions differ");
    if (h.rows != h.steps_done + 1 || h.rows < 1 || h.rows > lat->cfg.max_records)
        return fail(LPC_ERR_STATE, "checkpoint holds %lld records, lattice keeps %lld",
                    (long long)h.rows, (long long)lat->cfg.max_records);
    const size_t need = sizeof(SaveHeader) + state_bytes(lat) + size_t(h.rows) * lat->L.K * 8;
    if (len < need)
        return fail(LPC_ERR_ARG, "checkpoint has %zu bytes, needs %zu", len, need);
    if (lpc_status s = use_device(lat))
        return s;
    if (lpc_status s = sync(lat))
        return s;
    const char *p = static_cast<const char *>(buf) + sizeof h;
    lat->cur = 0;
    const lpc::StateView &v = lat->st[0];
    const size_t n = size_t(lat->L.n), ns = n * lat->L.storage;
    LPC_HIP(copy_sync(lat, v.rho, p, n * 8, hipMemcpyHostToDevice));
    p += n * 8;
    if (fid_of(lat->cfg)) {
        LPC_HIP(copy_sync(lat, v.re, p, ns, hipMemcpyHostToDevice));
        p += ns;
        LPC_HIP(copy_sync(lat, v.im, p, ns, hipMemcpyHostToDevice));
        p += ns;
    }
    if (msd_of(lat->cfg)) {
        for (int a = 0; a < 3; ++a) {
            LPC_HIP(copy_sync(lat, v.m1[a], p, ns, hipMemcpyHostToDevice));
            p += ns;
        }
        for (int a = 0; a < 3; ++a) {
            LPC_HIP(copy_sync(lat, v.m2[a], p, ns, hipMemcpyHostToDevice));
            p += ns;
        }
    }
    if (vacf_of(lat->cfg)) {
        for (int a = 0; a < 3; ++a) {
            LPC_HIP(copy_sync(lat, v.v[a], p, ns, hipMemcpyHostToDevice));
            p += ns;
        }
    }
    LPC_HIP(copy_sync(lat, lat->records(), p, size_t(h.rows) * lat->L.K * 8, hipMemcpyHostToDevice));
    lat->steps_done = h.steps_done;
    lat->initialized = true;
    return ok();
}

lpc_status lpc_spectrum_length(const lpc_lattice *lat, int64_t *n_fft)
{
    if (!lat || !n_fft)
        return fail(LPC_ERR_ARG, "NULL argument");
    if (!fid_of(lat->cfg))
        return fail(LPC_ERR_STATE, "magnetisation is not tracked");
    *n_fft = fft_length(lat->steps_done + 1);
    return ok();
}

namespace {

// Runs the spectrum of `region` on the device; leaves the sorted real/imaginary parts in
// device memory at *sorted (2 L doubles).
lpc_status device_spectrum(lpc_lattice *lat, int32_t region, int64_t L, double **sorted)
{
    if (!fid_of(lat->cfg))
        return fail(LPC_ERR_STATE, "magnetisation is not tracked");
    if (!lat->initialized)
        return fail(LPC_ERR_STATE, "state not initialised");
    const int R = lat->cfg.n_regions;
    if (region < -1 || region >= R)
        return fail(LPC_ERR_ARG, "region %d outside -1..%d", region, R - 1);
    const int64_t rows = lat->steps_done + 1;
    if (L < rows || (L & (L - 1)) != 0 || L > lat->L.fft_max)
        return fail(LPC_ERR_ARG,
                    "n_fft = %lld must be a power of two >= %lld samples and <= %lld",
                    (long long)L, (long long)rows, (long long)lat->L.fft_max);
    std::vector<double> row0(size_t(lat->L.K));
    if (lpc_status s = sync(lat))
        return s;
    LPC_HIP(copy_sync(lat, row0.data(), lat->records(), row0.size() * 8, hipMemcpyDeviceToHost));
    double c = 0.0, d = 0.0;
    for (int r = 0; r < R; ++r)
        if (region < 0 || r == region) {
            c += row0[2 * r];
            d += row0[2 * r + 1];
        }
    if (c == 0.0 && d == 0.0)
        return fail(LPC_ERR_STATE, "the FID of region %d starts at zero", region);
    auto *a = lat->at<double2>(lat->L.off_fft);
    auto *b = a + lat->L.fft_max;
    // the sorted output goes to the buffer the last pass did not write
    int passes = 0;
    for (int64_t p = 1; p < L; p *= 2)
        ++passes;
    double *out = reinterpret_cast<double *>(passes % 2 == 0 ? b : a);
    LPC_HIP(lpc::launch_fid_spectrum(lat->records(), rows, lat->L.K, R, region, L, a, b, out,
                                     lat->stream));
    *sorted = out;
    return LPC_OK;
}

}  // namespace

lpc_status lpc_spectrum(lpc_lattice *lat, int32_t region, int64_t n_fft, double *ppm, double *re,
                        double *im, int64_t cap)
{
    if (!lat || !ppm || !re || !im)
        return fail(LPC_ERR_ARG, "NULL argument");
    const int64_t L = n_fft == 0 ? fft_length(lat->steps_done + 1) : n_fft;
    if (cap < L)
        return fail(LPC_ERR_OOM, "spectrum has %lld points, buffers hold %lld", (long long)L,
                    (long long)cap);
    if (lpc_status s = use_device(lat))
        return s;
    double *sorted = nullptr;
    if (lpc_status s = device_spectrum(lat, region, L, &sorted))
        return s;
    if (lpc_status s = sync(lat))
        return s;
    LPC_HIP(copy_sync(lat, re, sorted, size_t(L) * 8, hipMemcpyDeviceToHost));
    LPC_HIP(copy_sync(lat, im, sorted + L, size_t(L) * 8, hipMemcpyDeviceToHost));
    // frequency axis of the sorted bins: f_j = (j - L/2) / (L dt), in ppm of the Larmor frequency
    const double step = 1e6 / (double(L) * lat->cfg.dt_s * lat->cfg.larmor_hz);
    for (int64_t j = 0; j < L; ++j)
        ppm[j] = double(j - L / 2) * step;
    return ok();
}

lpc_status lpc_spectrum_peak(lpc_lattice *lat, int32_t region, double *peak_ppm)
{
    if (!lat || !peak_ppm)
        return fail(LPC_ERR_ARG, "NULL argument");
    if (lpc_status s = use_device(lat))
        return s;
    const int64_t L = fft_length(lat->steps_done + 1);
    double *sorted = nullptr;
    if (lpc_status s = device_spectrum(lat, region, L, &sorted))
        return s;
    double *pval = lat->at<double>(lat->L.off_argmax);
    auto *pidx = reinterpret_cast<int64_t *>(pval + kArgmaxParts);
    auto *where = pidx + kArgmaxParts;
    LPC_HIP(lpc::launch_argmax(sorted, L, pval, pidx, kArgmaxParts, where, lat->stream));
    if (lpc_status s = sync(lat))
        return s;
    int64_t j = -1;
    LPC_HIP(copy_sync(lat, &j, where, 8, hipMemcpyDeviceToHost));
    if (j < 0)
        return fail(LPC_ERR_NONFINITE, "spectrum has no finite maximum");
    const double step = 1e6 / (double(L) * lat->cfg.dt_s * lat->cfg.larmor_hz);
    double off = 0.0;
    if (j > 0 && j < L - 1) {
        double y[3];
        LPC_HIP(copy_sync(lat, y, sorted + j - 1, 24, hipMemcpyDeviceToHost));
        // vertex of the parabola through the three highest bins
        const double den = y[0] - 2.0 * y[1] + y[2];
        off = den != 0.0 ? 0.5 * (y[0] - y[2]) / den : 0.0;
    }
    *peak_ppm = (double(j - L / 2) + off) * step;
    return ok();
}

lpc_status lpc_diffusion(lpc_lattice *lat, double *D_m2_s, double *ratio)
{
    if (!lat || !D_m2_s || !ratio)
        return fail(LPC_ERR_ARG, "NULL argument");
    if (!msd_of(lat->cfg))
        return fail(LPC_ERR_STATE, "displacement moments are not tracked");
    if (lat->steps_done < 2)
        return fail(LPC_ERR_STATE, "the slope needs at least 2 steps");
    std::vector<double> rec;
    if (lpc_status s = fetch_records(lat, rec))
        return s;
    if (lpc_status s = health(lat, rec))
        return s;
    const int K = lat->L.K, R = lat->cfg.n_regions;
    const int64_t N = lat->steps_done, h = N / 2;
    auto msd = [&](int64_t t, int a) {
        double m = 0.0;
        for (int r = 0; r < R; ++r)
            m += rec[size_t(t * K + 2 * R + r)];
        return rec[size_t(t * K + 3 * R + 3 + a)] / m;
    };
    const double a2 = lat->cfg.spacing_m * lat->cfg.spacing_m;
    for (int a = 0; a < 3; ++a) {
        const double slope = (msd(N, a) - msd(h, a)) / double(N - h);   // lattice units^2 / step
        D_m2_s[a] = a2 * slope / (2.0 * lat->cfg.dt_s);
        ratio[a] = lat->cfg.p_hop > 0.0 ? slope / (2.0 * lat->cfg.p_hop) : 0.0;
    }
    return ok();
}

lpc_status lpc_read_vacf(lpc_lattice *lat, double *vacf_xyz, int64_t cap, int64_t *len)
{
    if (!lat || !vacf_xyz || !len)
        return fail(LPC_ERR_ARG, "NULL argument");
    if (!msd_of(lat->cfg))
        return fail(LPC_ERR_STATE, "displacement moments are not tracked");
    const int64_t N = lat->steps_done;
    if (N < 2)
        return fail(LPC_ERR_STATE, "the autocorrelation needs at least 2 steps");
    if (cap < N)
        return fail(LPC_ERR_OOM, "autocorrelation has %lld rows, buffer holds %lld", (long long)N,
                    (long long)cap);
    std::vector<double> rec;
    if (lpc_status s = fetch_records(lat, rec))
        return s;
    if (lpc_status s = health(lat, rec))
        return s;
    const int K = lat->L.K, R = lat->cfg.n_regions;
    auto mass = [&](int64_t t) {
        double m = 0.0;
        for (int r = 0; r < R; ++r)
            m += rec[size_t(t * K + 2 * R + r)];
        return m;
    };
    if (vacf_of(lat->cfg)) {
        // the tag sums: row t + 1 holds sum over particles of dx_1 dx_{1+t}; per particle of the
        // start
        const double m0 = mass(0);
        if (m0 == 0.0)
            return fail(LPC_ERR_STATE, "the lattice holds no population");
        for (int64_t tau = 0; tau < N; ++tau)
            for (int a = 0; a < 3; ++a)
                vacf_xyz[3 * tau + a] = rec[size_t((tau + 1) * K + 3 * R + 6 + a)] / m0;
        *len = N;
        return ok();
    }
    auto msd = [&](int64_t t, int a) { return rec[size_t(t * K + 3 * R + 3 + a)] / mass(t); };
    for (int a = 0; a < 3; ++a) {
        vacf_xyz[a] = msd(1, a) - msd(0, a);
        for (int64_t tau = 1; tau < N; ++tau)
            vacf_xyz[3 * tau + a] = 0.5 * ((msd(tau + 1, a) - msd(tau, a)) - (msd(tau, a) - msd(tau - 1, a)));
    }
    *len = N;
    return ok();
}

lpc_status lpc_kohn_diffusion(lpc_lattice *lat, int64_t lag, double *D_m2_s)
{
    if (!lat || !D_m2_s)
        return fail(LPC_ERR_ARG, "NULL argument");
    const int64_t N = lat->steps_done;
    if (N >= 2 && (lag < -1 || lag > N - 1))
        return fail(LPC_ERR_ARG, "lag %lld outside -1..%lld", (long long)lag, (long long)(N - 1));
    std::vector<double> C(size_t(std::max<int64_t>(N, 1)) * 3);
    int64_t len = 0;
    if (lpc_status s = lpc_read_vacf(lat, C.data(), N, &len))
        return s;
    const int64_t T = lag < 0 ? len - 1 : lag;
    const double scale = lat->cfg.spacing_m * lat->cfg.spacing_m / lat->cfg.dt_s;
    for (int a = 0; a < 3; ++a) {
        double sum = 0.5 * C[size_t(a)];
        for (int64_t tau = 1; tau <= T; ++tau)
            sum += C[size_t(3 * tau + a)];
        D_m2_s[a] = scale * sum;
    }
    return ok();
}

lpc_status lpc_region_moments(lpc_lattice *lat, double *sums, int64_t cap)
{
    if (!lat || !sums)
        return fail(LPC_ERR_ARG, "NULL argument");
    if (!msd_of(lat->cfg))
        return fail(LPC_ERR_STATE, "displacement moments are not tracked");
    if (!lat->initialized)
        return fail(LPC_ERR_STATE, "state not initialised");
    const int32_t R = lat->cfg.n_regions;
    if (cap < 7 * R)
        return fail(LPC_ERR_OOM, "region sums have %d values, buffer holds %lld", 7 * R,
                    (long long)cap);
    if (lpc_status s = use_device(lat))
        return s;
    // workgroup partials in the per-step partial buffer: queued after the last finalisation
    constexpr int32_t kParts = 1024;
    static_assert(int64_t(kParts) * 7 * LPC_MAX_REGIONS * 8 <= kPartialBudget,
                  "region partials exceed the buffer");
    double *dev = lat->at<double>(lat->L.off_regsum);
    LPC_HIP(lpc::launch_region_sums(lat->cfg.precision, lat->st[lat->cur],
                                    lat->at<uint8_t>(lat->L.off_region), lat->L.n, R,
                                    lat->partials(), kParts, lat->stream));
    LPC_HIP(lpc::launch_finalize(lat->partials(), kParts, 7 * R, 1, dev, lat->stream));
    if (lpc_status s = sync(lat))
        return s;
    LPC_HIP(copy_sync(lat, sums, dev, size_t(7 * R) * 8, hipMemcpyDeviceToHost));
    return ok();
}

lpc_status lpc_uptake_profile(lpc_lattice *lat, int32_t axis, double *profile, int64_t cap)
{
    if (!lat || !profile)
        return fail(LPC_ERR_ARG, "NULL argument");
    if (axis < 0 || axis > 2)
        return fail(LPC_ERR_ARG, "axis %d outside 0..2", axis);
    if (!lat->initialized)
        return fail(LPC_ERR_STATE, "state not initialised");
    const int64_t n = lat->cfg.n[axis];
    if (cap < n)
        return fail(LPC_ERR_OOM, "profile has %lld values, buffer holds %lld", (long long)n,
                    (long long)cap);
    if (lpc_status s = use_device(lat))
        return s;
    lpc::Geometry g{lat->cfg.n[0], lat->cfg.n[1], lat->cfg.n[2],
                    {lat->cfg.bc[0], lat->cfg.bc[1], lat->cfg.bc[2]}};
    double *dev = lat->at<double>(lat->L.off_profile);
    LPC_HIP(lpc::launch_profile(lat->st[lat->cur].rho, g, axis, dev, lat->stream));
    if (lpc_status s = sync(lat))
        return s;
    LPC_HIP(copy_sync(lat, profile, dev, size_t(n) * 8, hipMemcpyDeviceToHost));
    return ok();
}

}  // extern "C"

struct lpc_batch {
    std::vector<lpc_lattice *> lats;
    hipStream_t stream = nullptr;
    int device = 0;
    char *arena = nullptr;
    int32_t precision = 0;
    uint32_t track = 0;
    int32_t maxr = 1;
    lpc::SweepItem *items = nullptr;      // count entries
    int64_t *prefix = nullptr;            // count + 3 entries (one list per tile width)
    lpc::FinalizeItem *fin = nullptr;     // count entries
    int64_t *kprefix = nullptr;           // count + 1 entries
    int64_t *row_counter = nullptr;       // first record row of the chunk a graph replay runs
    hipEvent_t done = nullptr;            // end of the last batch run, awaited by the lattices
    // Graph of one chunk of steps of the current phase (launches captured once, replayed per
    // chunk); destroyed when the phase's tables change, after the stream has drained.
    bool use_graph = true;
    hipStream_t capture = nullptr;        // stream the graph is recorded on (never run)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t graph_replays = 0;            // chunks run through graphs (for lpc_batch_describe)
    int64_t direct_steps = 0;             // steps launched one by one
};

namespace {

struct BatchLayout {
    size_t items, prefix, fin, kprefix, counter, total;
};

void drop_graph(lpc_batch *b)
{
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

BatchLayout batch_layout(int32_t count)
{
    BatchLayout b{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    b.items = take(size_t(count) * sizeof(lpc::SweepItem));
    b.prefix = take(size_t(count + 3) * 8);
    b.fin = take(size_t(count) * sizeof(lpc::FinalizeItem));
    b.kprefix = take(size_t(count + 1) * 8);
    b.counter = take(8);
    b.total = o;
    return b;
}

}  // namespace

extern "C" {

lpc_status lpc_batch_query_footprint(int32_t count, size_t *bytes)
{
    if (count < 1 || !bytes)
        return fail(LPC_ERR_ARG, "count must be >= 1 and bytes non-NULL");
    *bytes = batch_layout(count).total;
    return ok();
}

lpc_status lpc_batch_create(lpc_lattice *const *lats, int32_t count, void *arena, size_t bytes,
                            void *stream, lpc_batch **out)
{
    if (!lats || count < 1 || !arena || !out)
        return fail(LPC_ERR_ARG, "NULL argument or empty batch");
    if (reinterpret_cast<uintptr_t>(arena) % kAlign)
        return fail(LPC_ERR_ARG, "arena must be %zu-byte aligned", kAlign);
    const BatchLayout bl = batch_layout(count);
    if (bytes < bl.total)
        return fail(LPC_ERR_OOM, "batch arena has %zu bytes, needs %zu", bytes, bl.total);
    for (int32_t l = 0; l < count; ++l) {
        if (!lats[l])
            return fail(LPC_ERR_ARG, "lattice %d is NULL", l);
        if (lats[l]->cfg.precision != lats[0]->cfg.precision ||
            lats[l]->cfg.track != lats[0]->cfg.track)
            return fail(LPC_ERR_ARG, "lattice %d differs in precision or track set", l);
        if (lats[l]->device != lats[0]->device)
            return fail(LPC_ERR_ARG, "lattice %d is on another device", l);
        for (int32_t m = 0; m < l; ++m)
            if (lats[m] == lats[l])
                return fail(LPC_ERR_ARG, "lattice %d appears twice", l);
    }
    auto *b = new (std::nothrow) lpc_batch;
    if (!b)
        return fail(LPC_ERR_OOM, "host allocation failed");
    b->lats.assign(lats, lats + count);
    b->stream = static_cast<hipStream_t>(stream);
    b->device = lats[0]->device;
    b->arena = static_cast<char *>(arena);
    b->precision = lats[0]->cfg.precision;
    b->track = lats[0]->cfg.track;
    for (lpc_lattice *l : b->lats)
        b->maxr = std::max(b->maxr, l->cfg.n_regions);
    b->items = reinterpret_cast<lpc::SweepItem *>(b->arena + bl.items);
    b->prefix = reinterpret_cast<int64_t *>(b->arena + bl.prefix);
    b->fin = reinterpret_cast<lpc::FinalizeItem *>(b->arena + bl.fin);
    b->kprefix = reinterpret_cast<int64_t *>(b->arena + bl.kprefix);
    b->row_counter = reinterpret_cast<int64_t *>(b->arena + bl.counter);
    if (hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
        delete b;
        return fail(LPC_ERR_DEVICE, "hipEventCreateWithFlags failed");
    }
    // default priority, like every stream here
    if (hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess) {
        (void)hipEventDestroy(b->done);
        delete b;
        return fail(LPC_ERR_DEVICE, "hipStreamCreateWithFlags failed");
    }
    *out = b;
    return ok();
}

lpc_status lpc_batch_destroy(lpc_batch *batch)
{
    if (!batch)
        return fail(LPC_ERR_ARG, "batch is NULL");
    (void)hipStreamSynchronize(batch->stream);
    drop_graph(batch);
    (void)hipStreamDestroy(batch->capture);
    (void)hipEventDestroy(batch->done);
    delete batch;
    return ok();
}

lpc_status lpc_batch_run(lpc_batch *batch, const int64_t *n_steps)
{
    if (!batch || !n_steps)
        return fail(LPC_ERR_ARG, "NULL argument");
    const int32_t count = int32_t(batch->lats.size());
    for (int32_t l = 0; l < count; ++l) {
        const lpc_lattice *lat = batch->lats[l];
        if (n_steps[l] < 0)
            return fail(LPC_ERR_ARG, "n_steps[%d] is negative", l);
        if (n_steps[l] > 0 && !lat->initialized)
            return fail(LPC_ERR_STATE, "lattice %d is not initialised", l);
        if (lat->steps_done + n_steps[l] > lat->cfg.max_records - 1)
            return fail(LPC_ERR_STATE, "lattice %d: records hold %lld steps; %lld done, %lld asked",
                        l, (long long)(lat->cfg.max_records - 1), (long long)lat->steps_done,
                        (long long)n_steps[l]);
    }
    int d = -1;
    LPC_HIP(hipGetDevice(&d));
    if (d != batch->device)
        LPC_HIP(hipSetDevice(batch->device));
    // the lattices' own streams may still hold work on them
    for (lpc_lattice *lat : batch->lats)
        LPC_HIP(hipStreamSynchronize(lat->stream));
    // a lattice that tracks autocorrelation tags and starts from step 0 takes its tagging
    // step alone (the same kernel and plan as in the batch), then joins the batch
    std::vector<int64_t> steps_left(n_steps, n_steps + count);
    for (int32_t l = 0; l < count; ++l) {
        lpc_lattice *lat = batch->lats[l];
        if (steps_left[size_t(l)] > 0 && vacf_of(lat->cfg) && lat->steps_done == 0) {
            if (lpc_status st = queue_steps(lat, 1, batch->stream))
                return st;
            --steps_left[size_t(l)];
        }
    }
    n_steps = steps_left.data();
    std::vector<lpc::SweepItem> items;
    std::vector<int64_t> prefix, kprefix;
    std::vector<lpc::FinalizeItem> fin;
    std::vector<int32_t> active;
    int64_t done = 0;
    for (;;) {
        active.clear();
        int64_t phase_end = INT64_MAX;
        for (int32_t l = 0; l < count; ++l)
            if (n_steps[l] > done) {
                active.push_back(l);
                phase_end = std::min(phase_end, n_steps[l]);
            }
        if (active.empty())
            break;
        const int64_t steps = phase_end - done;
        // work tables of this phase: one list per tile width and kernel variant (each lattice
        // runs the kernel it runs alone), then the finalisation list
        items.clear();
        prefix.clear();
        fin.clear();
        kprefix.assign(1, 0);
        struct Group {
            int32_t tile_x, first, n;
            uint32_t variant;
            size_t prefix_at;
            int64_t total;
        };
        std::vector<Group> groups;
        int64_t chunk = kChunkMax;
        for (uint32_t ext : {0u, lpc::kVariantExtended}) {
            for (int32_t tx : {64, 32, 16, lpc::kTileLinear}) {
                Group gr{tx, int32_t(items.size()), 0, ext, prefix.size(), 0};
                prefix.push_back(0);
                for (int32_t l : active) {
                    lpc_lattice *lat = batch->lats[l];
                    if (lat->L.plan.tx != tx ||
                        (variant_of(lat->cfg) & lpc::kVariantExtended) != ext)
                        continue;
                    items.push_back(lat->sweep_item(lat->cur));
                    gr.total += lat->L.plan.nblocks;
                    prefix.push_back(gr.total);
                    ++gr.n;
                }
                if (gr.n > 0)
                    groups.push_back(gr);
            }
        }
        for (int32_t l : active) {
            lpc_lattice *lat = batch->lats[l];
            fin.push_back(lat->finalize_item(lat->steps_done));
            kprefix.push_back(kprefix.back() + lat->L.K);
            chunk = std::min(chunk, lat->L.chunk);
        }
        LPC_HIP(hipStreamSynchronize(batch->stream));
        drop_graph(batch);          // the stream has drained: no replay of it is pending
        LPC_HIP(hipMemcpyAsync(batch->items, items.data(), items.size() * sizeof(items[0]),
                               hipMemcpyHostToDevice, batch->stream));
        LPC_HIP(hipMemcpyAsync(batch->prefix, prefix.data(), prefix.size() * 8,
                               hipMemcpyHostToDevice, batch->stream));
        LPC_HIP(hipMemcpyAsync(batch->fin, fin.data(), fin.size() * sizeof(fin[0]),
                               hipMemcpyHostToDevice, batch->stream));
        LPC_HIP(hipMemcpyAsync(batch->kprefix, kprefix.data(), kprefix.size() * 8,
                               hipMemcpyHostToDevice, batch->stream));
        LPC_HIP(hipStreamSynchronize(batch->stream));
        const int64_t total_k = kprefix.back();
        // the launches of one chunk of c steps: c steps of every group, then the records
        auto enqueue_chunk = [&](hipStream_t st, int64_t s0, int64_t c,
                                 const int64_t *row_offset) -> lpc_status {
            for (int64_t s = 0; s < c; ++s) {
                for (const Group &gr : groups) {
                    lpc::StepList list{batch->items + gr.first, batch->prefix + gr.prefix_at,
                                       gr.n, gr.tile_x, gr.total, int32_t((s0 + s) & 1), s};
                    LPC_HIP(lpc::launch_step_list(list, batch->precision,
                                                  batch->track | gr.variant, batch->maxr, st));
                }
            }
            LPC_HIP(lpc::launch_finalize_list(batch->fin, batch->kprefix, int32_t(active.size()),
                                              total_k, c, row_offset ? 0 : s0 + 1, st,
                                              row_offset));
            return LPC_OK;
        };
        int64_t s0 = 0;
        // Whole chunks of an even number of steps (the same parities every chunk) replay one
        // captured graph; its record rows come from a device counter that the graph advances.
        const int64_t gc = chunk - chunk % 2;
        if (batch->use_graph && gc >= 2 && steps >= gc) {
            LPC_HIP(lpc::launch_set_counter(batch->row_counter, 1, 0, batch->stream));
            LPC_HIP(hipStreamBeginCapture(batch->capture, hipStreamCaptureModeRelaxed));
            lpc_status st = enqueue_chunk(batch->capture, 0, gc, batch->row_counter);
            if (st == LPC_OK &&
                lpc::launch_set_counter(batch->row_counter, 0, gc, batch->capture) != hipSuccess)
                st = fail(LPC_ERR_DEVICE, "counter launch failed during capture");
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(batch->capture, &g);
            if (st != LPC_OK) {
                if (g)
                    (void)hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess)
                return fail(LPC_ERR_DEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
            batch->graph = g;
            LPC_HIP(hipGraphInstantiate(&batch->exec, batch->graph, nullptr, nullptr, 0));
            const int64_t replays = steps / gc;
            for (int64_t r = 0; r < replays; ++r)
                LPC_HIP(hipGraphLaunch(batch->exec, batch->stream));
            batch->graph_replays += replays;
            s0 = replays * gc;
        }
        batch->direct_steps += steps - s0;
        for (; s0 < steps; s0 += chunk) {
            const int64_t c = std::min(chunk, steps - s0);
            if (lpc_status st = enqueue_chunk(batch->stream, s0, c, nullptr))
                return st;
        }
        for (int32_t l : active) {
            lpc_lattice *lat = batch->lats[l];
            lat->steps_done += steps;
            lat->cur ^= int(steps & 1);
        }
        done = phase_end;
    }
    // later work and reads on each lattice's own stream come after the batch
    LPC_HIP(hipEventRecord(batch->done, batch->stream));
    for (lpc_lattice *lat : batch->lats)
        LPC_HIP(hipStreamWaitEvent(lat->stream, batch->done, 0));
    return ok();
}

}  // extern "C"

namespace {

// Work area of lpc_spectrum_noalloc: the two ping-pong buffers of the FFT at its largest
// length. Each device holds its own copy from the library's load until the process ends.
constexpr int64_t kNoallocFftMax = int64_t(1) << 20;
static __device__ __align__(256) double2 scratch[2 * kNoallocFftMax];

std::mutex g_scratch_mutex;
std::vector<double2 *> g_scratch_ptr;   // device address of `scratch`, per device

// Device address of the scratch array on the current device, looked up once per device.
// The host-side name of the array is not a device address; only this pointer may reach a
// kernel or a copy.
lpc_status scratch_on_current_device(double2 **out)
{
    int dev = -1;
    LPC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr.size() <= size_t(dev))
        g_scratch_ptr.resize(size_t(dev) + 1, nullptr);
    if (!g_scratch_ptr[size_t(dev)]) {
        void *p = nullptr;
        LPC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p)
            return fail(LPC_ERR_DEVICE, "no device address for the scratch area on device %d", dev);
        g_scratch_ptr[size_t(dev)] = static_cast<double2 *>(p);
    }
    *out = g_scratch_ptr[size_t(dev)];
    return LPC_OK;
}

}  // namespace

extern "C" {

lpc_status lpc_spectrum_noalloc(const double *fid, int64_t n_samples, int64_t n_fft, double *spec,
                                void *stream)
{
    if (!fid || !spec)
        return fail(LPC_ERR_ARG, "NULL buffer");
    if (n_samples < 1)
        return fail(LPC_ERR_ARG, "n_samples = %lld must be >= 1", (long long)n_samples);
    const int64_t L = n_fft == 0 ? fft_length(n_samples) : n_fft;
    if (L < n_samples || (L & (L - 1)) != 0)
        return fail(LPC_ERR_ARG, "n_fft = %lld must be a power of two >= %lld samples",
                    (long long)L, (long long)n_samples);
    if (L > kNoallocFftMax)
        return fail(LPC_ERR_OOM, "n_fft = %lld exceeds the scratch area's %lld points",
                    (long long)L, (long long)kNoallocFftMax);
    double2 *work = nullptr;
    if (lpc_status s = scratch_on_current_device(&work))
        return s;
    // the FID as a record table of one region: K = 2 values (Re, Im) per row; the first
    // kernel writes all L points of the first buffer, so nothing needs clearing
    LPC_HIP(lpc::launch_fid_spectrum(fid, n_samples, 2, 1, -1, L, work, work + kNoallocFftMax,
                                     spec, static_cast<hipStream_t>(stream)));
    return ok();
}

lpc_status lpc_batch_use_graph(lpc_batch *batch, int32_t enable)
{
    if (!batch)
        return fail(LPC_ERR_ARG, "batch is NULL");
    batch->use_graph = enable != 0;
    return ok();
}

lpc_status lpc_batch_describe(const lpc_batch *batch, char *buf, size_t cap)
{
    if (!batch || !buf || cap == 0)
        return fail(LPC_ERR_ARG, "NULL argument");
    snprintf(buf, cap, "%zu lattices, graphs %s, %lld chunks replayed from graphs, %lld steps "
                       "launched directly",
             batch->lats.size(), batch->use_graph ? "on" : "off",
             (long long)batch->graph_replays, (long long)batch->direct_steps);
    return ok();
}

lpc_status lpc_stream_copy(const void *src, void *dst, size_t bytes, void *stream)
{
    if (!src || !dst)
        return fail(LPC_ERR_ARG, "NULL buffer");
    if (bytes % 16 || reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
        return fail(LPC_ERR_ARG, "buffers and size must be 16-byte aligned");
    const char *a = static_cast<const char *>(src);
    const char *b = static_cast<const char *>(dst);
    if (a < b + bytes && b < a + bytes)
        return fail(LPC_ERR_ARG, "buffers overlap");
    LPC_HIP(lpc::launch_stream_copy(src, dst, int64_t(bytes / 16), static_cast<hipStream_t>(stream)));
    return ok();
}

lpc_status lpc_stream_columns(const double *const *in, double *const *out, int32_t nx,
                              int32_t ny, int32_t nz, int32_t zc, void *stream)
{
    if (!in || !out)
        return fail(LPC_ERR_ARG, "NULL array list");
    if (nx < 1 || ny < 1 || nz < 1 || zc < 1)
        return fail(LPC_ERR_ARG, "sizes and zc must be >= 1");
    const int64_t n = int64_t(nx) * ny * nz;
    const int64_t blocks = int64_t((nx + 63) / 64) * ((ny + 3) / 4) * ((nz + zc - 1) / zc);
    if (blocks > INT32_MAX)
        return fail(LPC_ERR_ARG, "too many workgroups; raise zc");
    const size_t bytes = size_t(n) * 8;
    lpc::ColumnArrays c{};
    for (int k = 0; k < lpc::kColumnIn; ++k) {
        if (!in[k])
            return fail(LPC_ERR_ARG, "input array %d is NULL", k);
        c.in[k] = in[k];
    }
    for (int k = 0; k < lpc::kColumnOut; ++k) {
        if (!out[k])
            return fail(LPC_ERR_ARG, "output array %d is NULL", k);
        c.out[k] = out[k];
    }
    // outputs overlap nothing (inputs may repeat: they are only read)
    auto overlap = [bytes](const void *p, const void *q) {
        const char *a = static_cast<const char *>(p), *b = static_cast<const char *>(q);
        return a < b + bytes && b < a + bytes;
    };
    for (int k = 0; k < lpc::kColumnOut; ++k) {
        for (int j = 0; j < lpc::kColumnIn; ++j)
            if (overlap(out[k], in[j]))
                return fail(LPC_ERR_ARG, "output %d overlaps input %d", k, j);
        for (int j = 0; j < k; ++j)
            if (overlap(out[k], out[j]))
                return fail(LPC_ERR_ARG, "outputs %d and %d overlap", j, k);
    }
    LPC_HIP(lpc::launch_stream_columns(c, nx, ny, nz, zc, static_cast<hipStream_t>(stream)));
    return ok();
}

lpc_status lpc_stream_columns_mixed(const double *rho_in, const float *const *in,
                                    const uint8_t *region, double *rho_out, float *const *out,
                                    int32_t nx, int32_t ny, int32_t nz, int32_t zc, void *stream)
{
    if (!rho_in || !in || !region || !rho_out || !out)
        return fail(LPC_ERR_ARG, "NULL array");
    if (nx < 1 || ny < 1 || nz < 1 || zc < 1)
        return fail(LPC_ERR_ARG, "sizes and zc must be >= 1");
    const int64_t n = int64_t(nx) * ny * nz;
    const int64_t blocks = int64_t((nx + 63) / 64) * ((ny + 3) / 4) * ((nz + zc - 1) / zc);
    if (blocks > INT32_MAX)
        return fail(LPC_ERR_ARG, "too many workgroups; raise zc");
    lpc::MixedColumns c{};
    c.rho_in = rho_in;
    c.region = region;
    c.rho_out = rho_out;
    // every array with its size; the outputs (the last 9) overlap nothing
    struct Span {
        const void *p;
        size_t bytes;
    };
    Span spans[2 + lpc::kMixedIn + 1 + lpc::kMixedOut];
    int ns = 0;
    spans[ns++] = {rho_in, size_t(n) * 8};
    for (int k = 0; k < lpc::kMixedIn; ++k) {
        if (!in[k])
            return fail(LPC_ERR_ARG, "input array %d is NULL", k);
        c.in[k] = in[k];
        spans[ns++] = {in[k], size_t(n) * 4};
    }
    spans[ns++] = {region, size_t(n)};
    const int first_out = ns;
    spans[ns++] = {rho_out, size_t(n) * 8};
    for (int k = 0; k < lpc::kMixedOut; ++k) {
        if (!out[k])
            return fail(LPC_ERR_ARG, "output array %d is NULL", k);
        c.out[k] = out[k];
        spans[ns++] = {out[k], size_t(n) * 4};
    }
    for (int a = first_out; a < ns; ++a)
        for (int b = 0; b < a; ++b) {
            const char *p = static_cast<const char *>(spans[a].p);
            const char *q = static_cast<const char *>(spans[b].p);
            if (p < q + spans[b].bytes && q < p + spans[a].bytes)
                return fail(LPC_ERR_ARG, "output array %d overlaps array %d", a, b);
        }
    LPC_HIP(lpc::launch_stream_columns_mixed(c, nx, ny, nz, zc, static_cast<hipStream_t>(stream)));
    return ok();
}

lpc_status lpc_set_plan(lpc_lattice *lat, int32_t tile_x, int32_t zc)
{
    if (!lat)
        return fail(LPC_ERR_ARG, "lattice is NULL");
    if (tile_x != 0 && tile_x != 64 && tile_x != 32 && tile_x != 16 && tile_x != LPC_TILE_LINEAR &&
        tile_x != LPC_TILE_TWO_STEP)
        return fail(LPC_ERR_ARG, "tile_x = %d is not 0, 1, 2, 64, 32 or 16", tile_x);
    if (zc < 0)
        return fail(LPC_ERR_ARG, "zc = %d is negative", zc);
    if (tile_x == LPC_TILE_TWO_STEP) {
        if (!two_step_available(lat->cfg))
            return fail(LPC_ERR_ARG, "two steps per pass need the plain variant (no mobility "
                                     "field, no reservoir axis)");
        if (lpc_status s = use_device(lat))
            return s;
        lpc::Geometry g{lat->cfg.n[0], lat->cfg.n[1], lat->cfg.n[2],
                        {lat->cfg.bc[0], lat->cfg.bc[1], lat->cfg.bc[2]}};
        lpc::SweepPlan p = lpc::make_plan2(g, lat->occupancy2, lat->cus, zc_floor(lat->cfg));
        if (zc > 0)
            p = lpc::with_z_chunk(p, g, zc);
        if (2 * size_t(p.nblocks) * lat->L.K * 8 > lat->L.partial_bytes)
            return fail(LPC_ERR_ARG, "plan with %lld workgroups does not fit the partial sums",
                        (long long)p.nblocks);
        if (lpc_status s = sync(lat))
            return s;
        lat->plan2 = p;
        lat->chunk2 = two_step_chunk(lat->L, p);
        lat->steps_per_pass = 2;
        if (lpc_status s = upload_solo(lat))
            return s;
        return ok();
    }
    const int32_t linear_max = lpc::linear_tile_max_nx(lat->cfg.precision, variant_of(lat->cfg));
    if (tile_x == LPC_TILE_LINEAR && lat->cfg.n[0] > linear_max)
        return fail(LPC_ERR_ARG,
                    "linear tiles take nx <= %d for this precision, track set and variant "
                    "(nx = %d)", linear_max, lat->cfg.n[0]);
    if (lpc_status s = use_device(lat))
        return s;
    lpc::Geometry g{lat->cfg.n[0], lat->cfg.n[1], lat->cfg.n[2],
                    {lat->cfg.bc[0], lat->cfg.bc[1], lat->cfg.bc[2]}};
    lpc::SweepPlan p = lpc::make_plan(g, lat->occupancy, lat->cus, tile_x, linear_max,
                                      zc_floor(lat->cfg));
    if (zc > 0)
        p = lpc::with_z_chunk(p, g, zc);
    if (size_t(p.nblocks) * lat->L.K * 8 > lat->L.partial_bytes)
        return fail(LPC_ERR_ARG, "plan with %lld workgroups does not fit the partial sums",
                    (long long)p.nblocks);
    if (lpc_status s = sync(lat))
        return s;
    Layout L = lat->L;
    L.plan = p;
    set_chunk(L);
    lat->L = L;
    lat->steps_per_pass = 1;
    if (lpc_status s = upload_solo(lat))
        return s;
    return ok();
}

lpc_status lpc_describe(const lpc_lattice *lat, char *buf, size_t cap)
{
    if (!lat || !buf || cap == 0)
        return fail(LPC_ERR_ARG, "NULL argument");
    const lpc::SweepPlan &p = lat->L.plan;
    int n = snprintf(buf, cap,
                     "tile %dx%d, zc %d, grid %dx%dx%d = %lld workgroups, %lld steps per finalize, "
                     "arena %zu bytes, steps per pass %d",
                     p.tx, p.ty, p.zc, p.gx, p.gy, p.gz, (long long)p.nblocks,
                     (long long)lat->L.chunk, lat->L.total, lat->steps_per_pass);
    if (lat->steps_per_pass == 2 && n >= 0 && size_t(n) < cap) {
        const lpc::SweepPlan &q = lat->plan2;
        snprintf(buf + n, cap - size_t(n),
                 ", two-step tile %dx%d, zc %d, grid %dx%dx%d = %lld workgroups, %lld steps per "
                 "finalize",
                 lpc::kTwoStepTileX, lpc::kTwoStepTileY, q.zc, q.gx, q.gy, q.gz,
                 (long long)q.nblocks, (long long)lat->chunk2);
    }
    return ok();
}

lpc_status lpc_p_hop_from_residence_time(double tau_s, double dt_s, double *p_hop)
{
    if (!p_hop)
        return fail(LPC_ERR_ARG, "p_hop is NULL");
    if (!std::isfinite(tau_s) || !std::isfinite(dt_s) || !(dt_s > 0.0) || !(tau_s >= dt_s))
        return fail(LPC_ERR_ARG, "need finite tau_s >= dt_s > 0 (tau_s = %g, dt_s = %g)", tau_s,
                    dt_s);
    // a free site is left with probability 6 p_hop per step: mean stay dt / (6 p_hop)
    *p_hop = dt_s / (6.0 * tau_s);
    return ok();
}

lpc_status lpc_region_diffusion(const double *sums_a, const double *sums_b, int32_t n_regions,
                                int64_t steps_between, double p_hop, double dt_s,
                                double spacing_m, uint32_t axes, double *D_m2_s, double *ratio)
{
    if (!sums_a || !sums_b || !D_m2_s || !ratio)
        return fail(LPC_ERR_ARG, "NULL argument");
    if (n_regions < 1 || n_regions > LPC_MAX_REGIONS)
        return fail(LPC_ERR_ARG, "n_regions = %d outside 1..%d", n_regions, LPC_MAX_REGIONS);
    if (steps_between < 1)
        return fail(LPC_ERR_ARG, "steps_between must be >= 1");
    if (axes < 1 || axes > 7)
        return fail(LPC_ERR_ARG, "axes mask 0x%x: need bits of axes 0..2, at least one", axes);
    for (double v : {p_hop, dt_s, spacing_m})
        if (!std::isfinite(v) || !(v > 0.0))
            return fail(LPC_ERR_ARG, "p_hop, dt_s and spacing_m must be positive and finite");
    for (int32_t r = 0; r < n_regions; ++r)
        if (!(sums_a[7 * r] != 0.0) || !(sums_b[7 * r] != 0.0))
            return fail(LPC_ERR_STATE, "region %d holds no population", r);
    int n_axes = 0;
    for (int a = 0; a < 3; ++a)
        n_axes += (axes >> a) & 1u;
    for (int32_t r = 0; r < n_regions; ++r) {
        const double *A = sums_a + 7 * r, *B = sums_b + 7 * r;
        double slope = 0.0;
        for (int a = 0; a < 3; ++a) {
            if (!((axes >> a) & 1u))
                continue;
            // mean-square displacement of the particles now in the region, per step
            slope += (B[4 + a] / B[0] - A[4 + a] / A[0]) / double(steps_between);
        }
        slope /= n_axes;
        D_m2_s[r] = spacing_m * spacing_m * slope / (2.0 * dt_s);
        ratio[r] = slope / (2.0 * p_hop);
    }
    return ok();
}

const char *lpc_last_error(void)
{
    return g_error.c_str();
}

const char *lpc_version(void)
{
    return "liblpc 0.2 (gfx950)";
}

}  // extern "C"
