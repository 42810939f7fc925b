/*
 * lpc.h -- C ABI of liblpc, the MI355X lattice sweep of the LPC3D mesoscopic model.
 *
 * The model (LPC3D paper, section 2): densities of non-interacting species on a simple
 * cubic lattice hop between nearest neighbours with Metropolis probabilities set by
 * site free energies (Eq. (1)); their Boltzmann distribution (Eq. (2)) is stationary.
 * Moment propagation (section 2.2) carries displacement moments for diffusion
 * coefficients (Eqs. (4)-(7)); the complex magnetisation of each site is gathered from
 * its neighbours and rotated by the site's chemical-shift phase every step (Eqs. (8),
 * (10)-(13)), and its sum over sites is the free-induction decay (FID) whose Fourier
 * transform is the NMR spectrum (Eq. (9)).
 *
 * One step, per site i with neighbours j (attempt probability p0 per neighbour):
 *   p(i->j)  = p0 * min(1, exp(-(F_j - F_i)))           F in units of kT
 *   stay(i)  = 1 - sum_j p(i->j)                         closed faces: no neighbour
 *   rho'_i   = stay(i) rho_i + sum_j p(j->i) rho_j
 *   m'_i     = exp(i theta_i) [stay(i) m_i + sum_j p(j->i) m_j],
 *              theta_i = 2 pi delta_i[ppm] 1e-6 larmor_hz dt_s
 *   M1'_a,i  = stay(i) M1_a,i + sum_j p(j->i) (M1_a,j + d_a rho_j)
 *   M2'_a,i  = stay(i) M2_a,i + sum_j p(j->i) (M2_a,j + 2 d_a M1_a,j + d_a^2 rho_j)
 * with d_a the unwrapped a-component of the hop j -> i. After every step, and once for
 * the initial state, the library records in FP64, per region r, Re/Im of sum m and
 * sum rho, and over all sites sum M1_a and sum M2_a.
 *
 * Conventions
 *  - Every call returns an lpc_status; on error the out-parameters are left untouched
 *    and lpc_last_error() returns a message (thread-local). Nothing aborts and no C++
 *    exception crosses this boundary.
 *  - Device memory: the caller owns one device buffer (the arena) of at least
 *    lpc_query_footprint() bytes, aligned to 256 bytes, for the lifetime of the lattice.
 *    The library places all of its device data in it and never allocates or frees device
 *    memory itself.
 *  - Host arrays passed in are copied before the call returns; no pointer is kept.
 *  - Host site arrays hold nx*ny*nz values with x fastest: index x + nx*(y + ny*z).
 *  - Streams: work is queued on the stream given at creation (a hipStream_t passed as
 *    void*, NULL = the null stream). lpc_run returns once the work is queued; device
 *    errors surface at the next lpc_synchronize or read. Reads synchronize the stream.
 *    Every copy between host and device also runs on that stream, so a call that waits
 *    (a set, a read, a checkpoint) waits for the lattice's own work only, not for work
 *    queued on other streams.
 *  - A handle is not thread-safe: one thread at a time may use it.
 */
#ifndef LPC_H
#define LPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lpc_status {
    LPC_OK = 0,
    LPC_ERR_ARG = 1,          /* bad argument: NULL, size mismatch, out of range */
    LPC_ERR_OOM = 2,          /* arena or host buffer too small */
    LPC_ERR_DEVICE = 3,       /* a HIP call failed */
    LPC_ERR_STATE = 4,        /* call out of order, or record capacity exceeded */
    LPC_ERR_NONFINITE = 5,    /* NaN/Inf in an input, or in the recorded FID */
    LPC_ERR_CONSERVATION = 6  /* total population drifted beyond conservation_tol */
} lpc_status;

/* Boundary per axis. PERIODIC wraps; CLOSED has no neighbour beyond the faces (attempts
 * across them stay); RESERVOIR puts a ghost site with fixed values beyond each face (the
 * Dirichlet ghost layers of section 3.2, set by lpc_set_reservoir): moves into it leave
 * the lattice and moves out of it bring its population and magnetisation in, so the
 * total is not conserved and the conservation check is off for such a lattice. */
enum { LPC_BC_PERIODIC = 0, LPC_BC_CLOSED = 1, LPC_BC_RESERVOIR = 2 };

/* Options. MOBILITY adds a per-site mobility field mu (lpc_set_mobility): both hop
 * probabilities of the link i-j are scaled by alpha_ij = min(mu_i, mu_j), one factor for
 * both directions as detailed balance requires (section 2.2, after Eq. (7)). BATCHED
 * plans the lattice for stepping in a batch (lpc_batch_run) with others: its automatic
 * plan takes z-chunks of at least 16 planes (fewer, longer workgroups with less re-read
 * at chunk ends), since the batch rather than the lattice alone fills the device. It
 * changes no result beyond the order of the per-step sums; solo runs of the lattice use
 * the same plan and give the same bits as its batched runs. */
enum { LPC_OPT_MOBILITY = 1u, LPC_OPT_BATCHED = 2u };

/* FP64: every field, state array and operation in double. MIXED: populations stored
 * and updated in double; free energy, phase, magnetisation and moments stored and
 * updated in float (hop probabilities in float, promoted for the population update);
 * every record sum in double. */
enum { LPC_PREC_FP64 = 0, LPC_PREC_MIXED = 1 };

/* Track set. Populations are always propagated. FID: the magnetisation; MSD: the
 * displacement moments M1, M2 per axis; VACF (with MSD): three more fields that carry each
 * particle's first displacement, from which the velocity autocorrelation of Eq. (4) is
 * recorded every step without differencing the moments (lpc_read_vacf). */
enum { LPC_TRACK_FID = 1u, LPC_TRACK_MSD = 2u, LPC_TRACK_VACF = 4u };

enum { LPC_INIT_UNIFORM = 0, LPC_INIT_BOLTZMANN = 1, LPC_INIT_USER = 2 };

#define LPC_MAX_REGIONS 8

typedef struct lpc_config {
    int32_t n[3];             /* nx, ny, nz >= 1 */
    int32_t bc[3];            /* LPC_BC_PERIODIC, LPC_BC_CLOSED or LPC_BC_RESERVOIR */
    int32_t precision;        /* LPC_PREC_FP64 or LPC_PREC_MIXED */
    uint32_t track;           /* LPC_TRACK_FID | LPC_TRACK_MSD (0 = populations only) */
    int32_t n_regions;        /* 1..LPC_MAX_REGIONS */
    uint32_t options;         /* LPC_OPT_* bits (0: none) */
    double p_hop;             /* attempt probability per neighbour, 0 <= 6 p_hop <= 1 (1/7) */
    double dt_s;              /* time step in seconds (5e-6) */
    double larmor_hz;         /* spectrometer Larmor frequency (400e6) */
    double spacing_m;         /* lattice spacing a in metres (0.5e-9) */
    int64_t max_records;      /* record rows kept: the initial state + steps, >= 1 */
    double conservation_tol;  /* relative mass drift that reads report; 0 disables */
} lpc_config;

typedef struct lpc_lattice lpc_lattice;
typedef struct lpc_batch lpc_batch;

/* Fills the defaults above for an n^3 periodic FP64 lattice with full tracking. */
lpc_status lpc_config_default(lpc_config *cfg, int32_t n);

/* Device bytes the lattice needs for cfg (fields, two state buffers, per-step
 * partial sums, records and a staging area). */
lpc_status lpc_query_footprint(const lpc_config *cfg, size_t *bytes);

/* Creates a lattice in the caller's arena (device pointer, >= footprint bytes, 256-byte
 * aligned). Fields start at F = 0, delta = 0, region 0; the state is uninitialised until
 * lpc_init_state. stream: hipStream_t as void*. */
lpc_status lpc_create(const lpc_config *cfg, void *arena, size_t arena_bytes, void *stream,
                      lpc_lattice **out);
lpc_status lpc_destroy(lpc_lattice *lat);

/* Site free energies in kT (Eq. (1)); n must be nx*ny*nz. F = +INFINITY marks an
 * inaccessible site (solid matrix, section 2.1 and Fig. 1): it holds nothing and every
 * move towards it is rejected. NaN or -Inf -> LPC_ERR_NONFINITE; a finite |F| above 1e30,
 * or accessible free energies spanning more than 1400 kT -> LPC_ERR_ARG. */
lpc_status lpc_set_free_energy(lpc_lattice *lat, const double *F_kT, int64_t n);
/* Per-site mobility mu in [0, 1] (n values; needs LPC_OPT_MOBILITY, else LPC_ERR_STATE;
 * out of range -> LPC_ERR_ARG, NaN -> LPC_ERR_NONFINITE). Starts at 1 everywhere. */
lpc_status lpc_set_mobility(lpc_lattice *lat, const double *mu, int64_t n);
/* Ghost site beyond face `side` (0: below coordinate 0, 1: above n - 1) of a RESERVOIR
 * axis: free energy F_kT (finite, |F| <= 1e30), population rho >= 0 and magnetisation
 * (m_re, m_im); its displacement moments are zero and its mobility 1. Starts at F = 0,
 * rho = m = 0 (an empty, absorbing reservoir). LPC_ERR_STATE if the axis is not a
 * reservoir axis. Takes effect from the next queued step. */
lpc_status lpc_set_reservoir(lpc_lattice *lat, int32_t axis, int32_t side, double F_kT,
                             double rho, double m_re, double m_im);
/* Site chemical shifts in ppm (Eq. (11) phase per step); NaN/Inf -> LPC_ERR_NONFINITE. */
lpc_status lpc_set_shift(lpc_lattice *lat, const double *delta_ppm, int64_t n);
/* Region id per site, each < n_regions, else LPC_ERR_ARG. */
lpc_status lpc_set_regions(lpc_lattice *lat, const uint8_t *region, int64_t n);

/* Initial state: UNIFORM rho = 1; BOLTZMANN rho_i = N_open exp(-F_i) / sum_j exp(-F_j)
 * (Eq. (2), mean density 1 over the N_open accessible sites); USER rho from the host
 * array (finite, n values). Inaccessible sites get rho = 0 in every mode. In every mode
 * m = rho (real), M1 = M2 = 0, the step counter is reset and record row 0 is written. rho
 * may be NULL unless mode is USER. */
lpc_status lpc_init_state(lpc_lattice *lat, int32_t mode, const double *rho, int64_t n);

/* Equilibration phase (section 3.2 of the paper): steps the populations alone, from the
 * current state, until the largest change of one step relative to the largest population,
 * max_i |rho_i(t+1) - rho_i(t)| / max_i rho_i(t+1), is <= tol, checked every check_every
 * steps (>= 1), or until max_steps steps. Then restarts the propagation from the
 * equilibrated populations: m = rho (real), M1 = M2 = 0, step counter 0, record row 0
 * rewritten. *steps_taken (a multiple of check_every, or max_steps) and *residual (the
 * last checked change) are optional. Synchronous. */
lpc_status lpc_equilibrate(lpc_lattice *lat, int64_t max_steps, double tol, int64_t check_every,
                           int64_t *steps_taken, double *residual);

/* Queues n_steps steps. LPC_ERR_STATE if not initialised or if steps_done + n_steps
 * would exceed max_records - 1. */
lpc_status lpc_run(lpc_lattice *lat, int64_t n_steps);
lpc_status lpc_synchronize(lpc_lattice *lat);
lpc_status lpc_steps_done(const lpc_lattice *lat, int64_t *n);

/* Record width K = 3 R + 6 (+ 3 with LPC_TRACK_VACF) and raw records: rows of
 * [Re G_r, Im G_r] (r < R), U_r (r < R), S1_x, S1_y, S1_z, S2_x, S2_y, S2_z, then with the
 * tags C_x, C_y, C_z; row t is after t steps. C of row t >= 1 is the sum over particles of
 * dx_a(1) dx_a(t) (the lag t - 1 of lpc_read_vacf, not normalised); row 0 holds zeros. */
lpc_status lpc_record_width(const lpc_lattice *lat, int32_t *K);
lpc_status lpc_read_records(lpc_lattice *lat, double *records, int64_t cap_rows, int64_t *rows);

/* Final-state arrays (n values each, double). */
lpc_status lpc_read_population(lpc_lattice *lat, double *rho, int64_t n);
lpc_status lpc_read_magnetization(lpc_lattice *lat, double *re, double *im, int64_t n);

/* Derived record series (steps_done + 1 rows). These check the run first: a non-finite
 * FID gives LPC_ERR_NONFINITE and a relative mass drift above conservation_tol gives
 * LPC_ERR_CONSERVATION. region = -1 sums all regions. msd/drift: S2/mass, S1/mass
 * per axis, 3 values per row. uptake: R values per row. */
lpc_status lpc_read_fid(lpc_lattice *lat, int32_t region, double *re, double *im, int64_t cap,
                        int64_t *len);
lpc_status lpc_read_moments(lpc_lattice *lat, double *mass, double *msd_xyz, double *drift_xyz,
                            int64_t cap, int64_t *len);
lpc_status lpc_read_uptake(lpc_lattice *lat, double *per_step_per_region, int64_t cap,
                           int64_t *len);
lpc_status lpc_check(lpc_lattice *lat);

/* Post-processing on the device. */

/* Default FFT length of lpc_spectrum: the smallest power of two >= 8 (N + 1), N the steps
 * done. The largest length the arena holds is the smallest power of two >= 8 max_records. */
lpc_status lpc_spectrum_length(const lpc_lattice *lat, int64_t *n_fft);

/* NMR spectrum, Eq. (9): the FID of `region` (-1: all regions) divided by its first sample,
 * zero-filled to n_fft points (a power of two >= N + 1 and <= the largest length; 0 selects
 * the default) and transformed with exp(-2 pi i k n / n_fft), so that a magnetisation
 * precessing by +theta per step peaks at f = theta / (2 pi dt). Writes n_fft values in
 * ascending frequency: ppm[j] = 1e6 f_j / larmor_hz with f_j = (j - n_fft/2) / (n_fft dt_s),
 * and the real and imaginary parts. LPC_ERR_STATE if the FID is not tracked or starts at
 * zero. */
lpc_status lpc_spectrum(lpc_lattice *lat, int32_t region, int64_t n_fft, double *ppm, double *re,
                        double *im, int64_t cap);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops that must not allocate): the spectrum of lpc_spectrum for an FID already in device
 * memory, computed in a work area of the library's own instead of a lattice's arena.
 *  - fid: n_samples >= 1 complex samples on the device as interleaved (re, im) doubles. It
 *    is divided by its first sample (a first sample of zero gives non-finite output),
 *    zero-filled to n_fft points and transformed with exp(-2 pi i k n / n_fft) (Eq. (9)).
 *  - n_fft: a power of two >= n_samples and <= 2^20; 0 selects the smallest power of two
 *    >= 8 n_samples, which must then be <= 2^20.
 *  - spec: 2 n_fft doubles on the device: the real parts in ascending frequency, then the
 *    imaginary parts; bin j is at f_j = (j - n_fft/2) / (n_fft dt), as in lpc_spectrum.
 * Queued on `stream` (hipStream_t as void*) and asynchronous. The work area is one static
 * device array of 2^21 complex doubles (32 MiB) per device, held from the library's load
 * until the process ends; nothing is allocated or freed. Every call on a device uses the
 * same area, and each call writes it entirely before reading it: calls that overlap in
 * time on one device (on different streams, or from several threads) race and must be
 * serialised by the caller. LPC_ERR_ARG for NULL buffers, n_samples < 1, or n_fft not a
 * power of two >= n_samples; LPC_ERR_OOM for n_fft beyond 2^20. */
lpc_status lpc_spectrum_noalloc(const double *fid, int64_t n_samples, int64_t n_fft, double *spec,
                                void *stream);

/* Position in ppm of the maximum of Re F of the default-length spectrum, refined by the
 * vertex of the parabola through the highest bin and its two neighbours. */
lpc_status lpc_spectrum_peak(lpc_lattice *lat, int32_t region, double *peak_ppm);

/* Diffusion coefficient per axis from the slope of the mean-square displacement between
 * steps N/2 and N (the long-time form of Eqs. (6)-(7)): D_a = a^2 (MSD_a(N) - MSD_a(N/2)) /
 * (2 (N - N/2) dt_s) in m^2/s, and ratio_a = D_a / D_bulk with D_bulk = p_hop a^2 / dt_s, the
 * free-lattice value. Needs LPC_TRACK_MSD and N >= 2; 3 values each. */
lpc_status lpc_diffusion(lpc_lattice *lat, double *D_m2_s, double *ratio);

/* Discrete velocity autocorrelation of Eq. (4) per axis, C(0) = <dx_1^2> and
 * C(tau) = <dx_1 dx_{1+tau}> per particle of the start, for tau = 0..N-1. With
 * LPC_TRACK_VACF it is measured directly: every particle carries its first displacement in a
 * tag field (set on the first step after a start, then moved like a population), and each
 * step records sum_i V_a,i v_a(i), where v_a(i) is the mean displacement of the next move
 * from site i (on the first step, sum_i rho_i <dx_a^2>_i); C is that record over the initial
 * population. Without it, C is taken from the recorded mean-square displacement through the
 * identity of a stationary increment process, MSD(t) = t C(0) + 2 sum_{tau=1}^{t-1} (t - tau)
 * C(tau): C(0) = MSD(1) - MSD(0), C(tau) = (MSD(tau+1) - 2 MSD(tau) + MSD(tau-1)) / 2. Both
 * are meant for runs started from equilibrium (Boltzmann start, or after lpc_equilibrate),
 * where the two agree; the tags need no stationarity. The Kohn estimate of Eq. (4)
 * truncated at lag T is D_a(T) = a^2 [C(0)/2 + sum_{tau=1}^{T} C(tau)] / dt_s. Writes N rows
 * of 3 values (lattice units^2); needs LPC_TRACK_MSD and N >= 2. */
lpc_status lpc_read_vacf(lpc_lattice *lat, double *vacf_xyz, int64_t cap, int64_t *len);

/* Kohn estimate of the diffusion coefficient, Eq. (4) (section 2.2): the discrete velocity
 * autocorrelation of lpc_read_vacf summed up to lag T, D_a(T) = a^2 [C_a(0)/2 +
 * sum_{tau=1}^{T} C_a(tau)] / dt_s per axis, in m^2/s (3 values). lag = -1 takes every
 * recorded lag (T = N - 1); otherwise 0 <= lag <= N - 1. Valid for runs started from
 * equilibrium, as lpc_read_vacf. Needs LPC_TRACK_MSD and N >= 2. */
lpc_status lpc_kohn_diffusion(lpc_lattice *lat, int64_t lag, double *D_m2_s);

/* Attempt probability per neighbour for a mean residence time tau_s on a free site (the
 * residence times of section 4): a particle on a site with six accessible neighbours of
 * equal free energy leaves with probability 6 p_hop per step, so its stay is geometric with
 * mean dt_s / (6 p_hop), and p_hop = dt_s / (6 tau_s). Host-only. LPC_ERR_ARG unless
 * tau_s >= dt_s > 0 (both finite), or for a NULL p_hop. */
lpc_status lpc_p_hop_from_residence_time(double tau_s, double dt_s, double *p_hop);

/* Per-part diffusion coefficients (section 4, Table 1) from two tables of lpc_region_moments
 * taken steps_between >= 1 steps apart (sums_a first, sums_b later; 7 values per region, as
 * lpc_region_moments writes them). For region r the mean-square displacement of the
 * particles now in it is MSD_r,a = sum M2_a / sum rho over its sites; its slope per step,
 * averaged over the axes whose bit is set in `axes` (bit a for axis a, 1..7), gives
 * D_r = spacing_m^2 slope / (2 dt_s) in m^2/s and ratio_r = slope / (2 p_hop), the
 * free-lattice value being 1 (Eq. (7)). Writes n_regions values to each of D_m2_s and
 * ratio. Host-only. LPC_ERR_ARG for NULL arrays, n_regions outside 1..LPC_MAX_REGIONS,
 * steps_between < 1, axes outside 1..7, or p_hop, dt_s, spacing_m not positive and finite;
 * LPC_ERR_STATE if a region holds no population in either table. */
lpc_status lpc_region_diffusion(const double *sums_a, const double *sums_b, int32_t n_regions,
                                int64_t steps_between, double p_hop, double dt_s,
                                double spacing_m, uint32_t axes, double *D_m2_s, double *ratio);

/* Per-region sums over the current state, 7 per region r < n_regions: the population and
 * the first and second displacement moments along x, y, z (moment propagation, section
 * 2.2): sums[7 r + q], q = 0 rho, 1..3 M1_x..z, 4..6 M2_x..z. M2 / rho of a region is the
 * mean-square displacement of the particles now in it, from which per-part diffusion
 * coefficients follow (section 4, Table 1). Needs LPC_TRACK_MSD; cap >= 7 n_regions.
 * Deterministic (fixed summation order). Synchronous. */
lpc_status lpc_region_moments(lpc_lattice *lat, double *sums, int64_t cap);

/* Populations of the current state summed over the planes perpendicular to `axis`
 * (0 x, 1 y, 2 z): n[axis] values (the uptake profile across a film along x). */
lpc_status lpc_uptake_profile(lpc_lattice *lat, int32_t axis, double *profile, int64_t cap);

/* Checkpoint: the state arrays, step counter and records, into / from host memory.
 * With buf == NULL, save reports the size needed in *len. Load requires a lattice of
 * the same configuration; fields are not part of the checkpoint. */
lpc_status lpc_save_state(lpc_lattice *lat, void *buf, size_t cap, size_t *len);
lpc_status lpc_load_state(lpc_lattice *lat, const void *buf, size_t len);

/* Batches: many lattices stepped together (independent particles of different sizes).
 * Every step is one launch per tile width covering the tiles of all lattices that still
 * have steps left, replayed from captured graphs (lpc_batch_use_graph); each lattice keeps
 * its own tiles and reduction order, so its state and records end bit for bit as if it had
 * been run alone with lpc_run on its one-step plan. */

/* Device bytes the work tables of a batch of `count` lattices need. */
lpc_status lpc_batch_query_footprint(int32_t count, size_t *bytes);

/* Groups `count` lattices (same device, precision and track set; any sizes, boundaries
 * and region counts) in the caller's arena (>= footprint bytes, 256-byte aligned). The
 * batch borrows the lattices: they must stay alive, and must not be stepped on their own,
 * while the batch is in use. Work goes to `stream` (hipStream_t as void*). */
lpc_status lpc_batch_create(lpc_lattice *const *lats, int32_t count, void *arena, size_t bytes,
                            void *stream, lpc_batch **out);
lpc_status lpc_batch_destroy(lpc_batch *batch);

/* Advances lattice l by n_steps[l] >= 0 steps (count values). All lattices must be
 * initialised and have record room for their steps (LPC_ERR_STATE otherwise; nothing is
 * queued then). Synchronizes the stream each time the set of lattices still stepping
 * changes (to rewrite the work tables); otherwise asynchronous. */
lpc_status lpc_batch_run(lpc_batch *batch, const int64_t *n_steps);

/* Whether lpc_batch_run replays captured graphs (enable != 0, the default) or launches every
 * step itself. With graphs, the launches of one chunk of steps (an even number, up to the
 * steps whose partial sums the lattices hold together) are recorded once per phase (a stretch
 * in which the set of lattices still stepping does not change) into a HIP graph, which is
 * then launched once per chunk on the batch's stream; the remaining steps of a phase are
 * launched directly. The kernels, their arguments and their order are the same either way,
 * so the results are bit for bit the same. */
lpc_status lpc_batch_use_graph(lpc_batch *batch, int32_t enable);

/* The batch's launch mode and counters (chunks replayed from graphs, steps launched
 * directly) as text, NUL-terminated and truncated to cap bytes. */
lpc_status lpc_batch_describe(const lpc_batch *batch, char *buf, size_t cap);

/* Calibration utility: copies `bytes` bytes from device buffer src to device buffer dst
 * (16-byte aligned, non-overlapping) with a plain streaming kernel on `stream`, so that
 * achieved HBM bandwidth and hardware traffic counters can be compared with a kernel of
 * known traffic (bytes read + bytes written = 2 * bytes). Asynchronous. */
lpc_status lpc_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

/* Calibration utility: the memory pattern of the FP64 sweep with FID and moments, without
 * its arithmetic. in[0..11] and out[0..8] are device arrays of nx * ny * nz doubles (x
 * fastest); outputs must not overlap any array. Workgroups take 64 x 4 blocks of columns
 * and runs of zc planes; each thread reads the 12 values of its column one plane ahead and
 * writes 9 past the caches, with one barrier per plane, as the sweep does (minus its halo
 * and its arithmetic). out[k] = in[k] + in[9] + in[10] * in[11]. Bytes moved are
 * 21 * 8 * nx * ny * nz: the bandwidth this pattern allows, against which the sweep's
 * counter traffic can be set. LPC_ERR_ARG on NULL arrays, overlapping outputs, sizes or zc
 * below 1, or a grid beyond 2^31 - 1 workgroups. Asynchronous on `stream`. */
lpc_status lpc_stream_columns(const double *const *in, double *const *out, int32_t nx,
                              int32_t ny, int32_t nz, int32_t zc, void *stream);

/* Calibration utility: the same for the mixed path with FID and moments. Reads rho_in
 * (doubles), in[0..9] (floats: 8 state arrays, free energy, shift) and region (bytes);
 * writes rho_out (doubles) and out[0..7] (floats); nx * ny * nz values each, outputs
 * overlapping no array. e = in[8] + in[9] * region (float); rho_out = rho_in + e and
 * out[k] = in[k] + e. Bytes moved are 89 * nx * ny * nz, the mixed sweep's algorithmic
 * count. Errors and stream as for lpc_stream_columns. */
lpc_status lpc_stream_columns_mixed(const double *rho_in, const float *const *in,
                                    const uint8_t *region, double *rho_out, float *const *out,
                                    int32_t nx, int32_t ny, int32_t nz, int32_t zc, void *stream);

/* tile_x of lpc_set_plan for linear tiles: each workgroup takes 256 consecutive sites of
 * the x-y plane (x fastest) instead of a block of columns, so a narrow lattice leaves
 * almost no lane idle. Available up to an nx that depends on the precision and track set
 * (the LDS window holds 256 + 2 nx sites), and not for lattices with a mobility field or a
 * reservoir axis. */
#define LPC_TILE_LINEAR 1

/* tile_x of lpc_set_plan for temporal blocking, two steps per sweep pass: each pass reads
 * the state and the fields once and writes the state once for two steps, so a step moves
 * about half the HBM bytes of a one-step pass. A workgroup takes the first step on a block of
 * 32 x 8 columns and the second on the inner 30 x 6 columns it owns (the first step of the
 * ring is repeated by the neighbouring tiles). The state after any number of steps is bit
 * for bit that of one step per pass; the per-step sums are taken over other tiles and agree
 * to rounding. A run of an odd number of steps ends with a one-step pass. Available for the
 * plain variant (no mobility field, no reservoir axis); batches step one step per pass. */
#define LPC_TILE_TWO_STEP 2

/* Widest x extent (nx) that lattices of this configuration's precision, track set and
 * variant can run on linear tiles, in *max_nx (0: none; lattices with a mobility field or a
 * reservoir axis run block tiles only). Host-only: needs no device. LPC_ERR_ARG for an
 * invalid configuration or NULL max_nx. */
lpc_status lpc_query_linear_tiles(const lpc_config *cfg, int32_t *max_nx);

/* Overrides the launch plan of the sweep: tile_x 64, 32 or 16 columns per tile row,
 * LPC_TILE_LINEAR, LPC_TILE_TWO_STEP (two steps per pass), or 0 (automatic: one step per
 * pass, the block width with the least padding in x within 1.5x, or linear tiles where they
 * leave fewer lanes idle and are available), and zc planes per workgroup (0: chosen from the
 * device's resident workgroups). Any plan computes the
 * same step; the plan fixes the order of the per-step sums, so results are bitwise
 * reproducible for a given plan and agree to rounding across plans. LPC_ERR_ARG if the
 * plan's partial sums do not fit the arena, or linear tiles are asked for where they are
 * not available. */
lpc_status lpc_set_plan(lpc_lattice *lat, int32_t tile_x, int32_t zc);

/* Launch plan of the sweep as text (tile shape, z-chunk, workgroups, steps finalised
 * together), NUL-terminated and truncated to cap bytes. */
lpc_status lpc_describe(const lpc_lattice *lat, char *buf, size_t cap);

const char *lpc_last_error(void);
const char *lpc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LPC_H */
