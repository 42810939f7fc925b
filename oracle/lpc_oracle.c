/*
 * Plain FP64 CPU oracle for the LPC3D lattice sweep. TEST INFRASTRUCTURE ONLY: it is
 * called by the tests, by the entry point's smoke check and by the benchmark's CPU
 * baseline, never by the library. It shares no code with the GPU path.
 *
 * What one time step computes (LPC3D paper, section 2, "Description of the model"
 * and "NMR spectra"; section 3.1, Eqs. (10)-(13)):
 *
 *  - Hop probability from site i to nearest neighbour j (simple cubic lattice, six
 *    neighbours): p(i->j) = p0 * P(i->j), where P is the Metropolis acceptance of
 *    Eq. (1): exp(-(F_j - F_i)) if F_j > F_i, else 1 (F in units of kT). p0 is the
 *    per-neighbour attempt probability (alpha / 6 in the notation of Eq. (7)).
 *  - A particle that does not hop stays (Fig. 1 caption): stay(i) = 1 - sum_j p(i->j),
 *    where attempts across a closed face have no target and count as staying.
 *  - Populations (densities, not particles; end of section 2.1):
 *        rho'_i = stay(i) rho_i + sum_j p(j->i) rho_j.
 *  - Magnetisation, Eq. (13) in 3-D with the stay term: gather first, then rotate by
 *    the destination's phase per step theta_i = 2 pi delta_i 1e-6 nu0 dt (Eq. (11)):
 *        m'_i = exp(i theta_i) [ stay(i) m_i + sum_j p(j->i) m_j ].
 *  - Displacement moments (moment propagation, section 2.2) per axis a, with d_a the
 *    unwrapped a-component of the hop vector j -> i:
 *        M1'_i = stay(i) M1_i + sum_j p(j->i) (M1_j + d_a rho_j)
 *        M2'_i = stay(i) M2_i + sum_j p(j->i) (M2_j + 2 d_a M1_j + d_a^2 rho_j).
 *  - Records after every step (and before the first), Eqs. (11)-(12): per region r the
 *    sums of m (real, imaginary) and rho, and over all sites the sums of M1_a, M2_a.
 *    Record layout, K = 3R + 6 doubles: [Re G_r, Im G_r] for r < R, then U_r for r < R,
 *    then S1_x, S1_y, S1_z, S2_x, S2_y, S2_z.
 *
 * Boundaries: a periodic axis wraps the neighbour index (the hop vector stays +-1); a
 * closed axis has no neighbour beyond its faces. A reservoir axis (Dirichlet ghost layer,
 * section 3.2, item "Input reading and initialization") has beyond each face a ghost site
 * whose values are fixed: free energy F_g, population rho_g, magnetisation m_g, zero
 * displacement moments. Moves into the ghost leave the lattice; moves out of it bring
 * p(g->i) times the ghost's values in. The lattice total is then not conserved.
 *
 * Inaccessible sites (section 2.1 and Fig. 1): a site whose free energy is +infinity is
 * part of the solid matrix. It holds nothing, and a move attempted towards it is rejected
 * (the particle stays), as is the zero acceptance into obstacles in Eq. (5).
 *
 * Link mobility (section 2.2, after Eq. (7)): with a per-site factor mu_i in [0, 1] the
 * link i-j gets alpha_ij = min(mu_i, mu_j), the same for both directions so that detailed
 * balance (and with it the Boltzmann equilibrium of Eq. (2)) is kept; both hop
 * probabilities of the link are multiplied by it. A ghost site has mobility 1.
 *
 * Plain loops over z, y, x; OpenMP splits z-planes only. Record sums are taken per
 * z-plane in index order and then over planes in order, so results do not depend on
 * the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_PERIODIC 0
#define ORACLE_CLOSED 1
#define ORACLE_RESERVOIR 2

static const int HOP[6][3] = {
    {+1, 0, 0}, {-1, 0, 0}, {0, +1, 0}, {0, -1, 0}, {0, 0, +1}, {0, 0, -1}};

/* Metropolis acceptance of a move from free energy Fi to Fj (kT units), Eq. (1). */
static double acceptance(double Fi, double Fj)
{
    if (Fj > Fi)
        return exp(-(Fj - Fi));
    return 1.0;
}

typedef struct {
    int64_t n[3];
    int bc[3];
} geometry;

/* Index of the neighbour of (x, y, z) one hop along direction d; -1 across a closed face;
 * -2 - f across reservoir face f = 2 * axis + (0 low, 1 high). */
static int64_t neighbour(const geometry *g, int64_t x, int64_t y, int64_t z, int d)
{
    int64_t c[3] = {x + HOP[d][0], y + HOP[d][1], z + HOP[d][2]};
    for (int a = 0; a < 3; ++a) {
        if (c[a] < 0 || c[a] >= g->n[a]) {
            if (g->bc[a] == ORACLE_CLOSED)
                return -1;
            if (g->bc[a] == ORACLE_RESERVOIR)
                return -2 - (2 * a + (c[a] < 0 ? 0 : 1));
            c[a] = (c[a] + g->n[a]) % g->n[a];
        }
    }
    return c[0] + g->n[0] * (c[1] + g->n[1] * c[2]);
}

static int blocked(double F) { return isinf(F) && F > 0.0; }

/* Site-independent extras of a run: per-site mobility (NULL: all 1) and the ghost values of
 * the six faces, ghost[4 * f + k] with k = F, rho, Re m, Im m (NULL: no reservoir face). */
typedef struct {
    const double *mobility;
    const double *ghost;
} extras;

typedef struct {
    double *rho, *re, *im, *M1, *M2; /* M1, M2: 3 blocks of n (axis-major) or NULL */
} state;

static void one_step(const geometry *g, double p0, const double *F, const double *cos_t,
                     const double *sin_t, const extras *ex, const state *s, state *o)
{
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const int64_t n = nx * ny * nz;
    const int moments = s->M1 != NULL;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z) {
        for (int64_t y = 0; y < ny; ++y) {
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t i = x + nx * (y + ny * z);
                if (blocked(F[i])) { /* solid matrix: holds nothing */
                    o->rho[i] = o->re[i] = o->im[i] = 0.0;
                    if (moments)
                        for (int a = 0; a < 3; ++a)
                            o->M1[a * n + i] = o->M2[a * n + i] = 0.0;
                    continue;
                }
                double out = 0.0;
                double in_rho = 0.0, in_re = 0.0, in_im = 0.0;
                double in1[3] = {0.0, 0.0, 0.0}, in2[3] = {0.0, 0.0, 0.0};
                for (int d = 0; d < 6; ++d) {
                    const int64_t j = neighbour(g, x, y, z, d);
                    if (j == -1)
                        continue; /* attempt across a closed face: the particle stays */
                    /* the neighbour's values: a lattice site or a fixed ghost site */
                    double Fj, rj, rej, imj, alpha = 1.0;
                    double m1j[3] = {0.0, 0.0, 0.0}, m2j[3] = {0.0, 0.0, 0.0};
                    if (j >= 0) {
                        Fj = F[j];
                        if (blocked(Fj))
                            continue; /* attempt towards an obstacle: the particle stays */
                        rj = s->rho[j];
                        rej = s->re[j];
                        imj = s->im[j];
                        if (moments)
                            for (int a = 0; a < 3; ++a) {
                                m1j[a] = s->M1[a * n + j];
                                m2j[a] = s->M2[a * n + j];
                            }
                        if (ex->mobility)
                            alpha = fmin(ex->mobility[i], ex->mobility[j]);
                    } else {
                        const double *gh = ex->ghost + 4 * (-2 - j);
                        Fj = gh[0];
                        rj = gh[1];
                        rej = gh[2];
                        imj = gh[3];
                        if (ex->mobility)
                            alpha = fmin(ex->mobility[i], 1.0);
                    }
                    const double p_out = p0 * alpha * acceptance(F[i], Fj); /* i -> j */
                    const double p_in = p0 * alpha * acceptance(Fj, F[i]);  /* j -> i */
                    out += p_out;
                    in_rho += p_in * rj;
                    in_re += p_in * rej;
                    in_im += p_in * imj;
                    if (moments) {
                        for (int a = 0; a < 3; ++a) {
                            const double da = -HOP[d][a]; /* the move j -> i goes against d */
                            in1[a] += p_in * (m1j[a] + da * rj);
                            in2[a] += p_in * (m2j[a] + 2.0 * da * m1j[a] + da * da * rj);
                        }
                    }
                }
                const double stay = 1.0 - out;
                o->rho[i] = stay * s->rho[i] + in_rho;
                const double gre = stay * s->re[i] + in_re;
                const double gim = stay * s->im[i] + in_im;
                o->re[i] = gre * cos_t[i] - gim * sin_t[i];
                o->im[i] = gre * sin_t[i] + gim * cos_t[i];
                if (moments) {
                    for (int a = 0; a < 3; ++a) {
                        o->M1[a * n + i] = stay * s->M1[a * n + i] + in1[a];
                        o->M2[a * n + i] = stay * s->M2[a * n + i] + in2[a];
                    }
                }
            }
        }
    }
}

static void record(const geometry *g, const uint8_t *region, int R, const state *s,
                   double *plane_buf, double *rec)
{
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const int64_t n = nx * ny * nz, plane = nx * ny;
    const int K = 3 * R + 6;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z) {
        double *acc = plane_buf + z * K;
        for (int k = 0; k < K; ++k)
            acc[k] = 0.0;
        for (int64_t q = 0; q < plane; ++q) {
            const int64_t i = z * plane + q;
            const int r = region[i];
            acc[2 * r] += s->re[i];
            acc[2 * r + 1] += s->im[i];
            acc[2 * R + r] += s->rho[i];
            if (s->M1 != NULL) {
                for (int a = 0; a < 3; ++a) {
                    acc[3 * R + a] += s->M1[a * n + i];
                    acc[3 * R + 3 + a] += s->M2[a * n + i];
                }
            }
        }
    }
    for (int k = 0; k < K; ++k)
        rec[k] = 0.0;
    for (int64_t z = 0; z < nz; ++z)
        for (int k = 0; k < K; ++k)
            rec[k] += plane_buf[z * K + k];
}

int lpc_oracle_record_width(int n_regions) { return 3 * n_regions + 6; }

int lpc_oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Runs n_steps steps from the state held in rho, re, im (and M1, M2 when non-NULL; each
 * 3*n doubles, axis-major), overwriting it with the final state. records receives
 * (n_steps + 1) * (3 R + 6) doubles: the record of the initial state, then one per step.
 * Returns 0 on success, 1 on a bad argument, 2 when memory runs out.
 */
static int bad_extras(const int32_t *bc, const double *ghost)
{
    for (int a = 0; a < 3; ++a) {
        if (bc[a] < ORACLE_PERIODIC || bc[a] > ORACLE_RESERVOIR)
            return 1;
        if (bc[a] == ORACLE_RESERVOIR && !ghost)
            return 1;
    }
    return 0;
}

int lpc_oracle_run(int64_t nx, int64_t ny, int64_t nz, const int32_t *bc, double p0,
                   double dt_s, double larmor_hz, const double *F, const double *delta_ppm,
                   const uint8_t *region, int32_t n_regions, const double *mobility,
                   const double *ghost, double *rho, double *re, double *im, double *M1,
                   double *M2, int64_t n_steps, double *records)
{
    if (nx < 1 || ny < 1 || nz < 1 || n_regions < 1 || n_steps < 0 || !F || !delta_ppm ||
        !region || !rho || !re || !im || !records || ((M1 == NULL) != (M2 == NULL)) ||
        bad_extras(bc, ghost))
        return 1;
    geometry g = {{nx, ny, nz}, {bc[0], bc[1], bc[2]}};
    const extras ex = {mobility, ghost};
    const int64_t n = nx * ny * nz;
    const int K = 3 * n_regions + 6;
    const int moments = M1 != NULL;
    double *cos_t = malloc(sizeof(double) * n), *sin_t = malloc(sizeof(double) * n);
    double *plane_buf = malloc(sizeof(double) * nz * K);
    state a = {rho, re, im, M1, M2};
    state b = {malloc(sizeof(double) * n), malloc(sizeof(double) * n),
               malloc(sizeof(double) * n), moments ? malloc(sizeof(double) * 3 * n) : NULL,
               moments ? malloc(sizeof(double) * 3 * n) : NULL};
    int rc = 0;
    if (!cos_t || !sin_t || !plane_buf || !b.rho || !b.re || !b.im ||
        (moments && (!b.M1 || !b.M2))) {
        rc = 2;
        goto done;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (region[i] >= n_regions) {
            rc = 1;
            goto done;
        }
        /* phase accumulated in one step at the site's Larmor offset, Eq. (11) */
        const double theta = 2.0 * M_PI * delta_ppm[i] * 1e-6 * larmor_hz * dt_s;
        cos_t[i] = cos(theta);
        sin_t[i] = sin(theta);
    }
    record(&g, region, n_regions, &a, plane_buf, records);
    state *cur = &a, *nxt = &b;
    for (int64_t t = 1; t <= n_steps; ++t) {
        one_step(&g, p0, F, cos_t, sin_t, &ex, cur, nxt);
        record(&g, region, n_regions, nxt, plane_buf, records + t * K);
        state *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    if (cur != &a) {
        memcpy(a.rho, cur->rho, sizeof(double) * n);
        memcpy(a.re, cur->re, sizeof(double) * n);
        memcpy(a.im, cur->im, sizeof(double) * n);
        if (moments) {
            memcpy(a.M1, cur->M1, sizeof(double) * 3 * n);
            memcpy(a.M2, cur->M2, sizeof(double) * 3 * n);
        }
    }
done:
    free(cos_t);
    free(sin_t);
    free(plane_buf);
    free(b.rho);
    free(b.re);
    free(b.im);
    free(b.M1);
    free(b.M2);
    return rc;
}

/*
 * Equilibration phase (section 3.2, item "Equilibration process"): populations alone are
 * stepped until they stop changing, max_i |rho_i(t+1) - rho_i(t)| <= tol * max_i rho_i(t+1),
 * or until max_steps. rho holds the start and receives the result; *steps the number of steps
 * taken and *residual the last relative change. Returns 0, 1 (bad argument) or 2 (memory).
 */
int lpc_oracle_equilibrate(int64_t nx, int64_t ny, int64_t nz, const int32_t *bc, double p0,
                           const double *F, const double *mobility, const double *ghost,
                           double *rho, double tol, int64_t max_steps, int64_t *steps,
                           double *residual)
{
    if (nx < 1 || ny < 1 || nz < 1 || !F || !rho || !steps || !residual || max_steps < 0 ||
        bad_extras(bc, ghost))
        return 1;
    geometry g = {{nx, ny, nz}, {bc[0], bc[1], bc[2]}};
    const extras ex = {mobility, ghost};
    const int64_t n = nx * ny * nz;
    double *zeros = calloc((size_t)n, sizeof(double));
    double *ones = malloc(sizeof(double) * n);
    double *b = malloc(sizeof(double) * n), *tmp_re = malloc(sizeof(double) * n),
           *tmp_im = malloc(sizeof(double) * n), *re = calloc((size_t)n, sizeof(double)),
           *im = calloc((size_t)n, sizeof(double));
    if (!zeros || !ones || !b || !tmp_re || !tmp_im || !re || !im) {
        free(zeros); free(ones); free(b); free(tmp_re); free(tmp_im); free(re); free(im);
        return 2;
    }
    for (int64_t i = 0; i < n; ++i)
        ones[i] = 1.0;
    state cur = {rho, re, im, NULL, NULL}, nxt = {b, tmp_re, tmp_im, NULL, NULL};
    double res = INFINITY;
    int64_t t = 0;
    while (t < max_steps) {
        one_step(&g, p0, F, ones, zeros, &ex, &cur, &nxt);
        ++t;
        double dmax = 0.0, rmax = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            const double d = fabs(nxt.rho[i] - cur.rho[i]);
            dmax = d > dmax ? d : dmax;
            rmax = nxt.rho[i] > rmax ? nxt.rho[i] : rmax;
        }
        res = rmax > 0.0 ? dmax / rmax : 0.0;
        state tmp = cur;
        cur = nxt;
        nxt = tmp;
        if (res <= tol)
            break;
    }
    if (cur.rho != rho)
        memcpy(rho, cur.rho, sizeof(double) * n);
    *steps = t;
    *residual = res;
    free(zeros);
    free(ones);
    free(b);
    free(tmp_re);
    free(tmp_im);
    free(re);
    free(im);
    return 0;
}

/*
 * Velocity autocorrelation of Eq. (4) (section 2.2) by moment propagation, independent of
 * the displacement moments: C_a(tau) = <dx_a(1) dx_a(1 + tau)>, summed over the particles of
 * the start rho (not normalised), tau = 0 .. n_lags - 1, for each axis a.
 *  - C_a(0) = sum_i rho_i sum_j p(i->j) d_a(i->j)^2: the mean square of one step.
 *  - A tag field carries each particle's first displacement: after the first step
 *    V_a,i = sum_j p(j->i) d_a(j->i) rho_j (d_a of the move j -> i), and every later step
 *    moves it like a population, V_a,i' = stay(i) V_a,i + sum_j p(j->i) V_a,j. A reservoir
 *    ghost holds no tagged particle; moves into a ghost take their tag out of the lattice.
 *  - After tau steps the tagged particles at i make their next move with mean displacement
 *    v_a(i) = sum_j p(i->j) d_a(i->j), so C_a(tau) = sum_i V_a,i(tau) v_a(i) for tau >= 1.
 * rho (n values) is not modified. C receives n_lags * 3 values (row tau: x, y, z).
 * Returns 0, 1 (bad argument) or 2 (memory).
 */
int lpc_oracle_vacf(int64_t nx, int64_t ny, int64_t nz, const int32_t *bc, double p0,
                    const double *F, const double *mobility, const double *ghost,
                    const double *rho, int64_t n_lags, double *C)
{
    if (nx < 1 || ny < 1 || nz < 1 || !F || !rho || !C || n_lags < 1 || bad_extras(bc, ghost))
        return 1;
    geometry g = {{nx, ny, nz}, {bc[0], bc[1], bc[2]}};
    const int64_t n = nx * ny * nz;
    double *V = calloc((size_t)(3 * n), sizeof(double));
    double *W = malloc(sizeof(double) * 3 * n);
    double *vel = malloc(sizeof(double) * 3 * n);   /* v_a(i) */
    double *msq = malloc(sizeof(double) * 3 * n);   /* sum_j p(i->j) d_a^2 */
    double *stay = malloc(sizeof(double) * n);
    if (!V || !W || !vel || !msq || !stay) {
        free(V); free(W); free(vel); free(msq); free(stay);
        return 2;
    }
    /* per site: the mean displacement and mean square displacement of its next move, and
     * its staying probability */
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t i = x + nx * (y + ny * z);
                double out = 0.0;
                for (int a = 0; a < 3; ++a)
                    vel[a * n + i] = msq[a * n + i] = 0.0;
                if (!blocked(F[i]))
                    for (int d = 0; d < 6; ++d) {
                        const int64_t j = neighbour(&g, x, y, z, d);
                        if (j == -1 || (j >= 0 && blocked(F[j])))
                            continue;
                        const double Fj = j >= 0 ? F[j] : ghost[4 * (-2 - j)];
                        double alpha = 1.0;
                        if (mobility)
                            alpha = fmin(mobility[i], j >= 0 ? mobility[j] : 1.0);
                        const double p = p0 * alpha * acceptance(F[i], Fj);
                        out += p;
                        for (int a = 0; a < 3; ++a) {
                            vel[a * n + i] += p * HOP[d][a];
                            msq[a * n + i] += p * HOP[d][a] * HOP[d][a];
                        }
                    }
                stay[i] = 1.0 - out;
            }
    for (int a = 0; a < 3; ++a) {
        double c0 = 0.0;
        for (int64_t i = 0; i < n; ++i)
            c0 += rho[i] * msq[a * n + i];
        C[a] = c0;
    }
    /* gathers V' from V (first: the tagging step, with the displacement source d rho) */
    for (int64_t tau = 1; tau < n_lags; ++tau) {
        const int first = tau == 1;
#pragma omp parallel for schedule(static)
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    const int64_t i = x + nx * (y + ny * z);
                    double in[3] = {0.0, 0.0, 0.0};
                    if (!blocked(F[i]))
                        for (int d = 0; d < 6; ++d) {
                            const int64_t j = neighbour(&g, x, y, z, d);
                            if (j < 0 || blocked(F[j]))
                                continue;   /* closed face, obstacle, or an untagged ghost */
                            double alpha = 1.0;
                            if (mobility)
                                alpha = fmin(mobility[i], mobility[j]);
                            const double p_in = p0 * alpha * acceptance(F[j], F[i]);
                            for (int a = 0; a < 3; ++a) {
                                const double src = first ? -HOP[d][a] * rho[j] : V[a * n + j];
                                in[a] += p_in * src;
                            }
                        }
                    for (int a = 0; a < 3; ++a)
                        W[a * n + i] = (first ? 0.0 : stay[i] * V[a * n + i]) + in[a];
                }
        double *t = V;
        V = W;
        W = t;
        for (int a = 0; a < 3; ++a) {
            double c = 0.0;
            for (int64_t i = 0; i < n; ++i)
                c += V[a * n + i] * vel[a * n + i];
            C[3 * tau + a] = c;
        }
    }
    free(V); free(W); free(vel); free(msq); free(stay);
    return 0;
}
