// Lattice sweep kernels for gfx950 (MI355X).
//
// One step of the LPC3D lattice model (paper section 2; Eqs. (1), (11)-(13) and moment
// propagation of section 2.2) for populations rho, complex magnetisation m and per-axis
// displacement moments M1, M2, plus the per-step sums over sites of Eqs. (11)-(12).
//
// Per site i the step gathers from the six neighbours j with the hop probabilities of
// Eq. (1), p(i->j) = p0 min(1, e^{F_i - F_j}), and keeps the staying fraction
// stay(i) = 1 - P_out(i), P_out(i) = sum_j p(i->j). The float path takes one exponential
// per link for both directions (p0 e^{-|dF|} one way, p0 the other). The FP64 path turns
// each cell's free energy into the two factors E = e^{F - c} and G = e^{c - F} once, at the
// cell's first use (c centres the accessible range), and a link's acceptances are the
// products E_i G_j and E_j G_i clipped at 1: two exponentials per loaded cell instead of
// one per link end. The two ends of a link form the same products, so they see the same
// probabilities bit for bit.
//     x'_i = stay(i) x_i + sum_j p(j->i) x_j'        (x_j' with the hop's displacement)
// Totals are only preserved step after step if stay(i) + P_out(i) is exactly one, so the
// rounding of P_out must not repeat the same bias every step:
//  - FP64 path: the population uses the flux form x'_i = x_i + sum_j [p(j->i) x_j -
//    p(i->j) x_i], whose per-link terms are exactly antisymmetric between the two ends
//    (both products rounded before the difference), so the total population is conserved
//    to rounding noise. Magnetisation and moments use the stay form (a 1e-16 bias per
//    step is far below any tolerance).
//  - Mixed path (float storage and float hop probabilities): P_out is summed in double. Six
//    floats add exactly in double while their exponents lie within about 29 binary orders
//    (free-energy steps up to about 20 kT among the links of a site), and stay(i) =
//    1 - P_out is then exact; beyond that span the smallest terms round, by at most 2^-53 of
//    the sum. The update stay * x_i + sum is finished in double before the one rounding to
//    float, so the rounding of each stored value is unbiased.
// Inaccessible sites (section 2.1, Fig. 1) carry a huge finite free energy, so the same
// arithmetic gives exact zero hop probabilities towards them, and they hold nothing. The
// extended kernel variant (EXT) adds link mobility, both probabilities of the link i-j
// scaled by min(mu_i, mu_j), and reservoir axes, where the neighbour beyond a face is a
// ghost cell of fixed values (F, rho, m, zero moments, mobility 1); lattices that use
// neither run the plain variant, which carries none of their registers.
// Magnetisation rotates after the gather by the destination's phase (Eq. (13)), applied
// as m + m (cos t - 1) + i m sin t with cos t - 1 evaluated without cancellation, which
// keeps |m| from drifting when t is stored in float.
//
// Per-step sums are deterministic: each workgroup reduces its sites with wave-level
// butterflies and a fixed-order pass over its waves into one partial per record entry,
// and a finalize kernel sums the partials of all workgroups in a fixed order. No
// floating-point atomics are used anywhere.
#include "lpc_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>

// The sweep's kernel instances are compiled in parts, one translation unit each, so that
// the build runs them in parallel: LPC_SWEEP_PART 0 and 1 hold the FP64 instances (plain,
// extended), 2 and 3 the float ones, and 4 the planning, the dispatch and every other
// kernel. Without the macro one unit holds everything.
#ifndef LPC_SWEEP_PART
#define LPC_SWEEP_PART -1
#endif
#define LPC_PART_IS(k) (LPC_SWEEP_PART < 0 || LPC_SWEEP_PART == (k))
#define LPC_HOST_PART LPC_PART_IS(4)

namespace lpc {
namespace {

constexpr int kWave = 64;

template <typename S>
struct View {
    double *rho;
    S *re, *im;
    S *m1[3], *m2[3];
    S *v[3];
};

template <typename S>
__host__ __device__ inline View<S> typed(const StateView &v)
{
    View<S> t;
    t.rho = v.rho;
    t.re = static_cast<S *>(v.re);
    t.im = static_cast<S *>(v.im);
    for (int a = 0; a < 3; ++a) {
        t.m1[a] = static_cast<S *>(v.m1[a]);
        t.m2[a] = static_cast<S *>(v.m2[a]);
        t.v[a] = static_cast<S *>(v.v[a]);
    }
    return t;
}

// Device global memory. Pointers that come from a work list in memory (not from kernel
// arguments) are generic to the compiler; addressing them as global keeps the loads off the
// flat path, whose completion would also be awaited by every LDS wait.
#define LPC_GLOBAL __attribute__((address_space(1)))

// Element at a 32-bit byte offset from a workgroup-uniform base: the base lives in scalar
// registers and the per-lane offset in one vector register.
template <typename T>
__device__ inline T ld(const T *base, uint32_t boff)
{
    const LPC_GLOBAL char *b = (const LPC_GLOBAL char *)base;
    return *(const LPC_GLOBAL T *)(b + boff);
}

// State arrays are written once per step and not read again within it: stream them past
// the caches.
template <typename T>
__device__ inline void st(T *base, uint32_t boff, T v)
{
    LPC_GLOBAL char *b = (LPC_GLOBAL char *)base;
    __builtin_nontemporal_store(v, (LPC_GLOBAL T *)(b + boff));
}

// Population flux of a link with both products rounded separately, so that the value
// computed at site j is exactly the negation of the one computed at site i.
__device__ inline double exact_flux(double p_in, double xj, double p_out, double xi)
{
#pragma clang fp contract(off)
    const double a = p_in * xj;
    const double b = p_out * xi;
    return a - b;
}

// Register accumulators of one thread's record contributions.
template <int MAXR>
struct RecAcc {
    double re[MAXR], im[MAXR], u[MAXR], s1[3], s2[3], c[3];

    __device__ void zero()
    {
#pragma unroll
        for (int r = 0; r < MAXR; ++r)
            re[r] = im[r] = u[r] = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            s1[a] = s2[a] = c[a] = 0.0;
    }

    __device__ void add_site(int r, double vre, double vim, double vu)
    {
        if (MAXR == 1) {
            re[0] += vre;
            im[0] += vim;
            u[0] += vu;
            return;
        }
        // Regions come in large blocks, so the sites of a wave mostly share one: the wave then
        // adds to that region's accumulators alone, behind a uniform branch. A wave that
        // straddles regions adds to every accumulator through selects. Adding zero leaves an
        // accumulator's bits unchanged (it starts at +0), so both forms give the same sums.
        const int r0 = __builtin_amdgcn_readfirstlane(r);
        if (__builtin_amdgcn_ballot_w64(r != r0) == 0) {
#pragma unroll
            for (int k = 0; k < MAXR; ++k) {
                if (k == r0) {
                    re[k] += vre;
                    im[k] += vim;
                    u[k] += vu;
                }
            }
            return;
        }
#pragma unroll
        for (int k = 0; k < MAXR; ++k) {
            const bool hit = k == r;
            re[k] += hit ? vre : 0.0;
            im[k] += hit ? vim : 0.0;
            u[k] += hit ? vu : 0.0;
        }
    }
};

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        v += __shfl_xor(v, off, kWave);
    return v;
}

// Record entries per region and after the regions: K = 3 R + 6, plus 3 with the velocity
// autocorrelation (moment template parameter 2).
__host__ __device__ constexpr int record_slots(int R, int MSD)
{
    return 3 * R + 6 + (MSD == 2 ? 3 : 0);
}

// Reduces the block's accumulators into partials[k * nblocks + blk], k < K, in a fixed
// order (butterfly inside each wave, then waves in index order).
template <int MAXR, int NWAVES, bool VAC = false>
__device__ void block_reduce(RecAcc<MAXR> &acc, int R, int K, double *partials, int64_t nblocks,
                             int64_t blk, double *lds)
{
    const int tid = threadIdx.x;
    const int lane = tid % kWave, wave = tid / kWave;
    auto push = [&](double v, int slot) {
        v = wave_sum(v);
        if (lane == 0)
            lds[wave * K + slot] = v;
    };
#pragma unroll
    for (int r = 0; r < MAXR; ++r) {
        if (r < R) {
            push(acc.re[r], 2 * r);
            push(acc.im[r], 2 * r + 1);
            push(acc.u[r], 2 * R + r);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        push(acc.s1[a], 3 * R + a);
        push(acc.s2[a], 3 * R + 3 + a);
    }
    if (VAC) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
            push(acc.c[a], 3 * R + 6 + a);
    }
    __syncthreads();
    if (tid < K) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NWAVES; ++w)
            t += lds[w * K + tid];
        partials[static_cast<int64_t>(tid) * nblocks + blk] = t;
    }
}

// Logical tile of a hardware workgroup id: XCD x (= b mod 8) gets the contiguous range
// [x * per, (x + 1) * per) of tiles, so halo-sharing neighbours mostly meet in one L2. Each
// XCD walks its range from a point x/8 of the way in (wrapping round), so that the XCDs do
// not stream the same rows of their z-chunks at the same time: with a power-of-two plane
// size those rows lie a multiple of a large power of two apart and meet in the same HBM
// channels (256^3 particle: +2 % mixed, +1.6 % FP64).
__device__ inline int64_t logical_block(int64_t b, int64_t padded)
{
    const int64_t per = padded / 8;
    const int64_t x = b % 8;
    return x * per + (b / 8 + x * per / 8) % per;
}

// ---------------------------------------------------------------------------- one site

// Values of one site that its neighbours read: population, free energy, magnetisation,
// displacement moments and (extended variant) mobility, in the storage type S (rho is
// always double).
template <typename S, bool FID, int MSD, bool EXT>
struct Cell {
    double rho;
    S F;      // FP64 path: free energy when loaded, then E = e^{F - c} once weighed
    S G;      // FP64 path: G = e^{c - F} once weighed
    S re, im;
    S m1[3], m2[3];
    S v[3];   // first-displacement tags (moment parameter 2)
    S mu;
};

// Whether the storage type's path works with per-cell Boltzmann factors (FP64) or with one
// exponential per link (float).
template <typename S>
struct PerCellWeights {
    static constexpr bool on = false;
};
template <>
struct PerCellWeights<double> {
    static constexpr bool on = true;
};

// Boltzmann factor E = e^{F - c} of a free energy on the FP64 path (c centres the accessible
// range). The sweep reads a field of these factors, set once per free-energy field by
// k_boltzmann_factors, instead of the free energies.
__device__ inline double boltzmann_factor(double F, double fc)
{
    return exp(F - fc);
}

// 1/e for the factors of the FP64 path: the hardware reciprocal estimate refined by two
// Newton-Raphson steps r <- r + r (1 - e r), each of which doubles its correct bits, to
// within an ulp or two of 1/e; e = inf (an inaccessible site) gives 0. The factors lie in
// [e^-700, e^700] (free-energy spans are capped at 1400 kT), where every step stays normal.
// One value per cell serves both ends of each of its links, so the acceptances of a link
// stay the same products at both ends whatever the last bits of 1/e.
__device__ inline double factor_reciprocal(double e)
{
    double r = __builtin_amdgcn_rcp(e);
    r = fma(r, fma(-e, r, 1.0), r);
    r = fma(r, fma(-e, r, 1.0), r);
    return __builtin_isinf(e) ? 0.0 : r;
}

// FP64 path: adds G = 1/E = e^{c - F} to a cell loaded with its factor E. An inaccessible site
// (sentinel F) has E = inf, so G = 0: zero acceptance towards it.
template <typename S, bool FID, int MSD, bool EXT>
__device__ inline void weigh(Cell<S, FID, MSD, EXT> &c, double)
{
    if (PerCellWeights<S>::on)
        c.G = static_cast<S>(factor_reciprocal(static_cast<double>(c.F)));
}

// Byte offsets of one column (or halo column) in the 8-byte, S-sized and 1-byte arrays.
struct Off {
    uint32_t b8, bs, b1;
};

// Loads the values of a site that its neighbours read.
template <typename S, bool FID, int MSD, bool EXT>
__device__ inline void load_cell(Cell<S, FID, MSD, EXT> &c, const View<S> &v, const S *F,
                                 const S *MU, int64_t pz, Off o)
{
    c.rho = ld(v.rho + pz, o.b8);
    c.F = ld(F + pz, o.bs);
    if (EXT)
        c.mu = MU ? ld(MU + pz, o.bs) : S(1);
    if (FID) {
        c.re = ld(v.re + pz, o.bs);
        c.im = ld(v.im + pz, o.bs);
    }
    if (MSD) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            c.m1[b] = ld(v.m1[b] + pz, o.bs);
            c.m2[b] = ld(v.m2[b] + pz, o.bs);
        }
    }
    if (MSD == 2) {
#pragma unroll
        for (int b = 0; b < 3; ++b)
            c.v[b] = ld(v.v[b] + pz, o.bs);
    }
}

// The fixed ghost site beyond reservoir face `face` (2 * axis + side): free energy,
// population and magnetisation from the table, zero moments, mobility 1; weighed.
template <typename S, bool FID, int MSD, bool EXT>
__device__ inline void ghost_cell(Cell<S, FID, MSD, EXT> &c, const double *ghost, int face,
                                  double fc)
{
    const double *v = ghost + 4 * face;
    c.F = PerCellWeights<S>::on ? static_cast<S>(boltzmann_factor(v[0], fc))
                                : static_cast<S>(v[0]);
    weigh(c, fc);
    c.rho = v[1];
    if (FID) {
        c.re = static_cast<S>(v[2]);
        c.im = static_cast<S>(v[3]);
    }
    if (MSD) {
#pragma unroll
        for (int b = 0; b < 3; ++b)
            c.m1[b] = c.m2[b] = c.v[b] = S(0);   // a ghost holds no tagged particle
    }
    if (EXT)
        c.mu = S(1);
}

// Gather accumulators of one site: sum_j p(j->i) x_j per field, the population term
// (flux sum on the FP64 path, gather sum on the mixed path) and P_out in double.
template <typename S>
struct Acc {
    double rho, pout;
    S re, im, m1[3], m2[3], v[3];
    double mv[3], ms[3];   // mean displacement and mean square of the site's next move
};

__device__ inline float fast_exp(float v)
{
    return __expf(v);
}

// Hop probabilities of one link in float, Eq. (1): p_out = p(i->j), p_in = p(j->i). The
// same (|dF|, direction) gives bit-identical values at both ends.
__device__ inline void link_pair(float Fi, float Fj, float p0, float &p_out, float &p_in)
{
    const float dF = Fj - Fi;
    const float pe = p0 * fast_exp(-(dF > 0.0f ? dF : -dF));
    const bool up = dF > 0.0f;
    p_out = up ? pe : p0;
    p_in = up ? p0 : pe;
}

// The same from the weighed cells of the FP64 path: the acceptance of i -> j is
// min(1, e^{F_i - F_j}) = min(1, E_i G_j). The clip is written so that a product that is
// not a number (only between two inaccessible sites, which hold nothing) gives 1.
__device__ inline void link_pair_weighed(double Ei, double Gi, double Ej, double Gj, double p0,
                                         double &p_out, double &p_in)
{
    const double ro = Ei * Gj, ri = Ej * Gi;
    p_out = p0 * (ro < 1.0 ? ro : 1.0);
    p_in = p0 * (ri < 1.0 ? ri : 1.0);
}

// Gathers the fields arriving over one link from neighbour `nb`, which lies one hop along
// axis AX with sign SGN; the arriving move nb -> i has hop component d = -SGN.
template <int AX, int SGN, typename S, bool FID, int MSD, bool EXT>
__device__ inline void gather(const Cell<S, FID, MSD, EXT> &nb, S p_in, Acc<S> &f, bool tag)
{
    if (MSD == 2) {
        // the tags: each particle's first displacement, set on the first step (the tags
        // before it are zero), then carried like a population
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            S x = nb.v[b];
            if (b == AX && tag)
                x = SGN > 0 ? x - static_cast<S>(nb.rho) : x + static_cast<S>(nb.rho);
            f.v[b] = fma(p_in, x, f.v[b]);
        }
    }
    if (FID) {
        f.re = fma(p_in, nb.re, f.re);
        f.im = fma(p_in, nb.im, f.im);
    }
    if (MSD) {
        const S rj = static_cast<S>(nb.rho);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if (b == AX) {
                // (X + d) and (X + d)^2 = X^2 + 2 d X + d^2 with d = -SGN = +-1
                const S x1 = SGN > 0 ? nb.m1[b] - rj : nb.m1[b] + rj;
                const S x2 = SGN > 0 ? fma(S(-2), nb.m1[b], nb.m2[b] + rj)
                                     : fma(S(2), nb.m1[b], nb.m2[b] + rj);
                f.m1[b] = fma(p_in, x1, f.m1[b]);
                f.m2[b] = fma(p_in, x2, f.m2[b]);
            } else {
                f.m1[b] = fma(p_in, nb.m1[b], f.m1[b]);
                f.m2[b] = fma(p_in, nb.m2[b], f.m2[b]);
            }
        }
    }
}

// Attempt probability of the link: p0, scaled in the extended variant by the smaller
// mobility of its two ends (the same value at both ends; exactly p0 without a mobility
// field).
template <typename S, bool FID, int MSD, bool EXT>
__device__ inline S link_p0(const Cell<S, FID, MSD, EXT> &c, const Cell<S, FID, MSD, EXT> &nb,
                            S p0)
{
    return EXT ? p0 * fmin(c.mu, nb.mu) : p0;
}

template <int AX, int SGN, bool FID, int MSD, bool EXT>
__device__ inline void add_link(const Cell<double, FID, MSD, EXT> &c,
                                const Cell<double, FID, MSD, EXT> &nb, double p0, Acc<double> &f,
                                bool tag)
{
    double p_out, p_in;
    link_pair_weighed(c.F, c.G, nb.F, nb.G, link_p0(c, nb, p0), p_out, p_in);
    f.rho += exact_flux(p_in, nb.rho, p_out, c.rho);
    f.pout += p_out;
    if (MSD == 2) {
        f.mv[AX] += SGN > 0 ? p_out : -p_out;
        f.ms[AX] += p_out;
    }
    gather<AX, SGN>(nb, p_in, f, tag);
}

template <int AX, int SGN, bool FID, int MSD, bool EXT>
__device__ inline void add_link(const Cell<float, FID, MSD, EXT> &c,
                                const Cell<float, FID, MSD, EXT> &nb, float p0, Acc<float> &f,
                                bool tag)
{
    float p_out, p_in;
    link_pair(c.F, nb.F, link_p0(c, nb, p0), p_out, p_in);
    f.rho = fma(static_cast<double>(p_in), nb.rho, f.rho);
    f.pout += static_cast<double>(p_out);
    if (MSD == 2) {
        const double q = static_cast<double>(p_out);
        f.mv[AX] += SGN > 0 ? q : -q;
        f.ms[AX] += q;
    }
    gather<AX, SGN>(nb, p_in, f, tag);
}

// stay * x + gathered, finished in double for float storage (one rounding to float).
__device__ inline double stay_update(double stay, double x, double g)
{
    return fma(stay, x, g);
}
__device__ inline float stay_update(double stay, float x, float g)
{
    return static_cast<float>(fma(stay, static_cast<double>(x), static_cast<double>(g)));
}

__device__ inline double new_rho(double stay, double rho, const Acc<double> &f)
{
    (void)stay;
    return rho + f.rho;
}
__device__ inline double new_rho(double stay, double rho, const Acc<float> &f)
{
    return fma(stay, rho, f.rho);
}

// sin t and cos t - 1 of the per-step phase, without branches (a full-range library sincos
// next to a short path costs every sweep variant registers). t is reduced to r in
// [-pi, pi] with 2 pi split into a leading and a trailing part (Cody and Waite), the
// Maclaurin series of sin and cos - 1 are summed at x = r / 8 (|x| <= pi / 8, where the
// first omitted terms are below 1e-18 in double and 2e-9 relative in float), and the angle
// is doubled three times: sin 2x = 2 sin x (1 + (cos x - 1)), cos 2x - 1 =
// 2 (cos x - 1) (cos x - 1 + 2). Both results stay within 4 ulp, cos t - 1 in relative
// terms, so small phases lose nothing to cancellation.
__device__ inline void rotation(double t, double &sn, double &cm1)
{
    const double k = rint(t * 0.15915494309189535);       // 1 / (2 pi)
    double r = fma(-k, 6.283185307179586, t);              // 2 pi, leading part
    r = fma(-k, 2.4492935982947064e-16, r);                // 2 pi, trailing part
    const double x = 0.125 * r, u = x * x;
    double a = 1.0 / 6227020800.0;                         // 1/13!
    a = fma(a, u, -1.0 / 39916800.0);                      // 1/11!
    a = fma(a, u, 1.0 / 362880.0);                         // 1/9!
    a = fma(a, u, -1.0 / 5040.0);
    a = fma(a, u, 1.0 / 120.0);
    a = fma(a, u, -1.0 / 6.0);
    double s = fma(x * u, a, x);
    double b = -1.0 / 87178291200.0;                       // 1/14!
    b = fma(b, u, 1.0 / 479001600.0);                      // 1/12!
    b = fma(b, u, -1.0 / 3628800.0);                       // 1/10!
    b = fma(b, u, 1.0 / 40320.0);
    b = fma(b, u, -1.0 / 720.0);
    b = fma(b, u, 1.0 / 24.0);
    b = fma(b, u, -0.5);
    double c = u * b;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double s2 = 2.0 * fma(s, c, s);
        c = 2.0 * c * (c + 2.0);
        s = s2;
    }
    sn = s;
    cm1 = c;
}
__device__ inline void rotation(float t, float &sn, float &cm1)
{
    const float k = rintf(t * 0.15915494f);
    float r = fmaf(-k, 6.2831855f, t);
    r = fmaf(-k, -1.7484555e-07f, r);
    const float x = 0.125f * r, u = x * x;
    float a = -1.0f / 5040.0f;                             // 1/7!
    a = fmaf(a, u, 1.0f / 120.0f);
    a = fmaf(a, u, -1.0f / 6.0f);
    float s = fmaf(x * u, a, x);
    float b = 1.0f / 40320.0f;                             // 1/8!
    b = fmaf(b, u, -1.0f / 720.0f);
    b = fmaf(b, u, 1.0f / 24.0f);
    b = fmaf(b, u, -0.5f);
    float c = u * b;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float s2 = 2.0f * fmaf(s, c, s);
        c = 2.0f * c * (c + 2.0f);
        s = s2;
    }
    sn = s;
    cm1 = c;
}

// New state of a site from its old values and gather sums, into n (its fields F, G and mu
// are carried over): one step of Eqs. (1), (13) and the moment recursion.
template <typename S, bool FID, int MSD, bool EXT>
__device__ inline void advance_site(const Cell<S, FID, MSD, EXT> &c, const Acc<S> &f, S theta,
                                    Cell<S, FID, MSD, EXT> &n)
{
    const double stay = 1.0 - f.pout;
    n.rho = new_rho(stay, c.rho, f);
    n.F = c.F;
    if (PerCellWeights<S>::on)
        n.G = c.G;
    if (EXT)
        n.mu = c.mu;
    if (FID) {
        const S gre = stay_update(stay, c.re, f.re), gim = stay_update(stay, c.im, f.im);
        S sn, cm1;                                            // sin t, cos t - 1
        rotation(theta, sn, cm1);
        n.re = gre + (gre * cm1 - gim * sn);
        n.im = gim + (gim * cm1 + gre * sn);
    }
    if (MSD) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            n.m1[b] = stay_update(stay, c.m1[b], f.m1[b]);
            n.m2[b] = stay_update(stay, c.m2[b], f.m2[b]);
        }
    }
    if (MSD == 2) {
#pragma unroll
        for (int b = 0; b < 3; ++b)
            n.v[b] = stay_update(stay, c.v[b], f.v[b]);
    }
}

// Record contributions of a site's new values (region r).
template <typename S, bool FID, int MSD, bool EXT, int MAXR>
__device__ inline void record_cell(const Cell<S, FID, MSD, EXT> &n, int r, RecAcc<MAXR> &acc)
{
    if (MSD) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            acc.s1[b] += static_cast<double>(n.m1[b]);
            acc.s2[b] += static_cast<double>(n.m2[b]);
        }
    }
    acc.add_site(r, FID ? static_cast<double>(n.re) : 0.0, FID ? static_cast<double>(n.im) : 0.0,
                 n.rho);
}

// New state of a site from its old values and gather sums; stores it and adds its record
// contributions.
template <typename S, bool FID, int MSD, bool EXT, int MAXR>
__device__ inline void finish_site(const Cell<S, FID, MSD, EXT> &c, const Acc<S> &f, S theta, int r,
                                   const View<S> &dst, int64_t pz, Off o, RecAcc<MAXR> &acc,
                                   bool tag = false)
{
    Cell<S, FID, MSD, EXT> n;
    advance_site(c, f, theta, n);
    if (MSD == 2) {
        // Eq. (4): the tagged particles at the site make their next move with mean
        // displacement mv, so sum_i V_i mv_i is <dx_1 dx_{1+tau}> of the state's lag tau; on
        // the tagging step (no tags yet) the entry is the mean square of one step, C(0)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            acc.c[b] += tag ? c.rho * f.ms[b] : static_cast<double>(c.v[b]) * f.mv[b];
            st(dst.v[b] + pz, o.bs, n.v[b]);
        }
    }
    st(dst.rho + pz, o.b8, n.rho);
    if (FID) {
        st(dst.re + pz, o.bs, n.re);
        st(dst.im + pz, o.bs, n.im);
    }
    if (MSD) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            st(dst.m1[b] + pz, o.bs, n.m1[b]);
            st(dst.m2[b] + pz, o.bs, n.m2[b]);
        }
    }
    record_cell<S, FID, MSD, EXT, MAXR>(n, r, acc);
}

// LDS image of one z-plane of a tile with a one-site halo in x and y, one array per field.
template <typename S, bool FID, int MSD, bool EXT, int NL>
struct TileLds {
    double rho[NL];
    S F[NL];
    S G[PerCellWeights<S>::on ? NL : 1];
    S re[FID ? NL : 1], im[FID ? NL : 1];
    S m1[3][MSD ? NL : 1], m2[3][MSD ? NL : 1];
    S v[3][MSD == 2 ? NL : 1];
    S mu[EXT ? NL : 1];

    template <typename C>
    __device__ void put(int s, const C &c)
    {
        rho[s] = c.rho;
        F[s] = c.F;
        if (PerCellWeights<S>::on)
            G[s] = c.G;
        if (EXT)
            mu[s] = c.mu;
        if (FID) {
            re[s] = c.re;
            im[s] = c.im;
        }
        if (MSD) {
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                m1[b][s] = c.m1[b];
                m2[b][s] = c.m2[b];
            }
        }
        if (MSD == 2) {
#pragma unroll
            for (int b = 0; b < 3; ++b)
                v[b][s] = c.v[b];
        }
    }

    template <typename C>
    __device__ void get(int s, C &c) const
    {
        c.rho = rho[s];
        c.F = F[s];
        if (PerCellWeights<S>::on)
            c.G = G[s];
        if (EXT)
            c.mu = mu[s];
        if (FID) {
            c.re = re[s];
            c.im = im[s];
        }
        if (MSD) {
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                c.m1[b] = m1[b][s];
                c.m2[b] = m2[b][s];
            }
        }
        if (MSD == 2) {
#pragma unroll
            for (int b = 0; b < 3; ++b)
                c.v[b] = v[b][s];
        }
    }
};

// ---------------------------------------------------------------------------- kernels

// Workgroups are 256 threads: one thread per column of a TX x (256 / TX) tile of x-y
// columns. TX is 64 for wide lattices (a wave covers one 64-site row) and 32 or 16 for
// narrow ones, so that small boxes do not leave most lanes idle. A linear tile
// (TX = kTileLinear) instead takes 256 consecutive sites of the plane in x-fastest order,
// whatever the row length: a lattice narrower than 128 sites then keeps nearly every lane
// busy, and each wave still reads 64 consecutive sites.
constexpr int kThreads = 256;

// LDS of one workgroup when two are resident per compute unit (160 KiB each), less room
// for the record reduction.
constexpr int64_t kLdsShare = 80 * 1024 - 1024;

// Widest x extent run on linear tiles: their double-buffered LDS window of 256 + 2 nx cells
// must fit the share (and one halo site per thread needs 2 nx <= 256).
template <typename S, bool FID, int MSD>
constexpr int linear_nx_max()
{
    constexpr int64_t cell = int64_t(sizeof(TileLds<S, FID, MSD, false, 2>)) -
                             int64_t(sizeof(TileLds<S, FID, MSD, false, 1>));
    constexpr int64_t nx = (kLdsShare / 2 / cell - kThreads) / 2;
    return static_cast<int>(nx > kThreads / 2 ? kThreads / 2 : nx) & ~3;
}

__device__ inline void tile_coords(const SweepPlan &p, int64_t blk, int &bx, int &by, int &bz)
{
    bx = static_cast<int>(blk % p.gx);
    const int64_t rest = blk / p.gx;
    by = static_cast<int>(rest % p.gy);
    bz = static_cast<int>(rest / p.gy);
}

// Per-thread constants of one tile: the thread's column, its neighbours' existence and its
// halo site.
struct TileThread {
    Off own, halo;
    int li, hslot, hghost;   // hghost: reservoir face whose ghost fills the halo slot, or -1
    int oxm, oxp, oy;        // LDS offsets of the x-1, x+1 and (+-) y neighbours from li
    bool act, has_xm, has_xp, has_ym, has_yp;
    uint32_t ghosts;         // bits 0..3: the x-1, x+1, y-1, y+1 neighbour is a reservoir ghost
};

// Whether a sweep instance fetches its halo two planes ahead into a third LDS buffer (float
// block tiles of the plain variant, without autocorrelation tags) rather than one plane
// ahead into the other of two. A halo row is a row its neighbour tile loads for itself two
// planes ahead; fetched at the same time, the second load finds the row in L2. One plane
// later, on a lattice with wide rows, it mostly does not: the neighbour row then belongs to
// a tile launched a whole tile row earlier or later, which is at another plane. The third
// buffer leaves these tiles as many resident workgroups per CU as their registers allow
// (three with FID and moments, six with FID alone); FP64, tagged cells, moments without
// FID and linear tiles would lose a workgroup to it. The population-only sweep, whose short
// z-chunks pay the longer start more often, ran 3 % slower with it and keeps the one-plane
// halo. Measured on the 256^3 particle with FID alone: 102.0 -> 110.5 GSU/s.
template <typename S, bool FID, int MSD, bool EXT, int TX>
constexpr bool early_halo()
{
    return sizeof(S) == 4 && FID && MSD < 2 && !EXT && TX != kTileLinear;
}

// The FP64 sweep with FID and moments fetches its halo two planes ahead too, into a second
// halo register set that alternates with the first from plane to plane: its LDS already
// allows only two workgroups per CU, which its registers (up to 256 with the extra set, to
// four regions) allow as well. Its halo threads read fewer lines from HBM; FID alone and
// more regions would lose a workgroup or spill.
template <typename S, bool FID, int MSD, bool EXT, int MAXR, int TX>
constexpr bool early_halo_regs()
{
    return sizeof(S) == 8 && FID && MSD == 1 && !EXT && MAXR <= 4 && TX != kTileLinear;
}

// One z-plane of the tile: stage it in LDS buffer `L` (own site, and the halo site unless
// the halo comes early), prefetch plane z+2 (own column) into `nx2` and the halo of plane
// z+1 into `halo` (early halo: put the halo of plane z+1, fetched a plane ago, into `Ln`, the
// buffer of plane z+1, and fetch that of plane z+2; two halo registers: `halo` holds the
// halo of plane z and receives that of plane z+2), wait for the whole tile, then update
// every site of the plane from LDS (x, y) and registers (z).
template <typename S, bool FID, int MSD, bool EXT, int MAXR, int TX, typename LDS>
__device__ __forceinline__ void plane_step(LDS &L, LDS &Ln, const StepArgs &a, const TileThread &th,
                                           const View<S> &src, const View<S> &dst, const S *F,
                                           const S *MU, const S *TH, int64_t plane, int z,
                                           int z1, const Cell<S, FID, MSD, EXT> &prv,
                                           const Cell<S, FID, MSD, EXT> &cur,
                                           Cell<S, FID, MSD, EXT> &nxt,
                                           Cell<S, FID, MSD, EXT> &nx2,
                                           Cell<S, FID, MSD, EXT> &halo, RecAcc<MAXR> &acc)
{
    constexpr bool EARLY = early_halo<S, FID, MSD, EXT, TX>();
    constexpr bool REG2 = early_halo_regs<S, FID, MSD, EXT, MAXR, TX>();
    const Geometry &g = a.g;
    const bool zper = g.bc[2] == 0, zres = EXT && g.bc[2] == kBcReservoir;
    if (th.act)
        L.put(th.li, cur);
    if (EARLY) {
        if (th.hslot >= 0 && z + 1 < z1) {
            weigh(halo, a.fc);
            Ln.put(th.hslot, halo);
        }
    } else if (th.hslot >= 0) {
        if (!EXT || th.hghost < 0)      // a loaded halo cell; a ghost one is weighed already
            weigh(halo, a.fc);
        L.put(th.hslot, halo);
    }
    // The column offsets are re-materialised every plane so that base + offset is not
    // hoisted into per-array 64-bit vector registers: each load then takes the plane's
    // scalar base plus one 32-bit vector offset.
    Off own = th.own, hal = th.halo;
    asm volatile("" : "+v"(own.b8), "+v"(own.bs), "+v"(own.b1), "+v"(hal.b8), "+v"(hal.bs));
    // The prefetches go out before the barrier (their registers are free once the puts
    // have read them), so the wait at the barrier also covers their latency.
    if (z + 1 < z1) {
        // z + 2 <= nz here, so a periodic wrap lands on plane 0
        const int zn = z + 2 < g.nz ? z + 2 : (zper ? 0 : -1);
        if (th.act && zn >= 0)
            load_cell(nx2, src, F, MU, plane * zn, own);
        if (!EARLY && !REG2 && th.hslot >= 0 && (!EXT || th.hghost < 0))
            load_cell(halo, src, F, MU, plane * (z + 1), hal);
    }
    if ((EARLY || REG2) && th.hslot >= 0 && z + 2 < z1)
        load_cell(halo, src, F, MU, plane * (z + 2), hal);
    __syncthreads();
    if (!th.act)
        return;
    const S p0 = static_cast<S>(a.p0);
    const bool tag = MSD == 2 && a.tag;
    weigh(nxt, a.fc);                   // first use of the plane above (prefetched earlier)
    Acc<S> f{};
    Cell<S, FID, MSD, EXT> nb;
    // particles that come in from a reservoir ghost were not in the lattice at the start:
    // they carry no autocorrelation tag
    if (th.has_xm) {
        L.get(th.li + th.oxm, nb);
        add_link<0, -1>(cur, nb, p0, f, tag && !(th.ghosts & 1u));
    }
    if (th.has_xp) {
        L.get(th.li + th.oxp, nb);
        add_link<0, +1>(cur, nb, p0, f, tag && !(th.ghosts & 2u));
    }
    if (th.has_ym) {
        L.get(th.li - th.oy, nb);
        add_link<1, -1>(cur, nb, p0, f, tag && !(th.ghosts & 4u));
    }
    if (th.has_yp) {
        L.get(th.li + th.oy, nb);
        add_link<1, +1>(cur, nb, p0, f, tag && !(th.ghosts & 8u));
    }
    // the z ghost cells are built where they are used: filling window registers with them
    // inside the plane loop costs the whole loop registers
    if (z > 0 || zper) {
        add_link<2, -1>(cur, prv, p0, f, tag);
    } else if (zres) {
        Cell<S, FID, MSD, EXT> gz;
        ghost_cell(gz, a.ghost, 4, a.fc);
        add_link<2, -1>(cur, gz, p0, f, false);
    }
    if (z + 1 < g.nz || zper) {
        add_link<2, +1>(cur, nxt, p0, f, tag);
    } else if (zres) {
        Cell<S, FID, MSD, EXT> gz;
        ghost_cell(gz, a.ghost, 5, a.fc);
        add_link<2, +1>(cur, gz, p0, f, false);
    }
    const int64_t pz = plane * z;
    const S theta = FID ? ld(TH + pz, own.bs) : S(0);
    const int r = MAXR == 1 ? 0 : ld(a.region + pz, own.b1);
    finish_site<S, FID, MSD, EXT, MAXR>(cur, f, theta, r, dst, pz, own, acc, tag);
}

// At least two resident workgroups per compute unit (two waves per SIMD): every variant
// fits its registers in the 256 this allows; without the bound the widest one (FP64,
// extended, FID + moments) takes 257 and drops to one wave per SIMD.
#ifndef LPC_MIN_WAVES
#define LPC_MIN_WAVES 2
#endif

// Waves per SIMD the register allocation of a one-step sweep instance must leave room for.
// A float linear tile's LDS window admits three workgroups per compute unit; the instances
// with FID + moments over up to four regions and FID alone over up to eight would otherwise
// take 170-171 VGPRs, one wave per SIMD fewer than the LDS allows. With three waves they fit
// in 168 without spilling (four 100 x 100 x 300 systems in one batch: 36.7 -> 43.3 GSU/s).
// Block tiles keep two: the same bound costs them 1-2 %, and four waves (128 VGPRs, with
// spills) 8 % or more.
template <typename S, bool FID, int MSD, bool EXT, int MAXR, int TX>
constexpr int sweep_min_waves()
{
    if (sizeof(S) == 4 && TX == kTileLinear &&
        ((MSD == 1 && MAXR > 2 && MAXR <= 4) || (MSD == 0 && FID && MAXR > 4)))
        return 3;
    return LPC_MIN_WAVES;
}

// Tile geometry of the sweep: TY rows of TX columns with a one-site halo, or a linear tile
// of 256 sites with a window of one row on either side (NL cells in LDS).
template <typename S, bool FID, int MSD, bool EXT, int TX>
struct TileShape {
    static constexpr bool linear = TX == kTileLinear;
    static constexpr int TY = linear ? kThreads : kThreads / TX;
    static constexpr int COLS = linear ? 0 : TX + 2;
    static constexpr int NL = linear ? kThreads + 2 * linear_nx_max<S, FID, MSD>()
                                     : COLS * (TY + 2);
    static_assert(linear || TX * TY >= 2 * TX + 2 * TY, "one halo site per thread");
    static_assert(!(linear && EXT), "linear tiles run the plain variant only");
};

// Per-thread constants of a linear tile: sites s0 .. s0 + n - 1 of the plane (n <= 256).
// LDS slot j holds plane site s0 - nx + j: the row below the run, the run, the row above
// it. Threads t < 2 nx each fetch one halo site (slot t below, slot t + n above), wrapped
// modulo the plane on a periodic y axis (the row below row 0 is row ny - 1), absent across
// a closed y face. An x neighbour across a periodic x face is in the same row, nx - 1 sites
// away; it lies inside the window too.
__device__ inline void linear_thread(TileThread &th, const Geometry &g, int bx, int t,
                                     uint32_t storage)
{
    const int nx = g.nx;
    const int64_t P = static_cast<int64_t>(g.nx) * g.ny;
    const int64_t s0 = static_cast<int64_t>(bx) * kThreads;
    const int n = static_cast<int>(min(static_cast<int64_t>(kThreads), P - s0));
    const bool xper = g.bc[0] == 0, yper = g.bc[1] == 0;
    const int64_t s = s0 + t;
    th.act = t < n;
    const int x = th.act ? static_cast<int>(s % nx) : 0;
    const int y = th.act ? static_cast<int>(s / nx) : 0;
    th.has_xm = x > 0 || xper;
    th.has_xp = x + 1 < nx || xper;
    th.has_ym = y > 0 || yper;
    th.has_yp = y + 1 < g.ny || yper;
    th.ghosts = 0u;
    const uint32_t col = th.act ? static_cast<uint32_t>(s) : 0u;
    th.own = {col * 8u, col * storage, col};
    th.li = nx + t;
    th.oxm = x > 0 ? -1 : nx - 1;
    th.oxp = x + 1 < nx ? 1 : 1 - nx;
    th.oy = nx;
    th.hslot = -1;
    th.hghost = -1;
    uint32_t hcol = 0u;
    if (t < 2 * nx) {
        const int j = t < nx ? t : t + n;
        int64_t q = s0 - nx + j;
        if (q < 0)
            q = yper ? q + P : -1;
        else if (q >= P)
            q = yper ? q - P : -1;
        if (q >= 0) {
            th.hslot = j;
            hcol = static_cast<uint32_t>(q);
        }
    }
    th.halo = {hcol * 8u, hcol * storage, hcol};
}

// Per-thread constants of a TX x TY block of columns: the thread's column, its neighbours'
// existence and its halo site (a row below and above the block, a column left and right of
// it; wrapped on periodic axes, absent across closed faces, a ghost cell across reservoir
// faces).
template <bool EXT, int TX>
__device__ inline void block_thread(TileThread &th, const Geometry &g, int bx, int by, int t,
                                    uint32_t storage)
{
    constexpr int TY = kThreads / TX, COLS = TX + 2;
    const int tx = t % TX, ty = t / TX;
    const int x0 = bx * TX, y0 = by * TY;
    const int x = x0 + tx, y = y0 + ty;
    const int cols = min(TX, g.nx - x0), rows = min(TY, g.ny - y0);
    const bool xper = g.bc[0] == 0, yper = g.bc[1] == 0;
    const bool xres = EXT && g.bc[0] == kBcReservoir, yres = EXT && g.bc[1] == kBcReservoir;
    th.act = tx < cols && ty < rows;
    th.has_xm = x > 0 || xper || xres;
    th.has_xp = x + 1 < g.nx || xper || xres;
    th.has_ym = y > 0 || yper || yres;
    th.has_yp = y + 1 < g.ny || yper || yres;
    th.ghosts = (x == 0 && xres ? 1u : 0u) | (x + 1 == g.nx && xres ? 2u : 0u) |
                (y == 0 && yres ? 4u : 0u) | (y + 1 == g.ny && yres ? 8u : 0u);
    const uint32_t col = th.act ? static_cast<uint32_t>(x + g.nx * y) : 0u;
    th.own = {col * 8u, col * storage, col};
    th.li = (ty + 1) * COLS + tx + 1;
    th.oxm = -1;
    th.oxp = 1;
    th.oy = COLS;
    th.hslot = -1;
    {
        int hx = -1, hy = -1, face = -1;
        if (t < TX) {                                   // row below the tile
            if (t < cols) {
                hx = x0 + t;
                hy = y0 > 0 ? y0 - 1 : (yper ? g.ny - 1 : -1);
                face = hy < 0 && yres ? 2 : -1;
                th.hslot = t + 1;
            }
        } else if (t < 2 * TX) {                        // row above the tile
            const int u = t - TX;
            if (u < cols) {
                hx = x0 + u;
                hy = y0 + rows < g.ny ? y0 + rows : (yper ? (y0 + rows) % g.ny : -1);
                face = hy < 0 && yres ? 3 : -1;
                th.hslot = (rows + 1) * COLS + u + 1;
            }
        } else if (t < 2 * TX + TY) {                   // column left of the tile
            const int v = t - 2 * TX;
            if (v < rows) {
                hy = y0 + v;
                hx = x0 > 0 ? x0 - 1 : (xper ? g.nx - 1 : -1);
                face = hx < 0 && xres ? 0 : -1;
                th.hslot = (v + 1) * COLS;
            }
        } else if (t < 2 * TX + 2 * TY) {               // column right of the tile
            const int v = t - 2 * TX - TY;
            if (v < rows) {
                hy = y0 + v;
                hx = x0 + cols < g.nx ? x0 + cols : (xper ? (x0 + cols) % g.nx : -1);
                face = hx < 0 && xres ? 1 : -1;
                th.hslot = (v + 1) * COLS + cols + 1;
            }
        }
        if ((hx < 0 || hy < 0) && face < 0)
            th.hslot = -1;
        th.hghost = th.hslot >= 0 ? face : -1;
        const uint32_t hcol = th.hslot >= 0 && face < 0 ? static_cast<uint32_t>(hx + g.nx * hy)
                                                        : 0u;
        th.halo = {hcol * 8u, hcol * storage, hcol};
    }
}

// One step over a tile of x-y columns (a TX x TY block, or a linear run of 256 sites) and
// the workgroup's run of z-planes. Each thread owns one column and keeps planes z-1, z, z+1
// of it in registers, with plane z+2 in flight; the four register sets rotate roles from
// plane to plane, so no move forces an early wait on a prefetch. The x and y neighbours of
// plane z come from an LDS image of the plane with its halo, double-buffered so that one
// barrier per plane suffices. The halo sites are spread over threads, one site each, and
// fetched one plane ahead. Plane offsets are workgroup-uniform; each thread keeps only the
// 32-bit byte offsets of its column. Beyond a reservoir face in x or y the halo slot holds
// the face's ghost cell, set once and never reloaded; in z the ghost cell is built at the
// first or last plane where its link is added.
template <typename S, bool FID, int MSD, bool EXT, int MAXR, int TX>
__device__ __forceinline__ void sweep_tile(const StepArgs &a, const SweepPlan &p, int64_t blk)
{
    using Shape = TileShape<S, FID, MSD, EXT, TX>;
    constexpr int NL = Shape::NL;
    constexpr bool EARLY = early_halo<S, FID, MSD, EXT, TX>();
    constexpr bool REG2 = early_halo_regs<S, FID, MSD, EXT, MAXR, TX>();
    using C = Cell<S, FID, MSD, EXT>;
    __shared__ TileLds<S, FID, MSD, EXT, NL> Lb[EARLY ? 3 : 2];
    __shared__ double red[(kThreads / kWave) * record_slots(MAXR, MSD)];
    const Geometry &g = a.g;
    int bx, by, bz;
    tile_coords(p, blk, bx, by, bz);
    const int t = static_cast<int>(threadIdx.x);
    TileThread th;
    if constexpr (Shape::linear)
        linear_thread(th, g, bx, t, static_cast<uint32_t>(sizeof(S)));
    else
        block_thread<EXT, TX>(th, g, bx, by, t, static_cast<uint32_t>(sizeof(S)));
    const bool zper = g.bc[2] == 0;
    const S *F = static_cast<const S *>(a.F);
    const S *MU = static_cast<const S *>(a.mu);
    const S *TH = static_cast<const S *>(a.theta);
    const View<S> src = typed<S>(a.src);
    const View<S> dst = typed<S>(a.dst);
    const int64_t plane = static_cast<int64_t>(g.nx) * g.ny;
    const int z0 = bz * p.zc, z1 = min(g.nz, z0 + p.zc);
    C w0, w1, w2, w3, halo, halo2;
    // the halo register of odd planes (the same as that of even ones without REG2)
    C &hodd = REG2 ? halo2 : halo;
    RecAcc<MAXR> acc;
    acc.zero();
    if (th.act) {
        load_cell(w1, src, F, MU, plane * z0, th.own);
        const int zm = z0 > 0 ? z0 - 1 : (zper ? g.nz - 1 : -1);
        const int zp = z0 + 1 < g.nz ? z0 + 1 : (zper ? (z0 + 1) % g.nz : -1);
        if (zm >= 0)
            load_cell(w0, src, F, MU, plane * zm, th.own);
        if (zp >= 0)
            load_cell(w2, src, F, MU, plane * zp, th.own);
        // the first plane's prv and cur are used at once; nxt is weighed where first used
        weigh(w0, a.fc);
        weigh(w1, a.fc);
    }
    if (th.hslot >= 0) {
        if (EXT && th.hghost >= 0) {
            ghost_cell(halo, a.ghost, th.hghost, a.fc);
        } else {
            load_cell(halo, src, F, MU, plane * z0, th.halo);
            if (REG2 && z0 + 1 < z1)
                load_cell(halo2, src, F, MU, plane * (z0 + 1), th.halo);
            if (EARLY) {
                // the first plane's halo goes straight into its buffer; the register then
                // carries the next plane's, which the first step puts into the next buffer
                weigh(halo, a.fc);
                Lb[0].put(th.hslot, halo);
                if (z0 + 1 < z1)
                    load_cell(halo, src, F, MU, plane * (z0 + 1), th.halo);
            }
        }
    }
    // roles (prv, cur, nxt, in-flight) rotate through w0..w3 with period 4; LDS buffers
    // alternate with period 2, or rotate with period 3 (early halo: plane z in buffer
    // (z - z0) mod 3)
    int b = 0;
    auto nb = [](int i) { return EARLY ? (i == 2 ? 0 : i + 1) : 1 - i; };
    for (int z = z0; z < z1; z += 4) {
        plane_step<S, FID, MSD, EXT, MAXR, TX>(Lb[b], Lb[nb(b)], a, th, src, dst, F, MU, TH,
                                               plane, z, z1, w0, w1, w2, w3, halo, acc);
        b = nb(b);
        if (z + 1 >= z1)
            break;
        plane_step<S, FID, MSD, EXT, MAXR, TX>(Lb[b], Lb[nb(b)], a, th, src, dst, F, MU, TH,
                                               plane, z + 1, z1, w1, w2, w3, w0, hodd, acc);
        b = nb(b);
        if (z + 2 >= z1)
            break;
        plane_step<S, FID, MSD, EXT, MAXR, TX>(Lb[b], Lb[nb(b)], a, th, src, dst, F, MU, TH,
                                               plane, z + 2, z1, w2, w3, w0, w1, halo, acc);
        b = nb(b);
        if (z + 3 >= z1)
            break;
        plane_step<S, FID, MSD, EXT, MAXR, TX>(Lb[b], Lb[nb(b)], a, th, src, dst, F, MU, TH,
                                               plane, z + 3, z1, w3, w0, w1, w2, hodd, acc);
        b = nb(b);
    }
    __syncthreads();
    block_reduce<MAXR, kThreads / kWave, MSD == 2>(acc, a.R, a.K, a.partials, p.nblocks, blk, red);
}

// One step of every lattice in a work list: workgroup w (after the XCD renumbering) runs
// tile w - prefix[l] of item l, prefix[l] <= w < prefix[l + 1]. The items hold the views
// of the step with parity 0; parity 1 swaps source and destination. Each lattice keeps its
// own plan, so a lattice gives the same bits alone (a list of one) and in any batch.
template <typename S, bool FID, int MSD, bool EXT, int MAXR, int TX>
__global__ __launch_bounds__(kThreads, (sweep_min_waves<S, FID, MSD, EXT, MAXR, TX>())) void k_sweep_tile(
    const SweepItem *__restrict__ items, const int64_t *__restrict__ prefix, int32_t n_items,
    int64_t total, int64_t padded, int32_t parity, int64_t slot)
{
    const int64_t w = logical_block(blockIdx.x, padded);
    if (w >= total)
        return;
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (prefix[mid] <= w)
            lo = mid;
        else
            hi = mid - 1;
    }
    StepArgs a = items[lo].a;
    const SweepPlan p = items[lo].plan;
    if (parity) {
        const StateView t = a.src;
        a.src = a.dst;
        a.dst = t;
    }
    a.partials += slot * a.K * p.nblocks;
    sweep_tile<S, FID, MSD, EXT, MAXR, TX>(a, p, w - prefix[lo]);
}

// ---------------------------------------------------------------------------- two steps per pass

// Temporal blocking: one pass advances a lattice by two steps, reading the state and the
// fields once and writing the state once. The 256 threads of a workgroup cover a 32 x 8
// block of x-y columns (the A columns) and take the first step on them; the inner 30 x 6
// columns are the tile the workgroup owns, and it takes the second step there from the
// first step's values of the A columns, which never leave the chip. The first step on the
// ring of A columns around the tile repeats work of the neighbouring tiles. z is marched as
// in the one-step sweep, with the first step one plane ahead of the second: the first step
// reads x-y neighbours from a double-buffered LDS image of the level-0 plane with a halo of
// one more site (34 x 10), the second from a double-buffered image of the level-1 plane
// (32 x 8); each thread keeps the z-window of its column at both levels in registers. Per
// site the arithmetic is that of the one-step sweep, so the state after the pass is bit for
// bit that of two one-step sweeps; the per-step sums run over other tiles.
constexpr int kTwoAX = 32, kTwoAY = 8;                      // A columns of a tile
constexpr int kTwoOX = kTwoAX - 2, kTwoOY = kTwoAY - 2;     // owned columns
constexpr int kTwoL0X = kTwoAX + 2, kTwoL0Y = kTwoAY + 2;   // level-0 image with its halo
constexpr int kTwoHalo = 2 * kTwoL0X + 2 * kTwoAY;          // halo cells of that image
static_assert(kTwoAX * kTwoAY == kThreads, "one A column per thread");
static_assert(kTwoHalo <= kThreads, "one halo cell per thread");
static_assert(kTwoOX == kTwoStepTileX && kTwoOY == kTwoStepTileY, "two-step tile of the plans");

// v on an axis of n sites: itself inside, wrapped on a periodic axis, -1 beyond a closed
// face.
__device__ inline int wrap_axis(int v, int n, bool periodic)
{
    if (v >= 0 && v < n)
        return v;
    if (!periodic)
        return -1;
    v %= n;
    return v < 0 ? v + n : v;
}

// Per-thread constants of a two-step tile: the thread's A column (its slots in both LDS
// images, whether it exists and whether the tile owns it), the existence of its x and y
// neighbours, and the level-0 halo cell the thread loads.
struct TwoThread {
    Off own, halo;
    int l0, l1, hslot;
    bool act, owned, has_xm, has_xp, has_ym, has_yp;
};

__device__ inline void two_thread(TwoThread &th, const Geometry &g, int bx, int by, int t,
                                  uint32_t storage)
{
    const bool xper = g.bc[0] == 0, yper = g.bc[1] == 0;
    const int tx = t % kTwoAX, ty = t / kTwoAX;
    const int x0 = bx * kTwoOX, y0 = by * kTwoOY;       // the first owned column
    const int ax = x0 - 1 + tx, ay = y0 - 1 + ty;       // the A column, before wrapping
    const int px = wrap_axis(ax, g.nx, xper), py = wrap_axis(ay, g.ny, yper);
    th.act = px >= 0 && py >= 0;
    th.owned = tx >= 1 && tx <= kTwoOX && ty >= 1 && ty <= kTwoOY && ax < g.nx && ay < g.ny;
    th.has_xm = th.act && (xper || px > 0);
    th.has_xp = th.act && (xper || px + 1 < g.nx);
    th.has_ym = th.act && (yper || py > 0);
    th.has_yp = th.act && (yper || py + 1 < g.ny);
    const uint32_t col = th.act ? static_cast<uint32_t>(px + g.nx * py) : 0u;
    th.own = {col * 8u, col * storage, col};
    th.l0 = (ty + 1) * kTwoL0X + tx + 1;
    th.l1 = ty * kTwoAX + tx;
    th.hslot = -1;
    uint32_t hcol = 0u;
    if (t < kTwoHalo) {
        int i, j;                                       // cell (i, j) of the 34 x 10 image
        if (t < kTwoL0X) {
            i = t;
            j = 0;
        } else if (t < 2 * kTwoL0X) {
            i = t - kTwoL0X;
            j = kTwoL0Y - 1;
        } else if (t < 2 * kTwoL0X + kTwoAY) {
            i = 0;
            j = t - 2 * kTwoL0X + 1;
        } else {
            i = kTwoL0X - 1;
            j = t - 2 * kTwoL0X - kTwoAY + 1;
        }
        const bool corner = (i == 0 || i == kTwoL0X - 1) && (j == 0 || j == kTwoL0Y - 1);
        const int hx = wrap_axis(x0 - 2 + i, g.nx, xper), hy = wrap_axis(y0 - 2 + j, g.ny, yper);
        if (!corner && hx >= 0 && hy >= 0) {              // corners are nobody's neighbour
            th.hslot = j * kTwoL0X + i;
            hcol = static_cast<uint32_t>(hx + g.nx * hy);
        }
    }
    th.halo = {hcol * 8u, hcol * storage, hcol};
}

// Gather sums of one site from its x and y neighbours in an LDS image `w` cells wide and its
// z neighbours in registers (each only where it exists).
template <typename S, bool FID, int MSD, typename LDS>
__device__ inline void gather_site(const LDS &L, int slot, int w, const TwoThread &th,
                                   const Cell<S, FID, MSD, false> &cur,
                                   const Cell<S, FID, MSD, false> &below, bool zm,
                                   const Cell<S, FID, MSD, false> &above, bool zp, S p0,
                                   Acc<S> &f)
{
    Cell<S, FID, MSD, false> nb;
    if (th.has_xm) {
        L.get(slot - 1, nb);
        add_link<0, -1>(cur, nb, p0, f, false);
    }
    if (th.has_xp) {
        L.get(slot + 1, nb);
        add_link<0, +1>(cur, nb, p0, f, false);
    }
    if (th.has_ym) {
        L.get(slot - w, nb);
        add_link<1, -1>(cur, nb, p0, f, false);
    }
    if (th.has_yp) {
        L.get(slot + w, nb);
        add_link<1, +1>(cur, nb, p0, f, false);
    }
    if (zm)
        add_link<2, -1>(cur, below, p0, f, false);
    if (zp)
        add_link<2, +1>(cur, above, p0, f, false);
}

template <typename S, bool FID, int MSD, int MAXR>
__device__ __forceinline__ void sweep2_tile(const StepArgs &a, const SweepPlan &p, int64_t blk,
                                            double *part1, double *part2)
{
    using C = Cell<S, FID, MSD, false>;
    __shared__ TileLds<S, FID, MSD, false, kTwoL0X * kTwoL0Y> LA[2];   // level 0, first step
    __shared__ TileLds<S, FID, MSD, false, kTwoAX * kTwoAY> LB[2];     // level 1, second step
    __shared__ double red[(kThreads / kWave) * (3 * MAXR + 6)];
    const Geometry &g = a.g;
    int bx, by, bz;
    tile_coords(p, blk, bx, by, bz);
    TwoThread th;
    two_thread(th, g, bx, by, static_cast<int>(threadIdx.x), static_cast<uint32_t>(sizeof(S)));
    const bool zper = g.bc[2] == 0;
    const S *F = static_cast<const S *>(a.F);
    const S *TH = static_cast<const S *>(a.theta);
    const View<S> src = typed<S>(a.src);
    const View<S> dst = typed<S>(a.dst);
    const S p0 = static_cast<S>(a.p0);
    const int64_t plane = static_cast<int64_t>(g.nx) * g.ny;
    // owned planes [z0, z1); the first step runs on [za_lo, za_hi] (one more plane on each
    // side where one exists), the second on [z0, z1)
    const int z0 = bz * p.zc, z1 = min(g.nz, z0 + p.zc);
    const int za_lo = z0 > 0 || zper ? z0 - 1 : z0;
    const int za_hi = z1 < g.nz || zper ? z1 : z1 - 1;
    auto pz_of = [&](int z) { return wrap_axis(z, g.nz, zper); };
    C w_prv, w_cur, w_nxt, w_fly, halo;   // level 0 of the own column at za - 1 .. za + 2
    C v_prv, v_cur, c1;                   // level 1 at zb - 1, zb and za (zb = za - 1)
    S th_cur = S(0), th_nxt = S(0);       // phases at zb and za
    int r_cur = 0, r_nxt = 0;             // regions at zb and za
    RecAcc<MAXR> acc1, acc2;
    acc1.zero();
    acc2.zero();
    if (th.act) {
        int q = pz_of(za_lo - 1);
        if (q >= 0)
            load_cell(w_prv, src, F, static_cast<const S *>(nullptr), plane * q, th.own);
        load_cell(w_cur, src, F, static_cast<const S *>(nullptr), plane * pz_of(za_lo), th.own);
        q = pz_of(za_lo + 1);
        if (q >= 0)
            load_cell(w_nxt, src, F, static_cast<const S *>(nullptr), plane * q, th.own);
        weigh(w_prv, a.fc);
        weigh(w_cur, a.fc);
    }
    if (th.hslot >= 0)
        load_cell(halo, src, F, static_cast<const S *>(nullptr), plane * pz_of(za_lo), th.halo);
    int i = 0;
    for (int za = za_lo; za <= za_hi; ++za, ++i) {
        auto &A = LA[i & 1];
        auto &B = LB[i & 1];
        const auto &Bp = LB[(i & 1) ^ 1];
        if (th.act)
            A.put(th.l0, w_cur);
        if (th.hslot >= 0) {
            weigh(halo, a.fc);
            A.put(th.hslot, halo);
        }
        Off own = th.own, hal = th.halo;
        asm volatile("" : "+v"(own.b8), "+v"(own.bs), "+v"(own.b1), "+v"(hal.b8), "+v"(hal.bs));
        if (za < za_hi) {
            const int q = pz_of(za + 2);
            if (th.act && q >= 0)
                load_cell(w_fly, src, F, static_cast<const S *>(nullptr), plane * q, own);
            if (th.hslot >= 0)
                load_cell(halo, src, F, static_cast<const S *>(nullptr), plane * pz_of(za + 1),
                          hal);
        }
        __syncthreads();
        const bool zm = pz_of(za - 1) >= 0, zp = pz_of(za + 1) >= 0;
        if (th.act) {
            // first step at plane za, on every A column
            if (zp)
                weigh(w_nxt, a.fc);
            Acc<S> f{};
            gather_site(A, th.l0, kTwoL0X, th, w_cur, w_prv, zm, w_nxt, zp, p0, f);
            const int64_t pz = plane * pz_of(za);
            th_nxt = FID ? ld(TH + pz, own.bs) : S(0);
            advance_site(w_cur, f, th_nxt, c1);
            B.put(th.l1, c1);
            if (th.owned && za >= z0 && za < z1) {
                r_nxt = MAXR == 1 ? 0 : ld(a.region + pz, own.b1);
                record_cell<S, FID, MSD, false, MAXR>(c1, r_nxt, acc1);
            }
        }
        const int zb = za - 1;
        if (th.owned && zb >= z0 && zb < z1) {
            // second step at plane zb, on the owned columns, from level 1
            Acc<S> f{};
            gather_site(Bp, th.l1, kTwoAX, th, v_cur, v_prv, pz_of(zb - 1) >= 0, c1, true, p0,
                        f);
            finish_site<S, FID, MSD, false, MAXR>(v_cur, f, th_cur, r_cur, dst,
                                                  plane * pz_of(zb), own, acc2);
        }
        v_prv = v_cur;
        v_cur = c1;
        th_cur = th_nxt;
        r_cur = r_nxt;
        w_prv = w_cur;
        w_cur = w_nxt;
        w_nxt = w_fly;
    }
    if (za_hi >= z0 && za_hi < z1) {
        // the top owned plane below a closed face: its second step has no plane above
        __syncthreads();
        if (th.owned) {
            Acc<S> f{};
            Off own = th.own;
            gather_site(LB[(i - 1) & 1], th.l1, kTwoAX, th, v_cur, v_prv, pz_of(za_hi - 1) >= 0,
                        v_cur, false, p0, f);
            finish_site<S, FID, MSD, false, MAXR>(v_cur, f, th_cur, r_cur, dst,
                                                  plane * pz_of(za_hi), own, acc2);
        }
    }
    __syncthreads();
    block_reduce<MAXR, kThreads / kWave>(acc1, a.R, a.K, part1, p.nblocks, blk, red);
    __syncthreads();
    block_reduce<MAXR, kThreads / kWave>(acc2, a.R, a.K, part2, p.nblocks, blk, red);
}

// Two steps of every lattice in a work list (two-step plans), as k_sweep_tile does one: the
// first step's sums go to step slot `slot`, the second's to slot + 1.
template <typename S, bool FID, int MSD, int MAXR>
__global__ __launch_bounds__(kThreads, LPC_MIN_WAVES) void k_sweep2_tile(
    const SweepItem *__restrict__ items, const int64_t *__restrict__ prefix, int32_t n_items,
    int64_t total, int64_t padded, int32_t parity, int64_t slot)
{
    const int64_t w = logical_block(blockIdx.x, padded);
    if (w >= total)
        return;
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (prefix[mid] <= w)
            lo = mid;
        else
            hi = mid - 1;
    }
    StepArgs a = items[lo].a;
    const SweepPlan p = items[lo].plan;
    if (parity) {
        const StateView t = a.src;
        a.src = a.dst;
        a.dst = t;
    }
    double *part1 = a.partials + slot * a.K * p.nblocks;
    sweep2_tile<S, FID, MSD, MAXR>(a, p, w - prefix[lo], part1, part1 + a.K * p.nblocks);
}

template <typename S, bool FID, int MSD, int MAXR>
__device__ inline void record_site(const StepArgs &a, const View<S> &v, int64_t i,
                                   RecAcc<MAXR> &acc)
{
    double re = 0.0, im = 0.0;
    if (FID) {
        re = static_cast<double>(v.re[i]);
        im = static_cast<double>(v.im[i]);
    }
    if (MSD) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            acc.s1[b] += static_cast<double>(v.m1[b][i]);
            acc.s2[b] += static_cast<double>(v.m2[b][i]);
        }
    }
    acc.add_site(MAXR == 1 ? 0 : a.region[i], re, im, v.rho[i]);
}

// Record contributions of the current state (no step), on the same tiles as the sweep.
template <typename S, bool FID, int MSD, int MAXR>
__global__ __launch_bounds__(kThreads) void k_record_tile(StepArgs a, SweepPlan p, int64_t padded)
{
    __shared__ double red[(kThreads / kWave) * record_slots(MAXR, MSD)];
    const int64_t blk = logical_block(blockIdx.x, padded);
    if (blk >= p.nblocks)
        return;
    int bx, by, bz;
    tile_coords(p, blk, bx, by, bz);
    const int64_t plane = static_cast<int64_t>(a.g.nx) * a.g.ny;
    int64_t col = -1;
    if (p.tx == kTileLinear) {
        const int64_t s = static_cast<int64_t>(bx) * kThreads + threadIdx.x;
        col = s < plane ? s : -1;
    } else {
        const int x = bx * p.tx + static_cast<int>(threadIdx.x) % p.tx;
        const int y = by * p.ty + static_cast<int>(threadIdx.x) / p.tx;
        col = x < a.g.nx && y < a.g.ny ? x + static_cast<int64_t>(a.g.nx) * y : -1;
    }
    const View<S> src = typed<S>(a.src);
    RecAcc<MAXR> acc;
    acc.zero();
    if (col >= 0) {
        const int z1 = min(a.g.nz, (bz + 1) * p.zc);
        for (int z = bz * p.zc; z < z1; ++z)
            record_site<S, FID, MSD, MAXR>(a, src, col + plane * z, acc);
    }
    // the autocorrelation entries of a state with no step are zero
    block_reduce<MAXR, kThreads / kWave, MSD == 2>(acc, a.R, a.K, a.partials, p.nblocks, blk, red);
}

#if LPC_HOST_PART
// Sum of one record entry over the workgroup partials p[0, nblocks), in a fixed order.
__device__ inline double partial_sum(const double *p, int64_t nblocks, double *w)
{
    double v = 0.0;
    for (int64_t b = threadIdx.x; b < nblocks; b += 256)
        v += p[b];
    v = wave_sum(v);
    if (threadIdx.x % kWave == 0)
        w[threadIdx.x / kWave] = v;
    __syncthreads();
    return ((w[0] + w[1]) + w[2]) + w[3];
}

__global__ __launch_bounds__(256) void k_finalize(const double *partials, int64_t nblocks, int K,
                                                  double *out)
{
    __shared__ double w[4];
    const int s = blockIdx.x / K, k = blockIdx.x % K;
    const double t = partial_sum(partials + (static_cast<int64_t>(s) * K + k) * nblocks, nblocks, w);
    if (threadIdx.x == 0)
        out[static_cast<int64_t>(s) * K + k] = t;
}

// Records of `steps` steps of every lattice in a list: workgroup (s, e) with
// kprefix[l] <= e < kprefix[l + 1] writes entry e - kprefix[l] of row first_row + s of
// lattice l (first_row counted from the lattice's own row base).
__global__ __launch_bounds__(256) void k_finalize_list(const FinalizeItem *__restrict__ items,
                                                       const int64_t *__restrict__ kprefix,
                                                       int32_t n_items, int64_t total_k,
                                                       int64_t first_row,
                                                       const int64_t *__restrict__ row_offset)
{
    if (row_offset)          // a graph replayed per chunk reads its chunk's rows from memory
        first_row += *row_offset;
    __shared__ double w[4];
    const int64_t s = blockIdx.x / total_k, e = blockIdx.x % total_k;
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (kprefix[mid] <= e)
            lo = mid;
        else
            hi = mid - 1;
    }
    const FinalizeItem it = items[lo];
    const int64_t k = e - kprefix[lo];
    const double t = partial_sum(it.partials + (s * it.K + k) * it.nblocks, it.nblocks, w);
    if (threadIdx.x == 0)
        it.records[(it.row_base + first_row + s) * it.K + k] = t;
}

// *counter = value, or += add when add is non-zero (one thread): the row counter that the
// finalisation of a replayed graph reads.
__global__ void k_set_counter(int64_t *counter, int64_t value, int64_t add)
{
    *counter = add != 0 ? *counter + add : value;
}

// E_i = e^{F_i - c} of the FP64 free energies F (the field the FP64 sweep reads).
__global__ void k_boltzmann_factors(const double *F, double *E, int64_t n, double fc)
{
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        E[i] = boltzmann_factor(F[i], fc);
}

template <typename S>
__global__ void k_store_field(const double *src, S *dst, int64_t n, double scale)
{
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        dst[i] = static_cast<S>(scale == 1.0 ? src[i] : scale * src[i]);
}

template <typename S>
__global__ void k_init_state(View<S> st, bool fid, bool msd, const double *rho_src, const S *F,
                             int64_t n)
{
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const bool open = static_cast<double>(F[i]) < kBlockedTest;   // not solid matrix
        const double r = open ? (rho_src ? rho_src[i] : 1.0) : 0.0;
        st.rho[i] = r;
        if (fid) {
            st.re[i] = static_cast<S>(r);
            st.im[i] = static_cast<S>(0);
        }
        if (msd) {
            for (int b = 0; b < 3; ++b) {
                st.m1[b][i] = static_cast<S>(0);
                st.m2[b][i] = static_cast<S>(0);
            }
        }
        if (st.v[0]) {
            for (int b = 0; b < 3; ++b)
                st.v[b][i] = static_cast<S>(0);
        }
    }
}

template <typename S>
__global__ void k_fill(S *dst, int64_t n, S value)
{
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        dst[i] = value;
}

constexpr int kWeightBlocks = 1024;

template <typename S>
__global__ __launch_bounds__(256) void k_boltzmann_weights(const S *F, double Fmin, double *w,
                                                           int64_t n, double *partials)
{
    __shared__ double lds[4];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += static_cast<int64_t>(gridDim.x) * 256) {
        const double v = exp(-(static_cast<double>(F[i]) - Fmin));
        w[i] = v;
        acc += v;
    }
    acc = wave_sum(acc);
    if (threadIdx.x % kWave == 0)
        lds[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        partials[blockIdx.x] = ((lds[0] + lds[1]) + lds[2]) + lds[3];
}

__global__ void k_boltzmann_scale(double *w, int64_t n, double numer, const double *Z)
{
    const double z = *Z;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        w[i] = numer * w[i] / z;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Four 16-byte words per thread, loaded before any is stored, streamed past the caches.
__global__ __launch_bounds__(256) void k_stream_copy(const f32x4 *__restrict__ src,
                                                      f32x4 *__restrict__ dst, int64_t n)
{
    const int64_t base = static_cast<int64_t>(blockIdx.x) * 1024 + threadIdx.x;
    f32x4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + k * 256 < n)
            v[k] = __builtin_nontemporal_load(src + base + k * 256);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + k * 256 < n)
            __builtin_nontemporal_store(v[k], dst + base + k * 256);
}

// The FP64 full sweep's memory pattern without its arithmetic: workgroups of 64 x 4 columns
// marching a run of z-planes, each thread reading the 12 values of its column one plane
// ahead and writing 9 past the caches, one barrier per plane. Each output is its input plus
// a value formed from the other three inputs, so no load can be dropped.
__global__ __launch_bounds__(kThreads, 2) void k_stream_columns(ColumnArrays c, int nx, int ny,
                                                                int nz, int zc, int tiles_x,
                                                                int tiles_y)
{
    constexpr int TX = 64, TY = kThreads / TX;
    const int t = static_cast<int>(threadIdx.x);
    const int tiles = tiles_x * tiles_y;
    const int tile = static_cast<int>(blockIdx.x % tiles);
    const int chunk = static_cast<int>(blockIdx.x / tiles);
    const int x = (tile % tiles_x) * TX + t % TX, y = (tile / tiles_x) * TY + t / TX;
    const int z0 = chunk * zc, z1 = min(nz, z0 + zc);
    const bool act = x < nx && y < ny;
    const int64_t plane = static_cast<int64_t>(nx) * ny, col = x + static_cast<int64_t>(nx) * y;
    double v[2][kColumnIn];
    auto load = [&](double *d, int z) {
#pragma unroll
        for (int k = 0; k < kColumnIn; ++k)
            d[k] = act && z < z1 ? c.in[k][plane * z + col] : 0.0;
    };
    auto store = [&](const double *d, int z) {
        if (!(act && z < z1))
            return;
        const double e = d[kColumnOut] + d[kColumnOut + 1] * d[kColumnOut + 2];
#pragma unroll
        for (int k = 0; k < kColumnOut; ++k)
            __builtin_nontemporal_store(d[k] + e, c.out[k] + plane * z + col);
    };
    load(v[0], z0);
    for (int z = z0; z < z1; z += 2) {
        load(v[1], z + 1);
        __syncthreads();
        store(v[0], z);
        load(v[0], z + 2);
        __syncthreads();
        store(v[1], z + 1);
    }
}

int grid_for(int64_t n, int threads)
{
    int64_t g = (n + threads - 1) / threads;
    if (g > 8192)
        g = 8192;
    return static_cast<int>(g < 1 ? 1 : g);
}

#endif  // LPC_HOST_PART

// ---------------------------------------------------------------------------- dispatch

struct RecordLauncher {
    template <typename S, bool FID, int MSD, bool, int MAXR>
    static hipError_t go(const SweepPlan &p, const StepArgs &a, hipStream_t s)
    {
        const int64_t padded = (p.nblocks + 7) / 8 * 8;
        hipLaunchKernelGGL((k_record_tile<S, FID, MSD, MAXR>), dim3(static_cast<unsigned>(padded)),
                           dim3(kThreads), 0, s, a, p, padded);
        return hipGetLastError();
    }
};

struct ListLauncher {
    template <typename S, bool FID, int MSD, bool EXT, int MAXR>
    static hipError_t go(const SweepPlan &, const StepArgs &, hipStream_t s, const StepList *L)
    {
        const int64_t padded = (L->total + 7) / 8 * 8;
        const dim3 grid(static_cast<unsigned>(padded)), block(kThreads);
        if (L->tile_x == kTileTwoStep) {
            if constexpr (EXT || MSD == 2)
                return hipErrorInvalidValue;        // two-step plans: plain variant, no tags
            else
                hipLaunchKernelGGL((k_sweep2_tile<S, FID, MSD, MAXR>), grid, block, 0, s, L->items,
                                   L->prefix, L->n_items, L->total, padded, L->parity, L->slot);
        } else if (L->tile_x == kTileLinear) {
            if constexpr (EXT)
                return hipErrorInvalidValue;        // plans never give the extended variant these
            else
                hipLaunchKernelGGL((k_sweep_tile<S, FID, MSD, false, MAXR, kTileLinear>), grid, block,
                                   0, s, L->items, L->prefix, L->n_items, L->total, padded,
                                   L->parity, L->slot);
        } else if (L->tile_x == 64)
            hipLaunchKernelGGL((k_sweep_tile<S, FID, MSD, EXT, MAXR, 64>), grid, block, 0, s, L->items,
                               L->prefix, L->n_items, L->total, padded, L->parity, L->slot);
        else if (L->tile_x == 32)
            hipLaunchKernelGGL((k_sweep_tile<S, FID, MSD, EXT, MAXR, 32>), grid, block, 0, s, L->items,
                               L->prefix, L->n_items, L->total, padded, L->parity, L->slot);
        else
            hipLaunchKernelGGL((k_sweep_tile<S, FID, MSD, EXT, MAXR, 16>), grid, block, 0, s, L->items,
                               L->prefix, L->n_items, L->total, padded, L->parity, L->slot);
        return hipGetLastError();
    }
};

template <typename L, typename S, bool FID, int MSD, bool EXT, typename... X>
hipError_t by_regions(const SweepPlan &p, const StepArgs &a, hipStream_t s, X... x)
{
    if (a.R == 1)
        return L::template go<S, FID, MSD, EXT, 1>(p, a, s, x...);
    if (a.R == 2)
        return L::template go<S, FID, MSD, EXT, 2>(p, a, s, x...);
    if (a.R <= 4)
        return L::template go<S, FID, MSD, EXT, 4>(p, a, s, x...);
    return L::template go<S, FID, MSD, EXT, 8>(p, a, s, x...);
}

template <typename L, typename S, bool EXT, typename... X>
hipError_t by_fields(const SweepPlan &p, const StepArgs &a, hipStream_t s, X... x)
{
    const bool fid = a.track & 1u, msd = a.track & 2u, vacf = a.track & kTrackVacf;
    if (vacf)      // the tags come with the moments
        return fid ? by_regions<L, S, true, 2, EXT>(p, a, s, x...)
                   : by_regions<L, S, false, 2, EXT>(p, a, s, x...);
    if (fid && msd)
        return by_regions<L, S, true, true, EXT>(p, a, s, x...);
    if (fid)
        return by_regions<L, S, true, false, EXT>(p, a, s, x...);
    if (msd)
        return by_regions<L, S, false, true, EXT>(p, a, s, x...);
    return by_regions<L, S, false, false, EXT>(p, a, s, x...);
}

struct OccupancyQuery {
    template <typename S, bool FID, int MSD, bool EXT, int MAXR>
    static hipError_t go(const SweepPlan &, const StepArgs &, hipStream_t, int *out)
    {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            out, reinterpret_cast<const void *>(&k_sweep_tile<S, FID, MSD, EXT, MAXR, 64>),
            kThreads, 0);
    }
};

struct OccupancyQuery2 {
    template <typename S, bool FID, int MSD, bool EXT, int MAXR>
    static hipError_t go(const SweepPlan &, const StepArgs &, hipStream_t, int *out)
    {
        if constexpr (EXT || MSD == 2)
            return hipErrorInvalidValue;
        else
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                out, reinterpret_cast<const void *>(&k_sweep2_tile<S, FID, MSD, MAXR>), kThreads,
                0);
    }
};

}  // namespace

// Per-part entry points: the sweep work list, the occupancy query and the record kernel of
// one storage type and variant (defined in the part that compiles those instances).
template <typename S, bool EXT>
hipError_t step_list_part(const StepList &L, uint32_t track, int32_t maxr, hipStream_t s);
template <typename S, bool EXT>
int occupancy_part(uint32_t track, int32_t R, int32_t steps_per_pass);
template <typename S>
hipError_t record_part(const SweepPlan &plan, const StepArgs &a, hipStream_t s);

#if !(LPC_SWEEP_PART == 4)
template <typename S, bool EXT>
hipError_t step_list_part(const StepList &L, uint32_t track, int32_t maxr, hipStream_t s)
{
    StepArgs a{};
    a.track = track;
    a.R = maxr;
    return by_fields<ListLauncher, S, EXT>(SweepPlan{}, a, s, &L);
}

template <typename S, bool EXT>
int occupancy_part(uint32_t track, int32_t R, int32_t steps_per_pass)
{
    StepArgs a{};
    a.track = track;
    a.R = R;
    int n = 0;
    const hipError_t e = steps_per_pass == 2
                             ? by_fields<OccupancyQuery2, S, EXT>(SweepPlan{}, a, nullptr, &n)
                             : by_fields<OccupancyQuery, S, EXT>(SweepPlan{}, a, nullptr, &n);
    if (e != hipSuccess || n < 1)
        return 1;
    return n;
}

template <typename S>
hipError_t record_part(const SweepPlan &plan, const StepArgs &a, hipStream_t s)
{
    return by_fields<RecordLauncher, S, false>(plan, a, s);
}
#endif

#if LPC_PART_IS(0)
template hipError_t step_list_part<double, false>(const StepList &, uint32_t, int32_t, hipStream_t);
template int occupancy_part<double, false>(uint32_t, int32_t, int32_t);
template hipError_t record_part<double>(const SweepPlan &, const StepArgs &, hipStream_t);
#endif
#if LPC_PART_IS(1)
template hipError_t step_list_part<double, true>(const StepList &, uint32_t, int32_t, hipStream_t);
template int occupancy_part<double, true>(uint32_t, int32_t, int32_t);
#endif
#if LPC_PART_IS(2)
template hipError_t step_list_part<float, false>(const StepList &, uint32_t, int32_t, hipStream_t);
template int occupancy_part<float, false>(uint32_t, int32_t, int32_t);
template hipError_t record_part<float>(const SweepPlan &, const StepArgs &, hipStream_t);
#endif
#if LPC_PART_IS(3)
template hipError_t step_list_part<float, true>(const StepList &, uint32_t, int32_t, hipStream_t);
template int occupancy_part<float, true>(uint32_t, int32_t, int32_t);
#endif

#if LPC_HOST_PART

// Tile width for a lattice of nx columns: the widest tile whose padded width is within
// 1.5 times the least padded width. Full 64-site rows load far better than narrow ones, more
// than the idle lanes of moderate padding cost (100 columns: 64 wide padded to 128 runs
// 1.4 times faster than 16 wide padded to 112).
int32_t tile_width(int32_t nx)
{
    int64_t least = -1;
    for (int32_t tx : {64, 32, 16}) {
        const int64_t pad = (nx + tx - 1) / tx * int64_t(tx);
        least = least < 0 || pad < least ? pad : least;
    }
    for (int32_t tx : {64, 32, 16}) {
        const int64_t pad = (nx + tx - 1) / tx * int64_t(tx);
        if (2 * pad <= 3 * least)
            return tx;
    }
    return 16;
}

// Tiles of one plane for tile width tx (kTileLinear: linear tiles).
int64_t plane_tiles(const Geometry &g, int32_t tx)
{
    if (tx == kTileLinear)
        return (int64_t(g.nx) * g.ny + kThreads - 1) / kThreads;
    if (tx == kTileTwoStep)
        return int64_t((g.nx + kTwoStepTileX - 1) / kTwoStepTileX) *
               ((g.ny + kTwoStepTileY - 1) / kTwoStepTileY);
    const int32_t ty = kThreads / tx;
    return int64_t((g.nx + tx - 1) / tx) * ((g.ny + ty - 1) / ty);
}

int64_t max_sweep_blocks(const Geometry &g)
{
    int64_t most = 0;
    for (int32_t tx : {64, 32, 16, kTileLinear, kTileTwoStep}) {
        const int64_t tiles = plane_tiles(g, tx);
        const int64_t gz = std::max<int64_t>((g.nz + 7) / 8, (8192 + tiles - 1) / tiles);
        most = std::max(most, tiles * std::min<int64_t>(g.nz, gz));
    }
    return most;
}

// Pick the z-chunk of a plan with `tiles` tiles per plane: every resident slot busy until
// the end (greedy makespan of the chunks against the ideal), few extra planes per chunk
// (each chunk re-reads the planes around it, mostly from cache; `extra` planes' worth of work
// per chunk), and a few rounds to absorb uneven progress. A chunk of at least zc_floor planes
// (or the whole axis): shorter chunks re-read too large a share of planes around them. 4 for
// a lattice stepped alone; a lattice stepped in a batch takes 16 (the 512-particle batch:
// 46.0 GSU/s at 16 against 41.3 at 4), since the other lattices fill the device.
int32_t choose_z_chunk(const Geometry &g, int64_t tiles, int32_t blocks_per_cu, int32_t cus,
                       int32_t zc_floor, double extra)
{
    const int64_t conc = std::max(1, blocks_per_cu) * static_cast<int64_t>(std::max(1, cus));
    const int64_t gz_cap = std::max<int64_t>((g.nz + 7) / 8, (8192 + tiles - 1) / tiles);
    const int64_t gz_max = std::min<int64_t>(g.nz, gz_cap);
    const int32_t zc_min = std::min(g.nz, std::max(1, zc_floor));
    double best = -1.0;
    int32_t best_zc = g.nz;
    for (int64_t gz = 1; gz <= gz_max; ++gz) {
        const int32_t zc = static_cast<int32_t>((g.nz + gz - 1) / gz);
        const int64_t gze = (g.nz + zc - 1) / zc;
        if (gze != gz || zc < zc_min)
            continue;
        const int64_t T = tiles * gze;
        const int64_t rounds = (T + conc - 1) / conc;
        const double ideal = static_cast<double>(tiles) * g.nz / static_cast<double>(conc);
        const double fill = ideal / static_cast<double>(rounds * zc);
        const double pro = zc / (zc + extra);
        const double eff = fill * pro * (1.0 - 0.05 / static_cast<double>(rounds));
        if (eff > best + 1e-12) {
            best = eff;
            best_zc = zc;
        }
    }
    return best_zc;
}

SweepPlan make_plan(const Geometry &g, int32_t blocks_per_cu, int32_t cus, int32_t tile_x,
                    int32_t linear_nx_max, int32_t zc_floor)
{
    SweepPlan p{};
    const bool linear_ok = g.nx <= linear_nx_max;
    if (tile_x == 64 || tile_x == 32 || tile_x == 16 || (tile_x == kTileLinear && linear_ok)) {
        p.tx = tile_x;
    } else {
        // block tiles by the padding rule, unless linear tiles leave fewer lanes idle
        p.tx = tile_width(g.nx);
        if (linear_ok && plane_tiles(g, kTileLinear) < plane_tiles(g, p.tx))
            p.tx = kTileLinear;
    }
    if (p.tx == kTileLinear) {
        p.ty = kThreads;
        p.gx = static_cast<int32_t>(plane_tiles(g, kTileLinear));
        p.gy = 1;
    } else {
        p.ty = kThreads / p.tx;
        p.gx = (g.nx + p.tx - 1) / p.tx;
        p.gy = (g.ny + p.ty - 1) / p.ty;
    }
    const int64_t tiles = static_cast<int64_t>(p.gx) * p.gy;
    p.zc = choose_z_chunk(g, tiles, blocks_per_cu, cus, zc_floor, 0.5);
    p.gz = (g.nz + p.zc - 1) / p.zc;
    p.nblocks = tiles * p.gz;
    return p;
}

SweepPlan make_plan2(const Geometry &g, int32_t blocks_per_cu, int32_t cus, int32_t zc_floor)
{
    SweepPlan p{};
    p.tx = kTileTwoStep;
    p.ty = kTwoStepTileY;
    p.gx = (g.nx + kTwoStepTileX - 1) / kTwoStepTileX;
    p.gy = (g.ny + kTwoStepTileY - 1) / kTwoStepTileY;
    const int64_t tiles = static_cast<int64_t>(p.gx) * p.gy;
    // a chunk's first step also runs on the plane on either side of it, and its level-0
    // window reads two planes on either side
    p.zc = choose_z_chunk(g, tiles, blocks_per_cu, cus, zc_floor, 2.0);
    p.gz = (g.nz + p.zc - 1) / p.zc;
    p.nblocks = tiles * p.gz;
    return p;
}

SweepPlan with_z_chunk(SweepPlan p, const Geometry &g, int32_t zc)
{
    p.zc = std::max(1, std::min(zc, g.nz));
    p.gz = (g.nz + p.zc - 1) / p.zc;
    p.nblocks = static_cast<int64_t>(p.gx) * p.gy * p.gz;
    return p;
}

int32_t linear_tile_max_nx(int32_t precision, uint32_t track)
{
    if (track & kVariantExtended)
        return 0;
    const bool fid = track & 1u;
    const int mom = (track & kTrackVacf) ? 2 : ((track & 2u) ? 1 : 0);
    if (precision == 0) {
        if (mom == 2)
            return fid ? linear_nx_max<double, true, 2>() : linear_nx_max<double, false, 2>();
        return fid ? (mom ? linear_nx_max<double, true, 1>() : linear_nx_max<double, true, 0>())
                   : (mom ? linear_nx_max<double, false, 1>() : linear_nx_max<double, false, 0>());
    }
    if (mom == 2)
        return fid ? linear_nx_max<float, true, 2>() : linear_nx_max<float, false, 2>();
    return fid ? (mom ? linear_nx_max<float, true, 1>() : linear_nx_max<float, true, 0>())
               : (mom ? linear_nx_max<float, false, 1>() : linear_nx_max<float, false, 0>());
}

int sweep_blocks_per_cu(int32_t precision, uint32_t track, int32_t R, int32_t steps_per_pass)
{
    const bool ext = track & kVariantExtended;
    const int k = steps_per_pass;
    if (precision == 0)
        return ext ? occupancy_part<double, true>(track, R, k)
                   : occupancy_part<double, false>(track, R, k);
    return ext ? occupancy_part<float, true>(track, R, k) : occupancy_part<float, false>(track, R, k);
}

hipError_t launch_step_list(const StepList &L, int32_t precision, uint32_t track, int32_t maxr,
                            hipStream_t s)
{
    if (L.total <= 0)
        return hipSuccess;
    const bool ext = track & kVariantExtended;
    if (precision == 0)
        return ext ? step_list_part<double, true>(L, track, maxr, s)
                   : step_list_part<double, false>(L, track, maxr, s);
    return ext ? step_list_part<float, true>(L, track, maxr, s)
               : step_list_part<float, false>(L, track, maxr, s);
}

hipError_t launch_record(const SweepPlan &plan, const StepArgs &a, hipStream_t s)
{
    return a.precision == 0 ? record_part<double>(plan, a, s) : record_part<float>(plan, a, s);
}

hipError_t launch_finalize_list(const FinalizeItem *items, const int64_t *kprefix, int32_t n_items,
                                int64_t total_k, int64_t steps, int64_t first_row, hipStream_t s,
                                const int64_t *row_offset)
{
    if (steps <= 0 || total_k <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_finalize_list, dim3(static_cast<unsigned>(steps * total_k)), dim3(256), 0,
                       s, items, kprefix, n_items, total_k, first_row, row_offset);
    return hipGetLastError();
}

hipError_t launch_set_counter(int64_t *counter, int64_t value, int64_t add, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(1), 0, s, counter, value, add);
    return hipGetLastError();
}

hipError_t launch_finalize(const double *partials, int64_t nblocks, int32_t K, int64_t steps,
                           double *records_out, hipStream_t s)
{
    if (steps <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3(static_cast<unsigned>(steps * K)), dim3(256), 0, s,
                       partials, nblocks, K, records_out);
    return hipGetLastError();
}

hipError_t launch_store_field(int32_t precision, const double *src, void *dst, int64_t n,
                              double scale, hipStream_t s)
{
    const int g = grid_for(n, 256);
    if (precision == 0)
        hipLaunchKernelGGL(k_store_field<double>, dim3(g), dim3(256), 0, s, src,
                           static_cast<double *>(dst), n, scale);
    else
        hipLaunchKernelGGL(k_store_field<float>, dim3(g), dim3(256), 0, s, src,
                           static_cast<float *>(dst), n, scale);
    return hipGetLastError();
}

hipError_t launch_init_state(int32_t precision, uint32_t track, const StateView &st,
                             const double *rho_src, const void *F, int64_t n, hipStream_t s)
{
    const int g = grid_for(n, 256);
    const bool fid = track & 1u, msd = track & 2u;
    if (precision == 0)
        hipLaunchKernelGGL(k_init_state<double>, dim3(g), dim3(256), 0, s, typed<double>(st), fid,
                           msd, rho_src, static_cast<const double *>(F), n);
    else
        hipLaunchKernelGGL(k_init_state<float>, dim3(g), dim3(256), 0, s, typed<float>(st), fid,
                           msd, rho_src, static_cast<const float *>(F), n);
    return hipGetLastError();
}

hipError_t launch_fill_field(int32_t precision, void *dst, int64_t n, double value,
                             hipStream_t s)
{
    const int g = grid_for(n, 256);
    if (precision == 0)
        hipLaunchKernelGGL(k_fill<double>, dim3(g), dim3(256), 0, s, static_cast<double *>(dst), n,
                           value);
    else
        hipLaunchKernelGGL(k_fill<float>, dim3(g), dim3(256), 0, s, static_cast<float *>(dst), n,
                           static_cast<float>(value));
    return hipGetLastError();
}

hipError_t launch_boltzmann_weights(int32_t precision, const void *F, double Fmin, double *w,
                                    int64_t n, double *partials, int64_t *nb, hipStream_t s)
{
    *nb = kWeightBlocks;
    if (precision == 0)
        hipLaunchKernelGGL(k_boltzmann_weights<double>, dim3(kWeightBlocks), dim3(256), 0, s,
                           static_cast<const double *>(F), Fmin, w, n, partials);
    else
        hipLaunchKernelGGL(k_boltzmann_weights<float>, dim3(kWeightBlocks), dim3(256), 0, s,
                           static_cast<const float *>(F), Fmin, w, n, partials);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const void *src, void *dst, int64_t n16, hipStream_t s)
{
    if (n16 <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_stream_copy, dim3(static_cast<unsigned>((n16 + 1023) / 1024)), dim3(256),
                       0, s, static_cast<const f32x4 *>(src), static_cast<f32x4 *>(dst), n16);
    return hipGetLastError();
}

hipError_t launch_stream_columns(const ColumnArrays &c, int32_t nx, int32_t ny, int32_t nz,
                                 int32_t zc, hipStream_t s)
{
    const int tiles_x = (nx + 63) / 64, tiles_y = (ny + 3) / 4;
    const int64_t blocks = int64_t(tiles_x) * tiles_y * ((nz + zc - 1) / zc);
    hipLaunchKernelGGL(k_stream_columns, dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0, s,
                       c, nx, ny, nz, zc, tiles_x, tiles_y);
    return hipGetLastError();
}

hipError_t launch_boltzmann_factors(const double *F, double *E, int64_t n, double fc,
                                    hipStream_t s)
{
    hipLaunchKernelGGL(k_boltzmann_factors, dim3(grid_for(n, 256)), dim3(256), 0, s, F, E, n, fc);
    return hipGetLastError();
}

hipError_t launch_boltzmann_scale(double *w, int64_t n, double numer, const double *Z,
                                  hipStream_t s)
{
    hipLaunchKernelGGL(k_boltzmann_scale, dim3(grid_for(n, 256)), dim3(256), 0, s, w, n, numer, Z);
    return hipGetLastError();
}

#endif  // LPC_HOST_PART

}  // namespace lpc
