// Lattice sweep kernels for gfx950 (MI355X).
//
// One step of the LPC3D lattice model (paper section 2; Eqs. (1), (11)-(13) and moment
// propagation of section 2.2) for populations rho, complex magnetisation m and per-axis
// displacement moments M1, M2, plus the per-step sums over sites of Eqs. (11)-(12).
//
// The update is written in flux form: for every link (i, j),
//     x'_i += p(j->i) x_j - p(i->j) x_i,
// which equals stay(i) x_i + sum_j p(j->i) x_j since stay(i) = 1 - sum_j p(i->j). The
// flux of a link evaluated at its two ends is exactly antisymmetric in floating point,
// so no per-site rounding of stay(i) can bias the totals from step to step: the total
// population is conserved to rounding noise and the float-stored fields of the mixed
// path do not drift. The one exponential of a link gives both directions:
// p(i->j) = p0 e^{-|dF|} if F_j > F_i else p0, and p(j->i) the other way round (Eq. (1)).
//
// Magnetisation rotates after the gather by the destination's phase (Eq. (13)), applied
// as m + m (cos t - 1) + i m sin t with cos t - 1 = -2 sin^2(t/2), which keeps |m| from
// drifting when t is stored in float.
//
// Per-step sums are deterministic: each workgroup reduces its sites with wave-level
// butterflies and a fixed-order pass over its waves into one partial per record entry,
// and a finalize kernel sums the partials of all workgroups in a fixed order. No
// floating-point atomics are used anywhere.
#include "lpc_internal.h"

#include <hip/hip_runtime.h>

namespace lpc {
namespace {

constexpr int kWave = 64;

template <typename S>
struct View {
    double *rho;
    S *re, *im;
    S *m1[3], *m2[3];
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
    }
    return t;
}

// Hop probabilities of one link, Eq. (1): p_out = p(i->j), p_in = p(j->i).
__device__ inline void link_probs(double Fi, double Fj, double p0, double &p_out, double &p_in)
{
    const double dF = Fj - Fi;
    const double pe = p0 * exp(-fabs(dF));
    const bool up = dF > 0.0;
    p_out = up ? pe : p0;
    p_in = up ? p0 : pe;
}

__device__ inline void link_probs(float Fi, float Fj, float p0, double &p_out, double &p_in)
{
    const float dF = Fj - Fi;
    const float pe = p0 * expf(-fabsf(dF));
    const bool up = dF > 0.0f;
    p_out = static_cast<double>(up ? pe : p0);
    p_in = static_cast<double>(up ? p0 : pe);
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

// Neighbour index one hop along an axis (sign +1 / -1); false across a closed face.
__device__ inline bool neighbour(int c, int n, int bc, int64_t stride, int sgn, int64_t i,
                                 int64_t &j)
{
    if (sgn > 0) {
        if (c + 1 < n) {
            j = i + stride;
            return true;
        }
        if (bc == 0) {
            j = i - static_cast<int64_t>(n - 1) * stride;
            return true;
        }
        return false;
    }
    if (c > 0) {
        j = i - stride;
        return true;
    }
    if (bc == 0) {
        j = i + static_cast<int64_t>(n - 1) * stride;
        return true;
    }
    return false;
}

// Register accumulators of one thread's record contributions.
template <int MAXR>
struct RecAcc {
    double re[MAXR], im[MAXR], u[MAXR], s1[3], s2[3];

    __device__ void zero()
    {
#pragma unroll
        for (int r = 0; r < MAXR; ++r)
            re[r] = im[r] = u[r] = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            s1[a] = s2[a] = 0.0;
    }

    __device__ void add_site(int r, double vre, double vim, double vu)
    {
        if (MAXR == 1) {
            re[0] += vre;
            im[0] += vim;
            u[0] += vu;
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

// Reduces the block's accumulators into partials[k * nblocks + blk], k < K, in a fixed
// order (butterfly inside each wave, then waves in index order).
template <int MAXR, int NWAVES>
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
// [x * per, (x + 1) * per) of tiles, so halo-sharing neighbours mostly meet in one L2.
__device__ inline int64_t logical_block(int64_t b, int64_t padded)
{
    const int64_t per = padded / 8;
    return (b % 8) * per + b / 8;
}

// ---------------------------------------------------------------------------- one site

template <typename S, bool FID, bool MSD, int MAXR>
__device__ inline void step_site(const StepArgs &a, const View<S> &src, const View<S> &dst, int x,
                                 int y, int z, RecAcc<MAXR> &acc)
{
    const Geometry &g = a.g;
    const S *F = static_cast<const S *>(a.F);
    const S *TH = static_cast<const S *>(a.theta);
    const int64_t sx = 1, sy = g.nx, sz = static_cast<int64_t>(g.nx) * g.ny;
    const int64_t i = x + sy * y + sz * z;
    const S Fi = F[i];
    const S p0 = static_cast<S>(a.p0);
    const double rho_i = src.rho[i];
    double f_rho = 0.0;
    double re_i = 0.0, im_i = 0.0, f_re = 0.0, f_im = 0.0;
    if (FID) {
        re_i = static_cast<double>(src.re[i]);
        im_i = static_cast<double>(src.im[i]);
    }
    double m1_i[3] = {0.0, 0.0, 0.0}, m2_i[3] = {0.0, 0.0, 0.0};
    double f1[3] = {0.0, 0.0, 0.0}, f2[3] = {0.0, 0.0, 0.0};
    if (MSD) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            m1_i[b] = static_cast<double>(src.m1[b][i]);
            m2_i[b] = static_cast<double>(src.m2[b][i]);
        }
    }
    const int c[3] = {x, y, z};
    const int n[3] = {g.nx, g.ny, g.nz};
    const int64_t st[3] = {sx, sy, sz};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
#pragma unroll
        for (int sg = 0; sg < 2; ++sg) {
            const int sgn = sg == 0 ? 1 : -1;
            int64_t j;
            if (!neighbour(c[ax], n[ax], g.bc[ax], st[ax], sgn, i, j))
                continue;  // attempt across a closed face: the particle stays
            double p_out, p_in;
            link_probs(Fi, F[j], p0, p_out, p_in);
            const double rho_j = src.rho[j];
            f_rho += exact_flux(p_in, rho_j, p_out, rho_i);
            if (FID) {
                f_re += p_in * static_cast<double>(src.re[j]) - p_out * re_i;
                f_im += p_in * static_cast<double>(src.im[j]) - p_out * im_i;
            }
            if (MSD) {
                const double d = -sgn;  // hop j -> i along ax (unwrapped)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const double m1j = static_cast<double>(src.m1[b][j]);
                    const double m2j = static_cast<double>(src.m2[b][j]);
                    if (b == ax) {
                        f1[b] += p_in * (m1j + d * rho_j) - p_out * m1_i[b];
                        f2[b] += p_in * (m2j + 2.0 * d * m1j + rho_j) - p_out * m2_i[b];
                    } else {
                        f1[b] += p_in * m1j - p_out * m1_i[b];
                        f2[b] += p_in * m2j - p_out * m2_i[b];
                    }
                }
            }
        }
    }
    const double rho_n = rho_i + f_rho;
    dst.rho[i] = rho_n;
    double out_re = 0.0, out_im = 0.0;
    if (FID) {
        const double gre = re_i + f_re, gim = im_i + f_im;
        double sh, ch;
        sincos(0.5 * static_cast<double>(TH[i]), &sh, &ch);
        const double sn = 2.0 * sh * ch, cm1 = -2.0 * sh * sh;
        const S nre = static_cast<S>(gre + (gre * cm1 - gim * sn));
        const S nim = static_cast<S>(gim + (gim * cm1 + gre * sn));
        dst.re[i] = nre;
        dst.im[i] = nim;
        out_re = static_cast<double>(nre);
        out_im = static_cast<double>(nim);
    }
    if (MSD) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const S v1 = static_cast<S>(m1_i[b] + f1[b]);
            const S v2 = static_cast<S>(m2_i[b] + f2[b]);
            dst.m1[b][i] = v1;
            dst.m2[b][i] = v2;
            acc.s1[b] += static_cast<double>(v1);
            acc.s2[b] += static_cast<double>(v2);
        }
    }
    acc.add_site(MAXR == 1 ? 0 : a.region[i], out_re, out_im, rho_n);
}

template <typename S, bool FID, bool MSD, int MAXR>
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

// ---------------------------------------------------------------------------- kernels

constexpr int kDirectTX = 64, kDirectTY = 4, kDirectThreads = kDirectTX * kDirectTY;

// One thread per (x, y) of a 64 x 4 tile, marching the workgroup's run of z-planes;
// neighbours are read straight from global memory (cache hits inside the tile).
template <typename S, bool FID, bool MSD, int MAXR, bool RECORD_ONLY>
__global__ __launch_bounds__(kDirectThreads) void k_sweep_direct(StepArgs a, SweepPlan p,
                                                                 int64_t padded)
{
    __shared__ double lds[(kDirectThreads / kWave) * (3 * MAXR + 6)];
    const int64_t blk = logical_block(blockIdx.x, padded);
    if (blk >= p.nblocks)
        return;
    const int bx = static_cast<int>(blk % p.gx);
    const int64_t rest = blk / p.gx;
    const int by = static_cast<int>(rest % p.gy);
    const int bz = static_cast<int>(rest / p.gy);
    const int x = bx * kDirectTX + static_cast<int>(threadIdx.x % kDirectTX);
    const int y = by * kDirectTY + static_cast<int>(threadIdx.x / kDirectTX);
    const View<S> src = typed<S>(a.src);
    const View<S> dst = typed<S>(a.dst);
    RecAcc<MAXR> acc;
    acc.zero();
    if (x < a.g.nx && y < a.g.ny) {
        const int z0 = bz * p.zc;
        const int z1 = min(a.g.nz, z0 + p.zc);
        for (int z = z0; z < z1; ++z) {
            if (RECORD_ONLY) {
                const int64_t i = x + static_cast<int64_t>(a.g.nx) * (y + static_cast<int64_t>(a.g.ny) * z);
                record_site<S, FID, MSD, MAXR>(a, src, i, acc);
            } else {
                step_site<S, FID, MSD, MAXR>(a, src, dst, x, y, z, acc);
            }
        }
    }
    block_reduce<MAXR, kDirectThreads / kWave>(acc, a.R, a.K, a.partials, p.nblocks, blk, lds);
}

__global__ __launch_bounds__(256) void k_finalize(const double *partials, int64_t nblocks, int K,
                                                  double *out)
{
    __shared__ double w[4];
    const int s = blockIdx.x / K, k = blockIdx.x % K;
    const double *p = partials + (static_cast<int64_t>(s) * K + k) * nblocks;
    double v = 0.0;
    for (int64_t b = threadIdx.x; b < nblocks; b += 256)
        v += p[b];
    v = wave_sum(v);
    if (threadIdx.x % kWave == 0)
        w[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        out[static_cast<int64_t>(s) * K + k] = ((w[0] + w[1]) + w[2]) + w[3];
}

template <typename S>
__global__ void k_store_field(const double *src, S *dst, int64_t n, double scale)
{
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        dst[i] = static_cast<S>(scale == 1.0 ? src[i] : scale * src[i]);
}

template <typename S>
__global__ void k_init_state(View<S> st, bool fid, bool msd, const double *rho_src, int64_t n)
{
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double r = rho_src ? rho_src[i] : 1.0;
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
    }
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

int grid_for(int64_t n, int threads)
{
    int64_t g = (n + threads - 1) / threads;
    if (g > 8192)
        g = 8192;
    return static_cast<int>(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------------------- dispatch

template <bool RECORD_ONLY>
struct DirectLauncher {
    template <typename S, bool FID, bool MSD, int MAXR>
    static hipError_t go(const SweepPlan &p, const StepArgs &a, hipStream_t s)
    {
        const int64_t padded = (p.nblocks + 7) / 8 * 8;
        hipLaunchKernelGGL((k_sweep_direct<S, FID, MSD, MAXR, RECORD_ONLY>),
                           dim3(static_cast<unsigned>(padded)), dim3(kDirectThreads), 0, s, a, p,
                           padded);
        return hipGetLastError();
    }
};

template <typename L, typename S, bool FID, bool MSD>
hipError_t by_regions(const SweepPlan &p, const StepArgs &a, hipStream_t s)
{
    if (a.R == 1)
        return L::template go<S, FID, MSD, 1>(p, a, s);
    if (a.R == 2)
        return L::template go<S, FID, MSD, 2>(p, a, s);
    if (a.R <= 4)
        return L::template go<S, FID, MSD, 4>(p, a, s);
    return L::template go<S, FID, MSD, 8>(p, a, s);
}

template <typename L, typename S>
hipError_t by_track(const SweepPlan &p, const StepArgs &a, hipStream_t s)
{
    const bool fid = a.track & 1u, msd = a.track & 2u;
    if (fid && msd)
        return by_regions<L, S, true, true>(p, a, s);
    if (fid)
        return by_regions<L, S, true, false>(p, a, s);
    if (msd)
        return by_regions<L, S, false, true>(p, a, s);
    return by_regions<L, S, false, false>(p, a, s);
}

template <typename L>
hipError_t by_precision(const SweepPlan &p, const StepArgs &a, hipStream_t s)
{
    if (a.precision == 0)
        return by_track<L, double>(p, a, s);
    return by_track<L, float>(p, a, s);
}

}  // namespace

SweepPlan make_plan(const Geometry &g, int32_t kernel_hint)
{
    (void)kernel_hint;
    SweepPlan p{};
    p.kernel = 0;
    p.tx = kDirectTX;
    p.ty = kDirectTY;
    p.gx = (g.nx + p.tx - 1) / p.tx;
    p.gy = (g.ny + p.ty - 1) / p.ty;
    const int64_t tiles = static_cast<int64_t>(p.gx) * p.gy;
    const int64_t target = 4096;
    int64_t gz = (target + tiles - 1) / tiles;
    if (gz > g.nz)
        gz = g.nz;
    if (gz < 1)
        gz = 1;
    p.zc = static_cast<int32_t>((g.nz + gz - 1) / gz);
    p.gz = (g.nz + p.zc - 1) / p.zc;
    p.nblocks = tiles * p.gz;
    return p;
}

hipError_t launch_step(const SweepPlan &plan, const StepArgs &a, hipStream_t s)
{
    return by_precision<DirectLauncher<false>>(plan, a, s);
}

hipError_t launch_record(const SweepPlan &plan, const StepArgs &a, hipStream_t s)
{
    return by_precision<DirectLauncher<true>>(plan, a, s);
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
                             const double *rho_src, int64_t n, hipStream_t s)
{
    const int g = grid_for(n, 256);
    const bool fid = track & 1u, msd = track & 2u;
    if (precision == 0)
        hipLaunchKernelGGL(k_init_state<double>, dim3(g), dim3(256), 0, s, typed<double>(st), fid,
                           msd, rho_src, n);
    else
        hipLaunchKernelGGL(k_init_state<float>, dim3(g), dim3(256), 0, s, typed<float>(st), fid,
                           msd, rho_src, n);
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

hipError_t launch_boltzmann_scale(double *w, int64_t n, double numer, const double *Z,
                                  hipStream_t s)
{
    hipLaunchKernelGGL(k_boltzmann_scale, dim3(grid_for(n, 256)), dim3(256), 0, s, w, n, numer, Z);
    return hipGetLastError();
}

}  // namespace lpc
