// Post-processing kernels for gfx950: the NMR spectrum of a recorded FID (Eq. (9) of the
// LPC3D paper), its peak, and population profiles of the state.
//
// The spectrum is a zero-filled radix-2 Stockham FFT in FP64 (out of place, ping-pong
// between two device buffers, one launch per pass, twiddles from sincospi), with the
// forward kernel exp(-2 pi i k n / L): a site precessing as exp(+i theta n) then peaks at
// f = +theta / (2 pi dt). Reductions are deterministic (fixed-order tree per workgroup,
// then a fixed-order pass over workgroups).
#include "lpc_internal.h"

#include <hip/hip_runtime.h>

namespace lpc {
namespace {

constexpr int kThreads = 256;

__device__ inline double warp_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// g[t] = G(t) / G(0) for t < rows (G summed over `region`, or over all regions if < 0),
// zero for rows <= t < L.
__global__ __launch_bounds__(kThreads) void k_fid_series(const double *rec, int64_t rows, int K,
                                                         int R, int region, int64_t L, double2 *g)
{
    double c = 0.0, d = 0.0;
    for (int r = 0; r < R; ++r) {
        if (region >= 0 && r != region)
            continue;
        c += rec[2 * r];
        d += rec[2 * r + 1];
    }
    const double den = c * c + d * d;
    for (int64_t t = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; t < L;
         t += static_cast<int64_t>(gridDim.x) * kThreads) {
        double2 out = {0.0, 0.0};
        if (t < rows) {
            double a = 0.0, b = 0.0;
            const double *row = rec + t * K;
            for (int r = 0; r < R; ++r) {
                if (region >= 0 && r != region)
                    continue;
                a += row[2 * r];
                b += row[2 * r + 1];
            }
            out.x = (a * c + b * d) / den;
            out.y = (b * c - a * d) / den;
        }
        g[t] = out;
    }
}

// One radix-2 Stockham pass: sub-transforms of length p are merged into length 2p.
__global__ __launch_bounds__(kThreads) void k_fft_pass(const double2 *__restrict__ x,
                                                       double2 *__restrict__ y, int64_t n,
                                                       int64_t p)
{
    const int64_t half = n / 2;
    for (int64_t j = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; j < half;
         j += static_cast<int64_t>(gridDim.x) * kThreads) {
        const int64_t k = j & (p - 1);
        double s, c;
        sincospi(-static_cast<double>(k) / static_cast<double>(p), &s, &c);
        const double2 a = x[j], b = x[j + half];
        const double2 bw = {b.x * c - b.y * s, b.x * s + b.y * c};
        y[2 * j - k] = {a.x + bw.x, a.y + bw.y};
        y[2 * j - k + p] = {a.x - bw.x, a.y - bw.y};
    }
}

// Ascending-frequency order: output j holds FFT bin (j + L/2) mod L; real parts in
// out[0, L), imaginary parts in out[L, 2L).
__global__ __launch_bounds__(kThreads) void k_spectrum_sorted(const double2 *X, int64_t L,
                                                              double *out)
{
    for (int64_t j = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; j < L;
         j += static_cast<int64_t>(gridDim.x) * kThreads) {
        const double2 v = X[(j + L / 2) & (L - 1)];
        out[j] = v.x;
        out[L + j] = v.y;
    }
}

// Largest value and its smallest index over v[0, n): per-workgroup candidates.
__global__ __launch_bounds__(kThreads) void k_argmax_partial(const double *v, int64_t n,
                                                             double *pval, int64_t *pidx)
{
    __shared__ double sv[kThreads];
    __shared__ int64_t si[kThreads];
    double best = -INFINITY;
    int64_t bi = -1;
    for (int64_t j = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; j < n;
         j += static_cast<int64_t>(gridDim.x) * kThreads) {
        if (v[j] > best) {
            best = v[j];
            bi = j;
        }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double ov = sv[threadIdx.x + s];
            const int64_t oi = si[threadIdx.x + s];
            if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi >= 0 &&
                                         (si[threadIdx.x] < 0 || oi < si[threadIdx.x]))) {
                sv[threadIdx.x] = ov;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pval[blockIdx.x] = sv[0];
        pidx[blockIdx.x] = si[0];
    }
}

__global__ void k_argmax_final(const double *pval, const int64_t *pidx, int nparts,
                               int64_t *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    double best = -INFINITY;
    int64_t bi = -1;
    for (int b = 0; b < nparts; ++b) {
        if (pidx[b] < 0)
            continue;
        if (pval[b] > best || (pval[b] == best && pidx[b] < bi)) {
            best = pval[b];
            bi = pidx[b];
        }
    }
    *out = bi;
}

// profile[c] = sum of rho over the plane at coordinate c along `axis`; one workgroup per
// plane, fixed summation order.
__global__ __launch_bounds__(kThreads) void k_profile(const double *rho, int nx, int ny, int nz,
                                                      int axis, double *profile)
{
    __shared__ double w[kThreads / 64];
    const int c = blockIdx.x;
    const int64_t n0 = axis == 0 ? ny : nx;           // first remaining axis (fastest)
    const int64_t n1 = axis == 2 ? ny : nz;           // second remaining axis
    const int64_t m = n0 * n1;
    double acc = 0.0;
    for (int64_t q = threadIdx.x; q < m; q += kThreads) {
        const int64_t u = q % n0, v = q / n0;
        int64_t x, y, z;
        if (axis == 0) {
            x = c; y = u; z = v;
        } else if (axis == 1) {
            x = u; y = c; z = v;
        } else {
            x = u; y = v; z = c;
        }
        acc += rho[x + static_cast<int64_t>(nx) * (y + static_cast<int64_t>(ny) * z)];
    }
    acc = warp_sum(acc);
    if (threadIdx.x % 64 == 0)
        w[threadIdx.x / 64] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kThreads / 64; ++k)
            t += w[k];
        profile[c] = t;
    }
}

// Largest |a_i - b_i| and largest b_i over [0, n): per-workgroup maxima, then one pass.
__global__ __launch_bounds__(kThreads) void k_change_partial(const double *a, const double *b,
                                                             int64_t n, double *part)
{
    __shared__ double sd[kThreads], sb[kThreads];
    double d = 0.0, m = 0.0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kThreads) {
        d = fmax(d, fabs(a[i] - b[i]));
        m = fmax(m, b[i]);
    }
    sd[threadIdx.x] = d;
    sb[threadIdx.x] = m;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + s]);
            sb[threadIdx.x] = fmax(sb[threadIdx.x], sb[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sd[0];
        part[2 * blockIdx.x + 1] = sb[0];
    }
}

__global__ __launch_bounds__(kThreads) void k_change_final(const double *part, int nparts,
                                                           double *out)
{
    __shared__ double sd[kThreads], sb[kThreads];
    double d = 0.0, m = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kThreads) {
        d = fmax(d, part[2 * b]);
        m = fmax(m, part[2 * b + 1]);
    }
    sd[threadIdx.x] = d;
    sb[threadIdx.x] = m;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + s]);
            sb[threadIdx.x] = fmax(sb[threadIdx.x], sb[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sd[0];
        out[1] = sb[0];
    }
}

// Per-region sums of rho, M1_a and M2_a (7 values per region: rho, M1 x y z, M2 x y z)
// over the state: workgroup partials in part[k * nparts + b], k = 7 r + q, for a
// fixed-order finalisation. Butterflies inside each wave, waves in index order.
template <typename S, int MAXR>
__global__ __launch_bounds__(kThreads) void k_region_sums(const double *rho, const S *m1x,
                                                          const S *m1y, const S *m1z,
                                                          const S *m2x, const S *m2y,
                                                          const S *m2z, const uint8_t *region,
                                                          int64_t n, int R, double *part)
{
    __shared__ double lds[(kThreads / 64) * 7 * MAXR];
    double acc[MAXR][7];
#pragma unroll
    for (int k = 0; k < MAXR; ++k)
#pragma unroll
        for (int q = 0; q < 7; ++q)
            acc[k][q] = 0.0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kThreads) {
        const int r = MAXR == 1 ? 0 : region[i];
        const double v[7] = {rho[i],
                             static_cast<double>(m1x[i]), static_cast<double>(m1y[i]),
                             static_cast<double>(m1z[i]), static_cast<double>(m2x[i]),
                             static_cast<double>(m2y[i]), static_cast<double>(m2z[i])};
#pragma unroll
        for (int k = 0; k < MAXR; ++k)
#pragma unroll
            for (int q = 0; q < 7; ++q)
                acc[k][q] += k == r ? v[q] : 0.0;
    }
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
    for (int k = 0; k < MAXR; ++k)
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            const double t = warp_sum(acc[k][q]);
            if (lane == 0)
                lds[wave * 7 * MAXR + 7 * k + q] = t;
        }
    __syncthreads();
    if (static_cast<int>(threadIdx.x) < 7 * R) {
        double t = 0.0;
        for (int w = 0; w < kThreads / 64; ++w)
            t += lds[w * 7 * MAXR + threadIdx.x];
        part[static_cast<int64_t>(threadIdx.x) * gridDim.x + blockIdx.x] = t;
    }
}

template <typename S>
hipError_t region_sums_typed(const StateView &st, const uint8_t *region, int64_t n, int32_t R,
                             double *part, int32_t nparts, hipStream_t s)
{
    const S *m1[3], *m2[3];
    for (int a = 0; a < 3; ++a) {
        m1[a] = static_cast<const S *>(st.m1[a]);
        m2[a] = static_cast<const S *>(st.m2[a]);
    }
    const dim3 grid(nparts), block(kThreads);
    if (R == 1)
        hipLaunchKernelGGL((k_region_sums<S, 1>), grid, block, 0, s, st.rho, m1[0], m1[1], m1[2],
                           m2[0], m2[1], m2[2], region, n, R, part);
    else if (R == 2)
        hipLaunchKernelGGL((k_region_sums<S, 2>), grid, block, 0, s, st.rho, m1[0], m1[1], m1[2],
                           m2[0], m2[1], m2[2], region, n, R, part);
    else if (R <= 4)
        hipLaunchKernelGGL((k_region_sums<S, 4>), grid, block, 0, s, st.rho, m1[0], m1[1], m1[2],
                           m2[0], m2[1], m2[2], region, n, R, part);
    else
        hipLaunchKernelGGL((k_region_sums<S, 8>), grid, block, 0, s, st.rho, m1[0], m1[1], m1[2],
                           m2[0], m2[1], m2[2], region, n, R, part);
    return hipGetLastError();
}

int grid_for(int64_t n)
{
    int64_t g = (n + kThreads - 1) / kThreads;
    return static_cast<int>(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

// The mixed full sweep's memory pattern without its arithmetic: 64 x 4 blocks of columns
// marching runs of z-planes, each thread reading its column's population (double), 10
// floats and the region byte one plane ahead and writing the population and 8 floats past
// the caches, one barrier per plane. 89 bytes per site, as the sweep's algorithmic count.
__global__ __launch_bounds__(kThreads, 2) void k_stream_columns_mixed(MixedColumns c, int nx,
                                                                      int ny, int nz, int zc,
                                                                      int tiles_x, int tiles_y)
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
    struct Site {
        double rho;
        float v[kMixedIn];
        uint8_t r;
    } w[2];
    auto load = [&](Site &d, int z) {
        const bool on = act && z < z1;
        const int64_t i = plane * z + col;
        d.rho = on ? c.rho_in[i] : 0.0;
#pragma unroll
        for (int k = 0; k < kMixedIn; ++k)
            d.v[k] = on ? c.in[k][i] : 0.0f;
        d.r = on ? c.region[i] : uint8_t(0);
    };
    auto store = [&](const Site &d, int z) {
        if (!(act && z < z1))
            return;
        const int64_t i = plane * z + col;
        const float e = d.v[kMixedOut] + d.v[kMixedOut + 1] * static_cast<float>(d.r);
        __builtin_nontemporal_store(d.rho + e, c.rho_out + i);
#pragma unroll
        for (int k = 0; k < kMixedOut; ++k)
            __builtin_nontemporal_store(d.v[k] + e, c.out[k] + i);
    };
    load(w[0], z0);
    for (int z = z0; z < z1; z += 2) {
        load(w[1], z + 1);
        __syncthreads();
        store(w[0], z);
        load(w[0], z + 2);
        __syncthreads();
        store(w[1], z + 1);
    }
}

}  // namespace

hipError_t launch_fid_spectrum(const double *records, int64_t rows, int32_t K, int32_t R,
                               int32_t region, int64_t L, double2 *buf_a, double2 *buf_b,
                               double *sorted_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_fid_series, dim3(grid_for(L)), dim3(kThreads), 0, s, records, rows, K, R,
                       region, L, buf_a);
    double2 *x = buf_a, *y = buf_b;
    for (int64_t p = 1; p < L; p *= 2) {
        hipLaunchKernelGGL(k_fft_pass, dim3(grid_for(L / 2)), dim3(kThreads), 0, s, x, y, L, p);
        double2 *t = x;
        x = y;
        y = t;
    }
    // x holds the transform; the other buffer receives the sorted real / imaginary parts
    double *out = sorted_out ? sorted_out : reinterpret_cast<double *>(y);
    hipLaunchKernelGGL(k_spectrum_sorted, dim3(grid_for(L)), dim3(kThreads), 0, s, x, L, out);
    return hipGetLastError();
}

hipError_t launch_argmax(const double *v, int64_t n, double *pval, int64_t *pidx, int32_t nparts,
                         int64_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_argmax_partial, dim3(nparts), dim3(kThreads), 0, s, v, n, pval, pidx);
    hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(64), 0, s, pval, pidx, nparts, out);
    return hipGetLastError();
}

hipError_t launch_max_change(const double *prev, const double *next, int64_t n, double *part,
                             int32_t nparts, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_change_partial, dim3(nparts), dim3(kThreads), 0, s, prev, next, n, part);
    hipLaunchKernelGGL(k_change_final, dim3(1), dim3(kThreads), 0, s, part, nparts, out);
    return hipGetLastError();
}

hipError_t launch_region_sums(int32_t precision, const StateView &st, const uint8_t *region,
                              int64_t n, int32_t R, double *part, int32_t nparts, hipStream_t s)
{
    return precision == 0 ? region_sums_typed<double>(st, region, n, R, part, nparts, s)
                          : region_sums_typed<float>(st, region, n, R, part, nparts, s);
}

hipError_t launch_stream_columns_mixed(const MixedColumns &c, int32_t nx, int32_t ny, int32_t nz,
                                       int32_t zc, hipStream_t s)
{
    const int tiles_x = (nx + 63) / 64, tiles_y = (ny + 3) / 4;
    const int64_t blocks = int64_t(tiles_x) * tiles_y * ((nz + zc - 1) / zc);
    hipLaunchKernelGGL(k_stream_columns_mixed, dim3(static_cast<unsigned>(blocks)), dim3(kThreads),
                       0, s, c, nx, ny, nz, zc, tiles_x, tiles_y);
    return hipGetLastError();
}

hipError_t launch_profile(const double *rho, const Geometry &g, int32_t axis, double *profile,
                          hipStream_t s)
{
    const int n = axis == 0 ? g.nx : (axis == 1 ? g.ny : g.nz);
    hipLaunchKernelGGL(k_profile, dim3(n), dim3(kThreads), 0, s, rho, g.nx, g.ny, g.nz, axis,
                       profile);
    return hipGetLastError();
}

}  // namespace lpc
