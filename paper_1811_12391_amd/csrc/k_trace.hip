// Uncollided fluence by Siddon ray tracing, per-class cross-section tables,
// and the dose tally.
//
// Uncollided fluence (first-collision paragraph of Sec. II-A; "calculated
// analytically" in Sec. IV): phi_u,g(v) = w_g exp(-tau_g(v)) / (4 pi r^2)
// with tau_g the optical depth along the straight segment from the source to
// the centre of voxel v, zero outside the fan x cone window.  One thread per
// (source, target voxel); neighbouring threads trace neighbouring rays, so the
// density/material gathers of a wavefront hit the same cache lines.  The
// optical depth is accumulated in FP64 as path length x density per material
// (at most DCT_MAXMAT materials, kept in registers) and contracted with the
// mass attenuation table at the end.
#include <algorithm>

#include "dct_internal.h"

namespace dct {

// Siddon march from p along d (target = p + d, inside the grid): calls
// f(voxel, length) for every segment between consecutive plane crossings,
// the voxel being the one holding the segment midpoint.
template <class F>
__device__ inline void siddon_march(const Geo &g, const double *p, const double *d, double r, F f)
{
    const double del[3] = {g.dx, g.dy, g.dz};
    const int nn[3] = {g.nx, g.ny, g.nz};
    // entry into the grid box (slab method); the target is inside the box
    double a_in = 0.0;
    for (int t = 0; t < 3; ++t) {
        if (d[t] == 0.0) continue;
        double t0 = (g.org[t] - p[t]) / d[t];
        double t1 = (g.org[t] + nn[t] * del[t] - p[t]) / d[t];
        double tmin = t0 < t1 ? t0 : t1;
        if (tmin > a_in) a_in = tmin;
    }
    // first plane crossing strictly after the entry, per axis
    double anext[3];
    int mpl[3], stp[3];
    for (int t = 0; t < 3; ++t) {
        if (d[t] == 0.0) {
            anext[t] = 2.0;
            mpl[t] = 0;
            stp[t] = 0;
            continue;
        }
        stp[t] = d[t] > 0 ? 1 : -1;
        double u = (p[t] + a_in * d[t] - g.org[t]) / del[t];
        int m = d[t] > 0 ? (int)floor(u) + 1 : (int)ceil(u) - 1;
        double tt = (g.org[t] + m * del[t] - p[t]) / d[t];
        for (int guard = 0; guard < 4 && tt <= a_in; ++guard) {
            m += stp[t];
            tt = (g.org[t] + m * del[t] - p[t]) / d[t];
        }
        for (int guard = 0; guard < 4; ++guard) {
            double tb = (g.org[t] + (m - stp[t]) * del[t] - p[t]) / d[t];
            if (tb > a_in) {
                m -= stp[t];
                tt = tb;
            } else {
                break;
            }
        }
        mpl[t] = m;
        anext[t] = tt;
    }
    double a0 = a_in;
    const int cap = g.nx + g.ny + g.nz + 4;
    for (int it = 0; it < cap; ++it) {
        double a1 = fmin(anext[0], fmin(anext[1], anext[2]));
        bool last = a1 >= 1.0;
        if (last) a1 = 1.0;
        double len = (a1 - a0) * r;
        double mid = 0.5 * (a0 + a1);
        int idx[3];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            int c = (int)floor((p[t] + mid * d[t] - g.org[t]) / del[t]);
            idx[t] = c < 0 ? 0 : (c > nn[t] - 1 ? nn[t] - 1 : c);
        }
        f(idx[0] + (long)g.nx * (idx[1] + (long)g.ny * idx[2]), len);
        if (last) break;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            if (anext[t] == a1) {
                mpl[t] += stp[t];
                anext[t] = (g.org[t] + mpl[t] * del[t] - p[t]) / d[t];
            }
        }
        a0 = a1;
    }
}

// beam window: azimuth about z from the projected axis, elevation from z = 0
__device__ inline bool in_window(const double *d, const double *axis, double half_fan, double half_cone)
{
    double ax = axis[0], ay = axis[1];
    double an = hypot(ax, ay);
    ax /= an;
    ay /= an;
    double along = d[0] * ax + d[1] * ay;
    double across = -d[0] * ay + d[1] * ax;
    double az = atan2(across, along);
    double el = atan2(d[2], hypot(d[0], d[1]));
    return fabs(az) <= half_fan && fabs(el) <= half_cone;
}

__global__ __launch_bounds__(256) void k_trace(TraceArgs a)
{
    const Geo &g = a.geo;
    long v = (long)blockIdx.x * 256 + threadIdx.x;
    int b = blockIdx.y;
    if (v >= g.C) return;
    int i = (int)(v % g.nx);
    int j = (int)((v / g.nx) % g.ny);
    int k = (int)(v / ((long)g.nx * g.ny));
    const double *p = a.pos + 3 * b;
    double d[3];
    d[0] = g.org[0] + (i + 0.5) * g.dx - p[0];
    d[1] = g.org[1] + (j + 0.5) * g.dy - p[1];
    d[2] = g.org[2] + (k + 0.5) * g.dz - p[2];
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double r = sqrt(r2);
    double *out = a.phi_u + (long)b * a.G * g.C + v;
    if (!in_window(d, a.axis + 3 * b, a.half_fan, a.half_cone)) {
        for (int gg = 0; gg < a.G; ++gg) out[(long)gg * g.C] = 0.0;
        return;
    }
    double acc[DCT_MAXMAT];
#pragma unroll
    for (int mm = 0; mm < DCT_MAXMAT; ++mm) acc[mm] = 0.0;
    siddon_march(g, p, d, r, [&](long u, double len) {
        int m = a.mat[u];
        double lr = len * a.rho[u];
#pragma unroll
        for (int mm = 0; mm < DCT_MAXMAT; ++mm) acc[mm] += (m == mm) ? lr : 0.0;
    });
    double inv = 1.0 / (4.0 * DCT_PI * r2);
    for (int gg = 0; gg < a.G; ++gg) {
        double tau = 0.0;
#pragma unroll
        for (int mm = 0; mm < DCT_MAXMAT; ++mm)
            if (mm < a.M) tau += a.st[mm * a.G + gg] * acc[mm];
        out[(long)gg * g.C] = a.gw[gg] * exp(-tau) * inv;
    }
}

// Adjoint of the uncollided flux: with weights pbu_g(v) on phi_u,g(v),
//   dR/dw_g      += pbu_g(v) exp(-tau_g(v)) / (4 pi r^2)
//   dR/drho_u    -= l_{v,u} sum_g sigma_t,g[m_u]/rho * pbu_g(v) phi_u,g(v)
// for every voxel u the ray to v crosses (FP64 atomics on the crossed voxels).
__global__ __launch_bounds__(256) void k_adj_ray(AdjRayArgs a)
{
    __shared__ double red[4];
    const Geo &g = a.geo;
    long v = (long)blockIdx.x * 256 + threadIdx.x;
    int b = blockIdx.y;
    bool live = v < g.C;
    double d[3] = {0, 0, 0}, r2 = 1.0, r = 1.0;
    const double *p = a.pos + 3 * b;
    if (live) {
        int i = (int)(v % g.nx);
        int j = (int)((v / g.nx) % g.ny);
        int k = (int)(v / ((long)g.nx * g.ny));
        d[0] = g.org[0] + (i + 0.5) * g.dx - p[0];
        d[1] = g.org[1] + (j + 0.5) * g.dy - p[1];
        d[2] = g.org[2] + (k + 0.5) * g.dz - p[2];
        r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        r = sqrt(r2);
        live = in_window(d, a.axis + 3 * b, a.half_fan, a.half_cone);
    }
    double acc[DCT_MAXMAT];
#pragma unroll
    for (int mm = 0; mm < DCT_MAXMAT; ++mm) acc[mm] = 0.0;
    if (live)
        siddon_march(g, p, d, r, [&](long u, double len) {
            int m = a.mat[u];
            double lr = len * a.rho[u];
#pragma unroll
            for (int mm = 0; mm < DCT_MAXMAT; ++mm) acc[mm] += (m == mm) ? lr : 0.0;
        });
    const double inv = 1.0 / (4.0 * DCT_PI * r2);
    double am[DCT_MAXMAT];
#pragma unroll
    for (int mm = 0; mm < DCT_MAXMAT; ++mm) am[mm] = 0.0;
    for (int gg = 0; gg < a.G; ++gg) {
        double unit = 0.0, wgt = 0.0;
        if (live) {
            double tau = 0.0;
#pragma unroll
            for (int mm = 0; mm < DCT_MAXMAT; ++mm)
                if (mm < a.M) tau += a.st[mm * a.G + gg] * acc[mm];
            unit = exp(-tau) * inv;
            wgt = a.pbu[((long)b * a.G + gg) * g.C + v];
#pragma unroll
            for (int mm = 0; mm < DCT_MAXMAT; ++mm)
                if (mm < a.M) am[mm] += a.st[mm * a.G + gg] * wgt * a.gw[gg] * unit;
        }
        // group-weight gradient: block reduction, one atomic per block and group
        double x = wgt * unit;
        for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(&a.dgw[gg], red[0] + red[1] + red[2] + red[3]);
    }
    if (live)
        siddon_march(g, p, d, r, [&](long u, double len) {
            int m = a.mat[u];
            double t = 0.0;
#pragma unroll
            for (int mm = 0; mm < DCT_MAXMAT; ++mm) t = (m == mm) ? am[mm] : t;
            if (t != 0.0) atomicAdd(&a.drho_ray[u], -len * t);
        });
}

// Direct weight of the ROI dose on the uncollided flux: pbu[b][g][v] = roi_v kappa_g[m_v].
__global__ __launch_bounds__(256) void k_adj_init(long C, int G, int B, const uint8_t *mat, const double *kap,
                                                  const double *roi, double *pbu)
{
    long v = (long)blockIdx.x * 256 + threadIdx.x;
    if (v >= C) return;
    const int m = mat[v];
    for (int b = 0; b < B; ++b)
        for (int g = 0; g < G; ++g) pbu[((long)b * G + g) * C + v] = roi[v] * kap[m * G + g];
}

hipError_t launch_adj_init(long C, int G, int B, const uint8_t *mat, const double *kap, const double *roi,
                           double *pbu, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_init, dim3((unsigned)((C + 255) / 256)), dim3(256), 0, s, C, G, B, mat, kap, roi, pbu);
    return hipGetLastError();
}

// Density gradient of the whole response: the ray back-projection's share
// plus every right-hand side's share, added in that order (the order the
// host-buffer form uses, so both give the same bits).
__global__ __launch_bounds__(256) void k_adj_gather(const double *drho, const double *dray, long C, int B,
                                                    double *out)
{
    const long v = (long)blockIdx.x * 256 + threadIdx.x;
    if (v >= C) return;
    double t = dray[v];
    for (int b = 0; b < B; ++b) t += drho[(long)b * C + v];
    out[v] = t;
}

hipError_t launch_adj_gather(const double *drho, const double *dray, long C, int B, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_gather, dim3((unsigned)((C + 255) / 256)), dim3(256), 0, s, drho, dray, C, B, out);
    return hipGetLastError();
}

// Screening of a caller's device array: the lowest index whose value is not
// finite (or, with nonneg, is negative) into *bad, which starts at all ones.
__global__ __launch_bounds__(256) void k_screen(const double *x, long n, int nonneg, unsigned long long *bad)
{
    for (long v = (long)blockIdx.x * 256 + threadIdx.x; v < n; v += (long)gridDim.x * 256) {
        const double t = x[v];
        if (!__builtin_isfinite(t) || (nonneg && t < 0.0)) atomicMin(bad, (unsigned long long)v);
    }
}

hipError_t launch_screen(const double *x, long n, int nonneg, unsigned long long *bad, hipStream_t s)
{
    const int nb = (int)std::min<long>(1024, std::max<long>(1, (n + 255) / 256));
    hipLaunchKernelGGL(k_screen, dim3(nb), dim3(256), 0, s, x, n, nonneg, bad);
    return hipGetLastError();
}

hipError_t launch_adj_ray(const AdjRayArgs &a, hipStream_t s)
{
    dim3 grid((unsigned)((a.geo.C + 255) / 256), a.B);
    hipLaunchKernelGGL(k_adj_ray, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_trace(const TraceArgs &a, hipStream_t s)
{
    dim3 grid((unsigned)((a.geo.C + 255) / 256), a.B);
    hipLaunchKernelGGL(k_trace, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// Total macroscopic cross section of every group in both sweep layouts:
// sigc[cls][g][pos_cls(v)] = rho_v * sigma_t[m_v][g].
template <typename T>
__global__ __launch_bounds__(256) void k_sigc(Geo g, const uint8_t *mat, const double *rho, const double *st,
                                              int G, T *sigc)
{
    long v = (long)blockIdx.x * 256 + threadIdx.x;
    int gg = blockIdx.y;
    if (v >= g.C) return;
    int i = (int)(v % g.nx);
    int j = (int)((v / g.nx) % g.ny);
    int k = (int)(v / ((long)g.nx * g.ny));
    T val = (T)(rho[v] * st[mat[v] * G + gg]);
    sigc[(long)gg * g.C + cls_pos(0, i, j, k, g.nx, g.ny)] = val;
    sigc[((long)G + gg) * g.C + cls_pos(1, i, j, k, g.nx, g.ny)] = val;
}

hipError_t launch_sigc(const Geo &g, const uint8_t *mat, const double *rho, const double *st, int G, int M,
                       void *sigc, int is_f64, hipStream_t s)
{
    (void)M;
    dim3 grid((unsigned)((g.C + 255) / 256), G);
    if (is_f64) hipLaunchKernelGGL(k_sigc<double>, grid, dim3(256), 0, s, g, mat, rho, st, G, (double *)sigc);
    else hipLaunchKernelGGL(k_sigc<float>, grid, dim3(256), 0, s, g, mat, rho, st, G, (float *)sigc);
    return hipGetLastError();
}

// sigma_t in the chain layout of period K nx: chain row `row` of layer k holds
// the cells of class-layout row row mod nx, so the table is K copies of each
// layer's class rows.
template <typename T>
__global__ __launch_bounds__(256) void k_sigch(Geo g, const T *sigc, int K, T *sigch)
{
    const long KC = (long)K * g.C;
    const long p = (long)blockIdx.x * 256 + threadIdx.x;
    const int cg = blockIdx.y;                           // class * G + group
    if (p >= KC) return;
    const long plane = (long)K * g.nx * g.ny;
    const int k = (int)(p / plane);
    const long rem = p - (long)k * plane;
    const int row = (int)(rem / g.ny), j = (int)(rem - (long)row * g.ny);
    sigch[(long)cg * KC + p] = sigc[(long)cg * g.C + ((long)k * g.nx + row % g.nx) * g.ny + j];
}

hipError_t launch_sigch(const Geo &g, const void *sigc, int G, int K, void *sigch, int is_f64, hipStream_t s)
{
    dim3 grid((unsigned)(((long)K * g.C + 255) / 256), 2 * G);
    if (is_f64) hipLaunchKernelGGL(k_sigch<double>, grid, dim3(256), 0, s, g, (const double *)sigc, K, (double *)sigch);
    else hipLaunchKernelGGL(k_sigch<float>, grid, dim3(256), 0, s, g, (const float *)sigc, K, (float *)sigch);
    return hipGetLastError();
}

// Dose tally (Sec. II-A: collision kerma as absorbed dose; or, with per-group
// factors hg, a fluence-to-dose conversion such as effective dose, Sec. III-A,
// with the dose of flagged materials such as air neglected):
// dose_b(v) = sum_g kappa_g[m_v] (phi_u,g(v) + phi_00,g(v)), summed in group order;
// phi_u of a right-hand side is the sum of its S superposed sources' fluxes.
template <typename T>
__global__ __launch_bounds__(256) void k_dose(DoseArgs a)
{
    long v = (long)blockIdx.x * 256 + threadIdx.x;
    if (v >= a.C) return;
    const T *pa = (const T *)a.phi_all;
    int m = a.mat[v];
    const bool zero = a.zero_mat && a.zero_mat[m];
    double tot = 0.0;
    for (int b = 0; b < a.B; ++b) {
        double dsum = 0.0;
        for (int g = 0; g < a.G; ++g) {
            double pu = 0.0;
            for (int k = 0; k < a.S; ++k) pu += a.phi_u[(((long)b * a.S + k) * a.G + g) * a.C + v];
            double pc = (double)pa[(((long)b * a.G + g) * a.Nm) * a.C + v];
            dsum += (a.hg ? a.hg[g] : a.kap[m * a.G + g]) * (pu + pc);
            if (a.phi_c) a.phi_c[((long)b * a.G + g) * a.C + v] = pc;
            if (a.phi_u_out) a.phi_u_out[((long)b * a.G + g) * a.C + v] = pu;
        }
        if (zero) dsum = 0.0;
        if (a.summed) tot += dsum;
        else a.dose[(long)b * a.C + v] = dsum;
    }
    if (a.summed) a.dose[v] = tot;
}

hipError_t launch_dose(const DoseArgs &a, int is_f64, hipStream_t s)
{
    dim3 grid((unsigned)((a.C + 255) / 256));
    if (is_f64) hipLaunchKernelGGL(k_dose<double>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_dose<float>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// Weighted sum R = sum_v w[v] x[v] in FP64, in a fixed order: each of the
// (at most 1024) workgroups sums a grid-strided share and reduces it in the
// workgroup; k_wsum then adds the partial sums in workgroup order.
__global__ __launch_bounds__(256) void k_wdot(const double *w, const double *x, long n, double *part)
{
    __shared__ double red[4];
    double acc = 0.0;
    for (long v = (long)blockIdx.x * 256 + threadIdx.x; v < n; v += (long)gridDim.x * 256) acc += w[v] * x[v];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void k_wsum(double *part, int nb)
{
    __shared__ double red[4];
    double acc = 0.0;
    for (int q = threadIdx.x; q < nb; q += 256) acc += part[q];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[nb] = red[0] + red[1] + red[2] + red[3];
}

hipError_t launch_wdot(const double *w, const double *x, long n, double *part, hipStream_t s)
{
    const int nb = (int)std::min<long>(1024, std::max<long>(1, (n + 255) / 256));
    hipLaunchKernelGGL(k_wdot, dim3(nb), dim3(256), 0, s, w, x, n, part);
    hipLaunchKernelGGL(k_wsum, dim3(1), dim3(256), 0, s, part, nb);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_stage_consts(StageConsts c, double *dst_d, unsigned char *dst_b)
{
    const int t = threadIdx.x;
    if (t < c.nd) dst_d[t] = c.d[t];
    if (t < c.nb) dst_b[t] = c.b[t];
}

hipError_t launch_stage_consts(const StageConsts &c, double *dst_d, unsigned char *dst_b, hipStream_t s)
{
    if (c.nd < 0 || c.nd > 256 || c.nb < 0 || c.nb > DCT_MAXMAT) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stage_consts, dim3(1), dim3(256), 0, s, c, dst_d, dst_b);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_widen(const T *src, long n, double *dst)
{
    long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t < n) dst[t] = (double)src[t];
}

hipError_t launch_moments_out(const void *phi_all, long n, double *out, int is_f64, hipStream_t s)
{
    dim3 grid((unsigned)((n + 255) / 256));
    if (is_f64) hipLaunchKernelGGL(k_widen<double>, grid, dim3(256), 0, s, (const double *)phi_all, n, out);
    else hipLaunchKernelGGL(k_widen<float>, grid, dim3(256), 0, s, (const float *)phi_all, n, out);
    return hipGetLastError();
}

}  // namespace dct
