// Source assembly and the device-driven group / iteration machine.
//
// Each right-hand side b (one source position) carries its own state:
// current group g, iterations done, and flags.  One "iteration set" is the
// fixed launch sequence  transition -> M-map -> sweep -> D-map -> combine;
// the host enqueues sets without knowing where each RHS stands, and every
// kernel reads the RHS state to decide what to do.  This keeps the host out
// of the inner loop (it only polls one counter now and then), gives each RHS
// its own stopping point, and makes a set capturable in a HIP graph.
//
// transition: when the previous set finished group g-1 of b (pending = 1) it
//   closes the balance of group g-1 and builds the fixed source of group g:
//   first-collision source (Sec. II-A) + optional volumetric source + the
//   downscatter from every converged higher group (eq. 2, g' < g), in that
//   order, and starts the iteration from phi = 0.
// combine: merges the two class-layout halves of the direction->moment map
//   into phi (natural layout), measures the relative change of phi_00, builds
//   the next within-group source Q = ext + sigma_s^{gg} phi in both class
//   layouts, and (last block of b) applies the stopping rule.
#include "dct_internal.h"

namespace dct {

__device__ inline int l_of(int lm)
{
    int l = 0;
    while ((l + 1) * (l + 1) <= lm) ++l;
    return l;
}

template <typename T>
__device__ inline T *tptr(void *p) { return (T *)p; }
template <typename T>
__device__ inline const T *tptr(const void *p) { return (const T *)p; }

__device__ inline double block_sum(double v, double *red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
    return t;   // valid on thread 0
}

// max that keeps a NaN (fmax would drop it and hide a non-finite change)
__device__ inline double nan_max(double x, double y) { return (y > x || y != y) ? y : x; }

__device__ inline double block_max(double v, double *red)
{
    for (int o = 32; o > 0; o >>= 1) v = nan_max(v, __shfl_down(v, o, 64));
    int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t = nan_max(t, red[i]);
    return t;
}

// LT: the P_N order as a compile-time constant, so that the harmonics of a
// voxel's source direction stay in registers
template <typename T, int LT>
__global__ __launch_bounds__(256) void k_transition(TransArgs a)
{
    constexpr int NM = (LT + 1) * (LT + 1);
    __shared__ double red[8];
    const int b = a.b0 + (int)blockIdx.y;
    RhsState *st = a.state + b;
    if (!st->pending) return;
    const int g = st->g;
    const Geo &geo = a.geo;
    const long C = geo.C;
    const long v = (long)blockIdx.x * 256 + threadIdx.x;
    const bool inb = v < C;
    const int G = a.G, L = LT, Nm = NM;
    double Rp = 0.0, Pp = 0.0;
    T *phi_all = (T *)a.phi_all;
    if (inb) {
        const int m = a.mat[v];
        const double rho = a.rho[v];
        if (g > 0) {
            // removal of the finished group: (sigma_t - sigma_s0^{gg}) phi_00
            const int gp = g - 1;
            double s0 = rho * a.ss[(((long)m * (L + 1)) * G + gp) * G + gp];
            double sig = rho * a.st[m * G + gp];
            Rp = (sig - s0) * (double)phi_all[(((long)b * G + gp) * Nm) * C + v];
        }
        if (g < G) {
            const int i = (int)(v % geo.nx);
            const int j = (int)((v / geo.nx) % geo.ny);
            const int k = (int)(v / ((long)geo.nx * geo.ny));
            T *ext = (T *)a.ext + (long)b * Nm * C;   // the first source of the group (k_qinit lays it out for the sweep)
            // every moment accumulates in the same order as before: first-
            // collision terms g' = 0..g (per superposed source, each source's
            // sum added in turn), the volume source, then downscatter
            // g' = 0..g-1; each phi_u value is read once for all moments
            double e[NM];
#pragma unroll
            for (int lm = 0; lm < NM; ++lm) e[lm] = 0.0;
            // groups g' < band_lo[g] scatter into g in no material: they are
            // skipped; inside the band every term is added (a zero transfer
            // moment adds an exact zero), so the loads carry no branch
            const double *sm = a.ss + (long)m * (L + 1) * G * G;
            const int g0 = a.band_lo ? a.band_lo[g] : 0;
            for (int ks = 0; ks < a.S; ++ks) {
                // the uncollided flux of source ks is a delta in angle along
                // the direction from the source to the voxel centre
                const long src = (long)b * a.S + ks;
                const double *p = a.pos + 3 * src;
                double d0 = geo.org[0] + (i + 0.5) * geo.dx - p[0];
                double d1 = geo.org[1] + (j + 0.5) * geo.dy - p[1];
                double d2 = geo.org[2] + (k + 0.5) * geo.dz - p[2];
                double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                double Y[NM];
                real_sh_cart<double>(LT, d0 / r, d1 / r, d2 / r, Y);
                double es[NM];
#pragma unroll
                for (int lm = 0; lm < NM; ++lm) es[lm] = 0.0;
                for (int gp = g0; gp <= g; ++gp) {
                    const double pu = rho * a.phi_u[(src * G + gp) * C + v];
#pragma unroll
                    for (int lm = 0; lm < NM; ++lm) es[lm] += sm[((long)l_of(lm) * G + gp) * G + g] * pu * Y[lm];
                }
#pragma unroll
                for (int lm = 0; lm < NM; ++lm) e[lm] += es[lm];
            }
            if (a.ext_iso) e[0] += a.ext_iso[(long)g * C + v];
            for (int gp = g0; gp < g; ++gp) {
                const T *pa = phi_all + ((long)b * G + gp) * Nm * C + v;
                T f[NM];
#pragma unroll
                for (int lm = 0; lm < NM; ++lm) f[lm] = pa[(long)lm * C];
#pragma unroll
                for (int lm = 0; lm < NM; ++lm) e[lm] += rho * sm[((long)l_of(lm) * G + gp) * G + g] * (double)f[lm];
            }
#pragma unroll
            for (int lm = 0; lm < NM; ++lm) {
                T et = (T)e[lm];
                ext[(long)lm * C + v] = et;
                if (!a.warm) phi_all[(((long)b * G + g) * Nm + lm) * C + v] = (T)0;
                if (lm == 0 && a.aa_phik)
                    a.aa_phik[(long)b * C + v] = a.warm ? (double)phi_all[(((long)b * G + g) * Nm) * C + v] : 0.0;
                if (lm == 0) Pp = e[0];
            }
        }
    }
    double Rs = block_sum(Rp, red);
    double Ps = block_sum(Pp, red);
    // per-workgroup sums through device atomics (no contention: one slot
    // each); the last workgroup closes the finished group's balance and
    // opens the next one, summing in a fixed order
    __shared__ int last;
    if (threadIdx.x == 0) {
        unsigned long long *pb = (unsigned long long *)a.part_bal + ((long)b * gridDim.x + blockIdx.x) * 2;
        atomicExch(pb, (unsigned long long)__double_as_longlong(Rs));
        atomicExch(pb + 1, (unsigned long long)__double_as_longlong(Ps));
        last = last_block(a.cnt_sub + (long)b * a.nsub * 32, &st->cnt_trans, blockIdx.x, gridDim.x);
    }
    __syncthreads();
    if (!last) return;
    double r = 0.0, pr = 0.0, lk = 0.0, pin = 0.0;
    for (unsigned q = threadIdx.x; q < gridDim.x; q += blockDim.x) {
        const unsigned long long *pq = (const unsigned long long *)a.part_bal + ((long)b * gridDim.x + q) * 2;
        r += __longlong_as_double((long long)__hip_atomic_load(pq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        pr += __longlong_as_double((long long)__hip_atomic_load(pq + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    const double Ax = geo.dy * geo.dz, Ay = geo.dx * geo.dz, Az = geo.dx * geo.dy;
    for (int n = threadIdx.x; n < a.N; n += blockDim.x) {
        const double wx = a.w[n] * fabs(a.dirs[3 * n]) * Ax, wy = a.w[n] * fabs(a.dirs[3 * n + 1]) * Ay,
                     wz = a.w[n] * fabs(a.dirs[3 * n + 2]) * Az;
        if (g > 0) {
            // leakage of the finished group: boundary outflows of its final sweep
            double lx = 0, ly = 0, lz = 0;
            for (int q = 0; q < a.nblk; ++q) {
                const double *lp = a.leak_part + (((long)b * a.N + n) * a.nblk + q) * 3;
                lx += lp[0];
                ly += lp[1];
                lz += lp[2];
            }
            lk += wx * lx + wy * ly + wz * lz;
        }
        // boundary inflow production of the next group (isotropic inflow)
        pin += wx * geo.ny * geo.nz + wy * geo.nx * geo.nz + wz * geo.nx * geo.ny;
    }
    r = block_sum(r, red);
    pr = block_sum(pr, red);
    lk = block_sum(lk, red);
    pin = block_sum(pin, red);
    if (threadIdx.x == 0) {
        if (g > 0) {
            a.bal[((long)b * G + g - 1) * 3 + 1] = r * a.V;
            a.bal[((long)b * G + g - 1) * 3 + 2] = lk;
        }
        if (g < G) {
            const double fin = (a.inflow && a.inflow[g] != 0.0) ? a.inflow[g] * pin : 0.0;
            a.bal[((long)b * G + g) * 3 + 0] = pr * a.V + fin;
        }
        st->pending = 0;
        if (g >= G) {
            st->finished = 1;
            atomicSub(a.n_unfinished, 1);
        }
    }
}

// Adjoint machine transition (groups from G-1 down to 0).  When group gp has
// converged it adds that group's terms of dR/drho_v (cross-section term
// -sum_n lamc_n psi_n t_g and the source terms sum_lm lam_lm dQ_lm/drho) and
// moves the first-collision part of the adjoint onto the uncollided flux
// weights; then it builds the adjoint moment source of the next (higher)
// group: the dose seed plus what every lower group took from it by
// downscatter, and starts its iteration from lam = 0.
template <typename T, int LT>
__global__ __launch_bounds__(256) void k_adj_transition(AdjTransArgs a)
{
    constexpr int NM = (LT + 1) * (LT + 1);
    const int b = blockIdx.y;
    RhsState *st = a.state + b;
    if (!st->pending) return;
    const int gs = st->g;                          // position in the reversed group sequence
    const int G = a.G, L = LT, Nm = NM, N = a.N;
    const Geo &geo = a.geo;
    const long C = geo.C;
    const long v = (long)blockIdx.x * 256 + threadIdx.x;
    if (v < C) {
        const int m = a.mat[v];
        const double rho = a.rho[v];
        const int i = (int)(v % geo.nx);
        const int j = (int)((v / geo.nx) % geo.ny);
        const int k = (int)(v / ((long)geo.nx * geo.ny));
        const double *p = a.pos + 3 * b;
        double d0 = geo.org[0] + (i + 0.5) * geo.dx - p[0];
        double d1 = geo.org[1] + (j + 0.5) * geo.dy - p[1];
        double d2 = geo.org[2] + (k + 0.5) * geo.dz - p[2];
        double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        double Y[NM];
        real_sh_cart<double>(LT, d0 / r, d1 / r, d2 / r, Y);
        const T *phi_all = (const T *)a.phi_all;
        T *lam_all = (T *)a.lam_all;
        if (gs > 0) {
            const int gp = G - gs;                 // the group that just converged
            // cross-section term from the final sweeps of group gp
            const T *pk = (const T *)a.psi_keep + ((long)b * G + gp) * N * C;
            const T *lc = (const T *)a.lamc + (long)b * N * C;
            const long pos0 = cls_pos(0, i, j, k, geo.nx, geo.ny), pos1 = cls_pos(1, i, j, k, geo.nx, geo.ny);
            double sbar = 0.0;
            for (int n = 0; n < N; ++n) {
                const long pp = dir_class(a.dirs[3 * n], a.dirs[3 * n + 1]) == 0 ? pos0 : pos1;
                sbar -= (double)lc[(long)n * C + pp] * (double)pk[(long)n * C + pp];
            }
            double drv = a.st[m * G + gp] * sbar;
            const T *lamg = lam_all + ((long)b * G + gp) * Nm * C;
#pragma unroll
            for (int lm = 0; lm < NM; ++lm) {
                const int l = l_of(lm);
                const double *sl = a.ss + ((long)m * (L + 1) + l) * G * G;
                const double lv = (double)lamg[(long)lm * C + v];
                double dq = sl[gp * G + gp] * (double)phi_all[(((long)b * G + gp) * Nm + lm) * C + v];
                for (int g2 = 0; g2 < gp; ++g2) {
                    double s = sl[g2 * G + gp];
                    if (s != 0.0) dq += s * (double)phi_all[(((long)b * G + g2) * Nm + lm) * C + v];
                }
                for (int g2 = 0; g2 <= gp; ++g2) {
                    double s = sl[g2 * G + gp];
                    if (s != 0.0) {
                        const double pu = a.phi_u[((long)b * G + g2) * C + v];
                        dq += s * pu * Y[lm];
                        a.pbu[((long)b * G + g2) * C + v] += rho * s * Y[lm] * lv;
                    }
                }
                drv += lv * dq;
            }
            a.drho[(long)b * C + v] += drv;
        }
        if (gs < G) {
            const int g = G - 1 - gs;              // the group to set up
            T *pb = (T *)a.phibar + (long)b * Nm * C;
            // the first adjoint source of the group is phibar (k_qinit lays it out for the sweep)
#pragma unroll
            for (int lm = 0; lm < NM; ++lm) {
                const int l = l_of(lm);
                const double *sl = a.ss + ((long)m * (L + 1) + l) * G * G;
                double e = lm == 0 ? a.roi[v] * a.kap[m * G + g] : 0.0;
                for (int g2 = g + 1; g2 < G; ++g2) {
                    double s = sl[g * G + g2];
                    if (s != 0.0) e += rho * s * (double)lam_all[(((long)b * G + g2) * Nm + lm) * C + v];
                }
                const T et = (T)e;
                pb[(long)lm * C + v] = et;
                lam_all[(((long)b * G + g) * Nm + lm) * C + v] = (T)0;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (last_block(a.cnt_sub + (long)b * a.nsub * 32, &st->cnt_trans, blockIdx.x, gridDim.x)) {
            st->pending = 0;
            if (gs >= G) {
                st->finished = 1;
                atomicSub(a.n_unfinished, 1);
            }
        }
    }
}

#define DCT_BY_ORDER(KER, T, L, ...)                                                        \
    do {                                                                                     \
        switch (L) {                                                                         \
        case 0: hipLaunchKernelGGL((KER<T, 0>), __VA_ARGS__); break;                         \
        case 1: hipLaunchKernelGGL((KER<T, 1>), __VA_ARGS__); break;                         \
        case 2: hipLaunchKernelGGL((KER<T, 2>), __VA_ARGS__); break;                         \
        case 3: hipLaunchKernelGGL((KER<T, 3>), __VA_ARGS__); break;                         \
        case 4: hipLaunchKernelGGL((KER<T, 4>), __VA_ARGS__); break;                         \
        default: hipLaunchKernelGGL((KER<T, 5>), __VA_ARGS__); break;                        \
        }                                                                                    \
    } while (0)

hipError_t launch_adj_transition(const AdjTransArgs &a, int is_f64, hipStream_t s)
{
    if (a.L < 0 || a.L > DCT_MAXL) return hipErrorInvalidValue;
    dim3 grid((unsigned)((a.geo.C + 255) / 256), a.B);
    if (is_f64) DCT_BY_ORDER(k_adj_transition, double, a.L, grid, dim3(256), 0, s, a);
    else DCT_BY_ORDER(k_adj_transition, float, a.L, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_transition(const TransArgs &a, int is_f64, hipStream_t s)
{
    const int nb = a.nb > 0 ? a.nb : a.B;
    if (a.b0 < 0 || a.b0 + nb > a.B) return hipErrorInvalidValue;
    dim3 grid((unsigned)((a.geo.C + 255) / 256), nb);
    if (a.L < 0 || a.L > DCT_MAXL) return hipErrorInvalidValue;
    if (is_f64) DCT_BY_ORDER(k_transition, double, a.L, grid, dim3(256), 0, s, a);
    else DCT_BY_ORDER(k_transition, float, a.L, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// End of an iteration of right-hand side b (called by the one workgroup
// that completes it, after every workgroup's eps atomics): relative change
// of phi_00, the stopping rule, and the move to the next group.
__device__ inline void close_iteration(const CombArgs &a, RhsState *st, int b, int gseq, int g)
{
    const int G = a.G;
    wait_own_memory_ops();
    double num = __longlong_as_double((long long)atomicAdd(&st->eps_num, 0ull));
    double den = __longlong_as_double((long long)atomicAdd(&st->eps_den, 0ull));
    int it = st->it + 1;
    st->it = it;
    bool bad = !isfinite(num) || !isfinite(den);
    double e = den > 0.0 ? num / den : 0.0;
    bool stop;
    if (bad) {
        st->nan = 1;
        stop = true;
    } else if (a.fixed_iters) {
        stop = it >= a.fixed_iters[g];
    } else {
        bool conv = e <= a.tol;
        if (!conv && a.stall_window > 0) {
            // reduced precision: eps near tol that stops improving is
            // rounding noise (flipping set-to-zero decisions), not slow
            // convergence
            if (it == 1 || e < st->eps_best) {
                st->eps_best = e;
                st->stall = 0;
            } else if (e <= 10.0 * a.tol) {
                conv = ++st->stall >= a.stall_window;
            } else {
                st->stall = 0;
            }
        }
        stop = conv || (it >= a.max_iter);
        if (stop && !conv) st->notconv = 1;
    }
    if (stop) {
        a.iters[(long)b * G + g] = it;
        a.eps[(long)b * G + g] = e;
        st->g = bad ? G : gseq + 1;
        st->it = 0;
        st->pending = 1;
    }
    st->eps_num = 0ull;
    st->eps_den = 0ull;
    st->cnt_combine = 0;
}

// LDS tile of one slab (z layer k, 16 consecutive y rows, all x).
//
// E > 0: every thread holds E tile elements (16 nx <= 256 E) and issues all of
// its global loads (both class halves, the external source, the previous
// phi_00, material and density) before the first LDS phase, so the memory
// latency is paid once per workgroup.  E = 0: generic loop for wide grids.
template <typename T, int E>
__global__ __launch_bounds__(256) void k_combine(CombArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    T *tile = (T *)smem_raw;
    __shared__ double red[8];
    const int b = blockIdx.y;
    RhsState *st = a.state + b;
    if (st->finished) return;
    const int gseq = st->g;
    const int g = eff_group(gseq, a.G, a.reverse);
    const int nx = a.geo.nx, ny = a.geo.ny;
    const long C = a.geo.C;
    const int G = a.G, Nm = a.Nm, L = a.L;
    const int nslj = (ny + 15) >> 4;
    // moments lm_lo .. lm_hi - 1 of this workgroup, one after the other
    // (several per workgroup keep the slab's material and density in the
    // CU's caches for all of them)
    const int mg = blockIdx.z, nmg = gridDim.z;
    const int lm_lo = mg * a.mpw, lm_hi = min(Nm, lm_lo + a.mpw);
    const int nslab = a.geo.nz * nslj;
    const bool live = true;
    const int k = blockIdx.x / nslj;
    const int j0 = (blockIdx.x % nslj) * 16;
    // even pitch: row jl of the tile is read and written at i = r -+ jl, so
    // the bank of element (jl, r -+ jl) is (pitch -+ 1) jl + r, distinct over
    // the 16 rows when pitch -+ 1 are odd
    const int pitch = (nx | 1) + 1;
    const int tile_n = 16 * nx;
    T *phib = (T *)a.phi_all + ((long)b * G + g) * Nm * C;
    double dmax = 0.0, fmax_ = 0.0;
    // self-scatter moments of group g per material, for the next source
    __shared__ double ssg[DCT_MAXMAT * (DCT_MAXL + 1)];
    if (E > 0 && (int)threadIdx.x < a.M * (L + 1)) {
        const int mm = threadIdx.x / (L + 1), ll = threadIdx.x - mm * (L + 1);
        ssg[threadIdx.x] = a.ss[(((long)mm * (L + 1) + ll) * G + g) * G + g];
    }
    for (int lm = lm_lo; lm < lm_hi; ++lm) {
    const int l = l_of(lm);
    const T *partA = (const T *)a.part + ((long)b * Nm + lm) * C;
    const T *partB = (const T *)a.part + (((long)a.B + b) * Nm + lm) * C;
    T *QA = (T *)a.Qc + ((long)b * Nm + lm) * C;
    T *QB = (T *)a.Qc + (((long)a.B + b) * Nm + lm) * C;
    const T *ext = (const T *)a.ext + ((long)b * Nm + lm) * C;
    if (E > 0) {
        constexpr int EE = E > 0 ? E : 1;
        constexpr unsigned TS = sizeof(T);
        // every load is issued up front through descriptors; elements outside
        // the tile use an out-of-range offset (no branch, no memory access)
        const rsrc_t rA = mk_rsrc(partA, C * TS), rB = mk_rsrc(partB, C * TS);
        const rsrc_t rE = mk_rsrc(ext, C * TS), rP = mk_rsrc(phib, C * TS);
        const rsrc_t rM = mk_rsrc(a.mat, C), rR = mk_rsrc(a.rho, C * 8);
        const rsrc_t rPo = mk_rsrc(phib + (long)lm * C, C * TS);
        const rsrc_t rQA = mk_rsrc(QA, C * TS), rQB = mk_rsrc(QB, C * TS);
        T va[EE], vb[EE], ve[EE], vo[EE];
        double rh[EE];
        int mt[EE];
#pragma unroll
        for (int e = 0; e < EE; ++e) {
            const int idx = threadIdx.x + 256 * e;
            const int r = idx >> 4, jl = idx & 15, j = j0 + jl;
            const bool okr = idx < tile_n && j < ny;
            const unsigned orot = okr ? (unsigned)(((long)k * nx + r) * ny + j) * TS : DCT_OOB;
            va[e] = bld<T>(rA, orot);
            vb[e] = bld<T>(rB, orot);
            const int jn = idx / nx, in = idx - jn * nx, jj = j0 + jn;
            const bool okn = idx < tile_n && jj < ny;
            const unsigned v = okn ? (unsigned)(in + (long)nx * (jj + (long)ny * k)) : 0u;
            ve[e] = bld<T>(rE, okn ? v * TS : DCT_OOB);
            vo[e] = bld<T>(rP, (okn && lm == 0) ? v * TS : DCT_OOB);
            mt[e] = __builtin_amdgcn_raw_buffer_load_b8(rM, okn ? v : DCT_OOB, 0, 0);
            rh[e] = bld<double>(rR, okn ? v * 8 : DCT_OOB);
        }
#pragma unroll
        for (int e = 0; e < EE; ++e) {
            const int idx = threadIdx.x + 256 * e;
            const int r = idx >> 4, jl = idx & 15, j = j0 + jl;
            if (idx < tile_n && j < ny) tile[jl * pitch + rot_row(1, r, j % nx, nx)] = va[e];   // class A -> natural i
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EE; ++e) {
            const int idx = threadIdx.x + 256 * e;
            const int r = idx >> 4, jl = idx & 15, j = j0 + jl;
            if (idx < tile_n && j < ny) tile[jl * pitch + rot_row(0, r, j % nx, nx)] += vb[e];  // class B -> natural i
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EE; ++e) {
            const int idx = threadIdx.x + 256 * e;
            const int jn = idx / nx, in = idx - jn * nx, jj = j0 + jn;
            const bool okn = idx < tile_n && jj < ny;
            const unsigned v = okn ? (unsigned)(in + (long)nx * (jj + (long)ny * k)) : 0u;
            const int ti = okn ? jn * pitch + in : 0;
            const T pn = tile[ti];
            if (lm == 0 && okn) {
                const double dn = fabs((double)pn - (double)vo[e]);
                const double an = fabs((double)pn);
                dmax = (dn > dmax || dn != dn) ? dn : dmax;
                fmax_ = (an > fmax_ || an != an) ? an : fmax_;
            }
            bst(rPo, okn ? v * TS : DCT_OOB, pn);
            const double sc = rh[e] * ssg[mt[e] * (L + 1) + l];
            if (okn) tile[ti] = (T)((double)ve[e] + sc * (double)pn);
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EE; ++e) {
            const int idx = threadIdx.x + 256 * e;
            const int r = idx >> 4, jl = idx & 15, j = j0 + jl;
            const bool okr = idx < tile_n && j < ny;
            const int jm = okr ? j % nx : 0;
            const unsigned orot = okr ? (unsigned)(((long)k * nx + r) * ny + j) * TS : DCT_OOB;
            const int rr = okr ? r : 0, jr = okr ? jl : 0;
            bst(rQA, orot, tile[jr * pitch + rot_row(1, rr, jm, nx)]);
            bst(rQB, orot, tile[jr * pitch + rot_row(0, rr, jm, nx)]);
        }
        __syncthreads();
    } else {
        // class A half, rotated rows -> natural tile
        for (int idx = threadIdx.x; idx < tile_n; idx += 256) {
            int r = idx >> 4, jl = idx & 15, j = j0 + jl;
            if (j < ny) {
                int i = rot_row(1, r, j % nx, nx);          // inverse of (i + j) mod nx
                long p = ((long)k * nx + r) * ny + j;
                tile[jl * pitch + i] = partA[p];
            }
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < tile_n; idx += 256) {
            int r = idx >> 4, jl = idx & 15, j = j0 + jl;
            if (j < ny) {
                int i = rot_row(0, r, j % nx, nx);          // inverse of (i - j) mod nx
                long p = ((long)k * nx + r) * ny + j;
                tile[jl * pitch + i] += partB[p];
            }
        }
        __syncthreads();
        // natural order: new moments, change of phi_00, next within-group source
        for (int idx = threadIdx.x; idx < tile_n; idx += 256) {
            int jl = idx / nx, i = idx - jl * nx, j = j0 + jl;
            if (j < ny) {
                long v = i + (long)nx * (j + (long)ny * k);
                T pn = tile[jl * pitch + i];
                if (lm == 0) {
                    double old = (double)phib[v];
                    double dn = fabs((double)pn - old);
                    double an = fabs((double)pn);
                    dmax = (dn > dmax || dn != dn) ? dn : dmax;
                    fmax_ = (an > fmax_ || an != an) ? an : fmax_;
                }
                phib[(long)lm * C + v] = pn;
                int m = a.mat[v];
                double s = a.rho[v] * a.ss[(((long)m * (L + 1) + l) * G + g) * G + g];
                tile[jl * pitch + i] = (T)((double)ext[v] + s * (double)pn);
            }
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < tile_n; idx += 256) {
            int r = idx >> 4, jl = idx & 15, j = j0 + jl;
            if (j < ny) {
                int jm = j % nx;
                long p = ((long)k * nx + r) * ny + j;
                QA[p] = tile[jl * pitch + rot_row(1, r, jm, nx)];
                QB[p] = tile[jl * pitch + rot_row(0, r, jm, nx)];
            }
        }
        __syncthreads();
    }
    }   // moments of the workgroup
    double dm = 0.0, fm = 0.0;
    if (lm_lo == 0) {
        dm = block_max(dmax, red);
        fm = block_max(fmax_, red);
    }
    if (threadIdx.x == 0) {
        if (lm_lo == 0 && live) {
            atomicMax(&st->eps_num, (unsigned long long)__double_as_longlong(dm));
            atomicMax(&st->eps_den, (unsigned long long)__double_as_longlong(fm));
        }
        wait_own_memory_ops();
        // two-level completion count: the slabs of one moment on that
        // moment's counter (its own cache line), the last of them on the
        // right-hand side's counter, so no counter takes an atomic from every
        // workgroup; the last block of the last moment closes the iteration
        unsigned *cm = a.cnt_mom + ((long)b * Nm + mg) * 32;
        const unsigned prev1 = live ? atomicAdd(cm, 1u) : 0u;
        unsigned prev = 0u;
        if (live && prev1 == (unsigned)nslab - 1) {
            atomicExch(cm, 0u);
            wait_own_memory_ops();
            prev = atomicAdd(&st->cnt_combine, 1u) + 1u;
        }
        if (prev == (unsigned)nmg) close_iteration(a, st, b, gseq, g);
    }
}

// Fused direction->moment map, combine and moment->direction map of one
// source iteration (eq. 2 with the Legendre-expanded scattering kernel as
// M Sigma D; eq. 3 is row 0 of D).  The work item is a slab (z layer k, 16 y
// rows, all x) of one right-hand side; persistent workgroups (as many as the
// device holds at once) take the items in turn, loading the map tables once.
// A slab is closed under both class rotations, so everything between reading
// psi and writing the next q stays in LDS:
//   1. the D map of each class on the matrix cores, its moments scattered
//      into a natural-layout tile (class A stores, class B adds);
//   2. combine: the new moments phi (stored), the change of phi_00 and the
//      next within-group source Q = ext + sigma_s^{gg} phi, into the tile;
//   3. the M map of each class from the tile; q stored for the next sweep.
// The class partials and Q never reach HBM.  Each step does the arithmetic
// of k_dmap, k_combine and k_mmap in the same order, so the results are the
// same bit for bit.  The last slab of the right-hand side to finish applies
// the stopping rule; when the group stops, the q written here is replaced
// after the transition by the FIRST form of the kernel, which for the sources
// starting a group lays Q = ext (plus a warm start's self-scatter) into the
// tile and runs only step 3.
template <typename T, int NRB, int KC, bool FIRST>
__global__ __launch_bounds__(512) void k_dcm(CombArgs a, MapArgs m)
{
    constexpr bool first = FIRST;
    // issue priority above the sweep's waves: with the sources on two streams
    // this memory-bound kernel shares CUs with the other half's latency-bound
    // sweep, and issuing its loads first measured 116.0 against 116.8 ms on
    // the 36-source scan (one stream: unchanged)
    __builtin_amdgcn_s_setprio(1);
    typedef typename acc4<T>::type A4;                        // KC: K-steps of 4 directions, covering a class
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    __shared__ double red[16];
    __shared__ double ssg[DCT_MAXMAT * (DCT_MAXL + 1)];
    const int nx = a.geo.nx, ny = a.geo.ny;
    const int nslj = (ny + 15) >> 4;
    const unsigned nsl = (unsigned)(a.geo.nz * nslj);          // slabs of one right-hand side
    const unsigned NW = nsl * (unsigned)(a.nb > 0 ? a.nb : a.B);   // items of this launch's right-hand sides
    const long C = a.geo.C;
    const int G = a.G, Nm = a.Nm, L = a.L, N = m.N;
    const int pitch = (nx | 1) + 1;
    // moment stride of the tile: 16 rows plus 4 words, so that the 4 lane
    // groups of an MFMA output (moments 4 apart) fall in different banks
    const int LMS = 16 * pitch + 4;
    const int NcP = m.NcP, NmP = m.NmP, DST = NcP + 1, MST = NmP + 1;
    T *tile = (T *)smem_raw;                                  // [Nm][LMS]: 16 rows of pitch, natural x
    T *Dt = tile + (long)Nm * LMS;                            // [2][NmP][NcP + 1]
    T *Mt = Dt + 2 * NmP * DST;                               // [2][NcP][NmP + 1]
    int *cds = (int *)(Mt + 2 * NcP * MST);                   // [2][N] class-local -> global direction
    unsigned *cdo = (unsigned *)(cds + 2 * N);                // [2][N] its byte offset n C sizeof(T)
    for (int i = threadIdx.x; i < 2 * NmP * NcP; i += blockDim.x) {
        const int c = i / (NmP * NcP), r = (i / NcP) % NmP, q = i % NcP;
        Dt[(c * NmP + r) * DST + q] = ((const T *)m.Dtab)[i];
    }
    for (int i = threadIdx.x; i < 2 * NcP * NmP; i += blockDim.x) {
        const int c = i / (NcP * NmP), r = (i / NmP) % NcP, q = i % NmP;
        Mt[(c * NcP + r) * MST + q] = ((const T *)m.Mtab)[i];
    }
    for (int i = threadIdx.x; i < 2 * N; i += blockDim.x) {
        cds[i] = m.cdir[i];
        cdo[i] = (unsigned)((long)m.cdir[i] * C * (long)sizeof(T));
    }
    // in the class layouts an element's offset is (direction part) + (cell
    // part), both 32-bit (the host keeps N C sizeof(T) < 2^31); the chain
    // layout goes through dir_elem
    const bool fast = m.chainK <= 1;
    const int Nc0 = m.Nc[0], Nc1 = m.Nc[1];
    // persistent workgroups (the tables above are loaded once): workgroup h
    // takes work items h, h + gridDim.x, ...; item -> (right-hand side, slab).
    // Two slabs 16 rows apart share the 128-byte lines of psi (64 bytes each
    // per row and direction in FP32), so they are paired on one XCD: the items
    // of workgroups h and h + 8 in the same round (same XCD, running together)
    // are slabs j and j + 1 of the same layer
    const bool pair = (nslj & 1) == 0 && (NW & 15) == 0 && (gridDim.x & 15) == 0;
    for (unsigned lin = blockIdx.x; lin < NW; lin += gridDim.x) {
        // the lane indices pass through an opaque zero, so that the per-lane
        // address arithmetic of the item is formed inside the loop instead of
        // being hoisted out of it and held in registers across items
        int lz;
        asm volatile("v_mov_b32 %0, 0" : "=v"(lz));
        const int tid = (int)threadIdx.x + lz;
        const int l = tid & 63, col = l & 15, kr = l >> 4;
        const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), nwv = blockDim.x >> 6;
        unsigned W = lin;
        if (pair) {
            const unsigned xcd = lin & 7, slot = lin >> 3;
            W = 2 * ((slot >> 1) * 8 + xcd) + (slot & 1);
        }
        const int bl = __builtin_amdgcn_readfirstlane((int)(W / nsl));
        const int slab = __builtin_amdgcn_readfirstlane((int)(W - (unsigned)bl * nsl));
        const int b = a.b0 + bl;
        RhsState *st = a.state + b;
        if (st->finished) continue;
        // first iteration of a group: only the sources that start one
        if (first && (st->pending || st->it != 0)) continue;
        const int gseq = __builtin_amdgcn_readfirstlane(st->g);   // wave-uniform: the buffer descriptors below stay scalar
        const int g = __builtin_amdgcn_readfirstlane(eff_group(gseq, a.G, a.reverse));
        const int k = slab / nslj, j0 = (slab % nslj) * 16;
        if ((int)threadIdx.x < a.M * (L + 1)) {
            const int mm = threadIdx.x / (L + 1), ll = threadIdx.x - mm * (L + 1);
            ssg[threadIdx.x] = a.ss[(((long)mm * (L + 1) + ll) * G + g) * G + g];
        }
        __syncthreads();
        const int jj = j0 + col;                                  // y row of this lane's column
        const bool jok = jj < ny;
        const int jc = jok ? jj : ny - 1;
        const int jm = jc % nx;
        // ---- 1. D map of each class into the natural tile.  A wave takes two
        // rows at a time and loads the psi operands of its next pair (the first
        // pair of class B after the last of class A) before the matrix-core work
        // of the current one, so two pairs of loads are in flight.
        const T *psi = (const T *)m.psi + ((long)b * m.psi_bs + (long)g * m.psi_gs) * C;
        const rsrc_t rps = mk_rsrc(wave_ptr(psi), (long)N * C * (long)sizeof(T));
        T bA[2][KC], bB[2][KC];
        auto load_pair = [&](int c, int r0, T (&bv)[2][KC]) __attribute__((always_inline)) {
            const int Nc = c == 0 ? Nc0 : Nc1;
            if (fast) {
                const unsigned *co = cdo + c * N;
                unsigned o[KC];
    #pragma unroll
                for (int u = 0; u < KC; ++u) o[u] = co[min(4 * u + kr, Nc - 1)];
    #pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int r = min(r0 + h * nwv, nx - 1);
                    const unsigned p4 = (unsigned)((((long)k * nx + r) * ny + jc) * (long)sizeof(T));
    #pragma unroll
                    for (int u = 0; u < KC; ++u) bv[h][u] = bld<T>(rps, o[u] + p4);
                }
                return;
            }
            const int *cd = cds + c * N;
    #pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int r = min(r0 + h * nwv, nx - 1);
                const long p = ((long)k * nx + r) * ny + jc;
                const CellKJI cc{k, jc, c == 0 ? (r - jm + nx) % nx : (r + jm) % nx};
    #pragma unroll
                for (int u = 0; u < KC; ++u) bv[h][u] = psi[dir_elem(m, c, cd[min(4 * u + kr, Nc - 1)], p, cc)];
            }
        };
        bool have = false;                                        // bA holds the operands of the pair at hand
        for (int c = 0; c < (first ? 0 : 2); ++c) {
            const int Nc = c == 0 ? Nc0 : Nc1;
            if (!have && wv < nx) {
                load_pair(c, wv, bA);
                have = true;
            }
            for (int r0 = wv; r0 < nx; r0 += 2 * nwv) {
                // operands of the next pair: this class's, or class B's first
                int rn = r0 + 2 * nwv, cn = c;
                if (rn >= nx && c == 0) {
                    rn = wv;
                    cn = 1;
                }
                const bool next = rn < nx;
                if (next) load_pair(cn, rn, bB);
                A4 acc[2][NRB];
    #pragma unroll
                for (int h = 0; h < 2; ++h)
    #pragma unroll
                    for (int rb = 0; rb < NRB; ++rb) acc[h][rb] = A4{0, 0, 0, 0};
    #pragma unroll
                for (int u = 0; u < KC; ++u)
                    if (4 * u < Nc) {
    #pragma unroll
                        for (int rb = 0; rb < NRB; ++rb) {
                            const T av = Dt[(c * NmP + rb * 16 + col) * DST + 4 * u + kr];
    #pragma unroll
                            for (int h = 0; h < 2; ++h) acc[h][rb] = mfma_k4(av, bA[h][u], acc[h][rb]);
                        }
                    }
    #pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int r = r0 + h * nwv;
                    if (jok && r < nx) {
                        const int i = c == 0 ? (r - jm + nx) % nx : (r + jm) % nx;   // natural x of (r, j)
    #pragma unroll
                        for (int rb = 0; rb < NRB; ++rb)
    #pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const int lm = rb * 16 + out_row<T>(kr, e);
                                if (lm < Nm) {
                                    T *tp = &tile[lm * LMS + col * pitch + i];
                                    *tp = c == 0 ? acc[h][rb][e] : *tp + acc[h][rb][e];
                                }
                            }
                    }
                }
                have = next;
    #pragma unroll
                for (int h = 0; h < 2; ++h)
    #pragma unroll
                    for (int u = 0; u < KC; ++u) bA[h][u] = bB[h][u];
            }
            __syncthreads();
        }
        // ---- 2. combine in natural order: a thread takes one voxel of the slab at
        // a time (material, density and the old phi_00 read once) and all its
        // moments, with the group source of every moment requested up front
        double dmax = 0.0, fmax_ = 0.0;
        T *phib = (T *)a.phi_all + ((long)b * G + g) * Nm * C;
        const T *ext = (const T *)a.ext + (long)b * Nm * C;
        const int tile_n = 16 * nx;
        // ext and phi of this source and group through buffer descriptors: the
        // voxel's byte offset per lane, the moment's (lm C sizeof(T), below 2^31
        // by a host check) as a scalar
        const rsrc_t rex = mk_rsrc(wave_ptr(ext), (long)Nm * C * (long)sizeof(T));
        const rsrc_t rph = mk_rsrc(wave_ptr(phib), (long)Nm * C * (long)sizeof(T));
        const unsigned cst = (unsigned)(C * (long)sizeof(T));
        // first iteration: the source is the group source ext (plus the
        // within-group scatter of the moments a warm start begins from), laid
        // into the tile as k_qinit lays it out
        for (int idx = threadIdx.x; first && idx < tile_n; idx += blockDim.x) {
            const int jl = idx / nx, i = idx - jl * nx, jy = j0 + jl;
            if (jy >= ny) continue;
            const int v = i + nx * (jy + ny * k);
            const unsigned v4 = (unsigned)v * (unsigned)sizeof(T);
            const double rh = a.rho[v];
            const int mt = a.mat[v];
            // every moment's loads issued before the first is used
            T ev[16 * NRB], pv[16 * NRB];
#pragma unroll
            for (int lm = 0; lm < 16 * NRB; ++lm) {
                ev[lm] = bld_s<T>(rex, v4, min(lm, Nm - 1) * cst);
                pv[lm] = a.warm ? bld_s<T>(rph, v4, min(lm, Nm - 1) * cst) : (T)0;
            }
#pragma unroll
            for (int lm = 0; lm < 16 * NRB; ++lm) {
                if (lm >= Nm) continue;
                T *tp = &tile[lm * LMS + jl * pitch + i];
                if (a.warm) {
                    const double sc = rh * ssg[mt * (L + 1) + l_of(lm)];
                    *tp = (T)((double)ev[lm] + sc * (double)pv[lm]);
                } else {
                    *tp = ev[lm];
                }
            }
        }
        for (int idx = threadIdx.x; !first && idx < tile_n; idx += blockDim.x) {
            const int jl = idx / nx, i = idx - jl * nx, jy = j0 + jl;
            if (jy >= ny) continue;
            const int v = i + nx * (jy + ny * k);
            const unsigned v4 = (unsigned)v * (unsigned)sizeof(T);
            const double rh = a.rho[v];
            const int mt = a.mat[v];
            const T po = bld_s<T>(rph, v4, 0);
            T ev[16 * NRB];
    #pragma unroll
            for (int lm = 0; lm < 16 * NRB; ++lm) ev[lm] = bld_s<T>(rex, v4, min(lm, Nm - 1) * cst);
    #pragma unroll
            for (int lm = 0; lm < 16 * NRB; ++lm) {
                if (lm >= Nm) continue;
                T *tp = &tile[lm * LMS + jl * pitch + i];
                const T pn = *tp;
                if (lm == 0) {
                    const double dn = fabs((double)pn - (double)po);
                    const double an = fabs((double)pn);
                    dmax = (dn > dmax || dn != dn) ? dn : dmax;
                    fmax_ = (an > fmax_ || an != an) ? an : fmax_;
                }
                bst_s(rph, v4, lm * cst, pn);
                const double sc = rh * ssg[mt * (L + 1) + l_of(lm)];
                *tp = (T)((double)ev[lm] + sc * (double)pn);
            }
        }
        __syncthreads();
        // ---- 3. M map of each class from the tile
        T *q = (T *)m.q + (long)b * N * C;
        const int NS = (Nm + 3) / 4;                              // K-steps of 4 moments
        if (fast) {
            // q stored through a buffer descriptor: every lane stores, rows past
            // the class's directions or the grid take an out-of-range offset
            const rsrc_t rqq = mk_rsrc(wave_ptr(q), (long)N * C * (long)sizeof(T));
            for (int c = 0; c < 2; ++c) {
                const int Nc = c == 0 ? Nc0 : Nc1;
                const unsigned *co = cdo + c * N;
                unsigned qo[3][4];                                // up to 48 directions per class (host check)
    #pragma unroll
                for (int rb = 0; rb < 3; ++rb)
    #pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int nl = rb * 16 + out_row<T>(kr, e);
                        qo[rb][e] = (nl < Nc && jok) ? co[nl] : DCT_OOB;
                    }
                for (int r = wv; r < nx; r += nwv) {
                    const int i = c == 0 ? (r - jm + nx) % nx : (r + jm) % nx;
                    const unsigned p4 = (unsigned)((((long)k * nx + r) * ny + jc) * (long)sizeof(T));
                    T bq[4 * NRB];
    #pragma unroll
                    for (int s = 0; s < 4 * NRB; ++s) bq[s] = tile[min(4 * s + kr, Nm - 1) * LMS + col * pitch + i];
    #pragma unroll
                    for (int rb = 0; rb < 3; ++rb) {
                        if (rb * 16 >= Nc) break;
                        A4 acc = {0, 0, 0, 0};
    #pragma unroll
                        for (int s = 0; s < 4 * NRB; ++s)
                            if (s < NS) acc = mfma_k4(Mt[(c * NcP + rb * 16 + col) * MST + 4 * s + kr], bq[s], acc);
    #pragma unroll
                        for (int e = 0; e < 4; ++e) bst(rqq, qo[rb][e] == DCT_OOB ? DCT_OOB : qo[rb][e] + p4, acc[e]);
                    }
                }
            }
        }
        for (int c = 0; c < (fast ? 0 : 2); ++c) {
            const int Nc = c == 0 ? Nc0 : Nc1;
            const int *cd = cds + c * N;
            for (int r = wv; r < nx; r += nwv) {
                const long p = ((long)k * nx + r) * ny + jc;
                const int i = c == 0 ? (r - jm + nx) % nx : (r + jm) % nx;
                const CellKJI cc{k, jc, i};
                T bq[4 * NRB];
    #pragma unroll
                for (int s = 0; s < 4 * NRB; ++s) bq[s] = tile[min(4 * s + kr, Nm - 1) * LMS + col * pitch + i];
                for (int rb = 0; rb * 16 < Nc; ++rb) {
                    A4 acc = {0, 0, 0, 0};
    #pragma unroll
                    for (int s = 0; s < 4 * NRB; ++s)
                        if (s < NS) acc = mfma_k4(Mt[(c * NcP + rb * 16 + col) * MST + 4 * s + kr], bq[s], acc);
    #pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int nl = rb * 16 + out_row<T>(kr, e);
                        if (nl < Nc && jok) q[dir_elem(m, c, cd[nl], p, cc)] = acc[e];
                    }
                }
            }
        }
        // ---- 4. change of phi_00 and the end of the iteration
        if (!first) {
            const double dm = block_max(dmax, red);
            const double fm = block_max(fmax_, red);
            if (threadIdx.x == 0) {
                atomicMax(&st->eps_num, (unsigned long long)__double_as_longlong(dm));
                atomicMax(&st->eps_den, (unsigned long long)__double_as_longlong(fm));
                if (last_block(a.cnt_mom + (long)b * DCT_MAXNM * 32, &st->cnt_combine, (unsigned)slab, nsl))
                    close_iteration(a, st, b, gseq, g);
            }
        }
        __syncthreads();   // the tile and the scatter table are refilled for the next item
    }
}

size_t dcm_lds_bytes(const CombArgs &a, const MapArgs &m, int is_f64)
{
    const size_t ts = is_f64 ? 8 : 4;
    const size_t pitch = (size_t)((a.geo.nx | 1) + 1);
    return (size_t)a.Nm * (16 * pitch + 4) * ts + (size_t)2 * m.NmP * (m.NcP + 1) * ts +
           (size_t)2 * m.NcP * (m.NmP + 1) * ts + (size_t)4 * m.N * 4;
}

hipError_t launch_dcm(const CombArgs &a, const MapArgs &m, int is_f64, hipStream_t s, int first, int max_wg)
{
    const int nslj = (a.geo.ny + 15) >> 4;
    const int nb = a.nb > 0 ? a.nb : a.B;
    if (a.b0 < 0 || a.b0 + nb > a.B) return hipErrorInvalidValue;
    const long nw = (long)a.geo.nz * nslj * nb;
    const dim3 grid((unsigned)(max_wg > 0 && max_wg < nw ? max_wg : nw));
    const size_t shm = dcm_lds_bytes(a, m, is_f64);
    const int nrb = (a.Nm + 15) / 16;
#define DCT_DCM(T, R, K, F)                                                                               \
    do {                                                                                                  \
        hipError_t e_ = hipFuncSetAttribute((const void *)k_dcm<T, R, K, F>,                               \
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);        \
        if (e_ != hipSuccess) return e_;                                                                  \
        hipLaunchKernelGGL((k_dcm<T, R, K, F>), grid, dim3(512), shm, s, a, m);                            \
    } while (0)
    // the first-iteration form has no D map, so one K-step width serves it
#define DCT_DCM_K(T, R)                                                                                   \
    do {                                                                                                  \
        if (first) DCT_DCM(T, R, 4, true);                                                                 \
        else if (kc <= 4) DCT_DCM(T, R, 4, false);                                                         \
        else if (kc <= 8) DCT_DCM(T, R, 8, false);                                                         \
        else DCT_DCM(T, R, 12, false);                                                                    \
    } while (0)
    const int kc = ((m.Nc[0] > m.Nc[1] ? m.Nc[0] : m.Nc[1]) + 3) / 4;   // K-steps of one class (<= 12)
    if (kc > 12) return hipErrorInvalidValue;
    if (is_f64) {
        if (nrb == 1) DCT_DCM_K(double, 1); else if (nrb == 2) DCT_DCM_K(double, 2); else DCT_DCM_K(double, 3);
    } else {
        if (nrb == 1) DCT_DCM_K(float, 1); else if (nrb == 2) DCT_DCM_K(float, 2); else DCT_DCM_K(float, 3);
    }
#undef DCT_DCM_K
#undef DCT_DCM
    return hipGetLastError();
}

// Anderson acceleration (depth m) of the within-group source iteration,
// applied to the scalar-flux moment.  With G_k = F(phi_k) the moments of the
// sweep of iterate phi_k (as k_combine leaves them) and f_k = G_k - phi_k,
// the next iterate is
//   phi_{k+1} = G_k - sum_i gamma_i (G_{k-i+1} - G_{k-i}),
// gamma minimising || f_k - sum_i gamma_i (f_{k-i+1} - f_{k-i}) ||_2 over the
// voxels (i = 1 .. min(m, k - 1)); the higher moments keep G_k.  A fixed point
// of the accelerated iteration is one of the source iteration (f = 0), so the
// solve converges to the same discrete solution; the stopping rule of
// k_combine then measures max|f| / max|G|.
//
// k_aa_dots: f_k and G_k into the rings, the dot products (FP64, per
// workgroup, summed in a fixed order by the last workgroup) and the small
// least-squares problem (normal equations, Gaussian elimination).
template <typename T>
__global__ __launch_bounds__(256) void k_aa_dots(AAArgs a)
{
    __shared__ double red[8];
    __shared__ double sdots[DCT_AA_NDOT];
    const int b = blockIdx.y;
    RhsState *st = a.state + b;
    // only after an iteration that did not stop the group
    if (st->finished || st->pending || st->it == 0) return;
    const int it = st->it;
    const int g = eff_group(st->g, a.G, a.reverse);
    const long C = a.geo.C;
    const int m = a.m, R = m + 1;
    const int mk = min(m, it - 1);
    const int w = (it - 1) % R;                        // ring slot of iteration it
    const long v = (long)blockIdx.x * 256 + threadIdx.x;
    double dots[DCT_AA_NDOT];
#pragma unroll
    for (int q = 0; q < DCT_AA_NDOT; ++q) dots[q] = 0.0;
    if (v < C) {
        const double Gk = (double)((const T *)a.phi_all)[(((long)b * a.G + g) * a.Nm) * C + v];
        const double fk = Gk - a.phik[(long)b * C + v];
        double *hG = a.hG + (long)b * R * C, *hF = a.hF + (long)b * R * C;
        hG[(long)w * C + v] = Gk;
        hF[(long)w * C + v] = fk;
        double fr[DCT_AA_MAXM + 1];
        fr[0] = fk;
        for (int i = 1; i <= mk; ++i) fr[i] = hF[(long)((w - i + R) % R) * C + v];
        double df[DCT_AA_MAXM];
        for (int i = 0; i < mk; ++i) df[i] = fr[i] - fr[i + 1];   // f_{k-i} - f_{k-i-1}
        int q = 0;
        for (int i = 0; i < mk; ++i)
            for (int j = i; j < mk; ++j) dots[q++] = df[i] * df[j];
        for (int i = 0; i < mk; ++i) dots[q++] = df[i] * fk;
    }
    const int nd = mk * (mk + 1) / 2 + mk;
    for (int q = 0; q < nd; ++q) {
        const double t = block_sum(dots[q], red);
        if (threadIdx.x == 0) sdots[q] = t;
    }
    __shared__ int last;
    if (threadIdx.x == 0) {
        double *pp = a.part + ((long)b * gridDim.x + blockIdx.x) * DCT_AA_NDOT;
        for (int q = 0; q < nd; ++q)
            atomicExch((unsigned long long *)(pp + q), (unsigned long long)__double_as_longlong(sdots[q]));
        last = last_block(a.cnt_sub + (long)b * a.nsub * 32, a.cnt_top + (long)b * 32, blockIdx.x, gridDim.x);
    }
    __syncthreads();
    if (!last || threadIdx.x != 0) return;
    double tot[DCT_AA_NDOT];
    for (int q = 0; q < nd; ++q) tot[q] = 0.0;
    for (unsigned blk = 0; blk < gridDim.x; ++blk) {
        const unsigned long long *pp =
            (const unsigned long long *)(a.part + ((long)b * gridDim.x + blk) * DCT_AA_NDOT);
        for (int q = 0; q < nd; ++q)
            tot[q] += __longlong_as_double((long long)__hip_atomic_load(pp + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    // normal equations A gamma = r (A = Gram matrix of the differences)
    double A[DCT_AA_MAXM][DCT_AA_MAXM + 1];
    int q = 0;
    for (int i = 0; i < mk; ++i)
        for (int j = i; j < mk; ++j) {
            A[i][j] = tot[q];
            A[j][i] = tot[q];
            ++q;
        }
    for (int i = 0; i < mk; ++i) A[i][mk] = tot[q++];
    int use = mk;
    bool ok = mk > 0;
    for (int c = 0; c < mk && ok; ++c) {
        int pr = c;
        for (int r = c + 1; r < mk; ++r)
            if (fabs(A[r][c]) > fabs(A[pr][c])) pr = r;
        // a (nearly) dependent difference: mix with none (plain iteration)
        if (!(fabs(A[pr][c]) > 1e-13 * fabs(A[0][0])) || !isfinite(A[pr][c])) ok = false;
        if (!ok) break;
        if (pr != c)
            for (int k2 = c; k2 <= mk; ++k2) {
                const double t = A[c][k2];
                A[c][k2] = A[pr][k2];
                A[pr][k2] = t;
            }
        for (int r = c + 1; r < mk; ++r) {
            const double f = A[r][c] / A[c][c];
            for (int k2 = c; k2 <= mk; ++k2) A[r][k2] -= f * A[c][k2];
        }
    }
    double gam[DCT_AA_MAXM] = {0.0, 0.0, 0.0, 0.0};
    if (ok) {
        for (int r = mk - 1; r >= 0; --r) {
            double t = A[r][mk];
            for (int k2 = r + 1; k2 < mk; ++k2) t -= A[r][k2] * gam[k2];
            gam[r] = t / A[r][r];
        }
        for (int i = 0; i < mk; ++i) ok = ok && isfinite(gam[i]);
    }
    if (!ok) use = 0;
    st->aa_mk = use;
    for (int i = 0; i < DCT_AA_MAXM; ++i) st->aa_gam[i] = (ok && i < mk) ? gam[i] : 0.0;
}

// k_aa_mix: the mixed iterate phi_{k+1,00} (stored as the iterate of the next
// sweep and over moment 0 of the group's moments, against which k_combine
// measures the next change) and its moment-0 source ext_00 + rho s_0 phi in
// both class layouts, through the slab tile of k_qinit.
template <typename T>
__global__ __launch_bounds__(256) void k_aa_mix(AAArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    T *tile = (T *)smem_raw;
    const int b = blockIdx.y;
    const RhsState *st = a.state + b;
    if (st->finished || st->pending || st->it == 0) return;
    const int it = st->it;
    const int g = eff_group(st->g, a.G, a.reverse);
    const int nx = a.geo.nx, ny = a.geo.ny;
    const long C = a.geo.C;
    const int R = a.m + 1, mk = st->aa_mk, w = (it - 1) % R;
    double gam[DCT_AA_MAXM];
    for (int i = 0; i < DCT_AA_MAXM; ++i) gam[i] = st->aa_gam[i];
    const int nslj = (ny + 15) >> 4;
    const int k = blockIdx.x / nslj, j0 = (blockIdx.x % nslj) * 16;
    const int pitch = (nx | 1) + 1, tile_n = 16 * nx;
    const double *hG = a.hG + (long)b * R * C;
    T *ph0 = (T *)a.phi_all + (((long)b * a.G + g) * a.Nm) * C;
    const T *ext0 = (const T *)a.ext + (long)b * a.Nm * C;
    const int L = a.L;
    for (int idx = threadIdx.x; idx < tile_n; idx += 256) {
        const int jn = idx / nx, in = idx - jn * nx, jj = j0 + jn;
        if (jj >= ny) continue;
        const long v = in + (long)nx * (jj + (long)ny * k);
        double gp = hG[(long)w * C + v];
        double x = gp;
        for (int i = 0; i < mk; ++i) {
            const double gq = hG[(long)((w - i - 1 + R) % R) * C + v];
            x -= gam[i] * (gp - gq);                    // G_{k-i} - G_{k-i-1}
            gp = gq;
        }
        a.phik[(long)b * C + v] = x;
        ph0[v] = (T)x;
        const int mm = a.mat[v];
        const double sc = a.rho[v] * a.ss[(((long)mm * (L + 1)) * a.G + g) * a.G + g];
        tile[jn * pitch + in] = (T)((double)ext0[v] + sc * x);
    }
    __syncthreads();
    T *QA = (T *)a.Qc + (long)b * a.Nm * C;
    T *QB = (T *)a.Qc + ((long)a.B + b) * a.Nm * C;
    for (int idx = threadIdx.x; idx < tile_n; idx += 256) {
        const int r = idx >> 4, jl = idx & 15, j = j0 + jl;
        if (j < ny) {
            const int jm = j % nx;
            const long p = ((long)k * nx + r) * ny + j;
            QA[p] = tile[jl * pitch + rot_row(1, r, jm, nx)];
            QB[p] = tile[jl * pitch + rot_row(0, r, jm, nx)];
        }
    }
}

hipError_t launch_aa(const AAArgs &a, int is_f64, hipStream_t s)
{
    if (a.m < 1 || a.m > DCT_AA_MAXM) return hipErrorInvalidValue;
    const dim3 gd((unsigned)((a.geo.C + 255) / 256), a.B);
    const int nslj = (a.geo.ny + 15) >> 4;
    const dim3 gm((unsigned)(a.geo.nz * nslj), a.B);
    const size_t shm = (size_t)16 * ((a.geo.nx | 1) + 1) * (is_f64 ? 8 : 4);
    if (is_f64) {
        hipLaunchKernelGGL(k_aa_dots<double>, gd, dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_aa_mix<double>, gm, dim3(256), shm, s, a);
    } else {
        hipLaunchKernelGGL(k_aa_dots<float>, gd, dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_aa_mix<float>, gm, dim3(256), shm, s, a);
    }
    return hipGetLastError();
}

// First within-group source of a group (phi = 0, so Q = ext): after a group
// transition (iteration count 0, nothing pending) copy ext from the natural
// layout into both class layouts through an LDS slab tile, as k_combine does
// for the later iterations.  Every other iteration it returns at once.
template <typename T>
__global__ __launch_bounds__(256) void k_qinit(CombArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    T *tile = (T *)smem_raw;
    const int b = blockIdx.y;
    const RhsState *st = a.state + b;
    if (st->finished || st->pending || st->it != 0) return;
    const int nx = a.geo.nx, ny = a.geo.ny;
    const long C = a.geo.C;
    const int Nm = a.Nm;
    const int nslj = (ny + 15) >> 4;
    const int k = blockIdx.x / nslj;
    const int j0 = (blockIdx.x % nslj) * 16;
    const int lm = blockIdx.z;
    const int pitch = (nx | 1) + 1;
    const int tile_n = 16 * nx;
    const T *ext = (const T *)a.ext + ((long)b * Nm + lm) * C;
    T *QA = (T *)a.Qc + ((long)b * Nm + lm) * C;
    T *QB = (T *)a.Qc + (((long)a.B + b) * Nm + lm) * C;
    // warm start: the group starts from the moments phi already stored, so its
    // first source is ext + sigma_s^{gg} phi, as k_combine forms the later ones
    const int g = eff_group(st->g, a.G, a.reverse);
    const T *ph = (const T *)a.phi_all + (((long)b * a.G + g) * Nm + lm) * C;
    const int L = a.L, l = l_of(lm);
    for (int idx = threadIdx.x; idx < tile_n; idx += 256) {
        const int jn = idx / nx, in = idx - jn * nx, jj = j0 + jn;
        if (jj < ny) {
            const long v = in + (long)nx * (jj + (long)ny * k);
            if (a.warm) {
                const int mm = a.mat[v];
                const double sc = a.rho[v] * a.ss[(((long)mm * (L + 1) + l) * a.G + g) * a.G + g];
                tile[jn * pitch + in] = (T)((double)ext[v] + sc * (double)ph[v]);
            } else {
                tile[jn * pitch + in] = ext[v];
            }
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < tile_n; idx += 256) {
        const int r = idx >> 4, jl = idx & 15, j = j0 + jl;
        if (j < ny) {
            const int jm = j % nx;
            const long p = ((long)k * nx + r) * ny + j;
            QA[p] = tile[jl * pitch + rot_row(1, r, jm, nx)];
            QB[p] = tile[jl * pitch + rot_row(0, r, jm, nx)];
        }
    }
}

hipError_t launch_qinit(const CombArgs &a, int is_f64, hipStream_t s)
{
    const int nslj = (a.geo.ny + 15) >> 4;
    dim3 grid((unsigned)(a.geo.nz * nslj), a.B, a.Nm);
    size_t shm = (size_t)16 * ((a.geo.nx | 1) + 1) * (is_f64 ? 8 : 4);
    if (is_f64) hipLaunchKernelGGL(k_qinit<double>, grid, dim3(256), shm, s, a);
    else hipLaunchKernelGGL(k_qinit<float>, grid, dim3(256), shm, s, a);
    return hipGetLastError();
}

hipError_t launch_combine(const CombArgs &a, int is_f64, hipStream_t s)
{
    const int nslj = (a.geo.ny + 15) >> 4;
    dim3 grid((unsigned)(a.geo.nz * nslj), a.B, (a.Nm + a.mpw - 1) / a.mpw);
    size_t shm = (size_t)16 * ((a.geo.nx | 1) + 1) * (is_f64 ? 8 : 4);
    const int per = (16 * a.geo.nx + 255) / 256;   // tile elements per thread
#define DCT_LAUNCH_COMBINE(T)                                                                          do {                                                                                                   if (per <= 1) hipLaunchKernelGGL((k_combine<T, 1>), grid, dim3(256), shm, s, a);                  else if (per <= 2) hipLaunchKernelGGL((k_combine<T, 2>), grid, dim3(256), shm, s, a);             else if (per <= 4) hipLaunchKernelGGL((k_combine<T, 4>), grid, dim3(256), shm, s, a);             else if (per <= 8) hipLaunchKernelGGL((k_combine<T, 8>), grid, dim3(256), shm, s, a);             else hipLaunchKernelGGL((k_combine<T, 0>), grid, dim3(256), shm, s, a);                       } while (0)
    if (is_f64) DCT_LAUNCH_COMBINE(double);
    else DCT_LAUNCH_COMBINE(float);
#undef DCT_LAUNCH_COMBINE
    return hipGetLastError();
}

}  // namespace dct
