// Moment <-> direction maps of the P_N scattering expansion (eq. 2 with the
// Legendre expansion of sigma_s; eq. 3 is row 0 of the D map), as dense
// contractions over voxels on the matrix cores:
//   M map: q[n][p]    = sum_lm M[n][lm] Q[lm][p],  M[n][lm] = (2l+1)/(4pi) Y_lm(Omega_n)
//   D map: part[lm][p] = sum_n D[lm][n] psi[n][p], D[lm][n] = w_n Y_lm(Omega_n)
// Each class of octants (same rotated layout) is one GEMM: rows = the class's
// directions (M map) or the moments (D map), columns = voxel positions in that
// class's layout, K = moments (M map) or the class's directions (D map).
//
// One wave computes 16 x 16 output tiles with v_mfma_*_16x16x4 (f64, f32) or
// v_mfma_f32_16x16x16_bf16 (bf16 inputs, f32 accumulation).  Operand
// placement (64 lanes, lane = col + 16 * krow):
//   A[i][k]: lane i + 16 k        (16x16x16 bf16: k in [4 krow, 4 krow + 4) packed)
//   B[k][j]: lane j + 16 k
//   D[i][j]: f32 / bf16: lane j + 16 (i / 4), element i % 4
//            f64:        lane j + 16 (i % 4), element i / 4
// The 16 lanes of one k-row load 16 consecutive positions, so every load and
// store of q / psi / Q / part is a 16-element contiguous run.
#include "dct_internal.h"

namespace dct {


// round-to-nearest-even fp32 -> bf16 bits
__device__ inline short to_bf16(float f)
{
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// bf16 bits back to fp32 (exact)
__device__ inline float from_bf16(short h) { return __uint_as_float(((unsigned)(unsigned short)h) << 16); }

// bf16 product of split operands: a b ~ ah bh + ah bl + al bh (the high
// parts round to bf16, the low parts are the bf16-rounded remainders), summed
// in fp32 smallest terms first; SPLIT = false keeps the single product ah bh
template <bool SPLIT>
__device__ inline f4_t mfma_bf16x(s4_t ah, s4_t al, s4_t bh, s4_t bl, f4_t acc)
{
    if (SPLIT) {
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
    }
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
}

// One class's map table [rows][cols] into LDS with row stride ST, and its
// class-local -> global direction slots.  The loads of a round are issued
// together (clamped indices, guarded LDS stores), the slot load first.
template <typename T>
__device__ inline void stage_table(T *tab, int ST, const T *src, int rows, int cols, int *cds, const int *cdsrc,
                                   int nc)
{
    const int n = rows * cols;
    const int c0 = cdsrc[min((int)threadIdx.x, max(nc - 1, 0))];
    for (int i0 = threadIdx.x; i0 < n; i0 += 1024) {
        T v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = src[min(i0 + 256 * k, n - 1)];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = i0 + 256 * k;
            if (i < n) tab[(i / cols) * ST + i % cols] = v[k];
        }
    }
    if ((int)threadIdx.x < nc) cds[threadIdx.x] = c0;
    for (int i = threadIdx.x + 256; i < nc; i += 256) cds[i] = cdsrc[i];
}

// ---------------------------------------------------------------- M map
// Operands are loaded unconditionally and all at once (no load sits behind a
// branch, so none waits for the previous one): padded moments (lm >= Nm) read
// a real row whose table column is zero, positions past the grid read the
// last position and are never stored.  The class's table and direction
// slots are staged in LDS (row stride NmP + 1 against bank conflicts).
template <typename T, int NS>
__global__ __launch_bounds__(256) void k_mmap(MapArgs a)
{
    typedef typename acc4<T>::type A4;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_map[];
    const int b = blockIdx.z, c = blockIdx.y;
    if (a.state[b].finished) return;
    if (a.first_only && (a.state[b].it != 0 || a.state[b].pending)) return;
    const int l = threadIdx.x & 63, col = l & 15, kr = l >> 4;
    const long C = a.C;
    const long p = (long)blockIdx.x * 64 + (threadIdx.x >> 6) * 16 + col;
    const bool inb = p < C;
    const long pc = inb ? p : C - 1;
    const CellKJI cp = a.chainK > 1 ? cell_of(a, c, pc) : CellKJI{0, 0, 0};
    const int Nm = a.Nm, Nc = a.Nc[c], NmP = a.NmP, ST = a.NmP + 1;
    const T *Q = (const T *)a.Qc + ((long)c * a.B + b) * Nm * C;
    T bq[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) bq[s] = Q[(long)min(4 * s + kr, Nm - 1) * C + pc];
    T *tab = (T *)smem_map;                              // [NcP][NmP + 1]
    int *cds = (int *)(tab + (long)a.NcP * ST);
    stage_table(tab, ST, (const T *)a.Mtab + (long)c * a.NcP * NmP, a.NcP, NmP, cds, a.cdir + c * a.N, Nc);
    __syncthreads();
    T *q = (T *)a.q + (long)b * a.N * C;
    for (int rb = 0; rb * 16 < Nc; ++rb) {
        A4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < NS; ++s) acc = mfma_k4(tab[(rb * 16 + col) * ST + 4 * s + kr], bq[s], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int nl = rb * 16 + out_row<T>(kr, r);
            if (nl < Nc && inb) q[dir_elem(a, c, cds[nl], p, cp)] = acc[r];
        }
    }
}

template <int NS16, bool SPLIT>
__global__ __launch_bounds__(256) void k_mmap_bf16(MapArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_map[];
    const int b = blockIdx.z, c = blockIdx.y;
    if (a.state[b].finished) return;
    if (a.first_only && (a.state[b].it != 0 || a.state[b].pending)) return;
    const int l = threadIdx.x & 63, col = l & 15, kr = l >> 4;
    const long C = a.C;
    const long p = (long)blockIdx.x * 64 + (threadIdx.x >> 6) * 16 + col;
    const bool inb = p < C;
    const long pc = inb ? p : C - 1;
    const CellKJI cp = a.chainK > 1 ? cell_of(a, c, pc) : CellKJI{0, 0, 0};
    const int Nm = a.Nm, Nc = a.Nc[c], NmP = a.NmP, ST = a.NmP + 4;   // 8-byte aligned rows
    const float *Q = (const float *)a.Qc + ((long)c * a.B + b) * Nm * C;
    float fq[NS16][4];
#pragma unroll
    for (int s = 0; s < NS16; ++s)
#pragma unroll
        for (int e = 0; e < 4; ++e) fq[s][e] = Q[(long)min(16 * s + 4 * kr + e, Nm - 1) * C + pc];
    short *tab = (short *)smem_map;                      // [NcP][NmP + 4] (high parts)
    short *tabl = tab + (long)a.NcP * ST;                // [NcP][NmP + 4] (remainders, SPLIT)
    int *cds = (int *)(tab + (long)(SPLIT ? 2 : 1) * a.NcP * ST);
    stage_table(tab, ST, (const short *)a.Mtab + (long)c * a.NcP * NmP, a.NcP, NmP, cds, a.cdir + c * a.N, Nc);
    if (SPLIT)
        stage_table(tabl, ST, (const short *)a.Mtab + (long)(2 + c) * a.NcP * NmP, a.NcP, NmP, cds,
                    a.cdir + c * a.N, Nc);
    __syncthreads();
    s4_t bq[NS16], bql[NS16];
#pragma unroll
    for (int s = 0; s < NS16; ++s)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            bq[s][e] = to_bf16(fq[s][e]);
            bql[s][e] = SPLIT ? to_bf16(fq[s][e] - from_bf16(bq[s][e])) : (short)0;
        }
    float *q = (float *)a.q + (long)b * a.N * C;
    for (int rb = 0; rb * 16 < Nc; ++rb) {
        f4_t acc = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < NS16; ++s) {
            const int o = (rb * 16 + col) * ST + 16 * s + 4 * kr;
            const s4_t av = *(const s4_t *)(tab + o);
            const s4_t avl = SPLIT ? *(const s4_t *)(tabl + o) : av;
            acc = mfma_bf16x<SPLIT>(av, avl, bq[s], bql[s], acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int nl = rb * 16 + 4 * kr + r;
            if (nl < Nc && inb) q[dir_elem(a, c, cds[nl], p, cp)] = acc[r];
        }
    }
}

// ---------------------------------------------------------------- D map
// As the M map: the class's table in LDS, the psi operands of up to KC
// K-steps loaded at once (clamped, unconditional; the table columns of
// padded directions are zero; their direction slots read from global memory
// so the loads need not wait for the staging), NRB 16-row blocks of moments
// accumulated together so psi is read once.
template <typename T, int NRB>
__global__ __launch_bounds__(256) void k_dmap(MapArgs a)
{
    typedef typename acc4<T>::type A4;
    constexpr int KC = 16;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_map[];
    const int b = blockIdx.z, c = blockIdx.y;
    if (a.state[b].finished) return;
    const int l = threadIdx.x & 63, col = l & 15, kr = l >> 4;
    const long C = a.C;
    const long p = (long)blockIdx.x * 64 + (threadIdx.x >> 6) * 16 + col;
    const bool inb = p < C;
    const long pc = inb ? p : C - 1;
    const CellKJI cp = a.chainK > 1 ? cell_of(a, c, pc) : CellKJI{0, 0, 0};
    const int Nm = a.Nm, Nc = a.Nc[c], NcP = a.NcP, ST = a.NcP + 1;
    const int g = eff_group(a.state[b].g, a.G, a.reverse);
    const T *psi = (const T *)a.psi + ((long)b * a.psi_bs + (long)g * a.psi_gs) * C;
    // the psi operands of the first K-chunk are requested before the table
    // is staged, their direction slots read straight from global memory (a
    // few hundred bytes, cache-resident), so the table staging and its
    // barrier overlap the psi loads instead of preceding them
    const int *cdg = a.cdir + c * a.N;
    T bv[KC];
    auto load_chunk = [&](int k0) __attribute__((always_inline)) {
        int dn[KC];
#pragma unroll
        for (int u = 0; u < KC; ++u) dn[u] = cdg[min(k0 + 4 * u + kr, Nc - 1)];
#pragma unroll
        for (int u = 0; u < KC; ++u) bv[u] = psi[dir_elem(a, c, dn[u], pc, cp)];
    };
    load_chunk(0);
    T *tab = (T *)smem_map;                              // [NmP][NcP + 1]
    int *cds = (int *)(tab + (long)a.NmP * ST);
    stage_table(tab, ST, (const T *)a.Dtab + (long)c * a.NmP * NcP, a.NmP, NcP, cds, cdg, Nc);
    __syncthreads();
    T *part = (T *)a.part + ((long)c * a.B + b) * Nm * C;
    A4 acc[NRB];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) acc[rb] = A4{0, 0, 0, 0};
    for (int k0 = 0; k0 < Nc; k0 += 4 * KC) {
        if (k0 > 0) load_chunk(k0);
#pragma unroll
        for (int u = 0; u < KC; ++u)
            if (k0 + 4 * u < Nc) {
#pragma unroll
                for (int rb = 0; rb < NRB; ++rb)
                    acc[rb] = mfma_k4(tab[(rb * 16 + col) * ST + k0 + 4 * u + kr], bv[u], acc[rb]);
            }
    }
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int lm = rb * 16 + out_row<T>(kr, r);
            if (lm < Nm && inb) part[(long)lm * C + p] = acc[rb][r];
        }
}

template <bool SPLIT>
__global__ __launch_bounds__(256) void k_dmap_bf16(MapArgs a)
{
    constexpr int KC = 4;                                // K-steps of 16 directions per load round
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_map[];
    const int b = blockIdx.z, c = blockIdx.y;
    if (a.state[b].finished) return;
    const int l = threadIdx.x & 63, col = l & 15, kr = l >> 4;
    const long C = a.C;
    const long p = (long)blockIdx.x * 64 + (threadIdx.x >> 6) * 16 + col;
    const bool inb = p < C;
    const long pc = inb ? p : C - 1;
    const CellKJI cp = a.chainK > 1 ? cell_of(a, c, pc) : CellKJI{0, 0, 0};
    const int Nm = a.Nm, Nc = a.Nc[c], NcP = a.NcP, ST = a.NcP + 4;
    short *tab = (short *)smem_map;                      // [NmP][NcP + 4] (high parts)
    short *tabl = tab + (long)a.NmP * ST;                // [NmP][NcP + 4] (remainders, SPLIT)
    int *cds = (int *)(tab + (long)(SPLIT ? 2 : 1) * a.NmP * ST);
    stage_table(tab, ST, (const short *)a.Dtab + (long)c * a.NmP * NcP, a.NmP, NcP, cds, a.cdir + c * a.N, Nc);
    if (SPLIT)
        stage_table(tabl, ST, (const short *)a.Dtab + (long)(2 + c) * a.NmP * NcP, a.NmP, NcP, cds,
                    a.cdir + c * a.N, Nc);
    __syncthreads();
    const int g = eff_group(a.state[b].g, a.G, a.reverse);
    const float *psi = (const float *)a.psi + ((long)b * a.psi_bs + (long)g * a.psi_gs) * C;
    float *part = (float *)a.part + ((long)c * a.B + b) * Nm * C;
    f4_t acc[3] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    const int nrb = (Nm + 15) / 16;
    for (int k0 = 0; k0 < Nc; k0 += 16 * KC) {
        float fv[KC][4];
#pragma unroll
        for (int u = 0; u < KC; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                fv[u][e] = psi[dir_elem(a, c, cds[min(k0 + 16 * u + 4 * kr + e, Nc - 1)], pc, cp)];
#pragma unroll
        for (int u = 0; u < KC; ++u)
            if (k0 + 16 * u < Nc) {
                s4_t bv, bvl;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    bv[e] = to_bf16(fv[u][e]);
                    bvl[e] = SPLIT ? to_bf16(fv[u][e] - from_bf16(bv[e])) : (short)0;
                }
#pragma unroll
                for (int rb = 0; rb < 3; ++rb)
                    if (rb < nrb) {
                        const int o = (rb * 16 + col) * ST + k0 + 16 * u + 4 * kr;
                        const s4_t av = *(const s4_t *)(tab + o);
                        const s4_t avl = SPLIT ? *(const s4_t *)(tabl + o) : av;
                        acc[rb] = mfma_bf16x<SPLIT>(av, avl, bv, bvl, acc[rb]);
                    }
            }
    }
#pragma unroll
    for (int rb = 0; rb < 3; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int lm = rb * 16 + 4 * kr + r;
            if (rb < nrb && lm < Nm && inb) part[(long)lm * C + p] = acc[rb][r];
        }
}

// LDS of the FP map kernels: the class's table (padded row stride) and its
// direction slots
template <typename T> static size_t map_lds(const MapArgs &a, bool mmap)
{
    const size_t rows = mmap ? a.NcP : a.NmP, st = (mmap ? a.NmP : a.NcP) + 1;
    return rows * st * sizeof(T) + (size_t)a.N * 4;
}

template <typename T>
static void dispatch_mmap(const MapArgs &a, dim3 grid, hipStream_t s)
{
    int NS = (a.Nm + 3) / 4;
    const size_t shm = map_lds<T>(a, true);
    switch (NS) {
    case 1: hipLaunchKernelGGL((k_mmap<T, 1>), grid, dim3(256), shm, s, a); break;
    case 2: hipLaunchKernelGGL((k_mmap<T, 2>), grid, dim3(256), shm, s, a); break;
    case 3: hipLaunchKernelGGL((k_mmap<T, 3>), grid, dim3(256), shm, s, a); break;
    case 4: hipLaunchKernelGGL((k_mmap<T, 4>), grid, dim3(256), shm, s, a); break;
    case 5: hipLaunchKernelGGL((k_mmap<T, 5>), grid, dim3(256), shm, s, a); break;
    case 6: hipLaunchKernelGGL((k_mmap<T, 6>), grid, dim3(256), shm, s, a); break;
    case 7: hipLaunchKernelGGL((k_mmap<T, 7>), grid, dim3(256), shm, s, a); break;
    case 8: hipLaunchKernelGGL((k_mmap<T, 8>), grid, dim3(256), shm, s, a); break;
    default: hipLaunchKernelGGL((k_mmap<T, 9>), grid, dim3(256), shm, s, a); break;
    }
}

template <typename T>
static void dispatch_dmap(const MapArgs &a, dim3 grid, hipStream_t s)
{
    const size_t shm = map_lds<T>(a, false);
    const int nrb = (a.Nm + 15) / 16;
    if (nrb == 1) hipLaunchKernelGGL((k_dmap<T, 1>), grid, dim3(256), shm, s, a);
    else if (nrb == 2) hipLaunchKernelGGL((k_dmap<T, 2>), grid, dim3(256), shm, s, a);
    else hipLaunchKernelGGL((k_dmap<T, 3>), grid, dim3(256), shm, s, a);
}

hipError_t launch_mmap(const MapArgs &a, int mode, hipStream_t s)
{
    dim3 grid((unsigned)((a.C + 63) / 64), 2, a.B);
    if (mode == 0) dispatch_mmap<double>(a, grid, s);
    else if (mode == 1) dispatch_mmap<float>(a, grid, s);
    else {
        // mode 2: bf16 inputs; mode 3: split bf16 inputs (high part + remainder)
        const int NS16 = (a.Nm + 15) / 16;
        const size_t shm = (size_t)(mode == 3 ? 2 : 1) * a.NcP * (a.NmP + 4) * 2 + (size_t)a.N * 4;
#define DCT_MB(NS, SP) hipLaunchKernelGGL((k_mmap_bf16<NS, SP>), grid, dim3(256), shm, s, a)
        if (mode == 3) {
            if (NS16 == 1) DCT_MB(1, true); else if (NS16 == 2) DCT_MB(2, true); else DCT_MB(3, true);
        } else {
            if (NS16 == 1) DCT_MB(1, false); else if (NS16 == 2) DCT_MB(2, false); else DCT_MB(3, false);
        }
#undef DCT_MB
    }
    return hipGetLastError();
}

hipError_t launch_dmap(const MapArgs &a, int mode, hipStream_t s)
{
    dim3 grid((unsigned)((a.C + 63) / 64), 2, a.B);
    if (mode == 0) dispatch_dmap<double>(a, grid, s);
    else if (mode == 1) dispatch_dmap<float>(a, grid, s);
    else {
        const size_t shm = (size_t)(mode == 3 ? 2 : 1) * a.NmP * (a.NcP + 4) * 2 + (size_t)a.N * 4;
        if (mode == 3) hipLaunchKernelGGL(k_dmap_bf16<true>, grid, dim3(256), shm, s, a);
        else hipLaunchKernelGGL(k_dmap_bf16<false>, grid, dim3(256), shm, s, a);
    }
    return hipGetLastError();
}

}  // namespace dct
