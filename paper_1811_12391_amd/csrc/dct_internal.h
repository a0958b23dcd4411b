// Internal declarations of the dctsn HIP library (gfx950).
//
// Data layout in HBM
// ------------------
// Moment-space arrays (ext, phi, phi_u, dose, material, density) use the
// natural voxel order v = i + nx*(j + ny*k).
//
// Direction-space arrays (the angular source q and angular flux psi of every
// direction, and the per-class total cross section used by the sweep) use a
// "diagonal-rotated" layout chosen so that one wavefront step of the sweep
// touches consecutive addresses.  A sweep wave maps its 64 lanes to 64
// consecutive y indices of one z layer and walks x; at step t lane j handles
// the cell with i' + j' = const (primed = reflected into the octant's sweep
// direction).  Two layouts cover the eight octants:
//   class A (Ox*Oy > 0): pos = (k*nx + (i + j) mod nx) * ny + j
//   class B (Ox*Oy < 0): pos = (k*nx + (i - j) mod nx) * ny + j
// In both, the cells of one wave step share the row (k, r) and differ only in
// j, so the 64 lanes read 64 consecutive elements (descending for Oy < 0).
// The moment maps read/write these layouts directly; the combine kernel moves
// between them and the natural layout through LDS, one (k, 16-row) slab at a
// time (a slab is closed under both rotations).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define DCT_MAXMAT 8
#define DCT_MAXL 5
#define DCT_MAXNM ((DCT_MAXL + 1) * (DCT_MAXL + 1))
#define DCT_MAXCHAIN 16   // directions chained through one sweep workgroup
#define DCT_MAXRC 8       // right-hand sides chained through one sweep workgroup
#define DCT_PI 3.14159265358979323846

namespace dct {

// ---------------------------------------------------------------- layouts
__host__ __device__ inline int rot_row(int cls, int i, int jm, int nx)
{
    int r = cls == 0 ? i + jm : i - jm;
    if (r >= nx) r -= nx;
    if (r < 0) r += nx;
    return r;
}

__host__ __device__ inline long cls_pos(int cls, int i, int j, int k, int nx, int ny)
{
    int r = rot_row(cls, i, j % nx, nx);
    return ((long)k * nx + r) * ny + j;
}

// class of a direction: 0 when Ox and Oy have the same sign
__host__ __device__ inline int dir_class(double ox, double oy) { return ((ox > 0) == (oy > 0)) ? 0 : 1; }

// ---------------------------------------------------------------- harmonics
// Real spherical harmonics with Y_00 = 1 and sum_m Y_lm(a) Y_lm(b) = P_l(a.b),
// evaluated in Cartesian form: Y_lm = N_lm * T_l^|m|(z) * {Re, Im}(x + i y)^|m|
// where T_l^m = d^m P_l / dz^m (so no angle functions are needed) and
// N_lm = sqrt((2 - delta_m0) (l-m)! / (l+m)!).
template <typename R>
__host__ __device__ inline void real_sh_cart(int L, R x, R y, R z, R *Y)
{
    // (x + i y)^m
    R cr[DCT_MAXL + 1], ci[DCT_MAXL + 1];
    cr[0] = 1;
    ci[0] = 0;
    for (int m = 1; m <= L; ++m) {
        cr[m] = cr[m - 1] * x - ci[m - 1] * y;
        ci[m] = cr[m - 1] * y + ci[m - 1] * x;
    }
    for (int m = 0; m <= L; ++m) {
        // T_m^m = (2m-1)!!, T_{m+1}^m = (2m+1) z T_m^m, then the three-term recurrence
        R dfac = 1;
        for (int t = 1; t <= m; ++t) dfac *= (R)(2 * t - 1);
        R tm2 = 0, tm1 = dfac;
        for (int l = m; l <= L; ++l) {
            R tl;
            if (l == m) tl = dfac;
            else if (l == m + 1) tl = (R)(2 * m + 1) * z * dfac;
            else tl = ((R)(2 * l - 1) * z * tm1 - (R)(l + m - 1) * tm2) / (R)(l - m);
            if (l > m) { tm2 = tm1; tm1 = tl; }
            R ratio = 1;
            for (int t = l - m + 1; t <= l + m; ++t) ratio /= (R)t;
            R nrm = sqrt((m == 0 ? (R)1 : (R)2) * ratio);
            Y[l * l + l + m] = nrm * tl * cr[m];
            if (m > 0) Y[l * l + l - m] = nrm * tl * ci[m];
        }
    }
}

// Chain layout of the direction-space arrays (K consecutive directions of one
// octant swept by one workgroup): direction n = n0 + d of the chain starting
// at n0 keeps its cell (i, j, k) at element n0 C + (k K nx + row) ny + j with
//   X = d nx + i (Omega_x > 0) or (K - 1 - d) nx + i (Omega_x < 0),
//   row = (X + j) mod K nx (class A) or (X - j) mod K nx (class B).
// K = 1 is the class layout.  From a class-layout position (k, r, j):
// i = (r -+ j) mod nx.
__host__ __device__ inline long chain_pos(int cls, int K, int d, bool sxpos, int r, int j, int k, int nx, int ny)
{
    const int Knx = K * nx;
    int i = cls == 0 ? r - j % nx : r + j % nx;
    if (i < 0) i += nx;
    if (i >= nx) i -= nx;
    const int X = (sxpos ? d : K - 1 - d) * nx + i;
    int row = (cls == 0 ? X + j : X - j) % Knx;
    if (row < 0) row += Knx;
    return ((long)k * Knx + row) * ny + j;
}

// ---------------------------------------------------------------- matrix cores
// 16 x 16 x 4 MFMA tiles (f64, f32): operand placement over the 64 lanes,
// lane = col + 16 * krow:  A[i][k] at lane i + 16 k, B[k][j] at lane j + 16 k;
// D[i][j]: f32 at lane j + 16 (i / 4), element i % 4; f64 at lane j + 16 (i % 4),
// element i / 4 (out_row gives i for lane group kr and element r).
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));

__device__ inline d4_t mfma_k4(double a, double b, d4_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline f4_t mfma_k4(float a, float b, f4_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

template <typename T> struct acc4;
template <> struct acc4<double> { typedef d4_t type; };
template <> struct acc4<float> { typedef f4_t type; };

template <typename T> __device__ inline int out_row(int kr, int r) { return 4 * kr + r; }
template <> __device__ inline int out_row<double>(int kr, int r) { return kr + 4 * r; }

// ---------------------------------------------------------------- buffer access
// Raw buffer access through a descriptor (base, byte range): an offset at or
// beyond the range makes a load return 0 and a store do nothing.  Idle lanes
// pass DCT_OOB, so every lane issues the same memory instructions every step
// and no memory access sits inside a branch (the compiler can then wait on
// exactly the load a step consumes).
typedef __amdgpu_buffer_rsrc_t rsrc_t;
#define DCT_OOB 0x80000000u
// A pointer the compiler cannot prove wave-uniform (e.g. computed from a
// value loaded from memory) made wave-uniform, so that a buffer descriptor
// built from it lives in scalar registers.
__device__ inline const void *wave_ptr(const void *p)
{
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (const void *)(((unsigned long long)hi << 32) | lo);
}
__device__ inline rsrc_t mk_rsrc(const void *p, long bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, p ? (int)bytes : 0, 0x00020000);
}
template <typename T> __device__ inline T bld(rsrc_t r, unsigned off);
template <> __device__ inline float bld<float>(rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <> __device__ inline double bld<double>(rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ inline void bst(rsrc_t r, unsigned off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
__device__ inline void bst(rsrc_t r, unsigned off, double v)
{
    typedef decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)) u64v;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u64v, v), r, off, 0, 0);
}
// The same with a wave-uniform byte offset soff added (scalar operand).
template <typename T> __device__ inline T bld_s(rsrc_t r, unsigned off, unsigned soff);
template <> __device__ inline float bld_s<float>(rsrc_t r, unsigned off, unsigned soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
}
template <> __device__ inline double bld_s<double>(rsrc_t r, unsigned off, unsigned soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
}
__device__ inline void bst_s(rsrc_t r, unsigned off, unsigned soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, soff, 0);
}
__device__ inline void bst_s(rsrc_t r, unsigned off, unsigned soff, double v)
{
    typedef decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)) u64v;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u64v, v), r, off, soff, 0);
}


// Wait until this wave's own earlier memory operations (stores, atomics) have
// completed.  The "last workgroup" counters below need only that: the counter
// and the values it guards are all device atomics, performed in the order the
// wave completes them, and everything else is read by later kernels, after the
// kernel boundary.  (__threadfence() would also write back and invalidate the
// whole L2 of the XCD, once per workgroup.)
__device__ inline void wait_own_memory_ops() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Two-level "last workgroup" detection over the nblk workgroups of one
// right-hand side: workgroup i counts on sub-counter i / 32 (one 128-byte
// line each: sub[(i / 32) * 32]), the last of each group of 32 on `top`, so
// no counter takes an atomic from every workgroup.  True in exactly one
// workgroup, after the device atomics of every workgroup (issued before its
// call) are complete; the counters are left at zero.  One thread calls it.
__device__ inline bool last_block(unsigned *sub, unsigned *top, unsigned i, unsigned nblk)
{
    wait_own_memory_ops();
    const unsigned grp = i >> 5, ngrp = (nblk + 31) >> 5;
    const unsigned in_grp = nblk - (grp << 5) < 32u ? nblk - (grp << 5) : 32u;
    unsigned *c = sub + grp * 32;
    if (atomicAdd(c, 1u) != in_grp - 1) return false;
    atomicExch(c, 0u);
    wait_own_memory_ops();
    if (atomicAdd(top, 1u) != ngrp - 1) return false;
    atomicExch(top, 0u);
    wait_own_memory_ops();
    return true;
}

// ---------------------------------------------------------------- device state
// Per right-hand-side state of the device-driven group / iteration machine.
struct RhsState {
    int g;          // group being iterated (== G when every group is done)
    int it;         // iterations done in group g
    int pending;    // 1: the transition kernel must set up group g
    int finished;   // 1: all groups done
    int nan;        // NaN/Inf seen in a convergence reduction
    int notconv;    // some group stopped at max_iter above tol
    unsigned long long eps_num, eps_den;   // bit patterns of non-negative doubles (max)
    unsigned int cnt_combine, cnt_trans;   // last-block-done counters
    double eps_best;  // smallest eps of the group so far (reduced-precision stop)
    int stall;        // consecutive iterations near tol without a new minimum
    int aa_mk;        // Anderson acceleration: differences used in the last mixing
    double aa_gam[4]; //   and their coefficients
};



// group actually processed at position g of the group sequence
__host__ __device__ inline int eff_group(int g, int G, int reverse) { return reverse ? G - 1 - g : g; }

struct Geo {
    int nx, ny, nz;
    long C;
    double dx, dy, dz;
    double org[3];
};

#define DCT_AA_MAXM 4
#define DCT_AA_NDOT 14   // Gram entries (m (m + 1) / 2) + right-hand side (m) for m <= 4

// Anderson acceleration (depth m) of the within-group source iteration on the
// scalar-flux moment phi_00 of every right-hand side.
struct AAArgs {
    Geo geo;
    int G, Nm, L, B, m;
    int reverse;
    RhsState *state;
    const uint8_t *mat;
    const double *rho;
    const double *ss;         // [M][L+1][G][G]
    void *phi_all;            // T [B][G][Nm][C]
    const void *ext;          // T [B][Nm][C]
    void *Qc;                 // T [2][B][Nm][C]
    double *phik;             // [B][C] the iterate phi_k,00 whose sweep produced G_k
    double *hG, *hF;          // [B][m+1][C] rings of G_k,00 = F(phi_k) and f_k = G_k - phi_k
    double *part;             // [B][nblk][DCT_AA_NDOT] per-workgroup dot products
    unsigned *cnt_sub;        // [B][nsub][32] completion sub-counters (zero between launches)
    int nsub;
    unsigned *cnt_top;        // [B] (one per right-hand side, on its own 128-byte line)
};

struct TraceArgs {
    Geo geo;
    const uint8_t *mat;
    const double *rho;
    const double *st;     // [M][G]
    int G, M, B;
    const double *pos;    // [B][3]
    const double *axis;   // [B][3]
    double half_fan, half_cone;   // radians
    const double *gw;     // [G]
    double *phi_u;        // [B][G][C]
};

struct TransArgs {
    Geo geo;
    int G, M, L, Nm, N, B;
    int S;                    // sources per right-hand side (superposed beams)
    int warm;                 // 1: a new group starts from the moments already in phi_all
    double *aa_phik;          // [B][C] starting iterate phi_00 of the group (Anderson), or null
    double V;
    const uint8_t *mat;
    const double *rho;
    const double *st, *ss;    // [M][G], [M][L+1][G][G]
    const double *pos;        // [B*S][3]
    const double *phi_u;      // [B*S][G][C]
    const double *ext_iso;    // [G][C] or null
    const double *inflow;     // [G] or null
    const int *band_lo;       // [G] lowest group that scatters into g in any material (or null)
    const double *dirs, *w;   // [N][3], [N]
    const double *leak_part;  // [B][N][nblk][3]
    int nblk;
    void *phi_all;            // T [B][G][Nm][C]
    void *ext;                // T [B][Nm][C]
    void *Qc;                 // T [2][B][Nm][C]
    RhsState *state;
    double *bal;              // [B][G][3]
    int *n_unfinished;
    unsigned *cnt_sub;        // [B][nsub][32] completion sub-counters (zero between launches)
    int nsub;                 // ceil(workgroups per right-hand side / 32)
    double *part_bal;         // [B][workgroups][2] per-workgroup removal and production sums
    int b0 = 0;               // the launch covers right-hand sides b0 .. b0 + nb - 1
    int nb = 0;               // (0: all B); B stays the stride of every [B] array
};

struct CombArgs {
    Geo geo;
    int G, L, Nm, B, M;
    const uint8_t *mat;
    const double *rho;
    const double *ss;
    const void *part;         // T [2][B][Nm][C] (class layouts)
    const void *ext;          // T [B][Nm][C]
    void *phi_all;            // T [B][G][Nm][C]
    void *Qc;                 // T [2][B][Nm][C]
    RhsState *state;
    int *iters;               // [B][G]
    double *eps;              // [B][G]
    const int *fixed_iters;   // [G] or null
    double tol;
    int max_iter;
    int stall_window;         // reduced-precision stagnation stop (0 = off)
    int nblocks_per_b;
    int reverse;              // groups run from G-1 down to 0
    unsigned *cnt_mom;        // [B][Nm][32] completion counters of the moment groups, one per 128-byte line
    int mpw;                  // moments per workgroup (>= 1)
    int b0 = 0;               // the launch covers right-hand sides b0 .. b0 + nb - 1
    int nb = 0;               // (0: all B); B stays the stride of every [B] array
    int warm;                 // 1: the first source of a group includes the self-scatter of
                              //    the starting moments (warm start), not Q = ext
};

struct MapArgs {
    long C;
    int B, N, Nm;
    int Nc[2];
    const int *cdir;          // [2][N] global direction index of class-local index
    const void *Mtab;         // [2][NcP][NmP] (T or bf16)
    const void *Dtab;         // [2][NmP][NcP]
    int NcP, NmP;
    const void *Qc;           // T [2][B][Nm][C]
    void *q;                  // T [B][N][C]
    const void *psi;          // T, slot (b*psi_bs + g*psi_gs + n) * C
    long psi_bs, psi_gs;
    int G, reverse;
    void *part;               // T [2][B][Nm][C]
    const RhsState *state;
    int chainK;               // > 1: q and psi in the chain layout (K consecutive directions per block)
    int nx, ny;               // grid (for the chain layout)
    const int *chn0;          // [N] first direction of n's chain (chain layout only)
    const int *chxo;          // [N] x offset of n's slot in the chain's K nx columns: d nx, or
                              //     (K - 1 - d) nx when Omega_x < 0 (chain layout only)
    int first_only;           // M map: only right-hand sides at the first iteration of a group
};

// Cell of a class-layout position p = (k nx + r) ny + j of class cls, for
// addressing q / psi in the chain layout (x = i, y = j, z = k).
struct CellKJI {
    int k, j, i;
};
__device__ inline CellKJI cell_of(const MapArgs &a, int cls, long p)
{
    const int pl = a.nx * a.ny;                      // C < 2^28: 32-bit arithmetic
    const int pi = (int)p;
    const int k = pi / pl;
    const int rem = pi - k * pl;
    const int r = rem / a.ny, j = rem - r * a.ny;
    int i = cls == 0 ? r - j % a.nx : r + j % a.nx;
    if (i < 0) i += a.nx;
    if (i >= a.nx) i -= a.nx;
    return CellKJI{k, j, i};
}

// Element offset of direction n of class cls at class-layout position p (cell
// c = cell_of(p)) in q / psi: the class layout, or the chain layout when
// a.chainK > 1 (a.chn0[n]: first direction of n's chain, a.chxo[n]: x offset
// of n's slot in the chain's virtual grid of K nx columns).
__device__ inline long dir_elem(const MapArgs &a, int cls, int n, long p, const CellKJI &c)
{
    if (a.chainK <= 1) return (long)n * a.C + p;
    const int Knx = a.chainK * a.nx;
    const int X = a.chxo[n] + c.i;
    int row = cls == 0 ? X + c.j : X - c.j;
    if (row >= Knx) row -= Knx;
    if (row < 0) row += Knx;
    return (long)a.chn0[n] * a.C + ((long)c.k * Knx + row) * a.ny + c.j;
}

struct SweepArgs {
    int nx, ny, nz;
    long C;
    int N, B, G;
    int BK, NBJ, NBK, diag, nblk;
    const double *dirs;
    double dx, dy, dz;
    const void *q;            // T [B][N][C]
    void *psi;                // T, direction n of RHS b in group g at (b*psi_bs + g*psi_gs + n) * C
    long psi_bs, psi_gs;      // slot strides (in units of C): N, 0 normally; G*N, N when kept per group
    uint8_t *mask;            // fixed-face sets [B][G][N][C] (kept per group) or null
    int reverse;              // groups run from G-1 down to 0 (adjoint machine)
    int adjoint;              // transposed sweep: reverse traversal, frozen masks, no fixup decisions
    const void *sigc;         // T [2][G][C]
    void *yface;              // T [2][B*N][nx*nz]
    void *zface;              // T [2][B*N][NBJ][(nx+63)*64] (diagonal strips)
    double *leak_part;        // [B][N][nblk][3]
    const RhsState *state;
    const double *inflow;     // [G] or null
    int fixup;
    int sync;                 // 0: barrier per step, 1: LDS progress counters between waves
    int pipe;                 // 1: all blocks of a sweep in one launch, block faces handed over
                              //    through yface_p / zface_p as they are produced
    void *yface_p;            // T [B*N][NBJ][nx*nz], every element the empty marker between launches
    void *zface_p;            // T [B*N][NBK][NBJ][(nx+63)*64]
    unsigned long long *hint; // [B*N][nblk] progress of each pipelined block: (launch tag << 32) | steps done
    unsigned seq;             // host launch counter, part of the launch tag
    int *err;                 // set to non-zero when a bounded wait overflowed
    int layers;               // > 1: every wave sweeps this many z layers (single block, forward only)
    int chainK;               // > 1: K consecutive directions of one octant per workgroup (k_sweep_ch);
                              //      q, psi in the chain layout, sigma_t from sigch
    const void *sigch;        // T [2][G][K C] sigma_t in the chain layout of period K nx
    int b0 = 0;               // the launch covers right-hand sides b0 .. b0 + nb - 1 (layered
    int nb = 0;               // waves and chained sources; 0: all B); B stays the stride of every [B] array
    int rhsK;                 // > 1: one direction of up to rhsK unfinished right-hand sides per
                              //      workgroup, swept back to back (k_sweep_rc)
};

struct AdjTransArgs {
    Geo geo;
    int G, M, L, Nm, N, B;
    const uint8_t *mat;
    const double *rho;
    const double *st, *ss, *kap;
    const double *pos;        // [B][3]
    const double *roi;        // [C]
    const double *phi_u;      // [B][G][C]
    const void *phi_all;      // T [B][G][Nm][C] forward moments
    const void *psi_keep;     // T forward cell fluxes, slot (b*G*N + g*N + n) * C, class layouts
    const void *lamc;         // T adjoint cell values [B][N][C], class layouts
    const double *dirs;
    void *lam_all;            // T [B][G][Nm][C]
    void *phibar;             // T [B][Nm][C]
    void *Qc;                 // T [2][B][Nm][C]
    double *pbu;              // [B][G][C] weights on the uncollided flux
    double *drho;             // [B][C]
    RhsState *state;
    int *n_unfinished;
    unsigned *cnt_sub;        // [B][nsub][32] completion sub-counters (zero between launches)
    int nsub;
};

struct AdjRayArgs {
    Geo geo;
    const uint8_t *mat;
    const double *rho;
    const double *st;         // [M][G]
    int G, M, B;
    const double *pos, *axis;
    double half_fan, half_cone;
    const double *gw;
    const double *pbu;        // [B][G][C]
    double *drho_ray;         // [C] (atomics)
    double *dgw;              // [G] (atomics)
};

struct DoseArgs {
    long C;
    int G, B, Nm;
    int S;                    // sources per right-hand side (superposed beams)
    const uint8_t *mat;
    const double *kap;        // [M][G]
    const double *phi_u;      // [B*S][G][C]
    const void *phi_all;      // T [B][G][Nm][C]
    double *dose;             // [B][C]
    double *phi_c;            // [B][G][C] or null
    double *phi_u_out;        // [B][G][C] (summed over each right-hand side's sources) or null
    int summed;               // 1: dose[C] = sum_b
    const double *hg;         // [G] fluence-to-dose factor per group in place of kerma, or null
    const uint8_t *zero_mat;  // [M] nonzero: dose 0 in that material (fluences still written), or null
};

// Small constant tables passed by value to a one-workgroup kernel that stores
// them into device memory (no host buffer involved): nd doubles, nb bytes.
struct StageConsts {
    int nd, nb;
    double d[256];
    unsigned char b[DCT_MAXMAT];
};

// ---------------------------------------------------------------- launchers
hipError_t launch_trace(const TraceArgs &a, hipStream_t s);
hipError_t launch_sigc(const Geo &g, const uint8_t *mat, const double *rho, const double *st, int G, int M,
                       void *sigc, int is_f64, hipStream_t s);
// sigma_t of every group in the chain layout of period K nx (K copies)
hipError_t launch_sigch(const Geo &g, const void *sigc, int G, int K, void *sigch, int is_f64, hipStream_t s);
hipError_t launch_transition(const TransArgs &a, int is_f64, hipStream_t s);
hipError_t launch_combine(const CombArgs &a, int is_f64, hipStream_t s);
hipError_t launch_qinit(const CombArgs &a, int is_f64, hipStream_t s);
// Anderson acceleration: dot products and mixing coefficients, then the mixed
// iterate phi_00 (and the moment-0 source in both class layouts)
hipError_t launch_aa(const AAArgs &a, int is_f64, hipStream_t s);
// D map + combine + M map of one iteration in one kernel (forward FP64 / FP32 solves)
// first = 1: only the sources at the first iteration of a group, whose q the
// kernel forms from ext alone (the work of k_qinit and the M map)
// max_wg > 0: at most that many (persistent) workgroups, each taking several
// slabs in turn
hipError_t launch_dcm(const CombArgs &a, const MapArgs &m, int is_f64, hipStream_t s, int first = 0,
                      int max_wg = 0);
size_t dcm_lds_bytes(const CombArgs &a, const MapArgs &m, int is_f64);   // Q = ext in the class layouts after a transition
hipError_t launch_mmap(const MapArgs &a, int mode, hipStream_t s);   // mode 0 f64, 1 f32, 2 bf16
hipError_t launch_dmap(const MapArgs &a, int mode, hipStream_t s);
hipError_t launch_sweep(SweepArgs a, int is_f64, hipStream_t s, unsigned seq);
hipError_t launch_dose(const DoseArgs &a, int is_f64, hipStream_t s);
// sum_v w[v] x[v] (FP64, fixed order) into part[nb], nb = min(1024, ceil(n / 256));
// part needs nb + 1 entries
hipError_t launch_wdot(const double *w, const double *x, long n, double *part, hipStream_t s);
hipError_t launch_adj_transition(const AdjTransArgs &a, int is_f64, hipStream_t s);
hipError_t launch_adj_ray(const AdjRayArgs &a, hipStream_t s);
hipError_t launch_adj_init(long C, int G, int B, const uint8_t *mat, const double *kap, const double *roi,
                           double *pbu, hipStream_t s);
// d_density[v] = dray[v] + sum_b drho[b][v]
hipError_t launch_adj_gather(const double *drho, const double *dray, long C, int B, double *out, hipStream_t s);
// lowest index of x[0, n) that is not finite (nonneg: or is negative) into *bad
// (unchanged when every entry passes; the caller sets it to all ones first)
hipError_t launch_screen(const double *x, long n, int nonneg, unsigned long long *bad, hipStream_t s);
hipError_t launch_stage_consts(const StageConsts &c, double *dst_d, unsigned char *dst_b, hipStream_t s);
hipError_t launch_moments_out(const void *phi_all, long n, double *out, int is_f64, hipStream_t s);

}  // namespace dct
