// Diamond-difference transport sweep (eq. 2 on voxels, vacuum or prescribed
// isotropic inflow), one workgroup per (source, direction, block), as a
// diagonal wavefront:
//
//   - a workgroup owns up to 64 y-rows (lanes) x up to 16 z-layers (waves) of
//     one block and walks x; at step t, lane l of wave w handles the cell with
//     reflected x index i' = t - l - w, so all its upwind neighbours were
//     computed at step t-1;
//   - the x face stays in a register (same lane, previous step), the y face
//     comes from lane l-1 by a cross-lane shuffle (DPP), the z face from wave
//     w-1 through an LDS ring guarded by per-wave progress counters;
//   - faces crossing a block boundary go through small global buffers and the
//     blocks of a sweep run as a sequence of block diagonals (KBA ordering);
//   - q, sigma_t and psi live in the class-rotated layout, so the 64 lanes of
//     a wave step read and write 64 consecutive elements; the loads of step
//     t + PF are issued at step t through buffer descriptors.
//
// Cell update: with c_a = 2|Omega_a|/Delta_a,
//   psi_c = (q + sum_a c_a in_a) / (sigma + sum_a c_a),  out_a = 2 psi_c - in_a;
// a negative outgoing face is set to zero and psi_c recomputed from the cell
// balance without that face's diamond relation (its inflow then enters with
// weight c_a / 2), repeating while new negative faces appear.
#include "dct_internal.h"

namespace dct {

// q / d for d > 0 (d >= sum of the face coefficients, never tiny): hardware
// reciprocal refined by Newton-Raphson, then one residual correction of the
// quotient (Markstein); FP64 keeps full precision, FP32 is within an ulp.
__device__ inline double qdiv(double n, double d)
{
    double y = __builtin_amdgcn_rcp(d);
    double e = fma(-d, y, 1.0);
    y = fma(y, e, y);
    e = fma(-d, y, 1.0);
    y = fma(y, e, y);
    double q = n * y;
    double r = fma(-d, q, n);
    return fma(y, r, q);
}
__device__ inline float qdiv(float n, float d)
{
    float y = __builtin_amdgcn_rcpf(d);
    float q = n * y;
    float r = fmaf(-d, q, n);
    return fmaf(y, r, q);
}

// Set-to-zero fixup of one cell (rare path): faces with a negative outflow are
// closed (outflow 0, inflow weighted c_a / 2 in the balance) until no new
// negative face appears.  Returns (psi_c, out_x, out_y, out_z) by value.
template <typename T> struct Cell4 { T pc, xo, yo, zo; int fixed; };

template <typename T>
__device__ __forceinline__ Cell4<T> dd_fixup(T qv, T sv, T cx, T cy, T cz, T xin, T yin, T zin,
                                                         Cell4<T> c)
{
    bool fx = false, fy = false, fz = false;
    for (int pass = 0; pass < 3; ++pass) {
        bool fresh = false;
        if (!fx && c.xo < (T)0) { fx = true; fresh = true; }
        if (!fy && c.yo < (T)0) { fy = true; fresh = true; }
        if (!fz && c.zo < (T)0) { fz = true; fresh = true; }
        if (!fresh) break;
        T n2 = qv, d2 = sv;
        if (fx) n2 += (T)0.5 * cx * xin; else { n2 += cx * xin; d2 += cx; }
        if (fy) n2 += (T)0.5 * cy * yin; else { n2 += cy * yin; d2 += cy; }
        if (fz) n2 += (T)0.5 * cz * zin; else { n2 += cz * zin; d2 += cz; }
        c.pc = n2 / d2;
        c.xo = fx ? (T)0 : c.pc + c.pc - xin;
        c.yo = fy ? (T)0 : c.pc + c.pc - yin;
        c.zo = fz ? (T)0 : c.pc + c.pc - zin;
    }
    c.fixed = (fx ? 1 : 0) | (fy ? 2 : 0) | (fz ? 4 : 0);
    return c;
}

__device__ inline int wrap_row(int r, int nx) { return r == nx ? 0 : (r < 0 ? nx - 1 : r); }

// lane l receives lane l-1's value of v (DPP wave_shr:1); lane 0 receives old
template <typename T>
__device__ inline T dpp_shift_up_or(T v, T old);
template <>
__device__ inline double dpp_shift_up_or<double>(double v, double old)
{
    int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), 0x138, 0xf, 0xf, false);
    int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
template <>
__device__ inline float dpp_shift_up_or<float>(float v, float old)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), 0x138, 0xf, 0xf, false));
}

// Relaxed LDS int access for the inter-wave progress counters.
__device__ inline int lds_ld(const int *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }
__device__ inline void lds_st(int *p, int v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }

#define DCT_SPIN_LIMIT (1 << 20)

// Raw buffer access through a descriptor (base, byte range): an offset at or
// beyond the range makes a load return 0 and a store do nothing.  Idle lanes
// pass DCT_OOB, so every lane issues the same memory instructions every step
// and no memory access sits inside a branch (the compiler can then wait on
// exactly the load a step consumes).
typedef __amdgpu_buffer_rsrc_t rsrc_t;
#define DCT_OOB 0x80000000u
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

// One workgroup = one (source, direction, block).
//
// Wave coupling (SYNC = 1): instead of a workgroup barrier per step, wave w
// publishes its completed step count in LDS (prog[w]) after writing its z
// outflow into a ring of ZR slots; wave w+1 waits only until prog[w] covers
// the step it needs, and wave w waits for wave w+1 only when it would
// overwrite a slot not yet read.  Waves therefore drift out of phase and hide
// each other's latency.  No deadlock: a wave blocked on its successor is
// ahead of it, so the successor is not blocked on data; the last wave never
// waits on a successor.  Every wait is bounded (DCT_SPIN_LIMIT polls); on
// overflow the kernel raises a->err and leaves the loop.
// SYNC = 0 keeps one barrier per step (reference schedule).
//
// Every lane evaluates the cell relations every step; lanes outside the
// wavefront compute on clamped inputs and discard the result (their stores go
// out of range, their x face is not advanced).  A lane's y and z outflows are
// only ever consumed by a neighbour that is active at the next step, which is
// exactly when the lane itself was active.
//
// MODE 0: forward sweep; 1: forward sweep that also records the fixup set of
// every cell (kept for the adjoint); 2: the transposed sweep of the frozen-fixup
// forward sweep (adjoint of the cell relations): cells visited in the reverse
// order (the octant of -Omega), the adjoint face values h enter exactly like DD
// inflows on faces that were not fixed, while a fixed face contributes nothing
// and passes h_out = lambda:
//   lambda = (s + sum_{a free} c_a h_a) / (sigma + sum_{a free} c_a),
//   h_out,a = 2 lambda - h_a (free) or lambda (fixed).
template <typename T, int PF, bool MULTI, int SYNC, int MODE>
__global__ __launch_bounds__(1024) void k_sweep(SweepArgs a)
{
    constexpr bool ADJ = MODE == 2, KEEP = MODE == 1;
    constexpr int ZR = 4;                                   // z-face ring depth (SYNC = 1)
    constexpr unsigned TS = sizeof(T);
    __shared__ T zbuf[SYNC ? 16 : 2][SYNC ? ZR : 16][64];
    __shared__ int prog[16];
    __shared__ double red[3][16];
    const int item = blockIdx.x;
    const int b = item / a.N;
    const int n = item - b * a.N;
    if (a.state[b].finished) return;
    const int g = eff_group(a.state[b].g, a.G, a.reverse);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long C = a.C;
    const int bj = MULTI ? max(0, a.diag - (a.NBK - 1)) + (int)blockIdx.y : 0;
    const int bk = MULTI ? a.diag - bj : 0;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nwv = blockDim.x >> 6;
    const double ox = a.dirs[3 * n], oy = a.dirs[3 * n + 1], oz = a.dirs[3 * n + 2];
    const bool sx = ADJ ? !(ox > 0) : ox > 0, sy = ADJ ? !(oy > 0) : oy > 0, sz = ADJ ? !(oz > 0) : oz > 0;
    const int cls = dir_class(ox, oy);
    const T cx = (T)(2.0 * fabs(ox) / a.dx), cy = (T)(2.0 * fabs(oy) / a.dy), cz = (T)(2.0 * fabs(oz) / a.dz);
    const T csum = cx + cy + cz;
    const int jp = bj * 64 + l, kp = bk * a.BK + w;
    const int nl = min(64, ny - bj * 64), nw = min(a.BK, nz - bk * a.BK);
    const bool valid = l < nl && w < nw;
    const int j = valid ? (sy ? jp : ny - 1 - jp) : 0;
    const int k = valid ? (sz ? kp : nz - 1 - kp) : 0;
    const int jm = j % nx;
    const int rowbase = k * nx * ny + j;                    // element offsets fit in 32 bits (C*8 < 2^31)
    const rsrc_t rq = mk_rsrc((const T *)a.q + (long)item * C, C * TS);
    const rsrc_t rpsi = mk_rsrc((T *)a.psi + ((long)b * a.psi_bs + (long)g * a.psi_gs + n) * C, C * TS);
    const rsrc_t rmask = mk_rsrc((ADJ || KEEP) && a.mask ? a.mask + (((long)b * a.G + g) * a.N + n) * C : nullptr, C);
    const rsrc_t rsg = mk_rsrc((const T *)a.sigc + ((long)cls * a.G + g) * C, C * TS);
    // block faces, ping-pong by block parity so a block never reads a location
    // that a block of the same launch writes
    const long nitems = (long)a.B * a.N;
    const rsrc_t ryi = mk_rsrc((const T *)a.yface + ((long)(bj & 1) * nitems + item) * nx * nz, (long)nx * nz * TS);
    const rsrc_t ryo = mk_rsrc((T *)a.yface + ((long)((bj + 1) & 1) * nitems + item) * nx * nz, (long)nx * nz * TS);
    const rsrc_t rzi = mk_rsrc((const T *)a.zface + ((long)(bk & 1) * nitems + item) * nx * ny, (long)nx * ny * TS);
    const rsrc_t rzo = mk_rsrc((T *)a.zface + ((long)((bk + 1) & 1) * nitems + item) * nx * ny, (long)nx * ny * TS);
    const int jpc = min(jp, ny - 1), kpc = min(kp, nz - 1);   // clamped for padded lanes/waves
    const T bc = a.inflow ? (T)a.inflow[g] : (T)0;
    const int fixup = a.fixup;
    const int NT = nx + nl + nw - 2;
    const int NTp = ((NT + PF - 1) / PF) * PF;
    const int t0l = l + w;                                  // step at which this lane starts its row
    const int dr = sx ? 1 : -1;                             // rotated-row increment per x step
    const int wrap_at = sx ? nx : -1, wrap_to = sx ? 0 : nx - 1;
    const int rstart = rot_row(cls, sx ? 0 : nx - 1, jm, nx);
    const bool ylast = jp == ny - 1, zlast = kp == nz - 1;
    const bool ywriter = MULTI && valid && l == nl - 1 && jp < ny - 1;
    const bool zwriter = MULTI && valid && w == nw - 1 && kp < nz - 1;
    if (SYNC) {
        if (threadIdx.x < 16) prog[threadIdx.x] = 0;
        __syncthreads();
    }

    // The loop starts PF steps early: those steps only issue the first
    // prefetches (every lane is idle), so the loop is entered with no load in
    // flight and the wait counts inside it are those of the steady state.
    T qr[PF], sr[PF], yr[MULTI ? PF : 1], zr[MULTI ? PF : 1];
    int fr[ADJ ? PF : 1];
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        qr[u] = sr[u] = (T)0;
        if (MULTI) yr[MULTI ? u : 0] = zr[MULTI ? u : 0] = (T)0;
        if (ADJ) fr[ADJ ? u : 0] = 0;
    }
    int rp = rstart, rc = rstart;
    T xo = bc, yo = 0, zo = 0;                              // x inflow of a row starts at the boundary value
    double lyv = 0.0, lzv = 0.0;
    int known_prev = 0, known_next = 0, spins = 0;   // wave-uniform
    for (int tb = -PF; tb < NTp; tb += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int t = tb + u;
            const T qv = qr[u], sv = sr[u];
            const int fv = ADJ ? fr[ADJ ? u : 0] : 0;
            T yface_in = bc, zface_in = bc;
            if (MULTI) {
                yface_in = (jp == 0) ? bc : yr[MULTI ? u : 0];
                zface_in = (kp == 0) ? bc : zr[MULTI ? u : 0];
            }
            const int ip = t - t0l;
            const bool act = valid && (unsigned)ip < (unsigned)nx;
            // y inflow: lane l-1's outflow of the previous step; lane 0 takes the
            // boundary / block face value through the DPP "old" operand
            const T yin = dpp_shift_up_or<T>(yo, yface_in);
            T zin;
            if (SYNC) {
                if (w > 0) {
                    // wave-uniform bounded wait; an exhausted budget makes every
                    // later wait fall through (the error flag is raised below)
                    while (known_prev < t && spins < DCT_SPIN_LIMIT) {
                        known_prev = __builtin_amdgcn_readfirstlane(lds_ld(&prog[w - 1]));
                        if (known_prev < t) {
                            __builtin_amdgcn_s_sleep(1);
                            ++spins;
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
                    zin = zbuf[w - 1][(t - 1) & (ZR - 1)][l];
                } else {
                    zin = zface_in;
                }
            } else {
                zin = (w > 0) ? zbuf[(t + 1) & 1][w > 0 ? w - 1 : 0][l] : zface_in;
            }
            const T xin = xo;
            Cell4<T> c;
            if (ADJ) {
                const bool ux = !(fv & 1), uy = !(fv & 2), uz = !(fv & 4);
                const T ex = ux ? cx : (T)0, ey = uy ? cy : (T)0, ez = uz ? cz : (T)0;
                const T num = qv + ex * xin + ey * yin + ez * zin;
                c.pc = qdiv(num, sv + ex + ey + ez);
                c.xo = ux ? c.pc + c.pc - xin : c.pc;
                c.yo = uy ? c.pc + c.pc - yin : c.pc;
                c.zo = uz ? c.pc + c.pc - zin : c.pc;
                c.fixed = 0;
            } else {
                const T num = qv + cx * xin + cy * yin + cz * zin;
                c.pc = qdiv(num, sv + csum);
                c.xo = c.pc + c.pc - xin;
                c.yo = c.pc + c.pc - yin;
                c.zo = c.pc + c.pc - zin;
                c.fixed = 0;
                if (fixup && act && __builtin_expect(fmin(c.xo, fmin(c.yo, c.zo)) < (T)0, 0))
                    c = dd_fixup<T>(qv, sv, cx, cy, cz, xin, yin, zin, c);
            }
            const unsigned po = act ? (unsigned)(rowbase + rc * ny) : DCT_OOB;
            bst(rpsi, act ? po * TS : DCT_OOB, c.pc);
            if (KEEP) __builtin_amdgcn_raw_buffer_store_b8((unsigned char)c.fixed, rmask, po, 0, 0);
            if (MULTI) {
                bst(ryo, (ywriter && act) ? (unsigned)(ip + nx * kp) * TS : DCT_OOB, c.yo);
                bst(rzo, (zwriter && act) ? (unsigned)(ip + nx * jp) * TS : DCT_OOB, c.zo);
            }
            {
                int rn = rc + dr;
                rn = rn == wrap_at ? wrap_to : rn;
                rc = act ? rn : rc;
            }
            // prefetch step t + PF into the slots this step has just consumed
            // (issued after their last use so the new values need no copy)
            {
                const int tp = t + PF;
                const unsigned pp = (unsigned)(rowbase + rp * ny);
                qr[u] = bld<T>(rq, pp * TS);
                sr[u] = bld<T>(rsg, pp * TS);
                if (ADJ) fr[ADJ ? u : 0] = __builtin_amdgcn_raw_buffer_load_b8(rmask, pp, 0, 0);
                const bool inp = valid && (unsigned)(tp - t0l) < (unsigned)nx;
                if (MULTI) {
                    const int ipc = inp ? tp - t0l : 0;
                    yr[MULTI ? u : 0] = bld<T>(ryi, (unsigned)(ipc + nx * kpc) * TS);
                    zr[MULTI ? u : 0] = bld<T>(rzi, (unsigned)(ipc + nx * jpc) * TS);
                }
                int rn = rp + dr;
                rn = rn == wrap_at ? wrap_to : rn;
                rp = inp ? rn : rp;
            }
            lyv += act ? (double)c.yo : 0.0;
            lzv += act ? (double)c.zo : 0.0;
            xo = act ? c.xo : xo;
            yo = c.yo;
            zo = c.zo;
            if (SYNC) {
                if (w + 1 < nwv) {
                    const int need = t - ZR + 2;                // successor must have read slot t - ZR
                    while (known_next < need && spins < DCT_SPIN_LIMIT) {
                        known_next = __builtin_amdgcn_readfirstlane(lds_ld(&prog[w + 1]));
                        if (known_next < need) {
                            __builtin_amdgcn_s_sleep(1);
                            ++spins;
                        }
                    }
                }
                zbuf[w][t & (ZR - 1)][l] = zo;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
                if (l == 0) lds_st(&prog[w], t + 1);
            } else {
                zbuf[t & 1][w][l] = zo;
                __syncthreads();
            }
        }
    }
    if (SYNC && spins >= DCT_SPIN_LIMIT && l == 0) atomicOr(a.err, 1);
    // boundary outflow sums of this block (for the particle balance): the last
    // x outflow of every row, and the y / z outflows of the boundary rows
    double lx = valid ? (double)xo : 0.0;
    double ly = (valid && ylast) ? lyv : 0.0;
    double lz = (valid && zlast) ? lzv : 0.0;
    for (int o = 32; o > 0; o >>= 1) {
        lx += __shfl_down(lx, o, 64);
        ly += __shfl_down(ly, o, 64);
        lz += __shfl_down(lz, o, 64);
    }
    if (l == 0) {
        red[0][w] = lx;
        red[1][w] = ly;
        red[2][w] = lz;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double s = 0.0;
        for (int q = 0; q < nwv; ++q) s += red[threadIdx.x][q];
        a.leak_part[((long)item * a.nblk + bj * a.NBK + bk) * 3 + threadIdx.x] = s;
    }
}

hipError_t launch_sweep(const SweepArgs &a, int is_f64, hipStream_t s)
{
    const int NBJ = a.NBJ, NBK = a.NBK;
    int lo = max(0, a.diag - (NBK - 1));
    int hi = min(a.diag, NBJ - 1);
    dim3 grid((unsigned)(a.B * a.N), (unsigned)(hi - lo + 1));
    dim3 block(64 * a.BK);
    const bool multi = NBJ > 1 || NBK > 1;
    const int mode = a.adjoint ? 2 : (a.mask ? 1 : 0);
#define DCT_LAUNCH_SWEEP(T, PF, M, S, MD) hipLaunchKernelGGL((k_sweep<T, PF, M, S, MD>), grid, block, 0, s, a)
#define DCT_LAUNCH_SWEEP_M(T, PF, M, S)                 \
    do {                                                \
        if (mode == 2) DCT_LAUNCH_SWEEP(T, PF, M, S, 2); \
        else if (mode == 1) DCT_LAUNCH_SWEEP(T, PF, M, S, 1); \
        else DCT_LAUNCH_SWEEP(T, PF, M, S, 0);          \
    } while (0)
#define DCT_LAUNCH_SWEEP_S(T, PF, M) \
    do { if (a.sync) DCT_LAUNCH_SWEEP_M(T, PF, M, 1); else DCT_LAUNCH_SWEEP_M(T, PF, M, 0); } while (0)
    if (is_f64) { if (multi) DCT_LAUNCH_SWEEP_S(double, 4, true); else DCT_LAUNCH_SWEEP_S(double, 8, false); }
    else { if (multi) DCT_LAUNCH_SWEEP_S(float, 8, true); else DCT_LAUNCH_SWEEP_S(float, 8, false); }
#undef DCT_LAUNCH_SWEEP_S
#undef DCT_LAUNCH_SWEEP_M
#undef DCT_LAUNCH_SWEEP
    return hipGetLastError();
}

}  // namespace dct
