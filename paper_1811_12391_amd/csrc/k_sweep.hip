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

// q / d for d > 0 (a normal number): hardware reciprocal refined by
// Newton-Raphson (rcp_nr), then one residual correction of the quotient
// (Markstein, qdiv_y); FP64 keeps full precision, FP32 is within an ulp.
__device__ inline double rcp_nr(double d)
{
    double y = __builtin_amdgcn_rcp(d);
    double e = fma(-d, y, 1.0);
    y = fma(y, e, y);
    e = fma(-d, y, 1.0);
    return fma(y, e, y);
}
__device__ inline float rcp_nr(float d) { return __builtin_amdgcn_rcpf(d); }
template <typename T> __device__ inline T qdiv_y(T n, T d, T y)
{
    T q = n * y;
    T r = fma(-d, q, n);
    return fma(y, r, q);
}
template <typename T> __device__ inline T qdiv(T n, T d) { return qdiv_y(n, d, rcp_nr(d)); }

// Set-to-zero fixup of one cell: faces with a negative outflow are
// closed (outflow 0, inflow weighted c_a / 2 in the balance) until no new
// negative face appears.  Returns (psi_c, out_x, out_y, out_z) by value.
template <typename T> struct Cell4 { T pc, xo, yo, zo; int fixed; };

// q / d inside the fixup: FP64 as qdiv; FP32 takes the hardware reciprocal
// alone (the plain update already does), which keeps the pass short
__device__ inline double fix_div(double n, double d) { return qdiv(n, d); }
__device__ inline float fix_div(float n, float d) { return n * rcp_nr(d); }

// Every pass is free of branches: the open / closed state of a face is a
// multiplier e_a (1 open, 0 closed), so the balance is
//   psi_c (sigma + sum_a e_a c_a) = q + sum_a (1 + e_a) (c_a / 2) in_a
// with c_a pre-doubled, and a closed face's outflow e_a (2 psi_c - in_a) is 0.
// Only an open face can test negative (a closed one holds 0), so a pass
// closes exactly the new negative faces.  The loop ends for a lane as soon
// as it has none; the wave runs a pass while any lane needs it.
template <typename T>
__device__ __forceinline__ Cell4<T> dd_fixup(T qv, T sv, T cx, T cy, T cz, T xin, T yin, T zin,
                                                         Cell4<T> c)
{
    T ex = (T)1, ey = (T)1, ez = (T)1;
    const T hx = (T)0.5 * cx, hy = (T)0.5 * cy, hz = (T)0.5 * cz;
    for (int pass = 0; pass < 3; ++pass) {
        if (!(fmin(c.xo, fmin(c.yo, c.zo)) < (T)0)) break;
        ex = c.xo < (T)0 ? (T)0 : ex;
        ey = c.yo < (T)0 ? (T)0 : ey;
        ez = c.zo < (T)0 ? (T)0 : ez;
        T n2 = qv + fma(hx, ex, hx) * xin;
        n2 += fma(hy, ey, hy) * yin;
        n2 += fma(hz, ez, hz) * zin;
        T d2 = fma(cx, ex, sv);
        d2 = fma(cy, ey, d2);
        d2 = fma(cz, ez, d2);
        c.pc = fix_div(n2, d2);
        c.xo = ex * (c.pc + c.pc - xin);
        c.yo = ey * (c.pc + c.pc - yin);
        c.zo = ez * (c.pc + c.pc - zin);
    }
    c.fixed = (ex > (T)0 ? 0 : 1) | (ey > (T)0 ? 0 : 2) | (ez > (T)0 ? 0 : 4);
    return c;
}

// Streaming access for the two per-direction arrays of k_sweep: q of a
// direction is read once and psi written once per sweep, so both carry the
// non-temporal hint (aux bit 1, NT on gfx950) and do not push the class's
// sigma_t table, which every direction re-reads, out of the L2 (HBM bytes per
// single-source launch 50 -> 44 MB, time unchanged).  The layered-wave kernel
// keeps the default policy: with 36 sources the hint made it 15% slower.
template <typename T> __device__ inline T bld_nt(rsrc_t r, unsigned off);
template <> __device__ inline float bld_nt<float>(rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 2));
}
template <> __device__ inline double bld_nt<double>(rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 2));
}
__device__ inline void bst_nt(rsrc_t r, unsigned off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 2);
}
__device__ inline void bst_nt(rsrc_t r, unsigned off, double v)
{
    typedef decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)) u64v;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u64v, v), r, off, 0, 2);
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

// Device-coherent loads (sc1: served by L2, never by the CU's L1), used for
// block faces handed between workgroups inside one launch.
template <typename T> __device__ inline T bld_dev(rsrc_t r, unsigned off);
template <> __device__ inline float bld_dev<float>(rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 16));
}
template <> __device__ inline double bld_dev<double>(rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 16));
}
// Stores need no cache-policy bit: the CU's vector L1 is write-through, so a
// plain store reaches the L2 that the consumer's sc1 load reads.
__device__ inline void bst_dev(rsrc_t r, unsigned off, float v) { bst(r, off, v); }
__device__ inline void bst_dev(rsrc_t r, unsigned off, double v) { bst(r, off, v); }
// "Empty" marker of a handed-over face: all bits set, a NaN payload that the
// arithmetic never produces (generated NaNs are the canonical quiet NaN).
template <typename T> __device__ inline T face_empty();
template <> __device__ inline float face_empty<float>() { return __builtin_bit_cast(float, 0xffffffffu); }
template <> __device__ inline double face_empty<double>() { return __builtin_bit_cast(double, ~0ull); }
__device__ inline bool is_empty(float v) { return __builtin_bit_cast(unsigned, v) == 0xffffffffu; }
__device__ inline bool is_empty(double v) { return __builtin_bit_cast(unsigned long long, v) == ~0ull; }

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
// PIPE: every block of a sweep runs in the same launch.  The workgroup index
// is mapped so that all blocks of one (source, direction) share an XCD (the
// hardware deals workgroups to the 8 XCDs round robin, so indices congruent
// mod 8 share one L2) and upstream blocks come first in dispatch order.  A
// block face is handed over element by element: the producer stores the
// value, the consumer waits (bounded) until the element is no longer the
// empty marker, uses it and stores the marker back, so every face buffer is
// empty again when the launch ends.  Consumers never block producers, so the
// blocks form a pipeline along the sweep diagonal.  Inside a workgroup the
// waves of a pipelined block keep one barrier per step (SYNC = 0).
//
// MODE 0: forward sweep; 1: forward sweep that also records the fixup set of
// every cell (kept for the adjoint); 2: the transposed sweep of the frozen-fixup
// forward sweep (adjoint of the cell relations): cells visited in the reverse
// order (the octant of -Omega), the adjoint face values h enter exactly like DD
// inflows on faces that were not fixed, while a fixed face contributes nothing
// and passes h_out = lambda:
//   lambda = (s + sum_{a free} c_a h_a) / (sigma + sum_{a free} c_a),
//   h_out,a = 2 lambda - h_a (free) or lambda (fixed).
template <typename T, int PF, bool MULTI, int SYNC, int MODE, bool PIPE>
__global__ __launch_bounds__(1024) void k_sweep(SweepArgs a)
{
    constexpr bool ADJ = MODE == 2, KEEP = MODE == 1;
    constexpr int ZR = 4;                                   // z-face ring depth (SYNC = 1)
    constexpr int FD = PF;                                  // prefetch distance of block faces (as q, sigma)
    constexpr unsigned TS = sizeof(T);
    // SYNC = 0 without block faces: row w + 1 holds wave w's z outflow and
    // row 0 the boundary value, so every wave reads its z inflow from LDS
    constexpr bool ZROW = !SYNC && !MULTI;
    __shared__ T zbuf[SYNC ? 16 : 2][SYNC ? ZR : (ZROW ? 17 : 16)][64];
    __shared__ int prog[16];
    __shared__ double red[3][16];
    const long nitems = (long)a.B * a.N;
    int item, bj = 0, bk = 0;
    if (PIPE) {
        const int h = blockIdx.x, xcd = h & 7, slot = h >> 3;
        const int qq = slot / a.nblk, blk = slot - qq * a.nblk;
        item = qq * 8 + xcd;
        if (item >= nitems) return;
        // blk enumerates the blocks diagonal by diagonal (upstream first)
        int rem = blk;
        for (int d = 0; d < a.NBJ + a.NBK - 1; ++d) {
            const int lo = max(0, d - (a.NBK - 1)), hi = min(d, a.NBJ - 1);
            if (rem <= hi - lo) {
                bj = lo + rem;
                bk = d - bj;
                break;
            }
            rem -= hi - lo + 1;
        }
    } else {
        item = blockIdx.x;
        bj = MULTI ? max(0, a.diag - (a.NBK - 1)) + (int)blockIdx.y : 0;
        bk = MULTI ? a.diag - bj : 0;
    }
    const int b = item / a.N;
    const int n = item - b * a.N;
    if (a.state[b].finished) return;
    const int g = eff_group(a.state[b].g, a.G, a.reverse);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long C = a.C;
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
    // block faces: with PIPE one slot per block boundary (entering face of
    // block bj / bk); otherwise ping-pong by block parity so a block never
    // reads a location that a block of the same launch writes
    const long yslot_in = PIPE ? (long)item * a.NBJ + bj : (long)(bj & 1) * nitems + item;
    const long yslot_out = PIPE ? (long)item * a.NBJ + bj + 1 : (long)((bj + 1) & 1) * nitems + item;
    const long zslot_in = PIPE ? (long)item * a.NBK + bk : (long)(bk & 1) * nitems + item;
    const long zslot_out = PIPE ? (long)item * a.NBK + bk + 1 : (long)((bk + 1) & 1) * nitems + item;
    T *yfb = (T *)(PIPE ? a.yface_p : a.yface), *zfb = (T *)(PIPE ? a.zface_p : a.zface);
    const rsrc_t ryi = mk_rsrc(yfb + yslot_in * nx * nz, (long)nx * nz * TS);
    const rsrc_t ryo = mk_rsrc(yfb + yslot_out * nx * nz, (long)nx * nz * TS);
    // z faces are stored per y block along the wave diagonal: element
    // (ip + l) * 64 + l for lane l, so the 64 lanes that hand over (or take)
    // a face in one step touch 64 consecutive elements
    const long ZS = (long)(nx + 63) * 64;
    const rsrc_t rzi = mk_rsrc(zfb + (zslot_in * a.NBJ + bj) * ZS, ZS * TS);
    const rsrc_t rzo = mk_rsrc(zfb + (zslot_out * a.NBJ + bj) * ZS, ZS * TS);
    const bool ytaker = valid && l == 0 && bj > 0;            // lanes whose inflow is a block face
    const bool ztaker = valid && w == 0 && bk > 0;
    const bool yreader = PIPE && ytaker;                      // ... handed over inside the launch
    const bool zreader = PIPE && ztaker;
    // Pacing of pipelined blocks: the last wave of every block publishes its
    // step count (tagged with the launch's group / iteration) after each group
    // of PF steps; a downstream block holds back until its upstream blocks are
    // far enough ahead that the face elements its prefetches read have been
    // written.  The hint is advisory (relaxed, unordered with the face
    // stores): correctness rests on the empty-marker check alone.
    const unsigned tag = ((unsigned)(a.state[b].g * 65536 + a.state[b].it) ^ (a.seq * 0x9E3779B9u)) | 1u;
    const rsrc_t rh = mk_rsrc(PIPE ? a.hint : nullptr, (long)nitems * a.nblk * 8);
    const unsigned hoff_self = (unsigned)((item * a.nblk + bj * a.NBK + bk) * 8);
    const unsigned hoff_z = bk > 0 ? (unsigned)((item * a.nblk + bj * a.NBK + bk - 1) * 8) : DCT_OOB;
    const unsigned hoff_y = bj > 0 ? (unsigned)((item * a.nblk + (bj - 1) * a.NBK + bk) * 8) : DCT_OOB;
    const bool hint_writer = PIPE && w == nw - 1 && l == 0;
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
    if (ZROW) {
        if (w == 0) zbuf[0][0][l] = zbuf[1][0][l] = bc;
        __syncthreads();
    }

    // The loop starts PF steps early: those steps only issue the first
    // prefetches (every lane is idle), so the loop is entered with no load in
    // flight and the wait counts inside it are those of the steady state.
    // Step t loads the operands of step t + PF - 1 into the ring slot that
    // step t - 1 has just consumed.
    T qr[PF], sr[PF], yr[MULTI ? PF : 1], zr[MULTI ? PF : 1];
    int fr[ADJ ? PF : 1];
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        qr[u] = sr[u] = (T)0;
        if (MULTI) yr[MULTI ? u : 0] = zr[MULTI ? u : 0] = (T)0;
        if (ADJ) fr[ADJ ? u : 0] = 0;
    }
    // Element offsets: one rotated row (ny elements) per x step, wrapping
    // inside the (k, rotated row) plane.  Lane l reaches x index t - l - w at
    // step t and the rotation adds (or subtracts) its row j = j0 +- l, so the
    // rotated row of step t is the same for every lane of a wave: the row
    // part of the offset is a wave-uniform scalar (sre, for the prefetched
    // step), the lane part a constant (rowbase).  The offsets a prefetch used
    // are kept and reused by the stores of that step PF - 1 steps later.
    const int dny = sx ? ny : -ny;
    const int wrap_at_r = wrap_at * ny, wrap_to_r = wrap_to * ny;
    int sre = __builtin_amdgcn_readfirstlane((((rstart - dr * (t0l + 1)) % nx) + nx) % nx) * ny;   // step -1
    const unsigned lane_b = (unsigned)rowbase * TS;
    unsigned sbr[PF], ser[KEEP ? PF : 1];
    bool actr[PF];
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        sbr[u] = DCT_OOB;
        if (KEEP) ser[KEEP ? u : 0] = DCT_OOB;
        actr[u] = false;
    }
    T ycar = bc;                                            // lane 0 keeps the boundary value
    T xo = bc, yo = 0, zo = 0;                              // x inflow of a row starts at the boundary value
    // leakage: the y and z outflows of a lane are summed in T (at most nx
    // terms each per lane) and widened at the end; only the wave on the z
    // boundary sums z
    T lyv = 0;
    T lzv = 0;
    const bool zlast_wave = __builtin_amdgcn_readfirstlane(kp) == nz - 1;
    int known_prev = 0, known_next = 0, spins = 0;   // wave-uniform
    typedef decltype(__builtin_amdgcn_raw_buffer_load_b64(rh, 0, 0, 0)) u64v;
    u64v hz = {0u, 0u}, hy = {0u, 0u};
    // prefetch of step t + PF - 1 into the ring slot that step t - 1 consumed
    // (u = t mod PF, a constant once the step loop is unrolled)
    auto prefetch = [&](const int t, const int u) __attribute__((always_inline)) {
        const int tp = t + PF - 1;
        const int ps = (u + PF - 1) % PF;           // constant once the step loop is unrolled
        const bool inp = valid && (unsigned)(tp - t0l) < (unsigned)nx;
        // idle lanes sit on their first or last row, away from the
        // active ones: an out-of-range offset keeps their loads off
        // the memory system (they return 0, never used)
        const unsigned pp = inp ? (unsigned)(rowbase + sre) : DCT_OOB;
        const unsigned pb = inp ? lane_b + (unsigned)sre * TS : DCT_OOB;
        sbr[ps] = pb;
        actr[ps] = inp;
        if (KEEP) ser[KEEP ? ps : 0] = pp;
        qr[ps] = bld_nt<T>(rq, pb);
        sr[ps] = bld<T>(rsg, pb);
        if (ADJ) fr[ADJ ? ps : 0] = __builtin_amdgcn_raw_buffer_load_b8(rmask, pp, 0, 0);
        if (MULTI) {
            // block faces of step t + FD - 1 (only the lanes that take
            // a block face load one) into the slot consumed at that
            // step PF steps earlier
            const int tf = t + FD - 1;
            const bool inf = valid && (unsigned)(tf - t0l) < (unsigned)nx;
            const int ipn = tf - t0l;
            const unsigned yo_off = (inf && ytaker) ? (unsigned)(ipn + nx * kp) * TS : DCT_OOB;
            const unsigned zo_off = (inf && ztaker) ? (unsigned)((ipn + l) * 64 + l) * TS : DCT_OOB;
            const int fs = (u + FD - 1) % PF;
            if (PIPE) {
                yr[MULTI ? fs : 0] = bld_dev<T>(ryi, yo_off);
                zr[MULTI ? fs : 0] = bld_dev<T>(rzi, zo_off);
            } else {
                yr[MULTI ? fs : 0] = bld<T>(ryi, yo_off);
                zr[MULTI ? fs : 0] = bld<T>(rzi, zo_off);
            }
        }
        sre += dny;
        sre = sre == wrap_at_r ? wrap_to_r : sre;
    };
    for (int tb = -PF; tb < NTp; tb += PF) {
        if (PIPE && (bj > 0 || bk > 0)) {
            // this group of steps loads faces up to step tb + PF + FD - 2; the
            // face of step s is written by upstream step s + BK - 1 (z) or
            // s + 63 (y); an upstream block never reports more than its own
            // padded step count
            const int upz = ((nx + nl + a.BK - 2 + PF - 1) / PF) * PF;   // z upstream: same rows, full depth
            const int upy = ((nx + 64 + nw - 2 + PF - 1) / PF) * PF;     // y upstream: 64 rows, same depth
            const int needz = bk > 0 ? min(tb + PF + FD + a.BK + 2, upz) : -(1 << 30);
            const int needy = bj > 0 ? min(tb + PF + FD + 64 + 2, upy) : -(1 << 30);
            for (;;) {
                const int pz = __builtin_amdgcn_readfirstlane(hz[1] == tag ? (int)hz[0] : -(1 << 30));
                const int py = __builtin_amdgcn_readfirstlane(hy[1] == tag ? (int)hy[0] : -(1 << 30));
                if ((pz >= needz && py >= needy) || spins >= DCT_SPIN_LIMIT) break;
                __builtin_amdgcn_s_sleep(4);
                ++spins;
                hz = __builtin_amdgcn_raw_buffer_load_b64(rh, hoff_z, 0, 16);
                hy = __builtin_amdgcn_raw_buffer_load_b64(rh, hoff_y, 0, 16);
            }
            // read ahead for the next group's check
            hz = __builtin_amdgcn_raw_buffer_load_b64(rh, hoff_z, 0, 16);
            hy = __builtin_amdgcn_raw_buffer_load_b64(rh, hoff_y, 0, 16);
        }
        if (!MULTI && tb < 0) {
            // the first PF steps: every lane is idle, only the prefetches run
            // (each with a store that goes nowhere, so the loop is entered
            // with the memory-counter state of the steady state)
#pragma unroll
            for (int u = 0; u < PF; ++u) {
                prefetch(tb + u, u);
                bst(rpsi, DCT_OOB + 64u * u, (T)0);
                if (KEEP) __builtin_amdgcn_raw_buffer_store_b8((unsigned char)0, rmask, DCT_OOB + 64u * u, 0, 0);
            }
            continue;
        }
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            // Step order: the z inflow is requested first; the prefetch of a
            // later step and everything that does not depend on the z inflow
            // follow while it is in flight; a scheduling fence then keeps the
            // short chain that does (cell update, fixup, z handoff) free of
            // unrelated instructions, since a wave issues in program order.
            const int t = tb + u;
            const T qv = qr[u], sv = sr[u];
            const int fv = ADJ ? fr[ADJ ? u : 0] : 0;
            T yface_in = bc, zface_in = bc;
            if (MULTI) {
                yface_in = (jp == 0) ? bc : yr[MULTI ? u : 0];
                zface_in = (kp == 0) ? bc : zr[MULTI ? u : 0];
            }
            const int ip = t - t0l;
            const bool act = actr[u];                       // valid && 0 <= ip < nx
            if (PIPE) {
                // a prefetched face element that was still empty is polled
                // again (rare once the consumer trails its producer)
                bool ywait = act && yreader && is_empty(yface_in);
                bool zwait = act && zreader && is_empty(zface_in);
                while (__builtin_amdgcn_ballot_w64(ywait || zwait) != 0 && spins < DCT_SPIN_LIMIT) {
                    __builtin_amdgcn_s_sleep(2);
                    ++spins;
                    if (ywait) {
                        yface_in = bld_dev<T>(ryi, (unsigned)(ip + nx * kp) * TS);
                        ywait = is_empty(yface_in);
                    }
                    if (zwait) {
                        zface_in = bld_dev<T>(rzi, (unsigned)((ip + l) * 64 + l) * TS);
                        zwait = is_empty(zface_in);
                    }
                }
                // consumed: leave the element empty for the next launch
                bst_dev(ryi, (act && yreader) ? (unsigned)(ip + nx * kp) * TS : DCT_OOB, face_empty<T>());
                bst_dev(rzi, (act && zreader) ? (unsigned)((ip + l) * 64 + l) * TS : DCT_OOB, face_empty<T>());
            }
            // z inflow: wave w-1's outflow of the previous step
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
            } else if (ZROW) {
                zin = zbuf[(t + 1) & 1][w][l];
            } else {
                zin = (w > 0) ? zbuf[(t + 1) & 1][w > 0 ? w - 1 : 0][l] : zface_in;
            }
            __builtin_amdgcn_sched_barrier(0);
            prefetch(t, u);
            // y inflow: lane l-1's outflow of the previous step; lane 0 takes the
            // boundary / block face value through the DPP "old" operand
            T yin;
            if (MULTI) {
                yin = dpp_shift_up_or<T>(yo, yface_in);
            } else {
                ycar = dpp_shift_up_or<T>(yo, ycar);
                yin = ycar;
            }
            const T xin = xo;
            // Everything except the z term: psi_c = (n0 + cz zin) y0 with
            // n0 = q + cx xin + cy yin and y0 = 1 / d (FP64: the reciprocal
            // refined, so the quotient is within a few ulp)
            T n0, y0, zc;
            if (ADJ) {
                const bool ux = !(fv & 1), uy = !(fv & 2), uz = !(fv & 4);
                const T ex = ux ? cx : (T)0, ey = uy ? cy : (T)0, ez = uz ? cz : (T)0;
                y0 = rcp_nr(sv + ex + ey + ez);
                n0 = qv + ex * xin + ey * yin;
                zc = ez;
            } else {
                y0 = rcp_nr(sv + csum);
                n0 = qv + cx * xin + cy * yin;
                zc = cz;
            }
            __builtin_amdgcn_sched_barrier(0);
            Cell4<T> c;
            c.pc = fma(zc, zin, n0) * y0;
            if (ADJ) {
                const bool ux = !(fv & 1), uy = !(fv & 2), uz = !(fv & 4);
                c.xo = ux ? c.pc + c.pc - xin : c.pc;
                c.yo = uy ? c.pc + c.pc - yin : c.pc;
                c.zo = uz ? c.pc + c.pc - zin : c.pc;
                c.fixed = 0;
            } else {
                c.xo = c.pc + c.pc - xin;
                c.yo = c.pc + c.pc - yin;
                c.zo = c.pc + c.pc - zin;
                c.fixed = 0;
                if (fixup && act && fmin(c.xo, fmin(c.yo, c.zo)) < (T)0)
                    c = dd_fixup<T>(qv, sv, cx, cy, cz, xin, yin, zin, c);
            }
            // z handoff first (the next step of wave w+1 waits on it)
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
                zbuf[w][t & (ZR - 1)][l] = c.zo;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
                if (l == 0) lds_st(&prog[w], t + 1);
            } else {
                zbuf[t & 1][ZROW ? w + 1 : w][l] = c.zo;
            }
            __builtin_amdgcn_sched_barrier(0);
            bst_nt(rpsi, sbr[u], c.pc);
            if (KEEP) __builtin_amdgcn_raw_buffer_store_b8((unsigned char)c.fixed, rmask, ser[KEEP ? u : 0], 0, 0);
            if (MULTI) {
                if (PIPE) {
                    bst_dev(ryo, (ywriter && act) ? (unsigned)(ip + nx * kp) * TS : DCT_OOB, c.yo);
                    bst_dev(rzo, (zwriter && act) ? (unsigned)((ip + l) * 64 + l) * TS : DCT_OOB, c.zo);
                } else {
                    bst(ryo, (ywriter && act) ? (unsigned)(ip + nx * kp) * TS : DCT_OOB, c.yo);
                    bst(rzo, (zwriter && act) ? (unsigned)((ip + l) * 64 + l) * TS : DCT_OOB, c.zo);
                }
            }
            lyv += act ? c.yo : (T)0;
            if (zlast_wave) lzv += act ? c.zo : (T)0;
            xo = act ? c.xo : xo;
            yo = c.yo;
            zo = c.zo;
            if (!SYNC) __syncthreads();
            if (PIPE && (u == PF - 1 || u == PF / 2 - 1)) {
                const u64v hv = {(unsigned)(t + 1), tag};
                __builtin_amdgcn_raw_buffer_store_b64(hv, rh, hint_writer ? hoff_self : DCT_OOB, 0, 0);
            }
        }
    }
    if ((SYNC || PIPE) && spins >= DCT_SPIN_LIMIT && l == 0) atomicOr(a.err, 1);
    // boundary outflow sums of this block (for the particle balance): the last
    // x outflow of every row, and the y / z outflows of the boundary rows
    double lx = valid ? (double)xo : 0.0;
    double ly = (valid && ylast) ? (double)lyv : 0.0;
    double lz = (valid && zlast) ? (double)lzv : 0.0;
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

// Layered waves (single block, forward sweep): every wave owns ZL consecutive
// z layers and sweeps them as a skewed pipeline in registers.  Layer z of
// wave w handles reflected x index t - l - (ZL w + z) at step t, the same
// diagonal as one wave per layer, so its z inflow is layer z-1's outflow of
// the previous step (a register) and only the bottom layer of a wave takes
// its inflow from the wave below through LDS.  The ZL cell updates of a step
// are independent, so a wave hides its own latency with them instead of
// relying on several waves per SIMD; one barrier per step couples the
// (fewer) waves.  Each cell's arithmetic is the same as in k_sweep, so the
// results are bitwise the same.
template <typename T, int ZL, int PF, int MODE>
__global__ __launch_bounds__(1024 / ZL) void k_sweep_lw(SweepArgs a)
{
    static_assert(MODE != 2, "the transposed sweep uses k_sweep");
    constexpr bool KEEP = MODE == 1;
    constexpr unsigned TS = sizeof(T);
    __shared__ T zbuf[2][17][64];                            // row w + 1: top layer of wave w; row 0: boundary
    __shared__ double red[3][16];
    const int item = a.b0 * a.N + (int)blockIdx.x;          // this launch's right-hand sides start at b0
    const int b = item / a.N;
    const int n = item - b * a.N;
    if (a.state[b].finished) return;
    const int g = eff_group(a.state[b].g, a.G, a.reverse);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long C = a.C;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nwv = blockDim.x >> 6;
    const double ox = a.dirs[3 * n], oy = a.dirs[3 * n + 1], oz = a.dirs[3 * n + 2];
    const bool sx = ox > 0, sy = oy > 0, sz = oz > 0;
    const int cls = dir_class(ox, oy);
    const T cx = (T)(2.0 * fabs(ox) / a.dx), cy = (T)(2.0 * fabs(oy) / a.dy), cz = (T)(2.0 * fabs(oz) / a.dz);
    const T csum = cx + cy + cz;
    const bool lv = l < ny;                                  // one y block: ny <= 64
    const int j = lv ? (sy ? l : ny - 1 - l) : 0;
    const int jm = j % nx;
    const rsrc_t rq = mk_rsrc((const T *)a.q + (long)item * C, C * TS);
    const rsrc_t rpsi = mk_rsrc((T *)a.psi + ((long)b * a.psi_bs + (long)g * a.psi_gs + n) * C, C * TS);
    const rsrc_t rmask = mk_rsrc(KEEP && a.mask ? a.mask + (((long)b * a.G + g) * a.N + n) * C : nullptr, C);
    const rsrc_t rsg = mk_rsrc((const T *)a.sigc + ((long)cls * a.G + g) * C, C * TS);
    const T bc = a.inflow ? (T)a.inflow[g] : (T)0;
    const int fixup = a.fixup;
    const int NT = nx + min(ny, 64) + nz - 2;
    const int NTp = ((NT + PF - 1) / PF) * PF;
    const int dr = sx ? 1 : -1;
    const int dny = sx ? ny : -ny;
    const int wrap_at_r = (sx ? nx : -1) * ny, wrap_to_r = (sx ? 0 : nx - 1) * ny;
    const int rstart = rot_row(cls, sx ? 0 : nx - 1, jm, nx);
    // per layer: validity, lane part of the offsets, start step, wave-uniform
    // row offset of the prefetched step (step -1 first)
    bool vz[ZL];
    int rowbase[ZL], t0[ZL], sre[ZL];
    bool zlast[ZL];
#pragma unroll
    for (int z = 0; z < ZL; ++z) {
        const int kp = w * ZL + z;
        vz[z] = lv && kp < nz;
        const int k = vz[z] ? (sz ? kp : nz - 1 - kp) : 0;
        rowbase[z] = k * nx * ny + j;
        t0[z] = l + kp;
        sre[z] = __builtin_amdgcn_readfirstlane((((rstart - dr * (t0[z] + 1)) % nx) + nx) % nx) * ny;
        zlast[z] = kp == nz - 1;
    }
    if (w == 0) zbuf[0][0][l] = zbuf[1][0][l] = bc;
    __syncthreads();
    T qr[ZL][PF], sr[ZL][PF];
    unsigned sbr[ZL][PF], ser[KEEP ? ZL : 1][KEEP ? PF : 1];
    bool actr[ZL][PF];
#pragma unroll
    for (int z = 0; z < ZL; ++z)
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            qr[z][u] = sr[z][u] = (T)0;
            sbr[z][u] = DCT_OOB;
            if (KEEP) ser[KEEP ? z : 0][KEEP ? u : 0] = DCT_OOB;
            actr[z][u] = false;
        }
    T ycar[ZL], xo[ZL], yo[ZL], zo[ZL], lyv[ZL];
#pragma unroll
    for (int z = 0; z < ZL; ++z) {
        ycar[z] = xo[z] = bc;
        yo[z] = zo[z] = lyv[z] = (T)0;
    }
    T lzv = 0;
    for (int tb = -PF; tb < NTp; tb += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int t = tb + u;
            // z inflows of this step (outflows of the previous step)
            T zin[ZL];
            zin[0] = zbuf[(t + 1) & 1][w][l];
#pragma unroll
            for (int z = 1; z < ZL; ++z) zin[z] = zo[z - 1];
            __builtin_amdgcn_sched_barrier(0);
            // operands of step t + PF - 1 into the slot step t - 1 consumed
            {
                const int tp = t + PF - 1;
                const int ps = (u + PF - 1) % PF;
#pragma unroll
                for (int z = 0; z < ZL; ++z) {
                    const bool inp = vz[z] && (unsigned)(tp - t0[z]) < (unsigned)nx;
                    const unsigned pb = inp ? (unsigned)(rowbase[z] + sre[z]) * TS : DCT_OOB;
                    sbr[z][ps] = pb;
                    actr[z][ps] = inp;
                    if (KEEP) ser[KEEP ? z : 0][KEEP ? ps : 0] = inp ? (unsigned)(rowbase[z] + sre[z]) : DCT_OOB;
                    qr[z][ps] = bld<T>(rq, pb);
                    sr[z][ps] = bld<T>(rsg, pb);
                    sre[z] += dny;
                    sre[z] = sre[z] == wrap_at_r ? wrap_to_r : sre[z];
                }
            }
            // everything except the z term, for every layer
            T n0[ZL], y0[ZL], yin[ZL], xin[ZL];
#pragma unroll
            for (int z = 0; z < ZL; ++z) {
                ycar[z] = dpp_shift_up_or<T>(yo[z], ycar[z]);
                yin[z] = ycar[z];
                xin[z] = xo[z];
                y0[z] = rcp_nr(sr[z][u] + csum);
                n0[z] = qr[z][u] + cx * xin[z] + cy * yin[z];
            }
            __builtin_amdgcn_sched_barrier(0);
            // the ZL cell updates (independent of each other)
#pragma unroll
            for (int z = 0; z < ZL; ++z) {
                const bool act = actr[z][u];
                Cell4<T> c;
                c.pc = fma(cz, zin[z], n0[z]) * y0[z];
                c.xo = c.pc + c.pc - xin[z];
                c.yo = c.pc + c.pc - yin[z];
                c.zo = c.pc + c.pc - zin[z];
                c.fixed = 0;
                if (fixup && act && fmin(c.xo, fmin(c.yo, c.zo)) < (T)0)
                    c = dd_fixup<T>(qr[z][u], sr[z][u], cx, cy, cz, xin[z], yin[z], zin[z], c);
                if (z == ZL - 1) zbuf[t & 1][w + 1][l] = c.zo;   // z handoff to the wave above
                bst(rpsi, sbr[z][u], c.pc);
                if (KEEP)
                    __builtin_amdgcn_raw_buffer_store_b8((unsigned char)c.fixed, rmask, ser[KEEP ? z : 0][KEEP ? u : 0], 0, 0);
                lyv[z] += act ? c.yo : (T)0;
                if (zlast[z]) lzv += act ? c.zo : (T)0;
                xo[z] = act ? c.xo : xo[z];
                yo[z] = c.yo;
                zo[z] = c.zo;
            }
            __syncthreads();
        }
    }
    // boundary outflow sums (particle balance): last x outflow of every row,
    // y outflows of the last row, z outflows of the top layer
    const bool ylast = l == ny - 1;
    double lx = 0.0, ly = 0.0;
#pragma unroll
    for (int z = 0; z < ZL; ++z) {
        lx += vz[z] ? (double)xo[z] : 0.0;
        ly += (vz[z] && ylast) ? (double)lyv[z] : 0.0;
    }
    double lz = (double)lzv;
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
        a.leak_part[(long)item * a.nblk * 3 + threadIdx.x] = s;
    }
}

// Chained layered waves (single block, forward sweep, no kept fluxes): one
// workgroup sweeps the K consecutive directions n0 .. n0 + K - 1 of one
// octant of one right-hand side back to back.  Lane l of layer kp handles
// the combined index pos = t - l - kp, slot d = pos / nx and reflected x
// index pos mod nx: a lane that finishes direction d's row starts direction
// d + 1's row on the next step, so the fill and drain of the wavefront
// (ny + nz - 2 steps) are paid once per chain instead of once per direction.
// Every upwind neighbour of a cell is in the same slot at the previous step,
// exactly as in k_sweep_lw, so each cell's arithmetic (and result) is the same.
//
// q, psi and sigma_t use the chain layout: the K directions' x extents are
// concatenated into a virtual grid of K nx columns, X = d nx + i (X = (K - 1
// - d) nx + i when Omega_x < 0), rotated like the class layouts with period
// K nx: element (k K nx + (X +- j) mod K nx) ny + j of the chain's block of K
// C elements (+ in class A, - in class B).  The rotated row of a wave step
// is then the same for every lane of every slot, so no per-lane slot offset
// enters the addresses; sigma_t is stored K times over in the same layout.
//
// Per lane, the direction coefficients change when the lane starts a new
// row (l == pos-phase of the step, one lane per step), together with the
// reset of the x inflow.  The boundary outflows of each slot (particle
// balance) are reduced when the last lane starts the next slot.
template <typename T, int ZL, int PF>
__global__ __launch_bounds__(1024 / ZL) void k_sweep_ch(SweepArgs a)
{
    constexpr unsigned TS = sizeof(T);
    __shared__ T zbuf[2][17][64];                            // row w + 1: top layer of wave w; row 0: boundary
    __shared__ T ctab[DCT_MAXCHAIN][4];                      // per slot: c_x, c_y, c_z and their sum
    __shared__ double red[DCT_MAXCHAIN][16][3];              // per slot and z layer: x, y, z outflow sums
    const int K = a.chainK;
    const int cpb = a.N / K;                                 // chains per right-hand side
    const int b = blockIdx.x / cpb;
    const int n0 = (blockIdx.x - b * cpb) * K;
    if (a.state[b].finished) return;
    const int g = eff_group(a.state[b].g, a.G, a.reverse);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int Knx = K * nx;
    const long C = a.C;
    const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const double ox = a.dirs[3 * n0], oy = a.dirs[3 * n0 + 1], oz = a.dirs[3 * n0 + 2];
    const bool sx = ox > 0, sy = oy > 0, sz = oz > 0;
    const int cls = dir_class(ox, oy);
    if ((int)threadIdx.x < K) {
        const int n = n0 + threadIdx.x;
        const T cx = (T)(2.0 * fabs(a.dirs[3 * n]) / a.dx), cy = (T)(2.0 * fabs(a.dirs[3 * n + 1]) / a.dy),
                cz = (T)(2.0 * fabs(a.dirs[3 * n + 2]) / a.dz);
        ctab[threadIdx.x][0] = cx;
        ctab[threadIdx.x][1] = cy;
        ctab[threadIdx.x][2] = cz;
        ctab[threadIdx.x][3] = cx + cy + cz;
    }
    for (int i = threadIdx.x; i < DCT_MAXCHAIN * 16 * 3; i += blockDim.x) (&red[0][0][0])[i] = 0.0;
    const bool lv = l < ny;                                  // one y block: ny <= 64
    const int nl = min(ny, 64);
    const int j = lv ? (sy ? l : ny - 1 - l) : 0;
    const rsrc_t rq = mk_rsrc((const T *)a.q + ((long)b * a.N + n0) * C, (long)K * C * TS);
    const rsrc_t rpsi = mk_rsrc((T *)a.psi + ((long)b * a.psi_bs + (long)g * a.psi_gs + n0) * C, (long)K * C * TS);
    const rsrc_t rsg = mk_rsrc((const T *)a.sigch + ((long)cls * a.G + g) * K * C, (long)K * C * TS);
    const T bc = a.inflow ? (T)a.inflow[g] : (T)0;
    const int fixup = a.fixup;
    // one step more than the wavefront needs: the last lane's slot change
    // after the final row closes the last slot's outflow sums
    const int NT = Knx + nl + nz - 1;
    const int NTp = ((NT + PF - 1) / PF) * PF;
    const int dr = sx ? 1 : -1;
    const int dny = sx ? ny : -ny;
    const int wrap_at_r = (sx ? Knx : -1) * ny, wrap_to_r = (sx ? 0 : Knx - 1) * ny;
    // chain row of the lane's first cell (slot 0, first x of the sweep)
    int rs = (sx ? 0 : Knx - 1) + (cls == 0 ? j : -j);
    rs = ((rs % Knx) + Knx) % Knx;
    bool vz[ZL];
    int rowbase[ZL], t0[ZL], sre[ZL], Rz[ZL], Dz[ZL];
#pragma unroll
    for (int z = 0; z < ZL; ++z) {
        const int kp = w * ZL + z;
        vz[z] = lv && kp < nz;
        const int k = vz[z] ? (sz ? kp : nz - 1 - kp) : 0;
        rowbase[z] = k * Knx * ny + j;
        t0[z] = l + kp;
        sre[z] = __builtin_amdgcn_readfirstlane((((rs - dr * (t0[z] + 1)) % Knx) + Knx) % Knx) * ny;
        // phase of the compute step t = -PF (floor division by nx): the lane
        // with l == Rz starts slot Dz's row at that step
        const int sp = -PF - kp;
        const int dfl = (sp >= 0) ? sp / nx : -((-sp + nx - 1) / nx);
        Rz[z] = sp - dfl * nx;
        Dz[z] = dfl;
    }
    if (w == 0) zbuf[0][0][l] = zbuf[1][0][l] = bc;
    __syncthreads();
    T qr[ZL][PF], sr[ZL][PF];
    unsigned sbr[ZL][PF];
    bool actr[ZL][PF];
#pragma unroll
    for (int z = 0; z < ZL; ++z)
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            qr[z][u] = sr[z][u] = (T)0;
            sbr[z][u] = DCT_OOB;
            actr[z][u] = false;
        }
    T ycar[ZL], xo[ZL], yo[ZL], zo[ZL], lyv[ZL], lxv[ZL], cxl[ZL], cyl[ZL], czl[ZL], csl[ZL];
#pragma unroll
    for (int z = 0; z < ZL; ++z) {
        ycar[z] = xo[z] = lxv[z] = bc;
        yo[z] = zo[z] = lyv[z] = (T)0;
        cxl[z] = ctab[0][0];
        cyl[z] = ctab[0][1];
        czl[z] = ctab[0][2];
        csl[z] = ctab[0][3];
    }
    T lzv = 0, lzp = 0;                                      // top layer: z outflows of the current / previous row
    const int top_w = (nz - 1) / ZL, top_z = (nz - 1) - top_w * ZL;
    for (int tb = -PF; tb < NTp; tb += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int t = tb + u;
            T zin[ZL];
            zin[0] = zbuf[(t + 1) & 1][w][l];
#pragma unroll
            for (int z = 1; z < ZL; ++z) zin[z] = zo[z - 1];
            __builtin_amdgcn_sched_barrier(0);
            {
                const int tp = t + PF - 1;
                const int ps = (u + PF - 1) % PF;
#pragma unroll
                for (int z = 0; z < ZL; ++z) {
                    const bool inp = vz[z] && (unsigned)(tp - t0[z]) < (unsigned)Knx;
                    const unsigned pb = inp ? (unsigned)(rowbase[z] + sre[z]) * TS : DCT_OOB;
                    sbr[z][ps] = pb;
                    actr[z][ps] = inp;
                    qr[z][ps] = bld<T>(rq, pb);
                    sr[z][ps] = bld<T>(rsg, pb);
                    sre[z] += dny;
                    sre[z] = sre[z] == wrap_at_r ? wrap_to_r : sre[z];
                }
            }
            // slot changes: the lane with l == Rz starts slot Dz's row now
            // (its x inflow is the boundary value, its coefficients those of
            // the new direction); its previous row's last x outflow is kept
            // for the balance
            bool start[ZL];
            T n0v[ZL], y0[ZL], yin[ZL], xin[ZL];
#pragma unroll
            for (int z = 0; z < ZL; ++z) {
                start[z] = l == Rz[z];
                const int dc = min(max(Dz[z], 0), K - 1);
                const T ncx = ctab[dc][0], ncy = ctab[dc][1], ncz = ctab[dc][2], ncs = ctab[dc][3];
                cxl[z] = start[z] ? ncx : cxl[z];
                cyl[z] = start[z] ? ncy : cyl[z];
                czl[z] = start[z] ? ncz : czl[z];
                csl[z] = start[z] ? ncs : csl[z];
                lxv[z] = start[z] ? xo[z] : lxv[z];
                xin[z] = start[z] ? bc : xo[z];
                ycar[z] = dpp_shift_up_or<T>(yo[z], ycar[z]);
                yin[z] = ycar[z];
                y0[z] = rcp_nr(sr[z][u] + csl[z]);
                n0v[z] = qr[z][u] + cxl[z] * xin[z] + cyl[z] * yin[z];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int z = 0; z < ZL; ++z) {
                const int kp = w * ZL + z;
                // the last lane starts slot Dz: every lane of this layer has
                // finished slot Dz - 1, whose boundary outflows are summed now
                if (Rz[z] == nl - 1 && Dz[z] >= 1 && Dz[z] <= K && kp < nz) {
                    const bool top = w == top_w && z == top_z;
                    if (top) lzp = start[z] ? lzv : lzp;
                    double sx_ = vz[z] ? (double)lxv[z] : 0.0;
                    double sz_ = (top && vz[z]) ? (double)lzp : 0.0;
                    for (int o = 32; o > 0; o >>= 1) {
                        sx_ += __shfl_down(sx_, o, 64);
                        sz_ += __shfl_down(sz_, o, 64);
                    }
                    const double sy_ = (double)__shfl(lyv[z], nl - 1, 64);
                    if (l == 0) {
                        red[Dz[z] - 1][kp][0] = sx_;
                        red[Dz[z] - 1][kp][1] = sy_;
                        red[Dz[z] - 1][kp][2] = sz_;
                    }
                    lyv[z] = (T)0;
                    if (top) {
                        lzv = start[z] ? (T)0 : lzv;
                        lzp = (T)0;
                    }
                } else if (w == top_w && z == top_z) {
                    lzp = start[z] ? lzv : lzp;
                    lzv = start[z] ? (T)0 : lzv;
                }
                const bool act = actr[z][u];
                Cell4<T> c;
                c.pc = fma(czl[z], zin[z], n0v[z]) * y0[z];
                c.xo = c.pc + c.pc - xin[z];
                c.yo = c.pc + c.pc - yin[z];
                c.zo = c.pc + c.pc - zin[z];
                c.fixed = 0;
                if (fixup && act && fmin(c.xo, fmin(c.yo, c.zo)) < (T)0)
                    c = dd_fixup<T>(qr[z][u], sr[z][u], cxl[z], cyl[z], czl[z], xin[z], yin[z], zin[z], c);
                if (z == ZL - 1) zbuf[t & 1][w + 1][l] = c.zo;   // z handoff to the wave above
                bst(rpsi, sbr[z][u], c.pc);
                lyv[z] += act ? c.yo : (T)0;
                if (w == top_w && z == top_z) lzv += act ? c.zo : (T)0;
                xo[z] = act ? c.xo : xo[z];
                yo[z] = c.yo;
                zo[z] = c.zo;
                // next step's phase
                ++Rz[z];
                if (Rz[z] == nx) {
                    Rz[z] = 0;
                    ++Dz[z];
                }
            }
            __syncthreads();
        }
    }
    __syncthreads();
    // boundary outflow sums of every slot, summed over the z layers in order
    if ((int)threadIdx.x < 3 * K) {
        const int d = threadIdx.x / 3, cc = threadIdx.x - 3 * d;
        double s = 0.0;
        for (int kp = 0; kp < nz; ++kp) s += red[d][kp][cc];
        a.leak_part[((long)b * a.N + n0 + d) * a.nblk * 3 + cc] = s;
    }
}

// Source-chained layered waves (single block, forward sweep, no kept
// fluxes): one workgroup sweeps direction n for up to K right-hand sides back
// to back, the unfinished ones dealt to the ceil(B / K) chains of the
// direction round robin (so a chain shortens as sources finish).  As in k_sweep_lw, lane l of layer kp handles
// the combined index pos = t - l - kp at step t; here slot d = pos / nx is the
// d-th right-hand side of the chain and pos mod nx the reflected x index, so
// a lane that finishes a source's row starts the next source's row on the
// next step and the fill and drain of the wavefront (ny + nz - 2 steps) are
// paid once per chain.  Every upwind neighbour of a cell is in the same slot
// at the previous step, and each cell's arithmetic is that of k_sweep_lw, so
// the angular fluxes are bitwise the same.
//
// All sources share the direction, hence its coefficients and its class
// rotation: the rotated row of a wave step, (i +- j) mod nx, does not depend
// on the slot, so q, psi and sigma_t keep their class layouts and a lane only
// adds its slot's base offset (q and psi of (b, n); sigma_t of b's group),
// switched when it starts a new row.  Offsets are 32-bit: the host launches
// this kernel only while B N C sizeof(T) <= 2^31 (and nx >= PF, ny <= nx).
//
// Step bookkeeping is per wave: with ph = (t - ZL w) mod nx and slot sl =
// (t - ZL w) div nx at compute step t, the lane starting a row in layer z is
// (ph - z) mod nx, in slot sl or sl - 1; the load of step t + PF - 1 is
// PF - 1 further on, in slot sl or sl + 1, whose bases are kept
// wave-uniform and refreshed when ph wraps.  The boundary
// outflows of a row (its last x outflow; the y outflows of the last row; the
// z outflows of the top layer) are written by its lane into an LDS table per
// slot when the lane starts its next row, and summed in a fixed order at the
// end (particle balance); the inflow boundary value is zero (no test inflow).
template <typename T, int ZL, int PF>
__global__ __launch_bounds__(1024 / ZL) void k_sweep_rc(SweepArgs a)
{
    constexpr unsigned TS = sizeof(T);
    __shared__ T zbuf[2][17][64];                            // row w + 1: top layer of wave w; row 0: boundary
    __shared__ T ox_t[DCT_MAXRC + 1][16][64];                // per slot, z layer, lane: last x outflow of the row
    __shared__ T oy_t[DCT_MAXRC + 1][16];                    // per slot, z layer: y outflows of the last row
    __shared__ T oz_t[DCT_MAXRC + 1][64];                    // per slot, lane: z outflows of the top layer's row
    __shared__ int slot_b[DCT_MAXRC];                        // right-hand side of each slot
    __shared__ unsigned tab_q[DCT_MAXRC + 2], tab_s[DCT_MAXRC + 2];  // byte offsets (index d + 1 for slot d)
    __shared__ int kc_sh;
    const int K = a.rhsK;
    const int N = a.N;
    const int c = blockIdx.x / N;
    const int n = blockIdx.x - c * N;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long C = a.C;
    const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const double ox = a.dirs[3 * n], oy = a.dirs[3 * n + 1], oz = a.dirs[3 * n + 2];
    const bool sx = ox > 0, sy = oy > 0, sz = oz > 0;
    const int cls = dir_class(ox, oy);
    if (w == 0) {
        // the unfinished right-hand sides in order (ballot per 64), dealt to
        // the chains round robin: the s-th goes to chain s mod nch, slot
        // s div nch, so every chain stays busy as sources finish
        const int nch = gridDim.x / N;
        const int bend = a.b0 + (a.nb > 0 ? a.nb : a.B);      // this launch's right-hand sides: b0 .. bend - 1
        int before = 0;
        for (int base = a.b0; base < bend; base += 64) {
            const int b = base + l;
            const bool act = b < bend && !a.state[b].finished;
            const unsigned long long m = __ballot(act);
            const int s = before + __popcll(m & ((1ull << l) - 1ull));
            if (act && s % nch == c && s / nch < K) slot_b[s / nch] = b;
            before += __popcll(m);
        }
        if (l == 0) kc_sh = min(K, (before - c + nch - 1) / nch);
    }
    __syncthreads();
    const int Kc = kc_sh;
    if (Kc <= 0) return;
    if ((int)threadIdx.x < Kc + 2) {
        // slot d at index d + 1; the indices before and after repeat the ends
        const int d = min(max((int)threadIdx.x - 1, 0), Kc - 1), b = slot_b[d];
        const int g = eff_group(a.state[b].g, a.G, a.reverse);
        tab_q[threadIdx.x] = (unsigned)(((long)b * N + n) * C * TS);
        tab_s[threadIdx.x] = (unsigned)(((long)cls * a.G + g) * C * TS);
    }
    const T cx = (T)(2.0 * fabs(ox) / a.dx), cy = (T)(2.0 * fabs(oy) / a.dy), cz = (T)(2.0 * fabs(oz) / a.dz);
    const T csum = cx + cy + cz;
    const bool lv = l < ny;                                  // one y block: ny <= 64
    const int nl = min(ny, 64);
    const int j = lv ? (sy ? l : ny - 1 - l) : 0;
    const int jm = j % nx;
    const rsrc_t rq = mk_rsrc(a.q, (long)a.B * N * C * TS);
    const rsrc_t rpsi = mk_rsrc(a.psi, (long)a.B * N * C * TS);
    const rsrc_t rsg = mk_rsrc(a.sigc, 2L * a.G * C * TS);
    const T bc = (T)0;
    const int fixup = a.fixup;
    // one step more than the wavefront needs: every lane of every layer
    // starts the (empty) slot after the last, which records its last row
    const int Knx = Kc * nx;
    const int NT = Knx + nl + nz - 1;
    const int NTp = ((NT + PF - 1) / PF) * PF;
    const int dr = sx ? 1 : -1;
    const int dny = sx ? ny : -ny;
    const int wrap_at_r = (sx ? nx : -1) * ny, wrap_to_r = (sx ? 0 : nx - 1) * ny;
    const int rstart = rot_row(cls, sx ? 0 : nx - 1, jm, nx);
    const int top_w = (nz - 1) / ZL, top_z = (nz - 1) - top_w * ZL;
    __syncthreads();
    bool vz[ZL];
    int rowbase[ZL], t0[ZL], sre[ZL];
    unsigned lq[ZL], ls[ZL];
#pragma unroll
    for (int z = 0; z < ZL; ++z) {
        const int kp = w * ZL + z;
        vz[z] = lv && kp < nz;
        const int k = vz[z] ? (sz ? kp : nz - 1 - kp) : 0;
        rowbase[z] = k * nx * ny + j;
        t0[z] = l + kp;
        sre[z] = __builtin_amdgcn_readfirstlane((((rstart - dr * (t0[z] + 1)) % nx) + nx) % nx) * ny;
        lq[z] = tab_q[1];
        ls[z] = tab_s[1];
    }
    // wave phase at the first compute step t = -PF
    const int p0 = -PF - w * ZL;
    int sl = (p0 >= 0) ? p0 / nx : -((-p0 + nx - 1) / nx);
    int ph = p0 - sl * nx;
    auto tabq = [&](int d) { return tab_q[min(max(d, -1), Kc) + 1]; };
    auto tabs = [&](int d) { return tab_s[min(max(d, -1), Kc) + 1]; };
    unsigned bq_0 = tabq(sl), bq_p = tabq(sl + 1);
    unsigned bs_0 = tabs(sl), bs_p = tabs(sl + 1);
    if (w == 0) zbuf[0][0][l] = zbuf[1][0][l] = bc;
    __syncthreads();
    T qr[ZL][PF], sr[ZL][PF];
    unsigned sbr[ZL][PF];
    bool actr[ZL][PF];
#pragma unroll
    for (int z = 0; z < ZL; ++z)
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            qr[z][u] = sr[z][u] = (T)0;
            sbr[z][u] = DCT_OOB;
            actr[z][u] = false;
        }
    T ycar[ZL], xo[ZL], yo[ZL], zo[ZL], lyv[ZL];
#pragma unroll
    for (int z = 0; z < ZL; ++z) {
        ycar[z] = xo[z] = bc;
        yo[z] = zo[z] = lyv[z] = (T)0;
    }
    T lzv = 0;                                               // top layer: z outflows of the lane's current row
    for (int tb = -PF; tb < NTp; tb += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int t = tb + u;
            T zin[ZL];
            zin[0] = zbuf[(t + 1) & 1][w][l];
#pragma unroll
            for (int z = 1; z < ZL; ++z) zin[z] = zo[z - 1];
            __builtin_amdgcn_sched_barrier(0);
            // operands of step t + PF - 1 into the slot step t - 1 consumed;
            // the lane starting a row there takes its slot's bases first
            {
                const int ps = (u + PF - 1) % PF;
#pragma unroll
                for (int z = 0; z < ZL; ++z) {
                    // layer z at the load: the starting lane is ph - z + PF - 1
                    // (>= 0 as z < PF), in slot sl, or sl + 1 past nx (nx >= PF)
                    const int x = ph - z + PF - 1;
                    const bool hi = x >= nx;
                    const unsigned nq = hi ? bq_p : bq_0;
                    const unsigned ns = hi ? bs_p : bs_0;
                    const bool st = l == (hi ? x - nx : x);
                    lq[z] = st ? nq : lq[z];
                    ls[z] = st ? ns : ls[z];
                    const bool inp = vz[z] && (unsigned)(t + PF - 1 - t0[z]) < (unsigned)Knx;
                    const unsigned cell = (unsigned)(rowbase[z] + sre[z]) * TS;
                    const unsigned pb = inp ? lq[z] + cell : DCT_OOB;
                    const unsigned sb = inp ? ls[z] + cell : DCT_OOB;
                    sbr[z][ps] = pb;
                    actr[z][ps] = inp;
                    qr[z][ps] = bld<T>(rq, pb);
                    sr[z][ps] = bld<T>(rsg, sb);
                    sre[z] += dny;
                    sre[z] = sre[z] == wrap_at_r ? wrap_to_r : sre[z];
                }
            }
            // a lane starting a row takes the boundary x inflow and records
            // the outflows of its previous row (slot d - 1) for the balance
            bool start[ZL];
            T n0v[ZL], y0[ZL], yin[ZL], xin[ZL];
#pragma unroll
            for (int z = 0; z < ZL; ++z) {
                const int kp = w * ZL + z;
                const bool lo = ph < z;
                const int cph = lo ? ph - z + nx : ph - z;
                const int d = lo ? sl - 1 : sl;              // slot of the starting lane
                start[z] = l == cph;
                const bool rec = start[z] && d >= 1 && d <= Kc && vz[z];
                const int dd = rec ? d - 1 : DCT_MAXRC;      // row DCT_MAXRC takes the lanes that record nothing
                ox_t[dd][kp][l] = xo[z];
                if (l == nl - 1) oy_t[dd][kp] = lyv[z];
                if (w == top_w && z == top_z) {
                    oz_t[dd][l] = lzv;
                    lzv = start[z] ? (T)0 : lzv;
                }
                lyv[z] = start[z] ? (T)0 : lyv[z];
                xin[z] = start[z] ? bc : xo[z];
                ycar[z] = dpp_shift_up_or<T>(yo[z], ycar[z]);
                yin[z] = ycar[z];
                y0[z] = rcp_nr(sr[z][u] + csum);
                n0v[z] = qr[z][u] + cx * xin[z] + cy * yin[z];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int z = 0; z < ZL; ++z) {
                const bool act = actr[z][u];
                Cell4<T> cc;
                cc.pc = fma(cz, zin[z], n0v[z]) * y0[z];
                cc.xo = cc.pc + cc.pc - xin[z];
                cc.yo = cc.pc + cc.pc - yin[z];
                cc.zo = cc.pc + cc.pc - zin[z];
                cc.fixed = 0;
                if (fixup && act && fmin(cc.xo, fmin(cc.yo, cc.zo)) < (T)0)
                    cc = dd_fixup<T>(qr[z][u], sr[z][u], cx, cy, cz, xin[z], yin[z], zin[z], cc);
                if (z == ZL - 1) zbuf[t & 1][w + 1][l] = cc.zo;   // z handoff to the wave above
                bst(rpsi, sbr[z][u], cc.pc);
                lyv[z] += act ? cc.yo : (T)0;
                if (w == top_w && z == top_z) lzv += act ? cc.zo : (T)0;
                xo[z] = act ? cc.xo : xo[z];
                yo[z] = cc.yo;
                zo[z] = cc.zo;
            }
            // next step's phase; the slot bases follow the slot
            if (++ph == nx) {
                ph = 0;
                ++sl;
                bq_0 = bq_p;
                bq_p = tabq(sl + 1);
                bs_0 = bs_p;
                bs_p = tabs(sl + 1);
            }
            __syncthreads();
        }
    }
    // boundary outflow sums of every slot, in a fixed order (layers, then lanes)
    if ((int)threadIdx.x < 3 * Kc) {
        const int d = threadIdx.x / 3, cc = threadIdx.x - 3 * d;
        double s = 0.0;
        if (cc == 0) {
            for (int kp = 0; kp < nz; ++kp)
                for (int q = 0; q < nl; ++q) s += (double)ox_t[d][kp][q];
        } else if (cc == 1) {
            for (int kp = 0; kp < nz; ++kp) s += (double)oy_t[d][kp];
        } else {
            for (int q = 0; q < nl; ++q) s += (double)oz_t[d][q];
        }
        a.leak_part[((long)slot_b[d] * N + n) * a.nblk * 3 + cc] = s;
    }
}

hipError_t launch_sweep(SweepArgs a, int is_f64, hipStream_t s, unsigned seq)
{
    a.seq = seq;
    const int NBJ = a.NBJ, NBK = a.NBK;
    const bool multi = NBJ > 1 || NBK > 1;
    const bool pipe = a.pipe && multi;
    dim3 grid, block(64 * a.BK);
    if (pipe) {
        const long nitems = (long)a.B * a.N;
        grid = dim3((unsigned)(8 * ((nitems + 7) / 8) * a.nblk));
    } else {
        int lo = max(0, a.diag - (NBK - 1));
        int hi = min(a.diag, NBJ - 1);
        grid = dim3((unsigned)(a.B * a.N), (unsigned)(hi - lo + 1));
    }
    const int mode = a.adjoint ? 2 : (a.mask ? 1 : 0);
    // a launch over a subset of the right-hand sides: layered waves or chained sources
    const int nb = a.nb > 0 ? a.nb : a.B;
    const bool layered = (a.layers == 2 || a.layers == 4) && !multi && mode != 2 && a.ny <= 64 && a.nz <= 16;
    if (a.b0 < 0 || a.b0 + nb > a.B || ((a.b0 != 0 || nb != a.B) && (a.chainK > 1 || !(a.rhsK > 1 || layered))))
        return hipErrorInvalidValue;
    if (a.chainK > 1) {
        // chained directions: one block, forward sweep without kept fluxes,
        // ny <= nx, K divides N (checked by the host)
        if (multi || mode != 0 || a.ny > 64 || a.nz > 16 || a.ny > a.nx || a.N % a.chainK != 0 ||
            a.chainK > DCT_MAXCHAIN)
            return hipErrorInvalidValue;
        const int zl = a.layers == 2 || a.layers == 4 ? a.layers : 1;
        const int nwv = (a.nz + zl - 1) / zl;
        const dim3 cgrid((unsigned)(a.B * (a.N / a.chainK))), cblock(64 * nwv);
#define DCT_CH(T, ZL) hipLaunchKernelGGL((k_sweep_ch<T, ZL, 8>), cgrid, cblock, 0, s, a)
        if (is_f64) {
            if (zl == 4) DCT_CH(double, 4); else if (zl == 2) DCT_CH(double, 2); else DCT_CH(double, 1);
        } else {
            if (zl == 4) DCT_CH(float, 4); else if (zl == 2) DCT_CH(float, 2); else DCT_CH(float, 1);
        }
#undef DCT_CH
        return hipGetLastError();
    }
    if (a.rhsK > 1) {
        // chained sources: one block, forward sweep without kept fluxes or test
        // inflow, ny <= nx, 32-bit offsets (checked by the host)
        if (multi || mode != 0 || a.ny > 64 || a.nz > 16 || a.ny > a.nx || a.nx < 8 || a.rhsK > DCT_MAXRC || a.inflow ||
            a.psi_bs != a.N || a.psi_gs != 0 || (long)a.B * a.N * a.C * (is_f64 ? 8 : 4) > (1L << 31))
            return hipErrorInvalidValue;
        const int zl = a.layers == 2 ? 2 : 1;
        const int nwv = (a.nz + zl - 1) / zl;
        const dim3 rgrid((unsigned)(a.N * ((nb + a.rhsK - 1) / a.rhsK))), rblock(64 * nwv);
#define DCT_RC(T, ZL) hipLaunchKernelGGL((k_sweep_rc<T, ZL, 8>), rgrid, rblock, 0, s, a)
        if (is_f64) {
            if (zl == 2) DCT_RC(double, 2); else DCT_RC(double, 1);
        } else {
            if (zl == 2) DCT_RC(float, 2); else DCT_RC(float, 1);
        }
#undef DCT_RC
        return hipGetLastError();
    }
    if (layered) {
        const int nwv = (a.nz + a.layers - 1) / a.layers;
        const dim3 lgrid((unsigned)(nb * a.N)), lblock(64 * nwv);
        // operands prefetched 4 steps ahead: at 2 layers per wave that holds 69
        // VGPRs instead of 110 with 8 steps, so three workgroups fit a CU instead
        // of two, and the sweep of the 36-source scan runs 4% faster (332 against
        // 346 us); 2 steps (49 VGPRs) and 6 (89) were slower
#define DCT_LW(T, ZL, MD) hipLaunchKernelGGL((k_sweep_lw<T, ZL, 4, MD>), lgrid, lblock, 0, s, a)
        if (is_f64) {
            if (a.layers == 4) { if (mode == 1) DCT_LW(double, 4, 1); else DCT_LW(double, 4, 0); }
            else { if (mode == 1) DCT_LW(double, 2, 1); else DCT_LW(double, 2, 0); }
        } else {
            if (a.layers == 4) { if (mode == 1) DCT_LW(float, 4, 1); else DCT_LW(float, 4, 0); }
            else { if (mode == 1) DCT_LW(float, 2, 1); else DCT_LW(float, 2, 0); }
        }
#undef DCT_LW
        return hipGetLastError();
    }
#define DCT_LAUNCH_SWEEP(T, PF, M, S, MD, P) hipLaunchKernelGGL((k_sweep<T, PF, M, S, MD, P>), grid, block, 0, s, a)
#define DCT_LAUNCH_SWEEP_M(T, PF, M, S, P)                   \
    do {                                                     \
        if (mode == 2) DCT_LAUNCH_SWEEP(T, PF, M, S, 2, P);   \
        else if (mode == 1) DCT_LAUNCH_SWEEP(T, PF, M, S, 1, P); \
        else DCT_LAUNCH_SWEEP(T, PF, M, S, 0, P);             \
    } while (0)
#define DCT_LAUNCH_SWEEP_S(T, PF, M) \
    do { if (a.sync) DCT_LAUNCH_SWEEP_M(T, PF, M, 1, false); else DCT_LAUNCH_SWEEP_M(T, PF, M, 0, false); } while (0)
    if (pipe) {
        // pipelined blocks keep one barrier per step inside the workgroup
        if (is_f64) DCT_LAUNCH_SWEEP_M(double, 4, true, 0, true);
        else DCT_LAUNCH_SWEEP_M(float, 8, true, 0, true);
    } else if (is_f64) {
        if (multi) DCT_LAUNCH_SWEEP_S(double, 4, true); else DCT_LAUNCH_SWEEP_S(double, 8, false);
    } else {
        if (multi) DCT_LAUNCH_SWEEP_S(float, 8, true); else DCT_LAUNCH_SWEEP_S(float, 8, false);
    }
#undef DCT_LAUNCH_SWEEP_S
#undef DCT_LAUNCH_SWEEP_M
#undef DCT_LAUNCH_SWEEP
    return hipGetLastError();
}

}  // namespace dct
