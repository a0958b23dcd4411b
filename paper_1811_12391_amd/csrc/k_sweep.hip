// Diamond-difference transport sweep (eq. 2 on voxels, vacuum or prescribed
// isotropic inflow), one workgroup per (source, direction, block), as a
// diagonal wavefront:
//
//   - a workgroup owns up to 64 y-rows (lanes) x up to 16 z-layers (waves) of
//     one block and walks x; at step t, lane l of wave w handles the cell with
//     reflected x index i' = t - l - w, so all its upwind neighbours were
//     computed at step t-1;
//   - the x face stays in a register (same lane, previous step), the y face
//     comes from lane l-1 by a cross-lane shuffle, the z face from wave w-1
//     through a double-buffered LDS slot, with one workgroup barrier per step;
//   - faces crossing a block boundary go through small global buffers and the
//     blocks of a sweep run as a sequence of block diagonals (KBA ordering);
//   - q, sigma_t and psi live in the class-rotated layout, so the 64 lanes of
//     a wave step read and write 64 consecutive elements; the loads of step
//     t + PF are issued at step t.
//
// Cell update: with c_a = 2|Omega_a|/Delta_a,
//   psi_c = (q + sum_a c_a in_a) / (sigma + sum_a c_a),  out_a = 2 psi_c - in_a;
// a negative outgoing face is set to zero and psi_c recomputed from the cell
// balance without that face's diamond relation (its inflow then enters with
// weight c_a / 2), repeating while new negative faces appear.
#include "dct_internal.h"

namespace dct {

template <typename T>
__device__ inline void dd_cell(T qv, T sv, T cx, T cy, T cz, T csum, T xin, T yin, T zin, int fixup, T &pc,
                               T &xo, T &yo, T &zo)
{
    T num = qv + cx * xin + cy * yin + cz * zin;
    pc = num / (sv + csum);
    xo = pc + pc - xin;
    yo = pc + pc - yin;
    zo = pc + pc - zin;
    if (fixup && (xo < (T)0 || yo < (T)0 || zo < (T)0)) {
        bool fx = false, fy = false, fz = false;
        for (int pass = 0; pass < 3; ++pass) {
            bool fresh = false;
            if (!fx && xo < (T)0) { fx = true; fresh = true; }
            if (!fy && yo < (T)0) { fy = true; fresh = true; }
            if (!fz && zo < (T)0) { fz = true; fresh = true; }
            if (!fresh) break;
            T n2 = qv, d2 = sv;
            if (fx) n2 += (T)0.5 * cx * xin; else { n2 += cx * xin; d2 += cx; }
            if (fy) n2 += (T)0.5 * cy * yin; else { n2 += cy * yin; d2 += cy; }
            if (fz) n2 += (T)0.5 * cz * zin; else { n2 += cz * zin; d2 += cz; }
            pc = n2 / d2;
            xo = fx ? (T)0 : pc + pc - xin;
            yo = fy ? (T)0 : pc + pc - yin;
            zo = fz ? (T)0 : pc + pc - zin;
        }
    }
}

template <typename T, int PF>
__global__ __launch_bounds__(1024) void k_sweep(SweepArgs a)
{
    __shared__ T zbuf[2][16][64];
    __shared__ double red[3][16];
    const int item = blockIdx.x;
    const int b = item / a.N;
    const int n = item - b * a.N;
    if (a.state[b].finished) return;
    const int g = a.state[b].g;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long C = a.C;
    const int bj = max(0, a.diag - (a.NBK - 1)) + (int)blockIdx.y;
    const int bk = a.diag - bj;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double ox = a.dirs[3 * n], oy = a.dirs[3 * n + 1], oz = a.dirs[3 * n + 2];
    const bool sx = ox > 0, sy = oy > 0, sz = oz > 0;
    const int cls = dir_class(ox, oy);
    const T cx = (T)(2.0 * fabs(ox) / a.dx), cy = (T)(2.0 * fabs(oy) / a.dy), cz = (T)(2.0 * fabs(oz) / a.dz);
    const T csum = cx + cy + cz;
    const int jp = bj * 64 + l, kp = bk * a.BK + w;
    const int nl = min(64, ny - bj * 64), nw = min(a.BK, nz - bk * a.BK);
    const bool valid = l < nl && w < nw;
    const int j = valid ? (sy ? jp : ny - 1 - jp) : 0;
    const int k = valid ? (sz ? kp : nz - 1 - kp) : 0;
    const int jm = j % nx;
    const long rowbase = (long)k * nx * ny + j;
    const T *qb = (const T *)a.q + (long)item * C;
    T *pb = (T *)a.psi + (long)item * C;
    const T *sg = (const T *)a.sigc + ((long)cls * a.G + g) * C;
    T *yf = (T *)a.yface + (long)item * nx * nz;
    T *zf = (T *)a.zface + (long)item * nx * ny;
    const T bc = a.inflow ? (T)a.inflow[g] : (T)0;
    const int fixup = a.fixup;
    const int NT = nx + nl + nw - 2;

    // prefetch ring: slot u holds step t0 + u
    T qr[PF], sr[PF];
    auto pos_of = [&](int t, bool &act) -> long {
        int ip = t - l - w;
        act = valid && ip >= 0 && ip < nx;
        int i = sx ? ip : nx - 1 - ip;
        int r = rot_row(cls, act ? i : 0, jm, nx);
        return rowbase + (long)r * ny;
    };
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        bool act;
        long pos = pos_of(u, act);
        qr[u] = act ? qb[pos] : (T)0;
        sr[u] = act ? sg[pos] : (T)0;
    }
    T xo = 0, yo = 0, zo = 0;
    double lx = 0.0, ly = 0.0, lz = 0.0;
    for (int t0 = 0; t0 < NT; t0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int t = t0 + u;
            if (t < NT) {
                const T qv = qr[u], sv = sr[u];
                {
                    bool actn;
                    long posn = pos_of(t + PF, actn);
                    actn = actn && (t + PF < NT);
                    qr[u] = actn ? qb[posn] : (T)0;
                    sr[u] = actn ? sg[posn] : (T)0;
                }
                bool act;
                const long pos = pos_of(t, act);
                const int ip = t - l - w;
                T yin = __shfl_up(yo, 1, 64);
                if (l == 0) yin = (jp == 0) ? bc : (act ? yf[ip + nx * kp] : (T)0);
                T zin;
                if (w == 0) zin = (kp == 0) ? bc : (act ? zf[ip + nx * jp] : (T)0);
                else zin = zbuf[(t + 1) & 1][w - 1][l];
                const T xin = (ip == 0) ? bc : xo;
                if (act) {
                    T pc, ax_, ay_, az_;
                    dd_cell<T>(qv, sv, cx, cy, cz, csum, xin, yin, zin, fixup, pc, ax_, ay_, az_);
                    pb[pos] = pc;
                    if (ip == nx - 1) lx += (double)ax_;
                    if (jp == ny - 1) ly += (double)ay_;
                    if (kp == nz - 1) lz += (double)az_;
                    if (l == nl - 1 && jp < ny - 1) yf[ip + nx * kp] = ay_;
                    if (w == nw - 1 && kp < nz - 1) zf[ip + nx * jp] = az_;
                    xo = ax_;
                    yo = ay_;
                    zo = az_;
                }
                zbuf[t & 1][w][l] = zo;
                __syncthreads();
            }
        }
    }
    // boundary outflow sums of this block (for the particle balance)
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
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += red[threadIdx.x][q];
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
    if (is_f64) hipLaunchKernelGGL((k_sweep<double, 4>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_sweep<float, 8>), grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace dct
