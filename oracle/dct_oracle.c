/*
 * Plain FP64 CPU oracle for the discrete-ordinates CT dose method of
 * Norris & Liu, "Photon Fluence and Dose Estimation in Computed Tomography
 * using a Discrete Ordinates Boltzmann Solver" (arXiv:1811.12391).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the HIP library is checked against.  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the product
 * path never does.  It shares no code, header or table with the HIP library.
 *
 * What it computes (paper section in brackets):
 *   - uncollided fluence by ray tracing from a collimated isotropic point
 *     source, phi_u = w_g exp(-tau_g) / (4 pi r^2) [Sec. II-A, first-collision
 *     source paragraph; Sec. II-B source types];
 *   - the first-collision source built from phi_u, in Legendre/real spherical
 *     harmonic moments [Sec. II-A, eq. 2 and the first-collision paragraph];
 *   - per-group source iteration with downscatter on the discrete-ordinates
 *     equation, eq. (2), vacuum boundaries [Sec. II-A];
 *   - diamond-difference sweeps over voxels with a set-to-zero fixup;
 *   - scalar fluence by quadrature, eq. (3), and the collision-kerma dose
 *     tally dose = sum_g kappa_g (phi_u,g + phi_c,g) [Sec. II-A].
 *
 * Readings taken where the paper is silent (spatial scheme, iteration scheme,
 * weight placement in eq. 2, beam window, stopping rule) follow the method
 * description: diamond difference; group Gauss-Seidel from the highest group
 * with source iteration started from zero; the quadrature weight belongs to
 * the incoming direction; a rectangular window in azimuth and elevation with
 * full angles fan x cone, edges inclusive; stop when the relative max-norm
 * change of the scalar flux is <= tol.
 *
 * Index conventions: voxel v = i + nx*(j + ny*k); group g = 0 highest energy;
 * moment index lm = l*l + l + m for m = -l..l; arrays are C-order with the
 * voxel index innermost.
 *
 * Parity: every function below is pinned by the CPU test suite against closed
 * forms, hand values, brute force or invariants, except the phantom
 * generator, the fixup pattern and the stopping point, which have no external
 * values ("parity unpinned" beyond oracle <-> GPU self-consistency).  The
 * scattering source of every degree l (within-group and downscatter, forward
 * and adjoint) goes through orc_scatter_moments, which is pinned against the
 * direction-to-direction form of eq. (2) and, inside the full solve, against
 * the anisotropic infinite-medium closed form.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics, Schmidt semi-normalised, no Condon-Shortley      */
/* phase, polar axis z: Y_00 = 1 and sum_m Y_lm(a) Y_lm(b) = P_l(a.b).       */
/* Used for the Legendre scattering expansion of eq. (2).                     */
/* ------------------------------------------------------------------------ */
int orc_real_sh(int L, double ox, double oy, double oz, double *Y)
{
    if (L < 0 || L > 16) return -1;
    double P[17][17];
    double mu = oz;
    double s = hypot(ox, oy);
    double phi = atan2(oy, ox);
    for (int m = 0; m <= L; ++m) {
        double pmm = 1.0;
        for (int t = 1; t <= m; ++t) pmm *= (2.0 * t - 1.0) * s;   /* (2m-1)!! s^m */
        P[m][m] = pmm;
        if (m + 1 <= L) P[m + 1][m] = (2.0 * m + 1.0) * mu * pmm;
        for (int l = m + 2; l <= L; ++l)
            P[l][m] = ((2.0 * l - 1.0) * mu * P[l - 1][m] - (l + m - 1.0) * P[l - 2][m]) / (l - m);
    }
    for (int l = 0; l <= L; ++l) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double ratio = 1.0;                         /* (l-am)! / (l+am)! */
            for (int t = l - am + 1; t <= l + am; ++t) ratio /= (double)t;
            double nrm = sqrt((am == 0 ? 1.0 : 2.0) * ratio);
            double ang = (m >= 0) ? cos(am * phi) : sin(am * phi);
            Y[l * l + l + m] = nrm * P[l][am] * ang;
        }
    }
    return 0;
}

/* Moment <-> direction maps of the P_N expansion:
 *   M[n][lm] = (2l+1)/(4 pi) Y_lm(Omega_n)  (moments -> angular source)
 *   D[lm][n] = w_n Y_lm(Omega_n)            (angular flux -> moments; row 0 is eq. 3) */
int orc_moment_maps(int L, int N, const double *dirs, const double *w, double *Mmap, double *Dmap)
{
    int Nm = (L + 1) * (L + 1);
    double Y[289];
    for (int n = 0; n < N; ++n) {
        if (orc_real_sh(L, dirs[3 * n], dirs[3 * n + 1], dirs[3 * n + 2], Y)) return -1;
        for (int l = 0; l <= L; ++l)
            for (int m = -l; m <= l; ++m) {
                int lm = l * l + l + m;
                if (Mmap) Mmap[(size_t)n * Nm + lm] = (2.0 * l + 1.0) / (4.0 * ORC_PI) * Y[lm];
                if (Dmap) Dmap[(size_t)lm * N + n] = w[n] * Y[lm];
            }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Siddon ray trace: the segment p -> x (x a voxel centre) is cut at every    */
/* x, y and z grid plane strictly between the box entry and x.  Each segment  */
/* gets length (a_m - a_{m-1}) r and the voxel holding its midpoint.          */
/* ------------------------------------------------------------------------ */
static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

int orc_siddon(int nx, int ny, int nz, double dx, double dy, double dz, const double *org,
               const double *p, const double *x, int maxseg, int *vox, double *len)
{
    int n[3] = {nx, ny, nz};
    double del[3] = {dx, dy, dz};
    double d[3] = {x[0] - p[0], x[1] - p[1], x[2] - p[2]};
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double a_in = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) continue;
        double lo = org[a], hi = org[a] + n[a] * del[a];
        double t0 = (lo - p[a]) / d[a], t1 = (hi - p[a]) / d[a];
        double tmin = t0 < t1 ? t0 : t1;
        if (tmin > a_in) a_in = tmin;
    }
    int cap = nx + ny + nz + 3;
    double *al = (double *)malloc(sizeof(double) * (cap + 2));
    int na = 0;
    al[na++] = a_in;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) continue;
        for (int m = 0; m <= n[a]; ++m) {
            double t = (org[a] + m * del[a] - p[a]) / d[a];
            if (t > a_in && t < 1.0) al[na++] = t;
        }
    }
    al[na++] = 1.0;
    qsort(al + 1, na - 2, sizeof(double), cmp_double);
    int ns = 0;
    for (int s = 1; s < na; ++s) {
        if (ns >= maxseg) { free(al); return -1; }
        double a0 = al[s - 1], a1 = al[s];
        double mid = 0.5 * (a0 + a1);
        int idx[3];
        for (int a = 0; a < 3; ++a) {
            int t = (int)floor((p[a] + mid * d[a] - org[a]) / del[a]);
            if (t < 0) t = 0;
            if (t > n[a] - 1) t = n[a] - 1;
            idx[a] = t;
        }
        vox[ns] = idx[0] + nx * (idx[1] + ny * idx[2]);
        len[ns] = (a1 - a0) * r;
        ++ns;
    }
    free(al);
    return ns;
}

/* Beam window of a collimated point source: azimuth in the plane normal to z,
 * measured from the beam axis projected on that plane, and elevation from
 * that plane; full angles fan x cone, edges inclusive. */
static int in_beam(const double *d, const double *axis, double fan_deg, double cone_deg)
{
    double ax = axis[0], ay = axis[1];
    double an = hypot(ax, ay);
    ax /= an;
    ay /= an;
    double ex = -ay, ey = ax;                         /* z x a */
    double along = d[0] * ax + d[1] * ay;
    double across = d[0] * ex + d[1] * ey;
    double az = atan2(across, along);
    double el = atan2(d[2], hypot(d[0], d[1]));
    double hf = fan_deg * ORC_PI / 360.0, hc = cone_deg * ORC_PI / 360.0;
    return fabs(az) <= hf && fabs(el) <= hc;
}

/* Uncollided fluence phi_u[B][G][C]: no scatter term, so it follows from the
 * optical depth along the straight ray from the source to each voxel centre
 * (first-collision paragraph of Sec. II-A; Sec. IV obtains the uncollided
 * part in closed form).  tau_g is summed in ray order, source to target. */
int orc_uncollided(int nx, int ny, int nz, double dx, double dy, double dz, const double *org,
                   const uint8_t *mat, const double *rho, int G, int M, const double *st,
                   int B, const double *pos, const double *axis, double fan_deg, double cone_deg,
                   const double *gw, int nthreads, double *phi_u)
{
    size_t C = (size_t)nx * ny * nz;
    int cap = nx + ny + nz + 4;
    (void)M;
    for (int b = 0; b < B; ++b) {
        const double *p = pos + 3 * b;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
        for (long v = 0; v < (long)C; ++v) {
            int i = (int)(v % nx), j = (int)((v / nx) % ny), k = (int)(v / ((size_t)nx * ny));
            double x[3] = {org[0] + (i + 0.5) * dx, org[1] + (j + 0.5) * dy, org[2] + (k + 0.5) * dz};
            double d[3] = {x[0] - p[0], x[1] - p[1], x[2] - p[2]};
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!in_beam(d, axis + 3 * b, fan_deg, cone_deg)) {
                for (int g = 0; g < G; ++g) phi_u[((size_t)b * G + g) * C + v] = 0.0;
                continue;
            }
            int *vox = (int *)malloc(sizeof(int) * cap);
            double *len = (double *)malloc(sizeof(double) * cap);
            int ns = orc_siddon(nx, ny, nz, dx, dy, dz, org, p, x, cap, vox, len);
            for (int g = 0; g < G; ++g) {
                double tau = 0.0;
                for (int s = 0; s < ns; ++s) {
                    int u = vox[s];
                    tau += len[s] * rho[u] * st[(size_t)mat[u] * G + g];
                }
                phi_u[((size_t)b * G + g) * C + v] = gw[g] * exp(-tau) / (4.0 * ORC_PI * r2);
            }
            free(vox);
            free(len);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Diamond difference for one voxel and one direction.                         */
/* Cell balance of eq. (2) over a box with c_a = |Omega_a| / Delta_a:          */
/*   sum_a c_a (out_a - in_a) + sigma psi_c = q,  out_a = 2 psi_c - in_a.       */
/* Fixup: a negative outgoing face is set to zero and psi_c is recomputed from */
/* the balance with that face removed, until no new negative face appears.     */
/* Returns the number of fixed faces.                                          */
/* ------------------------------------------------------------------------ */
static int dd_cell_decide(double q, double sig, const double *c, const double *pin, int fixup,
                          double *pc, double *pout, int *F)
{
    double num = q + 2.0 * (c[0] * pin[0] + c[1] * pin[1] + c[2] * pin[2]);
    double den = sig + 2.0 * (c[0] + c[1] + c[2]);
    double psi = num / den;
    int fixed[3] = {0, 0, 0}, nf = 0;
    for (int a = 0; a < 3; ++a) pout[a] = 2.0 * psi - pin[a];
    if (fixup) {
        for (int pass = 0; pass < 3; ++pass) {
            int fresh = 0;
            for (int a = 0; a < 3; ++a)
                if (!fixed[a] && pout[a] < 0.0) { fixed[a] = 1; fresh = 1; ++nf; }
            if (!fresh) break;
            num = q;
            den = sig;
            for (int a = 0; a < 3; ++a) {
                if (fixed[a]) num += c[a] * pin[a];
                else { num += 2.0 * c[a] * pin[a]; den += 2.0 * c[a]; }
            }
            psi = num / den;
            for (int a = 0; a < 3; ++a) pout[a] = fixed[a] ? 0.0 : 2.0 * psi - pin[a];
        }
    }
    *pc = psi;
    if (F) *F = fixed[0] | (fixed[1] << 1) | (fixed[2] << 2);
    return nf;
}

int orc_dd_cell(double q, double sig, const double *c, const double *pin, int fixup,
                double *pc, double *pout)
{
    return dd_cell_decide(q, sig, c, pin, fixup, pc, pout, NULL);
}

/* The same cell with a frozen set F of fixed faces (bit a set: face a fixed):
 * the linear map (q, inflow) -> (psi_c, outflow) that the fixup produced. */
static void dd_cell_frozen(double q, double sig, const double *c, const double *pin, int F, double *pc,
                           double *pout)
{
    double num = q, den = sig;
    for (int a = 0; a < 3; ++a) {
        if ((F >> a) & 1) num += c[a] * pin[a];
        else { num += 2.0 * c[a] * pin[a]; den += 2.0 * c[a]; }
    }
    double psi = num / den;
    for (int a = 0; a < 3; ++a) pout[a] = ((F >> a) & 1) ? 0.0 : 2.0 * psi - pin[a];
    *pc = psi;
}

/* Transpose of dd_cell_frozen.  Inputs: weight s on psi_c and weights fin on
 * the outflow faces (the adjoint face values coming back from the downwind
 * neighbours); outputs: weight lc on q and fout on the inflow faces.  With
 * gamma_a = 0 for fixed faces (1 otherwise) and alpha_a = c_a (fixed) or
 * 2 c_a:  lc = (s + 2 sum gamma_a fin_a) / (sig + sum_{a not fixed} 2 c_a),
 *         fout_a = alpha_a lc - gamma_a fin_a. */
static void dd_cell_adjoint(double s, double sig, const double *c, const double *fin, int F, double *lc,
                            double *fout)
{
    double num = s, den = sig;
    for (int a = 0; a < 3; ++a)
        if (!((F >> a) & 1)) { num += 2.0 * fin[a]; den += 2.0 * c[a]; }
    double l = num / den;
    for (int a = 0; a < 3; ++a) fout[a] = ((F >> a) & 1) ? c[a] * l : 2.0 * c[a] * l - fin[a];
    *lc = l;
}

/* One transport sweep for every direction: cells visited in upwind order
 * (lexicographic in the octant's reflected coordinates), incoming boundary
 * angular flux = inflow[n] (0 for vacuum).  psi[N][C] receives the cell-centre
 * angular flux; leak[N][3] (optional) the sum of outgoing boundary face fluxes
 * per axis.  mask_out[N][C] (optional) records each cell's final fixed-face
 * set; with mask_in[N][C] the fixup is not decided but frozen to the given
 * sets (a linear map).  Returns the total number of fixed faces. */
long orc_sweep2(int nx, int ny, int nz, double dx, double dy, double dz, const double *sigt,
                int N, const double *dirs, const double *q, const double *inflow, int fixup,
                int nthreads, double *psi, double *leak, const uint8_t *mask_in, uint8_t *mask_out)
{
    size_t C = (size_t)nx * ny * nz;
    long nfix = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(+ : nfix)
    for (int n = 0; n < N; ++n) {
        const double *om = dirs + 3 * n;
        double c[3] = {fabs(om[0]) / dx, fabs(om[1]) / dy, fabs(om[2]) / dz};
        double bc = inflow ? inflow[n] : 0.0;
        double *fx = (double *)malloc(sizeof(double) * (size_t)ny * nz);
        double *fy = (double *)malloc(sizeof(double) * (size_t)nx * nz);
        double *fz = (double *)malloc(sizeof(double) * (size_t)nx * ny);
        for (size_t t = 0; t < (size_t)ny * nz; ++t) fx[t] = bc;
        for (size_t t = 0; t < (size_t)nx * nz; ++t) fy[t] = bc;
        for (size_t t = 0; t < (size_t)nx * ny; ++t) fz[t] = bc;
        double lx = 0.0, ly = 0.0, lz = 0.0;
        const double *qn = q + (size_t)n * C;
        double *pn = psi + (size_t)n * C;
        for (int kk = 0; kk < nz; ++kk) {
            int k = om[2] > 0 ? kk : nz - 1 - kk;
            for (int jj = 0; jj < ny; ++jj) {
                int j = om[1] > 0 ? jj : ny - 1 - jj;
                for (int ii = 0; ii < nx; ++ii) {
                    int i = om[0] > 0 ? ii : nx - 1 - ii;
                    size_t v = (size_t)i + (size_t)nx * (j + (size_t)ny * k);
                    double pin[3] = {fx[j + (size_t)ny * k], fy[i + (size_t)nx * k], fz[i + (size_t)nx * j]};
                    double pc, pout[3];
                    if (mask_in) {
                        dd_cell_frozen(qn[v], sigt[v], c, pin, mask_in[(size_t)n * C + v], &pc, pout);
                    } else {
                        int F = 0;
                        nfix += dd_cell_decide(qn[v], sigt[v], c, pin, fixup, &pc, pout, &F);
                        if (mask_out) mask_out[(size_t)n * C + v] = (uint8_t)F;
                    }
                    pn[v] = pc;
                    fx[j + (size_t)ny * k] = pout[0];
                    fy[i + (size_t)nx * k] = pout[1];
                    fz[i + (size_t)nx * j] = pout[2];
                    if (ii == nx - 1) lx += pout[0];
                    if (jj == ny - 1) ly += pout[1];
                    if (kk == nz - 1) lz += pout[2];
                }
            }
        }
        if (leak) {
            leak[3 * n + 0] = lx;
            leak[3 * n + 1] = ly;
            leak[3 * n + 2] = lz;
        }
        free(fx);
        free(fy);
        free(fz);
    }
    return nfix;
}

long orc_sweep(int nx, int ny, int nz, double dx, double dy, double dz, const double *sigt,
               int N, const double *dirs, const double *q, const double *inflow, int fixup,
               int nthreads, double *psi, double *leak)
{
    return orc_sweep2(nx, ny, nz, dx, dy, dz, sigt, N, dirs, q, inflow, fixup, nthreads, psi, leak, NULL, NULL);
}

/* Transpose of the frozen-mask sweep with vacuum inflow: given weights s[N][C]
 * on the cell-centre fluxes, returns lam[N][C], the weights on the sources q
 * (<s, L^-1 q> = <L^-T s, q>).  Cells are visited in the reverse of the
 * forward order; the adjoint face values travel upwind, starting from 0 at
 * the outflow boundary. */
int orc_sweep_adjoint(int nx, int ny, int nz, double dx, double dy, double dz, const double *sigt,
                      int N, const double *dirs, const double *s, const uint8_t *mask, int nthreads,
                      double *lam)
{
    size_t C = (size_t)nx * ny * nz;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int n = 0; n < N; ++n) {
        const double *om = dirs + 3 * n;
        double c[3] = {fabs(om[0]) / dx, fabs(om[1]) / dy, fabs(om[2]) / dz};
        double *fx = (double *)calloc((size_t)ny * nz, sizeof(double));
        double *fy = (double *)calloc((size_t)nx * nz, sizeof(double));
        double *fz = (double *)calloc((size_t)nx * ny, sizeof(double));
        const double *sn = s + (size_t)n * C;
        double *ln = lam + (size_t)n * C;
        for (int kk = nz - 1; kk >= 0; --kk) {
            int k = om[2] > 0 ? kk : nz - 1 - kk;
            for (int jj = ny - 1; jj >= 0; --jj) {
                int j = om[1] > 0 ? jj : ny - 1 - jj;
                for (int ii = nx - 1; ii >= 0; --ii) {
                    int i = om[0] > 0 ? ii : nx - 1 - ii;
                    size_t v = (size_t)i + (size_t)nx * (j + (size_t)ny * k);
                    double fin[3] = {fx[j + (size_t)ny * k], fy[i + (size_t)nx * k], fz[i + (size_t)nx * j]};
                    double lc, fout[3];
                    dd_cell_adjoint(sn[v], sigt[v], c, fin, mask[(size_t)n * C + v], &lc, fout);
                    ln[v] = lc;
                    fx[j + (size_t)ny * k] = fout[0];
                    fy[i + (size_t)nx * k] = fout[1];
                    fz[i + (size_t)nx * j] = fout[2];
                }
            }
        }
        free(fx);
        free(fy);
        free(fz);
    }
    return 0;
}

/* First-collision source of one right-hand side: the uncollided flux at voxel
 * v is a delta in angle along d/r (d = x_v - p), so its moments are
 * phi_u Y_lm(d/r) and the once-scattered source has moments
 *   ext[g][lm][v] = sum_{g' <= g} rho_v s_l^{g'->g}[m_v] phi_u,g'(v) Y_lm(d/r)
 * (first-collision paragraph of Sec. II-A), summed in increasing g'.  An
 * optional isotropic volumetric source S[g][v] (the S term of eq. 1) is added
 * to the l = 0 moment afterwards. */
int orc_first_collision(int nx, int ny, int nz, double dx, double dy, double dz, const double *org,
                        const uint8_t *mat, const double *rho, int G, int L, const double *ss,
                        const double *p, const double *pu, const double *ext_iso, int nthreads,
                        double *ext)
{
    size_t C = (size_t)nx * ny * nz;
    int Nm = (L + 1) * (L + 1);
    int lof[289];
    for (int l = 0; l <= L; ++l)
        for (int m = -l; m <= l; ++m) lof[l * l + l + m] = l;
    memset(ext, 0, sizeof(double) * (size_t)G * Nm * C);
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (long v = 0; v < (long)C; ++v) {
        int i = (int)(v % nx), j = (int)((v / nx) % ny), k = (int)(v / ((size_t)nx * ny));
        double d[3] = {org[0] + (i + 0.5) * dx - p[0], org[1] + (j + 0.5) * dy - p[1],
                       org[2] + (k + 0.5) * dz - p[2]};
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double Y[289];
        orc_real_sh(L, d[0] / r, d[1] / r, d[2] / r, Y);
        int m = mat[v];
        for (int g = 0; g < G; ++g)
            for (int gp = 0; gp <= g; ++gp) {
                double fu = pu[(size_t)gp * C + v];
                for (int lm = 0; lm < Nm; ++lm) {
                    double s = ss[(((size_t)m * (L + 1) + lof[lm]) * G + gp) * G + g];
                    ext[((size_t)g * Nm + lm) * C + v] += rho[v] * s * fu * Y[lm];
                }
            }
        if (ext_iso)
            for (int g = 0; g < G; ++g) ext[(size_t)g * Nm * C + v] += ext_iso[(size_t)g * C + v];
    }
    return 0;
}

/* Scattering source of eq. (2) in moment form.  With the scattering kernel
 * expanded in Legendre polynomials and P_l(Omega . Omega') written by the
 * addition theorem as sum_m Y_lm(Omega) Y_lm(Omega'), the direction-to-
 * direction sum of eq. (2) becomes one product per moment: the flux moments
 * phi[Nm][C] of group gf put the source  rho_v s_l^{gf->gt}[m_v] phi[lm][v]
 * into moment lm (degree l) of group gt.  This function writes
 *   out[lm][v] = base[lm][v] + rho_v s_l^{gf->gt}[m_v] phi[lm][v]
 * (base NULL: 0; base may be out itself, which accumulates).  gf == gt is the
 * within-group term, gf < gt the downscatter of eq. (2)'s group sum; the
 * adjoint applies the same products with the roles of the groups exchanged
 * (weights of gt carried back to gf).  ss is [M][L+1][G][G] (from, to). */
int orc_scatter_moments(long C, const uint8_t *mat, const double *rho, int G, int L, const double *ss, int gf,
                        int gt, const double *phi, const double *base, double *out, int nthreads)
{
    if (L < 0 || gf < 0 || gt < 0 || gf >= G || gt >= G) return -1;
    for (int l = 0; l <= L; ++l)
        for (int m = -l; m <= l; ++m) {
            const size_t lm = (size_t)(l * l + l + m);
#pragma omp parallel for schedule(static) num_threads(nthreads)
            for (long v = 0; v < C; ++v) {
                const double s = ss[(((size_t)mat[v] * (L + 1) + l) * G + gf) * G + gt];
                const double b = base ? base[lm * C + v] : 0.0;
                out[lm * C + v] = b + rho[v] * s * phi[lm * C + v];
            }
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Full solve: uncollided -> first-collision source -> per-group source        */
/* iteration with downscatter -> dose.  Each right-hand side (source) b is      */
/* solved on its own with its own stopping point.                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    int nx, ny, nz;
    double dx, dy, dz;
    const double *org;
    const uint8_t *mat;
    const double *rho;
    int G, M, L, Nm, N;
    const double *st, *ss, *kap, *dirs, *w;
    const double *Mmap, *Dmap;
    const int *lof;
} Prob;

static double ss_at(const Prob *P, int m, int l, int gf, int gt)
{
    return P->ss[(((size_t)m * (P->L + 1) + l) * P->G + gf) * P->G + gt];
}

/* Forward solve of one right-hand side.  ext = its first-collision source
 * [G][Nm][C] (owned by the call: downscatter is added to it in place), pu =
 * its uncollided flux [G][C].  Outputs phi[G][Nm][C], dose[C], iters[G],
 * eps[G], bal[G][3].  inflow_dir[G][N] (or NULL: vacuum) is the angular flux
 * entering through the boundary in each direction.  When psi_store /
 * mask_store are given, the cell fluxes
 * [G][N][C] and fixed-face sets of the final sweep of every group are kept
 * (for the adjoint). */
static int forward_rhs(const Prob *P, double *ext, const double *pu,
                       double tol, int max_iter, const int *fixed_iters, int fixup, const double *inflow_dir,
                       int nthreads, double *phi, double *dose, int *iters, double *eps, double *bal,
                       long *nfix_total, double *psi_store, uint8_t *mask_store)
{
    const int G = P->G, Nm = P->Nm, N = P->N, L = P->L;
    const size_t C = (size_t)P->nx * P->ny * P->nz;
    const double V = P->dx * P->dy * P->dz;
    const double Ax = P->dy * P->dz, Ay = P->dx * P->dz, Az = P->dx * P->dy;
    double *Q = (double *)malloc(sizeof(double) * (size_t)Nm * C);
    double *q = (double *)malloc(sizeof(double) * (size_t)N * C);
    double *ps = (double *)malloc(sizeof(double) * (size_t)N * C);
    double *cur = (double *)malloc(sizeof(double) * (size_t)Nm * C);
    double *nxt = (double *)malloc(sizeof(double) * (size_t)Nm * C);
    double *sigt = (double *)malloc(sizeof(double) * C);
    double *leak = (double *)malloc(sizeof(double) * 3 * N);
    double *inflow = (double *)malloc(sizeof(double) * N);
    uint8_t *mask = (uint8_t *)malloc((size_t)N * C);
    if (!Q || !q || !ps || !cur || !nxt || !sigt || !leak || !inflow || !mask) return -4;
    for (int g = 0; g < G; ++g) {
        const double *ig = inflow_dir ? inflow_dir + (size_t)g * N : NULL;
        for (int n = 0; n < N; ++n) inflow[n] = ig ? ig[n] : 0.0;
        for (size_t v = 0; v < C; ++v) sigt[v] = P->rho[v] * P->st[(size_t)P->mat[v] * G + g];
        double *eg = ext + (size_t)g * Nm * C;
        /* production: volumetric source plus boundary inflow */
        double Pr = 0.0;
        for (size_t v = 0; v < C; ++v) Pr += eg[v];
        Pr *= V;
        /* each direction enters through one face per axis */
        for (int n = 0; n < N; ++n)
            if (inflow[n] != 0.0)
                Pr += inflow[n] * P->w[n] * (fabs(P->dirs[3 * n]) * Ax * P->ny * P->nz + fabs(P->dirs[3 * n + 1]) * Ay * P->nx * P->nz +
                                             fabs(P->dirs[3 * n + 2]) * Az * P->nx * P->ny);
        memset(cur, 0, sizeof(double) * (size_t)Nm * C);
        int it = 0;
        double e = 0.0;
        for (;;) {
            /* scattering source within the group plus the fixed source */
            orc_scatter_moments((long)C, P->mat, P->rho, G, L, P->ss, g, g, cur, eg, Q, nthreads);
            /* moments -> directions */
#pragma omp parallel for schedule(static) num_threads(nthreads)
            for (long v = 0; v < (long)C; ++v)
                for (int n = 0; n < N; ++n) {
                    double acc = 0.0;
                    for (int lm = 0; lm < Nm; ++lm) acc += P->Mmap[(size_t)n * Nm + lm] * Q[(size_t)lm * C + v];
                    q[(size_t)n * C + v] = acc;
                }
            *nfix_total += orc_sweep2(P->nx, P->ny, P->nz, P->dx, P->dy, P->dz, sigt, N, P->dirs, q, inflow, fixup,
                                      nthreads, ps, leak, NULL, mask);
            /* directions -> moments (row 0 is the scalar flux, eq. 3) */
#pragma omp parallel for schedule(static) num_threads(nthreads)
            for (long v = 0; v < (long)C; ++v)
                for (int lm = 0; lm < Nm; ++lm) {
                    double acc = 0.0;
                    for (int n = 0; n < N; ++n) acc += P->Dmap[(size_t)lm * N + n] * ps[(size_t)n * C + v];
                    nxt[(size_t)lm * C + v] = acc;
                }
            double dmax = 0.0, fmax = 0.0;
            for (size_t v = 0; v < C; ++v) {
                double df = fabs(nxt[v] - cur[v]);
                double f = fabs(nxt[v]);
                if (df > dmax) dmax = df;
                if (f > fmax) fmax = f;
            }
            e = fmax > 0.0 ? dmax / fmax : 0.0;
            double *t = cur; cur = nxt; nxt = t;
            ++it;
            if (fixed_iters) { if (it >= fixed_iters[g]) break; }
            else if (e <= tol || it >= max_iter) break;
        }
        iters[g] = it;
        eps[g] = e;
        if (psi_store) memcpy(psi_store + (size_t)g * N * C, ps, sizeof(double) * (size_t)N * C);
        if (mask_store) memcpy(mask_store + (size_t)g * N * C, mask, (size_t)N * C);
        /* balance of the final sweep's group: production, removal, leakage */
        double R = 0.0;
        for (size_t v = 0; v < C; ++v) R += (sigt[v] - P->rho[v] * ss_at(P, P->mat[v], 0, g, g)) * cur[v];
        R *= V;
        double Lk = 0.0;
        for (int n = 0; n < N; ++n)
            Lk += P->w[n] * (fabs(P->dirs[3 * n]) * Ax * leak[3 * n] + fabs(P->dirs[3 * n + 1]) * Ay * leak[3 * n + 1] +
                             fabs(P->dirs[3 * n + 2]) * Az * leak[3 * n + 2]);
        bal[g * 3 + 0] = Pr;
        bal[g * 3 + 1] = R;
        bal[g * 3 + 2] = Lk;
        /* downscatter into every lower-energy group */
        for (int g2 = g + 1; g2 < G; ++g2) {
            double *e2 = ext + (size_t)g2 * Nm * C;
            orc_scatter_moments((long)C, P->mat, P->rho, G, L, P->ss, g, g2, cur, e2, e2, nthreads);
        }
        memcpy(phi + (size_t)g * Nm * C, cur, sizeof(double) * (size_t)Nm * C);
        /* dose: collision kerma of uncollided + collided scalar fluence */
        for (size_t v = 0; v < C; ++v) {
            double k0 = P->kap[(size_t)P->mat[v] * G + g];
            if (g == 0) dose[v] = 0.0;
            dose[v] += k0 * (pu[(size_t)g * C + v] + cur[v]);
        }
    }
    free(Q); free(q); free(ps); free(cur); free(nxt); free(sigt); free(leak); free(inflow); free(mask);
    return 0;
}

static void make_prob(Prob *P, int nx, int ny, int nz, double dx, double dy, double dz, const double *org,
                      const uint8_t *mat, const double *rho, int G, int M, int L, const double *st, const double *ss,
                      const double *kap, int N, const double *dirs, const double *w, int *lof)
{
    (void)M;
    P->nx = nx; P->ny = ny; P->nz = nz; P->dx = dx; P->dy = dy; P->dz = dz; P->org = org;
    P->mat = mat; P->rho = rho; P->G = G; P->M = M; P->L = L; P->Nm = (L + 1) * (L + 1); P->N = N;
    P->st = st; P->ss = ss; P->kap = kap; P->dirs = dirs; P->w = w;
    for (int l = 0; l <= L; ++l)
        for (int m = -l; m <= l; ++m) lof[l * l + l + m] = l;
    P->lof = lof;
    double *Mmap = (double *)malloc(sizeof(double) * N * P->Nm);
    double *Dmap = (double *)malloc(sizeof(double) * N * P->Nm);
    orc_moment_maps(L, N, dirs, w, Mmap, Dmap);
    P->Mmap = Mmap;
    P->Dmap = Dmap;
}

static void free_prob(Prob *P)
{
    free((void *)P->Mmap);
    free((void *)P->Dmap);
}

/* Superposed sources (the CT-scan form of Sec. III-C: several cone beams in
 * one simulation): the B sources form B / S right-hand sides of S consecutive
 * sources each.  The transport problem is linear in its source, so one
 * collided solve per right-hand side takes the sum of its sources'
 * first-collision sources, and its dose adds the sum of their uncollided
 * fluxes.  S = 1 solves every source on its own.  Outputs per right-hand
 * side: phi_u [B/S][G][C] (summed), phi, dose, iters, eps, bal. */
int orc_solve_sup(int nx, int ny, int nz, double dx, double dy, double dz, const double *org,
                  const uint8_t *mat, const double *rho,
                  int G, int M, int L, const double *st, const double *ss, const double *kap,
                  int N, const double *dirs, const double *w,
                  int B, int S, const double *pos, const double *axis, double fan_deg, double cone_deg,
                  const double *gw, const double *ext_iso,
                  double tol, int max_iter, const int *fixed_iters, int fixup,
                  const double *test_inflow, int nthreads,
                  double *phi_u, double *phi, double *dose, int *iters, double *eps, double *bal,
                  long *nfix_out)
{
    if (S < 1 || B % S != 0) return -1;
    size_t C = (size_t)nx * ny * nz;
    int lof[289];
    Prob P;
    make_prob(&P, nx, ny, nz, dx, dy, dz, org, mat, rho, G, M, L, st, ss, kap, N, dirs, w, lof);
    const int Nm = P.Nm, R = B / S;
    double *pu_src = (double *)malloc(sizeof(double) * (size_t)B * G * C);
    double *ext = (double *)malloc(sizeof(double) * (size_t)G * Nm * C);
    double *ext1 = (double *)malloc(sizeof(double) * (size_t)G * Nm * C);
    if (!pu_src || !ext || !ext1) return -4;
    orc_uncollided(nx, ny, nz, dx, dy, dz, org, mat, rho, G, M, st, B, pos, axis, fan_deg, cone_deg, gw, nthreads,
                   pu_src);
    double *inflow_dir = NULL;
    if (test_inflow) {
        inflow_dir = (double *)malloc(sizeof(double) * (size_t)G * N);
        if (!inflow_dir) return -4;
        for (int g = 0; g < G; ++g)
            for (int n = 0; n < N; ++n) inflow_dir[(size_t)g * N + n] = test_inflow[g];
    }
    long nfix = 0;
    int rc = 0;
    for (int r = 0; r < R && rc == 0; ++r) {
        double *pu = phi_u + (size_t)r * G * C;
        memset(pu, 0, sizeof(double) * (size_t)G * C);
        memset(ext, 0, sizeof(double) * (size_t)G * Nm * C);
        for (int k = 0; k < S; ++k) {
            const int b = r * S + k;
            const double *pb = pu_src + (size_t)b * G * C;
            /* the volumetric source belongs to the problem, not to a beam: once per right-hand side */
            orc_first_collision(nx, ny, nz, dx, dy, dz, org, mat, rho, G, L, ss, pos + 3 * b, pb,
                                k == 0 ? ext_iso : NULL, nthreads, ext1);
            for (size_t i = 0; i < (size_t)G * Nm * C; ++i) ext[i] += ext1[i];
            for (size_t i = 0; i < (size_t)G * C; ++i) pu[i] += pb[i];
        }
        rc = forward_rhs(&P, ext, pu, tol, max_iter, fixed_iters, fixup, inflow_dir, nthreads,
                         phi + (size_t)r * G * Nm * C, dose + (size_t)r * C, iters + r * G, eps + r * G,
                         bal + (size_t)r * G * 3, &nfix, NULL, NULL);
    }
    if (nfix_out) *nfix_out = nfix;
    free(inflow_dir);
    free(pu_src);
    free(ext);
    free(ext1);
    free_prob(&P);
    return rc;
}

int orc_solve(int nx, int ny, int nz, double dx, double dy, double dz, const double *org,
              const uint8_t *mat, const double *rho,
              int G, int M, int L, const double *st, const double *ss, const double *kap,
              int N, const double *dirs, const double *w,
              int B, const double *pos, const double *axis, double fan_deg, double cone_deg,
              const double *gw, const double *ext_iso,
              double tol, int max_iter, const int *fixed_iters, int fixup,
              const double *test_inflow, int nthreads,
              double *phi_u, double *phi, double *dose, int *iters, double *eps, double *bal,
              long *nfix_out)
{
    return orc_solve_sup(nx, ny, nz, dx, dy, dz, org, mat, rho, G, M, L, st, ss, kap, N, dirs, w, B, 1, pos, axis,
                         fan_deg, cone_deg, gw, ext_iso, tol, max_iter, fixed_iters, fixup, test_inflow, nthreads,
                         phi_u, phi, dose, iters, eps, bal, nfix_out);
}

/* Collided solve of one right-hand side from a given fixed source: the
 * per-group source iteration with downscatter and the dose tally of
 * forward_rhs, with ext[G][Nm][C] (any moments, anisotropic included) in place
 * of the first-collision source, no uncollided flux, and inflow_dir[G][N]
 * (or NULL: vacuum) the angular flux entering through the boundary in every
 * direction.  Outputs phi[G][Nm][C], dose[C], iters[G], eps[G], bal[G][3]. */
int orc_solve_fixed(int nx, int ny, int nz, double dx, double dy, double dz, const double *org,
                    const uint8_t *mat, const double *rho,
                    int G, int M, int L, const double *st, const double *ss, const double *kap,
                    int N, const double *dirs, const double *w,
                    const double *ext_in, const double *inflow_dir,
                    double tol, int max_iter, int fixup, int nthreads,
                    double *phi, double *dose, int *iters, double *eps, double *bal)
{
    size_t C = (size_t)nx * ny * nz;
    int lof[289];
    Prob P;
    make_prob(&P, nx, ny, nz, dx, dy, dz, org, mat, rho, G, M, L, st, ss, kap, N, dirs, w, lof);
    const int Nm = P.Nm;
    double *ext = (double *)malloc(sizeof(double) * (size_t)G * Nm * C);
    double *pu = (double *)calloc((size_t)G * C, sizeof(double));
    if (!ext || !pu) return -4;
    memcpy(ext, ext_in, sizeof(double) * (size_t)G * Nm * C);
    long nfix = 0;
    int rc = forward_rhs(&P, ext, pu, tol, max_iter, NULL, fixup, inflow_dir, nthreads, phi, dose, iters, eps, bal,
                         &nfix, NULL, NULL);
    free(ext);
    free(pu);
    free_prob(&P);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Adjoint: gradient of R = sum_b sum_v roi_v dose_b(v) with respect to every  */
/* voxel density and every source group weight, at the converged forward      */
/* state with the fixup frozen (the solve is then linear in its sources).      */
/*                                                                            */
/* Within a group the converged moments satisfy Q = ext + S phi, phi = T Q     */
/* with T = D L^-1 M (L: the frozen sweep) and S = rho s_l^{gg}.  The adjoint  */
/* moments lam solve lam = T^T (phibar + S lam), iterated like the forward     */
/* (T^T = M^T L^-T D^T, L^-T the reversed sweep); groups run from the lowest   */
/* energy up, each adding rho s_l^{g->g''} lam_{g''} to the moment weight of   */
/* every higher group that fed it.  Then                                        */
/*   dR/dsigma_t,g(v) = - sum_n lamc_n(v) psi_n(v)   (cell-centre adjoint x flux) */
/*   dR/drho_v = sum_g [ t_g dR/dsigma_t,g + sum_lm lam_lm,g dQ_lm,g/drho_v ]    */
/*   phibar_u,g(v) = roi kappa_g + sum_{g''>=g} sum_lm rho s_l^{g->g''} Y_lm lam  */
/* and the optical depth of every ray takes back d phi_u / d rho_u =           */
/* -phi_u l_{v,u} t_g[m_u] (ray back-projection); dR/dw_g follows from phi_u   */
/* being linear in w_g.                                                         */
/* ------------------------------------------------------------------------ */
int orc_adjoint(int nx, int ny, int nz, double dx, double dy, double dz, const double *org,
                const uint8_t *mat, const double *rho,
                int G, int M, int L, const double *st, const double *ss, const double *kap,
                int N, const double *dirs, const double *w,
                int B, const double *pos, const double *axis, double fan_deg, double cone_deg,
                const double *gw, const double *roi,
                double tol, int max_iter, const int *fixed_iters, const int *fixed_iters_adj, int fixup,
                int nthreads, double *R_out, double *d_rho, double *d_gw, int *iters_adj)
{
    const size_t C = (size_t)nx * ny * nz;
    int lof[289];
    Prob P;
    make_prob(&P, nx, ny, nz, dx, dy, dz, org, mat, rho, G, M, L, st, ss, kap, N, dirs, w, lof);
    const int Nm = P.Nm;
    double *phi_u = (double *)malloc(sizeof(double) * (size_t)B * G * C);
    double *unit = (double *)malloc(sizeof(double) * (size_t)B * G * C);
    double *ones = (double *)malloc(sizeof(double) * G);
    for (int g = 0; g < G; ++g) ones[g] = 1.0;
    orc_uncollided(nx, ny, nz, dx, dy, dz, org, mat, rho, G, M, st, B, pos, axis, fan_deg, cone_deg, gw, nthreads,
                   phi_u);
    orc_uncollided(nx, ny, nz, dx, dy, dz, org, mat, rho, G, M, st, B, pos, axis, fan_deg, cone_deg, ones, nthreads,
                   unit);
    double *phi = (double *)malloc(sizeof(double) * (size_t)G * Nm * C);
    double *psi = (double *)malloc(sizeof(double) * (size_t)G * N * C);
    uint8_t *mask = (uint8_t *)malloc((size_t)G * N * C);
    double *dose = (double *)malloc(sizeof(double) * C);
    int *it_f = (int *)malloc(sizeof(int) * G);
    double *eps_f = (double *)malloc(sizeof(double) * G);
    double *bal = (double *)malloc(sizeof(double) * 3 * G);
    double *lam = (double *)malloc(sizeof(double) * (size_t)G * Nm * C);
    double *pb = (double *)malloc(sizeof(double) * (size_t)Nm * C);
    double *mu = (double *)malloc(sizeof(double) * (size_t)Nm * C);
    double *sdir = (double *)malloc(sizeof(double) * (size_t)N * C);
    double *lc = (double *)malloc(sizeof(double) * (size_t)N * C);
    double *cur = (double *)malloc(sizeof(double) * (size_t)Nm * C);
    double *nxt = (double *)malloc(sizeof(double) * (size_t)Nm * C);
    double *sigt = (double *)malloc(sizeof(double) * C);
    double *pbu = (double *)malloc(sizeof(double) * (size_t)G * C);
    double *ext = (double *)malloc(sizeof(double) * (size_t)G * Nm * C);
    long nfix = 0;
    double R = 0.0;
    memset(d_rho, 0, sizeof(double) * C);
    memset(d_gw, 0, sizeof(double) * G);
    for (int b = 0; b < B; ++b) {
        const double *p = pos + 3 * b;
        const double *pu = phi_u + (size_t)b * G * C;
        orc_first_collision(nx, ny, nz, dx, dy, dz, org, mat, rho, G, L, ss, p, pu, NULL, nthreads, ext);
        forward_rhs(&P, ext, pu, tol, max_iter, fixed_iters, fixup, NULL, nthreads, phi, dose, it_f, eps_f, bal,
                    &nfix, psi, mask);
        for (size_t v = 0; v < C; ++v) R += roi[v] * dose[v];
        /* direct weights of the dose on both fluence parts */
        for (int g = 0; g < G; ++g)
            for (size_t v = 0; v < C; ++v) pbu[(size_t)g * C + v] = roi[v] * kap[(size_t)mat[v] * G + g];
        memset(lam, 0, sizeof(double) * (size_t)G * Nm * C);
        for (int g = G - 1; g >= 0; --g) {
            for (size_t v = 0; v < C; ++v) sigt[v] = rho[v] * st[(size_t)mat[v] * G + g];
            /* moment weight of phi_g: dose seed + what the lower groups took from it */
            for (int lm = 0; lm < Nm; ++lm)
                for (size_t v = 0; v < C; ++v) pb[(size_t)lm * C + v] = lm == 0 ? roi[v] * kap[(size_t)mat[v] * G + g] : 0.0;
            for (int g2 = g + 1; g2 < G; ++g2)
                orc_scatter_moments((long)C, mat, rho, G, L, ss, g, g2, lam + (size_t)g2 * Nm * C, pb, pb, nthreads);
            memset(cur, 0, sizeof(double) * (size_t)Nm * C);
            int it = 0;
            const uint8_t *mg = mask + (size_t)g * N * C;
            for (;;) {
                orc_scatter_moments((long)C, mat, rho, G, L, ss, g, g, cur, pb, mu, nthreads);
                /* D^T: moment weights -> direction weights */
#pragma omp parallel for schedule(static) num_threads(nthreads)
                for (long v = 0; v < (long)C; ++v)
                    for (int n = 0; n < N; ++n) {
                        double acc = 0.0;
                        for (int lm = 0; lm < Nm; ++lm) acc += P.Dmap[(size_t)lm * N + n] * mu[(size_t)lm * C + v];
                        sdir[(size_t)n * C + v] = acc;
                    }
                orc_sweep_adjoint(nx, ny, nz, dx, dy, dz, sigt, N, dirs, sdir, mg, nthreads, lc);
                /* M^T: direction weights -> moment weights */
#pragma omp parallel for schedule(static) num_threads(nthreads)
                for (long v = 0; v < (long)C; ++v)
                    for (int lm = 0; lm < Nm; ++lm) {
                        double acc = 0.0;
                        for (int n = 0; n < N; ++n) acc += P.Mmap[(size_t)n * Nm + lm] * lc[(size_t)n * C + v];
                        nxt[(size_t)lm * C + v] = acc;
                    }
                double dmax = 0.0, fmax = 0.0;
                for (size_t v = 0; v < C; ++v) {
                    double df = fabs(nxt[v] - cur[v]), f = fabs(nxt[v]);
                    if (df > dmax) dmax = df;
                    if (f > fmax) fmax = f;
                }
                double e = fmax > 0.0 ? dmax / fmax : 0.0;
                double *t = cur; cur = nxt; nxt = t;
                ++it;
                if (fixed_iters_adj) { if (it >= fixed_iters_adj[g]) break; }
                else if (e <= tol || it >= max_iter) break;
            }
            if (iters_adj) iters_adj[b * G + g] = it;
            memcpy(lam + (size_t)g * Nm * C, cur, sizeof(double) * (size_t)Nm * C);
            const double *psg = psi + (size_t)g * N * C;
            const double *phg = phi + (size_t)g * Nm * C;
            for (size_t v = 0; v < C; ++v) {
                const int m = mat[v];
                /* total cross section (cell-centre adjoint x flux of the final sweeps) */
                double sbar = 0.0;
                for (int n = 0; n < N; ++n) sbar -= lc[(size_t)n * C + v] * psg[(size_t)n * C + v];
                double drv = st[(size_t)m * G + g] * sbar;
                /* dQ/drho: within-group scatter, downscatter in, first collision */
                double dx_ = (org[0] + ((v % nx) + 0.5) * dx) - p[0];
                double dy_ = (org[1] + (((v / nx) % ny) + 0.5) * dy) - p[1];
                double dz_ = (org[2] + ((v / ((size_t)nx * ny)) + 0.5) * dz) - p[2];
                double r = sqrt(dx_ * dx_ + dy_ * dy_ + dz_ * dz_);
                double Y[289];
                orc_real_sh(L, dx_ / r, dy_ / r, dz_ / r, Y);
                for (int lm = 0; lm < Nm; ++lm) {
                    double lv = cur[(size_t)lm * C + v];
                    double dq = ss_at(&P, m, lof[lm], g, g) * phg[(size_t)lm * C + v];
                    for (int gp = 0; gp < g; ++gp)
                        dq += ss_at(&P, m, lof[lm], gp, g) * phi[((size_t)gp * Nm + lm) * C + v];
                    for (int gp = 0; gp <= g; ++gp) {
                        double s = ss_at(&P, m, lof[lm], gp, g);
                        dq += s * pu[(size_t)gp * C + v] * Y[lm];
                        /* the first-collision source also weighs the uncollided flux */
                        pbu[(size_t)gp * C + v] += rho[v] * s * Y[lm] * lv;
                    }
                    drv += lv * dq;
                }
                d_rho[v] += drv;
            }
        }
        /* ray back-projection of the uncollided weights, and the group weights */
        int cap = nx + ny + nz + 4;
        int *vox = (int *)malloc(sizeof(int) * cap);
        double *len = (double *)malloc(sizeof(double) * cap);
        for (size_t v = 0; v < C; ++v) {
            double amat[256];
            int any = 0;
            for (int m = 0; m < M; ++m) amat[m] = 0.0;
            for (int g = 0; g < G; ++g) {
                double wu = pbu[(size_t)g * C + v] * pu[(size_t)g * C + v];
                d_gw[g] += pbu[(size_t)g * C + v] * unit[((size_t)b * G + g) * C + v];
                if (wu != 0.0) any = 1;
                for (int m = 0; m < M; ++m) amat[m] += st[(size_t)m * G + g] * wu;
            }
            if (!any) continue;
            double x[3] = {org[0] + ((v % nx) + 0.5) * dx, org[1] + (((v / nx) % ny) + 0.5) * dy,
                           org[2] + ((v / ((size_t)nx * ny)) + 0.5) * dz};
            int ns = orc_siddon(nx, ny, nz, dx, dy, dz, org, p, x, cap, vox, len);
            for (int sgi = 0; sgi < ns; ++sgi) d_rho[vox[sgi]] -= len[sgi] * amat[mat[vox[sgi]]];
        }
        free(vox);
        free(len);
    }
    if (R_out) *R_out = R;
    free(phi_u); free(unit); free(ones); free(phi); free(psi); free(mask); free(dose); free(it_f); free(eps_f);
    free(bal); free(lam); free(pb); free(mu); free(sdir); free(lc); free(cur); free(nxt); free(sigt); free(pbu); free(ext);
    free_prob(&P);
    return 0;
}
