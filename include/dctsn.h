/*
 * dctsn — multigroup discrete-ordinates (S_N) photon fluence and dose solver
 * for CT, gfx950 (MI355X) native.  C ABI.
 *
 * The calls follow the statement of the problem in Norris & Liu,
 * "Photon Fluence and Dose Estimation in Computed Tomography using a Discrete
 * Ordinates Boltzmann Solver" (arXiv:1811.12391):
 *   geometry and materials      Sec. II-B (CT volume -> dosimetric materials), Sec. II-D (meshes)
 *   cross sections              Sec. II-B (cross-section set), Sec. II-D (multigroup library)
 *   quadrature / anisotropy     Sec. II-B, Sec. II-A eq. (3), Sec. II-D (S_N sets, P_N order)
 *   source                      Sec. II-B (point / fan / cone source, position, spectrum,
 *                               azimuthal and polar subtended angles), Sec. II-C
 *   solve                       Sec. II-A eq. (2) with vacuum boundaries, first-collision
 *                               source method, eq. (3) for the scalar fluence; Sec. II-B
 *                               ("Launch Solver" only with complete, consistent input)
 *   dose                        Sec. II-A (collision kerma taken as absorbed dose),
 *                               Sec. III-A (fluence split into uncollided and collided)
 *
 * Conventions shared by every call:
 *   - voxel index v = i + nx*(j + ny*k), x fastest; C = nx*ny*nz;
 *   - group g = 0 is the highest energy;
 *   - real spherical-harmonic moment index lm = l*l + l + m, Nm = (L+1)^2;
 *   - every input pointer is read during the call and never retained
 *     (the library copies what it needs); outputs are caller-allocated;
 *   - a context owns its device memory (hipMalloc on the context's device)
 *     and runs every kernel on the stream given to dct_create;
 *   - any set_* call invalidates earlier results;
 *   - status codes below; on failure dct_last_error() describes the cause.
 * A context is not thread-safe; distinct contexts are independent.
 */
#ifndef DCTSN_H
#define DCTSN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DCT_OK 0
#define DCT_EINVAL (-1)    /* bad argument, size or value */
#define DCT_ESTATE (-2)    /* an input is missing or inputs conflict (Sec. II-B) */
#define DCT_EDEVICE (-3)   /* HIP error or no GPU; message holds the HIP error string */
#define DCT_ENOMEM (-4)    /* device or host allocation failed */
#define DCT_ENOTCONV (-5)  /* max_iter reached before tol in some group; outputs valid */
#define DCT_ENUMERIC (-6)  /* NaN or Inf met in a convergence reduction */

/* Arithmetic of the collided solve.  The ray-traced optical depth, the
 * convergence reductions, the dose tally and the balance sums are FP64 in
 * every mode, except that in DCT_FP32 / DCT_FP32_BF16MAP each sweep row's
 * boundary outflows (at most nx, ny or nz terms) are summed in FP32 before
 * they enter the FP64 leakage sum. */
#define DCT_FP64 0          /* everything FP64 */
#define DCT_FP32 1          /* sweeps, moment maps and moment storage FP32 */
#define DCT_FP32_BF16MAP 2  /* as DCT_FP32, with bf16 inputs to both moment maps
                               (fp32 accumulation) */
#define DCT_FP32_BF16X3 3   /* as DCT_FP32_BF16MAP with every map input and table entry
                               split into its bf16 rounding and the bf16 rounding of the
                               remainder, a b ~ ah bh + ah bl + al bh (three bf16
                               products per term, fp32 accumulation) */

typedef struct dct_ctx dct_ctx;

typedef struct dct_opts {
    int precision;            /* DCT_FP64 / DCT_FP32 / DCT_FP32_BF16MAP / DCT_FP32_BF16X3 */
    double tol;               /* per-group stop: max|dphi_00| / max|phi_00| <= tol */
    int max_iter;             /* per-group iteration cap (>= 1) */
    const int *fixed_iters;   /* [G] or NULL: run exactly this many iterations per group
                                 (ignores tol; used to lock the stopping point) */
    int fixup;                /* 1: set-to-zero negative-flux fixup in the sweep */
    const double *test_inflow;/* [G] or NULL: isotropic angular flux entering through every
                                 boundary face (NULL = vacuum, Sec. II-A) */
    int chunk;                /* iteration sets enqueued between host convergence polls (0 = 4) */
    int use_graph;            /* 1: capture `chunk` iteration sets once in a HIP graph and
                                 replay it until every right-hand side has converged */
    int profile;              /* k >= 1: time every k-th sweep launch (and fused-map launch)
                                 with HIP events (dct_stats); ignored when use_graph = 1 */
    int keep_adjoint;         /* 1: keep every group's final angular flux and fixup pattern
                                 on the device so that dct_adjoint can follow this solve */
    int autotune;             /* 1: time the candidate sweep schedules (z layers per
                                 workgroup x wave coupling) on the first iteration and keep
                                 the fastest for this problem shape in the context */
    int sweep_bk;             /* z layers per sweep workgroup, 1..16 (0 = tuned or min(16, nz)) */
    int sweep_sync;           /* wave coupling: 1 = LDS progress counters between the waves of
                                 a workgroup, 2 = one barrier per step, 3 = as 2 with all
                                 blocks of a sweep in one launch, handing block faces over
                                 as they are produced (needs >= 2 blocks of >= 2 z layers,
                                 otherwise runs as 1), 4 / 5 = layered waves: every wave
                                 sweeps 4 / 2 z layers as a skewed pipeline in registers,
                                 one barrier per step (needs one block: ny <= 64, nz <= 16,
                                 sweep_bk >= nz; otherwise runs as 2; the transposed sweeps
                                 of dct_adjoint then use 2); 6 / 7 / 8 = chained directions
                                 (sweep_chain) with 1 / 2 / 4 z layers per wave; 9 / 10 =
                                 chained right-hand sides (sweep_rhs_chain) with 2 / 1 z
                                 layers per wave; 0 = tuned or 1 */
    int superpose;            /* sources per right-hand side S (0 or 1: one each).  With
                                 S > 1 the B sources of dct_set_source form B / S right-hand
                                 sides of S consecutive sources; each is solved once with
                                 the summed first-collision source of its beams and its dose
                                 adds their uncollided fluences (a CT scan as concurrent
                                 beams in one simulation, Sec. III-C).  Every [B] below then
                                 counts right-hand sides.  EINVAL if S does not divide B or
                                 if keep_adjoint is set with S > 1. */
    int stall_window;         /* reduced-precision stop (DCT_FP32 / DCT_FP32_BF16MAP; the
                                 forward solve's precision for dct_adjoint): a group also stops
                                 once eps <= 10 tol has gone stall_window consecutive
                                 iterations without a new minimum.  In FP32 the set-to-zero
                                 decisions of near-zero outflows flip with rounding and can
                                 hold eps at a few tol for many iterations.  0 = default (4 in
                                 the reduced-precision modes), < 0 = off; never used in FP64.
                                 Such a stop is not DCT_ENOTCONV; stats->eps shows its eps. */
    int sweep_chain;          /* directions chained through one sweep workgroup by couplings
                                 6 / 7 / 8 (1 / 2 / 4 z layers per wave): the K consecutive
                                 directions of one octant are swept back to back, so the
                                 wavefront fills and drains once per K directions.  Needs one
                                 block (ny <= 64, nz <= 16), ny <= nx, keep_adjoint = 0, K
                                 dividing N with every chain inside one octant; otherwise the
                                 solve runs coupling 2.  K in [2, 16]; 0 or 1 = no chaining
                                 (a whole octant when a chained coupling is asked for);
                                 -1 = the autotuner times the chain lengths with the other
                                 candidates.  q and psi then use the chain layout. */
    int fuse_maps;            /* 1: the direction->moment map, the combine (new moments,
                                 convergence, next within-group source) and the
                                 moment->direction map of every iteration run as one kernel
                                 per (z layer, 16 y rows) slab, with the moments and the next
                                 source kept in LDS (DCT_FP64 / DCT_FP32 only; needs the slab
                                 tile, about 16 (L+1)^2 nx words, within the workgroup LDS);
                                 -1: separate kernels; 0: fused when eligible and there are
                                 at least as many slabs over all right-hand sides as the
                                 device has compute units. */
    int warm_start;           /* 1: every group starts its source iteration from the moments
                                 the previous solve on this context left (same right-hand
                                 sides, groups, P_N order, grid and precision; e.g. the next
                                 position of a scan after dct_set_source, or perturbed
                                 densities), instead of from zero; the solve converges to the
                                 same fixed point.  Falls back to zero when shapes differ. */
    int accel_depth;          /* 0: plain source iteration within each group.  m in [1, 4]:
                                 Anderson acceleration of depth m on the scalar-flux moment:
                                 with G_k the moments from the sweep of iterate phi_k and
                                 f_k = G_k - phi_k, the next phi_00 is G_k minus the
                                 combination of the last m differences of G whose f
                                 differences best cancel f_k (least squares over the voxels,
                                 FP64); the higher moments keep G_k.  Converges to the same
                                 discrete solution; eps then measures max|f| / max|G|.  Uses
                                 the separate map and combine kernels (fuse_maps ignored). */
    int sweep_rhs_chain;      /* right-hand sides chained through one sweep workgroup by
                                 couplings 9 / 10 (2 / 1 z layers per wave): one direction of R
                                 unfinished right-hand sides is swept back to back, so the
                                 wavefront fills and drains once per R sources; q, psi and the
                                 results are those of the other schedules.  Needs one block
                                 (ny <= 64, nz <= 16), ny <= nx, nx >= 8, keep_adjoint = 0,
                                 no test_inflow, at least 2 right-hand sides and
                                 B N C sizeof(real) <= 2^31; otherwise the solve runs
                                 coupling 2.  R in [2, 8]; 0 = tuned among 2, 3, 4, 6, 8 (or
                                 min(B, 4) when a chained coupling is asked for without
                                 tuning); 1 = none. */
    int rhs_streams;          /* right-hand sides split in two halves whose iteration sets run
                                 on two streams, so that one half's sweep overlaps the other
                                 half's fused map kernel (the halves are independent; results
                                 are those of one stream bit for bit).  Needs the fused maps,
                                 graph off and layered waves (coupling 4 / 5, B >= 2) or
                                 chained sources (9 / 10, B >= 4: a half's launch keeps the
                                 ceil(B / R) chains per direction of one stream, with
                                 ceil(B_half / ceil(B / R)) sources each, at least 2);
                                 otherwise one stream.  0 = two streams when B N >= 4 x the
                                 compute units, 1 = one stream, 2 = two streams. */
} dct_opts;

typedef struct dct_stats {
    /* caller-owned arrays, each may be NULL ([B] = right-hand sides) */
    int *iters;               /* [B][G] iterations taken */
    double *eps;              /* [B][G] final relative change */
    double *balance;          /* [B][G][3] production, removal, leakage of the final sweep */
    /* filled by the library */
    long long sweep_updates;  /* sum over sweeps of C * N (cell-angle updates, all groups, RHS) */
    int sweep_launches;       /* sweep kernel launches whose time is in sweep_ms */
    double sweep_ms;          /* summed device time of the timed sweep launches (profile > 0) */
    double solve_ms;          /* device time of the whole dct_solve (HIP events) */
    int iteration_sets;       /* iteration launch sets enqueued (>= max over RHS of iterations) */
    int sweep_bk;             /* sweep schedule that ran: z layers per workgroup */
    int sweep_sync;           /* and coupling (1 LDS counters, 2 barriers, 3 pipelined blocks,
                                 4 / 5 layered waves of 4 / 2 z layers, 6 / 7 / 8 chained
                                 directions with 1 / 2 / 4 z layers per wave, 9 / 10 chained
                                 right-hand sides with 2 / 1 z layers per wave) */
    double tune_ms;           /* device time spent timing candidate schedules in this call */
    long long sweep_launches_all; /* sweep kernel launches of the iteration sets (timed or not) */
    int sweep_chain;          /* directions per chained sweep workgroup that ran (1 = none) */
    int fused_maps;           /* 1 when the maps and the combine ran as one kernel */
    int warm_start;           /* 1 when the solve started from the previous solve's moments */
    double fused_ms;          /* summed device time of the timed fused-map launches (profile > 0) */
    int fused_launches;       /* fused-map launches whose time is in fused_ms */
    int sweep_rhs_chain;      /* right-hand sides per chained sweep workgroup (1 = none); R of a
                                 one-stream launch, also with two streams (see rhs_streams) */
    int rhs_streams;          /* streams the iteration sets ran on (1 or 2) */
} dct_stats;

/* Environment read by the library:
 *   DCT_LOG = 0..3      messages to stderr: 1 schedule choices and tuning
 *                       results, 2 also one line per solve, 3 also every
 *                       tuning candidate (read once per process);
 *   DCT_TUNE_CACHE = p  text file of tuned sweep schedules: every tuning
 *                       result is appended to it, and dct_create loads the
 *                       entries made on a device of the same architecture and
 *                       compute-unit count (the last entry of a shape wins). */

/* Create a context on HIP device `device` using `stream` (a hipStream_t; NULL
 * means the device's default stream).  device = -1 creates a host-only
 * context that validates inputs but cannot solve (DCT_EDEVICE from solve). */
int dct_create(dct_ctx **out, int device, void *stream);

/* Release the context and all its device memory.  NULL is accepted. */
int dct_destroy(dct_ctx *ctx);

/* Message of the last failing call on ctx (valid until the next call); ""
 * after success.  A NULL ctx gives the message of the last failed
 * dct_create. */
const char *dct_last_error(const dct_ctx *ctx);

/* Voxel phantom (Sec. II-B: CT volume converted to dosimetric materials;
 * Sec. II-D: rectangular mesh of cubic or box voxels).
 *   nx, ny, nz in [1, 4096] with C = nx ny nz < 2^28 (the kernels use 32-bit
 *   byte offsets into per-voxel FP64 arrays); dx, dy, dz > 0 (cm);
 *   origin[3] = grid corner (cm);
 *   material[C] (uint8, < M of dct_set_xs); density[C] (g/cm^3, finite, >= 0).
 * EINVAL on bad sizes or values. */
int dct_set_geometry(dct_ctx *ctx, int nx, int ny, int nz, double dx, double dy, double dz,
                     const double *origin, const uint8_t *material, const double *density);

/* New voxel densities (Sec. II-B: the density scales every macroscopic cross
 * section) from a DEVICE buffer on the context's device, for callers whose
 * densities already live there (a differentiable pipeline): density[C] FP64
 * g/cm^3, C = nx ny nz of the last dct_set_geometry, whose grid and materials
 * are kept.  The values are screened and copied on the context's stream; the
 * call returns when the copy is done (the caller may then reuse the buffer),
 * and it does not wait for work on other streams that writes the buffer.
 * ESTATE without a geometry; EINVAL on a NULL pointer or a value that is not
 * finite or is negative (the lowest such voxel is named). */
int dct_set_density_dev(dct_ctx *ctx, const double *density);

/* Multigroup cross sections per unit density (Sec. II-B / II-D: multigroup
 * library; eq. (2) with a Legendre expansion of the scattering kernel).
 *   G >= 1 groups, edges_keV[G+1] strictly descending (may be NULL);
 *   M in [1, 8] materials; L in [0, 5] Legendre order;
 *   sigma_t[M][G] cm^2/g total;
 *   sigma_s[M][L+1][G][G] cm^2/g Legendre moments s_l^{g->g'} (from, to),
 *     zero for g' < g (no upscatter);
 *   kerma[M][G] keV cm^2/g, dose = sum_g kerma_g * fluence_g.
 * EINVAL on upscatter entries, negative or non-finite sigma_t / kerma. */
int dct_set_xs(dct_ctx *ctx, int G, const double *edges_keV, int M, int L, const double *sigma_t,
               const double *sigma_s, const double *kerma);

/* Discrete-ordinates quadrature (Sec. II-A eq. (3), Sec. II-D: S_N sets with
 * N(N+2) directions).  dirs[n][3] unit vectors with no zero component,
 * w[n] > 0; n a multiple of 8 when the set is octant-symmetric (not required).
 * ESTATE at solve time if the P_N order L exceeds what the set integrates
 * (checked as D M = I to 1e-10 on the moment maps); EINVAL at solve time if
 * one class of octants (same sign of Omega_x Omega_y) holds more directions
 * than the moment-map tables fit in 64 KiB of LDS (about 160 at P5 in FP64;
 * S16 = 144 per class fits). */
int dct_set_quadrature(dct_ctx *ctx, int n, const double *dirs, const double *w);

/* Collimated isotropic point sources (Sec. II-B: position, energy
 * distribution, azimuthal and polar subtended angles), one right-hand side
 * each, all solved together.
 *   B >= 1; pos[B][3] cm, each outside the voxel grid box;
 *   axis[B][3] beam axis (NULL: toward the z axis, -pos projected on z = 0);
 *     its projection on z = 0 must be non-zero;
 *   fan_deg in (0, 360]: full azimuthal opening about z (360 = no fan limit);
 *   cone_deg in (0, 180]: full polar opening from the z = 0 plane (180 = none);
 *   group_w[G] photons per source photon in each group (one source photon
 *     is emitted isotropically into 4 pi before collimation).
 * Window edges are inclusive. */
int dct_set_source(dct_ctx *ctx, int B, const double *pos, const double *axis, double fan_deg,
                   double cone_deg, const double *group_w);

/* Optional isotropic volumetric source S[G][C] (photons / cm^3 per source
 * photon, the S term of eq. (1)), added to every right-hand side.  NULL
 * removes it. */
int dct_set_volume_source(dct_ctx *ctx, const double *S);

/* Run the whole solve on the device (Sec. II-A): ray-traced uncollided
 * fluence, first-collision source, per-group source iteration with
 * downscatter (g = 0 .. G-1) on diamond-difference sweeps, scalar fluence by
 * quadrature, dose tally.  opts may be NULL (defaults: FP64, tol 1e-6,
 * max_iter 1000, fixup on, vacuum, graph off, profile off); stats may be NULL.
 * Returns ENOTCONV (outputs valid) if some group stopped at max_iter,
 * ENUMERIC on NaN/Inf, ESTATE if an input is missing or inputs conflict. */
int dct_solve(dct_ctx *ctx, const dct_opts *opts, dct_stats *stats);

/* Results of the last solve into caller-allocated HOST buffers ([B] counts
 * the right-hand sides of that solve: sources, or groups of superposed
 * sources).
 *   dose[B][C] (summed = 0) or dose[C] (summed = 1: sum over right-hand
 *     sides), keV/g per source photon;
 *   phi_u[B][G][C] uncollided scalar fluence (summed over superposed sources;
 *     may be NULL);
 *   phi_c[B][G][C] collided scalar fluence phi_00 (may be NULL).
 * ESTATE before a successful solve. */
int dct_dose(dct_ctx *ctx, double *dose, int summed, double *phi_u, double *phi_c);

/* As dct_dose, into DEVICE buffers of the context's device, written on the
 * context's stream (asynchronous). */
int dct_dose_dev(dct_ctx *ctx, double *dose, int summed, double *phi_u, double *phi_c);

/* Fluence-to-dose conversion of the last solve (Sec. III-A: group-wise
 * fluence-to-effective-dose factors interpolated linearly from a table, the
 * dose in air neglected; the paper's table, ICRP 116, is an input here).
 *   n >= 1 table points, energy_keV[n] strictly increasing, factor[n] dose per
 *     unit fluence (e.g. pSv cm^2);
 *   group factor h_g = the table at the group's mid energy (E_g + E_g+1) / 2,
 *     linear between points, the end value beyond either end (needs the
 *     group edges given to dct_set_xs);
 *   zero_material[M] (nonzero: voxels of that material get 0) or NULL;
 *   out[B][C] (summed = 0) or out[C] (summed = 1) HOST buffer:
 *     out_b(v) = sum_g h_g (phi_u,g(v) + phi_00,g(v)).
 * ESTATE before a solve or without group edges; EINVAL on a bad table. */
int dct_effective_dose(dct_ctx *ctx, int n, const double *energy_keV, const double *factor,
                       const uint8_t *zero_material, double *out, int summed);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * dct_effective_dose of the last solve written into a caller-allocated
 * DEVICE buffer out_dev ([B][C] or [C] doubles on the context's device), on
 * the context's stream (asynchronous; the host tables are read before the
 * call returns).  It allocates nothing: the per-group factors and material
 * flags go into a fixed scratch array of the library (2304 bytes per GPU,
 * held until the process ends) instead of context buffers.
 *   Limits: G <= 256, M <= 8 (EINVAL beyond).  Errors as dct_effective_dose.
 *   Every call on one GPU shares that GPU's scratch: calls that overlap on
 *   one GPU (other streams or threads) race and must be serialised by the
 *   caller. */
int dct_effective_dose_noalloc(dct_ctx *ctx, int n, const double *energy_keV, const double *factor,
                               const uint8_t *zero_material, double *out_dev, int summed);

/* The response R = sum_b sum_v roi[v] dose_b(v) of the last solve (the
 * collision-kerma dose of Sec. II-A summed over the right-hand sides, weighted
 * by roi), reduced on the device in FP64 in a fixed order: the value whose
 * gradient dct_adjoint computes.
 *   roi[C] host weights (finite, else EINVAL); R[1] host output.
 * ESTATE if there is no valid solve. */
int dct_roi_dose(dct_ctx *ctx, const double *roi, double *R);

/* Gradient of the response R = sum_b sum_v roi[v] dose_b(v) with respect to
 * every voxel density and every source group weight, by the adjoint of the
 * discretised solve at the converged state of the last dct_solve (which must
 * have run with keep_adjoint = 1): the fixup pattern is frozen, groups are
 * traversed from the lowest energy up, the within-group adjoint is iterated
 * with the transposed maps and reverse-direction sweeps, and the uncollided
 * flux's dependence on every density along each ray is back-projected.
 * (The paper computes the dose only, Sec. II-A; the gradient is an addition
 * built on the same discrete equations.)
 *   roi[C] host weights; opts: tol / max_iter / fixed_iters of the adjoint
 *   iterations (precision is that of the forward solve; NULL = tol 1e-6);
 *   outputs (host, caller-allocated, any may be NULL): R[1] (the forward
 *   solve's response, the value dct_roi_dose gives), d_density[C]
 *   (per g/cm^3), d_group_w[G].
 * ESTATE if there is no kept solve; EINVAL if roi holds a non-finite value. */
int dct_adjoint(dct_ctx *ctx, const double *roi, const dct_opts *opts, double *R, double *d_density,
                double *d_group_w, dct_stats *stats);

/* dct_adjoint with DEVICE buffers on the context's device: roi[C] input,
 * d_density[C] and d_group_w[G] outputs (either may be NULL); R[1] and stats
 * stay host.  The same R bit for bit and the same gradients up to the order
 * of the FP64 atomic additions of the ray back-projection (which varies from
 * run to run in both forms); the call returns when the outputs are written.  EINVAL if roi holds a value that is not finite (the lowest
 * such voxel is named). */
int dct_adjoint_dev(dct_ctx *ctx, const double *roi, const dct_opts *opts, double *R, double *d_density,
                    double *d_group_w, dct_stats *stats);

/* All collided flux moments of the last solve into a host buffer
 * phi[B][G][Nm][C] (B right-hand sides; FP64 whatever the precision). */
int dct_moments(dct_ctx *ctx, double *phi);

#ifdef __cplusplus
}
#endif
#endif /* DCTSN_H */
