/*
 * liblsfft -- FFT-based modified Lippmann-Schwinger solver for periodic
 * linear-elastic composites under a body force with compact support (BFCS),
 * with translated averaging of the solved fields, for AMD MI355X (gfx950).
 *
 * Method: V. A. Buryachenko, "New RVE concept and FFT methods in
 * micromechanics of composites subjected to body force with compact support",
 * arXiv 2601.00822.  Equation numbers below refer to that paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Grid (Sec. 4, Eq. 4.1): nodes x = k h, k_alpha = 0..n_alpha-1, every
 *    n_alpha even.  Supported axis lengths: 4, 6, 8, 12, 16, 24, 32, 48, 64,
 *    96, 128, 256.  2D grids are plane strain.
 *  - Layout: fields are component-major and C-ordered [comp][z][y][x] with x
 *    fastest (2D: [comp][y][x]); vector components (x, y[, z]); symmetric
 *    tensors in Voigt order (11,22,33,23,13,12) in 3D and (11,22,12) in 2D,
 *    tensor (not engineering) shear.  Phase maps are uint8 [z][y][x].
 *  - Precision: a plan computes in FP32 or FP64 (transforms, pointwise
 *    updates, all real and complex fields); the equilibrium residual norm, the
 *    stopping test and the translated-average accumulation are FP64 always.
 *  - Ownership: the caller owns every input and output buffer (device memory
 *    unless stated "host").  The plan owns its workspace (allocated lazily,
 *    grown as needed, freed by lsfft_plan_destroy).  The library never frees
 *    caller memory.
 *  - Synchrony: work is enqueued on the plan's HIP stream; every solve call
 *    returns after its outputs and reports are complete.  A plan is not
 *    re-entrant: use one plan per thread.
 *  - Errors: every argument check runs on the host before any kernel is
 *    launched (phase ids are checked by a small device reduction before the
 *    solve starts).  No exception crosses the ABI.
 *  - Determinism: for a fixed plan, device and input, results are bitwise
 *    reproducible (fixed-order reductions, no floating-point atomics).
 */
#ifndef LSFFT_H
#define LSFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LSFFT_OK = 0,
  LSFFT_W_STAGNATED = 1,   /* residual stopped improving above tol; result holds the last iterate */
  LSFFT_E_ARG = -1,        /* invalid argument (nothing was launched) */
  LSFFT_E_ALLOC = -2,      /* device allocation failed */
  LSFFT_E_DEVICE = -3,     /* HIP runtime error */
  LSFFT_E_NOCONV = -4,     /* max_iter reached; outputs hold the last iterate */
  LSFFT_E_NONEQUIL = -5,   /* LSFFT_STRICT_EQUIL set and the force is not self-equilibrated */
  LSFFT_E_DIVERGED = -6    /* residual became non-finite or grew in 20 consecutive iterations */
} lsfft_status;

typedef enum { LSFFT_F32 = 0, LSFFT_F64 = 1 } lsfft_prec;

/* LSFFT_BASIC: Algorithm 1 (modified basic scheme, Sec. 5, Eqs. 5.7-5.11).
 * LSFFT_CG: conjugate gradients on the displacement form of the same
 * discrete equilibrium system (Algorithm 2's operator in the displacement
 * unknown of Eqs. 5.14-5.22), preconditioned by the reference-medium Green
 * operator; same limit, fewer iterations at high contrast.
 * LSFFT_CG_PLAIN: Algorithm 3 (Sec. 5, Eqs. 5.17-5.22) as printed: the same
 * CG without a preconditioner, started at u1 = b^A (the residual of the free
 * term); the start costs one operator application and is not counted as an
 * iteration.  Same limit; far more iterations than LSFFT_CG (the operator's
 * spectrum spans |xi|^2 times the contrast).  Its stagnation window is 1000
 * iterations instead of 50.
 * LSFFT_ANDERSON: Anderson acceleration (Anderson 1965, in the form of
 * Walker and Ni 2011) of Algorithm 1's fixed-point map in displacement form,
 * one of the accelerated schemes Sec. 5 names for high contrast: with
 * F_k = N0 (i xi . sigma^(u_k) + P f^) the basic step and the differences
 * dF, dU of the last m steps, u_{k+1} = u_k + F_k - sum_j gamma_j (dU_j + dF_j),
 * gamma minimizing ||F_k - sum_j gamma_j dF_j|| (Parseval-weighted; FP64
 * normal equations).  Memory m = 5 unless set by lsfft_anderson_memory;
 * same stopping rule and limit as the basic scheme; two outer-axis launches
 * per iteration and 2 m + 1 extra displacement-sized fields per solve. */
typedef enum { LSFFT_BASIC = 0, LSFFT_CG = 1, LSFFT_CG_PLAIN = 2, LSFFT_ANDERSON = 3 } lsfft_scheme;

/* plan flags */
#define LSFFT_STRICT_EQUIL 0x1u  /* reject forces whose voxel sum is not ~0 (Eq. 2.5) instead of projecting */
#define LSFFT_TIMING       0x2u  /* time every kernel launch with a HIP event pair stamped at the kernel's start and end (see lsfft_kernel_times) */
/* LSFFT_REFINE64 (LSFFT_F32 plans only): mixed-precision defect correction.
 * The displacement state is kept in FP64; each outer step evaluates the FP64
 * residual P f + div(L sym grad u) of that state (the stopping rule below is
 * applied to it), solves the correction equation with that residual as its
 * force in FP32 with the plan's scheme to a relative residual of
 * 0.3 tol / (current FP64 residual), kept within [3e-5, 0.1] and not below
 * 1.5 times the level where an earlier inner solve of the same solve
 * stagnated, and adds the correction in FP64.  The FP32 rounding floor then limits only the
 * progress per step, so tol = 1e-8 is reachable at any contrast.  Reports:
 * iters = FP32 iterations summed over the inner solves, residual = FP64
 * residual of the returned state, at most 40 outer steps (else
 * LSFFT_E_NOCONV).  Outputs are the FP64 state rounded once to FP32 and
 * materialized in FP32.  The plan holds an FP64 companion workspace
 * (about 18 complex FP64 half-spectrum fields per solve) and max_batch must
 * not exceed 65535. */
#define LSFFT_REFINE64     0x4u

typedef struct {
  int dim;          /* 2 or 3 */
  int64_t n[3];     /* (nx, ny, nz); nz ignored (treated as 1) when dim == 2 */
  double h[3];      /* grid spacing per axis (> 0); the unit of length of u */
} lsfft_grid;

typedef struct {
  int nphase;            /* 1..256 */
  const double* lame;    /* host, [nphase][2] = (lambda, mu); mu > 0, lambda + 2 mu / d > 0 */
} lsfft_phases;

/* Reference medium L0 of Algorithm 1.  NaN in both fields selects the default
 * (mean of the smallest and largest Lame constants over the phases). */
typedef struct {
  double lambda0, mu0;
} lsfft_ref;

typedef struct {
  int iters;               /* Green updates applied (basic) or CG updates */
  double residual;         /* ||i xi . sigma^ + P f^|| / ||P f^|| of the returned iterate (FP64) */
  double removed_mean[3];  /* voxel mean of the force removed by the projection onto Eq. 2.5 */
  int status;              /* lsfft_status of this solve */
  double seconds;          /* wall time of the batch this solve ran in */
} lsfft_report;

typedef struct lsfft_plan_s* lsfft_plan_t;

/*
 * lsfft_plan -- create a plan for solves on the given grids.
 *  out        host, receives the plan handle (NULL on failure)
 *  grids      host [ngrid]; every axis length must be supported
 *  max_batch  largest number of solves (or shifts) run concurrently; larger
 *             requests are processed in successive batches (>= 1)
 *  prec       an lsfft_prec value, scheme an lsfft_scheme value (passed as
 *             int so that any value a caller holds is checked, not assumed)
 *  hip_stream hipStream_t to enqueue on (NULL = the null stream)
 * Errors: LSFFT_E_ARG for an unsupported grid, ngrid < 1, max_batch < 1,
 * an unknown precision, scheme or flag, LSFFT_REFINE64 on an LSFFT_F64 plan or with max_batch >
 * 65535; LSFFT_E_DEVICE if no HIP device is usable.
 */
lsfft_status lsfft_plan(lsfft_plan_t* out, const lsfft_grid* grids, int ngrid, int max_batch,
                        int prec, int scheme, unsigned flags, void* hip_stream);

/*
 * lsfft_solve_bfcs -- solve the modified Lippmann-Schwinger equation
 * (Eq. 2.14; Algorithm 1 or its CG variant) for nsolve independent problems,
 * run as one batch: material L(x) = table[phase(x)], reference medium c0,
 * body force f (projected onto the self-equilibrated subspace, Eq. 2.5),
 * free term u^b = G0 * f (Eqs. 2.8-2.9), stopping rule ||div sigma + Pf|| /
 * ||Pf|| <= tol (Eq. 5.11 adapted to body-force loading).  The returned
 * iterate is the first one meeting the rule.
 *  grid_idx  host [nsolve], index into the plan's grids
 *  phase     host array [nsolve] of device pointers, uint8 [nz][ny][nx]
 *  tab       host [nsolve] phase tables
 *  c0        host [nsolve] reference media, or NULL for the default of each
 *  f         host array [nsolve] of device pointers, force [d][N] in the plan precision
 *  tol       > 0
 *  max_iter  >= 0
 *  eps, sig  host arrays [nsolve] of device pointers [s][N] (plan precision),
 *            or NULL; an individual entry may be NULL to skip that output
 *  u         host array [nsolve] of device pointers [d][N], or NULL
 *  u_init    NULL (every solve starts from the free term u^b), or a host
 *            array [nsolve] of device pointers, starting displacements
 *            [d][N] in the plan precision, one for every solve: the
 *            iteration starts from their spectra projected off the xi = 0
 *            set (the mean displacement is not determined).  Warm starts
 *            need the basic scheme without LSFFT_REFINE64 (else LSFFT_E_ARG)
 *  rep       host [nsolve], filled on every return except LSFFT_E_ARG
 * Returns the worst per-solve status (errors before warnings before OK).
 */
lsfft_status lsfft_solve_bfcs(lsfft_plan_t p, int nsolve, const int* grid_idx,
                              const uint8_t* const* phase, const lsfft_phases* tab,
                              const lsfft_ref* c0, const void* const* f, double tol, int max_iter,
                              void* const* eps, void* const* sig, void* const* u,
                              const void* const* u_init, lsfft_report* rep);

/*
 * lsfft_translate_average -- translated (ensemble) averages of Sec. 3
 * (Eqs. 3.3-3.7): the microstructure is rigidly shifted by each chi
 * (phase_chi(x) = phase(x - chi)), the force stays fixed, every shifted
 * problem is solved, and
 *   avg = (1/nshift) sum_chi [u, u V, eps, eps V, sigma, sigma V, V]
 * with V the indicator of phase incl_phase in the shifted microstructure.
 *  shifts  host [nshift][dim] in (x, y[, z]) order, 0 <= shift_a < n_a
 *  avg     device FP64 [2d + 4s + 1][N] (overwritten); component order
 *          u[d], u1[d], eps[s], eps1[s], sig[s], sig1[s], occupancy[1]
 *  rep     host [nshift], per shift
 */
lsfft_status lsfft_translate_average(lsfft_plan_t p, int grid_idx, const uint8_t* phase,
                                     const lsfft_phases* tab, const lsfft_ref* c0, const void* f,
                                     const int32_t* shifts, int nshift, int incl_phase, double tol,
                                     int max_iter, double* avg, lsfft_report* rep);

/* One averaging group of lsfft_translate_average_batch. */
typedef struct {
  int grid_idx;
  const uint8_t* phase;       /* device */
  const lsfft_phases* tab;    /* host */
  const lsfft_ref* c0;        /* host or NULL */
  const void* f;              /* device force */
  const int32_t* shifts;      /* host [nshift][dim] */
  int nshift;
  int incl_phase;
  double* avg;                /* device FP64 [2d + 4s + 1][N] */
} lsfft_avg_group;

/*
 * lsfft_translate_average_batch -- several averaging groups (different
 * microstructures, forces and grid sizes) solved together as batches of up
 * to max_batch solves; rep is host [sum of nshift], groups in order.
 */
lsfft_status lsfft_translate_average_batch(lsfft_plan_t p, int ngroup, const lsfft_avg_group* groups,
                                           double tol, int max_iter, lsfft_report* rep);

/*
 * lsfft_realization_average -- the deterministic-structure dataset of Sec. 3
 * (Eq. 3.8): the force stays fixed and the ensemble average runs over
 * realisations X^j of the microstructure (separate phase maps of one grid,
 * e.g. samples of a CT image), each solved unshifted:
 *   avg = (1/nreal) sum_j [u, u V, eps, eps V, sigma, sigma V, V]
 * with V the indicator of phase incl_phase in realisation j.  The
 * realisations share the phase table (and with it the reference medium)
 * and one force spectrum; they are solved in batches of up to max_batch.
 *  phases  host array [nreal] of device phase maps [N]
 *  f       device force [d][N] in the plan precision
 *  avg     device FP64 [2d + 4s + 1][N] (overwritten), component order as
 *          for lsfft_translate_average
 *  rep     host [nreal], per realisation
 * Errors: LSFFT_E_ARG for a null map or pointer, nreal < 1, a bad table,
 * incl_phase outside the table, tol <= 0 or a phase id outside the table.
 */
lsfft_status lsfft_realization_average(lsfft_plan_t p, int grid_idx, int nreal, const uint8_t* const* phases,
                                       const lsfft_phases* tab, const lsfft_ref* c0, const void* f,
                                       int incl_phase, double tol, int max_iter, double* avg,
                                       lsfft_report* rep);

/* Result of lsfft_rve_identify. */
typedef struct {
  double radius;      /* B^RVE: both magnitudes stay below tol times their
                         maxima at distances >= radius; HUGE_VAL if the
                         outermost bin is still above */
  double box_radius;  /* radius of the largest ball in the cell, min_a n_a h_a / 2 */
  int fits;           /* 1 when radius + support_radius / 2 <= box_radius */
  int nbins;          /* bins used; bin b holds distances [b dr, (b + 1) dr) */
  double max_eps;     /* largest |eps| over the grid */
  double max_sig;     /* largest |sigma| over the grid */
} lsfft_rve;

/*
 * lsfft_rve_identify -- the RVE of Definition 2.2 (Sec. 3) from averaged
 * fields: with the body force's support centred at `center`, the RVE is the
 * ball about it outside which the averaged strain and stress vanish to the
 * relative tolerance `tol`, and the body-force unit cell is large enough
 * when the annulus of width support_radius / 2 around the RVE, where the
 * fields must stay stabilized, still lies inside the periodic cell.
 * Magnitudes are |t| = sqrt(sum_ab t_ab^2) (Voigt shear counted twice);
 * distances are minimum-image distances in the periodic cell in the grid's
 * spacing; the radial profile holds the largest magnitude per bin of width dr.
 *  avg       device FP64 [2d + 4s + 1][N], the layout of lsfft_translate_average
 *  center    host [dim] in (x, y[, z]) order, voxel units
 *  profile   host [2][max_bins] (|eps| maxima, then |sigma| maxima) or NULL;
 *            filled when max_bins >= out->nbins
 * Errors: LSFFT_E_ARG for null pointers, tol outside (0, 1), dr <= 0 or
 * more than 1024 bins.
 */
lsfft_status lsfft_rve_identify(lsfft_plan_t p, int grid_idx, const double* avg, const double* center,
                                double support_radius, double tol, double dr, double* profile, int max_bins,
                                lsfft_rve* out);

/*
 * lsfft_rve_identify_noalloc -- lsfft_rve_identify for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * lsfft_rve_identify; it allocates nothing: the radial maxima live in a fixed
 * device array inside the library (one per GPU, 2 x 1024 64-bit words =
 * 16 KiB, held until the process ends), cleared by a fill kernel at the start
 * of every call and read back into a stack buffer.
 * Limits: at most 1024 bins (LSFFT_E_ARG beyond, as for lsfft_rve_identify).
 * Every call on one GPU shares that GPU's array, so calls that overlap on
 * one GPU (from several threads or plans) race; serialise them.
 * LSFFT_E_DEVICE if the array's address could not be looked up on the plan's
 * device when the plan was made.  The call still synchronises the plan's
 * stream to return its results.
 */
lsfft_status lsfft_rve_identify_noalloc(lsfft_plan_t p, int grid_idx, const double* avg, const double* center,
                                        double support_radius, double tol, double dr, double* profile,
                                        int max_bins, lsfft_rve* out);

/*
 * lsfft_kernel_convolve -- periodic convolution of forces with a kernel of
 * the plan's grid, through the plan's own transforms (Sec. 6 dataset: with
 * every shift of a cell, the translated average of Eqs. 3.3-3.6 is linear
 * and commutes with grid translations, so it is the convolution of the
 * force with the averaged response to a point force at the origin):
 *   out_c = sum_j K_cj * P f_j   (c < s, j < d; * the periodic convolution,
 *                                 P the projection off the xi = 0 set)
 *  kernel  device [s][d][N] in the plan precision: K_cj = strain component c
 *          (Voigt order) of the response to a unit force along axis j at the
 *          origin voxel
 *  f       host array [nforce] of device pointers, forces [d][N]
 *  out     host array [nforce] of device pointers, results [s][N]
 * Runs in batches of up to max_batch forces; synchronous.  LSFFT_E_ARG for
 * null pointers, nforce < 1 or a bad grid index.
 */
lsfft_status lsfft_kernel_convolve(lsfft_plan_t p, int grid_idx, const void* kernel, int nforce,
                                   const void* const* f, void* const* out);

/*
 * lsfft_block_mean -- block means of `nfield` fields [nz][ny][nx]
 * (n = (nx, ny, nz), nz = 1 for 2D): out[f][Z][Y][X] = scale x the mean of
 * the factor^d fine voxels of block (X, Y, Z) (factor^2 when nz = 1), FP64
 * sums, rounded once to the output type; with factor 1 a scaled copy (and a
 * precision conversion).  prec / out_prec: LSFFT_F32 or LSFFT_F64, the types
 * of the device arrays in and out.  Every n_a > 1 must be a multiple of
 * factor.  Synchronises hip_stream.
 */
lsfft_status lsfft_block_mean(int prec, int out_prec, int nfield, const int64_t* n, int factor, double scale,
                              const void* in, void* out, void* hip_stream);

/*
 * lsfft_sample_norms -- per-sample Euclidean norms of nsample device arrays
 * of len values (sample s at offset s x len): norm_diff[s] = ||y_s - t_s||
 * (||t_s|| when y is NULL) and norm_t[s] = ||t_s||, FP64 sums in a fixed
 * order (host outputs, either may be NULL).  Allocates a small device buffer.
 */
lsfft_status lsfft_sample_norms(int prec, int nsample, int64_t len, const void* y, const void* t, double* norm_diff,
                                double* norm_t, void* hip_stream);

/*
 * lsfft_bump_forces -- body forces with compact support (Eq. 2.5's loading)
 * made of smooth bumps: force i = sum over its nbump[i] bumps of
 * exp(-1 / (1 - r^2 / R^2)) dir for r < R (zero outside), r the
 * minimum-image distance from the node to the bump's centre in the periodic
 * cell (voxel units).  bumps: host, per bump (centre x, y[, z], R,
 * dir x, y[, z]), forces in order; f: host array [nforce] of device
 * pointers [d][N] (overwritten).  Allocates a small device buffer.
 */
lsfft_status lsfft_bump_forces(int prec, int dim, const int64_t* n, int nforce, const int* nbump,
                               const double* bumps, void* const* f, void* hip_stream);

/*
 * Nonlocal kernel surrogate (Sec. 6, Eqs. 6.5-6.6).  The operator on the
 * periodic grid (h = 1):
 *   L_c[u](x) = sum over offsets r, 0 < |r| < delta, of K(r) (u(x + r) - u(x)),
 * with, by `form`:
 *   0  K(r) = K1(|r|) I                       (a scalar radial kernel on
 *                                              every component alike)
 *   1  K(r) = K1(|r|) I + K2(|r|) e e^T,      e = r / |r| (components x
 *                                              first): the isotropic matrix
 *                                              kernel of the bond (Eq. 6.7
 *                                              pairs the paper's kernels with
 *                                              the bond vector)
 *   Kj(rho) = sum_m cj_m B_{m,M}(rho / delta),  B_{m,M}(t) = C(M, m) t^m (1 - t)^(M - m);
 * coefficients c = (c1_0..c1_M[, c2_0..c2_M]), nc = (form + 1)(M + 1).
 * The fit of Eq. 6.6 to pairs (u_k, Gamma_k) minimises
 *   sum_k ||L_c[u_k] - Gamma_k||^2 + lam ||c||^2,
 * a quadratic in c: (G + lam I) c = g with G_ij = sum_k <Phi_i[u_k], Phi_j[u_k]>,
 * g_i = sum_k <Phi_i[u_k], Gamma_k>, Phi_i[u] = L_{e_i}[u] the features.
 * Horizon: 1 < delta <= 7 (voxels; at most 5 for the 3D normal equations of
 * form 1); degree M: 0..8.  Grids n = (nx, ny[, nz]), any positive sizes;
 * fields are [nsample][d][N] contiguous, in prec.
 */

/* The normal equations over nsample pairs, in FP64 (fixed summation order):
 *  u, gamma  device [nsample][d][N] (gamma: the operator type's response,
 *            -b_k for the displacement type)
 *  G         host [nc^2], row major, symmetric
 *  g         host [nc];  gg  host, sum_k ||Gamma_k||^2
 * Allocates a small device buffer; synchronises hip_stream.  LSFFT_E_ARG for
 * bad sizes, a form other than 0 or 1, a horizon outside its range or null
 * pointers. */
lsfft_status lsfft_nonlocal_normal_equations(int prec, int dim, const int64_t* n, int nsample, const void* u,
                                             const void* gamma, int degree, int form, double delta, double* G,
                                             double* g, double* gg, void* hip_stream);

/* out = L_c[u] for nsample fields (device [nsample][d][N] each, in prec; out
 * must not overlap u); c host [nc].  Allocates a small device buffer;
 * synchronises hip_stream. */
lsfft_status lsfft_nonlocal_apply(int prec, int dim, const int64_t* n, int nsample, const void* u, int degree,
                                  int form, const double* c, double delta, void* out, void* hip_stream);

/* Coefficients c (host [ncoef], 1 <= ncoef <= 18) of Eq. 6.6 from the normal
 * equations G (host [ncoef^2]) and g (host [ncoef]), host arithmetic, no
 * device use: adam_steps = 0 solves (G + lam I) c = g by Cholesky
 * (LSFFT_E_ARG if that matrix is not positive definite); adam_steps > 0 runs
 * that many Adam steps of size lr from c = 0 on the quadratic loss (beta1
 * 0.9, beta2 0.999, eps 1e-12, bias-corrected). */
lsfft_status lsfft_nonlocal_fit(int ncoef, const double* G, const double* g, double lam, int adam_steps, double lr,
                                double* c);

/* Memory m (1..8) of LSFFT_ANDERSON plans for later solves (default 5);
 * LSFFT_E_ARG outside that range. */
lsfft_status lsfft_anderson_memory(lsfft_plan_t p, int m);

/* Release the plan and its workspace.  NULL is accepted. */
lsfft_status lsfft_plan_destroy(lsfft_plan_t p);

/* Static, human-readable text for a status code.  Takes a plain int so that
   any value a caller holds is valid input; codes the library does not define
   give "unknown status". */
const char* lsfft_status_string(int status);

/* Isotropic (E, nu) pairs to Lame pairs (lambda, mu); host [nphase][2] each.
 * Returns LSFFT_E_ARG for nu outside (-1, 0.5) or E <= 0. */
lsfft_status lsfft_lame_from_young(int nphase, const double* e_nu, double* lame_out);

/* Kernel classes timed under LSFFT_TIMING. */
typedef enum {
  LSFFT_K_XPASS = 0,  /* x sweep: C2R, Hooke's law, R2C */
  LSFFT_K_YPASS = 1,  /* y sweeps (3D) */
  LSFFT_K_GREEN = 2,  /* outer-axis sweep fused with the Green/body-force update */
  LSFFT_K_REDUCE = 3, /* FP64 residual reduction and stopping rule */
  LSFFT_K_CGUPD = 4,  /* CG vector update */
  LSFFT_K_OTHER = 5,  /* setup, materialize, averaging */
  LSFFT_K_COUNT = 6
} lsfft_kernel_class;

/* Accumulated device time (ms) and launch count of one kernel class, restricted
 * to the iteration loop, since the last reset.  Requires LSFFT_TIMING. */
lsfft_status lsfft_kernel_times(lsfft_plan_t p, int kernel_class, double* total_ms, int64_t* launches);
lsfft_status lsfft_kernel_times_reset(lsfft_plan_t p);

/* Algorithmic HBM bytes that one iteration of one solve on grid grid_idx
 * moves in each kernel class (complex half-spectrum streams and phase map). */
lsfft_status lsfft_iteration_bytes(lsfft_plan_t p, int grid_idx, int kernel_class, double* bytes);

/*
 * Schedules and autotuning of the batched FFT passes (the plan-level
 * choice of tile and radix schedule per transform length).  A pass kind is
 * 0 (x pass), 1 (y pass) or 2 (outer pass).  Each (precision, dimension,
 * kind, length) has a number of compiled schedule variants; variant 0 is the
 * hand-tuned default and FP32 3D plans have 3 variants per pass for lengths
 * of 32 points and more (outer pass: default tile, half the pencils, twice
 * the pencils; y pass: default, twice the pencils, the other radix order; x
 * pass: default, row tiles of half the entries, the other radix order).
 * Every variant computes the same transforms; results differ only by
 * rounding order.
 *
 * Kind 3 is the spectral layout of one grid, `len` being the grid's index
 * in the plan: variant 0 keeps the spectra in rows of nx/2 entries
 * throughout (the default of FP64 plans); variant 1 (the default of FP32
 * plans, for 3D grids with nx a multiple of 16) keeps them between the y
 * and outer passes in 8-wide kx blocks, entry
 * (kx, y, z) at ((kx/8) ny + y) 8 nz + 8 z + kx mod 8, so that each outer
 * transform tile reads and writes contiguous blocks; the y passes then
 * convert between the two layouts out of place, and each such solve holds
 * s + d more spectral components of workspace.  Other grids have variant 0
 * only.  The layout changes addressing only: a basic-scheme solve's fields
 * are bit for bit the same under both (the residual sums, taken in another
 * tile order, may differ in the last bits).
 */
typedef struct {
  int kind;       /* 0 x pass, 1 y pass, 2 outer pass, 3 spectral layout */
  int len;        /* transform length; for kind 3 the grid's index in the plan */
  int variant;
  int chosen;     /* 1 for the variant the plan now uses */
  double us;      /* mean kernel time per launch in microseconds, summed over the plan's grids sharing that length;
                     kind 3: kernel time of the x, y and outer passes per iteration of the tuning batch */
} lsfft_tune_entry;

/* Current variant and number of variants of one pass of the plan's 3D (or
 * 2D) grids on an axis of `len` points (kind 3: of the layout of grid
 * `len`, whose dimension must be `dim`).  LSFFT_E_ARG for a bad kind,
 * dimension, unsupported length or grid index. */
lsfft_status lsfft_schedule_get(lsfft_plan_t p, int dim, int kind, int len, int* variant, int* nvariants);

/* Select a variant explicitly (0 <= variant < nvariants, else LSFFT_E_ARG);
 * applies to the plan's later solves (kind 3: to its FP64 companion's too).
 * 2D grids keep variant 0. */
lsfft_status lsfft_schedule_set(lsfft_plan_t p, int dim, int kind, int len, int variant);

/*
 * lsfft_autotune -- time every schedule variant of the plan's 3D grids and
 * keep the fastest per pass kind and length.  For each distinct 3D grid a
 * batch of identical synthetic solves (two phases of Young's contrast 10 in
 * 8-voxel blocks, a deterministic pseudo-random force; as many solves as
 * fill about 64 M voxels, at most the plan's max_batch, so a plan of one
 * solve is tuned on one solve) runs `iters` iterations (1..10000) once per
 * variant round with every launch timed by a HIP event pair; each pass kind
 * is judged by its own mean kernel time per launch.  A grid that has two
 * spectral layouts runs its rounds under each; it keeps the layout whose
 * fastest variants give the smaller kernel time of the x, y and outer
 * passes per iteration, and the variants are chosen on the times under the
 * chosen layouts.  The plan's own precision and scheme are used (FP32 inner
 * solves for LSFFT_REFINE64).
 *  cache_path  NULL, or a file to merge the choices into: a flat JSON object
 *              {"f32/3d/outer/256": 2, "f32/3d/layout/256x256x256": 1, ...}
 *              (layouts keyed by nx x ny x nz); lsfft_plan reads the file
 *              named by the environment variable LSFFT_TUNE_CACHE and applies
 *              the entries matching its grids
 *  out         host [max_out] or NULL: every variant timed (kind, length,
 *              variant, chosen flag, microseconds), *nout entries in all
 * Allocates device memory for the synthetic inputs; synchronises the plan's
 * stream.  LSFFT_E_ARG for bad arguments or a cache file that cannot be
 * written.  FP64 plans tune the layout only (their passes have one variant
 * each); 2D grids have nothing to tune (*nout = 0).
 */
lsfft_status lsfft_autotune(lsfft_plan_t p, int iters, const char* cache_path, lsfft_tune_entry* out, int max_out,
                            int* nout);

/* The cached variant for (precision, dimension, kind 0..2, length) in the
 * text of a schedule cache, or -1 if there is no valid entry (host only, no
 * GPU). */
int lsfft_tune_cache_lookup(const char* json_text, int prec, int dim, int kind, int len);

#ifdef __cplusplus
}
#endif

#endif /* LSFFT_H */
