/*
 * ffth.h - C-ABI of libffth, an MI355X (gfx950) implementation of FFT-based
 * numerical homogenization of orders 0 and 1:
 *
 *   F. Dietrich, D. Merkert, B. Simeon, "Derivation of higher-order terms in
 *   FFT-based numerical homogenization", arXiv:1712.05145.
 *
 * The library solves, on a periodic voxel grid of the unit cell [-1/2,1/2)^3
 * (Sec. 2), the linear system of eq. (6)
 *
 *      (Id + Gamma0 * (C - C0)) : eps = -Gamma0 * P_rhs
 *
 * with P_rhs = C:E for the classical cell problem ("order 0", the paper's
 * alpha = 1, Sec. 3 Definition) and P_rhs = p_2 + theta_2 for the
 * strain-gradient problem ("order 1", alpha = 2, built from the six order-0
 * correctors, Sec. 3 and eq. (12)).  Two iterations are offered: the Basic
 * Scheme (fixed point of eq. (5)) and conjugate gradients on eq. (6)
 * (Algorithm 1, CG version), in FP64, FP32, or FP32 with an FP64
 * defect-correction outer loop.
 *
 * Conventions (fixed by this library where the paper is silent):
 *   grid      n[3] voxels, C order, grid axis d carries x_{d+1}; voxel centres
 *             -1/2 + (j + 1/2)/n_d; every n_d even and in the supported set
 *             (ffth_size_supported), except n0 = 1 (2-D problems, Sec. 4).
 *   fields    strain-like fields are 6 tensor components per voxel in the
 *             order (11, 22, 33, 23, 13, 12), stored component-major:
 *             field[c * N + voxel], N = n0*n1*n2.
 *   E         macroscopic strain as an engineering Voigt 6-vector
 *             (e11, e22, e33, 2e23, 2e13, 2e12).
 *   G         strain-gradient load G[J*3 + j] = dE_kl/dY_j for the Voigt
 *             pair J = (k,l), tensor components.
 *   stiffness per phase, either (lambda, mu) or 21 upper-triangular Voigt
 *             coefficients C_11..C_16, C_22..C_26, ..., C_66 (engineering
 *             shear).
 *   DFT       forward exp(-2 pi i k.j/n), xi = 2 pi k; every mode with an index
 *             k_d = -n_d/2 is zero in the output of every spectral operator;
 *             the zero frequency is zero in the Green operator output.
 *   residual  ||b - A eps||_L2 / ||b||_L2 (equal to the Cauchy criterion stated
 *             after Algorithm 1 for the Basic Scheme).
 *
 * Memory ownership: every device buffer (phase ids, correctors, outputs and
 * the workspace) is allocated and freed by the caller.  The library never
 * allocates device memory; a plan owns host state only.  Host arrays passed
 * in are copied before the call returns.
 *
 * Errors: every call returns an ffth_status; arguments are validated before
 * any device work is queued.  On FFTH_ERR_NOT_CONVERGED / FFTH_ERR_DIVERGED the
 * output holds the last iterate and the result records are filled.  A plan is
 * not thread-safe: use one plan per host thread and stream.
 */
#ifndef FFTH_H
#define FFTH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FFTH_OK = 0,
  FFTH_ERR_INVALID = 1,        /* bad argument (sizes, reference medium, pointers)  */
  FFTH_ERR_OOM = 2,            /* workspace smaller than ffth_workspace_bytes()     */
  FFTH_ERR_NOT_CONVERGED = 3,  /* max_iter reached                                  */
  FFTH_ERR_DIVERGED = 4,       /* residual not finite or grew by more than 1e6      */
  FFTH_ERR_DEVICE = 5,         /* HIP runtime error or no usable device             */
  FFTH_ERR_BUSY = 6,           /* request still running (serving)                   */
  FFTH_ERR_CANCELLED = 7       /* request cancelled (serving)                       */
} ffth_status;

/* FFTH_BICGSTAB: BiCGSTAB on eq. (6), the Krylov method of the paper's
 * experiments (Sec. 4); FP64 or FP32 precision only.
 * FFTH_CG3: CG on eq. (6) in the C0 inner product through the three-term
 * (Rutishauser) recurrence, started from eps_0 = 0: the same iterates as
 * two-term CG from zero in exact arithmetic, one HBM pass fewer per
 * iteration (the update, its reductions and the next polarization share one
 * pass); FP64 or FP32 precision only (FFTH_MIXED runs it inside its FP32
 * inner solves already). */
typedef enum { FFTH_BASIC = 0, FFTH_CG = 1, FFTH_BICGSTAB = 2, FFTH_CG3 = 3 } ffth_scheme;
typedef enum { FFTH_FP64 = 0, FFTH_FP32 = 1, FFTH_MIXED = 2 } ffth_precision;

/* The cell problem of Sec. 2: stiffness field C(x) = table[phase[x]] with
 * major and minor symmetries, and the isotropic reference medium C0 with
 * Lame parameters (lambda0, mu0).  mu0 != 0 and lambda0 + 2 mu0 != 0 are
 * required (the Green operator formula below eq. (5) divides by both); the
 * CG schemes also need mu0 > 0 and 3 lambda0 + 2 mu0 > 0 (positive C0). */
typedef struct {
  int32_t n[3];               /* voxels per axis                                       */
  int32_t nphases;            /* entries in the phase table (1..65535)                 */
  const uint16_t *phase;      /* DEVICE, n0*n1*n2 ids < nphases, caller-owned; must stay
                                 valid for the lifetime of the plan                    */
  const double *lame;         /* HOST, nphases x 2 (lambda, mu), or NULL               */
  const double *stiffness;    /* HOST, nphases x 21 Voigt upper triangle, or NULL;
                                 exactly one of lame / stiffness is non-NULL           */
  double lambda0, mu0;        /* reference medium C0                                   */
} ffth_problem;

typedef struct {
  int32_t scheme;             /* ffth_scheme                                           */
  int32_t precision;          /* ffth_precision                                        */
  double tol;                 /* relative equilibrium residual to reach (e.g. 1e-8)    */
  int32_t max_iter;           /* iterations (FP64/FP32) or total inner iterations      */
  double inner_tol;           /* MIXED: tightest residual reduction asked of one FP32
                                 inner solve; the reduction the outer residual still
                                 needs (half the tolerance) is split evenly over the
                                 fewest solves that reach it at this bound            */
  int32_t max_outer;          /* MIXED: FP64 defect-correction sweeps (each sweep after
                                 the first also projects the residual onto compatible
                                 fields, one FP32 operator application)                */
  int32_t check_every;        /* iterations between host reads of the convergence flags */
  int32_t autotune;           /* 1: time the compiled tile shapes of every pass at plan
                                 creation (grids >= 64^3) and keep the fastest          */
  int32_t spectrum16;         /* MIXED CG: 1 keeps the FP32 inner solve's spectrum in
                                 binary16 from the forward transforms up to the Green
                                 operator (FP32 arithmetic, scaled into range; FP32
                                 after the operator), on grids of at least
                                 FFTH_SPECTRUM16_MIN_VOXELS voxels whose stiffness
                                 contrast (ffth_stiffness_contrast) is at most
                                 FFTH_SPECTRUM16_MAX_CONTRAST; 2: also on smaller
                                 grids (the contrast limit still applies: above it
                                 the perturbed inner operator can stall the inner
                                 solves); 0: FP32 throughout.  The FP64 defect
                                 correction sets the final accuracy                    */
} ffth_opts;

typedef struct {
  int32_t status;             /* ffth_status of this load case                         */
  int32_t iters;              /* operator applications in the iteration (FP32 inner
                                 ones for MIXED)                                       */
  int32_t outer_iters;        /* MIXED: FP64 residual sweeps; else 0                    */
  int32_t fp64_applications;  /* FP64 operator applications (incl. the right-hand side) */
  int32_t projections;        /* MIXED: FP32 compatible projections of the FP64 residual
                                 (one FFT round trip each); else 0                       */
  int32_t reserved;
  double residual;            /* final relative residual (FP64 true residual for MIXED) */
  double mean_stress[6];      /* order 0: Voigt <C:(E+eps)>; order 1: <C:eps + p_2>     */
  double g_mean[3];           /* order 1: the dropped mean <g> of the body force        */
  double seconds;             /* wall time of the call this load belonged to            */
} ffth_result;

typedef struct ffth_plan ffth_plan;

/* Default options: CG, MIXED, tol 1e-8, max_iter 20000, inner_tol 1e-3,
 * max_outer 30, check_every 8, autotune 1, spectrum16 1. */
void ffth_default_opts(ffth_opts *o);

/* Stiffness contrast of the phases of a problem (Sec. 2's stiffness table):
 * the largest eigen-modulus over the smallest, across all phases, where the
 * eigen-moduli of a phase are the eigenvalues of its stiffness in Mandel form
 * (Voigt matrix with the shear rows and columns scaled by sqrt 2; 3 lambda +
 * 2 mu and five times 2 mu for isotropic phases).  lame: HOST nphases x 2, or
 * NULL and stiffness: HOST nphases x 21 Voigt upper triangle.  Returns
 * INFINITY when a phase is not positive definite, and NAN for bad arguments
 * (nphases < 1, both tables NULL, a coefficient that is not a number).  Host only; no device is touched.
 * Binary16 rounding (unit 2^-11) times this contrast bounds the relative error
 * a binary16 spectrum adds to the inner operator; above the limit below a
 * MIXED CG plan keeps its spectrum in FP32 whatever spectrum16 says. */
#define FFTH_SPECTRUM16_MAX_CONTRAST 128.0
/* Smaller grids are bound by launch latency, where binary16 saves nothing. */
#define FFTH_SPECTRUM16_MIN_VOXELS 2097152
double ffth_stiffness_contrast(int32_t nphases, const double *lame, const double *stiffness);

/* 1 if n (one axis length) is supported by the compiled FFT kernels
 * (4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 256, 512, 1024).  Axis 0 may
 * also have length 1: a 2-D problem in the (x2, x3) plane (every field
 * invariant along x1; with plane-stress moduli the plane-stress problem). */
int32_t ffth_size_supported(int32_t n);

/* Bytes of caller-owned device workspace needed by a plan for grids of size
 * n[3], a phase table of `nphases` entries, up to `nloads` simultaneous load
 * cases, order 0, 1 or 2 and the given options.  Returns 0 for invalid
 * arguments. */
size_t ffth_workspace_bytes(const int32_t n[3], int32_t nphases, int32_t nloads, int32_t order,
                            const ffth_opts *o);

/* Create a plan for problem p (Sec. 2: stiffness field, reference medium).
 * workspace: DEVICE, at least ffth_workspace_bytes(p->n, nloads, order, o)
 * bytes, 256-byte aligned, caller-owned, must outlive the plan.
 * hip_stream: hipStream_t on which all work is queued (NULL = default). */
ffth_status ffth_plan_create(ffth_plan **out, const ffth_problem *p, const ffth_opts *o,
                             int32_t nloads, int32_t order, void *workspace, size_t bytes,
                             void *hip_stream);

ffth_status ffth_plan_destroy(ffth_plan *plan);

/* Order 0, the classical cell problem (Sec. 2 eqs. (1)-(6); Algorithm 1 with
 * the initialization eps_0 = -Gamma0 * (C:E)).
 *   E:   HOST [nloads][6] engineering Voigt macro strains.
 *   eps: DEVICE FP64 out [nloads][6][N] strain fluctuation (tensor components).
 *   res: HOST out [nloads]. */
ffth_status ffth_solve_order0(ffth_plan *plan, int32_t nloads, const double *E, double *eps,
                              ffth_result *res);

/* Order 1, the strain-gradient problem (Sec. 3, alpha = 2): right-hand side
 * p_2 = C : sym(X_1 . grad E) and body force g_2 = div_Y[C : (e_y(X_1:E) + E)]
 * built from the six order-0 correctors, turned into the polarization theta_2
 * of eq. (12) (mean of g dropped and reported), then the same iteration with
 * eps_0 = -Gamma0 * (p_2 + theta_2).
 *   eps0_six: DEVICE FP64 [6][6][N] order-0 strain fluctuations for the unit
 *             engineering loads e_1..e_6 (as returned by ffth_solve_order0).
 *   G:        HOST [nloads][18] strain gradients.
 *   eps:      DEVICE FP64 out [nloads][6][N]. */
ffth_status ffth_solve_order1(ffth_plan *plan, const double *eps0_six, int32_t nloads,
                              const double *G, double *eps, ffth_result *res);

/* Order 2, the problem of the paper's order alpha = 3 (Sec. 3, the definition
 * of p_alpha and g_alpha for alpha >= 3), read as the next step of the same
 * recursion: with u_2 = sum G[J,j] w^(J,j) the order-1 displacement and
 * H[J,j,m] = dG[J,j]/dY_m,
 *   p_3 = C : sym(X_2 . H),      (X_2 . H)_am = sum_{J,j} w^(J,j)_a H[J,j,m]
 *   g_3 = div_Y[C : (e_y(u_2) + e_Y(u_1))],  g_i = sum_{J,j,m} S^(J,j)_im H[J,j,m]
 * with S^(J,j) = C : eps1^(J,j) + p_2^(J,j) the local order-1 stress of the
 * unit gradient load; theta_3 from g by eq. (12), then the same iteration.
 * The plan must have been created with order 2.
 *   eps0_six: DEVICE FP64 [6][6][N] as for order 1.
 *   eps1_18:  DEVICE FP64 [18][6][N] order-1 solutions (ffth_solve_order1) for
 *             the unit gradient loads G[J*3 + j] = 1, in the order J*3 + j.
 *   H:        HOST [nloads][54], H[J*9 + j*3 + m] = d^2 E_J / dY_j dY_m
 *             (tensor components J, symmetric in j, m).
 *   eps:      DEVICE FP64 out [nloads][6][N]; res: mean_stress = <C:eps + p_3>,
 *             g_mean = <g_3>. */
ffth_status ffth_solve_order2(ffth_plan *plan, const double *eps0_six, const double *eps1_18,
                              int32_t nloads, const double *H, double *eps, ffth_result *res);

/* Order-2 right-hand side polarization P = p_3 + theta_3 for one load H [54]
 * (arguments as for ffth_solve_order2); P: DEVICE FP64 out [6][N]. */
ffth_status ffth_order2_rhs(ffth_plan *plan, const double *eps0_six, const double *eps1_18,
                            const double *H, double *P, double *g_mean);

/* Green operator application eta = -Gamma0 * tau (eq. (5) and the formula
 * below it; the Fourier-space steps of Algorithm 1), one 6-component field.
 *   tau, eta: DEVICE FP64 [6][N] (may alias).  precision: FFTH_FP64 or
 *   FFTH_FP32 (input rounded to FP32, output widened back). */
ffth_status ffth_green_apply(ffth_plan *plan, const double *tau, double *eta, int32_t precision);

/* Zero-mean periodic displacement u with sym grad u = eps (inverse of eq. (1),
 * used for the corrector X_1 of the ansatz u_1 = X_1 : E in Sec. 3).
 *   eps: DEVICE FP64 [6][N]; u: DEVICE FP64 out [3][N]. */
ffth_status ffth_displacement(ffth_plan *plan, const double *eps, double *u);

/* Order-1 right-hand side polarization P = p_2 + theta_2 (Sec. 3, eq. (12))
 * for one gradient load.  eps0_six as in ffth_solve_order1; G: HOST [18];
 * P: DEVICE FP64 out [6][N]; g_mean: HOST out [3] (may be NULL). */
ffth_status ffth_order1_rhs(ffth_plan *plan, const double *eps0_six, const double *G, double *P,
                            double *g_mean);

/* Kernel timing (diagnostics).  When enabled, every kernel launch of the plan
 * is bracketed by HIP events recorded on the plan's stream; the totals per
 * kernel category (0 .. 13: x-pass forward / y-pass / z-pass / x-pass inverse
 * in FP32, the same four in FP64, finalize, pointwise, fused three-term CG
 * x-pass and its start pass in FP32, the same two in FP64) accumulate until
 * the next ffth_profile_enable call, which also resets them.  launches: kernel launches; units: batch entries (loads) they
 * processed, summed; ms: summed event time. */
ffth_status ffth_profile_enable(ffth_plan *plan, int32_t on);
ffth_status ffth_profile_read(ffth_plan *plan, int32_t category, int64_t *launches, int64_t *units,
                              double *ms);
const char *ffth_profile_name(int32_t category);
/* Tile variant chosen per pass: out[2*pass + prec], pass 0..3 = x-forward, y,
 * z, x-inverse; prec 0 = FP32, 1 = FP64 (variant 0 = the default shape). */
ffth_status ffth_tile_variants(ffth_plan *plan, int32_t out[8]);
/* Pin the tile variants (same layout; each in [0, 6): 0..3 tile shapes with
 * the default radix order, 4 and 5 the default tile with the radix orders
 * 4-2-3-5-8-16 and 8-4-2-3-5-16); results of every variant agree to
 * rounding.  INVALID for a value out of range. */
ffth_status ffth_set_tile_variants(ffth_plan *plan, const int32_t in[8]);
/* Loads per launch of the iteration passes, out[prec] (0 = FP32, 1 = FP64):
 * 0 = every load of the iteration in one launch per pass; k > 0 = the loads
 * are taken k at a time, each group through all of the iteration's passes
 * (y, z, y and the x-passes) before the next (load-major order), and the
 * scalars of all of them finalized together.  Chosen by the autotuner like
 * the tile variants (0 unless a smaller width is measured faster). */
ffth_status ffth_launch_loads(ffth_plan *plan, int32_t out[2]);
/* Pin them (each >= 0); results do not depend on the width (every load's
 * blocks and sums are the same in any launch).  INVALID for a negative value. */
ffth_status ffth_set_launch_loads(ffth_plan *plan, const int32_t in[2]);

/* ---- Serving: continuous batching of order-0 solves ----------------------
 * A server owns no device memory: the caller hands it one device arena (the
 * HBM budget).  Requests (one RVE, 1..6 macro strains each, e.g. the six unit
 * loads of an effective-stiffness request) are admitted while one of
 * max_running slots is free: the waiting request of least work (voxels x
 * loads) whose memory (ffth_request_bytes) fits the free arena goes first
 * (ties: earlier arrival); a request passed over max_running times goes next
 * as soon as its memory fits, and nothing passes it meanwhile.  A round
 * advances every running request of a stream by one phase of the
 * mixed-precision solve (an FP64 residual sweep, the compatible projection,
 * or check_every FP32 iterations); requests of the same grid size, material
 * kind and spectrum precision share every kernel launch, and each grid size
 * is bound to one of four streams (the caller's and three the server
 * creates), so that sizes run concurrently, each stream at its own pace
 * (ffth_server_step).  A completed request returns its memory to the arena
 * and its results (mean stresses, i.e. C_eff columns for unit loads) to
 * ffth_poll.  Results do not depend on what else runs:
 * every load keeps its own iteration state and reductions are fixed-order.
 *   arena: DEVICE, 256-byte aligned, caller-owned, outlives the server.
 *   opts:  precision must be FFTH_MIXED.
 *   problem->phase must stay valid until the request completes.
 * Not thread-safe: drive a server from one host thread. */
typedef struct ffth_server ffth_server;
size_t ffth_request_bytes(const int32_t n[3], int32_t nphases, int32_t nloads, const ffth_opts *o);
ffth_status ffth_server_create(ffth_server **out, void *arena, size_t arena_bytes, const ffth_opts *o,
                               int32_t max_running, void *hip_stream);
/* FFTH_ERR_OOM if the request can never fit the arena. */
ffth_status ffth_submit(ffth_server *srv, const ffth_problem *p, int32_t nloads, const double *E,
                        uint64_t *request_id);
/* Advance the server.  Each of its streams runs rounds of its own (a round
 * advances every running request on the stream by one phase step): the call
 * admits what fits, starts a round on every idle stream that has running
 * requests, and completes every round that has finished (phase transitions,
 * finished requests, whose memory goes back to the arena) and starts that
 * stream's next one; if no round has finished it polls the rounds' events
 * until one has (the calling thread spins, yielding between polls).  So small
 * grids are not held to the pace of large ones.  running / waiting (may
 * be NULL) receive the queue sizes after it. */
ffth_status ffth_server_step(ffth_server *srv, int32_t *running, int32_t *waiting);
/* FFTH_ERR_BUSY until complete; then the request's status, res[nloads] filled,
 * and the id is released.  FFTH_ERR_CANCELLED for cancelled requests. */
ffth_status ffth_poll(ffth_server *srv, uint64_t request_id, ffth_result *res);
ffth_status ffth_cancel(ffth_server *srv, uint64_t request_id);
/* Multi-size launches: with the three-term CG inner solve, the inner
 * iterations of the running requests whose grids have all three axis lengths
 * in {16, 24, 32, 48, 64, 96, 128} run as one launch per pass across the grid
 * sizes that share a stream (more grids than streams; per material kind and
 * spectrum precision), each load with the default tile shape of its lengths
 * (a grid alone on its stream keeps the per-size kernels, with the same
 * tiles); such requests' plans are not autotuned, so their results equal the
 * plan path's with autotuning off, bit for bit.
 * multi_iterations: inner iterations run that way so far; multi_max_grids: the most
 * distinct grids one of those launches carried. */
ffth_status ffth_server_stats(ffth_server *srv, int64_t *multi_iterations, int32_t *multi_max_grids);
ffth_status ffth_server_destroy(ffth_server *srv);

/* ---- Allocation-free Green operator application ----------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  Computes
 * what ffth_green_apply computes on a plan of grid n with reference medium
 * (lambda0, mu0): eta = -Gamma0 * tau (eq. (5) and the formula below it), with
 * the same kernels, but needs neither a plan nor a workspace: every device
 * buffer beyond tau and eta (descriptor, state, block sums, phase ids, half
 * spectrum) lives in one fixed array of FFTH_NOALLOC_SCRATCH_BYTES bytes in
 * the library, one copy per GPU, held until the process ends.  The call
 * allocates nothing: no hipMalloc, hipFree or allocating library routine.
 *   n:       grid (as ffth_size_supported; n0 = 1 allowed), at most
 *            FFTH_NOALLOC_MAX_VOXELS voxels, else FFTH_ERR_INVALID (the
 *            message names the limit; nothing is queued).
 *   tau, eta: DEVICE FP64 [6][N] (may alias); precision FFTH_FP64 or
 *            FFTH_FP32 (input rounded to FP32, output widened back).
 *   hip_stream: hipStream_t to queue on (NULL = default).  The call returns
 *            once the work is queued; eta is ready when the stream reaches
 *            that point.
 * Every call on one GPU uses that GPU's single array, and each call
 * rewrites it before use: calls queued on one stream are ordered and
 * correct; calls that overlap on one GPU (different streams or threads)
 * race on the array and give wrong results. */
#define FFTH_NOALLOC_MAX_VOXELS 262144
#define FFTH_NOALLOC_SCRATCH_BYTES 21497088
ffth_status ffth_green_apply_noalloc(const int32_t n[3], double lambda0, double mu0, const double *tau,
                                     double *eta, int32_t precision, void *hip_stream);

const char *ffth_status_string(ffth_status s);

/* Last HIP error text recorded by the library on this thread ("" if none). */
const char *ffth_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FFTH_H */
