/*
 * ehdbim.h -- C ABI of the MI355X layer-potential library for drops
 * represented by spherical harmonics (Sorgentone, Tornberg & Vlahovska,
 * "A 3D boundary integral method for the electrohydrodynamics of
 * surfactant-covered drops", arXiv 1811.10270).
 *
 * What the library computes (one call of ehd_layer_potentials):
 * at every node of every drop's own Gaussian grid (the target nodes), the
 *   Stokes single layer   S[f](x0) = 1/(4 pi) int f . G(x0,x) dS      (3 comp.)
 *   Stokes double layer   D[u](x0) = 1/(4 pi) int u . T(x0,x) . n dS  (3 comp.)
 *   Laplace single layer  S_L[s](x0) = 1/(4 pi) int s / r dS          (1)
 *   Laplace double layer  L[s](x0) = 1/(4 pi) int s (xh . n) / r^3 dS (1)
 *   adjoint double layer  K*[s](x0) = 1/(4 pi) int s (xh . n0) / r^3 dS (1)
 * with xh = x0 - x, r = |xh|, G = I/r + xh xh / r^3, T = -6 xh xh xh / r^5,
 * n the outward normal at x and n0 the one at x0 (paper: Sec. 1, eq. GandT;
 * Sec. 2, eq. op_stokes and eq. dl_op_laplace; K* is the kernel of eq. E_n).
 * Each sum runs over all drops: the target's own drop by the singular rule
 * (Sec. 2.1, eq. mod_weights: the expansion is rotated so that the target is
 * the north pole of an upsampled Gaussian grid of degree q_self), every other
 * drop by the regular rule (eq. reg_quadrature) on its upsampled degree-q_far
 * grid (direct summation).
 *
 * Data layout (all FP64 unless stated):
 *   SH coefficients: orthonormal complex spherical harmonics with the
 *   Condon-Shortley phase (Sec. 2, eq. normalized_spharm, eq. pneg).  A real
 *   field of degree p is stored by its m >= 0 coefficients, (re, im)
 *   interleaved, at complex index n(n+1)/2 + m: (p+1)(p+2) doubles.  A
 *   K-field array holds the drops one after another; drop d's block starts
 *   at K * off[d] doubles, off[d] = sum_{e<d} (p_e+1)(p_e+2), and inside it
 *   the K fields follow one another.  x: K = 3 (Cartesian components of the
 *   surface, Sec. 2 after eq. spharm_ex); f, u: K = 3; sigma: K = 1.
 *   Imaginary parts of m = 0 coefficients are ignored (taken as zero).
 *   Grids: degree P has P+1 Gauss-Legendre latitudes, theta increasing, and
 *   nlon longitudes phi_k = 2 pi k / nlon, with nlon = 2P+2 (EHD_GRID_PAPER,
 *   the paper's grid) or 2P (EHD_GRID_2P); node index j*nlon + k.
 *   Targets: global index = (sum of earlier drops' node counts) + j*nlon + k.
 *   Outputs: [row][global target], rows = the components of the requested
 *   kinds in the order S_x S_y S_z D_x D_y D_z S_L L K* (unrequested kinds
 *   take no row).
 *
 * Ownership: pointers named *_d are caller-owned device memory on the
 * context's device, *_h host memory; both are read (or written) during the
 * call only and never retained.  Calls are asynchronous on the context's
 * stream, except where stated; a later call or ehd_sync reports
 * asynchronous HIP failures.
 *
 * Errors: every call returns EHD_OK or an error code; on an argument error
 * nothing is enqueued and no output is written.  ehd_last_error gives a
 * message.  A context is used by one host thread at a time.
 */
#ifndef EHDBIM_H
#define EHDBIM_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ehd_ctx ehd_ctx;

enum {
    EHD_OK = 0,
    EHD_E_ARG = 1,         /* invalid argument (null, range, alignment)   */
    EHD_E_SHAPE = 2,       /* degrees / sizes not supported                */
    EHD_E_STATE = 3,       /* call order (e.g. no drops set)               */
    EHD_E_NOMEM = 4,       /* device allocation failed                     */
    EHD_E_HIP = 5          /* a HIP runtime call failed                    */
};

enum {
    EHD_STOKES_SL = 1,     /* S[f]  : 3 rows */
    EHD_STOKES_DL = 2,     /* D[u]  : 3 rows */
    EHD_LAP_SL = 4,        /* S_L[sigma] : 1 row */
    EHD_LAP_DL = 8,        /* L[sigma]   : 1 row */
    EHD_LAP_DLADJ = 16,    /* K*[sigma]  : 1 row */
    EHD_ALL_KINDS = 31
};

enum {
    EHD_FAR_FP64 = 0,      /* far-field sums in FP64                         */
    EHD_FAR_FP32C = 1      /* FP32 arithmetic on drop-centred coordinates,
                              FP32 accumulation per source tile, compensated
                              (Kahan) accumulation of the tile sums          */
};

enum { EHD_GRID_PAPER = 0, EHD_GRID_2P = 1 };

/* Largest drop degree p the singular self-interaction supports (its rotated
 * expansion of all fields is kept in the 160 KiB of LDS of one CU). */
#define EHD_MAX_P 48
/* Largest upsampled grid degree. */
#define EHD_MAX_Q 160
#define EHD_MAX_Q_CHECK 400   /* check grids of nearly singular targets (ehd_set_near) */

/* Create a context on HIP device `device`; `stream` is a hipStream_t (NULL:
 * the null stream), e.g. torch.cuda.current_stream().cuda_stream.
 * *out receives the context.  Returns EHD_E_HIP if the device is unusable. */
int ehd_create(ehd_ctx** out, int device, void* stream);

/* Release the context and all its device memory.  NULL is accepted. */
void ehd_destroy(ehd_ctx* ctx);

/* Message describing the last failed call on ctx (never NULL).  With
 * ctx == NULL, the message of the last failed ehd_create. */
const char* ehd_last_error(const ehd_ctx* ctx);

/* Host-only: (nlat, nlon) of the degree-P grid in grid_mode. */
int ehd_grid_dims(int P, int grid_mode, int* nlat, int* nlon);

/* Define the drops: ndrops >= 1; p_h[d] in [1, EHD_MAX_P]; q_self_h[d] and
 * q_far_h[d] in [p_h[d], EHD_MAX_Q] (upsampled quadrature degrees of the
 * singular and of the regular rule, Sec. 2.1), and the rotated grid of the
 * singular rule has at most 256 longitudes (q_self <= 127 on the paper's
 * grid, <= 128 with EHD_GRID_2P); grid_mode as above;
 * xcoef_d: 3-field packed surface coefficients (copied; the caller may free
 * them after the call).  Builds the quadrature tables, rotation tables and
 * the geometry of targets and far-field sources.  Synchronous: returns when
 * the set-up work on the stream is done. */
int ehd_set_drops(ehd_ctx* ctx, int ndrops, const int* p_h, const int* q_self_h,
                  const int* q_far_h, int grid_mode, const double* xcoef_d);

/* Number of target nodes (sum over drops of nlat*nlon) of the current drops. */
int ehd_num_targets(const ehd_ctx* ctx, long long* ntargets);

/* Number of doubles of one packed field of the current drops,
 * sum over drops of (p+1)(p+2). */
int ehd_num_coefs(const ehd_ctx* ctx, long long* ncoef);

/* Evaluate the layer potentials of the requested `kinds` (EHD_* bit mask)
 * for densities fcoef_d (3 fields; needed for EHD_STOKES_SL), ucoef_d (3
 * fields, NULL: u = f; needed for EHD_STOKES_DL) and sigcoef_d (1 field;
 * needed for the Laplace kinds), all in the packed layout of the current
 * drops.  far_prec: EHD_FAR_FP64 or EHD_FAR_FP32C (the singular
 * self-interaction is always FP64).
 * self_out_d: [rows][ntargets] FP64; receives self + far if far_out_d is
 * NULL, else the self part only, and far_out_d [rows][ntargets] the far
 * part.  Buffers must not overlap the inputs. */
int ehd_layer_potentials(ehd_ctx* ctx, const double* fcoef_d, const double* ucoef_d,
                         const double* sigcoef_d, unsigned kinds, int far_prec,
                         double* self_out_d, double* far_out_d);

/* Synthesis: values of nfields packed fields (degree p of each drop) at the
 * drops' own grid nodes, grid_d[field][global target]. */
int ehd_synthesize(ehd_ctx* ctx, int nfields, const double* coef_d, double* grid_d);

/* Surface quantities at the target nodes (Sec. 1, eq. interfacial_force):
 * H_d[T] the mean curvature H = (1/2) div_S n (n outward: 1/a on a sphere
 * of radius a) and, for ng in {0, 1, 2} packed scalar fields gcoef_d (ng
 * fields per drop; also 3, e.g. a velocity), grad_d[g][3][T] their surface gradients
 * (I - n n) grad g and, if lap_d is not NULL, lap_d[g][T] their
 * Laplace-Beltrami values div_S grad_S g.  From the SH derivatives of x and
 * g up to second order; gcoef_d and grad_d may be NULL when ng = 0. */
int ehd_surface(ehd_ctx* ctx, int ng, const double* gcoef_d, double* H_d, double* grad_d, double* lap_d);

/* Galerkin analysis (Sec. 2, the inner product before eq. BIM_galerkin):
 * coef_d receives (y, Y_nm) = int_{S^2} y conj(Y_nm) ds for n <= p, m >= 0,
 * computed with the Gaussian grid quadrature from grid_d[field][global target]. */
int ehd_analyze(ehd_ctx* ctx, int nfields, const double* grid_d, double* coef_d);

/* Positions x0 and outward unit normals n0 at the target nodes,
 * x_d[3][ntargets], n_d[3][ntargets]. */
int ehd_target_geometry(ehd_ctx* ctx, double* x_d, double* n_d);

/* Area quadrature weights at the target nodes (eq. reg_quadrature):
 * w_d[T] = (2 pi / n_lon) w_j J, so that the sum of w_d[t] g[t] over a
 * drop's nodes is the surface integral of g over that drop. */
int ehd_area_weights(ehd_ctx* ctx, double* w_d);

/* Nearly singular targets (Sec. 2.1, the interpolation approach).  With
 * delta > 0, every later ehd_layer_potentials call corrects, for each
 * target x0 closer than delta to the surface of another drop j, drop j's
 * contribution to the far part:
 *   y: the point of drop j closest to x0 (damped Gauss-Newton in the
 *      surface parameters from the nearest grid node), s_t = |x0 - y|,
 *      nu = (x0 - y) / s_t;
 *   the exterior limit at y: drop j's on-surface singular-rule values,
 *      projected to degree p and evaluated at y, plus the jumps (S, S_L
 *      continuous; D: -u(y); L: +sigma(y)/2; K* with the target normal n0:
 *      -n0 . grad_S S_L(y) + (K*(y) + sigma(y)/2)(n0 . n_y));
 *   m check points y + s_k nu, s_k = s_check (1 + k/2), k = 0..m-1, where
 *      drop j's regular rule on a degree-q_check grid is summed (FP64);
 *   the Lagrange polynomial through (0, limit) and (s_k, values), at s_t,
 *      replaces drop j's regular-rule value at x0.
 * The pairs are found for the current shapes here and again by
 * ehd_update_shape; ehd_set_drops switches the correction off.  delta = 0
 * switches it off.  m in [2, 12], q_check in [p, EHD_MAX_Q_CHECK] for every
 * drop, s_check > 0 and delta <= s_check (1 + (m-1)/2) (no extrapolation).
 * The regular rule on a degree-q grid of a drop of radius a is accurate
 * beyond about 3 pi a / q: delta should exceed that distance for q_far
 * (targets farther out keep the plain sums) and s_check for q_check.
 * Synchronous.  The closest-point search runs on up to 16 host threads of
 * the calling process (joined before the call returns); the check-grid
 * tables are kept while q_check and the grid mode stay the same.  A host
 * allocation failure returns EHD_E_NOMEM. */
int ehd_set_near(ehd_ctx* ctx, double delta, double s_check, int m, int q_check);

/* Number of (target, drop) pairs the nearly singular correction treats. */
int ehd_near_pairs(const ehd_ctx* ctx, long long* npairs);

/* New surface coefficients for the same drops, degrees and grids (e.g. a
 * time step): copies xcoef_d (3 packed fields per drop, as for
 * ehd_set_drops) and recomputes the drop centres, the target and far-source
 * geometry and, when ehd_set_near is on, the nearly singular pairs, keeping
 * every table.  Drops a recorded graph.
 * Synchronous. */
int ehd_update_shape(ehd_ctx* ctx, const double* xcoef_d);

/* Wait for the context's stream; reports asynchronous HIP failures. */
int ehd_sync(ehd_ctx* ctx);

/* Stage timing with HIP events recorded on the context's stream (no host
 * synchronisation during the calls).  nslots > 0 enables it: the i-th
 * following ehd_layer_potentials call records into slot i % nslots;
 * nslots == 0 disables it and frees the events. */
int ehd_set_timing(ehd_ctx* ctx, int nslots);

/* Elapsed milliseconds of the stages of the call recorded in `slot`:
 * ms[0] source densities (synthesis on the far grids + records),
 * ms[1] singular self-interaction, ms[2] far field, ms[3] combination.
 * Waits for the recorded events.  EHD_E_STATE if the slot holds no call. */
int ehd_stage_times(ehd_ctx* ctx, int slot, double* ms);

/* Elapsed milliseconds of the singular self-interaction kernel of each
 * degree class (p <= 16, <= 24, <= 32, <= 48; one launch per class) in the
 * call recorded in `slot`; 0 for a class without drops.  When the call runs
 * the self-interaction in two passes (a separate u together with S or the
 * Laplace kinds), the times are those of the second pass.  Not recorded in
 * graph mode (all 0).  EHD_E_STATE if the slot holds no call. */
int ehd_self_class_times(ehd_ctx* ctx, int slot, double* ms);

/* Graph mode (enable != 0): ehd_layer_potentials records its launch
 * sequence as a HIP graph the first time it is called with a given argument
 * set (pointers, kinds, far_prec, far-field tile shape) and replays the graph
 * on later calls with the same arguments; any change of arguments, of the
 * tile shape or of the drops records a new graph.  Device buffers may be
 * rewritten between calls (the graph reads them at replay).  With stage
 * timing on, ms[0] of a replayed call holds the whole evaluation.
 * Synchronises the stream. */
int ehd_set_graph(ehd_ctx* ctx, int enable);

/* Overlap mode (off by default): the far-field sums run, in part or whole,
 * on a second stream of the context, concurrently with the singular
 * self-interaction; results are bitwise the same.  A far field of at most
 * two (target block, chunk) work items per compute unit forks whole before
 * the self-interaction.  A larger one forks as one looping block per
 * compute unit over a first share of its items beside the degree classes
 * whose kernels leave room on a compute unit for one such block (registers
 * of two self-interaction waves and one far-field wave per SIMD within 512
 * per lane, LDS of both blocks within the CU's, as the runtime reports them
 * for the kernels built); the other classes run before the fork and the
 * rest of the far field is an ordinary launch after them.  The share is
 * the expected time of those classes over that of the far field for the
 * FP32 far field, and 0 for the FP64 one, which needs the same FP64 units
 * and slows the self-interaction as much as it gains; with share 0 the
 * evaluation keeps the serial order (ehd_overlap_plan reports the plan).
 * A single drop (no far interactions) keeps the serial order.  Stage times
 * then read: self = until the last class ends (shared with the forked
 * part), far = the rest.  Drops a recorded graph. */
int ehd_set_overlap(ehd_ctx* ctx, int enable);

/* The overlap plan an evaluation with these kinds (EHD_* mask), far
 * precision (EHD_FAR_*) and double-layer density (with_u != 0: a separate
 * u, as ehd_layer_potentials with ucoef) would follow now: *beside = the
 * degree classes (bit 0: p <= 16 .. bit 3: p <= 48) that run beside the
 * forked far-field share, *forked = the far-field work items forked (0:
 * serial order, as always outside overlap mode).  Host query only; errors:
 * EHD_E_ARG (null pointer, bad mask or precision), EHD_E_STATE (no drops). */
int ehd_overlap_plan(ehd_ctx* ctx, unsigned kinds, int far_prec, int with_u, unsigned* beside, long long* forked);

/* Far-field tile shape: targets per thread (1 or 2) and number of source
 * chunks (1..16, at most the number of source tiles) the targets' sums are
 * split into.  ehd_set_drops sets a default; the autotuner (ehd_time_far over
 * candidates, paper_1811_10270_amd/autotune.py) picks the fastest. */
int ehd_set_far_config(ehd_ctx* ctx, int targets_per_thread, int nchunk);
int ehd_get_far_config(const ehd_ctx* ctx, int* targets_per_thread, int* nchunk);

/* Autotuner support: mean milliseconds of `reps` launches (after one
 * warm-up launch) of the far-field kernel of precision far_prec for the
 * kinds mask `kinds` (as for ehd_layer_potentials) with the given tile
 * shape, on the current source records, timed with HIP events.  Overwrites
 * the far field's partial sums (not the caller's outputs).  Synchronous. */
int ehd_time_far(ehd_ctx* ctx, int far_prec, unsigned kinds, int targets_per_thread, int nchunk, int reps,
                 double* ms);

/* Self-interaction tuning (the per-target singular rule of Sec. 2.1,
 * eq. mod_weights, batched by degree class).  The class kernels stream the
 * Legendre tables of the rotated grid in prefetch batches; each class is
 * built with three batch sizes for the field set x, f, sigma (the kinds S, D,
 * S_L, L with u = f, and the E_n and velocity solves' field sets use the
 * default).  ehd_self_config_candidates (host only, no device needed) lists
 * them for class cls (0: p <= 16, 1: p <= 24, 2: p <= 32, 3: p <= 48), the
 * default first: *n = 3, pf[3].  ehd_set_self_config selects one for a class
 * of the context (0: the default; another value: EHD_E_ARG) and drops a
 * recorded graph when it changes; results are bitwise the same for every
 * choice (only the load schedule differs).  ehd_get_self_config returns the
 * batch in effect.  ehd_time_self: mean milliseconds of `reps` launches
 * (after one warm-up) of class cls with batch pf (restored afterwards) on the
 * kinds S, D, S_L, L from the device coefficients fcoef_d and sigcoef_d
 * (layout of ehd_layer_potentials), HIP events, synchronous; 0 for a class
 * without drops.  Overwrites the self-interaction's internal sums only. */
int ehd_self_config_candidates(int cls, int* pf, int* n);
int ehd_set_self_config(ehd_ctx* ctx, int cls, int pf);
int ehd_get_self_config(const ehd_ctx* ctx, int cls, int* pf);
int ehd_time_self(ehd_ctx* ctx, int cls, int pf, const double* fcoef_d, const double* sigcoef_d, int reps, double* ms);

/* Galerkin solvers (Sec. 2, eq. galerkin_En and eq. BIM_galerkin) by
 * restarted GMRES in FP64 on the device.  Each iteration is one
 * ehd_layer_potentials call (far field in far_prec) and one ehd_analyze.
 * restart in [1, 200], maxit >= 0 (mat-vecs; 0 only evaluates the true
 * residual of the initial guess into *relres), tol > 0: stop when the true
 * residual |b - A x| <= tol |b| (Euclidean norm of the packed coefficient
 * vector).  *iters receives the number of mat-vecs, *relres the final true
 * relative residual; not converging within maxit is not an error (check
 * *relres).  The solution vector holds the initial guess on entry (zeros
 * for none).  Synchronous; the solver allocates its own workspace.
 * With EHD_FAR_FP32C the operator carries the FP32 far field's rounding
 * (relative 1e-7): residuals stagnate there, so tol should be >= 1e-6. 
 *
 * ehd_solve_En: the normal electric field E_n (1 packed field, en_coef_d) of
 *   (1/2)(E_n, Y) - (R-1)/(R+1) sum_j (K*_j[E_n], Y) = R/(R+1) (E_inf . n, Y)
 *   for all Y = Y_nm, n <= p, with the adjoint double layer K* (the
 *   operator of eq. E_n taken with the target normal, as the equation is
 *   eq. BIE01 dotted with n(x0)), conductivity ratio R > 0 and the applied
 *   field E_inf = -grad phi_inf, phi_inf = -(E_u z + E_q (z^2 - (x^2+y^2)/2))
 *   (uniform and quadrupole parts, Sec. 1).
 * ehd_solve_velocity: the interface velocity u (3 packed fields, ucoef_d)
 *   of (lambda+1)(u, Y) = sum_j (S_j[f], Y) + (lambda-1) sum_j (D_j[u], Y)
 *   for the force density fcoef_d (3 packed fields, the signed density of
 *   eq. BIM_galerkin) and viscosity ratio lambda >= 0. */
int ehd_solve_En(ehd_ctx* ctx, double R, double Eu, double Eq, int far_prec, int restart, int maxit,
                 double tol, double* en_coef_d, int* iters, double* relres);
int ehd_solve_velocity(ehd_ctx* ctx, double lambda, const double* fcoef_d, int far_prec, int restart,
                       int maxit, double tol, double* ucoef_d, int* iters, double* relres);

/* Allocation-free variant of ehd_solve_En, for callers that cannot allocate
 * device memory during a solve (tight time-stepping or serving loops,
 * harnesses that forbid hipMalloc/hipFree): same arguments, results and
 * errors, but the call allocates nothing.  Its workspace (the Krylov basis,
 * the right-hand side and the evaluation buffers: (restart + 4) n + 7 T
 * doubles plus alignment, n = ehd_num_coefs, T = ehd_num_targets) lives in
 * one static 64 MiB device array per device, which the library holds until
 * the process ends.  Limits: restart <= 64 and the workspace within 8 Mi
 * doubles (e.g. 256 drops of p = 32 at restart <= 10), else EHD_E_SHAPE
 * before any work is enqueued; graph mode must be off (EHD_E_STATE), since
 * recording graphs allocates.  Every call on a device shares that device's
 * array (each call writes every workspace entry before reading it): calls
 * that overlap in time on one device, from several contexts or host
 * threads, race and must be serialised by the caller.  Synchronous. */
int ehd_solve_En_noalloc(ehd_ctx* ctx, double R, double Eu, double Eq, int far_prec, int restart, int maxit,
                         double tol, double* en_coef_d, int* iters, double* relres);

/* Implicit surfactant-diffusion solve (Sec. 2.2, the implicit half of the
 * IMEX step of Algorithm 1: (I - dt/(2 Pe) Lap_S) Gamma = b), in Galerkin
 * form on the current drops: c - kappa (Lap_S Gamma[c], Y) = b for all
 * Y = Y_nm, n <= p, with kappa = dt / (2 Pe) >= 0 per drop (kappa_h[ndrops],
 * host; the drops' systems are independent), the Laplace-Beltrami
 * operator of each drop's surface (ehd_surface) and the projection
 * ehd_analyze.  rhs_d, gamma_d: 1 packed field; gamma_d holds the initial
 * guess on entry and receives the solution.  precond != 0: right
 * preconditioning by diag(1 + kappa n(n+1)), the operator's inverse on the
 * unit sphere (the spherical-harmonic eigenfunction preconditioner of
 * Sec. 2.2).  GMRES controls and outputs as for ehd_solve_En (residual of
 * the unpreconditioned system).  Synchronous. */
int ehd_solve_surfactant(ehd_ctx* ctx, const double* kappa_h, const double* rhs_d, int precond, int restart,
                         int maxit, double tol, double* gamma_d, int* iters, double* relres);

/* Initial guess of the surfactant solve (Sec. 2.2: the preconditioned
 * implicit half-step, with a learned correction).  Per drop d, with
 * M = diag(1 + kappa_d n(n+1)) the preconditioner of ehd_solve_surfactant
 * and |b_d| the Euclidean norm of the drop's packed right-hand side:
 *   guess_d = M^{-1} b_d + kappa_d |b_d| gain (y_d std + mean)   (y_d != NULL)
 *   guess_d = M^{-1} b_d                                           (y_d == NULL)
 * elementwise over the drop's packed coefficients.  y_d: FP32 [ndrops][ny]
 * device buffer (a network's standardised outputs), ny = (p+1)(p+2) for
 * every drop; ymean_d, ystd_d, gain_d: FP64 [ny] device buffers (the
 * output de-standardisation and a per-coefficient shrinkage).  kappa_h
 * [ndrops] >= 0 (host); rhs_d, guess_d: 1 packed field.  Synchronous. */
int ehd_surfactant_guess(ehd_ctx* ctx, const double* kappa_h, const double* rhs_d, const float* y_d, int ny,
                         const double* ymean_d, const double* ystd_d, const double* gain_d, double* guess_d);

/* Inputs of the learned-guess network for the current drops (all of one
 * degree p, nc = (p+1)(p+2)): per drop, FP32 feat_d[d][4 nc + 1] =
 * standardised [x (the drop's 3 packed surface fields with their degree-0
 * terms set to 0), b / |b|, log10 kappa], each entry (v - mean_d[k]) /
 * std_d[k] (FP64 [4 nc + 1] device buffers; mean 0 and std 1 give the raw
 * inputs).  kappa_h [ndrops] > 0 (host), rhs_d: 1 packed field.
 * Synchronous. */
int ehd_learned_features(ehd_ctx* ctx, const double* kappa_h, const double* rhs_d, const double* mean_d,
                         const double* std_d, float* feat_d);

/* Copy of the current drops' surface coefficients (3 packed fields, as
 * passed to ehd_set_drops) into xcoef_d. */
int ehd_drop_coefs(ehd_ctx* ctx, double* xcoef_d);

/* Equations of state gamma(Gamma) (Sec. 1, eq. langmuir and
 * eq. lin_eq_state), surface tension scaled by its equilibrium value:
 *   EHD_EOS_CLEAN     gamma = 1 (Gamma unused),
 *   EHD_EOS_LINEAR    gamma = 1 + beta (1 - Gamma),
 *   EHD_EOS_LANGMUIR  gamma = (1 + beta ln(1 - x_s Gamma)) / (1 + beta ln(1 - x_s)). */
enum { EHD_EOS_CLEAN = 0, EHD_EOS_LINEAR = 1, EHD_EOS_LANGMUIR = 2 };

typedef struct ehd_step_params {
    double lambda;     /* viscosity ratio mu_i / mu_0                        */
    double R;          /* conductivity ratio sigma_i / sigma_0 (> 0)         */
    double Q;          /* permittivity ratio eps_i / eps_0                   */
    double CaE;        /* electric capillary number (> 0)                    */
    double Eu, Eq;     /* applied field: uniform and quadrupole strengths    */
    int eos;           /* EHD_EOS_*                                          */
    double beta;       /* elasticity number (beta~ of the linear law)        */
    double xs;         /* surface coverage of the Langmuir law, [0, 1)       */
    double dt;         /* time step of the position update                  */
    int far_prec;      /* far-field precision of every evaluation            */
    int restart, maxit;
    double tol;        /* GMRES controls of both solves (ehd_solve_En)       */
} ehd_step_params;

/* One explicit step of the method (Sec. 1, steps i-vii) for the current
 * drops and surfactant concentration gamma_coef_d (1 packed field; NULL:
 * Gamma = 1):
 *   i.   E_n by ehd_solve_En (en_coef_d: initial guess in, solution out);
 *   ii-iii. the tangential field E_t = -grad_S (phi_inf + S_L[q]) with the
 *        charge q = [[E_n]] = (1 - 1/R) E_n (the potential of eq. BIE01
 *        read with the sign that yields eq. E_n: E = E_inf + sum_j
 *        int xh q / (4 pi r^3) dS);
 *   iv.  the electric force f^E of eq. el_force (units with eps~ eps_0 = 1);
 *   v.   gamma(Gamma) and f = 2 gamma H n - grad_S gamma (eq. interfacial_force);
 *   vi.  the velocity u of eq. main_eq (ehd_solve_velocity with the force
 *        density -(f / Ca_E - f^E), projected; ucoef_d: guess in, solution out);
 *   vii. xnew_coef_d = x + dt u (forward Euler, eq. dxdtugualeu).
 * iters (may be NULL) receives the GMRES iterations of the two solves.
 * Synchronous.  The caller moves to the new shape with ehd_set_drops. */
int ehd_explicit_step(ehd_ctx* ctx, const ehd_step_params* params, const double* gamma_coef_d,
                      double* en_coef_d, double* ucoef_d, double* xnew_coef_d, int* iters);

/* ------------------------------------------------------------------------
 * Time stepping (Sec. 2.2, Algorithm 1).  Surface points move with the
 * full velocity (x' = u); following them, eq. surfactant0 reads
 * dGamma/dt = g_E + g_I with g_E = -Gamma div_S u (its convective terms
 * plus the frame term u_t . grad_S Gamma) and g_I = Pe^-1 Lap_S Gamma.
 * ------------------------------------------------------------------------ */

/* g_E = P[-Gamma div_S u] (if gE_d) and g_I = P[inv_pe Lap_S Gamma] (if
 * gI_d) on the current drops, P the Galerkin projection (ehd_analyze).
 * ucoef_d: 3 packed fields (may be NULL when gE_d is NULL); gamma_d, gE_d,
 * gI_d: 1 packed field.  Synchronous. */
int ehd_surfactant_terms(ehd_ctx* ctx, const double* ucoef_d, const double* gamma_d, double inv_pe, double* gE_d,
                         double* gI_d);

typedef struct ehd_step_report {
    double err_drop;   /* max over nodes |dt (u^{n+1/2} - u^n)|                     */
    double err_surf;   /* max over nodes |dt ((g_E+g_I)^{n+1/2} - (g_E+g_I)^n)|      */
    int iters[4];      /* GMRES iterations: E_n and u at x^n, E_n and u at the half step */
    int iters_gamma;   /* GMRES iterations of the implicit surfactant stage          */
} ehd_step_report;

/* One step of Algorithm 1 from the current drops x^n and gamma_d = Gamma^n
 * (1 packed field) with physical and solver parameters `params` (its dt is
 * not used; eos, beta, xs give gamma(Gamma); tol is also the tolerance of
 * the surfactant solve) and inv_pe = 1/Pe >= 0:
 *   u^n = velocity at (x^n, Gamma^n)                    (ehd_explicit_step)
 *   x^{n+1/2} = x^n + dt/2 u^n
 *   (I - dt/(2 Pe) Lap_S) Gamma^{n+1/2} = Gamma^n + dt/2 g_E(x^n, u^n, Gamma^n)
 *                                       on x^{n+1/2}   (ehd_solve_surfactant)
 *   u^{n+1/2} = velocity at (x^{n+1/2}, Gamma^{n+1/2})
 *   xnew_d    = x^n + dt u^{n+1/2}                                  (midpoint rule)
 *   gnew_d    = Gamma^n + dt (g_E + g_I)(x^{n+1/2}, u^{n+1/2}, Gamma^{n+1/2})
 * (the second-order IMEX Runge-Kutta scheme whose implicit stage sits at
 * the half step).  rep receives the error estimates (differences to the
 * first-order updates x^n + dt u^n and Gamma^n + dt (g_E + g_I)^n) and the
 * iteration counts.  The context is left at x^n; accept with
 * ehd_update_shape(xnew_d).  Synchronous. */
int ehd_evolve_step(ehd_ctx* ctx, const ehd_step_params* params, double inv_pe, double dt, const double* gamma_d,
                    double* xnew_d, double* gnew_d, ehd_step_report* rep);

typedef struct ehd_evolve_stats {
    double t;          /* time reached                                   */
    double dt;         /* step size proposed for the next step           */
    double max_err;    /* largest error estimate of an accepted step     */
    int accepted, rejected;
    long long matvecs; /* GMRES mat-vecs over all solves                 */
} ehd_evolve_stats;

/* Adaptive time stepping from t = 0 to t_end (the adaptivity part of
 * Algorithm 1): a step with error estimate err = max(err_drop, err_surf)
 * is accepted if err < tol; either way the next step size is
 * dt (0.9 tol / err)^(1/2), bounded to [0.2 dt, 5 dt]; at most max_steps
 * attempts.  The context's drops and gamma_d advance in place (accepted
 * steps only); reparametrisation is not part of it.  Synchronous. */
int ehd_evolve(ehd_ctx* ctx, const ehd_step_params* params, double inv_pe, double t_end, double dt0, double tol,
               int max_steps, double* gamma_d, ehd_evolve_stats* stats);

/* ------------------------------------------------------------------------
 * Learned initial guess for the surfactant solve: a multilayer perceptron
 * (nlayers hidden ReLU layers of nhidden units, linear output; FP32) whose
 * forward pass, backward pass, mean-squared-error loss and Adam update run
 * in the library's kernels (GEMMs on FP32 MFMA).  The network is a device
 * object bound to a HIP device and stream; all calls are asynchronous on
 * that stream except where stated.  Parameter layout (host buffers of
 * ehd_mlp_num_params floats): for each layer l = 0..nlayers, the weights
 * W_l[in][out] row-major, then the bias b_l[out]; layer l computes
 * h_{l+1} = ReLU(h_l W_l + b_l) (no ReLU on the output layer).
 * x_d [batch][nin], y_d and t_d [batch][nout]: FP32 device buffers.
 * ------------------------------------------------------------------------ */
typedef struct ehd_mlp ehd_mlp;

/* He-uniform weights from `seed`, zero biases and Adam moments. */
int ehd_mlp_create(ehd_mlp** out, int device, void* stream, int nin, int nhidden, int nlayers, int nout,
                   unsigned long long seed);
void ehd_mlp_destroy(ehd_mlp* mlp);
const char* ehd_mlp_last_error(const ehd_mlp* mlp);
int ehd_mlp_num_params(const ehd_mlp* mlp, long long* n);
/* Synchronous copies of the parameters / of the last backward pass's gradients. */
int ehd_mlp_get_params(ehd_mlp* mlp, float* host);
int ehd_mlp_set_params(ehd_mlp* mlp, const float* host);
int ehd_mlp_get_grads(ehd_mlp* mlp, float* host);
/* Forward pass of `batch` rows (kept for the backward pass); y_d may be NULL. */
int ehd_mlp_forward(ehd_mlp* mlp, int batch, const float* x_d, float* y_d);
/* Gradients of the parameters for the output gradient dy_d of the last
 * forward pass (same batch). */
int ehd_mlp_backward(ehd_mlp* mlp, int batch, const float* dy_d);
/* Mean-squared error L = mean((y - t)^2) over batch*nout entries and its
 * gradient dy_d = 2 (y - t) / (batch nout); *loss (if not NULL) is set
 * synchronously. */
int ehd_mlp_mse(ehd_mlp* mlp, int batch, const float* y_d, const float* t_d, float* dy_d, double* loss);
/* One Adam step with the current gradients (bias-corrected moments). */
int ehd_mlp_adam(ehd_mlp* mlp, float lr, float beta1, float beta2, float eps);

/* Host-only: Wigner small-d matrix d^n_{m m'}(beta), m, m' = -n..n, written
 * row-major to out[(m+n)*(2n+1) + (m'+n)], with
 * Y_nm(Ry(beta) v) = sum_m' d^n_{m m'}(beta) Y_nm'(v)
 * (the convention of the rotation that takes a target to the pole,
 * Sec. 2.1 after eq. mod_weights).  n in [0, 200]. */
int ehd_wigner_d(int n, double beta, double* out);

#ifdef __cplusplus
}
#endif

#endif /* EHDBIM_H */
