/*
 * dbfft.h — C ABI of the MI355X (gfx950) DBFFT hot path.
 *
 * DBFFT (Lucarini & Segurado, "DBFFT: A displacement based FFT approach for
 * non-linear homogenization of the mechanical behavior", arXiv:1905.12725)
 * solves periodic cell problems of solid mechanics with the displacement
 * fluctuation, expressed by its Fourier coefficients, as the unknown.
 *
 * Problem statement (Sec. 2): a periodic unit cell discretized in
 * n1 x n2 x n3 voxels (Sec. 2.1), a constitutive law per voxel, and a
 * macroscopic load given by six (small strains) or nine (finite strains)
 * values, each one a prescribed strain / deformation gradient component or a
 * prescribed stress component (Sec. 2.2, 2.3, 2.4), applied in increments.
 *
 * Conventions of this library:
 *   - unit cell (all L_a = 1); fields sampled at voxel centres; even grids
 *     give the Nyquist frequency a zero wavenumber;
 *   - every grid size must factor into 2, 3, 5 and 7; odd sizes are
 *     allowed on every axis (the paper's grids are 63^3);
 *   - real fields are device arrays of doubles, component-major
 *     [c][x][y][z] with z fastest; symmetric tensors have 6 components in
 *     the order 11 22 33 23 13 12 (plain tensor components, no factors),
 *     full 3x3 tensors 9 components row-major;
 *   - Fourier unknowns are normalized coefficients a(k) = F[u](k)/N on the
 *     real-transform half spectrum k3 = 0..n3/2, as device arrays of
 *     interleaved complex doubles [3][n1][n2][n3/2+1];
 *   - 3x3 host arrays (load, mask, averages) are row-major.
 *
 * Ownership: every device pointer passed in is owned by the caller and must
 * stay valid until the call returns (all entry points synchronize the
 * context's stream before returning).  The context owns its workspaces.
 * Errors: every entry point returns a dbfft_status; dbfft_last_error()
 * gives a message for the calling thread.  No C++ exception crosses the ABI.
 * Threads: no state is shared between contexts, so calls on different
 * contexts may run at the same time from different host threads; contexts
 * created on different streams then overlap on the GPU.  A context (and a
 * batch) takes one call at a time.
 */
#ifndef DBFFT_H
#define DBFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dbfft_ctx dbfft_ctx;

typedef enum {
  DBFFT_OK = 0,
  DBFFT_EINVAL = 1,       /* bad argument (null pointer, size, mask, material) */
  DBFFT_ENOMEM = 2,       /* device allocation failed */
  DBFFT_EHIP = 3,         /* HIP runtime error; message has the hipError_t string */
  DBFFT_ENOTCONV = 4,     /* iteration cap reached; info is filled */
  DBFFT_EBREAKDOWN = 5,   /* <p, K p> <= 0 or NaN: tangent not positive definite */
  DBFFT_EUNSUPPORTED = 6, /* valid request this build does not handle */
  DBFFT_EMATERIAL = 7     /* constitutive update failed (J <= 0, local Newton) */
} dbfft_status;

enum { DBFFT_SMALL = 0, DBFFT_FINITE = 1 };          /* kinematics */
enum { DBFFT_FP64 = 0, DBFFT_FP32_MIXED = 1 };       /* precision */

/* Material kinds.  `field` is a device array of N = n1 n2 n3 entries;
 * `params` a host array of `nparams` doubles.
 *  ISO_PHASE   field uint8 phase id; params (E, nu) per phase (<= 8 phases).
 *              Linear isotropic elasticity (Sec. 2.2, Sec. 3.1 material).
 *  ISO_FIELD   field double E(x); params (nu).  Linear isotropic with a
 *              per-voxel Young's modulus; the linear kind dbfft_adjoint handles.
 *  ANISO_GRAIN field int32 grain id; params 36 doubles per grain: the 6x6
 *              stiffness in the orthonormal Mandel basis (11 22 33 √2·23
 *              √2·13 √2·12), row-major.  Linear anisotropic elasticity.
 *  J2VP_CUBIC  field int32 grain id; params (C11, C12, C44, sigma0, m,
 *              edot0) then 9 doubles per grain: the rotation R (row-major)
 *              mapping crystal to sample axes.  Cubic elasticity with rate-
 *              dependent J2 flow d eps_p/dt = edot0 (s_eq/sigma0)^m (3/2) s/s_eq,
 *              backward Euler; small strains; Newton outer loop (Sec. 2.4).
 *  NEOHOOKE    field uint8 phase id; params (mu, kappa) per phase.
 *              W = mu/2 (I1 - 3) - mu ln J + lambda/2 (ln J)^2 with
 *              lambda = kappa - 2 mu / 3; finite strains (Sec. 2.4).
 *  SVK         field uint8 phase id; params (E, nu) per phase.  Saint
 *              Venant-Kirchhoff hyperelasticity of Sec. 3.3: S = lambda
 *              tr(E) I + 2 mu E with E = (F^T F - I)/2, P = F S; finite
 *              strains (Sec. 2.4). */
enum {
  DBFFT_MAT_ISO_PHASE = 0,
  DBFFT_MAT_ISO_FIELD = 1,
  DBFFT_MAT_ANISO_GRAIN = 2,
  DBFFT_MAT_J2VP_CUBIC = 3,
  DBFFT_MAT_NEOHOOKE = 4,
  DBFFT_MAT_SVK = 5
};

typedef struct {
  double tol;          /* equilibrium residual ||div sigma||_L2/||<sigma>|| (Sec. 3, eq. chedckeq); 1e-8 */
  double tol_load;     /* loading residual ||<sigma>_S - sbar_S||/||<sigma>|| (eq. chedckimp); 1e-10 */
  int32_t max_iter;    /* PCG iteration cap per linear solve (Sec. 3.1); 10000 */
  double newton_tol;   /* max change of any strain / F component in a Newton update (Sec. 2.4); 1e-6 */
  int32_t max_newton;  /* Newton iterations per increment; 25 */
  int32_t refresh;     /* preconditioner mean tangent: 0 every increment, 1 first increment only (Sec. 2.5) */
  double inner_tol;    /* FP32_MIXED: reduction of the FP32 recursive residual, relative to the last
                          FP64 residual, after which the FP64 residual b - K x replaces it; 1e-2 */
  int32_t max_refine;  /* FP32_MIXED: FP64 residual replacements; 30 */
  int32_t check_every; /* PCG iterations enqueued between host convergence polls; 8 */
  int32_t fused_cg;    /* 1: fused CG iteration where it applies (small strains, n1 a power of two
                          from 8 to 256, n2 even): the divergence pass updates the residual, no
                          separate update kernel; 0: separate vector kernels.  Same arithmetic,
                          other summation order; 1 */
  int32_t graph;       /* 1: a single-cell solve that runs past its first chunk of check_every
                          iterations captures one chunk as a HIP graph (on a private stream) and
                          replays it on the context's stream; 0: every chunk launched eagerly.
                          Same launches, same results; 1 */
  int32_t checkpoint;  /* J2VP_CUBIC: 1 keeps, per increment, the converged solution and the
                          plastic strain the increment started from (device memory of
                          24 N + 48 N bytes per increment, held by the context until the next
                          solve) for dbfft_adjoint; single-cell solves only (a batch keeps
                          none); 0 */
  int32_t coarse_kc;   /* dbfft_solve_block: 0 uses M(xi) of Sec. 2.5 everywhere; kc >= 1 a two-level
                          preconditioner: on the coarse Fourier set (every signed frequency
                          |m_a| <= kc, xi != 0) the inverse of the operator's own block there
                          (assembled by applying the operator to every coarse unknown, 6 per
                          point), M(xi) elsewhere; 0 */
} dbfft_opts;

typedef struct {
  int32_t pcg_iters;    /* PCG iterations (operator applications) of the last dbfft_solve, all steps */
  int32_t newton_iters; /* Newton iterations, all increments */
  int32_t increments;   /* increments completed */
  int32_t refine_steps; /* FP32_MIXED outer corrections */
  int32_t status;       /* dbfft_status of the solve */
  int32_t pad;
  double eq_res;        /* equilibrium residual of the final state */
  double load_res;      /* loading residual of the final state */
  double sigma_bar[9];  /* <sigma> (or <P>), row-major */
  double eps_bar[9];    /* <eps> (or <F>), row-major */
} dbfft_info;

/* Fills the defaults listed above. */
void dbfft_default_opts(dbfft_opts* opts);

/* Creates a context for one cell (Sec. 2.1 discretization + material).
 * n: grid size (host, 3 values); kinematics DBFFT_SMALL / DBFFT_FINITE
 * (NEOHOOKE and SVK need FINITE, every other kind SMALL); precision DBFFT_FP64 or
 * DBFFT_FP32_MIXED (FP32 transforms and pointwise work, FP64 dot products,
 * residuals and outer corrections); hip_stream: hipStream_t the context
 * enqueues on (NULL = default stream).  The material field is copied.
 * EINVAL on null pointers, non-positive sizes, sizes with prime factors
 * other than 2, 3, 5, 7 or above 4096, unknown or mismatched material kind.
 * EUNSUPPORTED (before any GPU work) for lines longer than one block's LDS
 * holds: n1 or n2 above 1365, n3 above 744 (small strains) or 585 (finite
 * strains). */
dbfft_status dbfft_setup(dbfft_ctx** out, const int64_t n[3], int32_t kinematics, int32_t precision,
                         int32_t material, const void* field_dev, const double* params, int32_t nparams,
                         void* hip_stream);

/* Side lengths L_1, L_2, L_3 of the cell (Sec. 2.1: the frequencies are
 * xi_i = 2 pi m_i / L_i); a new context has 1, 1, 1, i.e. the unit cube,
 * whose voxels are cubic only when n1 = n2 = n3.  len: 3 host doubles,
 * positive and finite (EINVAL otherwise).  Takes effect for the calls that
 * follow: the last solution (and any J2 checkpoints) is dropped, since its
 * coefficients refer to the old frequencies.  Cells of a batch take the
 * lengths they have when dbfft_batch_create is called.  Homogenized
 * averages do not depend on a common scale of the three lengths, only on
 * their ratios. */
dbfft_status dbfft_set_lengths(dbfft_ctx* ctx, const double len[3]);

/* Real-space operator application of Sec. 2.2 eq. lineqf (sign flipped so
 * that it is positive semi-definite): f = -div(C : sym grad u) for small
 * strains, f = -div(K : grad u) for finite strains, with the tangent of the
 * current state (the elastic stiffness before any solve).  Steps: forward
 * transform of the 3 displacement components, Fourier gradient, inverse
 * transform, pointwise tangent, forward transform, Fourier divergence,
 * inverse transform.  u_dev, f_dev: device doubles [3][n1][n2][n3]. */
dbfft_status dbfft_apply(dbfft_ctx* ctx, const double* u_dev, double* f_dev);

/* The same operator on Fourier unknowns, as iterated by the solver:
 * (K a)(k) = -i xi_j s_ij(k) with s = F[C : (e + sum_k s(k).a(k) e^{i xi.x})]/N,
 * and its macroscopic row <sigma> (9 doubles, row-major, written to
 * sigma_bar_out if not NULL).  e_macro: host 3x3 macro strain added to the
 * field (NULL = 0).  a_dev, f_dev: device complex doubles [3][n1][n2][n3/2+1]. */
dbfft_status dbfft_apply_fourier(dbfft_ctx* ctx, const void* a_dev, const double* e_macro, void* f_dev,
                                 double* sigma_bar_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the operator of
 * dbfft_apply (FP64, small strains, elastic tangent, unit cell lengths)
 * without a context.
 * It calls no hipMalloc, hipFree or other allocating routine; its workspace
 * (twiddle tables, 12 half-spectrum components, partial sums, a checked copy
 * of the phase map) lives in a static device array of 64 MiB that every
 * GPU the library runs on holds until the process ends.  Grids whose
 * workspace exceeds it (about 12 n1 n2 (n3/2+1) x 16 bytes; 84^3 fits, 96^3
 * does not) are rejected with DBFFT_EUNSUPPORTED before any GPU work.
 * n: grid (host, 3 values, checked as in dbfft_setup); material
 * DBFFT_MAT_ISO_PHASE (field_dev uint8 phase ids, params (E, nu) per phase)
 * or DBFFT_MAT_ISO_FIELD (field_dev double E(x), params (nu)); u_dev, f_dev:
 * device doubles [3][n1][n2][n3] as for dbfft_apply; hip_stream: the stream
 * to enqueue on, whose device must be the current one.
 * Unlike every other entry point it does not synchronize: it enqueues its
 * kernels and returns, and f_dev is ready when the stream's work is done.
 * The field is read in place, not copied: keep it valid until then.  Phase
 * ids at or above the number of phases cannot be reported without reading
 * device memory back: f_dev is then filled with NaN.  All calls on one GPU
 * share its array, which keeps the last call's contents (every call clears
 * what must start at zero): calls enqueued on one stream run one after the
 * other, calls that overlap on one GPU (several streams or host threads)
 * race and must not be made. */
dbfft_status dbfft_apply_noalloc(const int64_t n[3], int32_t material, const void* field_dev, const double* params,
                                 int32_t nparams, const double* u_dev, double* f_dev, void* hip_stream);

/* Solves the cell problem (Sec. 2.2-2.5): PCG with the preconditioner
 * [xi.Cbar.xi]^-1 (eqs. pred2/pred3); Newton over increments for J2VP_CUBIC,
 * NEOHOOKE and SVK.  load: 9 host doubles, row-major; on components whose
 * stress_mask entry is 0 the prescribed strain (small) or deformation
 * gradient F (finite), elsewhere the prescribed stress (Sec. 2.3).  Small
 * strains need a symmetric mask and symmetric load.  The load is reached by
 * n_increments equal steps of the strain (or F - I) and stress; dt is the
 * time per increment (rate-dependent laws).  Linear materials use one step.
 * opts may be NULL (defaults).  info may be NULL.  The solution stays in
 * the context for dbfft_homogenize / dbfft_adjoint.  Returns ENOTCONV or
 * EBREAKDOWN with info filled when the iteration fails. */
dbfft_status dbfft_solve(dbfft_ctx* ctx, const double load[9], const uint8_t stress_mask[9], int32_t n_increments,
                         double dt, const dbfft_opts* opts, dbfft_info* info);

/* Several loads of one linear cell solved together by block PCG: the
 * iterates of every load come from one block Krylov space of the
 * preconditioned operator (Sec. 3, CG for complex numbers, with the
 * per-frequency preconditioner of Sec. 2.5 eqs. pred2/pred3), spanned by the
 * preconditioned residuals of all loads; blocks of K-conjugate directions
 * P give alpha = (P^T K P)^-1 P^T R and beta = -(P^T K P)^-1 (K P)^T M R,
 * each new direction block orthonormalized (dependent directions dropped).
 * A load whose residuals meet opts.tol / opts.tol_load stops and leaves the
 * block.  loads: nrhs x 9 host doubles (row-major 3x3 each, strain or
 * stress per stress_mask as for dbfft_solve, one mask for all loads);
 * nrhs 1 .. 6.  infos: nrhs entries (pcg_iters = the block iteration at
 * which that load stopped; sigma_bar, eps_bar and residuals recomputed from
 * its solution).  applies (may be NULL): operator applications in all.
 * opts.max_iter caps the block iterations.  FP64 contexts with linear
 * materials (EUNSUPPORTED otherwise).  The context's own solution (for
 * dbfft_homogenize, dbfft_get_solution, dbfft_adjoint) is not changed. */
dbfft_status dbfft_solve_block(dbfft_ctx* ctx, int32_t nrhs, const double* loads, const uint8_t stress_mask[9],
                               const dbfft_opts* opts, dbfft_info* infos, int32_t* applies);

/* Several loads of one linear cell solved as independent PCG solves
 * (Sec. 2.2-2.5, each load exactly as dbfft_solve solves it: the same
 * kernels in the same order, so the same results) running concurrently on
 * nstreams helper contexts, each with a HIP stream and a host thread of its
 * own, so that the kernels of one solve fill the launch gaps and partly
 * idle rounds of another.  loads: nrhs x 9 host doubles (row-major 3x3
 * each, strain or stress per stress_mask as for dbfft_solve, one mask for
 * all loads); infos: nrhs entries; nstreams 1 .. 8 (at most nrhs are used);
 * load j runs on helper j mod nstreams.  The helpers (a copy of the
 * material and of the workspaces per stream, on the context's device and
 * with its cell lengths) are created on the first call that needs them and
 * kept until dbfft_destroy.  The context's own solution is not changed and
 * its stream is synchronized first.  Linear materials (EUNSUPPORTED
 * otherwise).  Returns the status of the first load that failed (its info
 * is filled), after every load has run. */
dbfft_status dbfft_solve_many(dbfft_ctx* ctx, int32_t nrhs, const double* loads, const uint8_t stress_mask[9],
                              const dbfft_opts* opts, dbfft_info* infos, int32_t nstreams);

/* Homogenized response of the last solve (Sec. 3 post-processing):
 * <sigma> and <eps> (row-major, host, either may be NULL) and, when the
 * pointers are not NULL, the real fields of strain (6 or 9 comps), stress
 * (6 or 9 comps) and displacement fluctuation u~ (3 comps) as device doubles
 * [c][n1][n2][n3]. */
dbfft_status dbfft_homogenize(dbfft_ctx* ctx, double sigma_bar[9], double eps_bar[9], double* strain_dev,
                              double* stress_dev, double* disp_dev);

/* Error estimates of Sec. 3 for real fields on the context's grid, as the
 * paper checks a computed state:
 *  out[0] equilibrium (eq. chedckeq): ||div sigma||_L2 / ||<sigma>||, the L2
 *         norm the root mean square over the voxels; at finite strains the
 *         first Piola-Kirchhoff stress and the reference divergence
 *         (Sec. 3.3);
 *  out[1] compatibility (eq. chedckcomp): the largest |component| of
 *         curl curl eps over the grid, divided by ||<eps>||; at finite strains
 *         (Sec. 3.3) max |curl_0 F| / ||<F> - I||, the curl of every row of F;
 *  out[2] loading, strain part (eq. chedckimp): ||<eps>_E - load_E|| /
 *         ||load_E|| over the components whose stress_mask entry is 0 (at
 *         finite strains I + <H> against the prescribed F, relative to
 *         ||load_E - I_E||); 0 when every component is stress-controlled;
 *  out[3] loading, stress part: ||<sigma>_S - load_S|| / ||<sigma>|| over the
 *         stress-controlled components S (the denominator of opts.tol_load);
 *         0 when S is empty.
 * Derivatives are spectral with the frequencies of Sec. 2.1 for the
 * context's cell lengths (Nyquist zeroed on even axes).  strain_dev, stress_dev: device doubles
 * [c][n1][n2][n3] in dbfft_homogenize's layout (small strains: 6 components
 * 11 22 33 23 13 12; finite strains: 9 components of H = F - I and of P,
 * row-major); NULL takes that field of the context's last solve.  load,
 * stress_mask: host, as for dbfft_solve; load NULL leaves out[2] and out[3]
 * NaN (stress_mask NULL: strain control).  out: 4 host doubles.  The fields
 * are read, not changed; the context's solution is kept.  A zero
 * denominator gives 0 if the numerator is 0, else infinity.  EINVAL for a
 * NULL context or out, or a NULL field without a solve. */
dbfft_status dbfft_residuals(dbfft_ctx* ctx, const double* strain_dev, const double* stress_dev, const double load[9],
                             const uint8_t stress_mask[9], double out[4]);

/* Fourier unknowns of the last solve: a (device complex doubles
 * [3][n1][n2][n3/2+1]) and the macro strain on the stress-controlled
 * components (host 3x3 row-major); either may be NULL. */
dbfft_status dbfft_get_solution(dbfft_ctx* ctx, void* a_dev, double e_macro[9]);

/* Adjoint gradient of J = G:<sigma> + H:<eps> at the end of the last solve.
 *  ISO_FIELD (small strains, linear): with respect to the per-voxel Young's
 *    modulus.  A second PCG solve with the same operator and stress mask and
 *    load (G on the strain-controlled, -H on the stress-controlled
 *    components) gives eta; grad(x) = eta(x) : C1 : eps(x) / N with C1 the
 *    unit-modulus stiffness.
 *  NEOHOOKE, SVK (finite strains, hyperelastic): J = G:<P> + H:<F> with
 *    respect to a per-voxel factor theta(x) scaling the law's moduli, at
 *    theta = 1.  The response at the end of the path depends on the final
 *    state only, so the checkpoint is the final Newton state: its tangent K
 *    is recomputed, eta solves the linearized cell problem K eta with the
 *    same mask and load as above, and grad(x) = (G + grad eta)(x) : P(x) / N
 *    (P is linear in the moduli).  G, H need not be symmetric.
 *  J2VP_CUBIC (small strains, path-dependent): with respect to a per-voxel
 *    factor theta(x) on the flow stress s0, at theta = 1, through every
 *    increment of the last solve, which must have run with
 *    opts.checkpoint = 1 (EINVAL otherwise).  Backwards over the
 *    increments n, with the plastic-strain multiplier lambda (zero after the
 *    last increment): the return map at the checkpointed state gives the
 *    consistent tangent K_n and the flow increment dp_n; eta_n solves the
 *    linearized cell problem with stress law K_n : eps + lambda -
 *    K_n S lambda (S the grain's elastic compliance), load as above at the
 *    last increment and zero before it; then lambda <- K_n (S lambda -
 *    eps*_n) with eps*_n the adjoint strain, and grad(x) += -m dp_n(x) .
 *    lambda(x) / N.  G, H symmetric.  Every component stress-controlled is
 *    EUNSUPPORTED (the intermediate adjoint problems then have a zero mean
 *    stress, the scale of the residual test).  The context's state is left
 *    as the solve left it.
 * Other kinds (ANISO_GRAIN, ISO_PHASE) return EUNSUPPORTED.  G, H: host
 * row-major 3x3.  grad_dev: device doubles [N].  J_out (host, may be NULL)
 * receives J. */
dbfft_status dbfft_adjoint(dbfft_ctx* ctx, const double G[9], const double H[9], double* grad_dev, double* J_out);

/* Per-kernel timing of PCG iterations with HIP events (only iterations
 * that ran to completion are counted).  A step that is one kernel launch
 * is timed by events the launch itself records at the kernel's start and
 * end (its execution time, as a kernel trace reports it); a step of several
 * launches by events recorded on the context's stream around it.  One
 * iteration per chunk of check_every is timed (the middle one).  Timing
 * launches eagerly (no chunk graph).  Slot k of ms_total / launches
 * (host arrays of 16, either may be NULL) receives the accumulated
 * milliseconds and launch count of kernel kind k:
 *   0 x pass inverse + gradient      1 y pass inverse
 *   2 z pass C2R + tangent + R2C     3 y pass forward
 *   4 x pass forward + divergence    5 unused (the step length is taken by
 *                                      the first block of a pass)
 *   6 CG update x, r, <r, M r>       7 CG direction scalars (scalar)
 *   8 CG direction p = M r + beta p
 * The current totals are returned first; enable = 1 then starts (and, if
 * timing was off, resets) the counters, enable = 0 stops them. */
dbfft_status dbfft_kernel_timing(dbfft_ctx* ctx, int32_t enable, double ms_total[16], int64_t launches[16]);

/* Releases the context and its device memory. */
void dbfft_destroy(dbfft_ctx* ctx);

/* ---------------------------------------------------------------- batches
 * A batch solves the cell problems of several contexts together: the same
 * PCG (Sec. 2.5) and, for the non-linear materials, the same Newton loop
 * with load increments (Sec. 2.4) as dbfft_solve, run in lockstep.  Each
 * batched PCG iteration is one kernel launch per pass covering every cell
 * (grids may differ in size); every cell keeps its own CG scalars and
 * convergence flag, and a chunk of opts->check_every iterations is captured
 * once in a HIP graph and replayed.  The batching itself is not part of the
 * paper's method; per cell the results equal dbfft_solve's up to the order
 * of floating-point reductions, which is the same, so they match bit for
 * bit in practice.
 */
typedef struct dbfft_batch dbfft_batch;

/* Creates a batch over ncell existing contexts (host array of handles).
 * All contexts need the same precision, kinematics and material class
 * (linear: ISO_PHASE / ISO_FIELD / ANISO_GRAIN, mixed freely; non-linear:
 * one of J2VP_CUBIC, NEOHOOKE or SVK for every cell).  The contexts stay owned by the caller and must outlive the
 * batch; a context may belong to several batches but only one call may use
 * it at a time.  use_graph = 0 launches the chunks eagerly instead of
 * replaying a captured graph.  Autotunes the column tile of the x and y
 * passes per distinct grid size (a few timed launches each).  The batch
 * owns a non-blocking stream of its own.
 * Errors: EINVAL (null handle, ncell < 1, mixed classes), ENOMEM, EHIP. */
dbfft_status dbfft_batch_create(dbfft_batch** out, dbfft_ctx* const* cells, int32_t ncell, int32_t use_graph);

/* Solves every cell of the batch.  loads and stress_masks are host arrays
 * of ncell x 9 values (row-major 3x3 per cell, meaning as in dbfft_solve);
 * infos (ncell entries) receives each cell's dbfft_info.  n_increments and
 * dt are shared by all cells.  Afterwards dbfft_homogenize and
 * dbfft_get_solution read each context's result as after dbfft_solve.
 * Each pass runs as one launch over all cells, except when every cell is a
 * small-strain cell of at least 96^3 voxels: such cells are solved by
 * dbfft_solve, whose passes already fill the GPU (and, for power-of-two n1
 * with even n2 and opts.fused_cg, take the fused iteration), two cells at a
 * time, each pair on two non-blocking streams of the batch driven by two
 * host threads (a context listed twice: one at a time); each cell's own
 * stream is synchronized before its solve.  Returns OK when every cell
 * converged, else the status of the last cell that did not (each
 * info.status holds its own); another error of a cell is returned with
 * that cell's message. */
dbfft_status dbfft_batch_solve(dbfft_batch* b, const double* loads, const uint8_t* stress_masks,
                               int32_t n_increments, double dt, const dbfft_opts* opts, dbfft_info* infos);

/* Tiles chosen for each cell: tiles[3 r + 0] and [3 r + 1] are the column
 * tile widths of the x and y passes, tiles[3 r + 2] the z lines per block
 * (host array of 3 ncell int32). */
dbfft_status dbfft_batch_tiles(dbfft_batch* b, int32_t* tiles);

/* Releases the batch (not its contexts). */
void dbfft_batch_destroy(dbfft_batch* b);

/* Message of the last failing call on this thread ("" if none). */
const char* dbfft_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DBFFT_H */
