/*
 * pff.h -- C ABI of the MI355X crack-length-controlled phase-field FFT solver.
 *
 * Method: Aranda & Segurado, "A crack-length control technique for phase
 * field fracture in FFT homogenization".  A periodic voxel RVE (Sec. 3.1)
 * with per-phase stiffness and toughness (Table 2) is loaded along a fixed
 * strain direction f (E_M = f E, Sec. 2.3, Table 1); every step prescribes
 * the next crack length a += delta_a (Sec. 2.3, linear ramp) and solves the
 * monolithic system F(eps_tilde, phi, E) = 0 of Sec. 3.2 (eq.
 * System_CrackLength) by Newton (Algorithm 2) with BiCGSTAB on the
 * matrix-free bordered tangent (eq. CrackLength_linearization).
 *
 * Conventions
 *  - Voxel index i = x + nx*(y + ny*z); nz == 1 means 2D plane strain.
 *  - C = 3 strain components in 2D (Mandel [11, 22, sqrt2*12]), 6 in 3D
 *    (Mandel [11, 22, 33, sqrt2*23, sqrt2*13, sqrt2*12]).
 *  - Fields are structure-of-arrays, component-major: component k of voxel
 *    i at [k*N + i].
 *  - Krylov vectors ("v", "Jv") hold (C+1)*N + 1 entries
 *    [d eps_tilde | d phi | dE] in the solver's working precision: double
 *    for PFF_PREC_FP64, float for PFF_PREC_MIXED.
 *  - Units are voxels (h = 1).
 *  - All entry points return a pff_status: 0 = success, > 0 a solver
 *    outcome, < 0 an error whose text pff_last_error() returns.  No C++
 *    exception crosses the ABI.  A failed call leaves the handle usable.
 *  - Host buffers passed in are copied; the caller keeps ownership.  Device
 *    buffers passed in ("*_dev") belong to the caller, must be device
 *    memory of the current HIP device and must not alias each other.  All
 *    device work is queued on the stream given at creation.  Entry points
 *    returning host data synchronise that stream.
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef PFF_H
#define PFF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PFF_ABI_VERSION 4

typedef int pff_status;
enum {
  PFF_OK = 0,
  PFF_NOT_CONVERGED = 1,   /* Newton or Krylov limit reached; state rolled back */
  PFF_QUEUED = 2,          /* request server: the request has not finished yet */
  PFF_ERR_ARG = -1,        /* invalid argument (NULL, size, range) */
  PFF_ERR_OOM = -2,        /* device allocation failed */
  PFF_ERR_DEVICE = -3,     /* HIP runtime error */
  PFF_ERR_STATE = -4       /* call out of order (e.g. step before bootstrap) */
};

enum { PFF_PREC_FP64 = 0, PFF_PREC_MIXED = 1 };

typedef struct pff_solver pff_solver;

/* Voxel grid. nx, ny >= 2 and nz >= 1, each at most 512.  Lengths with
 * prime factors other than 2 and 3 are allowed: such a factor p takes a
 * generic-radix FFT stage with O(p) work per element. */
typedef struct {
  int nx, ny, nz;
} pff_grid;

/* One material phase (Table 2): Young modulus, Poisson ratio, toughness Gc. */
typedef struct {
  double E, nu, Gc;
} pff_phase;

/* Problem and solver controls.
 *  l            phase-field length scale (voxels), eq. CrackLenght
 *  k_resid      residual stiffness k of g(phi) = (1-phi)^2 + k (eq. gFunct)
 *  f[9]         loading-direction tensor f, 3x3 row-major, symmetric
 *  delta_a      crack-length increment per step (Sec. 2.3 ramp)
 *  alpha        Newton relaxation (Algorithm 2), 0 < alpha <= 1
 *  newton_tol   tolerance of the error measure of eq. errors_crack
 *  krylov_rtol  BiCGSTAB stop ||r|| <= rtol ||b||
 *  precision    PFF_PREC_FP64 or PFF_PREC_MIXED (FP32 tangent/FFT/Krylov
 *               vectors, FP64 residual, inner products, constraint and
 *               load-factor update)
 *  split        PFF_SPLIT_SPECTRAL (0): Miehe spectral split, g degrades
 *               psi0(+) (eq. PlusNegPsi); PFF_SPLIT_NONE (1): isotropic
 *               model of Sec. 5.4, g degrades the whole psi0, which also
 *               drives the history
 *  projection   PFF_PROJ_ROTATED (0): G built with Willot's rotated
 *               frequencies (Sec. 3.1); PFF_PROJ_STANDARD (1): the plain
 *               Fourier frequencies of eq. GFourier, with xi_j = 0 at an
 *               even axis' Nyquist index (its sign is undefined)
 *  w_gamma,     weights of the controlled quantity tau = w_gamma Gamma +
 *  w_load       w_load E (an FFT analogue of eq. FEMweights): F3 = tau(phi,
 *               E) - tau_n, raised by delta_a per increment.  (1, 0) is the
 *               crack-length control of eq. System_CrackLength and is taken
 *               when both are 0; (0, 1) is monolithic strain control, which
 *               can start an uncracked cell.  Both >= 0.
 *  control      PFF_CONTROL_LENGTH (0): Gamma as above; PFF_CONTROL_DISSIPATION
 *               (1): the dissipation D = sum of Gc gamma_f takes its place
 *               (eq. SystemDis, last line), with the border row dD/dphi =
 *               Gc phi/l - (l/2)(Gc Lap phi + Lap(Gc phi)).  Equal up to the
 *               factor Gc for homogeneous toughness.
 *  gc_form      PFF_GC_POINTWISE (0): the printed Gc l Lap phi with pointwise
 *               Gc; PFF_GC_VARIATIONAL (1): l div(Gc grad phi) in finite
 *               differences (forward differences, Gc on the faces as the mean
 *               of the two voxels, backward differences of the fluxes), with
 *               the crack functional on the same finite-difference Laplacian
 *               (symbol -sum 4 sin^2(q/2)).  Crack-length or weighted control
 *               only (not with PFF_CONTROL_DISSIPATION), and not with the
 *               staggered scheme.
 *  macro_bc     PFF_BC_STRAIN (0): the mean strain is f E (Sec. 2.3);
 *               PFF_BC_MIXED (1): the mixed macroscopic conditions that
 *               Sec. 2.3 names as the alternative: only the component of the
 *               mean strain along f is prescribed (by E), and the mean stress
 *               vanishes on every direction Frobenius-orthogonal to f, so
 *               Sigma_M = s f.  Taken in the Galerkin form: the zero mode of
 *               G projects onto the orthogonal complement of f instead of
 *               vanishing, and the strain fluctuation (eps - f E) carries the
 *               free mean strain.  Needs f != 0.
 *  resid_tol    0 (default): Newton stops on the measures of eq.
 *               errors_crack alone.  > 0 ("parity mode"): it also requires
 *               the residual of eq. System_CrackLength at the new state to
 *               satisfy ||F1|| / ||sigma|| <= resid_tol and ||F2|| / ||2H||
 *               <= resid_tol (norms over all voxels; F1 and sigma in the
 *               Mandel components of the strain unknowns).  With a relaxation
 *               alpha < 1 Newton converges linearly, and the update measure
 *               alone leaves the iterate as far from the root as its last
 *               step; the residual stop pins the root itself. */
typedef struct {
  double l, k_resid, f[9], delta_a, alpha, newton_tol, krylov_rtol;
  int newton_maxit, krylov_maxit, precision, split, projection, control, gc_form;
  double w_gamma, w_load;
  int macro_bc;
  double resid_tol;
} pff_params;

enum { PFF_BC_STRAIN = 0, PFF_BC_MIXED = 1 };

enum { PFF_CONTROL_LENGTH = 0, PFF_CONTROL_DISSIPATION = 1 };
enum { PFF_GC_POINTWISE = 0, PFF_GC_VARIATIONAL = 1 };

enum { PFF_SPLIT_SPECTRAL = 0, PFF_SPLIT_NONE = 1 };
enum { PFF_PROJ_ROTATED = 0, PFF_PROJ_STANDARD = 1 };

/* Per-increment outputs (Algorithm 2): macroscopic stress Sigma_M = <sigma>
 * as tensor components [11, 22, 33, 23, 13, 12] (sigma_33 of plane strain
 * included), load factor E, crack length Gamma(phi) and its target a, the
 * three error measures of the last Newton iteration and counters: tangent
 * applies (of which in FP64); in mixed mode the FP64 refinement steps (FP32
 * correction solves after the first) and the Newton iterations whose
 * refinement stalled and was finished by an FP64 BiCGSTAB. */
typedef struct {
  int increment, newton_iters, krylov_iters, converged;
  long long applies, applies_fp64;
  int fp64_fallbacks, refinements;
  double sigma_M[6];
  double load_factor, crack_length, target_a;
  double err[3];
  double seconds;
  double dissipation;      /* D = sum over voxels of Gc gamma_f (eq. JaviGc, middle form), h = 1 */
  double resid[2];         /* ||F1|| / ||sigma||, ||F2|| / ||2H|| at the last Newton iterate */
} pff_increment_result;

/* Device memory hook.  alloc returns at least `bytes` of device memory of
 * the device current at the call (aligned to 256 bytes), or NULL when it
 * cannot; free returns a block alloc gave, with its size.  ctx is passed
 * through.  The library calls them only from pff_create, from the lazy
 * allocation of pff_project (FP32 spectra of an FP64 solver) and from
 * pff_destroy, and for a request server from its worker threads, so they
 * must be thread-safe there.  A NULL pff_allocator, or NULL alloc/free,
 * means hipMalloc / hipFree.  A PyTorch caller passes its caching allocator,
 * so that the solver's fields count in torch's memory accounting. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, size_t bytes, void* ctx);
  void* ctx;
} pff_allocator;

int pff_abi_version(void);

/* Environment read by pff_create (tuning and measurement; the defaults are
 * the measured best on MI355X; none changes the equations solved or the
 * tolerances the results are held to, only launch shapes, fusion and the
 * path of the iterations):
 *   PFF_TRACE=1|2         per-Newton-iteration log (2: also the first BiCGSTAB scalars)
 *   PFF_FUSED=0|1|2       BiCGSTAB steps fused into the applies: 1 (default) the
 *                         inner products in the epilogues, 2 also the FP32 p / s
 *                         updates in the prologues (FP64 solves keep 1)
 *   PFF_INNER32=r         mixed precision: FP32 inner-solve tolerance (default 5e-2)
 *   PFF_ZSPEC=0|1         z pass with register-resident end stages (lengths 32/64/128)
 *   PFF_YREG=0|1|2|3      FP32 3D y passes with register-resident end stages,
 *                         tiles of 16 / 32 / 64 columns (0: LDS Stockham pass)
 *   PFF_FIT_SHAPES=0|1    launch shapes sized to the grid (solvers of a request
 *                         server keep the fixed shapes)
 *   PFF_SUBSTEPS=d        sub-increments of a failing increment (see pff_step)
 *   PFF_X_ROWS, PFF_SPEC_TX, PFF_SPEC_THREADS, PFF_AXIS_TX, PFF_AXIS_THREADS,
 *   PFF_XCD_REMAP         launch knobs of the FFT passes
 * and by pff_server_create: PFF_SERVER_BATCH, PFF_BATCH_CHUNK, PFF_BATCH_MAX,
 * PFF_BATCH_GRAPH (see the request server below). */

/* Create a solver.  phase_id: N bytes (host) with values < n_phases;
 * crack_mask: N bytes (host, 1 = initial crack, phi = 1 there) or NULL;
 * allocator: device memory hook (copied; NULL = hipMalloc), every device
 * buffer of the solver comes from it; hip_stream: a hipStream_t or NULL for
 * the default stream.
 * Errors: PFF_ERR_ARG, PFF_ERR_OOM, PFF_ERR_DEVICE (*out is NULL then). */
pff_status pff_create(const pff_grid* grid, const pff_phase* phases, int n_phases,
                      const uint8_t* phase_id, const uint8_t* crack_mask,
                      const pff_params* params, const pff_allocator* allocator,
                      void* hip_stream, pff_solver** out);

/* Bootstrap (the paper is silent on the start of the path): damage-free Helmholtz
 * solution phi0 with phi = 1 on the crack mask, the control value a0 =
 * w_gamma Gamma(phi0) (= Gamma(phi0) for crack-length control), and the
 * homogeneous-solution predictor E_s for the first increment (root of
 * w_gamma S(E) + w_load E = delta_a, S the crack length of the
 * gradient-free homogeneous damage).
 * Outputs (host, may be NULL): a0, E_s. */
pff_status pff_bootstrap(pff_solver* s, double* a0, double* E_s);

/* One crack-length increment (Algorithm 2): the control value rises by
 * delta_a.  If Newton does not converge (after increment 1), the increment is
 * retried as two half increments from the committed state, recursively down
 * to delta_a / 8 (env PFF_SUBSTEPS = maximum depth, default 3; 0: off); each
 * converged part commits its history, and out reports the final state with
 * the iteration counts of every attempt.  With sub-increments on, a Newton
 * solve whose update measure has not halved its best value for 12 iterations
 * stops early.  On PFF_NOT_CONVERGED the state is rolled back to the last
 * converged increment. */
pff_status pff_step(pff_solver* s, pff_increment_result* out);

/* Strain-controlled implicit staggered scheme (Sec. 3.1, Algorithm 1): the
 * baseline the crack-length control is compared with.  Tolerances:
 * tol_mech on max|d eps~| / (|E| ||f||) of a mechanical Newton step
 * (eq. errors_strain), tol_sta on the stagger error
 * max(||eps~_s - eps~_{s-1}|| / ||f E + eps~_s||, ||phi_s - phi_{s-1}|| / ||phi_s||),
 * cg_rtol on each conjugate-gradient solve (relative residual). */
typedef struct {
  double tol_mech;     /* default 1e-9 */
  double tol_sta;      /* default 1e-8 */
  double cg_rtol;      /* default 1e-11 */
  int max_stagger;     /* default 500 */
  int max_newton;      /* mechanical Newton steps per stagger iteration, default 50 */
  int cg_maxit;        /* default 20000 */
} pff_stagger_params;

typedef struct {
  int increment;
  int converged;
  int stagger_iters;
  int newton_iters;        /* mechanical Newton steps over all stagger iterations */
  long long cg_mech;       /* CG iterations of the mechanical solves */
  long long cg_helm;       /* CG iterations of the Helmholtz solves */
  double E;                /* prescribed load after the increment */
  double crack_length;     /* Gamma(phi) */
  double sigma_M[6];       /* Mandel */
  double err;              /* last stagger error */
  double seconds;
  double dissipation;      /* as in pff_increment_result */
} pff_stagger_result;

/* Effective toughness from a macroscopic path (eq. JaviGc, right-hand form),
 * host only, no device needed: work = integral of Sigma_M : f dE along the n
 * path points (E[k], sigma_M[6k..6k+5] in the order 11, 22, 33, 23, 13, 12,
 * as pff_increment_result reports them) by the trapezoidal rule, starting
 * from the unloaded state (0, 0) and following the path order (segments with
 * decreasing E, the snap-backs of crack-length control, count negative);
 * gceff = volume * work / L_g, with volume the cell volume (N voxels of unit
 * size) and L_g the crack length over which the toughness is measured (the
 * cell length across the crack path, less the initial crack where one is
 * given).  f: 3x3 row-major symmetric.  Outputs may be NULL.  Errors:
 * PFF_ERR_ARG (n < 0, NULL path with n > 0, NULL f, non-positive volume or
 * L_g, non-finite result). */
pff_status pff_effective_toughness(int n, const double* E, const double* sigma_M, const double* f,
                                   double volume, double L_g, double* work, double* gceff);

/* Fill *p with the defaults above.  Errors: PFF_ERR_ARG (p NULL). */
pff_status pff_stagger_defaults(pff_stagger_params* p);

/* One strain-controlled increment: E <- E + dE, then stagger iterations of
 * (i) the mechanical problem G[sigma(f E + eps~, phi)] = 0 at fixed phi,
 * Newton with G[C_i : d eps~] = -G[sigma_i] (eq. LinearOpe_Mech) solved by
 * FP64 conjugate gradients, and (ii) the Helmholtz problem (Gc/l + 2H) phi -
 * Gc l Lap phi = 2H (eq. LinearOpe_Helm) with H = max(psi+(eps), Hn) of the
 * new strain, phi = 1 on the crack mask, divided by Gc and solved by CG, until
 * the stagger error is below tol_sta; then the history is committed.  Starts
 * from the committed state (after pff_bootstrap: phi0, eps~ = 0, E = 0), and
 * leaves a = Gamma(phi) so that crack-length increments may follow.  Runs in
 * FP64 whatever the solver precision.  params may be NULL (defaults).  On
 * PFF_NOT_CONVERGED the state is rolled back.  Errors: PFF_ERR_STATE before
 * bootstrap, PFF_ERR_ARG for a non-positive tolerance or count. */
pff_status pff_stagger_step(pff_solver* s, double dE, const pff_stagger_params* params,
                            pff_stagger_result* out);

/* Copy the committed state to host buffers (any may be NULL):
 * eps_total C*N, phi N, Hn N (history), and scalars E, a. */
pff_status pff_get_state(pff_solver* s, double* eps_total, double* phi, double* Hn,
                         double* E, double* a);

/* Borrowed device pointers of the committed state (any output may be NULL):
 * eps_tilde C*N doubles (the compatible strain fluctuation; the total strain
 * adds f E), phi N doubles, Hn N doubles (history), in the layout of the
 * conventions above.  The solver keeps ownership; the memory is valid until
 * pff_destroy and holds the committed state between calls (pff_step,
 * pff_stagger_step, pff_set_state and pff_load rewrite it).  Work queued on
 * the solver's stream may still be writing it: synchronise that stream
 * before reading on another one.  Writing through the pointers changes the
 * committed state. */
pff_status pff_device_views(pff_solver* s, double** eps_tilde, double** phi, double** Hn);

/* Overwrite the committed state from host buffers (all required):
 * eps_tilde C*N (compatible fluctuation), phi N, Hn N, E, a.  Marks the
 * solver bootstrapped with n increments done. */
pff_status pff_set_state(pff_solver* s, const double* eps_tilde, const double* phi,
                         const double* Hn, double E, double a, int n);

/* Hot path, step (a1)+(a8): constitutive update at the current state and
 * the FP64 residual F = (F1, F2, F3) for target crack length `a`
 * (eq. System_CrackLength); F_dev receives (C+1)*N+1 doubles or may be
 * NULL.  Host outputs (may be NULL): gamma = Gamma(phi), sigma_M[6], and
 * dissipation = sum of Gc gamma_f (the Gc-weighted crack functional, eq.
 * JaviGc middle form). */
pff_status pff_residual(pff_solver* s, double a, double* F_dev, double* gamma,
                        double* sigma_M, double* dissipation);

/* Hot path, steps (a2)-(a6): Jv = dF(q; v) at the state of the last
 * pff_residual call (eq. CrackLength_linearization). v_dev, Jv_dev: Krylov
 * vectors in working precision. */
pff_status pff_apply_tangent(pff_solver* s, const void* v_dev, void* Jv_dev);

/* Steps (a3)-(a5) alone: out = [G(in_1..C) | Lap(in_{C+1})] on C+1 fields
 * of N values (eq. GFourier with rotated frequencies, eq. LinearOpe_Helm).
 * prec selects double (0) or float (1) buffers. */
pff_status pff_project(pff_solver* s, const void* in_dev, void* out_dev, int prec);

/* pff_project without a solver and without allocating: for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same output as pff_project of a
 * solver on this grid with the given projection scheme (PFF_PROJ_ROTATED or
 * PFF_PROJ_STANDARD), the prescribed-mean-strain zero mode and the spectral
 * Laplacian: out = [G(in_1..C) | Lap(in_{C+1})], C+1 fields of N values,
 * double (prec 0) or float (prec 1), device buffers of the current device.
 * The half spectra and axis tables live in a static device array of the
 * library (64 MiB per device, held until the process ends), so the grid is
 * limited to (C+1) (nx/2+1) ny nz complex values of the precision within
 * 64 MiB - 256 KiB (e.g. 128^3 in float, 96^3 in double, 512^2 in either);
 * larger grids return PFF_ERR_ARG before any device work.  The work is only
 * queued on hip_stream (NULL: the default stream); the call neither
 * allocates nor synchronises.  Every call on a device shares that device's
 * array: calls that overlap on one GPU (on different streams or host
 * threads) race and corrupt each other's results; serialise them.  Errors:
 * PFF_ERR_ARG (NULL or aliasing buffers, sizes, options), PFF_ERR_DEVICE. */
pff_status pff_project_noalloc(const pff_grid* grid, int projection, const void* in_dev, void* out_dev,
                               int prec, void* hip_stream);

/* Step (a7): BiCGSTAB on the tangent at the last residual state,
 * x = J^{-1} b.  b_dev, x_dev: Krylov vectors in working precision.
 * Outputs (may be NULL): iterations, relative residual of the returned
 * iterate.  Returns PFF_NOT_CONVERGED if rtol was not reached. */
pff_status pff_krylov_solve(pff_solver* s, const void* b_dev, void* x_dev, double rtol,
                            int maxit, int* iters, double* relres);

/* Kernel timing (measurement support).  With every > 0, each every-th
 * tangent apply brackets its FFT pass kernels with HIP events on the solver
 * stream; with every < 0, each |every|-th apply carries only the two events
 * around the whole apply (slot k = 5; the per-pass slots do not advance), which
 * perturbs the timed apply less; every = 0 disables.  pff_timing_read(slot) returns the number of
 * timed launches and their summed duration in milliseconds for
 * slot = 6 * (5 * prec + variant) + k, with prec 1 for FP32 applies and 0
 * for FP64 ones; variant 0 a plain apply, 1 (3) the apply whose epilogue
 * forms the BiCGSTAB product (r_hat, v) (and whose prologue forms the
 * direction p), 2 (4) the apply whose epilogue forms (t, s), (t, t) (and
 * whose prologue forms s); k = 0 x-forward pass (with the tangent prologue), 1 first strided-axis
 * pass (y; with the spectral stage in 2D), 2 z pass with the spectral stage
 * (3D), 3 inverse y pass (3D), 4 x-inverse pass (with the epilogue),
 * 5 the whole apply.  Reading synchronises the stream and resets nothing. */
pff_status pff_timing(pff_solver* s, int every);
pff_status pff_timing_read(pff_solver* s, int kernel, long long* count, double* ms);

/* Counters since creation: tangent applies, Krylov iterations. */
pff_status pff_counters(pff_solver* s, long long* applies, long long* krylov_iters);

/* Serialised committed state (checkpoint/resume).  pff_save with
 * buf == NULL returns the size in *bytes. */
pff_status pff_save(pff_solver* s, void* buf, size_t* bytes);
pff_status pff_load(pff_solver* s, const void* buf, size_t bytes);

/* Text of the last error on this handle ("" if none); with a NULL handle,
 * the text of the last failed pff_create on the calling thread ("null
 * handle" if none). */
const char* pff_last_error(const pff_solver* s);

void pff_destroy(pff_solver* s);

/* Device bytes held by a solver (all of its buffers). */
pff_status pff_solver_bytes(pff_solver* s, size_t* bytes);

/* Device bytes a solver of this grid and precision (PFF_PREC_*) allocates,
 * computed on the host without touching the device (the request server's
 * admission estimate; equal to pff_solver_bytes of such a solver). */
pff_status pff_footprint_bytes(const pff_grid* grid, int precision, size_t* bytes);

/* ---- Request server (continuous batching of RVE solves on one GPU) ----------
 * The paper solves one RVE; a service running many RVE problems (a
 * parametric or multiscale study) submits them here.  A request is one
 * problem as in pff_create plus a number of crack-length increments; its
 * results are the per-increment outputs of pff_step.  Requests wait in
 * arrival order and are admitted while one of max_slots slots is free and
 * their footprint (pff_footprint_bytes) fits into hbm_budget_bytes minus the
 * footprints of the running requests; a request that has been overtaken 8
 * times stops further overtaking.  Each slot is a host thread with its own
 * non-blocking HIP stream on the device current at pff_server_create, so
 * running requests overlap on the device.  The FP32 Krylov solves of the
 * mixed-precision requests are batched: an engine thread groups the solves
 * in flight by grid and advances each group by a chunk of BiCGSTAB
 * iterations (env PFF_BATCH_CHUNK, default 4) whose kernels each cover the
 * whole group (at most PFF_BATCH_MAX solves, default 8), replayed from a
 * captured HIP graph (PFF_BATCH_GRAPH=0: launched directly); a solve joins
 * or leaves its group between chunks.  PFF_SERVER_BATCH=0 solves every
 * request on its slot's stream instead.  The engine holds a few kilobytes of
 * hipMalloc memory per grid.  A request gives the same
 * results alone and in a mix.  Inputs are copied at submission.  All
 * functions are thread-safe.  Times are seconds since pff_server_create. */
typedef struct pff_server pff_server;

typedef struct {
  uint64_t ticket;
  int state;              /* 0 queued, 1 running, 2 done */
  int status;             /* final status of the solve once done */
  int n_done;             /* increments finished */
  int slot;               /* slot that ran it, -1 before admission */
  size_t footprint;       /* admission estimate, bytes */
  double t_submit, t_admit, t_done;
  double a0, E_s;         /* bootstrap outputs */
} pff_request_info;

typedef struct {
  long long submitted, completed, queued, running, max_running;
  int slots, reserved;
  size_t budget, bytes_in_use, peak_bytes;
  double clock;           /* server time of this snapshot */
  /* batched FP32 inner solves: chunks launched, solves and BiCGSTAB
   * iterations finished, graphs captured, the largest and the mean number
   * of solves in one chunk */
  long long batch_chunks, batch_solves, batch_iterations, batch_graphs;
  int batch_max, reserved2;
  double batch_mean;
} pff_server_stats;

/* Starts max_slots (1..64) worker threads.  allocator: as in pff_create
 * (copied; NULL = hipMalloc), used for every request's solver from the
 * worker threads.  PFF_ERR_DEVICE without a GPU. */
pff_status pff_server_create(size_t hbm_budget_bytes, int max_slots, const pff_allocator* allocator,
                             pff_server** out);
/* Queues a request; *ticket identifies it.  PFF_ERR_ARG if its footprint
 * exceeds the budget. */
pff_status pff_server_submit(pff_server* srv, const pff_grid* grid, const pff_phase* phases, int n_phases,
                             const uint8_t* phase_id, const uint8_t* crack_mask, const pff_params* params,
                             int n_increments, uint64_t* ticket);
/* Blocks until the request is done (timeout_seconds < 0: no limit).
 * PFF_OK when done, PFF_QUEUED on time-out. */
pff_status pff_server_wait(pff_server* srv, uint64_t ticket, double timeout_seconds);
pff_status pff_server_info(pff_server* srv, uint64_t ticket, pff_request_info* out);
/* Copies up to capacity per-increment results of a finished request;
 * *n_out = number available.  PFF_QUEUED if not finished. */
pff_status pff_server_results(pff_server* srv, uint64_t ticket, pff_increment_result* out, int capacity,
                              int* n_out);
/* Forgets a finished request.  PFF_ERR_STATE while it runs or while a
 * thread waits on it in pff_server_wait. */
pff_status pff_server_release(pff_server* srv, uint64_t ticket);
pff_status pff_server_get_stats(pff_server* srv, pff_server_stats* out);
/* Text of the last error of a server call, or of the last request that
 * ended with an error or without convergence ("request <ticket> (status
 * <status>): <text>"). */
const char* pff_server_last_error(pff_server* srv);
/* Finishes the running requests, drops the queued ones, joins the slots. */
void pff_server_destroy(pff_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* PFF_H */
