/*
 * klst.h -- C ABI of the MI355X kinetic linear stability (kLST) eigen-solver.
 *
 * The library solves the generalized eigenproblem A q = lambda B q of the
 * BGK-linearised reduced Boltzmann equation for a 1-D normal shock with a
 * transverse normal mode exp(i(beta y - omega t)), lambda = i omega
 * (paper Sec. 2.2, eqs. Comp1DHarm, comp_ghat1Dshock, comp_hhat1Dshock,
 * MatrixSystem; Sec. 4 eq. MatrixProblem), discretised with mapped
 * Chebyshev-Gauss-Lobatto collocation in x (Sec. 3.1) times a micro-velocity
 * node table (Sec. 3.2).  It returns the eigenvalues nearest a target sigma
 * with their right eigenvectors, computed by Jacobi-Davidson with a
 * block-Jacobi ILU(0) preconditioned GMRES correction equation (Sec. 4.2).
 *
 * Conventions shared by every entry point
 *  - Complex numbers cross the ABI as interleaved (re, im) double pairs.
 *  - Unknown ordering: q[(2 j + f) * Nxi + k], j = spatial node (j = 0 at
 *    x = +s_inf, downstream), f = 0 for g_hat and 1 for h_hat, k = velocity
 *    node.  n = 2 Ny Nxi.
 *  - Inflow rows (j = Ny-1 with xi_x > 0, j = 0 with xi_x < 0) are identity
 *    rows of A and zero rows of B (zero-perturbation Dirichlet conditions of
 *    Sec. 2.2), so finite eigenvectors vanish there.
 *  - Every entry point returns a klst_status; nothing throws or exits.  On
 *    error, klst_last_error() describes the cause.  Input arrays are copied;
 *    the caller keeps ownership of everything it passes.  Output buffers are
 *    caller-allocated.  A context is not thread-safe: use one per host thread.
 *  - "device" pointers are HIP device addresses on the context's device (for
 *    example torch tensor data_ptr()); work is ordered on the context's stream.
 */
#ifndef KLST_H
#define KLST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct klst_ctx klst_ctx;

typedef enum {
  KLST_OK = 0,
  KLST_EINVAL = 1,      /* bad argument or inconsistent input                   */
  KLST_ENOMEM = 2,      /* device or host allocation failed                     */
  KLST_EDEVICE = 3,     /* HIP runtime error, or no usable device               */
  KLST_ENOCONV = 4,     /* max_it reached; the first nconv results are valid    */
  KLST_EBUSY = 5,       /* (served mode) not admitted: slots or memory are full */
  KLST_ECANCELLED = 6,  /* (served mode) request was cancelled                  */
  KLST_ESTATE = 7       /* call out of order (e.g. solve before assemble)       */
} klst_status;

/* Solver options (defaults from klst_default_options).  Paper defaults for the
 * JD solve are listed in its Appendix C; the values here follow the same
 * scheme: tol on ||A u - theta B u|| / (|theta| ||u||) (JD locks a Schur pair at
 * tol / 2 so that the returned eigenvectors meet tol), restart from m_max to
 * m_min, correction equations solved by GMRES restarted every gmres_m steps,
 * up to inner_max_it steps or a residual reduction of inner_rtol. */
typedef struct {
  int device;           /* HIP device ordinal                                        */
  void* stream;         /* hipStream_t to order work on; NULL = the default stream   */
  int precision;        /* 0 = FP64 everywhere; 1 = FP32 inner GMRES + preconditioner
                           inside an FP64 iterative refinement of the correction eq. */
  int op_mode;          /* 0 = matrix-free operator; 1 = explicit CSR (built on device) */
  int lines_per_block;  /* block-Jacobi block = this many whole velocity lines       */
  int m_max, m_min;     /* search-space size before / after a restart (m_max <= 248) */
  int gmres_m;          /* GMRES restart length (Krylov vectors per cycle)           */
  int max_it;           /* outer-iteration budget                                    */
  double tol;           /* eigenpair acceptance: relative residual                   */
  double inner_rtol;    /* correction-equation relative tolerance                    */
  double fix;           /* correction shift = sigma until rel. residual < fix        */
  uint64_t seed;        /* start vector: counter-based SplitMix64 stream             */
  int pc_kernel;        /* preconditioner K ~ A - sigma B: 0 = block-Jacobi ILU(0)
                           (Sec. 4.3) applied by level-set triangular sweeps; 1 = the
                           same (L U)^{-1} applied as a stored dense inverse per block
                           (batched GEMV); 2 = the exact inverse in structured form:
                           velocity-line inverses of the streaming + relaxation part
                           and the (r Ny)^2 moment capacitance (Woodbury identity),
                           lines_per_block unused (the default).  Mixed precision
                           needs 1 or 2.                                             */
  int inner_max_it;     /* GMRES steps per correction equation, over all restarts;
                           values <= gmres_m give one unrestarted cycle; 0 (the
                           default) = gmres_m in FP64 and 3 gmres_m in mixed
                           precision (three FP64-refined FP32 cycles: one FP32
                           cycle alone can stall the outer iteration near
                           relative residual 1e-7 at ill-conditioned pairs)     */
  int reorth;           /* GMRES Arnoldi orthogonalisation: 0 = classical Gram-Schmidt
                           twice (CGS2, the default); 1 = second pass only when the
                           first keeps less than 1/sqrt(2) of the norm (DGKS test,
                           on the device)                                            */
  int method;           /* klst_solve's eigensolver: 0 = Jacobi-Davidson (default);
                           1 = shift-invert Krylov-Schur (klst_solve_shift_invert)  */
  int krylov32;         /* FP64 solves (precision 0): 1 = store the inner GMRES
                           Krylov basis in FP32 (arithmetic, operator,
                           preconditioner and the outer iteration stay FP64; the
                           Gram-Schmidt passes read half the bytes); 0 = FP64
                           basis (default).  Ignored in mixed precision, whose
                           basis is FP32 already.                                    */
} klst_options;

/* Spatial grid: Ny Chebyshev-Gauss-Lobatto points mapped to [-s_inf, s_inf]
 * by x = L y / sqrt(1 + s - y^2), s = (L/s_inf)^2 (Sec. 3.1, eq. Chebmapping). */
typedef struct {
  int Ny;
  double L;
  double s_inf;
} klst_grid;

/* Micro-velocity node table (Sec. 3.2), Nxi nodes with weights w > 0.  Dv = 2
 * resolves (xi_x, xi_y) and couples rho, u, v, E (rank 4); Dv = 1 requires
 * xi_y == 0 and couples rho, u, E (rank 3). */
typedef struct {
  int Nxi;
  const double* xi_x;   /* [Nxi] host */
  const double* xi_y;   /* [Nxi] host */
  const double* w;      /* [Nxi] host */
  int Dv;
} klst_vel;

/* Base flow on the Ny nodes.  mode 0 (EQ): macros rho, u, T given and the base
 * VDFs are the local Maxwellians.  mode 1 (NONEQ): reduced VDFs g_c, h_c
 * [Ny * Nxi] given; macros are their discrete moments.  Collision rate
 * nu = nu_inf * rho * T^(1 - s_visc) (BGK rate P/mu with mu ~ T^s, Sec. 2.1). */
typedef struct {
  int mode;
  const double *rho, *u, *T;   /* [Ny] host, mode 0 */
  const double *g_c, *h_c;     /* [Ny*Nxi] host, mode 1, row-major (j, k) */
  double s_visc;
  double nu_inf;
} klst_base;

/* Per-solve statistics of the last klst_solve. */
typedef struct {
  int outer_iterations;
  int inner_iterations;      /* total GMRES steps                               */
  int restarts;
  int nconv;
  int pivots_floored;        /* ILU(0) pivots raised to 1e-12 x row 1-norm      */
  double seconds_total;      /* wall time of klst_solve                         */
  double seconds_setup;      /* preconditioner set-up inside klst_solve         */
  double seconds_host;       /* host time in the projected dense problems       */
  double seconds_wait;       /* host time blocked on device results (syncs)     */
  int64_t op_applies;
  int64_t pc_applies;
} klst_stats;

void        klst_default_options(klst_options* opt);
const char* klst_strerror(klst_status s);
const char* klst_last_error(const klst_ctx* ctx);

/* Create a context bound to opt->device.  Allocates no problem memory yet.
 * Errors: EINVAL (bad options), EDEVICE (no such device / HIP failure). */
klst_status klst_create(klst_ctx** out, const klst_options* opt);
void        klst_destroy(klst_ctx* ctx);

/* Build the discrete operator of Sec. 2.2 for this grid, velocity table, base
 * flow and transverse wavenumber beta; uploads coefficient tables (and, in
 * op_mode 1, generates the CSR matrix on the device).  Replaces any previous
 * problem in ctx.  Errors: EINVAL (Ny < 3, Nxi < 1, w <= 0, non-finite input,
 * rho <= 0 or T <= 0 after moments, Dv = 1 with xi_y != 0), ENOMEM, EDEVICE. */
klst_status klst_assemble(klst_ctx* ctx, const klst_grid* grid, const klst_vel* vel,
                          const klst_base* base, double beta);

/* Problem sizes: n unknowns, structural nnz of A (n (Ny-1+2Nxi) - n_bc (Ny-2+2Nxi)),
 * number of inflow rows.  Any pointer may be NULL. */
klst_status klst_dims(const klst_ctx* ctx, int64_t* n, int64_t* nnz, int* n_bc);

/* y = (A - tau B) x for device vectors x, y of n complex doubles (the operator
 * rows of eqs. comp_ghat1Dshock / comp_hhat1Dshock).  x and y must not
 * overlap.  Uses op_mode's operator.  Errors: ESTATE (no problem), EINVAL. */
klst_status klst_apply(klst_ctx* ctx, const double tau[2], const void* x, void* y);

/* The same product in FP32, as the inner solve of a mixed-precision context
 * computes it (Sec. 4.2's operator with every table rounded to FP32, the
 * streaming sum on the FP32 matrix cores, FP32 accumulation): x and y are
 * device arrays of n complex floats (interleaved re, im).  Errors: ESTATE (no
 * problem, or the context is not mixed precision), EINVAL, EDEVICE. */
klst_status klst_apply_f32(klst_ctx* ctx, const double tau[2], const void* x, void* y);

/* The FP32 product batched over nvec vectors of n complex floats stored
 * contiguously (vector i at x + i n, device memory; x and y must not
 * overlap): the FP32 moment sums of every vector, then the FP32 matrix-core
 * operator over all of them in one launch.  Each vector's result is the FP32
 * product above up to the rounding of its tiling (the launch shape depends on
 * nvec).  The FP32 moment partials grow to nvec vectors on first use (context
 * memory, freed with the problem).  Errors: ESTATE (no problem, or the context
 * is not mixed precision), EINVAL (null pointer, nvec outside 1..65535),
 * ENOMEM, EDEVICE. */
klst_status klst_apply_many_f32(klst_ctx* ctx, const double tau[2], int nvec, const void* x, void* y);

/* Same product, batched over nvec vectors stored contiguously (vector i at
 * x + i n).  Matrix-free only. */
klst_status klst_apply_many(klst_ctx* ctx, const double tau[2], int nvec, const void* x, void* y);

/* klst_apply_many without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same product, same kernels and bit-identical results as
 * klst_apply_many; the moment partial sums and their totals go to a
 * library-owned device array of 2^19 complex doubles (8 MiB per GPU, held until
 * the process ends) instead of context memory, so nvec * Ny * r * 9 must not
 * exceed 2^19 (r = 4 for
 * Dv = 2, 3 for Dv = 1).  The array is shared by every call on the GPU: calls
 * that overlap on one GPU (two streams, two threads) race and give undefined
 * results; calls ordered on one stream are safe.  Nothing in it needs to start
 * at zero.  Errors: ESTATE (no problem), EINVAL (null pointer, nvec < 1, or the
 * size limit above), EDEVICE. */
klst_status klst_apply_many_noalloc(klst_ctx* ctx, const double tau[2], int nvec, const void* x, void* y);

/* y = (A - tau B) x with the explicit CSR matrix regardless of op_mode
 * (generated on first use).  Errors: ENOMEM if the matrix does not fit. */
klst_status klst_apply_csr(klst_ctx* ctx, const double tau[2], const void* x, void* y);

/* Set up the block-Jacobi ILU(0) preconditioner of (A - sigma B) (Sec. 4.2,
 * eqs. ilu and bjilu): contiguous row blocks of `lines_per_block` whole
 * velocity lines in the velocity-major ordering (field, velocity node, spatial
 * node).  klst_solve calls this itself; exposed for testing. */
klst_status klst_precond_setup(klst_ctx* ctx, const double sigma[2]);

/* y = K^{-1} x with the current preconditioner, device vectors. */
klst_status klst_precond_apply(klst_ctx* ctx, const void* x, void* y);

/* y = P^{-1} x for device vectors: one pass of the velocity-line inverses of
 * the structured preconditioner alone (the block-diagonal streaming +
 * relaxation part P of A - sigma B with unit inflow rows, one Ny x Ny inverse
 * per velocity node, Sec. 2.2 rows with the moment coupling left out), the
 * first half of what klst_precond_apply applies.  Needs klst_precond_setup
 * with pc_kernel 2.  x and y must not overlap.  Errors: ESTATE, EINVAL. */
klst_status klst_precond_apply_lines(klst_ctx* ctx, const void* x, void* y);

/* Copy out the structured inverse that klst_precond_setup built on the device
 * (pc_kernel 2; the exact (A - sigma B)^{-1} in the Woodbury form of the
 * velocity-line blocks of Sec. 2.2's streaming + relaxation rows and the
 * moment capacitance): Pinv [nslots][Ny x Ny] column-major line inverses
 * (slot s holds node slot_node[s]; with sigma real a node's xi_y mirror is
 * served by the conjugate and has no slot of its own), Sinv [(r Ny)^2]
 * row-major capacitance inverse (index q = j r + a), both complex doubles on
 * the host.  *nslots receives the slot count; any array may be NULL (query
 * nslots first to size Pinv).  Errors: ESTATE, EINVAL. */
klst_status klst_precond_export(klst_ctx* ctx, double* Pinv, double* Sinv, int* slot_node, int* nslots);

/* Host-only (no device needed): the same structured inverse built by the host
 * (LU with partial pivoting per line block and for the capacitance), in the
 * layout of klst_precond_export, for testing the device set-up.  Errors:
 * EINVAL (bad input, as klst_assemble), ENOCONV (a singular block). */
klst_status klst_host_structured_inverse(const klst_grid* grid, const klst_vel* vel, const klst_base* base,
                                         double beta, const double sigma[2], double* Pinv, double* Sinv,
                                         int* slot_node, int* nslots);

/* Copy out the explicit CSR matrix of A (Sec. 4.3's stored form; B is the
 * diagonal 0/1 mask of non-inflow rows): rowptr [n + 1] int64, col [nnz] int32
 * (ascending within a row), val [nnz] complex doubles (interleaved re, im),
 * nnz as klst_dims reports.  on_device = 1: the three buffers are device
 * memory, else host memory; all are caller-allocated.  Generates the matrix on
 * the device first if op_mode 0 had not.  Errors: ESTATE (no problem), EINVAL,
 * ENOMEM (the matrix does not fit). */
klst_status klst_export_csr(klst_ctx* ctx, void* rowptr, void* col, void* val, int on_device);

/* Jacobi-Davidson solve for the nev eigenvalues nearest sigma (Sec. 4.2).
 * Pairs are locked as they converge; once nev are locked the iteration goes on
 * until max(1, nev / 25) consecutive newly locked eigenvalues were not nearer
 * sigma than the nev-th nearest locked one (at most min(2 nev, 100, 250 - m_max)
 * pairs are locked), or until the current Petrov pair has stayed below relative
 * residual 1e-6 and, by a margin of sqrt(residual) |theta|, not nearer than
 * that eigenvalue for 50 consecutive outer iterations without a lock (a guard
 * next to a nearly defective pair, whose attainable residual lies above the
 * tolerance).  With sigma real and a problem symmetric under the xi_y
 * reflection R (mirrored velocity table, even coupling tables), each locked
 * complex eigenvalue also contributes its exact partner (conj(lambda),
 * R conj(x)) when that partner was not locked itself; partnership is read from
 * the eigenvectors as klst_host_select_output describes.  The
 * nev nearest are returned, ordered by |lambda - sigma| (ties: Im lambda > 0
 * first).
 * lambda: [2*nev] host doubles.  X: [nev * n] complex doubles (eigenvector i at
 * X + 2 n i doubles), on the host or the device (X_on_device), or NULL.
 * Eigenvectors are scaled to unit 2-norm with the largest entry real positive.
 * resid: [nev] host relative residuals ||A x - lambda B x|| / (|lambda| ||x||),
 * or NULL.  nconv: converged count.  Returns ENOCONV (with nconv < nev valid
 * results) when max_it is reached before nev pairs converge.  Errors: ESTATE,
 * EINVAL (nev < 1, nev > min(100, n - n_bc), nev + m_max > 250), ENOMEM, EDEVICE. */
klst_status klst_solve(klst_ctx* ctx, const double sigma[2], int nev, double* lambda,
                       void* X, int X_on_device, double* resid, int* nconv);

/* Shift-invert Krylov-Schur solve for the nev eigenvalues nearest sigma: Arnoldi
 * on (A - sigma B)^{-1} B as in the paper's Method 1 (Sec. 4.1), with the exact
 * structured inverse (pc_kernel 2's factorization) in place of a sparse LU, and
 * Krylov-Schur restarts that keep the min(m_max - 2, nev + (m_max - nev) / 2)
 * leading Schur vectors.  m_max is the search-space size (at least nev + 2),
 * max_it the number of restarts, tol the acceptance gate on the FP64 pencil
 * residual of all nev leading Ritz pairs.  Outputs as klst_solve (nev nearest,
 * ordered by distance); stats count restarts as outer iterations and operator
 * applications as inner ones.  Errors: as klst_solve; ENOCONV also on a Krylov
 * breakdown. */
klst_status klst_solve_shift_invert(klst_ctx* ctx, const double sigma[2], int nev, double* lambda,
                                    void* X, int X_on_device, double* resid, int* nconv);

/* ---------------------------------------------------------------------------
 * Launch autotuning.  The library keeps a process-wide table of launch choices
 * keyed by (Ny, Nxi, nvec, precision): row tiles and wavefronts of the
 * matrix-core operator (apply_tile, apply_waves; apply_waves = 8 selects the
 * streaming many-vector kernel, the default from 8 vectors on at shapes with
 * at least 4 groups of 8 column tiles; for FP32, apply_waves 1 or 4 select the
 * FP32 matrix-core kernel and apply_waves 0 the scalar one with apply_tile =
 * 4, 8 or 16 rows per thread), column parts of the moment sums
 * (moment_splits) and wavefronts of the block GEMVs of the preconditioners
 * (gemv_waves); 0 = the built-in heuristic.  FP64 tile and wave choices leave
 * results bit-identical (FP32 ones round differently); moment splits
 * and GEMV waves change the order of summation, so the table must be fixed
 * before the solves it serves (solves that run under one table give the same
 * results alone and together).  Moment splits and GEMV waves are per shape
 * (read from the nvec = 1 entry for every batch size).
 * ------------------------------------------------------------------------- */
typedef struct {
  int Ny, Nxi, nvec, precision;                                 /* key                   */
  int apply_tile, apply_waves, moment_splits, gemv_waves;       /* chosen (0: heuristic) */
  double us_default, us_tuned;   /* operator (+ preconditioner when set up, nvec = 1)
                                    microseconds per application, heuristic and tuned */
} klst_tune_entry;

/* Time the candidate launch choices on ctx's assembled problem (nvec vectors;
 * precision 0 = FP64 operator and preconditioner, 1 = the FP32 inner ones of a
 * mixed-precision context, nvec = 1), reps applications per candidate, on the
 * context's stream: operator tiling first, then (nvec = 1) the moment splits of
 * operator + preconditioner together, then the preconditioner's GEMV waves when
 * klst_precond_setup has run.  Installs the fastest in the table and reports it
 * in *out (may be NULL).  Allocates 2 nvec + 1 vectors of scratch.  Errors:
 * ESTATE (no problem), EINVAL, ENOMEM. */
klst_status klst_autotune(klst_ctx* ctx, int nvec, int precision, int reps, klst_tune_entry* out);

/* Write / read the launch table as text (one entry per line: Ny Nxi nvec
 * precision apply_tile apply_waves moment_splits gemv_waves; '#' comments).
 * Loading adds to or replaces entries of the current table.  Errors: EINVAL
 * (unreadable file or malformed line; entries before it are loaded). */
klst_status klst_tune_save(const char* path);
klst_status klst_tune_load(const char* path);
/* Empty the launch table (every launch back to the built-in heuristic). */
void        klst_tune_clear(void);

/* Statistics of the last solve. */
klst_status klst_get_stats(const klst_ctx* ctx, klst_stats* out);

/* Convergence history of the last solve: one record of KLST_HISTORY_FIELDS
 * doubles per outer iteration that ended in a correction equation, namely
 * (outer iteration, pairs locked so far, relative residual ||r|| / |theta| of the
 * selected Petrov pair, Re theta, Im theta, 1 if the correction equation was
 * shifted by theta rather than sigma).  Copies min(cap, count) records into rec
 * (host, caller-owned); *count receives the total.  Errors: EINVAL. */
#define KLST_HISTORY_FIELDS 6
klst_status klst_get_history(const klst_ctx* ctx, double* rec, int cap, int* count);

/* ---------------------------------------------------------------------------
 * Post-processing of eigenvectors and of the base flow.
 * ------------------------------------------------------------------------- */

/* Macroscopic perturbations carried by nvec vectors of the assembled problem
 * (eigenvectors returned by a solve, for instance), at every spatial node: the
 * velocity integrals that define rho_hat, u_hat, v_hat and E_hat (Sec. 2.2, the
 * perturbation-macro integrals), linearised about the base state like the
 * operator's moment coupling, T_hat = (4/3)(E_hat - u u_hat), and the velocity
 * amplitude |U_hat| = sqrt(|u_hat|^2 + |v_hat|^2) of Sec. 5 (eq. Unormpert).
 *   X      device, nvec x n complex doubles (interleaved re, im), vector v at
 *          X + 2 n v doubles, in the (2 j + f) Nxi + k ordering.
 *   macros device, [nvec][Ny][5] complex doubles: rho_hat, u_hat, v_hat (0 when
 *          Dv = 1), E_hat, T_hat.
 *   umag   device, [nvec][Ny] doubles: |U_hat| divided by its maximum over the
 *          nodes (all zero when that maximum is zero).
 * Queued on the ctx stream (asynchronous like klst_apply); X must not overlap
 * the outputs.  Errors: ESTATE (no problem), EINVAL (null pointer, nvec < 1 or
 * nvec > 65535), ENOMEM. */
klst_status klst_perturbation_macros(klst_ctx* ctx, const void* X, int nvec, void* macros, double* umag);

/* Translational non-equilibrium level of the assembled base flow at every
 * spatial node, E_neq(x_j) = sqrt(sum_k W_k (g_c - g^e)^2) (Sec. 5, eq. L2norm),
 * with the reduced base g_c in place of f and g^e the reduced Maxwellian at the
 * node's macros.  Zero for an EQ base (g_c = g^e).
 *   eneq   device, [Ny] doubles.
 * Queued on the ctx stream.  Errors: ESTATE (no problem), EINVAL (null pointer). */
klst_status klst_noneq_level(klst_ctx* ctx, double* eneq);

/* BE-BGK base-flow relaxation (Sec. 3.3): march the reduced 1D2V BGK equations
 * d(g, h)/dt = nu ((g^e, h^e) - (g, h)) - xi_x d(g, h)/dx to a steady shock with
 * classical RK4 steps of size dt.  x-derivative: finite volumes on the mapped
 * Chebyshev nodes of `grid` (cell widths (x_{j-1} - x_{j+1}) / 2), interface
 * values by MUSCL reconstruction upwinded on xi_x with the minmod limiter;
 * values beyond the two end nodes repeat the end node.  Collision: the reduced
 * Maxwellians at each node's discrete macros (transverse velocity 0),
 * nu = nu_inf rho T^(1 - s_visc).  The two end nodes keep their input states
 * (the Rankine-Hugoniot boundary conditions).
 *   g, h        host, [Ny][Nxi] row-major; in: the start state, out: the state
 *               after the last step (the caller keeps ownership).
 *   max_steps   step budget (0: only the residual is evaluated).
 *   tol, check_every  with tol > 0, max |RHS| is checked before every
 *               check_every-th step and the march stops once it is <= tol.
 *   steps_done  (optional) steps taken; resid (optional) max |RHS| of the
 *               returned state.
 * Runs on ctx's device and stream (no assembled problem needed) and returns
 * when the result is on the host.  Errors: EINVAL (Ny < 3, Nxi < 1, Dv not 1 or
 * 2, w <= 0, dt <= 0, non-finite input), ENOMEM, ENOCONV (the state became
 * non-finite: dt too large for the grid). */
klst_status klst_bgk_relax(klst_ctx* ctx, const klst_grid* grid, const klst_vel* vel, double nu_inf,
                           double s_visc, double* g, double* h, double dt, int max_steps, double tol,
                           int check_every, int* steps_done, double* resid);

/* ---------------------------------------------------------------------------
 * Served / batched stability sweeps: many independent solves (different grids,
 * wavenumbers, Mach numbers, base flows) sharing one GPU.  A server owns `slots`
 * contexts, each on its own stream and worker thread.  Requests are admitted in
 * submission order as soon as a slot is free and their modelled HBM footprint
 * (klst_footprint_bytes) fits under the budget, so requests that arrive while
 * others run overlap with them on the device (continuous batching).  Every
 * request runs alone on its context with deterministic kernels: its result is the
 * same whether it ran alone or in a mix.
 * ------------------------------------------------------------------------- */
typedef struct klst_server klst_server;

/* Device bytes one solve of this shape allocates with these options (tables,
 * preconditioner, workspace); the admission model. 0 for invalid sizes. */
size_t      klst_footprint_bytes(int Ny, int Nxi, int nev, const klst_options* opt);

/* Start a server: `slots` concurrent solves (1..64) on opt->device, admitting
 * requests while their summed footprints stay <= hbm_budget_bytes (0: 80% of the
 * free device memory).  want_vectors = 0 keeps only eigenvalues and residuals.
 * opt->stream is ignored (each slot creates its own default-priority stream).
 * Errors: EINVAL, EDEVICE, ENOMEM. */
klst_status klst_server_create(klst_server** out, const klst_options* opt, int slots,
                               size_t hbm_budget_bytes, int want_vectors);
/* Cancels everything queued or running, joins the workers, frees the device. */
void        klst_server_destroy(klst_server* sv);

/* Queue one solve (inputs are copied; the caller keeps ownership).  Returns a
 * ticket.  Errors: EINVAL (bad input, as klst_assemble / klst_solve), ENOMEM
 * (footprint larger than the whole budget), EBUSY (queue full). */
klst_status klst_submit(klst_server* sv, const klst_grid* grid, const klst_vel* vel,
                        const klst_base* base, double beta, const double sigma[2], int nev,
                        uint64_t* ticket);
/* state: 0 queued, 1 running, 2 done (OK or ENOCONV), 3 failed, 4 cancelled. */
klst_status klst_poll(klst_server* sv, uint64_t ticket, int* state);
/* Block until the request is finished (timeout_s < 0: no limit); EBUSY on timeout. */
klst_status klst_wait(klst_server* sv, uint64_t ticket, double timeout_s);
/* Ask a queued or running request to stop; a running solve stops at its next
 * outer iteration and finishes with ECANCELLED. */
klst_status klst_cancel(klst_server* sv, uint64_t ticket);
/* Copy out the results of a finished request and forget it.  lambda [2*nev],
 * X [nev*n] complex host (if vectors were kept), resid [nev], timing[3] =
 * {queueing s, service s, latency s = completion - submission}.  Any output may be
 * NULL.  Returns the request's own status (OK, ENOCONV, ECANCELLED, ...), or EBUSY
 * if it has not finished. */
klst_status klst_fetch(klst_server* sv, uint64_t ticket, double* lambda, void* X, double* resid,
                       int* nconv, double timing[3], klst_stats* stats);
/* Peak number of concurrently running solves, peak admitted footprint, budget. */
klst_status klst_server_stats(klst_server* sv, int* peak_running, size_t* peak_bytes,
                              size_t* budget);

/* Host-only (no device needed): the tables klst_assemble builds, for testing
 * against an independent implementation.  Dx [Ny*Ny] row-major, nu [Ny],
 * U [Ny][2][r][Nxi] (coupling columns: G_a on g rows, H_a on h rows), M
 * [Ny][r][2][Nxi] (moment functionals m_a), bc [Ny*2*Nxi] (1 = inflow row),
 * where r = 4 (Dv = 2) or 3.  Any output may be NULL. */
klst_status klst_host_tables(const klst_grid* grid, const klst_vel* vel, const klst_base* base,
                             double beta, double* Dx, double* nu, double* U, double* M,
                             uint8_t* bc);

/* Host-only: the selection of returned eigenpairs that klst_solve makes from
 * its k locked pairs, exposed for testing.  lam [2k] locked eigenvalues; G
 * [2 k^2] (or NULL) the overlaps <R conj(x_i), x_j> of the locked eigenvectors
 * (row-major, interleaved), R the xi_y reflection, and nrm2 [k] = ||x_i||^2.
 * With G, lambda_i counts as real when |G_ii| >= (1 - 1e-10) ||x_i||^2, locked
 * x_j as the conjugate partner of x_i when |G_ij| >= (1 - 1e-6) ||x_i|| ||x_j||
 * and |lambda_j - conj(lambda_i)| <= 1e-6 |lambda_i| (one to one, best
 * alignment first), and every other locked complex eigenvalue adds its partner
 * (conj(lambda_i), R conj(x_i)) as a candidate.  The min(nev, #) candidates
 * nearest sigma are returned (ties within 1e-12 relative: Im lambda > 0 first,
 * then locking order): out_lam [2 nev], out_src [nev] (the locked pair used),
 * out_mirrored [nev] (1: the partner of out_src), *nout the count.  Any output
 * array may be NULL.  Errors: EINVAL. */
klst_status klst_host_select_output(int k, const double* lam, const double* G, const double* nrm2,
                                    const double sigma[2], int nev, double* out_lam, int* out_src,
                                    int* out_mirrored, int* nout);

/* Host-only: continuum structure of a normal shock by the Gilbarg-Paolucci
 * equations (Sec. 2.1, eq. GB1DShockeqn): steady 1-D Navier-Stokes for a gas of
 * specific-heat ratio gamma, Prandtl number Pr (the paper sets 1 for its
 * comparisons with BGK) and viscosity mu ~ T^s_visc, upstream Mach number
 * mach > 1, lengths in upstream mean free paths
 * l_inf = (16/delta) mu_inf / (rho_inf sqrt(2 pi R T_inf)) (delta = 5: hard
 * spheres).  At the nz positions z (host, in l_inf, measured from the point of
 * steepest velocity gradient, positive downstream) it writes rho / rho_inf,
 * u / u_inf and T / T_inf (host arrays of nz), and *thickness (may be NULL)
 * receives Delta / l_inf of eq. ShockThickness.  Beyond the traced range the
 * end states are returned.  Errors: EINVAL (mach <= 1, gamma <= 1, Pr <= 0,
 * delta <= 0, non-finite input, null arrays with nz > 0). */
klst_status klst_gp_shock(double mach, double gamma, double Pr, double s_visc, double delta, int nz,
                          const double* z, double* rho, double* u, double* T, double* thickness);

/* Host-only: sorted complex Schur form of a small m x m complex matrix G
 * (row-major interleaved), G U = U T with |T_00| >= |T_11| >= ...; used by the
 * solver for its projected problems; exposed for testing.  U, T row-major. */
klst_status klst_host_sorted_schur(int m, const double* G, double* U, double* T);

#ifdef __cplusplus
}
#endif
#endif /* KLST_H */
