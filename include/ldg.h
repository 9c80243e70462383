/*
 * ldg.h -- C ABI of the MI355X line-DG library (libldg.so).
 *
 * Line-based discontinuous Galerkin discretisation of Persson, "A sparse and
 * high-order accurate line-based discontinuous Galerkin method for
 * unstructured meshes": the semi-discrete residual and its Jacobians on
 * curved quad/hex meshes, and the Newton-Krylov machinery of its Section 4
 * (split Jacobian-vector product, element-local line-pattern preconditioner,
 * preconditioned GMRES).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every call returns an ldg_status; no C++ exception crosses the ABI.  On
 *    failure ldg_last_error(ctx) returns a message (thread-unsafe, per ctx);
 *    ldg_last_error(NULL) returns the message of this thread's last failed
 *    call that takes no context (ldg_create, ldg_assign_switches).
 *  - Arrays named *_dev are device pointers owned by the caller (e.g. torch
 *    tensors on cuda:0), contiguous, float64, in the documented layout.  They
 *    must not alias unless a call says so.  Arrays named *_host are host
 *    pointers read only during the call.
 *  - Element e owns Np = (p+1)^D nodes; local node index i + (p+1) j
 *    [+ (p+1)^2 k], i fastest.  m = 1 (Poisson), D+2 (Euler / Navier-Stokes).
 *    Nodal fields are [E][m][Np]; the auxiliary gradient Q is [E][m][D][Np]
 *    (q_{c,d} = d u_c / d x_d).
 *  - Face 2n+s of an element is its face xi_n = s.  Its Nf = (p+1)^(D-1) face
 *    nodes are numbered by the direction-n reference lines that end on it (the
 *    other reference coordinates in increasing dimension order, lowest fastest).
 *  - All device work is ordered on the stream given to ldg_create.  Calls do
 *    not synchronise the host unless stated (ldg_newton_step and
 *    ldg_implicit_step do).
 *  - The context owns all internal device memory; it is allocated by
 *    ldg_create, grown by the first call that needs more (assembly, products,
 *    Newton and time steps), and released by ldg_destroy.
 */
#ifndef LDG_H
#define LDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ldg_ctx_s* ldg_ctx;

typedef enum {
  LDG_OK = 0,
  LDG_E_INVALID = -1,       /* bad argument value or null pointer               */
  LDG_E_SHAPE = -2,         /* inconsistent sizes / connectivity                */
  LDG_E_UNSUPPORTED = -3,   /* valid but not built (dimension, degree, option)  */
  LDG_E_HIP = -4,           /* a HIP runtime call failed                        */
  LDG_E_NOMEM = -5,         /* device allocation failed                         */
  LDG_E_NOT_ASSEMBLED = -6, /* jacvec / precond before ldg_jacobian_assemble    */
  LDG_E_NOT_CONVERGED = -7, /* linear solver did not reach the tolerance        */
  LDG_E_NONFINITE = -8      /* NaN / Inf produced                               */
} ldg_status;

typedef enum { LDG_POISSON = 0, LDG_EULER = 1, LDG_NS = 2 } ldg_equation;
typedef enum { LDG_F64 = 0, LDG_F32 = 1, LDG_BF16 = 2 } ldg_precision;
typedef enum { LDG_PRECOND_BILU0 = 0, LDG_PRECOND_BLOCK_LU = 1 } ldg_precond_kind;

/* Problem description (host memory, copied by ldg_create).
 * Section 2.1: the element nodes are the images x(X_ijk) of a tensor grid of
 * Gauss-Lobatto points (node_family 0) or equispaced points (1); the
 * isoparametric Q_p map through them defines G = grad_X x and J = det G.
 * Section 3: switch_plus[e][n] is S^+_n in {-1,+1} (S^-_n = -S^+_n); the two
 * elements of an interior face must carry opposite switch values on it. */
typedef struct {
  int32_t dim;            /* 2 or 3                                              */
  int32_t p;              /* polynomial degree, 1..4                             */
  int32_t equation;       /* ldg_equation                                        */
  int32_t node_family;    /* 0 = Gauss-Lobatto-Legendre, 1 = equispaced           */
  double gamma;           /* ratio of specific heats (Euler / NS)                */
  double mu;              /* dynamic viscosity (NS), constant                    */
  double prandtl;         /* Prandtl number (NS)                                 */
  double c11_interior;    /* LDG penalty C11 on interior faces (>= 0)            */
  double c11_dirichlet;   /* LDG penalty C11 on Dirichlet faces (> 0 if any)     */
  int64_t n_elem;         /* E >= 1                                              */
  const double* node_xyz_host;    /* [E][D][Np] physical node coordinates           */
  const int64_t* face_nbr_host;   /* [E][2D] neighbour element, or -(kind+1) for a boundary face:
                                     kind 0 Dirichlet (eqs. dirichlet1/2; for the inviscid flux
                                     Roe(g_D, u_in), the characteristic condition), 1 Neumann
                                     (eqs. neumann1/2 with C22 = 0: Fhat . n = |n| g_N,
                                     uhat = u_in), 2 slip wall (Euler / Navier-Stokes:
                                     Roe(u_m, u_in) with the mirror state u_m, normal momentum
                                     reversed; no viscous flux through the wall; uhat = u_in) */
  const int32_t* nbr_node_host;   /* [E][2D][Nf] local node index, inside the neighbour, of
                                     the node that coincides with each face node      */
  const int8_t* switch_plus_host; /* [E][D] S^+_n                                     */
} ldg_problem_desc;

/* Validate the description, copy mesh data to the device, build the 1-D
 * operators (Section 2.2: Gauss-Legendre rule with ceil((3p+1)/2) points,
 * mass matrix, its inverse folded into the lifting and test-derivative
 * operators).  hip_stream may be NULL (default stream).
 * Errors: LDG_E_INVALID / LDG_E_SHAPE (inconsistent connectivity, non-matching
 * switch signs, a slip wall with the Poisson equation; non-positive J is
 * reported later as LDG_E_NONFINITE), LDG_E_UNSUPPORTED (dim/p/equation or
 * boundary kind outside the built set). */
ldg_status ldg_create(const ldg_problem_desc* desc, void* hip_stream, ldg_ctx* out);

/* Section 3 (switch function, figure switchplt): a switch function for a mesh
 * with arbitrarily oriented elements, written to switch_plus_host [E][D]
 * (host memory, caller-owned), ready for ldg_problem_desc.switch_plus_host.
 * Host computation only (no device work, no context).  A chord enters an
 * element through a face of local direction n and leaves it through the other
 * face of direction n; one sign per chord makes the two elements of every
 * shared face carry opposite signs.  Chords are started in element order, then
 * local-direction order, with S^+ = +1 on the starting element, so the result
 * is unique (all +1 on a mesh whose elements are all aligned).
 * face_nbr_host [E][2D] and nbr_node_host [E][2D][Nf] as in ldg_problem_desc.
 * Errors: LDG_E_INVALID (dim, p, E, null pointers), LDG_E_SHAPE (a neighbour
 * out of range, or no face of the neighbour maps back to the face). */
ldg_status ldg_assign_switches(int32_t dim, int32_t p, int64_t n_elem, const int64_t* face_nbr_host,
                               const int32_t* nbr_node_host, int8_t* switch_plus_host);
void ldg_destroy(ldg_ctx ctx);

/* Source term S (eq. conslaw), added to R; S_dev [E][m][Np], copied.  NULL clears. */
ldg_status ldg_set_source(ldg_ctx ctx, const double* S_dev);
/* Dirichlet data g_D at boundary face nodes (eqs. dirichlet1/2); gD_dev
 * [E][2D][m][Nf] (only boundary faces are read), copied.  NULL = zero data. */
ldg_status ldg_set_dirichlet(ldg_ctx ctx, const double* gD_dev);

/* Neumann data g_N at boundary face nodes (eqs. neumann1/2: the prescribed
 * normal flux F . nhat, unit outward normal); gN_dev [E][2D][m][Nf] (only
 * Neumann faces are read), copied.  NULL = zero data. */
ldg_status ldg_set_neumann(ldg_ctx ctx, const double* gN_dev);

/* Q = D(U): the LDG gradient (eqs. splitdisc2, numfluxu1, semidisc2-2) with
 * the switch-selected traces; homogeneous != 0 uses g_D = 0 (then Q = K21 U).
 * U_dev [E][m][Np] -> Q_dev [E][m][D][Np]. */
ldg_status ldg_gradient(ldg_ctx ctx, const double* U_dev, double* Q_dev, int32_t homogeneous);

/* R = F(U) = -(1/J) sum_n r^(n) + S (eqs. galerkinscheme2, semidisc,
 * semidisc2-1, semidiscprimal), FP64.  Q_dev (may be NULL) receives D(U) and
 * is otherwise internal scratch.  U_dev [E][m][Np] -> R_dev [E][m][Np]. */
ldg_status ldg_residual(ldg_ctx ctx, const double* U_dev, double* R_dev, double* Q_dev);

/* Assemble K11 = dR/dU and K12 = dR/dQ (Section 4.1) in line-block form,
 * computed in FP64 and stored in storage_prec, then form the preconditioner
 * A~ = alpha I - gamma (K11 + K12 K21) restricted to the element-local line
 * pattern (Section 4.2) and factorise it by block ILU(0) in natural node
 * order (FP64 arithmetic for LDG_F64 storage, FP32 otherwise).  alpha is 1 for
 * an implicit time step ((alpha I - gamma A) dU = rhs, eq. dirkeqn with
 * gamma = alpha_dirk dt) and 0 for a steady solve.
 * U_dev [E][m][Np]. */
ldg_status ldg_jacobian_assemble(ldg_ctx ctx, const double* U_dev, double alpha, double gamma,
                                 int32_t storage_prec);

/* y = (alpha I - gamma A) x with the split product of eq. matvecsplit:
 * alpha x - gamma (K11 x + K12 (K21 x)), K21 x from the stored per-node K21
 * weights (FP64; an FP32 copy of them beside FP32 / BF16 storage), FP64
 * accumulation.  With exact_fp64 != 0, A x is the exact FP64 tangent of the
 * residual at the assembled state (forward-mode differentiation, FP64 K21
 * weights), independent of the stored precision.  x_dev, y_dev [E][m][Np],
 * must not alias.
 * Error: LDG_E_NOT_ASSEMBLED. */
ldg_status ldg_jacvec(ldg_ctx ctx, const double* x_dev, double* y_dev, int32_t exact_fp64);

/* Allocation-free variant of ldg_jacvec, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, result and errors as ldg_jacvec;
 * the intermediate w = K21 x goes to a static device array of
 * LDG_NOALLOC_SCRATCH_DOUBLES doubles (64 MiB, held by every GPU the library
 * runs on until the process ends) instead of context memory, and the call
 * performs no hipMalloc / hipFree.  It needs E m D Np <= LDG_NOALLOC_SCRATCH_DOUBLES
 * (e.g. the 16^3 p = 3 Navier-Stokes mesh, 3.9 M) and returns LDG_E_UNSUPPORTED
 * beyond.  All calls on one GPU share the array: calls that overlap on a GPU
 * (several streams or threads) race.  The context must have been assembled. */
#define LDG_NOALLOC_SCRATCH_DOUBLES (8 * 1024 * 1024)
ldg_status ldg_jacvec_noalloc(ldg_ctx ctx, const double* x_dev, double* y_dev, int32_t exact_fp64);

/* Preconditioner of Section 4.2: the block-Jacobi matrix A~ that keeps A only
 * on each element's line pattern (no K12 K21 fill, no inter-element
 * coupling), applied as z = P^{-1} r with its block ILU(0) factors (per
 * element, forward and backward block substitution in natural node order; the
 * paper factorises each block by a sparse direct LU and names ILU as an
 * improvement), plus the learned correction when the current assembly applies
 * one; or, when the assembly was made with LDG_PRECOND_BLOCK_LU, the exact LU
 * of each element block.  Linear in r.  r_dev, z_dev [E][m][Np], may not alias.
 * Error: LDG_E_NOT_ASSEMBLED. */
ldg_status ldg_precond_apply(ldg_ctx ctx, const double* r_dev, double* z_dev);

/* Section 4.2: how the element blocks of A~ are factorised from the next
 * ldg_jacobian_assemble on (also inside ldg_newton_step / ldg_implicit_step).
 * LDG_PRECOND_BILU0 (default): block ILU(0), storage precision as assembled.
 * LDG_PRECOND_BLOCK_LU: the paper's exact factorisation of each block -- A~_e
 * (formed as for BILU(0)) expanded to a dense NR x NR matrix, NR = Np m,
 * factorised in FP64 without pivoting, E NR^2 doubles of device memory; no
 * learned correction with it.  Changing the kind invalidates the assembly.
 * Errors: LDG_E_INVALID (kind), LDG_E_UNSUPPORTED (block LU with Np m > 768). */
ldg_status ldg_set_preconditioner(ldg_ctx ctx, int32_t kind);

/* Section 4.1, eqs. ldgflux1/ldgflux2 and neumann1/neumann2: the coefficient
 * C22 >= 0 of the jump of the normal viscous flux in the trace of u, used by
 * ldg_coupled_solve (Poisson only).  On an interior face the trace gains
 * C22 (F(q_in) - F(q_out)) . nhat_in with nhat_in the unit normal out of the
 * element whose equation is being formed; on a Neumann face
 * C22 (F(q_in) . nhat - g_N); none on Dirichlet faces.  The reduced scheme of
 * ldg_gradient / ldg_residual / ldg_newton_step (C22 = 0) is unaffected.
 * Errors: LDG_E_INVALID (negative or non-finite), LDG_E_UNSUPPORTED (C22 != 0
 * for an equation other than Poisson). */
ldg_status ldg_set_c22(ldg_ctx ctx, double c22);

/* Section 4.1: steady solution of the linear problem in the coupled unknowns
 * (U, Q), F(U, Q) = [-R(U, Q); Q - G(U, Q)] = 0 with G the gradient whose
 * trace carries the C22 term of ldg_set_c22, by flexible GMRES(restart) from
 * zero in FP64 (the paper uses a sparse direct solver here).  Preconditioner:
 * an approximate inverse of the C22 = 0 Jacobian [[-K11, -K12], [-K21, I]] --
 * U from an inner GMRES(restart) solve of the reduced system
 * -(K11 + K12 K21) U = r_U + K12 r_Q to inner_rtol (at most restart
 * iterations, with the element-block preconditioner of the kind set by
 * ldg_set_preconditioner), then Q = r_Q + K21 U.  Assembles K11, K12 and the
 * preconditioner with alpha = 0, gamma = 1 in FP64 (replacing any previous
 * assembly).  U_dev [E][m][Np] and Q_dev [E][m][D][Np] (out).  Stops when
 * ||b - A x|| <= rtol ||b|| (the true residual) or after max_iters outer
 * iterations; iters_out, inner_iters_out (total inner iterations) and
 * relres_out (any may be NULL) report them.  Work memory
 * ((2 restart + 6)(ndof + nq) + ndof doubles, and the reduced system's Krylov
 * space) is allocated by the first call.  Synchronises the stream.
 * Errors: LDG_E_INVALID (rtol <= 0, inner_rtol outside (0, 1), restart outside
 * 1..120, max_iters < 1, null or aliased U/Q), LDG_E_UNSUPPORTED (not
 * Poisson), LDG_E_NOT_CONVERGED (U, Q then hold the last iterate),
 * LDG_E_NONFINITE. */
ldg_status ldg_coupled_solve(ldg_ctx ctx, double* U_dev, double* Q_dev, double rtol, double inner_rtol,
                             int32_t restart, int32_t max_iters, int32_t* iters_out, int32_t* inner_iters_out,
                             double* relres_out);

/* Copy the assembled operators out in FP64, line-block layout:
 * K11_dev [E][Np][Dp+1+2D][m][m], K12_dev [E][Np][Dp+1+D][m][m*D] (columns
 * (c', d) like Q), F_dev [E][Np][Dp+1][m][m] the BILU(0) factors (strictly
 * lower slots hold L, the diagonal slot holds the INVERSE of the U diagonal
 * block, the rest U).  Slot order for a node with reference indices (i_0..):
 * slots 0..p the direction-0 line nodes (t, i_1, ..); then for n >= 1 the p
 * other nodes of its direction-n line in increasing t; then neighbour slots:
 * K11 face 2n+s, K12 the side of direction n whose switch is +1.  Any pointer
 * may be NULL.  Error: LDG_E_NOT_ASSEMBLED. */
ldg_status ldg_export_operators(ldg_ctx ctx, double* K11_dev, double* K12_dev, double* F_dev);

typedef struct {
  int32_t restart;        /* GMRES restart length (50)                          */
  int32_t max_iters;      /* total inner iterations allowed per solve            */
  int32_t max_refine;     /* outer FP64 refinement sweeps (low-precision storage) */
  int32_t storage_prec;   /* ldg_precision of K11/K12 and the factors             */
  double rtol;            /* ||b - (alpha I - gamma A) dU|| <= rtol ||b||  (1e-8)  */
  double inner_rtol;      /* GMRES tolerance inside a refinement sweep            */
  int32_t use_learned;    /* apply the learned correction if loaded              */
  int32_t reassemble;     /* 0 reuses the last assembly (same alpha, gamma)      */
} ldg_solver_opts;

typedef struct {
  int32_t gmres_iters;    /* total inner GMRES iterations                        */
  int32_t refine_steps;   /* outer refinement sweeps                             */
  int32_t fallback_used;  /* 1 if the learned correction was switched off        */
  int32_t converged;
  double lin_relres;      /* final ||b - (alpha I - gamma A) dU|| / ||b||, exact FP64 operator */
  double newton_res_before, newton_res_after; /* ||G(U)||_2 before / after        */
  double t_resid_ms, t_assemble_ms, t_solve_ms, t_total_ms;
  /* stream-timed (HIP events) kernels inside the linear solve: the stored
   * split product y = alpha x - gamma (K11 x + K12 w), the matrix-free
   * w = K21 x, and the block ILU(0) apply; totals over the step and counts */
  double t_jacvec_ms, t_k21_ms, t_precond_ms;
  int32_t n_jacvec, n_k21, n_precond;
} ldg_solver_report;

/* One Newton step of Section 4.2 (eqs. dirkeqn, fulldiscprimal) on
 * G(U) = alpha (U - Ucomb) - gamma R(U): solve (alpha I - gamma A) dU = -G(U)
 * with A = K11 + K12 K21, by right-preconditioned GMRES(restart) with the
 * split product (eq. matvecsplit) and the preconditioner of
 * ldg_precond_apply, then U += dU.  The paper's DIRK stage has alpha = 1,
 * gamma = alpha_dirk dt; BDF2: Ucomb = (4U^n - U^{n-1})/3, gamma = 2 dt/3;
 * steady: alpha = 0, gamma = 1.  With storage_prec != LDG_F64 the solve is
 * wrapped in FP64 iterative refinement using the exact tangent product.
 * The learned correction, when used, is judged by the outcome: if its solve
 * misses rtol, or the step does not lower ||G||, the step is repeated with the
 * plain BILU(0) factors and report->fallback_used is set.
 * U_dev (in/out) [E][m][Np]; Ucomb_dev may be NULL (zero), must not alias U.
 * Synchronises the stream.  On LDG_E_NOT_CONVERGED / LDG_E_NONFINITE, U is
 * unchanged and report says why. */
ldg_status ldg_newton_step(ldg_ctx ctx, double* U_dev, const double* Ucomb_dev, double alpha,
                           double gamma, const ldg_solver_opts* opts, ldg_solver_report* report);

/* Implicit time steps (Section 4.1) driven by Newton iterations of
 * ldg_newton_step's kind on each stage equation Y - Ucomb - gamma F(Y) = 0:
 *  LDG_DIRK3          Alexander's L-stable three-stage, third-order DIRK
 *                     (eqs. dirk1, dirk2) with alpha = 0.435866521508459,
 *                     tau_2 = (1 + alpha)/2, b_1 = -(6 alpha^2 - 16 alpha + 1)/4,
 *                     b_2 = (6 alpha^2 - 20 alpha + 5)/4; every stage has
 *                     gamma = alpha dt, so one Jacobian serves all stages;
 *                     U^{n+1} = Y_3 (the last tableau row equals b);
 *  LDG_BDF2           Ucomb = (4U^n - U^{n-1})/3, gamma = 2 dt/3;
 *  LDG_BACKWARD_EULER Ucomb = U^n, gamma = dt (pseudo-time to a steady state).
 * Jacobian re-use (Section 4.3): with reuse != 0 the assembled K11, K12 and
 * preconditioner are kept across Newton iterations, stages and steps as long
 * as gamma and the storage precision stay the same, and re-assembled at the
 * current iterate when a stage has taken reassemble_after Newton iterations
 * since the last assembly (the paper uses 15, with 5 GMRES iterations per
 * Newton iteration).  A stage has converged when
 * ||G|| <= max(newton_rtol ||G(Y_start)||, newton_atol); with both zero every
 * stage runs exactly max_newton Newton iterations and accepts the result (a
 * linearly implicit scheme when max_newton = 1).
 * With gmres_per_newton > 0 every Newton iteration runs that many GMRES
 * iterations on the stored operator (no refinement: the FP64 Newton residual
 * corrects the low-precision solve); with 0 each linear solve runs to
 * lin_opts->rtol as in ldg_newton_step.  lin_opts->reassemble is ignored.
 * U_dev (in/out) [E][m][Np].  Uprev_dev: BDF2 history U^{n-1} (in), replaced by
 * U^n on success; NULL starts BDF2 with U^{n-1} = U^n; unused otherwise.
 * Work arrays are allocated by the first call.  Synchronises the stream.
 * On failure U (and Uprev) are unchanged and the report says where it stopped.
 * Errors: LDG_E_INVALID, LDG_E_NOT_CONVERGED, LDG_E_NONFINITE. */
typedef enum { LDG_BDF2 = 0, LDG_DIRK3 = 1, LDG_BACKWARD_EULER = 2 } ldg_scheme;

typedef struct {
  int32_t scheme;           /* ldg_scheme                                          */
  int32_t max_newton;       /* Newton iterations allowed per stage (>= 1)          */
  double newton_rtol;       /* stage tolerance relative to ||G|| at its start      */
  double newton_atol;       /* absolute stage tolerance                            */
  int32_t gmres_per_newton; /* fixed GMRES iterations per Newton iteration, 0 = to rtol */
  int32_t reuse;            /* keep the assembled Jacobian across iterations/stages/steps */
  int32_t reassemble_after; /* with reuse: re-assemble after this many Newton iterations of a stage */
} ldg_step_opts;

typedef struct {
  int32_t stages;           /* stages attempted                                   */
  int32_t newton_iters;     /* Newton iterations over all stages                  */
  int32_t max_stage_newton; /* most Newton iterations in one stage                */
  int32_t assemblies;       /* Jacobian assemblies during the step                */
  int32_t gmres_iters;      /* GMRES iterations over the step                     */
  int32_t converged;
  int32_t fallback_used;    /* the learned correction was rejected at least once   */
  double newton_res_first;  /* ||G|| at the start of the first stage              */
  double newton_res_final;  /* ||G|| after the last Newton iteration              */
  double lin_relres_max;    /* largest relative linear residual of a Newton solve  */
  double t_assemble_ms;     /* stream-timed assemblies, summed                    */
  double t_solve_ms;        /* stream-timed linear solves, summed                 */
  double t_ms;              /* host wall time of the step                         */
} ldg_step_report;

ldg_status ldg_implicit_step(ldg_ctx ctx, double* U_dev, double* Uprev_dev, double dt, const ldg_step_opts* opts,
                             const ldg_solver_opts* lin_opts, ldg_step_report* report);

/* Classical four-stage Runge-Kutta on dU/dt = R(U) (Section 4.1), n_steps
 * steps of size dt, U_dev in/out [E][m][Np]. */
ldg_status ldg_rk4(ldg_ctx ctx, double* U_dev, double dt, int32_t n_steps);

/* ------------------------------------------------------------------------
 * Learned correction of the preconditioner (an addition beyond the paper).
 *
 * A small network maps, per element, the m x m diagonal blocks D_b of A~ and
 * the element's Newton residual to Np blocks Y_b; with C_b = Y_b D_b^{-1} the
 * corrected preconditioner is  z = z0 + C (r - A~ z0),  z0 = ILU(0)^{-1} r,
 * element by element.  C is evaluated once per assembly, so z is linear in r.
 * Features of an element (n_in = Np m^2 + Np m floats): D_b / sigma with
 * sigma = max |entries of all D_b| (index (b m + i) m + j), then
 * G / max|G| (index Np m^2 + b m + i) with G = -gamma R(U) at the assembly
 * state (zero if G = 0).  Network: H1 = tanh(X W1 + b1), H2 = tanh(H1 W2 + b2),
 * Y = H2 W3 + b3.  Parameters (FP32, flat): W1 [n_in][h], b1 [h], W2 [h][h],
 * b2 [h], W3 [h][n_out], b3 [n_out], n_out = Np m^2.  If any C entry is not
 * finite the assembly falls back to plain ILU(0) and reports it.
 * ---------------------------------------------------------------------- */
typedef struct ldg_net_s* ldg_net;

/* Training samples (device, FP32), one row per sampled element and K probes v:
 *  X [n][n_in] features;  A [n][Np][Dp+1][m][m] the rows of A~ on the line
 *  pattern (slot order as in ldg_export_operators);  S [n][K][Np][m] the
 *  defect s = v - A~ ILU^{-1} v and T [n][K][Np][m] t = D_b^{-1} s_b, both
 *  divided by the element norm of v (zero if that norm is zero).
 * Loss:  L = 1/(n K) sum ||s - A~ (Y t)||^2  (Y_b applied node by node). */
typedef struct {
  int64_t n;
  int32_t n_probe;
  const float* X_dev;
  const float* A_dev;
  const float* S_dev;
  const float* T_dev;
} ldg_sample_batch;

/* Create a network for elements of dimension dim, degree p and m components,
 * hidden width `hidden`.  W1, W2 are Glorot-uniform from a splitmix64 stream
 * seeded by `seed`; W3 and every bias start at zero (so the correction starts
 * as plain ILU(0)).  Adam state starts at zero.
 * Errors: LDG_E_INVALID, LDG_E_NOMEM. */
ldg_status ldg_net_create(int32_t dim, int32_t p, int32_t m, int32_t hidden, uint64_t seed, void* hip_stream,
                          ldg_net* out);
void ldg_net_destroy(ldg_net net);
/* Number of parameters, or -1 for NULL. */
int64_t ldg_net_num_params(ldg_net net);
/* Copy all parameters in (resets the Adam state) or out, flat FP32 device arrays. */
ldg_status ldg_net_set_params(ldg_net net, const float* params_dev);
ldg_status ldg_net_get_params(ldg_net net, float* params_dev);
/* Y [n][n_out] = network(X [n][n_in]); prec LDG_F32 (FP32 operands) or
 * LDG_BF16 (features, weights and hidden activations rounded to BF16, FP32
 * accumulation), both on matrix cores. */
ldg_status ldg_net_forward(ldg_net net, const float* X_dev, int64_t n, int32_t prec, float* Y_dev);
/* Loss of a batch and its gradient with respect to every parameter (kept for
 * ldg_net_adam_step, and copied to grad_dev [n_params] when not NULL); *loss
 * (host) receives L.  In LDG_BF16 mode the operands of every product are
 * BF16 (activation gradients too), accumulation and the loss are FP32. */
ldg_status ldg_net_loss_grad(ldg_net net, const ldg_sample_batch* batch, int32_t prec, float* grad_dev,
                             double* loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias corrected) with the
 * gradient of the last ldg_net_loss_grad; refreshes the BF16 weights. */
ldg_status ldg_net_adam_step(ldg_net net, double lr);
const char* ldg_net_last_error(ldg_net net);

/* Attach a network to a context (NULL detaches); it must have been created
 * for the context's dim, p and m.  infer_prec (LDG_F32 / LDG_BF16) is the
 * precision of its evaluation at assembly.  Attaching enables the correction
 * for ldg_jacobian_assemble; ldg_newton_step enables it per call from
 * opts.use_learned.  Errors: LDG_E_SHAPE, LDG_E_UNSUPPORTED (element too
 * large for the training kernel: Np > 128). */
ldg_status ldg_learned_attach(ldg_ctx ctx, ldg_net net, int32_t infer_prec);
/* on != 0: keep A~, the features and D^{-1} at every assembly so that
 * ldg_learned_samples can read them (also without a network). */
ldg_status ldg_learned_collect(ldg_ctx ctx, int32_t on);
/* 1 if the current assembly applies the correction, 0 otherwise. */
int32_t ldg_learned_active(ldg_ctx ctx);
/* Training samples from the current assembly for the elements
 * elems_host[0..n): probes V_dev [K][E][m][Np] (device, FP64), or NULL to use
 * the first K Arnoldi vectors of the last GMRES cycle.  Outputs as in
 * ldg_sample_batch.  Errors: LDG_E_NOT_ASSEMBLED (no assembly kept A~),
 * LDG_E_INVALID (element out of range, K larger than the Arnoldi vectors
 * available). */
ldg_status ldg_learned_samples(ldg_ctx ctx, const int64_t* elems_host, int64_t n, const double* V_dev, int32_t K,
                               float* X_dev, float* A_dev, float* S_dev, float* T_dev);

const char* ldg_status_string(ldg_status s);
const char* ldg_last_error(ldg_ctx ctx);
/* Number of degrees of freedom E*m*Np, or -1 for a NULL context. */
int64_t ldg_num_dofs(ldg_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif /* LDG_H */
