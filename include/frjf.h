/*
 * frjf.h -- C ABI of the MI355X (gfx950) Jacobian-free implicit solver for
 * flux reconstruction (FR/CPR) discretisations of the 2D Euler and
 * Navier-Stokes equations.
 *
 * Method: Wang & Yu, "A comparative study of implicit Jacobian-free
 * Rosenbrock-Wanner, ESDIRK and BDF methods for unsteady flow simulation with
 * high-order flux reconstruction formulations", arXiv:1904.04825.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Array arguments named d_* are DEVICE pointers (HBM of the current
 *   HIP device); h_* are host pointers.  The caller allocates and owns every
 *   buffer, including the workspace whose size fr_workspace_bytes() reports
 *   and the element-Jacobi store.  The library never allocates device memory.
 *   All device arrays must be 256-byte aligned (torch allocations are).
 * State layout.  A solution-shaped vector holds 4 * nel * Np doubles as
 *   U[v][e][k]: v in (rho, rho*u, rho*v, E); e = ey*nx + ex; k = b*(P+1) + a,
 *   where a indexes the Gauss point along the element's xi (i) direction and
 *   b along eta (j).  Np = (P+1)^2, ndof = 4 * nel * Np.
 * Mesh.  Structured, doubly periodic, nx * ny bilinear quadrilaterals given
 *   by a vertex array d_nodes[(ny+1)][(nx+1)][2] (x, y); element (ex, ey) has
 *   corners (ex,ey), (ex+1,ey), (ex,ey+1), (ex+1,ey+1), counter-clockwise
 *   orientation (positive |J|).  Column nx and row ny are the periodic copies
 *   of column 0 and row 0 shifted by the period.  nx, ny >= 2.
 * Streams.  fr_stream is a hipStream_t (NULL = the null stream).  Every call
 *   enqueues its work on that stream.  Functions that return statistics
 *   (fr_gmres_solve and the *_step functions) synchronise the stream before
 *   returning; the others return as soon as the work is enqueued.
 * Errors.  Negative status = caller or system error: nothing was enqueued and
 *   outputs are untouched; fr_last_error() returns a message (thread-local).
 *   Positive status = numerical outcome (statistics are filled).  The *_step
 *   functions are transactional: on any status other than FR_OK the state
 *   arrays they update are left unchanged.
 * Threads.  A fr_disc may be used from one host thread at a time.
 */
#ifndef FRJF_H
#define FRJF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* fr_stream; /* hipStream_t */

typedef enum {
  FR_OK = 0,
  FR_EINVAL = -1,  /* invalid argument (null pointer, bad size, bad enum) */
  FR_EHIP = -2,    /* a HIP runtime call failed */
  FR_ESIZE = -3,   /* workspace or store too small */
  FR_NOTCONV = 1,  /* iteration limit reached before the tolerance */
  FR_BREAKDOWN = 2,/* GMRES: zero Krylov direction with a nonzero residual */
  FR_ENAN = 3,     /* a NaN or Inf appeared in a norm */
  FR_REJECTED = 4  /* PTC: too many rejected pseudo-steps */
} fr_status;

enum { FR_EULER = 0, FR_NS_BR1 = 1 };            /* physics (FR_NS_BR1: Navier-Stokes, viscous scheme below) */
enum { FR_BR1 = 0, FR_BR2 = 1 };                 /* common gradient of the viscous flux */
enum { FR_BC_PERIODIC = 0, FR_BC_WALL = 1, FR_BC_FARFIELD = 2 };  /* eta-boundaries */
enum { FR_RUSANOV = 0, FR_ROE = 1 };             /* inviscid common flux */
enum { FR_F64 = 0, FR_F32 = 1 };                 /* element-Jacobi precision */
enum { FR_EPS_ABS = 0, FR_EPS_RMS = 1 };         /* JF perturbation rule */
enum { FR_ROW2 = 2, FR_ROW3 = 3, FR_ROW4 = 4 };  /* ROW schemes */
enum { FR_ESDIRK2 = 2, FR_ESDIRK3 = 3, FR_ESDIRK4 = 4 };
enum { FR_WS_RESIDUAL = 0, FR_WS_MATVEC = 1, FR_WS_GMRES = 2, FR_WS_STEP = 3 };

typedef struct fr_disc fr_disc; /* opaque: host metadata + borrowed device pointers */

typedef struct {
  int nx, ny;       /* elements per direction, >= 2 */
  int p;            /* polynomial degree: 2 .. 6 (Euler), 2 .. 4 (FR_NS_BR1) */
  int physics;      /* FR_EULER or FR_NS_BR1 */
  int flux;         /* FR_RUSANOV or FR_ROE */
  double gamma;     /* ratio of specific heats (Section 2: 1.4) */
  double rgas;      /* gas constant R, p = rho R T */
  double mu;        /* dynamic viscosity (FR_NS_BR1), constant */
  double prandtl;   /* Prandtl number (FR_NS_BR1), kappa = mu Cp / Pr */
  const double* d_nodes; /* device vertex array, see above; borrowed, must outlive the disc */
  /* Navier-Stokes only; all zero = BR1 on a doubly periodic mesh. */
  int viscous;      /* FR_BR1 (mean of the corrected gradients), or FR_BR2: each side's raw gradient
                       plus its face lifting c_P (q^com - q) n |grad xi| with c_P = (P+1)(P+2)/2
                       (Section 3, eq. com_grad_q and the lifting after it) */
  int bc_south;     /* FR_BC_* of the eta = -1 side of element row 0 */
  int bc_north;     /* FR_BC_* of the eta = +1 side of element row ny-1.  With either one not
                       periodic, vertex row ny is the outer boundary, not a copy of row 0; xi stays
                       periodic (column nx repeats column 0, e.g. the seam of an O-grid).
                       FR_BC_WALL: no-slip adiabatic wall (outside trace (rho, -rho u, -rho v,
                       E - rho|u|^2), pressure flux, viscous flux at zero velocity without heat flux);
                       FR_BC_FARFIELD: outside trace q_far through the Riemann solver. */
  double q_far[4];  /* far-field conservative state (rho, rho u, rho v, E) for FR_BC_FARFIELD */
} fr_disc_desc;

/* Create / destroy a discretisation handle.  Computes the Gauss points,
 * Lagrange extrapolation rows, differentiation matrix and Radau correction
 * derivatives of degree p (Section 3).  Returns FR_EINVAL for p outside 2..6
 * (2..4 for FR_NS_BR1), nx or ny < 2, physics/flux out of range or a null d_nodes, and for
 * a viscous scheme or boundary out of range, a non-periodic side with FR_EULER, or a
 * far-field state with rho <= 0 or p <= 0. */
fr_status fr_disc_create(const fr_disc_desc* desc, fr_disc** out);
void fr_disc_destroy(fr_disc* disc);

/* Number of doubles in a solution-shaped vector: 4 * nel * (p+1)^2. */
size_t fr_ndof(const fr_disc* disc);

/* Workspace bytes needed by the entry points of class `what` (FR_WS_*) with
 * GMRES restart m (ignored for FR_WS_RESIDUAL / FR_WS_MATVEC) and
 * element-Jacobi precision `precision` (FR_WS_STEP only: the step functions
 * keep their own element-Jacobi store in the workspace). */
size_t fr_workspace_bytes(const fr_disc* disc, int what, int m, int precision);

/* Bytes of an element-Jacobi store of the given precision:
 * nel * (4 Np)^2 * sizeof(double or float). */
size_t fr_ejacobi_bytes(const fr_disc* disc, int precision);

/* Physical coordinates of the solution points: d_xy[2][nel][Np] (x then y). */
fr_status fr_solution_points(const fr_disc* disc, double* d_xy, fr_stream stream);

/* Semi-discrete right-hand side R(q) of dq/dt = R(q) (Section 4, eq.
 * simplified_ode): the FR residual of Section 3 -- interpolated transformed
 * fluxes F = |J|(f xi_x + g xi_y), G = |J|(f eta_x + g eta_y) (eq.
 * trans_detail), common interface fluxes scaled by |J||grad xi| (eq.
 * norm_num_f; Rusanov or Roe, eq. invis_com), Radau correction and
 * R = -(1/|J|)(dF~/dxi + dG~/deta) (eq. discrete_ns).  For FR_NS_BR1 the
 * viscous flux of Section 2 with the BR1 common gradient is included.
 * d_U, d_R: ndof doubles (may not alias).  d_work: fr_workspace_bytes(
 * FR_WS_RESIDUAL) bytes (may be NULL when that is 0). */
fr_status fr_residual(const fr_disc* disc, const double* d_U, double* d_R, void* d_work,
                      fr_stream stream);

/* Jacobian-free product (Section 4.5):
 *   d_Av = shift * v - [R(U + e v) - R0] / e,
 * e = eps for FR_EPS_ABS (the paper's rule, eps = 1e-8) or
 * e = eps / rms(v), rms(v) = ||v||_2 / sqrt(ndof), for FR_EPS_RMS.
 * v = 0 gives Av = 0.  d_R0 must be R(U).  d_work: FR_WS_MATVEC bytes. */
fr_status fr_jf_matvec(const fr_disc* disc, const double* d_U, const double* d_R0,
                       const double* d_v, double shift, double eps, int eps_mode,
                       double* d_Av, void* d_work, fr_stream stream);

/* The same product for callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid allocation): no workspace
 * argument and no allocation.  Its scratch (the RMS norm's partial sums, and for
 * FR_NS_BR1 the gradient traces) is a static 4 MiB device array per GPU, held until
 * the process ends.  Returns FR_ESIZE, with the sizes in fr_last_error(), when the
 * mesh's BR1 traces (256 (P+1) bytes per element) exceed it.  Calls on one GPU share
 * that array: calls that overlap in time on one GPU (several streams or threads) race
 * and must be serialised by the caller.  Results are those of fr_jf_matvec. */
fr_status fr_jf_matvec_noalloc(const fr_disc* disc, const double* d_U, const double* d_R0,
                               const double* d_v, double shift, double eps, int eps_mode,
                               double* d_Av, fr_stream stream);

/* Element-Jacobi preconditioner store (Section 4.5: the diagonal element
 * blocks of the Jacobian).  d_factors: caller-allocated, fr_ejacobi_bytes(
 * precision) bytes; after fr_ejacobi_factor it holds, per element, the
 * explicit inverse of P_e = shift I - dR_e/dq_e, column-major, in
 * `precision`. */
struct fr_pmg;
typedef struct {
  void* d_factors;
  int precision; /* FR_F64 or FR_F32 */
  double shift;  /* set by fr_ejacobi_factor */
  const struct fr_pmg* mg;  /* FR_PC_PMG: the coarse level (fr_pmg_factor), else NULL */
} fr_ejacobi;

/* Assemble the raw blocks P_e = shift I - dR_e/dq_e by one-sided finite
 * differences (column j = (v,k) perturbs q[v][e][k] by 1e-8 max(1,|q|) with
 * every other entry of the state held fixed) into d_blocks: nel * Nb * Nb
 * doubles, Nb = 4 Np, block e column-major: entry (row i, col j) at
 * e*Nb*Nb + j*Nb + i, with row/col index v*Np + k.
 * d_work: FR_WS_RESIDUAL bytes (needed for FR_NS_BR1: the neighbours' corrected
 * gradients enter each block through the shared faces' common state; may be
 * NULL for FR_EULER). */
fr_status fr_ejacobi_assemble(const fr_disc* disc, const double* d_U, double shift,
                              double* d_blocks, void* d_work, fr_stream stream);

/* Assemble the blocks at state d_U and replace each by its inverse (Gauss-
 * Jordan elimination with partial pivoting), in pc->precision (FR_F32:
 * assembled in FP64, rounded to FP32, inverted in FP32).  Sets pc->shift.
 * A zero pivot gives Inf/NaN entries, which fr_gmres_solve reports as
 * FR_ENAN.  d_work as for fr_ejacobi_assemble. */
fr_status fr_ejacobi_factor(const fr_disc* disc, const double* d_U, double shift, fr_ejacobi* pc,
                            void* d_work, fr_stream stream);

/* Invert caller-provided FP64 blocks (layout as fr_ejacobi_assemble) into pc
 * (rounded to FP32 first when pc->precision == FR_F32). */
fr_status fr_ejacobi_factor_blocks(const fr_disc* disc, const double* d_blocks, fr_ejacobi* pc,
                                   fr_stream stream);

/* z = P_e^{-1} r for every element (the preconditioner application).
 * d_r, d_z: ndof doubles (may not alias).  FP32 stores convert r to FP32 and
 * accumulate in FP32; z is returned in FP64. */
fr_status fr_ejacobi_solve(const fr_disc* disc, const fr_ejacobi* pc, const double* d_r, double* d_z,
                           fr_stream stream);

/* z = M^{-1} r for the LU-SGS preconditioner M = (D + L) D^{-1} (D + U) at state d_U
 * (d_R0 = R(d_U)) with shift `shift` (FR_PC_LUSGS above): D^{-1} from pc (as left by
 * fr_ejacobi_factor at the same U and shift), L and U through Jacobian-free products
 * with eps / eps_mode as in fr_jf_matvec.  d_r, d_z: ndof doubles (may not alias).
 * d_work: fr_workspace_bytes(FR_WS_GMRES, m = 1) bytes.  FR_EINVAL for Navier-Stokes or
 * odd nx / ny. */
fr_status fr_lusgs_apply(const fr_disc* disc, const fr_ejacobi* pc, const double* d_U, const double* d_R0,
                         double shift, double eps, int eps_mode, const double* d_r, double* d_z, void* d_work,
                         fr_stream stream);

/* GMRES options and statistics. */
typedef struct {
  int m;            /* restart length (Section 4.5; the paper uses 60) */
  int max_iters;    /* total Arnoldi iterations; <= 0 means 50*m */
  double rtol;      /* stop when ||b - A x|| <= rtol * r_ref */
  double ref_norm;  /* r_ref; <= 0 means ||b - A x0|| (Section 5.1: relative to the first residual) */
  double eps;       /* JF perturbation, default 1e-8 */
  int eps_mode;     /* FR_EPS_RMS or FR_EPS_ABS */
  int precond;      /* FR_PC_EJACOBI (the paper's element-Jacobi), FR_PC_LUSGS or FR_PC_PMG
                       (fr_gmres_solve only: the coarse level comes with the pc) */
} fr_gmres_opts;

/* Preconditioners of the linear solves (Section 4.5 names matrix-free LU-SGS as the
 * low-storage alternative to element-Jacobi; the paper's results use element-Jacobi).
 * FR_PC_LUSGS: symmetric block Gauss-Seidel over the two checkerboard colours
 * (ex + ey even / odd; Euler meshes with even nx and ny), the element blocks of the
 * fr_ejacobi store as its diagonal and the couplings between colours applied through
 * Jacobian-free products (two per application, counted in residual_evals). */
enum { FR_PC_EJACOBI = 0, FR_PC_LUSGS = 1, FR_PC_PMG = 2 };

/* p-multigrid (FR_PC_PMG; Section 4.5 names it beside element-Jacobi): a coarse
 * discretisation of the same mesh at degree pc < p (its own handle, Euler, same flux)
 * with its own residual and element blocks, and a V-cycle preconditioner:
 *   z = D^{-1} r, nu1 - 1 more sweeps z += D^{-1}(r - A z);
 *   rc = Pi (r - A z), zc = Dc^{-1} rc, nc - 1 sweeps zc += Dc^{-1}(rc - Ac zc);
 *   z += I zc; nu2 sweeps z += D^{-1}(r - A z);
 * Pi the L2 projection onto degree pc and I the interpolation of the coarse polynomial
 * at the fine points (per element and variable, tensor products of 1D operators), A and
 * Ac the Jacobian-free products of the two levels (the coarse one at Uc = Pi U).
 * Caller-allocated buffers; set by fr_pmg_factor. */
typedef struct fr_pmg {
  const fr_disc* coarse;
  fr_ejacobi coarse_pc;  /* fr_ejacobi_bytes(coarse, precision) bytes at d_factors */
  double* d_Uc;          /* coarse ndof: Pi U */
  double* d_R0c;         /* coarse ndof: R_c(Uc) */
  double* d_work_c;      /* 4 coarse ndof + 32 doubles */
  int nu1, nu2, nc;      /* smoothing sweeps: nu1 >= 1, nu2 >= 0, nc >= 1 */
} fr_pmg;

/* Fine element-Jacobi at (d_U, shift) into pc (as fr_ejacobi_factor), Uc = Pi U,
 * R_c(Uc) and the coarse element-Jacobi at (Uc, shift) into mg->coarse_pc; sets
 * pc->mg = mg.  d_work: FR_WS_RESIDUAL bytes of the fine disc.  FR_EINVAL when the
 * levels do not match (mesh, flux, physics Euler, pc < p). */
fr_status fr_pmg_factor(const fr_disc* fine, const double* d_U, double shift, fr_ejacobi* pc, fr_pmg* mg,
                        void* d_work, fr_stream stream);

/* z = M^{-1} r for the p-multigrid preconditioner of pc (pc->mg set by fr_pmg_factor at
 * d_U with d_R0 = R(d_U)).  d_work: fr_workspace_bytes(FR_WS_GMRES, m = 1) bytes of the
 * fine disc.  r and z may not alias. */
fr_status fr_pmg_apply(const fr_disc* fine, const fr_ejacobi* pc, const double* d_U, const double* d_R0,
                       double shift, double eps, int eps_mode, const double* d_r, double* d_z, void* d_work,
                       fr_stream stream);

typedef struct {
  int iters;         /* Arnoldi iterations */
  int restarts;      /* completed cycles that did not converge */
  int converged;     /* 1 if ||r|| <= rtol * r_ref */
  double r_ref;      /* reference norm used */
  double r_final;    /* least-squares residual estimate (true residual after a restart) */
  long residual_evals; /* residual evaluations (one per JF product) */
} fr_gmres_stats;

/* Solve (shift I - dR/dq(U)) x = b (Section 4.5, eq. for A = D - dR/dq with
 * D = shift I) by restarted flexible GMRES(m), right-preconditioned by the
 * element-Jacobi store pc (which must have been factored with the same
 * shift), with the Jacobian-free product about (U, R0 = R(U)).
 * d_x: in = initial guess x0, out = solution.  d_work: FR_WS_GMRES bytes for
 * opts->m.  Returns FR_OK, FR_NOTCONV, FR_BREAKDOWN or FR_ENAN (x holds the
 * last iterate in all three numerical cases). */
fr_status fr_gmres_solve(const fr_disc* disc, const fr_ejacobi* pc, const double* d_U,
                         const double* d_R0, double shift, const double* d_b, double* d_x,
                         const fr_gmres_opts* opts, fr_gmres_stats* stats, void* d_work,
                         fr_stream stream);

/* ---- learned warm start (an addition to the paper's method) --------------
 * A per-element MLP predicts a stage increment Y_i from the element's entries of
 * [U, R(U), Y_{i-1}/dt, Y_{i-2}/dt]: n_in = 16 Np inputs (field, variable, point),
 * standardised per (field, variable); two GELU hidden layers of n_hidden;
 * n_out = 4 Np outputs = Y_i/dt standardised per variable.  BF16 weights and layer
 * inputs, FP32 accumulation (MFMA), FP32 biases. */
typedef struct fr_mlp {
  int n_in, n_hidden, n_out;
  void* d_w;      /* bf16: W1[h][in], W2[h][h], W3[out][h], then W1^T, W2^T, W3^T (fr_mlp_weight_bytes) */
  float* d_b;     /* b1[h], b2[h], b3[out] */
  float* d_norm;  /* (mean, std) of the 16 input groups [field][var], then of the 4 output variables: 40 floats */
} fr_mlp;

/* Training state: FP32 master parameters W1, b1, W2, b2, W3, b3 (fr_mlp_param_count
 * floats each for master, gradient, and Adam's first and second moments). */
typedef struct {
  fr_mlp net;
  float* d_master;
  float* d_grad;
  float* d_m;
  float* d_v;
  int t;           /* Adam step counter */
  float lr, beta1, beta2, eps;  /* lr <= 0: compute gradients only */
} fr_mlp_trainer;

/* Samples logged by the ROW step for one stage: per sample 20 Np floats, the
 * unnormalised inputs (16 Np) followed by the converged Y_i/dt (4 Np). */
typedef struct {
  float* d_samples;      /* capacity x 20 Np floats */
  const int* d_elems;    /* per_stage element indices logged after each solve of this stage */
  int per_stage;
  int capacity;          /* samples */
  int count;             /* samples stored so far (advanced by the step) */
} fr_stage_log;

/* Options and statistics of one time step. */
typedef struct {
  fr_gmres_opts lin;     /* linear solver (ROW: every stage; ESDIRK/BDF2: every PTC iteration) */
  double tol_nl;         /* PTC: stop when ||F|| <= tol_nl ||F(q0)|| */
  double dtau_init;      /* PTC initial pseudo-step; <= 0 means dt (Section 4.4) */
  double dtau_max;       /* PTC cap (Section 4.4: 1e20); halved on each rejection */
  int max_ptc;           /* PTC iterations per stage; <= 0 means 200 */
  int max_reject;        /* PTC rejections per stage; <= 0 means 30 */
  int precond_precision; /* FR_F64 or FR_F32 element-Jacobi */
  int commit_unconverged;/* 1: apply the update even if a linear/nonlinear solve did not converge */
  /* Learned starts (an addition to the method).  ROW: one network per stage; stage i
     starts GMRES from its prediction of Y_i; if that guess's residual is not below ||b||
     (the zero guess's), GMRES starts from zero instead, the tolerance staying relative to
     ||b||.  ESDIRK: one network per implicit stage (s - 1); BDF2: one network; the
     prediction y of the increment q_i - q^n gives a second PTC starting point q^n + y,
     used when its ||F|| is below that of the plain start (q_{i-1}, or q^n), the
     nonlinear tolerance staying relative to the plain start's ||F||.  Network inputs:
     q^n, R(q^n) and the two previous increments (stage increments Y or q_j - q^n; for
     the first stages, and for BDF2, the previous step's, from d_yhist). */
  const fr_mlp* warm;    /* NULL, or the networks */
  fr_stage_log* log;     /* NULL, or one log per (implicit) stage: training samples after
                            each converged stage */
  double* d_yhist;       /* NULL, or 2 x ndof: in, the previous step's last two increments
                            (older first); out, this step's.  NULL = zeros. */
  void* d_mlp_work;      /* fr_mlp_work_bytes bytes when warm != NULL */
} fr_solver_opts;

typedef struct {
  int gmres_iters;     /* all Arnoldi iterations of the step */
  int ptc_iters;       /* accepted PTC iterations (ESDIRK, BDF2) */
  int rejections;      /* rejected PTC iterations */
  int linear_solves;   /* GMRES calls */
  int unconverged;     /* GMRES calls that ended above tolerance */
  int warm_used;       /* stages whose GMRES started from the learned guess */
  int warm_rejected;   /* stages whose learned guess lost to the zero guess */
  long residual_evals; /* residual evaluations incl. JF products */
  double wall_s;       /* host wall time of the call */
} fr_step_stats;

/* One step of a linearly implicit ROW scheme (Section 4.3, eq.
 * Rosenbrock_General) in transformed form, Jacobian and preconditioner frozen
 * at q^n, shift 1/(gamma dt):
 *   (I/(gamma dt) - dR/dq)^n Y_i = R(q^n + sum_{j<i} a_ij Y_j) + (1/dt) sum_{j<i} c_ij Y_j,
 *   q^{n+1} = q^n + sum_j m_j Y_j.
 * scheme: FR_ROW2 (3-stage order-2 stiffly accurate scheme with gamma = 1/4),
 * FR_ROW3 (ROS34PW2), FR_ROW4 (RODASP).  Stage solves start from zero.
 * d_U: in q^n, out q^{n+1}.  d_work: FR_WS_STEP bytes. */
fr_status fr_row_step(const fr_disc* disc, int scheme, double dt, double* d_U,
                      const fr_solver_opts* opts, fr_step_stats* stats, void* d_work,
                      fr_stream stream);

/* One ESDIRK step (Section 4.2, eq. ESDIRK2): explicit first stage; stage
 * i >= 2 solves F(q_i) = (q_i - q^n - dt sum_{j<i} a_ij R(q_j))/(omega dt)
 * - R(q_i) = 0 (eq. SDIRK_newton) by pseudo-transient continuation (Section
 * 4.4: eq. linearized_pseudo_transient_final, SER pseudo-step, rejection and
 * halving of dtau_max when GMRES does not gain one order of magnitude),
 * starting from q_{i-1}; q^{n+1} = q^n + dt sum_i b_i R(q_i).
 * scheme: FR_ESDIRK2/3/4.  d_U in/out.  d_work: FR_WS_STEP bytes. */
fr_status fr_esdirk_step(const fr_disc* disc, int scheme, double dt, double* d_U,
                         const fr_solver_opts* opts, fr_step_stats* stats, void* d_work,
                         fr_stream stream);

/* One BDF2 step (Section 4.1, eq. BDF: omega = 2/3, a_1 = 4/3, a_2 = -1/3),
 * F from eq. BDF_newton solved by the same PTC starting from q^n.  With
 * d_Unm1 == NULL a BDF1 step (omega = 1, a_1 = 1) is taken (start-up).
 * d_Unp1 receives q^{n+1} and may alias neither input. */
fr_status fr_bdf2_step(const fr_disc* disc, double dt, const double* d_Unm1, const double* d_Un,
                       double* d_Unp1, const fr_solver_opts* opts, fr_step_stats* stats,
                       void* d_work, fr_stream stream);

/* Vector helpers used around the solver (device arrays of ndof doubles). */
/* L2 error of Section 5.1 for variable `var` (0 = rho, 1 = u velocity) of
 * d_U against the exact isentropic vortex (eq. VP_Solution) at time t:
 * sqrt(sum_e sum_k w_k |J|_k (s_exact - s_num)^2 / V), Gauss quadrature at
 * the solution points.  Vortex parameters in h_params[14]: rho_inf, u_inf,
 * v_inf, p_inf, R, gamma, alpha, phi, xc, yc, xlo, ylo, Lx, Ly.
 * Synchronises; result in *h_err. */
fr_status fr_l2_error_vortex(const fr_disc* disc, const double* d_U, int var, double t,
                             const double* h_params, double* h_err, void* d_work, fr_stream stream);

/* Sizes: bf16 weight bytes (with the transposed copies), FP32 parameter count,
 * and workspace bytes for inference on the disc's mesh and training batches of
 * `batch` samples. */
size_t fr_mlp_weight_bytes(int n_in, int n_hidden, int n_out);
size_t fr_mlp_param_count(int n_in, int n_hidden, int n_out);
size_t fr_mlp_work_bytes(const fr_disc* disc, int n_hidden, int batch);

/* Stage-increment guess x0 (ndof doubles) of every element from U, R = R(U) and the
 * two previous increments (NULL = zero). */
fr_status fr_mlp_infer(const fr_disc* disc, const fr_mlp* net, const double* d_U, const double* d_R,
                       const double* d_Y1, const double* d_Y2, double dt, double* d_x0, void* d_work,
                       fr_stream stream);

/* Raw forward pass on standardised bf16 features d_x[batch][n_in] -> d_y[batch][n_out] (FP32). */
fr_status fr_mlp_forward(const fr_mlp* net, const uint16_t* d_x, int batch, float* d_y, void* d_work,
                         fr_stream stream);

/* Standardisation statistics of net->d_norm from the logged samples of `log`. */
fr_status fr_mlp_fit_stats(const fr_disc* disc, const fr_stage_log* log, fr_mlp* net, fr_stream stream);

/* Write the bf16 weights and FP32 biases of tr->net from the master copy. */
fr_status fr_mlp_sync(fr_mlp_trainer* tr, fr_stream stream);

/* One training step on the logged samples d_idx[0..batch): forward, mean-squared-error
 * gradients (tr->d_grad), and an Adam update of the master copy followed by fr_mlp_sync
 * (skipped when tr->lr <= 0).  With h_loss != NULL it synchronises and returns the batch
 * MSE before the update; with h_loss == NULL it only enqueues the step (no host read). */
fr_status fr_mlp_train_step(const fr_disc* disc, fr_mlp_trainer* tr, const fr_stage_log* log, const int* d_idx,
                            int batch, double* h_loss, void* d_work, fr_stream stream);

/* Several networks of equal sizes (one per stage, say) trained together: `steps` training
 * steps of each of the `count` (1..8) trainers trs[q] on its own log logs[q], every kernel
 * of a step launched once for all networks.  d_idx: device int32 [count][steps][batch]
 * logged-row indices (each below its log's count; not checked, device data).  h_lr: host
 * [steps] learning rates, written to every trs[q].lr before step k (NULL: each keeps its
 * own).  Network q's arithmetic is that of fr_mlp_train_step, in the same order, so it
 * ends bitwise where `steps` calls of fr_mlp_train_step would have left it.  h_loss:
 * host [count], the batch MSE of each network's last step before its update (the call
 * then synchronises), or NULL (enqueue only).  d_work: fr_mlp_group_work_bytes bytes. */
size_t fr_mlp_group_work_bytes(const fr_disc* disc, int n_hidden, int batch, int count);
fr_status fr_mlp_train_group(const fr_disc* disc, fr_mlp_trainer* trs, const fr_stage_log* logs, int count,
                             const int* d_idx, int steps, int batch, const float* h_lr, double* h_loss,
                             void* d_work, fr_stream stream);

/* Coefficients of the built-in schemes, for inspection: kind 0 = ROW
 * (transformed a_ij, c_ij, m_j, gamma), kind 1 = ESDIRK (a_ij, b_i).
 * h_a and h_c: s*s row-major (c unused for ESDIRK), h_b: s.  Returns the
 * number of stages s, or a negative status. */
int fr_scheme_table(int kind, int scheme, double* h_a, double* h_c, double* h_b, double* h_gamma);

/* Force of the fluid on the wall at the eta = -1 side of row 0 (bc_south = FR_BC_WALL),
 * per unit depth: minus the momentum part of the common flux F^num on the wall faces
 * (pressure minus viscous stress, the wall's reading of the boundary above), integrated
 * with the Gauss weights along each face; the drag and lift coefficients of the cylinder
 * case (Section 5.2) are h_force / (rho u^2 D / 2).  d_work: fr_workspace_bytes(disc,
 * FR_WS_RESIDUAL, 0, 0) bytes.  Synchronises; FR_EINVAL without a wall. */
fr_status fr_wall_force(const fr_disc* disc, const double* d_U, double* h_force, void* d_work, fr_stream stream);

/* ---- 3D hexahedral FR (Section 3's hexahedral forms; the Taylor-Green vortex of
 * Section 5.3) ---------------------------------------------------------------
 * Uniform hexahedra of a triply periodic box, nx x ny x nz elements of size
 * len / (nx, ny, nz); Gauss solution points; state q = (rho, rho u, rho v, rho w, E)
 * stored [v][e][k] with e = (ez ny + ey) nx + ex and k = (c n + b) n + a (a along x,
 * c along z), n = p + 1.  mu > 0: Navier-Stokes with the BR2 common gradient (as
 * FR_BR2 above: each side's raw gradient plus its lifting with (P+1)(P+2)/2), zero
 * bulk viscosity; mu = 0: Euler.  Common inviscid flux FR_RUSANOV or FR_ROE. */
typedef struct fr3d_disc fr3d_disc;  /* opaque */
typedef struct {
  int nx, ny, nz;   /* elements per direction, >= 2 */
  int p;            /* 2 .. 4 */
  int flux;         /* FR_RUSANOV or FR_ROE */
  double lo[3];     /* box corner */
  double len[3];    /* box side lengths, > 0 */
  double gamma, rgas, mu, prandtl;
} fr3d_desc;

/* FR_EINVAL for sizes or parameters out of range. */
fr_status fr3d_create(const fr3d_desc* desc, fr3d_disc** out);
void fr3d_destroy(fr3d_disc* disc);
/* 5 * nel * (p+1)^3. */
size_t fr3d_ndof(const fr3d_disc* disc);
/* Workspace of every fr3d_ call below: the face traces (and raw face gradients with
 * mu > 0), reduction partials and two state vectors (SSPRK3 stages). */
size_t fr3d_workspace_bytes(const fr3d_disc* disc);
/* Physical coordinates of the solution points: h_xyz[3][nel (p+1)^3] on the host. */
fr_status fr3d_solution_points(const fr3d_disc* disc, double* h_xyz);
/* R(q): -sum_d (2/h_d)(D f_d + correction terms), f_d inviscid minus viscous flux. */
fr_status fr3d_residual(const fr3d_disc* disc, const double* d_U, double* d_R, void* d_work, fr_stream stream);
/* w = shift v - [R(U + e v) - R0] / e, e = eps / rms(v) (FR_EPS_RMS) or eps (Section 4.5). */
fr_status fr3d_jf_matvec(const fr3d_disc* disc, const double* d_U, const double* d_R0, const double* d_v,
                         double shift, double eps, int eps_mode, double* d_w, void* d_work, fr_stream stream);
/* One SSPRK3 step in place (the paper's explicit reference integrator, Section 5.3):
 * U1 = U + dt R(U), U2 = 3/4 U + 1/4 (U1 + dt R(U1)), U = 1/3 U + 2/3 (U2 + dt R(U2)). */
fr_status fr3d_ssprk3_step(const fr3d_disc* disc, double* d_U, double dt, void* d_work, fr_stream stream);
/* Kinetic energy and dissipation rates of Section 5.3 (h_out = E_k, eps1, eps3; eps2 = 0
 * at zero bulk viscosity): E_k = int rho |u|^2/2 dV / (rho0 V), eps1 = 2 mu int S^d:S^d dV /
 * (rho0 V), eps3 = -int (p - <p>) div u dV / (rho0 V), the velocity gradient from the raw
 * gradient of each element's solution polynomial, Gauss quadrature.  <p> is the volume mean
 * of p: int div u dV = 0 on the periodic box for the exact field, and taking p about its
 * mean drops <p> times the inter-element velocity jumps that the element-local gradient
 * leaves in that integral.  Synchronises. */
fr_status fr3d_dissipation(const fr3d_disc* disc, const double* d_U, double rho0, double* h_out, void* d_work,
                           fr_stream stream);

/* ---- implicit steps on the 3D path (Sections 4.1-4.5 on the hexahedral
 * discretisation; the implicit comparison of Section 5.3) --------------------------
 * Element-Jacobi blocks P_e = shift I - dR_e/dq_e of Nb = 5 (p+1)^3 rows (p = 2: 135,
 * p = 3: 320; other p: FR_EINVAL), FP64, column-major per element: the entry in row i,
 * column j of block e at [(e Nb + j) Nb + i], rows and columns ordered v (p+1)^3 + k.
 * Column j is the one-sided difference -(R_e(q + delta u_j) - R_e(q)) / delta with
 * delta = 1e-8 max(1, |q_j|) and every neighbour's state unchanged (the elements are
 * coloured so that face neighbours differ, and one evaluation of the residual on the
 * elements of a colour gives column j of all of them: c Nb such evaluations per assembly,
 * c = 2 when nx, ny, nz are even).  The inverses come from Gauss-Jordan with partial
 * pivoting, same layout. */
size_t fr3d_ejacobi_bytes(const fr3d_disc* disc);  /* nel Nb^2 doubles */
/* Workspace of the calls below for restart length m (1 .. 64): the residual's face data,
 * the steps' assembled blocks and inverses (2 fr3d_ejacobi_bytes), eight copies of the
 * state, its residual and its face data (the assembly evaluates eight block columns per
 * launch), m + 1 Krylov and m preconditioned vectors, and 14 more state vectors; 0 for a
 * bad m. */
size_t fr3d_step_workspace_bytes(const fr3d_disc* disc, int m);
/* The blocks at (d_U, shift) into d_blocks (fr3d_ejacobi_bytes bytes).  d_work:
 * fr3d_step_workspace_bytes(disc, 1) bytes. */
fr_status fr3d_ejacobi_assemble(const fr3d_disc* disc, const double* d_U, double shift, double* d_blocks,
                                void* d_work, fr_stream stream);
/* The inverse blocks at (d_U, shift) into d_inv (fr3d_ejacobi_bytes bytes).  d_work as above. */
fr_status fr3d_ejacobi_factor(const fr3d_disc* disc, const double* d_U, double shift, double* d_inv,
                              void* d_work, fr_stream stream);
/* z = P^{-1} r element by element (ndof doubles each, not aliased). */
fr_status fr3d_ejacobi_apply(const fr3d_disc* disc, const double* d_inv, const double* d_r, double* d_z,
                             fr_stream stream);
/* (shift I - dR/dq(U)) x = b by restarted flexible GMRES(m) (classical Gram-Schmidt
 * applied twice), right-preconditioned by d_inv (factored with the same shift), with the
 * Jacobian-free product about (d_U, d_R0 = R(d_U)); options, statistics and returns as
 * fr_gmres_solve (element-Jacobi only; a breakdown counts as converged).  d_x: in the
 * initial guess, out the solution.  d_work: fr3d_step_workspace_bytes(disc, opts->m)
 * bytes.  Synchronises. */
fr_status fr3d_gmres_solve(const fr3d_disc* disc, const double* d_inv, const double* d_U, const double* d_R0,
                           double shift, const double* d_b, double* d_x, const fr_gmres_opts* opts,
                           fr_gmres_stats* stats, void* d_work, fr_stream stream);
/* One ROW, ESDIRK or BDF2 step as fr_row_step, fr_esdirk_step and fr_bdf2_step (same
 * schemes, options, statistics and returns): element-Jacobi formed once per ROW step and
 * at every PTC iterate, in FP64 or (opts->precond_precision = FR_F32) assembled, inverted
 * and applied in FP32; no learned starts (opts->warm, log and d_yhist must be NULL); residual_evals includes the c Nb single-colour evaluations of every
 * assembly.  d_work:
 * fr3d_step_workspace_bytes(disc, opts->lin.m) bytes.  Synchronises. */
fr_status fr3d_row_step(const fr3d_disc* disc, int scheme, double dt, double* d_U, const fr_solver_opts* opts,
                        fr_step_stats* stats, void* d_work, fr_stream stream);
fr_status fr3d_esdirk_step(const fr3d_disc* disc, int scheme, double dt, double* d_U, const fr_solver_opts* opts,
                           fr_step_stats* stats, void* d_work, fr_stream stream);
fr_status fr3d_bdf2_step(const fr3d_disc* disc, double dt, const double* d_Unm1, const double* d_Un, double* d_Unp1,
                         const fr_solver_opts* opts, fr_step_stats* stats, void* d_work, fr_stream stream);

/* Last error message of this thread ("" if none). */
const char* fr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FRJF_H */
