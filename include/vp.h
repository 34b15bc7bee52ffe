/*
 * vp.h - C ABI of libvp, the MI355X (gfx950) stress-velocity Newton-Krylov solver
 * for one implicit Euler step of the viscous-plastic sea-ice momentum equation.
 *
 * Paper: Shih, Mehlmann, Losch, Stadler, "Robust and efficient primal-dual
 * Newton-Krylov solvers for viscous-plastic sea-ice models" (arXiv 2204.10822).
 *
 * Problem (Sec. 3, eq. Av=F, eq. A, eq. F): given the previous velocity v^n, the
 * (already advanced) thickness H and concentration A, wind v_air and ocean
 * current v_ocean, find v = v^{n+1} with A(v, phi) = F(phi) for all Q1 test
 * functions phi vanishing on the boundary.  The stress-velocity Newton method of
 * Sec. 4.2 introduces pi = tau(v)/Delta(v) (eq. pi) and solves each linearisation
 * (eq. linearSVNewton with eq. modification) by AMG-preconditioned Krylov.
 *
 * Discretisation: uniform structured quadrilateral mesh of [0,Lx]x[0,Ly] with
 * nx x ny cells, Q1 velocity, cellwise-constant H and A (Sec. 5.1), 2x2 Gauss
 * quadrature for every term, zero velocity on the whole boundary (Sec. 2).
 *
 * Conventions (all entry points):
 *  - Array arguments are caller-owned, contiguous DEVICE pointers (e.g. torch
 *    tensor data_ptr() values on the context's stream) unless stated as host.
 *    The library never keeps a caller pointer past the call; vp_set_state copies.
 *  - Layouts:  cell field   [ny][nx]                     (double)
 *              node vector  [(ny+1)(nx+1)][2]  node n = j*(nx+1)+i, x comp first
 *              pi           [4 qp][3 comp][ny][nx], comps (xx, yy, xy) of the
 *                           symmetric 2x2 tensor; qp = qx + 2*qy, where qx (qy)
 *                           is 0 at the Gauss point 1/2 - 1/(2 sqrt 3) of the
 *                           cell's x (y) extent and 1 at 1/2 + 1/(2 sqrt 3).
 *  - All work is enqueued on the stream given to vp_create.  Calls returning
 *    host scalars synchronise that stream.
 *  - Return codes: 0 = OK, > 0 = soft outcome with valid outputs, < 0 = error
 *    (outputs unspecified; vp_last_error() gives text).  No C++ exception
 *    crosses the ABI.  One context per host thread at a time.
 */
#ifndef VP_H
#define VP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Mesh, physics constants (Table tab:params) and step settings (Sec. 5.2/5.3). */
typedef struct {
  int32_t nx, ny;          /* cells per side; nodes (nx+1)(ny+1) for Q1 velocity,    */
                           /* (2nx+1)(2ny+1) for Q2                                 */
  double Lx, Ly;           /* domain size [m]                                       */
  double rho_ice, rho_air, rho_ocean;  /* densities [kg/m^3]                        */
  double C_air, C_ocean;   /* drag coefficients                                     */
  double P_star;           /* ice strength parameter [N/m^2]                        */
  double C_strength;       /* concentration parameter C in P = P* H exp(-C(1-A))    */
  double e_ratio;          /* ellipse ratio e                                       */
  double f_coriolis;       /* Coriolis parameter [1/s], explicit (Sec. 3 footnote)  */
  double dt;               /* time step [s]                                         */
  double delta_min;        /* Delta_min [1/s] (eq. Delta)                           */
  int32_t order;           /* velocity elements: 1 (or 0) = Q1 with 2x2 Gauss, 2 = Q2 */
                           /* (biquadratic, 3x3 Gauss; Sec. 5).  With Q2 the          */
                           /* operator is a block 25-point stencil, pi has 9 points   */
                           /* per cell, and the AMG smooths with the Q2 operator and   */
                           /* coarsens it with the unsmoothed aggregation prolongator  */
                           /* (level 1 = Ptent^T K2 Ptent, a 9-point block stencil)    */
} vp_problem_desc;

typedef struct vp_ctx_s* vp_ctx;

enum {
  VP_OK = 0,
  VP_NOT_CONVERGED = 1,    /* Newton hit its iteration cap                          */
  VP_LINESEARCH_FAIL = 2,  /* backtracking found no acceptable step                 */
  VP_KRYLOV_MAXIT = 3,     /* Krylov hit maxit before rtol (outputs are the iterate)*/
  VP_EINVAL = -1,          /* bad argument                                          */
  VP_EHIP = -2,            /* HIP runtime error                                     */
  VP_ENOMEM = -3,          /* device allocation failed                              */
  VP_ESTATE = -4,          /* call out of order (e.g. solve before assemble)        */
  VP_ENONFINITE = -5,      /* NaN/Inf met in a residual, energy or Krylov scalar    */
  VP_EBREAKDOWN = -6       /* Krylov breakdown (indefinite or singular operator)    */
};
enum { VP_SVN = 0, VP_STDN = 1 };                         /* linearisation          */
enum { VP_PREC_FP64 = 0, VP_PREC_FP32 = 1, VP_PREC_FP32_BF16COARSE = 2, VP_PREC_BF16 = 3,
       VP_PREC_FP16_BF16COARSE = 4, VP_PREC_FP16 = 5, VP_PREC_FP16_FP32COARSE = 6 };
enum { VP_KRYLOV_FGMRES = 0, VP_KRYLOV_FCG = 1 };
enum { VP_LS_ENERGY = 0, VP_LS_RESIDUAL = 1 };

/* Create a context for one mesh.  hip_stream: a hipStream_t (NULL = null stream).
 * Errors: VP_EINVAL for nx or ny < 2, non-positive sizes, dt, delta_min, e_ratio
 * or negative P_star/densities; VP_ENOMEM/VP_EHIP on device failure. */
int vp_create(const vp_problem_desc* desc, void* hip_stream, vp_ctx* out);
void vp_destroy(vp_ctx ctx);
/* Text of the last error on this context (or of the last vp_create failure when
 * ctx is NULL).  Valid until the next call on the context. */
const char* vp_last_error(vp_ctx ctx);

/* Set the step's data (copied): H, A cell fields [ny][nx]; v_air, v_ocean, v_prev
 * node vectors.  Computes P = P* H exp(-C(1-A)) (eq. ice-strength), rho_ice*H and
 * the load vector F(phi_i) of eq. F (explicit Coriolis on v_prev - v_ocean,
 * air stress C_a rho_a |v_a| v_a of eq. force at quadrature points).
 * The data are checked first (one device pass, synchronises): VP_EINVAL if any H
 * is negative or not finite, any A lies outside [0, 1] or is not finite, or any
 * velocity component is not finite; the context then keeps its previous state.
 * A copy of H, A, v_air and v_prev is kept for vpnet_infer (vpnet.h). */
int vp_set_state(vp_ctx ctx, const double* H, const double* A, const double* v_air,
                 const double* v_ocean, const double* v_prev);

/* Residual of eq. Av=F: r_i = A(v, phi_i) - F(phi_i) with sigma in the tau form of
 * eq. sigma; r = 0 at boundary dofs.  r may be NULL.  rnorm (host, nullable):
 * l2 norm over free dofs.  energy (host, nullable): Phi(v) of eq. energy.
 * Synchronises when rnorm or energy is requested.  VP_ENONFINITE if either is
 * not finite. */
int vp_residual(vp_ctx ctx, const double* v, double* r, double* rnorm, double* energy);

/* Assemble the linearised operator at (v, pi) into the context:
 *  VP_SVN : eq. linearSVNewton with tau_l (x) pi_l replaced as in eq. modification
 *  VP_STDN: eq. standardNewton1 (pi ignored, may be NULL)
 * plus the ocean-drag Jacobian of eq. standardNewton2 and the mass term.  Stored
 * as a 9-point block stencil with identity rows/columns at boundary dofs. */
int vp_newton_assemble(vp_ctx ctx, const double* v, const double* pi, int variant);
/* y = K x with the last assembled operator (FP64).  VP_ESTATE before assembly. */
int vp_operator_apply(vp_ctx ctx, const double* x, double* y);
/* Copy the assembled operator to a device buffer of 20*(nx+1)*(ny+1) doubles,
 * layout [blk][node n][r][c]: entry (r,c) of the 2x2 block coupling node n (row
 * dofs) to node n+off(blk), blk 0..4 = self, east (+1,0), north (0,+1),
 * north-east (+1,+1), north-west (-1,+1); the other four neighbours are the
 * transposes held by those nodes (the operator is symmetric). */
int vp_operator_export(vp_ctx ctx, double* blocks);

/* AMG preconditioner built on the last assembled operator, of one of two kinds:
 *  VP_AMG_SA (default): smoothed aggregation (the library's replacement for the
 *    paper's BoomerAMG, Sec. 5.4): structured 3x3-node aggregates, rigid-body
 *    near-null space, one block-Jacobi smoothing of the prolongator, Galerkin
 *    coarse operators, Chebyshev smoothing, dense coarsest solve;
 *  VP_AMG_RS: classical Ruge-Stueben AMG with the settings Sec. 5.4 reports for
 *    BoomerAMG: scalar strength of connection with threshold strong_threshold
 *    (0.5) and the max_row_sum rule for diagonally dominant rows, first-pass
 *    coarsening (parallel rounds), classical interpolation, Galerkin coarse
 *    operators, `sweeps` (3) symmetric Gauss-Seidel sweeps per smoothing
 *    (multicolour ordering), Gaussian elimination once a level has <= max_coarse
 *    rows (or 25 levels); FP64 only (precision must be VP_PREC_FP64).
 * The Chebyshev fields apply to VP_AMG_SA only; the last four to VP_AMG_RS only. */
enum { VP_AMG_SA = 0, VP_AMG_RS = 1 };
typedef struct {
  int cheb_degree;       /* Chebyshev degree per pre/post smoothing (>= 1)         */
  int max_coarse;        /* coarsest level dof bound (<= 1024)                     */
  int precision;         /* VP_PREC_*: V-cycle arithmetic and operator storage:
                            FP64; FP32; FP32 finest + BF16 Jacobi-scaled coarse levels;
                            BF16 Jacobi-scaled on every level (FP32 arithmetic;
                            experimental: ~4x the Krylov iterations of FP32);
                            FP16 Jacobi-scaled finest + BF16 Jacobi-scaled coarse;
                            FP16 Jacobi-scaled on every level;
                            FP16 Jacobi-scaled finest smoothing with the residual
                            after the coarse-grid correction in FP32, and FP32
                            Jacobi-scaled coarse levels.  In the FP32 and FP32 +
                            BF16-coarse modes the hierarchy is built from FP32
                            copies: spectral bounds, prolongator smoothing and
                            the Galerkin products (A P accumulated in FP32, the
                            coarse sums in FP64) read each level's FP32 operator */
  double cheb_ratio;     /* smoothing interval [lmax/ratio, lmax]                  */
  double omega_scale;    /* prolongator damping scale (1 = 4/(3 lmax))             */
  int kind;              /* VP_AMG_SA or VP_AMG_RS                                 */
  int sweeps;            /* RS: symmetric Gauss-Seidel sweeps per smoothing (1..16) */
  double strong_threshold; /* RS: strength threshold theta in (0, 1)              */
  double max_row_sum;    /* RS: rows with |row sum| > max_row_sum |a_ii| have no
                            strong couplings (1 switches the rule off)             */
  int variant;           /* SA, for verification: 0 = the fastest kernels; a set of
                            VP_AMG_VAR_* flags selects reference kernels that
                            compute the same V-cycle bit for bit                  */
  int walk4_rows;        /* SA, for verification: 0 = automatic strip height of
                            the four-sweep walk (degree-4 FP32/FP64 smoothing on the
                            finest level); 1..4096 = that height                   */
} vp_amg_opts;
enum {
  VP_AMG_VAR_NO_TAIL = 1,      /* one launch per sweep on the smallest levels too      */
  VP_AMG_VAR_NO_PAIRS = 2,     /* one launch per Chebyshev sweep (no fused sweeps)     */
  VP_AMG_VAR_NO_TAIL_LDS = 4,  /* the single-workgroup tail reloads its vectors        */
  VP_AMG_VAR_NO_P16 = 8        /* FP16 modes: FP32 finest restriction/prolongation     */
};
int vp_amg_setup(vp_ctx ctx, const vp_amg_opts* opts);
/* z = M^{-1} r, one V-cycle.  VP_ESTATE before vp_amg_setup. */
int vp_amg_apply(vp_ctx ctx, const double* r, double* z);
/* Number of AMG levels (host out) and their node grids (host arrays of >= 25). */
int vp_amg_info(vp_ctx ctx, int* levels, int* nxn, int* nyn, int* dofs_per_node);
/* Copy AMG level `level` (0 = finest) to device buffers, for inspection.
 *  A (nullable): the level's FP64 operator, 5*B*B*nn doubles in the layout of
 *    vp_operator_export with B x B blocks (B = dofs per node and nn = nxn*nyn
 *    from vp_amg_info).
 *  P (nullable; not on the coarsest level): the smoothed prolongator to level+1,
 *    12*B*nn doubles, P[((s*B + r)*3 + c)*nn + n] = entry (fine dof r of node n,
 *    coarse dof c) for the coarse node in slot s = sx + 2*sy.  Along x, sx = 0
 *    names the aggregate holding the node (aggregates are runs of 3 nodes, the
 *    last run 3..5) and sx = 1 the neighbouring aggregate that a run's first or
 *    last node also touches; the same along y.  Absent slots hold 0.  In the
 *    FP32 and FP32 + BF16-coarse modes the prolongators are made in FP32 only
 *    (from the FP32 operators): their values widened to FP64.
 * Asynchronous on the context's stream.  VP_ESTATE before vp_amg_setup; VP_EINVAL
 * for a level out of range or P asked for on the coarsest level. */
int vp_amg_export(vp_ctx ctx, int level, double* A, double* P);
/* Classical AMG (VP_AMG_RS) level sizes, for inspection: out (host, 5 entries) =
 * {rows n, entries of A, coarse points nc, entries of P, colours}; nc, P entries
 * and colours are 0 on the coarsest level.  vp_amg_info reports the rows of each
 * level in nxn, 1 in nyn and dofs_per_node.  VP_ESTATE unless the last setup was
 * VP_AMG_RS; VP_EINVAL for a level out of range. */
int vp_amg_rs_info(vp_ctx ctx, int level, int64_t* out);
/* Copy classical-AMG level `level` to device buffers (each nullable), sizes from
 * vp_amg_rs_info: A as CSR (A_ptr n+1, A_col and A_val entries of A; columns
 * ascending in each row; level 0 uses the vectors' dof numbering 2*node + comp);
 * cf[n] (1 = coarse point, 0 = fine point); P as CSR (n+1 / entries of P; coarse
 * points are numbered in fine order); colour[n] (the smoother's colour of each
 * row).  Asynchronous except for cf.  VP_EINVAL for cf, P or colour on the
 * coarsest level. */
int vp_amg_rs_export(vp_ctx ctx, int level, int32_t* A_ptr, int32_t* A_col, double* A_val, int32_t* cf,
                     int32_t* P_ptr, int32_t* P_col, double* P_val, int32_t* colour);

/* Krylov solve K x = b with the last assembled operator and AMG (Sec. 5.4):
 * FGMRES(restart) right-preconditioned with classical Gram-Schmidt applied twice,
 * or flexible CG.  x holds the initial guess on entry.  Stops at
 * ||b - K x|| <= rtol ||b||.  VP_KRYLOV_MAXIT (soft) after maxit iterations. */
typedef struct { int method; int restart; int maxit; double rtol; } vp_krylov_opts;
typedef struct { int iters; double rel_resid; } vp_krylov_info;
int vp_krylov_solve(vp_ctx ctx, const double* b, double* x, const vp_krylov_opts* opts,
                    vp_krylov_info* info);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the flexible-CG solve of
 * vp_krylov_solve (opts->method must be VP_KRYLOV_FCG; restart is ignored) with
 * its four work vectors in a static device array of the library instead of a
 * workspace allocated on the first solve.  The call allocates nothing; the
 * operator and AMG hierarchy come from earlier vp_newton_assemble / vp_amg_setup
 * calls.  Limit: at most 2,359,296 dofs (a 1085 x 1085-cell Q1 mesh); the array
 * takes 72 MiB on every GPU the library runs on, from the first vp_create on that
 * GPU until the process ends.  All contexts on one GPU share it and it keeps the
 * last call's contents (the solve overwrites every entry it reads), so calls on
 * one GPU that overlap in time (other host threads, other streams) race.  Event
 * profiling (vp_profile) records nothing during this call.  Results are those of
 * vp_krylov_solve with method VP_KRYLOV_FCG.  VP_EINVAL for null pointers, another
 * method or a larger mesh; VP_ESTATE before assembly or AMG setup. */
int vp_krylov_solve_noalloc(vp_ctx ctx, const double* b, double* x, const vp_krylov_opts* opts,
                            vp_krylov_info* info);

/* Dual update (eq. tautilde with eq. modification, Sec. 4.2):
 * pi <- pi + alpha * pi~(v, dv, pi), in place. */
int vp_pi_update(vp_ctx ctx, const double* v, const double* dv, double* pi, double alpha);
/* pi <- tau(v)/Delta(v) at every quadrature point (eq. pi). */
int vp_pi_init(vp_ctx ctx, const double* v, double* pi);

/* One Newton iteration in place on (v, pi): residual, assembly, AMG setup, Krylov
 * solve to the Eisenstat-Walker tolerance, energy backtracking (halving from 1,
 * Sec. 5.1), dual update, velocity update.  tol: relative target on
 * ||R|| / ||R(0)|| (used for the inner-tolerance floor). */
typedef struct {
  int variant;           /* VP_SVN or VP_STDN                                      */
  double tol;            /* nonlinear target, relative to ||R(v=0)||               */
  double eta_max;        /* cap of the inner relative tolerance                    */
  int max_backtracks;    /* halvings before VP_LINESEARCH_FAIL                     */
  int ls_mode;           /* VP_LS_ENERGY or VP_LS_RESIDUAL                         */
} vp_newton_opts;
typedef struct {
  double rnorm;          /* ||R|| at the start of the iteration                    */
  double rnorm0;         /* ||R(v=0)||                                             */
  double rnorm_new;      /* ||R|| after the step                                   */
  double energy, energy_new, alpha, eta;
  int backtracks, krylov_iters;
} vp_newton_info;
int vp_newton_step(vp_ctx ctx, double* v, double* pi, const vp_newton_opts* nopts,
                   const vp_amg_opts* aopts, const vp_krylov_opts* kopts,
                   vp_newton_info* info);

/* Newton loop (Sec. 5.1 stopping rule with a relative target): iterate
 * vp_newton_step until ||R(v)|| <= tol ||R(0)|| or maxit iterations.  The AMG
 * spectral estimates restart from a fixed vector, so the result depends only on
 * the inputs (kernels are deterministic).  Returns
 * VP_OK, VP_NOT_CONVERGED or VP_LINESEARCH_FAIL.  history (host, nullable,
 * maxit+1 entries) receives ||R||/||R(0)|| per iterate. */
typedef struct {
  int iterations, krylov_iters;
  double rnorm0, rel_resid;
} vp_solve_info;
int vp_newton_solve(vp_ctx ctx, double* v, double* pi, int maxit,
                    const vp_newton_opts* nopts, const vp_amg_opts* aopts,
                    const vp_krylov_opts* kopts, vp_solve_info* info, double* history);

/* One explicit Euler step (Sec. 3) of the transport equations eq. model:A and
 * eq. model:H for the cell fields A and H, finite volumes on the cells (Q0, Sec. 5)
 * with the mesh and time step of the context: the normal velocity of a face is
 * the mean of its two nodal values of v (Q1; Simpson's rule on the face's end and
 * midpoint nodes for Q2 velocity), the flux is first-order upwind, the
 * boundary carries no flux (v = 0 there, so the inflow values never enter).  A is
 * clipped to [0, 1] and H to [0, inf) afterwards.  Positivity needs
 * dt (max|u|/hx + max|v|/hy) <= 1 (not checked).
 *  v: device nodes [(ny+1)(nx+1)][2] (Q2: [(2ny+1)(2nx+1)][2]); A, H, A_out, H_out:
 *  device cells [ny][nx].
 * Asynchronous on the context's stream.  VP_EINVAL for null pointers or outputs
 * that alias an input or each other. */
int vp_advect(vp_ctx ctx, const double* v, const double* A, const double* H, double* A_out, double* H_out);

/* Per-kernel timing with HIP events recorded on the context's stream around the
 * launches of selected kernels (finest level only).  vp_profile(ctx, 1) clears
 * and starts recording, vp_profile(ctx, 0) stops.  vp_profile_read synchronises
 * and returns, for kernel id kid, the summed duration [ms], the launch count and
 * the algorithmic bytes one launch must move (each stored value read once, each
 * vector read or written once).  VP_EINVAL for an unknown kid. */
enum {
  VP_KID_APPLY_FINE = 0,   /* y = K x, FP64, the Krylov operator product            */
  VP_KID_CHEB_STEP0 = 1,   /* Chebyshev step on the finest level (fused SpMV)       */
  VP_KID_STEN_RESID0 = 2,  /* r = b - A x on the finest level                        */
  VP_KID_RESIDUAL = 3,     /* nonlinear residual + energy                            */
  VP_KID_ASSEMBLE = 4,     /* operator assembly                                      */
  VP_KID_VCYCLE = 5,       /* one whole V-cycle (composite, not a single kernel)     */
  VP_KID_CHEB_PAIR0 = 6,   /* two fused Chebyshev steps on the finest level          */
  VP_KID_CHEB_WALK4 = 7,   /* a whole degree-4 pre- or post-smoothing on the finest
                              level in one kernel (FP64 and FP32 operators)          */
  VP_KID_COUNT = 8
};
int vp_profile(vp_ctx ctx, int enable);
int vp_profile_read(vp_ctx ctx, int kid, double* total_ms, int* launches, double* bytes_per_launch);

/* Default option sets: svN, tol 1e-8, eta_max 0.1, 30 halvings, energy line
 * search; Chebyshev degree 4 on [lmax/30, lmax], coarsest level <= 140 dofs,
 * FP64 V-cycle, omega scale 1; flexible CG, restart 30 (FGMRES), 500
 * iterations, rtol 1e-2 (replaced by the forcing term inside Newton). */
void vp_default_opts(vp_newton_opts* n, vp_amg_opts* a, vp_krylov_opts* k);

#ifdef __cplusplus
}
#endif
#endif /* VP_H */
