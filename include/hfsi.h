/*
 * hfsi.h — C ABI of the MI355X solid-mechanics hot path.
 *
 * One Newton step of the stabilised equal-order (P1-P1) displacement-pressure
 * hyperelastic solid (Langer & Yang, "Numerical simulation of fluid-structure
 * interaction problems with hyperelastic models I", Sections "The structure
 * sub-problem", "Stabilization for the structure sub-problem" and "Newton's
 * Method"): assemble the residual R and the consistent tangent
 * K = [A B1^T; B2 -C] (eq. globsys), build an algebraic multigrid hierarchy on
 * the displacement block A, solve K dv = -R with FGMRES right-preconditioned by
 * the block-triangular P_L of eq. lpre, and update the state.
 *
 * Conventions shared by every call
 *  - Every call returns hfsi_status: 0 on success, 1 (HFSI_NOT_CONVERGED) is a
 *    warning, negative values are errors.  No C++ exception crosses the ABI;
 *    hfsi_last_error() returns a message for the last failing call.
 *  - "host" pointers are read during the call only and stay owned by the
 *    caller.  "device" pointers are caller-owned device memory of the
 *    context's device (e.g. PyTorch tensors), contiguous, fp64 unless stated.
 *  - Dofs are node-interleaved: dof 4*i + c, c = 0,1,2 the displacement
 *    components and c = 3 the pressure of node i (n nodes, N = 4n dofs).
 *  - All device work is queued on the stream given to hfsi_create.  Calls
 *    that fill an *_info struct synchronise that stream before returning.
 *  - One context per host thread; contexts are independent.
 *  - Call order: set_mesh -> set_materials -> set_bc, then any of
 *    assemble / amg_setup / krylov_amg_solve / newton_step.  Out-of-order
 *    calls return HFSI_E_ORDER.
 *  - Index type is int32: meshes whose matrices exceed 2^31-1 stored
 *    entries are rejected with HFSI_E_ARG.
 */
#ifndef HFSI_H
#define HFSI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HFSI_OK = 0,
  HFSI_NOT_CONVERGED = 1, /* warning: iteration limit reached            */
  HFSI_E_ARG = -1,        /* invalid argument or unsupported size          */
  HFSI_E_HIP = -2,        /* HIP runtime error                             */
  HFSI_E_OOM = -3,        /* device allocation failed                      */
  HFSI_E_ORDER = -4,      /* call sequence violated                        */
  HFSI_E_INVERTED = -5,   /* an element has J <= 0 (message names it)      */
  HFSI_E_BREAKDOWN = -6,  /* Krylov breakdown without convergence          */
  HFSI_E_NAN = -7,        /* NaN/Inf in a residual or update               */
  HFSI_E_CAPACITY = -8    /* a fixed-capacity internal table overflowed    */
} hfsi_status;

typedef struct hfsi_ctx hfsi_ctx;

/* Material record (Section "Nonlinear hyperelastic modeling").
 * model 0: modified Mooney-Rivlin, energy c10/2 (J1-3) + c01/2 (J2-3)
 *          + kappa/2 (J-1)^2 (eq. mmreng);
 * model 1: two-layer artery layer, neo-Hookean c10/2 (J1-3) plus the
 *          exponential fibre energy k1/(2 k2) sum_{i=4,6} (exp(k2 (J_i-1)^2)-1)
 *          active while J_i > 1, plus kappa/2 (J-1)^2 (eq. areng).
 * theta: the Schur-complement parameter of eq. lpreschur; <= 0 selects
 *        mu^l / 5, mu^l the linear shear modulus of the stabilisation
 *        paragraph (the paper takes theta = O(c10), adjusted by tests on a
 *        coarse mesh and then held fixed; mu^l / 5 needed the fewest Krylov
 *        iterations on the 16^3 cube). */
typedef struct {
  size_t struct_size; /* = sizeof(hfsi_material)                      */
  int32_t model;
  double c10, c01, kappa, k1, k2;
  double theta;
} hfsi_material;

/* Views of the assembled tangent owned by the context; valid until the next
 * assemble, set_* or destroy.  K is block-CSR over nodes with dense 4x4
 * blocks (row-major, rows/cols = components 0..3); A is scalar CSR over the
 * 3n displacement dofs (dof 3*i + c) after Dirichlet elimination. */
typedef struct {
  int32_t n_block_rows;     /* n                                           */
  int32_t n_blocks;         /* stored 4x4 blocks                           */
  const int32_t* block_ptr; /* device [n+1]                                */
  const int32_t* block_col; /* device [n_blocks], ascending per row        */
  const double* block_val;  /* device [n_blocks*16]                        */
  int32_t a_rows;           /* 3n                                          */
  int32_t a_nnz;
  const int32_t* a_ptr;     /* device [3n+1]                               */
  const int32_t* a_col;     /* device [a_nnz]                              */
  const double* a_val;      /* device [a_nnz]                              */
  const double* schur_diag; /* device [n]: (1/theta+1/kappa) diag(M_p)     */
} hfsi_csr_view;

typedef struct {
  size_t struct_size;
  double seconds;       /* assembly wall time on the stream (HIP events)   */
  int32_t n_colours;    /* element colours used for atomic-free assembly   */
  double min_J;         /* smallest element J = det F                      */
} hfsi_assembly_info;

/* AMG parameters.  smoother: 0 = l1-Jacobi, 1 = Chebyshev (polynomial in
 * D^{-1}A over [lmax/cheb_ratio, 1.1 lmax], lmax from 10 Lanczos steps).
 * Smoothing schedule of the V-cycle: on level 0, nu_pre sweeps of degree
 * cheb_degree_pre before the coarse correction and nu_post sweeps of degree
 * cheb_degree after it; on the coarser levels nu_pre_coarse sweeps of degree
 * cheb_degree_pre before and nu_post_coarse sweeps of degree
 * cheb_degree_coarse after (degrees apply to Chebyshev only; a level without
 * pre-smoothing restricts its right-hand side directly).
 * precision: 0 = fp64 V-cycle, 1 = fp32 V-cycle (coarsest solve stays fp64).
 * Coarsening stops at max_coarse rows, after max_levels levels, or when a
 * level would keep more than 90% of its rows (a stall, e.g. on the
 * mass-dominated fluid operator, whose couplings are not strong); the
 * coarsest level is inverted densely when it has at most 4096 rows; a larger
 * coarsest level left by a stall is solved by 16 l1-Jacobi sweeps from zero,
 * one left by max_levels is HFSI_E_CAPACITY.
 * interp: 0 = classical, 1 = learned correction on level 0 (needs MLP
 * weights and lattice coordinates), judged by the convergence factor rho of
 * its V-cycle (10 stationary cycles from the SplitMix64 vector of seed 777):
 * the learned rows are kept only if rho <= fallback_rho and, with
 * judge_classical > 0, the learned hierarchy solves at least as fast as the
 * classical one on the same tangent: on a hierarchy of the assembled tangent
 * the FGMRES rates of hfsi_amg_info.krylov_rho are compared, on one of a
 * caller matrix (hfsi_amg_setup_csr) the V-cycle factors; otherwise the
 * classical hierarchy is built (the fallback). */
typedef struct {
  size_t struct_size;
  double strength_theta; /* default 0.15                                   */
  int32_t max_coarse;    /* default 500                                    */
  int32_t max_levels;    /* default 25                                     */
  uint64_t seed;         /* PMIS weight seed, default 12345                */
  int32_t smoother;
  int32_t nu_pre, nu_post;  /* level 0: sweeps before / after the coarse
                               correction, default 1 / 1                   */
  int32_t precision;
  int32_t interp;
  double fallback_rho;   /* default 0.5                                    */
  int32_t cheb_degree;   /* level-0 post-smoothing degree, 1..8, default 3 */
  double cheb_ratio;     /* lmax / lower bound of the interval, > 1, default 30 */
  int32_t interp_kind;   /* 0 = modified classical (distance one), 1 = extended+i
                            (distance two, De Sterck et al. 2008); the learned
                            correction (interp = 1) adjusts the level-0 row
                            entries inside the 3x3x3 lattice box; default 1 */
  int32_t p_max;         /* extended+i: entries kept per row (largest |w|,
                            rescaled to the row sum), 0 = all, default 4   */
  int32_t cheb_degree_pre;    /* pre-smoothing degree, 1..8, default 1     */
  int32_t nu_post_coarse;     /* post-smoothing sweeps on levels >= 1, default 1 */
  int32_t cheb_degree_coarse; /* their degree, 1..8, default 3             */
  int32_t nu_pre_coarse;      /* pre-smoothing sweeps on levels >= 1, default 0 */
  int32_t judge_classical;    /* learned interpolation only: 0 = threshold
                                 fallback_rho alone; 1 = also compare with the
                                 classical hierarchy's factor on every full
                                 set-up (up to three hierarchy builds); 2 =
                                 compare on the first full set-up of a mesh,
                                 boundary set, material table, weight set and
                                 parameter set, and keep that verdict for the
                                 later set-ups (default)                   */
  double drop_tol;            /* coarse operators: off-diagonal entries with
                                 |a_ij| < drop_tol sqrt(|a_ii a_jj|) of each
                                 Galerkin product are dropped (compared in
                                 float32), in [0, 1), 0 = exact Galerkin
                                 (default); a re-set-up keeps the
                                 set-up's sparsified patterns              */
  int32_t coupled;            /* 0 = AMG on the displacement block inside the
                                 block preconditioner P_L (eq. lpre, default);
                                 1 = the paper's own solid AMG (section "AMG
                                 methods for the mixed problems"): one V-cycle
                                 on the whole tangent K (eq. globsys) replaces
                                 P_L.  Transfer P = diag(P_u, P_p), P_u from
                                 the displacement hierarchy on A, P_p from a
                                 hierarchy built by the same rules on the
                                 pressure block C (the shorter one continues
                                 with the identity), coarse systems P^T K P,
                                 the coarsest inverted densely (at most 4096
                                 unknowns); smoother: the multiplicative Vanka
                                 sweep (eq. locsys, eq. vankasmooth), one patch
                                 per pressure unknown with the displacement
                                 unknowns of its B2 row (at most 2048 per
                                 patch), local LU with partial pivoting, the
                                 patches visited by first-fit colours (in
                                 increasing index on the pattern of K between
                                 patches) and by index within a colour.  Uses
                                 strength_theta, max_coarse, max_levels, seed,
                                 interp_kind and p_max for both hierarchies;
                                 needs interp = 0 and drop_tol = 0; every
                                 set-up and re-set-up builds it anew, in
                                 fp64; precision = 1 rounds the patches'
                                 inverses to fp32 (the local solves read
                                 them in fp32 and accumulate in fp64; half
                                 the bytes of the sweeps' dominant reads).
                                 2 = the same hierarchy with the additive
                                 variant of the Vanka smoother (the paper
                                 mentions an additive form, weights not
                                 fixed): all patches solve with the residual
                                 of the same iterate and every unknown adds
                                 omega times the mean of the corrections of
                                 the patches that hold it (an unknown in no
                                 patch is left unchanged); no colours are
                                 formed                                     */
  double vanka_omega;         /* relaxation omega of eq. vankasmooth, in (0, 2)
                                 (the paper: 0.78 Mooney-Rivlin, 0.86 artery) */
  int32_t vanka_steps;        /* sweeps before and after the coarse correction
                                 on every level, 0..64 (the paper: 6 or 12)  */
} hfsi_amg_params;

typedef struct {
  size_t struct_size;
  int32_t levels;
  int32_t rows[32];      /* rows per level                                 */
  int64_t nnz[32];       /* stored entries per level                       */
  double op_complexity;
  double grid_complexity;
  double seconds;
  double rho;            /* convergence factor measured by the judge (or -1) */
  int32_t learned_used;  /* 1 if the learned level-0 interpolation is kept */
  int32_t pmis_rounds;   /* PMIS rounds summed over levels                 */
  double rho_classical;  /* the classical hierarchy's V-cycle factor (the
                            judge's comparison, measured now or kept from
                            the first set-up), -1 if none                  */
  double krylov_rho;     /* judge on an assembled tangent: the learned
                            hierarchy's FGMRES rate (||r_20||/||r_0||)^(1/20)
                            on K x = b (b a SplitMix64 vector of seed 777,
                            fixed dofs zeroed), -1 if not measured         */
  double krylov_rho_classical; /* the same with the classical hierarchy    */
} hfsi_amg_info;

typedef struct {
  size_t struct_size;
  double tol;           /* relative residual ||b-Kx||/||b||, default 1e-8   */
  int32_t restart;      /* m, default 50 (FGMRES)                          */
  int32_t max_iter;     /* default 500                                     */
  int32_t method;       /* 0 = FGMRES(m) (default), 1 = BiCGStab, the
                           paper's Krylov method for the structure
                           sub-problem (right preconditioning; restart
                           unused), 2 = the AMG method as the solver:
                           x <- x + M^{-1}(b - K x) with the preconditioner
                           of the last set-up (one V-cycle, normally the
                           coupled one) until the tolerance; iterations =
                           V-cycles; 3 = GCR(m), the paper's Krylov method
                           for the fluid sub-problem (right preconditioning,
                           two classical Gram-Schmidt passes, restart m)    */
  int32_t precond_form; /* 0 = P_L (eq. lpre, default); 1 = P_R (eq. rpre):
                           z_p = -Stilde^{-1} r_p, z_u = Atilde^{-1} (r_u -
                           B1^T z_p), with the same Atilde (one V-cycle) and
                           diagonal Stilde; the block forms of the last
                           set-up only (HFSI_E_ARG with the coupled
                           hierarchy)                                      */
} hfsi_solve_params;

typedef struct {
  size_t struct_size;
  int32_t iterations;
  int32_t restarts;
  double rel_residual;  /* true ||b - K x|| / ||b|| at exit                */
  int32_t converged;
  int32_t breakdown;
  double seconds;
} hfsi_solve_info;

typedef struct {
  size_t struct_size;
  hfsi_amg_params amg;
  hfsi_solve_params solve;
  int32_t amg_reuse;    /* 0 = full AMG set-up every step (default); 1 =
                           re-set-up on the coarse grids of the previous
                           set-up of this mesh when there is one (see
                           hfsi_amg_resetup), else a full set-up; 3 = no
                           set-up at all: keep the whole preconditioner of
                           the last set-up that a Newton iteration made on
                           this context while it has the same AMG
                           parameters and stays usable (FGMRES applies the
                           new tangent exactly and only its preconditioner
                           is older).  It is given up, for a set-up as with
                           1, after a Krylov solve with it fails or reduces
                           the residual at under half the mean log rate per
                           iteration of the first solve after its set-up;
                           any other set-up, assembly through the public
                           entry point or change of mesh, conditions,
                           materials, inertia or physics also ends it (new
                           fluid fields, hfsi_set_fluid_fields, do not).  2 = as 1 (in
                           hfsi_newton_solve: also on its first iteration) */
} hfsi_newton_params;

typedef struct {
  size_t struct_size;
  double dv_mass_norm;  /* ||dv||_M, M = diag(M1, M2) consistent masses    */
  double residual_norm; /* ||R||_2 of the state before the update          */
  int32_t krylov_iterations;
  double rel_residual;
  double t_assemble, t_setup, t_solve, t_total;
  int32_t amg_levels;
  int32_t amg_reused;   /* 1 if this step re-used the previous coarse grids,
                           2 if it kept the whole preconditioner          */
} hfsi_newton_info;

typedef struct {
  size_t struct_size;
  hfsi_newton_params step;  /* AMG and Krylov settings of every iteration;
                               step.solve.tol is the inner tolerance when
                               adaptive = 0; step.amg_reuse = 1 keeps the
                               first iteration's coarse grids for the later
                               ones, 2 also starts from the coarse grids of
                               an earlier call on this mesh when there are
                               some (time steps), 3 keeps the whole
                               preconditioner across iterations and calls
                               while it stays usable (hfsi_newton_params) */
  double eps2;              /* stop at ||dv_k||_M <= eps2 ||dv_0||_M (eq.
                               newstop, relative form), default 1e-10       */
  int32_t max_newton;       /* default 25                                   */
  int32_t adaptive;         /* 1: inner tolerance eps_1,k = eps_2,k-1^2 with
                               eps_2,k-1 = ||dv_k-1||_M / ||dv_0||_M (the
                               inexact-Newton rule of Section "Newton's
                               Method"), clamped to [eps1_min, eps1_max];
                               eps1_max for the first iteration             */
  double eps1_max;          /* default 1e-2                                 */
  double eps1_min;          /* default 1e-12                                */
  int32_t line_search;      /* 1: damped Newton: v += a dv with the largest
                               a in {1, 1/2, ..., 1/1024} for which every
                               element keeps J > 0 and the residual decreases,
                               ||R(v + a dv)||_2 <= (1 - 1e-4 a) ||R(v)||_2;
                               the stopping rule needs a full step (a = 1),
                               and a correction that already meets it is
                               taken whole without a search;
                               no admissible a ends the call with
                               HFSI_NOT_CONVERGED and v at the last accepted
                               state.  0: full steps (default)              */
  double ref_norm;          /* > 0: the reference of the relative rule,
                               ||dv_k||_M <= eps2 ref_norm from k = 0 on, in
                               place of ||dv_0||_M (a solve warm-started
                               inside an outer iteration passes the first
                               correction of its first, cold solve); 0 =
                               this call's first correction (default)       */
} hfsi_newton_solve_params;

typedef struct {
  size_t struct_size;
  int32_t newton_iterations;
  int32_t krylov_iterations;  /* summed over the iterations                 */
  int32_t converged;
  double dv_mass_norm[32];    /* ||dv_k||_M of the first 32 iterations      */
  double eps1[32];            /* their inner tolerances                     */
  int32_t krylov[32];         /* their Krylov iterations                    */
  double seconds;             /* wall time of the call                      */
  double step_length[32];     /* their step lengths a (1 without damping; 0:
                                 no admissible step, the call failed there) */
} hfsi_newton_solve_info;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`; `stream` is a hipStream_t (NULL =
 * the null stream) on which every later call queues its work. */
hfsi_status hfsi_create(hfsi_ctx** out, int device, void* stream);
hfsi_status hfsi_destroy(hfsi_ctx* ctx);
const char* hfsi_last_error(const hfsi_ctx* ctx);
int32_t hfsi_abi_version(void);

/* Mesh (Section "Stabilization for the structure sub-problem": P1 elements on
 * a tetrahedral triangulation).  host X [n][3] reference coordinates; host
 * tets [m][4] node indices of positively oriented tetrahedra; host mat_id [m]
 * material index; host lattice [n][3] integer lattice coordinates of each
 * node or NULL (the learned interpolation needs them); host fibres [m][2][3]
 * unit fibre directions a_01, a_02 (eq. arinv46) or NULL for isotropic meshes.
 * Builds geometry, the node-block sparsity pattern and an element colouring.
 * Errors: HFSI_E_ARG on bad sizes, indices or non-positive volumes. */
hfsi_status hfsi_set_mesh(hfsi_ctx* ctx, int64_t n_nodes, const double* X, int64_t n_tets,
                          const int32_t* tets, const int32_t* mat_id, const int32_t* lattice,
                          const double* fibres);

/* Material table (eq. mmreng, eq. areng); host array of n_mat records. */
hfsi_status hfsi_set_materials(hfsi_ctx* ctx, int32_t n_mat, const hfsi_material* mats);

/* Boundary data (eq. elasbnd): host dir_mask [n][4], 1 = dof fixed to zero;
 * host tris [k][3] loaded boundary triangles with host traction [k][3], the
 * dead nominal traction per unit reference area at load factor 1. */
hfsi_status hfsi_set_bc(hfsi_ctx* ctx, const uint8_t* dir_mask, int64_t n_tris, const int32_t* tris,
                        const double* traction);

/* Newmark-beta inertia of the structure (sections "Temporal discretization
 * for the structure sub-problem" and "The time semi-discretized structure
 * weak formulation", and the stabilisation term eq. stelas).  rho = density
 * rho_s (0 turns inertia off: quasi-static, the default and the state after
 * hfsi_set_mesh); beta in (0, 1], gamma in [0, 1], dt > 0 (the paper takes
 * beta = 0.625, gamma = 1).  With inertia on, every assembly adds
 * rho_s/(beta dt^2) (d, v) - (r_s, v) to the displacement rows and
 * tau (r_s - rho_s/(beta dt^2) d, F^{-T} grad q) to the pressure rows, with
 * their exact derivatives, r_s being the P1 history field of the current
 * time step (zero after this call: a body at rest at d = 0).
 * HFSI_E_ARG on bad values. */
hfsi_status hfsi_set_newmark(hfsi_ctx* ctx, double rho, double beta, double gamma, double dt);

/* Start a time step from device state v_prev [N] (its displacement entries
 * are d^{n-1}) and device nodal velocity vel and acceleration acc [n][3]:
 * r_s = rho_s/(beta dt^2) d^{n-1} + rho_s/(beta dt) vel + rho_s (1-2 beta)/(2 beta) acc.
 * HFSI_E_ORDER when inertia is off. */
hfsi_status hfsi_newmark_history(hfsi_ctx* ctx, const double* v_prev, const double* vel, const double* acc);

/* End a time step: with d^n from device v_new [N] and d^{n-1} from v_prev,
 * overwrite device acc [n][3] with (d^n - d^{n-1})/(beta dt^2) - vel/(beta dt)
 * - (1-2 beta)/(2 beta) acc and device vel [n][3] with vel + gamma dt acc^n +
 * (1-gamma) dt acc^{n-1}.  HFSI_E_ORDER when inertia is off. */
hfsi_status hfsi_newmark_update(hfsi_ctx* ctx, const double* v_new, const double* v_prev, double* vel,
                                double* acc);

/* --------------------------------------------------------------- hot path */

/* Residual and consistent tangent at device state v [N] for load factor
 * `load` (eq. stabweakelas, linearised as eq. linsys / eq. globsys).  Writes
 * device R [N] (internal minus external forces, zero on fixed dofs) and the
 * Dirichlet-eliminated K (unit diagonal and zero row/column on fixed dofs),
 * A, B2 and the Schur diagonal into context storage described by *K (may be
 * NULL).  HFSI_E_INVERTED when some element has J <= 0. */
hfsi_status hfsi_assemble_residual_tangent(hfsi_ctx* ctx, const double* v, double load, double* R,
                                           hfsi_csr_view* K, hfsi_assembly_info* info);

/* AMG hierarchy on the displacement block A of the last assembly (the AMG
 * cycles of eq. lpre; Galerkin coarse operators as in "AMG methods for the
 * mixed problems"). */
hfsi_status hfsi_amg_setup(hfsi_ctx* ctx, const hfsi_amg_params* prm, hfsi_amg_info* info);

/* Re-set-up of the hierarchy for the displacement block of the last
 * assembly, keeping the coarse grids of the last hfsi_amg_setup (or Newton
 * step set-up) on this mesh: its C/F splittings and interpolations P (R =
 * P^T, the learned level-0 rows included) are kept, and only the Galerkin
 * coarse operators R A P (as in "AMG methods for the mixed problems"), the
 * smoother data and the coarsest inverse are recomputed.  The smoothing
 * settings and precision come from *prm; its coarsening settings (theta,
 * seed, interp, interp_kind, p_max, drop_tol, level limits) are those of the
 * kept grids and are ignored (the coarse operators keep the set-up's
 * sparsified patterns).  No judge runs (info->rho = -1).  For a sequence of
 * nearby tangents (Newton or time steps) this trades a slower V-cycle for a
 * cheaper set-up.  HFSI_E_ORDER if no set-up of this mesh's tangent is
 * available (a new mesh or boundary data, a set-up from a caller CSR, or a
 * failed set-up discard it). */
hfsi_status hfsi_amg_resetup(hfsi_ctx* ctx, const hfsi_amg_params* prm, hfsi_amg_info* info);

/* Solve K x = b (device b, device x [N]; x is the initial guess on entry)
 * with FGMRES(m) right-preconditioned by P_L^{-1} = [Atilde^{-1} 0;
 * Stilde^{-1} B2 Atilde^{-1}  -Stilde^{-1}] (eq. lpre, eq. lpreschur), Atilde^{-1}
 * one V-cycle of the hierarchy; the Arnoldi basis is orthogonalised by
 * classical Gram-Schmidt with delayed reorthogonalisation (two passes over
 * the basis per step), all fp64; stop at ||b - K x||_2 <= tol ||b||_2 (the
 * true residual decides after every restart cycle).  HFSI_NOT_CONVERGED if
 * max_iter is reached. */
hfsi_status hfsi_krylov_amg_solve(hfsi_ctx* ctx, const double* b, double* x, const hfsi_solve_params* prm,
                                  hfsi_solve_info* info);

/* One Newton iteration at load factor `load` (Section "Newton's Method"):
 * assemble, set up AMG (or re-set it up, prm->amg_reuse), solve K dv = -R,
 * v += dv in place (device v [N]),
 * report ||dv||_M for the stopping rule eq. newstop. */
hfsi_status hfsi_newton_step(hfsi_ctx* ctx, double* v, double load, const hfsi_newton_params* prm,
                             hfsi_newton_info* info);

/* Newton's method at load factor `load` from device state v [N] (updated in
 * place): iterations of hfsi_newton_step until eq. newstop holds in the
 * relative form ||dv_k||_M <= eps2 ||dv_0||_M, with a fixed or an adaptive
 * inner tolerance (Section "Newton's Method"; see
 * hfsi_newton_solve_params).  A first correction at the rounding level of
 * the starting state, ||dv_0||_M <= 1e-14 ||v_0||_M (a time step from an
 * equilibrium at rest, say), is taken whole and ends the increment: the
 * relative rule has no usable reference then.  An iteration whose linear solve stops at
 * step.solve.max_iter is kept (inexact Newton).  HFSI_NOT_CONVERGED when
 * max_newton iterations do not meet the criterion. */
hfsi_status hfsi_newton_solve(hfsi_ctx* ctx, double* v, double load, const hfsi_newton_solve_params* prm,
                              hfsi_newton_solve_info* info);

/* One Newmark-beta time step (inertia on, hfsi_set_newmark): from device
 * state v [N], velocity vel and acceleration acc [n][3] at t^{n-1}, form the
 * history r_s, solve the step's nonlinear problem at load factor `load` with
 * hfsi_newton_solve (prm->step.amg_reuse = 2 keeps the coarse grids of the
 * previous step) and update v, vel and acc in place to t^n.  When Newton
 * does not converge, v, vel and acc are left as they were and
 * HFSI_NOT_CONVERGED is returned; after an error (negative status) v may
 * hold a partial Newton iterate.  HFSI_E_ORDER when inertia is off. */
hfsi_status hfsi_time_step(hfsi_ctx* ctx, double* v, double* vel, double* acc, double load,
                           const hfsi_newton_solve_params* prm, hfsi_newton_solve_info* info);

/* ------------------------------------------- fluid and partitioned FSI */

/* Switch a context to the fluid sub-problem (section "The fluid
 * sub-problem", eq. ns; implicit Euler, eq. nstdis; weak form eq. weakns
 * with SUPG/PSPG stabilisation, eq. stabweakfluid): rho > 0 fluid density,
 * mu >= 0 dynamic viscosity, dt > 0 time step; oseen = 1 takes the
 * previous step's velocity as the convective field, c = u_old - w (the
 * Oseen step, linear in (u, p)), 0 the Navier-Stokes c = u - w.  Needs a
 * mesh (stage 1);
 * set_materials (any valid record: unused by the fluid) and set_bc (dir_mask
 * fixes the velocity dofs with prescribed values, e.g. the interface; the
 * triangles and their traction are the inlet Neumann data g_in at load
 * factor 1) complete it.  The state vector keeps the node-interleaved layout
 * (u_x, u_y, u_z, p).  From then on hfsi_assemble_residual_tangent,
 * hfsi_newton_step and hfsi_newton_solve work on the fluid step on the mesh
 * X + d_f: per tetrahedron, with c = u - w, the strong residual per unit
 * mass r = (u - u_old)/dt + (c.grad)u + grad p/rho and tau =
 * ((2/dt)^2 + (2|c_mean|/h)^2 + (4 mu/(rho h^2))^2)^(-1/2) (c_mean the mean
 * of c over the corners, h the longest current edge),
 *   R^u_a = int [rho (u - u_old)/dt + rho (c.grad)u] N_a
 *           + 2 mu (eps(u), eps(N_a)) - (p, div N_a) + rho tau int (c.grad N_a) r
 *   R^p_a = -(N_a, div u) - tau int grad N_a . r,
 * exact 4-point quadrature, the Jacobian exact at fixed tau, and P_L's
 * Schur diagonal s_i = C_ii + sum_j B2_ij B1^T_ji / A_jj.  The mesh
 * displacement d_f, the previous velocity u_old and the mesh velocity w
 * start at zero (hfsi_set_fluid_fields).  A later hfsi_set_mesh returns the
 * context to the structure.  HFSI_E_ARG on bad values. */
hfsi_status hfsi_set_fluid(hfsi_ctx* ctx, double rho, double mu, double dt, int32_t oseen);

/* Device fields [n][3] of a fluid context, each copied when not NULL: mesh
 * displacement d_f, previous step's velocity u_old (nodal values: the ALE
 * map carries nodes to nodes), mesh velocity w.  HFSI_E_ORDER when the
 * context is not a fluid. */
hfsi_status hfsi_set_fluid_fields(hfsi_ctx* ctx, const double* dmesh, const double* u_old, const double* w);

/* Switch a context (after set_materials) to the P1 Laplacian of its
 * reference mesh on each displacement component (eq. harext): R^u_a =
 * sum_b V (G_a . G_b) d_b, pressure rows empty.  With every boundary node's
 * displacement and every pressure fixed in set_bc, one hfsi_newton_step
 * from a state holding the boundary values leaves the harmonic extension
 * in it. */
hfsi_status hfsi_set_mesh_laplace(hfsi_ctx* ctx);

/* Force device f [count][3] that the fluid exerts on the wall at host
 * nodes [count]: minus the momentum rows of the fluid residual at state v
 * (device [N]) and inlet load factor `load`, before the Dirichlet rows are
 * replaced (by Green's formula that residual is the boundary integral of
 * sigma n_f N_a).  HFSI_E_INVERTED if the moved mesh has an inverted
 * element. */
hfsi_status hfsi_fluid_interface_force(hfsi_ctx* ctx, const double* v, double load, int32_t count,
                                       const int32_t* nodes, double* f);

typedef struct {
  size_t struct_size;
  double omega0;        /* first Aitken factor of the time step, > 0; a
                           caller may carry the last factor of the previous
                           step, info.omega[dn_iterations - 2]           */
  double eps;           /* stop at |r_k| / sqrt(n_iface) < eps (the paper: 1e-8) */
  int32_t max_dn;       /* at most this many DN iterations, 1..128          */
  double eps2;          /* the nested Newton rule eq. newstop, e.g. 1e-10   */
  hfsi_newton_params fluid_step;  /* AMG and Krylov settings of the fluid  */
  hfsi_newton_params solid_step;  /* ... of the structure                  */
  hfsi_newton_params mesh_step;   /* ... of the harmonic extension (one
                                     linear solve per DN iteration)         */
  int32_t adaptive;     /* 1: the nested fluid and structure Newton solves
                           take the adaptive inner tolerance (see
                           hfsi_newton_solve_params.adaptive, with eps1_max
                           1e-2 and eps1_min 1e-12); 0: the fixed tolerance
                           of fluid_step / solid_step (default)             */
} hfsi_fsi_params;

typedef struct {
  size_t struct_size;
  int32_t dn_iterations;
  int32_t converged;
  int32_t fluid_newton;   /* Newton iterations summed over the DN iterations */
  int32_t solid_newton;
  int32_t krylov;         /* Krylov iterations of all nested solves          */
  double residual[128];   /* |r_k| / sqrt(n_iface) of DN iteration k+1      */
  double omega[128];      /* the factor applied after DN iteration k+1       */
  double seconds;
} hfsi_fsi_info;

/* One time step of the partitioned FSI problem by the Dirichlet-Neumann
 * iteration (section "A Dirichlet-Neumann FSI iteration") with Aitken
 * relaxation (eq. acceit, eq. dnomega).  Contexts: `fluid` (hfsi_set_fluid,
 * velocity fixed on the interface), `mesh` (hfsi_set_mesh_laplace on the
 * same fluid mesh, every boundary displacement and every pressure fixed),
 * `solid` (a structure with Newmark inertia, hfsi_set_newmark, its step
 * equal to the fluid's dt); host iface_f / iface_s [n_iface]: the interface
 * nodes in fluid and structure numbering, pairwise the same points.  Device
 * state at t^{n-1}, advanced in place to t^n: vf [4 nf] fluid (u, p), df
 * [nf][3] mesh displacement, vs [4 ns], vel, acc [ns][3] structure.  Each
 * DN iteration extends the interface displacement d_G harmonically into the
 * fluid mesh (mesh velocity w = (d_f - d_f^{n-1})/dt), solves the fluid with
 * u = w on the interface and the inlet traction scaled by inlet_load, takes
 * the fluid's force on the wall as the structure's nodal load and solves the
 * structure; r_k = d_G(structure) - d_G, stop when |r_k|/sqrt(n_iface) <
 * eps, else d_G += omega_k r_k with omega from eq. dnomega (omega0 first).
 * The first d_G is the structure's interface displacement extrapolated to
 * t^n with its velocity, d^{n-1} + dt vel^{n-1}; every
 * nested Newton solve continues from its latest iterate with the rule of
 * eq. newstop relative to the first correction of its sub-problem in this
 * step (hfsi_newton_solve_params.ref_norm).  The contexts' streams are
 * synchronised at every hand-over.  HFSI_NOT_CONVERGED after max_dn
 * iterations (state partly advanced); a failing nested solve returns its
 * status with the sub-problem and the DN iteration named in
 * hfsi_last_error(fluid), and info holds the iterations up to it. */
hfsi_status hfsi_fsi_time_step(hfsi_ctx* fluid, hfsi_ctx* mesh, hfsi_ctx* solid, int32_t n_iface,
                               const int32_t* iface_f, const int32_t* iface_s, double* vf, double* df, double* vs,
                               double* vel, double* acc, double inlet_load, const hfsi_fsi_params* prm,
                               hfsi_fsi_info* info);

/* ------------------------------------------------ inspection and testing */

/* AMG setup on a caller-given scalar CSR matrix instead of the assembled A
 * (host arrays; comp [n] the unknown component of each row).  Used to feed
 * identical inputs to the GPU and the CPU oracle level by level. */
hfsi_status hfsi_amg_setup_csr(hfsi_ctx* ctx, int32_t n, const int32_t* ptr, const int32_t* col,
                               const double* val, const int32_t* comp, const hfsi_amg_params* prm,
                               hfsi_amg_info* info);

/* Copy level `level` of the current hierarchy to host buffers.  which: 0 = A
 * (ptr [rows+1], col, val), 1 = P, 2 = strength flags (u8 per A entry, in
 * val_u8), 3 = C/F state (int8 per row in val_u8: +1 C, -1 F), 4 = component
 * per row (int32 in col).  Of the coupled hierarchy (coupled = 1 or 2): 10 = Kuu
 * (the displacement block A of the level), 11 = Kup (B1^T), 12 = Kpu (B2),
 * 13 = Kpp (-C), each as CSR; 14 = the Vanka colour of every patch (int32
 * per pressure unknown in col, the colour count in *cols); 15 = P_u, 16 =
 * P_p (HFSI_E_ARG where the transfer is the identity, on the coarsest
 * level, and for 14 with the additive variant).  Pass NULL buffers to query
 * sizes in *rows, *cols, *nnz. */
hfsi_status hfsi_amg_export(hfsi_ctx* ctx, int32_t level, int32_t which, int32_t* rows, int32_t* cols,
                            int64_t* nnz, int32_t* ptr, int32_t* col, double* val, uint8_t* val_u8);

/* One V-cycle z = Atilde^{-1} r on device vectors of length rows(level 0),
 * in the hierarchy's precision (inputs and outputs fp64). */
hfsi_status hfsi_vcycle(hfsi_ctx* ctx, const double* r, double* z);

/* y = M^{-1} r with the preconditioner of the last set-up (P_L^{-1} of
 * eq. lpre, or one V-cycle of the coupled hierarchy when it was set up with
 * coupled = 1 or 2) and y = K x (device [N]). */
hfsi_status hfsi_apply_preconditioner(hfsi_ctx* ctx, const double* r, double* y);
hfsi_status hfsi_apply_tangent(hfsi_ctx* ctx, const double* x, double* y);

/* Copy the last assembled tangent to host buffers (any may be NULL): the
 * block pattern and values of K (sizes from hfsi_csr_view: n+1, n_blocks,
 * 16*n_blocks), the CSR of A (3n+1, a_nnz, a_nnz) and the Schur diagonal (n). */
hfsi_status hfsi_export_tangent(hfsi_ctx* ctx, int32_t* block_ptr, int32_t* block_col, double* block_val,
                                int32_t* a_ptr, int32_t* a_col, double* a_val, double* schur);

/* ||dv||_M for a device vector dv [N]. */
hfsi_status hfsi_mass_norm(hfsi_ctx* ctx, const double* dv, double* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * ||dv||_M as hfsi_mass_norm, written to the device scalar `out` (fp64, [1],
 * caller-owned) with neither an allocation nor a host wait.  The block
 * partial sums live in a fixed file-scope device array of 256 doubles (2 KiB
 * per GPU, held until the process ends, independent of the mesh size, so no
 * input exceeds it); every call on one GPU shares that array, and calls that
 * overlap on one GPU (several streams or threads at once) race on it.  The
 * result is ready when the context's stream reaches the call.  HFSI_E_ORDER
 * before hfsi_set_mesh, HFSI_E_ARG for a null pointer. */
hfsi_status hfsi_mass_norm_noalloc(hfsi_ctx* ctx, const double* dv, double* out);

/* ------------------------------------------------ learned interpolation */

/* The learned level-0 interpolation (no counterpart in the paper, whose AMG
 * uses its own coarsening): a 64-64-64-27 network with ReLU, weights and
 * activations in bfloat16 on MFMA with fp32 accumulation, adds a correction
 * to the classical weights w_ij of the strong C points of every F point, by
 * the slot of j in the 3x3x3 lattice box of node(i).  Inputs: the
 * same-component couplings a_ij/a_ii in the box, the C flags, log10(kappa)/6,
 * two material constants and the one-hot component.  With a zero last layer
 * the result equals classical interpolation exactly.
 *
 * Parameters are one host fp32 array of HFSI_MLP_NPARAM values: W1 [64x64]
 * (row = input), b1 [64], W2 [64x64], b2 [64], W3 [64x32] (columns 27..31
 * unused), b3 [32].  The context keeps fp32 master weights, their bf16 copy
 * and the Adam moments. */
#define HFSI_MLP_NPARAM 10400

typedef struct {
  size_t struct_size;
  int32_t batch;                 /* samples per Adam step                  */
  double lr, beta1, beta2, eps;  /* Adam (Kingma & Ba 2015)                */
} hfsi_train_params;

typedef struct {
  size_t struct_size;
  int64_t samples;               /* training-set size                      */
  double loss_first, loss_last;  /* masked MSE of the first / last batch   */
  int32_t steps;
  double seconds;
} hfsi_train_info;

hfsi_status hfsi_mlp_set_weights(hfsi_ctx* ctx, const float* w /* host [HFSI_MLP_NPARAM] */);

/* Weights from / to a raw checkpoint file (little endian): the 8 bytes
 * "HFSIMLP" plus a zero byte, int32 version (1), int32 parameter count
 * (HFSI_MLP_NPARAM), the fp32 parameters in the layout above, and the uint64
 * FNV-1a hash of those parameter bytes.  Load replaces the weights as
 * hfsi_mlp_set_weights does (Adam moments reset); HFSI_E_ARG when the file
 * cannot be read or its magic, version, count or hash is wrong (the
 * weights are then unchanged).  Save writes the current weights;
 * HFSI_E_ORDER before any weights are set, HFSI_E_ARG when the file cannot
 * be written. */
#define HFSI_MLP_FILE_VERSION 1
hfsi_status hfsi_mlp_load(hfsi_ctx* ctx, const char* path);
hfsi_status hfsi_mlp_save(hfsi_ctx* ctx, const char* path);
hfsi_status hfsi_mlp_get_weights(hfsi_ctx* ctx, float* w /* host [HFSI_MLP_NPARAM] */);
/* host m [HFSI_MLP_NPARAM] and v: Adam moments; *step: Adam steps taken */
hfsi_status hfsi_mlp_adam_state(hfsi_ctx* ctx, float* m, float* v, int64_t* step);

/* Network output for m host feature rows X [m][64] -> host out [m][32] (fp32);
 * optional host copies of the bf16 input and hidden activations [m][64]. */
hfsi_status hfsi_mlp_forward(hfsi_ctx* ctx, int32_t m, const float* X, float* out, uint16_t* x_bf16,
                             uint16_t* h1_bf16, uint16_t* h2_bf16);

/* Masked MSE loss sum(mask (wcl + out - wstar)^2) / sum(mask) of m host rows
 * (mask, wcl, wstar [m][32]) and its gradient (host [HFSI_MLP_NPARAM]). */
hfsi_status hfsi_mlp_loss_grad(hfsi_ctx* ctx, int32_t m, const float* X, const float* mask, const float* wcl,
                               const float* wstar, float* grad, double* loss);

/* Append the level-0 samples of the current classical hierarchy (needs
 * lattice coordinates) to the context's training set: features, mask,
 * classical weights and the local ideal-interpolation target.  *n_failed
 * counts samples whose local system was singular or too large (target 0). */
hfsi_status hfsi_mlp_collect(hfsi_ctx* ctx, int32_t* n_added, int32_t* n_failed);
/* The same for a seeded subset (large meshes): the sample of level-0 row r
 * is kept when the top 53 bits of SplitMix64 output r of the stream `seed`,
 * divided by 2^53, are below `fraction` (in (0, 1], else HFSI_E_ARG); the
 * kept samples are appended in increasing row order. */
hfsi_status hfsi_mlp_collect_sampled(hfsi_ctx* ctx, double fraction, uint64_t seed, int32_t* n_added,
                                     int32_t* n_failed);
hfsi_status hfsi_mlp_clear(hfsi_ctx* ctx);
/* Copy rows [first, first+count) of the training set to host arrays (any may
 * be NULL); *total receives the set size. */
hfsi_status hfsi_mlp_samples(hfsi_ctx* ctx, int64_t first, int64_t count, int64_t* total, float* X, float* mask,
                             float* wcl, float* wstar);

/* Adam training on the collected set: host order [n_order] lists the sample
 * of every position (epochs x permutation, chosen by the caller); one step
 * per `batch` consecutive positions. */
hfsi_status hfsi_mlp_train(hfsi_ctx* ctx, const hfsi_train_params* prm, const int32_t* order, int64_t n_order,
                           hfsi_train_info* info);

/* Convergence factor of the current hierarchy: rho = (||e_k||_A/||e_0||_A)^(1/k)
 * for k stationary V-cycles e <- e - V(A e) from the SplitMix64 vector of
 * `seed` (stream 0, values in [-1,1)). */
hfsi_status hfsi_amg_convergence_factor(hfsi_ctx* ctx, int32_t cycles, uint64_t seed, double* rho);

/* ------------------------------------------------------------ measurement */

/* Launch one hot-path kernel `reps` times back to back on the context stream,
 * bracketed by HIP events, and report the average duration of one launch in
 * *avg_ms and the algorithmic bytes one launch must move in *bytes (the
 * minimum traffic of its inputs and outputs).  kernel:
 *   0 = level-0 smoother sweep (hierarchy precision), 1 = level-0 residual,
 *   100 + l = smoother sweep on level l, 200 + l = residual on level l
 *   (HFSI_E_ARG if the hierarchy has no level l),
 *   2 = tangent SpMV y = K x (fp64 4x4 blocks), 3 = element assembly
 *   (all colours), 9 = plain device copy of `bytes_hint` bytes (counter
 *   calibration).  Needs the state the kernel reads (assembled K, hierarchy).
 * For kernels 0, 1, 2, 100 + l and 200 + l with bytes_hint > 0, consecutive
 * launches cycle through copies of the operator (temporary device memory)
 * that together hold at least bytes_hint bytes (at most 16 copies): above the
 * 256 MB last-level cache each launch then reads its operator from HBM.
 * bytes_hint = 0 times repeated launches on the one operator.
 * Work buffers are context-owned; results are discarded, except that kernel
 * 3 leaves the zero-state tangent in the context (assemble again after it). */
hfsi_status hfsi_time_kernel(hfsi_ctx* ctx, int32_t kernel, int32_t reps, int64_t bytes_hint, double* avg_ms,
                             double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* HFSI_H */
