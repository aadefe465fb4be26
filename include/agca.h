/*
 * agca.h -- C ABI of the AGCA multigrid library for MI355X (gfx950).
 *
 * Adaptive Galerkin coarse-grid approximation (AGCA) multigrid for the
 * variable-coefficient P1 operators of "Large-scale multigrid with adaptive
 * Galerkin coarsening" (Boehm, Kohl, Koestler, Ruede):
 *   - scalar diffusion      -div(nu grad u) = f                  (ncomp = 1)
 *   - vector viscous block  -div(2 nu eps(u)) = f, eq. (3.1)/(3.5) (ncomp = 3)
 * on the unit cube with homogeneous Dirichlet data, discretised on the
 * uniformly refined 48-tetrahedron macro grid (2x2x2 cubes, 6 tets each along
 * the (1,1,1) diagonal), Section 2.1, eq. (2.2).
 *
 * Grid and numbering (all levels l = 0..L, n_l = 2^(l+1) cells per axis):
 *   node  p = x + (n+1) (y + (n+1) z),        0 <= x,y,z <= n
 *   elem  e = s + 6 (cx + n (cy + n cz)),     0 <= cx,cy,cz < n
 *   where s = 0..5 is the axis order of the element's three unit steps from
 *   its lowest corner: 0 xyz, 1 xzy, 2 yxz, 3 yzx, 4 zxy, 5 zyx.
 *   Uniform (Bey) refinement maps element (C, s) to 8 children in the cubes
 *   2C + {0, e_a1, e_a1 + e_a2, (1,1,1)}.
 *
 * Vectors ("level vectors") are SoA: ncomp blocks of (n_l+1)^3 values,
 * component-major, one slot per lattice node including the boundary.
 * Boundary slots are ignored on input and written as 0 on output.
 * Coefficients are one value per element (P0), indexed by element id.
 *
 * Memory and streams: every pointer documented "device" is device memory owned
 * by the caller (for example a contiguous torch tensor's data pointer).  The
 * library copies the coefficients it keeps; it owns flags, Galerkin blocks,
 * diagonals and work vectors.  Work is enqueued on the HIP stream given to
 * agca_create.  apply / residual / smooth / restrict / prolong_add / vcycle /
 * cast / grad / load_vector are asynchronous; create, set_nu, query, get_*,
 * dot and solve synchronise that stream.
 *
 * Errors: every function returns an agca_status and never aborts or throws
 * across the ABI.  A message describing the last error of the calling thread
 * is available from agca_last_error().  After AGCA_E_HIP the hierarchy refuses
 * further work with AGCA_E_STATE.
 */
#ifndef AGCA_H
#define AGCA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AGCA_OK = 0,
    AGCA_E_INVALID = -1, /* bad argument, config or coefficient (non-finite or <= 0) */
    AGCA_E_OOM = -2,     /* device allocation failed or mem_limit_bytes exceeded      */
    AGCA_E_HIP = -3,     /* a HIP runtime call failed                                 */
    AGCA_E_NOCONV = -4,  /* solver stopped at max_iter; x and stats are still filled   */
    AGCA_E_NUMERIC = -5, /* solver saw a non-finite or exploding residual             */
    AGCA_E_STATE = -6    /* hierarchy is in an error state                            */
} agca_status;

typedef enum { AGCA_F64 = 0, AGCA_F32 = 1, AGCA_BF16 = 2 } agca_dtype;

/* Coarse-operator selection (Section 2.3).
 *  RATIO : a level-l element (l < L) uses its stored Galerkin block when the
 *          maximum of the finest coefficient over its finest descendants exceeds
 *          flag_ratio times the minimum (strict, FP64); DCA otherwise.
 *  MACRO : the paper's macro granularity (eqs. (2.8)-(2.9)): every coarse element
 *          inside a macro element k (level-0 element id k, 0..47) with
 *          macro_flags[k] != 0 uses its stored Galerkin block, every other one
 *          DCA.  agca_macro_gradient() gives the gradient test of (2.8).
 *  NONE  : DCA on every coarse element (eq. (2.5)).
 *  ALL   : Galerkin blocks on every coarse element (eqs. (2.6)-(2.7)). */
enum { AGCA_FLAG_RATIO = 0, AGCA_FLAG_MACRO = 1, AGCA_FLAG_NONE = 2, AGCA_FLAG_ALL = 3 };

/* How a flagged element's Galerkin operator is kept.
 *  BLOCKS : its 4 ncomp x 4 ncomp Galerkin block (eq. (2.7)), computed in FP64 from
 *           the finest coefficient (plus an FP32 copy for the FP32 V-cycle).
 *  MEAN   : one scalar: with P1 functions the block equals the element's DCA matrix
 *           with the arithmetic mean of the finest coefficient over its descendants,
 *           so that mean replaces the element's coarse coefficient and nothing else is
 *           stored (the same operator up to rounding; agca_get_blocks then fails). */
enum { AGCA_STORE_BLOCKS = 0, AGCA_STORE_MEAN = 1 };

/* Smoother of the V-cycle.
 *  JACOBI    : damped Jacobi, pre_sweeps / post_sweeps sweeps with damping omega.
 *  CHEBYSHEV : the Chebyshev polynomial smoother of Section 4, degree pre_sweeps /
 *              post_sweeps: the Chebyshev iteration for D^-1 A on
 *              [lambda_max / 10, lambda_max], lambda_max = 1.1 x an estimate per level
 *              formed at setup (the largest Ritz value of 20 Lanczos steps for the
 *              pencil (A, D) from (-1)^(X+Y+Z) on the free nodes, in FP64; a lower
 *              bound of the eigenvalue).  omega is not used. */
enum { AGCA_SMOOTH_JACOBI = 0, AGCA_SMOOTH_CHEBYSHEV = 1 };

typedef struct {
    int32_t L;               /* finest level, 1 <= L <= 9                                  */
    int32_t ncomp;           /* 1 or 3                                                      */
    int32_t flag_mode;       /* AGCA_FLAG_*                                                 */
    int32_t mg_dtype;        /* AGCA_F64 or AGCA_F32: precision of the V-cycle, its stored
                                blocks, diagonals and work vectors                          */
    int32_t mg_nu_dtype;     /* AGCA_F64, AGCA_F32 or AGCA_BF16: finest-level coefficient
                                copy used by the V-cycle (must not be wider than mg_dtype)  */
    int32_t pre_sweeps;      /* smoothing passes before / after the coarse correction; the
                                CG-type solvers (PCG, FCG) need pre_sweeps == post_sweeps:
                                the V-cycle is a symmetric preconditioner only then        */
    int32_t post_sweeps;
    int32_t smoother;        /* AGCA_SMOOTH_*                                               */
    double flag_ratio;       /* tau (10 in the paper's experiments)                         */
    double omega;            /* Jacobi damping (2/3)                                        */
    uint64_t mem_limit_bytes;/* 0 = unlimited; larger totals fail with AGCA_E_OOM           */
    uint8_t macro_flags[48]; /* AGCA_FLAG_MACRO: nonzero = Galerkin-coarsen that macro element */
    int32_t coarse_storage;  /* AGCA_STORE_*                                                */
} agca_config;

typedef struct {
    int64_t n;               /* cells per axis                                              */
    int64_t nodes;           /* (n+1)^3                                                     */
    int64_t free_nodes;      /* (n-1)^3                                                     */
    int64_t elements;        /* 6 n^3                                                       */
    int64_t flagged;         /* elements with a stored Galerkin block (0 on level L)        */
    int64_t block_bytes;     /* bytes of stored Galerkin blocks on this level               */
    int64_t level_bytes;     /* all device bytes the library holds for this level           */
    double lambda_max;       /* Chebyshev: the eigenvalue estimate of D^-1 A (0 otherwise)  */
} agca_level_info;

typedef struct agca_hier agca_hier;

/* Fill a config with the defaults: L = 3, scalar, ratio flags, tau = 10,
 * FP64 V-cycle, V(2,2) damped Jacobi with omega = 2/3.  Host only. */
void agca_default_config(agca_config* cfg);

/* Check a config without touching the device.  Host only. */
int32_t agca_validate_config(const agca_config* cfg);

/* Build the hierarchy (Sections 2.1-2.3): copy the coefficients, check them
 * (finite, > 0), flag coarse elements, form the local Galerkin blocks of the
 * flagged elements by the element-wise recursion (2.7) in FP64, and the Jacobi
 * diagonals and the coarsest-level inverse.
 *   nu_fine   : device, 6 n_L^3 doubles, finest-level coefficient by element id.
 *   nu_coarse : host array of L device pointers; nu_coarse[l] holds 6 n_l^3
 *               doubles, the coefficient evaluated on level l for DCA (eq. (2.5)).
 *   stream    : hipStream_t (NULL = default stream).
 * On success *out receives the handle; free it with agca_destroy. */
int32_t agca_create(const agca_config* cfg, const double* nu_fine,
                    const double* const* nu_coarse, void* stream, agca_hier** out);

int32_t agca_destroy(agca_hier* h);

/* Replace the coefficients and rebuild flags, blocks and diagonals. */
int32_t agca_set_nu(agca_hier* h, const double* nu_fine, const double* const* nu_coarse);

/* agca_set_nu with the finest coefficient given as log nu (device, 6 n_L^3 doubles in
 * element-id order, exponentiated on the device); nu_coarse as in agca_create.  This
 * is the parameterisation of the adjoint gradient (agca_grad_log_nu): the gradient is
 * taken with respect to these values.  Errors as agca_set_nu (AGCA_E_INVALID when
 * exp(log nu) is not finite and positive). */
int32_t agca_set_log_nu(agca_hier* h, const double* log_nu_fine, const double* const* nu_coarse);

int32_t agca_query(const agca_hier* h, int32_t level, agca_level_info* out);

/* Sorted ids of the flagged elements of a coarse level (host buffer of cap
 * entries); *n receives the count even when cap is too small (then AGCA_E_INVALID). */
int32_t agca_get_flags(const agca_hier* h, int32_t level, int32_t* ids_host, int64_t cap,
                       int64_t* n);

/* FP64 Galerkin blocks of a coarse level, in flagged-id order: flagged x
 * (4 ncomp)^2 doubles, row (c, a) = 4 c + a, column (d, b) = 4 d + b, vertices a,b
 * in path order (lowest corner first).  Host buffer of cap doubles. */
int32_t agca_get_blocks(const agca_hier* h, int32_t level, double* blocks_host, int64_t cap);

/* Jacobi diagonal of a level operator, FP64, as a host level vector (0 on the boundary). */
int32_t agca_get_diagonal(const agca_hier* h, int32_t level, double* diag_host, int64_t cap);

/* v = A_l u (eq. (2.3) on the finest level, eq. (2.9) on coarser levels).
 * dtype AGCA_F64 uses the FP64 coefficients and blocks; AGCA_F32 needs
 * mg_dtype == AGCA_F32 and uses the V-cycle's copies.  u, v: device level vectors. */
int32_t agca_apply(agca_hier* h, int32_t level, int32_t dtype, const void* u, void* v);

/* r = b - A_l x. */
int32_t agca_residual(agca_hier* h, int32_t level, int32_t dtype, const void* b,
                      const void* x, void* r);

/* sweeps of damped Jacobi x <- x + omega D^-1 (b - A_l x), in place on x. */
int32_t agca_smooth(agca_hier* h, int32_t level, int32_t dtype, int32_t sweeps, double omega,
                    const void* b, void* x);

/* r_c = P^T r_f with P the linear interpolation from level fine_level-1 (Section 2.1). */
int32_t agca_restrict(agca_hier* h, int32_t fine_level, int32_t dtype, const void* r_f,
                      void* r_c);

/* x_f += P e_c, from level coarse_level to coarse_level+1. */
int32_t agca_prolong_add(agca_hier* h, int32_t coarse_level, int32_t dtype, const void* e_c,
                         void* x_f);

/* x = B b: one V(pre,post)-cycle on level L from a zero initial guess, in the
 * hierarchy's mg_dtype (dtype must equal it).  b, x: device level vectors. */
int32_t agca_vcycle(agca_hier* h, int32_t dtype, const void* b, void* x);

/* Deterministic reduction: *out = sum over all slots of x * y (FP64 accumulation). */
int32_t agca_dot(agca_hier* h, int32_t level, int32_t dtype, const void* x, const void* y,
                 double* out);

/* Elementwise precision conversion with round-to-nearest-even:
 * F64 -> F32, F32 -> F64, F64 -> BF16 (BF16 stored as uint16). count elements. */
int32_t agca_cast(agca_hier* h, int32_t from, int32_t to, const void* src, void* dst,
                  int64_t count);

enum { AGCA_SOLVER_PCG = 0, AGCA_SOLVER_FCG = 1, AGCA_SOLVER_IR = 2, AGCA_SOLVER_STATIONARY = 3 };

#define AGCA_MAX_MILESTONES 8
typedef struct {
    int32_t solver;          /* AGCA_SOLVER_*                                              */
    int32_t max_iter;
    double tol;              /* stop when ||b - A x||_2 <= tol ||b||_2 (eq. (4.3))          */
    int32_t use_x0;          /* 0: start from x = 0; 1: start from the given x              */
    int32_t record_history;  /* store the relative residual of every iteration             */
    int32_t n_milestones;    /* 0..AGCA_MAX_MILESTONES (PCG and FCG only)                  */
    double milestones[AGCA_MAX_MILESTONES]; /* tolerances above tol: the solve records when
                                the true residual first falls below each (checked, like the
                                final stop, by a residual replacement when the recurrence
                                crosses it), so one solve gives several times to tolerance */
} agca_solve_opts;

#define AGCA_MAX_HISTORY 1024
typedef struct {
    int32_t iterations;
    int32_t converged;       /* the true FP64 residual of x is <= tol                       */
    int32_t floor_limited;   /* PCG/FCG: the true residual stopped improving above tol
                                and is at most max(tol, floor_estimate): FP64 rounding of
                                x, not the solver, limits it (Stokes FGMRES: see
                                agca_stokes_solve)                                          */
    int32_t replacements;    /* times the true residual replaced the recurrence's           */
    double rel_residual;     /* final ||b - A x|| / ||b|| in FP64 with FP64 coefficients,
                                norms over the free dofs                                    */
    double recursive_rel_residual; /* the Krylov recurrence's last residual estimate        */
    double floor_estimate;   /* agca_solve: rounding floor rho of the returned x
                                (agca_residual_floor); Stokes FGMRES: the velocity block's
                                part at the last floor test (0 if none ran)                 */
    double seconds;          /* wall time of the solve (after setup)                        */
    int32_t milestone_iterations[AGCA_MAX_MILESTONES]; /* iteration at which the true
                                residual was first found <= milestones[i]; -1 if never      */
    double milestone_seconds[AGCA_MAX_MILESTONES];     /* solve wall time at that point     */
    double milestone_residuals[AGCA_MAX_MILESTONES];   /* the true relative residual there  */
    double history[AGCA_MAX_HISTORY]; /* recurrence residuals, one per iteration           */
} agca_solve_stats;

/* Solve A_L x = b with the AGCA V-cycle as preconditioner inside an FP64 outer
 * loop (PCG for an FP64 V-cycle; FCG(1) or iterative refinement around an FP32
 * V-cycle; stationary V-cycle iteration).  PCG and FCG run one loop whose new search
 * direction is A-orthogonalised against the previous one (beta = -z.q / p.q), which
 * for PCG equals the textbook z.r / rz_old in exact arithmetic and stays conjugate
 * after residual replacements.  b, x: device FP64 level vectors (boundary
 * slots of b are ignored; norms are taken over the free dofs).
 * Stopping (eq. (4.3)): PCG and FCG replace their recurrence's residual by the true
 * residual b - A x whenever the recurrence has halved since the last replacement, and
 * when it reaches tol (the search direction is kept).  They stop when the true residual
 * is <= tol (converged), or when it has stopped improving (two windows in a row
 * without a 10 % gain over its best, a window being the iterations the recurrence last
 * took to halve) and is at most max(tol, rho), rho the rounding floor of x
 * (agca_residual_floor): floor_limited.  A stalled solve above that level keeps
 * checking at each later replacement and gives up after six windows without progress.
 * Returns AGCA_OK when converged or floor_limited; AGCA_E_NOCONV (x and stats filled)
 * when max_iter is reached first or the true residual stalls above max(tol, rho). */
int32_t agca_solve(agca_hier* h, const agca_solve_opts* opts, const double* b, double* x,
                   agca_solve_stats* stats);

/* Rounding floor of the relative residual of x (stopping test of eq. (4.3) in FP64):
 *   *rho = u || |b| + sum_e |A_e| |x_e| ||_2 / ||b||_2,   u = 2^-53,
 * norms over the free dofs of level L, |A_e| the entrywise absolute element matrix of
 * the finest operator.  Rounding each entry of x once more moves b - A x by at most
 * u sum_e |A_e| |x_e| entrywise, so relative residuals much below rho cannot be
 * certified for an FP64 iterate near x.  b, x: device FP64 level vectors on level L
 * (boundary slots ignored).  Synchronises the stream.  *rho = 0 when b = 0 on the
 * free dofs. */
int32_t agca_residual_floor(agca_hier* h, const double* b, const double* x, double* rho);

/* Adjoint gradient (not in the paper): g_e = -w_e^T A_e u_e for every finest
 * element, i.e. dJ/dlog nu_e when w solves A w = u - u_obs.
 * u, w: device FP64 level vectors on level L; g: device, 6 n_L^3 doubles. */
int32_t agca_grad_log_nu(agca_hier* h, const double* u, const double* w, double* g);

/* ---- Generalized Stokes (Section 3.1, eqs. (3.1)-(3.5)) --------------------------
 * Velocity: this hierarchy's finest level L (ncomp = 3, P1-iso-P2); pressure: P1 on
 * every node of level L-1 (no pressure boundary condition), (n_{L-1}+1)^3 doubles.
 * B = -integral psi_k div Phi_j (the sign that makes [[A, B^T], [B, 0]] symmetric),
 * formed as -P^T B_L: psi_k is linear on each level-L simplex, so its integral
 * against the constant divergence is |d| times its mean vertex value.  All
 * pointers are device FP64 vectors; velocity boundary slots are ignored on input
 * and written as 0.  Errors: AGCA_E_INVALID for ncomp != 3 or L < 2. */

/* q = B u (u: velocity level vector; q: pressure vector). */
int32_t agca_stokes_div(agca_hier* h, const double* u, double* q);

/* v = B^T p (p: pressure vector; v: velocity level vector, overwritten). */
int32_t agca_stokes_grad(agca_hier* h, const double* p, double* v);

/* m = lumped pressure mass weighted by 1/nu: m_k = sum_d |d| / nu_d psi_k(centroid_d),
 * d over the level-L simplices (the pressure block of the preconditioner). */
int32_t agca_stokes_mass(agca_hier* h, double* m);

typedef enum { AGCA_STOKES_FGMRES = 0, AGCA_STOKES_MINRES = 1 } agca_stokes_solver;
/* DIAGONAL   : diag(V-cycle, S^-1).
 * TRIANGULAR : the upper block-triangular preconditioner of eq. (4.1) with the same
 *              blocks, [[V, V B^T S^-1], [0, -S^-1]] (the sign of the pressure block
 *              for which exact blocks make the preconditioned matrix unipotent);
 *              FGMRES only.
 * S approximates the positive Schur complement B A^-1 B^T (agca_stokes_schur). */
typedef enum { AGCA_STOKES_DIAGONAL = 0, AGCA_STOKES_TRIANGULAR = 1 } agca_stokes_precond;
/* The Schur approximation S in either preconditioner:
 * MASS : S = diag(m), the 1/nu-weighted lumped pressure mass.
 * BFBT : the diag(A)-BFBT least-squares commutator of eq. (4.2),
 *        S^-1 = Z^-1 (B W^-1 A W^-1 B^T) Z^-1, W = diag(A), Z = B W^-1 B^T, where each
 *        Z^-1 is schur_iters steps of Jacobi-preconditioned CG on Z from zero (a step
 *        of zero Z-energy has step size zero).  diag(Z) is formed exactly at the first
 *        solve after every coefficient rebuild (27 products with Z, one per colour of
 *        the nodes by coordinates mod 3).  Not linear in r: FGMRES only.
 * BFBT_MG : the same S^-1 with each Z^-1 being schur_iters steps of CG on Z from zero
 *        preconditioned by one V-cycle of a geometric multigrid for Z (the paper uses
 *        an algebraic multigrid cycle there): levels L-1 (the pressure space) down to
 *        0 with the linear interpolation P over all nodes, Galerkin operators
 *        Z_l = P^T Z_{l+1} P, each stored as a stencil over the 65 offsets o in
 *        [-2,2]^3 with max(o,0) - min(o,0) <= 2 (sums of two Kuhn edges: every
 *        coupling of Z and of its Galerkin coarsenings), damped Jacobi V(2,2) cycles
 *        with omega = 2/3 from zero, and on level 0 (27 nodes) the minimal-norm
 *        solution (bordered system [[Z_0, 1], [1^T, 0]]).  The stencils are assembled
 *        at the first use after every coefficient rebuild, by probing: Z (then
 *        P^T Z_{l+1} P) applied to the indicators of 65 node colours
 *        (x + 34 y + 44 z) mod 65, a colouring that separates the 65 offsets.
 *        Z is symmetric: each level stores the centre and 32 of the offsets per node
 *        over a lattice padded by 2 nodes, 33 (n_l+5)^3 + 4 (n_l+1)^3 doubles per level
 *        (about 37 * 8/7 (n_{L-1}+1)^3 doubles in all), kept until destroy.  FGMRES only. */
typedef enum { AGCA_SCHUR_MASS = 0, AGCA_SCHUR_BFBT = 1, AGCA_SCHUR_BFBT_MG = 2 } agca_stokes_schur;
typedef struct {
    int32_t solver;          /* agca_stokes_solver                                          */
    int32_t restart;         /* FGMRES restart length, 1..510                              */
    int32_t max_iter;
    int32_t record_history;
    double tol;              /* stop when ||r||_2 <= tol ||(f, g)||_2 (eq. (4.3))           */
    int32_t precond;         /* agca_stokes_precond                                         */
    int32_t schur;           /* agca_stokes_schur                                           */
    int32_t schur_iters;     /* BFBT, BFBT_MG: CG steps per Z solve, 1..1000 (ignored for MASS) */
    int32_t velocity_cycles; /* V-cycles per application of the velocity block's approximate
                                inverse, as a stationary iteration from zero (x = V r, then
                                x += V (r - A x)); 0 or 1: the single V-cycle of the paper
                                (Section 4), at most 8.  With a symmetric cycle the result is
                                a fixed SPD operator, so MINRES accepts it too. */
    int32_t basis_dtype;     /* FGMRES: storage of the Arnoldi basis V, AGCA_F64 (0, the
                                default) or AGCA_F32 (half the Gram-Schmidt traffic; each new
                                basis vector is rounded to FP32 once, its dot products and
                                updates are FP64, the preconditioned vectors Z, the iterate and
                                the residual at restarts stay FP64).  The basis's rounding
                                bounds what one restart cycle can gain (about 1e-7 of the
                                cycle's starting residual); lower tolerances take more cycles */
} agca_stokes_opts;

/* Solve [[A, B^T], [B, 0]] (u, p) = (f, g) in FP64 with a block preconditioner built
 * from one AGCA V-cycle of A and a Schur approximation (opts->precond, opts->schur):
 * FGMRES(restart), right preconditioned, classical Gram-Schmidt with a second pass where
 * the first loses more than 90 % of the norm (any mg_dtype: the FP32 V-cycle makes the
 * preconditioner non-linear), or MINRES with the block-diagonal one (its theory needs a
 * fixed SPD preconditioner, which the FP32 V-cycle is only up to FP32 rounding; the true
 * residual is checked every step, so a run that stagnates reports AGCA_E_NOCONV, never a
 * false convergence).  The returned p has zero mean over the pressure nodes.  Work
 * space: 2 restart + 5 (FGMRES; with an FP32 basis about 1.5 restart + 6.5; one
 * more with TRIANGULAR) or 10 (MINRES) vectors of 3 (n_L+1)^3 + (n_{L-1}+1)^3 doubles,
 * kept until destroy;
 * BFBT and BFBT_MG add 3 velocity and 8 pressure vectors, BFBT_MG its multigrid.
 * FGMRES stops early with stats->floor_limited when a restart cycle's residual
 * estimate reached tol but the true residual after it is above tol, less than 5 %
 * below its value four cycles earlier, and at most max(tol, rho_A), rho_A the
 * rounding floor of the velocity block (the terms of agca_residual_floor for A and
 * f, over the norm of the whole right-hand side; a lower bound of the system's
 * floor), reported in stats->floor_estimate.
 * Returns AGCA_OK when converged or floor_limited, AGCA_E_NOCONV (u, p, stats filled)
 * otherwise;
 * stats->history holds the FGMRES residual estimates (true residual at restarts)
 * or the MINRES true residuals. */
int32_t agca_stokes_solve(agca_hier* h, const agca_stokes_opts* opts, const double* f,
                          const double* g, double* u, double* p, agca_solve_stats* stats);

/* q = S^-1 rp with the Schur approximation `schur` (agca_stokes_schur; schur_iters CG
 * steps per Z solve for BFBT and BFBT_MG, ignored for MASS): the pressure block of the
 * block-diagonal preconditioner.  rp, q: device pressure vectors, distinct.  Assembles
 * what the approximation needs on first use after a coefficient rebuild.
 * AGCA_E_INVALID for an unknown schur or schur_iters outside [1, 1000]. */
int32_t agca_stokes_schur_apply(agca_hier* h, int32_t schur, int32_t schur_iters, const double* rp,
                                double* q);

/* The BFBT_MG pressure multigrid's operator on level `level` (0..L-1; L-1 is the pressure
 * space itself, Z = B W^-1 B^T): out (device, 65 (n_level+1)^3 doubles) receives
 * S[i (n+1)^3 + k] = Z_level(k, k + o_i), o_i the i-th of the 65 stencil offsets ordered
 * by z, then y, then x ascending, 0 where node k + o_i lies outside the lattice.
 * Assembles the hierarchy if needed.  AGCA_E_INVALID for a level out of range. */
int32_t agca_stokes_z_stencil(agca_hier* h, int32_t level, double* out);

/* y = one V-cycle of the BFBT_MG pressure multigrid applied to r (device pressure
 * vectors, distinct; a zero-sum r gives the cycle's approximation to the zero-sum
 * solution of Z y = r).  Assembles the hierarchy if needed. */
int32_t agca_stokes_z_vcycle(agca_hier* h, const double* r, double* y);

/* Gradient test of eq. (2.8): for every macro element k (level-0 element id, 0..47)
 * the largest norm of grad eta_h over the finest elements inside it, eta_h the P1
 * function on level L with nodal values eta_nodes (device, (2^(L+1)+1)^3 doubles by
 * node id x + (n+1)(y + (n+1) z)).  gmax: host, 48 doubles.  Runs on `stream`
 * (a hipStream_t, may be null) and waits for it; allocates 384 bytes of device memory
 * for the call.  AGCA_E_INVALID for a bad L or a non-finite result. */
int32_t agca_macro_gradient(int32_t L, const double* eta_nodes, double* gmax, void* stream);

/* agca_macro_gradient without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the per-macro maxima live in a fixed file-scope device array of 48 64-bit slots (384
 * bytes, one per macro element, whatever L) that each GPU keeps until the process ends,
 * instead of the 384 bytes agca_macro_gradient allocates per call.  The first call on a
 * device looks the array's address up on that device (AGCA_E_HIP if that fails).  The
 * slots are cleared by a fill kernel at the start of every call.  All calls on one GPU
 * share its array: calls that overlap on one GPU (other streams or threads) race and
 * must be serialised by the caller.  Arguments, results and errors as
 * agca_macro_gradient (L in [1, 9], else AGCA_E_INVALID); the copy of the 48 results to
 * the host synchronises `stream`. */
int32_t agca_macro_gradient_noalloc(int32_t L, const double* eta_nodes, double* gmax, void* stream);

/* b = load vector of a per-element constant source: b_i = sum_e f_e |e| / 4 on
 * level L.  f: device, ncomp blocks of 6 n_L^3 doubles; b: device FP64 level vector. */
int32_t agca_load_vector(agca_hier* h, const double* f, double* b);

/* Bytes of device memory the library holds for this hierarchy. */
int64_t agca_device_bytes(const agca_hier* h);

const char* agca_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AGCA_H */
