/*
 * otbb.h -- C ABI of the MI355X interior-point solver for finite-volume
 * dynamical (Benamou-Brenier) optimal transport.
 *
 * Paper: E. Facca, G. Todeschi, A. Natale, M. Benzi, "Efficient
 * preconditioners for solving dynamical optimal transport via interior point
 * methods", arXiv 2209.00315.
 *
 * The problem (Sec. 1 and Sec. 2): given two densities rho_in, rho_f of equal
 * mass on a polygonal domain, find the time-dependent density rho, the
 * potential phi and the slack s solving the relaxed discrete optimality
 * system (Sec. 2.3-2.4) on a two-level finite-volume mesh with staggered
 * time levels: K density levels, K+1 potential levels, dt = 1/(K+1).
 * Each interior-point step runs inexact Newton iterations; each Newton
 * system is the projected saddle-point system of Sec. 4.4.2, solved by
 * flexible GMRES preconditioned by the BB block-triangular preconditioner of
 * Sec. 4.4.3.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Return value: 0 on success, a negative OT_E* code on failure.  No C++
 *    exception crosses this boundary; ot_last_error() gives a message.
 *  - Ownership: the caller owns every array it passes; the library copies
 *    inputs in and writes outputs to caller memory.  Handles (ot_mesh,
 *    ot_state) are library-owned; destroy them with the matching call.
 *    A handle must not be used from two threads at once.
 *  - Memory kind: with ot_options.mem_kind == OT_HOST every vector pointer is
 *    host memory; with OT_DEVICE it is device memory of the current HIP
 *    device (e.g. a torch tensor's data_ptr), read and written on
 *    ot_options.stream (NULL = the null stream).  Mesh descriptions are
 *    always host memory.
 *  - Layout: all vectors are FP64, slice-major.  phi has (K+1) * n_fine
 *    entries (level k at offset k * n_fine), rho and s have K * n_coarse.
 *    A "saddle vector" of length N = (K+1) n_fine + K n_coarse is the phi
 *    block followed by the rho block.
 *  - Errors leave handles usable and in their state before the call, except
 *    OT_ELINSOLVE / OT_ENEWTON from ot_newton_step and ot_solve, which leave
 *    the last accepted iterate in the state.
 */
#ifndef OTBB_H
#define OTBB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define OT_OK          0
#define OT_EINVAL     -1   /* null pointer, bad size or bad option          */
#define OT_EMESH      -2   /* area or distance <= 0, bad index, overlaps not
                              summing to the cell areas                     */
#define OT_EMASS      -3   /* |a'.rho_in - a'.rho_f| > 1e-12 a'.rho_in       */
#define OT_ENEG       -4   /* negative or non-finite marginal                */
#define OT_ELINSOLVE  -5   /* FGMRES did not reach its tolerance             */
#define OT_ENEWTON    -6   /* Newton iteration cap reached at some mu        */
#define OT_EDEVICE    -7   /* HIP runtime error                              */
#define OT_ENOMEM     -8   /* device or host allocation failed               */
#define OT_ETIME      -9   /* ot_options.max_seconds reached in a solve      */

#define OT_FP64   0        /* every kernel in FP64                           */
#define OT_MIXED  1        /* preconditioner in FP32, the rest in FP64       */
#define OT_STEP_COMMON 0   /* step rules, see ot_options.step_rule           */
#define OT_STEP_SPLIT  1

#define OT_PREC_BB     0   /* BB block-triangular preconditioner (Sec. 4.4.3) */
#define OT_PREC_SIMPLE 1   /* SIMPLE preconditioner (Sec. 4.3), FP64       */
#define OT_PREC_HYBRID 2   /* BB, handing over to SIMPLE when BB degrades  */
#define OT_PREC_PRIMAL 3   /* primal-Schur preconditioner (Sec. 4.2), FP64 */

#define OT_HOST   0
#define OT_DEVICE 1

typedef struct ot_mesh  ot_mesh;    /* opaque, immutable after creation      */
typedef struct ot_state ot_state;   /* opaque: (phi, rho, s, mu) + workspaces */

/*
 * Generic two-level FV mesh (Sec. 2.1).  Host arrays, copied in.
 *  fine cells carry phi, coarse cells carry rho and s.
 *  Omega = M J is given by its nonzeros (ov_fine[t], ov_coarse[t], ov_area[t]):
 *    rows must sum to fine_area, columns to coarse_area (relative 1e-10).
 *  Fine interior edges e: fe_cell[2e] = K, fe_cell[2e+1] = L with
 *    E(K,e) = +1, E(L,e) = -1, grad phi_e = (phi_K - phi_L) / fe_dist[e];
 *    fe_rho[2e], fe_rho[2e+1] = coarse cells feeding the density
 *    reconstruction R_E on the K and L side, with weights fe_lambda[e] and
 *    1 - fe_lambda[e].  Boundary edges are omitted (no-flux).
 *  Coarse interior edges (ce_*) define the coarse Laplacian of the BB
 *    approximation (Sec. 4.4.3); they never change the solution.
 *  All lengths and distances must be > 0 and lambdas in [0, 1].
 */
typedef struct {
    int32_t n_fine, n_coarse;
    const double *fine_area, *coarse_area;
    int32_t n_overlap;
    const int32_t *ov_fine, *ov_coarse;
    const double *ov_area;
    int32_t n_fedge;
    const int32_t *fe_cell;      /* [2 * n_fedge] */
    const int32_t *fe_rho;       /* [2 * n_fedge] */
    const double *fe_len, *fe_dist, *fe_lambda;
    int32_t n_cedge;
    const int32_t *ce_cell;      /* [2 * n_cedge] */
    const double *ce_len, *ce_dist, *ce_lambda;
} ot_mesh_desc;

/*
 * Solver options; ot_options_default() fills the paper's settings:
 *  tol 1e-6 (Newton, absolute Euclidean norm of (F_phi; F_rho; F_s - mu),
 *  Sec. 2.4), eps_out 1e-5 (FGMRES, relative to |(f;g;h)|, Sec. 3.1),
 *  eps_in_S 1e-1 (pseudo-Schur inner solve, Sec. 4.4.4), eps_in_A 1e-6
 *  (Laplacian inner solves: PCG stops on the residual, which at the
 *  paper's 5e-2, or even 1e-4, leaves low-energy error that the outer
 *  FGMRES pays for once mu is small: 1e-6 cuts its iterations up to 8x;
 *  FP32 vectors still reach it),
 *  mu0 1, mu_factor 0.2, step fraction 0.99, caps 400 FGMRES / 200 inner
 *  (Laplacian PCG, SIMPLE's inner PCG) / 10 pseudo-Schur GMRES / 20 Newton
 *  per mu (the pseudo-Schur solve stops at eps_in_S or at its cap,
 *  whichever comes first: past ~10 iterations its extra accuracy no longer
 *  lowers the FGMRES count; the paper gives no Newton cap and reports 3-7
 *  steps per mu, which the step-length tightening of eps_out and the
 *  hybrid preconditioner below reproduce on the benchmark grids), restart 400
 *  (FGMRES runs unrestarted within its cap, as in Sec. 4; its basis grows
 *  on demand up to (restart + 1) + restart vectors of N doubles), inner
 *  restart 30, accept_relres 1e-2, eps_out_min 1e-10, OT_STEP_COMMON,
 *  neighborhood 0, OT_PREC_HYBRID, hybrid_alpha 0.5, batch_streams 8,
 *  OT_MIXED, OT_HOST, null stream, no time limit.
 */
typedef struct {
    double tol, eps_out, eps_in_S, eps_in_A;
    double mu0, mu_factor, frac_to_boundary;
    double final_tol;        /* <= 0: use tol for the last mu as well       */
    double mu_stop;          /* > 0: stop after solving the first mu <= mu_stop
                                (a truncated continuation); 0: run down to the
                                first mu below tol                           */
    double accept_relres;    /* a Newton step whose FGMRES stopped at the cap
                                is still taken when its relative residual is
                                below this value (counted as a failure)     */
    int32_t max_fgmres, restart, max_inner, max_newton, inner_restart;
    int32_t max_inner_S;     /* cap of the pseudo-Schur inner GMRES (see above) */
    double eps_out_min;      /* tightest FGMRES tolerance of a Newton step
                                (relative, like eps_out; default 1e-10).
                                Once FGMRES meets eps_out, the step length
                                of its direction is checked; below 0.9 (and
                                still growing by 10% per check) the
                                tolerance is divided by 100, down to this
                                value, and FGMRES continues in the same
                                Krylov space.  eps_out_min >= eps_out
                                switches the rule off.                      */
    double max_seconds;      /* > 0: a solve (ot_solve, ot_state_solve) starts
                                no further Newton step once this much wall
                                time has passed and returns OT_ETIME with the
                                last iterate kept; 0: no limit             */
    double neighborhood;     /* gamma in [0, 1): > 0 shortens the common step
                                further so that every cell keeps
                                rho s >= gamma mu (a neighbourhood of the
                                central path, keeping the next Newton system
                                well scaled); 0 (default): positivity only */
    int32_t preconditioner;  /* OT_PREC_HYBRID (default), OT_PREC_BB,
                                OT_PREC_SIMPLE or OT_PREC_PRIMAL.  OT_PREC_HYBRID uses BB until
                                a Newton system whose BB solve misses eps_out
                                with a direction that the positivity line
                                search would cut below hybrid_alpha, or ends
                                above accept_relres; that system and every
                                later one of the state (until
                                ot_state_import) are solved with SIMPLE.
                                OT_PREC_SIMPLE: the
                                SIMPLE preconditioner of Sec. 4.3 on the
                                projected system, u = Diag(A)^-1 c,
                                P (C + B Diag(A)^-1 B^T) P^T y = P B u - d
                                by PCG to eps_in_S (cap max_inner) with its
                                exact time-line tridiagonal part T as
                                preconditioner (applied as T^-1 (r - a' l),
                                l chosen per slice so that the result lies
                                in the range of P^T), x = u - Diag(A)^-1
                                B^T P^T y; always FP64 (precision applies to
                                BB).
                                OT_PREC_PRIMAL: the primal-Schur
                                factorisation of Sec. 4.2 with the diagonal
                                C kept in the (2,2) block, S_p = A + B^T P^T
                                C^-1 P B solved by PCG to eps_in_S (cap
                                max_inner) with one V-cycle of the K+1
                                Laplacian multigrid as preconditioner;
                                always FP64                                 */
    double hybrid_alpha;     /* step-length threshold of OT_PREC_HYBRID
                                (default 0.5)                               */
    int32_t batch_streams;   /* ot_solve_batched: members solved at once,
                                each on its own stream and host thread
                                (default 8; 1 = one after another)         */
    int32_t step_rule;       /* OT_STEP_COMMON (default): one step length for
                                (phi, rho, s), the largest that keeps rho and
                                s positive times frac_to_boundary (Sec. 2.4);
                                OT_STEP_SPLIT: phi and rho take the largest
                                such step for rho, s its own                */
    int32_t precision, mem_kind;
    int32_t verbose;
    void *stream;            /* hipStream_t */
} ot_options;

/* Per-solve statistics (the paper's Outer/Lin.sys, Inner/Outer metrics). */
typedef struct {
    int32_t ip_steps, newton_steps, linear_systems;
    int64_t outer_iters, inner_S_iters, inner_A_iters, prec_applies;
    int32_t failures;        /* linear solves that missed eps_out           */
    double seconds_total, seconds_linear, seconds_setup;
    double final_residual, mu;
    double cost, dual, gap;
    double last_relres;      /* FGMRES relative residual of the last system  */
    int32_t tightenings;     /* FGMRES tolerance tightenings (eps_out_min)   */
    int32_t simple_systems;  /* Newton systems solved with SIMPLE            */
} ot_stats;

void ot_options_default(ot_options *opt);

/* Create a mesh from a generic description.  Errors: OT_EINVAL, OT_EMESH. */
int  ot_mesh_create(const ot_mesh_desc *desc, ot_mesh **out);
/* The n x n right-triangle grid (n even >= 2): phi on the n^2 squares (the
 * two triangles of a square share a circumcentre, so their potentials are
 * tied), rho on the 2 (n/2)^2 coarse triangles; index conventions
 * fine i = b n + a, coarse j = 2 (B n/2 + A) + t, t = 0 below the SW-NE
 * diagonal.  cartesian = 1 instead gives the single n x n Cartesian grid
 * (J = identity).  Errors: OT_EINVAL. */
int  ot_mesh_create_structured(int32_t n, int32_t cartesian, ot_mesh **out);
/* The n x n x n grid of cubes on [0,1]^3 for both levels (J = identity),
 * the three-dimensional workload of Sec. 4.1: cell (c n + b) n + a, the
 * interior faces as TPFA edges (|e| = h^2, d_e = h, lambda_e = 1/2), cell
 * volumes h^3 as areas; the coarse edges of the BB coarse Laplacian are
 * the same faces.  Errors: OT_EINVAL (n outside [2, 1024]). */
int  ot_mesh_create_cartesian3d(int32_t n, ot_mesh **out);
void ot_mesh_destroy(ot_mesh *mesh);
int  ot_mesh_sizes(const ot_mesh *mesh, int32_t *n_fine, int32_t *n_coarse,
                   int32_t *n_fedge, int32_t *n_cedge);

/*
 * Full interior-point solve (Sec. 2.4): mu_l = mu0 mu_factor^l, inexact
 * Newton until |F_mu| <= tol at each mu (final_tol at the last one), stop
 * after the first mu < tol, or after the first mu <= opt->mu_stop when that
 * is positive.
 * Outputs: rho_out [K n_coarse], phi_out [(K+1) n_fine] shifted so that
 * sum_k a^T phi^k = 0, cost_out = discrete kinetic energy.  Any output
 * pointer may be NULL.  stats may be NULL.
 * Errors: OT_EINVAL, OT_EMASS, OT_ENEG, OT_ELINSOLVE, OT_ENEWTON, OT_EDEVICE,
 * OT_ENOMEM.
 */
int  ot_solve(const ot_mesh *mesh, const double *rho_in, const double *rho_f,
              int32_t K, double tol, const ot_options *opt,
              double *rho_out, double *phi_out, double *cost_out, ot_stats *stats);

/*
 * Solve nprob independent problems (meshes and K may differ), each with its
 * own state and its own convergence as in ot_solve.  Up to
 * opt->batch_streams members run at the same time, each on a stream of the
 * library's own (created and destroyed by this call) driven by one host
 * thread; opt->stream is synchronised before the members start, and the
 * call returns when every member is done.  Arrays of pointers have nprob
 * entries; costs[nprob]; stats[nprob] or NULL.  All members are attempted;
 * the return value is the error of the lowest-numbered failing member
 * (ot_last_error names it).
 */
int  ot_solve_batched(int32_t nprob, const ot_mesh *const *meshes,
                      const double *const *rho_in, const double *const *rho_f,
                      const int32_t *K, double tol, const ot_options *opt,
                      double *const *rho_out, double *const *phi_out,
                      double *costs, ot_stats *stats);

/*
 * Create a state: validates the marginals (OT_ENEG, OT_EMASS) and sets the
 * start point phi = 0, rho = m0 / |Omega|, s = mu0 / rho, mu = mu0.
 */
int  ot_state_create(const ot_mesh *mesh, const double *rho_in, const double *rho_f,
                     int32_t K, const ot_options *opt, ot_state **out);
void ot_state_destroy(ot_state *st);
int  ot_state_sizes(const ot_state *st, int64_t *n_phi, int64_t *m_rho);
/* Copy (phi, rho, s, mu) out / in (any pointer may be NULL on export). */
int  ot_state_export(const ot_state *st, double *phi, double *rho, double *s, double *mu);
int  ot_state_import(ot_state *st, const double *phi, const double *rho,
                     const double *s, double mu);
/* Set mu without touching (phi, rho, s). */
int  ot_state_set_mu(ot_state *st, double mu);
/* Residual (F_phi; F_rho; F_s - mu) of Sec. 2.3-2.4 at the current state,
 * written to F [(K+1) n_fine + 2 K n_coarse] (may be NULL); norm to *nrm. */
int  ot_residual(ot_state *st, double *F, double *nrm);

/*
 * One inexact Newton step at the current mu: residual, linearisation, FGMRES
 * on the projected system with the BB preconditioner, recovery of
 * (delta phi, delta rho, delta s) (Sec. 4.4.1-4.4.2, Sec. 3.1), positivity
 * line search with the step fraction, update, per-slice renormalisation of
 * rho.  *res_norm (may be NULL) receives |F_mu| before the step.  When
 * FGMRES ends above eps_out: at most accept_relres the step is taken and
 * OT_ELINSOLVE returned (counted as a failure); above it the system is
 * solved again with the FP64 preconditioner and inner tolerances / 10, and
 * if that also ends above accept_relres the state is left unchanged.
 * Errors: OT_ELINSOLVE, OT_EDEVICE.
 */
int  ot_newton_step(ot_state *st, ot_stats *stats, double *res_norm);

/*
 * y = J_P x: the projected saddle operator of Sec. 4.4.2 linearised at the
 * current state, J_P = [[A, B^T P^T], [P B, -P C P^T]].  x, y: length N.
 */
int  ot_apply_saddle(ot_state *st, const double *x, double *y);

/*
 * Allocation-free y = J_P x, for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same operator and kernels as ot_apply_saddle, but x and y are always
 * device pointers (whatever opt.mem_kind says), the work is queued on
 * `stream` (NULL: the state's stream) without any host synchronisation, and
 * the kernels' scratch (slice sums and per-block partial sums) lives in a
 * library-held device array of 1 MiB per GPU (131072 doubles) instead of
 * the state's workspaces.  The call allocates nothing and calls no
 * allocating routine; the scratch array of a GPU is held until the process
 * ends.  Limit: 2 (K + 2) + ceil(n_coarse / 256) K <= 131072.
 * Every call on one GPU shares that GPU's scratch: calls that overlap in
 * time on one GPU (different streams or threads) race, so serialise them.
 * The scratch needs no clearing: every value is written before it is read.
 * The state's device must be current.
 * Errors: OT_EINVAL (null pointer, problem above the limit, wrong current
 * device), OT_EDEVICE.
 */
int  ot_apply_saddle_noalloc(const ot_state *st, const double *x, double *y, void *stream);

/*
 * z = P_BB^-1 r: one application of the BB preconditioner (Sec. 4.4.3)
 * linearised at the current state: pseudo-Schur solve
 * (Diag(s) A~ - Diag(rho) B M^-1 B~) w = -Diag(rho) P r_rho, then
 * z_rho = P^T M'^-1 A~ w, then the K+1 Laplacian solves
 * A^k z_phi^k = (r_phi - B^T z_rho)^k projected to zero sum; z_phi^k is
 * returned with zero sum.  Inner tolerances and caps come from the state's
 * options; for (near-)exact inner solves set eps_in_S and eps_in_A to ~1e-13
 * and raise max_inner_S and max_inner.
 */
int  ot_apply_schur_prec(ot_state *st, const double *r, double *z);

/*
 * Gradient of the transport cost at the current (converged) state with
 * respect to rho_in and rho_f (envelope term plus one adjoint saddle solve),
 * projected orthogonal to the coarse areas a'.  g_in, g_f: n_coarse each.
 * The objective is the kinetic energy of Sec. 1 in the discrete form of
 * Sec. 2.3; the adjoint system is the symmetric saddle system of Sec. 3.1,
 * solved through the projected system of Sec. 4.4.2 with the BB
 * preconditioner.  Every step runs on the device.  When the adjoint FGMRES
 * solve misses eps_out it is repeated once with the FP64 preconditioner and
 * inner tolerances / 10; if that also misses, the gradient is still written
 * and OT_ELINSOLVE is returned.
 * Errors: OT_EINVAL, OT_ELINSOLVE, OT_EDEVICE.
 */
int  ot_gradient(ot_state *st, double *g_in, double *g_f);

/*
 * Interior-point continuation (Sec. 2.4) on an existing state, from its
 * current iterate and mu (mu0 after ot_state_create; an imported iterate
 * and mu resume a run): mu, mu * mu_factor, ... each solved by inexact
 * Newton steps to |F_mu| <= tol (final_tol at the last one), ending after
 * the first mu below tol or at or below opt.mu_stop.  The state keeps the
 * last iterate, so ot_outputs, ot_state_export and ot_gradient can follow.
 * tol <= 0 takes the state's option.  stats (may be NULL) receives the
 * counts of this call and cost, dual and gap at its end.
 * Errors: OT_EINVAL, OT_ELINSOLVE, OT_ENEWTON, OT_ETIME, OT_EDEVICE,
 * OT_ENOMEM.
 */
int  ot_state_solve(ot_state *st, double tol, ot_stats *stats);

/* Outputs at the current state: cost (kinetic energy), dual value D*, and
 * phi normalised so that sum_k a^T phi^k = 0 (phi_out may be NULL). */
int  ot_outputs(ot_state *st, double *cost, double *dual, double *phi_out);

/* Change options of an existing state (tolerances, precision, caps). */
int  ot_state_set_options(ot_state *st, const ot_options *opt);

/* Message of the last error on this thread (never NULL). */
const char *ot_last_error(void);

/* sizeof(ot_options), sizeof(ot_stats) and sizeof(ot_mesh_desc) as this
 * library was built (any pointer may be NULL): a binding checks them
 * against its own declarations before it passes any of these structs. */
void ot_abi_sizes(int32_t *options_bytes, int32_t *stats_bytes, int32_t *mesh_desc_bytes);

/*
 * Kernel timing (instrumentation of the hot path, process-wide).
 * ot_kprof_select(id, elem_bytes) picks one kernel and clears the counters;
 * from then on every launch of it, in any state, whose floating-point
 * operands are elem_bytes wide (4: the FP32 preconditioner instantiation,
 * 8: FP64, 0: both) is launched with a start / stop HIP event pair stamped
 * by the dispatch itself on the stream it runs on, and its algorithmic
 * bytes (each operand read once, each result written once) are summed.  ot_kprof_read drains pending events (it synchronises with them)
 * and returns launches, total kernel milliseconds and total bytes; any
 * output pointer may be NULL.  OT_KPROF_NONE switches timing off.  Not for
 * concurrent use from several threads.
 *   CHEB_FINE     Chebyshev smoothing step of the K+1 Laplacians at the fine
 *                 multigrid level (the Laplacian solves of the BB
 *                 preconditioner, Sec. 4.4.3)
 *   SCHUR_BTILDE  pseudo-Schur operator, pass M^-1 B~ z (B~ of Sec. 4.4.3)
 *   SCHUR_OUT     pseudo-Schur operator, pass Diag(s) A~ z - Diag(rho) B v
 *                 (Sec. 4.4.3)
 *   TRI_FINE      time-line tridiagonal solve on the density cells
 *   MULTIDOT      dot products of one vector with a Krylov basis (Arnoldi)
 *   SADDLE_PHI    potential block of the saddle operator J_P (Sec. 4.4.2)
 */
enum {
    OT_KPROF_NONE = 0, OT_KPROF_CHEB_FINE = 1, OT_KPROF_SCHUR_BTILDE = 2, OT_KPROF_SCHUR_OUT = 3,
    OT_KPROF_TRI_FINE = 4, OT_KPROF_MULTIDOT = 5, OT_KPROF_SADDLE_PHI = 6
};
int  ot_kprof_select(int32_t kernel, int32_t elem_bytes);
int  ot_kprof_read(int64_t *launches, double *ms, double *bytes);

#ifdef __cplusplus
}
#endif
#endif /* OTBB_H */
