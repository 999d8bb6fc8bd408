/*
 * otbb_debug.h -- host-only inspection entry points of the otbb library.
 *
 * They run the mesh generator, the validation and the derivation of the
 * index structures (multigrid aggregation, coarse-cell coloring) on the host
 * and never touch a device, so host logic can be checked without a GPU.
 * Same error codes and ownership rules as otbb.h.
 */
#ifndef OTBB_DEBUG_H
#define OTBB_DEBUG_H

#include "otbb.h"

#ifdef __cplusplus
extern "C" {
#endif

/* out = {n_fine, n_coarse, n_fedge, n_cedge, n_overlap, multigrid levels,
 *        coarse-cell colors, fine-cell ELL width} of the structured mesh of
 * ot_mesh_create_structured(n, cartesian), or of ot_mesh_create_cartesian3d(n)
 * when cartesian == 3.  Errors: OT_EINVAL. */
int otbb_debug_structured_sizes(int32_t n, int32_t cartesian, int32_t out[8]);

/* Copy the arrays of that mesh into caller buffers sized from
 * otbb_debug_structured_sizes (any pointer may be NULL): fine edges
 * (cells, density sides, length, distance, lambda), overlaps, coarse edges
 * (cells, length, distance) and the coarse-cell coloring. */
int otbb_debug_structured_arrays(int32_t n, int32_t cartesian, int32_t *fe_cell, int32_t *fe_rho,
                                 double *fe_len, double *fe_dist, double *fe_lambda, int32_t *ov_fine,
                                 int32_t *ov_coarse, double *ov_area, int32_t *ce_cell, double *ce_len,
                                 double *ce_dist, int32_t *color);

/* Validate a mesh description and derive its structures on the host only.
 * Returns OT_OK, OT_EINVAL or OT_EMESH exactly as ot_mesh_create would
 * before its device upload. */
int otbb_debug_validate_desc(const ot_mesh_desc *desc);

/* Pseudo-Schur multigrid hierarchy of that structured mesh: out[0] = number
 * of levels, then (cells, stencil width, colours) per level, up to cap
 * entries in total. */
int otbb_debug_schur_levels(int32_t n, int32_t cartesian, int32_t *out, int32_t cap);

/*
 * Components of the BB preconditioner at the state's current linearisation
 * (built on first use), host pointers in and out, FP64 at the interface and
 * the state's precision inside:
 *  schur_apply:   out = (Diag(s) A~ - Diag(rho) B M^-1 B~) z      (m_rho)
 *  schur_solve:   right-preconditioned restarted GMRES on that system,
 *                 relative tolerance tol, cap maxit, iterations to *iters
 *  tri_diagonals: its three time diagonals per coarse cell (probed):
 *                 d0 = (k,k), dl = (k,k-1), du = (k,k+1) entries (m_rho)
 *  tri_solve:     the time-line tridiagonal solve built from those
 *                 diagonals (Thomas factors; weak pivots replaced by the
 *                 plain diagonal)                                    (m_rho)
 *  laplace_solve: PCG with the multigrid V-cycle on the K+1 Laplacians
 *                 A^k x^k = b^k (b zero-sum per slice)             (n_phi)
 *  vcycle:        one multigrid V-cycle x = M^-1 b on all slices  (n_phi)
 */
int otbb_debug_schur_apply(ot_state *st, const double *z, double *out);
int otbb_debug_schur_solve(ot_state *st, const double *rhs, double *z, double tol, int32_t maxit,
                           int32_t *iters);
int otbb_debug_tri_diagonals(ot_state *st, double *d0, double *dl, double *du);
int otbb_debug_tri_solve(ot_state *st, const double *r, double *x);
/* Time levels per thread of the two time-blocked pseudo-Schur passes for
 * FP32 (elem_bytes 4), FP64 (8) or both (0) operands, for the BB
 * preconditioners created afterwards (process-wide knob; 0 levels = one
 * level per thread).  By default the first preconditioner of a given shape
 * (mesh sizes, K, precision) in the process times the candidates 0, 4, 8,
 * 16, 32 at its first linearisation and keeps the fastest, and later ones
 * of that shape reuse the choice (the blocked and per-level passes round
 * differently, so results do not depend on which stream timed faster);
 * this call fixes the values instead, and both values negative returns to
 * the autotuner. */
int otbb_debug_set_schur_blocking(int32_t elem_bytes, int32_t btilde_levels, int32_t out_levels);
/* V-cycle of the pseudo-Schur multigrid (Sec. 4.4.3 solves that system
 * iteratively; the multigrid is this library's own) for the BB
 * preconditioners created afterwards (process-wide knob): damping omega of
 * the time-line Jacobi smoother in (0, 1], nu pre- and post-smoothing steps
 * in [1, 16], coarse_its smoothing steps on the coarsest level in [1, 200],
 * alpha in (0, 3] scales the prolongated coarse correction.  Defaults
 * 0.5, 2, 6, 1.0.  OT_EINVAL for values out of range. */
int otbb_debug_set_schur_mg(double omega, int32_t nu, int32_t coarse_its, double alpha);
int otbb_debug_laplace_solve(ot_state *st, const double *b, double *x, double tol, int32_t maxit,
                             int32_t *iters);
int otbb_debug_vcycle(ot_state *st, const double *b, double *x);
/* Multigrid level data of the current linearisation: what = 0 edge weights
 * [(K+1) x edges of the level], what = 1 inverse diagonals [(K+1) x cells].
 * *count receives the length; out may be NULL to query it. */
int otbb_debug_mg_level(ot_state *st, int32_t level, int32_t what, double *out, int64_t *count);

#ifdef __cplusplus
}
#endif
#endif /* OTBB_DEBUG_H */
