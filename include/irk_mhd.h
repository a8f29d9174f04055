/*
 * irk_mhd.h -- the linearised 2D MHD stage system on the stage-coupled Vanka multigrid
 * of libirkmg.so (part of the same library as irk_mg.h).
 *
 * Model (Sec. 3.3): incompressible resistive MHD with velocity u (vector P2, zero on
 * the boundary), magnetic field B (lowest-order Nedelec of the first kind, B x n = 0
 * on the boundary), pressure p (P1) and a Lagrange multiplier gamma (P1, zero on the
 * boundary) enforcing div B = 0.  In 2D the curl of a field is the scalar
 * d_x B_y - d_y B_x, and the cross products follow from three-dimensional fields with
 * zero third component.  The weak form is linearised (one Newton step) at a state
 * (w, B0), which gives the spatial bilinear forms, with test functions (v, c, q, s):
 *
 *   (2/Re)(eps(u), eps(v)) + ((w.grad)u + (u.grad)w, v)
 *     - ((curl B) x B0 + (curl B0) x B, v) - (p, div v) - (q, div u)
 *   + (1/Rem)(curl B, curl c) - (u x B0 + w x B, curl c) - (grad gamma, c) - (B, grad s)
 *
 * and the mass M = diag(M_u, M_B, 0, 0).  The viscous term carries the sign that makes
 * the operator dissipative (integration by parts of -div((2/Re) eps(u))).  The IRK
 * stage system of Sec. 3.1 applied to this DAE is
 *
 *     ( I_r (x) M + dt A (x) S ) k = F,
 *
 * solved by FGMRES (Sec. 4) with a geometric V-cycle (Sec. 4.1): rediscretisation on
 * every level (w injected at the coarse P2 nodes, the coarse B0 degrees of freedom
 * summed from the two fine halves of each coarse edge), transfers I_r (x)
 * diag(P_u, P_B, P_p, P_gamma) (canonical P2, Nedelec and P1 interpolation) and the
 * additive vertex-star Vanka relaxation of Fig. 1 (right): for each vertex v, the free
 * velocity nodes and the interior edges of the closure of the cells around v, the
 * pressure at v and, for an interior v, the multiplier at v, in every stage.  The
 * patch kernels are those of irk_mg.h (dense stage-coupled inverses in LDS, one
 * wavefront per patch, owner gather); the spatial operator is one sliced sparse
 * matrix applied to all r stages.
 *
 * Conventions: those of irk_mg.h (device vectors, float64, stream-ordered, errors via
 * irk_last_error), with these numberings on a level:
 *   P2 nodes   vertices, then edges sorted by (smaller, larger) vertex index;
 *   edges      in that order; a Nedelec degree of freedom is the line integral of the
 *              tangential component along the edge from its smaller to its larger
 *              vertex index; boundary edges (on a facet of one cell) are eliminated;
 *   layout     stage blocks in stage order, each of ns = 2 nfree + nB + nverts + ng
 *              values: u_x over the free P2 nodes, u_y over them, B over the interior
 *              edges, p at every vertex, gamma at the interior vertices.
 * The pressure is determined up to a constant per stage: preconditioner outputs and
 * solutions have each stage's pressure mean removed, and the coarsest solve pins the
 * pressure of vertex 0 of every stage.
 */
#ifndef IRK_MHD_H
#define IRK_MHD_H

#include "irk_mg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct irk_mhd irk_mhd; /* opaque handle */

/* Relaxation options: smoother 0, `pre` / `post` damped additive sweeps
 * k += omega W S (F - J k) per level (Sec. 4.2), W = I (weighting 0) or each unknown's
 * correction divided by the number of patches containing it (weighting 1); smoother 1,
 * `pre` / `post` steps of the Chebyshev semi-iteration (Sec. 5.1) accelerating W S for
 * the spectrum interval [cheb_lo, cheb_hi] of W S J (omega unused; the paper's MHD runs
 * use 3 / 3 steps on [2, 10] with the unweighted operator).  patch_form: how the exact inverse
 * of each stage-coupled patch matrix I (x) M_v + dt A (x) S_v is stored (the operator
 * applied is the same): 0 dense, (r n_s)^2 values; 1 factored through A = W T W^{-1}
 * (irk_stage_basis), r n_s^2 values, IRK_EINVAL from setup if A has no
 * well-conditioned real block diagonalisation; 2 automatic (1 when r >= 2 and the
 * decomposition exists, else 0).  Defaults: 2, 2, 0.5, 1, 2, smoother 0, interval [2, 10]. */
typedef struct irk_mhd_opts {
  int pre, post;
  double omega;
  int weighting;
  int patch_form;
  int smoother;
  double cheb_lo, cheb_hi;
} irk_mhd_opts;
void irk_mhd_default_opts(irk_mhd_opts* opt);
/* The patch form the handle uses (0 or 1), -1 for NULL. */
int irk_mhd_patch_form(const irk_mhd* h);

/* Build the hierarchy, assemble every level's M and S, factorise every patch on the
 * GPU and the coarsest operator (dense, FP64).
 *   levels   2D nested meshes, coarse to fine (irk_mesh_level of irk_mg.h); dim = 2
 *   tab      Butcher tableau, 1 <= r <= 4
 *   Re, Rem  fluid and magnetic Reynolds numbers (> 0)
 *   w        host, finest P2 nodes x 2 (row-major): the velocity of the linearisation
 *   b0       host, finest edges: Nedelec degrees of freedom of B0 on every edge
 * Host inputs are borrowed.  IRK_EINVAL for invalid sizes or values (before any
 * device work), IRK_ESINGULAR for a zero pivot in a patch or the coarse operator. */
irk_status irk_mhd_setup(const irk_mesh_level* levels, int nlevels, const irk_tableau* tab, double dt,
                         double Re, double Rem, const double* w, const double* b0, const irk_mhd_opts* opt,
                         void* stream, irk_mhd** out);
void irk_mhd_destroy(irk_mhd* h);
/* Host only (no device work): the spatial operators of one level as irk_mhd_setup
 * assembles them, for inspection.  M and S share one CSR pattern (ns x ns, sorted
 * columns, unknowns in the per-stage order above); P is the prolongation from level
 * level-1 (ns x ns_coarse, absent on level 0).  Two calls: with ptr NULL, sizes
 * receives {ns, nnz(S), nnz(P), ns_coarse}; then with arrays of those sizes (ptr ns+1,
 * col / mval / sval nnz(S), P_ptr ns+1, P_col / P_val nnz(P)) and the same sizes. */
irk_status irk_mhd_host_operators(const irk_mesh_level* levels, int nlevels, int level, double Re, double Rem,
                                  const double* w, const double* b0, int64_t* sizes, int32_t* ptr, int32_t* col,
                                  double* mval, double* sval, int32_t* P_ptr, int32_t* P_col, double* P_val);
/* r * ns of level `level` (0 = coarsest; -1 = finest), or -1 for a bad argument. */
int64_t irk_mhd_ndofs(const irk_mhd* h, int level);
/* out[0..4] = per-stage offsets of u_x, u_y, B, p, gamma; out[5] = ns; out[6] = r. */
irk_status irk_mhd_layout(const irk_mhd* h, int level, int64_t* out);

/* y = J_l x on level l. */
irk_status irk_mhd_apply(irk_mhd* h, int level, const double* x, double* y, void* stream);
/* One damped additive Vanka sweep on level l >= 1: k <- k + omega W sum_v R_v^T
 * A_v^{-1} R_v (F - J_l k), A_v = R_v J_l R_v^T (Sec. 4.2); with smoother 1 one
 * Chebyshev step from k, k <- k + W S (F - J_l k) / theta. */
irk_status irk_mhd_sweep(irk_mhd* h, int level, const double* F, double* k, void* stream);
/* xc = (I_r (x) P_l)^T xf, level l >= 1 to l-1; xf += (I_r (x) P_l) xc (Sec. 4.1). */
irk_status irk_mhd_restrict(irk_mhd* h, int level, const double* xf, double* xc, void* stream);
irk_status irk_mhd_prolong(irk_mhd* h, int level, const double* xc, double* xf, void* stream);
/* x = J_0^{-1} b on the coarsest level, the pressure of vertex 0 pinned per stage (b's
 * pinned entries are ignored and those of x are zero). */
irk_status irk_mhd_coarse_solve(irk_mhd* h, const double* b, double* x, void* stream);
/* z = V r: one V-cycle from a zero initial guess on the finest level, each stage's
 * pressure mean removed. */
irk_status irk_mhd_vcycle(irk_mhd* h, const double* r, double* z, void* stream);
/* Right-preconditioned restarted FGMRES (modified Gram--Schmidt, Givens rotations) on
 * the finest level with the V-cycle; k is the initial guess on entry and the solution
 * (pressure means removed) on exit.  Stops when the residual estimate reaches
 * rtol ||F - J k0||.  IRK_ENOCONV (> 0) at maxit; 1 <= restart <= 1000. */
irk_status irk_mhd_fgmres_solve(irk_mhd* h, const double* F, double* k, double rtol, int maxit, int restart,
                                irk_solve_info* info, void* stream);

/* Per-kernel timing with HIP events on the calls' stream: enable = 1 records the
 * finest level's launches, 2 every level's, 0 stops; enabling clears what was recorded.
 * irk_mhd_kernel_stats reports, for kernel 0 (patch apply), 1 (Kronecker residual) or
 * 2 (gather update) on one level, the launches recorded, their total time and the
 * algorithmic bytes of one launch (8-byte values, 4-byte indices):
 *   patch apply    every stored inverse (sum over patches of (r n_s)^2 values), the
 *                  residual once, the patch outputs;
 *   residual       one column index and the M and S values per operator entry, x and F
 *                  read once, the result written;
 *   gather update  the patch outputs with their slot indices, x read and written, the
 *                  weights. */
irk_status irk_mhd_profile(irk_mhd* h, int enable);
irk_status irk_mhd_kernel_stats(irk_mhd* h, int kernel, int level, irk_kernel_stats* out);

#ifdef __cplusplus
}
#endif
#endif /* IRK_MHD_H */
