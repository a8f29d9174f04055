/*
 * irk_mg.h -- C ABI of the MI355X stage-coupled Vanka multigrid library (libirkmg.so).
 *
 * The library solves the stage system of a fully implicit Runge--Kutta step for the
 * Taylor--Hood (P2-P1) discretisation of the time-dependent Stokes equations and of
 * their Oseen linearisation (Abu-Labdeh, MacLachlan, Farrell, "Monolithic multigrid for
 * implicit Runge--Kutta discretizations of incompressible fluid flow", Sec. 3.1, the
 * stage system in Kronecker form):
 *
 *     ( I_r (x) [M 0; 0 0] + dt A (x) [K(+C) B; B^T 0] ) k = F,
 *
 * preconditioning FGMRES (Sec. 4) with a geometric V-cycle whose relaxation is the
 * additive vertex-star Vanka sweep coupling all stages (Sec. 4.2) and whose transfers
 * are I_r (x) P and its transpose (Sec. 4.1); and Newton's method on the nonlinear
 * Navier--Stokes stage equations (Sec. 3.2) with these solves as its linear steps.  All
 * arithmetic runs in HIP kernels on a gfx950 GPU; host code only builds the mesh
 * topology and sparse structures and runs the Krylov and Newton loops' scalar logic.
 *
 * Conventions used by every entry point
 * -------------------------------------
 * Numbering.  On a mesh level the P2 nodes are the vertices in input order followed
 *   by the edges sorted by (smaller vertex index, larger vertex index).  A node is a
 *   boundary node when it lies on a facet that belongs to exactly one cell; boundary
 *   velocity values are eliminated: zero, unless irk_rhs_dirichlet adds prescribed
 *   data.  Free nodes are the others, in ascending node order.
 * Vector layout ("ABI layout"), length r * ns with ns = dim * nfree + nverts: stage
 *   blocks in stage order (Sec. 3.1 orders the stages consecutively, each stage's
 *   velocity and pressure together); inside a stage block the velocity components one
 *   after the other, each over the free nodes, then the pressure at every vertex.
 * Pressure.  The pressure is determined up to a constant per stage.  Every
 *   preconditioner application and every solution returned has each stage's
 *   arithmetic pressure mean removed; the coarsest-level solve pins the pressure of
 *   vertex 0 of every stage.
 * Memory.  Host inputs to irk_mg_setup are borrowed (copied during the call).  Vector
 *   arguments of the other calls are DEVICE pointers owned by the caller, float64,
 *   contiguous, not aliasing each other unless stated; the handle owns all its device
 *   memory.  `stream` is a hipStream_t (NULL: the null stream); work is stream-ordered
 *   and calls return without synchronising unless stated.
 * Errors.  Calls return IRK_OK (0), a negative error, or a positive warning.  Arguments
 *   are validated before any device work.  irk_last_error() describes the last failure
 *   on the calling thread.  A handle is not thread safe; distinct handles are
 *   independent.
 */
#ifndef IRK_MG_H
#define IRK_MG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int irk_status;
enum {
  IRK_OK = 0,
  IRK_EINVAL = -1,     /* invalid argument (checked before any device work)       */
  IRK_ENOMEM = -2,     /* device or host allocation failed                        */
  IRK_EHIP = -3,       /* a HIP runtime call failed                               */
  IRK_ESINGULAR = -4,  /* zero pivot in a patch or coarse factorisation           */
  IRK_ENAN = -5,       /* non-finite value met in a solve                         */
  IRK_ENOCONV = 1      /* warning: FGMRES hit maxit before reaching rtol          */
};

/* One level of a nested simplicial mesh hierarchy (Sec. 4.1: uniform refinements of
 * a coarsest grid).  Levels are passed coarse to fine.  cells[c*(dim+1)+k] is the k-th
 * vertex of cell c; parent[c] is the cell of the next coarser level that contains
 * cell c (NULL on level 0).  Every level must be a red refinement of the previous one
 * (each coarse vertex and edge midpoint is a fine vertex). */
typedef struct irk_mesh_level {
  int dim;                /* 2 (triangles) or 3 (tetrahedra)                 */
  int64_t nverts, ncells;
  const double* xyz;      /* host, nverts x dim, row-major                    */
  const int64_t* cells;   /* host, ncells x (dim+1)                           */
  const int64_t* parent;  /* host, ncells, or NULL on level 0                 */
} irk_mesh_level;

/* Butcher tableau (Sec. 2, eq. "general RK"): r x r matrix A (row-major), weights b,
 * nodes c.  1 <= r <= 4.  A must be invertible (fully implicit). */
typedef struct irk_tableau {
  int r;
  const double* A;
  const double* b;
  const double* c;
} irk_tableau;

/* Solver options.  Defaults (irk_mg_default_opts): 2 pre- and 2 post-sweeps (Sec. 5.1),
 * omega = 0.5, partition-of-unity weighting, FP64, automatic patch form, damped
 * sweeps (Chebyshev interval preset to the paper's [2, 8]). */
typedef struct irk_mg_opts {
  int pre, post;     /* Vanka sweeps before / after the coarse correction        */
  double omega;      /* damping of the additive sweep (Sec. 4.2)                 */
  int weighting;     /* 0: literal sum over patches; 1: each DOF's correction
                        divided by the number of patches containing it          */
  int precision;     /* 0: FP64 V-cycle; 1: FP32 patch factors and FP32 V-cycle
                        (coarse solve, FGMRES and outer residual stay FP64)      */
  int patch_form;    /* how the exact inverse of each stage-coupled patch matrix
                        I (x) M_v + dt A (x) S_v is stored (the operator applied
                        is the same in every form):
                        0: dense (r n_s)^2 inverse;
                        1: factored through A = W T W^{-1} (irk_stage_basis):
                           r n_s^2 stored values, IRK_EINVAL from setup if A has
                           no well-conditioned real block diagonalisation;
                        2: automatic: 3 for Stokes (wind NULL), else 1, when
                           r >= 2 and the decomposition exists; else 0;
                        3: symmetric factored (Stokes only, wind NULL): every
                           block M_v + dt T_k S_v is then real or complex
                           symmetric, and each block inverse is kept by its
                           n_s/2 + 1 wrapped diagonals, r n_s (n_s/2 + 1)
                           stored values; used on levels whose patches have at
                           most 256 unknowns per stage (form 1 on the others
                           under 2; IRK_EINVAL from setup under 3)              */
  int smoother;      /* relaxation: 0 = `pre`/`post` damped additive sweeps
                        k += omega W S r; 1 = `pre`/`post` steps of the Chebyshev
                        semi-iteration (Sec. 5.1) accelerating W S, S the additive
                        Vanka operator, for the spectrum interval [cheb_lo,
                        cheb_hi] of W S J (omega unused; the paper's runs use the
                        unweighted operator, weighting = 0, on [2, 8]);
                        2 = one cycle of `pre`/`post` (at most 8) steps of GMRES
                        left-preconditioned by W S (Sec. 4.2, 5.4), from the
                        current iterate, classical Gram--Schmidt: a nonlinear
                        relaxation, so the V-cycle is a nonlinear preconditioner
                        (the solvers here are flexible); omega unused          */
  double cheb_lo, cheb_hi; /* 0 < cheb_lo < cheb_hi, else IRK_EINVAL            */
} irk_mg_opts;

/* Per-solve report.  history (host, may be NULL) receives up to history_cap residual
 * 2-norms: the initial one, then one per iteration. */
typedef struct irk_solve_info {
  int iterations;
  int converged;
  double rel_residual;     /* ||F - J k|| / ||F - J k0|| recomputed at exit */
  double* history;
  int history_cap;
  double ms_vcycle;        /* GPU time inside the preconditioner (ms)       */
  double ms_total;         /* GPU time of the whole solve (ms)              */
} irk_solve_info;

typedef struct irk_mg irk_mg; /* opaque handle */

/* Fill *opt with the defaults listed above. */
void irk_mg_default_opts(irk_mg_opts* opt);

/* Built-in tableaux (Sec. 5: Gauss, RadauIIA, LobattoIIIC): family 0 = RadauIIA
 * (r = 1..3), 1 = Gauss (r = 1..3), 2 = LobattoIIIC (r = 2..3).  Writes r*r + 2r
 * values to A, b, c (host arrays of size >= 16, 4, 4).  Returns IRK_EINVAL for an
 * unknown (family, r). */
irk_status irk_tableau_builtin(int family, int r, double* A, double* b, double* c);

/* P2 node coordinates of one mesh level without building a handle (so that nodal data
 * such as the wind can be evaluated before irk_mg_setup): writes the node count to
 * *nnodes and, if xyz is not NULL, the coordinates (host, nnodes x dim) in the node
 * numbering above.  Errors: IRK_EINVAL for null or out-of-range input. */
irk_status irk_mesh_p2_nodes(const irk_mesh_level* level, int64_t* nnodes, double* xyz);

/* Build the hierarchy for the stage operator with step dt, viscosity nu (K is nu times
 * the P2 Laplacian, Sec. 3.1-3.2) and optional wind (Oseen convection C(w), Sec. 3.2):
 * `wind` is host, nnodes_finest x dim nodal P2 values on the finest level (NULL for
 * Stokes); coarser levels take the values at coincident nodes.  Assembles every level
 * (rediscretisation, Sec. 4.1), builds the vertex-star patches (Sec. 4.2, Fig. 1),
 * factorises every patch on the GPU and the coarsest operator, and returns the handle
 * in *out.  Synchronises `stream` before returning.  Errors: IRK_EINVAL (dims, sizes,
 * r outside 1..4, non-nested levels, nlevels < 1), IRK_ENOMEM, IRK_EHIP,
 * IRK_ESINGULAR (a zero pivot in a patch or in the coarse operator). */
irk_status irk_mg_setup(const irk_mesh_level* levels, int nlevels, const irk_tableau* tab,
                        double dt, double nu, const double* wind, const irk_mg_opts* opt,
                        void* stream, irk_mg** out);

/* Patch form of the finest level (0 dense, 1 factored, 3 symmetric factored; see
 * irk_mg_opts), or -1 for NULL. */
int irk_mg_patch_form(const irk_mg* h);

/* Estimate of the spectrum of the relaxation's preconditioned operator W S J_l on level
 * l >= 1 (S the additive Vanka operator, W the handle's weighting), from which Sec. 5.1's
 * rule takes the Chebyshev interval [lambda_max / 4, lambda_max]: `steps` (1..64)
 * Arnoldi steps with classical Gram--Schmidt from v0 (device, ABI layout of level l,
 * not modified), then the Ritz values, eigenvalues of the leading Hessenberg block, in
 * ritz_re / ritz_im (host, `steps` values each, decreasing real part, zero past
 * *nritz).  H (host, (steps + 1) x steps column-major, may be NULL) receives the
 * Hessenberg matrix.  An invariant Krylov space ends the estimate early (*nritz <
 * steps; nritz may be NULL).  Allocates its Arnoldi basis for the call; synchronises
 * `stream`.  IRK_ENOCONV if the small eigenvalue iteration fails. */
irk_status irk_mg_ritz(irk_mg* h, int level, int steps, const double* v0, double* H, double* ritz_re,
                       double* ritz_im, int* nritz, void* stream);

/* irk_mg_ritz without any allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and errors as irk_mg_ritz, bitwise equal to them.  The Arnoldi
 * basis, Hessenberg matrix and reduction partial sums live in a static device array of
 * 64 MiB that the library holds on every GPU it runs on until the process ends (its
 * address is looked up on the first call made with that GPU current): (steps + 1) level
 * vectors of the handle's precision plus (steps + 1)^2 + 256 * 9 doubles must fit, each
 * part rounded up to 256 bytes, else IRK_EINVAL with a message naming the need.  The
 * host side uses fixed-size stack storage.  All calls on one GPU share that array and
 * it keeps the last call's contents (each call initialises what it reads): calls that
 * overlap in time on one GPU, from several threads or streams, race and must not be
 * made.  Synchronises `stream`. */
irk_status irk_mg_ritz_noalloc(irk_mg* h, int level, int steps, const double* v0, double* H, double* ritz_re,
                               double* ritz_im, int* nritz, void* stream);

/* Change the Chebyshev interval of a handle (smoother 1) after setup, for example to
 * [lambda/4, lambda] from irk_mg_ritz.  IRK_EINVAL unless 0 < lo < hi < inf. */
irk_status irk_mg_set_interval(irk_mg* h, double lo, double hi);


/* Eigenvalues of the leading m x m block (1 <= m <= 1024) of an upper Hessenberg matrix
 * H (host, column-major, leading dimension ldh >= m) by the shifted QR iteration,
 * sorted by decreasing real part into wr / wi (host, m values).  Host-only. */
irk_status irk_hessenberg_eigs(int m, const double* H, int ldh, double* wr, double* wi);

/* Real block diagonalisation of a Butcher matrix, A = W T W^{-1}, as used by the
 * factored patch form: T is block diagonal with 1x1 blocks (real eigenvalues,
 * ascending) followed by 2x2 blocks [[a, b], [-b, a]] (pairs a +- ib, b > 0, ascending
 * a); the columns of W are the real eigenvectors and the real and imaginary parts of
 * the pairs' eigenvectors.  A, W, Winv, T: host, r x r row-major (outputs may be NULL).
 * Errors: IRK_EINVAL for r outside 1..4, null A, repeated or defective eigenvalues,
 * cond(W) > 1e6 or a failed reconstruction check. */
irk_status irk_stage_basis(int r, const double* A, double* W, double* Winv, double* T);

/* Release the handle and all its device memory (NULL is ignored). */
void irk_mg_destroy(irk_mg* h);

/* Number of unknowns r * ns of level `level` (0 = coarsest; -1 = finest), or -1. */
int64_t irk_mg_ndofs(const irk_mg* h, int level);

/* Level sizes: out[0..4] = nverts, nnodes, nfree, ns (= dim*nfree + nverts), nlevels.
 * level -1 is the finest. */
irk_status irk_mg_sizes(const irk_mg* h, int level, int64_t* out);

/* Where each field of each stage sits in the ABI layout of level `level` (-1: finest;
 * Sec. 3.1 orders the unknowns stage by stage, velocity then pressure): offsets (host,
 * r x (dim + 1), may be NULL) receives, for stage s, offsets[s*(dim+1) + c] = the index
 * of the first value of velocity component c (c < dim) and offsets[s*(dim+1) + dim] =
 * that of the pressure; lengths (host, dim + 1, may be NULL) the number of values of
 * each field (nfree per velocity component, nverts for the pressure).  Velocity value
 * i of a component belongs to free node i (irk_mg_p2_nodes gives the node numbers);
 * pressure value v to vertex v.  Errors: IRK_EINVAL (null handle, level out of range,
 * both outputs NULL). */
irk_status irk_mg_layout(const irk_mg* h, int level, int64_t* offsets, int64_t* lengths);

/* Coordinates of the P2 nodes of a level (host out, nnodes x dim) and the node index of
 * every free node (host out, nfree; may be NULL). */
irk_status irk_mg_p2_nodes(const irk_mg* h, int level, double* xyz, int64_t* free_nodes);

/* y = J x (transpose = 0) or y = J^T x (transpose = 1) on the finest level. */
irk_status irk_mg_apply(irk_mg* h, const double* x, double* y, int transpose, void* stream);

/* z = V r: one V-cycle (Sec. 4.1-4.2, 5.1) from a zero initial guess on the finest
 * level, pressure means removed.  In FP32 mode r is rounded to FP32 on entry and the
 * cycle runs in FP32 except for the coarse solve.  r and z may not alias. */
irk_status irk_mg_vcycle(irk_mg* h, const double* r, double* z, void* stream);

/* z = V^T r: the transpose of irk_mg_vcycle as a linear map (used by adjoint solves).
 * With the GMRES relaxation (smoother 2) the V-cycle is not linear; this is then the
 * same cycle for J^T with the transposed patch solves and relaxations. */
irk_status irk_mg_vcycle_transpose(irk_mg* h, const double* r, double* z, void* stream);

/* Solve J k = F by restarted FGMRES(restart) right-preconditioned with irk_mg_vcycle
 * (Sec. 4), modified Gram--Schmidt, stopping when the residual estimate is at most
 * rtol * ||F - J k0|| or after maxit iterations.  k holds k0 on entry and the solution
 * (pressure means removed) on exit.  Synchronises `stream`.  Returns IRK_ENOCONV when
 * maxit is reached, IRK_ENAN when a non-finite value appears.  info may be NULL. */
irk_status irk_fgmres_solve(irk_mg* h, const double* F, double* k, double rtol, int maxit,
                            int restart, irk_solve_info* info, void* stream);

/* Solve J^T lam = G the same way, preconditioned by irk_mg_vcycle_transpose.  G must
 * have zero pressure sum in every stage (the left null vectors of J^T). */
irk_status irk_adjoint_solve(irk_mg* h, const double* G, double* lam, double rtol, int maxit,
                             int restart, irk_solve_info* info, void* stream);

/* Right-hand side of the stage system (Sec. 3.1): F_i = [M f_i - L u - B p ; -B^T u]
 * with L = K (+C).  f: device, r x nnodes x dim (stage, node, component) nodal forcing
 * values at every P2 node of the finest level; state: device, ns values (u as in a
 * stage block of the ABI layout, then p). */
irk_status irk_rhs(irk_mg* h, const double* f, const double* state, double* F, void* stream);

/* Add the terms of prescribed (non-zero) boundary velocities to a right-hand side F
 * built by irk_rhs (Sec. 3.1 with Dirichlet data g(t); the paper does not say how the
 * data enter the stages: here every stage value equals the data at its stage time,
 * U_{i,b} = g(t_n + c_i dt), so the boundary stage derivatives are
 * k_b = (dt A)^{-1} (G - 1 (x) g(t_n)) and
 *   velocity rows:   F_i -= M_fb k_{i,b} + L_fb G_i,
 *   divergence rows: F_i -= B_b^T G_i.)
 * g_n: device, nnodes x dim (finest-level node numbering, values at t_n); g_stages:
 * device, r x nnodes x dim (values at t_n + c_i dt); only boundary nodes are read.
 * F: device, ndofs, ABI layout, updated in place.  The state passed to irk_rhs and
 * irk_update keeps free velocities only; the boundary values are g at that time.
 * Errors: IRK_EINVAL (null pointers, singular A), IRK_EHIP. */
irk_status irk_rhs_dirichlet(irk_mg* h, const double* g_n, const double* g_stages, double* F, void* stream);

/* state += dt * sum_j b_j k_j (the update of Sec. 3.1), state and k as above. */
irk_status irk_update(irk_mg* h, const double* k, double* state, void* stream);

/* Navier--Stokes stage equations and Newton's method (Sec. 3.2)
 * --------------------------------------------------------------
 * With inertia the velocity rows of stage i gain N(U_i), the discrete <U . grad U, v> at
 * the stage value U_i = u^n + dt sum_j a_ij k_j^u (free nodes; at boundary nodes the
 * stage data G_i of irk_rhs_dirichlet, or zero), so the stage system is nonlinear:
 *   G(k) = (I (x) M^ + dt A (x) S^_Stokes) k - F_Stokes + [N(U_i); 0]_i = 0.
 * These calls evaluate it on the finest level of a handle set up for the same mesh,
 * tableau, dt and nu, with any wind w (NULL: Stokes): F is the right-hand side that
 * irk_rhs (+ irk_rhs_dirichlet) builds on that handle, whose wind terms the calls cancel
 * (they add c(U_i - w, U_i) = N(U_i) - C(w) U_i).  The Newton Jacobian, block (i, j) =
 * delta_ij M^ + dt a_ij (S^ + N'(U_i)) with N'(U) z = c(z, U) + c(U, z), is not a
 * Kronecker product; it is applied matrix-free (two kernels: element vectors per cell
 * and stage, then a fixed-order sum per unknown) while the handle's V-cycle, built for
 * its own Kronecker operator (wind w), preconditions FGMRES.  state: device, free
 * velocities in the stage-block layout (the pressure part is not read); g_stages: device
 * r x nnodes x dim stage boundary data or NULL.  All vectors in the ABI layout.
 * Errors: IRK_EINVAL (null pointers, invalid options), IRK_ENAN (non-finite residual),
 * IRK_EHIP, IRK_ENOMEM (the first call allocates the element data, about
 * (nloc dim r + (dim+1) dim + nloc + 1) 8 ncells bytes, the stage values, nnodes dim r
 * doubles, and four vectors of ndofs doubles).  irk_ns_residual and irk_ns_jacobian_apply
 * are stream-ordered; irk_ns_newton_solve reads norms on the host and returns
 * synchronised. */

/* R = F - J_w k - c(U - w, U), i.e. -G(k). */
irk_status irk_ns_residual(irk_mg* h, const double* F, const double* state, const double* g_stages,
                           const double* k, double* R, void* stream);
/* y = G'(k) x, the Newton Jacobian at k applied to x. */
irk_status irk_ns_jacobian_apply(irk_mg* h, const double* state, const double* g_stages, const double* k,
                                 const double* x, double* y, void* stream);

/* Newton (Sec. 3.2): k <- k + delta with G'(k) delta = -G(k) solved by FGMRES (the
 * handle's V-cycle as preconditioner) from delta = 0 to the relative residual eta_l;
 * the forcing terms follow Eisenstat and Walker's choice 2, eta_0 = eta0,
 * eta_l = gamma (||G_l|| / ||G_{l-1}||)^alpha, raised to gamma eta_{l-1}^alpha when that
 * exceeds the threshold, capped at eta_max, and kept at least 0.5 tau / ||G_l|| (a
 * final-step safeguard against solving the last step far below what the stopping test
 * needs) with tau = max(atol, rtol ||G(k0)||) (the paper names the criterion only;
 * these constants are the defaults below); or eta_fixed when > 0.  Stops at
 * ||G|| <= tau.  k: initial guess in (the previous step's stages,
 * Sec. 3.2), solution out. */
typedef struct irk_newton_opts {
  double rtol, atol;    /* defaults 1e-8, 0                                         */
  int maxit;            /* Newton steps, default 20                                 */
  int linear_maxit;     /* FGMRES iterations per step, default 200                  */
  int restart;          /* FGMRES restart length, default 30                        */
  double eta0, eta_max; /* 0.3, 0.9 (both in (0, 1))                                */
  double ew_gamma;      /* 1 (in (0, 1])                                            */
  double ew_alpha;      /* (1 + sqrt 5) / 2 (in (1, 2])                             */
  double ew_threshold;  /* 0.1                                                      */
  double eta_fixed;     /* 0: Eisenstat--Walker; in (0, 1): this constant forcing    */
  int linesearch;       /* 1: backtracking line search on ||G|| (not in the paper;
                           default 0, full Newton steps): k + lam delta with the first
                           lam in 1, 1/2, ... (at most ls_maxit halvings) giving
                           ||G(k + lam delta)|| <= (1 - ls_alpha lam) ||G(k)||          */
  int ls_maxit;         /* 12 (0 .. 60)                                              */
  double ls_alpha;      /* 1e-4 (in (0, 1))                                          */
  int precond;          /* FGMRES preconditioner of the Newton steps: 0 (default) the
                           handle's own V-cycle, built for its Kronecker operator; 1 the
                           V-cycle of the Newton Jacobian itself, rebuilt at every Newton
                           iterate (irk_ns_newton_preconditioner; FP64 handles only)      */
} irk_newton_opts;
/* history (host, may be NULL): ||G|| before each step and at exit; etas, linear_its and
 * lambdas (host, may be NULL): each step's forcing term, FGMRES iterations and step
 * length; all hold at most history_cap values. */
typedef struct irk_newton_info {
  int iterations, converged, linear_iterations;
  double norm0, norm;   /* ||G(k0)|| and ||G|| at exit                              */
  double* history;
  double* etas;
  int* linear_its;
  int history_cap;
  double ms_linear;     /* GPU time of the linear solves                            */
  double ms_wall;       /* host wall time of the call (returns synchronised)        */
  double* lambdas;
} irk_newton_info;
void irk_newton_default_opts(irk_newton_opts* opt);
/* Returns IRK_OK, IRK_ENOCONV (maxit Newton steps without convergence, or no step length
 * of the line search gave sufficient decrease; k holds the last accepted iterate) or an
 * error. */
irk_status irk_ns_newton_solve(irk_mg* h, const double* F, const double* state, const double* g_stages,
                               double* k, const irk_newton_opts* opt, irk_newton_info* info, void* stream);

/* The V-cycle of the Newton Jacobian (Sec. 3.2): block (i, j) = delta_ij M^ +
 * dt a_ij [K + N'(U_i) B; B^T 0], not a Kronecker product, rediscretised on every level
 * at the stage velocities U_i of (state, k, g_stages) (as for irk_ns_residual) carried to
 * the coarser levels by injection at their P2 nodes (which are nodes of the next finer
 * level).  enable = 1 assembles the per-stage velocity blocks of every level,
 * factorises the stage-coupled patch matrices of every level in the dense form and
 * inverts the coarse operator (all on the GPU; the coarsest level's blocks pass through
 * the host for its dense operator), and switches the handle's V-cycle
 * (irk_mg_vcycle, irk_level_sweep, irk_level_apply, irk_coarse_solve, and the
 * preconditioner of irk_fgmres_solve) to these operators; enable = 0 switches back to
 * the handle's own operator (state, g_stages and k are then not read).  FP64 handles
 * only; no transposed form while enabled (IRK_EINVAL).  The first call allocates the
 * per-stage blocks (r dim^2 doubles per entry of each level's scalar pattern, and again
 * in the sliced order of the residual kernel), the element data of every level, the dense
 * patch inverses (sum over patches of (r n_v)^2 doubles per level) and three dense
 * coarse matrices.  Synchronises `stream`.  Errors: IRK_EINVAL, IRK_ESINGULAR (zero
 * pivot), IRK_ENOMEM, IRK_EHIP. */
irk_status irk_ns_newton_preconditioner(irk_mg* h, const double* state, const double* g_stages, const double* k,
                                        int enable, void* stream);

/* Adjoint building blocks (transposes of the maps above; used to differentiate a
 * sequence of IRK steps with respect to the forcing, the viscosity and the state).
 * irk_rhs_adjoint: the transpose of (f, state) -> F of irk_rhs: given lam (ABI layout),
 *   gf (device, r x nnodes x dim, overwritten) = M_fa^T lam_i^u per stage and component,
 *   gstate (device, ns) = [-L^T sum_i lam_i^u - B sum_i lam_i^p ; -B^T sum_i lam_i^u],
 *   overwritten (accumulate = 0) or added to it (accumulate = 1: the reverse sweep's
 *   state adjoint gbar_n = gbar_{n+1} + (dF/dstate)^T lam^n in place).
 * irk_update_adjoint: the transpose of irk_update with respect to k: G_i = dt b_i gstate
 *   (G in the ABI layout, overwritten).
 * irk_nu_sensitivity: out (device, one double) =
 *   lam^T (dF/dnu - dJ/dnu k) = -sum_i lam_i^u . (K_1 u) - dt sum_ij a_ij lam_i^u . (K_1 k_j^u),
 *   K_1 the vector P2 Laplacian with nu = 1 and u the velocity of `state`
 *   (F and J depend on nu through K = nu K_1; the convection term does not);
 *   overwritten (accumulate = 0) or added to *out (accumulate = 1: summing the steps).
 * irk_mass_apply: out (ns) = [M u ; 0] for a state vector (velocity mass).
 * irk_tracking_loss: the misfit of a state to a target, L = 1/2 e^T M e with e the
 *   velocity part of state - target (state, target: device, ns values; the pressure is
 *   not compared).  loss (device, one double, may be NULL) receives L; grad_state and
 *   grad_target (device, ns, may be NULL) receive s [M e ; 0] and -s [M e ; 0], the
 *   gradients of s L, with s = *scale (device, one double; NULL means 1).  At least
 *   one output must be given.  Uses the handle's workspace (stream-ordered).
 * The accumulate flags take 0 or 1 (else IRK_EINVAL). */
irk_status irk_rhs_adjoint(irk_mg* h, const double* lam, double* gf, double* gstate, int accumulate,
                           void* stream);
irk_status irk_update_adjoint(irk_mg* h, const double* gstate, double* G, void* stream);
irk_status irk_nu_sensitivity(irk_mg* h, const double* lam, const double* k, const double* state,
                              double* out, int accumulate, void* stream);
irk_status irk_mass_apply(irk_mg* h, const double* state, double* out, void* stream);
irk_status irk_tracking_loss(irk_mg* h, const double* state, const double* target, const double* scale,
                             double* loss, double* grad_state, double* grad_target, void* stream);

/* Per-level building blocks, exposed so that each step of the cycle can be checked on
 * its own.  Vectors use the ABI layout of the level named. */
/* y = J_l x or J_l^T x on level l. */
irk_status irk_level_apply(irk_mg* h, int level, int transpose, const double* x, double* y,
                           void* stream);
/* One additive Vanka sweep on level l >= 1 (Sec. 4.2): k <- k + omega W sum_v R_v^T
 * A_v^{-1} R_v (F - J_l k); transpose = 1 gives the transposed sweep for J_l^T.  With
 * smoother 1 it is one Chebyshev step, with smoother 2 one GMRES step (the relaxation
 * the handle uses, with one step). */
irk_status irk_level_sweep(irk_mg* h, int level, int transpose, const double* F, double* k,
                           void* stream);
/* xc = (I_r (x) P_l)^T xf: restriction from level l >= 1 to level l-1 (Sec. 4.1). */
irk_status irk_level_restrict(irk_mg* h, int level, const double* xf, double* xc, void* stream);
/* xf += (I_r (x) P_l) xc: prolongation from level l-1 to level l >= 1 (Sec. 4.1). */
irk_status irk_level_prolong(irk_mg* h, int level, const double* xc, double* xf, void* stream);
/* x = J_0^{-1} b on the coarsest level with pinned pressures (transpose: J_0^{-T}). */
irk_status irk_coarse_solve(irk_mg* h, int transpose, const double* b, double* x, void* stream);

/* Batched solves in one persistent launch.  irk_batch_create groups n FP64 2D handles
 * (distinct, set up independently, of any sizes and stage counts, patches of at most
 * 256 unknowns); each call of
 * irk_batch_fgmres_solve then runs the whole FGMRES solve of every handle -- the same
 * algorithm as irk_fgmres_solve: layout conversion, residuals, V-cycles, Gram--Schmidt,
 * Givens updates, solution update and projection -- inside ONE persistent kernel in
 * which workgroups take work items of any unfinished solve.  F[q] and k[q] are device
 * vectors of handle q (ABI layout); k[q] is the initial guess on entry.  infos[q]
 * (may be NULL) gets iterations, convergence and the recomputed relative residual;
 * latency_ms[q] (may be NULL) the device-clock time from the start of the launch to
 * the moment solve q finished.  Returns IRK_ENOCONV if some solve reached maxit,
 * IRK_ENAN on a non-finite value.  restart <= 64.
 * Schedule (irk_batch_opts): rows_per_item (x256 rows or vector entries per work
 * item), patches_per_wave (patches one wavefront takes per item; 4 wavefronts per
 * item), workgroups_per_cu (resident workgroups per compute unit), autotune (1: the
 * first solve call times 2-iteration trial runs of a grid of schedules, writing to
 * scratch, and keeps the fastest; irk_batch_get_opts reports the choice).  Every wait
 * in the kernel is bounded: a workgroup that finds no work for a long time aborts the
 * launch and the call returns IRK_EHIP. */
typedef struct irk_batch irk_batch;
typedef struct irk_batch_opts {
  int rows_per_item;
  int patches_per_wave;
  int workgroups_per_cu;
  int autotune;
  int mode;     /* 0: one persistent launch; 1: concurrent streams: `streams` host
                   threads, each with its own HIP stream, take whole solves (largest
                   first) and run irk_fgmres_solve on them (any handle: FP32, 3D,
                   Chebyshev; the persistent kernel needs FP64 2D damped-sweep handles
                   with patches of <= 256 unknowns, else mode 1 is used) */
  int streams;  /* 1..16; 1 is the one-by-one baseline.  Autotuning times streams
                   1, 2, 4, 8 and the persistent tiles and keeps the fastest */
} irk_batch_opts;
void irk_batch_default_opts(irk_batch_opts* opt);
irk_status irk_batch_create(irk_mg* const* solves, int n, const irk_batch_opts* opt, void* stream,
                            irk_batch** out);
irk_status irk_batch_fgmres_solve(irk_batch* b, const double* const* F, double* const* k, double rtol,
                                  int maxit, int restart, irk_solve_info* infos, double* latency_ms,
                                  void* stream);
irk_status irk_batch_get_opts(const irk_batch* b, irk_batch_opts* out);
void irk_batch_destroy(irk_batch* b);

/* Measurement of the V-cycle kernels.  irk_mg_profile(h, mode) with mode 1..3 clears
 * the counters and brackets later launches with HIP events on the stream they are
 * launched on: mode 1 only the finest level's patch apply (least intrusive), mode 2
 * every kernel below on the finest level, mode 3 on every level; irk_mg_profile(h, 0)
 * stops recording (IRK_EINVAL for other modes).  irk_mg_kernel_stats waits for the
 * recorded events and reports, for one kernel on one level (-1: finest), the number
 * of launches, their summed GPU time and the algorithmic bytes one launch moves:
 *   kernel 0  patch apply:   stored patch factors (sum_v n_v^2 values dense,
 *                            sum_v r n_s^2 factored) + one read of the residual
 *                            (N values) + the local corrections written (sum_v n_v);
 *   kernel 1  residual:      scalar P2 blocks (column index + M + L per entry), B and
 *                            B^T (index + dim values per entry), F and x read, r written;
 *   kernel 2  gather update: local corrections and their slot indices read, x read and
 *                            written, weights read;
 *   kernel 3  Navier--Stokes element vectors (finest level, Jacobian mode): cell nodes,
 *                            their free indices and the geometry, stage values and wind once per node, the
 *                            direction once, element vectors written (FP64);
 *   kernel 4  Navier--Stokes gather: incidence lists, the element entries of free
 *                            nodes, y read and written.
 * Values are 8 bytes (FP64 mode) or 4 bytes (FP32 mode), indices 4 bytes. */
typedef struct irk_kernel_stats {
  int64_t launches;
  double ms_total;
  double bytes_per_launch;
} irk_kernel_stats;
irk_status irk_mg_profile(irk_mg* h, int enable);
irk_status irk_mg_kernel_stats(irk_mg* h, int kernel, int level, irk_kernel_stats* out);

/* Description of the last error on the calling thread ("" if none). */
const char* irk_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IRK_MG_H */
