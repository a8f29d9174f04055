// Internal structures of libirkmg: host-side level data built at setup, the device
// copies the kernels read, and the launchers the driver calls.
//
// Internal vector layout of a level (device only; the ABI layout is converted at the
// boundary): velocity first, node-major with component and stage innermost,
//   V[(i * dim + c) * r + s]        i < nfree, c < dim, s < r
// then pressure, vertex-major with stage innermost,
//   P[offV + v * r + s]             offV = nfree * dim * r.
// Every sparse operator reads the dim*r (or r) values of a node as one contiguous
// chunk, so one CSR traversal serves all stages and components (the Kronecker
// structure is never expanded).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <exception>
#include <string>
#include <complex>
#include <thread>
#include <vector>

namespace irk {

constexpr int kMaxStages = 4;
// most GMRES relaxation steps per cycle (smoother 2)
constexpr int kMaxGr = 8;

// Sliced copy of a CSR operator for the residual kernel: rows in slices of 64, each slice
// padded to its longest row, entries of a slice stored column-major (entry k of the 64
// rows contiguous) so that a wavefront reads its rows' k-th entries in one coalesced
// access.  src[e] is the CSR position of sliced entry e, or -1 for padding (column 0,
// value 0).
struct Sell {
  int64_t nslices = 0;
  std::vector<int32_t> off, w, col;  // entry offset and width of each slice, columns
  std::vector<int64_t> src;
};
Sell build_sell(int64_t nrows, const std::vector<int32_t>& ptr, const std::vector<int32_t>& col);
// Values of a CSR value array (k values per entry) in the sliced order.
std::vector<double> sell_values(const Sell& S, const std::vector<double>& v, int k);

// ----------------------------------------------------------------- host level data
struct HostLevel {
  int dim = 0;
  int64_t nv = 0, nc = 0, ne = 0, nn = 0, nfree = 0;
  std::vector<double> xyz;          // nv x dim
  std::vector<int64_t> cells;       // nc x (dim+1)
  std::vector<int64_t> edges;       // ne x 2
  std::vector<int64_t> cell_nodes;  // nc x nloc (vertices, then local edges)
  std::vector<int32_t> free_of_node, node_of_free;
  std::vector<int32_t> node_cell_ptr, node_cell;  // node -> cells containing it

  // scalar P2 operators on free x free: mass M, L = nu K (+ C), and L^T on the
  // same (symmetric) pattern
  std::vector<int32_t> s_ptr, s_col;
  std::vector<double> s_M, s_L, s_Lt, s_K1;  // s_K1: Laplacian with nu = 1
  // weak gradient B (free node x vertex, dim values per entry) and its transpose
  std::vector<int32_t> b_ptr, b_col;
  std::vector<double> b_val;
  std::vector<int32_t> bt_ptr, bt_col;
  std::vector<double> bt_val;
  // free-row x all-node mass (forcing term of the right-hand side)
  std::vector<int32_t> mfa_ptr, mfa_col;
  std::vector<double> mfa_val;
  // prescribed boundary velocities (finest level): free rows x boundary nodes (M and L
  // values) and vertex rows x boundary nodes (B^T, dim values per entry)
  std::vector<int32_t> fb_ptr, fb_col, vb_ptr, vb_col;
  std::vector<double> fb_m, fb_l, vb_val;

  // vertex-star patches: free nodes of each patch (ascending) and the CSR entries
  // that couple them
  std::vector<int32_t> pn_ptr, pn_node;
  std::vector<int32_t> pvv_ptr, pvv;  // triples (local a, local b, scalar CSR pos)
  std::vector<int32_t> pvp;           // per patch node: B CSR pos of (node, vertex)

  // transfers from the next coarser level (fine rows): scalar P2 on free nodes,
  // P1 on vertices, and their transposes (coarse rows)
  std::vector<int32_t> pu_ptr, pu_col, put_ptr, put_col;
  std::vector<double> pu_val, put_val;
  std::vector<int32_t> pp_ptr, pp_col, ppt_ptr, ppt_col;
  std::vector<double> pp_val, ppt_val;
  std::vector<int64_t> coarse_node_to_fine_vertex;  // injection (wind)

  // sliced copies for the residual: velocity rows x free nodes (M, L, L^T), velocity
  // rows x vertices (B), vertex rows x free nodes (B^T)
  Sell sell_s, sell_b, sell_bt;
};

// Element reference tensors (integrals over the cell divided by its measure).
void build_topology(HostLevel& L, int dim, int64_t nv, int64_t nc, const double* xyz,
                    const int64_t* cells);
void assemble_level(HostLevel& L, double nu, const std::vector<double>* wind_nodal,
                    bool with_mfa);
void build_patches(HostLevel& L);

// body(lo, hi) over contiguous ranges of [0, n) on up to 16 host threads, at least `grain`
// items each; the ranges partition [0, n) in order.  An exception thrown by a range is
// rethrown on the calling thread after every range has finished.
template <typename F>
void parallel_ranges(int64_t n, F&& body, int64_t grain = 4096) {
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>({16, (int64_t)std::thread::hardware_concurrency(),
                                                              n / grain}));
  if (nt == 1) {
    body((int64_t)0, n);
    return;
  }
  std::vector<std::exception_ptr> err(nt);
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&body, &err, n, nt, t] {
      try {
        body(n * t / nt, n * (t + 1) / nt);
      } catch (...) {
        err[t] = std::current_exception();
      }
    });
  for (auto& th : pool) th.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
}
// Cells grouped so that no two cells of a group share a vertex (greedy, in cell order).
// Every row that a cell's element matrices touch belongs to one of its vertices or edges,
// so the cells of one group scatter into disjoint rows and can be assembled concurrently.
// Group g holds cells[gptr[g] .. gptr[g+1]), ascending.  A mesh needing more than 64
// groups (more than 64 cells around some vertex) gets one group of every cell, which
// callers then assemble on one thread.
void vertex_disjoint_groups(const HostLevel& L, std::vector<int64_t>& gptr, std::vector<int64_t>& cells);
// Scatter cell_body(c) over every cell, group by group (vertex_disjoint_groups).
template <typename F>
void for_cells_by_groups(const HostLevel& L, F&& cell_body) {
  std::vector<int64_t> gptr, cells;
  vertex_disjoint_groups(L, gptr, cells);
  if (gptr.size() == 2 && L.nc > 1) {  // one group: cells may share vertices
    for (int64_t c = 0; c < L.nc; ++c) cell_body(c);
    return;
  }
  for (size_t g = 0; g + 1 < gptr.size(); ++g)
    parallel_ranges(gptr[g + 1] - gptr[g], [&](int64_t i0, int64_t i1) {
      for (int64_t i = i0; i < i1; ++i) cell_body(cells[gptr[g] + i]);
    }, 256);
}
// Element data of the Navier--Stokes terms: per cell the barycentric gradients
// ((dim+1) x dim) and the measure; int32 cell nodes and their free indices (-1 for
// prescribed nodes); per free node the incidences cell * nloc + a (cell order) of its node.
void ns_cell_data(const HostLevel& L, std::vector<double>& geo, std::vector<int32_t>& cell_nodes,
                  std::vector<int32_t>& cell_free, std::vector<int32_t>& inc_ptr, std::vector<int32_t>& inc);
// Returns an empty string on success, else a description of the nesting failure.
std::string build_transfer(const HostLevel& coarse, HostLevel& fine, const int64_t* parent);
// Dense coarse operator (row-major N x N, internal layout) with the pressure of vertex 0
// pinned in every stage; *max_abs = its largest entry in magnitude.
void coarse_matrix(const HostLevel& L, int r, const double* A, double dt, std::vector<double>& J,
                   double* max_abs);
// Per-stage velocity operator of the Newton Jacobian for one stage velocity U (nodal,
// nn x dim): adds (nu K + C(U)) delta_ce + R(U)_ce to out[p dim^2 + c dim + e] for every
// entry p of the scalar pattern.
void assemble_newton_block(const HostLevel& L, double nu, const double* U, double* out);
// Dense coarse Newton Jacobian (row-major, pinned pressures) from the per-stage blocks
// nw[(p r + s) dim^2 + c dim + e].
void coarse_matrix_newton(const HostLevel& L, int r, const double* A, double dt, const double* nw,
                          std::vector<double>& J, double* max_abs);

// ------------------------------------------------------------- stage eigenbasis
// Real block diagonalisation A = W T W^{-1} of the Butcher matrix.  T is block diagonal
// with 1x1 blocks (real eigenvalues) and 2x2 blocks [[a, b], [-b, a]] (pairs a +- ib,
// b > 0).  Since every stage-coupled patch matrix has the Kronecker form
// I (x) M_v + dt A (x) S_v (the stage operator of Sec. 3 restricted to one patch), its
// inverse is (W (x) I) blockdiag_k (I (x) M_v + dt T_k (x) S_v)^{-1} (W^{-1} (x) I):
// the same operator, stored as r blocks of n_s^2 values instead of (r n_s)^2.
struct StageEig {
  int r = 0, nblk = 0;
  int type[kMaxStages] = {0};  // stages spanned by the block: 1 (real) or 2 (pair)
  int st0[kMaxStages] = {0};   // first transformed stage of the block
  double Tb[kMaxStages][4] = {{0}};  // the block of T, row-major type x type
  double W[kMaxStages * kMaxStages] = {0};
  double Winv[kMaxStages * kMaxStages] = {0};  // row-major r x r
  double cond = 0;   // ||W||_inf ||W^{-1}||_inf
  double recon = 0;  // max |W T W^{-1} - A|
};
// Returns false (with the reason in *why) when A has no well-conditioned real block
// diagonalisation (repeated or defective eigenvalues, cond(W) > 1e6).
bool stage_eigenbasis(const double* A, int r, StageEig& out, std::string* why);
// Eigenvalues of the leading m x m block of an upper Hessenberg matrix (column-major,
// leading dimension ldh) by the shifted QR iteration in complex arithmetic (Givens
// rotations, Wilkinson shifts, deflation at negligible subdiagonal entries), sorted by
// decreasing real part.  False if the iteration does not converge.
bool hessenberg_eigs(int m, const double* H, int ldh, double* wr, double* wi);
// the same with caller storage: work holds m*m + 3m complex values, iwork m ints
bool hessenberg_eigs_ws(int m, const double* H, int ldh, double* wr, double* wi, std::complex<double>* work,
                        int* iwork);

// Stored values per column of one eigen-block of a factored patch inverse: a real block
// keeps its n_s entries, a pair keeps n_s complex entries (re, im interleaved); both
// padded to whole 16-byte vectors of `vec` elements.
__host__ __device__ inline int eig_block_rows(int type, int ns, int vec) {
  return type == 1 ? (ns + vec - 1) / vec * vec : 2 * ((ns + vec / 2 - 1) / (vec / 2) * (vec / 2));
}

// Symmetric factored form (a symmetric spatial operator, Stokes): each block inverse Z
// (n_s x n_s, real or complex symmetric) is kept as its wrapped diagonals
// Z(i, (i + s) mod n_s), s = 0 .. n_s/2, which hold every entry at least once, in
// descending order: with G = sym_group and ng = sym_words diagonals per word and words
// per row, word (g, i), 16 bytes, holds row i's entries on the diagonals
// s = ng G - 1 - g G - k, k = 0 .. G-1 (a pair entry as re, im); diagonals past n_s/2
// are zero.  Word (g, i) sits at value offset (g * n_s + i) * vec, so one 16-byte load
// per lane reads word g of every row.
__host__ __device__ inline int sym_diags(int ns) { return ns / 2 + 1; }
__host__ __device__ inline int sym_group(int type, int vec) { return type == 1 ? vec : vec / 2; }
__host__ __device__ inline int sym_words(int type, int ns, int vec) {
  const int G = sym_group(type, vec);
  return (sym_diags(ns) + G - 1) / G;
}
__host__ __device__ inline int64_t sym_block_values(int type, int ns, int vec) {
  return (int64_t)sym_words(type, ns, vec) * ns * vec;
}

// The basis as the patch kernels read it (by value, in the working precision).
template <typename T>
struct StageBasis {
  int r = 0, nblk = 0;
  int type[kMaxStages] = {0};
  int st0[kMaxStages] = {0};
  T W[kMaxStages * kMaxStages] = {0};
  T Winv[kMaxStages * kMaxStages] = {0};
};

// ---------------------------------------------------------------- device level data
template <typename T>
struct DevOps {
  T* s_M = nullptr;
  T* s_L = nullptr;
  T* s_Lt = nullptr;
  T* b_val = nullptr;
  T* bt_val = nullptr;
  T* pu_val = nullptr;
  T* put_val = nullptr;
  T* pp_val = nullptr;
  T* ppt_val = nullptr;
  T* W = nullptr;  // per internal DOF weight of the additive correction
  // values of the sliced operators (residual kernel)
  T *u_M = nullptr, *u_L = nullptr, *u_Lt = nullptr, *u_B = nullptr, *p_Bt = nullptr;
};

struct DevLevel {
  int dim = 0, r = 0;
  int64_t nv = 0, nfree = 0, N = 0, offV = 0;
  int32_t *s_ptr = nullptr, *s_col = nullptr;
  int32_t *b_ptr = nullptr, *b_col = nullptr, *bt_ptr = nullptr, *bt_col = nullptr;
  int32_t *pu_ptr = nullptr, *pu_col = nullptr, *put_ptr = nullptr, *put_col = nullptr;
  int32_t *pp_ptr = nullptr, *pp_col = nullptr, *ppt_ptr = nullptr, *ppt_col = nullptr;
  int32_t *mfa_ptr = nullptr, *mfa_col = nullptr;
  double* mfa_val = nullptr;
  int32_t *mfat_ptr = nullptr, *mfat_col = nullptr;  // M_fa^T (node rows)
  double* mfat_val = nullptr;
  double* s_K1 = nullptr;
  int32_t *fb_ptr = nullptr, *fb_col = nullptr, *vb_ptr = nullptr, *vb_col = nullptr;
  double *fb_m = nullptr, *fb_l = nullptr, *vb_val = nullptr;
  int64_t nnodes = 0;
  DevOps<double> d64;
  DevOps<float> d32;
  // sliced operator indices (see Sell): velocity slices, then vertex slices
  int64_t nsl_u = 0, nsl_p = 0;
  int32_t *su_off = nullptr, *su_w = nullptr, *su_col = nullptr;
  int32_t *sb_off = nullptr, *sb_w = nullptr, *sb_col = nullptr;
  int32_t *sp_off = nullptr, *sp_w = nullptr, *sp_col = nullptr;

  // patches
  int64_t npatch = 0;
  int32_t* p_nloc = nullptr;     // r * (dim * nn + 1)
  int32_t* p_ld = nullptr;       // leading dimension of the stored inverse
  int64_t* p_inv_off = nullptr;  // element offset of the inverse
  int64_t* p_slot_off = nullptr; // offset of the patch's output slots
  int32_t* p_gidx = nullptr;     // concatenated local -> internal DOF index
  int32_t* p_nn = nullptr;
  int32_t* p_vertex = nullptr;
  int32_t *pvv_ptr = nullptr, *pvv = nullptr, *pvp = nullptr, *pn_ptr = nullptr;
  int32_t *gat_ptr = nullptr, *gat_slot = nullptr;  // DOF -> its patch slots
  // the same lists sliced (Sell layout; padding -> slot `slots`, which stays zero)
  int64_t nsl_g = 0;
  int32_t *g_off = nullptr, *g_w = nullptr, *g_slot = nullptr;
  void* inv = nullptr;                              // double or float inverses
  int64_t inv_elems = 0, slots = 0;
  int max_nloc = 0;
  int32_t* sched = nullptr;  // patch launch order (largest first)
  // patch form: 0 = dense inverse of the stage-coupled patch matrix (column-major,
  // n x ld); 1 = factored through the stage eigenbasis: n_s columns of ld = sum over
  // blocks of eig_block_rows values each (p_ld holds that column length)
  // 3 = symmetric factored (Stokes, n_s <= 64): each block inverse kept by its wrapped
  // diagonals (sym_block_values); factorised in the form-1 layout, whose offsets
  // p_full_off and size full_elems are kept for that step
  int pform = 0;
  int max_ld = 0;
  int64_t* p_full_off = nullptr;
  int64_t full_elems = 0;
  StageBasis<double> sb64;
  StageBasis<float> sb32;

  // algorithmic bytes per launch of patch apply, residual and gather update
  double alg_bytes[5] = {0, 0, 0, 0, 0};

  // work vectors (internal layout) in the working precision
  void *b = nullptr, *x = nullptr, *res = nullptr, *Y = nullptr;
  void* dch = nullptr;  // Chebyshev direction vector
  void* grv = nullptr;  // GMRES relaxation basis: (steps + 1) vectors of N
};

struct Handle {
  int dim = 0, r = 0, nlevels = 0, precision = 0;
  double dt = 0, nu = 0, omega = 0.5;
  int pre = 2, post = 2, weighting = 1;
  int patch_form = 0;  // form in use: 0 dense, 1 stage eigenbasis, 3 symmetric eigenbasis
  int patch_form_req = 2;  // the requested form (2 = automatic)
  int smoother = 0;    // 0 damped sweeps, 1 Chebyshev on [cheb_lo, cheb_hi]
  double cheb_lo = 2.0, cheb_hi = 8.0;
  StageEig eig;
  double A[kMaxStages * kMaxStages] = {0}, At[kMaxStages * kMaxStages] = {0};
  double b[kMaxStages] = {0}, c[kMaxStages] = {0};
  double Ainv_dt[kMaxStages * kMaxStages] = {0};  // (dt A)^{-1}, row-major
  bool A_invertible = false;
  std::vector<HostLevel> host;
  std::vector<DevLevel> dev;
  double* coarse_inv = nullptr;   // column-major, internal layout
  double* coarse_invT = nullptr;  // column-major inverse of the transpose
  double* coarse_mat = nullptr;   // the pinned coarse operator, column-major
  double* coarse_matT = nullptr;  // its transpose, column-major
  double *cb = nullptr, *cx = nullptr;  // FP64 coarse vectors
  double* cpart = nullptr;               // coarse GEMV partial sums
  // FGMRES workspace (finest level, internal layout, FP64)
  int krylov_cap = 0;
  double *kv = nullptr, *kz = nullptr, *kw = nullptr, *kF = nullptr, *kx = nullptr,
         *kr = nullptr;
  double* scal = nullptr;      // device scalars (dot results)
  double* partials = nullptr;  // reduction partials
  double* gr = nullptr;        // GMRES relaxation: Hessenberg, norms, coefficients
  double* grpart = nullptr;    // GMRES relaxation: per-block partial sums
  double* hbuf = nullptr;      // device Hessenberg column
  std::vector<void*> allocations;
  int64_t* pins = nullptr;  // device: pinned coarse pressure DOFs (one per stage)
  int* flag = nullptr;      // device: error flag of the factorisation kernels
  // measurement mode: event pairs around kernel launches
  struct ProfEv {
    hipEvent_t a = nullptr, b = nullptr;
    int kernel = 0, level = 0;
  };
  bool prof = false;
  int prof_mode = 3;
  std::vector<ProfEv> prof_pool;
  size_t prof_used = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr, ev4 = nullptr, ev5 = nullptr,
             evh = nullptr;
  double* hpin = nullptr;  // pinned host: FGMRES Hessenberg column and update coefficients
  // Navier--Stokes (Newton) data of the finest level, built at first use
  std::vector<double> wind_fine;  // host copy of the finest-level wind (empty: none)
  bool ns_ready = false;
  bool ns_jac = false;  // FGMRES operator = the Newton Jacobian at ns_U
  int32_t *ns_cells = nullptr, *ns_cell_free = nullptr, *ns_free = nullptr, *ns_inc_ptr = nullptr,
          *ns_inc = nullptr;
  double *ns_geo = nullptr, *ns_w = nullptr, *ns_U = nullptr, *ns_elem = nullptr;
  double *ns_k = nullptr, *ns_kt = nullptr, *ns_F = nullptr, *ns_G = nullptr;  // iterate, trial, rhs, residual
  // Newton Jacobian preconditioner (Sec. 3.2): per level the per-stage velocity blocks
  // N_s = K + N'(U_s) on the scalar pattern ((p r + s) dim^2 + c dim + e), and on levels
  // >= 1 the dense inverses of the stage-coupled patch matrices with their layout; the
  // coarse inverse and pinned operator (column-major) with scratch for their set-up.
  // Allocated on first use; nw_active switches the V-cycle to these operators.
  bool nw_active = false, nw_ready = false;
  std::vector<double*> nw_vals, nw_inv;
  std::vector<double*> nw_sl;     // the blocks in the sliced order of each level (residual)
  std::vector<int32_t*> nw_src;   // CSR position of each sliced entry of the velocity operator
  std::vector<int32_t*> nw_ld;
  std::vector<int64_t*> nw_off;
  double *nw_cinv = nullptr, *nw_cmat = nullptr, *nw_ctmp = nullptr, *nw_colk = nullptr;
  int64_t* nw_swp = nullptr;
  // their assembly on the GPU: per level the element data of ns_cell_data, the stiffness
  // values on the scalar pattern, the stage velocities at the P2 nodes ((node dim + c) r
  // + s; the finest level's are ns_U) and, below the finest level, the fine vertex of each
  // P2 node; the reference tensor int phi_e phi_a d_k phi_b / |T|
  std::vector<double*> nwa_geo, nwa_K1, nwa_U;
  std::vector<int32_t*> nwa_cn, nwa_cf, nwa_inc_ptr, nwa_inc, nwa_c2f;
  double* nwa_C = nullptr;
};

// ------------------------------------------------------------------------ launchers
// All launchers enqueue on `s` and return hipGetLastError().
namespace k {
template <typename T>
hipError_t residual(const DevLevel& L, const DevOps<T>& ops, const double* A, double dt,
                    const T* F, const T* x, T* y, hipStream_t s);
template <typename T>
hipError_t patch_apply(const DevLevel& L, const DevOps<T>& ops, const T* res, T* Y,
                       int transpose, hipStream_t s);
template <typename T>
hipError_t gather_update(const DevLevel& L, const DevOps<T>& ops, const T* Y, T* x, T omega,
                         int mode, hipStream_t s);
// Chebyshev step: d = c1 d + c2 W sum(slots) (d not read when first; W omitted when
// transpose), x = d (xzero) or x + d.
template <typename T>
hipError_t gather_cheb(const DevLevel& L, const DevOps<T>& ops, const T* Y, T c1, T c2, int first, int xzero,
                       int transpose, T* d, T* x, hipStream_t s);
// F += terms of prescribed boundary velocities (finest level, ABI layout): velocity
// rows -M_fb k_{i,b} - L_fb G_i with k_b = (dt A)^{-1}(G - 1 (x) g_n), divergence rows
// -B_b^T G_i; g_n (nnodes x dim) and g_st (r x nnodes x dim) are node arrays.
hipError_t rhs_dirichlet(const DevLevel& L, const double* Ainv_dt, const double* g_n, const double* g_st,
                         double* F, hipStream_t s);
template <typename T>
hipError_t restrict_(const DevLevel& fine, const DevLevel& coarse, const DevOps<T>& fops,
                     const T* xf, T* xc, hipStream_t s);
template <typename T>
hipError_t prolong_add(const DevLevel& fine, const DevLevel& coarse, const DevOps<T>& fops,
                       const T* xc, T* xf, hipStream_t s);
// Factorise (invert) patches [p0, p1) with an R-stage coefficient matrix coef
// (I (x) M_v + dt coef (x) S_v; R = r and coef = A for the dense form, R = 1 or 2 and
// coef = a block of T for one eigen-block); inverse of patch p written column-major
// (n x ld[p]) at out + off[p] - off0.  nmax: the largest n in the range.  nw (dense form
// only, R = r, coef = A): the Newton Jacobian's per-stage velocity blocks (see
// residual_newton) replace the Kronecker velocity block.
template <typename T>
hipError_t patch_factor_range(const DevLevel& L, const DevOps<T>& ops, int R, const double* coef,
                              double dt, const int32_t* ld, const int64_t* off, T* out, int64_t p0,
                              int64_t p1, int64_t off0, int nmax, int* d_fail, hipStream_t s,
                              const T* nw = nullptr);
// r = F - J x (F null: J x) on a level for the Newton Jacobian of the Navier--Stokes stage
// equations, block (s, t) = delta_st M + dt a_st [N_s B; B^T 0], with N_s = K + N'(U_s)
// as dim x dim blocks on the scalar pattern, nw[(p r + s) dim^2 + c dim + e] at CSR
// position p, given in the sliced order of the level's velocity operator (sell_blocks
// with k = r dim^2) (FP64).
hipError_t residual_newton(const DevLevel& L, const double* nws, const double* A, double dt, const double* F,
                           const double* x, double* y, hipStream_t s);
// out = the values v (k per CSR entry) in the sliced order, value q of sliced entry e at
// ((e / 64) k + q) 64 + e mod 64; src[e] is the CSR position of sliced entry e (-1: padding,
// value 0); ne sliced entries (a multiple of 64)
hipError_t sell_blocks(int64_t ne, int k, const int32_t* src, const double* v, double* out, hipStream_t s);
// Complex eigenvalue pair block b (a + ib): invert C = M_v + dt (a - ib) S_v per patch in
// LDS and write (Re, Im) of C^{-1} into the factored layout; zr = dt a, zi = -dt b.
// hipErrorInvalidConfiguration when the n_s x n_s complex matrix does not fit in LDS.
template <typename T>
hipError_t patch_factor_cplx(const DevLevel& L, const DevOps<T>& ops, double zr, double zi, int b, int nmax,
                             int* d_fail, hipStream_t s);
// Copy eigen-block b of patches [p0, p1) from dense inverses (layout of
// patch_factor_range with tmp_ld / tmp_off / off0) into the factored layout of L.inv.
template <typename T>
hipError_t pack_sym(const DevLevel& L, const int64_t* full_off, const T* full, hipStream_t s);
template <typename T>
hipError_t eig_extract(const DevLevel& L, const StageBasis<T>& sb, int b, const int32_t* tmp_ld,
                       const int64_t* tmp_off, int64_t off0, const T* tmp, int64_t p0, int64_t p1,
                       hipStream_t s);
// In-place inverse of a dense row-major N x N matrix on the device by Gauss--Jordan with
// partial pivoting (ties to the smaller row); a pivot below tol sets *fail.  colk:
// N-value workspace, swp: N-entry workspace.
hipError_t dense_inverse(double* J, int64_t N, double tol, double* colk, int64_t* swp, int* fail, hipStream_t s);
// out (N x N) = transpose of in (N x N)
hipError_t transpose(const double* in, double* out, int64_t N, hipStream_t s);
// x = M^{-1} b on the coarsest level: the pinned entries of b are zeroed, x = inv b with
// the stored inverse (column-major), then, when mat (the pinned operator M, column-major)
// is given, one step of iterative refinement in FP64, b <- b - M x, x <- x + inv b (b is
// overwritten).  Solving through an explicit inverse alone leaves a forward error of
// order |M^{-1}| |M| |M^{-1}| |b| eps; the refinement step computes the residual with M
// itself and brings the error down to order cond(M, x) eps (componentwise condition).
hipError_t coarse_solve(const double* inv, const double* mat, int64_t N, double* b, double* x,
                        const int64_t* pins, int npins, double* part, hipStream_t s);
int coarse_split();  // number of partial sums per row used by coarse_solve
template <typename T>
hipError_t to_internal(const DevLevel& L, const double* abi, T* x, hipStream_t s);
template <typename T>
hipError_t to_abi(const DevLevel& L, const T* x, double* abi, hipStream_t s);
template <typename S, typename D>
hipError_t cast(const S* in, D* out, int64_t n, hipStream_t s);
hipError_t project_pressure(const DevLevel& L, double* x, double* partials, hipStream_t s);
// GMRES relaxation pieces (smoother 2).  `gr` holds H column-major with leading
// dimension kMaxGr + 1, then the norm slots (kGrNorm + i) and the coefficients
// (kGrY + j); `part` holds kGrBlocks partial sums per vector.
constexpr int kGrH = 0, kGrNorm = (kMaxGr + 1) * kMaxGr, kGrY = kGrNorm + kMaxGr + 2,
              kGrSize = kGrY + kMaxGr, kGrBlocks = 256;
template <typename T>
hipError_t gr_dots(const T* V, int64_t ldv, int nv, const T* w, int64_t n, double* part, double* out,
                   hipStream_t s);
template <typename T>
hipError_t gr_orth_norm(T* w, const T* V, int64_t ldv, int j, int64_t n, const double* h, double* part,
                        double* nrm, hipStream_t s);
template <typename T>
hipError_t gr_scale(T* v, int64_t n, const double* d, hipStream_t s);
hipError_t gr_solve(double* gr, int m, hipStream_t s);
template <typename T>
hipError_t gr_update(T* x, const T* V, int64_t ldv, int m, int64_t n, const double* y, int assign, hipStream_t s);
// deterministic reductions: result written to device scalar *out
hipError_t dot(const double* a, const double* b, int64_t n, double* partials, double* out,
               hipStream_t s, int take_sqrt = 0);
// Arnoldi orthogonalisation of w against the j+1 basis vectors V (n apart) by modified
// Gram--Schmidt, then normalisation: hcol[0..j] = projections, hcol[j+1] = norm (device);
// partials: 1024-value workspace.
hipError_t mgs_arnoldi(double* w, const double* V, int64_t n, int j, double* partials, double* hcol,
                       hipStream_t s);
// y += alpha * x with alpha = sign * (*dev_scalar) (or the host value if dev_scalar null)
hipError_t axpy_dev(double* y, const double* x, int64_t n, const double* dev_scalar,
                    double sign, hipStream_t s);
// y = x / (*dev_scalar)
hipError_t scale_inv_dev(double* y, const double* x, int64_t n, const double* dev_scalar,
                         hipStream_t s);
// x += sum_i c_i Z_i (Z: m vectors of n, c on the device), accumulated per entry in the
// order i = 0, 1, ..., m - 1
hipError_t update_sum(double* x, const double* Z, int64_t n, const double* c, int m, hipStream_t s);
hipError_t axpby(double* y, const double* x, int64_t n, double alpha, double beta,
                 hipStream_t s);  // y = alpha x + beta y
hipError_t fill(double* y, int64_t n, double v, hipStream_t s);
hipError_t fillf(float* y, int64_t n, float v, hipStream_t s);
hipError_t nonfinite(const double* x, int64_t n, int* flag, hipStream_t s);
hipError_t rhs(const DevLevel& L, int64_t nnodes, const double* f, const double* state,
               double* F, hipStream_t s);
hipError_t update(const DevLevel& L, const double* b, double dt, const double* k,
                  double* state, hipStream_t s);
hipError_t rhs_adjoint(const DevLevel& L, int64_t nnodes, const int32_t* mt_ptr, const int32_t* mt_col,
                       const double* mt_val, const double* lam, double* gf, double* gstate, int accumulate,
                       hipStream_t s);
hipError_t update_adjoint(const DevLevel& L, const double* b, double dt, const double* gs, double* G,
                          hipStream_t s);
hipError_t nu_sensitivity(const DevLevel& L, const double* A, double dt, const double* lam, const double* kv,
                          const double* state, double* rowsum, double* partials, double* out, int accumulate,
                          hipStream_t s);
// loss = 1/2 e^T M e with e the velocity part of state - target (if loss is given);
// grad_state = s [M e; 0], grad_target = -s [M e; 0] with s = *scale (1 if null), each
// if given.  e and Me: ns-value workspaces; partials: the reduction workspace.
hipError_t tracking_loss(const DevLevel& L, const double* state, const double* target, const double* scale,
                         double* loss, double* grad_state, double* grad_target, double* e, double* Me,
                         double* partials, hipStream_t s);
hipError_t mass_apply(const DevLevel& L, const double* st, double* out, hipStream_t s);

// Navier--Stokes terms (Sec. 3.2), finest level.  dt a_ij (or a_ij) by value.
struct NsCoef {
  double a[kMaxStages * kMaxStages];
};
struct NsElemArgs {
  int64_t nc = 0;
  int r = 0;
  int mode = 0;                       // 0: c(U - w, U); 1: c(U - w, z) + c(z, U)
  const int32_t* cell_nodes = nullptr;  // nc x nloc node indices
  const double* geo = nullptr;        // nc x ((dim+1) dim + 1): grad lam_k, then |cell|
  const int32_t* cell_free = nullptr;  // nc x nloc free indices of the cell nodes (-1: prescribed)
  const double* U = nullptr;          // stage values [node][d][i]
  const double* w = nullptr;          // wind [node][d] (NULL: none)
  const double* x = nullptr;          // mode 1: direction, internal layout
  double a[kMaxStages * kMaxStages] = {0};  // mode 1: a_ij
  double* elem = nullptr;             // out: [cell][a][d][i]
};
hipError_t ns_stage_values(int64_t nn, int dim, int r, int64_t nfree, const int32_t* free_of_node,
                           const double* state, const double* x, const NsCoef& dtA, const double* g_st,
                           double* U, hipStream_t s);
hipError_t ns_element(int dim, const NsElemArgs& a, hipStream_t s);
hipError_t ns_gather(int64_t nfree, int dim, int r, const int32_t* inc_ptr, const int32_t* inc,
                     const double* elem, double scale, double* y, hipStream_t s);
// Per-stage velocity blocks of the Newton Jacobian on one level (assemble_newton_block on
// the device, every stage at once): nw[(p r + s) dim^2 + c dim + e] = (nu K + C(U_s))
// delta_ce + R(U_s)_ce for every entry p of the scalar pattern; geo / cn / cf / inc_ptr /
// inc from ns_cell_data, K1 the stiffness values, Cref fe_p2_conv_tensor, U the stage
// velocities ((node dim + c) r + s).  One thread per (free row, stage), which owns its
// row's entries; the row's cells are summed in incidence order.
hipError_t newton_blocks(int dim, int r, int64_t nfree, const int32_t* s_ptr, const int32_t* s_col, const double* K1,
                         double nu, const double* geo, const int32_t* cn, const int32_t* cf, const int32_t* inc_ptr,
                         const int32_t* inc, const double* Cref, const double* U, double* nw, hipStream_t s);
// Uc[n w + q] = Uf[c2f[n] w + q] for n < nc, q < w (injection at the coarse P2 nodes)
hipError_t inject_nodal(int64_t nc, int w, const int32_t* c2f, const double* Uf, double* Uc, hipStream_t s);
}  // namespace k

}  // namespace irk

// the opaque handle of the C ABI
struct irk_mg : irk::Handle {};

namespace irk {
// FGMRES workspace of a handle sized for `restart` (used by the batched solver too)
int ensure_krylov_ws(irk_mg* h, int restart);
// message returned by irk_last_error() on the calling thread
void set_error(const std::string& msg);
// Ritz estimate of a level's relaxation operator (irk_mg_ritz) in parts: argument
// checks (level -1 is resolved to the finest); the Arnoldi process in caller-provided
// device storage (V: (steps + 1) level vectors in the handle's precision, dH:
// (steps + 1)^2 doubles, part: ritz_partials_bytes()), the Hessenberg matrix copied to
// the host array Hh ((steps + 1) x steps) and the stream synchronised; the eigenvalues
// from Hh with caller storage (work: steps^2 + 3 steps complex values, iwork: steps).
int ritz_check(irk_mg* h, int& level, int steps, const double* v0, const double* ritz_re, const double* ritz_im);
int ritz_into(irk_mg* h, int level, int steps, const double* v0, void* V, double* dH, double* part, double* Hh,
              hipStream_t s);
int ritz_finish(int steps, const double* Hh, double* H, double* ritz_re, double* ritz_im, int* nritz,
                std::complex<double>* work, int* iwork);
size_t ritz_partials_bytes();
// stored failure (IRK_* code and message) for the calling thread
int fail_with(int code, const std::string& msg);
// IRK_MG_POISON_ALLOC set (and not "0"): every allocation of a handle is filled with the
// byte 0xFF (NaN) before first use
bool poison_requested();

// Element helpers of the P2 assembly, for the other model assemblies: barycentric
// gradients ((dim+1) x dim) and measure of cell c; barycentric coordinates of x in
// cell c; CSR position of column c in a sorted row (-1 if absent); CSR from sorted
// rows; CSR transpose (columns sorted); int_T phi_a lam_i / |T| for the P2 basis
// ((nloc x (dim+1)), row-major); int_T d_k phi_a d_l phi_b / |T| indexed
// [((a nloc + b)(dim+1) + k)(dim+1) + l], derivatives in barycentric coordinates.
void fe_cell_geometry(const HostLevel& L, int64_t c, double* glam, double* vol);
void fe_barycentric(const HostLevel& L, int64_t c, const double* x, double* lam);
int32_t fe_find_in_row(const std::vector<int32_t>& ptr, const std::vector<int32_t>& col, int64_t row, int64_t c);
void fe_csr_from_rows(std::vector<std::vector<int32_t>>& rows, std::vector<int32_t>& ptr, std::vector<int32_t>& col);
void fe_transpose_csr(int64_t nrows, int64_t ncols, const std::vector<int32_t>& ptr, const std::vector<int32_t>& col,
                      const std::vector<double>& val, std::vector<int32_t>& tptr, std::vector<int32_t>& tcol,
                      std::vector<double>& tval);
void fe_p2_lam_moments(int dim, double* out);
const double* fe_p2_grad_grad(int dim);
// int_T phi_e phi_a d_k phi_b / |T| indexed [((e nloc + a) nloc + b)(dim+1) + k]
const double* fe_p2_conv_tensor(int dim);
}  // namespace irk
