// Internal structures of the linearised 2D MHD stage solver (Sec. 3.3) in libirkmg.
//
// Spatial unknowns of a level, in the order of the ABI layout of one stage:
//   [0, nfree)             u_x at the free P2 nodes
//   [nfree, 2 nfree)       u_y
//   [off_B, off_B + nB)    B at the interior edges (Nedelec degrees of freedom)
//   [off_p, off_p + nv)    p at every vertex
//   [off_g, off_g + ng)    gamma at the interior vertices
// Internal device layout: unknown-major with the stage innermost, x[q * r + s], so that
// one sparse traversal of the spatial operator serves all stages.
#pragma once

#include <string>
#include <vector>

#include "irk_internal.h"

namespace irk {

struct MhdHost {
  HostLevel L;  // topology, scalar P2 blocks, P2 / P1 transfers from the coarser level
  int64_t nfree = 0, nB = 0, nv = 0, ng = 0, ns = 0, off_B = 0, off_p = 0, off_g = 0;
  std::vector<int32_t> eidx, efree;  // edge -> interior edge index (-1), and back
  std::vector<int32_t> gidx, vint;   // vertex -> interior vertex index (-1), and back
  // spatial operator S and mass M on one pattern (ns x ns CSR, sorted columns)
  std::vector<int32_t> ptr, col;
  std::vector<double> mval, sval;
  // vertex patches: spatial unknowns (sorted) of patch v in pdof[pptr[v] .. pptr[v+1]),
  // and the operator entries coupling them as triples (local a, local b, CSR position)
  std::vector<int32_t> pptr, pdof, pvv_ptr, pvv;
  // prolongation from the next coarser level: fine unknowns x coarse unknowns
  std::vector<int32_t> P_ptr, P_col;
  std::vector<double> P_val;
};

// Index maps and offsets of the unknowns (after build_topology).
void mhd_index(MhdHost& H);
// M and S at the state (w: P2 nodes x 2, b0: every edge); needs assemble_level's
// scalar blocks (mass, stiffness, divergence) on H.L.
void mhd_assemble(MhdHost& H, double Re, double Rem, const double* w, const double* b0);
void mhd_patches(MhdHost& H);
// Prolongation of F from C (build_transfer already run on their HostLevels); returns an
// empty string on success.
std::string mhd_transfer(const MhdHost& C, MhdHost& F, const int64_t* parent);
// The state on C from the state on F: w at the coarse P2 nodes, B0 on the coarse edges.
void mhd_coarsen_state(const MhdHost& C, const MhdHost& F, const double* wf, const double* bf,
                       std::vector<double>& wc, std::vector<double>& bc);
// Dense I_r (x) M + dt A (x) S in the internal layout, column-major, with the pressure of
// vertex 0 pinned in every stage (row and column zero, diagonal one).
void mhd_coarse_matrix(const MhdHost& H, int r, const double* A, double dt, std::vector<double>& J,
                       double* max_abs);

namespace k {
// y = F - (I (x) M + dt A (x) S) x over the sliced operator (F null: y = J x)
hipError_t kron_residual(int64_t nrows, int64_t nsl, const int32_t* sl_off, const int32_t* sl_w,
                         const int32_t* sl_col, const double* sl_m, const double* sl_s, int R, const double* A,
                         double dt, const double* F, const double* x, double* y, hipStream_t s);
// y = P x (accumulate: y += P x) for a CSR P applied to each of R stages
hipError_t kron_csr(int64_t nrows, const int32_t* ptr, const int32_t* col, const double* val, int R,
                    const double* x, double* y, int accumulate, hipStream_t s);
// between the ABI layout (stage blocks of ns) and the internal layout (stage innermost)
hipError_t stage_to_internal(int64_t ns, int R, const double* abi, double* x, hipStream_t s);
hipError_t stage_to_abi(int64_t ns, int R, const double* x, double* abi, hipStream_t s);
// Dense inverses of I_R (x) M_v + dt A (x) S_v for the patches [p0, p1) of a generic
// Kronecker operator (A: R x R, the stage matrix or one block of its eigenbasis form):
// patch p has n_s = pn_ptr[p+1] - pn_ptr[p] + 1 spatial unknowns, its entries come from
// the triples pvv (M and S values at their CSR positions); patch p's inverse is stored
// column-major (R n_s x ld[p]) at out + off[p] - off0; nmax bounds R n_s.
template <typename T>
hipError_t patch_factor_scalar(const DevLevel& L, const DevOps<T>& ops, int R, const double* A, double dt,
                               const int32_t* ld, const int64_t* off, T* out, int64_t p0, int64_t p1, int64_t off0,
                               int nmax, int* d_fail, hipStream_t s);
}  // namespace k

}  // namespace irk
