// Navier--Stokes terms of the stage equations and of their Newton Jacobian (Sec. 3.2)
// on the finest level, for gfx950.
//
// With c(a, b; v) = int ((a . grad) b) . v, the stage equations of Sec. 3.2 add N(U_i) =
// c(U_i, U_i; .) to the velocity rows of stage i, U_i = u^n + dt sum_j a_ij k_j^u, and
// the Newton Jacobian adds dt a_ij (c(z, U_i; .) + c(U_i, z; .)) to block (i, j).  The
// library's own operator is the Kronecker (Oseen) one with the prescribed wind w, so what
// is computed here is the difference to it:
//   residual:  c(U_i - w, U_i; .)                        (N(U_i) - C(w) U_i)
//   Jacobian:  c(U_i - w, z_i; .) + c(z_i, U_i; .),  z_i = sum_j a_ij x_j
// (C(w) is linear in w, so c(U_i, z) - c(w, z) = c(U_i - w, z)).
//
// Two launches, both deterministic (no atomics, so every solve repeats bit for bit):
//   k_ns_element  one thread per (cell, stage): gathers the cell's nodal fields and
//                 writes the element vector, exactly (the integrands are polynomials of
//                 degree 5) by a quadrature rule of that degree (7 points on a triangle,
//                 14 on a tetrahedron);
//   k_ns_gather   one thread per free velocity unknown (internal layout): sums the element
//                 vectors of the cells around its node in a fixed order, y += scale * sum.
#include <hip/hip_runtime.h>

#include "irk_internal.h"

namespace irk {
namespace k {
namespace {

template <int D>
struct Elem {
  static constexpr int NL = D == 2 ? 6 : 10;
  static constexpr int NB = D + 1;
};

// Quadrature rules exact for polynomials of degree 5, which covers every integrand
// phi_a ((a . grad) b)_d of P2 fields: points in barycentric coordinates, weights summing
// to 1 (the integral is |cell| sum_q w_q f(x_q)).
//   triangle: Radon's seven points (centroid and two three-point orbits);
//   tetrahedron: 14 points, two four-point orbits (a, a, a, 1 - 3a) and one six-point
//   orbit (a, a, 1/2 - a, 1/2 - a), the orbit parameters solving the moment equations.
// Both were checked on every monomial of degree <= 5 in 40-digit arithmetic.
template <int D>
struct Rule;
template <>
struct Rule<2> {
  static constexpr int NQ = 7;
  static constexpr double a1 = 0.10128650732345633880, b1 = 0.79742698535308732240;
  static constexpr double a2 = 0.47014206410511508977, b2 = 0.059715871789769820459;
  static constexpr double c = 1.0 / 3.0;
  static constexpr double w0 = 0.225, w1 = 0.12593918054482715260, w2 = 0.13239415278850618074;
  static constexpr double L[NQ][3] = {{c, c, c}, {a1, a1, b1}, {a1, b1, a1}, {b1, a1, a1},
                                      {a2, a2, b2}, {a2, b2, a2}, {b2, a2, a2}};
  static constexpr double W[NQ] = {w0, w1, w1, w1, w2, w2, w2};
};
template <>
struct Rule<3> {
  static constexpr int NQ = 14;
  static constexpr double a1 = 0.09273525031089122640, b1 = 1.0 - 3.0 * a1;
  static constexpr double a2 = 0.31088591926330060980, b2 = 1.0 - 3.0 * a2;
  static constexpr double a3 = 0.45449629587435035051, b3 = 0.5 - a3;
  static constexpr double w1 = 0.073493043116361949544, w2 = 0.11268792571801585080;
  static constexpr double w3 = 0.042546020777081466438;
  static constexpr double L[NQ][4] = {
      {b1, a1, a1, a1}, {a1, b1, a1, a1}, {a1, a1, b1, a1}, {a1, a1, a1, b1},
      {b2, a2, a2, a2}, {a2, b2, a2, a2}, {a2, a2, b2, a2}, {a2, a2, a2, b2},
      {a3, a3, b3, b3}, {a3, b3, a3, b3}, {a3, b3, b3, a3}, {b3, a3, a3, b3}, {b3, a3, b3, a3}, {b3, b3, a3, a3}};
  static constexpr double W[NQ] = {w1, w1, w1, w1, w2, w2, w2, w2, w3, w3, w3, w3, w3, w3};
};
template <int D>
struct Edges;
template <>
struct Edges<2> {  // local edge order of the P2 basis
  static constexpr int E[3][2] = {{0, 1}, {0, 2}, {1, 2}};
};
template <>
struct Edges<3> {
  static constexpr int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
};

// Per point: the fields and their derivatives along the barycentric coordinates from the
// P2 basis, grad = sum_k d/dlam_k grad lam_k.  MODE 0: (V . grad) U; MODE 1:
// (V . grad) Z + (Z . grad) U.  out[a][d] += w_q phi_a(x_q) g_d.
template <int D, int MODE>
__device__ __forceinline__ void quad_terms(const double (&V)[Elem<D>::NL][D], const double (&Z)[Elem<D>::NL][D],
                                           const double (&U)[Elem<D>::NL][D], const double (&glam)[D + 1][D],
                                           double (&out)[Elem<D>::NL][D]) {
  constexpr int NL = Elem<D>::NL, NB = D + 1;
  using R = Rule<D>;
#pragma unroll
  for (int q = 0; q < R::NQ; ++q) {
    double phi[NL], dphi[NL][NB];
#pragma unroll
    for (int v = 0; v < NB; ++v) {
      phi[v] = R::L[q][v] * (2.0 * R::L[q][v] - 1.0);
#pragma unroll
      for (int k = 0; k < NB; ++k) dphi[v][k] = k == v ? 4.0 * R::L[q][v] - 1.0 : 0.0;
    }
#pragma unroll
    for (int e = 0; e < NL - NB; ++e) {
      const int i = Edges<D>::E[e][0], j = Edges<D>::E[e][1];
      phi[NB + e] = 4.0 * R::L[q][i] * R::L[q][j];
#pragma unroll
      for (int k = 0; k < NB; ++k)
        dphi[NB + e][k] = (k == i ? 4.0 * R::L[q][j] : 0.0) + (k == j ? 4.0 * R::L[q][i] : 0.0);
    }
    double vq[D];
#pragma unroll
    for (int d = 0; d < D; ++d) vq[d] = 0.0;
#pragma unroll
    for (int b = 0; b < NL; ++b)
#pragma unroll
      for (int d = 0; d < D; ++d) vq[d] += phi[b] * V[b][d];
    double g[D];
#pragma unroll
    for (int d = 0; d < D; ++d) g[d] = 0.0;
    const double (&X)[NL][D] = MODE == 0 ? U : Z;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      double vg = 0.0;
#pragma unroll
      for (int d = 0; d < D; ++d) vg += vq[d] * glam[k][d];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        double dx = 0.0;
#pragma unroll
        for (int b = 0; b < NL; ++b) dx += dphi[b][k] * X[b][d];
        g[d] += vg * dx;
      }
    }
    if constexpr (MODE == 1) {
      double zq[D];
#pragma unroll
      for (int d = 0; d < D; ++d) zq[d] = 0.0;
#pragma unroll
      for (int b = 0; b < NL; ++b)
#pragma unroll
        for (int d = 0; d < D; ++d) zq[d] += phi[b] * Z[b][d];
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        double zg = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) zg += zq[d] * glam[k][d];
#pragma unroll
        for (int d = 0; d < D; ++d) {
          double du = 0.0;
#pragma unroll
          for (int b = 0; b < NL; ++b) du += dphi[b][k] * U[b][d];
          g[d] += zg * du;
        }
      }
    }
#pragma unroll
    for (int a = 0; a < NL; ++a)
#pragma unroll
      for (int d = 0; d < D; ++d) out[a][d] += (R::W[q] * phi[a]) * g[d];
  }
}

template <int D>
__global__ __launch_bounds__(256) void k_ns_element(NsElemArgs p) {
  constexpr int NL = Elem<D>::NL, NB = Elem<D>::NB;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = p.r;
  if (t >= p.nc * r) return;
  const int64_t c = t / r;  // consecutive threads: the stages of one cell
  const int i = (int)(t - c * r);
  const double* g = p.geo + c * (NB * D + 1);
  double glam[NB][D];
#pragma unroll
  for (int k = 0; k < NB; ++k)
#pragma unroll
    for (int d = 0; d < D; ++d) glam[k][d] = g[k * D + d];
  const double vol = g[NB * D];
  int node[NL];
#pragma unroll
  for (int a = 0; a < NL; ++a) node[a] = p.cell_nodes[c * NL + a];
  double out[NL][D];
#pragma unroll
  for (int a = 0; a < NL; ++a)
#pragma unroll
    for (int d = 0; d < D; ++d) out[a][d] = 0.0;
  // V = U_i - w at the nodes
  double V[NL][D];
#pragma unroll
  for (int a = 0; a < NL; ++a)
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const double u = p.U[((int64_t)node[a] * D + d) * r + i];
      V[a][d] = p.w ? u - p.w[(int64_t)node[a] * D + d] : u;
    }
  if (p.mode == 0) {
    double U[NL][D];
#pragma unroll
    for (int a = 0; a < NL; ++a)
#pragma unroll
      for (int d = 0; d < D; ++d) U[a][d] = p.U[((int64_t)node[a] * D + d) * r + i];
    quad_terms<D, 0>(V, U, U, glam, out);
  } else {
    // z_i = sum_j a_ij x_j at the nodes; prescribed (boundary) nodes do not vary
    double Z[NL][D];
#pragma unroll
    for (int a = 0; a < NL; ++a) {
      const int f = p.cell_free[c * NL + a];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        double s = 0.0;
        if (f >= 0)
          for (int j = 0; j < r; ++j) s += p.a[i * r + j] * p.x[((int64_t)f * D + d) * r + j];
        Z[a][d] = s;
      }
    }
    double U[NL][D];
#pragma unroll
    for (int a = 0; a < NL; ++a)
#pragma unroll
      for (int d = 0; d < D; ++d) U[a][d] = p.U[((int64_t)node[a] * D + d) * r + i];
    quad_terms<D, 1>(V, Z, U, glam, out);
  }
#pragma unroll
  for (int a = 0; a < NL; ++a)
#pragma unroll
    for (int d = 0; d < D; ++d) p.elem[((c * NL + a) * D + d) * r + i] = vol * out[a][d];
}

// y[t] += scale * sum over the incidences (cell, local node) of free node f of the
// element entries; t = (f * D + d) * r + i, inc[q] = cell * NL + a.
__global__ __launch_bounds__(256) void k_ns_gather(int64_t n, int dr, const int32_t* __restrict__ inc_ptr,
                                                   const int32_t* __restrict__ inc,
                                                   const double* __restrict__ elem, double scale,
                                                   double* __restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t f = t / dr;
  const int rem = (int)(t - f * dr);
  double s = 0.0;
  for (int32_t q = inc_ptr[f]; q < inc_ptr[f + 1]; ++q) s += elem[(int64_t)inc[q] * dr + rem];
  y[t] += scale * s;
}

// U[(node * D + d) * r + i]: free nodes u^n + dt sum_j a_ij k_j (state in the stage-block
// layout, k internal), prescribed nodes the stage data (or zero).
__global__ __launch_bounds__(256) void k_ns_stage_values(int64_t nn, int D, int r, int64_t nfree,
                                                         const int32_t* __restrict__ free_of_node,
                                                         const double* __restrict__ state,
                                                         const double* __restrict__ x, NsCoef dtA,
                                                         const double* __restrict__ g_st,
                                                         double* __restrict__ U) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int dr = D * r;
  if (t >= nn * dr) return;
  const int64_t node = t / dr;
  const int rem = (int)(t - node * dr);
  const int d = rem / r, i = rem - d * r;
  const int f = free_of_node[node];
  double v;
  if (f >= 0) {
    v = state[(int64_t)d * nfree + f];
    for (int j = 0; j < r; ++j) v += dtA.a[i * r + j] * x[((int64_t)f * D + d) * r + j];
  } else {
    v = g_st ? g_st[((int64_t)i * nn + node) * D + d] : 0.0;
  }
  U[t] = v;
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// The Newton Jacobian's per-stage velocity blocks, one thread per (free row, stage): the
// thread owns its row's pattern entries, visits the cells around the row's node in
// incidence order and adds, for each free column node b of the cell, the convection
// int phi_a (U . grad phi_b) on the diagonal component blocks and the reaction
// int phi_a phi_b d_e U_c on block (c, e), by the exact reference tensor; the stiffness
// nu K on the diagonal blocks last.
template <int D>
__global__ __launch_bounds__(256) void k_newton_blocks(int r, int64_t nfree, const int32_t* __restrict__ s_ptr,
                                                       const int32_t* __restrict__ s_col,
                                                       const double* __restrict__ K1, double nu,
                                                       const double* __restrict__ geo,
                                                       const int32_t* __restrict__ cn,
                                                       const int32_t* __restrict__ cf,
                                                       const int32_t* __restrict__ inc_ptr,
                                                       const int32_t* __restrict__ inc,
                                                       const double* __restrict__ Cref,
                                                       const double* __restrict__ U, double* __restrict__ nw) {
  constexpr int NL = Elem<D>::NL, NB = D + 1, DD = D * D, PER = NB * D + 1;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= nfree * r) return;
  const int64_t ia = t / r;
  const int i = (int)(t - ia * r);
  const int32_t p0 = s_ptr[ia], p1 = s_ptr[ia + 1];
  for (int32_t p = p0; p < p1; ++p)
#pragma unroll
    for (int q = 0; q < DD; ++q) nw[((int64_t)p * r + i) * DD + q] = 0.0;
  for (int32_t q = inc_ptr[ia]; q < inc_ptr[ia + 1]; ++q) {
    const int32_t e = inc[q];
    const int64_t c = e / NL;
    const int a = e - (int)c * NL;
    const double* g = geo + c * PER;
    const double vol = g[NB * D];
    double Uf[NL][D], wg[NL][NB];
#pragma unroll
    for (int f = 0; f < NL; ++f) {
      const int64_t node = cn[c * NL + f];
#pragma unroll
      for (int cc = 0; cc < D; ++cc) Uf[f][cc] = U[(node * D + cc) * r + i];
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        double sum = 0.0;
#pragma unroll
        for (int cc = 0; cc < D; ++cc) sum += Uf[f][cc] * g[k * D + cc];
        wg[f][k] = sum;
      }
    }
    for (int b = 0; b < NL; ++b) {
      const int32_t ib = cf[c * NL + b];
      if (ib < 0) continue;
      double ce = 0.0;
#pragma unroll
      for (int f = 0; f < NL; ++f)
#pragma unroll
        for (int k = 0; k < NB; ++k) ce += wg[f][k] * Cref[((f * NL + a) * NL + b) * NB + k];
      double Tg[NL][D];
#pragma unroll
      for (int f = 0; f < NL; ++f)
#pragma unroll
        for (int ee = 0; ee < D; ++ee) {
          double sum = 0.0;
#pragma unroll
          for (int k = 0; k < NB; ++k) sum += g[k * D + ee] * Cref[((a * NL + b) * NL + f) * NB + k];
          Tg[f][ee] = sum;
        }
      int32_t lo = p0, hi = p1;  // the column ib in the row's sorted pattern
      while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (s_col[mid] < ib) lo = mid + 1;
        else hi = mid;
      }
      double* o = nw + ((int64_t)lo * r + i) * DD;
#pragma unroll
      for (int cc = 0; cc < D; ++cc) {
        o[cc * D + cc] += vol * ce;
#pragma unroll
        for (int ee = 0; ee < D; ++ee) {
          double tt = 0.0;
#pragma unroll
          for (int f = 0; f < NL; ++f) tt += Uf[f][cc] * Tg[f][ee];
          o[cc * D + ee] += vol * tt;
        }
      }
    }
  }
  for (int32_t p = p0; p < p1; ++p)
#pragma unroll
    for (int cc = 0; cc < D; ++cc) nw[((int64_t)p * r + i) * DD + cc * D + cc] += nu * K1[p];
}

__global__ __launch_bounds__(256) void k_inject_nodal(int64_t n, int w, const int32_t* __restrict__ c2f,
                                                      const double* __restrict__ Uf, double* __restrict__ Uc) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const int64_t node = t / w;
  const int q = (int)(t - node * w);
  Uc[t] = Uf[(int64_t)c2f[node] * w + q];
}

}  // namespace

hipError_t ns_stage_values(int64_t nn, int dim, int r, int64_t nfree, const int32_t* free_of_node,
                           const double* state, const double* x, const NsCoef& dtA, const double* g_st,
                           double* U, hipStream_t s) {
  const int64_t n = nn * dim * r;
  if (n == 0) return hipSuccess;
  k_ns_stage_values<<<blocks_for(n, 256), 256, 0, s>>>(nn, dim, r, nfree, free_of_node, state, x, dtA, g_st, U);
  return hipGetLastError();
}

hipError_t ns_element(int dim, const NsElemArgs& a, hipStream_t s) {
  const int64_t n = a.nc * a.r;
  if (n == 0) return hipSuccess;
  if (dim == 2)
    k_ns_element<2><<<blocks_for(n, 256), 256, 0, s>>>(a);
  else
    k_ns_element<3><<<blocks_for(n, 256), 256, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t newton_blocks(int dim, int r, int64_t nfree, const int32_t* s_ptr, const int32_t* s_col, const double* K1,
                         double nu, const double* geo, const int32_t* cn, const int32_t* cf, const int32_t* inc_ptr,
                         const int32_t* inc, const double* Cref, const double* U, double* nw, hipStream_t s) {
  const int64_t n = nfree * r;
  if (n == 0) return hipSuccess;
  if (dim == 2)
    k_newton_blocks<2><<<blocks_for(n, 256), 256, 0, s>>>(r, nfree, s_ptr, s_col, K1, nu, geo, cn, cf, inc_ptr, inc,
                                                         Cref, U, nw);
  else
    k_newton_blocks<3><<<blocks_for(n, 256), 256, 0, s>>>(r, nfree, s_ptr, s_col, K1, nu, geo, cn, cf, inc_ptr, inc,
                                                         Cref, U, nw);
  return hipGetLastError();
}

hipError_t inject_nodal(int64_t nc, int w, const int32_t* c2f, const double* Uf, double* Uc, hipStream_t s) {
  const int64_t n = nc * w;
  if (n == 0) return hipSuccess;
  k_inject_nodal<<<blocks_for(n, 256), 256, 0, s>>>(n, w, c2f, Uf, Uc);
  return hipGetLastError();
}

hipError_t ns_gather(int64_t nfree, int dim, int r, const int32_t* inc_ptr, const int32_t* inc,
                     const double* elem, double scale, double* y, hipStream_t s) {
  const int64_t n = nfree * dim * r;
  if (n == 0) return hipSuccess;
  k_ns_gather<<<blocks_for(n, 256), 256, 0, s>>>(n, dim * r, inc_ptr, inc, elem, scale, y);
  return hipGetLastError();
}

}  // namespace k
}  // namespace irk
