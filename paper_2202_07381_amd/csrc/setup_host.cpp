// Host-side setup of libirkmg: mesh topology and P2 numbering, exact element matrices,
// sparse assembly (rediscretisation on every level, Sec. 4.1), vertex-star patches
// (Sec. 4.2, Fig. 1), transfer operators from the parent map (Sec. 4.1) and the dense
// coarse inverse.  Everything here is untimed setup; all solve-time arithmetic runs in
// the HIP kernels.
//
// Element integrals use the exact formula for monomials in barycentric coordinates on a
// d-simplex T:  int_T lam^a = |T| d! prod(a_k!) / (|a| + d)!.  P2 basis functions are
// lam_i (2 lam_i - 1) (vertex i) and 4 lam_i lam_j (edge ij), gradients follow from
// grad lam_k, so the reference tensors below depend on nothing but the dimension.
#include <algorithm>
#include <array>
#include <climits>
#include <complex>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <stdexcept>
#include <thread>
#include <vector>

#include "irk_internal.h"

namespace irk {
namespace {

const int kEdges2[3][2] = {{0, 1}, {0, 2}, {1, 2}};
const int kEdges3[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

inline int nloc_of(int dim) { return dim == 2 ? 6 : 10; }
inline const int (*edges_of(int dim))[2] { return dim == 2 ? kEdges2 : kEdges3; }

// ------------------------------------------------ polynomials in barycentric coords
struct Term {
  double c;
  std::array<int, 4> e;
};
using Poly = std::vector<Term>;

Poly mul(const Poly& a, const Poly& b) {
  Poly out;
  for (const Term& x : a)
    for (const Term& y : b) {
      Term t;
      t.c = x.c * y.c;
      for (int k = 0; k < 4; ++k) t.e[k] = x.e[k] + y.e[k];
      out.push_back(t);
    }
  return out;
}

Poly dlam(const Poly& p, int k) {  // formal derivative with respect to lam_k
  Poly out;
  for (const Term& t : p)
    if (t.e[k] > 0) {
      Term u = t;
      u.c *= t.e[k];
      u.e[k] -= 1;
      out.push_back(u);
    }
  return out;
}

double fact(int n) {
  double f = 1;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

double integrate(const Poly& p, int dim) {  // int_T p / |T|
  double s = 0;
  for (const Term& t : p) {
    int tot = 0;
    double num = fact(dim);
    for (int k = 0; k <= dim; ++k) {
      num *= fact(t.e[k]);
      tot += t.e[k];
    }
    s += t.c * num / fact(tot + dim);
  }
  return s;
}

Poly lam_pow(int i, int pw, double c) {
  Term t;
  t.c = c;
  t.e = {0, 0, 0, 0};
  t.e[i] = pw;
  return {t};
}

Poly basis(int dim, int a) {
  if (a <= dim) {
    Poly p = lam_pow(a, 2, 2.0);
    p.push_back(lam_pow(a, 1, -1.0)[0]);
    return p;
  }
  const int* e = edges_of(dim)[a - dim - 1];
  Term t;
  t.c = 4.0;
  t.e = {0, 0, 0, 0};
  t.e[e[0]] = 1;
  t.e[e[1]] = 1;
  return {t};
}

struct RefTensors {
  int dim, nl;
  std::vector<double> M;  // [a][b]
  std::vector<double> S;  // [a][b][k][l]  int d_k phi_a d_l phi_b
  std::vector<double> B;  // [a][q][k]     int lam_q d_k phi_a
  std::vector<double> C;  // [e][a][b][k]  int phi_e phi_a d_k phi_b
};

const RefTensors& ref_tensors(int dim) {
  static RefTensors cache[2];
  RefTensors& R = cache[dim - 2];
  if (!R.M.empty()) return R;
  const int nl = nloc_of(dim), nb = dim + 1;
  R.dim = dim;
  R.nl = nl;
  std::vector<Poly> phi(nl);
  std::vector<std::vector<Poly>> dphi(nl, std::vector<Poly>(nb));
  for (int a = 0; a < nl; ++a) {
    phi[a] = basis(dim, a);
    for (int k = 0; k < nb; ++k) dphi[a][k] = dlam(phi[a], k);
  }
  R.M.resize(nl * nl);
  R.S.resize(nl * nl * nb * nb);
  R.B.resize(nl * nb * nb);
  R.C.resize(nl * nl * nl * nb);
  for (int a = 0; a < nl; ++a)
    for (int b = 0; b < nl; ++b) {
      R.M[a * nl + b] = integrate(mul(phi[a], phi[b]), dim);
      for (int k = 0; k < nb; ++k)
        for (int l = 0; l < nb; ++l)
          R.S[((a * nl + b) * nb + k) * nb + l] = integrate(mul(dphi[a][k], dphi[b][l]), dim);
    }
  for (int a = 0; a < nl; ++a)
    for (int q = 0; q < nb; ++q)
      for (int k = 0; k < nb; ++k)
        R.B[(a * nb + q) * nb + k] = integrate(mul(lam_pow(q, 1, 1.0), dphi[a][k]), dim);
  for (int e = 0; e < nl; ++e)
    for (int a = 0; a < nl; ++a) {
      Poly pe = mul(phi[e], phi[a]);
      for (int b = 0; b < nl; ++b)
        for (int k = 0; k < nb; ++k)
          R.C[((e * nl + a) * nl + b) * nb + k] = integrate(mul(pe, dphi[b][k]), dim);
    }
  return R;
}

// gradients of barycentric coordinates and measure of a cell
void cell_geometry(const HostLevel& L, int64_t c, double* glam /* (dim+1) x dim */,
                   double* vol) {
  const int d = L.dim;
  const int64_t* v = &L.cells[c * (d + 1)];
  double J[3][3], Ji[3][3];
  for (int i = 0; i < d; ++i)
    for (int k = 0; k < d; ++k) J[i][k] = L.xyz[v[k + 1] * d + i] - L.xyz[v[0] * d + i];
  double det;
  if (d == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    Ji[0][0] = J[1][1] / det;
    Ji[0][1] = -J[0][1] / det;
    Ji[1][0] = -J[1][0] / det;
    Ji[1][1] = J[0][0] / det;
  } else {
    det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
          J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
          J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  }
  // lam_{k+1} = row k of J^{-1} applied to (x - x0); lam_0 = 1 - sum
  for (int i = 0; i < d; ++i) glam[0 * d + i] = 0;
  for (int k = 0; k < d; ++k)
    for (int i = 0; i < d; ++i) {
      glam[(k + 1) * d + i] = Ji[k][i];
      glam[0 * d + i] -= Ji[k][i];
    }
  *vol = std::fabs(det) / (d == 2 ? 2.0 : 6.0);
}

// barycentric coordinates of point x in cell c
void barycentric(const HostLevel& L, int64_t c, const double* x, double* lam) {
  const int d = L.dim;
  double glam[12], vol;
  cell_geometry(L, c, glam, &vol);
  const int64_t* v = &L.cells[c * (d + 1)];
  double s = 0;
  for (int k = 1; k <= d; ++k) {
    double acc = 0;
    for (int i = 0; i < d; ++i) acc += glam[k * d + i] * (x[i] - L.xyz[v[0] * d + i]);
    lam[k] = acc;
    s += acc;
  }
  lam[0] = 1.0 - s;
}

void node_coord(const HostLevel& L, int64_t node, double* x) {
  const int d = L.dim;
  if (node < L.nv) {
    for (int i = 0; i < d; ++i) x[i] = L.xyz[node * d + i];
  } else {
    const int64_t a = L.edges[(node - L.nv) * 2], b = L.edges[(node - L.nv) * 2 + 1];
    for (int i = 0; i < d; ++i) x[i] = 0.5 * (L.xyz[a * d + i] + L.xyz[b * d + i]);
  }
}

void p2_values(int dim, const double* lam, double* w) {
  for (int i = 0; i <= dim; ++i) w[i] = lam[i] * (2 * lam[i] - 1);
  const int(*E)[2] = edges_of(dim);
  const int ne = dim == 2 ? 3 : 6;
  for (int e = 0; e < ne; ++e) w[dim + 1 + e] = 4 * lam[E[e][0]] * lam[E[e][1]];
}

int32_t find_in_row(const std::vector<int32_t>& ptr, const std::vector<int32_t>& col,
                    int64_t row, int64_t c) {
  auto b = col.begin() + ptr[row], e = col.begin() + ptr[row + 1];
  auto it = std::lower_bound(b, e, (int32_t)c);
  if (it == e || *it != c) return -1;
  return (int32_t)(it - col.begin());
}

void csr_from_rows(std::vector<std::vector<int32_t>>& rows, std::vector<int32_t>& ptr,
                   std::vector<int32_t>& col) {
  ptr.assign(rows.size() + 1, 0);
  for (size_t i = 0; i < rows.size(); ++i) ptr[i + 1] = ptr[i] + (int32_t)rows[i].size();
  col.resize(ptr.back());
  for (size_t i = 0; i < rows.size(); ++i)
    std::copy(rows[i].begin(), rows[i].end(), col.begin() + ptr[i]);
}

void transpose_csr(int64_t nrows, int64_t ncols, const std::vector<int32_t>& ptr,
                   const std::vector<int32_t>& col, const std::vector<double>& val, int vw,
                   std::vector<int32_t>& tptr, std::vector<int32_t>& tcol,
                   std::vector<double>& tval) {
  tptr.assign(ncols + 1, 0);
  for (int32_t c : col) tptr[c + 1]++;
  for (int64_t i = 0; i < ncols; ++i) tptr[i + 1] += tptr[i];
  tcol.resize(col.size());
  tval.resize(val.size());
  std::vector<int32_t> fillp(tptr.begin(), tptr.end() - 1);
  for (int64_t i = 0; i < nrows; ++i)  // ascending rows -> sorted transposed columns
    for (int32_t p = ptr[i]; p < ptr[i + 1]; ++p) {
      int32_t q = fillp[col[p]]++;
      tcol[q] = (int32_t)i;
      for (int k = 0; k < vw; ++k) tval[(size_t)q * vw + k] = val[(size_t)p * vw + k];
    }
}

}  // namespace

// -------------------------------------------------------------------------- topology
void build_topology(HostLevel& L, int dim, int64_t nv, int64_t nc, const double* xyz,
                    const int64_t* cells) {
  L.dim = dim;
  L.nv = nv;
  L.nc = nc;
  const int nb = dim + 1, nl = nloc_of(dim), nle = nl - nb;
  L.xyz.assign(xyz, xyz + nv * dim);
  L.cells.assign(cells, cells + nc * nb);
  const int(*E)[2] = edges_of(dim);
  std::vector<int64_t> keys;
  keys.reserve(nc * nle);
  for (int64_t c = 0; c < nc; ++c)
    for (int e = 0; e < nle; ++e) {
      int64_t a = L.cells[c * nb + E[e][0]], b = L.cells[c * nb + E[e][1]];
      keys.push_back(std::min(a, b) * nv + std::max(a, b));
    }
  std::vector<int64_t> uk(keys);
  std::sort(uk.begin(), uk.end());
  uk.erase(std::unique(uk.begin(), uk.end()), uk.end());
  L.ne = (int64_t)uk.size();
  L.nn = nv + L.ne;
  L.edges.resize(L.ne * 2);
  for (int64_t i = 0; i < L.ne; ++i) {
    L.edges[2 * i] = uk[i] / nv;
    L.edges[2 * i + 1] = uk[i] % nv;
  }
  L.cell_nodes.resize(nc * nl);
  for (int64_t c = 0; c < nc; ++c) {
    for (int k = 0; k < nb; ++k) L.cell_nodes[c * nl + k] = L.cells[c * nb + k];
    for (int e = 0; e < nle; ++e) {
      int64_t key = keys[c * nle + e];
      L.cell_nodes[c * nl + nb + e] =
          nv + (int64_t)(std::lower_bound(uk.begin(), uk.end(), key) - uk.begin());
    }
  }
  // boundary: facets owned by a single cell
  std::vector<std::array<int64_t, 3>> fac;
  fac.reserve(nc * nb);
  for (int64_t c = 0; c < nc; ++c)
    for (int skip = 0; skip < nb; ++skip) {
      std::array<int64_t, 3> f = {-1, -1, -1};
      int m = 0;
      for (int k = 0; k < nb; ++k)
        if (k != skip) f[m++] = L.cells[c * nb + k];
      std::sort(f.begin(), f.begin() + dim);
      fac.push_back(f);
    }
  std::sort(fac.begin(), fac.end());
  std::vector<char> bnd(L.nn, 0);
  for (size_t i = 0; i < fac.size();) {
    size_t j = i;
    while (j < fac.size() && fac[j] == fac[i]) ++j;
    if (j - i == 1) {
      const auto& f = fac[i];
      for (int k = 0; k < dim; ++k) bnd[f[k]] = 1;
      for (int a = 0; a < dim; ++a)
        for (int b = a + 1; b < dim; ++b) {
          int64_t key = std::min(f[a], f[b]) * nv + std::max(f[a], f[b]);
          bnd[nv + (std::lower_bound(uk.begin(), uk.end(), key) - uk.begin())] = 1;
        }
    }
    i = j;
  }
  L.free_of_node.assign(L.nn, -1);
  L.node_of_free.clear();
  for (int64_t n = 0; n < L.nn; ++n)
    if (!bnd[n]) {
      L.free_of_node[n] = (int32_t)L.node_of_free.size();
      L.node_of_free.push_back((int32_t)n);
    }
  L.nfree = (int64_t)L.node_of_free.size();
  // node -> cells
  L.node_cell_ptr.assign(L.nn + 1, 0);
  for (int64_t c = 0; c < nc; ++c)
    for (int a = 0; a < nl; ++a) L.node_cell_ptr[L.cell_nodes[c * nl + a] + 1]++;
  for (int64_t n = 0; n < L.nn; ++n) L.node_cell_ptr[n + 1] += L.node_cell_ptr[n];
  L.node_cell.resize(L.node_cell_ptr.back());
  std::vector<int32_t> fp(L.node_cell_ptr.begin(), L.node_cell_ptr.end() - 1);
  for (int64_t c = 0; c < nc; ++c)
    for (int a = 0; a < nl; ++a) L.node_cell[fp[L.cell_nodes[c * nl + a]]++] = (int32_t)c;
}

// -------------------------------------------------------------------------- assembly
void assemble_level(HostLevel& L, double nu, const std::vector<double>* wind, bool with_mfa) {
  const int d = L.dim, nb = d + 1, nl = nloc_of(d);
  const RefTensors& R = ref_tensors(d);
  // patterns from node -> cell adjacency
  std::vector<std::vector<int32_t>> srows(L.nfree), brows(L.nfree), mrows;
  if (with_mfa) mrows.resize(L.nfree);
  parallel_ranges(L.nfree, [&](int64_t i0, int64_t i1) {  // rows independent
    for (int64_t i = i0; i < i1; ++i) {
      const int64_t n = L.node_of_free[i];
      for (int32_t p = L.node_cell_ptr[n]; p < L.node_cell_ptr[n + 1]; ++p) {
        const int64_t c = L.node_cell[p];
        for (int a = 0; a < nl; ++a) {
          int64_t m = L.cell_nodes[c * nl + a];
          if (L.free_of_node[m] >= 0) srows[i].push_back(L.free_of_node[m]);
          if (with_mfa) mrows[i].push_back((int32_t)m);
        }
        for (int q = 0; q < nb; ++q) brows[i].push_back((int32_t)L.cells[c * nb + q]);
      }
      for (auto* v : {&srows[i], &brows[i]}) {
        std::sort(v->begin(), v->end());
        v->erase(std::unique(v->begin(), v->end()), v->end());
      }
      if (with_mfa) {
        std::sort(mrows[i].begin(), mrows[i].end());
        mrows[i].erase(std::unique(mrows[i].begin(), mrows[i].end()), mrows[i].end());
      }
    }
  });
  csr_from_rows(srows, L.s_ptr, L.s_col);
  csr_from_rows(brows, L.b_ptr, L.b_col);
  const size_t snnz = L.s_col.size();
  L.s_M.assign(snnz, 0.0);
  L.s_L.assign(snnz, 0.0);
  L.s_K1.assign(snnz, 0.0);
  std::vector<double> conv(snnz, 0.0);
  L.b_val.assign(L.b_col.size() * d, 0.0);
  std::vector<std::array<double, 5>> bnd_trip;  // (vertex, node, B values) of boundary rows
  if (with_mfa) {
    csr_from_rows(mrows, L.mfa_ptr, L.mfa_col);
    L.mfa_val.assign(L.mfa_col.size(), 0.0);
    std::vector<std::vector<int32_t>> fbrows(L.nfree);
    for (int64_t i = 0; i < L.nfree; ++i)
      for (int32_t m : mrows[i])
        if (L.free_of_node[m] < 0) fbrows[i].push_back(m);
    csr_from_rows(fbrows, L.fb_ptr, L.fb_col);
    L.fb_m.assign(L.fb_col.size(), 0.0);
    L.fb_l.assign(L.fb_col.size(), 0.0);
  }
  // element matrices scattered by vertex-disjoint groups of cells (disjoint rows); the
  // boundary triples of each range are appended under a lock and sorted on every field
  // below, so their order does not depend on the threads
  std::mutex trip_lock;
  auto cell_body = [&](int64_t c, std::vector<std::array<double, 5>>& trips) {
    double glam[12], vol;
    double G[4][4], Me[10][10], Ke[10][10], Ce[10][10], Be[10][4][3];
    cell_geometry(L, c, glam, &vol);
    for (int k = 0; k < nb; ++k)
      for (int l = 0; l < nb; ++l) {
        double s = 0;
        for (int i = 0; i < d; ++i) s += glam[k * d + i] * glam[l * d + i];
        G[k][l] = s;
      }
    for (int a = 0; a < nl; ++a)
      for (int b = 0; b < nl; ++b) {
        Me[a][b] = vol * R.M[a * nl + b];
        double s = 0;
        for (int k = 0; k < nb; ++k)
          for (int l = 0; l < nb; ++l) s += G[k][l] * R.S[((a * nl + b) * nb + k) * nb + l];
        Ke[a][b] = vol * s;
        Ce[a][b] = 0;
      }
    if (wind) {
      // C_ab = sum_e sum_k (w_e . grad lam_k) int phi_e phi_a d_k phi_b
      double wg[10][4];
      for (int e = 0; e < nl; ++e) {
        const int64_t node = L.cell_nodes[c * nl + e];
        for (int k = 0; k < nb; ++k) {
          double s = 0;
          for (int i = 0; i < d; ++i) s += (*wind)[node * d + i] * glam[k * d + i];
          wg[e][k] = s;
        }
      }
      for (int a = 0; a < nl; ++a)
        for (int b = 0; b < nl; ++b) {
          double s = 0;
          for (int e = 0; e < nl; ++e)
            for (int k = 0; k < nb; ++k) s += wg[e][k] * R.C[((e * nl + a) * nl + b) * nb + k];
          Ce[a][b] = vol * s;
        }
    }
    for (int a = 0; a < nl; ++a)
      for (int q = 0; q < nb; ++q)
        for (int i = 0; i < d; ++i) {
          double s = 0;
          for (int k = 0; k < nb; ++k) s += R.B[(a * nb + q) * nb + k] * glam[k * d + i];
          Be[a][q][i] = -vol * s;  // B_(a,i),q = - int lam_q d_i phi_a
        }
    for (int a = 0; a < nl; ++a) {
      const int64_t na = L.cell_nodes[c * nl + a];
      const int64_t ia = L.free_of_node[na];
      if (ia < 0) {
        if (with_mfa)
          for (int q = 0; q < nb; ++q) {
            std::array<double, 5> t{(double)L.cells[c * nb + q], (double)na, 0, 0, 0};
            for (int i = 0; i < d; ++i) t[2 + i] = Be[a][q][i];
            trips.push_back(t);
          }
        continue;
      }
      for (int b = 0; b < nl; ++b) {
        const int64_t nbn = L.cell_nodes[c * nl + b];
        if (with_mfa) {
          int32_t p = find_in_row(L.mfa_ptr, L.mfa_col, ia, nbn);
          L.mfa_val[p] += Me[a][b];
          if (L.free_of_node[nbn] < 0) {
            int32_t q = find_in_row(L.fb_ptr, L.fb_col, ia, nbn);
            L.fb_m[q] += Me[a][b];
            L.fb_l[q] += nu * Ke[a][b] + Ce[a][b];
          }
        }
        const int64_t ib = L.free_of_node[nbn];
        if (ib < 0) continue;
        int32_t p = find_in_row(L.s_ptr, L.s_col, ia, ib);
        L.s_M[p] += Me[a][b];
        L.s_K1[p] += Ke[a][b];
        conv[p] += Ce[a][b];
      }
      for (int q = 0; q < nb; ++q) {
        int32_t p = find_in_row(L.b_ptr, L.b_col, ia, L.cells[c * nb + q]);
        for (int i = 0; i < d; ++i) L.b_val[(size_t)p * d + i] += Be[a][q][i];
      }
    }
  };
  std::vector<int64_t> gptr, gcells;
  vertex_disjoint_groups(L, gptr, gcells);
  const bool one_group = gptr.size() == 2 && L.nc > 1;  // cells may share vertices
  for (size_t g = 0; g + 1 < gptr.size(); ++g) {
    auto range = [&](int64_t i0, int64_t i1) {
      std::vector<std::array<double, 5>> trips;
      for (int64_t i = i0; i < i1; ++i) cell_body(gcells[gptr[g] + i], trips);
      std::lock_guard<std::mutex> lk(trip_lock);
      bnd_trip.insert(bnd_trip.end(), trips.begin(), trips.end());
    };
    if (one_group) range(0, L.nc);
    else parallel_ranges(gptr[g + 1] - gptr[g], range, 256);
  }
  for (size_t p = 0; p < snnz; ++p) L.s_L[p] = nu * L.s_K1[p] + conv[p];
  // L^T on the same symmetric pattern
  L.s_Lt.assign(snnz, 0.0);
  parallel_ranges(L.nfree, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i)
      for (int32_t p = L.s_ptr[i]; p < L.s_ptr[i + 1]; ++p) {
        int32_t q = find_in_row(L.s_ptr, L.s_col, L.s_col[p], i);
        L.s_Lt[p] = L.s_L[q];
      }
  });
  transpose_csr(L.nfree, L.nv, L.b_ptr, L.b_col, L.b_val, d, L.bt_ptr, L.bt_col, L.bt_val);
  if (with_mfa) {
    // vertex rows x boundary nodes of B^T (the divergence of prescribed velocities)
    std::sort(bnd_trip.begin(), bnd_trip.end());  // by (vertex, node), then the values
    L.vb_ptr.assign(L.nv + 1, 0);
    L.vb_col.clear();
    L.vb_val.clear();
    for (size_t t = 0; t < bnd_trip.size(); ++t) {
      const int64_t v = (int64_t)bnd_trip[t][0];
      const int32_t node = (int32_t)bnd_trip[t][1];
      if (!L.vb_col.empty() && t > 0 && (int64_t)bnd_trip[t - 1][0] == v && L.vb_col.back() == node) {
        for (int i = 0; i < d; ++i) L.vb_val[L.vb_val.size() - d + i] += bnd_trip[t][2 + i];
        continue;
      }
      L.vb_col.push_back(node);
      for (int i = 0; i < d; ++i) L.vb_val.push_back(bnd_trip[t][2 + i]);
      L.vb_ptr[v + 1]++;
    }
    for (int64_t v = 0; v < L.nv; ++v) L.vb_ptr[v + 1] += L.vb_ptr[v];
  }
}

void vertex_disjoint_groups(const HostLevel& L, std::vector<int64_t>& gptr, std::vector<int64_t>& cells) {
  const int nb = L.dim + 1;
  std::vector<uint64_t> used(L.nv, 0);
  std::vector<int8_t> colour(L.nc);
  int ng = 0;
  for (int64_t c = 0; c < L.nc; ++c) {
    const int64_t* v = &L.cells[c * nb];
    uint64_t taken = 0;
    for (int j = 0; j < nb; ++j) taken |= used[v[j]];
    if (taken == ~0ull) {  // more than 64 groups: one group, assembled on one thread
      gptr = {0, L.nc};
      cells.resize(L.nc);
      std::iota(cells.begin(), cells.end(), (int64_t)0);
      return;
    }
    int g = 0;
    while (taken >> g & 1) ++g;
    colour[c] = (int8_t)g;
    ng = std::max(ng, g + 1);
    for (int j = 0; j < nb; ++j) used[v[j]] |= 1ull << g;
  }
  gptr.assign(ng + 1, 0);
  for (int64_t c = 0; c < L.nc; ++c) ++gptr[colour[c] + 1];
  for (int g = 0; g < ng; ++g) gptr[g + 1] += gptr[g];
  cells.resize(L.nc);
  std::vector<int64_t> fill(gptr.begin(), gptr.end() - 1);
  for (int64_t c = 0; c < L.nc; ++c) cells[fill[colour[c]]++] = c;
}

// --------------------------------------------------------------------------- patches
void build_patches(HostLevel& L) {
  const int nl = nloc_of(L.dim);
  // Vertices are independent: ranges of them are handled concurrently in two passes, the
  // first listing each patch's free nodes and counting its coupling entries, the second
  // writing the triples and B positions straight to their final place.
  const int64_t nchunks = std::max<int64_t>(1, std::min<int64_t>(256, L.nv / 1024));
  std::vector<std::vector<int32_t>> cnode(nchunks);
  L.pn_ptr.assign(L.nv + 1, 0);
  L.pvv_ptr.assign(L.nv + 1, 0);
  // the triples (a, b, CSR position) coupling the sorted free nodes of one patch, rows of
  // the list in order and, within a row, its columns in order (one merge of two sorted lists)
  auto couplings = [&](const int32_t* nodes, int32_t n, int32_t* out) {
    int32_t cnt = 0;
    for (int32_t la = 0; la < n; ++la) {
      int32_t p = L.s_ptr[nodes[la]];
      const int32_t pe = L.s_ptr[nodes[la] + 1];
      int32_t lb = 0;
      while (p < pe && lb < n) {
        const int32_t c = L.s_col[p];
        if (c < nodes[lb]) ++p;
        else if (c > nodes[lb]) ++lb;
        else {
          if (out) {
            out[cnt * 3] = la;
            out[cnt * 3 + 1] = lb;
            out[cnt * 3 + 2] = p;
          }
          ++cnt, ++p, ++lb;
        }
      }
    }
    return cnt;
  };
  auto chunk_lo = [&](int64_t k) { return L.nv * k / nchunks; };
  parallel_ranges(nchunks, [&](int64_t k0, int64_t k1) {
    std::vector<int32_t> nodes;
    for (int64_t k = k0; k < k1; ++k)
      for (int64_t v = chunk_lo(k); v < chunk_lo(k + 1); ++v) {
        nodes.clear();
        for (int32_t p = L.node_cell_ptr[v]; p < L.node_cell_ptr[v + 1]; ++p) {
          const int64_t c = L.node_cell[p];
          for (int a = 0; a < nl; ++a) {
            int32_t f = L.free_of_node[L.cell_nodes[c * nl + a]];
            if (f >= 0) nodes.push_back(f);
          }
        }
        std::sort(nodes.begin(), nodes.end());
        nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
        cnode[k].insert(cnode[k].end(), nodes.begin(), nodes.end());
        L.pn_ptr[v + 1] = (int32_t)nodes.size();
        L.pvv_ptr[v + 1] = couplings(nodes.data(), (int32_t)nodes.size(), nullptr);
      }
  }, 1);
  for (int64_t v = 0; v < L.nv; ++v) {
    L.pn_ptr[v + 1] += L.pn_ptr[v];
    if ((int64_t)L.pvv_ptr[v] + L.pvv_ptr[v + 1] > INT32_MAX)
      throw std::runtime_error("patches: more than 2^31 coupling entries on one level");
    L.pvv_ptr[v + 1] += L.pvv_ptr[v];
  }
  L.pn_node.clear();
  L.pn_node.reserve(L.pn_ptr[L.nv]);
  for (const auto& c : cnode) L.pn_node.insert(L.pn_node.end(), c.begin(), c.end());
  L.pvv.assign((size_t)L.pvv_ptr[L.nv] * 3, 0);
  L.pvp.assign(L.pn_node.size(), 0);
  parallel_ranges(L.nv, [&](int64_t v0, int64_t v1) {
    for (int64_t v = v0; v < v1; ++v) {
      const int32_t q0 = L.pn_ptr[v], n = L.pn_ptr[v + 1] - q0;
      couplings(&L.pn_node[q0], n, &L.pvv[(size_t)L.pvv_ptr[v] * 3]);
      for (int32_t la = 0; la < n; ++la) L.pvp[q0 + la] = find_in_row(L.b_ptr, L.b_col, L.pn_node[q0 + la], v);
    }
  }, 1024);
}

// ------------------------------------------------------------------------- transfers
std::string build_transfer(const HostLevel& C, HostLevel& F, const int64_t* parent) {
  const int d = F.dim, nb = d + 1, nlc = nloc_of(d), nlf = nloc_of(d);
  std::vector<char> done_u(F.nfree, 0), done_p(F.nv, 0);
  std::vector<std::vector<std::pair<int32_t, double>>> pu(F.nfree), pp(F.nv);
  F.coarse_node_to_fine_vertex.assign(C.nn, -1);
  double x[3], lam[4], w[10];
  for (int64_t f = 0; f < F.nc; ++f) {
    const int64_t pc = parent[f];
    if (pc < 0 || pc >= C.nc) return "parent index out of range";
    for (int a = 0; a < nlf; ++a) {
      const int64_t node = F.cell_nodes[f * nlf + a];
      const bool is_vertex = a < nb;
      const int64_t fi = F.free_of_node[node];
      const bool need_u = fi >= 0 && !done_u[fi];
      const bool need_p = is_vertex && !done_p[node];
      if (!need_u && !need_p) continue;
      node_coord(F, node, x);
      barycentric(C, pc, x, lam);
      for (int k = 0; k < nb; ++k)
        if (lam[k] < -1e-9) return "fine node outside its parent cell: levels are not nested";
      if (need_u) {
        done_u[fi] = 1;
        p2_values(d, lam, w);
        for (int b = 0; b < nlc; ++b) {
          const int32_t cf = C.free_of_node[C.cell_nodes[pc * nlc + b]];
          if (cf >= 0 && std::fabs(w[b]) > 1e-12) pu[fi].push_back({cf, w[b]});
        }
      }
      if (need_p) {
        done_p[node] = 1;
        for (int k = 0; k < nb; ++k)
          if (std::fabs(lam[k]) > 1e-12) pp[node].push_back({(int32_t)C.cells[pc * nb + k], lam[k]});
        // a fine vertex is a coarse vertex or a coarse edge midpoint
        int ones = 0, halves = 0, kk[2] = {-1, -1};
        for (int k = 0; k < nb; ++k) {
          if (std::fabs(lam[k] - 1.0) < 1e-9) kk[ones++] = k;
          else if (std::fabs(lam[k] - 0.5) < 1e-9 && halves < 2) kk[halves++] = k;
        }
        if (ones == 1) {
          F.coarse_node_to_fine_vertex[C.cells[pc * nb + kk[0]]] = node;
        } else if (halves == 2) {
          const int64_t a0 = C.cells[pc * nb + kk[0]], a1 = C.cells[pc * nb + kk[1]];
          for (int e = 0; e < nlc - nb; ++e) {
            const int64_t cn = C.cell_nodes[pc * nlc + nb + e];
            const int64_t ea = C.edges[(cn - C.nv) * 2], eb = C.edges[(cn - C.nv) * 2 + 1];
            if ((ea == a0 && eb == a1) || (ea == a1 && eb == a0))
              F.coarse_node_to_fine_vertex[cn] = node;
          }
        }
      }
    }
  }
  for (int64_t i = 0; i < F.nfree; ++i)
    if (!done_u[i]) return "fine free node not covered by any cell";
  for (int64_t n = 0; n < C.nn; ++n)
    if (F.coarse_node_to_fine_vertex[n] < 0)
      return "coarse node without a coincident fine vertex: levels are not nested";
  auto to_csr = [](std::vector<std::vector<std::pair<int32_t, double>>>& rows,
                   std::vector<int32_t>& ptr, std::vector<int32_t>& col,
                   std::vector<double>& val) {
    ptr.assign(rows.size() + 1, 0);
    col.clear();
    val.clear();
    for (size_t i = 0; i < rows.size(); ++i) {
      std::sort(rows[i].begin(), rows[i].end());
      for (auto& e : rows[i]) {
        col.push_back(e.first);
        val.push_back(e.second);
      }
      ptr[i + 1] = (int32_t)col.size();
    }
  };
  to_csr(pu, F.pu_ptr, F.pu_col, F.pu_val);
  to_csr(pp, F.pp_ptr, F.pp_col, F.pp_val);
  transpose_csr(F.nfree, C.nfree, F.pu_ptr, F.pu_col, F.pu_val, 1, F.put_ptr, F.put_col,
                F.put_val);
  transpose_csr(F.nv, C.nv, F.pp_ptr, F.pp_col, F.pp_val, 1, F.ppt_ptr, F.ppt_col, F.ppt_val);
  return "";
}

// ---------------------------------------------------------------- coarse inverse
// The per-stage velocity operator of the Newton Jacobian (Sec. 3.2) on the scalar pattern
// of level L for one stage velocity U (nodal, nn x d, node-major): out[p d^2 + c d + e]
// (added to, out zeroed by the caller) = (nu K + C(U))[p] delta_ce + R(U)[p][c][e], with
//   C(U)_ab = int phi_a (U . grad phi_b),   R(U)_(a,c),(b,e) = int phi_a phi_b d_e U_c,
// the two halves of the derivative of the trilinear form c(z, U) + c(U, z).  Exact
// integration with the reference tensor int phi_e phi_a d_lam_k phi_b / |cell| (U is
// quadratic on each cell, so every integrand is a polynomial of degree 5).
// Assembled by rows: each free node sums the contributions of the cells around it to its
// own row, in the order of its cell list, so threads over disjoint row ranges write
// disjoint entries and the result does not depend on the thread count.
void assemble_newton_block(const HostLevel& L, double nu, const double* U, double* out) {
  const int d = L.dim, nb = d + 1, nl = nloc_of(d), dd = d * d;
  const RefTensors& R = ref_tensors(d);
  auto rows = [&](int64_t i0, int64_t i1) {
    double glam[12], vol, wg[10][4], Tg[10][3];
    for (int64_t ia = i0; ia < i1; ++ia) {
      const int64_t na = L.node_of_free[ia];
      for (int32_t q = L.node_cell_ptr[na]; q < L.node_cell_ptr[na + 1]; ++q) {
        const int64_t c = L.node_cell[q];
        const int64_t* cn = &L.cell_nodes[c * nl];
        int a = 0;
        while (cn[a] != na) ++a;
        cell_geometry(L, c, glam, &vol);
        for (int f = 0; f < nl; ++f)
          for (int k = 0; k < nb; ++k) {
            double sum = 0;
            for (int i = 0; i < d; ++i) sum += U[cn[f] * d + i] * glam[k * d + i];
            wg[f][k] = sum;
          }
        for (int b = 0; b < nl; ++b) {
          const int64_t ib = L.free_of_node[cn[b]];
          if (ib < 0) continue;
          double ce = 0;
          for (int f = 0; f < nl; ++f)
            for (int k = 0; k < nb; ++k) ce += wg[f][k] * R.C[((f * nl + a) * nl + b) * nb + k];
          for (int f = 0; f < nl; ++f)
            for (int e = 0; e < d; ++e) {
              double t = 0;
              for (int k = 0; k < nb; ++k) t += glam[k * d + e] * R.C[((a * nl + b) * nl + f) * nb + k];
              Tg[f][e] = t;
            }
          double* o = out + (size_t)find_in_row(L.s_ptr, L.s_col, ia, ib) * dd;
          for (int cc = 0; cc < d; ++cc) {
            o[cc * d + cc] += vol * ce;
            for (int e = 0; e < d; ++e) {
              double t = 0;
              for (int f = 0; f < nl; ++f) t += U[cn[f] * d + cc] * Tg[f][e];
              o[cc * d + e] += vol * t;
            }
          }
        }
      }
      for (int32_t p = L.s_ptr[ia]; p < L.s_ptr[ia + 1]; ++p)
        for (int cc = 0; cc < d; ++cc) out[(size_t)p * dd + cc * d + cc] += nu * L.s_K1[p];
    }
  };
  const int64_t n = L.nfree;
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>({16, (int64_t)std::thread::hardware_concurrency(),
                                                              n / 4096}));
  if (nt == 1) {
    rows(0, n);
    return;
  }
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t) pool.emplace_back(rows, n * t / nt, n * (t + 1) / nt);
  for (auto& th : pool) th.join();
}

// Dense coarse operator of the Newton Jacobian (row-major, internal layout, pressure of
// vertex 0 pinned in every stage): block (s, t) = delta_st M + dt a_st [N_s B; B^T 0] with
// N_s from nw[(p r + s) d^2 + c d + e].
void coarse_matrix_newton(const HostLevel& L, int r, const double* A, double dt, const double* nw,
                          std::vector<double>& J, double* max_abs) {
  const int d = L.dim, dd = d * d;
  const int64_t offV = L.nfree * d * r;
  const int64_t N = offV + L.nv * r;
  J.assign((size_t)N * N, 0.0);
  auto vel = [&](int64_t i, int c, int s) { return (i * d + c) * r + s; };
  auto pre = [&](int64_t v, int s) { return offV + v * r + s; };
  for (int64_t i = 0; i < L.nfree; ++i) {
    for (int32_t p = L.s_ptr[i]; p < L.s_ptr[i + 1]; ++p) {
      const int64_t j = L.s_col[p];
      for (int s = 0; s < r; ++s)
        for (int t = 0; t < r; ++t)
          for (int c = 0; c < d; ++c)
            for (int e = 0; e < d; ++e)
              J[vel(i, c, s) * N + vel(j, e, t)] += (s == t && c == e ? L.s_M[p] : 0.0) +
                                                    dt * A[s * r + t] * nw[((size_t)p * r + s) * dd + c * d + e];
    }
    for (int32_t p = L.b_ptr[i]; p < L.b_ptr[i + 1]; ++p) {
      const int64_t v = L.b_col[p];
      for (int c = 0; c < d; ++c)
        for (int s = 0; s < r; ++s)
          for (int t = 0; t < r; ++t) {
            const double val = dt * A[s * r + t] * L.b_val[(size_t)p * d + c];
            J[vel(i, c, s) * N + pre(v, t)] += val;
            J[pre(v, s) * N + vel(i, c, t)] += val;
          }
    }
  }
  for (int s = 0; s < r; ++s) {
    const int64_t q = pre(0, s);
    for (int64_t k = 0; k < N; ++k) {
      J[q * N + k] = 0.0;
      J[k * N + q] = 0.0;
    }
    J[q * N + q] = 1.0;
  }
  double scale = 0;
  for (double v : J) scale = std::max(scale, std::fabs(v));
  *max_abs = scale;
}

void coarse_matrix(const HostLevel& L, int r, const double* A, double dt, std::vector<double>& J,
                   double* max_abs) {
  const int d = L.dim;
  const int64_t offV = L.nfree * d * r;
  const int64_t N = offV + L.nv * r;
  J.assign((size_t)N * N, 0.0);  // row-major
  auto vel = [&](int64_t i, int c, int s) { return (i * d + c) * r + s; };
  auto pre = [&](int64_t v, int s) { return offV + v * r + s; };
  for (int64_t i = 0; i < L.nfree; ++i) {
    for (int32_t p = L.s_ptr[i]; p < L.s_ptr[i + 1]; ++p) {
      const int64_t j = L.s_col[p];
      for (int c = 0; c < d; ++c)
        for (int s = 0; s < r; ++s)
          for (int t = 0; t < r; ++t)
            J[vel(i, c, s) * N + vel(j, c, t)] +=
                (s == t ? L.s_M[p] : 0.0) + dt * A[s * r + t] * L.s_L[p];
    }
    for (int32_t p = L.b_ptr[i]; p < L.b_ptr[i + 1]; ++p) {
      const int64_t v = L.b_col[p];
      for (int c = 0; c < d; ++c)
        for (int s = 0; s < r; ++s)
          for (int t = 0; t < r; ++t) {
            const double val = dt * A[s * r + t] * L.b_val[(size_t)p * d + c];
            J[vel(i, c, s) * N + pre(v, t)] += val;
            J[pre(v, s) * N + vel(i, c, t)] += val;
          }
    }
  }
  for (int s = 0; s < r; ++s) {  // pin the pressure of vertex 0 in every stage
    const int64_t q = pre(0, s);
    for (int64_t k = 0; k < N; ++k) {
      J[q * N + k] = 0.0;
      J[k * N + q] = 0.0;
    }
    J[q * N + q] = 1.0;
  }
  double scale = 0;
  for (double v : J) scale = std::max(scale, std::fabs(v));
  *max_abs = scale;
}

void ns_cell_data(const HostLevel& L, std::vector<double>& geo, std::vector<int32_t>& cell_nodes,
                  std::vector<int32_t>& cell_free, std::vector<int32_t>& inc_ptr, std::vector<int32_t>& inc) {
  const int d = L.dim, nb = d + 1, nl = nloc_of(d);
  const int per = nb * d + 1;
  geo.assign((size_t)L.nc * per, 0.0);
  for (int64_t c = 0; c < L.nc; ++c) cell_geometry(L, c, &geo[(size_t)c * per], &geo[(size_t)c * per + nb * d]);
  cell_nodes.resize(L.cell_nodes.size());
  cell_free.resize(L.cell_nodes.size());
  for (size_t i = 0; i < L.cell_nodes.size(); ++i) {
    cell_nodes[i] = (int32_t)L.cell_nodes[i];
    cell_free[i] = L.free_of_node[L.cell_nodes[i]];
  }
  inc_ptr.assign(L.nfree + 1, 0);
  inc.clear();
  for (int64_t f = 0; f < L.nfree; ++f) {
    const int64_t n = L.node_of_free[f];
    for (int32_t q = L.node_cell_ptr[n]; q < L.node_cell_ptr[n + 1]; ++q) {
      const int64_t c = L.node_cell[q];
      for (int a = 0; a < nl; ++a)
        if (L.cell_nodes[c * nl + a] == n) inc.push_back((int32_t)(c * nl + a));
    }
    inc_ptr[f + 1] = (int32_t)inc.size();
  }
}

}  // namespace irk

// ------------------------------------------------------------- stage eigenbasis
namespace irk {
namespace {
using cplx = std::complex<double>;

// Solve B x = y for a small complex matrix (Gaussian elimination, partial pivoting);
// false on an exactly zero pivot.
bool csolve(int r, std::vector<cplx> B, std::vector<cplx>& y) {
  for (int k = 0; k < r; ++k) {
    int piv = k;
    for (int i = k + 1; i < r; ++i)
      if (std::abs(B[i * r + k]) > std::abs(B[piv * r + k])) piv = i;
    if (std::abs(B[piv * r + k]) == 0.0) return false;
    if (piv != k) {
      for (int j = 0; j < r; ++j) std::swap(B[k * r + j], B[piv * r + j]);
      std::swap(y[k], y[piv]);
    }
    for (int i = k + 1; i < r; ++i) {
      const cplx f = B[i * r + k] / B[k * r + k];
      for (int j = k; j < r; ++j) B[i * r + j] -= f * B[k * r + j];
      y[i] -= f * y[k];
    }
  }
  for (int k = r - 1; k >= 0; --k) {
    cplx s = y[k];
    for (int j = k + 1; j < r; ++j) s -= B[k * r + j] * y[j];
    y[k] = s / B[k * r + k];
  }
  return true;
}

bool rinverse(int r, const double* M, double* inv) {
  std::vector<cplx> cols(r * r);
  for (int j = 0; j < r; ++j) {
    std::vector<cplx> B(r * r), e(r, 0.0);
    for (int i = 0; i < r * r; ++i) B[i] = M[i];
    e[j] = 1.0;
    if (!csolve(r, B, e)) return false;
    for (int i = 0; i < r; ++i) inv[i * r + j] = e[i].real();
  }
  return true;
}

double inf_norm(int r, const double* M) {
  double m = 0;
  for (int i = 0; i < r; ++i) {
    double s = 0;
    for (int j = 0; j < r; ++j) s += std::fabs(M[i * r + j]);
    m = std::max(m, s);
  }
  return m;
}
}  // namespace

bool hessenberg_eigs_ws(int m, const double* H, int ldh, double* wr, double* wi, std::complex<double>* work,
                        int* iwork) {
  using C = std::complex<double>;
  if (m < 1) return true;
  C* a = work;  // row-major working copy
  for (size_t q = 0; q < (size_t)m * m; ++q) a[q] = C(0.0);
  double nrm = 0.0;
  for (int j = 0; j < m; ++j)
    for (int i = 0; i <= std::min(j + 1, m - 1); ++i) {
      a[(size_t)i * m + j] = H[(size_t)j * ldh + i];
      nrm = std::max(nrm, std::abs(H[(size_t)j * ldh + i]));
    }
  auto A = [&](int i, int j) -> C& { return a[(size_t)i * m + j]; };
  C* ev = work + (size_t)m * m;
  C* cs = ev + m;
  C* sn = cs + m;
  const double eps = 4.0 * 2.220446049250313e-16;
  int hi = m - 1, iter = 0;
  while (hi >= 0) {
    // the active block is [l, hi]: the subdiagonal entry above row l is negligible
    int l = hi;
    while (l > 0) {
      double s = std::abs(A(l - 1, l - 1)) + std::abs(A(l, l));
      if (s == 0.0) s = nrm;
      if (std::abs(A(l, l - 1)) <= eps * s) {
        A(l, l - 1) = 0.0;
        break;
      }
      --l;
    }
    if (l == hi) {  // a 1 x 1 block: its entry is an eigenvalue
      ev[hi] = A(hi, hi);
      --hi;
      iter = 0;
      continue;
    }
    if (++iter > 100 * m) return false;
    // shift: the eigenvalue of the trailing 2 x 2 closer to its last diagonal entry
    // (Wilkinson), replaced by an ad hoc value every 11th iteration to break cycles
    const C p = A(hi - 1, hi - 1), q = A(hi - 1, hi), r = A(hi, hi - 1), d = A(hi, hi);
    const C half = 0.5 * (p + d), disc = std::sqrt(0.25 * (p - d) * (p - d) + q * r);
    C mu = std::abs(half + disc - d) < std::abs(half - disc - d) ? half + disc : half - disc;
    if (iter % 11 == 0) mu = d + 0.75 * std::abs(r);
    // one QR step on the block: B - mu I = Q R by Givens rotations, B <- R Q + mu I
    for (int k = l; k <= hi; ++k) A(k, k) -= mu;
    for (int k = l; k < hi; ++k) {
      const C x = A(k, k), y = A(k + 1, k);
      const double rr = std::sqrt(std::norm(x) + std::norm(y));
      const C c = rr > 0.0 ? x / rr : C(1.0), s = rr > 0.0 ? y / rr : C(0.0);
      cs[k - l] = c;
      sn[k - l] = s;
      for (int j = k; j <= hi; ++j) {
        const C t1 = A(k, j), t2 = A(k + 1, j);
        A(k, j) = std::conj(c) * t1 + std::conj(s) * t2;
        A(k + 1, j) = -s * t1 + c * t2;
      }
    }
    for (int k = l; k < hi; ++k) {
      const C c = cs[k - l], s = sn[k - l];
      for (int i = l; i <= std::min(k + 1, hi); ++i) {
        const C t1 = A(i, k), t2 = A(i, k + 1);
        A(i, k) = t1 * c + t2 * s;
        A(i, k + 1) = -t1 * std::conj(s) + t2 * std::conj(c);
      }
    }
    for (int k = l; k <= hi; ++k) A(k, k) += mu;
  }
  // order by decreasing real part, ties in index order (a stable insertion sort, no
  // temporary storage)
  int* order = iwork;
  for (int k = 0; k < m; ++k) {
    int q = k;
    while (q > 0 && ev[order[q - 1]].real() < ev[k].real()) {
      order[q] = order[q - 1];
      --q;
    }
    order[q] = k;
  }
  for (int k = 0; k < m; ++k) {
    wr[k] = ev[order[k]].real();
    wi[k] = ev[order[k]].imag();
  }
  return true;
}

bool hessenberg_eigs(int m, const double* H, int ldh, double* wr, double* wi) {
  if (m < 1) return true;
  std::vector<std::complex<double>> work((size_t)m * m + 3 * (size_t)m);
  std::vector<int> iwork(m);
  return hessenberg_eigs_ws(m, H, ldh, wr, wi, work.data(), iwork.data());
}

bool stage_eigenbasis(const double* A, int r, StageEig& out, std::string* why) {
  auto fail = [&](const std::string& m) {
    if (why) *why = m;
    return false;
  };
  out = StageEig();
  out.r = r;
  if (r < 1 || r > kMaxStages) return fail("stage count outside 1..4");
  double amax = 0;
  for (int i = 0; i < r * r; ++i) amax = std::max(amax, std::fabs(A[i]));
  const double scale = std::max(amax, 1e-300);
  // characteristic polynomial (Faddeev--LeVerrier): p(z) = sum_k c[k] z^k, c[r] = 1
  std::vector<double> c(r + 1, 0.0), Mk(r * r, 0.0), AM(r * r);
  c[r] = 1.0;
  for (int k = 1; k <= r; ++k) {
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < r; ++j) {
        double s = 0;
        for (int q = 0; q < r; ++q) s += A[i * r + q] * Mk[q * r + j];
        AM[i * r + j] = s;
      }
    for (int i = 0; i < r * r; ++i) Mk[i] = AM[i];
    for (int i = 0; i < r; ++i) Mk[i * r + i] += c[r - k + 1];
    double tr = 0;
    for (int i = 0; i < r; ++i)
      for (int q = 0; q < r; ++q) tr += A[i * r + q] * Mk[q * r + i];
    c[r - k] = -tr / k;
  }
  auto peval = [&](cplx z, cplx* dp) {
    cplx p = c[r], d = 0.0;
    for (int k = r - 1; k >= 0; --k) {
      d = d * z + p;
      p = p * z + c[k];
    }
    if (dp) *dp = d;
    return p;
  };
  // roots: Durand--Kerner (simultaneous Weierstrass iteration), then Newton polishing
  std::vector<cplx> z(r);
  const cplx seed(0.4, 0.9);
  for (int i = 0; i < r; ++i) z[i] = scale * std::pow(seed, i);
  for (int it = 0; it < 2000; ++it) {
    double change = 0;
    for (int i = 0; i < r; ++i) {
      cplx den = 1.0;
      for (int j = 0; j < r; ++j)
        if (j != i) den *= z[i] - z[j];
      if (std::abs(den) == 0.0) den = 1e-300;
      const cplx dz = peval(z[i], nullptr) / den;
      z[i] -= dz;
      change = std::max(change, std::abs(dz));
    }
    if (change <= 1e-16 * scale) break;
  }
  for (int i = 0; i < r; ++i)
    for (int it = 0; it < 3; ++it) {
      cplx d;
      const cplx p = peval(z[i], &d);
      if (std::abs(d) == 0.0) break;
      z[i] -= p / d;
    }
  for (int i = 0; i < r; ++i)
    for (int j = i + 1; j < r; ++j)
      if (std::abs(z[i] - z[j]) <= 1e-6 * scale) return fail("repeated eigenvalues of A");
  // blocks: real eigenvalues first (ascending), then pairs with b > 0 (ascending a)
  std::vector<double> reals;
  std::vector<cplx> pairs;
  for (int i = 0; i < r; ++i) {
    if (std::fabs(z[i].imag()) <= 1e-10 * scale) reals.push_back(z[i].real());
    else if (z[i].imag() > 0) pairs.push_back(z[i]);
  }
  if ((int)reals.size() + 2 * (int)pairs.size() != r) return fail("unpaired complex eigenvalue");
  std::sort(reals.begin(), reals.end());
  std::sort(pairs.begin(), pairs.end(), [](cplx a, cplx b) { return a.real() < b.real(); });
  // eigenvectors by inverse iteration with a slightly shifted eigenvalue
  auto eigvec = [&](cplx lam) {
    std::vector<cplx> v(r);
    for (int i = 0; i < r; ++i) v[i] = 1.0 + 0.1 * i;
    const cplx mu = lam + cplx(1e-10, 1e-10) * std::max(1.0, std::abs(lam));
    for (int it = 0; it < 4; ++it) {
      std::vector<cplx> B(r * r);
      for (int i = 0; i < r; ++i)
        for (int j = 0; j < r; ++j) B[i * r + j] = A[i * r + j] - (i == j ? mu : cplx(0.0));
      if (!csolve(r, B, v)) break;  // mu hit the eigenvalue exactly: v is converged
      double nrm = 0;
      int big = 0;
      for (int i = 0; i < r; ++i) {
        nrm += std::norm(v[i]);
        if (std::abs(v[i]) > std::abs(v[big])) big = i;
      }
      const cplx ph = v[big] / std::abs(v[big]);
      for (int i = 0; i < r; ++i) v[i] /= ph * std::sqrt(nrm);
    }
    return v;
  };
  int col = 0;
  for (double lam : reals) {
    const std::vector<cplx> v = eigvec(lam);
    for (int i = 0; i < r; ++i) out.W[i * r + col] = v[i].real();
    out.type[out.nblk] = 1;
    out.st0[out.nblk] = col;
    out.Tb[out.nblk][0] = lam;
    ++out.nblk;
    col += 1;
  }
  for (cplx lam : pairs) {
    // A (p + iq) = (a + ib)(p + iq)  =>  A [p q] = [p q] [[a, b], [-b, a]]
    const std::vector<cplx> v = eigvec(lam);
    for (int i = 0; i < r; ++i) {
      out.W[i * r + col] = v[i].real();
      out.W[i * r + col + 1] = v[i].imag();
    }
    out.type[out.nblk] = 2;
    out.st0[out.nblk] = col;
    out.Tb[out.nblk][0] = lam.real();
    out.Tb[out.nblk][1] = lam.imag();
    out.Tb[out.nblk][2] = -lam.imag();
    out.Tb[out.nblk][3] = lam.real();
    ++out.nblk;
    col += 2;
  }
  if (!rinverse(r, out.W, out.Winv)) return fail("singular eigenvector matrix");
  out.cond = inf_norm(r, out.W) * inf_norm(r, out.Winv);
  if (!(out.cond <= 1e6)) return fail("ill-conditioned eigenvector matrix");
  // reconstruction W T W^{-1} against A
  std::vector<double> T(r * r, 0.0), WT(r * r, 0.0);
  for (int b = 0; b < out.nblk; ++b)
    for (int i = 0; i < out.type[b]; ++i)
      for (int j = 0; j < out.type[b]; ++j)
        T[(out.st0[b] + i) * r + out.st0[b] + j] = out.Tb[b][i * out.type[b] + j];
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j)
      for (int q = 0; q < r; ++q) WT[i * r + j] += out.W[i * r + q] * T[q * r + j];
  double err = 0;
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      double s = 0;
      for (int q = 0; q < r; ++q) s += WT[i * r + q] * out.Winv[q * r + j];
      err = std::max(err, std::fabs(s - A[i * r + j]));
    }
  out.recon = err;
  if (!(err <= 1e-13 * scale * std::max(1.0, out.cond))) return fail("eigen-decomposition check failed");
  return true;
}
}  // namespace irk

// ---------------------------------------------------------------- sliced operators
namespace irk {
Sell build_sell(int64_t nrows, const std::vector<int32_t>& ptr, const std::vector<int32_t>& col) {
  Sell S;
  S.nslices = (nrows + 63) / 64;
  S.off.resize(S.nslices + 1);
  S.w.resize(S.nslices);
  int64_t total = 0;
  for (int64_t sl = 0; sl < S.nslices; ++sl) {
    int w = 0;
    for (int64_t row = sl * 64; row < std::min(nrows, sl * 64 + 64); ++row) w = std::max(w, ptr[row + 1] - ptr[row]);
    S.w[sl] = w;
    S.off[sl] = (int32_t)total;
    total += (int64_t)w * 64;
    if (total > INT32_MAX) throw std::runtime_error("operator too large for 32-bit sliced offsets");
  }
  S.off[S.nslices] = (int32_t)total;
  S.col.assign(total, 0);
  S.src.assign(total, -1);
  for (int64_t sl = 0; sl < S.nslices; ++sl)
    for (int lane = 0; lane < 64; ++lane) {
      const int64_t row = sl * 64 + lane;
      if (row >= nrows) continue;
      for (int32_t p = ptr[row]; p < ptr[row + 1]; ++p) {
        const int64_t e = S.off[sl] + (int64_t)(p - ptr[row]) * 64 + lane;
        S.col[e] = col[p];
        S.src[e] = p;
      }
    }
  return S;
}

std::vector<double> sell_values(const Sell& S, const std::vector<double>& v, int k) {
  std::vector<double> out(S.src.size() * k, 0.0);
  for (size_t e = 0; e < S.src.size(); ++e)
    if (S.src[e] >= 0)
      for (int c = 0; c < k; ++c) out[e * k + c] = v[S.src[e] * k + c];
  return out;
}

// ---------------------------------------------- element helpers for other assemblies
void fe_cell_geometry(const HostLevel& L, int64_t c, double* glam, double* vol) { cell_geometry(L, c, glam, vol); }
void fe_barycentric(const HostLevel& L, int64_t c, const double* x, double* lam) { barycentric(L, c, x, lam); }
int32_t fe_find_in_row(const std::vector<int32_t>& ptr, const std::vector<int32_t>& col, int64_t row, int64_t c) {
  return find_in_row(ptr, col, row, c);
}
void fe_csr_from_rows(std::vector<std::vector<int32_t>>& rows, std::vector<int32_t>& ptr, std::vector<int32_t>& col) {
  csr_from_rows(rows, ptr, col);
}
void fe_transpose_csr(int64_t nrows, int64_t ncols, const std::vector<int32_t>& ptr, const std::vector<int32_t>& col,
                      const std::vector<double>& val, std::vector<int32_t>& tptr, std::vector<int32_t>& tcol,
                      std::vector<double>& tval) {
  transpose_csr(nrows, ncols, ptr, col, val, 1, tptr, tcol, tval);
}
void fe_p2_lam_moments(int dim, double* out) {
  const int nl = nloc_of(dim), nb = dim + 1;
  for (int a = 0; a < nl; ++a)
    for (int i = 0; i < nb; ++i) out[a * nb + i] = integrate(mul(basis(dim, a), lam_pow(i, 1, 1.0)), dim);
}
const double* fe_p2_grad_grad(int dim) { return ref_tensors(dim).S.data(); }
const double* fe_p2_conv_tensor(int dim) { return ref_tensors(dim).C.data(); }
}  // namespace irk
