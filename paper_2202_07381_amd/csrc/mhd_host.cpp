// Host setup of the linearised 2D MHD stage system (Sec. 3.3): index maps, exact element
// matrices of the P2 / Nedelec / P1 couplings, the vertex patches of Fig. 1 (right), the
// Nedelec interpolation between nested levels (Sec. 4.1) and the rediscretised coarse
// states.  Untimed setup; the solve-time arithmetic runs in the HIP kernels.
//
// Nedelec basis on a cell: for the edge with end vertices lo, hi (lo the smaller global
// number) phi = lam_lo grad lam_hi - lam_hi grad lam_lo, so each component is linear in
// the barycentric coordinates, phi = sum_i lam_i alpha_i with alpha_lo = grad lam_hi,
// alpha_hi = -grad lam_lo and alpha_i = 0 at the third vertex; its curl is the constant
// 2 grad lam_lo x grad lam_hi.  A field sum_e b_e phi_e has coefficients
// beta_i = sum_e b_e alpha^e_i and curl sum_e b_e curl phi_e.  Every integral below is a
// product of such linear factors with at most one P2 function (or two constants), so it
// reduces exactly to the moments int lam_i lam_j / |T| = (1 + delta_ij) / 12,
// int lam_i / |T| = 1/3 and int phi_a lam_i / |T| (phi_a a P2 basis function).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <stdexcept>
#include <utility>

#include "mhd_internal.h"

namespace irk {
namespace {

const int kE2[3][2] = {{0, 1}, {0, 2}, {1, 2}};  // local edges, the P2 numbering's order

struct CellNed {
  double glam[3][2], vol;
  double alpha[3][3][2];  // [edge][vertex][component]
  double curl[3];
  int64_t edge[3];  // global edge ids
};

void cell_nedelec(const HostLevel& L, int64_t c, CellNed& N) {
  double g[6];
  fe_cell_geometry(L, c, g, &N.vol);
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 2; ++k) N.glam[i][k] = g[i * 2 + k];
  const int64_t* v = &L.cells[c * 3];
  for (int e = 0; e < 3; ++e) {
    int lo = kE2[e][0], hi = kE2[e][1];
    if (v[lo] > v[hi]) std::swap(lo, hi);
    for (int i = 0; i < 3; ++i) N.alpha[e][i][0] = N.alpha[e][i][1] = 0.0;
    for (int k = 0; k < 2; ++k) {
      N.alpha[e][lo][k] = N.glam[hi][k];
      N.alpha[e][hi][k] = -N.glam[lo][k];
    }
    N.curl[e] = 2.0 * (N.glam[lo][0] * N.glam[hi][1] - N.glam[lo][1] * N.glam[hi][0]);
    N.edge[e] = L.cell_nodes[c * 6 + 3 + e] - L.nv;
  }
}

// sorted position of the edge (a, b) of L, or -1
int64_t find_edge(const HostLevel& L, int64_t a, int64_t b) {
  if (a > b) std::swap(a, b);
  int64_t lo = 0, hi = L.ne;
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    const int64_t ma = L.edges[2 * mid], mb = L.edges[2 * mid + 1];
    if (ma < a || (ma == a && mb < b)) lo = mid + 1;
    else hi = mid;
  }
  return lo < L.ne && L.edges[2 * lo] == a && L.edges[2 * lo + 1] == b ? lo : -1;
}

// the unknowns of one cell: velocity (component c, local node a) or -1, interior edges,
// vertices (pressure), interior vertices (multiplier) or -1
struct CellDofs {
  int64_t u[2][6], e[3], p[3], g[3];
};

void cell_dofs(const MhdHost& H, int64_t c, CellDofs& d) {
  const HostLevel& L = H.L;
  for (int a = 0; a < 6; ++a) {
    const int32_t f = L.free_of_node[L.cell_nodes[c * 6 + a]];
    for (int k = 0; k < 2; ++k) d.u[k][a] = f < 0 ? -1 : k * H.nfree + f;
  }
  for (int e = 0; e < 3; ++e) {
    const int32_t b = H.eidx[L.cell_nodes[c * 6 + 3 + e] - L.nv];
    d.e[e] = b < 0 ? -1 : H.off_B + b;
  }
  for (int j = 0; j < 3; ++j) {
    const int64_t v = L.cells[c * 3 + j];
    d.p[j] = H.off_p + v;
    d.g[j] = H.gidx[v] < 0 ? -1 : H.off_g + H.gidx[v];
  }
}

}  // namespace

void mhd_index(MhdHost& H) {
  const HostLevel& L = H.L;
  H.nfree = L.nfree;
  H.nv = L.nv;
  H.eidx.assign(L.ne, -1);
  H.efree.clear();
  for (int64_t e = 0; e < L.ne; ++e)
    if (L.free_of_node[L.nv + e] >= 0) {
      H.eidx[e] = (int32_t)H.efree.size();
      H.efree.push_back((int32_t)e);
    }
  H.gidx.assign(L.nv, -1);
  H.vint.clear();
  for (int64_t v = 0; v < L.nv; ++v)
    if (L.free_of_node[v] >= 0) {
      H.gidx[v] = (int32_t)H.vint.size();
      H.vint.push_back((int32_t)v);
    }
  H.nB = (int64_t)H.efree.size();
  H.ng = (int64_t)H.vint.size();
  H.off_B = 2 * H.nfree;
  H.off_p = H.off_B + H.nB;
  H.off_g = H.off_p + H.nv;
  H.ns = H.off_g + H.ng;
}

void mhd_assemble(MhdHost& H, double Re, double Rem, const double* w, const double* b0) {
  const HostLevel& L = H.L;
  const int64_t nf = H.nfree;
  // ---- pattern: the couplings of the weak form within each cell; a row's columns are
  // the unknowns its cells couple it to, so each row is gathered from the cells around
  // its node (rows independent, built concurrently)
  {
    std::vector<std::vector<int32_t>> rows(H.ns);
    parallel_ranges(H.ns, [&](int64_t r0, int64_t r1) {
      CellDofs d;
      for (int64_t r = r0; r < r1; ++r) {
        std::vector<int32_t>& row = rows[r];
        int kind;  // 0 velocity, 1 field, 2 pressure, 3 multiplier
        int64_t node;
        if (r < 2 * nf) kind = 0, node = L.node_of_free[r < nf ? r : r - nf];
        else if (r < H.off_p) kind = 1, node = L.nv + H.efree[r - H.off_B];
        else if (r < H.off_g) kind = 2, node = r - H.off_p;
        else kind = 3, node = H.vint[r - H.off_g];
        auto add = [&](int64_t c) {
          if (c >= 0) row.push_back((int32_t)c);
        };
        for (int32_t q = L.node_cell_ptr[node]; q < L.node_cell_ptr[node + 1]; ++q) {
          cell_dofs(H, L.node_cell[q], d);
          if (kind <= 2)
            for (int k2 = 0; k2 < 2; ++k2)
              for (int b = 0; b < 6; ++b) add(d.u[k2][b]);
          if (kind != 2)
            for (int f = 0; f < 3; ++f) add(d.e[f]);
          for (int j = 0; j < 3; ++j) {
            if (kind == 0) add(d.p[j]);
            if (kind == 1) add(d.g[j]);
          }
        }
        std::sort(row.begin(), row.end());
        row.erase(std::unique(row.begin(), row.end()), row.end());
      }
    });
    fe_csr_from_rows(rows, H.ptr, H.col);
  }
  H.mval.assign(H.col.size(), 0.0);
  H.sval.assign(H.col.size(), 0.0);
  auto at = [&](int64_t r, int64_t c) -> size_t {
    const int32_t p = fe_find_in_row(H.ptr, H.col, r, c);
    if (p < 0) throw std::runtime_error("MHD assembly: entry outside the pattern");
    return (size_t)p;
  };
  // ---- velocity blocks from the scalar P2 ones: mass, (1/Re) grad-grad on each
  // component, the Newton convection N'(w), and the divergence couplings
  {
    std::vector<double> nw(L.s_col.size() * 4, 0.0);
    assemble_newton_block(L, 0.0, w, nw.data());
    // rows of the free node i (both components): written by i's range only
    parallel_ranges(nf, [&](int64_t i0, int64_t i1) {
      for (int64_t i = i0; i < i1; ++i) {
        for (int32_t p = L.s_ptr[i]; p < L.s_ptr[i + 1]; ++p) {
          const int64_t j = L.s_col[p];
          for (int c = 0; c < 2; ++c) {
            const size_t q = at(c * nf + i, c * nf + j);
            H.mval[q] += L.s_M[p];
            H.sval[q] += L.s_K1[p] / Re;
            for (int e = 0; e < 2; ++e) H.sval[at(c * nf + i, e * nf + j)] += nw[(size_t)p * 4 + c * 2 + e];
          }
        }
        for (int32_t p = L.b_ptr[i]; p < L.b_ptr[i + 1]; ++p)
          for (int c = 0; c < 2; ++c) H.sval[at(c * nf + i, H.off_p + L.b_col[p])] += L.b_val[(size_t)p * 2 + c];
      }
    });
    // pressure rows from the transposed divergence (B^T: vertex -> free nodes)
    parallel_ranges(H.nv, [&](int64_t v0, int64_t v1) {
      for (int64_t v = v0; v < v1; ++v)
        for (int32_t p = L.bt_ptr[v]; p < L.bt_ptr[v + 1]; ++p)
          for (int c = 0; c < 2; ++c) H.sval[at(H.off_p + v, c * nf + L.bt_col[p])] += L.bt_val[(size_t)p * 2 + c];
    });
  }
  // ---- cell terms
  double T1[6][3];
  fe_p2_lam_moments(2, &T1[0][0]);
  const double* RS = fe_p2_grad_grad(2);
  auto cell_terms = [&](int64_t c) {
    CellNed N;
    CellDofs d;
    cell_nedelec(L, c, N);
    cell_dofs(H, c, d);
    const double vol = N.vol;
    const int64_t* cn = &L.cell_nodes[c * 6];
    double bc[3], beta[3][2] = {{0, 0}, {0, 0}, {0, 0}}, j0 = 0.0;
    for (int e = 0; e < 3; ++e) {
      bc[e] = b0[N.edge[e]];
      j0 += bc[e] * N.curl[e];
      for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 2; ++k) beta[i][k] += bc[e] * N.alpha[e][i][k];
    }
    // int phi_a B0_k / |T| and int phi_a (phi_f)_k / |T|
    double SB[6][2], SA[6][3][2];
    for (int a = 0; a < 6; ++a)
      for (int k = 0; k < 2; ++k) {
        double s = 0;
        for (int i = 0; i < 3; ++i) s += beta[i][k] * T1[a][i];
        SB[a][k] = s;
        for (int f = 0; f < 3; ++f) {
          double t = 0;
          for (int i = 0; i < 3; ++i) t += N.alpha[f][i][k] * T1[a][i];
          SA[a][f][k] = t;
        }
      }
    // velocity-velocity: the second half of the symmetric gradient,
    // (1/Re) int d_e phi_a d_c phi_b for test (c, a), trial (e, b)
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b < 6; ++b)
        for (int cc = 0; cc < 2; ++cc) {
          if (d.u[cc][a] < 0) continue;
          for (int e = 0; e < 2; ++e) {
            if (d.u[e][b] < 0) continue;
            double s = 0;
            for (int k = 0; k < 3; ++k)
              for (int l = 0; l < 3; ++l) s += N.glam[k][e] * N.glam[l][cc] * RS[((a * 6 + b) * 3 + k) * 3 + l];
            H.sval[at(d.u[cc][a], d.u[e][b])] += vol * s / Re;
          }
        }
    // Lorentz force -((curl B) x B0 + (curl B0) x B) . v: test (c, a), trial edge f
    for (int a = 0; a < 6; ++a)
      for (int f = 0; f < 3; ++f) {
        if (d.e[f] < 0) continue;
        if (d.u[0][a] >= 0) H.sval[at(d.u[0][a], d.e[f])] += vol * (N.curl[f] * SB[a][1] + j0 * SA[a][f][1]);
        if (d.u[1][a] >= 0) H.sval[at(d.u[1][a], d.e[f])] -= vol * (N.curl[f] * SB[a][0] + j0 * SA[a][f][0]);
      }
    // induction from the velocity -(u x B0, curl c): test edge g, trial (e, b)
    for (int g = 0; g < 3; ++g) {
      if (d.e[g] < 0) continue;
      for (int b = 0; b < 6; ++b) {
        if (d.u[0][b] >= 0) H.sval[at(d.e[g], d.u[0][b])] -= vol * N.curl[g] * SB[b][1];
        if (d.u[1][b] >= 0) H.sval[at(d.e[g], d.u[1][b])] += vol * N.curl[g] * SB[b][0];
      }
    }
    // magnetic block (1/Rem)(curl B, curl c) - (w x B, curl c) and the mass (B, c)
    for (int g = 0; g < 3; ++g) {
      if (d.e[g] < 0) continue;
      for (int f = 0; f < 3; ++f) {
        if (d.e[f] < 0) continue;
        double wx = 0;  // int (w_x phi_f,y - w_y phi_f,x) / |T|
        for (int n = 0; n < 6; ++n) wx += w[cn[n] * 2] * SA[n][f][1] - w[cn[n] * 2 + 1] * SA[n][f][0];
        const size_t q = at(d.e[g], d.e[f]);
        H.sval[q] += vol * (N.curl[f] * N.curl[g] / Rem - N.curl[g] * wx);
        double m = 0;
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j)
            m += (N.alpha[f][i][0] * N.alpha[g][j][0] + N.alpha[f][i][1] * N.alpha[g][j][1]) *
                 (i == j ? 2.0 : 1.0) / 12.0;
        H.mval[q] += vol * m;
      }
    }
    // multiplier: -(grad gamma, c) and -(B, grad s), int phi_g . grad lam_j
    for (int g = 0; g < 3; ++g) {
      if (d.e[g] < 0) continue;
      for (int j = 0; j < 3; ++j) {
        if (d.g[j] < 0) continue;
        double s = 0;
        for (int k = 0; k < 2; ++k) {
          double ak = 0;
          for (int i = 0; i < 3; ++i) ak += N.alpha[g][i][k];
          s += N.glam[j][k] * ak / 3.0;
        }
        H.sval[at(d.e[g], d.g[j])] -= vol * s;
        H.sval[at(d.g[j], d.e[g])] -= vol * s;
      }
    }
  };
  // cells of one vertex-disjoint group write disjoint rows
  for_cells_by_groups(L, cell_terms);
}

void mhd_patches(MhdHost& H) {
  const HostLevel& L = H.L;
  // Vertices are independent: ranges of them are handled concurrently in two passes, the
  // first listing each patch's unknowns and counting its coupling entries, the second
  // writing the triples straight to their final place (no list grows while threads run).
  const int64_t nchunks = std::max<int64_t>(1, std::min<int64_t>(256, H.nv / 1024));
  std::vector<std::vector<int32_t>> cdof(nchunks);
  H.pptr.assign(H.nv + 1, 0);
  H.pvv_ptr.assign(H.nv + 1, 0);
  // the triples (a, b, CSR position) coupling the sorted unknowns dl of one patch, in the
  // order of the rows of dl and, within a row, of its columns
  auto couplings = [&](const int32_t* dl, int32_t n, int32_t* out) {
    int32_t cnt = 0;
    for (int32_t la = 0; la < n; ++la) {
      int32_t p = H.ptr[dl[la]];
      const int32_t pe = H.ptr[dl[la] + 1];
      int32_t lb = 0;
      while (p < pe && lb < n) {  // both sorted: one merge
        const int32_t c = H.col[p];
        if (c < dl[lb]) ++p;
        else if (c > dl[lb]) ++lb;
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
  auto chunk_lo = [&](int64_t k) { return H.nv * k / nchunks; };
  parallel_ranges(nchunks, [&](int64_t k0, int64_t k1) {
    std::vector<int32_t> dl;
    CellDofs d;
    for (int64_t k = k0; k < k1; ++k)
      for (int64_t v = chunk_lo(k); v < chunk_lo(k + 1); ++v) {
        dl.clear();
        for (int32_t p = L.node_cell_ptr[v]; p < L.node_cell_ptr[v + 1]; ++p) {
          cell_dofs(H, L.node_cell[p], d);
          for (int c = 0; c < 2; ++c)
            for (int a = 0; a < 6; ++a)
              if (d.u[c][a] >= 0) dl.push_back((int32_t)d.u[c][a]);
          for (int e = 0; e < 3; ++e)
            if (d.e[e] >= 0) dl.push_back((int32_t)d.e[e]);
        }
        dl.push_back((int32_t)(H.off_p + v));
        if (H.gidx[v] >= 0) dl.push_back((int32_t)(H.off_g + H.gidx[v]));
        std::sort(dl.begin(), dl.end());
        dl.erase(std::unique(dl.begin(), dl.end()), dl.end());
        cdof[k].insert(cdof[k].end(), dl.begin(), dl.end());
        H.pptr[v + 1] = (int32_t)dl.size();
        H.pvv_ptr[v + 1] = couplings(dl.data(), (int32_t)dl.size(), nullptr);
      }
  }, 1);
  for (int64_t v = 0; v < H.nv; ++v) {
    H.pptr[v + 1] += H.pptr[v];
    if ((int64_t)H.pvv_ptr[v] + H.pvv_ptr[v + 1] > INT32_MAX)
      throw std::runtime_error("MHD patches: more than 2^31 coupling entries on one level");
    H.pvv_ptr[v + 1] += H.pvv_ptr[v];
  }
  H.pdof.clear();
  H.pdof.reserve(H.pptr[H.nv]);
  for (const auto& c : cdof) H.pdof.insert(H.pdof.end(), c.begin(), c.end());
  H.pvv.assign((size_t)H.pvv_ptr[H.nv] * 3, 0);
  parallel_ranges(H.nv, [&](int64_t v0, int64_t v1) {
    for (int64_t v = v0; v < v1; ++v)
      couplings(&H.pdof[H.pptr[v]], H.pptr[v + 1] - H.pptr[v], &H.pvv[(size_t)H.pvv_ptr[v] * 3]);
  });
}

std::string mhd_transfer(const MhdHost& C, MhdHost& F, const int64_t* parent) {
  const HostLevel &LC = C.L, &LF = F.L;
  std::vector<std::vector<std::pair<int32_t, double>>> rows(F.ns);
  // velocity: P2 interpolation on each component
  for (int64_t i = 0; i < F.nfree; ++i)
    for (int32_t p = LF.pu_ptr[i]; p < LF.pu_ptr[i + 1]; ++p)
      for (int k = 0; k < 2; ++k) rows[k * F.nfree + i].push_back({(int32_t)(k * C.nfree + LF.pu_col[p]), LF.pu_val[p]});
  // field: a fine degree of freedom is the line integral of the coarse field along the
  // fine edge, the midpoint value times the edge vector (the tangential component of a
  // lowest-order Nedelec function is linear along a segment)
  CellNed N;
  for (int64_t i = 0; i < F.nB; ++i) {
    const int64_t ef = F.efree[i];
    const int64_t a = LF.edges[2 * ef], b = LF.edges[2 * ef + 1];
    const int64_t node = LF.nv + ef;
    if (LF.node_cell_ptr[node + 1] == LF.node_cell_ptr[node]) return "an edge without cells";
    const int64_t pc = parent[LF.node_cell[LF.node_cell_ptr[node]]];
    double mid[2], t[2], lam[3];
    for (int k = 0; k < 2; ++k) {
      mid[k] = 0.5 * (LF.xyz[a * 2 + k] + LF.xyz[b * 2 + k]);
      t[k] = LF.xyz[b * 2 + k] - LF.xyz[a * 2 + k];
    }
    fe_barycentric(LC, pc, mid, lam);
    for (int k = 0; k < 3; ++k)
      if (lam[k] < -1e-9) return "fine edge outside its parent cell: levels are not nested";
    cell_nedelec(LC, pc, N);
    for (int e = 0; e < 3; ++e) {
      const int32_t ce = C.eidx[N.edge[e]];
      if (ce < 0) continue;
      double val = 0;
      for (int v = 0; v < 3; ++v) val += lam[v] * (N.alpha[e][v][0] * t[0] + N.alpha[e][v][1] * t[1]);
      if (std::fabs(val) > 1e-14) rows[F.off_B + i].push_back({(int32_t)(C.off_B + ce), val});
    }
  }
  // pressure and multiplier: P1 interpolation (the multiplier's restricted to interior
  // vertices on both levels)
  for (int64_t v = 0; v < F.nv; ++v)
    for (int32_t p = LF.pp_ptr[v]; p < LF.pp_ptr[v + 1]; ++p) {
      const int64_t cv = LF.pp_col[p];
      rows[F.off_p + v].push_back({(int32_t)(C.off_p + cv), LF.pp_val[p]});
      if (F.gidx[v] >= 0 && C.gidx[cv] >= 0)
        rows[F.off_g + F.gidx[v]].push_back({(int32_t)(C.off_g + C.gidx[cv]), LF.pp_val[p]});
    }
  F.P_ptr.assign(F.ns + 1, 0);
  F.P_col.clear();
  F.P_val.clear();
  for (int64_t r = 0; r < F.ns; ++r) {
    std::sort(rows[r].begin(), rows[r].end());
    for (const auto& e : rows[r]) {
      F.P_col.push_back(e.first);
      F.P_val.push_back(e.second);
    }
    F.P_ptr[r + 1] = (int32_t)F.P_col.size();
  }
  return "";
}

void mhd_coarsen_state(const MhdHost& C, const MhdHost& F, const double* wf, const double* bf,
                       std::vector<double>& wc, std::vector<double>& bc) {
  const HostLevel &LC = C.L, &LF = F.L;
  const std::vector<int64_t>& c2f = LF.coarse_node_to_fine_vertex;
  wc.assign(LC.nn * 2, 0.0);
  for (int64_t n = 0; n < LC.nn; ++n)
    for (int k = 0; k < 2; ++k) wc[n * 2 + k] = wf[c2f[n] * 2 + k];
  // line integral over a coarse edge = the sum over its two fine halves, each traversed
  // from the coarse edge's smaller to its larger vertex
  bc.assign(LC.ne, 0.0);
  for (int64_t e = 0; e < LC.ne; ++e) {
    const int64_t fa = c2f[LC.edges[2 * e]], fb = c2f[LC.edges[2 * e + 1]], fm = c2f[LC.nv + e];
    double tot = 0;
    for (const auto& h : {std::make_pair(fa, fm), std::make_pair(fm, fb)}) {
      const int64_t fe = find_edge(LF, h.first, h.second);
      if (fe < 0) throw std::runtime_error("coarse edge halves are not fine edges");
      tot += (h.first < h.second ? 1.0 : -1.0) * bf[fe];
    }
    bc[e] = tot;
  }
}

void mhd_coarse_matrix(const MhdHost& H, int r, const double* A, double dt, std::vector<double>& J,
                       double* max_abs) {
  const int64_t N = H.ns * r;
  J.assign((size_t)N * N, 0.0);
  double mx = 0;
  for (int64_t q = 0; q < H.ns; ++q)
    for (int32_t p = H.ptr[q]; p < H.ptr[q + 1]; ++p) {
      const int64_t c = H.col[p];
      for (int s = 0; s < r; ++s)
        for (int t = 0; t < r; ++t) {
          const double v = (s == t ? H.mval[p] : 0.0) + dt * A[s * r + t] * H.sval[p];
          J[(size_t)(c * r + t) * N + (q * r + s)] += v;
        }
    }
  for (double v : J) mx = std::max(mx, std::fabs(v));
  for (int s = 0; s < r; ++s) {
    const int64_t q = H.off_p * r + s;
    for (int64_t i = 0; i < N; ++i) {
      J[(size_t)q * N + i] = 0.0;
      J[(size_t)i * N + q] = 0.0;
    }
    J[(size_t)q * N + q] = 1.0;
  }
  *max_abs = mx;
}

}  // namespace irk
