// C ABI of libirkmg (include/irk_mg.h): argument validation, setup orchestration, the
// multi-launch V-cycle (Sec. 4.1-4.2, 5.1) and the restarted FGMRES driver (Sec. 4).
// Host code only sequences kernels; all vector arithmetic runs on the GPU.
#include "../../include/irk_mg.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

#include "irk_internal.h"

using namespace irk;

namespace {

thread_local std::string g_err;

irk_status fail(irk_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(e_ == hipErrorOutOfMemory ? IRK_ENOMEM : IRK_EHIP,                    \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                   \
  } while (0)

#define CHK(expr)                       \
  do {                                  \
    irk_status s_ = (expr);             \
    if (s_ != IRK_OK) return s_;        \
  } while (0)

// IRK_MG_POISON_ALLOC=1 in the environment fills every allocation of a handle with the
// byte 0xFF (a NaN in FP64 and FP32) before first use, so that a kernel reading a
// workspace entry it never wrote shows up as a non-finite result instead of passing
// on whatever the allocator happened to return.
bool poison_allocations() {
  const char* v = std::getenv("IRK_MG_POISON_ALLOC");
  return v && *v && std::strcmp(v, "0") != 0;
}

template <typename T>
irk_status dalloc(Handle* h, T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc((void**)p, n * sizeof(T));
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? IRK_ENOMEM : IRK_EHIP,
                "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed: " + hipGetErrorName(e));
  h->allocations.push_back(*p);
  if (poison_allocations()) HIPCHK(hipMemset(*p, 0xFF, n * sizeof(T)));
  return IRK_OK;
}

template <typename T, typename S>
irk_status upload(Handle* h, T** p, const std::vector<S>& v, hipStream_t s) {
  CHK(dalloc(h, p, v.size()));
  if (v.empty()) return IRK_OK;
  std::vector<T> tmp(v.begin(), v.end());
  HIPCHK(hipMemcpyAsync(*p, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return IRK_OK;
}

template <typename T>
DevOps<T>& ops_of(DevLevel& L);
template <>
DevOps<double>& ops_of<double>(DevLevel& L) { return L.d64; }
template <>
DevOps<float>& ops_of<float>(DevLevel& L) { return L.d32; }

template <typename T>
irk_status upload_ops(Handle* h, HostLevel& H, DevLevel& D, DevOps<T>& o, const std::vector<double>& W,
                      hipStream_t s) {
  CHK(upload(h, &o.s_M, H.s_M, s));
  CHK(upload(h, &o.s_L, H.s_L, s));
  CHK(upload(h, &o.s_Lt, H.s_Lt, s));
  CHK(upload(h, &o.b_val, H.b_val, s));
  CHK(upload(h, &o.bt_val, H.bt_val, s));
  CHK(upload(h, &o.W, W, s));
  CHK(upload(h, &o.u_M, irk::sell_values(H.sell_s, H.s_M, 1), s));
  CHK(upload(h, &o.u_L, irk::sell_values(H.sell_s, H.s_L, 1), s));
  CHK(upload(h, &o.u_Lt, irk::sell_values(H.sell_s, H.s_Lt, 1), s));
  CHK(upload(h, &o.u_B, irk::sell_values(H.sell_b, H.b_val, H.dim), s));
  CHK(upload(h, &o.p_Bt, irk::sell_values(H.sell_bt, H.bt_val, H.dim), s));
  if (!H.pu_val.empty()) {
    CHK(upload(h, &o.pu_val, H.pu_val, s));
    CHK(upload(h, &o.put_val, H.put_val, s));
    CHK(upload(h, &o.pp_val, H.pp_val, s));
    CHK(upload(h, &o.ppt_val, H.ppt_val, s));
  }
  (void)D;
  return IRK_OK;
}

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

void transpose_host(int64_t nrows, int64_t ncols, const std::vector<int32_t>& ptr, const std::vector<int32_t>& col,
                    const std::vector<double>& val, std::vector<int32_t>& tptr, std::vector<int32_t>& tcol,
                    std::vector<double>& tval) {
  tptr.assign(ncols + 1, 0);
  for (int32_t cc : col) tptr[cc + 1]++;
  for (int64_t i = 0; i < ncols; ++i) tptr[i + 1] += tptr[i];
  tcol.resize(col.size());
  tval.resize(val.size());
  std::vector<int32_t> fp(tptr.begin(), tptr.end() - 1);
  for (int64_t i = 0; i < nrows; ++i)
    for (int32_t p = ptr[i]; p < ptr[i + 1]; ++p) {
      const int32_t q = fp[col[p]]++;
      tcol[q] = (int32_t)i;
      tval[q] = val[p];
    }
}

// ------------------------------------------------------------------- measurement
int prof_begin(Handle* h, int kernel, int level, hipStream_t s) {
  if (!h->prof) return -1;
  // mode 1: finest-level patch apply only; 2: every kernel of the finest level; 3: all
  if (h->prof_mode < 3 && level != h->nlevels - 1) return -1;
  if (h->prof_mode == 1 && kernel != 0) return -1;
  if (h->prof_used == h->prof_pool.size()) {
    Handle::ProfEv e;
    if (hipEventCreate(&e.a) != hipSuccess || hipEventCreate(&e.b) != hipSuccess) return -1;
    h->prof_pool.push_back(e);
  }
  Handle::ProfEv& e = h->prof_pool[h->prof_used];
  e.kernel = kernel;
  e.level = level;
  if (hipEventRecord(e.a, s) != hipSuccess) return -1;
  return (int)h->prof_used++;
}

void prof_end(Handle* h, int idx, hipStream_t s) {
  if (idx >= 0) (void)hipEventRecord(h->prof_pool[idx].b, s);
}

// ----------------------------------------------------------------------- V-cycle
// Level operators of the cycle: the handle's stage operator, or, while the Newton
// Jacobian preconditioner is active (FP64 only, forward only), the per-stage Newton
// Jacobian of the level and its dense patch inverses.
template <typename T>
hipError_t lev_residual(Handle* h, int l, const DevOps<T>& o, const double* A, const T* b, const T* x, T* y,
                        hipStream_t s) {
  if constexpr (std::is_same<T, double>::value) {
    if (h->nw_active) return k::residual_newton(h->dev[l], h->nw_sl[l], h->A, h->dt, b, x, y, s);
  }
  return k::residual<T>(h->dev[l], o, A, h->dt, b, x, y, s);
}

// the level with the Newton Jacobian's dense patch inverses in place of its own factors
DevLevel newton_view(const Handle* h, int l) {
  DevLevel V = h->dev[l];
  V.pform = 0;
  V.inv = h->nw_inv[l];
  V.p_ld = h->nw_ld[l];
  V.p_inv_off = h->nw_off[l];
  return V;
}

template <typename T>
hipError_t lev_patch(Handle* h, int l, const DevOps<T>& o, const T* r, T* Y, int tr, hipStream_t s) {
  if constexpr (std::is_same<T, double>::value) {
    if (h->nw_active) return k::patch_apply<double>(newton_view(h, l), o, r, Y, tr, s);
  }
  return k::patch_apply<T>(h->dev[l], o, r, Y, tr, s);
}

template <typename T>
irk_status smooth(Handle* h, int l, int nsweeps, bool zero_start, bool tr, hipStream_t s) {
  DevLevel& L = h->dev[l];
  DevOps<T>& o = ops_of<T>(L);
  T* b = (T*)L.b;
  T* x = (T*)L.x;
  T* res = (T*)L.res;
  T* Y = (T*)L.Y;
  const double* A = tr ? h->At : h->A;
  if (nsweeps == 0) {
    if (zero_start) {
      if constexpr (std::is_same<T, double>::value) HIPCHK(k::fill(x, L.N, 0.0, s));
      else HIPCHK(k::fillf(x, L.N, 0.f, s));
    }
    return IRK_OK;
  }
  DevOps<T> ot = o;
  if (tr) {
    ot.s_L = o.s_Lt;
    ot.u_L = o.u_Lt;
  }
  if (h->smoother == 2) {
    // GMRES relaxation (Sec. 4.2, 5.4): one cycle of nsweeps left-preconditioned GMRES
    // steps with the additive operator from the current x (zero when zero_start),
    // classical Gram--Schmidt, least squares on the device
    const int m = nsweeps;
    T* V = (T*)L.grv;
    const int64_t N = L.N;
    double* gr = h->gr;
    const int mode = tr ? 2 : 0;  // assign W S r (forward) or S (W r) (transposed)
    const T* r = b;
    if (!zero_start) {
      const int p0 = prof_begin(h, 1, l, s);
      HIPCHK(lev_residual<T>(h, l, ot, A, b, x, res, s));
      prof_end(h, p0, s);
      r = res;
    }
    int p1 = prof_begin(h, 0, l, s);
    HIPCHK(lev_patch<T>(h, l, o, r, Y, tr ? 1 : 0, s));
    prof_end(h, p1, s);
    int p2 = prof_begin(h, 2, l, s);
    HIPCHK(k::gather_update<T>(L, o, Y, V, (T)1, mode, s));
    prof_end(h, p2, s);
    // beta = ||v_0|| (an orthogonalisation against no vectors), v_0 /= beta
    HIPCHK(k::gr_orth_norm<T>(V, V, N, -1, N, gr, h->grpart, gr + k::kGrNorm, s));
    HIPCHK(k::gr_scale<T>(V, N, gr + k::kGrNorm, s));
    for (int j = 0; j < m; ++j) {
      T* Vj = V + (int64_t)j * N;
      T* Vn = V + (int64_t)(j + 1) * N;
      const int p3 = prof_begin(h, 1, l, s);
      HIPCHK(lev_residual<T>(h, l, ot, A, nullptr, Vj, res, s));
      prof_end(h, p3, s);
      p1 = prof_begin(h, 0, l, s);
      HIPCHK(lev_patch<T>(h, l, o, res, Y, tr ? 1 : 0, s));
      prof_end(h, p1, s);
      p2 = prof_begin(h, 2, l, s);
      HIPCHK(k::gather_update<T>(L, o, Y, Vn, (T)1, mode, s));
      prof_end(h, p2, s);
      double* hcol = gr + k::kGrH + (int64_t)j * (kMaxGr + 1);
      HIPCHK(k::gr_dots<T>(V, N, j + 1, Vn, N, h->grpart, hcol, s));
      HIPCHK(k::gr_orth_norm<T>(Vn, V, N, j, N, hcol, h->grpart, hcol + j + 1, s));
      HIPCHK(k::gr_scale<T>(Vn, N, hcol + j + 1, s));
    }
    HIPCHK(k::gr_solve(gr, m, s));
    HIPCHK(k::gr_update<T>(x, V, N, m, N, gr + k::kGrY, zero_start ? 1 : 0, s));
    return IRK_OK;
  }
  if (h->smoother == 1) {
    // Chebyshev relaxation (Sec. 5.1) on [cheb_lo, cheb_hi]: theta, delta, sigma and the
    // rho recurrence of the Chebyshev semi-iteration, coefficients formed in FP64
    const double theta = 0.5 * (h->cheb_hi + h->cheb_lo), delta = 0.5 * (h->cheb_hi - h->cheb_lo);
    const double sigma = theta / delta;
    double rho = 0.0;
    T* d = (T*)L.dch;
    for (int it = 0; it < nsweeps; ++it) {
      const bool xzero = zero_start && it == 0;
      const T* r = b;
      if (!xzero) {
        const int p0 = prof_begin(h, 1, l, s);
        HIPCHK(lev_residual<T>(h, l, ot, A, b, x, res, s));
        prof_end(h, p0, s);
        r = res;
      }
      const int p1 = prof_begin(h, 0, l, s);
      HIPCHK(lev_patch<T>(h, l, o, r, Y, tr ? 1 : 0, s));
      prof_end(h, p1, s);
      double c1 = 0.0, c2;
      if (it == 0) {
        rho = 1.0 / sigma;
        c2 = 1.0 / theta;
      } else {
        const double rn = 1.0 / (2.0 * sigma - rho);
        c1 = rn * rho;
        c2 = 2.0 * rn / delta;
        rho = rn;
      }
      const int p2 = prof_begin(h, 2, l, s);
      HIPCHK(k::gather_cheb<T>(L, o, Y, (T)c1, (T)c2, it == 0 ? 1 : 0, xzero ? 1 : 0, tr ? 1 : 0, d, x, s));
      prof_end(h, p2, s);
    }
    return IRK_OK;
  }
  for (int it = 0; it < nsweeps; ++it) {
    const bool first = zero_start && it == 0;
    const T* r = b;
    if (!first) {
      const int p0 = prof_begin(h, 1, l, s);
      HIPCHK(lev_residual<T>(h, l, ot, A, b, x, res, s));
      prof_end(h, p0, s);
      r = res;
    }
    const int p1 = prof_begin(h, 0, l, s);
    HIPCHK(lev_patch<T>(h, l, o, r, Y, tr ? 1 : 0, s));
    prof_end(h, p1, s);
    const int mode = (tr ? 2 : 0) + (first ? 0 : 1);
    const int p2 = prof_begin(h, 2, l, s);
    HIPCHK(k::gather_update<T>(L, o, Y, x, (T)h->omega, mode, s));
    prof_end(h, p2, s);
  }
  return IRK_OK;
}

// One V-cycle (Sec. 4.1) by its legs: descend_T pre-smooths level l and restricts its
// residual into the right-hand side of level l-1; coarse_T solves on level 0; ascend_T
// prolongs the correction into level l and post-smooths.
template <typename T>
irk_status descend_T(Handle* h, int l, bool tr, hipStream_t s) {
  DevLevel& L = h->dev[l];
  DevOps<T> o = ops_of<T>(L);
  if (tr) {
    o.s_L = o.s_Lt;
    o.u_L = o.u_Lt;
  }
  CHK(smooth<T>(h, l, tr ? h->post : h->pre, true, tr, s));
  const int p0 = prof_begin(h, 1, l, s);
  HIPCHK(lev_residual<T>(h, l, o, tr ? h->At : h->A, (const T*)L.b, (const T*)L.x, (T*)L.res, s));
  prof_end(h, p0, s);
  HIPCHK(k::restrict_<T>(L, h->dev[l - 1], ops_of<T>(L), (const T*)L.res, (T*)h->dev[l - 1].b, s));
  return IRK_OK;
}

template <typename T>
irk_status coarse_T(Handle* h, bool tr, hipStream_t s, const int64_t* pins) {
  DevLevel& L = h->dev[0];
  HIPCHK((k::cast<T, double>((const T*)L.b, h->cb, L.N, s)));
  if (h->nw_active)
    HIPCHK(k::coarse_solve(h->nw_cinv, h->nw_cmat, L.N, h->cb, h->cx, pins, h->r, h->cpart, s));
  else
    HIPCHK(k::coarse_solve(tr ? h->coarse_invT : h->coarse_inv, tr ? h->coarse_matT : h->coarse_mat, L.N, h->cb,
                           h->cx, pins, h->r, h->cpart, s));
  HIPCHK((k::cast<double, T>(h->cx, (T*)L.x, L.N, s)));
  return IRK_OK;
}

template <typename T>
irk_status ascend_T(Handle* h, int l, bool tr, hipStream_t s) {
  DevLevel& L = h->dev[l];
  HIPCHK(k::prolong_add<T>(L, h->dev[l - 1], ops_of<T>(L), (const T*)h->dev[l - 1].x, (T*)L.x, s));
  CHK(smooth<T>(h, l, tr ? h->pre : h->post, false, tr, s));
  return IRK_OK;
}

// the cycle restricted to levels 0..lt, entered with the right-hand side of level lt
template <typename T>
irk_status subcycle_T(Handle* h, int lt, bool tr, hipStream_t s, const int64_t* pins) {
  for (int l = lt; l >= 1; --l) CHK(descend_T<T>(h, l, tr, s));
  CHK(coarse_T<T>(h, tr, s, pins));
  for (int l = 1; l <= lt; ++l) CHK(ascend_T<T>(h, l, tr, s));
  return IRK_OK;
}

template <typename T>
irk_status vcycle_T(Handle* h, bool tr, hipStream_t s, const int64_t* pins) {
  if (h->nw_active && tr) return fail(IRK_EINVAL, "the Newton Jacobian V-cycle has no transpose");
  return subcycle_T<T>(h, h->nlevels - 1, tr, s, pins);
}


irk_status precondition(irk_mg* h, const double* v, double* z, bool tr, hipStream_t s) {
  DevLevel& L = h->dev[h->nlevels - 1];
  if (tr) {
    HIPCHK((k::cast<double, double>(v, h->kw, L.N, s)));
    HIPCHK(k::project_pressure(L, h->kw, h->partials, s));
    v = h->kw;
  }
  if (h->precision == 0) {
    HIPCHK((k::cast<double, double>(v, (double*)L.b, L.N, s)));
    CHK(vcycle_T<double>(h, tr, s, h->pins));
    HIPCHK((k::cast<double, double>((const double*)L.x, z, L.N, s)));
  } else {
    HIPCHK((k::cast<double, float>(v, (float*)L.b, L.N, s)));
    CHK(vcycle_T<float>(h, tr, s, h->pins));
    HIPCHK((k::cast<float, double>((const float*)L.x, z, L.N, s)));
  }
  if (!tr) HIPCHK(k::project_pressure(L, z, h->partials, s));
  return IRK_OK;
}

// ------------------------------------------------------- Navier--Stokes (Sec. 3.2)
// Element data, the wind and the Newton work vectors of the finest level, on first use.
irk_status ns_init(irk_mg* h, hipStream_t s) {
  if (h->ns_ready) return IRK_OK;
  HostLevel& H = h->host[h->nlevels - 1];
  DevLevel& L = h->dev[h->nlevels - 1];
  std::vector<double> geo;
  std::vector<int32_t> cn, cf, ip, inc;
  ns_cell_data(H, geo, cn, cf, ip, inc);
  CHK(upload(h, &h->ns_geo, geo, s));
  CHK(upload(h, &h->ns_cells, cn, s));
  CHK(upload(h, &h->ns_cell_free, cf, s));
  CHK(upload(h, &h->ns_inc_ptr, ip, s));
  CHK(upload(h, &h->ns_inc, inc, s));
  CHK(upload(h, &h->ns_free, H.free_of_node, s));
  if (!h->wind_fine.empty()) CHK(upload(h, &h->ns_w, h->wind_fine, s));
  const int d = h->dim, r = h->r, nl = d == 2 ? 6 : 10;
  CHK(dalloc(h, &h->ns_U, (size_t)H.nn * d * r));
  CHK(dalloc(h, &h->ns_elem, (size_t)H.nc * nl * d * r));
  CHK(dalloc(h, &h->ns_k, (size_t)L.N));
  CHK(dalloc(h, &h->ns_kt, (size_t)L.N));
  CHK(dalloc(h, &h->ns_F, (size_t)L.N));
  CHK(dalloc(h, &h->ns_G, (size_t)L.N));
  HIPCHK(hipStreamSynchronize(s));
  // algorithmic bytes of one Jacobian-mode launch: cell nodes, their free indices and the
  // geometry, stage values and wind once per node, the direction once, element vectors
  // written; the gather reads
  // the incidences and element entries of free nodes and updates y
  const double nc = (double)H.nc, nn = (double)H.nn, nf = (double)H.nfree;
  L.alg_bytes[3] = 2 * nc * nl * 4 + nc * ((d + 1) * d + 1) * 8 + nn * d * r * 8 +
                   (h->ns_w ? nn * d * 8 : 0) + nf * d * r * 8 + nc * nl * d * r * 8;
  L.alg_bytes[4] = nf * 4 + (double)inc.size() * 4 + (double)inc.size() * d * r * 8 + 2 * nf * d * r * 8;
  h->ns_ready = true;
  return IRK_OK;
}

// ns_U from the state (free velocities, stage-block layout), k (internal) and the stage
// boundary data (r x nnodes x dim, or NULL: zero)
irk_status ns_stage_values(irk_mg* h, const double* state, const double* k_int, const double* g_st, hipStream_t s) {
  HostLevel& H = h->host[h->nlevels - 1];
  k::NsCoef c;
  for (int i = 0; i < h->r * h->r; ++i) c.a[i] = h->dt * h->A[i];
  HIPCHK(k::ns_stage_values(H.nn, h->dim, h->r, H.nfree, h->ns_free, state, k_int, c, g_st, h->ns_U, s));
  return IRK_OK;
}

// Operators of the Newton Jacobian V-cycle (Sec. 3.2) at the stage velocities in ns_U
// (finest level): the stage velocities carried to every coarser level by injection (its
// P2 nodes are nodes of the next finer level), the per-stage velocity blocks
// K + N'(U_i) assembled on the GPU for every level (and copied to the sliced order of the
// residual), the stage-coupled patch matrices
// factorised on the GPU in the dense form, and the coarse operator inverted on the
// GPU.  Allocates on first use; FP64 handles only.
irk_status nw_build(irk_mg* h, hipStream_t s) {
  if (h->precision != 0) return fail(IRK_EINVAL, "the Newton Jacobian V-cycle needs an FP64 handle");
  const int nl = h->nlevels, top = nl - 1, d = h->dim, r = h->r, dd = d * d;
  constexpr int VEC = 2;  // dense inverse columns padded to 16-byte words
  if (!h->nw_ready) {
    h->nw_vals.assign(nl, nullptr);
    h->nw_sl.assign(nl, nullptr);
    h->nw_src.assign(nl, nullptr);
    h->nw_inv.assign(nl, nullptr);
    h->nw_ld.assign(nl, nullptr);
    h->nw_off.assign(nl, nullptr);
    for (int l = 0; l < nl; ++l) {
      const HostLevel& H = h->host[l];
      CHK(dalloc(h, &h->nw_vals[l], H.s_col.size() * r * dd));
      std::vector<int32_t> src(H.sell_s.src.size());
      for (size_t e = 0; e < src.size(); ++e) src[e] = (int32_t)H.sell_s.src[e];
      CHK(upload(h, &h->nw_src[l], src, s));
      CHK(dalloc(h, &h->nw_sl[l], src.size() * r * dd));
      if (l == 0) continue;
      const DevLevel& D = h->dev[l];
      std::vector<int32_t> ld(D.npatch);
      std::vector<int64_t> off(D.npatch);
      int64_t io = 0;
      for (int64_t p = 0; p < D.npatch; ++p) {
        const int n = r * (d * (H.pn_ptr[p + 1] - H.pn_ptr[p]) + 1);
        ld[p] = (n + VEC - 1) / VEC * VEC;
        off[p] = io;
        io += (int64_t)ld[p] * n;
      }
      CHK(upload(h, &h->nw_ld[l], ld, s));
      CHK(upload(h, &h->nw_off[l], off, s));
      CHK(dalloc(h, &h->nw_inv[l], (size_t)io));
    }
    const int64_t N0 = h->dev[0].N;
    CHK(dalloc(h, &h->nw_cinv, (size_t)N0 * N0));
    CHK(dalloc(h, &h->nw_cmat, (size_t)N0 * N0));
    CHK(dalloc(h, &h->nw_ctmp, (size_t)N0 * N0));
    CHK(dalloc(h, &h->nw_colk, (size_t)N0));
    CHK(dalloc(h, &h->nw_swp, (size_t)N0));
    // element data for the assembly of the blocks on the device
    for (auto* v : {&h->nwa_geo, &h->nwa_K1, &h->nwa_U}) v->assign(nl, nullptr);
    for (auto* v : {&h->nwa_cn, &h->nwa_cf, &h->nwa_inc_ptr, &h->nwa_inc, &h->nwa_c2f}) v->assign(nl, nullptr);
    for (int l = 0; l < nl; ++l) {
      const HostLevel& H = h->host[l];
      std::vector<double> geo;
      std::vector<int32_t> cn, cf, ip, inc;
      irk::ns_cell_data(H, geo, cn, cf, ip, inc);
      CHK(upload(h, &h->nwa_geo[l], geo, s));
      CHK(upload(h, &h->nwa_cn[l], cn, s));
      CHK(upload(h, &h->nwa_cf[l], cf, s));
      CHK(upload(h, &h->nwa_inc_ptr[l], ip, s));
      CHK(upload(h, &h->nwa_inc[l], inc, s));
      CHK(upload(h, &h->nwa_K1[l], H.s_K1, s));
      if (l < top) {
        CHK(dalloc(h, &h->nwa_U[l], (size_t)H.nn * d * r));
        CHK(upload(h, &h->nwa_c2f[l], h->host[l + 1].coarse_node_to_fine_vertex, s));
      }
    }
    const int nloc = d == 2 ? 6 : 10;
    const double* C = irk::fe_p2_conv_tensor(d);
    CHK(upload(h, &h->nwa_C, std::vector<double>(C, C + nloc * nloc * nloc * (d + 1)), s));
    h->nw_ready = true;
  }
  // stage velocities on every level: the finest level's at its P2 nodes (ns_U), injected
  // at the coarser levels' P2 nodes, which are vertices of the next finer level
  h->nwa_U[top] = h->ns_U;
  for (int l = top - 1; l >= 0; --l)
    HIPCHK(k::inject_nodal(h->host[l].nn, d * r, h->nwa_c2f[l], h->nwa_U[l + 1], h->nwa_U[l], s));
  HIPCHK(hipMemsetAsync(h->flag, 0, sizeof(int), s));
  std::vector<double> Jc;
  double scale = 0;
  for (int l = 0; l < nl; ++l) {
    const HostLevel& H = h->host[l];
    HIPCHK(k::newton_blocks(d, r, H.nfree, h->dev[l].s_ptr, h->dev[l].s_col, h->nwa_K1[l], h->nu, h->nwa_geo[l],
                            h->nwa_cn[l], h->nwa_cf[l], h->nwa_inc_ptr[l], h->nwa_inc[l], h->nwa_C, h->nwa_U[l],
                            h->nw_vals[l], s));
    HIPCHK(k::sell_blocks((int64_t)H.sell_s.src.size(), r * dd, h->nw_src[l], h->nw_vals[l], h->nw_sl[l], s));
    if (l == 0) {
      // the dense coarse operator is built on the host from the coarsest level's blocks
      std::vector<double> vals(H.s_col.size() * r * dd);
      HIPCHK(hipMemcpyAsync(vals.data(), h->nw_vals[0], vals.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      irk::coarse_matrix_newton(H, r, h->A, h->dt, vals.data(), Jc, &scale);
    }
    if (l >= 1) {
      DevLevel V = newton_view(h, l);
      if (V.max_nloc > 1024)
        return fail(IRK_EINVAL, "patch of " + std::to_string(V.max_nloc) + " unknowns exceeds the limit of 1024");
      HIPCHK(k::patch_factor_range<double>(V, V.d64, r, h->A, h->dt, V.p_ld, V.p_inv_off,
                                           reinterpret_cast<double*>(V.inv), 0, V.npatch, 0, V.max_nloc, h->flag, s,
                                           h->nw_vals[l]));
    }
  }
  // coarse: the column-major operator (transpose of the row-major one) and its inverse
  // (Gauss--Jordan in place on the row-major operator, then transposed)
  const int64_t N0 = h->dev[0].N;
  HIPCHK(hipMemcpyAsync(h->nw_ctmp, Jc.data(), Jc.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(k::transpose(h->nw_ctmp, h->nw_cmat, N0, s));
  HIPCHK(k::dense_inverse(h->nw_ctmp, N0, std::max(1e-300, 1e-14 * scale), h->nw_colk, h->nw_swp, h->flag, s));
  HIPCHK(k::transpose(h->nw_ctmp, h->nw_cinv, N0, s));
  int fl = 0;
  HIPCHK(hipMemcpyAsync(&fl, h->flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (fl) return fail(IRK_ESINGULAR, "zero pivot in a patch or the coarse operator of the Newton Jacobian");
  return IRK_OK;
}

// y += scale * (mode 0: c(U - w, U); mode 1: c(U - w, z) + c(z, U), z_i = sum_j a_ij x_j)
irk_status ns_correction(irk_mg* h, int mode, const double* x, double* y, double scale, hipStream_t s) {
  HostLevel& H = h->host[h->nlevels - 1];
  const int lf = h->nlevels - 1;
  k::NsElemArgs a;
  a.nc = H.nc;
  a.r = h->r;
  a.mode = mode;
  a.cell_nodes = h->ns_cells;
  a.geo = h->ns_geo;
  a.cell_free = h->ns_cell_free;
  a.U = h->ns_U;
  a.w = h->ns_w;
  a.x = x;
  for (int i = 0; i < h->r * h->r; ++i) a.a[i] = h->A[i];
  a.elem = h->ns_elem;
  const int p0 = prof_begin(h, 3, lf, s);
  HIPCHK(k::ns_element(h->dim, a, s));
  prof_end(h, p0, s);
  const int p1 = prof_begin(h, 4, lf, s);
  HIPCHK(k::ns_gather(H.nfree, h->dim, h->r, h->ns_inc_ptr, h->ns_inc, h->ns_elem, scale, y, s));
  prof_end(h, p1, s);
  return IRK_OK;
}

irk_status apply_J(irk_mg* h, const double* x, double* y, bool tr, const double* F, hipStream_t s) {
  DevLevel& L = h->dev[h->nlevels - 1];
  DevOps<double> o = L.d64;
  if (tr) {
    o.s_L = o.s_Lt;
    o.u_L = o.u_Lt;
  }
  HIPCHK(k::residual<double>(L, o, tr ? h->At : h->A, h->dt, F, x, y, s));
  // Newton mode: the operator is the Jacobian of the Navier--Stokes stage equations
  if (h->ns_jac && !tr) CHK(ns_correction(h, 1, x, y, F ? -h->dt : h->dt, s));
  return IRK_OK;
}

irk_status ensure_krylov(irk_mg* h, int restart) {
  if (h->krylov_cap >= restart) return IRK_OK;
  const int64_t N = h->dev[h->nlevels - 1].N;
  if (h->kv) {
    (void)hipFree(h->kv);
    (void)hipFree(h->kz);
    h->allocations.erase(std::remove(h->allocations.begin(), h->allocations.end(), (void*)h->kv), h->allocations.end());
    h->allocations.erase(std::remove(h->allocations.begin(), h->allocations.end(), (void*)h->kz), h->allocations.end());
    h->kv = h->kz = nullptr;
    h->krylov_cap = 0;  // no usable basis until the new one is in place
  }
  CHK(dalloc(h, &h->kv, (size_t)(restart + 1) * N));
  CHK(dalloc(h, &h->kz, (size_t)restart * N));
  h->krylov_cap = restart;
  return IRK_OK;
}

// Start the next FGMRES iteration's V-cycle before the host has read the Hessenberg column
// when the predicted residual estimate stays above this many tolerances.
constexpr double kSpecMargin = 20.0;

// FGMRES on the finest level in the internal layout: solves J x = kF starting from the x
// held in kx and leaves the solution in kx (and, when k_abi is given, in k_abi).  The
// caller records ev0 and fills kF, kx; the Krylov workspace must hold `restart` vectors.
irk_status fgmres_int(irk_mg* h, double* k_abi, double rtol, int maxit, int restart, irk_solve_info* info,
                      bool tr, hipStream_t s) {
  DevLevel& L = h->dev[h->nlevels - 1];
  const int64_t N = L.N;
  double* H = nullptr;
  std::vector<double> Hm((size_t)(restart + 1) * restart), cs(restart), sn(restart), g(restart + 1),
      y(restart);
  double* hcol = h->hpin;          // pinned: restart + 2 values
  double* ycoef = h->hpin + 1032;  // pinned: restart values
  auto host_scalar = [&](double* dev, double* out) -> irk_status {
    HIPCHK(hipMemcpyAsync(out, dev, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return IRK_OK;
  };
  (void)H;
  CHK(apply_J(h, h->kx, h->kr, tr, h->kF, s));
  HIPCHK(k::dot(h->kr, h->kr, N, h->partials, h->scal, s, 1));
  double beta0;
  CHK(host_scalar(h->scal, &beta0));
  int hist_n = 0;
  auto push_hist = [&](double v) {
    if (info && info->history && hist_n < info->history_cap) info->history[hist_n++] = v;
  };
  push_hist(beta0);
  if (!std::isfinite(beta0)) return fail(IRK_ENAN, "non-finite initial residual");
  int its = 0;
  bool converged = beta0 == 0.0;
  float ms_v = 0.f;
  while (!converged && its < maxit) {
    CHK(apply_J(h, h->kx, h->kr, tr, h->kF, s));
    HIPCHK(k::dot(h->kr, h->kr, N, h->partials, h->scal, s, 1));
    double beta;
    CHK(host_scalar(h->scal, &beta));
    if (!std::isfinite(beta)) return fail(IRK_ENAN, "non-finite residual");
    if (beta <= rtol * beta0) {
      converged = true;
      break;
    }
    HIPCHK(k::axpby(h->kv, h->kr, N, 1.0 / beta, 0.0, s));
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jend = 0;
    bool z_ready = false;  // z_j was started by the previous iteration
    double res_prev = -1.0, res_cur = beta;
    for (int j = 0; j < restart; ++j) {
      double* vj = h->kv + (size_t)j * N;
      double* zj = h->kz + (size_t)j * N;
      double* vn = h->kv + (size_t)(j + 1) * N;
      hipEvent_t ea = (j & 1) ? h->ev4 : h->ev2, eb = (j & 1) ? h->ev5 : h->ev3;
      if (!z_ready) {
        HIPCHK(hipEventRecord(ea, s));
        CHK(precondition(h, vj, zj, tr, s));
        HIPCHK(hipEventRecord(eb, s));
      }
      CHK(apply_J(h, zj, vn, tr, nullptr, s));
      HIPCHK(k::mgs_arnoldi(vn, h->kv, N, j, h->partials, h->hbuf, s));
      HIPCHK(hipMemcpyAsync(hcol, h->hbuf, (j + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipEventRecord(h->evh, s));
      // The next V-cycle needs only v_{j+1}, which is on the device: start it before the host
      // reads column j when the residual estimates (the last contraction applied once more)
      // put the end of this cycle more than kSpecMargin tolerances away.  A wrong guess costs
      // one unused V-cycle; the iterates are the same either way.
      bool spec = false;
      if (j + 1 < restart && its + 1 < maxit && res_prev > 0.0) {
        const double rho = std::min(1.0, res_cur / res_prev);
        spec = res_cur * rho > kSpecMargin * rtol * beta0;
      }
      if (spec) {
        hipEvent_t na = (j & 1) ? h->ev2 : h->ev4, nb = (j & 1) ? h->ev3 : h->ev5;
        HIPCHK(hipEventRecord(na, s));
        CHK(precondition(h, vn, h->kz + (size_t)(j + 1) * N, tr, s));
        HIPCHK(hipEventRecord(nb, s));
      }
      HIPCHK(hipEventSynchronize(h->evh));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, ea, eb));
      ms_v += ms;
      z_ready = spec;
      for (int i = 0; i <= j + 1; ++i) {
        if (!std::isfinite(hcol[i])) {
          if (spec) (void)hipStreamSynchronize(s);
          return fail(IRK_ENAN, "non-finite value in the Arnoldi process");
        }
        Hm[i * restart + j] = hcol[i];
      }
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * Hm[i * restart + j] + sn[i] * Hm[(i + 1) * restart + j];
        Hm[(i + 1) * restart + j] = -sn[i] * Hm[i * restart + j] + cs[i] * Hm[(i + 1) * restart + j];
        Hm[i * restart + j] = t;
      }
      const double den = std::hypot(Hm[j * restart + j], Hm[(j + 1) * restart + j]);
      cs[j] = Hm[j * restart + j] / den;
      sn[j] = Hm[(j + 1) * restart + j] / den;
      Hm[j * restart + j] = den;
      Hm[(j + 1) * restart + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++its;
      jend = j + 1;
      push_hist(std::fabs(g[j + 1]));
      res_prev = res_cur;
      res_cur = std::fabs(g[j + 1]);
      if (std::fabs(g[j + 1]) <= rtol * beta0 || its >= maxit) break;
    }
    for (int i = jend - 1; i >= 0; --i) {
      double acc = g[i];
      for (int m = i + 1; m < jend; ++m) acc -= Hm[i * restart + m] * y[m];
      y[i] = acc / Hm[i * restart + i];
    }
    // x += Z y in one pass (the coefficients through the pinned buffer, which the host next
    // writes after later synchronisations; the device column buffer is free until the next
    // cycle's Arnoldi step)
    std::copy(y.begin(), y.begin() + jend, ycoef);
    HIPCHK(hipMemcpyAsync(h->hbuf, ycoef, (size_t)jend * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(k::update_sum(h->kx, h->kz, N, h->hbuf, jend, s));
    if (std::fabs(g[jend]) <= rtol * beta0) converged = true;
  }
  HIPCHK(k::project_pressure(L, h->kx, h->partials, s));
  CHK(apply_J(h, h->kx, h->kr, tr, h->kF, s));
  HIPCHK(k::dot(h->kr, h->kr, N, h->partials, h->scal, s, 1));
  double fin;
  CHK(host_scalar(h->scal, &fin));
  if (k_abi) HIPCHK(k::to_abi<double>(L, h->kx, k_abi, s));
  HIPCHK(hipEventRecord(h->ev1, s));
  HIPCHK(hipEventSynchronize(h->ev1));
  float ms_t = 0;
  HIPCHK(hipEventElapsedTime(&ms_t, h->ev0, h->ev1));
  if (info) {
    info->iterations = its;
    info->converged = converged ? 1 : 0;
    info->rel_residual = beta0 > 0 ? fin / beta0 : 0.0;
    info->ms_vcycle = ms_v;
    info->ms_total = ms_t;
  }
  if (!std::isfinite(fin)) return fail(IRK_ENAN, "non-finite final residual");
  if (!converged) {
    g_err = "FGMRES reached maxit";
    return IRK_ENOCONV;
  }
  return IRK_OK;
}

irk_status fgmres(irk_mg* h, const double* F_abi, double* k_abi, double rtol, int maxit, int restart,
                  irk_solve_info* info, bool tr, hipStream_t s) {
  if (!F_abi || !k_abi) return fail(IRK_EINVAL, "null vector");
  if (!(rtol > 0) || maxit < 1 || restart < 1 || restart > 1000)
    return fail(IRK_EINVAL, "rtol must be > 0, maxit >= 1, 1 <= restart <= 1000");
  CHK(ensure_krylov(h, restart));
  DevLevel& L = h->dev[h->nlevels - 1];
  HIPCHK(hipEventRecord(h->ev0, s));
  HIPCHK(k::to_internal<double>(L, F_abi, h->kF, s));
  HIPCHK(k::to_internal<double>(L, k_abi, h->kx, s));
  return fgmres_int(h, k_abi, rtol, maxit, restart, info, tr, s);
}

irk_status check_handle(irk_mg* h) {
  if (!h) return fail(IRK_EINVAL, "null handle");
  return IRK_OK;
}

irk_status check_level(irk_mg* h, int& level) {
  CHK(check_handle(h));
  if (level < 0) level = h->nlevels - 1;
  if (level >= h->nlevels) return fail(IRK_EINVAL, "level out of range");
  return IRK_OK;
}

template <typename T>
irk_status level_sweep_T(irk_mg* h, int level, int transpose, const double* F, double* kv,
                                hipStream_t s) {
  DevLevel& L = h->dev[level];
  HIPCHK(k::to_internal<T>(L, F, (T*)L.b, s));
  HIPCHK(k::to_internal<T>(L, kv, (T*)L.x, s));
  CHK(smooth<T>(h, level, 1, false, transpose != 0, s));
  HIPCHK(k::to_abi<T>(L, (const T*)L.x, kv, s));
  return IRK_OK;
}

// Arnoldi on the relaxation's preconditioned operator W S J_l of level l (classical
// Gram--Schmidt, the GMRES relaxation's kernels) in caller-provided device storage: V
// holds steps + 1 vectors of the level, dH (steps + 1)^2 doubles, part the reduction
// partial sums; the Hessenberg matrix ((steps + 1) x steps, column-major) is copied to
// Hh on the host and the stream synchronised.
template <typename T>
irk_status ritz_ws_T(irk_mg* h, int level, int steps, const double* v0, T* V, double* dH, double* part,
                     double* Hh, hipStream_t s) {
  DevLevel& L = h->dev[level];
  DevOps<T>& o = ops_of<T>(L);
  const int64_t N = L.N;
  const int ld = steps + 1;
  hipError_t e = k::fill(dH, (int64_t)ld * (steps + 1), 0.0, s);
  double* nrm0 = dH + (size_t)ld * steps;  // spare column: the start vector's norm
  if (e == hipSuccess) e = k::to_internal<T>(L, v0, V, s);
  if (e == hipSuccess) e = k::gr_orth_norm<T>(V, V, N, -1, N, dH, part, nrm0, s);
  if (e == hipSuccess) e = k::gr_scale<T>(V, N, nrm0, s);
  for (int j = 0; j < steps && e == hipSuccess; ++j) {
    T* Vj = V + (int64_t)j * N;
    T* Vn = V + (int64_t)(j + 1) * N;
    double* hcol = dH + (size_t)j * ld;
    e = k::residual<T>(L, o, h->A, h->dt, nullptr, Vj, (T*)L.res, s);
    if (e == hipSuccess) e = k::patch_apply<T>(L, o, (const T*)L.res, (T*)L.Y, 0, s);
    if (e == hipSuccess) e = k::gather_update<T>(L, o, (const T*)L.Y, Vn, (T)1, 0, s);
    for (int c0 = 0; c0 <= j && e == hipSuccess; c0 += kMaxGr + 1)
      e = k::gr_dots<T>(V + (int64_t)c0 * N, N, std::min(kMaxGr + 1, j + 1 - c0), Vn, N, part, hcol + c0, s);
    if (e == hipSuccess) e = k::gr_orth_norm<T>(Vn, V, N, j, N, hcol, part, hcol + j + 1, s);
    if (e == hipSuccess) e = k::gr_scale<T>(Vn, N, hcol + j + 1, s);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(Hh, dH, (size_t)ld * steps * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(IRK_EHIP, std::string("Arnoldi estimate: ") + hipGetErrorString(e));
  return IRK_OK;
}

template <typename T>
irk_status ritz_T(irk_mg* h, int level, int steps, const double* v0, double* Hh, hipStream_t s) {
  const int64_t N = h->dev[level].N;
  T* V = nullptr;
  double *dH = nullptr, *part = nullptr;
  auto release = [&]() {
    (void)hipStreamSynchronize(s);
    if (V) (void)hipFree(V);
    if (dH) (void)hipFree(dH);
    if (part) (void)hipFree(part);
  };
  if (hipMalloc(&V, (size_t)(steps + 1) * N * sizeof(T)) != hipSuccess ||
      hipMalloc(&dH, (size_t)(steps + 1) * (steps + 1) * sizeof(double)) != hipSuccess ||
      hipMalloc(&part, irk::ritz_partials_bytes()) != hipSuccess) {
    release();
    return fail(IRK_ENOMEM, "device allocation of the Arnoldi basis failed");
  }
  const irk_status st = ritz_ws_T<T>(h, level, steps, v0, V, dH, part, Hh, s);
  release();
  return st;
}

}  // namespace

size_t irk::ritz_partials_bytes() { return (size_t)k::kGrBlocks * (kMaxGr + 1) * sizeof(double); }

irk_status irk::ritz_check(irk_mg* h, int& level, int steps, const double* v0, const double* ritz_re,
                           const double* ritz_im) {
  CHK(check_level(h, level));
  if (level < 1) return fail(IRK_EINVAL, "the coarsest level has no relaxation");
  if (steps < 1 || steps > 64) return fail(IRK_EINVAL, "steps must be in 1..64");
  if (!v0 || !ritz_re || !ritz_im) return fail(IRK_EINVAL, "null argument");
  return IRK_OK;
}

irk_status irk::ritz_into(irk_mg* h, int level, int steps, const double* v0, void* V, double* dH, double* part,
                          double* Hh, hipStream_t s) {
  if (h->precision == 0) return ritz_ws_T<double>(h, level, steps, v0, (double*)V, dH, part, Hh, s);
  return ritz_ws_T<float>(h, level, steps, v0, (float*)V, dH, part, Hh, s);
}

// Ritz values from the Hessenberg matrix Hh ((steps + 1) x steps, column-major); an
// invariant Krylov space (zero subdiagonal entry) ends the estimate early.
irk_status irk::ritz_finish(int steps, const double* Hh, double* H, double* ritz_re, double* ritz_im, int* nritz,
                            std::complex<double>* work, int* iwork) {
  const int ld = steps + 1;
  int m = steps;
  for (int j = 0; j < steps; ++j)
    if (!(Hh[(size_t)j * ld + j + 1] != 0.0)) {
      m = j + 1;
      break;
    }
  if (H) std::memcpy(H, Hh, (size_t)ld * steps * sizeof(double));
  for (int j = 0; j < steps; ++j) ritz_re[j] = ritz_im[j] = 0.0;
  if (!irk::hessenberg_eigs_ws(m, Hh, ld, ritz_re, ritz_im, work, iwork))
    return fail(IRK_ENOCONV, "Hessenberg QR iteration did not converge");
  if (nritz) *nritz = m;
  return IRK_OK;
}


int irk::ensure_krylov_ws(irk_mg* h, int restart) { return ensure_krylov(h, restart); }
void irk::set_error(const std::string& msg) { g_err = msg; }
irk_status irk::fail_with(irk_status code, const std::string& msg) { return fail(code, msg); }
bool irk::poison_requested() { return poison_allocations(); }

// =========================================================================== ABI
extern "C" {

void irk_mg_default_opts(irk_mg_opts* o) {
  if (!o) return;
  o->pre = 2;
  o->post = 2;
  o->omega = 0.5;
  o->weighting = 1;
  o->precision = 0;
  o->patch_form = 2;
  o->smoother = 0;
  o->cheb_lo = 2.0;
  o->cheb_hi = 8.0;
}

irk_status irk_tableau_builtin(int family, int r, double* A, double* b, double* c) {
  if (!A || !b || !c) return fail(IRK_EINVAL, "null output");
  const double s6 = std::sqrt(6.0), s3 = std::sqrt(3.0), s15 = std::sqrt(15.0);
  std::vector<double> a, bb, cc;
  if (family == 0 && r == 1) {
    a = {1.0};
    bb = {1.0};
    cc = {1.0};
  } else if (family == 0 && r == 2) {
    a = {5.0 / 12, -1.0 / 12, 3.0 / 4, 1.0 / 4};
    bb = {3.0 / 4, 1.0 / 4};
    cc = {1.0 / 3, 1.0};
  } else if (family == 0 && r == 3) {
    a = {(88 - 7 * s6) / 360,      (296 - 169 * s6) / 1800, (-2 + 3 * s6) / 225,
         (296 + 169 * s6) / 1800,  (88 + 7 * s6) / 360,     (-2 - 3 * s6) / 225,
         (16 - s6) / 36,           (16 + s6) / 36,          1.0 / 9};
    bb = {(16 - s6) / 36, (16 + s6) / 36, 1.0 / 9};
    cc = {(4 - s6) / 10, (4 + s6) / 10, 1.0};
  } else if (family == 1 && r == 1) {
    a = {0.5};
    bb = {1.0};
    cc = {0.5};
  } else if (family == 1 && r == 2) {
    a = {0.25, 0.25 - s3 / 6, 0.25 + s3 / 6, 0.25};
    bb = {0.5, 0.5};
    cc = {0.5 - s3 / 6, 0.5 + s3 / 6};
  } else if (family == 1 && r == 3) {
    a = {5.0 / 36,            2.0 / 9 - s15 / 15, 5.0 / 36 - s15 / 30,
         5.0 / 36 + s15 / 24, 2.0 / 9,            5.0 / 36 - s15 / 24,
         5.0 / 36 + s15 / 30, 2.0 / 9 + s15 / 15, 5.0 / 36};
    bb = {5.0 / 18, 4.0 / 9, 5.0 / 18};
    cc = {0.5 - s15 / 10, 0.5, 0.5 + s15 / 10};
  } else if (family == 2 && r == 2) {
    a = {0.5, -0.5, 0.5, 0.5};
    bb = {0.5, 0.5};
    cc = {0.0, 1.0};
  } else if (family == 2 && r == 3) {
    a = {1.0 / 6, -1.0 / 3, 1.0 / 6, 1.0 / 6, 5.0 / 12, -1.0 / 12, 1.0 / 6, 2.0 / 3, 1.0 / 6};
    bb = {1.0 / 6, 2.0 / 3, 1.0 / 6};
    cc = {0.0, 0.5, 1.0};
  } else {
    return fail(IRK_EINVAL, "unknown tableau (family, r)");
  }
  std::copy(a.begin(), a.end(), A);
  std::copy(bb.begin(), bb.end(), b);
  std::copy(cc.begin(), cc.end(), c);
  return IRK_OK;
}

const char* irk_last_error(void) { return g_err.c_str(); }

irk_status irk_mesh_p2_nodes(const irk_mesh_level* m, int64_t* nnodes, double* xyz) {
  if (!m || !nnodes || !m->xyz || !m->cells) return fail(IRK_EINVAL, "null argument");
  if ((m->dim != 2 && m->dim != 3) || m->nverts < m->dim + 1 || m->ncells < 1)
    return fail(IRK_EINVAL, "bad mesh sizes");
  for (int64_t i = 0; i < m->ncells * (m->dim + 1); ++i)
    if (m->cells[i] < 0 || m->cells[i] >= m->nverts) return fail(IRK_EINVAL, "vertex index out of range");
  HostLevel H;
  try {
    build_topology(H, m->dim, m->nverts, m->ncells, m->xyz, m->cells);
  } catch (const std::bad_alloc&) {
    return fail(IRK_ENOMEM, "host allocation failed");
  }
  *nnodes = H.nn;
  if (xyz) {
    const int d = H.dim;
    for (int64_t n = 0; n < H.nn; ++n) {
      if (n < H.nv) {
        for (int i = 0; i < d; ++i) xyz[n * d + i] = H.xyz[n * d + i];
      } else {
        const int64_t a = H.edges[(n - H.nv) * 2], b = H.edges[(n - H.nv) * 2 + 1];
        for (int i = 0; i < d; ++i) xyz[n * d + i] = 0.5 * (H.xyz[a * d + i] + H.xyz[b * d + i]);
      }
    }
  }
  return IRK_OK;
}

irk_status irk_mg_profile(irk_mg* h, int enable) {
  CHK(check_handle(h));
  if (enable < 0 || enable > 3) return fail(IRK_EINVAL, "profile mode must be 0..3");
  h->prof = enable != 0;
  if (enable) {
    h->prof_mode = enable;
    h->prof_used = 0;
  }
  return IRK_OK;
}

irk_status irk_mg_kernel_stats(irk_mg* h, int kernel, int level, irk_kernel_stats* out) {
  CHK(check_level(h, level));
  if (!out || kernel < 0 || kernel > 4) return fail(IRK_EINVAL, "kernel must be 0..4 and out non-NULL");
  out->launches = 0;
  out->ms_total = 0;
  out->bytes_per_launch = h->dev[level].alg_bytes[kernel];
  for (size_t i = 0; i < h->prof_used; ++i) {
    Handle::ProfEv& e = h->prof_pool[i];
    if (e.kernel != kernel || e.level != level) continue;
    HIPCHK(hipEventSynchronize(e.b));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e.a, e.b));
    out->launches++;
    out->ms_total += ms;
  }
  return IRK_OK;
}

void irk_mg_destroy(irk_mg* h) {
  if (!h) return;
  for (auto& e : h->prof_pool) {
    if (e.a) (void)hipEventDestroy(e.a);
    if (e.b) (void)hipEventDestroy(e.b);
  }
  for (void* p : h->allocations) (void)hipFree(p);
  for (hipEvent_t e : {h->ev0, h->ev1, h->ev2, h->ev3, h->ev4, h->ev5, h->evh})
    if (e) (void)hipEventDestroy(e);
  if (h->hpin) (void)hipHostFree(h->hpin);
  delete h;
}

}  // extern "C"

template <typename T>
const irk::StageBasis<T>& basis(const DevLevel& D);
template <>
const irk::StageBasis<double>& basis<double>(const DevLevel& D) { return D.sb64; }
template <>
const irk::StageBasis<float>& basis<float>(const DevLevel& D) { return D.sb32; }

// Factorise every patch of level l.  Dense form: one launch over all patches.  Factored
// form: for each eigen-block, the (1- or 2-stage) block matrix of a chunk of patches is
// inverted into a temporary buffer by the same kernels and copied into the factored
// layout; chunks keep the temporary under 2 GiB.
template <typename T>
static irk_status factor_level(irk_mg* h, int l, const DevOps<T>& ops, double dt, int* dfail, hipStream_t s) {
  DevLevel& D = h->dev[l];
  const HostLevel& H = h->host[l];
  const int r = h->r, dim = h->dim;
  if (D.pform == 0) {
    HIPCHK(k::patch_factor_range<T>(D, ops, r, h->A, dt, D.p_ld, D.p_inv_off, reinterpret_cast<T*>(D.inv), 0,
                                    D.npatch, 0, D.max_nloc, dfail, s));
    return IRK_OK;
  }
  if (D.pform == 3) {
    // factorise in the factored layout (temporary), then keep the wrapped diagonals
    T* full = nullptr;
    hipError_t e = hipMalloc(&full, (size_t)std::max<int64_t>(D.full_elems, 1) * sizeof(T));
    if (e != hipSuccess) return fail(IRK_ENOMEM, "device allocation of the factorisation workspace failed");
    void* sym = D.inv;
    int64_t* sym_off = D.p_inv_off;
    D.inv = full;
    D.p_inv_off = D.p_full_off;
    D.pform = 1;
    const irk_status st = factor_level<T>(h, l, ops, dt, dfail, s);
    D.pform = 3;
    D.inv = sym;
    D.p_inv_off = sym_off;
    if (st == IRK_OK) e = k::pack_sym<T>(D, D.p_full_off, full, s);
    hipStreamSynchronize(s);
    hipFree(full);
    if (st != IRK_OK) return st;
    if (e != hipSuccess) return fail(IRK_EHIP, std::string("symmetric patch form: ") + hipGetErrorString(e));
    return IRK_OK;
  }
  const irk::StageEig& E = h->eig;
  const int VEC = 16 / (int)sizeof(T);
  const int64_t np = D.npatch;
  int max_ns = 0;
  for (int64_t p = 0; p < np; ++p) max_ns = std::max(max_ns, dim * (H.pn_ptr[p + 1] - H.pn_ptr[p]) + 1);
  const int64_t budget = ((int64_t)2 << 30) / (int64_t)sizeof(T);
  for (int b = 0; b < E.nblk; ++b) {
    const int m = E.type[b];
    if (m == 2 && 2.0 * max_ns * max_ns * sizeof(T) + 2.0 * max_ns * sizeof(T) + max_ns * 4.0 + 64 <= 160 * 1024) {
      // complex pair small enough for LDS: inverted as the n_s x n_s complex matrix
      HIPCHK(k::patch_factor_cplx<T>(D, ops, dt * E.Tb[b][0], -dt * E.Tb[b][1], b, max_ns, dfail, s));
      continue;
    }
    std::vector<int32_t> tld(np);
    std::vector<int64_t> toff(np + 1, 0);
    for (int64_t p = 0; p < np; ++p) {
      const int n = m * (dim * (H.pn_ptr[p + 1] - H.pn_ptr[p]) + 1);
      tld[p] = (n + VEC - 1) / VEC * VEC;
      toff[p + 1] = toff[p] + (int64_t)tld[p] * n;
    }
    int32_t* d_tld = nullptr;
    int64_t* d_toff = nullptr;
    T* tmp = nullptr;
    int64_t chunk_max = 0;
    {
      int64_t p0 = 0;
      while (p0 < np) {
        int64_t p1 = p0 + 1;
        while (p1 < np && toff[p1 + 1] - toff[p0] <= budget) ++p1;
        chunk_max = std::max(chunk_max, toff[p1] - toff[p0]);
        p0 = p1;
      }
    }
    auto release = [&]() {
      hipStreamSynchronize(s);
      if (d_tld) hipFree(d_tld);
      if (d_toff) hipFree(d_toff);
      if (tmp) hipFree(tmp);
    };
    if (hipMalloc(&d_tld, np * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&d_toff, (np + 1) * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&tmp, (size_t)chunk_max * sizeof(T)) != hipSuccess) {
      release();
      return fail(IRK_ENOMEM, "device allocation of the factorisation workspace failed");
    }
    hipError_t e = hipMemcpyAsync(d_tld, tld.data(), np * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_toff, toff.data(), (np + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s);
    double coef[4];
    for (int i = 0; i < m * m; ++i) coef[i] = E.Tb[b][i];
    int64_t p0 = 0;
    while (e == hipSuccess && p0 < np) {
      int64_t p1 = p0 + 1;
      while (p1 < np && toff[p1 + 1] - toff[p0] <= budget) ++p1;
      e = k::patch_factor_range<T>(D, ops, m, coef, dt, d_tld, d_toff, tmp, p0, p1, toff[p0], m * max_ns, dfail, s);
      if (e == hipSuccess) e = k::eig_extract<T>(D, basis<T>(D), b, d_tld, d_toff, toff[p0], tmp, p0, p1, s);
      p0 = p1;
    }
    release();
    if (e != hipSuccess) return fail(IRK_EHIP, std::string("patch factorisation: ") + hipGetErrorString(e));
  }
  return IRK_OK;
}

extern "C" {

// Patch counts below which a non-finest level takes the factored form where the automatic
// choice is the symmetric one (8 x 8 to 32 x 32 on the 256 x 256 hierarchy: 12.6 against
// 15.4 us per patch apply at 8 x 8, 16.5 against 19.7 at 32 x 32; 31.9 against 25.7 at 64 x 64)
constexpr int64_t kFactoredBelowPatches = 2048;

static irk_status setup_impl(const irk_mesh_level* lv, int nlevels, const irk_tableau* tab, double dt,
                             double nu, const double* wind, const irk_mg_opts* opt, hipStream_t s,
                             irk_mg* h) {
  const int dim = lv[0].dim;
  const int r = tab->r;
  h->dim = dim;
  h->r = r;
  h->nlevels = nlevels;
  h->dt = dt;
  h->nu = nu;
  irk_mg_opts o;
  irk_mg_default_opts(&o);
  if (opt) o = *opt;
  h->pre = o.pre;
  h->post = o.post;
  h->omega = o.omega;
  h->weighting = o.weighting;
  h->precision = o.precision;
  h->smoother = o.smoother;
  h->cheb_lo = o.cheb_lo;
  h->cheb_hi = o.cheb_hi;
  for (int i = 0; i < r; ++i) {
    h->b[i] = tab->b[i];
    h->c[i] = tab->c[i];
    for (int j = 0; j < r; ++j) {
      h->A[i * r + j] = tab->A[i * r + j];
      h->At[i * r + j] = tab->A[j * r + i];
    }
  }
  {
    // (dt A)^{-1} for the boundary stage derivatives (Gauss--Jordan, partial pivoting)
    const int n = r;
    double M[kMaxStages][2 * kMaxStages];
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < 2 * n; ++j) M[i][j] = j < n ? dt * h->A[i * n + j] : (j - n == i ? 1.0 : 0.0);
    bool ok = true;
    for (int k = 0; k < n && ok; ++k) {
      int piv = k;
      for (int i = k + 1; i < n; ++i)
        if (std::fabs(M[i][k]) > std::fabs(M[piv][k])) piv = i;
      if (!(std::fabs(M[piv][k]) > 0)) {
        ok = false;
        break;
      }
      for (int j = 0; j < 2 * n; ++j) std::swap(M[k][j], M[piv][j]);
      const double ip = 1.0 / M[k][k];
      for (int j = 0; j < 2 * n; ++j) M[k][j] *= ip;
      for (int i = 0; i < n; ++i)
        if (i != k) {
          const double f = M[i][k];
          for (int j = 0; j < 2 * n; ++j) M[i][j] -= f * M[k][j];
        }
    }
    h->A_invertible = ok;
    if (ok)
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) h->Ainv_dt[i * n + j] = M[i][n + j];
  }
  {
    std::string why;
    irk::StageEig eig;
    const bool ok = o.patch_form != 0 && irk::stage_eigenbasis(h->A, r, eig, &why);
    if ((o.patch_form == 1 || o.patch_form == 3) && !ok)
      return fail(IRK_EINVAL, "factored patch form unavailable: " + why);
    if (o.patch_form == 3 && wind)
      return fail(IRK_EINVAL, "the symmetric patch form needs a symmetric spatial operator (no wind)");
    int form = ok && (o.patch_form == 1 || o.patch_form == 3 || r >= 2) ? 1 : 0;
    // a symmetric spatial operator (Stokes) makes every eigen-block inverse symmetric
    if (form == 1 && !wind && o.patch_form != 1) form = 3;
    h->patch_form = form;
    h->patch_form_req = o.patch_form;
    if (h->patch_form) h->eig = eig;
  }
  // ---- host: topology, transfers, assembly, patches
  h->host.resize(nlevels);
  for (int l = 0; l < nlevels; ++l)
    build_topology(h->host[l], dim, lv[l].nverts, lv[l].ncells, lv[l].xyz, lv[l].cells);
  for (int l = 1; l < nlevels; ++l) {
    std::string e = build_transfer(h->host[l - 1], h->host[l], lv[l].parent);
    if (!e.empty()) return fail(IRK_EINVAL, "level " + std::to_string(l) + ": " + e);
  }
  std::vector<std::vector<double>> winds(nlevels);
  if (wind) {
    const HostLevel& Ft = h->host[nlevels - 1];
    winds[nlevels - 1].assign(wind, wind + Ft.nn * dim);
    for (int l = nlevels - 2; l >= 0; --l) {
      const HostLevel& C = h->host[l];
      const HostLevel& F = h->host[l + 1];
      winds[l].resize(C.nn * dim);
      for (int64_t n = 0; n < C.nn; ++n)
        for (int i = 0; i < dim; ++i)
          winds[l][n * dim + i] = winds[l + 1][F.coarse_node_to_fine_vertex[n] * dim + i];
    }
    for (double w : winds[nlevels - 1])
      if (!std::isfinite(w)) return fail(IRK_EINVAL, "non-finite wind value");
    h->wind_fine = winds[nlevels - 1];
  }
  for (int l = 0; l < nlevels; ++l) {
    assemble_level(h->host[l], nu, wind ? &winds[l] : nullptr, l == nlevels - 1);
    if (l >= 1) build_patches(h->host[l]);
    HostLevel& H = h->host[l];
    H.sell_s = irk::build_sell(H.nfree, H.s_ptr, H.s_col);
    H.sell_b = irk::build_sell(H.nfree, H.b_ptr, H.b_col);
    H.sell_bt = irk::build_sell(H.nv, H.bt_ptr, H.bt_col);
  }
  // ---- device
  const int VEC = h->precision == 0 ? 2 : 4;
  h->dev.resize(nlevels);
  for (int l = 0; l < nlevels; ++l) {
    HostLevel& H = h->host[l];
    DevLevel& D = h->dev[l];
    D.dim = dim;
    D.r = r;
    D.nv = H.nv;
    D.nfree = H.nfree;
    D.offV = H.nfree * dim * r;
    D.N = D.offV + H.nv * r;
    CHK(upload(h, &D.s_ptr, H.s_ptr, s));
    CHK(upload(h, &D.s_col, H.s_col, s));
    CHK(upload(h, &D.b_ptr, H.b_ptr, s));
    CHK(upload(h, &D.b_col, H.b_col, s));
    CHK(upload(h, &D.bt_ptr, H.bt_ptr, s));
    CHK(upload(h, &D.bt_col, H.bt_col, s));
    D.nsl_u = H.sell_s.nslices;
    D.nsl_p = H.sell_bt.nslices;
    CHK(upload(h, &D.su_off, H.sell_s.off, s));
    CHK(upload(h, &D.su_w, H.sell_s.w, s));
    CHK(upload(h, &D.su_col, H.sell_s.col, s));
    CHK(upload(h, &D.sb_off, H.sell_b.off, s));
    CHK(upload(h, &D.sb_w, H.sell_b.w, s));
    CHK(upload(h, &D.sb_col, H.sell_b.col, s));
    CHK(upload(h, &D.sp_off, H.sell_bt.off, s));
    CHK(upload(h, &D.sp_w, H.sell_bt.w, s));
    CHK(upload(h, &D.sp_col, H.sell_bt.col, s));
    if (l >= 1) {
      CHK(upload(h, &D.pu_ptr, H.pu_ptr, s));
      CHK(upload(h, &D.pu_col, H.pu_col, s));
      CHK(upload(h, &D.put_ptr, H.put_ptr, s));
      CHK(upload(h, &D.put_col, H.put_col, s));
      CHK(upload(h, &D.pp_ptr, H.pp_ptr, s));
      CHK(upload(h, &D.pp_col, H.pp_col, s));
      CHK(upload(h, &D.ppt_ptr, H.ppt_ptr, s));
      CHK(upload(h, &D.ppt_col, H.ppt_col, s));
    }
    if (l == nlevels - 1) {
      CHK(upload(h, &D.mfa_ptr, H.mfa_ptr, s));
      CHK(upload(h, &D.mfa_col, H.mfa_col, s));
      CHK(upload(h, &D.mfa_val, H.mfa_val, s));
      {
        std::vector<int32_t> tp, tc;
        std::vector<double> tv;
        transpose_host(H.nfree, H.nn, H.mfa_ptr, H.mfa_col, H.mfa_val, tp, tc, tv);
        CHK(upload(h, &D.mfat_ptr, tp, s));
        CHK(upload(h, &D.mfat_col, tc, s));
        CHK(upload(h, &D.mfat_val, tv, s));
      }
      CHK(upload(h, &D.s_K1, H.s_K1, s));
      CHK(upload(h, &D.fb_ptr, H.fb_ptr, s));
      CHK(upload(h, &D.fb_col, H.fb_col, s));
      CHK(upload(h, &D.fb_m, H.fb_m, s));
      CHK(upload(h, &D.fb_l, H.fb_l, s));
      CHK(upload(h, &D.vb_ptr, H.vb_ptr, s));
      CHK(upload(h, &D.vb_col, H.vb_col, s));
      CHK(upload(h, &D.vb_val, H.vb_val, s));
      D.nnodes = H.nn;
    }
    // patches: sizes, offsets, local -> internal index, DOF -> slot lists, weights
    std::vector<double> W(D.N, 1.0);
    if (l >= 1) {
      const int64_t np = H.nv;
      D.npatch = np;
      std::vector<int32_t> nloc(np), ld(np), nnv(np), gidx, gptr(D.N + 1, 0), gslot;
      std::vector<int64_t> inv_off(np), slot_off(np);
      std::vector<int64_t> sym_off(np);
      int64_t io = 0, so = 0, sio = 0;
      // 128-byte lines: patch outputs written and symmetric factors read line by line
      const int64_t kLine = 128 / (h->precision == 0 ? 8 : 4);
      int maxn = 0, maxld = 0;
      D.pform = h->patch_form;
      // automatic form: below the finest level, levels of few patches use the factored
      // form, whose column stream has a shorter per-patch chain than the symmetric form's
      // diagonals; their factors are cache-resident, so the extra bytes cost nothing
      if (D.pform == 3 && h->patch_form_req == 2 && l < nlevels - 1 && np < kFactoredBelowPatches) D.pform = 1;
      if (D.pform == 3) {
        int maxns = 0;
        for (int64_t p = 0; p < np; ++p) maxns = std::max(maxns, dim * (H.pn_ptr[p + 1] - H.pn_ptr[p]) + 1);
        if (maxns > 256) {
          if (h->patch_form_req == 3)
            return fail(IRK_EINVAL, "the symmetric patch form needs patches of at most 256 unknowns per stage");
          D.pform = 1;
        }
      }
      for (int64_t p = 0; p < np; ++p) {
        const int nn = H.pn_ptr[p + 1] - H.pn_ptr[p];
        const int ns = dim * nn + 1;
        const int n = r * ns;
        nnv[p] = nn;
        nloc[p] = n;
        inv_off[p] = io;
        slot_off[p] = so;
        if (D.pform == 1 || D.pform == 3) {
          // factored: ns columns, each the concatenation of the eigen-blocks' rows
          int lc = 0;
          for (int b = 0; b < h->eig.nblk; ++b) lc += irk::eig_block_rows(h->eig.type[b], ns, VEC);
          ld[p] = lc;
          io += (int64_t)lc * ns;
          sym_off[p] = sio;
          for (int b = 0; b < h->eig.nblk; ++b) sio += irk::sym_block_values(h->eig.type[b], ns, VEC);
          sio = (sio + kLine - 1) / kLine * kLine;  // next patch on a whole cache line
        } else {
          ld[p] = (n + VEC - 1) / VEC * VEC;
          io += (int64_t)ld[p] * n;
        }
        so = (so + n + kLine - 1) / kLine * kLine;  // each patch's slots on whole cache lines
        maxn = std::max(maxn, n);
        maxld = std::max(maxld, ld[p]);
        for (int st = 0; st < r; ++st) {
          for (int c = 0; c < dim; ++c)
            for (int a = 0; a < nn; ++a)
              gidx.push_back((int32_t)(((int64_t)H.pn_node[H.pn_ptr[p] + a] * dim + c) * r + st));
          gidx.push_back((int32_t)(D.offV + p * r + st));
        }
        gidx.resize(so, -1);  // gidx is indexed by slot: padding entries, never read
      }
      D.inv_elems = D.pform == 3 ? sio : io;
      D.full_elems = io;
      D.slots = so;
      D.max_nloc = maxn;
      D.max_ld = maxld;
      if (D.pform == 1 || D.pform == 3) {
        const irk::StageEig& E = h->eig;
        for (auto* sbp : {&D.sb64}) {
          sbp->r = r;
          sbp->nblk = E.nblk;
          for (int b = 0; b < E.nblk; ++b) {
            sbp->type[b] = E.type[b];
            sbp->st0[b] = E.st0[b];
          }
          for (int i = 0; i < r * r; ++i) {
            sbp->W[i] = E.W[i];
            sbp->Winv[i] = E.Winv[i];
          }
        }
        D.sb32.r = r;
        D.sb32.nblk = E.nblk;
        for (int b = 0; b < E.nblk; ++b) {
          D.sb32.type[b] = E.type[b];
          D.sb32.st0[b] = E.st0[b];
        }
        for (int i = 0; i < r * r; ++i) {
          D.sb32.W[i] = (float)E.W[i];
          D.sb32.Winv[i] = (float)E.Winv[i];
        }
      }
      if (so > INT32_MAX || D.N > INT32_MAX) return fail(IRK_EINVAL, "problem too large for 32-bit patch indices");
      for (int32_t g : gidx)
        if (g >= 0) gptr[g + 1]++;
      for (int64_t g = 0; g < D.N; ++g) gptr[g + 1] += gptr[g];
      gslot.resize(so);
      std::vector<int32_t> fillp(gptr.begin(), gptr.end() - 1);
      // patch outputs are stored node-major within each patch (the patch kernels write
      // local index e to slot slot_off + node_major_slot(e)); the lists name those slots
      for (int64_t p = 0; p < np; ++p) {
        const int n = nloc[p], ns = n / r, nn = nnv[p];
        for (int e = 0; e < n; ++e) {
          const int st = e / ns, q = e - st * ns;
          const int slot = q < dim * nn ? ((q % nn) * dim + q / nn) * r + st : nn * dim * r + st;
          const int64_t g = gidx[slot_off[p] + e];
          gslot[fillp[g]++] = (int32_t)(slot_off[p] + slot);
        }
      }
      {
        irk::Sell G = irk::build_sell(D.N, gptr, gslot);
        for (size_t e = 0; e < G.col.size(); ++e)
          if (G.src[e] < 0) G.col[e] = (int32_t)so;  // the zero slot
        D.nsl_g = G.nslices;
        CHK(upload(h, &D.g_off, G.off, s));
        CHK(upload(h, &D.g_w, G.w, s));
        CHK(upload(h, &D.g_slot, G.col, s));
      }
      for (int64_t g = 0; g < D.N; ++g) {
        const int cnt = gptr[g + 1] - gptr[g];
        if (cnt == 0) return fail(IRK_EINVAL, "a DOF is covered by no patch");
        W[g] = h->weighting ? 1.0 / cnt : 1.0;
      }
      std::vector<int32_t> sched(np);
      std::iota(sched.begin(), sched.end(), 0);
      std::stable_sort(sched.begin(), sched.end(), [&](int32_t a, int32_t b) { return nloc[a] > nloc[b]; });
      CHK(upload(h, &D.p_nloc, nloc, s));
      CHK(upload(h, &D.p_ld, ld, s));
      CHK(upload(h, &D.p_nn, nnv, s));
      CHK(upload(h, &D.p_inv_off, D.pform == 3 ? sym_off : inv_off, s));
      if (D.pform == 3) CHK(upload(h, &D.p_full_off, inv_off, s));
      CHK(upload(h, &D.p_slot_off, slot_off, s));
      CHK(upload(h, &D.p_gidx, gidx, s));
      CHK(upload(h, &D.gat_ptr, gptr, s));
      CHK(upload(h, &D.gat_slot, gslot, s));
      CHK(upload(h, &D.sched, sched, s));
      CHK(upload(h, &D.pvv_ptr, H.pvv_ptr, s));
      CHK(upload(h, &D.pvv, H.pvv, s));
      CHK(upload(h, &D.pvp, H.pvp, s));
      CHK(upload(h, &D.pn_ptr, H.pn_ptr, s));
    }
    {
      const double es = h->precision == 0 ? 8.0 : 4.0;
      double sum_n = 0, sum_n2 = 0;
      if (l >= 1)
        for (int64_t p = 0; p < H.nv; ++p) {
          const double ns = dim * (double)(H.pn_ptr[p + 1] - H.pn_ptr[p]) + 1;
          sum_n += r * ns;
          // stored values read per application: (r ns)^2 dense, r ns^2 factored,
          // r ns (ns/2 + 1) symmetric factored
          sum_n2 += D.pform == 3 ? r * ns * (double)irk::sym_diags((int)ns)
                                 : (D.pform == 1 ? r * ns * ns : r * r * ns * ns);
        }
      D.alg_bytes[0] = es * (sum_n2 + (double)D.N + sum_n);
      D.alg_bytes[1] = (double)H.s_col.size() * (4 + 2 * es) +
                       2.0 * (double)H.b_col.size() * (4 + dim * es) + 3.0 * es * (double)D.N;
      D.alg_bytes[2] = sum_n * (es + 4) + 3.0 * es * (double)D.N;
    }
    CHK(upload_ops<double>(h, H, D, D.d64, W, s));
    if (h->precision == 1) CHK(upload_ops<float>(h, H, D, D.d32, W, s));
    const size_t es = h->precision == 0 ? sizeof(double) : sizeof(float);
    double* tmp;
    for (void** buf : {&D.b, &D.x, &D.res}) {
      CHK(dalloc(h, &tmp, (D.N * es + 7) / 8));
      *buf = tmp;
    }
    if (l >= 1) {
      // one extra slot at the end, zeroed here and never written: the sliced gather's
      // padding entries point at it
      CHK(dalloc(h, &tmp, ((D.slots + 1) * es + 7) / 8));
      HIPCHK(hipMemsetAsync(tmp, 0, (D.slots + 1) * es, s));
      D.Y = tmp;
      if (h->smoother == 1) {
        CHK(dalloc(h, &tmp, (D.N * es + 7) / 8));
        D.dch = tmp;
      }
      if (h->smoother == 2) {
        const int64_t nv = std::max(std::max(h->pre, h->post), 1) + 1;
        CHK(dalloc(h, &tmp, (nv * D.N * es + 7) / 8));
        D.grv = tmp;
      }
      CHK(dalloc(h, &tmp, (D.inv_elems * es + 7) / 8));
      D.inv = tmp;
    }
  }
  if (h->smoother == 2) {
    CHK(dalloc(h, &h->gr, (size_t)k::kGrSize));
    CHK(dalloc(h, &h->grpart, (size_t)k::kGrBlocks * (kMaxGr + 1)));
  }
  // ---- patch factorisation on the GPU
  int* dfail;
  CHK(dalloc(h, &dfail, 1));
  h->flag = dfail;
  HIPCHK(hipMemsetAsync(dfail, 0, sizeof(int), s));
  for (int l = 1; l < nlevels; ++l) {
    DevLevel& D = h->dev[l];
    const size_t es = h->precision == 0 ? sizeof(double) : sizeof(float);
    if (D.max_nloc > 1024)
      return fail(IRK_EINVAL, "patch of " + std::to_string(D.max_nloc) +
                                  " unknowns exceeds the factorisation limit of 1024");
    if (h->precision == 0) CHK(factor_level<double>(h, l, D.d64, dt, dfail, s));
    else CHK(factor_level<float>(h, l, D.d32, dt, dfail, s));
  }
  int hfail = 0;
  HIPCHK(hipMemcpyAsync(&hfail, dfail, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hfail) return fail(IRK_ESINGULAR, "zero pivot in a patch factorisation");
  // ---- coarse inverse (and of the transpose): dense operator assembled on the host,
  // inverted on the GPU in place (row-major result = column-major inverse of the
  // transpose), transposed for the column-major inverse
  {
    std::vector<double> Jc;
    double scale = 0;
    coarse_matrix(h->host[0], r, h->A, dt, Jc, &scale);
    const int64_t N0 = h->dev[0].N;
    CHK(upload(h, &h->coarse_invT, Jc, s));
    // the row-major operator is the column-major transpose; its transpose is the
    // column-major operator (both kept for the refinement step of the coarse solve)
    CHK(upload(h, &h->coarse_matT, Jc, s));
    Jc.clear();
    Jc.shrink_to_fit();
    double* colk;
    int64_t* swp;
    CHK(dalloc(h, &colk, (size_t)N0));
    CHK(dalloc(h, &swp, (size_t)N0));
    HIPCHK(hipMemsetAsync(dfail, 0, sizeof(int), s));
    HIPCHK(k::dense_inverse(h->coarse_invT, N0, std::max(1e-300, 1e-14 * scale), colk, swp, dfail, s));
    int cfail = 0;
    HIPCHK(hipMemcpyAsync(&cfail, dfail, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (cfail) return fail(IRK_ESINGULAR, "singular coarse operator");
    CHK(dalloc(h, &h->coarse_inv, (size_t)N0 * N0));
    HIPCHK(k::transpose(h->coarse_invT, h->coarse_inv, N0, s));
    CHK(dalloc(h, &h->coarse_mat, (size_t)N0 * N0));
    HIPCHK(k::transpose(h->coarse_matT, h->coarse_mat, N0, s));
    CHK(dalloc(h, &h->cb, N0));
    CHK(dalloc(h, &h->cx, N0));
    CHK(dalloc(h, &h->cpart, (size_t)N0 * k::coarse_split()));
    std::vector<int64_t> pins(r);
    for (int st = 0; st < r; ++st) pins[st] = h->dev[0].offV + st;
    CHK(upload(h, &h->pins, pins, s));
  }
  // ---- Krylov and reduction workspace
  const int64_t N = h->dev[nlevels - 1].N;
  CHK(dalloc(h, &h->kw, N));
  CHK(dalloc(h, &h->kF, N));
  CHK(dalloc(h, &h->kx, N));
  CHK(dalloc(h, &h->kr, N));
  CHK(dalloc(h, &h->scal, 16));
  CHK(dalloc(h, &h->partials, 1024));
  CHK(dalloc(h, &h->hbuf, 1024 + 2));
  for (hipEvent_t* e : {&h->ev0, &h->ev1, &h->ev2, &h->ev3, &h->ev4, &h->ev5, &h->evh}) HIPCHK(hipEventCreate(e));
  HIPCHK(hipHostMalloc((void**)&h->hpin, 2 * 1032 * sizeof(double), hipHostMallocDefault));
  HIPCHK(hipStreamSynchronize(s));
  return IRK_OK;
}

irk_status irk_mg_setup(const irk_mesh_level* lv, int nlevels, const irk_tableau* tab, double dt,
                        double nu, const double* wind, const irk_mg_opts* opt, void* stream,
                        irk_mg** out) {
  if (!out) return fail(IRK_EINVAL, "out is NULL");
  *out = nullptr;
  if (!lv || nlevels < 1 || nlevels > 16) return fail(IRK_EINVAL, "need 1..16 mesh levels");
  if (!tab || tab->r < 1 || tab->r > kMaxStages || !tab->A || !tab->b || !tab->c)
    return fail(IRK_EINVAL, "tableau must have 1 <= r <= 4 and non-null A, b, c");
  for (int i = 0; i < tab->r * tab->r; ++i)
    if (!std::isfinite(tab->A[i])) return fail(IRK_EINVAL, "non-finite tableau entry");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(IRK_EINVAL, "dt must be positive and finite");
  if (!(nu > 0) || !std::isfinite(nu)) return fail(IRK_EINVAL, "nu must be positive and finite");
  if (opt) {
    if (opt->pre < 0 || opt->post < 0 || opt->pre > 64 || opt->post > 64)
      return fail(IRK_EINVAL, "sweep counts must be in 0..64");
    if (!(opt->omega > 0) || !std::isfinite(opt->omega)) return fail(IRK_EINVAL, "omega must be positive");
    if (opt->weighting != 0 && opt->weighting != 1) return fail(IRK_EINVAL, "weighting must be 0 or 1");
    if (opt->precision != 0 && opt->precision != 1) return fail(IRK_EINVAL, "precision must be 0 or 1");
    if (opt->patch_form < 0 || opt->patch_form > 3) return fail(IRK_EINVAL, "patch_form must be 0, 1, 2 or 3");
    if (opt->smoother < 0 || opt->smoother > 2) return fail(IRK_EINVAL, "smoother must be 0, 1 or 2");
    if (opt->smoother == 2 && (opt->pre > kMaxGr || opt->post > kMaxGr))
      return fail(IRK_EINVAL, "GMRES relaxation takes at most " + std::to_string(kMaxGr) + " steps");
    if (opt->smoother == 1 && !(opt->cheb_lo > 0 && opt->cheb_hi > opt->cheb_lo && std::isfinite(opt->cheb_hi)))
      return fail(IRK_EINVAL, "Chebyshev interval must satisfy 0 < cheb_lo < cheb_hi < inf");
  }
  const int dim = lv[0].dim;
  if (dim != 2 && dim != 3) return fail(IRK_EINVAL, "dim must be 2 or 3");
  for (int l = 0; l < nlevels; ++l) {
    const irk_mesh_level& m = lv[l];
    if (m.dim != dim) return fail(IRK_EINVAL, "all levels must have the same dim");
    if (m.nverts < dim + 1 || m.ncells < 1 || !m.xyz || !m.cells)
      return fail(IRK_EINVAL, "level " + std::to_string(l) + ": empty mesh or null arrays");
    if (m.nverts > (1LL << 30) || m.ncells > (1LL << 30)) return fail(IRK_EINVAL, "mesh too large");
    if (l > 0 && !m.parent) return fail(IRK_EINVAL, "level " + std::to_string(l) + ": parent is NULL");
    if (l > 0 && m.ncells != lv[l - 1].ncells * (dim == 2 ? 4 : 8))
      return fail(IRK_EINVAL, "level " + std::to_string(l) + " is not a uniform refinement of level " +
                                  std::to_string(l - 1));
    for (int64_t i = 0; i < m.ncells * (dim + 1); ++i)
      if (m.cells[i] < 0 || m.cells[i] >= m.nverts)
        return fail(IRK_EINVAL, "level " + std::to_string(l) + ": vertex index out of range");
    for (int64_t i = 0; i < m.nverts * dim; ++i)
      if (!std::isfinite(m.xyz[i])) return fail(IRK_EINVAL, "non-finite coordinate");
    if (l > 0)
      for (int64_t c = 0; c < m.ncells; ++c)
        if (m.parent[c] < 0 || m.parent[c] >= lv[l - 1].ncells)
          return fail(IRK_EINVAL, "level " + std::to_string(l) + ": parent index out of range");
  }
  irk_mg* h = new (std::nothrow) irk_mg();
  if (!h) return fail(IRK_ENOMEM, "handle allocation failed");
  irk_status st;
  try {
    st = setup_impl(lv, nlevels, tab, dt, nu, wind, opt, S(stream), h);
  } catch (const std::bad_alloc&) {
    st = fail(IRK_ENOMEM, "host allocation failed during setup");
  } catch (const std::exception& e) {
    st = fail(IRK_EINVAL, std::string("setup failed: ") + e.what());
  }
  if (st != IRK_OK) {
    irk_mg_destroy(h);
    return st;
  }
  *out = h;
  g_err.clear();
  return IRK_OK;
}

int irk_mg_patch_form(const irk_mg* h) {
  if (!h) return -1;
  return h->nlevels >= 2 ? h->dev[h->nlevels - 1].pform : h->patch_form;
}

irk_status irk_rhs_dirichlet(irk_mg* h, const double* g_n, const double* g_stages, double* F, void* stream) {
  CHK(check_handle(h));
  if (!g_n || !g_stages || !F) return fail(IRK_EINVAL, "null vector");
  if (!h->A_invertible) return fail(IRK_EINVAL, "boundary stage derivatives need an invertible A");
  const DevLevel& L = h->dev[h->nlevels - 1];
  HIPCHK(k::rhs_dirichlet(L, h->Ainv_dt, g_n, g_stages, F, S(stream)));
  return IRK_OK;
}

irk_status irk_hessenberg_eigs(int m, const double* H, int ldh, double* wr, double* wi) {
  if (m < 1 || m > 1024 || ldh < m || !H || !wr || !wi) return fail(IRK_EINVAL, "need 1 <= m <= 1024, ldh >= m");
  if (!irk::hessenberg_eigs(m, H, ldh, wr, wi)) return fail(IRK_ENOCONV, "Hessenberg QR iteration did not converge");
  return IRK_OK;
}

irk_status irk_mg_ritz(irk_mg* h, int level, int steps, const double* v0, double* H, double* ritz_re,
                       double* ritz_im, int* nritz, void* stream) {
  CHK(irk::ritz_check(h, level, steps, v0, ritz_re, ritz_im));
  std::vector<double> Hh((size_t)(steps + 1) * steps);
  hipStream_t s = S(stream);
  if (h->precision == 0) CHK(ritz_T<double>(h, level, steps, v0, Hh.data(), s));
  else CHK(ritz_T<float>(h, level, steps, v0, Hh.data(), s));
  std::vector<std::complex<double>> work((size_t)steps * steps + 3 * (size_t)steps);
  std::vector<int> iwork(steps);
  return irk::ritz_finish(steps, Hh.data(), H, ritz_re, ritz_im, nritz, work.data(), iwork.data());
}

irk_status irk_mg_set_interval(irk_mg* h, double lo, double hi) {
  CHK(check_handle(h));
  if (!(lo > 0 && hi > lo && std::isfinite(hi))) return fail(IRK_EINVAL, "need 0 < lo < hi < inf");
  h->cheb_lo = lo;
  h->cheb_hi = hi;
  return IRK_OK;
}

irk_status irk_stage_basis(int r, const double* A, double* W, double* Winv, double* T) {
  if (r < 1 || r > irk::kMaxStages || !A) return fail(IRK_EINVAL, "need 1 <= r <= 4 and a non-null A");
  irk::StageEig E;
  std::string why;
  if (!irk::stage_eigenbasis(A, r, E, &why)) return fail(IRK_EINVAL, why);
  if (W) std::memcpy(W, E.W, sizeof(double) * r * r);
  if (Winv) std::memcpy(Winv, E.Winv, sizeof(double) * r * r);
  if (T) {
    for (int i = 0; i < r * r; ++i) T[i] = 0.0;
    for (int b = 0; b < E.nblk; ++b)
      for (int i = 0; i < E.type[b]; ++i)
        for (int j = 0; j < E.type[b]; ++j) T[(E.st0[b] + i) * r + E.st0[b] + j] = E.Tb[b][i * E.type[b] + j];
  }
  return IRK_OK;
}

int64_t irk_mg_ndofs(const irk_mg* h, int level) {
  if (!h) return -1;
  if (level < 0) level = h->nlevels - 1;
  if (level >= h->nlevels) return -1;
  return h->dev[level].N;
}

irk_status irk_mg_sizes(const irk_mg* hc, int level, int64_t* out) {
  irk_mg* h = const_cast<irk_mg*>(hc);
  CHK(check_level(h, level));
  if (!out) return fail(IRK_EINVAL, "out is NULL");
  const HostLevel& H = h->host[level];
  out[0] = H.nv;
  out[1] = H.nn;
  out[2] = H.nfree;
  out[3] = H.dim * H.nfree + H.nv;
  out[4] = h->nlevels;
  return IRK_OK;
}

irk_status irk_mg_p2_nodes(const irk_mg* hc, int level, double* xyz, int64_t* free_nodes) {
  irk_mg* h = const_cast<irk_mg*>(hc);
  CHK(check_level(h, level));
  const HostLevel& H = h->host[level];
  const int d = H.dim;
  if (xyz)
    for (int64_t n = 0; n < H.nn; ++n) {
      if (n < H.nv) {
        for (int i = 0; i < d; ++i) xyz[n * d + i] = H.xyz[n * d + i];
      } else {
        const int64_t a = H.edges[(n - H.nv) * 2], b = H.edges[(n - H.nv) * 2 + 1];
        for (int i = 0; i < d; ++i) xyz[n * d + i] = 0.5 * (H.xyz[a * d + i] + H.xyz[b * d + i]);
      }
    }
  if (free_nodes)
    for (int64_t i = 0; i < H.nfree; ++i) free_nodes[i] = H.node_of_free[i];
  return IRK_OK;
}

irk_status irk_mg_apply(irk_mg* h, const double* x, double* y, int transpose, void* stream) {
  return irk_level_apply(h, -1, transpose, x, y, stream);
}

irk_status irk_mg_vcycle(irk_mg* h, const double* r, double* z, void* stream) {
  CHK(check_handle(h));
  if (!r || !z) return fail(IRK_EINVAL, "null vector");
  if (r == z) return fail(IRK_EINVAL, "r and z may not alias");
  DevLevel& L = h->dev[h->nlevels - 1];
  hipStream_t s = S(stream);
  HIPCHK(k::to_internal<double>(L, r, h->kr, s));
  CHK(precondition(h, h->kr, h->kF, false, s));
  HIPCHK(k::to_abi<double>(L, h->kF, z, s));
  return IRK_OK;
}

irk_status irk_mg_vcycle_transpose(irk_mg* h, const double* r, double* z, void* stream) {
  CHK(check_handle(h));
  if (!r || !z) return fail(IRK_EINVAL, "null vector");
  if (r == z) return fail(IRK_EINVAL, "r and z may not alias");
  DevLevel& L = h->dev[h->nlevels - 1];
  hipStream_t s = S(stream);
  HIPCHK(k::to_internal<double>(L, r, h->kr, s));
  CHK(precondition(h, h->kr, h->kF, true, s));
  HIPCHK(k::to_abi<double>(L, h->kF, z, s));
  return IRK_OK;
}

irk_status irk_fgmres_solve(irk_mg* h, const double* F, double* k, double rtol, int maxit, int restart,
                            irk_solve_info* info, void* stream) {
  CHK(check_handle(h));
  return fgmres(h, F, k, rtol, maxit, restart, info, false, S(stream));
}

void irk_newton_default_opts(irk_newton_opts* o) {
  if (!o) return;
  o->rtol = 1e-8;
  o->atol = 0.0;
  o->maxit = 20;
  o->linear_maxit = 200;
  o->restart = 30;
  o->eta0 = 0.3;
  o->eta_max = 0.9;
  o->ew_gamma = 1.0;
  o->ew_alpha = 0.5 * (1.0 + std::sqrt(5.0));
  o->ew_threshold = 0.1;
  o->eta_fixed = 0.0;
  o->linesearch = 0;
  o->ls_maxit = 12;
  o->ls_alpha = 1e-4;
  o->precond = 0;
}

irk_status irk_ns_newton_preconditioner(irk_mg* h, const double* state, const double* g_stages, const double* k,
                                        int enable, void* stream) {
  CHK(check_handle(h));
  if (enable != 0 && enable != 1) return fail(IRK_EINVAL, "enable must be 0 or 1");
  if (!enable) {
    h->nw_active = false;
    return IRK_OK;
  }
  if (!state || !k) return fail(IRK_EINVAL, "null vector");
  if (h->precision != 0) return fail(IRK_EINVAL, "the Newton Jacobian V-cycle needs an FP64 handle");
  hipStream_t s = S(stream);
  CHK(ns_init(h, s));
  DevLevel& L = h->dev[h->nlevels - 1];
  HIPCHK(k::to_internal<double>(L, k, h->ns_kt, s));
  CHK(ns_stage_values(h, state, h->ns_kt, g_stages, s));
  h->nw_active = false;
  CHK(nw_build(h, s));
  h->nw_active = true;
  return IRK_OK;
}

// R = F - J k - c(U - w, U): minus the residual of the stage equations of Sec. 3.2 (F
// from irk_rhs on this handle, in ns_F) at k (internal layout), into ns_G; state and g_st
// as in the public calls.
static irk_status ns_residual_int(irk_mg* h, const double* state, const double* g_st, const double* kk,
                                  hipStream_t s) {
  CHK(ns_stage_values(h, state, kk, g_st, s));
  const bool jac = h->ns_jac;
  h->ns_jac = false;
  irk_status st = apply_J(h, kk, h->ns_G, false, h->ns_F, s);
  h->ns_jac = jac;
  CHK(st);
  CHK(ns_correction(h, 0, nullptr, h->ns_G, -1.0, s));
  return IRK_OK;
}

irk_status irk_ns_residual(irk_mg* h, const double* F, const double* state, const double* g_stages,
                           const double* k, double* R, void* stream) {
  CHK(check_handle(h));
  if (!F || !state || !k || !R) return fail(IRK_EINVAL, "null vector");
  hipStream_t s = S(stream);
  CHK(ns_init(h, s));
  DevLevel& L = h->dev[h->nlevels - 1];
  HIPCHK(k::to_internal<double>(L, k, h->ns_k, s));
  HIPCHK(k::to_internal<double>(L, F, h->ns_F, s));
  CHK(ns_residual_int(h, state, g_stages, h->ns_k, s));
  HIPCHK(k::to_abi<double>(L, h->ns_G, R, s));
  return IRK_OK;
}

irk_status irk_ns_jacobian_apply(irk_mg* h, const double* state, const double* g_stages, const double* k,
                                 const double* x, double* y, void* stream) {
  CHK(check_handle(h));
  if (!state || !k || !x || !y) return fail(IRK_EINVAL, "null vector");
  hipStream_t s = S(stream);
  CHK(ns_init(h, s));
  DevLevel& L = h->dev[h->nlevels - 1];
  HIPCHK(k::to_internal<double>(L, k, h->ns_k, s));
  CHK(ns_stage_values(h, state, h->ns_k, g_stages, s));
  HIPCHK(k::to_internal<double>(L, x, h->ns_F, s));
  h->ns_jac = true;
  irk_status st = apply_J(h, h->ns_F, h->ns_G, false, nullptr, s);
  h->ns_jac = false;
  CHK(st);
  HIPCHK(k::to_abi<double>(L, h->ns_G, y, s));
  return IRK_OK;
}

irk_status irk_ns_newton_solve(irk_mg* h, const double* F, const double* state, const double* g_stages,
                               double* k, const irk_newton_opts* opt, irk_newton_info* info, void* stream) {
  CHK(check_handle(h));
  if (!F || !state || !k) return fail(IRK_EINVAL, "null vector");
  irk_newton_opts o;
  irk_newton_default_opts(&o);
  if (opt) o = *opt;
  if (!(o.rtol >= 0) || !(o.atol >= 0) || o.maxit < 0 || o.linear_maxit < 1 || o.restart < 1 ||
      o.restart > 1000 || !(o.eta0 > 0 && o.eta0 < 1) || !(o.eta_max > 0 && o.eta_max < 1) ||
      !(o.ew_gamma > 0 && o.ew_gamma <= 1) || !(o.ew_alpha > 1 && o.ew_alpha <= 2) || !(o.ew_threshold >= 0) ||
      !(o.eta_fixed >= 0 && o.eta_fixed < 1) || o.linesearch < 0 || o.linesearch > 1 || o.ls_maxit < 0 ||
      o.ls_maxit > 60 || !(o.ls_alpha > 0 && o.ls_alpha < 1) || o.precond < 0 || o.precond > 1)
    return fail(IRK_EINVAL, "invalid Newton options");
  if (o.precond == 1 && h->precision != 0)
    return fail(IRK_EINVAL, "the Newton Jacobian V-cycle (precond 1) needs an FP64 handle");
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = S(stream);
  CHK(ns_init(h, s));
  CHK(ensure_krylov(h, o.restart));
  DevLevel& L = h->dev[h->nlevels - 1];
  const int64_t N = L.N;
  HIPCHK(k::to_internal<double>(L, F, h->ns_F, s));
  HIPCHK(k::to_internal<double>(L, k, h->ns_k, s));
  int it = 0, lin = 0, nhist = 0;
  bool converged = false, ls_failed = false;
  double norm0 = 0, norm = 0, norm_prev = 0, eta_prev = o.eta0;
  float ms_lin = 0;
  irk_status st = IRK_OK;
  // ||G(kk)||, the residual left in ns_G
  auto residual_norm = [&](const double* kk, double* out) -> irk_status {
    CHK(ns_residual_int(h, state, g_stages, kk, s));
    HIPCHK(k::dot(h->ns_G, h->ns_G, N, h->partials, h->scal, s, 1));
    HIPCHK(hipMemcpyAsync(out, h->scal, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return IRK_OK;
  };
  CHK(residual_norm(h->ns_k, &norm));
  for (;;) {
    if (info && info->history && nhist < info->history_cap) info->history[nhist] = norm;
    ++nhist;
    if (!std::isfinite(norm)) return fail(IRK_ENAN, "non-finite Navier--Stokes residual");
    if (it == 0) norm0 = norm;
    const double tol = std::max(o.atol, o.rtol * norm0);
    if (norm <= tol) {
      converged = true;
      break;
    }
    if (it >= o.maxit) break;
    // forcing term: Eisenstat--Walker choice 2 with its safeguard, or a fixed value
    double eta;
    if (o.eta_fixed > 0) {
      eta = o.eta_fixed;
    } else if (it == 0) {
      eta = std::min(o.eta0, o.eta_max);
    } else {
      eta = o.ew_gamma * std::pow(norm / norm_prev, o.ew_alpha);
      const double guard = o.ew_gamma * std::pow(eta_prev, o.ew_alpha);
      if (guard > o.ew_threshold) eta = std::max(eta, guard);
      eta = std::min(eta, o.eta_max);
    }
    // final-step safeguard: no forcing term below half the stopping tolerance over ||G||
    if (o.eta_fixed <= 0 && tol > 0) eta = std::min(o.eta_max, std::max(eta, 0.5 * tol / norm));
    if (info && it < info->history_cap) {
      if (info->etas) info->etas[it] = eta;
    }
    // J delta = R from delta = 0, to ||R - J delta|| <= eta ||R||
    HIPCHK(hipMemcpyAsync(h->kF, h->ns_G, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(k::fill(h->kx, N, 0.0, s));
    irk_solve_info li{};
    if (o.precond == 1) CHK(nw_build(h, s));  // ns_U holds the stage values at the iterate
    HIPCHK(hipEventRecord(h->ev0, s));
    const bool nw_prev = h->nw_active;
    h->nw_active = o.precond == 1 || nw_prev;
    h->ns_jac = true;
    st = fgmres_int(h, nullptr, eta, o.linear_maxit, o.restart, &li, false, s);
    h->ns_jac = false;
    h->nw_active = nw_prev;
    if (st < 0) return st;
    lin += li.iterations;
    ms_lin += (float)li.ms_total;
    if (info && info->linear_its && it < info->history_cap) info->linear_its[it] = li.iterations;
    // k + lam delta: lam = 1, or with the line search the first of 1, 1/2, ... giving
    // ||G|| <= (1 - ls_alpha lam) ||G(k)|| (sufficient decrease)
    double lam = 1.0, nt = 0.0;
    bool ok = false;
    for (int t = 0; t <= (o.linesearch ? o.ls_maxit : 0); ++t) {
      HIPCHK(hipMemcpyAsync(h->ns_kt, h->ns_k, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIPCHK(k::axpby(h->ns_kt, h->kx, N, lam, 1.0, s));
      CHK(residual_norm(h->ns_kt, &nt));
      if (!o.linesearch || (std::isfinite(nt) && nt <= (1.0 - o.ls_alpha * lam) * norm)) {
        ok = true;
        break;
      }
      lam *= 0.5;
    }
    if (!ok) {  // no sufficient decrease: k stays the last accepted iterate
      ls_failed = true;
      break;
    }
    std::swap(h->ns_k, h->ns_kt);
    if (info && info->lambdas && it < info->history_cap) info->lambdas[it] = lam;
    eta_prev = eta;
    norm_prev = norm;
    norm = nt;
    ++it;
  }
  HIPCHK(k::to_abi<double>(L, h->ns_k, k, s));
  HIPCHK(hipStreamSynchronize(s));
  if (info) {
    info->iterations = it;
    info->converged = converged ? 1 : 0;
    info->linear_iterations = lin;
    info->norm0 = norm0;
    info->norm = norm;
    info->ms_linear = ms_lin;
    info->ms_wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (!converged) {
    g_err = ls_failed ? "Newton line search found no sufficient decrease" : "Newton reached maxit";
    return IRK_ENOCONV;
  }
  return IRK_OK;
}

irk_status irk_adjoint_solve(irk_mg* h, const double* G, double* lam, double rtol, int maxit, int restart,
                             irk_solve_info* info, void* stream) {
  CHK(check_handle(h));
  return fgmres(h, G, lam, rtol, maxit, restart, info, true, S(stream));
}

irk_status irk_rhs(irk_mg* h, const double* f, const double* state, double* F, void* stream) {
  CHK(check_handle(h));
  if (!f || !state || !F) return fail(IRK_EINVAL, "null vector");
  const int top = h->nlevels - 1;
  HIPCHK(k::rhs(h->dev[top], h->host[top].nn, f, state, F, S(stream)));
  return IRK_OK;
}

irk_status irk_update(irk_mg* h, const double* kv, double* state, void* stream) {
  CHK(check_handle(h));
  if (!kv || !state) return fail(IRK_EINVAL, "null vector");
  HIPCHK(k::update(h->dev[h->nlevels - 1], h->b, h->dt, kv, state, S(stream)));
  return IRK_OK;
}

irk_status irk_rhs_adjoint(irk_mg* h, const double* lam, double* gf, double* gstate, int accumulate,
                           void* stream) {
  CHK(check_handle(h));
  if (!lam || !gf || !gstate) return fail(IRK_EINVAL, "null vector");
  if (accumulate != 0 && accumulate != 1) return fail(IRK_EINVAL, "accumulate must be 0 or 1");
  const int top = h->nlevels - 1;
  DevLevel& L = h->dev[top];
  HIPCHK(k::rhs_adjoint(L, h->host[top].nn, L.mfat_ptr, L.mfat_col, L.mfat_val, lam, gf, gstate, accumulate,
                        S(stream)));
  return IRK_OK;
}

irk_status irk_update_adjoint(irk_mg* h, const double* gstate, double* G, void* stream) {
  CHK(check_handle(h));
  if (!gstate || !G) return fail(IRK_EINVAL, "null vector");
  HIPCHK(k::update_adjoint(h->dev[h->nlevels - 1], h->b, h->dt, gstate, G, S(stream)));
  return IRK_OK;
}

irk_status irk_nu_sensitivity(irk_mg* h, const double* lam, const double* kv, const double* state, double* out,
                              int accumulate, void* stream) {
  CHK(check_handle(h));
  if (!lam || !kv || !state || !out) return fail(IRK_EINVAL, "null vector");
  if (accumulate != 0 && accumulate != 1) return fail(IRK_EINVAL, "accumulate must be 0 or 1");
  DevLevel& L = h->dev[h->nlevels - 1];
  HIPCHK(k::nu_sensitivity(L, h->A, h->dt, lam, kv, state, h->kw, h->partials, out, accumulate, S(stream)));
  return IRK_OK;
}

irk_status irk_tracking_loss(irk_mg* h, const double* state, const double* target, const double* scale,
                             double* loss, double* grad_state, double* grad_target, void* stream) {
  CHK(check_handle(h));
  if (!state || !target) return fail(IRK_EINVAL, "null vector");
  if (!loss && !grad_state && !grad_target) return fail(IRK_EINVAL, "no output requested");
  DevLevel& L = h->dev[h->nlevels - 1];
  HIPCHK(k::tracking_loss(L, state, target, scale, loss, grad_state, grad_target, h->kw, h->kr, h->partials,
                          S(stream)));
  return IRK_OK;
}

irk_status irk_mg_layout(const irk_mg* hc, int level, int64_t* offsets, int64_t* lengths) {
  irk_mg* h = const_cast<irk_mg*>(hc);
  CHK(check_level(h, level));
  if (!offsets && !lengths) return fail(IRK_EINVAL, "no output requested");
  const HostLevel& H = h->host[level];
  const int d = H.dim;
  const int64_t ns = d * H.nfree + H.nv;
  for (int st = 0; st < h->r && offsets; ++st) {
    for (int c = 0; c < d; ++c) offsets[st * (d + 1) + c] = st * ns + c * H.nfree;
    offsets[st * (d + 1) + d] = st * ns + d * H.nfree;
  }
  if (lengths) {
    for (int c = 0; c < d; ++c) lengths[c] = H.nfree;
    lengths[d] = H.nv;
  }
  return IRK_OK;
}

irk_status irk_mass_apply(irk_mg* h, const double* state, double* out, void* stream) {
  CHK(check_handle(h));
  if (!state || !out) return fail(IRK_EINVAL, "null vector");
  HIPCHK(k::mass_apply(h->dev[h->nlevels - 1], state, out, S(stream)));
  return IRK_OK;
}

irk_status irk_level_apply(irk_mg* h, int level, int transpose, const double* x, double* y,
                           void* stream) {
  CHK(check_level(h, level));
  if (!x || !y) return fail(IRK_EINVAL, "null vector");
  if (x == y) return fail(IRK_EINVAL, "x and y may not alias");
  DevLevel& L = h->dev[level];
  hipStream_t s = S(stream);
  double* tmp_in = h->kw;  // finest-level FGMRES scratch, large enough for any level
  double* tmp_out = h->kr;
  HIPCHK(k::to_internal<double>(L, x, tmp_in, s));
  DevOps<double> o = L.d64;
  if (transpose) {
    o.s_L = o.s_Lt;
    o.u_L = o.u_Lt;
  }
  if (h->nw_active && transpose) return fail(IRK_EINVAL, "the Newton Jacobian level operators have no transpose");
  HIPCHK(lev_residual<double>(h, level, o, transpose ? h->At : h->A, nullptr, tmp_in, tmp_out, s));
  HIPCHK(k::to_abi<double>(L, tmp_out, y, s));
  return IRK_OK;
}

irk_status irk_level_sweep(irk_mg* h, int level, int transpose, const double* F, double* kv,
                           void* stream) {
  CHK(check_level(h, level));
  if (level < 1) return fail(IRK_EINVAL, "the coarsest level has no patches");
  if (!F || !kv) return fail(IRK_EINVAL, "null vector");
  if (h->nw_active && transpose) return fail(IRK_EINVAL, "the Newton Jacobian relaxation has no transpose");
  if (h->precision == 0) return level_sweep_T<double>(h, level, transpose, F, kv, S(stream));
  return level_sweep_T<float>(h, level, transpose, F, kv, S(stream));
}

irk_status irk_level_restrict(irk_mg* h, int level, const double* xf, double* xc, void* stream) {
  CHK(check_level(h, level));
  if (level < 1) return fail(IRK_EINVAL, "level must be >= 1");
  if (!xf || !xc) return fail(IRK_EINVAL, "null vector");
  DevLevel& F = h->dev[level];
  DevLevel& C = h->dev[level - 1];
  hipStream_t s = S(stream);
  HIPCHK(k::to_internal<double>(F, xf, h->kw, s));
  HIPCHK(k::restrict_<double>(F, C, F.d64, h->kw, h->kr, s));
  HIPCHK(k::to_abi<double>(C, h->kr, xc, s));
  return IRK_OK;
}

irk_status irk_level_prolong(irk_mg* h, int level, const double* xc, double* xf, void* stream) {
  CHK(check_level(h, level));
  if (level < 1) return fail(IRK_EINVAL, "level must be >= 1");
  if (!xf || !xc) return fail(IRK_EINVAL, "null vector");
  DevLevel& F = h->dev[level];
  DevLevel& C = h->dev[level - 1];
  hipStream_t s = S(stream);
  HIPCHK(k::to_internal<double>(C, xc, h->kw, s));
  HIPCHK(k::to_internal<double>(F, xf, h->kr, s));
  HIPCHK(k::prolong_add<double>(F, C, F.d64, h->kw, h->kr, s));
  HIPCHK(k::to_abi<double>(F, h->kr, xf, s));
  return IRK_OK;
}

irk_status irk_coarse_solve(irk_mg* h, int transpose, const double* b, double* x, void* stream) {
  CHK(check_handle(h));
  if (!b || !x) return fail(IRK_EINVAL, "null vector");
  DevLevel& L = h->dev[0];
  hipStream_t s = S(stream);
  HIPCHK(k::to_internal<double>(L, b, h->cb, s));
  if (h->nw_active) {
    if (transpose) return fail(IRK_EINVAL, "the Newton Jacobian coarse solve has no transpose");
    HIPCHK(k::coarse_solve(h->nw_cinv, h->nw_cmat, L.N, h->cb, h->cx, h->pins, h->r, h->cpart, s));
  } else {
    HIPCHK(k::coarse_solve(transpose ? h->coarse_invT : h->coarse_inv, transpose ? h->coarse_matT : h->coarse_mat,
                           L.N, h->cb, h->cx, h->pins, h->r, h->cpart, s));
  }
  HIPCHK(k::to_abi<double>(L, h->cx, x, s));
  return IRK_OK;
}

}  // extern "C"
