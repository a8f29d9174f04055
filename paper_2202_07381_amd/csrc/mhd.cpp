// C ABI of the linearised 2D MHD stage solver (include/irk_mhd.h): argument checks, setup
// orchestration, the multi-launch V-cycle (Sec. 4.1, 4.2) and restarted FGMRES (Sec. 4).
// The relaxation reuses the patch kernels of the fluid solver (dense stage-coupled
// inverses, one wavefront per patch, owner gather); host code only sequences kernels.
#include "../../include/irk_mhd.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

#include "mhd_internal.h"

using namespace irk;

namespace {

struct MhdDev {
  int64_t ns = 0, N = 0;
  int64_t off[5] = {0, 0, 0, 0, 0};  // u_x, u_y, B, p, gamma
  // spatial operator, sliced: M and S values on one pattern
  int64_t nsl = 0;
  int32_t *sl_off = nullptr, *sl_w = nullptr, *sl_col = nullptr;
  double *sl_m = nullptr, *sl_s = nullptr;
  // prolongation from the coarser level (fine rows) and its transpose (coarse rows)
  int64_t nc_rows = 0;
  int32_t *P_ptr = nullptr, *P_col = nullptr, *Pt_ptr = nullptr, *Pt_col = nullptr;
  double *P_val = nullptr, *Pt_val = nullptr;
  // what the shared patch kernels read (dim = 1: one value per unknown and stage), and
  // the pressure block for the projection (offV, nv)
  DevLevel pv;
  DevOps<double> ops;
  double *b = nullptr, *x = nullptr, *res = nullptr, *Y = nullptr;
  double* dch = nullptr;  // Chebyshev direction
  // algorithmic bytes per launch: patch apply, residual, gather update
  double alg_bytes[3] = {0, 0, 0};
};

struct ProfEv {
  hipEvent_t a = nullptr, b = nullptr;
  int kernel = 0, level = 0;
};

}  // namespace

struct irk_mhd {
  int r = 0, nlevels = 0;
  double dt = 0, A[kMaxStages * kMaxStages] = {0};
  int pre = 2, post = 2, weighting = 1;
  double omega = 0.5;
  int smoother = 0;  // 0 damped additive sweeps, 1 Chebyshev (Sec. 5.1)
  double cheb_lo = 2.0, cheb_hi = 10.0;
  int pform = 0;     // patch storage: 0 dense, 1 factored through the stage eigenbasis
  StageEig eig;      // A = W T W^{-1} when pform = 1
  std::vector<MhdDev> dev;
  double *cinv = nullptr, *cmat = nullptr, *cpart = nullptr;
  int64_t* pins = nullptr;
  int restart_cap = 0;
  double *kv = nullptr, *kz = nullptr, *kF = nullptr, *kx = nullptr, *kr = nullptr;
  double *partials = nullptr, *scal = nullptr, *hbuf = nullptr;
  int* flag = nullptr;
  // 0, 1: the solve; 2, 3 and 4, 5: V-cycles of alternate FGMRES iterations; 6: the
  // Hessenberg column's copy
  hipEvent_t ev[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  double* hpin = nullptr;  // pinned host: Hessenberg column and update coefficients
  int prof = 0;  // 0 off, 1 finest level, 2 every level
  std::vector<ProfEv> prof_pool;
  size_t prof_used = 0;
  std::vector<void*> allocations;
};

namespace {

irk_status fail(irk_status code, const std::string& msg) { return fail_with(code, msg); }

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(e_ == hipErrorOutOfMemory ? IRK_ENOMEM : IRK_EHIP,                  \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                 \
  } while (0)

#define CHK(expr)                \
  do {                           \
    irk_status s_ = (expr);      \
    if (s_ != IRK_OK) return s_; \
  } while (0)

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

template <typename T>
irk_status dalloc(irk_mhd* h, T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc((void**)p, n * sizeof(T));
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? IRK_ENOMEM : IRK_EHIP,
                "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
  h->allocations.push_back(*p);
  if (poison_requested()) HIPCHK(hipMemset(*p, 0xFF, n * sizeof(T)));
  return IRK_OK;
}

template <typename T, typename Src>
irk_status upload(irk_mhd* h, T** p, const std::vector<Src>& v, hipStream_t s) {
  CHK(dalloc(h, p, v.size()));
  if (v.empty()) return IRK_OK;
  // same element type: copied from the source itself (no staging copy); the wait keeps
  // the source (or the converted copy) alive until the transfer has read it
  if constexpr (std::is_same<T, Src>::value) {
    HIPCHK(hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  } else {
    std::vector<T> tmp(v.begin(), v.end());
    HIPCHK(hipMemcpyAsync(*p, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  return IRK_OK;
}

// ------------------------------------------------------------------- measurement
int prof_begin(irk_mhd* h, int kernel, int level, hipStream_t s) {
  if (!h->prof || (h->prof == 1 && level != h->nlevels - 1)) return -1;
  if (h->prof_used == h->prof_pool.size()) {
    ProfEv e;
    if (hipEventCreate(&e.a) != hipSuccess || hipEventCreate(&e.b) != hipSuccess) return -1;
    h->prof_pool.push_back(e);
  }
  ProfEv& e = h->prof_pool[h->prof_used];
  e.kernel = kernel;
  e.level = level;
  if (hipEventRecord(e.a, s) != hipSuccess) return -1;
  return (int)h->prof_used++;
}

void prof_end(irk_mhd* h, int idx, hipStream_t s) {
  if (idx >= 0) (void)hipEventRecord(h->prof_pool[idx].b, s);
}

// ------------------------------------------------------------------ level operations
irk_status residual(irk_mhd* h, int l, const double* F, const double* x, double* y, hipStream_t s) {
  const MhdDev& D = h->dev[l];
  const int pe = prof_begin(h, 1, l, s);
  HIPCHK(k::kron_residual(D.ns, D.nsl, D.sl_off, D.sl_w, D.sl_col, D.sl_m, D.sl_s, h->r, h->A, h->dt, F, x, y, s));
  prof_end(h, pe, s);
  return IRK_OK;
}

// one damped additive sweep x += omega W S (b - J x); from x = 0 (zero) the residual is b
irk_status sweep(irk_mhd* h, int l, const double* b, double* x, bool zero, hipStream_t s) {
  MhdDev& D = h->dev[l];
  const double* res = b;
  if (!zero) {
    CHK(residual(h, l, b, x, D.res, s));
    res = D.res;
  }
  int pe = prof_begin(h, 0, l, s);
  HIPCHK(k::patch_apply<double>(D.pv, D.ops, res, D.Y, 0, s));
  prof_end(h, pe, s);
  pe = prof_begin(h, 2, l, s);
  HIPCHK(k::gather_update<double>(D.pv, D.ops, D.Y, x, h->omega, zero ? 0 : 1, s));
  prof_end(h, pe, s);
  return IRK_OK;
}

// n relaxation steps on level l from x (from zero when zero): damped sweeps, or the
// Chebyshev semi-iteration on [cheb_lo, cheb_hi] for the spectrum of W S J (theta, delta,
// sigma and the rho recurrence, coefficients in FP64)
irk_status relax(irk_mhd* h, int l, const double* b, double* x, int n, bool zero, hipStream_t s) {
  MhdDev& D = h->dev[l];
  if (n == 0) {
    if (zero) HIPCHK(k::fill(x, D.N, 0.0, s));
    return IRK_OK;
  }
  if (h->smoother == 0) {
    for (int i = 0; i < n; ++i) CHK(sweep(h, l, b, x, zero && i == 0, s));
    return IRK_OK;
  }
  const double theta = 0.5 * (h->cheb_hi + h->cheb_lo), delta = 0.5 * (h->cheb_hi - h->cheb_lo);
  const double sigma = theta / delta;
  double rho = 0.0;
  for (int it = 0; it < n; ++it) {
    const bool xzero = zero && it == 0;
    const double* r = b;
    if (!xzero) {
      CHK(residual(h, l, b, x, D.res, s));
      r = D.res;
    }
    int pe = prof_begin(h, 0, l, s);
    HIPCHK(k::patch_apply<double>(D.pv, D.ops, r, D.Y, 0, s));
    prof_end(h, pe, s);
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
    pe = prof_begin(h, 2, l, s);
    HIPCHK(k::gather_cheb<double>(D.pv, D.ops, D.Y, c1, c2, it == 0 ? 1 : 0, xzero ? 1 : 0, 0, D.dch, x, s));
    prof_end(h, pe, s);
  }
  return IRK_OK;
}

irk_status coarse(irk_mhd* h, double* b, double* x, hipStream_t s) {
  HIPCHK(k::coarse_solve(h->cinv, h->cmat, h->dev[0].N, b, x, h->pins, h->r, h->cpart, s));
  return IRK_OK;
}

// x = V_l b from zero (b is not modified on level l >= 1)
irk_status cycle(irk_mhd* h, int l, const double* b, double* x, hipStream_t s) {
  MhdDev& D = h->dev[l];
  if (l == 0) {
    // the coarse solve overwrites its right-hand side (refinement step)
    if (b != D.b) HIPCHK(hipMemcpyAsync(D.b, b, D.N * sizeof(double), hipMemcpyDeviceToDevice, s));
    return coarse(h, D.b, x, s);
  }
  CHK(relax(h, l, b, x, h->pre, true, s));
  CHK(residual(h, l, b, x, D.res, s));
  MhdDev& C = h->dev[l - 1];
  HIPCHK(k::kron_csr(C.ns, D.Pt_ptr, D.Pt_col, D.Pt_val, h->r, D.res, C.b, 0, s));
  CHK(cycle(h, l - 1, C.b, C.x, s));
  HIPCHK(k::kron_csr(D.ns, D.P_ptr, D.P_col, D.P_val, h->r, C.x, x, 1, s));
  CHK(relax(h, l, b, x, h->post, false, s));
  return IRK_OK;
}

irk_status precondition(irk_mhd* h, const double* v, double* z, hipStream_t s) {
  MhdDev& F = h->dev[h->nlevels - 1];
  CHK(cycle(h, h->nlevels - 1, v, z, s));
  HIPCHK(k::project_pressure(F.pv, z, h->partials, s));
  return IRK_OK;
}

irk_status ensure_krylov(irk_mhd* h, int restart) {
  if (restart <= h->restart_cap) return IRK_OK;
  const int64_t N = h->dev[h->nlevels - 1].N;
  h->restart_cap = 0;  // no usable basis until the new one is in place
  for (double** p : {&h->kv, &h->kz}) {
    if (*p) {
      h->allocations.erase(std::find(h->allocations.begin(), h->allocations.end(), (void*)*p));
      HIPCHK(hipFree(*p));
      *p = nullptr;
    }
  }
  CHK(dalloc(h, &h->kv, (size_t)(restart + 1) * N));
  CHK(dalloc(h, &h->kz, (size_t)restart * N));
  if (h->hbuf) {
    h->allocations.erase(std::find(h->allocations.begin(), h->allocations.end(), (void*)h->hbuf));
    HIPCHK(hipFree(h->hbuf));
    h->hbuf = nullptr;
  }
  CHK(dalloc(h, &h->hbuf, (size_t)restart + 2));
  h->restart_cap = restart;
  return IRK_OK;
}

// Start the next FGMRES iteration's V-cycle before the host has read the Hessenberg column
// when the predicted residual estimate stays above this many tolerances.
constexpr double kSpecMargin = 20.0;

irk_status fgmres(irk_mhd* h, double rtol, int maxit, int restart, irk_solve_info* info, hipStream_t s) {
  const int fl = h->nlevels - 1;
  MhdDev& L = h->dev[fl];
  const int64_t N = L.N;
  std::vector<double> Hm((size_t)(restart + 1) * restart), cs(restart), sn(restart), g(restart + 1), y(restart);
  double* hcol = h->hpin;          // pinned: restart + 2 values
  double* ycoef = h->hpin + 1032;  // pinned: restart values
  auto host_scalar = [&](double* out) -> irk_status {
    HIPCHK(hipMemcpyAsync(out, h->scal, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return IRK_OK;
  };
  CHK(residual(h, fl, h->kF, h->kx, h->kr, s));
  HIPCHK(k::dot(h->kr, h->kr, N, h->partials, h->scal, s, 1));
  double beta0;
  CHK(host_scalar(&beta0));
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
    CHK(residual(h, fl, h->kF, h->kx, h->kr, s));
    HIPCHK(k::dot(h->kr, h->kr, N, h->partials, h->scal, s, 1));
    double beta;
    CHK(host_scalar(&beta));
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
      hipEvent_t ea = h->ev[(j & 1) ? 4 : 2], eb = h->ev[(j & 1) ? 5 : 3];
      if (!z_ready) {
        HIPCHK(hipEventRecord(ea, s));
        CHK(precondition(h, vj, zj, s));
        HIPCHK(hipEventRecord(eb, s));
      }
      CHK(residual(h, fl, nullptr, zj, vn, s));
      HIPCHK(k::mgs_arnoldi(vn, h->kv, N, j, h->partials, h->hbuf, s));
      HIPCHK(hipMemcpyAsync(hcol, h->hbuf, (j + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipEventRecord(h->ev[6], s));
      // the next V-cycle needs only v_{j+1}: started before the host reads column j when
      // the last contraction, applied once more, leaves the estimate above kSpecMargin
      // tolerances (the iterates are the same either way)
      bool spec = false;
      if (j + 1 < restart && its + 1 < maxit && res_prev > 0.0) {
        const double rho = std::min(1.0, res_cur / res_prev);
        spec = res_cur * rho > kSpecMargin * rtol * beta0;
      }
      if (spec) {
        HIPCHK(hipEventRecord(h->ev[(j & 1) ? 2 : 4], s));
        CHK(precondition(h, vn, h->kz + (size_t)(j + 1) * N, s));
        HIPCHK(hipEventRecord(h->ev[(j & 1) ? 3 : 5], s));
      }
      HIPCHK(hipEventSynchronize(h->ev[6]));
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
    // x += Z y in one pass (coefficients through the pinned buffer into the device column
    // buffer, free until the next cycle's Arnoldi step)
    std::copy(y.begin(), y.begin() + jend, ycoef);
    HIPCHK(hipMemcpyAsync(h->hbuf, ycoef, (size_t)jend * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(k::update_sum(h->kx, h->kz, N, h->hbuf, jend, s));
    if (std::fabs(g[jend]) <= rtol * beta0) converged = true;
  }
  HIPCHK(k::project_pressure(L.pv, h->kx, h->partials, s));
  CHK(residual(h, fl, h->kF, h->kx, h->kr, s));
  HIPCHK(k::dot(h->kr, h->kr, N, h->partials, h->scal, s, 1));
  double fin;
  CHK(host_scalar(&fin));
  HIPCHK(hipEventRecord(h->ev[1], s));
  HIPCHK(hipEventSynchronize(h->ev[1]));
  float ms_t = 0;
  HIPCHK(hipEventElapsedTime(&ms_t, h->ev[0], h->ev[1]));
  if (info) {
    info->iterations = its;
    info->converged = converged ? 1 : 0;
    info->rel_residual = beta0 > 0 ? fin / beta0 : 0.0;
    info->ms_vcycle = ms_v;
    info->ms_total = ms_t;
  }
  if (!std::isfinite(fin)) return fail(IRK_ENAN, "non-finite final residual");
  if (!converged) return fail(IRK_ENOCONV, "FGMRES reached maxit");
  return IRK_OK;
}

// ----------------------------------------------------------------------------- setup
// Factored form: for each block of the stage eigenbasis (one real eigenvalue or one
// complex pair), the 1- or 2-stage block matrix I (x) M_v + dt T_b (x) S_v of a chunk of
// patches is inverted densely into a temporary buffer, and its first block column is
// copied into the factored layout; chunks keep the temporary under 2 GiB.
irk_status factor_blocks(irk_mhd* h, const DevLevel& V, const DevOps<double>& ops, const std::vector<int32_t>& nloc,
                         int max_ns, hipStream_t s) {
  const StageEig& E = h->eig;
  const int r = h->r, VEC = 2;
  const int64_t np = V.npatch;
  const int64_t budget = ((int64_t)2 << 30) / (int64_t)sizeof(double);
  for (int b = 0; b < E.nblk; ++b) {
    const int m = E.type[b];
    std::vector<int32_t> tld(np);
    std::vector<int64_t> toff(np + 1, 0);
    for (int64_t p = 0; p < np; ++p) {
      const int n = m * (nloc[p] / r);
      tld[p] = (n + VEC - 1) / VEC * VEC;
      toff[p + 1] = toff[p] + (int64_t)tld[p] * n;
    }
    int64_t chunk_max = 0;
    for (int64_t p0 = 0; p0 < np;) {
      int64_t p1 = p0 + 1;
      while (p1 < np && toff[p1 + 1] - toff[p0] <= budget) ++p1;
      chunk_max = std::max(chunk_max, toff[p1] - toff[p0]);
      p0 = p1;
    }
    int32_t* d_tld = nullptr;
    int64_t* d_toff = nullptr;
    double* tmp = nullptr;
    auto release = [&]() {
      (void)hipStreamSynchronize(s);
      if (d_tld) (void)hipFree(d_tld);
      if (d_toff) (void)hipFree(d_toff);
      if (tmp) (void)hipFree(tmp);
    };
    if (hipMalloc(&d_tld, np * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&d_toff, (np + 1) * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&tmp, (size_t)chunk_max * sizeof(double)) != hipSuccess) {
      release();
      return fail(IRK_ENOMEM, "device allocation of the factorisation workspace failed");
    }
    hipError_t e = hipMemcpyAsync(d_tld, tld.data(), np * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_toff, toff.data(), (np + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s);
    for (int64_t p0 = 0; e == hipSuccess && p0 < np;) {
      int64_t p1 = p0 + 1;
      while (p1 < np && toff[p1 + 1] - toff[p0] <= budget) ++p1;
      e = k::patch_factor_scalar<double>(V, ops, m, E.Tb[b], h->dt, d_tld, d_toff, tmp, p0, p1, toff[p0],
                                         m * max_ns, h->flag, s);
      if (e == hipSuccess) e = k::eig_extract<double>(V, V.sb64, b, d_tld, d_toff, toff[p0], tmp, p0, p1, s);
      p0 = p1;
    }
    release();
    if (e != hipSuccess) return fail(IRK_EHIP, std::string("patch factorisation: ") + hipGetErrorString(e));
  }
  return IRK_OK;
}

irk_status build_device_level(irk_mhd* h, MhdHost& H, int l, hipStream_t s) {
  MhdDev& D = h->dev[l];
  const int r = h->r;
  D.ns = H.ns;
  D.N = H.ns * r;
  const int64_t off[5] = {0, H.nfree, H.off_B, H.off_p, H.off_g};
  std::copy(off, off + 5, D.off);
  if (D.N > INT32_MAX) return fail(IRK_EINVAL, "problem too large for 32-bit indices");
  {
    Sell Sl = build_sell(H.ns, H.ptr, H.col);
    D.nsl = Sl.nslices;
    CHK(upload(h, &D.sl_off, Sl.off, s));
    CHK(upload(h, &D.sl_w, Sl.w, s));
    CHK(upload(h, &D.sl_col, Sl.col, s));
    CHK(upload(h, &D.sl_m, sell_values(Sl, H.mval, 1), s));
    CHK(upload(h, &D.sl_s, sell_values(Sl, H.sval, 1), s));
  }
  DevLevel& V = D.pv;
  V.dim = 1;
  V.r = r;
  V.N = D.N;
  V.nv = H.nv;
  V.offV = H.off_p * r;
  for (double** b : {&D.b, &D.x, &D.res}) CHK(dalloc(h, b, (size_t)D.N));
  if (h->smoother == 1 && l > 0) CHK(dalloc(h, &D.dch, (size_t)D.N));
  // residual: column index and two values per operator entry, x, F read and y written
  D.alg_bytes[1] = (double)H.col.size() * (4 + 2 * 8) + 3.0 * 8 * (double)D.N;
  if (l == 0) return IRK_OK;
  // transfers
  {
    std::vector<int32_t> tp, tc;
    std::vector<double> tv;
    const int64_t nsc = h->dev[l - 1].ns;
    fe_transpose_csr(H.ns, nsc, H.P_ptr, H.P_col, H.P_val, tp, tc, tv);
    CHK(upload(h, &D.P_ptr, H.P_ptr, s));
    CHK(upload(h, &D.P_col, H.P_col, s));
    CHK(upload(h, &D.P_val, H.P_val, s));
    CHK(upload(h, &D.Pt_ptr, tp, s));
    CHK(upload(h, &D.Pt_col, tc, s));
    CHK(upload(h, &D.Pt_val, tv, s));
  }
  // patches: sizes, storage, local -> internal index, the slots each unknown gathers
  const int64_t np = H.nv;
  const int VEC = 2;
  const int64_t kLine = 16;  // 128-byte lines of doubles
  std::vector<int32_t> nloc(np), ld(np), gidx, gptr(D.N + 1, 0), gslot, pn_ptr(np + 1, 0);
  std::vector<int64_t> inv_off(np), slot_off(np);
  int64_t io = 0, so = 0;
  int maxn = 0;
  const int pform = h->pform;
  for (int64_t p = 0; p < np; ++p) {
    const int nsp = H.pptr[p + 1] - H.pptr[p];
    const int n = r * nsp;
    nloc[p] = n;
    inv_off[p] = io;
    if (pform == 1) {
      // n_s columns, each the concatenation of the eigen-blocks' rows
      int lc = 0;
      for (int b = 0; b < h->eig.nblk; ++b) lc += irk::eig_block_rows(h->eig.type[b], nsp, VEC);
      ld[p] = lc;
      io += (int64_t)lc * nsp;
    } else {
      ld[p] = (n + VEC - 1) / VEC * VEC;
      io += (int64_t)ld[p] * n;
    }
    slot_off[p] = so;
    so = (so + n + kLine - 1) / kLine * kLine;
    maxn = std::max(maxn, n);
    pn_ptr[p + 1] = pn_ptr[p] + nsp - 1;  // the factor kernel's node count: n_s - 1
    for (int st = 0; st < r; ++st)
      for (int a = 0; a < nsp; ++a) gidx.push_back((int32_t)((int64_t)H.pdof[H.pptr[p] + a] * r + st));
    gidx.resize(so, -1);
  }
  if (maxn > 1024) return fail(IRK_EINVAL, "patch of " + std::to_string(maxn) + " unknowns exceeds the limit of 1024");
  if (so > INT32_MAX) return fail(IRK_EINVAL, "problem too large for 32-bit patch indices");
  for (int32_t g : gidx)
    if (g >= 0) gptr[g + 1]++;
  for (int64_t g = 0; g < D.N; ++g) gptr[g + 1] += gptr[g];
  gslot.resize(gptr.back());
  std::vector<int32_t> fillp(gptr.begin(), gptr.end() - 1);
  // the patch kernels write local unknown e = s n_s + q to slot q r + s
  for (int64_t p = 0; p < np; ++p) {
    const int n = nloc[p], nsp = n / r;
    for (int e = 0; e < n; ++e) {
      const int st = e / nsp, q = e - st * nsp;
      const int64_t g = gidx[slot_off[p] + e];
      gslot[fillp[g]++] = (int32_t)(slot_off[p] + q * r + st);
    }
  }
  std::vector<double> W(D.N, 1.0);
  for (int64_t g = 0; g < D.N; ++g) {
    const int cnt = gptr[g + 1] - gptr[g];
    if (cnt == 0) return fail(IRK_EINVAL, "an unknown is covered by no patch");
    W[g] = h->weighting ? 1.0 / cnt : 1.0;
  }
  {
    Sell G = build_sell(D.N, gptr, gslot);
    for (size_t e = 0; e < G.col.size(); ++e)
      if (G.src[e] < 0) G.col[e] = (int32_t)so;  // the zero slot
    V.nsl_g = G.nslices;
    CHK(upload(h, &V.g_off, G.off, s));
    CHK(upload(h, &V.g_w, G.w, s));
    CHK(upload(h, &V.g_slot, G.col, s));
  }
  {
    // patch apply: every stored inverse once, the residual once, the patch outputs;
    // gather update: the slots with their indices, x read and written, the weights
    // (stored values: (r n_s)^2 dense, r n_s^2 factored)
    double sum_n = 0, sum_n2 = 0;
    for (int64_t p = 0; p < np; ++p) {
      sum_n += nloc[p];
      sum_n2 += pform == 1 ? (double)nloc[p] * nloc[p] / r : (double)nloc[p] * nloc[p];
    }
    D.alg_bytes[0] = 8.0 * (sum_n2 + (double)D.N + sum_n);
    D.alg_bytes[2] = sum_n * (8 + 4) + 3.0 * 8 * (double)D.N;
  }
  std::vector<int32_t> sched(np);
  std::iota(sched.begin(), sched.end(), 0);
  std::stable_sort(sched.begin(), sched.end(), [&](int32_t a, int32_t b) { return nloc[a] > nloc[b]; });
  V.npatch = np;
  V.pform = pform;
  if (pform == 1) {
    const StageEig& E = h->eig;
    V.sb64.r = r;
    V.sb64.nblk = E.nblk;
    for (int b = 0; b < E.nblk; ++b) {
      V.sb64.type[b] = E.type[b];
      V.sb64.st0[b] = E.st0[b];
    }
    for (int i = 0; i < r * r; ++i) {
      V.sb64.W[i] = E.W[i];
      V.sb64.Winv[i] = E.Winv[i];
    }
  }
  V.max_nloc = maxn;
  V.max_ld = *std::max_element(ld.begin(), ld.end());
  V.inv_elems = io;
  V.slots = so;
  CHK(upload(h, &V.p_nloc, nloc, s));
  CHK(upload(h, &V.p_ld, ld, s));
  CHK(upload(h, &V.p_inv_off, inv_off, s));
  CHK(upload(h, &V.p_slot_off, slot_off, s));
  CHK(upload(h, &V.p_gidx, gidx, s));
  CHK(upload(h, &V.sched, sched, s));
  CHK(upload(h, &V.pn_ptr, pn_ptr, s));
  CHK(upload(h, &V.pvv_ptr, H.pvv_ptr, s));
  CHK(upload(h, &V.pvv, H.pvv, s));
  CHK(upload(h, &V.pvp, std::vector<int32_t>(std::max<int64_t>(1, pn_ptr[np]), -1), s));
  CHK(upload(h, &D.ops.W, W, s));
  // the factor kernels read M and S at the operator's CSR positions
  CHK(upload(h, &D.ops.s_M, H.mval, s));
  CHK(upload(h, &D.ops.s_L, H.sval, s));
  double* inv;
  CHK(dalloc(h, &inv, (size_t)io));
  V.inv = inv;
  // one extra slot at the end, zero: the sliced gather's padding entries point at it
  CHK(dalloc(h, &D.Y, (size_t)so + 1));
  HIPCHK(hipMemsetAsync(D.Y, 0, (so + 1) * sizeof(double), s));
  HIPCHK(hipMemsetAsync(h->flag, 0, sizeof(int), s));
  if (pform == 0) {
    HIPCHK(k::patch_factor_scalar<double>(V, D.ops, r, h->A, h->dt, V.p_ld, V.p_inv_off, inv, 0, np, 0, maxn,
                                          h->flag, s));
  } else {
    CHK(factor_blocks(h, V, D.ops, nloc, maxn / r, s));
  }
  int fl = 0;
  HIPCHK(hipMemcpyAsync(&fl, h->flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (fl) return fail(IRK_ESINGULAR, "zero pivot in a patch of level " + std::to_string(l));
  return IRK_OK;
}

// Host part of the setup: topology, index maps and transfers of every level, and the
// linearisation state on every level (ws, bs); the operators are assembled per level.
irk_status build_host(const irk_mesh_level* lv, int nlevels, const double* w, const double* b0,
                      std::vector<MhdHost>& host, std::vector<std::vector<double>>& ws,
                      std::vector<std::vector<double>>& bs) {
  host.assign(nlevels, MhdHost());
  for (int l = 0; l < nlevels; ++l) {
    build_topology(host[l].L, 2, lv[l].nverts, lv[l].ncells, lv[l].xyz, lv[l].cells);
    mhd_index(host[l]);
  }
  for (int l = 1; l < nlevels; ++l) {
    std::string e = build_transfer(host[l - 1].L, host[l].L, lv[l].parent);
    if (e.empty()) e = mhd_transfer(host[l - 1], host[l], lv[l].parent);
    if (!e.empty()) return fail(IRK_EINVAL, "level " + std::to_string(l) + ": " + e);
  }
  const HostLevel& Lf = host[nlevels - 1].L;
  for (int64_t i = 0; i < Lf.nn * 2; ++i)
    if (!std::isfinite(w[i])) return fail(IRK_EINVAL, "non-finite value in w");
  for (int64_t i = 0; i < Lf.ne; ++i)
    if (!std::isfinite(b0[i])) return fail(IRK_EINVAL, "non-finite value in b0");
  ws.assign(nlevels, {});
  bs.assign(nlevels, {});
  ws[nlevels - 1].assign(w, w + Lf.nn * 2);
  bs[nlevels - 1].assign(b0, b0 + Lf.ne);
  for (int l = nlevels - 2; l >= 0; --l)
    mhd_coarsen_state(host[l], host[l + 1], ws[l + 1].data(), bs[l + 1].data(), ws[l], bs[l]);
  return IRK_OK;
}

irk_status check_meshes(const irk_mesh_level* lv, int nlevels) {
  if (!lv || nlevels < 1 || nlevels > 16) return fail(IRK_EINVAL, "need 1..16 mesh levels");
  for (int l = 0; l < nlevels; ++l) {
    const irk_mesh_level& m = lv[l];
    if (m.dim != 2) return fail(IRK_EINVAL, "the MHD solver takes triangle meshes (dim 2)");
    if (m.nverts < 3 || m.ncells < 1 || !m.xyz || !m.cells)
      return fail(IRK_EINVAL, "level " + std::to_string(l) + ": empty mesh or null arrays");
    if (m.nverts > (1LL << 30) || m.ncells > (1LL << 30)) return fail(IRK_EINVAL, "mesh too large");
    if (l > 0 && !m.parent) return fail(IRK_EINVAL, "level " + std::to_string(l) + ": parent is NULL");
    if (l > 0 && m.ncells != lv[l - 1].ncells * 4)
      return fail(IRK_EINVAL, "level " + std::to_string(l) + " is not a uniform refinement of level " +
                                  std::to_string(l - 1));
    for (int64_t i = 0; i < m.ncells * 3; ++i)
      if (m.cells[i] < 0 || m.cells[i] >= m.nverts)
        return fail(IRK_EINVAL, "level " + std::to_string(l) + ": vertex index out of range");
    for (int64_t i = 0; i < m.nverts * 2; ++i)
      if (!std::isfinite(m.xyz[i])) return fail(IRK_EINVAL, "non-finite coordinate");
    if (l > 0)
      for (int64_t c = 0; c < m.ncells; ++c)
        if (m.parent[c] < 0 || m.parent[c] >= lv[l - 1].ncells)
          return fail(IRK_EINVAL, "level " + std::to_string(l) + ": parent index out of range");
  }
  return IRK_OK;
}

irk_status setup_impl(const irk_mesh_level* lv, int nlevels, const irk_tableau* tab, double dt, double Re,
                      double Rem, const double* w, const double* b0, hipStream_t s, irk_mhd* h) {
  const int r = tab->r;
  std::vector<MhdHost> host;
  std::vector<std::vector<double>> ws, bs;
  CHK(build_host(lv, nlevels, w, b0, host, ws, bs));
  HIPCHK(hipMalloc((void**)&h->flag, sizeof(int)));
  h->allocations.push_back(h->flag);
  CHK(dalloc(h, &h->partials, 1024));
  CHK(dalloc(h, &h->scal, 4));
  for (auto& e : h->ev) HIPCHK(hipEventCreate(&e));
  HIPCHK(hipHostMalloc((void**)&h->hpin, 2 * 1032 * sizeof(double), hipHostMallocDefault));
  h->dev.resize(nlevels);
  for (int l = 0; l < nlevels; ++l) {
    MhdHost& H = host[l];
    assemble_level(H.L, 1.0, nullptr, false);
    mhd_assemble(H, Re, Rem, ws[l].data(), bs[l].data());
    if (l >= 1) mhd_patches(H);
    CHK(build_device_level(h, H, l, s));
    if (l == 0) {
      // coarse operator, column-major; Gauss--Jordan on the column-major storage inverts
      // the transpose, which is the inverse stored column-major
      std::vector<double> Jc;
      double mx = 0;
      mhd_coarse_matrix(H, r, h->A, dt, Jc, &mx);
      const int64_t N0 = h->dev[0].N;
      CHK(upload(h, &h->cmat, Jc, s));
      CHK(upload(h, &h->cinv, Jc, s));
      double* colk;
      int64_t* swp;
      CHK(dalloc(h, &colk, (size_t)N0));
      CHK(dalloc(h, &swp, (size_t)N0));
      HIPCHK(hipMemsetAsync(h->flag, 0, sizeof(int), s));
      HIPCHK(k::dense_inverse(h->cinv, N0, std::max(1e-300, 1e-14 * mx), colk, swp, h->flag, s));
      int fl = 0;
      HIPCHK(hipMemcpyAsync(&fl, h->flag, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (fl) return fail(IRK_ESINGULAR, "singular coarse operator");
      CHK(dalloc(h, &h->cpart, (size_t)N0 * k::coarse_split()));
      std::vector<int64_t> pins(r);
      for (int st = 0; st < r; ++st) pins[st] = H.off_p * r + st;
      CHK(upload(h, &h->pins, pins, s));
    }
    // the host copies of the finished level are no longer needed
    H = MhdHost();
  }
  HIPCHK(hipStreamSynchronize(s));
  return IRK_OK;
}

irk_status check(const irk_mhd* h) {
  if (!h || h->nlevels < 1) return fail(IRK_EINVAL, "null or empty handle");
  return IRK_OK;
}

irk_status level_of(const irk_mhd* h, int& level, bool fine_only) {
  if (level == -1) level = h->nlevels - 1;
  if (level < (fine_only ? 1 : 0) || level >= h->nlevels)
    return fail(IRK_EINVAL, fine_only ? "level must be in 1..nlevels-1" : "level out of range");
  return IRK_OK;
}

}  // namespace

extern "C" {

void irk_mhd_default_opts(irk_mhd_opts* opt) {
  if (!opt) return;
  opt->pre = 2;
  opt->post = 2;
  opt->omega = 0.5;
  opt->weighting = 1;
  opt->patch_form = 2;
  opt->smoother = 0;
  opt->cheb_lo = 2.0;
  opt->cheb_hi = 10.0;
}

irk_status irk_mhd_setup(const irk_mesh_level* lv, int nlevels, const irk_tableau* tab, double dt, double Re,
                         double Rem, const double* w, const double* b0, const irk_mhd_opts* opt, void* stream,
                         irk_mhd** out) {
  if (!out) return fail(IRK_EINVAL, "out is NULL");
  *out = nullptr;
  if (!tab || tab->r < 1 || tab->r > kMaxStages || !tab->A) return fail(IRK_EINVAL, "tableau must have 1 <= r <= 4");
  for (int i = 0; i < tab->r * tab->r; ++i)
    if (!std::isfinite(tab->A[i])) return fail(IRK_EINVAL, "non-finite tableau entry");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(IRK_EINVAL, "dt must be positive and finite");
  if (!(Re > 0) || !std::isfinite(Re) || !(Rem > 0) || !std::isfinite(Rem))
    return fail(IRK_EINVAL, "Re and Rem must be positive and finite");
  if (!w || !b0) return fail(IRK_EINVAL, "w and b0 are required");
  irk_mhd_opts o;
  irk_mhd_default_opts(&o);
  if (opt) o = *opt;
  if (o.pre < 0 || o.post < 0 || o.pre > 64 || o.post > 64) return fail(IRK_EINVAL, "sweep counts must be in 0..64");
  if (!(o.omega > 0) || !std::isfinite(o.omega)) return fail(IRK_EINVAL, "omega must be positive");
  if (o.weighting != 0 && o.weighting != 1) return fail(IRK_EINVAL, "weighting must be 0 or 1");
  if (o.patch_form < 0 || o.patch_form > 2) return fail(IRK_EINVAL, "patch_form must be 0, 1 or 2");
  if (o.smoother != 0 && o.smoother != 1) return fail(IRK_EINVAL, "smoother must be 0 or 1");
  if (o.smoother == 1 && !(o.cheb_lo > 0 && o.cheb_hi > o.cheb_lo && std::isfinite(o.cheb_hi)))
    return fail(IRK_EINVAL, "Chebyshev interval must satisfy 0 < cheb_lo < cheb_hi < inf");
  CHK(check_meshes(lv, nlevels));
  irk_mhd* h = new (std::nothrow) irk_mhd();
  if (!h) return fail(IRK_ENOMEM, "handle allocation failed");
  h->r = tab->r;
  h->nlevels = nlevels;
  h->dt = dt;
  std::copy(tab->A, tab->A + tab->r * tab->r, h->A);
  h->pre = o.pre;
  h->post = o.post;
  h->omega = o.omega;
  h->weighting = o.weighting;
  h->smoother = o.smoother;
  h->cheb_lo = o.cheb_lo;
  h->cheb_hi = o.cheb_hi;
  {
    std::string why;
    const bool ok = o.patch_form != 0 && stage_eigenbasis(h->A, h->r, h->eig, &why);
    if (o.patch_form == 1 && !ok) {
      delete h;
      return fail(IRK_EINVAL, "factored patch form unavailable: " + why);
    }
    h->pform = ok && (o.patch_form == 1 || h->r >= 2) ? 1 : 0;
  }
  irk_status st;
  try {
    st = setup_impl(lv, nlevels, tab, dt, Re, Rem, w, b0, S(stream), h);
  } catch (const std::bad_alloc&) {
    st = fail(IRK_ENOMEM, "host allocation failed during setup");
  } catch (const std::exception& e) {
    st = fail(IRK_EINVAL, std::string("setup failed: ") + e.what());
  }
  if (st != IRK_OK) {
    irk_mhd_destroy(h);
    return st;
  }
  *out = h;
  return IRK_OK;
}

irk_status irk_mhd_host_operators(const irk_mesh_level* lv, int nlevels, int level, double Re, double Rem,
                                  const double* w, const double* b0, int64_t* sizes, int32_t* ptr, int32_t* col,
                                  double* mval, double* sval, int32_t* P_ptr, int32_t* P_col, double* P_val) {
  CHK(check_meshes(lv, nlevels));
  if (level == -1) level = nlevels - 1;
  if (level < 0 || level >= nlevels) return fail(IRK_EINVAL, "level out of range");
  if (!(Re > 0) || !std::isfinite(Re) || !(Rem > 0) || !std::isfinite(Rem))
    return fail(IRK_EINVAL, "Re and Rem must be positive and finite");
  if (!w || !b0 || !sizes) return fail(IRK_EINVAL, "w, b0 and sizes are required");
  try {
    std::vector<MhdHost> host;
    std::vector<std::vector<double>> ws, bs;
    CHK(build_host(lv, nlevels, w, b0, host, ws, bs));
    MhdHost& H = host[level];
    assemble_level(H.L, 1.0, nullptr, false);
    mhd_assemble(H, Re, Rem, ws[level].data(), bs[level].data());
    const int64_t nnzP = level > 0 ? (int64_t)H.P_col.size() : 0;
    const int64_t want[4] = {H.ns, (int64_t)H.col.size(), nnzP, level > 0 ? host[level - 1].ns : 0};
    const bool fill = ptr != nullptr;
    if (fill) {
      for (int i = 0; i < 4; ++i)
        if (sizes[i] != want[i]) return fail(IRK_EINVAL, "sizes do not match the first call's");
      if (!col || !mval || !sval || (level > 0 && (!P_ptr || !P_col || !P_val)))
        return fail(IRK_EINVAL, "null output array");
      std::copy(H.ptr.begin(), H.ptr.end(), ptr);
      std::copy(H.col.begin(), H.col.end(), col);
      std::copy(H.mval.begin(), H.mval.end(), mval);
      std::copy(H.sval.begin(), H.sval.end(), sval);
      if (level > 0) {
        std::copy(H.P_ptr.begin(), H.P_ptr.end(), P_ptr);
        std::copy(H.P_col.begin(), H.P_col.end(), P_col);
        std::copy(H.P_val.begin(), H.P_val.end(), P_val);
      }
    }
    std::copy(want, want + 4, sizes);
  } catch (const std::bad_alloc&) {
    return fail(IRK_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(IRK_EINVAL, std::string("assembly failed: ") + e.what());
  }
  return IRK_OK;
}

irk_status irk_mhd_profile(irk_mhd* h, int enable) {
  CHK(check(h));
  if (enable < 0 || enable > 2) return fail(IRK_EINVAL, "profile mode must be 0..2");
  h->prof = enable;
  h->prof_used = 0;
  return IRK_OK;
}

irk_status irk_mhd_kernel_stats(irk_mhd* h, int kernel, int level, irk_kernel_stats* out) {
  CHK(check(h));
  CHK(level_of(h, level, false));
  if (!out || kernel < 0 || kernel > 2) return fail(IRK_EINVAL, "kernel must be 0..2 and out non-NULL");
  out->launches = 0;
  out->ms_total = 0;
  out->bytes_per_launch = h->dev[level].alg_bytes[kernel];
  for (size_t i = 0; i < h->prof_used; ++i) {
    ProfEv& e = h->prof_pool[i];
    if (e.kernel != kernel || e.level != level) continue;
    HIPCHK(hipEventSynchronize(e.b));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e.a, e.b));
    out->launches++;
    out->ms_total += ms;
  }
  return IRK_OK;
}

void irk_mhd_destroy(irk_mhd* h) {
  if (!h) return;
  for (auto& e : h->prof_pool) {
    if (e.a) (void)hipEventDestroy(e.a);
    if (e.b) (void)hipEventDestroy(e.b);
  }
  for (void* p : h->allocations) (void)hipFree(p);
  for (auto& e : h->ev)
    if (e) (void)hipEventDestroy(e);
  if (h->hpin) (void)hipHostFree(h->hpin);
  delete h;
}

int irk_mhd_patch_form(const irk_mhd* h) { return h ? h->pform : -1; }

int64_t irk_mhd_ndofs(const irk_mhd* h, int level) {
  if (!h) return -1;
  if (level == -1) level = h->nlevels - 1;
  if (level < 0 || level >= h->nlevels) return -1;
  return h->dev[level].N;
}

irk_status irk_mhd_layout(const irk_mhd* h, int level, int64_t* out) {
  CHK(check(h));
  CHK(level_of(h, level, false));
  if (!out) return fail(IRK_EINVAL, "null output");
  for (int i = 0; i < 5; ++i) out[i] = h->dev[level].off[i];
  out[5] = h->dev[level].ns;
  out[6] = h->r;
  return IRK_OK;
}

irk_status irk_mhd_apply(irk_mhd* h, int level, const double* x, double* y, void* stream) {
  CHK(check(h));
  CHK(level_of(h, level, false));
  if (!x || !y) return fail(IRK_EINVAL, "null vector");
  MhdDev& D = h->dev[level];
  hipStream_t s = S(stream);
  HIPCHK(k::stage_to_internal(D.ns, h->r, x, D.b, s));
  CHK(residual(h, level, nullptr, D.b, D.res, s));
  HIPCHK(k::stage_to_abi(D.ns, h->r, D.res, y, s));
  return IRK_OK;
}

irk_status irk_mhd_sweep(irk_mhd* h, int level, const double* F, double* kk, void* stream) {
  CHK(check(h));
  CHK(level_of(h, level, true));
  if (!F || !kk) return fail(IRK_EINVAL, "null vector");
  MhdDev& D = h->dev[level];
  hipStream_t s = S(stream);
  HIPCHK(k::stage_to_internal(D.ns, h->r, F, D.b, s));
  HIPCHK(k::stage_to_internal(D.ns, h->r, kk, D.x, s));
  CHK(relax(h, level, D.b, D.x, 1, false, s));
  HIPCHK(k::stage_to_abi(D.ns, h->r, D.x, kk, s));
  return IRK_OK;
}

irk_status irk_mhd_restrict(irk_mhd* h, int level, const double* xf, double* xc, void* stream) {
  CHK(check(h));
  CHK(level_of(h, level, true));
  if (!xf || !xc) return fail(IRK_EINVAL, "null vector");
  MhdDev &D = h->dev[level], &C = h->dev[level - 1];
  hipStream_t s = S(stream);
  HIPCHK(k::stage_to_internal(D.ns, h->r, xf, D.res, s));
  HIPCHK(k::kron_csr(C.ns, D.Pt_ptr, D.Pt_col, D.Pt_val, h->r, D.res, C.b, 0, s));
  HIPCHK(k::stage_to_abi(C.ns, h->r, C.b, xc, s));
  return IRK_OK;
}

irk_status irk_mhd_prolong(irk_mhd* h, int level, const double* xc, double* xf, void* stream) {
  CHK(check(h));
  CHK(level_of(h, level, true));
  if (!xf || !xc) return fail(IRK_EINVAL, "null vector");
  MhdDev &D = h->dev[level], &C = h->dev[level - 1];
  hipStream_t s = S(stream);
  HIPCHK(k::stage_to_internal(C.ns, h->r, xc, C.x, s));
  HIPCHK(k::stage_to_internal(D.ns, h->r, xf, D.x, s));
  HIPCHK(k::kron_csr(D.ns, D.P_ptr, D.P_col, D.P_val, h->r, C.x, D.x, 1, s));
  HIPCHK(k::stage_to_abi(D.ns, h->r, D.x, xf, s));
  return IRK_OK;
}

irk_status irk_mhd_coarse_solve(irk_mhd* h, const double* b, double* x, void* stream) {
  CHK(check(h));
  if (!b || !x) return fail(IRK_EINVAL, "null vector");
  MhdDev& D = h->dev[0];
  hipStream_t s = S(stream);
  HIPCHK(k::stage_to_internal(D.ns, h->r, b, D.b, s));
  CHK(coarse(h, D.b, D.x, s));
  HIPCHK(k::stage_to_abi(D.ns, h->r, D.x, x, s));
  return IRK_OK;
}

irk_status irk_mhd_vcycle(irk_mhd* h, const double* r, double* z, void* stream) {
  CHK(check(h));
  if (!r || !z) return fail(IRK_EINVAL, "null vector");
  if (r == z) return fail(IRK_EINVAL, "r and z may not alias");
  CHK(ensure_krylov(h, 1));
  MhdDev& D = h->dev[h->nlevels - 1];
  hipStream_t s = S(stream);
  HIPCHK(k::stage_to_internal(D.ns, h->r, r, h->kv, s));
  CHK(precondition(h, h->kv, h->kz, s));
  HIPCHK(k::stage_to_abi(D.ns, h->r, h->kz, z, s));
  return IRK_OK;
}

irk_status irk_mhd_fgmres_solve(irk_mhd* h, const double* F, double* kk, double rtol, int maxit, int restart,
                                irk_solve_info* info, void* stream) {
  CHK(check(h));
  if (!F || !kk) return fail(IRK_EINVAL, "null vector");
  if (!(rtol > 0) || maxit < 1 || restart < 1 || restart > 1000)
    return fail(IRK_EINVAL, "rtol must be > 0, maxit >= 1, 1 <= restart <= 1000");
  CHK(ensure_krylov(h, restart));
  MhdDev& D = h->dev[h->nlevels - 1];
  if (!h->kF) {
    CHK(dalloc(h, &h->kF, (size_t)D.N));
    CHK(dalloc(h, &h->kx, (size_t)D.N));
    CHK(dalloc(h, &h->kr, (size_t)D.N));
  }
  hipStream_t s = S(stream);
  HIPCHK(hipEventRecord(h->ev[0], s));
  HIPCHK(k::stage_to_internal(D.ns, h->r, F, h->kF, s));
  HIPCHK(k::stage_to_internal(D.ns, h->r, kk, h->kx, s));
  irk_status st = fgmres(h, rtol, maxit, restart, info, s);
  if (st == IRK_OK || st == IRK_ENOCONV) HIPCHK(k::stage_to_abi(D.ns, h->r, h->kx, kk, s));
  return st;
}

}  // extern "C"
