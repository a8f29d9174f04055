// Many independent stage systems solved by FGMRES + Vanka V-cycle in ONE persistent
// kernel launch.
//
// Every solve is a state machine in device memory whose states are the steps of the
// method: layout load, residual, norms, the V-cycle's sweeps (residual, patch apply,
// owner gather), restriction, coarse solve, prolongation, pressure projection, the
// Arnoldi/MGS steps, the Givens update and the solution update.  A state is split into
// work items (chunks of rows, patches or vector entries).  Resident workgroups loop
// over the solves, take one item at a time with a 64-bit ticket (epoch << 32 | item),
// execute it, and count it done; the workgroup that completes the last item of a state
// finishes its reductions in a fixed order and moves the solve to its next state.  The
// sizes of the work items and the number of resident workgroups are the tunable
// schedule (chosen by timing trial runs when autotuning is on).
//
// Every wait is bounded: a workgroup that polls too long without finding work raises
// the abort flag, and every workgroup leaves the loop once all solves are finished or
// the flag is set.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <atomic>
#include <chrono>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "../../include/irk_mg.h"
#include "device_ops.h"
#include "irk_internal.h"

namespace irk {
namespace batch {

constexpr int kBlock = 1024;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxLevels = 12;
constexpr int kMaxRestart = 64;
constexpr int kNmax = 256;
constexpr int kCoarseChunks = 64;  // column chunks of the coarse GEMV (16 items x 4 waves)

// states of a solve
constexpr int PH_LOAD = 0, PH_R0 = 1, PH_N0 = 2, PH_RES = 3, PH_NRM = 4, PH_V0 = 5, PH_VC_IN = 6,
              PH_SM_RES = 7, PH_SM_PATCH = 8, PH_SM_GATHER = 9, PH_ZERO = 10, PH_DN_RES = 11,
              PH_DN_RESTRICT = 12, PH_CO_IN = 13, PH_CO_MV = 14, PH_CO_RED = 15, PH_UP_PROLONG = 16,
              PH_VC_OUT = 17, PH_PJ_SUM = 18, PH_PJ_SUB = 19, PH_AP = 20, PH_DOT = 21, PH_AXPY = 22,
              PH_WNRM = 23, PH_VSCALE = 24, PH_XUPD = 25, PH_FR = 26, PH_FN = 27, PH_STORE = 28,
              PH_DONE = 29;

struct BLevel {
  int64_t nfree, nv, N, offV, npatch;
  int rb;     // row blocks of the patch apply (ceil(max stored column / 128))
  int pform;  // patch form: 0 dense inverse, 1 factored through the stage eigenbasis, 3 symmetric factored
  int dim, r;
  irk::StageBasis<double> sb;
  const int32_t *s_ptr, *s_col, *b_ptr, *b_col, *bt_ptr, *bt_col;
  const double *sM, *sL, *b_val, *bt_val, *W;
  const int32_t *pu_ptr, *pu_col, *put_ptr, *put_col, *pp_ptr, *pp_col, *ppt_ptr, *ppt_col;
  const double *pu_val, *put_val, *pp_val, *ppt_val;
  const int32_t *p_nloc, *p_ld, *sched, *p_gidx, *gat_ptr, *gat_slot;
  const int64_t *p_inv_off, *p_slot_off;
  const double* inv;
  double *b, *x, *res, *Y;
};

struct BSolve {
  int dim, r, nlevels, pre, post, restart, maxit;
  double omega, rtol;
  dev::Coef<double> dtA;
  int64_t ns;  // ABI stage block of the finest level
  BLevel lv[kMaxLevels];
  const double *cinv, *cmat;  // coarse inverse and pinned operator, column-major
  double *cb, *cpart;
  int64_t pins[kMaxStages];
  int64_t N0;
  const double* F_abi;
  double* k_abi;
  double *F, *x, *V, *Z, *w, *rv, *partials;
};

struct BState {
  unsigned long long ticket;  // (epoch << 32) | next item
  unsigned long long meta;    // (epoch << 32) | items of that epoch, published as one word
  int done;                   // items completed over all states (never reset)
  int done_base;              // value of `done` when the current state started
  int epoch, phase, n_items;
  int level, sweep, first, leg, j, i, jend, pj_final;
  int its, converged, status;
  double beta0, beta, final_rel;
  double mean[kMaxStages];
  double H[(kMaxRestart + 1) * kMaxRestart], cs[kMaxRestart], sn[kMaxRestart], g[kMaxRestart + 1],
      y[kMaxRestart];
  unsigned long long t_end;
  int ntrans, last_phase;
};

// the part of a solve's state that a work item reads (copied to LDS per item)
struct BCur {
  int phase, n_items, done_base, level, first, j, i, jend, pj_final, sweep;
  double beta;
  double mean[kMaxStages];
};

struct Ctl {
  int finished, abort;
  unsigned long long t0;
  long long max_idle;
  // on an idle abort: per solve phase, epoch, done, done_base, n_items, ticket item, ticket epoch
  int dbg[16 * 7];
};

struct Tun {
  int rows;   // rows per item / 256
  int ppw;    // patches per wavefront per item
  int elems;  // vector entries per item / 256
};

// state fields are read with device-scope atomic loads so that no cache level can
// serve a value older than the last release
template <typename T>
__device__ __forceinline__ T ald(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void ast(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------ item counts
__host__ __device__ inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

__host__ __device__ int items_of_raw(const BSolve& S, const BState& st, int phase, const Tun& t);
__host__ __device__ int items_of(const BSolve& S, const BState& st, int phase, const Tun& t) {
  return max(1, items_of_raw(S, st, phase, t));
}
__host__ __device__ int items_of_raw(const BSolve& S, const BState& st, int phase, const Tun& t) {
  const BLevel& F = S.lv[S.nlevels - 1];
  const int64_t er = (int64_t)kBlock * t.elems, rr = (int64_t)kBlock * t.rows;
  switch (phase) {
    case PH_LOAD: case PH_N0: case PH_NRM: case PH_V0: case PH_VC_IN: case PH_VC_OUT: case PH_DOT:
    case PH_AXPY: case PH_WNRM: case PH_VSCALE: case PH_XUPD: case PH_STORE: case PH_FN:
      return cdiv(F.N, er);
    case PH_R0: case PH_RES: case PH_AP: case PH_FR:
      return cdiv(F.nfree + F.nv, rr);
    case PH_SM_RES: case PH_DN_RES: {
      const BLevel& L = S.lv[st.level];
      return cdiv(L.nfree + L.nv, rr);
    }
    case PH_SM_PATCH:
      return cdiv(S.lv[st.level].npatch, (int64_t)kWaves * t.ppw);
    case PH_SM_GATHER: case PH_ZERO:
      return cdiv(S.lv[st.level].N, er);
    case PH_DN_RESTRICT: {
      const BLevel& C = S.lv[st.level - 1];
      return cdiv(C.nfree + C.nv, rr);
    }
    case PH_UP_PROLONG: {
      const BLevel& L = S.lv[st.level];
      return cdiv(L.nfree + L.nv, rr);
    }
    case PH_CO_IN: case PH_CO_RED:
      return cdiv(S.N0, er);
    case PH_CO_MV:
      return cdiv(S.N0, 64) * (kCoarseChunks / kWaves);
    case PH_PJ_SUM: case PH_PJ_SUB:
      return cdiv(F.nv, er);
    default:
      return 0;
  }
}

// ------------------------------------------------------------- dispatch helpers
template <int D, int R>
__device__ void resid_rows(const BLevel& L, const dev::Coef<double>& c, const double* F, const double* x,
                           double* y, int64_t r0, int64_t r1) {
  for (int64_t row = r0 + threadIdx.x; row < r1; row += kBlock)
    dev::residual_row<D, R, double>(row, L.nfree, L.nv, L.offV, L.s_ptr, L.s_col, L.sM, L.sL, L.b_ptr, L.b_col,
                                    L.b_val, L.bt_ptr, L.bt_col, L.bt_val, c, F, x, y);
}

__device__ void residual(int D, int R, const BLevel& L, const dev::Coef<double>& c, const double* F,
                         const double* x, double* y, int64_t r0, int64_t r1) {
#define IRK_B_RES(DD, RR) \
  if (D == DD && R == RR) return resid_rows<DD, RR>(L, c, F, x, y, r0, r1);
  IRK_B_RES(2, 1) IRK_B_RES(2, 2) IRK_B_RES(2, 3) IRK_B_RES(2, 4)
#undef IRK_B_RES
}

template <int D, int R>
__device__ void spmv_rows(int64_t nu, int64_t np, int64_t out_offV, int64_t in_offV, const int32_t* up,
                          const int32_t* uc, const double* uv, const int32_t* pp, const int32_t* pc,
                          const double* pv, const double* in, double* out, int add, int64_t r0, int64_t r1) {
  for (int64_t row = r0 + threadIdx.x; row < r1; row += kBlock)
    dev::spmv_nodes_row<D, R, double>(row, nu, np, out_offV, in_offV, up, uc, uv, pp, pc, pv, in, out, add);
}

__device__ void spmv(int D, int R, int64_t nu, int64_t np, int64_t out_offV, int64_t in_offV, const int32_t* up,
                     const int32_t* uc, const double* uv, const int32_t* pp, const int32_t* pc, const double* pv,
                     const double* in, double* out, int add, int64_t r0, int64_t r1) {
#define IRK_B_SP(DD, RR) \
  if (D == DD && R == RR) return spmv_rows<DD, RR>(nu, np, out_offV, in_offV, up, uc, uv, pp, pc, pv, in, out, add, r0, r1);
  IRK_B_SP(2, 1) IRK_B_SP(2, 2) IRK_B_SP(2, 3) IRK_B_SP(2, 4)
#undef IRK_B_SP
}

__device__ void patches(const BLevel& L, double* xs, double* xt, const double* in, int64_t p0, int ppw) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int q = 0; q < ppw; ++q) {
    const int64_t idx = p0 + (int64_t)wave * ppw + q;
    if (idx >= L.npatch) break;
    const int p = L.sched[idx];
    if (L.pform == 3) {
      dev::patch_apply_sym_one<double, 4, 1, 0>(p, lane, xs, xt, L.sb, L.p_nloc, L.p_inv_off, L.p_slot_off, L.p_gidx,
                                             L.inv, in, nullptr, L.Y, 0, L.dim);
      continue;
    }
    if (L.pform == 1) {
      if (L.rb == 1)
        dev::patch_apply_eig_one<double, 1, 4, 1>(p, lane, xs, xt, L.sb, L.p_nloc, L.p_ld, L.p_inv_off, L.p_slot_off,
                                               L.p_gidx, L.inv, in, nullptr, L.Y, 0, L.dim);
      else
        dev::patch_apply_eig_one<double, 2, 4, 1>(p, lane, xs, xt, L.sb, L.p_nloc, L.p_ld, L.p_inv_off, L.p_slot_off,
                                               L.p_gidx, L.inv, in, nullptr, L.Y, 0, L.dim);
      continue;
    }
    switch (L.rb) {
      case 1: dev::patch_apply_one<double, 1, 8>(p, lane, xs, L.p_nloc, L.p_ld, L.p_inv_off, L.p_slot_off, L.p_gidx, L.inv, in, nullptr, L.Y, 0, L.dim, L.r); break;
      case 2: dev::patch_apply_one<double, 2>(p, lane, xs, L.p_nloc, L.p_ld, L.p_inv_off, L.p_slot_off, L.p_gidx, L.inv, in, nullptr, L.Y, 0, L.dim, L.r); break;
      default: dev::patch_apply_one<double, 2>(p, lane, xs, L.p_nloc, L.p_ld, L.p_inv_off, L.p_slot_off, L.p_gidx, L.inv, in, nullptr, L.Y, 0, L.dim, L.r); break;
    }
  }
}

__device__ inline int64_t abi_index(int64_t g, int64_t offV, int64_t nfree, int64_t ns, int D, int R) {
  if (g < offV) {
    const int64_t i = g / (D * R), rem = g - i * D * R;
    const int c = (int)(rem / R), s = (int)(rem - (int64_t)c * R);
    return s * ns + c * nfree + i;
  }
  const int64_t v = (g - offV) / R;
  const int s = (int)(g - offV - v * R);
  return s * ns + D * nfree + v;
}

// block sum of one value per thread (fixed order)
__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}

// ------------------------------------------------------------------ one work item
__device__ void exec_item(const BSolve& S, const BCur& st, const BState* gst, int item, const Tun& t, double* xs,
                          double* xt, double* red) {
  const int D = S.dim, R = S.r, top = S.nlevels - 1;
  const BLevel& Fl = S.lv[top];
  const int64_t N = Fl.N;
  const int64_t er = (int64_t)kBlock * t.elems, rr = (int64_t)kBlock * t.rows;
  const int64_t e0 = (int64_t)item * er, e1 = min(N, e0 + er);
  const int64_t r0 = (int64_t)item * rr;
  const int tid = threadIdx.x;
  switch (st.phase) {
    case PH_LOAD:
      for (int64_t g = e0 + tid; g < e1; g += kBlock) {
        const int64_t a = abi_index(g, Fl.offV, Fl.nfree, S.ns, D, R);
        S.F[g] = S.F_abi[a];
        S.x[g] = S.k_abi[a];
      }
      break;
    case PH_R0: case PH_RES: case PH_FR:
      residual(D, R, Fl, S.dtA, S.F, S.x, S.rv, r0, min(Fl.nfree + Fl.nv, r0 + rr));
      break;
    case PH_AP:
      residual(D, R, Fl, S.dtA, nullptr, S.Z + (int64_t)st.j * N, S.w, r0, min(Fl.nfree + Fl.nv, r0 + rr));
      break;
    case PH_N0: case PH_NRM: case PH_FN: case PH_DOT: case PH_WNRM: {
      const double* a = (st.phase == PH_DOT || st.phase == PH_WNRM) ? S.w : S.rv;
      const double* b = st.phase == PH_DOT ? S.V + (int64_t)st.i * N : a;
      double acc = 0;
      for (int64_t g = e0 + tid; g < e1; g += kBlock) acc += a[g] * b[g];
      const double s = block_sum(acc, red);
      if (tid == 0) S.partials[item] = s;
      break;
    }
    case PH_V0:
      for (int64_t g = e0 + tid; g < e1; g += kBlock) S.V[g] = S.rv[g] / st.beta;
      break;
    case PH_VC_IN:
      for (int64_t g = e0 + tid; g < e1; g += kBlock) Fl.b[g] = S.V[(int64_t)st.j * N + g];
      break;
    case PH_VC_OUT:
      for (int64_t g = e0 + tid; g < e1; g += kBlock) S.Z[(int64_t)st.j * N + g] = Fl.x[g];
      break;
    case PH_SM_RES: case PH_DN_RES: {
      const BLevel& L = S.lv[st.level];
      residual(D, R, L, S.dtA, L.b, L.x, L.res, r0, min(L.nfree + L.nv, r0 + rr));
      break;
    }
    case PH_SM_PATCH: {
      const BLevel& L = S.lv[st.level];
      const int wave = tid >> 6;
      patches(L, xs + wave * kNmax, xt + wave * 2 * kNmax, st.first ? L.b : L.res, (int64_t)item * kWaves * t.ppw,
              t.ppw);
      break;
    }
    case PH_SM_GATHER: {
      const BLevel& L = S.lv[st.level];
      const int64_t g1 = min(L.N, e0 + er);
      for (int64_t g = e0 + tid; g < g1; g += kBlock)
        dev::gather_one<double>(g, L.gat_ptr, L.gat_slot, L.Y, L.W, S.omega, st.first ? 0 : 1, L.x);
      break;
    }
    case PH_ZERO: {
      const BLevel& L = S.lv[st.level];
      const int64_t g1 = min(L.N, e0 + er);
      for (int64_t g = e0 + tid; g < g1; g += kBlock) L.x[g] = 0.0;
      break;
    }
    case PH_DN_RESTRICT: {
      const BLevel& L = S.lv[st.level];
      const BLevel& C = S.lv[st.level - 1];
      spmv(D, R, C.nfree, C.nv, C.offV, L.offV, L.put_ptr, L.put_col, L.put_val, L.ppt_ptr, L.ppt_col, L.ppt_val,
           L.res, C.b, 0, r0, min(C.nfree + C.nv, r0 + rr));
      break;
    }
    case PH_UP_PROLONG: {
      const BLevel& L = S.lv[st.level];
      const BLevel& C = S.lv[st.level - 1];
      spmv(D, R, L.nfree, L.nv, L.offV, C.offV, L.pu_ptr, L.pu_col, L.pu_val, L.pp_ptr, L.pp_col, L.pp_val, C.x,
           L.x, 1, r0, min(L.nfree + L.nv, r0 + rr));
      break;
    }
    case PH_CO_IN: {
      const int64_t g1 = min(S.N0, e0 + er);
      for (int64_t g = e0 + tid; g < g1; g += kBlock) {
        bool pin = false;
        for (int s = 0; s < R; ++s) pin |= (S.pins[s] == g);
        S.cb[g] = pin ? 0.0 : S.lv[0].b[g];
      }
      break;
    }
    case PH_CO_MV: {
      const int rbk = item / (kCoarseChunks / kWaves), ks = item % (kCoarseChunks / kWaves);
      const int lane = tid & 63, wave = tid >> 6;
      const int chunk = ks * kWaves + wave;
      const int64_t i = (int64_t)rbk * 64 + lane;
      const int64_t per = (S.N0 + kCoarseChunks - 1) / kCoarseChunks;
      const int64_t j0 = chunk * per, j1 = min(S.N0, j0 + per);
      // coarse solve step st.sweep: 0 inv * b, 1 M * x (residual of the refinement
      // step), 2 inv * (b - M x) (its correction)
      const double* mat = st.sweep == 1 ? S.cmat : S.cinv;
      const double* vec = st.sweep == 1 ? S.lv[0].x : S.cb;
      if (i < S.N0) {
        double acc = 0;
        for (int64_t j = j0; j < j1; ++j) acc += mat[j * S.N0 + i] * vec[j];
        S.cpart[(int64_t)chunk * S.N0 + i] = acc;
      }
      break;
    }
    case PH_CO_RED: {
      const int64_t g1 = min(S.N0, e0 + er);
      for (int64_t g = e0 + tid; g < g1; g += kBlock) {
        double acc = 0;
        for (int c = 0; c < kCoarseChunks; ++c) acc += S.cpart[(int64_t)c * S.N0 + g];
        if (st.sweep == 0) S.lv[0].x[g] = acc;
        else if (st.sweep == 1) S.cb[g] -= acc;
        else S.lv[0].x[g] += acc;
      }
      break;
    }
    case PH_PJ_SUM: {
      const double* vec = st.pj_final ? S.x : S.Z + (int64_t)st.j * N;
      const int64_t v1 = min(Fl.nv, e0 + er);
      for (int s = 0; s < R; ++s) {
        double acc = 0;
        for (int64_t v = e0 + tid; v < v1; v += kBlock) acc += vec[Fl.offV + v * R + s];
        const double bs = block_sum(acc, red);
        if (tid == 0) S.partials[(int64_t)item * kMaxStages + s] = bs;
      }
      break;
    }
    case PH_PJ_SUB: {
      double* vec = st.pj_final ? S.x : S.Z + (int64_t)st.j * N;
      const int64_t v1 = min(Fl.nv, e0 + er);
      for (int64_t v = e0 + tid; v < v1; v += kBlock)
        for (int s = 0; s < R; ++s) vec[Fl.offV + v * R + s] -= st.mean[s];
      break;
    }
    case PH_AXPY: {
      const double hij = ald(&gst->H[st.i * kMaxRestart + st.j]);
      const double* vi = S.V + (int64_t)st.i * N;
      for (int64_t g = e0 + tid; g < e1; g += kBlock) S.w[g] -= hij * vi[g];
      break;
    }
    case PH_VSCALE: {
      const double hn = ald(&gst->H[(st.j + 1) * kMaxRestart + st.j]);
      double* vn = S.V + (int64_t)(st.j + 1) * N;
      for (int64_t g = e0 + tid; g < e1; g += kBlock) vn[g] = S.w[g] / hn;
      break;
    }
    case PH_XUPD: {
      double* yv = red;  // LDS staging of the update coefficients
      if (tid < st.jend) yv[tid] = ald(&gst->y[tid]);
      __syncthreads();
      for (int64_t g = e0 + tid; g < e1; g += kBlock) {
        double acc = S.x[g];
        for (int q = 0; q < st.jend; ++q) acc += yv[q] * S.Z[(int64_t)q * N + g];
        S.x[g] = acc;
      }
      __syncthreads();
      break;
    }
    case PH_STORE:
      for (int64_t g = e0 + tid; g < e1; g += kBlock)
        S.k_abi[abi_index(g, Fl.offV, Fl.nfree, S.ns, D, R)] = S.x[g];
      break;
    default:
      break;
  }
}

// ------------------------------------------------------------- state transitions
// shared arrays of the state go through device-scope loads and stores (plain on the host)
template <typename T>
__host__ __device__ inline T gld(const T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#else
  return *p;
#endif
}
template <typename T>
__host__ __device__ inline void gst(T* p, T v) {
#if defined(__HIP_DEVICE_COMPILE__)
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#else
  *p = v;
#endif
}
__host__ __device__ inline bool finite(double v) { return v == v && v - v == 0.0; }
// Reductions of the finished state (all threads), in item order.
__device__ double reduce_partials(const BSolve& S, int n, int stride, int off, double* red) {
  double acc = 0;
  for (int q = threadIdx.x; q < n; q += kBlock) acc += S.partials[(int64_t)q * stride + off];
  return block_sum(acc, red);
}

// smoothing on level l: set the first sweep's phase
__host__ __device__ void end_smooth(const BSolve& S, BState& st);

// smoothing on level l: set the first sweep's state; with no sweeps go on directly
__host__ __device__ void start_smooth(const BSolve& S, BState& st, int l, int nsweeps, int zero_start) {
  st.level = l;
  st.sweep = 0;
  st.first = zero_start;
  if (nsweeps > 0) {
    if (zero_start) st.phase = PH_SM_PATCH;
    else st.phase = PH_SM_RES;
  } else if (zero_start) {
    st.phase = PH_ZERO;
  } else {
    end_smooth(S, st);
  }
}

__host__ __device__ void after_coarse(const BSolve& S, BState& st) {
  if (S.nlevels == 1) {
    st.phase = PH_VC_OUT;
    return;
  }
  st.leg = 1;
  st.level = 1;
  st.phase = PH_UP_PROLONG;
}

__host__ __device__ void end_smooth(const BSolve& S, BState& st) {
  const int top = S.nlevels - 1;
  if (st.leg == 0) {
    st.phase = PH_DN_RES;
  } else if (st.level == top) {
    st.phase = PH_VC_OUT;
  } else {
    st.level += 1;
    st.phase = PH_UP_PROLONG;
  }
}

// decide the next state (thread 0, after the reductions of the finished one)
__host__ __device__ void advance(const BSolve& S, BState& st, double red_val, const double* means, Ctl* ctl) {
  const int top = S.nlevels - 1;
  const int m = S.restart;
  switch (st.phase) {
    case PH_LOAD: st.phase = PH_R0; break;
    case PH_R0: st.phase = PH_N0; break;
    case PH_N0:
      st.beta0 = sqrt(red_val);
      st.its = 0;
      if (!finite(st.beta0)) { st.status = IRK_ENAN; st.phase = PH_DONE; break; }
      if (st.beta0 == 0.0) { st.converged = 1; st.pj_final = 1; st.phase = PH_PJ_SUM; break; }
      st.phase = PH_RES;
      break;
    case PH_RES: st.phase = PH_NRM; break;
    case PH_NRM:
      st.beta = sqrt(red_val);
      if (!finite(st.beta)) { st.status = IRK_ENAN; st.phase = PH_DONE; break; }
      if (st.beta <= S.rtol * st.beta0) { st.converged = 1; st.pj_final = 1; st.phase = PH_PJ_SUM; break; }
      for (int q = 0; q <= m; ++q) gst(&st.g[q], 0.0);
      gst(&st.g[0], st.beta);
      st.j = 0;
      st.phase = PH_V0;
      break;
    case PH_V0: st.phase = PH_VC_IN; break;
    case PH_VC_IN:
      st.leg = 0;
      if (top == 0) { st.phase = PH_CO_IN; break; }
      start_smooth(S, st, top, S.pre, 1);
      break;
    case PH_ZERO:
      end_smooth(S, st);
      break;
    case PH_SM_RES: st.phase = PH_SM_PATCH; break;
    case PH_SM_PATCH: st.phase = PH_SM_GATHER; break;
    case PH_SM_GATHER: {
      const int nsw = st.leg == 0 ? S.pre : S.post;
      st.sweep += 1;
      st.first = 0;
      if (st.sweep < nsw) st.phase = PH_SM_RES;
      else end_smooth(S, st);
      break;
    }
    case PH_DN_RES: st.phase = PH_DN_RESTRICT; break;
    case PH_DN_RESTRICT:
      if (st.level - 1 == 0) {
        st.level = 0;
        st.phase = PH_CO_IN;
      } else {
        start_smooth(S, st, st.level - 1, S.pre, 1);
      }
      break;
    case PH_CO_IN: st.sweep = 0; st.phase = PH_CO_MV; break;
    case PH_CO_MV: st.phase = PH_CO_RED; break;
    case PH_CO_RED:  // inverse times b, then one refinement step (residual, correction)
      if (st.sweep < 2) {
        st.sweep += 1;
        st.phase = PH_CO_MV;
      } else {
        after_coarse(S, st);
      }
      break;
    case PH_UP_PROLONG:
      start_smooth(S, st, st.level, S.post, 0);
      break;
    case PH_VC_OUT: st.pj_final = 0; st.phase = PH_PJ_SUM; break;
    case PH_PJ_SUM:
      for (int s = 0; s < S.r; ++s) st.mean[s] = means[s] / (double)S.lv[top].nv;
      st.phase = PH_PJ_SUB;
      break;
    case PH_PJ_SUB:
      st.phase = st.pj_final ? PH_FR : PH_AP;
      break;
    case PH_AP: st.i = 0; st.phase = PH_DOT; break;
    case PH_DOT:
      gst(&st.H[st.i * kMaxRestart + st.j], red_val);
      st.phase = PH_AXPY;
      break;
    case PH_AXPY:
      st.i += 1;
      st.phase = st.i <= st.j ? PH_DOT : PH_WNRM;
      break;
    case PH_WNRM:
      gst(&st.H[(st.j + 1) * kMaxRestart + st.j], sqrt(red_val));
      st.phase = PH_VSCALE;
      break;
    case PH_VSCALE: {
      const int j = st.j;
      double* H = st.H;
      double col[kMaxRestart + 1];
      for (int q = 0; q <= j + 1; ++q) {
        col[q] = gld(&H[q * kMaxRestart + j]);
        if (!finite(col[q])) { st.status = IRK_ENAN; st.phase = PH_DONE; return; }
      }
      for (int q = 0; q < j; ++q) {
        const double c = gld(&st.cs[q]), sn = gld(&st.sn[q]);
        const double a = col[q], b = col[q + 1];
        col[q] = c * a + sn * b;
        col[q + 1] = -sn * a + c * b;
      }
      const double den = hypot(col[j], col[j + 1]);
      const double cj = col[j] / den, sj = col[j + 1] / den;
      gst(&st.cs[j], cj);
      gst(&st.sn[j], sj);
      col[j] = den;
      col[j + 1] = 0.0;
      for (int q = 0; q <= j + 1; ++q) gst(&H[q * kMaxRestart + j], col[q]);
      const double gj = gld(&st.g[j]);
      const double gj1 = -sj * gj;
      gst(&st.g[j + 1], gj1);
      gst(&st.g[j], cj * gj);
      st.its += 1;
      const bool conv = fabs(gj1) <= S.rtol * st.beta0;
      if (conv || st.its >= S.maxit || j + 1 == m) {
        const int jend = j + 1;
        for (int q = jend - 1; q >= 0; --q) {
          double acc = gld(&st.g[q]);
          for (int c = q + 1; c < jend; ++c) acc -= gld(&H[q * kMaxRestart + c]) * gld(&st.y[c]);
          gst(&st.y[q], acc / gld(&H[q * kMaxRestart + q]));
        }
        st.jend = jend;
        if (conv) st.converged = 1;
        st.phase = PH_XUPD;
      } else {
        st.j = j + 1;
        st.phase = PH_VC_IN;
      }
      break;
    }
    case PH_XUPD:
      if (st.converged || st.its >= S.maxit) {
        st.pj_final = 1;
        st.phase = PH_PJ_SUM;
      } else {
        st.phase = PH_RES;
      }
      break;
    case PH_FR: st.phase = PH_FN; break;
    case PH_FN:
      st.final_rel = st.beta0 > 0 ? sqrt(red_val) / st.beta0 : 0.0;
      if (!finite(st.final_rel)) st.status = IRK_ENAN;
      st.phase = PH_STORE;
      break;
    case PH_STORE:
      st.phase = PH_DONE;
      break;
    default:
      st.phase = PH_DONE;
      break;
  }
  (void)ctl;
}

__global__ __launch_bounds__(kBlock, 1) void k_batch(const BSolve* __restrict__ Sv, BState* Stv, Ctl* ctl,
                                                  int nsolves, Tun tun) {
  __shared__ double xs[kWaves * kNmax];
  __shared__ double xt[kWaves * 2 * kNmax];  // doubled copies for the symmetric form
  __shared__ double red[kBlock];
  __shared__ int s_item, s_ok, s_last, s_exit, s_solve, s_epoch, s_viol;
  __shared__ BCur s_st;  // snapshot of the solve's state for the item being executed
  __shared__ double s_means[kMaxStages];
  const int tid = threadIdx.x;
  if (blockIdx.x == 0 && tid == 0) __hip_atomic_store(&ctl->t0, wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  int cursor = blockIdx.x % nsolves;
  long long idle = 0;
  while (true) {
    if (tid == 0) {
      const int fin = __hip_atomic_load(&ctl->finished, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
      const int ab = __hip_atomic_load(&ctl->abort, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
      s_exit = (fin >= nsolves || ab) ? 1 : 0;
      s_ok = 0;
      if (!s_exit) {
        BState* st = &Stv[cursor];
        const int ph = __hip_atomic_load(&st->phase, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long tk0 = __hip_atomic_load(&st->ticket, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int n0 = __hip_atomic_load(&st->n_items, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (ph != PH_DONE && (int)(tk0 & 0xffffffffull) < n0) {
          const unsigned long long tk =
              __hip_atomic_fetch_add(&st->ticket, 1ull, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
          const int e = (int)(tk >> 32), item = (int)(tk & 0xffffffffull);
          // epoch and item count of the current state, read as one word
          const unsigned long long mt = __hip_atomic_load(&st->meta, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
          if ((int)(mt >> 32) == e && item < (int)(mt & 0xffffffffull)) {
            s_ok = 1;
            s_item = item;
            s_solve = cursor;
            s_epoch = e;
          }
        }
      }
    }
    __syncthreads();
    if (s_exit) break;
    if (!s_ok) {
      cursor = (cursor + 1) % nsolves;
      if (++idle > ctl->max_idle) {
        if (tid == 0) {
          int expected = 0;
          if (__hip_atomic_compare_exchange_strong(&ctl->abort, &expected, 1, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT))
            for (int q = 0; q < min(nsolves, 16); ++q) {
              BState* sq = &Stv[q];
              const unsigned long long tk = ald(&sq->ticket);
              ast(&ctl->dbg[q * 7 + 0], ald(&sq->phase));
              ast(&ctl->dbg[q * 7 + 1], ald(&sq->epoch));
              ast(&ctl->dbg[q * 7 + 2], ald(&sq->done));
              ast(&ctl->dbg[q * 7 + 3], ald(&sq->done_base));
              ast(&ctl->dbg[q * 7 + 4], ald(&sq->n_items));
              ast(&ctl->dbg[q * 7 + 5], (int)(tk & 0xffffffffull));
              ast(&ctl->dbg[q * 7 + 6], (int)(tk >> 32));
            }
        }
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    idle = 0;
    // thread 0's ticket acquire (device scope) invalidated this CU's L1 and this XCD's
    // L2 before the barrier, so every wave reads data released by earlier states
    const BSolve& S = Sv[s_solve];
    BState* st = &Stv[s_solve];
    // snapshot of the state (stable while this item is outstanding)
    if (tid == 0) {
      s_viol = (ald(&st->epoch) != s_epoch) ? 1 : 0;
      s_st.phase = ald(&st->phase);
      s_st.n_items = ald(&st->n_items);
      s_st.done_base = ald(&st->done_base);
      s_st.level = ald(&st->level);
      s_st.first = ald(&st->first);
      s_st.sweep = ald(&st->sweep);
      s_st.j = ald(&st->j);
      s_st.i = ald(&st->i);
      s_st.jend = ald(&st->jend);
      s_st.pj_final = ald(&st->pj_final);
      s_st.beta = ald(&st->beta);
      for (int q = 0; q < kMaxStages; ++q) s_st.mean[q] = ald(&st->mean[q]);
    }
    __syncthreads();
    if (s_viol) {
      if (tid == 0) __hip_atomic_store(&ctl->abort, 2, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    exec_item(S, s_st, st, s_item, tun, xs, xt, red);
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have reached L2
    __syncthreads();
    if (tid == 0) {
      __threadfence();  // release (device scope): write back this XCD's L2
      const int d = __hip_atomic_fetch_add(&st->done, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      s_last = (d == s_st.done_base + s_st.n_items - 1) ? 1 : 0;
    }
    __syncthreads();
    if (s_last) {
      // thread 0's acq_rel increment acquired every other item's results
      // reductions of the finished state, then the transition
      double rv = 0.0;
      const int ph = s_st.phase;
      if (ph == PH_N0 || ph == PH_NRM || ph == PH_FN || ph == PH_DOT || ph == PH_WNRM)
        rv = reduce_partials(S, s_st.n_items, 1, 0, red);
      if (ph == PH_PJ_SUM)
        for (int s = 0; s < S.r; ++s) {
          const double v = reduce_partials(S, s_st.n_items, kMaxStages, s, red);
          if (tid == 0) s_means[s] = v;
        }
      __syncthreads();
      if (tid == 0) {
        BState& w = *st;
        if (ald(&st->epoch) != s_epoch || ald(&st->phase) != s_st.phase) s_viol |= 2;
        w.ntrans += 1;
        w.last_phase = s_st.phase;
        w.phase = s_st.phase;
        w.level = ald(&st->level);
        w.sweep = ald(&st->sweep);
        w.first = ald(&st->first);
        w.leg = ald(&st->leg);
        w.j = ald(&st->j);
        w.i = ald(&st->i);
        w.jend = ald(&st->jend);
        w.pj_final = ald(&st->pj_final);
        w.its = ald(&st->its);
        w.converged = ald(&st->converged);
        w.status = ald(&st->status);
        w.beta0 = ald(&st->beta0);
        w.beta = ald(&st->beta);
        w.final_rel = ald(&st->final_rel);
        for (int q = 0; q < kMaxStages; ++q) w.mean[q] = ald(&st->mean[q]);
        advance(S, w, rv, s_means, ctl);
        const int nph = w.phase;
        const int nitems = (nph == PH_DONE) ? 0 : items_of(S, w, nph, tun);
        if (nph == PH_DONE) w.t_end = wall_clock64();
        // publish the new state with device-scope stores, then release the ticket
        ast(&st->done_base, s_st.done_base + s_st.n_items);
        ast(&st->n_items, nitems);
        ast(&st->level, w.level);
        ast(&st->sweep, w.sweep);
        ast(&st->first, w.first);
        ast(&st->leg, w.leg);
        ast(&st->j, w.j);
        ast(&st->i, w.i);
        ast(&st->jend, w.jend);
        ast(&st->pj_final, w.pj_final);
        ast(&st->its, w.its);
        ast(&st->converged, w.converged);
        ast(&st->status, w.status);
        ast(&st->beta0, w.beta0);
        ast(&st->beta, w.beta);
        ast(&st->final_rel, w.final_rel);
        for (int q = 0; q < kMaxStages; ++q) ast(&st->mean[q], w.mean[q]);
        ast(&st->epoch, s_epoch + 1);
        ast(&st->phase, nph);
        ast(&st->meta, (((unsigned long long)(s_epoch + 1)) << 32) | (unsigned long long)(unsigned)nitems);
        __threadfence();
        __hip_atomic_store(&st->ticket, ((unsigned long long)(s_epoch + 1)) << 32, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
        if (nph == PH_DONE) __hip_atomic_fetch_add(&ctl->finished, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
      __syncthreads();
      if (s_viol) {
        if (tid == 0) __hip_atomic_store(&ctl->abort, 3, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
}

}  // namespace batch
}  // namespace irk

// ============================================================================ host
using namespace irk;
using namespace irk::batch;

struct irk_batch {
  std::vector<irk_mg*> hs;
  BSolve* dS = nullptr;
  BState* dSt = nullptr;
  Ctl* dctl = nullptr;
  std::vector<double*> partials, ktrial;
  std::vector<void*> allocs;
  irk_batch_opts opts{};
  bool tuned = false;
  bool persistent_ok = true;  // every handle fits the persistent kernel
  int wg_per_cu = 0, cus = 0, device = 0;
  double wall_khz = 100000.0;
  std::vector<hipStream_t> streams;  // concurrent-streams schedule
};

namespace {
irk_status bfail(irk_status c, const std::string& m) {
  irk::set_error(m);
  return c;
}

#define BHIP(expr)                                                                            \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return bfail(IRK_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
irk_status balloc(irk_batch* b, T** p, size_t n) {
  if (hipMalloc((void**)p, std::max<size_t>(1, n) * sizeof(T)) != hipSuccess)
    return bfail(IRK_ENOMEM, "hipMalloc failed in the batched solver");
  b->allocs.push_back(*p);
  return IRK_OK;
}

// The work-queue state (tickets, counters, scalars) lives in fine-grained device
// memory: atomics on ordinary device memory are resolved in the L2 cache of the XCD
// that issues them, so workgroups on different XCDs could draw the same ticket.
template <typename T>
irk_status balloc_fine(irk_batch* b, T** p, size_t n) {
  if (hipExtMallocWithFlags((void**)p, std::max<size_t>(1, n) * sizeof(T), hipDeviceMallocFinegrained) != hipSuccess)
    return bfail(IRK_ENOMEM, "fine-grained allocation failed in the batched solver");
  b->allocs.push_back(*p);
  return IRK_OK;
}

BLevel level_view(const DevLevel& L) {
  BLevel v{};
  v.nfree = L.nfree;
  v.nv = L.nv;
  v.N = L.N;
  v.offV = L.offV;
  v.npatch = L.npatch;
  v.pform = L.pform;
  v.dim = L.dim;
  v.r = L.r;
  v.rb = L.pform == 1 ? (L.max_ld <= 128 ? 1 : 2) : (L.max_nloc <= 128 ? 1 : 2);
  v.sb = L.sb64;
  v.s_ptr = L.s_ptr; v.s_col = L.s_col; v.b_ptr = L.b_ptr; v.b_col = L.b_col; v.bt_ptr = L.bt_ptr; v.bt_col = L.bt_col;
  v.sM = L.d64.s_M; v.sL = L.d64.s_L; v.b_val = L.d64.b_val; v.bt_val = L.d64.bt_val; v.W = L.d64.W;
  v.pu_ptr = L.pu_ptr; v.pu_col = L.pu_col; v.put_ptr = L.put_ptr; v.put_col = L.put_col;
  v.pp_ptr = L.pp_ptr; v.pp_col = L.pp_col; v.ppt_ptr = L.ppt_ptr; v.ppt_col = L.ppt_col;
  v.pu_val = L.d64.pu_val; v.put_val = L.d64.put_val; v.pp_val = L.d64.pp_val; v.ppt_val = L.d64.ppt_val;
  v.p_nloc = L.p_nloc; v.p_ld = L.p_ld; v.sched = L.sched; v.p_gidx = L.p_gidx; v.gat_ptr = L.gat_ptr;
  v.gat_slot = L.gat_slot; v.p_inv_off = L.p_inv_off; v.p_slot_off = L.p_slot_off;
  v.inv = reinterpret_cast<const double*>(L.inv);
  v.b = (double*)L.b; v.x = (double*)L.x; v.res = (double*)L.res; v.Y = (double*)L.Y;
  return v;
}

int host_items_first(const BSolve& S, const Tun& t) {  // items of PH_LOAD
  return cdiv(S.lv[S.nlevels - 1].N, (int64_t)kBlock * t.elems);
}

irk_status run(irk_batch* b, const double* const* F, double* const* k, bool trial, double rtol, int maxit,
               int restart, hipStream_t s, float* ms_out, std::vector<BState>* states_out,
               unsigned long long* t0_out) {
  const int n = (int)b->hs.size();
  const Tun tun{b->opts.rows_per_item, b->opts.patches_per_wave, b->opts.rows_per_item};
  std::vector<BSolve> hS(n);
  for (int q = 0; q < n; ++q) {
    irk_mg* h = b->hs[q];
    if (ensure_krylov_ws(h, restart) != IRK_OK) return bfail(IRK_ENOMEM, "Krylov workspace allocation failed");
    BSolve& S = hS[q];
    std::memset(&S, 0, sizeof(S));
    S.dim = h->dim;
    S.r = h->r;
    S.nlevels = h->nlevels;
    S.pre = h->pre;
    S.post = h->post;
    S.restart = restart;
    S.maxit = maxit;
    S.omega = h->omega;
    S.rtol = rtol;
    for (int i = 0; i < h->r * h->r; ++i) S.dtA.v[i] = h->dt * h->A[i];
    const DevLevel& Ft = h->dev[h->nlevels - 1];
    S.ns = h->dim * Ft.nfree + Ft.nv;
    for (int l = 0; l < h->nlevels; ++l) S.lv[l] = level_view(h->dev[l]);
    S.cinv = h->coarse_inv;
    S.cmat = h->coarse_mat;
    S.cb = h->cb;
    S.cpart = h->cpart;
    for (int st = 0; st < h->r; ++st) S.pins[st] = h->dev[0].offV + st;
    S.N0 = h->dev[0].N;
    S.F_abi = F[q];
    S.k_abi = trial ? b->ktrial[q] : k[q];
    S.F = h->kF;
    S.x = h->kx;
    S.V = h->kv;
    S.Z = h->kz;
    S.w = h->kw;
    S.rv = h->kr;
    S.partials = b->partials[q];
  }
  std::vector<BState> hSt(n);
  for (int q = 0; q < n; ++q) {
    std::memset(&hSt[q], 0, sizeof(BState));
    hSt[q].phase = PH_LOAD;
    hSt[q].n_items = host_items_first(hS[q], tun);
    hSt[q].meta = (unsigned long long)(unsigned)hSt[q].n_items;
  }
  Ctl c{};
  c.max_idle = 2000000LL;
  BHIP(hipMemcpyAsync(b->dS, hS.data(), n * sizeof(BSolve), hipMemcpyHostToDevice, s));
  BHIP(hipMemcpyAsync(b->dSt, hSt.data(), n * sizeof(BState), hipMemcpyHostToDevice, s));
  BHIP(hipMemcpyAsync(b->dctl, &c, sizeof(Ctl), hipMemcpyHostToDevice, s));
  const int grid = std::max(1, b->cus * std::max(1, b->opts.workgroups_per_cu));
  hipEvent_t e0, e1;
  BHIP(hipEventCreate(&e0));
  BHIP(hipEventCreate(&e1));
  BHIP(hipEventRecord(e0, s));
  k_batch<<<dim3(grid), dim3(kBlock), 0, s>>>(b->dS, b->dSt, b->dctl, n, tun);
  BHIP(hipGetLastError());
  BHIP(hipEventRecord(e1, s));
  BHIP(hipEventSynchronize(e1));
  float ms = 0;
  BHIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (ms_out) *ms_out = ms;
  BHIP(hipMemcpy(&c, b->dctl, sizeof(Ctl), hipMemcpyDeviceToHost));
  if (c.abort == 1) {
    if (std::getenv("IRK_BATCH_DEBUG"))
      for (int q = 0; q < std::min(n, 16); ++q)
        fprintf(stderr, "stuck solve %d: phase %d epoch %d done %d base %d n_items %d ticket item %d epoch %d\n", q,
                c.dbg[q * 7], c.dbg[q * 7 + 1], c.dbg[q * 7 + 2], c.dbg[q * 7 + 3], c.dbg[q * 7 + 4], c.dbg[q * 7 + 5],
                c.dbg[q * 7 + 6]);
    return bfail(IRK_EHIP, "batched solver aborted: a workgroup found no work for too long");
  }
  if (c.abort) return bfail(IRK_EHIP, "batched solver aborted: work-queue protocol violation " + std::to_string(c.abort));
  if (states_out) {
    states_out->resize(n);
    BHIP(hipMemcpy(states_out->data(), b->dSt, n * sizeof(BState), hipMemcpyDeviceToHost));
  }
  if (t0_out) *t0_out = c.t0;
  return IRK_OK;
}
}  // namespace

namespace {
// Concurrent-streams schedule: `streams` host threads, each with its own HIP stream,
// take whole solves (largest first) from a shared counter and run the launch-per-step
// FGMRES-MG solver on them.  Outputs go to k (or to scratch for trial runs).
irk_status run_streams(irk_batch* b, const double* const* F, double* const* k, bool trial, double rtol, int maxit,
                       int restart, hipStream_t s, float* ms_out, irk_solve_info* infos, double* latency_ms) {
  const int n = (int)b->hs.size();
  const int S = std::max(1, std::min(b->opts.streams, (int)b->streams.size()));
  BHIP(hipStreamSynchronize(s));  // inputs produced on the caller's stream are ready
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    return b->hs[a]->dev[b->hs[a]->nlevels - 1].N > b->hs[c]->dev[b->hs[c]->nlevels - 1].N;
  });
  std::atomic<int> next{0};
  std::vector<irk_status> status(n, IRK_OK);
  std::vector<std::string> errs(n);
  std::vector<irk_solve_info> res(n);
  std::vector<double> lat(n, 0.0);
  const auto t0 = std::chrono::steady_clock::now();
  auto worker = [&](int w) {
    (void)hipSetDevice(b->device);
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= n) break;
      const int q = order[i];
      irk_solve_info info{};
      double* out = trial ? b->ktrial[q] : k[q];
      if (trial) (void)hipMemcpyAsync(out, k[q], sizeof(double) * b->hs[q]->dev[b->hs[q]->nlevels - 1].N,
                                       hipMemcpyDeviceToDevice, b->streams[w]);
      status[q] = irk_fgmres_solve(b->hs[q], F[q], out, rtol, maxit, restart, &info, b->streams[w]);
      if (status[q] != IRK_OK) errs[q] = irk_last_error();
      res[q] = info;
      lat[q] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
  };
  std::vector<std::thread> pool;
  for (int w = 0; w < S; ++w) pool.emplace_back(worker, w);
  for (auto& t : pool) t.join();
  *ms_out = (float)std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  irk_status ret = IRK_OK;
  for (int q = 0; q < n; ++q) {
    if (infos && !trial) {
      infos[q].iterations = res[q].iterations;
      infos[q].converged = res[q].converged;
      infos[q].rel_residual = res[q].rel_residual;
      infos[q].ms_vcycle = res[q].ms_vcycle;
      infos[q].ms_total = res[q].ms_total;
    }
    if (latency_ms && !trial) latency_ms[q] = lat[q];
    const irk_status st = status[q];
    if (st == IRK_OK || (st == IRK_ENOCONV && trial)) continue;
    if (st == IRK_ENOCONV) {
      if (ret == IRK_OK) ret = IRK_ENOCONV;
      continue;
    }
    return bfail(st, "batched solve " + std::to_string(q) + ": " + errs[q]);
  }
  if (ret == IRK_ENOCONV) irk::set_error("a batched solve reached maxit");
  return ret;
}
}  // namespace

extern "C" {

void irk_batch_default_opts(irk_batch_opts* o) {
  if (!o) return;
  o->rows_per_item = 1;
  o->patches_per_wave = 1;
  o->workgroups_per_cu = 2;
  o->autotune = 1;
  o->mode = 0;
  o->streams = 4;
}

irk_status irk_batch_create(irk_mg* const* hs, int n, const irk_batch_opts* opts, void* stream, irk_batch** out) {
  if (!out) return bfail(IRK_EINVAL, "out is NULL");
  *out = nullptr;
  if (!hs || n < 1 || n > 4096) return bfail(IRK_EINVAL, "need 1..4096 handles");
  irk_batch_opts o;
  irk_batch_default_opts(&o);
  if (opts) o = *opts;
  if (o.rows_per_item < 1 || o.rows_per_item > 64 || o.patches_per_wave < 1 || o.patches_per_wave > 64 ||
      o.workgroups_per_cu < 1 || o.workgroups_per_cu > 8)
    return bfail(IRK_EINVAL, "rows_per_item and patches_per_wave in 1..64, workgroups_per_cu in 1..8");
  if ((o.mode != 0 && o.mode != 1) || o.streams < 1 || o.streams > 16)
    return bfail(IRK_EINVAL, "mode must be 0 or 1 and streams in 1..16");
  // the persistent kernel runs FP64 2D handles with the damped-sweep smoother and
  // patches of at most 256 unknowns; the concurrent-streams schedule runs any handle
  bool persistent_ok = true;
  std::string why;
  for (int q = 0; q < n; ++q) {
    if (!hs[q]) return bfail(IRK_EINVAL, "null handle in the batch");
    for (int p = 0; p < q; ++p)
      if (hs[p] == hs[q]) return bfail(IRK_EINVAL, "a handle appears twice in the batch");
    if (hs[q]->precision != 0) why = "the persistent kernel runs FP64 handles only";
    else if (hs[q]->smoother != 0) why = "the persistent kernel runs the damped-sweep smoother only";
    else if (hs[q]->dim != 2) why = "the persistent kernel runs 2D handles only";
    else if (hs[q]->nlevels > kMaxLevels) why = "too many levels for the persistent kernel";
    else
      for (int l = 1; l < hs[q]->nlevels; ++l)
        if (hs[q]->dev[l].max_nloc > kNmax || hs[q]->dev[l].max_ld > 2 * 128)
          why = "patch too large for the persistent kernel";
    if (!why.empty()) persistent_ok = false;
  }
  if (!persistent_ok && o.mode == 0 && !o.autotune) return bfail(IRK_EINVAL, why);
  if (!persistent_ok) o.mode = 1;
  irk_batch* b = new (std::nothrow) irk_batch();
  if (!b) return bfail(IRK_ENOMEM, "allocation failed");
  b->hs.assign(hs, hs + n);
  b->opts = o;
  b->persistent_ok = persistent_ok;
  int dev = 0;
  irk_status st = IRK_OK;
  auto cleanup = [&](irk_status code) {
    for (void* p : b->allocs) (void)hipFree(p);
    delete b;
    return code;
  };
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return cleanup(bfail(IRK_EHIP, "device query failed"));
  b->device = dev;
  for (int i = 0; i < 16; ++i) {
    hipStream_t st_i;
    if (hipStreamCreate(&st_i) != hipSuccess) {
      for (hipStream_t x : b->streams) (void)hipStreamDestroy(x);
      return cleanup(bfail(IRK_EHIP, "stream creation failed"));
    }
    b->streams.push_back(st_i);
  }
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0) b->wall_khz = khz;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k_batch, kBlock, 0) != hipSuccess || occ < 1)
    return cleanup(bfail(IRK_EHIP, "occupancy query failed"));
  b->wg_per_cu = occ;
  b->opts.workgroups_per_cu = std::min(b->opts.workgroups_per_cu, occ);
  if ((st = balloc(b, &b->dS, n)) != IRK_OK) return cleanup(st);
  if ((st = balloc_fine(b, &b->dSt, n)) != IRK_OK) return cleanup(st);
  if ((st = balloc_fine(b, &b->dctl, 1)) != IRK_OK) return cleanup(st);
  b->partials.resize(n);
  b->ktrial.resize(n);
  for (int q = 0; q < n; ++q) {
    const DevLevel& Ft = hs[q]->dev[hs[q]->nlevels - 1];
    const size_t np = (size_t)kMaxStages * (size_t)cdiv(Ft.N, kBlock) + 64;
    if ((st = balloc(b, &b->partials[q], np)) != IRK_OK) return cleanup(st);
    if ((st = balloc(b, &b->ktrial[q], (size_t)Ft.N)) != IRK_OK) return cleanup(st);
  }
  (void)stream;
  *out = b;
  return IRK_OK;
}

void irk_batch_destroy(irk_batch* b) {
  if (!b) return;
  for (hipStream_t x : b->streams) (void)hipStreamDestroy(x);
  for (void* p : b->allocs) (void)hipFree(p);
  delete b;
}

irk_status irk_batch_get_opts(const irk_batch* b, irk_batch_opts* out) {
  if (!b || !out) return bfail(IRK_EINVAL, "null argument");
  *out = b->opts;
  return IRK_OK;
}

irk_status irk_batch_fgmres_solve(irk_batch* b, const double* const* F, double* const* k, double rtol, int maxit,
                                  int restart, irk_solve_info* infos, double* latency_ms, void* stream) {
  if (!b || !F || !k) return bfail(IRK_EINVAL, "null argument");
  if (!(rtol > 0) || maxit < 1 || restart < 1 || restart > kMaxRestart)
    return bfail(IRK_EINVAL, "rtol > 0, maxit >= 1 and 1 <= restart <= 64 required");
  const int n = (int)b->hs.size();
  for (int q = 0; q < n; ++q)
    if (!F[q] || !k[q]) return bfail(IRK_EINVAL, "null vector in the batch");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (b->opts.autotune && !b->tuned) {
    // time short trial runs (2 iterations per solve, outputs to scratch) over the
    // schedule space (concurrent streams, then the persistent kernel's tiles) and keep
    // the fastest; one stream is the one-by-one baseline
    float best = 1e30f;
    irk_batch_opts bo = b->opts;
    for (int S : {1, 2, 4, 8}) {
      b->opts.mode = 1;
      b->opts.streams = S;
      float ms = 0;
      irk_status st = run_streams(b, F, k, true, rtol, 2, restart, s, &ms, nullptr, nullptr);
      if (std::getenv("IRK_BATCH_DEBUG")) fprintf(stderr, "autotune streams %d: %.3f ms (status %d)\n", S, ms, st);
      if (st != IRK_OK) return st;
      if (ms < best) {
        best = ms;
        bo = b->opts;
      }
    }
    b->opts.mode = 0;
    for (int wg : {1, 2, 4})
      for (int rows : {1, 2, 4})
        for (int ppw : {1, 2, 4}) {
          if (!b->persistent_ok) continue;
          if (wg > b->wg_per_cu) continue;
          b->opts.workgroups_per_cu = wg;
          b->opts.rows_per_item = rows;
          b->opts.patches_per_wave = ppw;
          float ms = 0;
          irk_status st = run(b, F, k, true, rtol, 2, restart, s, &ms, nullptr, nullptr);
          if (std::getenv("IRK_BATCH_DEBUG"))
            fprintf(stderr, "autotune wg %d rows %d ppw %d: %.3f ms (status %d)\n", wg, rows, ppw, ms, st);
          if (st != IRK_OK) return st;
          if (ms < best) {
            best = ms;
            bo = b->opts;
          }
        }
    b->opts = bo;
    b->tuned = true;
  }
  if (b->opts.mode == 1) {
    float ms = 0;
    return run_streams(b, F, k, false, rtol, maxit, restart, s, &ms, infos, latency_ms);
  }
  std::vector<BState> states;
  unsigned long long t0 = 0;
  float ms = 0;
  irk_status st = run(b, F, k, false, rtol, maxit, restart, s, &ms, &states, &t0);
  if (st != IRK_OK) return st;
  irk_status ret = IRK_OK;
  if (std::getenv("IRK_BATCH_DEBUG"))
    for (int q = 0; q < n; ++q)
      fprintf(stderr, "batch solve %d: ntrans %d last_phase %d its %d conv %d status %d beta0 %g beta %g rel %g size %zu\n", q,
              states[q].ntrans, states[q].last_phase, states[q].its, states[q].converged, states[q].status,
              states[q].beta0, states[q].beta, states[q].final_rel, sizeof(BState));
  for (int q = 0; q < n; ++q) {
    const BState& x = states[q];
    if (infos) {
      infos[q].iterations = x.its;
      infos[q].converged = x.converged;
      infos[q].rel_residual = x.final_rel;
      infos[q].ms_vcycle = 0;
      infos[q].ms_total = ms;
      if (infos[q].history && infos[q].history_cap > 0) infos[q].history[0] = x.beta0;
    }
    if (latency_ms) latency_ms[q] = (double)(x.t_end - t0) / b->wall_khz;
    if (x.status == IRK_ENAN) ret = IRK_ENAN;
    else if (!x.converged && ret == IRK_OK) ret = IRK_ENOCONV;
  }
  if (ret == IRK_ENAN) return bfail(IRK_ENAN, "non-finite value in a batched solve");
  if (ret == IRK_ENOCONV) irk::set_error("a batched solve reached maxit");
  return ret;
}

}  // extern "C"
