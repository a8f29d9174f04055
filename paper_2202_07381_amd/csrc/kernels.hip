// HIP kernels of libirkmg for gfx950 (CDNA4, 64-wide wavefronts).
//
//  residual       r = F - J x (or y = J x) for the Kronecker stage operator
//                 J = I_r (x) [M 0;0 0] + dt A (x) [L B; B^T 0]   (Sec. 3.1).
//                 One CSR traversal of the scalar P2 blocks serves all dim*r values
//                 of a node; the r x r stage mixing is applied once per row.
//  patch_factor   A_v = R_v J R_v^T assembled in LDS and inverted by Gauss--Jordan with
//                 partial pivoting (Sec. 4.2 patch solves), stored column-major.
//  patch_apply    one wavefront per patch: gather R_v res, stream the stored inverse
//                 column by column (each column one coalesced 16-byte-per-lane load),
//                 write the local correction to the patch's private output slots.
//  gather_update  owner gather: every DOF sums its patches' slots in a fixed order and
//                 applies x += omega W sum (deterministic, no atomics).
//  restrict_ / prolong_add   I_r (x) P and its transpose (Sec. 4.1), node-chunked CSR.
//  coarse_solve   dense coarse solve with the stored inverse, one refinement step.
//  dot / axpy / ... deterministic fixed-order reductions for FGMRES.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device_ops.h"
#include "irk_internal.h"
#include "mhd_internal.h"

namespace irk {
namespace k {
namespace {

constexpr int kBlock = 256;
constexpr int kReduceBlocks = 512;

inline unsigned blocks_for(int64_t n, int block = kBlock) {
  int64_t b = (n + block - 1) / block;
  return (unsigned)std::max<int64_t>(1, b);
}

using dev::Coef;

template <typename T, int R>
Coef<T> scaled(const double* A, double dt) {
  Coef<T> c{};
  for (int i = 0; i < R * R; ++i) c.v[i] = (T)(dt * A[i]);
  return c;
}

template <typename T>
const StageBasis<T>& basis_of(const DevLevel& L);
template <>
const StageBasis<double>& basis_of<double>(const DevLevel& L) { return L.sb64; }
template <>
const StageBasis<float>& basis_of<float>(const DevLevel& L) { return L.sb32; }

// Patch counts up to kSmallPatches mark the small levels (64 x 64 and below on the
// 256 x 256 hierarchy): their stored factors fit the last-level cache, so the patch
// kernels read them with ordinary loads there and with non-temporal loads on the
// large levels, whose factors stream through once per application.
constexpr int64_t kSmallPatches = 8192;
// Residual slices below which each slice is split between two wavefronts (k_residual_sell)
constexpr int64_t kSplitSlices = 4096;

// ------------------------------------------------------------------------ residual
template <int D, int R, typename T>
__global__ __launch_bounds__(kBlock) void k_residual(
    int64_t nfree, int64_t nv, int64_t offV, const int32_t* __restrict__ s_ptr,
    const int32_t* __restrict__ s_col, const T* __restrict__ sM, const T* __restrict__ sL,
    const int32_t* __restrict__ b_ptr, const int32_t* __restrict__ b_col,
    const T* __restrict__ b_val, const int32_t* __restrict__ bt_ptr,
    const int32_t* __restrict__ bt_col, const T* __restrict__ bt_val, Coef<T> dtA,
    const T* __restrict__ F, const T* __restrict__ x, T* __restrict__ y) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  dev::residual_row<D, R, T>(row, nfree, nv, offV, s_ptr, s_col, sM, sL, b_ptr, b_col, b_val, bt_ptr, bt_col,
                             bt_val, dtA, F, x, y);
}

// Same residual from the sliced operator copies: NW wavefronts per slice of 64 rows
// (velocity slices first, then vertex slices), lane = row.  Wavefront h of a slice takes
// its entries k = h, h + NW, ..., each read column-major (coalesced indices and values),
// with kSellUnroll entries' gathers in flight per lane (4: more lowered occupancy and
// measured slower on every level); with NW = 2 the odd wavefront's partial sums reach the
// even one through LDS.  Two wavefronts per slice halve each lane's chain of dependent
// gathers and double the wavefronts in flight, which pays on levels with too few slices
// to fill the chip (128 x 128 and below: 17.6 -> 14.1 us at 128 x 128, 12.4 -> 8.9 us at
// 64 x 64) but not on the 256 x 256 level (47.3 -> 49.4 us).
template <int D, int R, typename T, int kSellUnroll, int NW>
__global__ __launch_bounds__(256) void k_residual_sell(
    int64_t nfree, int64_t nv, int64_t offV, int64_t nsu, int64_t nsp, const int32_t* __restrict__ su_off,
    const int32_t* __restrict__ su_w, const int32_t* __restrict__ su_col, const T* __restrict__ uM,
    const T* __restrict__ uL, const int32_t* __restrict__ sb_off, const int32_t* __restrict__ sb_w,
    const int32_t* __restrict__ sb_col, const T* __restrict__ uB, const int32_t* __restrict__ sp_off,
    const int32_t* __restrict__ sp_w, const int32_t* __restrict__ sp_col, const T* __restrict__ pBt,
    Coef<T> dtA, const T* __restrict__ F, const T* __restrict__ x, T* __restrict__ y) {
  constexpr int DR = D * R;
  constexpr int64_t kStride = 64 * NW;  // from this wavefront's entry to its next
  constexpr int kSlices = 4 / NW;       // slices per workgroup of four wavefronts
  __shared__ T part[NW == 2 ? kSlices : 1][NW == 2 ? 2 * DR : 1][64];
  const int lane = threadIdx.x & 63;
  const int half = (threadIdx.x >> 6) % NW;
  const int pair = (threadIdx.x >> 6) / NW;
  const int64_t sl = (int64_t)blockIdx.x * kSlices + pair;
  T am[DR], al[DR];
#pragma unroll
  for (int q = 0; q < DR; ++q) am[q] = al[q] = T(0);
  if (sl < nsu) {
    {
      const int w = su_w[sl];
      const int wh = w > half ? (w - half + NW - 1) / NW : 0;
      const int64_t e0 = su_off[sl] + (int64_t)half * 64 + lane;
      // software pipelined: the next round's column indices are fetched while this
      // round's gathers are in flight
      int32_t jn[kSellUnroll];
      if (kSellUnroll <= wh)
#pragma unroll
        for (int u = 0; u < kSellUnroll; ++u) jn[u] = su_col[e0 + (int64_t)u * kStride];
      int k = 0;
      for (; k + kSellUnroll <= wh; k += kSellUnroll) {
        int32_t j[kSellUnroll];
        T m[kSellUnroll], l[kSellUnroll], xv[kSellUnroll][DR];
#pragma unroll
        for (int u = 0; u < kSellUnroll; ++u) {
          const int64_t e = e0 + (int64_t)(k + u) * kStride;
          j[u] = jn[u];
          m[u] = uM[e];
          l[u] = uL[e];
        }
#pragma unroll
        for (int u = 0; u < kSellUnroll; ++u)
#pragma unroll
          for (int q = 0; q < DR; ++q) xv[u][q] = x[(int64_t)j[u] * DR + q];
        if (k + 2 * kSellUnroll <= wh)
#pragma unroll
          for (int u = 0; u < kSellUnroll; ++u) jn[u] = su_col[e0 + (int64_t)(k + kSellUnroll + u) * kStride];
#pragma unroll
        for (int u = 0; u < kSellUnroll; ++u)
#pragma unroll
          for (int q = 0; q < DR; ++q) {
            am[q] += m[u] * xv[u][q];
            al[q] += l[u] * xv[u][q];
          }
      }
      for (; k < wh; ++k) {
        const int64_t e = e0 + (int64_t)k * kStride;
        const int64_t jj = su_col[e];
        const T mm = uM[e], ll = uL[e];
#pragma unroll
        for (int q = 0; q < DR; ++q) {
          const T v = x[jj * DR + q];
          am[q] += mm * v;
          al[q] += ll * v;
        }
      }
    }
    {
      const int w = sb_w[sl];
      const int wh = w > half ? (w - half + NW - 1) / NW : 0;
      const int64_t e0 = sb_off[sl] + (int64_t)half * 64 + lane;
      int32_t jn[kSellUnroll];
      if (kSellUnroll <= wh)
#pragma unroll
        for (int u = 0; u < kSellUnroll; ++u) jn[u] = sb_col[e0 + (int64_t)u * kStride];
      int k = 0;
      for (; k + kSellUnroll <= wh; k += kSellUnroll) {
        int32_t j[kSellUnroll];
        T pv[kSellUnroll][R], bv[kSellUnroll][D];
#pragma unroll
        for (int u = 0; u < kSellUnroll; ++u) j[u] = jn[u];
        if (k + 2 * kSellUnroll <= wh)
#pragma unroll
          for (int u = 0; u < kSellUnroll; ++u) jn[u] = sb_col[e0 + (int64_t)(k + kSellUnroll + u) * kStride];
#pragma unroll
        for (int u = 0; u < kSellUnroll; ++u) {
          const int64_t e = e0 + (int64_t)(k + u) * kStride;
#pragma unroll
          for (int t = 0; t < R; ++t) pv[u][t] = x[offV + (int64_t)j[u] * R + t];
#pragma unroll
          for (int c = 0; c < D; ++c) bv[u][c] = uB[e * D + c];
        }
#pragma unroll
        for (int u = 0; u < kSellUnroll; ++u)
#pragma unroll
          for (int c = 0; c < D; ++c)
#pragma unroll
            for (int t = 0; t < R; ++t) al[c * R + t] += bv[u][c] * pv[u][t];
      }
      for (; k < wh; ++k) {
        const int64_t e = e0 + (int64_t)k * kStride;
        const T* xp = x + offV + (int64_t)sb_col[e] * R;
        T pv[R];
#pragma unroll
        for (int t = 0; t < R; ++t) pv[t] = xp[t];
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const T bv = uB[e * D + c];
#pragma unroll
          for (int t = 0; t < R; ++t) al[c * R + t] += bv * pv[t];
        }
      }
    }
  } else if (sl < nsu + nsp) {
    // vertex rows: the R sums go to am[0 .. R)
    const int64_t ps = sl - nsu;
    const int w = sp_w[ps];
    const int wh = w > half ? (w - half + NW - 1) / NW : 0;
    const int64_t e0 = sp_off[ps] + (int64_t)half * 64 + lane;
    int32_t jn[kSellUnroll];
    if (kSellUnroll <= wh)
#pragma unroll
      for (int u = 0; u < kSellUnroll; ++u) jn[u] = sp_col[e0 + (int64_t)u * kStride];
    int k = 0;
    for (; k + kSellUnroll <= wh; k += kSellUnroll) {
      int32_t j[kSellUnroll];
      T xv[kSellUnroll][DR];
#pragma unroll
      for (int u = 0; u < kSellUnroll; ++u) j[u] = jn[u];
#pragma unroll
      for (int u = 0; u < kSellUnroll; ++u)
#pragma unroll
        for (int q = 0; q < DR; ++q) xv[u][q] = x[(int64_t)j[u] * DR + q];
      if (k + 2 * kSellUnroll <= wh)
#pragma unroll
        for (int u = 0; u < kSellUnroll; ++u) jn[u] = sp_col[e0 + (int64_t)(k + kSellUnroll + u) * kStride];
#pragma unroll
      for (int u = 0; u < kSellUnroll; ++u) {
        const int64_t e = e0 + (int64_t)(k + u) * kStride;
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const T bv = pBt[e * D + c];
#pragma unroll
          for (int t = 0; t < R; ++t) am[t] += bv * xv[u][c * R + t];
        }
      }
    }
    for (; k < wh; ++k) {
      const int64_t e = e0 + (int64_t)k * kStride;
      const T* xi = x + (int64_t)sp_col[e] * DR;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const T bv = pBt[e * D + c];
#pragma unroll
        for (int t = 0; t < R; ++t) am[t] += bv * xi[c * R + t];
      }
    }
  }
  if constexpr (NW == 2) {
    if (half) {
#pragma unroll
      for (int q = 0; q < DR; ++q) {
        part[pair][q][lane] = am[q];
        part[pair][DR + q][lane] = al[q];
      }
    }
    __syncthreads();
    if (half) return;
#pragma unroll
    for (int q = 0; q < DR; ++q) {
      am[q] += part[pair][q][lane];
      al[q] += part[pair][DR + q][lane];
    }
  }
  if (sl < nsu) {
    const int64_t row = sl * 64 + lane;
    if (row < nfree) {
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int s = 0; s < R; ++s) {
          T acc = am[c * R + s];
#pragma unroll
          for (int t = 0; t < R; ++t) acc += dtA.v[s * R + t] * al[c * R + t];
          const int64_t o = row * DR + c * R + s;
          y[o] = F ? F[o] - acc : acc;
        }
    }
  } else if (sl < nsu + nsp) {
    const int64_t v = (sl - nsu) * 64 + lane;
    if (v < nv) {
#pragma unroll
      for (int s = 0; s < R; ++s) {
        T acc = T(0);
#pragma unroll
        for (int t = 0; t < R; ++t) acc += dtA.v[s * R + t] * am[t];
        const int64_t o = offV + v * R + s;
        y[o] = F ? F[o] - acc : acc;
      }
    }
  }
}

// r = F - J x (F null: r = J x) for the Newton Jacobian of the Navier--Stokes stage
// equations (Sec. 3.2): block (s, t) = delta_st M + dt a_st [N_s B; B^T 0] with the
// per-stage velocity operator N_s = K + N'(U_s) kept as dim x dim blocks on the scalar
// pattern.  N_s depends on the row's stage, so each gathered column is first mixed into
// its stage combinations z_s = sum_t dt a_st x_t and N_s applied to z_s; the B part is
// stage-independent and mixed once per row.  The sliced layout of k_residual_sell (a
// wavefront per slice of 64 rows, lane = row, velocity slices then vertex slices), with
// the blocks copied to the sliced order by k_sell_blocks: value q of sliced entry e at
// ((e / 64) R D^2 + q) 64 + e mod 64, so that every value is one coalesced load.  Each
// row sums its entries in CSR order (padding entries add zeros); with NW = 2 (levels of
// fewer than kSplitSlices slices, latency-bound) two wavefronts take alternate entries of
// a slice and add their sums through LDS.
template <int D, int R, int NW>
__global__ __launch_bounds__(256) void k_residual_newton_sell(
    int64_t nfree, int64_t nv, int64_t offV, int64_t nsu, int64_t nsp, const int32_t* __restrict__ su_off,
    const int32_t* __restrict__ su_w, const int32_t* __restrict__ su_col, const double* __restrict__ uM,
    const double* __restrict__ nws, const int32_t* __restrict__ sb_off, const int32_t* __restrict__ sb_w,
    const int32_t* __restrict__ sb_col, const double* __restrict__ uB, const int32_t* __restrict__ sp_off,
    const int32_t* __restrict__ sp_w, const int32_t* __restrict__ sp_col, const double* __restrict__ pBt,
    Coef<double> dtA, const double* __restrict__ F, const double* __restrict__ x, double* __restrict__ y) {
  constexpr int DR = D * R, RDD = R * D * D;
  constexpr int kSlices = 4 / NW;  // slices per workgroup of four wavefronts
  __shared__ double part[NW == 2 ? kSlices : 1][NW == 2 ? 2 * DR : 1][64];
  const int lane = threadIdx.x & 63;
  const int half = (threadIdx.x >> 6) % NW;
  const int pair = (threadIdx.x >> 6) / NW;
  const int64_t sl = (int64_t)blockIdx.x * kSlices + pair;
  // wavefront `half` of the slice takes entries k = half, half + NW, ...
  double acc[DR], ab[DR];
#pragma unroll
  for (int q = 0; q < DR; ++q) acc[q] = ab[q] = 0.0;
  if (sl < nsu) {
    {
      const int w = su_w[sl];
      const int64_t e0 = su_off[sl] + lane;
      for (int k = half; k < w; k += NW) {
        const int64_t e = e0 + (int64_t)k * 64;
        const int64_t j = su_col[e];
        double xv[DR], z[DR];
#pragma unroll
        for (int q = 0; q < DR; ++q) xv[q] = x[j * DR + q];
        const double m = uM[e];
#pragma unroll
        for (int ee = 0; ee < D; ++ee)
#pragma unroll
          for (int st = 0; st < R; ++st) {
            double v = 0.0;
#pragma unroll
            for (int t = 0; t < R; ++t) v += dtA.v[st * R + t] * xv[ee * R + t];
            z[ee * R + st] = v;
          }
        const double* nwp = nws + (e >> 6) * RDD * 64 + lane;
#pragma unroll
        for (int st = 0; st < R; ++st)
#pragma unroll
          for (int c = 0; c < D; ++c) {
            double v = m * xv[c * R + st];
#pragma unroll
            for (int ee = 0; ee < D; ++ee) v += nwp[(int64_t)((st * D + c) * D + ee) * 64] * z[ee * R + st];
            acc[c * R + st] += v;
          }
      }
    }
    {
      const int w = sb_w[sl];
      const int64_t e0 = sb_off[sl] + lane;
      for (int k = half; k < w; k += NW) {
        const int64_t e = e0 + (int64_t)k * 64;
        const int64_t v = sb_col[e];
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const double bv = uB[e * D + c];
#pragma unroll
          for (int t = 0; t < R; ++t) ab[c * R + t] += bv * x[offV + v * R + t];
        }
      }
    }
  } else if (sl < nsu + nsp) {
    // vertex rows: the R sums go to acc[0 .. R)
    const int64_t ps = sl - nsu;
    const int w = sp_w[ps];
    const int64_t e0 = sp_off[ps] + lane;
    for (int k = half; k < w; k += NW) {
      const int64_t e = e0 + (int64_t)k * 64;
      const int64_t j = sp_col[e];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const double bv = pBt[e * D + c];
#pragma unroll
        for (int t = 0; t < R; ++t) acc[t] += bv * x[j * DR + c * R + t];
      }
    }
  }
  if constexpr (NW == 2) {
    if (half) {
#pragma unroll
      for (int q = 0; q < DR; ++q) {
        part[pair][q][lane] = acc[q];
        part[pair][DR + q][lane] = ab[q];
      }
    }
    __syncthreads();
    if (half) return;
#pragma unroll
    for (int q = 0; q < DR; ++q) {
      acc[q] += part[pair][q][lane];
      ab[q] += part[pair][DR + q][lane];
    }
  }
  if (sl < nsu) {
    const int64_t row = sl * 64 + lane;
    if (row < nfree) {
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int st = 0; st < R; ++st) {
          double v = acc[c * R + st];
#pragma unroll
          for (int t = 0; t < R; ++t) v += dtA.v[st * R + t] * ab[c * R + t];
          const int64_t o = row * DR + c * R + st;
          y[o] = F ? F[o] - v : v;
        }
    }
  } else if (sl < nsu + nsp) {
    const int64_t vx = (sl - nsu) * 64 + lane;
    if (vx < nv) {
#pragma unroll
      for (int st = 0; st < R; ++st) {
        double v = 0.0;
#pragma unroll
        for (int t = 0; t < R; ++t) v += dtA.v[st * R + t] * acc[t];
        const int64_t o = offV + vx * R + st;
        y[o] = F ? F[o] - v : v;
      }
    }
  }
}

// Values of a CSR value array (k per entry) in the sliced order of k_residual_newton_sell:
// out[((e / 64) k + q) 64 + e mod 64] = v[src[e] k + q], zero for padding (src < 0).
__global__ __launch_bounds__(kBlock) void k_sell_blocks(int64_t ne, int k, const int32_t* __restrict__ src,
                                                        const double* __restrict__ v, double* __restrict__ out) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= ne * k) return;
  const int64_t rest = o >> 6, blk = rest / k;
  const int q = (int)(rest - blk * k);
  const int64_t e = blk * 64 + (o & 63);
  const int32_t p = src[e];
  out[o] = p >= 0 ? v[(int64_t)p * k + q] : 0.0;
}

// ------------------------------------------------------------------ patch factorise
// One workgroup per patch, matrix in dynamic LDS (row-major n x n).  With nw (the
// Newton Jacobian's per-stage dim x dim blocks, as for k_residual_newton) the
// velocity-velocity entries are delta_st delta_ce M_ab + dt a_st N_s[ab]_ce instead of
// the Kronecker delta_st M_ab + dt a_st L_ab on each component.
// Rows [r0, r1) of the patch matrix, row-major with stride n from row r0, zeroed and filled
// by the workgroup (ends with a barrier).  With nw (the Newton Jacobian's per-stage dim x dim blocks, as for
// k_residual_newton) the velocity-velocity entries are delta_st delta_ce M_ab + dt a_st
// N_s[ab]_ce instead of the Kronecker delta_st M_ab + dt a_st L_ab on each component.
template <int D, int R, typename T>
__device__ void assemble_patch(int64_t p, int nn, int n, const int32_t* __restrict__ pn_ptr,
                               const int32_t* __restrict__ pvv_ptr, const int32_t* __restrict__ pvv,
                               const int32_t* __restrict__ pvp, const T* __restrict__ sM, const T* __restrict__ sL,
                               const T* __restrict__ b_val, const Coef<T>& dtA, const T* __restrict__ nw, int r0,
                               int r1, T* Am) {
  const int sb = D * nn + 1;  // per-stage block size
  const int tid = threadIdx.x;
  for (int e = tid; e < (r1 - r0) * n; e += blockDim.x) Am[e] = T(0);
  __syncthreads();
  auto put = [&](int row, int col, T v) {
    if (row >= r0 && row < r1) Am[(row - r0) * n + col] = v;
  };
  // velocity-velocity: delta_st M_ab + dt a_st L_ab on every component
  const int32_t v0 = pvv_ptr[p], v1 = pvv_ptr[p + 1];
  for (int32_t e = v0 + tid; e < v1; e += blockDim.x) {
    const int la = pvv[3 * e], lb = pvv[3 * e + 1], pos = pvv[3 * e + 2];
    const T m = sM[pos];
    if (nw) {
      const T* nwp = nw + (int64_t)pos * R * D * D;
#pragma unroll 1
      for (int c = 0; c < D; ++c)
#pragma unroll 1
        for (int ce = 0; ce < D; ++ce)
          for (int s = 0; s < R; ++s)
            for (int t = 0; t < R; ++t)
              put(s * sb + c * nn + la, t * sb + ce * nn + lb,
                  (s == t && c == ce ? m : T(0)) + dtA.v[s * R + t] * nwp[(s * D + c) * D + ce]);
      continue;
    }
    const T l = sL[pos];
#pragma unroll 1
    for (int c = 0; c < D; ++c)
#pragma unroll 1
      for (int s = 0; s < R; ++s)
        for (int t = 0; t < R; ++t)
          put(s * sb + c * nn + la, t * sb + c * nn + lb, (s == t ? m : T(0)) + dtA.v[s * R + t] * l);
  }
  // velocity-pressure couplings with the patch vertex: dt a_st B and dt a_st B^T
  const int32_t n0 = pn_ptr[p];
  for (int la = tid; la < nn; la += blockDim.x) {
    const int pos = pvp[n0 + la];
    if (pos < 0) continue;
#pragma unroll 1
    for (int c = 0; c < D; ++c) {
      const T bv = b_val[(int64_t)pos * D + c];
      for (int s = 0; s < R; ++s)
        for (int t = 0; t < R; ++t) {
          const T val = dtA.v[s * R + t] * bv;
          put(s * sb + c * nn + la, t * sb + D * nn, val);
          put(s * sb + D * nn, t * sb + c * nn + la, val);
        }
    }
  }
  __syncthreads();
}

// One workgroup per patch, matrix in dynamic LDS (row-major n x n).
template <int D, int R, typename T>
__global__ __launch_bounds__(kBlock) void k_patch_factor(
    int64_t npatch, const int32_t* __restrict__ pn_ptr, const int32_t* __restrict__ pvv_ptr,
    const int32_t* __restrict__ pvv, const int32_t* __restrict__ pvp,
    const int32_t* __restrict__ p_ld, const int64_t* __restrict__ p_inv_off,
    const T* __restrict__ sM, const T* __restrict__ sL, const T* __restrict__ b_val,
    Coef<T> dtA, T* __restrict__ inv, int* __restrict__ fail, int64_t p0, int64_t off0,
    const T* __restrict__ nw) {
  extern __shared__ unsigned char smem_raw[];
  const int64_t p = p0 + blockIdx.x;
  if (p >= npatch) return;
  const int nn = pn_ptr[p + 1] - pn_ptr[p];
  const int n = R * (D * nn + 1);
  T* Am = reinterpret_cast<T*>(smem_raw);
  T* colk = Am + (size_t)n * n;
  int* perm = reinterpret_cast<int*>(colk + n);
  __shared__ int s_piv;
  __shared__ T s_best;
  const int tid = threadIdx.x;
  assemble_patch<D, R, T>(p, nn, n, pn_ptr, pvv_ptr, pvv, pvp, sM, sL, b_val, dtA, nw, 0, n, Am);
  // in-place Gauss--Jordan with partial pivoting (ties -> smallest row index)
  for (int kk = 0; kk < n; ++kk) {
    if (tid < 64) {
      T best = T(-1);
      int bi = kk;
      for (int i = kk + tid; i < n; i += 64) {
        const T a = fabs(Am[i * n + kk]);
        if (a > best) {
          best = a;
          bi = i;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const T ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (tid == 0) {
        s_piv = bi;
        s_best = best;
        perm[kk] = bi;
      }
    }
    __syncthreads();
    const int piv = s_piv;
    if (!(s_best > T(0))) {
      if (tid == 0) atomicMax(fail, 1);
      return;  // uniform across the workgroup
    }
    if (piv != kk)
      for (int j = tid; j < n; j += blockDim.x) {
        const T t = Am[kk * n + j];
        Am[kk * n + j] = Am[piv * n + j];
        Am[piv * n + j] = t;
      }
    __syncthreads();
    const T ip = T(1) / Am[kk * n + kk];
    for (int i = tid; i < n; i += blockDim.x) colk[i] = Am[i * n + kk];
    __syncthreads();
    for (int j = tid; j < n; j += blockDim.x) Am[kk * n + j] = (j == kk ? ip : Am[kk * n + j] * ip);
    __syncthreads();
    for (int e = tid; e < n * n; e += blockDim.x) {
      const int i = e / n, j = e - i * n;
      if (i == kk) continue;
      const T base = (j == kk) ? T(0) : Am[e];
      Am[e] = base - colk[i] * Am[kk * n + j];
    }
    __syncthreads();
  }
  for (int kk = n - 1; kk >= 0; --kk) {
    const int q = perm[kk];
    if (q != kk)
      for (int i = tid; i < n; i += blockDim.x) {
        const T t = Am[i * n + kk];
        Am[i * n + kk] = Am[i * n + q];
        Am[i * n + q] = t;
      }
    __syncthreads();
  }
  const int ld = p_ld[p];
  T* out = inv + (p_inv_off[p] - off0);
  for (int e = tid; e < n * ld; e += blockDim.x) {
    const int j = e / ld, i = e - j * ld;
    out[e] = i < n ? Am[i * n + j] : T(0);
  }
}

// Register-tiled Gauss--Jordan for mid-sized patches (64 < n <= 32 TM, TM <= 4): the
// matrix is assembled in LDS, then each of 1024 threads keeps a TM x TM tile of it in
// registers (wavefront w holds column tiles 2w and 2w + 1; lane l the row tile l mod 32
// of column tile 2w + l / 32).  Pivoting is implicit, the exchange form of Gauss--Jordan
// without row swaps: at step k the unused row p with the largest |a_pk| (smallest index
// on ties) becomes the pivot row of column k, so every register keeps its matrix
// position.  Row p is kept unscaled, multiplied by a_pk (its multiplier in step k is 0
// and its column-k entry becomes 1); the updates are linear in the row, so it stays so
// scaled, and it is divided by a_pk once, when the inverse is written.  The wavefront
// owning the next column publishes that column, its pivot and the reciprocal to LDS
// during the update, and one barrier separates the steps; the pivot row reaches the
// other lanes of its wavefront by a lane permutation.  At the end entry
// (i, j) of the exchanged matrix is entry (step at which row i was the pivot, pivot row
// of step j) of the inverse.
constexpr int kRtThreads = 1024;
// Rows per LDS pass of the register-tiled kernel: half of n, rounded up to whole tiles.
__host__ __device__ constexpr int rt_half_rows(int n, int tm) { return ((n + 1) / 2 + tm - 1) / tm * tm; }
// A thread's tile, entry (a, c) at a * TM + c: one vector value of at most 1024 bits, so
// that selecting a column by a wavefront-uniform index stays in registers (indexed
// register moves).
template <typename T, int TM>
struct RtTile {
  static_assert(TM * TM <= 16, "tile of at most 16 entries");
  typedef T type __attribute__((ext_vector_type(16)));
};

// Cross-lane moves for the register-tiled kernel: DPP lane permutations within rows of 16
// lanes (quad_perm [1,0,3,2] and [2,3,0,1], row_half_mirror, row_mirror) and reads of
// one lane (uniform lane index).
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_read(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float lane_read(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Column q of the register tiles of k_patch_factor_rt and its pivot (largest |a_iq| over
// the rows not yet used, smallest index on ties), by the wavefront that owns the
// column: the column into colbuf with the pivot row's entry 0, the pivot row into *piv
// (-1 for a zero or missing pivot) and its reciprocal into *ipv.  The largest magnitude
// comes from a butterfly of lane permutations over each row of 16 lanes and the two
// rows of the column's half, the pivot from the first lane holding it (lanes hold
// increasing rows).
template <typename T, int TM>
__device__ __forceinline__ void rt_publish(const typename RtTile<T, TM>::type& t, unsigned used, int q, int n,
                                           int w, int lane, T* colbuf, int* piv, T* ipv) {
  constexpr int NP = 32 * TM;
  const int cq = q / TM;
  if ((cq >> 1) != w) return;  // uniform across the wavefront
  const int cc = q - cq * TM, i0 = (lane & 31) * TM, hq = cq & 1;
  const bool mine = (lane >> 5) == hq;
  T best = T(-1), bv = T(0);
  int bi = NP;
  if (mine) {
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      const T v = t[a * TM + cc];
      if (i0 + a < n) {
        colbuf[i0 + a] = v;
        const T mag = fabs(v);
        if (!((used >> a) & 1u) && mag > best) {
          best = mag;
          bv = v;
          bi = i0 + a;
        }
      }
    }
  }
  T mx = best;
  mx = fmax(mx, dpp_mov<0xB1>(mx));
  mx = fmax(mx, dpp_mov<0x4E>(mx));
  mx = fmax(mx, dpp_mov<0x141>(mx));
  mx = fmax(mx, dpp_mov<0x140>(mx));
  const T gm = fmax(lane_read(mx, hq << 5), lane_read(mx, (hq << 5) + 16));
  const unsigned long long hit = __ballot(mine && best == gm);
  const int L = hit ? __ffsll((long long)hit) - 1 : 0;
  const int pb = __builtin_amdgcn_readlane(bi, L);
  const T pvv = hit ? lane_read(bv, L) : T(0);
  if (lane == 0) {
    const bool ok = pvv != T(0) && pb >= 0 && pb < n;
    *piv = ok ? pb : -1;
    *ipv = ok ? T(1) / pvv : T(0);
    if (ok) colbuf[pb] = T(0);  // after the column's writes (one wavefront, in order)
  }
}

template <int D, int R, typename T, int TM>
__global__ __launch_bounds__(kRtThreads, 8) void k_patch_factor_rt(
    int64_t npatch, const int32_t* __restrict__ pn_ptr, const int32_t* __restrict__ pvv_ptr,
    const int32_t* __restrict__ pvv, const int32_t* __restrict__ pvp,
    const int32_t* __restrict__ p_ld, const int64_t* __restrict__ p_inv_off,
    const T* __restrict__ sM, const T* __restrict__ sL, const T* __restrict__ b_val,
    Coef<T> dtA, T* __restrict__ inv, int* __restrict__ fail, int64_t p0, int64_t off0,
    const T* __restrict__ nw) {
  constexpr int NP = 32 * TM;
  extern __shared__ unsigned char smem_raw[];
  __shared__ T colbuf[2][NP];
  __shared__ T s_ip[2];            // reciprocal of the pivot
  __shared__ int s_piv[2];         // pivot row (-1: zero pivot)
  __shared__ int s_pivrow[NP];     // pivot row of each step
  __shared__ int s_rowstep[NP];    // step at which each row was the pivot
  __shared__ T s_rowip[NP];        // reciprocal of each row's pivot
  const int64_t p = p0 + blockIdx.x;
  if (p >= npatch) return;
  const int nn = pn_ptr[p + 1] - pn_ptr[p];
  const int n = R * (D * nn + 1);
  T* Am = reinterpret_cast<T*>(smem_raw);
  const int tid = threadIdx.x;
  for (int e = tid; e < 2 * NP; e += kRtThreads) colbuf[e / NP][e % NP] = T(0);
  const int w = tid >> 6, lane = tid & 63, half = lane >> 5, ri = lane & 31;
  const int i0 = ri * TM, j0 = (2 * w + half) * TM;
  // the matrix passes through LDS in two halves of rows (hr rows, a multiple of TM, each),
  // so that two patches' workgroups fit on a CU
  const int hr = rt_half_rows(n, TM);
  typename RtTile<T, TM>::type t;
  for (int r0 = 0; r0 < n; r0 += hr) {
    const int r1 = min(n, r0 + hr);
    assemble_patch<D, R, T>(p, nn, n, pn_ptr, pvv_ptr, pvv, pvp, sM, sL, b_val, dtA, nw, r0, r1, Am);
    if (i0 >= r0 && i0 < r1) {
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int c = 0; c < TM; ++c)
          t[a * TM + c] = (i0 + a < n && j0 + c < n) ? Am[(i0 + a - r0) * n + j0 + c] : T(0);
    }
    __syncthreads();
  }
  if (i0 >= n) {
#pragma unroll
    for (int e = 0; e < TM * TM; ++e) t[e] = T(0);
  }
  unsigned used = 0;  // bit a: row i0 + a has been a pivot row
  rt_publish<T, TM>(t, used, 0, n, w, lane, colbuf[0], &s_piv[0], &s_ip[0]);
  __syncthreads();
  for (int kk = 0; kk < n; ++kk) {
    const int buf = kk & 1;
    const int pv = __builtin_amdgcn_readfirstlane(s_piv[buf]);
    const T ip = s_ip[buf];
    T m[TM];
#pragma unroll
    for (int a = 0; a < TM; ++a) m[a] = colbuf[buf][i0 + a];
    if (pv < 0) {
      if (tid == 0) atomicMax(fail, 1);
      return;  // uniform across the workgroup
    }
    const int pr = pv / TM, pa = pv - pr * TM;
    // the pivot row of this lane's columns, from lane pr of this half
    T rrow[TM];
    const int src = (half << 5) + pr;
#pragma unroll
    for (int c = 0; c < TM; ++c) rrow[c] = __shfl(t[pa * TM + c], src, 64) * ip;
    if (ri == pr) used |= 1u << pa;
    const int ck = kk / TM;
    if ((ck >> 1) == w) {
      // the wavefront holding column kk: the column becomes -a_ik / pivot, and 1 in the
      // (unscaled) pivot row
      const bool own = half == (ck & 1);
      const int cc = kk - ck * TM;
#pragma unroll
      for (int c = 0; c < TM; ++c)
        if (own && c == cc) rrow[c] = ip;
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int c = 0; c < TM; ++c)
          t[a * TM + c] = ((own && c == cc) ? (i0 + a == pv ? T(1) : T(0)) : t[a * TM + c]) - m[a] * rrow[c];
    } else {
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int c = 0; c < TM; ++c) t[a * TM + c] = t[a * TM + c] - m[a] * rrow[c];
    }
    if (tid == 0) {
      s_pivrow[kk] = pv;
      s_rowstep[pv] = kk;
      s_rowip[pv] = ip;
    }
    if (kk + 1 < n) rt_publish<T, TM>(t, used, kk + 1, n, w, lane, colbuf[buf ^ 1], &s_piv[buf ^ 1], &s_ip[buf ^ 1]);
    __syncthreads();
  }
  // the inverse, column-major, staged in LDS by halves of its columns and written out with
  // whole columns
  const int ld = p_ld[p];
  T* out = inv + (p_inv_off[p] - off0);
  for (int c0 = 0; c0 < n; c0 += hr) {
    const int c1 = min(n, c0 + hr);
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int c = 0; c < TM; ++c)
        if (i0 + a < n && j0 + c < n) {
          const int b = s_pivrow[j0 + c];
          if (b >= c0 && b < c1) Am[(b - c0) * n + s_rowstep[i0 + a]] = t[a * TM + c] * s_rowip[i0 + a];
        }
    __syncthreads();
    for (int e = tid; e < (c1 - c0) * ld; e += kRtThreads) {
      const int j = e / ld, i = e - j * ld;
      out[(int64_t)c0 * ld + e] = i < n ? Am[j * n + i] : T(0);
    }
    __syncthreads();
  }
}

// The LDS-resident factorisation of patches of up to n unknowns: the register-tiled
// kernel for 64 < n <= 128, else the kernel with the whole matrix in LDS.
template <int D, int RR, typename T>
hipError_t launch_patch_factor_lds(unsigned g, size_t n, size_t lds, hipStream_t s, int64_t npatch,
                                   const int32_t* pn_ptr, const int32_t* pvv_ptr, const int32_t* pvv,
                                   const int32_t* pvp, const int32_t* ld, const int64_t* off, const T* sM,
                                   const T* sL, const T* b_val, Coef<T> cf, T* out, int* d_fail, int64_t p0,
                                   int64_t off0, const T* nw) {
  auto go = [&](auto kern, unsigned block, size_t bytes) -> hipError_t {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    kern<<<dim3(g), dim3(block), bytes, s>>>(npatch, pn_ptr, pvv_ptr, pvv, pvp, ld, off, sM, sL, b_val, cf, out,
                                             d_fail, p0, off0, nw);
    return hipGetLastError();
  };
  if constexpr (D < 3) {
    // static LDS of the register-tiled kernel: two columns, the row reciprocals, two
    // permutations
    // dynamic LDS: half of the rows (two workgroups per CU share its 160 KB)
    auto rt = [&](int tm) { return (size_t)rt_half_rows((int)n, tm) * n * sizeof(T); };
    auto fits = [&](int tm) {
      return rt(tm) + (size_t)96 * tm * sizeof(T) + (size_t)64 * tm * sizeof(int) + 64 <= 80 * 1024;
    };
    if (n > 64 && n <= 96 && fits(3)) return go(k_patch_factor_rt<D, RR, T, 3>, kRtThreads, rt(3));
    if (n > 96 && n <= 128 && fits(4)) return go(k_patch_factor_rt<D, RR, T, 4>, kRtThreads, rt(4));
  }
  return go(k_patch_factor<D, RR, T>, kBlock, lds);
}

// Patches too large for LDS: the matrix is assembled straight into its column-major
// inverse slot (n x ld) and inverted in place by the same Gauss--Jordan recurrence,
// blocked: a panel of BW columns is reduced in LDS (pivot search, row swaps, scaling,
// elimination within the panel), the panel's row swaps are applied to every other
// column, and the other columns receive the panel's transform as a rank-BW update
//   A[:, j] <- (A[:, j] with the panel's pivot rows zeroed) + P * A_old[pivot rows, j].
// Each thread keeps its rows of P in registers during the update.
constexpr int kGjBw = 16;     // panel width
constexpr int kGjJt = 64;     // columns per update tile
constexpr int kGjRows = 4;    // rows per thread (n <= 1024)

// Rank-bw update of k_patch_factor_global on the matrix cores (FP64): the columns outside
// the panel [kb, kb + bw) receive A[:, j] <- (A[:, j], pivot rows zeroed) + P A_old[pivot rows,
// j], P the panel's transform (P[c n + i], LDS), in tiles of 16 rows x 16 columns, one
// wavefront per tile, the tile accumulated by four v_mfma_f64_16x16x4 steps over the bw <= 16
// panel columns.  The product is formed transposed (A_old[pivot rows, j]^T P^T) so that
// the accumulator's lanes run along rows: lane l, element v of a tile holds row
// i0 + l mod 16 of column j0 + l / 16 + 4 v, and 16 lanes read and write 16 consecutive
// entries of one column.  Operand layouts of the instruction: lane l holds A(l mod 16,
// l / 16), B(l / 16, l mod 16).  Ak stages the pivot rows of kGjJt columns at a time.
__device__ __forceinline__ void gj_update_mfma(double* __restrict__ Am, int ld, int n, int kb, int bw,
                                               const double* P, double* Ak) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
  const int lr = ln & 15, lk = ln >> 4;
  const int nrt = (n + 15) / 16;
  for (int j0 = 0; j0 < n; j0 += kGjJt) {
    const int jt = min(kGjJt, n - j0);
    for (int e = tid; e < kGjBw * kGjJt; e += blockDim.x) {
      const int c = e / kGjJt, jj = e - c * kGjJt;
      Ak[e] = (c < bw && jj < jt) ? Am[(int64_t)(j0 + jj) * ld + kb + c] : 0.0;
    }
    __syncthreads();
    const int nct = (jt + 15) / 16;
    for (int tI = wv; tI < nrt * nct; tI += blockDim.x / 64) {
      const int rt = tI / nct, ct = tI - rt * nct;
      const int i = rt * 16 + lr;  // this lane's row
      const bool rok = i < n, rpan = i >= kb && i < kb + bw;
      d4 acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int jj = ct * 16 + lk + 4 * v, j = j0 + jj;
        const bool cok = jj < jt && !(j >= kb && j < kb + bw);
        acc[v] = (cok && rok && !rpan) ? Am[(int64_t)j * ld + i] : 0.0;
      }
#pragma unroll
      for (int kq = 0; kq < kGjBw / 4; ++kq) {
        const int c = kq * 4 + lk;
        const double a = Ak[c * kGjJt + ct * 16 + lr];  // A(lr, lk): pivot row c, column ct*16 + lr
        const double b = (c < bw && rok) ? P[c * n + i] : 0.0;  // B(lk, lr): P(i, c)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int jj = ct * 16 + lk + 4 * v, j = j0 + jj;
        if (jj < jt && !(j >= kb && j < kb + bw) && rok) Am[(int64_t)j * ld + i] = acc[v];
      }
    }
    __syncthreads();
  }
}

template <int D, int R, typename T>
__global__ __launch_bounds__(kBlock) void k_patch_factor_global(
    int64_t npatch, const int32_t* __restrict__ pn_ptr, const int32_t* __restrict__ pvv_ptr,
    const int32_t* __restrict__ pvv, const int32_t* __restrict__ pvp,
    const int32_t* __restrict__ p_ld, const int64_t* __restrict__ p_inv_off,
    const T* __restrict__ sM, const T* __restrict__ sL, const T* __restrict__ b_val,
    Coef<T> dtA, T* __restrict__ inv, int* __restrict__ fail, int64_t p0, int64_t off0,
    const T* __restrict__ nw) {
  extern __shared__ unsigned char smem_raw[];
  const int64_t p = p0 + blockIdx.x;
  if (p >= npatch) return;
  const int nn = pn_ptr[p + 1] - pn_ptr[p];
  const int sb = D * nn + 1;
  const int n = R * sb;
  const int ld = p_ld[p];
  T* __restrict__ Am = inv + (p_inv_off[p] - off0);  // column-major: Am[j * ld + i]
  T* P = reinterpret_cast<T*>(smem_raw);    // panel, P[c * n + i]
  T* colk = P + (size_t)kGjBw * n;
  T* Ak = colk + n;                          // Ak[c * kGjJt + jj]
  int* perm = reinterpret_cast<int*>(Ak + kGjBw * kGjJt);
  __shared__ int s_piv;
  __shared__ T s_best;
  const int tid = threadIdx.x;
  for (int64_t e = tid; e < (int64_t)n * ld; e += blockDim.x) Am[e] = T(0);
  __syncthreads();
  const int32_t v0 = pvv_ptr[p], v1 = pvv_ptr[p + 1];
  for (int32_t e = v0 + tid; e < v1; e += blockDim.x) {
    const int la = pvv[3 * e], lb = pvv[3 * e + 1], pos = pvv[3 * e + 2];
    const T m = sM[pos];
    if (nw) {
      const T* nwp = nw + (int64_t)pos * R * D * D;
      for (int c = 0; c < D; ++c)
        for (int ce = 0; ce < D; ++ce)
          for (int s = 0; s < R; ++s)
            for (int t = 0; t < R; ++t)
              Am[(int64_t)(t * sb + ce * nn + lb) * ld + (s * sb + c * nn + la)] =
                  (s == t && c == ce ? m : T(0)) + dtA.v[s * R + t] * nwp[(s * D + c) * D + ce];
      continue;
    }
    const T l = sL[pos];
    for (int c = 0; c < D; ++c)
      for (int s = 0; s < R; ++s)
        for (int t = 0; t < R; ++t)
          Am[(int64_t)(t * sb + c * nn + lb) * ld + (s * sb + c * nn + la)] =
              (s == t ? m : T(0)) + dtA.v[s * R + t] * l;
  }
  const int32_t n0 = pn_ptr[p];
  for (int la = tid; la < nn; la += blockDim.x) {
    const int pos = pvp[n0 + la];
    if (pos < 0) continue;
    for (int c = 0; c < D; ++c) {
      const T bv = b_val[(int64_t)pos * D + c];
      for (int s = 0; s < R; ++s)
        for (int t = 0; t < R; ++t) {
          const T val = dtA.v[s * R + t] * bv;
          Am[(int64_t)(t * sb + D * nn) * ld + (s * sb + c * nn + la)] = val;
          Am[(int64_t)(t * sb + c * nn + la) * ld + (s * sb + D * nn)] = val;
        }
    }
  }
  __syncthreads();
  for (int kb = 0; kb < n; kb += kGjBw) {
    const int bw = min(kGjBw, n - kb);
    for (int e = tid; e < bw * n; e += blockDim.x) {
      const int c = e / n, i = e - c * n;
      P[c * n + i] = Am[(int64_t)(kb + c) * ld + i];
    }
    __syncthreads();
    for (int cc = 0; cc < bw; ++cc) {
      const int c = kb + cc;
      if (tid < 64) {
        T best = T(-1);
        int bi = c;
        for (int i = c + tid; i < n; i += 64) {
          const T a = fabs(P[cc * n + i]);
          if (a > best) {
            best = a;
            bi = i;
          }
        }
        for (int off = 32; off > 0; off >>= 1) {
          const T ob = __shfl_xor(best, off, 64);
          const int oi = __shfl_xor(bi, off, 64);
          if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
          }
        }
        if (tid == 0) {
          s_piv = bi;
          s_best = best;
          perm[c] = bi;
        }
      }
      __syncthreads();
      const int piv = s_piv;
      if (!(s_best > T(0))) {
        if (tid == 0) atomicMax(fail, 1);
        return;  // uniform across the workgroup
      }
      if (piv != c && tid < bw) {
        const T t = P[tid * n + c];
        P[tid * n + c] = P[tid * n + piv];
        P[tid * n + piv] = t;
      }
      __syncthreads();
      const T ip = T(1) / P[cc * n + c];
      for (int i = tid; i < n; i += blockDim.x) colk[i] = P[cc * n + i];
      __syncthreads();
      if (tid < bw) P[tid * n + c] = (tid == cc) ? ip : P[tid * n + c] * ip;
      __syncthreads();
      for (int e = tid; e < bw * n; e += blockDim.x) {
        const int q = e / n, i = e - q * n;
        if (i == c) continue;
        const T base = (q == cc) ? T(0) : P[q * n + i];
        P[q * n + i] = base - colk[i] * P[q * n + c];
      }
      __syncthreads();
    }
    // the panel's row swaps, in order, on every other column
    for (int cc = 0; cc < bw; ++cc) {
      const int c = kb + cc, q = perm[c];
      if (q != c)
        for (int j = tid; j < n; j += blockDim.x) {
          if (j >= kb && j < kb + bw) continue;
          const T t = Am[(int64_t)j * ld + c];
          Am[(int64_t)j * ld + c] = Am[(int64_t)j * ld + q];
          Am[(int64_t)j * ld + q] = t;
        }
      __syncthreads();
    }
    // rank-bw update of the other columns
    if constexpr (std::is_same<T, double>::value) {
      gj_update_mfma(Am, ld, n, kb, bw, P, Ak);
    } else {
    T pr[kGjRows][kGjBw];
#pragma unroll
    for (int rr = 0; rr < kGjRows; ++rr) {
      const int i = tid + rr * kBlock;
#pragma unroll
      for (int c = 0; c < kGjBw; ++c) pr[rr][c] = (i < n && c < bw) ? P[c * n + i] : T(0);
    }
    for (int j0 = 0; j0 < n; j0 += kGjJt) {
      const int jt = min(kGjJt, n - j0);
      for (int e = tid; e < bw * jt; e += blockDim.x) {
        const int c = e / jt, jj = e - c * jt;
        Ak[c * kGjJt + jj] = Am[(int64_t)(j0 + jj) * ld + kb + c];
      }
      __syncthreads();
      for (int jj = 0; jj < jt; ++jj) {
        const int j = j0 + jj;
        if (j >= kb && j < kb + bw) continue;
        T* col = Am + (int64_t)j * ld;
#pragma unroll
        for (int rr = 0; rr < kGjRows; ++rr) {
          const int i = tid + rr * kBlock;
          if (i >= n) continue;
          T acc = (i >= kb && i < kb + bw) ? T(0) : col[i];
#pragma unroll
          for (int c = 0; c < kGjBw; ++c) acc += pr[rr][c] * Ak[c * kGjJt + jj];
          col[i] = acc;
        }
      }
      __syncthreads();
    }
    }
    for (int e = tid; e < bw * n; e += blockDim.x) {
      const int c = e / n, i = e - c * n;
      Am[(int64_t)(kb + c) * ld + i] = P[c * n + i];
    }
    __syncthreads();
  }
  for (int kk = n - 1; kk >= 0; --kk) {
    const int q = perm[kk];
    if (q != kk)
      for (int i = tid; i < n; i += blockDim.x) {
        const T t = Am[(int64_t)kk * ld + i];
        Am[(int64_t)kk * ld + i] = Am[(int64_t)q * ld + i];
        Am[(int64_t)q * ld + i] = t;
      }
    __syncthreads();
  }
}

// ------------------------------------------------------------------- patch apply
using dev::Vec16;
constexpr int kWaves = 4;  // wavefronts (patches) per workgroup

template <typename T, int RB, int NMAX>
__global__ __launch_bounds__(kWaves * 64) void k_patch_apply(
    int64_t npatch, const int32_t* __restrict__ sched, const int32_t* __restrict__ p_nloc,
    const int32_t* __restrict__ p_ld, const int64_t* __restrict__ p_inv_off,
    const int64_t* __restrict__ p_slot_off, const int32_t* __restrict__ gidx,
    const T* __restrict__ inv, const T* __restrict__ res, const T* __restrict__ W,
    T* __restrict__ Y, int transpose, int D, int R) {
  __shared__ T xs[kWaves][NMAX];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t idx = (int64_t)blockIdx.x * kWaves + wave;
  if (idx >= npatch) return;  // whole wavefront exits; no workgroup barrier below
  dev::patch_apply_one<T, RB>(sched[idx], lane, xs[wave], p_nloc, p_ld, p_inv_off, p_slot_off, gidx, inv, res,
                              W, Y, transpose, D, R);
}

// A complex eigenvalue pair's block I (x) M_v + dt [[a, b], [-b, a]] (x) S_v is the real
// form of the complex matrix C = M_v + dt (a - ib) S_v, and its inverse's first block
// column is (Re C^{-1}; Im C^{-1}).  So the pair block is inverted as the n_s x n_s complex
// matrix: half the flops and a quarter of the LDS of the real 2 n_s block.  One workgroup
// per patch, complex Gauss--Jordan with partial pivoting on |z|^2 (ties to the smaller
// row) in LDS, result written straight into the factored layout as (re, im) pairs.
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void k_patch_factor_cplx(
    int64_t npatch, const int32_t* __restrict__ pn_ptr, const int32_t* __restrict__ pvv_ptr,
    const int32_t* __restrict__ pvv, const int32_t* __restrict__ pvp, const T* __restrict__ sM,
    const T* __restrict__ sL, const T* __restrict__ b_val, T zr, T zi, int blk, irk::StageBasis<T> sb,
    const int32_t* __restrict__ p_ld, const int64_t* __restrict__ p_inv_off, T* __restrict__ inv,
    int* __restrict__ fail) {
  constexpr int VEC = Vec16<T>::n;
  extern __shared__ unsigned char smem_raw[];
  const int64_t p = blockIdx.x;
  if (p >= npatch) return;
  const int nn = pn_ptr[p + 1] - pn_ptr[p];
  const int n = D * nn + 1;
  T* Ar = reinterpret_cast<T*>(smem_raw);  // real parts, row-major n x n
  T* Ai = Ar + (size_t)n * n;              // imaginary parts
  T* cr = Ai + (size_t)n * n;              // saved pivot column
  T* ci = cr + n;
  int* perm = reinterpret_cast<int*>(ci + n);
  __shared__ int s_piv;
  __shared__ T s_best;
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += blockDim.x) Ar[e] = Ai[e] = T(0);
  __syncthreads();
  const int32_t v0 = pvv_ptr[p], v1 = pvv_ptr[p + 1];
  for (int32_t e = v0 + tid; e < v1; e += blockDim.x) {
    const int la = pvv[3 * e], lb = pvv[3 * e + 1], pos = pvv[3 * e + 2];
    const T m = sM[pos], l = sL[pos];
    for (int c = 0; c < D; ++c) {
      Ar[(c * nn + la) * n + (c * nn + lb)] = m + zr * l;
      Ai[(c * nn + la) * n + (c * nn + lb)] = zi * l;
    }
  }
  const int32_t n0 = pn_ptr[p];
  for (int la = tid; la < nn; la += blockDim.x) {
    const int pos = pvp[n0 + la];
    if (pos < 0) continue;
    for (int c = 0; c < D; ++c) {
      const T bv = b_val[(int64_t)pos * D + c];
      Ar[(c * nn + la) * n + D * nn] = zr * bv;
      Ai[(c * nn + la) * n + D * nn] = zi * bv;
      Ar[(D * nn) * n + (c * nn + la)] = zr * bv;
      Ai[(D * nn) * n + (c * nn + la)] = zi * bv;
    }
  }
  __syncthreads();
  for (int kk = 0; kk < n; ++kk) {
    if (tid < 64) {
      T best = T(-1);
      int bi = kk;
      for (int i = kk + tid; i < n; i += 64) {
        const T a2 = Ar[i * n + kk] * Ar[i * n + kk] + Ai[i * n + kk] * Ai[i * n + kk];
        if (a2 > best) {
          best = a2;
          bi = i;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const T ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (tid == 0) {
        s_piv = bi;
        s_best = best;
        perm[kk] = bi;
      }
    }
    __syncthreads();
    const int piv = s_piv;
    if (!(s_best > T(0))) {
      if (tid == 0) atomicMax(fail, 1);
      return;  // uniform across the workgroup
    }
    if (piv != kk)
      for (int j = tid; j < n; j += blockDim.x) {
        T t = Ar[kk * n + j];
        Ar[kk * n + j] = Ar[piv * n + j];
        Ar[piv * n + j] = t;
        t = Ai[kk * n + j];
        Ai[kk * n + j] = Ai[piv * n + j];
        Ai[piv * n + j] = t;
      }
    __syncthreads();
    // 1 / pivot
    const T pr = Ar[kk * n + kk], pim = Ai[kk * n + kk];
    const T den = pr * pr + pim * pim;
    const T ipr = pr / den, ipi = -pim / den;
    for (int i = tid; i < n; i += blockDim.x) {
      cr[i] = Ar[i * n + kk];
      ci[i] = Ai[i * n + kk];
    }
    __syncthreads();
    for (int j = tid; j < n; j += blockDim.x) {
      const T xr = j == kk ? T(1) : Ar[kk * n + j];
      const T xi = j == kk ? T(0) : Ai[kk * n + j];
      Ar[kk * n + j] = xr * ipr - xi * ipi;
      Ai[kk * n + j] = xr * ipi + xi * ipr;
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += blockDim.x) {
      const int i = e / n, j = e - i * n;
      if (i == kk) continue;
      const T br = (j == kk) ? T(0) : Ar[e];
      const T bi2 = (j == kk) ? T(0) : Ai[e];
      const T ur = Ar[kk * n + j], ui = Ai[kk * n + j];
      Ar[e] = br - (cr[i] * ur - ci[i] * ui);
      Ai[e] = bi2 - (cr[i] * ui + ci[i] * ur);
    }
    __syncthreads();
  }
  for (int kk = n - 1; kk >= 0; --kk) {
    const int q = perm[kk];
    if (q != kk)
      for (int i = tid; i < n; i += blockDim.x) {
        T t = Ar[i * n + kk];
        Ar[i * n + kk] = Ar[i * n + q];
        Ar[i * n + q] = t;
        t = Ai[i * n + kk];
        Ai[i * n + kk] = Ai[i * n + q];
        Ai[i * n + q] = t;
      }
    __syncthreads();
  }
  // factored layout: column j of the patch, the block's rows at its row offset
  const int lc = p_ld[p];
  int rowoff = 0;
  for (int q = 0; q < blk; ++q) rowoff += irk::eig_block_rows(sb.type[q], n, VEC);
  const int rows = irk::eig_block_rows(2, n, VEC);
  T* __restrict__ out = inv + p_inv_off[p] + rowoff;
  for (int e = tid; e < n * rows; e += blockDim.x) {
    const int j = e / rows, i = e - j * rows;
    const int c = i >> 1;
    T v = T(0);
    if (c < n) v = (i & 1) ? Ai[c * n + j] : Ar[c * n + j];
    out[(int64_t)j * lc + i] = v;
  }
}

// Copy eigen-block b of every patch in [p0, p1) from its dense inverse (column-major
// m n_s x ldt at tmp + tmp_off[p] - off0, m = 1 or 2 stages) into the factored layout:
// n_s columns of lc = p_ld[p] values, the block's rows starting at its row offset.  A
// pair keeps the first n_s columns of [[P, -Q], [Q, P]] as complex entries P + iQ.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_eig_extract(
    int64_t p0, int64_t p1, int r, int b, irk::StageBasis<T> sb, const int32_t* __restrict__ p_nloc,
    const int32_t* __restrict__ p_ld, const int64_t* __restrict__ p_inv_off,
    const int32_t* __restrict__ tmp_ld, const int64_t* __restrict__ tmp_off, int64_t off0,
    const T* __restrict__ tmp, T* __restrict__ inv) {
  constexpr int VEC = Vec16<T>::n;
  const int64_t p = p0 + blockIdx.x;
  if (p >= p1) return;
  const int ns = p_nloc[p] / r;
  const int lc = p_ld[p];
  int rowoff = 0;
  for (int q = 0; q < b; ++q) rowoff += irk::eig_block_rows(sb.type[q], ns, VEC);
  const int rows = irk::eig_block_rows(sb.type[b], ns, VEC);
  const int ldt = tmp_ld[p];
  const T* __restrict__ Z = tmp + (tmp_off[p] - off0);
  T* __restrict__ out = inv + p_inv_off[p] + rowoff;
  const bool pair = sb.type[b] == 2;
  for (int e = threadIdx.x; e < ns * rows; e += blockDim.x) {
    const int j = e / rows, i = e - j * rows;
    T v = T(0);
    if (!pair) {
      if (i < ns) v = Z[(int64_t)j * ldt + i];
    } else {
      const int c = i >> 1;
      if (c < ns) v = Z[(int64_t)j * ldt + ((i & 1) ? ns + c : c)];
    }
    out[(int64_t)j * lc + i] = v;
  }
}

template <typename T, int RB, int NMAX, int UNROLL, int NT, int WAVES, int WPE = 1>
__global__ __launch_bounds__(WAVES * 64) __attribute__((amdgpu_waves_per_eu(WPE))) void k_patch_apply_eig(
    int64_t npatch, irk::StageBasis<T> sb, const int32_t* __restrict__ sched,
    const int32_t* __restrict__ p_nloc, const int32_t* __restrict__ p_ld,
    const int64_t* __restrict__ p_inv_off, const int64_t* __restrict__ p_slot_off,
    const int32_t* __restrict__ gidx, const T* __restrict__ inv, const T* __restrict__ res,
    const T* __restrict__ W, T* __restrict__ Y, int transpose, int D) {
  __shared__ T xs[WAVES][NMAX];
  __shared__ T xt[WAVES][NMAX];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t idx = (int64_t)blockIdx.x * WAVES + wave;
  if (idx >= npatch) return;  // whole wavefront exits; no workgroup barrier below
  dev::patch_apply_eig_one<T, RB, UNROLL, NT>(sched[idx], lane, xs[wave], xt[wave], sb, p_nloc, p_ld, p_inv_off,
                                              p_slot_off, gidx, inv, res, W, Y, transpose, D);
}

template <typename T, int NMAX, int UNROLL, int PF, int WAVES, int NT = 1, int RS = 1>
__global__ __launch_bounds__(WAVES * 64) void k_patch_apply_sym(
    int64_t npatch, irk::StageBasis<T> sb, const int32_t* __restrict__ sched,
    const int32_t* __restrict__ p_nloc, const int64_t* __restrict__ p_inv_off,
    const int64_t* __restrict__ p_slot_off, const int32_t* __restrict__ gidx, const T* __restrict__ inv,
    const T* __restrict__ res, const T* __restrict__ W, T* __restrict__ Y, int transpose, int D) {
  __shared__ T xs[WAVES][NMAX];
  __shared__ T xt[WAVES][2 * NMAX];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t idx = (int64_t)blockIdx.x * WAVES + wave;
  if (idx >= npatch) return;  // whole wavefront exits; no workgroup barrier below
  dev::patch_apply_sym_one<T, UNROLL, NT, PF, RS>(sched[idx], lane, xs[wave], xt[wave], sb, p_nloc, p_inv_off,
                                             p_slot_off, gidx, inv, res, W, Y, transpose, D);
}

// Symmetric factored form from the factored form (one workgroup per patch): the wrapped
// diagonals of every block inverse in descending order, each entry the mean of Z(i, j)
// and Z(j, i), which agree up to the rounding of the factorisation.  Factored layout: column j of block b
// holds Z(i, j) at base_b + i (real) or base_b + 2 i + {0, 1} (pair, re and im).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pack_sym(int64_t np, irk::StageBasis<T> sb,
                                                     const int32_t* __restrict__ p_nloc,
                                                     const int32_t* __restrict__ p_ld,
                                                     const int64_t* __restrict__ full_off,
                                                     const int64_t* __restrict__ sym_off,
                                                     const T* __restrict__ full, T* __restrict__ out) {
  constexpr int VEC = Vec16<T>::n;
  const int64_t p = blockIdx.x;
  if (p >= np) return;
  const int ns = p_nloc[p] / sb.r, lc = p_ld[p];
  const int h = irk::sym_diags(ns);
  const T* __restrict__ F = full + full_off[p];
  T* __restrict__ O = out + sym_off[p];
  int base = 0;
  int64_t boff = 0;
  for (int b = 0; b < sb.nblk; ++b) {
    const int type = sb.type[b];
    const int G = irk::sym_group(type, VEC);
    const int64_t cnt = irk::sym_block_values(type, ns, VEC);
    for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) {
      const int v = (int)(e % VEC);
      const int64_t wi = e / VEC;
      const int i = (int)(wi % ns), g = (int)(wi / ns);
      const int k = v / type, comp = v - k * type;
      const int sd = (int)(cnt / ((int64_t)ns * VEC)) * G - 1 - g * G - k;  // descending diagonals
      T val = T(0);
      if (sd < h) {
        const int j = (i + sd) % ns;
        const T zij = F[(int64_t)j * lc + base + type * i + comp];
        const T zji = F[(int64_t)i * lc + base + type * j + comp];
        val = T(0.5) * (zij + zji);
      }
      O[boff + e] = val;
    }
    base += irk::eig_block_rows(type, ns, VEC);
    boff += cnt;
  }
}

// ------------------------------------------------------------------ gather update
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather_update(int64_t N, int64_t nsl, const int32_t* __restrict__ g_off,
                                                          const int32_t* __restrict__ g_w,
                                                          const int32_t* __restrict__ g_slot,
                                                          const T* __restrict__ Y,
                                                          const T* __restrict__ W, T omega,
                                                          int mode, T* __restrict__ x) {
  const int lane = threadIdx.x & 63;
  const int64_t sl = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (sl >= nsl) return;
  dev::gather_sell_one<T>(sl * 64 + lane, sl, lane, g_off, g_w, g_slot, Y, W, omega, mode, x, N);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather_cheb(int64_t N, int64_t nsl, const int32_t* __restrict__ g_off,
                                                        const int32_t* __restrict__ g_w,
                                                        const int32_t* __restrict__ g_slot, const T* __restrict__ Y,
                                                        const T* __restrict__ W, T c1, T c2, int first, int xzero,
                                                        T* __restrict__ d, T* __restrict__ x) {
  const int lane = threadIdx.x & 63;
  const int64_t sl = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (sl >= nsl) return;
  dev::gather_cheb_one<T>(sl * 64 + lane, sl, lane, g_off, g_w, g_slot, Y, W, c1, c2, first, xzero, d, x, N);
}

// ---------------------------------------------------------------------- transfers
template <int D, int R, typename T>
__global__ __launch_bounds__(kBlock) void k_spmv_nodes(
    int64_t nrow_u, int64_t nrow_p, int64_t out_offV, int64_t in_offV,
    const int32_t* __restrict__ u_ptr, const int32_t* __restrict__ u_col,
    const T* __restrict__ u_val, const int32_t* __restrict__ p_ptr,
    const int32_t* __restrict__ p_col, const T* __restrict__ p_val, const T* __restrict__ in,
    T* __restrict__ out, int add) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  dev::spmv_nodes_row<D, R, T>(row, nrow_u, nrow_p, out_offV, in_offV, u_ptr, u_col, u_val, p_ptr, p_col, p_val,
                               in, out, add);
}

// ------------------------------------------------------- coarse operator inverse
// Gauss--Jordan step k, part 1 (one workgroup): the largest |J[i][k]|, i >= k (ties to
// the smaller row), becomes the pivot row; rows k and piv are swapped, column k is
// saved, and row k is scaled so that it holds the inverse's pivot row.
__global__ __launch_bounds__(1024) void k_gj_pivot(double* __restrict__ J, int64_t N, int64_t k, double tol,
                                                   double* __restrict__ colk, int64_t* __restrict__ swp,
                                                   int* __restrict__ fail) {
  __shared__ double sb[1024];
  __shared__ int64_t si[1024];
  const int tid = threadIdx.x;
  double best = -1.0;
  int64_t bi = k;
  for (int64_t i = k + tid; i < N; i += blockDim.x) {
    const double a = fabs(J[i * N + k]);
    if (a > best) {
      best = a;
      bi = i;
    }
  }
  sb[tid] = best;
  si[tid] = bi;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w && (sb[tid + w] > sb[tid] || (sb[tid + w] == sb[tid] && si[tid + w] < si[tid]))) {
      sb[tid] = sb[tid + w];
      si[tid] = si[tid + w];
    }
    __syncthreads();
  }
  const int64_t piv = si[0];
  if (!(sb[0] > tol)) {
    if (tid == 0) atomicMax(fail, 1);
    return;  // uniform: every later step is void and the caller reports the failure
  }
  if (piv != k)
    for (int64_t j = tid; j < N; j += blockDim.x) {
      const double t = J[k * N + j];
      J[k * N + j] = J[piv * N + j];
      J[piv * N + j] = t;
    }
  __syncthreads();
  const double ip = 1.0 / J[k * N + k];
  for (int64_t i = tid; i < N; i += blockDim.x) colk[i] = i == k ? 0.0 : J[i * N + k];
  __syncthreads();
  for (int64_t j = tid; j < N; j += blockDim.x) J[k * N + j] = (j == k ? 1.0 : J[k * N + j]) * ip;
  if (tid == 0) swp[k] = piv;
}

// part 2: every other row i loses colk[i] times the scaled pivot row (column k starts
// from zero); rows with a zero multiplier are left as they are
__global__ __launch_bounds__(kBlock) void k_gj_update(double* __restrict__ J, int64_t N, int64_t k,
                                                      const double* __restrict__ colk, const int* __restrict__ fail) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * N || *fail) return;
  const int64_t i = e / N, j = e - i * N;
  const double f = colk[i];
  if (i == k || f == 0.0) return;
  const double base = j == k ? 0.0 : J[e];
  J[e] = base - f * J[k * N + j];
}

// the recorded row swaps undone as column swaps, last first (one workgroup)
__global__ __launch_bounds__(1024) void k_gj_unswap(double* __restrict__ J, int64_t N,
                                                    const int64_t* __restrict__ swp, const int* __restrict__ fail) {
  if (*fail) return;
  for (int64_t k = N - 1; k >= 0; --k) {
    const int64_t q = swp[k];
    if (q != k)
      for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
        const double t = J[i * N + k];
        J[i * N + k] = J[i * N + q];
        J[i * N + q] = t;
      }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_transpose(const double* __restrict__ in, double* __restrict__ out,
                                                      int64_t N) {
  __shared__ double tile[32][33];
  const int64_t bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  for (int yy = ty; yy < 32; yy += 8)
    if (by + yy < N && bx + tx < N) tile[yy][tx] = in[(by + yy) * N + bx + tx];
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8)
    if (bx + yy < N && by + tx < N) out[(bx + yy) * N + by + tx] = tile[tx][yy];
}

// ------------------------------------------------------------------- coarse solve
// x = inv * b with inv column-major N x N.  Grid (ceil(N/64), kCoarseSplit); each
// wavefront owns 64 rows and a contiguous range of columns; partial sums are reduced
// in a fixed order by k_coarse_reduce.
constexpr int kCoarseSplit = 16;

__global__ __launch_bounds__(kBlock) void k_coarse_gemv_part(const double* __restrict__ inv, int64_t N,
                                                             const double* __restrict__ b,
                                                             double* __restrict__ part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const int nchunk = kCoarseSplit * (kBlock / 64);
  const int chunk = blockIdx.y * (kBlock / 64) + wave;
  const int64_t per = (N + nchunk - 1) / nchunk;
  const int64_t j0 = chunk * per, j1 = min(N, j0 + per);
  double acc = 0;
  if (i < N)
    for (int64_t j = j0; j < j1; ++j) acc += inv[j * N + i] * b[j];
  if (i < N) part[(int64_t)chunk * N + i] = acc;
}

// mode 0: x = sum of the partial sums; 1: x -= sum (a residual b - M y formed in
// place of b); 2: x += sum (the correction of the refinement step)
__global__ __launch_bounds__(kBlock) void k_coarse_reduce(const double* __restrict__ part, int64_t N,
                                                          double* __restrict__ x, int mode) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double acc = 0;
  for (int c = 0; c < kCoarseSplit * (kBlock / 64); ++c) acc += part[(int64_t)c * N + i];
  x[i] = mode == 0 ? acc : (mode == 1 ? x[i] - acc : x[i] + acc);
}

__global__ void k_zero_pins(double* b, const int64_t* pins, int np) {
  const int i = threadIdx.x;
  if (i < np) b[pins[i]] = 0.0;
}

// ------------------------------------------------------------------------ layouts
template <typename T>
__global__ __launch_bounds__(kBlock) void k_permute(int64_t N, int64_t offV, int64_t nfree,
                                                    int64_t ns, int D, int R,
                                                    const double* __restrict__ in,
                                                    T* __restrict__ out, int to_internal,
                                                    const T* __restrict__ in_int,
                                                    double* __restrict__ out_abi) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  int64_t a;
  if (g < offV) {
    const int64_t i = g / (D * R), rem = g - i * D * R;
    const int c = (int)(rem / R), s = (int)(rem - (int64_t)c * R);
    a = s * ns + c * nfree + i;
  } else {
    const int64_t v = (g - offV) / R;
    const int s = (int)(g - offV - v * R);
    a = s * ns + D * nfree + v;
  }
  if (to_internal) out[g] = (T)in[a];
  else out_abi[a] = (double)in_int[g];
}

template <typename S, typename Dt>
__global__ __launch_bounds__(kBlock) void k_cast(const S* __restrict__ in, Dt* __restrict__ out,
                                                 int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (Dt)in[i];
}

// per-stage pressure mean removal in two passes with a fixed reduction order: partial
// sums of every stage over vertex chunks (grid-stride, one workgroup per chunk set),
// then every workgroup of the apply pass sums the partials in the same order and
// subtracts the means
constexpr int kProjBlocks = 256;

__global__ __launch_bounds__(kBlock) void k_project_partial(const double* __restrict__ x, int64_t offV,
                                                            int64_t nv, int R, double* __restrict__ partials) {
  __shared__ double red[kMaxStages][kBlock];
  double acc[kMaxStages] = {0, 0, 0, 0};
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < nv; v += (int64_t)gridDim.x * kBlock)
    for (int s = 0; s < R; ++s) acc[s] += x[offV + v * R + s];
  for (int s = 0; s < R; ++s) red[s][threadIdx.x] = acc[s];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int s = 0; s < R; ++s) red[s][threadIdx.x] += red[s][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int s = 0; s < R; ++s) partials[s * gridDim.x + blockIdx.x] = red[s][0];
}

__global__ __launch_bounds__(kBlock) void k_project_apply(double* __restrict__ x, int64_t offV, int64_t nv, int R,
                                                          const double* __restrict__ partials, int nb) {
  __shared__ double red[kMaxStages][kBlock];
  for (int s = 0; s < R; ++s) red[s][threadIdx.x] = (int)threadIdx.x < nb ? partials[s * nb + threadIdx.x] : 0.0;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int s = 0; s < R; ++s) red[s][threadIdx.x] += red[s][threadIdx.x + w];
    __syncthreads();
  }
  double mean[kMaxStages];
  for (int s = 0; s < R; ++s) mean[s] = red[s][0] / (double)nv;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nv * R; e += (int64_t)gridDim.x * kBlock)
    x[offV + e] -= mean[e % R];
}

// ------------------------------------------------------------- GMRES relaxation
// One cycle of left-preconditioned GMRES on a level (Arnoldi with classical
// Gram--Schmidt, Hessenberg least squares by Givens rotations): block partial sums in
// a fixed order, one workgroup finishing each reduction, the small problem on one
// thread; nothing returns to the host.
// part[i * gridDim + block] = block's share of <V_i, w> (i < nv), accumulated in FP64
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gr_dots(int64_t n, int nv, const T* __restrict__ V, int64_t ldv,
                                                    const T* __restrict__ w, double* __restrict__ part) {
  __shared__ double red[kBlock];
  double acc[kMaxGr + 1];
#pragma unroll
  for (int i = 0; i <= kMaxGr; ++i) acc[i] = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < n; g += (int64_t)gridDim.x * kBlock) {
    const double wg = (double)w[g];
#pragma unroll
    for (int i = 0; i <= kMaxGr; ++i)
      if (i < nv) acc[i] += (double)V[(int64_t)i * ldv + g] * wg;
  }
  for (int i = 0; i < nv; ++i) {
    red[threadIdx.x] = acc[i];
    __syncthreads();
    for (int k = kBlock / 2; k > 0; k >>= 1) {
      if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)i * gridDim.x + blockIdx.x] = red[0];
    __syncthreads();
  }
}

// out[i] = sum over blocks of part[i * nb + b] (fixed order); sq: out[0] = sqrt(sum)
__global__ __launch_bounds__(kBlock) void k_gr_finish(const double* __restrict__ part, int nb, int nv, int sq,
                                                      double* __restrict__ out) {
  __shared__ double red[kBlock];
  for (int i = 0; i < nv; ++i) {
    red[threadIdx.x] = (int)threadIdx.x < nb ? part[(int64_t)i * nb + threadIdx.x] : 0.0;
    __syncthreads();
    for (int k = kBlock / 2; k > 0; k >>= 1) {
      if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = sq ? sqrt(red[0]) : red[0];
    __syncthreads();
  }
}

// w -= sum_{i <= j} h_i V_i (in order), part = block's share of ||w||^2
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gr_orth(int64_t n, int j, const T* __restrict__ V, int64_t ldv,
                                                    const double* __restrict__ h, T* __restrict__ w,
                                                    double* __restrict__ part) {
  __shared__ double red[kBlock];
  double acc = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < n; g += (int64_t)gridDim.x * kBlock) {
    double v = (double)w[g];
    for (int i = 0; i <= j; ++i) v -= h[i] * (double)V[(int64_t)i * ldv + g];
    const T t = (T)v;
    w[g] = t;
    acc += (double)t * (double)t;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = kBlock / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// v /= d (a zero norm leaves a zero vector)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gr_scale(int64_t n, const double* __restrict__ d, T* __restrict__ v) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= n) return;
  const double dd = *d;
  v[g] = dd > 0.0 ? (T)((double)v[g] / dd) : T(0);
}

// y minimising ||beta e_1 - H y|| for the first m_eff columns, m_eff the steps before the
// first zero subdiagonal entry (an invariant Krylov space), and before a column whose
// rotated diagonal falls below 1e-12 of the largest one so far (a numerically rank
// deficient H, as when a basis vector lies in the pressure null space of J; a least
// squares solve with a rank cut-off drops the same direction); y = 0 past m_eff
__global__ void k_gr_solve(double* __restrict__ gr, int m) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  constexpr int ld = kMaxGr + 1;
  const double* H = gr + kGrH;
  const double beta = gr[kGrNorm];
  double* y = gr + kGrY;
  int me = m;
  for (int j = 0; j < m; ++j)
    if (!(H[j * ld + j + 1] != 0.0)) {
      me = j + 1;
      break;
    }
  double R[ld * kMaxGr], g[ld], c[kMaxGr], sn[kMaxGr];
  for (int i = 0; i < ld * kMaxGr; ++i) R[i] = H[i];
  for (int i = 0; i < ld; ++i) g[i] = 0.0;
  g[0] = beta;
  double rmax = 0.0;
  for (int j = 0; j < me; ++j) {
    for (int i = 0; i < j; ++i) {  // earlier rotations on column j
      const double a = R[j * ld + i], b = R[j * ld + i + 1];
      R[j * ld + i] = c[i] * a + sn[i] * b;
      R[j * ld + i + 1] = -sn[i] * a + c[i] * b;
    }
    const double a = R[j * ld + j], b = R[j * ld + j + 1];
    const double rr = hypot(a, b);
    if (!(rr > 1e-12 * rmax)) {  // also catches a non-finite rr
      me = j;
      break;
    }
    rmax = fmax(rmax, rr);
    c[j] = a / rr;
    sn[j] = b / rr;
    R[j * ld + j] = rr;
    R[j * ld + j + 1] = 0.0;
    const double g0 = g[j], g1 = g[j + 1];
    g[j] = c[j] * g0 + sn[j] * g1;
    g[j + 1] = -sn[j] * g0 + c[j] * g1;
  }
  for (int j = kMaxGr - 1; j >= 0; --j) y[j] = 0.0;
  for (int j = me - 1; j >= 0; --j) {
    double t = g[j];
    for (int k = j + 1; k < me; ++k) t -= R[k * ld + j] * y[k];
    y[j] = t / R[j * ld + j];
  }
}

// x = (assign ? 0 : x) + sum_j y_j V_j (in order)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gr_update(int64_t n, int m, const T* __restrict__ V, int64_t ldv,
                                                      const double* __restrict__ y, int assign, T* __restrict__ x) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= n) return;
  double v = assign ? 0.0 : (double)x[g];
  for (int j = 0; j < m; ++j) v += y[j] * (double)V[(int64_t)j * ldv + g];
  x[g] = (T)v;
}

// ------------------------------------------------------------------------- BLAS-1
__global__ __launch_bounds__(kBlock) void k_dot_partial(const double* __restrict__ a,
                                                        const double* __restrict__ b, int64_t n,
                                                        double* __restrict__ partials) {
  __shared__ double red[kBlock];
  double acc = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  constexpr int U = 4;  // loads of four grid-stride elements together, sums in order
  for (; i + (U - 1) * stride < n; i += U * stride) {
    double av[U], bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      av[u] = a[i + u * stride];
      bv[u] = b[i + u * stride];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc += av[u] * bv[u];
  }
  for (; i < n; i += stride) acc += a[i] * b[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBlock) void k_sum_partial(const double* __restrict__ a, int64_t n,
                                                        double* __restrict__ partials) {
  __shared__ double red[kBlock];
  double acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += a[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// mode 0: *out = sum; 1: *out = sqrt(sum); 2: *out += sum; 3: *out = sum / 2
__global__ __launch_bounds__(kBlock) void k_dot_final(const double* __restrict__ partials, int nb,
                                                      double* __restrict__ out, int mode) {
  __shared__ double red[kBlock];
  double acc = 0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += partials[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double v = red[0];
    *out = mode == 0 ? v : (mode == 1 ? sqrt(v) : (mode == 2 ? *out + v : 0.5 * v));
  }
}

// ---- Arnoldi step by modified Gram--Schmidt, one launch per projection: launch i
// finishes the inner product h_i = <w, v_i> from the previous launch's partial sums
// (same order as k_dot_final), applies w -= h_i v_i, and forms the partial sums of the
// next inner product <w, v_{i+1}> (or <w, w> after the last projection) with the
// grid-stride decomposition of k_dot_partial, so the values equal the unfused sequence.
__device__ double block_reduce_partials(const double* __restrict__ partials, int nb, double* red) {
  double acc = 0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += partials[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kBlock) void k_mgs_step(double* __restrict__ w, const double* __restrict__ vi,
                                                     const double* __restrict__ vnext, int64_t n,
                                                     const double* __restrict__ pin, int nb,
                                                     double* __restrict__ pout, double* __restrict__ hout) {
  __shared__ double red[kBlock];
  const double h = block_reduce_partials(pin, nb, red);
  if (blockIdx.x == 0 && threadIdx.x == 0) *hout = h;
  const double a = -1.0 * h;
  double acc = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // four grid-stride elements' loads issued together, then the same sums in the same order
  constexpr int U = 4;
  for (; e + (U - 1) * stride < n; e += U * stride) {
    double wv[U], vv[U], nv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      wv[u] = w[e + u * stride];
      vv[u] = vi[e + u * stride];
      nv[u] = vnext ? vnext[e + u * stride] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      double y = wv[u];
      y += a * vv[u];
      w[e + u * stride] = y;
      acc += y * (vnext ? nv[u] : y);
    }
  }
  for (; e < n; e += stride) {
    double y = w[e];
    y += a * vi[e];
    w[e] = y;
    acc += y * (vnext ? vnext[e] : y);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s2 = kBlock / 2; s2 > 0; s2 >>= 1) {
    if ((int)threadIdx.x < s2) red[threadIdx.x] += red[threadIdx.x + s2];
    __syncthreads();
  }
  if (threadIdx.x == 0) pout[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBlock) void k_mgs_normalize(double* __restrict__ w, int64_t n,
                                                          const double* __restrict__ pin, int nb,
                                                          double* __restrict__ hout) {
  __shared__ double red[kBlock];
  const double nrm = sqrt(block_reduce_partials(pin, nb, red));
  if (blockIdx.x == 0 && threadIdx.x == 0) *hout = nrm;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  constexpr int U = 4;  // loads of four grid-stride elements together
  for (; e + (U - 1) * stride < n; e += U * stride) {
    double wv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) wv[u] = w[e + u * stride];
#pragma unroll
    for (int u = 0; u < U; ++u) w[e + u * stride] = wv[u] / nrm;
  }
  for (; e < n; e += stride) w[e] = w[e] / nrm;
}

__global__ __launch_bounds__(kBlock) void k_axpy_dev(double* __restrict__ y,
                                                     const double* __restrict__ x, int64_t n,
                                                     const double* __restrict__ s, double sign,
                                                     double alpha_host) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = s ? sign * (*s) : alpha_host;
  y[i] += a * x[i];
}

__global__ __launch_bounds__(kBlock) void k_scale_inv(double* __restrict__ y,
                                                      const double* __restrict__ x, int64_t n,
                                                      const double* __restrict__ s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i] / (*s);
}

// y = a x + b y; with b = 0, y is not read (it may be fresh memory holding non-finite
// bit patterns, which 0 * y would carry into the result)
__global__ __launch_bounds__(kBlock) void k_axpby(double* __restrict__ y,
                                                  const double* __restrict__ x, int64_t n,
                                                  double a, double b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = b == 0.0 ? a * x[i] : a * x[i] + b * y[i];
}

__global__ __launch_bounds__(kBlock) void k_update_sum(double* __restrict__ x, const double* __restrict__ Z,
                                                       int64_t n, const double* __restrict__ c, int m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = x[i];
  for (int k = 0; k < m; ++k) acc = fma(c[k], Z[(size_t)k * n + i], acc);
  x[i] = acc;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T* y, int64_t n, T v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_nonfinite(const double* __restrict__ x, int64_t n,
                                                      int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(x[i])) atomicMax(flag, 1);
}

// ---------------------------------------------------------------- rhs and update
// F_i = [M_fa f_i - L u - B p ; -B^T u] in the ABI layout; state = (u, p) stage block.
__global__ __launch_bounds__(kBlock) void k_rhs(
    int64_t nfree, int64_t nv, int64_t nnodes, int D, int R, const int32_t* __restrict__ mfa_ptr,
    const int32_t* __restrict__ mfa_col, const double* __restrict__ mfa_val,
    const int32_t* __restrict__ s_ptr, const int32_t* __restrict__ s_col,
    const double* __restrict__ sL, const int32_t* __restrict__ b_ptr,
    const int32_t* __restrict__ b_col, const double* __restrict__ b_val,
    const int32_t* __restrict__ bt_ptr, const int32_t* __restrict__ bt_col,
    const double* __restrict__ bt_val, const double* __restrict__ f,
    const double* __restrict__ state, double* __restrict__ F) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ns = D * nfree + nv;
  const double* u = state;
  const double* pr = state + D * nfree;
  if (row < nfree) {
    for (int c = 0; c < D; ++c) {
      double lu = 0, bp = 0;
      for (int32_t p = s_ptr[row]; p < s_ptr[row + 1]; ++p) lu += sL[p] * u[c * nfree + s_col[p]];
      for (int32_t p = b_ptr[row]; p < b_ptr[row + 1]; ++p) bp += b_val[(int64_t)p * D + c] * pr[b_col[p]];
      for (int s = 0; s < R; ++s) {
        double mf = 0;
        for (int32_t p = mfa_ptr[row]; p < mfa_ptr[row + 1]; ++p)
          mf += mfa_val[p] * f[((int64_t)s * nnodes + mfa_col[p]) * D + c];
        F[s * ns + c * nfree + row] = mf - lu - bp;
      }
    }
  } else if (row < nfree + nv) {
    const int64_t v = row - nfree;
    double acc = 0;
    for (int32_t p = bt_ptr[v]; p < bt_ptr[v + 1]; ++p)
      for (int c = 0; c < D; ++c) acc += bt_val[(int64_t)p * D + c] * u[c * nfree + bt_col[p]];
    for (int s = 0; s < R; ++s) F[s * ns + D * nfree + v] = -acc;
  }
}

// F += the terms of prescribed boundary velocities (ABI layout).  Velocity row f, stage
// i, component c: -sum_b (M_fb k_{i,b,c} + L_fb G_{i,b,c}) with
// k_{i,b,c} = sum_j (dt A)^{-1}_ij (G_{j,b,c} - g_{n,b,c}); vertex row v, stage i:
// -sum_b sum_c B^T_{v,(b,c)} G_{i,b,c}.
__global__ __launch_bounds__(kBlock) void k_rhs_dirichlet(
    int64_t nfree, int64_t nv, int64_t nnodes, int D, int R, const int32_t* __restrict__ fb_ptr,
    const int32_t* __restrict__ fb_col, const double* __restrict__ fb_m, const double* __restrict__ fb_l,
    const int32_t* __restrict__ vb_ptr, const int32_t* __restrict__ vb_col, const double* __restrict__ vb_val,
    Coef<double> ainv, const double* __restrict__ gn, const double* __restrict__ gst, double* __restrict__ F) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ns = D * nfree + nv;
  if (row < nfree) {
    double acc[kMaxStages][3];
    for (int i = 0; i < R; ++i)
      for (int c = 0; c < D; ++c) acc[i][c] = 0.0;
    for (int32_t p = fb_ptr[row]; p < fb_ptr[row + 1]; ++p) {
      const int64_t b = fb_col[p];
      const double m = fb_m[p], l = fb_l[p];
      for (int c = 0; c < D; ++c) {
        const double g0 = gn[b * D + c];
        double G[kMaxStages];
        for (int j = 0; j < R; ++j) G[j] = gst[((int64_t)j * nnodes + b) * D + c];
        for (int i = 0; i < R; ++i) {
          double kb = 0.0;
          for (int j = 0; j < R; ++j) kb += ainv.v[i * R + j] * (G[j] - g0);
          acc[i][c] += m * kb + l * G[i];
        }
      }
    }
    for (int i = 0; i < R; ++i)
      for (int c = 0; c < D; ++c) F[i * ns + c * nfree + row] -= acc[i][c];
  } else if (row < nfree + nv) {
    const int64_t v = row - nfree;
    double acc[kMaxStages];
    for (int i = 0; i < R; ++i) acc[i] = 0.0;
    for (int32_t p = vb_ptr[v]; p < vb_ptr[v + 1]; ++p) {
      const int64_t b = vb_col[p];
      for (int c = 0; c < D; ++c) {
        const double bv = vb_val[(int64_t)p * D + c];
        for (int i = 0; i < R; ++i) acc[i] += bv * gst[((int64_t)i * nnodes + b) * D + c];
      }
    }
    for (int i = 0; i < R; ++i) F[i * ns + D * nfree + v] -= acc[i];
  }
}

__global__ __launch_bounds__(kBlock) void k_update(int64_t ns, int R, Coef<double> bdt,
                                                   const double* __restrict__ kv,
                                                   double* __restrict__ state) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  double acc = state[i];
  for (int j = 0; j < R; ++j) acc += bdt.v[j] * kv[j * ns + i];
  state[i] = acc;
}

// ------------------------------------------------------------- adjoint helpers
// gf[s][node][c] = sum_{rows i with column node} mfa[i,node] lam_s^{u,c}[i], computed by
// rows of M_fa^T (transposed CSR, node rows).
__global__ __launch_bounds__(kBlock) void k_rhs_adjoint_f(
    int64_t nnodes, int64_t nfree, int64_t nv, int D, int R, const int32_t* __restrict__ mt_ptr,
    const int32_t* __restrict__ mt_col, const double* __restrict__ mt_val,
    const double* __restrict__ lam, double* __restrict__ gf) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nnodes) return;
  const int64_t ns = D * nfree + nv;
  for (int s = 0; s < R; ++s)
    for (int c = 0; c < D; ++c) {
      double acc = 0;
      for (int32_t p = mt_ptr[node]; p < mt_ptr[node + 1]; ++p)
        acc += mt_val[p] * lam[s * ns + c * nfree + mt_col[p]];
      gf[((int64_t)s * nnodes + node) * D + c] = acc;
    }
}

// gstate = [-L^T su - B sp ; -B^T su], su = sum_i lam_i^u, sp = sum_i lam_i^p
__global__ __launch_bounds__(kBlock) void k_rhs_adjoint_s(
    int64_t nfree, int64_t nv, int D, int R, const int32_t* __restrict__ s_ptr,
    const int32_t* __restrict__ s_col, const double* __restrict__ sLt,
    const int32_t* __restrict__ b_ptr, const int32_t* __restrict__ b_col,
    const double* __restrict__ b_val, const int32_t* __restrict__ bt_ptr,
    const int32_t* __restrict__ bt_col, const double* __restrict__ bt_val,
    const double* __restrict__ lam, double* __restrict__ gs, int accumulate) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ns = D * nfree + nv;
  if (row < nfree) {
    for (int c = 0; c < D; ++c) {
      double acc = 0;
      for (int32_t p = s_ptr[row]; p < s_ptr[row + 1]; ++p) {
        double su = 0;
        for (int s = 0; s < R; ++s) su += lam[s * ns + c * nfree + s_col[p]];
        acc -= sLt[p] * su;
      }
      for (int32_t p = b_ptr[row]; p < b_ptr[row + 1]; ++p) {
        double sp = 0;
        for (int s = 0; s < R; ++s) sp += lam[s * ns + D * nfree + b_col[p]];
        acc -= b_val[(int64_t)p * D + c] * sp;
      }
      gs[c * nfree + row] = accumulate ? gs[c * nfree + row] + acc : acc;
    }
  } else if (row < nfree + nv) {
    const int64_t v = row - nfree;
    double acc = 0;
    for (int32_t p = bt_ptr[v]; p < bt_ptr[v + 1]; ++p)
      for (int c = 0; c < D; ++c) {
        double su = 0;
        for (int s = 0; s < R; ++s) su += lam[s * ns + c * nfree + bt_col[p]];
        acc -= bt_val[(int64_t)p * D + c] * su;
      }
    gs[D * nfree + v] = accumulate ? gs[D * nfree + v] + acc : acc;
  }
}

__global__ __launch_bounds__(kBlock) void k_update_adjoint(int64_t ns, int R, Coef<double> bdt,
                                                           const double* __restrict__ gs,
                                                           double* __restrict__ G) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const double g = gs[i];
  for (int j = 0; j < R; ++j) G[j * ns + i] = bdt.v[j] * g;
}

// per free-node-row contribution to lam^T(dF/dnu - dJ/dnu k): one value per row,
// reduced afterwards in a fixed order.
__global__ __launch_bounds__(kBlock) void k_nu_rows(int64_t nfree, int64_t nv, int D, int R,
                                                    Coef<double> dtA,
                                                    const int32_t* __restrict__ s_ptr,
                                                    const int32_t* __restrict__ s_col,
                                                    const double* __restrict__ K1,
                                                    const double* __restrict__ lam,
                                                    const double* __restrict__ kv,
                                                    const double* __restrict__ state,
                                                    double* __restrict__ rowsum) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nfree) return;
  const int64_t ns = D * nfree + nv;
  double tot = 0;
  for (int c = 0; c < D; ++c) {
    double ku = 0;
    double kk[kMaxStages] = {0, 0, 0, 0};
    for (int32_t p = s_ptr[row]; p < s_ptr[row + 1]; ++p) {
      const int64_t j = s_col[p];
      ku += K1[p] * state[c * nfree + j];
      for (int t = 0; t < R; ++t) kk[t] += K1[p] * kv[t * ns + c * nfree + j];
    }
    for (int s = 0; s < R; ++s) {
      double w = ku;
      for (int t = 0; t < R; ++t) w += dtA.v[s * R + t] * kk[t];
      tot -= lam[s * ns + c * nfree + row] * w;
    }
  }
  rowsum[row] = tot;
}

// e = state - target on the velocity entries, 0 on the pressure entries
__global__ __launch_bounds__(kBlock) void k_velocity_diff(int64_t nvel, int64_t ns, const double* __restrict__ a,
                                                          const double* __restrict__ b, double* __restrict__ e) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ns) e[i] = i < nvel ? a[i] - b[i] : 0.0;
}

// ga = s v, gb = -s v with s = *scale (1 when scale is null); ga or gb may be null
__global__ __launch_bounds__(kBlock) void k_scaled_pair(int64_t n, const double* __restrict__ scale,
                                                        const double* __restrict__ v, double* __restrict__ ga,
                                                        double* __restrict__ gb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double w = (scale ? *scale : 1.0) * v[i];
  if (ga) ga[i] = w;
  if (gb) gb[i] = -w;
}

__global__ __launch_bounds__(kBlock) void k_mass_apply(int64_t nfree, int64_t nv, int D,
                                                       const int32_t* __restrict__ s_ptr,
                                                       const int32_t* __restrict__ s_col,
                                                       const double* __restrict__ sM,
                                                       const double* __restrict__ st,
                                                       double* __restrict__ out) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row < nfree) {
    for (int c = 0; c < D; ++c) {
      double acc = 0;
      for (int32_t p = s_ptr[row]; p < s_ptr[row + 1]; ++p) acc += sM[p] * st[c * nfree + s_col[p]];
      out[c * nfree + row] = acc;
    }
  } else if (row < nfree + nv) {
    out[D * nfree + row - nfree] = 0.0;
  }
}

}  // namespace

// =========================================================================== launchers
#define IRK_DISPATCH_DR(D, R, ...)                        \
  do {                                                     \
    if ((D) == 2) {                                        \
      switch (R) {                                         \
        case 1: { constexpr int DD = 2, RR = 1; __VA_ARGS__; } break; \
        case 2: { constexpr int DD = 2, RR = 2; __VA_ARGS__; } break; \
        case 3: { constexpr int DD = 2, RR = 3; __VA_ARGS__; } break; \
        case 4: { constexpr int DD = 2, RR = 4; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue;              \
      }                                                    \
    } else {                                               \
      switch (R) {                                         \
        case 1: { constexpr int DD = 3, RR = 1; __VA_ARGS__; } break; \
        case 2: { constexpr int DD = 3, RR = 2; __VA_ARGS__; } break; \
        case 3: { constexpr int DD = 3, RR = 3; __VA_ARGS__; } break; \
        case 4: { constexpr int DD = 3, RR = 4; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue;              \
      }                                                    \
    }                                                      \
  } while (0)

template <typename T>
hipError_t residual(const DevLevel& L, const DevOps<T>& ops, const double* A, double dt,
                    const T* F, const T* x, T* y, hipStream_t s) {
  const int64_t nsl = L.nsl_u + L.nsl_p;
  // two wavefronts per slice where one per slice would leave the chip short of
  // wavefronts (fewer than four per SIMD: 256 CUs x 4 SIMDs x 4)
  if (nsl < kSplitSlices) {
    const unsigned g = (unsigned)((nsl + 1) / 2);
    IRK_DISPATCH_DR(L.dim, L.r, (k_residual_sell<DD, RR, T, 4, 2><<<dim3(g), dim3(256), 0, s>>>(
                                    L.nfree, L.nv, L.offV, L.nsl_u, L.nsl_p, L.su_off, L.su_w, L.su_col, ops.u_M,
                                    ops.u_L, L.sb_off, L.sb_w, L.sb_col, ops.u_B, L.sp_off, L.sp_w, L.sp_col,
                                    ops.p_Bt, scaled<T, RR>(A, dt), F, x, y)));
    return hipGetLastError();
  }
  const unsigned g = (unsigned)((nsl + 3) / 4);
  IRK_DISPATCH_DR(L.dim, L.r, (k_residual_sell<DD, RR, T, 4, 1><<<dim3(g), dim3(256), 0, s>>>(
                                  L.nfree, L.nv, L.offV, L.nsl_u, L.nsl_p, L.su_off, L.su_w, L.su_col, ops.u_M,
                                  ops.u_L, L.sb_off, L.sb_w, L.sb_col, ops.u_B, L.sp_off, L.sp_w, L.sp_col,
                                  ops.p_Bt, scaled<T, RR>(A, dt), F, x, y)));
  return hipGetLastError();
}

hipError_t residual_newton(const DevLevel& L, const double* nws, const double* A, double dt, const double* F,
                           const double* x, double* y, hipStream_t s) {
  const int64_t nsl = L.nsl_u + L.nsl_p;
  if (nsl < kSplitSlices) {
    // latency-bound levels: two wavefronts per slice
    const unsigned g = (unsigned)std::max<int64_t>(1, (nsl + 1) / 2);
    IRK_DISPATCH_DR(L.dim, L.r, (k_residual_newton_sell<DD, RR, 2><<<dim3(g), dim3(256), 0, s>>>(
                                    L.nfree, L.nv, L.offV, L.nsl_u, L.nsl_p, L.su_off, L.su_w, L.su_col,
                                    L.d64.u_M, nws, L.sb_off, L.sb_w, L.sb_col, L.d64.u_B, L.sp_off, L.sp_w,
                                    L.sp_col, L.d64.p_Bt, scaled<double, RR>(A, dt), F, x, y)));
    return hipGetLastError();
  }
  const unsigned g = (unsigned)std::max<int64_t>(1, (nsl + 3) / 4);
  IRK_DISPATCH_DR(L.dim, L.r, (k_residual_newton_sell<DD, RR, 1><<<dim3(g), dim3(256), 0, s>>>(
                                  L.nfree, L.nv, L.offV, L.nsl_u, L.nsl_p, L.su_off, L.su_w, L.su_col, L.d64.u_M,
                                  nws, L.sb_off, L.sb_w, L.sb_col, L.d64.u_B, L.sp_off, L.sp_w, L.sp_col,
                                  L.d64.p_Bt, scaled<double, RR>(A, dt), F, x, y)));
  return hipGetLastError();
}

hipError_t sell_blocks(int64_t ne, int k, const int32_t* src, const double* v, double* out, hipStream_t s) {
  if (ne <= 0) return hipSuccess;
  k_sell_blocks<<<dim3(blocks_for(ne * k)), dim3(kBlock), 0, s>>>(ne, k, src, v, out);
  return hipGetLastError();
}

template <typename T>
hipError_t patch_factor_range(const DevLevel& L, const DevOps<T>& ops, int R, const double* coef, double dt,
                              const int32_t* ld, const int64_t* off, T* out, int64_t p0, int64_t p1,
                              int64_t off0, int nmax, int* d_fail, hipStream_t s, const T* nw) {
  if (p1 <= p0) return hipSuccess;
  const unsigned g = (unsigned)(p1 - p0);
  const size_t n = (size_t)nmax;
  const size_t lds = n * n * sizeof(T) + n * sizeof(T) + n * sizeof(int) + 64;
  if (lds > 160 * 1024) {
    if (n > (size_t)kGjRows * kBlock) return hipErrorInvalidConfiguration;
    const size_t glds = (size_t)kGjBw * n * sizeof(T) + n * sizeof(T) + (size_t)kGjBw * kGjJt * sizeof(T) +
                        n * sizeof(int) + 64;
    IRK_DISPATCH_DR(L.dim, R, {
      auto kern = k_patch_factor_global<DD, RR, T>;
      hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)glds);
      if (e != hipSuccess) return e;
      kern<<<dim3(g), dim3(kBlock), glds, s>>>(p1, L.pn_ptr, L.pvv_ptr, L.pvv, L.pvp, ld, off, ops.s_M, ops.s_L,
                                               ops.b_val, scaled<T, RR>(coef, dt), out, d_fail, p0, off0, nw);
    });
    return hipGetLastError();
  }
  IRK_DISPATCH_DR(L.dim, R, {
    hipError_t e = launch_patch_factor_lds<DD, RR, T>(g, n, lds, s, p1, L.pn_ptr, L.pvv_ptr, L.pvv, L.pvp, ld, off,
                                                      ops.s_M, ops.s_L, ops.b_val, scaled<T, RR>(coef, dt), out,
                                                      d_fail, p0, off0, nw);
    if (e != hipSuccess) return e;
  });
  return hipGetLastError();
}

// Generic Kronecker operators (one value per spatial unknown and stage): the kernels
// above with D = 1, where the patch's last unknown takes the place of the pressure
// slot and every coupling, that one included, comes from the triples.
template <typename T>
hipError_t patch_factor_scalar(const DevLevel& L, const DevOps<T>& ops, int R, const double* A, double dt,
                               const int32_t* ld, const int64_t* off, T* out, int64_t p0, int64_t p1, int64_t off0,
                               int nmax, int* d_fail, hipStream_t s) {
  if (p1 <= p0) return hipSuccess;
  const unsigned g = (unsigned)(p1 - p0);
  const size_t n = (size_t)nmax;
  const size_t lds = n * n * sizeof(T) + n * sizeof(T) + n * sizeof(int) + 64;
#define IRK_PFS(KERN, LDS)                                                                                   \
  do {                                                                                                       \
    hipError_t e = hipFuncSetAttribute((const void*)KERN, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(LDS)); \
    if (e != hipSuccess) return e;                                                                           \
    KERN<<<dim3(g), dim3(kBlock), LDS, s>>>(p1, L.pn_ptr, L.pvv_ptr, L.pvv, L.pvp, ld, off, ops.s_M, ops.s_L,  \
                                           nullptr, cf, out, d_fail, p0, off0, nullptr);                      \
  } while (0)
#define IRK_PFS_R(RR)                                                                                        \
  {                                                                                                          \
    const Coef<T> cf = scaled<T, RR>(A, dt);                                                                 \
    if (lds <= 160 * 1024) {                                                                                 \
      hipError_t e = launch_patch_factor_lds<1, RR, T>(g, n, lds, s, p1, L.pn_ptr, L.pvv_ptr, L.pvv, L.pvp, ld, \
                                                       off, ops.s_M, ops.s_L, nullptr, cf, out, d_fail, p0,   \
                                                       off0, nullptr);                                        \
      if (e != hipSuccess) return e;                                                                         \
    } else {                                                                                                 \
      if (n > (size_t)kGjRows * kBlock) return hipErrorInvalidConfiguration;                                 \
      const size_t glds = (size_t)kGjBw * n * sizeof(T) + n * sizeof(T) + (size_t)kGjBw * kGjJt * sizeof(T) + \
                          n * sizeof(int) + 64;                                                              \
      IRK_PFS((k_patch_factor_global<1, RR, T>), glds);                                                      \
    }                                                                                                        \
  }
  switch (R) {
    case 1: IRK_PFS_R(1) break;
    case 2: IRK_PFS_R(2) break;
    case 3: IRK_PFS_R(3) break;
    case 4: IRK_PFS_R(4) break;
    default: return hipErrorInvalidValue;
  }
#undef IRK_PFS_R
#undef IRK_PFS
  return hipGetLastError();
}

template <typename T>
hipError_t patch_factor_cplx(const DevLevel& L, const DevOps<T>& ops, double zr, double zi, int b, int nmax,
                             int* d_fail, hipStream_t s) {
  const size_t n = (size_t)nmax;
  const size_t lds = 2 * n * n * sizeof(T) + 2 * n * sizeof(T) + n * sizeof(int) + 64;
  if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
  const StageBasis<T>& sb = basis_of<T>(L);
  if (L.dim == 2) {
    auto kern = k_patch_factor_cplx<2, T>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    kern<<<dim3((unsigned)L.npatch), dim3(kBlock), lds, s>>>(L.npatch, L.pn_ptr, L.pvv_ptr, L.pvv, L.pvp, ops.s_M,
                                                          ops.s_L, ops.b_val, (T)zr, (T)zi, b, sb, L.p_ld,
                                                          L.p_inv_off, reinterpret_cast<T*>(L.inv), d_fail);
  } else {
    auto kern = k_patch_factor_cplx<3, T>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    kern<<<dim3((unsigned)L.npatch), dim3(kBlock), lds, s>>>(L.npatch, L.pn_ptr, L.pvv_ptr, L.pvv, L.pvp, ops.s_M,
                                                          ops.s_L, ops.b_val, (T)zr, (T)zi, b, sb, L.p_ld,
                                                          L.p_inv_off, reinterpret_cast<T*>(L.inv), d_fail);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t eig_extract(const DevLevel& L, const StageBasis<T>& sb, int b, const int32_t* tmp_ld,
                       const int64_t* tmp_off, int64_t off0, const T* tmp, int64_t p0, int64_t p1,
                       hipStream_t s) {
  if (p1 <= p0) return hipSuccess;
  k_eig_extract<T><<<dim3((unsigned)(p1 - p0)), dim3(kBlock), 0, s>>>(p0, p1, L.r, b, sb, L.p_nloc, L.p_ld,
                                                                     L.p_inv_off, tmp_ld, tmp_off, off0, tmp,
                                                                     reinterpret_cast<T*>(L.inv));
  return hipGetLastError();
}

template <typename T>
hipError_t pack_sym(const DevLevel& L, const int64_t* full_off, const T* full, hipStream_t s) {
  if (L.npatch <= 0) return hipSuccess;
  k_pack_sym<T><<<dim3((unsigned)L.npatch), dim3(kBlock), 0, s>>>(L.npatch, basis_of<T>(L), L.p_nloc, L.p_ld,
                                                                  full_off, L.p_inv_off, full,
                                                                  reinterpret_cast<T*>(L.inv));
  return hipGetLastError();
}

template <typename T>
hipError_t patch_apply(const DevLevel& L, const DevOps<T>& ops, const T* res, T* Y,
                       int transpose, hipStream_t s) {
  constexpr int VEC = Vec16<T>::n;
  const unsigned g = blocks_for(L.npatch, kWaves);
  const T* W = transpose ? ops.W : nullptr;
  const T* inv = reinterpret_cast<const T*>(L.inv);
  const int rows_per_block = 64 * VEC;
  if (L.pform == 3) {
    const StageBasis<T>& sb = basis_of<T>(L);
    const int max_ns = L.max_nloc / L.r;
    if (L.max_nloc > 1024 || max_ns > 256) return hipErrorInvalidValue;
#define IRK_PAS(NM, U, PF, WV, NT, RS)                                                                   \
  k_patch_apply_sym<T, NM, U, PF, WV, NT, RS><<<dim3(blocks_for(L.npatch, WV)), dim3(WV * 64), 0, s>>>( \
      L.npatch, sb, L.sched, L.p_nloc, L.p_inv_off, L.p_slot_off, L.p_gidx, inv, res, W, Y, transpose, \
      L.dim)
    // one wavefront per workgroup, two 16-byte words per row in flight; non-temporal
    // loads where the factors stream from memory once per application, ordinary loads
    // on the small levels, whose factors the last-level cache keeps between
    // applications; one row per lane up to 64 rows per block, else four (3D patches)
    const int nt = L.npatch <= kSmallPatches ? 0 : 1;
    if (max_ns <= 64) {
      if (L.max_nloc <= 128) {
        if (nt) IRK_PAS(128, 2, 0, 1, 1, 1);
        else IRK_PAS(128, 2, 0, 1, 0, 1);
      } else if (nt) IRK_PAS(256, 2, 0, 1, 1, 1);
      else IRK_PAS(256, 2, 0, 1, 0, 1);
    } else if (L.max_nloc <= 256) {
      if (nt) IRK_PAS(256, 2, 0, 1, 1, 4);
      else IRK_PAS(256, 2, 0, 1, 0, 4);
    } else if (L.max_nloc <= 512) {
      if (nt) IRK_PAS(512, 2, 0, 1, 1, 4);
      else IRK_PAS(512, 2, 0, 1, 0, 4);
    } else if (nt) IRK_PAS(1024, 2, 0, 1, 1, 4);
    else IRK_PAS(1024, 2, 0, 1, 0, 4);
#undef IRK_PAS
    return hipGetLastError();
  }
  if (L.pform == 1) {
    const StageBasis<T>& sb = basis_of<T>(L);
    const int rbe = (L.max_ld + rows_per_block - 1) / rows_per_block;
#define IRK_PAE(RBV, NM, U, NT, WV, ...)                                                              \
  k_patch_apply_eig<T, RBV, NM, U, NT, WV, ##__VA_ARGS__><<<dim3(blocks_for(L.npatch, WV)), dim3(WV * 64), 0, s>>>( \
      L.npatch, sb, L.sched, L.p_nloc, L.p_ld, L.p_inv_off, L.p_slot_off, L.p_gidx, inv, res, W, Y,  \
      transpose, L.dim)
    // 4 columns in flight per lane, non-temporal loads (ordinary ones on the small
    // levels): at 62 VGPRs the 2D kernel runs 8 waves per SIMD; deeper unrolling
    // lowered occupancy and measured slower
    const bool small = L.npatch <= kSmallPatches;
    if (small && L.max_nloc <= 128 && rbe <= 1) IRK_PAE(1, 128, 4, 0, 4);
    else if (L.max_nloc <= 128 && rbe <= 1) IRK_PAE(1, 128, 4, 1, 4);
    else if (L.max_nloc <= 256 && rbe <= 2) IRK_PAE(2, 256, 4, 1, 4);
    else if (L.max_nloc <= 512 && rbe <= 2) IRK_PAE(2, 512, 4, 1, 4);
    else if (L.max_nloc <= 512 && rbe <= 4) IRK_PAE(4, 512, 2, 1, 4);
    else if (L.max_nloc <= 1024 && rbe <= 4) IRK_PAE(4, 1024, 2, 1, 4);
    else if (L.max_nloc <= 1024 && rbe <= 8) IRK_PAE(8, 1024, 2, 1, 4);
    else return hipErrorInvalidValue;
#undef IRK_PAE
    return hipGetLastError();
  }
  const int rb = (L.max_nloc + rows_per_block - 1) / rows_per_block;
#define IRK_PA(RBV, NM)                                                                        \
  k_patch_apply<T, RBV, NM><<<dim3(g), dim3(kWaves * 64), 0, s>>>(L.npatch,  \
                     L.sched, L.p_nloc, L.p_ld, L.p_inv_off, L.p_slot_off, L.p_gidx, inv, res, \
                     W, Y, transpose, L.dim, L.r)
  if (L.max_nloc <= 128) {
    if (rb == 1) IRK_PA(1, 128); else IRK_PA(2, 128);
  } else if (L.max_nloc <= 256) {
    if (rb == 1) IRK_PA(1, 256); else IRK_PA(2, 256);
  } else if (L.max_nloc <= 512) {
    if (rb <= 2) IRK_PA(2, 512); else if (rb <= 4) IRK_PA(4, 512); else return hipErrorInvalidValue;
  } else if (L.max_nloc <= 1024) {
    if (rb <= 4) IRK_PA(4, 1024); else if (rb <= 8) IRK_PA(8, 1024); else return hipErrorInvalidValue;
  } else {
    return hipErrorInvalidValue;
  }
#undef IRK_PA
  return hipGetLastError();
}

template <typename T>
hipError_t gather_update(const DevLevel& L, const DevOps<T>& ops, const T* Y, T* x, T omega,
                         int mode, hipStream_t s) {
  k_gather_update<T><<<dim3(blocks_for(L.nsl_g, kBlock / 64)), dim3(kBlock), 0, s>>>(
      L.N, L.nsl_g, L.g_off, L.g_w, L.g_slot, Y, ops.W, omega, mode, x);
  return hipGetLastError();
}

template <typename T>
hipError_t gather_cheb(const DevLevel& L, const DevOps<T>& ops, const T* Y, T c1, T c2, int first, int xzero,
                       int transpose, T* d, T* x, hipStream_t s) {
  k_gather_cheb<T><<<dim3(blocks_for(L.nsl_g, kBlock / 64)), dim3(kBlock), 0, s>>>(
      L.N, L.nsl_g, L.g_off, L.g_w, L.g_slot, Y, transpose ? nullptr : ops.W, c1, c2, first, xzero, d, x);
  return hipGetLastError();
}

template <typename T>
hipError_t restrict_(const DevLevel& F, const DevLevel& C, const DevOps<T>& fops, const T* xf,
                     T* xc, hipStream_t s) {
  const unsigned g = blocks_for(C.nfree + C.nv);
  IRK_DISPATCH_DR(F.dim, F.r, (k_spmv_nodes<DD, RR, T><<<dim3(g), dim3(kBlock), 0, s>>>(C.nfree, C.nv, C.offV, F.offV, F.put_ptr, F.put_col,
                                                  fops.put_val, F.ppt_ptr, F.ppt_col, fops.ppt_val, xf,
                                                  xc, 0)));
  return hipGetLastError();
}

template <typename T>
hipError_t prolong_add(const DevLevel& F, const DevLevel& C, const DevOps<T>& fops, const T* xc,
                       T* xf, hipStream_t s) {
  const unsigned g = blocks_for(F.nfree + F.nv);
  IRK_DISPATCH_DR(F.dim, F.r, (k_spmv_nodes<DD, RR, T><<<dim3(g), dim3(kBlock), 0, s>>>(F.nfree, F.nv, F.offV, C.offV, F.pu_ptr, F.pu_col,
                                                  fops.pu_val, F.pp_ptr, F.pp_col, fops.pp_val, xc,
                                                  xf, 1)));
  return hipGetLastError();
}

template <typename T>
hipError_t gr_dots(const T* V, int64_t ldv, int nv, const T* w, int64_t n, double* part, double* out,
                   hipStream_t s) {
  if (nv < 1 || nv > kMaxGr + 1) return hipErrorInvalidValue;
  const int nb = (int)std::min<int64_t>(kGrBlocks, blocks_for(n));
  k_gr_dots<T><<<dim3(nb), dim3(kBlock), 0, s>>>(n, nv, V, ldv, w, part);
  k_gr_finish<<<dim3(1), dim3(kBlock), 0, s>>>(part, nb, nv, 0, out);
  return hipGetLastError();
}

template <typename T>
hipError_t gr_orth_norm(T* w, const T* V, int64_t ldv, int j, int64_t n, const double* h, double* part,
                        double* nrm, hipStream_t s) {
  const int nb = (int)std::min<int64_t>(kGrBlocks, blocks_for(n));
  k_gr_orth<T><<<dim3(nb), dim3(kBlock), 0, s>>>(n, j, V, ldv, h, w, part);
  k_gr_finish<<<dim3(1), dim3(kBlock), 0, s>>>(part, nb, 1, 1, nrm);
  return hipGetLastError();
}

template <typename T>
hipError_t gr_scale(T* v, int64_t n, const double* d, hipStream_t s) {
  k_gr_scale<T><<<dim3(blocks_for(n)), dim3(kBlock), 0, s>>>(n, d, v);
  return hipGetLastError();
}

hipError_t gr_solve(double* gr, int m, hipStream_t s) {
  if (m < 1 || m > kMaxGr) return hipErrorInvalidValue;
  k_gr_solve<<<dim3(1), dim3(64), 0, s>>>(gr, m);
  return hipGetLastError();
}

template <typename T>
hipError_t gr_update(T* x, const T* V, int64_t ldv, int m, int64_t n, const double* y, int assign, hipStream_t s) {
  k_gr_update<T><<<dim3(blocks_for(n)), dim3(kBlock), 0, s>>>(n, m, V, ldv, y, assign, x);
  return hipGetLastError();
}

hipError_t dense_inverse(double* J, int64_t N, double tol, double* colk, int64_t* swp, int* fail, hipStream_t s) {
  const unsigned gu = (unsigned)((N * N + kBlock - 1) / kBlock);
  for (int64_t k = 0; k < N; ++k) {
    k_gj_pivot<<<dim3(1), dim3(1024), 0, s>>>(J, N, k, tol, colk, swp, fail);
    k_gj_update<<<dim3(gu), dim3(kBlock), 0, s>>>(J, N, k, colk, fail);
  }
  k_gj_unswap<<<dim3(1), dim3(1024), 0, s>>>(J, N, swp, fail);
  return hipGetLastError();
}

hipError_t transpose(const double* in, double* out, int64_t N, hipStream_t s) {
  const unsigned g = (unsigned)((N + 31) / 32);
  k_transpose<<<dim3(g, g), dim3(256), 0, s>>>(in, out, N);
  return hipGetLastError();
}

hipError_t coarse_solve(const double* inv, const double* mat, int64_t N, double* b, double* x,
                        const int64_t* pins, int npins, double* part, hipStream_t s) {
  const dim3 gp((unsigned)((N + 63) / 64), kCoarseSplit), gr(blocks_for(N));
  if (pins && npins > 0) k_zero_pins<<<dim3(1), dim3(64), 0, s>>>(b, pins, npins);
  k_coarse_gemv_part<<<gp, dim3(kBlock), 0, s>>>(inv, N, b, part);
  k_coarse_reduce<<<gr, dim3(kBlock), 0, s>>>(part, N, x, 0);
  if (mat) {  // one step of iterative refinement: b <- b - M x, x <- x + inv b
    k_coarse_gemv_part<<<gp, dim3(kBlock), 0, s>>>(mat, N, x, part);
    k_coarse_reduce<<<gr, dim3(kBlock), 0, s>>>(part, N, b, 1);
    k_coarse_gemv_part<<<gp, dim3(kBlock), 0, s>>>(inv, N, b, part);
    k_coarse_reduce<<<gr, dim3(kBlock), 0, s>>>(part, N, x, 2);
  }
  return hipGetLastError();
}

int coarse_split() { return kCoarseSplit * (kBlock / 64); }

template <typename T>
hipError_t to_internal(const DevLevel& L, const double* abi, T* x, hipStream_t s) {
  const int64_t ns = L.dim * L.nfree + L.nv;
  k_permute<T><<<dim3(blocks_for(L.N)), dim3(kBlock), 0, s>>>(L.N, L.offV,
                     L.nfree, ns, L.dim, L.r, abi, x, 1, nullptr, nullptr);
  return hipGetLastError();
}

template <typename T>
hipError_t to_abi(const DevLevel& L, const T* x, double* abi, hipStream_t s) {
  const int64_t ns = L.dim * L.nfree + L.nv;
  k_permute<T><<<dim3(blocks_for(L.N)), dim3(kBlock), 0, s>>>(L.N, L.offV,
                     L.nfree, ns, L.dim, L.r, nullptr, nullptr, 0, x, abi);
  return hipGetLastError();
}

template <typename S, typename D>
hipError_t cast(const S* in, D* out, int64_t n, hipStream_t s) {
  k_cast<S, D><<<dim3(blocks_for(n)), dim3(kBlock), 0, s>>>(in, out, n);
  return hipGetLastError();
}

hipError_t project_pressure(const DevLevel& L, double* x, double* partials, hipStream_t s) {
  static_assert(kProjBlocks <= kBlock && kProjBlocks * kMaxStages <= 1024, "partials buffer holds 1024 values");
  const int nb = (int)std::min<int64_t>(kProjBlocks, blocks_for(L.nv));
  k_project_partial<<<dim3(nb), dim3(kBlock), 0, s>>>(x, L.offV, L.nv, L.r, partials);
  const unsigned ga = (unsigned)std::min<int64_t>(1024, blocks_for(L.nv * L.r));
  k_project_apply<<<dim3(ga), dim3(kBlock), 0, s>>>(x, L.offV, L.nv, L.r, partials, nb);
  return hipGetLastError();
}

hipError_t dot(const double* a, const double* b, int64_t n, double* partials, double* out,
               hipStream_t s, int take_sqrt) {
  const int nb = (int)std::min<int64_t>(kReduceBlocks, blocks_for(n));
  k_dot_partial<<<dim3(nb), dim3(kBlock), 0, s>>>(a, b, n, partials);
  k_dot_final<<<dim3(1), dim3(kBlock), 0, s>>>(partials, nb, out, take_sqrt);
  return hipGetLastError();
}

hipError_t mgs_arnoldi(double* w, const double* V, int64_t n, int j, double* partials, double* hcol,
                       hipStream_t s) {
  const int nb = (int)std::min<int64_t>(kReduceBlocks, blocks_for(n));
  static_assert(2 * kReduceBlocks <= 1024, "two partial-sum buffers in the 1024-value workspace");
  double* pa = partials;
  double* pb = partials + kReduceBlocks;
  k_dot_partial<<<dim3(nb), dim3(kBlock), 0, s>>>(w, V, n, pa);
  for (int i = 0; i <= j; ++i) {
    const double* vnext = i < j ? V + (size_t)(i + 1) * n : nullptr;
    k_mgs_step<<<dim3(nb), dim3(kBlock), 0, s>>>(w, V + (size_t)i * n, vnext, n, pa, nb, pb, hcol + i);
    std::swap(pa, pb);
  }
  k_mgs_normalize<<<dim3(nb), dim3(kBlock), 0, s>>>(w, n, pa, nb, hcol + j + 1);
  return hipGetLastError();
}

hipError_t axpy_dev(double* y, const double* x, int64_t n, const double* dev_scalar,
                    double sign, hipStream_t s) {
  k_axpy_dev<<<dim3(blocks_for(n)), dim3(kBlock), 0, s>>>(y, x, n, dev_scalar,
                     sign, sign);
  return hipGetLastError();
}

hipError_t scale_inv_dev(double* y, const double* x, int64_t n, const double* dev_scalar,
                         hipStream_t s) {
  k_scale_inv<<<dim3(blocks_for(n)), dim3(kBlock), 0, s>>>(y, x, n, dev_scalar);
  return hipGetLastError();
}

hipError_t update_sum(double* x, const double* Z, int64_t n, const double* c, int m, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  k_update_sum<<<dim3(blocks_for(n)), dim3(kBlock), 0, s>>>(x, Z, n, c, m);
  return hipGetLastError();
}

hipError_t axpby(double* y, const double* x, int64_t n, double a, double b, hipStream_t s) {
  k_axpby<<<dim3(blocks_for(n)), dim3(kBlock), 0, s>>>(y, x, n, a, b);
  return hipGetLastError();
}

hipError_t fill(double* y, int64_t n, double v, hipStream_t s) {
  k_fill<double><<<dim3(blocks_for(n)), dim3(kBlock), 0, s>>>(y, n, v);
  return hipGetLastError();
}

hipError_t fillf(float* y, int64_t n, float v, hipStream_t s) {
  k_fill<float><<<dim3(blocks_for(n)), dim3(kBlock), 0, s>>>(y, n, v);
  return hipGetLastError();
}

hipError_t nonfinite(const double* x, int64_t n, int* flag, hipStream_t s) {
  k_nonfinite<<<dim3(blocks_for(n)), dim3(kBlock), 0, s>>>(x, n, flag);
  return hipGetLastError();
}

hipError_t rhs(const DevLevel& L, int64_t nnodes, const double* f, const double* state,
                    double* F, hipStream_t s) {
  k_rhs<<<dim3(blocks_for(L.nfree + L.nv)), dim3(kBlock), 0, s>>>(L.nfree, L.nv,
                     nnodes, L.dim, L.r, L.mfa_ptr, L.mfa_col, L.mfa_val, L.s_ptr, L.s_col,
                     L.d64.s_L, L.b_ptr, L.b_col, L.d64.b_val, L.bt_ptr, L.bt_col, L.d64.bt_val, f,
                     state, F);
  return hipGetLastError();
}

hipError_t rhs_dirichlet(const DevLevel& L, const double* Ainv_dt, const double* g_n, const double* g_st,
                         double* F, hipStream_t s) {
  Coef<double> c{};
  for (int i = 0; i < L.r * L.r; ++i) c.v[i] = Ainv_dt[i];
  k_rhs_dirichlet<<<dim3(blocks_for(L.nfree + L.nv)), dim3(kBlock), 0, s>>>(
      L.nfree, L.nv, L.nnodes, L.dim, L.r, L.fb_ptr, L.fb_col, L.fb_m, L.fb_l, L.vb_ptr, L.vb_col, L.vb_val, c, g_n,
      g_st, F);
  return hipGetLastError();
}

hipError_t update(const DevLevel& L, const double* b, double dt, const double* kv, double* state,
                  hipStream_t s) {
  Coef<double> c{};
  for (int j = 0; j < L.r; ++j) c.v[j] = dt * b[j];
  const int64_t ns = L.dim * L.nfree + L.nv;
  k_update<<<dim3(blocks_for(ns)), dim3(kBlock), 0, s>>>(ns, L.r, c, kv, state);
  return hipGetLastError();
}

hipError_t rhs_adjoint(const DevLevel& L, int64_t nnodes, const int32_t* mt_ptr, const int32_t* mt_col,
                       const double* mt_val, const double* lam, double* gf, double* gstate, int accumulate,
                       hipStream_t s) {
  k_rhs_adjoint_f<<<dim3(blocks_for(nnodes)), dim3(kBlock), 0, s>>>(nnodes, L.nfree, L.nv, L.dim, L.r, mt_ptr,
                                                                    mt_col, mt_val, lam, gf);
  k_rhs_adjoint_s<<<dim3(blocks_for(L.nfree + L.nv)), dim3(kBlock), 0, s>>>(
      L.nfree, L.nv, L.dim, L.r, L.s_ptr, L.s_col, L.d64.s_Lt, L.b_ptr, L.b_col, L.d64.b_val, L.bt_ptr, L.bt_col,
      L.d64.bt_val, lam, gstate, accumulate);
  return hipGetLastError();
}

hipError_t update_adjoint(const DevLevel& L, const double* b, double dt, const double* gs, double* G,
                          hipStream_t s) {
  Coef<double> c{};
  for (int j = 0; j < L.r; ++j) c.v[j] = dt * b[j];
  const int64_t ns = L.dim * L.nfree + L.nv;
  k_update_adjoint<<<dim3(blocks_for(ns)), dim3(kBlock), 0, s>>>(ns, L.r, c, gs, G);
  return hipGetLastError();
}

hipError_t nu_sensitivity(const DevLevel& L, const double* A, double dt, const double* lam, const double* kv,
                          const double* state, double* rowsum, double* partials, double* out, int accumulate,
                          hipStream_t s) {
  Coef<double> c{};
  for (int i = 0; i < L.r * L.r; ++i) c.v[i] = dt * A[i];
  k_nu_rows<<<dim3(blocks_for(L.nfree)), dim3(kBlock), 0, s>>>(L.nfree, L.nv, L.dim, L.r, c, L.s_ptr, L.s_col,
                                                               L.s_K1, lam, kv, state, rowsum);
  const int nb = (int)std::min<int64_t>(kReduceBlocks, blocks_for(L.nfree));
  k_sum_partial<<<dim3(nb), dim3(kBlock), 0, s>>>(rowsum, L.nfree, partials);
  k_dot_final<<<dim3(1), dim3(kBlock), 0, s>>>(partials, nb, out, accumulate ? 2 : 0);
  return hipGetLastError();
}

hipError_t tracking_loss(const DevLevel& L, const double* state, const double* target, const double* scale,
                         double* loss, double* grad_state, double* grad_target, double* e, double* Me,
                         double* partials, hipStream_t s) {
  const int64_t nvel = (int64_t)L.dim * L.nfree, ns = nvel + L.nv;
  k_velocity_diff<<<dim3(blocks_for(ns)), dim3(kBlock), 0, s>>>(nvel, ns, state, target, e);
  k_mass_apply<<<dim3(blocks_for(L.nfree + L.nv)), dim3(kBlock), 0, s>>>(L.nfree, L.nv, L.dim, L.s_ptr, L.s_col,
                                                                         L.d64.s_M, e, Me);
  if (loss) {
    const int nb = (int)std::min<int64_t>(kReduceBlocks, blocks_for(ns));
    k_dot_partial<<<dim3(nb), dim3(kBlock), 0, s>>>(e, Me, ns, partials);
    k_dot_final<<<dim3(1), dim3(kBlock), 0, s>>>(partials, nb, loss, 3);
  }
  if (grad_state || grad_target)
    k_scaled_pair<<<dim3(blocks_for(ns)), dim3(kBlock), 0, s>>>(ns, scale, Me, grad_state, grad_target);
  return hipGetLastError();
}

hipError_t mass_apply(const DevLevel& L, const double* st, double* out, hipStream_t s) {
  k_mass_apply<<<dim3(blocks_for(L.nfree + L.nv)), dim3(kBlock), 0, s>>>(L.nfree, L.nv, L.dim, L.s_ptr, L.s_col,
                                                                         L.d64.s_M, st, out);
  return hipGetLastError();
}

// explicit instantiations
#define IRK_INST(T)                                                                              \
  template hipError_t residual<T>(const DevLevel&, const DevOps<T>&, const double*, double,     \
                                  const T*, const T*, T*, hipStream_t);                         \
  template hipError_t patch_factor_range<T>(const DevLevel&, const DevOps<T>&, int, const double*, \
                                            double, const int32_t*, const int64_t*, T*, int64_t,   \
                                            int64_t, int64_t, int, int*, hipStream_t, const T*);   \
  template hipError_t patch_factor_scalar<T>(const DevLevel&, const DevOps<T>&, int, const double*, double,   \
                                             const int32_t*, const int64_t*, T*, int64_t, int64_t, int64_t,  \
                                             int, int*, hipStream_t);                                        \
  template hipError_t patch_factor_cplx<T>(const DevLevel&, const DevOps<T>&, double, double, int, int, \
                                           int*, hipStream_t);                                        \
  template hipError_t eig_extract<T>(const DevLevel&, const StageBasis<T>&, int, const int32_t*,  \
                                     const int64_t*, int64_t, const T*, int64_t, int64_t,          \
                                     hipStream_t);                                                 \
  template hipError_t patch_apply<T>(const DevLevel&, const DevOps<T>&, const T*, T*, int,      \
                                     hipStream_t);                                              \
  template hipError_t pack_sym<T>(const DevLevel&, const int64_t*, const T*, hipStream_t);      \
  template hipError_t gr_dots<T>(const T*, int64_t, int, const T*, int64_t, double*, double*, hipStream_t); \
  template hipError_t gr_orth_norm<T>(T*, const T*, int64_t, int, int64_t, const double*, double*, double*, \
                                      hipStream_t);                                                       \
  template hipError_t gr_scale<T>(T*, int64_t, const double*, hipStream_t);                              \
  template hipError_t gr_update<T>(T*, const T*, int64_t, int, int64_t, const double*, int, hipStream_t); \
  template hipError_t gather_cheb<T>(const DevLevel&, const DevOps<T>&, const T*, T, T, int, int, int, T*, \
                                     T*, hipStream_t);                                                  \
  template hipError_t gather_update<T>(const DevLevel&, const DevOps<T>&, const T*, T*, T, int, \
                                       hipStream_t);                                            \
  template hipError_t restrict_<T>(const DevLevel&, const DevLevel&, const DevOps<T>&, const T*, \
                                   T*, hipStream_t);                                            \
  template hipError_t prolong_add<T>(const DevLevel&, const DevLevel&, const DevOps<T>&,        \
                                     const T*, T*, hipStream_t);                                \
  template hipError_t to_internal<T>(const DevLevel&, const double*, T*, hipStream_t);         \
  template hipError_t to_abi<T>(const DevLevel&, const T*, double*, hipStream_t);
IRK_INST(double)
IRK_INST(float)
template hipError_t cast<double, float>(const double*, float*, int64_t, hipStream_t);
template hipError_t cast<float, double>(const float*, double*, int64_t, hipStream_t);
template hipError_t cast<double, double>(const double*, double*, int64_t, hipStream_t);

}  // namespace k
}  // namespace irk
