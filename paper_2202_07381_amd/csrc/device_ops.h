// Device-side bodies of the V-cycle operations, shared by the one-launch-per-step
// kernels (kernels.hip) and the persistent batched solver (batch.hip).  Each function
// does the work of one row, one DOF or one patch; the callers map threads to work.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "irk_internal.h"

namespace irk {
namespace dev {

template <typename T>
struct Coef {
  T v[kMaxStages * kMaxStages];
};

// r = F - J x (F may be null: y = J x) for one row of the internal layout:
// rows [0, nfree) are velocity nodes (dim*r outputs), rows [nfree, nfree+nv) vertices.
template <int D, int R, typename T>
__device__ __forceinline__ void residual_row(
    int64_t row, int64_t nfree, int64_t nv, int64_t offV, const int32_t* __restrict__ s_ptr,
    const int32_t* __restrict__ s_col, const T* __restrict__ sM, const T* __restrict__ sL,
    const int32_t* __restrict__ b_ptr, const int32_t* __restrict__ b_col,
    const T* __restrict__ b_val, const int32_t* __restrict__ bt_ptr,
    const int32_t* __restrict__ bt_col, const T* __restrict__ bt_val, const Coef<T>& dtA,
    const T* __restrict__ F, const T* __restrict__ x, T* __restrict__ y) {
  constexpr int DR = D * R;
  if (row < nfree) {
    T am[DR], al[DR];
#pragma unroll
    for (int q = 0; q < DR; ++q) am[q] = al[q] = T(0);
    const int32_t p0 = s_ptr[row], p1 = s_ptr[row + 1];
    for (int32_t p = p0; p < p1; ++p) {
      const int64_t j = s_col[p];
      const T m = sM[p], l = sL[p];
      const T* xj = x + j * DR;
#pragma unroll
      for (int q = 0; q < DR; ++q) {
        const T xv = xj[q];
        am[q] += m * xv;
        al[q] += l * xv;
      }
    }
    const int32_t q0 = b_ptr[row], q1 = b_ptr[row + 1];
    for (int32_t p = q0; p < q1; ++p) {
      const T* xp = x + offV + (int64_t)b_col[p] * R;
      T pv[R];
#pragma unroll
      for (int t = 0; t < R; ++t) pv[t] = xp[t];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const T bv = b_val[(int64_t)p * D + c];
#pragma unroll
        for (int t = 0; t < R; ++t) al[c * R + t] += bv * pv[t];
      }
    }
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
  } else if (row < nfree + nv) {
    const int64_t v = row - nfree;
    T a[R];
#pragma unroll
    for (int t = 0; t < R; ++t) a[t] = T(0);
    const int32_t p0 = bt_ptr[v], p1 = bt_ptr[v + 1];
    for (int32_t p = p0; p < p1; ++p) {
      const T* xi = x + (int64_t)bt_col[p] * DR;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const T bv = bt_val[(int64_t)p * D + c];
#pragma unroll
        for (int t = 0; t < R; ++t) a[t] += bv * xi[c * R + t];
      }
    }
#pragma unroll
    for (int s = 0; s < R; ++s) {
      T acc = T(0);
#pragma unroll
      for (int t = 0; t < R; ++t) acc += dtA.v[s * R + t] * a[t];
      const int64_t o = offV + v * R + s;
      y[o] = F ? F[o] - acc : acc;
    }
  }
}

template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int n = 2;
};
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int n = 4;
};

template <typename V, typename T>
__device__ inline void vload(const T* p, T* out);
template <>
__device__ inline void vload<double2, double>(const double* p, double* o) {
  const double2 v = *reinterpret_cast<const double2*>(p);
  o[0] = v.x;
  o[1] = v.y;
}
template <>
__device__ inline void vload<float4, float>(const float* p, float* o) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = v.x;
  o[1] = v.y;
  o[2] = v.z;
  o[3] = v.w;
}

// One wavefront applies the stored inverse of patch p.  Lane l owns rows
// [rb*64*VEC + l*VEC, +VEC) of row block rb.  Non-transposed: y = Ainv x streams
// column j with one 16-byte load per lane; transposed: y_j = column_j . x with a wave
// reduction per column.  xs is this wavefront's LDS staging area (>= n values).
template <typename T, int RB, int UNROLL = 4>
__device__ __forceinline__ void patch_apply_one(
    int p, int lane, T* xs, const int32_t* __restrict__ p_nloc, const int32_t* __restrict__ p_ld,
    const int64_t* __restrict__ p_inv_off, const int64_t* __restrict__ p_slot_off,
    const int32_t* __restrict__ gidx, const T* __restrict__ inv, const T* __restrict__ res,
    const T* __restrict__ W, T* __restrict__ Y, int transpose) {
  using VT = typename Vec16<T>::type;
  constexpr int VEC = Vec16<T>::n;
  const int n = p_nloc[p];
  const int ld = p_ld[p];
  const int64_t so = p_slot_off[p];
  const T* __restrict__ Ap = inv + p_inv_off[p];
  for (int i = lane; i < n; i += 64) {
    const int32_t g = gidx[so + i];
    xs[i] = W ? res[g] * W[g] : res[g];
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (!transpose) {
    T acc[RB][VEC];
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[b][v] = T(0);
    int j = 0;
    for (; j + UNROLL <= n; j += UNROLL) {
      T a[UNROLL][RB][VEC];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u)
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          const int r0 = b * 64 * VEC + lane * VEC;
          if (r0 < n) vload<VT, T>(Ap + (int64_t)(j + u) * ld + r0, a[u][b]);
          else
#pragma unroll
            for (int v = 0; v < VEC; ++v) a[u][b][v] = T(0);
        }
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const T xj = xs[j + u];
#pragma unroll
        for (int b = 0; b < RB; ++b)
#pragma unroll
          for (int v = 0; v < VEC; ++v) acc[b][v] += a[u][b][v] * xj;
      }
    }
    for (; j < n; ++j) {
      const T xj = xs[j];
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const int r0 = b * 64 * VEC + lane * VEC;
        if (r0 < n) {
          T a[VEC];
          vload<VT, T>(Ap + (int64_t)j * ld + r0, a);
#pragma unroll
          for (int v = 0; v < VEC; ++v) acc[b][v] += a[v] * xj;
        }
      }
    }
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const int row = b * 64 * VEC + lane * VEC + v;
        if (row < n) Y[so + row] = acc[b][v];
      }
  } else {
    for (int j = 0; j < n; ++j) {
      T part = T(0);
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const int r0 = b * 64 * VEC + lane * VEC;
        if (r0 < n) {
          T a[VEC];
          vload<VT, T>(Ap + (int64_t)j * ld + r0, a);
#pragma unroll
          for (int v = 0; v < VEC; ++v)
            if (r0 + v < n) part += a[v] * xs[r0 + v];
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
      if (lane == 0) Y[so + j] = part;
    }
  }
  // xs is reused by this wavefront's next patch
  __builtin_amdgcn_wave_barrier();
}

// Owner gather of one DOF.  mode 0: x = omega*W*s   1: x += omega*W*s
//                           2: x = omega*s     3: x += omega*s
template <typename T>
__device__ __forceinline__ void gather_one(int64_t g, const int32_t* __restrict__ gptr,
                                           const int32_t* __restrict__ gslot,
                                           const T* __restrict__ Y, const T* __restrict__ W,
                                           T omega, int mode, T* __restrict__ x) {
  T s = T(0);
  const int32_t q1 = gptr[g + 1];
  for (int32_t q = gptr[g]; q < q1; ++q) s += Y[gslot[q]];
  T c = omega * s;
  if (mode < 2) c *= W[g];
  x[g] = (mode & 1) ? x[g] + c : c;
}

// One row of a node-chunked CSR product (restriction / prolongation).
template <int D, int R, typename T>
__device__ __forceinline__ void spmv_nodes_row(
    int64_t row, int64_t nrow_u, int64_t nrow_p, int64_t out_offV, int64_t in_offV,
    const int32_t* __restrict__ u_ptr, const int32_t* __restrict__ u_col,
    const T* __restrict__ u_val, const int32_t* __restrict__ p_ptr,
    const int32_t* __restrict__ p_col, const T* __restrict__ p_val, const T* __restrict__ in,
    T* __restrict__ out, int add) {
  constexpr int DR = D * R;
  if (row < nrow_u) {
    T acc[DR];
#pragma unroll
    for (int q = 0; q < DR; ++q) acc[q] = T(0);
    for (int32_t p = u_ptr[row]; p < u_ptr[row + 1]; ++p) {
      const T w = u_val[p];
      const T* xi = in + (int64_t)u_col[p] * DR;
#pragma unroll
      for (int q = 0; q < DR; ++q) acc[q] += w * xi[q];
    }
#pragma unroll
    for (int q = 0; q < DR; ++q) {
      const int64_t o = row * DR + q;
      out[o] = add ? out[o] + acc[q] : acc[q];
    }
  } else if (row < nrow_u + nrow_p) {
    const int64_t v = row - nrow_u;
    T acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = T(0);
    for (int32_t p = p_ptr[v]; p < p_ptr[v + 1]; ++p) {
      const T w = p_val[p];
      const T* xi = in + in_offV + (int64_t)p_col[p] * R;
#pragma unroll
      for (int q = 0; q < R; ++q) acc[q] += w * xi[q];
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t o = out_offV + v * R + q;
      out[o] = add ? out[o] + acc[q] : acc[q];
    }
  }
}

}  // namespace dev
}  // namespace irk
