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

// 16-byte load that bypasses cache retention (the patch factors are streamed once per
// application and would only evict the gathered vectors)
template <typename T>
__device__ inline void vload_nt(const T* p, T* out);
template <>
__device__ inline void vload_nt<double>(const double* p, double* o) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  const d2 v = __builtin_nontemporal_load(reinterpret_cast<const d2*>(p));
  o[0] = v.x;
  o[1] = v.y;
}
template <>
__device__ inline void vload_nt<float>(const float* p, float* o) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const f4 v = __builtin_nontemporal_load(reinterpret_cast<const f4*>(p));
  o[0] = v.x;
  o[1] = v.y;
  o[2] = v.z;
  o[3] = v.w;
}
template <typename T, int NT>
__device__ __forceinline__ void vload_s(const T* p, T* o) {
  if constexpr (NT) vload_nt<T>(p, o);
  else vload<typename Vec16<T>::type, T>(p, o);
}

// Output slot of local index e of a patch (stage-major: e = s ns + q with q = c nn + a
// for velocity component c of patch node a, q = D nn for the pressure) in the patch's
// node-major output order ((a D + c) R + s, pressure nn D R + s), so that the D R values
// of one node, which the gather reads together, are contiguous.
__device__ __forceinline__ int node_major_slot(int e, int ns, int D, int R) {
  const int s = e / ns, q = e - s * ns;
  const int nn = (ns - 1) / D;
  if (q < D * nn) {
    const int c = q / nn, a = q - c * nn;
    return (a * D + c) * R + s;
  }
  return nn * D * R + s;
}

// One wavefront applies the stored inverse of patch p.  Lane l owns rows
// [rb*64*VEC + l*VEC, +VEC) of row block rb.  Non-transposed: y = Ainv x streams
// column j with one 16-byte load per lane; transposed: y_j = column_j . x with a wave
// reduction per column.  xs is this wavefront's LDS staging area (>= n values).
template <typename T, int RB, int UNROLL = 4, int NT = 1>
__device__ __forceinline__ void patch_apply_one(
    int p, int lane, T* xs, const int32_t* __restrict__ p_nloc, const int32_t* __restrict__ p_ld,
    const int64_t* __restrict__ p_inv_off, const int64_t* __restrict__ p_slot_off,
    const int32_t* __restrict__ gidx, const T* __restrict__ inv, const T* __restrict__ res,
    const T* __restrict__ W, T* __restrict__ Y, int transpose, int D, int R) {
  using VT = typename Vec16<T>::type;
  constexpr int VEC = Vec16<T>::n;
  const int n = p_nloc[p];
  const int ns = n / R;
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
          if (r0 < n) vload_s<T, NT>(Ap + (int64_t)(j + u) * ld + r0, a[u][b]);
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
          vload_s<T, NT>(Ap + (int64_t)j * ld + r0, a);
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
        if (row < n) Y[so + node_major_slot(row, ns, D, R)] = acc[b][v];
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
      if (lane == 0) Y[so + node_major_slot(j, ns, D, R)] = part;
    }
  }
  // xs is reused by this wavefront's next patch
  __builtin_amdgcn_wave_barrier();
}

// Gather of the (optionally weighted) patch residual into xs and its transform to the
// stage eigenbasis into xt: xt[k ns + q] = sum_s Tin(k, s) xs[s ns + q] with Tin = W^{-1}
// (forward) or W^T (transposed).  DUP: each transformed stage stored twice in a row,
// xt[k 2ns + q] = xt[k 2ns + ns + q], so that x[(q + s) mod ns] = xt[k 2ns + q + s].
template <typename T, bool DUP = false>
__device__ __forceinline__ void eig_in(int lane, int n, int ns, int64_t so, T* xs, T* xt,
                                       const irk::StageBasis<T>& sb, const int32_t* __restrict__ gidx,
                                       const T* __restrict__ res, const T* __restrict__ W, int transpose) {
  const int r = sb.r;
  for (int i = lane; i < n; i += 64) {
    const int32_t g = gidx[so + i];
    xs[i] = W ? res[g] * W[g] : res[g];
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int e = lane; e < n; e += 64) {
    const int k = e / ns, q = e - k * ns;
    T acc = T(0);
    for (int s = 0; s < r; ++s) acc += (transpose ? sb.W[s * r + k] : sb.Winv[k * r + s]) * xs[s * ns + q];
    if constexpr (DUP) {
      xt[k * 2 * ns + q] = acc;
      xt[k * 2 * ns + ns + q] = acc;
    } else {
      xt[e] = acc;
    }
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Back-transform of the block results in xs (forward W, transposed W^{-T}) and store of
// the n local corrections in the patch's node-major slots.
template <typename T>
__device__ __forceinline__ void eig_out(int lane, int n, int ns, int64_t so, const T* xs,
                                        const irk::StageBasis<T>& sb, T* __restrict__ Y, int transpose, int D) {
  const int r = sb.r;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int e = lane; e < n; e += 64) {
    const int s = e / ns, q = e - s * ns;
    T acc = T(0);
    for (int k = 0; k < r; ++k) acc += (transpose ? sb.Winv[k * r + s] : sb.W[s * r + k]) * xs[k * ns + q];
    Y[so + node_major_slot(e, ns, D, r)] = acc;
  }
  // xs and xt are reused by this wavefront's next patch
  __builtin_amdgcn_wave_barrier();
}

// Factored patch inverse (stage eigenbasis).  The stage-coupled patch matrix is
// I (x) M_v + dt A (x) S_v (Sec. 3 restricted to the patch of Sec. 4.2); with
// A = W T W^{-1} its inverse is (W (x) I) blockdiag_k(B_k^{-1}) (W^{-1} (x) I), where
// B_k = I (x) M_v + dt T_k (x) S_v.  Storage per patch: n_s columns of ld values; in a
// column the blocks follow each other, a real block as n_s values, a pair as n_s
// complex values (re, im).  For a pair, B_k^{-1} = [[P, -Q], [Q, P]] and the stored
// complex entry is P + iQ, so applying it is the complex product (P + iQ)(x1 + i x2).
//
// One wavefront per patch: gather x (LDS xs), transform to the eigenbasis (LDS xt),
// sweep the n_s columns (lane l owns VEC consecutive stored rows of every column, as in
// the dense form, and its chunk lies in one block), transform back and store the n
// local corrections.  Transposed (adjoint): x -> (W^T (x) I) x, B_k^{-T}, which for a
// pair is the conjugate transpose of P + iQ, and -> (W^{-T} (x) I); one wave reduction
// per column and block.
template <typename T>
__device__ __forceinline__ int eig_chunk_block(const irk::StageBasis<T>& sb, int ns, int row0, int* off) {
  constexpr int VEC = Vec16<T>::n;
  int base = 0;
  for (int b = 0; b < sb.nblk; ++b) {
    const int rows = irk::eig_block_rows(sb.type[b], ns, VEC);
    if (row0 < base + rows) {
      *off = row0 - base;
      return b;
    }
    base += rows;
  }
  return -1;
}

template <typename T, int RB, int UNROLL = 8, int NT = 0>
__device__ __forceinline__ void patch_apply_eig_one(
    int p, int lane, T* xs, T* xt, const irk::StageBasis<T>& sb, const int32_t* __restrict__ p_nloc,
    const int32_t* __restrict__ p_ld, const int64_t* __restrict__ p_inv_off,
    const int64_t* __restrict__ p_slot_off, const int32_t* __restrict__ gidx, const T* __restrict__ inv,
    const T* __restrict__ res, const T* __restrict__ W, T* __restrict__ Y, int transpose, int D) {
  using VT = typename Vec16<T>::type;
  constexpr int VEC = Vec16<T>::n;
  const int n = p_nloc[p];
  const int r = sb.r;
  const int ns = n / r;
  const int lc = p_ld[p];
  const int64_t so = p_slot_off[p];
  const T* __restrict__ Ap = inv + p_inv_off[p];
  eig_in<T>(lane, n, ns, so, xs, xt, sb, gidx, res, W, transpose);
  // this lane's chunks: block, offset inside the block, inputs (u, v) per column
  int blk[RB], off[RB], iu[RB], iv[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const int row0 = b * 64 * VEC + lane * VEC;
    off[b] = 0;
    blk[b] = row0 < lc ? eig_chunk_block(sb, ns, row0, &off[b]) : -1;
    iu[b] = blk[b] >= 0 ? sb.st0[blk[b]] * ns : 0;
    iv[b] = (blk[b] >= 0 && sb.type[blk[b]] == 2) ? iu[b] + ns : -1;
  }
  if (!transpose) {
    T acc[RB][VEC];
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[b][v] = T(0);
    int j = 0;
    for (; j + UNROLL <= ns; j += UNROLL) {
      T a[UNROLL][RB][VEC];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u)
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          if (blk[b] >= 0) vload_s<T, NT>(Ap + (int64_t)(j + u) * lc + b * 64 * VEC + lane * VEC, a[u][b]);
          else
#pragma unroll
            for (int v = 0; v < VEC; ++v) a[u][b][v] = T(0);
        }
#pragma unroll
      for (int u = 0; u < UNROLL; ++u)
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          const T xu = xt[iu[b] + j + u];
          const T xv = iv[b] >= 0 ? xt[iv[b] + j + u] : T(0);
#pragma unroll
          for (int m = 0; m < VEC / 2; ++m) {
            acc[b][2 * m] += a[u][b][2 * m] * xu - a[u][b][2 * m + 1] * xv;
            acc[b][2 * m + 1] += a[u][b][2 * m + 1] * xu + a[u][b][2 * m] * xv;
          }
        }
    }
    for (; j < ns; ++j)
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        if (blk[b] < 0) continue;
        T a[VEC];
        vload_s<T, NT>(Ap + (int64_t)j * lc + b * 64 * VEC + lane * VEC, a);
        const T xu = xt[iu[b] + j];
        const T xv = iv[b] >= 0 ? xt[iv[b] + j] : T(0);
#pragma unroll
        for (int m = 0; m < VEC / 2; ++m) {
          acc[b][2 * m] += a[2 * m] * xu - a[2 * m + 1] * xv;
          acc[b][2 * m + 1] += a[2 * m + 1] * xu + a[2 * m] * xv;
        }
      }
    // block results into xs (xs is no longer read): real rows off..off+VEC-1, or complex
    // rows off/2 .. off/2+VEC/2-1 with re -> stage st0, im -> stage st0+1
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      if (blk[b] < 0) continue;
      if (iv[b] < 0) {
#pragma unroll
        for (int v = 0; v < VEC; ++v)
          if (off[b] + v < ns) xs[iu[b] + off[b] + v] = acc[b][v];
      } else {
#pragma unroll
        for (int m = 0; m < VEC / 2; ++m) {
          const int c = off[b] / 2 + m;
          if (c < ns) {
            xs[iu[b] + c] = acc[b][2 * m];
            xs[iv[b] + c] = acc[b][2 * m + 1];
          }
        }
      }
    }
  } else {
    for (int j = 0; j < ns; ++j) {
      T pr[kMaxStages], pi[kMaxStages];
#pragma unroll
      for (int q = 0; q < kMaxStages; ++q) pr[q] = pi[q] = T(0);
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        if (blk[b] < 0) continue;
        T a[VEC];
        vload<VT, T>(Ap + (int64_t)j * lc + b * 64 * VEC + lane * VEC, a);
        T sr = T(0), si = T(0);
        if (iv[b] < 0) {
#pragma unroll
          for (int v = 0; v < VEC; ++v)
            if (off[b] + v < ns) sr += a[v] * xt[iu[b] + off[b] + v];
        } else {
#pragma unroll
          for (int m = 0; m < VEC / 2; ++m) {
            const int c = off[b] / 2 + m;
            if (c < ns) {
              const T zr = xt[iu[b] + c], zi = xt[iv[b] + c];
              sr += a[2 * m] * zr + a[2 * m + 1] * zi;
              si += a[2 * m] * zi - a[2 * m + 1] * zr;
            }
          }
        }
#pragma unroll
        for (int q = 0; q < kMaxStages; ++q)
          if (blk[b] == q) {
            pr[q] += sr;
            pi[q] += si;
          }
      }
#pragma unroll
      for (int q = 0; q < kMaxStages; ++q) {
        if (q >= sb.nblk) break;
        T vr = pr[q], vi = pi[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          vr += __shfl_xor(vr, o, 64);
          vi += __shfl_xor(vi, o, 64);
        }
        if (lane == 0) {
          xs[sb.st0[q] * ns + j] = vr;
          if (sb.type[q] == 2) xs[(sb.st0[q] + 1) * ns + j] = vi;
        }
      }
    }
  }
  eig_out<T>(lane, n, ns, so, xs, sb, Y, transpose, D);
}

// Value of lane l (uniform l) of v, for every lane.
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// rot over the ring of the block's n_s rows, row i taking row i-1's value (row 0 takes
// row n_s-1's).  Rows are held RS per lane, row q at slot q / 64 of lane q % 64.  One
// slot: one cross-lane read from the fixed source lane src.  More slots: each slot
// shifts by one lane (lane 0 reading lane 63 of the same slot), then lane 0 of slot k
// takes the previous slot's lane 63 (uniform reads of the values before the shift),
// and lane 0 of slot 0 row n_s-1 (slot kl, lane ll).
template <typename T, int RS>
__device__ __forceinline__ void sym_rot(T* t, int lane, int src, int kl, int ll) {
  if constexpr (RS == 1) {
    t[0] = __shfl(t[0], src, 64);
  } else {
    T edge[RS];
#pragma unroll
    for (int k = 0; k < RS; ++k) edge[k] = k == 0 ? T(0) : lane_value(t[k - 1], 63);
    T last = T(0);
#pragma unroll
    for (int k = 0; k < RS; ++k)
      if (k == kl) last = lane_value(t[k], ll);
#pragma unroll
    for (int k = 0; k < RS; ++k) {
      const T r = __shfl(t[k], src, 64);
      t[k] = lane == 0 ? (k == 0 ? last : edge[k]) : r;
    }
  }
}

// Work of one stored word (16 bytes per row) of a symmetric block for the rows iv[k] of
// this lane, the word holding the diagonals s0, s0-1, ..., s0-G+1 (descending).  Forward
// entries Z(i, i+s) x_{i+s}, x read from the doubled copy xu (xu[i + s] =
// x_{(i+s) mod n_s}).  Transposed entries Z(i-s, i) x_{i-s}, 1 <= s <= nb, by a Horner
// scheme over the descending diagonals: t <- rot(t) + Z(i, i+s) x_i (sym_rot), so that
// after the diagonal s = 0 row i holds sum_s Z(i-s, i) x_{i-s}.  Real blocks use
// (ar, tr); pairs (ar, ai, tr, ti) with x = (xu, xv) and cs = -1 for the conjugate.
template <typename T, int RS>
__device__ __forceinline__ void sym_word(const T (*a)[Vec16<T>::n], int type, int s0, const int* iv, int nb,
                                         int lane, int src, int kl, int ll, const T* xu, const T* xv,
                                         const T* xir, const T* xii, T cs, T* ar, T* ai, T* tr, T* ti) {
  constexpr int VEC = Vec16<T>::n;
  if (type == 1) {
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      const int sd = s0 - q;
#pragma unroll
      for (int k = 0; k < RS; ++k) ar[k] += a[k][q] * xu[iv[k] + sd];
      sym_rot<T, RS>(tr, lane, src, kl, ll);
      if (sd >= 1 && sd <= nb)  // wave-uniform test
#pragma unroll
        for (int k = 0; k < RS; ++k) tr[k] += a[k][q] * xir[k];
    }
  } else {
#pragma unroll
    for (int q = 0; q < VEC / 2; ++q) {
      const int sd = s0 - q;
#pragma unroll
      for (int k = 0; k < RS; ++k) {
        const T dr = a[k][2 * q], di = cs * a[k][2 * q + 1];
        const T zr = xu[iv[k] + sd], zi = xv[iv[k] + sd];
        ar[k] += dr * zr - di * zi;
        ai[k] += dr * zi + di * zr;
      }
      sym_rot<T, RS>(tr, lane, src, kl, ll);
      sym_rot<T, RS>(ti, lane, src, kl, ll);
      if (sd >= 1 && sd <= nb)  // wave-uniform test
#pragma unroll
        for (int k = 0; k < RS; ++k) {
          const T dr = a[k][2 * q], di = cs * a[k][2 * q + 1];
          tr[k] += dr * xir[k] - di * xii[k];
          ti[k] += dr * xii[k] + di * xir[k];
        }
    }
  }
}

// Symmetric factored patch inverse.  For a symmetric spatial operator (Stokes: K
// symmetric and the divergence coupling B, B^T) every eigen-block I (x) M_v + dt T_k (x)
// S_v is symmetric (real eigenvalue) or complex symmetric (pair), and so is its inverse,
// which is therefore stored by its wrapped diagonals s = 0 .. n_s/2 (layout with
// sym_block_values): about half the values of the factored form.  One wavefront per
// patch; the lane owns rows lane + 64 k, k < RS, of every block (n_s <= 64 RS); each
// stored entry is read once from memory and used for both Z(i, i+s) and Z(i+s, i).
// Transposed apply: real blocks are unchanged, a pair's conjugate transpose is its
// conjugate.  Gather and eigenbasis transforms as in the factored form (xt doubled, 2n
// values).
//
// The blocks of a patch follow each other, so its words form one sequence, word w of
// row i at ((w n_s) + i) vec, read U words at a time; with PF the next U words are in
// flight while the current ones are used (the first U before the gather).
template <typename T, int U = 4, int NT = 1, int PF = 0, int RS = 1>
__device__ __forceinline__ void patch_apply_sym_one(
    int p, int lane, T* xs, T* xt, const irk::StageBasis<T>& sb, const int32_t* __restrict__ p_nloc,
    const int64_t* __restrict__ p_inv_off, const int64_t* __restrict__ p_slot_off,
    const int32_t* __restrict__ gidx, const T* __restrict__ inv, const T* __restrict__ res,
    const T* __restrict__ W, T* __restrict__ Y, int transpose, int D) {
  constexpr int VEC = Vec16<T>::n;
  const int n = p_nloc[p];
  const int ns = n / sb.r;
  const int64_t so = p_slot_off[p];
  // rows past n_s repeat row 0's loads and arithmetic; no row reads their results
  int iv[RS];
#pragma unroll
  for (int k = 0; k < RS; ++k) iv[k] = lane + 64 * k < ns ? lane + 64 * k : 0;
  // rot: one slot reads lane i-1 (lane n_s-1 for lane 0); more slots shift by one lane
  const int src = RS == 1 ? (iv[0] == 0 ? ns - 1 : iv[0] - 1) : ((lane + 63) & 63);
  const int kl = (ns - 1) / 64, ll = (ns - 1) % 64;  // slot and lane of row n_s-1
  const T* __restrict__ Dp = inv + p_inv_off[p];
  const int64_t step = (int64_t)ns * VEC;
  int NG = 0;
  for (int b = 0; b < sb.nblk; ++b) NG += irk::sym_words(sb.type[b], ns, VEC);
  T a[U][RS][VEC];
  if constexpr (PF) {
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (u < NG)
#pragma unroll
        for (int k = 0; k < RS; ++k) vload_s<T, NT>(Dp + u * step + (int64_t)iv[k] * VEC, a[u][k]);
  }
  eig_in<T, true>(lane, n, ns, so, xs, xt, sb, gidx, res, W, transpose);
  const int nb = ns - irk::sym_diags(ns);  // diagonals also used transposed: 1 .. nb
  const T cs = transpose ? T(-1) : T(1);
  // current block: type, words done / total, top diagonal, x, accumulators
  int b = 0, type = sb.type[0], ng = irk::sym_words(type, ns, VEC), wb = 0;
  int G = type == 1 ? VEC : VEC / 2;
  int top = ng * G - 1;
  const T* xu = xt + sb.st0[0] * 2 * ns;
  const T* xv = xu + 2 * ns;
  T xir[RS], xii[RS], ar[RS], ai[RS], tr[RS], ti[RS];
#pragma unroll
  for (int k = 0; k < RS; ++k) {
    xir[k] = xu[iv[k]];
    xii[k] = type == 2 ? xv[iv[k]] : T(0);
    ar[k] = ai[k] = tr[k] = ti[k] = T(0);
  }
  for (int w0 = 0; w0 < NG; w0 += U) {
    T nx[U][RS][VEC];
    if constexpr (PF) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (w0 + U + u < NG)
#pragma unroll
          for (int k = 0; k < RS; ++k) vload_s<T, NT>(Dp + (w0 + U + u) * step + (int64_t)iv[k] * VEC, nx[u][k]);
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (w0 + u < NG)
#pragma unroll
          for (int k = 0; k < RS; ++k) vload_s<T, NT>(Dp + (w0 + u) * step + (int64_t)iv[k] * VEC, a[u][k]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (w0 + u >= NG) break;
      sym_word<T, RS>(a[u], type, top - wb * G, iv, nb, lane, src, kl, ll, xu, xv, xir, xii, cs, ar, ai, tr, ti);
      if (++wb == ng) {  // block done: store its rows, move to the next block
#pragma unroll
        for (int k = 0; k < RS; ++k)
          if (lane + 64 * k < ns) {
            xs[sb.st0[b] * ns + iv[k]] = ar[k] + tr[k];
            if (type == 2) xs[(sb.st0[b] + 1) * ns + iv[k]] = ai[k] + ti[k];
          }
        if (++b < sb.nblk) {
          type = sb.type[b];
          ng = irk::sym_words(type, ns, VEC);
          wb = 0;
          G = type == 1 ? VEC : VEC / 2;
          top = ng * G - 1;
          xu = xt + sb.st0[b] * 2 * ns;
          xv = xu + 2 * ns;
#pragma unroll
          for (int k = 0; k < RS; ++k) {
            xir[k] = xu[iv[k]];
            xii[k] = type == 2 ? xv[iv[k]] : T(0);
            ar[k] = ai[k] = tr[k] = ti[k] = T(0);
          }
        }
      }
    }
    if constexpr (PF) {
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < RS; ++k)
#pragma unroll
          for (int v = 0; v < VEC; ++v) a[u][k][v] = nx[u][k][v];
    }
  }
  eig_out<T>(lane, n, ns, so, xs, sb, Y, transpose, D);
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

// Owner gather of one DOF from the sliced slot lists (entry k of DOF g of slice sl at
// off[sl] + 64 k + lane; padding entries point at a slot that always holds zero).
template <typename T>
__device__ __forceinline__ void gather_sell_one(int64_t g, int64_t sl, int lane, const int32_t* __restrict__ g_off,
                                                const int32_t* __restrict__ g_w, const int32_t* __restrict__ g_slot,
                                                const T* __restrict__ Y, const T* __restrict__ W, T omega, int mode,
                                                T* __restrict__ x, int64_t N) {
  const int w = g_w[sl];
  const int64_t e0 = g_off[sl] + lane;
  T s = T(0);
  int k = 0;
  for (; k + 4 <= w; k += 4) {
    int32_t q[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u] = g_slot[e0 + (int64_t)(k + u) * 64];
#pragma unroll
    for (int u = 0; u < 4; ++u) s += Y[q[u]];
  }
  for (; k < w; ++k) s += Y[g_slot[e0 + (int64_t)k * 64]];
  if (g >= N) return;
  T c = omega * s;
  if (mode < 2) c *= W[g];
  x[g] = (mode & 1) ? x[g] + c : c;
}

// Chebyshev step of the relaxation for one DOF: with s the sum of its slots,
// d = c1 d + c2 (W s) (W null: weights already applied to the patch inputs; d not read
// when first), then x = d (xzero) or x + d.
template <typename T>
__device__ __forceinline__ void gather_cheb_one(int64_t g, int64_t sl, int lane, const int32_t* __restrict__ g_off,
                                                const int32_t* __restrict__ g_w, const int32_t* __restrict__ g_slot,
                                                const T* __restrict__ Y, const T* __restrict__ W, T c1, T c2,
                                                int first, int xzero, T* __restrict__ d, T* __restrict__ x,
                                                int64_t N) {
  const int w = g_w[sl];
  const int64_t e0 = g_off[sl] + lane;
  T s = T(0);
  int k = 0;
  for (; k + 4 <= w; k += 4) {
    int32_t q[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u] = g_slot[e0 + (int64_t)(k + u) * 64];
#pragma unroll
    for (int u = 0; u < 4; ++u) s += Y[q[u]];
  }
  for (; k < w; ++k) s += Y[g_slot[e0 + (int64_t)k * 64]];
  if (g >= N) return;
  const T z = W ? W[g] * s : s;
  const T dn = first ? c2 * z : c1 * d[g] + c2 * z;
  d[g] = dn;
  x[g] = xzero ? dn : x[g] + dn;
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
  constexpr int UN = 4;  // entries whose gathers are in flight together
  if (row < nrow_u) {
    T acc[DR];
#pragma unroll
    for (int q = 0; q < DR; ++q) acc[q] = T(0);
    const int32_t p1 = u_ptr[row + 1];
    int32_t p = u_ptr[row];
    for (; p + UN <= p1; p += UN) {
      int32_t c[UN];
      T w[UN], xv[UN][DR];
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        c[u] = u_col[p + u];
        w[u] = u_val[p + u];
      }
#pragma unroll
      for (int u = 0; u < UN; ++u)
#pragma unroll
        for (int q = 0; q < DR; ++q) xv[u][q] = in[(int64_t)c[u] * DR + q];
#pragma unroll
      for (int u = 0; u < UN; ++u)
#pragma unroll
        for (int q = 0; q < DR; ++q) acc[q] += w[u] * xv[u][q];
    }
    for (; p < p1; ++p) {
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
    const int32_t p1 = p_ptr[v + 1];
    int32_t p = p_ptr[v];
    for (; p + UN <= p1; p += UN) {
      int32_t c[UN];
      T w[UN], xv[UN][R];
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        c[u] = p_col[p + u];
        w[u] = p_val[p + u];
      }
#pragma unroll
      for (int u = 0; u < UN; ++u)
#pragma unroll
        for (int q = 0; q < R; ++q) xv[u][q] = in[in_offV + (int64_t)c[u] * R + q];
#pragma unroll
      for (int u = 0; u < UN; ++u)
#pragma unroll
        for (int q = 0; q < R; ++q) acc[q] += w[u] * xv[u][q];
    }
    for (; p < p1; ++p) {
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
