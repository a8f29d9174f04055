// HIP kernels of the generic Kronecker stage operator J = I_r (x) M + dt A (x) S
// (Sec. 3.1) used by the linearised MHD solver (Sec. 3.3), for gfx950.
//
//  kron_residual  r = F - J x over a sliced copy of the spatial operator: M and S share
//                 one pattern, each entry is read once and applied to the r stage
//                 values of its column (contiguous in the internal layout), and the
//                 r x r stage mixing dt A is applied once per row.
//  kron_csr       y (+)= P x for a CSR transfer on every stage (Sec. 4.1).
//  stage_to_*     ABI layout (stage blocks) <-> internal layout (stage innermost).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mhd_internal.h"
#include "device_ops.h"

namespace irk {
namespace k {
namespace {

constexpr int kBlock = 256;

inline unsigned blocks_for(int64_t n, int block = kBlock) {
  return (unsigned)std::max<int64_t>(1, (n + block - 1) / block);
}

// one lane per row; slices of 64 rows stored column-major, so the k-th entries of a
// wavefront's rows are one coalesced access (padding entries: column 0, values 0).  The
// entries are taken four at a time, all their loads issued before the first product, so
// that a lane has four gathers of x in flight; the products are summed in entry order.
template <int R>
__global__ __launch_bounds__(kBlock) void k_kron_residual(int64_t nrows, int64_t nsl, const int32_t* __restrict__ sl_off,
                                                          const int32_t* __restrict__ sl_w,
                                                          const int32_t* __restrict__ sl_col,
                                                          const double* __restrict__ sl_m,
                                                          const double* __restrict__ sl_s, dev::Coef<double> dtA,
                                                          const double* __restrict__ F, const double* __restrict__ x,
                                                          double* __restrict__ y) {
  const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t sl = row >> 6;
  if (sl >= nsl) return;
  const int lane = (int)(row & 63);
  const int w = sl_w[sl];
  const int64_t e0 = (int64_t)sl_off[sl] + lane;
  double am[R], as[R];
#pragma unroll
  for (int s = 0; s < R; ++s) am[s] = as[s] = 0.0;
  constexpr int U = 4;
  int k = 0;
  for (; k + U <= w; k += U) {
    int64_t c[U];
    double m[U], sv[U], xv[U][R];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + (int64_t)(k + u) * 64;
      c[u] = sl_col[e];
      m[u] = sl_m[e];
      sv[u] = sl_s[e];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int s = 0; s < R; ++s) xv[u][s] = x[c[u] * R + s];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int s = 0; s < R; ++s) {
        am[s] += m[u] * xv[u][s];
        as[s] += sv[u] * xv[u][s];
      }
  }
  for (; k < w; ++k) {
    const int64_t e = e0 + (int64_t)k * 64;
    const int64_t c = sl_col[e];
    const double m = sl_m[e], sv = sl_s[e];
    const double* xc = x + c * R;
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const double xv = xc[s];
      am[s] += m * xv;
      as[s] += sv * xv;
    }
  }
  if (row >= nrows) return;
#pragma unroll
  for (int s = 0; s < R; ++s) {
    double v = am[s];
#pragma unroll
    for (int t = 0; t < R; ++t) v += dtA.v[s * R + t] * as[t];
    const int64_t o = row * R + s;
    y[o] = F ? F[o] - v : v;
  }
}

__global__ __launch_bounds__(kBlock) void k_kron_csr(int64_t nrows, const int32_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ col, const double* __restrict__ val,
                                                     int R, const double* __restrict__ x, double* __restrict__ y,
                                                     int accumulate) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= nrows * R) return;
  const int64_t row = e / R;
  const int s = (int)(e - row * R);
  double acc = 0.0;
  for (int32_t p = ptr[row]; p < ptr[row + 1]; ++p) acc += val[p] * x[(int64_t)col[p] * R + s];
  y[e] = accumulate ? y[e] + acc : acc;
}

__global__ __launch_bounds__(kBlock) void k_stage_permute(int64_t ns, int R, const double* __restrict__ in,
                                                          double* __restrict__ out, int to_internal) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= ns * R) return;
  const int64_t q = e / R;
  const int s = (int)(e - q * R);
  if (to_internal) out[e] = in[s * ns + q];
  else out[s * ns + q] = in[e];
}

}  // namespace

hipError_t kron_residual(int64_t nrows, int64_t nsl, const int32_t* sl_off, const int32_t* sl_w,
                         const int32_t* sl_col, const double* sl_m, const double* sl_s, int R, const double* A,
                         double dt, const double* F, const double* x, double* y, hipStream_t s) {
  dev::Coef<double> c{};
  for (int i = 0; i < R * R; ++i) c.v[i] = dt * A[i];
  const dim3 g(blocks_for(nsl * 64)), b(kBlock);
  switch (R) {
    case 1: k_kron_residual<1><<<g, b, 0, s>>>(nrows, nsl, sl_off, sl_w, sl_col, sl_m, sl_s, c, F, x, y); break;
    case 2: k_kron_residual<2><<<g, b, 0, s>>>(nrows, nsl, sl_off, sl_w, sl_col, sl_m, sl_s, c, F, x, y); break;
    case 3: k_kron_residual<3><<<g, b, 0, s>>>(nrows, nsl, sl_off, sl_w, sl_col, sl_m, sl_s, c, F, x, y); break;
    case 4: k_kron_residual<4><<<g, b, 0, s>>>(nrows, nsl, sl_off, sl_w, sl_col, sl_m, sl_s, c, F, x, y); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t kron_csr(int64_t nrows, const int32_t* ptr, const int32_t* col, const double* val, int R,
                    const double* x, double* y, int accumulate, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  k_kron_csr<<<dim3(blocks_for(nrows * R)), dim3(kBlock), 0, s>>>(nrows, ptr, col, val, R, x, y, accumulate);
  return hipGetLastError();
}

hipError_t stage_to_internal(int64_t ns, int R, const double* abi, double* x, hipStream_t s) {
  k_stage_permute<<<dim3(blocks_for(ns * R)), dim3(kBlock), 0, s>>>(ns, R, abi, x, 1);
  return hipGetLastError();
}

hipError_t stage_to_abi(int64_t ns, int R, const double* x, double* abi, hipStream_t s) {
  k_stage_permute<<<dim3(blocks_for(ns * R)), dim3(kBlock), 0, s>>>(ns, R, x, abi, 0);
  return hipGetLastError();
}

}  // namespace k
}  // namespace irk
