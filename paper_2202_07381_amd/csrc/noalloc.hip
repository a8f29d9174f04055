// noalloc.hip -- the Ritz estimate of a level's relaxation operator (irk_mg_ritz) in a
// form that allocates no device memory, for callers that cannot allocate (code under
// HIP graph capture, serving loops, harnesses that forbid hipMalloc).
//
// Its Arnoldi basis, Hessenberg matrix and reduction partial sums live in `scratch`, a
// file-scope device array of kScratchBytes.  In host code the name `scratch` is only a
// host-side stand-in for the symbol; the device address of each GPU's copy is looked
// up once per device with hipGetSymbolAddress (on the first call made with that device
// current) and only that address is handed to kernels.
#include <hip/hip_runtime.h>

#include <complex>
#include <mutex>
#include <string>

#include "../../include/irk_mg.h"
#include "irk_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per GPU, held until exit
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device
irk_status scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return irk::fail_with(IRK_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return irk::fail_with(IRK_EINVAL, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return irk::fail_with(IRK_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return IRK_OK;
}

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

// scratch bytes the estimate needs: basis, Hessenberg matrix, partial sums
size_t ritz_scratch_bytes(const irk_mg* hc, int level, int steps) {
  irk_mg* h = const_cast<irk_mg*>(hc);
  if (!h || steps < 1 || steps > 64) return 0;
  if (level < 0) level = h->nlevels - 1;
  if (level >= h->nlevels) return 0;
  const size_t es = h->precision == 0 ? sizeof(double) : sizeof(float);
  return round256((size_t)(steps + 1) * (size_t)h->dev[level].N * es) +
         round256((size_t)(steps + 1) * (steps + 1) * sizeof(double)) + round256(irk::ritz_partials_bytes());
}

}  // namespace

extern "C" {

irk_status irk_mg_ritz_noalloc(irk_mg* h, int level, int steps, const double* v0, double* H, double* ritz_re,
                               double* ritz_im, int* nritz, void* stream) {
  irk_status st = irk::ritz_check(h, level, steps, v0, ritz_re, ritz_im);
  if (st != IRK_OK) return st;
  const size_t es = h->precision == 0 ? sizeof(double) : sizeof(float);
  const size_t bV = round256((size_t)(steps + 1) * (size_t)h->dev[level].N * es);
  const size_t bH = round256((size_t)(steps + 1) * (steps + 1) * sizeof(double));
  const size_t need = ritz_scratch_bytes(h, level, steps);
  if (need > kScratchBytes)
    return irk::fail_with(IRK_EINVAL, "irk_mg_ritz_noalloc: " + std::to_string(steps) + " steps on level " +
                                          std::to_string(level) + " need " + std::to_string(need) +
                                          " bytes of scratch, more than its 67108864 (64 MiB); take fewer "
                                          "steps or a coarser level");
  void* base = nullptr;
  st = scratch_address(&base);
  if (st != IRK_OK) return st;
  char* p = static_cast<char*>(base);
  double Hh[65 * 64];                        // host copy of the Hessenberg matrix
  std::complex<double> work[64 * 64 + 3 * 64];  // eigenvalue iteration
  int iwork[64];
  st = irk::ritz_into(h, level, steps, v0, p, reinterpret_cast<double*>(p + bV),
                      reinterpret_cast<double*>(p + bV + bH), Hh, static_cast<hipStream_t>(stream));
  if (st != IRK_OK) return st;
  return irk::ritz_finish(steps, Hh, H, ritz_re, ritz_im, nritz, work, iwork);
}

}  // extern "C"
