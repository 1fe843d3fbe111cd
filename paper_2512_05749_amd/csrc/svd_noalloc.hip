// The r x r Rayleigh-Ritz SVD (block one-sided Jacobi, the kernels of
// wssr_dbg_small_svd) as an entry point that allocates nothing: its working
// arrays live in one file-scope device array, `scratch`, of fixed size, which
// each GPU holds until the process ends.
//
// Host code never passes `scratch` itself to a kernel or a copy: on the host
// that name is only a stand-in.  The device address comes from
// hipGetSymbolAddress, taken once per device with that device current, and is
// kept per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"
#include "wssr.h"

using namespace wssr;

namespace {

constexpr int kNoallocRMax = 512;                // largest r
constexpr int64_t kRp = kNoallocRMax;            // r rounded up to 64, at most
// regions of the scratch array, in doubles (each a multiple of 32 doubles, so
// every region stays 256-byte aligned)
constexpr int64_t kMat = kRp * kRp;              // Ct, Bc, Pc, Ps: one r_p x r_p matrix each
constexpr int64_t kScal = 1024;                  // column sums of squares: r_p + 1
constexpr int64_t kSig = kRp;                    // singular values
constexpr int64_t kCos = kRp * kRp / 64;         // per-workgroup cosines
constexpr int64_t kSync = 32;                    // grid-barrier words (4 unsigned)
constexpr int64_t kStat = 32;                    // DevStatus
static_assert(sizeof(DevStatus) <= kStat * sizeof(double), "status region too small");
constexpr int64_t kScratchDoubles = 4 * kMat + kScal + kSig + kCos + kSync + kStat;

constexpr int kMaxDevices = 64;

}  // namespace

// About 8.4 MB per device.
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

const void* jacobi_kernel(int rp) {
  switch (rp / 64) {
    case 1: return (const void*)k_jacobi_coop<1>;
    case 2: return (const void*)k_jacobi_coop<2>;
    case 3: return (const void*)k_jacobi_coop<3>;
    case 4: return (const void*)k_jacobi_coop<4>;
    case 5: return (const void*)k_jacobi_coop<5>;
    case 6: return (const void*)k_jacobi_coop<6>;
    case 7: return (const void*)k_jacobi_coop<7>;
    default: return (const void*)k_jacobi_coop<8>;
  }
}

// Set-up, once per device with that device current: the device address of
// the scratch array and the dynamic-LDS limits of the sweep kernels.
double* scratch_on(int dev) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[dev]) return g_ptr[dev];
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return nullptr;
  }
  for (int k = 64; k <= kRp; k += 64)
    if (hipFuncSetAttribute(jacobi_kernel(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)jacobi_lds(k)) !=
        hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  g_ptr[dev] = static_cast<double*>(p);
  return g_ptr[dev];
}

}  // namespace

extern "C" wssr_status wssr_small_svd_noalloc(const double* C, int32_t r, double* s, double* P, int32_t* status,
                                              void* stream_) {
  if (!C || !s || !P) return WSSR_ERR_INVALID_ARG;
  if (r < 1 || r > kNoallocRMax) return WSSR_ERR_INVALID_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return WSSR_ERR_NO_DEVICE;
  }
  double* base = scratch_on(dev);
  if (!base) return WSSR_ERR_HIP;
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  int rp = (r + 63) / 64 * 64;
  double* Ct = base;
  double* Bc = Ct + kMat;
  double* Pc = Bc + kMat;
  double* Ps = Pc + kMat;
  double* scal = Ps + kMat;
  double* sig = scal + kScal;
  double* cosb = sig + kSig;
  unsigned* sy = reinterpret_cast<unsigned*>(cosb + kCos);
  DevStatus* st = reinterpret_cast<DevStatus*>(cosb + kCos + kSync);

  // every region the kernels read before writing is set here: the status
  // word, and (in k_jacobi_prep) the barrier words and the padded copies
  hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, stream, st);
  hipLaunchKernelGGL(k_transpose_pad, dim3((unsigned)(((int64_t)rp * rp + 255) / 256)), dim3(256), 0, stream, C, r,
                     rp, Ct);
  hipLaunchKernelGGL(k_jacobi_prep, dim3(rp / 4), dim3(256), 0, stream, (const double*)Ct, rp, r, Bc, Pc, scal, sy,
                     st);
  double tol = 1e-8;
  const double* scal_c = scal;
  int sweeps = 30, inner = 1;
  void* args[] = {&Bc, &Pc, &rp, &tol, &scal_c, &cosb, &sy, &st, &sweeps, &inner};
  hipError_t e = hipLaunchCooperativeKernel(jacobi_kernel(rp), dim3(rp / 32), dim3(256), args,
                                            (unsigned)jacobi_lds(rp), stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_raise, dim3(1), dim3(1), 0, stream, st, (int)WSSR_ERR_HIP);
  }
  hipLaunchKernelGGL(k_jacobi_final, dim3(1), dim3(1024), 0, stream, (const double*)Bc, (const double*)Pc, rp, r, sig,
                     Ps, st);
  (void)hipMemcpyAsync(s, sig, sizeof(double) * r, hipMemcpyDeviceToDevice, stream);
  (void)hipMemcpy2DAsync(P, sizeof(double) * r, Ps, sizeof(double) * rp, sizeof(double) * r, r,
                         hipMemcpyDeviceToDevice, stream);
  if (status) hipLaunchKernelGGL(k_status_save, dim3(1), dim3(1), 0, stream, (const DevStatus*)st, status);
  if (hipGetLastError() != hipSuccess) return WSSR_ERR_HIP;
  return e == hipSuccess ? WSSR_OK : WSSR_ERR_HIP;
}
