// Hydrogen photoionisation chemistry of the R-type expansion test (sec. 3.1.1),
// one step after a forward sweep: the step limit (a min-reduction over cells)
// and the photon-conserving update with implicit recombination.
//
// Per cell (u = 1 - y ionised fraction, V in cm^3, P = photons/s absorbed):
//   limit  = n_H V y / (P - alpha_B n_H^2 u^2 V)   where the denominator is > 0
//   update = the root in [0, 1] of  a u'^2 + u' - b = 0,  a = alpha_B n_H dt,
//            b = u + P dt / (n_H V), taken as 2b / (1 + sqrt(1 + 4ab)) (no
//            cancellation for any a, b >= 0)
// Both are elementwise and HBM-bound (20 bytes per cell); FP64 throughout.
#include <mutex>

#include "internal.h"

namespace sweep {

namespace {

__device__ __forceinline__ double cell_volume_cgs(const float* vol, int64_t c, double l3) {
  return (double)vol[c] * l3;
}

}  // namespace

// Positive doubles order like their bit patterns read as unsigned integers, so
// the minimum is an integer atomicMin on the bits.
__global__ __launch_bounds__(256) void k_ion_limit(IonArgs a, unsigned long long* out) {
  __shared__ double part[4];
  double m = __builtin_huge_val();
  const double nH = a.n_H;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.n; c += (int64_t)gridDim.x * blockDim.x) {
    const double V = cell_volume_cgs(a.vol, c, a.l3);
    const double y = a.neutral[c];
    const double u = 1.0 - y;
    const double net = a.photon_rate * (double)a.absorbed[c] - a.alpha_B * nH * nH * u * u * V;
    if (net > 0.0) m = fmin(m, nH * V * y / net);
  }
  for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) m = fmin(m, part[i]);
    atomicMin(out, (unsigned long long)__double_as_longlong(m));
  }
}

__global__ void k_ion_init(unsigned long long* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0)
    *out = (unsigned long long)__double_as_longlong(__builtin_huge_val());
}

__global__ __launch_bounds__(256) void k_ion_update(IonArgs a, double dt) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n) return;
  const double V = cell_volume_cgs(a.vol, c, a.l3);
  const double y = a.neutral[c];
  const double A = a.alpha_B * a.n_H * dt;
  const double b = (1.0 - y) + a.photon_rate * (double)a.absorbed[c] * dt / (a.n_H * V);
  const double un = fmin(2.0 * b / (1.0 + sqrt(1.0 + 4.0 * A * b)), 1.0);
  const double yn = 1.0 - un;
  a.neutral[c] = yn;
  a.kappa[c] = (float)(a.n_H * yn * a.sigma_H * a.length_unit);
}

// The absorption coefficient of the neutral hydrogen in length units:
// kappa = n_H y sigma_H length_unit.
__global__ __launch_bounds__(256) void k_ion_kappa(IonArgs a) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n) return;
  a.kappa[c] = (float)(a.n_H * a.neutral[c] * a.sigma_H * a.length_unit);
}

hipError_t launch_ion_kappa(const IonArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ion_kappa, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Scratch of sweep_ion_step_noalloc: the step limit's minimum over the cells,
// as the bits of a positive double (8 bytes, the whole of it).  Each GPU holds
// its own copy until the process ends; every call on that GPU shares it (calls
// that overlap on one GPU race for it).  Host code never passes this name to a
// kernel or a copy: it uses the device address ion_scratch() looks up.
static __device__ __align__(256) unsigned long long scratch[1];

constexpr int kMaxDevices = 64;

hipError_t ion_scratch(unsigned long long** out) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(mu);
  if (addr[dev] == nullptr) {  // once per device, with that device current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *out = static_cast<unsigned long long*>(addr[dev]);
  return hipSuccess;
}

hipError_t launch_ion_limit(const IonArgs& a, unsigned long long* out, hipStream_t s) {
  hipLaunchKernelGGL(k_ion_init, dim3(1), dim3(64), 0, s, out);
  if (a.n <= 0) return hipGetLastError();
  const int64_t blocks = std::min<int64_t>(2048, (a.n + 255) / 256);
  hipLaunchKernelGGL(k_ion_limit, dim3((unsigned)blocks), dim3(256), 0, s, a, out);
  return hipGetLastError();
}

hipError_t launch_ion_update(const IonArgs& a, double dt, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ion_update, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a, dt);
  return hipGetLastError();
}

}  // namespace sweep
