// Fixed device scratch for the allocation-free entry point helm_data_residual_static
// (include/helm.h): the block partial sums of the data term, its total and an
// index-error flag live in one file-scope device array instead of memory the
// library allocates.  Each GPU holds its own copy; host code reaches it only
// through the address hipGetSymbolAddress returns for the current device.
#include <algorithm>
#include <mutex>

#include "dev_common.h"
#include "kernels.h"

namespace {

// layout: [0, kStaticPartials) block partials, then the total, then the error flag
constexpr int kStaticPartials = 4096;
constexpr int kTotal = kStaticPartials;
constexpr int kFlag = kStaticPartials + 1;
static __device__ __align__(256) double scratch[kStaticPartials + 32];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

__global__ void k_static_clear(double* s) {
  if (threadIdx.x == 0) s[kFlag] = 0.0;
}

// s[kFlag] = 1 if any receiver index lies outside [0, N) (plain stores of the same value)
__global__ void k_static_check(int M, long long N, const int* idx, double* s) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < M; i += gridDim.x * blockDim.x) {
    const int v = idx[i];
    if (v < 0 || (long long)v >= N) s[kFlag] = 1.0;
  }
}

// total = partials summed in block order (FP64), the order the host sum of the
// allocating entry point uses
__global__ void k_static_total(int nbk, double* s) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double t = 0.0;
  for (int b = 0; b < nbk; ++b) t += s[b];
  s[kTotal] = t;
}

}  // namespace

int static_scratch_partials() { return kStaticPartials; }

hipError_t static_scratch_init() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[dev]) return hipSuccess;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[dev] = (double*)p;
  return hipSuccess;
}

double* static_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_scratch[dev];
}

void launch_static_check(hipStream_t s, int M, long long N, const int* idx, double* scr) {
  hipLaunchKernelGGL(k_static_clear, dim3(1), dim3(64), 0, s, scr);
  const unsigned g = (unsigned)std::min<long long>(((long long)M + 255) / 256, 1024);
  hipLaunchKernelGGL(k_static_check, dim3(g), dim3(256), 0, s, M, N, idx, scr);
}

void launch_static_total(hipStream_t s, int nbk, double* scr) {
  hipLaunchKernelGGL(k_static_total, dim3(1), dim3(64), 0, s, nbk, scr);
}

const double* static_flag(const double* scr) { return scr + kFlag; }
const double* static_total(const double* scr) { return scr + kTotal; }
