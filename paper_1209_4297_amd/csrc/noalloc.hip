// Device memory of the allocation-free 1D integration (ridc_integrate_noalloc): a fixed array in
// the library's code object, one copy per GPU, held until the process ends.  Holds the level
// rings, the quadrature weights and the PCR stage tables of one integration at a time.
#include <mutex>

#include "ridc_internal.h"

namespace ridc {

static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

__global__ void k_noalloc_tables(const NoAllocTables t, double* __restrict__ w,
                                 double* __restrict__ gamma, int32_t* __restrict__ shift) {
  for (int i = threadIdx.x; i < t.nw; i += blockDim.x) w[i] = t.w[i];
  for (int i = threadIdx.x; i < t.stages; i += blockDim.x) {
    gamma[i] = t.gamma[i];
    shift[i] = t.shift[i];
  }
}

}  // namespace

int noalloc_scratch(void** ptr) {
  int dev = 0;
  RIDC_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(RIDC_E_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    // the array's name is a host-side stand-in: only this device address may reach the GPU
    void* p = nullptr;
    RIDC_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(RIDC_E_HIP, "no device address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return RIDC_OK;
}

hipError_t launch_noalloc_tables(const NoAllocTables& t, void* base, hipStream_t stream) {
  char* b = static_cast<char*>(base);
  hipLaunchKernelGGL(k_noalloc_tables, dim3(1), dim3(64), 0, stream, t,
                     reinterpret_cast<double*>(b + kNoAllocWeightsOffset),
                     reinterpret_cast<double*>(b + kNoAllocGammaOffset),
                     reinterpret_cast<int32_t*>(b + kNoAllocShiftOffset));
  return hipGetLastError();
}

}  // namespace ridc
