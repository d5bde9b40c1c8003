// Allocation-free trace misfit: dgrtm_residual_noalloc computes what dgrtm_residual computes, the
// FP64 sum over all samples of (a - b)^2, with its partial sums in a static device array instead
// of a shot workspace, for callers that cannot allocate device memory.
//
// The sum is taken in a fixed order: chunk c of kChunk consecutive values is reduced by work-group
// c (strided per lane, then a tree in LDS) into scratch[c], and one work-group then reduces the
// chunk sums in the same way.  The result is therefore the same bit for bit on every call with the
// same inputs, whatever the device load.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/dgrtm.h"
#include "setup.hpp"

namespace {

constexpr int kThreads = 256;
constexpr int64_t kChunk = 16384;                 // values per partial sum
constexpr int64_t kMaxChunks = 65536;             // partial sums the static array holds
constexpr int64_t kMaxValues = kChunk * kMaxChunks;  // 2^30 values per call
constexpr int kMaxDevices = 64;

}  // namespace

// One FP64 partial sum per chunk (512 KiB per device, held until the process ends).  Host code
// never passes this name to a kernel: it is only a host-side stand-in for the device array, whose
// address on each device comes from hipGetSymbolAddress (scratch_ptr below).
static __device__ __align__(256) double scratch[kMaxChunks];

namespace {

std::once_flag g_once[kMaxDevices];
double *g_ptr[kMaxDevices];
hipError_t g_status[kMaxDevices];

// Device address of `scratch` on device dev, resolved once per device with dev current.
hipError_t scratch_ptr(int dev, double **out) {
  std::call_once(g_once[dev], [dev] {
    int prev = 0;
    g_status[dev] = hipGetDevice(&prev);
    if (g_status[dev] != hipSuccess) return;
    if (prev != dev && (g_status[dev] = hipSetDevice(dev)) != hipSuccess) return;
    void *p = nullptr;
    g_status[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_ptr[dev] = static_cast<double *>(p);
    if (prev != dev) {
      hipError_t e = hipSetDevice(prev);
      if (g_status[dev] == hipSuccess) g_status[dev] = e;
    }
  });
  *out = g_ptr[dev];
  return g_status[dev];
}

__device__ double block_sum(double s, double *red) {
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

// work-group c: sum of (a - b)^2 over values [c kChunk, min(n, (c + 1) kChunk))
__global__ __launch_bounds__(kThreads) void misfit_chunk_kernel(const float *a, const float *b, int64_t n,
                                                                double *part) {
  __shared__ double red[kThreads];
  const int64_t i0 = (int64_t)blockIdx.x * kChunk;
  const int64_t i1 = i0 + kChunk < n ? i0 + kChunk : n;
  double s = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kThreads) {
    const double d = (double)a[i] - (double)b[i];
    s += d * d;
  }
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// one work-group: the sum of the n_chunks partial sums into *out (0 when n_chunks = 0)
__global__ __launch_bounds__(kThreads) void misfit_total_kernel(const double *part, int64_t n_chunks, double *out) {
  __shared__ double red[kThreads];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n_chunks; i += kThreads) s += part[i];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) *out = t;
}

}  // namespace

extern "C" dgrtm_status dgrtm_residual_noalloc(const float *a, const float *b, int64_t n, double *out,
                                               void *hip_stream) {
  using dgrtm::report_error;
  if (!out || n < 0 || (n > 0 && (!a || !b)))
    return report_error(DGRTM_ERR_ARG, "dgrtm_residual_noalloc: bad argument");
  if (n > kMaxValues)
    return report_error(DGRTM_ERR_ARG, "dgrtm_residual_noalloc: n = " + std::to_string(n) +
                                           " exceeds the maximum of " + std::to_string(kMaxValues) +
                                           " values (the static scratch holds " + std::to_string(kMaxChunks) +
                                           " partial sums of " + std::to_string(kChunk) + " values)");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int dev = 0;
  hipError_t e = st ? hipStreamGetDevice(st, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) return report_error(DGRTM_ERR_HIP, std::string("dgrtm_residual_noalloc: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return report_error(DGRTM_ERR_ARG, "dgrtm_residual_noalloc: device index out of range");
  double *part = nullptr;
  if ((e = scratch_ptr(dev, &part)) != hipSuccess || !part)
    return report_error(DGRTM_ERR_HIP, std::string("dgrtm_residual_noalloc: scratch address: ") +
                                           hipGetErrorString(e != hipSuccess ? e : hipErrorInvalidSymbol));
  const int64_t n_chunks = (n + kChunk - 1) / kChunk;
  if (n_chunks > 0)
    hipLaunchKernelGGL(misfit_chunk_kernel, dim3((unsigned)n_chunks), dim3(kThreads), 0, st, a, b, n, part);
  hipLaunchKernelGGL(misfit_total_kernel, dim3(1), dim3(kThreads), 0, st, part, n_chunks, out);
  if ((e = hipGetLastError()) != hipSuccess)
    return report_error(DGRTM_ERR_HIP, std::string("dgrtm_residual_noalloc: ") + hipGetErrorString(e));
  return DGRTM_OK;
}
