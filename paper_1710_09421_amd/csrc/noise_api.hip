// The library's counter-based generator for given counters (ek_philox):
// callers reproduce or check the thermal noise with it.
#include <string>

#include "ek_context.h"
#include "philox.h"

using namespace ek;

namespace {

__global__ __launch_bounds__(256) void k_philox(const uint32_t* __restrict__ ctr, int n,
                                                uint32_t k0, uint32_t k1, uint32_t* __restrict__ words,
                                                double* __restrict__ normals) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Philox4 w = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1);
  double z[4];
  box_muller4<double>(w, z);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    words[4 * i + c] = w.v[c];
    normals[4 * i + c] = z[c];
  }
}

}  // namespace

extern "C" ek_status ek_philox(const uint32_t* counters, int32_t n, uint64_t seed, uint32_t* words,
                               double* normals, void* hip_stream) {
  if (n < 0 || n > (1 << 24) || (n > 0 && !counters)) {
    set_thread_error("ek_philox: n must be in [0, 2^24] and counters not NULL");
    return EK_EINVAL;
  }
  if (n == 0) return EK_OK;
  const hipStream_t s = (hipStream_t)hip_stream;
  const size_t nw = (size_t)4 * n;
  char* buf = nullptr;
  if (hipMalloc((void**)&buf, nw * (4 + 4 + 8)) != hipSuccess) {
    set_thread_error("ek_philox: device buffer");
    return EK_ENOMEM;
  }
  uint32_t* dctr = (uint32_t*)buf;
  uint32_t* dw = dctr + nw;
  double* dz = (double*)(dw + nw);
  hipError_t e = hipMemcpyAsync(dctr, counters, nw * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_philox, dim3((n + 255) / 256), dim3(256), 0, s, dctr, n,
                       uint32_t(seed & 0xFFFFFFFFull), uint32_t(seed >> 32), dw, dz);
    e = hipGetLastError();
  }
  if (e == hipSuccess && words) e = hipMemcpyAsync(words, dw, nw * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && normals) e = hipMemcpyAsync(normals, dz, nw * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (e != hipSuccess) {
    set_thread_error(std::string("ek_philox: ") + hipGetErrorString(e));
    return EK_EHIP;
  }
  return EK_OK;
}
