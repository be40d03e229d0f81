// Matrix-core throughput probe: the rate at which this device sustains the MFMA
// instructions the interval counters use, so that a counter's speed can be read
// against a measured peak as well as the published one.
//
// 4 waves per workgroup, one workgroup per CU (launch bounds), each wave issuing
// MFMAs into 16 independent accumulators (no dependency stalls) with operands held in
// registers.  The result depends on the clock the device holds under MFMA load.
#include <type_traits>
#include <vector>

#include "common.h"

namespace cs {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

template <bool FP4>
__global__ __launch_bounds__(256, 1) void k_peak(int iters, const int* __restrict__ in,
                                                 int* __restrict__ out) {
  using Acc = typename std::conditional<FP4, v16f, v16i>::type;
  Acc acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[i][e] = 0;
  int x = in[threadIdx.x & 7];
  for (int it = 0; it < iters; ++it) {
    if constexpr (FP4) {
      const v8i a = (v8i){x & 0x22222222, 0x02020202, 0x20202020, 0x22222222, 0, 0, 0, 0};
#pragma unroll
      for (int i = 0; i < 16; ++i)
        acc[i] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, a, acc[i], 4, 4, 0, 127, 0,
                                                                 127);
    } else {
      const v4i a = (v4i){x & 0x01010101, 1, 0x0101, 0x01000001};
#pragma unroll
      for (int i = 0; i < 16; ++i)
        acc[i] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, a, acc[i], 0, 0, 0);
    }
    x ^= it;
  }
  int s = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += (int)acc[i][threadIdx.x & 15];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace
}  // namespace cs

using namespace cs;

extern "C" cs_status cs_measure_mfma_peak(int counter, double* tops, void* stream) {
  if (!tops || (counter != CS_COUNT_MFMA && counter != CS_COUNT_MFMA_FP4)) return CS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int blocks = device_cu_count(), iters = 20000;  // ~5 ms per launch
  int *din = nullptr, *dout = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  cs_status s = CS_OK;
  const std::vector<int> seed(16, 0x01010101);
  if (hipMalloc(&din, 64) != hipSuccess || hipMalloc(&dout, sizeof(int) * 256 * blocks) != hipSuccess ||
      hipMemcpy(din, seed.data(), 64, hipMemcpyHostToDevice) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    s = CS_ERR_HIP;
  } else {
    float best = 1e30f;
    for (int rep = 0; rep < 3 && s == CS_OK; ++rep) {
      (void)hipEventRecord(e0, st);
      if (counter == CS_COUNT_MFMA_FP4)
        hipLaunchKernelGGL(k_peak<true>, dim3(blocks), dim3(256), 0, st, iters, din, dout);
      else
        hipLaunchKernelGGL(k_peak<false>, dim3(blocks), dim3(256), 0, st, iters, din, dout);
      (void)hipEventRecord(e1, st);
      if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) s = CS_ERR_HIP;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0 && ms < best) best = ms;  // first launch warms clocks and code
    }
    const double k = counter == CS_COUNT_MFMA_FP4 ? 64.0 : 32.0;
    *tops = 2.0 * 32 * 32 * k * 16.0 * iters * 4.0 * blocks / (best * 1e-3) / 1e12;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (din) (void)hipFree(din);
  if (dout) (void)hipFree(dout);
  return s;
}
