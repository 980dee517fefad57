// Matrix-core peak of the device, measured: every wave issues independent chains of
// the 16x16x4 MFMA the LU's trailing update uses (v_mfma_f64_16x16x4f64 for complex128,
// v_mfma_f32_16x16x4f32 for complex64), so the rate is bounded by the matrix cores'
// issue rate alone.  The datasheet peaks (78.6 / 157.3 TFLOP/s dense on MI355X) are the
// roofline denominators; this is their check on the device at hand.
#include <hip/hip_runtime.h>

#include "../../include/nep.h"
#include "common.h"

namespace nep {

constexpr int PEAK_CHAINS = 8;

template <typename T>
__global__ __launch_bounds__(256) void mfma_peak_kernel(int iters, T seed, T* __restrict__ out) {
  acc4<T> c[PEAK_CHAINS];
#pragma unroll
  for (int k = 0; k < PEAK_CHAINS; ++k) c[k] = acc_zero<T>();
  const T a = seed * (T)(threadIdx.x & 15), b = seed * (T)(threadIdx.x >> 4);
  // 8 rounds per loop pass, fully unrolled: the compiler moves the accumulators between
  // register files once per pass, which 64 instructions of 16 passes each hide
  for (int i = 0; i < iters; i += 8) {
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int k = 0; k < PEAK_CHAINS; ++k) c[k] = mfma16(a, b, c[k]);
  }
  T s = T(0);
#pragma unroll
  for (int k = 0; k < PEAK_CHAINS; ++k) s += c[k][0] + c[k][1] + c[k][2] + c[k][3];
  // one value per workgroup is stored so that the chains are not optimised away
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

}  // namespace nep

using namespace nep;

extern "C" nep_status nep_mfma_peak(int precision, int iters, double* tflops) {
  if (!tflops || iters < 1 || (precision != NEP_FP64 && precision != NEP_FP32_REFINE)) return NEP_ERR_ARG;
  constexpr int BLOCKS = 1024, THREADS = 256;
  void* out = nullptr;
  if (hipMalloc(&out, sizeof(double) * BLOCKS) != hipSuccess) {
    (void)hipGetLastError();
    return NEP_ERR_NOMEM;
  }
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  auto launch = [&](int it) {
    if (precision == NEP_FP64)
      mfma_peak_kernel<double><<<BLOCKS, THREADS>>>(it, 1e-3, static_cast<double*>(out));
    else
      mfma_peak_kernel<float><<<BLOCKS, THREADS>>>(it, 1e-3f, static_cast<float*>(out));
  };
  launch(iters);                                  // warm-up: code object load, clocks up
  hipEventRecord(e0, 0);
  launch(iters);
  hipEventRecord(e1, 0);
  nep_status st = NEP_OK;
  if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) st = NEP_ERR_HIP;
  float ms = 0.f;
  if (st == NEP_OK) hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(out);
  if (st != NEP_OK) return st;
  const double waves = (double)BLOCKS * THREADS / 64.0;
  const double flops = waves * (double)((iters + 7) / 8 * 8) * PEAK_CHAINS * (16.0 * 16.0 * 4.0 * 2.0);
  *tflops = ms > 0 ? flops / (ms * 1e-3) / 1e12 : 0.0;
  return NEP_OK;
}
