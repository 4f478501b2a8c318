// Vector-ALU issue ceiling of the part, measured: every lane runs independent
// FMA chains (FP32, then FP64) long enough that issue, not latency, bounds
// them.  Built with the same flags as the library (no packed FP32), so the
// FP32 figure is the ceiling the fit kernels can reach.  Prints one JSON line.
//
// Launch: 8192 workgroups of 256 lanes; each lane writes one value to a
// buffer of exactly that many elements (index blockIdx.x * 256 + threadIdx.x).
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

constexpr int kBlocks = 8192, kThreads = 256, kIters = 4096;

__device__ __forceinline__ float fma_of(float x, float a, float b) { return __builtin_fmaf(x, a, b); }
__device__ __forceinline__ double fma_of(double x, double a, double b) { return __builtin_fma(x, a, b); }

template <typename T, int NCH>
__global__ void __launch_bounds__(kThreads) fma_chains(T* out, int iters, T a, T b) {
  T x[NCH];
#pragma unroll
  for (int i = 0; i < NCH; ++i) x[i] = (T)threadIdx.x * (T)1e-3 + (T)i;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < NCH; ++i) x[i] = fma_of(x[i], a, b);
  }
  T s = 0;
#pragma unroll
  for (int i = 0; i < NCH; ++i) s += x[i];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

bool check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    std::fprintf(stderr, "peak_probe: %s: %s\n", what, hipGetErrorString(e));
    return false;
  }
  return true;
}

template <typename T, int NCH>
bool run(T* buf, double* ms_out) {
  hipEvent_t e0, e1;
  if (!check(hipEventCreate(&e0), "event") || !check(hipEventCreate(&e1), "event")) return false;
  fma_chains<T, NCH><<<kBlocks, kThreads>>>(buf, kIters, (T)0.999, (T)1e-3);  // warm-up
  if (!check(hipGetLastError(), "launch") || !check(hipDeviceSynchronize(), "sync")) return false;
  constexpr int reps = 5;
  hipEventRecord(e0, nullptr);
  for (int r = 0; r < reps; ++r) fma_chains<T, NCH><<<kBlocks, kThreads>>>(buf, kIters, (T)0.999, (T)1e-3);
  hipEventRecord(e1, nullptr);
  if (!check(hipEventSynchronize(e1), "sync")) return false;
  float ms = 0.f;
  hipEventElapsedTime(&ms, e0, e1);
  *ms_out = ms / reps;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return true;
}

}  // namespace

int main() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (!check(hipGetDeviceProperties(&prop, dev), "properties")) return 1;
  double* buf = nullptr;  // large enough for either element type
  if (!check(hipMalloc(&buf, sizeof(double) * kBlocks * kThreads), "malloc")) return 1;
  const double lanes = (double)kBlocks * kThreads;
  const double simds = 4.0 * prop.multiProcessorCount;
  const double clock_hz = 2.4e9;  // the part's peak engine clock
  double ms32 = 0, ms64 = 0;
  if (!run<float, 16>(reinterpret_cast<float*>(buf), &ms32) || !run<double, 8>(buf, &ms64)) return 1;
  const double fl32 = lanes * kIters * 16 * 2, fl64 = lanes * kIters * 8 * 2;
  const double ipc32 = lanes / 64 * kIters * 16 / (ms32 * 1e-3 * clock_hz * simds);
  const double ipc64 = lanes / 64 * kIters * 8 / (ms64 * 1e-3 * clock_hz * simds);
  std::printf("{\"device\": \"%s\", \"cus\": %d, \"fp32_fma_tflops\": %.2f, \"fp32_wave_instr_per_cycle_per_simd\": %.4f, "
              "\"fp64_fma_tflops\": %.2f, \"fp64_wave_instr_per_cycle_per_simd\": %.4f, \"ms_fp32\": %.4f, \"ms_fp64\": %.4f}\n",
              prop.gcnArchName, prop.multiProcessorCount, fl32 / (ms32 * 1e-3) / 1e12, ipc32,
              fl64 / (ms64 * 1e-3) / 1e12, ipc64, ms32, ms64);
  hipFree(buf);
  return 0;
}
