// Issue rate of single (non-packed) wave64 FP32 and INT32 VALU instructions
// on this GPU: every lane runs 8 independent chains of one instruction kind,
// 8 waves per SIMD, so neither dependencies nor occupancy limit the rate.
// Prints one JSON object: per kind, wave64 instructions per compute unit per
// cycle of the nominal clock, and for FMA the FP32 rate (2 FLOP per lane).
// This is the ceiling of the force kernels' arithmetic, which is built
// without packed FP32 instructions.
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

template <int KIND>
__global__ __launch_bounds__(256) void chains_kernel(float* out, int iters, float a, float b) {
  float x[8];
  int ix[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    x[k] = threadIdx.x * 1e-3f + k;
    ix[k] = threadIdx.x + k;
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if constexpr (KIND == 0) x[k] = fmaf(x[k], a, b);
      if constexpr (KIND == 1) x[k] = x[k] * a;
      if constexpr (KIND == 2) x[k] = x[k] + a;
      if constexpr (KIND == 3) x[k] = __builtin_amdgcn_rsqf(x[k]);
      if constexpr (KIND == 4) ix[k] = ix[k] + (int)b;
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k] + (float)ix[k];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int KIND>
void launch(float* out, int blocks, int iters) {
  chains_kernel<KIND><<<blocks, 256>>>(out, iters, 0.999f, 1e-3f);
}

}  // namespace

int main() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    std::fprintf(stderr, "no HIP device\n");
    return 1;
  }
  const int blocks = cus * 8, iters = 20000, reps = 5;  // 8 blocks of 4 waves per CU
  const double nominal_hz = 2.4e9;
  float* out = nullptr;
  if (hipMalloc(&out, (size_t)blocks * 256 * 4) != hipSuccess) return 1;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
  const char* names[] = {"fma_f32", "mul_f32", "add_f32", "rsq_f32", "add_u32"};
  void (*fns[])(float*, int, int) = {launch<0>, launch<1>, launch<2>, launch<3>, launch<4>};
  std::printf("{\"cus\": %d, \"nominal_ghz\": %.1f, \"rates\": {", cus, nominal_hz * 1e-9);
  double fma_rate = 0.0;
  for (int k = 0; k < 5; ++k) {
    fns[k](out, blocks, iters);  // warm-up
    if (hipDeviceSynchronize() != hipSuccess) return 1;
    hipEventRecord(e0);
    for (int r = 0; r < reps; ++r) fns[k](out, blocks, iters);
    hipEventRecord(e1);
    if (hipEventSynchronize(e1) != hipSuccess) return 1;
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    const double wave_instr = (double)reps * blocks * 4 * iters * 8;
    const double per_cu_cycle = wave_instr / (ms * 1e-3) / cus / nominal_hz;
    if (k == 0) fma_rate = wave_instr / (ms * 1e-3);
    std::printf("%s\"%s\": %.4f", k ? ", " : "", names[k], per_cu_cycle);
  }
  // one wave64 FMA = 64 lanes x 2 FLOP
  std::printf("}, \"fma_f32_tflops\": %.2f}\n", fma_rate * 128.0 * 1e-12);
  hipFree(out);
  return 0;
}
