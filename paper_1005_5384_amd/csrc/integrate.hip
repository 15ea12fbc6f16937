// Time integration around the force call: kick-drift-kick leapfrog on
// device-resident FP32 positions and velocities, and the FP64 kinetic energy
// and momentum of the state (energy-conservation runs, Sec. 3).
#include <hip/hip_runtime.h>

#include "octgrav_internal.h"

namespace octgrav {
namespace {

constexpr int kT = 256;
constexpr int kKinBlocks = 512;

// v += h a (n x 3 FP32)
__global__ void kick_kernel(float* __restrict__ vel, const float* __restrict__ acc, int64_t n3,
                            float h) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i < n3) vel[i] = fmaf(h, acc[i], vel[i]);
}

// x += dt v (n x 3 FP32)
__global__ void drift_kernel(float* __restrict__ pos, const float* __restrict__ vel, int64_t n3,
                             float dt) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i < n3) pos[i] = fmaf(dt, vel[i], pos[i]);
}

// Per-block FP64 sums of (1/2 m v^2, m vx, m vy, m vz), then one block adds
// the block sums in block order (deterministic).
__global__ __launch_bounds__(kT) void kin_partial_kernel(const float* __restrict__ mass,
                                                         const float* __restrict__ vel, int64_t n,
                                                         double* __restrict__ part) {
  __shared__ double sh[4][kT];
  double s[4] = {0, 0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    const double m = mass[i], vx = vel[3 * i], vy = vel[3 * i + 1], vz = vel[3 * i + 2];
    s[0] += 0.5 * m * (vx * vx + vy * vy + vz * vz);
    s[1] += m * vx;
    s[2] += m * vy;
    s[3] += m * vz;
  }
  for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[4 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void kin_final_kernel(const double* __restrict__ part, int nb, double* __restrict__ out) {
  if (threadIdx.x < 4) {
    double s = 0;
    for (int b = 0; b < nb; ++b) s += part[4 * b + threadIdx.x];
    out[threadIdx.x] = s;
  }
}

}  // namespace

int launch_kick(float* vel, const float* acc, int64_t n, float h, void* stream) {
  if (n <= 0) return 0;
  kick_kernel<<<(3 * n + kT - 1) / kT, kT, 0, (hipStream_t)stream>>>(vel, acc, 3 * n, h);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_drift(float* pos, const float* vel, int64_t n, float dt, void* stream) {
  if (n <= 0) return 0;
  drift_kernel<<<(3 * n + kT - 1) / kT, kT, 0, (hipStream_t)stream>>>(pos, vel, 3 * n, dt);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int64_t kinetic_scratch_entries() { return 4 * kKinBlocks; }

int launch_kinetic(const float* mass, const float* vel, int64_t n, double* part, double* out4,
                   void* stream) {
  hipStream_t s = (hipStream_t)stream;
  kin_partial_kernel<<<kKinBlocks, kT, 0, s>>>(mass, vel, n, part);
  kin_final_kernel<<<1, 64, 0, s>>>(part, kKinBlocks, out4);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace octgrav
