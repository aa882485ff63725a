// Particle kernels of liblpc: the fixed-point CIC deposit (Sec. 2.4 step 1, Sec. 4.2 "rounding down" to the cell),
// the CIC force gather fused with the COLA kick and drift (Sec. 2.4 step 4; Sec. 2.3 Eqs. 17-18), and the frame
// momentum removal / add-back (Sec. 2.3).
//
// Fixed point: per axis u = floor(x * (Nm 2^16 / L)) in FP64, reduced mod Nm 2^16; the cell is u >> 16 and the
// fraction f = u & 0xffff. The deposit adds prod_d (2^16 - f_d or f_d) to the 8 corners with 64-bit integer atomics,
// so every particle adds exactly 2^48 and the mesh does not depend on the order of the additions. The gather uses
// the same u, with weights f 2^-16 and 1 - f 2^-16 (exact in FP32), so it is the transpose of the deposit.
#include <hip/hip_runtime.h>

#include <cmath>

#include "lpc_kernels.h"

namespace lpc {
namespace kern {

namespace {

constexpr uint32_t kOne = 1u << kFracBits;
constexpr uint32_t kMask = kOne - 1u;

// Fixed-point coordinate of one axis; false if x is not finite or too far outside the box to convert.
__device__ __forceinline__ bool fixed_coord(float x, double scale, int64_t period, uint32_t* cell, uint32_t* frac) {
  const double xs = static_cast<double>(x) * scale;
  if (!(fabs(xs) < 4.0e18)) return false;  // also catches NaN
  int64_t u = static_cast<int64_t>(floor(xs)) % period;
  if (u < 0) u += period;
  *cell = static_cast<uint32_t>(u >> kFracBits);
  *frac = static_cast<uint32_t>(u) & kMask;
  return true;
}

__global__ __launch_bounds__(kNT) void k_fill_u64(uint64_t* __restrict__ p, size_t count) {
  const size_t stride = static_cast<size_t>(gridDim.x) * kNT;
  for (size_t i = static_cast<size_t>(blockIdx.x) * kNT + threadIdx.x; i < count; i += stride) p[i] = 0;
}

__global__ __launch_bounds__(kNT) void k_fill_i32(int* __restrict__ p, size_t count, int value) {
  const size_t stride = static_cast<size_t>(gridDim.x) * kNT;
  for (size_t i = static_cast<size_t>(blockIdx.x) * kNT + threadIdx.x; i < count; i += stride) p[i] = value;
}

__global__ __launch_bounds__(kNT) void k_deposit(const float* __restrict__ pos, int64_t n, int nm, double scale,
                                                 uint64_t* __restrict__ C, int* __restrict__ flags) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (i >= n) return;
  const int64_t period = static_cast<int64_t>(nm) << kFracBits;
  uint32_t c[3], f[3];
  bool ok = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) ok &= fixed_coord(pos[d * n + i], scale, period, &c[d], &f[d]);
  if (!ok) {
    atomicOr(flags + kFlagNonfinite, 1);
    return;
  }
  uint64_t wx[2] = {kOne - f[0], f[0]}, wy[2] = {kOne - f[1], f[1]}, wz[2] = {kOne - f[2], f[2]};
  const uint32_t xs[2] = {c[0], (c[0] + 1 == static_cast<uint32_t>(nm)) ? 0u : c[0] + 1};
  const uint32_t ys[2] = {c[1], (c[1] + 1 == static_cast<uint32_t>(nm)) ? 0u : c[1] + 1};
  const uint32_t zs[2] = {c[2], (c[2] + 1 == static_cast<uint32_t>(nm)) ? 0u : c[2] + 1};
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const uint64_t wab = wx[a] * wy[b];
      const size_t rowbase = (static_cast<size_t>(xs[a]) * nm + ys[b]) * nm;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const uint64_t w = wab * wz[e];
        if (w != 0)
          atomicAdd(reinterpret_cast<unsigned long long*>(C + rowbase + zs[e]), static_cast<unsigned long long>(w));
      }
    }
  }
}

// Interpolate the AoS float3 mesh to one particle; false if the position is not usable.
__device__ __forceinline__ bool cic_gather(const float* __restrict__ F, int nm, double scale, float x, float y,
                                           float z, float g[3]) {
  const int64_t period = static_cast<int64_t>(nm) << kFracBits;
  uint32_t c[3], f[3];
  bool ok = fixed_coord(x, scale, period, &c[0], &f[0]);
  ok &= fixed_coord(y, scale, period, &c[1], &f[1]);
  ok &= fixed_coord(z, scale, period, &c[2], &f[2]);
  if (!ok) return false;
  const float inv = 1.0f / static_cast<float>(kOne);
  const float wx[2] = {static_cast<float>(kOne - f[0]) * inv, static_cast<float>(f[0]) * inv};
  const float wy[2] = {static_cast<float>(kOne - f[1]) * inv, static_cast<float>(f[1]) * inv};
  const float wz[2] = {static_cast<float>(kOne - f[2]) * inv, static_cast<float>(f[2]) * inv};
  const uint32_t xs[2] = {c[0], (c[0] + 1 == static_cast<uint32_t>(nm)) ? 0u : c[0] + 1};
  const uint32_t ys[2] = {c[1], (c[1] + 1 == static_cast<uint32_t>(nm)) ? 0u : c[1] + 1};
  const uint32_t zs[2] = {c[2], (c[2] + 1 == static_cast<uint32_t>(nm)) ? 0u : c[2] + 1};
  float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const float wab = wx[a] * wy[b];
      const size_t rowbase = (static_cast<size_t>(xs[a]) * nm + ys[b]) * nm;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const float w = wab * wz[e];
        const float* p = F + 3 * (rowbase + zs[e]);
        gx += w * p[0];
        gy += w * p[1];
        gz += w * p[2];
      }
    }
  }
  g[0] = gx;
  g[1] = gy;
  g[2] = gz;
  return true;
}

__global__ __launch_bounds__(kNT) void k_gather_kick_drift(float* __restrict__ pos, float* __restrict__ vel,
                                                           const float* __restrict__ psi1,
                                                           const float* __restrict__ psi2, int64_t n,
                                                           const float* __restrict__ F, int nm, double scale,
                                                           float box, KickDrift kd, int* __restrict__ flags) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (i >= n) return;
  float x[3] = {pos[i], pos[n + i], pos[2 * n + i]};
  float g[3];
  if (!cic_gather(F, nm, scale, x[0], x[1], x[2], g)) {
    atomicOr(flags + kFlagNonfinite, 1);
    return;
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float acc = g[d];
    float p1 = 0.f, p2 = 0.f;
    if (kd.cola) {
      p1 = psi1[d * n + i];
      p2 = psi2[d * n + i];
      acc += kd.d1 * p1 + kd.d2m * p2;
    }
    float v = vel[d * n + i] + kd.kick * acc;
    vel[d * n + i] = v;
    if (kd.do_drift) {
      float xn = x[d] + kd.drift * v;
      if (kd.cola) xn += kd.dd1 * p1 + kd.dd2 * p2;
      if (xn >= box) xn -= box;
      if (xn < 0.f) xn += box;
      pos[d * n + i] = xn;
    }
  }
}

__global__ __launch_bounds__(kNT) void k_gather(const float* __restrict__ pos, int64_t n, const float* __restrict__ F,
                                                int nm, double scale, float* __restrict__ grad,
                                                int* __restrict__ flags) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (i >= n) return;
  float g[3];
  if (!cic_gather(F, nm, scale, pos[i], pos[n + i], pos[2 * n + i], g)) {
    atomicOr(flags + kFlagNonfinite, 1);
    g[0] = g[1] = g[2] = 0.f;
  }
  grad[i] = g[0];
  grad[n + i] = g[1];
  grad[2 * n + i] = g[2];
}

__global__ __launch_bounds__(kNT) void k_frame_velocity(float* __restrict__ vel, const float* __restrict__ psi1,
                                                        const float* __restrict__ psi2, int64_t count, float f1,
                                                        float f2) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (i < count) vel[i] += f1 * psi1[i] + f2 * psi2[i];
}

unsigned grid_for(int64_t n) { return static_cast<unsigned>((n + kNT - 1) / kNT); }

}  // namespace

hipError_t fill_u64(uint64_t* p, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + kNT - 1) / kNT;
  if (blocks > 65536) blocks = 65536;
  k_fill_u64<<<static_cast<unsigned>(blocks), kNT, 0, s>>>(p, count);
  return hipGetLastError();
}

hipError_t fill_i32(int* p, size_t count, int value, hipStream_t s) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + kNT - 1) / kNT;
  if (blocks > 65536) blocks = 65536;
  k_fill_i32<<<static_cast<unsigned>(blocks), kNT, 0, s>>>(p, count, value);
  return hipGetLastError();
}

hipError_t deposit(const float* pos, int64_t n, int nm, double scale, uint64_t* C, int* flags, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_deposit<<<grid_for(n), kNT, 0, s>>>(pos, n, nm, scale, C, flags);
  return hipGetLastError();
}

hipError_t gather_kick_drift(float* pos, float* vel, const float* psi1, const float* psi2, int64_t n,
                             const float* force, int nm, double scale, float box, KickDrift kd, int* flags,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_gather_kick_drift<<<grid_for(n), kNT, 0, s>>>(pos, vel, psi1, psi2, n, force, nm, scale, box, kd, flags);
  return hipGetLastError();
}

hipError_t gather(const float* pos, int64_t n, const float* force, int nm, double scale, float* grad, int* flags,
                  hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_gather<<<grid_for(n), kNT, 0, s>>>(pos, n, force, nm, scale, grad, flags);
  return hipGetLastError();
}

hipError_t frame_velocity(float* vel, const float* psi1, const float* psi2, int64_t n, float f1, float f2,
                          hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_frame_velocity<<<grid_for(3 * n), kNT, 0, s>>>(vel, psi1, psi2, 3 * n, f1, f2);
  return hipGetLastError();
}

}  // namespace kern
}  // namespace lpc
