// Particle kernels of liblpc: the fixed-point CIC deposit (Sec. 2.4 step 1, Sec. 4.2 "rounding down" to the cell),
// the CIC force gather fused with the COLA kick and drift (Sec. 2.4 step 4; Sec. 2.3 Eqs. 17-18), and the frame
// momentum removal / add-back (Sec. 2.3).
//
// Fixed point: per axis u = floor(x * (Nm 2^16 / L)) in FP64, reduced mod Nm 2^16; the cell is u >> 16 and the
// fraction f = u & 0xffff. The deposit adds prod_d (2^16 - f_d or f_d) to the 8 corners with 64-bit integer atomics,
// so every particle adds exactly 2^48 and the mesh does not depend on the order of the additions. The gather uses
// the same u, with weights f 2^-16 and 1 - f 2^-16 (exact in FP32), so it is the transpose of the deposit.
//
// The kernels are batched over the jobs (boxes) of a work table, with a capped grid that strides over the items;
// an item is kNT particles of one box.
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

__device__ __forceinline__ int find_job(const LPC_CONST int* __restrict__ offs, int njob, int w) {
  int lo = 0, hi = njob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (offs[mid] <= w)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

constexpr int kFillChunk = kNT * 16;  // words per fill item

__global__ __launch_bounds__(kNT) void k_fill(const FillJob* __restrict__ jobs, const int* __restrict__ offs, int njob,
                                              int total) {
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const int jb = __builtin_amdgcn_readfirstlane(find_job(to_const(offs), njob, w));
    const LPC_CONST FillJob& J = to_const(jobs)[jb];
    const int64_t base = static_cast<int64_t>(w - offs[jb]) * kFillChunk;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int64_t i = base + m * kNT + threadIdx.x;
      if (i < J.count) to_global(J.p)[i] = 0;
    }
  }
}

__global__ __launch_bounds__(kNT) void k_fill_i32(int* __restrict__ p, size_t count, int value) {
  const size_t stride = static_cast<size_t>(gridDim.x) * kNT;
  for (size_t i = static_cast<size_t>(blockIdx.x) * kNT + threadIdx.x; i < count; i += stride) p[i] = value;
}

template <class PJ>
__device__ __forceinline__ void deposit_one(const PJ& J, int64_t i, int* flags) {
  const int64_t n = J.n;
  const int nm = J.nm;
  const int64_t period = static_cast<int64_t>(nm) << kFracBits;
  uint32_t c[3], f[3];
  bool ok = true;
  LPC_GLOBAL const float* pos = to_global(J.pos);
#pragma unroll
  for (int d = 0; d < 3; ++d) ok &= fixed_coord(pos[d * n + i], J.scale, period, &c[d], &f[d]);
  if (!ok) {
    atomicOr(flags + kFlagNonfinite, 1);
    return;
  }
  const uint64_t wx[2] = {kOne - f[0], f[0]}, wy[2] = {kOne - f[1], f[1]}, wz[2] = {kOne - f[2], f[2]};
  const uint32_t xs[2] = {c[0], (c[0] + 1 == static_cast<uint32_t>(nm)) ? 0u : c[0] + 1};
  const uint32_t ys[2] = {c[1], (c[1] + 1 == static_cast<uint32_t>(nm)) ? 0u : c[1] + 1};
  const uint32_t zs[2] = {c[2], (c[2] + 1 == static_cast<uint32_t>(nm)) ? 0u : c[2] + 1};
  LPC_GLOBAL unsigned long long* C = to_global(reinterpret_cast<unsigned long long*>(J.dens));
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
          __hip_atomic_fetch_add(C + rowbase + zs[e], static_cast<unsigned long long>(w), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

__global__ __launch_bounds__(kNT) void k_deposit(const PartJob* __restrict__ jobs, const int* __restrict__ offs,
                                                 int njob, int total, int* __restrict__ flags) {
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const int jb = __builtin_amdgcn_readfirstlane(find_job(to_const(offs), njob, w));
    const LPC_CONST PartJob& J = to_const(jobs)[jb];
    const int64_t i = static_cast<int64_t>(w - offs[jb]) * kNT + threadIdx.x;
    if (i < J.n) deposit_one(J, i, flags);
  }
}

// Interpolate the AoS float3 mesh to one particle; false if the position is not usable.
__device__ __forceinline__ bool cic_gather(LPC_GLOBAL const float* __restrict__ F, int nm, double scale, float x, float y,
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
        LPC_GLOBAL const float* p = F + 3 * (rowbase + zs[e]);
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

__global__ __launch_bounds__(kNT) void k_gather_kick_drift(const PartJob* __restrict__ jobs,
                                                           const int* __restrict__ offs, int njob, int total,
                                                           KickDrift kd, int* __restrict__ flags) {
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const int jb = __builtin_amdgcn_readfirstlane(find_job(to_const(offs), njob, w));
    const LPC_CONST PartJob& J = to_const(jobs)[jb];
    const int64_t n = J.n;
    const int64_t i = static_cast<int64_t>(w - offs[jb]) * kNT + threadIdx.x;
    if (i >= n) continue;
    LPC_GLOBAL float* pos = to_global(J.pos);
    LPC_GLOBAL float* vel = to_global(J.vel);
    LPC_GLOBAL const float* psi1 = to_global(J.psi1);
    LPC_GLOBAL const float* psi2 = to_global(J.psi2);
    float x[3] = {pos[i], pos[n + i], pos[2 * n + i]};
    float g[3];
    if (!cic_gather(to_global(J.force), J.nm, J.scale, x[0], x[1], x[2], g)) {
      atomicOr(flags + kFlagNonfinite, 1);
      continue;
    }
    const float box = J.box;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      float acc = g[d];
      float p1 = 0.f, p2 = 0.f;
      if (kd.cola) {
        p1 = psi1[d * n + i];
        p2 = psi2[d * n + i];
        acc += kd.d1 * p1 + kd.d2m * p2;
      }
      const float v = vel[d * n + i] + kd.kick * acc;
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
}

__global__ __launch_bounds__(kNT) void k_gather(const PartJob* __restrict__ jobs, const int* __restrict__ offs,
                                                int njob, int total, int* __restrict__ flags) {
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const int jb = __builtin_amdgcn_readfirstlane(find_job(to_const(offs), njob, w));
    const LPC_CONST PartJob& J = to_const(jobs)[jb];
    const int64_t n = J.n;
    const int64_t i = static_cast<int64_t>(w - offs[jb]) * kNT + threadIdx.x;
    if (i >= n) continue;
    float g[3];
    LPC_GLOBAL const float* pos = to_global(J.pos);
    LPC_GLOBAL float* grad = to_global(J.grad);
    if (!cic_gather(to_global(J.force), J.nm, J.scale, pos[i], pos[n + i], pos[2 * n + i], g)) {
      atomicOr(flags + kFlagNonfinite, 1);
      g[0] = g[1] = g[2] = 0.f;
    }
    grad[i] = g[0];
    grad[n + i] = g[1];
    grad[2 * n + i] = g[2];
  }
}

// vel += f1 psi1 + f2 psi2 over the 3 n components (items of kNT values)
__global__ __launch_bounds__(kNT) void k_frame_velocity(const PartJob* __restrict__ jobs, const int* __restrict__ offs,
                                                        int njob, int total, float f1, float f2) {
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const int jb = __builtin_amdgcn_readfirstlane(find_job(to_const(offs), njob, w));
    const LPC_CONST PartJob& J = to_const(jobs)[jb];
    const int64_t i = static_cast<int64_t>(w - offs[jb]) * kNT + threadIdx.x;
    if (i < 3 * J.n) to_global(J.vel)[i] += f1 * to_global(J.psi1)[i] + f2 * to_global(J.psi2)[i];
  }
}

constexpr int kPartGridCap = 256 * 8 * 4;

unsigned grid_of(const WorkTable& wt, int cap) {
  return static_cast<unsigned>(wt.total < cap ? wt.total : cap);
}

}  // namespace

// items of a particle stage per job: ceil(n / kNT) (ceil(3n / kNT) for the frame velocity)
int fill_items(int64_t count) { return static_cast<int>((count + kFillChunk - 1) / kFillChunk); }

hipError_t fill_i32(int* p, size_t count, int value, hipStream_t s) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + kNT - 1) / kNT;
  if (blocks > 65536) blocks = 65536;
  k_fill_i32<<<static_cast<unsigned>(blocks), kNT, 0, s>>>(p, count, value);
  return hipGetLastError();
}

hipError_t launch_fill(const FillJob* jobs, WorkTable wt, hipStream_t s) {
  if (wt.total <= 0) return hipSuccess;
  k_fill<<<grid_of(wt, kPartGridCap), kNT, 0, s>>>(jobs, wt.offs, wt.njob, wt.total);
  return hipGetLastError();
}

hipError_t launch_deposit(const PartJob* jobs, WorkTable wt, int* flags, hipStream_t s) {
  if (wt.total <= 0) return hipSuccess;
  k_deposit<<<grid_of(wt, kPartGridCap), kNT, 0, s>>>(jobs, wt.offs, wt.njob, wt.total, flags);
  return hipGetLastError();
}

hipError_t launch_gather_kick_drift(const PartJob* jobs, WorkTable wt, KickDrift kd, int* flags, hipStream_t s) {
  if (wt.total <= 0) return hipSuccess;
  k_gather_kick_drift<<<grid_of(wt, kPartGridCap), kNT, 0, s>>>(jobs, wt.offs, wt.njob, wt.total, kd, flags);
  return hipGetLastError();
}

hipError_t launch_gather(const PartJob* jobs, WorkTable wt, int* flags, hipStream_t s) {
  if (wt.total <= 0) return hipSuccess;
  k_gather<<<grid_of(wt, kPartGridCap), kNT, 0, s>>>(jobs, wt.offs, wt.njob, wt.total, flags);
  return hipGetLastError();
}

hipError_t launch_frame(const PartJob* jobs, WorkTable wt, float f1, float f2, hipStream_t s) {
  if (wt.total <= 0) return hipSuccess;
  k_frame_velocity<<<grid_of(wt, kPartGridCap), kNT, 0, s>>>(jobs, wt.offs, wt.njob, wt.total, f1, f2);
  return hipGetLastError();
}

}  // namespace kern
}  // namespace lpc
