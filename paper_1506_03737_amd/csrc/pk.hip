// Clustering statistics of a periodic box, from the half spectrum delta_hat of the CIC density contrast:
//  * the binned power spectrum (the cubic-box form of the FKP estimator used in Sec. 7.1 of Howlett, Manera &
//    Percival 2015): P = V |delta_hat|^2 / (Nm^6 W^2) per mode with one CIC window W = prod sinc^2 removed, averaged
//    in linear |k| bins. Per-bin sums are FP64 and the mode counts exact integers;
//  * the pieces of the FFT shell estimator of the reduced bispectrum (Sec. 7.2): shell-filtered spectra (delta_hat / W
//    or the shell indicator) for an inverse transform, block sums of the product of three real fields, and block
//    sums of the shell power. Every block writes its own FP64 partial sum, so the totals (summed on the host in
//    block order) do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <cmath>

#include "lpc_kernels.h"

namespace lpc {
namespace kern {

namespace {

constexpr int kModesPerThread = 16;

__global__ __launch_bounds__(kNT) void k_pk_bin(const float2* __restrict__ spec, int nm, int pitch, double kf,
                                                double dk, int n_bins, double pscale, double* __restrict__ sums,
                                                unsigned long long* __restrict__ counts) {
  extern __shared__ double lds[];
  double* sk = lds;
  double* sp = lds + n_bins;
  unsigned long long* sc = reinterpret_cast<unsigned long long*>(lds + 2 * n_bins);
  float* win = reinterpret_cast<float*>(sc + n_bins);
  for (int b = threadIdx.x; b < n_bins; b += kNT) {
    sk[b] = 0.0;
    sp[b] = 0.0;
    sc[b] = 0ull;
  }
  for (int m = threadIdx.x; m < nm; m += kNT) {
    const int mm = min(m, nm - m);
    double w = 1.0;
    if (mm != 0) {
      const double x = static_cast<double>(mm) / nm;
      w = sinpi(x) / (M_PI * x);
      w = w * w;
    }
    win[m] = static_cast<float>(w);
  }
  __syncthreads();
  const int nh = nm / 2 + 1, half = nm / 2;
  const int64_t count = static_cast<int64_t>(nm) * nm * nh;
  const int64_t first = static_cast<int64_t>(blockIdx.x) * kNT * kModesPerThread;
  for (int t = 0; t < kModesPerThread; ++t) {
    const int64_t e = first + static_cast<int64_t>(t) * kNT + threadIdx.x;
    if (e >= count) break;
    const int kz = static_cast<int>(e % nh);
    const int64_t r = e / nh;
    const int ky = static_cast<int>(r % nm), kx = static_cast<int>(r / nm);
    const int nx = kx <= half ? kx : kx - nm, ny = ky <= half ? ky : ky - nm;
    const int64_t n2 = static_cast<int64_t>(nx) * nx + static_cast<int64_t>(ny) * ny + static_cast<int64_t>(kz) * kz;
    if (n2 == 0) continue;
    const double k = kf * sqrt(static_cast<double>(n2));
    const int b = static_cast<int>(floor(k / dk));
    if (b >= n_bins) continue;
    const float2 v = spec[r * pitch + kz];
    const double W = static_cast<double>(win[kx]) * win[ky] * win[kz];
    const double P = pscale * (static_cast<double>(v.x) * v.x + static_cast<double>(v.y) * v.y) / (W * W);
    const int mult = (kz > 0 && kz < half) ? 2 : 1;
    atomicAdd(sk + b, mult * k);
    atomicAdd(sp + b, mult * P);
    atomicAdd(sc + b, static_cast<unsigned long long>(mult));
  }
  __syncthreads();
  for (int b = threadIdx.x; b < n_bins; b += kNT) {
    if (sc[b] != 0ull) {
      atomicAdd(sums + 2 * b, sk[b]);
      atomicAdd(sums + 2 * b + 1, sp[b]);
      atomicAdd(counts + b, sc[b]);
    }
  }
}

// CIC window sinc^2(pi m / nm) of index m (either sign), in FP64.
__device__ __forceinline__ double cic_window(int m, int nm) {
  const int mm = min(m, nm - m);
  if (mm == 0) return 1.0;
  const double x = static_cast<double>(mm) / nm;
  const double w = sinpi(x) / (M_PI * x);
  return w * w;
}

// |k| of half-spectrum element (kx, ky, kz) and whether it lies in [klo, khi): the same FP64 operations as the
// oracle's kf sqrt(nx^2 + ny^2 + nz^2), so both take the same modes.
__device__ __forceinline__ bool in_shell(int kx, int ky, int kz, int nm, double kf, double klo, double khi) {
  const int half = nm / 2;
  const int nx = kx <= half ? kx : kx - nm, ny = ky <= half ? ky : ky - nm;
  const int64_t n2 = static_cast<int64_t>(nx) * nx + static_cast<int64_t>(ny) * ny + static_cast<int64_t>(kz) * kz;
  const double k = kf * sqrt(static_cast<double>(n2));
  return k >= klo && k < khi;
}

// out[kx][ky][kz] = delta_hat / W (indicator = 0) or 1 (indicator = 1) inside the shell, else 0; every element of
// the pitch, padding included. One thread per element.
__global__ __launch_bounds__(kNT) void k_shell_fill(const float2* __restrict__ spec, float2* __restrict__ out, int nm,
                                                    int pitch, double kf, double klo, double khi, int indicator) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  const int64_t count = static_cast<int64_t>(nm) * nm * pitch;
  if (e >= count) return;
  const int kz = static_cast<int>(e % pitch);
  const int64_t r = e / pitch;
  const int ky = static_cast<int>(r % nm), kx = static_cast<int>(r / nm);
  float2 v = make_float2(0.f, 0.f);
  if (kz <= nm / 2 && in_shell(kx, ky, kz, nm, kf, klo, khi)) {
    if (indicator) {
      v.x = 1.f;
    } else {
      const float2 d = spec[e];
      const double W = cic_window(kx, nm) * cic_window(ky, nm) * cic_window(kz, nm);
      v.x = static_cast<float>(static_cast<double>(d.x) / W);
      v.y = static_cast<float>(static_cast<double>(d.y) / W);
    }
  }
  out[e] = v;
}

constexpr int kSumBlocks = 256;  // blocks (and FP64 partial sums) of the reductions below

// Block reduction of one FP64 value per thread into part[blockIdx.x].
__device__ __forceinline__ void block_sum(double v, double* __restrict__ part) {
  __shared__ double sh[kNT];
  __syncthreads();  // sh may still be read by a previous reduction
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = kNT / 2; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// part[b] = sum over block b's cells of a b c (FP32 values, FP64 products and sums).
__global__ __launch_bounds__(kNT) void k_triple_sum(const float* __restrict__ a, const float* __restrict__ b,
                                                    const float* __restrict__ c, int64_t M, double* __restrict__ part) {
  double acc = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x; i < M; i += static_cast<int64_t>(kSumBlocks) * kNT)
    acc += static_cast<double>(a[i]) * b[i] * c[i];
  block_sum(acc, part);
}

// Per-block sums over the shell's modes of mult |delta_hat|^2 / W^2 (part_p) and of mult (part_n, exact in FP64),
// with mult = 2 for 0 < kz < Nm / 2 (the mode and its conjugate) and 1 on the kz = 0 and Nyquist planes.
__global__ __launch_bounds__(kNT) void k_shell_power(const float2* __restrict__ spec, int nm, int pitch, double kf,
                                                     double klo, double khi, double* __restrict__ part_p,
                                                     double* __restrict__ part_n) {
  const int nh = nm / 2 + 1, half = nm / 2;
  const int64_t count = static_cast<int64_t>(nm) * nm * nh;
  double p = 0.0, cnt = 0.0;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x; e < count;
       e += static_cast<int64_t>(kSumBlocks) * kNT) {
    const int kz = static_cast<int>(e % nh);
    const int64_t r = e / nh;
    const int ky = static_cast<int>(r % nm), kx = static_cast<int>(r / nm);
    if (!in_shell(kx, ky, kz, nm, kf, klo, khi)) continue;
    const float2 d = spec[r * pitch + kz];
    const double W = cic_window(kx, nm) * cic_window(ky, nm) * cic_window(kz, nm);
    const double mult = (kz > 0 && kz < half) ? 2.0 : 1.0;
    p += mult * (static_cast<double>(d.x) * d.x + static_cast<double>(d.y) * d.y) / (W * W);
    cnt += mult;
  }
  block_sum(p, part_p);
  block_sum(cnt, part_n);
}

}  // namespace

hipError_t shell_fill(const float2* spec, float2* out, int nm, int pitch, double box, double klo, double khi,
                      bool indicator, hipStream_t s) {
  const int64_t count = static_cast<int64_t>(nm) * nm * pitch;
  k_shell_fill<<<static_cast<unsigned>((count + kNT - 1) / kNT), kNT, 0, s>>>(spec, out, nm, pitch, 2.0 * M_PI / box,
                                                                              klo, khi, indicator ? 1 : 0);
  return hipGetLastError();
}

hipError_t triple_sum(const float* a, const float* b, const float* c, int64_t M, double* part, hipStream_t s) {
  k_triple_sum<<<kSumBlocks, kNT, 0, s>>>(a, b, c, M, part);
  return hipGetLastError();
}

hipError_t shell_power(const float2* spec, int nm, int pitch, double box, double klo, double khi, double* part_p,
                       double* part_n, hipStream_t s) {
  k_shell_power<<<kSumBlocks, kNT, 0, s>>>(spec, nm, pitch, 2.0 * M_PI / box, klo, khi, part_p, part_n);
  return hipGetLastError();
}

int sum_blocks() { return kSumBlocks; }

hipError_t pk_bin(const float2* spec, int nm, int pitch, double box, double k_max, int n_bins, double pscale,
                  double* sums, unsigned long long* counts, hipStream_t s) {
  const int64_t count = static_cast<int64_t>(nm) * nm * (nm / 2 + 1);
  const int64_t per_block = static_cast<int64_t>(kNT) * kModesPerThread;
  const unsigned blocks = static_cast<unsigned>((count + per_block - 1) / per_block);
  const size_t lds = static_cast<size_t>(n_bins) * 3 * sizeof(double) + sizeof(float) * nm;
  k_pk_bin<<<blocks, kNT, lds, s>>>(spec, nm, pitch, 2.0 * M_PI / box, k_max / n_bins, n_bins, pscale, sums,
                                    counts);
  return hipGetLastError();
}

}  // namespace kern
}  // namespace lpc
