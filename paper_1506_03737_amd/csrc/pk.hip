// Binned power spectrum of a periodic box (the cubic-box form of the FKP estimator used in Sec. 7.1 of Howlett,
// Manera & Percival 2015): P = V |delta_hat|^2 / (Nm^6 W^2) per mode with one CIC window W = prod sinc^2 removed,
// averaged in linear |k| bins. Per-bin sums are FP64 and the mode counts exact integers.
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

}  // namespace

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
