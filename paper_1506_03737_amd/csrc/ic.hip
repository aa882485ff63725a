// Initial-condition kernels of liblpc (Sec. 2.1 Eqs. 5-10 and Sec. 5 of Howlett, Manera & Percival 2015):
// counter-based white noise, scaling by the linear spectrum, the spectral derivatives that give Psi1, the second
// derivatives of phi1 that form the 2LPT source, and the final assembly of positions and momenta on the lattice.
#include <hip/hip_runtime.h>

#include <cmath>

#include "lpc_kernels.h"

namespace lpc {
namespace kern {

namespace {

// SplitMix64 (Steele, Lea & Flood 2014): the c-th output of a stream whose state starts at `seed`.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double uniform_open(uint64_t seed, uint64_t c) {
  return (static_cast<double>(splitmix64(seed, c) >> 11) + 0.5) * 0x1.0p-53;
}

__global__ __launch_bounds__(kNT) void k_ic_noise(uint64_t seed, int64_t count, float* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (i >= count) return;
  const uint64_t idx = static_cast<uint64_t>(i);
  const double u1 = uniform_open(seed, 2 * idx), u2 = uniform_open(seed, 2 * idx + 1);
  out[i] = static_cast<float>(sqrt(-2.0 * log(u1)) * cospi(2.0 * u2));  // Box-Muller
}

// signed frequency of index j on an axis of length N
__device__ __forceinline__ int signed_freq(int j, int N) { return (j <= N / 2) ? j : j - N; }

struct Mode {
  int nx, ny, nz;
  bool zero;  // k = 0 or a Nyquist index on any axis
};

__device__ __forceinline__ void mode_of(int64_t e, int N, int nh, Mode* m) {
  const int kz = static_cast<int>(e % nh);
  const int64_t r = e / nh;
  const int ky = static_cast<int>(r % N), kx = static_cast<int>(r / N);
  m->nx = signed_freq(kx, N);
  m->ny = signed_freq(ky, N);
  m->nz = kz;
  const int h = N / 2;
  m->zero = (m->nx == 0 && m->ny == 0 && kz == 0) || m->nx == h || m->nx == -h || m->ny == h || m->ny == -h ||
            kz == h;
}

__device__ __forceinline__ int64_t spec_index(int64_t e, int nh, int pitch) {
  const int kz = static_cast<int>(e % nh);
  const int64_t r = e / nh;
  return r * pitch + kz;
}

// BBKS transfer function (Bardeen et al. 1986), q = k / (Om h).
__device__ __forceinline__ double bbks(double k, double om_h) {
  const double q = k / om_h, x = 2.34 * q;
  const double a = 16.1 * q, b = 5.46 * q, d = 6.71 * q;
  const double poly = 1.0 + 3.89 * q + a * a + b * b * b + d * d * d * d;
  return log1p(x) / x / sqrt(sqrt(poly));
}

__global__ __launch_bounds__(kNT) void k_ic_scale(float2* __restrict__ spec, int N, int pitch, double kf,
                                                  double amp_norm, double A, double om_h, double n_s) {
  const int nh = N / 2 + 1;
  const int64_t count = static_cast<int64_t>(N) * N * nh;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (e >= count) return;
  Mode m;
  mode_of(e, N, nh, &m);
  const int64_t idx = spec_index(e, nh, pitch);
  if (m.zero) {
    spec[idx] = make_float2(0.f, 0.f);
    return;
  }
  const double k = kf * sqrt(static_cast<double>(m.nx * m.nx + m.ny * m.ny + m.nz * m.nz));
  const double t = bbks(k, om_h);
  const double amp = sqrt(A * pow(k, n_s) * t * t * amp_norm);
  const float2 v = spec[idx];
  spec[idx] = make_float2(static_cast<float>(v.x * amp), static_cast<float>(v.y * amp));
}

__global__ __launch_bounds__(kNT) void k_ic_factor(const float2* __restrict__ in, float2* __restrict__ out, int N,
                                                   int pitch, float kf, int kind) {
  const int nh = N / 2 + 1;
  const int64_t count = static_cast<int64_t>(N) * N * nh;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (e >= count) return;
  Mode m;
  mode_of(e, N, nh, &m);
  const int64_t idx = spec_index(e, nh, pitch);
  if (m.zero) {
    out[idx] = make_float2(0.f, 0.f);
    return;
  }
  const float k[3] = {kf * m.nx, kf * m.ny, kf * m.nz};
  const float inv_k2 = 1.0f / (k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
  const float2 v = in[idx];
  float2 o;
  if (kind < 3) {  // Psi1_j = i k_j delta / k^2
    const float s = k[kind] * inv_k2;
    o = make_float2(-s * v.y, s * v.x);
  } else if (kind < 9) {  // phi1_ij = k_i k_j delta / k^2
    const int ii[6] = {0, 1, 2, 0, 0, 1}, jj[6] = {0, 1, 2, 1, 2, 2};
    const float s = k[ii[kind - 3]] * k[jj[kind - 3]] * inv_k2;
    o = make_float2(s * v.x, s * v.y);
  } else {  // Psi2_j = i k_j phi2_hat with phi2_hat = -S_hat / k^2
    const float s = -k[kind - 9] * inv_k2;
    o = make_float2(-s * v.y, s * v.x);
  }
  out[idx] = o;
}

__global__ __launch_bounds__(kNT) void k_ic_source_init(float* __restrict__ a, const float* __restrict__ b,
                                                        const float* __restrict__ c, int64_t count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (i < count) {
    const float x = a[i], y = b[i], z = c[i];
    a[i] = x * y + x * z + y * z;
  }
}

__global__ __launch_bounds__(kNT) void k_ic_sub_square(float* __restrict__ S, const float* __restrict__ d,
                                                        int64_t count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (i < count) S[i] -= d[i] * d[i];
}

__global__ __launch_bounds__(kNT) void k_ic_assemble(float* __restrict__ pos, float* __restrict__ vel,
                                                     int32_t* __restrict__ id, const float* __restrict__ psi1,
                                                     const float* __restrict__ psi2, int N, double box, float d1,
                                                     float d2, float f1, float f2) {
  const int64_t n = static_cast<int64_t>(N) * N * N;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (i >= n) return;
  const int l = static_cast<int>(i % N), j = static_cast<int>((i / N) % N), ix = static_cast<int>(i / (N * N));
  const int lat[3] = {ix, j, l};
  const double spacing = box / N;
  const float fbox = static_cast<float>(box);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float p1 = psi1[d * n + i], p2 = psi2[d * n + i];
    double x = (lat[d] + 0.5) * spacing + static_cast<double>(d1) * p1 + static_cast<double>(d2) * p2;
    x -= box * floor(x / box);
    float xf = static_cast<float>(x);
    if (xf >= fbox) xf -= fbox;
    pos[d * n + i] = xf;
    vel[d * n + i] = f1 * p1 + f2 * p2;
  }
  id[i] = static_cast<int32_t>(i);
}

// Primordial non-Gaussianity (Sec. 5). Phi_hat = phi_hat + fNL NL_hat with phi the Gaussian primordial potential and
// NL = sum_j c_j D^g[(D^a phi)(D^b phi)], D^s multiplying mode k by k^(s (4 - ns) / 3); delta_L_hat = alpha(k) Phi_hat.

// phi_hat = noise_hat sqrt(A_phi k^(ns - 4) N^3 / V) in place; zero at k = 0 and on the Nyquist planes.
__global__ __launch_bounds__(kNT) void k_png_potential(float2* __restrict__ spec, int N, int pitch, double kf,
                                                       double amp_norm, double a_phi, double n_s) {
  const int nh = N / 2 + 1;
  const int64_t count = static_cast<int64_t>(N) * N * nh;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (e >= count) return;
  Mode m;
  mode_of(e, N, nh, &m);
  const int64_t idx = spec_index(e, nh, pitch);
  if (m.zero) {
    spec[idx] = make_float2(0.f, 0.f);
    return;
  }
  const double k = kf * sqrt(static_cast<double>(m.nx * m.nx + m.ny * m.ny + m.nz * m.nz));
  const double amp = sqrt(a_phi * pow(k, n_s - 4.0) * amp_norm);
  const float2 v = spec[idx];
  spec[idx] = make_float2(static_cast<float>(v.x * amp), static_cast<float>(v.y * amp));
}

// out = coef k^expo in (accumulate = 0) or out += coef k^expo in (accumulate = 1); zero at k = 0 and Nyquist.
__global__ __launch_bounds__(kNT) void k_png_power(const float2* __restrict__ in, float2* __restrict__ out, int N,
                                                   int pitch, double kf, double expo, double coef, int accumulate) {
  const int nh = N / 2 + 1;
  const int64_t count = static_cast<int64_t>(N) * N * nh;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (e >= count) return;
  Mode m;
  mode_of(e, N, nh, &m);
  const int64_t idx = spec_index(e, nh, pitch);
  float2 o = make_float2(0.f, 0.f);
  if (!m.zero) {
    const double k = kf * sqrt(static_cast<double>(m.nx * m.nx + m.ny * m.ny + m.nz * m.nz));
    const double f = coef * (expo == 0.0 ? 1.0 : pow(k, expo));
    const float2 v = in[idx];
    o = make_float2(static_cast<float>(v.x * f), static_cast<float>(v.y * f));
  }
  if (accumulate) {
    const float2 prev = out[idx];
    o = make_float2(prev.x + o.x, prev.y + o.y);
  }
  out[idx] = o;
}

__global__ __launch_bounds__(kNT) void k_png_products(PngProducts pp, int64_t count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (i >= count) return;
  float acc = 0.f;
  for (int t = 0; t < pp.n; ++t) acc += pp.c[t] * (pp.fa[t][i] * pp.fb[t][i]);
  pp.out[i] = acc;
}

// delta_L_hat = alpha0 k^2 T(k) (phi_hat + fNL NL_hat) into phi_hat's place; zero at k = 0 and Nyquist.
__global__ __launch_bounds__(kNT) void k_png_to_delta(float2* __restrict__ phi, const float2* __restrict__ nl, int N,
                                                      int pitch, double kf, double f_nl, double alpha0, double om_h) {
  const int nh = N / 2 + 1;
  const int64_t count = static_cast<int64_t>(N) * N * nh;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (e >= count) return;
  Mode m;
  mode_of(e, N, nh, &m);
  const int64_t idx = spec_index(e, nh, pitch);
  if (m.zero) {
    phi[idx] = make_float2(0.f, 0.f);
    return;
  }
  const double k = kf * sqrt(static_cast<double>(m.nx * m.nx + m.ny * m.ny + m.nz * m.nz));
  const double a = alpha0 * k * k * bbks(k, om_h);
  const float2 p = phi[idx], q = nl[idx];
  phi[idx] = make_float2(static_cast<float>(a * (p.x + f_nl * q.x)), static_cast<float>(a * (p.y + f_nl * q.y)));
}

unsigned grid_for(int64_t n) { return static_cast<unsigned>((n + kNT - 1) / kNT); }

}  // namespace

hipError_t ic_noise(uint64_t seed, int N, float* out, hipStream_t s) {
  const int64_t count = static_cast<int64_t>(N) * N * N;
  k_ic_noise<<<grid_for(count), kNT, 0, s>>>(seed, count, out);
  return hipGetLastError();
}

hipError_t ic_scale_spectrum(float2* spec, int N, int pitch, double box, double amplitude, double omega_m, double h,
                             double n_s, hipStream_t s) {
  const int64_t count = static_cast<int64_t>(N) * N * (N / 2 + 1);
  const double kf = 2.0 * M_PI / box;
  const double amp_norm = static_cast<double>(N) * N * N / (box * box * box);
  k_ic_scale<<<grid_for(count), kNT, 0, s>>>(spec, N, pitch, kf, amp_norm, amplitude, omega_m * h, n_s);
  return hipGetLastError();
}

hipError_t ic_spectral_factor(const float2* in, float2* out, int N, int pitch, double box, int kind, hipStream_t s) {
  const int64_t count = static_cast<int64_t>(N) * N * (N / 2 + 1);
  k_ic_factor<<<grid_for(count), kNT, 0, s>>>(in, out, N, pitch, static_cast<float>(2.0 * M_PI / box), kind);
  return hipGetLastError();
}

hipError_t ic_source_init(float* a, const float* b, const float* c, int64_t count, hipStream_t s) {
  k_ic_source_init<<<grid_for(count), kNT, 0, s>>>(a, b, c, count);
  return hipGetLastError();
}

hipError_t ic_sub_square(float* S, const float* d, int64_t count, hipStream_t s) {
  k_ic_sub_square<<<grid_for(count), kNT, 0, s>>>(S, d, count);
  return hipGetLastError();
}

hipError_t png_potential(float2* spec, int N, int pitch, double box, double a_phi, double n_s, hipStream_t s) {
  const int64_t count = static_cast<int64_t>(N) * N * (N / 2 + 1);
  const double amp_norm = static_cast<double>(N) * N * N / (box * box * box);
  k_png_potential<<<grid_for(count), kNT, 0, s>>>(spec, N, pitch, 2.0 * M_PI / box, amp_norm, a_phi, n_s);
  return hipGetLastError();
}

hipError_t png_power(const float2* in, float2* out, int N, int pitch, double box, double expo, double coef,
                     bool accumulate, hipStream_t s) {
  const int64_t count = static_cast<int64_t>(N) * N * (N / 2 + 1);
  k_png_power<<<grid_for(count), kNT, 0, s>>>(in, out, N, pitch, 2.0 * M_PI / box, expo, coef, accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t png_products(const PngProducts& pp, int64_t count, hipStream_t s) {
  if (pp.n < 1 || pp.n > kPngMaxTerms) return hipErrorInvalidValue;
  k_png_products<<<grid_for(count), kNT, 0, s>>>(pp, count);
  return hipGetLastError();
}

hipError_t png_to_delta(float2* phi, const float2* nl, int N, int pitch, double box, double f_nl, double alpha0,
                        double omega_m, double h, hipStream_t s) {
  const int64_t count = static_cast<int64_t>(N) * N * (N / 2 + 1);
  k_png_to_delta<<<grid_for(count), kNT, 0, s>>>(phi, nl, N, pitch, 2.0 * M_PI / box, f_nl, alpha0, omega_m * h);
  return hipGetLastError();
}

hipError_t ic_assemble(float* pos, float* vel, int32_t* id, const float* psi1, const float* psi2, int N, double box,
                       float d1, float d2, float f1, float f2, hipStream_t s) {
  const int64_t n = static_cast<int64_t>(N) * N * N;
  k_ic_assemble<<<grid_for(n), kNT, 0, s>>>(pos, vel, id, psi1, psi2, N, box, d1, d2, f1, f2);
  return hipGetLastError();
}

}  // namespace kern
}  // namespace lpc
