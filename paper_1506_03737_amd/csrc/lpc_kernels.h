// Internal launcher interface between the ABI layer and the HIP kernels of liblpc (not part of the C ABI).
//
// Every launcher enqueues on `s` and returns the launch status; none synchronises.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lpc {
namespace kern {

constexpr int kNT = 256;           // threads per workgroup of the particle and elementwise kernels
constexpr int kFftNT = 512;        // threads per workgroup of the FFT kernels
constexpr int kTileElems = 8192;   // complex values per LDS FFT tile (64 KiB)
constexpr int kFracBits = 16;      // fixed-point fractional bits per axis of the CIC deposit
constexpr int kMaxStages = 7;

// Device error flags, one int each, at the start of every workspace.
enum { kFlagOverflow = 0, kFlagNonfinite = 1, kNumFlags = 2 };

// One 1-D transform length factored into radix stages (applied in order; radices 2, 3, 4, 5, 8). For stage s,
// p[s] is the product of the earlier radices, pmask[s] = p[s] - 1 when p[s] is a power of two (else -1), and the
// stage's twiddles W_{p R}^{r k} (k < p, 1 <= r < R) sit at tw_off[s] + k (R - 1) + r - 1 of the twiddle table
// (n - 1 entries in all).
struct Plan1D {
  int n;
  int nst;
  int radix[kMaxStages];
  int p[kMaxStages];
  int pmask[kMaxStages];
  int tw_off[kMaxStages];
};

bool make_plan(int n, Plan1D* p);        // false if n has a prime factor > 5 or n < 1
int mesh_pitch(int n);                   // complex row pitch of the half-spectrum layout, >= n/2 + 1

// Per-kick scalars (FP64 table rows reduced to FP32 products).
struct KickDrift {
  float kick;        // K_i * (-3/2 Om)
  float d1;          // D1(a_i)            (COLA frame term)
  float d2m;         // D2(a_i) - D1(a_i)^2
  float drift;       // Q_i
  float dd1, dd2;    // D1(a_{i+1}) - D1(a_i), D2(a_{i+1}) - D2(a_i)
  int do_drift;
  int cola;
};

hipError_t fill_u64(uint64_t* p, size_t count, hipStream_t s);
hipError_t fill_i32(int* p, size_t count, int value, hipStream_t s);

// Fixed-point CIC deposit into C[nm^3] (must be zeroed). scale = nm 2^16 / box in FP64.
hipError_t deposit(const float* pos, int64_t n, int nm, double scale, uint64_t* C, int* flags, hipStream_t s);

// z-pass of the forward r2c 3-D FFT.
//   from fixed point: delta = C * mscale - 1 (FP64, rounded to FP32), rows of nm reals, nrows = nm^2
hipError_t fft_z_r2c_fixed(const uint64_t* C, int nm, double mscale, float2* out, int pitch, int* flags,
                           hipStream_t s);
//   from an FP32 real mesh (rows of n reals)
hipError_t fft_z_r2c_real(const float* in, int n, float2* out, int pitch, hipStream_t s);

// Complex FFT along a strided axis of `ncomp` meshes (in place). Element (axis j, outer o, column c, comp q) is at
// base + q*comp_stride + o*outer_stride + j*axis_stride + c.
hipError_t fft_axis(float2* base, int n, int64_t axis_stride, int64_t outer_stride, int n_outer, int ncols, int ncomp,
                    int64_t comp_stride, bool inverse, hipStream_t s);

// Fused x-pass: forward FFT along x of the half spectrum in A (after z and y passes), Poisson/deconvolution/
// gradient multiply for the three components, inverse FFT along x; outputs into A (x comp), B (y), C (z).
hipError_t fft_x_poisson(float2* A, float2* B, float2* C, int nm, int pitch, double box, int deconv_power,
                         hipStream_t s);

// z-pass of the inverse c2r 3-D FFT: three component spectra -> AoS float3 real mesh out[nm^3][3].
hipError_t fft_z_c2r_aos3(const float2* A, const float2* B, const float2* C, int nm, int pitch, float* out,
                          hipStream_t s);
//   one spectrum -> planar real mesh out[n^3] times `scale`
hipError_t fft_z_c2r_real(const float2* in, int n, int pitch, float* out, float scale, hipStream_t s);

// Fused CIC gather of the AoS force mesh + COLA kick (+ drift) per particle.
hipError_t gather_kick_drift(float* pos, float* vel, const float* psi1, const float* psi2, int64_t n,
                             const float* force, int nm, double scale, float box, KickDrift kd, int* flags,
                             hipStream_t s);
// CIC gather only: grad[3][n].
hipError_t gather(const float* pos, int64_t n, const float* force, int nm, double scale, float* grad, int* flags,
                  hipStream_t s);
// vel += sign * (f1 psi1 + f2 psi2)
hipError_t frame_velocity(float* vel, const float* psi1, const float* psi2, int64_t n, float f1, float f2,
                          hipStream_t s);

// Initial conditions on an N^3 lattice.
hipError_t ic_noise(uint64_t seed, int N, float* out, hipStream_t s);
// delta_hat = noise_hat * sqrt(P(k) N^3 / V) in place (half spectrum, pitch); zero k = 0 and Nyquist planes.
hipError_t ic_scale_spectrum(float2* spec, int N, int pitch, double box, double amplitude, double omega_m, double h,
                             double n_s, hipStream_t s);
// out = factor * in with factor one of: kind 0..2 -> i k_j / k^2 (Psi1_j), kind 3..8 -> k_i k_j / k^2 (phi1_ij for
// (xx, yy, zz, xy, xz, yz)), kind 9..11 -> -i k_j / k^2 (Psi2_j from the source spectrum); zero at k = 0 / Nyquist.
hipError_t ic_spectral_factor(const float2* in, float2* out, int N, int pitch, double box, int kind, hipStream_t s);
// S = a*b + a*c + b*c (written into a), then S -= d^2 via ic_sub_square
hipError_t ic_source_init(float* a, const float* b, const float* c, int64_t count, hipStream_t s);
hipError_t ic_sub_square(float* S, const float* d, int64_t count, hipStream_t s);
hipError_t ic_assemble(float* pos, float* vel, int32_t* id, const float* psi1, const float* psi2, int N, double box,
                       float d1, float d2, float f1, float f2, hipStream_t s);

// Power-spectrum binning of a half spectrum: sums[b] += (k, P) per mode, counts[b] += multiplicity.
hipError_t pk_bin(const float2* spec, int nm, int pitch, double box, double k_max, int n_bins, double pscale,
                  double* sums, unsigned long long* counts, hipStream_t s);

}  // namespace kern
}  // namespace lpc
