// 3-D real FFTs of liblpc as three LDS-staged passes over HBM (Sec. 2.4 steps 2-3 of Howlett, Manera & Percival
// 2015: forward FFT of the density, Poisson solve and gradient in k-space, inverse FFT per force component).
//
// Layout: a real mesh is x-major float[n][n][n]; its half spectrum is float2[n][n][pitch] with kz = 0..n/2 used
// (pitch = n/2 + 1 rounded up to 8 complex values, 64 bytes, so every row starts on a 64-byte boundary).
// Forward: z pass (r2c of each row via a length-n/2 complex FFT and the even/odd split), y pass, x pass.
// Inverse: x pass, y pass, z pass (c2r via the same split). The force path fuses the forward x pass, the Poisson /
// deconvolution / gradient multiply and the three inverse x passes into one kernel, so the density spectrum is
// read once and never written back.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fft_device.h"

namespace lpc {
namespace kern {

bool make_plan(int n, Plan1D* p) {
  if (n < 1) return false;
  int m = n, ns = 0;
  int radix[kMaxStages];
  for (int r : {5, 3}) {
    while (m % r == 0) {
      if (ns >= kMaxStages) return false;
      radix[ns++] = r;
      m /= r;
    }
  }
  int k = 0;
  while (m % 2 == 0) {
    m /= 2;
    ++k;
  }
  if (m != 1) return false;
  // powers of two: as many radix-8 stages as possible, the remainder as one radix-4 or radix-2 stage
  // (two radix-4 stages instead of 8 x 2 keep the work per stage even).
  int n8 = k / 3, rem = k % 3;
  if (rem == 1 && n8 > 0) {  // 8 x 2 -> 4 x 4
    --n8;
    rem = 4;
  }
  int pow2[kMaxStages], np = 0;
  for (int i = 0; i < n8; ++i) pow2[np++] = 8;
  if (rem == 1) pow2[np++] = 2;
  if (rem == 2) pow2[np++] = 4;
  if (rem == 4) {
    pow2[np++] = 4;
    pow2[np++] = 4;
  }
  if (ns + np > kMaxStages) return false;
  p->n = n;
  p->nst = 0;
  for (int i = 0; i < np; ++i) p->radix[p->nst++] = pow2[i];
  for (int i = 0; i < ns; ++i) p->radix[p->nst++] = radix[i];
  if (n == 1) {  // length-1 transform: no stage
    p->nst = 0;
  }
  return true;
}

int mesh_pitch(int n) { return ((n / 2 + 1) + 7) / 8 * 8; }

namespace {

template <class K>
void allow_big_lds(K kernel) {
  hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                      160 * 1024);
}

// log2 of the columns per tile of a strided pass of length n: B = 2^lgB <= 32 with n * B <= kTileElems.
int strided_lg_cols(int n) {
  int lg = 0;
  while (lg < 5 && (2 << lg) * n <= kTileElems) ++lg;
  return lg;
}

// log2 of the rows per workgroup of a z pass (transform length h = n/2) with `groups` column groups per row.
int z_lg_rows(int n, int groups) {
  int lg = 0;
  while (lg < 4 && groups * (2 << lg) * (n / 2) <= kTileElems) ++lg;
  return lg;
}

// ---------------------------------------------------------------------------------------------------------------
// z pass, forward r2c. A workgroup transforms B = 2^lgB consecutive rows of n reals. Each row is read as n/2 complex
// values z[m] = x[2m] + i x[2m+1]; after the length-n/2 FFT, X[k] = E[k] + exp(-2 pi i k / n) O[k] with
// E[k] = (Z[k] + conj Z[n/2-k]) / 2 and O[k] = (Z[k] - conj Z[n/2-k]) / (2 i), for k = 0..n/2.
template <bool FIXED>
__global__ __launch_bounds__(kFftNT) void k_fft_z_r2c(const void* __restrict__ in, int n, int nrows,
                                                      float2* __restrict__ out, int pitch, double mscale, Plan1D pl,
                                                      int lgB, int* __restrict__ flags) {
  extern __shared__ float2 smem[];
  const int h = n / 2, B = 1 << lgB, BP = B + 1, tid = threadIdx.x;
  float2* tile = smem;
  float2* tw = smem + h * BP;
  fill_twiddles(tw, n, tid);
  const int row0 = blockIdx.x * B;
  bool overflow = false;
  for (int b = 0; b < B; ++b) {
    const int row = row0 + b;
    if (FIXED) {
      const ulonglong2* src = reinterpret_cast<const ulonglong2*>(static_cast<const uint64_t*>(in) +
                                                                  static_cast<size_t>(row) * n);
      for (int j = tid; j < h; j += kFftNT) {
        float2 v = make_float2(0.f, 0.f);
        if (row < nrows) {
          const ulonglong2 c = src[j];
          overflow |= ((c.x | c.y) >> 63) != 0;
          v.x = static_cast<float>(static_cast<double>(c.x) * mscale - 1.0);
          v.y = static_cast<float>(static_cast<double>(c.y) * mscale - 1.0);
        }
        tile[j * BP + b] = v;
      }
    } else {
      const float2* src = static_cast<const float2*>(in) + static_cast<size_t>(row) * h;
      for (int j = tid; j < h; j += kFftNT) tile[j * BP + b] = (row < nrows) ? src[j] : make_float2(0.f, 0.f);
    }
  }
  if (FIXED && overflow) atomicOr(flags + kFlagOverflow, 1);
  __syncthreads();
  fft_tile<false>(tile, BP, tw, 2, pl, lgB, tid);
  for (int b = 0; b < B; ++b) {
    const int row = row0 + b;
    if (row >= nrows) break;
    float2* dst = out + static_cast<size_t>(row) * pitch;
    for (int k = tid; k <= h; k += kFftNT) {
      const float2 zk = tile[(k == h ? 0 : k) * BP + b];
      const float2 zm = tile[(k == 0 ? 0 : h - k) * BP + b];
      const float2 E = cscale(cadd(zk, cconj(zm)), 0.5f);
      const float2 O = cscale(rot<false>(csub(zk, cconj(zm))), 0.5f);  // (zk - conj zm) / (2 i)
      dst[k] = cadd(E, cmul(tw[k], O));
    }
  }
}

// Load/store of a strided tile: element (j, b) of the tile <-> ptr[j * astr + b], for b < bw.
__device__ __forceinline__ void load_strided(float2* tile, int BP, const float2* __restrict__ ptr, int64_t astr, int n,
                                             int lgB, int bw, int tid) {
  const int b = tid & ((1 << lgB) - 1), S = kFftNT >> lgB;
  const float2* p = ptr + b + static_cast<int64_t>(tid >> lgB) * astr;
  const int64_t step = static_cast<int64_t>(S) * astr;
  for (int j = tid >> lgB; j < n; j += S, p += step) tile[j * BP + b] = (b < bw) ? *p : make_float2(0.f, 0.f);
}

__device__ __forceinline__ void store_strided(const float2* tile, int BP, float2* __restrict__ ptr, int64_t astr,
                                              int n, int lgB, int bw, int tid) {
  const int b = tid & ((1 << lgB) - 1), S = kFftNT >> lgB;
  if (b >= bw) return;
  float2* p = ptr + b + static_cast<int64_t>(tid >> lgB) * astr;
  const int64_t step = static_cast<int64_t>(S) * astr;
  for (int j = tid >> lgB; j < n; j += S, p += step) *p = tile[j * BP + b];
}

// ---------------------------------------------------------------------------------------------------------------
// Strided complex pass (in place). Tile = B consecutive columns (contiguous in memory) x n points along the axis.
template <bool INV>
__global__ __launch_bounds__(kFftNT) void k_fft_axis(float2* __restrict__ base, int n, int64_t astr, int64_t ostr,
                                                     int n_outer, int ncols, int64_t cstr, Plan1D pl, int lgB) {
  extern __shared__ float2 smem[];
  const int B = 1 << lgB, BP = B + 1, tid = threadIdx.x;
  float2* tile = smem;
  float2* tw = smem + n * BP;
  fill_twiddles(tw, n, tid);
  const int ntc = (ncols + B - 1) >> lgB;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int outer = logical / ntc, ct = logical - outer * ntc;
  const int c0 = ct << lgB, bw = min(B, ncols - c0);
  float2* ptr = base + blockIdx.y * cstr + outer * ostr + c0;
  load_strided(tile, BP, ptr, astr, n, lgB, bw, tid);
  __syncthreads();
  fft_tile<INV>(tile, BP, tw, 1, pl, lgB, tid);
  store_strided(tile, BP, ptr, astr, n, lgB, bw, tid);
}

// ---------------------------------------------------------------------------------------------------------------
// Fused x pass of the force: forward FFT along x, then for each component j = x, y, z
//   g_hat_j = i k_j (-1/k^2) delta_hat / W^p / Nm^3     (zero at k = 0 and on the Nyquist plane of axis j),
// inverse FFT along x, store. W = prod_d sinc^2(pi n_d / Nm). The 1/Nm^3 of the inverse transform is folded in.
__global__ __launch_bounds__(kFftNT) void k_fft_x_poisson(float2* __restrict__ A, float2* __restrict__ Bm,
                                                          float2* __restrict__ Cm, int nm, int pitch, float kf,
                                                          float inv_m3, int deconv, Plan1D pl, int lgB) {
  extern __shared__ float2 smem[];
  const int n = nm, B = 1 << lgB, BP = B + 1, tid = threadIdx.x, nh = nm / 2 + 1;
  float2* tile = smem;
  float2* tw = smem + n * BP;
  float* win = reinterpret_cast<float*>(tw + n);  // sinc^2(pi m / n), m < n (even in m)
  fill_twiddles(tw, n, tid);
  for (int m = tid; m < n; m += kFftNT) {
    const int mm = min(m, n - m);
    double w = 1.0;
    if (mm != 0) {
      const double x = static_cast<double>(mm) / n;
      w = sinpi(x) / (M_PI * x);
      w = w * w;
    }
    win[m] = static_cast<float>(w);
  }
  const int ntc = (nh + B - 1) >> lgB;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int y = logical / ntc, ct = logical - y * ntc;
  const int c0 = ct << lgB, bw = min(B, nh - c0);
  const int64_t astr = static_cast<int64_t>(nm) * pitch;
  const int64_t off = static_cast<int64_t>(y) * pitch + c0;
  load_strided(tile, BP, A + off, astr, n, lgB, bw, tid);
  __syncthreads();
  fft_tile<false>(tile, BP, tw, 1, pl, lgB, tid);

  // This thread's elements (j = j0 + m S, column b): delta_hat stays in registers across the three components.
  const int b = tid & (B - 1), S = kFftNT >> lgB, j0 = tid >> lgB;
  const int half = nm / 2;
  const int ny = (y <= half) ? y : y - nm;
  const int nz = c0 + b;
  const bool col_ok = b < bw;
  const float wyz = win[y] * win[min(nz, n - 1)];
  const int nyz2 = ny * ny + nz * nz;
  float2 d[kEPT];
#pragma unroll
  for (int m = 0; m < kEPT; ++m) {
    const int j = j0 + m * S;
    d[m] = (j < n) ? tile[j * BP + b] : make_float2(0.f, 0.f);
  }
  float2* outs[3] = {A, Bm, Cm};
  for (int comp = 0; comp < 3; ++comp) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kEPT; ++m) {
      const int j = j0 + m * S;
      if (j < n) {
        const int nx = (j <= half) ? j : j - nm;
        const float k2 = kf * kf * static_cast<float>(nx * nx + nyz2);
        const int nc = (comp == 0) ? nx : (comp == 1 ? ny : nz);
        float s = 0.f;
        if (k2 > 0.f && col_ok && nc != half && nc != -half) {
          const float W = win[j] * wyz;
          const float wp = (deconv == 0) ? 1.f : (deconv == 1 ? W : W * W);
          s = -kf * static_cast<float>(nc) * inv_m3 / (k2 * wp);  // k_c * (-1 / (k^2 W^p Nm^3))
        }
        tile[j * BP + b] = make_float2(-s * d[m].y, s * d[m].x);  // i * s * delta_hat
      }
    }
    __syncthreads();
    fft_tile<true>(tile, BP, tw, 1, pl, lgB, tid);
    store_strided(tile, BP, outs[comp] + off, astr, n, lgB, bw, tid);
  }
}

// ---------------------------------------------------------------------------------------------------------------
// z pass, inverse c2r. A workgroup transforms R = 2^lgR rows of each of NC spectra; the tile has G * R columns
// (G = 1 for NC = 1, G = 4 for NC = 3: one column group stays zero so the column count is a power of two).
// With X the half spectrum of a real row,
//   Z[k] = (X[k] + conj X[h-k]) + i exp(+2 pi i k / n) (X[k] - conj X[h-k]),  h = n/2, k < h,
// and the unnormalised length-h inverse FFT of Z gives x[2m] + i x[2m+1].
template <int NC>
__global__ __launch_bounds__(kFftNT) void k_fft_z_c2r(const float2* __restrict__ in0, const float2* __restrict__ in1,
                                                      const float2* __restrict__ in2, int n, int nrows, int pitch,
                                                      float* __restrict__ out, float scale, Plan1D pl, int lgR) {
  constexpr int G = (NC == 1) ? 1 : 4;
  extern __shared__ float2 smem[];
  const int h = n / 2, R = 1 << lgR, ncol = G * R, BP = ncol + 1, tid = threadIdx.x;
  int lgB = lgR + ((G == 4) ? 2 : 0);
  float2* tile = smem;                 // (h + 1) x BP
  float2* tw = smem + (h + 1) * BP;    // n-th roots
  fill_twiddles(tw, n, tid);
  const int row0 = blockIdx.x * R;
  const float2* ins[3] = {in0, in1, in2};
  for (int col = 0; col < ncol; ++col) {
    const int c = col >> lgR, r = col & (R - 1);
    const int row = row0 + r;
    const bool live = (c < NC) && (row < nrows);
    const float2* src = ins[c < NC ? c : 0] + static_cast<size_t>(row) * pitch;
    for (int k = tid; k <= h; k += kFftNT) tile[k * BP + col] = live ? src[k] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  for (int col = 0; col < NC * R; ++col) {
    for (int k = tid; k <= h / 2; k += kFftNT) {
      const float2 xk = tile[k * BP + col];
      const float2 xm = tile[(h - k) * BP + col];
      const float2 t = tw[k];
      // Z[k] = (xk + conj xm) + i conj(t) (xk - conj xm)
      const float2 zk = cadd(cadd(xk, cconj(xm)), rot<true>(cmulc(csub(xk, cconj(xm)), t)));
      if (k != 0 && 2 * k != h) {
        // Z[h-k] = (xm + conj xk) - i t (xm - conj xk)
        const float2 zm = csub(cadd(xm, cconj(xk)), rot<true>(cmul(csub(xm, cconj(xk)), t)));
        tile[(h - k) * BP + col] = zm;
      }
      tile[k * BP + col] = zk;
    }
  }
  __syncthreads();
  fft_tile<true>(tile, BP, tw, 2, pl, lgB, tid);
  const int rowlen = NC * n;
  for (int r = 0; r < R; ++r) {
    const int row = row0 + r;
    if (row >= nrows) break;
    float* dst = out + static_cast<size_t>(row) * rowlen;
    for (int q = tid; q < rowlen; q += kFftNT) {
      const int jj = q / NC, c = q - jj * NC;
      const float2 z = tile[(jj >> 1) * BP + c * R + r];
      dst[q] = ((jj & 1) ? z.y : z.x) * scale;
    }
  }
}

size_t lds_z_r2c(int n, int B) { return sizeof(float2) * (static_cast<size_t>(n / 2) * (B + 1) + n); }
size_t lds_axis(int n, int B) { return sizeof(float2) * (static_cast<size_t>(n) * (B + 1) + n); }
size_t lds_x_poisson(int n, int B) { return lds_axis(n, B) + sizeof(float) * n; }
size_t lds_z_c2r(int n, int ncol) { return sizeof(float2) * (static_cast<size_t>(n / 2 + 1) * (ncol + 1) + n); }

struct Init {
  Init() {
    allow_big_lds(k_fft_z_r2c<true>);
    allow_big_lds(k_fft_z_r2c<false>);
    allow_big_lds(k_fft_axis<true>);
    allow_big_lds(k_fft_axis<false>);
    allow_big_lds(k_fft_x_poisson);
    allow_big_lds(k_fft_z_c2r<1>);
    allow_big_lds(k_fft_z_c2r<3>);
  }
};

void ensure_init() { static Init once; }

}  // namespace

hipError_t fft_z_r2c_fixed(const uint64_t* C, int nm, double mscale, float2* out, int pitch, int* flags,
                           hipStream_t s) {
  ensure_init();
  Plan1D pl;
  if (!make_plan(nm / 2, &pl)) return hipErrorInvalidValue;
  const int lgB = z_lg_rows(nm, 1), B = 1 << lgB, nrows = nm * nm;
  k_fft_z_r2c<true><<<(nrows + B - 1) / B, kFftNT, lds_z_r2c(nm, B), s>>>(C, nm, nrows, out, pitch, mscale, pl, lgB,
                                                                            flags);
  return hipGetLastError();
}

hipError_t fft_z_r2c_real(const float* in, int n, float2* out, int pitch, hipStream_t s) {
  ensure_init();
  Plan1D pl;
  if (!make_plan(n / 2, &pl)) return hipErrorInvalidValue;
  const int lgB = z_lg_rows(n, 1), B = 1 << lgB, nrows = n * n;
  k_fft_z_r2c<false><<<(nrows + B - 1) / B, kFftNT, lds_z_r2c(n, B), s>>>(in, n, nrows, out, pitch, 0.0, pl, lgB,
                                                                            nullptr);
  return hipGetLastError();
}

hipError_t fft_axis(float2* base, int n, int64_t axis_stride, int64_t outer_stride, int n_outer, int ncols, int ncomp,
                    int64_t comp_stride, bool inverse, hipStream_t s) {
  ensure_init();
  Plan1D pl;
  if (!make_plan(n, &pl)) return hipErrorInvalidValue;
  const int lgB = strided_lg_cols(n), B = 1 << lgB;
  const int ntc = (ncols + B - 1) / B;
  dim3 grid(n_outer * ntc, ncomp);
  if (inverse)
    k_fft_axis<true><<<grid, kFftNT, lds_axis(n, B), s>>>(base, n, axis_stride, outer_stride, n_outer, ncols,
                                                            comp_stride, pl, lgB);
  else
    k_fft_axis<false><<<grid, kFftNT, lds_axis(n, B), s>>>(base, n, axis_stride, outer_stride, n_outer, ncols,
                                                             comp_stride, pl, lgB);
  return hipGetLastError();
}

hipError_t fft_x_poisson(float2* A, float2* B, float2* C, int nm, int pitch, double box, int deconv_power,
                         hipStream_t s) {
  ensure_init();
  Plan1D pl;
  if (!make_plan(nm, &pl)) return hipErrorInvalidValue;
  const int lgB = strided_lg_cols(nm), Bc = 1 << lgB;
  const int nh = nm / 2 + 1, ntc = (nh + Bc - 1) / Bc;
  const float kf = static_cast<float>(2.0 * M_PI / box);
  const float inv_m3 = static_cast<float>(1.0 / (static_cast<double>(nm) * nm * nm));
  k_fft_x_poisson<<<nm * ntc, kFftNT, lds_x_poisson(nm, Bc), s>>>(A, B, C, nm, pitch, kf, inv_m3, deconv_power, pl,
                                                                    lgB);
  return hipGetLastError();
}

hipError_t fft_z_c2r_aos3(const float2* A, const float2* B, const float2* C, int nm, int pitch, float* out,
                          hipStream_t s) {
  ensure_init();
  Plan1D pl;
  if (!make_plan(nm / 2, &pl)) return hipErrorInvalidValue;
  const int lgR = z_lg_rows(nm, 4), R = 1 << lgR, nrows = nm * nm;
  k_fft_z_c2r<3><<<(nrows + R - 1) / R, kFftNT, lds_z_c2r(nm, 4 * R), s>>>(A, B, C, nm, nrows, pitch, out, 1.0f, pl,
                                                                             lgR);
  return hipGetLastError();
}

hipError_t fft_z_c2r_real(const float2* in, int n, int pitch, float* out, float scale, hipStream_t s) {
  ensure_init();
  Plan1D pl;
  if (!make_plan(n / 2, &pl)) return hipErrorInvalidValue;
  const int lgR = z_lg_rows(n, 1), R = 1 << lgR, nrows = n * n;
  k_fft_z_c2r<1><<<(nrows + R - 1) / R, kFftNT, lds_z_c2r(n, R), s>>>(in, in, in, n, nrows, pitch, out, scale, pl,
                                                                        lgR);
  return hipGetLastError();
}

}  // namespace kern
}  // namespace lpc
