// Kernels of the learned displacement correction (declared in net_kernels.h). The 3^3 convolutions (forward, data
// gradient, and weight gradient on grids a multiple of 32 per side) and the forward 2^3 down/up layers run on BF16
// MFMA with FP32 accumulation; the 2^3 data gradients, the other weight gradients and the element-wise steps run on
// the vector ALUs. Weight gradients are FP32 partial sums per voxel chunk, reduced in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "net_kernels.h"

namespace lpc {
namespace net {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNT = 256;
constexpr float kSlope = 0.1f;

__device__ __forceinline__ int wrapi(int a, int D) { return a < 0 ? a + D : (a >= D ? a - D : a); }
__device__ __forceinline__ float leaky(float v) { return v > 0.f ? v : kSlope * v; }
__device__ __forceinline__ float f(bf16 v) { return static_cast<float>(v); }

unsigned blocks_for(int64_t count, int per = kNT) { return static_cast<unsigned>((count + per - 1) / per); }

// ---------------------------------------------------------------------------------------------------------------
// 3^3 convolution, implicit GEMM on v_mfma_f32_16x16x32_bf16. Operand layout of the instruction: lane l supplies row
// (l % 16) of A and column (l % 16) of B with k = 8 (l / 16) + [0, 8), and receives column (l % 16), rows
// 4 (l / 16) + [0, 4) of the 16 x 16 result.
// A workgroup (4 waves) computes a 4 x 4 x 16 tile of output voxels: wave w takes x = x0 + w, its 4 row tiles are
// y = y0 + mt, and a row tile's 16 rows are z = z0 + [0, 16). The input halo of the tile (6 x 6 x 18 voxels, periodic)
// is staged in LDS one chunk of CC = min(CIN, 32) channels at a time, so every K step reads its A operands from LDS
// at a fixed offset per tap: no wrap-around arithmetic in the inner loop. B (weights) comes from global memory
// (a few hundred KB at most, cache resident).
constexpr int kHX = 6, kHY = 6, kHZ = 18, kHalo = kHX * kHY * kHZ;

__device__ __forceinline__ int modi(int a, int D) {
  const int m = a % D;
  return m < 0 ? m + D : m;
}

template <int CIN, int NB>
__global__ __launch_bounds__(kNT, (CIN >= 64 && NB >= 4) ? 2 : 3) void k_conv3(View in, const bf16* __restrict__ w, int kpad,
                                               const float* __restrict__ bias, int act, View out,
                                               float* __restrict__ outf, int cout, int D, View mask, int mask_ch) {
  constexpr int CC = CIN < 32 ? CIN : 32;   // channels per staged chunk
  constexpr int NCH = CIN / CC;             // chunks
  constexpr int VS = CC + 8;                // LDS voxel stride (bf16), padded against bank conflicts
  constexpr int TPS = 32 / CC;              // taps per K step (4, 2 or 1)
  constexpr int NS = (27 + TPS - 1) / TPS;  // K steps per chunk
  __shared__ bf16 halo[kHalo * VS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, tid = threadIdx.x;
  const int r = lane & 15, g = lane >> 4;
  const int ntxy = (D + 3) / 4, ntz = (D + 15) / 16;
  const int bz = blockIdx.x % ntz, by = (blockIdx.x / ntz) % ntxy, bx = blockIdx.x / (ntz * ntxy);
  const int x0 = bx * 4, y0 = by * 4, z0 = bz * 16;
  const bool wave_on = (x0 + wave) < D;
  f32x4 acc[4][NB];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mt][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  // this lane's tap slot within a K step and its channel offset within the chunk
  const int tsub = g / (CC / 8), cio = 8 * (g % (CC / 8));
  for (int ch = 0; ch < NCH; ++ch) {
    __syncthreads();  // the previous chunk's reads are done
    {
      // the chunk's loads are issued in at most two batches before they are written to LDS (one or two memory
      // latencies per chunk; a single batch of 11 loads for 32 channels would not fit the register budget)
      constexpr int NE = (kHalo * (CC / 8) + kNT - 1) / kNT;
      constexpr int NB1 = NE > 6 ? (NE + 1) / 2 : NE;
#pragma unroll
      for (int m0 = 0; m0 < NE; m0 += NB1) {
        bf16x8 hbuf[NB1];
#pragma unroll
        for (int m = 0; m < NB1; ++m) {
          const int e = tid + (m0 + m) * kNT;
          if (m0 + m < NE && e < kHalo * (CC / 8)) {
            const int hv = e / (CC / 8), grp = e % (CC / 8);
            const int hx = hv / (kHY * kHZ), hy = (hv / kHZ) % kHY, hz = hv % kHZ;
            int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
            if (D >= kHZ) {  // one wrap at most (uniform branch)
              gx = gx < 0 ? gx + D : (gx >= D ? gx - D : gx);
              gy = gy < 0 ? gy + D : (gy >= D ? gy - D : gy);
              gz = gz < 0 ? gz + D : (gz >= D ? gz - D : gz);
            } else {
              gx = modi(gx, D);
              gy = modi(gy, D);
              gz = modi(gz, D);
            }
            const bf16* src =
                in.p + static_cast<size_t>((gx * D + gy) * D + gz) * in.ld + in.off + ch * CC + grp * 8;
            hbuf[m] = *reinterpret_cast<const bf16x8*>(src);
          }
        }
#pragma unroll
        for (int m = 0; m < NB1; ++m) {
          const int e = tid + (m0 + m) * kNT;
          if (m0 + m < NE && e < kHalo * (CC / 8)) {
            const int hv = e / (CC / 8), grp = e % (CC / 8);
            *reinterpret_cast<bf16x8*>(halo + hv * VS + grp * 8) = hbuf[m];
          }
        }
      }
    }
    __syncthreads();
    if (wave_on) {
      // k of this lane's 8 values at step s: tap * CIN + ch * CC + cio (a padding tap points into the zero tail of the
      // row). The weight fragments of step s + 1 are loaded (from global memory) while step s runs.
      const bf16* wlane = w + static_cast<size_t>(r) * kpad + ch * CC + cio;
      bf16x8 Bn[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        Bn[nb] = *reinterpret_cast<const bf16x8*>(wlane + static_cast<size_t>(nb * 16) * kpad + tsub * CIN);
#pragma unroll 3
      for (int s = 0; s < NS; ++s) {
        const int tap = s * TPS + tsub;
        const bool tap_ok = tap < 27;
        const int tt = tap_ok ? tap : 26;
        const int tx = tt / 9, ty = (tt / 3) % 3, tz = tt % 3;
        const bf16* abase = halo + ((wave + tx) * kHY * kHZ + ty * kHZ + r + tz) * VS + cio;
        bf16x8 B[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) B[nb] = Bn[nb];
        if (s + 1 < NS) {
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            Bn[nb] = *reinterpret_cast<const bf16x8*>(wlane + static_cast<size_t>(nb * 16) * kpad + (tap + TPS) * CIN);
        }
        bf16x8 A[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          bf16x8 a = *reinterpret_cast<const bf16x8*>(abase + mt * kHZ * VS);
          if (!tap_ok) {
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = static_cast<bf16>(0.f);
          }
          A[mt] = a;
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
          for (int mt = 0; mt < 4; ++mt)
            acc[mt][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt], B[nb], acc[mt][nb], 0, 0, 0);
        }
      }
    }
  }
  // BF16 outputs with whole 8-channel groups: each wave stages its 4 x 16 voxels x 16 NB channels in the (now free)
  // halo buffer and writes them as 16-byte rows; every wave takes both barriers.
  constexpr int CO = 16 * NB;
  constexpr bool kStage = 4 * 64 * CO <= kHalo * VS;
  if (kStage && outf == nullptr && (cout & 7) == 0) {
    __syncthreads();  // every wave is done reading the halo
    bf16* st = halo + wave * (64 * CO);
    if (wave_on) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int co = nb * 16 + r;
        const float b = (bias && co < cout) ? bias[co] : 0.f;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float val = acc[mt][nb][j] + b;
            st[(mt * 16 + g * 4 + j) * CO + co] = static_cast<bf16>(act ? leaky(val) : val);
          }
      }
    }
    __syncthreads();
    if (!wave_on) return;
    const int x = x0 + wave, ng = cout / 8;
    for (int c = lane; c < 64 * ng; c += 64) {
      const int row = c / ng, q = c - row * ng;
      const int y = y0 + row / 16, z = z0 + row % 16;
      if (y < D && z < D) {
        const size_t v = static_cast<size_t>((x * D + y) * D + z);
        bf16x8 val = *reinterpret_cast<const bf16x8*>(st + row * CO + 8 * q);
        if (8 * q < mask_ch) {  // leaky-ReLU gradient, rounded as a separate pass over the stored values would be
          const bf16x8 a = *reinterpret_cast<const bf16x8*>(mask.p + v * mask.ld + mask.off + 8 * q);
#pragma unroll
          for (int j = 0; j < 8; ++j)
            if (!(f(a[j]) > 0.f)) val[j] = static_cast<bf16>(kSlope * f(val[j]));
        }
        *reinterpret_cast<bf16x8*>(out.p + v * out.ld + out.off + 8 * q) = val;
      }
    }
    return;
  }
  if (!wave_on) return;
  const int x = x0 + wave;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int co = nb * 16 + r;
    if (co >= cout) continue;
    const float b = bias ? bias[co] : 0.f;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const int y = y0 + mt;
      if (y >= D) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int z = z0 + g * 4 + j;
        if (z >= D) continue;
        const size_t v = static_cast<size_t>((x * D + y) * D + z);
        const float val = acc[mt][nb][j] + b;
        if (outf) {
          outf[v * cout + co] = val;
        } else {
          bf16 o = static_cast<bf16>(act ? leaky(val) : val);
          if (co < mask_ch && !(f(mask.p[v * mask.ld + mask.off + co]) > 0.f)) o = static_cast<bf16>(kSlope * f(o));
          out.p[v * out.ld + out.off + co] = o;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------------------------------------------
// 2^3 down / up layers as GEMMs on v_mfma_f32_16x16x32_bf16 (FP32 accumulation): a wave takes 16 coarse voxels (the
// rows). The FP32 canonical weights W[o][t][i] are rounded to BF16 as each B fragment is loaded (8 consecutive input
// channels of one (o, t) per lane). Outputs get the bias and the leaky ReLU and are stored as BF16.
__device__ __forceinline__ bf16x8 weight_frag(const float* __restrict__ w) {
  const float4 u = *reinterpret_cast<const float4*>(w), v = *reinterpret_cast<const float4*>(w + 4);
  bf16x8 r;
  r[0] = static_cast<bf16>(u.x);
  r[1] = static_cast<bf16>(u.y);
  r[2] = static_cast<bf16>(u.z);
  r[3] = static_cast<bf16>(u.w);
  r[4] = static_cast<bf16>(v.x);
  r[5] = static_cast<bf16>(v.y);
  r[6] = static_cast<bf16>(v.z);
  r[7] = static_cast<bf16>(v.w);
  return r;
}

__device__ __forceinline__ int fine_voxel(int y, int Dc, int t) {  // voxel 2 y + t of the (2 Dc)^3 grid
  const int yx = y / (Dc * Dc), yy = (y / Dc) % Dc, yz = y % Dc, Df = 2 * Dc;
  return ((2 * yx + (t >> 2)) * Df + 2 * yy + ((t >> 1) & 1)) * Df + 2 * yz + (t & 1);
}

// Each wave stages its BF16 outputs in its own LDS region and then writes them as 16-byte rows of 8 channels (a lane
// of the MFMA result holds one channel of four voxels). The kernels keep every wave to the barriers: a wave past the
// end of the grid only skips its loads and stores.

// out[y][o] = leaky(b[o] + sum_{t, i} W[o][t][i] x[2y + t][i])   (x on D^3, y on (D/2)^3): K = 8 CIN as (t, i).
// DG: the data gradient of a 2^3 up layer, the same product without bias and activation (W its weights transposed).
template <int CIN, int COUT, bool DG>
__global__ __launch_bounds__(kNT) void k_down2(View x, const float* __restrict__ W, const float* __restrict__ b,
                                               View out, int D, View mask, int mask_ch) {
  static_assert(CIN % 8 == 0 && COUT % 16 == 0, "fragment shapes");
  constexpr int KS = 8 * CIN / 32, NBLK = COUT / 16;
  __shared__ bf16 stage[4][16 * COUT];
  const int Dc = D / 2, Vc = Dc * Dc * Dc;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int y0 = (blockIdx.x * 4 + wave) * 16;
  const int y = y0 + r;
  const bool row_ok = y < Vc;
  f32x4 acc[NBLK];
#pragma unroll
  for (int nb = 0; nb < NBLK; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int k = 32 * ks + 8 * g, t = k / CIN, i0 = k % CIN;
    bf16x8 a;
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = static_cast<bf16>(0.f);
    if (row_ok)
      a = *reinterpret_cast<const bf16x8*>(x.p + static_cast<size_t>(fine_voxel(y, Dc, t)) * x.ld + x.off + i0);
#pragma unroll
    for (int nb = 0; nb < NBLK; ++nb) {
      const int o = nb * 16 + r;
      acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, weight_frag(W + (o * 8 + t) * CIN + i0), acc[nb], 0, 0, 0);
    }
  }
  bf16* st = stage[wave];
#pragma unroll
  for (int nb = 0; nb < NBLK; ++nb) {
    const int o = nb * 16 + r;
    const float bo = DG ? 0.f : b[o];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      st[(4 * g + j) * COUT + o] = static_cast<bf16>(DG ? acc[nb][j] : leaky(acc[nb][j] + bo));
  }
  __syncthreads();
  constexpr int NCH = 16 * COUT / 8;  // 16-byte chunks of the wave's rows
#pragma unroll
  for (int c = lane; c < NCH; c += 64) {
    const int row = c / (COUT / 8), q8 = c % (COUT / 8);
    const int yr = y0 + row;
    if (yr < Vc) {
      bf16x8 val = *reinterpret_cast<const bf16x8*>(st + row * COUT + 8 * q8);
      if (DG && 8 * q8 < mask_ch) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(mask.p + static_cast<size_t>(yr) * mask.ld + mask.off + 8 * q8);
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (!(f(a[j]) > 0.f)) val[j] = static_cast<bf16>(kSlope * f(val[j]));
      }
      *reinterpret_cast<bf16x8*>(out.p + static_cast<size_t>(yr) * out.ld + out.off + 8 * q8) = val;
    }
  }
}

// out[2y + t][o] = leaky(b[o] + sum_i W[o][t][i] x[y][i])   (x on D^3, out on (2D)^3): N = 8 COUT as (t, o).
// DG: the data gradient of a 2^3 down layer, the same product without bias and activation (W its weights transposed),
// added to what out holds when accumulate is set.
template <int CIN, int COUT, bool DG>
__global__ __launch_bounds__(kNT) void k_up2(View x, const float* __restrict__ W, const float* __restrict__ b,
                                             View out, int D, int accumulate, View mask, int mask_ch) {
  static_assert(CIN % 32 == 0 && COUT % 16 == 0, "fragment shapes");
  constexpr int KS = CIN / 32, NBLK = 8 * COUT / 16;
  __shared__ bf16 stage[4][16 * 8 * COUT];  // [coarse row][tap][channel] per wave
  const int V = D * D * D;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int y0 = (blockIdx.x * 4 + wave) * 16;
  const int y = y0 + r;
  bf16x8 A[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
    for (int j = 0; j < 8; ++j) A[ks][j] = static_cast<bf16>(0.f);
    if (y < V) A[ks] = *reinterpret_cast<const bf16x8*>(x.p + static_cast<size_t>(y) * x.ld + x.off + 32 * ks + 8 * g);
  }
  bf16* st = stage[wave];
#pragma unroll 2
  for (int nb = 0; nb < NBLK; ++nb) {
    const int n = nb * 16 + r, t = n / COUT, o = n % COUT;  // t is uniform over the block (COUT >= 16)
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ks], weight_frag(W + (o * 8 + t) * CIN + 32 * ks + 8 * g), acc,
                                                    0, 0, 0);
    const float bo = DG ? 0.f : b[o];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      st[((4 * g + j) * 8 + t) * COUT + o] = static_cast<bf16>(DG ? acc[j] : leaky(acc[j] + bo));
  }
  __syncthreads();
  constexpr int NCH = 16 * 8 * COUT / 8;  // 16-byte chunks: (coarse row, tap, channel group)
#pragma unroll
  for (int c = lane; c < NCH; c += 64) {
    const int row = c / (8 * COUT / 8), rest = c % (8 * COUT / 8), t = rest / (COUT / 8), q8 = rest % (COUT / 8);
    const int yr = y0 + row;
    if (yr < V) {
      bf16x8* dst =
          reinterpret_cast<bf16x8*>(out.p + static_cast<size_t>(fine_voxel(yr, D, t)) * out.ld + out.off + 8 * q8);
      bf16x8 val = *reinterpret_cast<const bf16x8*>(st + (row * 8 + t) * COUT + 8 * q8);
      if (DG && accumulate) {
        const bf16x8 old = *dst;
#pragma unroll
        for (int j = 0; j < 8; ++j) val[j] = static_cast<bf16>(f(old[j]) + f(val[j]));
      }
      if (DG && 8 * q8 < mask_ch) {
        const size_t fv = static_cast<size_t>(fine_voxel(yr, D, t));
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(mask.p + fv * mask.ld + mask.off + 8 * q8);
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (!(f(a[j]) > 0.f)) val[j] = static_cast<bf16>(kSlope * f(val[j]));
      }
      *dst = val;
    }
  }
}

// Wt[i][t][o] = W[o][t][i] for a 2^3 layer (the weights of its data gradient)
__global__ __launch_bounds__(kNT) void k_transpose2(const float* __restrict__ W, int cout, int cin,
                                                    float* __restrict__ Wt) {
  const int e = blockIdx.x * kNT + threadIdx.x;
  if (e >= cout * 8 * cin) return;
  const int o = e / (8 * cin), t = (e / cin) % 8, i = e % cin;
  Wt[(i * 8 + t) * cout + o] = W[e];
}

// ---------------------------------------------------------------------------------------------------------------
// Weight gradient of a 3^3 layer on the vector ALUs, for grids that are not a multiple of 32 per side (the MFMA
// kernels below take the rest). Workgroup (chunk, tap) sums dz[p][o] x[p + d_tap][i] over the output voxels p of its
// chunk, for every (o, i); tap 0 also sums dz[p][o] for the bias. Voxels, tiles of kTV, are staged in LDS as FP32;
// thread groups take interleaved voxels of a tile and are reduced in LDS at the end.
constexpr int kTV = 64;
constexpr int kMaxC = 64;

__device__ __forceinline__ int conv3_neighbour(int p, int tap, int D) {  // periodic voxel p + d_tap
  const int px = p / (D * D), py = (p / D) % D, pz = p % D;
  const int x = wrapi(px + tap / 9 - 1, D), y = wrapi(py + (tap / 3) % 3 - 1, D), z = wrapi(pz + tap % 3 - 1, D);
  return (x * D + y) * D + z;
}

template <int CI>
__global__ __launch_bounds__(kNT) void k_wgrad(View x, int cin, int cin_real, View dz, int cout, int D,
                                               float* __restrict__ partial) {
  constexpr int ntap = 27;
  const int nbase = D * D * D;
  __shared__ float sdz[kTV * kMaxC];
  __shared__ float sx[kTV * kMaxC];
  __shared__ int sxv[kTV], szv[kTV];
  const int chunk = blockIdx.x, tap = blockIdx.y, nchunk = gridDim.x;
  const int tid = threadIdx.x;
  const int ncb = cin / CI;
  const int npb = cout * ncb;           // (o, ci-block) pairs
  const int G = kNT / npb;              // thread groups over voxels
  const int pb = tid % npb, grp = tid / npb;
  const bool active = grp < G;
  const int o = pb / ncb, cb = pb % ncb;
  float acc[CI];
#pragma unroll
  for (int c = 0; c < CI; ++c) acc[c] = 0.f;
  float accb = 0.f;
  const int64_t per = (static_cast<int64_t>(nbase) + nchunk - 1) / nchunk;
  const int b0 = static_cast<int>(per * chunk);
  const int b1 = static_cast<int>(std::min<int64_t>(nbase, per * (chunk + 1)));
  const int gz = (cout + 7) / 8, gx = cin / 8;  // 16-byte groups per voxel (dz views are zero-padded to 8 channels)
  for (int t0 = b0; t0 < b1; t0 += kTV) {
    const int nv = min(kTV, b1 - t0);
    __syncthreads();
    if (tid < nv) {
      sxv[tid] = conv3_neighbour(t0 + tid, tap, D);
      szv[tid] = t0 + tid;
    }
    __syncthreads();
    for (int e = tid; e < nv * (gz + gx); e += kNT) {
      const int v = e / (gz + gx), q = e % (gz + gx);
      if (q < gz) {
        const bf16x8 u = *reinterpret_cast<const bf16x8*>(dz.p + static_cast<size_t>(szv[v]) * dz.ld + dz.off + 8 * q);
#pragma unroll
        for (int j = 0; j < 8; ++j) sdz[v * kMaxC + 8 * q + j] = f(u[j]);
      } else {
        const int qq = q - gz;
        const bf16x8 u = *reinterpret_cast<const bf16x8*>(x.p + static_cast<size_t>(sxv[v]) * x.ld + x.off + 8 * qq);
#pragma unroll
        for (int j = 0; j < 8; ++j) sx[v * kMaxC + 8 * qq + j] = f(u[j]);
      }
    }
    __syncthreads();
    if (active) {
      for (int v = grp; v < nv; v += G) {
        const float z = sdz[v * kMaxC + o];
        const float* xp = sx + v * kMaxC + cb * CI;
#pragma unroll
        for (int c = 0; c < CI; ++c) acc[c] += z * xp[c];
        accb += z;
      }
    }
  }
  // reduce the thread groups one after another into the (no longer needed) staging buffers
  __syncthreads();
  float* red = sx;
  const int slice = npb * CI;
  for (int gg = 0; gg < G; ++gg) {
    if (active && grp == gg) {
#pragma unroll
      for (int c = 0; c < CI; ++c) red[pb * CI + c] = (gg == 0 ? 0.f : red[pb * CI + c]) + acc[c];
      sdz[pb] = (gg == 0 ? 0.f : sdz[pb]) + accb;
    }
    __syncthreads();
  }
  // canonical layout W[o][t][i] over the real input channels, then the bias (each (o, cb) pair summed dz[o]; take
  // the cb == 0 one)
  const int nW = cout * ntap * cin_real;
  float* dst = partial + static_cast<size_t>(chunk) * (nW + cout);
  for (int e = tid; e < slice; e += kNT) {
    const int p = e / CI, c = e % CI;
    const int oo = p / ncb, ci = (p % ncb) * CI + c;
    if (ci < cin_real) dst[(oo * ntap + tap) * cin_real + ci] = red[e];
  }
  if (tap == 0)
    for (int e = tid; e < cout; e += kNT) dst[nW + e] = sdz[e * ncb];
}

// Weight gradient of a 3^3 layer on v_mfma_f32_16x16x32_bf16, for D a multiple of 32: dW[o][t][i] =
// sum_p dz[p][o] x[p + d_t][i] is a product whose k index is the voxel p. A workgroup takes one 16 (o) x 16 (i) tile
// of all 27 taps over a range of bricks of 4 x 4 x 32 output voxels. Per brick it stages dz (16 rows of 32 z) and the
// periodic x halo (6 x 6 rows of 34 z) in LDS channel-major with z contiguous, two BF16 of neighbouring z per dword,
// so a lane's 8 consecutive k (8 consecutive z of one row) are one 16-byte read. A tap's z offset (0, 1 or 2 halo
// elements) is applied in registers: the lane reads halo z 8 g .. 8 g + 9 once per (x, y) offset and takes its 8
// values by dword selection (offsets 0 and 2) or a 16-bit funnel shift (offset 1), so the three z taps share the
// reads. Wave w takes the brick rows at x = x0 + w (y = y0 + 0..3) and holds all 27 16 x 16 FP32 tiles; the four waves
// and, for the bias, the four lane groups are summed in a fixed order at the end.
constexpr int kWB = 32;                    // z extent of a brick: one K step
constexpr int kWRow = 20;                  // halo row pitch in dwords (17 used; a multiple of 4 for 16-byte reads)
constexpr int kWXC = 36 * kWRow + 20;      // halo channel pitch in dwords, = 4 mod 32: 8 lanes' 16-byte reads hit
constexpr int kWZC = 16 * 16 + 4;          // dz channel pitch in dwords (16 rows x 16), = 4 mod 32   distinct banks

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned half16(const u32x4& w, int j) {
  return (j & 1) ? (w[j >> 1] >> 16) : (w[j >> 1] & 0xffffu);
}
__device__ __forceinline__ unsigned funnel16(unsigned lo, unsigned hi) { return (lo >> 16) | (hi << 16); }
__device__ __forceinline__ float bf16_bits(unsigned h) { return __uint_as_float(h << 16); }

bool wgrad3_mfma(int kind, int D) { return kind == 0 && D >= kWB && D % kWB == 0; }

__global__ __launch_bounds__(kNT, 2) void k_wgrad3(View x, int cin, int cin_real, View dz, int cout, int D, int nchunk,
                                                   float* __restrict__ partial) {
  __shared__ __attribute__((aligned(16))) unsigned sx[16 * kWXC];
  __shared__ __attribute__((aligned(16))) unsigned sz[16 * kWZC];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c16 = lane & 15, g = lane >> 4;
  const int chunk = blockIdx.x;
  const int nib = (cin + 15) / 16;
  const int ob = blockIdx.y / nib, ib = blockIdx.y % nib;
  const int coutp = (cout + 7) & ~7;
  const int nb4 = D / 4, nbz = D / kWB;
  const int nbrick = nb4 * nb4 * nbz;
  const int per = (nbrick + nchunk - 1) / nchunk;
  const int k0 = per * chunk, k1 = min(nbrick, k0 + per);
  f32x4 acc[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  const bool do_bias = ib == 0;
  // Staging items of a thread: dz (8-channel group q, row r, z pair p), items tid and tid + 256; x halo (group q,
  // halo row hr = 6 hx + hy, z pair p; halo z 2 p, 2 p + 1 is voxel z0 - 1 + halo z), items tid + 256 m < 1224.
  // The next brick's items are loaded into registers before the current brick's MFMAs and written to LDS after them.
  constexpr int kHI = 2 * 36 * 17, kHM = (kHI + kNT - 1) / kNT;
  u32x4 rz[2][2], rh[kHM][2];
  auto load = [&](int k) {
    const int bzi = k % nbz, byi = (k / nbz) % nb4, bxi = k / (nbz * nb4);
    const int x0 = 4 * bxi, y0 = 4 * byi, z0 = kWB * bzi;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int e = tid + m * kNT;
      const int q = e >> 8, r = (e >> 4) & 15, p = e & 15;
      const int ch = 16 * ob + 8 * q;
      rz[m][0] = rz[m][1] = u32x4{0u, 0u, 0u, 0u};
      if (ch < coutp) {  // channels at or past coutp stay zero
        const size_t vox = (static_cast<size_t>(x0 + (r >> 2)) * D + (y0 + (r & 3))) * D + z0 + 2 * p;
        rz[m][0] = *reinterpret_cast<const u32x4*>(dz.p + vox * dz.ld + dz.off + ch);
        rz[m][1] = *reinterpret_cast<const u32x4*>(dz.p + (vox + 1) * dz.ld + dz.off + ch);
      }
    }
#pragma unroll
    for (int m = 0; m < kHM; ++m) {
      const int e = tid + m * kNT;
      rh[m][0] = rh[m][1] = u32x4{0u, 0u, 0u, 0u};
      if (e < kHI) {
        const int q = e / (36 * 17), rem = e - q * (36 * 17), hr = rem / 17, p = rem - hr * 17;
        const int ch = 16 * ib + 8 * q;
        if (ch < cin) {
          const int gx = wrapi(x0 - 1 + hr / 6, D), gy = wrapi(y0 - 1 + hr % 6, D);
          const size_t row = (static_cast<size_t>(gx) * D + gy) * D;
          const size_t v0 = row + wrapi(z0 - 1 + 2 * p, D), v1 = row + wrapi(z0 + 2 * p, D);
          rh[m][0] = *reinterpret_cast<const u32x4*>(x.p + v0 * x.ld + x.off + ch);
          rh[m][1] = *reinterpret_cast<const u32x4*>(x.p + v1 * x.ld + x.off + ch);
        }
      }
    }
  };
  if (k0 < k1) load(k0);
  for (int k = k0; k < k1; ++k) {
    __syncthreads();  // the previous brick's reads are done
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int e = tid + m * kNT;
      const int q = e >> 8, r = (e >> 4) & 15, p = e & 15;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        sz[(8 * q + j) * kWZC + r * 16 + p] = half16(rz[m][0], j) | (half16(rz[m][1], j) << 16);
    }
#pragma unroll
    for (int m = 0; m < kHM; ++m) {
      const int e = tid + m * kNT;
      if (e < kHI) {
        const int q = e / (36 * 17), rem = e - q * (36 * 17), hr = rem / 17, p = rem - hr * 17;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          sx[(8 * q + j) * kWXC + hr * kWRow + p] = half16(rh[m][0], j) | (half16(rh[m][1], j) << 16);
      }
    }
    __syncthreads();
    if (k + 1 < k1) load(k + 1);
    for (int ry = 0; ry < 4; ++ry) {
      const int r = wave * 4 + ry;
      const u32x4 a = *reinterpret_cast<const u32x4*>(sz + c16 * kWZC + r * 16 + 4 * g);
      if (do_bias) {
#pragma unroll
        for (int d = 0; d < 4; ++d) bsum += bf16_bits(a[d] & 0xffffu) + bf16_bits(a[d] >> 16);
      }
      const bf16x8 A = __builtin_bit_cast(bf16x8, a);
#pragma unroll
      for (int txy = 0; txy < 9; ++txy) {
        const int tx = txy / 3, ty = txy % 3;
        const unsigned* src = sx + c16 * kWXC + ((wave + tx) * 6 + ry + ty) * kWRow + 4 * g;
        const u32x4 q0 = *reinterpret_cast<const u32x4*>(src);
        const unsigned q4 = src[4];
        const u32x4 b1 = u32x4{funnel16(q0[0], q0[1]), funnel16(q0[1], q0[2]), funnel16(q0[2], q0[3]),
                               funnel16(q0[3], q4)};
        const u32x4 b2 = u32x4{q0[1], q0[2], q0[3], q4};
        acc[3 * txy + 0] =
            __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, __builtin_bit_cast(bf16x8, q0), acc[3 * txy + 0], 0, 0, 0);
        acc[3 * txy + 1] =
            __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, __builtin_bit_cast(bf16x8, b1), acc[3 * txy + 1], 0, 0, 0);
        acc[3 * txy + 2] =
            __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, __builtin_bit_cast(bf16x8, b2), acc[3 * txy + 2], 0, 0, 0);
      }
    }
  }
  // sum the waves in order into LDS (the staging buffers are free now), then write this tile of the chunk's partial
  __syncthreads();
  float* red = reinterpret_cast<float*>(sx);
  float* rb = reinterpret_cast<float*>(sz);
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int t = 0; t < 27; ++t) {
        f32x4* cell = reinterpret_cast<f32x4*>(red + (t * 64 + lane) * 4);
        *cell = (w == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : *cell) + acc[t];
      }
      rb[lane] = (w == 0 ? 0.f : rb[lane]) + bsum;
    }
    __syncthreads();
  }
  const int nW = cout * 27 * cin_real;
  float* dst = partial + static_cast<size_t>(chunk) * (nW + cout);
  for (int e = tid; e < 27 * 256; e += kNT) {
    const int t = e >> 8, ln = (e >> 2) & 63, j = e & 3;
    const int o = 16 * ob + 4 * (ln >> 4) + j, i = 16 * ib + (ln & 15);
    if (o < cout && i < cin_real) dst[(o * 27 + t) * cin_real + i] = red[e];
  }
  if (do_bias && tid < 16) {
    const int o = 16 * ob + tid;
    if (o < cout) dst[nW + o] = ((rb[tid] + rb[16 + tid]) + rb[32 + tid]) + rb[48 + tid];
  }
}

// Weight gradient of a 2^3 layer on v_mfma_f32_16x16x32_bf16: dW[o][t][i] = sum_y dz[.][o] x[.][i] over the coarse
// voxels y, with dz at y and x at 2 y + t (down layer) or dz at 2 y + t and x at y (up layer). A workgroup takes one
// 16 (o) x 16 (i) tile of all 8 taps over a range of blocks of 128 coarse voxels. Per block it stages the operand that
// depends on the tap (8 taps x 16 channels) and the one that does not (16 channels) in LDS channel-major, two BF16 of
// neighbouring y per dword, zero past the last voxel. Wave w takes the K step of voxels 32 w .. 32 w + 31 of the block.
// The bias (per tap for the up layer) is summed from the dz operand; waves and lane groups are summed in a fixed order.
constexpr int kW2Y = 128;                // coarse voxels per block
constexpr int kW2P = kW2Y / 2 + 4;       // channel pitch in dwords, = 4 mod 32

__global__ __launch_bounds__(kNT, 2) void k_wgrad2(int kind, View x, int cin, int cin_real, View dz, int cout, int D,
                                                   int nchunk, float* __restrict__ partial) {
  __shared__ __attribute__((aligned(16))) unsigned st[8 * 16 * kW2P];  // the operand at 2 y + t
  __shared__ __attribute__((aligned(16))) unsigned su[16 * kW2P];      // the operand at y
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c16 = lane & 15, g = lane >> 4;
  const int nib = (cin + 15) / 16;
  const int ob = blockIdx.y / nib, ib = blockIdx.y % nib;
  const int coutp = (cout + 7) & ~7;
  const bool down = kind == 1;
  const int Dc = down ? D / 2 : D;  // coarse grid side
  const int nbase = Dc * Dc * Dc;
  const int nblk = (nbase + kW2Y - 1) / kW2Y;
  const int per = (nblk + nchunk - 1) / nchunk;
  const int k0 = per * blockIdx.x, k1 = min(nblk, k0 + per);
  const View vt = down ? x : dz, vu = down ? dz : x;
  const int cht = down ? 16 * ib : 16 * ob, chu = down ? 16 * ob : 16 * ib;
  const int mt = down ? cin : coutp, mu = down ? coutp : cin;
  const bool do_bias = ib == 0;
  f32x4 acc[8];
  float bs[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    bs[t] = 0.f;
  }
  // Staging items of a thread: the tap operand (tap t, group q, voxel pair p) for items tid + 256 m, m < 4; the other
  // operand (group q, voxel pair p) for item tid < 128. The next block's items are loaded into registers before the
  // current block's MFMAs and written to LDS after them.
  constexpr int kTM = 8 * 2 * (kW2Y / 2) / kNT;
  u32x4 rt[kTM][2], ru[2];
  auto load = [&](int k) {
    const int y0 = k * kW2Y;
#pragma unroll
    for (int m = 0; m < kTM; ++m) {
      const int e = tid + m * kNT;
      const int t = e >> 7, q = (e >> 6) & 1, p = e & 63;
      const int ch = cht + 8 * q, y = y0 + 2 * p;
      rt[m][0] = rt[m][1] = u32x4{0u, 0u, 0u, 0u};
      if (ch < mt) {
        if (y < nbase)
          rt[m][0] =
              *reinterpret_cast<const u32x4*>(vt.p + static_cast<size_t>(fine_voxel(y, Dc, t)) * vt.ld + vt.off + ch);
        if (y + 1 < nbase)
          rt[m][1] = *reinterpret_cast<const u32x4*>(vt.p + static_cast<size_t>(fine_voxel(y + 1, Dc, t)) * vt.ld +
                                                     vt.off + ch);
      }
    }
    ru[0] = ru[1] = u32x4{0u, 0u, 0u, 0u};
    if (tid < 2 * (kW2Y / 2)) {
      const int q = tid >> 6, p = tid & 63;
      const int ch = chu + 8 * q, y = y0 + 2 * p;
      if (ch < mu) {
        if (y < nbase) ru[0] = *reinterpret_cast<const u32x4*>(vu.p + static_cast<size_t>(y) * vu.ld + vu.off + ch);
        if (y + 1 < nbase)
          ru[1] = *reinterpret_cast<const u32x4*>(vu.p + static_cast<size_t>(y + 1) * vu.ld + vu.off + ch);
      }
    }
  };
  if (k0 < k1) load(k0);
  for (int k = k0; k < k1; ++k) {
    __syncthreads();  // the previous block's reads are done
#pragma unroll
    for (int m = 0; m < kTM; ++m) {
      const int e = tid + m * kNT;
      const int t = e >> 7, q = (e >> 6) & 1, p = e & 63;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        st[(t * 16 + 8 * q + j) * kW2P + p] = half16(rt[m][0], j) | (half16(rt[m][1], j) << 16);
    }
    if (tid < 2 * (kW2Y / 2)) {
      const int q = tid >> 6, p = tid & 63;
#pragma unroll
      for (int j = 0; j < 8; ++j) su[(8 * q + j) * kW2P + p] = half16(ru[0], j) | (half16(ru[1], j) << 16);
    }
    __syncthreads();
    if (k + 1 < k1) load(k + 1);
    const int dw = 16 * wave + 4 * g;
    const u32x4 fu = *reinterpret_cast<const u32x4*>(su + c16 * kW2P + dw);
    if (down && do_bias) {
#pragma unroll
      for (int d = 0; d < 4; ++d) bs[0] += bf16_bits(fu[d] & 0xffffu) + bf16_bits(fu[d] >> 16);
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const u32x4 ft = *reinterpret_cast<const u32x4*>(st + (t * 16 + c16) * kW2P + dw);
      if (!down && do_bias) {
#pragma unroll
        for (int d = 0; d < 4; ++d) bs[t] += bf16_bits(ft[d] & 0xffffu) + bf16_bits(ft[d] >> 16);
      }
      // A is dz (rows o), B is x (columns i)
      const bf16x8 A = __builtin_bit_cast(bf16x8, down ? fu : ft), B = __builtin_bit_cast(bf16x8, down ? ft : fu);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, acc[t], 0, 0, 0);
    }
  }
  __syncthreads();
  float* red = reinterpret_cast<float*>(st);
  float* rb = reinterpret_cast<float*>(su);
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        f32x4* cell = reinterpret_cast<f32x4*>(red + (t * 64 + lane) * 4);
        *cell = (w == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : *cell) + acc[t];
        rb[t * 64 + lane] = (w == 0 ? 0.f : rb[t * 64 + lane]) + bs[t];
      }
    }
    __syncthreads();
  }
  const int nslot = down ? 1 : 8;
  const int nW = cout * 8 * cin_real;
  float* dst = partial + static_cast<size_t>(blockIdx.x) * (nW + nslot * cout);
  for (int e = tid; e < 8 * 256; e += kNT) {
    const int t = e >> 8, ln = (e >> 2) & 63, j = e & 3;
    const int o = 16 * ob + 4 * (ln >> 4) + j, i = 16 * ib + (ln & 15);
    if (o < cout && i < cin_real) dst[(o * 8 + t) * cin_real + i] = red[e];
  }
  if (do_bias && tid < 16 * nslot) {
    const int t = tid >> 4, c = tid & 15, o = 16 * ob + c;
    const float* b = rb + t * 64;
    if (o < cout) dst[nW + t * cout + o] = ((b[c] + b[16 + c]) + b[32 + c]) + b[48 + c];
  }
}

// grad[j] = sum over chunks (and, for the bias, over its nslot slots) of the partial sums, in a fixed order: a block
// of kRW waves takes 64 outputs, wave q sums the chunks c = q mod kRW, and the wave sums are added in order.
constexpr int kRW = 16;
__global__ __launch_bounds__(64 * kRW) void k_reduce(const float* __restrict__ partial, int nchunk, int nW, int cout,
                                                     int nslot, float* __restrict__ grad) {
  __shared__ float part[kRW][64];
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  const size_t stride = static_cast<size_t>(nW) + static_cast<size_t>(nslot) * cout;
  float s = 0.f;
  if (j < nW) {
    for (int c = q; c < nchunk; c += kRW) s += partial[c * stride + j];
  } else if (j < nW + cout) {
    for (int c = q; c < nchunk; c += kRW)
      for (int k = 0; k < nslot; ++k) s += partial[c * stride + nW + k * cout + (j - nW)];
  }
  part[q][lane] = s;
  __syncthreads();
  if (q == 0 && j < nW + cout) {
    float t = part[0][lane];
#pragma unroll
    for (int w = 1; w < kRW; ++w) t += part[w][lane];
    grad[j] = t;
  }
}

// ---------------------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kNT) void k_convert_conv3(const float* __restrict__ W, int cout, int cin,
                                                       bf16* __restrict__ wf, int cinp, int nbo, int kpad,
                                                       bf16* __restrict__ wb, int coutp, int nbi, int kpadb) {
  const int64_t nf = static_cast<int64_t>(16 * nbo) * kpad, nbk = static_cast<int64_t>(16 * nbi) * kpadb;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (idx < nf) {
    const int row = static_cast<int>(idx / kpad), k = static_cast<int>(idx % kpad);
    const int t = k / cinp, ci = k % cinp;
    float v = 0.f;
    if (row < cout && t < 27 && ci < cin) v = W[(row * 27 + t) * cin + ci];
    wf[idx] = static_cast<bf16>(v);
  } else if (idx < nf + nbk) {
    const int64_t j = idx - nf;
    const int row = static_cast<int>(j / kpadb), k = static_cast<int>(j % kpadb);
    const int t = k / coutp, o = k % coutp;
    float v = 0.f;
    if (row < cin && t < 27 && o < cout) v = W[(o * 27 + (26 - t)) * cin + row];
    wb[j] = static_cast<bf16>(v);
  }
}

// one thread per voxel: six FP32 features in, one 16-byte row of eight BF16 channels out
__global__ __launch_bounds__(kNT) void k_pack_input(const float* __restrict__ feat, bf16* __restrict__ x, int V) {
  const int64_t v = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (v >= V) return;
  const float* src = feat + v * kInputChannels;
  bf16x8 u;
#pragma unroll
  for (int c = 0; c < 8; ++c) u[c] = static_cast<bf16>(c < kInputChannels ? src[c] : 0.f);
  *reinterpret_cast<bf16x8*>(x + v * 8) = u;
}

__global__ __launch_bounds__(kNT) void k_loss_grad(const float* __restrict__ out, const float* __restrict__ target,
                                                   bf16* __restrict__ dout, double* __restrict__ part, int V) {
  __shared__ double sh[kNT];
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  double sq = 0.0;
  if (idx < static_cast<int64_t>(V) * 8) {
    const int64_t v = idx / 8;
    const int c = static_cast<int>(idx % 8);
    float g = 0.f;
    if (c < 3) {
      const float e = out[v * 3 + c] - target[v * 3 + c];
      sq = static_cast<double>(e) * e;
      g = 2.0f * e / (3.0f * static_cast<float>(V));
    }
    dout[idx] = static_cast<bf16>(g);
  }
  sh[threadIdx.x] = sq;
  __syncthreads();
  for (int off = kNT / 2; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// omb1 = 1 - beta1 and omb2 = 1 - beta2 come rounded from FP64 (1 - 0.999f in FP32 would be 1.3e-5 off).
__global__ __launch_bounds__(kNT) void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, int64_t count, float lr, float b1,
                                              float omb1, float b2, float omb2, float eps, float c1, float c2) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + omb1 * gi;
  const float vi = b2 * v[i] + omb2 * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// PACK: write the six features of the apply path (ref == NULL, psi1 given) straight into the network's BF16 input
// row x[id][0..8) (channels 6, 7 zero), rounded as the FP32 grid would be by pack_input.
template <bool PACK>
__global__ __launch_bounds__(kNT) void k_features(const float* __restrict__ pos, const int32_t* __restrict__ id,
                                                  int64_t n, const float* __restrict__ ref,
                                                  const float* __restrict__ psi1, int N, double box,
                                                  float* __restrict__ out, int ld, bf16* __restrict__ xpack,
                                                  int* __restrict__ flags) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (p >= n) return;
  const int64_t q = id[p];
  const int64_t V = static_cast<int64_t>(N) * N * N;
  if (q < 0 || q >= V) {
    atomicOr(flags, 1);
    return;
  }
  const double dp = box / N;
  const int64_t ijk[3] = {q / (static_cast<int64_t>(N) * N), (q / N) % N, q % N};
  float fv[6];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double base = ref ? static_cast<double>(ref[d * n + p]) : (static_cast<double>(ijk[d]) + 0.5) * dp;
    double dd = static_cast<double>(pos[d * n + p]) - base;
    dd -= box * rint(dd / box);
    fv[d] = static_cast<float>(dd / dp);
    fv[3 + d] = psi1 ? static_cast<float>(static_cast<double>(psi1[d * n + p]) / dp) : 0.f;
  }
  if constexpr (PACK) {
    bf16x8 u;
#pragma unroll
    for (int c = 0; c < 8; ++c) u[c] = static_cast<bf16>(c < kInputChannels ? fv[c] : 0.f);
    *reinterpret_cast<bf16x8*>(xpack + q * 8) = u;
  } else {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      out[q * ld + d] = fv[d];
      if (psi1) out[q * ld + 3 + d] = fv[3 + d];
    }
  }
}

__global__ __launch_bounds__(kNT) void k_apply(float* __restrict__ pos, const int32_t* __restrict__ id, int64_t n,
                                               const float* __restrict__ r, int N, float dp, float box,
                                               int* __restrict__ flags) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (p >= n) return;
  const int64_t q = id[p];
  if (q < 0 || q >= static_cast<int64_t>(N) * N * N) {
    atomicOr(flags, 1);
    return;
  }
  for (int d = 0; d < 3; ++d) {
    float x = pos[d * n + p] + r[q * 3 + d] * dp;
    if (x >= box) x -= box;
    if (x < 0.f) {  // x + box can round up to box: its periodic image is 0
      x += box;
      if (x >= box) x = 0.f;
    }
    pos[d * n + p] = x;
  }
}

__global__ __launch_bounds__(kNT) void k_scale(float* __restrict__ p, int64_t count, float g) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  if (i < count) p[i] *= g;
}

// The cube symmetry (perm, f) of a channels-last lattice field [N^3][C] of 3-vectors: output site o takes input site
// u with u[perm[d]] = f_d ? N - 1 - o_d : o_d, and its channel c = 3 m + d takes the input channel 3 m + perm[d],
// negated when f_d is set. One thread per output site; its C values are contiguous in both fields.
__global__ __launch_bounds__(kNT) void k_symmetry(const float* __restrict__ in, float* __restrict__ out, int N, int C,
                                                  int p0, int p1, int p2, int f) {
  const int64_t v = static_cast<int64_t>(blockIdx.x) * kNT + threadIdx.x;
  const int64_t V = static_cast<int64_t>(N) * N * N;
  if (v >= V) return;
  const int o[3] = {static_cast<int>(v / (static_cast<int64_t>(N) * N)), static_cast<int>((v / N) % N),
                    static_cast<int>(v % N)};
  const int perm[3] = {p0, p1, p2};
  int u[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) u[perm[d]] = ((f >> d) & 1) ? N - 1 - o[d] : o[d];
  const int64_t src = ((static_cast<int64_t>(u[0]) * N + u[1]) * N + u[2]) * C;
  const int64_t dst = v * C;
  for (int m = 0; m < C; m += 3) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float x = in[src + m + perm[d]];
      out[dst + m + d] = ((f >> d) & 1) ? -x : x;
    }
  }
}

}  // namespace

hipError_t conv3(View in, int cin, const bf16* w, int kpad, int nb, const float* bias, int leaky_act, View out,
                 float* outf, int cout, int D, hipStream_t s, View mask, int mask_ch) {
  if (mask_ch > 0 && (outf || !mask.p || (mask_ch & 7) != 0)) return hipErrorInvalidValue;
  const unsigned grid = static_cast<unsigned>(((D + 3) / 4) * ((D + 3) / 4) * ((D + 15) / 16));
#define LPC_CONV(CI, NBV) \
  k_conv3<CI, NBV><<<grid, kNT, 0, s>>>(in, w, kpad, bias, leaky_act, out, outf, cout, D, mask, mask_ch)
  if (cin == 8 && nb == 1) LPC_CONV(8, 1);
  else if (cin == 8 && nb == 2) LPC_CONV(8, 2);
  else if (cin == 8 && nb == 4) LPC_CONV(8, 4);
  else if (cin == 16 && nb == 1) LPC_CONV(16, 1);
  else if (cin == 16 && nb == 2) LPC_CONV(16, 2);
  else if (cin == 16 && nb == 4) LPC_CONV(16, 4);
  else if (cin == 32 && nb == 1) LPC_CONV(32, 1);
  else if (cin == 32 && nb == 2) LPC_CONV(32, 2);
  else if (cin == 32 && nb == 4) LPC_CONV(32, 4);
  else if (cin == 64 && nb == 1) LPC_CONV(64, 1);
  else if (cin == 64 && nb == 2) LPC_CONV(64, 2);
  else if (cin == 64 && nb == 4) LPC_CONV(64, 4);
  else return hipErrorInvalidValue;
#undef LPC_CONV
  return hipGetLastError();
}

hipError_t down2(View x, int cin, const float* W, const float* b, int cout, View out, int D, hipStream_t s) {
  const unsigned grid = blocks_for(static_cast<int64_t>(D / 2) * (D / 2) * (D / 2), 64);  // 64 coarse voxels per block
  const View none{nullptr, 0, 0};
  if (cin == 16 && cout == 32) k_down2<16, 32, false><<<grid, kNT, 0, s>>>(x, W, b, out, D, none, 0);
  else if (cin == 32 && cout == 64) k_down2<32, 64, false><<<grid, kNT, 0, s>>>(x, W, b, out, D, none, 0);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t up2(View x, int cin, const float* W, const float* b, int cout, View out, int D, hipStream_t s) {
  const unsigned grid = blocks_for(static_cast<int64_t>(D) * D * D, 64);  // 64 coarse voxels per block
  const View none{nullptr, 0, 0};
  if (cin == 64 && cout == 32) k_up2<64, 32, false><<<grid, kNT, 0, s>>>(x, W, b, out, D, 0, none, 0);
  else if (cin == 32 && cout == 16) k_up2<32, 16, false><<<grid, kNT, 0, s>>>(x, W, b, out, D, 0, none, 0);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// The data gradient of a 2^3 down layer has the form of an up layer from dz's grid, and that of an up layer the
// form of a down layer onto dx's grid, both with the transposed weights Wt[i][t][o].
hipError_t down2_dgrad(View dz, int cout, const float* Wt, int cin, View dx, int D, int accumulate, hipStream_t s,
                       View mask, int mask_ch) {
  if (mask_ch > 0 && (!mask.p || (mask_ch & 7) != 0)) return hipErrorInvalidValue;
  const int Dc = D / 2;
  const unsigned grid = blocks_for(static_cast<int64_t>(Dc) * Dc * Dc, 64);
  if (cin == 16 && cout == 32)
    k_up2<32, 16, true><<<grid, kNT, 0, s>>>(dz, Wt, nullptr, dx, Dc, accumulate, mask, mask_ch);
  else if (cin == 32 && cout == 64)
    k_up2<64, 32, true><<<grid, kNT, 0, s>>>(dz, Wt, nullptr, dx, Dc, accumulate, mask, mask_ch);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t up2_dgrad(View dz, int cout, const float* Wt, int cin, View dx, int D, hipStream_t s, View mask,
                     int mask_ch) {
  if (mask_ch > 0 && (!mask.p || (mask_ch & 7) != 0)) return hipErrorInvalidValue;
  const unsigned grid = blocks_for(static_cast<int64_t>(D) * D * D, 64);
  if (cin == 32 && cout == 16) k_down2<16, 32, true><<<grid, kNT, 0, s>>>(dz, Wt, nullptr, dx, 2 * D, mask, mask_ch);
  else if (cin == 64 && cout == 32)
    k_down2<32, 64, true><<<grid, kNT, 0, s>>>(dz, Wt, nullptr, dx, 2 * D, mask, mask_ch);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t transpose2(const float* W, int cout, int cin, float* Wt, hipStream_t s) {
  k_transpose2<<<blocks_for(static_cast<int64_t>(cout) * 8 * cin), kNT, 0, s>>>(W, cout, cin, Wt);
  return hipGetLastError();
}

int wgrad_chunks(int kind, int cin, int cout, int D) {
  const int ntile = ((cout + 15) / 16) * ((cin + 15) / 16);
  const int c512 = std::max(1, 512 / ntile);  // about 512 workgroups over the chunks and the (o, i) tiles
  if (wgrad3_mfma(kind, D)) return std::min(c512, (D / 4) * (D / 4) * (D / kWB));
  if (kind != 0) {
    const int Dc = (kind == 1) ? D / 2 : D;
    return std::min(c512, (Dc * Dc * Dc + kW2Y - 1) / kW2Y);
  }
  const int c = D * D * D / 4096;  // 3^3 layer on the VALU kernel
  return c < 1 ? 1 : (c > 64 ? 64 : c);
}

hipError_t wgrad(int kind, View x, int cin, int cin_real, View dz, int cout, int D, float* partial, hipStream_t s) {
  if (cin > kMaxC || cout > kMaxC || (cin % 8) != 0) return hipErrorInvalidValue;
  if (wgrad3_mfma(kind, D) || kind != 0) {
    const int nchunk = wgrad_chunks(kind, cin, cout, D);
    const dim3 grid(static_cast<unsigned>(nchunk), static_cast<unsigned>(((cout + 15) / 16) * ((cin + 15) / 16)));
    if (kind == 0)
      k_wgrad3<<<grid, kNT, 0, s>>>(x, cin, cin_real, dz, cout, D, nchunk, partial);
    else
      k_wgrad2<<<grid, kNT, 0, s>>>(kind, x, cin, cin_real, dz, cout, D, nchunk, partial);
    return hipGetLastError();
  }
  const dim3 grid(static_cast<unsigned>(wgrad_chunks(kind, cin, cout, D)), 27u);  // a 3^3 layer on a small grid
  if (cin == 8)
    k_wgrad<8><<<grid, kNT, 0, s>>>(x, cin, cin_real, dz, cout, D, partial);
  else if ((cin % 16) == 0 && cout * (cin / 16) <= kNT)
    k_wgrad<16><<<grid, kNT, 0, s>>>(x, cin, cin_real, dz, cout, D, partial);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t reduce_partials(const float* partial, int nchunk, int nW, int cout, int nslot, float* grad,
                           hipStream_t s) {
  k_reduce<<<blocks_for(nW + cout, 64), 64 * kRW, 0, s>>>(partial, nchunk, nW, cout, nslot, grad);
  return hipGetLastError();
}

hipError_t convert_conv3(const float* W, int cout, int cin, bf16* wf, int cinp, int nbo, int kpad, bf16* wb,
                         int coutp, int nbi, int kpadb, hipStream_t s) {
  const int64_t n = static_cast<int64_t>(16 * nbo) * kpad + static_cast<int64_t>(16 * nbi) * kpadb;
  k_convert_conv3<<<blocks_for(n), kNT, 0, s>>>(W, cout, cin, wf, cinp, nbo, kpad, wb, coutp, nbi, kpadb);
  return hipGetLastError();
}

hipError_t pack_input(const float* feat, bf16* x, int V, hipStream_t s) {
  k_pack_input<<<blocks_for(V), kNT, 0, s>>>(feat, x, V);
  return hipGetLastError();
}

int loss_blocks(int V) { return static_cast<int>(blocks_for(static_cast<int64_t>(V) * 8)); }

hipError_t loss_grad(const float* out, const float* target, bf16* dout, double* loss_part, int V, hipStream_t s) {
  k_loss_grad<<<static_cast<unsigned>(loss_blocks(V)), kNT, 0, s>>>(out, target, dout, loss_part, V);
  return hipGetLastError();
}

hipError_t adam(float* p, float* m, float* v, const float* g, int64_t count, float lr, double beta1, double beta2,
                float eps, int64_t t, hipStream_t s) {
  const float c1 = static_cast<float>(1.0 - std::pow(beta1, static_cast<double>(t)));
  const float c2 = static_cast<float>(1.0 - std::pow(beta2, static_cast<double>(t)));
  k_adam<<<blocks_for(count), kNT, 0, s>>>(p, m, v, g, count, lr, static_cast<float>(beta1),
                                           static_cast<float>(1.0 - beta1), static_cast<float>(beta2),
                                           static_cast<float>(1.0 - beta2), eps, c1, c2);
  return hipGetLastError();
}

hipError_t features(const float* pos, const int32_t* id, int64_t n, const float* ref, const float* psi1, int N,
                    double box, float* out, int* flags, hipStream_t s) {
  k_features<false><<<blocks_for(n), kNT, 0, s>>>(pos, id, n, ref, psi1, N, box, out, psi1 ? kInputChannels : 3,
                                                  nullptr, flags);
  return hipGetLastError();
}

hipError_t features_packed(const float* pos, const int32_t* id, int64_t n, const float* psi1, int N, double box,
                           bf16* x, int* flags, hipStream_t s) {
  if (!psi1) return hipErrorInvalidValue;
  k_features<true><<<blocks_for(n), kNT, 0, s>>>(pos, id, n, nullptr, psi1, N, box, nullptr, 0, x, flags);
  return hipGetLastError();
}

hipError_t scale(float* p, int64_t count, float g, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_scale<<<blocks_for(count), kNT, 0, s>>>(p, count, g);
  return hipGetLastError();
}

hipError_t symmetry(const float* in, float* out, int N, int C, int k, hipStream_t s) {
  static constexpr int kPerms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  if (k < 0 || k >= 48 || C < 3 || C % 3 != 0 || N < 1) return hipErrorInvalidValue;
  const int* p = kPerms[k / 8];
  const int64_t V = static_cast<int64_t>(N) * N * N;
  k_symmetry<<<blocks_for(V), kNT, 0, s>>>(in, out, N, C, p[0], p[1], p[2], k % 8);
  return hipGetLastError();
}

hipError_t apply_residual(float* pos, const int32_t* id, int64_t n, const float* r, int N, double box, int* flags,
                          hipStream_t s) {
  k_apply<<<blocks_for(n), kNT, 0, s>>>(pos, id, n, r, N, static_cast<float>(box / N), static_cast<float>(box),
                                        flags);
  return hipGetLastError();
}

}  // namespace net
}  // namespace lpc
